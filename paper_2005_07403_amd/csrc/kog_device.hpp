// kog_device.hpp -- the device side of the Kogbetliantz method shared by the
// single-problem drivers (kog.hip) and the uneven batch (kog_batch.hip): the
// circle-ordering pairs, the column-major matrix view, the pivot gather, the
// rotations with the placement rule, the single-step update tile, and the
// two-step (lane-shift) tile with its helpers.  Host helpers defined in
// kog.hip that the batch driver also uses are declared at the end.
#pragma once

#include <hip/hip_runtime.h>

#include <stdint.h>

#include "svd2.h"
#include "svd2_lane.hpp"

namespace kog {

using namespace svd2;

constexpr int kUpdBlock = 256;   // threads per update workgroup
constexpr int kRedBlocks = 1024; // partial sums of the norm reduction
constexpr unsigned kSpinLimit = 1u << 20;

__device__ __forceinline__ void pair_ab(int t, int k, int M, int &a, int &b) {
  if (k == 0) {
    a = t;
    b = M;
  } else {
    a = t + k;
    if (a >= M) a -= M;
    b = t - k;
    if (b < 0) b += M;
  }
}

template <class T, bool CPLX> struct Mat {
  T *A;
  size_t lda;
  __device__ __forceinline__ Cx<T> ld(int i, int j) const {
    size_t o = (size_t)i + (size_t)j * lda;
    if constexpr (CPLX) {
      typedef T V __attribute__((ext_vector_type(2)));
      V v = *reinterpret_cast<const V *>(A + 2 * o);
      return {v.x, v.y};
    } else {
      return {A[o], T(0)};
    }
  }
  __device__ __forceinline__ void st(int i, int j, Cx<T> x) const {
    size_t o = (size_t)i + (size_t)j * lda;
    if constexpr (CPLX) {
      typedef T V __attribute__((ext_vector_type(2)));
      V v;
      v.x = x.re;
      v.y = x.im;
      *reinterpret_cast<V *>(A + 2 * o) = v;
    } else {
      A[o] = x.re;
    }
  }
};

// Device-side view of the workspace: gathered pivots (SoA, NIN arrays of n)
// and the batched-SVD outputs (NOUT arrays of n), as the batched kernels
// read and write them.
template <class T, bool CPLX> struct Bufs {
  static constexpr int NIN = CPLX ? 8 : 4, NOUT = CPLX ? 19 : 11;
  T *piv[NIN];
  T *out[NOUT];
};

struct Bar {
  unsigned count, gen, abort, pad;
};

struct Layout {
  size_t piv, out, red, res, bar, flags, total;
  size_t piv1, out1, mat, total2;  // two-step mode: second rotation set and a matrix buffer
  size_t piv2, out2, total3;       // three-step mode: a third rotation set
};
constexpr int kMaxFusedBlocks = 4096;  // barrier slots (64 bytes each)

inline Layout layout(int N, size_t esz, bool cplx) {
  auto up = [](size_t x) { return (x + 255) & ~size_t(255); };
  size_t n = (size_t)N / 2;
  size_t nin = cplx ? 8 : 4, nout = cplx ? 19 : 11;
  Layout L;
  size_t arr = up(n * esz);
  L.piv = 0;
  L.out = L.piv + nin * arr;
  L.red = L.out + nout * arr;
  L.res = L.red + up(2 * kRedBlocks * sizeof(double));
  L.bar = L.res + 256;
  L.flags = L.bar + 256;
  L.total = L.flags + (size_t)kMaxFusedBlocks * 64;
  L.piv1 = L.total;
  L.out1 = L.piv1 + nin * arr;
  L.mat = L.out1 + nout * arr;
  L.total2 = L.mat + up((size_t)N * N * esz * (cplx ? 2 : 1));
  L.piv2 = L.total2;
  L.out2 = L.piv2 + nin * arr;
  L.total3 = L.out2 + nout * arr;
  return L;
}

template <class T, bool CPLX> Bufs<T, CPLX> make_bufs(void *ws, int N, int set = 0) {
  Layout L = layout(N, sizeof(T), CPLX);
  auto up = [](size_t x) { return (x + 255) & ~size_t(255); };
  size_t arr = up((size_t)(N / 2) * sizeof(T));
  Bufs<T, CPLX> b;
  char *base = (char *)ws;
  size_t piv = set == 2 ? L.piv2 : set ? L.piv1 : L.piv, out = set == 2 ? L.out2 : set ? L.out1 : L.out;
  for (int i = 0; i < Bufs<T, CPLX>::NIN; ++i) b.piv[i] = (T *)(base + piv + i * arr);
  for (int i = 0; i < Bufs<T, CPLX>::NOUT; ++i) b.out[i] = (T *)(base + out + i * arr);
  return b;
}

// ---------------------------------------------------------------------------
// gather: pivot block of pair k into the SoA trains (record order 11, 21, 12, 22)
// ---------------------------------------------------------------------------
template <class T, bool CPLX>
__device__ __forceinline__ void gather_one(const Mat<T, CPLX> &M, int N, int t, int k, T *x) {
  int a, b;
  pair_ab(t, k, N - 1, a, b);
  int p = a < b ? a : b, q = a < b ? b : a;
  Cx<T> e[4] = {M.ld(p, p), M.ld(q, p), M.ld(p, q), M.ld(q, q)};
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    if constexpr (CPLX) {
      x[2 * i] = e[i].re;
      x[2 * i + 1] = e[i].im;
    } else {
      x[i] = e[i].re;
    }
  }
}


// ---------------------------------------------------------------------------
// rotation of pair k as used by the update: U, V (swap applied), sigma at (p,p), (q,q)
// ---------------------------------------------------------------------------
template <class T> struct Rot {
  Cx<T> u11, u21, u12, u22, v11, v21, v12, v22;
  T sp, sq;
};

// out(e): element e of the SVD record (U, V, sigma); piv(e): of the pivot block
template <class T, bool CPLX, class FO, class FP>
__device__ __forceinline__ Rot<T> rot_of(FO out, FP piv) {
  Rot<T> r;
  constexpr int K = CPLX ? 16 : 8;
  auto g = [&](int e) -> Cx<T> {
    if constexpr (CPLX) return {out(2 * e), out(2 * e + 1)};
    else return {out(e), T(0)};
  };
  r.u11 = g(0); r.u21 = g(1); r.u12 = g(2); r.u22 = g(3);
  r.v11 = g(4); r.v21 = g(5); r.v12 = g(6); r.v22 = g(7);
  r.sp = out(K);
  r.sq = out(K + 1);
  bool sw;
  if constexpr (CPLX) {
    T pr = piv(0), pi = piv(1), qr = piv(6), qi = piv(7);
    sw = pr * pr + pi * pi < qr * qr + qi * qi;
  } else {
    sw = vabs(piv(0)) < vabs(piv(3));
  }
  if (sw) {
    Cx<T> t;
    t = r.u11; r.u11 = r.u12; r.u12 = t;
    t = r.u21; r.u21 = r.u22; r.u22 = t;
    t = r.v11; r.v11 = r.v12; r.v12 = t;
    t = r.v21; r.v21 = r.v22; r.v22 = t;
    T s = r.sp; r.sp = r.sq; r.sq = s;
  }
  return r;
}

template <class T, bool CPLX>
__device__ __forceinline__ Rot<T> load_rot(const Bufs<T, CPLX> &B, int k) {
  return rot_of<T, CPLX>([&](int e) { return B.out[e][k]; }, [&](int e) { return B.piv[e][k]; });
}

template <class T> __device__ __forceinline__ Cx<T> cadd(Cx<T> a, Cx<T> b) {
  return {a.re + b.re, a.im + b.im};
}

// B' = (U_k^* B) V_l, in the oracle's rounding order
template <class T, bool CPLX>
__device__ __forceinline__ void rotate_block(const Rot<T> &u, const Rot<T> &v, Cx<T> &b11,
                                             Cx<T> &b21, Cx<T> &b12, Cx<T> &b22) {
  if constexpr (CPLX) {
    Cx<T> t11 = cadd(cmulc(u.u11, b11), cmulc(u.u21, b21));
    Cx<T> t21 = cadd(cmulc(u.u12, b11), cmulc(u.u22, b21));
    Cx<T> t12 = cadd(cmulc(u.u11, b12), cmulc(u.u21, b22));
    Cx<T> t22 = cadd(cmulc(u.u12, b12), cmulc(u.u22, b22));
    b11 = cadd(cmul(t11, v.v11), cmul(t12, v.v21));
    b12 = cadd(cmul(t11, v.v12), cmul(t12, v.v22));
    b21 = cadd(cmul(t21, v.v11), cmul(t22, v.v21));
    b22 = cadd(cmul(t21, v.v12), cmul(t22, v.v22));
  } else {
    T t11 = vfma(u.u11.re, b11.re, u.u21.re * b21.re);
    T t21 = vfma(u.u12.re, b11.re, u.u22.re * b21.re);
    T t12 = vfma(u.u11.re, b12.re, u.u21.re * b22.re);
    T t22 = vfma(u.u12.re, b12.re, u.u22.re * b22.re);
    b11.re = vfma(t11, v.v11.re, t12 * v.v21.re);
    b12.re = vfma(t11, v.v12.re, t12 * v.v22.re);
    b21.re = vfma(t21, v.v11.re, t22 * v.v21.re);
    b22.re = vfma(t21, v.v12.re, t22 * v.v22.re);
  }
}

// One update tile: row pairs [k0, k0 + kc) x column pairs [l0, l0 + lc), on a
// workgroup of kUpdBlock threads: thread i takes row pair k0 + i % kc and every
// (kUpdBlock / kc)-th column pair of the tile (kc in {64, 128, 256}, so small
// orders still fill the workgroup).  Rows are addressed by (a, b) so that the
// loads and stores of a wavefront form contiguous runs; the orientation
// p < q is applied in registers.  The loads of UpdG column pairs are issued
// before their stores (the compiler cannot move a load past a store to the
// same matrix).  With ACC the thread returns the sum of |a_ij|^2 over the
// off-diagonal entries it wrote (FP64), for the convergence test.
struct Tile {
  int k0, kc, l0, lc;
};
template <bool CPLX> struct UpdG { static constexpr int v = CPLX ? 2 : 4; };

template <class T> __device__ __forceinline__ double abs2(Cx<T> x) {
  return (double)x.re * (double)x.re + (double)x.im * (double)x.im;
}

template <class T, bool CPLX, bool ACC>
__device__ __forceinline__ double update_tile(const Mat<T, CPLX> &M, int N, int t,
                                              const Bufs<T, CPLX> &B, Tile tl) {
  constexpr int G = UpdG<CPLX>::v;
  const int n = N / 2, Mo = N - 1;
  const int groups = kUpdBlock / tl.kc;
  const int k = tl.k0 + (int)threadIdx.x % tl.kc;
  const int g = (int)threadIdx.x / tl.kc;
  double off2 = 0.0;
  if (k >= n) return off2;
  int ra, rb;
  pair_ab(t, k, Mo, ra, rb);
  const bool kflip = ra > rb;  // then p = rb, q = ra
  Rot<T> u = load_rot<T, CPLX>(B, k);
  const int lend = tl.l0 + tl.lc < n ? tl.l0 + tl.lc : n;
  for (int lb = tl.l0 + g; lb < lend; lb += groups * G) {
    Cx<T> xa1[G], xb1[G], xa2[G], xb2[G];
    int cp[G], cq[G];
#pragma unroll
    for (int j = 0; j < G; ++j) {
      int l = lb + groups * j;
      if (l < lend) {
        int ca, cb;
        pair_ab(t, l, Mo, ca, cb);
        cp[j] = ca < cb ? ca : cb;
        cq[j] = ca < cb ? cb : ca;
        xa1[j] = M.ld(ra, cp[j]);
        xb1[j] = M.ld(rb, cp[j]);
        xa2[j] = M.ld(ra, cq[j]);
        xb2[j] = M.ld(rb, cq[j]);
      }
    }
#pragma unroll
    for (int j = 0; j < G; ++j) {
      int l = lb + groups * j;
      if (l < lend) {
        Cx<T> b11 = kflip ? xb1[j] : xa1[j], b21 = kflip ? xa1[j] : xb1[j];
        Cx<T> b12 = kflip ? xb2[j] : xa2[j], b22 = kflip ? xa2[j] : xb2[j];
        if (l == k) {  // pivot block: diag(sigma_p, sigma_q), exact zeros elsewhere
          b11 = Cx<T>{u.sp, T(0)};
          b22 = Cx<T>{u.sq, T(0)};
          b12 = b21 = Cx<T>{T(0), T(0)};
        } else {
          Rot<T> v = load_rot<T, CPLX>(B, l);
          rotate_block<T, CPLX>(u, v, b11, b21, b12, b22);
          if (ACC) off2 += (abs2(b11) + abs2(b21)) + (abs2(b12) + abs2(b22));
        }
        M.st(ra, cp[j], kflip ? b21 : b11);
        M.st(rb, cp[j], kflip ? b11 : b21);
        M.st(ra, cq[j], kflip ? b22 : b12);
        M.st(rb, cq[j], kflip ? b12 : b22);
      }
    }
  }
  return off2;
}

// tile shape by order: the first rule with N <= max_order applies
struct TileRule {
  int max_order, kc, lc;
};
constexpr int kMaxRules = 16;
__host__ __device__ inline TileRule default_rule() { return TileRule{0x7fffffff, 256, 8}; }


// ---------------------------------------------------------------------------
// two steps per pass (out of place).  Under the circle ordering row x is paired
// with partner_t(x) = (2t - x) mod (N-1) at step t, so a 2x2 output block of
// step t+1 (rows {p', q'}, columns {p'', q''}) depends only on the rows
// {p', q', partner_t(p'), partner_t(q')} and the matching columns of the
// matrix before step t: each entry after step t is one entry of one rotated
// 2x2 block of step t.  Every entry is computed with exactly the operations of
// the single-step update, so two steps per pass are bitwise equal to two
// single steps; the pivots of step t+1 are such entries too, so the rotations
// of step t+1 are known before the matrix is touched.
// ---------------------------------------------------------------------------
// pair index of row x at step t and its partner
__device__ __forceinline__ void pos_at(int t, int x, int M, int n, int &k, int &partner) {
  if (x == t) {
    k = 0;
    partner = M;
  } else if (x == M) {
    k = 0;
    partner = t;
  } else {
    int d = x - t;
    if (d < 0) d += M;
    k = d < n ? d : M - d;
    int pr = 2 * t - x;
    if (pr < 0) pr += M;
    if (pr >= M) pr -= M;
    partner = pr;
  }
}

// one row (or column) of a step-(t+1) block, seen from step t
struct Side {
  int x, partner, k;
  bool isq;  // x is the q (larger) index of its step-t pair
};
__device__ __forceinline__ Side side_at(int t, int x, int M, int n) {
  Side s;
  s.x = x;
  pos_at(t, x, M, n, s.k, s.partner);
  s.isq = x > s.partner;
  return s;
}

template <class T> struct RotU {
  Cx<T> u11, u21, u12, u22;
  T sp, sq;
};
template <class T> struct RotV {
  Cx<T> v11, v21, v12, v22;
};
template <class T, bool CPLX> __device__ __forceinline__ RotU<T> load_u(const Bufs<T, CPLX> &B, int k) {
  Rot<T> r = load_rot<T, CPLX>(B, k);
  return RotU<T>{r.u11, r.u21, r.u12, r.u22, r.sp, r.sq};
}
// entry (role of the row, role of the column) of U^* B V for a step-t block
// B given in (p-row, q-row) x (p-col, q-col) order; the operations are those
// of rotate_block for that entry
template <class T, bool CPLX>
__device__ __forceinline__ Cx<T> rotated_entry(const RotU<T> &u, bool rq, const RotV<T> &v, bool cq, Cx<T> b11,
                                               Cx<T> b21, Cx<T> b12, Cx<T> b22) {
  if constexpr (CPLX) {
    Cx<T> ua = rq ? u.u12 : u.u11, ub = rq ? u.u22 : u.u21;
    Cx<T> t1 = cadd(cmulc(ua, b11), cmulc(ub, b21));
    Cx<T> t2 = cadd(cmulc(ua, b12), cmulc(ub, b22));
    Cx<T> va = cq ? v.v12 : v.v11, vb = cq ? v.v22 : v.v21;
    return cadd(cmul(t1, va), cmul(t2, vb));
  } else {
    T ua = rq ? u.u12.re : u.u11.re, ub = rq ? u.u22.re : u.u21.re;
    T t1 = vfma(ua, b11.re, ub * b21.re);
    T t2 = vfma(ua, b12.re, ub * b22.re);
    T va = cq ? v.v12.re : v.v11.re, vb = cq ? v.v22.re : v.v21.re;
    return Cx<T>{vfma(t1, va, t2 * vb), T(0)};
  }
}

// A(r, c) after step t, from the matrix before it: xrc = A(r, c), xrp = A(r,
// partner_c), xpc = A(partner_r, c), xpp = A(partner_r, partner_c)
template <class T, bool CPLX>
__device__ __forceinline__ Cx<T> after_step(const Side &r, const RotU<T> &ur, const Side &c, const RotV<T> &vc,
                                            Cx<T> xrc, Cx<T> xrp, Cx<T> xpc, Cx<T> xpp) {
  if (r.k == c.k) {  // inside a pivot block of step t: diag(sigma_p, sigma_q), zeros elsewhere
    if (r.x == c.x) return Cx<T>{r.isq ? ur.sq : ur.sp, T(0)};
    return Cx<T>{T(0), T(0)};
  }
  // the step-t block in (p-row, q-row) x (p-col, q-col) order
  Cx<T> b11 = r.isq ? (c.isq ? xpp : xpc) : (c.isq ? xrp : xrc);
  Cx<T> b12 = r.isq ? (c.isq ? xpc : xpp) : (c.isq ? xrc : xrp);
  Cx<T> b21 = r.isq ? (c.isq ? xrp : xrc) : (c.isq ? xpp : xpc);
  Cx<T> b22 = r.isq ? (c.isq ? xrc : xrp) : (c.isq ? xpc : xpp);
  return rotated_entry<T, CPLX>(ur, r.isq, vc, c.isq, b11, b21, b12, b22);
}


// pivots of steps t and t+1 in one launch: lane k computes the SVD of pair k
// of step t (into B0) and, for pair k of step t+1, recomputes the step-t SVDs
// of the two pairs its rows belong to (the same arithmetic on the same
// inputs, so bitwise the rotations in B0), forms that pivot block after step
// t and computes its SVD (into B1)
template <class T, bool CPLX>
__device__ __forceinline__ void pivots2_one(int N, const Mat<T, CPLX> &M, int t, const Bufs<T, CPLX> &B0,
                                            const Bufs<T, CPLX> &B1, int k) {
  constexpr int RESC = sizeof(T) == 4 ? 1 : 0;
  constexpr int NI = Bufs<T, CPLX>::NIN, NO = Bufs<T, CPLX>::NOUT;
  const int n = N / 2, Mo = N - 1;
  int a, b;
  pair_ab(t + 1, k, Mo, a, b);
  const int p = a < b ? a : b, q = a < b ? b : a;
  Side S[2] = {side_at(t, p, Mo, n), side_at(t, q, Mo, n)};
  // every load first (the stores below could alias the matrix as far as the
  // compiler knows): the three step-t pivot blocks and the 4x4 neighbourhood
  T x0[NI], x1[NI], x2[NI];
  gather_one<T, CPLX>(M, N, t, k, x0);
  gather_one<T, CPLX>(M, N, t, S[0].k, x1);
  gather_one<T, CPLX>(M, N, t, S[1].k, x2);
  Cx<T> nb[2][2][2][2];  // [row i][col j][row or partner][col or partner]
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      nb[i][j][0][0] = M.ld(S[i].x, S[j].x);
      nb[i][j][0][1] = M.ld(S[i].x, S[j].partner);
      nb[i][j][1][0] = M.ld(S[i].partner, S[j].x);
      nb[i][j][1][1] = M.ld(S[i].partner, S[j].partner);
    }
  T y0[NO], y1[NO], y2[NO];
  one_matrix<T, CPLX, RESC>(x0, y0, 2);
  one_matrix<T, CPLX, RESC>(x1, y1, 2);
  one_matrix<T, CPLX, RESC>(x2, y2, 2);
  Rot<T> r1 = rot_of<T, CPLX>([&](int e) { return y1[e]; }, [&](int e) { return x1[e]; });
  Rot<T> r2 = rot_of<T, CPLX>([&](int e) { return y2[e]; }, [&](int e) { return x2[e]; });
  RotU<T> U[2] = {RotU<T>{r1.u11, r1.u21, r1.u12, r1.u22, r1.sp, r1.sq},
                  RotU<T>{r2.u11, r2.u21, r2.u12, r2.u22, r2.sp, r2.sq}};
  RotV<T> V[2] = {RotV<T>{r1.v11, r1.v21, r1.v12, r1.v22}, RotV<T>{r2.v11, r2.v21, r2.v12, r2.v22}};
  Cx<T> e[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
      e[i][j] = after_step<T, CPLX>(S[i], U[i], S[j], V[j], nb[i][j][0][0], nb[i][j][0][1], nb[i][j][1][0],
                                    nb[i][j][1][1]);
  Cx<T> rec[4] = {e[0][0], e[1][0], e[0][1], e[1][1]};
  T x3[NI], y3[NO];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    if constexpr (CPLX) {
      x3[2 * i] = rec[i].re;
      x3[2 * i + 1] = rec[i].im;
    } else {
      x3[i] = rec[i].re;
    }
  }
  one_matrix<T, CPLX, RESC>(x3, y3, 2);
#pragma unroll
  for (int i = 0; i < NI; ++i) B0.piv[i][k] = x0[i];
#pragma unroll
  for (int i = 0; i < NO; ++i) B0.out[i][k] = y0[i];
#pragma unroll
  for (int i = 0; i < NI; ++i) B1.piv[i][k] = x3[i];
#pragma unroll
  for (int i = 0; i < NO; ++i) B1.out[i][k] = y3[i];
}


// pivots of step t+2, after the pivots of steps t (B0) and t+1 (B1) are
// known, on four lanes per pair: lane sub = 2 a + b of pair k forms entry
// (a, b) of the pair's step-(t+2) pivot block (rows and columns p < q) from
// the matrix before step t.  Its row belongs to a pair of step t+1 and its
// column to another, each of whose two indices belongs to a pair of step t:
// the entry after step t+1 is one rotated entry of a step-(t+1) block of
// entries after step t, each of those one rotated entry of a step-t block of
// the matrix (16 loads per lane), with the rotations as stored in B0 and B1,
// so with exactly the operations of two single steps.  Lane 0 of the four
// gathers the block and puts its SVD into B2.  All four lanes call it.
template <class T, bool CPLX>
__device__ __forceinline__ void pivots3_quad(int N, const Mat<T, CPLX> &M, int t, const Bufs<T, CPLX> &B0,
                                             const Bufs<T, CPLX> &B1, const Bufs<T, CPLX> &B2, int k, int sub,
                                             bool valid) {
  constexpr int RESC = sizeof(T) == 4 ? 1 : 0;
  constexpr int NI = Bufs<T, CPLX>::NIN, NO = Bufs<T, CPLX>::NOUT;
  const int n = N / 2, Mo = N - 1;
  const int ia = sub >> 1, ib = sub & 1;
  Cx<T> ent{T(0), T(0)};
  if (valid) {
    int a, b;
    pair_ab(t + 2, k, Mo, a, b);
    const int xr = ia == 0 ? (a < b ? a : b) : (a < b ? b : a);
    const int xc = ib == 0 ? (a < b ? a : b) : (a < b ? b : a);
    const Side R1 = side_at(t + 1, xr, Mo, n), C1 = side_at(t + 1, xc, Mo, n);
    const int rr[2] = {R1.x, R1.partner}, cc[2] = {C1.x, C1.partner};
    Side R0[2], C0[2];
    RotU<T> U0[2];
    RotV<T> V0[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      R0[i] = side_at(t, rr[i], Mo, n);
      C0[i] = side_at(t, cc[i], Mo, n);
      const Rot<T> ru = load_rot<T, CPLX>(B0, R0[i].k), rv = load_rot<T, CPLX>(B0, C0[i].k);
      U0[i] = RotU<T>{ru.u11, ru.u21, ru.u12, ru.u22, ru.sp, ru.sq};
      V0[i] = RotV<T>{rv.v11, rv.v21, rv.v12, rv.v22};
    }
    const Rot<T> r1 = load_rot<T, CPLX>(B1, R1.k), c1 = load_rot<T, CPLX>(B1, C1.k);
    const RotU<T> U1{r1.u11, r1.u21, r1.u12, r1.u22, r1.sp, r1.sq};
    const RotV<T> V1{c1.v11, c1.v21, c1.v12, c1.v22};
    Cx<T> A1[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
        A1[i][j] = after_step<T, CPLX>(R0[i], U0[i], C0[j], V0[j], M.ld(rr[i], cc[j]), M.ld(rr[i], C0[j].partner),
                                       M.ld(R0[i].partner, cc[j]), M.ld(R0[i].partner, C0[j].partner));
    ent = after_step<T, CPLX>(R1, U1, C1, V1, A1[0][0], A1[0][1], A1[1][0], A1[1][1]);
  }
  // gather the block on lane 0 of the four: record order 11, 21, 12, 22 = sub 0, 2, 1, 3
  const int base = (int)(threadIdx.x & 63) & ~3;
  Cx<T> rec[4];
  const int src[4] = {0, 2, 1, 3};
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    rec[i].re = __shfl(ent.re, base + src[i], 64);
    if constexpr (CPLX) rec[i].im = __shfl(ent.im, base + src[i], 64);
    else rec[i].im = T(0);
  }
  if (!valid || sub != 0) return;
  T x[NI], y[NO];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    if constexpr (CPLX) {
      x[2 * i] = rec[i].re;
      x[2 * i + 1] = rec[i].im;
    } else {
      x[i] = rec[i].re;
    }
  }
  one_matrix<T, CPLX, RESC>(x, y, 2);
#pragma unroll
  for (int i = 0; i < NI; ++i) B2.piv[i][k] = x[i];
#pragma unroll
  for (int i = 0; i < NO; ++i) B2.out[i][k] = y[i];
}


// The two-step update proper ("lane-shift" form).  Lane j of a wavefront
// holds the rows of pair j of step t (P_j = t + j and Q_j = t - j mod N-1;
// pair 0 is rows t and N-1) and walks column pairs j' of step t in increasing
// order: it reads each 2x2 block (P_j, Q_j) x (P_j', Q_j') once and rotates it
// with U_j, V_j' as the single-step update would.  Pair k of step t+1 is made
// of rows P_{k+1} and Q_{k-1} (k = 0: P_1 and N-1; k = 1: P_2 and t = P_0;
// k = n-1: Q_{n-1} and Q_{n-2}), held one lane down and one lane up: they are
// exchanged with lane shuffles.  Its column pair l is made of the columns of
// iterations l+1 and l-1 of the walk (same exceptions), kept in a three-deep
// register window.  A wavefront computes 64 pairs of step t and writes the 62
// pairs of step t+1 it holds both neighbours for.
//
// The wavefronts of a workgroup share one block of rows and take consecutive
// runs of lc output column pairs.  A wavefront's first output needs a column
// of the wavefront before it and its last output one of the wavefront after
// it: each publishes its first and last walked columns in LDS, and those two
// outputs are written after a barrier.  Only the workgroup's outer edges read
// a column pair outside their own outputs.
constexpr int kShiftOut = 62;
// Column blocks the two-step walk loads ahead: 3 (real N = 4096 FP64: 32.4 ->
// 32.0 us per step against 1), except complex FP64, whose larger blocks would
// spill at the batch kernel's register cap and cost more than they gain.
template <class T, bool CPLX> constexpr int two_step_depth() { return (CPLX && sizeof(T) == 8) ? 1 : 3; }

// value select (a ternary on lvalues would select addresses and spill)
template <class T> __device__ __forceinline__ Cx<T> sel(bool c, Cx<T> x, Cx<T> y) {
  return Cx<T>{c ? x.re : y.re, c ? x.im : y.im};
}

template <class T, bool CPLX> struct VPack {
  static constexpr int W = CPLX ? 8 : 4;
  T v[W];
};
template <class T, bool CPLX> __device__ __forceinline__ VPack<T, CPLX> pack_v(const Rot<T> &r) {
  VPack<T, CPLX> p;
  if constexpr (CPLX) {
    p.v[0] = r.v11.re; p.v[1] = r.v11.im; p.v[2] = r.v21.re; p.v[3] = r.v21.im;
    p.v[4] = r.v12.re; p.v[5] = r.v12.im; p.v[6] = r.v22.re; p.v[7] = r.v22.im;
  } else {
    p.v[0] = r.v11.re; p.v[1] = r.v21.re; p.v[2] = r.v12.re; p.v[3] = r.v22.re;
  }
  return p;
}
template <class T, bool CPLX> __device__ __forceinline__ Rot<T> with_v(const RotU<T> &u, const VPack<T, CPLX> &p) {
  Rot<T> r;
  r.u11 = u.u11; r.u21 = u.u21; r.u12 = u.u12; r.u22 = u.u22;
  if constexpr (CPLX) {
    r.v11 = Cx<T>{p.v[0], p.v[1]}; r.v21 = Cx<T>{p.v[2], p.v[3]};
    r.v12 = Cx<T>{p.v[4], p.v[5]}; r.v22 = Cx<T>{p.v[6], p.v[7]};
  } else {
    r.v11 = Cx<T>{p.v[0], T(0)}; r.v21 = Cx<T>{p.v[1], T(0)};
    r.v12 = Cx<T>{p.v[2], T(0)}; r.v22 = Cx<T>{p.v[3], T(0)};
  }
  r.sp = u.sp;
  r.sq = u.sq;
  return r;
}

// rows of pair j of step t
__device__ __forceinline__ void rows_at(int t, int j, int Mo, int &P, int &Q) {
  if (j == 0) {
    P = t;
    Q = Mo;
  } else {
    P = t + j;
    if (P >= Mo) P -= Mo;
    Q = t - j;
    if (Q < 0) Q += Mo;
  }
}

// lane l takes the value of lane l+1 (dn) or l-1 (up): the wavefront
// shifts of the data-parallel primitives (wave_shl:1 / wave_shr:1), a VALU
// operand modifier instead of a round trip through the LDS crossbar; the end
// lanes keep their own value (no lane reads it)
template <int CTRL> __device__ __forceinline__ float wshift(float x) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, x),
                                                               __builtin_bit_cast(int, x), CTRL, 0xf, 0xf, false));
}
template <int CTRL> __device__ __forceinline__ double wshift(double x) {
  const long long b = __builtin_bit_cast(long long, x);
  const int lo = (int)b, hi = (int)(b >> 32);
  const int rlo = __builtin_amdgcn_update_dpp(lo, lo, CTRL, 0xf, 0xf, false);
  const int rhi = __builtin_amdgcn_update_dpp(hi, hi, CTRL, 0xf, 0xf, false);
  return __builtin_bit_cast(double, ((long long)rhi << 32) | (long long)(unsigned)rlo);
}
constexpr int kWaveShl1 = 0x130, kWaveShr1 = 0x138;
template <class T, bool CPLX> __device__ __forceinline__ Cx<T> shfl_dn1(Cx<T> x) {
  Cx<T> r;
  r.re = wshift<kWaveShl1>(x.re);
  if constexpr (CPLX) r.im = wshift<kWaveShl1>(x.im);
  else r.im = T(0);
  return r;
}
template <class T, bool CPLX> __device__ __forceinline__ Cx<T> shfl_up1(Cx<T> x) {
  Cx<T> r;
  r.re = wshift<kWaveShr1>(x.re);
  if constexpr (CPLX) r.im = wshift<kWaveShr1>(x.im);
  else r.im = T(0);
  return r;
}

// one column of the walk after the row exchange: the entries of the two rows
// of step t+1's pair k = j, smaller row index first
template <class T> struct ColPair {
  Cx<T> lo, hi;
};
template <class T> __device__ __forceinline__ ColPair<T> selp(bool c, ColPair<T> x, ColPair<T> y) {
  return ColPair<T>{sel(c, x.lo, y.lo), sel(c, x.hi, y.hi)};
}

// XCD-aware tile order.  Workgroups are dispatched round-robin over the 8
// XCDs, each with its own L2; XCD c takes a contiguous run of the tiles (row
// tile fastest), so tiles that share halo rows or columns run on the same L2
// at about the same time.
__device__ __forceinline__ int xcd_tile(int bid, int ntiles) {
  const int q = ntiles >> 3, r = ntiles & 7, c = bid & 7, k = bid >> 3;
  return c * q + (c < r ? c : r) + k;
}

// LDS bytes of the two-step kernel: a workgroup of wpg wavefronts writes
// span output column pairs
template <class T, bool CPLX> constexpr size_t two_step_lds(int wpg, int span) {
  return (size_t)(2 * span + 2) * sizeof(VPack<T, CPLX>) + (size_t)2 * wpg * 64 * sizeof(ColPair<T>);
}

// one tile: row block bx (62 row pairs), column tile by (span column pairs);
// all threads of the workgroup call it (it synchronises the workgroup)
// (the matrices are passed as restrict pointers: the pass reads one and
// writes the other, so loads of later iterations may move past stores)
template <class T, bool CPLX>
__device__ __forceinline__ void two_step_tile_r(char *kog_smem, int N, T *__restrict__ mc, size_t ldc,
                                                T *__restrict__ mn, size_t ldn, int t, const Bufs<T, CPLX> &B0,
                                                const Bufs<T, CPLX> &B1, int wpg, int span, int lc, int bx,
                                                int by) {
  const Mat<T, CPLX> Mc{mc, ldc}, Mn{mn, ldn};
  const int n = N / 2, Mo = N - 1, t1 = t + 1;
  const int lane = (int)threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);  // wavefront-uniform
  const int L0 = by * span;                              // outputs of the workgroup: [L0, Lend)
  const int Lend = L0 + span < n ? L0 + span : n;
  const int jlo = L0 > 0 ? L0 - 1 : 0;                   // pairs walked by the workgroup: [jlo, jhi]
  const int jhi = L0 + span < n - 1 ? L0 + span : n - 1;
  VPack<T, CPLX> *sv = (VPack<T, CPLX> *)kog_smem;      // V of step t, index j' - jlo
  VPack<T, CPLX> *sv1 = sv + (span + 2);                // V of step t+1, index l - L0
  ColPair<T> *xhead = (ColPair<T> *)(sv1 + span);       // [wavefront][lane]: first walked P column
  ColPair<T> *xtail = xhead + wpg * 64;                 // [wavefront][lane]: last own Q column
  for (int i = threadIdx.x; i <= jhi - jlo; i += blockDim.x) sv[i] = pack_v<T, CPLX>(load_rot<T, CPLX>(B0, jlo + i));
  for (int i = threadIdx.x; i < Lend - L0; i += blockDim.x) sv1[i] = pack_v<T, CPLX>(load_rot<T, CPLX>(B1, L0 + i));
  __syncthreads();

  // this wavefront: outputs [l0w, oend), walk [aw, bw] (lc >= 2; the last
  // wavefronts of a workgroup may have fewer outputs or none)
  const int l0w = L0 + w * lc;
  const int oend = l0w + lc < Lend ? l0w + lc : Lend;
  const bool has = l0w < oend;
  const bool next_has = w + 1 < wpg && l0w + lc < Lend;
  const int aw = w == 0 ? jlo : l0w;
  const int bw = next_has ? l0w + lc - 1 : (l0w + lc < n - 1 ? l0w + lc : n - 1);

  const int j = bx * kShiftOut - 1 + lane;
  const bool act = j >= 0 && j < n;
  const bool out = act && lane >= 1 && lane <= kShiftOut;
  int P = 0, Q = 1, ra = 0, rb = 0;
  RotU<T> u{}, u1{};
  if (act) {
    rows_at(t, j, Mo, P, Q);
    u = load_u<T, CPLX>(B0, j);
  }
  if (out) {
    pair_ab(t1, j, Mo, ra, rb);
    u1 = load_u<T, CPLX>(B1, j);
  }
  const bool rflip = P > Q, kflip = ra > rb;
  const int rp = rflip ? Q : P, rq = rflip ? P : Q;        // rows of step t's pair j in (p, q) order
  const int op = kflip ? rb : ra, oq = kflip ? ra : rb;     // rows of step t+1's pair j in (p, q) order
  // the smaller output row takes the value from one lane up (rb) when kflip,
  // else from one lane down (ra); the own-row exceptions of k = 0 and k = n-1
  const bool lo_own = kflip ? j == 0 : j == n - 1, hi_own = kflip ? j == n - 1 : j == 0;
  const Cx<T> zero{T(0), T(0)};

  // column pair l of step t+1 from its columns ca(l) (cplus) and cb(l) (cminus)
  auto emit = [&](int l, const ColPair<T> &cplus, const ColPair<T> &cminus) {
    int ca, cb;
    pair_ab(t1, l, Mo, ca, cb);
    const bool lflip = ca > cb;
    const int cp = lflip ? cb : ca, cq = lflip ? ca : cb;
    Cx<T> c11 = sel(lflip, cminus.lo, cplus.lo), c21 = sel(lflip, cminus.hi, cplus.hi);
    Cx<T> c12 = sel(lflip, cplus.lo, cminus.lo), c22 = sel(lflip, cplus.hi, cminus.hi);
    if (l == j) {
      c11 = Cx<T>{u1.sp, T(0)};
      c22 = Cx<T>{u1.sq, T(0)};
      c12 = c21 = zero;
    } else {
      Rot<T> r = with_v<T, CPLX>(u1, sv1[l - L0]);
      rotate_block<T, CPLX>(r, r, c11, c21, c12, c22);
    }
    if (out) {
      Mn.st(op, cp, c11);
      Mn.st(oq, cp, c21);
      Mn.st(op, cq, c12);
      Mn.st(oq, cq, c22);
    }
  };

  // the block (rp, rq) x (cp, cq) of one iteration, as loaded
  struct Blk {
    Cx<T> b11, b21, b12, b22;
  };
  auto load_blk = [&](int jj) -> Blk {
    int Pc, Qc;
    rows_at(t, jj, Mo, Pc, Qc);
    const int cp = Pc < Qc ? Pc : Qc, cq = Pc < Qc ? Qc : Pc;
    Blk d{zero, zero, zero, zero};
    if (act) {
      d.b11 = Mc.ld(rp, cp);
      d.b21 = Mc.ld(rq, cp);
      d.b12 = Mc.ld(rp, cq);
      d.b22 = Mc.ld(rq, cq);
    }
    return d;
  };
  ColPair<T> prev1P{zero, zero}, prev1Q{zero, zero}, prev2m{zero, zero}, firstc{zero, zero};
  if (has) {
    // the blocks of the next D iterations are in flight
    constexpr int D = two_step_depth<T, CPLX>();
    Blk q[D];
#pragma unroll
    for (int d = 0; d < D; ++d) q[d] = aw + d <= bw ? load_blk(aw + d) : Blk{zero, zero, zero, zero};
    for (int jj = aw; jj <= bw; ++jj) {
      const Blk a = q[0];
#pragma unroll
      for (int d = 0; d + 1 < D; ++d) q[d] = q[d + 1];
      if (jj + D <= bw) q[D - 1] = load_blk(jj + D);
      // step t on the block (j, jj), in (p, q) order
      int Pc, Qc;
      rows_at(t, jj, Mo, Pc, Qc);
      const bool cflip = Pc > Qc;
      Cx<T> b11 = a.b11, b21 = a.b21, b12 = a.b12, b22 = a.b22;
      if (j == jj) {
        b11 = Cx<T>{u.sp, T(0)};
        b22 = Cx<T>{u.sq, T(0)};
        b12 = b21 = zero;
      } else {
        Rot<T> r = with_v<T, CPLX>(u, sv[jj - jlo]);
        rotate_block<T, CPLX>(r, r, b11, b21, b12, b22);
      }
      // to P/Q labels
      const Cx<T> ePP = sel(rflip, sel(cflip, b22, b21), sel(cflip, b12, b11));
      const Cx<T> eQP = sel(rflip, sel(cflip, b12, b11), sel(cflip, b22, b21));
      const Cx<T> ePQ = sel(rflip, sel(cflip, b21, b22), sel(cflip, b11, b12));
      const Cx<T> eQQ = sel(rflip, sel(cflip, b11, b12), sel(cflip, b21, b22));
      // row exchange: ra(k) = P_{k+1} (one lane down) or Q_{n-1} (own, k = n-1);
      // rb(k) = Q_{k-1} (one lane up), P_0 (k = 1) or N-1 = Q_0 (own, k = 0)
      ColPair<T> curP, curQ;
      {
        Cx<T> dn = shfl_dn1<T, CPLX>(ePP), up = shfl_up1<T, CPLX>(sel(j == 0, ePP, eQP));
        curP.lo = sel(lo_own, eQP, sel(kflip, up, dn));
        curP.hi = sel(hi_own, eQP, sel(kflip, dn, up));
        dn = shfl_dn1<T, CPLX>(ePQ);
        up = shfl_up1<T, CPLX>(sel(j == 0, ePQ, eQQ));
        curQ.lo = sel(lo_own, eQQ, sel(kflip, up, dn));
        curQ.hi = sel(hi_own, eQQ, sel(kflip, dn, up));
      }
      if (jj == l0w && w > 0) {
        xhead[w * 64 + lane] = curP;
        if (l0w == n - 1) firstc = curQ;
      }
      if (jj == l0w + 1) firstc = curP;
      if (next_has && jj == l0w + lc - 1) xtail[w * 64 + lane] = curQ;
      const int l = jj - 1;
      if (l >= l0w && l < oend && (l == 0 || l - 1 >= aw)) emit(l, curP, selp(l == 0, prev1Q, prev2m));
      if (jj == n - 1 && n - 1 >= l0w && n - 1 < oend && n - 2 >= aw)
        emit(n - 1, curQ, selp(n - 1 == 1, prev1P, prev1Q));
      prev2m = selp(jj - 1 == 0, prev1P, prev1Q);
      prev1P = curP;
      prev1Q = curQ;
    }
  }
  __syncthreads();
  if (has && w > 0) emit(l0w, firstc, xtail[(w - 1) * 64 + lane]);
  if (has && next_has) emit(l0w + lc - 1, xhead[(w + 1) * 64 + lane], prev2m);
}

template <class T, bool CPLX>
__device__ __forceinline__ void two_step_tile(char *kog_smem, int N, const Mat<T, CPLX> &Mc,
                                              const Mat<T, CPLX> &Mn, int t, const Bufs<T, CPLX> &B0,
                                              const Bufs<T, CPLX> &B1, int wpg, int span, int lc, int bx, int by) {
  two_step_tile_r<T, CPLX>(kog_smem, N, Mc.A, Mc.lda, Mn.A, Mn.lda, t, B0, B1, wpg, span, lc, bx, by);
}

// ---------------------------------------------------------------------------
// Three steps per pass: the lane-shift walk with one more level.  Lane j of a
// wavefront holds the rows of pair j of step t; after the step-t rotation and
// the row exchange it holds the rows of pair j of step t+1 (valid on lanes
// 1..62), after the step-(t+1) rotation and a second exchange those of pair j
// of step t+2 (lanes 2..61), which it rotates and writes: 60 row pairs per
// wavefront.  The columns pass through two delay windows the same way: the
// walk over the column pairs of step t feeds the step-(t+1) column pairs one
// behind, and those feed the step-(t+2) column pairs one further behind.
// The wavefronts of a workgroup take consecutive blocks of 60 row pairs and
// the same run of lc output column pairs, whose rotations of all three steps
// are staged in LDS; each walks two column pairs beyond the run on either
// side (they only fill the windows), so nothing crosses between wavefronts.
// Every entry is computed with the operations of the single-step update.
// ---------------------------------------------------------------------------
constexpr int kShift3Out = 60;

template <class T, bool CPLX> constexpr size_t three_step_lds(int lc) {
  return (size_t)(3 * lc + 6) * sizeof(VPack<T, CPLX>);
}

// the entries of a block in (smaller row, larger row) x (smaller column,
// larger column) order, relabelled by roles: row P or Q of the lane's pair,
// column P or Q of the column pair (rflip: P is the larger row index, cflip:
// P is the larger column index)
template <class T> struct Lab {
  Cx<T> PP, QP, PQ, QQ;
};
template <class T>
__device__ __forceinline__ Lab<T> labelled(bool rflip, bool cflip, Cx<T> b11, Cx<T> b21, Cx<T> b12, Cx<T> b22) {
  return Lab<T>{sel(rflip, sel(cflip, b22, b21), sel(cflip, b12, b11)),
                sel(rflip, sel(cflip, b12, b11), sel(cflip, b22, b21)),
                sel(rflip, sel(cflip, b21, b22), sel(cflip, b11, b12)),
                sel(rflip, sel(cflip, b11, b12), sel(cflip, b21, b22))};
}

// the row exchange from the pairs of one step to those of the next (all
// lanes call it): the next pair j takes the P row of lane j+1 and the Q row
// of lane j-1 (P for j-1 = 0), or its own Q row at the two ends; lo and hi
// are its smaller and larger row, cP and cQ the columns P and Q
template <class T, bool CPLX>
__device__ __forceinline__ void exchange_rows(bool j0, bool kflip, bool lo_own, bool hi_own, const Lab<T> &e,
                                              ColPair<T> &cP, ColPair<T> &cQ) {
  Cx<T> dn = shfl_dn1<T, CPLX>(e.PP), up = shfl_up1<T, CPLX>(sel(j0, e.PP, e.QP));
  cP.lo = sel(lo_own, e.QP, sel(kflip, up, dn));
  cP.hi = sel(hi_own, e.QP, sel(kflip, dn, up));
  dn = shfl_dn1<T, CPLX>(e.PQ);
  up = shfl_up1<T, CPLX>(sel(j0, e.PQ, e.QQ));
  cQ.lo = sel(lo_own, e.QQ, sel(kflip, up, dn));
  cQ.hi = sel(hi_own, e.QQ, sel(kflip, dn, up));
}

// one tile: wavefront w of the workgroup takes row block bxg * wpg + w, the
// workgroup the output column pairs [by * lc, by * lc + lc); all threads of
// the workgroup call it
template <class T, bool CPLX>
__device__ __forceinline__ void three_step_tile(char *smem, int N, T *__restrict__ mc, size_t ldc,
                                                T *__restrict__ mn, size_t ldn, int t, const Bufs<T, CPLX> &B0,
                                                const Bufs<T, CPLX> &B1, const Bufs<T, CPLX> &B2, int wpg, int lc,
                                                int bxg, int by) {
  const Mat<T, CPLX> Mc{mc, ldc}, Mn{mn, ldn};
  const int n = N / 2, Mo = N - 1, t1 = t + 1, t2 = t + 2;
  const int lane = (int)threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);  // wavefront-uniform
  const int bx = bxg * wpg + w;
  const int m0 = by * lc;                                  // output column pairs [m0, mend)
  const int mend = m0 + lc < n ? m0 + lc : n;
  const int aw = m0 >= 2 ? m0 - 2 : 0;                     // walk [aw, bw]
  const int bw = m0 + lc + 1 < n - 1 ? m0 + lc + 1 : n - 1;
  const int l1lo = m0 >= 1 ? m0 - 1 : 0;                   // step-(t+1) column pairs [l1lo, l1hi]
  const int l1hi = m0 + lc < n - 1 ? m0 + lc : n - 1;
  VPack<T, CPLX> *sv0 = (VPack<T, CPLX> *)smem;            // index jj - aw (at most lc + 4)
  VPack<T, CPLX> *sv1 = sv0 + (lc + 4);                    // index l - l1lo (at most lc + 2)
  VPack<T, CPLX> *sv2 = sv1 + (lc + 2);                    // index m - m0 (at most lc)
  for (int i = threadIdx.x; i <= bw - aw; i += blockDim.x) sv0[i] = pack_v<T, CPLX>(load_rot<T, CPLX>(B0, aw + i));
  for (int i = threadIdx.x; i <= l1hi - l1lo; i += blockDim.x)
    sv1[i] = pack_v<T, CPLX>(load_rot<T, CPLX>(B1, l1lo + i));
  for (int i = threadIdx.x; i < mend - m0; i += blockDim.x) sv2[i] = pack_v<T, CPLX>(load_rot<T, CPLX>(B2, m0 + i));
  __syncthreads();

  const int j = bx * kShift3Out - 2 + lane;
  const bool act = j >= 0 && j < n;
  const bool mid = act && lane >= 1 && lane <= 62;
  const bool out = act && lane >= 2 && lane <= kShift3Out + 1;
  int P = 0, Q = 1, a1 = 0, b1 = 0, a2 = 0, b2 = 0;
  RotU<T> u0{}, u1{}, u2{};
  if (act) {
    rows_at(t, j, Mo, P, Q);
    u0 = load_u<T, CPLX>(B0, j);
  }
  if (mid) {
    pair_ab(t1, j, Mo, a1, b1);
    u1 = load_u<T, CPLX>(B1, j);
  }
  if (out) {
    pair_ab(t2, j, Mo, a2, b2);
    u2 = load_u<T, CPLX>(B2, j);
  }
  const bool rflip = P > Q;
  const int rp = rflip ? Q : P, rq = rflip ? P : Q;        // rows of step t's pair j in (p, q) order
  const bool kflip1 = a1 > b1, kflip2 = a2 > b2;
  const int op2 = kflip2 ? b2 : a2, oq2 = kflip2 ? a2 : b2; // rows written
  const bool lo1 = kflip1 ? j == 0 : j == n - 1, hi1 = kflip1 ? j == n - 1 : j == 0;
  const bool lo2 = kflip2 ? j == 0 : j == n - 1, hi2 = kflip2 ? j == n - 1 : j == 0;
  const Cx<T> zero{T(0), T(0)};

  // column pair m of step t+2 from its columns ca(m) (cplus) and cb(m) (cminus), written
  auto level2 = [&](int m, const ColPair<T> &cplus, const ColPair<T> &cminus) {
    int ca, cb;
    pair_ab(t2, m, Mo, ca, cb);
    const bool mflip = ca > cb;
    const int cp = mflip ? cb : ca, cq = mflip ? ca : cb;
    Cx<T> c11 = sel(mflip, cminus.lo, cplus.lo), c21 = sel(mflip, cminus.hi, cplus.hi);
    Cx<T> c12 = sel(mflip, cplus.lo, cminus.lo), c22 = sel(mflip, cplus.hi, cminus.hi);
    if (m == j) {
      c11 = Cx<T>{u2.sp, T(0)};
      c22 = Cx<T>{u2.sq, T(0)};
      c12 = c21 = zero;
    } else {
      Rot<T> r = with_v<T, CPLX>(u2, sv2[m - m0]);
      rotate_block<T, CPLX>(r, r, c11, c21, c12, c22);
    }
    if (out) {
      Mn.st(op2, cp, c11);
      Mn.st(oq2, cp, c21);
      Mn.st(op2, cq, c12);
      Mn.st(oq2, cq, c22);
    }
  };

  // the window over the step-(t+1) column pairs, in increasing order
  ColPair<T> q1P{zero, zero}, q1Q{zero, zero}, q2m{zero, zero};
  int lfirst = -1;
  auto feed2 = [&](int l, const Lab<T> &e) {
    ColPair<T> cP, cQ;
    exchange_rows<T, CPLX>(j == 0, kflip2, lo2, hi2, e, cP, cQ);
    if (lfirst < 0) lfirst = l;
    const int m = l - 1;
    if (m >= m0 && m < mend && (m == 0 ? lfirst == 0 : m - 1 >= lfirst)) level2(m, cP, selp(m == 0, q1Q, q2m));
    if (l == n - 1 && n - 1 >= m0 && n - 1 < mend && n - 2 >= lfirst)
      level2(n - 1, cQ, selp(n - 1 == 1, q1P, q1Q));
    q2m = selp(l - 1 == 0, q1P, q1Q);
    q1P = cP;
    q1Q = cQ;
  };

  // column pair l of step t+1 from its columns ca(l) (cplus) and cb(l) (cminus), rotated, into the window
  auto level1 = [&](int l, const ColPair<T> &cplus, const ColPair<T> &cminus) {
    int ca, cb;
    pair_ab(t1, l, Mo, ca, cb);
    const bool lflip = ca > cb;
    Cx<T> c11 = sel(lflip, cminus.lo, cplus.lo), c21 = sel(lflip, cminus.hi, cplus.hi);
    Cx<T> c12 = sel(lflip, cplus.lo, cminus.lo), c22 = sel(lflip, cplus.hi, cminus.hi);
    if (l == j) {
      c11 = Cx<T>{u1.sp, T(0)};
      c22 = Cx<T>{u1.sq, T(0)};
      c12 = c21 = zero;
    } else {
      Rot<T> r = with_v<T, CPLX>(u1, sv1[l - l1lo]);
      rotate_block<T, CPLX>(r, r, c11, c21, c12, c22);
    }
    feed2(l, labelled<T>(kflip1, lflip, c11, c21, c12, c22));
  };

  struct Blk {
    Cx<T> b11, b21, b12, b22;
  };
  auto load_blk = [&](int jj) -> Blk {
    int Pc, Qc;
    rows_at(t, jj, Mo, Pc, Qc);
    const int cp = Pc < Qc ? Pc : Qc, cq = Pc < Qc ? Qc : Pc;
    Blk d{zero, zero, zero, zero};
    if (act) {
      d.b11 = Mc.ld(rp, cp);
      d.b21 = Mc.ld(rq, cp);
      d.b12 = Mc.ld(rp, cq);
      d.b22 = Mc.ld(rq, cq);
    }
    return d;
  };
  if (bx * kShift3Out >= n) return;  // no rows here (after the only barrier)
  ColPair<T> p1P{zero, zero}, p1Q{zero, zero}, p2m{zero, zero};
  constexpr int D = two_step_depth<T, CPLX>();
  Blk q[D];
#pragma unroll
  for (int d = 0; d < D; ++d) q[d] = aw + d <= bw ? load_blk(aw + d) : Blk{zero, zero, zero, zero};
  for (int jj = aw; jj <= bw; ++jj) {
    const Blk a = q[0];
#pragma unroll
    for (int d = 0; d + 1 < D; ++d) q[d] = q[d + 1];
    if (jj + D <= bw) q[D - 1] = load_blk(jj + D);
    // step t on the block (j, jj), in (p, q) order
    int Pc, Qc;
    rows_at(t, jj, Mo, Pc, Qc);
    Cx<T> b11 = a.b11, b21 = a.b21, b12 = a.b12, b22 = a.b22;
    if (j == jj) {
      b11 = Cx<T>{u0.sp, T(0)};
      b22 = Cx<T>{u0.sq, T(0)};
      b12 = b21 = zero;
    } else {
      Rot<T> r = with_v<T, CPLX>(u0, sv0[jj - aw]);
      rotate_block<T, CPLX>(r, r, b11, b21, b12, b22);
    }
    ColPair<T> curP, curQ;
    exchange_rows<T, CPLX>(j == 0, kflip1, lo1, hi1, labelled<T>(rflip, Pc > Qc, b11, b21, b12, b22), curP, curQ);
    const int l = jj - 1;
    if (l >= l1lo && l <= l1hi && (l == 0 || l - 1 >= aw)) level1(l, curP, selp(l == 0, p1Q, p2m));
    if (jj == n - 1 && n - 1 >= l1lo && n - 1 <= l1hi && n - 2 >= aw)
      level1(n - 1, curQ, selp(n - 1 == 1, p1P, p1Q));
    p2m = selp(jj - 1 == 0, p1P, p1Q);
    p1P = curP;
    p1Q = curQ;
  }
}


// ---------------------------------------------------------------------------
// Accumulated transformations (the SVD entry points).  Section 1 updates the
// iterate by U_k^* from the left and V_k from the right, so with U <- U U_k
// and V <- V V_k after every step A_0 = U A V^* holds throughout.  Each is a
// rotation of the column pair (p, q) of U or V with the rounding order of the
// column half of the block update.
// ---------------------------------------------------------------------------
template <class T> struct W4 {
  Cx<T> w11, w21, w12, w22;
};
template <class T> __device__ __forceinline__ W4<T> w_of(const Rot<T> &r, bool v) {
  return v ? W4<T>{r.v11, r.v21, r.v12, r.v22} : W4<T>{r.u11, r.u21, r.u12, r.u22};
}

// [c1, c2] <- [c1, c2] W
template <class T, bool CPLX> __device__ __forceinline__ void rot_cols(const W4<T> &w, Cx<T> &c1, Cx<T> &c2) {
  if constexpr (CPLX) {
    const Cx<T> o1 = cadd(cmul(c1, w.w11), cmul(c2, w.w21));
    const Cx<T> o2 = cadd(cmul(c1, w.w12), cmul(c2, w.w22));
    c1 = o1;
    c2 = o2;
  } else {
    const T o1 = vfma(c1.re, w.w11.re, c2.re * w.w21.re);
    const T o2 = vfma(c1.re, w.w12.re, c2.re * w.w22.re);
    c1.re = o1;
    c2.re = o2;
  }
}

// One step t in place: grid (ceil(n / ppb), 2), blockIdx.y = 0 rotates U by
// the U_k, 1 rotates V by the V_k.  A workgroup of 256 threads takes ppb =
// 256 / min(N, 256) column pairs; its lanes run down the rows of a pair, so a
// wavefront reads and writes contiguous runs of both columns.
template <class T, bool CPLX>
__global__ __launch_bounds__(256) void kog_accum_kernel(int N, Mat<T, CPLX> U, Mat<T, CPLX> V, int t,
                                                        Bufs<T, CPLX> B) {
  constexpr int G = 4;
  const int n = N / 2, rows = N < 256 ? N : 256, ppb = 256 / rows;
  const int slot = (int)threadIdx.x / rows, l = (int)blockIdx.x * ppb + slot;
  if (slot >= ppb || l >= n) return;
  const bool isv = blockIdx.y != 0;
  const Mat<T, CPLX> X = isv ? V : U;
  int a, b;
  pair_ab(t, l, N - 1, a, b);
  const int p = a < b ? a : b, q = a < b ? b : a;
  const W4<T> w = w_of(load_rot<T, CPLX>(B, l), isv);
  for (int i0 = (int)threadIdx.x % rows; i0 < N; i0 += G * rows) {
    Cx<T> c1[G], c2[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int i = i0 + g * rows;
      if (i < N) {
        c1[g] = X.ld(i, p);
        c2[g] = X.ld(i, q);
      }
    }
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int i = i0 + g * rows;
      if (i < N) {
        rot_cols<T, CPLX>(w, c1[g], c2[g]);
        X.st(i, p, c1[g]);
        X.st(i, q, c2[g]);
      }
    }
  }
}

// S consecutive steps t .. t+S-1 of the accumulation from (U, V) into
// (U2, V2), bitwise S single steps.  Pair j of step tau has the columns
// x_j = (tau + j) mod (N-1) and y_j = (tau - j) mod (N-1) (x_0 = tau,
// y_0 = N-1); pair k of step tau+1 is made of the rotated columns f_k and g_k
// of step tau, where f_k = x_{k+1} (k < n-1) or y_{n-1} (k = n-1), and
// g_k = y_0 (k = 0), x_0 (k = 1) or y_{k-1} (k >= 2).  A lane owns one row
// and walks iterations j: level L takes pair j - L of step t+L, whose x
// column (t + j) mod (N-1) is the same at every level, so the x column
// rotated by level L goes straight on to level L+1 in the same iteration,
// while the y columns wait in a delay line of three entries per level (pair
// 0 enters it as y_0 then x_0, so the second input of the next step's pair
// is always the entry two iterations back).  Pair n of a level past the last
// one stands for f_{n-1}: it hands on the y column of pair n-1, one
// iteration late, which is when the next level takes pair n-1.  Iterations
// where a level's pair is outside its range compute values that never reach
// a written one (their rotation is zero and their delay-line entries are
// shifted out before they are read); only the last level writes, its pairs
// in the workgroup's segment.  Apart from the iterations that meet pair 0 or
// pair n, no level tests anything but the orientation of its rotation (the
// same for the whole wavefront, taken by a branch).  Grid (row blocks of 256
// x segments, 2): segments re-walk a few pairs at their edges, so the output
// is out of place.  The rotations of every level are staged in LDS first,
// and the level-0 columns are loaded three iterations ahead.  Segment
// lengths as measured best at N = 4096: 64 pairs, 32 for complex FP64
// (whose walk holds the most registers).  S = 2 and 4 serve two steps per
// pass (a pair of passes), S = 3 and 6 three steps per pass.
constexpr int kAccMaxS = 6;
// segment length (output pairs per workgroup)
template <class T, bool CPLX> struct AccShape {
  static constexpr int seg = CPLX && sizeof(T) == 8 ? 32 : 64;
};
template <class T, bool CPLX> struct AccSets {
  Bufs<T, CPLX> b[kAccMaxS];  // the rotations of steps t, t+1, ...
};

template <class T, bool CPLX, int S> struct AccRun {
  static constexpr int NIT = AccShape<T, CPLX>::seg + 2 * S - 2;  // iterations of a segment, at most
  static constexpr int D = 3;  // load distance (iterations): one delay-line period
  Mat<T, CPLX> X, Y;
  const W4<T> *ws;  // [level][iteration - jlo]
  int n, M, t, i, jlo, jend, jst, jld, dm;
  bool live;
  int twoL[S];                     // 2L mod M
  Cx<T> ring[S > 1 ? S - 1 : 1][3];  // the y delay lines, indexed by iteration mod 3
  Cx<T> inx[D], iny[D];            // level-0 columns of the next D iterations

  __device__ __forceinline__ void load(int slot, int ca, int cb) {
    if (live) {
      inx[slot] = X.ld(i, ca);
      iny[slot] = X.ld(i, cb);
    }
  }

  // level L of iteration j (PH = (j - jlo) mod 3), x column a, y column b
  template <int L, int PH, bool FAST>
  __device__ __forceinline__ void level(int j, int a, int b0, Cx<T> x, Cx<T> y) {
    int b = b0 + twoL[L];
    if (b >= M) b -= M;
    Cx<T> rx, ry;
    bool virt = false;
    if constexpr (!FAST && L < S - 1) virt = j - L == n;
    if (virt) {
      if constexpr (L < S - 1) rx = ry = ring[L][(PH + 2) % 3];
    } else {
      const W4<T> &w = ws[L * NIT + (j - jlo)];
      if (a > b) {
        Cx<T> c1 = y, c2 = x;
        rot_cols<T, CPLX>(w, c1, c2);
        ry = c1;
        rx = c2;
      } else {
        Cx<T> c1 = x, c2 = y;
        rot_cols<T, CPLX>(w, c1, c2);
        rx = c1;
        ry = c2;
      }
    }
    if constexpr (L == S - 1) {
      if (j >= jst && live) {
        if constexpr (!FAST) b = j - L == 0 ? M : b;
        Y.st(i, a, rx);
        Y.st(i, b, ry);
      }
    } else {
      bool first = false;
      if constexpr (!FAST) first = j - L == 0;
      if (first) {
        ring[L][PH] = rx;
        ring[L][(PH + 2) % 3] = ry;
      } else {
        ring[L][PH] = ry;
      }
      level<L + 1, PH, FAST>(j, a, b0, rx, ring[L][(PH + 1) % 3]);
    }
  }

  // iteration j: its level-0 columns from the load slots, then the loads of
  // iteration j + D; a and b0 are (t + j) mod M and (t - j) mod M
  template <int PH> __device__ __forceinline__ void iter(int j, int &a, int &b0) {
    constexpr int SL = PH;
    const Cx<T> x = inx[SL], y = iny[SL];
    if (j + D <= jld) {
      int ca = a + dm, cb = b0 - dm;
      if (ca >= M) ca -= M;
      if (cb < 0) cb += M;
      load(SL, ca, cb);
    }
    if (j >= S && j < n)
      level<0, PH, true>(j, a, b0, x, y);
    else
      level<0, PH, false>(j, a, b0, x, y);
    a = a + 1 < M ? a + 1 : 0;
    b0 = b0 >= 1 ? b0 - 1 : M - 1;
  }

  __device__ __forceinline__ void walk() {
    const Cx<T> zero{T(0), T(0)};
#pragma unroll
    for (int L = 0; L < S - 1; ++L) ring[L][0] = ring[L][1] = ring[L][2] = zero;
#pragma unroll
    for (int L = 0; L < S; ++L) twoL[L] = (2 * L) % M;
    dm = D % M;
    int a = t + jlo, b0 = t - jlo;
    if (a >= M) a -= M;
    if (b0 < 0) b0 += M;
    // the loads of the first D iterations (pair 0's y column is N-1)
#pragma unroll
    for (int d = 0; d < D; ++d) {
      inx[d] = iny[d] = zero;
      const int j = jlo + d;
      if (j <= jld) {
        int ca = a + d % M, cb = b0 - d % M;
        if (ca >= M) ca -= M;
        if (cb < 0) cb += M;
        load(d, ca, j == 0 ? M : cb);
      }
    }
    // three iterations per trip: one period of the delay lines and of the
    // load slots
    for (int j = jlo; j <= jend; j += 3) {
      iter<0>(j, a, b0);
      if (j + 1 > jend) break;
      iter<1>(j + 1, a, b0);
      if (j + 2 > jend) break;
      iter<2>(j + 2, a, b0);
    }
  }
};

// Waves per SIMD at least: 3 for the six-level complex FP64 walk (capped at
// the 128 VGPRs of 4 it spills 212 bytes per lane and its SVD sweep at
// N = 4096 takes 80 % longer than with 168 and 44 bytes spilled), 4 for the
// others (the four-level complex FP64 walk: 128 VGPRs, 12 bytes spilled).
template <class T, bool CPLX> constexpr int acc_min_waves(int S) { return CPLX && sizeof(T) == 8 && S > 4 ? 3 : 4; }
template <class T, bool CPLX, int S>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(acc_min_waves<T, CPLX>(S), 8))) void kog_accum_s_kernel(int N, Mat<T, CPLX> U, Mat<T, CPLX> V,
                                                          Mat<T, CPLX> U2, Mat<T, CPLX> V2, int t,
                                                          AccSets<T, CPLX> R) {
  static_assert(S >= 2 && S <= kAccMaxS, "levels");
  constexpr int SEG = AccShape<T, CPLX>::seg, NIT = AccRun<T, CPLX, S>::NIT;
  __shared__ W4<T> ws[S * NIT];
  const int n = N / 2;
  const int rb = (N + 255) / 256, nseg = (n + SEG - 1) / SEG;
  const int blk = (int)blockIdx.x % rb, sg = (int)blockIdx.x / rb;
  if (sg >= nseg) return;
  const int tid = (int)threadIdx.x;
  const bool isv = blockIdx.y != 0;
  AccRun<T, CPLX, S> A;
  A.X = isv ? V : U;
  A.Y = isv ? V2 : U2;
  A.n = n;
  A.M = N - 1;
  A.t = t;
  A.i = blk * 256 + tid;
  A.live = A.i < N;
  const int k0 = sg * SEG, k1 = k0 + SEG < n ? k0 + SEG : n;  // output pairs [k0, k1)
  A.jlo = k0 >= S - 1 ? k0 - (S - 1) : 0;
  A.jend = k1 + S - 2;
  A.jst = k0 + S - 1;                              // the last level's pairs from k0 on are written
  A.jld = A.jend < n - 1 ? A.jend : n - 1;         // iterations with level-0 columns to load
  const int nit = A.jend - A.jlo + 1;
  const W4<T> wz{{T(0), T(0)}, {T(0), T(0)}, {T(0), T(0)}, {T(0), T(0)}};
#pragma unroll
  for (int L = 0; L < S; ++L) {
    // level L takes the pairs [lo, hi] of step t+L
    const int lo = k0 >= S - 1 - L ? k0 - (S - 1 - L) : 0;
    const int hi = k1 - 1 + (S - 1 - L) < n - 1 ? k1 - 1 + (S - 1 - L) : n - 1;
    for (int q = tid; q < nit; q += 256) {
      const int p = A.jlo + q - L;
      ws[L * NIT + q] = (p >= lo && p <= hi) ? w_of(load_rot<T, CPLX>(R.b[L], p), isv) : wz;
    }
  }
  A.ws = ws;
  __syncthreads();
  A.walk();
}

template <class T, bool CPLX>
__global__ __launch_bounds__(256) void kog_copy_kernel(int N, Mat<T, CPLX> src, Mat<T, CPLX> dst) {
  for (int j = blockIdx.x; j < N; j += gridDim.x)
    for (int i = threadIdx.x; i < N; i += blockDim.x) dst.st(i, j, src.ld(i, j));
}

// Exact power-of-two scaling of the whole matrix around a solve (the idea of
// eq. (2) applied to A): with E the largest binary exponent among the finite
// nonzero components, the solve works on 2^-E A and returns 2^E times the
// result.  The steps commute with the factor exactly (each 2x2 SVD scales its
// pivot exactly and the rotations do not depend on scale) unless a value
// reaches the subnormal range, while the stopping test's sums of squares can
// neither overflow nor underflow to zero.
constexpr int kNoExp = -0x7fffffff - 1;  // no finite nonzero component

template <class T> __device__ __forceinline__ int comp_exp(T x) {
  return (x != T(0) && __builtin_isfinite(x)) ? vfrexp_exp(x) : kNoExp;
}
template <class T> __device__ __forceinline__ int elem_exp(Cx<T> v) {
  const int a = comp_exp(v.re), b = comp_exp(v.im);
  return a > b ? a : b;
}

// A <- 2^e A, every component
template <class T, bool CPLX>
__global__ __launch_bounds__(256) void kog_scale_kernel(int N, Mat<T, CPLX> M, int e) {
  for (int j = blockIdx.x; j < N; j += gridDim.x)
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
      const Cx<T> v = M.ld(i, j);
      M.st(i, j, Cx<T>{vldexp(v.re, e), vldexp(v.im, e)});
    }
}

// host helpers defined in kog.hip
svd2_status hip_st(hipError_t e);  // maps a HIP error, recording it for kog_last_hip_error
TileRule rule_for(int N);          // single-step update tile shape by order

}  // namespace kog
