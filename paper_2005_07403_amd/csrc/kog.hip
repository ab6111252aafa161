// kog.hip -- Kogbetliantz method for the SVD of a square matrix of even order
// N = 2n on gfx950, built on the batched 2x2 SVD (section 1 of the paper:
// one parallel step gathers the pivots (p,p), (q,p), (p,q), (q,q) of n
// disjoint pairs, computes their 2x2 SVDs, and updates rows p,q from the left
// by U_k^* and columns p,q from the right by V_k).
//
// Pivot ordering (not given by the paper): the circle-method round robin in
// closed form.  At step t (0 <= t < N-1), M = N-1: pair 0 = (t, M) and pair
// k >= 1 = ((t+k) mod M, (t-k) mod M), oriented p < q.  For consecutive k the
// rows (t+k) mod M run forward and (t-k) mod M run backward through memory,
// so a wavefront reads and writes both rows of its pairs as contiguous runs:
// the in-place update is coalesced without LDS staging or a second buffer,
// and the matrix keeps a footprint that fits the 256 MB Infinity Cache for
// N = 4096 in FP64.
//
// Pivot placement (reading): if |b_pp| < |b_qq| the columns of U_k and V_k and
// the two singular values are swapped, so sigma_min goes to (p,p); with the
// descending order of Theorem 1 alone the sweep keeps re-sorting the diagonal
// and converges only linearly.
//
// Two drivers per step: an unfused chain (gather kernel -> batched SVD entry
// point -> update kernel, optionally replayed from a hipGraph per sweep) and a
// fused persistent cooperative kernel that runs all steps of a sweep with two
// grid barriers per step.
#include "svd2.h"

#include <hip/hip_runtime.h>

#include <stdint.h>
#include <string.h>

#include <vector>

#include "svd2_lane.hpp"

using namespace svd2;

namespace {

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
};
constexpr int kMaxFusedBlocks = 4096;  // barrier slots (64 bytes each)

Layout layout(int N, size_t esz, bool cplx) {
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
  return L;
}

template <class T, bool CPLX> Bufs<T, CPLX> make_bufs(void *ws, int N, int set = 0) {
  Layout L = layout(N, sizeof(T), CPLX);
  auto up = [](size_t x) { return (x + 255) & ~size_t(255); };
  size_t arr = up((size_t)(N / 2) * sizeof(T));
  Bufs<T, CPLX> b;
  char *base = (char *)ws;
  size_t piv = set ? L.piv1 : L.piv, out = set ? L.out1 : L.out;
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

template <class T, bool CPLX>
__global__ __launch_bounds__(256) void kog_gather_kernel(int N, Mat<T, CPLX> M, int t,
                                                         Bufs<T, CPLX> B) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= N / 2) return;
  T x[Bufs<T, CPLX>::NIN];
  gather_one<T, CPLX>(M, N, t, k, x);
#pragma unroll
  for (int i = 0; i < Bufs<T, CPLX>::NIN; ++i) B.piv[i][k] = x[i];
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

template <class T, bool CPLX>
__global__ __launch_bounds__(kUpdBlock) void kog_update_kernel(int N, Mat<T, CPLX> M, int t,
                                                               Bufs<T, CPLX> B, int kc, int lc) {
  update_tile<T, CPLX, false>(M, N, t, B, Tile{(int)blockIdx.x * kc, kc, (int)blockIdx.y * lc, lc});
}

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

// gather + 2x2 SVD of the pivots of step t in one kernel
template <class T, bool CPLX>
__global__ __launch_bounds__(256) void kog_pivot_kernel(int N, Mat<T, CPLX> M, int t, Bufs<T, CPLX> B) {
  constexpr int RESC = sizeof(T) == 4 ? 1 : 0;
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= N / 2) return;
  T x[Bufs<T, CPLX>::NIN], y[Bufs<T, CPLX>::NOUT];
  gather_one<T, CPLX>(M, N, t, k, x);
  one_matrix<T, CPLX, RESC>(x, y, 2);
#pragma unroll
  for (int i = 0; i < Bufs<T, CPLX>::NIN; ++i) B.piv[i][k] = x[i];
#pragma unroll
  for (int i = 0; i < Bufs<T, CPLX>::NOUT; ++i) B.out[i][k] = y[i];
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

template <class T, bool CPLX>
__global__ __launch_bounds__(256) void kog_pivots2_kernel(int N, Mat<T, CPLX> M, int t, Bufs<T, CPLX> B0,
                                                          Bufs<T, CPLX> B1) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < N / 2) pivots2_one<T, CPLX>(N, M, t, B0, B1, k);
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

template <class T, bool CPLX> __device__ __forceinline__ Cx<T> shfl_dn1(Cx<T> x) {
  Cx<T> r;
  r.re = __shfl_down(x.re, 1, 64);
  if constexpr (CPLX) r.im = __shfl_down(x.im, 1, 64);
  else r.im = T(0);
  return r;
}
template <class T, bool CPLX> __device__ __forceinline__ Cx<T> shfl_up1(Cx<T> x) {
  Cx<T> r;
  r.re = __shfl_up(x.re, 1, 64);
  if constexpr (CPLX) r.im = __shfl_up(x.im, 1, 64);
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
    Blk nx = load_blk(aw);  // the block of the next iteration is in flight
    for (int jj = aw; jj <= bw; ++jj) {
      const Blk a = nx;
      if (jj < bw) nx = load_blk(jj + 1);
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

template <class T, bool CPLX>
__global__ __launch_bounds__(256) void kog_two_step_kernel(int N, Mat<T, CPLX> Mc, Mat<T, CPLX> Mn, int t,
                                                           Bufs<T, CPLX> B0, Bufs<T, CPLX> B1, int wpg,
                                                           int span, int lc, int gx, int ntiles) {
  extern __shared__ __align__(16) char kog_smem[];
  const int tile = xcd_tile((int)blockIdx.x, ntiles);
  two_step_tile<T, CPLX>(kog_smem, N, Mc, Mn, t, B0, B1, wpg, span, lc, tile % gx, tile / gx);
}

template <class T, bool CPLX>
__global__ __launch_bounds__(256) void kog_copy_kernel(int N, Mat<T, CPLX> src, Mat<T, CPLX> dst) {
  for (int j = blockIdx.x; j < N; j += gridDim.x)
    for (int i = threadIdx.x; i < N; i += blockDim.x) dst.st(i, j, src.ld(i, j));
}

// ---------------------------------------------------------------------------
// fused persistent sweep: for t in [t0, t1): gather + SVD, barrier, update, barrier
// ---------------------------------------------------------------------------
// Grid-wide barrier for a cooperative launch (all workgroups co-resident),
// without a contended counter: workgroup g publishes the barrier epoch in its
// own 64-byte slot flags[16 g]; the first wavefront of workgroup 0 polls all
// slots and then publishes the epoch in bar->gen, which the other workgroups
// poll.  Memory ordering at agent scope: a release before publishing (one L2
// write-back), relaxed polling (no cache invalidation per poll), one acquire
// after.  Every wait is bounded: after kSpinLimit polls the waiter sets the
// abort flag, all workgroups leave their loops, and the kernel terminates.
__device__ __forceinline__ bool spin_until(const unsigned *word, unsigned epoch, Bar *bar) {
  unsigned spins = 0;
  while (__hip_atomic_load(word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < epoch) {
    __builtin_amdgcn_s_sleep(1);
    if (++spins > kSpinLimit) {
      __hip_atomic_store(&bar->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return false;
    }
    if ((spins & 255u) == 0 && __hip_atomic_load(&bar->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
      return false;
  }
  return true;
}

__device__ __forceinline__ bool grid_sync(Bar *bar, unsigned *flags, unsigned nblocks, unsigned &epoch) {
  __shared__ unsigned s_abort;
  const unsigned e = ++epoch;
  __syncthreads();
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __hip_atomic_store(&flags[16 * blockIdx.x], e, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  if (blockIdx.x == 0) {
    if (threadIdx.x < 64) {
      bool ok = true;
      for (unsigned g = threadIdx.x; g < nblocks && ok; g += 64) ok = spin_until(&flags[16 * g], e, bar);
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __hip_atomic_store(&bar->gen, e, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
  } else if (threadIdx.x == 0) {
    spin_until(&bar->gen, e, bar);
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  if (threadIdx.x == 0) s_abort = __hip_atomic_load(&bar->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  return s_abort == 0;
}

template <class T, bool CPLX>
__global__ __launch_bounds__(kUpdBlock) void kog_fused_kernel(int N, Mat<T, CPLX> M, int t0, int t1,
                                                              Bufs<T, CPLX> B, Bar *bar,
                                                              unsigned *flags, int kc, int lc) {
  constexpr bool RESC = sizeof(T) == 4;
  const int n = N / 2;
  const unsigned G = gridDim.x;
  const int kt = (n + kc - 1) / kc, lt = (n + lc - 1) / lc;
  unsigned epoch = 0;  // barrier epochs restart at 1 in every launch
  for (int t = t0; t < t1; ++t) {
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += G * blockDim.x) {
      T x[Bufs<T, CPLX>::NIN], y[Bufs<T, CPLX>::NOUT];
      gather_one<T, CPLX>(M, N, t, k, x);
      one_matrix<T, CPLX, RESC ? 1 : 0>(x, y, 2);
#pragma unroll
      for (int i = 0; i < Bufs<T, CPLX>::NIN; ++i) B.piv[i][k] = x[i];
#pragma unroll
      for (int i = 0; i < Bufs<T, CPLX>::NOUT; ++i) B.out[i][k] = y[i];
    }
    if (!grid_sync(bar, flags, G, epoch)) return;
    for (int tile = blockIdx.x; tile < kt * lt; tile += G)
      update_tile<T, CPLX, false>(M, N, t, B, Tile{(tile % kt) * kc, kc, (tile / kt) * lc, lc});
    if (!grid_sync(bar, flags, G, epoch)) return;
  }
}

__global__ void kog_bar_reset_kernel(Bar *bar, unsigned *flags, int nflags) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) {
    bar->count = 0;
    bar->gen = 0;
    bar->abort = 0;
  }
  if (i < nflags) flags[16 * i] = 0;
}

// ---------------------------------------------------------------------------
// off(A)^2 and ||A||_F^2 in FP64: fixed-order two-pass reduction
// ---------------------------------------------------------------------------
template <class T, bool CPLX>
__global__ __launch_bounds__(256) void kog_norm_partial_kernel(int N, Mat<T, CPLX> M, double *part) {
  __shared__ double so[256], st[256];
  double off = 0, tot = 0;
  for (int j = blockIdx.x; j < N; j += gridDim.x)
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
      Cx<T> v = M.ld(i, j);
      double a2 = (double)v.re * (double)v.re + (double)v.im * (double)v.im;
      tot += a2;
      if (i != j) off += a2;
    }
  so[threadIdx.x] = off;
  st[threadIdx.x] = tot;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      so[threadIdx.x] += so[threadIdx.x + s];
      st[threadIdx.x] += st[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = so[0];
    part[2 * blockIdx.x + 1] = st[0];
  }
}

__global__ __launch_bounds__(256) void kog_norm_final_kernel(int nparts, const double *part, double *res) {
  __shared__ double so[256], st[256];
  double off = 0, tot = 0;
  for (int i = threadIdx.x; i < nparts; i += blockDim.x) {
    off += part[2 * i];
    tot += part[2 * i + 1];
  }
  so[threadIdx.x] = off;
  st[threadIdx.x] = tot;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      so[threadIdx.x] += so[threadIdx.x + s];
      st[threadIdx.x] += st[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    res[0] = so[0];
    res[1] = st[0];
  }
}


// ---------------------------------------------------------------------------
// Many problems of uneven order and mixed element type in one launch per
// phase.  A step of the batch is three kernels over a static work list:
// pivot chunks (gather + 2x2 SVD) of every active problem, update tiles of
// every active problem (each with its own tile shape and the off-diagonal mass
// it wrote), and a per-problem finish (advance the step, and at the end of a
// problem's sweep decide convergence on the device).  The host replays a
// hipGraph of K such steps and reads one counter per replay.
//
// In the two-step mode a pass takes every running problem two steps further
// (pivots of both steps, then the two-step tiles, out of place between the
// problem's matrix and a second one in the workspace), except the last step
// of a sweep (t = N-2; a sweep has an odd number of steps), which is a single
// in-place step with the convergence test as above.  The work list holds the
// tiles of both kinds; a tile of the kind a problem does not need in this
// pass returns at once.
// ---------------------------------------------------------------------------
struct DevProb {
  void *A;
  long long lda, piv_off, out_off;  // buffer offsets in bytes from the workspace base
  long long piv1_off, out1_off;     // second rotation set (two-step mode)
  long long w_off;                  // second matrix (two-step mode), lda = N
  int N, kind, kc, lc;
  int part_off, ntiles, max_sweeps, in_w;  // in_w: the iterate is in the second matrix
  int gx2, ny2, lc2, pad0;          // two-step tiles: row blocks, column tiles, pairs per wavefront
  double tol, tot0;                 // tot0 = ||A_0||_F
  int t, sweeps, status, pad1;      // status: 0 running, 1 converged, 2 max_sweeps reached
  double off_rel;
};
struct BatchHdr {
  int nA, nB, nprob, active;
  int c0[5];  // two-step tiles of element type k: items [c0[k], c0[k+1])
  int pad[3];
};

__host__ __device__ inline size_t arr_bytes(int N, int esz) {
  return (((size_t)(N / 2) * esz) + 255) & ~size_t(255);
}

template <class T, bool CPLX>
__device__ __forceinline__ Bufs<T, CPLX> bufs_of(char *ws, const DevProb &P, int set = 0) {
  Bufs<T, CPLX> b;
  size_t arr = arr_bytes(P.N, sizeof(T));
  const long long po = set ? P.piv1_off : P.piv_off, oo = set ? P.out1_off : P.out_off;
  for (int i = 0; i < Bufs<T, CPLX>::NIN; ++i) b.piv[i] = (T *)(ws + po + i * arr);
  for (int i = 0; i < Bufs<T, CPLX>::NOUT; ++i) b.out[i] = (T *)(ws + oo + i * arr);
  return b;
}

// the matrix that holds the iterate (other = false) or the other one
template <class T, bool CPLX>
__device__ __forceinline__ Mat<T, CPLX> mat_of(char *ws, const DevProb &P, bool other = false) {
  if (P.in_w != (other ? 1 : 0)) return Mat<T, CPLX>{(T *)(ws + P.w_off), (size_t)P.N};
  return Mat<T, CPLX>{(T *)P.A, (size_t)P.lda};
}

template <class T, bool CPLX> __device__ __forceinline__ void batch_pivot(char *ws, const DevProb &P, int k) {
  constexpr int RESC = sizeof(T) == 4 ? 1 : 0;
  Mat<T, CPLX> M = mat_of<T, CPLX>(ws, P);
  Bufs<T, CPLX> B = bufs_of<T, CPLX>(ws, P);
  T x[Bufs<T, CPLX>::NIN], y[Bufs<T, CPLX>::NOUT];
  gather_one<T, CPLX>(M, P.N, P.t, k, x);
  one_matrix<T, CPLX, RESC>(x, y, 2);
#pragma unroll
  for (int i = 0; i < Bufs<T, CPLX>::NIN; ++i) B.piv[i][k] = x[i];
#pragma unroll
  for (int i = 0; i < Bufs<T, CPLX>::NOUT; ++i) B.out[i][k] = y[i];
}

template <class T, bool CPLX> __device__ __forceinline__ void batch_pivots2(char *ws, const DevProb &P, int k) {
  pivots2_one<T, CPLX>(P.N, mat_of<T, CPLX>(ws, P), P.t, bufs_of<T, CPLX>(ws, P, 0), bufs_of<T, CPLX>(ws, P, 1),
                       k);
}

template <class T, bool CPLX> __device__ __forceinline__ double batch_update(char *ws, const DevProb &P, Tile tl) {
  return update_tile<T, CPLX, true>(mat_of<T, CPLX>(ws, P), P.N, P.t, bufs_of<T, CPLX>(ws, P), tl);
}

template <class T, bool CPLX>
__device__ __forceinline__ void batch_two_step(char *smem, char *ws, const DevProb &P, int bx, int by) {
  two_step_tile<T, CPLX>(smem, P.N, mat_of<T, CPLX>(ws, P), mat_of<T, CPLX>(ws, P, true), P.t,
                         bufs_of<T, CPLX>(ws, P, 0), bufs_of<T, CPLX>(ws, P, 1), kUpdBlock / 64,
                         (kUpdBlock / 64) * P.lc2, P.lc2, bx, by);
}

template <class T, bool CPLX> __device__ __forceinline__ void batch_norm(const DevProb &P, double &off, double &tot) {
  Mat<T, CPLX> M{(T *)P.A, (size_t)P.lda};
  for (int j = 0; j < P.N; ++j)
    for (int i = threadIdx.x; i < P.N; i += blockDim.x) {
      double a2 = abs2(M.ld(i, j));
      tot += a2;
      if (i != j) off += a2;
    }
}

// this pass takes problem P two steps further
__device__ __forceinline__ bool two_this_pass(int two, const DevProb &P) { return two && P.t + 1 < P.N - 1; }

__device__ __forceinline__ double block_sum(double v, double *red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int s = kUpdBlock / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  double r = red[0];
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(kUpdBlock) void kog_batch_init_kernel(BatchHdr *hdr, DevProb *probs) {
  __shared__ double red[kUpdBlock];
  for (int p = blockIdx.x; p < hdr->nprob; p += gridDim.x) {
    DevProb &P = probs[p];
    double off = 0, tot = 0;
    switch (P.kind) {
      case SVD2_KOG_F64: batch_norm<double, false>(P, off, tot); break;
      case SVD2_KOG_C128: batch_norm<double, true>(P, off, tot); break;
      case SVD2_KOG_F32: batch_norm<float, false>(P, off, tot); break;
      default: batch_norm<float, true>(P, off, tot); break;
    }
    off = block_sum(off, red);
    tot = block_sum(tot, red);
    if (threadIdx.x == 0) {
      double nrm = __builtin_sqrt(tot);
      double rel = nrm > 0 ? __builtin_sqrt(off) / nrm : 0.0;
      P.tot0 = nrm;
      P.off_rel = rel;
      P.t = 0;
      P.sweeps = 0;
      P.status = (rel < P.tol || nrm == 0) ? 1 : (P.max_sweeps == 0 ? 2 : 0);
      if (P.status != 0) atomicSub(&hdr->active, 1);
    }
  }
}

__global__ __launch_bounds__(kUpdBlock) void kog_batch_pivot_kernel(char *ws, const BatchHdr *hdr,
                                                                    const int2 *items, const DevProb *probs,
                                                                    int two) {
  const int nA = hdr->nA;
  for (int it = blockIdx.x; it < nA; it += gridDim.x) {
    const int2 item = items[it];
    const DevProb &P = probs[item.x];
    if (P.status != 0 || two_this_pass(two, P)) continue;
    const int k = item.y * kUpdBlock + (int)threadIdx.x;
    if (k >= P.N / 2) continue;
    switch (P.kind) {
      case SVD2_KOG_F64: batch_pivot<double, false>(ws, P, k); break;
      case SVD2_KOG_C128: batch_pivot<double, true>(ws, P, k); break;
      case SVD2_KOG_F32: batch_pivot<float, false>(ws, P, k); break;
      default: batch_pivot<float, true>(ws, P, k); break;
    }
  }
}

// the pivots of both steps of the problems of one element type in a
// two-step pass
template <class T, bool CPLX, int KIND>
__global__ __launch_bounds__(kUpdBlock) void kog_batch_pivots2_kernel(char *ws, const BatchHdr *hdr,
                                                                      const int2 *items, const DevProb *probs) {
  const int nA = hdr->nA;
  for (int it = blockIdx.x; it < nA; it += gridDim.x) {
    const int2 item = items[it];
    const DevProb &P = probs[item.x];
    if (P.kind != KIND || P.status != 0 || !two_this_pass(1, P)) continue;
    const int k = item.y * kUpdBlock + (int)threadIdx.x;
    if (k < P.N / 2) batch_pivots2<T, CPLX>(ws, P, k);
  }
}

// the two-step tiles (problem, row block, column tile) of the problems of one
// element type in a two-step pass
// (at least 3 wavefronts per SIMD: the complex FP64 instance would otherwise
// take 171 VGPRs and run at 2; measured 3.5 % faster on the uneven batch)
template <class T, bool CPLX, int KIND>
__global__ __launch_bounds__(kUpdBlock, 3) void kog_batch_two_step_kernel(char *ws, const BatchHdr *hdr,
                                                                       const int4 *items, const DevProb *probs) {
  extern __shared__ __align__(16) char kog_smem[];
  const int c0 = hdr->c0[KIND], c1 = hdr->c0[KIND + 1];
  for (int it = c0 + (int)blockIdx.x; it < c1; it += gridDim.x) {
    const int4 item = items[it];
    const DevProb &P = probs[item.x];
    if (P.status != 0 || !two_this_pass(1, P)) continue;
    batch_two_step<T, CPLX>(kog_smem, ws, P, item.y, item.z);
    __syncthreads();  // the next item reuses the LDS
  }
}

// single-step update tiles (problem, k0, l0, partial index) of the problems
// not in a two-step pass
__global__ __launch_bounds__(kUpdBlock) void kog_batch_update_kernel(char *ws, const BatchHdr *hdr,
                                                                     const int4 *items, const DevProb *probs,
                                                                     double *partials, int two) {
  __shared__ double red[kUpdBlock];
  const int nB = hdr->nB;
  for (int it = blockIdx.x; it < nB; it += gridDim.x) {
    const int4 item = items[it];
    const DevProb &P = probs[item.x];
    if (P.status != 0 || two_this_pass(two, P)) continue;
    const Tile tl{item.y, P.kc, item.z, P.lc};
    double off2;
    switch (P.kind) {
      case SVD2_KOG_F64: off2 = batch_update<double, false>(ws, P, tl); break;
      case SVD2_KOG_C128: off2 = batch_update<double, true>(ws, P, tl); break;
      case SVD2_KOG_F32: off2 = batch_update<float, false>(ws, P, tl); break;
      default: off2 = batch_update<float, true>(ws, P, tl); break;
    }
    off2 = block_sum(off2, red);
    if (threadIdx.x == 0) partials[P.part_off + item.w] = off2;
  }
}

__global__ __launch_bounds__(kUpdBlock) void kog_batch_finish_kernel(BatchHdr *hdr, DevProb *probs,
                                                                     const double *partials, int two) {
  __shared__ double red[kUpdBlock];
  for (int p = blockIdx.x; p < hdr->nprob; p += gridDim.x) {
    DevProb &P = probs[p];
    // every thread reads the state before thread 0 changes it
    const int status = P.status, t = P.t, N = P.N;
    __syncthreads();
    if (status != 0) continue;
    if (two && t + 1 < N - 1) {  // a two-step pass: no sweep ends inside it
      if (threadIdx.x == 0) {
        P.t = t + 2;
        P.in_w ^= 1;
      }
      continue;
    }
    const bool sweep_end = t == N - 2;
    double off2 = 0;
    if (sweep_end) {
      for (int i = threadIdx.x; i < P.ntiles; i += blockDim.x) off2 += partials[P.part_off + i];
      off2 = block_sum(off2, red);
    }
    if (threadIdx.x == 0) {
      if (sweep_end) {
        int sw = P.sweeps + 1;
        double rel = P.tot0 > 0 ? __builtin_sqrt(off2) / P.tot0 : 0.0;
        P.sweeps = sw;
        P.off_rel = rel;
        if (rel < P.tol) P.status = 1;
        else if (sw >= P.max_sweeps) P.status = 2;
        if (P.status != 0) atomicSub(&hdr->active, 1);
      }
      P.t = t + 1 == N - 1 ? 0 : t + 1;
    }
  }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
thread_local int g_kog_hip = 0;
int g_fused_per_cu = 1;  // co-resident workgroups per CU used by the fused kernel
TileRule g_rules[kMaxRules] = {default_rule()};
int g_nrules = 1;

TileRule rule_for(int N) {
  for (int i = 0; i < g_nrules; ++i)
    if (N <= g_rules[i].max_order) return g_rules[i];
  return default_rule();
}

// two-step kernel shapes: kc = wavefronts per workgroup, lc = column pairs per tile
TileRule default_rule2() { return TileRule{0x7fffffff, 4, 8}; }
TileRule g_rules2[kMaxRules] = {default_rule2()};
int g_nrules2 = 1;
TileRule rule2_for(int N) {
  for (int i = 0; i < g_nrules2; ++i)
    if (N <= g_rules2[i].max_order) return g_rules2[i];
  return default_rule2();
}

svd2_status hip_st(hipError_t e) {
  if (e == hipSuccess) return SVD2_OK;
  g_kog_hip = (int)e;
  return SVD2_ERR_HIP;
}

template <class T, bool CPLX> struct Ctx {
  int N;
  Mat<T, CPLX> M;
  Bufs<T, CPLX> B, B1;
  Mat<T, CPLX> W;  // two-step mode: the second matrix buffer (lda = N)
  Layout L;
  char *ws;
  unsigned flags;
  hipStream_t st;
};

template <class T, bool CPLX>
svd2_status validate(int N, T *A, int lda, void *ws, size_t ws_bytes, unsigned flags, Ctx<T, CPLX> &c) {
  if (!A || !ws) return SVD2_ERR_NULL;
  if (N < 2 || N % 2 || lda < N || N > (1 << 19)) return SVD2_ERR_SIZE;
  if (flags & ~(unsigned)(SVD2_KOG_UNFUSED | SVD2_KOG_GRAPH | SVD2_KOG_TWO_STEP)) return SVD2_ERR_FLAGS;
  if ((flags & SVD2_KOG_GRAPH) && !(flags & SVD2_KOG_UNFUSED)) return SVD2_ERR_FLAGS;
  if ((flags & SVD2_KOG_TWO_STEP) && (flags & (SVD2_KOG_UNFUSED | SVD2_KOG_GRAPH))) return SVD2_ERR_FLAGS;
  if ((uintptr_t)A % (CPLX ? 2 * sizeof(T) : sizeof(T))) return SVD2_ERR_ALIGN;
  if ((uintptr_t)ws % 256) return SVD2_ERR_ALIGN;
  c.L = layout(N, sizeof(T), CPLX);
  const size_t need = (flags & SVD2_KOG_TWO_STEP) ? c.L.total2 : c.L.total;
  if (ws_bytes < need) return SVD2_ERR_SIZE;
  size_t abytes = ((size_t)lda * (N - 1) + N) * sizeof(T) * (CPLX ? 2 : 1);
  uintptr_t a0 = (uintptr_t)A, a1 = a0 + abytes, w0 = (uintptr_t)ws, w1 = w0 + need;
  if (a0 < w1 && w0 < a1) return SVD2_ERR_ALIAS;
  c.N = N;
  c.M = Mat<T, CPLX>{A, (size_t)lda};
  c.B = make_bufs<T, CPLX>(ws, N, 0);
  c.B1 = make_bufs<T, CPLX>(ws, N, 1);
  c.W = Mat<T, CPLX>{(T *)((char *)ws + c.L.mat), (size_t)N};
  c.ws = (char *)ws;
  c.flags = flags;
  return SVD2_OK;
}

// the batched 2x2 SVD of the gathered pivots, backscaled (FP32: with the FP64 rescue)
template <class T, bool CPLX> svd2_status batch_svd(const Ctx<T, CPLX> &c);
template <> svd2_status batch_svd<double, false>(const Ctx<double, false> &c) {
  dsvd2_args a = {c.B.piv[0], c.B.piv[1], c.B.piv[2], c.B.piv[3], c.B.out[0], c.B.out[1], c.B.out[2],
                  c.B.out[3], c.B.out[4], c.B.out[5], c.B.out[6], c.B.out[7], c.B.out[8], c.B.out[9],
                  c.B.out[10]};
  return dsvd2_batch(c.N / 2, &a, SVD2_BACKSCALE_ALL, c.st);
}
template <> svd2_status batch_svd<double, true>(const Ctx<double, true> &c) {
  const Bufs<double, true> &b = c.B;
  zsvd2_args a = {b.piv[0], b.piv[1], b.piv[2], b.piv[3], b.piv[4], b.piv[5], b.piv[6], b.piv[7],
                  b.out[0], b.out[1], b.out[2], b.out[3], b.out[4], b.out[5], b.out[6], b.out[7],
                  b.out[8], b.out[9], b.out[10], b.out[11], b.out[12], b.out[13], b.out[14],
                  b.out[15], b.out[16], b.out[17], b.out[18]};
  return zsvd2_batch(c.N / 2, &a, SVD2_BACKSCALE_ALL, c.st);
}
template <> svd2_status batch_svd<float, false>(const Ctx<float, false> &c) {
  ssvd2_args a = {c.B.piv[0], c.B.piv[1], c.B.piv[2], c.B.piv[3], c.B.out[0], c.B.out[1], c.B.out[2],
                  c.B.out[3], c.B.out[4], c.B.out[5], c.B.out[6], c.B.out[7], c.B.out[8], c.B.out[9],
                  c.B.out[10], nullptr};
  return ssvd2_batch(c.N / 2, &a, SVD2_BACKSCALE_ALL | SVD2_RESCUE_FP64, nullptr, 0, c.st);
}
template <> svd2_status batch_svd<float, true>(const Ctx<float, true> &c) {
  const Bufs<float, true> &b = c.B;
  csvd2_args a = {b.piv[0], b.piv[1], b.piv[2], b.piv[3], b.piv[4], b.piv[5], b.piv[6], b.piv[7],
                  b.out[0], b.out[1], b.out[2], b.out[3], b.out[4], b.out[5], b.out[6], b.out[7],
                  b.out[8], b.out[9], b.out[10], b.out[11], b.out[12], b.out[13], b.out[14],
                  b.out[15], b.out[16], b.out[17], b.out[18], nullptr};
  return csvd2_batch(c.N / 2, &a, SVD2_BACKSCALE_ALL | SVD2_RESCUE_FP64, nullptr, 0, c.st);
}

template <class T, bool CPLX> svd2_status unfused_step(const Ctx<T, CPLX> &c, int t) {
  const int n = c.N / 2;
  hipLaunchKernelGGL((kog_gather_kernel<T, CPLX>), dim3((n + 255) / 256), dim3(256), 0, c.st, c.N, c.M,
                     t, c.B);
  svd2_status s = hip_st(hipGetLastError());
  if (s != SVD2_OK) return s;
  s = batch_svd<T, CPLX>(c);
  if (s != SVD2_OK) return s;
  TileRule r = rule_for(c.N);
  dim3 grid((n + r.kc - 1) / r.kc, (n + r.lc - 1) / r.lc);
  hipLaunchKernelGGL((kog_update_kernel<T, CPLX>), grid, dim3(kUpdBlock), 0, c.st, c.N, c.M, t, c.B,
                     r.kc, r.lc);
  return hip_st(hipGetLastError());
}

template <class T, bool CPLX> int fused_grid(int N) {
  thread_local int cus = 0, per = 0;  // CU count and occupancy of this kernel (first device used)
  if (cus == 0) {
    int dev = 0, c = 0, p = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&p, (const void *)kog_fused_kernel<T, CPLX>,
                                                     kUpdBlock, 0) != hipSuccess)
      return 0;
    per = p;
    cus = c;
  }
  int want = g_fused_per_cu < per ? g_fused_per_cu : per;
  int max_blocks = cus * want;
  const int n = N / 2;
  TileRule r = rule_for(N);
  int tiles = ((n + r.kc - 1) / r.kc) * ((n + r.lc - 1) / r.lc);
  return tiles < max_blocks ? tiles : max_blocks;
}

template <class T, bool CPLX> svd2_status fused_steps(const Ctx<T, CPLX> &c, int t0, int t1) {
  Bar *bar = (Bar *)(c.ws + c.L.bar);
  unsigned *flags = (unsigned *)(c.ws + c.L.flags);
  int grid = fused_grid<T, CPLX>(c.N);
  if (grid <= 0 || grid > kMaxFusedBlocks) return SVD2_ERR_HIP;
  hipLaunchKernelGGL(kog_bar_reset_kernel, dim3((grid + 255) / 256), dim3(256), 0, c.st, bar, flags, grid);
  svd2_status s = hip_st(hipGetLastError());
  if (s != SVD2_OK) return s;
  int N = c.N;
  Mat<T, CPLX> M = c.M;
  Bufs<T, CPLX> B = c.B;
  TileRule r = rule_for(N);
  int kc = r.kc, lc = r.lc;
  void *args[] = {&N, &M, &t0, &t1, &B, &bar, &flags, &kc, &lc};
  return hip_st(hipLaunchCooperativeKernel((const void *)kog_fused_kernel<T, CPLX>, dim3(grid),
                                           dim3(kUpdBlock), args, 0, c.st));
}

// Launch shape of the two-step kernel for order N.  With a fixed rule (lc > 0)
// each wavefront writes lc column pairs.  With lc <= 0 the column pairs are
// split so that the grid fills 1 - lc whole rounds of the workgroups the GPU
// holds at once (occupancy x CUs): all workgroups do the same work, so a
// partly filled last round would cost a whole round.
struct TwoStepShape {
  int wpg, span, lc, gx, ntiles;
  size_t lds;
};
template <class T, bool CPLX> TwoStepShape two_step_shape(int N) {
  // per host thread: concurrent solves on other threads do not share it
  thread_local int cached_N = 0, cached_wpg = 0, cached_lc = 0;
  thread_local TwoStepShape cached{};
  const TileRule r = rule2_for(N);
  if (N == cached_N && r.kc == cached_wpg && r.lc == cached_lc) return cached;
  TwoStepShape sh{};
  const int n = N / 2, wpg = r.kc;
  sh.wpg = wpg;
  sh.gx = (n + kShiftOut - 1) / kShiftOut;
  auto fix = [&](int span) {
    int lc = (span + wpg - 1) / wpg;
    lc = lc < 2 ? 2 : (lc > 64 ? 64 : lc);
    sh.lc = lc;
    sh.span = span < wpg * lc ? span : wpg * lc;
    if (sh.span < 2) sh.span = 2;
    sh.lds = two_step_lds<T, CPLX>(wpg, sh.span);
  };
  if (r.lc > 0) {
    fix(wpg * r.lc);
  } else {
    const int rounds = 1 - r.lc;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      return sh;
    fix(64 * wpg);  // the largest tile first, then refine with the occupancy it allows
    for (int it = 0; it < 3; ++it) {
      int per = 0;
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, (const void *)kog_two_step_kernel<T, CPLX>, 64 * wpg,
                                                       sh.lds) != hipSuccess || per < 1)
        return sh;
      const long cap = (long)per * cus * rounds;
      long tc = cap / sh.gx;
      if (tc < 1) tc = 1;
      fix((int)((n + tc - 1) / tc));
    }
  }
  sh.ntiles = sh.gx * ((n + sh.span - 1) / sh.span);
  cached_N = N;
  cached_wpg = r.kc;
  cached_lc = r.lc;
  cached = sh;
  return sh;
}

// two steps t, t+1 from `cur` into `nxt`
template <class T, bool CPLX>
svd2_status two_steps(const Ctx<T, CPLX> &c, const Mat<T, CPLX> &cur, const Mat<T, CPLX> &nxt, int t) {
  const int n = c.N / 2;
  hipLaunchKernelGGL((kog_pivots2_kernel<T, CPLX>), dim3((n + 63) / 64), dim3(64), 0, c.st, c.N, cur, t, c.B,
                     c.B1);
  svd2_status s = hip_st(hipGetLastError());
  if (s != SVD2_OK) return s;
  const TwoStepShape sh = two_step_shape<T, CPLX>(c.N);
  if (sh.ntiles <= 0) return SVD2_ERR_HIP;
  hipLaunchKernelGGL((kog_two_step_kernel<T, CPLX>), dim3(sh.ntiles), dim3(64 * sh.wpg), sh.lds, c.st, c.N, cur,
                     nxt, t, c.B, c.B1, sh.wpg, sh.span, sh.lc, sh.gx, sh.ntiles);
  return hip_st(hipGetLastError());
}

// one step t in place on `cur` (gather + SVD in one kernel, then the update)
template <class T, bool CPLX> svd2_status one_step_on(const Ctx<T, CPLX> &c, const Mat<T, CPLX> &cur, int t) {
  const int n = c.N / 2;
  hipLaunchKernelGGL((kog_pivot_kernel<T, CPLX>), dim3((n + 255) / 256), dim3(256), 0, c.st, c.N, cur, t, c.B);
  svd2_status s = hip_st(hipGetLastError());
  if (s != SVD2_OK) return s;
  TileRule r = rule_for(c.N);
  dim3 grid((n + r.kc - 1) / r.kc, (n + r.lc - 1) / r.lc);
  hipLaunchKernelGGL((kog_update_kernel<T, CPLX>), grid, dim3(kUpdBlock), 0, c.st, c.N, cur, t, c.B, r.kc, r.lc);
  return hip_st(hipGetLastError());
}

// a sweep of the two-step mode; *in_w tells (and is updated with) which
// buffer holds the iterate (false: the caller's A, true: the workspace copy)
template <class T, bool CPLX> svd2_status sweep_two_step(const Ctx<T, CPLX> &c, bool *in_w) {
  svd2_status s = SVD2_OK;
  int t = 0;
  for (; t + 1 < c.N - 1 && s == SVD2_OK; t += 2) {
    const Mat<T, CPLX> &cur = *in_w ? c.W : c.M, &nxt = *in_w ? c.M : c.W;
    s = two_steps<T, CPLX>(c, cur, nxt, t);
    *in_w = !*in_w;
  }
  if (s == SVD2_OK && t < c.N - 1) s = one_step_on<T, CPLX>(c, *in_w ? c.W : c.M, t);
  return s;
}

template <class T, bool CPLX> svd2_status copy_back(const Ctx<T, CPLX> &c) {
  int grid = c.N < 4096 ? c.N : 4096;
  hipLaunchKernelGGL((kog_copy_kernel<T, CPLX>), dim3(grid), dim3(256), 0, c.st, c.N, c.W, c.M);
  return hip_st(hipGetLastError());
}

template <class T, bool CPLX> svd2_status sweep(const Ctx<T, CPLX> &c) {
  if (c.flags & SVD2_KOG_TWO_STEP) {
    bool in_w = false;
    svd2_status s = sweep_two_step<T, CPLX>(c, &in_w);
    if (s == SVD2_OK && in_w) s = copy_back<T, CPLX>(c);
    return s;
  }
  if (!(c.flags & SVD2_KOG_UNFUSED)) return fused_steps<T, CPLX>(c, 0, c.N - 1);
  for (int t = 0; t < c.N - 1; ++t) {
    svd2_status s = unfused_step<T, CPLX>(c, t);
    if (s != SVD2_OK) return s;
  }
  return SVD2_OK;
}

template <class T, bool CPLX> svd2_status norms_async(const Ctx<T, CPLX> &c, bool in_w = false) {
  double *part = (double *)(c.ws + c.L.red), *res = (double *)(c.ws + c.L.res);
  int nb = c.N < kRedBlocks ? c.N : kRedBlocks;
  hipLaunchKernelGGL((kog_norm_partial_kernel<T, CPLX>), dim3(nb), dim3(256), 0, c.st, c.N, in_w ? c.W : c.M,
                     part);
  svd2_status s = hip_st(hipGetLastError());
  if (s != SVD2_OK) return s;
  hipLaunchKernelGGL(kog_norm_final_kernel, dim3(1), dim3(256), 0, c.st, nb, part, res);
  return hip_st(hipGetLastError());
}

template <class T, bool CPLX> svd2_status read_norms(const Ctx<T, CPLX> &c, double &off2, double &tot2) {
  double h[2];
  svd2_status s = hip_st(hipMemcpyAsync(h, c.ws + c.L.res, sizeof h, hipMemcpyDeviceToHost, c.st));
  if (s != SVD2_OK) return s;
  s = hip_st(hipStreamSynchronize(c.st));
  if (s != SVD2_OK) return s;
  off2 = h[0];
  tot2 = h[1];
  return SVD2_OK;
}

template <class T, bool CPLX> svd2_status check_abort(const Ctx<T, CPLX> &c) {
  if (c.flags & (SVD2_KOG_UNFUSED | SVD2_KOG_TWO_STEP)) return SVD2_OK;
  Bar h;
  svd2_status s = hip_st(hipMemcpyAsync(&h, c.ws + c.L.bar, sizeof h, hipMemcpyDeviceToHost, c.st));
  if (s != SVD2_OK) return s;
  s = hip_st(hipStreamSynchronize(c.st));
  if (s != SVD2_OK) return s;
  return h.abort ? SVD2_ERR_HIP : SVD2_OK;
}

// sweep replay from a hipGraph (unfused chain captured on a private stream)
template <class T, bool CPLX> svd2_status graph_build(Ctx<T, CPLX> c, hipGraphExec_t *exec) {
  hipStream_t cap;
  svd2_status s = hip_st(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
  if (s != SVD2_OK) return s;
  c.st = cap;
  hipGraph_t g = nullptr;
  s = hip_st(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
  if (s == SVD2_OK) {
    svd2_status s1 = SVD2_OK;
    for (int t = 0; t < c.N - 1 && s1 == SVD2_OK; ++t) s1 = unfused_step<T, CPLX>(c, t);
    svd2_status s2 = hip_st(hipStreamEndCapture(cap, &g));
    s = s1 != SVD2_OK ? s1 : s2;
  }
  if (s == SVD2_OK) s = hip_st(hipGraphInstantiate(exec, g, nullptr, nullptr, 0));
  if (g) hipGraphDestroy(g);
  hipStreamDestroy(cap);
  return s;
}

template <class T, bool CPLX>
svd2_status solve(Ctx<T, CPLX> &c, double tol, int max_sweeps, int *sweeps, double *off_rel) {
  if (max_sweeps < 0 || !(tol >= 0)) return SVD2_ERR_SIZE;
  hipGraphExec_t exec = nullptr;
  svd2_status s = SVD2_OK;
  if (c.flags & SVD2_KOG_GRAPH) s = graph_build<T, CPLX>(c, &exec);
  const bool two = c.flags & SVD2_KOG_TWO_STEP;
  bool in_w = false;
  double off2 = 0, tot2 = 0, nrm0 = 0;
  int sw = 0;
  if (s == SVD2_OK) s = norms_async<T, CPLX>(c);
  if (s == SVD2_OK) s = read_norms<T, CPLX>(c, off2, tot2);
  nrm0 = __builtin_sqrt(tot2);
  svd2_status result = SVD2_NOT_CONVERGED;
  while (s == SVD2_OK) {
    double rel = nrm0 > 0 ? __builtin_sqrt(off2) / nrm0 : 0.0;
    if (off_rel) *off_rel = rel;
    if (rel < tol || nrm0 == 0) {
      result = SVD2_OK;
      break;
    }
    if (sw == max_sweeps) break;
    if (exec) s = hip_st(hipGraphLaunch(exec, c.st));
    else if (two) s = sweep_two_step<T, CPLX>(c, &in_w);
    else s = sweep<T, CPLX>(c);
    if (s == SVD2_OK) s = norms_async<T, CPLX>(c, in_w);
    if (s == SVD2_OK) s = read_norms<T, CPLX>(c, off2, tot2);
    if (s == SVD2_OK) s = check_abort<T, CPLX>(c);
    ++sw;
  }
  if (s == SVD2_OK && in_w) {
    s = copy_back<T, CPLX>(c);
    if (s == SVD2_OK) s = hip_st(hipStreamSynchronize(c.st));
  }
  if (exec) hipGraphExecDestroy(exec);
  if (sweeps) *sweeps = sw;
  return s != SVD2_OK ? s : result;
}

template <class T, bool CPLX>
svd2_status api_step(int N, T *A, int lda, int t, void *ws, size_t wsb, unsigned flags, hipStream_t st) {
  Ctx<T, CPLX> c;
  if (flags & (SVD2_KOG_GRAPH | SVD2_KOG_TWO_STEP)) return SVD2_ERR_FLAGS;  // solve/sweep modes
  svd2_status s = validate<T, CPLX>(N, A, lda, ws, wsb, flags, c);
  if (s != SVD2_OK) return s;
  if (t < 0 || t >= N - 1) return SVD2_ERR_SIZE;
  c.st = st;
  return (c.flags & SVD2_KOG_UNFUSED) ? unfused_step<T, CPLX>(c, t) : fused_steps<T, CPLX>(c, t, t + 1);
}

template <class T, bool CPLX>
svd2_status api_sweep(int N, T *A, int lda, void *ws, size_t wsb, unsigned flags, hipStream_t st) {
  Ctx<T, CPLX> c;
  if (flags & SVD2_KOG_GRAPH) return SVD2_ERR_FLAGS;  // graph replay is a solve-only mode
  svd2_status s = validate<T, CPLX>(N, A, lda, ws, wsb, flags, c);
  if (s != SVD2_OK) return s;
  c.st = st;
  return sweep<T, CPLX>(c);
}

template <class T, bool CPLX>
svd2_status api_solve(int N, T *A, int lda, double tol, int max_sweeps, int *sweeps, double *off_rel,
                      void *ws, size_t wsb, unsigned flags, hipStream_t st) {
  Ctx<T, CPLX> c;
  svd2_status s = validate<T, CPLX>(N, A, lda, ws, wsb, flags, c);
  if (s != SVD2_OK) return s;
  c.st = st;
  return solve<T, CPLX>(c, tol, max_sweeps, sweeps, off_rel);
}

template <class T, bool CPLX>
svd2_status api_norms(int N, const T *A, int lda, double *off2, double *tot2, void *ws, size_t wsb,
                      hipStream_t st) {
  Ctx<T, CPLX> c;
  svd2_status s = validate<T, CPLX>(N, const_cast<T *>(A), lda, ws, wsb, 0, c);
  if (s != SVD2_OK) return s;
  if (!off2 || !tot2) return SVD2_ERR_NULL;
  c.st = st;
  s = norms_async<T, CPLX>(c);
  if (s == SVD2_OK) s = read_norms<T, CPLX>(c, *off2, *tot2);
  return s;
}


// ---------------------------------------------------------------------------
// batch host driver
// ---------------------------------------------------------------------------
struct BatchLayout {
  size_t hdr, probs, itemsA, itemsB, itemsC, parts, bufs, total;
  size_t lds[4];  // two-step LDS bytes per element type
  int maxA, maxB, maxC, nparts;
  int maxC_kind[4];
};

int esz_of(int kind) { return (kind == SVD2_KOG_F64 || kind == SVD2_KOG_C128) ? 8 : 4; }
bool cplx_of(int kind) { return kind == SVD2_KOG_C128 || kind == SVD2_KOG_C64; }

// column pairs per wavefront of the two-step tiles in a batch (workgroups of
// kUpdBlock / 64 wavefronts).  Fixed rather than taken from the single-problem
// shape table: a lone small problem wants many small tiles for parallelism,
// while a batch has parallelism from its many problems and loses to the halo
// reads of small tiles (256-problem batch: 8.6 s with 8, 9.5 s with the
// single-problem shapes).
int batch_lc2(int) { return 8; }

size_t two_step_lds_of(int kind, int span) {
  const int wpg = kUpdBlock / 64;
  switch (kind) {
    case SVD2_KOG_F64: return two_step_lds<double, false>(wpg, span);
    case SVD2_KOG_C128: return two_step_lds<double, true>(wpg, span);
    case SVD2_KOG_F32: return two_step_lds<float, false>(wpg, span);
    default: return two_step_lds<float, true>(wpg, span);
  }
}

svd2_status batch_layout(int nprob, const kog_problem *pr, BatchLayout &L, std::vector<DevProb> *dp,
                         bool two) {
  auto up = [](size_t x) { return (x + 255) & ~size_t(255); };
  if (nprob < 0 || nprob > (1 << 20)) return SVD2_ERR_SIZE;
  if (nprob > 0 && !pr) return SVD2_ERR_NULL;
  L.maxA = L.maxB = L.maxC = L.nparts = 0;
  for (int k = 0; k < 4; ++k) {
    L.lds[k] = 0;
    L.maxC_kind[k] = 0;
  }
  size_t bufs = 0;
  for (int p = 0; p < nprob; ++p) {
    const kog_problem &q = pr[p];
    if (q.dtype < SVD2_KOG_F64 || q.dtype > SVD2_KOG_C64) return SVD2_ERR_FLAGS;
    if (q.N < 2 || q.N % 2 || q.lda < q.N || q.N > (1 << 19)) return SVD2_ERR_SIZE;
    if (q.max_sweeps < 0 || !(q.tol >= 0)) return SVD2_ERR_SIZE;
    int n = q.N / 2;
    TileRule r = rule_for(q.N);
    int kt = (n + r.kc - 1) / r.kc, lt = (n + r.lc - 1) / r.lc;
    int nin = cplx_of(q.dtype) ? 8 : 4, nout = cplx_of(q.dtype) ? 19 : 11;
    size_t arr = arr_bytes(q.N, esz_of(q.dtype));
    const int lc2 = batch_lc2(q.N), span = (kUpdBlock / 64) * lc2;
    const int gx2 = (n + kShiftOut - 1) / kShiftOut, ny2 = (n + span - 1) / span;
    const size_t set = (nin + nout) * arr;
    const size_t wbytes = up((size_t)q.N * q.N * esz_of(q.dtype) * (cplx_of(q.dtype) ? 2 : 1));
    if (dp) {
      DevProb d = {};
      d.A = q.A;
      d.lda = q.lda;
      d.N = q.N;
      d.kind = q.dtype;
      d.kc = r.kc;
      d.lc = r.lc;
      d.part_off = L.nparts;
      d.ntiles = kt * lt;
      d.max_sweeps = q.max_sweeps;
      d.tol = q.tol;
      d.piv_off = (long long)bufs;  // relative to the buffer region; rebased below
      d.out_off = (long long)(bufs + nin * arr);
      if (two) {
        d.piv1_off = (long long)(bufs + set);
        d.out1_off = (long long)(bufs + set + nin * arr);
        d.w_off = (long long)(bufs + 2 * set);
        d.gx2 = gx2;
        d.ny2 = ny2;
        d.lc2 = lc2;
      }
      dp->push_back(d);
    }
    bufs += two ? 2 * set + wbytes : set;
    L.maxA += (n + kUpdBlock - 1) / kUpdBlock;
    L.maxB += kt * lt;
    L.maxC += two ? gx2 * ny2 : 0;
    L.maxC_kind[q.dtype] += two ? gx2 * ny2 : 0;
    L.nparts += kt * lt;
    if (two) {
      size_t l = two_step_lds_of(q.dtype, span);
      if (l > L.lds[q.dtype]) L.lds[q.dtype] = l;
    }
  }
  L.hdr = 0;
  L.probs = 256;
  L.itemsA = L.probs + up((size_t)nprob * sizeof(DevProb));
  L.itemsB = L.itemsA + up((size_t)L.maxA * sizeof(int2));
  L.itemsC = L.itemsB + up((size_t)L.maxB * sizeof(int4));
  L.parts = L.itemsC + up((size_t)L.maxC * sizeof(int4));
  L.bufs = L.parts + up((size_t)L.nparts * sizeof(double));
  L.total = L.bufs + bufs;
  if (dp)
    for (DevProb &d : *dp) {
      d.piv_off += (long long)L.bufs;
      d.out_off += (long long)L.bufs;
      if (two) {
        d.piv1_off += (long long)L.bufs;
        d.out1_off += (long long)L.bufs;
        d.w_off += (long long)L.bufs;
      }
    }
  return SVD2_OK;
}

// work lists of the problems still running
void build_items(const std::vector<DevProb> &dp, std::vector<int2> &A, std::vector<int4> &B,
                 std::vector<int4> &C, int *c0, bool two) {
  A.clear();
  B.clear();
  C.clear();
  for (int kind = 0; kind < 4; ++kind) {  // two-step tiles, grouped by element type
    c0[kind] = (int)C.size();
    if (!two) continue;
    for (int p = 0; p < (int)dp.size(); ++p) {
      const DevProb &d = dp[p];
      if (d.status != 0 || d.kind != kind) continue;
      for (int y = 0; y < d.ny2; ++y)
        for (int x = 0; x < d.gx2; ++x) C.push_back(int4{p, x, y, 0});
    }
  }
  c0[4] = (int)C.size();
  for (int p = 0; p < (int)dp.size(); ++p) {
    const DevProb &d = dp[p];
    if (d.status != 0) continue;
    int n = d.N / 2;
    for (int c = 0; c * kUpdBlock < n; ++c) A.push_back(int2{p, c});
    int kt = (n + d.kc - 1) / d.kc, lt = (n + d.lc - 1) / d.lc;
    for (int j = 0; j < lt; ++j)
      for (int i = 0; i < kt; ++i) B.push_back(int4{p, i * d.kc, j * d.lc, j * kt + i});
  }
}

struct BatchRun {
  char *ws;
  BatchLayout L;
  hipStream_t st;
  int gA, gB, gF, two;
};

template <class T, bool CPLX, int KIND> svd2_status batch_two_step_launch(const BatchRun &r, hipStream_t st) {
  if (r.L.maxC_kind[KIND] == 0) return SVD2_OK;
  BatchHdr *hdr = (BatchHdr *)(r.ws + r.L.hdr);
  DevProb *probs = (DevProb *)(r.ws + r.L.probs);
  hipLaunchKernelGGL((kog_batch_pivots2_kernel<T, CPLX, KIND>), dim3(r.gA), dim3(kUpdBlock), 0, st, r.ws, hdr,
                     (const int2 *)(r.ws + r.L.itemsA), probs);
  svd2_status s = hip_st(hipGetLastError());
  if (s != SVD2_OK) return s;
  const int g = r.L.maxC_kind[KIND] < 16384 ? r.L.maxC_kind[KIND] : 16384;
  hipLaunchKernelGGL((kog_batch_two_step_kernel<T, CPLX, KIND>), dim3(g), dim3(kUpdBlock), r.L.lds[KIND], st,
                     r.ws, hdr, (const int4 *)(r.ws + r.L.itemsC), probs);
  return hip_st(hipGetLastError());
}

svd2_status batch_step(const BatchRun &r, hipStream_t st) {
  BatchHdr *hdr = (BatchHdr *)(r.ws + r.L.hdr);
  DevProb *probs = (DevProb *)(r.ws + r.L.probs);
  hipLaunchKernelGGL(kog_batch_pivot_kernel, dim3(r.gA), dim3(kUpdBlock), 0, st, r.ws, hdr,
                     (const int2 *)(r.ws + r.L.itemsA), probs, r.two);
  svd2_status s = hip_st(hipGetLastError());
  if (s != SVD2_OK) return s;
  hipLaunchKernelGGL(kog_batch_update_kernel, dim3(r.gB), dim3(kUpdBlock), 0, st, r.ws, hdr,
                     (const int4 *)(r.ws + r.L.itemsB), probs, (double *)(r.ws + r.L.parts), r.two);
  s = hip_st(hipGetLastError());
  if (s == SVD2_OK && r.two) s = batch_two_step_launch<double, false, SVD2_KOG_F64>(r, st);
  if (s == SVD2_OK && r.two) s = batch_two_step_launch<double, true, SVD2_KOG_C128>(r, st);
  if (s == SVD2_OK && r.two) s = batch_two_step_launch<float, false, SVD2_KOG_F32>(r, st);
  if (s == SVD2_OK && r.two) s = batch_two_step_launch<float, true, SVD2_KOG_C64>(r, st);
  if (s != SVD2_OK) return s;
  hipLaunchKernelGGL(kog_batch_finish_kernel, dim3(r.gF), dim3(kUpdBlock), 0, st, hdr, probs,
                     (const double *)(r.ws + r.L.parts), r.two);
  return hip_st(hipGetLastError());
}

svd2_status upload_items(const BatchRun &r, const std::vector<DevProb> &dp, int active) {
  std::vector<int2> A;
  std::vector<int4> B, C;
  BatchHdr h = {};
  build_items(dp, A, B, C, h.c0, r.two != 0);
  h.nA = (int)A.size();
  h.nB = (int)B.size();
  h.nprob = (int)dp.size();
  h.active = active;
  svd2_status s = hip_st(hipMemcpyAsync(r.ws + r.L.hdr, &h, sizeof h, hipMemcpyHostToDevice, r.st));
  if (s == SVD2_OK && !A.empty())
    s = hip_st(hipMemcpyAsync(r.ws + r.L.itemsA, A.data(), A.size() * sizeof(int2), hipMemcpyHostToDevice, r.st));
  if (s == SVD2_OK && !B.empty())
    s = hip_st(hipMemcpyAsync(r.ws + r.L.itemsB, B.data(), B.size() * sizeof(int4), hipMemcpyHostToDevice, r.st));
  if (s == SVD2_OK && !C.empty())
    s = hip_st(hipMemcpyAsync(r.ws + r.L.itemsC, C.data(), C.size() * sizeof(int4), hipMemcpyHostToDevice, r.st));
  if (s == SVD2_OK) s = hip_st(hipStreamSynchronize(r.st));
  return s;
}

svd2_status batch_solve(int nprob, kog_problem *pr, void *ws, size_t wsb, unsigned flags, hipStream_t st) {
  if (flags & ~(unsigned)(SVD2_KOG_GRAPH | SVD2_KOG_TWO_STEP)) return SVD2_ERR_FLAGS;
  BatchRun r;
  r.two = (flags & SVD2_KOG_TWO_STEP) ? 1 : 0;
  std::vector<DevProb> dp;
  svd2_status s = batch_layout(nprob, pr, r.L, &dp, r.two != 0);
  if (s != SVD2_OK) return s;
  if (nprob == 0) return SVD2_OK;
  if (!ws) return SVD2_ERR_NULL;
  if ((uintptr_t)ws % 256) return SVD2_ERR_ALIGN;
  if (wsb < r.L.total) return SVD2_ERR_SIZE;
  for (int p = 0; p < nprob; ++p) {
    const kog_problem &q = pr[p];
    if (!q.A) return SVD2_ERR_NULL;
    int e = esz_of(q.dtype) * (cplx_of(q.dtype) ? 2 : 1);
    if ((uintptr_t)q.A % e) return SVD2_ERR_ALIGN;
    uintptr_t a0 = (uintptr_t)q.A, a1 = a0 + ((size_t)q.lda * (q.N - 1) + q.N) * e;
    uintptr_t w0 = (uintptr_t)ws, w1 = w0 + r.L.total;
    if (a0 < w1 && w0 < a1) return SVD2_ERR_ALIAS;
  }
  r.ws = (char *)ws;
  r.st = st;
  r.gA = r.L.maxA < 8192 ? r.L.maxA : 8192;
  r.gB = r.L.maxB < 16384 ? r.L.maxB : 16384;
  r.gF = nprob < 1024 ? nprob : 1024;
  // problem table and the full work lists
  s = hip_st(hipMemcpyAsync(r.ws + r.L.probs, dp.data(), dp.size() * sizeof(DevProb), hipMemcpyHostToDevice, st));
  if (s == SVD2_OK) s = upload_items(r, dp, nprob);
  if (s != SVD2_OK) return s;
  hipLaunchKernelGGL(kog_batch_init_kernel, dim3(r.gF), dim3(kUpdBlock), 0, st, (BatchHdr *)(r.ws + r.L.hdr),
                     (DevProb *)(r.ws + r.L.probs));
  s = hip_st(hipGetLastError());
  long long max_steps = 0;  // passes: steps, or (N/2 per sweep) two-step passes
  for (const DevProb &d : dp) {
    long long m = (long long)d.max_sweeps * (r.two ? d.N / 2 : d.N - 1);
    if (m > max_steps) max_steps = m;
  }
  const int K = 64;  // passes per replay / between host checks
  hipGraphExec_t exec = nullptr;
  hipStream_t cap = nullptr;
  auto capture = [&]() -> svd2_status {
    if (exec) {
      hipGraphExecDestroy(exec);
      exec = nullptr;
    }
    hipGraph_t g = nullptr;
    svd2_status c = hip_st(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
    if (c != SVD2_OK) return c;
    svd2_status c1 = SVD2_OK;
    for (int i = 0; i < K && c1 == SVD2_OK; ++i) c1 = batch_step(r, cap);
    svd2_status c2 = hip_st(hipStreamEndCapture(cap, &g));
    c = c1 != SVD2_OK ? c1 : c2;
    if (c == SVD2_OK) c = hip_st(hipGraphInstantiate(&exec, g, nullptr, nullptr, 0));
    if (g) hipGraphDestroy(g);
    return c;
  };
  if (s == SVD2_OK && (flags & SVD2_KOG_GRAPH)) {
    s = hip_st(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    if (s == SVD2_OK) s = capture();
  }
  int active = nprob, built_for = nprob;
  long long steps = 0;
  while (s == SVD2_OK) {
    BatchHdr h;
    s = hip_st(hipMemcpyAsync(&h, r.ws + r.L.hdr, sizeof h, hipMemcpyDeviceToHost, st));
    if (s == SVD2_OK) s = hip_st(hipStreamSynchronize(st));
    if (s != SVD2_OK) break;
    active = h.active;
    if (active <= 0 || steps > max_steps) break;
    if (active * 10 < built_for * 7) {  // compact the work lists to the running problems
      s = hip_st(hipMemcpyAsync(dp.data(), r.ws + r.L.probs, dp.size() * sizeof(DevProb), hipMemcpyDeviceToHost, st));
      if (s == SVD2_OK) s = hip_st(hipStreamSynchronize(st));
      if (s == SVD2_OK) s = upload_items(r, dp, active);
      if (s != SVD2_OK) break;
      built_for = active;
    }
    if (exec) {
      s = hip_st(hipGraphLaunch(exec, st));
    } else {
      for (int i = 0; i < K && s == SVD2_OK; ++i) s = batch_step(r, st);
    }
    steps += K;
  }
  if (exec) hipGraphExecDestroy(exec);
  if (cap) hipStreamDestroy(cap);
  if (s != SVD2_OK) return s;
  s = hip_st(hipMemcpyAsync(dp.data(), r.ws + r.L.probs, dp.size() * sizeof(DevProb), hipMemcpyDeviceToHost, st));
  if (s == SVD2_OK) s = hip_st(hipStreamSynchronize(st));
  if (s != SVD2_OK) return s;
  // iterates left in the second matrix go back to the caller's
  for (int p = 0; p < nprob && s == SVD2_OK; ++p) {
    const DevProb &d = dp[p];
    if (!d.in_w) continue;
    const int grid = d.N < 4096 ? d.N : 4096;
    char *w = r.ws + d.w_off;
    switch (d.kind) {
      case SVD2_KOG_F64:
        hipLaunchKernelGGL((kog_copy_kernel<double, false>), dim3(grid), dim3(256), 0, st, d.N,
                           Mat<double, false>{(double *)w, (size_t)d.N}, Mat<double, false>{(double *)d.A, (size_t)d.lda});
        break;
      case SVD2_KOG_C128:
        hipLaunchKernelGGL((kog_copy_kernel<double, true>), dim3(grid), dim3(256), 0, st, d.N,
                           Mat<double, true>{(double *)w, (size_t)d.N}, Mat<double, true>{(double *)d.A, (size_t)d.lda});
        break;
      case SVD2_KOG_F32:
        hipLaunchKernelGGL((kog_copy_kernel<float, false>), dim3(grid), dim3(256), 0, st, d.N,
                           Mat<float, false>{(float *)w, (size_t)d.N}, Mat<float, false>{(float *)d.A, (size_t)d.lda});
        break;
      default:
        hipLaunchKernelGGL((kog_copy_kernel<float, true>), dim3(grid), dim3(256), 0, st, d.N,
                           Mat<float, true>{(float *)w, (size_t)d.N}, Mat<float, true>{(float *)d.A, (size_t)d.lda});
        break;
    }
    s = hip_st(hipGetLastError());
  }
  if (s == SVD2_OK) s = hip_st(hipStreamSynchronize(st));
  if (s != SVD2_OK) return s;
  svd2_status all = SVD2_OK;
  for (int p = 0; p < nprob; ++p) {
    pr[p].sweeps = dp[p].sweeps;
    pr[p].off_rel = dp[p].off_rel;
    pr[p].status = dp[p].status == 1 ? SVD2_OK : SVD2_NOT_CONVERGED;
    if (dp[p].status != 1) all = SVD2_NOT_CONVERGED;
  }
  return all;
}

}  // namespace

// the last HIP error of a Kogbetliantz entry point defined in another file
void kog_note_hip_error(int e) { g_kog_hip = e; }

extern "C" {

size_t kog_workspace_bytes_flags(int N, int dtype, unsigned flags) {
  if (N < 2 || N % 2) return 0;
  Layout L;
  switch (dtype) {
    case SVD2_KOG_F64: L = layout(N, 8, false); break;
    case SVD2_KOG_C128: L = layout(N, 8, true); break;
    case SVD2_KOG_F32: L = layout(N, 4, false); break;
    case SVD2_KOG_C64: L = layout(N, 4, true); break;
    default: return 0;
  }
  return (flags & SVD2_KOG_TWO_STEP) ? L.total2 : L.total;
}

size_t kog_workspace_bytes(int N, int dtype) { return kog_workspace_bytes_flags(N, dtype, 0); }

svd2_status dkog_step(int N, double *A, int lda, int t, void *ws, size_t ws_bytes, unsigned flags,
                      hipStream_t stream) {
  return api_step<double, false>(N, A, lda, t, ws, ws_bytes, flags, stream);
}
svd2_status zkog_step(int N, double *A, int lda, int t, void *ws, size_t ws_bytes, unsigned flags,
                      hipStream_t stream) {
  return api_step<double, true>(N, A, lda, t, ws, ws_bytes, flags, stream);
}
svd2_status skog_step(int N, float *A, int lda, int t, void *ws, size_t ws_bytes, unsigned flags,
                      hipStream_t stream) {
  return api_step<float, false>(N, A, lda, t, ws, ws_bytes, flags, stream);
}
svd2_status ckog_step(int N, float *A, int lda, int t, void *ws, size_t ws_bytes, unsigned flags,
                      hipStream_t stream) {
  return api_step<float, true>(N, A, lda, t, ws, ws_bytes, flags, stream);
}

svd2_status dkog_sweep(int N, double *A, int lda, void *ws, size_t ws_bytes, unsigned flags,
                       hipStream_t stream) {
  return api_sweep<double, false>(N, A, lda, ws, ws_bytes, flags, stream);
}
svd2_status zkog_sweep(int N, double *A, int lda, void *ws, size_t ws_bytes, unsigned flags,
                       hipStream_t stream) {
  return api_sweep<double, true>(N, A, lda, ws, ws_bytes, flags, stream);
}
svd2_status skog_sweep(int N, float *A, int lda, void *ws, size_t ws_bytes, unsigned flags,
                       hipStream_t stream) {
  return api_sweep<float, false>(N, A, lda, ws, ws_bytes, flags, stream);
}
svd2_status ckog_sweep(int N, float *A, int lda, void *ws, size_t ws_bytes, unsigned flags,
                       hipStream_t stream) {
  return api_sweep<float, true>(N, A, lda, ws, ws_bytes, flags, stream);
}

svd2_status dkog_solve(int N, double *A, int lda, double tol, int max_sweeps, int *sweeps,
                       double *off_rel, void *ws, size_t ws_bytes, unsigned flags, hipStream_t stream) {
  return api_solve<double, false>(N, A, lda, tol, max_sweeps, sweeps, off_rel, ws, ws_bytes, flags, stream);
}
svd2_status zkog_solve(int N, double *A, int lda, double tol, int max_sweeps, int *sweeps,
                       double *off_rel, void *ws, size_t ws_bytes, unsigned flags, hipStream_t stream) {
  return api_solve<double, true>(N, A, lda, tol, max_sweeps, sweeps, off_rel, ws, ws_bytes, flags, stream);
}
svd2_status skog_solve(int N, float *A, int lda, double tol, int max_sweeps, int *sweeps,
                       double *off_rel, void *ws, size_t ws_bytes, unsigned flags, hipStream_t stream) {
  return api_solve<float, false>(N, A, lda, tol, max_sweeps, sweeps, off_rel, ws, ws_bytes, flags, stream);
}
svd2_status ckog_solve(int N, float *A, int lda, double tol, int max_sweeps, int *sweeps,
                       double *off_rel, void *ws, size_t ws_bytes, unsigned flags, hipStream_t stream) {
  return api_solve<float, true>(N, A, lda, tol, max_sweeps, sweeps, off_rel, ws, ws_bytes, flags, stream);
}

svd2_status dkog_norms(int N, const double *A, int lda, double *off2, double *tot2, void *ws,
                       size_t ws_bytes, hipStream_t stream) {
  return api_norms<double, false>(N, A, lda, off2, tot2, ws, ws_bytes, stream);
}
svd2_status zkog_norms(int N, const double *A, int lda, double *off2, double *tot2, void *ws,
                       size_t ws_bytes, hipStream_t stream) {
  return api_norms<double, true>(N, A, lda, off2, tot2, ws, ws_bytes, stream);
}
svd2_status skog_norms(int N, const float *A, int lda, double *off2, double *tot2, void *ws,
                       size_t ws_bytes, hipStream_t stream) {
  return api_norms<float, false>(N, A, lda, off2, tot2, ws, ws_bytes, stream);
}
svd2_status ckog_norms(int N, const float *A, int lda, double *off2, double *tot2, void *ws,
                       size_t ws_bytes, hipStream_t stream) {
  return api_norms<float, true>(N, A, lda, off2, tot2, ws, ws_bytes, stream);
}

int kog_last_hip_error(void) { return g_kog_hip; }

size_t kog_batch_workspace_bytes_flags(int nprob, const kog_problem *probs, unsigned flags) {
  BatchLayout L;
  if (batch_layout(nprob, probs, L, nullptr, (flags & SVD2_KOG_TWO_STEP) != 0) != SVD2_OK) return 0;
  return L.total;
}

size_t kog_batch_workspace_bytes(int nprob, const kog_problem *probs) {
  return kog_batch_workspace_bytes_flags(nprob, probs, 0);
}

svd2_status kog_batch_solve(int nprob, kog_problem *probs, void *ws, size_t ws_bytes, unsigned flags,
                            hipStream_t stream) {
  return batch_solve(nprob, probs, ws, ws_bytes, flags, stream);
}

svd2_status kog_set_tile_rules(int count, const int *max_order, const int *kc, const int *lc) {
  if (count < 0 || count > kMaxRules) return SVD2_ERR_SIZE;
  if (count > 0 && (!max_order || !kc || !lc)) return SVD2_ERR_NULL;
  for (int i = 0; i < count; ++i) {
    if (kc[i] != 64 && kc[i] != 128 && kc[i] != 256) return SVD2_ERR_SIZE;
    if (lc[i] < 1 || lc[i] > 4096 || max_order[i] < 2) return SVD2_ERR_SIZE;
    if (i > 0 && max_order[i] <= max_order[i - 1]) return SVD2_ERR_SIZE;
  }
  for (int i = 0; i < count; ++i) g_rules[i] = TileRule{max_order[i], kc[i], lc[i]};
  g_nrules = count;
  if (count == 0) {
    g_rules[0] = default_rule();
    g_nrules = 1;
  }
  return SVD2_OK;
}

svd2_status kog_set_two_step_tiles(int count, const int *max_order, const int *wpg, const int *lc) {
  if (count < 0 || count > kMaxRules) return SVD2_ERR_SIZE;
  if (count > 0 && (!max_order || !wpg || !lc)) return SVD2_ERR_NULL;
  for (int i = 0; i < count; ++i) {
    if (wpg[i] != 1 && wpg[i] != 2 && wpg[i] != 4) return SVD2_ERR_SIZE;
    if (lc[i] < -3 || lc[i] == 1 || lc[i] > 64 || max_order[i] < 2) return SVD2_ERR_SIZE;
    if (i > 0 && max_order[i] <= max_order[i - 1]) return SVD2_ERR_SIZE;
  }
  for (int i = 0; i < count; ++i) g_rules2[i] = TileRule{max_order[i], wpg[i], lc[i]};
  g_nrules2 = count;
  if (count == 0) {
    g_rules2[0] = default_rule2();
    g_nrules2 = 1;
  }
  return SVD2_OK;
}

svd2_status kog_set_fused_blocks_per_cu(int per_cu) {
  if (per_cu < 1 || per_cu > 16) return SVD2_ERR_SIZE;
  g_fused_per_cu = per_cu;
  return SVD2_OK;
}

}  // extern "C"
