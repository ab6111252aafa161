/*
 * svd2_oracle.cpp -- plain per-matrix CPU oracle of the batched 2x2 SVD.
 *
 * TEST INFRASTRUCTURE ONLY (see svd2_oracle.h).  Built with
 * -O2 -ffp-contract=off -fno-fast-math so that every +, -, *, /, sqrt and fma
 * below is one correctly rounded IEEE-754 operation, in the written order.
 *
 * The algorithm is the one of section 2 of arXiv:2005.07403, with the
 * operation order of its vectorised description (sections 5-7, Figs. 3-10,
 * and the expansion of eq. (29) in section 2.3).  Each matrix is processed on
 * its own; there is no blocking, fusion or reordering.
 */
#include "svd2_oracle.h"

#include <cfloat>
#include <algorithm>
#include <vector>
#include <cmath>
#include <cstring>
#include <omp.h>
#include <quadmath.h>
#include <type_traits>
#include <utility>

namespace {

/* ---------------------------------------------------------------------------
 * Constants per element type.
 *   h   : two less than the largest finite binary exponent (section 2.1)
 *   big : the finite upper bound on s in eq. (2)
 *   tm  : the smallest positive subnormal (eq. (1))
 *   f   : sqrt(MAX) rounded to T, the clamp of tan 2phi in eq. (14)
 * ------------------------------------------------------------------------- */
template <class T> struct Lim;
template <> struct Lim<double> {
  static constexpr int h = DBL_MAX_EXP - 3; /* 1021 */
  static constexpr int pk = 128;            /* phase of a subnormal |z|: 2^pk z is normal */
  static double big() { return DBL_MAX; }
  static double mn() { return DBL_MIN; }
  static double tm() { return DBL_TRUE_MIN; }
  static double f() { return 0x1.fffffffffffffp+511; }
};
template <> struct Lim<float> {
  static constexpr int h = FLT_MAX_EXP - 3; /* 125 */
  static constexpr int pk = 64;
  static float big() { return FLT_MAX; }
  static float mn() { return FLT_MIN; }
  static float tm() { return FLT_TRUE_MIN; }
  static float f() { return 0x1.fffffep+63f; }
};

/* "Relaxed" min/max of section 2: the minimum (maximum) of two non-NaN
 * arguments, or the second argument when the first is a NaN. */
template <class T> inline T rmin(T a, T b) { return (a < b) ? a : b; }
template <class T> inline T rmax(T a, T b) { return (a > b) ? a : b; }

template <class T> inline T fmaT(T a, T b, T c) { return std::fma(a, b, c); }
template <class T> inline T sqrtT(T a) { return std::sqrt(a); }

/* hypot, two readings (the paper only demands hypot(a,b)=0 <=> a=b=0).
 * MIRROR: the per-lane fallback of section 5 (Fig. 4 discussion):
 *   a' = max|.|, b' = min|.|, q = b'/max(a', TRUE_MIN), c = a' sqrt(fma(q,q,1)).
 * REF: sqrt(a^2+b^2) evaluated in binary128 and rounded once to T. */
template <class T> T hypot_mirror(T a, T b) {
  T aa = std::fabs(a), bb = std::fabs(b);
  T hi = rmax(aa, bb), lo = rmin(aa, bb);
  T q = lo / rmax(hi, Lim<T>::tm());
  return hi * sqrtT(fmaT(q, q, T(1)));
}
template <class T> T hypot_ref(T a, T b) {
  __float128 qa = a, qb = b;
  return (T)sqrtq(qa * qa + qb * qb);
}
/* invsqrt(x) = 1/sqrt(x) (section 2, eq. (7)); MIRROR takes the first remedy
 * of section 6 (divide one by the secant), REF rounds 1/sqrt once. */
template <class T> T invsqrt_mirror(T x) { return T(1) / sqrtT(x); }
template <class T> T invsqrt_ref(T x) { return (T)(1 / sqrtq((__float128)x)); }

template <class T> struct Prim {
  int policy;
  bool sine = false; /* assemble U by eq. (31) instead of eq. (29) */
  T hyp(T a, T b) const { return policy == ORACLE_REF ? hypot_ref(a, b) : hypot_mirror(a, b); }
  T isq(T x) const { return policy == ORACLE_REF ? invsqrt_ref(x) : invsqrt_mirror(x); }
};

/* exp2 of section 2.1: floor(lg|a|) for finite non-zero a (the true exponent,
 * also for subnormals), -inf for zero.  Returned as E = h - exp2(a), so a zero
 * component gives +inf. */
template <class T> T scale_exponent(T a) {
  if (a == T(0)) return (T)INFINITY;
  return (T)(Lim<T>::h - std::ilogb(a));
}
/* SCALEF(a, s) = a 2^s, correctly rounded.  s is an integer-valued T, or BIG
 * (then every component is zero and the zero is returned unchanged). */
template <class T> T scalef(T a, T s) {
  if (s == Lim<T>::big()) return a;
  return std::ldexp(a, (int)s);
}

template <class T> struct Cx { T re, im; };

/* eq. (5): c = a * b with one fma per component. */
template <class T> Cx<T> cmul(Cx<T> a, Cx<T> b) {
  return {fmaT(a.re, b.re, -(a.im * b.im)), fmaT(a.re, b.im, a.im * b.re)};
}
/* conj(a) * b, eq. (5) with the conjugation folded into the signs (Fig. 7):
 * re = fma(Re a, Re b, Im a Im b), im = fma(Re a, Im b, -(Im a Re b)). */
template <class T> Cx<T> cmulc(Cx<T> a, Cx<T> b) {
  return {fmaT(a.re, b.re, a.im * b.im), fmaT(a.re, b.im, -(a.im * b.re))};
}


/* eq. (1): e^{i arg z} from z and |z| = P.hyp(Re z, Im z), without complex
 * operations: cos = copysign(min(|Re z|/|z|, 1), Re z), sin = Im z /
 * max(|z|, TRUE_MIN).  Reading: below the normal range the rounding error of
 * |z| is no longer relative (z = (-4, 1) 2^-1074 gives |z| = 4 2^-1074 and the
 * "phase" (-1, 1/4), whose modulus is not one, so U would not be unitary);
 * there eq. (1) is applied to 2^k z instead, an exact scaling that leaves the
 * phase unchanged.  Whenever |z| is normal the result is the literal one. */
template <class T> Cx<T> phase(const Prim<T> &P, Cx<T> z, T absz) {
  if (absz < Lim<T>::mn()) {
    z = {std::ldexp(z.re, Lim<T>::pk), std::ldexp(z.im, Lim<T>::pk)};
    absz = P.hyp(z.re, z.im);
  }
  return {std::copysign(rmin(std::fabs(z.re) / absz, T(1)), z.re),
          z.im / rmax(absz, Lim<T>::tm())};
}

/* Output of one matrix, in the element order of the header. */
template <class T> struct Res {
  Cx<T> u[2][2], v[2][2];
  T smax, smin, s;
};

/* Intermediates kept for the trace entry point and for the FP64 rescue. */
template <class T> struct Mid {
  T s; bool c, r;
  Cx<T> ah[2][2];     /* scaled input A^ = 2^s A, original positions */
  Cx<T> d1, d2;       /* diagonal of D (conjugates of D*), eq. (4)   */
  bool neg1, neg2;    /* real case: sign bits of a''_11, a''_21      */
  T r11, r12, r22, mt, ca;
  Cx<T> e12;          /* e^{i arg r'_12}; D~_22 = conj(e12), eq. (8)  */
  bool negt;          /* real case: sign bit of r'_12                */
  Cx<T> dh;           /* e^{i arg r'_22} = D^_22, eq. (9)            */
  bool negh;          /* real case: sign bit of r'_22                */
  T n1, n2;
  T x, y, t2, tphi, sec2phi, cphi, tpsi, sec2psi, cpsi;
};

/* ---------------------------------------------------------------------------
 * Section 2.3, eqs. (13)-(17) with the operation order of Fig. 10: the SVD of
 * the non-negative upper-triangular R = [[r11, r12], [0, r22]].
 * ------------------------------------------------------------------------- */
template <class T> void triangular_svd(const Prim<T> &P, Mid<T> &m, T &smax, T &smin) {
  const T one = T(1), zero = T(0);
  m.x = rmax(m.r12 / m.r11, zero);                              /* eq. (13) */
  m.y = rmax(m.r22 / m.r11, zero);
  T lo = rmin(m.x, m.y), hi = rmax(m.x, m.y);
  T num = std::ldexp(lo, 1) * hi;                               /* (2 min) max */
  T den = fmaT(m.x - m.y, m.x + m.y, one);
  m.t2 = -rmin(rmax(num / den, zero), Lim<T>::f());             /* eq. (14), sign forced */
  m.tphi = m.t2 / (one + sqrtT(fmaT(m.t2, m.t2, one)));         /* eq. (15) */
  m.sec2phi = fmaT(m.tphi, m.tphi, one);
  m.cphi = P.isq(m.sec2phi);
  m.tpsi = fmaT(m.y, m.tphi, -m.x);                             /* eq. (16) */
  m.sec2psi = fmaT(m.tpsi, m.tpsi, one);
  m.cpsi = P.isq(m.sec2psi);
  T k = m.cphi * m.cpsi;                                        /* eq. (17) */
  smax = (k * m.sec2psi) * m.r11;
  smin = (k * m.sec2phi) * m.r22;
}

/* ---------------------------------------------------------------------------
 * The sine form of the assembly, eq. (31), for the comparison of section 8:
 * sin(alpha) = cos(alpha) tan(alpha) and sin(phi) = cos(phi) tan(phi) (the
 * relation section 7 gives), the four products cc = cos a cos p, ss = sin a
 * sin p, cs = cos a sin p, sc = sin a cos p, one fma per element with the
 * phase d^ (reading: eq. (31) fixes no operation order), then d_11 or d_22.
 * tan(alpha) = -mt.  V is the same in both forms (cos psi tan psi is sin psi).
 * ------------------------------------------------------------------------- */
template <class W> struct SineW { W cc, ss, cs, sc; };
template <class W> SineW<W> sine_products(W ca, W mt, W cphi, W tphi) {
  W sa = ca * -mt, sphi = cphi * tphi;
  return {ca * cphi, sa * sphi, ca * sphi, sa * cphi};
}
/* complex: P_r^* U before the row permutation */
template <class W>
void sine_u_cplx(const SineW<W> &q, Cx<W> dh, Cx<W> d1, Cx<W> d2, Cx<W> (&U)[2][2]) {
  Cx<W> w11 = {fmaT(-dh.re, q.ss, q.cc), -(dh.im * q.ss)};
  Cx<W> w12 = {fmaT(dh.re, q.sc, q.cs), dh.im * q.sc};
  Cx<W> w21 = {fmaT(dh.re, q.cs, q.sc), dh.im * q.cs};
  Cx<W> w22 = {fmaT(dh.re, q.cc, -q.ss), dh.im * q.cc};
  Cx<W> p21 = cmul(d2, w21);
  U[0][0] = cmul(d1, w11); U[0][1] = cmul(d1, w12);
  U[1][0] = {-p21.re, -p21.im}; U[1][1] = cmul(d2, w22);
}
/* real: the phases are signs (neg1, neg2: d_11, d_22 = -1; dh = +-1) */
template <class W> void sine_u_real(const SineW<W> &q, W dh, bool neg1, bool neg2, W (&U)[2][2]) {
  W w11 = fmaT(-dh, q.ss, q.cc), w12 = fmaT(dh, q.sc, q.cs), w21 = fmaT(dh, q.cs, q.sc),
    w22 = fmaT(dh, q.cc, -q.ss);
  U[0][0] = neg1 ? -w11 : w11; U[0][1] = neg1 ? -w12 : w12;
  U[1][0] = -(neg2 ? -w21 : w21); U[1][1] = neg2 ? -w22 : w22;
}

/* Section 2.1, eq. (2), Fig. 3: s and A^ = 2^s A over ncomp components. */
template <class T> T scaling(const T *a, int ncomp, T *ah) {
  T s = Lim<T>::big();
  for (int i = 0; i < ncomp; ++i) s = rmin(s, scale_exponent(a[i]));
  for (int i = 0; i < ncomp; ++i) ah[i] = scalef(a[i], s);
  return s;
}

/* ---------------------------------------------------------------------------
 * Assembly of U and V, eq. (29) and its expansion (section 2.3), or eq. (31)
 * with P.sine, then the row permutations P_r (U) and P_c (V).  Reads alpha
 * (ca, mt), the angles phi and psi (tphi, cphi, tpsi, cpsi) and the phases of
 * m; C = cos(alpha) cos(phi), t = -tan(alpha) tan(phi), tan(alpha) = -mt.
 * V = cos(psi) P_c [[1, tan psi], [-d~ tan psi, d~]], d~ = conj(e12).
 * ------------------------------------------------------------------------- */
template <class T> void assemble_cplx(const Prim<T> &P, const Mid<T> &m, Res<T> &o) {
  const T one = T(1);
  T C = m.ca * m.cphi, ta = -m.mt, t = m.mt * m.tphi;
  Cx<T> w11 = {fmaT(m.dh.re, t, one), m.dh.im * t};
  Cx<T> w21 = {fmaT(m.dh.re, m.tphi, ta), m.dh.im * m.tphi};
  Cx<T> w12 = {fmaT(m.dh.re, ta, m.tphi), m.dh.im * ta};
  Cx<T> w22 = {fmaT(m.mt, m.tphi, m.dh.re), m.dh.im};
  Cx<T> p11 = cmul(m.d1, w11), p21 = cmul(m.d2, w21), p12 = cmul(m.d1, w12), p22 = cmul(m.d2, w22);
  Cx<T> U[2][2] = {{{C * p11.re, C * p11.im}, {C * p12.re, C * p12.im}},
                   {{-(C * p21.re), -(C * p21.im)}, {C * p22.re, C * p22.im}}};
  if (P.sine) sine_u_cplx(sine_products(m.ca, m.mt, m.cphi, m.tphi), m.dh, m.d1, m.d2, U);
  if (m.r) { std::swap(U[0][0], U[1][0]); std::swap(U[0][1], U[1][1]); } /* P_r */
  T ct = m.cpsi * m.tpsi;
  Cx<T> V[2][2] = {{{m.cpsi, T(0)}, {ct, T(0)}},
                   {{-(ct * m.e12.re), ct * m.e12.im}, {m.cpsi * m.e12.re, -(m.cpsi * m.e12.im)}}};
  if (m.c) { std::swap(V[0][0], V[1][0]); std::swap(V[0][1], V[1][1]); } /* P_c */
  for (int i = 0; i < 2; ++i) for (int j = 0; j < 2; ++j) { o.u[i][j] = U[i][j]; o.v[i][j] = V[i][j]; }
}

/* the real case: the phases are the signs neg1, neg2, negt and dh = +-1 */
template <class T> void assemble_real(const Prim<T> &P, const Mid<T> &m, Res<T> &o) {
  const T one = T(1);
  T C = m.ca * m.cphi, ta = -m.mt, t = m.mt * m.tphi;
  T dh = m.dh.re;
  T w11 = fmaT(dh, t, one), w21 = fmaT(dh, m.tphi, ta), w12 = fmaT(dh, ta, m.tphi),
    w22 = fmaT(m.mt, m.tphi, dh);
  T U[2][2] = {{C * (m.neg1 ? -w11 : w11), C * (m.neg1 ? -w12 : w12)},
               {-(C * (m.neg2 ? -w21 : w21)), C * (m.neg2 ? -w22 : w22)}};
  if (P.sine) sine_u_real(sine_products(m.ca, m.mt, m.cphi, m.tphi), dh, m.neg1, m.neg2, U);
  if (m.r) { std::swap(U[0][0], U[1][0]); std::swap(U[0][1], U[1][1]); }
  T ct = m.cpsi * m.tpsi;
  T V[2][2] = {{m.cpsi, ct}, {m.negt ? ct : -ct, m.negt ? -m.cpsi : m.cpsi}};
  if (m.c) { std::swap(V[0][0], V[1][0]); std::swap(V[0][1], V[1][1]); }
  for (int i = 0; i < 2; ++i) for (int j = 0; j < 2; ++j) {
    o.u[i][j] = {U[i][j], T(0)};
    o.v[i][j] = {V[i][j], T(0)};
  }
}

/* ---------------------------------------------------------------------------
 * Complex case, one matrix.  a[8] = a11r,a11i,a21r,a21i,a12r,a12i,a22r,a22i.
 * ------------------------------------------------------------------------- */
template <class T> void zsvd2_one(const Prim<T> &P, const T *a, Res<T> &o, Mid<T> &m) {
  const T one = T(1);
  /* scaling, eq. (2) */
  T ahv[8];
  m.s = scaling(a, 8, ahv);
  Cx<T> A[2][2] = {{{ahv[0], ahv[1]}, {ahv[4], ahv[5]}},
                   {{ahv[2], ahv[3]}, {ahv[6], ahv[7]}}}; /* A[i][j] = a^_{i+1,j+1} */
  for (int i = 0; i < 2; ++i) for (int j = 0; j < 2; ++j) m.ah[i][j] = A[i][j];
  /* |a^_ij| by eq. (1) and the column norms of eq. (3), Fig. 4 */
  T mag[2][2];
  for (int i = 0; i < 2; ++i) for (int j = 0; j < 2; ++j) mag[i][j] = P.hyp(A[i][j].re, A[i][j].im);
  T nrm[2] = {P.hyp(mag[0][0], mag[1][0]), P.hyp(mag[0][1], mag[1][1])};
  /* column pivoting P_c (section 2.2, Fig. 5): swap iff ||a^_1|| < ||a^_2|| */
  m.c = nrm[0] < nrm[1];
  if (m.c) {
    for (int i = 0; i < 2; ++i) { std::swap(A[i][0], A[i][1]); std::swap(mag[i][0], mag[i][1]); }
    std::swap(nrm[0], nrm[1]);
  }
  m.n1 = nrm[0]; m.n2 = nrm[1];
  /* row sorting P_r* (Fig. 6): swap iff |a'_11| < |a'_21| */
  m.r = mag[0][0] < mag[1][0];
  if (m.r) {
    for (int j = 0; j < 2; ++j) { std::swap(A[0][j], A[1][j]); std::swap(mag[0][j], mag[1][j]); }
  }
  /* D*, eq. (4), Fig. 7: a'''_i1 = |a''_i1|, a'''_i2 = conj(d_i) a''_i2 */
  m.d1 = phase(P, A[0][0], mag[0][0]);
  m.d2 = phase(P, A[1][0], mag[1][0]);
  T a311 = mag[0][0], a321 = mag[1][0];
  Cx<T> a312 = cmulc(m.d1, A[0][1]);
  Cx<T> a322 = cmulc(m.d2, A[1][1]);
  /* Givens QR, eqs. (6)-(7), Fig. 8.  mt = -tan(alpha) >= 0. */
  m.r11 = nrm[0];
  m.mt = rmax(a321 / a311, T(0));
  m.ca = P.isq(fmaT(m.mt, m.mt, one));
  Cx<T> r12p = {m.ca * fmaT(m.mt, a322.re, a312.re), m.ca * fmaT(m.mt, a322.im, a312.im)};
  Cx<T> r22pp = {m.ca * fmaT(-m.mt, a312.re, a322.re), m.ca * fmaT(-m.mt, a312.im, a322.im)};
  /* D~, eq. (8), Fig. 9: r12 = |r'_12|, r'_22 = r''_22 conj(e^{i arg r'_12}) */
  m.r12 = P.hyp(r12p.re, r12p.im);
  m.e12 = phase(P, r12p, m.r12);
  Cx<T> r22p = {fmaT(r22pp.re, m.e12.re, r22pp.im * m.e12.im),
                fmaT(r22pp.im, m.e12.re, -(r22pp.re * m.e12.im))};
  /* D^, eq. (9), Fig. 9: r22 = |r'_22| */
  m.r22 = P.hyp(r22p.re, r22p.im);
  m.dh = phase(P, r22p, m.r22);
  /* triangular SVD, eqs. (13)-(17) */
  triangular_svd(P, m, o.smax, o.smin);
  assemble_cplx(P, m, o);
  o.s = m.s;
}

/* ---------------------------------------------------------------------------
 * Real case, one matrix.  a[4] = a11, a21, a12, a22.  D*, D~ and D^ of
 * eq. (10) are sign flips (the sign bit of the pivot, -0 counting as
 * negative), applied as negations.
 * ------------------------------------------------------------------------- */
template <class T> void dsvd2_one(const Prim<T> &P, const T *a, Res<T> &o, Mid<T> &m) {
  const T one = T(1);
  T ahv[4];
  m.s = scaling(a, 4, ahv);
  T A[2][2] = {{ahv[0], ahv[2]}, {ahv[1], ahv[3]}};
  for (int i = 0; i < 2; ++i) for (int j = 0; j < 2; ++j) m.ah[i][j] = {A[i][j], T(0)};
  T mag[2][2];
  for (int i = 0; i < 2; ++i) for (int j = 0; j < 2; ++j) mag[i][j] = std::fabs(A[i][j]);
  T nrm[2] = {P.hyp(mag[0][0], mag[1][0]), P.hyp(mag[0][1], mag[1][1])};
  m.c = nrm[0] < nrm[1];
  if (m.c) {
    for (int i = 0; i < 2; ++i) { std::swap(A[i][0], A[i][1]); std::swap(mag[i][0], mag[i][1]); }
    std::swap(nrm[0], nrm[1]);
  }
  m.n1 = nrm[0]; m.n2 = nrm[1];
  m.r = mag[0][0] < mag[1][0];
  if (m.r) {
    for (int j = 0; j < 2; ++j) { std::swap(A[0][j], A[1][j]); std::swap(mag[0][j], mag[1][j]); }
  }
  m.neg1 = std::signbit(A[0][0]);
  m.neg2 = std::signbit(A[1][0]);
  m.d1 = {m.neg1 ? -one : one, T(0)};
  m.d2 = {m.neg2 ? -one : one, T(0)};
  T a311 = mag[0][0], a321 = mag[1][0];
  T a312 = m.neg1 ? -A[0][1] : A[0][1];
  T a322 = m.neg2 ? -A[1][1] : A[1][1];
  m.r11 = nrm[0];
  m.mt = rmax(a321 / a311, T(0));
  m.ca = P.isq(fmaT(m.mt, m.mt, one));
  T r12p = m.ca * fmaT(m.mt, a322, a312);
  T r22pp = m.ca * fmaT(-m.mt, a312, a322);
  m.negt = std::signbit(r12p);
  m.e12 = {m.negt ? -one : one, T(0)};
  m.r12 = std::fabs(r12p);
  T r22p = m.negt ? -r22pp : r22pp;
  m.negh = std::signbit(r22p);
  m.dh = {m.negh ? -one : one, T(0)};
  m.r22 = std::fabs(r22p);
  triangular_svd(P, m, o.smax, o.smin);
  assemble_real(P, m, o);
  o.s = m.s;
}

/* ---------------------------------------------------------------------------
 * Backscaling, eq. (28) and Fig. 1.
 * ------------------------------------------------------------------------- */
template <class T> void backscale(Res<T> &o, int mode) {
  if (mode == ORACLE_BS_NONE) return;
  T smax = o.smax, smin = o.smin; /* zero matrix (s = BIG): sigma' = 0 already */
  if (o.s != Lim<T>::big()) {
    T ns = -o.s; /* negation by the sign bit, as in Fig. 1 */
    smax = scalef(o.smax, ns);
    smin = scalef(o.smin, ns);
  }
  if (mode == ORACLE_BS_SAFE) {
    bool exact = std::isfinite(smax) && std::isfinite(smin) &&
                 scalef(smax, o.s) == o.smax && scalef(smin, o.s) == o.smin;
    if (!exact) return;
  }
  o.smax = smax; o.smin = smin; o.s = -T(0);
}

/* ---------------------------------------------------------------------------
 * FP64 rescue of a near-degenerate FP32 lane.
 *
 * In FP32 the (2,2) entry of R'' in eq. (6) is a difference that cancels when
 * A is nearly singular, so sigma'_min loses relative accuracy.  Its magnitude
 * is fixed by det: r11 r'_22 = det(R') = det(Q*) det(D*) det(P_r*) det(A^)
 * det(P_c) det(D~) with det(Q*) = 1, each swap contributing -1, and
 * det(D*) = conj(d1 d2), det(D~) = conj(e12).  Products of two FP32 numbers
 * are exact in FP64, so det(A^) is formed in FP64 with a compensated sum, r'_22
 * is recomputed from it, and eqs. (9), (13)-(17) and (29) are evaluated in
 * FP64 from the FP32 pivots, phases and rotation alpha.  The result is
 * rounded to FP32.
 * ------------------------------------------------------------------------- */
inline void two_sum(double a, double b, double &s, double &e) {
  s = a + b;
  double bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}
/* a + b + c + d, accumulated with error-free transformations (cascaded
 * TwoSum with the rounding errors summed separately). */
inline double sum4(double a, double b, double c, double d) {
  double s, e, acc;
  two_sum(a, b, s, acc);
  two_sum(s, c, s, e); acc += e;
  two_sum(s, d, s, e); acc += e;
  return s + acc;
}

/* det(A^) in FP64 from the scaled FP32 entries: every product of two FP32
   numbers is exact in FP64; the complex case sums four exact terms per part. */
template <bool CPLX> Cx<double> det_fp64(const Mid<float> &m) {
  Cx<double> a[2][2];
  for (int i = 0; i < 2; ++i) for (int j = 0; j < 2; ++j) a[i][j] = {(double)m.ah[i][j].re, (double)m.ah[i][j].im};
  Cx<double> det;
  if (CPLX) {
    det.re = sum4(a[0][0].re * a[1][1].re, -(a[0][0].im * a[1][1].im),
                  -(a[0][1].re * a[1][0].re), a[0][1].im * a[1][0].im);
    det.im = sum4(a[0][0].re * a[1][1].im, a[0][0].im * a[1][1].re,
                  -(a[0][1].re * a[1][0].im), -(a[0][1].im * a[1][0].re));
  } else {
    det.re = a[0][0].re * a[1][1].re - a[0][1].re * a[1][0].re;
    det.im = 0.0;
  }
  return det;
}

/* The cheaper rescue: only sigma'_min = |det(A^)| / sigma'_max in FP64 (the
   product of the singular values is |det|); U, V and sigma'_max stay FP32. */
template <bool CPLX> void rescue_sigma(const Mid<float> &m, Res<float> &o) {
  Cx<double> det = det_fp64<CPLX>(m);
  double ad = CPLX ? hypot_mirror<double>(det.re, det.im) : std::fabs(det.re);
  o.smin = (float)(ad / (double)o.smax);
}

/* The FP64 half shared by the two rescues below: r'_22 from det(A^), D^ of
   eq. (9) and the triangular SVD of eqs. (13)-(17) in FP64, from the FP32
   r11, r12, alpha and phases of m.  w receives mt, ca, the angles and D^. */
template <bool CPLX> void fp64_triangle(const Prim<double> &P, const Mid<float> &m, Mid<double> &w,
                                        double &smax, double &smin) {
  const double one = 1.0;
  Cx<double> det = det_fp64<CPLX>(m);
  double sgn = (m.c != m.r) ? -one : one;
  w.r11 = m.r11; w.r12 = m.r12; w.mt = m.mt; w.ca = m.ca;
  double r22p_re, r22p_im;
  if (CPLX) {
    Cx<double> d1 = {m.d1.re, m.d1.im}, d2 = {m.d2.re, m.d2.im}, e = {m.e12.re, m.e12.im};
    Cx<double> ph = cmul(cmul(d1, d2), e);  /* d1 d2 e12; det(D*)det(D~) = conj of it */
    Cx<double> q = cmulc(ph, det);          /* conj(d1 d2 e12) det(A^) */
    r22p_re = sgn * (q.re / w.r11);
    r22p_im = sgn * (q.im / w.r11);
    w.r22 = P.hyp(r22p_re, r22p_im);
    w.dh = phase(P, Cx<double>{r22p_re, r22p_im}, w.r22);
  } else {
    if (m.neg1 != m.neg2) sgn = -sgn;
    if (m.negt) sgn = -sgn;
    r22p_re = sgn * (det.re / w.r11);
    w.negh = std::signbit(r22p_re);
    w.r22 = std::fabs(r22p_re);
    w.dh = {w.negh ? -one : one, 0.0};
  }
  triangular_svd(P, w, smax, smin);
}

/* The middle rescue: FP64 only up to the triangular SVD (the steps whose
   stability the near-singular case needs: r'_22 and with it sigma'_min, and
   the rotation angles phi and psi), whose tangents, cosines and phase d^ are
   rounded to FP32; U and V are then assembled in FP32 by the plain lane's
   formulas, with the FP32 alpha and phases. */
template <bool CPLX> void rescue_tri(const Mid<float> &m, Res<float> &o, bool sine = false) {
  Prim<double> P{ORACLE_MIRROR};
  Mid<double> w{};
  double smax, smin;
  fp64_triangle<CPLX>(P, m, w, smax, smin);
  Mid<float> f = m;
  f.tphi = (float)w.tphi; f.cphi = (float)w.cphi;
  f.tpsi = (float)w.tpsi; f.cpsi = (float)w.cpsi;
  f.dh = {(float)w.dh.re, (float)w.dh.im};
  f.negh = w.negh;
  Prim<float> P32{ORACLE_MIRROR, sine};
  if (CPLX) assemble_cplx(P32, f, o); else assemble_real(P32, f, o);
  o.smax = (float)smax;
  o.smin = (float)smin;
}

template <bool CPLX> void rescue_fp64(const Mid<float> &m, Res<float> &o, bool sine = false) {
  Prim<double> P{ORACLE_MIRROR};
  const double one = 1.0;
  Mid<double> w{};
  double smax, smin;
  fp64_triangle<CPLX>(P, m, w, smax, smin);
  double C = w.ca * w.cphi, ta = -w.mt, t = w.mt * w.tphi;
  Cx<double> U[2][2], V[2][2];
  double ct = w.cpsi * w.tpsi;
  if (CPLX) {
    Cx<double> d1 = {m.d1.re, m.d1.im}, d2 = {m.d2.re, m.d2.im}, e = {m.e12.re, m.e12.im};
    Cx<double> w11 = {fmaT(w.dh.re, t, one), w.dh.im * t};
    Cx<double> w21 = {fmaT(w.dh.re, w.tphi, ta), w.dh.im * w.tphi};
    Cx<double> w12 = {fmaT(w.dh.re, ta, w.tphi), w.dh.im * ta};
    Cx<double> w22 = {fmaT(w.mt, w.tphi, w.dh.re), w.dh.im};
    Cx<double> p11 = cmul(d1, w11), p21 = cmul(d2, w21), p12 = cmul(d1, w12), p22 = cmul(d2, w22);
    U[0][0] = {C * p11.re, C * p11.im}; U[0][1] = {C * p12.re, C * p12.im};
    U[1][0] = {-(C * p21.re), -(C * p21.im)}; U[1][1] = {C * p22.re, C * p22.im};
    if (sine) sine_u_cplx(sine_products(w.ca, w.mt, w.cphi, w.tphi), w.dh, d1, d2, U);
    V[0][0] = {w.cpsi, 0.0}; V[0][1] = {ct, 0.0};
    V[1][0] = {-(ct * e.re), ct * e.im}; V[1][1] = {w.cpsi * e.re, -(w.cpsi * e.im)};
  } else {
    double dh = w.dh.re;
    double w11 = fmaT(dh, t, one), w21 = fmaT(dh, w.tphi, ta), w12 = fmaT(dh, ta, w.tphi),
           w22 = fmaT(w.mt, w.tphi, dh);
    U[0][0] = {C * (m.neg1 ? -w11 : w11), 0.0}; U[0][1] = {C * (m.neg1 ? -w12 : w12), 0.0};
    U[1][0] = {-(C * (m.neg2 ? -w21 : w21)), 0.0}; U[1][1] = {C * (m.neg2 ? -w22 : w22), 0.0};
    if (sine) {
      double Ur[2][2];
      sine_u_real(sine_products(w.ca, w.mt, w.cphi, w.tphi), dh, m.neg1, m.neg2, Ur);
      for (int i = 0; i < 2; ++i) for (int j = 0; j < 2; ++j) U[i][j] = {Ur[i][j], 0.0};
    }
    V[0][0] = {w.cpsi, 0.0}; V[0][1] = {ct, 0.0};
    V[1][0] = {m.negt ? ct : -ct, 0.0}; V[1][1] = {m.negt ? -w.cpsi : w.cpsi, 0.0};
  }
  if (m.r) { std::swap(U[0][0], U[1][0]); std::swap(U[0][1], U[1][1]); }
  if (m.c) { std::swap(V[0][0], V[1][0]); std::swap(V[0][1], V[1][1]); }
  for (int i = 0; i < 2; ++i) for (int j = 0; j < 2; ++j) {
    o.u[i][j] = {(float)U[i][j].re, (float)U[i][j].im};
    o.v[i][j] = {(float)V[i][j].re, (float)V[i][j].im};
  }
  o.smax = (float)smax;
  o.smin = (float)smin;
}

/* Lane flag for the rescue: smin' < 2^-20 smax' (a zero matrix is not flagged). */
inline bool near_degenerate(float smax, float smin) { return smin < std::ldexp(smax, -20); }

/* ---------------------------------------------------------------------------
 * Batched drivers: the loop over matrices (Fig. 2 with a lane width of one).
 * ------------------------------------------------------------------------- */
template <class T, bool CPLX>
void run_one(const Prim<T> &P, const T *const *in, size_t k, Res<T> &o, Mid<T> &m) {
  if (CPLX) {
    T a[8];
    for (int i = 0; i < 8; ++i) a[i] = in[i][k];
    zsvd2_one(P, a, o, m);
  } else {
    T a[4];
    for (int i = 0; i < 4; ++i) a[i] = in[i][k];
    dsvd2_one(P, a, o, m);
  }
}

template <class T, bool CPLX>
void store(const Res<T> &o, T *const *out, size_t k) {
  /* element order 11, 21, 12, 22 */
  const int ii[4] = {0, 1, 0, 1}, jj[4] = {0, 0, 1, 1};
  if (CPLX) {
    for (int e = 0; e < 4; ++e) {
      out[2 * e][k] = o.u[ii[e]][jj[e]].re; out[2 * e + 1][k] = o.u[ii[e]][jj[e]].im;
      out[8 + 2 * e][k] = o.v[ii[e]][jj[e]].re; out[8 + 2 * e + 1][k] = o.v[ii[e]][jj[e]].im;
    }
    out[16][k] = o.smax; out[17][k] = o.smin; out[18][k] = o.s;
  } else {
    for (int e = 0; e < 4; ++e) {
      out[e][k] = o.u[ii[e]][jj[e]].re;
      out[4 + e][k] = o.v[ii[e]][jj[e]].re;
    }
    out[8][k] = o.smax; out[9][k] = o.smin; out[10][k] = o.s;
  }
}

template <class T, bool CPLX>
void batch(size_t n, const T *const *in, T *const *out, int policy, int bs, int rescue,
           uint8_t *flagged, int nthreads) {
  Prim<T> P{policy & ~ORACLE_SINE, (policy & ORACLE_SINE) != 0};
  if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(static) num_threads(nthreads)
  for (long long kk = 0; kk < (long long)n; ++kk) {
    size_t k = (size_t)kk;
    Res<T> o;
    Mid<T> m{};
    run_one<T, CPLX>(P, in, k, o, m);
    bool fl = false;
    if constexpr (std::is_same<T, float>::value) {
      if (rescue && near_degenerate(o.smax, o.smin)) {
        if (rescue == 2) rescue_sigma<CPLX>(m, o);
        else if (rescue == 3) rescue_tri<CPLX>(m, o, P.sine);
        else rescue_fp64<CPLX>(m, o, P.sine);
        fl = true;
      }
    }
    if (flagged) flagged[k] = fl ? 1 : 0;
    backscale(o, bs);
    store<T, CPLX>(o, out, k);
  }
}

/* ---------------------------------------------------------------------------
 * Phase outputs of section 2.2: R of eq. (9) and U_+ = P_r D Q_alpha D^,
 * V_+ = P_c D~ of eq. (11), in the operation order stated in the header.
 * ------------------------------------------------------------------------- */
template <class T> Cx<T> rscale(Cx<T> z, T a) { return {z.re * a, z.im * a}; }

template <class T, bool CPLX> void urv_one(const Mid<T> &m, T *const *f, size_t k) {
  const T one = T(1), zero = T(0);
  const T sa = m.ca * m.mt;
  const Cx<T> d1dh = cmul(m.d1, m.dh), d2dh = cmul(m.d2, m.dh);
  Cx<T> U[2][2] = {{rscale(m.d1, m.ca), rscale(d1dh, sa)}, {rscale(m.d2, sa), rscale(d2dh, m.ca)}};
  U[0][1] = {-U[0][1].re, -U[0][1].im};
  if (m.r) { std::swap(U[0][0], U[1][0]); std::swap(U[0][1], U[1][1]); } /* P_r */
  Cx<T> V[2][2] = {{{one, zero}, {zero, zero}}, {{zero, zero}, {m.e12.re, -m.e12.im}}};
  if (m.c) { std::swap(V[0][0], V[1][0]); std::swap(V[0][1], V[1][1]); } /* P_c */
  f[0][k] = m.r11; f[1][k] = m.r12; f[2][k] = m.r22;
  const int ii[4] = {0, 1, 0, 1}, jj[4] = {0, 0, 1, 1}; /* element order 11, 21, 12, 22 */
  for (int e = 0; e < 4; ++e) {
    if (CPLX) {
      f[3 + 2 * e][k] = U[ii[e]][jj[e]].re; f[4 + 2 * e][k] = U[ii[e]][jj[e]].im;
      f[11 + 2 * e][k] = V[ii[e]][jj[e]].re; f[12 + 2 * e][k] = V[ii[e]][jj[e]].im;
    } else {
      f[3 + e][k] = U[ii[e]][jj[e]].re;
      f[7 + e][k] = V[ii[e]][jj[e]].re;
    }
  }
}

template <class T, bool CPLX>
void urv_batch(size_t n, const T *const *in, T *const *f, int policy, int nthreads) {
  Prim<T> P{policy & ~ORACLE_SINE, false};
  if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(static) num_threads(nthreads)
  for (long long kk = 0; kk < (long long)n; ++kk) {
    Res<T> o;
    Mid<T> m{};
    run_one<T, CPLX>(P, in, (size_t)kk, o, m);
    urv_one<T, CPLX>(m, f, (size_t)kk);
  }
}

template <class T> void fill_trace(const Mid<T> &m, const Res<T> &o, double *tr) {
  double v[ORACLE_TRACE_LEN] = {(double)m.s, (double)m.c, (double)m.r, (double)m.r11,
      (double)m.r12, (double)m.r22, (double)m.mt, (double)m.ca, (double)m.x, (double)m.y,
      (double)m.t2, (double)m.tphi, (double)m.sec2phi, (double)m.cphi, (double)m.tpsi,
      (double)m.sec2psi, (double)m.cpsi, (double)o.smax, (double)o.smin, (double)m.n1,
      (double)m.n2, 0.0};
  std::memcpy(tr, v, sizeof v);
}

/* ---------------------------------------------------------------------------
 * Metrics of section 8 in binary128.
 * ------------------------------------------------------------------------- */
struct Q { __float128 re, im; };
inline Q qmul(Q a, Q b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
inline Q qconj(Q a) { return {a.re, -a.im}; }
inline __float128 qabs2(Q a) { return a.re * a.re + a.im * a.im; }

template <class T>
void metrics_one(int cplx, const T *const *in, const T *const *out, size_t k,
                 double &kappa, double &rho, double &delta, double &eta) {
  Q A[2][2], U[2][2], V[2][2];
  const int ii[4] = {0, 1, 0, 1}, jj[4] = {0, 0, 1, 1};
  for (int e = 0; e < 4; ++e) {
    if (cplx) {
      A[ii[e]][jj[e]] = {(__float128)in[2 * e][k], (__float128)in[2 * e + 1][k]};
      U[ii[e]][jj[e]] = {(__float128)out[2 * e][k], (__float128)out[2 * e + 1][k]};
      V[ii[e]][jj[e]] = {(__float128)out[8 + 2 * e][k], (__float128)out[8 + 2 * e + 1][k]};
    } else {
      A[ii[e]][jj[e]] = {(__float128)in[e][k], 0};
      U[ii[e]][jj[e]] = {(__float128)out[e][k], 0};
      V[ii[e]][jj[e]] = {(__float128)out[4 + e][k], 0};
    }
  }
  int base = cplx ? 16 : 8;
  T smax = out[base][k], smin = out[base + 1][k], s = out[base + 2][k];
  __float128 sig[2];
  if (s == Lim<T>::big()) { sig[0] = smax; sig[1] = smin; }
  else { sig[0] = ldexpq((__float128)smax, -(int)s); sig[1] = ldexpq((__float128)smin, -(int)s); }
  /* eq. (32): kappa = fmin(smax/smin, inf) */
  __float128 kq = sig[0] / sig[1];
  kappa = (kq != kq) ? INFINITY : (double)kq;
  /* eq. (33): ||U Sigma V* - A||_F / ||A||_F, NaN (zero A) -> 0 */
  __float128 num = 0, den = 0;
  for (int i = 0; i < 2; ++i) for (int j = 0; j < 2; ++j) {
    Q acc = {0, 0};
    for (int l = 0; l < 2; ++l) {
      Q t = qmul(U[i][l], qconj(V[j][l]));
      acc.re += sig[l] * t.re; acc.im += sig[l] * t.im;
    }
    Q d = {acc.re - A[i][j].re, acc.im - A[i][j].im};
    num += qabs2(d);
    den += qabs2(A[i][j]);
  }
  __float128 rq = sqrtq(num) / sqrtq(den);
  rho = (rq != rq) ? 0.0 : (double)rq;
  /* eqs. (34)-(35): ||X* X - I||_F */
  auto orth = [](Q X[2][2]) {
    __float128 acc = 0;
    for (int i = 0; i < 2; ++i) for (int j = 0; j < 2; ++j) {
      Q g = {0, 0};
      for (int l = 0; l < 2; ++l) {
        Q t = qmul(qconj(X[l][i]), X[l][j]);
        g.re += t.re; g.im += t.im;
      }
      if (i == j) g.re -= 1;
      acc += qabs2(g);
    }
    return (double)sqrtq(acc);
  };
  delta = orth(U);
  eta = orth(V);
}

template <class T>
void metrics(size_t n, int cplx, const T *const *in, const T *const *out, double *kappa,
             double *rho, double *delta, double *eta, int nthreads) {
  if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(static) num_threads(nthreads)
  for (long long kk = 0; kk < (long long)n; ++kk)
    metrics_one<T>(cplx, in, out, (size_t)kk, kappa[kk], rho[kk], delta[kk], eta[kk]);
}

} /* namespace */

extern "C" {

int oracle_dsvd2(size_t n, const double *const *in, double *const *out, int policy,
                 int backscale_mode, int nthreads) {
  batch<double, false>(n, in, out, policy, backscale_mode, 0, nullptr, nthreads);
  return 0;
}
int oracle_zsvd2(size_t n, const double *const *in, double *const *out, int policy,
                 int backscale_mode, int nthreads) {
  batch<double, true>(n, in, out, policy, backscale_mode, 0, nullptr, nthreads);
  return 0;
}
int oracle_ssvd2(size_t n, const float *const *in, float *const *out, int policy,
                 int backscale_mode, int rescue, uint8_t *flagged, int nthreads) {
  batch<float, false>(n, in, out, policy, backscale_mode, rescue, flagged, nthreads);
  return 0;
}
int oracle_csvd2(size_t n, const float *const *in, float *const *out, int policy,
                 int backscale_mode, int rescue, uint8_t *flagged, int nthreads) {
  batch<float, true>(n, in, out, policy, backscale_mode, rescue, flagged, nthreads);
  return 0;
}

int oracle_urv_d(size_t n, int cplx, const double *const *in, double *const *f, int policy,
                 int nthreads) {
  if (cplx) urv_batch<double, true>(n, in, f, policy, nthreads);
  else urv_batch<double, false>(n, in, f, policy, nthreads);
  return 0;
}
int oracle_urv_s(size_t n, int cplx, const float *const *in, float *const *f, int policy,
                 int nthreads) {
  if (cplx) urv_batch<float, true>(n, in, f, policy, nthreads);
  else urv_batch<float, false>(n, in, f, policy, nthreads);
  return 0;
}

int oracle_trace_d(const double *a, int cplx, int policy, double *trace) {
  Prim<double> P{policy};
  Res<double> o; Mid<double> m{};
  if (cplx) zsvd2_one(P, a, o, m); else dsvd2_one(P, a, o, m);
  fill_trace(m, o, trace);
  return 0;
}
int oracle_trace_s(const float *a, int cplx, int policy, int rescue, double *trace) {
  Prim<float> P{policy};
  Res<float> o; Mid<float> m{};
  if (cplx) zsvd2_one(P, a, o, m); else dsvd2_one(P, a, o, m);
  fill_trace(m, o, trace);
  if (rescue && near_degenerate(o.smax, o.smin)) {
    if (rescue == 2) {
      if (cplx) rescue_sigma<true>(m, o); else rescue_sigma<false>(m, o);
    } else if (rescue == 3) {
      if (cplx) rescue_tri<true>(m, o); else rescue_tri<false>(m, o);
    } else {
      if (cplx) rescue_fp64<true>(m, o); else rescue_fp64<false>(m, o);
    }
    trace[17] = o.smax; trace[18] = o.smin; trace[21] = 1.0;
  }
  return 0;
}

int oracle_metrics_d(size_t n, int cplx, const double *const *in, const double *const *out,
                     double *kappa, double *rho, double *delta, double *eta, int nthreads) {
  metrics<double>(n, cplx, in, out, kappa, rho, delta, eta, nthreads);
  return 0;
}
int oracle_metrics_s(size_t n, int cplx, const float *const *in, const float *const *out,
                     double *kappa, double *rho, double *delta, double *eta, int nthreads) {
  metrics<float>(n, cplx, in, out, kappa, rho, delta, eta, nthreads);
  return 0;
}

} /* extern "C" */

/* ===========================================================================
 * Kogbetliantz method (section 1), plain loops over the whole matrix.
 * =========================================================================== */
namespace {

/* circle-method round robin, see the header */
void kog_pairs(int N, int t, int *pairs) {
  const int M = N - 1, n = N / 2;
  pairs[0] = t;
  pairs[1] = M;
  for (int k = 1; k < n; ++k) {
    int a = (t + k) % M, b = ((t - k) % M + M) % M;
    pairs[2 * k] = a < b ? a : b;
    pairs[2 * k + 1] = a < b ? b : a;
  }
}

template <class T> struct Rot { Cx<T> u[2][2], v[2][2]; T smax, smin; };

/* 2x2 SVD of one pivot block with the batched algorithm above, backscaled. */
/* 2x2 SVD of one pivot block b = [[b_pp, b_pq], [b_qp, b_qq]] with the
 * batched algorithm above, backscaled (Fig. 1).  The paper's SVD always puts
 * sigma_max first (Theorem 1); inside the Kogbetliantz iteration that forces a
 * rotation by about pi/2 whenever |b_pp| < |b_qq|, and the sweep then keeps
 * re-sorting the diagonal.  Reading: in that case the columns of U and V and
 * the two singular values are swapped, so each pivot keeps its larger
 * singular value where its larger diagonal entry was. */
template <class T, bool CPLX> Rot<T> pivot_svd(const Cx<T> b[2][2]) {
  Prim<T> P{ORACLE_MIRROR};
  Res<T> o; Mid<T> m{};
  if (CPLX) {
    T a[8] = {b[0][0].re, b[0][0].im, b[1][0].re, b[1][0].im, b[0][1].re, b[0][1].im,
              b[1][1].re, b[1][1].im};
    zsvd2_one(P, a, o, m);
  } else {
    T a[4] = {b[0][0].re, b[1][0].re, b[0][1].re, b[1][1].re};
    dsvd2_one(P, a, o, m);
  }
  if constexpr (std::is_same<T, float>::value) {
    if (near_degenerate(o.smax, o.smin)) rescue_fp64<CPLX>(m, o);
  }
  backscale(o, ORACLE_BS_ALL);
  Rot<T> r;
  for (int i = 0; i < 2; ++i) for (int j = 0; j < 2; ++j) { r.u[i][j] = o.u[i][j]; r.v[i][j] = o.v[i][j]; }
  r.smax = o.smax; r.smin = o.smin;
  bool swap;
  if (CPLX)
    swap = b[0][0].re * b[0][0].re + b[0][0].im * b[0][0].im <
           b[1][1].re * b[1][1].re + b[1][1].im * b[1][1].im;
  else
    swap = std::fabs(b[0][0].re) < std::fabs(b[1][1].re);
  if (swap) {
    for (int i = 0; i < 2; ++i) { std::swap(r.u[i][0], r.u[i][1]); std::swap(r.v[i][0], r.v[i][1]); }
    std::swap(r.smax, r.smin);
  }
  return r;
}

template <class T, bool CPLX> struct Mat {
  T *A; int lda;
  Cx<T> get(int i, int j) const {
    size_t o = (size_t)i + (size_t)j * lda;
    return CPLX ? Cx<T>{A[2 * o], A[2 * o + 1]} : Cx<T>{A[o], T(0)};
  }
  void set(int i, int j, Cx<T> v) {
    size_t o = (size_t)i + (size_t)j * lda;
    if (CPLX) { A[2 * o] = v.re; A[2 * o + 1] = v.im; } else A[o] = v.re;
  }
};

template <class T> Cx<T> cadd(Cx<T> a, Cx<T> b) { return {a.re + b.re, a.im + b.im}; }

/* [x_.p, x_.q] <- [x_.p, x_.q] W for the 2x2 matrix W (rows i = 0 .. N-1):
 * the column half of a step, also the accumulation of the transformations */
template <class T, bool CPLX>
void rotate_columns(int N, Mat<T, CPLX> &M, int p, int q, const Cx<T> (&w)[2][2]) {
  for (int i = 0; i < N; ++i) {
    Cx<T> c1 = M.get(i, p), c2 = M.get(i, q), o1, o2;
    if (CPLX) {
      o1 = cadd(cmul(c1, w[0][0]), cmul(c2, w[1][0]));
      o2 = cadd(cmul(c1, w[0][1]), cmul(c2, w[1][1]));
    } else {
      o1 = {fmaT(c1.re, w[0][0].re, c2.re * w[1][0].re), T(0)};
      o2 = {fmaT(c1.re, w[0][1].re, c2.re * w[1][1].re), T(0)};
    }
    M.set(i, p, o1); M.set(i, q, o2);
  }
}

/* One parallel step t (section 1): the pivot SVDs, then A <- U_k^* A V_k for
 * every pair.  With U and V given, also U <- U U_k and V <- V V_k, so that
 * A_0 = U A V^* holds for the iterate A throughout. */
template <class T, bool CPLX>
void kog_step(int N, T *A, int lda, int t, T *U = nullptr, int ldu = 0, T *V = nullptr, int ldv = 0) {
  const int n = N / 2;
  Mat<T, CPLX> M{A, lda};
  int *pr = new int[2 * n];
  kog_pairs(N, t, pr);
  Rot<T> *R = new Rot<T>[n];
  for (int k = 0; k < n; ++k) {
    int p = pr[2 * k], q = pr[2 * k + 1];
    Cx<T> b[2][2] = {{M.get(p, p), M.get(p, q)}, {M.get(q, p), M.get(q, q)}};
    R[k] = pivot_svd<T, CPLX>(b);
  }
  /* rows: [a_p.; a_q.] <- U_k^* [a_p.; a_q.] */
  for (int k = 0; k < n; ++k) {
    int p = pr[2 * k], q = pr[2 * k + 1];
    const Rot<T> &r = R[k];
    for (int j = 0; j < N; ++j) {
      Cx<T> b1 = M.get(p, j), b2 = M.get(q, j), t1, t2;
      if (CPLX) {
        t1 = cadd(cmulc(r.u[0][0], b1), cmulc(r.u[1][0], b2));
        t2 = cadd(cmulc(r.u[0][1], b1), cmulc(r.u[1][1], b2));
      } else {
        t1 = {fmaT(r.u[0][0].re, b1.re, r.u[1][0].re * b2.re), T(0)};
        t2 = {fmaT(r.u[0][1].re, b1.re, r.u[1][1].re * b2.re), T(0)};
      }
      M.set(p, j, t1); M.set(q, j, t2);
    }
  }
  /* columns: [a_.p, a_.q] <- [a_.p, a_.q] V_l */
  for (int l = 0; l < n; ++l) rotate_columns<T, CPLX>(N, M, pr[2 * l], pr[2 * l + 1], R[l].v);
  /* accumulated transformations */
  if (U) {
    Mat<T, CPLX> MU{U, ldu}, MV{V, ldv};
    for (int l = 0; l < n; ++l) {
      rotate_columns<T, CPLX>(N, MU, pr[2 * l], pr[2 * l + 1], R[l].u);
      rotate_columns<T, CPLX>(N, MV, pr[2 * l], pr[2 * l + 1], R[l].v);
    }
  }
  /* pivot blocks become diag(sigma_max, sigma_min) */
  for (int k = 0; k < n; ++k) {
    int p = pr[2 * k], q = pr[2 * k + 1];
    M.set(p, p, {R[k].smax, T(0)}); M.set(q, q, {R[k].smin, T(0)});
    M.set(p, q, {T(0), T(0)}); M.set(q, p, {T(0), T(0)});
  }
  delete[] R;
  delete[] pr;
}

template <class T, bool CPLX> void kog_norms(int N, const T *A, int lda, double &off2, double &tot2) {
  off2 = 0; tot2 = 0;
  Mat<T, CPLX> M{const_cast<T *>(A), lda};
  for (int j = 0; j < N; ++j)
    for (int i = 0; i < N; ++i) {
      Cx<T> v = M.get(i, j);
      double a2 = (double)v.re * (double)v.re + (double)v.im * (double)v.im;
      tot2 += a2;
      if (i != j) off2 += a2;
    }
}

template <class T, bool CPLX>
int kog_solve(int N, T *A, int lda, double tol, int max_sweeps, int *sweeps, double *off_rel,
              double *history, T *U = nullptr, int ldu = 0, T *V = nullptr, int ldv = 0,
              int min_sweeps = 0) {
  // Exact power-of-two scaling around the iteration (the idea of eq. (2)
  // applied to the whole matrix): E is the largest binary exponent among the
  // finite nonzero components, A is multiplied by 2^-E before the first
  // sweep and by 2^E after the last.  Each step commutes with it exactly (the
  // 2x2 SVD scales its pivot exactly, the rotations do not depend on scale)
  // unless a value reaches the subnormal range, so the iterates are those of
  // A up to the factor, while the stopping test's sums of squares can neither
  // overflow nor underflow to zero whatever the magnitude of A.
  const int ncomp = CPLX ? 2 : 1;
  int E = 0;
  bool any = false;
  for (int j = 0; j < N; ++j)
    for (int i = 0; i < N * ncomp; ++i) {
      T x = A[(size_t)j * lda * ncomp + i];
      if (x != T(0) && std::isfinite(x)) {
        int e;
        std::frexp(x, &e);
        E = any ? std::max(E, e) : e;
        any = true;
      }
    }
  auto scale = [&](int k) {
    for (int j = 0; j < N; ++j)
      for (int i = 0; i < N * ncomp; ++i) {
        T &x = A[(size_t)j * lda * ncomp + i];
        x = std::ldexp(x, k);
      }
  };
  if (E != 0) scale(-E);
  double off2, tot2;
  kog_norms<T, CPLX>(N, A, lda, off2, tot2);
  const double nrm0 = std::sqrt(tot2);
  int sw = 0;
  int status = 7;
  for (;;) {
    double rel = nrm0 > 0 ? std::sqrt(off2) / nrm0 : 0.0;
    if (history) history[sw] = rel;
    if (off_rel) *off_rel = rel;
    if ((rel < tol || nrm0 == 0) && sw >= min_sweeps) { status = 0; break; }
    if (sw == max_sweeps) break;
    for (int t = 0; t < N - 1; ++t) kog_step<T, CPLX>(N, A, lda, t, U, ldu, V, ldv);
    ++sw;
    kog_norms<T, CPLX>(N, A, lda, off2, tot2);
  }
  if (E != 0) scale(E);
  if (sweeps) *sweeps = sw;
  return status;
}

/* The SVD A_0 = U diag(sigma) V^* of a square matrix by the Kogbetliantz
 * method (section 1): the iteration above with its transformations
 * accumulated from U = V = I, and at least one sweep, so that every diagonal
 * entry of the final iterate is a singular value of some pivot block (real,
 * non-negative).  Then sigma = the diagonal in descending order (equal values
 * by increasing index) and the columns of U and V permuted alike.  A keeps the
 * final iterate.  max_sweeps >= 1. */
template <class T, bool CPLX>
int kog_svd(int N, T *A, int lda, T *U, int ldu, T *V, int ldv, T *sigma, double tol, int max_sweeps,
            int *sweeps, double *off_rel) {
  const int nc = CPLX ? 2 : 1;
  for (int j = 0; j < N; ++j)
    for (int i = 0; i < N * nc; ++i) {
      U[(size_t)j * ldu * nc + i] = (i == j * nc) ? T(1) : T(0);
      V[(size_t)j * ldv * nc + i] = (i == j * nc) ? T(1) : T(0);
    }
  int status = kog_solve<T, CPLX>(N, A, lda, tol, max_sweeps, sweeps, off_rel, nullptr, U, ldu, V, ldv, 1);
  std::vector<int> perm(N);
  std::vector<T> d(N);
  for (int i = 0; i < N; ++i) { perm[i] = i; d[i] = A[(size_t)i * lda * nc + (size_t)i * nc]; }
  std::stable_sort(perm.begin(), perm.end(), [&](int a, int b) { return d[a] > d[b]; });
  std::vector<T> tmp((size_t)N * N * nc);
  for (T *X : {U, V}) {
    const int ld = X == U ? ldu : ldv;
    for (int j = 0; j < N; ++j)
      for (int i = 0; i < N * nc; ++i) tmp[(size_t)j * N * nc + i] = X[(size_t)j * ld * nc + i];
    for (int j = 0; j < N; ++j)
      for (int i = 0; i < N * nc; ++i) X[(size_t)j * ld * nc + i] = tmp[(size_t)perm[j] * N * nc + i];
  }
  for (int i = 0; i < N; ++i) sigma[i] = d[perm[i]];
  return status;
}

} /* namespace */

extern "C" {
int oracle_kog_svd_d(int N, double *A, int lda, double *U, int ldu, double *V, int ldv, double *sigma,
                     int cplx, double tol, int max_sweeps, int *sweeps, double *off_rel) {
  if (max_sweeps < 1) return 6;
  return cplx ? kog_svd<double, true>(N, A, lda, U, ldu, V, ldv, sigma, tol, max_sweeps, sweeps, off_rel)
              : kog_svd<double, false>(N, A, lda, U, ldu, V, ldv, sigma, tol, max_sweeps, sweeps, off_rel);
}
int oracle_kog_svd_s(int N, float *A, int lda, float *U, int ldu, float *V, int ldv, float *sigma,
                     int cplx, double tol, int max_sweeps, int *sweeps, double *off_rel) {
  if (max_sweeps < 1) return 6;
  return cplx ? kog_svd<float, true>(N, A, lda, U, ldu, V, ldv, sigma, tol, max_sweeps, sweeps, off_rel)
              : kog_svd<float, false>(N, A, lda, U, ldu, V, ldv, sigma, tol, max_sweeps, sweeps, off_rel);
}
int oracle_kog_pairs(int N, int t, int *pairs) { kog_pairs(N, t, pairs); return 0; }
int oracle_kog_step_d(int N, double *A, int lda, int t) { kog_step<double, false>(N, A, lda, t); return 0; }
int oracle_kog_step_z(int N, double *A, int lda, int t) { kog_step<double, true>(N, A, lda, t); return 0; }
int oracle_kog_step_s(int N, float *A, int lda, int t) { kog_step<float, false>(N, A, lda, t); return 0; }
int oracle_kog_step_c(int N, float *A, int lda, int t) { kog_step<float, true>(N, A, lda, t); return 0; }
int oracle_kog_norms_d(int N, const double *A, int lda, int cplx, double *off2, double *tot2) {
  if (cplx) kog_norms<double, true>(N, A, lda, *off2, *tot2);
  else kog_norms<double, false>(N, A, lda, *off2, *tot2);
  return 0;
}
int oracle_kog_norms_s(int N, const float *A, int lda, int cplx, double *off2, double *tot2) {
  if (cplx) kog_norms<float, true>(N, A, lda, *off2, *tot2);
  else kog_norms<float, false>(N, A, lda, *off2, *tot2);
  return 0;
}
int oracle_kog_solve_d(int N, double *A, int lda, double tol, int max_sweeps, int *sweeps,
                       double *off_rel, double *history) {
  return kog_solve<double, false>(N, A, lda, tol, max_sweeps, sweeps, off_rel, history);
}
int oracle_kog_solve_z(int N, double *A, int lda, double tol, int max_sweeps, int *sweeps,
                       double *off_rel, double *history) {
  return kog_solve<double, true>(N, A, lda, tol, max_sweeps, sweeps, off_rel, history);
}
int oracle_kog_solve_s(int N, float *A, int lda, double tol, int max_sweeps, int *sweeps,
                       double *off_rel, double *history) {
  return kog_solve<float, false>(N, A, lda, tol, max_sweeps, sweeps, off_rel, history);
}
int oracle_kog_solve_c(int N, float *A, int lda, double tol, int max_sweeps, int *sweeps,
                       double *off_rel, double *history) {
  return kog_solve<float, true>(N, A, lda, tol, max_sweeps, sweeps, off_rel, history);
}
} /* extern "C" */
