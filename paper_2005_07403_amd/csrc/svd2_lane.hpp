// svd2_lane.hpp -- per-lane pipeline of the 2x2 SVD for gfx950.
//
// One lane computes one matrix, branch-free (section 4), with the operation
// order of sections 5-7 (Figs. 3-10) and the expansion of eq. (29).  Every
// arithmetic operation is a single correctly rounded IEEE-754 operation:
// hipcc lowers '/' and sqrt to correctly rounded sequences (checked bitwise by
// the primitive probe), fma is the hardware fused multiply-add, and the file
// is compiled with -ffp-contract=off.
//
// Readings of points the paper leaves open (shared with the documentation):
//  * hypot(a, b) is the division-based fallback of section 5:
//      a' = max(|a|,|b|), b' = min(|a|,|b|), q = b'/max(a', TRUE_MIN),
//      hypot = a' sqrt(fma(q, q, 1)).
//  * invsqrt(x) = 1/sqrt(x), the first remedy named in section 6.
//  * The relaxed min/max of section 2 (NaN first argument -> second argument)
//    are the hardware v_min/v_max: at every use the first argument is a
//    non-negative number or a quiet NaN from 0/0 and the second is a positive
//    constant or a non-negative number, so the IEEE minNum/maxNum result is
//    the relaxed one.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace svd2 {

template <class T> struct Fmt;
template <> struct Fmt<double> {
  static constexpr int h = 1021;                        // DBL_MAX_EXP - 3
  static constexpr double big = 0x1.fffffffffffffp+1023; // DBL_MAX
  static constexpr double tm = 0x1p-1074;                // DBL_TRUE_MIN
  static constexpr double mn = 0x1p-1022;                // DBL_MIN
  static constexpr int pk = 128;                         // 2^pk |z| is normal for a subnormal |z|
  static constexpr double f = 0x1.fffffffffffffp+511;    // sqrt(DBL_MAX), Fig. 10
};
template <> struct Fmt<float> {
  static constexpr int h = 125;                          // FLT_MAX_EXP - 3
  static constexpr float big = 0x1.fffffep+127f;         // FLT_MAX
  static constexpr float tm = 0x1p-149f;                 // FLT_TRUE_MIN
  static constexpr float mn = 0x1p-126f;                 // FLT_MIN
  static constexpr int pk = 64;
  static constexpr float f = 0x1.fffffep+63f;            // sqrt(FLT_MAX) rounded down
};

// ---------------------------------------------------------------------------
// primitives
// ---------------------------------------------------------------------------
__device__ __forceinline__ double vfma(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float vfma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double vsqrt(double a) { return __builtin_sqrt(a); }
__device__ __forceinline__ float vsqrt(float a) { return __builtin_sqrtf(a); }
__device__ __forceinline__ double vmin(double a, double b) { return __builtin_fmin(a, b); }
__device__ __forceinline__ float vmin(float a, float b) { return __builtin_fminf(a, b); }
__device__ __forceinline__ double vmax(double a, double b) { return __builtin_fmax(a, b); }
__device__ __forceinline__ float vmax(float a, float b) { return __builtin_fmaxf(a, b); }
__device__ __forceinline__ double vabs(double a) { return __builtin_fabs(a); }
__device__ __forceinline__ float vabs(float a) { return __builtin_fabsf(a); }
__device__ __forceinline__ double vcopysign(double a, double b) { return __builtin_copysign(a, b); }
__device__ __forceinline__ float vcopysign(float a, float b) { return __builtin_copysignf(a, b); }
// frexp exponent: x = m 2^e, m in [0.5, 1); the true exponent also for subnormals
__device__ __forceinline__ int vfrexp_exp(double a) { return __builtin_amdgcn_frexp_exp(a); }
__device__ __forceinline__ int vfrexp_exp(float a) { return __builtin_amdgcn_frexp_expf(a); }
__device__ __forceinline__ double vldexp(double a, int e) { return __builtin_amdgcn_ldexp(a, e); }
__device__ __forceinline__ float vldexp(float a, int e) { return __builtin_amdgcn_ldexpf(a, e); }
__device__ __forceinline__ bool vsignbit(double a) { return __builtin_signbit(a); }
__device__ __forceinline__ bool vsignbit(float a) { return __builtin_signbit(a); }
// negate when the flag is set (an XOR of the sign bit)
template <class T> __device__ __forceinline__ T flip(bool neg, T a) { return neg ? -a : a; }

// Correctly rounded sqrt(x) and 1/x on the arguments the pipeline gives them.
// Every square root here is of a sum 1 + t^2 (t finite: q in [0, 1] in hyp,
// the tangents of eqs. (7), (15), (16)), so x >= 1, and every reciprocal is of
// such a root, so x is in [1, 2^64] (FP32) or [1, 2^512] (FP64) and 1/x is
// normal.  On that domain the general sequences need neither their range
// reduction of tiny arguments nor their fix-ups of 0, inf and NaN, which
// leaves
//  - FP32 sqrt: the hardware estimate s, then whichever of s - ulp, s,
//    s + ulp the signs of the exact residuals x - (s -+ ulp) s select;
//  - FP64 sqrt: the hardware reciprocal-root estimate y, g = x y, h = y/2,
//    one coupled Newton step on (g, h), then two corrections
//    g += (x - g^2) h;
//  - 1/x in FP64: the hardware reciprocal estimate r, Newton steps on r, and
//    the quotient q = r corrected by q += (1 - x q) r;
//  - 1/x in FP32: see vrcp_ge1 below.
// The square roots and the FP64 reciprocal are the operations the compiler's
// own correctly rounded sqrt and division perform on that domain, so the
// results are the correctly rounded ones bit for bit (checked by the
// primitive probe: FP32 on every argument of the domain, FP64 on samples).
// Non-finite inputs give unspecified lanes anyway, as with the general
// sequences.
__device__ __forceinline__ float vsqrt_ge1(float x) {
  const float s = __builtin_amdgcn_sqrtf(x);
  const float sd = __builtin_bit_cast(float, __builtin_bit_cast(int, s) - 1);
  const float su = __builtin_bit_cast(float, __builtin_bit_cast(int, s) + 1);
  const float rd = vfma(-sd, s, x), ru = vfma(-su, s, x);
  const float t = (rd <= 0.0f) ? sd : s;
  return (ru > 0.0f) ? su : t;
}
__device__ __forceinline__ double vsqrt_ge1(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  double g = x * y, h = y * 0.5;
  const double e = vfma(-h, g, 0.5);
  g = vfma(g, e, g);
  h = vfma(h, e, h);
  g = vfma(vfma(-g, g, x), h, g);
  return vfma(vfma(-g, g, x), h, g);
}
// FP32 reciprocal through FP64: the hardware FP64 reciprocal estimate of x
// after one Newton step, rounded to FP32.  Its relative error (about 2^-48.7
// at worst over all FP32 x) is no proof of correct rounding by itself, so
// the domain is settled by enumeration: the probe compares it with the
// correctly rounded division 1/x on every FP32 x in [1, 2^126).
__device__ __forceinline__ float vrcp_ge1(float x) {
  const double d = x, r = __builtin_amdgcn_rcp(d);
  return (float)vfma(r, vfma(-d, r, 1.0), r);
}
__device__ __forceinline__ double vrcp_ge1(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = vfma(r, vfma(-x, r, 1.0), r);
  r = vfma(r, vfma(-x, r, 1.0), r);
  return vfma(vfma(-x, r, 1.0), r, r);
}

template <class T> __device__ __forceinline__ T hyp(T a, T b) {
  T x = vabs(a), y = vabs(b);
  T hi = vmax(x, y), lo = vmin(x, y);
  T q = lo / vmax(hi, Fmt<T>::tm);
  return hi * vsqrt_ge1(vfma(q, q, T(1)));
}
// invsqrt(x) = 1/sqrt(x) (two correctly rounded operations); x >= 1 at every use
template <class T> __device__ __forceinline__ T rsq(T x) { return vrcp_ge1(vsqrt_ge1(x)); }

template <class T> struct Cx { T re, im; };

// eq. (5)
template <class T> __device__ __forceinline__ Cx<T> cmul(Cx<T> a, Cx<T> b) {
  return {vfma(a.re, b.re, -(a.im * b.im)), vfma(a.re, b.im, a.im * b.re)};
}
// conj(a) b, eq. (5) with the conjugation in the signs (Fig. 7)
template <class T> __device__ __forceinline__ Cx<T> cmulc(Cx<T> a, Cx<T> b) {
  return {vfma(a.re, b.re, a.im * b.im), vfma(a.re, b.im, -(a.im * b.re))};
}
// eq. (1): e^{i arg z} from z and |z| = hyp(Re z, Im z).  Below the normal
// range the rounding error of |z| is no longer relative (z = (-4, 1) 2^-1074
// gives |z| = 4 2^-1074 and a "phase" of modulus > 1, so U would not be
// unitary); there eq. (1) is applied to 2^pk z, an exact scaling that leaves
// the phase unchanged.  Whenever |z| is normal the result is the literal one.
template <class T> __device__ __forceinline__ Cx<T> phase(Cx<T> z, T az) {
  if (az < Fmt<T>::mn) {
    z = Cx<T>{vldexp(z.re, Fmt<T>::pk), vldexp(z.im, Fmt<T>::pk)};
    az = hyp(z.re, z.im);
  }
  return {vcopysign(vmin(vabs(z.re) / az, T(1)), z.re), z.im / vmax(az, Fmt<T>::tm)};
}

// ---------------------------------------------------------------------------
// Section 2.1, eq. (2), Fig. 3.  s = min over components of h - exp2(x), with
// zero components ignored; all-zero -> s = BIG.  Kept as an int (sentinel
// INT_MAX for BIG); ldexp(0, INT_MAX) = 0, so the scaling needs no branch.
// exp2 (the frexp exponent, true also for subnormals) never decreases as |x|
// grows, so the minimum is taken at the component of largest magnitude:
// s = scale_exp(max |x|), one exponent instead of one per component (a zero
// component never attains the maximum unless all are zero).
// ---------------------------------------------------------------------------
constexpr int kSBig = 0x7fffffff;
template <class T> __device__ __forceinline__ int scale_exp(T x) {
  return (x == T(0)) ? kSBig : (Fmt<T>::h + 1 - vfrexp_exp(x));
}
template <class T> __device__ __forceinline__ T s_value(int s) {
  return (s == kSBig) ? Fmt<T>::big : (T)s;
}

// ---------------------------------------------------------------------------
// Section 2.3, eqs. (13)-(17), Fig. 10.
// ---------------------------------------------------------------------------
template <class T> struct Tri {
  T tphi, cphi, tpsi, cpsi, smax, smin;
};
template <class T> __device__ __forceinline__ Tri<T> tri_svd(T r11, T r12, T r22) {
  const T one = T(1), zero = T(0);
  T x = vmax(r12 / r11, zero);
  T y = vmax(r22 / r11, zero);
  T lo = vmin(x, y), hi = vmax(x, y);
  T num = (lo * T(2)) * hi;
  T den = vfma(x - y, x + y, one);
  T t2 = -vmin(vmax(num / den, zero), Fmt<T>::f);
  Tri<T> o;
  o.tphi = t2 / (one + vsqrt_ge1(vfma(t2, t2, one)));
  T sec2phi = vfma(o.tphi, o.tphi, one);
  o.cphi = rsq(sec2phi);
  o.tpsi = vfma(y, o.tphi, -x);
  T sec2psi = vfma(o.tpsi, o.tpsi, one);
  o.cpsi = rsq(sec2psi);
  T k = o.cphi * o.cpsi;
  o.smax = (k * sec2psi) * r11;
  o.smin = (k * sec2phi) * r22;
  return o;
}

// ---------------------------------------------------------------------------
// Real case.  D*, D~, D^ of eq. (10) are sign bits (-0 counts as negative).
// ---------------------------------------------------------------------------
template <class T> struct RealRes {
  T u11, u21, u12, u22, v11, v21, v12, v22, smax, smin;
  int s;
  // kept for the FP64 rescue of FP32 lanes
  T ah11, ah21, ah12, ah22, r11, r12, mt, ca;
  bool c, r, neg1, neg2, negt;
  // kept for the phase outputs
  T r22;
  bool negh;
};

// The sine form of the assembly, eq. (31) (SINE = true, flag SVD2_SINE_FORM):
// sin(alpha) = cos(alpha) tan(alpha), sin(phi) = cos(phi) tan(phi) (section
// 7), the products cc = cos a cos p, ss = sin a sin p, cs = cos a sin p,
// sc = sin a cos p, one fma per element with the phase d^, then d_11 or d_22.
// tan(alpha) = -mt.  V is the same in both forms (cos psi tan psi = sin psi).
template <class W> struct SineW {
  W cc, ss, cs, sc;
};
template <class W> __device__ __forceinline__ SineW<W> sine_products(W ca, W mt, const Tri<W> &t) {
  const W sa = ca * -mt, sphi = t.cphi * t.tphi;
  return SineW<W>{ca * t.cphi, sa * sphi, ca * sphi, sa * t.cphi};
}

// eq. (29) expansion (or eq. (31)) and the final row permutations, real case.
template <class T, class W, bool SINE = false>
__device__ __forceinline__ void real_assemble(const Tri<W> &t, W mt, W ca, bool negh, bool neg1,
                                              bool neg2, bool negt, bool c, bool r, T *u, T *v) {
  const W one = W(1);
  W C = ca * t.cphi, ta = -mt, tt = mt * t.tphi;
  W dh = negh ? -one : one;
  W U11, U12, U21, U22;
  if constexpr (SINE) {
    const SineW<W> q = sine_products(ca, mt, t);
    U11 = flip(neg1, vfma(-dh, q.ss, q.cc));
    U12 = flip(neg1, vfma(dh, q.sc, q.cs));
    U21 = -flip(neg2, vfma(dh, q.cs, q.sc));
    U22 = flip(neg2, vfma(dh, q.cc, -q.ss));
  } else {
    W w11 = vfma(dh, tt, one), w21 = vfma(dh, t.tphi, ta), w12 = vfma(dh, ta, t.tphi),
      w22 = vfma(mt, t.tphi, dh);
    U11 = C * flip(neg1, w11);
    U12 = C * flip(neg1, w12);
    U21 = -(C * flip(neg2, w21));
    U22 = C * flip(neg2, w22);
  }
  W ct = t.cpsi * t.tpsi;
  W V11 = t.cpsi, V12 = ct, V21 = negt ? ct : -ct, V22 = flip(negt, t.cpsi);
  // P_r on the rows of U, P_c on the rows of V; element order 11, 21, 12, 22
  u[0] = (T)(r ? U21 : U11); u[1] = (T)(r ? U11 : U21);
  u[2] = (T)(r ? U22 : U12); u[3] = (T)(r ? U12 : U22);
  v[0] = (T)(c ? V21 : V11); v[1] = (T)(c ? V11 : V21);
  v[2] = (T)(c ? V22 : V12); v[3] = (T)(c ? V12 : V22);
}

template <class T, bool SINE = false>
__device__ __forceinline__ void real_lane(T a11, T a21, T a12, T a22, RealRes<T> &o) {
  const T one = T(1);
  // scaling (eq. (2), Fig. 3)
  int s = scale_exp(vmax(vmax(vabs(a11), vabs(a21)), vmax(vabs(a12), vabs(a22))));
  T b11 = vldexp(a11, s), b21 = vldexp(a21, s), b12 = vldexp(a12, s), b22 = vldexp(a22, s);
  o.s = s;
  o.ah11 = b11; o.ah21 = b21; o.ah12 = b12; o.ah22 = b22;
  // column norms (eq. (3), Fig. 4)
  T n1 = hyp(b11, b21), n2 = hyp(b12, b22);
  // column pivoting (Fig. 5)
  bool c = n1 < n2;
  T p11 = c ? b12 : b11, p21 = c ? b22 : b21, p12 = c ? b11 : b12, p22 = c ? b21 : b22;
  T r11 = c ? n2 : n1;
  // row sorting (Fig. 6)
  bool r = vabs(p11) < vabs(p21);
  T q11 = r ? p21 : p11, q21 = r ? p11 : p21, q12 = r ? p22 : p12, q22 = r ? p12 : p22;
  // D* (eq. (10), Fig. 7)
  bool neg1 = vsignbit(q11), neg2 = vsignbit(q21);
  T a311 = vabs(q11), a321 = vabs(q21);
  T a312 = flip(neg1, q12), a322 = flip(neg2, q22);
  // QR (eqs. (6)-(7), Fig. 8)
  T mt = vmax(a321 / a311, T(0));
  T ca = rsq(vfma(mt, mt, one));
  T r12p = ca * vfma(mt, a322, a312);
  T r22pp = ca * vfma(-mt, a312, a322);
  // D~, D^ (eq. (10), Fig. 9)
  bool negt = vsignbit(r12p);
  T r12 = vabs(r12p);
  T r22p = flip(negt, r22pp);
  bool negh = vsignbit(r22p);
  T r22 = vabs(r22p);
  Tri<T> t = tri_svd(r11, r12, r22);
  T u[4], v[4];
  real_assemble<T, T, SINE>(t, mt, ca, negh, neg1, neg2, negt, c, r, u, v);
  o.u11 = u[0]; o.u21 = u[1]; o.u12 = u[2]; o.u22 = u[3];
  o.v11 = v[0]; o.v21 = v[1]; o.v12 = v[2]; o.v22 = v[3];
  o.smax = t.smax; o.smin = t.smin;
  o.r11 = r11; o.r12 = r12; o.mt = mt; o.ca = ca;
  o.c = c; o.r = r; o.neg1 = neg1; o.neg2 = neg2; o.negt = negt;
  o.r22 = r22; o.negh = negh;
}

// ---------------------------------------------------------------------------
// Complex case.
// ---------------------------------------------------------------------------
template <class T> struct CplxRes {
  Cx<T> u[4], v[4];  // element order 11, 21, 12, 22
  T smax, smin;
  int s;
  Cx<T> ah[4];       // A^ in element order 11, 21, 12, 22 (for the rescue)
  Cx<T> d1, d2, e12;
  T r11, r12, mt, ca;
  bool c, r;
  // kept for the phase outputs
  T r22;
  Cx<T> dh;
};

template <class T, class W, bool SINE = false>
__device__ __forceinline__ void cplx_assemble(const Tri<W> &t, W mt, W ca, Cx<W> dh, Cx<W> d1,
                                              Cx<W> d2, Cx<W> e12, bool c, bool r, Cx<T> *u,
                                              Cx<T> *v) {
  const W one = W(1);
  W C = ca * t.cphi, ta = -mt, tt = mt * t.tphi;
  Cx<W> U11, U12, U21, U22;
  if constexpr (SINE) {
    const SineW<W> q = sine_products(ca, mt, t);
    const Cx<W> s11 = {vfma(-dh.re, q.ss, q.cc), -(dh.im * q.ss)};
    const Cx<W> s12 = {vfma(dh.re, q.sc, q.cs), dh.im * q.sc};
    const Cx<W> s21 = {vfma(dh.re, q.cs, q.sc), dh.im * q.cs};
    const Cx<W> s22 = {vfma(dh.re, q.cc, -q.ss), dh.im * q.cc};
    const Cx<W> p21 = cmul(d2, s21);
    U11 = cmul(d1, s11);
    U12 = cmul(d1, s12);
    U21 = Cx<W>{-p21.re, -p21.im};
    U22 = cmul(d2, s22);
  } else {
    Cx<W> w11 = {vfma(dh.re, tt, one), dh.im * tt};
    Cx<W> w21 = {vfma(dh.re, t.tphi, ta), dh.im * t.tphi};
    Cx<W> w12 = {vfma(dh.re, ta, t.tphi), dh.im * ta};
    Cx<W> w22 = {vfma(mt, t.tphi, dh.re), dh.im};
    Cx<W> p11 = cmul(d1, w11), p21 = cmul(d2, w21), p12 = cmul(d1, w12), p22 = cmul(d2, w22);
    U11 = Cx<W>{C * p11.re, C * p11.im};
    U12 = Cx<W>{C * p12.re, C * p12.im};
    U21 = Cx<W>{-(C * p21.re), -(C * p21.im)};
    U22 = Cx<W>{C * p22.re, C * p22.im};
  }
  W ct = t.cpsi * t.tpsi;
  Cx<W> V11 = {t.cpsi, W(0)}, V12 = {ct, W(0)};
  Cx<W> V21 = {-(ct * e12.re), ct * e12.im}, V22 = {t.cpsi * e12.re, -(t.cpsi * e12.im)};
  auto pick = [](bool sw, Cx<W> a, Cx<W> b) { return sw ? b : a; };
  auto cvt = [](Cx<W> a) { return Cx<T>{(T)a.re, (T)a.im}; };
  u[0] = cvt(pick(r, U11, U21)); u[1] = cvt(pick(r, U21, U11));
  u[2] = cvt(pick(r, U12, U22)); u[3] = cvt(pick(r, U22, U12));
  v[0] = cvt(pick(c, V11, V21)); v[1] = cvt(pick(c, V21, V11));
  v[2] = cvt(pick(c, V12, V22)); v[3] = cvt(pick(c, V22, V12));
}

// a[8] = a11r, a11i, a21r, a21i, a12r, a12i, a22r, a22i
template <class T, bool SINE = false>
__device__ __forceinline__ void cplx_lane(const T *a, CplxRes<T> &o) {
  const T one = T(1);
  T amax = vabs(a[0]);
#pragma unroll
  for (int i = 1; i < 8; ++i) amax = vmax(amax, vabs(a[i]));
  const int s = scale_exp(amax);
  o.s = s;
  Cx<T> b11 = {vldexp(a[0], s), vldexp(a[1], s)}, b21 = {vldexp(a[2], s), vldexp(a[3], s)};
  Cx<T> b12 = {vldexp(a[4], s), vldexp(a[5], s)}, b22 = {vldexp(a[6], s), vldexp(a[7], s)};
  o.ah[0] = b11; o.ah[1] = b21; o.ah[2] = b12; o.ah[3] = b22;
  // |a^_ij| (eq. (1)) and column norms (eq. (3), Fig. 4)
  T m11 = hyp(b11.re, b11.im), m21 = hyp(b21.re, b21.im);
  T m12 = hyp(b12.re, b12.im), m22 = hyp(b22.re, b22.im);
  T n1 = hyp(m11, m21), n2 = hyp(m12, m22);
  // column pivoting (Fig. 5)
  bool c = n1 < n2;
  auto pick = [](bool sw, Cx<T> x, Cx<T> y) { return sw ? y : x; };
  Cx<T> p11 = pick(c, b11, b12), p21 = pick(c, b21, b22);
  Cx<T> p12 = pick(c, b12, b11), p22 = pick(c, b22, b21);
  T g11 = c ? m12 : m11, g21 = c ? m22 : m21;
  T r11 = c ? n2 : n1;
  // row sorting (Fig. 6)
  bool r = g11 < g21;
  Cx<T> q11 = pick(r, p11, p21), q21 = pick(r, p21, p11);
  Cx<T> q12 = pick(r, p12, p22), q22 = pick(r, p22, p12);
  T h11 = r ? g21 : g11, h21 = r ? g11 : g21;
  // D* (eq. (4), Fig. 7)
  Cx<T> d1 = phase(q11, h11), d2 = phase(q21, h21);
  Cx<T> a312 = cmulc(d1, q12), a322 = cmulc(d2, q22);
  // QR (eqs. (6)-(7), Fig. 8); a'''_11 = h11, a'''_21 = h21
  T mt = vmax(h21 / h11, T(0));
  T ca = rsq(vfma(mt, mt, one));
  Cx<T> r12p = {ca * vfma(mt, a322.re, a312.re), ca * vfma(mt, a322.im, a312.im)};
  Cx<T> r22pp = {ca * vfma(-mt, a312.re, a322.re), ca * vfma(-mt, a312.im, a322.im)};
  // D~ (eq. (8), Fig. 9)
  T r12 = hyp(r12p.re, r12p.im);
  Cx<T> e12 = phase(r12p, r12);
  Cx<T> r22p = {vfma(r22pp.re, e12.re, r22pp.im * e12.im),
                vfma(r22pp.im, e12.re, -(r22pp.re * e12.im))};
  // D^ (eq. (9), Fig. 9)
  T r22 = hyp(r22p.re, r22p.im);
  Cx<T> dh = phase(r22p, r22);
  Tri<T> t = tri_svd(r11, r12, r22);
  cplx_assemble<T, T, SINE>(t, mt, ca, dh, d1, d2, e12, c, r, o.u, o.v);
  o.smax = t.smax; o.smin = t.smin;
  o.d1 = d1; o.d2 = d2; o.e12 = e12;
  o.r11 = r11; o.r12 = r12; o.mt = mt; o.ca = ca;
  o.c = c; o.r = r;
  o.r22 = r22; o.dh = dh;
}

// ---------------------------------------------------------------------------
// FP64 rescue of a near-degenerate FP32 lane (flag: smin' < 2^-20 smax').
// r11 r'_22 = det(R') = det(Q*) det(D*) det(P_r*) det(A^) det(P_c) det(D~),
// det(Q*) = 1, each swap -1, det(D*) = conj(d1 d2), det(D~) = conj(e12).
// FP32 products are exact in FP64; det(A^) is summed with TwoSum.  Then
// eqs. (9), (13)-(17), (29) run in FP64 and the results are rounded to FP32.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void two_sum(double a, double b, double &s, double &e) {
  s = a + b;
  double bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}
__device__ __forceinline__ double sum4(double a, double b, double c, double d) {
  double s, e, acc;
  two_sum(a, b, s, acc);
  two_sum(s, c, s, e);
  acc += e;
  two_sum(s, d, s, e);
  acc += e;
  return s + acc;
}

__device__ __forceinline__ bool near_degenerate(float smax, float smin) {
  return smin < vldexp(smax, -20);
}

// the cheaper rescue: only sigma'_min = |det(A^)| / sigma'_max in FP64
__device__ __forceinline__ void real_rescue_sigma(RealRes<float> &o) {
  double det = (double)o.ah11 * (double)o.ah22 - (double)o.ah12 * (double)o.ah21;
  o.smin = (float)(vabs(det) / (double)o.smax);
}

__device__ __forceinline__ Cx<double> cplx_det(const CplxRes<float> &o) {
  Cx<double> a11 = {o.ah[0].re, o.ah[0].im}, a21 = {o.ah[1].re, o.ah[1].im};
  Cx<double> a12 = {o.ah[2].re, o.ah[2].im}, a22 = {o.ah[3].re, o.ah[3].im};
  return {sum4(a11.re * a22.re, -(a11.im * a22.im), -(a12.re * a21.re), a12.im * a21.im),
          sum4(a11.re * a22.im, a11.im * a22.re, -(a12.re * a21.im), -(a12.im * a21.re))};
}

__device__ __forceinline__ void cplx_rescue_sigma(CplxRes<float> &o) {
  Cx<double> det = cplx_det(o);
  o.smin = (float)(hyp(det.re, det.im) / (double)o.smax);
}

// the FP64 half of the two rescues below: r'_22 from det(A^), D^ (eq. (9))
// and the triangular SVD (eqs. (13)-(17)) in FP64
__device__ __forceinline__ Tri<double> real_triangle64(const RealRes<float> &o, bool &negh) {
  double det = (double)o.ah11 * (double)o.ah22 - (double)o.ah12 * (double)o.ah21;
  bool neg = (o.c != o.r) != ((o.neg1 != o.neg2) != o.negt);
  double r11 = o.r11;
  double r22p = flip(neg, det / r11);
  negh = vsignbit(r22p);
  double r22 = vabs(r22p);
  return tri_svd(r11, (double)o.r12, r22);
}

__device__ __forceinline__ Tri<float> round_tri(const Tri<double> &t) {
  return Tri<float>{(float)t.tphi, (float)t.cphi, (float)t.tpsi, (float)t.cpsi, (float)t.smax, (float)t.smin};
}

// the middle rescue: FP64 up to the triangular SVD, its angles rounded to
// FP32, U and V by the FP32 assembly (the plain lane's formulas)
template <bool SINE = false> __device__ __forceinline__ void real_rescue_tri(RealRes<float> &o) {
  bool negh;
  const Tri<float> t = round_tri(real_triangle64(o, negh));
  float u[4], v[4];
  real_assemble<float, float, SINE>(t, o.mt, o.ca, negh, o.neg1, o.neg2, o.negt, o.c, o.r, u, v);
  o.u11 = u[0]; o.u21 = u[1]; o.u12 = u[2]; o.u22 = u[3];
  o.v11 = v[0]; o.v21 = v[1]; o.v12 = v[2]; o.v22 = v[3];
  o.smax = t.smax;
  o.smin = t.smin;
}

template <bool SINE = false> __device__ __forceinline__ void real_rescue(RealRes<float> &o) {
  bool negh;
  const Tri<double> t = real_triangle64(o, negh);
  float u[4], v[4];
  real_assemble<float, double, SINE>(t, (double)o.mt, (double)o.ca, negh, o.neg1, o.neg2, o.negt, o.c,
                                     o.r, u, v);
  o.u11 = u[0]; o.u21 = u[1]; o.u12 = u[2]; o.u22 = u[3];
  o.v11 = v[0]; o.v21 = v[1]; o.v12 = v[2]; o.v22 = v[3];
  o.smax = (float)t.smax;
  o.smin = (float)t.smin;
}

__device__ __forceinline__ Tri<double> cplx_triangle64(const CplxRes<float> &o, Cx<double> &dh) {
  Cx<double> det = cplx_det(o);
  double sgn = (o.c != o.r) ? -1.0 : 1.0;
  Cx<double> d1 = {o.d1.re, o.d1.im}, d2 = {o.d2.re, o.d2.im}, e = {o.e12.re, o.e12.im};
  Cx<double> ph = cmul(cmul(d1, d2), e);
  Cx<double> q = cmulc(ph, det);
  double r11 = o.r11;
  Cx<double> r22p = {sgn * (q.re / r11), sgn * (q.im / r11)};
  double r22 = hyp(r22p.re, r22p.im);
  dh = phase(r22p, r22);
  return tri_svd(r11, (double)o.r12, r22);
}

template <bool SINE = false> __device__ __forceinline__ void cplx_rescue_tri(CplxRes<float> &o) {
  Cx<double> dh;
  const Tri<float> t = round_tri(cplx_triangle64(o, dh));
  const Cx<float> dhf = {(float)dh.re, (float)dh.im};
  cplx_assemble<float, float, SINE>(t, o.mt, o.ca, dhf, o.d1, o.d2, o.e12, o.c, o.r, o.u, o.v);
  o.smax = t.smax;
  o.smin = t.smin;
}

template <bool SINE = false> __device__ __forceinline__ void cplx_rescue(CplxRes<float> &o) {
  Cx<double> dh;
  const Tri<double> t = cplx_triangle64(o, dh);
  Cx<double> d1 = {o.d1.re, o.d1.im}, d2 = {o.d2.re, o.d2.im}, e = {o.e12.re, o.e12.im};
  cplx_assemble<float, double, SINE>(t, (double)o.mt, (double)o.ca, dh, d1, d2, e, o.c, o.r, o.u, o.v);
  o.smax = (float)t.smax;
  o.smin = (float)t.smin;
}

// ---------------------------------------------------------------------------
// Backscale (eq. (28), Fig. 1).  mode 1: only where exact and finite.
// Returns the value to store for s.
// ---------------------------------------------------------------------------
template <class T> __device__ __forceinline__ T backscale(int mode, int s, T &smax, T &smin) {
  T sv = s_value<T>(s);
  if (mode == 0) return sv;
  if (s == kSBig) return -T(0);  // zero matrix: sigma' = Sigma = 0
  T bmax = vldexp(smax, -s), bmin = vldexp(smin, -s);
  if (mode == 1) {
    bool ok = __builtin_isfinite(bmax) && __builtin_isfinite(bmin) && vldexp(bmax, s) == smax &&
              vldexp(bmin, s) == smin;
    if (!ok) return sv;
  }
  smax = bmax;
  smin = bmin;
  return -T(0);
}

// ---------------------------------------------------------------------------
// Phase outputs of the URV factorization (section 2.2; section 4 allows the
// output of a phase to be written beside the final results): f = r11, r12,
// r22 of eq. (9), then, with UPV, U_+ = P_r D Q_alpha D^ and V_+ = P_c D~ of
// eq. (11) in the element order of U and V.  With D = diag(d1, d2), Q_alpha =
// cos(alpha) [[1, -mt], [mt, 1]] and D^ = diag(1, dh), before the row swap
// u11 = d1 ca, u21 = d2 sa, u12 = -((d1 dh) sa), u22 = (d2 dh) ca, sa = ca mt
// (one rounding per product, d1 dh by eq. (5)); V_+ is [[1, 0], [0,
// conj(e12)]] before the row swap.  In the real case the phases are the signs
// of eq. (10), so the products are exact sign changes.
// ---------------------------------------------------------------------------
template <class T, bool UPV> __device__ __forceinline__ void real_urv(const RealRes<T> &o, T *f) {
  f[0] = o.r11; f[1] = o.r12; f[2] = o.r22;
  if constexpr (UPV) {
    const T sa = o.ca * o.mt, one = T(1), zero = T(0);
    const T u11 = flip(o.neg1, o.ca), u21 = flip(o.neg2, sa);
    const T u12 = -flip(o.neg1 != o.negh, sa), u22 = flip(o.neg2 != o.negh, o.ca);
    f[3] = o.r ? u21 : u11; f[4] = o.r ? u11 : u21;
    f[5] = o.r ? u22 : u12; f[6] = o.r ? u12 : u22;
    const T v22 = o.negt ? -one : one;
    f[7] = o.c ? zero : one; f[8] = o.c ? one : zero;
    f[9] = o.c ? v22 : zero; f[10] = o.c ? zero : v22;
  }
}

template <class T, bool UPV> __device__ __forceinline__ void cplx_urv(const CplxRes<T> &o, T *f) {
  f[0] = o.r11; f[1] = o.r12; f[2] = o.r22;
  if constexpr (UPV) {
    const T sa = o.ca * o.mt, one = T(1), zero = T(0);
    const Cx<T> d1dh = cmul(o.d1, o.dh), d2dh = cmul(o.d2, o.dh);
    const Cx<T> u11 = {o.d1.re * o.ca, o.d1.im * o.ca}, u21 = {o.d2.re * sa, o.d2.im * sa};
    const Cx<T> u12 = {-(d1dh.re * sa), -(d1dh.im * sa)}, u22 = {d2dh.re * o.ca, d2dh.im * o.ca};
    const Cx<T> U[4] = {o.r ? u21 : u11, o.r ? u11 : u21, o.r ? u22 : u12, o.r ? u12 : u22};
    const Cx<T> e1 = {one, zero}, e0 = {zero, zero}, v22 = {o.e12.re, -o.e12.im};
    const Cx<T> V[4] = {o.c ? e0 : e1, o.c ? e1 : e0, o.c ? v22 : e0, o.c ? e0 : v22};
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      f[3 + 2 * e] = U[e].re; f[4 + 2 * e] = U[e].im;
      f[11 + 2 * e] = V[e].re; f[12 + 2 * e] = V[e].im;
    }
  }
}

// ---------------------------------------------------------------------------
// one matrix: inputs x[NIN] -> outputs y[NOUT]; returns the rescue flag
// RESCUE: 0 none, 1 in place (FP64 tail on flagged lanes), 2 flag only,
// 3 in place (FP64 sigma_min quotient only), 4 in place (FP64 up to the
// triangular SVD, FP32 assembly)
// ---------------------------------------------------------------------------
// URV (phase outputs into f): 0 none, 1 R, 2 R, U_+ and V_+; the FP32 lanes
// give the FP32 pipeline's values (the rescue recomputes none of them)
template <class T, bool CPLX, int RESCUE, bool SINE = false, int URV = 0>
__device__ __forceinline__ bool one_matrix(const T *x, T *y, int bs, T *f = nullptr) {
  bool flagged = false;
  if constexpr (!CPLX) {
    RealRes<T> o;
    real_lane<T, SINE>(x[0], x[1], x[2], x[3], o);
    if constexpr (URV != 0) real_urv<T, URV == 2>(o, f);
    if constexpr (RESCUE != 0) {
      flagged = near_degenerate(o.smax, o.smin);
      if constexpr (RESCUE == 1) {
        if (flagged) real_rescue<SINE>(o);
      } else if constexpr (RESCUE == 3) {
        if (flagged) real_rescue_sigma(o);
      } else if constexpr (RESCUE == 4) {
        if (flagged) real_rescue_tri<SINE>(o);
      }
    }
    y[0] = o.u11; y[1] = o.u21; y[2] = o.u12; y[3] = o.u22;
    y[4] = o.v11; y[5] = o.v21; y[6] = o.v12; y[7] = o.v22;
    T smax = o.smax, smin = o.smin;
    T sv = backscale<T>(bs, o.s, smax, smin);
    y[8] = smax; y[9] = smin; y[10] = sv;
  } else {
    CplxRes<T> o;
    cplx_lane<T, SINE>(x, o);
    if constexpr (URV != 0) cplx_urv<T, URV == 2>(o, f);
    if constexpr (RESCUE != 0) {
      flagged = near_degenerate(o.smax, o.smin);
      if constexpr (RESCUE == 1) {
        if (flagged) cplx_rescue<SINE>(o);
      } else if constexpr (RESCUE == 3) {
        if (flagged) cplx_rescue_sigma(o);
      } else if constexpr (RESCUE == 4) {
        if (flagged) cplx_rescue_tri<SINE>(o);
      }
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      y[2 * e] = o.u[e].re; y[2 * e + 1] = o.u[e].im;
      y[8 + 2 * e] = o.v[e].re; y[8 + 2 * e + 1] = o.v[e].im;
    }
    T smax = o.smax, smin = o.smin;
    T sv = backscale<T>(bs, o.s, smax, smin);
    y[16] = smax; y[17] = smin; y[18] = sv;
  }
  return flagged;
}

}  // namespace svd2
