// svd2_batch.hip -- batched 2x2 SVD kernels for gfx950 and the C ABI of
// include/svd2.h.
//
// Mapping (section 3 layout, section 4 pipeline): lane k of the grid computes
// matrix k (or matrices 2k, 2k+1 with 16-byte accesses).  Every input array
// is read once and every output array written once, coalesced, with
// non-temporal stores; nothing is staged in LDS because nothing is reused.
// The work is HBM-bound (120 B per real FP64 SVD against ~300 VALU
// instructions), so the kernels keep many loads in flight rather than
// shortening the arithmetic, which must stay bit-for-bit the paper's.
#include "svd2.h"

#include <hip/hip_runtime.h>

#include <atomic>
#include <stdint.h>
#include <string.h>

#include "svd2_lane.hpp"

using namespace svd2;

namespace {

thread_local int g_last_hip = 0;
// launch shape per element type: 0 real FP64, 1 complex FP64, 2 real FP32, 3 complex FP32
// (+4: singular values only)
std::atomic<int> g_block[8] = {{256}, {256}, {256}, {256}, {256}, {256}, {256}, {256}};
std::atomic<int> g_per_thread[8] = {{1}, {1}, {1}, {1}, {1}, {1}, {1}, {1}};
template <class T, bool CPLX> constexpr int kind_of() { return (sizeof(T) == 8 ? 0 : 2) + (CPLX ? 1 : 0); }

template <class T, int NIN, int NOUT> struct KArgs {
  const T *in[NIN];
  T *out[NOUT];
};

typedef double d2v __attribute__((ext_vector_type(2)));
typedef float f2v __attribute__((ext_vector_type(2)));
template <class T> struct Vec2;
template <> struct Vec2<double> { typedef d2v type; };
template <> struct Vec2<float> { typedef f2v type; };

template <class T> __device__ __forceinline__ void st_nt(T *p, T v) { __builtin_nontemporal_store(v, p); }

// ---------------------------------------------------------------------------
// loads / stores of PT consecutive matrices per lane (PT = 2: 16-byte
// accesses; the host launches that form on an even count only).  k is the
// matrix index within one launch, whose arrays span at most kChunkBytes, so
// every access is an array base (the same for the whole grid, held in scalar
// registers) plus one 32-bit byte offset shared by all arrays: no per-array
// 64-bit address arithmetic on the vector ALUs.
// ---------------------------------------------------------------------------
constexpr size_t kChunkBytes = size_t(1) << 30;

template <class P> __device__ __forceinline__ const P *at(const P *base, uint32_t off) {
  return reinterpret_cast<const P *>(reinterpret_cast<const char *>(base) + off);
}
template <class P> __device__ __forceinline__ P *at(P *base, uint32_t off) {
  return reinterpret_cast<P *>(reinterpret_cast<char *>(base) + off);
}

template <class T, int N, int PT>
__device__ __forceinline__ void load_lanes(const T *const (&in)[N], uint32_t k, int cnt, T (&x)[PT][N]) {
  const uint32_t off = k * (uint32_t)sizeof(T);
  if constexpr (PT == 2) {
    typedef typename Vec2<T>::type V;
#pragma unroll
    for (int i = 0; i < N; ++i) {
      V v = *at(reinterpret_cast<const V *>(in[i]), off);
      x[0][i] = v.x;
      x[PT - 1][i] = v.y;
    }
  } else {
#pragma unroll
    for (int j = 0; j < PT; ++j)
#pragma unroll
      for (int i = 0; i < N; ++i) x[j][i] = (j < cnt) ? at(in[i], off)[j] : T(0);
  }
}

// outputs LO .. N-1 only (LO = N-3: sigma'_max, sigma'_min, s)
template <class T, int N, int PT, int LO = 0>
__device__ __forceinline__ void store_lanes(T *const (&out)[N], uint32_t k, int cnt, const T (&y)[PT][N]) {
  const uint32_t off = k * (uint32_t)sizeof(T);
  if constexpr (PT == 2) {
    typedef typename Vec2<T>::type V;
#pragma unroll
    for (int i = LO; i < N; ++i) {
      V v;
      v.x = y[0][i];
      v.y = y[PT - 1][i];
      st_nt(at(reinterpret_cast<V *>(out[i]), off), v);
    }
  } else {
#pragma unroll
    for (int j = 0; j < PT; ++j)
      if (j < cnt) {
#pragma unroll
        for (int i = LO; i < N; ++i) st_nt(at(out[i], off) + j, y[j][i]);
      }
  }
}

__device__ __forceinline__ unsigned lane_prefix(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u));
}

// the flagged lanes of one matrix per lane (every lane of the wavefront
// calls it): their count is added to nresc (one atomic per wavefront) and,
// for RESCUE == 2, their batch indices idx are appended to the queue
template <int RESCUE>
__device__ __forceinline__ void note_flagged(bool fl, uint32_t idx, uint32_t *nresc, uint32_t *queue,
                                             uint32_t *qcount) {
  const uint64_t m = __ballot(fl);
  if (m == 0) return;
  const unsigned total = (unsigned)__popcll(m);
  const unsigned lane = __lane_id();
  const unsigned first = (unsigned)__ffsll((unsigned long long)m) - 1;
  if (nresc && lane == first) atomicAdd(nresc, total);
  if constexpr (RESCUE == 2) {
    unsigned base = 0;
    if (lane == first) base = atomicAdd(qcount, total);
    base = __shfl(base, (int)first);
    if (fl) queue[base + lane_prefix(m)] = idx;
  }
}

// ---------------------------------------------------------------------------
// Main batched kernel.  RESCUE: 0 plain, 1 in-place FP64 rescue, 2 queue the
// flagged lanes for svd2_rescue_kernel, 3 and 4 the in-place sigma-quotient
// and middle rescues.  UV = false: singular values only; U
// and V are neither stored nor, since nothing uses them, computed (the
// assembly of eq. (29) and its FP64 counterpart in the rescue drop out).
// ---------------------------------------------------------------------------
// One launch covers the n matrices of one chunk (at most kChunkBytes per
// array); k0 is the chunk's first matrix in the whole batch (queue entries
// are whole-batch indices).
template <class T, bool CPLX, int PT, int RESCUE, bool UV, bool SINE>
__global__ __launch_bounds__(256) void svd2_kernel(uint32_t n, KArgs<T, CPLX ? 8 : 4, CPLX ? 19 : 11> a,
                                                   int bs, uint32_t *nresc, uint32_t *queue,
                                                   uint32_t *qcount, uint32_t k0) {
  constexpr int NIN = CPLX ? 8 : 4, NOUT = CPLX ? 19 : 11, LO = UV ? 0 : NOUT - 3;
  const uint32_t k = (blockIdx.x * blockDim.x + threadIdx.x) * PT;
  int cnt = (k < n) ? (int)((n - k < (uint32_t)PT) ? (n - k) : PT) : 0;
  T x[PT][NIN], y[PT][NOUT];
  bool fl[PT];
  if (cnt > 0) load_lanes<T, NIN, PT>(a.in, k, cnt, x);
#pragma unroll
  for (int j = 0; j < PT; ++j) {
    fl[j] = false;
    if (j < cnt) fl[j] = one_matrix<T, CPLX, RESCUE, SINE>(x[j], y[j], bs);
  }
  if (cnt > 0) store_lanes<T, NOUT, PT, LO>(a.out, k, cnt, y);
  if constexpr (RESCUE != 0) {
#pragma unroll
    for (int j = 0; j < PT; ++j) note_flagged<RESCUE>(fl[j], k0 + k + (uint32_t)j, nresc, queue, qcount);
  }
}

// the phase-output arrays: r11, r12, r22, then U_+ and V_+ (11 real, 19 complex)
template <class T, int N> struct OutArgs {
  T *out[N];
};
template <bool CPLX> constexpr int urv_count() { return CPLX ? 19 : 11; }

// The batched kernel with the phase outputs of the URV factorization
// (section 2.2, written beside the final results as section 4 allows): the
// outputs of svd2_kernel, and in f the factor R (UPV = false) or R, U_+ and
// V_+ (UPV = true).  One matrix per lane.
template <class T, bool CPLX, int RESCUE, bool UV, bool SINE, bool UPV>
__global__ __launch_bounds__(256) void svd2_urv_kernel(uint32_t n, KArgs<T, CPLX ? 8 : 4, CPLX ? 19 : 11> a,
                                                       OutArgs<T, urv_count<CPLX>()> f, int bs, uint32_t *nresc,
                                                       uint32_t *queue, uint32_t *qcount, uint32_t k0) {
  constexpr int NIN = CPLX ? 8 : 4, NOUT = CPLX ? 19 : 11, LO = UV ? 0 : NOUT - 3;
  constexpr int NF = UPV ? urv_count<CPLX>() : 3;
  const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  bool fl = false;
  if (k < n) {
    T x[1][NIN], y[1][NOUT], fv[urv_count<CPLX>()];
    load_lanes<T, NIN, 1>(a.in, k, 1, x);
    fl = one_matrix<T, CPLX, RESCUE, SINE, UPV ? 2 : 1>(x[0], y[0], bs, fv);
    store_lanes<T, NOUT, 1, LO>(a.out, k, 1, y);
    const uint32_t off = k * (uint32_t)sizeof(T);
#pragma unroll
    for (int i = 0; i < NF; ++i) st_nt(at(f.out[i], off), fv[i]);
  }
  if constexpr (RESCUE != 0) note_flagged<RESCUE>(fl, k0 + k, nresc, queue, qcount);
}

// Second pass for RESCUE == 2: redo each queued lane with the FP64 tail.  The
// grid is fixed; every lane loops until the device-side count is exhausted.
template <class T, bool CPLX, int TAIL, bool UV, bool SINE>
__global__ __launch_bounds__(256) void svd2_rescue_kernel(KArgs<T, CPLX ? 8 : 4, CPLX ? 19 : 11> a,
                                                          int bs, const uint32_t *queue,
                                                          const uint32_t *qcount) {
  constexpr int NIN = CPLX ? 8 : 4, NOUT = CPLX ? 19 : 11, LO = UV ? 0 : NOUT - 3;
  uint32_t total = *qcount;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
    size_t k = queue[i];
    T x[NIN], y[NOUT];
#pragma unroll
    for (int e = 0; e < NIN; ++e) x[e] = a.in[e][k];
    one_matrix<T, CPLX, TAIL, SINE>(x, y, bs);
#pragma unroll
    for (int e = LO; e < NOUT; ++e) st_nt(a.out[e] + k, y[e]);
  }
}

__global__ void zero_u32_kernel(uint32_t *p) { *p = 0u; }

// ---------------------------------------------------------------------------
// primitive probe
// ---------------------------------------------------------------------------
template <class T>
__global__ __launch_bounds__(256) void probe_kernel(int op, size_t n, const T *x, const T *y,
                                                    const T *z, T *out) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  T r;
  switch (op) {
    case 0: r = x[i] / y[i]; break;
    case 1: r = vsqrt(x[i]); break;
    case 2: r = vfma(x[i], y[i], z[i]); break;
    case 3: r = vldexp(x[i], (int)y[i]); break;
    case 4: r = (T)vfrexp_exp(x[i]); break;
    case 5: r = vmin(x[i], y[i]); break;
    case 6: r = vmax(x[i], y[i]); break;
    case 7: r = vsqrt_ge1(x[i]); break;
    default: r = vrcp_ge1(x[i]); break;
  }
  out[i] = r;
}

// ---------------------------------------------------------------------------
// host-side validation
// ---------------------------------------------------------------------------
struct Span {
  uintptr_t lo, hi;
};

template <class T>
svd2_status check_ptrs(size_t n, const T *const *in, int nin, T *const *out, int nout) {
  for (int i = 0; i < nin; ++i)
    if (!in[i]) return SVD2_ERR_NULL;
  for (int i = 0; i < nout; ++i)
    if (!out[i]) return SVD2_ERR_NULL;
  for (int i = 0; i < nin; ++i)
    if ((uintptr_t)in[i] % sizeof(T)) return SVD2_ERR_ALIGN;
  for (int i = 0; i < nout; ++i)
    if ((uintptr_t)out[i] % sizeof(T)) return SVD2_ERR_ALIGN;
  if (n > SIZE_MAX / sizeof(T)) return SVD2_ERR_SIZE;
  const size_t bytes = n * sizeof(T);
  Span sp[19 + 19];
  int m = 0;
  for (int i = 0; i < nout; ++i) sp[m++] = {(uintptr_t)out[i], (uintptr_t)out[i] + bytes};
  for (int i = 0; i < m; ++i)
    for (int j = i + 1; j < m; ++j)
      if (sp[i].lo < sp[j].hi && sp[j].lo < sp[i].hi) return SVD2_ERR_ALIAS;
  for (int i = 0; i < nin; ++i) {
    Span s = {(uintptr_t)in[i], (uintptr_t)in[i] + bytes};
    for (int j = 0; j < m; ++j)
      if (s.lo < sp[j].hi && sp[j].lo < s.hi) return SVD2_ERR_ALIAS;
  }
  return SVD2_OK;
}

// every array the kernel touches 16-byte aligned (uv = false: U and V are not)
template <class T, int NIN, int NOUT>
bool all_aligned16(const KArgs<T, NIN, NOUT> &a, bool uv = true) {
  for (int i = 0; i < NIN; ++i)
    if ((uintptr_t)a.in[i] % 16) return false;
  for (int i = uv ? 0 : NOUT - 3; i < NOUT; ++i)
    if ((uintptr_t)a.out[i] % 16) return false;
  return true;
}

svd2_status hip_status(hipError_t e) {
  if (e == hipSuccess) return SVD2_OK;
  g_last_hip = (int)e;
  return SVD2_ERR_HIP;
}

template <class T, bool CPLX, int RESCUE, bool UV, bool SINE>
svd2_status launch(size_t n, const KArgs<T, CPLX ? 8 : 4, CPLX ? 19 : 11> &a, int bs,
                   uint32_t *nresc, uint32_t *queue, uint32_t *qcount, hipStream_t st) {
  constexpr int kind = kind_of<T, CPLX>() + (UV ? 0 : 4);
  constexpr int NIN = CPLX ? 8 : 4, NOUT = CPLX ? 19 : 11;
  constexpr size_t chunk = kChunkBytes / sizeof(T);  // matrices per launch (even)
  int block = g_block[kind].load(), pt = g_per_thread[kind].load();
  if (pt == 2 && !all_aligned16(a, UV)) pt = 1;
  // launches of m matrices from matrix c0 on: two matrices per lane over an
  // even count, one per lane for the rest
  auto go = [&](size_t c0, size_t m, int p) {
    KArgs<T, NIN, NOUT> ac = a;
    for (int i = 0; i < NIN; ++i) ac.in[i] = a.in[i] + c0;
    for (int i = 0; i < NOUT; ++i) ac.out[i] = a.out[i] + c0;
    const size_t grid = (m / p + block - 1) / block;
    if (p == 2)
      hipLaunchKernelGGL((svd2_kernel<T, CPLX, 2, RESCUE, UV, SINE>), dim3((unsigned)grid), dim3(block), 0, st,
                         (uint32_t)m, ac, bs, nresc, queue, qcount, (uint32_t)c0);
    else
      hipLaunchKernelGGL((svd2_kernel<T, CPLX, 1, RESCUE, UV, SINE>), dim3((unsigned)grid), dim3(block), 0, st,
                         (uint32_t)m, ac, bs, nresc, queue, qcount, (uint32_t)c0);
    return hip_status(hipGetLastError());
  };
  for (size_t c0 = 0; c0 < n; c0 += chunk) {
    const size_t m = n - c0 < chunk ? n - c0 : chunk;
    const size_t m2 = pt == 2 ? m & ~size_t(1) : 0;
    svd2_status s = m2 ? go(c0, m2, 2) : SVD2_OK;
    if (s == SVD2_OK && m > m2) s = go(c0 + m2, m - m2, 1);
    if (s != SVD2_OK) return s;
  }
  return SVD2_OK;
}

// the phase-output form: one matrix per lane, launches of at most
// kChunkBytes per array as above
template <class T, bool CPLX, int RESCUE, bool UV, bool SINE, bool UPV>
svd2_status launch_urv(size_t n, const KArgs<T, CPLX ? 8 : 4, CPLX ? 19 : 11> &a,
                       const OutArgs<T, urv_count<CPLX>()> &f, int bs, uint32_t *nresc, uint32_t *queue,
                       uint32_t *qcount, hipStream_t st) {
  constexpr int kind = kind_of<T, CPLX>() + (UV ? 0 : 4);
  constexpr int NIN = CPLX ? 8 : 4, NOUT = CPLX ? 19 : 11, NF = urv_count<CPLX>();
  constexpr size_t chunk = kChunkBytes / sizeof(T);
  const int block = g_block[kind].load();
  for (size_t c0 = 0; c0 < n; c0 += chunk) {
    const size_t m = n - c0 < chunk ? n - c0 : chunk;
    KArgs<T, NIN, NOUT> ac = a;
    OutArgs<T, NF> fc = f;
    for (int i = 0; i < NIN; ++i) ac.in[i] = a.in[i] + c0;
    for (int i = 0; i < NOUT; ++i) ac.out[i] = a.out[i] ? a.out[i] + c0 : nullptr;
    for (int i = 0; i < NF; ++i) fc.out[i] = f.out[i] ? f.out[i] + c0 : nullptr;
    const size_t grid = (m + block - 1) / block;
    hipLaunchKernelGGL((svd2_urv_kernel<T, CPLX, RESCUE, UV, SINE, UPV>), dim3((unsigned)grid), dim3(block), 0, st,
                       (uint32_t)m, ac, fc, bs, nresc, queue, qcount, (uint32_t)c0);
    svd2_status s = hip_status(hipGetLastError());
    if (s != SVD2_OK) return s;
  }
  return SVD2_OK;
}

template <class T, bool CPLX, int RESCUE, bool UPV>
svd2_status launch_urv_uv(bool uv, bool sine, size_t n, const KArgs<T, CPLX ? 8 : 4, CPLX ? 19 : 11> &a,
                          const OutArgs<T, urv_count<CPLX>()> &f, int bs, uint32_t *nresc, uint32_t *queue,
                          uint32_t *qcount, hipStream_t st) {
  if (!uv) return launch_urv<T, CPLX, RESCUE, false, false, UPV>(n, a, f, bs, nresc, queue, qcount, st);
  return sine ? launch_urv<T, CPLX, RESCUE, true, true, UPV>(n, a, f, bs, nresc, queue, qcount, st)
              : launch_urv<T, CPLX, RESCUE, true, false, UPV>(n, a, f, bs, nresc, queue, qcount, st);
}

// uv: U and V are wanted (else SVD2_NO_UV); sine: assembled by eq. (31);
// f: the phase outputs (R, and U_+, V_+ with upv), or none
template <class T, bool CPLX, int RESCUE>
svd2_status launch_uv(bool uv, bool sine, size_t n, const KArgs<T, CPLX ? 8 : 4, CPLX ? 19 : 11> &a, int bs,
                      uint32_t *nresc, uint32_t *queue, uint32_t *qcount, hipStream_t st,
                      const OutArgs<T, urv_count<CPLX>()> *f = nullptr, bool upv = false) {
  if (f) {
    return upv ? launch_urv_uv<T, CPLX, RESCUE, true>(uv, sine, n, a, *f, bs, nresc, queue, qcount, st)
               : launch_urv_uv<T, CPLX, RESCUE, false>(uv, sine, n, a, *f, bs, nresc, queue, qcount, st);
  }
  if (!uv) return launch<T, CPLX, RESCUE, false, false>(n, a, bs, nresc, queue, qcount, st);
  return sine ? launch<T, CPLX, RESCUE, true, true>(n, a, bs, nresc, queue, qcount, st)
              : launch<T, CPLX, RESCUE, true, false>(n, a, bs, nresc, queue, qcount, st);
}

// the second pass of the queued FP32 rescue
template <class T, bool CPLX, int TAIL>
void launch_rescue(bool uv, bool sine, const KArgs<T, CPLX ? 8 : 4, CPLX ? 19 : 11> &a, int bs,
                   const uint32_t *q, const uint32_t *qcount, hipStream_t st) {
  const dim3 g(1024), b(256);
  if (!uv) hipLaunchKernelGGL((svd2_rescue_kernel<T, CPLX, TAIL, false, false>), g, b, 0, st, a, bs, q, qcount);
  else if (sine) hipLaunchKernelGGL((svd2_rescue_kernel<T, CPLX, TAIL, true, true>), g, b, 0, st, a, bs, q, qcount);
  else hipLaunchKernelGGL((svd2_rescue_kernel<T, CPLX, TAIL, true, false>), g, b, 0, st, a, bs, q, qcount);
}

bool bad_bs_flags(unsigned flags) { return (flags & 3u) == 3u; }

template <class T, bool CPLX>
svd2_status run_fp32(size_t n, const KArgs<T, CPLX ? 8 : 4, CPLX ? 19 : 11> &a, unsigned flags,
                     uint32_t *nresc, void *ws, size_t ws_bytes, hipStream_t st,
                     const OutArgs<T, urv_count<CPLX>()> *f = nullptr, bool upv = false) {
  int bs = (int)(flags & 3u);
  bool resc = flags & SVD2_RESCUE_FP64, queue = flags & SVD2_RESCUE_QUEUE,
       sigma = flags & SVD2_RESCUE_SIGMA, tri = flags & SVD2_RESCUE_TRI, uv = !(flags & SVD2_NO_UV),
       sine = flags & SVD2_SINE_FORM;
  if (!resc) return launch_uv<T, CPLX, 0>(uv, sine, n, a, bs, nullptr, nullptr, nullptr, st, f, upv);
  if (!queue) {
    if (sigma) return launch_uv<T, CPLX, 3>(uv, sine, n, a, bs, nresc, nullptr, nullptr, st, f, upv);
    if (tri) return launch_uv<T, CPLX, 4>(uv, sine, n, a, bs, nresc, nullptr, nullptr, st, f, upv);
    return launch_uv<T, CPLX, 1>(uv, sine, n, a, bs, nresc, nullptr, nullptr, st, f, upv);
  }
  if (n >= 0xffffffffull) return SVD2_ERR_SIZE;
  if (!ws) return SVD2_ERR_NULL;
  if (ws_bytes < svd2_workspace_bytes(n, flags)) return SVD2_ERR_SIZE;
  if ((uintptr_t)ws % 4) return SVD2_ERR_ALIGN;
  uint32_t *qcount = (uint32_t *)ws;
  uint32_t *q = qcount + 64;  // keep the queue 256-byte aligned
  hipLaunchKernelGGL(zero_u32_kernel, dim3(1), dim3(1), 0, st, qcount);
  svd2_status s0 = hip_status(hipGetLastError());
  if (s0 != SVD2_OK) return s0;
  svd2_status s1 = launch_uv<T, CPLX, 2>(uv, sine, n, a, bs, nresc, q, qcount, st, f, upv);
  if (s1 != SVD2_OK) return s1;
  if (sigma) launch_rescue<T, CPLX, 3>(uv, sine, a, bs, q, qcount, st);
  else if (tri) launch_rescue<T, CPLX, 4>(uv, sine, a, bs, q, qcount, st);
  else launch_rescue<T, CPLX, 1>(uv, sine, a, bs, q, qcount, st);
  return hip_status(hipGetLastError());
}

template <class T>
svd2_status probe(int op, size_t n, const T *x, const T *y, const T *z, T *out,
                         hipStream_t stream) {
  if (op < 0 || op > 8) return SVD2_ERR_FLAGS;
  if (!x || !out || (!y && op != 1 && op != 4 && op < 7) || (!z && op == 2)) return SVD2_ERR_NULL;
  if (n == 0) return SVD2_OK;
  size_t grid = (n + 255) / 256;
  if (grid > 0x7fffffffu) return SVD2_ERR_SIZE;
  hipLaunchKernelGGL((probe_kernel<T>), dim3((unsigned)grid), dim3(256), 0, stream, op, n, x, y, z,
                     out);
  return hip_status(hipGetLastError());
}


// ---------------------------------------------------------------------------
// memory-pattern probe: the batched kernels' loads and stores with no SVD
// arithmetic (each output = sum of the inputs + its index), same launch shape
// ---------------------------------------------------------------------------
template <class T, int NIN, int NOUT, int PT>
__global__ __launch_bounds__(256) void stream_probe_kernel(uint32_t n, KArgs<T, NIN, NOUT> a) {
  const uint32_t k = (blockIdx.x * blockDim.x + threadIdx.x) * PT;
  int cnt = (k < n) ? (int)((n - k < (uint32_t)PT) ? (n - k) : PT) : 0;
  if (cnt == 0) return;
  T x[PT][NIN], y[PT][NOUT];
  load_lanes<T, NIN, PT>(a.in, k, cnt, x);
#pragma unroll
  for (int j = 0; j < PT; ++j) {
    T acc = T(0);
#pragma unroll
    for (int i = 0; i < NIN; ++i) acc += x[j][i];
#pragma unroll
    for (int i = 0; i < NOUT; ++i) y[j][i] = acc + T(i);
  }
  store_lanes<T, NOUT, PT>(a.out, k, cnt, y);
}

template <class T, int NIN, int NOUT>
svd2_status stream_probe(size_t n, const void *const *in, void *const *out, hipStream_t st, int kind) {
  KArgs<T, NIN, NOUT> a;
  for (int i = 0; i < NIN; ++i) a.in[i] = (const T *)in[i];
  for (int i = 0; i < NOUT; ++i) a.out[i] = (T *)out[i];
  svd2_status s = check_ptrs<T>(n, a.in, NIN, a.out, NOUT);
  if (s != SVD2_OK || n == 0) return s;
  int block = g_block[kind].load(), pt = g_per_thread[kind].load();
  if (pt == 2 && !all_aligned16(a)) pt = 1;
  constexpr size_t chunk = kChunkBytes / sizeof(T);
  auto go = [&](size_t c0, size_t m, int p) {
    KArgs<T, NIN, NOUT> ac = a;
    for (int i = 0; i < NIN; ++i) ac.in[i] = a.in[i] + c0;
    for (int i = 0; i < NOUT; ++i) ac.out[i] = a.out[i] + c0;
    const size_t grid = (m / p + block - 1) / block;
    if (p == 2)
      hipLaunchKernelGGL((stream_probe_kernel<T, NIN, NOUT, 2>), dim3((unsigned)grid), dim3(block), 0, st,
                         (uint32_t)m, ac);
    else
      hipLaunchKernelGGL((stream_probe_kernel<T, NIN, NOUT, 1>), dim3((unsigned)grid), dim3(block), 0, st,
                         (uint32_t)m, ac);
    return hip_status(hipGetLastError());
  };
  for (size_t c0 = 0; c0 < n; c0 += chunk) {
    const size_t m = n - c0 < chunk ? n - c0 : chunk;
    const size_t m2 = pt == 2 ? m & ~size_t(1) : 0;
    svd2_status s = m2 ? go(c0, m2, 2) : SVD2_OK;
    if (s == SVD2_OK && m > m2) s = go(c0 + m2, m - m2, 1);
    if (s != SVD2_OK) return s;
  }
  return SVD2_OK;
}

// the phase-output struct of an entry point as an OutArgs: R required, U_+
// and V_+ all given (upv) or all NULL
template <class T, int NF> svd2_status urv_args(T *const (&p)[NF], OutArgs<T, NF> &f, bool &upv) {
  int given = 0;
  for (int i = 0; i < NF; ++i) {
    f.out[i] = p[i];
    if (i >= 3 && p[i]) ++given;
  }
  if (!p[0] || !p[1] || !p[2]) return SVD2_ERR_NULL;
  if (given != 0 && given != NF - 3) return SVD2_ERR_NULL;
  upv = given != 0;
  return SVD2_OK;
}

// outputs of one call for the alias and alignment checks: the used outputs of
// the args struct, then the used phase outputs
template <class T, int NOUT, int NF>
int gather_outputs(T *const (&out)[NOUT], bool uv, const OutArgs<T, NF> &f, bool upv, T *(&all)[NOUT + NF]) {
  int m = 0;
  for (int i = uv ? 0 : NOUT - 3; i < NOUT; ++i) all[m++] = out[i];
  for (int i = 0; i < (upv ? NF : 3); ++i) all[m++] = f.out[i];
  return m;
}

template <class T, bool CPLX, class FS>
svd2_status urv_prepare(size_t n, const KArgs<T, CPLX ? 8 : 4, CPLX ? 19 : 11> &a, const FS *fs, unsigned flags,
                        OutArgs<T, urv_count<CPLX>()> &f, bool &upv) {
  constexpr int NIN = CPLX ? 8 : 4, NOUT = CPLX ? 19 : 11, NF = urv_count<CPLX>();
  if (!fs) return SVD2_ERR_NULL;
  // R, U_+ and V_+ belong to 2^s A: s must be returned, so no backscale
  if (flags & 3u) return SVD2_ERR_FLAGS;
  T *p[NF];
  static_assert(sizeof(FS) == NF * sizeof(T *), "phase-output struct layout");
  memcpy(p, fs, sizeof p);
  svd2_status st = urv_args<T, NF>(p, f, upv);
  if (st != SVD2_OK) return st;
  T *all[NOUT + NF];
  const int m = gather_outputs<T, NOUT, NF>(a.out, !(flags & SVD2_NO_UV), f, upv, all);
  return check_ptrs<T>(n, a.in, NIN, all, m);
}

}  // namespace

extern "C" {

svd2_status dsvd2_batch_urv(size_t n, const dsvd2_args *p, const dsvd2_urv *fs, unsigned flags,
                            hipStream_t stream) {
  if (!p) return SVD2_ERR_NULL;
  if (flags & ~(3u | SVD2_NO_UV | SVD2_SINE_FORM) || bad_bs_flags(flags)) return SVD2_ERR_FLAGS;
  KArgs<double, 4, 11> a = {{p->a11, p->a21, p->a12, p->a22},
                            {p->u11, p->u21, p->u12, p->u22, p->v11, p->v21, p->v12, p->v22,
                             p->smax, p->smin, p->s}};
  OutArgs<double, 11> f;
  bool upv = false;
  svd2_status st = urv_prepare<double, false>(n, a, fs, flags, f, upv);
  if (st != SVD2_OK || n == 0) return st;
  return launch_uv<double, false, 0>(!(flags & SVD2_NO_UV), (flags & SVD2_SINE_FORM) != 0, n, a, 0, nullptr,
                                     nullptr, nullptr, stream, &f, upv);
}

svd2_status zsvd2_batch_urv(size_t n, const zsvd2_args *p, const zsvd2_urv *fs, unsigned flags,
                            hipStream_t stream) {
  if (!p) return SVD2_ERR_NULL;
  if (flags & ~(3u | SVD2_NO_UV | SVD2_SINE_FORM) || bad_bs_flags(flags)) return SVD2_ERR_FLAGS;
  KArgs<double, 8, 19> a = {{p->a11r, p->a11i, p->a21r, p->a21i, p->a12r, p->a12i, p->a22r, p->a22i},
                            {p->u11r, p->u11i, p->u21r, p->u21i, p->u12r, p->u12i, p->u22r, p->u22i,
                             p->v11r, p->v11i, p->v21r, p->v21i, p->v12r, p->v12i, p->v22r, p->v22i,
                             p->smax, p->smin, p->s}};
  OutArgs<double, 19> f;
  bool upv = false;
  svd2_status st = urv_prepare<double, true>(n, a, fs, flags, f, upv);
  if (st != SVD2_OK || n == 0) return st;
  return launch_uv<double, true, 0>(!(flags & SVD2_NO_UV), (flags & SVD2_SINE_FORM) != 0, n, a, 0, nullptr,
                                    nullptr, nullptr, stream, &f, upv);
}

svd2_status dsvd2_batch(size_t n, const dsvd2_args *p, unsigned flags, hipStream_t stream) {
  if (!p) return SVD2_ERR_NULL;
  if (flags & ~(3u | SVD2_NO_UV | SVD2_SINE_FORM) || bad_bs_flags(flags)) return SVD2_ERR_FLAGS;
  KArgs<double, 4, 11> a = {{p->a11, p->a21, p->a12, p->a22},
                            {p->u11, p->u21, p->u12, p->u22, p->v11, p->v21, p->v12, p->v22,
                             p->smax, p->smin, p->s}};
  const bool uv = !(flags & SVD2_NO_UV);
  svd2_status st = check_ptrs<double>(n, a.in, 4, a.out + (uv ? 0 : 8), uv ? 11 : 3);
  if (st != SVD2_OK || n == 0) return st;
  return launch_uv<double, false, 0>(uv, (flags & SVD2_SINE_FORM) != 0, n, a, (int)(flags & 3u), nullptr, nullptr,
                                     nullptr, stream);
}

svd2_status zsvd2_batch(size_t n, const zsvd2_args *p, unsigned flags, hipStream_t stream) {
  if (!p) return SVD2_ERR_NULL;
  if (flags & ~(3u | SVD2_NO_UV | SVD2_SINE_FORM) || bad_bs_flags(flags)) return SVD2_ERR_FLAGS;
  KArgs<double, 8, 19> a = {{p->a11r, p->a11i, p->a21r, p->a21i, p->a12r, p->a12i, p->a22r, p->a22i},
                            {p->u11r, p->u11i, p->u21r, p->u21i, p->u12r, p->u12i, p->u22r, p->u22i,
                             p->v11r, p->v11i, p->v21r, p->v21i, p->v12r, p->v12i, p->v22r, p->v22i,
                             p->smax, p->smin, p->s}};
  const bool uv = !(flags & SVD2_NO_UV);
  svd2_status st = check_ptrs<double>(n, a.in, 8, a.out + (uv ? 0 : 16), uv ? 19 : 3);
  if (st != SVD2_OK || n == 0) return st;
  return launch_uv<double, true, 0>(uv, (flags & SVD2_SINE_FORM) != 0, n, a, (int)(flags & 3u), nullptr, nullptr,
                                    nullptr, stream);
}

static bool bad_fp32_flags(unsigned flags) {
  if (flags & ~(31u | SVD2_NO_UV | SVD2_SINE_FORM | SVD2_RESCUE_TRI) || bad_bs_flags(flags)) return true;
  if ((flags & (SVD2_RESCUE_QUEUE | SVD2_RESCUE_SIGMA | SVD2_RESCUE_TRI)) && !(flags & SVD2_RESCUE_FP64))
    return true;
  if ((flags & SVD2_RESCUE_SIGMA) && (flags & SVD2_RESCUE_TRI)) return true;
  return false;
}

svd2_status ssvd2_batch(size_t n, const ssvd2_args *p, unsigned flags, void *ws, size_t ws_bytes,
                        hipStream_t stream) {
  if (!p) return SVD2_ERR_NULL;
  if (bad_fp32_flags(flags)) return SVD2_ERR_FLAGS;
  KArgs<float, 4, 11> a = {{p->a11, p->a21, p->a12, p->a22},
                           {p->u11, p->u21, p->u12, p->u22, p->v11, p->v21, p->v12, p->v22,
                            p->smax, p->smin, p->s}};
  const bool uv = !(flags & SVD2_NO_UV);
  svd2_status st = check_ptrs<float>(n, a.in, 4, a.out + (uv ? 0 : 8), uv ? 11 : 3);
  if (st != SVD2_OK || n == 0) return st;
  return run_fp32<float, false>(n, a, flags, p->nrescued, ws, ws_bytes, stream);
}

svd2_status csvd2_batch(size_t n, const csvd2_args *p, unsigned flags, void *ws, size_t ws_bytes,
                        hipStream_t stream) {
  if (!p) return SVD2_ERR_NULL;
  if (bad_fp32_flags(flags)) return SVD2_ERR_FLAGS;
  KArgs<float, 8, 19> a = {{p->a11r, p->a11i, p->a21r, p->a21i, p->a12r, p->a12i, p->a22r, p->a22i},
                           {p->u11r, p->u11i, p->u21r, p->u21i, p->u12r, p->u12i, p->u22r, p->u22i,
                            p->v11r, p->v11i, p->v21r, p->v21i, p->v12r, p->v12i, p->v22r, p->v22i,
                            p->smax, p->smin, p->s}};
  const bool uv = !(flags & SVD2_NO_UV);
  svd2_status st = check_ptrs<float>(n, a.in, 8, a.out + (uv ? 0 : 16), uv ? 19 : 3);
  if (st != SVD2_OK || n == 0) return st;
  return run_fp32<float, true>(n, a, flags, p->nrescued, ws, ws_bytes, stream);
}

svd2_status ssvd2_batch_urv(size_t n, const ssvd2_args *p, const ssvd2_urv *fs, unsigned flags, void *ws,
                            size_t ws_bytes, hipStream_t stream) {
  if (!p) return SVD2_ERR_NULL;
  if (bad_fp32_flags(flags)) return SVD2_ERR_FLAGS;
  KArgs<float, 4, 11> a = {{p->a11, p->a21, p->a12, p->a22},
                           {p->u11, p->u21, p->u12, p->u22, p->v11, p->v21, p->v12, p->v22,
                            p->smax, p->smin, p->s}};
  OutArgs<float, 11> f;
  bool upv = false;
  svd2_status st = urv_prepare<float, false>(n, a, fs, flags, f, upv);
  if (st != SVD2_OK || n == 0) return st;
  return run_fp32<float, false>(n, a, flags, p->nrescued, ws, ws_bytes, stream, &f, upv);
}

svd2_status csvd2_batch_urv(size_t n, const csvd2_args *p, const csvd2_urv *fs, unsigned flags, void *ws,
                            size_t ws_bytes, hipStream_t stream) {
  if (!p) return SVD2_ERR_NULL;
  if (bad_fp32_flags(flags)) return SVD2_ERR_FLAGS;
  KArgs<float, 8, 19> a = {{p->a11r, p->a11i, p->a21r, p->a21i, p->a12r, p->a12i, p->a22r, p->a22i},
                           {p->u11r, p->u11i, p->u21r, p->u21i, p->u12r, p->u12i, p->u22r, p->u22i,
                            p->v11r, p->v11i, p->v21r, p->v21i, p->v12r, p->v12i, p->v22r, p->v22i,
                            p->smax, p->smin, p->s}};
  OutArgs<float, 19> f;
  bool upv = false;
  svd2_status st = urv_prepare<float, true>(n, a, fs, flags, f, upv);
  if (st != SVD2_OK || n == 0) return st;
  return run_fp32<float, true>(n, a, flags, p->nrescued, ws, ws_bytes, stream, &f, upv);
}

size_t svd2_workspace_bytes(size_t n, unsigned flags) {
  if (!(flags & SVD2_RESCUE_QUEUE)) return 0;
  return 256 + n * sizeof(uint32_t);
}

svd2_status svd2_set_launch_kind(int kind, int block, int per_thread) {
  if (kind < 0 || kind > 7) return SVD2_ERR_FLAGS;
  if (block < 64 || block > 256 || block % 64) return SVD2_ERR_SIZE;
  if (per_thread != 1 && per_thread != 2) return SVD2_ERR_SIZE;
  g_block[kind].store(block);
  g_per_thread[kind].store(per_thread);
  return SVD2_OK;
}

svd2_status svd2_set_launch(int block, int per_thread) {
  if (block < 64 || block > 256 || block % 64) return SVD2_ERR_SIZE;
  if (per_thread != 1 && per_thread != 2) return SVD2_ERR_SIZE;
  for (int k = 0; k < 8; ++k) svd2_set_launch_kind(k, block, per_thread);
  return SVD2_OK;
}

void svd2_get_launch(int *block, int *per_thread) { svd2_get_launch_kind(0, block, per_thread); }

void svd2_get_launch_kind(int kind, int *block, int *per_thread) {
  if (kind < 0 || kind > 7) kind = 0;
  if (block) *block = g_block[kind].load();
  if (per_thread) *per_thread = g_per_thread[kind].load();
}

const char *svd2_status_string(svd2_status st) {
  switch (st) {
    case SVD2_OK: return "ok";
    case SVD2_ERR_NULL: return "null pointer";
    case SVD2_ERR_ALIGN: return "misaligned pointer";
    case SVD2_ERR_ALIAS: return "output overlaps an input or another output";
    case SVD2_ERR_FLAGS: return "invalid flags";
    case SVD2_ERR_HIP: return "HIP error";
    case SVD2_ERR_SIZE: return "size out of range";
    case SVD2_NOT_CONVERGED: return "not converged";
  }
  return "unknown status";
}

int svd2_last_hip_error(void) { return g_last_hip; }

svd2_status svd2_stream_probe(int kind, size_t n, const void *const *in, void *const *out,
                              hipStream_t stream) {
  if (!in || !out) return SVD2_ERR_NULL;
  switch (kind) {
    case 0: return stream_probe<double, 4, 11>(n, in, out, stream, 0);
    case 1: return stream_probe<double, 8, 19>(n, in, out, stream, 1);
    case 2: return stream_probe<float, 4, 11>(n, in, out, stream, 2);
    case 3: return stream_probe<float, 8, 19>(n, in, out, stream, 3);
    case 4: return stream_probe<double, 4, 3>(n, in, out, stream, 4);
    case 5: return stream_probe<double, 8, 3>(n, in, out, stream, 5);
    case 6: return stream_probe<float, 4, 3>(n, in, out, stream, 6);
    case 7: return stream_probe<float, 8, 3>(n, in, out, stream, 7);
  }
  return SVD2_ERR_FLAGS;
}

svd2_status svd2_probe_f64(int op, size_t n, const double *x, const double *y, const double *z,
                           double *out, hipStream_t stream) {
  return probe<double>(op, n, x, y, z, out, stream);
}
svd2_status svd2_probe_f32(int op, size_t n, const float *x, const float *y, const float *z,
                           float *out, hipStream_t stream) {
  return probe<float>(op, n, x, y, z, out, stream);
}

}  // extern "C"
