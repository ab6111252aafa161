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
// Drivers: an unfused chain per step (gather kernel -> batched SVD entry point
// -> update kernel, optionally replayed from a hipGraph per sweep), a fused
// persistent cooperative kernel that runs all steps of a sweep with two grid
// barriers per step, and two steps per pass over the matrix (kog_device.hpp).
// The uneven multi-problem batch is in kog_batch.hip.
#include <atomic>
#include <mutex>
#include <stdint.h>
#include <string.h>

#include "kog_device.hpp"

namespace kog {

thread_local int g_kog_hip = 0;
std::atomic<int> g_fused_per_cu{1};  // co-resident workgroups per CU used by the fused kernel

// tile-shape tables, set by kog_set_tile_rules / kog_set_two_step_tiles from
// any thread and read at every launch: guarded by one mutex
std::mutex g_rules_mu;
TileRule g_rules[kMaxRules] = {default_rule()};
int g_nrules = 1;

TileRule rule_for(int N) {
  std::lock_guard<std::mutex> lock(g_rules_mu);
  for (int i = 0; i < g_nrules; ++i)
    if (N <= g_rules[i].max_order) return g_rules[i];
  return default_rule();
}

// two-step kernel shapes: kc = wavefronts per workgroup, lc = column pairs per tile
TileRule default_rule2() { return TileRule{0x7fffffff, 4, 8}; }
TileRule g_rules2[kMaxRules] = {default_rule2()};
int g_nrules2 = 1;
TileRule rule2_for(int N) {
  std::lock_guard<std::mutex> lock(g_rules_mu);
  for (int i = 0; i < g_nrules2; ++i)
    if (N <= g_rules2[i].max_order) return g_rules2[i];
  return default_rule2();
}

// three-step kernel shapes: kc = wavefronts (row blocks) per workgroup, lc =
// output column pairs per tile
TileRule default_rule3() { return TileRule{0x7fffffff, 1, 0}; }
TileRule g_rules3[kMaxRules] = {default_rule3()};
int g_nrules3 = 1;
TileRule rule3_for(int N) {
  std::lock_guard<std::mutex> lock(g_rules_mu);
  for (int i = 0; i < g_nrules3; ++i)
    if (N <= g_rules3[i].max_order) return g_rules3[i];
  return default_rule3();
}

svd2_status hip_st(hipError_t e) {
  if (e == hipSuccess) return SVD2_OK;
  g_kog_hip = (int)e;
  return SVD2_ERR_HIP;
}

}  // namespace kog

namespace {

using namespace kog;

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

template <class T, bool CPLX>
__global__ __launch_bounds__(kUpdBlock) void kog_update_kernel(int N, Mat<T, CPLX> M, int t,
                                                               Bufs<T, CPLX> B, int kc, int lc) {
  update_tile<T, CPLX, false>(M, N, t, B, Tile{(int)blockIdx.x * kc, kc, (int)blockIdx.y * lc, lc});
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

template <class T, bool CPLX>
__global__ __launch_bounds__(256) void kog_pivots2_kernel(int N, Mat<T, CPLX> M, int t, Bufs<T, CPLX> B0,
                                                          Bufs<T, CPLX> B1) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < N / 2) pivots2_one<T, CPLX>(N, M, t, B0, B1, k);
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
__global__ __launch_bounds__(256) void kog_pivots3_kernel(int N, Mat<T, CPLX> M, int t, Bufs<T, CPLX> B0,
                                                          Bufs<T, CPLX> B1, Bufs<T, CPLX> B2) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  const int k = g >> 2;
  pivots3_quad<T, CPLX>(N, M, t, B0, B1, B2, k, g & 3, k < N / 2);
}

template <class T, bool CPLX>
__global__ __launch_bounds__(256) void kog_three_step_kernel(int N, Mat<T, CPLX> Mc, Mat<T, CPLX> Mn, int t,
                                                             Bufs<T, CPLX> B0, Bufs<T, CPLX> B1, Bufs<T, CPLX> B2,
                                                             int wpg, int lc, int gx, int ntiles) {
  extern __shared__ __align__(16) char kog_smem[];
  const int tile = xcd_tile((int)blockIdx.x, ntiles);
  three_step_tile<T, CPLX>(kog_smem, N, Mc.A, Mc.lda, Mn.A, Mn.lda, t, B0, B1, B2, wpg, lc, tile % gx, tile / gx);
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

// Diagnostic: nbar grid barriers and nothing else, with the fused kernel's
// barrier and workgroup size; its time per barrier is what each of the fused
// kernel's two barriers per step costs.  With `violations`, the barrier is
// also checked by its epochs: after barrier e every workgroup reads every
// workgroup's published epoch, which must already be >= e (a workgroup that
// had not arrived would show e - 1), and counts those that are not; an
// aborted wait counts once more.
__global__ __launch_bounds__(kUpdBlock) void kog_barrier_probe_kernel(Bar *bar, unsigned *flags, int nbar,
                                                                       unsigned *violations) {
  unsigned epoch = 0;
  for (int i = 0; i < nbar; ++i) {
    if (!grid_sync(bar, flags, gridDim.x, epoch)) {
      if (violations && threadIdx.x == 0) atomicAdd(violations, 1u);
      return;
    }
    if (violations) {
      unsigned late = 0;
      for (unsigned g = threadIdx.x; g < gridDim.x; g += blockDim.x)
        late += __hip_atomic_load(&flags[16 * g], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < epoch ? 1u : 0u;
      if (late) atomicAdd(violations, late);
    }
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

// largest binary exponent among the finite nonzero components (kNoExp if
// none): per-block maxima, then one block over them
template <class T, bool CPLX>
__global__ __launch_bounds__(256) void kog_maxexp_partial_kernel(int N, Mat<T, CPLX> M, int *part) {
  __shared__ int se[256];
  int e = kNoExp;
  for (int j = blockIdx.x; j < N; j += gridDim.x)
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
      const int x = elem_exp(M.ld(i, j));
      e = x > e ? x : e;
    }
  se[threadIdx.x] = e;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s && se[threadIdx.x + s] > se[threadIdx.x]) se[threadIdx.x] = se[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = se[0];
}

__global__ __launch_bounds__(256) void kog_maxexp_final_kernel(int nparts, const int *part, int *res) {
  __shared__ int se[256];
  int e = kNoExp;
  for (int i = threadIdx.x; i < nparts; i += blockDim.x) e = part[i] > e ? part[i] : e;
  se[threadIdx.x] = e;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s && se[threadIdx.x + s] > se[threadIdx.x]) se[threadIdx.x] = se[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) res[0] = se[0];
}

// ---------------------------------------------------------------------------
// SVD entry points: U = V = I at the start; at the end sigma in descending
// order (equal values by increasing index) and the columns of U and V
// permuted alike
// ---------------------------------------------------------------------------
template <class T, bool CPLX> __global__ __launch_bounds__(256) void kog_eye_kernel(int N, Mat<T, CPLX> X) {
  for (int j = blockIdx.x; j < N; j += gridDim.x)
    for (int i = threadIdx.x; i < N; i += blockDim.x) X.st(i, j, Cx<T>{i == j ? T(1) : T(0), T(0)});
}

// keys[i] = a_ii (real and >= 0 after a sweep), idx[i] = i; -1 pads to P
template <class T, bool CPLX>
__global__ __launch_bounds__(256) void kog_svd_keys_kernel(int N, int P, Mat<T, CPLX> A, T *keys, int *idx) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P) return;
  keys[i] = i < N ? A.ld(i, i).re : T(-1);
  idx[i] = i;
}

// one compare-exchange stage (block size k, distance j) of a bitonic sort of
// the pairs (key, index) into the order: key descending, then index ascending
template <class T>
__global__ __launch_bounds__(256) void kog_svd_bitonic_kernel(T *keys, int *idx, int P, int j, int k) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P) return;
  const int l = i ^ j;
  if (l <= i) return;
  const T a = keys[i], b = keys[l];
  const int ia = idx[i], ib = idx[l];
  const bool l_first = b > a || (b == a && ib < ia);
  if ((i & k) == 0 ? l_first : !l_first) {
    keys[i] = b;
    keys[l] = a;
    idx[i] = ib;
    idx[l] = ia;
  }
}

// dst[:, j] = src[:, idx[j]]
template <class T, bool CPLX>
__global__ __launch_bounds__(256) void kog_gather_cols_kernel(int N, Mat<T, CPLX> src, Mat<T, CPLX> dst,
                                                              const int *idx) {
  for (int j = blockIdx.x; j < N; j += gridDim.x) {
    const int c = idx[j];
    if ((unsigned)c >= (unsigned)N) continue;  // only a NaN diagonal (non-finite input) sorts padding here
    for (int i = threadIdx.x; i < N; i += blockDim.x) dst.st(i, j, src.ld(i, c));
  }
}

template <class T> __global__ __launch_bounds__(256) void kog_vec_copy_kernel(int N, const T *src, T *dst) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N) dst[i] = src[i];
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
template <class T, bool CPLX> struct Ctx {
  int N;
  Mat<T, CPLX> M;
  Bufs<T, CPLX> B, B1;
  Mat<T, CPLX> W;  // two-step mode: the second matrix buffer (lda = N)
  Layout L;
  char *ws;
  unsigned flags;
  hipStream_t st;
  // SVD entry points: the accumulated transformations, rotated in place in
  // (U, V) one step per pass, or alternating with (U2, V2) like the iterate
  // two steps per pass
  bool acc = false;
  Mat<T, CPLX> U{}, V{}, U2{}, V2{};
  Bufs<T, CPLX> B2{}, B3{};  // two steps per pass: the rotations of every second pass
  Bufs<T, CPLX> Bt{};        // three steps per pass: the rotations of the third step
  Bufs<T, CPLX> B4{};        // SVD entry points, three steps per pass: with B2, B3 the odd passes' rotations
  // SVD entry points, three steps per pass: two more triples of rotation
  // sets, and a second stream on which the walks of U and V run beside the
  // passes over the iterate (piv_ev: a pass's rotations are there; walk_ev:
  // a walk is done, for the walks of even and odd index)
  Bufs<T, CPLX> X[6]{};
  hipStream_t side = nullptr;
  hipEvent_t piv_ev = nullptr, walk_ev[2] = {nullptr, nullptr};
};

template <class T, bool CPLX>
svd2_status validate(int N, T *A, int lda, void *ws, size_t ws_bytes, unsigned flags, Ctx<T, CPLX> &c) {
  if (!A || !ws) return SVD2_ERR_NULL;
  if (N < 2 || N % 2 || lda < N || N > (1 << 19)) return SVD2_ERR_SIZE;
  if (flags & ~(unsigned)(SVD2_KOG_UNFUSED | SVD2_KOG_GRAPH | SVD2_KOG_TWO_STEP | SVD2_KOG_THREE_STEP))
    return SVD2_ERR_FLAGS;
  if ((flags & SVD2_KOG_GRAPH) && !(flags & SVD2_KOG_UNFUSED)) return SVD2_ERR_FLAGS;
  if ((flags & SVD2_KOG_TWO_STEP) && (flags & (SVD2_KOG_UNFUSED | SVD2_KOG_GRAPH))) return SVD2_ERR_FLAGS;
  if ((flags & SVD2_KOG_THREE_STEP) && (flags & (SVD2_KOG_UNFUSED | SVD2_KOG_GRAPH | SVD2_KOG_TWO_STEP)))
    return SVD2_ERR_FLAGS;
  if ((uintptr_t)A % (CPLX ? 2 * sizeof(T) : sizeof(T))) return SVD2_ERR_ALIGN;
  if ((uintptr_t)ws % 256) return SVD2_ERR_ALIGN;
  c.L = layout(N, sizeof(T), CPLX);
  const size_t need = (flags & SVD2_KOG_THREE_STEP) ? c.L.total3 : (flags & SVD2_KOG_TWO_STEP) ? c.L.total2
                                                                                              : c.L.total;
  if (ws_bytes < need) return SVD2_ERR_SIZE;
  size_t abytes = ((size_t)lda * (N - 1) + N) * sizeof(T) * (CPLX ? 2 : 1);
  uintptr_t a0 = (uintptr_t)A, a1 = a0 + abytes, w0 = (uintptr_t)ws, w1 = w0 + need;
  if (a0 < w1 && w0 < a1) return SVD2_ERR_ALIAS;
  c.N = N;
  c.M = Mat<T, CPLX>{A, (size_t)lda};
  c.B = make_bufs<T, CPLX>(ws, N, 0);
  c.B1 = make_bufs<T, CPLX>(ws, N, 1);
  if (flags & SVD2_KOG_THREE_STEP) c.Bt = make_bufs<T, CPLX>(ws, N, 2);
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

// U <- U U_k, V <- V V_k for the pairs of step t (rotations in c.B), in place
template <class T, bool CPLX>
svd2_status accum_step(const Ctx<T, CPLX> &c, const Mat<T, CPLX> &U, const Mat<T, CPLX> &V, int t) {
  const int n = c.N / 2, rows = c.N < 256 ? c.N : 256, ppb = 256 / rows;
  hipLaunchKernelGGL((kog_accum_kernel<T, CPLX>), dim3((n + ppb - 1) / ppb, 2), dim3(256), 0, c.st, c.N, U, V, t,
                     c.B);
  return hip_st(hipGetLastError());
}

// S steps t .. t+S-1 (rotations in sets[0 .. S-1]), from the buffer pair
// that holds U and V (in_w: the workspace pair) into the other one, on
// stream st (default: the context's)
template <class T, bool CPLX, int S>
svd2_status accum_s(const Ctx<T, CPLX> &c, bool in_w, int t, const Bufs<T, CPLX> *sets, hipStream_t st = nullptr) {
  constexpr int SEG = AccShape<T, CPLX>::seg;
  const int n = c.N / 2, rb = (c.N + 255) / 256, nseg = (n + SEG - 1) / SEG;
  const Mat<T, CPLX> &U = in_w ? c.U2 : c.U, &V = in_w ? c.V2 : c.V;
  const Mat<T, CPLX> &U2 = in_w ? c.U : c.U2, &V2 = in_w ? c.V : c.V2;
  AccSets<T, CPLX> R{};
  for (int L = 0; L < S; ++L) R.b[L] = sets[L];
  hipLaunchKernelGGL((kog_accum_s_kernel<T, CPLX, S>), dim3(rb * nseg, 2), dim3(256), 0, st ? st : c.st, c.N, U, V,
                     U2, V2, t, R);
  return hip_st(hipGetLastError());
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
  s = hip_st(hipGetLastError());
  if (s == SVD2_OK && c.acc) s = accum_step<T, CPLX>(c, c.U, c.V, t);
  return s;
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
  const int fpc = g_fused_per_cu.load();
  int want = fpc < per ? fpc : per;
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
svd2_status two_steps(const Ctx<T, CPLX> &c, const Mat<T, CPLX> &cur, const Mat<T, CPLX> &nxt, int t,
                      const Bufs<T, CPLX> &B0, const Bufs<T, CPLX> &B1) {
  const int n = c.N / 2;
  hipLaunchKernelGGL((kog_pivots2_kernel<T, CPLX>), dim3((n + 63) / 64), dim3(64), 0, c.st, c.N, cur, t, B0, B1);
  svd2_status s = hip_st(hipGetLastError());
  if (s != SVD2_OK) return s;
  const TwoStepShape sh = two_step_shape<T, CPLX>(c.N);
  if (sh.ntiles <= 0) return SVD2_ERR_HIP;
  hipLaunchKernelGGL((kog_two_step_kernel<T, CPLX>), dim3(sh.ntiles), dim3(64 * sh.wpg), sh.lds, c.st, c.N, cur,
                     nxt, t, B0, B1, sh.wpg, sh.span, sh.lc, sh.gx, sh.ntiles);
  return hip_st(hipGetLastError());
}

struct ThreeStepShape {
  int wpg, lc, gx, ntiles;
  size_t lds;
};
// the launch shape of the three-step kernel for order N: wpg row blocks per
// workgroup; lc output column pairs per tile as the rule fixes it, or (rule
// lc in [-3, 0]) sized so that the grid fills 1 - lc whole rounds of the
// workgroups the GPU holds at once (a partial last round costs a whole one)
template <class T, bool CPLX> ThreeStepShape three_step_shape(int N) {
  // per host thread: concurrent solves on other threads do not share it
  thread_local int cached_N = 0, cached_wpg = 0, cached_lc = 0;
  thread_local ThreeStepShape cached{};
  const TileRule r = rule3_for(N);
  if (N == cached_N && r.kc == cached_wpg && r.lc == cached_lc) return cached;
  const int n = N / 2;
  ThreeStepShape sh{};
  sh.wpg = r.kc;
  const int nb = (n + kShift3Out - 1) / kShift3Out;
  sh.gx = (nb + sh.wpg - 1) / sh.wpg;
  auto fix = [&](int lc) {
    const int hi = n < 128 ? n : 128;
    lc = lc > hi ? hi : lc;
    lc = lc < 2 ? 2 : lc;
    sh.lc = lc;
    sh.ntiles = sh.gx * ((n + lc - 1) / lc);
    sh.lds = three_step_lds<T, CPLX>(lc);
  };
  if (r.lc > 0) {
    fix(r.lc);
  } else {
    const int rounds = 1 - r.lc;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      return ThreeStepShape{};
    fix(128);  // the widest tile first, then refine with the occupancy it allows
    for (int it = 0; it < 3; ++it) {
      int per = 0;
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, (const void *)kog_three_step_kernel<T, CPLX>,
                                                       64 * sh.wpg, sh.lds) != hipSuccess || per < 1)
        return ThreeStepShape{};
      long tc = (long)per * cus * rounds / sh.gx;
      if (tc < 1) tc = 1;
      fix((int)((n + tc - 1) / tc));
    }
  }
  cached_N = N;
  cached_wpg = r.kc;
  cached_lc = r.lc;
  cached = sh;
  return sh;
}

// three steps t, t+1, t+2 from `cur` into `nxt` (rotations into B0, B1, B2)
// (after_pivots: recorded on the stream once the three rotation sets are
// written, before the pass over the matrix)
template <class T, bool CPLX>
svd2_status three_steps(const Ctx<T, CPLX> &c, const Mat<T, CPLX> &cur, const Mat<T, CPLX> &nxt, int t,
                        const Bufs<T, CPLX> &B0, const Bufs<T, CPLX> &B1, const Bufs<T, CPLX> &B2,
                        hipEvent_t after_pivots = nullptr) {
  const int n = c.N / 2;
  hipLaunchKernelGGL((kog_pivots2_kernel<T, CPLX>), dim3((n + 63) / 64), dim3(64), 0, c.st, c.N, cur, t, B0, B1);
  svd2_status s = hip_st(hipGetLastError());
  if (s != SVD2_OK) return s;
  hipLaunchKernelGGL((kog_pivots3_kernel<T, CPLX>), dim3((4 * n + 63) / 64), dim3(64), 0, c.st, c.N, cur, t, B0, B1,
                     B2);
  s = hip_st(hipGetLastError());
  if (s == SVD2_OK && after_pivots) s = hip_st(hipEventRecord(after_pivots, c.st));
  if (s != SVD2_OK) return s;
  const ThreeStepShape sh = three_step_shape<T, CPLX>(c.N);
  if (sh.ntiles <= 0) return SVD2_ERR_HIP;
  hipLaunchKernelGGL((kog_three_step_kernel<T, CPLX>), dim3(sh.ntiles), dim3(64 * sh.wpg), sh.lds, c.st, c.N, cur,
                     nxt, t, B0, B1, B2, sh.wpg, sh.lc, sh.gx, sh.ntiles);
  return hip_st(hipGetLastError());
}

// one step t in place on `cur` (gather + SVD in one kernel, then the update)
template <class T, bool CPLX>
svd2_status one_step_on(const Ctx<T, CPLX> &c, const Mat<T, CPLX> &cur, int t, bool in_w = false) {
  const int n = c.N / 2;
  hipLaunchKernelGGL((kog_pivot_kernel<T, CPLX>), dim3((n + 255) / 256), dim3(256), 0, c.st, c.N, cur, t, c.B);
  svd2_status s = hip_st(hipGetLastError());
  if (s != SVD2_OK) return s;
  TileRule r = rule_for(c.N);
  dim3 grid((n + r.kc - 1) / r.kc, (n + r.lc - 1) / r.lc);
  hipLaunchKernelGGL((kog_update_kernel<T, CPLX>), grid, dim3(kUpdBlock), 0, c.st, c.N, cur, t, c.B, r.kc, r.lc);
  s = hip_st(hipGetLastError());
  if (s == SVD2_OK && c.acc) s = accum_step<T, CPLX>(c, in_w ? c.U2 : c.U, in_w ? c.V2 : c.V, t);
  return s;
}

// a sweep of the two-step mode; *in_w tells (and is updated with) which
// buffer holds the iterate (false: the caller's A, true: the workspace copy),
// *uv_in the same for the accumulated U and V.  With accumulation the passes
// alternate between the rotation sets (B, B1) and (B2, B3), and after every
// second pass one kernel takes U and V four steps further; an odd last pass
// gets a two-step accumulation, and the sweep's last single step an in-place
// one.
template <class T, bool CPLX> svd2_status sweep_two_step(const Ctx<T, CPLX> &c, bool *in_w, bool *uv_in) {
  svd2_status s = SVD2_OK;
  int t = 0;
  for (int p = 0; t + 1 < c.N - 1 && s == SVD2_OK; t += 2, ++p) {
    const Mat<T, CPLX> &cur = *in_w ? c.W : c.M, &nxt = *in_w ? c.M : c.W;
    const bool odd = c.acc && (p & 1);
    s = two_steps<T, CPLX>(c, cur, nxt, t, odd ? c.B2 : c.B, odd ? c.B3 : c.B1);
    *in_w = !*in_w;
    if (s != SVD2_OK || !c.acc) continue;
    if (odd) {
      const Bufs<T, CPLX> sets[4] = {c.B, c.B1, c.B2, c.B3};
      s = accum_s<T, CPLX, 4>(c, *uv_in, t - 2, sets);
      *uv_in = !*uv_in;
    } else if (t + 3 >= c.N - 1) {
      const Bufs<T, CPLX> sets[2] = {c.B, c.B1};
      s = accum_s<T, CPLX, 2>(c, *uv_in, t, sets);
      *uv_in = !*uv_in;
    }
  }
  if (s == SVD2_OK && t < c.N - 1) s = one_step_on<T, CPLX>(c, *in_w ? c.W : c.M, t, *uv_in);
  return s;
}

// a sweep of the three-step mode: passes of three steps, then what is left
// of the N-1 steps as one two-step pass or one single step; *in_w and *uv_in
// as in sweep_two_step.  With accumulation, after every second pass one
// kernel takes U and V six steps further, an unpaired last pass gets a
// three-step accumulation, the two-step rest a two-step one and a last single
// step an in-place one.  The passes take their rotation sets from two
// triples in turn ((B, B1, Bt), (B2, B3, B4)), or with the second stream
// from four (then X[0..2], X[3..5]): each walk of U and V then runs on that
// stream once its second pass's rotations are written, beside the passes
// over the iterate, and pass q waits for the walk that read its triple (the
// walk of passes q-4 and q-3); the stream joins back before the rest of the
// sweep.
template <class T, bool CPLX> svd2_status sweep_three_step(const Ctx<T, CPLX> &c, bool *in_w, bool *uv_in) {
  svd2_status s = SVD2_OK;
  const bool side = c.acc && c.side;
  const int ntri = side ? 4 : 2;
  auto set = [&](int tri, int i) -> const Bufs<T, CPLX> & {
    static_assert(sizeof(c.X) / sizeof(c.X[0]) == 6, "two extra triples");
    if (tri == 0) return i == 0 ? c.B : i == 1 ? c.B1 : c.Bt;
    if (tri == 1) return i == 0 ? c.B2 : i == 1 ? c.B3 : c.B4;
    return c.X[3 * (tri - 2) + i];
  };
  int last_walk = -1;
  auto join = [&]() -> svd2_status {
    return side && last_walk >= 0 ? hip_st(hipStreamWaitEvent(c.st, c.walk_ev[last_walk & 1], 0)) : SVD2_OK;
  };
  int t = 0;
  for (int p = 0; c.N - 1 - t >= 3 && s == SVD2_OK; t += 3, ++p) {
    const bool odd = c.acc && (p & 1);
    const int tri = c.acc ? p % ntri : 0;
    if (side && p >= 4 && !(p & 1)) s = hip_st(hipStreamWaitEvent(c.st, c.walk_ev[(p / 2) & 1], 0));
    if (s != SVD2_OK) break;
    s = three_steps<T, CPLX>(c, *in_w ? c.W : c.M, *in_w ? c.M : c.W, t, set(tri, 0), set(tri, 1), set(tri, 2),
                             side && odd ? c.piv_ev : nullptr);
    *in_w = !*in_w;
    if (s != SVD2_OK || !c.acc) continue;
    if (odd) {
      const int pt = tri - 1;  // the previous pass's triple
      const Bufs<T, CPLX> sets[6] = {set(pt, 0), set(pt, 1), set(pt, 2), set(tri, 0), set(tri, 1), set(tri, 2)};
      if (side) {
        s = hip_st(hipStreamWaitEvent(c.side, c.piv_ev, 0));
        if (s == SVD2_OK) s = accum_s<T, CPLX, 6>(c, *uv_in, t - 3, sets, c.side);
        if (s == SVD2_OK) s = hip_st(hipEventRecord(c.walk_ev[(p / 2) & 1], c.side));
        last_walk = p / 2;
      } else {
        s = accum_s<T, CPLX, 6>(c, *uv_in, t - 3, sets);
      }
      *uv_in = !*uv_in;
    } else if (c.N - 1 - (t + 3) < 3) {
      const Bufs<T, CPLX> sets[3] = {set(tri, 0), set(tri, 1), set(tri, 2)};
      s = join();
      if (s == SVD2_OK) s = accum_s<T, CPLX, 3>(c, *uv_in, t, sets);
      *uv_in = !*uv_in;
    }
  }
  if (s == SVD2_OK) s = join();
  if (s == SVD2_OK && c.N - 1 - t == 2) {
    s = two_steps<T, CPLX>(c, *in_w ? c.W : c.M, *in_w ? c.M : c.W, t, c.B, c.B1);
    *in_w = !*in_w;
    if (s == SVD2_OK && c.acc) {
      const Bufs<T, CPLX> sets[2] = {c.B, c.B1};
      s = accum_s<T, CPLX, 2>(c, *uv_in, t, sets);
      *uv_in = !*uv_in;
    }
    t += 2;
  }
  if (s == SVD2_OK && t < c.N - 1) s = one_step_on<T, CPLX>(c, *in_w ? c.W : c.M, t, *uv_in);
  return s;
}

template <class T, bool CPLX> svd2_status copy_back(const Ctx<T, CPLX> &c) {
  int grid = c.N < 4096 ? c.N : 4096;
  hipLaunchKernelGGL((kog_copy_kernel<T, CPLX>), dim3(grid), dim3(256), 0, c.st, c.N, c.W, c.M);
  return hip_st(hipGetLastError());
}

template <class T, bool CPLX> svd2_status sweep(const Ctx<T, CPLX> &c) {
  if (c.flags & SVD2_KOG_THREE_STEP) {
    bool in_w = false, uv_in = false;
    svd2_status s = sweep_three_step<T, CPLX>(c, &in_w, &uv_in);
    if (s == SVD2_OK && in_w) s = copy_back<T, CPLX>(c);
    return s;
  }
  if (c.flags & SVD2_KOG_TWO_STEP) {
    bool in_w = false, uv_in = false;
    svd2_status s = sweep_two_step<T, CPLX>(c, &in_w, &uv_in);
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

// E of the whole-matrix scaling (0 for a matrix with no finite nonzero
// component); synchronises
template <class T, bool CPLX> svd2_status max_exponent(const Ctx<T, CPLX> &c, int &E) {
  int *part = (int *)(c.ws + c.L.red), *res = (int *)(c.ws + c.L.res);
  int nb = c.N < kRedBlocks ? c.N : kRedBlocks;
  hipLaunchKernelGGL((kog_maxexp_partial_kernel<T, CPLX>), dim3(nb), dim3(256), 0, c.st, c.N, c.M, part);
  svd2_status s = hip_st(hipGetLastError());
  if (s != SVD2_OK) return s;
  hipLaunchKernelGGL(kog_maxexp_final_kernel, dim3(1), dim3(256), 0, c.st, nb, (const int *)part, res);
  s = hip_st(hipGetLastError());
  int h = kNoExp;
  if (s == SVD2_OK) s = hip_st(hipMemcpyAsync(&h, res, sizeof h, hipMemcpyDeviceToHost, c.st));
  if (s == SVD2_OK) s = hip_st(hipStreamSynchronize(c.st));
  E = h == kNoExp ? 0 : h;
  return s;
}

template <class T, bool CPLX> svd2_status scale_by(const Ctx<T, CPLX> &c, int e) {
  int grid = c.N < 4096 ? c.N : 4096;
  hipLaunchKernelGGL((kog_scale_kernel<T, CPLX>), dim3(grid), dim3(256), 0, c.st, c.N, c.M, e);
  return hip_st(hipGetLastError());
}

template <class T, bool CPLX> svd2_status check_abort(const Ctx<T, CPLX> &c) {
  if (c.flags & (SVD2_KOG_UNFUSED | SVD2_KOG_TWO_STEP | SVD2_KOG_THREE_STEP)) return SVD2_OK;
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
  if (g) (void)hipGraphDestroy(g);
  (void)hipStreamDestroy(cap);
  return s;
}

// sweeps until off(A) < tol ||A_0||_F (and at least min_sweeps); *uv_in_w
// (optional) tells whether the accumulated U, V ended in (U2, V2)
template <class T, bool CPLX>
svd2_status solve(Ctx<T, CPLX> &c, double tol, int max_sweeps, int *sweeps, double *off_rel,
                  int min_sweeps = 0, bool *uv_in_w = nullptr) {
  if (max_sweeps < 0 || !(tol >= 0)) return SVD2_ERR_SIZE;
  hipGraphExec_t exec = nullptr;
  svd2_status s = SVD2_OK;
  if (c.flags & SVD2_KOG_GRAPH) s = graph_build<T, CPLX>(c, &exec);
  const bool two = c.flags & SVD2_KOG_TWO_STEP, three = c.flags & SVD2_KOG_THREE_STEP;
  bool in_w = false, uv_in = false;
  double off2 = 0, tot2 = 0, nrm0 = 0;
  int sw = 0, E = 0;
  if (s == SVD2_OK) s = max_exponent<T, CPLX>(c, E);
  if (s == SVD2_OK && E != 0) s = scale_by<T, CPLX>(c, -E);
  if (s == SVD2_OK) s = norms_async<T, CPLX>(c);
  if (s == SVD2_OK) s = read_norms<T, CPLX>(c, off2, tot2);
  nrm0 = __builtin_sqrt(tot2);
  svd2_status result = SVD2_NOT_CONVERGED;
  while (s == SVD2_OK) {
    double rel = nrm0 > 0 ? __builtin_sqrt(off2) / nrm0 : 0.0;
    if (off_rel) *off_rel = rel;
    if ((rel < tol || nrm0 == 0) && sw >= min_sweeps) {
      result = SVD2_OK;
      break;
    }
    if (sw == max_sweeps) break;
    if (exec) s = hip_st(hipGraphLaunch(exec, c.st));
    else if (three) s = sweep_three_step<T, CPLX>(c, &in_w, &uv_in);
    else if (two) s = sweep_two_step<T, CPLX>(c, &in_w, &uv_in);
    else s = sweep<T, CPLX>(c);
    if (s == SVD2_OK) s = norms_async<T, CPLX>(c, in_w);
    if (s == SVD2_OK) s = read_norms<T, CPLX>(c, off2, tot2);
    if (s == SVD2_OK) s = check_abort<T, CPLX>(c);
    ++sw;
  }
  if (uv_in_w) *uv_in_w = uv_in;
  if (s == SVD2_OK && in_w) s = copy_back<T, CPLX>(c);
  if (s == SVD2_OK && E != 0) s = scale_by<T, CPLX>(c, E);
  if (s == SVD2_OK) s = hip_st(hipStreamSynchronize(c.st));
  if (exec) (void)hipGraphExecDestroy(exec);
  if (sweeps) *sweeps = sw;
  return s != SVD2_OK ? s : result;
}

template <class T, bool CPLX>
svd2_status api_step(int N, T *A, int lda, int t, void *ws, size_t wsb, unsigned flags, hipStream_t st) {
  Ctx<T, CPLX> c;
  if (flags & SVD2_KOG_GRAPH) return SVD2_ERR_FLAGS;  // graph replay is a solve-only mode
  svd2_status s = validate<T, CPLX>(N, A, lda, ws, wsb, flags, c);
  if (s != SVD2_OK) return s;
  c.st = st;
  if (c.flags & SVD2_KOG_THREE_STEP) {
    // steps t, t+1 and t+2 in one pass into the workspace matrix, then copied back
    if (t < 0 || t + 2 >= N - 1) return SVD2_ERR_SIZE;
    s = three_steps<T, CPLX>(c, c.M, c.W, t, c.B, c.B1, c.Bt);
    return s != SVD2_OK ? s : copy_back<T, CPLX>(c);
  }
  if (c.flags & SVD2_KOG_TWO_STEP) {
    // steps t and t+1 in one pass into the workspace matrix, then copied back
    if (t < 0 || t + 1 >= N - 1) return SVD2_ERR_SIZE;
    s = two_steps<T, CPLX>(c, c.M, c.W, t, c.B, c.B1);
    return s != SVD2_OK ? s : copy_back<T, CPLX>(c);
  }
  if (t < 0 || t >= N - 1) return SVD2_ERR_SIZE;
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


// workspace of the SVD entry points: the solve's, then the second U and V
// buffers (N x N, lda N), the sort keys and indices (next power of two) and,
// two steps per pass, two more rotation sets
struct SvdLayout {
  size_t u2, v2, keys, idx, b2, b3, b4, x, total;
  int P;
};
// passes: 1 (one step per pass), 2 or 3 steps per pass
inline SvdLayout svd_layout(int N, size_t esz, bool cplx, int passes) {
  auto up = [](size_t x) { return (x + 255) & ~size_t(255); };
  const Layout L = layout(N, esz, cplx);
  const size_t mat = up((size_t)N * N * esz * (cplx ? 2 : 1));
  const size_t set = (cplx ? 27 : 15) * up((size_t)(N / 2) * esz);
  SvdLayout S;
  S.P = 1;
  while (S.P < N) S.P <<= 1;
  S.u2 = passes == 3 ? L.total3 : passes == 2 ? L.total2 : L.total;
  S.v2 = S.u2 + mat;
  S.keys = S.v2 + mat;
  S.idx = S.keys + up((size_t)S.P * esz);
  S.b2 = S.idx + up((size_t)S.P * sizeof(int));
  S.b3 = S.b2 + (passes > 1 ? set : 0);
  S.b4 = S.b3 + (passes > 1 ? set : 0);
  S.x = S.b4 + (passes == 3 ? set : 0);  // three steps per pass: six more sets
  S.total = S.x + (passes == 3 ? 6 * set : 0);
  return S;
}
inline int svd_passes(unsigned flags) {
  return (flags & SVD2_KOG_THREE_STEP) ? 3 : (flags & SVD2_KOG_TWO_STEP) ? 2 : 1;
}

// a rotation set (pivot and SVD arrays, as make_bufs lays them out) at base
template <class T, bool CPLX> Bufs<T, CPLX> bufs_at(char *base, int N) {
  const size_t arr = ((size_t)(N / 2) * sizeof(T) + 255) & ~size_t(255);
  Bufs<T, CPLX> b;
  for (int i = 0; i < Bufs<T, CPLX>::NIN; ++i) b.piv[i] = (T *)(base + i * arr);
  for (int i = 0; i < Bufs<T, CPLX>::NOUT; ++i) b.out[i] = (T *)(base + (Bufs<T, CPLX>::NIN + i) * arr);
  return b;
}

// the flags of the SVD entry points: 0 = two steps per pass
inline unsigned svd_flags(unsigned flags) { return flags == 0 ? (unsigned)SVD2_KOG_TWO_STEP : flags; }

template <class T, bool CPLX>
svd2_status api_svd(int N, T *A, int lda, T *U, int ldu, T *V, int ldv, T *sigma, double tol, int max_sweeps,
                    int *sweeps, double *off_rel, void *ws, size_t wsb, unsigned flags, hipStream_t st) {
  flags = svd_flags(flags);
  if (flags != SVD2_KOG_TWO_STEP && flags != SVD2_KOG_THREE_STEP && flags != SVD2_KOG_UNFUSED &&
      flags != (SVD2_KOG_UNFUSED | SVD2_KOG_GRAPH))
    return SVD2_ERR_FLAGS;
  Ctx<T, CPLX> c;
  svd2_status s = validate<T, CPLX>(N, A, lda, ws, wsb, flags, c);
  if (s != SVD2_OK) return s;
  if (!U || !V || !sigma) return SVD2_ERR_NULL;
  if (ldu < N || ldv < N || max_sweeps < 1) return SVD2_ERR_SIZE;
  const size_t esz = sizeof(T) * (CPLX ? 2 : 1);
  if ((uintptr_t)U % esz || (uintptr_t)V % esz || (uintptr_t)sigma % sizeof(T)) return SVD2_ERR_ALIGN;
  const SvdLayout S = svd_layout(N, sizeof(T), CPLX, svd_passes(flags));
  if (wsb < S.total) return SVD2_ERR_SIZE;
  const uintptr_t r[5][2] = {{(uintptr_t)A, (uintptr_t)A + ((size_t)lda * (N - 1) + N) * esz},
                             {(uintptr_t)U, (uintptr_t)U + ((size_t)ldu * (N - 1) + N) * esz},
                             {(uintptr_t)V, (uintptr_t)V + ((size_t)ldv * (N - 1) + N) * esz},
                             {(uintptr_t)sigma, (uintptr_t)sigma + (size_t)N * sizeof(T)},
                             {(uintptr_t)ws, (uintptr_t)ws + S.total}};
  for (int a = 0; a < 5; ++a)
    for (int b = a + 1; b < 5; ++b)
      if (r[a][0] < r[b][1] && r[b][0] < r[a][1]) return SVD2_ERR_ALIAS;
  c.st = st;
  c.acc = true;
  c.U = Mat<T, CPLX>{U, (size_t)ldu};
  c.V = Mat<T, CPLX>{V, (size_t)ldv};
  c.U2 = Mat<T, CPLX>{(T *)(c.ws + S.u2), (size_t)N};
  c.V2 = Mat<T, CPLX>{(T *)(c.ws + S.v2), (size_t)N};
  c.B2 = bufs_at<T, CPLX>(c.ws + S.b2, N);
  c.B3 = bufs_at<T, CPLX>(c.ws + S.b3, N);
  c.B4 = bufs_at<T, CPLX>(c.ws + S.b4, N);
  // three steps per pass: the walks of U and V on a second stream
  struct Side {  // released on every return below
    Ctx<T, CPLX> &c;
    ~Side() {
      if (c.piv_ev) (void)hipEventDestroy(c.piv_ev);
      for (hipEvent_t e : c.walk_ev)
        if (e) (void)hipEventDestroy(e);
      if (c.side) (void)hipStreamDestroy(c.side);
    }
  } side_guard{c};
  if (flags == SVD2_KOG_THREE_STEP) {
    for (int i = 0; i < 6; ++i) c.X[i] = bufs_at<T, CPLX>(c.ws + S.x + i * (S.b3 - S.b2), N);
    s = hip_st(hipStreamCreateWithFlags(&c.side, hipStreamNonBlocking));
    if (s == SVD2_OK) s = hip_st(hipEventCreateWithFlags(&c.piv_ev, hipEventDisableTiming));
    for (int i = 0; i < 2 && s == SVD2_OK; ++i) s = hip_st(hipEventCreateWithFlags(&c.walk_ev[i], hipEventDisableTiming));
    if (s != SVD2_OK) return s;
  }
  const int grid = N < 4096 ? N : 4096;
  hipLaunchKernelGGL((kog_eye_kernel<T, CPLX>), dim3(grid), dim3(256), 0, st, N, c.U);
  hipLaunchKernelGGL((kog_eye_kernel<T, CPLX>), dim3(grid), dim3(256), 0, st, N, c.V);
  s = hip_st(hipGetLastError());
  if (s != SVD2_OK) return s;
  bool uv_in_w = false;
  const svd2_status res = solve<T, CPLX>(c, tol, max_sweeps, sweeps, off_rel, 1, &uv_in_w);
  if (res != SVD2_OK && res != SVD2_NOT_CONVERGED) return res;
  // sort the diagonal with its indices
  T *keys = (T *)(c.ws + S.keys);
  int *idx = (int *)(c.ws + S.idx);
  const dim3 pg((S.P + 255) / 256), blk(256);
  hipLaunchKernelGGL((kog_svd_keys_kernel<T, CPLX>), pg, blk, 0, st, N, S.P, c.M, keys, idx);
  s = hip_st(hipGetLastError());
  for (int k = 2; k <= S.P && s == SVD2_OK; k <<= 1)
    for (int j = k >> 1; j > 0 && s == SVD2_OK; j >>= 1) {
      hipLaunchKernelGGL(kog_svd_bitonic_kernel<T>, pg, blk, 0, st, keys, idx, S.P, j, k);
      s = hip_st(hipGetLastError());
    }
  // permuted columns into the caller's U and V (through the second buffers)
  for (int m = 0; m < 2 && s == SVD2_OK; ++m) {
    const Mat<T, CPLX> &X = m ? c.V : c.U, &X2 = m ? c.V2 : c.U2;
    if (!uv_in_w) {
      hipLaunchKernelGGL((kog_copy_kernel<T, CPLX>), dim3(grid), blk, 0, st, N, X, X2);
      s = hip_st(hipGetLastError());
    }
    if (s == SVD2_OK) {
      hipLaunchKernelGGL((kog_gather_cols_kernel<T, CPLX>), dim3(grid), blk, 0, st, N, X2, X, (const int *)idx);
      s = hip_st(hipGetLastError());
    }
  }
  if (s == SVD2_OK) {
    hipLaunchKernelGGL(kog_vec_copy_kernel<T>, dim3((N + 255) / 256), blk, 0, st, N, (const T *)keys, sigma);
    s = hip_st(hipGetLastError());
  }
  if (s == SVD2_OK) s = hip_st(hipStreamSynchronize(st));
  return s != SVD2_OK ? s : res;
}

}  // namespace

// Workspace of dkog_solve_noalloc: one copy of this array per GPU, allocated
// with the code object when it is loaded on that GPU and held until the
// process ends.  Host code never uses its name as an address: the device
// address comes from hipGetSymbolAddress, once per device (noalloc_scratch).
constexpr size_t kNoAllocScratchBytes = size_t(2) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxScratchDevices = 256;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxScratchDevices] = {};

// the device address of `scratch` on the current device, looked up on the
// first call on each device
svd2_status noalloc_scratch(void **out) {
  int dev = 0;
  svd2_status s = hip_st(hipGetDevice(&dev));
  if (s != SVD2_OK) return s;
  if (dev < 0 || dev >= kMaxScratchDevices) return SVD2_ERR_SIZE;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    s = hip_st(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (s != SVD2_OK) return s;
    if (!p || (uintptr_t)p % 256) return SVD2_ERR_HIP;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return SVD2_OK;
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
  return (flags & SVD2_KOG_THREE_STEP) ? L.total3 : (flags & SVD2_KOG_TWO_STEP) ? L.total2 : L.total;
}

size_t kog_workspace_bytes(int N, int dtype) { return kog_workspace_bytes_flags(N, dtype, 0); }

size_t kog_svd_workspace_bytes(int N, int dtype, unsigned flags) {
  if (N < 2 || N % 2 || N > (1 << 19)) return 0;
  const unsigned f = svd_flags(flags);
  if (f != SVD2_KOG_TWO_STEP && f != SVD2_KOG_THREE_STEP && f != SVD2_KOG_UNFUSED &&
      f != (SVD2_KOG_UNFUSED | SVD2_KOG_GRAPH))
    return 0;
  const int passes = svd_passes(f);
  switch (dtype) {
    case SVD2_KOG_F64: return svd_layout(N, 8, false, passes).total;
    case SVD2_KOG_C128: return svd_layout(N, 8, true, passes).total;
    case SVD2_KOG_F32: return svd_layout(N, 4, false, passes).total;
    case SVD2_KOG_C64: return svd_layout(N, 4, true, passes).total;
  }
  return 0;
}

svd2_status dkog_svd(int N, double *A, int lda, double *U, int ldu, double *V, int ldv, double *sigma, double tol,
                     int max_sweeps, int *sweeps, double *off_rel, void *ws, size_t ws_bytes, unsigned flags,
                     hipStream_t stream) {
  return api_svd<double, false>(N, A, lda, U, ldu, V, ldv, sigma, tol, max_sweeps, sweeps, off_rel, ws, ws_bytes,
                                flags, stream);
}
svd2_status zkog_svd(int N, double *A, int lda, double *U, int ldu, double *V, int ldv, double *sigma, double tol,
                     int max_sweeps, int *sweeps, double *off_rel, void *ws, size_t ws_bytes, unsigned flags,
                     hipStream_t stream) {
  return api_svd<double, true>(N, A, lda, U, ldu, V, ldv, sigma, tol, max_sweeps, sweeps, off_rel, ws, ws_bytes,
                               flags, stream);
}
svd2_status skog_svd(int N, float *A, int lda, float *U, int ldu, float *V, int ldv, float *sigma, double tol,
                     int max_sweeps, int *sweeps, double *off_rel, void *ws, size_t ws_bytes, unsigned flags,
                     hipStream_t stream) {
  return api_svd<float, false>(N, A, lda, U, ldu, V, ldv, sigma, tol, max_sweeps, sweeps, off_rel, ws, ws_bytes,
                               flags, stream);
}
svd2_status ckog_svd(int N, float *A, int lda, float *U, int ldu, float *V, int ldv, float *sigma, double tol,
                     int max_sweeps, int *sweeps, double *off_rel, void *ws, size_t ws_bytes, unsigned flags,
                     hipStream_t stream) {
  return api_svd<float, true>(N, A, lda, U, ldu, V, ldv, sigma, tol, max_sweeps, sweeps, off_rel, ws, ws_bytes,
                              flags, stream);
}

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

svd2_status dkog_solve_noalloc(int N, double *A, int lda, double tol, int max_sweeps, int *sweeps,
                               double *off_rel, unsigned flags, hipStream_t stream) {
  // argument checks first, so that a rejected call makes no HIP call at all
  if (!A) return SVD2_ERR_NULL;
  if (flags & ~(unsigned)SVD2_KOG_UNFUSED) return SVD2_ERR_FLAGS;
  if (N < 2 || N % 2 || lda < N) return SVD2_ERR_SIZE;
  if (kog_workspace_bytes(N, SVD2_KOG_F64) > kNoAllocScratchBytes) return SVD2_ERR_SIZE;
  void *ws = nullptr;
  svd2_status s = noalloc_scratch(&ws);
  if (s != SVD2_OK) return s;
  return api_solve<double, false>(N, A, lda, tol, max_sweeps, sweeps, off_rel, ws, kNoAllocScratchBytes, flags,
                                  stream);
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

svd2_status kog_set_tile_rules(int count, const int *max_order, const int *kc, const int *lc) {
  if (count < 0 || count > kMaxRules) return SVD2_ERR_SIZE;
  if (count > 0 && (!max_order || !kc || !lc)) return SVD2_ERR_NULL;
  for (int i = 0; i < count; ++i) {
    if (kc[i] != 64 && kc[i] != 128 && kc[i] != 256) return SVD2_ERR_SIZE;
    if (lc[i] < 1 || lc[i] > 4096 || max_order[i] < 2) return SVD2_ERR_SIZE;
    if (i > 0 && max_order[i] <= max_order[i - 1]) return SVD2_ERR_SIZE;
  }
  std::lock_guard<std::mutex> lock(g_rules_mu);
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
  std::lock_guard<std::mutex> lock(g_rules_mu);
  for (int i = 0; i < count; ++i) g_rules2[i] = TileRule{max_order[i], wpg[i], lc[i]};
  g_nrules2 = count;
  if (count == 0) {
    g_rules2[0] = default_rule2();
    g_nrules2 = 1;
  }
  return SVD2_OK;
}

svd2_status kog_set_three_step_tiles(int count, const int *max_order, const int *wpg, const int *lc) {
  if (count < 0 || count > kMaxRules) return SVD2_ERR_SIZE;
  if (count > 0 && (!max_order || !wpg || !lc)) return SVD2_ERR_NULL;
  for (int i = 0; i < count; ++i) {
    if (wpg[i] != 1 && wpg[i] != 2 && wpg[i] != 4) return SVD2_ERR_SIZE;
    if (lc[i] < -3 || lc[i] == 1 || lc[i] > 128 || max_order[i] < 2) return SVD2_ERR_SIZE;
    if (i > 0 && max_order[i] <= max_order[i - 1]) return SVD2_ERR_SIZE;
  }
  std::lock_guard<std::mutex> lock(g_rules_mu);
  for (int i = 0; i < count; ++i) g_rules3[i] = TileRule{max_order[i], wpg[i], lc[i]};
  g_nrules3 = count;
  if (count == 0) {
    g_rules3[0] = default_rule3();
    g_nrules3 = 1;
  }
  return SVD2_OK;
}

svd2_status kog_barrier_probe(int nbar, int blocks, unsigned *violations, void *ws, size_t ws_bytes,
                              hipStream_t stream) {
  if (!ws) return SVD2_ERR_NULL;
  if (nbar < 0 || blocks < 1 || blocks > kMaxFusedBlocks) return SVD2_ERR_SIZE;
  if (ws_bytes < 256 + (size_t)kMaxFusedBlocks * 64) return SVD2_ERR_SIZE;
  if ((uintptr_t)ws % 256) return SVD2_ERR_ALIGN;
  int dev = 0, cus = 0, per = 0;
  svd2_status s = hip_st(hipGetDevice(&dev));
  if (s == SVD2_OK) s = hip_st(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  if (s == SVD2_OK)
    s = hip_st(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, (const void *)kog_barrier_probe_kernel, kUpdBlock,
                                                            0));
  if (s != SVD2_OK) return s;
  if ((long)blocks > (long)per * cus) return SVD2_ERR_SIZE;  // not all co-resident
  Bar *bar = (Bar *)ws;
  unsigned *flags = (unsigned *)((char *)ws + 256);
  hipLaunchKernelGGL(kog_bar_reset_kernel, dim3((blocks + 255) / 256), dim3(256), 0, stream, bar, flags, blocks);
  s = hip_st(hipGetLastError());
  if (s != SVD2_OK) return s;
  void *args[] = {&bar, &flags, &nbar, &violations};
  return hip_st(hipLaunchCooperativeKernel((const void *)kog_barrier_probe_kernel, dim3(blocks), dim3(kUpdBlock), args,
                                           0, stream));
}

svd2_status kog_set_fused_blocks_per_cu(int per_cu) {
  if (per_cu < 1 || per_cu > 16) return SVD2_ERR_SIZE;
  g_fused_per_cu.store(per_cu);
  return SVD2_OK;
}

}  // extern "C"
