// Singular values of a Kogbetliantz iterate: the magnitudes of its diagonal,
// sorted into descending order on the device by a bitonic network over the
// next power of two (padding with -1, which sorts last), in the caller's
// workspace.  After the first step every diagonal entry lies in a pivot block
// that was set to diag(sigma_max, sigma_min), so the diagonal is real and
// non-negative and the magnitudes are exact copies of it.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "svd2.h"
#include "svd2_lane.hpp"

void kog_note_hip_error(int e);  // kog.hip: reported by kog_last_hip_error

namespace {

using svd2::hyp;
using svd2::vabs;

// keys[i] = |a_ii| for i < N, -1 for N <= i < P
template <class T, bool CPLX>
__global__ __launch_bounds__(256) void kog_diag_kernel(int N, int P, const T *A, size_t lda, T *keys) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P) return;
  if (i >= N) {
    keys[i] = T(-1);
    return;
  }
  const size_t o = (size_t)i + (size_t)i * lda;
  if constexpr (CPLX) {
    const T re = A[2 * o], im = A[2 * o + 1];
    keys[i] = im == T(0) ? vabs(re) : hyp(re, im);
  } else {
    keys[i] = vabs(A[o]);
  }
}

// one compare-exchange stage (block size k, distance j) of a descending
// bitonic sort of P = 2^m keys
template <class T> __global__ __launch_bounds__(256) void bitonic_kernel(T *keys, int P, int j, int k) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P) return;
  const int l = i ^ j;
  if (l <= i) return;
  const T a = keys[i], b = keys[l];
  const bool desc = (i & k) == 0;
  if (desc ? a < b : a > b) {
    keys[i] = b;
    keys[l] = a;
  }
}

template <class T> __global__ __launch_bounds__(256) void copy_kernel(int N, const T *src, T *dst) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N) dst[i] = src[i];
}

svd2_status hip_status(hipError_t e) {
  if (e == hipSuccess) return SVD2_OK;
  kog_note_hip_error((int)e);
  return SVD2_ERR_HIP;
}

constexpr size_t kAlign = 256;
size_t up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }
int pow2_at_least(int N) {
  int P = 1;
  while (P < N) P <<= 1;
  return P;
}

template <class T> size_t sigma_ws(int N) {
  if (N < 1 || N > (1 << 20)) return 0;
  return up((size_t)pow2_at_least(N) * sizeof(T));
}

template <class T, bool CPLX>
svd2_status sigma(int N, const T *A, int lda, T *out, void *ws, size_t wsb, hipStream_t st) {
  if (!A || !out || !ws) return SVD2_ERR_NULL;
  if (N < 1 || N > (1 << 20) || lda < N) return SVD2_ERR_SIZE;
  if ((uintptr_t)A % (CPLX ? 2 * sizeof(T) : sizeof(T)) || (uintptr_t)out % sizeof(T) ||
      (uintptr_t)ws % kAlign)
    return SVD2_ERR_ALIGN;
  const size_t need = sigma_ws<T>(N);
  if (wsb < need) return SVD2_ERR_SIZE;
  const size_t ebytes = sizeof(T) * (CPLX ? 2 : 1);
  const uintptr_t a0 = (uintptr_t)A, a1 = a0 + ((size_t)lda * (N - 1) + N) * ebytes;
  const uintptr_t o0 = (uintptr_t)out, o1 = o0 + (size_t)N * sizeof(T);
  const uintptr_t w0 = (uintptr_t)ws, w1 = w0 + need;
  if ((o0 < a1 && a0 < o1) || (w0 < a1 && a0 < w1) || (w0 < o1 && o0 < w1)) return SVD2_ERR_ALIAS;
  T *keys = (T *)ws;
  const int P = pow2_at_least(N);
  const dim3 grid((P + 255) / 256), block(256);
  hipLaunchKernelGGL((kog_diag_kernel<T, CPLX>), grid, block, 0, st, N, P, A, (size_t)lda, keys);
  svd2_status s = hip_status(hipGetLastError());
  for (int k = 2; k <= P && s == SVD2_OK; k <<= 1)
    for (int j = k >> 1; j > 0 && s == SVD2_OK; j >>= 1) {
      hipLaunchKernelGGL(bitonic_kernel<T>, grid, block, 0, st, keys, P, j, k);
      s = hip_status(hipGetLastError());
    }
  if (s != SVD2_OK) return s;
  hipLaunchKernelGGL(copy_kernel<T>, dim3((N + 255) / 256), block, 0, st, N, (const T *)keys, out);
  return hip_status(hipGetLastError());
}

}  // namespace

extern "C" {

size_t kog_sigma_workspace_bytes(int N, int dtype) {
  switch (dtype) {
    case SVD2_KOG_F64:
    case SVD2_KOG_C128: return sigma_ws<double>(N);
    case SVD2_KOG_F32:
    case SVD2_KOG_C64: return sigma_ws<float>(N);
  }
  return 0;
}

svd2_status dkog_sigma(int N, const double *A, int lda, double *sigma_out, void *ws, size_t ws_bytes,
                       hipStream_t stream) {
  return sigma<double, false>(N, A, lda, sigma_out, ws, ws_bytes, stream);
}
svd2_status zkog_sigma(int N, const double *A, int lda, double *sigma_out, void *ws, size_t ws_bytes,
                       hipStream_t stream) {
  return sigma<double, true>(N, A, lda, sigma_out, ws, ws_bytes, stream);
}
svd2_status skog_sigma(int N, const float *A, int lda, float *sigma_out, void *ws, size_t ws_bytes,
                       hipStream_t stream) {
  return sigma<float, false>(N, A, lda, sigma_out, ws, ws_bytes, stream);
}
svd2_status ckog_sigma(int N, const float *A, int lda, float *sigma_out, void *ws, size_t ws_bytes,
                       hipStream_t stream) {
  return sigma<float, true>(N, A, lda, sigma_out, ws, ws_bytes, stream);
}

}  // extern "C"
