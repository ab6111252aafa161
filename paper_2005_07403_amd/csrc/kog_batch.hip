// kog_batch.hip -- many Kogbetliantz problems of uneven order and mixed
// element type solved together (device-side convergence, hipGraph replay,
// work-list compaction; one, two or three steps per pass).  The shared device code is
// in kog_device.hpp.
#include <stdint.h>
#include <string.h>

#include <vector>

#include "kog_device.hpp"

namespace {

using namespace kog;

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
//
// In the three-step mode a pass takes a running problem three steps further
// while at least three steps remain before the last step of its sweep
// (pivots of the three steps, then the three-step tiles, out of place), and
// one step (in place, as in the one-step mode) otherwise: the last one or
// three steps of a sweep, so that every sweep still ends with the in-place
// step that tests convergence.
// ---------------------------------------------------------------------------
struct DevProb {
  void *A;
  long long lda, piv_off, out_off;  // buffer offsets in bytes from the workspace base
  long long piv1_off, out1_off;     // second rotation set (two- and three-step modes)
  long long piv2_off, out2_off;     // third rotation set (three-step mode)
  long long w_off;                  // second matrix (two- and three-step modes), lda = N
  int N, kind, kc, lc;
  int part_off, ntiles, max_sweeps, in_w;  // in_w: the iterate is in the second matrix
  int gx2, ny2, lc2;                // two-step tiles: row blocks, column tiles, pairs per wavefront
  int e;                            // the solve works on 2^-e A (kog_scale_kernel)
  int gx3, ny3, lc3, pad0;          // three-step tiles: row blocks, column tiles, output pairs per tile
  double tol, tot0;                 // tot0 = ||A_0||_F
  int t, sweeps, status, pad1;      // status: 0 running, 1 converged, 2 max_sweeps reached
  double off_rel;
};
struct BatchHdr {
  int nA, nB, nprob, active;
  int c0[5];  // multi-step tiles of element type k: items [c0[k], c0[k+1])
  int pad[3];
};

__host__ __device__ inline size_t arr_bytes(int N, int esz) {
  return (((size_t)(N / 2) * esz) + 255) & ~size_t(255);
}

template <class T, bool CPLX>
__device__ __forceinline__ Bufs<T, CPLX> bufs_of(char *ws, const DevProb &P, int set = 0) {
  Bufs<T, CPLX> b;
  size_t arr = arr_bytes(P.N, sizeof(T));
  const long long po = set == 2 ? P.piv2_off : set ? P.piv1_off : P.piv_off;
  const long long oo = set == 2 ? P.out2_off : set ? P.out1_off : P.out_off;
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

// the steps this pass takes problem P further (mode: steps per pass asked
// for): the last step of a sweep (t = N-2) is always a single one, and in the
// three-step mode so are those that leave fewer than three before it
__device__ __forceinline__ int pass_steps(int mode, const DevProb &P) {
  if (mode == 2) return P.t + 1 < P.N - 1 ? 2 : 1;
  if (mode == 3) return P.N - 2 - P.t >= 3 ? 3 : 1;
  return 1;
}

// pivots of step t+2 of a three-step pass, pair k, on lane sub of its four
// (all four lanes call it; valid where k is a pair of P)
template <class T, bool CPLX> __device__ __forceinline__ void batch_pivots3(char *ws, const DevProb &P, int k, int sub) {
  pivots3_quad<T, CPLX>(P.N, mat_of<T, CPLX>(ws, P), P.t, bufs_of<T, CPLX>(ws, P, 0), bufs_of<T, CPLX>(ws, P, 1),
                        bufs_of<T, CPLX>(ws, P, 2), k, sub, k < P.N / 2);
}

template <class T, bool CPLX>
__device__ __forceinline__ void batch_three_step(char *smem, char *ws, const DevProb &P, int bx, int by) {
  const Mat<T, CPLX> cur = mat_of<T, CPLX>(ws, P), nxt = mat_of<T, CPLX>(ws, P, true);
  three_step_tile<T, CPLX>(smem, P.N, cur.A, cur.lda, nxt.A, nxt.lda, P.t, bufs_of<T, CPLX>(ws, P, 0),
                           bufs_of<T, CPLX>(ws, P, 1), bufs_of<T, CPLX>(ws, P, 2), 1, P.lc3, bx, by);
}

// the largest binary exponent among the finite nonzero components of this
// thread's share of A
template <class T, bool CPLX> __device__ __forceinline__ int batch_maxexp(const DevProb &P) {
  Mat<T, CPLX> M{(T *)P.A, (size_t)P.lda};
  int e = kNoExp;
  for (int j = 0; j < P.N; ++j)
    for (int i = threadIdx.x; i < P.N; i += blockDim.x) {
      const int x = elem_exp(M.ld(i, j));
      e = x > e ? x : e;
    }
  return e;
}

// A <- 2^e A in place (e != 0) and the sums of squares of the result
template <class T, bool CPLX>
__device__ __forceinline__ void batch_scale_norm(const DevProb &P, int e, double &off, double &tot) {
  Mat<T, CPLX> M{(T *)P.A, (size_t)P.lda};
  for (int j = 0; j < P.N; ++j)
    for (int i = threadIdx.x; i < P.N; i += blockDim.x) {
      Cx<T> v = M.ld(i, j);
      if (e != 0) {
        v = Cx<T>{vldexp(v.re, e), vldexp(v.im, e)};
        M.st(i, j, v);
      }
      const double a2 = abs2(v);
      tot += a2;
      if (i != j) off += a2;
    }
}

__device__ __forceinline__ int block_max(int v, int *red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int s = kUpdBlock / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s && red[threadIdx.x + s] > red[threadIdx.x]) red[threadIdx.x] = red[threadIdx.x + s];
    __syncthreads();
  }
  int r = red[0];
  __syncthreads();
  return r;
}

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
  __shared__ int redi[kUpdBlock];
  for (int p = blockIdx.x; p < hdr->nprob; p += gridDim.x) {
    DevProb &P = probs[p];
    // scale A exactly by 2^-E (E: largest binary exponent), then take norms
    int E;
    switch (P.kind) {
      case SVD2_KOG_F64: E = batch_maxexp<double, false>(P); break;
      case SVD2_KOG_C128: E = batch_maxexp<double, true>(P); break;
      case SVD2_KOG_F32: E = batch_maxexp<float, false>(P); break;
      default: E = batch_maxexp<float, true>(P); break;
    }
    E = block_max(E, redi);
    if (E == kNoExp) E = 0;
    double off = 0, tot = 0;
    switch (P.kind) {
      case SVD2_KOG_F64: batch_scale_norm<double, false>(P, -E, off, tot); break;
      case SVD2_KOG_C128: batch_scale_norm<double, true>(P, -E, off, tot); break;
      case SVD2_KOG_F32: batch_scale_norm<float, false>(P, -E, off, tot); break;
      default: batch_scale_norm<float, true>(P, -E, off, tot); break;
    }
    off = block_sum(off, red);
    tot = block_sum(tot, red);
    if (threadIdx.x == 0) {
      double nrm = __builtin_sqrt(tot);
      double rel = nrm > 0 ? __builtin_sqrt(off) / nrm : 0.0;
      P.e = E;
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
                                                                    int mode) {
  const int nA = hdr->nA;
  for (int it = blockIdx.x; it < nA; it += gridDim.x) {
    const int2 item = items[it];
    const DevProb &P = probs[item.x];
    if (P.status != 0 || pass_steps(mode, P) != 1) continue;
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

// the pivots of steps t and t+1 of the problems of one element type in a
// two- or three-step pass
template <class T, bool CPLX, int KIND>
__global__ __launch_bounds__(kUpdBlock) void kog_batch_pivots2_kernel(char *ws, const BatchHdr *hdr,
                                                                      const int2 *items, const DevProb *probs,
                                                                      int mode) {
  const int nA = hdr->nA;
  for (int it = blockIdx.x; it < nA; it += gridDim.x) {
    const int2 item = items[it];
    const DevProb &P = probs[item.x];
    if (P.kind != KIND || P.status != 0 || pass_steps(mode, P) < 2) continue;
    const int k = item.y * kUpdBlock + (int)threadIdx.x;
    if (k < P.N / 2) batch_pivots2<T, CPLX>(ws, P, k);
  }
}

// the pivots of step t+2 of the problems of one element type in a
// three-step pass: four lanes per pair, so an item's kUpdBlock pairs are four
// work units of 64 (unit u: item u / 4, its pairs from (u % 4) 64 on)
template <class T, bool CPLX, int KIND>
__global__ __launch_bounds__(kUpdBlock) void kog_batch_pivots3_kernel(char *ws, const BatchHdr *hdr,
                                                                      const int2 *items, const DevProb *probs) {
  constexpr int R = kUpdBlock / 64;
  const int nU = hdr->nA * R;
  for (int u = blockIdx.x; u < nU; u += gridDim.x) {
    const int2 item = items[u / R];
    const DevProb &P = probs[item.x];
    if (P.kind != KIND || P.status != 0 || pass_steps(3, P) != 3) continue;
    const int k0 = item.y * kUpdBlock + (u % R) * 64;
    if (k0 >= P.N / 2) continue;  // uniform over the block
    batch_pivots3<T, CPLX>(ws, P, k0 + ((int)threadIdx.x >> 2), (int)threadIdx.x & 3);
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
    if (P.status != 0 || pass_steps(2, P) != 2) continue;
    batch_two_step<T, CPLX>(kog_smem, ws, P, item.y, item.z);
    __syncthreads();  // the next item reuses the LDS
  }
}

// the three-step tiles (problem, row block, column tile) of the problems of
// one element type in a three-step pass, one wavefront per tile
template <class T, bool CPLX, int KIND>
__global__ __launch_bounds__(64) void kog_batch_three_step_kernel(char *ws, const BatchHdr *hdr, const int4 *items,
                                                                  const DevProb *probs) {
  extern __shared__ __align__(16) char kog_smem[];
  const int c0 = hdr->c0[KIND], c1 = hdr->c0[KIND + 1];
  for (int it = c0 + (int)blockIdx.x; it < c1; it += gridDim.x) {
    const int4 item = items[it];
    const DevProb &P = probs[item.x];
    if (P.status != 0 || pass_steps(3, P) != 3) continue;
    batch_three_step<T, CPLX>(kog_smem, ws, P, item.y, item.z);
    __syncthreads();  // the next item reuses the LDS
  }
}

// single-step update tiles (problem, k0, l0, partial index) of the problems
// not in a two-step pass
__global__ __launch_bounds__(kUpdBlock) void kog_batch_update_kernel(char *ws, const BatchHdr *hdr,
                                                                     const int4 *items, const DevProb *probs,
                                                                     double *partials, int mode) {
  __shared__ double red[kUpdBlock];
  const int nB = hdr->nB;
  for (int it = blockIdx.x; it < nB; it += gridDim.x) {
    const int4 item = items[it];
    const DevProb &P = probs[item.x];
    if (P.status != 0 || pass_steps(mode, P) != 1) continue;
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
                                                                     const double *partials, int mode) {
  __shared__ double red[kUpdBlock];
  for (int p = blockIdx.x; p < hdr->nprob; p += gridDim.x) {
    DevProb &P = probs[p];
    // every thread reads the state before thread 0 changes it
    const int status = P.status, t = P.t, N = P.N, steps = pass_steps(mode, P);
    __syncthreads();
    if (status != 0) continue;
    if (steps > 1) {  // a multi-step pass: no sweep ends inside it
      if (threadIdx.x == 0) {
        P.t = t + steps;
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
// batch host driver
// ---------------------------------------------------------------------------
struct BatchLayout {
  size_t hdr, probs, itemsA, itemsB, itemsC, parts, bufs, total;
  size_t lds[4];  // multi-step tile LDS bytes per element type
  int maxA, maxB, maxC, nparts;
  int maxC_kind[4];
};

// steps per pass asked for by the flags (0: both multi-step modes, refused)
int batch_mode(unsigned flags) {
  const bool two = (flags & SVD2_KOG_TWO_STEP) != 0, three = (flags & SVD2_KOG_THREE_STEP) != 0;
  return two && three ? 0 : three ? 3 : two ? 2 : 1;
}

int esz_of(int kind) { return (kind == SVD2_KOG_F64 || kind == SVD2_KOG_C128) ? 8 : 4; }
bool cplx_of(int kind) { return kind == SVD2_KOG_C128 || kind == SVD2_KOG_C64; }

// column pairs per wavefront of the two-step tiles in a batch (workgroups of
// kUpdBlock / 64 wavefronts).  Fixed rather than taken from the single-problem
// shape table: a lone small problem wants many small tiles for parallelism,
// while a batch has parallelism from its many problems and loses to the halo
// reads of small tiles (256-problem batch: 8.6 s with 8, 9.5 s with the
// single-problem shapes).
int batch_lc2(int) { return 8; }

// output column pairs per three-step tile in a batch (one wavefront per
// tile), fixed for the same reason (256-problem batch: 8.46 s with 8, 7.81
// with 12, 7.62 with 16, 7.70 with 24, 7.88 with 32, 8.41 with 64; narrow
// tiles keep the GPU busy once only the largest problems are left)
int batch_lc3(int) { return 16; }

size_t three_step_lds_of(int kind, int lc) {
  switch (kind) {
    case SVD2_KOG_F64: return three_step_lds<double, false>(lc);
    case SVD2_KOG_C128: return three_step_lds<double, true>(lc);
    case SVD2_KOG_F32: return three_step_lds<float, false>(lc);
    default: return three_step_lds<float, true>(lc);
  }
}

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
                         int mode) {
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
    const int lc3 = batch_lc3(q.N), gx3 = (n + kShift3Out - 1) / kShift3Out, ny3 = (n + lc3 - 1) / lc3;
    const size_t set = (nin + nout) * arr;
    const int nsets = mode;  // rotation sets: one per step of a pass
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
      if (mode >= 2) {
        d.piv1_off = (long long)(bufs + set);
        d.out1_off = (long long)(bufs + set + nin * arr);
        d.w_off = (long long)(bufs + nsets * set);
      }
      if (mode == 2) {
        d.gx2 = gx2;
        d.ny2 = ny2;
        d.lc2 = lc2;
      }
      if (mode == 3) {
        d.piv2_off = (long long)(bufs + 2 * set);
        d.out2_off = (long long)(bufs + 2 * set + nin * arr);
        d.gx3 = gx3;
        d.ny3 = ny3;
        d.lc3 = lc3;
      }
      dp->push_back(d);
    }
    bufs += mode >= 2 ? nsets * set + wbytes : set;
    const int tiles = mode == 3 ? gx3 * ny3 : mode == 2 ? gx2 * ny2 : 0;
    L.maxA += (n + kUpdBlock - 1) / kUpdBlock;
    L.maxB += kt * lt;
    L.maxC += tiles;
    L.maxC_kind[q.dtype] += tiles;
    L.nparts += kt * lt;
    if (mode >= 2) {
      size_t l = mode == 3 ? three_step_lds_of(q.dtype, lc3) : two_step_lds_of(q.dtype, span);
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
      if (mode >= 2) {
        d.piv1_off += (long long)L.bufs;
        d.out1_off += (long long)L.bufs;
        d.w_off += (long long)L.bufs;
      }
      if (mode == 3) {
        d.piv2_off += (long long)L.bufs;
        d.out2_off += (long long)L.bufs;
      }
    }
  return SVD2_OK;
}

// work lists of the problems still running
void build_items(const std::vector<DevProb> &dp, std::vector<int2> &A, std::vector<int4> &B,
                 std::vector<int4> &C, int *c0, int mode) {
  A.clear();
  B.clear();
  C.clear();
  for (int kind = 0; kind < 4; ++kind) {  // multi-step tiles, grouped by element type
    c0[kind] = (int)C.size();
    if (mode < 2) continue;
    for (int p = 0; p < (int)dp.size(); ++p) {
      const DevProb &d = dp[p];
      if (d.status != 0 || d.kind != kind) continue;
      const int ny = mode == 3 ? d.ny3 : d.ny2, gx = mode == 3 ? d.gx3 : d.gx2;
      for (int y = 0; y < ny; ++y)
        for (int x = 0; x < gx; ++x) C.push_back(int4{p, x, y, 0});
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
  int gA, gB, gF, mode;
  // a second stream for the multi-step kernels of complex element types
  // (forked from and joined back to the pass's stream by events), so that
  // the problems of two element types advance concurrently: once few
  // problems are left, each type's kernels fill only part of the GPU
  hipStream_t side = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
};

// the multi-step part of a pass for the problems of one element type: the
// pivots, then the tiles
template <class T, bool CPLX, int KIND> svd2_status batch_multi_launch(const BatchRun &r, hipStream_t st) {
  if (r.L.maxC_kind[KIND] == 0) return SVD2_OK;
  BatchHdr *hdr = (BatchHdr *)(r.ws + r.L.hdr);
  DevProb *probs = (DevProb *)(r.ws + r.L.probs);
  const int2 *itemsA = (const int2 *)(r.ws + r.L.itemsA);
  const int4 *itemsC = (const int4 *)(r.ws + r.L.itemsC);
  hipLaunchKernelGGL((kog_batch_pivots2_kernel<T, CPLX, KIND>), dim3(r.gA), dim3(kUpdBlock), 0, st, r.ws, hdr,
                     itemsA, probs, r.mode);
  svd2_status s = hip_st(hipGetLastError());
  if (s != SVD2_OK) return s;
  const int g = r.L.maxC_kind[KIND] < 16384 ? r.L.maxC_kind[KIND] : 16384;
  if (r.mode == 3) {
    const int units = (kUpdBlock / 64) * r.L.maxA, g3 = units < 16384 ? units : 16384;
    hipLaunchKernelGGL((kog_batch_pivots3_kernel<T, CPLX, KIND>), dim3(g3), dim3(kUpdBlock), 0, st, r.ws, hdr,
                       itemsA, probs);
    s = hip_st(hipGetLastError());
    if (s != SVD2_OK) return s;
    hipLaunchKernelGGL((kog_batch_three_step_kernel<T, CPLX, KIND>), dim3(g), dim3(64), r.L.lds[KIND], st, r.ws,
                       hdr, itemsC, probs);
  } else {
    hipLaunchKernelGGL((kog_batch_two_step_kernel<T, CPLX, KIND>), dim3(g), dim3(kUpdBlock), r.L.lds[KIND], st,
                       r.ws, hdr, itemsC, probs);
  }
  return hip_st(hipGetLastError());
}

svd2_status batch_step(const BatchRun &r, hipStream_t st) {
  BatchHdr *hdr = (BatchHdr *)(r.ws + r.L.hdr);
  DevProb *probs = (DevProb *)(r.ws + r.L.probs);
  // the problems in a single step and those of each stream's element types
  // in a multi-step pass are disjoint: the two streams fork before the
  // single steps and join before the finish
  const bool multi = r.mode >= 2, two_streams = multi && r.side;
  hipStream_t cs = two_streams ? r.side : st;  // complex element types
  svd2_status s = SVD2_OK;
  if (two_streams) s = hip_st(hipEventRecord(r.fork, st));
  if (s == SVD2_OK && two_streams) s = hip_st(hipStreamWaitEvent(cs, r.fork, 0));
  if (s != SVD2_OK) return s;
  hipLaunchKernelGGL(kog_batch_pivot_kernel, dim3(r.gA), dim3(kUpdBlock), 0, st, r.ws, hdr,
                     (const int2 *)(r.ws + r.L.itemsA), probs, r.mode);
  s = hip_st(hipGetLastError());
  if (s != SVD2_OK) return s;
  hipLaunchKernelGGL(kog_batch_update_kernel, dim3(r.gB), dim3(kUpdBlock), 0, st, r.ws, hdr,
                     (const int4 *)(r.ws + r.L.itemsB), probs, (double *)(r.ws + r.L.parts), r.mode);
  s = hip_st(hipGetLastError());
  if (s == SVD2_OK && multi) s = batch_multi_launch<double, true, SVD2_KOG_C128>(r, cs);
  if (s == SVD2_OK && multi) s = batch_multi_launch<float, true, SVD2_KOG_C64>(r, cs);
  if (s == SVD2_OK && multi) s = batch_multi_launch<double, false, SVD2_KOG_F64>(r, st);
  if (s == SVD2_OK && multi) s = batch_multi_launch<float, false, SVD2_KOG_F32>(r, st);
  if (s == SVD2_OK && two_streams) s = hip_st(hipEventRecord(r.join, cs));
  if (s == SVD2_OK && two_streams) s = hip_st(hipStreamWaitEvent(st, r.join, 0));
  if (s != SVD2_OK) return s;
  hipLaunchKernelGGL(kog_batch_finish_kernel, dim3(r.gF), dim3(kUpdBlock), 0, st, hdr, probs,
                     (const double *)(r.ws + r.L.parts), r.mode);
  return hip_st(hipGetLastError());
}

// the iterate back into the caller's matrix (if it is in the second one),
// then A <- 2^e A
template <class T, bool CPLX> svd2_status finish_problem(const DevProb &d, char *ws, hipStream_t st) {
  const int grid = d.N < 4096 ? d.N : 4096;
  const Mat<T, CPLX> a{(T *)d.A, (size_t)d.lda};
  if (d.in_w) {
    hipLaunchKernelGGL((kog_copy_kernel<T, CPLX>), dim3(grid), dim3(256), 0, st, d.N,
                       Mat<T, CPLX>{(T *)(ws + d.w_off), (size_t)d.N}, a);
    svd2_status s = hip_st(hipGetLastError());
    if (s != SVD2_OK) return s;
  }
  if (d.e == 0) return SVD2_OK;
  hipLaunchKernelGGL((kog_scale_kernel<T, CPLX>), dim3(grid), dim3(256), 0, st, d.N, a, d.e);
  return hip_st(hipGetLastError());
}

svd2_status upload_items(const BatchRun &r, const std::vector<DevProb> &dp, int active) {
  std::vector<int2> A;
  std::vector<int4> B, C;
  BatchHdr h = {};
  build_items(dp, A, B, C, h.c0, r.mode);
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
  if (flags & ~(unsigned)(SVD2_KOG_GRAPH | SVD2_KOG_TWO_STEP | SVD2_KOG_THREE_STEP)) return SVD2_ERR_FLAGS;
  BatchRun r;
  r.mode = batch_mode(flags);
  if (r.mode == 0) return SVD2_ERR_FLAGS;
  std::vector<DevProb> dp;
  svd2_status s = batch_layout(nprob, pr, r.L, &dp, r.mode);
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
  // two streams when both real and complex problems take multi-step passes
  const bool real_multi = r.L.maxC_kind[SVD2_KOG_F64] + r.L.maxC_kind[SVD2_KOG_F32] > 0;
  const bool cplx_multi = r.L.maxC_kind[SVD2_KOG_C128] + r.L.maxC_kind[SVD2_KOG_C64] > 0;
  struct Side {  // released on every return below
    BatchRun &r;
    ~Side() {
      if (r.fork) (void)hipEventDestroy(r.fork);
      if (r.join) (void)hipEventDestroy(r.join);
      if (r.side) (void)hipStreamDestroy(r.side);
    }
  } side_guard{r};
  if (r.mode >= 2 && real_multi && cplx_multi) {
    s = hip_st(hipStreamCreateWithFlags(&r.side, hipStreamNonBlocking));
    if (s == SVD2_OK) s = hip_st(hipEventCreateWithFlags(&r.fork, hipEventDisableTiming));
    if (s == SVD2_OK) s = hip_st(hipEventCreateWithFlags(&r.join, hipEventDisableTiming));
    if (s != SVD2_OK) return s;
  }
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
  long long max_steps = 0;  // passes: at most N-1 per sweep (N/2 with two steps per pass)
  for (const DevProb &d : dp) {
    long long m = (long long)d.max_sweeps * (r.mode == 2 ? d.N / 2 : d.N - 1);
    if (m > max_steps) max_steps = m;
  }
  const int K = 64;  // passes per replay / between host checks
  hipGraphExec_t exec = nullptr;
  hipStream_t cap = nullptr;
  auto capture = [&]() -> svd2_status {
    if (exec) {
      (void)hipGraphExecDestroy(exec);
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
    if (g) (void)hipGraphDestroy(g);
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
  if (exec) (void)hipGraphExecDestroy(exec);
  if (cap) (void)hipStreamDestroy(cap);
  if (s != SVD2_OK) return s;
  s = hip_st(hipMemcpyAsync(dp.data(), r.ws + r.L.probs, dp.size() * sizeof(DevProb), hipMemcpyDeviceToHost, st));
  if (s == SVD2_OK) s = hip_st(hipStreamSynchronize(st));
  if (s != SVD2_OK) return s;
  // iterates left in the second matrix go back to the caller's, then every
  // matrix is scaled back by 2^e
  for (int p = 0; p < nprob && s == SVD2_OK; ++p) {
    switch (dp[p].kind) {
      case SVD2_KOG_F64: s = finish_problem<double, false>(dp[p], r.ws, st); break;
      case SVD2_KOG_C128: s = finish_problem<double, true>(dp[p], r.ws, st); break;
      case SVD2_KOG_F32: s = finish_problem<float, false>(dp[p], r.ws, st); break;
      default: s = finish_problem<float, true>(dp[p], r.ws, st); break;
    }
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

extern "C" {

size_t kog_batch_workspace_bytes_flags(int nprob, const kog_problem *probs, unsigned flags) {
  BatchLayout L;
  if (flags & ~(unsigned)(SVD2_KOG_GRAPH | SVD2_KOG_TWO_STEP | SVD2_KOG_THREE_STEP)) return 0;
  const int mode = batch_mode(flags);
  if (mode == 0 || batch_layout(nprob, probs, L, nullptr, mode) != SVD2_OK) return 0;
  return L.total;
}

size_t kog_batch_workspace_bytes(int nprob, const kog_problem *probs) {
  return kog_batch_workspace_bytes_flags(nprob, probs, 0);
}

svd2_status kog_batch_solve(int nprob, kog_problem *probs, void *ws, size_t ws_bytes, unsigned flags,
                            hipStream_t stream) {
  return batch_solve(nprob, probs, ws, ws_bytes, flags, stream);
}

}  // extern "C"
