/*
 * svd2.h -- C ABI of libsvd2: batched SVDs of order two on MI355X (gfx950).
 *
 * Method: V. Novakovic, "Batched computation of the singular value
 * decompositions of order two by the AVX-512 vectorization",
 * arXiv:2005.07403.  For each k < n the library computes A = U Sigma V* of a
 * real or complex 2x2 matrix A (section 1), as
 *   exact power-of-two scaling A^ = 2^s A            (section 2.1, eq. (2)),
 *   URV factorisation R = U+* A^ V+                  (section 2.2, eqs. (3)-(11)),
 *   SVD of the non-negative upper-triangular R       (section 2.3, eqs. (12)-(17)),
 *   assembly of U and V                              (eqs. (28)-(29)).
 * One GPU lane computes one matrix; there is no branching on data except the
 * optional FP64 rescue of near-degenerate FP32 lanes.
 *
 * Data layout (section 3): structure of arrays.  Every matrix element (and,
 * for complex data, its real and imaginary part) is its own contiguous array
 * of n elements; element k of every array belongs to matrix k.  Argument
 * order follows the record layout of section 8: 11, 21, 12, 22.
 *
 * Outputs: U, V in the same layout; smax, smin = the scaled singular values
 * sigma'_max >= sigma'_min >= 0 of eq. (12) (Theorem 1: always finite); s = the
 * exponent of eq. (2) stored in the element type: Sigma = 2^-s Sigma'.
 * s is the largest finite value of the type for a zero matrix, and -0 after a
 * backscale.  By default sigma' and s are returned unscaled, as the paper
 * recommends (eq. (28) and Fig. 1); see the SVD2_BACKSCALE_* flags.
 *
 * Conventions, for every entry point:
 *  - All array pointers are DEVICE pointers (hipMalloc / torch allocations)
 *    owned by the caller; the library keeps no reference after the call and
 *    allocates nothing.  The argument struct is read on the host during the
 *    call only.
 *  - Work is enqueued on `stream` and the call returns without waiting;
 *    results are valid once the stream has been synchronised.
 *  - Arguments are validated before any HIP call; on an argument error
 *    nothing is launched.  n == 0 is a no-op returning SVD2_OK.
 *  - Pointers must be aligned to the element size; 16-byte alignment of every
 *    array enables the wide-load path (hipMalloc gives 256 bytes).
 *  - No output may overlap an input or another output (SVD2_ERR_ALIAS).
 *  - Inputs must be finite (section 1).  A lane with a non-finite input gets
 *    unspecified outputs; no other lane is affected and no error is raised.
 */
#ifndef SVD2_H
#define SVD2_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SVD2_OK = 0,
  SVD2_ERR_NULL = 1,     /* a required pointer is NULL                       */
  SVD2_ERR_ALIGN = 2,    /* a pointer is not aligned to its element size     */
  SVD2_ERR_ALIAS = 3,    /* an output overlaps an input or another output    */
  SVD2_ERR_FLAGS = 4,    /* unknown or contradictory flag bits               */
  SVD2_ERR_HIP = 5,      /* a HIP call failed; see svd2_last_hip_error()     */
  SVD2_ERR_SIZE = 6,     /* n or a workspace size is out of range            */
  SVD2_NOT_CONVERGED = 7 /* Kogbetliantz: max_sweeps reached                 */
} svd2_status;

enum {
  /* backscale of eq. (28); at most one of these may be set */
  SVD2_BACKSCALE_NONE = 0,  /* default: write sigma' and s                          */
  SVD2_BACKSCALE_SAFE = 1,  /* per lane, only where 2^-s sigma' is exact and finite;
                               such lanes get Sigma and s = -0                       */
  SVD2_BACKSCALE_ALL = 2,   /* Fig. 1: unconditional (may overflow or underflow)     */
  /* FP32 entry points only: FP64 rescue of lanes with sigma'_min < 2^-20 sigma'_max.
     On such lanes the (2,2) entry of R is recomputed from det(A^) in FP64 (exact
     products, compensated sum), and eqs. (9), (13)-(17), (29) run in FP64. */
  SVD2_RESCUE_FP64 = 4,     /* rescue inside the main kernel (divergent, no queue)  */
  SVD2_RESCUE_QUEUE = 8,    /* with RESCUE_FP64: flagged lanes are compacted into a
                               queue (one atomic per wavefront) and redone by a
                               second kernel; needs a workspace                     */
  SVD2_RESCUE_SIGMA = 16,   /* with RESCUE_FP64: on flagged lanes only sigma'_min is
                               recomputed, as |det(A^)| / sigma'_max in FP64 (the
                               product of the singular values is |det|); U, V and
                               sigma'_max keep their FP32 values.  Same relative
                               accuracy of sigma_min for a fraction of the FP64 work */
  /* with RESCUE_FP64, instead of SVD2_RESCUE_SIGMA: on flagged lanes FP64 is
     used only up to the triangular SVD -- the (2,2) entry of R from det(A^)
     (and with it sigma'_min), its phase D^ (eq. (9)) and the rotation angles
     phi, psi with sigma' (eqs. (13)-(17)) -- whose tangents, cosines and phase
     are rounded to FP32 and assembled into U and V in FP32 by eq. (29) (or
     eq. (31)), as on an unflagged lane.  sigma' and s are bitwise those of the
     FP64 tail; U and V are within a few FP32 ulps of them. */
  SVD2_RESCUE_TRI = 128,
  /* all four entry points: singular values only, the counterpart of the
     values-only routine of section 2.  The last phase of section 4, the
     assembly of U and V (eq. (29)), is skipped; the U and V pointers may be
     NULL and are neither checked nor written.  smax, smin and s are bitwise
     those of the same call without the flag (they do not depend on the
     assembly), with every other flag including the rescues. */
  SVD2_NO_UV = 32,
  /* all four entry points: assemble U by the sine form of eq. (31), from
     sin = cos * tan (section 7), instead of the tangent form of eq. (29) (the
     default); V, sigma' and s are the same in both.  For the comparison of
     section 8, whose pointwise routine assembles this way: with the products
     cc = cos(a)cos(p), ss = sin(a)sin(p), cs = cos(a)sin(p), sc = sin(a)cos(p)
     of the angles alpha (QR) and phi (triangular SVD), the elements of P_r^* U
     are d_11 (cc - d^ ss), d_11 (cs + d^ sc), -d_22 (sc + d^ cs) and
     d_22 (d^ cc - ss), each bracket one fma per part, each product by d_ii as
     eq. (5).  Ignored with SVD2_NO_UV. */
  SVD2_SINE_FORM = 64
};

/* Real FP64: a_ij in, u_ij, v_ij, smax, smin, s out (all length n). */
typedef struct {
  const double *a11, *a21, *a12, *a22;
  double *u11, *u21, *u12, *u22;
  double *v11, *v21, *v12, *v22;
  double *smax, *smin, *s;
} dsvd2_args;

/* Complex FP64: real and imaginary parts as separate arrays (section 3). */
typedef struct {
  const double *a11r, *a11i, *a21r, *a21i, *a12r, *a12i, *a22r, *a22i;
  double *u11r, *u11i, *u21r, *u21i, *u12r, *u12i, *u22r, *u22i;
  double *v11r, *v11i, *v21r, *v21i, *v12r, *v12i, *v22r, *v22i;
  double *smax, *smin, *s;
} zsvd2_args;

/* Real FP32.  nrescued: optional device counter; when not NULL the number of
   rescued lanes is ADDED to it (the caller zeroes it). */
typedef struct {
  const float *a11, *a21, *a12, *a22;
  float *u11, *u21, *u12, *u22;
  float *v11, *v21, *v12, *v22;
  float *smax, *smin, *s;
  uint32_t *nrescued;
} ssvd2_args;

/* Complex FP32. */
typedef struct {
  const float *a11r, *a11i, *a21r, *a21i, *a12r, *a12i, *a22r, *a22i;
  float *u11r, *u11i, *u21r, *u21i, *u12r, *u12i, *u22r, *u22i;
  float *v11r, *v11i, *v21r, *v21i, *v12r, *v12i, *v22r, *v22i;
  float *smax, *smin, *s;
  uint32_t *nrescued;
} csvd2_args;

/* Batched SVDs of n matrices (sections 2-7).  flags: SVD2_BACKSCALE_* [| SVD2_NO_UV]
   [| SVD2_SINE_FORM].
   Errors: SVD2_ERR_NULL/ALIGN/ALIAS/FLAGS before launch, SVD2_ERR_HIP if the
   launch fails. */
svd2_status dsvd2_batch(size_t n, const dsvd2_args *p, unsigned flags, hipStream_t stream);
svd2_status zsvd2_batch(size_t n, const zsvd2_args *p, unsigned flags, hipStream_t stream);

/* FP32 form (the paper notes the method carries over to single precision,
   section 1; the tan 2phi clamp becomes sqrt(FLT_MAX), section 7).
   flags: SVD2_BACKSCALE_* | SVD2_RESCUE_FP64 [| SVD2_RESCUE_QUEUE] [| SVD2_RESCUE_SIGMA or
   SVD2_RESCUE_TRI]
   [| SVD2_NO_UV] [| SVD2_SINE_FORM] (with the FP64 tail rescue the rescued lanes are
   assembled in FP64 by the same form).
   ws / ws_bytes: device workspace, at least svd2_workspace_bytes(n, flags)
   bytes (may be NULL/0 when that is 0).  With RESCUE_QUEUE, n must be below
   2^32 (SVD2_ERR_SIZE otherwise).  Calls sharing one workspace must not
   overlap in time. */
svd2_status ssvd2_batch(size_t n, const ssvd2_args *p, unsigned flags, void *ws,
                        size_t ws_bytes, hipStream_t stream);
svd2_status csvd2_batch(size_t n, const csvd2_args *p, unsigned flags, void *ws,
                        size_t ws_bytes, hipStream_t stream);

/* Workspace needed by the FP32 entry points: 0 unless SVD2_RESCUE_QUEUE. */
size_t svd2_workspace_bytes(size_t n, unsigned flags);

/* Phase outputs of the URV factorization (section 2.2), written beside the
   final results in the same layout (section 4 allows the output of a phase
   to be kept this way): the real upper-triangular factor
   R = [[r11, r12], [0, r22]] of eq. (9), r11 >= max(r12, r22) >= 0, and the
   unitary factors of eq. (11), A^ = 2^s A = U_+ R V_+^*, with
   U_+ = P_r D Q_alpha D^ and V_+ = P_c D~:
     D = diag(d1, d2), the conjugate of D* of eq. (4) (signs in the real case);
     Q_alpha = cos(alpha) [[1, tan(alpha)], [-tan(alpha), 1]] of eqs. (6)-(7);
     D^ = diag(1, e^{i arg r'_22}) of eq. (9), D~ = diag(1, e^{-i arg r'_12})
     of eq. (8).
   Operation order (the paper gives none for U_+): with ca = cos(alpha) and
   sa = ca * (-tan(alpha)), one rounding, the rows of U_+ before the swap P_r
   are [d1 ca, -((d1 dh) sa)] and [d2 sa, (d2 dh) ca], dh = D^_22, each
   product rounded once per part (d1 dh by eq. (5)); V_+ is [[1, 0], [0, D~_22]]
   before the swap P_c (exact).  R, U_+ and V_+ are those of the scaled matrix,
   so the backscale flags are refused (SVD2_ERR_FLAGS): s is always returned.
   r11, r12, r22 are required; the U_+ and V_+ pointers are all given or all
   NULL (then only R is written).  Every other flag, pointer rule and error is
   that of the plain entry point; the main outputs are bitwise those of the
   plain call.  FP32: R, U_+ and V_+ are the FP32 pipeline's values on every
   lane (the rescues recompute later phases only). */
typedef struct {
  double *r11, *r12, *r22;
  double *u11, *u21, *u12, *u22;
  double *v11, *v21, *v12, *v22;
} dsvd2_urv;
typedef struct {
  double *r11, *r12, *r22;
  double *u11r, *u11i, *u21r, *u21i, *u12r, *u12i, *u22r, *u22i;
  double *v11r, *v11i, *v21r, *v21i, *v12r, *v12i, *v22r, *v22i;
} zsvd2_urv;
typedef struct {
  float *r11, *r12, *r22;
  float *u11, *u21, *u12, *u22;
  float *v11, *v21, *v12, *v22;
} ssvd2_urv;
typedef struct {
  float *r11, *r12, *r22;
  float *u11r, *u11i, *u21r, *u21i, *u12r, *u12i, *u22r, *u22i;
  float *v11r, *v11i, *v21r, *v21i, *v12r, *v12i, *v22r, *v22i;
} csvd2_urv;

svd2_status dsvd2_batch_urv(size_t n, const dsvd2_args *p, const dsvd2_urv *f, unsigned flags,
                            hipStream_t stream);
svd2_status zsvd2_batch_urv(size_t n, const zsvd2_args *p, const zsvd2_urv *f, unsigned flags,
                            hipStream_t stream);
svd2_status ssvd2_batch_urv(size_t n, const ssvd2_args *p, const ssvd2_urv *f, unsigned flags, void *ws,
                            size_t ws_bytes, hipStream_t stream);
svd2_status csvd2_batch_urv(size_t n, const csvd2_args *p, const csvd2_urv *f, unsigned flags, void *ws,
                            size_t ws_bytes, hipStream_t stream);

/* Launch shape of the batched kernels (set by the autotuner).  block: threads
   per workgroup, 64, 128, 192 or 256; per_thread: matrices per lane, 1 or 2
   (2 uses 16-byte loads and stores when every array is 16-byte aligned).
   svd2_set_launch sets every element type; svd2_set_launch_kind one of them:
   kind 0 real FP64, 1 complex FP64, 2 real FP32, 3 complex FP32 (the
   SVD2_KOG_* dtype codes), 4-7 the same with SVD2_NO_UV.  Takes effect for
   later calls from any thread.
   SVD2_ERR_SIZE / SVD2_ERR_FLAGS for values out of range.
   svd2_get_launch reports the real-FP64 shape. */
svd2_status svd2_set_launch(int block, int per_thread);
svd2_status svd2_set_launch_kind(int kind, int block, int per_thread);
void svd2_get_launch(int *block, int *per_thread);
void svd2_get_launch_kind(int kind, int *block, int *per_thread);

/* Text of a status code, and the last hipError_t seen by this thread. */
const char *svd2_status_string(svd2_status st);
int svd2_last_hip_error(void);

/* Memory-pattern probe, a diagnostic: the loads and stores of the batched
   kernel of element type `kind` (0 real FP64, 1 complex FP64, 2 real FP32,
   3 complex FP32; 4-7 the same with SVD2_NO_UV) with the same launch shape,
   but no SVD arithmetic (each output = the sum of the inputs plus its
   index).  in/out: host arrays of 4 or 8 input and 11, 19 or (kinds 4-7) 3
   output device pointers of n elements.  Its time is the ceiling the memory
   system sets for that access pattern. */
svd2_status svd2_stream_probe(int kind, size_t n, const void *const *in, void *const *out,
                              hipStream_t stream);

/* Conformance probe of the device primitives the kernels use (correct
   rounding of /, sqrt, fma, ldexp; frexp exponents of subnormals; NaN
   handling of fmin/fmax), for tests.  op: 0 div, 1 sqrt, 2 fma, 3 ldexp(x,
   (int)y), 4 frexp exponent of x (as a value), 5 fmin(x,y), 6 fmax(x,y),
   7 the kernels' square root for arguments x >= 1, 8 their reciprocal 1/x for
   x >= 1 with a normal result (ops 7 and 8 must equal ops 1 and 0 on that
   domain; y and z are unused by ops 1, 4, 7 and 8 and may be NULL).
   x, y, z, out: device arrays of n doubles (FP64) or floats (FP32). */
svd2_status svd2_probe_f64(int op, size_t n, const double *x, const double *y,
                           const double *z, double *out, hipStream_t stream);
svd2_status svd2_probe_f32(int op, size_t n, const float *x, const float *y,
                           const float *z, float *out, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Kogbetliantz method for the SVD of a square matrix A of even order N
 * (section 1): each parallel step gathers the pivot blocks
 * [[a_pp, a_pq], [a_qp, a_qq]] of N/2 disjoint index pairs, computes their
 * 2x2 SVDs with the batched kernels above (backscaled; FP32 with the FP64
 * rescue), and updates A <- U^* A V in place: rows p, q by U_k^*, columns
 * p, q by V_k, with each pivot block set to diag(sigma_p, sigma_q) and exact
 * zeros.  The paper gives neither the pivot ordering nor the stopping rule;
 * this library uses:
 *  - ordering: circle-method round robin, N-1 steps per sweep; at step t,
 *    pair 0 = (t, N-1), pair k >= 1 = ((t+k) mod (N-1), (t-k) mod (N-1)),
 *    oriented p < q;
 *  - placement: if |a_pp| < |a_qq| the singular values and the columns of
 *    U_k, V_k are swapped (sigma_min goes to (p,p)), keeping the rotations
 *    near the identity as the iteration converges;
 *  - stopping: off(A) = sqrt(sum_{i != j} |a_ij|^2) < tol * ||A_0||_F, tested
 *    before every sweep (one device-to-host copy per sweep);
 *  - scaling: *_solve and kog_batch_solve multiply A by 2^-E before the
 *    first sweep and by 2^E after the last, E the largest binary exponent
 *    among its finite nonzero components (eq. (2) applied to the whole
 *    matrix).  The factor is exact and commutes with the steps unless a value
 *    reaches the subnormal range; it keeps the sums of squares of the
 *    stopping test finite and nonzero for any finite A.  *_step and *_sweep
 *    do not scale.
 * On return A holds the singular values on its diagonal (unsorted, >= 0).
 *
 * Storage: column-major, leading dimension lda >= N (in elements; complex
 * elements are interleaved re, im).  A must be aligned to its element size.
 * ws: device workspace of kog_workspace_bytes(N, dtype) bytes
 * (kog_workspace_bytes_flags(N, dtype, flags) with SVD2_KOG_TWO_STEP),
 * 256-byte aligned, not overlapping A; calls sharing a workspace must not
 * overlap.
 * Entry points enqueue on `stream`; *_solve synchronises the stream once per
 * sweep and returns when done.  After an error return the contents of A are
 * unspecified.  Errors are as for the batched calls; a fused
 * sweep whose grid barrier does not complete within its spin bound aborts all
 * workgroups and *_solve returns SVD2_ERR_HIP.
 * flags: 0 = fused (one persistent cooperative kernel per sweep, gather + SVD
 * and update separated by grid barriers), SVD2_KOG_UNFUSED = per step a
 * gather kernel, the batched SVD entry point and an update kernel,
 * SVD2_KOG_UNFUSED | SVD2_KOG_GRAPH = that chain captured once per solve
 * into a hipGraph and replayed per sweep (solve only).
 * SVD2_KOG_TWO_STEP (sweep and solve only, alone): two steps per pass over
 * the matrix, out of place between A and a matrix buffer in the workspace.
 * Under the circle ordering each 2x2 block after step t+1 depends on a 4x4
 * neighbourhood before step t, and the pivots of step t+1 follow from the
 * rotations of step t and two blocks each, so both steps' rotations are known
 * before the matrix is read; every entry is computed with the operations of
 * the single-step update (bitwise the same result) and the matrix is read and
 * written once per two steps.  The result is always returned in A.
 * SVD2_KOG_THREE_STEP (step, sweep and solve, alone): the same with three
 * steps per pass (each 2x2 block after step t+2 depends on an 8x8
 * neighbourhood before step t; the pivots of step t+2 are formed from it with
 * the rotations of steps t and t+1), so the matrix is read and written once
 * per three steps; a sweep's N-1 steps end with a two-step pass or a single
 * step where three do not divide them.  Workspace of
 * kog_workspace_bytes_flags(N, dtype, SVD2_KOG_THREE_STEP).  Bitwise the
 * result of single steps, returned in A.  Also accepted by the SVD entry
 * points (U and V six steps per walk); not by the batch entry point.
 * ------------------------------------------------------------------------- */
enum { SVD2_KOG_UNFUSED = 1, SVD2_KOG_GRAPH = 2, SVD2_KOG_TWO_STEP = 4, SVD2_KOG_THREE_STEP = 8 };
enum { SVD2_KOG_F64 = 0, SVD2_KOG_C128 = 1, SVD2_KOG_F32 = 2, SVD2_KOG_C64 = 3 };

size_t kog_workspace_bytes(int N, int dtype);
/* the same for the given flags (SVD2_KOG_TWO_STEP adds N^2 elements,
   SVD2_KOG_THREE_STEP those and a third set of rotations) */
size_t kog_workspace_bytes_flags(int N, int dtype, unsigned flags);

/* one step t (0 <= t < N-1); flags 0 (fused kernel) or SVD2_KOG_UNFUSED.
   With SVD2_KOG_TWO_STEP (alone): steps t and t+1 (0 <= t, t+1 < N-1) in one
   two-step pass into the workspace matrix, which is then copied back into A
   (workspace of kog_workspace_bytes_flags(N, dtype, SVD2_KOG_TWO_STEP)).
   With SVD2_KOG_THREE_STEP (alone): steps t, t+1, t+2 (t + 2 < N-1) in one
   three-step pass, copied back the same way. */
svd2_status dkog_step(int N, double *A, int lda, int t, void *ws, size_t ws_bytes, unsigned flags,
                      hipStream_t stream);
svd2_status zkog_step(int N, double *A, int lda, int t, void *ws, size_t ws_bytes, unsigned flags,
                      hipStream_t stream);
svd2_status skog_step(int N, float *A, int lda, int t, void *ws, size_t ws_bytes, unsigned flags,
                      hipStream_t stream);
svd2_status ckog_step(int N, float *A, int lda, int t, void *ws, size_t ws_bytes, unsigned flags,
                      hipStream_t stream);
/* one sweep: steps 0 .. N-2 */
svd2_status dkog_sweep(int N, double *A, int lda, void *ws, size_t ws_bytes, unsigned flags,
                       hipStream_t stream);
svd2_status zkog_sweep(int N, double *A, int lda, void *ws, size_t ws_bytes, unsigned flags,
                       hipStream_t stream);
svd2_status skog_sweep(int N, float *A, int lda, void *ws, size_t ws_bytes, unsigned flags,
                       hipStream_t stream);
svd2_status ckog_sweep(int N, float *A, int lda, void *ws, size_t ws_bytes, unsigned flags,
                       hipStream_t stream);
/* sweeps until converged: SVD2_OK, or SVD2_NOT_CONVERGED after max_sweeps.
   sweeps, off_rel (host pointers, may be NULL): sweeps done, final off(A)/||A_0||_F */
svd2_status dkog_solve(int N, double *A, int lda, double tol, int max_sweeps, int *sweeps,
                       double *off_rel, void *ws, size_t ws_bytes, unsigned flags, hipStream_t stream);
svd2_status zkog_solve(int N, double *A, int lda, double tol, int max_sweeps, int *sweeps,
                       double *off_rel, void *ws, size_t ws_bytes, unsigned flags, hipStream_t stream);
svd2_status skog_solve(int N, float *A, int lda, double tol, int max_sweeps, int *sweeps,
                       double *off_rel, void *ws, size_t ws_bytes, unsigned flags, hipStream_t stream);
svd2_status ckog_solve(int N, float *A, int lda, double tol, int max_sweeps, int *sweeps,
                       double *off_rel, void *ws, size_t ws_bytes, unsigned flags, hipStream_t stream);
/* dkog_solve without a caller workspace, for callers that cannot allocate
 * device memory (code under stream capture, serving loops, harnesses that
 * forbid hipMalloc).  The library calls no hipMalloc, hipFree or other
 * allocating routine: the workspace is a 2 MiB array that the library's code
 * object holds on every GPU it runs on, until the process ends.
 *  - Arguments and results as dkog_solve; flags: 0 (fused) or
 *    SVD2_KOG_UNFUSED only (SVD2_ERR_FLAGS otherwise: the hipGraph mode
 *    allocates its graph and the two-step mode needs an N x N buffer).
 *  - N is limited by the array: kog_workspace_bytes(N, SVD2_KOG_F64) must not
 *    exceed 2 MiB, i.e. N <= 30272 (SVD2_ERR_SIZE otherwise, before any HIP
 *    call).
 *  - Every call on one GPU shares that GPU's array, and the array keeps the
 *    last call's contents (each call overwrites what it reads, so nothing
 *    carries over).  Calls that overlap in time on one GPU -- from several
 *    host threads or on several streams -- race on the array and give
 *    undefined results; serialise them. */
svd2_status dkog_solve_noalloc(int N, double *A, int lda, double tol, int max_sweeps, int *sweeps,
                               double *off_rel, unsigned flags, hipStream_t stream);
/* off(A)^2 and ||A||_F^2 accumulated in FP64 (host outputs; synchronises) */
svd2_status dkog_norms(int N, const double *A, int lda, double *off2, double *tot2, void *ws,
                       size_t ws_bytes, hipStream_t stream);
svd2_status zkog_norms(int N, const double *A, int lda, double *off2, double *tot2, void *ws,
                       size_t ws_bytes, hipStream_t stream);
svd2_status skog_norms(int N, const float *A, int lda, double *off2, double *tot2, void *ws,
                       size_t ws_bytes, hipStream_t stream);
svd2_status ckog_norms(int N, const float *A, int lda, double *off2, double *tot2, void *ws,
                       size_t ws_bytes, hipStream_t stream);
/* ---------------------------------------------------------------------------
 * Many Kogbetliantz problems of uneven order and mixed element type in one
 * solve.  Each step of the batch runs three kernels over all running problems
 * at once (pivot gathers + 2x2 SVDs; updates, with each problem's tile shape
 * from kog_set_tile_rules; a per-problem finish that advances the problem's
 * own step and, at the end of its sweep, decides convergence on the device
 * from the off-diagonal mass the update wrote).  Problems keep their own
 * sweep length N_p - 1; a converged problem stops.  The host checks one
 * counter every 64 steps and compacts the work lists as problems finish.
 * With SVD2_KOG_GRAPH the 64 steps are captured once into a hipGraph and
 * replayed.  With SVD2_KOG_TWO_STEP each pass takes every running problem
 * two steps further (the single-problem two-step mode: pivots of both
 * steps, then one out-of-place pass over the matrix), except the last step
 * of each sweep, which stays a single in-place step; every problem gets a
 * second matrix in the workspace, and results end in the caller's matrices,
 * bitwise equal to single steps.  With SVD2_KOG_THREE_STEP a pass takes a
 * running problem three steps further (the single-problem three-step mode)
 * while at least three steps remain before the last step of its sweep, and
 * one in-place step otherwise, so that every sweep ends with the in-place
 * step that tests convergence; three rotation sets and a second matrix per
 * problem.  In both multi-step modes, when the batch holds real and complex
 * problems, the complex problems' kernels of a pass run on a second stream,
 * created for the call, forked from `stream` and joined back to it in every
 * pass by events (also inside the hipGraphs), and destroyed before the call
 * returns.  Synchronises the stream; returns SVD2_OK if every problem
 * converged, SVD2_NOT_CONVERGED otherwise (see each problem's status).
 * ------------------------------------------------------------------------- */
typedef struct {
  int dtype;      /* in: SVD2_KOG_F64, _C128, _F32 or _C64                       */
  int N;          /* in: even order                                              */
  int lda;        /* in: leading dimension (elements), >= N                      */
  void *A;        /* in/out: device matrix, column-major; diagonal = sigma on exit */
  double tol;     /* in: stop when off(A) < tol ||A_0||_F (checked per sweep)    */
  int max_sweeps; /* in                                                          */
  int status;     /* out: SVD2_OK or SVD2_NOT_CONVERGED                          */
  int sweeps;     /* out: sweeps done                                            */
  double off_rel; /* out: off(A) / ||A_0||_F at the last check                   */
} kog_problem;

/* Device workspace for kog_batch_solve without SVD2_KOG_TWO_STEP (0 on
   invalid descriptors). */
size_t kog_batch_workspace_bytes(int nprob, const kog_problem *probs);
/* the same for the given flags (SVD2_KOG_TWO_STEP adds a second rotation set
   and an N^2 matrix per problem, SVD2_KOG_THREE_STEP two more sets and the
   matrix; 0 for flags kog_batch_solve refuses) */
size_t kog_batch_workspace_bytes_flags(int nprob, const kog_problem *probs, unsigned flags);
/* probs: host array, read and updated.  Matrices must not overlap each other
   or the workspace (the latter is checked).  flags: SVD2_KOG_GRAPH, with at
   most one of SVD2_KOG_TWO_STEP and SVD2_KOG_THREE_STEP (both:
   SVD2_ERR_FLAGS). */
svd2_status kog_batch_solve(int nprob, kog_problem *probs, void *ws, size_t ws_bytes, unsigned flags,
                            hipStream_t stream);

/* Singular values of a Kogbetliantz iterate (section 1: the iteration drives
 * A towards U* A V = diag(sigma)): sigma_out[0..N) = |a_ii| sorted
 * into descending order (after at least one step the diagonal is real and
 * non-negative, so these are the diagonal entries themselves; after
 * convergence they are the singular values of the input, the diagonal of
 * U* A V).  A: device, column-major, lda >= N (complex interleaved, read
 * only); sigma_out: device, N elements of the real type; ws: device scratch
 * of kog_sigma_workspace_bytes(N, dtype) bytes, 256-byte aligned.  A,
 * sigma_out and ws must not overlap (SVD2_ERR_ALIAS).  Asynchronous on
 * `stream` (a bitonic sorting network on the device). */
size_t kog_sigma_workspace_bytes(int N, int dtype);
svd2_status dkog_sigma(int N, const double *A, int lda, double *sigma_out, void *ws, size_t ws_bytes,
                       hipStream_t stream);
svd2_status zkog_sigma(int N, const double *A, int lda, double *sigma_out, void *ws, size_t ws_bytes,
                       hipStream_t stream);
svd2_status skog_sigma(int N, const float *A, int lda, float *sigma_out, void *ws, size_t ws_bytes,
                       hipStream_t stream);
svd2_status ckog_sigma(int N, const float *A, int lda, float *sigma_out, void *ws, size_t ws_bytes,
                       hipStream_t stream);

/* ---------------------------------------------------------------------------
 * SVD of a square matrix, A_0 = U diag(sigma) V^*, by the Kogbetliantz method
 * with the transformations accumulated (section 1: each step updates the
 * iterate by U_k^* from the left and V_k from the right, so with U <- U U_k
 * and V <- V V_k from U = V = I the identity A_0 = U A V^* holds throughout).
 * Each accumulation rotates the column pair (p, q) of U or V with the
 * rounding order of the column half of the block update.  The iteration,
 * ordering, stopping rule and scaling are those of *_solve, except that at
 * least one sweep is always done, so every diagonal entry of the final
 * iterate is a singular value of a pivot block (real, >= 0).  On return:
 *   sigma[0..N): that diagonal in descending order, equal values by
 *     increasing index (device, N elements of the real type);
 *   U, V: N x N, column-major, leading dimensions ldu, ldv >= N (complex
 *     interleaved), columns permuted alike, so A_0 ~ U diag(sigma) V^*;
 *   A: the final iterate (unsorted).
 * ws: kog_svd_workspace_bytes(N, dtype, flags) bytes, 256-byte aligned (the
 * solve's workspace plus two N x N matrices, the sort keys and, two or three
 * steps per pass, two or nine more rotation sets).  A, U, V,
 * sigma and ws must be pairwise disjoint (SVD2_ERR_ALIAS).  flags: 0 or
 * SVD2_KOG_TWO_STEP (two steps per pass over A; U and V are taken four steps
 * further per pass after every second pass, alternating with workspace
 * copies), SVD2_KOG_THREE_STEP (three steps per pass over A; U and V six
 * steps further after every second pass, on a second stream that the call
 * creates, forks from `stream` by events and joins back before it returns,
 * and destroys), SVD2_KOG_UNFUSED (one step per
 * pass, U and V rotated in place) or SVD2_KOG_UNFUSED | SVD2_KOG_GRAPH;
 * anything else is SVD2_ERR_FLAGS.  Every mode gives bitwise the same
 * results.  max_sweeps >= 1 (SVD2_ERR_SIZE).  Returns SVD2_OK or
 * SVD2_NOT_CONVERGED (outputs as above for the last iterate); synchronises
 * `stream` like *_solve.
 * kog_svd_workspace_bytes returns 0 for an order, element type or flags
 * these entry points do not accept.
 * ------------------------------------------------------------------------- */
size_t kog_svd_workspace_bytes(int N, int dtype, unsigned flags);
svd2_status dkog_svd(int N, double *A, int lda, double *U, int ldu, double *V, int ldv, double *sigma,
                     double tol, int max_sweeps, int *sweeps, double *off_rel, void *ws, size_t ws_bytes,
                     unsigned flags, hipStream_t stream);
svd2_status zkog_svd(int N, double *A, int lda, double *U, int ldu, double *V, int ldv, double *sigma,
                     double tol, int max_sweeps, int *sweeps, double *off_rel, void *ws, size_t ws_bytes,
                     unsigned flags, hipStream_t stream);
svd2_status skog_svd(int N, float *A, int lda, float *U, int ldu, float *V, int ldv, float *sigma,
                     double tol, int max_sweeps, int *sweeps, double *off_rel, void *ws, size_t ws_bytes,
                     unsigned flags, hipStream_t stream);
svd2_status ckog_svd(int N, float *A, int lda, float *U, int ldu, float *V, int ldv, float *sigma,
                     double tol, int max_sweeps, int *sweeps, double *off_rel, void *ws, size_t ws_bytes,
                     unsigned flags, hipStream_t stream);

/* last hipError_t seen by a Kogbetliantz entry point on this thread */
int kog_last_hip_error(void);
/* Workgroups per CU of the fused kernel's cooperative grid, 1..16 (capped by
   the kernel's occupancy); a tuning knob, default 1.  SVD2_ERR_SIZE if out of
   range. */
svd2_status kog_set_fused_blocks_per_cu(int per_cu);
/* Diagnostic: one cooperative launch of `blocks` workgroups of the fused
   kernel's size that pass nbar grid barriers (the fused kernel's barrier) and
   do nothing else, so that (time - time with nbar = 0) / nbar is the cost of
   one barrier.  violations: optional device counter (the caller zeroes it);
   when not NULL the barrier is checked by its epoch counters -- after barrier
   e every workgroup reads every workgroup's published epoch, which must be at
   least e -- and each one found behind, and each aborted wait, adds 1 (0 for
   a correct barrier).  ws: device, >= 256 + 4096 * 64 bytes, 256-byte aligned.
   SVD2_ERR_SIZE if blocks exceeds 4096 or what the GPU holds at once, nbar < 0
   or ws_bytes is short.  Asynchronous on `stream`; spins are bounded as in the
   fused kernel. */
svd2_status kog_barrier_probe(int nbar, int blocks, unsigned *violations, void *ws, size_t ws_bytes,
                              hipStream_t stream);
/* Update-tile shapes by order (set by the autotuner): for an order N the
   first rule i with N <= max_order[i] applies; a tile covers kc[i] row pairs
   (64, 128 or 256) and lc[i] column pairs (1..4096) on one 256-thread
   workgroup.  max_order must increase.  count == 0 restores the default
   (kc 256, lc 8 for every order).  Host arrays, copied; safe to call while
   other threads launch; affects later calls. */
svd2_status kog_set_tile_rules(int count, const int *max_order, const int *kc, const int *lc);

/* Workgroup shapes of the two-step kernel (SVD2_KOG_TWO_STEP), by order: the
 * first rule with N <= max_order[i] applies.  wpg[i] in {1, 2, 4} wavefronts
 * per workgroup; all of them share one block of 62 row pairs.  lc[i] in
 * [2, 64] fixes the column pairs each wavefront writes; lc[i] in [-3, 0]
 * sizes the column split so that the grid fills 1 - lc[i] whole rounds of
 * the workgroups the GPU holds at once.  count = 0 restores the default
 * (4, 8).  Host arrays, copied; safe to call while other threads launch
 * (the tables are guarded); affects later calls. */
svd2_status kog_set_two_step_tiles(int count, const int *max_order, const int *wpg, const int *lc);

/* Workgroup shapes of the three-step kernel (SVD2_KOG_THREE_STEP), by order:
 * the first rule with N <= max_order[i] applies.  wpg[i] in {1, 2, 4}
 * wavefronts per workgroup, each on its own block of 60 row pairs; lc[i] in
 * [2, 128] output column pairs per workgroup, shared by its wavefronts, or
 * lc[i] in [-3, 0]: as many as make the grid fill 1 - lc[i] whole rounds of
 * the workgroups the GPU holds at once.  count = 0 restores the default
 * (1, 0).  Host arrays, copied; safe to call while other threads launch;
 * affects later calls. */
svd2_status kog_set_three_step_tiles(int count, const int *max_order, const int *wpg, const int *lc);

#ifdef __cplusplus
}
#endif
#endif /* SVD2_H */
