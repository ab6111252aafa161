/*
 * svd2_oracle.h -- plain, slow CPU oracle for the batched 2x2 SVD.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this code; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no source with the GPU path.
 *
 * Source: V. Novakovic, "Batched computation of the singular value
 * decompositions of order two by the AVX-512 vectorization" (arXiv:2005.07403).
 * Every step is written per matrix, in the paper's order (section 2 for the
 * mathematics, sections 5-7 for the operation order), with correctly rounded
 * IEEE-754 basic operations (+, -, *, /, sqrt, fma, ldexp).
 *
 * Data layout (section 3): structure of arrays, one array per matrix element
 * and per real/imaginary part, in the record order of section 8:
 *   real:    a11, a21, a12, a22
 *   complex: a11r, a11i, a21r, a21i, a12r, a12i, a22r, a22i
 * Outputs, in the same element order:
 *   real:    u11,u21,u12,u22, v11,v21,v12,v22, smax, smin, s        (11 arrays)
 *   complex: u11r,u11i,...,u22i, v11r,...,v22i, smax, smin, s      (19 arrays)
 * smax/smin are the scaled singular values sigma' of eq. (12) and s is the
 * exponent of eq. (2), stored in the element type (BIG for a zero matrix, -0
 * after a backscale as in Fig. 1).
 */
#ifndef SVD2_ORACLE_H
#define SVD2_ORACLE_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* hypot / invsqrt policy (the paper fixes only their contract, section 2) */
enum { ORACLE_REF = 0,    /* hypot and 1/sqrt correctly rounded via __float128 */
       ORACLE_MIRROR = 1  /* hypot = the division-based fallback of section 5,
                             invsqrt = 1/sqrt(x): two correctly rounded ops    */ };

/* OR-ed into the policy argument of the batched entry points: assemble U by
 * the sine form of eq. (31) (sin = cos * tan, section 7) instead of the
 * tangent form of eq. (29); V is the same in both.  Pinned: the two forms give
 * U within a few eps of each other (two formulas of one matrix) and the sine
 * form's residual and orthogonality within 16 eps in binary128. */
enum { ORACLE_SINE = 16 };

/* backscale mode of eq. (28) */
enum { ORACLE_BS_NONE = 0, /* write sigma' and s (the paper's default)          */
       ORACLE_BS_SAFE = 1, /* per lane, only if 2^-s sigma' is exact and finite */
       ORACLE_BS_ALL = 2   /* Fig. 1: unconditional                             */ };

/* Batched SVD over n matrices.  in/out are arrays of host pointers as above.
 * rescue (float only): 0 = plain FP32 algorithm; 1 = recompute R's (2,2)
 * entry from det(A^) in FP64 on lanes with smin' < 2^-20 smax', then run the
 * triangular SVD and the assembly of U, V in FP64 for those lanes; 2 = on
 * those lanes only smin' = |det(A^)| / smax' in FP64 (U, V stay FP32); 3 = on
 * those lanes R's (2,2) entry, its phase and the triangular SVD in FP64, whose
 * tangents, cosines, phase and sigma' are rounded to FP32, and U, V assembled
 * in FP32 from them by the plain formulas.
 * flagged (optional, may be NULL): per-lane 0/1 marks of rescued lanes.
 * nthreads <= 0: use the OpenMP default.  Returns 0. */
int oracle_dsvd2(size_t n, const double *const *in, double *const *out,
                 int policy, int backscale, int nthreads);
int oracle_zsvd2(size_t n, const double *const *in, double *const *out,
                 int policy, int backscale, int nthreads);
int oracle_ssvd2(size_t n, const float *const *in, float *const *out,
                 int policy, int backscale, int rescue, uint8_t *flagged,
                 int nthreads);
int oracle_csvd2(size_t n, const float *const *in, float *const *out,
                 int policy, int backscale, int rescue, uint8_t *flagged,
                 int nthreads);

/* Intermediates of one matrix, for the invariant tests of Theorem 1.
 * Layout of trace[ORACLE_TRACE_LEN] (doubles, float results widened):
 *  0 s      1 c(col swap)  2 r(row swap)  3 r11   4 r12   5 r22
 *  6 mt(=-tan alpha)      7 cos alpha     8 x     9 y    10 tan 2phi
 * 11 tan phi 12 sec^2 phi 13 cos phi     14 tan psi 15 sec^2 psi 16 cos psi
 * 17 smax'  18 smin'  19 n1 (first column norm after pivoting) 20 n2
 * 21 rescued (float only) */
#define ORACLE_TRACE_LEN 22
int oracle_trace_d(const double *a, int cplx, int policy, double *trace);

/* Phase outputs of the URV factorization, section 2.2 (section 4: the output
 * of a phase may be written alongside the final results, in the same
 * layout), for the same pipeline as oracle_dsvd2 ... oracle_csvd2:
 *   R = [[r11, r12], [0, r22]] of eq. (9), real, of A^ = 2^s A;
 *   U_+ = P_r D Q_alpha D^ and V_+ = P_c D~, the unitary factors of eq. (11)
 *   (A^ = U_+ R V_+^*), with D = diag(d1, d2) the conjugate of D* (eq. (4)),
 *   Q_alpha = cos(alpha) [[1, -mt], [mt, 1]] (eq. (6), tan(alpha) = -mt),
 *   D^ = diag(1, dh) (dh = e^{i arg r'_22}, eq. (9)) and D~ = diag(1,
 *   conj(e12)) (e12 = e^{i arg r'_12}, eq. (8)); in the real case d1, d2, dh
 *   and e12 are the signs +-1 of eq. (10).
 * Reading (the paper gives no operation order for U_+): with ca = cos(alpha)
 * and sa = ca * mt (one rounding), before the row swap P_r
 *   u11 = d1 ca, u21 = d2 sa, u12 = -((d1 dh) sa), u22 = (d2 dh) ca,
 * each real-by-complex product one rounding per part and d1 dh, d2 dh by
 * eq. (5); V_+ before the row swap P_c is [[1, 0], [0, conj(e12)]] exactly.
 * f: r11, r12, r22, then U_+ and V_+ in the element order of U and V
 * (11 arrays real, 19 complex).  FP32: the FP32 pipeline's values (no rescue
 * is applied to them).  Returns 0. */
int oracle_urv_d(size_t n, int cplx, const double *const *in, double *const *f, int policy,
                 int nthreads);
int oracle_urv_s(size_t n, int cplx, const float *const *in, float *const *f, int policy,
                 int nthreads);
int oracle_trace_s(const float *a, int cplx, int policy, int rescue, double *trace);

/* Error metrics of section 8, eqs. (32)-(35), per lane, in __float128.
 * sigma = 2^-s sigma' is formed exactly in quad precision.
 * Results (rounded to double): kappa, rho, delta, eta (arrays of n). */
int oracle_metrics_d(size_t n, int cplx, const double *const *in,
                     const double *const *out, double *kappa, double *rho,
                     double *delta, double *eta, int nthreads);
int oracle_metrics_s(size_t n, int cplx, const float *const *in,
                     const float *const *out, double *kappa, double *rho,
                     double *delta, double *eta, int nthreads);


/* ---------------------------------------------------------------------------
 * Kogbetliantz method for the SVD of a square matrix of even order N = 2n
 * (section 1): a step gathers the pivots (p,p), (q,p), (p,q), (q,q) of n
 * disjoint pairs, computes their 2x2 SVDs (backscaled, Sigma = 2^-s Sigma'),
 * updates rows p,q by U_k^* and columns p,q by V_k, and writes
 * diag(sigma_max, sigma_min) with exact zeros into each pivot block.
 * The pivot ordering is not given by the paper; this is the circle-method
 * round robin: at step t (0 <= t < N-1) pair 0 is (t, N-1) and pair k >= 1 is
 * ((t+k) mod (N-1), (t-k) mod (N-1)), each oriented so that p < q.
 * Matrices are column-major with leading dimension lda; complex matrices are
 * interleaved (re, im) per element, lda counted in complex elements.
 * Block update order: T = U^* B first (rows), then T V (columns):
 *   real:    T1j = fma(u11, b1j, u21*b2j), T2j = fma(u12, b1j, u22*b2j),
 *            Bi1 = fma(Ti1, v11, Ti2*v21), Bi2 = fma(Ti1, v12, Ti2*v22)
 *   complex: T1j = conj(u11) b1j + conj(u21) b2j (each product as eq. (5)),
 *            Bi1 = Ti1 v11 + Ti2 v21, Bi2 = Ti1 v12 + Ti2 v22.
 * Pivot placement (reading): if |b_pp| < |b_qq| the columns of U_k and V_k
 * and the two singular values are swapped (sigma_min goes to (p,p)); with the
 * descending order of Theorem 1 alone the iteration converges only linearly.
 * FP32 matrices use the FP32 2x2 SVD with the FP64 rescue of near-degenerate
 * pivots.  Stopping rule: off(A) = sqrt(sum_{i != j} |a_ij|^2) below
 * tol * ||A_0||_F, tested before every sweep; a sweep is N-1 steps.  The solve
 * multiplies A by 2^-E before the first sweep and by 2^E after the last (E =
 * the largest binary exponent among its components), which changes no
 * rounding but keeps the sums of squares of the stopping test finite and
 * nonzero for any finite A.
 * ------------------------------------------------------------------------- */
int oracle_kog_pairs(int N, int t, int *pairs /* n x 2, row-major */);
int oracle_kog_step_d(int N, double *A, int lda, int t);
int oracle_kog_step_z(int N, double *A, int lda, int t);
int oracle_kog_step_s(int N, float *A, int lda, int t);
int oracle_kog_step_c(int N, float *A, int lda, int t);
/* off^2 and ||A||_F^2, accumulated in FP64 */
int oracle_kog_norms_d(int N, const double *A, int lda, int cplx, double *off2, double *tot2);
int oracle_kog_norms_s(int N, const float *A, int lda, int cplx, double *off2, double *tot2);
/* Full solve: returns 0 on convergence, 7 when max_sweeps is reached.
 * sweeps: sweeps performed; off_rel: off(A)/||A_0||_F at exit;
 * history (optional, max_sweeps+1 doubles): off/||A_0||_F before each sweep.
 * Pinned by the tests: every step keeps ||A||_F and lowers off(A)^2 by the
 * pivots' off-diagonal mass, and the converged diagonal matches an
 * independent SVD within 8 N eps sigma_max.  Parity unpinned: the number of
 * sweeps itself (the paper fixes neither the ordering nor the stopping rule,
 * so nothing outside this code determines it). */
int oracle_kog_solve_d(int N, double *A, int lda, double tol, int max_sweeps, int *sweeps,
                       double *off_rel, double *history);
int oracle_kog_solve_z(int N, double *A, int lda, double tol, int max_sweeps, int *sweeps,
                       double *off_rel, double *history);
int oracle_kog_solve_s(int N, float *A, int lda, double tol, int max_sweeps, int *sweeps,
                       double *off_rel, double *history);
int oracle_kog_solve_c(int N, float *A, int lda, double tol, int max_sweeps, int *sweeps,
                       double *off_rel, double *history);
/* SVD A_0 = U diag(sigma) V^* with the transformations of every step
 * accumulated (section 1: the iterate is updated by U_k^* from the left and
 * V_k from the right, so A_0 = (prod U_k) A (prod V_k)^*): U = V = I, then
 * each step also applies [x_.p, x_.q] <- [x_.p, x_.q] U_k to U and V_k to V,
 * with the rounding order of the column half of the block update.  At least
 * one sweep is done, so the final diagonal holds pivot singular values (real,
 * >= 0); sigma = that diagonal in descending order, equal values by
 * increasing index, and the columns of U and V permuted alike.  A keeps the
 * final iterate; U, V are N x N column-major with leading dimensions ldu,
 * ldv (complex interleaved); cplx selects complex data.  Returns 0, 7 (max
 * sweeps reached) or 6 (max_sweeps < 1).  Pinned against the definition of
 * the SVD and LAPACK: reconstruction and unitarity within a small multiple of
 * S N^1.5 eps, sigma within 8 N eps sigma_max, singular vectors of separated
 * singular values to 1e-11, exact signed permutations for a real diagonal
 * matrix, the iterate equal to the solve's. */
int oracle_kog_svd_d(int N, double *A, int lda, double *U, int ldu, double *V, int ldv,
                     double *sigma, int cplx, double tol, int max_sweeps, int *sweeps,
                     double *off_rel);
int oracle_kog_svd_s(int N, float *A, int lda, float *U, int ldu, float *V, int ldv, float *sigma,
                     int cplx, double tol, int max_sweeps, int *sweeps, double *off_rel);

#ifdef __cplusplus
}
#endif
#endif
