/*
 * bed_oracle.h -- binary64 CPU oracle for batched symmetric eigendecomposition
 * by Householder tridiagonalization and the batch-efficient divide-and-conquer
 * of Y. Song, "A Short Note on Batch-efficient Divide-and-Conquer Algorithm for
 * EigenDecomposition" (arXiv 2604.27325).
 *
 * TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only the test-suite, the smoke check
 * and the CPU-baseline leg of the benchmark may build, load or call anything in
 * this directory.  It shares no source, header, table or helper with the GPU
 * library; the two are compared only through their outputs.
 *
 * Conventions (all functions):
 *   - matrices are dense row-major n x n binary64; only the lower triangle of a
 *     symmetric input is read (LAPACK uplo='L');
 *   - Q[i*n+j] is component i of eigenvector j; eigenvalues ascending;
 *   - every eigenvector column is sign-canonical: its largest-magnitude entry
 *     is positive (lowest index on exact ties);
 *   - return value / info: 0 ok, -1 non-finite input (outputs NaN),
 *     k > 0 = k secular roots stopped at the iteration cap.
 */
#ifndef BED_ORACLE_H
#define BED_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Counters filled by the divide-and-conquer (may be NULL). */
typedef struct {
    int64_t merges;        /* rank-one merges performed                     */
    int64_t roots;         /* secular roots solved                          */
    int64_t evals;         /* secular-function evaluations (all phases)     */
    int64_t halley;        /* Halley steps taken                            */
    int64_t capped;        /* roots that hit the iteration cap              */
    int64_t defl_type1;    /* components deflated because rho*|z_i| <= tol  */
    int64_t defl_type2;    /* components deflated by a Givens rotation      */
} orc_stats;

/* Householder reduction A = Q_H T Q_H^T (textbook; Sec. 2 defers the batched
 * reflection to the author's earlier work).  a[n] diagonal, b[n-1]
 * subdiagonal, V[n*n] with reflector k in column k (V[(k+1)*n+k] = 1, zero
 * above), tau[n-2] (tau = 0 means "no reflection").  Q_H = H_0 H_1 ... H_{n-3},
 * H_k = I - tau_k v_k v_k^T.  Returns 0. */
int orc_tridiag(int n, const double *A, double *a, double *b, double *V, double *tau);

/* Eigendecomposition of the symmetric tridiagonal (a, b) by the divide step
 * (Sec. 2.1, Eq. (1)-(3)), 2x2 Givens leaves (Sec. 2.2) and the conquer step
 * (Sec. 2.3).  lam[n] ascending, Q[n*n] (NOT sign-canonicalized).  Returns the
 * number of capped roots. */
int orc_tridiag_eig(int n, const double *a, const double *b, double *lam, double *Q,
                    orc_stats *st);

/* One rank-one eigenproblem D + rho z z^T (Sec. 2.3, Eq. (4)-(25)) with the
 * same sorting, deflation, secular solver and Loewner eigenvectors as a merge.
 * d, z of length m in any order, rho >= 0.  lam[m] ascending, U[m*m] columns
 * are eigenvectors.  ub_frob > 0 adds the Frobenius upper bound of Eq. (10)-(11)
 * (pass 0 to use only d_max + rho z^T z).  Returns capped-root count. */
int orc_rank1_eig(int m, const double *d, const double *z, double rho, double ub_frob,
                  double *lam, double *U, orc_stats *st);

/* Secular solver alone (Sec. 2.3.1-2.3.4): d[k] strictly ascending, z[k]
 * nonzero, rho > 0.  For root j it returns the origin pole index origin[j]
 * and the offset tau[j] (lambda_j = d[origin[j]] + tau[j]); lam[j] is that sum.
 * ub > 0 caps the top root's offset from d[k-1].  iters[j] (may be NULL)
 * receives the evaluations spent on root j.  Returns capped-root count. */
int orc_secular(int k, const double *d, const double *z, double rho, double ub,
                double *lam, int *origin, double *tau, int *iters);

/* Gu-Eisenstat recomputed z (Sec. 2.3.5, Eq. (25)) from the roots in
 * (origin, tau) form; zsign supplies the signs.  zhat[k]. */
void orc_lowner(int k, const double *d, const double *zsign, double rho,
                const int *origin, const double *tau, double *zhat);

/* Deflation (not in the paper; Dongarra-Sorensen type 1 and type 2 with
 * tol = 8u max(max|d|, rho z^T z)).  In/out: d[m] ascending, z[m]; G[m*m]
 * receives the accumulated rotation (columns = new basis in the old one).
 * flag[m] = 1 for deflated components.  Returns the tolerance used. */
double orc_deflate(int m, double *d, double *z, double rho, double *G, int *flag,
                   orc_stats *st);

/* Full path for one matrix: Householder, divide-and-conquer, back-transform,
 * sign canonicalization.  Returns info (0, -1, or capped-root count). */
int orc_syevd(int n, const double *A, double *lam, double *Q, orc_stats *st);

/* Packed batch: matrix b starts at sum_{c<b} n_c^2, lam_b at sum_{c<b} n_c.
 * info[b] as for orc_syevd.  Returns the number of matrices with info != 0. */
int64_t orc_syevd_batch(int64_t batch, const int32_t *n, const double *A, double *lam,
                        double *Q, int32_t *info, orc_stats *st);

/* Backward of A = Q diag(lam) Q^T:
 *   dA = Q ( diag(dlam) + sym(F o (Q^T dQ)) ) Q^T,  F_ij = 1/(lam_j - lam_i),
 * F_ij = 0 when |lam_i - lam_j| <= eps * max(1, max|lam|) (and on i = j);
 * sym(X) = (X + X^T)/2.  dlam or dQ may be NULL (= zero).  dA[n*n]. */
void orc_syevd_backward(int n, const double *lam, const double *Q, const double *dlam,
                        const double *dQ, double eps, double *dA);

#ifdef __cplusplus
}
#endif
#endif
