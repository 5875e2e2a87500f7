/*
 * bed_oracle.c -- binary64 CPU oracle (TEST INFRASTRUCTURE ONLY; see the
 * header).  Plain and slow on purpose: every step follows the text of
 * Y. Song, "A Short Note on Batch-efficient Divide-and-Conquer Algorithm for
 * EigenDecomposition" (arXiv 2604.27325), or, where that note defers or is
 * silent, the textbook method named at the step.  No blocking, no fusion, no
 * reordering beyond what the method states.
 *
 * Readings taken where the note is silent or inconsistent (also listed in the
 * design notes of the repository):
 *   R-z     Eq. (5): z is sigma*(last row of Q1) over (first row of Q2), with
 *           sigma = sgn(beta); the block-diagonal product printed in Eq. (5)
 *           is read as the transposed blocks.
 *   R-rho   Eq. (12), (18), (21): rho = |beta| everywhere (Eq. (8) form).
 *   R-int   Eq. (9)-(11): ascending indexing d_1 < lam_1 < d_2 < ... < d_k <
 *           lam_k; no definiteness is assumed; the top root is bounded by
 *           min(d_k + rho z^T z, ||T_node||_F) (Eq. (10)), the Frobenius bound
 *           used only when the secular function confirms it.
 *   R-init  Eq. (13): the first estimate is the midpoint of the root's own
 *           bracket (one bisection step, Eq. (14)-(15)); its sign decides
 *           the nearer pole, which becomes the origin of the shifted variable
 *           tau = lambda - d_origin; all differences are formed as
 *           delta_i = (d_i - d_origin) - tau.
 *   R-multi Eq. (16): multi-section probes origin_end +/- (U-L)/4 (k = 4 sections)
 *           toward the origin pole, at most 3 probes, while the bracket is
 *           wider than 1e-2 of the initial one (Eq. (17) epsilon).
 *   R-halley Eq. (20): Halley from the bracket midpoint; a step that leaves the
 *           bracket or has a non-positive denominator is replaced by bisection;
 *           the bracket is updated by Eq. (14) after every evaluation.
 *   R-stop  Eq. (17)/(22) tolerances: a root stops when |f| <= 8u(1 + rho
 *           sum|z_i^2/delta_i|) or the bracket has no interior float; cap 100.
 *   R-zhat  Eq. (25): zhat_i takes the sign of z_i; evaluated as a product of
 *           positive ratios.
 *   R-vec   Eq. (23)-(24) are applied with zhat (the note recomputes z first).
 *   R-defl  deflation (absent from the note): type 1 rho|z_i| <= tol, type 2
 *           Givens when |(d_j - d_i) c s| <= tol, tol = 8u max(max|d|, rho z^T z).
 *   R-tree  Sec. 2.1 split points: node j of depth d covers [floor(j n/2^d),
 *           floor((j+1) n/2^d)); nodes of size <= 2 are leaves (Sec. 2.2,
 *           Givens 2x2), larger nodes split at their dyadic midpoint.
 *   R-house Householder (deferred by the note): alpha = -sgn(x0)||x||,
 *           sgn(0) = +1, tau = 0 when x(2:end) = 0 (Golub-Van Loan Sec. 8.3).
 */
#include "bed_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define U_F64 0x1p-53 /* unit roundoff of binary64 */
#define SEC_CAP 100   /* iteration cap per secular root */

static double sgn1(double x) { return x < 0.0 ? -1.0 : 1.0; }

static void *xcalloc(size_t count, size_t size)
{
    void *p = calloc(count ? count : 1, size);
    if (!p) abort();
    return p;
}

#define STAT(st, f, v)          \
    do {                         \
        if (st) (st)->f += (v);  \
    } while (0)

/* ------------------------------------------------------------------------ */
/* Householder tridiagonalization (Golub & Van Loan, Sec. 8.3.1; the note     */
/* defers the batched reflection to its predecessor).                         */
/* ------------------------------------------------------------------------ */
int orc_tridiag(int n, const double *A, double *a, double *b, double *V, double *tau)
{
    double *W = xcalloc((size_t)n * n, sizeof(double));
    double *p = xcalloc(n, sizeof(double));
    double *w = xcalloc(n, sizeof(double));
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) W[i * n + j] = (j <= i) ? A[i * n + j] : A[j * n + i];
    memset(V, 0, sizeof(double) * (size_t)n * n);

    for (int k = 0; k + 2 < n; ++k) {
        a[k] = W[k * n + k];
        double x0 = W[(k + 1) * n + k];
        double sig = 0.0; /* ||x(2:end)||^2 */
        for (int i = k + 2; i < n; ++i) sig += W[i * n + k] * W[i * n + k];
        V[(k + 1) * n + k] = 1.0;
        if (sig == 0.0) {
            tau[k] = 0.0;
            b[k] = x0;
            continue;
        }
        double alpha = -sgn1(x0) * sqrt(x0 * x0 + sig);
        double v0 = x0 - alpha;
        for (int i = k + 2; i < n; ++i) V[i * n + k] = W[i * n + k] / v0;
        double t = (alpha - x0) / alpha; /* = 2 / (v^T v) */
        tau[k] = t;
        b[k] = alpha;
        /* p = tau W' v ; w = p - (tau/2)(p^T v) v ; W' -= v w^T + w v^T */
        for (int i = k + 1; i < n; ++i) {
            double s = 0.0;
            for (int j = k + 1; j < n; ++j) s += W[i * n + j] * V[j * n + k];
            p[i] = t * s;
        }
        double pv = 0.0;
        for (int i = k + 1; i < n; ++i) pv += p[i] * V[i * n + k];
        for (int i = k + 1; i < n; ++i) w[i] = p[i] - 0.5 * t * pv * V[i * n + k];
        for (int i = k + 1; i < n; ++i)
            for (int j = k + 1; j < n; ++j)
                W[i * n + j] -= V[i * n + k] * w[j] + w[i] * V[j * n + k];
    }
    if (n >= 2) {
        a[n - 2] = W[(n - 2) * n + n - 2];
        b[n - 2] = W[(n - 1) * n + n - 2];
    }
    a[n - 1] = W[(n - 1) * n + n - 1];
    free(W);
    free(p);
    free(w);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* 2x2 leaf by one Givens/Jacobi rotation (Sec. 2.2; Golub & Van Loan,       */
/* Alg. 8.5.1 "symmetric Schur decomposition").  lam ascending; Q columns.   */
/* ------------------------------------------------------------------------ */
static void leaf2(double p, double q, double r, double lam[2], double Q[4])
{
    double c = 1.0, s = 0.0, t = 0.0;
    if (q != 0.0) {
        double th = (r - p) / (2.0 * q);
        t = sgn1(th) / (fabs(th) + hypot(1.0, th));
        c = 1.0 / hypot(1.0, t);
        s = t * c;
    }
    /* J = [c s; -s c], J^T [p q; q r] J = diag(p - t q, r + t q) */
    double l1 = p - t * q, l2 = r + t * q;
    if (l1 <= l2) {
        lam[0] = l1; lam[1] = l2;
        Q[0] = c;  Q[1] = s;
        Q[2] = -s; Q[3] = c;
    } else {
        lam[0] = l2; lam[1] = l1;
        Q[0] = s; Q[1] = c;
        Q[2] = c; Q[3] = -s;
    }
}

/* ------------------------------------------------------------------------ */
/* Secular function (Eq. (8)) and its derivatives (Eq. (18), (21)) in the     */
/* shifted variable tau = lambda - d_o: delta_i = (d_i - d_o) - tau.          */
/* ------------------------------------------------------------------------ */
typedef struct {
    double f, f1, f2, ebound;
} sec_val;

static sec_val sec_eval(int k, const double *d, const double *z, double rho, int o,
                        double tau)
{
    sec_val v = {1.0, 0.0, 0.0, 0.0};
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, e = 0.0;
    for (int i = 0; i < k; ++i) {
        double del = (d[i] - d[o]) - tau;
        double t = z[i] * z[i] / del;
        s0 += t;
        s1 += t / del;
        s2 += t / del / del;
        e += fabs(t);
    }
    v.f = 1.0 + rho * s0;
    v.f1 = rho * s1;
    v.f2 = 2.0 * rho * s2;
    v.ebound = 8.0 * U_F64 * (1.0 + rho * e);
    return v;
}

/* Bracket update of Eq. (14): f > 0 means the estimate is above the root. */
static void bracket_update(double f, double h, double *L, double *U)
{
    if (f > 0.0)
        *U = h;
    else
        *L = h;
}

/* One root of the secular equation (Sec. 2.3.1-2.3.3): j in [0,k). */
static int solve_root(int k, const double *d, const double *z, double rho, double ub,
                      int j, int *origin, double *tau_out, int *evals_out, int *halley_out)
{
    int evals = 0, halley = 0, o;
    double L, U, w0;
    double zz = 0.0;
    for (int i = 0; i < k; ++i) zz += z[i] * z[i];

    /* Bounded interlacing, Eq. (11): bracket of root j in the original variable. */
    if (j < k - 1) {
        double gap = d[j + 1] - d[j];
        double mid = 0.5 * gap; /* initial estimate, Eq. (13) (own bracket) */
        sec_val v = sec_eval(k, d, z, rho, j, mid);
        ++evals;
        if (v.f == 0.0) {
            *origin = j;
            *tau_out = mid;
            *evals_out = evals;
            *halley_out = 0;
            return 0;
        }
        if (v.f > 0.0) { /* root in (d_j, mid): origin d_j */
            o = j;
            L = 0.0;
            U = mid;
        } else { /* root in (mid, d_{j+1}): origin d_{j+1} */
            o = j + 1;
            L = mid - gap;
            U = 0.0;
        }
        w0 = gap;
    } else {
        o = j;
        double top = rho * zz;
        if (ub > 0.0 && ub < top) {
            sec_val vb = sec_eval(k, d, z, rho, o, ub);
            ++evals;
            if (vb.f >= 0.0) top = ub; /* Frobenius bound confirmed */
        }
        double mid = 0.5 * top;
        sec_val v = sec_eval(k, d, z, rho, o, mid);
        ++evals;
        if (v.f == 0.0) {
            *origin = o;
            *tau_out = mid;
            *evals_out = evals;
            *halley_out = 0;
            return 0;
        }
        if (v.f > 0.0) {
            L = 0.0;
            U = mid;
        } else {
            L = mid;
            U = top;
        }
        w0 = top;
    }

    /* Multi-section toward the origin pole, Eq. (16)-(17). */
    for (int it = 0; it < 3 && (U - L) > 1e-2 * w0; ++it) {
        double h = (o == j) ? L + 0.25 * (U - L) : U - 0.25 * (U - L);
        sec_val v = sec_eval(k, d, z, rho, o, h);
        ++evals;
        if (v.f == 0.0) {
            *origin = o;
            *tau_out = h;
            *evals_out = evals;
            *halley_out = 0;
            return 0;
        }
        bracket_update(v.f, h, &L, &U);
    }

    /* Safeguarded Halley iteration, Eq. (20)-(21). */
    double h = 0.5 * (L + U);
    int capped = 1;
    for (int it = 0; it < SEC_CAP; ++it) {
        sec_val v = sec_eval(k, d, z, rho, o, h);
        ++evals;
        if (fabs(v.f) <= v.ebound) {
            capped = 0;
            break;
        }
        bracket_update(v.f, h, &L, &U);
        if (U - L <= 2.0 * U_F64 * (fabs(L) + fabs(U))) {
            capped = 0;
            break;
        }
        double den = 2.0 * v.f1 * v.f1 - v.f * v.f2;
        double hn = (den > 0.0) ? h - 2.0 * v.f * v.f1 / den : NAN;
        if (!(hn > L && hn < U)) hn = 0.5 * (L + U);
        else ++halley;
        if (hn == h) {
            capped = 0;
            break;
        }
        h = hn;
    }
    *origin = o;
    *tau_out = h;
    *evals_out = evals;
    *halley_out = halley;
    return capped;
}

static int secular_impl(int k, const double *d, const double *z, double rho, double ub,
                        double *lam, int *origin, double *tau, int *iters, int *halley)
{
    int capped = 0;
    /* Every root is solved independently; the progressive batch shrinkage of
     * Sec. 2.3.4 only stops converged roots early and does not change values. */
    for (int j = 0; j < k; ++j) {
        int ev, hl;
        capped += solve_root(k, d, z, rho, ub, j, &origin[j], &tau[j], &ev, &hl);
        lam[j] = d[origin[j]] + tau[j];
        if (iters) iters[j] = ev;
        if (halley) halley[j] = hl;
    }
    return capped;
}

int orc_secular(int k, const double *d, const double *z, double rho, double ub,
                double *lam, int *origin, double *tau, int *iters)
{
    return secular_impl(k, d, z, rho, ub, lam, origin, tau, iters, NULL);
}

/* Eq. (25): zhat_i^2 = prod_j (lam_j - d_i) / (rho prod_{j!=i} (d_j - d_i)),
 * with lam_j - d_i = -delta_ij and delta_ij = (d_i - d_{o_j}) - tau_j. */
void orc_lowner(int k, const double *d, const double *zsign, double rho,
                const int *origin, const double *tau, double *zhat)
{
    for (int i = 0; i < k; ++i) {
        double p = -((d[i] - d[origin[i]]) - tau[i]) / rho;
        for (int j = 0; j < k; ++j) {
            if (j == i) continue;
            double lam_minus_di = -((d[i] - d[origin[j]]) - tau[j]);
            p *= lam_minus_di / (d[j] - d[i]);
        }
        zhat[i] = copysign(sqrt(p), zsign[i]);
    }
}

/* Deflation (see header).  G starts as identity and accumulates the rotations
 * applied to the basis: new basis column c = sum_r G[r*m+c] old_r. */
double orc_deflate(int m, double *d, double *z, double rho, double *G, int *flag,
                   orc_stats *st)
{
    double dmax = 0.0, zz = 0.0;
    for (int i = 0; i < m; ++i) {
        if (fabs(d[i]) > dmax) dmax = fabs(d[i]);
        zz += z[i] * z[i];
    }
    double tol = 8.0 * U_F64 * fmax(dmax, rho * zz);
    for (int i = 0; i < m * m; ++i) G[i] = 0.0;
    for (int i = 0; i < m; ++i) G[i * m + i] = 1.0;

    for (int i = 0; i < m; ++i) {
        flag[i] = (rho * fabs(z[i]) <= tol);
        if (flag[i]) {
            z[i] = 0.0;
            STAT(st, defl_type1, 1);
        }
    }
    int last = -1;
    for (int i = 0; i < m; ++i) {
        if (flag[i]) continue;
        if (last < 0) {
            last = i;
            continue;
        }
        double r = hypot(z[last], z[i]);
        double c = z[i] / r, s = z[last] / r;
        if (fabs((d[i] - d[last]) * c * s) <= tol) {
            /* rotation in the (last, i) plane that moves z_last into z_i */
            double dl = d[last] * c * c + d[i] * s * s;
            double di = d[last] * s * s + d[i] * c * c;
            d[last] = dl;
            d[i] = di;
            z[last] = 0.0;
            z[i] = r;
            for (int row = 0; row < m; ++row) {
                double gl = G[row * m + last], gi = G[row * m + i];
                G[row * m + last] = c * gl - s * gi;
                G[row * m + i] = s * gl + c * gi;
            }
            flag[last] = 1;
            STAT(st, defl_type2, 1);
        }
        last = i;
    }
    return tol;
}

/* ------------------------------------------------------------------------ */
/* Core of one merge (Sec. 2.3): ds ascending, zs, basis Qs (rows x m, row-   */
/* major, column c = basis vector of sorted component c).  Produces lam[m]    */
/* ascending and Qout (rows x m).                                            */
/* ------------------------------------------------------------------------ */
static int merge_core(int m, int rows, double *ds, double *zs, double rho, double ub,
                      const double *Qs, double *lam, double *Qout, orc_stats *st)
{
    double *G = xcalloc((size_t)m * m, sizeof(double));
    int *flag = xcalloc(m, sizeof(int));
    orc_deflate(m, ds, zs, rho, G, flag, st);

    /* rotated basis B = Qs G */
    double *B = xcalloc((size_t)rows * m, sizeof(double));
    for (int r = 0; r < rows; ++r)
        for (int c = 0; c < m; ++c) {
            double s = 0.0;
            for (int t = 0; t < m; ++t) s += Qs[r * m + t] * G[t * m + c];
            B[r * m + c] = s;
        }

    int k = 0;
    int *nd = xcalloc(m, sizeof(int));
    for (int i = 0; i < m; ++i)
        if (!flag[i]) nd[k++] = i;
    double *dk = xcalloc(m, sizeof(double)), *zk = xcalloc(m, sizeof(double));
    for (int i = 0; i < k; ++i) {
        dk[i] = ds[nd[i]];
        zk[i] = zs[nd[i]];
    }
    double *lk = xcalloc(m, sizeof(double)), *tk = xcalloc(m, sizeof(double));
    double *zh = xcalloc(m, sizeof(double)), *Uk = xcalloc((size_t)m * m, sizeof(double));
    int *ok = xcalloc(m, sizeof(int)), *it = xcalloc(m, sizeof(int));
    int *hl = xcalloc(m, sizeof(int));
    int capped = 0;
    if (k > 0) {
        double ubk = (ub > 0.0) ? ub - dk[k - 1] : 0.0;
        capped = secular_impl(k, dk, zk, rho, ubk, lk, ok, tk, it, hl);
        STAT(st, roots, k);
        STAT(st, capped, capped);
        for (int j = 0; j < k; ++j) {
            STAT(st, evals, it[j]);
            STAT(st, halley, hl[j]);
        }
        orc_lowner(k, dk, zk, rho, ok, tk, zh);
        /* Eq. (23)-(24): u_j = (lam_j I - D)^{-1} zhat, normalized */
        for (int j = 0; j < k; ++j) {
            double nrm = 0.0;
            for (int i = 0; i < k; ++i) {
                double lam_minus_di = -((dk[i] - dk[ok[j]]) - tk[j]);
                Uk[i * k + j] = zh[i] / lam_minus_di;
                nrm += Uk[i * k + j] * Uk[i * k + j];
            }
            nrm = sqrt(nrm);
            for (int i = 0; i < k; ++i) Uk[i * k + j] /= nrm;
        }
    }

    /* Items: roots (in order) and deflated components, then a stable sort of
     * the values gives the output column order (Eq. (4) back-multiplication). */
    double *val = xcalloc(m, sizeof(double));
    int *src = xcalloc(m, sizeof(int)); /* >= 0: deflated position, < 0: -(root+1) */
    int cnt = 0;
    for (int j = 0; j < k; ++j) {
        val[cnt] = lk[j];
        src[cnt++] = -(j + 1);
    }
    for (int i = 0; i < m; ++i)
        if (flag[i]) {
            val[cnt] = ds[i];
            src[cnt++] = i;
        }
    for (int a = 1; a < m; ++a) { /* insertion sort, stable */
        double v = val[a];
        int s = src[a], b2 = a - 1;
        while (b2 >= 0 && val[b2] > v) {
            val[b2 + 1] = val[b2];
            src[b2 + 1] = src[b2];
            --b2;
        }
        val[b2 + 1] = v;
        src[b2 + 1] = s;
    }
    for (int c = 0; c < m; ++c) {
        lam[c] = val[c];
        for (int r = 0; r < rows; ++r) {
            double s;
            if (src[c] >= 0) {
                s = B[r * m + src[c]];
            } else {
                int j = -src[c] - 1;
                s = 0.0;
                for (int i = 0; i < k; ++i) s += B[r * m + nd[i]] * Uk[i * k + j];
            }
            Qout[r * m + c] = s;
        }
    }
    STAT(st, merges, 1);
    free(G); free(flag); free(B); free(nd); free(dk); free(zk); free(lk); free(tk);
    free(zh); free(Uk); free(ok); free(it); free(hl); free(val); free(src);
    return capped;
}

int orc_rank1_eig(int m, const double *d, const double *z, double rho, double ub_frob,
                  double *lam, double *U, orc_stats *st)
{
    int *perm = xcalloc(m, sizeof(int));
    for (int i = 0; i < m; ++i) perm[i] = i;
    for (int a = 1; a < m; ++a) { /* stable insertion sort of d */
        int p = perm[a], b2 = a - 1;
        while (b2 >= 0 && d[perm[b2]] > d[p]) {
            perm[b2 + 1] = perm[b2];
            --b2;
        }
        perm[b2 + 1] = p;
    }
    double *ds = xcalloc(m, sizeof(double)), *zs = xcalloc(m, sizeof(double));
    double *Qs = xcalloc((size_t)m * m, sizeof(double));
    for (int c = 0; c < m; ++c) {
        ds[c] = d[perm[c]];
        zs[c] = z[perm[c]];
        Qs[perm[c] * m + c] = 1.0;
    }
    int capped = merge_core(m, m, ds, zs, rho, ub_frob, Qs, lam, U, st);
    free(perm); free(ds); free(zs); free(Qs);
    return capped;
}

/* ------------------------------------------------------------------------ */
/* Divide-and-conquer over the tearing tree (Sec. 2.1-2.3).                   */
/* ------------------------------------------------------------------------ */
typedef struct {
    int n;
    double *a;   /* diagonal, modified by the tears (Eq. (3)) */
    const double *b;
    double *lam; /* eigenvalues of the current nodes, per node ascending */
    double *Q;   /* n x n, block diagonal over the current nodes */
    orc_stats *st;
    int capped;
} dc_ctx;

static void dc_node(dc_ctx *c, int dep, int j)
{
    int n = c->n;
    int lo = (int)(((long)j * n) >> dep), hi = (int)(((long)(j + 1) * n) >> dep);
    int m = hi - lo;
    if (m == 1) {
        c->lam[lo] = c->a[lo];
        c->Q[lo * n + lo] = 1.0;
        return;
    }
    if (m == 2) {
        double l2[2], q2[4];
        leaf2(c->a[lo], c->b[lo], c->a[lo + 1], l2, q2);
        c->lam[lo] = l2[0];
        c->lam[lo + 1] = l2[1];
        c->Q[lo * n + lo] = q2[0];
        c->Q[lo * n + lo + 1] = q2[1];
        c->Q[(lo + 1) * n + lo] = q2[2];
        c->Q[(lo + 1) * n + lo + 1] = q2[3];
        return;
    }
    int s = (int)(((long)(2 * j + 1) * n) >> (dep + 1));
    /* ||T_node||_F before this node's own tear (bound of Eq. (10)) */
    double fro = 0.0;
    for (int i = lo; i < hi; ++i) fro += c->a[i] * c->a[i];
    for (int i = lo; i + 1 < hi; ++i) fro += 2.0 * c->b[i] * c->b[i];
    fro = sqrt(fro);
    /* Eq. (2)-(3): T = diag(T1^, T2^) + |beta| v v^T, v = [.., sigma, 1, ..] */
    double beta = c->b[s - 1];
    double rho = fabs(beta), sigma = sgn1(beta);
    c->a[s - 1] -= rho;
    c->a[s] -= rho;
    dc_node(c, dep + 1, 2 * j);
    dc_node(c, dep + 1, 2 * j + 1);

    /* Merge setup, Eq. (4)-(5): d = [D1; D2], z = [sigma Q1(last,:); Q2(first,:)] */
    int m1 = s - lo;
    double *d = xcalloc(m, sizeof(double)), *z = xcalloc(m, sizeof(double));
    for (int i = 0; i < m; ++i) {
        d[i] = c->lam[lo + i];
        z[i] = (i < m1) ? sigma * c->Q[(s - 1) * n + lo + i] : c->Q[s * n + lo + i];
    }
    /* stable merge of the two ascending halves */
    int *perm = xcalloc(m, sizeof(int));
    int p1 = 0, p2 = m1, q = 0;
    while (p1 < m1 && p2 < m) perm[q++] = (d[p2] < d[p1]) ? p2++ : p1++;
    while (p1 < m1) perm[q++] = p1++;
    while (p2 < m) perm[q++] = p2++;
    double *ds = xcalloc(m, sizeof(double)), *zs = xcalloc(m, sizeof(double));
    double *Qs = xcalloc((size_t)m * m, sizeof(double));
    for (int t = 0; t < m; ++t) {
        ds[t] = d[perm[t]];
        zs[t] = z[perm[t]];
        for (int r = 0; r < m; ++r) Qs[r * m + t] = c->Q[(lo + r) * n + lo + perm[t]];
    }
    double *lamo = xcalloc(m, sizeof(double)), *Qo = xcalloc((size_t)m * m, sizeof(double));
    c->capped += merge_core(m, m, ds, zs, rho, fro, Qs, lamo, Qo, c->st);
    for (int r = 0; r < m; ++r) {
        c->lam[lo + r] = lamo[r];
        for (int t = 0; t < m; ++t) c->Q[(lo + r) * n + lo + t] = Qo[r * m + t];
    }
    free(d); free(z); free(perm); free(ds); free(zs); free(Qs); free(lamo); free(Qo);
}

int orc_tridiag_eig(int n, const double *a, const double *b, double *lam, double *Q,
                    orc_stats *st)
{
    dc_ctx c;
    c.n = n;
    c.a = xcalloc(n, sizeof(double));
    memcpy(c.a, a, sizeof(double) * n);
    c.b = b;
    c.lam = lam;
    c.Q = Q;
    c.st = st;
    c.capped = 0;
    memset(Q, 0, sizeof(double) * (size_t)n * n);
    dc_node(&c, 0, 0);
    free(c.a);
    return c.capped;
}

/* ------------------------------------------------------------------------ */
/* Full path: Householder, D&C, back-transform Q = H_0 ... H_{n-3} Q_T,      */
/* sign canonicalization.                                                    */
/* ------------------------------------------------------------------------ */
int orc_syevd(int n, const double *A, double *lam, double *Q, orc_stats *st)
{
    if (n <= 0) return 0;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j <= i; ++j)
            if (!isfinite(A[i * n + j])) {
                for (int t = 0; t < n; ++t) lam[t] = NAN;
                for (int t = 0; t < n * n; ++t) Q[t] = NAN;
                return -1;
            }
    double *a = xcalloc(n, sizeof(double)), *b = xcalloc(n, sizeof(double));
    double *V = xcalloc((size_t)n * n, sizeof(double)), *tau = xcalloc(n, sizeof(double));
    orc_tridiag(n, A, a, b, V, tau);
    int capped = orc_tridiag_eig(n, a, b, lam, Q, st);
    for (int k = n - 3; k >= 0; --k) {
        if (tau[k] == 0.0) continue;
        for (int c = 0; c < n; ++c) {
            double s = 0.0;
            for (int r = k + 1; r < n; ++r) s += V[r * n + k] * Q[r * n + c];
            s *= tau[k];
            for (int r = k + 1; r < n; ++r) Q[r * n + c] -= V[r * n + k] * s;
        }
    }
    for (int c = 0; c < n; ++c) {
        int im = 0;
        for (int r = 1; r < n; ++r)
            if (fabs(Q[r * n + c]) > fabs(Q[im * n + c])) im = r;
        if (Q[im * n + c] < 0.0)
            for (int r = 0; r < n; ++r) Q[r * n + c] = -Q[r * n + c];
    }
    free(a); free(b); free(V); free(tau);
    return capped;
}

int64_t orc_syevd_batch(int64_t batch, const int32_t *n, const double *A, double *lam,
                        double *Q, int32_t *info, orc_stats *st)
{
    int64_t offA = 0, offL = 0, bad = 0;
    for (int64_t i = 0; i < batch; ++i) {
        int r = orc_syevd(n[i], A + offA, lam + offL, Q + offA, st);
        if (info) info[i] = r;
        bad += (r != 0);
        offA += (int64_t)n[i] * n[i];
        offL += n[i];
    }
    return bad;
}

void orc_syevd_backward(int n, const double *lam, const double *Q, const double *dlam,
                        const double *dQ, double eps, double *dA)
{
    double *M = xcalloc((size_t)n * n, sizeof(double));
    double *S = xcalloc((size_t)n * n, sizeof(double));
    double *T = xcalloc((size_t)n * n, sizeof(double));
    double lmax = 0.0;
    for (int i = 0; i < n; ++i) lmax = fmax(lmax, fabs(lam[i]));
    double guard = eps * fmax(1.0, lmax);
    if (dQ)
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                double s = 0.0;
                for (int r = 0; r < n; ++r) s += Q[r * n + i] * dQ[r * n + j];
                M[i * n + j] = s; /* Q^T dQ */
            }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double fm_ij = 0.0, fm_ji = 0.0;
            if (i != j && fabs(lam[j] - lam[i]) > guard) {
                fm_ij = M[i * n + j] / (lam[j] - lam[i]);
                fm_ji = M[j * n + i] / (lam[i] - lam[j]);
            }
            S[i * n + j] = 0.5 * (fm_ij + fm_ji);
        }
    if (dlam)
        for (int i = 0; i < n; ++i) S[i * n + i] += dlam[i];
    for (int i = 0; i < n; ++i) /* T = Q S */
        for (int j = 0; j < n; ++j) {
            double s = 0.0;
            for (int r = 0; r < n; ++r) s += Q[i * n + r] * S[r * n + j];
            T[i * n + j] = s;
        }
    for (int i = 0; i < n; ++i) /* dA = T Q^T */
        for (int j = 0; j < n; ++j) {
            double s = 0.0;
            for (int r = 0; r < n; ++r) s += T[i * n + r] * Q[j * n + r];
            dA[i * n + j] = s;
        }
    free(M); free(S); free(T);
}
