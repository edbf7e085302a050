/*
 * FP64 CPU oracle for the reduced-camera-system solve of bundle adjustment.
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  The product path
 * (the HIP library) shares no source with it and never calls it.
 *
 * Plain, slow, obviously-correct C.  Every routine follows one passage of
 * Weber, Demmel, Cremers, "Multidirectional Conjugate Gradients for Scalable
 * Bundle Adjustment" (GCPR 2021):
 *   - normal-equation blocks U_lambda, V_lambda, W, b_p, b_l:  Sec. 3.1, eq. (8)-(12)
 *   - damping lambda * D^T D with diagonal D:                  Sec. 3.1, eq. (6)
 *   - reduced camera system S, b~:                              Sec. 3.1, eq. (13)-(15)
 *   - back-substitution of the landmark update:                 Sec. 3.1, eq. (16)
 *     (printed with a sign error; the form used here follows from the second
 *      block row of eq. (7): dx_l = -V^-1 (b_l + W^T dx_p))
 *   - block-Jacobi preconditioner D(S):                         Sec. 3.2, before Alg. 1
 *   - PCG:                                                      Sec. 3.2, Algorithm 1
 *   - MCG with local preconditioners, tau-test, pseudo-inverse,
 *     full reorthogonalisation and the cheap Q update:         Sec. 3.2, Algorithm 2,
 *                                                               "Adaptive tau-test",
 *                                                               "Optimized implementation", eq. (19)
 *   - partition of the poses into N subsets:                    Sec. 3.2, "Optimized implementation"
 *
 * Readings where the paper is silent (all FP64):
 *   R1  D_p^T D_p = diag(J_p^T J_p), D_l^T D_l = diag(J_l^T J_l) (Marquardt).
 *   R2  stop test: Euclidean norm of the recursive residual, strict "<".
 *   R3  Delta_i is symmetrised, (Q^T P + P^T Q)/2, and pseudo-inverted through a
 *       cyclic Jacobi eigendecomposition; eigenvalues with |l| <= k * 2^-52 * max|l|
 *       are dropped (Moore-Penrose).
 *   R4  the first step is global; a step is multidirectional iff N > 1 and t_i < tau.
 *   R5  eq. (19) sums over j = 0..i and is used on multidirectional steps only;
 *       global steps take Q = S P.
 *   R6  partition: s = floor(n_p / N); subsets 0..N-2 hold s consecutive poses
 *       (input order), the last one the remaining n_p - (N-1) s.
 *   R7  duplicate (camera, landmark) observations are rejected.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_OK 0
#define OR_MAXITER 1
#define OR_ERR_INVALID (-1)
#define OR_ERR_NONFINITE (-2)
#define OR_ERR_NOT_SPD (-3)
#define OR_ERR_BREAKDOWN (-4)
#define OR_ERR_NOMEM (-7)

#define DPMAX 9   /* largest pose dimension d_p (Sec. 3.1: 6 extrinsics, 9 with intrinsics) */

typedef struct {
    int np, nl;
    int dp;                      /* pose dimension d_p: 6 or 9 */
    int64_t m;
    double lambda;
    const double *Jp, *Jl, *r;   /* kept for the build only; not owned */
    int *cam, *lm;               /* owned copies */
    double *U;                   /* np x dp^2 : U_lambda blocks */
    double *Vinv;                /* nl x 9    : V_lambda^-1 (3x3) */
    double *W;                   /* m x 3 dp  : W_o = J_p,o^T J_l,o (dp x 3 row-major) */
    double *bp, *bl, *bt;        /* dp np, 3 nl, dp np */
    double *D;                   /* np x dp^2 : D(S) blocks */
    double *Dchol;               /* np x dp^2 : lower Cholesky factors of D(S) */
    int64_t *lm_ptr, *lm_obs;    /* observations of each landmark */
    int64_t *cam_ptr, *cam_obs;  /* observations of each camera */
    double *Ulr;                 /* n x lr_rank (row-major) low-rank preconditioner term, or NULL */
    int lr_rank;
} or_sys;

typedef struct {
    int iterations;
    int multi_steps;
    int history_cols;
    int status;
    double rel_res_recursive;
    double rel_res_true;
} or_stats;

/* ------------------------------------------------------------------ small dense */

/* lower Cholesky of a k x k SPD matrix in place (row-major); returns 0 or -1. */
static int chol(double *A, int k) {
    for (int j = 0; j < k; ++j) {
        double d = A[j * k + j];
        for (int p = 0; p < j; ++p) d -= A[j * k + p] * A[j * k + p];
        if (!(d > 0.0)) return -1;
        d = sqrt(d);
        A[j * k + j] = d;
        for (int i = j + 1; i < k; ++i) {
            double s = A[i * k + j];
            for (int p = 0; p < j; ++p) s -= A[i * k + p] * A[j * k + p];
            A[i * k + j] = s / d;
        }
        for (int i = 0; i < j; ++i) A[i * k + j] = 0.0;
    }
    return 0;
}

/* solve L L^T x = b in place */
static void chol_solve(const double *L, int k, double *x) {
    for (int i = 0; i < k; ++i) {
        double s = x[i];
        for (int p = 0; p < i; ++p) s -= L[i * k + p] * x[p];
        x[i] = s / L[i * k + i];
    }
    for (int i = k - 1; i >= 0; --i) {
        double s = x[i];
        for (int p = i + 1; p < k; ++p) s -= L[p * k + i] * x[p];
        x[i] = s / L[i * k + i];
    }
}

/* Pseudo-inverse of a symmetric k x k matrix through a cyclic Jacobi
 * eigendecomposition (reading R3).  A is read, Ap (k x k) written, eig (k,
 * nullable) receives the eigenvalues.  Returns the numerical rank. */
int or_pinv(int k, const double *A, double *Ap, double *eig) {
    double *a = (double *)malloc(sizeof(double) * k * k);
    double *v = (double *)malloc(sizeof(double) * k * k);
    for (int i = 0; i < k * k; ++i) a[i] = A[i];
    for (int i = 0; i < k; ++i)
        for (int j = 0; j < k; ++j) v[i * k + j] = (i == j) ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        int rotated = 0;
        for (int p = 0; p < k - 1; ++p) {
            for (int q = p + 1; q < k; ++q) {
                double apq = a[p * k + q];
                double app = a[p * k + p], aqq = a[q * k + q];
                if (fabs(apq) <= 1e-300) continue;
                if (fabs(apq) <= 2.2e-16 * 0.5 * sqrt(fabs(app) * fabs(aqq))) continue;
                rotated = 1;
                double theta = (aqq - app) / (2.0 * apq);
                double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
                /* A <- J^T A J with J the rotation in the (p, q) plane */
                for (int r = 0; r < k; ++r) {
                    double arp = a[r * k + p], arq = a[r * k + q];
                    a[r * k + p] = c * arp - s * arq;
                    a[r * k + q] = s * arp + c * arq;
                }
                for (int r = 0; r < k; ++r) {
                    double apr = a[p * k + r], aqr = a[q * k + r];
                    a[p * k + r] = c * apr - s * aqr;
                    a[q * k + r] = s * apr + c * aqr;
                }
                a[p * k + q] = 0.0;
                a[q * k + p] = 0.0;
                for (int r = 0; r < k; ++r) {
                    double vrp = v[r * k + p], vrq = v[r * k + q];
                    v[r * k + p] = c * vrp - s * vrq;
                    v[r * k + q] = s * vrp + c * vrq;
                }
            }
        }
        if (!rotated) break;
    }
    double lmax = 0.0;
    for (int i = 0; i < k; ++i) lmax = fmax(lmax, fabs(a[i * k + i]));
    double thr = (double)k * ldexp(1.0, -52) * lmax;
    int rank = 0;
    for (int i = 0; i < k * k; ++i) Ap[i] = 0.0;
    for (int e = 0; e < k; ++e) {
        double l = a[e * k + e];
        if (eig) eig[e] = l;
        if (!(fabs(l) > thr)) continue;
        ++rank;
        double il = 1.0 / l;
        for (int i = 0; i < k; ++i)
            for (int j = 0; j < k; ++j) Ap[i * k + j] += v[i * k + e] * il * v[j * k + e];
    }
    free(a);
    free(v);
    return rank;
}

/* Partition of the poses into N consecutive subsets (reading R6). */
void or_partition(int np, int N, int *group) {
    if (N < 1 || N > np) {
        for (int c = 0; c < np; ++c) group[c] = -1;
        return;
    }
    int s = np / N;
    for (int c = 0; c < np; ++c) {
        int g = c / s;
        group[c] = g < N - 1 ? g : N - 1;
    }
}

/* ------------------------------------------------------------------ build */

static int64_t *csr_by(const int *key, int64_t m, int nk, int64_t **ptr_out) {
    int64_t *ptr = (int64_t *)calloc((size_t)nk + 1, sizeof(int64_t));
    int64_t *idx = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m > 0 ? m : 1));
    for (int64_t o = 0; o < m; ++o) ptr[key[o] + 1]++;
    for (int k = 0; k < nk; ++k) ptr[k + 1] += ptr[k];
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)nk);
    for (int k = 0; k < nk; ++k) fill[k] = ptr[k];
    for (int64_t o = 0; o < m; ++o) idx[fill[key[o]]++] = o;
    free(fill);
    *ptr_out = ptr;
    return idx;
}

static int cmp_int(const void *a, const void *b) {
    int x = *(const int *)a, y = *(const int *)b;
    return (x > y) - (x < y);
}

void or_free(or_sys *s) {
    if (!s) return;
    free(s->cam); free(s->lm); free(s->U); free(s->Vinv); free(s->W);
    free(s->bp); free(s->bl); free(s->bt); free(s->D); free(s->Dchol);
    free(s->lm_ptr); free(s->lm_obs); free(s->cam_ptr); free(s->cam_obs);
    free(s->Ulr);
    free(s);
}

/* Build every block of the damped normal equation (eq. (8)-(12)) and of the
 * reduced camera system (eq. (14)-(15)), plus the block-Jacobi blocks D(S), for
 * poses of dimension dp (6: extrinsics only; 9: with intrinsics; Sec. 3.1).
 * Host arrays: cam, lm [m]; Jp [m][2][dp]; Jl [m][2][3]; r [m][2]. */
or_sys *or_build_dp(int np, int nl, int64_t m, const int *cam, const int *lm, const double *Jp,
                    const double *Jl, const double *r, double lambda, int dp, int *status) {
    *status = OR_OK;
    if (np <= 0 || nl <= 0 || m < 0 || !(lambda >= 0.0) || !cam || !lm || !Jp || !Jl || !r ||
        (dp != 6 && dp != 9)) {
        *status = OR_ERR_INVALID;
        return NULL;
    }
    for (int64_t o = 0; o < m; ++o) {
        if (cam[o] < 0 || cam[o] >= np || lm[o] < 0 || lm[o] >= nl) {
            *status = OR_ERR_INVALID;
            return NULL;
        }
    }
    for (int64_t i = 0; i < m * 2 * dp; ++i) if (!isfinite(Jp[i])) { *status = OR_ERR_NONFINITE; return NULL; }
    for (int64_t i = 0; i < m * 6; ++i) if (!isfinite(Jl[i])) { *status = OR_ERR_NONFINITE; return NULL; }
    for (int64_t i = 0; i < m * 2; ++i) if (!isfinite(r[i])) { *status = OR_ERR_NONFINITE; return NULL; }

    or_sys *s = (or_sys *)calloc(1, sizeof(or_sys));
    s->np = np; s->nl = nl; s->m = m; s->lambda = lambda; s->dp = dp;
    s->cam = (int *)malloc(sizeof(int) * (size_t)(m > 0 ? m : 1));
    s->lm = (int *)malloc(sizeof(int) * (size_t)(m > 0 ? m : 1));
    memcpy(s->cam, cam, sizeof(int) * (size_t)m);
    memcpy(s->lm, lm, sizeof(int) * (size_t)m);
    s->lm_obs = csr_by(s->lm, m, nl, &s->lm_ptr);
    s->cam_obs = csr_by(s->cam, m, np, &s->cam_ptr);

    /* R7: no landmark may be observed twice by the same camera */
    int bad = 0;
    for (int l = 0; l < nl && !bad; ++l) {
        int64_t a = s->lm_ptr[l], b = s->lm_ptr[l + 1];
        int64_t c = b - a;
        if (c < 2) continue;
        int *tmp = (int *)malloc(sizeof(int) * (size_t)c);
        for (int64_t q = 0; q < c; ++q) tmp[q] = s->cam[s->lm_obs[a + q]];
        qsort(tmp, (size_t)c, sizeof(int), cmp_int);
        for (int64_t q = 1; q < c; ++q) if (tmp[q] == tmp[q - 1]) bad = 1;
        free(tmp);
    }
    if (bad) { or_free(s); *status = OR_ERR_INVALID; return NULL; }

    int n = dp * np;
    s->U = (double *)calloc((size_t)np * dp * dp, sizeof(double));
    s->Vinv = (double *)calloc((size_t)nl * 9, sizeof(double));
    s->W = (double *)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1) * 3 * dp);
    s->bp = (double *)calloc((size_t)n, sizeof(double));
    s->bl = (double *)calloc((size_t)nl * 3, sizeof(double));
    s->bt = (double *)calloc((size_t)n, sizeof(double));
    s->D = (double *)calloc((size_t)np * dp * dp, sizeof(double));
    s->Dchol = (double *)calloc((size_t)np * dp * dp, sizeof(double));
    if (!s->U || !s->Vinv || !s->W || !s->bp || !s->bl || !s->bt || !s->D || !s->Dchol) {
        or_free(s); *status = OR_ERR_NOMEM; return NULL;
    }

    /* eq. (11): W = J_p^T J_l, one dp x 3 block per observation (camera, landmark) */
#pragma omp parallel for schedule(static)
    for (int64_t o = 0; o < m; ++o) {
        const double *jp = Jp + o * 2 * dp, *jl = Jl + o * 6;
        double *w = s->W + o * 3 * dp;
        for (int i = 0; i < dp; ++i)
            for (int j = 0; j < 3; ++j)
                w[i * 3 + j] = jp[0 * dp + i] * jl[0 * 3 + j] + jp[1 * dp + i] * jl[1 * 3 + j];
    }

    /* eq. (9), (11): U_lambda = J_p^T J_p + lambda D_p^T D_p, b_p = J_p^T r0 */
#pragma omp parallel for schedule(dynamic, 16)
    for (int c = 0; c < np; ++c) {
        double *U = s->U + (size_t)c * dp * dp;
        double *bp = s->bp + (size_t)c * dp;
        for (int64_t q = s->cam_ptr[c]; q < s->cam_ptr[c + 1]; ++q) {
            int64_t o = s->cam_obs[q];
            const double *jp = Jp + o * 2 * dp, *ro = r + o * 2;
            for (int i = 0; i < dp; ++i) {
                for (int j = 0; j < dp; ++j) U[i * dp + j] += jp[i] * jp[j] + jp[dp + i] * jp[dp + j];
                bp[i] += jp[i] * ro[0] + jp[dp + i] * ro[1];
            }
        }
        for (int i = 0; i < dp; ++i) U[i * dp + i] += lambda * U[i * dp + i];
    }

    /* eq. (10), (12): V_lambda = J_l^T J_l + lambda D_l^T D_l, b_l = J_l^T r0 */
    int spd_fail = 0;
#pragma omp parallel for schedule(dynamic, 256) reduction(| : spd_fail)
    for (int l = 0; l < nl; ++l) {
        double V[9] = {0}, bl[3] = {0};
        for (int64_t q = s->lm_ptr[l]; q < s->lm_ptr[l + 1]; ++q) {
            int64_t o = s->lm_obs[q];
            const double *jl = Jl + o * 6, *ro = r + o * 2;
            for (int i = 0; i < 3; ++i) {
                for (int j = 0; j < 3; ++j) V[i * 3 + j] += jl[i] * jl[j] + jl[3 + i] * jl[3 + j];
                bl[i] += jl[i] * ro[0] + jl[3 + i] * ro[1];
            }
        }
        for (int i = 0; i < 3; ++i) V[i * 3 + i] += lambda * V[i * 3 + i];
        for (int i = 0; i < 3; ++i) s->bl[(size_t)l * 3 + i] = bl[i];
        /* V^-1 as the solutions of V x = e_j */
        double L[9];
        memcpy(L, V, sizeof L);
        if (chol(L, 3) != 0) { spd_fail = 1; continue; }
        for (int j = 0; j < 3; ++j) {
            double e[3] = {0, 0, 0};
            e[j] = 1.0;
            chol_solve(L, 3, e);
            for (int i = 0; i < 3; ++i) s->Vinv[(size_t)l * 9 + i * 3 + j] = e[i];
        }
    }
    if (spd_fail) { or_free(s); *status = OR_ERR_NOT_SPD; return NULL; }

    /* eq. (15): b~ = b_p - W V^-1 b_l ;  D(S) = diagonal blocks of eq. (14) */
#pragma omp parallel for schedule(dynamic, 16) reduction(| : spd_fail)
    for (int c = 0; c < np; ++c) {
        double *bt = s->bt + (size_t)c * dp;
        double *D = s->D + (size_t)c * dp * dp;
        for (int i = 0; i < dp; ++i) bt[i] = s->bp[(size_t)c * dp + i];
        for (int i = 0; i < dp * dp; ++i) D[i] = s->U[(size_t)c * dp * dp + i];
        for (int64_t q = s->cam_ptr[c]; q < s->cam_ptr[c + 1]; ++q) {
            int64_t o = s->cam_obs[q];
            int l = s->lm[o];
            const double *w = s->W + o * 3 * dp, *Vi = s->Vinv + (size_t)l * 9, *bl = s->bl + (size_t)l * 3;
            double vb[3], WV[DPMAX * 3];
            for (int i = 0; i < 3; ++i) vb[i] = Vi[i * 3 + 0] * bl[0] + Vi[i * 3 + 1] * bl[1] + Vi[i * 3 + 2] * bl[2];
            for (int i = 0; i < dp; ++i) bt[i] -= w[i * 3 + 0] * vb[0] + w[i * 3 + 1] * vb[1] + w[i * 3 + 2] * vb[2];
            for (int i = 0; i < dp; ++i)
                for (int j = 0; j < 3; ++j)
                    WV[i * 3 + j] = w[i * 3 + 0] * Vi[0 * 3 + j] + w[i * 3 + 1] * Vi[1 * 3 + j] + w[i * 3 + 2] * Vi[2 * 3 + j];
            for (int i = 0; i < dp; ++i)
                for (int j = 0; j < dp; ++j)
                    D[i * dp + j] -= WV[i * 3 + 0] * w[j * 3 + 0] + WV[i * 3 + 1] * w[j * 3 + 1] + WV[i * 3 + 2] * w[j * 3 + 2];
        }
        double *L = s->Dchol + (size_t)c * dp * dp;
        memcpy(L, D, sizeof(double) * dp * dp);
        if (chol(L, dp) != 0) spd_fail = 1;
    }
    if (spd_fail) { or_free(s); *status = OR_ERR_NOT_SPD; return NULL; }
    return s;
}

or_sys *or_build(int np, int nl, int64_t m, const int *cam, const int *lm, const double *Jp,
                 const double *Jl, const double *r, double lambda, int *status) {
    return or_build_dp(np, nl, m, cam, lm, Jp, Jl, r, lambda, 9, status);
}

int or_dp(const or_sys *s) { return s->dp; }
int or_n(const or_sys *s) { return s->dp * s->np; }
void or_get_rhs(const or_sys *s, double *bt) { memcpy(bt, s->bt, sizeof(double) * s->dp * (size_t)s->np); }
void or_get_bp_bl(const or_sys *s, double *bp, double *bl) {
    memcpy(bp, s->bp, sizeof(double) * s->dp * (size_t)s->np);
    memcpy(bl, s->bl, sizeof(double) * 3 * (size_t)s->nl);
}
void or_get_U(const or_sys *s, double *U) { memcpy(U, s->U, sizeof(double) * s->dp * s->dp * (size_t)s->np); }
void or_get_Vinv(const or_sys *s, double *V) { memcpy(V, s->Vinv, sizeof(double) * 9 * (size_t)s->nl); }
void or_get_Dblocks(const or_sys *s, double *D) { memcpy(D, s->D, sizeof(double) * s->dp * s->dp * (size_t)s->np); }

/* ------------------------------------------------------------------ operators */

/* y = S v with S = U_lambda - W V_lambda^-1 W^T (eq. (14)), applied factor by factor. */
void or_schur_matvec(const or_sys *s, const double *v, double *y) {
    int np = s->np, nl = s->nl, dp = s->dp;
    double *h = (double *)malloc(sizeof(double) * 3 * (size_t)nl);
    /* h = V^-1 (W^T v) */
#pragma omp parallel for schedule(dynamic, 256)
    for (int l = 0; l < nl; ++l) {
        double g[3] = {0, 0, 0};
        for (int64_t q = s->lm_ptr[l]; q < s->lm_ptr[l + 1]; ++q) {
            int64_t o = s->lm_obs[q];
            const double *w = s->W + o * 3 * dp, *vc = v + (size_t)s->cam[o] * dp;
            for (int j = 0; j < 3; ++j)
                for (int i = 0; i < dp; ++i) g[j] += w[i * 3 + j] * vc[i];
        }
        const double *Vi = s->Vinv + (size_t)l * 9;
        for (int i = 0; i < 3; ++i) h[(size_t)l * 3 + i] = Vi[i * 3 + 0] * g[0] + Vi[i * 3 + 1] * g[1] + Vi[i * 3 + 2] * g[2];
    }
    /* y = U_lambda v - W h */
#pragma omp parallel for schedule(dynamic, 16)
    for (int c = 0; c < np; ++c) {
        const double *U = s->U + (size_t)c * dp * dp, *vc = v + (size_t)c * dp;
        double yc[DPMAX];
        for (int i = 0; i < dp; ++i) {
            double a = 0.0;
            for (int j = 0; j < dp; ++j) a += U[i * dp + j] * vc[j];
            yc[i] = a;
        }
        for (int64_t q = s->cam_ptr[c]; q < s->cam_ptr[c + 1]; ++q) {
            int64_t o = s->cam_obs[q];
            const double *w = s->W + o * 3 * dp, *hl = h + (size_t)s->lm[o] * 3;
            for (int i = 0; i < dp; ++i) yc[i] -= w[i * 3 + 0] * hl[0] + w[i * 3 + 1] * hl[1] + w[i * 3 + 2] * hl[2];
        }
        for (int i = 0; i < dp; ++i) y[(size_t)c * dp + i] = yc[i];
    }
    free(h);
}

/* z = D(S)^-1 r, one dp x dp Cholesky solve per pose; with a low-rank term set by
 * or_set_lowrank, z = D(S)^-1 r + U (U^T r). */
void or_precond_apply(const or_sys *s, const double *r, double *z) {
    const int dp = s->dp;
#pragma omp parallel for schedule(static)
    for (int c = 0; c < s->np; ++c) {
        double x[DPMAX];
        for (int i = 0; i < dp; ++i) x[i] = r[(size_t)c * dp + i];
        chol_solve(s->Dchol + (size_t)c * dp * dp, dp, x);
        for (int i = 0; i < dp; ++i) z[(size_t)c * dp + i] = x[i];
    }
    if (s->Ulr) {
        int n = dp * s->np, k = s->lr_rank;
        double t[64];
        for (int a = 0; a < k; ++a) t[a] = 0.0;
        for (int i = 0; i < n; ++i)
            for (int a = 0; a < k; ++a) t[a] += s->Ulr[(size_t)i * k + a] * r[i];
        for (int i = 0; i < n; ++i) {
            double acc = 0.0;
            for (int a = 0; a < k; ++a) acc += s->Ulr[(size_t)i * k + a] * t[a];
            z[i] += acc;
        }
    }
}

/* Sets (U != NULL, 1 <= rank <= 64) or clears the low-rank preconditioner term. */
int or_set_lowrank(or_sys *s, const double *U, int rank) {
    free(s->Ulr);
    s->Ulr = NULL;
    s->lr_rank = 0;
    if (!U) return OR_OK;
    if (rank < 1 || rank > 64) return OR_ERR_INVALID;
    size_t cnt = (size_t)s->dp * s->np * rank;
    s->Ulr = (double *)malloc(sizeof(double) * cnt);
    memcpy(s->Ulr, U, sizeof(double) * cnt);
    s->lr_rank = rank;
    return OR_OK;
}

/* dx_l = -V_lambda^-1 (b_l + W^T dx_p): second block row of eq. (7). */
void or_back_substitute(const or_sys *s, const double *dxp, double *dxl) {
#pragma omp parallel for schedule(dynamic, 256)
    for (int l = 0; l < s->nl; ++l) {
        double g[3];
        for (int j = 0; j < 3; ++j) g[j] = s->bl[(size_t)l * 3 + j];
        for (int64_t q = s->lm_ptr[l]; q < s->lm_ptr[l + 1]; ++q) {
            int64_t o = s->lm_obs[q];
            const double *w = s->W + o * 3 * s->dp, *vc = dxp + (size_t)s->cam[o] * s->dp;
            for (int j = 0; j < 3; ++j)
                for (int i = 0; i < s->dp; ++i) g[j] += w[i * 3 + j] * vc[i];
        }
        const double *Vi = s->Vinv + (size_t)l * 9;
        for (int i = 0; i < 3; ++i)
            dxl[(size_t)l * 3 + i] = -(Vi[i * 3 + 0] * g[0] + Vi[i * 3 + 1] * g[1] + Vi[i * 3 + 2] * g[2]);
    }
}

static double dot(const double *a, const double *b, int n) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

static double true_rel_residual(const or_sys *s, const double *x) {
    int n = s->dp * s->np;
    double *y = (double *)malloc(sizeof(double) * (size_t)n);
    or_schur_matvec(s, x, y);
    double num = 0.0, den = 0.0;
    for (int i = 0; i < n; ++i) {
        double e = -s->bt[i] - y[i];
        num += e * e;
        den += s->bt[i] * s->bt[i];
    }
    free(y);
    return den > 0.0 ? sqrt(num / den) : sqrt(num);
}

/* ------------------------------------------------------------------ Algorithm 1 */

/* PCG on S dx_p = -b~ with the block-Jacobi preconditioner.  x0 nullable (=> 0).
 * trace (nullable, length imax) receives |r_{i+1}| / |r_0| per iteration. */
int or_pcg(const or_sys *s, const double *x0, double *x, double eps, int imax, or_stats *st,
           double *trace) {
    int n = s->dp * s->np;
    double *r = (double *)malloc(sizeof(double) * n), *Z = (double *)malloc(sizeof(double) * n);
    double *P = (double *)malloc(sizeof(double) * n), *Q = (double *)malloc(sizeof(double) * n);
    memset(st, 0, sizeof(*st));
    /* residual of the start point (x0 = 0 unless given) */
    if (x0) memcpy(x, x0, sizeof(double) * n); else memset(x, 0, sizeof(double) * n);
    or_schur_matvec(s, x, Q);
    for (int i = 0; i < n; ++i) r[i] = -s->bt[i] - Q[i];
    double r0 = sqrt(dot(r, r, n));
    int status = OR_OK, it = 0;
    double rn = r0;
    if (r0 == 0.0) goto done;
    or_precond_apply(s, r, Z);
    memcpy(P, Z, sizeof(double) * n);
    status = OR_MAXITER;
    for (it = 0; it < imax; ) {
        or_schur_matvec(s, P, Q);                         /* image of the direction under S */
        double Delta = dot(Q, P, n), gamma = dot(P, r, n);
        if (!(Delta > 0.0)) { status = OR_ERR_BREAKDOWN; break; }
        double alpha = gamma / Delta;
        for (int i = 0; i < n; ++i) { x[i] += alpha * P[i]; r[i] -= alpha * Q[i]; }
        ++it;
        rn = sqrt(dot(r, r, n));
        if (trace) trace[it - 1] = rn / r0;
        if (rn < eps * r0) { status = OR_OK; break; }
        or_precond_apply(s, r, Z);                        /* preconditioned residual */
        /* next direction: Z minus its S-projection on the current one, which makes the
         * two S-conjugate (coefficient (S P)^T Z / P^T S P) */
        double beta = dot(Q, Z, n) / Delta;
        for (int i = 0; i < n; ++i) P[i] = Z[i] - beta * P[i];
    }
done:
    st->iterations = it;
    st->status = status;
    st->history_cols = it;
    st->rel_res_recursive = r0 > 0.0 ? rn / r0 : 0.0;
    st->rel_res_true = true_rel_residual(s, x);
    free(r); free(Z); free(P); free(Q);
    return status;
}

/* ------------------------------------------------------------------ Algorithm 2 */

typedef struct {
    int k;           /* columns of this direction block */
    double *P, *Q;   /* n x k, column-major (each column contiguous) */
    double *Dp;      /* k x k pseudo-inverse of Delta */
} blk_t;

/* MCG.  q_mode 0: eq. (19) on multidirectional steps (R5); q_mode 1: Q = S P always.
 * trace (nullable, imax x 3): |r_{i+1}|/|r_0|, t_i (NaN when the loop stops before
 * the tau-test), k_{i+1} (0 when stopped).  P_out (nullable, n x P_cap column-major)
 * receives the direction history; the number of columns is stats.history_cols. */
int or_mcg(const or_sys *s, int N, double tau, const double *x0, double *x, double eps, int imax,
           int q_mode, or_stats *st, double *trace, double *P_out, int64_t P_cap) {
    int n = s->dp * s->np, np = s->np, dp = s->dp;
    memset(st, 0, sizeof(*st));
    if (N < 1 || N > np || !(tau >= 0.0)) { st->status = OR_ERR_INVALID; return OR_ERR_INVALID; }
    int *group = (int *)malloc(sizeof(int) * np);
    or_partition(np, N, group);
    double *r = (double *)malloc(sizeof(double) * n), *z = (double *)malloc(sizeof(double) * n);
    double *tmp = (double *)malloc(sizeof(double) * n);
    int cap = 64;
    blk_t *H = (blk_t *)calloc((size_t)cap, sizeof(blk_t));
    int nb = 0, hcols = 0, multi = 0;

    if (x0) memcpy(x, x0, sizeof(double) * n); else memset(x, 0, sizeof(double) * n);
    or_schur_matvec(s, x, tmp);
    for (int i = 0; i < n; ++i) r[i] = -s->bt[i] - tmp[i];
    double r0 = sqrt(dot(r, r, n)), rn = r0;
    int status = OR_OK, it = 0;
    if (r0 == 0.0) goto done;

    /* first block: the preconditioned residual of the start point, and its image under S */
    H[0].k = 1;
    H[0].P = (double *)malloc(sizeof(double) * n);
    H[0].Q = (double *)malloc(sizeof(double) * n);
    or_precond_apply(s, r, H[0].P);
    or_schur_matvec(s, H[0].P, H[0].Q);
    nb = 1;
    hcols = 1;
    status = OR_MAXITER;
    for (it = 0; it < imax; ) {
        blk_t *B = &H[nb - 1];
        int k = B->k;
        /* step along the whole block: the Galerkin condition P^T (r - S P a) = 0 asks for
         * (P^T S P) a = P^T r; the Gram block is symmetrised and pseudo-inverted (reading R3) */
        double *Delta = (double *)malloc(sizeof(double) * k * k);
        double *gamma = (double *)malloc(sizeof(double) * k), *alpha = (double *)malloc(sizeof(double) * k);
        for (int a = 0; a < k; ++a)
            for (int b = 0; b < k; ++b) Delta[a * k + b] = dot(B->Q + (size_t)a * n, B->P + (size_t)b * n, n);
        for (int a = 0; a < k; ++a)
            for (int b = a + 1; b < k; ++b) {
                double m_ = 0.5 * (Delta[a * k + b] + Delta[b * k + a]);
                Delta[a * k + b] = m_;
                Delta[b * k + a] = m_;
            }
        for (int a = 0; a < k; ++a) gamma[a] = dot(B->P + (size_t)a * n, r, n);
        B->Dp = (double *)malloc(sizeof(double) * k * k);
        int rank = or_pinv(k, Delta, B->Dp, NULL);
        free(Delta);
        if (rank == 0) { free(gamma); free(alpha); status = OR_ERR_BREAKDOWN; break; }
        for (int a = 0; a < k; ++a) {
            double t = 0.0;
            for (int b = 0; b < k; ++b) t += B->Dp[a * k + b] * gamma[b];
            alpha[a] = t;
        }
        /* move along the block; the residual moves by the stored image S P of the block */
        for (int a = 0; a < k; ++a) {
            const double *Pa = B->P + (size_t)a * n, *Qa = B->Q + (size_t)a * n;
            double al = alpha[a];
            for (int i = 0; i < n; ++i) { x[i] += al * Pa[i]; r[i] -= al * Qa[i]; }
        }
        ++it;
        rn = sqrt(dot(r, r, n));
        if (trace) { trace[(it - 1) * 3 + 0] = rn / r0; trace[(it - 1) * 3 + 1] = NAN; trace[(it - 1) * 3 + 2] = 0; }
        if (rn < eps * r0) { free(gamma); free(alpha); status = OR_OK; break; }
        /* tau-test (Sec. 3.2): the decrease of the energy error the step achieved, relative
         * to r^T D(S)^-1 r of the new residual; small values call for more directions */
        or_precond_apply(s, r, z);
        double rho = dot(r, z, n);
        double ga = dot(gamma, alpha, k);
        free(gamma); free(alpha);
        double t_i = rho > 0.0 ? ga / rho : INFINITY;
        int is_multi = (N > 1) && (t_i < tau);
        int kn = is_multi ? N : 1;
        if (trace) { trace[(it - 1) * 3 + 1] = t_i; trace[(it - 1) * 3 + 2] = kn; }
        /* candidate directions: the preconditioned residual, or its restriction to each of
         * the N pose subsets (columns summing to it) */
        double *Z = (double *)calloc((size_t)n * kn, sizeof(double));
        if (is_multi) {
            for (int c = 0; c < np; ++c)
                for (int q = 0; q < dp; ++q) Z[(size_t)group[c] * n + (size_t)c * dp + q] = z[(size_t)c * dp + q];
        } else {
            memcpy(Z, z, sizeof(double) * n);
        }
        /* full reorthogonalisation: remove from the candidates their S-projection onto every
         * earlier block, so that the new block is S-conjugate to all of them; the coefficients
         * solve each earlier block's Gram system with (S P_j)^T Z as right-hand side.  On a
         * multidirectional step the image S of the new block follows from S Z and the same
         * coefficients (eq. (19)); otherwise it is formed directly. */
        if (nb == cap) {
            cap *= 2;
            H = (blk_t *)realloc(H, sizeof(blk_t) * (size_t)cap);
        }
        blk_t *Nw = &H[nb];
        Nw->k = kn;
        Nw->P = (double *)malloc(sizeof(double) * (size_t)n * kn);
        Nw->Q = (double *)malloc(sizeof(double) * (size_t)n * kn);
        Nw->Dp = NULL;
        memcpy(Nw->P, Z, sizeof(double) * (size_t)n * kn);
        double *SZ = NULL;
        if (is_multi && q_mode == 0) {
            SZ = (double *)malloc(sizeof(double) * (size_t)n * kn);
            for (int p = 0; p < kn; ++p) or_schur_matvec(s, Z + (size_t)p * n, SZ + (size_t)p * n);
            memcpy(Nw->Q, SZ, sizeof(double) * (size_t)n * kn);
        }
        for (int j = 0; j < nb; ++j) {
            blk_t *Bj = &H[j];
            int kj = Bj->k;
            double *Phi = (double *)calloc((size_t)kj * kn, sizeof(double));
            double *beta = (double *)calloc((size_t)kj * kn, sizeof(double));
#pragma omp parallel for schedule(static)
            for (int a = 0; a < kj; ++a) {
                const double *Qa = Bj->Q + (size_t)a * n;
                if (is_multi) {
                    /* columns of Z are zero outside their subset: sum only the nonzero rows */
                    for (int c = 0; c < np; ++c) {
                        double sacc = 0.0;
                        for (int q = 0; q < dp; ++q) sacc += Qa[(size_t)c * dp + q] * z[(size_t)c * dp + q];
                        Phi[(size_t)a * kn + group[c]] += sacc;
                    }
                } else {
                    Phi[a] = dot(Qa, Z, n);
                }
            }
            for (int a = 0; a < kj; ++a)
                for (int p = 0; p < kn; ++p) {
                    double t = 0.0;
                    for (int b = 0; b < kj; ++b) t += Bj->Dp[a * kj + b] * Phi[(size_t)b * kn + p];
                    beta[(size_t)a * kn + p] = t;
                }
#pragma omp parallel for schedule(static)
            for (int p = 0; p < kn; ++p) {
                double *Pn = Nw->P + (size_t)p * n, *Qn = Nw->Q + (size_t)p * n;
                for (int a = 0; a < kj; ++a) {
                    double bt_ = beta[(size_t)a * kn + p];
                    const double *Pa = Bj->P + (size_t)a * n, *Qa = Bj->Q + (size_t)a * n;
                    for (int i = 0; i < n; ++i) Pn[i] -= Pa[i] * bt_;
                    if (SZ) for (int i = 0; i < n; ++i) Qn[i] -= Qa[i] * bt_;   /* eq. (19) */
                }
            }
            free(Phi);
            free(beta);
        }
        if (!SZ) {
            for (int p = 0; p < kn; ++p) or_schur_matvec(s, Nw->P + (size_t)p * n, Nw->Q + (size_t)p * n);
        }
        free(SZ);
        free(Z);
        nb++;
        hcols += kn;
        multi += is_multi;
    }
done:
    st->iterations = it;
    st->multi_steps = multi;
    st->history_cols = hcols;
    st->status = status;
    st->rel_res_recursive = r0 > 0.0 ? rn / r0 : 0.0;
    st->rel_res_true = true_rel_residual(s, x);
    if (P_out) {
        int64_t col = 0;
        for (int j = 0; j < nb; ++j)
            for (int a = 0; a < H[j].k; ++a, ++col)
                if (col < P_cap) memcpy(P_out + col * n, H[j].P + (size_t)a * n, sizeof(double) * n);
    }
    for (int j = 0; j < nb; ++j) { free(H[j].P); free(H[j].Q); free(H[j].Dp); }
    free(H); free(group); free(r); free(z); free(tmp);
    return status;
}

int or_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
