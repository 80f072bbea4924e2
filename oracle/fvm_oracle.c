/*
 * fvm_oracle.c -- plain, slow, FP64 CPU oracle of the incompressible
 * finite-volume PISO / SIMPLE hot path (Tomczak et al., "Complete PISO and
 * SIMPLE solvers on Graphics Processing Units").
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no source,
 * header, table or helper with the HIP path, and the HIP path never calls it.
 *
 * What it computes (the paper's Section 3 follows Jasak's thesis and
 * OpenFOAM; details the paper leaves open are fixed by the readings listed
 * in the design notes):
 *   - mesh: N polyhedral cells, faces owned by one cell and (internal faces)
 *     shared with a neighbour, unknowns at cell centres (Section 3.1);
 *   - one sparse system A x = b per solve, non-zero A_ij iff i, j share a face
 *     or i == j (Section 3.1), stored here in the plainest face-addressed
 *     form: diag[N], upper[f] = A(owner,neighbour), lower[f] =
 *     A(neighbour,owner);
 *   - operators: Gauss gradient, divergence of face fluxes, Laplacian with
 *     the over-relaxed non-orthogonal split, linear (or upwind) convection
 *     (Section 4.3.3 names gradient, divergence and Laplacian as the
 *     assembly operators);
 *   - Krylov solvers with Jacobi or diagonal-incomplete-Cholesky
 *     preconditioning: CG for pressure, BiCG for momentum (Section 3; the
 *     recurrences of Barrett et al., "Templates", which the paper cites);
 *   - PISO (transient) and SIMPLE (steady) outer algorithms (Section 3).
 *
 * Every loop runs in the plainest order: faces in the order given, cells
 * ascending, global sums sequential.  No blocking, fusion or reordering.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { BC_FIXED = 0, BC_ZERO_GRAD = 1, BC_EMPTY = 2 };
enum { PC_JACOBI = 0, PC_DIC = 1 };
enum { CONV_LINEAR = 0, CONV_UPWIND = 1 };
enum { ST_OK = 0, ST_MAXITER = 1, ST_EINVAL = -1, ST_ENOMEM = -2, ST_ENUMERIC = -3 };

typedef struct {
    int32_t n_cells, n_faces, n_internal, n_patches;
    const int32_t *owner;          /* [n_faces] */
    const int32_t *neighbour;      /* [n_internal] */
    const double *Sf;              /* [n_faces][3], pointing out of the owner */
    const double *Cf;              /* [n_faces][3] */
    const double *C;               /* [n_cells][3] */
    const double *V;               /* [n_cells] */
    const int32_t *patch_start;    /* [n_patches], boundary faces tile [n_internal, n_faces) */
    const int32_t *patch_size;
    const int32_t *patch_u_kind;
    const int32_t *patch_p_kind;
    const double *patch_u_value;   /* [n_patches][3] */
    const double *patch_p_value;   /* [n_patches] */
} orc_mesh;

typedef struct {
    double nu, dt, alpha_u, alpha_p, p_ref_value;
    double p_tol, p_rel_tol, u_tol, u_rel_tol;
    int32_t n_corr, n_non_orth_corr, convection, p_ref_cell;
    int32_t p_max_iter, p_precond, u_max_iter, u_solver;   /* u_solver: 0 BiCG, 1 BiCGStab */
} orc_opts;

typedef struct { int32_t iters, status; double res_initial, res_final; } orc_solve_info;
typedef struct { orc_solve_info u[3]; orc_solve_info p[16]; int32_t n_p_solves, status; } orc_step_info;

#define SMALL 1e-20

static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static double *dalloc(size_t n) { return (double *)calloc(n ? n : 1, sizeof(double)); }

/* ------------------------------------------------------------------------
 * Face geometry coefficients.
 *   internal f (P owner, N neighbour):  d = C_N - C_P
 *     w_f  = S.(C_N - C_f) / (S.d)       owner weight of linear interpolation
 *     dl_f = |S|^2 / (S.d)               orthogonal Laplacian coefficient
 *     k_f  = S - dl_f d                  non-orthogonal remainder (0 if S || d)
 *   boundary b of P: d = C_f - C_P, dl_b = |S|^2 / (S.d)
 * ---------------------------------------------------------------------- */
typedef struct {
    const orc_mesh *m;
    int32_t Fb;
    double *w, *dl, *k;    /* w,k: internal only; dl: all faces */
    int32_t *bpatch;       /* [Fb] patch of each boundary face */
    int nonorth;           /* any |k_f| > 0 */
} geom;

static int geom_init(geom *g, const orc_mesh *m)
{
    int32_t Fi = m->n_internal, F = m->n_faces;
    g->m = m;
    g->Fb = F - Fi;
    g->w = dalloc(Fi);
    g->dl = dalloc(F);
    g->k = dalloc((size_t)3 * Fi);
    g->bpatch = (int32_t *)calloc(g->Fb ? g->Fb : 1, sizeof(int32_t));
    g->nonorth = 0;
    if (!g->w || !g->dl || !g->k || !g->bpatch) return ST_ENOMEM;
    for (int32_t f = 0; f < Fi; ++f) {
        const double *S = m->Sf + 3 * f, *Cf = m->Cf + 3 * f;
        const double *CP = m->C + 3 * m->owner[f], *CN = m->C + 3 * m->neighbour[f];
        double d[3] = {CN[0] - CP[0], CN[1] - CP[1], CN[2] - CP[2]};
        double nd[3] = {CN[0] - Cf[0], CN[1] - Cf[1], CN[2] - Cf[2]};
        double Sd = dot3(S, d);
        if (!(Sd > 0.0)) return ST_EINVAL;
        g->w[f] = dot3(S, nd) / Sd;
        g->dl[f] = dot3(S, S) / Sd;
        for (int c = 0; c < 3; ++c) {
            g->k[3 * f + c] = S[c] - g->dl[f] * d[c];
            if (g->k[3 * f + c] != 0.0) g->nonorth = 1;
        }
    }
    for (int32_t f = Fi; f < F; ++f) {
        const double *S = m->Sf + 3 * f, *Cf = m->Cf + 3 * f, *CP = m->C + 3 * m->owner[f];
        double d[3] = {Cf[0] - CP[0], Cf[1] - CP[1], Cf[2] - CP[2]};
        double Sd = dot3(S, d);
        if (!(Sd > 0.0)) return ST_EINVAL;
        g->dl[f] = dot3(S, S) / Sd;
    }
    for (int32_t b = 0; b < g->Fb; ++b) g->bpatch[b] = -1;
    for (int32_t p = 0; p < m->n_patches; ++p)
        for (int32_t i = 0; i < m->patch_size[p]; ++i) {
            int32_t b = m->patch_start[p] + i - Fi;
            if (b < 0 || b >= g->Fb) return ST_EINVAL;
            g->bpatch[b] = p;
        }
    for (int32_t b = 0; b < g->Fb; ++b)
        if (g->bpatch[b] < 0) return ST_EINVAL;
    return ST_OK;
}

static void geom_free(geom *g)
{
    free(g->w); free(g->dl); free(g->k); free(g->bpatch);
}

/* per-boundary-face kinds and values of p and U, taken from the patches */
typedef struct {
    int32_t *pk, *uk;
    double *pv, *uv;     /* pv[Fb], uv[Fb][3] */
} bconds;

static int bconds_from_patches(bconds *bc, const geom *g)
{
    const orc_mesh *m = g->m;
    bc->pk = (int32_t *)calloc(g->Fb ? g->Fb : 1, sizeof(int32_t));
    bc->uk = (int32_t *)calloc(g->Fb ? g->Fb : 1, sizeof(int32_t));
    bc->pv = dalloc(g->Fb);
    bc->uv = dalloc((size_t)3 * g->Fb);
    if (!bc->pk || !bc->uk || !bc->pv || !bc->uv) return ST_ENOMEM;
    for (int32_t b = 0; b < g->Fb; ++b) {
        int32_t p = g->bpatch[b];
        bc->pk[b] = m->patch_p_kind[p];
        bc->uk[b] = m->patch_u_kind[p];
        bc->pv[b] = m->patch_p_value[p];
        for (int c = 0; c < 3; ++c) bc->uv[3 * b + c] = m->patch_u_value[3 * p + c];
    }
    return ST_OK;
}

static void bconds_free(bconds *bc) { free(bc->pk); free(bc->uk); free(bc->pv); free(bc->uv); }

/* ------------------------------------------------------------------------
 * Gauss gradient: (grad phi)_P = (1/V_P) sum_f s_Pf S_f phi_f, phi_f the
 * linear interpolate on internal faces; on boundary faces the FIXED value or
 * (ZERO_GRAD) the owner value; EMPTY faces are skipped.
 * phi has stride `st` (1 for a scalar, 3 for one component of U).
 * ---------------------------------------------------------------------- */
static void grad_gauss(const geom *g, const double *phi, int st, const int32_t *bk, const double *bv, int bst,
                       double *gr)
{
    const orc_mesh *m = g->m;
    int32_t N = m->n_cells, Fi = m->n_internal;
    memset(gr, 0, sizeof(double) * 3 * (size_t)N);
    for (int32_t f = 0; f < Fi; ++f) {
        int32_t P = m->owner[f], Q = m->neighbour[f];
        double pf = g->w[f] * phi[(size_t)st * P] + (1.0 - g->w[f]) * phi[(size_t)st * Q];
        for (int c = 0; c < 3; ++c) {
            gr[3 * P + c] += m->Sf[3 * f + c] * pf;
            gr[3 * Q + c] -= m->Sf[3 * f + c] * pf;
        }
    }
    for (int32_t b = 0; b < g->Fb; ++b) {
        int32_t f = Fi + b, P = m->owner[f];
        if (bk[b] == BC_EMPTY) continue;
        double pf = bk[b] == BC_FIXED ? bv[(size_t)bst * b] : phi[(size_t)st * P];
        for (int c = 0; c < 3; ++c) gr[3 * P + c] += m->Sf[3 * f + c] * pf;
    }
    for (int32_t i = 0; i < N; ++i)
        for (int c = 0; c < 3; ++c) gr[3 * i + c] /= m->V[i];
}

/* ------------------------------------------------------------------------
 * Face-addressed matrix products.
 *   A x : y_i = diag_i x_i + sum over faces of the off-diagonal products
 *   A^T x swaps the roles of upper and lower.
 * ---------------------------------------------------------------------- */
typedef struct {
    int32_t N, Fi;
    const int32_t *own, *nei;
    const double *diag, *upper, *lower;
} ldu;

static void amul(const ldu *A, const double *x, double *y)
{
    for (int32_t i = 0; i < A->N; ++i) y[i] = A->diag[i] * x[i];
    for (int32_t f = 0; f < A->Fi; ++f) {
        y[A->own[f]] += A->upper[f] * x[A->nei[f]];
        y[A->nei[f]] += A->lower[f] * x[A->own[f]];
    }
}

static void tmul(const ldu *A, const double *x, double *y)
{
    for (int32_t i = 0; i < A->N; ++i) y[i] = A->diag[i] * x[i];
    for (int32_t f = 0; f < A->Fi; ++f) {
        y[A->own[f]] += A->lower[f] * x[A->nei[f]];
        y[A->nei[f]] += A->upper[f] * x[A->own[f]];
    }
}

static double sumdot(int32_t n, const double *a, const double *b)
{
    double s = 0.0;
    for (int32_t i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

static double sumabs(int32_t n, const double *a)
{
    double s = 0.0;
    for (int32_t i = 0; i < n; ++i) s += fabs(a[i]);
    return s;
}

/* Normalisation of the L1 residual: with xbar = mean(x),
 *   n_f = sum_i |(A x)_i - xbar (A 1)_i| + |b_i - xbar (A 1)_i| + 1e-20
 * computed once per solve from the initial guess.  (The paper stops on
 * residual thresholds, Section 4.3.1; this is the normalised form of
 * the OpenFOAM solvers it matches.) */
static double norm_factor(const ldu *A, const double *x, const double *b, const double *Ax)
{
    int32_t N = A->N;
    double xbar = 0.0;
    for (int32_t i = 0; i < N; ++i) xbar += x[i];
    xbar /= (double)(N > 0 ? N : 1);
    double *A1 = dalloc(N);
    for (int32_t i = 0; i < N; ++i) A1[i] = A->diag[i];
    for (int32_t f = 0; f < A->Fi; ++f) {
        A1[A->own[f]] += A->upper[f];
        A1[A->nei[f]] += A->lower[f];
    }
    double nf = 0.0;
    for (int32_t i = 0; i < N; ++i) nf += fabs(Ax[i] - xbar * A1[i]) + fabs(b[i] - xbar * A1[i]);
    free(A1);
    return nf + SMALL;
}

/* ------------------------------------------------------------------------
 * Diagonal incomplete Cholesky (the D-ILU of Barrett et al., Sec. 3.4) for a
 * symmetric matrix (upper == lower): only the diagonal is modified,
 *   D*_i = A_ii - sum_{j<i, j~i} A_ij A_ji / D*_j        (i ascending)
 * and M = (D* + L) D*^-1 (D* + U) is applied by
 *   forward  y_i = (r_i - sum_{j<i} A_ij y_j) / D*_i     (i ascending)
 *   backward z_i = y_i - (sum_{j>i} A_ij z_j) / D*_i     (i descending)
 * Each sum over j runs in ascending j.
 * ---------------------------------------------------------------------- */
typedef struct {
    int32_t N;
    int32_t *lo_start, *lo_col, *lo_face;   /* row i: neighbours j < i, ascending */
    int32_t *up_start, *up_col, *up_face;   /* row i: neighbours j > i, ascending */
    double *dstar;
} dic;

static int cmp_pair(const void *a, const void *b)
{
    const int32_t *x = (const int32_t *)a, *y = (const int32_t *)b;
    return (x[0] > y[0]) - (x[0] < y[0]);
}

static int dic_init(dic *d, const ldu *A)
{
    int32_t N = A->N, Fi = A->Fi;
    d->N = N;
    d->lo_start = (int32_t *)calloc((size_t)N + 1, sizeof(int32_t));
    d->up_start = (int32_t *)calloc((size_t)N + 1, sizeof(int32_t));
    d->lo_col = (int32_t *)calloc(Fi ? Fi : 1, sizeof(int32_t));
    d->lo_face = (int32_t *)calloc(Fi ? Fi : 1, sizeof(int32_t));
    d->up_col = (int32_t *)calloc(Fi ? Fi : 1, sizeof(int32_t));
    d->up_face = (int32_t *)calloc(Fi ? Fi : 1, sizeof(int32_t));
    d->dstar = dalloc(N);
    int32_t *pair = (int32_t *)calloc(2 * (size_t)(Fi ? Fi : 1), sizeof(int32_t));
    int32_t *fill = (int32_t *)calloc((size_t)N + 1, sizeof(int32_t));
    if (!d->lo_start || !d->up_start || !d->lo_col || !d->lo_face || !d->up_col || !d->up_face || !d->dstar ||
        !pair || !fill)
        return ST_ENOMEM;
    for (int32_t f = 0; f < Fi; ++f) {
        int32_t a = A->own[f], b = A->nei[f];
        int32_t hi = a > b ? a : b, lo = a > b ? b : a;
        d->lo_start[hi + 1]++;
        d->up_start[lo + 1]++;
    }
    for (int32_t i = 0; i < N; ++i) {
        d->lo_start[i + 1] += d->lo_start[i];
        d->up_start[i + 1] += d->up_start[i];
    }
    memset(fill, 0, sizeof(int32_t) * ((size_t)N + 1));
    for (int32_t f = 0; f < Fi; ++f) {
        int32_t a = A->own[f], b = A->nei[f];
        int32_t hi = a > b ? a : b, lo = a > b ? b : a;
        int32_t s = d->lo_start[hi] + fill[hi]++;
        d->lo_col[s] = lo; d->lo_face[s] = f;
    }
    memset(fill, 0, sizeof(int32_t) * ((size_t)N + 1));
    for (int32_t f = 0; f < Fi; ++f) {
        int32_t a = A->own[f], b = A->nei[f];
        int32_t hi = a > b ? a : b, lo = a > b ? b : a;
        int32_t s = d->up_start[lo] + fill[lo]++;
        d->up_col[s] = hi; d->up_face[s] = f;
    }
    /* sort each row's entries by column */
    for (int pass = 0; pass < 2; ++pass) {
        int32_t *st = pass ? d->up_start : d->lo_start;
        int32_t *col = pass ? d->up_col : d->lo_col, *fc = pass ? d->up_face : d->lo_face;
        for (int32_t i = 0; i < N; ++i) {
            int32_t n = st[i + 1] - st[i];
            for (int32_t k = 0; k < n; ++k) { pair[2 * k] = col[st[i] + k]; pair[2 * k + 1] = fc[st[i] + k]; }
            qsort(pair, (size_t)n, 2 * sizeof(int32_t), cmp_pair);
            for (int32_t k = 0; k < n; ++k) { col[st[i] + k] = pair[2 * k]; fc[st[i] + k] = pair[2 * k + 1]; }
        }
    }
    free(pair); free(fill);
    for (int32_t i = 0; i < N; ++i) {
        double s = A->diag[i];
        for (int32_t k = d->lo_start[i]; k < d->lo_start[i + 1]; ++k) {
            double a = A->upper[d->lo_face[k]];
            s -= a * a / d->dstar[d->lo_col[k]];
        }
        d->dstar[i] = s;
    }
    return ST_OK;
}

static void dic_apply(const dic *d, const ldu *A, const double *r, double *z)
{
    int32_t N = d->N;
    for (int32_t i = 0; i < N; ++i) {
        double s = r[i];
        for (int32_t k = d->lo_start[i]; k < d->lo_start[i + 1]; ++k) s -= A->upper[d->lo_face[k]] * z[d->lo_col[k]];
        z[i] = s / d->dstar[i];
    }
    for (int32_t i = N - 1; i >= 0; --i) {
        double s = 0.0;
        for (int32_t k = d->up_start[i]; k < d->up_start[i + 1]; ++k) s += A->upper[d->up_face[k]] * z[d->up_col[k]];
        z[i] = z[i] - s / d->dstar[i];
    }
}

static void dic_free(dic *d)
{
    free(d->lo_start); free(d->lo_col); free(d->lo_face);
    free(d->up_start); free(d->up_col); free(d->up_face); free(d->dstar);
}

/* ------------------------------------------------------------------------
 * Preconditioned conjugate gradients (Barrett et al., Sec. 2.3.1):
 *   r = b - A x;  loop: z = M^-1 r, rho = r.z, p = z (+ beta p), q = A p,
 *   alpha = rho / (p.q), x += alpha p, r -= alpha q.
 * Stop on the normalised L1 residual of the recurrence residual r,
 * nres <= max(tol, rel_tol * nres0), tested before the first iteration.
 * Breakdown (rho <= 0, p.q <= 0, non-finite) -> ST_ENUMERIC.
 * ---------------------------------------------------------------------- */
static int pcg(const ldu *A, const double *b, double *x, double tol, double rel_tol, int32_t max_iter, int precond,
               orc_solve_info *info)
{
    int32_t N = A->N;
    double *r = dalloc(N), *z = dalloc(N), *p = dalloc(N), *q = dalloc(N);
    int st = ST_OK;
    dic D;
    int have_dic = 0;
    info->iters = 0;
    amul(A, x, q);
    for (int32_t i = 0; i < N; ++i) r[i] = b[i] - q[i];
    double nf = norm_factor(A, x, b, q);
    double nres = sumabs(N, r) / nf;
    info->res_initial = nres;
    info->res_final = nres;
    double tol_eff = fmax(tol, rel_tol * nres);
    if (!isfinite(nres)) { st = ST_ENUMERIC; goto done; }
    if (nres <= tol_eff) goto done;
    if (precond == PC_DIC) {
        if (dic_init(&D, A) != ST_OK) { st = ST_ENOMEM; goto done; }
        have_dic = 1;
    }
    double rho_old = 1.0;
    st = ST_MAXITER;
    for (int32_t it = 1; it <= max_iter; ++it) {
        if (have_dic) dic_apply(&D, A, r, z);
        else for (int32_t i = 0; i < N; ++i) z[i] = r[i] / A->diag[i];
        double rho = sumdot(N, r, z);
        if (!(rho > 0.0) || !isfinite(rho)) { st = ST_ENUMERIC; info->iters = it; break; }
        if (it == 1) {
            for (int32_t i = 0; i < N; ++i) p[i] = z[i];
        } else {
            double beta = rho / rho_old;
            for (int32_t i = 0; i < N; ++i) p[i] = z[i] + beta * p[i];
        }
        amul(A, p, q);
        double pq = sumdot(N, p, q);
        if (!(pq > 0.0) || !isfinite(pq)) { st = ST_ENUMERIC; info->iters = it; break; }
        double alpha = rho / pq;
        for (int32_t i = 0; i < N; ++i) { x[i] += alpha * p[i]; r[i] -= alpha * q[i]; }
        nres = sumabs(N, r) / nf;
        info->iters = it;
        info->res_final = nres;
        if (!isfinite(nres)) { st = ST_ENUMERIC; break; }
        if (nres <= tol_eff) { st = ST_OK; break; }
        rho_old = rho;
    }
done:
    if (have_dic) dic_free(&D);
    free(r); free(z); free(p); free(q);
    info->status = st;
    return st;
}

/* ------------------------------------------------------------------------
 * Preconditioned bi-conjugate gradients (Barrett et al., Sec. 2.3.5) with
 * Jacobi: r~0 = r0; loop: z = M^-1 r, z~ = M^-T r~, rho = z.r~, p and p~
 * updated with the same beta, q = A p, q~ = A^T p~, alpha = rho / (p~.q),
 * x += alpha p, r -= alpha q, r~ -= alpha q~.  Same stopping test as pcg().
 * Breakdown (rho == 0, p~.q == 0, non-finite) -> ST_ENUMERIC.
 * ---------------------------------------------------------------------- */
static int pbicg(const ldu *A, const double *b, double *x, double tol, double rel_tol, int32_t max_iter,
                 orc_solve_info *info)
{
    int32_t N = A->N;
    double *r = dalloc(N), *rt = dalloc(N), *z = dalloc(N), *zt = dalloc(N);
    double *p = dalloc(N), *pt = dalloc(N), *q = dalloc(N), *qt = dalloc(N);
    int st = ST_OK;
    info->iters = 0;
    amul(A, x, q);
    for (int32_t i = 0; i < N; ++i) { r[i] = b[i] - q[i]; rt[i] = r[i]; }
    double nf = norm_factor(A, x, b, q);
    double nres = sumabs(N, r) / nf;
    info->res_initial = nres;
    info->res_final = nres;
    double tol_eff = fmax(tol, rel_tol * nres);
    if (!isfinite(nres)) { st = ST_ENUMERIC; goto done; }
    if (nres <= tol_eff) goto done;
    double rho_old = 1.0;
    st = ST_MAXITER;
    for (int32_t it = 1; it <= max_iter; ++it) {
        for (int32_t i = 0; i < N; ++i) { z[i] = r[i] / A->diag[i]; zt[i] = rt[i] / A->diag[i]; }
        double rho = sumdot(N, z, rt);
        if (rho == 0.0 || !isfinite(rho)) { st = ST_ENUMERIC; info->iters = it; break; }
        if (it == 1) {
            for (int32_t i = 0; i < N; ++i) { p[i] = z[i]; pt[i] = zt[i]; }
        } else {
            double beta = rho / rho_old;
            for (int32_t i = 0; i < N; ++i) { p[i] = z[i] + beta * p[i]; pt[i] = zt[i] + beta * pt[i]; }
        }
        amul(A, p, q);
        tmul(A, pt, qt);
        double ptq = sumdot(N, pt, q);
        if (ptq == 0.0 || !isfinite(ptq)) { st = ST_ENUMERIC; info->iters = it; break; }
        double alpha = rho / ptq;
        for (int32_t i = 0; i < N; ++i) {
            x[i] += alpha * p[i];
            r[i] -= alpha * q[i];
            rt[i] -= alpha * qt[i];
        }
        nres = sumabs(N, r) / nf;
        info->iters = it;
        info->res_final = nres;
        if (!isfinite(nres)) { st = ST_ENUMERIC; break; }
        if (nres <= tol_eff) { st = ST_OK; break; }
        rho_old = rho;
    }
done:
    free(r); free(rt); free(z); free(zt); free(p); free(pt); free(q); free(qt);
    info->status = st;
    return st;
}

/* ------------------------------------------------------------------------
 * Preconditioned BiCGSTAB (Barrett et al., Sec. 2.3.8) with Jacobi M and
 * shadow residual r~ = r0.  Per iteration: rho = r~.r; p = r (first) or
 * r + beta (p - omega v) with beta = (rho / rho_old)(alpha / omega);
 * p^ = M^-1 p; v = A p^; alpha = rho / (r~.v); s = r - alpha v; if s passes
 * the stopping test, x += alpha p^ and stop; else s^ = M^-1 s; t = A s^;
 * omega = (t.s) / (t.t); x += alpha p^ + omega s^; r = s - omega t.
 * Stopping test as pcg() (normalised L1 residual, also on s).  Breakdown
 * (rho == 0, r~.v == 0, t.t == 0, omega == 0, non-finite) -> ST_ENUMERIC.
 * ---------------------------------------------------------------------- */
static int pbicgstab(const ldu *A, const double *b, double *x, double tol, double rel_tol, int32_t max_iter,
                     orc_solve_info *info)
{
    int32_t N = A->N;
    double *r = dalloc(N), *rt = dalloc(N), *p = dalloc(N), *v = dalloc(N);
    double *sv = dalloc(N), *t = dalloc(N), *ph = dalloc(N), *sh = dalloc(N);
    int st = ST_OK;
    info->iters = 0;
    amul(A, x, v);
    for (int32_t i = 0; i < N; ++i) { r[i] = b[i] - v[i]; rt[i] = r[i]; }
    double nf = norm_factor(A, x, b, v);
    double nres = sumabs(N, r) / nf;
    info->res_initial = nres;
    info->res_final = nres;
    double tol_eff = fmax(tol, rel_tol * nres);
    if (!isfinite(nres)) { st = ST_ENUMERIC; goto done; }
    if (nres <= tol_eff) goto done;
    double rho_old = 1.0, alpha = 1.0, omega = 1.0;
    st = ST_MAXITER;
    for (int32_t it = 1; it <= max_iter; ++it) {
        double rho = sumdot(N, rt, r);
        if (rho == 0.0 || !isfinite(rho)) { st = ST_ENUMERIC; info->iters = it; break; }
        if (it == 1) {
            for (int32_t i = 0; i < N; ++i) p[i] = r[i];
        } else {
            double beta = (rho / rho_old) * (alpha / omega);
            for (int32_t i = 0; i < N; ++i) p[i] = r[i] + beta * (p[i] - omega * v[i]);
        }
        for (int32_t i = 0; i < N; ++i) ph[i] = p[i] / A->diag[i];
        amul(A, ph, v);
        double rtv = sumdot(N, rt, v);
        if (rtv == 0.0 || !isfinite(rtv)) { st = ST_ENUMERIC; info->iters = it; break; }
        alpha = rho / rtv;
        for (int32_t i = 0; i < N; ++i) sv[i] = r[i] - alpha * v[i];
        double ns = sumabs(N, sv) / nf;
        info->iters = it;
        if (!isfinite(ns)) { info->res_final = ns; st = ST_ENUMERIC; break; }
        if (ns <= tol_eff) {
            for (int32_t i = 0; i < N; ++i) { x[i] += alpha * ph[i]; r[i] = sv[i]; }
            info->res_final = ns;
            st = ST_OK;
            break;
        }
        for (int32_t i = 0; i < N; ++i) sh[i] = sv[i] / A->diag[i];
        amul(A, sh, t);
        double tt = sumdot(N, t, t), ts = sumdot(N, t, sv);
        if (tt == 0.0 || !isfinite(tt) || !isfinite(ts)) { st = ST_ENUMERIC; break; }
        omega = ts / tt;
        for (int32_t i = 0; i < N; ++i) {
            x[i] += alpha * ph[i] + omega * sh[i];
            r[i] = sv[i] - omega * t[i];
        }
        nres = sumabs(N, r) / nf;
        info->res_final = nres;
        if (!isfinite(nres)) { st = ST_ENUMERIC; break; }
        if (nres <= tol_eff) { st = ST_OK; break; }
        if (omega == 0.0) { st = ST_ENUMERIC; break; }
        rho_old = rho;
    }
done:
    free(r); free(rt); free(p); free(v); free(sv); free(t); free(ph); free(sh);
    info->status = st;
    return st;
}

/* ------------------------------------------------------------------------
 * Momentum matrix (one matrix for all three components).
 * Internal face f, P owner, N neighbour, face flux F = phi_f, weight w
 * (upwind: w = 1 if F >= 0 else 0):
 *   convection  a_PP += F w,     a_PN += F (1-w),  a_NN -= F (1-w),  a_NP -= F w
 *   diffusion   a_PP += nu dl,   a_PN -= nu dl,    a_NN += nu dl,    a_NP -= nu dl
 *   non-orth.   b_P  += nu k.(grad U)_f,  b_N -= nu k.(grad U)_f
 * Boundary face: FIXED  a_PP += nu dl_b,  b_P += (nu dl_b - F_b) U_b
 *                ZERO_GRAD a_PP += F_b;   EMPTY nothing.
 * Transient (dt > 0): a_PP += V/dt, b_P += V U_old/dt.
 * The pressure gradient is not part of src.
 * ---------------------------------------------------------------------- */
static void momentum_system(const geom *g, const bconds *bc, double nu, double dt, int convection,
                            const double *phi, const double *U_old, const double *U_grad, double *diag,
                            double *upper, double *lower, double *src)
{
    const orc_mesh *m = g->m;
    int32_t N = m->n_cells, Fi = m->n_internal;
    memset(diag, 0, sizeof(double) * (size_t)N);
    memset(src, 0, sizeof(double) * 3 * (size_t)N);
    if (dt > 0.0)
        for (int32_t i = 0; i < N; ++i) {
            diag[i] += m->V[i] / dt;
            for (int c = 0; c < 3; ++c) src[3 * i + c] += m->V[i] * U_old[3 * i + c] / dt;
        }
    for (int32_t f = 0; f < Fi; ++f) {
        int32_t P = m->owner[f], Q = m->neighbour[f];
        double F = phi[f];
        double w = convection == CONV_UPWIND ? (F >= 0.0 ? 1.0 : 0.0) : g->w[f];
        double D = nu * g->dl[f];
        upper[f] = F * (1.0 - w) - D;
        lower[f] = -F * w - D;
        diag[P] += F * w + D;
        diag[Q] += -F * (1.0 - w) + D;
    }
    for (int32_t b = 0; b < g->Fb; ++b) {
        int32_t f = Fi + b, P = m->owner[f];
        double F = phi[f];
        if (bc->uk[b] == BC_FIXED) {
            double D = nu * g->dl[f];
            diag[P] += D;
            for (int c = 0; c < 3; ++c) src[3 * P + c] += (D - F) * bc->uv[3 * b + c];
        } else if (bc->uk[b] == BC_ZERO_GRAD) {
            diag[P] += F;
        }
    }
    if (g->nonorth && U_grad) {
        double *gU = dalloc((size_t)9 * N), *tmp = dalloc((size_t)3 * N);
        for (int c = 0; c < 3; ++c) {
            grad_gauss(g, U_grad + c, 3, bc->uk, bc->uv + c, 3, tmp);
            for (int32_t i = 0; i < N; ++i)
                for (int d = 0; d < 3; ++d) gU[9 * i + 3 * c + d] = tmp[3 * i + d];
        }
        for (int32_t f = 0; f < Fi; ++f) {
            int32_t P = m->owner[f], Q = m->neighbour[f];
            double w = g->w[f];
            for (int c = 0; c < 3; ++c) {
                double gf[3];
                for (int d = 0; d < 3; ++d) gf[d] = w * gU[9 * P + 3 * c + d] + (1.0 - w) * gU[9 * Q + 3 * c + d];
                double s = nu * dot3(g->k + 3 * f, gf);
                src[3 * P + c] += s;
                src[3 * Q + c] -= s;
            }
        }
        free(gU); free(tmp);
    }
}

/* H_P = b_P - sum_N a_PN U_N;  rAU_P = V_P / a_PP;  HbyA_P = H_P / a_PP */
static void h_by_a(const geom *g, const double *diag, const double *upper, const double *lower, const double *src,
                   const double *U, double *rAU, double *HbyA)
{
    const orc_mesh *m = g->m;
    int32_t N = m->n_cells, Fi = m->n_internal;
    double *H = dalloc((size_t)3 * N);
    memcpy(H, src, sizeof(double) * 3 * (size_t)N);
    for (int32_t f = 0; f < Fi; ++f) {
        int32_t P = m->owner[f], Q = m->neighbour[f];
        for (int c = 0; c < 3; ++c) {
            H[3 * P + c] -= upper[f] * U[3 * Q + c];
            H[3 * Q + c] -= lower[f] * U[3 * P + c];
        }
    }
    for (int32_t i = 0; i < N; ++i) {
        rAU[i] = m->V[i] / diag[i];
        for (int c = 0; c < 3; ++c) HbyA[3 * i + c] = H[3 * i + c] / diag[i];
    }
    free(H);
}

/* predicted face flux: internal S.(w HbyA_P + (1-w) HbyA_N); boundary
 * U FIXED -> S.U_b, ZERO_GRAD -> S.HbyA_P, EMPTY -> 0 */
static void flux_hbya(const geom *g, const bconds *bc, const double *HbyA, double *phiH)
{
    const orc_mesh *m = g->m;
    int32_t Fi = m->n_internal;
    for (int32_t f = 0; f < Fi; ++f) {
        int32_t P = m->owner[f], Q = m->neighbour[f];
        double w = g->w[f], v[3];
        for (int c = 0; c < 3; ++c) v[c] = w * HbyA[3 * P + c] + (1.0 - w) * HbyA[3 * Q + c];
        phiH[f] = dot3(m->Sf + 3 * f, v);
    }
    for (int32_t b = 0; b < g->Fb; ++b) {
        int32_t f = Fi + b, P = m->owner[f];
        if (bc->uk[b] == BC_FIXED) phiH[f] = dot3(m->Sf + 3 * f, bc->uv + 3 * b);
        else if (bc->uk[b] == BC_ZERO_GRAD) phiH[f] = dot3(m->Sf + 3 * f, HbyA + 3 * P);
        else phiH[f] = 0.0;
    }
}

static int has_fixed_p(const bconds *bc, int32_t Fb)
{
    for (int32_t b = 0; b < Fb; ++b)
        if (bc->pk[b] == BC_FIXED) return 1;
    return 0;
}

/* ------------------------------------------------------------------------
 * Pressure system in its symmetric positive form A_p p = b_p, built from a
 * face diffusivity Gamma (internal: Gamma_f; boundary: Gamma_b):
 *   g_f = Gamma_f dl_f,  (A_p)_PN = -g_f,
 *   (A_p)_PP = sum_internal g_f + sum_{p FIXED b} g_b,
 *   b_p,P = -sum_f s_Pf phiH_f + sum_{p FIXED b} g_b p_b
 *           + sum_internal s_Pf Gamma_f k_f.(grad p)_f      (non-orthogonal)
 * With no FIXED-p face the system is pinned at cell r: A_rr doubles and
 * b_r gains the old A_rr times p_ref.
 * ---------------------------------------------------------------------- */
static void pressure_system(const geom *g, const bconds *bc, const double *gam, const double *phiH,
                            const double *gradp, int32_t pin_cell, double p_ref, double *diag, double *offd, double *bp)
{
    const orc_mesh *m = g->m;
    int32_t N = m->n_cells, Fi = m->n_internal;
    memset(diag, 0, sizeof(double) * (size_t)N);
    memset(bp, 0, sizeof(double) * (size_t)N);
    for (int32_t f = 0; f < Fi; ++f) {
        int32_t P = m->owner[f], Q = m->neighbour[f];
        double gf = gam[f] * g->dl[f];
        offd[f] = -gf;
        diag[P] += gf;
        diag[Q] += gf;
        if (phiH) { bp[P] -= phiH[f]; bp[Q] += phiH[f]; }
    }
    for (int32_t b = 0; b < g->Fb; ++b) {
        int32_t f = Fi + b, P = m->owner[f];
        if (bc->pk[b] == BC_EMPTY) continue;
        if (phiH) bp[P] -= phiH[f];
        if (bc->pk[b] == BC_FIXED) {
            double gb = gam[f] * g->dl[f];
            diag[P] += gb;
            bp[P] += gb * bc->pv[b];
        }
    }
    if (gradp && g->nonorth)
        for (int32_t f = 0; f < Fi; ++f) {
            int32_t P = m->owner[f], Q = m->neighbour[f];
            double w = g->w[f], gf[3];
            for (int d = 0; d < 3; ++d) gf[d] = w * gradp[3 * P + d] + (1.0 - w) * gradp[3 * Q + d];
            double t = gam[f] * dot3(g->k + 3 * f, gf);
            bp[P] += t;
            bp[Q] -= t;
        }
    if (pin_cell >= 0 && !has_fixed_p(bc, g->Fb)) {
        double a = diag[pin_cell];
        diag[pin_cell] = 2.0 * a;
        bp[pin_cell] += a * p_ref;
    }
}

/* Gamma from rAU: internal w rAU_P + (1-w) rAU_N, boundary rAU_P */
static void gamma_from_rau(const geom *g, const double *rAU, double *gam)
{
    const orc_mesh *m = g->m;
    int32_t Fi = m->n_internal;
    for (int32_t f = 0; f < Fi; ++f)
        gam[f] = g->w[f] * rAU[m->owner[f]] + (1.0 - g->w[f]) * rAU[m->neighbour[f]];
    for (int32_t f = Fi; f < m->n_faces; ++f) gam[f] = rAU[m->owner[f]];
}

/* conservative flux after the pressure solve:
 *   internal phi = phiH - g_f (p_N - p_P) - Gamma_f k_f.(grad p_pre)_f
 *   p FIXED  phi_b = phiH_b - g_b (p_b - p_P);   otherwise phi_b = phiH_b */
static void flux_correct(const geom *g, const bconds *bc, const double *gam, const double *phiH, const double *p,
                         const double *gradp_pre, double *phi)
{
    const orc_mesh *m = g->m;
    int32_t Fi = m->n_internal;
    for (int32_t f = 0; f < Fi; ++f) {
        int32_t P = m->owner[f], Q = m->neighbour[f];
        double v = phiH[f] - gam[f] * g->dl[f] * (p[Q] - p[P]);
        if (gradp_pre && g->nonorth) {
            double w = g->w[f], gf[3];
            for (int d = 0; d < 3; ++d) gf[d] = w * gradp_pre[3 * P + d] + (1.0 - w) * gradp_pre[3 * Q + d];
            v -= gam[f] * dot3(g->k + 3 * f, gf);
        }
        phi[f] = v;
    }
    for (int32_t b = 0; b < g->Fb; ++b) {
        int32_t f = Fi + b, P = m->owner[f];
        if (bc->pk[b] == BC_FIXED) phi[f] = phiH[f] - gam[f] * g->dl[f] * (bc->pv[b] - p[P]);
        else phi[f] = phiH[f];
    }
}

static void worst_status(int32_t *acc, int32_t s)
{
    if (s < 0) { if (*acc >= 0 || s < *acc) *acc = s; }
    else if (*acc >= 0 && s > *acc) *acc = s;
}

/* ------------------------------------------------------------------------
 * Shared pieces of one PISO step / SIMPLE iteration.
 * ---------------------------------------------------------------------- */
typedef struct {
    geom g;
    bconds bc;
    int32_t N, F, Fi;
    double *diag, *upper, *lower, *src, *rhs, *xc;
    double *gradp, *rAU, *HbyA, *phiH, *gam, *pd, *po, *bp, *U0;
} work;

static int work_init(work *w, const orc_mesh *m)
{
    memset(w, 0, sizeof(*w));
    int st = geom_init(&w->g, m);
    if (st != ST_OK) return st;
    st = bconds_from_patches(&w->bc, &w->g);
    if (st != ST_OK) return st;
    w->N = m->n_cells; w->F = m->n_faces; w->Fi = m->n_internal;
    size_t N = (size_t)w->N;
    w->diag = dalloc(N); w->upper = dalloc(w->Fi); w->lower = dalloc(w->Fi);
    w->src = dalloc(3 * N); w->rhs = dalloc(N); w->xc = dalloc(N);
    w->gradp = dalloc(3 * N); w->rAU = dalloc(N); w->HbyA = dalloc(3 * N);
    w->phiH = dalloc(w->F); w->gam = dalloc(w->F); w->pd = dalloc(N); w->po = dalloc(w->Fi);
    w->bp = dalloc(N); w->U0 = dalloc(3 * N);
    return ST_OK;
}

static void work_free(work *w)
{
    geom_free(&w->g); bconds_free(&w->bc);
    free(w->diag); free(w->upper); free(w->lower); free(w->src); free(w->rhs); free(w->xc);
    free(w->gradp); free(w->rAU); free(w->HbyA); free(w->phiH); free(w->gam); free(w->pd); free(w->po);
    free(w->bp); free(w->U0);
}

/* momentum predictor: solve each component with rhs = src - V grad p */
static int32_t momentum_solve(work *w, const orc_opts *o, double *U, orc_step_info *info)
{
    const orc_mesh *m = w->g.m;
    ldu A = {w->N, w->Fi, m->owner, m->neighbour, w->diag, w->upper, w->lower};
    int32_t st = ST_OK;
    for (int c = 0; c < 3; ++c) {
        for (int32_t i = 0; i < w->N; ++i) {
            w->rhs[i] = w->src[3 * i + c] - m->V[i] * w->gradp[3 * i + c];
            w->xc[i] = U[3 * i + c];
        }
        if (o->u_solver == 1) pbicgstab(&A, w->rhs, w->xc, o->u_tol, o->u_rel_tol, o->u_max_iter, &info->u[c]);
        else pbicg(&A, w->rhs, w->xc, o->u_tol, o->u_rel_tol, o->u_max_iter, &info->u[c]);
        worst_status(&st, info->u[c].status);
        for (int32_t i = 0; i < w->N; ++i) U[3 * i + c] = w->xc[i];
    }
    return st;
}

/* pressure corrector: H/A, flux, pressure solve(s), flux and U correction */
static int32_t pressure_corrector(work *w, const orc_opts *o, double *U, double *p, double *phi, int n_nonorth,
                                  orc_step_info *info)
{
    const orc_mesh *m = w->g.m;
    int32_t st = ST_OK;
    h_by_a(&w->g, w->diag, w->upper, w->lower, w->src, U, w->rAU, w->HbyA);
    flux_hbya(&w->g, &w->bc, w->HbyA, w->phiH);
    gamma_from_rau(&w->g, w->rAU, w->gam);
    ldu Ap = {w->N, w->Fi, m->owner, m->neighbour, w->pd, w->po, w->po};
    for (int k = 0; k <= n_nonorth; ++k) {
        grad_gauss(&w->g, p, 1, w->bc.pk, w->bc.pv, 1, w->gradp);
        pressure_system(&w->g, &w->bc, w->gam, w->phiH, w->gradp, o->p_ref_cell, o->p_ref_value, w->pd, w->po, w->bp);
        orc_solve_info *si = &info->p[info->n_p_solves < 16 ? info->n_p_solves : 15];
        pcg(&Ap, w->bp, p, o->p_tol, o->p_rel_tol, o->p_max_iter, o->p_precond, si);
        if (info->n_p_solves < 16) info->n_p_solves++;
        worst_status(&st, si->status);
        if (st < 0) return st;
        if (k == n_nonorth) flux_correct(&w->g, &w->bc, w->gam, w->phiH, p, w->gradp, phi);
    }
    grad_gauss(&w->g, p, 1, w->bc.pk, w->bc.pv, 1, w->gradp);
    for (int32_t i = 0; i < w->N; ++i)
        for (int c = 0; c < 3; ++c) U[3 * i + c] = w->HbyA[3 * i + c] - w->rAU[i] * w->gradp[3 * i + c];
    return st;
}

/* ========================================================================
 * Exported entry points
 * ====================================================================== */

/* face flux of a velocity field: internal S.(w U_P + (1-w) U_N); boundary
 * FIXED S.U_b, ZERO_GRAD S.U_P, EMPTY 0 */
int orc_flux_from_U(const orc_mesh *m, const double *U, double *phi)
{
    geom g; bconds bc;
    int st = geom_init(&g, m);
    if (st == ST_OK) st = bconds_from_patches(&bc, &g);
    if (st != ST_OK) return st;
    flux_hbya(&g, &bc, U, phi);
    geom_free(&g); bconds_free(&bc);
    return ST_OK;
}

int orc_face_coeffs(const orc_mesh *m, double *w, double *dl, double *k, int32_t *nonorth)
{
    geom g;
    int st = geom_init(&g, m);
    if (st != ST_OK) { geom_free(&g); return st; }
    memcpy(w, g.w, sizeof(double) * (size_t)m->n_internal);
    memcpy(dl, g.dl, sizeof(double) * (size_t)m->n_faces);
    memcpy(k, g.k, sizeof(double) * 3 * (size_t)m->n_internal);
    *nonorth = g.nonorth;
    geom_free(&g);
    return ST_OK;
}

/* gradient of a cell scalar with explicit per-boundary-face kinds/values */
int orc_grad(const orc_mesh *m, const double *phi, const int32_t *bkind, const double *bval, double *grad)
{
    geom g;
    int st = geom_init(&g, m);
    if (st == ST_OK) grad_gauss(&g, phi, 1, bkind, bval, 1, grad);
    geom_free(&g);
    return st;
}

/* momentum matrix with the patch BCs; dt <= 0 means steady (no ddt) */
int orc_momentum_system(const orc_mesh *m, double nu, double dt, int32_t convection, const double *phi,
                        const double *U_old, const double *U_grad, double *diag, double *upper, double *lower,
                        double *src)
{
    geom g; bconds bc;
    int st = geom_init(&g, m);
    if (st == ST_OK) st = bconds_from_patches(&bc, &g);
    if (st != ST_OK) return st;
    momentum_system(&g, &bc, nu, dt, convection, phi, U_old, U_grad, diag, upper, lower, src);
    geom_free(&g); bconds_free(&bc);
    return ST_OK;
}

/* pressure system from a face diffusivity with explicit p boundary
 * kinds/values (pin_cell < 0: no pin); phiH and gradp may be NULL */
int orc_pressure_system(const orc_mesh *m, const double *gam, const double *phiH, const double *gradp,
                        const int32_t *pbkind, const double *pbval, int32_t pin_cell, double p_ref, double *diag,
                        double *offd, double *bp)
{
    geom g;
    int st = geom_init(&g, m);
    if (st != ST_OK) { geom_free(&g); return st; }
    bconds bc;
    bc.pk = (int32_t *)pbkind; bc.pv = (double *)pbval; bc.uk = NULL; bc.uv = NULL;
    pressure_system(&g, &bc, gam, phiH, gradp, pin_cell, p_ref, diag, offd, bp);
    geom_free(&g);
    return ST_OK;
}

int orc_amul(int32_t N, int32_t Fi, const int32_t *own, const int32_t *nei, const double *diag, const double *upper,
             const double *lower, const double *x, double *y, int32_t transpose)
{
    ldu A = {N, Fi, own, nei, diag, upper, lower};
    if (transpose) tmul(&A, x, y); else amul(&A, x, y);
    return ST_OK;
}

int orc_pcg(int32_t N, int32_t Fi, const int32_t *own, const int32_t *nei, const double *diag, const double *offd,
            const double *b, double *x, double tol, double rel_tol, int32_t max_iter, int32_t precond,
            orc_solve_info *info)
{
    ldu A = {N, Fi, own, nei, diag, offd, offd};
    return pcg(&A, b, x, tol, rel_tol, max_iter, precond, info);
}

int orc_pbicg(int32_t N, int32_t Fi, const int32_t *own, const int32_t *nei, const double *diag, const double *upper,
              const double *lower, const double *b, double *x, double tol, double rel_tol, int32_t max_iter,
              orc_solve_info *info)
{
    ldu A = {N, Fi, own, nei, diag, upper, lower};
    return pbicg(&A, b, x, tol, rel_tol, max_iter, info);
}

int orc_pbicgstab(int32_t N, int32_t Fi, const int32_t *own, const int32_t *nei, const double *diag, const double *upper,
              const double *lower, const double *b, double *x, double tol, double rel_tol, int32_t max_iter,
              orc_solve_info *info)
{
    ldu A = {N, Fi, own, nei, diag, upper, lower};
    return pbicgstab(&A, b, x, tol, rel_tol, max_iter, info);
}

int orc_dic(int32_t N, int32_t Fi, const int32_t *own, const int32_t *nei, const double *diag, const double *offd,
            const double *r, double *dstar, double *z)
{
    ldu A = {N, Fi, own, nei, diag, offd, offd};
    dic D;
    int st = dic_init(&D, &A);
    if (st == ST_OK) {
        memcpy(dstar, D.dstar, sizeof(double) * (size_t)N);
        if (r && z) dic_apply(&D, &A, r, z);
    }
    dic_free(&D);
    return st;
}

/* normalised residual sum|b - A x| / n_f of a face-addressed system */
double orc_nres(int32_t N, int32_t Fi, const int32_t *own, const int32_t *nei, const double *diag,
                const double *upper, const double *lower, const double *b, const double *x)
{
    ldu A = {N, Fi, own, nei, diag, upper, lower};
    double *Ax = dalloc(N), s = 0.0;
    amul(&A, x, Ax);
    double nf = norm_factor(&A, x, b, Ax);
    for (int32_t i = 0; i < N; ++i) s += fabs(b[i] - Ax[i]);
    free(Ax);
    return s / nf;
}

/* ------------------------------------------------------------------------
 * PISO (transient, Section 3): per step
 *   1. momentum matrix from (phi, U_old) incl. V/dt, predictor solve with
 *      rhs = src - V grad p;
 *   2. n_corr times: H/A, predicted flux, pressure system + CG (repeated
 *      n_non_orth_corr + 1 times), conservative flux, U = HbyA - rAU grad p.
 * U[N][3], p[N], phi[F] are advanced in place.  `last` receives the solver
 * record of the final step.
 * ---------------------------------------------------------------------- */
int orc_piso(const orc_mesh *m, const orc_opts *o, double *U, double *p, double *phi, int32_t n_steps,
             orc_step_info *last)
{
    work w;
    int st = work_init(&w, m);
    if (st != ST_OK) { work_free(&w); return st; }
    int32_t worst = ST_OK;
    for (int32_t s = 0; s < n_steps; ++s) {
        orc_step_info info;
        memset(&info, 0, sizeof(info));
        int32_t sst = ST_OK;
        memcpy(w.U0, U, sizeof(double) * 3 * (size_t)w.N);
        momentum_system(&w.g, &w.bc, o->nu, o->dt, o->convection, phi, w.U0, w.U0, w.diag, w.upper, w.lower, w.src);
        grad_gauss(&w.g, p, 1, w.bc.pk, w.bc.pv, 1, w.gradp);
        worst_status(&sst, momentum_solve(&w, o, U, &info));
        if (sst >= 0)
            for (int32_t c = 0; c < o->n_corr; ++c) {
                worst_status(&sst, pressure_corrector(&w, o, U, p, phi, o->n_non_orth_corr, &info));
                if (sst < 0) break;
            }
        info.status = sst;
        if (last) *last = info;
        worst_status(&worst, sst);
        if (sst < 0) break;
    }
    work_free(&w);
    return worst;
}

/* ------------------------------------------------------------------------
 * SIMPLE (steady, Section 3): per iteration
 *   momentum matrix without ddt, implicit relaxation
 *     a_PP <- a_PP/alpha_U,  src += (1-alpha_U)/alpha_U a_PP,orig U_prev,
 *   predictor (records the three initial residuals), H/A with the relaxed
 *   diagonal, pressure system (non-orthogonal part from the current p) and
 *   CG (records p's initial residual), conservative flux, explicit p
 *   relaxation p = p_prev + alpha_p (p - p_prev), U = HbyA - rAU grad p.
 * Stops once all four initial residuals are <= res_tol, or after max_iters.
 * ---------------------------------------------------------------------- */
int orc_simple(const orc_mesh *m, const orc_opts *o, double *U, double *p, double *phi, int32_t max_iters,
               double res_tol, int32_t *iters_done, orc_step_info *last)
{
    work w;
    int st = work_init(&w, m);
    if (st != ST_OK) { work_free(&w); return st; }
    double *p_prev = dalloc((size_t)w.N);
    int32_t worst = ST_OK, it;
    for (it = 0; it < max_iters; ++it) {
        orc_step_info info;
        memset(&info, 0, sizeof(info));
        int32_t sst = ST_OK;
        memcpy(w.U0, U, sizeof(double) * 3 * (size_t)w.N);
        momentum_system(&w.g, &w.bc, o->nu, 0.0, o->convection, phi, NULL, w.U0, w.diag, w.upper, w.lower, w.src);
        for (int32_t i = 0; i < w.N; ++i) {
            double d0 = w.diag[i];
            w.diag[i] = d0 / o->alpha_u;
            for (int c = 0; c < 3; ++c) w.src[3 * i + c] += (1.0 - o->alpha_u) / o->alpha_u * d0 * w.U0[3 * i + c];
        }
        grad_gauss(&w.g, p, 1, w.bc.pk, w.bc.pv, 1, w.gradp);
        worst_status(&sst, momentum_solve(&w, o, U, &info));
        if (sst >= 0) {
            memcpy(p_prev, p, sizeof(double) * (size_t)w.N);
            h_by_a(&w.g, w.diag, w.upper, w.lower, w.src, U, w.rAU, w.HbyA);
            flux_hbya(&w.g, &w.bc, w.HbyA, w.phiH);
            gamma_from_rau(&w.g, w.rAU, w.gam);
            grad_gauss(&w.g, p, 1, w.bc.pk, w.bc.pv, 1, w.gradp);
            pressure_system(&w.g, &w.bc, w.gam, w.phiH, w.gradp, o->p_ref_cell, o->p_ref_value, w.pd, w.po, w.bp);
            ldu Ap = {w.N, w.Fi, m->owner, m->neighbour, w.pd, w.po, w.po};
            pcg(&Ap, w.bp, p, o->p_tol, o->p_rel_tol, o->p_max_iter, o->p_precond, &info.p[0]);
            info.n_p_solves = 1;
            worst_status(&sst, info.p[0].status);
            if (sst >= 0) {
                flux_correct(&w.g, &w.bc, w.gam, w.phiH, p, w.gradp, phi);
                for (int32_t i = 0; i < w.N; ++i) p[i] = p_prev[i] + o->alpha_p * (p[i] - p_prev[i]);
                grad_gauss(&w.g, p, 1, w.bc.pk, w.bc.pv, 1, w.gradp);
                for (int32_t i = 0; i < w.N; ++i)
                    for (int c = 0; c < 3; ++c) U[3 * i + c] = w.HbyA[3 * i + c] - w.rAU[i] * w.gradp[3 * i + c];
            }
        }
        info.status = sst;
        if (last) *last = info;
        worst_status(&worst, sst);
        if (sst < 0) { ++it; break; }
        if (info.u[0].res_initial <= res_tol && info.u[1].res_initial <= res_tol && info.u[2].res_initial <= res_tol &&
            info.p[0].res_initial <= res_tol) { ++it; break; }
    }
    if (iters_done) *iters_done = it;
    free(p_prev);
    work_free(&w);
    return worst;
}

/* ------------------------------------------------------------------------
 * Stand-alone pressure solve: the symmetric system built from a given face
 * diffusivity gamma[F] (in place of interpolated rAU) and the mesh's p
 * patches, right-hand side b = rhs + fixed-p boundary terms (no
 * non-orthogonal part), pinned at opts->p_ref_cell when no p patch is FIXED;
 * CG with the given controls, starting from p.
 * ---------------------------------------------------------------------- */
int orc_solve_pressure(const orc_mesh *m, const orc_opts *o, const double *gam, const double *rhs, double *p,
                       double tol, double rel_tol, int32_t max_iter, int32_t precond, orc_solve_info *info)
{
    work w;
    int st = work_init(&w, m);
    if (st != ST_OK) { work_free(&w); return st; }
    pressure_system(&w.g, &w.bc, gam, NULL, NULL, o->p_ref_cell, o->p_ref_value, w.pd, w.po, w.bp);
    for (int32_t i = 0; i < w.N; ++i) w.bp[i] += rhs[i];
    ldu Ap = {w.N, w.Fi, m->owner, m->neighbour, w.pd, w.po, w.po};
    st = pcg(&Ap, w.bp, p, tol, rel_tol, max_iter, precond, info);
    work_free(&w);
    return st;
}
