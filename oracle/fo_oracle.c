/*
 * FP64 CPU oracle for the level-set compliance hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the benchmark's CPU
 * baseline leg use it.  It shares no code with the HIP implementation.
 *
 * It is written to be obviously correct rather than fast: explicit element
 * matrices from their definitions, assembly into a compressed-row matrix,
 * elimination of clamped unknowns by extracting the free sub-matrix, and a
 * textbook Jacobi-preconditioned conjugate gradient method.  All arithmetic
 * is double precision.  OpenMP is used only for the sparse matrix-vector
 * product and the vector reductions of the solver.
 *
 * Paper sections followed (arXiv 2601.05709):
 *   - linear elasticity: strain/stress and the stiffness tensor C_ijkl
 *     (Section "Shape derivative for a model problem");
 *   - level-set domain Omega = {phi < 0}  (Section "Main algorithm", eq. subdomain);
 *   - compliance state problem, cost, ersatz coefficient A_Omega, and the
 *     derivative tensors S1^J, S1^C (Section "Compliance minimization",
 *     eqs. compli_cost, compli_weak, compli_AOmega and the S0/S1 display);
 *   - S1 = S1^J + lambda S1^C (Section "Lagrangian method", eq. S0andS1);
 *   - velocity problem B(theta, xi) = -dJ(xi) with the bilinear form of
 *     eq. compli1_bili: mass + gradient term + subdomain penalty (eq. sub_dom)
 *     + boundary normal penalty (eq. bd_plt)  (Section "Velocity");
 *   - level-set transport theta . grad(phi) (eq. transport), advanced by one
 *     explicit step with a recovered nodal gradient;
 *   - the paper's own transport step (Section "Transport equation", eqs.
 *     transport, weak_transport, tau_lv): Petrov-Galerkin test functions
 *     psi + tau theta . grad psi, Crank-Nicolson in time, optional h^2
 *     diffusion; each time step solved by Jacobi-preconditioned BiCGStab.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OC_MAXV 4 /* vertices of a simplex, d <= 3 */

/* ------------------------------------------------------------------------ */
/* geometry of one P1 simplex                                               */

/* Barycentric gradients g[a][i] = d lambda_a / d x_i and measure |T| of
 * element e.  lambda_a(x) = c_a + g_a . x with lambda_a(x_b) = delta_ab, so
 * the coefficients are the columns of the inverse of the (d+1)x(d+1) matrix
 * whose row b is [1, x_b].  Inverse by Gauss-Jordan with partial pivoting;
 * |T| = |det| / d!.  Returns 0 on success, -1 for a degenerate element. */
static int oc_simplex(int dim, const double *coords, const int32_t *conn, int64_t E,
                      int64_t e, double g[OC_MAXV][3], double *vol)
{
    int n = dim + 1;
    double M[OC_MAXV][2 * OC_MAXV];
    for (int b = 0; b < n; ++b) {
        int64_t node = conn[(int64_t)b * E + e];
        M[b][0] = 1.0;
        for (int i = 0; i < dim; ++i) M[b][1 + i] = coords[node * dim + i];
        for (int c = 0; c < n; ++c) M[b][n + c] = (b == c) ? 1.0 : 0.0;
    }
    double det = 1.0;
    for (int col = 0; col < n; ++col) {
        int piv = col;
        for (int r = col + 1; r < n; ++r)
            if (fabs(M[r][col]) > fabs(M[piv][col])) piv = r;
        if (M[piv][col] == 0.0) return -1;
        if (piv != col) {
            for (int c = 0; c < 2 * n; ++c) {
                double t = M[col][c];
                M[col][c] = M[piv][c];
                M[piv][c] = t;
            }
            det = -det;
        }
        double p = M[col][col];
        det *= p;
        for (int c = 0; c < 2 * n; ++c) M[col][c] /= p;
        for (int r = 0; r < n; ++r) {
            if (r == col) continue;
            double f = M[r][col];
            if (f == 0.0) continue;
            for (int c = 0; c < 2 * n; ++c) M[r][c] -= f * M[col][c];
        }
    }
    /* inverse = right half; row (1+i), column a is d lambda_a / d x_i */
    for (int a = 0; a < n; ++a)
        for (int i = 0; i < dim; ++i) g[a][i] = M[1 + i][n + a];
    double fact = (dim == 2) ? 2.0 : 6.0;
    *vol = fabs(det) / fact;
    return 0;
}

/* Measure of a boundary facet (segment in 2D, triangle in 3D). */
static double oc_facet_measure(int dim, const double *coords, const int32_t *bf, int64_t F,
                               int64_t f)
{
    const double *p0 = coords + (int64_t)bf[f] * dim;
    const double *p1 = coords + (int64_t)bf[F + f] * dim;
    if (dim == 2) {
        double dx = p1[0] - p0[0], dy = p1[1] - p0[1];
        return sqrt(dx * dx + dy * dy);
    }
    const double *p2 = coords + (int64_t)bf[2 * F + f] * dim;
    double u[3], v[3], c[3];
    for (int i = 0; i < 3; ++i) {
        u[i] = p1[i] - p0[i];
        v[i] = p2[i] - p0[i];
    }
    c[0] = u[1] * v[2] - u[2] * v[1];
    c[1] = u[2] * v[0] - u[0] * v[2];
    c[2] = u[0] * v[1] - u[1] * v[0];
    return 0.5 * sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
}

/* ------------------------------------------------------------------------ */
/* material and level-set coefficient                                       */

/* Lame parameters from Young's modulus and Poisson ratio.  In 2D plane
 * stress the first parameter is replaced by E nu / (1 - nu^2). */
void oc_lame(double E, double nu, int dim, int plane_stress, double *lam, double *mu)
{
    *mu = E / (2.0 * (1.0 + nu));
    if (dim == 2 && plane_stress)
        *lam = E * nu / (1.0 - nu * nu);
    else
        *lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
}

/* A_e = 1 where the element lies in Omega = {phi < 0}, judged by the value of
 * the P1 level set at the element centroid (the vertex mean), else the ersatz
 * weight; chi_e is the indicator of Omega.  A tie at 0 is outside Omega. */
void oc_element_coef(int dim, int64_t E, const int32_t *conn, const double *phi, double ersatz,
                     double *A, double *chi)
{
    for (int64_t e = 0; e < E; ++e) {
        double s = 0.0;
        for (int a = 0; a <= dim; ++a) s += phi[conn[(int64_t)a * E + e]];
        double mean = s / (double)(dim + 1);
        int inside = mean < 0.0;
        A[e] = inside ? 1.0 : ersatz;
        chi[e] = inside ? 1.0 : 0.0;
    }
}

/* ------------------------------------------------------------------------ */
/* compressed-row matrices                                                  */

typedef struct {
    int64_t n;       /* rows = columns */
    int64_t *rowptr; /* n + 1 */
    int64_t *col;    /* nnz */
    double *val;     /* nnz */
    int dim;         /* unknowns per node */
    int64_t *nadj_ptr; /* node adjacency (sorted), for locating entries */
    int64_t *nadj;
} oc_csr;

static int cmp_i64(const void *a, const void *b)
{
    int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    return (x > y) - (x < y);
}

/* Sparsity of a vector P1 operator: row (n, i) couples to (m, j) for every
 * node m sharing an element with n (or n itself) and every component j. */
static oc_csr *oc_csr_structure(int dim, int64_t N, int64_t E, const int32_t *conn,
                                int64_t nbf, const int32_t *bfacets)
{
    int nv = dim + 1;
    int64_t *cnt = calloc((size_t)N + 1, sizeof(int64_t));
    for (int64_t e = 0; e < E; ++e)
        for (int a = 0; a < nv; ++a) cnt[conn[(int64_t)a * E + e] + 1] += nv;
    for (int64_t f = 0; f < nbf; ++f)
        for (int a = 0; a < dim; ++a) cnt[bfacets[(int64_t)a * nbf + f] + 1] += dim;
    for (int64_t n = 0; n < N; ++n) cnt[n + 1] += cnt[n];
    int64_t *lst = malloc((size_t)cnt[N] * sizeof(int64_t));
    int64_t *fill = malloc((size_t)N * sizeof(int64_t));
    memcpy(fill, cnt, (size_t)N * sizeof(int64_t));
    for (int64_t e = 0; e < E; ++e)
        for (int a = 0; a < nv; ++a) {
            int64_t na = conn[(int64_t)a * E + e];
            for (int b = 0; b < nv; ++b) lst[fill[na]++] = conn[(int64_t)b * E + e];
        }
    for (int64_t f = 0; f < nbf; ++f)
        for (int a = 0; a < dim; ++a) {
            int64_t na = bfacets[(int64_t)a * nbf + f];
            for (int b = 0; b < dim; ++b) lst[fill[na]++] = bfacets[(int64_t)b * nbf + f];
        }
    /* sort + unique each node's list */
    int64_t *uptr = calloc((size_t)N + 1, sizeof(int64_t));
    for (int64_t n = 0; n < N; ++n) {
        int64_t s = cnt[n], len = cnt[n + 1] - cnt[n];
        qsort(lst + s, (size_t)len, sizeof(int64_t), cmp_i64);
        int64_t u = 0;
        for (int64_t k = 0; k < len; ++k)
            if (k == 0 || lst[s + k] != lst[s + k - 1]) lst[s + u++] = lst[s + k];
        uptr[n + 1] = u;
    }
    for (int64_t n = 0; n < N; ++n) uptr[n + 1] += uptr[n];
    int64_t *adj = malloc((size_t)uptr[N] * sizeof(int64_t));
    for (int64_t n = 0; n < N; ++n)
        memcpy(adj + uptr[n], lst + cnt[n], (size_t)(uptr[n + 1] - uptr[n]) * sizeof(int64_t));
    free(lst);
    free(fill);
    free(cnt);

    oc_csr *A = calloc(1, sizeof(oc_csr));
    A->dim = dim;
    A->n = N * dim;
    A->nadj_ptr = uptr;
    A->nadj = adj;
    A->rowptr = malloc((size_t)(A->n + 1) * sizeof(int64_t));
    A->rowptr[0] = 0;
    for (int64_t n = 0; n < N; ++n)
        for (int i = 0; i < dim; ++i) {
            int64_t r = n * dim + i;
            A->rowptr[r + 1] = A->rowptr[r] + (uptr[n + 1] - uptr[n]) * dim;
        }
    int64_t nnz = A->rowptr[A->n];
    A->col = malloc((size_t)nnz * sizeof(int64_t));
    A->val = calloc((size_t)nnz, sizeof(double));
    for (int64_t n = 0; n < N; ++n)
        for (int i = 0; i < dim; ++i) {
            int64_t r = n * dim + i, p = A->rowptr[r];
            for (int64_t k = uptr[n]; k < uptr[n + 1]; ++k)
                for (int j = 0; j < dim; ++j) A->col[p++] = adj[k] * dim + j;
        }
    return A;
}

/* Add v to entry (row dof (na, i), column dof (nb, j)). */
static void oc_csr_add(oc_csr *A, int64_t na, int i, int64_t nb, int j, double v)
{
    int64_t lo = A->nadj_ptr[na], hi = A->nadj_ptr[na + 1] - 1;
    while (lo <= hi) { /* binary search for nb in the adjacency of na */
        int64_t mid = (lo + hi) / 2;
        if (A->nadj[mid] == nb) {
            int64_t pos = A->rowptr[na * A->dim + i] + (mid - A->nadj_ptr[na]) * A->dim + j;
            A->val[pos] += v;
            return;
        }
        if (A->nadj[mid] < nb) lo = mid + 1;
        else hi = mid - 1;
    }
    fprintf(stderr, "oc_csr_add: entry (%lld,%lld) outside the sparsity pattern\n",
            (long long)na, (long long)nb);
    abort();
}

void oc_csr_free(oc_csr *A)
{
    if (!A) return;
    free(A->rowptr);
    free(A->col);
    free(A->val);
    free(A->nadj_ptr);
    free(A->nadj);
    free(A);
}

int64_t oc_csr_rows(const oc_csr *A) { return A->n; }
int64_t oc_csr_nnz(const oc_csr *A) { return A->rowptr[A->n]; }

void oc_csr_export(const oc_csr *A, int64_t *rowptr, int64_t *col, double *val)
{
    memcpy(rowptr, A->rowptr, (size_t)(A->n + 1) * sizeof(int64_t));
    memcpy(col, A->col, (size_t)oc_csr_nnz(A) * sizeof(int64_t));
    memcpy(val, A->val, (size_t)oc_csr_nnz(A) * sizeof(double));
}

void oc_csr_matvec(const oc_csr *A, const double *x, double *y)
{
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < A->n; ++r) {
        double s = 0.0;
        for (int64_t k = A->rowptr[r]; k < A->rowptr[r + 1]; ++k) s += A->val[k] * x[A->col[k]];
        y[r] = s;
    }
}

/* ------------------------------------------------------------------------ */
/* operators                                                                 */

/* Level-set-weighted P1 elasticity stiffness:
 *   K = sum_e A_e K_e,
 *   K_e[(a,i),(b,j)] = |T_e| C_ikjl g_ak g_bl
 *                    = |T_e| [lam g_ai g_bj + mu (g_aj g_bi + delta_ij g_a . g_b)],
 * which is the element integral of A sigma(N_b e_j) : eps(N_a e_i).
 * Returns NULL if an element is degenerate. */
oc_csr *oc_assemble_elasticity(int dim, int64_t N, int64_t E, const double *coords,
                               const int32_t *conn, const double *A_e, double lam, double mu)
{
    oc_csr *K = oc_csr_structure(dim, N, E, conn, 0, NULL);
    int nv = dim + 1;
    for (int64_t e = 0; e < E; ++e) {
        double g[OC_MAXV][3], vol;
        if (oc_simplex(dim, coords, conn, E, e, g, &vol)) {
            oc_csr_free(K);
            return NULL;
        }
        double w = vol * A_e[e];
        for (int a = 0; a < nv; ++a)
            for (int b = 0; b < nv; ++b) {
                double gab = 0.0;
                for (int k = 0; k < dim; ++k) gab += g[a][k] * g[b][k];
                for (int i = 0; i < dim; ++i)
                    for (int j = 0; j < dim; ++j) {
                        double v = lam * g[a][i] * g[b][j] + mu * g[a][j] * g[b][i];
                        if (i == j) v += mu * gab;
                        oc_csr_add(K, conn[(int64_t)a * E + e], i, conn[(int64_t)b * E + e], j,
                                   w * v);
                    }
            }
    }
    return K;
}

/* Velocity bilinear form (eq. compli1_bili with the weights as parameters):
 *   B(theta, xi) = alpha int theta.xi + int D theta : D xi
 *                + gamma_s int chi_Omega0 theta.xi
 *                + gamma_n int_{boundary} (theta.n)(xi.n).
 * P1 element mass |T|(1+delta_ab)/((d+1)(d+2)); facet mass
 * |F|(1+delta_ab)/(d(d+1)); chi_Omega0 is 1 on elements whose centroid lies
 * strictly inside one of the boxes [lo_0,hi_0]x...  (boxes[k] = lo..., hi...). */
oc_csr *oc_assemble_descent(int dim, int64_t N, int64_t E, const double *coords,
                            const int32_t *conn, int64_t nbf, const int32_t *bfacets,
                            const double *bnormal, double alpha, double gamma_n, double gamma_s,
                            int n_boxes, const double *boxes)
{
    oc_csr *B = oc_csr_structure(dim, N, E, conn, nbf, bfacets);
    int nv = dim + 1;
    double mass_den = (double)((dim + 1) * (dim + 2));
    for (int64_t e = 0; e < E; ++e) {
        double g[OC_MAXV][3], vol;
        if (oc_simplex(dim, coords, conn, E, e, g, &vol)) {
            oc_csr_free(B);
            return NULL;
        }
        double cen[3] = {0, 0, 0};
        for (int a = 0; a < nv; ++a)
            for (int i = 0; i < dim; ++i) cen[i] += coords[(int64_t)conn[(int64_t)a * E + e] * dim + i];
        for (int i = 0; i < dim; ++i) cen[i] /= (double)nv;
        int in0 = 0;
        for (int k = 0; k < n_boxes && !in0; ++k) {
            int ok = 1;
            for (int i = 0; i < dim; ++i) {
                double lo = boxes[k * 2 * dim + i], hi = boxes[k * 2 * dim + dim + i];
                if (!(cen[i] > lo && cen[i] < hi)) ok = 0;
            }
            in0 = ok;
        }
        double mw = alpha + (in0 ? gamma_s : 0.0);
        for (int a = 0; a < nv; ++a)
            for (int b = 0; b < nv; ++b) {
                double m = vol * (a == b ? 2.0 : 1.0) / mass_den;
                double lap = 0.0;
                for (int k = 0; k < dim; ++k) lap += g[a][k] * g[b][k];
                lap *= vol;
                for (int i = 0; i < dim; ++i)
                    oc_csr_add(B, conn[(int64_t)a * E + e], i, conn[(int64_t)b * E + e], i,
                               mw * m + lap);
            }
    }
    double fden = (double)(dim * (dim + 1));
    for (int64_t f = 0; f < nbf; ++f) {
        double area = oc_facet_measure(dim, coords, bfacets, nbf, f);
        const double *n = bnormal + f * dim;
        for (int a = 0; a < dim; ++a)
            for (int b = 0; b < dim; ++b) {
                double m = area * (a == b ? 2.0 : 1.0) / fden;
                for (int i = 0; i < dim; ++i)
                    for (int j = 0; j < dim; ++j)
                        oc_csr_add(B, bfacets[(int64_t)a * nbf + f], i, bfacets[(int64_t)b * nbf + f],
                                   j, gamma_n * m * n[i] * n[j]);
            }
    }
    return B;
}

/* Sub-matrix on the unknowns with keep[r] != 0 (clamped unknowns eliminated). */
oc_csr *oc_csr_restrict(const oc_csr *A, const uint8_t *keep, int64_t *map_out)
{
    int64_t *map = map_out;
    int64_t m = 0;
    for (int64_t r = 0; r < A->n; ++r) map[r] = keep[r] ? m++ : -1;
    oc_csr *S = calloc(1, sizeof(oc_csr));
    S->n = m;
    S->dim = 0;
    S->rowptr = malloc((size_t)(m + 1) * sizeof(int64_t));
    S->rowptr[0] = 0;
    int64_t nnz = 0;
    for (int64_t r = 0; r < A->n; ++r) {
        if (map[r] < 0) continue;
        for (int64_t k = A->rowptr[r]; k < A->rowptr[r + 1]; ++k)
            if (map[A->col[k]] >= 0) ++nnz;
        S->rowptr[map[r] + 1] = nnz;
    }
    S->col = malloc((size_t)nnz * sizeof(int64_t));
    S->val = malloc((size_t)nnz * sizeof(double));
    int64_t p = 0;
    for (int64_t r = 0; r < A->n; ++r) {
        if (map[r] < 0) continue;
        for (int64_t k = A->rowptr[r]; k < A->rowptr[r + 1]; ++k)
            if (map[A->col[k]] >= 0) {
                S->col[p] = map[A->col[k]];
                S->val[p] = A->val[k];
                ++p;
            }
    }
    return S;
}

/* ------------------------------------------------------------------------ */
/* Jacobi-preconditioned conjugate gradients                                */

static double oc_dot(int64_t n, const double *x, const double *y)
{
    double s = 0.0;
#pragma omp parallel for reduction(+ : s) schedule(static)
    for (int64_t i = 0; i < n; ++i) s += x[i] * y[i];
    return s;
}

/* Solve A x = b from x = 0 until ||b - A x||_2 <= rtol ||b||_2, where the
 * stopping test uses the recomputed (true) residual.  Returns the number of
 * operator applications; *relres receives the final true relative residual.
 * status: 0 converged, 1 iteration limit, -5 breakdown (p.Ap <= 0 or NaN). */
int64_t oc_pcg(const oc_csr *A, const double *b, double *x, double rtol, int64_t max_iter,
               double *relres, int *status)
{
    int64_t n = A->n;
    double *r = malloc((size_t)n * sizeof(double));
    double *z = malloc((size_t)n * sizeof(double));
    double *p = malloc((size_t)n * sizeof(double));
    double *q = malloc((size_t)n * sizeof(double));
    double *dinv = malloc((size_t)n * sizeof(double));
    for (int64_t i = 0; i < n; ++i) {
        double d = 0.0;
        for (int64_t k = A->rowptr[i]; k < A->rowptr[i + 1]; ++k)
            if (A->col[k] == i) d = A->val[k];
        dinv[i] = d != 0.0 ? 1.0 / d : 0.0;
        x[i] = 0.0;
    }
    double bnorm = sqrt(oc_dot(n, b, b));
    int64_t it = 0;
    *status = 1;
    if (bnorm == 0.0) {
        *relres = 0.0;
        *status = 0;
        goto done;
    }
    for (int restart = 0; restart < 50; ++restart) {
        /* r = b - A x (true residual) */
        oc_csr_matvec(A, x, q);
        if (restart > 0) ++it;
        for (int64_t i = 0; i < n; ++i) r[i] = b[i] - q[i];
        double rn = sqrt(oc_dot(n, r, r));
        *relres = rn / bnorm;
        if (!(rn == rn)) {
            *status = -5;
            goto done;
        }
        if (rn <= rtol * bnorm) {
            *status = 0;
            goto done;
        }
        if (it >= max_iter) goto done;
        for (int64_t i = 0; i < n; ++i) {
            z[i] = dinv[i] * r[i];
            p[i] = z[i];
        }
        double rho = oc_dot(n, r, z);
        while (it < max_iter) {
            oc_csr_matvec(A, p, q);
            ++it;
            double pq = oc_dot(n, p, q);
            if (!(pq > 0.0)) {
                *status = -5;
                goto done;
            }
            double alpha = rho / pq;
#pragma omp parallel for schedule(static)
            for (int64_t i = 0; i < n; ++i) {
                x[i] += alpha * p[i];
                r[i] -= alpha * q[i];
                z[i] = dinv[i] * r[i];
            }
            double rr = oc_dot(n, r, r);
            if (sqrt(rr) <= rtol * bnorm) break; /* verify with the true residual */
            double rho_new = oc_dot(n, r, z);
            double beta = rho_new / rho;
            rho = rho_new;
#pragma omp parallel for schedule(static)
            for (int64_t i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
        }
    }
done:
    free(r);
    free(z);
    free(p);
    free(q);
    free(dinv);
    return it;
}

/* State problem with clamped unknowns eliminated: K_ff u_f = b_f, u = 0 on
 * the clamped unknowns.  Returns iterations (operator applications). */
int64_t oc_solve_constrained(const oc_csr *K, const uint8_t *fixed, const double *b, double *u,
                             double rtol, int64_t max_iter, double *relres, int *status)
{
    int64_t n = K->n;
    uint8_t *keep = calloc((size_t)(n ? n : 1), 1);
    for (int64_t i = 0; i < n; ++i) keep[i] = fixed ? (uint8_t)!fixed[i] : 1;
    int64_t *map = malloc((size_t)n * sizeof(int64_t));
    oc_csr *S = oc_csr_restrict(K, keep, map);
    double *bf = malloc((size_t)(S->n ? S->n : 1) * sizeof(double));
    double *uf = malloc((size_t)(S->n ? S->n : 1) * sizeof(double));
    for (int64_t i = 0; i < n; ++i)
        if (map[i] >= 0) bf[map[i]] = b[i];
    int64_t it = oc_pcg(S, bf, uf, rtol, max_iter, relres, status);
    for (int64_t i = 0; i < n; ++i) u[i] = map[i] >= 0 ? uf[map[i]] : 0.0;
    free(bf);
    free(uf);
    free(map);
    free(keep);
    oc_csr_free(S);
    return it;
}

/* ------------------------------------------------------------------------ */
/* shape derivative of the compliance                                       */

/* For each load case k (column k of u, leading dimension ld):
 *   Du_e = sum_a u_a (x) g_a,  eps = sym Du,  sigma = lam tr(eps) I + 2 mu eps,
 *   S1_e = A_e (2 Du^T sigma - (sigma : eps) I)  +  lambda_vol chi_e I / V,
 *   rhs_{a,i} = - sum_e |T_e| (S1_e g_a)_i     (summed over the load cases),
 *   J_k = sum_e A_e |T_e| sigma : eps           (compliance of case k),
 *   vol = sum_e chi_e |T_e|.
 * The volume term lambda_vol chi I / V enters once (not per load case).
 * S1 (nullable) receives the summed tensor, layout [d*d][E] (row-major i*d+j).
 * Returns 0, or -1 for a degenerate element. */
int oc_shape_derivative(int dim, int64_t N, int64_t E, const double *coords, const int32_t *conn,
                        const double *A_e, const double *chi_e, double lam, double mu,
                        const double *u, int n_rhs, int64_t ld, double lambda_vol, double V,
                        double *rhs, double *S1_out, double *J, double *vol_out)
{
    int nv = dim + 1;
    memset(rhs, 0, (size_t)N * dim * sizeof(double));
    for (int k = 0; k < n_rhs; ++k) J[k] = 0.0;
    double vol_sum = 0.0;
    for (int64_t e = 0; e < E; ++e) {
        double g[OC_MAXV][3], vol;
        if (oc_simplex(dim, coords, conn, E, e, g, &vol)) return -1;
        double S[3][3] = {{0}};
        for (int k = 0; k < n_rhs; ++k) {
            double Du[3][3] = {{0}};
            for (int a = 0; a < nv; ++a) {
                int64_t node = conn[(int64_t)a * E + e];
                for (int i = 0; i < dim; ++i)
                    for (int j = 0; j < dim; ++j)
                        Du[i][j] += u[(node * dim + i) * ld + k] * g[a][j];
            }
            double eps[3][3], sig[3][3], tr = 0.0;
            for (int i = 0; i < dim; ++i) tr += Du[i][i];
            for (int i = 0; i < dim; ++i)
                for (int j = 0; j < dim; ++j) {
                    eps[i][j] = 0.5 * (Du[i][j] + Du[j][i]);
                    sig[i][j] = 2.0 * mu * eps[i][j] + (i == j ? lam * tr : 0.0);
                }
            double se = 0.0;
            for (int i = 0; i < dim; ++i)
                for (int j = 0; j < dim; ++j) se += sig[i][j] * eps[i][j];
            J[k] += A_e[e] * vol * se;
            for (int i = 0; i < dim; ++i)
                for (int j = 0; j < dim; ++j) {
                    double DuTs = 0.0; /* (Du^T sigma)_ij = sum_m Du_mi sigma_mj */
                    for (int m = 0; m < dim; ++m) DuTs += Du[m][i] * sig[m][j];
                    S[i][j] += A_e[e] * (2.0 * DuTs - (i == j ? se : 0.0));
                }
        }
        for (int i = 0; i < dim; ++i) S[i][i] += lambda_vol * chi_e[e] / V;
        vol_sum += chi_e[e] * vol;
        if (S1_out)
            for (int i = 0; i < dim; ++i)
                for (int j = 0; j < dim; ++j) S1_out[(int64_t)(i * dim + j) * E + e] = S[i][j];
        for (int a = 0; a < nv; ++a) {
            int64_t node = conn[(int64_t)a * E + e];
            for (int i = 0; i < dim; ++i) {
                double s = 0.0;
                for (int j = 0; j < dim; ++j) s += S[i][j] * g[a][j];
                rhs[node * dim + i] -= vol * s;
            }
        }
    }
    *vol_out = vol_sum;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* level-set update                                                         */

/* phi_i <- phi_i - dt theta_i . G_i, where G_i is the |T|-weighted mean of
 * the (element-constant) gradients grad phi_e over the elements containing
 * node i -- one explicit step of the transport d/dt phi + theta.grad phi = 0.
 * Returns 0, or -1 for a degenerate element. */
int oc_levelset_update(int dim, int64_t N, int64_t E, const double *coords, const int32_t *conn,
                       const double *theta, double dt, const double *phi_in, double *phi_out)
{
    int nv = dim + 1;
    double *G = calloc((size_t)N * dim, sizeof(double));
    double *W = calloc((size_t)N, sizeof(double));
    for (int64_t e = 0; e < E; ++e) {
        double g[OC_MAXV][3], vol;
        if (oc_simplex(dim, coords, conn, E, e, g, &vol)) {
            free(G);
            free(W);
            return -1;
        }
        double grad[3] = {0, 0, 0};
        for (int a = 0; a < nv; ++a) {
            double ph = phi_in[conn[(int64_t)a * E + e]];
            for (int i = 0; i < dim; ++i) grad[i] += ph * g[a][i];
        }
        for (int a = 0; a < nv; ++a) {
            int64_t node = conn[(int64_t)a * E + e];
            W[node] += vol;
            for (int i = 0; i < dim; ++i) G[node * dim + i] += vol * grad[i];
        }
    }
    for (int64_t n = 0; n < N; ++n) {
        double s = 0.0;
        for (int i = 0; i < dim; ++i) s += theta[n * dim + i] * G[n * dim + i];
        phi_out[n] = phi_in[n] - dt * (W[n] > 0.0 ? s / W[n] : 0.0);
    }
    free(G);
    free(W);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* transport step of the paper (Section "Transport equation")               */

/* The diffusion coefficient h^2.  The paper's "mesh diameter" expression,
 * 4|D|/(N_T sqrt 3) in 2D and (6 sqrt 2 |D|/N_T)^(2/3) in 3D, is the square
 * of the edge length of N_T equilateral triangles / regular tetrahedra
 * filling D, so it is used as h^2 itself.  |D| = sum of element measures. */
double oc_transport_h2(int dim, int64_t E, const double *coords, const int32_t *conn)
{
    double area = 0.0;
    for (int64_t e = 0; e < E; ++e) {
        double g[OC_MAXV][3], vol;
        if (oc_simplex(dim, coords, conn, E, e, g, &vol)) return -1.0;
        area += vol;
    }
    if (dim == 2) return 4.0 * area / ((double)E * sqrt(3.0));
    return pow(6.0 * sqrt(2.0) * area / (double)E, 2.0 / 3.0);
}

/* Sparsity of a scalar P1 operator (one unknown per node). */
static oc_csr *oc_csr_scalar(int dim, int64_t N, int64_t E, const int32_t *conn)
{
    /* the vector structure with one component: build it for "dimension 1"
     * connectivity rows of dim+1 vertices */
    int nv = dim + 1;
    int64_t *cnt = calloc((size_t)N + 1, sizeof(int64_t));
    for (int64_t e = 0; e < E; ++e)
        for (int a = 0; a < nv; ++a) cnt[conn[(int64_t)a * E + e] + 1] += nv;
    for (int64_t n = 0; n < N; ++n) cnt[n + 1] += cnt[n];
    int64_t *lst = malloc((size_t)(cnt[N] ? cnt[N] : 1) * sizeof(int64_t));
    int64_t *fill = malloc((size_t)(N ? N : 1) * sizeof(int64_t));
    memcpy(fill, cnt, (size_t)N * sizeof(int64_t));
    for (int64_t e = 0; e < E; ++e)
        for (int a = 0; a < nv; ++a) {
            int64_t na = conn[(int64_t)a * E + e];
            for (int b = 0; b < nv; ++b) lst[fill[na]++] = conn[(int64_t)b * E + e];
        }
    int64_t *uptr = calloc((size_t)N + 1, sizeof(int64_t));
    for (int64_t n = 0; n < N; ++n) {
        int64_t s0 = cnt[n], len = cnt[n + 1] - cnt[n];
        qsort(lst + s0, (size_t)len, sizeof(int64_t), cmp_i64);
        int64_t u = 0;
        for (int64_t k = 0; k < len; ++k)
            if (k == 0 || lst[s0 + k] != lst[s0 + k - 1]) lst[s0 + u++] = lst[s0 + k];
        uptr[n + 1] = u;
    }
    for (int64_t n = 0; n < N; ++n) uptr[n + 1] += uptr[n];
    int64_t *adj = malloc((size_t)(uptr[N] ? uptr[N] : 1) * sizeof(int64_t));
    for (int64_t n = 0; n < N; ++n)
        memcpy(adj + uptr[n], lst + cnt[n], (size_t)(uptr[n + 1] - uptr[n]) * sizeof(int64_t));
    free(lst);
    free(fill);
    free(cnt);
    oc_csr *A = calloc(1, sizeof(oc_csr));
    A->dim = 1;
    A->n = N;
    A->nadj_ptr = uptr;
    A->nadj = adj;
    A->rowptr = malloc((size_t)(N + 1) * sizeof(int64_t));
    A->rowptr[0] = 0;
    for (int64_t n = 0; n < N; ++n) A->rowptr[n + 1] = A->rowptr[n] + (uptr[n + 1] - uptr[n]);
    A->col = malloc((size_t)(A->rowptr[N] ? A->rowptr[N] : 1) * sizeof(int64_t));
    A->val = calloc((size_t)(A->rowptr[N] ? A->rowptr[N] : 1), sizeof(double));
    for (int64_t n = 0; n < N; ++n)
        for (int64_t k = uptr[n]; k < uptr[n + 1]; ++k) A->col[A->rowptr[n] + (k - uptr[n])] = adj[k];
    return A;
}

/* One time step of eq. weak_transport reads, with F(u, v) = (theta . grad u)
 * v / 2 + h^2 grad u . grad v / 2 and the test function psi_hat = psi + tau
 * theta . grad psi,
 *   int phi' psi_hat + dt F(phi', psi_hat) = int phi psi_hat - dt F(phi, psi_hat).
 * theta and tau enter per element, at the element mean of the nodal theta
 * (a one-point rule; tau = (1/2) (dt^-2 + |theta|^2 / h^2)^(-1/2), eq.
 * tau_lv), so the stabilised test function is linear on the element and its
 * second derivatives vanish.  With lambda_a the hat functions, g_a = grad
 * lambda_a and |T| the measure, the element entries (row a = test, column b
 * = trial) are
 *   mass          |T| (1 + delta_ab) / ((d+1)(d+2))
 *   stab. mass    tau (theta . g_a) |T| / (d+1)
 *   advection     (1/2) (theta . g_b) |T| / (d+1)
 *   stab. advect. (1/2) tau (theta . g_a) (theta . g_b) |T|
 *   diffusion     (1/2) h^2 (g_a . g_b) |T|                (smooth only)
 * and the step matrix is mass + stab. mass + sign dt (advection + stab.
 * advection + diffusion): sign +1 gives the left-hand side L, -1 the
 * right-hand side R.  Returns NULL for a degenerate element. */
oc_csr *oc_assemble_transport(int dim, int64_t N, int64_t E, const double *coords,
                              const int32_t *conn, const double *theta, double h2, int smooth,
                              double dt, double sign)
{
    oc_csr *A = oc_csr_scalar(dim, N, E, conn);
    int nv = dim + 1;
    for (int64_t e = 0; e < E; ++e) {
        double g[OC_MAXV][3], vol;
        if (oc_simplex(dim, coords, conn, E, e, g, &vol)) {
            oc_csr_free(A);
            return NULL;
        }
        double th[3] = {0, 0, 0};
        for (int a = 0; a < nv; ++a) {
            int64_t node = conn[(int64_t)a * E + e];
            for (int i = 0; i < dim; ++i) th[i] += theta[node * dim + i] / nv;
        }
        double t2 = 0.0;
        for (int i = 0; i < dim; ++i) t2 += th[i] * th[i];
        double tau = 0.5 / sqrt(1.0 / (dt * dt) + t2 / h2);
        double tg[OC_MAXV];
        for (int a = 0; a < nv; ++a) {
            tg[a] = 0.0;
            for (int i = 0; i < dim; ++i) tg[a] += th[i] * g[a][i];
        }
        for (int a = 0; a < nv; ++a) {
            int64_t na = conn[(int64_t)a * E + e];
            for (int b = 0; b < nv; ++b) {
                int64_t nb = conn[(int64_t)b * E + e];
                double gg = 0.0;
                for (int i = 0; i < dim; ++i) gg += g[a][i] * g[b][i];
                double mass = vol * (a == b ? 2.0 : 1.0) / ((dim + 1) * (dim + 2));
                double smass = tau * tg[a] * vol / nv;
                double adv = 0.5 * tg[b] * vol / nv;
                double sadv = 0.5 * tau * tg[a] * tg[b] * vol;
                double diff = smooth ? 0.5 * h2 * gg * vol : 0.0;
                oc_csr_add(A, na, 0, nb, 0, mass + smass + sign * dt * (adv + sadv + diff));
            }
        }
    }
    return A;
}

/* Jacobi-preconditioned BiCGStab (van der Vorst's method with the
 * preconditioner on the right: search directions M^-1 p and M^-1 s) for a
 * nonsymmetric A x = b, from the given x, until the recomputed residual
 * ||b - A x||_2 <= rtol ||b||_2.  Returns operator applications; status 0
 * converged, 1 iteration limit, -5 breakdown. */
int64_t oc_bicgstab(const oc_csr *A, const double *b, double *x, double rtol, int64_t max_iter,
                    double *relres, int *status)
{
    int64_t n = A->n;
    double *r = malloc((size_t)n * sizeof(double));
    double *rh = malloc((size_t)n * sizeof(double));
    double *p = calloc((size_t)n, sizeof(double));
    double *v = calloc((size_t)n, sizeof(double));
    double *y = malloc((size_t)n * sizeof(double));
    double *z = malloc((size_t)n * sizeof(double));
    double *s = malloc((size_t)n * sizeof(double));
    double *t = malloc((size_t)n * sizeof(double));
    double *dinv = malloc((size_t)n * sizeof(double));
    for (int64_t i = 0; i < n; ++i) {
        double d = 0.0;
        for (int64_t k = A->rowptr[i]; k < A->rowptr[i + 1]; ++k)
            if (A->col[k] == i) d = A->val[k];
        dinv[i] = d != 0.0 ? 1.0 / d : 0.0;
    }
    double bnorm = sqrt(oc_dot(n, b, b));
    int64_t it = 0;
    *status = 1;
    for (int restart = 0; restart < 50; ++restart) {
        oc_csr_matvec(A, x, t);
        if (restart > 0) ++it;
        for (int64_t i = 0; i < n; ++i) r[i] = b[i] - t[i];
        double rn = sqrt(oc_dot(n, r, r));
        *relres = bnorm > 0.0 ? rn / bnorm : 0.0;
        if (!(rn == rn)) {
            *status = -5;
            break;
        }
        if (rn <= rtol * bnorm) {
            *status = 0;
            break;
        }
        if (it >= max_iter) break;
        memcpy(rh, r, (size_t)n * sizeof(double));
        memset(p, 0, (size_t)n * sizeof(double));
        memset(v, 0, (size_t)n * sizeof(double));
        double rho = 1.0, alpha = 1.0, omega = 1.0;
        int bad = 0;
        while (it < max_iter) {
            double rho_new = oc_dot(n, rh, r);
            if (rho_new == 0.0 || !(rho_new == rho_new)) {
                bad = 1;
                break;
            }
            double beta = (rho_new / rho) * (alpha / omega);
            rho = rho_new;
            for (int64_t i = 0; i < n; ++i) {
                p[i] = r[i] + beta * (p[i] - omega * v[i]);
                y[i] = dinv[i] * p[i];
            }
            oc_csr_matvec(A, y, v);
            ++it;
            double rv = oc_dot(n, rh, v);
            if (rv == 0.0) {
                bad = 1;
                break;
            }
            alpha = rho / rv;
            for (int64_t i = 0; i < n; ++i) {
                x[i] += alpha * y[i];
                s[i] = r[i] - alpha * v[i];
                z[i] = dinv[i] * s[i];
            }
            if (sqrt(oc_dot(n, s, s)) <= rtol * bnorm) break;
            oc_csr_matvec(A, z, t);
            ++it;
            double tt = oc_dot(n, t, t);
            if (tt == 0.0) {
                bad = 1;
                break;
            }
            omega = oc_dot(n, t, s) / tt;
            for (int64_t i = 0; i < n; ++i) {
                x[i] += omega * z[i];
                r[i] = s[i] - omega * t[i];
            }
            if (sqrt(oc_dot(n, r, r)) <= rtol * bnorm) break;
            if (omega == 0.0) {
                bad = 1;
                break;
            }
        }
        if (bad && restart == 49) *status = -5;
    }
    free(r);
    free(rh);
    free(p);
    free(v);
    free(y);
    free(z);
    free(s);
    free(t);
    free(dinv);
    return it;
}

/* `steps` time steps of eq. weak_transport from phi_in: each solves
 * L phi' = R phi with L, R from oc_assemble_transport (the same for every
 * step), starting from phi.  iters: total operator applications.  Returns 0,
 * -1 for a degenerate element, -5 if a solve broke down or did not converge. */
int oc_transport(int dim, int64_t N, int64_t E, const double *coords, const int32_t *conn,
                 const double *theta, double h2, int smooth, double dt, int steps, double rtol,
                 int64_t max_iter, const double *phi_in, double *phi_out, int64_t *iters)
{
    oc_csr *L = oc_assemble_transport(dim, N, E, coords, conn, theta, h2, smooth, dt, 1.0);
    oc_csr *R = oc_assemble_transport(dim, N, E, coords, conn, theta, h2, smooth, dt, -1.0);
    if (!L || !R) {
        oc_csr_free(L);
        oc_csr_free(R);
        return -1;
    }
    double *b = malloc((size_t)(N ? N : 1) * sizeof(double));
    memcpy(phi_out, phi_in, (size_t)N * sizeof(double));
    int rc = 0;
    *iters = 0;
    for (int k = 0; k < steps && rc == 0; ++k) {
        oc_csr_matvec(R, phi_out, b);
        double rr;
        int st;
        *iters += oc_bicgstab(L, b, phi_out, rtol, max_iter, &rr, &st);
        if (st != 0) rc = -5;
    }
    free(b);
    oc_csr_free(L);
    oc_csr_free(R);
    return rc;
}

/* Element measures and barycentric gradients, exported for tests. */
int oc_element_geometry(int dim, int64_t E, const double *coords, const int32_t *conn,
                        double *vol_out, double *grad_out /* [E][d+1][d] */)
{
    for (int64_t e = 0; e < E; ++e) {
        double g[OC_MAXV][3], vol;
        if (oc_simplex(dim, coords, conn, E, e, g, &vol)) return -1;
        vol_out[e] = vol;
        for (int a = 0; a <= dim; ++a)
            for (int i = 0; i < dim; ++i) grad_out[(e * (dim + 1) + a) * dim + i] = g[a][i];
    }
    return 0;
}

void oc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int oc_get_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
