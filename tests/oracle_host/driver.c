/* Runs every entry point of the C oracle (oracle/fo_oracle.c) on small
 * meshes, for a build under AddressSanitizer and UndefinedBehaviorSanitizer:
 * element coefficients, elasticity and descent assembly, the constrained
 * state solve, the shape derivative, the level-set update, the transport
 * assembly and step, restriction, export.  Exit status 0 = clean run with
 * finite results. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct oc_csr oc_csr;
void oc_lame(double E, double nu, int dim, int plane_stress, double *lam, double *mu);
void oc_element_coef(int dim, int64_t E, const int32_t *conn, const double *phi, double ersatz, double *A,
                     double *chi);
oc_csr *oc_assemble_elasticity(int dim, int64_t N, int64_t E, const double *coords, const int32_t *conn,
                               const double *A_e, double lam, double mu);
oc_csr *oc_assemble_descent(int dim, int64_t N, int64_t E, const double *coords, const int32_t *conn,
                            int64_t nbf, const int32_t *bfacets, const double *bnormal, double alpha,
                            double gamma_n, double gamma_s, int n_boxes, const double *boxes);
void oc_csr_free(oc_csr *A);
int64_t oc_csr_rows(const oc_csr *A);
int64_t oc_csr_nnz(const oc_csr *A);
void oc_csr_export(const oc_csr *A, int64_t *rowptr, int64_t *col, double *val);
void oc_csr_matvec(const oc_csr *A, const double *x, double *y);
oc_csr *oc_csr_restrict(const oc_csr *A, const uint8_t *keep, int64_t *map_out);
int64_t oc_pcg(const oc_csr *A, const double *b, double *x, double rtol, int64_t max_iter, double *relres,
               int *status);
int64_t oc_solve_constrained(const oc_csr *K, const uint8_t *fixed, const double *b, double *u, double rtol,
                             int64_t max_iter, double *relres, int *status);
int oc_shape_derivative(int dim, int64_t N, int64_t E, const double *coords, const int32_t *conn,
                        const double *A_e, const double *chi_e, double lam, double mu, const double *u,
                        int n_rhs, int64_t ld, double lambda_vol, double V, double *rhs, double *S1_out,
                        double *J, double *vol_out);
int oc_levelset_update(int dim, int64_t N, int64_t E, const double *coords, const int32_t *conn,
                       const double *theta, double dt, const double *phi_in, double *phi_out);
int oc_transport(int dim, int64_t N, int64_t E, const double *coords, const int32_t *conn,
                 const double *theta, double h2, int smooth, double dt, int steps, double rtol,
                 int64_t max_iter, const double *phi_in, double *phi_out, int64_t *iters);
void oc_set_threads(int n);

static int fails = 0;
#define CHECK(c)                                                              \
    do {                                                                      \
        if (!(c)) {                                                           \
            fprintf(stderr, "oracle driver: check failed at %d: %s\n", __LINE__, #c); \
            ++fails;                                                          \
        }                                                                     \
    } while (0)

static int finite_all(const double *v, int64_t n)
{
    for (int64_t i = 0; i < n; ++i)
        if (!isfinite(v[i])) return 0;
    return 1;
}

/* nx x ny squares on [0,2]x[0,1], each split along its (i,j)-(i+1,j+1)
 * diagonal; or nx x ny x nz cubes split into the 6 Kuhn tetrahedra. */
static void mesh(int dim, int nx, int ny, int nz, double **X, int32_t **conn, int64_t *N, int64_t *E)
{
    const int mx = nx + 1, my = ny + 1, mz = dim == 3 ? nz + 1 : 1;
    *N = (int64_t)mx * my * mz;
    *X = calloc((size_t)*N * dim, sizeof(double));
    for (int k = 0; k < mz; ++k)
        for (int j = 0; j < my; ++j)
            for (int i = 0; i < mx; ++i) {
                const int64_t v = ((int64_t)k * my + j) * mx + i;
                (*X)[v * dim] = 2.0 * i / nx;
                (*X)[v * dim + 1] = 1.0 * j / ny;
                if (dim == 3) (*X)[v * dim + 2] = 1.0 * k / nz;
            }
    const int per = dim == 2 ? 2 : 6;
    *E = (int64_t)nx * ny * (dim == 3 ? nz : 1) * per;
    *conn = calloc((size_t)*E * (dim + 1), sizeof(int32_t));
    int64_t e = 0;
    const int perm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    for (int k = 0; k < (dim == 3 ? nz : 1); ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                if (dim == 2) {
                    const int32_t a = j * mx + i, b = a + 1, c = a + mx + 1, d = a + mx;
                    const int32_t t[2][3] = {{a, b, c}, {a, c, d}};
                    for (int q = 0; q < 2; ++q, ++e)
                        for (int s = 0; s < 3; ++s) (*conn)[(int64_t)s * *E + e] = t[q][s];
                } else {
                    for (int p = 0; p < 6; ++p, ++e) {
                        int c[3] = {i, j, k};
                        for (int s = 0; s < 4; ++s) {
                            if (s > 0) c[perm[p][s - 1]] += 1;
                            (*conn)[(int64_t)s * *E + e] = (int32_t)(((int64_t)c[2] * my + c[1]) * mx + c[0]);
                        }
                    }
                }
            }
}

static void run(int dim, int nx, int ny, int nz)
{
    double *X;
    int32_t *conn;
    int64_t N, E;
    mesh(dim, nx, ny, nz, &X, &conn, &N, &E);
    const int64_t n = N * dim;
    double lam, mu;
    oc_lame(1.0, 0.3, dim, 1, &lam, &mu);
    double *phi = malloc(N * sizeof(double)), *phi2 = malloc(N * sizeof(double));
    for (int64_t i = 0; i < N; ++i) phi[i] = X[i * dim] - 1.3 + 0.2 * X[i * dim + 1];
    double *A = malloc(E * sizeof(double)), *chi = malloc(E * sizeof(double));
    oc_element_coef(dim, E, conn, phi, 1e-3, A, chi);
    oc_csr *K = oc_assemble_elasticity(dim, N, E, X, conn, A, lam, mu);
    CHECK(K && oc_csr_rows(K) == n);
    uint8_t *fixed = calloc(n, 1);
    double *b = calloc(n, sizeof(double)), *u = calloc(n, sizeof(double));
    for (int64_t i = 0; i < N; ++i) {
        if (X[i * dim] == 0.0)
            for (int c = 0; c < dim; ++c) fixed[i * dim + c] = 1;
        if (X[i * dim] == 2.0) b[i * dim + 1] = -0.1;
    }
    double rr = 0;
    int st = 0;
    int64_t it = oc_solve_constrained(K, fixed, b, u, 1e-12, 10000, &rr, &st);
    CHECK(it > 0 && st == 0 && rr <= 1e-12 && finite_all(u, n));
    double *rhs = calloc(n, sizeof(double)), *S1 = calloc(E * dim * dim, sizeof(double));
    double J = 0, vol = 0;
    CHECK(oc_shape_derivative(dim, N, E, X, conn, A, chi, lam, mu, u, 1, 1, 0.3, 1.0, rhs, S1, &J, &vol) == 0);
    CHECK(J > 0 && vol > 0 && finite_all(rhs, n) && finite_all(S1, E * dim * dim));
    const int32_t bf2[2] = {0, 1};
    const double bn2[2] = {0.0, -1.0};
    int32_t bf3[3] = {0, 1, (int32_t)(nx + 2)};
    const double bn3[3] = {0.0, 0.0, -1.0};
    const double boxes2[4] = {1.5, 0.2, 2.0, 0.8}, boxes3[6] = {1.5, 0.2, 0.2, 2.0, 0.8, 0.8};
    oc_csr *B = dim == 2 ? oc_assemble_descent(dim, N, E, X, conn, 1, bf2, bn2, 0.01, 1e4, 1e4, 1, boxes2)
                         : oc_assemble_descent(dim, N, E, X, conn, 1, bf3, bn3, 0.01, 1e4, 1e4, 1, boxes3);
    CHECK(B != NULL);
    double *theta = calloc(n, sizeof(double));
    it = oc_pcg(B, rhs, theta, 1e-12, 10000, &rr, &st);
    CHECK(it > 0 && st == 0 && finite_all(theta, n));
    CHECK(oc_levelset_update(dim, N, E, X, conn, theta, 1e-3, phi, phi2) == 0 && finite_all(phi2, N));
    double *thn = calloc(N * dim, sizeof(double));
    for (int64_t i = 0; i < N * dim; ++i) thn[i] = (i % dim == 0) ? 0.3 : -0.1;
    int64_t tits = 0;
    CHECK(oc_transport(dim, N, E, X, conn, thn, 0.01, 1, 0.01, 3, 1e-12, 1000, phi, phi2, &tits) == 0);
    CHECK(tits > 0 && finite_all(phi2, N));
    uint8_t *keep = malloc(n);
    for (int64_t i = 0; i < n; ++i) keep[i] = !fixed[i];
    int64_t *map = malloc(n * sizeof(int64_t));
    oc_csr *Kf = oc_csr_restrict(K, keep, map);
    CHECK(Kf && oc_csr_rows(Kf) > 0);
    const int64_t nnz = oc_csr_nnz(K);
    int64_t *rp = malloc((n + 1) * sizeof(int64_t)), *col = malloc(nnz * sizeof(int64_t));
    double *val = malloc(nnz * sizeof(double)), *y = malloc(n * sizeof(double));
    oc_csr_export(K, rp, col, val);
    CHECK(rp[n] == nnz);
    oc_csr_matvec(K, u, y);
    CHECK(finite_all(y, n));
    oc_csr_free(K);
    oc_csr_free(B);
    oc_csr_free(Kf);
    free(X), free(conn), free(phi), free(phi2), free(A), free(chi), free(fixed), free(b), free(u);
    free(rhs), free(S1), free(theta), free(thn), free(keep), free(map), free(rp), free(col), free(val), free(y);
}

int main(void)
{
    oc_set_threads(2);
    run(2, 4, 2, 0);
    run(2, 7, 3, 0);
    run(3, 2, 1, 1);
    run(3, 3, 2, 2);
    printf("oracle driver: %d failed checks\n", fails);
    return fails ? 1 : 0;
}
