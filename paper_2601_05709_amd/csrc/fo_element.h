// Per-element P1 arithmetic on the device.
//
// Geometry is recomputed from vertex coordinates on every use (no stored
// Jacobians): with r_a = x_a - x_0 (a = 1..d) the cofactor vectors c_a satisfy
// c_a . r_b = det * delta_ab, so grad(lambda_a) = c_a / det for a >= 1,
// grad(lambda_0) = -sum_a c_a / det and |T| = |det| / d!.  Every operator below
// is written in terms of c_a and a single 1/|det| so that each element needs
// one reciprocal and no division per entry.
#pragma once

#include <hip/hip_runtime.h>

namespace fo {

template <int D, typename T>
struct Geom {
    T c[D][D];  // c[a-1][j]: cofactor vector of vertex a (a = 1..D)
    T det;      // signed det[r_1 .. r_D]
};

template <typename T>
__device__ __forceinline__ Geom<2, T> geom2(const T *x0, const T *x1, const T *x2)
{
    Geom<2, T> g;
    T r1x = x1[0] - x0[0], r1y = x1[1] - x0[1];
    T r2x = x2[0] - x0[0], r2y = x2[1] - x0[1];
    g.c[0][0] = r2y;
    g.c[0][1] = -r2x;
    g.c[1][0] = -r1y;
    g.c[1][1] = r1x;
    g.det = r1x * r2y - r1y * r2x;
    return g;
}

template <typename T>
__device__ __forceinline__ Geom<3, T> geom3(const T *x0, const T *x1, const T *x2, const T *x3)
{
    Geom<3, T> g;
    T r[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        r[0][i] = x1[i] - x0[i];
        r[1][i] = x2[i] - x0[i];
        r[2][i] = x3[i] - x0[i];
    }
    // c_1 = r_2 x r_3, c_2 = r_3 x r_1, c_3 = r_1 x r_2
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const T *u = r[(a + 1) % 3];
        const T *v = r[(a + 2) % 3];
        g.c[a][0] = u[1] * v[2] - u[2] * v[1];
        g.c[a][1] = u[2] * v[0] - u[0] * v[2];
        g.c[a][2] = u[0] * v[1] - u[1] * v[0];
    }
    g.det = r[0][0] * g.c[0][0] + r[0][1] * g.c[0][1] + r[0][2] * g.c[0][2];
    return g;
}

template <int D, typename T>
__device__ __forceinline__ Geom<D, T> geom(const T *const *X)
{
    if constexpr (D == 2)
        return geom2<T>(X[0], X[1], X[2]);
    else
        return geom3<T>(X[0], X[1], X[2], X[3]);
}

// 1 / (d! |det|): |T| / det^2.  Multiplying det-scaled quantities by it gives
// the element integral of products of two gradients.
template <int D, typename T>
__device__ __forceinline__ T inv_measure_det2(T det)
{
    T a = det < T(0) ? -det : det;
    return T(1) / (a * (D == 2 ? T(2) : T(6)));
}

// Dt[i][j] = sum_{a>=1} (u_a - u_0)_i c_a[j]  (= det * Du).
template <int D, typename T>
__device__ __forceinline__ void grad_scaled(const Geom<D, T> &g, const T *const *U, T Dt[D][D])
{
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = 0; j < D; ++j) Dt[i][j] = T(0);
#pragma unroll
    for (int a = 1; a <= D; ++a) {
#pragma unroll
        for (int i = 0; i < D; ++i) {
            T du = U[a][i] - U[0][i];
#pragma unroll
            for (int j = 0; j < D; ++j) Dt[i][j] += du * g.c[a - 1][j];
        }
    }
}

// sigma applied to a (scaled) gradient: lam tr(G) I + mu (G + G^T).
template <int D, typename T>
__device__ __forceinline__ void stress(const T G[D][D], T lam, T mu, T S[D][D])
{
    T tr = T(0);
#pragma unroll
    for (int i = 0; i < D; ++i) tr += G[i][i];
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = 0; j < D; ++j) S[i][j] = mu * (G[i][j] + G[j][i]) + (i == j ? lam * tr : T(0));
}

// out[a] = w * M c_a for a = 1..D and out[0] = -sum: the vertex loads of the
// element integral of M : D(N_a e_i) when M is constant on the element.
template <int D, typename T>
__device__ __forceinline__ void vertex_loads(const Geom<D, T> &g, const T M[D][D], T w,
                                             T out[D + 1][D])
{
#pragma unroll
    for (int i = 0; i < D; ++i) out[0][i] = T(0);
#pragma unroll
    for (int a = 1; a <= D; ++a)
#pragma unroll
        for (int i = 0; i < D; ++i) {
            T s = T(0);
#pragma unroll
            for (int j = 0; j < D; ++j) s += M[i][j] * g.c[a - 1][j];
            s *= w;
            out[a][i] = s;
            out[0][i] -= s;
        }
}

// Elasticity: y_a = A |T| sigma(Du) grad(lambda_a).
template <int D, typename T>
__device__ __forceinline__ void elas_element(const T *const *X, const T *const *U, T A, T lam,
                                             T mu, T out[D + 1][D])
{
    Geom<D, T> g = geom<D, T>(X);
    T Dt[D][D], S[D][D];
    grad_scaled<D, T>(g, U, Dt);
    stress<D, T>(Dt, lam, mu, S);
    vertex_loads<D, T>(g, S, A * inv_measure_det2<D, T>(g.det), out);
}

// Diagonal of the elasticity element matrix:
// K_e[(a,i),(a,i)] = A |T| ((lam + mu) g_ai^2 + mu |g_a|^2).
template <int D, typename T>
__device__ __forceinline__ void elas_diag_element(const T *const *X, T A, T lam, T mu,
                                                  T out[D + 1][D])
{
    Geom<D, T> g = geom<D, T>(X);
    T w = A * inv_measure_det2<D, T>(g.det);
    T c0[D];
#pragma unroll
    for (int j = 0; j < D; ++j) {
        c0[j] = T(0);
#pragma unroll
        for (int a = 0; a < D; ++a) c0[j] -= g.c[a][j];
    }
#pragma unroll
    for (int a = 0; a <= D; ++a) {
        const T *c = a == 0 ? c0 : g.c[a - 1];
        T n2 = T(0);
#pragma unroll
        for (int j = 0; j < D; ++j) n2 += c[j] * c[j];
#pragma unroll
        for (int i = 0; i < D; ++i) out[a][i] = w * ((lam + mu) * c[i] * c[i] + mu * n2);
    }
}

// Descent element: mw * M_e (x) I + K_lap,e (x) I with the P1 mass
// M_ab = |T| (1 + delta_ab) / ((d+1)(d+2)) and K_lap,ab = |T| g_a . g_b.
template <int D, typename T>
__device__ __forceinline__ void descent_element(const T *const *X, const T *const *U, T mw,
                                                T out[D + 1][D])
{
    Geom<D, T> g = geom<D, T>(X);
    T Dt[D][D];
    grad_scaled<D, T>(g, U, Dt);
    vertex_loads<D, T>(g, Dt, inv_measure_det2<D, T>(g.det), out);
    T adet = g.det < T(0) ? -g.det : g.det;
    T vol = adet / (D == 2 ? T(2) : T(6));
    T m = mw * vol / T((D + 1) * (D + 2));
    T sum[D];
#pragma unroll
    for (int i = 0; i < D; ++i) {
        sum[i] = T(0);
#pragma unroll
        for (int a = 0; a <= D; ++a) sum[i] += U[a][i];
    }
#pragma unroll
    for (int a = 0; a <= D; ++a)
#pragma unroll
        for (int i = 0; i < D; ++i) out[a][i] += m * (U[a][i] + sum[i]);
}

template <int D, typename T>
__device__ __forceinline__ void descent_diag_element(const T *const *X, T mw, T out[D + 1][D])
{
    Geom<D, T> g = geom<D, T>(X);
    T w = inv_measure_det2<D, T>(g.det);
    T adet = g.det < T(0) ? -g.det : g.det;
    T vol = adet / (D == 2 ? T(2) : T(6));
    T m = mw * vol * T(2) / T((D + 1) * (D + 2));
    T c0[D];
#pragma unroll
    for (int j = 0; j < D; ++j) {
        c0[j] = T(0);
#pragma unroll
        for (int a = 0; a < D; ++a) c0[j] -= g.c[a][j];
    }
#pragma unroll
    for (int a = 0; a <= D; ++a) {
        const T *c = a == 0 ? c0 : g.c[a - 1];
        T n2 = T(0);
#pragma unroll
        for (int j = 0; j < D; ++j) n2 += c[j] * c[j];
#pragma unroll
        for (int i = 0; i < D; ++i) out[a][i] = w * n2 + m;
    }
}

// Compliance shape tensor of one load case, scaled: with Dt = det Du and
// St = sigma(Dt) = det sigma(Du), returns E = 2 Dt^T St - (St : Dt) I
// (= det^2 (2 Du^T sigma - sigma:eps I)) and se = St : Dt.
template <int D, typename T>
__device__ __forceinline__ void shape_tensor_scaled(const T Dt[D][D], T lam, T mu, T Sacc[D][D],
                                                    T scale, T *se_out)
{
    T St[D][D];
    stress<D, T>(Dt, lam, mu, St);
    T se = T(0);
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = 0; j < D; ++j) se += St[i][j] * Dt[i][j];
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = 0; j < D; ++j) {
            T dts = T(0);
#pragma unroll
            for (int m = 0; m < D; ++m) dts += Dt[m][i] * St[m][j];
            Sacc[i][j] += scale * (T(2) * dts - (i == j ? se : T(0)));
        }
    *se_out = se;
}

}  // namespace fo
