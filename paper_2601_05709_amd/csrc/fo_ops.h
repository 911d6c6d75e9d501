// Element operators used by the scatter kernels (atomic and tiled).
#pragma once

#include <hip/hip_runtime.h>

#include "fo_element.h"

namespace fo {

// Ops read vertex coordinates X[a] and staged vertex values U[a] and return
// NV values per vertex.  Element index e is in tile order.
template <int D, typename T>
struct ElasOp {
    static constexpr int NX = D, NV = D;
    const uint8_t *chi;
    T ersatz, lam, mu;
    __device__ void operator()(int64_t e, const int32_t *, const T *const *X, const T *const *U,
                               T out[D + 1][NV]) const
    {
        T A = chi[e] ? T(1) : ersatz;
        elas_element<D, T>(X, U, A, lam, mu, out);
    }
};

template <int D, typename T>
struct ElasDiagOp {
    static constexpr int NX = 0, NV = D;
    const uint8_t *chi;
    T ersatz, lam, mu;
    __device__ void operator()(int64_t e, const int32_t *, const T *const *X, const T *const *,
                               T out[D + 1][NV]) const
    {
        T A = chi[e] ? T(1) : ersatz;
        elas_diag_element<D, T>(X, A, lam, mu, out);
    }
};

template <int D>
struct DescentOp {
    static constexpr int NX = D, NV = D;
    const uint8_t *in0;
    double alpha, gamma_s;
    __device__ void operator()(int64_t e, const int32_t *, const double *const *X,
                               const double *const *U, double out[D + 1][NV]) const
    {
        double mw = alpha + (in0[e] ? gamma_s : 0.0);
        descent_element<D, double>(X, U, mw, out);
    }
};

template <int D>
struct DescentDiagOp {
    static constexpr int NX = 0, NV = D;
    const uint8_t *in0;
    double alpha, gamma_s;
    __device__ void operator()(int64_t e, const int32_t *, const double *const *X,
                               const double *const *, double out[D + 1][NV]) const
    {
        double mw = alpha + (in0[e] ? gamma_s : 0.0);
        descent_diag_element<D, double>(X, mw, out);
    }
};

// Recovered-gradient accumulation: vertex values (|T| grad phi, |T|).
template <int D>
struct PhiGradOp {
    static constexpr int NX = 1, NV = D + 1;
    __device__ void operator()(int64_t, const int32_t *, const double *const *X,
                               const double *const *U, double out[D + 1][NV]) const
    {
        Geom<D, double> g = geom<D, double>(X);
        double adet = fabs(g.det);
        double vol = adet / (D == 2 ? 2.0 : 6.0);
        double grad[D];
#pragma unroll
        for (int j = 0; j < D; ++j) grad[j] = 0.0;
#pragma unroll
        for (int a = 1; a <= D; ++a) {
            double dphi = U[a][0] - U[0][0];
#pragma unroll
            for (int j = 0; j < D; ++j) grad[j] += dphi * g.c[a - 1][j];
        }
        // |T| grad phi = |T| Dt / det
        double s = vol / g.det;
#pragma unroll
        for (int a = 0; a <= D; ++a) {
#pragma unroll
            for (int j = 0; j < D; ++j) out[a][j] = s * grad[j];
            out[a][D] = vol;
        }
    }
};

// Descent right-hand side from stored element tensors:
// rhs_a -= |T| S1_e grad(lambda_a) = (|T| / det) S1_e c_a  (with the sign).
template <int D>
struct SdRhsOp {
    static constexpr int NX = 0, NV = D;
    const double *s1;  // [E][D*D], tile element order
    __device__ void operator()(int64_t e, const int32_t *, const double *const *X,
                               const double *const *, double out[D + 1][NV]) const
    {
        Geom<D, double> g = geom<D, double>(X);
        double S[D][D];
#pragma unroll
        for (int i = 0; i < D; ++i)
#pragma unroll
            for (int j = 0; j < D; ++j) S[i][j] = s1[e * D * D + i * D + j];
        double vol = fabs(g.det) / (D == 2 ? 2.0 : 6.0);
        vertex_loads<D, double>(g, S, -vol / g.det, out);
    }
};

}  // namespace fo
