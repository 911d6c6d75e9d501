// Element operators used by the scatter kernels (atomic and tiled).
#pragma once

#include <hip/hip_runtime.h>

#include "fo_element.h"

namespace fo {

// An op maps one element to NV values per vertex.  `load(e)` fetches the
// element's own data (element index e in tile order) so that kernels can
// prefetch it; the call operator receives it with the vertex coordinates
// X[a] and NX staged values U[a] per vertex.
template <int D, typename T>
struct ElasOp {
    static constexpr int NX = D, NV = D;
    using Elem = uint8_t;
    const uint8_t *chi;
    T ersatz, lam, mu;
    __device__ Elem load(int64_t e) const { return chi[e]; }
    __device__ void operator()(Elem in, const T *const *X, const T *const *U, T out[D + 1][NV]) const
    {
        T A = in ? T(1) : ersatz;
        elas_element<D, T>(X, U, A, lam, mu, out);
    }
};

template <int D, typename T>
struct ElasDiagOp {
    static constexpr int NX = 0, NV = D;
    using Elem = uint8_t;
    const uint8_t *chi;
    T ersatz, lam, mu;
    __device__ Elem load(int64_t e) const { return chi[e]; }
    __device__ void operator()(Elem in, const T *const *X, const T *const *, T out[D + 1][NV]) const
    {
        T A = in ? T(1) : ersatz;
        elas_diag_element<D, T>(X, A, lam, mu, out);
    }
};

template <int D, typename T = double>
struct DescentOp {
    static constexpr int NX = D, NV = D;
    using Elem = uint8_t;
    const uint8_t *in0;
    T alpha, gamma_s;
    __device__ Elem load(int64_t e) const { return in0[e]; }
    __device__ void operator()(Elem in, const T *const *X, const T *const *U, T out[D + 1][NV]) const
    {
        T mw = alpha + (in ? gamma_s : T(0));
        descent_element<D, T>(X, U, mw, out);
    }
};

template <int D>
struct DescentDiagOp {
    static constexpr int NX = 0, NV = D;
    using Elem = uint8_t;
    const uint8_t *in0;
    double alpha, gamma_s;
    __device__ Elem load(int64_t e) const { return in0[e]; }
    __device__ void operator()(Elem in, const double *const *X, const double *const *,
                               double out[D + 1][NV]) const
    {
        double mw = alpha + (in ? gamma_s : 0.0);
        descent_diag_element<D, double>(X, mw, out);
    }
};

// Recovered-gradient accumulation: vertex values (|T| grad phi, |T|).
template <int D>
struct PhiGradOp {
    static constexpr int NX = 1, NV = D + 1;
    using Elem = uint8_t;
    __device__ Elem load(int64_t) const { return 0; }
    __device__ void operator()(Elem, const double *const *X, const double *const *U,
                               double out[D + 1][NV]) const
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
    struct Elem {
        double s[D * D];
    };
    const double *s1;  // [E][D*D], tile element order
    __device__ Elem load(int64_t e) const
    {
        Elem v;
#pragma unroll
        for (int k = 0; k < D * D; ++k) v.s[k] = s1[e * D * D + k];
        return v;
    }
    __device__ void operator()(const Elem &in, const double *const *X, const double *const *,
                               double out[D + 1][NV]) const
    {
        Geom<D, double> g = geom<D, double>(X);
        double S[D][D];
#pragma unroll
        for (int i = 0; i < D; ++i)
#pragma unroll
            for (int j = 0; j < D; ++j) S[i][j] = in.s[i * D + j];
        double vol = fabs(g.det) / (D == 2 ? 2.0 : 6.0);
        vertex_loads<D, double>(g, S, -vol / g.det, out);
    }
};

}  // namespace fo
