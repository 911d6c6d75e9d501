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

// Transport step of the level set (Section "Transport equation", eqs.
// weak_transport, tau_lv): the Crank-Nicolson Petrov-Galerkin step matrix
// applied to a nodal scalar.  Per element the velocity theta and tau are the
// element-mean values (coef); with g_a the hat-function gradients, |T| the
// measure, grad x = sum_b x_b g_b and s = sum_b x_b, row a is
//   |T| [ (x_a + s) / ((d+1)(d+2))                        mass
//       + tau (theta.g_a) s / (d+1)                        stabilised mass
//       + sdt ( (theta.grad x) / (2 (d+1))                  advection
//             + tau (theta.g_a) (theta.grad x) / 2          stabilised advection
//             + h2 (g_a . grad x) / 2 ) ]                   diffusion
// sdt = +dt gives the left-hand side L, -dt the right-hand side R.
// Element-mean velocity and tau = (1/2) (dt^-2 + |theta|^2 / h^2)^(-1/2) of
// the Petrov-Galerkin test functions (eq. tau_lv), from the tile-staged nodal
// velocity A[a][0..D).
template <int D>
__device__ __forceinline__ double transport_tau(const double *const *A, double rdt2, double h2, double th[D])
{
#pragma unroll
    for (int i = 0; i < D; ++i) th[i] = 0.0;
#pragma unroll
    for (int a = 0; a <= D; ++a)
#pragma unroll
        for (int i = 0; i < D; ++i) th[i] += A[a][i];
    double t2 = 0.0;
#pragma unroll
    for (int i = 0; i < D; ++i) {
        th[i] /= (double)(D + 1);
        t2 += th[i] * th[i];
    }
    return 0.5 / sqrt(rdt2 + t2 / h2);
}

// Transport step matrices (eq. weak_transport): y = L x (which 0) or R x
// (which 1).  The nodal velocity is staged per tile (aux, NA values per
// node) and the step parameters come from device memory (par: [0] dt, [1]
// -dt, [2] h2 of the diffusion, 0 without it, [3] h2 of tau, [4] 1 / dt^2),
// so one captured graph of the solver serves every call.
template <int D>
struct TransportOp {
    static constexpr int NX = 1, NV = 1, NA = D;
    struct Elem {
        double sdt, h2e, rdt2, h2;
    };
    const double *aux;  // [N][D] nodal velocity theta
    const double *par;
    int which;
    __device__ Elem load(int64_t) const { return Elem{par[which], par[2], par[4], par[3]}; }
    __device__ void operator()(const Elem &in, const double *const *X, const double *const *U,
                               const double *const *A, double out[D + 1][1]) const
    {
        const double sdt = in.sdt, h2 = in.h2e;
        double th[D];
        const double tau = transport_tau<D>(A, in.rdt2, in.h2, th);
        const Geom<D, double> g = geom<D, double>(X);
        const double inv = 1.0 / g.det;
        const double vol = fabs(g.det) / (D == 2 ? 2.0 : 6.0);
        double ga[D + 1][D];
#pragma unroll
        for (int j = 0; j < D; ++j) {
            ga[0][j] = 0.0;
#pragma unroll
            for (int a = 1; a <= D; ++a) {
                ga[a][j] = g.c[a - 1][j] * inv;
                ga[0][j] -= ga[a][j];
            }
        }
        double sx = 0.0, gx[D];
#pragma unroll
        for (int j = 0; j < D; ++j) gx[j] = 0.0;
#pragma unroll
        for (int a = 0; a <= D; ++a) {
            sx += U[a][0];
#pragma unroll
            for (int j = 0; j < D; ++j) gx[j] += U[a][0] * ga[a][j];
        }
        double tgx = 0.0;
#pragma unroll
        for (int j = 0; j < D; ++j) tgx += th[j] * gx[j];
#pragma unroll
        for (int a = 0; a <= D; ++a) {
            double tg = 0.0, ggx = 0.0;
#pragma unroll
            for (int j = 0; j < D; ++j) {
                tg += th[j] * ga[a][j];
                ggx += ga[a][j] * gx[j];
            }
            out[a][0] = vol * ((U[a][0] + sx) / ((D + 1) * (D + 2)) + tau * tg * sx / (D + 1) +
                               sdt * (0.5 * tgx / (D + 1) + 0.5 * tau * tg * tgx + 0.5 * h2 * ggx));
        }
    }
};

// Diagonal of the transport left-hand side L.
template <int D>
struct TransportDiagOp {
    static constexpr int NX = 0, NV = 1, NA = D;
    using Elem = typename TransportOp<D>::Elem;
    const double *aux;
    const double *par;
    __device__ Elem load(int64_t e) const { return TransportOp<D>{aux, par, 0}.load(e); }
    __device__ void operator()(const Elem &in, const double *const *X, const double *const *,
                               const double *const *A, double out[D + 1][1]) const
    {
        const double dt = in.sdt, h2 = in.h2e;
        double th[D];
        const double tau = transport_tau<D>(A, in.rdt2, in.h2, th);
        const Geom<D, double> g = geom<D, double>(X);
        const double inv = 1.0 / g.det;
        const double vol = fabs(g.det) / (D == 2 ? 2.0 : 6.0);
        double ga[D + 1][D];
#pragma unroll
        for (int j = 0; j < D; ++j) {
            ga[0][j] = 0.0;
#pragma unroll
            for (int a = 1; a <= D; ++a) {
                ga[a][j] = g.c[a - 1][j] * inv;
                ga[0][j] -= ga[a][j];
            }
        }
#pragma unroll
        for (int a = 0; a <= D; ++a) {
            double tg = 0.0, gg = 0.0;
#pragma unroll
            for (int j = 0; j < D; ++j) {
                tg += th[j] * ga[a][j];
                gg += ga[a][j] * ga[a][j];
            }
            out[a][0] = vol * (2.0 / ((D + 1) * (D + 2)) + tau * tg / (D + 1) +
                               dt * (0.5 * tg / (D + 1) + 0.5 * tau * tg * tg + 0.5 * h2 * gg));
        }
    }
};

// Reinitialisation step of the level set (eqs. HJ, grad_H, weak_HJ), from
// the tile-staged nodal values A[a] = (u = varphi(t), v = varphi(t - dt),
// S(phi)): S_e = element mean of S, g = grad u, grad H = S_e g / |g|,
// tau_e = 1/2 (dt^-2 + S_e^2 / h^2)^(-1/2).  p / |p| has no limit at 0: on
// an element whose vertex values agree to 1e-12 relative (g is rounding
// noise) or with g = 0, grad H = 0.  par: device [4] dt, h^2, 1/dt^2, 1 for
// the explicit Euler first step (else Adams-Bashforth).
template <int D>
struct ReinitCoef {
    double ga[D + 1][D];  // gradients of the barycentric functions
    double vol, S, tau, nu;
    double gu[D], gH[D];
};

template <int D>
__device__ __forceinline__ ReinitCoef<D> reinit_coef(const double *const *X, const double *const *A, double rdt2,
                                                     double h2)
{
    ReinitCoef<D> k;
    const Geom<D, double> g = geom<D, double>(X);
    const double inv = 1.0 / g.det;
    k.vol = fabs(g.det) / (D == 2 ? 2.0 : 6.0);
#pragma unroll
    for (int j = 0; j < D; ++j) {
        k.ga[0][j] = 0.0;
#pragma unroll
        for (int a = 1; a <= D; ++a) {
            k.ga[a][j] = g.c[a - 1][j] * inv;
            k.ga[0][j] -= k.ga[a][j];
        }
    }
    double S = 0.0, n2 = 0.0, umax = A[0][0], umin = A[0][0], uabs = fabs(A[0][0]);
#pragma unroll
    for (int a = 0; a <= D; ++a) {
        S += A[a][2];
        umax = fmax(umax, A[a][0]);
        umin = fmin(umin, A[a][0]);
        uabs = fmax(uabs, fabs(A[a][0]));
    }
    k.S = S / (double)(D + 1);
    const bool flat = umax - umin <= 1e-12 * uabs;
#pragma unroll
    for (int j = 0; j < D; ++j) {
        double s = 0.0;
#pragma unroll
        for (int a = 0; a <= D; ++a) s += A[a][0] * k.ga[a][j];
        k.gu[j] = s;
        n2 += s * s;
    }
    k.nu = sqrt(n2);
#pragma unroll
    for (int j = 0; j < D; ++j) k.gH[j] = (!flat && k.nu > 0.0) ? k.S * k.gu[j] / k.nu : 0.0;
    k.tau = 0.5 / sqrt(rdt2 + k.S * k.S / h2);
    return k;
}

// y = Lhat x with Lhat_ab = int lambda_b psi_hat_a = M_ab + tau (grad H .
// grad lambda_a) |T| / (d+1).
template <int D>
struct ReinitOp {
    static constexpr int NX = 1, NV = 1, NA = 3;
    struct Elem {
        double rdt2, h2;
    };
    const double *aux;  // [N][3]: u, v, S
    const double *par;
    __device__ Elem load(int64_t) const { return Elem{par[2], par[1]}; }
    __device__ void operator()(const Elem &in, const double *const *X, const double *const *U,
                               const double *const *A, double out[D + 1][1]) const
    {
        const ReinitCoef<D> k = reinit_coef<D>(X, A, in.rdt2, in.h2);
        double sx = 0.0;
#pragma unroll
        for (int a = 0; a <= D; ++a) sx += U[a][0];
#pragma unroll
        for (int a = 0; a <= D; ++a) {
            double tg = 0.0;
#pragma unroll
            for (int j = 0; j < D; ++j) tg += k.gH[j] * k.ga[a][j];
            out[a][0] = k.vol * ((U[a][0] + sx) / ((D + 1) * (D + 2)) + k.tau * tg * sx / (D + 1));
        }
    }
};

// Diagonal of Lhat.
template <int D>
struct ReinitDiagOp {
    static constexpr int NX = 0, NV = 1, NA = 3;
    using Elem = typename ReinitOp<D>::Elem;
    const double *aux;
    const double *par;
    __device__ Elem load(int64_t e) const { return ReinitOp<D>{aux, par}.load(e); }
    __device__ void operator()(const Elem &in, const double *const *X, const double *const *,
                               const double *const *A, double out[D + 1][1]) const
    {
        const ReinitCoef<D> k = reinit_coef<D>(X, A, in.rdt2, in.h2);
#pragma unroll
        for (int a = 0; a <= D; ++a) {
            double tg = 0.0;
#pragma unroll
            for (int j = 0; j < D; ++j) tg += k.gH[j] * k.ga[a][j];
            out[a][0] = k.vol * (2.0 / ((D + 1) * (D + 2)) + k.tau * tg / (D + 1));
        }
    }
};

// Right-hand side of one step: int (u + dt S) psi_hat_a + dt int G(u, v,
// psi_hat_a), G(u, v, w) = (H(grad v) - 3 H(grad u)) / 2 w + h^2 (grad v -
// 3 grad u) / 2 . grad w; the Euler step takes -H(grad u) w - h^2 grad u .
// grad w.  grad psi_hat_a = grad lambda_a (the tau term is constant per
// element).
template <int D>
struct ReinitRhsOp {
    static constexpr int NX = 0, NV = 1, NA = 3;
    struct Elem {
        double dt, h2, rdt2, euler;
    };
    const double *aux;
    const double *par;
    __device__ Elem load(int64_t) const { return Elem{par[0], par[1], par[2], par[3]}; }
    __device__ void operator()(const Elem &in, const double *const *X, const double *const *,
                               const double *const *A, double out[D + 1][1]) const
    {
        const ReinitCoef<D> k = reinit_coef<D>(X, A, in.rdt2, in.h2);
        const bool euler = in.euler != 0.0;
        double su = 0.0, gv[D], nv2 = 0.0;
#pragma unroll
        for (int a = 0; a <= D; ++a) su += A[a][0];
#pragma unroll
        for (int j = 0; j < D; ++j) {
            double s = 0.0;
#pragma unroll
            for (int a = 0; a <= D; ++a) s += A[a][1] * k.ga[a][j];
            gv[j] = s;
            nv2 += s * s;
        }
        const double c = euler ? -k.S * k.nu : 0.5 * k.S * (sqrt(nv2) - 3.0 * k.nu);
        double dv[D];
#pragma unroll
        for (int j = 0; j < D; ++j) dv[j] = euler ? -k.gu[j] : 0.5 * (gv[j] - 3.0 * k.gu[j]);
#pragma unroll
        for (int a = 0; a <= D; ++a) {
            double tg = 0.0, dg = 0.0;
#pragma unroll
            for (int j = 0; j < D; ++j) {
                tg += k.gH[j] * k.ga[a][j];
                dg += dv[j] * k.ga[a][j];
            }
            const double ones_hat = k.vol / (D + 1) + k.tau * tg * k.vol;
            out[a][0] = k.vol * (A[a][0] + su) / ((D + 1) * (D + 2)) + k.tau * tg * k.vol * su / (D + 1) +
                        in.dt * (k.S + c) * ones_hat + in.dt * in.h2 * k.vol * dg;
        }
    }
};

// Gradients of the barycentric functions and the measure of a P1 element.
template <int D>
__device__ __forceinline__ double p1_grads(const double *const *X, double ga[D + 1][D])
{
    const Geom<D, double> g = geom<D, double>(X);
    const double inv = 1.0 / g.det;
#pragma unroll
    for (int j = 0; j < D; ++j) {
        ga[0][j] = 0.0;
#pragma unroll
        for (int a = 1; a <= D; ++a) {
            ga[a][j] = g.c[a - 1][j] * inv;
            ga[0][j] -= ga[a][j];
        }
    }
    return fabs(g.det) / (D == 2 ? 2.0 : 6.0);
}

// Heat-conduction model (eqs. heat_prob, heat_weak, heat_AOmega): scalar
// P1 operator y_a = sum_b A_e |T| grad lambda_a . grad lambda_b x_b with A_e
// = 1 in Omega, the ersatz value outside.
template <int D>
struct HeatOp {
    static constexpr int NX = 1, NV = 1;
    using Elem = uint8_t;
    const uint8_t *chi;
    double ersatz;
    __device__ Elem load(int64_t e) const { return chi[e]; }
    __device__ void operator()(Elem in, const double *const *X, const double *const *U,
                               double out[D + 1][1]) const
    {
        double ga[D + 1][D];
        const double w = (in ? 1.0 : ersatz) * p1_grads<D>(X, ga);
        double gx[D];
#pragma unroll
        for (int j = 0; j < D; ++j) {
            gx[j] = 0.0;
#pragma unroll
            for (int b = 0; b <= D; ++b) gx[j] += U[b][0] * ga[b][j];
        }
#pragma unroll
        for (int a = 0; a <= D; ++a) {
            double s = 0.0;
#pragma unroll
            for (int j = 0; j < D; ++j) s += ga[a][j] * gx[j];
            out[a][0] = w * s;
        }
    }
};

template <int D>
struct HeatDiagOp {
    static constexpr int NX = 0, NV = 1;
    using Elem = uint8_t;
    const uint8_t *chi;
    double ersatz;
    __device__ Elem load(int64_t e) const { return chi[e]; }
    __device__ void operator()(Elem in, const double *const *X, const double *const *,
                               double out[D + 1][1]) const
    {
        double ga[D + 1][D];
        const double w = (in ? 1.0 : ersatz) * p1_grads<D>(X, ga);
#pragma unroll
        for (int a = 0; a <= D; ++a) {
            double s = 0.0;
#pragma unroll
            for (int j = 0; j < D; ++j) s += ga[a][j] * ga[a][j];
            out[a][0] = w * s;
        }
    }
};

// Scalar P1 mass: y_a = int lambda_a x = |T| (x_a + sum_b x_b) / ((d+1)(d+2)).
template <int D>
struct MassOp {
    static constexpr int NX = 1, NV = 1;
    using Elem = uint8_t;
    __device__ Elem load(int64_t) const { return 0; }
    __device__ void operator()(Elem, const double *const *X, const double *const *U, double out[D + 1][1]) const
    {
        double ga[D + 1][D];
        const double vol = p1_grads<D>(X, ga);
        double sx = 0.0;
#pragma unroll
        for (int a = 0; a <= D; ++a) sx += U[a][0];
#pragma unroll
        for (int a = 0; a <= D; ++a) out[a][0] = vol * (U[a][0] + sx) / ((D + 1) * (D + 2));
    }
};

// Descent right-hand side of the heat model from u (input) and the P1 heat
// source f (tile-staged, aux): S0 = 2 u grad f, S1 = (2 u f - A |grad u|^2) I
// + 2 A grad u (x) grad u + lambda chi I / V; out[a][i] = -(int S0_i lambda_a
// + int (S1 grad lambda_a)_i), exact for P1 u and f.
template <int D>
struct HeatSdOp {
    static constexpr int NX = 1, NV = D, NA = 1;
    using Elem = uint8_t;
    const uint8_t *chi;
    const double *aux;  // [N] f
    double ersatz, lambda_vol, V;
    __device__ Elem load(int64_t e) const { return chi[e]; }
    __device__ void operator()(Elem in, const double *const *X, const double *const *U, const double *const *F,
                               double out[D + 1][D]) const
    {
        double ga[D + 1][D];
        const double vol = p1_grads<D>(X, ga);
        const double A = in ? 1.0 : ersatz;
        double su = 0.0, gu[D], gf[D], Mu[D + 1];
#pragma unroll
        for (int a = 0; a <= D; ++a) su += U[a][0];
        double uf = 0.0;
#pragma unroll
        for (int a = 0; a <= D; ++a) {
            Mu[a] = vol * (U[a][0] + su) / ((D + 1) * (D + 2));
            uf += Mu[a] * F[a][0];
        }
        double g2 = 0.0;
#pragma unroll
        for (int j = 0; j < D; ++j) {
            gu[j] = gf[j] = 0.0;
#pragma unroll
            for (int a = 0; a <= D; ++a) {
                gu[j] += U[a][0] * ga[a][j];
                gf[j] += F[a][0] * ga[a][j];
            }
            g2 += gu[j] * gu[j];
        }
        const double iso = 2.0 * uf - A * vol * g2 + (in ? lambda_vol * vol / V : 0.0);
#pragma unroll
        for (int a = 0; a <= D; ++a) {
            double ug = 0.0;
#pragma unroll
            for (int j = 0; j < D; ++j) ug += gu[j] * ga[a][j];
#pragma unroll
            for (int i = 0; i < D; ++i)
                out[a][i] = -(2.0 * gf[i] * Mu[a] + iso * ga[a][i] + 2.0 * A * vol * gu[i] * ug);
        }
    }
};

// Vector P1 mass: y_(a,i) = int lambda_a x_i = |T| (x_(a,i) + sum_b x_(b,i)) /
// ((d+1)(d+2)), component by component.
template <int D>
struct VecMassOp {
    static constexpr int NX = D, NV = D;
    using Elem = uint8_t;
    __device__ Elem load(int64_t) const { return 0; }
    __device__ void operator()(Elem, const double *const *X, const double *const *U, double out[D + 1][D]) const
    {
        const Geom<D, double> g = geom<D, double>(X);
        const double m = fabs(g.det) / (D == 2 ? 2.0 : 6.0) / ((D + 1) * (D + 2));
#pragma unroll
        for (int i = 0; i < D; ++i) {
            double sx = 0.0;
#pragma unroll
            for (int a = 0; a <= D; ++a) sx += U[a][i];
#pragma unroll
            for (int a = 0; a <= D; ++a) out[a][i] = m * (U[a][i] + sx);
        }
    }
};

// Linear-elastic stress of a displacement Jacobian Dm ((Dm)_ij = d_j u_i):
// eps = sym(Dm), sigma = lam tr(eps) I + 2 mu eps.
template <int D>
__device__ __forceinline__ void lin_stress(const double Dm[D][D], double lam, double mu, double S[D][D],
                                           double Ep[D][D])
{
    double tr = 0.0;
#pragma unroll
    for (int i = 0; i < D; ++i) tr += Dm[i][i];
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = 0; j < D; ++j) {
            Ep[i][j] = 0.5 * (Dm[i][j] + Dm[j][i]);
            S[i][j] = 2.0 * mu * Ep[i][j] + (i == j ? lam * tr : 0.0);
        }
}

// Descent right-hand side of the inverse elasticity problem (Section "Inverse
// problem", eq. SDelast_inv) for one force-displacement pair, with A = kappa
// in Omega and 1 outside (eq. AOmega), u the input and v, p, q, g tile-staged
// (aux [N][4d]); w = u - v - g:
//   S0 = -alpha Dg^T w   (the sigma(q) : grad eps(g) term vanishes for P1 g),
//   S1 = [alpha/2 |w|^2 + A (sigma(u):eps(p) + sigma(v+g):eps(q))] I
//        - A (Du^T sigma(p) + Dp^T sigma(u) + Dv^T sigma(q) + Dq^T sigma(v+g)),
// out[a][i] = -(int S0_i lambda_a + int (S1 grad lambda_a)_i), exact for P1
// fields (the |w|^2 and S0 integrals with the P1 mass).
template <int D>
struct InvSdOp {
    static constexpr int NX = D, NV = D, NA = 4 * D;
    using Elem = uint8_t;
    const uint8_t *chi;
    const double *aux;  // [N][4D]: v, p, q, g
    double kappa, alpha, lam, mu;
    __device__ Elem load(int64_t e) const { return chi[e]; }
    __device__ void operator()(Elem in, const double *const *X, const double *const *U, const double *const *F,
                               double out[D + 1][D]) const
    {
        double ga[D + 1][D];
        const double vol = p1_grads<D>(X, ga);
        const double Av = (in ? kappa : 1.0) * vol;
        double Du[D][D], Dv[D][D], Dp[D][D], Dq[D][D], Dg[D][D], Dy[D][D];
#pragma unroll
        for (int i = 0; i < D; ++i)
#pragma unroll
            for (int j = 0; j < D; ++j) {
                double su = 0.0, sv = 0.0, sp = 0.0, sq = 0.0, sg = 0.0;
#pragma unroll
                for (int a = 0; a <= D; ++a) {
                    su += U[a][i] * ga[a][j];
                    sv += F[a][i] * ga[a][j];
                    sp += F[a][D + i] * ga[a][j];
                    sq += F[a][2 * D + i] * ga[a][j];
                    sg += F[a][3 * D + i] * ga[a][j];
                }
                Du[i][j] = su;
                Dv[i][j] = sv;
                Dp[i][j] = sp;
                Dq[i][j] = sq;
                Dg[i][j] = sg;
                Dy[i][j] = sv + sg;
            }
        double Su[D][D], Eu[D][D], Sp[D][D], Ep[D][D], Sq[D][D], Eq[D][D], Sy[D][D], Ey[D][D];
        lin_stress<D>(Du, lam, mu, Su, Eu);
        lin_stress<D>(Dp, lam, mu, Sp, Ep);
        lin_stress<D>(Dq, lam, mu, Sq, Eq);
        lin_stress<D>(Dy, lam, mu, Sy, Ey);
        // int w lambda_a and int |w|^2 with the P1 mass
        const double m = vol / ((D + 1) * (D + 2));
        double w[D + 1][D], Mw[D + 1][D], ww = 0.0;
#pragma unroll
        for (int a = 0; a <= D; ++a)
#pragma unroll
            for (int i = 0; i < D; ++i) w[a][i] = U[a][i] - F[a][i] - F[a][3 * D + i];
#pragma unroll
        for (int i = 0; i < D; ++i) {
            double sw = 0.0;
#pragma unroll
            for (int a = 0; a <= D; ++a) sw += w[a][i];
#pragma unroll
            for (int a = 0; a <= D; ++a) {
                Mw[a][i] = m * (w[a][i] + sw);
                ww += Mw[a][i] * w[a][i];
            }
        }
        double se = 0.0;
#pragma unroll
        for (int i = 0; i < D; ++i)
#pragma unroll
            for (int j = 0; j < D; ++j) se += Su[i][j] * Ep[i][j] + Sy[i][j] * Eq[i][j];
        const double iso = 0.5 * alpha * ww + Av * se;
        double T[D][D];
#pragma unroll
        for (int i = 0; i < D; ++i)
#pragma unroll
            for (int j = 0; j < D; ++j) {
                double t = 0.0;
#pragma unroll
                for (int k = 0; k < D; ++k)
                    t += Du[k][i] * Sp[k][j] + Dp[k][i] * Su[k][j] + Dv[k][i] * Sq[k][j] + Dq[k][i] * Sy[k][j];
                T[i][j] = Av * t;
            }
#pragma unroll
        for (int a = 0; a <= D; ++a)
#pragma unroll
            for (int i = 0; i < D; ++i) {
                double s0 = 0.0, tg = 0.0;
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    s0 += Dg[k][i] * Mw[a][k];
                    tg += T[i][k] * ga[a][k];
                }
                out[a][i] = alpha * s0 - iso * ga[a][i] + tg;
            }
    }
};

}  // namespace fo
