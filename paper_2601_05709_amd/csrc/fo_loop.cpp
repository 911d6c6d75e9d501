// The level-set loop (Algorithm 1): state solve, cost and constraint, the
// stopping test, the Proximal-Perturbed Lagrangian multiplier update
// (Section "Lagrangian method", eqs. lagrangian, lag_method, S0andS1), the
// velocity solve, the adaptive final time and step count (Section "Other
// implementation aspects", eqs. tend and steps), the paper's transport step
// and, every reinit_step iterations, the reinitialisation.  Every step runs
// on the device through the library's entry points; the host keeps the
// multipliers and the histories (a few scalars per iteration).  The same
// loop drives the compliance problem (fo_optimize) and the inverse problem
// (fo_optimize_inverse: states, adjoints and derivative of Section "Inverse
// problem", no constraint).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <limits>
#include <vector>

#include "fo_internal.h"

namespace {

// Multiplier state for one constraint (N_c = 1).
struct Ppl {
    double r, alpha, beta, delta;
    double z = 0.0, lam = 0.0, mu = 0.0;

    void update(double C)
    {
        const double d = lam - mu;
        mu += delta * d / (d * d + 1.0);
        lam = mu + alpha / (1.0 + alpha * beta) * (C - 1.0);
        z = (lam - mu) / alpha;
        delta *= r;
    }
    double lagrangian(double J, double C) const
    {
        const double d = lam - mu;
        return J + lam * (C - 1.0) + mu * z + 0.5 * alpha * z * z + 0.5 * beta * d * d;
    }
};

// Largest |v_i - v_j| over the `prev` entries before i.
double window_change(const std::vector<double> &v, int i, int prev)
{
    double m = 0.0;
    for (int j = i - prev; j < i; ++j) m = std::max(m, std::fabs(v[i] - v[j]));
    return m;
}

bool stop_test(int i, const std::vector<double> &J, const std::vector<double> &L, const std::vector<double> &C,
               bool constrained, const fo_loop_opts &o)
{
    if (i <= o.start_to_check || i < o.prev) return false;
    if (!constrained) return window_change(J, i, o.prev) < o.cost_tol * std::fabs(J[i]);
    return window_change(L, i, o.prev) < o.lgrn_tol * std::fabs(L[i]) && std::fabs(C[i] - 1.0) < o.ctrn_tol;
}

// t_end = dfactor / B(theta, theta) and the step count (eqs. tend, steps),
// both clamped; the count is rounded half to even.
void time_steps(double B_tt, const fo_loop_opts &o, double *t_end, int *steps)
{
    double t = o.dfactor / std::max(B_tt, 1e-300);
    t = std::min(std::max(t, o.t_min), o.t_max);
    double s = (double)(o.s_max - o.s_min) * std::pow((t - o.t_min) / (o.t_max - o.t_min), 1.0 / 6.0) +
               (double)o.s_min;
    s = std::min(std::max(s, (double)o.s_min), (double)o.s_max);
    *t_end = t;
    *steps = (int)std::nearbyint(s);
}

int worse(int a, int b)
{
    if (a < 0 || b < 0) return std::min(a, b);
    return std::max(a, b);
}

}  // namespace

extern "C" {

int fo_optimize(fo_ctx *c, const fo_loop_opts *o, const double *b, double *phi, fo_loop_record *records,
                int32_t *n_done, int32_t *stopped)
{
    if (!c || !o || !b || !phi || !records || !n_done || !stopped) return FO_ERR_ARG;
    if (o->n_iter < 0 || !(o->dfactor > 0.0) || !(o->t_min > 0.0) || !(o->t_max > o->t_min) || o->s_min < 1 ||
        o->s_max < o->s_min || o->prev < 1 || o->start_to_check < 0)
        return FO_ERR_ARG;
    if (o->reinit_step < 0 || (o->reinit_step > 0 && (o->reinit_iters < 1 || !(o->reinit_t > 0.0))))
        return FO_ERR_ARG;
    const bool constrained = o->V > 0.0;
    if (constrained && (!(o->ppl_r > 0.0 && o->ppl_r < 1.0) || !(o->ppl_alpha > 0.0) || !(o->ppl_beta > 0.0) ||
                        !(o->ppl_delta0 > 0.0)))
        return FO_ERR_ARG;
    *n_done = 0;
    *stopped = 0;
    const int64_t n = c->ndof;
    double *work = nullptr;
    if (hipMalloc(&work, (size_t)(3 * n + 4) * sizeof(double)) != hipSuccess) return FO_ERR_NOMEM;
    double *u = work, *rhs = u + n, *theta = rhs + n, *scal = theta + n;  // scal: J, vol, B_tt
    const double Vd = constrained ? o->V : 1.0;
    Ppl ppl{o->ppl_r, o->ppl_alpha, o->ppl_beta, o->ppl_delta0};
    std::vector<double> Jh, Lh, Ch;
    int result = FO_OK;
    auto fetch = [&](double *host, const double *dev, int k) -> int {
        if (hipMemcpyAsync(host, dev, k * sizeof(double), hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
            hipStreamSynchronize(c->stream) != hipSuccess)
            return FO_ERR_HIP;
        return FO_OK;
    };
    for (int i = 0; i < o->n_iter; ++i) {
        fo_loop_record &rec = records[i];
        rec = fo_loop_record{};
        rec.B_tt = rec.t_end = rec.dt = std::numeric_limits<double>::quiet_NaN();
        int st = fo_set_levelset(c, phi);
        fo_solve_stats ss{}, ds{}, ts{};
        if (st == FO_OK) st = fo_state_solve(c, b, u, 1, 1, &o->state, &ss);
        if (st >= 0) st = worse(st, fo_shape_derivative(c, u, 1, 1, 0.0, Vd, rhs, nullptr, scal, scal + 1));
        double h[3] = {0.0, 0.0, 0.0};
        if (st >= 0) st = worse(st, fetch(h, scal, 2));
        rec.state_iters = ss.iters_inner;
        if (st < 0) {
            rec.status = st;
            result = st;
            *n_done = i + 1;
            break;
        }
        rec.J = h[0];
        rec.vol = h[1];
        rec.C = h[1] / Vd;
        if (constrained) {
            if (i >= 1) ppl.update(rec.C);
            rec.lambda = ppl.lam;
            rec.L = ppl.lagrangian(rec.J, rec.C);
        } else {
            rec.L = rec.J;
        }
        Jh.push_back(rec.J);
        Lh.push_back(rec.L);
        Ch.push_back(rec.C);
        *n_done = i + 1;
        if (stop_test(i, Jh, Lh, Ch, constrained, *o)) {
            rec.status = st;
            result = worse(result, st);
            *stopped = 1;
            break;
        }
        // S = S^J + lambda S^C: the derivative again, with the multiplier
        if (rec.lambda != 0.0)
            st = worse(st, fo_shape_derivative(c, u, 1, 1, rec.lambda, Vd, rhs, nullptr, scal, scal + 1));
        if (st >= 0) st = worse(st, fo_descent_solve(c, &o->velocity, rhs, theta, &o->descent, &ds, scal + 2));
        if (st >= 0) st = worse(st, fetch(h + 2, scal + 2, 1));
        rec.descent_iters = ds.iters_inner;
        if (st >= 0) {
            rec.B_tt = h[2];
            int steps = 0;
            time_steps(rec.B_tt, *o, &rec.t_end, &steps);
            rec.steps = steps;
            rec.dt = rec.t_end / steps;
            st = worse(st, fo_transport(c, theta, rec.dt, steps, o->smooth, phi, &o->transport, &ts));
            rec.transport_iters = ts.iters_inner;
        }
        if (st >= 0 && o->reinit_step > 0 && i % o->reinit_step == 0) {
            fo_solve_stats rs{};
            st = worse(st, fo_reinit(c, phi, o->reinit_iters, o->reinit_t, &o->transport, &rs));
            rec.reinit_iters = rs.iters_inner;
        }
        rec.status = st;
        result = worse(result, st);
        if (st < 0) break;
    }
    (void)hipStreamSynchronize(c->stream);
    (void)hipFree(work);
    return result;
}

int fo_optimize_inverse(fo_ctx *cf, fo_ctx *cg, const fo_loop_opts *o, int32_t n_pairs, int64_t ld, const double *f,
                        const double *g, double kappa, double alpha, double beta, double *phi,
                        fo_loop_record *records, int32_t *n_done, int32_t *stopped)
{
    if (!cf || !cg || !o || !f || !g || !phi || !records || !n_done || !stopped) return FO_ERR_ARG;
    if (n_pairs < 1 || ld < n_pairs || o->V > 0.0) return FO_ERR_ARG;  // the inverse problem has no constraint
    if (o->n_iter < 0 || !(o->dfactor > 0.0) || !(o->t_min > 0.0) || !(o->t_max > o->t_min) || o->s_min < 1 ||
        o->s_max < o->s_min || o->prev < 1 || o->start_to_check < 0)
        return FO_ERR_ARG;
    if (o->reinit_step < 0 || (o->reinit_step > 0 && (o->reinit_iters < 1 || !(o->reinit_t > 0.0))))
        return FO_ERR_ARG;
    *n_done = 0;
    *stopped = 0;
    const int64_t n = cf->ndof;
    double *work = nullptr;
    const size_t n_dbl = (size_t)(4 * n * ld + 2 * n + n_pairs + 1);
    if (hipMalloc(&work, n_dbl * sizeof(double)) != hipSuccess) return FO_ERR_NOMEM;
    double *u = work, *v = u + n * ld, *p = v + n * ld, *q = p + n * ld, *rhs = q + n * ld, *theta = rhs + n,
           *Jd = theta + n, *btt = Jd + n_pairs;
    std::vector<double> Jh, Jk((size_t)n_pairs);
    int result = FO_OK;
    auto fetch = [&](double *host, const double *dev, int k) -> int {
        if (hipMemcpyAsync(host, dev, k * sizeof(double), hipMemcpyDeviceToHost, cf->stream) != hipSuccess ||
            hipStreamSynchronize(cf->stream) != hipSuccess)
            return FO_ERR_HIP;
        return FO_OK;
    };
    for (int i = 0; i < o->n_iter; ++i) {
        fo_loop_record &rec = records[i];
        rec = fo_loop_record{};
        rec.B_tt = rec.t_end = rec.dt = std::numeric_limits<double>::quiet_NaN();
        fo_solve_stats ss{}, ds{}, ts{};
        int st = fo_inverse_states(cf, cg, phi, n_pairs, ld, f, g, kappa, alpha, beta, &o->state, u, v, p, q, Jd,
                                   &ss);
        if (st >= 0) st = worse(st, fetch(Jk.data(), Jd, n_pairs));
        rec.state_iters = ss.iters_inner;
        if (st < 0) {
            rec.status = st;
            result = st;
            *n_done = i + 1;
            break;
        }
        double J = 0.0;
        for (int k = 0; k < n_pairs; ++k) J += Jk[(size_t)k];  // pair order
        rec.J = rec.L = J;
        Jh.push_back(J);
        *n_done = i + 1;
        if (stop_test(i, Jh, Jh, Jh, false, *o)) {
            rec.status = st;
            result = worse(result, st);
            *stopped = 1;
            break;
        }
        st = worse(st, fo_inverse_derivative(cf, n_pairs, ld, u, v, p, q, g, kappa, alpha, rhs));
        if (st >= 0) st = worse(st, fo_descent_solve(cf, &o->velocity, rhs, theta, &o->descent, &ds, btt));
        double h = 0.0;
        if (st >= 0) st = worse(st, fetch(&h, btt, 1));
        rec.descent_iters = ds.iters_inner;
        if (st >= 0) {
            rec.B_tt = h;
            int steps = 0;
            time_steps(rec.B_tt, *o, &rec.t_end, &steps);
            rec.steps = steps;
            rec.dt = rec.t_end / steps;
            st = worse(st, fo_transport(cf, theta, rec.dt, steps, o->smooth, phi, &o->transport, &ts));
            rec.transport_iters = ts.iters_inner;
        }
        if (st >= 0 && o->reinit_step > 0 && i % o->reinit_step == 0) {
            fo_solve_stats rs{};
            st = worse(st, fo_reinit(cf, phi, o->reinit_iters, o->reinit_t, &o->transport, &rs));
            rec.reinit_iters = rs.iters_inner;
        }
        rec.status = st;
        result = worse(result, st);
        if (st < 0) break;
    }
    (void)hipStreamSynchronize(cf->stream);
    (void)hipFree(work);
    return result;
}

}  // extern "C"
