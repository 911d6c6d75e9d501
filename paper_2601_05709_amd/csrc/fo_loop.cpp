// The level-set loop (Algorithm 1): state solve, cost and constraint, the
// stopping test, the Proximal-Perturbed Lagrangian multiplier update
// (Section "Lagrangian method", eqs. lagrangian, lag_method, S0andS1), the
// velocity solve, the adaptive final time and step count (Section "Other
// implementation aspects", eqs. tend and steps), the paper's transport step
// and, every reinit_step iterations, the reinitialisation.  Every step runs
// on the device through the library's entry points; the host keeps the
// multipliers and the histories (a few scalars per iteration).  One driver
// runs the loop for each model: the compliance problem (fo_optimize), the
// heat-conduction model (fo_optimize_heat) and the inverse problem
// (fo_optimize_inverse, no constraint); a model supplies the evaluation of
// cost and volume for the current level set and the descent right-hand side.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <functional>
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

bool loop_opts_ok(const fo_loop_opts *o)
{
    if (o->n_iter < 0 || !(o->dfactor > 0.0) || !(o->t_min > 0.0) || !(o->t_max > o->t_min) || o->s_min < 1 ||
        o->s_max < o->s_min || o->prev < 1 || o->start_to_check < 0)
        return false;
    if (o->reinit_step < 0 || (o->reinit_step > 0 && (o->reinit_iters < 1 || !(o->reinit_t > 0.0)))) return false;
    if (o->V > 0.0 && (!(o->ppl_r > 0.0 && o->ppl_r < 1.0) || !(o->ppl_alpha > 0.0) || !(o->ppl_beta > 0.0) ||
                       !(o->ppl_delta0 > 0.0)))
        return false;
    return true;
}

// A model's part of an iteration.  eval: set the level set phi, solve the
// state (and adjoints), return the cost and the volume on the host and the
// state solves' operator applications.  rhs: the descent right-hand side of
// S^J + lambda S^C for the last evaluation (device [n_dofs]).
struct Model {
    std::function<int(const double *phi, double *J, double *vol, int32_t *state_iters)> eval;
    std::function<int(double lambda, double *rhs)> rhs;
};

// Copies k device doubles to the host (stream-ordered, then waits).
int fetch(fo_ctx *c, double *host, const double *dev, int k)
{
    if (hipMemcpyAsync(host, dev, k * sizeof(double), hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
        fo::wait_stream(c->stream) != hipSuccess)
        return FO_ERR_HIP;
    return FO_OK;
}

// The loop on the context c (velocity, transport and reinitialisation run
// on c); rhs, theta, btt: device work space [n_dofs], [n_dofs], [1].
int run_loop(fo_ctx *c, const fo_loop_opts *o, Model &m, double *phi, double *rhs, double *theta, double *btt,
             fo_loop_record *records, int32_t *n_done, int32_t *stopped)
{
    const bool constrained = o->V > 0.0;
    const double Vd = constrained ? o->V : 1.0;
    Ppl ppl{o->ppl_r, o->ppl_alpha, o->ppl_beta, o->ppl_delta0};
    std::vector<double> Jh, Lh, Ch;
    int result = FO_OK;
    for (int i = 0; i < o->n_iter; ++i) {
        fo_loop_record &rec = records[i];
        rec = fo_loop_record{};
        rec.B_tt = rec.t_end = rec.dt = std::numeric_limits<double>::quiet_NaN();
        fo_solve_stats ds{}, ts{};
        double J = 0.0, vol = 0.0;
        int st = m.eval(phi, &J, &vol, &rec.state_iters);
        if (st < 0) {
            rec.status = st;
            result = st;
            *n_done = i + 1;
            break;
        }
        rec.J = J;
        rec.vol = vol;
        rec.C = vol / Vd;
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
        // S = S^J + lambda S^C
        st = worse(st, m.rhs(rec.lambda, rhs));
        if (st >= 0) st = worse(st, fo_descent_solve(c, &o->velocity, rhs, theta, &o->descent, &ds, btt));
        double h = 0.0;
        if (st >= 0) st = worse(st, fetch(c, &h, btt, 1));
        rec.descent_iters = ds.iters_inner;
        if (st >= 0) {
            rec.B_tt = h;
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
    (void)fo::wait_stream(c->stream);
    return result;
}

}  // namespace

size_t fo::optimize_work_doubles(const fo_ctx *c) { return (size_t)(3 * c->ndof + 4); }

// fo_optimize on caller-provided work vectors (optimize_work_doubles).
int fo::optimize_on(fo_ctx *c, const fo_loop_opts *o, const double *b, double *phi, fo_loop_record *records,
                    int32_t *n_done, int32_t *stopped, double *work)
{
    if (!c || !o || !b || !phi || !records || !n_done || !stopped || !work || !loop_opts_ok(o)) return FO_ERR_ARG;
    *n_done = 0;
    *stopped = 0;
    const int64_t n = c->ndof;
    double *u = work, *rhs = u + n, *theta = rhs + n, *scal = theta + n;  // scal: J, vol, B_tt
    const double Vd = o->V > 0.0 ? o->V : 1.0;
    Model m;
    m.eval = [&](const double *ph, double *J, double *vol, int32_t *its) -> int {
        fo_solve_stats ss{};
        int st = fo_set_levelset(c, ph);
        if (st == FO_OK) st = fo_state_solve(c, b, u, 1, 1, &o->state, &ss);
        *its = ss.iters_inner;
        // the derivative without the constraint term: the multiplier is not known yet
        if (st >= 0) st = worse(st, fo_shape_derivative(c, u, 1, 1, 0.0, Vd, rhs, nullptr, scal, scal + 1));
        double h[2] = {0.0, 0.0};
        if (st >= 0) st = worse(st, fetch(c, h, scal, 2));
        *J = h[0];
        *vol = h[1];
        return st;
    };
    m.rhs = [&](double lambda, double *r) -> int {
        if (lambda == 0.0) return FO_OK;  // rhs holds the derivative without the constraint term
        return fo_shape_derivative(c, u, 1, 1, lambda, Vd, r, nullptr, scal, scal + 1);
    };
    return run_loop(c, o, m, phi, rhs, theta, scal + 2, records, n_done, stopped);
}

extern "C" {

int fo_time_steps(double B_tt, double dfactor, double t_min, double t_max, int32_t s_min, int32_t s_max,
                  double *t_end, int32_t *steps, double *dt)
{
    if (!t_end || !steps || !dt || !(dfactor > 0.0) || !(t_min > 0.0) || !(t_max > t_min) || s_min < 1 ||
        s_max < s_min || !(B_tt == B_tt))
        return FO_ERR_ARG;
    fo_loop_opts o{};
    o.dfactor = dfactor;
    o.t_min = t_min;
    o.t_max = t_max;
    o.s_min = s_min;
    o.s_max = s_max;
    int s = 0;
    time_steps(B_tt, o, t_end, &s);
    *steps = s;
    *dt = *t_end / s;
    return FO_OK;
}

int fo_optimize(fo_ctx *c, const fo_loop_opts *o, const double *b, double *phi, fo_loop_record *records,
                int32_t *n_done, int32_t *stopped)
{
    if (!c || !o || !b || !phi || !records || !n_done || !stopped || !loop_opts_ok(o)) return FO_ERR_ARG;
    double *work = nullptr;
    if (fo::device_malloc((void **)&work, fo::optimize_work_doubles(c) * sizeof(double)) != hipSuccess)
        return FO_ERR_NOMEM;
    const int rc = fo::optimize_on(c, o, b, phi, records, n_done, stopped, work);
    (void)hipFree(work);
    return rc;
}

int fo_optimize_heat(fo_ctx *c, const fo_loop_opts *o, const uint8_t *gamma0, const double *f, double *phi,
                     fo_loop_record *records, int32_t *n_done, int32_t *stopped)
{
    if (!c || !o || !gamma0 || !f || !phi || !records || !n_done || !stopped || !loop_opts_ok(o)) return FO_ERR_ARG;
    *n_done = 0;
    *stopped = 0;
    const int64_t N = c->N, n = c->ndof;
    double *work = nullptr;
    if (fo::device_malloc((void **)&work, (size_t)(2 * N + 2 * n + 4) * sizeof(double)) != hipSuccess)
        return FO_ERR_NOMEM;
    double *b = work, *u = b + N, *rhs = u + N, *theta = rhs + n, *scal = theta + n;  // scal: J, vol, B_tt
    const double Vd = o->V > 0.0 ? o->V : 1.0;
    int rc = fo_heat_load(c, f, b);  // the load does not depend on the level set
    if (rc != FO_OK) {
        (void)hipFree(work);
        return rc;
    }
    Model m;
    m.eval = [&](const double *ph, double *J, double *vol, int32_t *its) -> int {
        fo_solve_stats ss{};
        int st = fo_set_levelset(c, ph);
        if (st == FO_OK) st = fo_heat_solve(c, gamma0, b, u, &o->state, &ss);
        *its = ss.iters_inner;
        if (st >= 0) st = worse(st, fo_heat_derivative(c, u, f, 0.0, Vd, rhs, scal, scal + 1));
        double h[2] = {0.0, 0.0};
        if (st >= 0) st = worse(st, fetch(c, h, scal, 2));
        *J = h[0];
        *vol = h[1];
        return st;
    };
    m.rhs = [&](double lambda, double *r) -> int {
        if (lambda == 0.0) return FO_OK;
        return fo_heat_derivative(c, u, f, lambda, Vd, r, scal, scal + 1);
    };
    rc = run_loop(c, o, m, phi, rhs, theta, scal + 2, records, n_done, stopped);
    (void)hipFree(work);
    return rc;
}

int fo_optimize_inverse(fo_ctx *cf, fo_ctx *cg, const fo_loop_opts *o, int32_t n_pairs, int64_t ld, const double *f,
                        const double *g, double kappa, double alpha, double beta, double *phi,
                        fo_loop_record *records, int32_t *n_done, int32_t *stopped)
{
    if (!cf || !cg || !o || !f || !g || !phi || !records || !n_done || !stopped || !loop_opts_ok(o))
        return FO_ERR_ARG;
    if (n_pairs < 1 || ld < n_pairs || o->V > 0.0) return FO_ERR_ARG;  // the inverse problem has no constraint
    *n_done = 0;
    *stopped = 0;
    const int64_t n = cf->ndof;
    double *work = nullptr;
    const size_t n_dbl = (size_t)(4 * n * ld + 2 * n + n_pairs + 1);
    if (fo::device_malloc((void **)&work, n_dbl * sizeof(double)) != hipSuccess) return FO_ERR_NOMEM;
    double *u = work, *v = u + n * ld, *p = v + n * ld, *q = p + n * ld, *rhs = q + n * ld, *theta = rhs + n,
           *Jd = theta + n, *btt = Jd + n_pairs;
    std::vector<double> Jk((size_t)n_pairs);
    Model m;
    m.eval = [&](const double *ph, double *J, double *vol, int32_t *its) -> int {
        fo_solve_stats ss{};
        int st = fo_inverse_states(cf, cg, ph, n_pairs, ld, f, g, kappa, alpha, beta, &o->state, u, v, p, q, Jd,
                                   &ss);
        *its = ss.iters_inner;
        if (st >= 0) st = worse(st, fetch(cf, Jk.data(), Jd, n_pairs));
        *J = 0.0;
        for (int k = 0; k < n_pairs; ++k) *J += Jk[(size_t)k];  // pair order
        *vol = 0.0;
        return st;
    };
    m.rhs = [&](double, double *r) -> int {
        return fo_inverse_derivative(cf, n_pairs, ld, u, v, p, q, g, kappa, alpha, r);
    };
    const int rc = run_loop(cf, o, m, phi, rhs, theta, btt, records, n_done, stopped);
    (void)hipFree(work);
    return rc;
}

}  // extern "C"
