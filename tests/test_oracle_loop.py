"""Pins of the oracle's level-set loop (Algorithm 1 with the PPL constraint
method, Section "Lagrangian method", eqs. lagrangian, lag_method, S0andS1,
and the stopping criterion of Section "Other implementation aspects")
against facts that do not come from the oracle's formulas: convergence of
the multiplier iteration to the KKT point of a constrained quadratic when a
gradient step takes the place of the transport, its fixed points, the value
of the Lagrangian there, the stopping rule on histories whose outcome is
fixed by the definition, and the direction in which the loop moves the cost
and the volume."""
import numpy as np
import pytest

import fo_inputs as fi
from oracle import loop as ol


def gradient_ppl(a, Cm, eta=0.2, iters=20000):
    """min 1/2 |x - a|^2 subject to Cm x = 1, with the PPL multipliers and a
    gradient step on the Lagrangian in place of the transport equation."""
    ppl = ol.PPL(Cm.shape[0])
    x = np.zeros_like(a)
    for i in range(iters):
        C = Cm @ x
        if i >= 1:
            ppl.update(C)
        x = x - eta * ((x - a) + Cm.T @ ppl.lam)
    return x, ppl


@pytest.mark.parametrize("nc", [1, 2])
def test_ppl_reaches_the_kkt_point_of_a_constrained_quadratic(nc):
    rng = np.random.default_rng(3 + nc)
    a = rng.uniform(-1, 1, 4)
    Cm = rng.uniform(-1, 1, (nc, 4))
    # KKT of min 1/2|x-a|^2, Cm x = 1: x = a - Cm^T lam, Cm Cm^T lam = Cm a - 1
    lam_star = np.linalg.solve(Cm @ Cm.T, Cm @ a - 1.0)
    x_star = a - Cm.T @ lam_star
    x, ppl = gradient_ppl(a, Cm)
    np.testing.assert_allclose(x, x_star, atol=1e-9)
    np.testing.assert_allclose(ppl.lam, lam_star, atol=1e-9)
    np.testing.assert_allclose(ppl.mu, lam_star, atol=1e-6)
    np.testing.assert_allclose(ppl.z, 0.0, atol=1e-9)
    # at the KKT point the Lagrangian is the cost
    J = 0.5 * float((x - a) @ (x - a))
    assert ppl.lagrangian(J, Cm @ x) == pytest.approx(J, abs=1e-9)


def test_ppl_fixed_point_and_step_decay():
    """Constraint met and lambda = mu: the multipliers stay; delta still
    shrinks geometrically."""
    ppl = ol.PPL(2, lam=[0.7, -0.2], mu=[0.7, -0.2], z=[0.0, 0.0])
    d0 = ppl.delta
    for k in range(5):
        ppl.update([1.0, 1.0])
    np.testing.assert_array_equal(ppl.lam, [0.7, -0.2])
    np.testing.assert_array_equal(ppl.mu, [0.7, -0.2])
    np.testing.assert_array_equal(ppl.z, [0.0, 0.0])
    assert ppl.delta == pytest.approx(d0 * ol.PPL_R ** 5, rel=1e-15)


def test_ppl_multiplier_sign_follows_the_violation():
    """Too much volume (C > 1) makes lambda positive, too little negative."""
    for C, sign in ((1.2, 1.0), (0.8, -1.0)):
        ppl = ol.PPL(1)
        ppl.update([C])
        assert np.sign(ppl.lam[0]) == sign and np.sign(ppl.z[0]) == sign


def test_stopping_rule_on_fixed_histories():
    n = 40
    flat = [5.0] * n
    # unconstrained: a constant cost stops at the first checked iteration
    stops = [i for i in range(n) if ol.should_stop(i, flat, None, None, start_to_check=30, prev=10)]
    assert stops and stops[0] == 31
    # a cost that grows 5% per iteration never meets cost_tol = 1e-2
    grow = [1.05 ** i for i in range(n)]
    assert not any(ol.should_stop(i, grow, None, None, start_to_check=30, prev=10) for i in range(n))
    # a single jump inside the window blocks the stop until it leaves it
    jump = [5.0] * n
    jump[31] = 6.0  # in the windows of iterations 31 (as J_i) to 34
    first = next(i for i in range(n) if ol.should_stop(i, jump, None, None, start_to_check=30, prev=3))
    assert first == 35
    # constrained: a flat Lagrangian still needs the constraint within ctrn_tol
    Cbad = [np.array([1.05])] * n
    Cok = [np.array([1.005])] * n
    assert not any(ol.should_stop(i, flat, flat, Cbad, start_to_check=30, prev=10) for i in range(n))
    assert ol.should_stop(31, flat, flat, Cok, start_to_check=30, prev=10)


def test_loop_lowers_the_cost_and_the_constraint_pulls_the_volume():
    """Compliance falls over the first iterations of the unconstrained loop
    (each step follows a descent direction: dJ(theta) = -B(theta, theta));
    with a volume target below the current volume the multiplier turns
    positive and the volume ends below the unconstrained run's.  dfactor = 1
    (the paper's upper recommendation) makes the steps long enough to move
    the interface across elements on this coarse mesh."""
    w = fi.cantilever_2d((48, 24))
    free = ol.optimize(w, 3, V=None, rtol=1e-11, dfactor=1.0)
    J = [r.J for r in free.records]
    assert J[1] < J[0] and J[2] < J[1]
    assert all(r.lam == 0.0 for r in free.records)
    vol0 = free.records[0].vol
    con = ol.optimize(w, 3, V=0.8 * vol0, rtol=1e-11, dfactor=1.0)
    assert con.records[0].lam == 0.0 and con.records[0].J == pytest.approx(free.records[0].J, rel=1e-12)
    assert con.records[1].C > 1.0 and con.records[1].lam > 0.0
    assert con.records[2].vol < free.records[2].vol
    for r in con.records:
        assert r.steps >= 8 and r.steps <= 16 and r.dt * r.steps == pytest.approx(r.t_end, rel=1e-14)
