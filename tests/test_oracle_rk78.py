"""Pins of the oracle's seventh-order orbit integrator (cfg.ode = 2): the
"7th-order Runge-Kutta scheme" of Sec. 3 ("Waveform computation"), read as
Fehlberg's embedded 7(8) pair, stepped node to node.

The pins do not re-run the oracle's own formulas:
  * the oracle's constants, recovered as exact rationals, satisfy the
    Runge-Kutta order conditions (Butcher rooted trees generated here) in
    exact arithmetic: every tree up to order 7 for the kept weights (and not
    every tree of order 8), up to order 8 for the error-estimate weights;
  * with one step per coarse interval, halving the interval divides the
    node error by about 2^7 (the order-7 solution is the one propagated);
  * the nodes agree with an independent integrator (SciPy's DOP853 at a far
    tighter tolerance, sampled with its own dense output);
  * Peters' closed form nu(e) holds on the orbit to the tolerance where the
    step control has to subdivide the coarse intervals;
  * the nodes and the stopping node agree with the classical RK4 path
    (pinned elsewhere), forward and backward from the LSO.
"""
from fractions import Fraction

import numpy as np
import pytest
from scipy.integrate import solve_ivp

import oracle as O
from paper_2311_17174_amd import workloads as W
from tests.butcher import defects, exact_failures

TSUN = 4.925490947641267e-6


def cfg(w, **kw):
    return O.OracleConfig(T_obs=w.T_obs, dt=w.dt, N=w.N, n_harm=w.n_harm,
                          coarse_log2=w.coarse_log2, **kw)


def _rational(x):
    q = Fraction(float(x)).limit_denominator(10000)
    assert float(q) == float(x), x
    return q


def test_tableau_order_conditions():
    c, A, b7, b8 = O.rk78_tableau()
    assert A.shape == (13, 12)
    At = np.zeros((13, 13))
    At[:, :12] = A
    assert np.all(np.triu(At) == 0.0)                            # explicit
    np.testing.assert_allclose(At.sum(axis=1), c, rtol=0, atol=2e-15)
    Aq = [[_rational(v) for v in row] for row in At]
    cq = [_rational(v) for v in c]
    assert all(sum(Aq[i]) == cq[i] for i in range(13))
    w7 = [_rational(v) for v in b7]
    w8 = [_rational(v) for v in b8]
    assert exact_failures(w7, Aq, 8) == [8]                      # exactly order 7
    assert exact_failures(w8, Aq, 9) == [9]                      # exactly order 8
    # floating point: a planted wrong digit in any weight breaks the conditions
    assert defects(b7, At, 7) < 5e-15 and defects(b8, At, 8) < 5e-15
    for i in np.flatnonzero(b7):
        bad = b7.copy()
        bad[i] *= 1 + 1e-9
        assert defects(bad, At, 7) > 1e-12


def _scipy_orbit(p, t_nodes, rtol=1e-13, lo_only=False, backward_from=None):
    """Eq. (1) by SciPy's DOP853 with the oracle's right-hand side, sampled at
    t_nodes with SciPy's own dense output."""
    def f(t, y):
        return O.rhs(y, p, lo_only)
    if backward_from is None:
        y0 = np.array([p[5], p[4], p[6], p[3], p[7]])
        span = (0.0, t_nodes[-1])
    else:
        y0 = backward_from
        span = (t_nodes[-1], 0.0)
    s = solve_ivp(f, span, y0, method="DOP853", rtol=rtol, atol=1e-30 + rtol * 1e-3,
                  dense_output=True)
    assert s.success
    return s.sol(t_nodes).T


def _near_plunge(M=1e5, e0=0.3, frac=0.5):
    p = W.injection(M=M, e0=e0)
    p[4] = frac * ((1 - e0 * e0) / (6 + 2 * e0)) ** 1.5 / (2 * np.pi * M * TSUN)
    return p


@pytest.mark.parametrize("M,frac,lg,cl", [(1e5, 0.5, 16, 13), (1e5, 0.3, 18, 15)])
def test_seventh_order_convergence(M, frac, lg, cl):
    """rtol 1e-3: every step is one whole coarse interval (no rejections), so
    the nodes are those of the fixed-step method.  Halving the interval
    divides the error in nu by 2^7 = 128 for an order-7 method, pulled up
    a little by the next term (about 160 here); propagating the order-8
    weights instead gives 250-270 at the same steps."""
    p = _near_plunge(M=M, frac=frac)
    errs = []
    for c_l in (cl, cl - 1):
        c = O.OracleConfig(T_obs=10.0 * 2 ** lg, dt=10.0, N=1 << lg, n_harm=2, coarse_log2=c_l,
                           ode=2, rtol=1e-3, atol=1e-3)
        orb, kw = O.orbit(p[None], c)
        K = c.n_intervals
        assert kw[0] == K
        assert list(O.orbit_steps(p[None], c)[0]) == [K, 0]
        ref = _scipy_orbit(p, np.arange(K + 1) * 10.0 * 2 ** c_l, rtol=2.3e-14)
        errs.append(np.max(np.abs(orb[0, :, 1] / ref[:, 1] - 1)))
    assert errs[1] > 3e-13                    # well above the reference's own error
    assert 110 < errs[0] / errs[1] < 200, errs


@pytest.mark.parametrize("rtol", [1e-8, 1e-11])
def test_nodes_match_an_independent_integrator(rtol):
    w = W.config1()
    p = W.injection()
    c = cfg(w, ode=2, rtol=rtol, atol=rtol)
    orb, kw = O.orbit(p[None], c)
    K = w.n_intervals
    assert kw[0] == K
    hc = w.dt * (1 << w.coarse_log2)
    ref = _scipy_orbit(p, np.arange(K + 1) * hc)
    y = orb[0, :, :5]
    assert np.max(np.abs(y[:, 1] / ref[:, 1] - 1)) < rtol
    assert np.max(np.abs(y[:, 3] - ref[:, 3])) < rtol
    assert np.max(np.abs(y[:, 0] - ref[:, 0])) < rtol * np.max(np.abs(ref[:, 0]))
    assert np.max(np.abs(y[:, 2] - ref[:, 2])) < rtol * np.max(np.abs(ref[:, 2])) + rtol
    assert np.max(np.abs(y[:, 4] - ref[:, 4])) < rtol * np.max(np.abs(ref[:, 4])) + rtol
    # node derivatives are the right-hand side at the node state
    for k in (0, 7, K // 2, K):
        np.testing.assert_allclose(orb[0, k, 5:], O.rhs(orb[0, k, :5], p), rtol=1e-15, atol=0)


def test_subdivided_intervals_match_an_independent_integrator():
    """Coarse intervals of 2^19 dt near the plunge: the step control splits
    them, and the nodes still hold the tolerance (backward from the LSO)."""
    p = W.injection(M=3e5, e0=0.3)
    rtol = 1e-10
    c = O.OracleConfig(T_obs=W.YEAR, dt=10.0, N=1 << 22, n_harm=2, coarse_log2=19,
                       ic_lso=True, ode=2, rtol=rtol, atol=rtol)
    orb, kw = O.orbit(p[None], c)
    K = c.n_intervals
    assert kw[0] == K
    steps = O.orbit_steps(p[None], c)[0]
    assert steps[0] > 2 * K
    ref = _scipy_orbit(p, np.arange(K + 1) * 10.0 * 2 ** 19,
                       backward_from=orb[0, K, :5].copy())
    assert np.max(np.abs(orb[0, :, 1] / ref[:, 1] - 1)) < 10 * rtol
    assert np.max(np.abs(orb[0, :, 3] - ref[:, 3])) < 10 * rtol


def test_peters_invariant_tracks_the_tolerance():
    """Leading-order ODE, a = 0, backward from the LSO over coarse intervals
    of 2^19 dt (so that the step control subdivides them): nu(e) of Peters'
    closed form through (e_LSO, nu_LSO) holds to about rtol, and tighter
    tolerances take more steps."""
    eL = 0.2
    p = W.injection(M=3e5, a=0.0, e0=eL)
    nuL = ((1 - eL * eL) / (6 + 2 * eL)) ** 1.5 / (2 * np.pi * p[0] * TSUN)

    def nu_of_e(e):
        r = ((1 - e * e) / (1 - eL * eL) * (eL / e) ** (12 / 19) *
             ((1 + 121 * eL ** 2 / 304) / (1 + 121 * e * e / 304)) ** (870 / 2299))
        return nuL * r ** 1.5

    prev_err, prev_steps = np.inf, 0
    for rtol in (1e-6, 1e-8, 1e-10, 1e-12):
        c = O.OracleConfig(T_obs=W.YEAR, dt=10.0, N=1 << 22, n_harm=2, coarse_log2=19,
                           lo_only=True, ic_lso=True, ode=2, rtol=rtol, atol=rtol)
        orb, kw = O.orbit(p[None], c)
        assert kw[0] == c.n_intervals
        assert orb[0, -1, 1] == nuL and orb[0, -1, 3] == eL
        err = np.max(np.abs(orb[0, :, 1] / nu_of_e(orb[0, :, 3]) - 1))
        steps = O.orbit_steps(p[None], c)[0]
        assert err < 5 * rtol and err < prev_err
        assert steps[0] > prev_steps
        prev_err, prev_steps = err, steps[0]


def test_step_count_follows_the_order_eight_estimate():
    """Error-per-step control on an estimate of order 8 in the step: steps
    h ~ rtol^(1/8), so six decades of tolerance multiply the accepted steps
    by about 10^(6/8) = 5.6 (an estimate of order 5 would give 16)."""
    for M in (1e5, 3e5):
        p = W.injection(M=M, e0=0.3)
        s = [O.orbit_steps(p[None], O.OracleConfig(
            T_obs=W.YEAR, dt=10.0, N=1 << 22, n_harm=2, coarse_log2=19, ic_lso=True,
            ode=2, rtol=r, atol=r))[0, 0] for r in (1e-7, 1e-13)]
        assert 3.0 < s[1] / s[0] < 8.0, s


def test_agrees_with_rk4():
    """At config 2's coarse step the order-7 nodes agree with the classical
    RK4 nodes within RK4's own error, and stop at the same node."""
    w = W.config2()
    P = W.walkers(w, B=4)
    a, ka = O.orbit(P, cfg(w, ode=2, rtol=1e-12, atol=1e-12))
    r, kr = O.orbit(P, cfg(w))
    assert np.array_equal(ka, kr)
    for b in range(4):
        n = kr[b] + 1
        assert np.max(np.abs(a[b, :n, 1] / r[b, :n, 1] - 1)) < 1e-11
        assert np.max(np.abs(a[b, :n, 0] - r[b, :n, 0])) < 1e-6          # radians
        assert np.max(np.abs(a[b, :n, 3] - r[b, :n, 3])) < 1e-11


def test_plunge_inside_the_window():
    """A walker that reaches the LSO inside the window stops at the same node
    as with RK4 (or one apart, where the crossing falls next to a node)."""
    w = W.config1()
    p = W.injection()
    e0 = p[3]
    p[4] = 0.97 * ((1 - e0 * e0) / (6 + 2 * e0)) ** 1.5 / (2 * np.pi * p[0] * TSUN)
    a, ka = O.orbit(p[None], cfg(w, ode=2, rtol=1e-11, atol=1e-11))
    r, kr = O.orbit(p[None], cfg(w))
    assert 0 < kr[0] < w.n_intervals
    assert abs(int(ka[0]) - int(kr[0])) <= 1
    n = min(ka[0], kr[0]) + 1
    assert np.max(np.abs(a[0, :n, 1] / r[0, :n, 1] - 1)) < 1e-9
    assert np.all(a[0, ka[0] + 1:] == 0.0)


def test_lso_mode_matches_rk4_backward():
    w = W.config1()
    p = W.injection(e0=0.3)
    a, ka = O.orbit(p[None], cfg(w, ic_lso=True, ode=2, rtol=1e-12, atol=1e-12))
    r, kr = O.orbit(p[None], cfg(w, ic_lso=True))
    assert ka[0] == kr[0] == w.n_intervals
    assert np.array_equal(a[0, -1], r[0, -1])               # the LSO state itself
    assert np.max(np.abs(a[0, :, 1] / r[0, :, 1] - 1)) < 1e-11
    # an unphysical history is still flagged
    q = W.injection(M=2e4, mu=10.0, e0=0.7)
    long = O.OracleConfig(T_obs=1.0 * W.YEAR, dt=10.0, N=1 << 22, n_harm=2, ic_lso=True,
                          ode=2, rtol=1e-10, atol=1e-10)
    _, kw = O.orbit(q[None], long)
    assert kw[0] == -1


def test_waveform_agrees_with_the_other_integrators():
    """The same walker's two-channel waveform from the order-7 orbit, the RK4
    orbit and the Dormand-Prince orbit agree to the orbits' errors: the 5(4)
    pair's nodes come from its order-4 continuous extension (a few 1e-9 rad
    of phase at rtol 1e-12), RK4 and the order-7 pair agree to 2e-12 rad at
    this coarse step."""
    w = W.config1()
    p = W.injection()
    x7 = O.waveform(p[None], cfg(w, ode=2, rtol=1e-12, atol=1e-12))
    x5 = O.waveform(p[None], cfg(w, ode=1, rtol=1e-12, atol=1e-12))
    x4 = O.waveform(p[None], cfg(w))
    scale = np.max(np.abs(x4))
    assert scale > 0
    assert np.max(np.abs(x7 - x4)) < 1e-10 * scale
    assert np.max(np.abs(x7 - x5)) < 1e-7 * scale


def test_bad_tolerances_are_rejected():
    w = W.config1()
    p = W.injection()
    for rtol, atol in ((0.0, 1e-10), (1e-14, 1e-10), (1e-2, 1e-10), (1e-10, -1.0),
                       (1e-10, float("inf")), (float("nan"), 1e-10)):
        with pytest.raises(ValueError):
            O.orbit(p[None], cfg(w, ode=2, rtol=rtol, atol=atol))
