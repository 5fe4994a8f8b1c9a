"""Pin of the 1PN terms of the oracle's orbital equations (Eq. (1), the
BC04 forms) against the post-Newtonian chirp of a test mass on a circular
orbit, a result independent of BC04.

At e = 0 and a = 0, BC04 evolve the radial (mean-motion) frequency nu with
dnu/dt = (96 / 10 pi) (mu / M^3) x^{11/3} (1 + (1273/336) x^{2/3}), and the
pericentre with dgamma~/dt = 6 pi nu x^{2/3} (1 + ...), x = 2 pi M nu.  The
orbital (azimuthal) frequency is nu_phi = nu + (dgamma~/dt) / (2 pi); in its
variable y = (2 pi M nu_phi)^{2/3} the chirp of a test mass at 1PN order is
dnu_phi/dt = (96 / 10 pi) (mu / M^3) (2 pi M nu_phi)^{11/3} (1 - (743/336) y + ...)
(the 1PN flux and binding energy, mass ratio -> 0).  The two forms agree
only if both 1PN coefficients of the oracle are right: 1273/336 - 6 = -743/336.
"""
import numpy as np

import oracle as O
from paper_2311_17174_amd import workloads as W

TSUN = 4.925490947641267e-6


def _coef(p, nu):
    """(dnu_phi/dt / leading - 1) / y at nu, from the oracle's right-hand side."""
    M, mu = p[0] * TSUN, p[1] * TSUN
    f = O.rhs(np.array([0.0, nu, 0.0, 0.0, 0.0]), p)
    dn = nu * 1e-5
    dg = (O.rhs(np.array([0.0, nu + dn, 0.0, 0.0, 0.0]), p)[2] -
          O.rhs(np.array([0.0, nu - dn, 0.0, 0.0, 0.0]), p)[2]) / (2 * dn)
    nuphi = nu + f[2] / (2 * np.pi)
    dnuphi = f[1] * (1.0 + dg / (2 * np.pi))
    x = 2 * np.pi * M * nuphi
    lead = 96.0 / (10.0 * np.pi) * (mu / M ** 3) * x ** (11.0 / 3.0)
    y = x ** (2.0 / 3.0)
    return (dnuphi / lead - 1.0) / y


def test_circular_1pn_chirp_of_a_test_mass():
    p = W.injection(a=0.0, e0=0.0)
    nu = 1e-8                        # y ~ 5e-5: deep in the post-Newtonian regime
    # Richardson in y (y doubles when nu grows by 2^{3/2}) removes the O(y) term
    c = 2 * _coef(p, nu) - _coef(p, nu * 2 ** 1.5)
    # a wrong digit in 1273/336 moves the limit by at least 1/336 (2e-3
    # relative), a wrong pericentre-advance coefficient by O(1)
    assert abs(c / (-743.0 / 336.0) - 1) < 1e-5, c


def test_1pn_pericentre_advance_at_any_eccentricity():
    """The 1PN pericentre advance per radial period, 6 pi M / (a (1 - e^2)),
    i.e. (dgamma~/dt) / (2 pi nu) -> 3 x^{2/3} / (1 - e^2) as x -> 0, for
    circular and eccentric orbits (Richardson-extrapolated in x^{2/3})."""
    for e in (0.0, 0.3, 0.6, 0.8):
        p = W.injection(a=0.0, e0=e)
        M = p[0] * TSUN

        def ratio(nu):
            f = O.rhs(np.array([0.0, nu, 0.0, e, 0.0]), p)
            y = (2 * np.pi * M * nu) ** (2.0 / 3.0)
            return f[2] / (2 * np.pi * nu) / (3 * y / (1 - e * e))

        nu = 1e-8
        lim = 2 * ratio(nu) - ratio(nu * 2 ** 1.5)
        assert abs(lim - 1) < 1e-6, (e, lim)


def test_lense_thirring_precessions():
    """The spin terms of the precession equations are the Lense-Thirring
    rates of an orbit around a spinning mass (J = a M^2, Kepler's a_orb =
    (M / omega^2)^{1/3}, omega = 2 pi nu): the node of L about S advances at
    2 J / (a_orb^3 (1 - e^2)^{3/2}) (dalpha/dt), the pericentre at
    -6 J cos(lambda) / (a_orb^3 (1 - e^2)^{3/2}) (the spin part of
    dgamma~/dt, which is linear in the spin)."""
    for (a, e, cl, nu) in ((0.9, 0.0, 0.5, 1e-3), (0.5, 0.3, -0.2, 3e-4), (0.3, 0.7, 0.9, 2e-3)):
        p = W.injection(a=a, e0=e)
        p[8] = cl
        q = p.copy()
        q[2] = 0.0
        M = p[0] * TSUN
        om = 2 * np.pi * nu
        aorb3 = M / om ** 2
        J = a * M * M
        f = O.rhs(np.array([0.0, nu, 0.0, e, 0.0]), p)
        f0 = O.rhs(np.array([0.0, nu, 0.0, e, 0.0]), q)
        node = 2 * J / (aorb3 * (1 - e * e) ** 1.5)
        peri = -6 * J * cl / (aorb3 * (1 - e * e) ** 1.5)
        np.testing.assert_allclose(f[4], node, rtol=1e-13)
        np.testing.assert_allclose(f[2] - f0[2], peri, rtol=1e-10)
