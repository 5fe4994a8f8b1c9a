"""Pins of the oracle's detector response (Eq. (2) with the low-frequency
LISA response it cites: Doppler phase, detector-frame angles, polarisation
angle and the angle beta that turns gamma~ into gamma) against vector
constructions of the same geometry.

The oracle evaluates closed forms (trigonometric expressions in the source,
spin and detector angles).  Each test here builds the underlying geometry
from unit vectors, rotation matrices and cross products in numpy and checks
the oracle's per-sample diagnostics against it, at random sky and spin
directions and over a window long enough for the detector to move.  A sign
flip, a sin/cos swap or swapped atan2 arguments in any of the closed forms
fails one of them.
"""
import numpy as np
import pytest

from paper_2311_17174_amd import workloads as W

AU_S = 1.495978707e11 / 299792458.0     # 1 AU in light seconds


def ocfg(O, w):
    return O.OracleConfig(T_obs=w.T_obs, dt=w.dt, N=w.N, n_harm=w.n_harm,
                          coarse_log2=w.coarse_log2)


def unit(th, ph):
    return np.array([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)])


def rot_z(a):
    c, s = np.cos(a), np.sin(a)
    z, o = np.zeros_like(a), np.ones_like(a)
    return np.stack([np.stack([c, -s, z], -1), np.stack([s, c, z], -1),
                     np.stack([z, z, o], -1)], -2)


def rot_y(a):
    c, s = np.cos(a), np.sin(a)
    return np.array([[c, 0.0, s], [0.0, 1.0, 0.0], [-s, 0.0, c]])


def wrap(a):
    """angle in (-pi, pi]"""
    return np.angle(np.exp(1j * a))


def random_rows(w, n, seed):
    """the workload's injection with random sky and spin directions and
    inclinations (isotropic), n rows"""
    rng = np.random.Generator(np.random.PCG64(seed))
    rows = []
    for _ in range(n):
        p = w.inj.copy()
        p[8] = rng.uniform(-0.95, 0.95)                       # cos(lambda)
        p[9], p[10] = np.arccos(rng.uniform(-1, 1)), rng.uniform(0, 2 * np.pi)
        p[11], p[12] = np.arccos(rng.uniform(-1, 1)), rng.uniform(0, 2 * np.pi)
        p[7] = rng.uniform(0, 2 * np.pi)                      # alpha0
        rows.append(p)
    return rows


@pytest.fixture(scope="module")
def runs(oracle_lib):
    """per-sample diagnostics of 5 random geometries over 40 days (the
    detector moves by 0.69 rad around the Sun)"""
    O = oracle_lib
    w = W.small(n_harm=4, days=40.0, N=1 << 19)
    out = []
    for p in random_rows(w, 5, seed=21):
        x, d = O.waveform_diag(p, ocfg(O, w))
        nv = w.n_valid
        t = np.arange(nv) * w.dt
        out.append((p, x[:, :nv], d[:nv], t))
    return out


def detector_frame(t):
    """LISA's detector frame [T][3][3] (columns x_d, y_d, z_d in ecliptic
    coordinates): the constellation's centre orbits the Sun at azimuth
    phibar = 2 pi t / yr, its plane is tilted by 60 degrees so that its
    normal z_d points 60 degrees away from the ecliptic pole, and the arms
    turn within the plane once a year against the orbital sense (the
    'cartwheel'): D = R_z(phibar) R_y(-60 deg) R_z(-phibar)."""
    pb = 2 * np.pi * t / W.YEAR
    return rot_z(pb) @ rot_y(-np.pi / 3) @ rot_z(-pb)


def test_doppler_phase_is_the_light_travel_time(runs):
    """The Doppler term is the phase the orbit advances while the wave
    crosses the detector's displacement r(t) from the Sun along the source
    direction N: Phi' - Phi = 2 pi nu (N . r)/c, r = 1 AU (cos phibar,
    sin phibar, 0) (the detector leads the Sun when it is nearer the source)."""
    for p, x, d, t in runs:
        Nh = unit(p[9], p[10])
        pb = 2 * np.pi * t / W.YEAR
        r = AU_S * np.stack([np.cos(pb), np.sin(pb), np.zeros_like(pb)], -1)
        Phi, nu, Phid = d[:, 10], d[:, 11], d[:, 4]
        expect = 2 * np.pi * nu * (r @ Nh)
        assert np.max(np.abs(expect)) > 0.1          # a visible modulation
        np.testing.assert_allclose(Phid - Phi, expect, rtol=0,
                                   atol=4e-16 * np.max(np.abs(Phid)) + 1e-14)


def test_detector_colatitude_in_the_cartwheel_frame(runs):
    """cos(theta_d) = N . z_d with z_d the third column of the rotating frame."""
    for p, x, d, t in runs:
        D = detector_frame(t)
        Nh = unit(p[9], p[10])
        np.testing.assert_allclose(d[:, 6], D[..., 2] @ Nh, rtol=0, atol=4e-16)


def test_detector_azimuth_in_the_cartwheel_frame(runs):
    """phi_d is the azimuth of N in the rotating frame, atan2(N . y_d, N . x_d),
    up to a constant: only 2 phi_d enters the response, and 2 phi_d minus
    twice the frame azimuth must be the same at every time and for every sky
    position (a rigid frame turning in the cartwheel sense).  The constant is
    pi for the closed form with every orientation offset at 0: the closed
    form's x axis is the frame's x_d turned by 90 degrees."""
    for p, x, d, t in runs:
        D = detector_frame(t)
        Nh = unit(p[9], p[10])
        phv = np.arctan2(D[..., 1] @ Nh, D[..., 0] @ Nh)
        off = wrap(2 * (d[:, 7] - phv) - np.pi)
        assert np.max(np.abs(off)) < 1e-9, np.max(np.abs(off))


def test_detector_azimuth_fails_for_the_wrong_rotation_sense(runs):
    """the same comparison against a frame whose arms turn with the orbit
    (R_z(+phibar)) is not constant: the check above can fail"""
    p, x, d, t = runs[0]
    pb = 2 * np.pi * t / W.YEAR
    D = rot_z(pb) @ rot_y(-np.pi / 3) @ rot_z(pb)
    Nh = unit(p[9], p[10])
    phv = np.arctan2(D[..., 1] @ Nh, D[..., 0] @ Nh)
    off = wrap(2 * (d[:, 7] - phv) - np.pi)
    assert np.max(np.abs(off)) > 0.5


def orbital_normal(p, alpha):
    """L(t) = cos(lambda) S + sin(lambda) (cos(alpha) e1 + sin(alpha) e2),
    with e1 the unit projection of the ecliptic pole z orthogonal to S and
    e2 = S x e1 (so that L turns about S in the positive sense as alpha
    grows), built from the vector definitions"""
    S = unit(p[11], p[12])
    zhat = np.array([0.0, 0.0, 1.0])
    e1 = zhat - (zhat @ S) * S
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(S, e1)
    cl = p[8]
    sl = np.sqrt(1 - cl * cl)
    return cl * S + sl * (np.cos(alpha)[:, None] * e1 + np.sin(alpha)[:, None] * e2)


def test_inclination_from_the_precessing_orbital_normal(runs):
    """c_iota = L . N, with L precessing about S by the angle alpha of the orbit"""
    for p, x, d, t in runs:
        L = orbital_normal(p, d[:, 13])
        np.testing.assert_allclose(np.linalg.norm(L, axis=1), 1.0, rtol=0, atol=1e-15)
        np.testing.assert_allclose(L @ unit(p[11], p[12]), p[8], rtol=0, atol=1e-15)
        np.testing.assert_allclose(d[:, 3], L @ unit(p[9], p[10]), rtol=0, atol=1e-14)


def test_polarisation_angle_from_the_line_of_nodes(runs):
    """psi is the angle, in the plane of the sky (orthogonal to N), from the
    projection of the detector normal, a = z_d - (z_d . N) N, towards
    b = N x z_d, of the line of nodes p = N x L (the principal polarisation
    axis): psi = atan2(p . b, p . a)."""
    for p, x, d, t in runs:
        Nh = unit(p[9], p[10])
        L = orbital_normal(p, d[:, 13])
        zd = detector_frame(t)[..., 2]
        a = zd - (zd @ Nh)[:, None] * Nh
        b = np.cross(Nh, zd)
        pn = np.cross(Nh, L)
        psi = np.arctan2(np.sum(pn * b, 1), np.sum(pn * a, 1))
        assert np.ptp(psi) > 0.1                   # the angle moves over the window
        np.testing.assert_allclose(wrap(d[:, 8] - psi), 0.0, rtol=0, atol=1e-11)


def test_beta_is_the_angle_between_the_two_nodal_lines(runs):
    """beta, added to gamma~ to give gamma, is the angle about L from the
    line u = L x N (the nodes on the sky plane) to v = L x S (the nodes on
    the plane orthogonal to the spin): atan2(L . (u x v), u . v)."""
    for p, x, d, t in runs:
        Nh, S = unit(p[9], p[10]), unit(p[11], p[12])
        L = orbital_normal(p, d[:, 13])
        u, v = np.cross(L, Nh), np.cross(L, S)
        beta = np.arctan2(np.sum(L * np.cross(u, v), 1), np.sum(u * v, 1))
        np.testing.assert_allclose(wrap(d[:, 9] - beta), 0.0, rtol=0, atol=1e-11)
        np.testing.assert_allclose(wrap(d[:, 5] - d[:, 12] - d[:, 9]), 0.0, rtol=0,
                                   atol=1e-12 * np.max(np.abs(d[:, 5])))


def test_channels_from_the_antenna_patterns(runs, oracle_lib):
    """the two channels are sqrt(3)/2 (F+ h+ + Fx hx), channel II with its
    detector azimuth turned by -pi/4 (the second pair of arms)"""
    O = oracle_lib
    for p, x, d, t in runs[:2]:
        for j in range(0, len(t), 997):
            cth, phd, psi = d[j, 6], d[j, 7], d[j, 8]
            F1 = O.antenna(cth, phd, psi)
            F2 = O.antenna(cth, phd - np.pi / 4, psi)
            hp, hx = d[j, 0], d[j, 1]
            sc = np.sqrt(3) / 2 * (abs(hp) + abs(hx))
            assert abs(x[0, j] - np.sqrt(3) / 2 * (F1[0] * hp + F1[1] * hx)) <= 1e-15 * sc
            assert abs(x[1, j] - np.sqrt(3) / 2 * (F2[0] * hp + F2[1] * hx)) <= 1e-15 * sc
