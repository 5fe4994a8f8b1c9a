"""Pins of the oracle's Robson-Cornish-Liu noise model (the paper's second
noise model, Sec. 3 get_noise()).  Its constants are parity unpinned (no
printed values are at hand); these checks fix its shape: the power laws of
its acceleration- and shot-noise limits, the confusion noise's switch-off
above its knee, its sign, and the order of the confusion levels with the
observation time."""
import numpy as np

import oracle as O


def slope(f1, f2, conf=None):
    s1, s2 = O.psd_rcl(np.array([f1, f2]), conf)
    return np.log(s2 / s1) / np.log(f2 / f1)


def test_low_frequency_limit_is_f_minus_six():
    # acceleration noise (1 + (0.4 mHz / f)^2) / f^4 dominates well below 0.1 mHz
    assert abs(slope(1e-7, 2e-7) + 6.0) < 1e-3


def test_high_frequency_limit_is_f_squared():
    # shot noise times the transfer factor (1 + 0.6 (f/f*)^2); the acceleration
    # term, flat there at about 1 % of the shot noise, wobbles with cos^2(f/f*)
    for f1 in (2.0, 20.0, 200.0):
        assert abs(slope(f1, 2 * f1) - 2.0) < 0.03


def test_bucket_between_the_limits():
    f = np.logspace(-5, 0, 501)
    S = O.psd_rcl(f)
    i = int(np.argmin(S))
    assert 3e-3 < f[i] < 3e-2                  # the bucket sits near the transfer frequency
    assert np.all(np.diff(S[:i]) < 0) and np.all(np.diff(S[i + 5:]) > 0)


def test_confusion_noise_shape():
    f = np.logspace(-5, -0.5, 400)
    base = O.psd_rcl(f)
    for years in (0.5, 1.0, 2.0, 4.0):
        Sc = O.psd_rcl(f, years) - base
        assert np.all(Sc >= 0.0)
        hi = f > 0.05                           # tanh saturates: 1 + tanh(-gamma f) = 0
        assert np.all(Sc[hi] == 0.0)
        assert np.max(Sc / base) > 1.0          # it dominates somewhere near a mHz
    # more binaries are resolved in longer observations: the confusion noise
    # raises the curve less, integrated over log f across 0.1-10 mHz (at a
    # single frequency the fit's oscillating term can reorder neighbours)
    g = np.logspace(-4, -2, 2000)
    gb = O.psd_rcl(g)
    lv = [np.trapezoid(O.psd_rcl(g, y) / gb - 1.0, np.log(g)) for y in (0.5, 1.0, 2.0, 4.0)]
    assert lv[0] > lv[1] > lv[2] > lv[3] > 0.0


def test_zero_frequency_is_infinite():
    assert np.isinf(O.psd_rcl(np.array([0.0]))[0])
