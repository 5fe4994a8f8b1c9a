"""GPU parity of the seventh-order orbit integrator (emri_cfg.ode =
EMRI_ODE_RK78: Fehlberg's 7(8) pair, the order-7 solution kept, stepped node
to node) through the C ABI, against the CPU oracle.  The two sides run the
same steps, so they differ by rounding alone: the orbit nodes themselves
(emri_orbit_batch) to 1e-12 of each component's scale, also where the step
control splits intervals; the waveform and lnL with the RK4 path's
tolerances.  Intervals are split only where the amplitude tables' cubic
Hermite interpolation between nodes is no longer exact to rounding (coarse
steps of 2^12 samples near the plunge), so split intervals are checked on
the orbit, and the waveform where one step spans each interval."""
import numpy as np
import pytest

import oracle as O
from paper_2311_17174_amd import workloads as W
from tests.gpu_common import EPS64, max_phase, ocfg, oracle_dataset, say, to_device_data

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def E():
    from paper_2311_17174_amd import emri
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return emri


def rk78(w, rtol=1e-12):
    return w.with_(ode=2, ode_rtol=rtol, ode_atol=rtol)


def gpu(P):
    return torch.from_numpy(np.ascontiguousarray(P)).cuda()


def fast_inspiral(prec, coarse_log2=8):
    """M = 1e5: reaches the LSO mid-window (coarse step 2560 s, 675 nodes).
    With coarse_log2 = 12 (40960 s, 43 nodes) tight tolerances split the
    intervals near the plunge, with rejected steps."""
    w = W.small(prec, n_harm=6, days=20.0, N=1 << 18, M=1e5, e0=0.5, a=0.9, nu0=6.3e-3)
    return w.with_(coarse_log2=coarse_log2)


def edge_rows(w):
    P = list(W.walkers(w, B=3))
    p = w.inj.copy(); p[3] = 0.0; P.append(p)              # circular: e stays 0
    p = w.inj.copy(); p[1] = 2e6; P.append(p)              # mu > M: invalid
    p = w.inj.copy(); p[4] = 1.0; P.append(p)              # starts past the LSO
    return np.array(P)


def _orbit_close(got, ref, kw):
    """Node by node: the state and derivative to a few ulps of each
    component's scale over the orbit (Phi, gamma~, alpha grow linearly)."""
    for b in range(len(kw)):
        n = kw[b] + 1
        if n <= 0:
            assert np.all(got[b] == 0.0)
            continue
        assert np.all(got[b, n:] == 0.0)
        scale = np.max(np.abs(ref[b, :n]), axis=0) + 1e-300
        err = np.max(np.abs(got[b, :n] - ref[b, :n]), axis=0) / scale
        assert np.all(err < 1e-12), (b, err)


@pytest.mark.parametrize("ic", [0, 1])
@pytest.mark.parametrize("rtol", [1e-11, 1e-13])
def test_rk78_orbit_parity_with_split_intervals(E, ic, rtol):
    """The orbit stage alone (emri_orbit_batch) at 40960 s per coarse interval:
    near the plunge (forward) or the LSO (backward) the step control splits
    intervals and rejects steps; every node and K_w against the oracle."""
    w = rk78(fast_inspiral("fp64", 12).with_(ic=ic), rtol)
    P = edge_rows(w)
    if ic:
        P = np.concatenate([P[:4], [W.injection(M=2e4, mu=10.0, e0=0.7)]])
    ref, kw = O.orbit(P, ocfg(w))
    steps = O.orbit_steps(P, ocfg(w))
    say("RK78 orbit", ic, rtol, "K_w", kw, "of", w.n_intervals, "steps", steps.tolist())
    if ic == 0:
        assert np.all(kw[:3] < w.n_intervals - 8) and kw[3] == w.n_intervals
        assert kw[4] == kw[5] == -1
        assert np.all(steps[:3, 0] > kw[:3] + 1)           # split intervals
    else:
        assert list(kw[:4]) == [w.n_intervals] * 4 and kw[4] == -1
        assert np.any(steps[:4, 0] > w.n_intervals)          # split intervals
    assert np.any(steps[:, 1] > 0) or rtol == 1e-13
    orb, gkw = E.orbit_batch(gpu(P), E.Config.from_workload(w))
    assert np.array_equal(gkw.cpu().numpy(), kw)
    _orbit_close(orb.cpu().numpy(), ref, kw)


def test_all_integrators_orbit_parity(E):
    """RK4, DP5 and RK78 orbits through emri_orbit_batch against the oracle at
    config 1's coarse step, forward and backward."""
    base = W.config1().with_(n_harm=6)
    P = np.concatenate([W.walkers(base, B=6), edge_rows(base)[3:]])
    for ode in (0, 1, 2):
        for ic in (0, 1):
            w = base.with_(ode=ode, ode_rtol=1e-10, ode_atol=1e-10, ic=ic)
            ref, kw = O.orbit(P, ocfg(w))
            orb, gkw = E.orbit_batch(gpu(P), E.Config.from_workload(w))
            say("orbit ode", ode, "ic", ic, "K_w", kw)
            assert np.array_equal(gkw.cpu().numpy(), kw)
            _orbit_close(orb.cpu().numpy(), ref, kw)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("rtol", [1e-9, 1e-13])
def test_rk78_waveform_parity(E, prec, rtol):
    """The whole waveform at 2560 s per coarse interval, where the amplitude
    tables are exact to rounding: one step per interval, the walkers plunge
    mid-window."""
    w = rk78(fast_inspiral(prec), rtol)
    P = edge_rows(w)
    _, kw = O.orbit(P, ocfg(w))
    say("RK78", prec, rtol, "plunge nodes", kw, "of", w.n_intervals)
    assert np.all(kw[:3] < w.n_intervals - 8) and kw[3] == w.n_intervals
    assert kw[4] == kw[5] == -1
    got = E.waveform_batch(gpu(P), E.Config.from_workload(w)).cpu().numpy().astype(np.float64)
    got = got.transpose(0, 2, 1)
    ref = O.waveform(P, ocfg(w))
    scale = np.max(np.abs(ref))
    err = np.max(np.abs(got - ref), axis=(1, 2)) / scale
    say("max rel err per walker", err)
    tol = 64 * w.n_harm * max_phase(w, P[:4]) * EPS64 if prec == "fp64" else 2e-5
    assert np.all(err <= tol), (err, tol)
    assert np.all(got[4] == 0.0) and np.all(got[5] == 0.0)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_rk78_loglike_parity(E, prec):
    """30 days at 2^18 samples, one step per coarse interval."""
    w = rk78(W.config1().with_(n_harm=6, precision=prec), 1e-10)
    P = np.concatenate([W.walkers(w, B=6), edge_rows(w)[3:]])
    d, S = oracle_dataset(w, True)
    ref = O.loglike(P, d, S, ocfg(w))
    dd, ss = to_device_data(d, S)
    got = E.loglike_batch(gpu(P), dd, ss, E.Config.from_workload(w)).cpu().numpy()
    say("lnL ref", ref, "got", got)
    fin = np.isfinite(ref)
    assert list(np.where(~fin)[0]) == [7, 8]
    assert np.array_equal(fin, np.isfinite(got))
    rel = np.abs(got[fin] - ref[fin]) / np.abs(ref[fin])
    assert np.all(rel <= (1e-10 if prec == "fp64" else 1e-4)), rel


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_rk78_lso_convention(E, prec):
    """Backward from the LSO; an unphysical history is invalid."""
    w = rk78(W.small(prec, n_harm=6, days=20.0, N=1 << 18).with_(ic=1), 1e-10)
    P = list(W.walkers(w, B=4))
    P.append(W.injection(M=1e5, e0=0.8))
    P.append(W.injection(M=2e4, mu=10.0, e0=0.7))
    P = np.array(P)
    _, kw = O.orbit(P, ocfg(w))
    assert list(kw[:5]) == [w.n_intervals] * 5 and kw[5] == -1
    d, S = oracle_dataset(w, True)
    ref = O.loglike(P, d, S, ocfg(w))
    dd, ss = to_device_data(d, S)
    got = E.loglike_batch(gpu(P), dd, ss, E.Config.from_workload(w)).cpu().numpy()
    say("LSO lnL ref", ref, "got", got)
    assert got[5] == -np.inf and np.all(np.isfinite(got[:5]))
    rel = np.abs(got[:5] - ref[:5]) / np.abs(ref[:5])
    assert np.all(rel <= (1e-10 if prec == "fp64" else 1e-4)), rel


@pytest.mark.parametrize("segs", [3, 7])
def test_rk78_segments_bitwise(E, segs):
    """The step sequence does not depend on where orbit segments end: the
    waveform in segments equals the one-segment waveform bit for bit (with
    split intervals, rejected steps and a plunge)."""
    w = rk78(fast_inspiral("fp64", 12), 1e-11)
    P = edge_rows(w)
    cfg = E.Config.from_workload(w)
    E.set_tuning(orbit_segments=1)
    one = E.waveform_batch(gpu(P), cfg).cpu().numpy()
    E.set_tuning(orbit_segments=segs)
    for _ in range(2):
        assert np.array_equal(E.waveform_batch(gpu(P), cfg).cpu().numpy(), one)


def test_rk78_close_to_rk4_and_dp5(E):
    """The three integrators give likelihoods within far less than one unit
    of each other (accurate discretisations of Eq. (1))."""
    w = W.config1()
    P = W.walkers(w, B=16)
    d, S = oracle_dataset(w, True)
    dd, ss = to_device_data(d, S)
    a = E.loglike_batch(gpu(P), dd, ss, E.Config.from_workload(w)).cpu().numpy()
    b = E.loglike_batch(gpu(P), dd, ss, E.Config.from_workload(rk78(w))).cpu().numpy()
    c = E.loglike_batch(gpu(P), dd, ss,
                        E.Config.from_workload(w.with_(ode=1, ode_rtol=1e-12,
                                                       ode_atol=1e-12))).cpu().numpy()
    say("RK4 - RK78", np.max(np.abs(a - b)), "DP5 - RK78", np.max(np.abs(c - b)))
    assert np.max(np.abs(a - b)) < 1e-3 and np.max(np.abs(c - b)) < 1e-3


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_rk78_config2_sampled_parity(E, prec):
    """B=256, 1 yr, 2^22 samples, 30 harmonics in the benchmark's launch
    configuration (orbit segments on); the oracle checks sampled walkers."""
    base = W.config2() if prec == "fp64" else W.config3()
    w = rk78(base)
    P = W.walkers(w)
    d, S = oracle_dataset(rk78(W.config2()), True)
    dd, ss = to_device_data(d, S)
    got = E.loglike_batch(gpu(P), dd, ss, E.Config.from_workload(w)).cpu().numpy()
    assert np.all(np.isfinite(got))
    idx = np.array([5, 200])
    say("RK78 config2 oracle lnL for", idx)
    ref = O.loglike(P[idx], d, S, ocfg(w))
    rel = np.abs(got[idx] - ref) / np.abs(ref)
    say(prec, "rel err", rel)
    assert np.all(rel <= (1e-10 if prec == "fp64" else 1e-4))


def test_rk78_batch_invariance_chunking_and_paths(E):
    """Per-walker results do not depend on the batch (permuted, split,
    chunked through a small workspace) nor on the entry point (resident data
    set)."""
    w = rk78(W.small("fp64", n_harm=6, days=20.0, N=1 << 18), 1e-10)
    P = np.concatenate([W.walkers(w, B=11), edge_rows(w)[4:5]])       # last: invalid
    d, S = oracle_dataset(w, True)
    cfg = E.Config.from_workload(w)
    dd, ss = to_device_data(d, S)
    full = E.loglike_batch(gpu(P), dd, ss, cfg).cpu().numpy()
    assert full[-1] == -np.inf and np.all(np.isfinite(full[:-1]))
    perm = np.random.Generator(np.random.PCG64(4)).permutation(len(P))
    assert np.array_equal(E.loglike_batch(gpu(P[perm]), dd, ss, cfg).cpu().numpy(), full[perm])
    assert np.array_equal(E.loglike_batch(gpu(P[2:5]), dd, ss, cfg).cpu().numpy(), full[2:5])
    n = E.dataset_bytes(cfg) + 256 + E.workspace_bytes(cfg, 5)        # 3 chunks
    ws = torch.empty(n, dtype=torch.uint8, device="cuda")
    assert np.array_equal(E.loglike_batch(gpu(P), dd, ss, cfg, ws=ws).cpu().numpy(), full)
    ds = E.dataset_init(dd, ss, cfg)
    assert np.array_equal(E.loglike_dataset(gpu(P), ds, cfg).cpu().numpy(), full)
