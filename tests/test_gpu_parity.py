"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Tolerances (derived in the design notes):
  FP64 waveform  |dh| <= 64 n_max Phi_max eps64 max|h|: the only non-rounding
                 differences are the phase roundings (Phi ~ 1e3..1e6 rad,
                 multiplied by n up to n_max) and the coarse-table
                 interpolation of the Bessel amplitudes (~1e-14)
  FP64 spectrum  |dX| <= 1e-12 max|X|
  FP64 lnL       relative 1e-10 (the stated FP64 target)
  mixed lnL      relative 1e-4 (the stated mixed target)
"""
import numpy as np
import pytest

import oracle as O
from paper_2311_17174_amd import workloads as W
from tests.gpu_common import (EPS64, data_fingerprint, golden, max_phase, ocfg,
                               oracle_dataset, say, to_device_data)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def E():
    from paper_2311_17174_amd import emri
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return emri


def gpu_params(P):
    return torch.from_numpy(np.ascontiguousarray(P)).cuda()


def edge_walkers(w):
    """walkers around the injection plus modified gravity, a GW-speed delay,
    degenerate geometry and invalid rows"""
    P = list(W.walkers(w, B=6))
    p = w.inj.copy(); p[14], p[15] = 0.9, 2.0; P.append(p)                  # Xi(z)
    p = w.inj.copy(); p[16] = -2.4e-13; P.append(p)                         # delay ~1e4 s
    p = w.inj.copy(); p[3] = 0.0; P.append(p)                               # circular
    p = w.inj.copy(); p[8] = 1.0; P.append(p)                               # L || S
    p = w.inj.copy(); p[2] = 0.0; P.append(p)                               # no spin
    p = w.inj.copy(); p[1] = 2e6; P.append(p)                               # mu > M
    p = w.inj.copy(); p[4] = 1.0; P.append(p)                               # past the LSO
    p = w.inj.copy(); p[13] = np.nan; P.append(p)                           # NaN
    return np.array(P)


# ------------------------------------------------------------------ waveform
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_waveform_parity_small(E, prec):
    w = W.small(prec, n_harm=8)
    P = edge_walkers(w)
    say("waveform", w.name, P.shape)
    cfg = E.Config.from_workload(w)
    got = E.waveform_batch(gpu_params(P), cfg).cpu().numpy().astype(np.float64)
    torch.cuda.synchronize()
    ref = O.waveform(P, ocfg(w))                    # [B][2][N]
    got = got.transpose(0, 2, 1)
    scale = np.max(np.abs(ref))
    err = np.max(np.abs(got - ref), axis=(1, 2)) / scale
    say("max rel err per walker", err)
    if prec == "fp64":
        tol = 64 * w.n_harm * max_phase(w, P[:5]) * EPS64
    else:
        tol = 2e-5
    assert np.all(err <= tol), (err, tol)
    # invalid walkers: all zero; padding after N_valid: zero
    assert np.all(got[-3:] == 0.0)
    assert np.all(got[:, :, w.n_valid:] == 0.0)


def harmonic_contributions(w, P) -> np.ndarray:
    """max_t |h^(n)(t)| per harmonic n = 1..n_harm and walker: the oracle's
    waveform with n harmonics minus the one with n - 1"""
    prev = np.zeros((len(P), 2, w.N))
    out = []
    for n in range(1, w.n_harm + 1):
        cur = O.waveform(P, ocfg(w.with_(n_harm=n)))
        out.append(np.max(np.abs(cur - prev), axis=(1, 2)))
        prev = cur
    return np.array(out)                                  # [n_harm][B]


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_high_harmonics_at_high_eccentricity(E, prec):
    """cos/sin(n Phi') come from the three-term recurrence.  At e0 = 0.85
    harmonics 33..64 carry about a quarter of max|h| (the oracle's waveform
    with 32 harmonics differs by 0.28 max|h|), so the top harmonics' error
    shows in the waveform.  FP64: the phase-rounding tolerance of the other
    waveform tests.  FP32, per harmonic n in units u = 2^-24 of its largest
    contribution A_n: (3/2) n^2 from the recurrence (n^2/2 from its steps'
    roundings, n^2 from the rounding of cos Phi'), 20 n from the phase
    (reduced modulo 2 pi in FP64, rounded to FP32: pi u; then at most 7
    rotations of 2 u along a lane's samples), 70 for the amplitude cubic and
    the sum of up to 64 terms; and 64 u of max|h| for the response:
    |dh| <= u (sum_n (1.5 n^2 + 20 n + 70) A_n + 64 max|h|)."""
    w = W.small(prec, n_harm=64, e0=0.85, nu0=1.5e-4)
    P = W.walkers(w, B=2)
    say("high harmonics", prec, w.n_harm, P.shape)
    cfg = E.Config.from_workload(w)
    got = E.waveform_batch(gpu_params(P), cfg).cpu().numpy().astype(np.float64)
    torch.cuda.synchronize()
    got = got.transpose(0, 2, 1)
    ref = O.waveform(P, ocfg(w))
    scale = np.max(np.abs(ref))
    err = np.max(np.abs(got - ref), axis=(1, 2)) / scale
    say("max rel err per walker", err)
    if prec == "fp64":
        tol = 64 * w.n_harm * max_phase(w, P) * EPS64
    else:
        A = harmonic_contributions(w.with_(precision="fp64"), P)
        n = np.arange(1, w.n_harm + 1)[:, None]
        u = 2.0 ** -24
        tol = u * ((1.5 * n ** 2 + 20 * n + 70) * A).sum(axis=0) / scale + 64 * u
        say("bound per walker", tol)
    assert np.all(err <= tol), (err, tol)


@pytest.mark.parametrize("e0", [1e-4, 1e-7])
def test_nearly_circular_orbits(E, e0):
    """Bessel functions at X = n e down to 1e-7: Miller's recurrence grows by
    about 2q/X per step (by some 1e480 from order 70 to 0 at X = 6.4e-6), so
    at e0 = 1e-7 its running rescale (checked once per pair of steps) fires,
    and the high orders reach the FP64 underflow range (the oracle's
    J_67(67e-4) is 4e-261, smaller ones are 0).  FP64
    waveform against the oracle with 64 harmonics, the phase-rounding
    tolerance of the other waveform tests."""
    w = W.small("fp64", n_harm=64, e0=e0)
    P = W.walkers(w, B=2)
    say("nearly circular", e0, P[:, 3])
    got = E.waveform_batch(gpu_params(P), E.Config.from_workload(w)).cpu().numpy()
    torch.cuda.synchronize()
    got = got.transpose(0, 2, 1)
    ref = O.waveform(P, ocfg(w))
    err = np.max(np.abs(got - ref), axis=(1, 2)) / np.max(np.abs(ref))
    say("max rel err per walker", err)
    assert np.all(np.isfinite(got))
    assert np.all(err <= 64 * w.n_harm * max_phase(w, P) * EPS64), err


def plunge_workload(cl):
    w = W.small("fp64", n_harm=6, days=20.0, N=1 << 18, M=1e5, e0=0.5, a=0.9, nu0=6.3e-3)
    return w.with_(coarse_log2=cl)


def test_waveform_plunge_inside_window(E):
    """A fast inspiral (M = 1e5) that reaches the LSO mid-window: zeros after
    the last node, FP64 parity elsewhere (coarse step 2560 s)."""
    w = plunge_workload(8)
    P = W.walkers(w, B=3)
    orb, kw = O.orbit(P, ocfg(w))
    say("plunge nodes", kw, "of", w.n_intervals)
    assert np.all(kw < w.n_intervals - 8)
    cfg = E.Config.from_workload(w)
    got = E.waveform_batch(gpu_params(P), cfg).cpu().numpy().transpose(0, 2, 1)
    ref = O.waveform(P, ocfg(w))
    scale = np.max(np.abs(ref))
    tol = 64 * w.n_harm * max_phase(w, P) * EPS64
    say("plunge rel err", np.max(np.abs(got - ref)) / scale, "tol", tol)
    assert np.max(np.abs(got - ref)) <= tol * scale
    for b in range(3):
        assert np.all(got[b, :, kw[b] << w.coarse_log2:] == 0.0)
        assert np.any(got[b, :, (kw[b] << w.coarse_log2) - 1] != 0.0)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_loglike_plunge_inside_window(E, prec):
    """The likelihood path leaves the samples after each walker's plunge
    unwritten and unread (taken as zero): against the oracle on noise-less
    data, where lnL is the signal part alone, for walkers that plunge at
    different nodes and one that is invalid."""
    w = plunge_workload(8).with_(precision=prec)
    P = W.walkers(w, B=4)
    P[1, 4] *= 1.03                                    # plunges at node 426
    P[2, 4] *= 0.97                                    # at node 508 (walker 0: 465)
    P[3, 1] = 2e5                                      # mu > M: invalid, lnL = -inf
    d, S = oracle_dataset(w, noise=False)
    ref = O.loglike(P, d, S, ocfg(w))
    cfg = E.Config.from_workload(w)
    dd, ss = to_device_data(d, S)
    got = E.loglike_batch(gpu_params(P), dd, ss, cfg).cpu().numpy()
    hh = -2.0 * O.loglike(w.inj[None], np.zeros_like(d), S, ocfg(w))[0]
    say("plunge lnL ref", ref, "got", got, "<h|h>", hh)
    assert got[3] == -np.inf and ref[3] == -np.inf
    tol = 1e-10 if prec == "fp64" else 1e-5
    assert np.max(np.abs(got[:3] - ref[:3])) <= tol * hh


def test_amplitude_table_error_converges():
    """The HIP path interpolates the Peters-Mathews amplitudes (Bessel
    brackets times A) with cubic Hermite polynomials per coarse interval; the
    oracle evaluates them exactly per sample.  Near a fast plunge the
    difference is visible (~1e-7 at h = 10240 s) and falls as h^4."""
    from paper_2311_17174_amd import emri as E
    errs = []
    for cl in (10, 9, 8):
        w = plunge_workload(cl)
        P = W.walkers(w, B=1)
        got = E.waveform_batch(gpu_params(P), E.Config.from_workload(w)).cpu().numpy()
        ref = O.waveform(P, ocfg(w))
        errs.append(np.max(np.abs(got.transpose(0, 2, 1) - ref)) / np.max(np.abs(ref)))
    say("table interpolation error vs coarse step", errs)
    assert errs[0] < 1e-6
    assert errs[0] / errs[1] > 10.0 and errs[1] / errs[2] > 6.0


# ----------------------------------------------------------------------- FFT
def _waveform_and_lnl(E, w, P):
    cfg = E.Config.from_workload(w)
    got = E.waveform_batch(gpu_params(P), cfg).cpu().numpy().astype(np.float64).transpose(0, 2, 1)
    ref = O.waveform(P, ocfg(w))
    werr = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    d, S = oracle_dataset(w, True)
    dd, ss = to_device_data(d, S)
    lnl = E.loglike_batch(gpu_params(P), dd, ss, cfg).cpu().numpy()
    lref = O.loglike(P, d, S, ocfg(w))
    lerr = np.max(np.abs(lnl - lref) / np.abs(lref))
    return werr, lerr


# the edges of the accepted configurations: every samples-per-lane variant of
# the synthesis (coarse step 2^cl samples), the largest harmonic count, the
# smallest transform (rows of 128 points, columns of 32); and the amplitude
# tables' blocking (ranges of 63 intervals, groups of 16 harmonics): 84
# intervals with 17 harmonics (a full and a ragged range, a one-harmonic
# group) and a single harmonic
EDGE_CASES = [("cl9", dict(coarse_log2=9), {}), ("cl11", dict(coarse_log2=11), {}),
              ("cl12", dict(coarse_log2=12), {}), ("nh64", {}, dict(n_harm=64)),
              ("N4096", {}, dict(days=0.4, N=1 << 12)),
              ("cl8_nh17", dict(coarse_log2=8), dict(n_harm=17)), ("nh1", {}, dict(n_harm=1))]


@pytest.mark.parametrize("case", EDGE_CASES, ids=[c[0] for c in EDGE_CASES])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_configuration_edges(E, prec, case):
    name, over, kw = case
    w = W.small(prec, **{"n_harm": 8, **kw}).with_(**over)
    P = W.walkers(w, B=6)
    say("edge case", name, prec, w.coarse_log2, w.n_harm, w.N)
    werr, lerr = _waveform_and_lnl(E, w, P)
    say("waveform rel err", werr, "lnL rel err", lerr)
    if prec == "fp64":
        assert werr <= 64 * w.n_harm * max_phase(w, P) * EPS64
        assert lerr <= 1e-10
    else:
        assert werr <= 2e-5
        assert lerr <= 1e-4


@pytest.mark.parametrize("logN", [12, 13, 15, 18, 20, 21, 22, 23, 24])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_fft_parity(E, logN, prec):
    """emri_fft_batch against the oracle's radix-2 FFT element by element,
    at every transform length the likelihood uses up to 2^24 (rows of 4096
    points and columns of 4096 points at 2^24)"""
    N = 1 << logN
    dt = 10.0
    B = 3 if logN <= 20 else 2
    w = W.Workload("fft", B, (N - 5) * dt, dt, N, 1, 10, prec)
    cfg = E.Config.from_workload(w)
    x = np.random.Generator(np.random.PCG64(logN)).standard_normal((B, N, 2))
    x[:, N - 5:] = 0.0
    dtype = torch.float64 if prec == "fp64" else torch.float32
    say("fft", logN, prec)
    xt = torch.from_numpy(x).to(dtype).cuda().contiguous()
    got = E.fft_batch(xt, cfg).cpu().numpy().astype(np.complex128)
    ref = O.rfft(xt.cpu().double().numpy().transpose(0, 2, 1), dt)   # [3][2][N/2+1]
    err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    say("rel err", err)
    assert err <= (1e-12 if prec == "fp64" else 2e-6)


# ---------------------------------------------------------------- likelihood
@pytest.mark.parametrize("noise", [True, False])
def test_loglike_parity_fp64_small(E, noise):
    w = W.small("fp64", n_harm=8)
    P = edge_walkers(w)
    d, S = oracle_dataset(w, noise)
    ref = O.loglike(P, d, S, ocfg(w))
    cfg = E.Config.from_workload(w)
    dd, ss = to_device_data(d, S)
    got = E.loglike_batch(gpu_params(P), dd, ss, cfg).cpu().numpy()
    say("lnL ref", ref)
    say("lnL got", got)
    fin = np.isfinite(ref)
    assert np.array_equal(fin, np.isfinite(got))
    assert np.all(got[~fin] == -np.inf)
    if noise:
        np.testing.assert_allclose(got[fin], ref[fin], rtol=1e-10, atol=0)
    else:
        # noise-less data: lnL(injection) = 0; scale by the optimal SNR^2
        zero = np.zeros_like(d)
        hh = -2.0 * O.loglike(w.inj[None], zero, S, ocfg(w))[0]
        assert np.max(np.abs(got[fin] - ref[fin])) <= 1e-10 * hh
        assert abs(got[0]) <= 1e-10 * hh


def test_loglike_parity_mixed_small(E):
    w = W.small("mixed", n_harm=8)
    P = edge_walkers(w)
    d, S = oracle_dataset(w, True)
    ref = O.loglike(P, d, S, ocfg(w))
    cfg = E.Config.from_workload(w)
    dd, ss = to_device_data(d, S)
    got = E.loglike_batch(gpu_params(P), dd, ss, cfg).cpu().numpy()
    fin = np.isfinite(ref)
    assert np.array_equal(fin, np.isfinite(got))
    rel = np.abs(got[fin] - ref[fin]) / np.abs(ref[fin])
    say("mixed rel err", rel)
    assert np.all(rel <= 1e-4)


def test_batch_invariance_and_chunking(E):
    """Per-walker results do not depend on the batch: permuted, split and
    chunked evaluations are bitwise equal."""
    w = W.small("fp64", n_harm=6)
    P = W.walkers(w, B=12)
    d, S = oracle_dataset(w, True)
    cfg = E.Config.from_workload(w)
    dd, ss = to_device_data(d, S)
    full = E.loglike_batch(gpu_params(P), dd, ss, cfg).cpu().numpy()
    perm = np.random.Generator(np.random.PCG64(9)).permutation(12)
    permuted = E.loglike_batch(gpu_params(P[perm]), dd, ss, cfg).cpu().numpy()
    assert np.array_equal(permuted, full[perm])
    part = E.loglike_batch(gpu_params(P[3:5]), dd, ss, cfg).cpu().numpy()
    assert np.array_equal(part, full[3:5])
    # workspace for 5 walkers + the data set: 3 chunks
    n = E.dataset_bytes(cfg) + 256 + E.workspace_bytes(cfg, 5)
    ws = torch.empty(n, dtype=torch.uint8, device="cuda")
    chunked = E.loglike_batch(gpu_params(P), dd, ss, cfg, ws=ws).cpu().numpy()
    assert np.array_equal(chunked, full)
    # resident data set
    ds = E.dataset_init(dd, ss, cfg)
    res = E.loglike_dataset(gpu_params(P), ds, cfg).cpu().numpy()
    assert np.array_equal(res, full)
    # repeated calls are deterministic
    again = E.loglike_batch(gpu_params(P), dd, ss, cfg).cpu().numpy()
    assert np.array_equal(again, full)


@pytest.mark.parametrize("segs", [2, 5, 16])
def test_orbit_segments_bitwise(E, segs):
    """The orbit integrated in segments, with the tables and samples of each
    finished segment built on a second stream, gives the same bits as one
    segment: edge walkers, and fast inspirals that reach the LSO inside a
    middle segment."""
    w = plunge_workload(8)
    P = np.concatenate([W.walkers(w, B=3), edge_walkers(w)])
    _, kw = O.orbit(P[:3], ocfg(w))
    say("segments", segs, "plunge nodes", kw, "of", w.n_intervals)
    cfg = E.Config.from_workload(w)
    E.set_tuning(orbit_segments=1)
    ref = E.waveform_batch(gpu_params(P), cfg).cpu().numpy()
    E.set_tuning(orbit_segments=segs)
    got = E.waveform_batch(gpu_params(P), cfg).cpu().numpy()
    assert np.array_equal(got, ref)
    # likelihood through the same pipeline, twice (events and streams reused)
    ws = W.small("fp64", n_harm=6)
    Q = edge_walkers(ws)
    d, S = oracle_dataset(ws, True)
    dd, ss = to_device_data(d, S)
    cs = E.Config.from_workload(ws)
    E.set_tuning(orbit_segments=1)
    one = E.loglike_batch(gpu_params(Q), dd, ss, cs).cpu().numpy()
    E.set_tuning(orbit_segments=segs)
    for _ in range(2):
        assert np.array_equal(E.loglike_batch(gpu_params(Q), dd, ss, cs).cpu().numpy(), one)


# ---------------------------------------------------------- full-size cases
def test_config1_full_parity(E):
    """Config 1 (FP64, B=32, 30 days, 2^18 samples, 16 harmonics): every walker."""
    w = W.config1()
    P = W.walkers(w)
    say("config1 oracle data")
    d, S = oracle_dataset(w, True)
    cfg = E.Config.from_workload(w)
    dd, ss = to_device_data(d, S)
    got = E.loglike_batch(gpu_params(P), dd, ss, cfg).cpu().numpy()
    say("config1 oracle lnL")
    ref = O.loglike(P, d, S, ocfg(w))
    rel = np.abs(got - ref) / np.abs(ref)
    say("config1 max rel", rel.max())
    assert np.all(rel <= 1e-10)


# Tolerances of the full-size comparisons (Eq. (8) with the inner product of
# Eq. (7)).  |lnL| ~ N is dominated by the noise term <d|d>/2, which both
# sides form from the same data, so a relative bound on lnL cannot see an
# error of the model; the signal part is bounded against <m|m> of the walker:
# |lnL_gpu - lnL_oracle| <= SIGNAL_TOL * <m|m>.  FP64 differs from the oracle
# only by rounding and the amplitude tables (section on tolerances of the
# design notes); the mixed path carries FP32 rounding of a waveform whose
# relative error is ~1e-6.
LNL_REL_TOL = {"fp64": 1e-10, "mixed": 1e-4}
SIGNAL_TOL = {"fp64": 1e-10, "mixed": 1e-5}


def _golden_checks(E, w, P, g, idx, prec, ws=None):
    """lnL of walkers P on the noisy, noise-less and zero data sets of w,
    against the oracle's golden values of walkers idx; returns the worst
    ratios for the report"""
    d, S = oracle_dataset(w, True)
    assert data_fingerprint(d) == g["data_sha256"], \
        "golden values do not match the oracle's data: rerun tests/golden/make_golden.py"
    clean, _ = oracle_dataset(w, False)
    sets = {"noisy": d, "noiseless": clean, "zero": np.zeros_like(clean)}
    cfg = E.Config.from_workload(w)
    mm = np.asarray(g["mm"])
    assert np.all(mm > 0)
    worst = {}
    for name, data in sets.items():
        dd, ss = to_device_data(data, S)
        kw = {} if ws is None else {"ws": ws}
        got = E.loglike_batch(gpu_params(P), dd, ss, cfg, **kw).cpu().numpy()[idx]
        ref = {"noisy": np.asarray(g["lnl_noisy"]), "noiseless": np.asarray(g["lnl_noiseless"]),
               "zero": -0.5 * mm}[name]
        assert np.all(np.isfinite(got)) and np.all(np.isfinite(ref))
        sig = np.abs(got - ref) / mm
        worst[name] = float(sig.max())
        say(prec, name, "max |dlnL|", np.abs(got - ref).max(), "max |dlnL|/<m|m>", sig.max(),
            "at walker", idx[int(np.argmax(sig))])
        assert np.all(sig <= SIGNAL_TOL[prec]), (name, sig.max())
        if name == "noisy":
            rel = np.abs(got - ref) / np.abs(ref)
            say(prec, "noisy max rel", rel.max())
            assert np.all(rel <= LNL_REL_TOL[prec])
    return worst


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_config2_every_walker_against_the_oracle(E, prec):
    """Config 2 / 3 (B=256, 1 yr, 2^22 samples, 30 harmonics) in the launch
    configuration of the benchmark: every walker against the oracle's values
    (tests/golden/cfg2_fp64_B256_1yr_2p22_lnl.json, written by the oracle
    alone), on noisy, noise-less and zero data (the last is -<m|m>/2)."""
    w = W.config2() if prec == "fp64" else W.config3()
    g = golden("cfg2_fp64_B256_1yr_2p22")
    P = W.walkers(w)
    idx = np.asarray(g["idx"])
    assert len(idx) == w.B == 256
    say("config2 against golden", prec)
    _golden_checks(E, w, P, g, idx, prec)


# ------------------------------------------------------- model and noise PSD
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_model_batch_parity(E, prec):
    """Propagated frequency-domain model exp(-2 pi i f DT) h~ / (Xi d_L)."""
    w = W.small(prec, n_harm=8)
    P = edge_walkers(w)
    cfg = E.Config.from_workload(w)
    got = E.model_batch(gpu_params(P), cfg).cpu().numpy().astype(np.complex128)
    S = O.psd_bc04(W.frequencies(w.N, w.dt))
    valid = O.scalars(P)[:, 0] == 1.0
    spec = O.spectrum(P, ocfg(w))
    scale = 0.0
    errs = []
    for b in range(len(P)):
        if not valid[b]:
            assert np.all(got[b] == 0)
            continue
        ref = O.make_data(spec[b], P[b], S, None, w.N, w.dt)
        scale = max(scale, np.max(np.abs(ref)))
        errs.append(np.max(np.abs(got[b] - ref)))
    rel = np.max(errs) / scale
    say("model rel err", rel)
    assert rel <= (1e-10 if prec == "fp64" else 2e-5)


def test_noise_psd_parity(E):
    N, dt = 1 << 16, 10.0
    got = E.noise_psd(N, dt).cpu().numpy()
    ref = O.psd_bc04(W.frequencies(N, dt))
    assert np.isinf(got[0]) and np.isinf(ref[0])
    np.testing.assert_allclose(got[1:], ref[1:], rtol=4e-15)   # a few ulps


@pytest.mark.parametrize("model,years", [(1, None), (2, 0.5), (3, 1.0), (4, 2.0), (5, 4.0)])
def test_noise_psd_rcl_parity(E, model, years):
    """Robson-Cornish-Liu sensitivity, with and without confusion noise, at
    dt = 5 s (up to 0.1 Hz): pow/exp/tanh/cos of two libraries, relative 1e-13."""
    N, dt = 1 << 20, 5.0
    got = E.noise_psd(N, dt, model=model).cpu().numpy()
    ref = O.psd_rcl(W.frequencies(N, dt), years)
    assert np.isinf(got[0])
    np.testing.assert_allclose(got[1:], ref[1:], rtol=1e-13)
    with pytest.raises(E.EmriError):
        E.noise_psd(N, dt, model=6)


def test_config5_stress_chunked(E):
    """Config 5 (B=1024, 2 yr at dt = 5 s, 2^24 samples, 40 harmonics; the
    injection plunges at ~0.6 yr) through workspaces that hold a quarter and a
    half of the batch: FP64 and mixed on the same inputs for every walker, and
    64 seeded walkers against the oracle's values
    (tests/golden/cfg5_fp64_B1024_2yr_2p24_lnl.json) on noisy, noise-less and
    zero data."""
    w64, wmx = W.config5("fp64"), W.config5("mixed")
    g = golden("cfg5_fp64_B1024_2yr_2p24")
    idx = np.asarray(g["idx"])
    assert len(idx) == 64 and idx[0] == 0
    P = W.walkers(w64)
    say("config5 oracle data")
    d, S = oracle_dataset(w64, True)
    dd, ss = to_device_data(d, S)
    out = {}
    for w, part in ((w64, 256), (wmx, 512)):
        cfg = E.Config.from_workload(w)
        ws = torch.empty(E.dataset_bytes(cfg) + 256 + E.workspace_bytes(cfg, part),
                         dtype=torch.uint8, device="cuda")
        out[w.precision] = E.loglike_batch(gpu_params(P), dd, ss, cfg, ws=ws).cpu().numpy()
        if w is w64:
            _golden_checks(E, w, P, g, idx, "fp64", ws=ws)
        else:
            _golden_checks(E, w, P, g, idx, "mixed", ws=ws)
        del ws
        torch.cuda.empty_cache()
    a, b = out["fp64"], out["mixed"]
    assert np.all(np.isfinite(a)) and np.all(np.isfinite(b))
    rel = np.abs(a - b) / np.abs(a)
    say("config5 mixed vs fp64: max rel", rel.max(), "max abs", np.abs(a - b).max())
    assert rel.max() <= 1e-4


def test_gr_limit_of_the_propagation(E):
    """The modified-gravity factors reduce to GR on the HIP path: Xi0 = 1
    (any n) and n = 0 (any Xi0) give Xi = 1 up to one rounding of
    Xi0 + (1 - Xi0), alpha_T = 0 gives no delay; against the GR row."""
    w = W.small("fp64", n_harm=6)
    base = w.inj.copy()
    rows = [base.copy() for _ in range(4)]
    rows[1][14], rows[1][15] = 1.0, 3.0          # Xi0 = 1, n = 3
    rows[2][14], rows[2][15] = 0.7, 0.0          # n = 0
    rows[3][16] = 0.0                            # explicit GR speed
    P = np.array(rows)
    d, S = oracle_dataset(w, True)
    cfg = E.Config.from_workload(w)
    dd, ss = to_device_data(d, S)
    got = E.loglike_batch(gpu_params(P), dd, ss, cfg).cpu().numpy()
    say("GR-limit lnL", got)
    assert got[1] == got[0] and got[3] == got[0]
    assert abs(got[2] - got[0]) <= 1e-14 * abs(got[0])


@pytest.mark.parametrize("ode", [0, 1])
def test_empty_batches(E, ode):
    """B = 0 on every batch entry point (both orbit integrators): empty
    results, nothing launched, no error."""
    w = W.small("fp64", n_harm=4).with_(ode=ode, ode_rtol=1e-10, ode_atol=1e-10)
    cfg = E.Config.from_workload(w)
    P = torch.zeros((0, 17), dtype=torch.float64, device="cuda")
    assert E.waveform_batch(P, cfg).shape[0] == 0
    x = torch.zeros((0, w.N, 2), dtype=torch.float64, device="cuda")
    assert E.fft_batch(x, cfg).shape[0] == 0
    assert E.model_batch(P, cfg).shape[0] == 0
    d, S = oracle_dataset(w, True)
    dd, ss = to_device_data(d, S)
    assert E.loglike_batch(P, dd, ss, cfg).shape[0] == 0
    ds = E.dataset_init(dd, ss, cfg)
    assert E.loglike_dataset(P, ds, cfg).shape[0] == 0
    # and a batch of one right after
    one = E.loglike_dataset(gpu_params(w.inj[None]), ds, cfg).cpu().numpy()
    assert np.isfinite(one[0])
