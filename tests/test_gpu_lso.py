"""GPU parity of the LSO convention for initial conditions (Sec. 3
"Waveform computation": state at the last stable orbit, orbit integrated
backward) through the C ABI, against the CPU oracle.  Tolerances as for the
t = 0 convention."""
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


def lso_walkers(w):
    P = list(W.walkers(w, B=4))
    p = W.injection(M=1e5, e0=0.8); P.append(p)            # fast: e 0.81 -> 0.80 over the window
    p = w.inj.copy(); p[4] = -1.0; P.append(p)              # nu0 is unused at the LSO
    p = W.injection(M=2e4, mu=10.0, e0=0.7); P.append(p)    # backward history leaves the range
    return np.array(P)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_lso_waveform_parity(E, prec):
    w = W.small(prec, n_harm=6).with_(ic=1)
    P = lso_walkers(w)
    orb, kw = O.orbit(P, ocfg(w))
    say("LSO nodes", kw)
    assert list(kw[:6]) == [w.n_intervals] * 6 and kw[6] == -1
    cfg = E.Config.from_workload(w)
    got = E.waveform_batch(torch.from_numpy(P).cuda(), cfg).cpu().numpy().astype(np.float64)
    got = got.transpose(0, 2, 1)
    ref = O.waveform(P, ocfg(w))
    scale = np.max(np.abs(ref))
    err = np.max(np.abs(got - ref), axis=(1, 2)) / scale
    say("max rel err per walker", err)
    tol = 64 * w.n_harm * max_phase(w, P[:6]) * EPS64 if prec == "fp64" else 2e-5
    assert np.all(err <= tol), (err, tol)
    assert np.all(got[6] == 0.0)
    assert np.array_equal(got[5], got[0])                 # only the unused nu0 differs
    # the same row under the t = 0 convention is a different signal
    cfg0 = E.Config.from_workload(w.with_(ic=0))
    g0 = E.waveform_batch(torch.from_numpy(P[:1]).cuda(), cfg0).cpu().numpy()
    assert np.max(np.abs(g0[0].T - got[0])) > 0.1 * scale


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_lso_loglike_parity(E, prec):
    w = W.small(prec, n_harm=6).with_(ic=1)
    P = lso_walkers(w)
    d, S = oracle_dataset(w, True)
    ref = O.loglike(P, d, S, ocfg(w))
    cfg = E.Config.from_workload(w)
    dd, ss = to_device_data(d, S)
    got = E.loglike_batch(torch.from_numpy(P).cuda(), dd, ss, cfg).cpu().numpy()
    say("lnL ref", ref, "got", got)
    fin = np.isfinite(ref)
    assert list(np.where(~fin)[0]) == [6]
    assert np.array_equal(fin, np.isfinite(got)) and got[6] == -np.inf
    rel = np.abs(got[fin] - ref[fin]) / np.abs(ref[fin])
    assert np.all(rel <= (1e-10 if prec == "fp64" else 1e-4)), rel


@pytest.mark.parametrize("ode", [0, 1])
@pytest.mark.parametrize("segs", [3, 7])
def test_lso_segments_bitwise(E, ode, segs):
    """The backward orbit in segments (reverse time order, each segment's
    tables and samples built while the orbit goes on back in time) gives the
    likelihood and the model of one segment bit for bit, with a walker whose
    history leaves the physical range in a late segment (lnL = -inf, zero
    model)."""
    w = W.small("fp64", n_harm=6, days=20.0, N=1 << 18).with_(ic=1, ode=ode, ode_rtol=1e-10,
                                                              ode_atol=1e-10)
    # the last two histories leave the range about 14 and 119 nodes before
    # the LSO: in the first segments and in a late one
    P = np.concatenate([W.walkers(w, B=4), lso_walkers(w)[4:],
                        W.injection(M=5e4, mu=10.0, e0=0.6)[None]])
    _, kw = O.orbit(P, ocfg(w))
    say("LSO segments", segs, "ode", ode, "K", w.n_intervals, "kw", kw)
    assert np.all(kw[-2:] == -1) and np.all(kw[:-2] == w.n_intervals)
    d, S = oracle_dataset(w, True)
    dd, ss = to_device_data(d, S)
    cfg = E.Config.from_workload(w)
    ds = E.dataset_init(dd, ss, cfg)
    Pt = torch.from_numpy(P).cuda()
    E.set_tuning(orbit_segments=1)
    one = E.loglike_dataset(Pt, ds, cfg).cpu().numpy()
    m1 = E.model_batch(Pt, cfg).cpu().numpy()
    E.set_tuning(orbit_segments=segs)
    for _ in range(2):
        assert np.array_equal(E.loglike_dataset(Pt, ds, cfg).cpu().numpy(), one)
    assert np.array_equal(E.loglike_batch(Pt, dd, ss, cfg).cpu().numpy(), one)
    assert np.array_equal(E.model_batch(Pt, cfg).cpu().numpy(), m1)
    assert np.all(one[-2:] == -np.inf) and np.all(m1[-2:] == 0)
    ref = O.loglike(P, d, S, ocfg(w))
    fin = np.isfinite(ref)
    assert np.array_equal(fin, np.isfinite(one))
    assert np.all(np.abs(one[fin] - ref[fin]) <= 1e-10 * np.abs(ref[fin]))


@pytest.mark.parametrize("ode", [0, 1])
def test_lso_empty_first_segments(E, ode):
    """16 segments of a 22-interval orbit: the first backward segments are
    empty (node K alone); the likelihood equals the one-segment one."""
    w = W.small("fp64", n_harm=6).with_(ic=1, ode=ode, ode_rtol=1e-10, ode_atol=1e-10)
    P = lso_walkers(w)
    d, S = oracle_dataset(w, True)
    dd, ss = to_device_data(d, S)
    cfg = E.Config.from_workload(w)
    ds = E.dataset_init(dd, ss, cfg)
    Pt = torch.from_numpy(P).cuda()
    E.set_tuning(orbit_segments=1)
    one = E.loglike_dataset(Pt, ds, cfg).cpu().numpy()
    E.set_tuning(orbit_segments=16)
    assert np.array_equal(E.loglike_dataset(Pt, ds, cfg).cpu().numpy(), one)
    assert one[6] == -np.inf and np.all(np.isfinite(one[:6]))


def test_lso_config2_sampled_parity(E):
    """The paper's convention at full size (256 walkers, 1 yr, 2^22 samples,
    30 harmonics; the backward orbit in eight pipelined segments), against
    the oracle on sampled walkers."""
    w = W.config2().with_(ic=1)
    P = W.walkers(w)
    d, S = oracle_dataset(w, True)
    dd, ss = to_device_data(d, S)
    got = E.loglike_batch(torch.from_numpy(P).cuda(), dd, ss, E.Config.from_workload(w)).cpu().numpy()
    assert np.all(np.isfinite(got))
    idx = np.array([5, 250])
    say("LSO config2 oracle lnL for", idx)
    ref = O.loglike(P[idx], d, S, ocfg(w))
    rel = np.abs(got[idx] - ref) / np.abs(ref)
    say("rel err", rel)
    assert np.all(rel <= 1e-10)


def test_config4_shaped_requests_match_the_oracle(E):
    """The serving workload's own shape without the server: two of its chains
    (state at the LSO, orbits integrated backward over the window), half a
    year at dt = 10 s (2^21 samples), 30 harmonics, mixed precision, data
    made by the oracle, requests of 3, 4, 2 and 3 walkers drawn as the bench
    draws them, each evaluated on the resident data set.  Every walker:
    relative lnL within 1e-4 and |dlnL| within 1e-5 <m|m> (the signal
    scale).  (Served results equal these bitwise:
    test_served_equals_alone_in_the_mix.)"""
    chains = W.serving_chains()
    sets = []
    for c in (1, 6):
        w = W.serving_workload(chains[c], 0)
        d, S = oracle_dataset(w, True)
        dd, ss = to_device_data(d, S)
        cfg = E.Config.from_workload(w)
        sets.append((w, cfg, d, S, E.dataset_init(dd, ss, cfg)))
    reqs = [(0, 3, 21), (1, 4, 22), (0, 2, 23), (1, 3, 24)]
    for k in range(len(sets)):
        w, cfg, d, S, ds = sets[k]
        mine = [i for i, r in enumerate(reqs) if r[0] == k]
        P = np.concatenate([W.walkers(w, B=reqs[i][1], seed=reqs[i][2]) for i in mine])
        say("config-4 shape, data set", k, "walkers", len(P))
        r = O.loglike_sets(P, [d, np.zeros_like(d)], S, ocfg(w))
        ref, mm = r[:, 0], -2.0 * r[:, 1]
        at = 0
        for i in mine:
            n = reqs[i][1]
            got = E.loglike_dataset(torch.from_numpy(P[at:at + n]).cuda(), ds, cfg).cpu().numpy()
            fin = np.isfinite(ref[at:at + n])
            assert np.array_equal(fin, np.isfinite(got))
            err = np.abs(got[fin] - ref[at:at + n][fin])
            say("request", i, "max |dlnL|/<m|m>", (err / mm[at:at + n][fin]).max())
            assert np.all(err <= 1e-4 * np.abs(ref[at:at + n][fin]))
            assert np.all(err <= 1e-5 * mm[at:at + n][fin])
            at += n
