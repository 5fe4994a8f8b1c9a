"""GPU tests of the serving loop (emri_server_*): continuous batching over
resident data sets, admission by HBM footprint, hipGraph replays.

Every served result is compared bitwise with the same walkers evaluated alone
by emri_loglike_dataset (whose parity with the oracle is tested elsewhere),
over several rounds so that graph replays run between eager work."""
import threading

import numpy as np
import pytest

import oracle as O
from paper_2311_17174_amd import workloads as W
from tests.gpu_common import ocfg, oracle_dataset, say, to_device_data

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def E():
    from paper_2311_17174_amd import emri
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return emri


def two_datasets(E):
    """two resident data sets with different shapes (N = 2^15 and 2^16)"""
    wa = W.small("mixed", n_harm=6)
    wb = W.small("mixed", n_harm=8, days=5.0, N=1 << 16, e0=0.2, M=8e5)
    out = []
    for w in (wa, wb):
        d, S = oracle_dataset(w, True)
        dd, ss = to_device_data(d, S)
        out.append((w, E.Config.from_workload(w), dd, ss))
    return out


def alone(E, cfg, dd, ss, P):
    ds = E.dataset_init(dd, ss, cfg)
    return E.loglike_dataset(torch.from_numpy(np.ascontiguousarray(P)).cuda(), ds,
                             cfg).cpu().numpy()


@pytest.mark.parametrize("segs", [None, "3"])
def test_served_equals_alone_in_the_mix(E, segs):
    """segs = "3": the captured graphs hold the orbit-segment pipeline's
    second stream (fork and join inside the capture)"""
    if segs:
        E.set_tuning(orbit_segments=int(segs))
    sets = two_datasets(E)
    arena = torch.empty(3 << 30, dtype=torch.uint8, device="cuda")
    reqs = []
    for i in range(12):
        k = i % 2
        w, cfg, dd, ss = sets[k]
        Wn = [5, 17, 40, 64, 3, 33][i % 6]
        reqs.append((k, W.walkers(w, B=Wn, seed=1000 + i)))
    expect = [alone(E, sets[k][1], sets[k][2], sets[k][3], P) for k, P in reqs]
    with E.Server(arena, n_streams=3, max_batch=64, use_graphs=True) as srv:
        ids = [srv.add_dataset(dd, ss, cfg) for (w, cfg, dd, ss) in sets]
        for rnd in range(4):
            # submit from several threads at once, then collect
            tickets = [None] * len(reqs)

            def sub(i):
                k, P = reqs[i]
                tickets[i] = srv.submit(ids[k], P)

            th = [threading.Thread(target=sub, args=(i,)) for i in range(len(reqs))]
            for t in th:
                t.start()
            for t in th:
                t.join()
            for i, t in enumerate(tickets):
                got, lat = srv.wait(t, timeout=120.0)
                assert np.array_equal(got, expect[i]), (rnd, i)
                assert lat > 0
            # eager work between graph replays
            k, P = reqs[0]
            assert np.array_equal(alone(E, sets[k][1], sets[k][2], sets[k][3], P), expect[0])
        st = srv.stats()
    say("server stats", st)
    assert st["completed"] == 4 * len(reqs)
    assert st["graph_launches"] > 0 and st["graph_captures"] >= 1
    assert st["batches"] < 4 * len(reqs)          # requests were batched together


def test_served_matches_oracle(E):
    """A served request agrees with the oracle at the mixed-path tolerance."""
    sets = two_datasets(E)
    w, cfg, dd, ss = sets[1]
    P = W.walkers(w, B=7, seed=77)
    d, S = oracle_dataset(w, True)
    ref = O.loglike(P, d, S, ocfg(w))
    arena = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
    with E.Server(arena, n_streams=2, max_batch=32) as srv:
        i = srv.add_dataset(dd, ss, cfg)
        got, _ = srv.wait(srv.submit(i, P), timeout=120.0)
    assert np.all(np.abs(got - ref) / np.abs(ref) <= 1e-4)


def test_served_lso_dataset(E):
    """A data set in the LSO convention (orbits integrated backward from the
    last stable orbit) served eagerly, captured and replayed: bitwise the
    same walkers evaluated alone, and those agree with the oracle (FP64)."""
    w = W.small("fp64", n_harm=6).with_(ic=1)
    d, S = oracle_dataset(w, True)
    dd, ss = to_device_data(d, S)
    cfg = E.Config.from_workload(w)
    P = W.walkers(w, B=9, seed=5)
    ref = O.loglike(P, d, S, ocfg(w))
    expect = alone(E, cfg, dd, ss, P)
    assert np.all(np.abs(expect - ref) <= 1e-10 * np.abs(ref))
    arena = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
    with E.Server(arena, n_streams=1, max_batch=32, use_graphs=True) as srv:
        i = srv.add_dataset(dd, ss, cfg)
        for _ in range(3):                          # eager, captured, replayed
            got, _ = srv.wait(srv.submit(i, P), timeout=120.0)
            assert np.array_equal(got, expect)
        st = srv.stats()
    assert st["graph_launches"] >= 1


@pytest.mark.parametrize("ic", [0, 1])
def test_served_adaptive_orbit(E, ic):
    """Data sets whose orbits use the adaptive integrator (one wave per
    walker, lanes sharing each step's nodes; at t = 0 in three pipelined
    segments, or backward from the LSO) served eagerly, captured and replayed:
    bitwise the walkers evaluated alone, which agree with the oracle."""
    E.set_tuning(orbit_segments=3)
    w = W.small("fp64", n_harm=6, days=20.0, N=1 << 18).with_(ic=ic, ode=1, ode_rtol=1e-10,
                                                              ode_atol=1e-10)
    d, S = oracle_dataset(w, True)
    dd, ss = to_device_data(d, S)
    cfg = E.Config.from_workload(w)
    P = W.walkers(w, B=9, seed=7)
    ref = O.loglike(P, d, S, ocfg(w))
    expect = alone(E, cfg, dd, ss, P)
    assert np.all(np.abs(expect - ref) <= 1e-10 * np.abs(ref))
    arena = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
    with E.Server(arena, n_streams=2, max_batch=32, use_graphs=True) as srv:
        i = srv.add_dataset(dd, ss, cfg)
        for _ in range(3):                          # eager, captured, replayed
            got, _ = srv.wait(srv.submit(i, P), timeout=120.0)
            assert np.array_equal(got, expect)
        st = srv.stats()
    assert st["graph_launches"] >= 1


def test_admission_by_footprint(E):
    """An arena that holds one batch block at a time still serves every
    request (admission waits for memory); a request larger than the budget is
    rejected at submit."""
    sets = two_datasets(E)
    w, cfg, dd, ss = sets[0]
    one = E.workspace_bytes(cfg, 32) + 32 * 17 * 8 + 32 * 8 + 4096
    arena = torch.empty(E.dataset_bytes(cfg) + int(1.5 * one), dtype=torch.uint8, device="cuda")
    reqs = [W.walkers(w, B=b, seed=500 + b) for b in (4, 20, 31, 9, 16)]
    expect = [alone(E, cfg, dd, ss, P) for P in reqs]
    with E.Server(arena, n_streams=4, max_batch=64) as srv:
        i = srv.add_dataset(dd, ss, cfg)
        with pytest.raises(E.EmriError) as ex:
            srv.submit(i, W.walkers(w, B=64))
        assert ex.value.status == -2
        ts = [srv.submit(i, P) for P in reqs]
        for t, e in zip(ts, expect):
            got, _ = srv.wait(t, timeout=120.0)
            assert np.array_equal(got, e)
        st = srv.stats()
    assert st["rejected"] == 1
    assert st["arena_peak"] <= arena.numel()
