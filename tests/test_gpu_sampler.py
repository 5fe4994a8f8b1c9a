"""GPU parity of the ensemble sampler step (stretch move, two halves) and the
ensemble log-posterior, through the C ABI, against the CPU oracle.

The step is a deterministic function of its uniforms, so the HIP chain and
the oracle chain take the same decisions wherever the oracle's acceptance
margin ln u2 - [(D-1) ln z + lnp(Y) - lnp(X)] is wider than the likelihood
tolerance (relative 1e-10 of the log-posteriors involved); the test reports
the narrowest margin and requires every decision to be outside that band.
Coordinates: relative 1e-13 (a stretch is y = x_j + z (x_k - x_j), a few
roundings per step, which an accepted move carries on); lnp: relative 1e-10.
"""
import numpy as np
import pytest

import oracle as O
from paper_2311_17174_amd import workloads as W
from tests.gpu_common import ocfg, oracle_dataset, say, to_device_data

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

EINVAL, EWORKSPACE = -1, -2


@pytest.fixture(scope="module")
def E():
    from paper_2311_17174_amd import emri
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return emri


def sampler_case(width=2.0, Wh=8, seed=3):
    w = W.small("fp64", n_harm=6, Xi0=0.9, n_Xi=2.0)
    fi = W.SAMPLER_FREE
    lo, hi = W.sampler_prior(w, fi, width=width)
    X0 = W.sampler_ensemble(w, Wh, fi, seed=seed)
    return w, fi, lo, hi, X0


def oracle_step_with_margins(X, lnp, fi, lo, hi, a, u, d, S, oc):
    """The oracle step taken in its parts (proposals, log-posterior of the
    proposals, acceptance) so that the decision margins can be reported."""
    X, lnp = X.copy(), lnp.copy()
    Wh = X.shape[0] // 2
    acc = np.zeros(2 * Wh, dtype=np.int32)
    margins, n_out = [], 0
    for h in (0, 1):
        Y, lnz, lpr = O.stretch_propose(X, h, fi, lo, hi, a, u[h])
        n_out += int(np.sum(np.isinf(lpr)))
        lnpY = O.ensemble_lnprob(Y, fi, lo, hi, d, S, oc)
        old = lnp[h * Wh:(h + 1) * Wh]
        both = np.isfinite(lnpY) & np.isfinite(old)
        with np.errstate(invalid="ignore"):
            m = np.abs(np.log(u[h][:, 2]) - (lnz + lnpY - old))
            band = 1e-10 * (np.abs(lnpY) + np.abs(old))
        margins.append(np.where(both, m / np.where(both, band, 1.0), np.inf))
        acc += O.stretch_accept(X, lnp, h, Y, lnpY, lnz, u[h])
    return X, lnp, acc, np.concatenate(margins), n_out


def assert_lnp_close(got, ref):
    fin = np.isfinite(ref)
    assert np.array_equal(fin, np.isfinite(got)), (got, ref)
    assert np.all(got[~fin] == -np.inf)
    np.testing.assert_allclose(got[fin], ref[fin], rtol=1e-10, atol=0)


def test_ensemble_lnprob_parity(E):
    w, fi, lo, hi, X0 = sampler_case()
    X0[1, 0] = 1.0                     # M = 1 Msun < mu: outside the box and unphysical
    d, S = oracle_dataset(w, True)
    ref = O.ensemble_lnprob(X0, fi, lo, hi, d, S, ocfg(w))
    cfg = E.Config.from_workload(w)
    dd, ss = to_device_data(d, S)
    ds = E.dataset_init(dd, ss, cfg)
    got = E.ensemble_lnprob(torch.from_numpy(X0).cuda(), E.make_prior(fi, lo, hi), ds,
                            cfg).cpu().numpy()
    say("lnp ref", ref)
    say("lnp got", got)
    assert np.sum(np.isinf(ref)) >= 2 and np.sum(np.isfinite(ref)) >= 4
    assert_lnp_close(got, ref)
    # a box that holds every walker: lnp equals lnL
    wide_lo, wide_hi = W.sampler_prior(w, fi, width=1e3)
    wide_lo[0] = 0.5
    lnl = E.loglike_dataset(torch.from_numpy(X0).cuda(), ds, cfg).cpu().numpy()
    got = E.ensemble_lnprob(torch.from_numpy(X0).cuda(), E.make_prior(fi, wide_lo, wide_hi),
                            ds, cfg).cpu().numpy()
    assert np.array_equal(got, lnl)


def test_stretch_chain_parity(E):
    """Six steps of 2W = 16 walkers, D = 8, against the oracle chain; the
    narrow box puts walkers and proposals outside it, so both -inf rules are
    taken."""
    run_chain(E, *sampler_case())


def test_stretch_chain_parity_lso(E):
    """The paper's own setting (Sec. 3): orbital state at the LSO, fixed
    eccentricity and angles, free masses, spin and Xi0 (D = 4)."""
    fi = (0, 1, 2, 14)
    w = W.small("fp64", n_harm=6, Xi0=0.9, n_Xi=2.0).with_(ic=1)
    lo, hi = W.sampler_prior(w, fi, width=2.0)
    run_chain(E, w, fi, lo, hi, W.sampler_ensemble(w, 8, fi, seed=3))


def run_chain(E, w, fi, lo, hi, X0):
    Wh, steps, a = X0.shape[0] // 2, 6, 2.0
    U = W.sampler_uniforms(Wh, steps, seed=11)
    d, S = oracle_dataset(w, True)
    oc = ocfg(w)
    cfg = E.Config.from_workload(w)
    dd, ss = to_device_data(d, S)
    ds = E.dataset_init(dd, ss, cfg)
    prior = E.make_prior(fi, lo, hi)

    Xo = X0.copy()
    lpo = O.ensemble_lnprob(Xo, fi, lo, hi, d, S, oc)
    Xg = torch.from_numpy(X0.copy()).cuda()
    lpg = E.ensemble_lnprob(Xg, prior, ds, cfg)
    assert_lnp_close(lpg.cpu().numpy(), lpo)
    ws = torch.empty(E.sampler_workspace_bytes(cfg, Wh), dtype=torch.uint8, device="cuda")
    took_from_inf = n_out = n_acc = 0
    for s in range(steps):
        was_inf = ~np.isfinite(lpo)
        Xc, lpc, accc = O.stretch_step(Xo, lpo, fi, lo, hi, a, U[s], d, S, oc)
        Xo, lpo, acco, margins, nout = oracle_step_with_margins(Xo, lpo, fi, lo, hi, a, U[s],
                                                                d, S, oc)
        # the composed oracle step is the same function as its parts
        assert np.array_equal(Xc, Xo) and np.array_equal(lpc, lpo) and np.array_equal(accc, acco)
        accg = E.stretch_step(Xg, lpg, prior, a, torch.from_numpy(U[s]).cuda(), ds, cfg, ws=ws)
        accg = accg.cpu().numpy()
        say(f"step {s}: acc oracle {acco.tolist()} hip {accg.tolist()}; "
            f"narrowest margin / band {np.min(margins):.3g}; proposals outside box {nout}")
        assert np.min(margins) > 1.0, "a decision inside the likelihood tolerance band"
        assert np.array_equal(accg, acco)
        np.testing.assert_allclose(Xg.cpu().numpy(), Xo, rtol=1e-13, atol=0)
        assert_lnp_close(lpg.cpu().numpy(), lpo)
        took_from_inf += int(np.sum(was_inf & (acco == 1)))
        n_out += nout
        n_acc += int(acco.sum())
    say("accepted", n_acc, "of", 2 * Wh * steps, "; walkers leaving -inf", took_from_inf,
        "; proposals outside the box", n_out)
    assert 0 < n_acc < 2 * Wh * steps
    assert took_from_inf > 0 and n_out > 0


def test_stretch_step_chunked_and_errors(E):
    """A workspace that holds the proposals plus 3 walkers evaluates each half
    in chunks: bitwise the same step.  Bad arguments are rejected before any
    work, leaving the ensemble untouched."""
    w, fi, lo, hi, X0 = sampler_case()
    Wh = X0.shape[0] // 2
    U = torch.from_numpy(W.sampler_uniforms(Wh, 1, seed=5)[0]).cuda()
    d, S = oracle_dataset(w, True)
    cfg = E.Config.from_workload(w)
    dd, ss = to_device_data(d, S)
    ds = E.dataset_init(dd, ss, cfg)
    prior = E.make_prior(fi, lo, hi)
    X1 = torch.from_numpy(X0.copy()).cuda()
    lp1 = E.ensemble_lnprob(X1, prior, ds, cfg)
    X2, lp2 = X1.clone(), lp1.clone()
    a1 = E.stretch_step(X1, lp1, prior, 2.0, U, ds, cfg)
    head = E.sampler_workspace_bytes(cfg, Wh) - E.workspace_bytes(cfg, Wh)
    ws = torch.empty(head + E.workspace_bytes(cfg, 3), dtype=torch.uint8, device="cuda")
    a2 = E.stretch_step(X2, lp2, prior, 2.0, U, ds, cfg, ws=ws)
    torch.cuda.synchronize()
    assert torch.equal(a1, a2) and torch.equal(X1, X2) and torch.equal(lp1, lp2)

    Xs, ls = X1.clone(), lp1.clone()

    def status(fn):
        with pytest.raises(E.EmriError) as ei:
            fn()
        return ei.value.status

    bad_priors = [
        E.make_prior([], [], []),                              # D = 0
        E.make_prior([0, 0], [0, 0], [1, 1]),                  # repeated index
        E.make_prior([17], [0], [1]),                          # index out of range
        E.make_prior([0], [2.0], [1.0]),                       # lo > hi
        E.make_prior([0], [float("nan")], [1.0]),              # NaN bound
    ]
    for pr in bad_priors:
        assert status(lambda: E.stretch_step(X1, lp1, pr, 2.0, U, ds, cfg)) == EINVAL
        assert status(lambda: E.ensemble_lnprob(X1, pr, ds, cfg)) == EINVAL
    for a in (1.0, 0.5, float("nan"), float("inf")):
        assert status(lambda: E.stretch_step(X1, lp1, prior, a, U, ds, cfg)) == EINVAL
    small = torch.empty(head, dtype=torch.uint8, device="cuda")
    assert status(lambda: E.stretch_step(X1, lp1, prior, 2.0, U, ds, cfg, ws=small)) == EWORKSPACE
    torch.cuda.synchronize()
    assert torch.equal(X1, Xs) and torch.equal(lp1, ls)


def test_ensemble_lnprob_with_adaptive_orbit(E):
    """The log-posterior of an ensemble whose orbits use the adaptive
    integrator (Dormand-Prince 5(4), rtol 1e-10) against the oracle's."""
    w, fi, lo, hi, X0 = sampler_case()
    w = w.with_(ode=1, ode_rtol=1e-10, ode_atol=1e-10)
    X0[1, 0] = 1.0                     # outside the box and unphysical
    d, S = oracle_dataset(w, True)
    ref = O.ensemble_lnprob(X0, fi, lo, hi, d, S, ocfg(w))
    cfg = E.Config.from_workload(w)
    dd, ss = to_device_data(d, S)
    ds = E.dataset_init(dd, ss, cfg)
    got = E.ensemble_lnprob(torch.from_numpy(X0).cuda(), E.make_prior(fi, lo, hi), ds,
                            cfg).cpu().numpy()
    say("DP5 lnp ref", ref, "got", got)
    assert np.sum(np.isfinite(ref)) >= 4
    assert_lnp_close(got, ref)
