"""The likelihood entry point that allocates nothing
(emri_loglike_dataset_noalloc) against the workspace entry point
(emri_loglike_dataset) on the same data sets: bitwise equal results, on two
calls in a row, the second with a smaller input; and chunking through the
library's scratch array at the 1-year, 2^22-sample shape."""
import numpy as np
import pytest
import torch

from paper_2311_17174_amd import workloads as W
from tests.gpu_common import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def E():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_2311_17174_amd import emri
    return emri


def _dataset(E, w):
    """a data set of walker 0's propagated model plus seeded noise (made by
    the HIP path: both entry points see the same bytes)"""
    cfg = E.Config.from_workload(w)
    psd = E.noise_psd(w.N, w.dt)
    m = E.model_batch(torch.from_numpy(w.inj[None]).cuda(), cfg)[0]
    g = torch.from_numpy(W.gaussian_draws(w.N, w.noise_seed)).cuda()
    sig = torch.sqrt(psd * (w.N * w.dt / 4.0))
    sig[0] = 0.0
    sig[-1] = 0.0
    data = (torch.view_as_real(m).double() + sig[None, :, None] * g).contiguous()
    return cfg, E.dataset_init(data, psd, cfg)


def _both(E, w, P):
    cfg, ds = _dataset(E, w)
    params = torch.from_numpy(P).cuda()
    ref = E.loglike_dataset(params, ds, cfg)
    out = torch.full((len(P),), 7.0, dtype=torch.float64, device="cuda")
    got = E.loglike_dataset_noalloc(params, ds, cfg, out)
    torch.cuda.synchronize()
    return ref.cpu().numpy(), got.cpu().numpy()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_noalloc_equals_workspace_entry_two_calls(E, prec):
    # first call: the 30-day, 2^18-sample shape with 32 walkers and plunging,
    # invalid and edge rows mixed in; second: a smaller batch and signal
    w1 = W.config1().with_(precision=prec)
    P1 = W.walkers(w1)
    P1[3, 3] = 1.2                              # e0 >= 1: invalid, lnL = -inf
    P1[5, 4] = 1.6e-3                            # starts close to the LSO, plunges early
    w2 = W.small(prec, B=5, n_harm=6)
    P2 = W.walkers(w2)
    for w, P in ((w1, P1), (w2, P2)):
        say("noalloc", prec, w.name, "B", len(P), "N", w.N)
        ref, got = _both(E, w, P)
        assert np.isneginf(ref).sum() >= (1 if w is w1 else 0)
        assert np.array_equal(ref, got, equal_nan=False), (ref - got)


def test_noalloc_chunks_through_the_scratch_array(E):
    # 1 yr at 2^22 samples, FP64: about 89 MiB of workspace per walker, so
    # 12 walkers take several chunks of the 512 MiB array
    w = W.config2().with_(B=12)
    per = E.workspace_bytes(E.Config.from_workload(w), 1)
    assert 12 * per > E.NOALLOC_SCRATCH_BYTES
    P = W.walkers(w)
    say("noalloc chunked", w.name, "B", len(P), "per-walker MiB", per / 2 ** 20)
    ref, got = _both(E, w, P)
    assert np.all(np.isfinite(ref))
    assert np.array_equal(ref, got)


def test_noalloc_refuses_what_the_scratch_cannot_hold(E):
    # 2^24 samples, 64 harmonics, coarse step 2^8 dt: one walker needs more
    # than the array; the host check refuses before any launch
    w = W.Workload("big", 1, (1 << 24) * 5.0, 5.0, 1 << 24, 64, 8, "fp64", W.injection())
    cfg = E.Config.from_workload(w)
    assert E.workspace_bytes(cfg, 1) > E.NOALLOC_SCRATCH_BYTES
    params = torch.from_numpy(W.walkers(w)).cuda()
    ds = torch.empty(16, dtype=torch.uint8, device="cuda")
    out = torch.empty(1, dtype=torch.float64, device="cuda")
    with pytest.raises(E.EmriError) as ei:
        E.loglike_dataset_noalloc(params, ds, cfg, out)
    assert ei.value.status == -2                   # EMRI_EWORKSPACE
