"""Host-side checks of the C ABI (no GPU compute): the library loads, exports
every entry point include/emri.h declares, and its planning functions
validate configurations and size workspaces consistently."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_2311_17174_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "emri.h")


@pytest.fixture(scope="module")
def E():
    from paper_2311_17174_amd import emri
    return emri


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:[\w\s\*]+?)\b(emri_\w+)\s*\(", text, re.M)))


def test_header_declares_the_api():
    names = declared_functions()
    for n in ("emri_waveform_batch", "emri_fft_batch", "emri_loglike_batch",
              "emri_workspace_bytes", "emri_dataset_init", "emri_loglike_dataset"):
        assert n in names


def test_library_exports_every_declared_symbol(E):
    out = subprocess.check_output(["nm", "-D", "--defined-only", E.LIB_PATH]).decode()
    exported = {line.split()[-1] for line in out.splitlines() if line.strip()}
    missing = [n for n in declared_functions() if n not in exported]
    assert not missing, missing
    assert set(E.EXPORTED) == set(declared_functions())
    assert E.lib.emri_abi_version() == 8


def test_struct_layout_matches_header(E):
    # int64 N at offset 16, six int32, then the two integrator tolerances: 64 bytes
    assert ctypes.sizeof(E._Cfg) == 64
    assert E._Cfg.N.offset == 16 and E._Cfg.n_harm.offset == 24
    assert E._Cfg.ode.offset == 40 and E._Cfg.reserved.offset == 44
    assert E._Cfg.ode_rtol.offset == 48 and E._Cfg.ode_atol.offset == 56
    # emri_fmg: two int32 then the pivot frequency; emri_prior: n_free, idx[17], lo, hi
    assert ctypes.sizeof(E._Fmg) == 16 and E._Fmg.f_star.offset == 8
    assert E._Prior.idx.offset == 4 and E._Prior.lo.offset == 72
    assert E._Prior.hi.offset == 72 + 17 * 8 and ctypes.sizeof(E._Prior) == 72 + 34 * 8


@pytest.mark.parametrize("bad", [
    dict(N=3 << 12), dict(N=1 << 11), dict(N=1 << 25), dict(dt=0.0), dict(T_obs=-1.0),
    dict(n_harm=0), dict(n_harm=65), dict(precision=2), dict(coarse_log2=7),
    dict(coarse_log2=13), dict(T_obs=1e7), dict(ode=3), dict(ode=-1),
    dict(ode=1, ode_rtol=0.0), dict(ode=1, ode_rtol=1e-14), dict(ode=1, ode_rtol=1e-2),
    dict(ode=1, ode_rtol=float("nan")), dict(ode=1, ode_atol=-1e-12),
    dict(ode=1, ode_atol=float("inf")), dict(ode=2, ode_rtol=1e-14),
    dict(ode=2, ode_atol=float("nan")),
])
def test_invalid_configurations_are_rejected(E, bad):
    base = dict(T_obs=2.5 * 86400, dt=10.0, N=1 << 15, n_harm=8, precision=0, coarse_log2=10)
    base.update(bad)
    c = E.Config(**base)
    assert E.lib.emri_workspace_bytes(ctypes.byref(c.c()), 4) == 0
    assert E.lib.emri_dataset_bytes(ctypes.byref(c.c())) == 0


def test_reserved_field_and_ignored_tolerances(E):
    c = E.Config(T_obs=2.5 * 86400, dt=10.0, N=1 << 15, n_harm=8).c()
    assert E.lib.emri_workspace_bytes(ctypes.byref(c), 4) > 0
    c.reserved = 1
    assert E.lib.emri_workspace_bytes(ctypes.byref(c), 4) == 0
    c.reserved = 0
    c.ode_rtol = -1.0                  # RK4 ignores the tolerances
    assert E.lib.emri_workspace_bytes(ctypes.byref(c), 4) > 0


def test_workspace_grows_with_batch_and_precision(E):
    for w in (W.config1(), W.config2(), W.small()):
        c = E.Config.from_workload(w)
        sizes = [E.workspace_bytes(c, b) for b in (1, 2, 8, 64)]
        assert sizes == sorted(sizes) and sizes[0] < sizes[-1]
        per = (sizes[3] - sizes[2]) / 56
        # the packed signal dominates: N complex elements per walker
        assert per >= w.N * 16
        cm = E.Config.from_workload(w.with_(precision="mixed"))
        assert E.workspace_bytes(cm, 64) < sizes[3]
        assert E.dataset_bytes(cm) < E.dataset_bytes(c)


def test_config2_fits_one_mi355x(E):
    c = E.Config.from_workload(W.config2())
    total = E.workspace_bytes(c, 256) + E.dataset_bytes(c)
    assert total < 32 * 2 ** 30     # well inside 288 GB of HBM


def test_call_errors_without_launch(E):
    """A null workspace or a mismatched T_obs is a call error that is caught on
    the host before anything touches a device."""
    c = E.Config.from_workload(W.small())
    cc = c.c()
    rc = E.lib.emri_loglike_batch(None, 4, None, None, c.T_obs, c.dt, ctypes.byref(cc), None,
                                  None, 0, None)
    assert rc == -1
    assert b"null" in E.lib.emri_last_error()
    rc = E.lib.emri_loglike_batch(None, 4, None, None, c.T_obs + 1, c.dt, ctypes.byref(cc),
                                  None, None, 0, None)
    assert rc == -1
    rc = E.lib.emri_loglike_batch(None, 0, None, None, c.T_obs, c.dt, ctypes.byref(cc), None,
                                  None, 0, None)
    assert rc == 0
    rc = E.lib.emri_waveform_batch(ctypes.c_void_p(8), 4, ctypes.byref(cc), ctypes.c_void_p(8),
                                   ctypes.c_void_p(8), 16, None)
    assert rc == -2
    # the orbit alone: the same checks (null outputs, small workspace, B = 0)
    rc = E.lib.emri_orbit_batch(ctypes.c_void_p(8), 4, ctypes.byref(cc), None, None,
                                ctypes.c_void_p(8), 1 << 30, None)
    assert rc == -1 and b"null" in E.lib.emri_last_error()
    rc = E.lib.emri_orbit_batch(ctypes.c_void_p(8), 4, ctypes.byref(cc), ctypes.c_void_p(8),
                                ctypes.c_void_p(8), ctypes.c_void_p(8), 16, None)
    assert rc == -2
    assert E.lib.emri_orbit_batch(None, 0, ctypes.byref(cc), None, None, None, 0, None) == 0
    bad = E.Config.from_workload(W.small().with_(ode=2, ode_rtol=1e-2, ode_atol=1e-12)).c()
    rc = E.lib.emri_orbit_batch(ctypes.c_void_p(8), 4, ctypes.byref(bad), ctypes.c_void_p(8),
                                ctypes.c_void_p(8), ctypes.c_void_p(8), 1 << 30, None)
    assert rc == -1 and b"tolerances" in E.lib.emri_last_error()


def test_workspace_sizes_are_consistent(E):
    """Host-side sizing (no GPU): the workspace grows with the batch and by
    at least the signal per walker; the sampler's adds the proposals'
    staging to a whole batch of W; the data set does not depend on B."""
    c = E.Config(T_obs=2.5 * 86400, dt=10.0, N=1 << 15, n_harm=8)
    sizes = [E.workspace_bytes(c, b) for b in (1, 2, 8, 64)]
    assert all(b > a for a, b in zip(sizes, sizes[1:]))
    per = (sizes[3] - sizes[2]) / 56
    assert per >= c.N * 16                          # the complex FP64 signal
    assert E.sampler_workspace_bytes(c, 8) >= E.workspace_bytes(c, 8) + 8 * 17 * 8 + 3 * 8 * 8
    mixed = E.Config(T_obs=2.5 * 86400, dt=10.0, N=1 << 15, n_harm=8, precision=E.MIXED)
    assert E.workspace_bytes(mixed, 64) < E.workspace_bytes(c, 64)
    assert E.dataset_bytes(mixed) < E.dataset_bytes(c)
    lso = E.Config(T_obs=2.5 * 86400, dt=10.0, N=1 << 15, n_harm=8, ic=E.IC_LSO)
    assert E.workspace_bytes(lso, 8) == E.workspace_bytes(c, 8)
    bad = E.Config(T_obs=2.5 * 86400, dt=10.0, N=1 << 15, n_harm=8, ic=2)
    assert E.lib.emri_workspace_bytes(ctypes.byref(bad.c()), 4) == 0


def test_documented_array_layouts():
    """The header documents the time-domain waveform as [B][N][2] (channels
    interleaved per sample: the complex sample h_I + i h_II the FFT reads),
    the spectra as [B][2][N/2+1] complex and row entry 16 as alpha_T; the
    binding allocates and checks the same shapes (no GPU needed)."""
    with open(HEADER) as f:
        h = f.read()
    assert "ht      [B][N][2] real, channel-interleaved (I, II) per sample" in h
    assert "hf   [B][2][N/2+1] complex (re, im interleaved)" in h
    assert "16 alpha_T" in h
    import inspect
    from paper_2311_17174_amd import emri as E
    src = inspect.getsource(E.waveform_batch)
    assert "(B, cfg.N, 2)" in src
    src = inspect.getsource(E.fft_batch)
    assert "(B, 2, H, 2)" in src
