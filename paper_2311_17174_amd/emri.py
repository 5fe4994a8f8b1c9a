"""Thin Python binding of libemri (include/emri.h): argument marshalling only.

Every step of the likelihood runs in the HIP kernels of ``libemri.so``; this
module passes torch device pointers and the current stream through ctypes.
Importing it loads the library and fails loudly if it has not been built
(``python -m paper_2311_17174_amd.build``).  There is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass

import torch  # must be imported before the library so one HIP runtime is used

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libemri.so")

NPAR = 17
FP64 = 0
MIXED = 1
PRECISIONS = {"fp64": FP64, "mixed": MIXED}
IC_START = 0     # initial conditions at t = 0
IC_LSO = 1       # at the last stable orbit, integrated backward (the paper's convention)
ODE_RK4 = 0      # classical RK4 on the coarse nodes
ODE_DP5 = 1      # adaptive Dormand-Prince 5(4), continuous extension at the nodes
ODE_RK78 = 2     # adaptive Fehlberg 7(8), order 7 kept, stepped node to node

EXPORTED = ("emri_abi_version", "emri_last_error", "emri_workspace_bytes", "emri_orbit_batch",
            "emri_waveform_batch", "emri_fft_batch", "emri_loglike_batch",
            "emri_dataset_bytes", "emri_dataset_init", "emri_loglike_dataset",
            "emri_model_batch", "emri_noise_psd", "emri_trace_enable", "emri_trace_read",
            "emri_trace_stage_name", "emri_sampler_workspace_bytes", "emri_ensemble_lnprob",
            "emri_stretch_step", "emri_loglike_dataset_fmg", "emri_tuning_set",
            "emri_tuning_get", "emri_loglike_dataset_noalloc")
NOALLOC_SCRATCH_BYTES = 512 << 20     # EMRI_NOALLOC_SCRATCH_BYTES


class EmriError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where} failed with status {status}: {msg}")
        self.status = status


class _Cfg(ctypes.Structure):
    _fields_ = [("T_obs", ctypes.c_double), ("dt", ctypes.c_double), ("N", ctypes.c_int64),
                ("n_harm", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("coarse_log2", ctypes.c_int32), ("ic", ctypes.c_int32),
                ("ode", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("ode_rtol", ctypes.c_double), ("ode_atol", ctypes.c_double)]


class _Prior(ctypes.Structure):
    _fields_ = [("n_free", ctypes.c_int32), ("idx", ctypes.c_int32 * NPAR),
                ("lo", ctypes.c_double * NPAR), ("hi", ctypes.c_double * NPAR)]


def make_prior(free_idx, lo, hi) -> _Prior:
    """Box prior on the parameters free_idx (lo <= p[i] <= hi), as emri_prior."""
    free_idx, lo, hi = list(free_idx), list(lo), list(hi)
    if not (len(free_idx) == len(lo) == len(hi)) or len(free_idx) > NPAR:
        raise ValueError("free_idx, lo and hi must have the same length, at most 17")
    pr = _Prior()
    pr.n_free = len(free_idx)
    for d, (i, a, b) in enumerate(zip(free_idx, lo, hi)):
        pr.idx[d], pr.lo[d], pr.hi[d] = int(i), float(a), float(b)
    return pr


class _Tuning(ctypes.Structure):
    _fields_ = [("orbit_segments", ctypes.c_int32), ("fft_row_log2", ctypes.c_int32),
                ("fft_col_run_bytes", ctypes.c_int32), ("like_walkers_per_wg", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class _Fmg(ctypes.Structure):
    _fields_ = [("order", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("f_star", ctypes.c_double)]


@dataclass(frozen=True)
class Config:
    T_obs: float
    dt: float
    N: int
    n_harm: int
    precision: int = FP64
    coarse_log2: int = 10
    ic: int = IC_START       # IC_LSO: the row's orbital state is at the LSO
    ode: int = ODE_RK4       # ODE_DP5, ODE_RK78: adaptive integrators with the tolerances below
    ode_rtol: float = 1e-12
    ode_atol: float = 1e-12

    @staticmethod
    def from_workload(w) -> "Config":
        return Config(w.T_obs, w.dt, w.N, w.n_harm, PRECISIONS[w.precision], w.coarse_log2,
                      w.ic, w.ode, w.ode_rtol, w.ode_atol)

    def c(self) -> _Cfg:
        return _Cfg(float(self.T_obs), float(self.dt), int(self.N), int(self.n_harm),
                    int(self.precision), int(self.coarse_log2), int(self.ic), int(self.ode), 0,
                    float(self.ode_rtol), float(self.ode_atol))

    @property
    def n_intervals(self) -> int:
        """K = ceil(N_valid / 2^coarse_log2), N_valid = round(T_obs / dt)."""
        nv = int(math.floor(self.T_obs / self.dt + 0.5))      # llround, as the library
        m = 1 << int(self.coarse_log2)
        return (nv + m - 1) // m

    @property
    def real_dtype(self) -> torch.dtype:
        return torch.float64 if self.precision == FP64 else torch.float32


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2311_17174_amd.build` (hipcc, gfx950)")
    L = ctypes.CDLL(LIB_PATH)
    vp, sz, i64 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int64
    cp = ctypes.POINTER(_Cfg)
    d = ctypes.c_double
    sig = {
        "emri_abi_version": ([], ctypes.c_int),
        "emri_last_error": ([], ctypes.c_char_p),
        "emri_workspace_bytes": ([cp, i64], sz),
        "emri_dataset_bytes": ([cp], sz),
        "emri_waveform_batch": ([vp, i64, cp, vp, vp, sz, vp], ctypes.c_int),
        "emri_orbit_batch": ([vp, i64, cp, vp, vp, vp, sz, vp], ctypes.c_int),
        "emri_fft_batch": ([vp, i64, cp, vp, vp, sz, vp], ctypes.c_int),
        "emri_loglike_batch": ([vp, i64, vp, vp, d, d, cp, vp, vp, sz, vp], ctypes.c_int),
        "emri_dataset_init": ([vp, vp, cp, vp, sz, vp], ctypes.c_int),
        "emri_loglike_dataset": ([vp, i64, vp, cp, vp, vp, sz, vp], ctypes.c_int),
        "emri_loglike_dataset_noalloc": ([vp, i64, vp, cp, vp, vp], ctypes.c_int),
        "emri_model_batch": ([vp, i64, cp, vp, vp, sz, vp], ctypes.c_int),
        "emri_noise_psd": ([ctypes.c_int, i64, d, vp, vp], ctypes.c_int),
        "emri_trace_enable": ([ctypes.c_int], ctypes.c_int),
        "emri_trace_read": ([ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64),
                             ctypes.c_int], ctypes.c_int),
        "emri_trace_stage_name": ([ctypes.c_int], ctypes.c_char_p),
        "emri_sampler_workspace_bytes": ([cp, i64], sz),
        "emri_ensemble_lnprob": ([vp, i64, ctypes.POINTER(_Prior), vp, cp, vp, vp, sz, vp],
                                 ctypes.c_int),
        "emri_loglike_dataset_fmg": ([vp, i64, vp, ctypes.POINTER(_Fmg), vp, cp, vp, vp, sz, vp],
                                     ctypes.c_int),
        "emri_stretch_step": ([vp, vp, i64, ctypes.POINTER(_Prior), d, vp, vp, cp, vp, vp, sz,
                               vp], ctypes.c_int),
        "emri_tuning_set": ([ctypes.POINTER(_Tuning)], ctypes.c_int),
        "emri_tuning_get": ([ctypes.POINTER(_Tuning)], ctypes.c_int),
    }
    for name, (a, r) in sig.items():
        f = getattr(L, name)
        f.argtypes = a
        f.restype = r
    return L


lib = _load()


def _check(rc: int, where: str):
    if rc != 0:
        raise EmriError(rc, where, lib.emri_last_error().decode())


def _stream(stream) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def _dev(t: torch.Tensor, dtype: torch.dtype, shape, name: str):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return t.data_ptr()


TUNING_FIELDS = ("orbit_segments", "fft_row_log2", "fft_col_run_bytes", "like_walkers_per_wg")


def get_tuning() -> dict:
    """The process-wide launch-plan overrides (emri_tuning_get); 0 = automatic."""
    t = _Tuning()
    _check(lib.emri_tuning_get(ctypes.byref(t)), "emri_tuning_get")
    return {n: getattr(t, n) for n in TUNING_FIELDS}


def set_tuning(**kw) -> None:
    """Set the launch-plan overrides (emri_tuning_set); fields not named are
    automatic (0)."""
    bad = set(kw) - set(TUNING_FIELDS)
    if bad:
        raise KeyError(sorted(bad))
    t = _Tuning(*[int(kw.get(n, 0)) for n in TUNING_FIELDS], 0)
    _check(lib.emri_tuning_set(ctypes.byref(t)), "emri_tuning_set")


class tuning:
    """Context manager: the overrides kw inside, the previous ones after."""

    def __init__(self, **kw):
        self.kw = kw

    def __enter__(self):
        self.prev = get_tuning()
        set_tuning(**self.kw)
        return self

    def __exit__(self, *exc):
        set_tuning(**self.prev)


def workspace_bytes(cfg: Config, B: int) -> int:
    c = cfg.c()
    n = lib.emri_workspace_bytes(ctypes.byref(c), int(B))
    if n == 0:
        raise EmriError(-1, "emri_workspace_bytes", "invalid configuration")
    return n


def dataset_bytes(cfg: Config) -> int:
    c = cfg.c()
    n = lib.emri_dataset_bytes(ctypes.byref(c))
    if n == 0:
        raise EmriError(-1, "emri_dataset_bytes", "invalid configuration")
    return n


def alloc_workspace(cfg: Config, B: int, device="cuda", with_dataset: bool = False):
    n = workspace_bytes(cfg, B) + (dataset_bytes(cfg) + 256 if with_dataset else 0)
    return torch.empty(n, dtype=torch.uint8, device=device)


def orbit_batch(params: torch.Tensor, cfg: Config, ws: torch.Tensor | None = None,
                stream=None) -> tuple[torch.Tensor, torch.Tensor]:
    """([B][K+1][10] fp64 orbit nodes: state then derivative, [B] int32 K_w)."""
    B = params.shape[0]
    pp = _dev(params, torch.float64, (B, NPAR), "params")
    K = cfg.n_intervals
    orb = torch.empty((B, K + 1, 10), dtype=torch.float64, device=params.device)
    kw = torch.empty(B, dtype=torch.int32, device=params.device)
    if ws is None:
        ws = alloc_workspace(cfg, B, params.device)
    c = cfg.c()
    _check(lib.emri_orbit_batch(pp, B, ctypes.byref(c), orb.data_ptr(), kw.data_ptr(),
                                ws.data_ptr(), ws.numel(), _stream(stream)), "emri_orbit_batch")
    return orb, kw


def waveform_batch(params: torch.Tensor, cfg: Config, out: torch.Tensor | None = None,
                   ws: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """[B][N][2] channel-interleaved time-domain waveforms (unit distance)."""
    B = params.shape[0]
    pp = _dev(params, torch.float64, (B, NPAR), "params")
    if out is None:
        out = torch.empty((B, cfg.N, 2), dtype=cfg.real_dtype, device=params.device)
    op = _dev(out, cfg.real_dtype, (B, cfg.N, 2), "out")
    if ws is None:
        ws = alloc_workspace(cfg, B, params.device)
    c = cfg.c()
    _check(lib.emri_waveform_batch(pp, B, ctypes.byref(c), op, ws.data_ptr(), ws.numel(),
                                   _stream(stream)), "emri_waveform_batch")
    return out


def fft_batch(ht: torch.Tensor, cfg: Config, out: torch.Tensor | None = None,
              ws: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """[B][2][N/2+1] complex spectra (dt-normalised) of [B][N][2] waveforms."""
    B = ht.shape[0]
    hp = _dev(ht, cfg.real_dtype, (B, cfg.N, 2), "ht")
    H = cfg.N // 2 + 1
    if out is None:
        out = torch.empty((B, 2, H, 2), dtype=cfg.real_dtype, device=ht.device)
    op = _dev(out, cfg.real_dtype, (B, 2, H, 2), "out")
    if ws is None:
        ws = alloc_workspace(cfg, B, ht.device)
    c = cfg.c()
    _check(lib.emri_fft_batch(hp, B, ctypes.byref(c), op, ws.data_ptr(), ws.numel(),
                              _stream(stream)), "emri_fft_batch")
    return torch.view_as_complex(out)


def loglike_batch(params: torch.Tensor, data: torch.Tensor, psd: torch.Tensor, cfg: Config,
                  out: torch.Tensor | None = None, ws: torch.Tensor | None = None,
                  stream=None) -> torch.Tensor:
    """lnL[B] (fp64).  data: [2][N/2+1][2] fp64 (re, im), psd: [N/2+1] fp64."""
    B = params.shape[0]
    H = cfg.N // 2 + 1
    pp = _dev(params, torch.float64, (B, NPAR), "params")
    dp = _dev(data, torch.float64, (2, H, 2), "data")
    sp = _dev(psd, torch.float64, (H,), "psd")
    if out is None:
        out = torch.empty(B, dtype=torch.float64, device=params.device)
    op = _dev(out, torch.float64, (B,), "out")
    if ws is None:
        ws = alloc_workspace(cfg, B, params.device, with_dataset=True)
    c = cfg.c()
    _check(lib.emri_loglike_batch(pp, B, dp, sp, float(cfg.T_obs), float(cfg.dt),
                                  ctypes.byref(c), op, ws.data_ptr(), ws.numel(),
                                  _stream(stream)), "emri_loglike_batch")
    return out


def dataset_init(data: torch.Tensor, psd: torch.Tensor, cfg: Config,
                 out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    H = cfg.N // 2 + 1
    dp = _dev(data, torch.float64, (2, H, 2), "data")
    sp = _dev(psd, torch.float64, (H,), "psd")
    n = dataset_bytes(cfg)
    if out is None:
        out = torch.empty(n, dtype=torch.uint8, device=data.device)
    c = cfg.c()
    _check(lib.emri_dataset_init(dp, sp, ctypes.byref(c), out.data_ptr(), out.numel(),
                                 _stream(stream)), "emri_dataset_init")
    return out


def loglike_dataset(params: torch.Tensor, ds: torch.Tensor, cfg: Config,
                    out: torch.Tensor | None = None, ws: torch.Tensor | None = None,
                    stream=None) -> torch.Tensor:
    B = params.shape[0]
    pp = _dev(params, torch.float64, (B, NPAR), "params")
    if out is None:
        out = torch.empty(B, dtype=torch.float64, device=params.device)
    op = _dev(out, torch.float64, (B,), "out")
    if ws is None:
        ws = alloc_workspace(cfg, B, params.device)
    c = cfg.c()
    _check(lib.emri_loglike_dataset(pp, B, ds.data_ptr(), ctypes.byref(c), op, ws.data_ptr(),
                                    ws.numel(), _stream(stream)), "emri_loglike_dataset")
    return out


def loglike_dataset_noalloc(params: torch.Tensor, ds: torch.Tensor, cfg: Config,
                            out: torch.Tensor, stream=None) -> torch.Tensor:
    """emri_loglike_dataset_noalloc: the library's own device scratch array
    instead of a workspace; `out` [B] fp64 is the caller's."""
    B = params.shape[0]
    pp = _dev(params, torch.float64, (B, NPAR), "params")
    op = _dev(out, torch.float64, (B,), "out")
    c = cfg.c()
    _check(lib.emri_loglike_dataset_noalloc(pp, B, ds.data_ptr(), ctypes.byref(c), op,
                                            _stream(stream)), "emri_loglike_dataset_noalloc")
    return out


def loglike_dataset_fmg(params: torch.Tensor, coef: torch.Tensor, f_star: float,
                        ds: torch.Tensor, cfg: Config, out: torch.Tensor | None = None,
                        ws: torch.Tensor | None = None, stream=None, order: int | None = None):
    """lnL with frequency-dependent alpha_M, alpha_T: coef [B][2][P] (device,
    float64): per walker the alpha_M series coefficients, then alpha_T's."""
    B = params.shape[0]
    pp = _dev(params, torch.float64, (B, NPAR), "params")
    P = coef.shape[2] if order is None else order
    cp_ = _dev(coef, torch.float64, (B, 2, P), "coef") if coef.numel() else None
    if out is None:
        out = torch.empty(B, dtype=torch.float64, device=params.device)
    op = _dev(out, torch.float64, (B,), "out")
    if ws is None:
        ws = alloc_workspace(cfg, max(B, 1), params.device)
    c = cfg.c()
    f = _Fmg(int(P), 0, float(f_star))
    _check(lib.emri_loglike_dataset_fmg(pp, B, cp_, ctypes.byref(f), ds.data_ptr(),
                                        ctypes.byref(c), op, ws.data_ptr(), ws.numel(),
                                        _stream(stream)), "emri_loglike_dataset_fmg")
    return out


def sampler_workspace_bytes(cfg: Config, W: int) -> int:
    c = cfg.c()
    n = lib.emri_sampler_workspace_bytes(ctypes.byref(c), int(W))
    if n == 0:
        raise EmriError(-1, "emri_sampler_workspace_bytes", "invalid configuration")
    return n


def ensemble_lnprob(X: torch.Tensor, prior: _Prior, ds: torch.Tensor, cfg: Config,
                    out: torch.Tensor | None = None, ws: torch.Tensor | None = None,
                    stream=None) -> torch.Tensor:
    """Box log-prior plus log-likelihood of the walkers X[n][17]."""
    n = X.shape[0]
    xp = _dev(X, torch.float64, (n, NPAR), "X")
    if out is None:
        out = torch.empty(n, dtype=torch.float64, device=X.device)
    op = _dev(out, torch.float64, (n,), "out")
    if ws is None:
        ws = alloc_workspace(cfg, max(n, 1), X.device)
    c = cfg.c()
    _check(lib.emri_ensemble_lnprob(xp, n, ctypes.byref(prior), ds.data_ptr(), ctypes.byref(c),
                                    op, ws.data_ptr(), ws.numel(), _stream(stream)),
           "emri_ensemble_lnprob")
    return out


def stretch_step(X: torch.Tensor, lnp: torch.Tensor, prior: _Prior, a: float, u: torch.Tensor,
                 ds: torch.Tensor, cfg: Config, accepted: torch.Tensor | None = None,
                 ws: torch.Tensor | None = None, stream=None):
    """One stretch-move step of the ensemble X[2W][17], lnp[2W] (both in place);
    u[2][W][3] uniforms.  Returns accepted[2W] (int32, 1 where the walker moved)."""
    n = X.shape[0]
    if n % 2:
        raise ValueError("the ensemble must have an even number of walkers")
    W = n // 2
    xp = _dev(X, torch.float64, (n, NPAR), "X")
    lp = _dev(lnp, torch.float64, (n,), "lnp")
    up = _dev(u, torch.float64, (2, W, 3), "u")
    if accepted is None:
        accepted = torch.empty(n, dtype=torch.int32, device=X.device)
    ap = _dev(accepted, torch.int32, (n,), "accepted")
    if ws is None:
        ws = torch.empty(sampler_workspace_bytes(cfg, W), dtype=torch.uint8, device=X.device)
    c = cfg.c()
    _check(lib.emri_stretch_step(xp, lp, W, ctypes.byref(prior), float(a), up, ds.data_ptr(),
                                 ctypes.byref(c), ap, ws.data_ptr(), ws.numel(), _stream(stream)),
           "emri_stretch_step")
    return accepted


def model_batch(params: torch.Tensor, cfg: Config, out: torch.Tensor | None = None,
                ws: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """[B][2][N/2+1] complex propagated model exp(-2 pi i f DT) h~ / (Xi d_L)."""
    B = params.shape[0]
    pp = _dev(params, torch.float64, (B, NPAR), "params")
    H = cfg.N // 2 + 1
    if out is None:
        out = torch.empty((B, 2, H, 2), dtype=cfg.real_dtype, device=params.device)
    op = _dev(out, cfg.real_dtype, (B, 2, H, 2), "out")
    if ws is None:
        ws = alloc_workspace(cfg, B, params.device)
    c = cfg.c()
    _check(lib.emri_model_batch(pp, B, ctypes.byref(c), op, ws.data_ptr(), ws.numel(),
                                _stream(stream)), "emri_model_batch")
    return torch.view_as_complex(out)


def noise_psd(N: int, dt: float, model: int = 0, device="cuda", stream=None) -> torch.Tensor:
    out = torch.empty(N // 2 + 1, dtype=torch.float64, device=device)
    _check(lib.emri_noise_psd(int(model), int(N), float(dt), out.data_ptr(), _stream(stream)),
           "emri_noise_psd")
    return out


class Tracer:
    """Per-stage HIP-event timing of the library's kernels (context manager)."""

    def __init__(self):
        n = 32
        self._ms = (ctypes.c_double * n)()
        self._cnt = (ctypes.c_int64 * n)()

    def __enter__(self):
        self.read()                      # drop anything recorded before
        lib.emri_trace_enable(1)
        return self

    def __exit__(self, *exc):
        lib.emri_trace_enable(0)

    def read(self) -> dict:
        """{stage: (total_ms, launches)} since the previous read (synchronises)."""
        k = lib.emri_trace_read(self._ms, self._cnt, 32)
        out = {}
        for i in range(k):
            if self._cnt[i]:
                out[lib.emri_trace_stage_name(i).decode()] = (self._ms[i], int(self._cnt[i]))
        return out


# --------------------------------------------------------------------------
# serving loop (emri_server_*)
# --------------------------------------------------------------------------
class _ServerCfg(ctypes.Structure):
    _fields_ = [("arena", ctypes.c_void_p), ("arena_bytes", ctypes.c_size_t),
                ("n_streams", ctypes.c_int32), ("max_batch", ctypes.c_int32),
                ("use_graphs", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class _ServerStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in ("submitted", "completed", "rejected", "batches",
                                              "graph_launches", "graph_captures", "walkers",
                                              "padded_walkers")] + \
               [("arena_in_use", ctypes.c_size_t), ("arena_peak", ctypes.c_size_t)]


def _bind_server(L):
    vp, i64, u64 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint64
    sig = {
        "emri_server_create": ([ctypes.POINTER(_ServerCfg), ctypes.POINTER(vp)], ctypes.c_int),
        "emri_server_destroy": ([vp], ctypes.c_int),
        "emri_server_add_dataset": ([vp, ctypes.POINTER(_Cfg), vp, vp,
                                     ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
        "emri_server_submit": ([vp, ctypes.c_int32, vp, i64, vp, ctypes.POINTER(u64)],
                               ctypes.c_int),
        "emri_server_wait": ([vp, u64, ctypes.c_double, ctypes.POINTER(ctypes.c_double)],
                             ctypes.c_int),
        "emri_server_stats_get": ([vp, ctypes.POINTER(_ServerStats)], ctypes.c_int),
    }
    for name, (a, r) in sig.items():
        f = getattr(L, name)
        f.argtypes = a
        f.restype = r


_bind_server(lib)
EXPORTED = EXPORTED + ("emri_server_create", "emri_server_destroy", "emri_server_add_dataset",
                       "emri_server_submit", "emri_server_wait", "emri_server_stats_get")


class Server:
    """Persistent likelihood server (continuous batching, HBM admission,
    hipGraph launches).  The arena is a torch uint8 CUDA tensor that the
    server sub-allocates; it must outlive the server."""

    def __init__(self, arena: torch.Tensor, n_streams: int = 4, max_batch: int = 512,
                 use_graphs: bool = True):
        if not (arena.is_cuda and arena.dtype == torch.uint8):
            raise TypeError("arena must be a CUDA uint8 tensor")
        self._arena = arena
        c = _ServerCfg(arena.data_ptr(), arena.numel(), n_streams, max_batch,
                       1 if use_graphs else 0, 0)
        h = ctypes.c_void_p()
        _check(lib.emri_server_create(ctypes.byref(c), ctypes.byref(h)), "emri_server_create")
        self._h = h
        self._out = {}          # ticket -> host result array (kept alive until waited)

    def add_dataset(self, data: torch.Tensor, psd: torch.Tensor, cfg: Config) -> int:
        H = cfg.N // 2 + 1
        dp = _dev(data, torch.float64, (2, H, 2), "data")
        sp = _dev(psd, torch.float64, (H,), "psd")
        torch.cuda.synchronize()
        c = cfg.c()
        i = ctypes.c_int32()
        _check(lib.emri_server_add_dataset(self._h, ctypes.byref(c), dp, sp, ctypes.byref(i)),
               "emri_server_add_dataset")
        return i.value

    def submit(self, dataset: int, params) -> int:
        import numpy as np
        P = np.ascontiguousarray(params, dtype=np.float64).reshape(-1, NPAR)
        out = np.empty(P.shape[0], dtype=np.float64)
        t = ctypes.c_uint64()
        _check(lib.emri_server_submit(self._h, int(dataset), P.ctypes.data, P.shape[0],
                                      out.ctypes.data, ctypes.byref(t)), "emri_server_submit")
        self._out[t.value] = out
        return t.value

    def wait(self, ticket: int, timeout: float = -1.0):
        """(lnL[W] numpy array, latency in seconds)."""
        lat = ctypes.c_double()
        _check(lib.emri_server_wait(self._h, ticket, float(timeout), ctypes.byref(lat)),
               "emri_server_wait")
        return self._out.pop(ticket), lat.value

    def stats(self) -> dict:
        s = _ServerStats()
        _check(lib.emri_server_stats_get(self._h, ctypes.byref(s)), "emri_server_stats_get")
        return {n: getattr(s, n) for n, _ in s._fields_}

    def close(self):
        if self._h:
            _check(lib.emri_server_destroy(self._h), "emri_server_destroy")
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
