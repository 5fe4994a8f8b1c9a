"""Plain FP64 CPU oracle for the batched EMRI log-likelihood (arXiv:2311.17174).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It shares no code
with the HIP library under ``paper_2311_17174_amd``; the two meet only through
the seeded input generators of ``paper_2311_17174_amd.workloads``, which hold
none of the method's arithmetic.

The numerics live in ``emri_oracle.c`` (plain C, FP64, OpenMP over walkers);
this module compiles it with gcc and marshals numpy arrays through ctypes.

Layouts (all float64, C order):
  params  [B][17]                 parameter rows, see ``PARAM_NAMES``
  orbit   [B][K+1][10]            node values Y_k then dY/dt at t_k = k h_c
  waveform[B][2][N]               channels I and II, unit distance, GR
  spectrum[B][2][N/2+1] complex   dt * DFT of each channel, bins 0..N/2
  data    [2][N/2+1] complex      frequency-domain data
  psd     [N/2+1]                 one-sided noise PSD
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "emri_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

PARAM_NAMES = ("M", "mu", "a", "e0", "nu0", "Phi0", "gamma0", "alpha0", "cos_lambda",
               "theta_S", "phi_S", "theta_K", "phi_K", "d_L", "Xi0", "n_Xi", "alpha_T")
NPAR = 17


class _Cfg(ctypes.Structure):
    _fields_ = [("T_obs", ctypes.c_double), ("dt", ctypes.c_double), ("N", ctypes.c_int64),
                ("n_harm", ctypes.c_int32), ("coarse_log2", ctypes.c_int32),
                ("lo_only", ctypes.c_int32), ("ic_lso", ctypes.c_int32),
                ("ode", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("rtol", ctypes.c_double), ("atol", ctypes.c_double)]


@dataclass(frozen=True)
class OracleConfig:
    T_obs: float
    dt: float
    N: int
    n_harm: int
    coarse_log2: int = 10
    lo_only: bool = False
    ic_lso: bool = False      # initial conditions at the LSO, orbit integrated backward
    ode: int = 0              # 0: classical RK4 on the nodes; 1: adaptive Dormand-Prince 5(4);
                              # 2: Fehlberg 7(8), node to node
    rtol: float = 1e-10       # tolerances of the adaptive integrator
    atol: float = 1e-10

    @property
    def n_valid(self) -> int:
        return int(round(self.T_obs / self.dt))

    @property
    def n_intervals(self) -> int:
        m = 1 << self.coarse_log2
        return (self.n_valid + m - 1) // m

    def c(self) -> _Cfg:
        return _Cfg(self.T_obs, self.dt, self.N, self.n_harm, self.coarse_log2,
                    1 if self.lo_only else 0, 1 if self.ic_lso else 0, int(self.ode), 0,
                    float(self.rtol), float(self.atol))


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-Wall", "-Wno-unknown-pragmas", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int32)
        cp = ctypes.POINTER(_Cfg)
        i64 = ctypes.c_int64
        sig = {
            "oracle_scalars": ([dp, i64, dp], ctypes.c_int),
            "oracle_rhs": ([dp, dp, ctypes.c_int, dp], ctypes.c_int),
            "oracle_orbit": ([dp, i64, cp, dp, ip], ctypes.c_int),
            "oracle_orbit_steps": ([dp, i64, cp, ip], ctypes.c_int),
            "oracle_dp5_tableau": ([dp], ctypes.c_int),
            "oracle_rk78_tableau": ([dp], ctypes.c_int),
            "oracle_waveform": ([dp, i64, cp, dp], ctypes.c_int),
            "oracle_waveform_diag": ([dp, cp, dp, dp], ctypes.c_int),
            "oracle_rfft": ([dp, i64, i64, ctypes.c_double, dp], ctypes.c_int),
            "oracle_loglike": ([dp, i64, dp, dp, cp, dp], ctypes.c_int),
            "oracle_loglike_sets": ([dp, i64, dp, ctypes.c_int32, dp, cp, dp, dp], ctypes.c_int),
            "oracle_loglike_fmg": ([dp, i64, dp, ctypes.c_int32, ctypes.c_double, dp, dp, cp,
                                    dp], ctypes.c_int),
            "oracle_psd_bc04": ([dp, i64, dp], ctypes.c_int),
            "oracle_psd_rcl": ([dp, i64, ctypes.c_int32, dp], ctypes.c_int),
            "oracle_make_data": ([dp, dp, dp, dp, i64, ctypes.c_double, dp], ctypes.c_int),
            "oracle_besselj": ([ctypes.c_int, ctypes.c_double], ctypes.c_double),
            "oracle_pm_coeffs": ([ctypes.c_int, ctypes.c_double, dp], ctypes.c_int),
            "oracle_antenna": ([ctypes.c_double, ctypes.c_double, ctypes.c_double, dp], ctypes.c_int),
            "oracle_hermite": ([ctypes.c_double] * 6, ctypes.c_double),
            "oracle_dl_of_z": ([ctypes.c_double], ctypes.c_double),
            "oracle_z_of_dl": ([ctypes.c_double], ctypes.c_double),
            "oracle_num_threads": ([], ctypes.c_int),
            "oracle_stretch_propose": ([dp, i64, ctypes.c_int32, ip, ctypes.c_int32, dp, dp,
                                        ctypes.c_double, dp, dp, dp, dp], ctypes.c_int),
            "oracle_stretch_accept": ([dp, dp, i64, ctypes.c_int32, dp, dp, dp, dp, ip],
                                      ctypes.c_int),
            "oracle_ensemble_lnprob": ([dp, i64, ip, ctypes.c_int32, dp, dp, dp, dp, cp, dp],
                                       ctypes.c_int),
            "oracle_stretch_step": ([dp, dp, i64, ip, ctypes.c_int32, dp, dp, ctypes.c_double,
                                     dp, dp, dp, cp, ip], ctypes.c_int),
        }
        for name, (argt, rest) in sig.items():
            f = getattr(L, name)
            f.argtypes = argt
            f.restype = rest
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _check(rc: int, what: str):
    if rc != 0:
        raise ValueError(f"oracle {what} failed with status {rc}")


# --------------------------------------------------------------------------
# step wrappers
# --------------------------------------------------------------------------
def scalars(params) -> np.ndarray:
    """[B][8] = valid, z, Xi, chi[s], DeltaT[s], g=1/(Xi D), D[s], 0."""
    p = _f64(params).reshape(-1, NPAR)
    out = np.zeros((p.shape[0], 8))
    _check(lib().oracle_scalars(_p(p), p.shape[0], _p(out)), "scalars")
    return out


def rhs(y5, prow, lo_only: bool = False) -> np.ndarray:
    y = _f64(y5)
    pr = _f64(prow)
    dy = np.zeros(5)
    lib().oracle_rhs(_p(y), _p(pr), 1 if lo_only else 0, _p(dy))
    return dy


def orbit(params, cfg: OracleConfig):
    p = _f64(params).reshape(-1, NPAR)
    B = p.shape[0]
    orb = np.zeros((B, cfg.n_intervals + 1, 10))
    kw = np.zeros(B, dtype=np.int32)
    c = cfg.c()
    _check(lib().oracle_orbit(_p(p), B, ctypes.byref(c), _p(orb),
                              kw.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))), "orbit")
    return orb, kw


def orbit_steps(params, cfg: OracleConfig) -> np.ndarray:
    """[B][2] accepted and rejected steps of the adaptive integrators (ode=1, 2)."""
    p = _f64(params).reshape(-1, NPAR)
    out = np.zeros((p.shape[0], 2), dtype=np.int32)
    c = cfg.c()
    _check(lib().oracle_orbit_steps(_p(p), p.shape[0], ctypes.byref(c),
                                    out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))),
           "orbit_steps")
    return out


def dp5_tableau():
    """The oracle's Dormand-Prince 5(4) constants: c[7], A[7][7], b[7],
    b - b*[7] and the continuous-extension vector d[7]."""
    out = np.zeros(77)
    lib().oracle_dp5_tableau(_p(out))
    return (out[:7], out[7:56].reshape(7, 7), out[56:63], out[63:70], out[70:77])


def rk78_tableau():
    """The oracle's Fehlberg 7(8) constants: c[13], A[13][12], the order-7
    weights b7[13] and the order-8 weights b8[13]."""
    out = np.zeros(195)
    lib().oracle_rk78_tableau(_p(out))
    return out[:13], out[13:169].reshape(13, 12), out[169:182], out[182:195]


def waveform(params, cfg: OracleConfig) -> np.ndarray:
    p = _f64(params).reshape(-1, NPAR)
    B = p.shape[0]
    x = np.zeros((B, 2, cfg.N))
    c = cfg.c()
    _check(lib().oracle_waveform(_p(p), B, ctypes.byref(c), _p(x)), "waveform")
    return x


def waveform_diag(prow, cfg: OracleConfig):
    """One walker: channels [2][N] and per-sample diagnostics [N][16] =
    (h+, hx, A, c_iota, Phi', gamma, cos theta_d, phi_d, psi, beta, Phi, nu,
    gamma~, alpha, e, 0); rows past the last sample written are zero."""
    p = _f64(prow).reshape(NPAR)
    x = np.zeros((2, cfg.N))
    d = np.zeros((cfg.N, 16))
    c = cfg.c()
    _check(lib().oracle_waveform_diag(_p(p), ctypes.byref(c), _p(x), _p(d)), "waveform_diag")
    return x, d


def rfft(x, dt: float) -> np.ndarray:
    """dt * DFT of each real row (last axis), bins 0..N/2, complex128."""
    a = _f64(x)
    N = a.shape[-1]
    rows = a.reshape(-1, N)
    out = np.zeros((rows.shape[0], N // 2 + 1, 2))
    _check(lib().oracle_rfft(_p(rows), rows.shape[0], N, dt, _p(out)), "rfft")
    return (out[..., 0] + 1j * out[..., 1]).reshape(a.shape[:-1] + (N // 2 + 1,))


def spectrum(params, cfg: OracleConfig) -> np.ndarray:
    """[B][2][N/2+1] complex: unit-distance GR spectrum of each walker."""
    return rfft(waveform(params, cfg), cfg.dt)


def _cplx_pairs(z) -> np.ndarray:
    z = np.asarray(z)
    out = np.empty(z.shape + (2,))
    out[..., 0] = z.real
    out[..., 1] = z.imag
    return np.ascontiguousarray(out)


def loglike(params, data, psd, cfg: OracleConfig) -> np.ndarray:
    p = _f64(params).reshape(-1, NPAR)
    d = _cplx_pairs(data)
    s = _f64(psd)
    H = cfg.N // 2 + 1
    assert d.shape == (2, H, 2) and s.shape == (H,)
    out = np.zeros(p.shape[0])
    c = cfg.c()
    _check(lib().oracle_loglike(_p(p), p.shape[0], _p(d), _p(s), ctypes.byref(c), _p(out)),
           "loglike")
    return out


def loglike_sets(params, datasets, psd, cfg: OracleConfig, return_spectra: bool = False):
    """[B][nset]: lnL of each walker against each data set [2][N/2+1]
    complex, from one evaluation of the walker's spectrum (each entry equals
    loglike() for that data set).  With return_spectra, also the walkers'
    unit-distance GR spectra [B][2][N/2+1] complex (as spectrum())."""
    p = _f64(params).reshape(-1, NPAR)
    d = np.ascontiguousarray(np.stack([_cplx_pairs(x) for x in datasets]))
    s = _f64(psd)
    H = cfg.N // 2 + 1
    assert d.shape[1:] == (2, H, 2) and s.shape == (H,)
    out = np.zeros((p.shape[0], d.shape[0]))
    c = cfg.c()
    spec = np.zeros((p.shape[0], 2, H, 2)) if return_spectra else None
    _check(lib().oracle_loglike_sets(_p(p), p.shape[0], _p(d), d.shape[0], _p(s),
                                     ctypes.byref(c), _p(out),
                                     _p(spec) if spec is not None else None), "loglike_sets")
    if return_spectra:
        return out, spec[..., 0] + 1j * spec[..., 1]
    return out


def loglike_fmg(params, coef, f_star, data, psd, cfg: OracleConfig) -> np.ndarray:
    """lnL with frequency-dependent alpha_M, alpha_T: coef [B][2][P] (alpha_M
    series coefficients, then alpha_T's), pivot frequency f_star [Hz]."""
    p = _f64(params).reshape(-1, NPAR)
    B = p.shape[0]
    cf = np.asarray(coef, dtype=np.float64)
    P = cf.size // (2 * B)
    cf = np.ascontiguousarray(cf.reshape(B, 2, P))
    d = _cplx_pairs(data)
    s = _f64(psd)
    out = np.zeros(B)
    c = cfg.c()
    _check(lib().oracle_loglike_fmg(_p(p), B, _p(cf), P, float(f_star), _p(d), _p(s),
                                    ctypes.byref(c), _p(out)), "loglike_fmg")
    return out


def psd_bc04(f) -> np.ndarray:
    f = _f64(f)
    S = np.zeros_like(f)
    lib().oracle_psd_bc04(_p(f), f.size, _p(S))
    return S


def psd_rcl(f, confusion_years: float | None = None) -> np.ndarray:
    """Robson-Cornish-Liu sky-averaged sensitivity; confusion noise for 0.5,
    1, 2 or 4 years of observation, or none."""
    f = _f64(f)
    S = np.zeros_like(f)
    conf = -1 if confusion_years is None else {0.5: 0, 1.0: 1, 2.0: 2, 4.0: 3}[float(confusion_years)]
    _check(lib().oracle_psd_rcl(_p(f), f.size, conf, _p(S)), "psd_rcl")
    return S


def frequency_grid(N: int, dt: float) -> np.ndarray:
    return np.arange(N // 2 + 1) / (N * dt)


def make_data(hinj, pinj, psd, gauss, N: int, dt: float) -> np.ndarray:
    """data[2][N/2+1] complex = propagated injection + coloured noise."""
    h = _cplx_pairs(hinj)
    pi = _f64(pinj).reshape(NPAR)
    s = _f64(psd)
    out = np.zeros((2, N // 2 + 1, 2))
    gp = None
    if gauss is not None:
        g = _f64(gauss)
        assert g.shape == (2, N // 2 + 1, 2)
        gp = _p(g)
    _check(lib().oracle_make_data(_p(h), _p(pi), _p(s), gp, N, dt, _p(out)), "make_data")
    return out[..., 0] + 1j * out[..., 1]


def besselj(n: int, x: float) -> float:
    return lib().oracle_besselj(int(n), float(x))


def pm_coeffs(n: int, e: float):
    out = np.zeros(3)
    _check(lib().oracle_pm_coeffs(int(n), float(e), _p(out)), "pm_coeffs")
    return out


def antenna(cth: float, phi: float, psi: float):
    out = np.zeros(2)
    lib().oracle_antenna(float(cth), float(phi), float(psi), _p(out))
    return out


def hermite(y0, d0, y1, d1, h, u) -> float:
    return lib().oracle_hermite(y0, d0, y1, d1, h, u)


def dl_of_z(z: float) -> float:
    """luminosity distance in light-seconds"""
    return lib().oracle_dl_of_z(float(z))


def z_of_dl(D_seconds: float) -> float:
    return lib().oracle_z_of_dl(float(D_seconds))


def num_threads() -> int:
    return lib().oracle_num_threads()


# --------------------------------------------------------------------------
# ensemble sampler (stretch move of Goodman & Weare 2010, two-half form)
def _ip(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _prior(free_idx, lo, hi):
    fi = np.ascontiguousarray(free_idx, dtype=np.int32)
    return fi, _f64(lo), _f64(hi)


def stretch_propose(X, h, free_idx, lo, hi, a, u):
    """Proposals for half h of the ensemble X [2W][17]: (Y [W][17],
    (D-1) ln z [W], log-prior [W]); u is [W][3]."""
    X = _f64(X).reshape(-1, NPAR)
    W = X.shape[0] // 2
    fi, lo, hi = _prior(free_idx, lo, hi)
    u = _f64(u).reshape(W, 3)
    Y = np.zeros((W, NPAR))
    lnz = np.zeros(W)
    lpr = np.zeros(W)
    _check(lib().oracle_stretch_propose(_p(X), W, int(h), _ip(fi), len(fi), _p(lo), _p(hi),
                                        float(a), _p(u), _p(Y), _p(lnz), _p(lpr)), "propose")
    return Y, lnz, lpr


def stretch_accept(X, lnp, h, Y, lnpY, lnz, u):
    """Acceptance for half h; updates X [2W][17] and lnp [2W] in place and
    returns the accepted flags [2W] (entries of the other half are 0)."""
    W = X.shape[0] // 2
    acc = np.zeros(2 * W, dtype=np.int32)
    _check(lib().oracle_stretch_accept(_p(X), _p(lnp), W, int(h), _p(_f64(Y)), _p(_f64(lnpY)),
                                       _p(_f64(lnz)), _p(_f64(u).reshape(W, 3)), _ip(acc)),
           "accept")
    return acc


def ensemble_lnprob(X, free_idx, lo, hi, data, psd, cfg: OracleConfig) -> np.ndarray:
    X = _f64(X).reshape(-1, NPAR)
    fi, lo, hi = _prior(free_idx, lo, hi)
    d = _cplx_pairs(data)
    s = _f64(psd)
    out = np.zeros(X.shape[0])
    c = cfg.c()
    _check(lib().oracle_ensemble_lnprob(_p(X), X.shape[0], _ip(fi), len(fi), _p(lo), _p(hi),
                                        _p(d), _p(s), ctypes.byref(c), _p(out)), "lnprob")
    return out


def stretch_step(X, lnp, free_idx, lo, hi, a, u, data, psd, cfg: OracleConfig):
    """One step of the ensemble X [2W][17] with log-posteriors lnp [2W];
    u [2][W][3].  Returns (X, lnp, accepted) as new arrays."""
    X = _f64(X).reshape(-1, NPAR).copy()
    lnp = _f64(lnp).copy()
    W = X.shape[0] // 2
    fi, lo, hi = _prior(free_idx, lo, hi)
    d = _cplx_pairs(data)
    s = _f64(psd)
    acc = np.zeros(2 * W, dtype=np.int32)
    c = cfg.c()
    _check(lib().oracle_stretch_step(_p(X), _p(lnp), W, _ip(fi), len(fi), _p(lo), _p(hi),
                                     float(a), _p(_f64(u).reshape(2, W, 3)), _p(d), _p(s),
                                     ctypes.byref(c), _ip(acc)), "stretch step")
    return X, lnp, acc
