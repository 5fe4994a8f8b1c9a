"""Shared helpers of the GPU parity tests: oracle-side inputs and expected
values (computed only by the CPU oracle), and the HIP binding."""
from __future__ import annotations

import hashlib
import json
import os
import sys

import numpy as np

import oracle as O
from paper_2311_17174_amd import workloads as W

EPS64 = 2.0 ** -52
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def ocfg(w) -> O.OracleConfig:
    return O.OracleConfig(T_obs=w.T_obs, dt=w.dt, N=w.N, n_harm=w.n_harm,
                          coarse_log2=w.coarse_log2, ic_lso=bool(w.ic), ode=w.ode,
                          rtol=w.ode_rtol, atol=w.ode_atol)


_DATA_CACHE: dict = {}
_SPEC_CACHE: dict = {}


def _key(w):
    return (w.T_obs, w.dt, w.N, w.n_harm, w.coarse_log2, w.inj.tobytes(), w.ic, w.ode,
            w.ode_rtol, w.ode_atol)


def oracle_injection_spectrum(w):
    """the oracle's unit-distance GR spectrum [2][N/2+1] of w's injection"""
    k = _key(w)
    if k not in _SPEC_CACHE:
        _SPEC_CACHE[k] = O.spectrum(w.inj[None], ocfg(w))[0]
    return _SPEC_CACHE[k]


def oracle_dataset(w, noise: bool = True):
    """(data[2][N/2+1] complex, psd[N/2+1]) for workload w, from the oracle:
    the propagated injection, plus coloured noise from w.noise_seed."""
    key = _key(w) + (w.noise_seed, noise)
    if key not in _DATA_CACHE:
        f = W.frequencies(w.N, w.dt)
        S = O.psd_bc04(f)
        g = W.gaussian_draws(w.N, w.noise_seed) if noise else None
        d = O.make_data(oracle_injection_spectrum(w), w.inj, S, g, w.N, w.dt)
        _DATA_CACHE[key] = (d, S)
    return _DATA_CACHE[key]


def golden(name: str) -> dict:
    """per-walker oracle values written by tests/golden/make_golden.py"""
    with open(os.path.join(GOLDEN, f"{name}_lnl.json")) as f:
        return json.load(f)


def data_fingerprint(d) -> str:
    return hashlib.sha256(np.ascontiguousarray(d, dtype=np.complex128).tobytes()).hexdigest()


def to_device_data(d, S):
    import torch
    dd = torch.view_as_real(torch.from_numpy(np.ascontiguousarray(d))).contiguous().cuda()
    ss = torch.from_numpy(np.ascontiguousarray(S)).cuda()
    return dd, ss


def max_phase(w, P) -> float:
    """largest Doppler-shifted orbital phase reached, for rounding tolerances"""
    orb, kw = O.orbit(P, ocfg(w))
    return float(np.max(np.abs(orb[..., 0]))) + 10.0
