"""Shared helpers of the GPU parity tests: oracle-side inputs and expected
values (computed only by the CPU oracle), and the HIP binding."""
from __future__ import annotations

import sys

import numpy as np

import oracle as O
from paper_2311_17174_amd import workloads as W

EPS64 = 2.0 ** -52


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def ocfg(w) -> O.OracleConfig:
    return O.OracleConfig(T_obs=w.T_obs, dt=w.dt, N=w.N, n_harm=w.n_harm,
                          coarse_log2=w.coarse_log2, ic_lso=bool(w.ic), ode=w.ode,
                          rtol=w.ode_rtol, atol=w.ode_atol)


_DATA_CACHE: dict = {}


def oracle_dataset(w, noise: bool = True):
    """(data[2][N/2+1] complex, psd[N/2+1]) for workload w, from the oracle."""
    key = (w.T_obs, w.dt, w.N, w.n_harm, w.coarse_log2, w.noise_seed, w.inj.tobytes(), noise,
           w.ic, w.ode, w.ode_rtol, w.ode_atol)
    if key not in _DATA_CACHE:
        _DATA_CACHE[key] = _oracle_dataset(w, noise)
    return _DATA_CACHE[key]


def _oracle_dataset(w, noise):
    cfg = ocfg(w)
    f = W.frequencies(w.N, w.dt)
    S = O.psd_bc04(f)
    hinj = O.spectrum(w.inj[None], cfg)[0]
    g = W.gaussian_draws(w.N, w.noise_seed) if noise else None
    d = O.make_data(hinj, w.inj, S, g, w.N, w.dt)
    return d, S


def to_device_data(d, S):
    import torch
    dd = torch.view_as_real(torch.from_numpy(np.ascontiguousarray(d))).contiguous().cuda()
    ss = torch.from_numpy(np.ascontiguousarray(S)).cuda()
    return dd, ss


def max_phase(w, P) -> float:
    """largest Doppler-shifted orbital phase reached, for rounding tolerances"""
    orb, kw = O.orbit(P, ocfg(w))
    return float(np.max(np.abs(orb[..., 0]))) + 10.0
