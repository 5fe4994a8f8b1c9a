"""Write the oracle's per-walker log-likelihoods at full size.

Calls only ``oracle`` and the seeded input generators of
``paper_2311_17174_amd.workloads``; nothing here comes from the HIP path.

For each workload, every listed walker is evaluated (one oracle spectrum per
walker) against three data sets on the same frequency grid and noise PSD:

  noisy      propagated injection + coloured Gaussian noise (the bench's data)
  noiseless  the propagated injection alone
  zero       d = 0, so lnL = -<m|m>/2 with m the walker's propagated model

The likelihood is Eq. (8) with the inner product of Eq. (7) over bins
1..N/2-1 of both channels.  ``mm`` = <m|m> per walker sets the scale of the
signal part of lnL, against which the parity tests state their tolerances.
``data_sha256`` fingerprints the oracle's noisy data so that a test detects
stale values.

Usage:  python tests/golden/make_golden.py [cfg2] [cfg5]
Writes tests/golden/<workload>_lnl.json.
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle as O                                   # noqa: E402
from paper_2311_17174_amd import workloads as W      # noqa: E402

# seeded subset of the 1024 stress walkers checked against the oracle
CFG5_SUBSET_SEED = 5
CFG5_SUBSET = 64


def ocfg(w) -> O.OracleConfig:
    return O.OracleConfig(T_obs=w.T_obs, dt=w.dt, N=w.N, n_harm=w.n_harm,
                          coarse_log2=w.coarse_log2, ic_lso=bool(w.ic), ode=w.ode,
                          rtol=w.ode_rtol, atol=w.ode_atol)


def cfg5_subset() -> np.ndarray:
    """Walker 0 (the injection) plus 63 others drawn from PCG64(5)."""
    r = np.random.Generator(np.random.PCG64(CFG5_SUBSET_SEED))
    rest = r.choice(np.arange(1, 1024), CFG5_SUBSET - 1, replace=False)
    return np.sort(np.concatenate([[0], rest])).astype(np.int64)


def data_fingerprint(d: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(d, dtype=np.complex128).tobytes()).hexdigest()


def datasets(w):
    """(noisy, noiseless, zero, psd) from the oracle's injection spectrum."""
    cfg = ocfg(w)
    S = O.psd_bc04(W.frequencies(w.N, w.dt))
    hinj = O.spectrum(w.inj[None], cfg)[0]
    noisy = O.make_data(hinj, w.inj, S, W.gaussian_draws(w.N, w.noise_seed), w.N, w.dt)
    clean = O.make_data(hinj, w.inj, S, None, w.N, w.dt)
    zero = np.zeros_like(clean)
    return noisy, clean, zero, S


def golden(w, idx: np.ndarray) -> dict:
    t0 = time.time()
    P = W.walkers(w)[idx]
    noisy, clean, zero, S = datasets(w)
    print(f"[golden] {w.name}: data in {time.time() - t0:.1f} s; {len(idx)} walkers on "
          f"{O.num_threads()} threads", flush=True)
    out = np.empty((len(idx), 3))
    chunk = max(1, O.num_threads())
    for s in range(0, len(idx), chunk):
        out[s:s + chunk] = O.loglike_sets(P[s:s + chunk], [noisy, clean, zero], S, ocfg(w))
        print(f"[golden] {w.name}: {min(s + chunk, len(idx))}/{len(idx)} walkers, "
              f"{time.time() - t0:.0f} s", flush=True)
    return {
        "_source": "oracle/ (FP64 C) via tests/golden/make_golden.py; Eq. (8) with the "
                   "inner product of Eq. (7), bins 1..N/2-1, channels I and II",
        "workload": w.name, "B": w.B, "N": w.N, "n_harm": w.n_harm, "dt": w.dt,
        "T_obs": w.T_obs, "walker_seed": w.walker_seed, "noise_seed": w.noise_seed,
        "data_sha256": data_fingerprint(noisy),
        "idx": [int(i) for i in idx],
        "lnl_noisy": [float(v) for v in out[:, 0]],
        "lnl_noiseless": [float(v) for v in out[:, 1]],
        "mm": [float(-2.0 * v) for v in out[:, 2]],
        "oracle_seconds": round(time.time() - t0, 1),
    }


def main(argv):
    which = argv or ["cfg2", "cfg5"]
    for name in which:
        if name == "cfg2":
            w, idx = W.config2(), np.arange(256)
        elif name == "cfg5":
            w, idx = W.config5("fp64"), cfg5_subset()
        else:
            raise SystemExit(f"unknown workload {name}")
        g = golden(w, idx)
        path = os.path.join(HERE, f"{w.name}_lnl.json")
        with open(path, "w") as f:
            json.dump(g, f, indent=1)
            f.write("\n")
        print(f"[golden] wrote {path}", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
