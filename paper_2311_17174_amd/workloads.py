"""Seeded synthetic workloads for the batched EMRI log-likelihood.

This module holds the workload definitions (sizes, injections) and the seeded
random draws that both the HIP path and the CPU oracle consume.  It contains
none of the method's arithmetic: no waveform, transform, noise colouring or
likelihood is computed here.  Randomness the method needs (Gaussian noise
draws) is produced here and passed in as an input.

Parameter rows follow the C ABI (17 doubles per walker):
  0 M [Msun]  1 mu [Msun]  2 a = S/M^2  3 e0  4 nu0 [Hz]  5 Phi0  6 gamma~0
  7 alpha0  8 cos(lambda)  9 theta_S  10 phi_S  11 theta_K  12 phi_K [rad]
  13 d_L [Gpc]  14 Xi0  15 n  16 alpha_T (c_T^2 = 1 + alpha_T; GR: 0)
The first three entries are the masses and the spin, as the paper's code
convention requires (Sec. 3, "Extending the parameters in the MCMC run").
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace

import numpy as np

NPAR = 17
YEAR = 31557600.0          # Julian year [s]
DAY = 86400.0

# relative perturbation scale per parameter: 1e-5 on the masses and nu0,
# 1e-3 on the others; alpha_T is never perturbed (the GR value is 0, and any
# perturbation of the GW speed at the 1e-3 level is a delay of ~1e14 s).
SIGMA_REL = np.array([1e-5, 1e-5, 1e-3, 1e-3, 1e-5, 1e-3, 1e-3, 1e-3, 1e-3, 1e-3,
                      1e-3, 1e-3, 1e-3, 1e-3, 1e-3, 1e-3, 0.0])


def injection(**kw) -> np.ndarray:
    """Fiducial parameter row; keyword overrides by name."""
    base = dict(M=1e6, mu=10.0, a=0.5, e0=0.3, nu0=1e-3, Phi0=1.0, gamma0=1.0, alpha0=1.0,
                cos_lambda=0.5, theta_S=0.8, phi_S=0.8, theta_K=0.8, phi_K=0.8, d_L=1.0,
                Xi0=1.0, n_Xi=0.0, alpha_T=0.0)
    names = list(base)
    for k, v in kw.items():
        if k not in base:
            raise KeyError(k)
        base[k] = v
    return np.array([base[n] for n in names], dtype=np.float64)


@dataclass(frozen=True)
class Workload:
    name: str
    B: int
    T_obs: float
    dt: float
    N: int
    n_harm: int
    coarse_log2: int
    precision: str                    # "fp64" or "mixed"
    inj: np.ndarray = field(compare=False, repr=False, default=None)
    walker_seed: int = 0
    noise_seed: int = 1
    ic: int = 0                       # 1: the orbital state of a row is at the LSO
    ode: int = 0                      # 0: RK4 on the coarse nodes; 1: adaptive DP5(4)
    ode_rtol: float = 1e-12           # tolerances of the adaptive integrator
    ode_atol: float = 1e-12

    @property
    def n_valid(self) -> int:
        return int(round(self.T_obs / self.dt))

    @property
    def n_intervals(self) -> int:
        m = 1 << self.coarse_log2
        return (self.n_valid + m - 1) // m

    def with_(self, **kw) -> "Workload":
        return replace(self, **kw)


def config1() -> Workload:
    """Plain FP64, B=32, 30 days at dt=10 s padded to 2^18, 16 harmonics, GR."""
    return Workload("cfg1_fp64_B32_30d_2p18", 32, 30 * DAY, 10.0, 1 << 18, 16, 10, "fp64",
                    injection())


def config2() -> Workload:
    """Plain FP64, B=256, 1 yr at dt=10 s padded to 2^22, 30 harmonics, Xi0=0.9, n=2."""
    return Workload("cfg2_fp64_B256_1yr_2p22", 256, YEAR, 10.0, 1 << 22, 30, 10, "fp64",
                    injection(Xi0=0.9, n_Xi=2.0))


def config3() -> Workload:
    """Mixed precision, same shape and inputs as config2."""
    return config2().with_(name="cfg3_mixed_B256_1yr_2p22", precision="mixed")


def config5(precision: str = "mixed") -> Workload:
    """Stress: B=1024, 2 yr at dt=5 s padded to 2^24, 40 harmonics."""
    return Workload(f"cfg5_{precision}_B1024_2yr_2p24", 1024, 2 * YEAR, 5.0, 1 << 24, 40, 11,
                    precision, injection(e0=0.5, a=0.9, Xi0=0.8, n_Xi=3.0))


def small(precision: str = "fp64", B: int = 8, days: float = 2.5, n_harm: int = 8,
          N: int = 1 << 15, **inj) -> Workload:
    """Oracle-sized case: a few coarse intervals plus a ragged tail."""
    return Workload(f"small_{precision}_B{B}", B, days * DAY, 10.0, N, n_harm, 10, precision,
                    injection(**inj))


def walkers(w: Workload, B: int | None = None, seed: int | None = None,
            sigma: np.ndarray | None = None) -> np.ndarray:
    """[B][17]: walker 0 is the injection, walker i>0 is inj*(1 + sigma*eps_i)
    with eps ~ N(0,1) from PCG64(seed), drawn row-major [B][17]."""
    B = w.B if B is None else B
    seed = w.walker_seed if seed is None else seed
    sigma = SIGMA_REL if sigma is None else np.asarray(sigma, dtype=np.float64)
    eps = np.random.Generator(np.random.PCG64(seed)).standard_normal((B, NPAR))
    P = np.tile(w.inj, (B, 1)) * (1.0 + sigma[None, :] * eps)
    P[0] = w.inj
    return np.ascontiguousarray(P)


def gaussian_draws(N: int, seed: int) -> np.ndarray:
    """Standard normal draws [2][N/2+1][2] (channel, bin, re/im) from PCG64(seed)."""
    g = np.random.Generator(np.random.PCG64(seed)).standard_normal((2, N // 2 + 1, 2))
    return np.ascontiguousarray(g)


def frequencies(N: int, dt: float) -> np.ndarray:
    """f_k = k / (N dt), k = 0..N/2."""
    return np.arange(N // 2 + 1, dtype=np.float64) / (N * dt)


# ---------------------------------------------------------------------------
# serving workload: several concurrent chains issuing likelihood requests
# ---------------------------------------------------------------------------
SERVING_T_OBS_YR = (0.5, 1.0, 2.0)          # 2^21, 2^22, 2^23 samples at 10 s


def serving_chains(n_chains: int = 8):
    """Injection row of each chain c, drawn from PCG64(100 + c): e0 ~ U[0.05,
    0.5], a ~ U[0, 0.9], log10 M ~ U[log10 3e5, log10 3e6], mu = 10, the other
    entries as config 1 (GR).  The serving workloads put the orbital state of a
    row at the last stable orbit (``ic = 1``, the paper's convention: e0 is the
    eccentricity at the LSO, the orbit is integrated backward over the window
    and nu0 is not used), so every drawn mass has a valid history."""
    rows = []
    for c in range(n_chains):
        r = np.random.Generator(np.random.PCG64(100 + c))
        e0 = r.uniform(0.05, 0.5)
        a = r.uniform(0.0, 0.9)
        M = 10.0 ** r.uniform(np.log10(3e5), np.log10(3e6))
        rows.append(injection(M=M, mu=10.0, a=a, e0=e0))
    return np.array(rows)


def serving_workload(chain_inj: np.ndarray, t_index: int, precision: str = "mixed") -> Workload:
    T = SERVING_T_OBS_YR[t_index] * YEAR
    N = 1 << (21 + t_index)
    return Workload(f"serve_T{SERVING_T_OBS_YR[t_index]}yr", 0, T, 10.0, N, 30, 10, precision,
                    chain_inj, ic=1)


def serving_requests(n: int, n_chains: int = 8, seed: int = 4, w_min: int = 16,
                     w_max: int = 512):
    """Request schedule: (gap in units of the mean inter-arrival time, chain,
    T_obs index, walkers W, walker seed = request id); Poisson arrivals."""
    r = np.random.Generator(np.random.PCG64(seed))
    gaps = r.exponential(1.0, n)
    chains = r.integers(0, n_chains, n)
    tidx = r.integers(0, len(SERVING_T_OBS_YR), n)
    Ws = r.integers(w_min, w_max + 1, n)
    return [(float(gaps[i]), int(chains[i]), int(tidx[i]), int(Ws[i]), i) for i in range(n)]


# ---------------------------------------------------------------------------
# ensemble sampler inputs: prior box, initial ensemble, uniforms
# ---------------------------------------------------------------------------
# free parameters of the sampler workloads: the masses, spin, eccentricity,
# frequency, distance and the two propagation parameters Xi0 and n
SAMPLER_FREE = (0, 1, 2, 3, 4, 13, 14, 15)


def sampler_prior(w: Workload, free_idx=SAMPLER_FREE, width: float = 50.0):
    """Box of the free parameters: inj[i] (1 -/+ width SIGMA_REL[i]), or
    -/+ width 1e-3 around an injected 0.  Returns (lo, hi) in free order."""
    lo, hi = [], []
    for i in free_idx:
        v, s = w.inj[i], SIGMA_REL[i] if SIGMA_REL[i] > 0 else 1e-3
        half = width * s * (abs(v) if v != 0 else 1.0)
        lo.append(v - half)
        hi.append(v + half)
    return np.array(lo), np.array(hi)


def sampler_ensemble(w: Workload, W: int, free_idx=SAMPLER_FREE, seed: int = 7) -> np.ndarray:
    """Initial ensemble [2W][17]: the injection, with the free parameters of
    each walker drawn as in walkers(w, 2W, seed)."""
    P = walkers(w, 2 * W, seed)
    X = np.tile(w.inj, (2 * W, 1))
    X[:, list(free_idx)] = P[:, list(free_idx)]
    return np.ascontiguousarray(X)


def sampler_uniforms(W: int, steps: int, seed: int = 11) -> np.ndarray:
    """Uniforms in [0, 1) [steps][2][W][3] from PCG64(seed): per walker the
    partner, stretch and acceptance draws of each step's two halves."""
    return np.random.Generator(np.random.PCG64(seed)).random((steps, 2, W, 3))
