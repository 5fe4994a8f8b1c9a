#!/usr/bin/env python3
"""Benchmark of the batched AK EMRI log-likelihood on one MI355X.

A step is one emri_loglike_batch call over the whole batch: per-walker
scalars and RK4 orbit, amplitude tables, waveform synthesis with the LISA
response, FFT, and the noise-weighted inner product (data and PSD resident in
HBM).  The workload is 256 walkers around the 1-yr injection, 2^22 samples,
30 harmonics, FP64 ("value"); the same inputs on the mixed-precision path are
reported beside it.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps 10] [--warmup 2]

The JSON line also carries the serving loop (mixed precision, 8 chains with
resident data at 0.5/1/2 yr, Poisson arrivals at 0.8x the saturated rate):
request latency p50/p99 and served lnL evals/s.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
FP64_VECTOR_TFLOPS = 78.6      # MI355X vector FP64
FP32_VECTOR_TFLOPS = 157.3     # MI355X vector FP32 (published, packed)


def synth_flops_per_sample(n_harm: int) -> int:
    """Algorithmic floating-point operations of one waveform sample (both
    channels), counted from the kernel's arithmetic: per harmonic three cubic
    amplitude polynomials (3 x 6), three accumulations (3 x 2) and the
    three-term recurrence to the next harmonic's cos and sin (2 x 2); per
    sample the four orbital Hermite cubics (4 x 6), the azimuth rotation
    (12), the Doppler phase (6), three sin/cos pairs (3 x 20, counted as 20
    each), the orientation and detector geometry with three double-angle
    pairs (~130) and the projection (14)."""
    return 28 * n_harm + 24 + 12 + 6 + 60 + 130 + 14


def stage_work(stage: str, B: int, w, esz: int, valid_samples: int):
    """(kind, amount per launch) of algorithmic work of one stage."""
    N = w.N
    if stage == "synthesis":
        return "flop", valid_samples * synth_flops_per_sample(w.n_harm)
    if stage == "fft_columns":
        # read the valid samples (the zero tail is not read), write the whole signal
        return "byte", (valid_samples + B * N) * esz
    if stage == "fft_rows":
        return "byte", 2 * B * N * esz
    if stage == "inner_product":
        # the column-transformed signal, and the per-bin data and weight
        # arrays once (every bin of the packed spectrum)
        dsz = N * esz + N * (8 if esz == 16 else 4)
        return "byte", B * N * esz + dsz
    return None, 0


def profiled_traffic(stage: str):
    """HBM bytes per launch of `stage` from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE, scaled by a plain copy of known size),
    or None when the summary is missing or the kernel's sources have changed
    since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "hbm_traffic_B256_2p22_fp64.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    try:
        block = text.split("```json", 1)[1].split("```", 1)[0]
        rec = json.loads(block)["kernels"].get(stage)
    except (IndexError, ValueError, KeyError):
        return None
    if not rec:
        return None
    files = {"synth": "synth.hip", "fft": "fft.hip", "fft_lds": "fft_lds.hpp", "like": "like.hip",
             "walker": "walker.hip"}
    for key, want in rec["source_sha256_16"].items():
        src = os.path.join(ROOT, "paper_2311_17174_amd", "csrc", files[key])
        if hashlib.sha256(open(src, "rb").read()).hexdigest()[:16] != want:
            return None
    return rec["traffic_bytes"]


def plain_copy_gbs(gib: int = 4, reps: int = 5) -> float:
    """Read + write rate of a plain device-to-device copy of `gib` GiB (HIP
    events), the practical HBM ceiling next to the 8 TB/s peak."""
    import torch
    n = (gib << 30) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    torch.cuda.empty_cache()
    return 2.0 * (gib << 30) / (ms * 1e-3) / 1e9


def run_path(E, W, w, P, data, psd, steps, warmup):
    import torch
    cfg = E.Config.from_workload(w)
    ws = E.alloc_workspace(cfg, w.B, "cuda", with_dataset=True)
    Pd = torch.from_numpy(P).cuda()
    out = torch.empty(w.B, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        E.loglike_batch(Pd, data, psd, cfg, out=out, ws=ws)
    torch.cuda.synchronize()
    lat = []
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    with E.Tracer() as tr:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps):
            ev[i][0].record(stream)
            E.loglike_batch(Pd, data, psd, cfg, out=out, ws=ws)
            ev[i][1].record(stream)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        stages = tr.read()
    lat = [a.elapsed_time(b) for a, b in ev]
    return (t1 - t0), stages, np.array(lat), out.cpu().numpy()


def noise_weighted_mismatch(a, b, psd, df):
    """1 - <a|b> / sqrt(<a|a><b|b>) per walker, <a|b> = 4 df sum_{I,II}
    sum_{k=1}^{N/2-1} Re(conj(a) b) / S_k (no maximisation over time or
    phase).  a, b: [W][2][N/2+1] complex (device), psd [N/2+1]."""
    import torch
    a = a.to(torch.complex128)[..., 1:-1]
    b = b.to(torch.complex128)[..., 1:-1]
    w = (4.0 * df / psd[1:-1]).to(torch.float64)

    def ip(x, y):
        return ((x.conj() * y).real * w).sum(dim=(1, 2))

    m = 1.0 - ip(a, b) / torch.sqrt(ip(a, a) * ip(b, b))
    return m.cpu().numpy()


def run_config5(E, W, steps: int, warmup: int, ws_gib: float):
    """Stress configuration: 1024 walkers, 2 yr at dt = 5 s (2^24 samples),
    40 harmonics; the workspace holds a fraction of the batch, so the call
    runs in HBM-admitted chunks.  FP64 and mixed on the same inputs."""
    import torch
    out = {}
    w5 = W.config5("fp64")
    P = torch.from_numpy(W.walkers(w5)).cuda()
    cfg = E.Config.from_workload(w5)
    psd = E.noise_psd(w5.N, w5.dt)
    minj = E.model_batch(torch.from_numpy(w5.inj[None]).cuda(), cfg)[0]
    g = torch.from_numpy(W.gaussian_draws(w5.N, w5.noise_seed)).cuda()
    sig = torch.sqrt(psd * (w5.N * w5.dt / 4.0))
    sig[0] = 0.0
    sig[-1] = 0.0
    data = (torch.view_as_real(minj).clone() + sig[None, :, None] * g).contiguous()
    del minj, g, sig
    # share of the window after the injection's plunge (zero samples)
    h = E.waveform_batch(torch.from_numpy(w5.inj[None]).cuda(), cfg)[0]
    nz = torch.nonzero(h.abs().sum(dim=1)).max().item() + 1
    del h
    ws = torch.empty(int(ws_gib * (1 << 30)), dtype=torch.uint8, device="cuda")
    lnl = {}
    for prec in ("fp64", "mixed"):
        w = W.config5(prec)
        c = E.Config.from_workload(w)
        per = E.workspace_bytes(c, 1)
        chunk = 1
        while chunk < w.B and E.workspace_bytes(c, 2 * chunk) + E.dataset_bytes(c) + 256 <= ws.numel():
            chunk *= 2
        res = torch.empty(w.B, dtype=torch.float64, device="cuda")
        for _ in range(warmup):
            E.loglike_batch(P, data, psd, c, out=res, ws=ws)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            E.loglike_batch(P, data, psd, c, out=res, ws=ws)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        lnl[prec] = res.cpu().numpy()
        out[prec] = {"value": w.B / dt, "unit": "lnL evals/s", "ms_per_step": 1e3 * dt,
                     "walkers_per_chunk_at_least": chunk,
                     "workspace_gib": ws.numel() / 2 ** 30,
                     "workspace_per_walker_mib": per / 2 ** 20}
    rel = np.abs(lnl["mixed"] - lnl["fp64"]) / np.abs(lnl["fp64"])
    out.update({"workload": w5.name, "walkers": w5.B, "samples": w5.N, "n_harm": w5.n_harm,
                "dt": w5.dt, "injection_zero_tail_fraction": 1.0 - nz / w5.N,
                "mixed_vs_fp64_max_rel_dlnL": float(rel.max()), "steps": steps})
    del ws, data
    torch.cuda.empty_cache()
    return out


def run_sampler(E, W, w, data, psd, steps: int, warmup: int, fi=None):
    """Ensemble sampler on the likelihood's workload: 2W walkers with W the
    workload's batch, so each half is one batch; stretch scale 2, box prior on
    the free parameters fi (default: those of the sampler workloads).  The
    uniforms of every step are resident before the timed steps."""
    import torch
    Wh = w.B
    fi = W.SAMPLER_FREE if fi is None else tuple(fi)
    lo, hi = W.sampler_prior(w, fi)
    cfg = E.Config.from_workload(w)
    prior = E.make_prior(fi, lo, hi)
    ds = E.dataset_init(data, psd, cfg)
    X = torch.from_numpy(W.sampler_ensemble(w, Wh, fi)).cuda()
    U = torch.from_numpy(W.sampler_uniforms(Wh, warmup + steps)).cuda()
    ws = torch.empty(E.sampler_workspace_bytes(cfg, Wh), dtype=torch.uint8, device="cuda")
    lnp = E.ensemble_lnprob(X, prior, ds, cfg, ws=ws)
    acc = torch.empty(2 * Wh, dtype=torch.int32, device="cuda")
    for i in range(warmup):
        E.stretch_step(X, lnp, prior, 2.0, U[i], ds, cfg, accepted=acc, ws=ws)
    n_acc = torch.zeros((), dtype=torch.int64, device="cuda")
    torch.cuda.synchronize()
    with E.Tracer() as tr:
        t0 = time.perf_counter()
        for i in range(steps):
            E.stretch_step(X, lnp, prior, 2.0, U[warmup + i], ds, cfg, accepted=acc, ws=ws)
            n_acc += acc.sum()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        stages = tr.read()
    dt = (t1 - t0) / steps
    own = stages.get("sampler", (0.0, 0))[0] / steps
    return {"workload": w.name, "walkers": 2 * Wh, "free_parameters": len(fi),
            "stretch_scale": 2.0, "steps": steps, "ms_per_step": 1e3 * dt,
            "steps_per_s": 1.0 / dt, "lnL_evals_per_s": 2 * Wh / dt,
            "sampler_kernels_ms_per_step": own, "sampler_kernels_share": own / (1e3 * dt),
            "acceptance_fraction": float(n_acc.item()) / (2 * Wh * steps),
            "finite_lnp_walkers": int(torch.isfinite(lnp).sum().item())}


def run_fmg(E, W, w, data, psd, steps: int, warmup: int):
    """Likelihood with frequency-dependent alpha_M, alpha_T (three series
    terms per walker, pivot 10 mHz) on the same walkers and data as the main
    line, against the constant-propagation path on the resident data set."""
    import torch
    cfg = E.Config.from_workload(w)
    ds = E.dataset_init(data, psd, cfg)
    P = torch.from_numpy(W.walkers(w)).cuda()
    C = np.zeros((w.B, 2, 3))
    C[:, 0] = [0.1, 0.05, 0.01]
    C[:, 1] = [1e-15, 5e-16, 1e-16]
    coef = torch.from_numpy(C).cuda()
    ws = E.alloc_workspace(cfg, w.B)
    out = torch.empty(w.B, dtype=torch.float64, device="cuda")
    res = {}
    for name, call in (("constant", lambda: E.loglike_dataset(P, ds, cfg, out=out, ws=ws)),
                       ("fmg", lambda: E.loglike_dataset_fmg(P, coef, 1e-2, ds, cfg, out=out,
                                                             ws=ws))):
        for _ in range(warmup):
            call()
        torch.cuda.synchronize()
        with E.Tracer() as tr:
            t0 = time.perf_counter()
            for _ in range(steps):
                call()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            st = tr.read()
        res[name] = {"value": steps * w.B / (t1 - t0), "ms_per_step": 1e3 * (t1 - t0) / steps,
                     "inner_product_ms": st["inner_product"][0] / steps}
    res.update({"unit": "lnL evals/s", "workload": w.name, "series_terms": 3, "f_star_hz": 1e-2,
                "fmg_over_constant_step": res["fmg"]["ms_per_step"] / res["constant"]["ms_per_step"]})
    return res


def run_dp5(E, W, w, data, psd, steps: int, warmup: int, rtol: float = 1e-12):
    """The adaptive orbit integrators against the classical RK4 path: the
    Dormand-Prince 5(4) pair (continuous extension at the coarse nodes) and
    Fehlberg's 7(8) pair (order 7 kept, stepped node to node), both at
    tolerance rtol, on the same walkers and resident data as the main line,
    with the state at t = 0 and at the LSO (both in the orbit-segment
    pipeline)."""
    import torch
    P = torch.from_numpy(W.walkers(w)).cuda()
    out = torch.empty(w.B, dtype=torch.float64, device="cuda")
    res = {}
    lnl = {}
    for ic, tag in ((0, ""), (1, "_lso")):
        for name, wk in (("rk4", w), ("dp5", w.with_(ode=1, ode_rtol=rtol, ode_atol=rtol)),
                         ("rk78", w.with_(ode=2, ode_rtol=rtol, ode_atol=rtol))):
            cfg = E.Config.from_workload(wk.with_(ic=ic))
            ds = E.dataset_init(data, psd, cfg)
            ws = E.alloc_workspace(cfg, w.B)
            for _ in range(warmup):
                E.loglike_dataset(P, ds, cfg, out=out, ws=ws)
            torch.cuda.synchronize()
            with E.Tracer() as tr:
                t0 = time.perf_counter()
                for _ in range(steps):
                    E.loglike_dataset(P, ds, cfg, out=out, ws=ws)
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                st = tr.read()
            lnl[name + tag] = out.cpu().numpy().copy()
            res[name + tag] = {"value": steps * w.B / (t1 - t0),
                               "ms_per_step": 1e3 * (t1 - t0) / steps,
                               "orbit_ms_per_step": st["walker_setup"][0] / steps}
            del ds, ws
    res.update({"unit": "lnL evals/s", "workload": w.name, "rtol": rtol, "atol": rtol,
                "max_abs_dlnL_vs_rk4": float(np.max(np.abs(lnl["dp5"] - lnl["rk4"]))),
                "max_abs_dlnL_rk78_vs_rk4": float(np.max(np.abs(lnl["rk78"] - lnl["rk4"]))),
                "max_abs_dlnL_rk78_vs_dp5": float(np.max(np.abs(lnl["rk78"] - lnl["dp5"]))),
                "orbit_speedup": res["rk4"]["orbit_ms_per_step"] / res["dp5"]["orbit_ms_per_step"],
                "orbit_speedup_lso": (res["rk4_lso"]["orbit_ms_per_step"]
                                      / res["dp5_lso"]["orbit_ms_per_step"])})
    return res


def run_serving(E, W, n_burst: int, n_requests: int, arena_gib: float, n_streams: int,
                max_batch: int, n_sweep: int = 0):
    """Serving loop (mixed precision): 8 chains x 3 observation times of
    resident data, Poisson request arrivals at 0.8x the saturated rate
    measured first with a burst, then n_sweep requests each at 0.5x and
    1.0x; returns the report dict."""
    import threading
    import queue
    import torch
    chains = W.serving_chains()
    arena = torch.empty(int(arena_gib * (1 << 30)), dtype=torch.uint8, device="cuda")
    srv = E.Server(arena, n_streams=n_streams, max_batch=max_batch, use_graphs=True)
    ids = {}
    for c in range(len(chains)):
        for t in range(len(W.SERVING_T_OBS_YR)):
            w = W.serving_workload(chains[c], t)
            cfg = E.Config.from_workload(w)
            psd = E.noise_psd(w.N, w.dt)
            m = E.model_batch(torch.from_numpy(chains[c][None]).cuda(), cfg)[0]
            g = torch.from_numpy(W.gaussian_draws(w.N, 1000 + 10 * c + t)).cuda()
            sig = torch.sqrt(psd * (w.N * w.dt / 4.0))
            sig[0] = 0.0
            sig[-1] = 0.0
            data = (torch.view_as_real(m).double() + sig[None, :, None] * g).contiguous()
            ids[(c, t)] = (srv.add_dataset(data, psd, cfg), w, data, psd, cfg)
            del m, g, sig
    torch.cuda.synchronize()

    def params_of(req):
        gap, c, t, Wn, seed = req
        return W.walkers(ids[(c, t)][1], B=Wn, seed=seed)

    reqs = W.serving_requests(n_burst + n_requests + 2 * n_sweep)
    burst, timed = reqs[:n_burst], reqs[n_burst:n_burst + n_requests]
    sweep_reqs = reqs[n_burst + n_requests:]
    # saturated throughput: everything submitted at once
    t0 = time.perf_counter()
    tk = [srv.submit(ids[(r[1], r[2])][0], params_of(r)) for r in burst]
    for t in tk:
        srv.wait(t)
    mu = n_burst / (time.perf_counter() - t0)

    def open_loop(rs, rate, keep=()):
        """Poisson arrivals at `rate` per s; returns latencies, span, outputs kept"""
        arrivals = np.cumsum([r[0] for r in rs]) / rate
        pre = [params_of(r) for r in rs]   # walker rows drawn before the clock starts
        q = queue.Queue()
        lat = np.zeros(len(rs))
        kept = {}

        def collect():
            for _ in range(len(rs)):
                i, t = q.get()
                out, lat[i] = srv.wait(t)
                if i in keep:
                    kept[i] = out.copy()

        th = threading.Thread(target=collect)
        th.start()
        start = time.perf_counter()
        for i, r in enumerate(rs):
            dtw = arrivals[i] - (time.perf_counter() - start)
            if dtw > 0:
                time.sleep(dtw)
            q.put((i, srv.submit(ids[(r[1], r[2])][0], pre[i])))
            if (i + 1) % 1000 == 0:
                print(f"[bench] serving: {i + 1}/{len(rs)} requests submitted at "
                      f"{rate:.1f}/s", file=sys.stderr, flush=True)
        th.join()
        return lat, time.perf_counter() - start, kept, pre

    lam = 0.8 * mu
    sample = set(range(0, len(timed), max(1, len(timed) // 8)))
    lat, span, served, pre = open_loop(timed, lam, sample)
    sweep = []
    half = len(sweep_reqs) // 2
    for frac, rs in ((0.5, sweep_reqs[:half]), (1.0, sweep_reqs[half:])):
        if not rs:
            continue
        l2, sp2, _, _ = open_loop(rs, frac * mu)
        sweep.append({"lambda_over_mu": frac, "arrival_rate_per_s": frac * mu,
                      "requests": len(rs), "p50_ms": float(np.percentile(l2, 50) * 1e3),
                      "p99_ms": float(np.percentile(l2, 99) * 1e3),
                      "evals_per_s": sum(r[3] for r in rs) / sp2})
    st = srv.stats()
    srv.close()
    # the same walkers alone (eager emri_loglike_dataset) must give the same bits
    same = True
    for i, out in served.items():
        r = timed[i]
        _, w, data, psd, cfg = ids[(r[1], r[2])]
        ds = E.dataset_init(data, psd, cfg)
        alone = E.loglike_dataset(torch.from_numpy(pre[i]).cuda(), ds, cfg).cpu().numpy()
        same = same and bool(np.array_equal(alone, out))
    walkers = sum(r[3] for r in timed)
    del arena
    torch.cuda.empty_cache()
    return {
        "precision": "mixed", "chains": len(chains), "datasets": len(ids),
        "requests": len(timed), "burst_requests": n_burst,
        "saturated_requests_per_s": mu, "arrival_rate_per_s": lam,
        "latency_ms": {"p50": float(np.percentile(lat, 50) * 1e3),
                       "p99": float(np.percentile(lat, 99) * 1e3),
                       "mean": float(lat.mean() * 1e3)},
        "evals_per_s": walkers / span, "mean_walkers_per_request": walkers / len(timed),
        "alone_vs_mix_bitwise": same, "checked_requests": len(served),
        "batches": st["batches"], "graph_launches": st["graph_launches"],
        "graph_captures": st["graph_captures"], "padded_walkers": st["padded_walkers"],
        "arena_gib": arena_gib, "arena_peak_gib": st["arena_peak"] / 2 ** 30,
        "n_streams": n_streams, "max_batch": max_batch, "rate_sweep": sweep,
    }


def host_cpu() -> dict:
    """CPU model and core counts of the host that runs the oracle"""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"cpu_model": model, "nproc": usable, "os_cpu_count": os.cpu_count()}


def golden_values(name: str):
    """per-walker oracle values written by tests/golden/make_golden.py (the
    oracle alone), or None"""
    path = os.path.join(ROOT, "tests", "golden", f"{name}_lnl.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return json.load(f)


def parity_report(got, ref, mm):
    """|dlnL|, relative dlnL and |dlnL| / <m|m> (the signal scale) per walker"""
    d = np.abs(np.asarray(got) - np.asarray(ref))
    return {"walkers": int(d.size), "max_abs_dlnL": float(d.max()),
            "median_abs_dlnL": float(np.median(d)),
            "max_rel_dlnL": float(np.max(d / np.abs(ref))),
            "max_abs_dlnL_over_mm": float(np.max(d / mm)),
            "median_mm": float(np.median(mm))}


def run_oracle_leg(E, W, w64, wmx, P, w1, n_cpu: int):
    """The CPU oracle beside the GPU: the oracle's own data set of the
    headline workload (checked against the golden values' fingerprint), every
    walker of the FP64 and mixed GPU paths on it against the oracle's golden
    per-walker lnL, the oracle timed on a bounded sample of walkers (whose
    spectra also give the waveform mismatch of both GPU paths), and config 1
    (32 walkers, 2^18 samples) checked walker by walker live."""
    import hashlib
    import torch
    import oracle as O
    out = {}
    nthr = O.num_threads()
    ocfg = O.OracleConfig(w64.T_obs, w64.dt, w64.N, w64.n_harm, w64.coarse_log2)
    S = O.psd_bc04(W.frequencies(w64.N, w64.dt))
    t0 = time.perf_counter()
    hinj = O.spectrum(w64.inj[None], ocfg)[0]
    d = O.make_data(hinj, w64.inj, S, W.gaussian_draws(w64.N, w64.noise_seed), w64.N, w64.dt)
    print(f"[bench] oracle data set in {time.perf_counter() - t0:.1f} s", file=sys.stderr,
          flush=True)
    dd = torch.view_as_real(torch.from_numpy(d)).contiguous().cuda()
    ss = torch.from_numpy(S).cuda()
    Pd = torch.from_numpy(P).cuda()
    gpu = {k: E.loglike_batch(Pd, dd, ss, E.Config.from_workload(w)).cpu().numpy()
           for k, w in (("fp64", w64), ("mixed", wmx))}
    g = golden_values(w64.name)
    fp = hashlib.sha256(np.ascontiguousarray(d).tobytes()).hexdigest()
    if g is not None and g["data_sha256"] == fp and len(g["idx"]) == w64.B:
        ref, mm = np.asarray(g["lnl_noisy"]), np.asarray(g["mm"])
        out["every_walker"] = {k: parity_report(v, ref, mm) for k, v in gpu.items()}
        out["every_walker"]["source"] = ("tests/golden (oracle lnL of all walkers on the "
                                         "oracle's data)")

    # the oracle's own rate on a bounded sample (one walker per thread)
    n = n_cpu or min(max(nthr, 1), 16)
    print(f"[bench] cpu baseline: oracle on {n} walkers, {nthr} threads", file=sys.stderr,
          flush=True)
    t0 = time.perf_counter()
    lnl_o, spec_o = O.loglike_sets(P[:n], [d], S, ocfg, return_spectra=True)
    tc = time.perf_counter() - t0
    lnl_o = lnl_o[:, 0]
    # waveform mismatch against the oracle's propagated models of the sample
    mo = np.stack([O.make_data(spec_o[i], P[i], S, None, w64.N, w64.dt) for i in range(n)])
    mo = torch.from_numpy(mo).cuda()
    df = 1.0 / (w64.N * w64.dt)
    mism = {}
    for k, w in (("fp64", w64), ("mixed", wmx)):
        mg = E.model_batch(torch.from_numpy(P[:n]).cuda(), E.Config.from_workload(w))
        m = noise_weighted_mismatch(mg, mo, ss, df)
        mism[k] = {"mismatch_walkers": n, "mismatch_max": float(np.max(np.abs(m))),
                   "mismatch_median": float(np.median(np.abs(m)))}
        del mg
    del mo
    torch.cuda.empty_cache()
    out["mismatch_vs_oracle"] = mism
    out["sample_rel_dlnL"] = {k: float(np.max(np.abs(v[:n] - lnl_o) / np.abs(lnl_o)))
                              for k, v in gpu.items()}
    out["cpu"] = {"value": n / tc, "unit": "lnL evals/s", "cores": nthr, "kind": "oracle",
                  "sample": f"{n} of {w64.B} walkers of {w64.name} (FP64 C oracle, OpenMP one "
                            f"walker per thread), the oracle's data; {tc:.1f} s",
                  **host_cpu()}

    # config 1: every walker against the oracle, computed here
    c1 = O.OracleConfig(w1.T_obs, w1.dt, w1.N, w1.n_harm, w1.coarse_log2)
    S1 = O.psd_bc04(W.frequencies(w1.N, w1.dt))
    h1 = O.spectrum(w1.inj[None], c1)[0]
    d1 = O.make_data(h1, w1.inj, S1, W.gaussian_draws(w1.N, w1.noise_seed), w1.N, w1.dt)
    P1 = W.walkers(w1)
    r1 = O.loglike_sets(P1, [d1, np.zeros_like(d1)], S1, c1)
    g1 = E.loglike_batch(torch.from_numpy(P1).cuda(),
                         torch.view_as_real(torch.from_numpy(d1)).contiguous().cuda(),
                         torch.from_numpy(S1).cuda(), E.Config.from_workload(w1)).cpu().numpy()
    out["config1_every_walker"] = parity_report(g1, r1[:, 0], -2.0 * r1[:, 1])
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-config1", action="store_true")
    ap.add_argument("--no-mismatch", action="store_true",
                    help="skip the mixed-vs-FP64 waveform mismatch (64-walker model batches)")
    ap.add_argument("--cpu-walkers", type=int, default=0,
                    help="oracle sample size (default: one walker per host thread, <= 16)")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=10000,
                    help="timed serving requests (the serving workload: 10000)")
    ap.add_argument("--serve-burst", type=int, default=60)
    ap.add_argument("--serve-arena-gib", type=float, default=160.0)
    ap.add_argument("--serve-sweep", type=int, default=100,
                    help="requests at each of 0.5x and 1.0x the saturated rate")
    ap.add_argument("--no-sampler", action="store_true")
    ap.add_argument("--no-fmg", action="store_true")
    ap.add_argument("--no-dp5", action="store_true")
    ap.add_argument("--sampler-steps", type=int, default=4)
    ap.add_argument("--no-config5", action="store_true")
    ap.add_argument("--config5-steps", type=int, default=2)
    ap.add_argument("--config5-ws-gib", type=float, default=100.0,
                    help="workspace for the 1024-walker stress case (it runs in chunks)")
    ap.add_argument("--calibration-copy-mib", type=int, default=0,
                    help="run one plain device copy of this size first (scale reference for "
                         "HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this benchmark measures one GPU only (asked for {args.gpus}); the "
              "likelihood batch is independent per walker and is not sharded here.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2311_17174_amd import emri as E
    from paper_2311_17174_amd import workloads as W

    if args.calibration_copy_mib:
        n = args.calibration_copy_mib << 20
        a = torch.ones(n // 8, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    w64 = W.config2()
    wmx = W.config3()
    P = W.walkers(w64)
    print(f"[bench] workload {w64.name}: B={w64.B} N={w64.N} n_harm={w64.n_harm}",
          file=sys.stderr, flush=True)

    # synthetic data: propagated injection model (HIP path) + coloured noise
    cfg64 = E.Config.from_workload(w64)
    psd = E.noise_psd(w64.N, w64.dt)
    minj = E.model_batch(torch.from_numpy(w64.inj[None]).cuda(), cfg64)[0]   # [2][H] complex
    g = torch.from_numpy(W.gaussian_draws(w64.N, w64.noise_seed)).cuda()
    sig = torch.sqrt(psd * (w64.N * w64.dt / 4.0))
    sig[0] = 0.0
    sig[-1] = 0.0
    data = torch.view_as_real(minj).clone()
    data += sig[None, :, None] * g
    data = data.contiguous()
    torch.cuda.synchronize()

    dt64, st64, lat64, lnl64 = run_path(E, W, w64, P, data, psd, args.steps, args.warmup)
    evals64 = args.steps * w64.B / dt64
    print(f"[bench] fp64: {evals64:.1f} evals/s, {1e3 * dt64 / args.steps:.2f} ms/step",
          file=sys.stderr, flush=True)

    # config 1: 32 walkers, 30 days, 2^18 samples, 16 harmonics, FP64
    w1 = W.config1()
    config1 = None
    if not args.no_config1:
        c1 = E.Config.from_workload(w1)
        psd1 = E.noise_psd(w1.N, w1.dt)
        m1 = E.model_batch(torch.from_numpy(w1.inj[None]).cuda(), c1)[0]
        g1 = torch.from_numpy(W.gaussian_draws(w1.N, w1.noise_seed)).cuda()
        sig1 = torch.sqrt(psd1 * (w1.N * w1.dt / 4.0))
        sig1[0] = 0.0
        sig1[-1] = 0.0
        data1 = (torch.view_as_real(m1).clone() + sig1[None, :, None] * g1).contiguous()
        dt1, st1, lat1, _ = run_path(E, W, w1, W.walkers(w1), data1, psd1, args.steps,
                                     args.warmup)
        config1 = {"workload": w1.name, "value": args.steps * w1.B / dt1,
                   "unit": "lnL evals/s", "ms_per_step": 1e3 * dt1 / args.steps, "dtype": "f64",
                   "batch_latency_ms": {"p50": float(np.percentile(lat1, 50)),
                                        "p99": float(np.percentile(lat1, 99))}}
        del m1, g1, sig1, data1
        print(f"[bench] config 1: {config1['value']:.1f} evals/s, {config1['ms_per_step']:.3f} "
              "ms/step", file=sys.stderr, flush=True)

    mixed = None
    if not args.no_mixed:
        dtm, stm, latm, lnlm = run_path(E, W, wmx, P, data, psd, args.steps, args.warmup)
        rel = np.abs(lnlm - lnl64) / np.abs(lnl64)
        mixed = {
            "value": args.steps * wmx.B / dtm, "unit": "lnL evals/s",
            "ms_per_step": 1e3 * dtm / args.steps, "dtype": "f32+f64",
            "config": {"workload": wmx.name},
            "batch_latency_ms": {"p50": float(np.percentile(latm, 50)),
                                 "p99": float(np.percentile(latm, 99))},
            "vs_fp64_path": {"max_rel_dlnL": float(rel.max()),
                             "max_abs_dlnL": float(np.abs(lnlm - lnl64).max())},
            "stages_ms_per_step": {k: v[0] / args.steps for k, v in stm.items()},
        }
        # the HBM-bound stages of the mixed path against the 8 TB/s peak
        mst = {}
        for name, (ms, launches) in stm.items():
            kind, amount = stage_work(name, wmx.B, wmx, 8, wmx.B * wmx.n_valid)
            if kind != "byte":
                continue
            per = ms / launches
            gbs = amount / (launches / args.steps) / (per * 1e-3) / 1e9
            mst[name] = {"ms_per_launch": per, "achieved_gbs": gbs,
                         "frac_of_peak": gbs / HBM_PEAK_GBS}
        mixed["stages"] = mst
        # waveform mismatch of the mixed path against the FP64 path (whose
        # parity with the oracle is tested) for every walker, 64 at a time
        if not args.no_mismatch:
            cmx = E.Config.from_workload(wmx)
            mm = []
            for w0 in range(0, wmx.B, 64):
                Pd = torch.from_numpy(P[w0:w0 + 64]).cuda()
                mm.append(noise_weighted_mismatch(E.model_batch(Pd, cmx),
                                                  E.model_batch(Pd, cfg64), psd,
                                                  1.0 / (w64.N * w64.dt)))
                torch.cuda.empty_cache()
            mm = np.concatenate(mm)
            mixed["vs_fp64_path"]["mismatch_max"] = float(np.max(np.abs(mm)))
            mixed["vs_fp64_path"]["mismatch_median"] = float(np.median(np.abs(mm)))
            mixed["vs_fp64_path"]["mismatch_walkers"] = int(mm.size)
        # the mixed synthesis against the FP32 vector peak (the FP64 path's
        # roofline is the top-level one)
        ms_mx = stm["synthesis"][0] / stm["synthesis"][1]
        kind, amount = stage_work("synthesis", wmx.B, wmx, 8, wmx.B * wmx.n_valid)
        amount = amount / (stm["synthesis"][1] / args.steps)
        ach = amount / (ms_mx * 1e-3) / 1e12
        mixed["roofline"] = {"kernel": "synthesis", "bound": "alu", "achieved": ach,
                             "peak": FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
                             "frac": ach / FP32_VECTOR_TFLOPS, "ms_per_launch": ms_mx}
        # <d|d> is common to both paths, so max_abs_dlnL is also the error of
        # the signal part lnL + <d|d>/2
        print(f"[bench] mixed: {mixed['value']:.1f} evals/s", file=sys.stderr, flush=True)

    sampler = None
    if not args.no_sampler:
        sampler = {}
        for wk in (w64, wmx):
            sampler["fp64" if wk is w64 else "mixed"] = run_sampler(
                E, W, wk, data, psd, args.sampler_steps, 1)
        # the paper's own setting (Sec. 3): state at the LSO, free masses, spin
        # and Xi0, against the injection's noise-less model
        wl = w64.with_(ic=1)
        cl = E.Config.from_workload(wl)
        ml = E.model_batch(torch.from_numpy(wl.inj[None]).cuda(), cl)[0]
        dl = torch.view_as_real(ml).double().contiguous()
        sampler["fp64_lso_masses_spin_xi0"] = run_sampler(E, W, wl, dl, psd, args.sampler_steps,
                                                          1, fi=(0, 1, 2, 14))
        del ml, dl
        print(f"[bench] sampler: fp64 {sampler['fp64']['steps_per_s']:.2f} steps/s, mixed "
              f"{sampler['mixed']['steps_per_s']:.2f} steps/s ({2 * w64.B} walkers); the paper's "
              f"setting {sampler['fp64_lso_masses_spin_xi0']['steps_per_s']:.2f} steps/s",
              file=sys.stderr, flush=True)

    fmg = None
    if not args.no_fmg:
        fmg = {"fp64": run_fmg(E, W, w64, data, psd, max(2, args.steps // 2), 1),
               "mixed": run_fmg(E, W, wmx, data, psd, max(2, args.steps // 2), 1)}
        print(f"[bench] frequency-dependent propagation: fp64 {fmg['fp64']['fmg']['value']:.1f} "
              f"evals/s, mixed {fmg['mixed']['fmg']['value']:.1f} evals/s", file=sys.stderr,
              flush=True)

    dp5 = None
    if not args.no_dp5:
        dp5 = {"fp64": run_dp5(E, W, w64, data, psd, max(2, args.steps // 2), 1),
               "mixed": run_dp5(E, W, wmx, data, psd, max(2, args.steps // 2), 1)}
        print(f"[bench] adaptive orbit: fp64 {dp5['fp64']['dp5']['value']:.1f} evals/s (orbit "
              f"{dp5['fp64']['orbit_speedup']:.2f}x faster than RK4; LSO convention "
              f"{dp5['fp64']['dp5_lso']['value']:.1f} evals/s, orbit "
              f"{dp5['fp64']['orbit_speedup_lso']:.2f}x), mixed "
              f"{dp5['mixed']['dp5']['value']:.1f} evals/s; order 7: fp64 "
              f"{dp5['fp64']['rk78']['value']:.1f} evals/s (orbit "
              f"{dp5['fp64']['rk78']['orbit_ms_per_step']:.2f} ms per step)",
              file=sys.stderr, flush=True)

    serving = None
    if not args.no_serving:
        torch.cuda.empty_cache()
        print("[bench] serving loop", file=sys.stderr, flush=True)
        serving = run_serving(E, W, args.serve_burst, args.serve_requests,
                              args.serve_arena_gib, 4, 512, args.serve_sweep)
        print(f"[bench] serving: {serving['evals_per_s']:.1f} evals/s, p50 "
              f"{serving['latency_ms']['p50']:.1f} ms, p99 {serving['latency_ms']['p99']:.1f} ms",
              file=sys.stderr, flush=True)

    config5 = None
    if not args.no_config5:
        torch.cuda.empty_cache()
        print("[bench] stress configuration (1024 walkers, 2^24 samples)", file=sys.stderr,
              flush=True)
        config5 = run_config5(E, W, args.config5_steps, 1, args.config5_ws_gib)
        print(f"[bench] config 5: fp64 {config5['fp64']['value']:.1f} evals/s, mixed "
              f"{config5['mixed']['value']:.1f} evals/s", file=sys.stderr, flush=True)

    # roofline of the dominant kernel of the value path
    valid = w64.B * w64.n_valid
    dom = max(st64.items(), key=lambda kv: kv[1][0])[0]
    stages_out = {}
    # work per step divided over the stage's launches per step (the batch call
    # may split a stage into several launches); achieved = work / time summed
    # over the stage's launches
    for name, (ms, launches) in st64.items():
        kind, amount = stage_work(name, w64.B, w64, 16, valid)
        per = ms / launches
        lps = launches / args.steps
        ent = {"ms_per_launch": per, "launches_per_step": lps}
        if kind == "flop":
            ent["achieved_tflops"] = amount / lps / (per * 1e-3) / 1e12
        elif kind == "byte":
            ent["achieved_gbs"] = amount / lps / (per * 1e-3) / 1e9
        stages_out[name] = ent
    kind, amount = stage_work(dom, w64.B, w64, 16, valid)
    dms = st64[dom][0] / st64[dom][1]
    amount = amount / (st64[dom][1] / args.steps)          # per launch
    if kind == "byte":
        ach = amount / (dms * 1e-3) / 1e9
        roof = {"kernel": dom, "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": ach / HBM_PEAK_GBS, "traffic": profiled_traffic(dom)}
    else:
        ach = amount / (dms * 1e-3) / 1e12
        roof = {"kernel": dom, "bound": "alu", "achieved": ach, "peak": FP64_VECTOR_TFLOPS,
                "unit": "TFLOP/s", "frac": ach / FP64_VECTOR_TFLOPS,
                "traffic": profiled_traffic(dom)}
    roof["ms_per_launch"] = dms
    roof["launches_per_step"] = st64[dom][1] / args.steps
    # the HBM-bound stages against a plain copy measured on the same device
    copy = plain_copy_gbs()
    roof["plain_copy_gbs"] = copy
    for ent in stages_out.values():
        if "achieved_gbs" in ent:
            ent["frac_of_peak"] = ent["achieved_gbs"] / HBM_PEAK_GBS
            ent["frac_of_plain_copy"] = ent["achieved_gbs"] / copy
        if "achieved_tflops" in ent:
            ent["frac_of_peak"] = ent["achieved_tflops"] / FP64_VECTOR_TFLOPS

    cpu = None
    if not args.no_cpu_baseline:
        leg = run_oracle_leg(E, W, w64, wmx, P, w1, args.cpu_walkers)
        cpu = leg["cpu"]
        cpu["parity_sample_max_rel_dlnL"] = leg["sample_rel_dlnL"]["fp64"]
        if config1 is not None:
            config1["vs_oracle"] = leg["config1_every_walker"]
        ev = leg.get("every_walker")
        roof_vs = {"fp64": {**(ev["fp64"] if ev else {}),
                            **leg["mismatch_vs_oracle"]["fp64"]}}
        if mixed is not None:
            mixed["vs_oracle"] = {**(ev["mixed"] if ev else {}),
                                  **leg["mismatch_vs_oracle"]["mixed"]}
        vs_oracle = roof_vs["fp64"]
        if ev:
            vs_oracle["source"] = ev["source"]
            if mixed is not None:
                mixed["vs_oracle"]["source"] = ev["source"]
    else:
        vs_oracle = None

    rec = {
        "metric": "AK lnL evals/sec at 1 yr/2^22 samples, mixed vs FP64; p50/p99 request latency",
        "value": evals64, "unit": "lnL evals/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * dt64 / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic: seeded walkers around the injection; data = propagated injection "
                "model + Gaussian noise coloured by the BC04 instrumental PSD",
        "config": {"workload": w64.name, "walkers": w64.B, "samples": w64.N,
                   "n_valid": w64.n_valid, "n_harm": w64.n_harm, "dt": w64.dt,
                   "coarse_step_s": w64.dt * (1 << w64.coarse_log2)},
        "batch_latency_ms": {"p50": float(np.percentile(lat64, 50)),
                             "p99": float(np.percentile(lat64, 99))},
        "roofline": roof,
        "cpu_baseline": cpu,
        "vs_oracle": vs_oracle,
        "config1": config1,
        "mixed": mixed,
        "serving": serving,
        "stress": config5,
        "sampler": sampler,
        "frequency_dependent_propagation": fmg,
        "adaptive_orbit": dp5,
        "stages": stages_out,
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
