#!/usr/bin/env python3
"""Benchmark: Chebyshev-filtered subspace iteration on one MI355X.

One step = one filter iteration of the hot path on one block: Chebyshev
filter of degree m (H*psi applications), Cholesky orthonormalisation and
Rayleigh-Ritz (one more H*psi), exactly as the solver runs it.  Inputs are
synthetic diamond cells (see synth/), resident in HBM before timing.

Prints one JSON line (rank 0):
  value       = band*H*psi applications per second over the timed steps
  ms_per_step = filter-iteration time
  roofline    = the dominant kernel against its roofline (HIP events on the
                library's stream), traffic from rocprofv3 counters if given
  cpu_baseline= the FP64 oracle timed on the host on a bounded band sample
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "band·H·ψ applies/sec + filter-iter time, mixed vs FP64, eig err ≤1e-6 Ha"
UNIT = "band·H·ψ applies/s"
PEAK_FP64_TFLOPS = 78.6     # MI355X dense FP64 (matrix and vector)
PEAK_HBM_GBS = 8000.0       # MI355X HBM3E

WORKLOADS = {
    "C1": "8-atom diamond cell a=10.26 bohr, Gamma, ecut 8 Ha, 1189 PW, box 24^3, 8 s-projectors, "
          "16 bands, Chebyshev degree 8",
    "C3": "64-atom 2x2x2 diamond supercell (jitter 0.05 bohr), Gamma, ecut 20 Ha, 37073 PW, box 96^3, "
          "256 s+p projectors, 160 bands, Chebyshev degree 8",
    "C5": "216-atom 3x3x3 diamond supercell a=30.78 bohr, Gamma, ecut 20 Ha, 124289 PW, box 144^3, "
          "864 s+p projectors, 512 bands, Chebyshev degree 12",
}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def make_workload(name):
    import synth
    return {"C1": synth.config_c1, "C3": synth.config_c3, "C5": synth.config_c5}[name]()


def stage_flops_bytes(w, ham, nb):
    """Algorithmic work of one launch of each single-kernel stage (FP64)."""
    npw, nproj = w.npw, w.nproj
    N1, N2, N3 = w.box
    ncols, xr = ham.ncolumns, ham.extent1
    per_band_fft_bytes = 16 * (2 * npw + 4 * ncols * N3)     # 3-kernel model
    return {
        "nonlocal": {"flops": 8.0 * npw * nproj * nb, "bytes": 16.0 * (npw * nproj + 2 * npw * nb)},
        "proj": {"flops": 8.0 * npw * nproj * nb, "bytes": 16.0 * (npw * nproj + npw * nb)},
        "fft_per_band_bytes": per_band_fft_bytes,
        "fft_col_inv_bytes_per_band": 16.0 * (npw + ncols * N3),
        "fft_plane_bytes_per_band": 16.0 * (2 * ncols * N3),
        "fft_col_fwd_bytes_per_band": 16.0 * (ncols * N3 + 2 * npw),
    }


def cpu_baseline(w, nb_sample, seed=0):
    """Oracle H*psi on nb_sample bands of the same workload, timed on the host."""
    import numpy as np
    import oracle
    import synth
    try:
        from threadpoolctl import threadpool_info
        blas = [p for p in threadpool_info() if p.get("user_api") == "blas"]
        threads = max([p.get("num_threads", 1) for p in blas] or [1])
    except Exception:
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    oh = oracle.OracleHam.from_workload(w)
    X = synth.start_block(w.npw, nb_sample, seed).T
    oracle.apply_h(oh, X[:, :1])                 # first-touch
    t0 = time.perf_counter()
    oracle.apply_h(oh, X)
    dt = time.perf_counter() - t0
    return {"value": nb_sample / dt, "unit": UNIT, "cores": int(threads), "kind": "oracle",
            "sample": f"{nb_sample} bands of one FP64 oracle H*psi on {w.name} "
                      f"(numpy FFT + BLAS), {dt:.2f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="C5", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-bands", type=int, default=0, help="oracle band sample (0 = auto)")
    ap.add_argument("--traffic-json", default=os.path.join(ROOT, "profiles", "traffic.json"),
                    help="per-kernel HBM bytes measured with rocprofv3 counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        sys.exit(2)

    import numpy as np
    import torch
    import synth
    import paper_2507_08578_amd as pw

    log(f"generating workload {args.config}")
    w = make_workload(args.config)
    nb = w.nb
    log(f"npw={w.npw} nproj={w.nproj} box={w.box} nb={nb} degree={w.degree}")
    ctx = pw.Context(0)
    ham = pw.Hamiltonian.from_workload(ctx, w, nb_max=nb)
    X0 = torch.from_numpy(synth.start_block(w.npw, nb, 0)).cuda()
    Y = X0.clone()
    HY = torch.empty_like(Y)
    eig = torch.empty(nb, dtype=torch.float64, device="cuda")
    resid = torch.empty(nb, dtype=torch.float64, device="cuda")
    log("upper bound + iteration 0")
    b = ham.upper_bound()
    ham.orthonormalize(Y)
    ham.rayleigh_ritz(Y, HY, eig, resid)
    lam = eig.cpu()

    sweeps = []

    def step():
        nonlocal lam
        ham.cheb_filter(Y, w.degree, float(lam[-1]), b, float(lam[0]), hx=HY)
        ham.orthonormalize(Y)
        ham.rayleigh_ritz(Y, HY, eig, resid)
        sweeps.append(ctx.last_sweeps())
        lam = eig.cpu()

    for i in range(args.warmup):
        step()
        log(f"warmup {i + 1}/{args.warmup} done")
    ctx.set_timing(True)
    ctx.reset_timing()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step()
        log(f"step {i + 1}/{args.steps} done")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    stages = ctx.stage_times()
    ctx.set_timing(False)
    applies_per_step = (w.degree - 1) + 1          # filter reuses H Y from Rayleigh-Ritz
    ms_per_step = 1e3 * dt / args.steps
    value = applies_per_step * nb * args.steps / dt

    # dominant single-kernel stage and its roofline
    work = stage_flops_bytes(w, ham, nb)
    cand = {k: v for k, v in stages.items() if k in ("nonlocal", "fft_plane", "fft_col_inv",
                                                      "fft_col_fwd") and v[1] > 0}
    dom = max(cand, key=lambda k: cand[k][0])
    avg_ms = cand[dom][0] / cand[dom][1]
    traffic = None
    try:
        with open(args.traffic_json) as f:
            tj = json.load(f)
        traffic = tj.get(args.config, {}).get(dom)
    except (OSError, ValueError):
        traffic = None
    if dom == "nonlocal":
        ach = work["nonlocal"]["flops"] / (avg_ms * 1e-3) / 1e12
        roof = {"kernel": "k_gemm_nn (H psi += P C)", "bound": "mfma", "achieved": ach,
                "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s", "frac": ach / PEAK_FP64_TFLOPS,
                "traffic": traffic, "avg_launch_ms": avg_ms,
                "per_launch": f"8*npw*nproj*nb = {work['nonlocal']['flops']:.4g} flop"}
    else:
        per_band = work[f"{dom}_bytes_per_band"]
        # launches per step = number of band chunks; bytes per launch = bands per launch * per_band
        launches_per_apply = max(1, round(cand[dom][1] / (args.steps * applies_per_step)))
        chunk_bands = nb / launches_per_apply
        ach = per_band * chunk_bands / (avg_ms * 1e-3) / 1e9
        roof = {"kernel": dom, "bound": "hbm", "achieved": ach, "peak": PEAK_HBM_GBS,
                "unit": "GB/s", "frac": ach / PEAK_HBM_GBS, "traffic": traffic,
                "avg_launch_ms": avg_ms,
                "per_launch": f"{per_band:.4g} B/band x {chunk_bands:.0f} bands"}
    out = {
        "metric": METRIC, "value": value, "unit": UNIT, "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{args.config}: {WORKLOADS[args.config]}", "precision": "fp64",
                   "step": f"filter (degree {w.degree}, H*Y reused) + Cholesky + Rayleigh-Ritz",
                   "applies_per_step": applies_per_step, "nb": nb},
        "filter_iter_ms": ms_per_step,
        "max_resid": float(resid.max().cpu()),
        "eigensolver_sweeps": sweeps,
        "roofline": roof,
        "stages_ms_per_step": {k: v[0] / args.steps for k, v in stages.items()},
    }
    if not args.no_cpu_baseline:
        nbs = args.cpu_bands or {"C1": 256, "C3": 64, "C5": 64}[args.config]
        log(f"cpu baseline: oracle H*psi on {nbs} bands")
        out["cpu_baseline"] = cpu_baseline(w, nbs)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
