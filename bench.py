#!/usr/bin/env python3
"""Benchmark: Chebyshev-filtered subspace iteration on one MI355X.

One step = one filter iteration of the hot path on one block: Chebyshev
filter of degree m (H*psi applications, reusing the H*Y left by the previous
Rayleigh-Ritz), Cholesky orthonormalisation and Rayleigh-Ritz (one more
H*psi, always FP64).  Inputs are synthetic diamond cells (synth/), resident
in HBM before timing.

The default run times the mixed path (filter in FP32: FFT route in FP32,
projector products on FP32 MFMA; orthonormalisation and Rayleigh-Ritz in
FP64) and then the plain FP64 path from the same start block, and prints one
JSON line for the mixed path with the FP64 figures and the Ritz-value
difference between the two trajectories beside it.

  value        band*H*psi applications per second over the timed steps
  ms_per_step  filter-iteration time
  roofline     dominant kernel vs its roofline, from HIP events recorded by
               the library on its own stream over the timed steps
  cpu_baseline the FP64 oracle's H*psi timed on the host on a band sample
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
PEAK = {   # MI355X published dense peaks
    "fp64_mfma": 78.6, "fp32_mfma": 157.3, "bf16_mfma": 2500.0,
    "fp64_valu": 78.6, "fp32_valu": 157.3, "hbm_gbs": 8000.0,
}

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


def fft_flops(n):
    import math
    return 5.0 * n * math.log2(n)


def roofline(stages, steps, applies, w, ham, nb, prec):
    """Dominant single-kernel stage of the filter path against its bound.

    nonlocal (k_gemm_nn: H psi += P C): MFMA, 8 npw nproj nb flop per launch.
    fft_plane: vector ALU, per band and z-plane 2 (xr 5 N2 log2 N2 + N2 5 N1 log2 N1)
               + 2 N1 N2 flop (the V product), per launch x bands in the launch.
    fft_col_inv / fft_col_fwd: HBM, (npw + ncols N3) / (ncols N3 + 2 npw) elements per band.
    """
    N1, N2, N3 = w.box
    ncols, xr = ham.ncolumns, ham.extent1
    elem = 16 if prec == "fp64" else 8
    cand = {k: v for k, v in stages.items()
            if k in ("nonlocal", "fft_plane", "fft_col_inv", "fft_col_fwd") and v[1] > 0}
    dom = max(cand, key=lambda k: cand[k][0])
    total_ms, launches = cand[dom]
    avg_ms = total_ms / launches
    # bands per launch: the FFT kernels run once per band chunk and application
    bands_per_launch = nb * steps * applies / launches
    if dom == "nonlocal":
        fl = 8.0 * w.npw * w.nproj * nb
        peak = PEAK["fp64_mfma" if prec == "fp64" else ("bf16_mfma" if prec == "bf16" else "fp32_mfma")]
        ach = fl / (avg_ms * 1e-3) / 1e12
        return {"kernel": "k_gemm_nn (H psi += P C)", "bound": "mfma", "achieved": ach, "peak": peak,
                "unit": "TFLOP/s", "frac": ach / peak, "avg_launch_ms": avg_ms,
                "per_launch": f"8*npw*nproj*nb = {fl:.4g} flop"}
    if dom == "fft_plane":
        per_band = N3 * (2 * (xr * fft_flops(N2) + N2 * fft_flops(N1)) + 2.0 * N1 * N2)
        fl = per_band * bands_per_launch
        peak = PEAK["fp64_valu" if prec == "fp64" else "fp32_valu"]
        ach = fl / (avg_ms * 1e-3) / 1e12
        return {"kernel": "k_plane_reg (N2/N1 transforms x V per z-plane)", "bound": "alu",
                "achieved": ach, "peak": peak, "unit": "TFLOP/s", "frac": ach / peak,
                "avg_launch_ms": avg_ms,
                "per_launch": f"{per_band:.4g} flop/band (5 N log2 N per transform) x "
                              f"{bands_per_launch:.0f} bands",
                "hbm_view": {"bytes_per_band": elem * 2 * ncols * N3,
                             "GBs": elem * 2 * ncols * N3 * bands_per_launch / (avg_ms * 1e-3) / 1e9}}
    per_band = elem * ((w.npw + ncols * N3) if dom == "fft_col_inv" else (ncols * N3 + 2 * w.npw))
    ach = per_band * bands_per_launch / (avg_ms * 1e-3) / 1e9
    return {"kernel": dom, "bound": "hbm", "achieved": ach, "peak": PEAK["hbm_gbs"], "unit": "GB/s",
            "frac": ach / PEAK["hbm_gbs"], "avg_launch_ms": avg_ms,
            "per_launch": f"{per_band:.4g} B/band x {bands_per_launch:.0f} bands"}


def cpu_baseline(w, nb_sample, seed=0):
    """Oracle H*psi on nb_sample bands of the same workload, timed on the host."""
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


def run_path(pw, ctx, ham, w, X0, b, prec, steps, warmup):
    """Iteration 0 + warmup + timed steps from X0; returns timings and the last Ritz values."""
    import torch
    nb = w.nb
    Y = X0.clone()
    HY = torch.empty_like(Y)
    eig = torch.empty(nb, dtype=torch.float64, device="cuda")
    resid = torch.empty(nb, dtype=torch.float64, device="cuda")
    ham.orthonormalize(Y)
    ham.rayleigh_ritz(Y, HY, eig, resid)
    lam = eig.cpu()
    sweeps = []

    def step():
        nonlocal lam
        ham.cheb_filter(Y, w.degree, float(lam[-1]), b, float(lam[0]), hx=HY, prec=prec)
        ham.orthonormalize(Y)
        ham.rayleigh_ritz(Y, HY, eig, resid)
        sweeps.append(ctx.last_sweeps())
        lam = eig.cpu()

    for i in range(warmup):
        step()
        log(f"{prec}: warmup {i + 1}/{warmup} done")
    ctx.set_timing(True)
    ctx.reset_timing()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        step()
        log(f"{prec}: step {i + 1}/{steps} done")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    stages = ctx.stage_times()
    ctx.set_timing(False)
    applies = w.degree                       # (degree - 1) filter products + 1 in Rayleigh-Ritz
    return {"ms_per_step": 1e3 * dt / steps, "value": applies * nb * steps / dt,
            "stages": stages, "applies": applies, "lam": lam.numpy().copy(),
            "max_resid": float(resid.max().cpu()), "sweeps": sweeps}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="C5", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default="fp32", choices=["fp64", "fp32", "bf16"],
                    help="filter precision of the reported path (subspace steps are FP64)")
    ap.add_argument("--no-compare", action="store_true", help="skip the FP64 comparison run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-bands", type=int, default=0, help="oracle band sample (0 = auto)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        sys.exit(2)

    import torch
    import synth
    import paper_2507_08578_amd as pw

    log(f"generating workload {args.config}")
    w = make_workload(args.config)
    nb = w.nb
    log(f"npw={w.npw} nproj={w.nproj} box={w.box} nb={nb} degree={w.degree}")
    ctx = pw.Context(0)
    mixed = args.precision != "fp64"
    ham = pw.Hamiltonian.from_workload(ctx, w, nb_max=nb, low_prec=mixed)
    X0 = torch.from_numpy(synth.start_block(w.npw, nb, 0)).cuda()
    log("upper bound")
    b = ham.upper_bound()
    res = run_path(pw, ctx, ham, w, X0, b, args.precision, args.steps, args.warmup)
    ref = None
    if mixed and not args.no_compare:
        ref = run_path(pw, ctx, ham, w, X0, b, "fp64", args.steps, args.warmup)
    roof = roofline(res["stages"], args.steps, res["applies"], w, ham, nb, args.precision)
    dtype = "f64" if not mixed else ("f32+f64" if args.precision == "fp32" else "bf16/f32+f64")
    out = {
        "metric": METRIC, "value": res["value"], "unit": UNIT, "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": res["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": dtype, "data": "synthetic",
        "config": {"workload": f"{args.config}: {WORKLOADS[args.config]}",
                   "filter_precision": args.precision, "subspace_precision": "fp64",
                   "step": f"filter (degree {w.degree}, H*Y reused) + Cholesky + Rayleigh-Ritz",
                   "applies_per_step": res["applies"], "nb": nb},
        "filter_iter_ms": res["ms_per_step"],
        "max_resid": res["max_resid"],
        "eigensolver_sweeps": res["sweeps"],
        "roofline": roof,
        "stages_ms_per_step": {k: v[0] / args.steps for k, v in res["stages"].items()},
    }
    if ref is not None:
        d = float(abs(res["lam"] - ref["lam"]).max())
        out["fp64_path"] = {"ms_per_step": ref["ms_per_step"], "value": ref["value"],
                            "speedup_mixed_over_fp64": ref["ms_per_step"] / res["ms_per_step"],
                            "stages_ms_per_step": {k: v[0] / args.steps
                                                   for k, v in ref["stages"].items()}}
        out["eig_diff_vs_fp64_Ha"] = d
    if not args.no_cpu_baseline:
        nbs = args.cpu_bands or {"C1": 256, "C3": 64, "C5": 64}[args.config]
        log(f"cpu baseline: oracle H*psi on {nbs} bands")
        out["cpu_baseline"] = cpu_baseline(w, nbs)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
