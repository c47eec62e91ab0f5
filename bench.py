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
  ms_per_step  filter-iteration time (no stage events in the timed steps)
  roofline     dominant kernel vs its roofline, from HIP events recorded by
               the library on its own stream over a few further steps
  cpu_baseline the FP64 oracle's H*psi timed on the host on a band sample

Beside the headline the same line carries the FP64 path (with its own
roofline), LOBPCG and RMM-DIIS passes on the same block, the electron
density, and (default C5 run) the batched C2 (FP64) and C4 (mixed) forms.
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
    "C2": "8-atom diamond cell a=10.26 bohr, 27 k-points on the shifted 3x3x3 grid (1088-1180 PW "
          "each), ecut 8 Ha, box 24^3, 8 s-projectors, 16 bands per k-point, Chebyshev degree 8, "
          "all k-points in one batch (HIP graph)",
    "C4": "64 independent 8-atom diamond cells, strain +-6%, ecut 8-16 Ha (1.1k-3.6k PW, boxes "
          "24-36 per axis), 8 s-projectors, 16-32 bands, Chebyshev degree 8, one batch (HIP graph)",
    "C3": "64-atom 2x2x2 diamond supercell (jitter 0.05 bohr), Gamma, ecut 20 Ha, 37073 PW, box 96^3, "
          "256 s+p projectors, 160 bands, Chebyshev degree 8",
    "C5": "216-atom 3x3x3 diamond supercell a=30.78 bohr, Gamma, ecut 20 Ha, 124289 PW, box 144^3, "
          "864 s+p projectors, 512 bands, Chebyshev degree 12",
}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def make_workload(name):
    import synth
    return {"C1": synth.config_c1, "C2": synth.config_c2, "C3": synth.config_c3,
            "C4": synth.config_c4, "C5": synth.config_c5}[name]()


BATCHED = ("C2", "C4")


# (config, precision, stage, kernel) -> committed rocprofv3 counter summary and
# the sources whose hash it records
COUNTER_FILES = {
    ("C5", "fp64", "fft_plane", "k_plane_reg"): (
        "profiles/c5_plane_fp64_counters.md",
        ("paper_2507_08578_amd/csrc/fft_reg.hip", "paper_2507_08578_amd/csrc/fft_common.h")),
    ("C5", "fp32", "proj", "k_gemm_cn32_s3"): (
        "profiles/c5_gemm_fp32_counters.md",
        ("paper_2507_08578_amd/csrc/gemm32_kernels.hip",)),
    ("C5", "fp32", "nonlocal", "k_gemm_nn32_s3"): (
        "profiles/c5_gemm_nn32_fp32_counters.md",
        ("paper_2507_08578_amd/csrc/gemm32_kernels.hip",)),
    ("C5", "fp64", "density", "k_density_reg"): (
        "profiles/c5_density_counters.md",
        ("paper_2507_08578_amd/csrc/density.hip", "paper_2507_08578_amd/csrc/fft_common.h")),
    ("C5", "fp32", "fft_plane", "k_plane_ls"): (
        "profiles/c5_plane_ls_fp32_counters.md",
        ("paper_2507_08578_amd/csrc/fft_ls.hip", "paper_2507_08578_amd/csrc/fft_common.h")),
}


def plane_kernel(ham, prec):
    """Name of the plane kernel the handle's tuning selects for this precision."""
    t = ham.get_tuning()
    if prec != "fp64" and t["reg_plane"] and t["plane_variant32"] == 2:
        return "k_plane_ls"
    return "k_plane_reg" if t["reg_plane"] else "k_plane"


def measured_traffic(config, prec, stage, kernel, bands_per_launch):
    """HBM bytes per launch from the committed FETCH_SIZE / WRITE_SIZE summary,
    or None when there is none or the kernel sources changed since it was taken."""
    import hashlib
    entry = COUNTER_FILES.get((config, prec, stage, kernel))
    if entry is None or not os.path.exists(os.path.join(ROOT, entry[0])):
        return None
    rel, sources = entry
    vals = {}
    for line in open(os.path.join(ROOT, rel)):
        if ":" in line and not line.startswith(("#", "|", "`")):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    h = hashlib.sha1()
    for f in sources:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    if vals.get("kernel_source_sha1") != h.hexdigest():
        return None
    if "traffic_bytes_per_launch" in vals:
        return float(vals["traffic_bytes_per_launch"])
    if "traffic_bytes_per_band" not in vals:
        return None
    return float(vals["traffic_bytes_per_band"]) * bands_per_launch


def fft_flops(n):
    import math
    return 5.0 * n * math.log2(n)


def roofline(stages, steps, w, ham, nb, prec, config=None):
    """Dominant single-kernel stage of the filter path against its bound.

    The stages of the precision being reported are used (the low-precision
    path times its FP32 / BF16 kernels under their own stage ids; its
    Rayleigh-Ritz product stays FP64 and is not counted here).
    proj (P^H psi, split-K + reduce) and nonlocal (H psi += P C): MFMA,
               8 npw nproj nb flop per launch.
    fft_plane: vector ALU, per band and z-plane 2 (xr 5 N2 log2 N2 + N2 5 N1 log2 N1)
               + 2 N1 N2 flop (the V product), per launch x bands in the launch
               (full-length transforms: a kernel that prunes the zero inputs and
               unused outputs does less arithmetic than this count).
    fft_col_inv / fft_col_fwd: HBM, (npw + ncols N3) / (ncols N3 + 2 npw) elements per band.
    """
    N1, N2, N3 = w.box
    ncols, xr = ham.ncolumns, ham.extent1
    lp = prec != "fp64"
    sfx = "_lp" if lp else ""
    applies = w.degree - 1 if lp else w.degree     # H*psi products of this precision per step
    elem = 16 if prec == "fp64" else 8
    cand = {k[:len(k) - len(sfx)] if sfx else k: v for k, v in stages.items()
            if k in (f"proj{sfx}", f"nonlocal{sfx}", f"fft_plane{sfx}", f"fft_col_inv{sfx}",
                     f"fft_col_fwd{sfx}")
            and v[1] > 0}
    dom = max(cand, key=lambda k: cand[k][0])
    total_ms, launches = cand[dom]
    avg_ms = total_ms / launches
    # bands per launch: the FFT kernels run once per band chunk and application
    bands_per_launch = nb * steps * applies / launches
    if dom in ("proj", "nonlocal"):
        fl = 8.0 * w.npw * w.nproj * nb
        # the matrix cores' own dtype: FP64, or bf16 (the FP32 path's products take
        # their FP32 operands as three bf16 terms, six MFMA products per real
        # product; the bf16 path rounds its operands to bf16)
        on_bf16 = prec in ("bf16", "fp32")
        peak = PEAK["fp64_mfma" if prec == "fp64" else ("bf16_mfma" if on_bf16 else "fp32_mfma")]
        ach = fl / (avg_ms * 1e-3) / 1e12
        mode = "" if prec == "fp64" else ("<F32>" if prec == "fp32" else "<BF16>")
        sx = "" if prec == "fp64" else "32"
        extra = {}
        if dom == "proj":
            key = f"k_gemm_cn{sx}"
            kname = f"k_gemm_cn{sx}{mode} + k_splitk_reduce{sx} (P^H psi, split-K, KB scale)"
            if prec == "fp32":
                key = "k_gemm_cn32_s3"
                kname = ("k_gemm_cn32_s3 + k_splitk_reduce32 (P^H psi, split-K, KB scale; P as "
                         "a stored three-term bf16 copy, psi split per stage, bf16 MFMA)")
                extra = {"executed_mfma_flop_per_launch": 6.0 * fl,
                         "executed_TFLOPs": 6.0 * ach, "executed_frac": 6.0 * ach / peak}
        elif prec == "fp32":
            key = "k_gemm_nn32_s3"
            kname = ("k_gemm_nn32_s3 (H psi += P C; P and C as stored three-term bf16 copies, "
                     "bf16 MFMA)")
            extra = {"executed_mfma_flop_per_launch": 6.0 * fl,
                     "executed_TFLOPs": 6.0 * ach, "executed_frac": 6.0 * ach / peak}
        else:
            tall = ham.get_tuning()["nn_tile" if prec == "fp64" else "nn_tile32"] == 1
            key = f"k_gemm_nn{sx}{'_tall' if tall else ''}"
            kname = f"{key}{mode} (H psi += P C)"
        return dict({"kernel": kname, "bound": "mfma", "achieved": ach, "peak": peak,
                     "unit": "TFLOP/s", "frac": ach / peak,
                     "traffic": measured_traffic(config, prec, dom, key, 1),
                     "avg_launch_ms": avg_ms,
                     "per_launch": f"8*npw*nproj*nb = {fl:.4g} flop"}, **extra)
    if dom == "fft_plane":
        per_band = N3 * (2 * (xr * fft_flops(N2) + N2 * fft_flops(N1)) + 2.0 * N1 * N2)
        fl = per_band * bands_per_launch
        peak = PEAK["fp64_valu" if prec == "fp64" else "fp32_valu"]
        ach = fl / (avg_ms * 1e-3) / 1e12
        kname = plane_kernel(ham, prec)
        extra = {}
        if prec != "fp64":
            # 157.3 counts packed FP32 (two FMAs per lane and instruction); the
            # kernels are built without packed-FP32 code, so 78.6 is what they can issue
            extra = {"peak_unpacked_fp32": PEAK["fp64_valu"],
                     "frac_unpacked_fp32": ach / PEAK["fp64_valu"]}
        return {**extra, "kernel": f"{kname} (N2/N1 transforms x V per z-plane)", "bound": "alu",
                "achieved": ach, "peak": peak, "unit": "TFLOP/s", "frac": ach / peak,
                "traffic": measured_traffic(config, prec, dom, kname, bands_per_launch),
                "avg_launch_ms": avg_ms,
                "per_launch": f"{per_band:.4g} flop/band (5 N log2 N per transform) x "
                              f"{bands_per_launch:.0f} bands",
                "hbm_view": {"bytes_per_band": elem * 2 * ncols * N3,
                             "GBs": elem * 2 * ncols * N3 * bands_per_launch / (avg_ms * 1e-3) / 1e9}}
    per_band = elem * ((w.npw + ncols * N3) if dom == "fft_col_inv" else (ncols * N3 + 2 * w.npw))
    ach = per_band * bands_per_launch / (avg_ms * 1e-3) / 1e9
    return {"kernel": dom, "bound": "hbm", "achieved": ach, "peak": PEAK["hbm_gbs"], "unit": "GB/s",
            "frac": ach / PEAK["hbm_gbs"], "traffic": None, "avg_launch_ms": avg_ms,
            "per_launch": f"{per_band:.4g} B/band x {bands_per_launch:.0f} bands"}


def host_cpu():
    """CPU model string and the threads the oracle uses: BLAS threads for
    its matrix products, scipy.fft workers (every CPU the OS reports) for
    its transforms."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        from threadpoolctl import threadpool_info
        blas = [p for p in threadpool_info() if p.get("user_api") == "blas"]
        blas_threads = max([p.get("num_threads", 1) for p in blas] or [1])
    except Exception:
        blas_threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    fft_workers = os.cpu_count() or 1
    try:
        affinity = len(os.sched_getaffinity(0))
    except Exception:
        affinity = fft_workers
    return {"cpu_model": model, "blas_threads": int(blas_threads), "fft_workers": int(fft_workers),
            "cpus_allowed": int(affinity)}


def cpu_baseline(w, nb_sample, seed=0):
    """Oracle H*psi on nb_sample bands of the same workload, timed on the host."""
    import oracle
    import synth
    hc = host_cpu()
    threads = min(max(hc["blas_threads"], hc["fft_workers"]), hc["cpus_allowed"])
    oh = oracle.OracleHam.from_workload(w)
    X = synth.start_block(w.npw, nb_sample, seed).T
    oracle.apply_h(oh, X[:, :1])                 # first-touch
    t0 = time.perf_counter()
    oracle.apply_h(oh, X)
    dt = time.perf_counter() - t0
    return {"value": nb_sample / dt, "unit": UNIT, "cores": int(threads), "kind": "oracle",
            "sample": f"{nb_sample} bands of one FP64 oracle H*psi on {w.name} "
                      f"(scipy FFT + BLAS), {dt:.2f} s", **hc}


def density_leg(ctx, ham, w, X0, steps, warmup, config=None):
    """Electron density of the resident block (section 2.4, Eq. nandtau), every
    band with occupation 2: `steps` pw_density calls timed after `warmup`.
    Roofline of its plane kernel (vector ALU, FP64): per band and z-plane
    xr 5 N2 log2 N2 + N2 5 N1 log2 N1 + 4 N1 N2 flop (the two backward
    transforms, w |.|^2 added), x bands per launch, over the kernel's average
    launch time; charge = (Omega / N_box) sum_j n(r_j) against
    sum_b w_b |c_b|^2 (Parseval) as a check of the timed result."""
    import torch
    nb = X0.shape[0]
    wt = torch.full((nb,), 2.0, dtype=torch.float64, device="cuda")
    rho = ham.density(X0, wt)
    for _ in range(warmup):
        ham.density(X0, wt, rho=rho)
    torch.cuda.synchronize()
    ctx.set_timing(True)
    ctx.reset_timing()
    t0 = time.perf_counter()
    for _ in range(steps):
        ham.density(X0, wt, rho=rho)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    st = ctx.stage_times()
    ctx.set_timing(False)
    N1, N2, N3 = w.box
    xr = ham.extent1
    total, launches = st["density"]
    avg_ms = total / launches
    bands_per_launch = nb * steps / launches
    per_band = N3 * (xr * fft_flops(N2) + N2 * fft_flops(N1) + 4.0 * N1 * N2)
    ach = per_band * bands_per_launch / (avg_ms * 1e-3) / 1e12
    reg = N1 == N2 and N1 in (24, 30, 32, 36, 48, 64, 72, 96, 120, 128, 144, 160)
    kname = f"k_density_reg<{N1},16>" if reg else "k_density_plane"
    charge = w.cell.volume / (N1 * N2 * N3) * float(rho.sum().item())
    ref_charge = 2.0 * float((X0.abs() ** 2).sum().item())
    return {"ms_per_call": 1e3 * dt, "nb": nb, "value": nb / dt, "unit": "band densities/s",
            "stages_ms_per_call": {k: v[0] / steps for k, v in st.items() if v[1]},
            "charge_rel_err": abs(charge - ref_charge) / ref_charge,
            "roofline": {"kernel": f"{kname} (N2/N1 backward transforms, w |psi|^2 summed)",
                         "bound": "alu", "achieved": ach, "peak": PEAK["fp64_valu"],
                         "unit": "TFLOP/s", "frac": ach / PEAK["fp64_valu"],
                         "traffic": measured_traffic(config, "fp64", "density", "k_density_reg",
                                                     bands_per_launch) if reg else None,
                         "avg_launch_ms": avg_ms,
                         "per_launch": f"{per_band:.4g} flop/band x {bands_per_launch:.0f} bands"}}


def cpu_density_baseline(w, nb_sample, seed=0):
    """Oracle density (numpy FFT per band) on nb_sample bands, timed on the host."""
    import numpy as np
    import oracle
    import synth
    oh = oracle.OracleHam.from_workload(w)
    X = synth.start_block(w.npw, nb_sample, seed).T
    wt = np.full(nb_sample, 2.0)
    oracle.density(oh, X[:, :1], wt[:1])          # first-touch
    t0 = time.perf_counter()
    oracle.density(oh, X, wt)
    dt = time.perf_counter() - t0
    hc = host_cpu()
    return {"value": nb_sample / dt, "unit": "band densities/s",
            "cores": min(hc["fft_workers"], hc["cpus_allowed"]), "kind": "oracle",
            "sample": f"{nb_sample} bands of the FP64 oracle density on {w.name} "
                      f"(scipy FFT on all workers), {dt:.2f} s", **hc}


def run_path(pw, ctx, ham, w, X0, b, prec, steps, warmup, stage_steps, gram_prec="fp64"):
    """Iteration 0 + warmup + timed steps from X0 (no stage events in the timed
    steps), then stage_steps more steps with per-stage HIP events for the
    roofline.  The only host reads per step are the deferred status and the
    Ritz values (and the eigensolver's sweep count)."""
    import torch
    nb = w.nb
    Y = X0.clone()
    HY = torch.empty_like(Y)
    eig = torch.empty(nb, dtype=torch.float64, device="cuda")
    resid = torch.empty(nb, dtype=torch.float64, device="cuda")
    ham.orthonormalize(Y, check=False)
    ham.rayleigh_ritz(Y, HY, eig, resid, check=False)
    ctx.check_status()
    lam = eig.cpu()
    sweeps = []

    it = [0]

    def step():
        nonlocal lam
        it[0] += 1
        fp = prec(it[0]) if callable(prec) else prec
        ham.cheb_filter(Y, w.degree, float(lam[-1]), b, float(lam[0]), hx=HY, prec=fp)
        ham.orthonormalize(Y, gram_prec=gram_prec, check=False)
        ham.rayleigh_ritz(Y, HY, eig, resid, check=False)
        ctx.check_status()
        lam = eig.cpu()
        sweeps.append(ctx.last_sweeps())

    name = "ladder" if callable(prec) else prec
    for i in range(warmup):
        step()
        log(f"{name}: warmup {i + 1}/{warmup} done")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        step()
        log(f"{name}: step {i + 1}/{steps} done")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ctx.set_timing(True)
    ctx.reset_timing()
    for i in range(stage_steps):
        step()
    torch.cuda.synchronize()
    stages = ctx.stage_times()
    ctx.set_timing(False)
    log(f"{name}: {stage_steps} stage-timed steps done")
    applies = w.degree                       # (degree - 1) filter products + 1 in Rayleigh-Ritz
    log(f"{name}: {it[0]} iterations, Ritz values sum {float(lam.sum()):.15e} "
        f"top {float(lam[-1]):.15e}")
    return {"ms_per_step": 1e3 * dt / steps, "value": applies * nb * steps / dt,
            "stages": stages, "stage_steps": stage_steps, "applies": applies,
            "lam": lam.numpy().copy(), "max_resid": float(resid.max().cpu()), "sweeps": sweeps,
            "Y": Y, "HY": HY}


def lobpcg_leg(ctx, ham, w, X0, passes, nblock=4, nline=4):
    """Block LOBPCG (pw_lobpcg; the paper's run settings nblock_lobpcg = 4,
    nline = 4) from the random start block: one untimed pass (allocates the
    solver's workspace), then `passes` timed passes continuing the same
    iteration.  H*psi applications per pass: nb (nline + 1)."""
    import torch
    nb = w.nb
    Y = X0.clone()
    HY = torch.empty_like(Y)
    eig = torch.empty(nb, dtype=torch.float64, device="cuda")
    res = torch.empty_like(eig)
    ham.lobpcg(Y, HY, eig, res, nblock=nblock, nline=nline)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(passes):
        ham.lobpcg(Y, HY, eig, res, nblock=nblock, nline=nline, check=False)
        ctx.check_status()
        log(f"lobpcg: pass {i + 1}/{passes} done")
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / passes
    ctx.set_timing(True)
    ctx.reset_timing()
    ham.lobpcg(Y, HY, eig, res, nblock=nblock, nline=nline)
    st = ctx.stage_times()
    ctx.set_timing(False)
    applies = nb * (nline + 1)
    return {"ms_per_pass": 1e3 * dt, "value": applies / dt, "unit": UNIT,
            "nblock": nblock, "nline": nline, "applies_per_pass": applies,
            "max_resid": float(res.max().cpu()), "lowest_ritz_Ha": float(eig[0].cpu()),
            "stages_ms_per_pass": {k: v[0] for k, v in st.items() if v[1]}}


def rmm_leg(ctx, ham, w, Y0, HY0, passes, ndiis=3):
    """RMM-DIIS (pw_rmm_diis) from the Ritz vectors the FP64 filter path left
    (H Y carried in): `passes` timed passes; H*psi applications per pass:
    nb ndiis.  Residuals before and after say what the passes bought."""
    import torch
    nb = w.nb
    Y, HY = Y0.clone(), HY0.clone()
    eig = torch.empty(nb, dtype=torch.float64, device="cuda")
    res = torch.empty_like(eig)
    before = None
    # one untimed pass allocates the solver's workspace
    Yw, HYw = Y.clone(), HY.clone()
    ham.rmm_diis(Yw, HYw, eig, res, ndiis=ndiis, hy_valid=True)
    del Yw, HYw
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(passes):
        ham.rmm_diis(Y, HY, eig, res, ndiis=ndiis, hy_valid=True, check=False)
        ctx.check_status()
        if before is None:
            before = float(res.max().cpu())
        log(f"rmm-diis: pass {i + 1}/{passes} done")
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / passes
    applies = nb * ndiis
    return {"ms_per_pass": 1e3 * dt, "value": applies / dt, "unit": UNIT, "ndiis": ndiis,
            "applies_per_pass": applies, "max_resid_after_first_pass": before,
            "max_resid_after_last_pass": float(res.max().cpu()),
            "start": "Ritz vectors and H Y of the FP64 filter path's last iteration"}


def batch_roofline(stages, items, prec, degree):
    """Dominant kernel of a directly issued batch iteration (per-branch HIP
    events; concurrent branches overlap, so durations include sharing)."""
    elem = 16 if prec == "fp64" else 8
    sfx = "_lp" if prec != "fp64" else ""
    cand = {k[:len(k) - len(sfx)] if sfx else k: v for k, v in stages.items()
            if k in tuple(n + sfx for n in ("nonlocal", "proj", "fft_plane", "fft_col_inv",
                                            "fft_col_fwd")) and v[1] > 0}
    dom = max(cand, key=lambda k: cand[k][0])
    total_ms, launches = cand[dom]
    # one iteration: degree-1 filter products in the filter precision (the
    # Rayleigh-Ritz product of the mixed path is FP64 and timed elsewhere)
    units = []
    for w, ham in items:
        N1, N2, N3 = w.box
        nc, xr = ham.ncolumns, ham.extent1
        pairs = ((elem, degree - 1),) if sfx else ((elem, degree),)
        for e, napp in pairs:
            if dom == "fft_col_inv":
                units.append(e * (w.npw + nc * N3) * w.nb * napp)
            elif dom == "fft_col_fwd":
                units.append(e * (nc * N3 + 2 * w.npw) * w.nb * napp)
            elif dom == "fft_plane":
                units.append(e * 2 * nc * N3 * w.nb * napp)
            else:
                units.append(e * (w.npw * w.nproj + w.nproj * w.nb + w.npw * w.nb) * napp)
    total_bytes = sum(units)
    ach = total_bytes / (total_ms * 1e-3) / 1e9
    return {"kernel": dom, "bound": "hbm", "achieved": ach, "peak": PEAK["hbm_gbs"], "unit": "GB/s",
            "frac": ach / PEAK["hbm_gbs"], "traffic": None, "avg_launch_ms": total_ms / launches,
            "per_launch": f"algorithmic bytes of all {len(items)} items over one iteration "
                          f"({total_bytes:.4g} B) / summed kernel time",
            "note": "latency-bound configuration: kernels of concurrent branches overlap"}


def run_batch(args):
    print(json.dumps(batch_leg(args.config, args.precision, args.steps, args.warmup, args.streams,
                               args.graph, args.no_autotune, args.no_compare,
                               args.no_cpu_baseline, args.cpu_bands)), flush=True)


def batch_leg(config, precision, steps, warmup, streams=8, graph="fused", no_autotune=False,
              no_compare=False, no_cpu_baseline=False, cpu_bands=0):
    """C2 / C4: all items in one pw_batch (graph replays), against the plain
    FP64 per-item path (host-driven iterations, one item after another).
    The roofline comes from one more iteration of the same fused launches
    issued without the graph, each stage timed with HIP events."""
    import argparse as _ap
    args = _ap.Namespace(config=config, precision=precision, steps=steps, warmup=warmup,
                         streams=streams, graph=graph, no_autotune=no_autotune,
                         no_compare=no_compare, no_cpu_baseline=no_cpu_baseline,
                         cpu_bands=cpu_bands)
    import numpy as np
    import torch
    import synth
    import paper_2507_08578_amd as pw
    ws = make_workload(args.config)
    mixed = args.precision != "fp64"
    log(f"{len(ws)} items, npw {min(w.npw for w in ws)}-{max(w.npw for w in ws)}, "
        f"nb {min(w.nb for w in ws)}-{max(w.nb for w in ws)}")
    ctx = pw.Context(0)
    hams = [pw.Hamiltonian.from_workload(ctx, w, nb_max=w.nb, low_prec=mixed) for w in ws]
    X0 = [torch.from_numpy(synth.start_block(w.npw, w.nb, 100 + i)).cuda() for i, w in enumerate(ws)]
    degree = ws[0].degree
    bands = sum(w.nb for w in ws)
    tuning = None
    if not args.no_autotune:
        t0 = time.perf_counter()
        res = [h.autotune(args.precision, nb=w.nb, reps=3) for h, w in zip(hams, ws)]
        tuning = {"items_tuned": len(res),
                  "apply_ms_default_sum": sum(r["default_ms"] for r in res),
                  "apply_ms_tuned_sum": sum(r["ms"] for r in res),
                  "choices": sorted({json.dumps({k: r[k] for k in ("reg_col", "reg_plane",
                                                                   "plane_variant",
                                                                   "plane_variant32", "chunk",
                                                                   "gemm_blocks")})
                                     for r in res}),
                  "tuning_s": time.perf_counter() - t0}
        log(f"autotuned {len(res)} items in {tuning['tuning_s']:.1f} s")
    bt = pw.Batch(ctx, hams, X0, degree=degree, filter_prec=args.precision,
                  nstreams=args.streams)
    bt.start()
    gmode = False if args.graph == "none" else args.graph
    bt.iterate(args.warmup, graph=gmode)
    log("batch warmup done")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        bt.iterate(1, graph=gmode)
        log(f"batch step {i + 1}/{args.steps} done")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    lam_batch = bt.eigenvalues()
    sweeps = bt.max_sweeps()
    max_resid = max(float(r.max().cpu()) for r in bt.resid)
    # one more iteration of the timed launches issued without the graph, stage-timed
    ctx.set_timing(True)
    ctx.reset_timing()
    bt.iterate(1, graph="fused_direct" if gmode == "fused" else False)
    stages = ctx.stage_times()
    ctx.set_timing(False)
    roof = batch_roofline(stages, list(zip(ws, hams)), args.precision, degree)
    roof["timed_launches"] = ("the fused launches (one per stage for all items of a box), "
                              "issued directly with per-stage HIP events"
                              if gmode == "fused" else "per-item kernels issued directly")
    value = bands * degree * args.steps / dt
    out = {
        "metric": METRIC, "value": value, "unit": UNIT, "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * dt / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if not mixed else ("f32+f64" if args.precision == "fp32" else "bf16/f32+f64"),
        "data": "synthetic",
        "config": {"workload": f"{args.config}: {WORKLOADS[args.config]}",
                   "filter_precision": args.precision, "subspace_precision": "fp64",
                   "items": len(ws), "bands_total": bands, "streams": args.streams,
                   "graph": args.graph,
                   "step": f"one iteration of every item: filter (degree {degree}, H*Y reused) "
                           "+ Cholesky + Rayleigh-Ritz, replayed from HIP graphs"},
        "filter_iter_ms": 1e3 * dt / args.steps,
        "max_resid": max_resid, "eigensolver_max_sweeps": sweeps,
        "roofline": roof,
        "autotune": tuning,
    }
    bt.close()
    if not args.no_compare:
        # plain FP64 path: per-item handles and host-driven iterations, item after item
        hams64 = hams if not mixed else [pw.Hamiltonian.from_workload(ctx, w, nb_max=w.nb)
                                         for w in ws]
        if mixed and not args.no_autotune:
            for h, w in zip(hams64, ws):
                h.autotune("fp64", nb=w.nb, reps=3)
        states = []
        for h, x in zip(hams64, X0):
            Y = x.clone()
            HY = torch.empty_like(Y)
            eig = torch.empty(Y.shape[0], dtype=torch.float64, device="cuda")
            res = torch.empty_like(eig)
            h.orthonormalize(Y)
            h.rayleigh_ritz(Y, HY, eig, res)
            states.append([h, Y, HY, eig, res, eig.cpu(), h.upper_bound()])

        def step_all():
            for st in states:
                h, Y, HY, eig, res, lam, b = st
                h.cheb_filter(Y, degree, float(lam[-1]), b, float(lam[0]), hx=HY)
                h.orthonormalize(Y, check=False)
                h.rayleigh_ritz(Y, HY, eig, res, check=False)
                ctx.check_status()
                st[5] = eig.cpu()

        for _ in range(args.warmup):
            step_all()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(args.steps):
            step_all()
            log(f"per-item fp64 step {i + 1}/{args.steps} done")
        torch.cuda.synchronize()
        dt64 = time.perf_counter() - t0
        d = max(float(np.abs(lb - st[5].numpy()).max()) for lb, st in zip(lam_batch, states))
        out["fp64_per_item_path"] = {"ms_per_step": 1e3 * dt64 / args.steps,
                                     "value": bands * degree * args.steps / dt64,
                                     "speedup_batch_over_per_item": dt64 / dt}
        out["eig_diff_vs_fp64_Ha"] = d
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_items(ws, args.cpu_bands or 32)
    return out


def cpu_baseline_items(ws, nb_each, min_s=10.0, max_reps=10000):
    """Oracle H*psi on nb_each bands of every item, timed on the host; the
    pass over all items is repeated until at least min_s seconds have run."""
    import oracle
    import synth
    hc = host_cpu()
    threads = min(max(hc["blas_threads"], hc["fft_workers"]), hc["cpus_allowed"])
    hs = [oracle.OracleHam.from_workload(w) for w in ws]
    Xs = [synth.start_block(w.npw, min(nb_each, w.nb), 7).T for w in ws]
    oracle.apply_h(hs[0], Xs[0][:, :1])
    t0 = time.perf_counter()
    n = reps = 0
    while True:
        for h, X in zip(hs, Xs):
            oracle.apply_h(h, X)
            n += X.shape[1]
        reps += 1
        dt = time.perf_counter() - t0
        if dt >= min_s or reps >= max_reps:
            break
    return {"value": n / dt, "unit": UNIT, "cores": int(threads), "kind": "oracle",
            "sample": f"{reps} passes of one FP64 oracle H*psi on {min(nb_each, max(w.nb for w in ws))}"
                      f" bands of each of the {len(ws)} items ({n} band applies), {dt:.1f} s", **hc}


def calibrate_copy(nbytes=1 << 30, reps=3):
    """A plain device-to-device copy of known size: the reference that scales
    the HBM byte counters (FETCH_SIZE, WRITE_SIZE) of a profiled run."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "copies": reps}),
          flush=True)


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
    ap.add_argument("--no-density", action="store_true",
                    help="skip the electron-density measurement")
    ap.add_argument("--cpu-bands", type=int, default=0, help="oracle band sample (0 = auto)")
    ap.add_argument("--streams", type=int, default=8, help="batch branches (C2, C4)")
    ap.add_argument("--graph", default="fused", choices=["single", "per_stream", "fused", "none"],
                    help="batch replay mode (C2, C4)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default launch shapes instead of timing alternatives")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a 1 GiB device copy (reference for HBM byte counters)")
    ap.add_argument("--stage-steps", type=int, default=3,
                    help="extra stage-timed steps after the timed ones (roofline, stage split)")
    ap.add_argument("--overlap", action="store_true",
                    help="run P^H psi on a second stream beside the FFT route")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the bf16->FP32 ladder and low-precision Gram runs")
    ap.add_argument("--no-solvers", action="store_true",
                    help="skip the LOBPCG and RMM-DIIS legs")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the batched C2 / C4 legs of the default run")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU; --gpus must be 1"}))
        sys.exit(2)
    if args.calibrate_copy:
        return calibrate_copy()
    if args.config in BATCHED:
        return run_batch(args)

    import torch
    import synth
    import paper_2507_08578_amd as pw

    log(f"generating workload {args.config}")
    w = make_workload(args.config)
    nb = w.nb
    log(f"npw={w.npw} nproj={w.nproj} box={w.box} nb={nb} degree={w.degree}")
    ctx = pw.Context(0)
    ctx.set_overlap(args.overlap)
    mixed = args.precision != "fp64"
    ham = pw.Hamiltonian.from_workload(ctx, w, nb_max=nb, low_prec=mixed)
    X0 = torch.from_numpy(synth.start_block(w.npw, nb, 0)).cuda()
    log("upper bound")
    b = ham.upper_bound()
    tunings = {}

    def tune(prec):
        if args.no_autotune:
            return
        t0 = time.perf_counter()
        r = ham.autotune(prec, nb=nb, reps=2)
        r["tuning_s"] = time.perf_counter() - t0
        tunings[prec] = r
        log(f"autotune {prec}: {r}")

    tune(args.precision)
    ss = max(1, args.stage_steps)
    res = run_path(pw, ctx, ham, w, X0, b, args.precision, args.steps, args.warmup, ss)
    # (before the FP64 run retunes the handle: the roofline names the kernels just timed)
    roof = roofline(res["stages"], ss, w, ham, nb, args.precision, args.config)
    ref = None
    if mixed and not args.no_compare:
        tune("fp64")
        ref = run_path(pw, ctx, ham, w, X0, b, "fp64", args.steps, args.warmup, ss)
        ref_roof = roofline(ref["stages"], ss, w, ham, nb, "fp64", args.config)
    dtype = "f64" if not mixed else ("f32+f64" if args.precision == "fp32" else "bf16/f32+f64")
    out = {
        "metric": METRIC, "value": res["value"], "unit": UNIT, "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": res["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": dtype, "data": "synthetic",
        "config": {"workload": f"{args.config}: {WORKLOADS[args.config]}",
                   "filter_precision": args.precision, "subspace_precision": "fp64",
                   "step": f"filter (degree {w.degree}, H*Y reused) + Cholesky + Rayleigh-Ritz",
                   "applies_per_step": res["applies"], "nb": nb,
                   "proj_overlap": args.overlap},
        "filter_iter_ms": res["ms_per_step"],
        "max_resid": res["max_resid"],
        "eigensolver_sweeps": res["sweeps"],
        "roofline": roof,
        "stages_ms_per_step": {k: v[0] / ss for k, v in res["stages"].items()},
        "stage_timing": f"{ss} further steps with per-stage HIP events after the timed steps "
                        "(the timed steps record no events)",
        "autotune": tunings or None,
    }
    if ref is not None:
        d = float(abs(res["lam"] - ref["lam"]).max())
        # the valence bands of the diamond cells (4 electrons per atom, two per
        # band): the states a calculation keeps; the bands above them are the
        # block's buffer, still converging after a few iterations
        nocc = min(nb, 2 * w.cell.natoms)
        d_occ = lambda a, r: float(abs(a[:nocc] - r[:nocc]).max())
        out["fp64_path"] = {"ms_per_step": ref["ms_per_step"], "value": ref["value"],
                            "speedup_mixed_over_fp64": ref["ms_per_step"] / res["ms_per_step"],
                            "max_resid": ref["max_resid"], "roofline": ref_roof,
                            "stages_ms_per_step": {k: v[0] / ss
                                                   for k, v in ref["stages"].items()}}
        out["eig_diff_vs_fp64_Ha"] = d
        out["eig_diff_vs_fp64_occupied_Ha"] = d_occ(res["lam"], ref["lam"])
        out["occupied_bands"] = nocc
    if ref is not None and args.precision == "fp32" and not args.no_variants:
        # the other mixed forms over the same number of iterations from the same
        # start: the bf16 -> FP32 filter ladder, and the low-precision first
        # Gram pass (Cholesky QR twice); each against the FP64 trajectory
        if args.precision in tunings:
            ham.set_tuning(tunings[args.precision])
        total = args.warmup + args.steps + ss
        # bf16 for the first third of the iterations, then FP32 filters clean up
        switch = max(1, total // 3)
        lad = run_path(pw, ctx, ham, w, X0, b, lambda t: "bf16" if t <= switch else "fp32",
                       args.steps, args.warmup, ss)
        out["ladder_bf16_fp32"] = {
            "ms_per_step": lad["ms_per_step"], "value": lad["value"],
            "schedule": f"bf16 projector operands for iterations 1..{switch}, FP32 after "
                        f"({total} iterations in all)",
            "eig_diff_vs_fp64_Ha": float(abs(lad["lam"] - ref["lam"]).max()),
            "eig_diff_vs_fp64_occupied_Ha": d_occ(lad["lam"], ref["lam"]),
            "eig_diff_vs_fp32_Ha": float(abs(lad["lam"] - res["lam"]).max()),
            "max_resid": lad["max_resid"]}
        del lad
        gq = run_path(pw, ctx, ham, w, X0, b, "fp32", args.steps, args.warmup, ss, gram_prec="bf16")
        out["gram_bf16_cholqr2"] = {
            "ms_per_step": gq["ms_per_step"], "value": gq["value"],
            "form": "FP32 filter; orthonormalisation with a bf16 Gram pass then the FP64 pass",
            "eig_diff_vs_fp64_Ha": float(abs(gq["lam"] - ref["lam"]).max()),
            "eig_diff_vs_fp64_occupied_Ha": d_occ(gq["lam"], ref["lam"]),
            "eig_diff_vs_fp32_Ha": float(abs(gq["lam"] - res["lam"]).max()),
            "gram_ms_per_step": gq["stages"]["gram"][0] / ss,
            "max_resid": gq["max_resid"]}
        del gq
        if "fp64" in tunings:
            ham.set_tuning(tunings["fp64"])
    if not args.no_solvers:
        log("LOBPCG")
        out["lobpcg"] = lobpcg_leg(ctx, ham, w, X0, passes=2 if args.config == "C5" else 4)
        src = ref if ref is not None else res
        log("RMM-DIIS")
        out["rmm_diis"] = rmm_leg(ctx, ham, w, src["Y"], src["HY"], passes=3)
        out["rmm_diis"]["chfsi_fp64_iteration_ms"] = src["ms_per_step"]
    if not args.no_density:
        log("electron density")
        out["density"] = density_leg(ctx, ham, w, X0, args.steps, args.warmup, args.config)
        if not args.no_cpu_baseline:
            nbd = {"C1": 2048, "C3": 256, "C5": 64}[args.config]
            out["density"]["cpu_baseline"] = cpu_density_baseline(w, nbd)
    if not args.no_cpu_baseline:
        nbs = args.cpu_bands or {"C1": 2048, "C3": 64, "C5": 160}[args.config]
        log(f"cpu baseline: oracle H*psi on {nbs} bands")
        out["cpu_baseline"] = cpu_baseline(w, nbs)
    if args.config == "C5" and not args.no_batched:
        # the batched forms, measured by every default run (each its own line's
        # fields; the headline above is C5)
        del res, ref
        ham.close()
        torch.cuda.empty_cache()
        out["batched"] = {}
        for cfg, prec in (("C2", "fp64"), ("C4", "fp32")):
            log(f"batched leg {cfg} ({prec})")
            out["batched"][cfg] = batch_leg(cfg, prec, min(args.steps, 10), max(1, args.warmup),
                                            no_cpu_baseline=args.no_cpu_baseline, cpu_bands=16)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
