"""MI355X plane-wave H*psi + Chebyshev-filtered subspace iteration (arXiv 2507.08578, section 5).

Python face of libpwdft.so: a thin ctypes layer over the C ABI in include/pw.h.
PyTorch supplies device memory and streams; every step of the path runs in
the library's HIP kernels.  Blocks of bands are complex128 CUDA tensors of
shape (nb, npw) whose rows are bands (column-major npw x nb with leading
dimension tensor.stride(0)).
"""
from __future__ import annotations

import ctypes
from typing import Optional

import numpy as np

from . import _lib
from ._lib import PWError, PW_FP64, PW_FP32, PW_BF16, STAGES  # noqa: F401

_LIB = _lib.load()


def lib() -> ctypes.CDLL:
    return _LIB


def version() -> str:
    return _LIB.pw_version().decode()


def status_string(s: int) -> str:
    return _LIB.pw_status_string(s).decode()


def _check(status: int, ctx_handle=None):
    if status != _lib.PW_OK:
        msg = _LIB.pw_last_error(ctx_handle).decode()
        raise PWError(status, f"{status_string(status)}: {msg}")


PRECISIONS = {"fp64": PW_FP64, "fp32": PW_FP32, "bf16": PW_BF16}


def _prec(p) -> int:
    if isinstance(p, str):
        if p not in PRECISIONS:
            raise ValueError(f"precision must be one of {sorted(PRECISIONS)}")
        return PRECISIONS[p]
    return int(p)


def to_bf16_pairs(x):
    """A complex block (nb, npw) as the bf16-pair storage of PW_BF16: a
    bfloat16 tensor (nb, npw, 2), each part rounded to nearest even."""
    import torch
    return torch.view_as_real(x.to(torch.complex64)).to(torch.bfloat16).contiguous()


def from_bf16_pairs(t):
    """bf16-pair block (nb, npw, 2) -> complex64 (nb, npw), exactly."""
    import torch
    return torch.view_as_complex(t.to(torch.float32).contiguous())


def _bf16_block_args(t, npw: int, name: str):
    import torch
    if (not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.bfloat16
            or t.dim() != 3 or t.shape[1] != npw or t.shape[2] != 2 or t.stride(2) != 1
            or t.stride(1) != 2 or t.stride(0) % 2):
        raise TypeError(f"{name} must be a bfloat16 CUDA tensor (nb, npw={npw}, 2) of "
                        "interleaved (re, im) pairs, contiguous along npw")
    return ctypes.c_void_p(t.data_ptr()), t.stride(0) // 2


def _block_args(t, npw: int, name: str, complex64: bool = False):
    import torch
    want = torch.complex64 if complex64 else torch.complex128
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != want:
        raise TypeError(f"{name} must be a {want} CUDA tensor")
    if t.dim() != 2 or t.shape[1] != npw or t.stride(1) != 1:
        raise ValueError(f"{name} must have shape (nb, npw={npw}) with unit stride along npw")
    return ctypes.c_void_p(t.data_ptr()), t.stride(0)


class Context:
    """pw_ctx on one HIP device and stream (default: torch's current stream)."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        handle = ctypes.c_void_p()
        sh = ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else stream)
        _check(_LIB.pw_ctx_create(device, sh, ctypes.byref(handle)))
        self.handle = handle
        self.device = device

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            _LIB.pw_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def check(self, status: int):
        _check(status, self.handle)

    def check_status(self):
        """Wait for the context's stream and raise the first failure the hot
        calls recorded on the device since the last check (pw_ctx_check)."""
        self.check(_LIB.pw_ctx_check(self.handle))

    def set_overlap(self, enable: bool):
        """P^H psi on a second stream beside the FFT route (pw_ctx_set_overlap)."""
        self.check(_LIB.pw_ctx_set_overlap(self.handle, int(bool(enable))))

    def set_sweep_limit(self, max_sweeps: int):
        self.check(_LIB.pw_ctx_set_sweep_limit(self.handle, int(max_sweeps)))

    # --- stage timing ---
    def set_timing(self, enable: bool):
        self.check(_LIB.pw_ctx_set_timing(self.handle, int(enable)))

    def reset_timing(self):
        self.check(_LIB.pw_ctx_reset_timing(self.handle))

    def last_sweeps(self) -> int:
        n = ctypes.c_int()
        self.check(_LIB.pw_ctx_last_sweeps(self.handle, ctypes.byref(n)))
        return n.value

    def stage_times(self) -> dict:
        out = {}
        for i, name in enumerate(STAGES):
            ms = ctypes.c_double()
            n = ctypes.c_int64()
            self.check(_LIB.pw_ctx_stage_time(self.handle, i, ctypes.byref(ms), ctypes.byref(n)))
            out[name] = (ms.value, n.value)
        return out

    # --- dense building blocks (complex128 column-major = torch (ncols, nrows) row-major) ---
    def gemm_cn(self, A, B, alpha: float = 1.0):
        """C = alpha A^H B for A (m, k) and B (n, k) tensors holding column-major k x m / k x n."""
        import torch
        m, k = A.shape
        n = B.shape[0]
        C = torch.empty((n, m), dtype=torch.complex128, device=A.device)
        self.check(_LIB.pw_gemm_cn(self.handle, m, n, k, alpha, A.data_ptr(), A.stride(0),
                                   B.data_ptr(), B.stride(0), C.data_ptr(), C.stride(0)))
        return C

    def gemm_nn(self, A, B, alpha: float = 1.0, beta: float = 0.0, C=None):
        """C = alpha A B + beta C, column-major A (m x k) as tensor (k, m), B (k x n) as (n, k)."""
        import torch
        k, m = A.shape
        n = B.shape[0]
        if C is None:
            C = torch.zeros((n, m), dtype=torch.complex128, device=A.device)
        self.check(_LIB.pw_gemm_nn(self.handle, m, n, k, alpha, A.data_ptr(), A.stride(0),
                                   B.data_ptr(), B.stride(0), beta, C.data_ptr(), C.stride(0)))
        return C

    def heev(self, A):
        """Eigen-decomposition of a Hermitian matrix held column-major in tensor (n, n).
        Returns (w ascending, Q column-major in a tensor (n, n))."""
        import torch
        n = A.shape[0]
        a = A.clone()
        w = torch.empty(n, dtype=torch.float64, device=A.device)
        Q = torch.empty((n, n), dtype=torch.complex128, device=A.device)
        self.check(_LIB.pw_heev(self.handle, n, a.data_ptr(), a.stride(0), w.data_ptr(),
                                Q.data_ptr(), Q.stride(0)))
        return w, Q

    def heev_noalloc(self, A, w=None, Q=None, check=True):
        """pw_heev_noalloc: the same eigensolver with its workspace in the
        library's static device array (n <= 512).  w, Q: optional outputs
        (float64 (n,), complex128 (n, n) CUDA tensors); A is not modified."""
        import torch
        n = A.shape[0]
        if w is None:
            w = torch.empty(n, dtype=torch.float64, device=A.device)
        if Q is None:
            Q = torch.empty((n, n), dtype=torch.complex128, device=A.device)
        self.check(_LIB.pw_heev_noalloc(self.handle, n, A.data_ptr(), A.stride(0), w.data_ptr(),
                                        Q.data_ptr(), Q.stride(0)))
        if check:
            self.check_status()
        return w, Q

    def potrf_inv(self, S):
        """Upper Cholesky S = U^H U and U^{-1}, column-major tensors (n, n)."""
        import torch
        n = S.shape[0]
        U = S.clone()
        X = torch.empty_like(S)
        self.check(_LIB.pw_potrf_inv(self.handle, n, U.data_ptr(), U.stride(0), X.data_ptr(),
                                     X.stride(0)))
        return U, X


class Hamiltonian:
    """pw_ham: H at one k-point (section 5.2, Eq. ham-nl, norm-conserving form).

    miller: (npw, 3) int, recip: (3, 3) rows b_i, kpt: reduced (3,), box: (N1, N2, N3),
    vloc: float64 CUDA tensor (N3, N2, N1), proj: complex128 CUDA tensor (nproj, npw)
    (row j = projector j; kept referenced for the lifetime of this object),
    ekb: (nproj,) KB energies.
    """

    def __init__(self, ctx: Context, miller, recip, kpt, box, vloc, proj, ekb, nb_max: int,
                 low_prec: bool = False):
        import torch
        self.ctx = ctx
        miller = np.ascontiguousarray(np.asarray(miller, dtype=np.int32))
        if miller.ndim != 2 or miller.shape[1] != 3:
            raise ValueError("miller must be (npw, 3)")
        self.npw = int(miller.shape[0])
        if not (isinstance(vloc, torch.Tensor) and vloc.is_cuda and vloc.dtype == torch.float64
                and vloc.is_contiguous()):
            raise TypeError("vloc must be a contiguous float64 CUDA tensor (N3, N2, N1)")
        N1, N2, N3 = (int(x) for x in box)
        if tuple(vloc.shape) != (N3, N2, N1):
            raise ValueError(f"vloc shape {tuple(vloc.shape)} != (N3, N2, N1) = {(N3, N2, N1)}")
        self.nproj = 0 if proj is None else int(proj.shape[0])
        if self.nproj:
            if not (proj.is_cuda and proj.dtype == torch.complex128 and proj.is_contiguous()
                    and proj.shape[1] == self.npw):
                raise TypeError("proj must be a contiguous complex128 CUDA tensor (nproj, npw)")
        self._proj = proj                    # the library references this memory
        ekb = np.ascontiguousarray(np.asarray(ekb if ekb is not None else [], dtype=np.float64))
        self._miller = miller
        self._ekb = ekb
        d = _lib.PwHamDesc()
        d.n[:] = [N1, N2, N3]
        d.npw = self.npw
        d.miller = miller.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        d.recip[:] = [float(x) for x in np.asarray(recip, dtype=np.float64).reshape(9)]
        d.kpt[:] = [float(x) for x in np.asarray(kpt, dtype=np.float64).reshape(3)]
        d.vloc_dev = vloc.data_ptr()
        d.nproj = self.nproj
        d.proj_dev = proj.data_ptr() if self.nproj else None
        d.ekb = ekb.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if self.nproj else None
        d.nb_max = int(nb_max)
        d.low_prec = 1 if low_prec else 0
        self.nb_max = int(nb_max)
        self.low_prec = bool(low_prec)
        handle = ctypes.c_void_p()
        ctx.check(_LIB.pw_ham_create(ctx.handle, ctypes.byref(d), ctypes.byref(handle)))
        self.handle = handle
        vals = [ctypes.c_int64() for _ in range(5)]
        ctx.check(_LIB.pw_ham_info(handle, *[ctypes.byref(v) for v in vals]))
        self.ncolumns = vals[3].value
        self.extent1 = vals[4].value
        self.box = (N1, N2, N3)

    @staticmethod
    def from_workload(ctx: Context, w, nb_max: Optional[int] = None, device: str = "cuda",
                      low_prec: bool = False):
        """Build from a synth.Workload (arrays copied to the device here)."""
        import torch
        vloc = torch.from_numpy(np.ascontiguousarray(w.vloc)).to(device)
        proj = torch.from_numpy(np.ascontiguousarray(w.proj)).to(device) if w.nproj else None
        return Hamiltonian(ctx, w.miller, w.recip, w.kred, w.box, vloc, proj, w.ekb,
                           nb_max or w.nb, low_prec=low_prec)

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            _LIB.pw_ham_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # --- hot path ---
    def apply_h(self, psi, out=None, prec="fp64"):
        """H psi; complex128 blocks for fp64, complex64 for fp32, bf16-pair
        blocks (bfloat16 (nb, npw, 2), see to_bf16_pairs) for bf16."""
        import torch
        pr = _prec(prec)
        if out is None:
            out = torch.empty_like(psi)
        if pr == PW_BF16:
            p, ldp = _bf16_block_args(psi, self.npw, "psi")
            o, ldo = _bf16_block_args(out, self.npw, "out")
        else:
            c64 = pr != PW_FP64
            p, ldp = _block_args(psi, self.npw, "psi", c64)
            o, ldo = _block_args(out, self.npw, "out", c64)
        self.ctx.check(_LIB.pw_apply_h(self.handle, pr, psi.shape[0], p, ldp, o, ldo))
        return out

    def density(self, psi, w, rho=None, accumulate=False):
        """rho(r_j) [+]= (1/Omega) sum_b w_b |psi_b(r_j)|^2 on the box, float64 (N3, N2, N1).

        psi: complex128 block (nb, npw); w: float64 CUDA tensor of nb weights
        (occupation x k-point weight); accumulate adds to rho instead of
        overwriting it."""
        import torch
        p, ldp = _block_args(psi, self.npw, "psi")
        nb = psi.shape[0]
        if (not isinstance(w, torch.Tensor) or not w.is_cuda or w.dtype != torch.float64
                or w.dim() != 1 or w.shape[0] != nb or not w.is_contiguous()):
            raise TypeError(f"w must be a contiguous float64 CUDA tensor of {nb} weights")
        N1, N2, N3 = self.box
        if rho is None:
            rho = torch.empty((N3, N2, N1), dtype=torch.float64, device=psi.device)
        if (not isinstance(rho, torch.Tensor) or not rho.is_cuda or rho.dtype != torch.float64
                or not rho.is_contiguous() or rho.numel() != N1 * N2 * N3):
            raise TypeError(f"rho must be a contiguous float64 CUDA tensor of {N1 * N2 * N3} values")
        self.ctx.check(_LIB.pw_density(self.handle, nb, p, ldp, ctypes.c_void_p(w.data_ptr()),
                                       ctypes.c_void_p(rho.data_ptr()), int(bool(accumulate))))
        return rho

    def cheb_filter(self, y, degree: int, a: float, b: float, a0: float, hx=None, prec="fp64"):
        """y <- p_m(H) y in place (complex128 block; prec selects the internal arithmetic)."""
        p, ld = _block_args(y, self.npw, "y")
        if hx is not None:
            hp, ldh = _block_args(hx, self.npw, "hx")
        else:
            hp, ldh = None, 0
        self.ctx.check(_LIB.pw_cheb_filter(self.handle, _prec(prec), int(degree), float(a),
                                           float(b), float(a0), y.shape[0], p, ld, hp, ldh))
        return y

    def orthonormalize(self, y, hy=None, gram_prec="fp64", check=True):
        """Cholesky orthonormalisation in place.  check: wait and raise a
        failing pivot now (pw_ctx_check); False leaves it to a later check."""
        p, ld = _block_args(y, self.npw, "y")
        if hy is not None:
            hp, ldh = _block_args(hy, self.npw, "hy")
        else:
            hp, ldh = None, 0
        self.ctx.check(_LIB.pw_orthonormalize(self.handle, _prec(gram_prec), y.shape[0], p, ld,
                                              hp, ldh))
        if check:
            self.ctx.check_status()
        return y

    def rayleigh_ritz(self, y, hy, eig, resid=None, check=True):
        import torch
        p, ld = _block_args(y, self.npw, "y")
        hp, ldh = _block_args(hy, self.npw, "hy")
        for t, nm in ((eig, "eig"), (resid, "resid")):
            if t is not None and not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()
                                      and t.numel() >= y.shape[0]):
                raise TypeError(f"{nm} must be a float64 CUDA tensor of >= nb elements")
        self.ctx.check(_LIB.pw_rayleigh_ritz(self.handle, y.shape[0], p, ld, hp, ldh,
                                             eig.data_ptr(),
                                             resid.data_ptr() if resid is not None else None))
        if check:
            self.ctx.check_status()
        return eig

    @staticmethod
    def _dvec(t, n, name):
        import torch
        if t is None:
            return None
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64
                and t.is_contiguous() and t.numel() >= n):
            raise TypeError(f"{name} must be a contiguous float64 CUDA tensor of >= {n} elements")
        return t.data_ptr()

    def lobpcg(self, y, hy, eig, resid=None, nblock: int = 1, nline: int = 4, hist=None,
               check=True):
        """One block-LOBPCG pass in place (pw_lobpcg): y <- Ritz vectors, hy <- H y.
        hist (optional): float64 tensor of (nline + 1) * nb Ritz values per line."""
        p, ld = _block_args(y, self.npw, "y")
        hp, ldh = _block_args(hy, self.npw, "hy")
        nb = y.shape[0]
        self.ctx.check(_LIB.pw_lobpcg(self.handle, nb, int(nblock), int(nline), p, ld, hp, ldh,
                                      self._dvec(eig, nb, "eig"), self._dvec(resid, nb, "resid"),
                                      self._dvec(hist, (int(nline) + 1) * nb, "hist")))
        if check:
            self.ctx.check_status()
        return eig

    def rmm_diis(self, y, hy, eig, resid=None, ndiis: int = 3, hy_valid=False, band_resid=None,
                 check=True):
        """One RMM-DIIS pass in place (pw_rmm_diis): y <- Ritz vectors, hy <- H y.
        band_resid (optional): float64 tensor of (ndiis + 1) * nb relative residuals."""
        p, ld = _block_args(y, self.npw, "y")
        hp, ldh = _block_args(hy, self.npw, "hy")
        nb = y.shape[0]
        self.ctx.check(_LIB.pw_rmm_diis(self.handle, nb, int(ndiis), p, ld, hp, ldh,
                                        int(bool(hy_valid)), self._dvec(eig, nb, "eig"),
                                        self._dvec(resid, nb, "resid"),
                                        self._dvec(band_resid, (int(ndiis) + 1) * nb, "band_resid")))
        if check:
            self.ctx.check_status()
        return eig

    def cprj(self, nb: int, out=None):
        """Projections <p_j|y_b> of the Ritz vectors the last Rayleigh-Ritz,
        LOBPCG or RMM-DIIS call returned (pw_ham_cprj): complex128 tensor
        (nb, nproj), row b = band b."""
        import torch
        if out is None:
            out = torch.empty((nb, max(self.nproj, 1)), dtype=torch.complex128, device="cuda")
        self.ctx.check(_LIB.pw_ham_cprj(self.handle, int(nb), ctypes.c_void_p(out.data_ptr()),
                                        out.stride(0)))
        return out[:, :self.nproj]

    def upper_bound(self) -> float:
        b = ctypes.c_double()
        self.ctx.check(_LIB.pw_upper_bound(self.handle, ctypes.byref(b)))
        return b.value

    # --- launch-shape tuning ---
    _TUNING_KEYS = ("reg_col", "reg_plane", "plane_variant", "plane_variant32", "chunk",
                    "gemm_blocks", "nn_tile", "nn_tile32")

    def get_tuning(self) -> dict:
        t = _lib.PwTuning()
        self.ctx.check(_LIB.pw_ham_get_tuning(self.handle, ctypes.byref(t)))
        return {k: getattr(t, k) for k in self._TUNING_KEYS}

    def set_tuning(self, tuning: dict):
        t = _lib.PwTuning()
        cur = self.get_tuning()
        cur.update({k: int(v) for k, v in tuning.items() if k in self._TUNING_KEYS})
        for k in self._TUNING_KEYS:
            setattr(t, k, cur[k])
        self.ctx.check(_LIB.pw_ham_set_tuning(self.handle, ctypes.byref(t)))

    def tuning_key(self, prec, nb: int) -> str:
        """Shape key of the tuning cache (as pw_autotune writes it): box, sphere
        columns and extent, npw, nproj, nb, precision code."""
        N1, N2, N3 = self.box
        return (f"{N1}x{N2}x{N3}/cols{self.ncolumns}/xr{self.extent1}/npw{self.npw}/"
                f"proj{self.nproj}/nb{nb}/{_prec(prec)}")

    def autotune(self, prec="fp64", nb: Optional[int] = None, reps: int = 3,
                 cache: Optional[str] = None) -> dict:
        """Time launch-shape alternatives on the device and keep the fastest
        (pw_autotune).  cache: path of the library's tuning cache file; a hit
        is applied without timing, a miss is tuned and stored."""
        nb = int(nb or self.nb_max)
        best, init = _lib.PwTuning(), _lib.PwTuning()
        cached = ctypes.c_int32()
        path = cache.encode() if cache else None
        self.ctx.check(_LIB.pw_autotune(self.handle, _prec(prec), nb, int(reps), path,
                                        ctypes.byref(best), ctypes.byref(init),
                                        ctypes.byref(cached)))
        out = {k: getattr(best, k) for k in self._TUNING_KEYS}
        out.update(ms=best.ms, default_ms=init.ms, cached=bool(cached.value))
        return out


class Batch:
    """pw_batch: the Chebyshev-filtered subspace iteration of many independent
    Hamiltonians at once (k-points or cells), each iteration captured once into
    one HIP graph with a branch per item.

    hams: distinct Hamiltonians of one Context; X0s: start blocks, complex128
    CUDA tensors (nb_i, npw_i) with nb_i <= 64 (copied; the batch owns Y, HY,
    eig and resid, whose addresses live in the captured graph)."""

    def __init__(self, ctx: Context, hams, X0s, degree: int, filter_prec="fp64",
                 nstreams: int = 8):
        import torch
        if len(hams) != len(X0s) or not hams:
            raise ValueError("need one start block per Hamiltonian")
        self.ctx = ctx
        self.hams = list(hams)
        self.Y = [x.contiguous().clone() for x in X0s]
        for h, y in zip(self.hams, self.Y):
            _block_args(y, h.npw, "X0")
        self.HY = [torch.empty_like(y) for y in self.Y]
        self.eig = [torch.empty(y.shape[0], dtype=torch.float64, device=y.device) for y in self.Y]
        self.resid = [torch.empty_like(e) for e in self.eig]
        n = len(self.hams)
        ptrs = lambda ts: (ctypes.c_void_p * n)(*[t.data_ptr() for t in ts])  # noqa: E731
        hh = (ctypes.c_void_p * n)(*[h.handle.value for h in self.hams])
        nbs = (ctypes.c_int64 * n)(*[y.shape[0] for y in self.Y])
        handle = ctypes.c_void_p()
        ctx.check(_LIB.pw_batch_create(ctx.handle, n, hh, nbs, ptrs(self.Y), ptrs(self.HY),
                                       ptrs(self.eig), ptrs(self.resid), int(degree),
                                       _prec(filter_prec), int(nstreams), ctypes.byref(handle)))
        self.handle = handle
        self.degree = int(degree)

    def start(self):
        """Iteration 0: orthonormalise the start blocks, then Rayleigh-Ritz."""
        self.ctx.check(_LIB.pw_batch_start(self.handle))

    def iterate(self, iters: int = 1, graph=True):
        """graph: True / "single" (one graph, a branch per stream), "per_stream"
        (one graph per branch stream), "fused" (one launch per stage for all
        items of a box, replayed from a graph), "fused_direct" (the same
        launches issued without a graph; stage-timed when timing is on),
        False (per-item kernels issued directly)."""
        mode = {True: 1, "single": 1, "per_stream": 2, "fused": 3, "fused_direct": 4,
                False: 0}[graph]
        self.ctx.check(_LIB.pw_batch_iterate(self.handle, int(iters), mode))

    def chfsi(self, iters: int, graph="fused"):
        """The whole batched solve (pw_batch_chfsi): iteration 0, then iters
        iterations in the given replay mode (as iterate)."""
        mode = {True: 1, "single": 1, "per_stream": 2, "fused": 3, "fused_direct": 4,
                False: 0}[graph]
        self.ctx.check(_LIB.pw_batch_chfsi(self.handle, int(iters), mode))

    def max_sweeps(self) -> int:
        n = ctypes.c_int32()
        self.ctx.check(_LIB.pw_batch_max_sweeps(self.handle, ctypes.byref(n)))
        return n.value

    def eigenvalues(self):
        return [e.cpu().numpy().copy() for e in self.eig]

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            _LIB.pw_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


from .chfsi import chfsi, ChfsiState  # noqa: E402,F401
