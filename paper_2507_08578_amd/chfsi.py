"""Chebyshev-filtered block subspace iteration driven through the C ABI
(section 5.1: filtering keeps Rayleigh-Ritz calls few and leans on H*psi).

Iteration 0 orthonormalises the start block and runs Rayleigh-Ritz.  Each
later iteration filters with a = largest Ritz value, a0 = smallest,
b = the spectral upper bound, then orthonormalises (Cholesky) and runs
Rayleigh-Ritz.  With reuse_hx the W = H Y left by Rayleigh-Ritz serves as
the filter's first product (H (Y Q) = (H Y) Q, exact up to rounding).
The only host reads per iteration are the deferred status of the
orthonormalisation and Rayleigh-Ritz (pw_ctx_check) and the Ritz values that
set the next filter interval.
"""
from __future__ import annotations

import dataclasses
from typing import Callable, List, Optional


@dataclasses.dataclass
class ChfsiState:
    Y: object                 # (nb, npw) complex128 CUDA tensor, orthonormal Ritz vectors
    HY: object                # H Y
    eig: object               # (nb,) float64 CUDA tensor, ascending Ritz values
    resid: object             # (nb,) float64 CUDA tensor, ||H y - lambda y||
    upper: float
    eig_history: List = dataclasses.field(default_factory=list)
    resid_history: List = dataclasses.field(default_factory=list)
    applies: int = 0          # H*psi block applications executed


def chfsi(ham, X0, degree: int, iters: int, upper: Optional[float] = None,
          reuse_hx: bool = True, record: bool = True, filter_prec="fp64", gram_prec="fp64",
          callback: Optional[Callable[[int, ChfsiState], None]] = None) -> ChfsiState:
    """filter_prec: "fp64", "fp32", "bf16", or a callable t -> precision for
    iteration t (a precision ladder, e.g. bf16 early and fp32 late).
    gram_prec: precision of the first Gram matrix of the orthonormalisation
    ("fp32" / "bf16" add a low-precision Cholesky-QR pass before the FP64
    one).  The factorisations and Rayleigh-Ritz always run in FP64."""
    import torch
    nb = X0.shape[0]
    Y = X0.clone()
    HY = torch.empty_like(Y)
    eig = torch.empty(nb, dtype=torch.float64, device=Y.device)
    resid = torch.empty(nb, dtype=torch.float64, device=Y.device)
    b = ham.upper_bound() if upper is None else float(upper)
    st = ChfsiState(Y=Y, HY=HY, eig=eig, resid=resid, upper=b)
    ham.orthonormalize(Y, check=False)
    ham.rayleigh_ritz(Y, HY, eig, resid, check=False)
    ham.ctx.check_status()
    st.applies += 1
    lam = eig.cpu()
    if record:
        st.eig_history.append(lam.numpy().copy())
        st.resid_history.append(resid.cpu().numpy().copy())
    if callback:
        callback(0, st)
    for t in range(1, iters + 1):
        fp = filter_prec(t) if callable(filter_prec) else filter_prec
        ham.cheb_filter(Y, degree, float(lam[-1]), b, float(lam[0]), hx=HY if reuse_hx else None,
                        prec=fp)
        st.applies += degree - 1 if reuse_hx else degree
        ham.orthonormalize(Y, gram_prec=gram_prec, check=False)
        ham.rayleigh_ritz(Y, HY, eig, resid, check=False)
        ham.ctx.check_status()
        st.applies += 1
        lam = eig.cpu()
        if record:
            st.eig_history.append(lam.numpy().copy())
            st.resid_history.append(resid.cpu().numpy().copy())
        if callback:
            callback(t, st)
    return st
