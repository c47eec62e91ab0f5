"""FP64 CPU oracle of the two other iterative eigensolvers of section 5: LOBPCG
(the band-block conjugate-gradient solver that section 5.1 measures beside
Chebyshev filtering, with its block count and line count) and RMM-DIIS
(section 5.4: no orthogonalisation inside the band updates, one full-band
Cholesky orthogonalisation and one subspace rotation per call).

TEST INFRASTRUCTURE ONLY (see the package docstring): imported by tests/,
the smoke check and the benchmark's CPU-baseline leg, never by the library.

The paper names the solvers and cites their sources without giving their
steps; the steps below are the published algorithms as I read them:
  * LOBPCG (Knyazev 2001; in blocks of bands, each kept orthogonal to the
    blocks below it, as in the band-block scheme the paper cites): per block,
    nline iterations of Rayleigh-Ritz on span{X, W, P}, W the preconditioned
    residual, P the previous step's search direction.
  * RMM-DIIS (Kresse and Furthmuller 1996): per band, a first preconditioned
    step whose length comes from a line minimisation of the Rayleigh
    quotient, then DIIS steps that minimise the residual norm over the band's
    history; afterwards one Cholesky orthonormalisation and a Rayleigh-Ritz.
  * The preconditioner is Teter, Payne and Allan's (1989) kinetic-energy
    polynomial, the standard one of plane-wave codes.
Every reading is listed in the design notes of the repository.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np

from .pw_oracle import OracleHam, apply_h, kinetic, orthonormalize, rayleigh_ritz


# ----------------------------------------------------------------------------
# Preconditioner
# ----------------------------------------------------------------------------

def teter_factor(x: np.ndarray) -> np.ndarray:
    """K(x) = (27 + 18x + 12x^2 + 8x^3) / (27 + 18x + 12x^2 + 8x^3 + 16x^4):
    1 at x = 0, about 1/(2x) for large x (x = plane-wave kinetic energy over
    the band's kinetic energy)."""
    num = 27.0 + x * (18.0 + x * (12.0 + 8.0 * x))
    return num / (num + 16.0 * x ** 4)


def band_kinetic(ham: OracleHam, X: np.ndarray) -> np.ndarray:
    """<x_b|T|x_b> / <x_b|x_b> for every column x_b of X."""
    T = kinetic(ham)
    return np.sum(T[:, None] * np.abs(X) ** 2, axis=0) / np.sum(np.abs(X) ** 2, axis=0)


def precondition(ham: OracleHam, X: np.ndarray, R: np.ndarray) -> np.ndarray:
    """W[g, b] = K(T_g / Ekin_b) R[g, b], Ekin_b the kinetic energy of band x_b."""
    ek = band_kinetic(ham, X)
    return teter_factor(kinetic(ham)[:, None] / ek[None, :]) * R


# ----------------------------------------------------------------------------
# LOBPCG
# ----------------------------------------------------------------------------

def block_bounds(nb: int, nblock: int) -> List[tuple]:
    """nblock contiguous band blocks, sizes differing by at most one (the
    larger ones first)."""
    q, r = divmod(nb, nblock)
    out, lo = [], 0
    for j in range(nblock):
        hi = lo + q + (1 if j < r else 0)
        out.append((lo, hi))
        lo = hi
    return out


def _normalize_columns(B: np.ndarray, HB: Optional[np.ndarray] = None):
    s = 1.0 / np.linalg.norm(B, axis=0)
    return (B * s, None if HB is None else HB * s)


def _remove(B, HB, X, HX):
    """B <- B - X (X^H B), and HB alike with HX (X orthonormal)."""
    c = X.conj().T @ B
    return B - X @ c, (None if HB is None else HB - HX @ c)


@dataclasses.dataclass
class LobpcgResult:
    eig: np.ndarray            # Ritz values after the final Rayleigh-Ritz (ascending)
    Y: np.ndarray              # Ritz vectors
    HY: np.ndarray
    resid: np.ndarray          # ||H y_b - lambda_b y_b||
    block_history: List[List[np.ndarray]]   # per block: Ritz values after each line


def lobpcg(ham: OracleHam, X0: np.ndarray, nblock: int, nline: int,
           use_precond: bool = True) -> LobpcgResult:
    """One pass of block LOBPCG over the bands of X0 (npw x nb).

    The start block is orthonormalised (Cholesky).  Block j (bands lo:hi) is
    made orthogonal to the blocks below it (already updated in this pass),
    orthonormalised and Rayleigh-Ritzed; then, nline times:
      R = H X - X Lambda;  W = K R (K: Teter preconditioner);
      W orthogonal to the lower blocks and to X, orthonormal;  H W;
      P (from the second line on) orthogonal to X and W, orthonormal, with
      H P carried along;
      Rayleigh-Ritz on V = [X, W, P]: Hs = V^H H V, Hs Z = Z Theta (ascending);
      X <- V Z_m, H X <- (H V) Z_m, Lambda <- Theta_m (the m lowest),
      P <- [W, P] Z_m[m:], H P <- [H W, H P] Z_m[m:].
    The products H X and H P ride the rotations; H is applied to W only.
    Finally one Rayleigh-Ritz over all bands (with the carried H X).
    """
    X = orthonormalize(np.asarray(X0, dtype=np.complex128))
    npw, nb = X.shape
    HX = np.zeros_like(X)
    history = []
    for lo, hi in block_bounds(nb, nblock):
        m = hi - lo
        Xc, HXc = X[:, :lo], HX[:, :lo]
        Xj = X[:, lo:hi]
        if lo:
            Xj, _ = _remove(Xj, None, Xc, None)
        Xj = orthonormalize(Xj)
        HXj = apply_h(ham, Xj)
        Hs = Xj.conj().T @ HXj
        lam, Q = np.linalg.eigh(0.5 * (Hs + Hs.conj().T))
        Xj, HXj = Xj @ Q, HXj @ Q
        P = HP = None
        hist = [lam.copy()]
        for _ in range(nline):
            R = HXj - Xj * lam[None, :]
            W = precondition(ham, Xj, R) if use_precond else R.copy()
            if lo:
                W, _ = _remove(W, None, Xc, None)
            W, _ = _remove(W, None, Xj, None)
            W, _ = _normalize_columns(W)
            W = orthonormalize(W)
            HW = apply_h(ham, W)
            if P is None:
                V, HV = np.hstack([Xj, W]), np.hstack([HXj, HW])
            else:
                P, HP = _remove(P, HP, Xj, HXj)
                P, HP = _remove(P, HP, W, HW)
                P, HP = _normalize_columns(P, HP)
                P, HP = orthonormalize(P, HP)
                V, HV = np.hstack([Xj, W, P]), np.hstack([HXj, HW, HP])
            Hs = V.conj().T @ HV
            theta, Z = np.linalg.eigh(0.5 * (Hs + Hs.conj().T))
            Zm = Z[:, :m]
            Xj, HXj = V @ Zm, HV @ Zm
            P, HP = V[:, m:] @ Zm[m:], HV[:, m:] @ Zm[m:]
            lam = theta[:m]
            hist.append(lam.copy())
        X[:, lo:hi], HX[:, lo:hi] = Xj, HXj
        history.append(hist)
    lam, Y, HY, r = rayleigh_ritz(ham, X, W=HX)
    return LobpcgResult(eig=lam, Y=Y, HY=HY, resid=r, block_history=history)


# ----------------------------------------------------------------------------
# RMM-DIIS
# ----------------------------------------------------------------------------

def _lowest_pencil(A: np.ndarray, B: np.ndarray, rtol: float = 1e-12) -> np.ndarray:
    """Lowest eigenvector a of the pencil A a = e B a (A, B Hermitian, B
    positive semidefinite): B = U diag(s) U^H, the directions with
    s <= rtol max(s) dropped (a history of nearly equal vectors makes B
    singular), the reduced standard problem solved, a B-normalised
    (a^H B a = 1) with sum_i a_i real and non-negative."""
    s, U = np.linalg.eigh(0.5 * (B + B.conj().T))
    keep = s > rtol * s[-1]
    Uk = U[:, keep] / np.sqrt(s[keep])[None, :]
    C = Uk.conj().T @ (0.5 * (A + A.conj().T)) @ Uk
    _, Z = np.linalg.eigh(0.5 * (C + C.conj().T))
    a = Uk @ Z[:, 0]
    t = a.sum()
    if abs(t) > 0.0:
        a = a * (np.conj(t) / abs(t))
    return a


def line_step(psi: np.ndarray, hpsi: np.ndarray, d: np.ndarray, hd: np.ndarray,
              rtol: float = 1e-12) -> complex:
    """Step lam of psi + lam d minimising the Rayleigh quotient on span{psi, d}
    (the lowest Ritz vector c0 psi + c1 d of the 2 x 2 pencil, lam = c1 / c0);
    0 when d vanishes or lies along psi (the pencil's overlap matrix has an
    eigenvalue at or below rtol times its largest)."""
    V = np.stack([psi, d], axis=1)
    HV = np.stack([hpsi, hd], axis=1)
    B = V.conj().T @ V
    s = np.linalg.eigvalsh(0.5 * (B + B.conj().T))
    if not s[0] > rtol * s[-1]:
        return 0.0
    c = _lowest_pencil(V.conj().T @ HV, B, rtol)
    return c[1] / c[0]


@dataclasses.dataclass
class RmmDiisResult:
    eig: np.ndarray
    Y: np.ndarray
    HY: np.ndarray
    resid: np.ndarray
    band_resid: List[np.ndarray]   # per DIIS step: ||R|| / ||psi|| of every band
    steps: np.ndarray              # trial step lam of every band


def rmm_diis(ham: OracleHam, X0: np.ndarray, ndiis: int) -> RmmDiisResult:
    """One RMM-DIIS pass over the bands of X0 (npw x nb, normally the Ritz
    vectors of a previous Rayleigh-Ritz), each band on its own:

      psi^0 = x_b;  R(psi) = (H - e(psi)) psi,  e(psi) = <psi|H|psi>/<psi|psi>;
      lam = the line-minimisation step of psi^0 along K R(psi^0);
      psi^1 = psi^0 + lam K R(psi^0);
      for M = 1 .. ndiis - 1:
        alpha minimises ||sum_i alpha_i R(psi^i)||^2 / ||sum_i alpha_i psi^i||^2
        over i = 0..M (lowest eigenvector of <R^i|R^j> a = e <psi^i|psi^j> a);
        psi_bar = sum alpha_i psi^i, R_bar = sum alpha_i R(psi^i);
        psi^{M+1} = psi_bar + lam K R_bar;
    then every band is the last psi; the block gets one Cholesky
    orthonormalisation and a Rayleigh-Ritz.  K is the Teter preconditioner
    with each band's kinetic energy taken from psi^0.
    """
    X0 = np.asarray(X0, dtype=np.complex128)
    npw, nb = X0.shape
    T = kinetic(ham)
    ek = band_kinetic(ham, X0)
    K = teter_factor(T[:, None] / ek[None, :])
    psis = [X0.copy()]
    hpsis = [apply_h(ham, X0)]

    def resid_of(psi, hpsi):
        e = np.sum(psi.conj() * hpsi, axis=0).real / np.sum(np.abs(psi) ** 2, axis=0)
        return hpsi - psi * e[None, :]

    Rs = [resid_of(psis[0], hpsis[0])]
    D = K * Rs[0]
    HD = apply_h(ham, D)
    lam = np.array([line_step(psis[0][:, b], hpsis[0][:, b], D[:, b], HD[:, b])
                    for b in range(nb)])
    psis.append(psis[0] + D * lam[None, :])
    hpsis.append(hpsis[0] + HD * lam[None, :])
    Rs.append(resid_of(psis[1], hpsis[1]))
    band_resid = [np.linalg.norm(R, axis=0) / np.linalg.norm(p, axis=0)
                  for R, p in zip(Rs, psis)]
    for M in range(1, ndiis):
        new_psi = np.empty_like(X0)
        for b in range(nb):
            Pm = np.stack([p[:, b] for p in psis], axis=1)
            Rm = np.stack([R[:, b] for R in Rs], axis=1)
            a = _lowest_pencil(Rm.conj().T @ Rm, Pm.conj().T @ Pm)
            new_psi[:, b] = Pm @ a + lam[b] * K[:, b] * (Rm @ a)
        psis.append(new_psi)
        hpsis.append(apply_h(ham, new_psi))
        Rs.append(resid_of(psis[-1], hpsis[-1]))
        band_resid.append(np.linalg.norm(Rs[-1], axis=0) / np.linalg.norm(psis[-1], axis=0))
    Y, HY = orthonormalize(psis[-1], hpsis[-1])
    eig, Y, HY, r = rayleigh_ritz(ham, Y, W=HY)
    return RmmDiisResult(eig=eig, Y=Y, HY=HY, resid=r, band_resid=band_resid, steps=lam)
