"""FP64 CPU oracle: plane-wave Hamiltonian application and the Chebyshev-filtered
block subspace iteration it drives.

TEST INFRASTRUCTURE ONLY (see the package docstring): imported by tests/,
the smoke check and the benchmark's CPU-baseline leg, never by the library.

Paper anchors (arXiv 2507.08578, "Abinit 2025"):
  * section 1 (Introduction): Hartree atomic units throughout.
  * section 5.1 (GPU use for the ground state and DFPT): the matrix-free
    iterative diagonalisation = apply H to a set of vectors + Rayleigh-Ritz;
    Chebyshev filtering is the preferred eigensolver because it needs few
    Rayleigh-Ritz calls; many FFTs are batched over bands.
  * section 5.2 (Optimization of non-local operations), Eq. (ham-nl): the
    non-local term sum_a sum_ij |p_aik> h_aij <p_ajk|psi>, with h diagonal
    (Kleinman-Bylander energies) for norm-conserving pseudopotentials; the
    projections c = <p|psi> ("cprj") make it a pair of matrix products.
  * section 5.4 (RMM DIIS): full-band Cholesky orthogonalisation.
The paper gives no formula for the filter itself (it cites Levitt and
Bottin, 2015); the scaled three-term Chebyshev recurrence used here is the
textbook one (Zhou and Saad), and every reading of the paper taken where it
is silent is listed in the design notes of the repository.

Conventions:
  * Blocks are complex128 matrices of shape (npw, nb): column b is band b.
  * Box arrays have shape (N3, N2, N1); box index of G = n B is m = n mod N.
  * Backward transform (sphere -> real space):  X(r_j) = sum_m X[m] e^{+2 pi i m.j/N},
    unnormalised.  Forward transform: X[m] = (1/N_box) sum_j X(r_j) e^{-2 pi i m.j/N}.
  * No e^{ik.r} factor enters the FFT; k appears only in the kinetic term
    and in the projector table.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np
import scipy.fft
import scipy.linalg


# ----------------------------------------------------------------------------
# Hamiltonian pieces (section 5.2, Eq. ham-nl; section 5.1)
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class OracleHam:
    """The data that define H at one k-point (all arrays host float64/complex128)."""
    miller: np.ndarray      # (npw, 3) int
    recip: np.ndarray       # (3, 3) rows b1, b2, b3 (bohr^-1)
    kred: np.ndarray        # (3,) reduced k
    box: tuple              # (N1, N2, N3)
    vloc: np.ndarray        # (N3, N2, N1) real, Ha
    proj: np.ndarray        # (nproj, npw): row j is <k+G|p_j>
    ekb: np.ndarray         # (nproj,) KB energies h_jj (Ha)

    @staticmethod
    def from_workload(w) -> "OracleHam":
        return OracleHam(miller=np.asarray(w.miller), recip=np.asarray(w.recip),
                         kred=np.asarray(w.kred), box=tuple(w.box),
                         vloc=np.asarray(w.vloc), proj=np.asarray(w.proj),
                         ekb=np.asarray(w.ekb))

    @property
    def npw(self) -> int:
        return int(self.miller.shape[0])


def kinetic(ham: OracleHam) -> np.ndarray:
    """T_g = 1/2 |k + G_g|^2 (Ha), G_g = n_g . B."""
    q = (ham.miller.astype(np.float64) + ham.kred) @ ham.recip
    return 0.5 * np.sum(q * q, axis=1)


def _box_index(ham: OracleHam):
    N1, N2, N3 = ham.box
    n = ham.miller
    return (np.mod(n[:, 2], N3), np.mod(n[:, 1], N2), np.mod(n[:, 0], N1))


def scatter_to_box(ham: OracleHam, psi: np.ndarray) -> np.ndarray:
    """Zero box (nb, N3, N2, N1) holding psi[g, b] at m(g) = n_g mod N."""
    N1, N2, N3 = ham.box
    nb = psi.shape[1]
    box = np.zeros((nb, N3, N2, N1), dtype=np.complex128)
    i3, i2, i1 = _box_index(ham)
    box[:, i3, i2, i1] = psi.T
    return box


def gather_from_box(ham: OracleHam, box: np.ndarray) -> np.ndarray:
    """Inverse of scatter_to_box on the sphere: (npw, nb)."""
    i3, i2, i1 = _box_index(ham)
    return box[:, i3, i2, i1].T.copy()


def fft_backward(box: np.ndarray) -> np.ndarray:
    """X(r_j) = sum_m X[m] exp(+2 pi i m.j / N) over the last three axes (unnormalised).

    Evaluated by pocketfft (scipy.fft) on every host core (workers=-1); the
    direct O(N^2) sums below pin it."""
    nbox = box.shape[-1] * box.shape[-2] * box.shape[-3]
    return scipy.fft.ifftn(box, axes=(-3, -2, -1), workers=-1) * nbox


def fft_forward(grid: np.ndarray) -> np.ndarray:
    """X[m] = (1/N_box) sum_j X(r_j) exp(-2 pi i m.j / N) over the last three axes."""
    nbox = grid.shape[-1] * grid.shape[-2] * grid.shape[-3]
    return scipy.fft.fftn(grid, axes=(-3, -2, -1), workers=-1) / nbox


def _dft_matrix(N: int, sign: int) -> np.ndarray:
    j = np.arange(N)
    return np.exp(sign * 2j * np.pi * np.outer(j, j) / N)


def dft_backward_direct(box: np.ndarray) -> np.ndarray:
    """Brute-force O(N^2) evaluation of fft_backward for one (N3, N2, N1) box:
    the full N_box x N_box matrix of phases exp(+2 pi i sum_i m_i j_i / N_i)."""
    N3, N2, N1 = box.shape
    m3, m2, m1 = np.meshgrid(np.arange(N3), np.arange(N2), np.arange(N1), indexing="ij")
    m3, m2, m1 = m3.ravel(), m2.ravel(), m1.ravel()
    phase = (np.outer(m3, m3) / N3 + np.outer(m2, m2) / N2 + np.outer(m1, m1) / N1)
    F = np.exp(2j * np.pi * phase)
    return (F @ box.ravel()).reshape(box.shape)


def dft_forward_direct(grid: np.ndarray) -> np.ndarray:
    """Brute-force O(N^2) evaluation of fft_forward for one (N3, N2, N1) grid."""
    N3, N2, N1 = grid.shape
    m3, m2, m1 = np.meshgrid(np.arange(N3), np.arange(N2), np.arange(N1), indexing="ij")
    m3, m2, m1 = m3.ravel(), m2.ravel(), m1.ravel()
    phase = (np.outer(m3, m3) / N3 + np.outer(m2, m2) / N2 + np.outer(m1, m1) / N1)
    F = np.exp(-2j * np.pi * phase)
    return (F @ grid.ravel()).reshape(grid.shape) / grid.size


def apply_local(ham: OracleHam, psi: np.ndarray) -> np.ndarray:
    """Local term: gather(F_fwd(V . F_bwd(scatter(psi)))) (section 5.1, batched FFTs)."""
    box = scatter_to_box(ham, psi)
    real_space = fft_backward(box)
    real_space *= ham.vloc[None, :, :, :]
    return gather_from_box(ham, fft_forward(real_space))


def apply_nonlocal(ham: OracleHam, psi: np.ndarray) -> np.ndarray:
    """Eq. (ham-nl) with diagonal h: sum_j |p_j> E_j <p_j|psi>, via cprj c = P^H psi."""
    if ham.proj.shape[0] == 0:
        return np.zeros_like(psi)
    P = ham.proj.T                                  # (npw, nproj), column j = p_j
    cprj = P.conj().T @ psi                         # c_{j,b} = <p_j|psi_b>
    return P @ (ham.ekb[:, None] * cprj)


def apply_h(ham: OracleHam, psi: np.ndarray) -> np.ndarray:
    """H psi = T psi + V_loc psi + V_nl psi for a block psi of shape (npw, nb)."""
    psi = np.asarray(psi, dtype=np.complex128)
    return kinetic(ham)[:, None] * psi + apply_local(ham, psi) + apply_nonlocal(ham, psi)


def dense_h(ham: OracleHam) -> np.ndarray:
    """Explicit npw x npw matrix of the same operator.

    H_gg' = T_g delta_gg' + Vt[(n_g - n_g') mod N] + sum_j P_gj E_j conj(P_g'j),
    with Vt = F_fwd(V) the grid Fourier coefficients of V (a box-periodic
    convolution, which is what the FFT route computes).
    """
    Vt = fft_forward(ham.vloc)
    N1, N2, N3 = ham.box
    n = ham.miller
    d = n[:, None, :] - n[None, :, :]
    H = Vt[np.mod(d[..., 2], N3), np.mod(d[..., 1], N2), np.mod(d[..., 0], N1)]
    H = H + np.diag(kinetic(ham))
    if ham.proj.shape[0]:
        P = ham.proj.T
        H = H + (P * ham.ekb[None, :]) @ P.conj().T
    return H


def upper_bound(ham: OracleHam) -> float:
    """Weyl upper bound of the spectrum: max T + max V + lambda_max(D+^1/2 P^H P D+^1/2),
    D+ = max(E_KB, 0).  Each term bounds its operator from above."""
    b = float(kinetic(ham).max()) + float(ham.vloc.max())
    if ham.proj.shape[0]:
        P = ham.proj.T
        s = np.sqrt(np.maximum(ham.ekb, 0.0))
        M = (s[:, None] * (P.conj().T @ P)) * s[None, :]
        M = 0.5 * (M + M.conj().T)
        b += max(float(np.linalg.eigvalsh(M)[-1]), 0.0)
    return b


# ----------------------------------------------------------------------------
# Chebyshev filter (section 5.1; recurrence: textbook scaled Chebyshev form)
# ----------------------------------------------------------------------------

def cheb_filter(ham: OracleHam, X: np.ndarray, m: int, a: float, b: float, a0: float,
                hx: Optional[np.ndarray] = None) -> np.ndarray:
    """Y = p_m(H) X,  p_m(t) = T_m((t - c)/e) / T_m((a0 - c)/e),  c = (a+b)/2, e = (b-a)/2.

    Scaled three-term recurrence (values stay O(1) on the wanted part):
      sigma = e/(a0 - c), tau = 2/sigma, Y1 = (sigma/e)(H X - c X);
      for i = 2..m: sigma' = 1/(tau - sigma),
                    Y_i = (2 sigma'/e)(H Y_{i-1} - c Y_{i-1}) - sigma sigma' Y_{i-2},
                    sigma = sigma'.
    hx, if given, is H X already computed (used in place of the first product).
    """
    if m < 1:
        raise ValueError("degree must be >= 1")
    e = (b - a) / 2.0
    c = (b + a) / 2.0
    sigma = e / (a0 - c)
    tau = 2.0 / sigma
    HX = apply_h(ham, X) if hx is None else hx
    y_prev = X
    y = (sigma / e) * (HX - c * X)
    for _ in range(2, m + 1):
        sigma_new = 1.0 / (tau - sigma)
        y_new = (2.0 * sigma_new / e) * (apply_h(ham, y) - c * y) - (sigma * sigma_new) * y_prev
        y_prev, y = y, y_new
        sigma = sigma_new
    return y


def cheb_filter_closed_form(evals: np.ndarray, evecs: np.ndarray, X: np.ndarray, m: int,
                            a: float, b: float, a0: float) -> np.ndarray:
    """U diag(p_m(lambda)) U^H X from a full eigendecomposition, p_m evaluated with
    numpy's Chebyshev series (independent of the recurrence above)."""
    e = (b - a) / 2.0
    c = (b + a) / 2.0
    coef = np.zeros(m + 1)
    coef[m] = 1.0
    p = np.polynomial.chebyshev.chebval((evals - c) / e, coef) / \
        np.polynomial.chebyshev.chebval((a0 - c) / e, coef)
    return evecs @ (p[:, None] * (evecs.conj().T @ X))


# ----------------------------------------------------------------------------
# Subspace steps (section 5.1 Rayleigh-Ritz; section 5.4 Cholesky)
# ----------------------------------------------------------------------------

class NotPositiveDefinite(np.linalg.LinAlgError):
    pass


def orthonormalize(Y: np.ndarray, HY: Optional[np.ndarray] = None):
    """Cholesky orthonormalisation: S = Y^H Y = L L^H, Y <- Y L^{-H} (and HY alike).

    Raises NotPositiveDefinite when S is not numerically positive definite:
    a squared Cholesky pivot at or below n * eps * max_i S_ii.
    """
    S = Y.conj().T @ Y
    S = 0.5 * (S + S.conj().T)
    try:
        L = np.linalg.cholesky(S)
    except np.linalg.LinAlgError as exc:
        raise NotPositiveDefinite(str(exc)) from exc
    # numerically singular: a squared pivot at or below n * eps * max diag(S)
    tol = S.shape[0] * np.finfo(np.float64).eps * float(np.max(np.diag(S).real))
    bad = np.nonzero(np.diag(L).real ** 2 <= tol)[0]
    if bad.size:
        raise NotPositiveDefinite(f"pivot {int(bad[0])} of the Gram matrix is not positive")
    # Y L^{-H}:  solve X L^H = Y  <=>  L X^H = Y^H
    Yn = scipy.linalg.solve_triangular(L, Y.conj().T, lower=True).conj().T
    if HY is None:
        return Yn
    HYn = scipy.linalg.solve_triangular(L, HY.conj().T, lower=True).conj().T
    return Yn, HYn


def rayleigh_ritz(ham: OracleHam, Y: np.ndarray, W: Optional[np.ndarray] = None):
    """W = H Y; Hs = (Y^H W + (Y^H W)^H)/2; Hs = Q diag(lam) Q^H (ascending);
    Y <- Y Q; W <- W Q; r_b = ||W_b - lam_b Y_b||_2.  Y must be orthonormal.
    W, if given, is H Y already formed by apply_h (e.g. band by band for a
    block whose whole FFT box would not fit in host memory)."""
    if W is None:
        W = apply_h(ham, Y)
    Hs = Y.conj().T @ W
    Hs = 0.5 * (Hs + Hs.conj().T)
    lam, Q = np.linalg.eigh(Hs)
    Y = Y @ Q
    W = W @ Q
    resid = np.linalg.norm(W - Y * lam[None, :], axis=0)
    return lam, Y, W, resid


@dataclasses.dataclass
class ChfsiResult:
    eig_history: List[np.ndarray]      # Ritz values after iteration 0, 1, ..., iters
    resid_history: List[np.ndarray]
    Y: np.ndarray
    upper: float


def chfsi(ham: OracleHam, X0: np.ndarray, degree: int, iters: int,
          upper: Optional[float] = None) -> ChfsiResult:
    """Chebyshev-filtered block subspace iteration (section 5.1).

    Iteration 0: orthonormalise X0 and Rayleigh-Ritz it.  Iteration t >= 1:
    filter with a = largest Ritz value, a0 = smallest, b = Weyl upper bound;
    orthonormalise; Rayleigh-Ritz.
    """
    b = upper_bound(ham) if upper is None else upper
    Y = orthonormalize(np.asarray(X0, dtype=np.complex128))
    lam, Y, W, r = rayleigh_ritz(ham, Y)
    eigs, res = [lam], [r]
    for _ in range(iters):
        Y = cheb_filter(ham, Y, degree, float(lam[-1]), b, float(lam[0]))
        Y = orthonormalize(Y)
        lam, Y, W, r = rayleigh_ritz(ham, Y)
        eigs.append(lam)
        res.append(r)
    return ChfsiResult(eig_history=eigs, resid_history=res, Y=Y, upper=b)


# ----------------------------------------------------------------------------
# Electron density of a block of bands (section 2.4, Eq. nandtau; the
# band-and-k sum of Eq. extfpmd_density in section 2.3, without its
# free-electron term N_ext / Omega)
# ----------------------------------------------------------------------------

def cell_volume(ham: OracleHam) -> float:
    """Omega = (2 pi)^3 / |det B| for reciprocal rows b_i (a_i . b_j = 2 pi delta_ij)."""
    return float((2.0 * np.pi) ** 3 / abs(np.linalg.det(ham.recip)))


def density(ham: OracleHam, psi: np.ndarray, w: np.ndarray) -> np.ndarray:
    """n(r_j) = sum_b w_b |psi_b(r_j)|^2 at the box points r_j = (j1/N1, j2/N2, j3/N3) A.

    psi_b(r) = Omega^{-1/2} sum_G c_b(G) e^{i(k+G).r}: a band whose
    coefficients have unit norm holds one electron in the cell, and the
    factor e^{ik.r} has modulus one, so |psi_b(r_j)|^2 is
    |fft_backward(scatter(c_b))[j]|^2 / Omega.  w_b is the band's occupation
    times its k-point weight.  Returns shape (N3, N2, N1).
    """
    grid = fft_backward(scatter_to_box(ham, np.asarray(psi, dtype=np.complex128)))
    dens = np.zeros(grid.shape[1:], dtype=np.float64)
    for b in range(grid.shape[0]):
        dens += float(w[b]) * np.abs(grid[b]) ** 2
    return dens / cell_volume(ham)


def density_at(ham: OracleHam, psi: np.ndarray, w: np.ndarray, points: np.ndarray) -> np.ndarray:
    """n at selected box points, each summed directly over the sphere:
    psi_b(r_j) = Omega^{-1/2} sum_g c_b(g) exp(2 pi i sum_i n_i(g) j_i / N_i).
    points: (P, 3) integer (j1, j2, j3).  For full-size blocks the box never
    has to exist."""
    N = np.asarray(ham.box, dtype=np.float64)
    n = ham.miller.astype(np.float64)
    out = np.empty(len(points))
    for p, j in enumerate(np.asarray(points)):
        phase = np.exp(2j * np.pi * (n @ (np.asarray(j, dtype=np.float64) / N)))
        amp = phase @ np.asarray(psi, dtype=np.complex128)      # (nb,)
        out[p] = float(np.sum(np.asarray(w, dtype=np.float64) * np.abs(amp) ** 2))
    return out / cell_volume(ham)
