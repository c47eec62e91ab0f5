"""Synthetic diamond-lattice cells standing in for the paper's workload.

The paper measures its Chebyshev-filtered solver on a PAW Ga2O3 system
(section 5.1, figure "cpu_gpu_speedup"); no pseudopotential datasets are
available here, so Si-like diamond cells with Gaussian wells and Gaussian
Kleinman-Bylander projectors take its place.  Everything is seeded and
deterministic; Hartree atomic units throughout (section 2).

Array conventions shared with the library:
  * Miller indices: int32 array (npw, 3), columns (n1, n2, n3), sorted
    lexicographically ascending, G = n1*b1 + n2*b2 + n3*b3.
  * Blocks of wavefunctions: complex128 arrays of shape (nb, npw), one band
    per row, i.e. column-major npw x nb with leading dimension npw.
  * Projector table: complex128 array (nproj, npw) (column-major npw x nproj).
  * Local potential on the grid: float64 array (N3, N2, N1), N1 fastest,
    grid point r_j = (j1/N1, j2/N2, j3/N3) A.

Only orthorhombic cells (diagonal lattice matrix) are generated: diamond
supercells, positional jitter and diagonal strain all keep that property,
which makes the periodic Gaussian sum separable per Cartesian axis.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

BOHR_DIAMOND = 10.26          # conventional cubic cell edge of the Si-like cells
WELL_DEPTH = 2.0              # Ha, depth of each Gaussian well
WELL_SIGMA = 1.2              # bohr, V ~ exp(-r^2 / (2 sigma^2))
PROJ_RADIUS = 1.2             # bohr, projector Gaussian width
E_KB = 0.5                    # Ha, KB energy of every channel
IMAGES = 2                    # periodic images summed over R in {-2..2}^3

_DIAMOND_FRAC = np.array([
    [0.0, 0.0, 0.0], [0.0, 0.5, 0.5], [0.5, 0.0, 0.5], [0.5, 0.5, 0.0],
    [0.25, 0.25, 0.25], [0.25, 0.75, 0.75], [0.75, 0.25, 0.75], [0.75, 0.75, 0.25],
])


@dataclasses.dataclass
class Cell:
    A: np.ndarray            # (3,3) rows are lattice vectors (bohr)
    tau: np.ndarray          # (natoms, 3) Cartesian positions (bohr)

    @property
    def volume(self) -> float:
        return float(abs(np.linalg.det(self.A)))

    @property
    def recip(self) -> np.ndarray:
        """Rows b_i with a_i . b_j = 2 pi delta_ij."""
        return 2.0 * np.pi * np.linalg.inv(self.A).T

    @property
    def natoms(self) -> int:
        return int(self.tau.shape[0])


def diamond_cell(a: float = BOHR_DIAMOND, reps: Sequence[int] = (1, 1, 1),
                 jitter: float = 0.0, geom_seed: int = 0,
                 strain: Optional[Sequence[float]] = None) -> Cell:
    """Diamond supercell reps[0] x reps[1] x reps[2] of the 8-atom cubic cell.

    jitter: standard deviation (bohr) of an i.i.d. Gaussian displacement of
    every Cartesian component, drawn from default_rng(geom_seed).
    strain: diagonal strain u, A' = A (I + diag(u)); fractional positions kept.
    """
    reps = np.asarray(reps, dtype=np.int64)
    frac = []
    for i in range(reps[0]):
        for j in range(reps[1]):
            for k in range(reps[2]):
                frac.append((_DIAMOND_FRAC + np.array([i, j, k])) / reps)
    frac = np.concatenate(frac, axis=0)
    A = np.diag(a * reps.astype(np.float64))
    if strain is not None:
        A = A @ (np.eye(3) + np.diag(np.asarray(strain, dtype=np.float64)))
    tau = frac @ A
    if jitter > 0.0:
        tau = tau + np.random.default_rng(geom_seed).normal(0.0, jitter, size=tau.shape)
    return Cell(A=A, tau=tau)


def sphere_miller(recip: np.ndarray, kred: Sequence[float], ecut: float) -> np.ndarray:
    """All integer n with 1/2 |(n + k) B|^2 <= ecut, lexicographic (n1, n2, n3)."""
    kred = np.asarray(kred, dtype=np.float64)
    gmax = math.sqrt(2.0 * ecut)
    # |n_i + k_i| = |(k+G) . a_i| / (2 pi) <= gmax |a_i| / (2 pi)
    A = 2.0 * np.pi * np.linalg.inv(recip).T
    lim = [int(math.floor(gmax * np.linalg.norm(A[i]) / (2.0 * np.pi) + abs(kred[i]))) + 1
           for i in range(3)]
    r = [np.arange(-lim[i], lim[i] + 1) for i in range(3)]
    n = np.stack(np.meshgrid(r[0], r[1], r[2], indexing="ij"), axis=-1).reshape(-1, 3)
    q = (n + kred) @ recip
    keep = 0.5 * np.einsum("ij,ij->i", q, q) <= ecut
    n = n[keep]
    order = np.lexsort((n[:, 2], n[:, 1], n[:, 0]))
    return np.ascontiguousarray(n[order].astype(np.int32))


def _smooth235(n: int) -> bool:
    for p in (2, 3, 5):
        while n % p == 0:
            n //= p
    return n == 1


def box_rule(miller: np.ndarray) -> tuple:
    """Per axis the smallest {2,3,5}-smooth N >= 4 max|n_i| (box not stated)."""
    out = []
    for i in range(3):
        n = max(4 * int(np.abs(miller[:, i]).max()), 1)
        while not _smooth235(n):
            n += 1
        out.append(n)
    return tuple(out)


def local_potential(cell: Cell, box: Sequence[int], depth: float = WELL_DEPTH,
                    sigma: float = WELL_SIGMA, images: int = IMAGES) -> np.ndarray:
    """V(r_j) = -depth * sum_atoms sum_{R in {-images..images}^3} exp(-|r_j - tau - R A|^2/(2 sigma^2)).

    Returned as float64 (N3, N2, N1).  Orthorhombic cells only: the sum over
    images then factorises into one 1D periodic Gaussian per axis.
    """
    A = cell.A
    if np.abs(A - np.diag(np.diag(A))).max() > 0.0:
        raise ValueError("local_potential: only orthorhombic (diagonal) lattices are generated")
    N1, N2, N3 = (int(x) for x in box)
    L = np.diag(A)
    R = np.arange(-images, images + 1)

    def axis_profile(N, Ld, t):
        x = np.arange(N) / N * Ld                                # (N,)
        d = x[None, :, None] - t[:, None, None] - R[None, None, :] * Ld
        return np.exp(-d * d / (2.0 * sigma * sigma)).sum(axis=2)   # (natoms, N)

    gx = axis_profile(N1, L[0], cell.tau[:, 0])
    gy = axis_profile(N2, L[1], cell.tau[:, 1])
    gz = axis_profile(N3, L[2], cell.tau[:, 2])
    zy = (gz[:, :, None] * gy[:, None, :]).reshape(cell.natoms, N3 * N2)
    V = -depth * (zy.T @ gx)
    return np.ascontiguousarray(V.reshape(N3, N2, N1))


def kb_projectors(cell: Cell, miller: np.ndarray, kred: Sequence[float],
                  channels: str = "s", rp: float = PROJ_RADIUS,
                  ekb: float = E_KB) -> tuple:
    """Unit-norm Gaussian KB projectors <k+G|p_{a,i}> and their KB energies.

    s:  p(r) ~ exp(-r^2/(2 rp^2));  p_m(r) ~ x_m exp(-r^2/(2 rp^2)), m = x, y, z.
    Plane-wave components with q = k+G, Omega the cell volume:
      s:   Omega^-1/2 (4 pi rp^2)^(3/4) exp(-q^2 rp^2/2) e^{-i q.tau}
      p_m: Omega^-1/2 Np (-i q_m rp^2) (2 pi rp^2)^(3/2) exp(-q^2 rp^2/2) e^{-i q.tau},
           Np = (2 / (pi^(3/2) rp^5))^(1/2).
    Order: atom-major, channels s[, px, py, pz].
    Returns (proj (nproj, npw) complex128, ekb (nproj,) float64).
    """
    if channels not in ("s", "sp"):
        raise ValueError("channels must be 's' or 'sp'")
    q = (miller.astype(np.float64) + np.asarray(kred, dtype=np.float64)) @ cell.recip
    q2 = np.einsum("ij,ij->i", q, q)
    gauss = np.exp(-0.5 * q2 * rp * rp)
    inv_sqrt_vol = 1.0 / math.sqrt(cell.volume)
    pref_s = inv_sqrt_vol * (4.0 * np.pi * rp * rp) ** 0.75
    n_p = math.sqrt(2.0 / (np.pi ** 1.5 * rp ** 5))
    pref_p = inv_sqrt_vol * n_p * (2.0 * np.pi * rp * rp) ** 1.5
    nch = 1 if channels == "s" else 4
    nproj = cell.natoms * nch
    proj = np.empty((nproj, q.shape[0]), dtype=np.complex128)
    for a in range(cell.natoms):
        phase = np.exp(-1j * (q @ cell.tau[a]))
        base = gauss * phase
        proj[a * nch] = pref_s * base
        if nch == 4:
            for m in range(3):
                proj[a * nch + 1 + m] = pref_p * (-1j * rp * rp) * q[:, m] * base
    return proj, np.full(nproj, ekb, dtype=np.float64)


def start_block(npw: int, nb: int, seed: int) -> np.ndarray:
    """Random complex start block, shape (nb, npw): i.i.d. N(0,1) real and imaginary parts."""
    s = np.random.default_rng(seed).standard_normal((nb, npw, 2))
    return s[..., 0] + 1j * s[..., 1]


def kpoint_grid_shifted(n: int = 3) -> np.ndarray:
    """Reduced k-points ((i+1/2)/n, (j+1/2)/n, (l+1/2)/n), i,j,l in 0..n-1."""
    r = (np.arange(n) + 0.5) / n
    return np.stack(np.meshgrid(r, r, r, indexing="ij"), axis=-1).reshape(-1, 3)


@dataclasses.dataclass
class Workload:
    """One k-point of one cell: everything the H*psi path takes as input."""
    name: str
    cell: Cell
    kred: np.ndarray
    ecut: float
    miller: np.ndarray
    box: tuple                      # (N1, N2, N3)
    vloc: np.ndarray                # (N3, N2, N1) float64
    proj: np.ndarray                # (nproj, npw) complex128
    ekb: np.ndarray                 # (nproj,)
    nb: int
    degree: int
    iters: int

    @property
    def npw(self) -> int:
        return int(self.miller.shape[0])

    @property
    def nproj(self) -> int:
        return int(self.proj.shape[0])

    @property
    def recip(self) -> np.ndarray:
        return self.cell.recip


def make_workload(name: str, cell: Cell, kred, ecut: float, box, channels: str,
                  nb: int, degree: int, iters: int, with_proj: bool = True) -> Workload:
    B = cell.recip
    miller = sphere_miller(B, kred, ecut)
    if box is None:
        box = box_rule(miller)
    vloc = local_potential(cell, box)
    if with_proj:
        proj, ekb = kb_projectors(cell, miller, kred, channels)
    else:
        proj = np.zeros((0, miller.shape[0]), dtype=np.complex128)
        ekb = np.zeros(0)
    return Workload(name=name, cell=cell, kred=np.asarray(kred, dtype=np.float64), ecut=ecut,
                    miller=miller, box=tuple(int(x) for x in box), vloc=vloc, proj=proj,
                    ekb=ekb, nb=nb, degree=degree, iters=iters)


def config_c1(nb: int = 16) -> Workload:
    """8-atom diamond cell, Gamma, ecut 8 Ha, box 24^3, one s projector per atom."""
    return make_workload("C1", diamond_cell(), (0.0, 0.0, 0.0), 8.0, (24, 24, 24), "s",
                         nb=nb, degree=8, iters=20)


def config_c2() -> List[Workload]:
    """C1 cell at the 27 k-points of the shifted 3x3x3 grid, 16 bands each."""
    cell = diamond_cell()
    return [make_workload(f"C2.k{i}", cell, k, 8.0, (24, 24, 24), "s", nb=16, degree=8, iters=20)
            for i, k in enumerate(kpoint_grid_shifted(3))]


def config_c3(geom_seed: int = 0, nb: int = 160) -> Workload:
    """64-atom 2x2x2 supercell, jitter 0.05 bohr, Gamma, ecut 20 Ha, box 96^3, s+p projectors."""
    cell = diamond_cell(reps=(2, 2, 2), jitter=0.05, geom_seed=geom_seed)
    return make_workload("C3", cell, (0.0, 0.0, 0.0), 20.0, (96, 96, 96), "sp",
                         nb=nb, degree=8, iters=20)


def c4_cell_params(c: int) -> tuple:
    """Per-cell strain u (3,), ecut and band count for cell c of the uneven batch."""
    rng = np.random.default_rng(4000 + c)
    u = rng.uniform(-0.06, 0.06, size=3)
    ecut = float(rng.uniform(8.0, 16.0))
    nb = int(rng.integers(16, 33))
    return u, ecut, nb


def config_c4(ncells: int = 64) -> List[Workload]:
    """64 strained 8-atom cells, ecut U(8,16) Ha, 16-32 bands, boxes by the smooth-size rule."""
    out = []
    for c in range(ncells):
        u, ecut, nb = c4_cell_params(c)
        cell = diamond_cell(strain=u)
        out.append(make_workload(f"C4.c{c}", cell, (0.0, 0.0, 0.0), ecut, None, "s",
                                 nb=nb, degree=8, iters=20))
    return out


def config_c5(nb: int = 512, with_proj: bool = True) -> Workload:
    """216-atom 3x3x3 supercell, Gamma, ecut 20 Ha, box 144^3, s+p projectors (864)."""
    cell = diamond_cell(reps=(3, 3, 3))
    return make_workload("C5", cell, (0.0, 0.0, 0.0), 20.0, (144, 144, 144), "sp",
                         nb=nb, degree=12, iters=20, with_proj=with_proj)


CONFIGS = {"C1": config_c1, "C2": config_c2, "C3": config_c3, "C4": config_c4, "C5": config_c5}
