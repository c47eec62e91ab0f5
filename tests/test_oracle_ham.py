"""Pins of the oracle's Hamiltonian application (kinetic + local + non-local).

Each test checks the oracle against something other than itself: a direct
(non-FFT) DFT, a closed form, or an invariance of the exact operator.
"""
import numpy as np
import pytest

import oracle
import synth


def _ham(w):
    return oracle.OracleHam.from_workload(w)


@pytest.fixture(scope="module")
def c1():
    return synth.config_c1()


def _direct_vtilde(V):
    """Grid Fourier coefficients (1/N) sum_j V_j exp(-2 pi i m.j/N) with explicit
    per-axis DFT matrices (no FFT)."""
    N3, N2, N1 = V.shape
    F = [np.exp(-2j * np.pi * np.outer(np.arange(N), np.arange(N)) / N) for N in (N3, N2, N1)]
    return np.einsum("aj,bk,cl,jkl->abc", F[0], F[1], F[2], V, optimize=True) / V.size


def test_local_term_equals_convolution_matrix(c1):
    """FFT route (scatter, backward, x V, forward, gather) = box-periodic convolution
    by the directly computed coefficients Vt[(n_g - n_g') mod N]."""
    ham = _ham(c1)
    Vt = _direct_vtilde(ham.vloc)
    N1, N2, N3 = ham.box
    n = ham.miller
    d = n[:, None, :] - n[None, :, :]
    Vmat = Vt[np.mod(d[..., 2], N3), np.mod(d[..., 1], N2), np.mod(d[..., 0], N1)]
    rng = np.random.default_rng(5)
    psi = rng.standard_normal((ham.npw, 3)) + 1j * rng.standard_normal((ham.npw, 3))
    got = oracle.apply_local(ham, psi)
    ref = Vmat @ psi
    assert np.linalg.norm(got - ref) <= 1e-13 * np.linalg.norm(ref)


def test_apply_h_equals_dense(c1):
    ham = _ham(c1)
    H = oracle.dense_h(ham)
    rng = np.random.default_rng(6)
    psi = rng.standard_normal((ham.npw, 4)) + 1j * rng.standard_normal((ham.npw, 4))
    ref = H @ psi
    assert np.linalg.norm(oracle.apply_h(ham, psi) - ref) <= 1e-13 * np.linalg.norm(ref)


def test_hermiticity(c1):
    """<phi|H psi> = <H phi|psi> for random phi, psi (H is Hermitian)."""
    ham = _ham(c1)
    rng = np.random.default_rng(7)
    phi = rng.standard_normal((ham.npw, 1)) + 1j * rng.standard_normal((ham.npw, 1))
    psi = rng.standard_normal((ham.npw, 1)) + 1j * rng.standard_normal((ham.npw, 1))
    lhs = np.vdot(phi, oracle.apply_h(ham, psi))
    rhs = np.vdot(oracle.apply_h(ham, phi), psi)
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)
    H = oracle.dense_h(ham)
    assert np.abs(H - H.conj().T).max() <= 1e-14 * np.abs(H).max()


def test_constant_potential_shifts_spectrum(c1):
    """V == V0 everywhere and no projectors: H psi = (T + V0) psi exactly."""
    ham = _ham(c1)
    V0 = -0.731
    ham.vloc = np.full_like(ham.vloc, V0)
    ham.proj = ham.proj[:0]
    ham.ekb = ham.ekb[:0]
    rng = np.random.default_rng(8)
    psi = rng.standard_normal((ham.npw, 2)) + 1j * rng.standard_normal((ham.npw, 2))
    a = 10.26
    q2 = ((2 * np.pi / a) ** 2) * np.sum(ham.miller.astype(float) ** 2, axis=1)
    ref = (0.5 * q2 + V0)[:, None] * psi
    assert np.abs(oracle.apply_h(ham, psi) - ref).max() < 1e-12


@pytest.mark.parametrize("kred", [(0.0, 0.0, 0.0), (0.25, -0.125, 0.375)])
def test_empty_lattice_eigenvalues(kred):
    """V = 0, no projectors: the eigenvalues are 1/2 |k+G|^2 (simple-cubic reciprocal
    lattice of edge 2 pi / a).  Checked through the whole ChFSI path of the oracle."""
    a = 10.26
    w = synth.make_workload("empty", synth.diamond_cell(a=a), kred, 8.0, (24, 24, 24), "s",
                            nb=16, degree=8, iters=12)
    ham = _ham(w)
    ham.vloc = np.zeros_like(ham.vloc)
    ham.proj = ham.proj[:0]
    ham.ekb = ham.ekb[:0]
    # closed form: enumerate integer vectors directly
    r = np.arange(-4, 5)
    n = np.stack(np.meshgrid(r, r, r, indexing="ij"), -1).reshape(-1, 3)
    exact = np.sort(0.5 * (2 * np.pi / a) ** 2 * np.sum((n + np.asarray(kred)) ** 2, axis=1))
    # block edge between multiplets at Gamma (1 + 6 + 12 + 8 = 27); checked bands keep a buffer
    nb, ncheck = (27, 19) if kred == (0.0, 0.0, 0.0) else (16, 10)
    X0 = synth.start_block(ham.npw, nb, seed=3).T
    res = oracle.chfsi(ham, X0, degree=8, iters=12)
    assert np.abs(res.eig_history[-1][:ncheck] - exact[:ncheck]).max() < 1e-9
    if kred == (0.0, 0.0, 0.0):
        assert abs(exact[1] - 0.1875145705) < 1e-9        # 1/2 (2 pi / 10.26)^2


def test_single_projector_secular_equation(c1):
    """H = T + E |p><p| (V = 0): every eigenvalue lambda not in spec(T) solves
    1 + E sum_g |p_g|^2 / (T_g - lambda) = 0 (rank-one update)."""
    ham = _ham(c1)
    ham.vloc = np.zeros_like(ham.vloc)
    ham.proj = ham.proj[:1]
    ham.ekb = np.array([0.5])
    lam = np.linalg.eigvalsh(oracle.dense_h(ham))
    a = 10.26
    T = 0.5 * (2 * np.pi / a) ** 2 * np.sum(ham.miller.astype(float) ** 2, axis=1)
    w2 = np.abs(ham.proj[0]) ** 2
    Tu = np.unique(np.round(T, 12))
    checked = 0
    for x in lam[:60]:
        if np.min(np.abs(Tu - x)) < 1e-7:
            continue
        f = 1.0 + 0.5 * np.sum(w2 / (T - x))
        scale = 0.5 * np.sum(w2 / (T - x) ** 2)      # |f'| for a relative tolerance
        assert abs(f) < 1e-9 * max(1.0, scale)
        checked += 1
    assert checked >= 3
    # interlacing: a repulsive rank-one term moves each eigenvalue up by at most one gap
    Ts = np.sort(T)
    assert np.all(lam[:-1] >= Ts[:-1] - 1e-12) and np.all(lam[:-1] <= Ts[1:] + 1e-12)


def _spectrum(cell, kred, nlow=24):
    w = synth.make_workload("sym", cell, kred, 8.0, (24, 24, 24), "s", nb=16, degree=8, iters=1)
    return np.linalg.eigvalsh(oracle.dense_h(_ham(w)))[:nlow]


def test_time_reversal_and_reciprocal_shift():
    """Real V: spec H(k) = spec H(-k); and spec H(k + b1) = spec H(k) (same set of k+G)."""
    cell = synth.diamond_cell()
    k = (0.1, 0.2, 0.3)
    s0 = _spectrum(cell, k)
    assert np.abs(_spectrum(cell, (-0.1, -0.2, -0.3)) - s0).max() < 1e-11
    assert np.abs(_spectrum(cell, (1.1, 0.2, 0.3)) - s0).max() < 1e-11


def test_translation_by_grid_vector():
    """Moving every atom by a grid vector leaves the spectrum unchanged."""
    cell = synth.diamond_cell()
    s0 = _spectrum(cell, (0.0, 0.0, 0.0))
    shifted = synth.Cell(A=cell.A, tau=cell.tau + np.array([3, 5, 0]) / 24.0 * 10.26)
    assert np.abs(_spectrum(shifted, (0.0, 0.0, 0.0)) - s0).max() < 1e-11
