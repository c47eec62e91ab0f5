"""Pins of the oracle's electron density (section 2.4, Eq. nandtau):
n(r_j) = sum_b w_b |psi_b(r_j)|^2, psi_b(r) = Omega^{-1/2} sum_G c_b(G) e^{i(k+G).r}.

Each pin is fixed by something other than the oracle's own formula: closed
forms for one and two plane waves (sign of the exponent, box axis order,
the 1/Omega factor), Parseval's charge sum, a direct per-point sum over the
sphere, invariance under a unitary rotation of an equally weighted block,
and the cell volume of a cubic / strained cell.
"""
import dataclasses

import numpy as np
import pytest

import oracle
import synth


def _ham(strain=(0.03, -0.02, 0.05), ecut=6.0, box=None, kred=(0.0, 0.0, 0.0)):
    cell = synth.diamond_cell(strain=strain)
    w = synth.make_workload("dens", cell, kred, ecut, box, "s", nb=4, degree=4, iters=1,
                            with_proj=False)
    return oracle.OracleHam.from_workload(w)


def _grid(ham):
    N1, N2, N3 = ham.box
    return np.meshgrid(np.arange(N3), np.arange(N2), np.arange(N1), indexing="ij")


def test_cell_volume_closed_form():
    a = 10.26   # the cubic cell edge of synth.diamond_cell
    cubic = oracle.OracleHam.from_workload(
        synth.make_workload("v", synth.diamond_cell(), (0, 0, 0), 4.0, (12, 12, 12), "s",
                            nb=1, degree=1, iters=1, with_proj=False))
    assert abs(oracle.cell_volume(cubic) - a ** 3) < 1e-9 * a ** 3
    u = (0.03, -0.02, 0.05)
    ham = _ham(strain=u)
    ref = a ** 3 * (1 + u[0]) * (1 + u[1]) * (1 + u[2])
    assert abs(oracle.cell_volume(ham) - ref) < 1e-9 * ref


def test_single_plane_wave_is_uniform():
    """One coefficient c at a point with negative Miller indices: n = w |c|^2 / Omega everywhere."""
    ham = _ham()
    g = int(np.flatnonzero((ham.miller[:, 0] < 0) & (ham.miller[:, 2] < 0))[0])
    psi = np.zeros((ham.npw, 1), dtype=np.complex128)
    psi[g, 0] = 0.6 - 0.8j
    n = oracle.density(ham, psi, np.array([2.0]))
    ref = 2.0 * 1.0 / oracle.cell_volume(ham)
    assert n.shape == tuple(reversed(ham.box))
    assert np.abs(n - ref).max() < 1e-12 * ref


def test_two_plane_waves_closed_form():
    """c(G1) = alpha, c(G2) = beta: n(r_j) = (|alpha|^2 + |beta|^2
    + 2 Re(alpha conj(beta) exp(2 pi i sum_i (n1_i - n2_i) j_i / N_i))) / Omega,
    on a box with three different lengths (array order [j3][j2][j1])."""
    ham = _ham(box=(15, 16, 18))
    rng = np.random.default_rng(5)
    g1, g2 = rng.choice(ham.npw, size=2, replace=False)
    alpha, beta = 0.3 + 0.4j, -0.7 + 0.2j
    psi = np.zeros((ham.npw, 1), dtype=np.complex128)
    psi[g1, 0], psi[g2, 0] = alpha, beta
    n = oracle.density(ham, psi, np.array([1.0]))
    j3, j2, j1 = _grid(ham)
    N1, N2, N3 = ham.box
    d = ham.miller[g1] - ham.miller[g2]
    phase = np.exp(2j * np.pi * (d[0] * j1 / N1 + d[1] * j2 / N2 + d[2] * j3 / N3))
    ref = (abs(alpha) ** 2 + abs(beta) ** 2 + 2 * np.real(alpha * np.conj(beta) * phase))
    ref = ref / oracle.cell_volume(ham)
    assert np.abs(n - ref).max() < 1e-12 * np.abs(ref).max()


def test_parseval_charge():
    """(Omega / N_box) sum_j n(r_j) = sum_b w_b sum_G |c_b(G)|^2 (discrete Parseval)."""
    ham = _ham(box=(20, 18, 16), kred=(0.25, 0.0, 0.5))
    rng = np.random.default_rng(7)
    nb = 5
    psi = rng.standard_normal((ham.npw, nb)) + 1j * rng.standard_normal((ham.npw, nb))
    w = rng.uniform(0.1, 2.0, nb)
    n = oracle.density(ham, psi, w)
    nbox = np.prod(ham.box)
    charge = oracle.cell_volume(ham) / nbox * n.sum()
    ref = float(np.sum(w * np.sum(np.abs(psi) ** 2, axis=0)))
    assert abs(charge - ref) < 1e-12 * ref
    assert n.min() >= 0.0


def test_direct_sum_matches_grid():
    """density_at (explicit phase sum over the sphere per point) equals the FFT route."""
    ham = _ham(box=(18, 20, 15))
    rng = np.random.default_rng(9)
    nb = 3
    psi = rng.standard_normal((ham.npw, nb)) + 1j * rng.standard_normal((ham.npw, nb))
    w = np.array([2.0, 1.0, 0.5])
    n = oracle.density(ham, psi, w)
    N1, N2, N3 = ham.box
    pts = np.stack([rng.integers(0, N1, 12), rng.integers(0, N2, 12), rng.integers(0, N3, 12)], 1)
    direct = oracle.density_at(ham, psi, w, pts)
    grid = n[pts[:, 2], pts[:, 1], pts[:, 0]]
    assert np.abs(direct - grid).max() < 1e-12 * np.abs(grid).max()


def test_unitary_rotation_invariance_and_linearity():
    """Equal weights: n depends on the spanned subspace only (psi -> psi U, U unitary).
    Linear in w: n(w) = sum_b w_b n(e_b)."""
    ham = _ham()
    rng = np.random.default_rng(11)
    nb = 4
    psi = rng.standard_normal((ham.npw, nb)) + 1j * rng.standard_normal((ham.npw, nb))
    z = rng.standard_normal((nb, nb)) + 1j * rng.standard_normal((nb, nb))
    U, _ = np.linalg.qr(z)
    w = np.full(nb, 2.0)
    n0 = oracle.density(ham, psi, w)
    n1 = oracle.density(ham, psi @ U, w)
    assert np.abs(n0 - n1).max() < 1e-12 * np.abs(n0).max()
    wv = np.array([0.5, 1.5, 0.0, 2.0])
    parts = sum(wv[b] * oracle.density(ham, psi[:, b:b + 1], np.array([1.0])) for b in range(nb))
    assert np.abs(oracle.density(ham, psi, wv) - parts).max() < 1e-12 * np.abs(parts).max()


@pytest.mark.parametrize("mistake", ["no_volume", "conj_sign", "swap_axes", "abs_not_squared"])
def test_pins_catch_planted_mistakes(mistake):
    """Each plausible slip in the density definition fails the two-wave closed form."""
    ham = _ham(box=(15, 16, 18))
    psi = np.zeros((ham.npw, 1), dtype=np.complex128)
    alpha, beta = 0.3 + 0.4j, -0.7 + 0.2j
    psi[3, 0], psi[40, 0] = alpha, beta
    vol = oracle.cell_volume(ham)
    if mistake == "no_volume":
        bad = oracle.density(ham, psi, np.array([1.0])) * vol
    elif mistake == "conj_sign":      # e^{-iG.r} in place of e^{+iG.r}
        grid = np.fft.fftn(oracle.scatter_to_box(ham, psi), axes=(-3, -2, -1))
        bad = np.abs(grid[0]) ** 2 / vol
    elif mistake == "swap_axes":      # Miller index n1 taken as n3 and n3 as n1
        bad = oracle.density(dataclasses.replace(ham, miller=ham.miller[:, ::-1].copy()), psi,
                             np.array([1.0]))
    else:
        bad = np.abs(oracle.fft_backward(oracle.scatter_to_box(ham, psi))[0]) / vol
    j3, j2, j1 = _grid(ham)
    N1, N2, N3 = ham.box
    d = ham.miller[3] - ham.miller[40]
    phase = np.exp(2j * np.pi * (d[0] * j1 / N1 + d[1] * j2 / N2 + d[2] * j3 / N3))
    ref = (abs(alpha) ** 2 + abs(beta) ** 2 + 2 * np.real(alpha * np.conj(beta) * phase)) / vol
    good = oracle.density(ham, psi, np.array([1.0]))
    assert np.abs(good - ref).max() < 1e-12 * np.abs(ref).max()
    assert np.abs(bad - ref).max() > 1e-3 * np.abs(ref).max()
