"""Pins of the oracle's LOBPCG and RMM-DIIS (section 5.1's band-block
conjugate-gradient solver; section 5.4's RMM-DIIS), independent of the
oracle's own formulas:

* the preconditioner at values worked by hand (K(0) = 1, K(1) = 65/81, the
  large-x limit 1/(2x)) and on a single plane wave, whose kinetic energy is
  exactly its T_g;
* the two-dimensional minimum behind the first LOBPCG line and the RMM-DIIS
  step against a brute-force search of the Rayleigh quotient over the plane;
* the pencil solve against scipy's generalised eigensolver;
* convergence to the dense eigen-decomposition of the explicit H (C1 at Gamma
  and a shifted C2 k-point) for several block splits, the Ritz values never
  rising within a block (min-max), and RMM-DIIS leaving exact eigenvectors
  unchanged;
* a planted mistake (blocks not kept orthogonal to the blocks below them)
  breaks convergence.
"""
import numpy as np
import pytest
import scipy.linalg
import scipy.optimize

import oracle
import synth
from oracle import eigensolvers as es


@pytest.fixture(scope="module")
def c1():
    w = synth.config_c1()
    ham = oracle.OracleHam.from_workload(w)
    lam, U = np.linalg.eigh(oracle.dense_h(ham))
    return ham, lam, U


def test_teter_factor_hand_values():
    assert es.teter_factor(np.array([0.0]))[0] == 1.0
    assert abs(es.teter_factor(np.array([1.0]))[0] - 65.0 / 81.0) < 1e-15
    x = np.array([1e4, 1e6])
    assert np.abs(es.teter_factor(x) * 2 * x - 1.0).max() < 1e-3
    # monotone decreasing from 1
    xs = np.linspace(0, 50, 501)
    k = es.teter_factor(xs)
    assert np.all(np.diff(k) < 0) and k.max() == 1.0


def test_precondition_single_plane_wave(c1):
    """A band holding one plane wave g has kinetic energy T_g, so x = 1 at g:
    the residual component there is scaled by 65/81."""
    ham, _, _ = c1
    T = oracle.kinetic(ham)
    g = int(np.argsort(T)[40])
    X = np.zeros((ham.npw, 1), dtype=np.complex128)
    X[g, 0] = 0.6 - 0.8j
    assert abs(es.band_kinetic(ham, X)[0] - T[g]) < 1e-15 * T[g]
    R = np.zeros_like(X)
    R[g, 0] = 2.0 + 1.0j
    W = es.precondition(ham, X, R)
    assert abs(W[g, 0] - (65.0 / 81.0) * R[g, 0]) < 1e-14


def _brute_min_rq(Hd, a, b):
    """min over the plane span{a, b} of the Rayleigh quotient, by a grid over
    (theta, phi) of cos(theta) a + e^{i phi} sin(theta) b (a, b orthonormal)
    refined by Nelder-Mead."""
    def rq(t):
        v = np.cos(t[0]) * a + np.exp(1j * t[1]) * np.sin(t[0]) * b
        return float(np.real(v.conj() @ (Hd @ v)) / np.real(v.conj() @ v))
    best = min(((rq((th, ph)), th, ph) for th in np.linspace(0, np.pi, 61)
                for ph in np.linspace(0, 2 * np.pi, 61)))
    res = scipy.optimize.minimize(rq, [best[1], best[2]], method="Nelder-Mead",
                                  options={"xatol": 1e-12, "fatol": 1e-15, "maxiter": 4000})
    return res.fun


def test_first_line_is_the_plane_minimum(c1):
    """One band, one line: the new Ritz value is the minimum of the Rayleigh
    quotient over span{x, K r} (no previous direction yet)."""
    ham, _, _ = c1
    Hd = oracle.dense_h(ham)
    x0 = synth.start_block(ham.npw, 1, 11).T
    res = es.lobpcg(ham, x0, nblock=1, nline=1)
    got = res.block_history[0][1][0]
    x = x0[:, 0] / np.linalg.norm(x0)
    r = Hd @ x - (x.conj() @ Hd @ x).real * x
    wv = es.precondition(ham, x[:, None], r[:, None])[:, 0]
    wv = wv - x * (x.conj() @ wv)
    wv /= np.linalg.norm(wv)
    ref = _brute_min_rq(Hd, x, wv)
    assert abs(got - ref) < 1e-9 * abs(ref), (got, ref)


def test_rmm_line_step_is_the_plane_minimum(c1):
    ham, _, _ = c1
    Hd = oracle.dense_h(ham)
    rng = np.random.default_rng(3)
    psi = rng.standard_normal(ham.npw) + 1j * rng.standard_normal(ham.npw)
    d = rng.standard_normal(ham.npw) + 1j * rng.standard_normal(ham.npw)
    lam = es.line_step(psi, Hd @ psi, d, Hd @ d)
    v = psi + lam * d
    got = float(np.real(v.conj() @ Hd @ v) / np.real(v.conj() @ v))
    a = psi / np.linalg.norm(psi)
    b = d - a * (a.conj() @ d)
    b /= np.linalg.norm(b)
    ref = _brute_min_rq(Hd, a, b)
    assert abs(got - ref) < 1e-9 * abs(ref)
    assert es.line_step(psi, Hd @ psi, 0 * d, 0 * d) == 0.0
    assert es.line_step(psi, Hd @ psi, 2j * psi, 2j * (Hd @ psi)) == 0.0


def test_pencil_matches_scipy():
    rng = np.random.default_rng(4)
    for n in (2, 3, 6):
        M = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
        A = M + M.conj().T
        N = rng.standard_normal((n + 3, n)) + 1j * rng.standard_normal((n + 3, n))
        B = N.conj().T @ N
        a = es._lowest_pencil(A, B)
        w, V = scipy.linalg.eigh(A, B)
        e = (a.conj() @ A @ a).real / (a.conj() @ B @ a).real
        assert abs(e - w[0]) < 1e-10 * max(1.0, abs(w[0]))
        assert abs((a.conj() @ B @ a).real - 1.0) < 1e-12
        assert abs(a.sum().imag) < 1e-12 and a.sum().real >= 0


@pytest.mark.parametrize("nblock", [1, 3])
def test_lobpcg_converges_to_dense_c1(c1, nblock):
    """C1, 24-band block (the lowest 16 below the block-edge multiplet):
    repeated passes reach the dense eigenvalues; Ritz values never rise
    within a block."""
    ham, lam, _ = c1
    X = synth.start_block(ham.npw, 24, 1).T
    for _ in range(7):
        res = es.lobpcg(ham, X, nblock=nblock, nline=4)
        X = res.Y
        for hist in res.block_history:
            assert np.diff(np.array(hist), axis=0).max() < 1e-12
    assert np.abs(res.eig[:16] - lam[:16]).max() < 1e-10
    assert res.resid[:16].max() < 1e-6
    y = res.Y
    assert np.abs(y.conj().T @ y - np.eye(24)).max() < 1e-12


def test_lobpcg_converges_c2_kpoint():
    k = synth.kpoint_grid_shifted(3)[13]
    w = synth.make_workload("C2", synth.diamond_cell(), k, 8.0, (24, 24, 24), "s", 16, 8, 20)
    ham = oracle.OracleHam.from_workload(w)
    lam = np.linalg.eigvalsh(oracle.dense_h(ham))
    X = synth.start_block(ham.npw, 20, 5).T
    for _ in range(7):
        X = es.lobpcg(ham, X, nblock=2, nline=4).Y
    res = es.lobpcg(ham, X, nblock=2, nline=4)
    assert np.abs(res.eig[:14] - lam[:14]).max() < 1e-10


def test_lobpcg_without_lower_block_orthogonality_fails(c1, monkeypatch):
    """Planted mistake: blocks not kept orthogonal to the blocks below them
    converge onto the same eigenvectors (the final block is no longer
    orthonormal before its Cholesky step, or duplicates appear)."""
    ham, lam, _ = c1
    orig = es._remove
    calls = {"n": 0}

    def skip_lower(B, HB, X, HX):
        # drop the removal of the lower blocks (X wider than the current block)
        if X.shape[1] != B.shape[1]:
            calls["n"] += 1
            return B, HB
        return orig(B, HB, X, HX)

    monkeypatch.setattr(es, "_remove", skip_lower)
    X = synth.start_block(ham.npw, 24, 1).T
    try:
        for _ in range(7):
            res = es.lobpcg(ham, X, nblock=3, nline=4)
            X = res.Y
        bad = np.abs(res.eig[:16] - lam[:16]).max()
    except np.linalg.LinAlgError:
        bad = np.inf
    assert calls["n"] > 0 and bad > 1e-6


def test_rmm_diis_fixed_point(c1):
    """Exact eigenvectors (complete multiplets: 1 + 6) have zero residuals:
    RMM-DIIS leaves their eigenvalues exact."""
    ham, lam, U = c1
    res = es.rmm_diis(ham, U[:, :7].copy(), ndiis=3)
    assert np.abs(res.eig - lam[:7]).max() < 1e-12
    assert res.resid.max() < 1e-10
    assert np.all(res.steps == 0.0)


def test_rmm_diis_converges_from_near_start(c1):
    ham, lam, U = c1
    rng = np.random.default_rng(7)
    X = U[:, :14] + 0.01 * (rng.standard_normal((ham.npw, 14)) +
                            1j * rng.standard_normal((ham.npw, 14)))
    errs = []
    for _ in range(6):
        res = es.rmm_diis(ham, X, ndiis=4)
        X = res.Y
        errs.append(np.abs(res.eig - lam[:14]).max())
    assert errs[-1] < 1e-9 and errs[-1] < 1e-3 * errs[0], errs
    # residual norms fall along the DIIS history of every call
    assert res.band_resid[-1].max() < res.band_resid[0].max()
