"""Pins of the oracle's filter, orthonormalisation, Rayleigh-Ritz and full ChFSI."""
import os

import numpy as np
import pytest

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def c1_dense():
    w = synth.config_c1()
    ham = oracle.OracleHam.from_workload(w)
    H = oracle.dense_h(ham)
    lam, U = np.linalg.eigh(H)
    return w, ham, lam, U


def test_filter_matches_closed_form(c1_dense):
    """Scaled recurrence = U diag(p_m(lambda)) U^H X with p_m from numpy's Chebyshev series."""
    w, ham, lam, U = c1_dense
    X = synth.start_block(ham.npw, 6, seed=1).T
    b = oracle.upper_bound(ham)
    for m, a, a0 in [(1, 0.2, -0.3), (2, 0.0, -0.2), (8, 0.1, -0.18), (11, -0.05, -0.2)]:
        got = oracle.cheb_filter(ham, X, m, a, b, a0)
        ref = oracle.cheb_filter_closed_form(lam, U, X, m, a, b, a0)
        assert np.linalg.norm(got - ref) <= 1e-11 * np.linalg.norm(ref), m


def test_filter_chebyshev_values_known(monkeypatch):
    """On a diagonal H the filter multiplies component i by T_m(l(x_i))/T_m(l(a0));
    T_3(u) = 4u^3 - 3u and T_4(u) = 8u^4 - 8u^2 + 1 written out (closed forms).
    Checked for both the closed-form helper and the recurrence (driven by diag(x))."""
    x = np.array([-1.5, -0.7, 0.3, 0.9, 2.0, 3.0])
    X = np.ones((6, 1), dtype=np.complex128)
    a, b, a0 = 0.0, 3.0, -1.5
    c, e = 1.5, 1.5
    t = (x - c) / e
    t0 = (a0 - c) / e
    closed = {3: lambda u: 4 * u ** 3 - 3 * u, 4: lambda u: 8 * u ** 4 - 8 * u ** 2 + 1}
    ham = oracle.OracleHam(miller=np.zeros((6, 3), dtype=np.int32), recip=np.eye(3),
                           kred=np.zeros(3), box=(1, 1, 1), vloc=np.zeros((1, 1, 1)),
                           proj=np.zeros((0, 6), dtype=np.complex128), ekb=np.zeros(0))
    monkeypatch.setattr(oracle.pw_oracle, "apply_h", lambda _h, v: x[:, None] * v)
    for m, Tm in closed.items():
        ref = Tm(t) / Tm(t0)
        got = oracle.cheb_filter_closed_form(x, np.eye(6), X, m, a, b, a0)[:, 0]
        assert np.abs(got - ref).max() < 1e-12
        got2 = oracle.cheb_filter(ham, X, m, a, b, a0)[:, 0]
        assert np.abs(got2 - ref).max() < 1e-12


def test_orthonormalize_matches_qr():
    """Cholesky-QR: Y L^{-H} = Q of the QR factorisation with a positive real R diagonal."""
    rng = np.random.default_rng(2)
    Y = rng.standard_normal((300, 12)) + 1j * rng.standard_normal((300, 12))
    HY = rng.standard_normal((300, 12)) + 1j * rng.standard_normal((300, 12))
    Yn, HYn = oracle.orthonormalize(Y, HY)
    assert np.abs(Yn.conj().T @ Yn - np.eye(12)).max() < 1e-13
    Q, R = np.linalg.qr(Y)
    ph = np.diag(R) / np.abs(np.diag(R))
    Q = Q * ph[None, :]
    R = R / ph[:, None]
    assert np.abs(Yn - Q).max() < 1e-12
    # the same right factor applied to HY
    assert np.abs(HYn - HY @ np.linalg.inv(R)).max() < 1e-10


def test_orthonormalize_rank_deficient_raises():
    rng = np.random.default_rng(3)
    Y = rng.standard_normal((50, 4)) + 1j * rng.standard_normal((50, 4))
    Y[:, 3] = Y[:, 1]
    with pytest.raises(oracle.pw_oracle.NotPositiveDefinite):
        oracle.orthonormalize(Y)


def test_rayleigh_ritz_exact_subspace(c1_dense):
    """If Y spans an invariant subspace, RR returns its exact eigenvalues, zero residuals."""
    w, ham, lam, U = c1_dense
    rng = np.random.default_rng(4)
    M = rng.standard_normal((10, 10)) + 1j * rng.standard_normal((10, 10))
    Qm, _ = np.linalg.qr(M)
    Y = U[:, :10] @ Qm                              # rotated basis of the lowest 10
    ritz, Yr, Wr, r = oracle.rayleigh_ritz(ham, Y)
    assert np.abs(ritz - lam[:10]).max() < 1e-12
    assert r.max() < 1e-11


def test_rayleigh_ritz_bounds_and_trace(c1_dense):
    """Ritz values from any orthonormal block lie above the exact eigenvalues (min-max),
    and sum(ritz) = trace(Y^H H Y)."""
    w, ham, lam, U = c1_dense
    Y = oracle.orthonormalize(synth.start_block(ham.npw, 12, seed=9).T)
    ritz, Yr, Wr, r = oracle.rayleigh_ritz(ham, Y)
    assert np.all(ritz >= lam[:12] - 1e-12)
    H = oracle.dense_h(ham)
    assert abs(ritz.sum() - np.trace(Y.conj().T @ H @ Y).real) < 1e-10
    assert np.abs(Wr - H @ Yr).max() < 1e-12


def test_upper_bound_is_an_upper_bound(c1_dense):
    w, ham, lam, U = c1_dense
    b = oracle.upper_bound(ham)
    assert b >= lam[-1]
    assert b - lam[-1] < 2.0              # and not uselessly loose


def _max_kinetic_cubic(w):
    """max over the sphere of 1/2 |k + G|^2 for a cubic cell of edge a, from the
    integer Miller indices alone: |k + G|^2 = (2 pi / a)^2 |n + k|^2."""
    a = float(w.cell.A[0, 0])
    assert np.allclose(w.cell.A, a * np.eye(3))
    n = w.miller.astype(np.float64) + np.asarray(w.kred)
    return 0.5 * (2.0 * np.pi / a) ** 2 * float(np.max(np.sum(n * n, axis=1)))


def _ham_with(w, vloc=None, proj=None, ekb=None):
    return oracle.OracleHam(miller=w.miller, recip=w.recip, kred=w.kred, box=w.box,
                            vloc=w.vloc if vloc is None else vloc,
                            proj=w.proj if proj is None else proj,
                            ekb=w.ekb if ekb is None else ekb)


@pytest.mark.parametrize("kred", [(0.0, 0.0, 0.0), (0.5, 0.5, 0.5), (0.1, -0.3, 0.2)])
def test_upper_bound_terms_closed_forms(kred):
    """The Weyl bound b = max T + max V + lambda_max(D+^1/2 P^H P D+^1/2) pinned term by
    term, each against a formula the oracle does not use:
      * empty lattice (V = 0, no projectors): b = max 1/2 |k+G|^2 from the Miller indices;
      * constant V = V0: b = max T + V0 (also for negative V0);
      * one projector p with energy E > 0: b = max T + max V + E ||p||^2 (rank one);
      * a projector with E < 0 adds nothing (D+ clamps it);
      * several projectors: the last term equals lambda_max of the explicit npw x npw
        matrix P D+ P^H (same non-zero spectrum as D+^1/2 P^H P D+^1/2)."""
    w = synth.make_workload("ub", synth.diamond_cell(), kred, 8.0, (24, 24, 24), "s", 4, 8, 1)
    tmax = _max_kinetic_cubic(w)
    none = np.zeros((0, w.npw), dtype=np.complex128)
    zero_v = np.zeros_like(w.vloc)
    assert abs(oracle.upper_bound(_ham_with(w, vloc=zero_v, proj=none, ekb=np.zeros(0)))
               - tmax) < 1e-12 * tmax
    for v0 in (0.7, -1.3):
        b = oracle.upper_bound(_ham_with(w, vloc=np.full_like(w.vloc, v0), proj=none,
                                         ekb=np.zeros(0)))
        assert abs(b - (tmax + v0)) < 1e-12 * tmax
    vmax = float(w.vloc.max())
    p = w.proj[3:4]
    b = oracle.upper_bound(_ham_with(w, proj=p, ekb=np.array([0.8])))
    pn2 = float(np.sum(np.abs(p) ** 2))
    assert abs(b - (tmax + vmax + 0.8 * pn2)) < 1e-12 * b
    b = oracle.upper_bound(_ham_with(w, proj=p, ekb=np.array([-0.8])))
    assert abs(b - (tmax + vmax)) < 1e-12 * b
    ekb = np.array([0.5, 0.25, -0.4, 1.5, 0.0, 0.5, 0.75, 0.1])
    b = oracle.upper_bound(_ham_with(w, ekb=ekb))
    P = w.proj.T                                           # (npw, nproj)
    M = (P * np.maximum(ekb, 0.0)[None, :]) @ P.conj().T   # npw x npw, Hermitian PSD
    lam_nl = float(np.linalg.eigvalsh(M)[-1])
    assert abs(b - (tmax + vmax + lam_nl)) < 1e-11 * b


def test_upper_bound_planted_mistakes_fail():
    """Dropping any term of the bound, or taking min V for max V, changes b on C1
    by more than the tolerance of the pins above (so those pins would catch it)."""
    w = synth.config_c1()
    b = oracle.upper_bound(_ham_with(w))
    tmax = _max_kinetic_cubic(w)
    P = w.proj.T
    lam_nl = float(np.linalg.eigvalsh((P * w.ekb[None, :]) @ P.conj().T)[-1])
    vmax, vmin = float(w.vloc.max()), float(w.vloc.min())
    assert abs(b - (tmax + vmax + lam_nl)) < 1e-11 * b
    for wrong in (vmax + lam_nl, tmax + lam_nl, tmax + vmax, tmax + vmin + lam_nl):
        assert abs(b - wrong) > 1e-3


def test_chfsi_converges_to_exact_c1(c1_dense):
    """C1 with a 24-vector block: the lowest 16 Ritz values reach the exact spectrum."""
    w, ham, lam, U = c1_dense
    X0 = synth.start_block(ham.npw, 24, seed=1).T
    res = oracle.chfsi(ham, X0, degree=8, iters=20)
    assert np.abs(res.eig_history[-1][:16] - lam[:16]).max() < 1e-10
    # monotone (non-increasing) Ritz values across iterations up to rounding
    for t in range(1, len(res.eig_history)):
        assert np.all(res.eig_history[t] <= res.eig_history[t - 1] + 1e-10)


def test_golden_c1_eigenvalues(c1_dense):
    """The stored C1 spectrum (written by tests/golden/make_golden.py from the oracle's
    dense H) still matches; guards the oracle against unnoticed drift."""
    w, ham, lam, U = c1_dense
    ref = np.loadtxt(os.path.join(GOLDEN, "c1_exact_eigs.txt"))
    assert np.abs(lam[:ref.size] - ref).max() < 1e-11
