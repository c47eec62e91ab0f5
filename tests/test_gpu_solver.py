"""Filter, Cholesky orthonormalisation, Rayleigh-Ritz and the whole ChFSI
trajectory on the GPU against the FP64 oracle run from the same start block.

Bars (stated targets for the FP64 path): Ritz values within 1e-8 Ha of the
oracle's; blocks within 1e-10 relative (filter, orthonormalisation).
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import rel_err, to_dev, to_host

pytestmark = pytest.mark.gpu
EIG_TOL = 1e-8


def setup(pw, ctx, w, nb, seed=1):
    ham = pw.Hamiltonian.from_workload(ctx, w, nb_max=nb)
    oh = oracle.OracleHam.from_workload(w)
    X0 = synth.start_block(w.npw, nb, seed)
    return ham, oh, X0


def test_upper_bound_matches_oracle(pw, ctx):
    for w in (synth.config_c1(), synth.config_c3()):
        ham = pw.Hamiltonian.from_workload(ctx, w, nb_max=1)
        b = ham.upper_bound()
        assert abs(b - oracle.upper_bound(oracle.OracleHam.from_workload(w))) < 1e-10 * abs(b)


def test_filter_matches_oracle(pw, ctx):
    w = synth.config_c1()
    ham, oh, X0 = setup(pw, ctx, w, 16)
    b = oracle.upper_bound(oh)
    for m, a, a0, use_hx in [(8, 0.1, -0.18, False), (8, 0.1, -0.18, True), (1, 0.0, -0.2, False),
                             (5, -0.05, -0.2, True)]:
        Y = to_dev(X0)
        hx = ham.apply_h(Y) if use_hx else None
        ham.cheb_filter(Y, m, a, b, a0, hx=hx)
        ref = oracle.cheb_filter(oh, X0.T, m, a, b, a0).T
        assert rel_err(to_host(Y), ref) < 1e-10, (m, use_hx)


def test_orthonormalize_matches_oracle(pw, ctx):
    w = synth.config_c1()
    ham, oh, X0 = setup(pw, ctx, w, 16)
    HX0 = oracle.apply_h(oh, X0.T).T
    Y, HY = to_dev(X0), to_dev(HX0)
    ham.orthonormalize(Y, HY)
    ry, rhy = oracle.orthonormalize(X0.T, HX0.T)
    assert rel_err(to_host(Y), ry.T) < 1e-12
    assert rel_err(to_host(HY), rhy.T) < 1e-12
    y = to_host(Y)
    assert np.abs(y.conj() @ y.T - np.eye(16)).max() < 1e-13


def test_orthonormalize_rank_deficient(pw, ctx):
    w = synth.config_c1()
    ham, oh, X0 = setup(pw, ctx, w, 8)
    X0[5] = X0[2]
    with pytest.raises(pw.PWError) as e:
        ham.orthonormalize(to_dev(X0))
    assert e.value.status == 5


def test_rayleigh_ritz_matches_oracle(pw, ctx):
    import torch
    w = synth.config_c1()
    ham, oh, X0 = setup(pw, ctx, w, 16)
    Yo = oracle.orthonormalize(X0.T)
    lam, Yr, Wr, r = oracle.rayleigh_ritz(oh, Yo)
    Y = to_dev(Yo.T)
    HY = torch.empty_like(Y)
    eig = torch.empty(16, dtype=torch.float64, device="cuda")
    res = torch.empty(16, dtype=torch.float64, device="cuda")
    ham.rayleigh_ritz(Y, HY, eig, res)
    assert np.abs(to_host(eig) - lam).max() < 1e-12
    assert np.abs(to_host(res) - r).max() < 1e-11
    y, hy = to_host(Y), to_host(HY)
    assert rel_err(hy, oracle.apply_h(oh, y.T).T) < 1e-12        # W = H Y after rotation
    assert np.abs(y.conj() @ y.T - np.eye(16)).max() < 1e-13
    assert np.abs(y.conj() @ hy.T - np.diag(lam)).max() < 1e-12


@pytest.mark.parametrize("nb,ncheck", [(16, 14), (24, 16)])
def test_chfsi_c1_trajectory(pw, ctx, nb, ncheck):
    """C1, degree 8, 20 iterations: Ritz values track the oracle's every iteration;
    the bands below the block-edge multiplet reach the exact spectrum."""
    w = synth.config_c1()
    ham, oh, X0 = setup(pw, ctx, w, nb, seed=1)
    st = pw.chfsi(ham, to_dev(X0), degree=8, iters=20, reuse_hx=True)
    ores = oracle.chfsi(oh, X0.T, degree=8, iters=20, upper=st.upper)
    for t, (g, o) in enumerate(zip(st.eig_history, ores.eig_history)):
        assert np.abs(g - o).max() < EIG_TOL, (t, np.abs(g - o).max())
    exact = np.linalg.eigvalsh(oracle.dense_h(oh))
    assert np.abs(st.eig_history[-1][:ncheck] - exact[:ncheck]).max() < EIG_TOL
    assert st.resid_history[-1][:ncheck].max() < 1e-6


@pytest.mark.parametrize("kidx", [4, 22])
def test_chfsi_c2_kpoint(pw, ctx, kidx):
    k = synth.kpoint_grid_shifted(3)[kidx]
    w = synth.make_workload("C2", synth.diamond_cell(), k, 8.0, (24, 24, 24), "s", 16, 8, 20)
    ham, oh, X0 = setup(pw, ctx, w, 16, seed=kidx)
    st = pw.chfsi(ham, to_dev(X0), degree=8, iters=6, reuse_hx=False)
    ores = oracle.chfsi(oh, X0.T, degree=8, iters=6, upper=st.upper)
    d = max(np.abs(g - o).max() for g, o in zip(st.eig_history, ores.eig_history))
    assert d < EIG_TOL, d


def test_chfsi_c4_cell(pw, ctx):
    u, ecut, nb = synth.c4_cell_params(7)
    w = synth.make_workload("C4.7", synth.diamond_cell(strain=u), (0, 0, 0), ecut, None, "s", nb,
                            8, 20)
    ham, oh, X0 = setup(pw, ctx, w, nb, seed=7)
    st = pw.chfsi(ham, to_dev(X0), degree=8, iters=4)
    ores = oracle.chfsi(oh, X0.T, degree=8, iters=4, upper=st.upper)
    d = max(np.abs(g - o).max() for g, o in zip(st.eig_history, ores.eig_history))
    assert d < EIG_TOL, d


def test_chfsi_c3_one_iteration(pw, ctx):
    """C3 at its full block (160 bands, 96^3, 256 projectors): iteration 0 and one
    filter iteration against the oracle."""
    w = synth.config_c3()
    ham, oh, X0 = setup(pw, ctx, w, 160, seed=0)
    st = pw.chfsi(ham, to_dev(X0), degree=8, iters=1, reuse_hx=False)
    ores = oracle.chfsi(oh, X0.T, degree=8, iters=1, upper=st.upper)
    for g, o in zip(st.eig_history, ores.eig_history):
        assert np.abs(g - o).max() < EIG_TOL
    y = to_host(st.Y)
    assert np.abs(y.conj() @ y.T - np.eye(160)).max() < 1e-12
