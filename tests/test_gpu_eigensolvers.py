"""LOBPCG (pw_lobpcg) and RMM-DIIS (pw_rmm_diis) on the GPU against the FP64
oracle run from the same start block.

Bars: Ritz values within 1e-8 Ha of the oracle's after every line of every
block (LOBPCG) and at the end; relative band residuals of every RMM-DIIS step
within 1e-8 of the oracle's; the carried H y equal to H applied to the
returned y (1e-10 relative, element by element); y orthonormal.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import rel_err, to_dev, to_host

pytestmark = pytest.mark.gpu
EIG_TOL = 1e-8


def _bufs(nb, rows=1):
    import torch
    eig = torch.empty(nb, dtype=torch.float64, device="cuda")
    res = torch.empty(nb, dtype=torch.float64, device="cuda")
    hist = torch.empty(rows * nb, dtype=torch.float64, device="cuda")
    return eig, res, hist


def _check_block(oh, y, hy, eig, nb):
    assert np.abs(y.conj() @ y.T - np.eye(nb)).max() < 1e-12
    assert rel_err(hy, oracle.apply_h(oh, y.T).T) < 1e-10
    assert np.abs(y.conj() @ hy.T - np.diag(eig)).max() < 1e-10


def _lobpcg_case(pw, ctx, w, nb, nblock, nline, seed):
    import torch
    ham = pw.Hamiltonian.from_workload(ctx, w, nb_max=nb)
    oh = oracle.OracleHam.from_workload(w)
    X0 = synth.start_block(w.npw, nb, seed)
    Y = to_dev(X0)
    HY = torch.empty_like(Y)
    eig, res, hist = _bufs(nb, nline + 1)
    ham.lobpcg(Y, HY, eig, res, nblock=nblock, nline=nline, hist=hist)
    ref = oracle.lobpcg(oh, X0.T, nblock, nline)
    h = to_host(hist).reshape(nline + 1, nb)
    for j, (lo, hi) in enumerate(oracle.block_bounds(nb, nblock)):
        for t in range(nline + 1):
            d = np.abs(h[t, lo:hi] - ref.block_history[j][t]).max()
            assert d < EIG_TOL, (j, t, d)
    e = to_host(eig)
    assert np.abs(e - ref.eig).max() < EIG_TOL
    assert np.abs(to_host(res) - ref.resid).max() < 1e-7
    _check_block(oh, to_host(Y), to_host(HY), e, nb)
    return e, ref


@pytest.mark.parametrize("nb,nblock,nline", [(16, 2, 3), (16, 16, 1), (24, 1, 4), (17, 3, 2)])
def test_lobpcg_c1_matches_oracle(pw, ctx, nb, nblock, nline):
    """Block splits with equal and unequal sizes, one band per block, and one
    block of 24 (a 72-wide subspace problem: the block Jacobi solver)."""
    _lobpcg_case(pw, ctx, synth.config_c1(), nb, nblock, nline, seed=1)


def test_lobpcg_c2_kpoint(pw, ctx):
    k = synth.kpoint_grid_shifted(3)[13]
    w = synth.make_workload("C2", synth.diamond_cell(), k, 8.0, (24, 24, 24), "s", 16, 8, 20)
    _lobpcg_case(pw, ctx, w, 16, 4, 2, seed=13)


def test_lobpcg_c3_block_split(pw, ctx):
    """C3 at 160 bands (96^3, 256 s+p projectors) in 4 blocks of 40: the
    120-wide subspace problems run on the block Jacobi solver."""
    _lobpcg_case(pw, ctx, synth.config_c3(), 160, 4, 2, seed=0)


def test_lobpcg_converges_to_exact(pw, ctx):
    """Eight passes on C1 (24 bands in 2 blocks, 4 lines): the lowest 16 Ritz
    values reach the dense spectrum."""
    import torch
    w = synth.config_c1()
    ham = pw.Hamiltonian.from_workload(ctx, w, nb_max=24)
    oh = oracle.OracleHam.from_workload(w)
    Y = to_dev(synth.start_block(w.npw, 24, 2))
    HY = torch.empty_like(Y)
    eig, res, _ = _bufs(24)
    for _ in range(8):
        ham.lobpcg(Y, HY, eig, res, nblock=2, nline=4)
    exact = np.linalg.eigvalsh(oracle.dense_h(oh))
    assert np.abs(to_host(eig)[:16] - exact[:16]).max() < 1e-10
    assert to_host(res)[:16].max() < 1e-6


def _ritz_start(oh, w, nb, seed, iters):
    """Ritz vectors after a few oracle ChFSI iterations: RMM-DIIS starts from
    an earlier solver's output."""
    st = oracle.chfsi(oh, synth.start_block(w.npw, nb, seed).T, degree=8, iters=iters)
    return st.Y.T.copy()


def _rmm_case(pw, ctx, w, nb, ndiis, seed, iters, hy_valid=False):
    import torch
    ham = pw.Hamiltonian.from_workload(ctx, w, nb_max=nb)
    oh = oracle.OracleHam.from_workload(w)
    X0 = _ritz_start(oh, w, nb, seed, iters)
    Y = to_dev(X0)
    HY = to_dev(oracle.apply_h(oh, X0.T).T) if hy_valid else torch.empty_like(Y)
    eig, res, br = _bufs(nb, ndiis + 1)
    ham.rmm_diis(Y, HY, eig, res, ndiis=ndiis, hy_valid=hy_valid, band_resid=br)
    ref = oracle.rmm_diis(oh, X0.T, ndiis)
    got = to_host(br).reshape(ndiis + 1, nb)
    for m in range(ndiis + 1):
        d = np.abs(got[m] - ref.band_resid[m]).max()
        assert d < 1e-8, (m, d)
    e = to_host(eig)
    assert np.abs(e - ref.eig).max() < EIG_TOL
    assert np.abs(to_host(res) - ref.resid).max() < 1e-7
    _check_block(oh, to_host(Y), to_host(HY), e, nb)
    return ref


@pytest.mark.parametrize("ndiis", [1, 3, 5])
def test_rmm_diis_c1_matches_oracle(pw, ctx, ndiis):
    _rmm_case(pw, ctx, synth.config_c1(24), 24, ndiis, seed=4, iters=2)


def test_rmm_diis_reuses_hy(pw, ctx):
    _rmm_case(pw, ctx, synth.config_c1(16), 16, 3, seed=5, iters=2, hy_valid=True)


def test_rmm_diis_c2_kpoint(pw, ctx):
    k = synth.kpoint_grid_shifted(3)[22]
    w = synth.make_workload("C2", synth.diamond_cell(), k, 8.0, (24, 24, 24), "s", 16, 8, 20)
    _rmm_case(pw, ctx, w, 16, 4, seed=22, iters=2)


def test_rmm_diis_c3(pw, ctx):
    _rmm_case(pw, ctx, synth.config_c3(), 160, 3, seed=0, iters=1)


def test_solver_argument_errors(pw, ctx):
    import torch
    w = synth.config_c1()
    ham = pw.Hamiltonian.from_workload(ctx, w, nb_max=8)
    Y = to_dev(synth.start_block(w.npw, 8, 0))
    HY = torch.empty_like(Y)
    eig, res, _ = _bufs(8)
    for kw in ({"nblock": 0}, {"nblock": 9}, {"nline": 0}):
        with pytest.raises(pw.PWError) as e:
            ham.lobpcg(Y, HY, eig, res, **kw)
        assert e.value.status == 1
    for nd in (0, 9):
        with pytest.raises(pw.PWError) as e:
            ham.rmm_diis(Y, HY, eig, res, ndiis=nd)
        assert e.value.status == 1
    with pytest.raises(pw.PWError):
        ham.lobpcg(Y, Y, eig, res)
    big = to_dev(synth.start_block(w.npw, 9, 0))
    e9, r9, _ = _bufs(9)
    with pytest.raises(pw.PWError) as e:
        ham.rmm_diis(big, torch.empty_like(big), e9, r9)     # nb > nb_max
    assert e.value.status == 1
