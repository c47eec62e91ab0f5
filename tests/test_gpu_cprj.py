"""Projections kept in memory: after Rayleigh-Ritz (the ChFSI loop), LOBPCG
and RMM-DIIS the handle holds C = P^H Y of the Ritz vectors it returned,
carried through the Cholesky solves, projections and rotations by small
products.  Checked element by element against P^H Y formed on the host from
the returned Y (1e-12 of max |C|), and that fetching them forms no
projection product."""
import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import max_err, to_dev, to_host

pytestmark = pytest.mark.gpu


def _ref(w, Y):
    proj = oracle.OracleHam.from_workload(w).proj      # (nproj, npw): row j = <k+G|p_j>
    return (proj.conj() @ to_host(Y).T).T               # (nb, nproj): <p_j|y_b>


def _ham(pw, ctx, w, nb):
    return pw.Hamiltonian.from_workload(ctx, w, nb_max=nb)


def _bufs(nb):
    import torch
    return (torch.empty(nb, dtype=torch.float64, device="cuda"),
            torch.empty(nb, dtype=torch.float64, device="cuda"))


@pytest.mark.parametrize("cfg,nb", [("C1", 16), ("C3", 160)])
def test_cprj_after_chfsi(pw, ctx, cfg, nb):
    w = synth.config_c1() if cfg == "C1" else synth.config_c3()
    ham = _ham(pw, ctx, w, nb)
    st = pw.chfsi(ham, to_dev(synth.start_block(w.npw, nb, 3)), degree=8, iters=2)
    ctx.set_timing(True)
    ctx.reset_timing()
    C = ham.cprj(nb)
    stages = ctx.stage_times()
    ctx.set_timing(False)
    assert stages["proj"][1] == 0                         # no projection product formed
    assert max_err(to_host(C), _ref(w, st.Y)) < 1e-12


@pytest.mark.parametrize("nblock,nline", [(2, 3), (1, 2)])
def test_cprj_after_lobpcg(pw, ctx, nblock, nline):
    import torch
    w = synth.config_c1()
    ham = _ham(pw, ctx, w, 16)
    Y = to_dev(synth.start_block(w.npw, 16, 4))
    HY = torch.empty_like(Y)
    eig, res = _bufs(16)
    ham.lobpcg(Y, HY, eig, res, nblock=nblock, nline=nline)
    assert max_err(to_host(ham.cprj(16)), _ref(w, Y)) < 1e-12
    assert max_err(to_host(ham.cprj(5)), _ref(w, Y)[:5]) < 1e-12


def test_cprj_after_lobpcg_c3(pw, ctx):
    import torch
    w = synth.config_c3()
    ham = _ham(pw, ctx, w, 160)
    Y = to_dev(synth.start_block(w.npw, 160, 0))
    HY = torch.empty_like(Y)
    eig, res = _bufs(160)
    ham.lobpcg(Y, HY, eig, res, nblock=4, nline=2)
    assert max_err(to_host(ham.cprj(160)), _ref(w, Y)) < 1e-12


@pytest.mark.parametrize("ndiis,hy_valid", [(1, False), (1, True), (3, True), (4, False)])
def test_cprj_after_rmm_diis(pw, ctx, ndiis, hy_valid):
    w = synth.config_c1()
    ham = _ham(pw, ctx, w, 16)
    st = pw.chfsi(ham, to_dev(synth.start_block(w.npw, 16, 5)), degree=8, iters=2)
    Y, HY = st.Y, st.HY
    eig, res = _bufs(16)
    ham.rmm_diis(Y, HY, eig, res, ndiis=ndiis, hy_valid=hy_valid)
    assert max_err(to_host(ham.cprj(16)), _ref(w, Y)) < 1e-12


def test_cprj_availability(pw, ctx):
    import torch
    w = synth.config_c1()
    ham = _ham(pw, ctx, w, 8)
    with pytest.raises(pw.PWError) as e:                  # no Rayleigh-Ritz yet
        ham.cprj(8)
    assert e.value.status == 1
    Y = to_dev(synth.start_block(w.npw, 8, 1))
    HY = torch.empty_like(Y)
    eig, res = _bufs(8)
    ham.orthonormalize(Y)
    ham.rayleigh_ritz(Y[:6], HY[:6], eig, res)
    ham.cprj(6)
    with pytest.raises(pw.PWError):                       # only 6 Ritz vectors were returned
        ham.cprj(7)
