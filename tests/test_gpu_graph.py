"""The single-k hot calls neither synchronise nor allocate, so one whole
Chebyshev-filtered iteration -- filter reusing H Y, Cholesky
orthonormalisation, Rayleigh-Ritz, the shape of the benchmarked step -- can
be captured into one HIP graph.  Replays must equal the same calls issued
directly, bit for bit, with unrelated eager work between replays.  Failures
only the device sees (a Cholesky pivot, the eigensolver's sweep limit) come
back through the context's deferred status.
"""
import numpy as np
import pytest

import synth
from gpu_helpers import to_dev

pytestmark = pytest.mark.gpu


def _state(pw, nb, seed):
    import torch
    w = synth.config_c1()
    s = torch.cuda.Stream()
    ctx = pw.Context(0, stream=s)
    ham = pw.Hamiltonian.from_workload(ctx, w, nb_max=nb)
    with torch.cuda.stream(s):
        Y = to_dev(synth.start_block(w.npw, nb, seed))
        HY = torch.empty_like(Y)
        eig = torch.empty(nb, dtype=torch.float64, device="cuda")
        res = torch.empty_like(eig)
    s.synchronize()
    return ctx, ham, s, Y, HY, eig, res


@pytest.mark.parametrize("nb", [16, 96])   # one-workgroup eigensolver; block Jacobi (n > 64)
def test_iteration_graph_replay_is_bit_identical(pw, nb):
    import torch
    ctx, ham, s, Y, HY, eig, res = _state(pw, nb, seed=3)
    with torch.cuda.stream(s):
        ham.orthonormalize(Y, check=False)
        ham.rayleigh_ritz(Y, HY, eig, res, check=False)
    ctx.check_status()
    lam = eig.cpu().numpy()
    a, a0, b = float(lam[-1]), float(lam[0]), ham.upper_bound()
    with torch.cuda.stream(s):
        Y0, HY0 = Y.clone(), HY.clone()

    def step():
        ham.cheb_filter(Y, 8, a, b, a0, hx=HY)
        ham.orthonormalize(Y, check=False)
        ham.rayleigh_ritz(Y, HY, eig, res, check=False)

    with torch.cuda.stream(s):
        step()
    ctx.check_status()
    ref = [t.clone() for t in (Y, HY, eig, res)]
    assert np.all(np.diff(ref[2].cpu().numpy()) >= 0)

    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        Y.copy_(Y0)
        HY.copy_(HY0)
    s.synchronize()
    with torch.cuda.graph(g, stream=s):
        step()
    for rep in range(3):
        with torch.cuda.stream(s):
            Y.copy_(Y0)
            HY.copy_(HY0)
            eig.zero_()
            res.zero_()
            g.replay()
        junk = torch.randn(4096, 64, device="cuda") @ torch.randn(64, 64, device="cuda")
        torch.cuda.synchronize()
        del junk
        ctx.check_status()
        for got, want, name in zip((Y, HY, eig, res), ref, ("Y", "HY", "eig", "resid")):
            assert torch.equal(got, want), (rep, name)


def test_deferred_not_posdef_then_cleared(pw):
    import torch
    ctx, ham, s, Y, HY, eig, res = _state(pw, 8, seed=1)
    with torch.cuda.stream(s):
        Y[5].copy_(Y[2])
        ham.orthonormalize(Y, check=False)          # enqueued; returns without a status
    with pytest.raises(pw.PWError) as e:
        ctx.check_status()
    assert e.value.status == 5 and "pw_orthonormalize" in str(e.value) and "pivot 5" in str(e.value)
    ctx.check_status()                               # the word was cleared


def test_deferred_nonfinite_column_then_cleared(pw):
    """A NaN in one band of the block makes that band's Gram diagonal entry
    NaN: the Cholesky step's init kernel reports the column as non-finite
    (PW_ERR_NONFINITE), not as a failed pivot; an infinity likewise."""
    import torch
    for bad in (float("nan"), float("inf")):
        ctx, ham, s, Y, HY, eig, res = _state(pw, 8, seed=1)
        with torch.cuda.stream(s):
            Y[6, 17] = bad
            ham.orthonormalize(Y, check=False)
        with pytest.raises(pw.PWError) as e:
            ctx.check_status()
        assert e.value.status == 6 and "pw_orthonormalize" in str(e.value), str(e.value)
        assert "column 6 " in str(e.value), str(e.value)
        ctx.check_status()


def test_deferred_sweep_limit(pw):
    """A random 96 x 96 subspace matrix cannot be diagonalised in one Jacobi
    sweep: with the limit at 1 the device reports NO_CONVERGENCE; at the
    default limit the same call succeeds."""
    import torch
    ctx, ham, s, Y, HY, eig, res = _state(pw, 96, seed=2)
    with torch.cuda.stream(s):
        ham.orthonormalize(Y, check=False)
        Y1 = Y.clone()
    ctx.check_status()
    ctx.set_sweep_limit(1)
    with torch.cuda.stream(s):
        ham.rayleigh_ritz(Y, HY, eig, res, check=False)
    with pytest.raises(pw.PWError) as e:
        ctx.check_status()
    assert e.value.status == 7 and "pw_rayleigh_ritz" in str(e.value)
    ctx.set_sweep_limit(24)
    with torch.cuda.stream(s):
        Y.copy_(Y1)
        ham.rayleigh_ritz(Y, HY, eig, res, check=False)
    ctx.check_status()
    assert 1 < ctx.last_sweeps() <= 24
    with pytest.raises(pw.PWError):
        ctx.set_sweep_limit(0)


def test_low_precision_gram_needs_low_prec_handle(pw, ctx):
    w = synth.config_c1()
    ham = pw.Hamiltonian.from_workload(ctx, w, nb_max=8)          # FP64 only
    Y = to_dev(synth.start_block(w.npw, 8, 0))
    with pytest.raises(pw.PWError) as e:
        ham.orthonormalize(Y, gram_prec="bf16")
    assert e.value.status == 2


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_overlap_is_bit_identical(pw, prec):
    """P^H psi on the second stream (default) or on the context's stream:
    the same kernels on the same data, so the same bits (C3, 160 bands, a
    degree-8 filter reusing H Y, orthonormalisation, Rayleigh-Ritz)."""
    import torch
    w = synth.config_c3()
    out = {}
    for ov in (False, True):
        ctx = pw.Context(0)
        ctx.set_overlap(ov)
        ham = pw.Hamiltonian.from_workload(ctx, w, nb_max=160, low_prec=prec != "fp64")
        st = pw.chfsi(ham, to_dev(synth.start_block(w.npw, 160, 2)), degree=8, iters=1,
                      filter_prec=prec)
        torch.cuda.synchronize()
        out[ov] = (st.Y.clone(), st.HY.clone(), st.eig.clone())
    for a, b in zip(out[False], out[True]):
        assert torch.equal(a, b)
