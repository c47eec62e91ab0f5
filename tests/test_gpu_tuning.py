"""Launch-shape tuning: every tuning a handle accepts gives the same H*psi
(to the FP64 bar against the oracle), the tuner keeps a valid choice, and the
JSON cache replays it."""
import itertools

import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import rel_err, to_dev, to_host

pytestmark = pytest.mark.gpu


def all_tunings(ham, nb):
    base = ham.get_tuning()
    out = []
    for rc, rp, pv, pv32 in itertools.product((0, 1), (0, 1), (0, 1), (0, 1, 2)):
        for ch in sorted({base["chunk"], max(1, base["chunk"] // 2), 1}):
            for gb in (4096, 2048, 256):
                out.append(dict(reg_col=rc, reg_plane=rp, plane_variant=pv, plane_variant32=pv32,
                                chunk=ch, gemm_blocks=gb, nn_tile=0, nn_tile32=0))
    out.append(dict(base, nn_tile=1))
    out.append(dict(base, nn_tile32=1))
    out.append(dict(base, nn_tile=1, nn_tile32=1, gemm_blocks=1))
    return out


@pytest.mark.parametrize("which", ["C1", "C4.2", "C3"])
def test_every_accepted_tuning_matches_oracle(pw, ctx, which):
    if which == "C1":
        w, nb = synth.config_c1(), 16
    elif which == "C3":
        w, nb = synth.config_c3(), 6
    else:
        w, nb = synth.config_c4()[2], 12
    import torch
    ham = pw.Hamiltonian.from_workload(ctx, w, nb_max=nb, low_prec=True)
    X0 = synth.start_block(w.npw, nb, 3)
    ref = oracle.apply_h(oracle.OracleHam.from_workload(w), X0.T).T
    X = to_dev(X0)
    X32 = X.to(torch.complex64)
    accepted = 0
    for t in all_tunings(ham, nb):
        try:
            ham.set_tuning(t)
        except pw.PWError as e:
            assert e.status == 2, (t, e)            # no such kernel for this box
            continue
        accepted += 1
        err = rel_err(to_host(ham.apply_h(X)), ref)
        assert err < 1e-10, (t, err)
        e32 = rel_err(to_host(ham.apply_h(X32, prec="fp32")).astype(np.complex128), ref)
        assert e32 < 2e-6, (t, e32)
    assert accepted >= 4


def test_set_tuning_rejects(pw, ctx):
    w = synth.config_c4()[0]                 # box 32 x 36 x 32: no register plane kernel
    ham = pw.Hamiltonian.from_workload(ctx, w, nb_max=8)
    with pytest.raises(pw.PWError) as e:
        ham.set_tuning({"reg_plane": 1})
    assert e.value.status == 2
    for bad in ({"chunk": 0}, {"chunk": 10 ** 6}, {"gemm_blocks": 4097}, {"reg_col": 2},
                {"nn_tile": 2}, {"nn_tile32": -1}):
        with pytest.raises(pw.PWError) as e:
            ham.set_tuning(bad)
        assert e.value.status == 1, bad


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_autotune_and_cache(pw, ctx, tmp_path, prec):
    w = synth.config_c1()
    ham = pw.Hamiltonian.from_workload(ctx, w, nb_max=16, low_prec=True)
    cache = str(tmp_path / "tune.txt")
    r = ham.autotune(prec, nb=16, reps=2, cache=cache)
    assert not r["cached"] and r["ms"] <= r["default_ms"] * 1.0001
    chosen = ham.get_tuning()
    assert all(chosen[k] == r[k] for k in chosen)
    lines = open(cache).read().splitlines()
    assert [ln.split()[0] for ln in lines] == [ham.tuning_key(prec, 16)]
    assert all(f"{k}={chosen[k]}" in lines[0].split() for k in chosen)
    ham2 = pw.Hamiltonian.from_workload(ctx, w, nb_max=16, low_prec=True)
    r2 = ham2.autotune(prec, nb=16, cache=cache)
    assert r2["cached"] and ham2.get_tuning() == chosen
    X0 = synth.start_block(w.npw, 16, 0)
    ref = oracle.apply_h(oracle.OracleHam.from_workload(w), X0.T).T
    assert rel_err(to_host(ham2.apply_h(to_dev(X0))), ref) < 1e-10
