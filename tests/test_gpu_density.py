"""Electron density on the GPU (pw_density) against the FP64 oracle
(section 2.4, Eq. nandtau): n(r_j) = (1/Omega) sum_b w_b |psi_b(r_j)|^2.

Small boxes are compared element by element with oracle.density; the full
C5 block (512 bands in 77-band chunks, the last one ragged) at sampled
points with oracle.density_at (direct sums over the sphere) and as a whole
through Parseval's charge sum.  Both sides sum the same FP64 terms in
different orders: tolerance max |n - n_ref| <= 1e-12 max |n_ref|.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import to_dev, to_host

pytestmark = pytest.mark.gpu
TOL = 1e-12


def _weights(nb, seed):
    w = np.random.default_rng(seed).uniform(-0.5, 2.0, nb)
    w[::5] = 0.0
    return w


def _c4_cell(box):
    for w in synth.config_c4(ncells=3):
        if tuple(w.box) == box:
            return w
    raise AssertionError(f"no C4 cell with box {box}")


CASES = {
    "C1-24^3": lambda: synth.config_c1(),                # register kernel, one row part
    "C2-k13": lambda: synth.config_c2()[13],             # shifted k-point (k enters only the sphere)
    "C4-30x30x24": lambda: _c4_cell((30, 30, 24)),       # register kernel, odd lane groups
    "C4-32x36x32": lambda: _c4_cell((32, 36, 32)),       # N1 != N2: generic LDS kernel
}


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("nb", [16, 3])
def test_density_matches_oracle(pw, ctx, case, nb):
    import torch
    w = CASES[case]()
    ham = pw.Hamiltonian.from_workload(ctx, w, nb_max=16)
    X = synth.start_block(w.npw, nb, 300 + nb)
    wt = _weights(nb, 7)
    rho = to_host(ham.density(to_dev(X), torch.from_numpy(wt).cuda()))
    ref = oracle.density(oracle.OracleHam.from_workload(w), X.T, wt)
    assert rho.shape == ref.shape == tuple(reversed(w.box))
    err = np.abs(rho - ref).max() / np.abs(ref).max()
    assert err < TOL, err


def test_density_accumulate_deterministic_and_empty(pw, ctx):
    """accumulate adds (k-point sums); repeated calls give the same bits; nb = 0
    writes zeros or leaves rho as it is."""
    import torch
    w = synth.config_c1()
    ham = pw.Hamiltonian.from_workload(ctx, w, nb_max=16)
    Xa, Xb = synth.start_block(w.npw, 16, 1), synth.start_block(w.npw, 9, 2)
    wa, wb = _weights(16, 3), _weights(9, 4)
    r1 = ham.density(to_dev(Xa), torch.from_numpy(wa).cuda())
    r2 = ham.density(to_dev(Xa), torch.from_numpy(wa).cuda())
    assert torch.equal(r1, r2)
    ham.density(to_dev(Xb), torch.from_numpy(wb).cuda(), rho=r1, accumulate=True)
    oh = oracle.OracleHam.from_workload(w)
    ref = oracle.density(oh, Xa.T, wa) + oracle.density(oh, Xb.T, wb)
    assert np.abs(to_host(r1) - ref).max() < TOL * np.abs(ref).max()
    keep = r1.clone()
    empty = torch.zeros((0, w.npw), dtype=torch.complex128, device="cuda")
    ew = torch.zeros(0, dtype=torch.float64, device="cuda")
    ham.density(empty, ew, rho=r1, accumulate=True)
    assert torch.equal(r1, keep)
    ham.density(empty, ew, rho=r1)
    assert torch.count_nonzero(r1).item() == 0


def test_density_padded_leading_dimension(pw, ctx):
    import torch
    w = synth.config_c1()
    ham = pw.Hamiltonian.from_workload(ctx, w, nb_max=8)
    X = synth.start_block(w.npw, 5, 9)
    buf = torch.zeros((5, w.npw + 13), dtype=torch.complex128, device="cuda")
    buf[:, :w.npw] = to_dev(X)
    wt = _weights(5, 10)
    rho = to_host(ham.density(buf[:, :w.npw], torch.from_numpy(wt).cuda()))
    ref = oracle.density(oracle.OracleHam.from_workload(w), X.T, wt)
    assert np.abs(rho - ref).max() < TOL * np.abs(ref).max()


def test_density_rejects_bad_arguments(pw, ctx):
    import torch
    w = synth.config_c1()
    ham = pw.Hamiltonian.from_workload(ctx, w, nb_max=4)
    X = to_dev(synth.start_block(w.npw, 5, 0))
    with pytest.raises(pw.PWError, match="INVALID_ARG"):
        ham.density(X, torch.ones(5, dtype=torch.float64, device="cuda"))       # nb > nb_max
    with pytest.raises(TypeError):
        ham.density(X[:4], torch.ones(4, dtype=torch.float32, device="cuda"))   # weight dtype
    with pytest.raises(TypeError):
        ham.density(X[:4], torch.ones(4, dtype=torch.float64, device="cuda"),
                    rho=torch.zeros(7, dtype=torch.float64, device="cuda"))     # rho size
    # rho sharing memory with psi or with w
    nbox = 24 ** 3
    big = torch.zeros(nbox + 16, dtype=torch.float64, device="cuda")
    psi_alias = big[:8 * w.npw].view(torch.complex128).view(4, w.npw)
    with pytest.raises(pw.PWError, match="rho and psi overlap"):
        ham.density(psi_alias, torch.ones(4, dtype=torch.float64, device="cuda"), rho=big[:nbox])
    with pytest.raises(pw.PWError, match="rho and w overlap"):
        ham.density(X[:4], big[nbox - 2:nbox + 2], rho=big[:nbox])


def test_c5_full_block_sampled_and_charge(pw, ctx):
    """C5 (box 144^3, 124,289 plane waves, 512 bands: seven 77-band chunks, the
    last of 50; two row parts per plane): sampled points against direct sums,
    and Parseval's charge sum over the whole box."""
    import torch
    w = synth.config_c5(with_proj=False)
    ham = pw.Hamiltonian.from_workload(ctx, w, nb_max=512)
    nb = 512
    X = synth.start_block(w.npw, nb, 55)
    wt = _weights(nb, 56)
    rho = ham.density(to_dev(X), torch.from_numpy(wt).cuda())
    oh = oracle.OracleHam.from_workload(w)
    rng = np.random.default_rng(57)
    pts = rng.integers(0, 144, size=(12, 3))
    ref = oracle.density_at(oh, X.T, wt, pts)
    got = to_host(rho)[pts[:, 2], pts[:, 1], pts[:, 0]]
    assert np.abs(got - ref).max() < TOL * np.abs(ref).max()
    charge = oracle.cell_volume(oh) / 144 ** 3 * float(rho.sum().item())
    ref_charge = float(np.sum(wt * np.sum(np.abs(X) ** 2, axis=1)))
    assert abs(charge - ref_charge) < 1e-11 * abs(ref_charge)
