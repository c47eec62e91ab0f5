"""The subspace steps at the benchmarked size against the oracle: C5 (216
atoms, 124,289 plane waves, 864 projectors, 512 bands, box 144^3), one
Cholesky orthonormalisation (section 5.4) and one Rayleigh-Ritz (section 5.1)
on the GPU from the same seeded start block as the oracle, element by element;
and the degree-12 Chebyshev filter (section 5.1) on C3 in FP64 and FP32.

Bars: orthonormalised block within 1e-10 of the oracle's (largest element
error over the largest element; the Cholesky factor is unique, so the block
is); Ritz values within 1e-9 Ha (FP64 target 1e-8); residual norms within
1e-9 of the largest; Ritz vectors, which are unique up to a phase per band,
compared after aligning each band's phase with the oracle's, with a bar scaled
by the smallest gap between Ritz values (the conditioning of an eigenvector).
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import max_err, rel_err, to_dev, to_host

pytestmark = pytest.mark.gpu


def _align_phases(got, ref):
    """Multiply each row (band) of got by the phase that best matches ref's."""
    ov = np.sum(got.conj() * ref, axis=1)
    return got * (ov / np.abs(ov))[:, None]


def _apply_h_chunked(oh, Y, chunk=32):
    """oracle.apply_h band chunk by band chunk (each band independent)."""
    return np.concatenate([oracle.apply_h(oh, Y[:, c:c + chunk])
                           for c in range(0, Y.shape[1], chunk)], axis=1)


@pytest.mark.timeout(600)
def test_c5_orthonormalize_then_rayleigh_ritz(pw, ctx):
    import torch
    w = synth.config_c5()
    nb = 512
    ham = pw.Hamiltonian.from_workload(ctx, w, nb_max=nb)
    oh = oracle.OracleHam.from_workload(w)
    X0 = synth.start_block(w.npw, nb, 0)
    Y = to_dev(X0)
    ham.orthonormalize(Y)
    Yo = oracle.orthonormalize(X0.T)                          # (npw, nb)
    del X0
    e_orth = max_err(to_host(Y), Yo.T)
    print(f"C5 orthonormalize: max element error {e_orth:.3e}")
    assert e_orth < 1e-10
    HY = torch.empty_like(Y)
    eig = torch.empty(nb, dtype=torch.float64, device="cuda")
    res = torch.empty(nb, dtype=torch.float64, device="cuda")
    ham.rayleigh_ritz(Y, HY, eig, res)
    Wo = _apply_h_chunked(oh, Yo)
    lam, Yr, Wr, r = oracle.rayleigh_ritz(oh, Yo, W=Wo)
    del Yo, Wo
    d_eig = float(np.abs(to_host(eig) - lam).max())
    d_res = float(np.abs(to_host(res) - r).max() / r.max())
    gap = float(np.diff(lam).min())
    print(f"C5 Rayleigh-Ritz: |dlambda| {d_eig:.3e} Ha, residual {d_res:.3e}, "
          f"smallest Ritz gap {gap:.3e} Ha")
    assert d_eig < 1e-9
    assert d_res < 1e-9
    vec_tol = max(1e-10, 1e-13 * float(lam[-1] - lam[0]) / gap)
    yg = _align_phases(to_host(Y), Yr.T)
    e_y = max_err(yg, Yr.T)
    del yg
    wg = _align_phases(to_host(HY), Wr.T)
    e_w = max_err(wg, Wr.T)
    print(f"C5 Ritz vectors: Y {e_y:.3e}, W {e_w:.3e} (bar {vec_tol:.3e})")
    assert e_y < vec_tol and e_w < vec_tol
    del Y, HY
    torch.cuda.empty_cache()


@pytest.fixture(scope="module")
def c3_filter_case():
    w = synth.config_c3()
    oh = oracle.OracleHam.from_workload(w)
    X0 = synth.start_block(w.npw, w.nb, 3)
    b = oracle.upper_bound(oh)
    a, a0 = 0.9, -0.45                       # inside the C3 spectrum, as after a few iterations
    ref = oracle.cheb_filter(oh, X0.T, 12, a, b, a0).T
    return w, X0, a, b, a0, ref


@pytest.mark.timeout(300)
def test_c3_degree12_filter_fp64(pw, ctx, c3_filter_case):
    w, X0, a, b, a0, ref = c3_filter_case
    ham = pw.Hamiltonian.from_workload(ctx, w, nb_max=w.nb)
    Y = to_dev(X0)
    ham.cheb_filter(Y, 12, a, b, a0)
    err = rel_err(to_host(Y), ref)
    print(f"C3 degree-12 FP64 filter: {err:.3e}")
    assert err < 1e-10


@pytest.mark.timeout(300)
def test_c3_degree12_filter_fp32(pw, ctx, c3_filter_case):
    """The mixed path's filter (FFT route in FP32, three-term bf16 projector
    products): FP32 rounding through twelve products, bar 1e-4 on the largest
    element (measured value printed)."""
    w, X0, a, b, a0, ref = c3_filter_case
    ham = pw.Hamiltonian.from_workload(ctx, w, nb_max=w.nb, low_prec=True)
    Y = to_dev(X0)
    ham.cheb_filter(Y, 12, a, b, a0, prec="fp32")
    err = rel_err(to_host(Y), ref)
    print(f"C3 degree-12 FP32 filter: {err:.3e}")
    assert err < 1e-4
