"""Pins of the oracle's 3D transforms against brute force and invariants.

Convention (oracle docstring): backward e^{+2 pi i m.j/N} unnormalised,
forward e^{-2 pi i m.j/N} scaled by 1/N_box.  The brute-force reference is
the explicit N_box x N_box phase matrix; radices 2, 3, 5 and mixed sizes.
"""
import numpy as np
import pytest

import oracle

SHAPES = [(6, 6, 6), (5, 9, 15), (8, 10, 12), (12, 6, 9), (4, 5, 3)]   # (N3, N2, N1)


@pytest.mark.parametrize("shape", SHAPES)
def test_backward_matches_direct_dft(shape):
    rng = np.random.default_rng(11)
    x = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    got = oracle.fft_backward(x)
    ref = oracle.dft_backward_direct(x)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("shape", SHAPES)
def test_forward_matches_direct_dft(shape):
    rng = np.random.default_rng(12)
    x = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    got = oracle.fft_forward(x)
    ref = oracle.dft_forward_direct(x)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


def test_direct_dft_single_mode():
    """A single box coefficient at m0 gives the plane wave exp(+2 pi i m0.j/N) (closed form)."""
    N3, N2, N1 = 5, 6, 9
    m0 = (2, 4, 7)
    x = np.zeros((N3, N2, N1), dtype=np.complex128)
    x[m0] = 1.0
    j3, j2, j1 = np.meshgrid(np.arange(N3), np.arange(N2), np.arange(N1), indexing="ij")
    wave = np.exp(2j * np.pi * (m0[0] * j3 / N3 + m0[1] * j2 / N2 + m0[2] * j1 / N1))
    assert np.abs(oracle.dft_backward_direct(x) - wave).max() < 1e-12
    assert np.abs(oracle.fft_backward(x) - wave).max() < 1e-12
    back = oracle.fft_forward(wave)
    assert abs(back[m0] - 1.0) < 1e-12 and np.abs(back).sum() - 1.0 < 1e-10


@pytest.mark.parametrize("shape", SHAPES)
def test_roundtrip_and_parseval(shape):
    rng = np.random.default_rng(13)
    x = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    nbox = x.size
    y = oracle.fft_backward(x)
    assert np.abs(oracle.fft_forward(y) - x).max() < 1e-12
    # Parseval for the unnormalised backward transform
    assert abs(np.vdot(y, y).real - nbox * np.vdot(x, x).real) < 1e-10 * nbox * np.vdot(x, x).real
