"""Dense building blocks on the GPU against numpy/LAPACK (FP64 complex):
split-K A^H B, A B, upper Cholesky + inverse, Jacobi Hermitian eigensolver."""
import numpy as np
import pytest

from gpu_helpers import to_dev, to_host

pytestmark = pytest.mark.gpu


def crand(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


@pytest.mark.parametrize("m,n,k", [(8, 16, 1189), (70, 33, 5000), (1, 1, 3), (64, 64, 128),
                                   (256, 160, 37073), (17, 130, 257)])
def test_gemm_cn(ctx, m, n, k):
    rng = np.random.default_rng(m * 7 + n)
    A = crand(rng, m, k)          # tensor (m, k) = column-major k x m
    B = crand(rng, n, k)
    C = to_host(ctx.gemm_cn(to_dev(A), to_dev(B), alpha=0.5))   # (n, m) = column-major m x n
    ref = 0.5 * (A.conj() @ B.T)  # (m, n): sum_k conj(A[i,k]) B[j,k]
    assert np.abs(C.T - ref).max() < 1e-12 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("m,n,k", [(1189, 16, 8), (130, 70, 65), (1000, 100, 300), (3, 1, 1)])
def test_gemm_nn(ctx, m, n, k):
    rng = np.random.default_rng(m + n + k)
    A = crand(rng, k, m)          # column-major m x k
    B = crand(rng, n, k)          # column-major k x n
    C0 = crand(rng, n, m)
    Cd = to_dev(C0)
    out = to_host(ctx.gemm_nn(to_dev(A), to_dev(B), alpha=-1.5, beta=0.25, C=Cd))
    ref = -1.5 * (A.T @ B.T) + 0.25 * C0.T      # (m, n)
    assert np.abs(out.T - ref).max() < 1e-12 * max(1.0, np.abs(ref).max())


def test_gemm_nn_empty_contraction(pw, ctx):
    """k = 0: C = beta C (no operand element is read)."""
    import torch
    rng = np.random.default_rng(5)
    m, n = 70, 9
    C0 = crand(rng, n, m)
    Cd = to_dev(C0)
    one = torch.zeros(1, dtype=torch.complex128, device="cuda")   # valid pointers, never read
    ctx.check(pw._LIB.pw_gemm_nn(ctx.handle, m, n, 0, 2.0, one.data_ptr(), m, one.data_ptr(),
                                      1, 0.5, Cd.data_ptr(), m))
    assert np.array_equal(to_host(Cd), 0.5 * C0)


def hpd(rng, n, cond=1e3):
    Q, _ = np.linalg.qr(crand(rng, n, n))
    d = np.geomspace(1.0, cond, n)
    return (Q * d) @ Q.conj().T


@pytest.mark.parametrize("n", [1, 16, 64, 100, 160, 200, 256, 511, 512])
def test_potrf_inv(ctx, n):
    rng = np.random.default_rng(n)
    S = hpd(rng, n)
    Ud, Xd = ctx.potrf_inv(to_dev(S.T.copy()))     # column-major storage
    U, X = to_host(Ud).T, to_host(Xd).T
    assert np.abs(np.tril(U, -1)).max() == 0.0
    assert np.all(np.diag(U).real > 0) and np.abs(np.diag(U).imag).max() == 0.0
    assert np.abs(U.conj().T @ U - S).max() < 1e-12 * np.abs(S).max()
    assert np.abs(U @ X - np.eye(n)).max() < 1e-11
    L = np.linalg.cholesky(S)                          # LAPACK: S = L L^H, U = L^H
    assert np.abs(U - L.conj().T).max() < 1e-11 * np.abs(L).max()


@pytest.mark.parametrize("n,cond", [(512, 1e8), (512, 1e12), (160, 1e12)])
def test_potrf_inv_ill_conditioned(ctx, n, cond):
    """Gram matrices of a filtered block are ill-conditioned (the filter
    amplifies the wanted directions by large factors): backward error of the
    factor and of its inverse at the sizes of the C3 and C5 blocks."""
    rng = np.random.default_rng(int(n + np.log10(cond)))
    S = hpd(rng, n, cond)
    Ud, Xd = ctx.potrf_inv(to_dev(S.T.copy()))
    U, X = to_host(Ud).T, to_host(Xd).T
    assert np.abs(U.conj().T @ U - S).max() < 1e-13 * n * np.abs(S).max()
    # U X = I up to the conditioning of U (sqrt(cond))
    assert np.abs(U @ X - np.eye(n)).max() < 1e-15 * n * np.sqrt(cond)
    L = np.linalg.cholesky(S)
    assert np.abs(U - L.conj().T).max() < 1e-15 * n * cond * np.abs(L).max()


def test_potrf_not_posdef(pw, ctx):
    rng = np.random.default_rng(1)
    Y = crand(rng, 40, 6)
    Y[:, 4] = Y[:, 2]
    S = Y.conj().T @ Y
    with pytest.raises(pw.PWError) as e:
        ctx.potrf_inv(to_dev(S.T.copy()))
    assert e.value.status == 5 and "pivot 4" in str(e.value)


def test_potrf_nonfinite_diagonal(pw, ctx):
    """A NaN column of Y gives S = Y^H Y a NaN diagonal entry: reported as
    PW_ERR_NONFINITE with its index (the first one, here in the second
    64-wide diagonal block), ahead of any pivot test."""
    rng = np.random.default_rng(2)
    Y = crand(rng, 200, 90)
    Y[7, 70] = np.nan
    Y[3, 81] = np.inf
    S = Y.conj().T @ Y
    with pytest.raises(pw.PWError) as e:
        ctx.potrf_inv(to_dev(S.T.copy()))
    assert e.value.status == 6 and "diagonal entry 70 " in str(e.value), str(e.value)


@pytest.mark.parametrize("n", [1, 2, 16, 24, 63, 64, 65, 100, 160, 257, 512])
def test_heev_random(ctx, n):
    rng = np.random.default_rng(100 + n)
    M = crand(rng, n, n)
    A = 0.5 * (M + M.conj().T)
    w, Qd = ctx.heev(to_dev(A.T.copy()))
    w, Q = to_host(w), to_host(Qd).T
    ref = np.linalg.eigvalsh(A)
    scale = np.abs(ref).max()
    assert ctx.last_sweeps() > 0 or n == 1
    assert np.abs(w - ref).max() < 1e-12 * scale
    assert np.abs(Q.conj().T @ Q - np.eye(n)).max() < 1e-12
    assert np.abs(A @ Q - Q * w[None, :]).max() < 1e-11 * scale


@pytest.mark.parametrize("n", [24, 96, 129])
def test_heev_degenerate(ctx, n):
    """Exactly repeated eigenvalues (multiplets, as cubic cells produce)."""
    rng = np.random.default_rng(n)
    Q0, _ = np.linalg.qr(crand(rng, n, n))
    lam = np.repeat(np.linspace(-1.0, 2.0, -(-n // 6)), 6)[:n]
    A = (Q0 * lam) @ Q0.conj().T
    A = 0.5 * (A + A.conj().T)
    w, Qd = ctx.heev(to_dev(A.T.copy()))
    w, Q = to_host(w), to_host(Qd).T
    assert np.abs(w - np.sort(lam)).max() < 1e-12
    assert np.abs(Q.conj().T @ Q - np.eye(n)).max() < 1e-12
    assert np.abs(A @ Q - Q * w[None, :]).max() < 1e-11
