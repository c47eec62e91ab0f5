"""pw_heev_noalloc (the eigensolver with its workspace in the library's
static device array, for callers that cannot allocate) against pw_heev (the
same solver with an allocated workspace) through the C ABI: two calls in a
row, the second smaller, each bit-identical to pw_heev and within 1e-12 of
LAPACK; sizes beyond the static workspace are refused."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _herm(n, seed):
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    return 0.5 * (a + a.conj().T)


@pytest.mark.parametrize("sizes", [(300, 130), (512, 40)])
def test_heev_noalloc_matches_heev(pw, sizes):
    import torch
    ctx = pw.Context(0)
    for i, n in enumerate(sizes):
        a = _herm(n, 100 + n)
        A = torch.from_numpy(a.T.copy()).cuda()          # column-major a as tensor (n, n)
        w_ref, q_ref = ctx.heev(A)
        w, q = ctx.heev_noalloc(A)
        assert torch.equal(w, w_ref), (n, i)
        assert torch.equal(q, q_ref), (n, i)
        wl = np.linalg.eigvalsh(a)
        assert np.abs(w.cpu().numpy() - wl).max() < 1e-12 * np.abs(wl).max()
        qm = q.cpu().numpy().T                           # column-major back to (n, n)
        assert np.abs(qm.conj().T @ a @ qm - np.diag(w.cpu().numpy())).max() < 1e-11 * np.abs(wl).max()
        assert ctx.last_sweeps() > 0


def test_heev_noalloc_rejects_oversize(pw):
    import torch
    ctx = pw.Context(0)
    A = torch.eye(513, dtype=torch.complex128, device="cuda")
    with pytest.raises(pw.PWError) as e:
        ctx.heev_noalloc(A)
    assert e.value.status == 1 and "static workspace" in str(e.value)
