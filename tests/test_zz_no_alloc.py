"""ntf_inner_update_noalloc (scratch in the library's fixed device array, no
workspace) against ntf_inner_update (caller workspace), through the C ABI.

Both run the same kernels, so H, U, the per-row iteration counts and Ht must
agree bitwise.  Two calls in a row on the no-alloc side, the second with a
smaller problem (fewer rows, smaller F), check that the array's leftover
contents from the first call do not leak into the second; a third call with
a given penalty and row-wise early stop covers the other prepare policy.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1409_2383_amd as ntf
    ntf.library_path()
    return torch.device("cuda:0")


def _row_problem(rows, F, seed, dtype, dev):
    rng = np.random.default_rng(seed)
    A = rng.random((3 * F, F))
    G = A.T @ A                                    # PSD, like a Gram Hadamard product
    W = rng.random((rows, F)) @ G                  # rows whose NNLS solutions are mostly interior
    W[:, ::3] -= 0.5 * np.abs(W[:, ::3]).mean()    # and some active bounds
    H = rng.random((rows, F))
    U = np.zeros((rows, F))
    t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a, dtype=dt)).to(dev)
    return t(W, np.float64), t(G, np.float64), t(H, dtype), t(U, dtype)


def _both(dev, rows, F, seed, dtype, rho, T, eps):
    import paper_1409_2383_amd as ntf
    W, G, H, U = _row_problem(rows, F, seed, dtype, dev)
    H2, U2 = H.clone(), U.clone()
    print(f"[no-alloc] rows={rows} F={F} dtype={dtype.__name__} rho={rho} T={T} eps={eps}",
          flush=True)
    it_ref, ht_ref = ntf.inner_update(W, H, U, G, rho, T, eps, eps, want_iters=True, want_ht=True)
    it = torch.zeros(rows, dtype=torch.int32, device=dev)
    ht = torch.empty_like(H2)
    ntf.inner_update_noalloc(W, H2, U2, G, rho, T, eps, eps, iters=it, ht=ht)
    torch.cuda.synchronize()
    assert torch.equal(H2, H)
    assert torch.equal(U2, U)
    assert torch.equal(ht, ht_ref)
    assert torch.equal(it, it_ref)
    assert bool(torch.isfinite(H2).all())


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_noalloc_matches_workspace_call(dev, dtype):
    _both(dev, 1000, 64, 1, dtype, 0.0, 10, 0.0)    # rho = tr(G)/F, fixed T
    _both(dev, 333, 21, 2, dtype, 0.0, 7, 0.0)      # smaller: fewer rows, smaller F
    _both(dev, 97, 5, 3, dtype, 2.5, 200, 1e-8)     # given rho, row-wise early stop


def test_noalloc_scratch_size_and_errors(dev):
    import paper_1409_2383_amd as ntf
    from paper_1409_2383_amd import _lib
    L = _lib.lib()
    sizes = [int(L.ntf_inner_static_scratch_bytes(F)) for F in (1, 8, 64)]
    assert 0 < sizes[0] <= sizes[1] <= sizes[2] <= 128 * 1024
    assert int(L.ntf_inner_static_scratch_bytes(65)) == 0
    W, G, H, U = _row_problem(8, 4, 4, np.float64, dev)
    with pytest.raises(Exception):
        ntf.inner_update_noalloc(W, H, U, G, 0.0, 0)          # T < 1
