"""Pins of the oracle's sparse-tensor functions (Section IV-A, item 1: the
MTTKRP from the non-zeros alone; Section VI-A: the RFE) against the dense
definitions, brute force and special cases."""
import itertools

import numpy as np
import pytest

import ntf_synth
from oracle import ntf_oracle as orc


def _random_sparse(dims, n, seed):
    rng = np.random.default_rng(seed)
    flat = rng.choice(int(np.prod(dims)), size=n, replace=False)
    idx = np.stack(np.unravel_index(flat, dims), axis=1).astype(np.int32)
    return orc.SparseTensor(idx=idx, val=rng.standard_normal(n), dims=tuple(dims))


@pytest.mark.parametrize("dims,n,F", [((5, 7, 6), 40, 3), ((12, 3, 9), 100, 5), ((1, 8, 8), 20, 2)])
def test_sparse_mttkrp_equals_dense_mttkrp_of_the_densified_tensor(dims, n, F):
    T = _random_sparse(dims, n, 1)
    rng = np.random.default_rng(2)
    fac = [rng.random((d, F)) for d in dims]
    X = orc.densify(T)
    for m in range(3):
        np.testing.assert_allclose(orc.mttkrp_sparse(T, fac, m), orc.mttkrp(X, fac, m),
                                   rtol=1e-12, atol=1e-13)


def test_sparse_mttkrp_bruteforce_loops():
    T = _random_sparse((4, 3, 5), 17, 3)
    rng = np.random.default_rng(4)
    F = 2
    fac = [rng.random((d, F)) for d in T.dims]
    for m in range(3):
        W = np.zeros((T.dims[m], F))
        X = orc.densify(T)
        for i, j, k in itertools.product(*(range(d) for d in T.dims)):
            c = (i, j, k)
            others = [q for q in range(3) if q != m]
            for f in range(F):
                W[c[m], f] += X[i, j, k] * fac[others[0]][c[others[0]], f] * fac[others[1]][c[others[1]], f]
        np.testing.assert_allclose(orc.mttkrp_sparse(T, fac, m), W, rtol=1e-13, atol=1e-14)


def test_single_nonzero_and_empty_tensor():
    F = 3
    rng = np.random.default_rng(5)
    fac = [rng.random((d, F)) for d in (4, 5, 6)]
    T = orc.SparseTensor(idx=np.array([[2, 4, 1]], dtype=np.int32), val=np.array([1.5]), dims=(4, 5, 6))
    W = orc.mttkrp_sparse(T, fac, 0)
    expect = np.zeros((4, F))
    expect[2] = 1.5 * fac[1][4] * fac[2][1]
    np.testing.assert_allclose(W, expect, rtol=1e-15, atol=0)
    E = orc.SparseTensor(idx=np.zeros((0, 3), dtype=np.int32), val=np.zeros(0), dims=(4, 5, 6))
    for m in range(3):
        assert not np.any(orc.mttkrp_sparse(E, fac, m))


@pytest.mark.parametrize("seed", [6, 7])
def test_sparse_rfe_equals_dense_rfe(seed):
    T = _random_sparse((6, 5, 7), 60, seed)
    rng = np.random.default_rng(seed + 10)
    fac = [rng.random((d, 4)) for d in T.dims]
    assert orc.rfe_sparse(T, fac) == pytest.approx(orc.rfe(orc.densify(T), fac), rel=1e-12)


def test_outer_step_on_sparse_equals_outer_step_on_dense():
    s = ntf_synth.sparse_planted((9, 8, 7), 3, 150, seed=8)
    T = orc.SparseTensor(idx=s.idx, val=s.val.astype(np.float64), dims=s.dims)
    H0 = ntf_synth.init_factors(s.dims, 3, 8)
    a, b = orc.init_state(H0), orc.init_state(H0)
    opts = orc.Opts(inner_iters=4)
    for _ in range(3):
        orc.outer_step(T, a, opts)
        orc.outer_step(orc.densify(T), b, opts)
    for n in range(3):
        np.testing.assert_allclose(a.H[n], b.H[n], rtol=1e-10, atol=1e-12)


def test_sparse_generator_draws_distinct_skewed_coordinates():
    s = ntf_synth.sparse_planted((200, 150, 100), 4, 20000, seed=9)
    n = s.idx.shape[0]
    assert 15000 < n <= 20000
    key = (s.idx[:, 0].astype(np.int64) * 150 + s.idx[:, 1]) * 100 + s.idx[:, 2]
    assert np.unique(key).size == n
    for m, d in enumerate(s.dims):
        assert s.idx[:, m].min() >= 0 and s.idx[:, m].max() < d
        counts = np.bincount(s.idx[:, m], minlength=d)
        # heavy and light slices: the busiest slice holds several times the mean
        assert counts.max() > 4 * counts.mean()
    again = ntf_synth.sparse_planted((200, 150, 100), 4, 20000, seed=9)
    np.testing.assert_array_equal(s.idx, again.idx)
    np.testing.assert_array_equal(s.val, again.val)
