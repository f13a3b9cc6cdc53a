"""Pins of the oracle's structural constraints (Section IV-E: box and
cardinality sets; Section VI-D: rows that are probability mass functions)
against brute force over active sets and exact properties."""
import itertools

import numpy as np
import pytest

from oracle import ntf_oracle as orc


def _spd(F, seed):
    rng = np.random.default_rng(seed)
    M = rng.random((F + 3, F))
    return M.T @ M


def _box_qp_bruteforce(G, w, lo, hi):
    """min 1/2 x^T G x - w^T x over lo <= x <= hi: every assignment of each
    variable to its lower bound, upper bound or free; the free block solves
    its stationarity equations; the best feasible candidate is the minimiser."""
    F = len(w)
    best, best_x = np.inf, None
    for assign in itertools.product((0, 1, 2), repeat=F):
        x = np.zeros(F)
        free = [i for i in range(F) if assign[i] == 2]
        for i in range(F):
            if assign[i] == 0:
                x[i] = lo
            elif assign[i] == 1:
                x[i] = hi
        if free:
            fixed = [i for i in range(F) if assign[i] != 2]
            rhs = w[free] - G[np.ix_(free, fixed)] @ x[fixed]
            x[free] = np.linalg.solve(G[np.ix_(free, free)], rhs)
            if np.any(x[free] < lo - 1e-12) or np.any(x[free] > hi + 1e-12):
                continue
        obj = 0.5 * x @ G @ x - w @ x
        if obj < best:
            best, best_x = obj, x
    return best_x


def _simplex_qp_bruteforce(G, w):
    """min 1/2 x^T G x - w^T x over x >= 0, sum(x) = 1: for every support S
    the equality-constrained minimiser on S; the best feasible one wins."""
    F = len(w)
    best, best_x = np.inf, None
    for r in range(1, F + 1):
        for S in itertools.combinations(range(F), r):
            S = list(S)
            K = np.zeros((r + 1, r + 1))
            K[:r, :r] = G[np.ix_(S, S)]
            K[:r, r] = 1.0
            K[r, :r] = 1.0
            sol = np.linalg.solve(K, np.concatenate([w[S], [1.0]]))
            if np.any(sol[:r] < -1e-12):
                continue
            x = np.zeros(F)
            x[S] = sol[:r]
            obj = 0.5 * x @ G @ x - w @ x
            if obj < best:
                best, best_x = obj, x
    return best_x


@pytest.mark.parametrize("F", [1, 2, 3, 4])
def test_box_inner_sweep_converges_to_bruteforce(F):
    G = _spd(F, 10 + F)
    rng = np.random.default_rng(20 + F)
    W = rng.standard_normal((6, F)) * 2.0
    c = orc.Constraint(kind="box", lo=0.1, hi=0.6)
    rho = orc.rho_trace(G)
    H = np.full((6, F), 0.3)
    H, U, Ht, _ = orc.inner_sweep(W, H, np.zeros_like(H), G, rho, 3000, constraint=c)
    assert np.all(H >= 0.1) and np.all(H <= 0.6)
    for r in range(6):
        np.testing.assert_allclose(H[r], _box_qp_bruteforce(G, W[r], 0.1, 0.6), atol=1e-8)


@pytest.mark.parametrize("F", [1, 2, 3, 5])
def test_pmf_rows_converge_to_simplex_qp(F):
    G = _spd(F, 30 + F)
    rng = np.random.default_rng(40 + F)
    W = rng.standard_normal((5, F)) * 3.0
    rho = orc.rho_trace(G)
    H = np.full((5, F), 1.0 / F)
    c = orc.Constraint(kind="pmf_rows")
    # the primal rows sum to one after every inner iteration (the equality is
    # part of the least-squares step)
    Hk, Uk = H.copy(), np.zeros_like(H)
    for _ in range(5):
        Hk, Uk, Ht, _ = orc.inner_sweep(W, Hk, Uk, G, rho, 1, constraint=c)
        np.testing.assert_allclose(Ht.sum(axis=1), 1.0, atol=1e-13)
        assert np.all(Hk >= 0.0)
    H, U, Ht, _ = orc.inner_sweep(W, H, np.zeros_like(H), G, rho, 4000, constraint=c)
    for r in range(5):
        np.testing.assert_allclose(H[r], _simplex_qp_bruteforce(G, W[r]), atol=1e-8)
        np.testing.assert_allclose(Ht[r], H[r], atol=1e-8)


def test_pmf_ls_step_is_the_constrained_minimiser():
    # the KKT solve against an explicit elimination of the last variable
    F = 4
    G = _spd(F, 50)
    rho = 0.7
    rng = np.random.default_rng(51)
    rhs = rng.standard_normal((3, F))
    X = orc.pmf_rows_ls(G, rho, rhs)
    M = G + rho * np.eye(F)
    for r in range(3):
        # x = e_F + Z y with Z the basis of {sum = 0}: minimise over y
        Z = np.vstack([np.eye(F - 1), -np.ones((1, F - 1))])
        x0 = np.zeros(F)
        x0[-1] = 1.0
        y = np.linalg.solve(Z.T @ M @ Z, Z.T @ (rhs[r] - M @ x0))
        np.testing.assert_allclose(X[r], x0 + Z @ y, atol=1e-12)


def test_cardinality_projection_is_the_nearest_sparse_nonnegative_matrix():
    rng = np.random.default_rng(60)
    V = rng.standard_normal((3, 3))
    for card in range(0, 6):
        P = orc.project(V, orc.Constraint(kind="cardinality", card=card))
        # brute force: over every support of size <= card, the nearest
        # non-negative matrix with that support
        best, best_P = np.inf, None
        flat = V.ravel()
        for r in range(card + 1):
            for S in itertools.combinations(range(flat.size), r):
                Q = np.zeros(flat.size)
                Q[list(S)] = np.maximum(flat[list(S)], 0.0)
                d = np.sum((flat - Q) ** 2)
                if d < best - 1e-15:
                    best, best_P = d, Q
        np.testing.assert_allclose(P.ravel(), best_P)
        assert np.count_nonzero(P) <= card


def test_cardinality_sweep_keeps_at_most_card_nonzeros():
    F = 4
    G = _spd(F, 70)
    rng = np.random.default_rng(71)
    W = rng.random((8, F)) * 3.0
    rho = orc.rho_trace(G)
    c = orc.Constraint(kind="cardinality", card=11)
    H, U = rng.random((8, F)), np.zeros((8, F))
    for _ in range(10):
        H, U, Ht, _ = orc.inner_sweep(W, H, U, G, rho, 1, constraint=c)
        assert np.count_nonzero(H) <= 11 and np.all(H >= 0.0)
        assert not np.any(H * U)
    with pytest.raises(ValueError):
        orc.inner_sweep(W, H, U, G, rho, 2, eps_rel=1e-6, constraint=c)


def test_box_with_zero_lower_bound_and_infinite_upper_is_nonneg():
    F = 3
    G = _spd(F, 80)
    rng = np.random.default_rng(81)
    W = rng.standard_normal((4, F))
    rho = orc.rho_trace(G)
    H0 = rng.random((4, F))
    a = orc.inner_sweep(W, H0, np.zeros_like(H0), G, rho, 7)
    b = orc.inner_sweep(W, H0, np.zeros_like(H0), G, rho, 7,
                        constraint=orc.Constraint(kind="box", lo=0.0, hi=np.inf))
    for x, y in zip(a[:3], b[:3]):
        np.testing.assert_array_equal(x, y)
