"""Pins of the oracle's order-N form (Appendix A): unfoldings, Khatri-Rao
matrices and MTTKRP of four- and five-way tensors against brute force and the
appendix's unfolding relations, and one ADMoM iteration in the sweep form
against the explicit form of eqs. ADMoM_NTF / ADMM_NTF_ALS_C."""
import itertools

import numpy as np
import pytest

import ntf_synth
from oracle import ntf_oracle as orc


@pytest.mark.parametrize("dims", [(3, 4, 2, 5), (2, 3, 2, 2, 3)])
def test_mttkrp_nway_bruteforce(dims):
    rng = np.random.default_rng(1)
    F = 3
    X = rng.standard_normal(dims)
    fac = [rng.random((d, F)) for d in dims]
    N = len(dims)
    for n in range(N):
        W = np.zeros((dims[n], F))
        for idx in itertools.product(*(range(d) for d in dims)):
            prod = np.ones(F)
            for m in range(N):
                if m != n:
                    prod = prod * fac[m][idx[m]]
            W[idx[n]] += X[idx] * prod
        np.testing.assert_allclose(orc.mttkrp(X, fac, n), W, rtol=1e-12, atol=1e-13)


def test_unfoldings_of_a_four_way_model_follow_appendix_a():
    # [A, B, C, D] unfolds as W^(1) = A (D (.) (C (.) B))^T, ..., W^(4) = D (C (.) (B (.) A))^T
    rng = np.random.default_rng(2)
    A, B, C, D = (rng.random((d, 3)) for d in (3, 4, 2, 5))
    Wt = orc.reconstruct([A, B, C, D])
    kr = orc.khatri_rao
    np.testing.assert_allclose(orc.unfold(Wt, 0), A @ kr(D, kr(C, B)).T, rtol=1e-13)
    np.testing.assert_allclose(orc.unfold(Wt, 1), B @ kr(D, kr(C, A)).T, rtol=1e-13)
    np.testing.assert_allclose(orc.unfold(Wt, 2), C @ kr(D, kr(B, A)).T, rtol=1e-13)
    np.testing.assert_allclose(orc.unfold(Wt, 3), D @ kr(C, kr(B, A)).T, rtol=1e-13)


def test_reconstruct_nway_entries():
    rng = np.random.default_rng(3)
    fac = [rng.random((d, 2)) for d in (2, 3, 2, 2)]
    M = orc.reconstruct(fac)
    for idx in itertools.product(*(range(f.shape[0]) for f in fac)):
        v = sum(np.prod([fac[m][idx[m], f] for m in range(4)]) for f in range(2))
        assert M[idx] == pytest.approx(v, rel=1e-14)


def test_gram_hadamard_nway_equals_explicit_kr_gram():
    rng = np.random.default_rng(4)
    fac = [rng.random((d, 3)) for d in (3, 4, 2, 5)]
    for n in range(4):
        K = orc.kr_for_mode(fac, n)
        np.testing.assert_allclose(orc.gram_hadamard(fac, n), K.T @ K, rtol=1e-12)


def test_four_way_sweep_form_equals_explicit_form():
    dims, F = (5, 4, 6, 3), 2
    X, _, _ = ntf_synth.planted_nway(dims, F, seed=5, sigma2=1e-2, dtype=np.float64)
    H0 = ntf_synth.init_factors(dims, F, 5)
    rho = [1.3, 0.7, 2.1, 0.9]
    P = [h.copy() for h in H0]
    Aux = [np.zeros_like(h) for h in H0]
    Y = [np.zeros_like(h) for h in H0]
    st = orc.init_state(H0, paper=True)
    st.rho = list(rho)
    opts = orc.Opts(inner_iters=1, rho_policy=orc.RHO_FIXED, factor_source=1)
    for _ in range(5):
        P, Aux, Y = orc.paper_admom_iteration(X, P, Aux, Y, rho)
        orc.outer_step(X, st, opts)
        for n in range(4):
            np.testing.assert_allclose(st.P[n], P[n], rtol=1e-9, atol=1e-11)
            np.testing.assert_allclose(st.H[n], Aux[n], rtol=1e-9, atol=1e-11)


def test_planted_nway_noiseless_is_the_model_and_fits():
    dims, F = (6, 5, 4, 3), 2
    X, fac, sigma = ntf_synth.planted_nway(dims, F, seed=6, dtype=np.float64)
    assert sigma == 0.0
    np.testing.assert_allclose(X, orc.reconstruct(fac), rtol=1e-13)
    assert orc.rfe(X, fac) < 1e-14
    H0 = ntf_synth.init_factors(dims, F, 6)
    st = orc.init_state(H0)
    orc.run(X, st, orc.Opts(inner_iters=5), 150)
    assert orc.rfe(X, st.H) < orc.rfe(X, H0) * 0.2
