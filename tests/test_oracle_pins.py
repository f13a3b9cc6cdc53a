"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these tests needs a GPU.  Each one checks the oracle against something
other than itself: brute-force loops, closed forms of the planted data model,
exhaustive NNLS, exact invariants of the projection/dual update, the paper's
own form of the iteration, the block-partitioned form of Appendix B, and the
mean RFE values printed in Tables 1 and 2.
"""
import json
import math
import os

import numpy as np
import pytest

import ntf_synth
from oracle import ntf_oracle as orc

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rand_factors(dims, F, seed):
    rng = np.random.default_rng(seed)
    return [rng.random((d, F)) for d in dims]


# --------------------------------------------------------------------------- Section II

def test_khatri_rao_entries():
    rng = np.random.default_rng(1)
    P, Q = rng.random((3, 4)), rng.random((5, 4))
    KR = orc.khatri_rao(P, Q)
    for p in range(3):
        for q in range(5):
            for f in range(4):
                assert KR[p * 5 + q, f] == P[p, f] * Q[q, f]


def test_unfoldings_match_cp_model_bruteforce():
    # eq. f_X_matr: W^(1) = A (C.B)^T, W^(2) = B (C.A)^T, W^(3) = C (B.A)^T,
    # against a CP tensor built with explicit index loops.
    I, J, K, F = 3, 4, 5, 2
    A, B, C = _rand_factors((I, J, K), F, 2)
    W = np.zeros((I, J, K))
    for i in range(I):
        for j in range(J):
            for k in range(K):
                W[i, j, k] = sum(A[i, f] * B[j, f] * C[k, f] for f in range(F))
    np.testing.assert_allclose(orc.reconstruct([A, B, C]), W, rtol=1e-14)
    for n, Hn in enumerate((A, B, C)):
        np.testing.assert_allclose(orc.unfold(W, n), Hn @ orc.kr_for_mode([A, B, C], n).T, rtol=1e-13)


def test_mttkrp_bruteforce_loops():
    I, J, K, F = 4, 3, 5, 3
    rng = np.random.default_rng(3)
    X = rng.standard_normal((I, J, K))
    Hs = _rand_factors((I, J, K), F, 4)
    dims = (I, J, K)
    for n in range(3):
        Wb = np.zeros((dims[n], F))
        for i in range(I):
            for j in range(J):
                for k in range(K):
                    idx = (i, j, k)
                    for f in range(F):
                        prod = X[i, j, k]
                        for m in range(3):
                            if m != n:
                                prod *= Hs[m][idx[m], f]
                        Wb[idx[n], f] += prod
        np.testing.assert_allclose(orc.mttkrp(X, Hs, n), Wb, rtol=1e-12, atol=1e-13)


def test_mttkrp_planted_closed_form():
    # Noiseless planted X = [A0,B0,C0]:  W_1 = A0 ((B0^T H2) * (C0^T H3)) and
    # cyclically; derived from eq. f_X_matr and the Gram identity of IV-A.
    dims, F = (20, 30, 25), 4
    pt = ntf_synth.planted(dims, F, seed=11, dtype=np.float64)
    Hs = _rand_factors(dims, 6, 12)   # a different rank for the probes
    P0 = [pt.A0, pt.B0, pt.C0]
    for n in range(3):
        others = [m for m in range(3) if m != n]
        closed = P0[n] @ ((P0[others[0]].T @ Hs[others[0]]) * (P0[others[1]].T @ Hs[others[1]]))
        np.testing.assert_allclose(orc.mttkrp(pt.X, Hs, n), closed, rtol=1e-12)


def test_rfe_expanded_equals_the_definition():
    # The expansion ||X||^2 - 2<X,M> + ||M||^2 against the residual formed
    # entry by entry from the reconstructed model, on a noisy planted tensor
    # and on factors far from it.
    dims, F = (9, 7, 11), 4
    pt = ntf_synth.planted(dims, F, seed=31, snr_db=20.0, dtype=np.float64)
    for fac in ([pt.A0, pt.B0, pt.C0], _rand_factors(dims, F, 32)):
        M = np.zeros(dims)
        for i in range(dims[0]):
            for j in range(dims[1]):
                for k in range(dims[2]):
                    M[i, j, k] = sum(fac[0][i, f] * fac[1][j, f] * fac[2][k, f] for f in range(F))
        direct = math.sqrt(np.sum((pt.X - M) ** 2) / np.sum(pt.X ** 2))
        assert abs(orc.rfe_expanded(pt.X, fac) - direct) < 1e-12 * max(direct, 1e-3)
        assert abs(orc.rfe(pt.X, fac) - direct) < 1e-13 * direct


def test_gram_hadamard_identity():
    Hs = _rand_factors((6, 7, 8), 5, 5)
    for n in range(3):
        KR = orc.kr_for_mode(Hs, n)
        np.testing.assert_allclose(orc.gram_hadamard(Hs, n), KR.T @ KR, rtol=1e-13)


def test_rho_trace_and_guard():
    G = np.diag([1.0, 2.0, 3.0, 6.0])
    assert orc.rho_trace(G) == 3.0
    assert orc.rho_trace(np.zeros((3, 3)), rho0=1.0) == 1.0
    assert orc.rho_trace(np.full((2, 2), np.nan), rho0=2.5) == 2.5


# --------------------------------------------------------------------------- inner sweep

def _spd(F, seed, cond=None):
    rng = np.random.default_rng(seed)
    M = rng.random((F + 3, F))
    return M.T @ M


def test_inner_invariants_exact_every_iteration():
    # H >= 0, U >= 0 and H * U == 0 exactly after every iteration (either h or
    # u is exactly zero because u = h - v with h = max(0, v)).
    F = 7
    G = _spd(F, 21)
    rng = np.random.default_rng(22)
    W = rng.standard_normal((50, F)) * 3
    H = rng.random((50, F))
    U = np.zeros((50, F))
    rho = orc.rho_trace(G)
    for _ in range(25):
        H, U, Ht, _ = orc.inner_sweep(W, H, U, G, rho, 1)
        assert np.all(H >= 0) and np.all(U >= 0)
        assert np.all(H * U == 0.0)
        assert np.all(np.isfinite(U))


@pytest.mark.parametrize("F", [1, 3, 6])
def test_inner_converges_to_bruteforce_nnls(F):
    G = _spd(F, 30 + F)
    rng = np.random.default_rng(31)
    W = rng.standard_normal((12, F)) * 2
    H, U, _, _ = orc.inner_sweep(W, np.zeros_like(W), np.zeros_like(W), G, orc.rho_trace(G), 4000)
    for i in range(W.shape[0]):
        np.testing.assert_allclose(H[i], orc.nnls_bruteforce(G, W[i]), atol=1e-9)
    # stationarity of eq. KKT_NTF with Y = -rho U:  rho U = H G - W
    rho = orc.rho_trace(G)
    np.testing.assert_allclose(rho * U, H @ G - W, atol=1e-8)


def test_inner_converges_to_lawson_hanson_larger_F():
    F = 12
    G = _spd(F, 40)
    rng = np.random.default_rng(41)
    W = rng.standard_normal((20, F))
    H, _, _, _ = orc.inner_sweep(W, np.zeros_like(W), np.zeros_like(W), G, orc.rho_trace(G), 20000)
    np.testing.assert_allclose(H, orc.nnls_rows(G, W), atol=1e-8)
    assert np.max(orc.kkt_violation(G, W, H)) < 1e-8


def test_F1_closed_form():
    # F = 1: the per-row NNLS is h* = max(0, w/g).
    g = 2.5
    w = np.array([[3.0], [-1.0], [0.5], [0.0]])
    H, _, _, _ = orc.inner_sweep(w, np.zeros_like(w), np.zeros_like(w), np.array([[g]]), 1.7, 3000)
    np.testing.assert_allclose(H[:, 0], np.maximum(0.0, w[:, 0] / g), atol=1e-12)


def test_bruteforce_nnls_is_the_minimiser():
    # The exhaustive solver must beat random feasible points (sanity of the pin itself).
    F = 5
    G = _spd(F, 50)
    w = np.random.default_rng(51).standard_normal(F)
    h = orc.nnls_bruteforce(G, w)
    val = 0.5 * h @ G @ h - w @ h
    rng = np.random.default_rng(52)
    for _ in range(2000):
        z = np.maximum(0.0, h + 0.1 * rng.standard_normal(F))
        assert 0.5 * z @ G @ z - w @ z >= val - 1e-12


def test_early_stop_rows():
    F = 6
    G = _spd(F, 60)
    rng = np.random.default_rng(61)
    W = rng.standard_normal((30, F))
    z = np.zeros_like(W)
    rho = orc.rho_trace(G)
    Hf, _, _, inf_f = orc.inner_sweep(W, z, z, G, rho, 50)
    He, _, _, inf_e = orc.inner_sweep(W, z, z, G, rho, 50, eps_abs=1e-30, eps_rel=1e-30)
    np.testing.assert_array_equal(Hf, He)            # never met -> same as fixed T
    assert np.all(inf_e["iters"] == 50)
    H3, _, _, inf3 = orc.inner_sweep(W, z, z, G, rho, 5000, eps_abs=1e-9, eps_rel=1e-9)
    assert np.all(inf3["iters"] < 5000) and np.all(inf3["iters"] >= 1)
    assert np.max(orc.kkt_violation(G, W, H3)) < 1e-6


# --------------------------------------------------------------------------- outer loop

def test_exact_block_coordinate_descent_is_monotone():
    # Inner iterations run to convergence -> each mode update is an exact NNLS
    # block update (NALS), so f never increases.
    dims, F = (9, 10, 11), 3
    pt = ntf_synth.planted(dims, F, seed=70, sigma2=1e-2, dtype=np.float64)
    st = orc.init_state(ntf_synth.init_factors(dims, F, 70))
    opts = orc.Opts(inner_iters=3000, eps_abs=1e-13, eps_rel=1e-13)
    f_prev = orc.objective(pt.X, st.H)
    for _ in range(8):
        orc.outer_step(pt.X, st, opts)
        f = orc.objective(pt.X, st.H)
        assert f <= f_prev * (1 + 1e-12) + 1e-14
        f_prev = f


def test_planted_noiseless_recovery():
    # Noiseless exact-rank data: no error floor (Section VI-C).  Restarts from
    # another random point are allowed, as in the paper's restart strategy.
    dims, F = (10, 12, 14), 3
    pt = ntf_synth.planted(dims, F, seed=80, dtype=np.float64)
    best = 1.0
    for restart in range(4):
        st = orc.init_state(ntf_synth.init_factors(dims, F, 80 + 17 * restart))
        orc.run(pt.X, st, orc.Opts(inner_iters=5), 1500)
        best = min(best, orc.rfe(pt.X, st.H))
        if best < 1e-6:
            break
    assert best < 1e-6


def test_kkt_at_convergence():
    # eq. KKT_NTF at a converged point, with Y = -rho U.
    dims, F = (8, 9, 10), 2
    pt = ntf_synth.planted(dims, F, seed=90, sigma2=1e-3, dtype=np.float64)
    st = orc.init_state(ntf_synth.init_factors(dims, F, 90))
    orc.run(pt.X, st, orc.Opts(inner_iters=5), 3000)
    scale = np.linalg.norm(pt.X)
    for n in range(3):
        KR = orc.kr_for_mode(st.H, n)
        Y = -st.rho[n] * st.U[n]
        grad = (orc.unfold(pt.X, n) - st.H[n] @ KR.T) @ KR - Y
        assert np.linalg.norm(grad) < 1e-6 * scale ** 2
        assert np.linalg.norm(st.H[n] - st.P[n]) < 1e-8 * np.linalg.norm(st.H[n])
        assert np.all(Y <= 0) and np.all(Y * st.H[n] == 0)


def test_paper_form_equals_inner_sweep_form():
    # Eq. ADMoM_NTF / ADMM_NTF_ALS_C as printed (explicit Y, explicit KR^T KR,
    # general solve) equals the sweep form with T = 1, fixed rho, the primal
    # fed forward and the paper's initialisation, under H = A-tilde, U = -Y/rho.
    dims, F = (7, 8, 9), 3
    pt = ntf_synth.planted(dims, F, seed=100, sigma2=1e-2, dtype=np.float64)
    H0 = ntf_synth.init_factors(dims, F, 100)
    rho = [1.3, 0.7, 2.1]
    P = [h.copy() for h in H0]
    Aux = [np.zeros_like(h) for h in H0]
    Y = [np.zeros_like(h) for h in H0]
    st = orc.init_state(H0, paper=True)
    st.rho = list(rho)
    opts = orc.Opts(inner_iters=1, rho_policy=orc.RHO_FIXED, factor_source=1)
    for _ in range(6):
        P, Aux, Y = orc.paper_admom_iteration(pt.X, P, Aux, Y, rho)
        orc.outer_step(pt.X, st, opts)
        for n in range(3):
            np.testing.assert_allclose(st.P[n], P[n], rtol=1e-9, atol=1e-11)
            np.testing.assert_allclose(st.H[n], Aux[n], rtol=1e-9, atol=1e-11)
            np.testing.assert_allclose(-rho[n] * st.U[n], Y[n], rtol=1e-9, atol=1e-11)


def _paper_form_along(X, H0, rho_seq):
    """Eq. ADMoM_NTF / ADMM_NTF_ALS_C as printed, explicit unscaled Y, with
    the penalty of every mode taken from rho_seq[k] at iteration k (Y is the
    state and is never rescaled: Section IV-D changes rho only)."""
    P = [h.copy() for h in H0]
    Aux = [np.zeros_like(h) for h in H0]
    Y = [np.zeros_like(h) for h in H0]
    out = []
    for rho in rho_seq:
        P, Aux, Y = orc.paper_admom_iteration(X, P, Aux, Y, rho)
        out.append(([p.copy() for p in P], [a.copy() for a in Aux], [y.copy() for y in Y]))
    return out


def test_paper_form_equals_sweep_form_under_adaptive_rho():
    # Residual balancing (eq. varying_penalty_rule) changes each mode's rho
    # between iterations; the sweep form carries U = -Y/rho and must rescale
    # it on every change.  The paper form keeps Y itself, so both must give
    # the same A, A-tilde and Y along the whole run.  A rescale in the wrong
    # direction (rho_new/rho_old) or a missing one diverges at the first change.
    dims, F = (7, 8, 9), 3
    pt = ntf_synth.planted(dims, F, seed=101, sigma2=1e-2, dtype=np.float64)
    H0 = ntf_synth.init_factors(dims, F, 101)
    st = orc.init_state(H0, rho0=1.0, paper=True)
    opts = orc.Opts(inner_iters=1, rho_policy=orc.RHO_ADAPTIVE, rho0=1.0, mu=8.0, tau_incr=4.0,
                    tau_decr=2.0, factor_source=1)
    rho_used, snaps = [], []
    for _ in range(25):
        rho_used.append(list(st.rho))                 # the penalties this iteration runs with
        orc.outer_step(pt.X, st, opts)
        assert any(np.any(u != 0) for u in st.U)       # the rescale has something to act on
        snaps.append(([p.copy() for p in st.P], [h.copy() for h in st.H],
                      [-st.rho[n] * st.U[n] for n in range(3)]))     # U already on the new rho
    seq = np.array(rho_used)
    assert np.any(seq[1:] > seq[:-1]) and np.any(seq[1:] < seq[:-1]), seq   # both directions taken
    ref = _paper_form_along(pt.X, H0, rho_used)
    for k, ((P, Aux, Y), (Ps, Hs, Ys)) in enumerate(zip(ref, snaps)):
        for n in range(3):
            np.testing.assert_allclose(Ps[n], P[n], rtol=1e-8, atol=1e-10, err_msg=f"A, iter {k}")
            np.testing.assert_allclose(Hs[n], Aux[n], rtol=1e-8, atol=1e-10, err_msg=f"A~, iter {k}")
            np.testing.assert_allclose(Ys[n], Y[n], rtol=1e-8, atol=1e-10, err_msg=f"Y, iter {k}")


def test_paper_form_equals_sweep_form_with_trace_rho_rescaled():
    # rho = tr(G)/F changes at every mode update; with the dual rescale on,
    # the sweep form is the paper's form run with that penalty sequence.
    # (noise at sigma2 = 0.5 puts negative entries in the LS solutions, so U
    # is non-zero and the rescale matters; with little noise U stays zero)
    dims, F = (6, 9, 8), 3
    pt = ntf_synth.planted(dims, F, seed=102, sigma2=0.5, dtype=np.float64)
    H0 = ntf_synth.init_factors(dims, F, 102)
    st = orc.init_state(H0, rho0=1.0, paper=True)
    opts = orc.Opts(inner_iters=1, rho_policy=orc.RHO_TRACE, factor_source=1,
                    rescale_dual_on_rho_change=True)
    rho_used, snaps = [], []
    for _ in range(12):
        orc.outer_step(pt.X, st, opts)
        assert any(np.any(u != 0) for u in st.U)       # the rescale has something to act on
        rho_used.append(list(st.rho))
        snaps.append(([p.copy() for p in st.P], [h.copy() for h in st.H],
                      [-st.rho[n] * st.U[n] for n in range(3)]))
    seq = np.array(rho_used)
    assert np.all(np.abs(seq[1:] / seq[:-1] - 1.0) > 1e-6)        # every update changes rho
    ref = _paper_form_along(pt.X, H0, rho_used)
    for k, ((P, Aux, Y), (Ps, Hs, Ys)) in enumerate(zip(ref, snaps)):
        for n in range(3):
            np.testing.assert_allclose(Ps[n], P[n], rtol=1e-8, atol=1e-10, err_msg=f"A, iter {k}")
            np.testing.assert_allclose(Hs[n], Aux[n], rtol=1e-8, atol=1e-10, err_msg=f"A~, iter {k}")
            np.testing.assert_allclose(Ys[n], Y[n], rtol=1e-8, atol=1e-10, err_msg=f"Y, iter {k}")


def _stop_infos():
    # Hand-set residuals for dims (4, 9, 16), F = 4: sqrt(d F) = 4, 6, 8.
    # With eps_abs = 0.01, eps_rel = 0.1 the Section IV-C thresholds are
    #   mode 1: primal 0.04 + 0.1 max(3, 5) = 0.54,  dual 0.04 + 0.1 * 2 = 0.24
    #   mode 2: primal 0.06 + 0.1 max(7, 1) = 0.76,  dual 0.06 + 0.1 * 4 = 0.46
    #   mode 3: primal 0.08 + 0.1 max(2, 2) = 0.28,  dual 0.08 + 0.1 * 1 = 0.18
    return [
        {"prim": 0.535, "dual": 0.235, "norm_p": 3.0, "norm_h": 5.0, "norm_y": 2.0},
        {"prim": 0.755, "dual": 0.455, "norm_p": 7.0, "norm_h": 1.0, "norm_y": 4.0},
        {"prim": 0.275, "dual": 0.175, "norm_p": 2.0, "norm_h": 2.0, "norm_y": 1.0},
    ]


def test_stop_test_hand_computed_thresholds():
    dims, F, ea, er = (4, 9, 16), 4, 0.01, 0.1
    assert orc.converged_paper(_stop_infos(), dims, F, ea, er)
    # each of the six conditions pushed just past its threshold alone stops nothing
    for n, key, val in [(0, "prim", 0.545), (0, "dual", 0.245), (1, "prim", 0.765),
                        (1, "dual", 0.465), (2, "prim", 0.285), (2, "dual", 0.185)]:
        infos = _stop_infos()
        infos[n][key] = val
        assert not orc.converged_paper(infos, dims, F, ea, er), (n, key)
    # the relative part uses the larger of ||A|| and ||A-tilde||, whichever it is
    infos = _stop_infos()
    infos[0]["norm_p"], infos[0]["norm_h"] = 5.0, 3.0
    assert orc.converged_paper(infos, dims, F, ea, er)
    # the absolute part alone: with eps_rel = 0 the thresholds are sqrt(d F) eps_abs
    infos = [{"prim": 0.039, "dual": 0.039, "norm_p": 1e9, "norm_h": 1e9, "norm_y": 1e9},
             {"prim": 0.059, "dual": 0.059, "norm_p": 1e9, "norm_h": 1e9, "norm_y": 1e9},
             {"prim": 0.079, "dual": 0.079, "norm_p": 1e9, "norm_h": 1e9, "norm_y": 1e9}]
    assert orc.converged_paper(infos, dims, F, 0.01, 0.0)
    infos[2]["dual"] = 0.081
    assert not orc.converged_paper(infos, dims, F, 0.01, 0.0)


def test_run_stops_at_the_first_iteration_meeting_the_test():
    # run(..., stop_eps) ends after the first outer iteration whose residuals
    # pass the Section IV-C test and not before: replaying the same iterations
    # one at a time finds that iteration by the test on each iteration's infos.
    dims, F = (12, 10, 9), 3
    pt = ntf_synth.planted(dims, F, seed=103, sigma2=1e-2, dtype=np.float64)
    H0 = ntf_synth.init_factors(dims, F, 103)
    opts = orc.Opts(inner_iters=1, rho_policy=orc.RHO_ADAPTIVE, factor_source=1)
    eps = (1e-3, 1e-3)
    st = orc.run(pt.X, orc.init_state(H0, paper=True), opts, 2000, stop_eps=eps)
    assert st.outer < 2000
    st2 = orc.init_state(H0, paper=True)
    first = None
    for k in range(st.outer):
        infos = orc.outer_step(pt.X, st2, opts)
        if first is None and orc.converged_paper(infos, dims, F, *eps):
            first = k + 1
    assert first == st.outer
    for n in range(3):
        np.testing.assert_array_equal(st.H[n], st2.H[n])


@pytest.mark.parametrize("blocks", [2, 3])
def test_partitioned_update_equals_centralized(blocks):
    # Appendix B: the block-partitioned update evolves exactly like the centralized one.
    dims, F = (9, 11, 7), 3
    pt = ntf_synth.planted(dims, F, seed=110, sigma2=1e-2, dtype=np.float64)
    Hs = ntf_synth.init_factors(dims, F, 110)
    rng = np.random.default_rng(111)
    for n in range(3):
        U = rng.random(Hs[n].shape) * 0.1
        W = orc.mttkrp(pt.X, Hs, n)
        G = orc.gram_hadamard(Hs, n)
        rho = orc.rho_trace(G)
        Hc, Uc, _, _ = orc.inner_sweep(W, Hs[n], U, G, rho, 3)
        Hp, Up = orc.partitioned_mode_update(pt.X, Hs, Hs[n], U, n, rho, 3, blocks)
        np.testing.assert_allclose(Hp, Hc, rtol=1e-11, atol=1e-12)
        np.testing.assert_allclose(Up, Uc, rtol=1e-11, atol=1e-12)


def test_adaptive_rho_rule():
    # eq. varying_penalty_rule
    o = orc.Opts(mu=8, tau_incr=4, tau_decr=2)
    assert orc._adapt_rho(1.0, 9.0, 1.0, o) == 4.0
    assert orc._adapt_rho(1.0, 1.0, 9.0, o) == 0.5
    assert orc._adapt_rho(1.0, 1.0, 1.0, o) == 1.0


# --------------------------------------------------------------------------- noise floor

def _rfe_floor(dims, F, sigma2=None, snr_db=None, factor_ms=None):
    I, J, K = dims
    n = I * J * K
    dof = (I + J + K - 2) * F
    if snr_db is not None:
        base = math.sqrt(1.0 / (1.0 + 10 ** (snr_db / 10)))
    else:
        ex2 = F * F / 64.0 + F * (1 / 27.0 - 1 / 64.0)    # E[x0^2] for iid U[0,1] factors
        base = math.sqrt(sigma2 / (ex2 + sigma2))
    return base * math.sqrt(1.0 - dof / n)


def test_noise_floor_formula_reproduces_tables():
    # The closed-form noise floor (derived for U[0,1] planted factors) against
    # every mean RFE printed in Tables 1 and 2.
    with open(os.path.join(GOLDEN, "table1_mean_rfe.json")) as fh:
        rows = json.load(fh)["rows"]
    for r in rows:
        pred = _rfe_floor(r["dims"], r["F"], sigma2=r["sigma2"])
        assert abs(pred - r["mean_rfe"]) <= 0.01 * r["mean_rfe"] + 5e-5, r


def test_oracle_reaches_noise_floor_40cubed():
    # 40^3, F = 5, 20 dB (the small FP64 workload): the converged RFE sits on
    # the noise floor of the data model (statistical, +-3%).
    dims, F = (40, 40, 40), 5
    pt = ntf_synth.planted(dims, F, seed=ntf_synth.config_seed(1), snr_db=20.0, clip=True,
                           dtype=np.float64)
    st = orc.init_state(ntf_synth.init_factors(dims, F, ntf_synth.config_seed(1)))
    orc.run(pt.X, st, orc.Opts(inner_iters=5), 400)
    r = orc.rfe(pt.X, st.H)
    assert abs(r - _rfe_floor(dims, F, snr_db=20.0)) < 0.03 * r


# --------------------------------------------------------------------------- mixed precision input

def test_slab_quantisation_against_torch_bfloat16():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(120)
    X = (rng.random((5, 6, 7)) * np.array([1e-3, 1.0, 7.0, 300.0, 0.0])[:, None, None]).astype(np.float32)
    Xq, s = orc.quantize_slabs_bf16(X)
    for i in range(5):
        m = np.max(np.abs(X[i]))
        if m == 0:
            assert s[i] == 1.0
            continue
        assert 1.0 <= m / s[i] < 2.0
        assert math.log2(s[i]) == int(math.log2(s[i]))
        ref = torch.from_numpy(X[i] / np.float32(s[i])).to(torch.bfloat16).to(torch.float64).numpy()
        np.testing.assert_array_equal(Xq[i], ref)


def test_mixed_mttkrp_reduces_to_exact_on_bfloat16_values():
    # With every operand that the recipe rounds already a bfloat16 value (X a
    # small-integer tensor, the rounded factors multiples of 1/8 in [0, 2]),
    # the mixed-precision MTTKRP is the exact one.  The factor that the
    # factored mode-3 form keeps in float32 (A) is left arbitrary: rounding it
    # by mistake would move the result by ~1e-3.
    rng = np.random.default_rng(121)
    I, J, K, F = 6, 5, 7, 3
    X = rng.integers(0, 9, (I, J, K)).astype(np.float32)
    A = rng.random((I, F)).astype(np.float32).astype(np.float64)
    B = (rng.integers(0, 17, (J, F)) / 8.0)
    C = (rng.integers(0, 17, (K, F)) / 8.0)
    fac = [A, B, C]
    X64 = X.astype(np.float64)
    for n in (0, 1):
        for m3 in ("kr", "factored", "split"):
            np.testing.assert_allclose(orc.mttkrp_mixed(X, fac, n, mode3=m3), orc.mttkrp(X64, fac, n),
                                       rtol=1e-14, atol=0)
    for m3 in ("factored", "split"):   # (lo is zero when B is a bfloat16 value)
        np.testing.assert_allclose(orc.mttkrp_mixed(X, fac, 2, mode3=m3), orc.mttkrp(X64, fac, 2),
                                   rtol=1e-14, atol=0)
    # the Khatri-Rao form rounds the products A[i,f] B[j,f]: not exact here
    kr = orc.mttkrp_mixed(X, fac, 2, mode3="kr")
    assert np.max(np.abs(kr - orc.mttkrp(X64, fac, 2))) > 1e-6 * np.max(np.abs(kr))


def test_mixed_mttkrp_factored_brute_force():
    # the factored mode-3 rounding written out element by element
    rng = np.random.default_rng(122)
    I, J, K, F = 3, 4, 5, 2
    X = (rng.random((I, J, K)) * 3.0).astype(np.float32)
    A, B, C = (rng.random((d, F)) for d in (I, J, K))
    Xq, s = orc.quantize_slabs_bf16(X)
    Bb = orc._round_bf16(B.astype(np.float32)).astype(np.float64)
    A32 = A.astype(np.float32).astype(np.float64)
    W = np.zeros((K, F))
    for k in range(K):
        for f in range(F):
            tot = 0.0
            for i in range(I):
                inner = sum(Xq[i, j, k] * Bb[j, f] for j in range(J))
                tot += s[i] * A32[i, f] * inner
            W[k, f] = tot
    np.testing.assert_allclose(orc.mttkrp_mixed(X, [A, B, C], 2, mode3="factored"), W, rtol=1e-12)


def test_mixed_mttkrp_split_brute_force():
    # the split factored mode-3 rounding written out element by element: B as
    # a bfloat16 pair (hi, lo) whose sum differs from B by at most 2^-16 |B|
    rng = np.random.default_rng(123)
    I, J, K, F = 3, 4, 5, 2
    X = (rng.random((I, J, K)) * 3.0).astype(np.float32)
    A, B, C = (rng.random((d, F)) for d in (I, J, K))
    Xq, s = orc.quantize_slabs_bf16(X)
    B32 = B.astype(np.float32)
    W = np.zeros((K, F))
    for k in range(K):
        for f in range(F):
            tot = 0.0
            for i in range(I):
                inner = 0.0
                for j in range(J):
                    b = float(B32[j, f])
                    hi = float(orc._round_bf16(np.float32(b)))
                    lo = float(orc._round_bf16(np.float32(b - hi)))
                    assert abs((hi + lo) - b) <= 2.0 ** -16 * abs(b)
                    inner += float(Xq[i, j, k]) * (hi + lo)
                tot += float(s[i]) * float(np.float32(A[i, f])) * inner
            W[k, f] = tot
    np.testing.assert_allclose(orc.mttkrp_mixed(X, [A, B, C], 2, mode3="split"), W, rtol=1e-12)


def test_mixed_mttkrp_split_is_closer_to_exact_than_factored():
    # the same quantised X: only the rounding of B differs, and the split form
    # carries B to ~2^-16, so its error against the MTTKRP of the quantised
    # tensor with float32 factors is far below the factored form's
    rng = np.random.default_rng(124)
    I, J, K, F = 20, 30, 25, 4
    X = (rng.random((I, J, K)) * 2.0).astype(np.float32)
    fac = [rng.random((d, F)).astype(np.float32) for d in (I, J, K)]
    Xq, s = orc.quantize_slabs_bf16(X)
    ref = orc.mttkrp(Xq * s[:, None, None], [f.astype(np.float64) for f in fac], 2)
    e_f = np.abs(orc.mttkrp_mixed(X, fac, 2, mode3="factored") - ref).max()
    e_s = np.abs(orc.mttkrp_mixed(X, fac, 2, mode3="split") - ref).max()
    assert e_s < e_f / 64, (e_s, e_f)


def test_row_restricted_mttkrps_equal_the_full_ones():
    # the selected-row forms used by the full-size checks return exactly the
    # rows of the whole-tensor functions
    rng = np.random.default_rng(300)
    dims, F = (7, 9, 8), 4
    X = rng.standard_normal(dims).astype(np.float32)
    fac = [rng.random((d, F)).astype(np.float32) for d in dims]
    for n in range(3):
        rows = np.array(sorted(rng.choice(dims[n], 3, replace=False)))
        np.testing.assert_allclose(orc.mttkrp_rows(X, fac, n, rows), orc.mttkrp(X, fac, n)[rows],
                                   rtol=1e-12)
        for m3 in ("kr", "factored", "split"):
            np.testing.assert_allclose(orc.mttkrp_mixed_rows(X, fac, n, rows, m3),
                                       orc.mttkrp_mixed(X, fac, n, m3)[rows], rtol=1e-12, atol=1e-12)
    X4 = rng.standard_normal((4, 5, 3, 6))
    fac4 = [rng.random((d, 2)) for d in X4.shape]
    for n in range(4):
        np.testing.assert_allclose(orc.mttkrp_rows(X4, fac4, n, [0, 2]), orc.mttkrp(X4, fac4, n)[[0, 2]],
                                   rtol=1e-12)
    idx = np.stack(np.unravel_index(rng.choice(7 * 9 * 8, 120, replace=False), dims), 1).astype(np.int32)
    T = orc.SparseTensor(idx=idx, val=rng.standard_normal(120), dims=dims)
    for n in range(3):
        np.testing.assert_allclose(orc.mttkrp_sparse_rows(T, fac, n, [1, 3]),
                                   orc.mttkrp_sparse(T, fac, n)[[1, 3]], rtol=1e-12, atol=1e-14)
