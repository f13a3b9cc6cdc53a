"""Planted mistakes in the oracle must make its pins fail.

Each case patches one step of the FP64 oracle (on the CPU) with a plausible
error -- a transposed Khatri-Rao operand, a sum instead of a Hadamard product,
a flipped dual update, a dropped penalty term, a wrong projection -- and checks
that at least one pin in ``test_oracle_pins`` rejects it.
"""
import numpy as np
import pytest

from oracle import ntf_oracle as orc
from tests import test_oracle_pins as pins


def _fails(fn, *args):
    try:
        fn(*args)
    except AssertionError:
        return True
    return False


def test_swapped_khatri_rao_operands_caught(monkeypatch):
    good = orc.khatri_rao
    monkeypatch.setattr(orc, "khatri_rao", lambda P, Q: good(Q, P))
    assert _fails(pins.test_unfoldings_match_cp_model_bruteforce)
    assert _fails(pins.test_mttkrp_bruteforce_loops)


def test_gram_sum_instead_of_hadamard_caught(monkeypatch):
    def bad(factors, n):
        return sum(orc.gram(factors[m]) for m in range(3) if m != n)
    monkeypatch.setattr(orc, "gram_hadamard", bad)
    assert _fails(pins.test_gram_hadamard_identity)


def test_flipped_dual_update_caught(monkeypatch):
    monkeypatch.setattr(orc, "dual_update", lambda Hn, V: V - Hn)
    assert _fails(pins.test_inner_invariants_exact_every_iteration)
    assert _fails(pins.test_inner_converges_to_bruteforce_nnls, 3)


def test_abs_instead_of_projection_caught(monkeypatch):
    monkeypatch.setattr(orc, "project_nonneg", lambda V: np.abs(V))
    assert _fails(pins.test_inner_converges_to_bruteforce_nnls, 3)


def test_dropped_penalty_in_solve_caught(monkeypatch):
    good = orc.regularised_ls

    def bad(L, rhs):
        # solve with G only (rho I dropped) -- emulate by rescaling the factor
        return good(L * 1.3, rhs)
    monkeypatch.setattr(orc, "regularised_ls", bad)
    assert _fails(pins.test_inner_converges_to_bruteforce_nnls, 3)
    assert _fails(pins.test_F1_closed_form)


def test_transposed_unfolding_caught(monkeypatch):
    good = orc.unfold

    def bad(X, n):
        X = np.asarray(X, dtype=np.float64)
        if n == 0:
            return X.reshape(X.shape[0], -1)          # (j,k) order instead of (k,j)
        return good(X, n)
    monkeypatch.setattr(orc, "unfold", bad)
    assert _fails(pins.test_unfoldings_match_cp_model_bruteforce)


def test_dual_rescale_in_wrong_direction_caught(monkeypatch):
    monkeypatch.setattr(orc, "rescale_dual", lambda U, rho_old, rho_new: U * (rho_new / rho_old))
    assert _fails(pins.test_paper_form_equals_sweep_form_under_adaptive_rho)
    assert _fails(pins.test_paper_form_equals_sweep_form_with_trace_rho_rescaled)


def test_missing_dual_rescale_caught(monkeypatch):
    monkeypatch.setattr(orc, "rescale_dual", lambda U, rho_old, rho_new: U)
    assert _fails(pins.test_paper_form_equals_sweep_form_under_adaptive_rho)
    assert _fails(pins.test_paper_form_equals_sweep_form_with_trace_rho_rescaled)


def _bad_stop(variant):
    import math

    def conv(infos, dims, F, eps_abs, eps_rel):
        for n, inf in enumerate(infos):
            s = {"sqrt_d_times_F": math.sqrt(dims[n]) * F * eps_abs,
                 "sqrt_F": math.sqrt(F) * eps_abs}.get(variant, math.sqrt(dims[n] * F) * eps_abs)
            big = min(inf["norm_p"], inf["norm_h"]) if variant == "min" else max(inf["norm_p"], inf["norm_h"])
            ny = inf["norm_y"] / 2.0 if variant == "y_over_rho" else inf["norm_y"]
            if inf["prim"] > s + eps_rel * big:
                return False
            if inf["dual"] > s + eps_rel * ny:
                return False
        return True
    return conv


@pytest.mark.parametrize("variant", ["sqrt_d_times_F", "sqrt_F", "min", "y_over_rho"])
def test_wrong_stop_test_caught(monkeypatch, variant):
    monkeypatch.setattr(orc, "converged_paper", _bad_stop(variant))
    assert _fails(pins.test_stop_test_hand_computed_thresholds)
