"""The outer stop test, the penalty guard and the restart rule on the GPU,
through the C ABI, against the FP64 oracle.

* ntf_admm_run with a stop test (Section IV-C: every mode's primal and dual
  residual under sqrt(d_n F) eps_abs + eps_rel (norm)) stops after the same
  outer iteration as the oracle's run(..., stop_eps=...) on the same tensor
  and start, in the paper's variant (one inner iteration, residual balancing,
  Section VI-A) and in the default form (T inner iterations, rho = tr(G)/F);
  the residuals it reports at that iteration are the oracle's.
* An all-zero factor makes the other modes' Gram Hadamard product zero:
  rho = tr(G)/F would be 0 and G + rho I singular, so rho falls back to rho0
  (the guard both sides implement); the run stays finite and follows the oracle.
* n_max = 1 forces the restart rule of Section VI-A on every run.
"""
import math

import numpy as np
import pytest

from oracle import ntf_oracle as orc
from tests.gpu_helpers import problem, rel, to_dev
from paper_1409_2383_amd import _lib

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1409_2383_amd as ntf
    ntf.library_path()
    return torch.device("cuda:0")


def _oracle_run(X, H0, opts, cap, eps, paper):
    st = orc.init_state([np.asarray(h, dtype=np.float64) for h in H0], rho0=opts.rho0, paper=paper)
    last = None
    for _ in range(cap):
        last = orc.outer_step(np.asarray(X, dtype=np.float64), st, opts)
        if orc.converged_paper(last, X.shape, H0[0].shape[1], *eps):
            return st, last, True
    return st, last, False


def _margin(infos, dims, F, eps):
    """Smallest relative distance of any residual from its threshold."""
    m = math.inf
    for n, inf in enumerate(infos):
        s = math.sqrt(dims[n] * F) * eps[0]
        tp = s + eps[1] * max(inf["norm_p"], inf["norm_h"])
        td = s + eps[1] * inf["norm_y"]
        m = min(m, abs(inf["prim"] - tp) / tp, abs(inf["dual"] - td) / td)
    return m


CASES = [
    # dims, F, seed, paper variant, inner iterations, eps
    ((20, 30, 25), 4, 110, True, 1, (1e-4, 1e-4)),
    ((30, 25, 20), 3, 120, True, 1, (1e-4, 1e-4)),
    ((30, 25, 20), 3, 120, False, 3, (1e-6, 1e-6)),
]


@pytest.mark.parametrize("dims,F,seed,paper,T,eps", CASES)
def test_stop_iteration_matches_oracle(dev, dims, F, seed, paper, T, eps):
    import paper_1409_2383_amd as ntf
    pt, H0 = problem(dims, F, seed, True)
    if paper:
        opts = ntf.AdmmOptions(inner_iters=1, precision=ntf.PREC_F64, rho_policy=ntf.RHO_ADAPTIVE,
                               factor_source=1, rescale_dual_on_rho_change=1, paper_init=1,
                               stop_eps_abs=eps[0], stop_eps_rel=eps[1])
        oopts = orc.Opts(inner_iters=1, rho_policy=orc.RHO_ADAPTIVE, factor_source=1,
                         rescale_dual_on_rho_change=True)
    else:
        opts = ntf.AdmmOptions(inner_iters=T, precision=ntf.PREC_F64, stop_eps_abs=eps[0],
                               stop_eps_rel=eps[1])
        oopts = orc.Opts(inner_iters=T)
    cap = 600
    ref, infos, conv = _oracle_run(pt.X, H0, oopts, cap, eps, paper)
    assert conv
    X = torch.from_numpy(pt.X).to(dev)
    H = to_dev(H0, dev)
    s = ntf.NtfAdmm(X, H, opts=opts)
    st = s.run(cap, check_every=1)
    print(f"[stop] {dims} F={F} paper={paper}: GPU stopped after {st['outer']}, oracle after "
          f"{ref.outer}; smallest threshold margin there {_margin(infos, dims, F, eps):.2e}", flush=True)
    assert st["converged"] == 1 and st["status"] == _lib.NTF_OK
    assert st["outer"] == ref.outer
    for n in range(3):
        assert abs(st["prim"][n] - infos[n]["prim"]) <= 1e-6 * infos[n]["prim"], n
        assert abs(st["dual"][n] - infos[n]["dual"]) <= 1e-6 * infos[n]["dual"], n
        assert abs(st["norm_h"][n] - infos[n]["norm_h"]) <= 1e-10 * infos[n]["norm_h"], n
        assert abs(st["norm_p"][n] - infos[n]["norm_p"]) <= 1e-10 * infos[n]["norm_p"], n
        assert abs(st["norm_y"][n] - infos[n]["norm_y"]) <= 1e-8 * infos[n]["norm_y"], n
        assert rel(H[n].cpu().numpy(), ref.H[n]) < 1e-8, n
    s.close()


def test_stop_not_met_runs_to_the_cap(dev):
    import paper_1409_2383_amd as ntf
    dims, F, seed, eps = (20, 30, 25), 4, 110, (1e-4, 1e-4)
    pt, H0 = problem(dims, F, seed, True)
    opts = ntf.AdmmOptions(inner_iters=1, precision=ntf.PREC_F64, rho_policy=ntf.RHO_ADAPTIVE,
                           factor_source=1, rescale_dual_on_rho_change=1, paper_init=1,
                           stop_eps_abs=eps[0], stop_eps_rel=eps[1])
    oopts = orc.Opts(inner_iters=1, rho_policy=orc.RHO_ADAPTIVE, factor_source=1,
                     rescale_dual_on_rho_change=True)
    ref, _, conv = _oracle_run(pt.X, H0, oopts, 5, eps, True)
    assert not conv
    s = ntf.NtfAdmm(torch.from_numpy(pt.X).to(dev), to_dev(H0, dev), opts=opts)
    st = s.run(5, check_every=1)
    assert st["status"] == _lib.NTF_NOT_CONVERGED and st["converged"] == 0 and st["outer"] == 5
    s.close()


@pytest.mark.parametrize("rho0", [1.0, 2.5])
def test_all_zero_factor_falls_back_to_rho0(dev, rho0):
    # B = 0 at the start: mode 1's G = (B^T B) * (C^T C) = 0, so its update
    # runs with rho = rho0 and leaves A unchanged; modes 2 and 3 then proceed.
    import paper_1409_2383_amd as ntf
    dims, F = (21, 17, 19), 4
    pt, H0 = problem(dims, F, 130, True)
    H0[1][:] = 0.0
    opts = ntf.AdmmOptions(inner_iters=3, precision=ntf.PREC_F64, rho0=rho0)
    s = ntf.NtfAdmm(torch.from_numpy(pt.X).to(dev), to_dev(H0, dev), opts=opts)
    st1 = s.step(stats=True)
    assert st1["numeric_error"] == 0
    assert st1["rho"][0] == rho0
    ref = orc.init_state(H0, rho0=rho0)
    orc.outer_step(pt.X, ref, orc.Opts(inner_iters=3, rho0=rho0))
    assert ref.rho[0] == rho0
    assert rel(s.H[0].cpu().numpy(), H0[0]) < 1e-15     # (rho h) / rho
    for _ in range(3):
        s.step()
        orc.outer_step(pt.X, ref, orc.Opts(inner_iters=3, rho0=rho0))
    for n in range(3):
        assert rel(s.H[n].cpu().numpy(), ref.H[n]) < 1e-10, n
    assert abs(s.fit() - orc.rfe(pt.X, ref.H)) < 1e-10
    s.close()


def test_all_factors_zero_stay_zero(dev):
    # Every Gram is zero and every MTTKRP is zero: rho = rho0 everywhere, the
    # factors stay at zero, nothing becomes NaN and the fit is exactly 1.
    import paper_1409_2383_amd as ntf
    dims, F = (12, 13, 14), 3
    pt, H0 = problem(dims, F, 131, False)
    H0 = [np.zeros_like(h) for h in H0]
    s = ntf.NtfAdmm(torch.from_numpy(pt.X).to(dev), to_dev(H0, dev),
                    opts=ntf.AdmmOptions(inner_iters=2, precision=ntf.PREC_F32))
    for _ in range(2):
        st = s.step(stats=True)
        assert st["numeric_error"] == 0 and st["rho"] == [1.0, 1.0, 1.0]
    for n in range(3):
        assert torch.count_nonzero(s.H[n]).item() == 0
        assert torch.count_nonzero(s.U[n]).item() == 0
    assert abs(s.fit() - 1.0) < 1e-12
    s.close()


def test_forced_restarts_with_n_max_1(dev):
    # n_max = 1: no run meets the stop test after one iteration, so every run
    # is abandoned and restarted from the next seed's start, and the
    # iterations of all runs count.
    from paper_1409_2383_amd import paper_mode
    import ntf_synth
    dims, F, seed = (30, 25, 20), 3, 120
    pt = ntf_synth.planted(dims, F, seed, snr_db=20.0, dtype=np.float64)
    X = torch.from_numpy(pt.X).to(dev)
    r = paper_mode.solve_with_restarts(X, F, seed, n_max=1, max_restarts=3)
    assert not r["converged"] and r["restarts"] == 3 and r["total_iters"] == 4
    # with room to converge the first run stops where the oracle's does
    r = paper_mode.solve_with_restarts(X, F, seed, n_max=400, max_restarts=3)
    H0 = ntf_synth.init_factors(dims, F, seed, dtype=np.float64)
    ref, _, conv = _oracle_run(pt.X, H0, orc.Opts(inner_iters=1, rho_policy=orc.RHO_ADAPTIVE,
                                                  factor_source=1, rescale_dual_on_rho_change=True),
                               400, (1e-4, 1e-4), True)
    assert conv and r["converged"] and r["restarts"] == 0
    assert r["iters"] == ref.outer
