"""GPU parity of the batched solver (many problems of uneven shapes, one
persistent kernel per outer iteration) against the oracle, through the C ABI.

Expected values come from the oracle with the batched path's operand rounding
(mttkrp_mixed, mode 3 in split factored form): the same bfloat16 operands, exact
accumulation.  Tolerances (relative Frobenius norm):
  MTTKRP, every mode of every problem: 1e-5 (FP32 MFMA accumulation of at
    most a few thousand terms per slab, FP64 across slabs); against the exact
    MTTKRP: 2e-2 (the bfloat16 rounding itself).
  One outer iteration from a common state: at most 3x the distance between
    the oracle and the same recipe evaluated with float32 library arithmetic
    (floors 1e-5 on H, 1e-4 on U).  The W and Gram differences of float32
    accumulation pass through T regularised least-squares solves and three
    Gauss-Seidel mode updates, which amplify them by 1e2 - 1e3 on ill-posed
    shapes (e.g. I = 3 < F); the gate scales with that sensitivity.
  Fit after 15 outer iterations: at most 3x the larger of the drift of the
    float32 recipe reference from the oracle over the same iterations and the
    oracle's own spread when its initial factors are perturbed by one float32
    rounding (+-2^-24 relative): these short runs on small, unconverged
    problems amplify such a perturbation to 1e-4 in the fit, so a single
    float32 replay can land closer to the oracle than another float32
    summation order does.
"""
import numpy as np
import pytest

from oracle import ntf_oracle as orc
from tests.gpu_helpers import problem, rel

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

# uneven shapes and ranks: one slab, thin modes, F = 1, F = 64 (four 16-column
# tiles), F > 32 (64 inner lanes), contraction lengths not multiples of 32 or 64.
# Every pair of modes has d_a * d_b >= F, so no Gram Hadamard product is
# singular (with I * J < F the mode-3 update amplifies rounding by ~1e4 and
# no finite-precision implementation can track the oracle).
BATCH = [((40, 50, 30), 8), ((1, 1, 1), 1), ((5, 70, 33), 17), ((40, 9, 130), 5),
         ((3, 200, 100), 33), ((17, 64, 64), 64), ((2, 9, 300), 12), ((60, 31, 97), 20)]


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1409_2383_amd as ntf
    ntf.library_path()
    return torch.device("cuda:0")


def _batch(dev, spec, T=10, seed0=700, **kw):
    import paper_1409_2383_amd as ntf
    pts, H0s, Xs, Hs = [], [], [], []
    for t, (dims, F) in enumerate(spec):
        pt, H0 = problem(dims, F, seed0 + t, False)
        pts.append(pt)
        H0s.append(H0)
        Xs.append(torch.from_numpy(np.ascontiguousarray(pt.X)).to(dev))
        Hs.append([torch.from_numpy(h.copy()).to(dev) for h in H0])
    opts = ntf.AdmmOptions(inner_iters=T, precision=ntf.PREC_BF16_MIXED, **kw)
    print(f"[batch] {len(spec)} problems, T={T}", flush=True)
    return ntf.NtfBatch(Xs, Hs, opts=opts), pts, H0s, Hs


def _check_mttkrp(b, pts, H0s, tag):
    worst = 0.0
    for p, (pt, H0) in enumerate(zip(pts, H0s)):
        for n in range(3):
            W = b.mttkrp(p, n).cpu().numpy()
            ref = orc.mttkrp_mixed(pt.X, H0, n, mode3="split")
            e = rel(W, ref)
            worst = max(worst, e)
            assert e < 1e-5, (tag, p, n, e)
            assert rel(W, orc.mttkrp(pt.X.astype(np.float64), H0, n)) < 2e-2, (tag, p, n)
    print(f"[batch] mttkrp {tag}: worst {worst:.2e}", flush=True)


def test_batch_mttkrp_all_modes(dev):
    b, pts, H0s, _ = _batch(dev, BATCH)
    _check_mttkrp(b, pts, H0s, "default tiles")
    # one slab per item (many items and pass-3 partials), single-row tiles
    b.set_tiles([{"kind": k, "ft": ft, "qbucket": q, "mt": 1, "item_elems": 1}
                 for k in (1, 3) for ft in (1, 2, 3, 4) for q in (0, 1, 2, 3)])
    _check_mttkrp(b, pts, H0s, "one slab per item")
    # as many slabs per item as allowed
    b.set_tiles([{"kind": k, "ft": ft, "qbucket": q, "mt": 2, "item_elems": 1 << 30}
                 for k in (1, 3) for ft in (1, 2, 3, 4) for q in (0, 1, 2, 3)])
    _check_mttkrp(b, pts, H0s, "largest items")
    b.close()


def _oracle_after(pts, H0s, steps, T):
    out = []
    for pt, H0 in zip(pts, H0s):
        st = orc.init_state([h.astype(np.float64) for h in H0])
        opts = orc.Opts(inner_iters=T, mttkrp_operands="bf16_split")
        for _ in range(steps):
            orc.outer_step(pt.X, st, opts)
        out.append(st)
    return out


def _f32_recipe_reference(X, H0, T, steps=1):
    """One outer iteration with the batched recipe's arithmetic precision (not
    its summation order): the same bfloat16 operands with float32 library
    matmuls (float32 accumulation) for the MTTKRPs, FP64 across slabs where
    the kernels use it, and float32 Grams.  Its distance from the oracle
    measures how much float32 arithmetic alone moves one outer iteration."""
    Xq, s = orc.quantize_slabs_bf16(X)
    Xq32 = Xq.astype(np.float32)
    s32 = s.astype(np.float32)
    I, J, K = X.shape
    st = orc.init_state([h.astype(np.float64) for h in H0])
    Tm = None
    for n in [0, 1, 2] * steps:
        A, B, C = (h.astype(np.float32) for h in st.H)
        F = A.shape[1]
        if n == 0:
            Cb = orc._round_bf16(C)
            Tm = (Xq32.reshape(I * J, K) @ Cb).reshape(I, J, F) * s32[:, None, None]
            W = np.sum(Tm * B[None, :, :], axis=1, dtype=np.float32).astype(np.float64)
        elif n == 1:
            W = np.einsum("ijf,if->jf", Tm.astype(np.float64), A.astype(np.float64))
        else:
            Bh = orc._round_bf16(B)
            Bl = orc._round_bf16((B - Bh).astype(np.float32))
            W = np.zeros((K, F))
            for i in range(I):
                W += (s32[i] * A[i][None, :] * (Xq32[i].T @ Bh + Xq32[i].T @ Bl)).astype(np.float64)
        grams = [(h.astype(np.float32).T @ h.astype(np.float32)).astype(np.float64) for h in st.H]
        G = np.ones((F, F))
        for m in range(3):
            if m != n:
                G = G * grams[m]
        rho = orc.rho_trace(G)
        st.H[n], st.U[n], _, _ = orc.inner_sweep(W, st.H[n], st.U[n], G, rho, T)
    return st


def test_batch_one_step_matches_oracle(dev):
    # Gate: no worse than 3x the distance float32 arithmetic alone gives (see
    # _f32_recipe_reference), with floors of 1e-5 (H) and 1e-4 (U).
    T = 10
    b, pts, H0s, Hs = _batch(dev, BATCH, T=T)
    b.step(1)
    assert b.sync() == 0
    ref = _oracle_after(pts, H0s, 1, T)
    for p, st in enumerate(ref):
        f32 = _f32_recipe_reference(pts[p].X, H0s[p], T)
        for n in range(3):
            eh = rel(Hs[p][n].cpu().numpy(), st.H[n])
            eu = rel(b.U[p][n].cpu().numpy(), st.U[n])
            bh = max(1e-5, 3.0 * rel(f32.H[n], st.H[n]))
            bu = max(1e-4, 3.0 * rel(f32.U[n], st.U[n]))
            print(f"[batch] step p={p} n={n} H {eh:.2e} (bound {bh:.2e}) U {eu:.2e} (bound {bu:.2e})",
                  flush=True)
            assert eh < bh, (p, n, eh, bh)
            assert eu < bu or np.linalg.norm(st.U[n]) < 1e-12, (p, n, eu, bu)
    b.close()


def _oracle_fit_spread(X, H0, steps, T):
    """Fits of the oracle after `steps` outer iterations from the initial
    factors perturbed by +-2^-24 relative (one float32 rounding)."""
    out = []
    for sgn in (1.0, -1.0):
        rng = np.random.default_rng(0)
        H = [h.astype(np.float64) * (1.0 + sgn * 2.0 ** -24 * rng.standard_normal(h.shape)) for h in H0]
        st = orc.init_state(H)
        opts = orc.Opts(inner_iters=T, mttkrp_operands="bf16_split")
        for _ in range(steps):
            orc.outer_step(X, st, opts)
        out.append(orc.rfe(X, st.H))
    return out


def test_batch_fit_and_invariants_after_run(dev):
    # Fit after 15 outer iterations: within 3x the larger of the float32
    # recipe reference's drift and the oracle's spread under a one-rounding
    # perturbation of the start (floor 1e-6 relative), and complementarity of
    # H and U exact.
    T, steps = 5, 15
    spec = BATCH[:1] + BATCH[2:6]
    b, pts, H0s, Hs = _batch(dev, spec, T=T, seed0=760)
    b.step(steps)
    assert b.sync() == 0
    fits = b.fit()
    ref = _oracle_after(pts, H0s, steps, T)
    for p, st in enumerate(ref):
        r = orc.rfe(pts[p].X, st.H)
        r32 = orc.rfe(pts[p].X, _f32_recipe_reference(pts[p].X, H0s[p], T, steps).H)
        spread = max(abs(x - r) for x in _oracle_fit_spread(pts[p].X, H0s[p], steps, T))
        bound = max(1e-6 * r, 3.0 * abs(r32 - r), 3.0 * spread)
        print(f"[batch] fit p={p} gpu {fits[p]:.8f} oracle {r:.8f} f32 recipe {r32:.8f} "
              f"spread {spread:.2e}", flush=True)
        assert abs(fits[p] - r) < bound, (p, fits[p], r, bound)
        for n in range(3):
            h = Hs[p][n].cpu().numpy()
            u = b.U[p][n].cpu().numpy()
            assert (h >= 0).all() and (u >= 0).all()
            assert not np.any(h * u), (p, n)     # complementarity holds exactly
    b.close()


def test_batch_deterministic(dev):
    spec = BATCH[:4]
    runs = []
    for _ in range(2):
        b, _, _, Hs = _batch(dev, spec, T=5, seed0=800)
        b.step(4)
        assert b.sync() == 0
        runs.append([[h.cpu().numpy().copy() for h in hs] for hs in Hs])
        b.close()
    for a, c in zip(runs[0], runs[1]):
        for x, y in zip(a, c):
            np.testing.assert_array_equal(x, y)


def test_batch_autotune_keeps_results(dev):
    b, pts, H0s, _ = _batch(dev, BATCH[:5], seed0=820)
    tiles = b.autotune(reps=1)
    assert tiles and all(t["mt"] in (1, 2) and t["item_elems"] >= 1 for t in tiles)
    assert b.tiles() == tiles
    info = b.info()
    assert info["n_items"] == sum(info["items_by_kind"])
    _check_mttkrp(b, pts, H0s, "autotuned")
    b.step(2)
    assert b.sync() == 0
    b.close()


def test_batch_rejects_unsupported(dev):
    import paper_1409_2383_amd as ntf
    pt, H0 = problem((8, 9, 10), 3, 900, False)
    X = [torch.from_numpy(pt.X).to(dev)]
    H = [[torch.from_numpy(h.copy()).to(dev) for h in H0]]
    with pytest.raises(ntf.NtfError):
        ntf.NtfBatch(X, H, opts=ntf.AdmmOptions(precision=ntf.PREC_BF16_MIXED,
                                                rho_policy=ntf.RHO_ADAPTIVE))
    with pytest.raises(ValueError):
        ntf.NtfBatch(X, H, opts=ntf.AdmmOptions(precision=ntf.PREC_F32))
    # a contraction too long for the LDS at F = 64
    big = torch.zeros((1, 2, 4000), dtype=torch.float32, device=dev)
    Hb = [[torch.zeros((d, 64), dtype=torch.float32, device=dev) for d in (1, 2, 4000)]]
    with pytest.raises(ntf.NtfError):
        ntf.NtfBatch([big], Hb)
