"""Checks at the benchmark's full sizes, in the configuration bench.py times:
sampled output rows of every MTTKRP against the oracle's row-restricted
forms (the oracle computes each row from the slice of X it reads), and the
exact invariants of a full-size step.  Inputs come from the same generators
and seeds as the benchmark workloads."""
import numpy as np
import pytest

import ntf_synth
from oracle import ntf_oracle as orc
from tests.gpu_helpers import rel, to_dev

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1409_2383_amd as ntf
    ntf.library_path()
    return torch.device("cuda:0")


def _rows(d, rng, k=12, extra=()):
    r = set(int(x) for x in rng.choice(d, size=min(k, d), replace=False))
    r.update(int(x) for x in extra if 0 <= x < d)
    r.update((0, d - 1))
    return np.array(sorted(r))


@pytest.fixture(scope="module")
def c3():
    dims, F = (1000, 800, 600), 64
    seed = ntf_synth.config_seed(3)
    pt = ntf_synth.planted(dims, F, seed, dist="exponential", snr_db=30.0, dtype=np.float32)
    H0 = ntf_synth.init_factors(dims, F, seed, dtype=np.float64)
    return pt.X, H0


@pytest.mark.parametrize("arm", ["mixed", "fp32"])
def test_c3_mttkrp_sampled_rows(dev, c3, arm):
    import paper_1409_2383_amd as ntf
    X, H0 = c3
    prec = ntf.PREC_BF16_MIXED if arm == "mixed" else ntf.PREC_F32
    print(f"[fullsize] 1000x800x600 F=64 {arm}: MTTKRP rows", flush=True)
    H = [torch.from_numpy(h).to(dev, dtype=torch.float32) for h in H0]
    s = ntf.NtfAdmm(torch.from_numpy(X).to(dev), H, opts=ntf.AdmmOptions(inner_iters=10, precision=prec))
    fac = [h.astype(np.float32) for h in H0]
    rng = np.random.default_rng(7)
    for n in range(3):
        rows = _rows(X.shape[n], rng)
        W = s.mttkrp(n).cpu().numpy()[rows]
        if arm == "mixed":
            ref = orc.mttkrp_mixed_rows(X, fac, n, rows, mode3="split")
        else:
            ref = orc.mttkrp_rows(X, fac, n, rows)
        tol = 1e-6
        e = rel(W, ref)
        print(f"[fullsize]   mode {n + 1}: {len(rows)} rows, rel err {e:.2e}", flush=True)
        assert e < tol, (n, e)
    s.close()


def test_c3_mixed_step_invariants(dev, c3):
    import paper_1409_2383_amd as ntf
    X, H0 = c3
    print("[fullsize] 1000x800x600 F=64 mixed: 3 steps, invariants", flush=True)
    H = [torch.from_numpy(h).to(dev, dtype=torch.float32) for h in H0]
    s = ntf.NtfAdmm(torch.from_numpy(X).to(dev), H,
                    opts=ntf.AdmmOptions(inner_iters=10, precision=ntf.PREC_BF16_MIXED))
    r0 = s.fit()
    for _ in range(3):
        st = s.step(stats=True)
        assert st["numeric_error"] == 0
    r3 = s.fit()
    for n in range(3):
        h, u = s.H[n].cpu().numpy(), s.U[n].cpu().numpy()
        assert np.all(np.isfinite(h)) and np.all(h >= 0.0)
        assert not np.any(h * u)                     # projection and dual update are exact
    assert r3 < r0
    # the monitoring fit from ||X||^2 - 2<W3,H3> + sum(G1*G2*G3) agrees with the direct one
    assert st["rfe_cheap"] == pytest.approx(r3, rel=2e-2)
    s.close()


def test_sparse_bench_size_sampled_rows(dev):
    import paper_1409_2383_amd as ntf
    dims, F = (12092, 9184, 28818), 32
    seed = ntf_synth.config_seed(6)
    sp = ntf_synth.sparse_planted(dims, 8, 76_000_000, seed, skew=2.0, dtype=np.float32)
    H0 = ntf_synth.init_factors(dims, F, seed, dtype=np.float32)
    print(f"[fullsize] sparse {dims}, {sp.idx.shape[0]} non-zeros, F={F}: MTTKRP rows", flush=True)
    H = [torch.from_numpy(h).to(dev) for h in H0]
    s = ntf.NtfAdmmSparse(torch.from_numpy(sp.idx).to(dev), torch.from_numpy(sp.val).to(dev), dims, H,
                          opts=ntf.AdmmOptions(inner_iters=10, precision=ntf.PREC_F32))
    T = orc.SparseTensor(idx=sp.idx, val=sp.val.astype(np.float64), dims=dims)
    rng = np.random.default_rng(8)
    for n in range(3):
        counts = np.bincount(sp.idx[:, n], minlength=dims[n])
        heavy = np.argsort(counts)[-4:]                # rows cut into the most segment pieces
        rows = _rows(dims[n], rng, extra=heavy)
        W = s.mttkrp(n).cpu().numpy()[rows]
        ref = orc.mttkrp_sparse_rows(T, [h.astype(np.float64) for h in H0], n, rows)
        e = rel(W, ref)
        print(f"[fullsize]   mode {n + 1}: {len(rows)} rows (heaviest {counts[heavy].max()} non-zeros), "
              f"rel err {e:.2e}", flush=True)
        assert e < 1e-6, (n, e)
    s.close()


def test_nway_bench_size_sampled_rows(dev):
    import paper_1409_2383_amd as ntf
    dims, F = (120, 110, 100, 90), 32
    seed = ntf_synth.config_seed(7)
    X, _, _ = ntf_synth.planted_nway(dims, F, seed, snr_db=20.0, dtype=np.float32)
    H0 = ntf_synth.init_factors(dims, F, seed, dtype=np.float32)
    print(f"[fullsize] 4-way {dims} F={F}: MTTKRP rows", flush=True)
    H = [torch.from_numpy(h).to(dev) for h in H0]
    s = ntf.NtfNway(torch.from_numpy(X).to(dev), H, opts=ntf.AdmmOptions(inner_iters=10))
    rng = np.random.default_rng(9)
    for n in range(4):
        rows = _rows(dims[n], rng, k=6)
        W = s.mttkrp(n).cpu().numpy()[rows]
        ref = orc.mttkrp_rows(X, H0, n, rows)
        e = rel(W, ref)
        print(f"[fullsize]   mode {n + 1}: {len(rows)} rows, rel err {e:.2e}", flush=True)
        assert e < 2e-6, (n, e)
    s.close()
