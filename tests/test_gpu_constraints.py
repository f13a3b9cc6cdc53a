"""GPU parity of the structural constraints (Section IV-E: box and
cardinality; Section VI-D: rows that are probability mass functions) against
the oracle, through the C ABI.  FP64 mode: after one outer iteration the
factors match to 1e-11 (the GPU solves with (G + rho I)^{-1} and its row sums,
the oracle with a Cholesky solve or the KKT system: rounding order only; the
cardinality selection is a discrete decision that both sides take on FP64
values whose gaps at the threshold are far above that rounding)."""
import numpy as np
import pytest

from oracle import ntf_oracle as orc
from tests.gpu_helpers import problem, rel, to_dev

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1409_2383_amd as ntf
    ntf.library_path()
    return torch.device("cuda:0")


def _oracle_cons(spec):
    out = []
    for c in spec:
        if c is None:
            out.append(orc.NONNEG)
        elif c == "pmf_rows":
            out.append(orc.Constraint(kind="pmf_rows"))
        elif c[0] == "cardinality":
            out.append(orc.Constraint(kind="cardinality", card=c[1]))
        else:
            out.append(orc.Constraint(kind="box", lo=c[1], hi=c[2]))
    return tuple(out)


SPECS = [(("box", 0.05, 0.8), ("box", 0.0, 0.5), ("box", 0.1, 1.5)),
         (None, None, "pmf_rows"),
         ("pmf_rows", ("box", 0.02, 0.9), None)]


@pytest.mark.parametrize("spec", SPECS)
@pytest.mark.parametrize("dims,F", [((30, 41, 25), 6), ((17, 9, 40), 20)])
def test_constrained_steps_match_oracle(dev, spec, dims, F):
    import paper_1409_2383_amd as ntf
    pt, H0 = problem(dims, F, 950, True)
    X = torch.from_numpy(np.ascontiguousarray(pt.X)).to(dev)
    H = to_dev([h.copy() for h in H0], dev)
    s = ntf.NtfAdmm(X, H, opts=ntf.AdmmOptions(inner_iters=7, precision=ntf.PREC_F64))
    s.set_constraints(spec)
    st = orc.init_state([h.astype(np.float64) for h in H0])
    opts = orc.Opts(inner_iters=7, constraints=_oracle_cons(spec))
    for it in range(3):
        s.step()
        torch.cuda.synchronize()
        orc.outer_step(pt.X, st, opts)
        for n in range(3):
            e = rel(H[n].cpu().numpy(), st.H[n])
            assert e < 1e-11 * (10 ** it), (spec, it, n, e)
    for n, c in enumerate(spec):
        h = H[n].cpu().numpy()
        if isinstance(c, tuple):
            assert np.all(h >= c[1]) and np.all(h <= c[2])
        else:
            assert np.all(h >= 0.0)
    s.close()


def test_box_at_zero_and_infinity_is_the_default(dev):
    import paper_1409_2383_amd as ntf
    pt, H0 = problem((20, 30, 25), 5, 951, True)
    X = torch.from_numpy(np.ascontiguousarray(pt.X)).to(dev)
    out = []
    for spec in (None, (("box", 0.0, np.inf),) * 3):
        H = to_dev([h.copy() for h in H0], dev)
        s = ntf.NtfAdmm(X, H, opts=ntf.AdmmOptions(inner_iters=5, precision=ntf.PREC_F64))
        s.set_constraints(spec)
        for _ in range(3):
            s.step()
        torch.cuda.synchronize()
        out.append([h.cpu().numpy() for h in H])
        s.close()
    for a, b in zip(*out):
        np.testing.assert_array_equal(a, b)


def test_pmf_rows_recover_a_planted_tensor(dev):
    # the experiment of Section VI-D in small: A, B non-negative, the rows of C
    # probability mass functions, noiseless: the fit goes to zero and the
    # GPU trajectory stays on the oracle's
    import ntf_synth
    import paper_1409_2383_amd as ntf
    rng = np.random.default_rng(5)
    I, J, K, F = 40, 40, 20, 4
    A, B, C = rng.random((I, F)), rng.random((J, F)), rng.random((K, F))
    C /= C.sum(axis=1, keepdims=True)
    Xn = orc.reconstruct([A, B, C])
    H0 = ntf_synth.init_factors((I, J, K), F, 900)
    H0[2] = H0[2] / H0[2].sum(axis=1, keepdims=True)
    X = torch.from_numpy(Xn).to(dev)
    H = to_dev([h.copy() for h in H0], dev)
    s = ntf.NtfAdmm(X, H, opts=ntf.AdmmOptions(inner_iters=10, precision=ntf.PREC_F64))
    s.set_constraints((None, None, "pmf_rows"))
    s.run(400, stats=False)
    r_gpu = s.fit()
    st = orc.init_state([h.astype(np.float64) for h in H0])
    orc.run(Xn, st, orc.Opts(inner_iters=10, constraints=(orc.NONNEG, orc.NONNEG,
                                                            orc.Constraint(kind="pmf_rows"))), 400)
    r_orc = orc.rfe(Xn, st.H)
    print(f"[constraints] pmf rows, noiseless: RFE gpu {r_gpu:.3e} oracle {r_orc:.3e}", flush=True)
    assert r_gpu < 1e-5
    assert abs(r_gpu - r_orc) < 1e-3 * r_orc
    np.testing.assert_allclose(H[2].cpu().numpy().sum(axis=1), 1.0, atol=1e-5)
    s.close()


CARD_CASES = [
    # dims, F, spec, inner iterations, factor source, rho policy
    ((30, 41, 25), 6, (("cardinality", 70), None, None), 1, 0, "trace"),
    ((30, 41, 25), 6, (("cardinality", 61), ("cardinality", 100), ("cardinality", 90)), 3, 0, "trace"),
    ((17, 9, 40), 20, (None, ("cardinality", 50), ("box", 0.0, 0.7)), 4, 0, "trace"),
    ((40, 35, 30), 5, (("cardinality", 120), None, ("cardinality", 0)), 1, 1, "adaptive"),
    ((700, 12, 10), 7, (("cardinality", 2500), None, None), 2, 1, "adaptive"),
]


@pytest.mark.parametrize("dims,F,spec,T,src,policy", CARD_CASES)
def test_cardinality_steps_match_oracle(dev, dims, F, spec, T, src, policy):
    import paper_1409_2383_amd as ntf
    pt, H0 = problem(dims, F, 953, True)
    X = torch.from_numpy(np.ascontiguousarray(pt.X)).to(dev)
    H = to_dev([h.copy() for h in H0], dev)
    rp = ntf.RHO_ADAPTIVE if policy == "adaptive" else ntf.RHO_TRACE
    s = ntf.NtfAdmm(X, H, opts=ntf.AdmmOptions(inner_iters=T, precision=ntf.PREC_F64,
                                               factor_source=src, rho_policy=rp,
                                               rescale_dual_on_rho_change=1 if rp == ntf.RHO_ADAPTIVE else 0))
    s.set_constraints(spec)
    st = orc.init_state([h.astype(np.float64) for h in H0])
    opts = orc.Opts(inner_iters=T, constraints=_oracle_cons(spec), factor_source=src,
                    rho_policy=orc.RHO_ADAPTIVE if rp == ntf.RHO_ADAPTIVE else orc.RHO_TRACE,
                    rescale_dual_on_rho_change=rp == ntf.RHO_ADAPTIVE)
    for it in range(3):
        stats = s.step(stats=True)
        torch.cuda.synchronize()
        infos = orc.outer_step(pt.X, st, opts)
        for n in range(3):
            e = rel(H[n].cpu().numpy(), st.H[n])
            assert e < 1e-11 * (10 ** it), (spec, it, n, e)
            # residuals of each mode update (Section IV-C) and the iteration count
            tol = 1e-9 * (10 ** it)
            assert stats["prim"][n] == pytest.approx(infos[n]["prim"], rel=tol, abs=1e-12)
            assert stats["dual"][n] == pytest.approx(infos[n]["dual"], rel=tol, abs=1e-12)
            assert stats["inner_iters_mean"][n] == pytest.approx(T)
    for n, c in enumerate(spec):
        h = H[n].cpu().numpy()
        assert np.all(h >= 0.0)
        if isinstance(c, tuple) and c[0] == "cardinality":
            assert np.count_nonzero(h) <= c[1]
    s.close()


def test_cardinality_ties_keep_the_first_in_row_major_order(dev):
    # Mode 1 of a tensor whose two halves along mode 1 are equal, started
    # from equal halves of A with small integer data (exact MTTKRP): every
    # entry of V = Ht^T - U appears twice, so with an odd budget the
    # threshold value is tied and only its top-half copy is kept.
    import paper_1409_2383_amd as ntf
    rng = np.random.default_rng(954)
    I2, J, K, F = 12, 9, 8, 4
    Y = rng.integers(0, 4, (I2, J, K)).astype(np.float64)
    Xn = np.concatenate([Y, Y], axis=0)
    A0 = rng.integers(1, 4, (I2, F)).astype(np.float64)
    H0 = [np.concatenate([A0, A0], axis=0), rng.integers(1, 4, (J, F)).astype(np.float64),
          rng.integers(1, 4, (K, F)).astype(np.float64)]
    card = 2 * 11 + 1
    spec = (("cardinality", card), None, None)
    X = torch.from_numpy(Xn).to(dev)
    H = to_dev([h.copy() for h in H0], dev)
    s = ntf.NtfAdmm(X, H, opts=ntf.AdmmOptions(inner_iters=1, precision=ntf.PREC_F64))
    s.set_constraints(spec)
    s.step()
    torch.cuda.synchronize()
    A = H[0].cpu().numpy()
    top, bot = A[:I2], A[I2:]
    assert np.count_nonzero(A) == card
    diff = np.argwhere(top != bot)
    assert diff.shape[0] == 1, diff
    r, f = diff[0]
    assert top[r, f] > 0.0 and bot[r, f] == 0.0
    # the oracle takes the same decision where its own V carries the tie
    st = orc.init_state(H0)
    orc.outer_step(Xn, st, orc.Opts(inner_iters=1, constraints=_oracle_cons(spec)))
    if np.array_equal(st.P[0][:I2], st.P[0][I2:]):
        assert rel(A, st.H[0]) < 1e-12
    s.close()


def test_unsupported_and_invalid_constraints(dev):
    import paper_1409_2383_amd as ntf
    pt, H0 = problem((10, 11, 12), 3, 952, True)
    X = torch.from_numpy(np.ascontiguousarray(pt.X)).to(dev)
    s = ntf.NtfAdmm(X, to_dev(H0, dev), opts=ntf.AdmmOptions(precision=ntf.PREC_F64))
    with pytest.raises(ntf.NtfError):
        s.set_constraints((("cardinality", -1), None, None))
    s.close()
    s = ntf.NtfAdmm(X, to_dev(H0, dev), opts=ntf.AdmmOptions(precision=ntf.PREC_F64,
                                                             inner_iters=5, inner_eps_rel=1e-4))
    with pytest.raises(ntf.NtfError):
        s.set_constraints((("cardinality", 5), None, None))
    with pytest.raises(ntf.NtfError):
        s.set_constraints((("box", 1.0, 0.5), None, None))
    with pytest.raises(ntf.NtfError):
        s.set_constraints((("box", -np.inf, 1.0), None, None))
    s.close()
