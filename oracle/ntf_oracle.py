"""FP64 CPU oracle for ADMoM non-negative CP factorisation (NTF).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import or call this
module; only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark do.  It shares no code with the GPU library.

Everything here is plain NumPy/SciPy in float64, written to be checked against
the paper by eye (Liavas & Sidiropoulos, "Parallel algorithms for constrained
tensor factorization via the alternating direction method of multipliers"):

* matrix unfoldings and the Khatri-Rao product are formed explicitly
  (Section II, eq. f_X_matr), and MTTKRP is the plain matrix product of the
  unfolding with the Khatri-Rao matrix (Section IV, eq. ADMM_NTF_ALS_C);
* the F x F system matrix is the Hadamard product of the other factors' Gram
  matrices (Section IV-A, item 2);
* the regularised least-squares step uses a Cholesky factorisation
  (LAPACK via numpy/scipy);
* the projection and dual update follow eq. ADMoM_NTF (Section IV);
* residuals and stopping follow Section IV-C, penalty adaptation Section IV-D;
* a sparse tensor (``SparseTensor``: coordinates and values of the non-zeros)
  takes the MTTKRP from its non-zeros alone (Section IV-A, item 1), by a
  scatter-add of one product per non-zero; everything else is unchanged.

State convention (the "inner ADMM sweep" form).  For each mode n the state is
the non-negative auxiliary factor H_n (the paper's A-tilde), the scaled dual
U_n = -Y_n / rho_n and, in paper mode, the unconstrained primal P_n (the
paper's A).  One inner iteration for mode n is

    Ht^T = (W_n + rho (H_n + U_n)) (G_n + rho I)^{-1}     (regularised LS)
    V    = Ht^T - U_n
    H_n  = max(0, V)                                      (projection)
    U_n  = H_n - V            ( = U_n + H_n - Ht^T )      (dual update)

which is eq. ADMoM_NTF with A = Ht^T, A-tilde = H and Y = -rho U.  The paper
runs one such step per ADMoM iteration (footnote to eq. ADMM_NTF_ALS_C);
``inner_iters`` generalises that to T steps per mode.

Readings of points the paper leaves open are listed with each option below.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from itertools import combinations
from typing import List, Optional, Sequence

import numpy as np
import scipy.linalg

__all__ = [
    "Opts", "State", "unfold", "khatri_rao", "kr_for_mode", "mttkrp", "gram", "gram_hadamard",
    "rho_trace", "inner_sweep", "mode_update", "outer_step", "run", "reconstruct", "rfe",
    "rfe_expanded", "rescale_dual",
    "objective", "nnls_bruteforce", "nnls_rows", "kkt_violation", "init_state",
    "paper_admom_iteration", "partitioned_mode_update", "quantize_slabs_bf16",
    "RHO_TRACE", "RHO_FIXED", "RHO_ADAPTIVE",
]

RHO_TRACE, RHO_FIXED, RHO_ADAPTIVE = 0, 1, 2


# ---------------------------------------------------------------------------
# Section II: unfoldings, Khatri-Rao product, CP model
# ---------------------------------------------------------------------------

def khatri_rao(P: np.ndarray, Q: np.ndarray) -> np.ndarray:
    """Column-wise Kronecker product P (.) Q (notation, Section I-A).

    Column f is kron(P[:, f], Q[:, f]); row index p * Q.shape[0] + q."""
    P = np.asarray(P, dtype=np.float64)
    Q = np.asarray(Q, dtype=np.float64)
    if P.shape[1] != Q.shape[1]:
        raise ValueError("Khatri-Rao operands need the same number of columns")
    F = P.shape[1]
    out = np.empty((P.shape[0] * Q.shape[0], F))
    for f in range(F):
        out[:, f] = np.kron(P[:, f], Q[:, f])
    return out


def unfold(X: np.ndarray, n: int) -> np.ndarray:
    """Matrix unfolding X^(n), column order matching eq. f_X_matr for three
    modes and Appendix A for N modes: the remaining modes index the columns
    with the first of them fastest and the last slowest.

    X^(1) = A (C (.) B)^T : column index k*J + j
    X^(2) = B (C (.) A)^T : column index k*I + i
    X^(3) = C (B (.) A)^T : column index j*I + i
    (order 4: X^(1) = A (D (.) (C (.) B))^T, and so on)
    """
    X = np.asarray(X, dtype=np.float64)
    if not 0 <= n < X.ndim:
        raise ValueError("mode out of range")
    others = [m for m in range(X.ndim) if m != n]
    return X.transpose([n] + others[::-1]).reshape(X.shape[n], -1)


def kr_for_mode(factors: Sequence[np.ndarray], n: int) -> np.ndarray:
    """The Khatri-Rao matrix that multiplies X^(n) in eq. ADMM_NTF_ALS_C
    (Appendix A for N modes): the other factors, the last one slowest."""
    if not 0 <= n < len(factors):
        raise ValueError("mode out of range")
    others = [m for m in range(len(factors)) if m != n]
    K = np.asarray(factors[others[-1]], dtype=np.float64)
    for m in reversed(others[:-1]):
        K = khatri_rao(K, factors[m])
    return K


def mttkrp(X: np.ndarray, factors: Sequence[np.ndarray], n: int) -> np.ndarray:
    """W_n = X^(n) (Khatri-Rao of the other two factors), eq. ADMM_NTF_ALS_C."""
    return unfold(X, n) @ kr_for_mode(factors, n)


@dataclass(frozen=True)
class SparseTensor:
    """A sparse 3-way tensor by its non-zeros (Section IV-A, item 1: n
    non-zeros, n << IJK): coordinates ``idx`` [n][3] (distinct) and values
    ``val`` [n]; every other entry is zero."""
    idx: np.ndarray
    val: np.ndarray
    dims: tuple

    @property
    def shape(self):
        return tuple(self.dims)


def densify(T: SparseTensor) -> np.ndarray:
    """The dense tensor the non-zeros describe."""
    X = np.zeros(tuple(T.dims))
    for e in range(T.idx.shape[0]):
        i, j, k = (int(v) for v in T.idx[e])
        X[i, j, k] += float(T.val[e])
    return X


def mttkrp_sparse(T: SparseTensor, factors: Sequence[np.ndarray], n: int) -> np.ndarray:
    """W_n from the non-zeros alone (Section IV-A, item 1): each non-zero
    x_ijk adds x_ijk times the elementwise product of the other two factors'
    rows to row i (mode 1), j (mode 2) or k (mode 3) of W_n; three flops per
    non-zero and column, the Khatri-Rao matrix never formed."""
    others = [m for m in range(3) if m != n]
    P = np.asarray(factors[others[0]], dtype=np.float64)
    Q = np.asarray(factors[others[1]], dtype=np.float64)
    idx = np.asarray(T.idx, dtype=np.int64)
    contrib = np.asarray(T.val, dtype=np.float64)[:, None] * (P[idx[:, others[0]]] * Q[idx[:, others[1]]])
    W = np.zeros((int(T.dims[n]), P.shape[1]))
    np.add.at(W, idx[:, n], contrib)
    return W


def rfe_sparse(T: SparseTensor, factors: Sequence[np.ndarray]) -> float:
    """RFE (Section VI-A) of a sparse tensor without forming the model:
    ||X - M||^2 = sum over the non-zeros of (x - m)^2 plus the model's energy
    off them, ||M||^2 - sum over the non-zeros of m^2, with
    ||M||^2 = sum(A^T A * B^T B * C^T C) (Hadamard product of the Grams)."""
    A, B, C = (np.asarray(f, dtype=np.float64) for f in factors)
    idx = np.asarray(T.idx, dtype=np.int64)
    x = np.asarray(T.val, dtype=np.float64)
    m = np.sum(A[idx[:, 0]] * B[idx[:, 1]] * C[idx[:, 2]], axis=1)
    model2 = float(np.sum((A.T @ A) * (B.T @ B) * (C.T @ C)))
    err2 = float(np.sum((x - m) ** 2)) + model2 - float(np.sum(m * m))
    return math.sqrt(max(err2, 0.0)) / math.sqrt(float(np.sum(x * x)))


def reconstruct(factors: Sequence[np.ndarray]) -> np.ndarray:
    """[A, B, C] = sum_f a_f o b_f o c_f (Section II; any number of factors,
    Appendix A), summed term by term."""
    fac = [np.asarray(f, dtype=np.float64) for f in factors]
    out = np.zeros(tuple(f.shape[0] for f in fac))
    for f in range(fac[0].shape[1]):
        term = fac[0][:, f]
        for g in fac[1:]:
            term = np.multiply.outer(term, g[:, f])
        out += term
    return out


def objective(X: np.ndarray, factors: Sequence[np.ndarray]) -> float:
    """f_X(A,B,C) = 1/2 ||X - [A,B,C]||_F^2 (Section II)."""
    R = np.asarray(X, dtype=np.float64) - reconstruct(factors)
    return 0.5 * float(np.sum(R * R))


def rfe(X: np.ndarray, factors: Sequence[np.ndarray]) -> float:
    """Relative factorisation error ||X - [A,B,C]||_F / ||X||_F (Section VI-A)."""
    X = np.asarray(X, dtype=np.float64)
    R = X - reconstruct(factors)
    return math.sqrt(float(np.sum(R * R))) / math.sqrt(float(np.sum(X * X)))


def rfe_expanded(X: np.ndarray, factors: Sequence[np.ndarray], xnorm2: Optional[float] = None) -> float:
    """The RFE of Section VI-A from the expansion
    ||X - M||^2 = ||X||^2 - 2 <X, M> + ||M||^2, with <X, M> = sum(W_3 * C)
    (W_3 the mode-3 MTTKRP of the factors) and ||M||^2 = sum(A^T A * B^T B *
    C^T C) (Hadamard product of the Grams).  Equal to ``rfe`` up to the
    cancellation in the difference (relative error ~1e-16 / RFE^2), without
    forming the model; for fits of large tensors along a run."""
    X = np.asarray(X, dtype=np.float64)
    fac = [np.asarray(f, dtype=np.float64) for f in factors]
    if xnorm2 is None:
        xnorm2 = float(np.dot(X.ravel(), X.ravel()))
    inner = float(np.sum(mttkrp(X, fac, 2) * fac[2]))
    model2 = float(np.sum((fac[0].T @ fac[0]) * (fac[1].T @ fac[1]) * (fac[2].T @ fac[2])))
    return math.sqrt(max(xnorm2 - 2.0 * inner + model2, 0.0)) / math.sqrt(xnorm2)


# ---------------------------------------------------------------------------
# Section IV-A: Gram matrices through the Hadamard identity
# ---------------------------------------------------------------------------

def gram(H: np.ndarray) -> np.ndarray:
    H = np.asarray(H, dtype=np.float64)
    return H.T @ H


def gram_hadamard(factors: Sequence[np.ndarray], n: int) -> np.ndarray:
    """G_n = Hadamard product of H_m^T H_m over m != n (Section IV-A, item 2;
    N - 1 factors for N modes)."""
    G = None
    for m in range(len(factors)):
        if m == n:
            continue
        Gm = gram(factors[m])
        G = Gm if G is None else G * Gm
    return G


def rho_trace(G: np.ndarray, rho0: float = 1.0) -> float:
    """rho = trace(G)/F.  Guard (not in the paper): a non-positive or
    non-finite trace (an all-zero factor) falls back to rho0."""
    t = float(np.trace(G)) / G.shape[0]
    if not math.isfinite(t) or t <= 0.0:
        return float(rho0)
    return t


# ---------------------------------------------------------------------------
# Options and state
# ---------------------------------------------------------------------------

@dataclass
class Opts:
    inner_iters: int = 1                 # T; the paper uses 1 (footnote to eq. ADMM_NTF_ALS_C)
    rho_policy: int = RHO_TRACE          # RHO_TRACE: tr(G)/F each update; RHO_FIXED; RHO_ADAPTIVE (IV-D)
    rho0: float = 1.0                    # initial / fixed penalty (Section VI-A uses 1)
    mu: float = 8.0                      # residual-balancing parameters, Section VI-A values
    tau_incr: float = 4.0
    tau_decr: float = 2.0
    eps_abs: float = 0.0                 # per-row inner early stop (Section IV-C form); 0,0 = fixed T
    eps_rel: float = 0.0
    factor_source: int = 0               # 0: later modes use projected H; 1: the primal (paper)
    rescale_dual_on_rho_change: bool = False   # keep Y = -rho U fixed when rho changes
    # operand rounding of the MTTKRP (the mixed-precision recipe; not in the
    # paper): "exact", or bfloat16 operands as in mttkrp_mixed with mode 3 in
    # Khatri-Rao ("bf16_kr"), factored ("bf16_factored") or split factored
    # ("bf16_split") form
    mttkrp_operands: str = "exact"
    # per-mode set constraints (None: non-negativity on every factor)
    constraints: Optional[tuple] = None


@dataclass(frozen=True)
class Constraint:
    """Set constraint of one factor (Section IV-E; Section VI-D for pmf rows).

    kind "nonneg": H >= 0 (eq. g_M_def, the default).
    kind "box": lo <= H <= hi elementwise; the auxiliary update projects onto
        the box instead of the non-negative orthant.
    kind "pmf_rows": every row is a probability mass function: the auxiliary
        update stays the non-negative projection while the primal update is
        the least-squares step with the linear constraint that each row sums
        to one.
    kind "cardinality": H >= 0 with at most `card` non-zero entries in the
        whole factor (eq. g_new_def); the auxiliary update keeps the `card`
        largest positive entries of the matrix (ties by row-major index).
    """
    kind: str = "nonneg"
    lo: float = 0.0
    hi: float = math.inf
    card: int = 0


NONNEG = Constraint()


@dataclass
class State:
    H: List[np.ndarray]                  # non-negative factors (A-tilde, B-tilde, C-tilde)
    U: List[np.ndarray]                  # scaled duals U_n = -Y_n / rho_n
    P: List[np.ndarray]                  # primal factors (A, B, C); used when factor_source == 1
    rho: List[float]                     # rho used by the last update of each mode
    outer: int = 0
    stats: List[dict] = field(default_factory=list)

    def copy(self) -> "State":
        return State(H=[h.copy() for h in self.H], U=[u.copy() for u in self.U],
                     P=[p.copy() for p in self.P], rho=list(self.rho), outer=self.outer,
                     stats=list(self.stats))


def init_state(H0: Sequence[np.ndarray], rho0: float = 1.0, paper: bool = False) -> State:
    """Initial state.  Default: H_n = given non-negative factors, U_n = 0.

    Paper mode (Section VI-A): the primal B^0, C^0 take the given random values
    while every auxiliary and dual variable starts at zero."""
    H0 = [np.asarray(h, dtype=np.float64).copy() for h in H0]
    if paper:
        H = [np.zeros_like(h) for h in H0]
        P = [h.copy() for h in H0]
    else:
        H = [h.copy() for h in H0]
        P = [h.copy() for h in H0]
    U = [np.zeros_like(h) for h in H0]
    return State(H=H, U=U, P=P, rho=[float(rho0)] * len(H0))


# ---------------------------------------------------------------------------
# Section IV: inner ADMM sweep for one mode
# ---------------------------------------------------------------------------

def regularised_ls(L: np.ndarray, rhs: np.ndarray) -> np.ndarray:
    """Solve (G + rho I) Ht^T = rhs^T for every row with the Cholesky factor
    L (lower, G + rho I = L L^T): the least-squares step of eq. ADMM_NTF_ALS_C."""
    return scipy.linalg.cho_solve((L, True), rhs.T).T


def project_nonneg(V: np.ndarray) -> np.ndarray:
    """(V)_+ with +0 for ties and negative values (eq. ADMoM_NTF, auxiliary update)."""
    return np.where(V > 0.0, V, 0.0)


def project(V: np.ndarray, c: Constraint) -> np.ndarray:
    """Projection onto the constraint set of the auxiliary variable (Section
    IV-E: the only change a set constraint makes to the auxiliary update)."""
    if c.kind in ("nonneg", "pmf_rows"):
        return project_nonneg(V)
    if c.kind == "box":
        return np.minimum(np.maximum(V, c.lo), c.hi)
    if c.kind == "cardinality":
        P = project_nonneg(V)
        flat = P.ravel()
        order = np.argsort(-flat, kind="stable")          # descending, ties by index
        keep = np.zeros(flat.size, dtype=bool)
        keep[order[:c.card]] = True
        return np.where(keep.reshape(P.shape) & (P > 0.0), P, 0.0)
    raise ValueError(f"unknown constraint {c.kind!r}")


def pmf_rows_ls(G: np.ndarray, rho: float, rhs: np.ndarray) -> np.ndarray:
    """Least-squares step with each row of the result summing to one (Section
    VI-D): min_x 1/2 x^T (G + rho I) x - rhs^T x  s.t.  1^T x = 1, row by row,
    from its KKT system [[G + rho I, 1], [1^T, 0]] [x; lam] = [rhs; 1]."""
    F = G.shape[0]
    K = np.zeros((F + 1, F + 1))
    K[:F, :F] = G + rho * np.eye(F)
    K[:F, F] = 1.0
    K[F, :F] = 1.0
    R = np.concatenate([rhs, np.ones((rhs.shape[0], 1))], axis=1)
    return np.linalg.solve(K, R.T).T[:, :F]


def rescale_dual(U: np.ndarray, rho_old: float, rho_new: float) -> np.ndarray:
    """Scaled dual after a penalty change: the unscaled multiplier Y = -rho U
    is the ADMoM state (Section IV-D changes rho only), so U_new = -Y/rho_new
    = U rho_old / rho_new."""
    return U * (rho_old / rho_new)


def dual_update(Hn: np.ndarray, V: np.ndarray) -> np.ndarray:
    """U_new = U + H - Ht^T = H - V with V = Ht^T - U (eq. ADMoM_NTF, dual update
    in the scaled form U = -Y/rho)."""
    return Hn - V


def inner_sweep(W: np.ndarray, H: np.ndarray, U: np.ndarray, G: np.ndarray, rho: float,
                T: int, eps_abs: float = 0.0, eps_rel: float = 0.0,
                constraint: Constraint = NONNEG):
    """Run T inner ADMoM iterations on every row (rows are independent).

    Returns (H, U, Ht, info).  ``Ht`` is the last regularised-LS solution
    (the paper's primal A^{k+1}).  With eps_abs or eps_rel non-zero a row stops
    as soon as its own primal and dual residuals meet the Section IV-C test
    with the row sizes in place of the matrix sizes:
        ||h - ht||          <= sqrt(F) eps_abs + eps_rel max(||ht||, ||h||)
        rho ||h - h_prev||  <= sqrt(F) eps_abs + eps_rel rho ||u||
    (rho ||u|| = ||y||).  ``info['iters']`` holds the iterations each row ran.
    """
    W = np.asarray(W, dtype=np.float64)
    H = np.asarray(H, dtype=np.float64).copy()
    U = np.asarray(U, dtype=np.float64).copy()
    rows, F = W.shape
    if constraint.kind == "cardinality" and (eps_abs > 0.0 or eps_rel > 0.0):
        raise ValueError("the cardinality projection couples all rows: no row-wise early stop")
    M = G + rho * np.eye(F)
    L = np.linalg.cholesky(M)                       # lower, M = L L^T
    Ht = np.zeros_like(W)
    active = np.ones(rows, dtype=bool)
    iters = np.zeros(rows, dtype=np.int64)
    prim2 = dual2 = 0.0
    early = (eps_abs > 0.0) or (eps_rel > 0.0)
    for t in range(T):
        idx = np.nonzero(active)[0]
        if idx.size == 0:
            break
        Wa, Ha, Ua = W[idx], H[idx], U[idx]
        rhs = Wa + rho * (Ha + Ua)
        Xt = pmf_rows_ls(G, rho, rhs) if constraint.kind == "pmf_rows" else regularised_ls(L, rhs)
        V = Xt - Ua
        Hn = project(V, constraint)
        Un = dual_update(Hn, V)
        dH = Hn - Ha
        Ht[idx] = Xt
        H[idx] = Hn
        U[idx] = Un
        iters[idx] += 1
        if t == T - 1 or early:
            pr = np.linalg.norm(Hn - Xt, axis=1)
            du = rho * np.linalg.norm(dH, axis=1)
            if t == T - 1:
                prim2 = float(np.sum(np.linalg.norm(H - Ht, axis=1) ** 2))
                dual2 = float(np.sum(du ** 2))
            if early:
                tol_p = math.sqrt(F) * eps_abs + eps_rel * np.maximum(
                    np.linalg.norm(Xt, axis=1), np.linalg.norm(Hn, axis=1))
                tol_d = math.sqrt(F) * eps_abs + eps_rel * rho * np.linalg.norm(Un, axis=1)
                done = (pr <= tol_p) & (du <= tol_d)
                active[idx[done]] = False
    info = {"iters": iters, "prim2": prim2, "dual2": dual2}
    return H, U, Ht, info


def mode_update(X: np.ndarray, st: State, n: int, opts: Opts) -> dict:
    """Update mode n in place (one line of eq. ADMM_NTF_ALS_C plus the
    projection and dual update of eq. ADMoM_NTF)."""
    feed = st.P if opts.factor_source == 1 else st.H
    factors = list(feed)
    if isinstance(X, SparseTensor):
        W = mttkrp_sparse(X, factors, n)
    elif opts.mttkrp_operands == "exact":
        W = mttkrp(X, factors, n)
    else:
        m3 = {"bf16_factored": "factored", "bf16_split": "split"}.get(opts.mttkrp_operands, "kr")
        W = mttkrp_mixed(X, factors, n, mode3=m3)
    G = gram_hadamard(factors, n)
    if opts.rho_policy == RHO_TRACE:
        rho = rho_trace(G, opts.rho0)
    else:
        rho = st.rho[n]
    U = st.U[n]
    if opts.rescale_dual_on_rho_change and rho != st.rho[n]:
        U = rescale_dual(U, st.rho[n], rho)         # keep Y = -rho U unchanged
    H_prev = st.H[n].copy()
    cons = opts.constraints[n] if opts.constraints is not None else NONNEG
    H, U, Ht, info = inner_sweep(W, st.H[n], U, G, rho, opts.inner_iters, opts.eps_abs, opts.eps_rel,
                                 cons)
    st.H[n], st.U[n], st.P[n] = H, U, Ht
    st.rho[n] = rho
    # Section IV-C residuals of this mode update (matrix form)
    info.update({
        "mode": n, "rho": rho,
        "prim": float(np.linalg.norm(H - Ht)),               # ||P|| = ||A - A-tilde||
        "dual": float(rho * np.linalg.norm(H - H_prev)),     # ||D|| = rho ||A-tilde^k - A-tilde^{k-1}||
        "norm_p": float(np.linalg.norm(Ht)), "norm_h": float(np.linalg.norm(H)),
        "norm_y": float(rho * np.linalg.norm(U)),
    })
    return info


def _adapt_rho(rho: float, prim: float, dual: float, opts: Opts) -> float:
    """Residual balancing, eq. varying_penalty_rule (Section IV-D)."""
    if prim > opts.mu * dual:
        return rho * opts.tau_incr
    if dual > opts.mu * prim:
        return rho / opts.tau_decr
    return rho


def outer_step(X: np.ndarray, st: State, opts: Opts) -> List[dict]:
    """One ADMoM iteration: modes 1, 2, 3 in Gauss-Seidel order (eq.
    ADMM_NTF_ALS_C: B uses the new A, C uses the new A and B)."""
    infos = [mode_update(X, st, n, opts) for n in range(len(st.H))]
    if opts.rho_policy == RHO_ADAPTIVE:
        for n in range(len(st.H)):
            new = _adapt_rho(st.rho[n], infos[n]["prim"], infos[n]["dual"], opts)
            if new != st.rho[n]:
                st.U[n] = rescale_dual(st.U[n], st.rho[n], new)   # Y = -rho U is the state
            st.rho[n] = new
    st.outer += 1
    return infos


def converged_paper(infos: List[dict], dims: Sequence[int], F: int, eps_abs: float, eps_rel: float) -> bool:
    """Stopping test of Section IV-C on every mode."""
    for n, inf in enumerate(infos):
        s = math.sqrt(dims[n] * F) * eps_abs
        if inf["prim"] > s + eps_rel * max(inf["norm_p"], inf["norm_h"]):
            return False
        if inf["dual"] > s + eps_rel * inf["norm_y"]:
            return False
    return True


def run(X: np.ndarray, st: State, opts: Opts, outer_iters: int, fit_every: int = 0,
        stop_eps: Optional[tuple] = None) -> State:
    """Run ``outer_iters`` ADMoM iterations (or until the Section IV-C test
    with ``stop_eps = (eps_abs, eps_rel)`` holds)."""
    for _ in range(outer_iters):
        infos = outer_step(X, st, opts)
        rec = {"outer": st.outer, "rho": list(st.rho),
               "prim": [i["prim"] for i in infos], "dual": [i["dual"] for i in infos]}
        if fit_every and st.outer % fit_every == 0:
            rec["rfe"] = rfe_sparse(X, st.H) if isinstance(X, SparseTensor) else rfe(X, st.H)
        st.stats.append(rec)
        if stop_eps is not None and converged_paper(infos, X.shape, st.H[0].shape[1], *stop_eps):
            break
    return st


# ---------------------------------------------------------------------------
# The paper's own form of one ADMoM iteration (eqs. ADMoM_NTF, ADMM_NTF_ALS_C),
# with explicit primal A, auxiliary A-tilde and unscaled dual Y.
# ---------------------------------------------------------------------------

def paper_admom_iteration(X: np.ndarray, P: List[np.ndarray], Aux: List[np.ndarray],
                          Y: List[np.ndarray], rho: Sequence[float]):
    """One iteration exactly as printed: each primal update is
        A^{k+1} = (X^(1)(C^k (.) B^k) + rho A-tilde^k - Y^k)
                  ((C^k (.) B^k)^T (C^k (.) B^k) + rho I)^{-1}
    with B using A^{k+1} and C using A^{k+1}, B^{k+1}; then
        A-tilde^{k+1} = (A^{k+1} + Y^k / rho)_+,  Y^{k+1} = Y^k + rho (A^{k+1} - A-tilde^{k+1}).
    The Gram is formed as the explicit (KR)^T (KR), not via the Hadamard identity."""
    P = [p.copy() for p in P]
    for n in range(len(P)):
        KR = kr_for_mode(P, n)
        lhs = KR.T @ KR + rho[n] * np.eye(KR.shape[1])
        rhs = unfold(X, n) @ KR + rho[n] * Aux[n] - Y[n]
        P[n] = np.linalg.solve(lhs, rhs.T).T       # lhs is symmetric: (rhs) lhs^{-1}
    Aux_new, Y_new = [], []
    for n in range(len(P)):
        a = np.maximum(P[n] + Y[n] / rho[n], 0.0)
        Aux_new.append(a)
        Y_new.append(Y[n] + rho[n] * (P[n] - a))
    return P, Aux_new, Y_new


# ---------------------------------------------------------------------------
# Section V / Appendix B: block-partitioned update of one mode
# ---------------------------------------------------------------------------

def partitioned_mode_update(X: np.ndarray, factors: Sequence[np.ndarray], H: np.ndarray,
                            U: np.ndarray, n: int, rho: float, T: int, blocks: int):
    """Mode-n update computed block by block as in eq. C_nC_sol: the rows of
    the updated factor are split into ``blocks`` row blocks and the other
    factor with the longest mode is split into ``blocks`` row blocks too; each
    block update sums the partial MTTKRPs and partial Grams over the blocks of
    that factor and then solves with the common system matrix."""
    X = np.asarray(X, dtype=np.float64)
    others = [m for m in range(3) if m != n]
    split_m = others[0] if factors[others[0]].shape[0] >= factors[others[1]].shape[0] else others[1]
    dn = H.shape[0]
    row_blocks = np.array_split(np.arange(dn), blocks)
    other_blocks = np.array_split(np.arange(factors[split_m].shape[0]), blocks)
    F = H.shape[1]
    Hn = np.empty_like(np.asarray(H, dtype=np.float64))
    Un = np.empty_like(Hn)
    Gsum = np.zeros((F, F))
    for ob in other_blocks:
        fb = [np.asarray(f, dtype=np.float64) for f in factors]
        fb[split_m] = fb[split_m][ob]
        Gsum += kr_for_mode(fb, n).T @ kr_for_mode(fb, n)
    for rb in row_blocks:
        Wb = np.zeros((rb.size, F))
        for ob in other_blocks:
            fb = [np.asarray(f, dtype=np.float64) for f in factors]
            fb[split_m] = fb[split_m][ob]
            Xb = X.take(rb, axis=n).take(ob, axis=split_m)     # block (rb, ob) of the unfolding
            Wb += unfold(Xb, n) @ kr_for_mode(fb, n)
        hb, ub, _, _ = inner_sweep(Wb, np.asarray(H)[rb], np.asarray(U)[rb], Gsum, rho, T)
        Hn[rb], Un[rb] = hb, ub
    return Hn, Un


# ---------------------------------------------------------------------------
# Non-negative least squares per row: min_{h >= 0} 1/2 h^T G h - w^T h
# ---------------------------------------------------------------------------

def nnls_bruteforce(G: np.ndarray, w: np.ndarray) -> np.ndarray:
    """Exact minimiser by enumerating all 2^F active sets (G positive
    definite, so the minimiser is unique and is the only KKT point)."""
    G = np.asarray(G, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    F = G.shape[0]
    best, best_val = np.zeros(F), 0.0
    for r in range(1, F + 1):
        for S in combinations(range(F), r):
            S = list(S)
            hS = np.linalg.solve(G[np.ix_(S, S)], w[S])
            if np.any(hS < 0.0):
                continue
            h = np.zeros(F)
            h[S] = hS
            val = 0.5 * h @ G @ h - w @ h
            if val < best_val:
                best, best_val = h, val
    return best


def nnls_rows(G: np.ndarray, W: np.ndarray) -> np.ndarray:
    """Row-wise NNLS with Lawson-Hanson (scipy) on the Cholesky factor:
    1/2 h^T G h - w^T h = 1/2 ||R h - R^{-T} w||^2 + const with G = R^T R."""
    from scipy.optimize import nnls
    R = np.linalg.cholesky(G).T
    out = np.empty_like(np.asarray(W, dtype=np.float64))
    for i, w in enumerate(np.asarray(W, dtype=np.float64)):
        b = scipy.linalg.solve_triangular(R, w, trans="T")
        out[i], _ = nnls(R, b, maxiter=50 * G.shape[0])
    return out


def kkt_violation(G: np.ndarray, W: np.ndarray, H: np.ndarray) -> np.ndarray:
    """Per-row size of the NNLS KKT violation ||min(h, h G - w)|| (eq. KKT_NTF
    restricted to one factor: gradient h G - w >= 0, h >= 0, complementarity)."""
    g = H @ G - W
    return np.linalg.norm(np.minimum(H, g), axis=1)


# ---------------------------------------------------------------------------
# Mixed-precision input: bfloat16 copy with a power-of-two scale per mode-1 slab
# ---------------------------------------------------------------------------

def _round_bf16(x: np.ndarray) -> np.ndarray:
    """Round float32 values to bfloat16 (round to nearest, ties to even),
    returned as float32 holding the bfloat16 value."""
    b = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (b >> 16) & 1
    r = ((b + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32)


def slab_scales(X: np.ndarray) -> np.ndarray:
    """Per-slab scale s_i = 2^e_i with max|X[i]| / s_i in [1, 2) (s_i = 1 for
    an all-zero slab)."""
    X = np.asarray(X, dtype=np.float32)
    s = np.ones(X.shape[0])
    for i in range(X.shape[0]):
        m = float(np.max(np.abs(X[i])))
        if m > 0.0 and math.isfinite(m):
            _, e = math.frexp(m)                    # m = mant * 2^e, mant in [0.5, 1)
            s[i] = math.ldexp(1.0, e - 1)
    return s


def quantize_slabs_bf16(X: np.ndarray, s: Optional[np.ndarray] = None):
    """The bfloat16 values of X[i] / s_i (scales from ``slab_scales`` unless
    given).  Returns (Xq as float64 holding the bfloat16 values, s as
    float64)."""
    X = np.asarray(X, dtype=np.float32)
    if s is None:
        s = slab_scales(X)
    Xq = np.empty(X.shape, dtype=np.float64)
    for i in range(X.shape[0]):
        Xq[i] = _round_bf16((X[i].astype(np.float64) / s[i]).astype(np.float32)).astype(np.float64)
    return Xq, s


def _mode3_b(B: np.ndarray, mode3: str) -> np.ndarray:
    """The B operand of the factored mode-3 forms (float32 B in): bf16(B),
    or bf16(B) + bf16(fl32(B - bf16(B))) for the split form."""
    hi = _round_bf16(B)
    if mode3 == "factored":
        return hi.astype(np.float64)
    lo = _round_bf16((B - hi.astype(np.float32)).astype(np.float32))
    return hi.astype(np.float64) + lo.astype(np.float64)


def mttkrp_mixed(X: np.ndarray, factors: Sequence[np.ndarray], n: int, mode3: str = "kr") -> np.ndarray:
    """MTTKRP with the operand rounding of the mixed-precision recipe (the
    method itself is unchanged): X is replaced by its per-slab bfloat16 copy
    s_i * Xq[i]; modes 1 and 2 contract against bfloat16(C) with the other
    factor in float32.  Mode 3, mode3="kr": against Khatri-Rao rows formed in
    float32 as (s_i * A[i,:]) * B[j,:] and rounded to bfloat16; mode3=
    "factored": against bfloat16(B) with A in float32 applied per slab
    (W3[k,:] = sum_i s_i A[i,:] * sum_j Xq[i,j,k] bf16(B[j,:])); mode3=
    "split": as "factored" with B carried as two bfloat16 terms, hi =
    bf16(B) and lo = bf16(fl32(B - hi)) (then a rounding of B shared by all
    slabs no longer biases every slab the same way).  Accumulation is exact
    up to float64 rounding."""
    if mode3 not in ("kr", "factored", "split"):
        raise ValueError("mode3 must be 'kr', 'factored' or 'split'")
    Xq, s = quantize_slabs_bf16(X)
    A, B, C = (np.asarray(f, dtype=np.float32) for f in factors)
    Xs = Xq * s[:, None, None]
    if n == 0:
        Cb = _round_bf16(C).astype(np.float64)
        return mttkrp(Xs, [A.astype(np.float64), B.astype(np.float64), Cb], 0)
    if n == 1:
        Cb = _round_bf16(C).astype(np.float64)
        return mttkrp(Xs, [A.astype(np.float64), B.astype(np.float64), Cb], 1)
    if mode3 in ("factored", "split"):
        return mttkrp(Xs, [A.astype(np.float64), _mode3_b(B, mode3), C.astype(np.float64)], 2)
    # mode 3: KR[(i,j), f] = bf16(fl32(fl32(s_i A[i,f]) B[j,f]))
    I, J = A.shape[0], B.shape[0]
    sA = (s.astype(np.float32)[:, None] * A).astype(np.float32)
    KR = (sA[:, None, :] * B[None, :, :]).astype(np.float32)          # [I, J, F], float32 products
    KRb = _round_bf16(KR).astype(np.float64).reshape(I * J, -1)
    Xflat = Xq.reshape(I * J, -1)                                      # rows (i, j), columns k
    return Xflat.T @ KRb


# ---------------------------------------------------------------------------
# Selected output rows (for checks of full-size runs, one row at a time)
# ---------------------------------------------------------------------------

def mttkrp_rows(X: np.ndarray, factors: Sequence[np.ndarray], n: int, rows) -> np.ndarray:
    """Rows ``rows`` of W_n = X^(n) (Khatri-Rao of the other factors): the
    MTTKRP of the sub-tensor holding only those indices of mode n (any order
    N; each output row depends on its own slice of X only)."""
    rows = np.asarray(rows, dtype=np.int64)
    Xs = np.take(np.asarray(X), rows, axis=n).astype(np.float64)
    fac = [np.asarray(f, dtype=np.float64) for f in factors]
    fac[n] = fac[n][rows]
    return mttkrp(Xs, fac, n)


def mttkrp_mixed_rows(X: np.ndarray, factors: Sequence[np.ndarray], n: int, rows,
                      mode3: str = "kr") -> np.ndarray:
    """Rows ``rows`` of ``mttkrp_mixed`` (three modes): the per-slab scales
    come from the whole tensor, the rounding and contraction from the slice
    of X that the rows read."""
    rows = np.asarray(rows, dtype=np.int64)
    X = np.asarray(X, dtype=np.float32)
    s = slab_scales(X)
    fac = [np.asarray(f, dtype=np.float32) for f in factors]
    if n == 0:
        Xq, _ = quantize_slabs_bf16(X[rows], s[rows])
        A = fac[0][rows]
        return mttkrp_mixed_from(Xq, s[rows], [A, fac[1], fac[2]], 0, mode3)
    Xsub = np.ascontiguousarray(X[:, rows, :] if n == 1 else X[:, :, rows])
    Xq, _ = quantize_slabs_bf16(Xsub, s)
    sub = list(fac)
    sub[n] = fac[n][rows]
    return mttkrp_mixed_from(Xq, s, sub, n, mode3)


def mttkrp_mixed_from(Xq: np.ndarray, s: np.ndarray, factors: Sequence[np.ndarray], n: int,
                      mode3: str = "kr") -> np.ndarray:
    """The contraction step of ``mttkrp_mixed`` for given bfloat16 values Xq
    and slab scales s."""
    A, B, C = (np.asarray(f, dtype=np.float32) for f in factors)
    Xs = Xq * s[:, None, None]
    if n in (0, 1):
        Cb = _round_bf16(C).astype(np.float64)
        return mttkrp(Xs, [A.astype(np.float64), B.astype(np.float64), Cb], n)
    if mode3 in ("factored", "split"):
        return mttkrp(Xs, [A.astype(np.float64), _mode3_b(B, mode3), C.astype(np.float64)], 2)
    I, J = A.shape[0], B.shape[0]
    sA = (s.astype(np.float32)[:, None] * A).astype(np.float32)
    KR = (sA[:, None, :] * B[None, :, :]).astype(np.float32)
    KRb = _round_bf16(KR).astype(np.float64).reshape(I * J, -1)
    return Xq.reshape(I * J, -1).T @ KRb


def mttkrp_sparse_rows(T: SparseTensor, factors: Sequence[np.ndarray], n: int, rows) -> np.ndarray:
    """Rows ``rows`` of ``mttkrp_sparse``: the non-zeros of those rows only."""
    rows = np.asarray(rows, dtype=np.int64)
    idx = np.asarray(T.idx, dtype=np.int64)
    keep = np.isin(idx[:, n], rows)
    sub = SparseTensor(idx=idx[keep], val=np.asarray(T.val)[keep], dims=T.dims)
    return mttkrp_sparse(sub, factors, n)[rows]
