"""Oracle steps II-IV of dOpInf (arXiv:2504.14338, Sec. 3.3-3.5).

TEST INFRASTRUCTURE ONLY (see the package docstring): never imported by the
product path.  Pins: tests/test_oracle_pins.py.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "temporal_mean", "variable_scales", "apply_statistics", "preprocess", "gram", "eig_desc",
    "fix_signs", "energy_rank", "reduce_basis_free", "qhat_by_projection",
    "quad_features", "quad_pairs", "n_quad", "opinf_data", "regularizer",
    "solve_operators", "split_operators", "rollout", "train_error",
    "growth_ratio", "score", "select_best", "sweep", "pipeline",
    "lift", "LIFT_COPY", "LIFT_PRODUCT", "LIFT_RECIPROCAL", "basis_rows", "postprocess",
]


# ---------------------------------------------------------------------------
# Step II (Sec. 3.3): centering and scaling
# ---------------------------------------------------------------------------

def temporal_mean(Q):
    """Temporal mean of every row (each row is one variable at one point).

    Sec. 3.3: snapshots are centered by their temporal mean over the training
    horizon; the listing takes the mean along the snapshot axis, i.e. per row
    (READING: per-row centering).
    """
    return np.mean(Q, axis=1)


def variable_scales(Qc, var_rows):
    """Per-variable scaling factor: the largest |entry| of the centered
    variable over all its rows and all snapshots (Sec. 3.3, max-abs scaling).

    A variable whose centered data are identically zero gets factor 1 and is
    reported in ``zero_range`` (READING: the paper does not treat it).
    """
    nvars = len(var_rows) - 1
    s = np.empty(nvars)
    zero_range = []
    for v in range(nvars):
        blk = Qc[var_rows[v]:var_rows[v + 1], :]
        m = float(np.max(np.abs(blk))) if blk.size else 0.0
        if m == 0.0:
            zero_range.append(v)
            m = 1.0
        s[v] = m
    return s, zero_range


def apply_statistics(Q, mu, s_rows):
    """(Q - mu 1^T) / s, row by row, for given row means mu and per-row scale
    factors s_rows (each row carries its variable's s_v): the transform of
    Sec. 3.3 with division, as in its listing."""
    Q = np.asarray(Q, dtype=np.float64)
    return (Q - np.asarray(mu, dtype=np.float64)[:, None]) / np.asarray(s_rows, dtype=np.float64)[:, None]


def preprocess(Q, var_rows, center=True, scale=True):
    """Step II: returns (mu, s, Qs, zero_range) with Qs = (Q - mu 1^T) / s_v.

    Division (not multiplication by a reciprocal), as in Sec. 3.3's listing.
    """
    Q = np.asarray(Q, dtype=np.float64)
    mu = temporal_mean(Q) if center else np.zeros(Q.shape[0])
    Qc = Q - mu[:, None]
    if scale:
        s, zr = variable_scales(Qc, var_rows)
    else:
        s, zr = np.ones(len(var_rows) - 1), []
    s_rows = np.repeat(s, np.diff(np.asarray(var_rows)))
    Qs = apply_statistics(Q, mu, s_rows)
    return mu, s, Qs, zr


LIFT_COPY, LIFT_PRODUCT, LIFT_RECIPROCAL = 0, 1, 2


def lift(Q, n_cells, spec):
    """Lifting transformation (Sec. 3.3: new variables that expose polynomial
    structure, applied point by point before centering).

    Q holds the input variables as consecutive blocks of n_cells rows (one
    row per cell, one column per snapshot).  spec lists the output variables
    in order, each (op, a, b): LIFT_COPY -> variable a; LIFT_PRODUCT ->
    variable a times variable b; LIFT_RECIPROCAL -> 1 / variable a.  Returns
    the lifted snapshots, len(spec) blocks of n_cells rows.
    """
    Q = np.asarray(Q, dtype=np.float64)
    k = Q.shape[1]
    nv = Q.shape[0] // n_cells
    if nv * n_cells != Q.shape[0]:
        raise ValueError("Q must hold whole blocks of n_cells rows")
    out = np.empty((len(spec) * n_cells, k))
    for j, (op, a, b) in enumerate(spec):
        if not (0 <= a < nv and (op != LIFT_PRODUCT or 0 <= b < nv)):
            raise ValueError(f"lifting output {j} names a variable outside [0, {nv})")
        va = Q[a * n_cells:(a + 1) * n_cells, :]
        if op == LIFT_COPY:
            y = va.copy()
        elif op == LIFT_PRODUCT:
            y = va * Q[b * n_cells:(b + 1) * n_cells, :]
        elif op == LIFT_RECIPROCAL:
            with np.errstate(divide="ignore"):
                y = 1.0 / va
        else:
            raise ValueError(f"unknown lifting op {op}")
        out[j * n_cells:(j + 1) * n_cells, :] = y
    return out


# ---------------------------------------------------------------------------
# Step III (Sec. 3.4): Gram matrix, eigenpairs, reduced data
# ---------------------------------------------------------------------------

def gram(Qs):
    """D = Qs^T Qs (Eq. (5)); the lower triangle is computed, then mirrored."""
    D = Qs.T @ Qs
    L = np.tril(D)
    return L + np.tril(L, -1).T


def fix_signs(U):
    """Fix the sign of each eigenvector (Eq. (6) defines them only up to sign).

    READING: the entry of largest magnitude is made positive (lowest index on
    an exact tie).  If the two largest magnitudes agree to 1e-8 relative but
    carry opposite signs, the sign of sum_t (t+1) u_t decides instead.
    """
    U = np.array(U, dtype=np.float64, copy=True)
    k = U.shape[0]
    w = np.arange(1, k + 1, dtype=np.float64)
    for j in range(U.shape[1]):
        u = U[:, j]
        a = np.abs(u)
        i1 = int(np.argmax(a))            # lowest index among maxima
        sgn = 1.0 if u[i1] >= 0 else -1.0
        if k > 1:
            a2 = a.copy()
            a2[i1] = -1.0
            i2 = int(np.argmax(a2))
            if (a[i1] - a[i2]) <= 1e-8 * a[i1] and u[i1] * u[i2] < 0:
                m = float(np.dot(w, u))
                sgn = 1.0 if m >= 0 else -1.0
        U[:, j] = sgn * u
    return U


def eig_desc(D):
    """Eigenpairs of the symmetric Gram matrix, eigenvalues in descending
    order (Sec. 3.4 requires lambda_1 >= ... >= lambda_k; the listing sorts
    eigh's output by decreasing value), eigenvector signs fixed."""
    lam, U = np.linalg.eigh(D)
    order = np.argsort(lam, kind="stable")[::-1]
    return lam[order], fix_signs(U[:, order])


def energy_rank(lam, tau):
    """Smallest r whose retained energy exceeds tau (Eq. (9); the listing uses
    a strict '>' and divides by the sum of all eigenvalues)."""
    e = np.cumsum(lam) / np.sum(lam)
    hit = np.nonzero(e > tau)[0]
    if hit.size == 0:
        return len(lam)
    return int(hit[0]) + 1


def reduce_basis_free(lam, U, r):
    """T_r = U_r Lambda_r^{-1/2} (below Eq. (8)) and Qhat = Lambda_r^{1/2} U_r^T.

    Qhat = T_r^T D (Eq. (8)) equals Lambda_r^{1/2} U_r^T exactly because
    D U_r = U_r Lambda_r (Eq. (6)); the second form is used (READING) and the
    first is checked as an invariant.

    READING: T_r needs lambda_r > 0; an eigenvalue at or below the rounding
    level of the spectrum, k * u * lambda_1, counts as zero and is rejected.
    """
    if r < 1 or r > len(lam):
        raise ValueError("r out of range")
    if not lam[r - 1] > len(lam) * np.finfo(np.float64).eps * lam[0]:
        raise ValueError("lambda_r is numerically zero: r exceeds the numerical rank of D")
    Ur = U[:, :r]
    Tr = Ur * (lam[:r] ** -0.5)[None, :]
    Qhat = (np.sqrt(lam[:r])[:, None]) * Ur.T
    return Tr, Qhat


def qhat_by_projection(Tr, D):
    """Qhat = T_r^T D (Eq. (8))."""
    return Tr.T @ D


# ---------------------------------------------------------------------------
# Step IV (Sec. 3.5): operator inference
# ---------------------------------------------------------------------------

def n_quad(r):
    """Number of non-redundant quadratic terms, r(r+1)/2 (Sec. 3.5)."""
    return r * (r + 1) // 2


def quad_pairs(r):
    """Index pairs (i, j), i <= j, in the column order of the non-redundant
    quadratic features: (0,0),(0,1),...,(0,r-1),(1,1),...,(r-1,r-1)."""
    return [(i, j) for i in range(r) for j in range(i, r)]


def quad_features(X):
    """Non-redundant entries of x kron x for every row x of X (K x r) -> K x s.

    Sec. 3.5: products x_i x_j with j >= i, grouped by i.
    """
    X = np.atleast_2d(X)
    K, r = X.shape
    out = np.empty((K, n_quad(r)))
    c = 0
    for i in range(r):
        for j in range(i, r):
            out[:, c] = X[:, i] * X[:, j]
            c += 1
    return out


def opinf_data(Qhat):
    """Data of the discrete OpInf problem (Eqs. (12)-(13)).

    Qhat_1 = columns 0..k-2, Qhat_2 = columns 1..k-1;
    Dhat = [Qhat_1^T | quad(Qhat_1^T) | 1]  ((k-1) x d, d = r + s + 1);
    returns (Dhat, G = Dhat^T Dhat, B = Dhat^T Qhat_2^T).
    """
    Q1t = Qhat[:, :-1].T
    Q2t = Qhat[:, 1:].T
    Dhat = np.concatenate([Q1t, quad_features(Q1t), np.ones((Q1t.shape[0], 1))], axis=1)
    return Dhat, Dhat.T @ Dhat, Dhat.T @ Q2t


def regularizer(r, beta1, beta2):
    """Diagonal Tikhonov term of Eq. (12): beta1 on the r linear and the
    constant columns, beta2 on the s quadratic columns (added as beta, not
    beta^2, as in the listing)."""
    s = n_quad(r)
    g = np.empty(r + s + 1)
    g[:r] = beta1
    g[r:r + s] = beta2
    g[r + s] = beta1
    return g


def split_operators(O, r):
    """O = [A | H | c] (r x d) -> (A, H, c) (Sec. 3.5)."""
    s = n_quad(r)
    return O[:, :r], O[:, r:r + s], O[:, r + s]


def solve_operators(G, B, r, beta1, beta2, method="lu"):
    """Regularized normal equations (G + diag(reg)) O^T = B (Sec. 3.5).

    method="lu": general solve as in the paper's listing; method="cholesky":
    Cholesky factorization plus two triangular solves (used to measure how far
    two correct float64 solvers drift apart on an ill-conditioned system).
    Returns O (r x d).
    """
    M = G + np.diag(regularizer(r, beta1, beta2))
    if method == "lu":
        X = np.linalg.solve(M, B)
    elif method == "cholesky":
        import scipy.linalg as sla
        L = np.linalg.cholesky(M)
        Y = sla.solve_triangular(L, B, lower=True)
        X = sla.solve_triangular(L.T, Y, lower=False)
    else:
        raise ValueError(method)
    return X.T


def rollout(O, r, q0, n_states):
    """Iterate the discrete quadratic ROM of Eq. (11) for n_states states,
    q0 included (READING: an N-state rollout makes N-1 updates)."""
    A, H, c = split_operators(O, r)
    Qt = np.empty((r, n_states))
    Qt[:, 0] = q0
    with np.errstate(all="ignore"):
        for t in range(n_states - 1):
            x = Qt[:, t]
            Qt[:, t + 1] = A @ x + H @ quad_features(x[None, :])[0] + c
    return Qt


def train_error(Qtilde, Qhat, k_train):
    """max over t < k_train of ||qtilde_t - qhat_t||_2 / ||qhat_t||_2 (Sec. 3.5)."""
    diff = Qtilde[:, :k_train] - Qhat[:, :k_train]
    with np.errstate(all="ignore"):
        rel = np.sqrt(np.sum(diff ** 2, axis=0) / np.sum(Qhat[:, :k_train] ** 2, axis=0))
    return float(np.max(rel))


def growth_ratio(Qtilde, Qhat):
    """Largest deviation of the rollout from the temporal mean of the training
    data, over the whole horizon and all modes, divided by the same quantity
    for the training data (Sec. 3.5)."""
    m = np.mean(Qhat, axis=1)
    with np.errstate(all="ignore"):
        return float(np.max(np.abs(Qtilde - m[:, None])) / np.max(np.abs(Qhat - m[:, None])))


def score(Qtilde, Qhat, k_train, max_growth):
    """(finite, train_err, growth, passed) for one rollout (Sec. 3.5).

    READING: any non-finite value rejects the pair (the listing tests NaN;
    an Inf fails the growth bound anyway).  Growth must be strictly below
    max_growth.
    """
    finite = bool(np.all(np.isfinite(Qtilde)))
    if not finite:
        return False, float("nan"), float("nan"), False
    te = train_error(Qtilde, Qhat, k_train)
    g = growth_ratio(Qtilde, Qhat)
    return True, te, g, bool(g < max_growth)


def select_best(train_errs, passed):
    """Index of the smallest training error among passing candidates, the
    first in candidate order on ties; -1 if none passes (Sec. 3.5)."""
    best, best_e = -1, None
    for i, (e, p) in enumerate(zip(train_errs, passed)):
        if p and (best_e is None or e < best_e):
            best, best_e = i, e
    return best


def sweep(Qhat_full, r_list, beta1s, beta2s, n_states, max_growth=1.2,
          keep_traj=False):
    """Grid search of Sec. 3.5 over (r, beta1, beta2): beta1 outer, beta2
    inner (itertools.product order), Qhat at r = first r rows of Qhat_full.

    Returns a dict of per-item arrays plus the best item index per r.
    """
    k = Qhat_full.shape[1]
    out = {"r": [], "beta1": [], "beta2": [], "O": [], "finite": [],
           "train_err": [], "growth": [], "passed": [], "traj": [], "best": []}
    for r in r_list:
        Qhat = Qhat_full[:r, :]
        _, G, B = opinf_data(Qhat)
        errs, oks = [], []
        for b1 in beta1s:
            for b2 in beta2s:
                O = solve_operators(G, B, r, b1, b2)
                Qt = rollout(O, r, Qhat[:, 0], n_states)
                fin, te, g, ok = score(Qt, Qhat, k, max_growth)
                for key, val in (("r", r), ("beta1", b1), ("beta2", b2), ("O", O),
                                 ("finite", fin), ("train_err", te), ("growth", g),
                                 ("passed", ok)):
                    out[key].append(val)
                if keep_traj:
                    out["traj"].append(Qt)
                errs.append(te)
                oks.append(ok)
        out["best"].append(select_best(errs, oks))
    return out


# ---------------------------------------------------------------------------
# Step V (Sec. 3.6): postprocessing of the reduced solution
# ---------------------------------------------------------------------------

def basis_rows(Qs, Tr, rows):
    """Rows of the rank-r POD basis, V_r[rows] = Qs[rows] T_r (Eq. (7) with
    the method of snapshots: V_r = Qs T_r), from the transformed snapshots
    Qs of Step II; the basis itself is never formed."""
    return np.asarray(Qs)[np.asarray(rows, dtype=np.int64), :] @ Tr


def postprocess(Q, mu, s, var_rows, Tr, rows, Qtilde):
    """Step V: the reduced solution Qtilde (r x N) mapped back to the original
    coordinates at the given rows (Sec. 3.6): V_r[rows] Qtilde, then the
    inverse of Step II's transformation, x = s_v * y + mu (the listing adds
    the temporal mean; the scale factor undoes max-abs scaling).

    Returns (Vrows (m x r), prediction (m x N))."""
    rows = np.asarray(rows, dtype=np.int64)
    s_rows = np.repeat(np.asarray(s, dtype=np.float64), np.diff(np.asarray(var_rows)))
    # Step II's transform of the requested rows only (row by row, as for Qs)
    Qs_sel = apply_statistics(np.asarray(Q)[rows, :], np.asarray(mu)[rows], s_rows[rows])
    V = basis_rows(Qs_sel, Tr, np.arange(len(rows)))
    pred = s_rows[rows][:, None] * (V @ Qtilde) + np.asarray(mu)[rows][:, None]
    return V, pred


def pipeline(Q, var_rows, r, beta1, beta2, n_states, center=True, scale=True,
             max_growth=1.2):
    """Steps II-IV for one regularization pair: returns every intermediate."""
    mu, s, Qs, zr = preprocess(Q, var_rows, center, scale)
    D = gram(Qs)
    lam, U = eig_desc(D)
    Tr, Qhat = reduce_basis_free(lam, U, r)
    Dhat, G, B = opinf_data(Qhat)
    O = solve_operators(G, B, r, beta1, beta2)
    Qt = rollout(O, r, Qhat[:, 0], n_states)
    fin, te, g, ok = score(Qt, Qhat, Qhat.shape[1], max_growth)
    return dict(mu=mu, s=s, Qs=Qs, zero_range=zr, D=D, lam=lam, U=U, Tr=Tr,
                Qhat=Qhat, Dhat=Dhat, G=G, B=B, O=O, traj=Qt, finite=fin,
                train_err=te, growth=g, passed=ok)
