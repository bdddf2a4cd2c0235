"""Operator checks shared by the GPU tests and the smoke run (the tolerance
lives here only).

For the regularized normal equations M X = B, M = G + diag(beta1, beta2,
beta1) (Sec. 3.5), d unknowns per right-hand side:
  * end to end (check_operators): the GPU forms G = Dhat^T Dhat and B itself
    with (k-1)-term sums, |dG| <= gamma_{k-1} |Dhat|^T |Dhat|, so
    ||dG||_F <= gamma_{k-1} trace(G) <= gamma_{k-1} sqrt(d) ||G||_F, and the
    Cholesky solve adds a backward error of order d u: the GPU solution's
    backward error on the oracle's own M, B is at most
    u ((k - 1) sqrt(d) + 10 d); its distance to the oracle's LU solution is
    within the first-order bound 2 kappa_2(M) max(eta_gpu, eta_oracle, u)
    (at least 1e-10);
  * solver only (check_solver_only): on the G and B that the GPU forms
    itself (the Gram kernel on the same data matrix E, the same bytes and
    leading dimension as the inference call), the GPU solution must agree
    with the oracle's LU solution to max(1e-10, 10 eps_self), where eps_self
    is the oracle's own spread between its LU and Cholesky solutions of the
    same system: two correct float64 solvers of one system differ by that
    much, and the GPU's solver may differ by ten times that.
"""
import numpy as np

import oracle as orc

U = 2.0 ** -53


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def eta_bound(k, d):
    return U * ((k - 1) * np.sqrt(d) + 10 * d)


def backward_error(M, B, O):
    X = O.T
    return float(np.linalg.norm(M @ X - B) / (np.linalg.norm(M) * np.linalg.norm(X) + np.linalg.norm(B)))


def check_operators(G, B, r, b1, b2, O_gpu, k, where=None):
    M = G + np.diag(orc.regularizer(r, b1, b2))
    O_ref = orc.solve_operators(G, B, r, b1, b2, method="lu")
    e_gpu, e_ref = backward_error(M, B, O_gpu), backward_error(M, B, O_ref)
    assert e_gpu <= eta_bound(k, M.shape[0]), (where, e_gpu)
    tol = max(1e-10, 2 * np.linalg.cond(M) * max(e_gpu, e_ref, U))
    assert rel(O_gpu, O_ref) <= tol, (where, rel(O_gpu, O_ref), tol)


def _qcol(i, j, rmax):
    return rmax + i * rmax - i * (i - 1) // 2 + (j - i)


def gpu_normal_equations(dp, Qhat, rmax):
    """The GPU's own G_E = E^T E for E = [Qhat_1^T | quad(Qhat_1^T) | 1 |
    Qhat_2^T] at rmax, laid out as the inference call lays it out ((k-1) x m,
    leading dimension m rounded up to even).  E's entries are single
    products (the same bits on both sides); G_E comes from the GPU's Gram
    kernel.  Returns G_E as a numpy array."""
    import torch
    Qh = np.asarray(Qhat)[:rmax]
    s = orc.n_quad(rmax)
    d = rmax + s + 1
    m = d + rmax
    lde = (m + 1) // 2 * 2
    Q1t, Q2t = Qh[:, :-1].T, Qh[:, 1:].T
    E = np.zeros((Q1t.shape[0], lde))
    E[:, :rmax] = Q1t
    E[:, rmax:rmax + s] = orc.quad_features(Q1t)
    E[:, rmax + s] = 1.0
    E[:, d:d + rmax] = Q2t
    Ed = torch.from_numpy(E).cuda()
    GE = dp.gram(Ed[:, :m])
    torch.cuda.synchronize()
    return GE.cpu().numpy()


def normal_equations_at(GE, r, rmax):
    """(G, B) of reduced size r as index submatrices of G_E at rmax."""
    s_max = orc.n_quad(rmax)
    dmax = rmax + s_max + 1
    cols = list(range(r)) + [_qcol(i, j, rmax) for i in range(r) for j in range(i, r)] + [rmax + s_max]
    rhs = [dmax + c for c in range(r)]
    return GE[np.ix_(cols, cols)], GE[np.ix_(cols, rhs)]


def check_solver_only(G, B, r, b1, b2, O_gpu, where=None, log=print):
    M = G + np.diag(orc.regularizer(r, b1, b2))
    O_lu = orc.solve_operators(G, B, r, b1, b2, method="lu")
    O_ch = orc.solve_operators(G, B, r, b1, b2, method="cholesky")
    eps_self = rel(O_ch, O_lu)
    diff = rel(O_gpu, O_lu)
    tol = max(1e-10, 10 * eps_self)
    if log:
        log(f"solver-only {where}: kappa2(M)={np.linalg.cond(M):.3e} diff={diff:.3e} eps_self={eps_self:.3e} "
            f"tol={tol:.3e}")
    assert diff <= tol, (where, diff, tol)
    return dict(diff=diff, eps_self=eps_self, tol=tol)
