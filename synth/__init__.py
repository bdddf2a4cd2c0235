"""Seeded synthetic snapshot generators.

These produce the *inputs* of the reduction: snapshot matrices Q (n rows =
degrees of freedom, k columns = time instants, row-major, each state variable a
contiguous row block as in the data layout of the paper's Sec. 3.2) and, for the
reduced-space workloads, ground-truth trajectories.  Nothing here performs a
step of the reduction method itself (no centering, Gram, eigensolve, operator
inference or rollout); both the HIP path and the CPU oracle consume the same
bytes produced here.

Two families stand in for the paper's cylinder-wake dataset (Sec. 2.2), which
is not available:

* ``c1_*``: a ground-truth discrete quadratic system (the form of Eq. (11)) of
  size 10, lifted to 8192 rows by a random orthonormal basis, plus noise.
* ``c2_*``: travelling and standing waves on a periodic 1-D grid with several
  state variables, exactly orthonormal spatial and temporal modes and
  exponentially decaying singular values, plus noise.

Noise levels are given as variances (N(mean, variance)).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "QuadSystem",
    "c1_system",
    "c1_snapshots",
    "WaveModes",
    "c2_modes",
    "c2_snapshots",
    "quad_trajectory",
    "logspace_points",
    "mlp_init",
    "perturbed_states",
]


# ---------------------------------------------------------------------------
# Family 1: lifted ground-truth quadratic system
# ---------------------------------------------------------------------------

@dataclass
class QuadSystem:
    A: np.ndarray      # r x r
    H: np.ndarray      # r x r^2, column j*r + l multiplies q_j * q_l
    c: np.ndarray      # r
    q: np.ndarray      # r x k trajectory, q[:, 0] = initial state
    seed_used: int


def quad_trajectory(A, H, c, q0, k):
    """Iterate q+ = A q + H (q kron q) + c for k states (q0 included)."""
    r = q0.shape[0]
    q = np.empty((r, k))
    q[:, 0] = q0
    for t in range(k - 1):
        x = q[:, t]
        q[:, t + 1] = A @ x + H @ np.kron(x, x) + c
    return q


def c1_system(seed: int = 1, r: int = 10, k: int = 600, rho: float = 0.98,
              h_fro: float = 0.05, c_var: float = 1e-3, q_bound: float = 10.0,
              max_tries: int = 50) -> QuadSystem:
    """Random stable quadratic system and its trajectory.

    A = rho * G / spectral_radius(G), G ~ N(0,1); H energy preserving,
    H[i, (j,l)] = T[i,j,l] - T[j,i,l] with T ~ N(0,1), scaled to ||H||_F = h_fro;
    c ~ N(0, c_var); q0 ~ N(0, 1).  A draw whose trajectory leaves
    |q|_inf <= q_bound is rejected and the seed advanced by 1000.
    """
    s = seed
    for _ in range(max_tries):
        rng = np.random.default_rng(s)
        G = rng.standard_normal((r, r))
        A = rho * G / np.max(np.abs(np.linalg.eigvals(G)))
        T = rng.standard_normal((r, r, r))
        H3 = T - T.transpose(1, 0, 2)
        H3 *= h_fro / np.linalg.norm(H3)
        H = H3.reshape(r, r * r)
        c = rng.standard_normal(r) * math.sqrt(c_var)
        q0 = rng.standard_normal(r)
        with np.errstate(all="ignore"):
            q = quad_trajectory(A, H, c, q0, k)
        if np.all(np.isfinite(q)) and np.max(np.abs(q)) <= q_bound:
            return QuadSystem(A, H, c, q, s)
        s += 1000
    raise RuntimeError("no bounded quadratic system found")


def c1_snapshots(seed: int = 1, n_per_var: int = 4096, nvars: int = 2,
                 r: int = 10, k: int = 600, noise_var: float = 1e-6,
                 system: QuadSystem | None = None):
    """Q = V q + N(0, noise_var): V is (nvars*n_per_var) x r orthonormal.

    Returns (Q, var_rows, system, V).  var_rows[v]..var_rows[v+1] are the rows
    of variable v.
    """
    if system is None:
        system = c1_system(seed=seed, r=r, k=k)
    n = nvars * n_per_var
    rng_lift = np.random.default_rng([seed, 1])
    V, _ = np.linalg.qr(rng_lift.standard_normal((n, r)))
    Q = V @ system.q
    if noise_var > 0:
        rng_noise = np.random.default_rng([seed, 2])
        Q += math.sqrt(noise_var) * rng_noise.standard_normal(Q.shape)
    var_rows = np.arange(nvars + 1, dtype=np.int64) * n_per_var
    return np.ascontiguousarray(Q), var_rows, system, V


# ---------------------------------------------------------------------------
# Family 2: travelling / standing waves with orthonormal modes
# ---------------------------------------------------------------------------

@dataclass
class WaveModes:
    nvars: int
    ncell: int
    k: int
    kappa: np.ndarray      # per mode integer wavenumber
    omega: np.ndarray      # per mode integer frequency
    sp_kind: np.ndarray    # 0: sin(2 pi kappa x), 1: cos(2 pi kappa x)
    tm_kind: np.ndarray    # 0: sin(2 pi omega t / k), 1: cos(...)
    weights: np.ndarray    # n_modes x nvars, rows of unit 2-norm
    sigma: np.ndarray      # n_modes, strictly decreasing
    amp: float             # a = sqrt(n k / sum sigma^2): signal RMS 1

    @property
    def n(self):
        return self.nvars * self.ncell

    @property
    def n_modes(self):
        return self.sigma.shape[0]

    def temporal(self, t: np.ndarray) -> np.ndarray:
        """Psi[t, i] = sqrt(2/k) * (sin|cos)(2 pi omega_i t / k)."""
        ph = 2.0 * np.pi * np.outer(t, self.omega) / self.k
        out = np.where(self.tm_kind[None, :] == 1, np.cos(ph), np.sin(ph))
        return math.sqrt(2.0 / self.k) * out

    def spatial(self, rows: np.ndarray) -> np.ndarray:
        """Phi[row, i] = w[i, v] * sqrt(2/ncell) * (sin|cos)(2 pi kappa_i j / ncell)."""
        v = rows // self.ncell
        j = rows % self.ncell
        ph = 2.0 * np.pi * np.outer(j, self.kappa) / self.ncell
        out = np.where(self.sp_kind[None, :] == 1, np.cos(ph), np.sin(ph))
        return math.sqrt(2.0 / self.ncell) * out * self.weights.T[v, :]


def c2_modes(nvars: int = 4, ncell: int = 1_000_000, k: int = 2000,
             n_modes: int = 200, n_pairs: int = 60, decay: float = 40.0,
             seed: int = 2) -> WaveModes:
    """Mode table: n_pairs travelling pairs (sin kx cos wt, cos kx sin wt)
    followed by standing waves sin kx sin wt; sigma_i = exp(-i/decay), i = 1..

    Each pair / standing wave gets its own integer wavenumber (0 < kappa <
    ncell/2) and frequency (0 < omega < k/2), so spatial and temporal modes are
    exactly orthonormal by discrete Fourier orthogonality and every temporal
    mode has zero mean.
    """
    assert 2 * n_pairs <= n_modes
    n_distinct = n_pairs + (n_modes - 2 * n_pairs)
    assert n_distinct < k // 2 and n_distinct < ncell // 2
    rng = np.random.default_rng([seed, 7])
    kap = rng.choice(np.arange(1, (ncell + 1) // 2), size=n_distinct, replace=False)
    omg = rng.choice(np.arange(1, (k + 1) // 2), size=n_distinct, replace=False)
    kappa = np.empty(n_modes, dtype=np.int64)
    omega = np.empty(n_modes, dtype=np.int64)
    sp = np.empty(n_modes, dtype=np.int64)
    tm = np.empty(n_modes, dtype=np.int64)
    for m in range(n_pairs):
        kappa[2 * m:2 * m + 2] = kap[m]
        omega[2 * m:2 * m + 2] = omg[m]
        sp[2 * m], tm[2 * m] = 0, 1          # sin(kx) cos(wt)
        sp[2 * m + 1], tm[2 * m + 1] = 1, 0  # cos(kx) sin(wt)
    for i in range(2 * n_pairs, n_modes):
        d = n_pairs + (i - 2 * n_pairs)
        kappa[i], omega[i], sp[i], tm[i] = kap[d], omg[d], 0, 0
    w = rng.standard_normal((n_modes, nvars)) + 0.5
    w /= np.linalg.norm(w, axis=1, keepdims=True)
    sigma = np.exp(-np.arange(1, n_modes + 1) / decay)
    amp = math.sqrt(nvars * ncell * k / np.sum(sigma ** 2))
    return WaveModes(nvars, ncell, k, kappa, omega, sp, tm, w, sigma, amp)


def c2_snapshots(modes: WaveModes, noise_var: float = 1e-8, seed: int = 2,
                 device="cpu", t0: float = 0, chunk_rows: int = 1 << 18,
                 out=None):
    """Q = a * Phi diag(sigma) Psi^T + N(0, noise_var), float64, n x k.

    Built with torch on ``device`` (CPU for small cases, the GPU for the
    full-size ones: the GPU copy is the input both sides read).  ``t0`` shifts
    the time window (t = t0 .. t0+k-1) for held-out snapshots.
    """
    import torch

    n, k = modes.n, modes.k
    Q = out if out is not None else torch.empty((n, k), dtype=torch.float64, device=device)
    assert Q.shape == (n, k) and Q.dtype == torch.float64 and Q.is_contiguous()
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    psi = torch.from_numpy(modes.temporal(np.arange(t0, t0 + k))).to(device)
    coef = torch.from_numpy(modes.amp * modes.sigma).to(device)
    kap = torch.from_numpy(modes.kappa.astype(np.float64)).to(device)
    cosm = torch.from_numpy(modes.sp_kind == 1).to(device)
    wts = torch.from_numpy(modes.weights.T.copy()).to(device)   # nvars x n_modes
    std = math.sqrt(noise_var)
    for r0 in range(0, n, chunk_rows):
        r1 = min(n, r0 + chunk_rows)
        rows = torch.arange(r0, r1, device=device, dtype=torch.int64)
        jj = (rows % modes.ncell).to(torch.float64)
        ph = (2.0 * math.pi / modes.ncell) * torch.outer(jj, kap)
        phi = torch.where(cosm[None, :], torch.cos(ph), torch.sin(ph))
        phi *= math.sqrt(2.0 / modes.ncell) * wts[rows // modes.ncell]
        blk = Q[r0:r1]
        if std > 0:
            blk.normal_(0.0, std, generator=gen)
        else:
            blk.zero_()
        blk.addmm_(phi * coef, psi.T)
    return Q


def logspace_points(lo_exp: float, hi_exp: float, num: int) -> np.ndarray:
    """num points 10**e, e evenly spaced on [lo_exp, hi_exp], endpoints included."""
    if num == 1:
        return np.array([10.0 ** lo_exp])
    return np.array([10.0 ** (lo_exp + (hi_exp - lo_exp) * i / (num - 1)) for i in range(num)])


def mlp_init(r: int, hidden: int = 128, seed: int = 5) -> np.ndarray:
    """Initial closure parameters (float32, packed [W1|b1|W2|b2|W3|b3]):
    weights U(-1/sqrt(fan_in), 1/sqrt(fan_in)), biases zero."""
    rng = np.random.default_rng([seed, 11])
    parts = []
    for fan_out, fan_in in ((hidden, r), (hidden, hidden), (r, hidden)):
        b = 1.0 / math.sqrt(fan_in)
        parts.append(rng.uniform(-b, b, size=fan_out * fan_in))
        parts.append(np.zeros(fan_out))
    return np.concatenate(parts).astype(np.float32)


def perturbed_states(q0: np.ndarray, M: int, std: float = 0.05, seed: int = 5) -> np.ndarray:
    """M copies of q0 plus N(0, std^2) noise (M x r)."""
    rng = np.random.default_rng([seed, 13])
    return q0[None, :] + std * rng.standard_normal((M, q0.shape[0]))


def duffing_trajectory(q0, k: int, h: float = 0.05, beta: float = 1.0, coupling: float = 0.2) -> np.ndarray:
    """Two coupled oscillators with cubic stiffness, x'' = -w x - beta x^3 +
    coupling (x_other - x) (w = 1 and 1.3), stepped by symplectic Euler with
    step h: state (x1, v1, x2, v2), k states including q0 (4 x k)."""
    Q = np.empty((4, k))
    Q[:, 0] = q0
    for t in range(k - 1):
        x1, v1, x2, v2 = Q[:, t]
        v1n = v1 + h * (-x1 - beta * x1 ** 3 + coupling * (x2 - x1))
        v2n = v2 + h * (-1.3 * x2 - beta * x2 ** 3 + coupling * (x1 - x2))
        Q[:, t + 1] = (x1 + h * v1n, v1n, x2 + h * v2n, v2n)
    return Q


def duffing_snapshots(seed: int = 9, n_per_var: int = 2048, nvars: int = 2, k: int = 2000,
                      q0=(1.2, 0.0, -0.8, 0.3), q0_test=(0.9, 0.4, -1.0, -0.2), noise_var: float = 1e-10):
    """Training and held-out snapshots of the cubic oscillators, lifted by one
    random orthonormal basis V ((nvars * n_per_var) x 4) plus N(0, noise_var):
    returns (Q_train, Q_test, var_rows, q_train, q_test)."""
    rng = np.random.default_rng([seed, 17])
    n = nvars * n_per_var
    V, _ = np.linalg.qr(rng.standard_normal((n, 4)))
    qa = duffing_trajectory(np.asarray(q0, dtype=float), k)
    qb = duffing_trajectory(np.asarray(q0_test, dtype=float), k)
    std = math.sqrt(noise_var)
    Qa = V @ qa + std * rng.standard_normal((n, k))
    Qb = V @ qb + std * rng.standard_normal((n, k))
    var_rows = np.arange(nvars + 1) * n_per_var
    return Qa, Qb, var_rows, qa, qb
