"""CPU emulation of the int8 Gram form I8X6 from its definition (shared by
the CPU bound tests and the GPU parity tests; no kernel code).

Column j of the transformed data x is scaled by 127 / a_j, a_j = max_i
|x_ij|, and split in radix 254 with round-half-to-even at every step:
xs = t1 + t2 / 254 + t3 / 254^2 + d.  The Gram keeps the six slice products
of weight at most 254^-2, summed exactly per level (integer-valued float64
sums stay below 2^53 at these sizes) and combined in float64:
D ~ a_j a_l / 127^2 (L0 + (L1 + L2 / 254) / 254)."""
import numpy as np

RADIX = 254.0
TOP = 127.0


def split3(xs):
    """The three slices of xs in [-127, 127] (round half to even)."""
    t1 = np.rint(xs)
    e = (xs - t1) * RADIX
    t2 = np.rint(e)
    t3 = np.rint((e - t2) * RADIX)
    return t1, t2, t3


def levels(t, u):
    """L0, L1, L2 of the slice triples t (rows x j) and u (rows x l)."""
    L0 = t[0].T @ u[0]
    L1 = t[0].T @ u[1] + t[1].T @ u[0]
    L2 = t[0].T @ u[2] + t[1].T @ u[1] + t[2].T @ u[0]
    return L0, L1, L2


def i8_gram(x, drop_level=None, global_scale=False):
    """Emulated I8X6 Gram of the float64 matrix x (rows x columns).  The two
    keyword arguments plant mistakes for the tests that show the derived
    bound catches them: a dropped level, one max-abs for all columns."""
    a = np.max(np.abs(x), axis=0)
    if global_scale:
        a = np.full_like(a, np.max(a))
    sc = np.where(a > 0, TOP / np.where(a > 0, a, 1.0), 0.0)
    t = split3(x * sc[None, :])
    for s in t:
        assert np.max(np.abs(s)) <= TOP
    L0, L1, L2 = levels(t, t)
    if drop_level == 1:
        L1 = np.zeros_like(L1)
    if drop_level == 2:
        L2 = np.zeros_like(L2)
    return ((L2 / RADIX + L1) / RADIX + L0) * np.outer(a, a) / TOP ** 2


def i8_emulate(Q, mean, scale, var_rows):
    """The form's arithmetic on float32 data Q: the float64 transform
    (q - mean) / scale per variable, then i8_gram.  Returns (D, x)."""
    n, k = Q.shape
    rinv = np.empty(n)
    for v in range(len(var_rows) - 1):
        rinv[var_rows[v]:var_rows[v + 1]] = 1.0 / scale[v]
    x = (Q.astype(np.float64) - mean[:, None]) * rinv[:, None]
    return i8_gram(x), x
