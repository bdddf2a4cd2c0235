"""CPU pins of the error bound that the GPU parity tests of the int8 Gram form
I8X6 rely on (Step III Gram, Eq. (5), in fixed-point int8 slices).

The derivation (also in the GPU test's header): with xs = x 127 / a scaled
into [-127, 127] and split as t1 + t2 / 254 + t3 / 254^2 + d, the kept
products of one row differ from x_j x_l by the dropped slice products and
the d terms, at most 3.95e-3 in units of a_j a_l / 127^2; summed exactly over
n rows that is |dD_jl| <= n 2.45e-7 a_j a_l, used as 2.5e-7.  These tests
check the per-product constant by dense sampling (it holds, and a value
just off a half unit loses within 3% of it), the slice ranges and the reconstruction, the
bound on data whose columns span twelve decades, and that planted mistakes
(a dropped level, one max-abs for all columns) exceed it, so the GPU tests'
bound can tell a correct kernel from those mistakes.  The last test pins
the splits of the two bfloat16 forms that their GPU tolerances rest on.
CPU only."""
import numpy as np

from lowp_emu import RADIX, TOP, i8_gram, split3

PER_PRODUCT = 3.95e-3      # dropped part of one product, units of (a / 127)^2
I8_ROW = 2.5e-7            # per row, units of a_j a_l (PER_PRODUCT / 127^2 = 2.449e-7)


def kept(tx, ty):
    """The kept part of the product of two split values (elementwise)."""
    return (tx[0] * ty[0] + (tx[0] * ty[1] + tx[1] * ty[0]) / RADIX
            + (tx[0] * ty[2] + tx[1] * ty[1] + tx[2] * ty[0]) / RADIX ** 2)


def test_slices_in_range_and_reconstruct():
    rng = np.random.default_rng(0)
    edge = np.array([-127.0, 127.0, 0.0, 126.5, -126.5, 0.5, -0.5, 126.99999, 1e-300, -1e-12])
    xs = np.concatenate([rng.uniform(-127.0, 127.0, 200_000), edge])
    t1, t2, t3 = split3(xs)
    for t in (t1, t2, t3):
        assert np.max(np.abs(t)) <= TOP
        assert np.array_equal(t, np.round(t))
    d = xs - (t1 + t2 / RADIX + t3 / RADIX ** 2)
    assert np.max(np.abs(d)) <= 0.5 / RADIX ** 2 * (1 + 1e-9)
    assert np.array_equal(split3(np.array([127.0]))[0], [127.0])


def worst_value():
    """The value in [0, 127] whose square loses the most to the dropped
    terms, and that loss.  The largest losses sit just off a half unit,
    where t2 and t3 reach +-127: the search covers m + 0.5 +- delta for
    every m and delta up to 2 / 254 in steps of 1e-7."""
    m = np.arange(0.0, TOP)
    dl = np.linspace(0.0, 2.0 / RADIX, 20001)
    v = np.concatenate([(m[:, None] + 0.5 + dl[None, :]).ravel(), (m[:, None] + 0.5 - dl[None, :]).ravel()])
    v = v[v <= TOP]
    t = split3(v)
    err = np.abs(v * v - kept(t, t))
    i = int(np.argmax(err))
    return float(v[i]), float(err[i])


def test_per_product_constant_holds_and_is_tight():
    rng = np.random.default_rng(1)
    x = rng.uniform(-TOP, TOP, 1_000_000)
    y = rng.uniform(-TOP, TOP, 1_000_000)
    assert float(np.max(np.abs(x * y - kept(split3(x), split3(y))))) <= PER_PRODUCT
    v, worst = worst_value()
    assert worst <= PER_PRODUCT
    # the constant is within 3% of a loss that occurs
    assert worst >= 0.97 * PER_PRODUCT, (v, worst)
    assert PER_PRODUCT / TOP ** 2 <= I8_ROW


def wide_columns(n, k, seed):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((n, k)) * np.geomspace(1e-6, 1e6, k)[None, :]
    x[:, 3] = np.abs(x[:, 3])           # a one-signed column: its errors add coherently
    x[:, 4] = 7.0 * np.geomspace(1e-6, 1e6, k)[4]   # a constant column
    return x


def excess(D, x):
    a = np.max(np.abs(x), axis=0)
    den = x.shape[0] * np.outer(a, a)
    return float(np.max(np.abs(D - x.T @ x) / den))


def test_emulated_form_within_bound_on_columns_of_twelve_decades():
    for n, k, seed in ((3000, 24, 2), (64, 9, 3), (1, 5, 4)):
        x = wide_columns(n, k, seed)
        D = i8_gram(x)
        assert np.array_equal(D, D.T)
        assert excess(D, x) <= I8_ROW


def test_worst_case_rows_reach_the_bound():
    """Every row but one at the worst value (the remaining row holds the
    column's max-abs 127, so the scaling is 1): each row loses the same
    amount with the same sign, and the diagonal entry's error comes within
    10% of the bound, so the bound cannot be tightened much."""
    v, _ = worst_value()
    x = np.full((5000, 3), v)
    x[0, :] = TOP
    x[:, 1] *= -1.0
    x[1:, 2] = 0.5 * v
    D = i8_gram(x)
    e = excess(D, x)
    assert e <= I8_ROW
    a = np.max(np.abs(x), axis=0)
    e00 = abs(D[0, 0] - x[:, 0] @ x[:, 0]) / (x.shape[0] * a[0] * a[0])
    assert e00 >= 0.9 * I8_ROW, e00


def test_planted_mistakes_exceed_the_bound():
    x = wide_columns(3000, 24, 2)
    assert excess(i8_gram(x, drop_level=2), x) > 4 * I8_ROW
    assert excess(i8_gram(x, drop_level=1), x) > 4 * I8_ROW
    # one max-abs for all columns loses the small columns entirely
    assert excess(i8_gram(x, global_scale=True), x) > 4 * I8_ROW


def bf16_rn(x):
    """float32 -> nearest bfloat16 (ties to even) -> float32, by torch's CPU
    conversion."""
    import torch
    return torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()


def test_bfloat16_splits_of_the_two_split_forms():
    """The split-bfloat16 forms write a float32 value x as hi = bf16(x),
    lo = bf16(x - hi) (BF16X3) and further mid, lo (BF16X6), each
    difference exact in float32.  Their GPU tolerances rest on
    |x - hi - lo| <= 2^-16 |x| and on the three parts holding x with an error
    of at most 2^-24 |x|; while all parts are normal float32 values the
    three parts are exact, which this pins together with the two-part bound,
    on random values over the whole exponent range and on low-bit patterns
    at rounding ties."""
    rng = np.random.default_rng(9)
    x = (rng.standard_normal(400_000) * np.exp2(rng.integers(-100, 100, 400_000))).astype(np.float32)
    bits = rng.integers(0, 1 << 23, 20_000).astype(np.uint32)
    ties = ((bits & ~np.uint32(0xFFFF)) | np.uint32(0x8000) | (np.uint32(127) << 23)).view(np.float32)
    x = np.concatenate([x, ties, -ties, ties * np.float32(2.0 ** -60)])
    hi = bf16_rn(x)
    r1 = x - hi
    assert np.array_equal(r1.astype(np.float64), x.astype(np.float64) - hi.astype(np.float64))
    lo2 = bf16_rn(r1)
    ax = np.abs(x.astype(np.float64))
    err2 = np.abs(x.astype(np.float64) - hi.astype(np.float64) - lo2.astype(np.float64))
    assert np.max(err2 / ax) <= 2.0 ** -16
    mid = bf16_rn(r1)
    r2 = r1 - mid
    lo3 = bf16_rn(r2)
    err3 = x.astype(np.float64) - hi.astype(np.float64) - mid.astype(np.float64) - lo3.astype(np.float64)
    # while the last part stays a normal float32 (|x| >= 2^-110; the data
    # the forms see are scaled to at most 1, and values below 2^-110 of a
    # column's max-abs do not move its Gram entries)
    big = ax >= 2.0 ** -110
    assert np.count_nonzero(~big) > 0
    assert np.max(np.abs(err3[big]) / ax[big]) <= 2.0 ** -24
    assert np.all(err3[big] == 0.0)
    # the two-part remainder is not vacuous: it reaches ~2^-17 relative
    assert np.max(err2 / ax) >= 2.0 ** -18
