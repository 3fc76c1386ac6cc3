"""Host-side checks of the arithmetic behind the heavy-row Gram kernel: an fp32
value x splits exactly into three bfloat16 numbers h + m + l (h = x rounded to
nearest bfloat16, m = x - h rounded to nearest, l = x - h - m), and the six
products h h' + h m' + m h' + m m' + h l' + l h' of two split values reproduce
x x' to within 2^-23 |x x'| (the dropped m l' + l m' + l l', with |m| <= 2^-8
|x| and |l| <= 2^-16 |x|), with errors of both signs.  numpy emulation of the
kernel's operations; no GPU."""
import numpy as np

HI = np.uint32(0xFFFF0000)


def bf16_rne(x: np.ndarray) -> np.ndarray:
    """float32 -> nearest bfloat16 (ties to even), returned as float32: what
    v_cvt_pk_bf16_f32 computes for finite values."""
    u = x.astype(np.float32).view(np.uint32).astype(np.uint64)
    r = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return r.astype(np.uint32).view(np.float32)


def split3(x: np.ndarray):
    """The kernel's split, in float32: round, subtract, round, subtract."""
    x = x.astype(np.float32)
    h = bf16_rne(x)
    r1 = (x - h).astype(np.float32)
    m = bf16_rne(r1)
    l = (r1 - m).astype(np.float32)
    return h, m, l


def random_fp32(n, seed):
    rng = np.random.default_rng(seed)
    mant = rng.random(n) + 1.0
    expo = rng.integers(-60, 60, n)
    sign = rng.choice([-1.0, 1.0], n)
    return (sign * mant * np.exp2(expo)).astype(np.float32)


def test_split_is_exact_and_each_part_is_bf16():
    # (for |x| near the fp32 subnormal range the last part can itself be
    # subnormal with more than 8 bits; the kernel's truncation then drops
    # less than 2^-133 in absolute value: not exercised here)
    # (above 3.39e38 the rounding of h overflows to infinity; any Gram entry
    # overflows FP32 long before, at |x| near 1.8e19)
    x = np.concatenate([random_fp32(200000, 1), np.float32([0.0, -0.0, 1.0, -1.5, 3.3e38, 1e-30])])
    h, m, l = split3(x)
    # exact: the parts add up to x in exact (float64) arithmetic
    assert np.array_equal(h.astype(np.float64) + m.astype(np.float64) + l.astype(np.float64), x.astype(np.float64))
    # each part has a zero low half: it is a bfloat16 number, taken by truncation
    for part in (h, m, l):
        assert not np.any(part.view(np.uint32) & np.uint32(0xFFFF))
    # magnitudes decrease by a factor 2^8 per part
    ax = np.abs(x.astype(np.float64))
    assert np.all(np.abs(m) <= ax * 2.0 ** -8)
    assert np.all(np.abs(l) <= ax * 2.0 ** -16)
    # and l is exactly its own rounding
    assert np.array_equal(bf16_rne(l), l)


def test_six_products_within_2_pow_minus_23():
    x = random_fp32(100000, 2)
    y = random_fp32(100000, 3)
    hx, mx, lx = (p.astype(np.float64) for p in split3(x))
    hy, my, ly = (p.astype(np.float64) for p in split3(y))
    six = hx * hy + hx * my + mx * hy + mx * my + hx * ly + lx * hy
    exact = x.astype(np.float64) * y.astype(np.float64)
    rel = np.abs(six - exact) / np.abs(exact)
    assert rel.max() <= 2.0 ** -23
    # errors of both signs (no bias that long sums would accumulate), also on
    # squares (the Gram's diagonal)
    err = six - exact
    assert (err > 0).mean() > 0.3 and (err < 0).mean() > 0.3
    sq = hx * hx + 2 * hx * mx + mx * mx + 2 * hx * lx - x.astype(np.float64) ** 2
    assert (sq > 0).mean() > 0.2 and (sq < 0).mean() > 0.2
    # each bf16 x bf16 product is exact in float32 (8 + 8 significant bits)
    # where it lies in the normal float32 range
    for a, b in ((hx, hy), (hx, my), (mx, hy), (mx, my), (hx, ly), (lx, hy)):
        p = a * b
        ok = (np.abs(p) < 3e38) & (np.abs(p) >= 2.0 ** -126)
        assert np.array_equal(p[ok].astype(np.float32).astype(np.float64), p[ok])


def test_dropping_any_of_the_six_products_loses_accuracy():
    """The six are needed: without m m' (or h l' / l h') the error reaches
    2^-18 relative or more, far above FP32 rounding."""
    x = random_fp32(100000, 4)
    y = random_fp32(100000, 5)
    hx, mx, lx = (p.astype(np.float64) for p in split3(x))
    hy, my, ly = (p.astype(np.float64) for p in split3(y))
    exact = x.astype(np.float64) * y.astype(np.float64)
    terms = [hx * hy, hx * my, mx * hy, mx * my, hx * ly, lx * hy]
    for drop in range(6):
        approx = sum(t for k, t in enumerate(terms) if k != drop)
        rel = np.abs(approx - exact) / np.abs(exact)
        assert rel.max() > 2.0 ** -20
