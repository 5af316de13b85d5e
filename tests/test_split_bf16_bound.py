"""The error bound of the three-term split-bf16 products, checked on the CPU by emulation (no GPU).

The GPU tests of the split-bf16 path (tests/test_gpu_bf16x3.py) hold C' and the projected half-row
to a bound derived from the split: hi = bf16(x), lo = bf16(x - hi) (round to nearest even),
a b ~ hi_a hi_b + hi_a lo_b + lo_a hi_b, with |error| <= e3 |a b| per product,
e3 = 2 ub^2 (1 + ub) + ub^2 (1 + ub)^2 + ub^4, ub = 2^-8, plus FP32 accumulation of the 3 K
products (at most 3 K u32 of the sum of |a b|).  Here the split, the exact bf16 products and the
FP32 accumulation are emulated with numpy on seeded inputs (normal, log-uniform over 30 binades,
values next to powers of two), and the bound is compared with the emulated error against the
exact sum; the bound must hold everywhere and not be loose by more than a few hundred.
"""
import numpy as np
import pytest

UB = 2.0 ** -8
U32 = 2.0 ** -24
E3 = 2 * UB ** 2 * (1 + UB) + UB ** 2 * (1 + UB) ** 2 + UB ** 4


def bf16_rne(x: np.ndarray) -> np.ndarray:
    """FP32 -> bf16 (round to nearest even), returned as FP32 values."""
    u = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32)


def split(x: np.ndarray):
    hi = bf16_rne(x)
    lo = bf16_rne((x - hi).astype(np.float32))
    return hi, lo


def dot3(a: np.ndarray, b: np.ndarray) -> float:
    """sum_k (hi_a hi_b + hi_a lo_b + lo_a hi_b), each bf16 product exact, accumulated in FP32
    in the order lo hi, hi lo, hi hi per k."""
    ah, al = split(a)
    bh, bl = split(b)
    acc = np.float32(0.0)
    for k in range(a.size):
        for p in (al[k] * bh[k], ah[k] * bl[k], ah[k] * bh[k]):  # exact in FP32 (8 x 8 bits)
            acc = np.float32(acc + np.float32(p))
    return float(acc)


def inputs(kind: str, n: int, rng):
    if kind == "normal":
        return rng.standard_normal(n).astype(np.float32)
    if kind == "loguniform":
        return (rng.choice([-1.0, 1.0], n) * 2.0 ** rng.uniform(-15, 15, n)).astype(np.float32)
    # values next to powers of two, where bf16 rounding carries over into the exponent
    e = rng.integers(-10, 10, n)
    return (2.0 ** e * (1.0 - rng.uniform(0, 2 ** -7, n))).astype(np.float32)


def test_split_represents_to_2_pow_minus_16():
    rng = np.random.default_rng(0)
    x = np.concatenate([inputs(k, 4000, rng) for k in ("normal", "loguniform", "pow2")])
    hi, lo = split(x)
    xd = x.astype(np.float64)
    assert np.all(np.abs(xd - hi - lo) <= UB ** 2 * np.abs(xd))
    assert np.all(np.abs(lo) <= UB * (1 + UB) * np.abs(xd))
    # the lo part is really needed: hi alone misses by up to 2^-9
    assert np.max(np.abs(xd - hi) / np.abs(xd)) > 2.0 ** -10


@pytest.mark.parametrize("kind", ["normal", "loguniform", "pow2"])
@pytest.mark.parametrize("n", [1, 37, 400])
def test_split_products_within_the_bound(kind, n):
    rng = np.random.default_rng(n + len(kind))
    worst = 0.0
    for _ in range(20):
        a, b = inputs(kind, n, rng), inputs(kind, n, rng)
        exact = float(np.dot(a.astype(np.float64), b.astype(np.float64)))
        absum = float(np.dot(np.abs(a.astype(np.float64)), np.abs(b.astype(np.float64))))
        err = abs(dot3(a, b) - exact)
        bound = (E3 + 3 * n * U32) * absum
        assert err <= bound, (err, bound)
        worst = max(worst, err / bound)
    assert worst > 1e-3  # the bound is not vacuous
