"""Pins for the oracle's round-to-nearest-even conversions.

The storage and operand formats (fp32, fp16, bf16, fp8 e4m3fn) are fixed
by IEEE 754 and the OCP 8-bit floating point specification; the oracle's
conversions are written from those definitions and pinned here against
independent library conversions and exact rational rounding.
"""
from fractions import Fraction

import numpy as np
import pytest
import torch

import oracle


def _rand_doubles(rng, k, lo, hi):
    mag = np.exp2(rng.uniform(lo, hi, k))
    return mag * rng.choice([-1.0, 1.0], k)


def _ties(p, lo, hi):
    # midpoints between consecutive p-bit significands: exact ties
    out = []
    for e in range(lo, hi):
        for m in (1, 2, 3, 5, 2 ** (p - 1) - 1):
            out.append(float(Fraction(2 ** (p - 1) + m) * Fraction(2) ** (e - p + 1) + Fraction(2) ** (e - p)))
    return out


def test_fp16_matches_numpy():
    rng = np.random.default_rng(0)
    xs = np.concatenate([_rand_doubles(rng, 20000, -26, 16.5), _ties(11, -14, 15), [65519.99, 65520.0, 6e-8, 3e-8]])
    got = oracle.round_array(oracle.FMT_F16, xs)
    want = xs.astype(np.float16).astype(np.float64)
    assert np.array_equal(got, want)
    for v in xs[:2000]:
        y = oracle.round_fmt(oracle.FMT_F16, v)
        if np.isfinite(y):
            assert oracle.encode_fmt(oracle.FMT_F16, y) == int(np.float16(v).view(np.uint16))


def test_fp32_matches_numpy():
    rng = np.random.default_rng(1)
    xs = np.concatenate([_rand_doubles(rng, 20000, -150, 127), _ties(24, -126, 100)])
    got = oracle.round_array(oracle.FMT_F32, xs)
    want = xs.astype(np.float32).astype(np.float64)
    assert np.array_equal(got, want)


def _exact_rne(x, p, emin):
    # nearest of the two representable neighbours, ties to even, in rationals
    fx = Fraction(x)
    a = abs(fx)
    e = emin
    while Fraction(2) ** (e + 1) <= a:
        e += 1
    q = Fraction(2) ** (e - p + 1)
    lo = (a // q) * q
    hi = lo + q
    if a - lo < hi - a or (a - lo == hi - a and (lo / q) % 2 == 0):
        r = lo
    else:
        r = hi
    return float(r if fx > 0 else -r)


def test_bf16_matches_exact_rational_rounding():
    rng = np.random.default_rng(2)
    xs = np.concatenate([_rand_doubles(rng, 3000, -130, 120), _ties(8, -126, 100)])
    for v in xs:
        assert oracle.round_fmt(oracle.FMT_BF16, v) == _exact_rne(v, 8, -126)


def test_bf16_matches_torch_on_float32_inputs():
    rng = np.random.default_rng(3)
    xs = _rand_doubles(rng, 20000, -120, 120).astype(np.float32)  # no double rounding in torch
    want = torch.from_numpy(xs).to(torch.bfloat16).to(torch.float64).numpy()
    got = oracle.round_array(oracle.FMT_BF16, xs.astype(np.float64))
    assert np.array_equal(got, want)


def test_e4m3_matches_torch_in_range_and_saturates():
    rng = np.random.default_rng(4)
    xs = _rand_doubles(rng, 20000, -12, 8.8).astype(np.float32)
    xs = xs[np.abs(xs) < 448]
    want = torch.from_numpy(xs).to(torch.float8_e4m3fn).to(torch.float64).numpy()
    got = oracle.round_array(oracle.FMT_E4M3, xs.astype(np.float64))
    assert np.array_equal(got, want)
    assert oracle.round_fmt(oracle.FMT_E4M3, 1000.0) == 448.0
    assert oracle.round_fmt(oracle.FMT_E4M3, -463.9) == -448.0
    assert oracle.encode_fmt(oracle.FMT_E4M3, 448.0) == 0x7E
    for v in xs[:500]:
        y = oracle.round_fmt(oracle.FMT_E4M3, float(v))
        assert oracle.encode_fmt(oracle.FMT_E4M3, y) == int(torch.tensor([float(v)], dtype=torch.float32)
                                                            .to(torch.float8_e4m3fn).view(torch.uint8)[0])


@pytest.mark.parametrize("fmt", [oracle.FMT_F16, oracle.FMT_BF16, oracle.FMT_E4M3])
def test_power_of_two_scaling_commutes_with_rounding(fmt):
    # scaling by 2^e before rounding is exact while no value leaves the normal range
    rng = np.random.default_rng(5)
    xs = _rand_doubles(rng, 500, -3, 3)
    for v in xs:
        assert oracle.round_fmt(fmt, v * 4.0) == 4.0 * oracle.round_fmt(fmt, v)
