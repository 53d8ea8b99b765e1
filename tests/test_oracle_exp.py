"""Pins of the oracle's binary32 exp (used in alpha = gamma exp(-d^2/beta^2), Sec. 3.3).

The exact value is the mathematical exp, taken from the C library in binary64.
"""
from concurrent.futures import ThreadPoolExecutor

import numpy as np


def _ulp32(y):
    # spacing of binary32 numbers in the binade of y (y > 0, normal)
    _, e = np.frexp(y)
    return np.ldexp(1.0, e - 24)


def test_exp32_exhaustive_within_2ulp(orc):
    """Every binary32 x in [-86, 0]: |E(x) - exp(x)| <= 2 ulp, E(x) <= 1."""
    lo_bits = np.uint32(0x80000000)           # -0.0
    hi_bits = np.float32(-86.0).view(np.uint32)
    total = int(hi_bits - lo_bits) + 1
    chunk = 1 << 24

    def check(start):
        bits = (np.arange(start, min(start + chunk, total), dtype=np.uint64)
                + int(lo_bits)).astype(np.uint32)
        x = bits.view(np.float32)
        y = orc.exp32(x).astype(np.float64)
        ex = np.exp(x.astype(np.float64))
        err = np.abs(y - ex) / _ulp32(ex)
        return float(err.max()), bool((y <= 1.0).all()), bool((y > 0.0).all())

    with ThreadPoolExecutor(8) as pool:
        res = list(pool.map(check, range(0, total, chunk)))
    worst = max(r[0] for r in res)
    assert all(r[1] for r in res)
    assert all(r[2] for r in res)
    assert worst <= 2.0, worst


def test_exp32_special_values(orc):
    x = np.array([0.0, -0.0, -1.0, -np.log(2.0), -86.0, -86.0001, -1000.0, np.nan, -np.inf],
                 np.float32)
    y = orc.exp32(x)
    assert y[0] == 1.0 and y[1] == 1.0
    assert abs(y[2] - np.exp(-1.0)) < 2e-7
    assert abs(y[3] - 0.5) < 1e-7
    assert y[4] > 0.0
    assert (y[5:] == 0.0).all()


def test_exp32_monotone_on_grid(orc):
    x = np.linspace(-86.0, 0.0, 2_000_001, dtype=np.float32)
    y = orc.exp32(x)
    assert (np.diff(y.astype(np.float64)) >= 0).all()
