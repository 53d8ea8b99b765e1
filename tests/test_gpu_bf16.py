"""The device's rounding to bfloat16, the operation the BF16 decoder applies
to every operand (R22: round to nearest, ties to even), against the oracle's
definition bit for bit: every non-negative finite binary32 value (all
exponents, subnormals and the largest values included), and every 7th
negative one."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu


def _check_range(lo_bits, hi_bits, step=1):
    import torch
    from paper_2404_14044_amd import hashpoint as hp
    dev = torch.device("cuda:0")
    chunk = 1 << 24
    ramp = torch.arange(chunk, dtype=torch.int64, device=dev) * step
    yg = torch.empty(chunk, dtype=torch.float32, device=dev)
    checked = 0
    start = lo_bits
    while start <= hi_bits:
        n = min(chunk, (hi_bits - start) // step + 1)
        bits = ramp[:n] + start
        bits = torch.where(bits >= 1 << 31, bits - (1 << 32), bits).to(torch.int32)
        x = bits.view(torch.float32)
        hp.bf16_eval(x, out=yg[:n])
        y_dev = yg[:n].cpu().numpy()
        x_host = x.cpu().numpy()
        y_orc = oracle.bf16_f32(x_host)
        if not np.array_equal(y_dev.view(np.uint32), y_orc.view(np.uint32)):
            bad = np.nonzero(y_dev.view(np.uint32) != y_orc.view(np.uint32))[0]
            i = int(bad[0])
            raise AssertionError(f"{bad.size} values differ, first x={x_host[i]!r} "
                                 f"({x_host[i:i + 1].view(np.uint32)[0]:#010x}): "
                                 f"device {y_dev[i]!r}, oracle {y_orc[i]!r}")
        checked += n
        start += n * step
    return checked


def test_bf16_rounding_bitwise_equal_to_oracle():
    # 0x00000000 .. 0x7F7FFFFF: zero, subnormals, every normal value
    assert _check_range(0x00000000, 0x7F7FFFFF) == 0x7F800000
    # negative values, every 7th bit pattern
    assert _check_range(0x80000000, 0xFF7FFFFF, step=7) > 300_000_000


def test_bf16_rounding_ties_and_limits():
    import torch
    from paper_2404_14044_amd import hashpoint as hp
    x = np.array([1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 1.0 + 2 ** -8 + 2 ** -23, -1.0 - 2 ** -8,
                  np.float32(3.3895314e38), np.finfo(np.float32).max, 1e-45, 2.9e-39, -0.0, 0.0],
                 np.float32)
    y = hp.bf16_eval(torch.from_numpy(x).to("cuda:0")).cpu().numpy()
    assert np.array_equal(y.view(np.uint32), oracle.bf16_f32(x).view(np.uint32))
    assert y[0] == 1.0 and y[1] == 1.0 + 2 ** -6 and y[2] == 1.0 + 2 ** -7
