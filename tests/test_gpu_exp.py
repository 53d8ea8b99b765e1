"""The device's binary32 exp (alpha = gamma exp(-d^2 / beta^2), Sec. 3.3)
against the oracle's, bit for bit, for every binary32 in [-86, 0].

Which candidates become samples depends on these bits (w_j > eps_w), so the
two implementations of the same operation sequence must agree exactly, not
only to within the oracle's pinned 2-ulp error."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu


def test_exp32_bitwise_equal_to_oracle_exhaustive():
    import torch
    from paper_2404_14044_amd import hashpoint as hp
    dev = torch.device("cuda:0")
    lo_bits = 0x80000000                            # -0.0
    hi_bits = int(np.float32(-86.0).view(np.uint32))  # -86.0
    total = hi_bits - lo_bits + 1
    chunk = 1 << 24
    xg = torch.empty(chunk, dtype=torch.int32, device=dev)
    yg = torch.empty(chunk, dtype=torch.float32, device=dev)
    ramp = torch.arange(chunk, dtype=torch.int64, device=dev)
    checked = 0
    for start in range(0, total, chunk):
        n = min(chunk, total - start)
        # bit patterns lo_bits + start .. + n - 1 as int32 (two's complement)
        bits = (ramp[:n] + (lo_bits + start)).to(torch.int64)
        bits = torch.where(bits >= 1 << 31, bits - (1 << 32), bits).to(torch.int32)
        xg[:n].copy_(bits)
        x = xg[:n].view(torch.float32)
        hp.exp32_eval(x, out=yg[:n])
        y_dev = yg[:n].cpu().numpy()
        x_host = x.cpu().numpy()
        y_orc = oracle.exp32(x_host)
        if not np.array_equal(y_dev.view(np.uint32), y_orc.view(np.uint32)):
            bad = np.nonzero(y_dev.view(np.uint32) != y_orc.view(np.uint32))[0]
            i = int(bad[0])
            raise AssertionError(f"{bad.size} values differ, first x={x_host[i]!r}: "
                                 f"device {y_dev[i]!r}, oracle {y_orc[i]!r}")
        checked += n
    assert checked == total


def test_exp32_special_values_match_oracle():
    import torch
    from paper_2404_14044_amd import hashpoint as hp
    x = np.array([0.0, -0.0, -1e-45, -1e-38, -86.0, -86.00001, -87.0, -1e30, -np.inf, np.nan,
                  -0.34657359, -0.6931472, -88.72], np.float32)
    y = hp.exp32_eval(torch.from_numpy(x).to("cuda:0")).cpu().numpy()
    assert np.array_equal(y.view(np.uint32), oracle.exp32(x).view(np.uint32))
