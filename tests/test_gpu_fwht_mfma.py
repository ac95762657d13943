"""Split-FP16 matrix-core Walsh-Hadamard transform against the oracle's FP64
FWHT: normwise error within the FP32 transform tolerance, over sizes that
exercise a leftover of 1-3 index bits, one pass and two passes, and data
spanning a wide dynamic range (the per-stage power-of-two scaling)."""
import numpy as np
import pytest
import torch

import paper_2502_14256_amd as ldk
from ldk_dev import record, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def orc():
    import oracle
    oracle.build(force=False)
    return oracle


@pytest.mark.parametrize("m", [0, 1, 2, 3, 4, 5, 7, 8, 11, 12, 13, 14, 16, 17, 20])
def test_fwht_split16_matches_oracle(orc, m):
    rng = np.random.default_rng(600 + m)
    B = 3 if m < 18 else 1
    x = (rng.standard_normal((B, 2**m)) * np.exp(rng.uniform(-8, 8, (B, 2**m)))).astype(np.float32)
    ref = orc.transform("dnet", x.astype(np.float64), precise=True)
    xd = torch.from_numpy(x).cuda()
    y = ldk.fwht_split16(xd).cpu().numpy()
    err = rel(y, ref)
    # the FP32 butterfly transform on the same data, for comparison
    e32 = rel(ldk.transform("dnet", xd).cpu().numpy(), ref)
    record(f"fwht_split16_m{m}", err=err, err_fp32_butterflies=e32)
    assert err < 2e-6, (err, e32)
    # in place
    ldk.fwht_split16(xd, out=xd)
    assert np.array_equal(xd.cpu().numpy(), y)


def test_fwht_split16_zero_and_tiny_rows():
    x = torch.zeros((2, 2**12), dtype=torch.float32, device="cuda")
    x[1, 5] = 1e-30  # far below the FP16 range: scaled up before the split
    y = ldk.fwht_split16(x).cpu().numpy()
    assert np.all(y[0] == 0)
    assert np.allclose(y[1], 1e-30 / 64 * np.where(np.array([bin(k & 5).count("1") % 2 for k in range(4096)]) == 1, -1, 1), rtol=1e-6, atol=0)
