"""Device layout conversion between element-major words and the limb-planar
layout: bit-exact against numpy's transpose, at sizes with ragged last tiles."""
import numpy as np
import pytest
import torch

from gpu_util import say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("limbs", [2, 3, 8, 12, 31, 32])
@pytest.mark.parametrize("n", [1, 255, 256, 257, 1000, 70001])
def test_pack_unpack_match_transpose(limbs, n):
    import paper_2501_07535_amd as moma
    rng = np.random.default_rng(limbs * 100003 + n)
    elems = rng.integers(0, 2**32, size=(n, limbs), dtype=np.uint64).astype(np.uint32)
    say(f"layout limbs={limbs} n={n}")
    d = torch.from_numpy(elems.view(np.int32)).to("cuda:0")
    planar = moma.pack(d)
    got = planar.cpu().numpy().view(np.uint32)
    assert got.shape == (limbs, n) and (got == elems.T).all()
    back = moma.unpack(planar)
    assert torch.equal(back, d)
    out = torch.full((n, limbs), -1, dtype=torch.int32, device="cuda:0")
    moma.unpack(planar, out=out)
    assert torch.equal(out, d)
