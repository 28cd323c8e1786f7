"""lbm_reduce_noalloc (the reduction with its partial sums in the library's
static device array, for callers that cannot allocate) against lbm_reduce
(the caller's scratch) through the C ABI: identical bits on two calls in a
row, the second on a smaller grid, in every storage type."""
import ctypes

import numpy as np
import pytest
import torch

from paper_1112_0850_amd import _abi as A
from paper_1112_0850_amd import inputs as I
from paper_1112_0850_amd.lbm import LBM
from tests.gpu_util import say

pytestmark = pytest.mark.gpu
P = lambda t: ctypes.c_void_p(t.data_ptr())


@pytest.mark.parametrize("storage", ["f32", "f16", "bf16", "f64", "f32x"])
def test_reduce_noalloc_matches_reduce(storage):
    for shape in [(40, 36, 150), (5, 7, 13)]:  # the second call on a smaller grid
        say("reduce without allocation", storage, shape)
        flags = I.random_flags(shape, 3, solid_fraction=0.15, noforce_fraction=0.1)
        rng = np.random.default_rng(len(shape) + shape[0])
        u0 = torch.from_numpy(0.03 * (rng.random((3,) + shape) - 0.5)).float()
        sim = LBM(shape, 0.7, (1e-5, -2e-6, 0), storage, flags=flags, u0=u0,
                  f16_scale_log2=8 if storage == "f16" else 0).step(7)
        ref = sim.reduce()
        got = torch.full((5,), float("nan"), dtype=torch.float64, device="cuda")
        A.lbm_reduce_noalloc(sim.ctx, P(got))
        torch.cuda.synchronize()
        say(f"  {got.cpu().tolist()}")
        assert torch.equal(got, ref)
        with pytest.raises(A.LBMError):
            A.lbm_reduce_noalloc(sim.ctx, None)
        del sim
