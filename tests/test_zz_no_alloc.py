"""hevmc_eval_config_noalloc against hevmc_eval_config, through the C ABI.

The no-alloc entry runs the same kernels on the same inputs, with its staging
buffers in the library's fixed device array, so every output must equal the
allocating entry's bit for bit.  Two calls in a row, the second on a smaller
configuration, so stale contents of the shared array from the first call
would show; both precisions; a size beyond the array's limit is refused.
"""
import numpy as np
import pytest

import oracle as O
from paper_1312_1282_amd import abi, configs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

RHO = configs.RHO_EQ
B = configs.C1_SMALL_FP64.b


def _config(n, precision, seed):
    p = abi.make_params(n, 1, precision=precision, density=RHO, b=B, step_sigma=0.63, seed=seed)
    s_ = O.system(n, O.box_side(n, RHO, precision == abi.FP32), B, step_sigma=0.63, seed=seed,
                  fp32_coords=precision == abi.FP32)
    x = O.fcc_start(s_, 3)
    rng = np.random.default_rng(seed)
    s = int(rng.integers(n))
    delta = rng.normal(0.0, 0.63, 3)
    return p, x, s, delta


@pytest.mark.parametrize("precision", [abi.FP64, abi.FP32])
def test_noalloc_matches_eval_config_on_two_calls(precision):
    for n, seed in ((2048, 11), (256, 12)):     # second call smaller than the first
        p, x, s, delta = _config(n, precision, seed)
        ref = abi.eval_config(p, x, s, delta)
        got = abi.eval_config(p, x, s, delta, noalloc=True)
        assert got[0] == ref[0] and got[1] == ref[1], (n, got[:2], ref[:2])
        assert np.array_equal(got[2], ref[2]), (n, got[2], ref[2])
        assert np.all(np.isfinite(got[2]))


def test_noalloc_largest_size_and_limit():
    n = abi.NOALLOC_MAX_N
    p = abi.make_params(n, 1, precision=abi.FP32, density=RHO, b=B, step_sigma=0.63, seed=5)
    s_ = O.system(n, O.box_side(n, RHO, True), B, step_sigma=0.63, seed=5, fp32_coords=True)
    x = O.fcc_start(s_, 0)
    ref = abi.eval_config(p, x, 7, np.array([0.1, -0.2, 0.3]))
    got = abi.eval_config(p, x, 7, np.array([0.1, -0.2, 0.3]), noalloc=True)
    assert got[0] == ref[0] and got[1] == ref[1] and np.array_equal(got[2], ref[2])
    big = abi.make_params(n + 1, 1, precision=abi.FP32, density=RHO, b=B, step_sigma=0.63, seed=5)
    with pytest.raises(abi.HevmcError, match="no-alloc scratch") as ei:
        abi.eval_config(big, np.full((3, n + 1), 1.0), 0, np.zeros(3), noalloc=True)
    assert ei.value.code == -1
