"""The allocation-free sampler against lgt_sample: the same shots, bit for bit, on two calls
in a row (the second with a smaller state and fewer shots, on the per-GPU array the first call
left behind), and its size limits.  Calls go through the C ABI."""
import numpy as np
import pytest

import workloads
from paper_1910_08020_amd import lgt
from tests.harness import gpu_ctx

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


@pytest.mark.parametrize("dtype", [lgt.LGT_C128, lgt.LGT_C64], ids=["c128", "c64"])
def test_sample_noalloc_equals_sample(dtype):
    cases = [((3, (2, 2, 2)), 200_000, 77), ((2, (3, 3)), 3000, 5)]   # the second is smaller
    for (d, L), shots, seed in cases:
        n_links = d * int(np.prod(L))
        psi = workloads.random_state(n_links, stream=60 + n_links)
        _say(f"sample_noalloc {L} shots={shots}")
        with gpu_ctx(d, L, dtype, psi) as ctx:
            want = lgt.lgt_sample(ctx, shots, seed)
            got = lgt.lgt_sample_noalloc(ctx, shots, seed)
            again = lgt.lgt_sample_noalloc(ctx, shots, seed)
        assert np.array_equal(got, want)
        assert np.array_equal(again, want)
        assert int(got.max()) < (1 << n_links)


def test_sample_noalloc_limits():
    with gpu_ctx(2, (2, 2), lgt.LGT_C64) as ctx:
        for bad in (0, (1 << 20) + 1):
            with pytest.raises(lgt.LgtError) as e:
                lgt.lgt_sample_noalloc(ctx, bad, 1)
            assert e.value.status == lgt.LGT_E_INVALID
        got = lgt.lgt_sample_noalloc(ctx, 1 << 20, 3)
        assert np.array_equal(got, lgt.lgt_sample(ctx, 1 << 20, 3))
