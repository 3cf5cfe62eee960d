"""HIP-graph replay of batched evolutions: every replay equals direct launches bit for bit.

The graph holds the kernel launches of one batch structure; the tables and the instance
array are uploaded before each replay.  The test replays each graph several times with
other work of the program (resets, state reads, observables, single-context runs)
between the replays, and checks every replay against a batch launched directly."""
import numpy as np
import pytest

from paper_1910_08020_amd import lgt
from tests.harness import get_state

pytestmark = pytest.mark.gpu

C64, C128 = lgt.LGT_C64, lgt.LGT_C128
TROT, SYM = lgt.LGT_ORDER_TROTTER, lgt.LGT_ORDER_SYMMETRIC


def _batch(d, L, dtype, scheds, order, splits, graphs, ctxs=None):
    own = ctxs is None
    if own:
        ctxs = [lgt.lgt_create(d, list(L), 1, dtype) for _ in scheds]
    try:
        for c in ctxs:
            lgt.lgt_set_graphs(c, graphs)
            lgt.lgt_reset(c, lgt.LGT_INIT_PLUS, 0)
        for a, b in zip(splits[:-1], splits[1:]):
            lgt.lgt_batch_evolve(ctxs, scheds, [order] * len(scheds), a, b - a)
        return [get_state(c) for c in ctxs]
    finally:
        if own:
            for c in ctxs:
                lgt.lgt_destroy(c)


@pytest.mark.parametrize("order", [TROT, SYM], ids=["trotter", "symmetric"])
@pytest.mark.parametrize("dtype", [C64, C128], ids=["c64", "c128"])
@pytest.mark.parametrize("d,L", [(2, (2, 2)), (2, (2, 4)), (2, (3, 3))], ids=["2x2", "2x4", "3x3"])
def test_graph_replays_equal_direct_launches(d, L, dtype, order):
    n, T = 40, 2.0
    # two batches of one structure (all steps in the tan form), one of another (the
    # coupling ramp turns to the cot form part way)
    tan_a = [lgt.make_schedule(T, n, lam, 1.0) for lam in (0.3, 0.7, 1.1)]
    tan_b = [lgt.make_schedule(T, n, lam, 1.0) for lam in (0.5, 0.9, 1.3)]
    mixed = [lgt.make_schedule(T, n, ramp=lgt.LGT_RAMP_COUPLING, g0=0.0, g1=40.0)] * 3
    splits = [0, 15, n]
    want = {k: _batch(d, L, dtype, s, order, splits, False)
            for k, s in (("a", tan_a), ("b", tan_b), ("m", mixed))}
    ctxs = [lgt.lgt_create(d, list(L), 1, dtype) for _ in range(3)]
    other = lgt.lgt_create(d, list(L), 1, dtype)
    try:
        for rep, key in enumerate(["a", "b", "m", "a", "m", "b", "a"]):
            scheds = {"a": tan_a, "b": tan_b, "m": mixed}[key]
            got = _batch(d, L, dtype, scheds, order, splits, True, ctxs)
            for g, w in zip(got, want[key]):
                assert np.array_equal(g, w), f"replay {rep} ({key}) differs from direct launches"
            # the program's own work between replays
            lgt.lgt_evolve(other, tan_a[rep % 3], order, lgt.LGT_FORM_FUSED, 0, 7)
            lgt.lgt_measure(ctxs[rep % 3], lgt.LGT_OBS_PLAQ)
            lgt.lgt_reset(other, lgt.LGT_INIT_BASIS, rep)
        lgt.lgt_set_graphs(ctxs[0], False)
        got = _batch(d, L, dtype, tan_b, order, splits, False, ctxs)
        for g, w in zip(got, want["b"]):
            assert np.array_equal(g, w)
    finally:
        for c in ctxs + [other]:
            lgt.lgt_destroy(c)


def test_graph_cache_bound_and_profiling_bypass():
    """More structures than the cache holds, and a profiled batch, still give the direct
    result."""
    d, L, dtype = 2, (2, 4), C64
    ctx = lgt.lgt_create(d, list(L), 1, dtype)
    try:
        for n in range(1, 70):
            s = [lgt.make_schedule(0.05 * n, n, 1.0, 1.0)]
            got = _batch(d, L, dtype, s, SYM, [0, n], True, [ctx])
            if n % 17 == 1:
                assert np.array_equal(got[0], _batch(d, L, dtype, s, SYM, [0, n], False)[0])
        lgt.lgt_set_profiling(ctx, True)
        s = [lgt.make_schedule(1.0, 20, 0.8, 1.0)]
        got = _batch(d, L, dtype, s, SYM, [0, 20], True, [ctx])
        lgt.lgt_set_profiling(ctx, False)
        assert np.array_equal(got[0], _batch(d, L, dtype, s, SYM, [0, 20], False)[0])
    finally:
        lgt.lgt_destroy(ctx)
