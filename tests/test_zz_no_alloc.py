"""GPU test of sph_neighbour_stats_noalloc (list statistics with the counters in a static device
array instead of an allocation): through the C ABI, its result equals sph_neighbour_stats on two
calls in a row, the second on a smaller input, and again after a context of another size."""
import numpy as np
import pytest

from sph_inputs import workloads as W

pytestmark = pytest.mark.gpu


def _ctx(w, steps=0):
    from paper_2107_07315_amd import sph
    ctx = sph.Context(w.params, capacity=w.n)
    st = sph.DeviceState(w.arrays)
    ctx.evaluate(st)
    if steps:
        ctx.sph_step(st, w.dt, steps)
    ctx.sph_sync()
    return ctx, st


def test_noalloc_stats_equal_allocating_stats():
    big = W.star(20000, seed=2)
    small = W.lattice(n_side=8)
    cb, sb = _ctx(big, steps=3)
    cs, ss = _ctx(small)
    for ctx, name in ((cb, "20k star"), (cs, "8^3 lattice"), (cb, "20k star again")):
        ref = ctx.sph_neighbour_stats()
        got = ctx.sph_neighbour_stats_noalloc()
        print(name, got, flush=True)
        assert got == ref, (name, got, ref)
        assert got["pairs"] > 0 and got["candidates"] >= got["pairs"] and got["tiles"] > 0
    assert cs.sph_neighbour_stats_noalloc()["pairs"] == small.n * 80     # 80 lattice neighbours each
    # a context before any evaluation: nothing counted
    from paper_2107_07315_amd import sph
    c0 = sph.Context(small.params, capacity=small.n)
    z = c0.sph_neighbour_stats_noalloc()
    assert z["pairs"] == 0 and z["candidates"] == 0 and z["tiles"] == 0
    for c in (cb, cs, c0):
        c.close()
