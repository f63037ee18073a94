"""GPU checks of the boundary calls around the stage calls: a context-owned EoS table
(sph_eos_table_create), a network loaded from BF16 weights (sph_mlp_load) and the error detail
(sph_last_error_detail).  All through the C ABI."""
import numpy as np
import pytest

from sph_inputs import workloads as W
from sph_inputs.eos_table import mlp_init

pytestmark = pytest.mark.gpu


def _eval(ctx, w):
    from paper_2107_07315_amd import sph
    st = sph.DeviceState(w.arrays)
    ctx.evaluate(st)
    ctx.sph_sync()
    g = st.numpy()
    o = np.argsort(g["id"])
    return {k: g[k][..., o] for k in ("D", "rho", "P", "cs", "ax", "dudt")}


def test_context_owned_table_equals_caller_table():
    from paper_2107_07315_amd import sph
    w = W.pp_star(5000, seed=4, eos="TABLE")
    ref = sph.Context(w.params, capacity=w.n)
    a = _eval(ref, w)
    ref.close()
    ctx = sph.Context(w.params.replace(table=None), capacity=w.n)
    st = sph.DeviceState(w.arrays)
    with pytest.raises(sph.SphError) as e:
        ctx.sph_build_cells(st)
    assert e.value.code == 1 and "table" in (e.value.detail or ""), e.value
    ctx.eos_table_create(w.params.table)
    b = _eval(ctx, w)
    for k in a:
        assert np.array_equal(a[k], b[k]), k
    # a wrong table size is refused with a reason
    bad = w.params.table
    rc = ctx.lib.sph_eos_table_create(ctx.h, bad.lnP.ctypes.data, bad.lncs2.ctypes.data, 1, bad.nu, bad.lnr0,
                                      bad.dlnr, bad.lnu0, bad.dlnu)
    assert rc == 1 and "table size" in ctx.last_error_detail()
    ctx.close()


def test_network_from_bf16_weights():
    import torch

    from paper_2107_07315_amd import sph
    w = W.pp_star(2000, seed=4, eos="MLP")
    # a network whose every weight is a BF16 number (round to nearest even), as trained elsewhere
    u = mlp_init(4).view(np.uint32).astype(np.uint64)
    bits = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)
    wb = (bits.astype(np.uint32) << 16).view(np.float32)
    c1 = sph.Context(w.params, capacity=w.n)
    c1.mlp_set_params(wb)
    wr = c1.mlp_get_params(rounded=True)              # the values the kernels use
    assert np.array_equal(wr, wb)                      # BF16 numbers stay as they are
    c2 = sph.Context(w.params, capacity=w.n)
    c2.mlp_load(bits)
    assert np.array_equal(c2.mlp_get_params(rounded=False), wb)
    assert np.array_equal(c2.mlp_get_params(rounded=True), wb)
    t = w.params.table
    rng = np.random.default_rng(1)
    lr = torch.as_tensor(t.lnr0 + rng.uniform(0, (t.nr - 1) * t.dlnr, 4096), device="cuda")
    lu = torch.as_tensor(t.lnu0 + rng.uniform(0, (t.nu - 1) * t.dlnu, 4096), device="cuda")
    p1, q1 = c1.mlp_eval(lr, lu)
    p2, q2 = c2.mlp_eval(lr, lu)
    torch.cuda.synchronize()
    assert torch.equal(p1, p2) and torch.equal(q1, q2)
    c1.close()
    c2.close()


def test_error_detail_names_the_cause():
    from paper_2107_07315_amd import sph
    w = W.lattice(n_side=8)
    ctx = sph.Context(w.params, capacity=w.n, max_neighbours=40)
    st = sph.DeviceState(w.arrays)
    with pytest.raises(sph.SphError) as e:
        ctx.sph_density(st)
    assert "sph_build_cells" in e.value.detail
    ctx.evaluate(st)
    with pytest.raises(sph.SphError) as e:
        ctx.sph_sync()
    assert e.value.code == 5 and "particle" in e.value.detail and "capacity" in e.value.detail, e.value.detail
    with pytest.raises(sph.SphError) as e:
        ctx.sph_step(st, float("nan"), 1)
    assert "dt" in e.value.detail
    ctx.close()
    with pytest.raises(sph.SphError) as e:
        sph.Context(w.params.replace(m=-1.0), capacity=w.n)
    assert "mass" in e.value.detail
