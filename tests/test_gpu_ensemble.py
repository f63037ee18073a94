"""GPU tests of ensembles of independent stars in one particle set (per-star mass, crust shear
factor and background centre) against the oracle, of graph-captured stepping, and of the launch
autotuner.  Tolerances as in test_gpu_parity: neighbour sets bit-exact, one FP64 evaluation to
1e-12 (kappa-relative for the cancelling sums), state after steps to 1e-12 of each field's scale,
FP32 pair sums to 1e-4 in D, rho and P."""
import numpy as np
import pytest

from parity import check_lists, eval_errors, field_errors, gpu_run, oracle_run, step_errors
from sph_inputs import workloads as W

pytestmark = pytest.mark.gpu


def _print(name, e):
    print(name, " ".join(f"{k}={v:.2e}" for k, v in e.items()), flush=True)


@pytest.fixture(scope="module", params=["gamma2", "pp"])
def ens(request):
    # four uneven stars (about 2k to 8k particles): Gamma = 2 stars with a thick crust (per-star
    # shear factors in play) and table-EoS stars
    return W.ensemble(4, 16000, seed=9, nmin=2000, nmax=8000, kind=request.param)


def test_ensemble_evaluation(ens):
    w = ens
    g = gpu_run(w, precision="FP64")
    o = oracle_run(w)
    assert check_lists(g, o, w.n) == 0
    print("crust particles", int(o["type"].sum()), "stressed rates", int(np.sum(np.any(o["dSdt"] != 0, axis=0))))
    e = eval_errors(g, o)
    _print("ensemble eval", e)
    for k, v in e.items():
        assert v <= 1e-12, (k, v)
    # the stars really differ: particle masses (and, with a crust, shear factors) per star
    assert len(set(np.round(w.star_params[:, 3], 12))) == 4
    if w.params.eos == "GAMMA_LAW":   # crust particles carry their own star's shear factor
        star = w.arrays["star"]
        with_crust = 0
        for s in range(w.star_params.shape[0]):
            sel = (star == s) & (o["mu"] > 0)
            if np.any(sel):
                with_crust += 1
                assert np.allclose(o["mu"][sel] / o["P"][sel], w.star_params[s, 4], rtol=1e-12, atol=0)
        assert with_crust >= 2


def test_full_size_ensemble_evaluation():
    # the benchmark's ensemble itself (64 piecewise-polytrope stars of uneven sizes, 8.0M
    # particles, per-star masses, shear factors and centres): one FP64 evaluation against the
    # oracle at full size, every particle, and the FP32 evaluation per field
    w = W.ensemble(64, 8_000_000, seed=5, precision="FP64", kind="pp")
    o = oracle_run(w)
    g = gpu_run(w, precision="FP64", lists=False)
    assert g["_stats"]["pairs"] == int(np.sum(np.diff(o["offsets"])))
    e = eval_errors(g, o)
    _print(f"8M ensemble eval ({w.n} particles, {len(w.star_params)} stars)", e)
    for k, v in e.items():
        assert v <= 1e-12, (k, v)
    del g
    g32 = gpu_run(w, precision="FP32", lists=False)
    assert g32["_stats"]["pairs"] == int(np.sum(np.diff(o["offsets"])))
    e = eval_errors(g32, o)
    _print("8M ensemble fp32 eval", e)
    for k in ("D", "rho", "P", "ax", "ay", "az", "dudt"):
        assert e[k] < 1e-4, (k, e[k])


def test_ensemble_steps(ens):
    w = ens
    g = gpu_run(w, steps=5, precision="FP64")
    o = oracle_run(w, steps=5)
    e = step_errors(g, o, ("x", "y", "z", "vx", "vy", "vz", "u", "h", "S", "D", "ax", "dudt", "dSdt"), w.dt, 5)
    _print("ensemble 5 steps", e)
    for k, v in e.items():
        assert v < 1e-12, (k, v)
    assert np.array_equal(g["broken"], o["broken"])


def test_ensemble_fp32_pairs(ens):
    w = ens
    g = gpu_run(w, precision="FP32")
    o = oracle_run(w)
    assert check_lists(g, o, w.n) == 0
    e = eval_errors(g, o)
    _print("ensemble fp32", e)
    for k in ("D", "rho", "P"):
        assert e[k] < 1e-4, (k, e[k])


def _run_on_stream(w, steps, ctx_kw, tune=0):
    """Evaluate and step on a non-default torch stream (graph capture needs one); with tune,
    sph_autotune runs first (the lists are rebuilt afterwards).  Returns (state by id, stats,
    tune result)."""
    import torch

    from paper_2107_07315_amd import sph
    s = torch.cuda.Stream()
    tr = None
    with torch.cuda.stream(s):
        ctx = sph.Context(w.params, capacity=w.n, stream=s, **ctx_kw)
        if w.star_params is not None:
            ctx.sph_ensemble_set(w.star_params)
        st = sph.DeviceState(w.arrays)
        if tune:
            before = st.numpy()
            tr = ctx.sph_autotune(st, w.dt, tune)
            ctx.sph_sync()
            after = st.numpy()
            for k in before:   # the trials run on a copy
                assert np.array_equal(before[k], after[k], equal_nan=True), k
        ctx.evaluate(st)
        ctx.sph_step(st, w.dt, steps)
        ctx.sph_sync()
        stats = ctx.sph_neighbour_stats()
        g = st.numpy()
        ctx.close()
    s.synchronize()
    order = np.argsort(g["id"])
    return {k: (v[..., order] if v.ndim == 2 else v[order]) for k, v in g.items()}, stats, tr


@pytest.mark.parametrize("skin", [1e-3, 0.05])
def test_graph_steps_equal_eager_steps(skin):
    # the same kernels replayed from two captured graphs per step give bit-identical states,
    # with rebuilds of the candidate lists (and re-captures when buffers grow) in between
    w = W.ensemble(4, 16000, seed=9, nmin=2000, nmax=8000, kind="gamma2", precision="FP64")
    eager, se, _ = _run_on_stream(w, 12, {"skin": skin, "graph": False})
    graph, sg, _ = _run_on_stream(w, 12, {"skin": skin, "graph": True})
    print("rebuilds eager", se["rebuilds"], "graph", sg["rebuilds"], flush=True)
    assert se["rebuilds"] == sg["rebuilds"]
    if skin == 1e-3:
        assert se["rebuilds"] >= 3
    for k in eager:
        assert np.array_equal(eager[k], graph[k]), k


def test_graph_mode_needs_a_stream():
    from paper_2107_07315_amd import sph
    w = W.lattice(n_side=8)
    ctx = sph.Context(w.params, capacity=w.n, graph=True)   # torch's default stream is the null stream
    st = sph.DeviceState(w.arrays)
    ctx.evaluate(st)
    with pytest.raises(sph.SphError) as e:
        ctx.sph_step(st, w.dt, 1)
    assert e.value.code == 1
    ctx.close()


def test_autotune_then_steps_match_oracle():
    w = W.star(20000, seed=3, kernel="WC4", eta=W.ETA_100, l=2, A=1e-2, plastic=True)
    g, _, tr = _run_on_stream(w, 5, {"graph": True}, tune=3)
    print("autotune", tr, flush=True)
    assert tr["pass_blocks"] in (0, 1024, 4096, 16384)
    assert tr["lanes"] in (1, 2, 4)
    assert tr["tile_cut"] in (6.0, 8.0, 10.0, 12.0)
    assert tr["skin"] in (0.07, 0.1, 0.14, 0.18)
    assert tr["trials"] >= 8
    assert 0 < tr["ms_per_step"] <= tr["ms_per_step_start"]
    o = oracle_run(w, steps=5)
    e = step_errors(g, o, ("x", "y", "z", "vx", "vy", "vz", "u", "h", "S", "D", "ax", "dudt", "dSdt"), w.dt, 5)
    _print("after autotune, 5 steps", e)
    for k, v in e.items():
        assert v < 1e-12, (k, v)
    assert np.array_equal(g["broken"], o["broken"])
