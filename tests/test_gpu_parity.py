"""GPU (HIP C-ABI) vs CPU FP64 oracle parity on seeded inputs.

Tolerances: neighbour sets bit-exact; one FP64 evaluation agrees to 1e-12, relative for
positive pointwise fields (D, rho, P, c_s) and relative to the summation bound kappa (the sum of
|terms|) for the cancelling sums (accelerations, du/dt, dS/dt), since the two sides add the
same terms in different orders.  After k time steps the state is compared field by field
relative to each field's largest magnitude, to TOL_STEPS (roundoff of order 1e-16 per operation
grows through the pair dynamics; a few to ten steps stay below 1e-13).
"""
import math

import numpy as np
import pytest

import oracle
from parity import check_lists, eval_errors, field_errors, gpu_run, oracle_keys, oracle_run, step_errors
from sph_inputs import workloads as W
from sph_inputs.lattice import random_box
from sph_inputs.params import MethodParams

pytestmark = pytest.mark.gpu

TOL_EVAL = 1e-12
TOL_STEPS = 1e-12


def _print(name, e):
    print(name, " ".join(f"{k}={v:.2e}" for k, v in e.items()), flush=True)


def _assert_eval(g, o, tol=TOL_EVAL, skip=()):
    e = eval_errors(g, o)
    _print("eval", e)
    for k, v in e.items():
        if k in skip:
            continue
        assert v <= tol, (k, v)


def test_lattice_evaluation_and_neighbour_sets():
    w = W.lattice()
    g = gpu_run(w)
    o = oracle_run(w, mode=oracle.BRUTE)
    assert check_lists(g, o, w.n) == 0
    assert all(len(v) == 80 for v in g["_lists"].values())
    _assert_eval(g, o)


@pytest.mark.parametrize("seed,n", [(0, 3000), (1, 1000), (2, 777)])
def test_random_variable_h_box(seed, n):
    # ragged n (not a multiple of 64), smoothing lengths varying 16x, a few huge ones
    x, y, z = random_box(n, 1.0, seed)
    rng = np.random.default_rng(50 + seed)
    h = 0.035 * rng.uniform(0.5, 2.0, n)
    S = rng.normal(scale=0.2, size=(6, n))
    S[:3] -= S[:3].mean(0)
    typ = (rng.uniform(size=n) < 0.5).astype(np.int8)
    S[:, typ == 0] = 0
    arr = dict(x=x, y=y, z=z, vx=rng.normal(scale=0.1, size=n), vy=rng.normal(scale=0.1, size=n),
               vz=rng.normal(scale=0.1, size=n), u=rng.uniform(0.5, 2, n), h=h, S=S, type=typ,
               broken=np.zeros(n, np.uint8), id=np.arange(n, dtype=np.int32))
    big = np.zeros(n, bool)
    big[rng.choice(n, 6, replace=False)] = True
    for periodic in (False, True):
        # one periodic image per pair needs 2 h < box / 2
        arr["h"] = np.where(big, h * (2.0 if periodic else 4.0), h)
        p = MethodParams(m=1.0 / n, kernel="WC4", periodic=periodic, box=1.0, eos="GAMMA_LAW",
                         gamma=5 / 3, mu_mode="CONST", mu_const=0.5)
        w = W.Workload("rand", p, dict(arr), 1e-3, 0)
        g = gpu_run(w, ctx_kw={"max_neighbours": 1024})
        o = oracle_run(w, mode=oracle.BRUTE)
        assert check_lists(g, o, n) == 0
        _assert_eval(g, o)


def test_star_evaluation_tov():
    w = W.star(20000, seed=2)
    g = gpu_run(w)
    o = oracle_run(w)
    assert check_lists(g, o, w.n) == 0
    _assert_eval(g, o)
    assert o["type"].sum() > 100


def test_plastic_star_evaluation_and_steps():
    w = W.star(20000, seed=3, kernel="WC4", eta=W.ETA_100, l=2, A=1e-2, plastic=True)
    g = gpu_run(w)
    o = oracle_run(w)
    assert check_lists(g, o, w.n) == 0
    _assert_eval(g, o)
    g = gpu_run(w, steps=5)
    o = oracle_run(w, steps=5)
    e = step_errors(g, o, ("x", "y", "z", "vx", "vy", "vz", "u", "h", "S", "D", "ax", "dudt", "dSdt"), w.dt, 5)
    _print("5 steps", e)
    for k, v in e.items():
        assert v < TOL_STEPS, (k, v)
    assert np.array_equal(g["broken"], o["broken"])


def test_lattice_ten_steps():
    w = W.lattice()
    g = gpu_run(w, steps=10)
    o = oracle_run(w, steps=10)
    e = step_errors(g, o, ("x", "y", "z", "vx", "vy", "vz", "u", "S", "D", "ax", "dudt", "dSdt"), w.dt, 10)
    _print("10 steps", e)
    for k, v in e.items():
        assert v < TOL_STEPS, (k, v)


def test_table_eos_star():
    w = W.pp_star(20000, seed=4, eos="TABLE")
    g = gpu_run(w)
    o = oracle_run(w)
    _assert_eval(g, o)


def test_full_size_star_matches_oracle():
    # the benchmark workload itself (2M-particle piecewise-polytrope star, table EoS) in the
    # configuration bench.py times (default context: 4 lanes per target, default skin, run-ahead
    # multi-step call): one evaluation and 2 steps in FP64 against the oracle at full size, and
    # the FP32 evaluation per field; every particle is compared
    w = W.pp_star(2_000_000, seed=3, eos="TABLE")
    o = oracle_run(w)
    ok = oracle_keys(o, w.n)
    print("2M ordered pairs", ok.size, flush=True)
    g = gpu_run(w, csr_keys=True)
    assert np.array_equal(g["_keys"], ok)      # exact neighbour sets, FP64 decision
    _assert_eval(g, o)
    del g
    g32 = gpu_run(w, precision="FP32", csr_keys=True)
    assert np.array_equal(g32["_keys"], ok)    # FP32 decision with the FP64 guard band
    e = eval_errors(g32, o)
    _print("2M fp32 eval", e)
    for k in ("D", "rho", "P", "ax", "ay", "az", "dudt", "dSdt"):
        assert e[k] < 1e-4, (k, e[k])
    del g32, o, ok
    g = gpu_run(w, steps=2, lists=False)
    o = oracle_run(w, steps=2)
    e = step_errors(g, o, ("x", "y", "z", "vx", "vy", "vz", "u", "h", "S", "D", "ax", "dudt", "dSdt"), w.dt, 2)
    _print("2M 2 steps", e)
    for k, v in e.items():
        assert v < TOL_STEPS, (k, v)
    assert np.array_equal(g["broken"], o["broken"])


def test_c2_star_at_its_size():
    # configuration C2 as specified: the 200k-particle Gamma = 2 star (Wendland C2, eta 1.3, crust
    # mu = 0.01 P, elastic, l = 0 perturbation of 1e-3), 100 steps against the oracle in FP64, and
    # the FP32-pairs path after the same 100 steps per field
    w = W.star(200_000, seed=2)
    o = oracle_run(w, steps=100)
    g = gpu_run(w, steps=100, lists=False)
    keys = ("x", "y", "z", "vx", "vy", "vz", "u", "h", "S", "D", "ax", "dudt", "dSdt")
    e = step_errors(g, o, keys, w.dt, 100)
    _print("C2 200k, 100 steps", e)
    for k, v in e.items():
        assert v < TOL_STEPS, (k, v)
    del g
    g32 = gpu_run(w, steps=100, precision="FP32", lists=False)
    e = field_errors(g32, o, ("x", "vx", "u", "h", "S", "D", "rho", "P"))
    _print("C2 200k FP32 pairs, 100 steps", e)
    for k in ("D", "rho", "P", "S"):
        assert e[k] < 1e-4, (k, e[k])


def test_fp32_pairs_error_per_field():
    # the FP32 path takes the neighbour decision in FP32 with an FP64 guard band: its exact lists
    # must still equal the FP64 ones
    w = W.star(20000, seed=3, kernel="WC4", eta=W.ETA_100, l=2, A=1e-2, plastic=True)
    g = gpu_run(w, precision="FP32")
    o = oracle_run(w)
    assert check_lists(g, o, w.n) == 0
    e = eval_errors(g, o)
    _print("fp32 eval", e)
    for k in ("D", "rho", "P"):
        assert e[k] < 1e-4, (k, e[k])
    for k in ("ax", "ay", "az", "dudt", "dSdt"):
        assert e[k] < 1e-4, (k, e[k])


# ---------------------------------------------------------------------------------------------
# edge cases and error paths (all forced from the host; every kernel exits normally)


def _ctx_state(w, **kw):
    from paper_2107_07315_amd import sph
    return sph, sph.Context(w.params, capacity=max(w.n, 1), **kw), sph.DeviceState(w.arrays)


def _subset(w, idx):
    arr = {k: (v[..., idx] if np.ndim(v) == 2 else v[idx]) for k, v in w.arrays.items()}
    arr["id"] = np.arange(len(idx), dtype=np.int32)
    return W.Workload(w.name, w.params, arr, w.dt, 0)


def test_tiny_and_empty_inputs():
    w = W.lattice()
    for n in (1, 2, 63, 65):
        ws = _subset(w, np.arange(n))
        ws.params = ws.params.replace(periodic=False, box=0.0)
        g = gpu_run(ws)
        o = oracle_run(ws, mode=oracle.BRUTE)
        assert check_lists(g, o, n) == 0
        _assert_eval(g, o)
    # n = 0: every stage is a no-op that succeeds
    from paper_2107_07315_amd import sph
    ctx = sph.Context(w.params, capacity=16)
    st = sph.DeviceState({k: (v[..., :0] if np.ndim(v) == 2 else v[:0]) for k, v in w.arrays.items()})
    ctx.evaluate(st)
    ctx.sph_step(st, w.dt, 3)
    ctx.sph_sync()


def test_stage_order_and_argument_errors():
    w = W.lattice(n_side=8)
    sph, ctx, st = _ctx_state(w)
    with pytest.raises(sph.SphError) as e:
        ctx.sph_density(st)
    assert e.value.code == 4
    ctx.sph_build_cells(st)
    with pytest.raises(sph.SphError) as e:
        ctx.sph_forces(st)
    assert e.value.code == 4
    with pytest.raises(sph.SphError) as e:
        ctx.sph_step(st, w.dt, 1)
    assert e.value.code == 4
    ctx.sph_density(st)
    ctx.sph_stress_rate(st)
    ctx.sph_forces(st)
    with pytest.raises(sph.SphError) as e:
        ctx.sph_step(st, float("nan"), 1)
    assert e.value.code == 1
    ctx.sph_sync()
    # more particles than the context holds
    big = sph.DeviceState(W.lattice(n_side=9).arrays)
    with pytest.raises(sph.SphError) as e:
        ctx.sph_build_cells(big)
    assert e.value.code == 1


def test_neighbour_capacity_error_is_latched():
    w = W.lattice(n_side=8)
    sph, ctx, st = _ctx_state(w, max_neighbours=40)   # each particle has 80 neighbours
    ctx.evaluate(st)                                  # exact lists overflow in the density pass
    with pytest.raises(sph.SphError) as e:
        ctx.sph_sync()
    assert e.value.code == 5
    assert 0 <= e.value.particle < w.n                # the first particle that overflowed
    ctx.sph_sync()    # the status word was cleared
    sph, ctx, st = _ctx_state(w, max_neighbours=20)   # candidate lists (twice that) overflow too
    ctx.sph_build_cells(st)
    with pytest.raises(sph.SphError) as e:
        ctx.sph_sync()
    assert e.value.code == 5


def test_periodic_smoothing_length_limit():
    w = W.lattice(n_side=8)
    w.arrays["h"][3] = 0.3          # 2h >= box/2: a pair could have two periodic images
    sph, ctx, st = _ctx_state(w)
    ctx.sph_build_cells(st)
    with pytest.raises(sph.SphError) as e:
        ctx.sph_sync()
    assert e.value.code == 1


def test_nonfinite_and_eos_domain_errors():
    w = W.lattice(n_side=8)
    w.arrays["u"][5] = np.nan
    sph, ctx, st = _ctx_state(w)
    ctx.evaluate(st)
    with pytest.raises(sph.SphError) as e:
        ctx.sph_sync()
    assert e.value.code == 6
    wp = W.pp_star(5000, seed=4, eos="TABLE")
    wp.arrays["u"][0] = 50.0       # above the table's u range
    sph, ctx, st = _ctx_state(wp)
    ctx.evaluate(st)
    with pytest.raises(sph.SphError) as e:
        ctx.sph_sync()
    assert e.value.code == 7


def test_skin_lists_match_rebuild_every_evaluation():
    # candidate lists kept across steps with a Verlet skin give the same exact neighbour sets and
    # the same fields as rebuilding at every evaluation; a tiny skin forces rebuilds mid-run
    w = W.star(20000, seed=2)
    runs = {s: gpu_run(w, steps=8, ctx_kw={"skin": s}, lists=True) for s in (0.0, 1e-3, 0.05)}
    ref = runs[0.0]
    assert ref["_stats"]["rebuilds"] == 9
    for s in (1e-3, 0.05):
        g = runs[s]
        bad = sum(1 for a in range(w.n) if not np.array_equal(g["_lists"][a], ref["_lists"][a]))
        assert bad == 0, (s, bad)
        assert g["_stats"]["pairs"] == ref["_stats"]["pairs"]
        assert g["_stats"]["candidates"] > g["_stats"]["pairs"]
        e = field_errors(g, ref, ("x", "vx", "u", "D", "ax", "dudt"))
        _print(f"skin {s} rebuilds={g['_stats']['rebuilds']}", e)
        for k, v in e.items():
            assert v < TOL_STEPS, (s, k, v)
    assert runs[0.05]["_stats"]["rebuilds"] <= runs[1e-3]["_stats"]["rebuilds"] <= 9
    assert runs[1e-3]["_stats"]["rebuilds"] >= 2


def test_one_multi_step_call_equals_single_step_calls():
    # inside one sph_step call the host queues each step before reading the previous step's skin
    # test back and a step behind a failed test is cancelled on the device and re-run after the
    # rebuild; the result must equal stepping one call at a time (where no step runs ahead), bit
    # for bit, with the same list builds
    from paper_2107_07315_amd import sph
    w = W.star(20000, seed=5)
    out = {}
    for mode in ("one_call", "single_calls"):
        ctx = sph.Context(w.params.replace(precision="FP32"), capacity=w.n, skin=0.01)
        st = sph.DeviceState(w.arrays)
        ctx.evaluate(st)
        if mode == "one_call":
            ctx.sph_step(st, w.dt, 16)
        else:
            for _ in range(16):
                ctx.sph_step(st, w.dt, 1)
        ctx.sph_sync()
        g = st.numpy()
        order = np.argsort(g["id"])
        out[mode] = ({k: (v[..., order] if v.ndim == 2 else v[order]) for k, v in g.items()},
                     ctx.sph_neighbour_stats()["rebuilds"])
        ctx.close()
    (a, ra), (b, rb) = out["one_call"], out["single_calls"]
    _print(f"rebuilds {ra} (one call) {rb} (single calls)", {})
    assert ra == rb and ra >= 3
    for k in ("x", "y", "z", "vx", "vy", "vz", "u", "h", "S", "D", "ax", "dudt"):
        assert np.array_equal(a[k], b[k]), k


def test_force_pass_with_stress_records_in_lds():
    # most tiles hold stressed particles (60% of a random box are crust), so the FP32 force pass
    # stages the neighbours' S/D^2 in LDS; stressed and unstressed neighbours mix in every list
    n = 3000
    x, y, z = random_box(n, 1.0, 11)
    rng = np.random.default_rng(12)
    S = rng.normal(scale=0.2, size=(6, n))
    S[:3] -= S[:3].mean(0)
    typ = (rng.uniform(size=n) < 0.6).astype(np.int8)
    S[:, typ == 0] = 0
    arr = dict(x=x, y=y, z=z, vx=rng.normal(scale=0.1, size=n), vy=rng.normal(scale=0.1, size=n),
               vz=rng.normal(scale=0.1, size=n), u=rng.uniform(0.5, 2, n), h=0.035 * rng.uniform(0.5, 2.0, n),
               S=S, type=typ, broken=np.zeros(n, np.uint8), id=np.arange(n, dtype=np.int32))
    for periodic in (False, True):
        p = MethodParams(m=1.0 / n, kernel="WC4", periodic=periodic, box=1.0, eos="GAMMA_LAW", gamma=5 / 3,
                         mu_mode="CONST", mu_const=0.5, precision="FP32")
        wr = W.Workload("rand", p, dict(arr), 1e-3, 0)
        o = oracle_run(wr, mode=oracle.BRUTE)
        g = gpu_run(wr)
        assert check_lists(g, o, n) == 0
        e = eval_errors(g, o)
        _print(f"S/D^2 in LDS, periodic={periodic}", e)
        for k in ("D", "rho", "P", "ax", "ay", "az", "dudt", "dSdt"):
            assert e[k] < 1e-4, (k, e[k])


@pytest.mark.parametrize("cell_div", [2, 4])
def test_cell_size_leaves_the_neighbour_sets(cell_div):
    # finer cells than the default (2, 4 per smoothing diameter instead of 1) change the cell
    # enumeration, the tile splits and the order of the candidate unions, not the exact sets
    w = W.star(20000, seed=3, kernel="WC4", eta=W.ETA_100, l=2, A=1e-2, plastic=True)
    o = oracle_run(w)
    for prec in ("FP64", "FP32"):
        g = gpu_run(w, precision=prec, ctx_kw={"cell_div": cell_div})
        assert check_lists(g, o, w.n) == 0, prec
        if prec == "FP64":
            _assert_eval(g, o)
        else:
            e = eval_errors(g, o)
            for k in ("D", "rho", "P"):
                assert e[k] < 1e-4, (k, e[k])
    x, y, z = random_box(777, 1.0, 9)
    rng = np.random.default_rng(10)
    n = 777
    arr = dict(x=x, y=y, z=z, vx=rng.normal(scale=0.1, size=n), vy=rng.normal(scale=0.1, size=n),
               vz=rng.normal(scale=0.1, size=n), u=rng.uniform(0.5, 2, n), h=0.035 * rng.uniform(0.5, 2.0, n),
               S=np.zeros((6, n)), type=np.zeros(n, np.int8), broken=np.zeros(n, np.uint8),
               id=np.arange(n, dtype=np.int32))
    for periodic in (False, True):
        p = MethodParams(m=1.0 / n, kernel="WC2", periodic=periodic, box=1.0, eos="GAMMA_LAW", gamma=5 / 3)
        wr = W.Workload("rand", p, dict(arr), 1e-3, 0)
        g = gpu_run(wr, ctx_kw={"cell_div": cell_div})
        o2 = oracle_run(wr, mode=oracle.BRUTE)
        assert check_lists(g, o2, n) == 0, periodic
        _assert_eval(g, o2)


@pytest.mark.parametrize("lanes", [1, 2])
def test_lanes_per_target(lanes):
    # 1 and 2 lanes per target (the default is 4): same exact neighbour sets, fields to the
    # evaluation tolerance, steps to the state tolerance
    w = W.star(20000, seed=3, kernel="WC4", eta=W.ETA_100, l=2, A=1e-2, plastic=True)
    g = gpu_run(w, ctx_kw={"lanes": lanes})
    o = oracle_run(w)
    assert check_lists(g, o, w.n) == 0
    _assert_eval(g, o)
    g = gpu_run(w, steps=5, ctx_kw={"lanes": lanes})
    o = oracle_run(w, steps=5)
    e = step_errors(g, o, ("x", "y", "z", "vx", "vy", "vz", "u", "h", "S", "D", "ax", "dudt", "dSdt"), w.dt, 5)
    _print(f"lanes {lanes}, 5 steps", e)
    for k, v in e.items():
        assert v < TOL_STEPS, (k, v)
    for ker, periodic in (("WC2", True), ("WC4", False)):   # ragged tiles, both kernels, periodic
        x, y, z = random_box(1000, 1.0, 7)
        rng = np.random.default_rng(8)
        n = 1000
        S = rng.normal(scale=0.2, size=(6, n))
        S[:3] -= S[:3].mean(0)
        typ = (rng.uniform(size=n) < 0.5).astype(np.int8)
        S[:, typ == 0] = 0      # fluid particles carry no deviatoric stress
        arr = dict(x=x, y=y, z=z, vx=rng.normal(scale=0.1, size=n), vy=rng.normal(scale=0.1, size=n),
                   vz=rng.normal(scale=0.1, size=n), u=rng.uniform(0.5, 2, n), h=0.035 * rng.uniform(0.5, 2.0, n),
                   S=S, type=typ, broken=np.zeros(n, np.uint8), id=np.arange(n, dtype=np.int32))
        p = MethodParams(m=1.0 / n, kernel=ker, periodic=periodic, box=1.0, eos="GAMMA_LAW", gamma=5 / 3,
                         mu_mode="CONST", mu_const=0.5, precision="FP32")
        wr = W.Workload("rand", p, arr, 1e-3, 0)
        g = gpu_run(wr, ctx_kw={"lanes": lanes})
        o = oracle_run(wr, mode=oracle.BRUTE)
        assert check_lists(g, o, n) == 0
        ef = eval_errors(g, o)
        _print(f"lanes {lanes} {ker} periodic={periodic} fp32", ef)
        for k in ("D", "rho", "P", "ax", "ay", "az", "dudt", "dSdt"):
            assert ef[k] < 1e-4, (k, ef[k])


def test_fp32_neighbour_decision_at_the_support_edge():
    # isolated pairs whose separation is within 1e-12 (relative) of the support h_a + h_b, where
    # the FP32 test cannot decide and the FP64 fallback must: the lists equal the oracle's, and the
    # error reported through sph_error_particle is absent
    eps = np.array([-1e-6, -1e-9, -1e-12, -1e-15, 0.0, 1e-15, 1e-12, 1e-9, 1e-6])
    rng = np.random.default_rng(12)
    xs, ys, zs, hs = [], [], [], []
    for k, e in enumerate(eps):
        ha, hb = 0.05 * rng.uniform(0.8, 1.2), 0.05 * rng.uniform(0.8, 1.2)
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        c = np.array([3.0 * k + 1.0, 2.0, 2.0])
        b = c + d * (ha + hb) * (1.0 + e)
        xs += [c[0], b[0]]
        ys += [c[1], b[1]]
        zs += [c[2], b[2]]
        hs += [ha, hb]
    n = len(xs)
    arr = dict(x=np.array(xs), y=np.array(ys), z=np.array(zs), vx=np.zeros(n), vy=np.zeros(n), vz=np.zeros(n),
               u=np.ones(n), h=np.array(hs), S=np.zeros((6, n)), type=np.zeros(n, np.int8),
               broken=np.zeros(n, np.uint8), id=np.arange(n, dtype=np.int32))
    for precision in ("FP32", "FP64"):
        p = MethodParams(m=1e-3, kernel="WC4", periodic=False, box=0.0, eos="GAMMA_LAW", gamma=5 / 3,
                         mu_mode="CONST", mu_const=0.0, precision=precision)
        w = W.Workload("edge", p, dict(arr), 1e-3, 0)
        g = gpu_run(w)
        o = oracle_run(w, mode=oracle.BRUTE)
        assert check_lists(g, o, n) == 0, precision
        pairs = len(o["ids"])   # ordered pairs; the 4 pairs inside the support at least 1e-12 count twice
        print(precision, "ordered pairs in the oracle lists:", pairs, flush=True)
        assert 8 <= pairs <= 12
