"""Helpers for GPU-vs-oracle parity tests: run both sides on the same seeded input and compare
in the oracle's particle order (the GPU reorders particles; `id` follows them)."""
import numpy as np

import oracle

FIELDS_EVAL = ("D", "rho", "P", "cs", "ax", "ay", "az", "dudt")


def gpu_run(w, steps=0, precision=None, ctx_kw=None, params=None, lists=None, csr_keys=False):
    """Evaluate (and step) on the GPU; returns the state in id order.  With lists (default: only
    when steps == 0) the exact neighbour lists of the last evaluation come back as "_lists" (by
    id), and the list statistics as "_stats".  With csr_keys the lists come back instead as
    "_keys", the sorted array of a * n + b over the ordered pairs (by id), for large n."""
    from paper_2107_07315_amd import sph
    p = params or w.params
    if precision:
        p = p.replace(precision=precision)
    ctx = sph.Context(p, capacity=w.n, **(ctx_kw or {}))
    if w.star_params is not None:
        ctx.sph_ensemble_set(w.star_params)
    st = sph.DeviceState(w.arrays)
    ctx.evaluate(st)
    if steps:
        ctx.sph_step(st, w.dt, steps)
    ctx.sph_sync()
    nb = None
    if csr_keys or (lists if lists is not None else steps == 0):
        nb = ctx.sph_export_neighbours(w.n)
    stats = ctx.sph_neighbour_stats()
    g = st.numpy()
    order = np.argsort(g["id"])
    out = {k: (v[..., order] if v.ndim == 2 else v[order]) for k, v in g.items()}
    out["_stats"] = stats
    if nb is not None and csr_keys:
        off, ids = nb
        ident = g["id"].astype(np.int64)
        rows = np.repeat(ident, np.diff(off))
        out["_keys"] = np.sort(rows * w.n + ident[ids])
    elif nb is not None:
        off, ids = nb
        ident = g["id"]
        lst = {}
        for a in range(w.n):
            lst[int(ident[a])] = np.sort(ident[ids[off[a]:off[a + 1]]])
        out["_lists"] = lst
    ctx.close()
    return out


def oracle_run(w, steps=0, mode=oracle.GRID, params=None):
    orc = oracle.Oracle(params or w.params, star_info=w.star_params)
    st = oracle.OracleState(w.arrays)
    k = oracle.run_stages(orc, st, mode, want_kappa=True)
    if steps:
        oracle.step(orc, st, w.dt, steps, mode)
    out = dict(st.a)
    out.update(kappa_a=k["kappa_a"], kappa_u=k["kappa_u"], kappa_G=k["kappa_G"],
               offsets=k["offsets"], ids=k["ids"])
    return out


def rel_err(a, b, floor=0.0):
    return np.abs(a - b) / np.maximum(np.abs(b), floor)


def oracle_keys(o, n):
    """Sorted a * n + b over the oracle's ordered pairs (its lists are ascending, by id)."""
    off, ids = o["offsets"], o["ids"]
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(off))
    return rows * n + ids.astype(np.int64)


def check_lists(g, o, n):
    off, ids = o["offsets"], o["ids"]
    bad = 0
    for a in range(n):
        if not np.array_equal(g["_lists"][a], ids[off[a]:off[a + 1]]):
            bad += 1
    return bad


def eval_errors(g, o, mu_scale=1.0):
    """Per-field worst error of one evaluation, each normalised as the parity criterion states."""
    e = {}
    for k in ("D", "rho", "P", "cs"):
        e[k] = float(np.max(rel_err(g[k], o[k], 1e-300)))
    ka = o["kappa_a"]
    for k in ("ax", "ay", "az"):
        e[k] = float(np.max(np.abs(g[k] - o[k]) / np.maximum(ka, 1e-300)))
    ku = o["kappa_u"]
    e["dudt"] = float(np.max(np.abs(g["dudt"] - o["dudt"]) / np.maximum(ku, 1e-300)))
    # stress rate: absolute error against the scale of its terms
    kG = o["kappa_G"] / np.maximum(o["D"], 1e-300)
    Snorm = np.sqrt((o["S"] ** 2).sum(0))
    mu = o["mu"]
    scale = (2 * mu + 4 * Snorm) * kG + np.sqrt((o["dSdt"] ** 2).sum(0))
    diff = np.sqrt(((g["dSdt"] - o["dSdt"]) ** 2).sum(0))
    e["dSdt"] = float(np.max(np.where(scale > 0, diff / np.maximum(scale, 1e-300), 0.0)))
    return e


def field_errors(g, o, keys):
    """max |gpu - oracle| / max |oracle| per field (state after time steps)."""
    e = {}
    for k in keys:
        a, b = g[k], o[k]
        e[k] = float(np.max(np.abs(a - b)) / max(float(np.max(np.abs(b))), 1e-300))
    return e


def step_errors(g, o, keys, dt, steps):
    """Per-field worst error of the state after `steps` time steps of size dt.  Pointwise fields
    (positions, h, u, D, S) are compared relative to the field's largest magnitude.  Sums with
    cancellation are compared against their summation bound, as in one evaluation (R14): the
    accelerations against max kappa_a, du/dt against max kappa_u, dS/dt against the scale of its
    terms.  Velocities integrate the accelerations, so their error is measured against
    max |v| + steps dt max kappa_a (roundoff of the summed terms, carried through the kicks).
    The kappas are those of the oracle's evaluation at t = 0 (a few steps change them little)."""
    ka = float(np.max(o["kappa_a"]))
    ku = float(np.max(o["kappa_u"]))
    e = {}
    for k in keys:
        a, b = g[k], o[k]
        if k in ("ax", "ay", "az"):
            sc = max(ka, float(np.max(np.abs(b))))
        elif k == "dudt":
            # at t = 0 a state at rest has kappa_u = 0; the rate after steps is its own scale then
            sc = max(ku, float(np.max(np.abs(b))))
        elif k == "dSdt":
            kG = o["kappa_G"] / np.maximum(o["D"], 1e-300)
            Snorm = np.sqrt((o["S"] ** 2).sum(0))
            sc = float(np.max((2 * o["mu"] + 4 * Snorm) * kG + np.sqrt((b ** 2).sum(0))))
        elif k in ("vx", "vy", "vz"):
            sc = float(np.max(np.abs(b))) + steps * dt * ka
        else:
            sc = float(np.max(np.abs(b)))
        e[k] = float(np.max(np.abs(a - b)) / max(sc, 1e-300))
    return e
