"""GPU tests of the EoS surrogate network: gradients and forward pass against the oracle's FP64
network with the same weights (the matrix-core layers' rounded to BF16), training on the GPU and
the least-squares readout against the oracle's, the trust mask and table fallback, the density
stage with the surrogate against the oracle's table EoS, and what the trained network gains over
the table."""
import numpy as np
import pytest

import oracle
from sph_inputs import eos_table as E
from sph_inputs import workloads as W

from parity import gpu_run, oracle_run, rel_err

pytestmark = pytest.mark.gpu

BLOCKS = {"W1": (0, 128), "b1": (128, 192), "W2": (192, 4288), "b2": (4288, 4352), "W3": (4352, 8448),
          "b3": (8448, 8512), "W4": (8512, 8640), "b4": (8640, 8642)}
# BF16 activations (relative rounding 2^-9) feed the two 64x64 products; their effect on each
# gradient block stays a few 2^-9 in relative Frobenius norm
TOL_GRAD = 1e-2


def _ctx(n=2000):
    from paper_2107_07315_amd import sph
    w = W.pp_star(n, seed=4, eos="MLP")
    return sph, sph.Context(w.params, capacity=w.n), w


def _print(name, d):
    print(name, " ".join(f"{k}={v:.3e}" for k, v in d.items()), flush=True)


def _to_dev(a, dtype):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a, dtype=dtype), device="cuda")


@pytest.mark.parametrize("n", [64, 320])
def test_gradient_matches_oracle(n):
    sph, ctx, _ = _ctx()
    ctx.mlp_set_params(E.mlp_init(4))
    wr = ctx.mlp_get_params(rounded=True).astype(np.float64)
    rng = np.random.default_rng(n)
    x = rng.uniform(-1, 1, (n, 2)).astype(np.float32)
    t = rng.uniform(-1, 1, (n, 2)).astype(np.float32)
    g, loss = ctx.mlp_grad(_to_dev(x, np.float32), _to_dev(t, np.float32))
    lo, go = oracle.mlp_loss_grad(wr, x.astype(np.float64), t.astype(np.float64))
    err = {k: float(np.linalg.norm(g[a:b] - go[a:b]) / np.linalg.norm(go[a:b])) for k, (a, b) in BLOCKS.items()}
    _print(f"grad n={n}", err)
    assert abs(loss - lo) <= TOL_GRAD * lo
    for k, v in err.items():
        assert v < TOL_GRAD, (k, v)
    # the weights did not move
    assert np.array_equal(ctx.mlp_get_params(rounded=True), wr.astype(np.float32))


def _mask(lo, hi, p):
    return (p >= lo) & (p < hi)


def test_forward_matches_oracle_and_rounding():
    sph, ctx, _ = _ctx()
    w0 = E.mlp_init(7) * 3.0
    ctx.mlp_set_params(w0)
    wr = ctx.mlp_get_params(rounded=True)
    idx = np.arange(w0.size)
    mfma = _mask(*BLOCKS["W2"], idx) | _mask(*BLOCKS["W3"], idx)
    # the matrix-core weights are rounded to the nearest BF16 (8 significant bits): within half a
    # spacing, 2^-8 relative, and their FP32 patterns have zero low halves; the rest stay FP32
    assert np.all(np.abs(wr[mfma] - w0[mfma]) <= 2.0 ** -8 * np.abs(w0[mfma]))
    assert np.all((wr[mfma].view(np.uint32) & 0xffff) == 0)
    assert np.array_equal(wr[~mfma], w0[~mfma].astype(np.float32))
    nm = ctx.mlp_get_norm()
    rng = np.random.default_rng(8)
    xs = rng.uniform(-1, 1, (777, 2))      # a ragged count: 12 waves and a partial one
    lnr = (xs[:, 0] + 1) / nm[2] + nm[0]
    lnu = (xs[:, 1] + 1) / nm[3] + nm[1]
    lp, lc = ctx.mlp_eval(_to_dev(lnr, np.float64), _to_dev(lnu, np.float64))
    yg = np.stack([(lp.cpu().numpy() - nm[4]) / nm[6], (lc.cpu().numpy() - nm[5]) / nm[7]], 1)
    xo = np.stack([(lnr - nm[0]) * nm[2] - 1, (lnu - nm[1]) * nm[3] - 1], 1).astype(np.float32).astype(np.float64)
    yo = oracle.mlp_forward(wr.astype(np.float64), xo)
    err = float(np.max(np.abs(yg - yo)) / np.max(np.abs(yo)))
    print("forward rel err", err, flush=True)
    # FP32 arithmetic with the activations carried as two BF16 parts (about 2^-17 each)
    assert err < 1e-4


# The network's domain: the densest polytrope piece of the benchmark star (its central third of
# the particles by count), from the first table node above the dividing density to 1.15 rho_c,
# in a band of +-0.045 in ln u around the cold curve.
def _domain():
    pp = E.default_pp()
    lo, hi, wd = E.piece_band(pp, 2, W.PP_RHOC, W.pp_table(), 0.045)
    return pp, lo, hi, wd, E.band_domain(pp, lo, hi, wd)


@pytest.fixture(scope="module")
def trained():
    """A network trained on the GPU as configured for the 2M-particle runs: 1M seeded samples in
    the band (10% held out), Adam with a cosine schedule from lr 1e-3, batch 4096, 400 epochs
    (about 88k steps, a few seconds), then the least-squares readout."""
    import torch
    sph, ctx, w = _ctx(20000)
    pp, lo, hi, wd, dom = _domain()
    ctx.mlp_set_domain(*dom)
    ctx.mlp_set_params(E.mlp_init(4))
    samples = _to_dev(E.mlp_band_samples(pp, lo, hi, wd, 1_000_000, 4), np.float64)
    before = ctx.mlp_grad(*_holdout_pairs(ctx, samples))[1]
    hist = ctx.mlp_train(samples, 100_000, 400, 4096, 1e-3)
    after_lsq = ctx.mlp_fit_readout(samples, 100_000, 1e-12)
    torch.cuda.synchronize()
    return sph, ctx, w, samples, before, hist, after_lsq, dom


def _holdout_pairs(ctx, samples, k=4096):
    """Normalised (x, t) of the last k samples, targets from the table (numpy bilinear)."""
    tab = W.pp_table()
    nm = ctx.mlp_get_norm()
    s = samples[-k:].cpu().numpy()
    x = np.stack([(s[:, 0] - nm[0]) * nm[2] - 1, (s[:, 1] - nm[1]) * nm[3] - 1], 1)
    t = np.stack([(_bil(tab.lnP, tab, s[:, 0], s[:, 1]) - nm[4]) / nm[6],
                  (_bil(tab.lncs2, tab, s[:, 0], s[:, 1]) - nm[5]) / nm[7]], 1)
    return _to_dev(x, np.float32), _to_dev(t, np.float32)


def _bil(T, tab, lnr, lnu, lnr0=None, dlnr=None, lnu0=None, dlnu=None):
    lnr0 = tab.lnr0 if lnr0 is None else lnr0
    dlnr = tab.dlnr if dlnr is None else dlnr
    lnu0 = tab.lnu0 if lnu0 is None else lnu0
    dlnu = tab.dlnu if dlnu is None else dlnu
    fr = (lnr - lnr0) / dlnr
    fu = (lnu - lnu0) / dlnu
    i = np.clip(np.floor(fr).astype(int), 0, T.shape[0] - 2)
    j = np.clip(np.floor(fu).astype(int), 0, T.shape[1] - 2)
    a, b = fr - i, fu - j
    return (1 - a) * ((1 - b) * T[i, j] + b * T[i, j + 1]) + a * ((1 - b) * T[i + 1, j] + b * T[i + 1, j + 1])


def test_training_reduces_holdout_loss(trained):
    sph, ctx, w, samples, before, hist, after_lsq, dom = trained
    print("loss before", before, "history", hist[[0, 9, 99, 399]].tolist(), "after the readout fit", after_lsq,
          flush=True)
    assert np.all(np.isfinite(hist))
    assert hist[-1, 1] < before / 1e4
    assert hist[-1, 1] < hist[0, 1]
    # the least-squares readout does not lose on the held-out samples
    assert after_lsq <= 1.05 * hist[-1, 1]
    after = ctx.mlp_grad(*_holdout_pairs(ctx, samples))[1]
    assert after_lsq / 3 < after < 3 * after_lsq   # the same holdout metric on a subset


def test_readout_fit_matches_oracle():
    # the device's normal-equation readout against the oracle's (its FP64 features of the same
    # hidden layers, numpy's solve) on the same normalised samples and table targets: the two fitted
    # networks agree on held-out points to well below the 1e-4 the network serves at
    import torch
    sph, ctx, w = _ctx()
    pp, lo, hi, wd, dom = _domain()
    ctx.mlp_set_domain(*dom)
    ctx.mlp_set_params(E.mlp_init(5) * 1.5)
    samples = _to_dev(E.mlp_band_samples(pp, lo, hi, wd, 24_000, 9), np.float64)
    ctx.mlp_fit_readout(samples, 4096, 1e-12)
    torch.cuda.synchronize()
    wg = ctx.mlp_get_params(rounded=True).astype(np.float64)
    x_all, t_all = _holdout_pairs(ctx, samples, 24_000)
    x_all = x_all.cpu().numpy().astype(np.float64)
    t_all = t_all.cpu().numpy().astype(np.float64)
    wo = oracle.mlp_fit_readout(wg, x_all[:-4096], t_all[:-4096], 1e-12)
    # the hidden layers are the device's, the readout the fit's
    yg = oracle.mlp_forward(wg, x_all[-4096:])
    yo = oracle.mlp_forward(wo, x_all[-4096:])
    nm = ctx.mlp_get_norm()
    d = np.max(np.abs(yg - yo) * np.array([nm[6], nm[7]]))   # in ln P, ln c_s^2
    print("readout fit: device vs oracle max |d ln| =", d, flush=True)
    assert d < 1e-5


def _cells_in(dom):
    tab = W.pp_table()
    i = np.arange(tab.lnP.shape[0] - 1)
    j = np.arange(tab.lnP.shape[1] - 1)
    e = 1e-9
    ri = (tab.lnr0 + i * tab.dlnr >= dom[0] - e * tab.dlnr) & (tab.lnr0 + (i + 1) * tab.dlnr <= dom[1] + e * tab.dlnr)
    uj = (tab.lnu0 + j * tab.dlnu >= dom[2] - e * tab.dlnu) & (tab.lnu0 + (j + 1) * tab.dlnu <= dom[3] + e * tab.dlnu)
    return int(ri.sum()) * int(uj.sum())


def test_trust_mask_and_fallback(trained):
    sph, ctx, w, samples, before, hist, after_lsq, dom = trained
    counts = {tol: ctx.mlp_build_trust_mask(tol) for tol in (1e-4, 3e-2, 1e300)}
    print("trusted cells", counts, "cells in the domain", _cells_in(dom), flush=True)
    assert counts[1e300] == _cells_in(dom)          # every cell in the domain is tested, none outside
    assert 0 < counts[1e-4] <= counts[3e-2] <= counts[1e300]
    # density stage with the surrogate (FP64 pairs) against the table path: untrusted cells are
    # the table bit for bit, trusted ones within the tolerance
    for tol in (1e-4, 3e-2):
        ctx.mlp_build_trust_mask(tol)
        st = sph.DeviceState(w.arrays)
        ctx.evaluate(st)
        ctx.sph_sync()
        g = st.numpy(["P", "cs", "D", "id"])
        ref = gpu_run(w, params=w.params.replace(eos="TABLE"))
        o = np.argsort(g["id"])
        r = np.abs(g["P"][o] / ref["P"] - 1)
        rc = np.abs((g["cs"][o] / ref["cs"]) ** 2 - 1)
        assert np.array_equal(g["D"][o], ref["D"])
        print(f"tol {tol}: particles on the network {np.mean(r > 0):.4f}, max rel dP {r.max():.2e}", flush=True)
        assert np.mean(r > 0) > 0.01
        assert r.max() <= tol and rc.max() <= tol


def test_surrogate_path_meets_oracle_tolerance(trained):
    # the whole FP32-pairs + surrogate path against the FP64 oracle with the table EoS: at the
    # 1e-4 threshold the network serves a stated share of the particles (those in trusted cells
    # of its domain, the star's dense core), and D, rho, P stay within 1e-4 of the oracle
    sph, ctx, w, samples, before, hist, after_lsq, dom = trained
    o = oracle_run(w, params=w.params.replace(eos="TABLE", precision="FP64"))
    p32 = w.params.replace(precision="FP32")
    from paper_2107_07315_amd import sph as S
    st = sph.DeviceState(w.arrays)
    c32 = S.Context(p32, capacity=w.n)
    c32.mlp_set_domain(*dom)
    c32.mlp_set_params(ctx.mlp_get_params())
    cells = c32.mlp_build_trust_mask(1e-4)
    c32.evaluate(st)
    c32.sph_sync()
    served = c32.mlp_count_served(st)
    g = st.numpy()
    c32.close()
    order = np.argsort(g["id"])
    e = {k: float(np.max(rel_err(g[k][order], o[k], 1e-300))) for k in ("D", "rho", "P")}
    _print(f"FP32+MLP at 1e-4: trusted cells {cells}, particles on the network {served} of {w.n}", e)
    assert served > 0.05 * w.n
    assert e["D"] < 1e-4 and e["rho"] < 1e-4 and e["P"] < 1e-4


@pytest.mark.parametrize("prec", ["FP32", "FP64"])
def test_courant_step_with_the_network(trained, prec):
    # dt <= 0 while the network serves particles: the step is cfl min h / (c_L + |v|) over all the
    # particles of the evaluation before it, those finished by the table pass and by the network
    # pass alike (every workgroup and wave of both passes leaves its minimum)
    sph, ctx, w, samples, before, hist, after_lsq, dom = trained
    from paper_2107_07315_amd import sph as S
    p = w.params.replace(precision=prec)
    c = S.Context(p, capacity=w.n)
    c.mlp_set_domain(*dom)
    c.mlp_set_params(ctx.mlp_get_params())
    c.mlp_build_trust_mask(1e-4)
    st = sph.DeviceState(w.arrays)
    c.evaluate(st)
    c.sph_sync()
    served = c.mlp_count_served(st)
    a = st.numpy()
    c.sph_step(st, 0.0, 1)
    t = c.sph_get_time()
    c.sph_sync()
    c.close()
    solid = (a["type"] == 1) & ~((a["broken"] != 0) & (p.break_mode == "FLUIDIZE"))
    mu = np.where(solid, p.mu_pfactor * a["P"] if p.mu_mode == "PFACTOR" else p.mu_const, 0.0)
    cl = np.sqrt(a["cs"] * a["cs"] + 4.0 * mu / (3.0 * a["rho"]))
    vm = np.sqrt(a["vx"] * a["vx"] + a["vy"] * a["vy"] + a["vz"] * a["vz"])
    want = p.cfl * float(np.min(a["h"] / (cl + vm)))
    print(f"{prec} Courant step with the network serving {served} of {w.n}: {t:.17g} (host {want:.17g})", flush=True)
    assert served > 0.05 * w.n
    assert abs(t / want - 1) < 1e-14


def test_surrogate_gain_is_measured(trained):
    """What the trained network gains over the table it replaces, and what it costs, in its
    domain: the EoS from 17 KB of weights instead of the 16 MB table (970x less memory), at about
    1e-5 median relative error against it; a bilinear table of the network's size over the same
    domain (34 x 34 nodes of FP64 ln P and ln c_s^2, 18.5 KB) for comparison; and the density
    epilogue's time per evaluation with the network (serving its share at 1e-4) and with the
    table."""
    sph, ctx, w, samples, before, hist, after_lsq, dom = trained
    tab = W.pp_table()
    s = samples[-40_000:]
    lp, lc = ctx.mlp_eval(s[:, 0].contiguous(), s[:, 1].contiguous())
    sn = s.cpu().numpy()
    ref_p = _bil(tab.lnP, tab, sn[:, 0], sn[:, 1])
    ref_c = _bil(tab.lncs2, tab, sn[:, 0], sn[:, 1])
    e_net = np.maximum(np.abs(np.expm1(lp.cpu().numpy() - ref_p)), np.abs(np.expm1(lc.cpu().numpy() - ref_c)))
    # the small table: 34 x 34 nodes over the domain box, node values from the big table
    k = 34
    gr = np.linspace(dom[0], dom[1], k)
    gu = np.linspace(dom[2], dom[3], k)
    R, U = np.meshgrid(gr, gu, indexing="ij")
    small_p = _bil(tab.lnP, tab, R.ravel(), U.ravel()).reshape(k, k)
    small_c = _bil(tab.lncs2, tab, R.ravel(), U.ravel()).reshape(k, k)
    dr, du = gr[1] - gr[0], gu[1] - gu[0]
    e_small = np.maximum(np.abs(np.expm1(_bil(small_p, tab, sn[:, 0], sn[:, 1], dom[0], dr, dom[2], du) - ref_p)),
                         np.abs(np.expm1(_bil(small_c, tab, sn[:, 0], sn[:, 1], dom[0], dr, dom[2], du) - ref_c)))
    from paper_2107_07315_amd import sph as S
    ms = {}
    served = None
    for mode in ("table", "network"):
        c = S.Context(w.params.replace(precision="FP32", eos="MLP" if mode == "network" else "TABLE"), capacity=w.n)
        if mode == "network":
            c.mlp_set_domain(*dom)
            c.mlp_set_params(ctx.mlp_get_params())
            c.mlp_build_trust_mask(1e-4)
        st = sph.DeviceState(w.arrays)
        c.evaluate(st)
        if mode == "network":
            served = c.mlp_count_served(st)
        c.sph_set_timing(True)
        for _ in range(20):
            c.sph_density(st)
        c.sph_sync()
        n, t = c.sph_get_timing("eos")
        ms[mode] = t / n
        c.close()
    net_bytes = 2 * 8642
    table_bytes = tab.lnP.nbytes + tab.lncs2.nbytes
    rep = {"compression": table_bytes / net_bytes, "net_median": float(np.median(e_net)),
           "net_p90": float(np.percentile(e_net, 90)), "net_max": float(np.max(e_net)),
           "small_table_median": float(np.median(e_small)), "small_table_p90": float(np.percentile(e_small, 90)),
           "served": served, "epilogue_ms_table": ms["table"], "epilogue_ms_network": ms["network"]}
    _print("gain", rep)
    assert np.all(np.isfinite(e_net))
    assert rep["compression"] > 900
    assert rep["net_median"] < 5e-5
    assert rep["epilogue_ms_network"] > 0 and rep["epilogue_ms_table"] > 0
