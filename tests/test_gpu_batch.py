"""GPU batched launch (many uneven problems in one persistent, graph-
replayed launch): per-packet results equal to running each problem on its
own, parity of each problem with the oracle, and the autotuner."""
import numpy as np
import pytest
from scipy import stats

from paper_2001_11252_amd import workloads as W

pytestmark = pytest.mark.gpu


def _small_batch(orc, n=12, seed=0x5EED0004, packet_scale=0.02, work_cap=2e7):
    # C4's mix (slab/sphere, Lya/MgII doublet, lognormal n_HI, uneven grids
    # and packet counts) at tau0 <= 1e4 so that each packet's walk stays short
    s0 = lambda ln, T: orc.line_quantities(ln, T)["sigma0"]
    return W.c4_batch(s0, n_problems=n, seed=seed, work_cap=work_cap, packet_scale=packet_scale, max_level=5,
                      log_tau_range=(3.0, 4.0))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_batch_equals_single_runs(orc, prec):
    from paper_2001_11252_amd import rmc
    probs = _small_batch(orc)
    ctxs = [rmc.Context.from_problem(p, prec) for p in probs]
    npk = [len(p.sources.x) for p in probs]
    seeds = [p.seed for p in probs]
    per, tot = rmc.batch_run(ctxs, seeds, npk)
    assert tot["emitted"] == sum(npk)
    outs = [c.get_packets() for c in ctxs]
    for p, c, o, st, n in zip(probs, ctxs, outs, per, npk):
        assert st["emitted"] == n and st["escaped"] + st["absorbed"] + st["stuck"] == n
        single = rmc.Context.from_problem(p, prec)
        s1 = single.run(p.seed, 0, n)
        o1 = single.get_packets()
        for k in o:
            assert np.array_equal(o[k], o1[k]), (p.name, k)
        for k in ("scatterings", "crossings", "escaped", "absorbed"):
            assert st[k] == s1[k], (p.name, k)
    # the captured launch replays with the same results
    per2, _ = rmc.batch_run(ctxs, seeds, npk)
    for c, o in zip(ctxs, outs):
        o2 = c.get_packets()
        for k in o:
            assert np.array_equal(o[k], o2[k])


def test_batch_matches_oracle(orc):
    from paper_2001_11252_amd import rmc
    probs = _small_batch(orc, n=6, seed=77, packet_scale=1.0, work_cap=5e6)
    ctxs = [rmc.Context.from_problem(p, "fp32") for p in probs]
    npk = [len(p.sources.x) for p in probs]
    rmc.batch_run(ctxs, [p.seed for p in probs], npk)
    for p, c, n in zip(probs, ctxs, npk):
        g = c.get_packets()
        o = orc.run(p, p.seed)
        xg = g["x"][g["status"] == 1]
        xo = o["x"][o["status"] == 1]
        assert stats.ks_2samp(xg, xo).pvalue > 0.01, (p.name, p.meta)
        se = np.sqrt(g["n_scat"].var() / n + o["n_scat"].var() / n)
        assert abs(g["n_scat"].mean() - o["n_scat"].mean()) < 4 * se + 1e-9, p.name


def test_batch_autotune_picks_a_valid_shape(orc):
    from paper_2001_11252_amd import rmc
    probs = _small_batch(orc, n=8, seed=3)
    ctxs = [rmc.Context.from_problem(p, "fp32") for p in probs]
    npk = [len(p.sources.x) for p in probs]
    seeds = [p.seed for p in probs]
    best = rmc.batch_autotune(ctxs, seeds, npk, trial_slices=2)
    assert best["block"] in (64, 128, 256) and best["refill"] in (1, 8, 32) and best["slice_iters"] in (256, 2048, 8192)
    # the tuned run gives the same packets as an untuned one
    rmc.batch_run(ctxs, seeds, npk)
    tuned = [c.get_packets() for c in ctxs]
    ref = [rmc.Context.from_problem(p, "fp32") for p in probs]
    rmc.batch_run(ref, seeds, npk)
    for a, b in zip(tuned, ref):
        bb = b.get_packets()
        for k in a:
            assert np.array_equal(a[k], bb[k])


def test_batch_stream_equals_batch_run(orc):
    # the streaming form (begin, steps, end on the first context) gives the
    # packets and totals of one rmc_batch_run call
    from paper_2001_11252_amd import rmc
    probs = _small_batch(orc, n=10, seed=11)
    npk = [len(p.sources.x) for p in probs]
    seeds = [p.seed for p in probs]
    a = [rmc.Context.from_problem(p, "fp32") for p in probs]
    _, ta = rmc.batch_run(a, seeds, npk)
    b = [rmc.Context.from_problem(p, "fp32") for p in probs]
    b[0].set_option(rmc.OPT_SLICE_ITERS, 16)
    rmc.batch_begin(b, seeds, npk)
    steps, work = 0, 0
    while True:
        sl, rem = b[0].stream_step()
        steps += 1
        work += sl["scatterings"]
        if rem == 0:
            break
    tb = b[0].stream_end()
    assert steps > 2
    for k in ("emitted", "escaped", "absorbed", "scatterings", "crossings"):
        assert ta[k] == tb[k], k
    assert work == tb["scatterings"]
    for ca, cb in zip(a, b):
        pa, pb_ = ca.get_packets(), cb.get_packets()
        for k in pa:
            assert np.array_equal(pa[k], pb_[k]), k


@pytest.mark.parametrize("prec,compact", [("fp64", 1), ("fp32", 1), ("fp32", 0)])
def test_batch_with_observers_equals_single_runs(orc, prec, compact):
    # problems with different observer counts and line sets in one batch:
    # the deferred peel-off rays of every problem land in that problem's
    # cubes (queue entries carry their problem and observer), with the
    # batch's last packets gathered into fewer waves or not
    from paper_2001_11252_amd import rmc
    s0 = lambda ln, T: orc.line_quantities(ln, T)["sigma0"]
    probs = []
    for i, (tau0, nobs) in enumerate(((3e3, 1), (1e4, 2), (1e3, 3), (5e3, 2))):
        pb = W.static_sphere(s0, tau0, 1e4, 1500 + 500 * i, level=3 + i % 2, tau_dust=0.3)
        pb.gas.v[:] = np.random.default_rng(i).standard_normal((pb.mesh.n, 3)) * 10e5
        dirs = [(0.0, 0.0, 1.0), (0.6, 0.0, 0.8), (0.0, -0.8, 0.6)][:nobs]
        pb.observers = [W.Observer(d, 8, 8, 10, (-0.5, 0.5, -0.5, 0.5), -25, 25) for d in dirs]
        pb.seed = 100 + i
        probs.append(pb)
    npk = [len(p.sources.x) for p in probs]
    seeds = [p.seed for p in probs]
    ctxs = [rmc.Context.from_problem(p, prec) for p in probs]
    ctxs[0].set_option(rmc.OPT_SLICE_ITERS, 64)
    ctxs[0].set_option(rmc.OPT_COMPACT, compact)
    per, tot = rmc.batch_run(ctxs, seeds, npk)
    assert tot["peel_deferred"] > 0
    for p, c, st, n in zip(probs, ctxs, per, npk):
        single = rmc.Context.from_problem(p, prec)
        s1 = single.run(p.seed, 0, n)
        pa, pb_ = c.get_packets(), single.get_packets()
        for k in pa:
            assert np.array_equal(pa[k], pb_[k]), (p.name, k)
        for k in ("scatterings", "crossings", "peel_rays", "peel_crossings", "peel_dropped"):
            assert st[k] == s1[k], (p.name, k)
        for o in range(len(p.observers)):
            ca, cb = c.get_cube(o), single.get_cube(o)
            assert ca.sum() > 0
            assert np.allclose(ca, cb, rtol=1e-5 if prec == "fp32" else 1e-12, atol=0), (p.name, o)


def test_batch_autotune_leaves_the_cubes_alone(orc):
    # the tuner's trial launches deposit peel-off rays; it puts every
    # member's cubes back, so a later run adds to what they held before
    from paper_2001_11252_amd import rmc
    s0 = lambda ln, T: orc.line_quantities(ln, T)["sigma0"]
    probs = []
    for i, tau0 in enumerate((2e3, 5e3, 1e3)):
        pb = W.static_sphere(s0, tau0, 1e4, 1200, level=3, tau_dust=0.3)
        pb.observers = [W.Observer((0.0, 0.6, 0.8), 8, 8, 10, (-0.5, 0.5, -0.5, 0.5), -25, 25)]
        pb.seed = 300 + i
        probs.append(pb)
    npk = [len(p.sources.x) for p in probs]
    seeds = [p.seed for p in probs]
    a = [rmc.Context.from_problem(p, "fp64") for p in probs]
    rmc.batch_run(a, seeds, npk)
    before = [c.get_cube(0) for c in a]
    rmc.batch_autotune(a, seeds, npk, trial_slices=1)
    for c, cb in zip(a, before):
        assert np.array_equal(c.get_cube(0), cb)
    rmc.batch_run(a, seeds, npk)
    b = [rmc.Context.from_problem(p, "fp64") for p in probs]
    rmc.batch_run(b, seeds, npk)
    rmc.batch_run(b, seeds, npk)
    for ca, cb in zip(a, b):
        x, y = ca.get_cube(0), cb.get_cube(0)
        assert x.sum() > 0 and np.allclose(x, y, rtol=1e-12, atol=0)
