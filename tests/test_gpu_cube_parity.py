"""Peel-off cubes (Sect. 5.1, the peeling product) against the oracle, per
element and per bin:

* a thin dusty sphere, where the double path follows the oracle packet by
  packet: the cube equals the oracle's element by element to 1e-12
  (relative; the deposits differ only by rounding and the order of the
  additions);
* the dusty-sphere configuration (287,064 leaves, 128x128x100 cube) at a
  reduced line-centre optical depth, both precisions: per pixel block of
  the image, per spectral bin, per cell of a coarse cube and per annulus of
  the radial profile, two-sample z from the spread of independent packet
  ranges (|z| <= 3 allowing 1% of bins over), and a KS test of the
  escaped packets' radii projected on the image plane."""
import numpy as np
import pytest
from scipy import stats

from paper_2001_11252_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rmc():
    from paper_2001_11252_amd import rmc as R
    return R


def s0(orc):
    return lambda ln, T: orc.line_quantities(ln, T)["sigma0"]


def _runs(idx_ok):
    """Contiguous runs [a, b) of the True entries of a boolean array."""
    d = np.diff(np.concatenate([[0], idx_ok.astype(int), [0]]))
    return list(zip(np.nonzero(d == 1)[0], np.nonzero(d == -1)[0]))


def test_fp64_thin_cube_equals_oracle_element_by_element(rmc, orc):
    n, seed = 6000, 41
    pb = W.static_sphere(s0(orc), 4.0, 1e4, n, level=4, tau_dust=0.4)
    pb.gas.v[:] = np.random.default_rng(6).standard_normal((pb.mesh.n, 3)) * 15e5
    pb.observers = [W.Observer((0.0, 0.0, 1.0), 24, 24, 30, (-0.5, 0.5, -0.5, 0.5), -12, 12),
                    W.Observer((0.6, 0.0, 0.8), 16, 16, 20, (-0.5, 0.5, -0.5, 0.5), -12, 12)]
    ctx = rmc.Context.from_problem(pb, "fp64")
    ctx.run(seed, 0, n)
    out = ctx.get_packets()
    ref = orc.run(pb, seed, threads=0, with_cubes=False)
    same = (out["status"] == ref["status"]) & (out["n_scat"] == ref["n_scat"])
    same &= np.abs(out["x"] - ref["x"]) < 1e-9
    same &= np.all(np.abs(out["pos"] - ref["pos"]) < 1e-12, axis=1)
    assert same.mean() > 0.99, same.mean()
    # cubes of exactly the packets that agree: runs over the matching ranges
    ctx.reset_cubes()
    co = [np.zeros((o.ny, o.nx, o.nbins)) for o in pb.observers]
    for a, b in _runs(same):
        ctx.run(seed, int(a), int(b - a))
        r = orc.run(pb, seed, first=int(a), n=int(b - a), threads=0)
        for i in range(2):
            co[i] += r["cubes"][i]
    for i in range(2):
        cg = ctx.get_cube(i)
        assert co[i].sum() > 0 and np.count_nonzero(co[i]) > 1000
        assert np.array_equal(cg > 0, co[i] > 0)
        # a deposit W P exp(-tau) carries the absolute error of tau, 2e-12 tau
        # at a relative optical depth error of 2e-12 (the two sides evaluate
        # the same closed forms with their own elementary functions, each
        # within 2 ulp, and round differently along each walk and each
        # peel-off ray's sum over leaves; observed up to 1.0e-12); an
        # element's tau is at most ln(w_max / value) (w_max = 2 bounds
        # P / 2 pi for HG at g = 0.73)
        nz = co[i] > 0
        rel = np.abs(cg[nz] - co[i][nz]) / co[i][nz]
        tol = 2e-12 * np.maximum(1.0, np.log(2.0 / co[i][nz]))
        worst = np.argsort(rel / tol)[-3:]
        print("observer", i, "rel/tol worst", (rel / tol)[worst], "rel", rel[worst], "value", co[i][nz][worst],
              "median rel", np.median(rel))
        assert np.all(rel <= tol), (rel.max(), (rel / tol).max())
        assert np.median(rel) < 1e-14


K = 20            # independent packet ranges per side
N = 20000         # packets per side


@pytest.fixture(scope="module")
def c2_reduced(orc):
    """The dusty-sphere configuration (full mesh and cube) at tau0 = 1e4 and
    the oracle's K packet ranges (peel-off rays stopped where exp(-tau)
    is zero, which leaves every deposit unchanged)."""
    pb = W.c2_dusty_sphere(s0(orc), n_packets=N, tau0=1e4)
    edges = np.linspace(0, N, K + 1).astype(int)
    cubes, esc = [], []
    for a, b in zip(edges[:-1], edges[1:]):
        r = orc.run(pb, 29, first=int(a), n=int(b - a), threads=0, peel_tau_cut=746.0)
        cubes.append(r["cubes"][0])
        esc.append(r["pos"][r["status"] == 1])
    return pb, np.array(cubes), esc


def _views(c):
    """Per-batch projections of a [K, 128, 128, 100] stack of cubes: 16x16
    image blocks, the 100-bin spectrum, an 8x8x10 coarse cube and the
    radial profile (16 annuli about the centre)."""
    k, ny, nx, nb = c.shape
    img = c.sum(axis=3)
    blocks = img.reshape(k, 16, ny // 16, 16, nx // 16).sum(axis=(2, 4)).reshape(k, -1)
    spec = c.sum(axis=(1, 2))
    coarse = c.reshape(k, 8, ny // 8, 8, nx // 8, 10, nb // 10).sum(axis=(2, 4, 6)).reshape(k, -1)
    yy, xx = np.mgrid[0:ny, 0:nx]
    r = np.hypot((xx + 0.5) / nx - 0.5, (yy + 0.5) / ny - 0.5)
    ring = np.minimum((r / 0.5 * 16).astype(int), 16)
    prof = np.stack([np.bincount(ring.ravel(), weights=im.ravel(), minlength=17)[:16] for im in img])
    return dict(image_blocks=blocks, spectrum=spec, coarse_cube=coarse, radial=prof)


# A batch reaches a bin with a deposit above this floor: the float cube
# holds nothing below ~1e-38 (and the float path cuts peel-off rays at
# optical depth 104), while the double path's deposits go down to 1e-323;
# at the line centre a quarter of the oracle's batches reach a bin only with
# deposits below the float range.
REACH = 1e-30


def _z_equiv(g, o):
    """Two-sample Welch t per bin over the batches, as the equivalent normal
    |z| (same two-sided p), for bins that at least three quarters of the
    batches of each side reach."""
    k = len(g)
    sel = ((g > REACH).sum(axis=0) >= 0.75 * k) & ((o > REACH).sum(axis=0) >= 0.75 * k)
    mg, mo = g[:, sel].mean(axis=0), o[:, sel].mean(axis=0)
    vg, vo = g[:, sel].var(axis=0, ddof=1) / k, o[:, sel].var(axis=0, ddof=1) / k
    t = (mg - mo) / np.sqrt(vg + vo)
    df = (vg + vo) ** 2 / (vg ** 2 / (k - 1) + vo ** 2 / (k - 1))
    p = 2 * stats.t.sf(np.abs(t), df)
    return stats.norm.isf(p / 2), sel.sum()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_c2_cube_per_bin_matches_oracle(rmc, orc, c2_reduced, prec):
    pb, oc, oesc = c2_reduced
    ctx = rmc.Context.from_problem(pb, prec)
    edges = np.linspace(0, N, K + 1).astype(int)
    gc, gesc = [], []
    for a, b in zip(edges[:-1], edges[1:]):
        ctx.reset_cubes()
        ctx.run(29, int(a), int(b - a))
        gc.append(ctx.get_cube(0))
        p = ctx.get_packets()
        gesc.append(p["pos"][p["status"] == 1])
    gv, ov = _views(np.array(gc)), _views(oc)
    summary, bad = {}, []
    for name in gv:
        z, nsel = _z_equiv(gv[name], ov[name])
        summary[name] = (int(nsel), int((z > 3).sum()), float(z.max()))
        # (spectrum: the double-peaked profile has 6 bins that every batch
        # reaches, 9 that three quarters of the oracle's batches reach)
        if nsel < {"image_blocks": 30, "spectrum": 6, "coarse_cube": 30, "radial": 10}[name]:
            bad.append((name, "too few bins"))
        if (z > 3).sum() > max(1, int(0.01 * nsel)) or z.max() >= 5:
            bad.append((name, "z"))
    print(prec, summary)
    k = len(gc)
    for side, v in (("gpu", gv["spectrum"]), ("oracle", ov["spectrum"])):
        reach = (v > REACH).sum(axis=0)
        on = np.nonzero(reach)[0]
        print(prec, side, "spectral bins reached (bin: batches of", k, "/ mean):",
              [(int(i), int(reach[i]), float(v[:, i].mean())) for i in on])
    assert not bad, (prec, bad, summary)
    # escaped packets: radius projected on the +z observer's image plane
    rg = np.concatenate([np.hypot(q[:, 0] - 0.5, q[:, 1] - 0.5) for q in gesc])
    ro = np.concatenate([np.hypot(q[:, 0] - 0.5, q[:, 1] - 0.5) for q in oesc])
    assert len(rg) > 500 and len(ro) > 500
    assert stats.ks_2samp(rg, ro).pvalue > 0.01
