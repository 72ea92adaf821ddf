"""Fluorescent decay channels on the GPU (Sect. 3.2.1, Fe II UV1 of
Table 1), against the oracle.

* an optically thin Fe II 2587 sphere (two channels): double-path packets
  follow the oracle one by one; the float path's first decays split among
  the channels as A_j / sum A; the peel-off weight at the fluorescent
  frequency is 1/(4 pi) per fluorescent packet;
* the Fe II wind of the paper's idealised-set-up example (2587 and 2600
  with their three channels, flat continuum 2570-2640 A, v ~ r to
  100 km/s, density ~ r^-3): double-path packets follow the oracle one by
  one, and the float path's spectrum shows the blue-shifted absorption of
  the two resonances and emission at the three fluorescent wavelengths."""
import numpy as np
import pytest

from paper_2001_11252_amd import workloads as W

pytestmark = pytest.mark.gpu
C_CM = 2.99792458e10


@pytest.fixture(scope="module")
def rmc():
    from paper_2001_11252_amd import rmc as R
    return R


def s0(orc):
    return lambda ln, T: orc.line_quantities(ln, T)["sigma0"]


def _same(ref, out, i, tol_pos=None):
    tol = tol_pos if tol_pos is not None else 1e-13 + 1e-15 * float(out["n_scat"][i])
    return (ref["status"][i] == out["status"][i] and ref["n_scat"][i] == out["n_scat"][i]
            and abs(ref["x"][i] - out["x"][i]) < 1e-9 * max(1.0, abs(ref["x"][i]))
            and np.abs(ref["pos"][i] - out["pos"][i]).max() < tol)


def _channel_x(orc, line, j):
    b = orc.line_quantities(line, 1e4)["vth"] / C_CM
    lam = line.fluor[j][0]
    return (line.lambda0_A - lam) / (lam * b)


def test_thin_sphere_packets_channels_and_peel_off(rmc, orc):
    line = W.FEII_2587
    # double path, one by one (tau0 = 3: a few resonant scatterings first)
    n = 2000
    pb = W.static_sphere(s0(orc), 3.0, 1e4, n, level=2, line=line)
    c = rmc.Context.from_problem(pb, "fp64", observers=False)
    c.run(101, 0, n)
    out = c.get_packets()
    c.close()
    ref = orc.run(pb, 101, threads=8, with_cubes=False)
    same = sum(_same(ref, out, i) for i in range(n))
    assert same >= n - 2, same
    # float path: first decays by channel
    n = 200000
    pb = W.static_sphere(s0(orc), 0.4, 1e4, n, level=2, line=line)
    xs = [_channel_x(orc, line, j) for j in range(2)]
    pb.observers = [W.Observer((0.0, 0.0, 1.0), 4, 4, 40, (-0.5, 0.5, -0.5, 0.5), xs[0] - 20.0, xs[0] + 20.0)]
    c = rmc.Context.from_problem(pb, "fp32")
    c.run(102, 0, n)
    out = c.get_packets()
    cube = c.get_cube(0)
    c.close()
    hit = out["n_scat"] >= 1
    m = hit.sum()
    a_tot = line.A_ul + sum(a for _, a in line.fluor)
    for j, (_, a) in enumerate(line.fluor):
        p = a / a_tot
        k = ((np.abs(out["x"] - xs[j]) < 20) & (out["n_scat"] == 1)).sum()
        z = (k - m * p) / np.sqrt(m * p * (1 - p))
        assert abs(z) < 4, (j, z)
    # peel-off at channel 0's frequency: 1/(4 pi) per fluorescent packet
    # (float cube: ~3e4 atomic additions into bins of up to ~30)
    nf = (np.abs(out["x"] - xs[0]) < 20).sum()
    assert abs(cube.sum() / (nf / (4 * np.pi)) - 1) < 1e-4


def test_fe_ii_wind(rmc, orc):
    s = s0(orc)
    # double path against the oracle, one by one
    n = 3000
    pb = W.feii_wind(s, n)
    c = rmc.Context.from_problem(pb, "fp64", observers=False)
    c.run(103, 0, n)
    out = c.get_packets()
    c.close()
    ref = orc.run(pb, 103, threads=8, with_cubes=False)
    assert out["n_scat"].max() > 20
    # status, scattering count and frequency as tight as before; positions to
    # 1e-10: in the r^-3 wind the optical depth left on reaching the event's
    # cell is the draw minus many nearly equal segment depths, so the last-ulp
    # opacity differences of the two sides move an event by up to ~1e-10
    same = sum(_same(ref, out, i, tol_pos=1e-10) for i in range(n))
    assert same >= n - 3, same
    # float path: the spectrum of the paper's figure
    n = 400000
    pb = W.feii_wind(s, n)
    c = rmc.Context.from_problem(pb, "fp32", observers=False)
    c.run(104, 0, n)
    out = c.get_packets()
    c.close()
    assert np.all(out["status"] == 1)
    b = np.sqrt(2 * 1.380649e-16 * pb.T_ref / (W.M_FE_AMU * 1.66053907e-24)) / C_CM
    lam = W.FEII_2587.lambda0_A / (1.0 + b * out["x"])
    h, edges = np.histogram(lam, bins=np.arange(2570.0, 2640.01, 0.5))
    mid = 0.5 * (edges[1:] + edges[:-1])
    cont = h[(mid > 2572) & (mid < 2584)].mean()
    # absorption just blueward of each resonance (outflow up to 100 km/s ~ 0.9 A)
    for lam0 in (2586.65, 2600.17):
        trough = h[(mid > lam0 - 1.0) & (mid < lam0)].mean()
        assert trough < 0.5 * cont, (lam0, trough, cont)
    # fluorescent emission at the three channel wavelengths
    for lamf in (2612.65, 2626.45, 2632.11):
        peak = h[np.abs(mid - lamf) < 0.6].max()
        assert peak > cont + 6 * np.sqrt(cont), (lamf, peak, cont)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_batch_with_a_fluorescent_problem_equals_single_runs(rmc, orc, prec):
    # the batch runs the multi-line kernel for both problems; each problem's
    # packets depend only on the problem and their index
    s = s0(orc)
    pbs = [W.static_sphere(s, 3.0, 1e4, 3000, level=2, line=W.FEII_2587), W.c1_slab(s, n_packets=500)]
    seeds = [111, 112]
    npk = [3000, 500]
    single = []
    for p, sd, n in zip(pbs, seeds, npk):
        c = rmc.Context.from_problem(p, prec, observers=False)
        c.run(sd, 0, n)
        single.append(c.get_packets())
        c.close()
    ctxs = [rmc.Context.from_problem(p, prec, observers=False) for p in pbs]
    rmc.batch_run(ctxs, seeds, npk)
    for c, ref in zip(ctxs, single):
        out = c.get_packets()
        for k in ("status", "x", "n_scat", "pos", "k"):
            assert np.array_equal(out[k], ref[k]), k
        c.close()
