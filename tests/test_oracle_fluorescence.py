"""Fluorescent decay channels in the oracle (Sect. 3.2.1; Fe II UV1 data
from Table 1).

Pins, in optically thin Fe II spheres at 1e4 K with a central source at the
resonance (x = 0):
* the channel of each decay: the first decays of the packets that
  interacted go through fluorescent channel j with probability A_j / sum A
  (one channel for 2600, two for 2587);
* the fluorescent frequency: x - x_j = s_j (k_out . U) (U the atom velocity
  in thermal units, s_j = nu_j/nu_ref); absorbed at line centre, U is nearly
  perpendicular to k_in and Gaussian, and k_out is isotropic, so
  k_out . U = sqrt(1 - mu^2) g with g ~ N(0, 1/2): mean 0, variance 1/3,
  kurtosis 3.6;
* peel-off: the cube's weight at the fluorescent frequency is 1/(4 pi) per
  fluorescent event (isotropic re-emission), against the escaped packets."""
import numpy as np
import pytest

from paper_2001_11252_amd import workloads as W
from tests.analytic import golden

C_CM = 2.99792458e10


def _sphere(orc, line, n, tau0=0.4, observer=None):
    s0 = lambda ln, T: orc.line_quantities(ln, T)["sigma0"]
    pb = W.static_sphere(s0, tau0, 1e4, n, level=2, line=line)
    if observer:
        pb.observers = [observer]
    return pb


def _channel_x(orc, line, j):
    b = orc.line_quantities(line, 1e4)["vth"] / C_CM
    lam = line.fluor[j][0]
    return (line.lambda0_A - lam) / (lam * b), line.lambda0_A / lam


def test_table1_fe_ii_channels():
    rows = {r[0]: r[1:] for r in golden("fe_ii_uv1")}
    for ln in (W.FEII_2587, W.FEII_2600):
        assert (ln.lambda0_A, ln.A_ul, ln.f_lu) == tuple(rows[ln.name])
        for (lam, a), name in zip(ln.fluor, rows[ln.name + "_channels"][::2]):
            assert (lam, a) == tuple(rows[name])


@pytest.mark.parametrize("line", [W.FEII_2600, W.FEII_2587], ids=["2600", "2587"])
def test_decay_channel_fractions(orc, line):
    n = 60000
    pb = _sphere(orc, line, n)
    r = orc.run(pb, 5, threads=8, with_cubes=False)
    # a fluorescent photon is not absorbed again, so a packet whose first
    # decay was fluorescent ends with one interaction at that channel's
    # frequency; the first decays are those of every packet that interacted
    hit = r["n_scat"] >= 1
    m = hit.sum()
    assert m > 5000
    a_tot = line.A_ul + sum(a for _, a in line.fluor)
    x = r["x"]
    labels = np.full(n, -1)
    for j in range(len(line.fluor)):
        xj, _ = _channel_x(orc, line, j)
        labels[np.abs(x - xj) < 20] = j
    assert np.all((labels >= 0) | (np.abs(x) < 60))
    for j, (_, a) in enumerate(line.fluor):
        p = a / a_tot
        k = ((labels == j) & (r["n_scat"] == 1)).sum()
        z = (k - m * p) / np.sqrt(m * p * (1 - p))
        assert abs(z) < 4, (j, z)
    # and a fluorescent photon never interacts again
    assert np.all(r["n_scat"][labels >= 0] >= 1)


def test_fluorescent_frequency_distribution(orc):
    line = W.FEII_2600
    n = 60000
    pb = _sphere(orc, line, n)
    r = orc.run(pb, 6, threads=8, with_cubes=False)
    xj, sj = _channel_x(orc, line, 0)
    once = r["n_scat"] == 1
    d = (r["x"][once] - xj) / sj
    d = d[np.abs(d) < 20]
    m = len(d)
    assert m > 500
    var = np.mean(d ** 2)
    assert abs(d.mean()) < 4 * np.sqrt(1 / 3 / m)
    assert abs(var / (1 / 3) - 1) < 4 * np.sqrt(3.6 - 1) / np.sqrt(m) + 0.01
    kurt = np.mean(d ** 4) / var ** 2
    assert abs(kurt - 3.6) < 0.35


def test_fluorescent_peel_off_normalisation(orc):
    line = W.FEII_2600
    n = 40000
    xj, _ = _channel_x(orc, line, 0)
    ob = W.Observer((0.0, 0.0, 1.0), 4, 4, 40, (-0.5, 0.5, -0.5, 0.5), xj - 20.0, xj + 20.0)
    pb = _sphere(orc, line, n, observer=ob)
    r = orc.run(pb, 7, threads=8)
    fluor = np.abs(r["x"] - xj) < 20
    # each fluorescent packet deposited 1/(4 pi) (the sphere is transparent at
    # the fluorescent frequency); escaped packets sample the same events
    total = r["cubes"][0].sum()
    expect = fluor.sum() / (4 * np.pi)
    assert abs(total / expect - 1) < 1e-9


@pytest.mark.parametrize("name", ["SiII1190", "SiII1193", "SiII1260"])
def test_si_ii_lines_and_branching(orc, name):
    # Table 1 Si II data; a fluorescent channel stronger than the resonance
    # (1190 -> 1194: A_f / sum A = 0.84) still splits the first decays as A_j / sum A
    row = {r[0]: r[1:] for r in golden("si_ii")}[name]
    line = {"SiII1190": W.SIII_1190, "SiII1193": W.SIII_1193, "SiII1260": W.SIII_1260}[name]
    assert (line.lambda0_A, line.A_ul, line.f_lu) == tuple(row[:3])
    assert line.fluor == ((row[3], row[4]),)
    n = 40000
    r = orc.run(_sphere(orc, line, n), 8, threads=8, with_cubes=False)
    m = (r["n_scat"] >= 1).sum()
    xj = _channel_x(orc, line, 0)[0]
    k = ((np.abs(r["x"] - xj) < 20) & (r["n_scat"] == 1)).sum()
    p = row[4] / (row[1] + row[4])
    z = (k - m * p) / np.sqrt(m * p * (1 - p))
    assert abs(z) < 4, z
