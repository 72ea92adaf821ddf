"""Pins of one resonant scattering inside the oracle's transport loop
(Sect. 3.2.1), taken from packets stopped at their second interaction
(max_events = 2), so that the recorded frequency and direction are those
the first scattering produced:

* recoil: the outgoing-frequency relation nu_out = nu_in (1 + (k_out -
  k_in).v/c) / (1 + (1 - mu) h nu_in / (m c^2)) (Eq. for nu_out).  With the
  same draws, the runs with and without recoil differ only by its
  denominator, so the recoil run's frequency follows from the other one's
  and mu exactly; with isotropic phase the mean shift is -g_r <1 - mu> =
  -g_r, g_r = h nu0 / (m c v_th) (2.535e-4 for Lya at 1e4 K);
* the Lya core/wing switch: a scattering uses P_core when the frequency
  seen by the atom, nu_in (1 - k_in.v/c), lies within 0.2 Doppler widths
  of the line centre.  Which inverse CDF gave a packet's mu is read off its
  direction (the phase-function draw is a known uniform), and the fraction
  of core scatterings at x_in must equal the probability that the atom
  velocity u_par, drawn from its density f(u_par) (Eq. for f(u_par)), puts
  the atom-frame frequency x_in - u_par nu_in/nu_0 inside that window.

Every expected value is computed here from the paper's definitions and
CODATA constants; nothing is taken from the oracle but its outputs and the
uniform draws (pinned separately against the published Philox vectors)."""
from dataclasses import replace

import numpy as np
import pytest
from scipy import integrate
from scipy.special import wofz

from paper_2001_11252_amd import workloads as W

C = 2.99792458e10
H_PL = 6.62607015e-27
K_B = 1.380649e-16
AMU = 1.66053906660e-24
J_MU = 1   # slot of the phase-function uniform of an event (see the oracle's stream layout)


def _line_consts(line, T):
    nu0 = C / (line.lambda0_A * 1e-8)
    m = line.mass_amu * AMU
    vth = np.sqrt(2 * K_B * T / m)
    return nu0, vth, nu0 * vth / C, m


def _first_scatterings(orc, sigma0, x_in, T, n, seed, phase, recoil):
    """Packets from the centre of a very thick static sphere, each along
    its own direction, stopped at their second interaction: returns
    (k_in, k_out, x_out) of the first scattering."""
    line = replace(W.LYA, phase=phase, recoil=int(recoil))
    pb = W.static_sphere(sigma0, 1e10, T, n, level=0, line=line)
    rng = np.random.default_rng(seed)
    d = rng.standard_normal((n, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    pb.sources.dir = d
    pb.sources.x[:] = x_in
    r = orc.run(pb, seed, threads=8, max_events=2, with_cubes=False)
    assert np.all(r["status"] == 3) and np.all(r["n_scat"] == 1)
    return d, r["k"], r["x"]


@pytest.mark.parametrize("phase,x_in", [(W.PHASE_ISO, 0.0), (W.PHASE_ISO, 2.5), (W.PHASE_LYA, 0.7)])
def test_recoil_follows_the_outgoing_frequency_relation(orc, sigma0_oracle, phase, x_in):
    T, n, seed = 1e4, 20000, 31
    kin, k1, x1 = _first_scatterings(orc, sigma0_oracle, x_in, T, n, seed, phase, True)
    _, k0, x0 = _first_scatterings(orc, sigma0_oracle, x_in, T, n, seed, phase, False)
    # recoil enters only the outgoing frequency: the draws and directions agree
    assert np.array_equal(k1, k0)
    mu = np.sum(kin * k1, axis=1)
    nu0, vth, dnu, m = _line_consts(W.LYA, T)
    nu_in = nu0 + x_in * dnu
    r = (1 - mu) * H_PL * nu_in / (m * C * C)
    # nu_rec = nu_norec / (1 + r); in Doppler units of the static gas
    x_pred = (x0 - r * nu0 / dnu) / (1 + r)
    assert np.max(np.abs(x1 - x_pred)) < 1e-10
    # the recoil parameter and the mean shift per scattering
    g_r = H_PL * nu0 / (m * C * vth)
    assert abs(g_r / 2.535e-4 - 1) < 1e-3
    shift = x1 - x0
    se = shift.std() / np.sqrt(n)
    # to first order in h nu / m c^2 (the exact relation is checked above)
    expect = -g_r * (nu_in / nu0) * np.mean(1 - mu)
    assert abs(shift.mean() - expect) < 1e-4 * g_r
    if phase == W.PHASE_ISO:
        # isotropic: <1 - mu> = 1
        assert abs(shift.mean() + g_r * nu_in / nu0) < 3 * se


def _cdf_core(mu):
    # integral of P_core = 11/24 + 3 mu^2/24 from -1
    return 11.0 / 24.0 * (mu + 1) + (mu ** 3 + 1) / 24.0


def _cdf_wing(mu):
    # integral of P_wing = 3 (1 + mu^2) / 8 from -1
    return 3.0 / 8.0 * ((mu + 1) + (mu ** 3 + 1) / 3.0)


def _invert(cdf, r):
    lo, hi = -np.ones_like(r), np.ones_like(r)
    for _ in range(64):
        mid = 0.5 * (lo + hi)
        below = cdf(mid) < r
        lo = np.where(below, mid, lo)
        hi = np.where(below, hi, mid)
    return 0.5 * (lo + hi)


def _core_probability(x, a, b):
    """P(|x - u (1 + b x)| < 0.2) for u ~ f(u) of Eq. f(u_par): the window
    integral by quadrature, the normalisation (pi/a) H(a,x) from the
    Faddeeva function."""
    f = lambda u: np.exp(-u * u) / (a * a + (x - u) ** 2)
    lo, hi = (x - 0.2) / (1 + b * x), (x + 0.2) / (1 + b * x)
    pts = [x] if lo < x < hi else None
    num, _ = integrate.quad(f, lo, hi, points=pts, limit=500, epsabs=0, epsrel=1e-11)
    norm = np.pi / a * wofz(x + 1j * a).real
    return num / norm


# 1e4 K (a = 4.7e-4): the fraction is set by whether the atom is resonant
# (atom-frame frequency), 10 K (a = 0.015): the Lorentzian tail makes it
# depend on the 0.2 width itself (next test)
@pytest.mark.parametrize("T,x_in", [(1e4, 0.0), (1e4, 1.0), (1e4, 3.0), (1e4, 4.0),
                                    (10.0, 0.0), (10.0, 0.3), (10.0, 1.0), (10.0, 2.0), (10.0, 3.0)])
def test_lya_core_wing_switch_at_02_doppler_widths(orc, sigma0_oracle, T, x_in):
    n, seed = 40000, 53 + int(10 * x_in) + int(T)
    kin, k1, _ = _first_scatterings(orc, sigma0_oracle, x_in, T, n, seed, W.PHASE_LYA, False)
    mu = np.sum(kin * k1, axis=1)
    ru = np.array([orc.uniform(seed, i, 1, J_MU) for i in range(n)])
    mc, mw = _invert(_cdf_core, ru), _invert(_cdf_wing, ru)
    dc, dw = np.abs(mu - mc), np.abs(mu - mw)
    # every packet's mu is one of the two inverses of its uniform
    assert np.all(np.minimum(dc, dw) < 1e-12)
    ok = np.abs(mc - mw) > 1e-9
    core = (dc < dw)[ok]
    nu0, vth, dnu, m = _line_consts(W.LYA, T)
    a = orc.line_quantities(W.LYA, T)["a"]
    p = _core_probability(x_in, a, vth / C)
    f = core.mean()
    assert abs(f - p) < 3 * np.sqrt(p * (1 - p) / core.size) + 1e-5, (f, p)


def _window_probability(x, a, w):
    f = lambda u: np.exp(-u * u) / (a * a + (x - u) ** 2)
    num, _ = integrate.quad(f, x - w, x + w, points=[x], limit=500)
    return num / (np.pi / a * wofz(x + 1j * a).real)


def test_core_probability_is_sensitive_to_the_threshold():
    # at 10 K a width of 0.1 or 0.3 instead of 0.2 Doppler widths moves the
    # core fraction far beyond the binomial error of the test above
    a = 1.49e-2
    for x in (0.0, 1.0, 2.0):
        p2 = _window_probability(x, a, 0.2)
        sig = np.sqrt(p2 * (1 - p2) / 40000)
        assert abs(_window_probability(x, a, 0.3) - p2) > 9 * sig
        assert abs(_window_probability(x, a, 0.1) - p2) > 9 * sig
