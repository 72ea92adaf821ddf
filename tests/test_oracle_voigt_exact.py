"""The oracle's H from its defining integral (Sect. 3.1.1; the accurate
evaluator the paper compares its approximations with in Sect. 3.3.2),
used by the transport when voigt_exact is set.

Pins: the Faddeeva function (a library routine, another method: H = Re w),
the closed form H(a, 0) = e^{a^2} erfc(a), the normalisation over x, the
expansion to first order in a (Dawson's integral), the large-|x| series,
and, through the transport, the optical depth of a uniform static sphere from its centre, tau0 H(a, x)
(tau0 is defined with sigma0 at H = 1)."""
import numpy as np
import pytest
from scipy import integrate, special

from paper_2001_11252_amd import workloads as W


@pytest.mark.parametrize("a", [1e-8, 1e-6, 4.7e-4, 2.2e-2, 0.1, 1.0])
def test_exact_h_matches_the_faddeeva_function(orc, a):
    xs = np.concatenate([np.linspace(-12, 12, 241), [-30.0, 20.0, 55.0, 1e3]])
    v = orc.voigt_h_exact(a, xs)
    ref = special.wofz(xs + 1j * a).real
    assert np.max(np.abs(v / ref - 1)) < 1e-13


def test_exact_h_special_values(orc):
    for a in (1e-6, 1e-3, 0.05, 0.5, 2.0):
        assert abs(orc.voigt_h_exact(a, 0.0) / special.erfcx(a) - 1) < 1e-13, a
    # small a: H = e^{-x^2} - (2a/sqrt(pi)) (1 - 2x F(x)) + O(a^2), F Dawson's integral
    xs = np.linspace(-4, 4, 41)
    for a in (1e-12, 1e-8):
        first = np.exp(-xs ** 2) - 2 * a / np.sqrt(np.pi) * (1 - 2 * xs * special.dawsn(xs))
        assert np.max(np.abs(orc.voigt_h_exact(a, xs) / first - 1)) < 1e-12, a
    # |z| >> 1 (z = x + ia): w(z) = (i / sqrt(pi)) (1/z + 1/(2 z^3) + 3/(4 z^5) + ...),
    # so H = -Im(1/z + 1/(2 z^3) + 3/(4 z^5)) / sqrt(pi) ~ a / (sqrt(pi) x^2)
    for a, x in ((4.7e-4, 200.0), (0.02, 500.0)):
        z = complex(x, a)
        series = -(1 / z + 0.5 / z ** 3 + 0.75 / z ** 5).imag / np.sqrt(np.pi)
        assert abs(orc.voigt_h_exact(a, x) / series - 1) < 1e-11
    # symmetric in x
    xs = np.linspace(0.1, 9, 30)
    assert np.max(np.abs(orc.voigt_h_exact(0.01, xs) / orc.voigt_h_exact(0.01, -xs) - 1)) < 1e-13


def test_exact_h_is_normalised(orc):
    # int H dx = sqrt(pi) (the profile phi = H / sqrt(pi) integrates to one)
    for a in (0.01, 0.3):
        f = lambda x: orc.voigt_h_exact(a, x)
        core, _ = integrate.quad(f, -30, 30, points=[0.0], limit=400, epsabs=0, epsrel=1e-12)
        # beyond |x| = X = 30, the series of w integrated term by term:
        # int_X^inf -Im(1/z + 1/(2z^3) + 3/(4z^5)) dx = atan(a/X) - Im(1/(4 z_X^2) + 3/(16 z_X^4))
        zX = complex(30.0, a)
        wings = 2 / np.sqrt(np.pi) * (np.arctan(a / 30.0) - (0.25 / zX ** 2 + 0.1875 / zX ** 4).imag)
        assert abs((core + wings) / np.sqrt(np.pi) - 1) < 1e-8, a


def test_transport_optical_depth_uses_the_exact_h(orc, sigma0_oracle):
    # uniform static sphere, rays from the centre: tau = tau0 H(a, x) exactly
    for line, T in ((W.LYA, 1e4), (W.MGII_2796, 100.0)):
        tau0 = 1e4
        pb = W.static_sphere(sigma0_oracle, tau0, T, 1, level=3, line=line)
        a = orc.line_quantities(line, T)["a"]
        xs = np.array([0.0, 0.7, 1.9, 3.3, 6.0, 25.0])
        n = len(xs)
        orig = np.tile([0.5, 0.5, 0.5], (n, 1))
        dirs = np.tile([0.6, 0.0, 0.8], (n, 1))
        # x_ext is in Doppler units at T_ref = T: the gas-frame x of a static cell
        tau = orc.tau(pb, orig, dirs, xs, voigt_exact=True)
        want = tau0 * orc.voigt_h_exact(a, xs)
        assert np.max(np.abs(tau / want - 1)) < 1e-12, (line.name, tau / want - 1)
        # the production form differs by up to a few percent at these a
        approx = orc.tau(pb, orig, dirs, xs)
        assert np.max(np.abs(approx / want - 1)) > 1e-4
