"""GPU single-scattering frequency redistribution against Hummer's R_II-A
(the paper's own check, Sect. 3.4.1): T = 100 K, isotropic angular
redistribution, no recoil, in both precisions.  Each packet is stopped at
its second interaction, so the frequency it carries is the one after
exactly one scattering in a static medium."""
import numpy as np
import pytest

from paper_2001_11252_amd import workloads as W
from tests.analytic import r2a_expected_counts

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("x_in", [0.0, 1.0, 2.0, 3.0, 4.0, 5.0])
def test_single_scattering_redistribution(orc, prec, x_in):
    from paper_2001_11252_amd import rmc
    s0 = lambda ln, T: orc.line_quantities(ln, T)["sigma0"]
    T, n = 100.0, 400_000
    pb = W.static_sphere(s0, 1e8, T, n, level=2, isotropic=True, recoil=False)
    pb.sources.x[:] = x_in
    ctx = rmc.Context.from_problem(pb, prec)
    ctx.set_option(rmc.OPT_MAX_EVENTS, 2)
    st = ctx.run(31 + int(x_in), 0, n)
    out = ctx.get_packets()
    assert np.all(out["status"] == rmc.ST_STUCK) and np.all(out["n_scat"] == 1)
    a = orc.line_quantities(W.LYA, T)["a"]
    edges = np.linspace(-6.0, 6.0 + x_in, 121)
    counts, _ = np.histogram(out["x"], bins=edges)
    exp = r2a_expected_counts(x_in, a, edges, n)
    sel = exp >= 20
    z = (counts[sel] - exp[sel]) / np.sqrt(exp[sel])
    chi2dof = (z ** 2).sum() / sel.sum()
    assert chi2dof < 1.5, (x_in, chi2dof, np.abs(z).max())
    assert (np.abs(z) > 3.5).sum() <= max(2, int(0.02 * sel.sum())), (x_in, np.abs(z).max())
