"""The allocation-free spectrum entry point (rmc_get_spectrum_noalloc)
against rmc_get_spectrum, called through the C ABI: two calls in a row,
the second with fewer bins (the fixed counters keep the first call's
values and must be cleared), and the size limit."""
import ctypes as C

import numpy as np
import pytest

from paper_2001_11252_amd import workloads as W

pytestmark = pytest.mark.gpu


def test_noalloc_spectrum_equals_spectrum(orc):
    import torch
    from paper_2001_11252_amd import rmc
    s0 = lambda ln, T: orc.line_quantities(ln, T)["sigma0"]
    pb = W.static_sphere(s0, 1e3, 1e4, 20000, level=3, tau_dust=0.2)
    ctx = rmc.Context.from_problem(pb, "fp32", observers=False)
    ctx.run(5, 0, 20000)
    lib, h = rmc.lib(), ctx.handle
    dev = torch.device("cuda:0")
    for nbins, lo, hi in ((4000, -40.0, 40.0), (37, -25.0, 20.0)):
        ref = np.zeros(nbins)
        assert lib.rmc_get_spectrum(h, nbins, lo, hi, ref.ctypes.data_as(C.c_void_p), rmc.HOST) == 0
        out = torch.full((nbins,), -1.0, dtype=torch.float64, device=dev)
        rc = lib.rmc_get_spectrum_noalloc(h, nbins, lo, hi, C.c_void_p(out.data_ptr()))
        assert rc == 0, lib.rmc_last_error(h)
        got = out.cpu().numpy()
        assert ref.sum() > 1000
        assert np.array_equal(got, ref)
    big = torch.zeros(65537, dtype=torch.float64, device=dev)
    assert lib.rmc_get_spectrum_noalloc(h, 65537, -1.0, 1.0, C.c_void_p(big.data_ptr())) == rmc.EINVAL
    assert b"65536" in lib.rmc_last_error(h)
