"""The C-ABI library loads and exports every symbol include/rmc.h declares;
host-only entry points work without a GPU (CPU)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2001_11252_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "rmc.h")).read()
    return sorted(set(re.findall(r"\b(rmc_[a-z_0-9]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    from paper_2001_11252_amd import rmc
    names = _declared()
    assert len(names) >= 25
    lib = ctypes.CDLL(rmc.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert rmc.lib().rmc_abi_version() == 9


def test_host_line_quantities_match_oracle(orc):
    from paper_2001_11252_amd import rmc
    for ln in (W.LYA, W.MGII_2796, W.MGII_2804):
        for T in (10.0, 1e4):
            a = rmc.line_quantities(ln, T)
            b = orc.line_quantities(ln, T)
            for k in a:
                assert abs(a[k] / b[k] - 1) < 1e-14


def test_host_mesh_check_agrees_with_oracle_validation(orc):
    from paper_2001_11252_amd import rmc
    rng = np.random.default_rng(2)
    cases = []
    m = W.refined_mesh(1, 4, lambda lev, lo, hi: rng.random(len(lo)) < 0.35)
    cases.append((m.level, m.ijk, 0))
    u = W.uniform_mesh(2)
    cases.append((u.level[1:], u.ijk[1:], -3))                                  # gap
    cases.append((np.concatenate([u.level, [1]]), np.concatenate([u.ijk, [[0, 0, 0]]]), -2))  # overlap
    bad = u.ijk.copy()
    bad[0] = [4, 0, 0]
    cases.append((u.level, bad, -1))
    # a level-1 leaf beside level-3 leaves
    base = W.uniform_mesh(1)
    mask = np.zeros(8, bool)
    mask[0] = True
    lv, ij = W._split(base.level, base.ijk, mask)
    idx = np.nonzero(lv == 2)[0]
    far = idx[np.argmax(ij[idx].sum(axis=1))]
    m2 = np.zeros(len(lv), bool)
    m2[far] = True
    lv, ij = W._split(lv, ij, m2)
    cases.append((lv, ij, -4))
    for level, ijk, want in cases:
        rc, msg = rmc.mesh_check(level, ijk)
        o = orc.mesh_validate(level, ijk)
        assert (rc == 0) == (o == 0) == (want == 0), (rc, o, want, msg)
        if want:
            assert rc == rmc.EMESH and msg


def test_context_creation_fails_loudly_without_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from paper_2001_11252_amd import rmc
    with pytest.raises(rmc.RmcError):
        rmc.Context("fp64")


def test_bench_refuses_more_than_one_gpu():
    # the benchmark runs on one GPU; asking for more exits with a message
    # before touching a device
    import subprocess
    import sys
    import os
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    p = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr
