"""GPU parity of the deterministic probes against the oracle: cell
sequences and segment lengths bit-exact, optical depths within 1e-12
(FP64) and 1e-5 (FP32 bulk) relative."""
import zlib

import numpy as np
import pytest

from paper_2001_11252_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rmc():
    from paper_2001_11252_amd import rmc as R
    return R


def _gas(mesh, rng, vel=True, dust=True, n0=1e-6):
    n = mesh.n
    return W.Gas(n0 * np.exp(rng.standard_normal(n)), 10 ** rng.uniform(2, 4.5, n),
                 (rng.standard_normal((n, 3)) * 30e5) if vel else np.zeros((n, 3)),
                 (1e-23 * np.exp(rng.standard_normal(n))) if dust else np.zeros(n))


def _problem(mesh, gas, domain, lines=(W.LYA,), T_ref=1e4):
    return W.Problem("p", mesh, gas, domain, list(lines), T_ref, W.Dust(), W._point_sources(1))


def _ctx(rmc, pb, prec):
    return rmc.Context.from_problem(pb, prec, sources=False, observers=False)


def _rays(rng, n, inside_sphere=False):
    d = rng.standard_normal((n, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    o = rng.random((n, 3))
    if inside_sphere:
        o = 0.5 + 0.3 * (o - 0.5)
    return o, d


def _special():
    s3 = 1 / np.sqrt(3.0)
    o = np.array([[0.5, 0.5, 0.5], [0.5, 0.5, 0.5], [0.25, 0.125, 0.0625], [0.0, 0.5, 0.25],
                  [0.5, 0.25, 0.75], [0.3, 0.5, 0.5], [0.5, 0.5, 0.5], [0.125, 0.125, 0.125],
                  [0.5, 0.5, 0.5], [0.75, 0.75, 0.25]])
    d = np.array([[s3, s3, s3], [-s3, s3, -s3], [1, 0, 0], [1, 0, 0], [0, -1, 0], [0.6, 0.8, 0],
                  [0, 0, -1], [1 / np.sqrt(2), 1 / np.sqrt(2), 0], [-1, 0, 0], [0, -0.6, 0.8]])
    return o, d


MESHES = {
    "uniform3": lambda: W.uniform_mesh(3),
    "graded": lambda: W.refined_mesh(1, 5, (lambda r: lambda lev, lo, hi: r.random(len(lo)) < 0.3)(
        np.random.default_rng(11))),
    "c2": W.c2_mesh,
    # levels 2-10 about a small sphere's surface: leaves coarser than the
    # level-6 cell table and up to four levels below it
    "deep": lambda: W.refined_mesh(2, 10, lambda lev, lo, hi: (lambda nf: (nf[0] <= 0.06) & (nf[1] >= 0.06))(
        W._near_far(np.array([0.43, 0.56, 0.52]), lo, hi))),
}
DOMAINS = {
    "box": W.Domain(W.DOM_BOX, (0, 0, 0, 0)),
    "sphere": W.Domain(W.DOM_SPHERE, (0.5, 0.5, 0.5, 0.5)),
    "slab": W.Domain(W.DOM_SLAB_Z, (0.5, 0.5, 0, 0)),
}


@pytest.mark.parametrize("mname", list(MESHES))
@pytest.mark.parametrize("dname", list(DOMAINS))
def test_trace_cells_bit_exact(rmc, orc, mname, dname):
    mesh = MESHES[mname]()
    rng = np.random.default_rng(5)
    pb = _problem(mesh, _gas(mesh, rng), DOMAINS[dname])
    o, d = _rays(rng, 3000, inside_sphere=(dname == "sphere"))
    so, sd = _special()
    o, d = np.concatenate([o, so]), np.concatenate([d, sd])
    if dname == "slab":
        d[:, 2] = np.where(np.abs(d[:, 2]) < 0.05, 0.05, d[:, 2])
        d /= np.linalg.norm(d, axis=1)[:, None]
    mc = 4096
    lo, so_, co = orc.trace(pb, o, d, mc)
    ctx = _ctx(rmc, pb, "fp64")
    lg, sg, cg = ctx.trace_cells(o, d, mc)
    assert np.array_equal(co, cg)
    for r in range(len(o)):
        n = co[r]
        assert np.array_equal(lo[r, :n], lg[r, :n]), r
        assert np.array_equal(so_[r, :n], sg[r, :n]), r


# FP32 leaf records hold v / v_th,ref to float precision eps32 ~ 6e-8; the
# relative optical-depth error this causes near the line core is about
# 2|x| eps32 |w| / rho (w = k.v / v_th,ref, rho = sqrt(T/T_ref)).  For
# Lya at the configurations' temperatures and speeds that is below 1e-5.
# The "strong shift" case (MgII, T down to 100 K, 30 km/s: shifts of ~100
# cell thermal widths) has 2*3*6e-8*21*5.5 ~ 4e-5, so its FP32 bound is 1e-4.
FP32_TOL = {"mgii_doublet_slab": 1e-4}


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
@pytest.mark.parametrize("case", ["lya_graded_box", "lya_c2_sphere", "mgii_doublet_slab", "mgii_doublet_slow",
                                  "static_uniform"])
def test_tau_matches_oracle(rmc, orc, prec, tol, case):
    if prec == "fp32":
        tol = FP32_TOL.get(case, tol)
    rng = np.random.default_rng(zlib.crc32(case.encode()))
    if case == "lya_graded_box":
        mesh = MESHES["graded"]()
        pb = _problem(mesh, _gas(mesh, rng), DOMAINS["box"])
    elif case == "lya_c2_sphere":
        mesh = W.c2_mesh()
        pb = _problem(mesh, _gas(mesh, rng, n0=1e-8), DOMAINS["sphere"])
    elif case == "mgii_doublet_slab":
        mesh = W.uniform_mesh(4)
        from dataclasses import replace
        lines = [replace(W.MGII_2796, abundance=3e-5), replace(W.MGII_2804, abundance=3e-5)]
        pb = _problem(mesh, _gas(mesh, rng, n0=1e-2), DOMAINS["slab"], lines, T_ref=3e3)
    elif case == "mgii_doublet_slow":
        mesh = W.uniform_mesh(4)
        from dataclasses import replace
        lines = [replace(W.MGII_2796, abundance=3e-5), replace(W.MGII_2804, abundance=3e-5)]
        g = _gas(mesh, rng, n0=1e-2)
        g.T[:] = 10 ** rng.uniform(3, 4.5, mesh.n)
        g.v[:] *= 5.0 / 30.0
        pb = _problem(mesh, g, DOMAINS["slab"], lines, T_ref=3e3)
    else:
        mesh = W.uniform_mesh(3)
        g = W.Gas(np.full(mesh.n, 1e-6), np.full(mesh.n, 1e4), np.zeros((mesh.n, 3)), np.zeros(mesh.n))
        pb = _problem(mesh, g, DOMAINS["box"])
    o, d = _rays(rng, 4000, inside_sphere=(pb.domain.kind == W.DOM_SPHERE))
    if pb.domain.kind == W.DOM_SLAB_Z:
        d[:, 2] = np.where(np.abs(d[:, 2]) < 0.05, 0.05, d[:, 2])
        d /= np.linalg.norm(d, axis=1)[:, None]
    x = rng.uniform(-40, 40, len(o))
    x[:200] = rng.uniform(-2, 2, 200)
    if prec == "fp32":
        # FP32 bulk: directions as the float path sees them
        d = d.astype(np.float32).astype(np.float64)
    t_o = orc.tau(pb, o, d, x)
    ctx = _ctx(rmc, pb, prec)
    t_g = ctx.tau(o, d, x)
    rel = np.abs(t_g - t_o) / np.maximum(np.abs(t_o), 1e-300)
    assert np.all((rel <= tol) | (np.abs(t_g - t_o) < 1e-300)), (rel.max(), np.argmax(rel))
