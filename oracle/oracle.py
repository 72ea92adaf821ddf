"""ctypes front of the FP64 CPU oracle (oracle/liboracle.so).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark.  The GPU library never imports it, and it
never imports the GPU library.  It accepts the problem descriptions built by
``paper_2001_11252_amd.workloads`` (plain data: meshes, gas fields, sources,
lines, observers).
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

DOM_BOX, DOM_SLAB_Z, DOM_SPHERE = 0, 1, 2
ST_NONE, ST_ESCAPED, ST_ABSORBED, ST_STUCK = 0, 1, 2, 3


class OrcLine(C.Structure):
    _fields_ = [("lambda0_A", C.c_double), ("A_ul", C.c_double), ("f_lu", C.c_double),
                ("mass_amu", C.c_double), ("abundance", C.c_double),
                ("phase", C.c_int), ("recoil", C.c_int),
                ("n_fluor", C.c_int), ("fluor_lambda_A", C.c_double * 2), ("fluor_A_ul", C.c_double * 2)]


class OrcProblem(C.Structure):
    _fields_ = [("n_leaves", C.c_int64), ("level", C.c_void_p), ("ijk", C.c_void_p),
                ("box_cm", C.c_double), ("n_hi", C.c_void_p), ("T", C.c_void_p),
                ("v", C.c_void_p), ("kappa_d", C.c_void_p), ("domain_kind", C.c_int),
                ("domain", C.c_double * 4), ("n_lines", C.c_int), ("lines", OrcLine * 4),
                ("T_ref", C.c_double), ("albedo", C.c_double), ("g_hg", C.c_double),
                ("forward_only", C.c_int), ("max_events", C.c_int64),
                ("core_skip_tau", C.c_double), ("core_skip_frac", C.c_double), ("voigt_exact", C.c_int),
                ("spec_kind", C.c_int), ("spec_p", C.c_double * 3),
                ("spec_n", C.c_int), ("spec_lambda", C.c_void_p), ("spec_flux", C.c_void_p),
                ("peel_tau_cut", C.c_double)]


class OrcObserver(C.Structure):
    _fields_ = [("k", C.c_double * 3), ("nx", C.c_int), ("ny", C.c_int), ("nbins", C.c_int),
                ("fov", C.c_double * 4), ("x_min", C.c_double), ("x_max", C.c_double)]


class OrcStats(C.Structure):
    _fields_ = [(n, C.c_int64) for n in ("emitted", "escaped", "absorbed", "stuck", "scatterings",
                                         "dust_scatterings", "crossings", "peel_rays",
                                         "peel_crossings", "peel_dropped")]

    def as_dict(self):
        return {n: int(getattr(self, n)) for n, _ in self._fields_}


def _threads(n):
    if n and n > 0:
        return n
    return max(1, min(16, os.cpu_count() or 1))


def lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(HERE, "liboracle.so")
        if not os.path.exists(path):
            from oracle import build as _b
            _b.build()
        L = C.CDLL(path)
        P = C.c_void_p
        L.orc_philox4x32_10.argtypes = [P, P, P]
        L.orc_uniform.restype = C.c_double
        L.orc_uniform.argtypes = [C.c_uint64, C.c_uint64, C.c_uint32, C.c_uint32]
        L.orc_line_quantities.argtypes = [P, C.c_double, P]
        L.orc_voigt_h.restype = C.c_double
        L.orc_voigt_h.argtypes = [C.c_double, C.c_double]
        L.orc_voigt_dhdx.restype = C.c_double
        L.orc_voigt_dhdx.argtypes = [C.c_double, C.c_double]
        L.orc_voigt_h_exact.restype = C.c_double
        L.orc_voigt_h_exact.argtypes = [C.c_double, C.c_double]
        L.orc_sample_upar.argtypes = [C.c_int64, C.c_double, C.c_double, C.c_uint64, P]
        L.orc_sample_mu.argtypes = [C.c_int64, C.c_int, C.c_double, C.c_uint64, P]
        L.orc_sample_uperp.argtypes = [C.c_int64, C.c_double, C.c_uint64, P]
        L.orc_single_scatter.argtypes = [C.c_int64, P, C.c_double, C.c_double, C.c_uint64, P]
        L.orc_mesh_validate.restype = C.c_int
        L.orc_mesh_validate.argtypes = [C.c_int64, P, P]
        L.orc_locate.restype = C.c_int64
        L.orc_locate.argtypes = [P, P, P]
        L.orc_trace.restype = C.c_int
        L.orc_trace.argtypes = [P, C.c_int64, P, P, C.c_int32, P, P, P]
        L.orc_tau.restype = C.c_int
        L.orc_tau.argtypes = [P, C.c_int64, P, P, P, P]
        L.orc_run.restype = C.c_int
        L.orc_run.argtypes = [P, C.c_int64, P, P, P, C.c_uint64, C.c_int64, C.c_int64, C.c_int,
                              P, P, P, P, P, P, P, P, C.c_int, P]
        L.orc_raycast_image.restype = C.c_int
        L.orc_raycast_image.argtypes = [P, P, C.c_int64, P, P, P, P, P, P, P, P, C.c_int, P]
        _LIB = L
    return _LIB


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def _line_struct(ln):
    s = OrcLine(ln.lambda0_A, ln.A_ul, ln.f_lu, ln.mass_amu, ln.abundance, ln.phase, ln.recoil)
    fl = getattr(ln, "fluor", ())
    s.n_fluor = len(fl)
    for j, (lam, a) in enumerate(fl):
        s.fluor_lambda_A[j] = lam
        s.fluor_A_ul[j] = a
    return s


class _Prob:
    """Keeps the numpy buffers alive for the lifetime of the C struct."""

    def __init__(self, pb, forward_only=False, max_events=0, core_skip=None, voigt_exact=False, peel_tau_cut=0.0):
        m = pb.mesh
        self.level = np.ascontiguousarray(m.level, dtype=np.int8)
        self.ijk = np.ascontiguousarray(m.ijk, dtype=np.int32)
        g = pb.gas
        self.n_hi = np.ascontiguousarray(g.n_hi, dtype=np.float64)
        self.T = np.ascontiguousarray(g.T, dtype=np.float64)
        self.v = np.ascontiguousarray(g.v, dtype=np.float64)
        self.kd = np.ascontiguousarray(g.kappa_d, dtype=np.float64)
        s = OrcProblem()
        s.n_leaves = len(self.level)
        s.level = _ptr(self.level)
        s.ijk = _ptr(self.ijk)
        s.box_cm = m.box_cm
        s.n_hi, s.T, s.v, s.kappa_d = _ptr(self.n_hi), _ptr(self.T), _ptr(self.v), _ptr(self.kd)
        s.domain_kind = pb.domain.kind
        for i in range(4):
            s.domain[i] = pb.domain.params[i]
        s.n_lines = len(pb.lines)
        for i, ln in enumerate(pb.lines):
            s.lines[i] = _line_struct(ln)
        s.T_ref = pb.T_ref
        s.albedo = pb.dust.albedo
        s.g_hg = pb.dust.g
        s.forward_only = int(forward_only)
        s.max_events = int(max_events)
        s.core_skip_tau, s.core_skip_frac = core_skip if core_skip else (0.0, 0.0)
        s.voigt_exact = int(bool(voigt_exact))
        s.peel_tau_cut = float(peel_tau_cut)
        sp = getattr(pb, "spectrum", None)
        if sp and int(sp[0]) == 3:
            # tabulated continuum: (3, lambda[], F_lambda[])
            s.spec_kind = 3
            self.spec_l = np.ascontiguousarray(sp[1], dtype=np.float64)
            self.spec_f = np.ascontiguousarray(sp[2], dtype=np.float64)
            s.spec_n = len(self.spec_l)
            s.spec_lambda, s.spec_flux = _ptr(self.spec_l), _ptr(self.spec_f)
        elif sp:
            s.spec_kind = int(sp[0])
            for i, v in enumerate(sp[1:4]):
                s.spec_p[i] = float(v)
        self.s = s


def _obs_struct(o):
    s = OrcObserver()
    for i in range(3):
        s.k[i] = o.k[i]
    s.nx, s.ny, s.nbins = o.nx, o.ny, o.nbins
    for i in range(4):
        s.fov[i] = o.fov[i]
    s.x_min, s.x_max = o.x_min, o.x_max
    return s


def philox(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def uniform(seed, pid, event, j):
    return lib().orc_uniform(seed, pid, event, j)


def line_quantities(line, T):
    out = np.zeros(5)
    s = _line_struct(line)
    lib().orc_line_quantities(C.byref(s), T, _ptr(out))
    return dict(nu0=out[0], vth=out[1], dnu=out[2], a=out[3], sigma0=out[4])


def voigt_h(a, x):
    return lib().orc_voigt_h(a, x)


def voigt_dhdx(a, x):
    return lib().orc_voigt_dhdx(a, x)


def voigt_h_exact(a, x):
    """H(a, x) from its defining integral (adaptive quadrature), elementwise."""
    f = np.vectorize(lambda aa, xx: lib().orc_voigt_h_exact(float(aa), float(xx)))
    return f(a, x)


def sample_upar(n, x, a, seed=1):
    out = np.zeros(n)
    lib().orc_sample_upar(n, x, a, seed, _ptr(out))
    return out


def sample_mu(n, kind, g=0.0, seed=1):
    kinds = {"core": 0, "wing": 1, "hg": 2, "iso": 3}
    out = np.zeros(n)
    lib().orc_sample_mu(n, kinds[kind], g, seed, _ptr(out))
    return out


def sample_uperp(n, x_crit, seed=1):
    """n core-skipping perpendicular velocity pairs, shape (n, 2)."""
    out = np.zeros((n, 2))
    lib().orc_sample_uperp(n, x_crit, seed, _ptr(out))
    return out


def single_scatter(n, line, T, x_in, seed=1):
    out = np.zeros(n)
    s = _line_struct(line)
    lib().orc_single_scatter(n, C.byref(s), T, x_in, seed, _ptr(out))
    return out


def mesh_validate(level, ijk):
    lv = np.ascontiguousarray(level, dtype=np.int8)
    ij = np.ascontiguousarray(ijk, dtype=np.int32)
    return lib().orc_mesh_validate(len(lv), _ptr(lv), _ptr(ij))


def locate(pb, p, k):
    P = _Prob(pb)
    pa = np.ascontiguousarray(p, dtype=np.float64)
    ka = np.ascontiguousarray(k, dtype=np.float64)
    return int(lib().orc_locate(C.byref(P.s), _ptr(pa), _ptr(ka)))


def trace(pb, orig, dirs, max_cells):
    P = _Prob(pb)
    o = np.ascontiguousarray(orig, dtype=np.float64).reshape(-1, 3)
    d = np.ascontiguousarray(dirs, dtype=np.float64).reshape(-1, 3)
    n = len(o)
    leaf = np.full((n, max_cells), -1, dtype=np.int32)
    seg = np.zeros((n, max_cells))
    cnt = np.zeros(n, dtype=np.int32)
    rc = lib().orc_trace(C.byref(P.s), n, _ptr(o), _ptr(d), max_cells, _ptr(leaf), _ptr(seg), _ptr(cnt))
    if rc:
        raise RuntimeError(f"orc_trace failed: {rc}")
    return leaf, seg, cnt


def tau(pb, orig, dirs, x_ext, voigt_exact=False):
    P = _Prob(pb, voigt_exact=voigt_exact)
    o = np.ascontiguousarray(orig, dtype=np.float64).reshape(-1, 3)
    d = np.ascontiguousarray(dirs, dtype=np.float64).reshape(-1, 3)
    x = np.ascontiguousarray(x_ext, dtype=np.float64)
    out = np.zeros(len(o))
    rc = lib().orc_tau(C.byref(P.s), len(o), _ptr(o), _ptr(d), _ptr(x), _ptr(out))
    if rc:
        raise RuntimeError(f"orc_tau failed: {rc}")
    return out


def run(pb, seed, first=0, n=None, threads=0, forward_only=False, max_events=0, with_cubes=True,
        core_skip=None, voigt_exact=False, peel_tau_cut=0.0):
    """Forward transport of packets [first, first+n) of pb.sources.
    core_skip = (tau_skip, frac) turns core-skipping on (x_crit per cell:
    min(sqrt(ln(tau_cell / tau_skip)), frac (a tau_cell)^(1/3))).
    voigt_exact: H from its defining integral instead of the Tasitsiomi form.
    peel_tau_cut > 0: peel-off rays stop once their optical depth reaches it
    (746: exp(-tau) is exactly 0 beyond, the cubes do not change).

    Returns a dict with per-packet arrays (status, x, k, pos, n_scat, path),
    the observer cubes (list of [ny, nx, nbins] float64) and the stats."""
    P = _Prob(pb, forward_only, max_events, core_skip, voigt_exact, peel_tau_cut)
    src = pb.sources
    pos = np.ascontiguousarray(src.pos, dtype=np.float64)
    dirs = None if src.dir is None else np.ascontiguousarray(src.dir, dtype=np.float64)
    xs = np.ascontiguousarray(src.x, dtype=np.float64)
    n_src = len(xs)
    if n is None:
        n = n_src - first
    obs = pb.observers if with_cubes else []
    n_obs = len(obs)
    obs_arr = (OrcObserver * max(1, n_obs))()
    for i, o in enumerate(obs):
        obs_arr[i] = _obs_struct(o)
    cubes = [np.zeros((o.ny, o.nx, o.nbins)) for o in obs]
    cube_ptrs = (C.c_void_p * max(1, n_obs))(*[c.ctypes.data for c in cubes])
    status = np.zeros(n, dtype=np.int32)
    x_out = np.zeros(n)
    k_out = np.zeros((n, 3))
    pos_out = np.zeros((n, 3))
    n_scat = np.zeros(n, dtype=np.int32)
    path = np.zeros(n)
    st = OrcStats()
    rc = lib().orc_run(C.byref(P.s), n_src, _ptr(pos), _ptr(dirs), _ptr(xs), seed, first, n, n_obs,
                       obs_arr, cube_ptrs, _ptr(status), _ptr(x_out), _ptr(k_out), _ptr(pos_out),
                       _ptr(n_scat), _ptr(path), _threads(threads), C.byref(st))
    if rc:
        raise RuntimeError(f"orc_run failed: {rc}")
    return dict(status=status, x=x_out, k=k_out, pos=pos_out, n_scat=n_scat, path=path,
                cubes=cubes, stats=st.as_dict())


def raycast_image(pb, observer, orig, x_ext, w, grad_image=None, threads=0, crossings=None, voigt_exact=False):
    """Peel-off image of fixed rays toward `observer` and, if grad_image is
    given, the exact gradient of sum(grad_image * image) with respect to the
    per-leaf n_HI, kappa_d and v_los = k_obs . v.  crossings (optional, a
    one-element int64 array) receives the ray-cell segments walked."""
    P = _Prob(pb, voigt_exact=voigt_exact)
    ob = _obs_struct(observer)
    o = np.ascontiguousarray(orig, dtype=np.float64).reshape(-1, 3)
    x = np.ascontiguousarray(x_ext, dtype=np.float64)
    ww = np.ascontiguousarray(w, dtype=np.float64)
    img = np.zeros((observer.ny, observer.nx))
    nl = len(pb.mesh.level)
    G = None if grad_image is None else np.ascontiguousarray(grad_image, dtype=np.float64)
    gn = np.zeros(nl) if G is not None else None
    gk = np.zeros(nl) if G is not None else None
    gv = np.zeros(nl) if G is not None else None
    rc = lib().orc_raycast_image(C.byref(P.s), C.byref(ob), len(o), _ptr(o), _ptr(x), _ptr(ww),
                                 _ptr(img), _ptr(G), _ptr(gn), _ptr(gk), _ptr(gv), _threads(threads),
                                 None if crossings is None else _ptr(crossings))
    if rc:
        raise RuntimeError(f"orc_raycast_image failed: {rc}")
    if G is None:
        return img
    return img, gn, gk, gv
