"""Python binding of librmc (include/rmc.h): argument marshalling only.

Every step of the transport runs in the HIP kernels of librmc.so.  Buffers
may be numpy arrays (host) or torch tensors on the GPU (device, used in
place on the context's stream).  Importing this module loads librmc.so and
raises if it is missing: there is no fallback.
"""
import ctypes as C
import os

import numpy as np

from . import workloads as W

_HERE = os.path.dirname(os.path.abspath(__file__))
# RMC_LIBRARY selects another build of the library (e.g. one compiled for
# a different register budget); default: the in-tree librmc.so
LIB_PATH = os.environ.get("RMC_LIBRARY") or os.path.join(_HERE, "librmc.so")

OK, EINVAL, ENOMEM, EDEVICE, EMESH, ESTATE, EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
FP64, FP32_BULK = 0, 1
HOST, DEVICE = 0, 1
F32, F64 = 0, 1
OPT_FORWARD_ONLY, OPT_MAX_EVENTS, OPT_BLOCK, OPT_WAVES_PER_CU, OPT_REFILL, OPT_PEEL_DEFER = 1, 2, 3, 4, 5, 6
OPT_SLICE_ITERS = 7
OPT_VOIGT = 8
OPT_REGROUP = 9
OPT_COMPACT = 10
ST_NONE, ST_ESCAPED, ST_ABSORBED, ST_STUCK = 0, 1, 2, 3
_NAMES = {EINVAL: "RMC_EINVAL", ENOMEM: "RMC_ENOMEM", EDEVICE: "RMC_EDEVICE", EMESH: "RMC_EMESH",
          ESTATE: "RMC_ESTATE", EUNSUPPORTED: "RMC_EUNSUPPORTED"}


class RmcError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")
        self.code = code


class RmcLine(C.Structure):
    _fields_ = [("lambda0_A", C.c_double), ("A_ul", C.c_double), ("f_lu", C.c_double),
                ("mass_amu", C.c_double), ("abundance", C.c_double), ("phase", C.c_int), ("recoil", C.c_int),
                ("n_fluor", C.c_int), ("fluor_lambda_A", C.c_double * 2), ("fluor_A_ul", C.c_double * 2)]


class RmcRunStats(C.Structure):
    _fields_ = [(n, C.c_uint64) for n in ("emitted", "escaped", "absorbed", "stuck", "scatterings",
                                          "dust_scatterings", "crossings", "peel_rays", "peel_crossings",
                                          "peel_dropped", "peel_deferred")] + [("kernel_ms", C.c_double),
                                                                             ("peel_pass_ms", C.c_double),
                                                                             ("slices_cut", C.c_uint64)]

    def as_dict(self):
        return {n: (float(getattr(self, n)) if t is C.c_double else int(getattr(self, n))) for n, t in self._fields_}


if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() (hipcc, gfx950)")
# PyTorch provides the device memory and streams; it carries its own HIP
# runtime.  Loading it first makes librmc bind to that same runtime (the
# library's libamdhip64.so.7 dependency resolves to the one already loaded),
# so a process holds a single HIP runtime and torch streams and pointers
# are valid in the library.
try:
    import torch as _torch  # noqa: F401
except ImportError:
    _torch = None
_L = C.CDLL(LIB_PATH)
_P = C.c_void_p
_i64 = C.c_int64
_sig = {
    "rmc_abi_version": (C.c_int, []),
    "rmc_create": (C.c_int, [C.POINTER(_P), C.c_int, C.c_int]),
    "rmc_destroy": (None, [_P]),
    "rmc_last_error": (C.c_char_p, [_P]),
    "rmc_set_stream": (C.c_int, [_P, _P]),
    "rmc_set_option": (C.c_int, [_P, C.c_int, _i64]),
    "rmc_set_core_skip": (C.c_int, [_P, C.c_double, C.c_double]),
    "rmc_set_source_spectrum": (C.c_int, [_P, C.c_int, _P]),
    "rmc_set_source_table": (C.c_int, [_P, C.c_int, _P, _P]),
    "rmc_set_mesh": (C.c_int, [_P, _i64, _P, _P, C.c_double]),
    "rmc_set_gas": (C.c_int, [_P, _P, _P, _P, _P, C.c_int, C.c_int]),
    "rmc_set_lines": (C.c_int, [_P, C.c_int, _P, C.c_double]),
    "rmc_set_dust": (C.c_int, [_P, C.c_double, C.c_double]),
    "rmc_set_domain": (C.c_int, [_P, C.c_int, _P]),
    "rmc_set_sources": (C.c_int, [_P, _i64, _P, _P, _P, C.c_int]),
    "rmc_add_observer": (C.c_int, [_P, _P, C.c_int, C.c_int, C.c_int, _P, C.c_double, C.c_double,
                                   C.POINTER(C.c_int)]),
    "rmc_reset_cubes": (C.c_int, [_P]),
    "rmc_run": (C.c_int, [_P, C.c_uint64, _i64, _i64, C.POINTER(RmcRunStats)]),
    "rmc_stream_begin": (C.c_int, [_P, C.c_uint64, _i64, _i64]),
    "rmc_stream_step": (C.c_int, [_P, C.POINTER(RmcRunStats), C.POINTER(_i64)]),
    "rmc_stream_end": (C.c_int, [_P, C.POINTER(RmcRunStats)]),
    "rmc_get_packets": (C.c_int, [_P, _P, _P, _P, _P, _P, _P, C.c_int]),
    "rmc_get_spectrum": (C.c_int, [_P, C.c_int, C.c_double, C.c_double, _P, C.c_int]),
    "rmc_get_spectrum_noalloc": (C.c_int, [_P, C.c_int, C.c_double, C.c_double, _P]),
    "rmc_get_cube": (C.c_int, [_P, C.c_int, _P, C.c_int, C.c_int]),
    "rmc_trace_cells": (C.c_int, [_P, _i64, _P, _P, C.c_int32, _P, _P, _P, C.c_int]),
    "rmc_tau": (C.c_int, [_P, _i64, _P, _P, _P, _P, C.c_int]),
    "rmc_raycast_image": (C.c_int, [_P, C.c_int, _i64, _P, _P, _P, _P, C.c_int]),
    "rmc_raycast_image_backward": (C.c_int, [_P, C.c_int, _i64, _P, _P, _P, _P, _P, _P, _P, _P, C.c_int]),
    "rmc_raycast_image_tape": (C.c_int, [_P, C.c_int, _i64, _P, _P, _P, _P, C.c_int]),
    "rmc_raycast_image_backward_tape": (C.c_int, [_P, _P, _P, _P, _P, _P, C.c_int]),
    "rmc_image_stats": (C.c_int, [_P, C.POINTER(C.c_uint64), C.POINTER(C.c_double)]),
    "rmc_batch_run": (C.c_int, [_P, C.c_int, _P, _P, C.POINTER(RmcRunStats), C.POINTER(RmcRunStats)]),
    "rmc_batch_begin": (C.c_int, [_P, C.c_int, _P, _P]),
    "rmc_batch_autotune": (C.c_int, [_P, C.c_int, _P, _P, C.c_int, _P]),
    "rmc_mesh_check": (C.c_int, [_i64, _P, _P, C.c_char_p, C.c_int]),
    "rmc_line_quantities": (C.c_int, [_P, C.c_double, _P]),
}
for _n, (_r, _a) in _sig.items():
    _f = getattr(_L, _n)
    _f.restype = _r
    _f.argtypes = _a


def lib():
    return _L


def _is_dev(a):
    if a is None or type(a).__module__.split(".")[0] != "torch":
        return False
    return bool(a.is_cuda)


def _ptr(a):
    if a is None:
        return None
    if _is_dev(a):
        return C.c_void_p(a.data_ptr())
    return a.ctypes.data_as(C.c_void_p)


def _host(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def _dev(a, name, device, dtypes, numel):
    """A device tensor handed to the library in place: checked to be on the
    context's device, of an accepted dtype, contiguous and of the expected
    size (the kernels read numel elements from its pointer)."""
    import torch
    if not _is_dev(a):
        raise TypeError(f"{name}: expected a torch tensor on the GPU (the other arguments are)")
    if a.device != device:
        raise ValueError(f"{name}: on {a.device}, expected {device}")
    if a.dtype not in dtypes:
        raise TypeError(f"{name}: dtype {a.dtype}, expected one of {dtypes}")
    if not a.is_contiguous():
        raise ValueError(f"{name}: not contiguous")
    if a.numel() != numel:
        raise ValueError(f"{name}: {a.numel()} elements, expected {numel}")
    return a


def _f64():
    import torch
    return (torch.float64,)


def _line(ln):
    s = RmcLine(ln.lambda0_A, ln.A_ul, ln.f_lu, ln.mass_amu, ln.abundance, ln.phase, ln.recoil)
    fl = getattr(ln, "fluor", ())
    s.n_fluor = len(fl)
    for j, (lam, a) in enumerate(fl):
        s.fluor_lambda_A[j] = lam
        s.fluor_A_ul[j] = a
    return s


def line_quantities(line, T):
    out = np.zeros(5)
    s = _line(line)
    rc = _L.rmc_line_quantities(C.byref(s), T, _ptr(out))
    if rc:
        raise RmcError(rc, "rmc_line_quantities")
    return dict(nu0=out[0], vth=out[1], dnu=out[2], a=out[3], sigma0=out[4])


def sigma0(line, T):
    return line_quantities(line, T)["sigma0"]


def mesh_check(level, ijk):
    lv = _host(level, np.int8)
    ij = _host(ijk, np.int32)
    buf = C.create_string_buffer(256)
    rc = _L.rmc_mesh_check(len(lv), _ptr(lv), _ptr(ij), buf, 256)
    return rc, buf.value.decode()


class Context:
    """One transfer problem on one GPU (an rmc_ctx)."""

    def __init__(self, precision="fp64", device=0):
        self.precision = FP64 if precision in ("fp64", FP64) else FP32_BULK
        h = _P()
        rc = _L.rmc_create(C.byref(h), device, self.precision)
        if rc:
            raise RmcError(rc, "rmc_create")
        self._h = h
        self.n_leaves = 0
        self.observers = []
        self.stream = None

    def close(self):
        if getattr(self, "_h", None) and _L is not None:
            _L.rmc_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def _chk(self, rc, what):
        if rc:
            raise RmcError(rc, f"{what}: {_L.rmc_last_error(self._h).decode()}")

    @property
    def handle(self):
        return self._h

    # ----------------------------------------------------------- inputs
    def set_stream(self, stream):
        """stream: a torch.cuda.Stream (or its raw handle)."""
        raw = getattr(stream, "cuda_stream", stream)
        self.stream = stream
        self._chk(_L.rmc_set_stream(self._h, C.c_void_p(raw or 0)), "set_stream")

    def set_option(self, opt, value):
        self._chk(_L.rmc_set_option(self._h, opt, int(value)), "set_option")

    def set_source_spectrum(self, kind, params=(0.0, 0.0, 0.0)):
        """Source spectrum: 0 monochromatic, 1 Gaussian (sigma_x,), 2 power
        law (lambda_min, lambda_max, beta); see rmc_set_source_spectrum."""
        p = np.zeros(3)
        p[:len(params)] = params
        self._chk(_L.rmc_set_source_spectrum(self._h, int(kind), p.ctypes.data), "set_source_spectrum")

    def set_source_table(self, lambda_A, f_lambda):
        """Tabulated continuum source (see rmc_set_source_table)."""
        lam = np.ascontiguousarray(lambda_A, dtype=np.float64)
        f = np.ascontiguousarray(f_lambda, dtype=np.float64)
        if len(lam) != len(f):
            raise ValueError("lambda_A and f_lambda differ in length")
        self._chk(_L.rmc_set_source_table(self._h, len(lam), lam.ctypes.data, f.ctypes.data), "set_source_table")

    def set_core_skip(self, tau_skip=1.0, frac=0.2):
        """Core-skipping on (tau_skip > 0) or off (tau_skip = 0); see
        rmc_set_core_skip for the per-cell x_crit."""
        self._chk(_L.rmc_set_core_skip(self._h, float(tau_skip), float(frac)), "set_core_skip")

    def set_mesh(self, level, ijk, box_cm):
        lv = _host(level, np.int8)
        ij = _host(ijk, np.int32)
        self._chk(_L.rmc_set_mesh(self._h, len(lv), _ptr(lv), _ptr(ij), float(box_cm)), "set_mesh")
        self.n_leaves = len(lv)

    def set_lines(self, lines, T_ref):
        arr = (RmcLine * len(lines))(*[_line(l) for l in lines])
        self._chk(_L.rmc_set_lines(self._h, len(lines), arr, float(T_ref)), "set_lines")

    def set_gas(self, n_hi, T, v, kappa_d):
        """Per-leaf gas: numpy arrays (host), or torch tensors on the GPU, all
        float32 or all float64 (read in place on the device, no host copy)."""
        n = self.n_leaves
        if _is_dev(n_hi):
            import torch
            dt = n_hi.dtype
            if dt not in (torch.float32, torch.float64):
                raise TypeError(f"n_hi: dtype {dt}, expected float32 or float64")
            a = _dev(n_hi, "n_hi", n_hi.device, (dt,), n)
            b = _dev(T, "T", n_hi.device, (dt,), n)
            c = _dev(v, "v", n_hi.device, (dt,), 3 * n)
            d = _dev(kappa_d, "kappa_d", n_hi.device, (dt,), n)
            self._chk(_L.rmc_set_gas(self._h, _ptr(a), _ptr(b), _ptr(c), _ptr(d),
                                     F32 if dt == torch.float32 else F64, DEVICE), "set_gas")
            return
        a, b, c, d = (_host(n_hi, np.float64), _host(T, np.float64), _host(v, np.float64),
                      _host(kappa_d, np.float64))
        if not (len(a) == len(b) == len(d) == n and c.size == 3 * n):
            raise ValueError(f"gas arrays must hold {n} leaves (v: {3 * n} values)")
        self._chk(_L.rmc_set_gas(self._h, _ptr(a), _ptr(b), _ptr(c), _ptr(d), F64, HOST), "set_gas")

    def set_dust(self, albedo, g):
        self._chk(_L.rmc_set_dust(self._h, float(albedo), float(g)), "set_dust")

    def set_domain(self, kind, params=(0.0, 0.0, 0.0, 0.0)):
        p = _host(params, np.float64)
        self._chk(_L.rmc_set_domain(self._h, int(kind), _ptr(p)), "set_domain")

    def set_sources(self, pos, x, dirs=None):
        if _is_dev(pos):
            n = pos.shape[0]
            _dev(pos, "pos", pos.device, _f64(), 3 * n)
            _dev(x, "x", pos.device, _f64(), n)
            if dirs is not None:
                _dev(dirs, "dirs", pos.device, _f64(), 3 * n)
            self._chk(_L.rmc_set_sources(self._h, n, _ptr(pos), _ptr(dirs), _ptr(x), DEVICE), "set_sources")
            return
        p = _host(pos, np.float64)
        xx = _host(x, np.float64)
        d = None if dirs is None else _host(dirs, np.float64)
        self._chk(_L.rmc_set_sources(self._h, len(xx), _ptr(p), _ptr(d), _ptr(xx), HOST), "set_sources")

    def add_observer(self, k, nx, ny, nbins, fov, x_min, x_max):
        kk = _host(k, np.float64)
        ff = _host(fov, np.float64)
        oid = C.c_int(-1)
        self._chk(_L.rmc_add_observer(self._h, _ptr(kk), nx, ny, nbins, _ptr(ff), float(x_min), float(x_max),
                                      C.byref(oid)), "add_observer")
        self.observers.append((ny, nx, nbins))
        return oid.value

    def reset_cubes(self):
        self._chk(_L.rmc_reset_cubes(self._h), "reset_cubes")

    # -------------------------------------------------------- transport
    def run(self, seed, first=0, n=None, n_src=None):
        if n is None:
            n = n_src - first
        st = RmcRunStats()
        self._chk(_L.rmc_run(self._h, C.c_uint64(int(seed) & 0xFFFFFFFFFFFFFFFF), first, n, C.byref(st)), "run")
        self.last_n = n
        return st.as_dict()

    def stream_begin(self, seed, first, n):
        self._chk(_L.rmc_stream_begin(self._h, C.c_uint64(int(seed) & 0xFFFFFFFFFFFFFFFF), first, n), "stream_begin")
        self.last_n = n

    def stream_step(self):
        st = RmcRunStats()
        rem = _i64(0)
        self._chk(_L.rmc_stream_step(self._h, C.byref(st), C.byref(rem)), "stream_step")
        return st.as_dict(), rem.value

    def stream_end(self):
        st = RmcRunStats()
        self._chk(_L.rmc_stream_end(self._h, C.byref(st)), "stream_end")
        return st.as_dict()

    def get_packets(self, n=None):
        n = self.last_n if n is None else n
        out = dict(status=np.zeros(n, np.int32), x=np.zeros(n), k=np.zeros((n, 3)), pos=np.zeros((n, 3)),
                   n_scat=np.zeros(n, np.int32), path=np.zeros(n))
        self._chk(_L.rmc_get_packets(self._h, _ptr(out["status"]), _ptr(out["x"]), _ptr(out["k"]), _ptr(out["pos"]),
                                     _ptr(out["n_scat"]), _ptr(out["path"]), HOST), "get_packets")
        return out

    def get_spectrum(self, nbins, x_min, x_max):
        h = np.zeros(nbins)
        self._chk(_L.rmc_get_spectrum(self._h, nbins, float(x_min), float(x_max), _ptr(h), HOST), "get_spectrum")
        return h

    def get_cube(self, oid, dtype=np.float64):
        ny, nx, nb = self.observers[oid]
        out = np.zeros((ny, nx, nb), dtype=dtype)
        self._chk(_L.rmc_get_cube(self._h, oid, _ptr(out), F64 if dtype == np.float64 else F32, HOST), "get_cube")
        return out

    # ----------------------------------------------------------- probes
    def trace_cells(self, orig, dirs, max_cells):
        o = _host(orig, np.float64).reshape(-1, 3)
        d = _host(dirs, np.float64).reshape(-1, 3)
        n = len(o)
        leaf = np.full((n, max_cells), -1, np.int32)
        seg = np.zeros((n, max_cells))
        cnt = np.zeros(n, np.int32)
        self._chk(_L.rmc_trace_cells(self._h, n, _ptr(o), _ptr(d), max_cells, _ptr(leaf), _ptr(seg), _ptr(cnt), HOST),
                  "trace_cells")
        return leaf, seg, cnt

    def tau(self, orig, dirs, x_ext):
        o = _host(orig, np.float64).reshape(-1, 3)
        d = _host(dirs, np.float64).reshape(-1, 3)
        x = _host(x_ext, np.float64)
        t = np.zeros(len(o))
        self._chk(_L.rmc_tau(self._h, len(o), _ptr(o), _ptr(d), _ptr(x), _ptr(t), HOST), "tau")
        return t

    # ----------------------------------------------------- image/adjoint
    def _rays_dev(self, orig, x_ext, w):
        n = orig.shape[0]
        _dev(orig, "orig", orig.device, _f64(), 3 * n)
        _dev(x_ext, "x_ext", orig.device, _f64(), n)
        _dev(w, "w", orig.device, _f64(), n)
        return n

    def raycast_image(self, oid, orig, x_ext, w):
        ny, nx, _ = self.observers[oid]
        if _is_dev(orig):
            import torch
            self._rays_dev(orig, x_ext, w)
            img = torch.zeros((ny, nx), dtype=torch.float64, device=orig.device)
            self._chk(_L.rmc_raycast_image(self._h, oid, orig.shape[0], _ptr(orig), _ptr(x_ext), _ptr(w), _ptr(img),
                                           DEVICE), "raycast_image")
            return img
        o, x, ww = _host(orig, np.float64), _host(x_ext, np.float64), _host(w, np.float64)
        img = np.zeros((ny, nx))
        self._chk(_L.rmc_raycast_image(self._h, oid, len(x), _ptr(o), _ptr(x), _ptr(ww), _ptr(img), HOST),
                  "raycast_image")
        return img

    def raycast_image_backward(self, oid, orig, x_ext, w, grad_image, with_v=False):
        """(g_nhi, g_kd, g_vlos) per leaf of sum(grad_image * image); with_v
        adds g_v [n, 3], the gradient with respect to the velocity vector."""
        ny, nx, _ = self.observers[oid]
        n = self.n_leaves
        if _is_dev(orig):
            import torch
            self._rays_dev(orig, x_ext, w)
            gn, gk, gv = (torch.zeros(n, dtype=torch.float64, device=orig.device) for _ in range(3))
            g3 = torch.zeros((n, 3), dtype=torch.float64, device=orig.device) if with_v else None
            G = _dev(grad_image.contiguous().to(torch.float64), "grad_image", orig.device, _f64(), ny * nx)
            self._chk(_L.rmc_raycast_image_backward(self._h, oid, orig.shape[0], _ptr(orig), _ptr(x_ext), _ptr(w),
                                                    _ptr(G), _ptr(gn), _ptr(gk), _ptr(gv), _ptr(g3), DEVICE),
                      "raycast_image_backward")
            return (gn, gk, gv, g3) if with_v else (gn, gk, gv)
        o, x, ww = _host(orig, np.float64), _host(x_ext, np.float64), _host(w, np.float64)
        G = _host(grad_image, np.float64)
        if G.size != ny * nx or o.size != 3 * len(x) or len(ww) != len(x):
            raise ValueError("ray arrays or grad_image of the wrong size")
        gn, gk, gv = np.zeros(n), np.zeros(n), np.zeros(n)
        g3 = np.zeros((n, 3)) if with_v else None
        self._chk(_L.rmc_raycast_image_backward(self._h, oid, len(x), _ptr(o), _ptr(x), _ptr(ww), _ptr(G), _ptr(gn),
                                                _ptr(gk), _ptr(gv), _ptr(g3), HOST), "raycast_image_backward")
        return (gn, gk, gv, g3) if with_v else (gn, gk, gv)

    def raycast_image_tape(self, oid, orig, x_ext, w):
        """raycast_image that keeps the rays' crossing lists on the device
        for raycast_image_backward_tape (tape_serial counts these calls)."""
        ny, nx, _ = self.observers[oid]
        if _is_dev(orig):
            import torch
            self._rays_dev(orig, x_ext, w)
            img = torch.zeros((ny, nx), dtype=torch.float64, device=orig.device)
            self._chk(_L.rmc_raycast_image_tape(self._h, oid, orig.shape[0], _ptr(orig), _ptr(x_ext), _ptr(w),
                                                _ptr(img), DEVICE), "raycast_image_tape")
        else:
            o, x, ww = _host(orig, np.float64), _host(x_ext, np.float64), _host(w, np.float64)
            img = np.zeros((ny, nx))
            self._chk(_L.rmc_raycast_image_tape(self._h, oid, len(x), _ptr(o), _ptr(x), _ptr(ww), _ptr(img), HOST),
                      "raycast_image_tape")
        self.tape_serial = getattr(self, "tape_serial", 0) + 1
        return img

    def raycast_image_backward_tape(self, grad_image, with_v=False):
        """(g_nhi, g_kd, g_vlos) per leaf of sum(grad_image * image) for the
        rays of the last raycast_image_tape call, read from its tape; with_v
        adds g_v [n, 3] (velocity-vector gradient)."""
        n = self.n_leaves
        if _is_dev(grad_image):
            import torch
            gn, gk, gv = (torch.zeros(n, dtype=torch.float64, device=grad_image.device) for _ in range(3))
            g3 = torch.zeros((n, 3), dtype=torch.float64, device=grad_image.device) if with_v else None
            G = grad_image.contiguous().to(torch.float64)
            self._chk(_L.rmc_raycast_image_backward_tape(self._h, _ptr(G), _ptr(gn), _ptr(gk), _ptr(gv), _ptr(g3),
                                                         DEVICE), "raycast_image_backward_tape")
            return (gn, gk, gv, g3) if with_v else (gn, gk, gv)
        G = _host(grad_image, np.float64)
        gn, gk, gv = np.zeros(n), np.zeros(n), np.zeros(n)
        g3 = np.zeros((n, 3)) if with_v else None
        self._chk(_L.rmc_raycast_image_backward_tape(self._h, _ptr(G), _ptr(gn), _ptr(gk), _ptr(gv), _ptr(g3), HOST),
                  "raycast_image_backward_tape")
        return (gn, gk, gv, g3) if with_v else (gn, gk, gv)

    def image_stats(self):
        """(ray-cell crossings, device ms) of the last image call."""
        n = C.c_uint64(0)
        ms = C.c_double(0.0)
        self._chk(_L.rmc_image_stats(self._h, C.byref(n), C.byref(ms)), "image_stats")
        return int(n.value), float(ms.value)

    # ------------------------------------------------------ convenience
    @classmethod
    def from_problem(cls, pb, precision="fp64", device=0, observers=True, sources=True):
        """Configure a context from a workloads.Problem."""
        c = cls(precision, device)
        try:
            c.set_mesh(pb.mesh.level, pb.mesh.ijk, pb.mesh.box_cm)
            c.set_lines(pb.lines, pb.T_ref)
            c.set_gas(pb.gas.n_hi, pb.gas.T, pb.gas.v, pb.gas.kappa_d)
            c.set_dust(pb.dust.albedo, pb.dust.g)
            c.set_domain(pb.domain.kind, pb.domain.params)
            if sources:
                c.set_sources(pb.sources.pos, pb.sources.x, pb.sources.dir)
                c.n_src = len(pb.sources.x)
                sp = getattr(pb, "spectrum", None)
                if sp and int(sp[0]) == 3:
                    c.set_source_table(sp[1], sp[2])
                elif sp:
                    c.set_source_spectrum(sp[0], sp[1:])
            if observers:
                for o in pb.observers:
                    c.add_observer(o.k, o.nx, o.ny, o.nbins, o.fov, o.x_min, o.x_max)
        except BaseException:
            c.close()
            raise
        return c


def batch_run(contexts, seeds, n_packets):
    n = len(contexts)
    hs = (C.c_void_p * n)(*[c.handle.value for c in contexts])
    sd = np.ascontiguousarray([int(s) & 0xFFFFFFFFFFFFFFFF for s in seeds], dtype=np.uint64)
    npk = np.ascontiguousarray(n_packets, dtype=np.int64)
    per = (RmcRunStats * n)()
    tot = RmcRunStats()
    rc = _L.rmc_batch_run(hs, n, _ptr(sd), _ptr(npk), per, C.byref(tot))
    if rc:
        raise RmcError(rc, "batch_run: " + _L.rmc_last_error(contexts[0].handle).decode())
    for c, k in zip(contexts, npk):
        c.last_n = int(k)
    return [p.as_dict() for p in per], tot.as_dict()


def batch_begin(contexts, seeds, n_packets):
    """Open the batch's stream on contexts[0]: advance it with
    contexts[0].stream_step(), finish with contexts[0].stream_end()."""
    n = len(contexts)
    hs = (C.c_void_p * n)(*[c.handle.value for c in contexts])
    sd = np.ascontiguousarray([int(s) & 0xFFFFFFFFFFFFFFFF for s in seeds], dtype=np.uint64)
    npk = np.ascontiguousarray(n_packets, dtype=np.int64)
    rc = _L.rmc_batch_begin(hs, n, _ptr(sd), _ptr(npk))
    if rc:
        raise RmcError(rc, "batch_begin: " + _L.rmc_last_error(contexts[0].handle).decode())
    for c, k in zip(contexts, npk):
        c.last_n = int(k)


def batch_autotune(contexts, seeds, n_packets, trial_slices=3):
    """Measure launch shapes on this batch; returns {block, refill,
    slice_iters} now set on contexts[0] for later batch_run calls."""
    n = len(contexts)
    hs = (C.c_void_p * n)(*[c.handle.value for c in contexts])
    sd = np.ascontiguousarray([int(s) & 0xFFFFFFFFFFFFFFFF for s in seeds], dtype=np.uint64)
    npk = np.ascontiguousarray(n_packets, dtype=np.int64)
    best = np.zeros(3, dtype=np.int32)
    rc = _L.rmc_batch_autotune(hs, n, _ptr(sd), _ptr(npk), int(trial_slices), _ptr(best))
    if rc:
        raise RmcError(rc, "batch_autotune: " + _L.rmc_last_error(contexts[0].handle).decode())
    return dict(block=int(best[0]), refill=int(best[1]), slice_iters=int(best[2]))


def _make_raycast_fn():
    import torch

    class RayCastImage(torch.autograd.Function):
        """Peel-off image of fixed rays as a differentiable function of the
        per-leaf gas: image = f(n_HI, kappa_d, v).  The gas tensors (float32
        or float64, on the context's GPU) go to the library in place
        (rmc_set_gas with RMC_DEVICE).  The forward pass keeps the rays'
        crossing lists (rmc_raycast_image_tape) and the backward pass reads
        them (rmc_raycast_image_backward_tape); if the context has recorded
        another tape since, the backward sets this call's gas again and
        replays the rays (rmc_raycast_image_backward).  The library returns
        the gradient with respect to the velocity vector directly."""

        @staticmethod
        def _set_gas(rmc_ctx, n_hi, kappa_d, v, T):
            n_hi, kappa_d, v = n_hi.detach(), kappa_d.detach(), v.detach()
            if _is_dev(n_hi):
                T = torch.as_tensor(T, dtype=n_hi.dtype, device=n_hi.device)
                if T.numel() == 1:
                    T = T.expand(n_hi.numel())
                rmc_ctx.set_gas(n_hi.contiguous(), T.contiguous(), v.contiguous(), kappa_d.contiguous())
            else:
                rmc_ctx.set_gas(n_hi.numpy(), T, v.numpy(), kappa_d.numpy())

        @staticmethod
        def forward(ctx, n_hi, kappa_d, v, rmc_ctx, T, oid, orig, x_ext, w):
            RayCastImage._set_gas(rmc_ctx, n_hi, kappa_d, v, T)
            img = rmc_ctx.raycast_image_tape(oid, orig, x_ext, w)
            # this call's gas, kept by reference for the replay fallback
            ctx.save_for_backward(n_hi, kappa_d, v)
            ctx.rmc = (rmc_ctx, oid, orig, x_ext, w, T, rmc_ctx.tape_serial)
            return img

        @staticmethod
        def backward(ctx, grad_image):
            rmc_ctx, oid, orig, x_ext, w, T, serial = ctx.rmc
            if rmc_ctx.tape_serial == serial:
                gn, gk, _, g3 = rmc_ctx.raycast_image_backward_tape(grad_image, with_v=True)
            else:
                n_hi, kappa_d, v = ctx.saved_tensors
                RayCastImage._set_gas(rmc_ctx, n_hi, kappa_d, v, T)
                gn, gk, _, g3 = rmc_ctx.raycast_image_backward(oid, orig, x_ext, w, grad_image, with_v=True)
            n_hi, kappa_d, v = ctx.saved_tensors
            return (gn.to(n_hi.dtype), gk.to(kappa_d.dtype), g3.reshape(v.shape).to(v.dtype),
                    None, None, None, None, None, None)

    return RayCastImage


def raycast_image_fn():
    return _make_raycast_fn()
