"""Seeded synthetic inputs for resonant-line Monte Carlo transfer.

This module only builds plain input data -- octree leaves, per-leaf gas
fields, sources, observers, the atomic constants of the paper's Table 1 --
shaped like the idealised set-ups of the paper (static slab and sphere,
Sect. 3.4; outflowing sphere, Sect. 3.4; a galaxy-like adaptive mesh,
Sect. 5.1).  It holds none of the transfer method's arithmetic: where a
density has to be set from a line-centre optical depth, the caller passes
the line-centre cross-section as a function ``sigma0_fn(line, T)``.

It imports neither the GPU library nor the oracle, so both may be fed from
it.
"""
from dataclasses import dataclass, field, replace
from typing import Callable, List, Optional

import numpy as np

# ---------------------------------------------------------------- constants
KPC_CM = 3.0857e21          # box side used by every configuration
KMS = 1.0e5                 # km/s in cm/s

DOM_BOX, DOM_SLAB_Z, DOM_SPHERE = 0, 1, 2
PHASE_LYA, PHASE_ISO = 0, 1
M_H_AMU = 1.00794
M_MG_AMU = 24.305


@dataclass(frozen=True)
class Line:
    """One transition (Table 1 of the paper)."""
    name: str
    lambda0_A: float
    A_ul: float
    f_lu: float
    mass_amu: float
    abundance: float = 1.0
    phase: int = PHASE_LYA
    recoil: int = 1
    fluor: tuple = ()        # fluorescent channels ((lambda_A, A_ul), ...)


LYA = Line("Lya", 1215.67, 6.265e8, 0.416, M_H_AMU, 1.0, PHASE_LYA, 1)
D_LYA = Line("DLya", 1215.34, 6.265e8, 0.416, 2.01410, 3e-5, PHASE_LYA, 1)
MGII_2796 = Line("MgII2796", 2796.35, 2.60e8, 0.608, M_MG_AMU, 1.0, PHASE_ISO, 1)
MGII_2804 = Line("MgII2804", 2803.53, 2.57e8, 0.303, M_MG_AMU, 1.0, PHASE_ISO, 1)
# Fe II UV1 (Table 1): the two resonant lines and their fluorescent channels
M_FE_AMU = 55.845
FEII_2587 = Line("FeII2587", 2586.65, 8.94e7, 0.0717, M_FE_AMU, 1.0, PHASE_ISO, 1,
                 ((2612.65, 1.20e8), (2632.11, 6.29e7)))
FEII_2600 = Line("FeII2600", 2600.17, 2.35e8, 0.239, M_FE_AMU, 1.0, PHASE_ISO, 1, ((2626.45, 3.52e7),))
# Si II (Table 1): three resonant lines, each with one fluorescent channel
M_SI_AMU = 28.0855
SIII_1190 = Line("SiII1190", 1190.42, 6.53e8, 0.277, M_SI_AMU, 1.0, PHASE_ISO, 1, ((1194.50, 3.45e9),))
SIII_1193 = Line("SiII1193", 1193.28, 2.69e9, 0.575, M_SI_AMU, 1.0, PHASE_ISO, 1, ((1197.39, 1.40e9),))
SIII_1260 = Line("SiII1260", 1260.42, 2.57e9, 1.22, M_SI_AMU, 1.0, PHASE_ISO, 1, ((1265.02, 4.73e8),))


@dataclass
class Mesh:
    level: np.ndarray        # int8  [n]
    ijk: np.ndarray          # int32 [n,3] coordinates at the leaf's own level
    box_cm: float = KPC_CM

    @property
    def n(self):
        return len(self.level)

    def centres(self):
        h = np.ldexp(1.0, -self.level.astype(np.int64))
        return (self.ijk + 0.5) * h[:, None], h


@dataclass
class Gas:
    n_hi: np.ndarray         # cm^-3 [n]
    T: np.ndarray            # K [n]
    v: np.ndarray            # cm/s [n,3]
    kappa_d: np.ndarray      # cm^-1 [n]


@dataclass
class Domain:
    kind: int
    params: tuple            # sphere (cx,cy,cz,R); slab (zc, half_z, 0, 0); box (0,0,0,0)


@dataclass
class Dust:
    albedo: float = 0.32     # Sect. 3.2.2 default at Lya
    g: float = 0.73


@dataclass
class Sources:
    pos: np.ndarray          # [N,3] box units
    x: np.ndarray            # [N] external-frame x
    dir: Optional[np.ndarray] = None   # [N,3] or None for isotropic


@dataclass
class Observer:
    k: tuple
    nx: int
    ny: int
    nbins: int
    fov: tuple               # (u0,u1,v0,v1) relative to the box centre
    x_min: float = -60.0
    x_max: float = 60.0


@dataclass
class Problem:
    name: str
    mesh: Mesh
    gas: Gas
    domain: Domain
    lines: List[Line]
    T_ref: float
    dust: Dust
    sources: Sources
    observers: List[Observer] = field(default_factory=list)
    seed: int = 0
    # source spectrum: None (monochromatic at each source's x) or
    # (1, sigma_x) Gaussian, (2, lambda_min, lambda_max, beta) power law,
    # (3, lambda[], F_lambda[]) tabulated continuum
    spectrum: tuple = None
    meta: dict = field(default_factory=dict)


# ------------------------------------------------------------------ meshes
def uniform_mesh(level, box_cm=KPC_CM):
    s = 1 << level
    g = np.indices((s, s, s)).reshape(3, -1).T.astype(np.int32)
    return Mesh(np.full(len(g), level, dtype=np.int8), np.ascontiguousarray(g), box_cm)


def _split(level, ijk, mask):
    """Replace the masked leaves by their 8 children."""
    keep_l, keep_i = level[~mask], ijk[~mask]
    pl, pi = level[mask], ijk[mask]
    off = np.indices((2, 2, 2)).reshape(3, -1).T.astype(np.int32)
    ci = (2 * pi[:, None, :] + off[None, :, :]).reshape(-1, 3)
    cl = np.repeat(pl + 1, 8).astype(np.int8)
    return np.concatenate([keep_l, cl]), np.concatenate([keep_i, ci]).astype(np.int32)


def _keys(level, ijk):
    lv = level.astype(np.int64)
    return (lv << 57) | (ijk[:, 0].astype(np.int64) << 38) | (ijk[:, 1].astype(np.int64) << 19) | ijk[:, 2].astype(np.int64)


def balance_2to1(level, ijk, max_iter=64):
    """Refine leaves until no two face-adjacent leaves differ by more than
    one level (the grading rule of Sect. 4.3)."""
    for _ in range(max_iter):
        keys = _keys(level, ijk)
        order = np.argsort(keys)
        sk = keys[order]
        refine = np.zeros(len(level), dtype=bool)
        lv = level.astype(np.int64)
        side = np.left_shift(1, lv)
        for d in range(3):
            for sgn in (-1, 1):
                nb = ijk.astype(np.int64).copy()
                nb[:, d] += sgn
                ok = (nb[:, d] >= 0) & (nb[:, d] < side)
                idx = np.nonzero(ok)[0]
                # find the containing leaf among ancestors two or more levels up
                for up in range(2, int(lv.max()) + 1):
                    sel = idx[lv[idx] >= up]
                    if len(sel) == 0:
                        break
                    al = lv[sel] - up
                    ai = nb[sel] >> up
                    k = (al << 57) | (ai[:, 0] << 38) | (ai[:, 1] << 19) | ai[:, 2]
                    pos = np.searchsorted(sk, k)
                    pos = np.minimum(pos, len(sk) - 1)
                    hit = sk[pos] == k
                    refine[order[pos[hit]]] = True
        if not refine.any():
            return level, ijk
        level, ijk = _split(level, ijk, refine)
    raise RuntimeError("2:1 balancing did not converge")


def refined_mesh(base_level, max_level, rule, box_cm=KPC_CM, balance=True, max_leaves=None):
    """Start from a uniform grid at base_level and split every leaf for
    which rule(level, lo, hi) is true (lo, hi: [n,3] cell bounds in box
    units), level by level up to max_level; then enforce 2:1 grading.
    With max_leaves, returns None as soon as the unbalanced mesh exceeds it."""
    m = uniform_mesh(base_level, box_cm)
    level, ijk = m.level, m.ijk
    for lev in range(base_level, max_level):
        cand = level == lev
        h = np.ldexp(1.0, -lev)
        lo = ijk[cand] * h
        mask = np.zeros(len(level), dtype=bool)
        mask[np.nonzero(cand)[0]] = rule(lev, lo, lo + h)
        if not mask.any():
            continue
        if max_leaves is not None and len(level) + 7 * int(mask.sum()) > max_leaves:
            return None
        level, ijk = _split(level, ijk, mask)
    if balance:
        level, ijk = balance_2to1(level, ijk)
    return Mesh(level.astype(np.int8), np.ascontiguousarray(ijk, dtype=np.int32), box_cm)


def _near_far(c, lo, hi):
    near = np.linalg.norm(np.clip(c, lo, hi) - c, axis=1)
    far = np.linalg.norm(np.maximum(np.abs(lo - c), np.abs(hi - c)), axis=1)
    return near, far


# -------------------------------------------------------------- set-ups
def _gas_uniform(n, n_hi, T, kappa_d=0.0):
    return Gas(np.full(n, n_hi, dtype=np.float64), np.full(n, T, dtype=np.float64),
               np.zeros((n, 3)), np.full(n, kappa_d, dtype=np.float64))


def _point_sources(n, p=(0.5, 0.5, 0.5), x=0.0):
    return Sources(np.tile(np.asarray(p, dtype=np.float64), (n, 1)), np.full(n, x, dtype=np.float64))


def static_slab(sigma0_fn, tau0, T, n_packets, level=3, line=LYA, recoil=None, isotropic=False,
                tau_dust=0.0, albedo=0.32, g=0.73, name="slab"):
    """Uniform slab |z - 1/2| < 1/2, periodic in x and y, central
    monochromatic source at x = 0; tau0 is the line-centre optical depth of
    the half-thickness."""
    ln = replace(line, phase=PHASE_ISO if isotropic else line.phase,
                 recoil=line.recoil if recoil is None else int(recoil))
    mesh = uniform_mesh(level)
    half = 0.5 * mesh.box_cm
    n_hi = tau0 / (sigma0_fn(ln, T) * half)
    gas = _gas_uniform(mesh.n, n_hi, T, tau_dust / half)
    return Problem(name, mesh, gas, Domain(DOM_SLAB_Z, (0.5, 0.5, 0.0, 0.0)), [ln], T,
                   Dust(albedo, g), _point_sources(n_packets),
                   meta=dict(tau0=tau0, T=T, n_hi=n_hi))


def static_sphere(sigma0_fn, tau0, T, n_packets, level=0, line=LYA, recoil=None, isotropic=False,
                  tau_dust=0.0, albedo=0.32, g=0.73, name="sphere"):
    """Uniform sphere of radius 1/2 centred in the box, central source."""
    ln = replace(line, phase=PHASE_ISO if isotropic else line.phase,
                 recoil=line.recoil if recoil is None else int(recoil))
    mesh = uniform_mesh(level)
    R = 0.5 * mesh.box_cm
    n_hi = tau0 / (sigma0_fn(ln, T) * R)
    gas = _gas_uniform(mesh.n, n_hi, T, tau_dust / R)
    return Problem(name, mesh, gas, Domain(DOM_SPHERE, (0.5, 0.5, 0.5, 0.5)), [ln], T,
                   Dust(albedo, g), _point_sources(n_packets),
                   meta=dict(tau0=tau0, T=T, n_hi=n_hi))


def c1_slab(sigma0_fn, n_packets=1000):
    """Plain slab: tau0 = 1e4, T = 1e4 K, uniform level-3 grid (512 leaves),
    no dust, no velocity, 1000 packets at x = 0 from the mid-plane."""
    p = static_slab(sigma0_fn, 1e4, 1e4, n_packets, level=3, name="c1_slab")
    p.seed = 0x5EED0001
    return p


def c2_rule(lev, lo, hi):
    r = {3: 0.5, 4: 0.4, 5: 0.33, 6: 0.3}[lev]
    near, _ = _near_far(np.array([0.5, 0.5, 0.5]), lo, hi)
    return near <= r


def c2_mesh():
    """Levels 3-7 refined toward the centre, then 2:1 graded (~3e5 leaves)."""
    return refined_mesh(3, 7, c2_rule)


def c2_dusty_sphere(sigma0_fn, n_packets=1_000_000, tau0=1e6, mesh=None, nx=128, nbins=100):
    """Static uniform sphere R = 1/2 with dust (tau_dust = 1, albedo 0.32,
    g = 0.73), T = 1e4 K, packets from the centre at x = 0, one observer
    along +z with a 128x128x100 cube."""
    mesh = c2_mesh() if mesh is None else mesh
    T = 1e4
    R = 0.5 * mesh.box_cm
    n_hi = tau0 / (sigma0_fn(LYA, T) * R)
    gas = _gas_uniform(mesh.n, n_hi, T, 1.0 / R)
    obs = [Observer((0.0, 0.0, 1.0), nx, nx, nbins, (-0.5, 0.5, -0.5, 0.5), -60.0, 60.0)]
    return Problem("c2_dusty_sphere", mesh, gas, Domain(DOM_SPHERE, (0.5, 0.5, 0.5, 0.5)), [LYA], T,
                   Dust(0.32, 0.73), _point_sources(n_packets), obs, seed=0x5EED0002,
                   meta=dict(tau0=tau0, T=T, n_hi=n_hi))


def deuterium_sphere(sigma0_fn, n_packets, N_HI=2e19, T=1e4, d_to_h=3e-5, level=3):
    """Static uniform sphere R = 1/2 of H I mixed with deuterium (the paper's
    appendix test: T = 1e4 K, column N_HI = 2e19 cm^-2 from the centre,
    D/H = 3e-5), Lya and D Lya with the dipole phase function and recoil,
    central source at x = 0, one +z observer (128x128x100 over x in
    [-20, 20))."""
    from dataclasses import replace
    tau0 = N_HI * sigma0_fn(LYA, T)
    pb = static_sphere(sigma0_fn, tau0, T, n_packets, level=level, name="deuterium_sphere")
    pb.lines = [LYA, replace(D_LYA, abundance=d_to_h)]
    pb.observers = [Observer((0.0, 0.0, 1.0), 128, 128, 100, (-0.5, 0.5, -0.5, 0.5), -20.0, 20.0)]
    pb.seed = 0x5EED0007
    pb.meta.update(N_HI=N_HI, d_to_h=d_to_h)
    return pb


def feii_wind(sigma0_fn, n_packets, N=1e17, vmax_kms=100.0, b_kms=30.0, level=6, r_min_frac=0.05):
    """Fe II UV1 wind (the paper's idealised-set-up example, Sect. 5):
    sphere R = 1/2 with Fe II from r_min = R/20 to R, density ~ r^-3 (column
    N from r_min outwards), radial velocity v_max r/R, Doppler parameter
    b = 30 km/s (as the temperature m b^2 / 2k), the Fe II 2587 and 2600
    lines with their fluorescent channels (2612, 2632; 2626), central
    source with a flat continuum F_lambda over 2570-2640 A; uniform grid of
    level 6, values at cell centres."""
    mesh = uniform_mesh(level)
    R = 0.5
    r_min = r_min_frac * R
    cen, _ = mesh.centres()
    rv = cen - 0.5
    r = np.linalg.norm(rv, axis=1)
    # N = int_rmin^R n0 (r/rmin)^-3 dr = n0 rmin (1 - (rmin/R)^2) / 2 (box units)
    n0 = 2.0 * N / (r_min * mesh.box_cm * (1.0 - r_min_frac ** 2))
    inside = (r >= r_min) & (r < R)
    n = np.where(inside, n0 * (np.maximum(r, r_min) / r_min) ** -3.0, 0.0)
    v = np.zeros((mesh.n, 3))
    v[inside] = (vmax_kms * KMS / R) * rv[inside]
    T = M_FE_AMU * 1.66053907e-24 * (b_kms * KMS) ** 2 / (2.0 * 1.380649e-16)
    gas = Gas(n, np.full(mesh.n, T), v, np.zeros(mesh.n))
    pb = Problem("feii_wind", mesh, gas, Domain(DOM_SPHERE, (0.5, 0.5, 0.5, R)), [FEII_2587, FEII_2600], T,
                 Dust(0.0, 0.0), _point_sources(n_packets), [], seed=0x5EED0008,
                 meta=dict(N=N, vmax_kms=vmax_kms, b_kms=b_kms, T=T))
    pb.spectrum = (2, 2570.0, 2640.0, 0.0)
    return pb


def thick_sphere(sigma0_fn, n_packets=1_000_000, tau0=1e7, level=3, nx=128, nbins=100):
    """Dust-free static sphere R = 1/2 at T = 1e4 K with tau0 = 1e7 from the
    centre on a uniform 8^3 grid (a tau of a cell ~ 1.2e3: the thick-cell
    regime where core-skipping acts), Lya with the dipole phase function and
    recoil, packets from the centre at x = 0, one +z observer with a
    128x128x100 cube over x in [-60, 60)."""
    pb = static_sphere(sigma0_fn, tau0, 1e4, n_packets, level=level, name="thick_sphere")
    pb.observers = [Observer((0.0, 0.0, 1.0), nx, nx, nbins, (-0.5, 0.5, -0.5, 0.5), -60.0, 60.0)]
    pb.seed = 0x5EED0006
    return pb


def c3_rule_factory(R=0.25):
    c = np.array([0.5, 0.5, 0.5])

    def rule(lev, lo, hi):
        near, far = _near_far(c, lo, hi)
        inner = (near <= 0.8 * R) & (far >= 0.8 * R) & (lev < 10)
        outer = (near <= R) & (far >= R) & (lev < 8)
        return inner | outer
    return rule


def c3_mesh(R=0.25, max_level=10, base=5):
    return refined_mesh(base, max_level, c3_rule_factory(R))


def c3_shell(sigma0_fn, vmax_kms=200.0, n_packets=10_000_000, tau0=1e7, mesh=None, R=0.25,
             nx=256, nbins=200):
    """Outflowing shell 0.8R <= r < R (cell centres), v = Vmax r/R radial,
    T = 1e4 K, tau0 across the shell, dust with tau_dust = 1 across the
    shell, three observers with 256x256x200 cubes."""
    mesh = c3_mesh(R) if mesh is None else mesh
    T = 1e4
    thick = 0.2 * R * mesh.box_cm
    n0 = tau0 / (sigma0_fn(LYA, T) * thick)
    cen, _ = mesh.centres()
    rv = cen - 0.5
    r = np.linalg.norm(rv, axis=1)
    inshell = (r >= 0.8 * R) & (r < R)
    n_hi = np.where(inshell, n0, 0.0)
    kd = np.where(inshell, 1.0 / thick, 0.0)
    v = np.zeros((mesh.n, 3))
    inside = r < R
    v[inside] = (vmax_kms * KMS / R) * rv[inside]
    gas = Gas(n_hi, np.full(mesh.n, T), v, kd)
    s3 = 1.0 / np.sqrt(3.0)
    obs = [Observer(k, nx, nx, nbins, (-R, R, -R, R), -60.0, 60.0)
           for k in ((0.0, 0.0, 1.0), (1.0, 0.0, 0.0), (s3, s3, s3))]
    return Problem(f"c3_shell_v{int(vmax_kms)}", mesh, gas, Domain(DOM_SPHERE, (0.5, 0.5, 0.5, R)), [LYA], T,
                   Dust(0.32, 0.73), _point_sources(n_packets), obs, seed=0x5EED0003,
                   meta=dict(tau0=tau0, T=T, n_hi=n0, vmax_kms=vmax_kms))


def c4_batch(sigma0_fn, n_problems=64, seed=0x5EED0004, work_cap=1e10, packet_scale=1.0,
             max_level=7, log_tau_range=(3.0, 7.0)):
    """Many uneven problems: slab or sphere, tau0 log-uniform in [1e3,1e7],
    T log-uniform in [1e2,1e5] K, Lya or the MgII 2796/2804 doublet,
    uniform grids 8^3..128^3 with lognormal n_HI (sigma_ln = 1, mean
    preserving), 1e3..1e6 packets.  A problem whose expected scattering
    count (1.6 tau0 N_p) exceeds work_cap is drawn again."""
    rng = np.random.default_rng(seed)
    probs = []
    for pid in range(n_problems):
        while True:
            geom = rng.integers(2)
            ltau = rng.uniform(*log_tau_range)
            lT = rng.uniform(2, 5)
            mg = rng.integers(2)
            lev = int(rng.integers(3, max_level + 1))
            lnp = rng.uniform(3, 6)
            tau0, T = 10.0 ** ltau, 10.0 ** lT
            npk = int(round(10.0 ** lnp * packet_scale))
            npk = max(npk, 1)
            if 1.6 * tau0 * npk <= work_cap:
                break
        mesh = uniform_mesh(lev)
        half = 0.5 * mesh.box_cm
        if mg:
            ab = 1e-5
            lines = [replace(MGII_2796, abundance=ab), replace(MGII_2804, abundance=ab)]
            nbar = tau0 / (ab * sigma0_fn(lines[0], T) * half)
        else:
            lines = [LYA]
            nbar = tau0 / (sigma0_fn(LYA, T) * half)
        g = rng.standard_normal(mesh.n)
        n_hi = nbar * np.exp(g - 0.5)
        gas = Gas(n_hi, np.full(mesh.n, T), np.zeros((mesh.n, 3)), np.zeros(mesh.n))
        dom = Domain(DOM_SLAB_Z, (0.5, 0.5, 0.0, 0.0)) if geom == 0 else Domain(DOM_SPHERE, (0.5, 0.5, 0.5, 0.5))
        probs.append(Problem(f"c4_{pid:02d}", mesh, gas, dom, lines, T, Dust(0.32, 0.73),
                             _point_sources(npk), [], seed=seed + pid + 1,
                             meta=dict(tau0=tau0, T=T, geom="slab" if geom == 0 else "sphere",
                                       line="MgII" if mg else "Lya", level=lev, n_packets=npk)))
    return probs


# --------------------------------------------------- galaxy-like field (C5)
def gaussian_field(n, slope=-3.0, seed=0):
    """Periodic Gaussian random field on n^3 with power spectrum k^slope,
    normalised to unit variance."""
    rng = np.random.default_rng(seed)
    kf = np.fft.fftfreq(n) * n
    kr = np.fft.rfftfreq(n) * n
    k2 = kf[:, None, None] ** 2 + kf[None, :, None] ** 2 + kr[None, None, :] ** 2
    amp = np.zeros_like(k2)
    nz = k2 > 0
    amp[nz] = k2[nz] ** (slope / 4.0)
    noise = rng.standard_normal((n, n, n))
    f = np.fft.irfftn(np.fft.rfftn(noise) * amp, s=(n, n, n), axes=(0, 1, 2))
    f -= f.mean()
    f /= f.std()
    return f.astype(np.float32)


def _trilinear_periodic(field, pos):
    n = field.shape[0]
    g = pos * n - 0.5
    i0 = np.floor(g).astype(np.int64)
    f = (g - i0).astype(np.float32)
    out = np.zeros(len(pos), dtype=np.float32)
    for dx in (0, 1):
        wx = f[:, 0] if dx else 1 - f[:, 0]
        ix = (i0[:, 0] + dx) % n
        for dy in (0, 1):
            wy = f[:, 1] if dy else 1 - f[:, 1]
            iy = (i0[:, 1] + dy) % n
            for dz in (0, 1):
                wz = f[:, 2] if dz else 1 - f[:, 2]
                iz = (i0[:, 2] + dz) % n
                out += wx * wy * wz * field[ix, iy, iz]
    return out


def c5_galaxy(sigma0_fn, grid=256, min_level=6, max_level=12, target_leaves=2.0e7, n_sources=100_000,
              rays_per_source=100, seed=0x5EED0005, tau_mean=1e4, tau_dust=1.0, vrms_kms=30.0,
              nx=512, log=None):
    """Galaxy-like adaptive mesh: lognormal n_HI (sigma_ln = 2) from a k^-3
    Gaussian field, dust proportional to n_HI, three k^-3 velocity fields
    with 30 km/s rms per component, T = 1e4 K; levels min..max refined where
    the cell's n_HI h^3 exceeds a threshold chosen for ~target_leaves;
    sources at leaves drawn proportionally to n_HI h^3, rays toward +z.
    log (optional) receives a line per stage (a full-size build takes
    minutes)."""
    log = log or (lambda msg: None)
    g = gaussian_field(grid, -3.0, seed)
    vf = [gaussian_field(grid, -3.0, seed + 1 + i) for i in range(3)]
    dens = np.exp(2.0 * g - 2.0)                     # mean 1 (sigma_ln = 2)
    T = 1e4
    box = KPC_CM
    nbar = tau_mean / (sigma0_fn(LYA, T) * box)

    def mass_of(lev, lo, hi):
        c = 0.5 * (lo + hi)
        h = np.ldexp(1.0, -lev)
        return _trilinear_periodic(dens, c) * h ** 3

    # choose the threshold so that the leaf count lands near the target:
    # trial builds skip the balancing (which adds ~15% leaves) and stop once
    # they exceed twice the goal; the threshold is found by bracketing and
    # regula falsi on log N against log threshold
    def rule_for(thr):
        return lambda lev, lo, hi: mass_of(lev, lo, hi) > thr

    goal = target_leaves / 1.15

    def count(thr):
        m = refined_mesh(min_level, max_level, rule_for(thr), balance=False, max_leaves=2 * goal)
        n = np.inf if m is None else m.n
        log(f"c5 trial threshold {thr:.3e}: {n} leaves before balancing")
        return n

    t_a, n_a = 1e-6, count(1e-6)
    step = 10.0 if n_a > goal else 0.1
    t_b, n_b = t_a * step, count(t_a * step)
    for _ in range(12):
        if (n_a > goal) != (n_b > goal) or (n_b == n_a and np.isfinite(n_b)):
            break                       # bracketed, or the count no longer moves
        t_a, n_a = t_b, n_b
        t_b *= step
        n_b = count(t_b)
    thr = t_b
    for _ in range(10 if (n_a > goal) != (n_b > goal) else 0):
        la, lb = np.log(t_a), np.log(t_b)
        fa = np.log(min(n_a, 4 * goal) / goal)
        fb = np.log(min(n_b, 4 * goal) / goal)
        lt = lb - fb * (lb - la) / (fb - fa) if fb != fa else 0.5 * (la + lb)
        lt = min(max(lt, min(la, lb) + 0.05 * abs(lb - la)), max(la, lb) - 0.05 * abs(lb - la))
        thr = float(np.exp(lt))
        n_t = count(thr)
        if abs(n_t / goal - 1.0) < 0.1:
            break
        if (n_t > goal) == (n_a > goal):
            t_a, n_a = thr, n_t
        else:
            t_b, n_b = thr, n_t
    mesh = refined_mesh(min_level, max_level, rule_for(thr), balance=True)
    log(f"c5 mesh: {mesh.n} leaves")
    cen, h = mesh.centres()
    rho = _trilinear_periodic(dens, cen).astype(np.float64)
    n_hi = nbar * rho
    kd = rho * (tau_dust / box)
    v = np.stack([_trilinear_periodic(f, cen) for f in vf], axis=1).astype(np.float64) * (vrms_kms * KMS)
    gas = Gas(n_hi, np.full(mesh.n, T), v, kd)
    log("c5 gas fields done")
    rng = np.random.default_rng(seed + 7)
    wts = rho * h ** 3
    wts /= wts.sum()
    leaf = rng.choice(mesh.n, size=n_sources, p=wts)
    src = (mesh.ijk[leaf] + rng.random((n_sources, 3))) * h[leaf, None]
    nr = n_sources * rays_per_source
    orig = np.repeat(src, rays_per_source, axis=0)
    x_ext = rng.uniform(-20.0, 20.0, nr)
    w = np.full(nr, 1.0 / (4.0 * np.pi))
    G = rng.standard_normal((nx, nx))
    obs = [Observer((0.0, 0.0, 1.0), nx, nx, 1, (-0.5, 0.5, -0.5, 0.5), -1e30, 1e30)]
    p = Problem("c5_galaxy", mesh, gas, Domain(DOM_BOX, (0.0, 0.0, 0.0, 0.0)), [LYA], T, Dust(0.32, 0.73),
                Sources(src, np.zeros(n_sources)), obs, seed=seed, meta=dict(n_hi_mean=nbar))
    p.meta.update(rays=dict(orig=orig, x_ext=x_ext, w=w), grad_image=G)
    return p
