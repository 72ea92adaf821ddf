"""Throughput benchmark: Monte Carlo Lya transfer through a dusty sphere.

Workload (the configuration the metric is quoted on): static uniform HI
sphere, tau0 = 1e6 at line centre along the radius, T = 1e4 K, dust with
tau_dust = 1 (albedo 0.32, g = 0.73), octree refined from level 3 to 7
toward the centre (287,064 leaves), packets emitted at x = 0 from the
centre, one observer along +z with a 128x128x100 peel-off cube, 1e6
packets queued.  A step is one transport launch and the ray-cast pass that
follows it: every lane of the grid advances the packet it holds by up to
--slice loop iterations (emission, propagation, scattering, dust, peel-off
of every event through the scattering's own leaf, termination) and lanes
whose packet finished take the next one from the queue; packets that are
still alive are parked in device memory for the next step, and peel-off
rays that leave their first leaf are walked to the border by the ray-cast
pass.  Timed steps follow warm-up steps, so they measure the steady state
of the resident packet pool.  The FP32 bulk path is the headline; the FP64
path runs beside it on the same packets.

Prints one JSON line.  Inputs are synthetic and seeded.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic floating-point work per unit, counted from the formulas of
# the transport step (one elementary function, division or square root
# counted as 8 operations):
#   one line scattering, including building its peel-off source: 480
#   one ray-cell segment (opacity of the leaf + exit geometry):    110
FLOP_PER_SCATTERING = 480.0
FLOP_PER_CROSSING = 110.0
# Algorithmic HBM bytes: one leaf record per segment (24 B float, 48 B
# double) plus one 4 B node entry.
BYTES_PER_CROSSING = {"fp32": 28.0, "fp64": 52.0}
MATCH_SLICE = 1024          # loop iterations per launch of the FP32/FP64 comparison sample
PEAK = {"fp32": 157.3, "fp64": 78.6}       # TFLOP/s, MI355X vector


def kernel_source_digest():
    """Digest of the device code (kernels and the header they include),
    comments and layout removed, so that only a change of the code itself
    invalidates a traffic measurement."""
    import hashlib
    import re
    h = hashlib.sha256()
    src = os.path.join(ROOT, "paper_2001_11252_amd", "csrc")
    for f in ("rmc_device.h", "rmc_kernels.hip"):
        text = open(os.path.join(src, f)).read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def measured_traffic(prec, name="transport_traffic.json"):
    """HBM bytes per launch of a kernel from the profiler's FETCH_SIZE and
    WRITE_SIZE counters (profiles/<name>, entry prec), or None if the kernel
    sources changed since they were taken."""
    import json as _j
    f = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(f):
        return None
    d = _j.load(open(f))
    e = d.get(prec)
    if not e or d.get("source_digest") != kernel_source_digest():
        return None
    return e["bytes_per_launch"]


def host_cores():
    """Host cores this process may run on: the CPU affinity mask, reduced
    to the cgroup CPU quota when one is set (a container's share of the
    host), with what nproc, os.cpu_count() and lscpu report."""
    aff = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    quota = None
    try:
        q, per = open("/sys/fs/cgroup/cpu.max").read().split()[:2]
        if q != "max":
            quota = float(q) / float(per)
    except (OSError, ValueError):
        pass
    n = max(1, min(aff, int(quota)) if quota else aff)
    model = None
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                model = ln.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    import subprocess
    try:
        nproc = int(subprocess.run(["nproc"], capture_output=True, text=True).stdout.strip())
    except (OSError, ValueError):
        nproc = None
    return n, {"threads": n, "nproc": nproc, "os_cpu_count": os.cpu_count(), "affinity": aff,
               "cgroup_cpu_quota": quota, "model": model}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--slice", type=int, default=8192, help="loop iterations per lane per step")
    ap.add_argument("--packets", type=int, default=1_000_000, help="packets queued")
    ap.add_argument("--fp64-steps", type=int, default=5)
    ap.add_argument("--match-launches", type=int, default=32,
                    help="launches of the untimed FP32/FP64 comparison sample (0: skip)")
    ap.add_argument("--tau0", type=float, default=1e6)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-packets", type=int, default=0,
                    help="oracle packets, full peel-off rays (0: six per core)")
    ap.add_argument("--cpu-packets-cut", type=int, default=0,
                    help="oracle packets with the exp(-tau) = 0 cut (0: 64 per core)")
    ap.add_argument("--regroup", type=int, default=None, choices=[0, 1],
                    help="transport loop with one rejection round per pass (1) or the looping draw (0); "
                         "default: the library's default")
    ap.add_argument("--compact", type=int, default=None, choices=[0, 1],
                    help="complete run: gather the last packets into fewer waves (library default 1)")
    ap.add_argument("--complete-run", type=int, default=1,
                    help="dusty_sphere: also time one complete FP32 run of all queued packets (1) or not (0)")
    ap.add_argument("--only", choices=["fp32", "fp64", "both"], default="both")
    ap.add_argument("--copy-gib", type=float, default=1.0, help="size of the copy used to measure HBM bandwidth")
    ap.add_argument("--workload", choices=["dusty_sphere", "shell", "batch", "adjoint", "core_skip",
                                           "voigt_accuracy", "upar_cost", "c1_slab", "multi_species", "mesh_overhead"],
                    default="dusty_sphere",
                    help="dusty_sphere: the headline; the others: the other configurations")
    ap.add_argument("--skip-packets", type=int, default=4_000_000, help="core_skip: packets per complete run")
    ap.add_argument("--voigt-packets", type=int, default=200_000, help="voigt_accuracy: packets per run")
    ap.add_argument("--upar-packets", type=int, default=1_000_000, help="upar_cost: packets per run")
    ap.add_argument("--vmax", type=float, default=200.0, help="shell: outflow speed at R (km/s)")
    ap.add_argument("--leaves", type=float, default=2e7, help="adjoint: target leaf count")
    ap.add_argument("--sources", type=int, default=100_000, help="adjoint: sources (100 rays each)")
    ap.add_argument("--galaxy-cache", default=None, help="adjoint: .npz file holding the generated galaxy")
    return ap.parse_args()


def _line(metric, value, unit, steps, warm, ms_per_step, dtype, config, roofline, **extra):
    d = {"metric": metric, "value": value, "unit": unit, "n_gpus": 1, "steps": steps, "warmup": warm,
         "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
         "dtype": dtype, "data": "synthetic", "config": config, "roofline": roofline}
    d.update(extra)
    return d


def stream_rate(ctx, steps, warm, tag):
    """Warm-up then timed stream steps of an open stream; totals and wall."""
    import torch
    for _ in range(warm):
        ctx.stream_step()
    torch.cuda.synchronize()
    tot, kms = {}, []
    t0 = time.perf_counter()
    for _ in range(steps):
        st, rem = ctx.stream_step()
        kms.append(st["kernel_ms"])
        for k, v in st.items():
            tot[k] = tot.get(k, 0) + v
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    print(f"# {tag}: {steps} steps in {wall:.3f} s, transport ms {[round(k, 1) for k in kms]}, remaining {rem}, "
          f"stats {tot}", file=sys.stderr, flush=True)
    return wall, tot, kms


def oracle_transport_baseline(a, probs, packets_each, max_events):
    """The oracle on a bounded sample: packets_each packets of every problem,
    each stopped after max_events interactions; FP64, full peel-off rays."""
    if a.no_cpu_baseline:
        return None
    from oracle import oracle as O
    cores = host_cores()[0]
    scat, dt, setup = 0, 0.0, 0.0
    for p in probs:
        n = min(packets_each, len(p.sources.x))
        # the oracle rebuilds its leaf hash map on every call: time that
        # with a one-event call and subtract it
        t0 = time.perf_counter()
        O.run(p, p.seed, first=0, n=1, threads=1, max_events=1, with_cubes=False)
        t_set = time.perf_counter() - t0
        t0 = time.perf_counter()
        r = O.run(p, p.seed, first=0, n=n, threads=cores, max_events=max_events)
        dt += max(time.perf_counter() - t0 - t_set, 1e-9)
        setup += t_set
        scat += r["stats"]["scatterings"]
    return {"value": scat / dt, "unit": "scatterings/s", "cores": cores, "kind": "oracle",
            "sample": f"{packets_each} packets of each of {len(probs)} problem(s), each stopped after "
                      f"{max_events} interactions: {scat} scatterings in {dt:.1f} s (set-up {setup:.1f} s "
                      f"subtracted)"}


def transport_roofline(tot, kms, prec, kernel):
    n = len(kms)
    avg_ms = sum(kms) / n
    fl = (FLOP_PER_SCATTERING * tot["scatterings"] + FLOP_PER_CROSSING * (tot["crossings"] + tot["peel_rays"])) / n
    ach = fl / (avg_ms * 1e-3) / 1e12
    return {"bound": "alu", "achieved": ach, "peak": PEAK[prec], "unit": "TFLOP/s", "frac": ach / PEAK[prec],
            "traffic": None, "kernel": kernel}


def bench_shell(a, rmc, W):
    """C3: outflowing shell, 2.36e6 leaves, tau0 = 1e7 across the shell,
    tau_dust = 1, three observers with 256x256x200 cubes, 1e7 packets
    queued; FP32, streaming steps as the headline."""
    pb = W.c3_shell(rmc.sigma0, vmax_kms=a.vmax, n_packets=10_000_000)
    print(f"# shell: {pb.mesh.n} leaves, vmax {a.vmax} km/s", file=sys.stderr, flush=True)
    ctx = rmc.Context.from_problem(pb, "fp32")
    import torch
    ctx.set_stream(torch.cuda.current_stream())
    ctx.set_option(rmc.OPT_SLICE_ITERS, a.slice)
    ctx.stream_begin(pb.seed, 0, 10_000_000)
    wall, tot, kms = stream_rate(ctx, a.steps, a.warmup, "shell fp32")
    ctx.close()
    cpu = oracle_transport_baseline(a, [pb], 8 * host_cores()[0], 20000)
    return _line("scatterings/s + ray-cell crossings/s (1 GPU), FP32", tot["scatterings"] / wall, "scatterings/s",
                 a.steps, a.warmup, 1e3 * wall / a.steps, "f32",
                 {"workload": f"outflowing_shell_vmax{int(a.vmax)}_tau1e7_{pb.mesh.n}_leaves_3x256x256x200",
                  "packets_queued": 10_000_000, "iterations_per_lane_per_step": a.slice, "parallelism": "none"},
                 transport_roofline(tot, kms, "fp32", "k_transport<float,false,true,1>"),
                 crossings_per_s=(tot["crossings"] + tot["peel_crossings"]) / wall,
                 transport_ms_avg=sum(kms) / len(kms), peel_pass_ms_avg=tot["peel_pass_ms"] / len(kms),
                 cpu_baseline=cpu)


def bench_batch(a, rmc, W):
    """C4: 64 uneven problems (slab/sphere, Lya or the MgII doublet, tau0 in
    [1e3, 1e7], T in [1e2, 1e5] K, 8^3-128^3 lognormal grids, 1e3-1e6
    packets) in one persistent launch; launch shape from the autotuner;
    FP32, streaming steps over the whole batch."""
    probs = W.c4_batch(rmc.sigma0)
    ctxs = [rmc.Context.from_problem(p, "fp32") for p in probs]
    import torch
    for c in ctxs:
        c.set_stream(torch.cuda.current_stream())
    seeds = [p.seed for p in probs]
    npk = [len(p.sources.x) for p in probs]
    best = rmc.batch_autotune(ctxs, seeds, npk)
    print(f"# batch: {len(probs)} problems, {sum(npk)} packets, tuned {best}", file=sys.stderr, flush=True)
    rmc.batch_begin(ctxs, seeds, npk)
    wall, tot, kms = stream_rate(ctxs[0], a.steps, a.warmup, "batch fp32")
    for c in ctxs:
        c.close()
    cpu = oracle_transport_baseline(a, probs, 4, 20000)
    return _line("scatterings/s + ray-cell crossings/s (1 GPU), FP32", tot["scatterings"] / wall, "scatterings/s",
                 a.steps, a.warmup, 1e3 * wall / a.steps, "f32",
                 {"workload": "batch_64_problems_slab_sphere_lya_mgii", "problems": len(probs),
                  "packets": int(sum(npk)), "tuned": best, "parallelism": "none"},
                 transport_roofline(tot, kms, "fp32", "k_transport<float,true,true,4>"),
                 crossings_per_s=(tot["crossings"] + tot["peel_crossings"]) / wall, cpu_baseline=cpu)


def bench_core_skip(a, rmc, W):
    """Core-skipping on a thick static sphere (tau0 = 1e7, T = 1e4 K, 8^3
    grid, Lya dipole with recoil, +z 128x128x100 cube): each step is a
    complete FP32 run of 4e6 packets with core-skipping (tau_skip = 1,
    f = 0.2).  Unbiased walks here take ~1e7 scatterings each, so the
    unbiased path is not run to completion: its scattering rate on the same
    problem is measured over a few streaming launches."""
    import torch
    n = a.skip_packets
    pb = W.thick_sphere(rmc.sigma0, n_packets=n)
    print(f"# core_skip: {pb.mesh.n} leaves, {n} packets per step", file=sys.stderr, flush=True)
    ctx = rmc.Context.from_problem(pb, "fp32")
    ctx.set_stream(torch.cuda.current_stream())
    ctx.set_core_skip(1.0, 0.2)
    for _ in range(a.warmup):
        ctx.run(pb.seed, 0, min(n, 20000))
    torch.cuda.synchronize()
    tot, kms = {}, []
    t0 = time.perf_counter()
    for i in range(a.steps):
        ctx.reset_cubes()
        st = ctx.run(pb.seed, 0, n)
        kms.append(st["kernel_ms"])
        for k, v in st.items():
            tot[k] = tot.get(k, 0) + v
        print(f"# core_skip run {i}: transport {st['kernel_ms']:.1f} ms, {st['scatterings']} scatterings, "
              f"{st['escaped']} escaped", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ctx.close()
    # the unbiased path on the same problem, streaming
    cu = rmc.Context.from_problem(pb, "fp32")
    cu.set_stream(torch.cuda.current_stream())
    cu.set_option(rmc.OPT_SLICE_ITERS, a.slice)
    cu.stream_begin(pb.seed, 0, n)
    wall_u, tot_u, _ = stream_rate(cu, 3, 1, "unbiased fp32")
    cu.close()
    cpu = None
    if not a.no_cpu_baseline:
        from oracle import oracle as O
        cores = host_cores()[0]
        m = 8 * cores
        t0 = time.perf_counter()
        r = O.run(pb, pb.seed, first=0, n=m, threads=cores, core_skip=(1.0, 0.2))
        dt = time.perf_counter() - t0
        cpu = {"value": m / dt, "unit": "packets/s", "cores": cores, "kind": "oracle",
               "sample": f"{m} complete packets of the same problem with core-skipping and peel-off: "
                         f"{r['stats']['scatterings']} scatterings in {dt:.1f} s"}
    return _line("packets/s (complete runs, 1 GPU), FP32, core-skipping", n * a.steps / wall, "packets/s",
                 a.steps, a.warmup, 1e3 * wall / a.steps, "f32",
                 {"workload": f"thick_sphere_tau1e7_T1e4_{pb.mesh.n}_leaves_128x128x100", "packets": n,
                  "core_skip": {"tau_skip": 1.0, "frac": 0.2}, "parallelism": "none"},
                 transport_roofline(tot, kms, "fp32", "k_transport<float,false,true,1>"),
                 scatterings_per_s=tot["scatterings"] / wall,
                 scatterings_per_packet=tot["scatterings"] / (n * a.steps),
                 unbiased_scatterings_per_s=tot_u["scatterings"] / wall_u,
                 cpu_baseline=cpu)


def bench_voigt_accuracy(a, rmc, W):
    """The paper's accumulated Voigt-error experiment (Sect. 4.2, static
    slab, central monochromatic Lya source, T = 10 K so a = 0.015) at
    tau0 = 1e6: the same packets run to completion on the double path with
    the Tasitsiomi form and with the accurate H (RMC_OPT_VOIGT = 1), and
    the two escape spectra are compared bin by bin in units of the Poisson
    error.  The accurate run's scatterings/s is the line's value."""
    import numpy as np
    import torch
    from scipy import stats
    n = a.voigt_packets
    pb = W.static_slab(rmc.sigma0, 1e6, 10.0, n, level=0)
    print(f"# voigt_accuracy: slab tau0 = 1e6, T = 10 K, {n} packets, FP64", file=sys.stderr, flush=True)
    res = {}
    for mode in (0, 1):
        ctx = rmc.Context.from_problem(pb, "fp64", observers=False)
        ctx.set_stream(torch.cuda.current_stream())
        ctx.set_option(rmc.OPT_VOIGT, mode)
        ctx.set_option(rmc.OPT_SLICE_ITERS, a.slice)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.stream_begin(pb.seed, 0, n)
        tot, kms, step, rem = {}, [], 0, n
        while rem > 0:
            st, rem = ctx.stream_step()
            kms.append(st["kernel_ms"])
            for k, v in st.items():
                tot[k] = tot.get(k, 0) + v
            step += 1
            if step % 200 == 0:
                print(f"# voigt {mode}: step {step}, {rem} packets left", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        out = ctx.get_packets()
        ctx.close()
        print(f"# voigt {mode}: {step} launches in {wall:.1f} s, {tot['scatterings']} scatterings",
              file=sys.stderr, flush=True)
        res[mode] = (wall, tot, kms, out)
    (w0, t0_, k0, o0), (w1, t1_, k1, o1) = res[0], res[1]
    e0, e1 = o0["status"] == 1, o1["status"] == 1
    h0, edges = np.histogram(o0["x"][e0], bins=120, range=(-60, 60))
    h1, _ = np.histogram(o1["x"][e1], bins=120, range=(-60, 60))
    sel = (h0 + h1) > 0
    zb = (h1[sel] - h0[sel]) / np.sqrt(h0[sel] + h1[sel])
    both = e0 & e1
    dx = np.abs(o1["x"][both]) - np.abs(o0["x"][both])
    steps = len(k1)
    rl = transport_roofline(t1_, k1, "fp64", "k_transport<double,false,true,1>")
    return _line("scatterings/s (1 GPU), FP64 with the accurate Voigt function", t1_["scatterings"] / w1,
                 "scatterings/s", steps, 0, 1e3 * w1 / steps, "f64",
                 {"workload": "static_slab_tau1e6_T10_lya_central_source", "packets": n,
                  "iterations_per_lane_per_step": a.slice, "parallelism": "none"}, rl,
                 tasitsiomi_scatterings_per_s=t0_["scatterings"] / w0,
                 packets_per_s={"accurate": n / w1, "tasitsiomi": n / w0},
                 spectrum_difference={
                     "bins": int(sel.sum()), "within_1_sigma": float(np.mean(np.abs(zb) <= 1)),
                     "within_2_sigma": float(np.mean(np.abs(zb) <= 2)), "chi2_per_bin": float(np.mean(zb ** 2)),
                     "note": "same packets and draws in both runs (common random numbers): the bin "
                             "differences are the systematic effect of H plus the walks it decorrelates",
                     "ks_p": float(stats.ks_2samp(o0["x"][e0], o1["x"][e1]).pvalue),
                     "mean_abs_x": {"tasitsiomi": float(np.abs(o0["x"][e0]).mean()),
                                    "accurate": float(np.abs(o1["x"][e1]).mean())},
                     "paired_abs_x_shift": float(dx.mean()),
                     "paired_abs_x_shift_se": float(dx.std() / np.sqrt(max(len(dx), 1))),
                     "mean_scatterings": {"tasitsiomi": float(o0["n_scat"].mean()),
                                          "accurate": float(o1["n_scat"].mean())}},
                 cpu_baseline=None if a.no_cpu_baseline else oracle_voigt_baseline(pb))


def oracle_voigt_baseline(pb):
    """The oracle with the accurate H on a bounded sample of the same slab."""
    from oracle import oracle as O
    cores = host_cores()[0]
    m, ev = 2 * cores, 20000
    t0 = time.perf_counter()
    r = O.run(pb, pb.seed, first=0, n=m, threads=cores, max_events=ev, with_cubes=False, voigt_exact=True)
    dt = time.perf_counter() - t0
    return {"value": r["stats"]["scatterings"] / dt, "unit": "scatterings/s", "cores": cores, "kind": "oracle",
            "sample": f"{m} packets of the same slab with the accurate H (quadrature), each stopped after {ev} "
                      f"interactions: {r['stats']['scatterings']} scatterings in {dt:.1f} s"}


def bench_multi_species(a, rmc, W):
    """Multi-species media: the Fe II wind of the paper's idealised-set-up
    example (Fe II 2587 and 2600 with their three fluorescent channels,
    flat continuum source, v ~ r to 100 km/s, density ~ r^-3, 64^3 grid) as
    complete FP32 runs of 4e6 packets, and the appendix's H I + D sphere
    (N_HI = 2e19, D/H = 3e-5, T = 1e4 K) as FP32 streaming steps."""
    import torch
    n = 4_000_000
    pb = W.feii_wind(rmc.sigma0, n)
    ctx = rmc.Context.from_problem(pb, "fp32", observers=False)
    ctx.set_stream(torch.cuda.current_stream())
    ctx.run(pb.seed, 0, 100_000)
    torch.cuda.synchronize()
    tot, t0 = {}, time.perf_counter()
    for _ in range(a.steps):
        st = ctx.run(pb.seed, 0, n)
        for k, v in st.items():
            tot[k] = tot.get(k, 0) + v
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ctx.close()
    print(f"# feii wind: {a.steps} runs of {n} packets in {wall:.2f} s, {tot['scatterings']} scatterings",
          file=sys.stderr, flush=True)
    pd = W.deuterium_sphere(rmc.sigma0, 1_000_000)
    cd = rmc.Context.from_problem(pd, "fp32", observers=False)
    cd.set_stream(torch.cuda.current_stream())
    cd.set_option(rmc.OPT_SLICE_ITERS, a.slice)
    cd.stream_begin(pd.seed, 0, 1_000_000)
    wd, td, kd = stream_rate(cd, a.steps, a.warmup, "H+D sphere fp32")
    cd.close()
    cpu = None
    if not a.no_cpu_baseline:
        from oracle import oracle as O
        cores = host_cores()[0]
        m = 250000 * cores     # a few seconds of the oracle
        pw = W.feii_wind(rmc.sigma0, m)
        t1 = time.perf_counter()
        r = O.run(pw, pw.seed, threads=cores, with_cubes=False)
        dt = time.perf_counter() - t1
        cpu = {"value": m / dt, "unit": "packets/s", "cores": cores, "kind": "oracle",
               "sample": f"{m} complete packets of the Fe II wind ({r['stats']['scatterings']} scatterings) "
                         f"in {dt:.1f} s"}
    return _line("packets/s (complete runs, 1 GPU), FP32, Fe II wind with fluorescence", n * a.steps / wall,
                 "packets/s", a.steps, 1, 1e3 * wall / a.steps, "f32",
                 {"workload": "feii_wind_2587_2600_fluorescent_flat_continuum_64cubed", "packets": n,
                  "parallelism": "none"},
                 transport_roofline(td, kd, "fp32", "k_transport<float,false,true,4>"),
                 feii_wind={"packets_per_s": n * a.steps / wall, "scatterings_per_s": tot["scatterings"] / wall,
                            "scatterings_per_packet": tot["scatterings"] / (n * a.steps)},
                 deuterium_sphere={"scatterings_per_s": td["scatterings"] / wd,
                                   "transport_ms_avg": sum(kd) / len(kd),
                                   "workload": "static_sphere_NHI2e19_DH3e-5_T1e4_lya_dlya",
                                   "note": "the roofline object is this sphere's transport kernel (two lines: "
                                           "the multi-line kernel)"},
                 cpu_baseline=cpu)


def bench_c1_slab(a, rmc, W):
    """C1: the plain FP64 slab (tau0 = 1e4, T = 1e4 K, 512 leaves, 1000
    packets from the mid-plane at x = 0): a latency and parity case.  Each
    step is a complete run of the 1000 packets; the oracle runs the same
    packets, and the two 200-bin spectra over x in [-60, 60) and mean
    scattering counts are compared."""
    import numpy as np
    import torch
    from scipy import stats
    from oracle import oracle as O
    pb = W.c1_slab(rmc.sigma0)
    n = len(pb.sources.x)
    ctx = rmc.Context.from_problem(pb, "fp64", observers=False)
    ctx.set_stream(torch.cuda.current_stream())
    for _ in range(a.warmup):
        ctx.run(pb.seed, 0, n)
    torch.cuda.synchronize()
    sc, t0 = 0, time.perf_counter()
    for _ in range(a.steps):
        st = ctx.run(pb.seed, 0, n)
        sc += st["scatterings"]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    out = ctx.get_packets()
    ctx.close()
    cores = host_cores()[0]
    t1 = time.perf_counter()
    ref = O.run(pb, pb.seed, threads=cores, with_cubes=False)
    dt = time.perf_counter() - t1
    hg, _ = np.histogram(out["x"], bins=200, range=(-60, 60))
    ho, _ = np.histogram(ref["x"], bins=200, range=(-60, 60))
    return _line("run time of the slab (1 GPU, FP64), as scatterings/s", sc / wall, "scatterings/s", a.steps,
                 a.warmup, 1e3 * wall / a.steps, "f64",
                 {"workload": "c1_slab_tau1e4_T1e4_512_leaves_1000_packets", "packets": n, "parallelism": "none"},
                 None, ms_per_complete_run=1e3 * wall / a.steps,
                 parity={"identical_packets": int(np.sum((out["status"] == ref["status"]) &
                                                         (out["n_scat"] == ref["n_scat"]) &
                                                         (np.abs(out["x"] - ref["x"]) < 1e-9))),
                         "histogram_identical": bool(np.array_equal(hg, ho)),
                         "mean_scatterings": {"gpu": float(out["n_scat"].mean()), "oracle": float(ref["n_scat"].mean())},
                         "ks_p": float(stats.ks_2samp(out["x"], ref["x"]).pvalue)},
                 cpu_baseline={"value": ref["stats"]["scatterings"] / dt, "unit": "scatterings/s", "cores": cores,
                               "kind": "oracle", "sample": f"the same {n} packets, complete: "
                                                           f"{ref['stats']['scatterings']} scatterings in {dt:.1f} s"})


def bench_mesh_overhead(a, rmc, W):
    """The cost of the mesh (the paper's timing beside its error budget,
    Sect. 4.5): packets from the centre of a uniform sphere whose
    scatterings keep their direction, the sphere in one cell and on a
    256^3 mesh, at tau0 = 1e-10 (no scattering: the packet only crosses
    cells) and 1e4 (ten thousand scatterings per packet), 1e6 packets (a
    full GPU), both precisions.  Each step is a complete run; the line's
    value is the FP32 crossings/s on the mesh at tau0 = 1e-10, a lower
    bound on the traversal rate (the run's per-packet costs included)."""
    import numpy as np
    import torch
    from oracle import oracle as O
    cases = {}
    sigma0 = rmc.sigma0(W.LYA, 1e4)
    for level in (0, 8):
        pb = W.static_sphere(rmc.sigma0, 1.0, 1e4, 1_000_000, level=level)
        nl, R = pb.mesh.n, 0.5 * pb.mesh.box_cm
        for prec in ("fp32", "fp64"):
            ctx = rmc.Context.from_problem(pb, prec, observers=False)
            ctx.set_stream(torch.cuda.current_stream())
            ctx.set_option(rmc.OPT_FORWARD_ONLY, 1)
            for tau0, n in ((1e-10, 1_000_000), (1e4, 1_000_000)):
                ctx.set_gas(np.full(nl, tau0 / (sigma0 * R)), np.full(nl, 1e4), np.zeros(3 * nl), np.zeros(nl))
                ctx.run(1, 0, min(n, 20_000))
                torch.cuda.synchronize()
                t0, tot = time.perf_counter(), {}
                for s in range(a.steps):
                    st = ctx.run(2 + s, 0, n)
                    for k, v in st.items():
                        tot[k] = tot.get(k, 0) + v
                torch.cuda.synchronize()
                wall = (time.perf_counter() - t0) / a.steps
                key = f"{prec}_level{level}_tau{tau0:g}"
                cases[key] = {"packets": n, "ms_per_run": 1e3 * wall, "us_per_packet": 1e6 * wall / n,
                              "scatterings_per_s": tot["scatterings"] / a.steps / wall,
                              "crossings_per_s": tot["crossings"] / a.steps / wall,
                              "crossings_per_packet": tot["crossings"] / a.steps / n}
                print(f"# mesh_overhead {key}: {cases[key]}", file=sys.stderr, flush=True)
            ctx.close()
    ratio = {f"{p}_tau{t:g}": cases[f"{p}_level8_tau{t:g}"]["us_per_packet"] / cases[f"{p}_level0_tau{t:g}"]["us_per_packet"]
             for p in ("fp32", "fp64") for t in (1e-10, 1e4)}
    # the oracle on the same mesh, no scattering: crossings/s on the host
    # cores, its set-up (tree build) subtracted with a run of 1000 packets
    cores = host_cores()[0]
    runs = []
    for m in (1000, 400_000):
        pbo = W.static_sphere(rmc.sigma0, 1e-10, 1e4, m, level=8)
        t1 = time.perf_counter()
        r = O.run(pbo, 3, threads=cores, forward_only=True, with_cubes=False)
        runs.append((time.perf_counter() - t1, r["stats"]["crossings"]))
    dt, ncr = runs[1][0] - runs[0][0], runs[1][1] - runs[0][1]
    main = cases["fp32_level8_tau1e-10"]
    return _line("ray-cell crossings/s (1 GPU), FP32, packets crossing a 256^3 mesh without scattering",
                 main["crossings_per_s"], "crossings/s", a.steps, 1, main["ms_per_run"], "f32",
                 {"workload": "uniform_sphere_256cubed_forward_only", "parallelism": "none"}, None,
                 cases=cases, mesh_over_one_cell_time_per_packet=ratio,
                 cpu_baseline={"value": ncr / dt, "unit": "crossings/s", "cores": cores,
                               "kind": "oracle", "sample": f"399000 packets of the same mesh at tau0 = 1e-10 "
                                                           f"(a 400000-packet run less a 1000-packet one): "
                                                           f"{ncr} crossings in {dt:.2f} s"})


def bench_upar_cost(a, rmc, W):
    """Cost of the scattering against the incoming frequency (the paper's
    u_parallel timing, Sect. 3.3.3): forward-only flights (each scattering
    keeps direction and frequency but draws its atom velocity as usual) in
    a static Lya medium of tau0 = 1e12, every packet emitted at x_in and
    stopped at its 2000th event, so the kernel's time is that of scatterings
    at x_in; a = 1e-4, 1e-3, 1e-2 (T from a), x_in = 0..10.  The oracle's
    u_parallel sampler is timed on one core beside it."""
    import numpy as np
    import torch
    from oracle import oracle as O
    n = a.upar_packets
    q1 = O.line_quantities(W.LYA, 1e4)
    xs = [0.0, 1.0, 2.0, 3.0, 4.0, 5.0, 6.0, 8.0, 10.0]
    rows, rates, walls = [], [], []
    for av in (1e-4, 1e-3, 1e-2):
        T = 1e4 * (q1["a"] / av) ** 2          # a ~ T^-1/2
        for x in xs:
            pb = W.static_sphere(rmc.sigma0, 1e12, T, n, level=0, isotropic=True, recoil=False)
            pb.sources.x[:] = x
            ctx = rmc.Context.from_problem(pb, "fp32", observers=False)
            ctx.set_stream(torch.cuda.current_stream())
            ctx.set_option(rmc.OPT_FORWARD_ONLY, 1)
            ctx.set_option(rmc.OPT_MAX_EVENTS, 2000)
            ctx.run(pb.seed, 0, n)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ms, sc = 0.0, 0
            for _ in range(a.steps):
                st = ctx.run(pb.seed, 0, n)
                ms += st["kernel_ms"]
                sc += st["scatterings"]
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            walls.append(wall / a.steps)
            ctx.close()
            m = 20000
            t1 = time.perf_counter()
            O.sample_upar(m, x, av, seed=3)
            cpu = m / (time.perf_counter() - t1)
            rate = sc / (ms * 1e-3)
            rates.append(rate)
            rows.append({"a": av, "x_in": x, "gpu_scatterings_per_s": rate, "wall_scatterings_per_s": sc / wall,
                         "oracle_draws_per_s_1core": cpu})
            print(f"# upar a={av:g} x={x:g}: {rate:.3e} scatterings/s (kernel), oracle {cpu:.3e} draws/s",
                  file=sys.stderr, flush=True)
    geo = float(np.exp(np.mean(np.log(rates))))
    return _line("scatterings/s at fixed x_in (1 GPU, FP32), u_parallel cost against x_in", geo, "scatterings/s",
                 a.steps, 1, 1e3 * float(np.mean(walls)), "f32",
                 {"workload": "forward_only_scatterings_lya_tau1e12_a1e-4_1e-3_1e-2_x0-10", "packets": n,
                  "events_per_packet": 2000,
                  "parallelism": "none"}, None,
                 note="value: geometric mean over the (a, x_in) grid of the transport kernel's rate; every "
                      "scattering of a run happens at x_in",
                 grid=rows, spread=float(max(rates) / min(rates)),
                 cpu_baseline={"value": float(np.exp(np.mean(np.log([r["oracle_draws_per_s_1core"] for r in rows])))),
                               "unit": "u_parallel draws/s", "cores": 1, "kind": "oracle",
                               "sample": "20,000 u_parallel draws per grid point on one core (geometric mean)"})


def measure_copy(a):
    """Achievable HBM bandwidth: a plain copy kernel (an elementwise multiply
    by one, reading and writing copy_gib each, so that it runs as a kernel
    rather than a DMA transfer); the same kernel calibrates the profiler's
    traffic counters."""
    import torch
    n_el = int(a.copy_gib * (1 << 30)) // 4
    src = torch.ones(n_el, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        torch.mul(src, 1.0, out=dst)
    e1.record()
    torch.cuda.synchronize()
    gbps = 5 * 2 * n_el * 4 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    print(f"# copy: {gbps:.1f} GB/s (read+write of {a.copy_gib} GiB)", file=sys.stderr, flush=True)
    return gbps


def galaxy_problem(a, rmc, W):
    """The C5 galaxy (a few minutes to generate at full size); with
    --galaxy-cache PATH it is read from / written to an .npz file, so that
    several profiler passes of one session generate it once."""
    import numpy as np
    if a.galaxy_cache and os.path.exists(a.galaxy_cache):
        z = np.load(a.galaxy_cache)
        mesh = W.Mesh(z["level"], z["ijk"])
        gas = W.Gas(z["n_hi"], z["T"], z["v"], z["kappa_d"])
        nx = int(z["nx"])
        obs = [W.Observer((0.0, 0.0, 1.0), nx, nx, 1, (-0.5, 0.5, -0.5, 0.5), -1e30, 1e30)]
        pb = W.Problem("c5_galaxy", mesh, gas, W.Domain(W.DOM_BOX, (0.0, 0.0, 0.0, 0.0)), [W.LYA], 1e4,
                       W.Dust(0.32, 0.73), W.Sources(z["src"], np.zeros(len(z["src"]))), obs)
        pb.meta.update(rays=dict(orig=z["orig"], x_ext=z["x_ext"], w=z["w"]), grad_image=z["G"])
        return pb
    pb = W.c5_galaxy(rmc.sigma0, target_leaves=a.leaves, n_sources=a.sources,
                     log=lambda m: print("# " + m, file=sys.stderr, flush=True))
    if a.galaxy_cache:
        r = pb.meta["rays"]
        np.savez(a.galaxy_cache, level=pb.mesh.level, ijk=pb.mesh.ijk, n_hi=pb.gas.n_hi, T=pb.gas.T, v=pb.gas.v,
                 kappa_d=pb.gas.kappa_d, src=pb.sources.pos, orig=r["orig"], x_ext=r["x_ext"], w=r["w"],
                 G=pb.meta["grad_image"], nx=pb.observers[0].nx)
    return pb


def bench_adjoint(a, rmc, W):
    """C5: galaxy-like adaptive mesh (~2e7 leaves), 1e7 fixed rays toward
    +z, 512^2 image; one forward image and one backward (gradients per
    leaf) per step, FP32 leaf records; the backward reads the forward's
    crossing lists (the replaying backward is measured beside it)."""
    import torch
    copy_GBps = measure_copy(a)
    t0 = time.perf_counter()
    pb = galaxy_problem(a, rmc, W)
    r = pb.meta["rays"]
    print(f"# adjoint: {pb.mesh.n} leaves, {len(r['x_ext'])} rays, generated in {time.perf_counter() - t0:.0f} s",
          file=sys.stderr, flush=True)
    ctx = rmc.Context.from_problem(pb, "fp32", sources=False)
    ctx.set_stream(torch.cuda.current_stream())
    dev = torch.device("cuda:0")
    o = torch.tensor(r["orig"], dtype=torch.float64, device=dev)
    x = torch.tensor(r["x_ext"], dtype=torch.float64, device=dev)
    w = torch.tensor(r["w"], dtype=torch.float64, device=dev)
    G = torch.tensor(pb.meta["grad_image"], dtype=torch.float64, device=dev)

    def run(tape):
        fwd, bwd = [], []
        t_all = 0.0
        for i in range(a.warmup + a.steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if tape:
                ctx.raycast_image_tape(0, o, x, w)
            else:
                ctx.raycast_image(0, o, x, w)
            f = ctx.image_stats()
            if tape:
                ctx.raycast_image_backward_tape(G)
            else:
                ctx.raycast_image_backward(0, o, x, w, G)
            b = ctx.image_stats()
            torch.cuda.synchronize()
            if i >= a.warmup:
                fwd.append(f)
                bwd.append(b)
                t_all += time.perf_counter() - t0
        n = a.steps
        cf = sum(c for c, _ in fwd) / n
        cb = sum(c for c, _ in bwd) / n
        mf = sum(m for _, m in fwd) / n
        mb = sum(m for _, m in bwd) / n
        return cf, cb, mf, mb, t_all

    # the tape path (forward records the crossing lists, backward reads
    # them) and the replaying backward, on the same rays
    tf, tb, tmf, tmb, t_tape = run(True)
    rf, rb, rmf, rmb, t_rep = run(False)
    n = a.steps
    # algorithmic bytes per crossing, FP32 records: forward 24-B leaf record +
    # 4-B node entry, plus the 8-B tape entry it writes; tape backward 8-B
    # tape entry + 24-B leaf record + three 8-B gradient read-modify-writes
    gbs_tf = tf * (28.0 + 8.0) / (tmf * 1e-3) / 1e9
    gbs_tb = tb * (8.0 + 24.0 + 48.0) / (tmb * 1e-3) / 1e9
    gbs_rf = rf * 28.0 / (rmf * 1e-3) / 1e9
    tr_f = measured_traffic("k_image_fwd_tape", "adjoint_traffic.json")
    tr_b = measured_traffic("k_image_bwd_tape", "adjoint_traffic.json")
    if tmf >= tmb:
        roof = {"bound": "hbm", "achieved": gbs_tf, "peak": 8000.0, "unit": "GB/s", "frac": gbs_tf / 8000.0,
                "traffic": tr_f, "kernel": "k_image_fwd_tape<float>"}
    else:
        roof = {"bound": "hbm", "achieved": gbs_tb, "peak": 8000.0, "unit": "GB/s", "frac": gbs_tb / 8000.0,
                "traffic": tr_b, "kernel": "k_image_bwd_tape<float>"}
    ctx.close()
    cpu = None
    if not a.no_cpu_baseline:
        # the oracle on a bounded sample of the same rays (image and exact
        # gradient in one call: one walk per ray plus the gradient of each
        # crossing, counted twice like the GPU's forward + backward); its
        # set-up (hash map of the leaves), timed with a one-ray call, is
        # subtracted
        from oracle import oracle as O
        import numpy as np
        cores = host_cores()[0]
        ns = 2_000_000
        ob = pb.observers[0]
        t0 = time.perf_counter()
        O.raycast_image(pb, ob, r["orig"][:1], r["x_ext"][:1], r["w"][:1], pb.meta["grad_image"], threads=cores)
        t_setup = time.perf_counter() - t0
        nc = np.zeros(1, dtype=np.int64)
        t0 = time.perf_counter()
        O.raycast_image(pb, ob, r["orig"][:ns], r["x_ext"][:ns], r["w"][:ns], pb.meta["grad_image"], threads=cores,
                        crossings=nc)
        dt = max(time.perf_counter() - t0 - t_setup, 1e-9)
        cpu = {"value": 2 * int(nc[0]) / dt, "unit": "crossings/s", "cores": cores, "kind": "oracle",
               "sample": f"first {ns} rays, image + exact gradient: {int(nc[0])} crossings walked (counted twice) "
                         f"in {dt:.1f} s after a {t_setup:.1f} s set-up"}
    # crossings of the forward walk, counted twice (image and its adjoint)
    return _line("adjoint ray-cell crossings/s (forward image + backward gradients, 1 GPU), FP32 records",
                 2.0 * tf * n / t_tape, "crossings/s", n, a.warmup, 1e3 * t_tape / n, "f32",
                 {"workload": f"galaxy_{pb.mesh.n}_leaves_{len(r['x_ext'])}_rays_512x512", "parallelism": "none",
                  "backward": "tape"},
                 roof,
                 forward={"crossings_per_launch": tf, "ms": tmf, "GBps_algorithmic": gbs_tf,
                          "GBps_measured": None if tr_f is None else tr_f / (tmf * 1e-3) / 1e9},
                 backward={"crossings_per_launch": tb, "ms": tmb, "GBps_algorithmic": gbs_tb,
                           "GBps_measured": None if tr_b is None else tr_b / (tmb * 1e-3) / 1e9},
                 hbm_copy_GBps=copy_GBps,
                 replay={"crossings_per_s": 2.0 * rf * n / t_rep, "ms_per_step": 1e3 * t_rep / n,
                         "forward_ms": rmf, "backward_ms": rmb, "forward_GBps_algorithmic": gbs_rf},
                 cpu_baseline=cpu)


def complete_run(pb, P, rmc, torch, regroup=None, compact=None):
    """One complete FP32 run of all P queued packets (every walk to its end,
    the tail of the longest walks included), timed by the wall clock and by
    the library's events; its outputs feed the comparison with the oracle."""
    ctx = rmc.Context.from_problem(pb, "fp32")
    ctx.set_stream(torch.cuda.current_stream())
    if regroup is not None:
        ctx.set_option(rmc.OPT_REGROUP, regroup)
    if compact is not None:
        ctx.set_option(rmc.OPT_COMPACT, compact)
    ctx.set_option(rmc.OPT_SLICE_ITERS, 8192)
    # streamed launch by launch (the same packets as rmc_run), so that the
    # bulk, while every lane holds a packet, and the tail, while the last
    # walks finish, can be told apart
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.stream_begin(pb.seed, 0, P)
    hist = []
    rem = P
    while rem > 0:
        sl, rem = ctx.stream_step()
        hist.append((time.perf_counter() - t0, rem, sl["scatterings"]))
    st = ctx.stream_end()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    out = ctx.get_packets()
    out["cube"] = ctx.get_cube(0)
    ctx.close()
    print(f"# complete fp32 run: {P} packets in {wall:.2f} s, {st}", file=sys.stderr, flush=True)
    # the tail: launches after the one in which 90% of the packets had ended
    k90 = next(i for i, (_, r, _) in enumerate(hist) if r <= 0.1 * P)
    t90 = hist[k90][0]
    t_end = {f: next(h[0] for h in hist if h[1] <= (1.0 - f) * P) for f in (0.99, 0.999)}
    scat_tail = sum(h[2] for h in hist[k90 + 1:])
    rec = {"packets": P, "seconds": wall, "scatterings": st["scatterings"],
           "scatterings_per_s": st["scatterings"] / wall,
           "crossings_per_s": (st["crossings"] + st["peel_crossings"]) / wall,
           "device_ms": {"transport": st["kernel_ms"], "ray_cast_pass": st["peel_pass_ms"]},
           "launches": len(hist),
           "tail": {"seconds_to_90pct_ended": t90, "seconds_after": wall - t90,
                    "scatterings_after": scat_tail,
                    "gathered": 1 if compact is None else compact,
                    "seconds_to_99pct_ended": t_end[0.99], "seconds_to_99.9pct_ended": t_end[0.999],
                    "longest_walk_scatterings": int(out["n_scat"].max()),
                    "note": "the last 10% of the packets are the longest walks; they run on a "
                            "shrinking number of lanes (gathered: into the waves they fill, "
                            "RMC_OPT_COMPACT)"},
           "escaped": st["escaped"], "absorbed": st["absorbed"], "stuck": st["stuck"]}
    return rec, out


def fp32_against_oracle(g, o, pb):
    """Each output of the complete FP32 run against the oracle's packets
    (a prefix of the same packet list, FP64): the value on each side, the
    relative difference and its z from the two sides' Monte Carlo errors
    (the oracle's, from 8 equal slices of its sample, dominates)."""
    import numpy as np
    from scipy import stats
    n_o = len(o["status"])
    k = len(o["cube_slices"])
    edges = np.linspace(0, n_o, k + 1).astype(int)
    sl = [np.arange(lo, hi) for lo, hi in zip(edges[:-1], edges[1:])]
    res = {"oracle_packets": n_o, "gpu_packets": len(g["status"])}

    def entry(vg, vo_slices, vg_se=0.0):
        vo_slices = np.asarray(vo_slices, dtype=float)
        vo = vo_slices.mean()
        se = np.sqrt(vo_slices.var(ddof=1) / k + vg_se ** 2)
        return {"fp32": float(vg), "oracle": float(vo), "rel_diff": float(vg / vo - 1) if vo else None,
                "z": float((vg - vo) / se) if se > 0 else None}

    eg = g["status"] == 1
    res["escape_fraction"] = entry(eg.mean(), [(o["status"][i] == 1).mean() for i in sl],
                                   np.sqrt(eg.mean() * (1 - eg.mean()) / len(eg)))
    res["absorbed_fraction"] = entry((g["status"] == 2).mean(), [(o["status"][i] == 2).mean() for i in sl])
    res["mean_line_scatterings"] = entry(g["n_scat"].mean(), [o["n_scat"][i].mean() for i in sl],
                                         g["n_scat"].std() / np.sqrt(len(eg)))
    xg, xo = g["x"][eg], o["x"][o["status"] == 1]
    if len(xo) >= 20:
        res["escaped_x_ks_p"] = float(stats.ks_2samp(xg, xo).pvalue)
        res["escaped_x_mean"] = entry(xg.mean(), [o["x"][i][o["status"][i] == 1].mean() for i in sl])
        res["escaped_abs_x_mean"] = entry(np.abs(xg).mean(),
                                          [np.abs(o["x"][i][o["status"][i] == 1]).mean() for i in sl])
    # the peel-off cube per emitted packet: total, spectrum and image
    # moments, against the oracle's per-slice cubes
    res["cube"] = cube_moments(g["cube"] / len(g["status"]), o, pb)
    return res


def oracle_slices(O, pb, n, cores, k):
    """The oracle on packets [0, n) in k consecutive slices (peel-off rays
    stopped where exp(-tau) = 0): packet records, per-slice cubes per
    packet, summed stats and the transport time (each call's set-up, the
    leaf hash map, measured with a one-event call and subtracted)."""
    import numpy as np
    t0 = time.perf_counter()
    O.run(pb, pb.seed, first=0, n=1, threads=1, max_events=1, with_cubes=False)
    t_set = time.perf_counter() - t0
    edges = np.linspace(0, n, k + 1).astype(int)
    recs, cubes, stats, secs = [], [], {}, 0.0
    for lo, hi in zip(edges[:-1], edges[1:]):
        t0 = time.perf_counter()
        r = O.run(pb, pb.seed, first=int(lo), n=int(hi - lo), threads=cores, peel_tau_cut=746.0)
        secs += max(time.perf_counter() - t0 - t_set, 1e-9)
        recs.append(r)
        cubes.append(r["cubes"][0] / (hi - lo))
        for key, v in r["stats"].items():
            stats[key] = stats.get(key, 0) + v
    out = {key: np.concatenate([r[key] for r in recs]) for key in ("status", "x", "n_scat")}
    out.update(cube_slices=cubes, stats=stats, seconds=secs)
    return out


def cube_moments(cg, o, pb):
    """Per-packet cube totals and the mean |x| and mean projected radius of
    the peel-off flux, GPU (complete run) against the oracle slices."""
    import numpy as np
    ob = pb.observers[0]
    xs = ob.x_min + (np.arange(ob.nbins) + 0.5) * (ob.x_max - ob.x_min) / ob.nbins
    yy, xx = np.mgrid[0:ob.ny, 0:ob.nx]
    r = np.hypot((xx + 0.5) / ob.nx - 0.5, (yy + 0.5) / ob.ny - 0.5)

    def mom(c):
        t = c.sum()
        return t, (c.sum(axis=(0, 1)) * np.abs(xs)).sum() / t, (c.sum(axis=2) * r).sum() / t

    g = mom(cg)
    vals = np.array([mom(oc) for oc in o["cube_slices"]])
    out = {}
    for j, name in enumerate(("total_per_packet", "mean_abs_x", "mean_projected_radius")):
        v = vals[:, j]
        se = np.sqrt(v.var(ddof=1) / len(v))
        out[name] = {"fp32": float(g[j]), "oracle": float(v.mean()), "rel_diff": float(g[j] / v.mean() - 1),
                     "z": float((g[j] - v.mean()) / se) if se > 0 else None}
    return out


def matched_spectra(early, launches):
    """FP32 against FP64 on the packets each finished within the same loop
    iterations per lane: escape fraction (two-proportion z), mean line
    scatterings (z of the difference) and the escaped x_ext distributions
    (two-sample KS)."""
    import numpy as np
    from scipy import stats
    out = {"sample": f"packets finished within {launches * MATCH_SLICE} loop iterations per lane "
                     f"({launches} launches of {MATCH_SLICE}, untimed) in each precision"}
    f, d = early["fp32"], early["fp64"]
    n_f, n_d = len(f["status"]), len(d["status"])
    out["finished"] = {"fp32": n_f, "fp64": n_d}
    out["slices_cut"] = {"fp32": f["slices_cut"], "fp64": d["slices_cut"]}
    if n_f < 20 or n_d < 20:
        return out
    e_f, e_d = f["status"] == 1, d["status"] == 1
    p_f, p_d = e_f.mean(), e_d.mean()
    p = (e_f.sum() + e_d.sum()) / (n_f + n_d)
    se = np.sqrt(max(p * (1 - p), 1e-300) * (1 / n_f + 1 / n_d))
    out["escape_fraction"] = {"fp32": float(p_f), "fp64": float(p_d), "z": float((p_f - p_d) / se)}
    m_f, m_d = f["n_scat"].mean(), d["n_scat"].mean()
    se = np.sqrt(f["n_scat"].var() / n_f + d["n_scat"].var() / n_d)
    out["mean_line_scatterings"] = {"fp32": float(m_f), "fp64": float(m_d), "z": float((m_f - m_d) / max(se, 1e-300))}
    if e_f.sum() >= 20 and e_d.sum() >= 20:
        out["escaped_x_ks_p"] = float(stats.ks_2samp(f["x"][e_f], d["x"][e_d]).pvalue)
    return out


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {a.gpus} is not supported "
              "(packets shard by range across GPUs with one sum-reduction of the cubes; not built here)",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from paper_2001_11252_amd import rmc, workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if a.workload != "dusty_sphere":
        fn = {"shell": bench_shell, "batch": bench_batch, "adjoint": bench_adjoint,
              "core_skip": bench_core_skip, "voigt_accuracy": bench_voigt_accuracy,
              "upar_cost": bench_upar_cost, "c1_slab": bench_c1_slab,
              "multi_species": bench_multi_species, "mesh_overhead": bench_mesh_overhead}[a.workload]
        print(json.dumps(fn(a, rmc, W)), flush=True)
        return
    steps, warm, P = a.steps, a.warmup, a.packets
    pb = W.c2_dusty_sphere(rmc.sigma0, n_packets=P, tau0=a.tau0)
    print(f"# workload: {pb.mesh.n} leaves, n_HI={pb.meta['n_hi']:.4e}, {P} packets queued, "
          f"{a.slice} iterations/lane/step", file=sys.stderr, flush=True)

    setup = {}
    early = {}

    def measure(prec, nsteps):
        t0 = time.perf_counter()
        ctx = rmc.Context.from_problem(pb, prec)
        torch.cuda.synchronize()
        setup[prec] = time.perf_counter() - t0
        ctx.set_stream(torch.cuda.current_stream())
        ctx.set_option(rmc.OPT_SLICE_ITERS, a.slice)
        if a.regroup is not None:
            ctx.set_option(rmc.OPT_REGROUP, a.regroup)
        # a first stream, abandoned after two launches, lets the peel-off
        # queue grow to its working size (it grows after a launch in which
        # a wave ended its slice early for room) before the measured stream
        ctx.stream_begin(pb.seed, 0, P)
        for _ in range(2):
            ctx.stream_step()
        ctx.stream_begin(pb.seed, 0, P)
        for _ in range(warm):
            ctx.stream_step()
        torch.cuda.synchronize()
        tot = {}
        kms = []
        t0 = time.perf_counter()
        for _ in range(nsteps):
            st, rem = ctx.stream_step()
            kms.append(st["kernel_ms"])
            for k, v in st.items():
                tot[k] = tot.get(k, 0) + v
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        print(f"# {prec}: {nsteps} steps in {wall:.3f} s, transport ms {[round(k, 1) for k in kms]}, "
              f"remaining {rem}, stats {tot}", file=sys.stderr, flush=True)
        if a.match_launches:
            # sample for the FP32/FP64 comparison (untimed): the packets
            # finished within the same number of loop iterations per lane in
            # either precision, so both samples are selected alike (short
            # walks first); launches short enough that no wave runs out of
            # queue room, which would end its slice early
            ctx.set_option(rmc.OPT_SLICE_ITERS, MATCH_SLICE)
            # the same loop in both precisions, so that equal iterations
            # select the packets alike
            ctx.set_option(rmc.OPT_REGROUP, 0)
            ctx.stream_begin(pb.seed, 0, P)
            cut = 0
            for _ in range(a.match_launches):
                cut += ctx.stream_step()[0]["slices_cut"]
            pk = ctx.get_packets()
            fin = pk["status"] > 0
            early[prec] = {"status": pk["status"][fin], "x": pk["x"][fin], "n_scat": pk["n_scat"][fin],
                           "slices_cut": cut}
        ctx.close()
        return wall, tot, kms

    copy_GBps = measure_copy(a)

    res = {}
    full = full_out = None
    if a.only in ("fp32", "both"):
        res["fp32"] = measure("fp32", steps)
        if a.complete_run:
            full, full_out = complete_run(pb, P, rmc, torch, a.regroup, a.compact)
    if a.only in ("fp64", "both"):
        res["fp64"] = measure("fp64", a.fp64_steps if a.only == "both" else steps)
    head = "fp32" if "fp32" in res else "fp64"
    wall, tot, kms = res[head]
    nsteps = len(kms)
    scat_s = tot["scatterings"] / wall
    cross = tot["crossings"] + tot["peel_crossings"]
    cross_s = cross / wall
    # roofline of the dominant kernel (the transport launch): its
    # algorithmic work per launch (every scattering, every transport
    # segment, and the first leaf of every peel-off ray) over its average
    # device duration; the rest of the peel-off rays is the ray-cast pass
    avg_ms = sum(kms) / nsteps
    traffic = measured_traffic(head)
    # the step against the HBM roof, one definition: algorithmic bytes = a
    # leaf record and a node entry per ray-cell crossing, transport and
    # peel-off alike (28 B float, 52 B double); events inside a leaf use the
    # record the lane holds (0 B); over the step's wall time.  Beside it,
    # when the profiler's counters match these sources, the bytes the
    # transport launch moved over its own duration.
    alg_bytes = cross * BYTES_PER_CROSSING[head] / nsteps
    hbm = {"peak_GBps": 8000.0,
           "definition": "ray-cell crossings (transport + peel-off) x (leaf record + node entry) per step "
                         "wall time; scatterings use the register-held record",
           "algorithmic_bytes_per_step": alg_bytes,
           "algorithmic_GBps": alg_bytes / (wall / nsteps) / 1e9,
           "transport_launch_measured_GBps": None if traffic is None else traffic / (avg_ms * 1e-3) / 1e9}
    hbm["frac_algorithmic"] = hbm["algorithmic_GBps"] / 8000.0
    hbm["frac_measured"] = None if traffic is None else hbm["transport_launch_measured_GBps"] / 8000.0
    transport_cross = tot["crossings"] + tot["peel_rays"]
    flops_per_launch = (FLOP_PER_SCATTERING * tot["scatterings"] + FLOP_PER_CROSSING * transport_cross) / nsteps
    achieved = flops_per_launch / (avg_ms * 1e-3) / 1e12
    side = {}
    for prec, (w, t, k) in res.items():
        pass_cross = t["peel_crossings"] - t["peel_rays"]
        side[prec] = {"scatterings_per_s": t["scatterings"] / w,
                      "crossings_per_s": (t["crossings"] + t["peel_crossings"]) / w,
                      "ms_per_step": 1e3 * w / len(k),
                      "transport_ms_avg": sum(k) / len(k),
                      "peel_pass_ms_avg": t["peel_pass_ms"] / len(k),
                      "peel_rays_deferred_per_step": t["peel_deferred"] / len(k),
                      "slices_cut": t["slices_cut"],
                      "peel_pass_crossings_per_s": pass_cross / max(t["peel_pass_ms"] * 1e-3, 1e-30),
                      "hbm_GBps_algorithmic": (t["crossings"] + t["peel_crossings"]) * BYTES_PER_CROSSING[prec]
                      / w / 1e9,
                      "packets_finished": t["emitted"]}
    line = {
        "metric": "scatterings/s + ray-cell crossings/s (1 GPU), FP32 vs FP64 at matched spectra",
        "value": scat_s,
        "unit": "scatterings/s",
        "crossings_per_s": cross_s,
        "n_gpus": 1,
        "steps": nsteps,
        "warmup": warm,
        "ms_per_step": 1e3 * wall / nsteps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if head == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": "dusty_sphere_tau1e6_T1e4_287k_leaves_peel_128x128x100",
                   "tau0": a.tau0, "packets_queued": P, "iterations_per_lane_per_step": a.slice,
                   "leaves": int(pb.mesh.n), "observer": "+z 128x128x100", "parallelism": "none",
                   "regroup": a.regroup},
        "precisions": side,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK[head], "unit": "TFLOP/s",
                     "frac": achieved / PEAK[head], "traffic": traffic,
                     "kernel": "k_transport<float,false,true,1>" if head == "fp32" else "k_transport<double,false,true,1>"},
        "hbm": hbm,
        "hbm_copy_GBps": copy_GBps,
        # context set-up outside the timed region: octree build and
        # validation, leaf records, uploads (seconds)
        "setup_s": setup,
    }
    if len(early) == 2:
        line["matched_spectra"] = matched_spectra(early, a.match_launches)
    if full is not None:
        line["complete_run"] = full
    if not a.no_cpu_baseline:
        from oracle import oracle as O
        cores, host = host_cores()
        # the oracle as it stands: every peel-off ray walked to the border
        n_cpu = a.cpu_packets or 6 * cores
        t0 = time.perf_counter()
        r = O.run(pb, pb.seed, first=0, n=n_cpu, threads=cores)
        dt = time.perf_counter() - t0
        st = r["stats"]
        # like for like: peel-off rays stopped where exp(-tau) is exactly 0,
        # as the GPU stops them (the same deposits); its packets are also
        # the oracle sample the FP32 outputs are compared with
        n_cut = a.cpu_packets_cut or 64 * cores
        rc = oracle_slices(O, pb, n_cut, cores, 8)
        dc, sc = rc["seconds"], rc["stats"]
        line["cpu_baseline"] = {
            "value": st["scatterings"] / dt, "unit": "scatterings/s", "cores": cores, "kind": "oracle",
            "sample": f"{n_cpu} packets of the same workload (FP64 oracle, every peel-off ray walked to the "
                      f"border), {st['scatterings']} scatterings in {dt:.1f} s",
            "crossings_per_s": (st["crossings"] + st["peel_crossings"]) / dt,
            "like_for_like": {"scatterings_per_s": sc["scatterings"] / dc,
                              "crossings_per_s": (sc["crossings"] + sc["peel_crossings"]) / dc,
                              "sample": f"{n_cut} packets, peel-off rays stopped once tau >= 746 "
                                        f"(exp(-tau) = 0 in double, deposits unchanged), "
                                        f"{sc['scatterings']} scatterings in {dc:.1f} s"},
            "host": host}
        if full_out is not None:
            line["fp32_vs_oracle"] = fp32_against_oracle(full_out, rc, pb)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
