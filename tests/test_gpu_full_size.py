"""The benchmark's configurations at full size, in its launch configuration.

Dusty sphere (287,064 leaves, tau0 = 1e6, T = 1e4 K, tau_dust = 1, 1e6
packets queued, +z observer with a 128x128x100 cube; streaming launches of
8192 loop iterations per lane, deferred peel-off):

* packets the double path finishes follow the oracle packet by packet: a
  sample of them is recomputed one by one on the CPU (same counter-based
  draws, so status, scattering count, frequency, position and direction
  agree);
* the float path's finished packets match the double path's in distribution,
  on samples selected alike (the packets each finishes within the same loop
  iterations per lane).

Outflowing shell (2,360,576 leaves, V_max = 200 km/s, 1e7 packets queued,
three 256x256x200 cubes) and the batch of 64 uneven problems (launch shape
from the autotuner): packets the double path finishes follow the oracle
packet by packet, as for the sphere (in the batch's lognormal gas, on
status, scattering count and frequency; see the test)."""
import numpy as np
import pytest
from scipy import stats

from paper_2001_11252_amd import workloads as W

pytestmark = pytest.mark.gpu

N_PACKETS = 1_000_000


@pytest.fixture(scope="module")
def sphere(orc):
    s0 = lambda ln, T: orc.line_quantities(ln, T)["sigma0"]
    return W.c2_dusty_sphere(s0, n_packets=N_PACKETS, tau0=1e6)


def test_fp64_packets_follow_the_oracle_at_full_size(orc, sphere):
    from paper_2001_11252_amd import rmc
    pb = sphere
    c = rmc.Context.from_problem(pb, "fp64")
    c.set_option(rmc.OPT_SLICE_ITERS, 8192)
    c.stream_begin(pb.seed, 0, N_PACKETS)
    for _ in range(3):
        c.stream_step()
    out = c.get_packets()
    c.close()
    fin = np.flatnonzero(out["status"] > 0)
    assert len(fin) > 1000
    # the 8 shortest walks, the 4 longest and 12 others at random
    pick = _sample(out, 8, 12, 4, 2_000_000, np.random.default_rng(11))
    assert out["n_scat"][pick].max() > 1000
    # the draws are the same; a last-ulp difference of a library function
    # flips a decision of a long walk only rarely
    same = _compare_with_oracle(orc, pb, pb.seed, out, pick)
    assert same >= len(pick) - 2, (same, len(pick))


def test_fp32_matches_fp64_at_full_size(orc, sphere):
    from paper_2001_11252_amd import rmc
    pb = sphere
    fin = {}
    for prec in ("fp32", "fp64"):
        c = rmc.Context.from_problem(pb, prec)
        c.set_option(rmc.OPT_SLICE_ITERS, 1024)
        # the same loop in both precisions (a pending rejection round takes
        # a loop iteration with RMC_OPT_REGROUP, which would select other
        # packets into the sample below)
        c.set_option(rmc.OPT_REGROUP, 0)
        # a first stream, abandoned after two launches, grows the peel-off
        # queue to its working size (the first launch of a fresh context can
        # end slices early for room)
        c.stream_begin(pb.seed, 0, N_PACKETS)
        for _ in range(2):
            c.stream_step()
        c.stream_begin(pb.seed, 0, N_PACKETS)
        cut = 0
        for _ in range(32):
            cut += c.stream_step()[0]["slices_cut"]
        out = c.get_packets()
        c.close()
        # no wave ended a launch early, so every lane ran 32768 iterations
        assert cut == 0
        f = out["status"] > 0
        fin[prec] = {k: out[k][f] for k in ("status", "x", "n_scat")}
    a, b = fin["fp32"], fin["fp64"]
    assert len(b["status"]) > 5000
    ea, eb = a["status"] == 1, b["status"] == 1
    p = (ea.sum() + eb.sum()) / (len(ea) + len(eb))
    z = (ea.mean() - eb.mean()) / np.sqrt(p * (1 - p) * (1 / len(ea) + 1 / len(eb)))
    assert abs(z) < 4.0, z
    zs = (a["n_scat"].mean() - b["n_scat"].mean()) / np.sqrt(a["n_scat"].var() / len(ea) + b["n_scat"].var() / len(eb))
    assert abs(zs) < 4.0, zs
    assert stats.ks_2samp(a["x"][ea], b["x"][eb]).pvalue > 1e-3


def _compare_with_oracle(orc, pb, seed, out, pick):
    """Packets of `pick` recomputed one by one by the oracle: how many end
    identically — same status and scattering count, frequency within 1e-9,
    position and direction within the last-ulp differences of the two
    sides' library functions accumulated along the walk.  (Such a
    difference can also send a long walk through a neighbouring cell at a
    corner, after which it differs; the callers allow a couple of those.)"""
    same = 0
    for pid in pick:
        ref = orc.run(pb, seed, first=int(pid), n=1, threads=1, with_cubes=False)
        tol = 1e-13 + 1e-15 * float(out["n_scat"][pid])
        same += int(ref["status"][0] == out["status"][pid] and ref["n_scat"][0] == out["n_scat"][pid]
                    and abs(ref["x"][0] - out["x"][pid]) < 1e-9
                    and np.abs(ref["pos"][0] - out["pos"][pid]).max() < tol
                    and np.abs(ref["k"][0] - out["k"][pid]).max() < tol)
    return same


def _sample(out, n_short, n_random, n_long, max_scat, rng):
    """Finished packets: the n_short shortest walks, the n_long longest
    below max_scat scatterings, and n_random others at random."""
    fin = np.flatnonzero(out["status"] > 0)
    order = fin[np.argsort(out["n_scat"][fin], kind="stable")]
    short = order[:n_short]
    below = order[out["n_scat"][order] < max_scat]
    long_ = np.setdiff1d(below[len(below) - n_long:] if n_long else below[:0], short)
    pool = np.setdiff1d(below, np.concatenate([short, long_]))
    extra = rng.choice(pool, min(n_random, len(pool)), replace=False) if len(pool) else pool
    return np.concatenate([short, long_, extra]).astype(np.int64)


def test_fp64_shell_packets_follow_the_oracle_at_full_size(orc):
    from paper_2001_11252_amd import rmc
    s0 = lambda ln, T: orc.line_quantities(ln, T)["sigma0"]
    n = 10_000_000
    pb = W.c3_shell(s0, vmax_kms=200.0, n_packets=n)
    c = rmc.Context.from_problem(pb, "fp64")
    c.set_option(rmc.OPT_SLICE_ITERS, 8192)
    c.stream_begin(pb.seed, 0, n)
    for _ in range(2):
        c.stream_step()
    out = c.get_packets()
    c.close()
    assert np.count_nonzero(out["status"] > 0) > 1000
    pick = _sample(out, 4, 6, 6, 1_000_000, np.random.default_rng(12))
    assert out["n_scat"][pick].max() > 1000
    same = _compare_with_oracle(orc, pb, pb.seed, out, pick)
    assert same >= len(pick) - 2, (same, len(pick))


def test_fp64_batch_packets_follow_the_oracle_at_full_size(orc):
    from paper_2001_11252_amd import rmc
    s0 = lambda ln, T: orc.line_quantities(ln, T)["sigma0"]
    probs = W.c4_batch(s0)
    ctxs = [rmc.Context.from_problem(p, "fp64") for p in probs]
    seeds = [p.seed for p in probs]
    npk = [len(p.sources.x) for p in probs]
    rmc.batch_autotune(ctxs, seeds, npk)
    # a prefix of each problem's packets, so that every problem has packets
    # in flight in the first launches (a packet's result depends only on its
    # problem and index, not on what else the batch holds)
    rmc.batch_begin(ctxs, seeds, [min(k, 2000) for k in npk])
    for _ in range(2):
        ctxs[0].stream_step()
    # up to 12 problems with finished packets, 2 packets each: the shortest
    # walk and one drawn among those under 3000 scatterings.  The batch's
    # gas is lognormal (neighbouring cells differ in opacity by factors of
    # several), so a last-ulp difference in where a packet crosses a face
    # moves its next event by that factor: the two sides' differences grow
    # along a walk until long walks part (they stay alike in distribution,
    # which the batch tests check); short walks still agree one by one.
    rng = np.random.default_rng(13)
    outs = [c.get_packets() for c in ctxs]
    done = [i for i in range(len(probs)) if np.count_nonzero(outs[i]["status"] > 0) > 0]
    # (The same growth separates positions first, so these walks are
    # compared on status, scattering count and final frequency.)
    checked = same = 0
    for i in rng.choice(done, min(12, len(done)), replace=False):
        out = outs[i]
        for pid in _sample(out, 1, 1, 0, 3000, rng):
            ref = orc.run(probs[i], seeds[i], first=int(pid), n=1, threads=1, with_cubes=False)
            checked += 1
            same += int(ref["status"][0] == out["status"][pid] and ref["n_scat"][0] == out["n_scat"][pid]
                        and abs(ref["x"][0] - out["x"][pid]) < 1e-6)
    for c in ctxs:
        c.close()
    assert checked >= 8, (checked, done)
    assert same >= checked - 2, (same, checked)

