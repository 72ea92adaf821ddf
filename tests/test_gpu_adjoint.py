"""GPU peel-off image of fixed rays and its adjoint (d image / d n_HI,
kappa_d, v_los per leaf): against the oracle's exact forward and gradient,
against central finite differences of the GPU forward, and through the
torch.autograd.Function wrapper.  Galaxy-like field (lognormal n_HI with a
k^-3 spectrum, dust proportional to n_HI, turbulent velocities) on a small
adaptive mesh."""
import numpy as np
import pytest

from paper_2001_11252_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def galaxy(orc):
    s0 = lambda ln, T: orc.line_quantities(ln, T)["sigma0"]
    pb = W.c5_galaxy(s0, grid=32, min_level=3, max_level=7, target_leaves=4e4, n_sources=400,
                     rays_per_source=25, nx=32, tau_mean=30.0, tau_dust=0.3)
    return pb


def _rays(pb):
    r = pb.meta["rays"]
    return r["orig"], r["x_ext"], r["w"], pb.meta["grad_image"]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_image_and_gradient_match_oracle(orc, galaxy, prec):
    from paper_2001_11252_amd import rmc
    pb = galaxy
    orig, x, w, G = _rays(pb)
    ob = pb.observers[0]
    img_o, gn_o, gk_o, gv_o = orc.raycast_image(pb, ob, orig, x, w, G)
    ctx = rmc.Context.from_problem(pb, prec, sources=False)
    img = ctx.raycast_image(0, orig, x, w)
    gn, gk, gv = ctx.raycast_image_backward(0, orig, x, w, G)
    assert img_o.sum() > 0 and np.count_nonzero(gn_o) > 100
    nb, mb = ctx.image_stats()
    img = ctx.raycast_image(0, orig, x, w)
    nf, mf = ctx.image_stats()
    assert nf > len(x) and nb >= nf and mf > 0 and mb > 0
    if prec == "fp64":
        assert np.allclose(img, img_o, rtol=1e-12, atol=1e-300)
        for a, b in ((gn, gn_o), (gk, gk_o), (gv, gv_o)):
            assert np.abs(a - b).max() <= 1e-10 * np.abs(b).max()
    else:
        # float leaf records and opacities: per-ray weight error ~1e-5 max(1, tau)
        tau = orc.tau(pb, orig, np.tile(ob.k, (len(x), 1)), x)
        bound = np.zeros_like(img_o)
        e1 = np.array([1.0, 0.0, 0.0])
        e2 = np.array([0.0, 1.0, 0.0])
        ix = np.floor(((orig - 0.5) @ e1 + 0.5) * 32).astype(int)
        iy = np.floor(((orig - 0.5) @ e2 + 0.5) * 32).astype(int)
        ok = (ix >= 0) & (ix < 32) & (iy >= 0) & (iy < 32)
        np.add.at(bound, (iy[ok], ix[ok]), 1e-5 * (w * np.exp(-tau) * np.maximum(1.0, tau))[ok])
        assert np.all(np.abs(img - img_o) <= bound + 1e-300)
        for a, b in ((gn, gn_o), (gk, gk_o), (gv, gv_o)):
            assert np.abs(a - b).max() <= 1e-4 * np.abs(b).max()


def test_gradient_matches_central_differences(orc, galaxy):
    from paper_2001_11252_amd import rmc
    pb = galaxy
    orig, x, w, G = _rays(pb)
    ctx = rmc.Context.from_problem(pb, "fp64", sources=False)
    gn, gk, gv = ctx.raycast_image_backward(0, orig, x, w, G)
    g = pb.gas

    def L():
        ctx.set_gas(g.n_hi, g.T, g.v, g.kappa_d)
        return (ctx.raycast_image(0, orig, x, w) * G).sum()

    L0 = L()
    for c in np.argsort(-np.abs(gn))[:5]:
        for arr, grad in ((g.n_hi, gn), (g.kappa_d, gk)):
            old = arr[c]
            h = 1e-4 * old
            arr[c] = old + h
            Lp = L()
            arr[c] = old - h
            Lm = L()
            arr[c] = old
            fd = (Lp - Lm) / (2 * h)
            assert abs(fd - grad[c]) <= 1e-5 * abs(grad[c]) + 1e-12 * abs(L0) / h, (c, fd, grad[c])
    for c in np.argsort(-np.abs(gv))[:5]:
        old = g.v[c, 2]
        h = 1e3     # 10 m/s along the line of sight (+z)
        g.v[c, 2] = old + h
        Lp = L()
        g.v[c, 2] = old - h
        Lm = L()
        g.v[c, 2] = old
        fd = (Lp - Lm) / (2 * h)
        assert abs(fd - gv[c]) <= 1e-4 * abs(gv[c]) + 1e-10 * abs(L0) / h, (c, fd, gv[c])
    ctx.set_gas(g.n_hi, g.T, g.v, g.kappa_d)


def test_autograd_function(orc, galaxy):
    import torch
    from paper_2001_11252_amd import rmc
    pb = galaxy
    orig, x, w, G = _rays(pb)
    dev = torch.device("cuda:0")
    ctx = rmc.Context.from_problem(pb, "fp64", sources=False)
    fn = rmc.raycast_image_fn()
    n_hi = torch.tensor(pb.gas.n_hi, dtype=torch.float64, device=dev, requires_grad=True)
    kd = torch.tensor(pb.gas.kappa_d, dtype=torch.float64, device=dev, requires_grad=True)
    v = torch.tensor(pb.gas.v, dtype=torch.float64, device=dev, requires_grad=True)
    o_t = torch.tensor(orig, dtype=torch.float64, device=dev)
    x_t = torch.tensor(x, dtype=torch.float64, device=dev)
    w_t = torch.tensor(w, dtype=torch.float64, device=dev)
    G_t = torch.tensor(G, dtype=torch.float64, device=dev)
    img = fn.apply(n_hi, kd, v, ctx, pb.gas.T, 0, o_t, x_t, w_t)
    loss = (img * G_t).sum()
    loss.backward()
    gn, gk, gv = ctx.raycast_image_backward(0, orig, x, w, G)
    img_np = ctx.raycast_image(0, orig, x, w)
    assert np.allclose(img.detach().cpu().numpy(), img_np, rtol=1e-14, atol=0)
    assert np.allclose(n_hi.grad.cpu().numpy(), gn, rtol=1e-12, atol=1e-300)
    assert np.allclose(kd.grad.cpu().numpy(), gk, rtol=1e-12, atol=1e-300)
    gvz = v.grad.cpu().numpy()
    assert np.allclose(gvz[:, 2], gv, rtol=1e-12, atol=1e-300)
    assert np.all(gvz[:, :2] == 0.0)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_tape_matches_replay(orc, galaxy, prec):
    # the backward read from the forward's crossing lists gives the
    # replaying backward's gradients (summation order aside; the float
    # path keeps its segments as float)
    from paper_2001_11252_amd import rmc
    pb = galaxy
    orig, x, w, G = _rays(pb)
    ctx = rmc.Context.from_problem(pb, prec, sources=False)
    with pytest.raises(rmc.RmcError, match="no tape"):
        ctx.raycast_image_backward_tape(G)
    img = ctx.raycast_image(0, orig, x, w)
    nf, _ = ctx.image_stats()
    ref = ctx.raycast_image_backward(0, orig, x, w, G)
    img_t = ctx.raycast_image_tape(0, orig, x, w)
    nf_t, _ = ctx.image_stats()
    got = ctx.raycast_image_backward_tape(G)
    nb_t, mb_t = ctx.image_stats()
    assert nf_t == nf and 0 < nb_t <= nf_t and mb_t > 0
    assert np.allclose(img_t, img, rtol=1e-13, atol=0)
    tol = 1e-10 if prec == "fp64" else 1e-5
    for a, b in zip(got, ref):
        assert np.count_nonzero(b) > 100
        assert np.abs(a - b).max() <= tol * np.abs(b).max()
    # the tape is kept for further backward calls of the same model
    again = ctx.raycast_image_backward_tape(2.0 * G)
    for a, b in zip(again, got):
        assert np.abs(a - 2.0 * b).max() <= 1e-12 * np.abs(b).max()
    # and dropped when the model changes
    ctx.set_gas(pb.gas.n_hi, pb.gas.T, pb.gas.v, pb.gas.kappa_d)
    with pytest.raises(rmc.RmcError, match="no tape"):
        ctx.raycast_image_backward_tape(G)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_tape_grows_for_long_rays(orc, prec):
    # diagonal rays through a periodic slab of 64^3 leaves cross ~190 leaves,
    # more than the tape's first guess (128 per ray): the forward pass asks
    # for more chunks and runs again; the results still match the replay
    from paper_2001_11252_amd import rmc
    s0 = lambda ln, T: orc.line_quantities(ln, T)["sigma0"]
    pb = W.static_slab(s0, 20.0, 1e4, 1, level=6)
    k = np.ones(3) / np.sqrt(3.0)
    pb.observers = [W.Observer(tuple(k), 16, 16, 1, (-0.8, 0.8, -0.8, 0.8), -50.0, 50.0)]
    rng = np.random.default_rng(3)
    n = 3000
    orig = np.column_stack([rng.uniform(0.2, 0.8, n), rng.uniform(0.2, 0.8, n), np.full(n, 1e-3)])
    x = rng.uniform(-4.0, 4.0, n)
    w = np.full(n, 1.0 / (4.0 * np.pi))
    G = rng.standard_normal((16, 16))
    ctx = rmc.Context.from_problem(pb, prec, sources=False)
    img = ctx.raycast_image(0, orig, x, w)
    nf, _ = ctx.image_stats()
    assert nf > 150 * n
    ref = ctx.raycast_image_backward(0, orig, x, w, G)
    img_t = ctx.raycast_image_tape(0, orig, x, w)
    assert ctx.image_stats()[0] == nf
    got = ctx.raycast_image_backward_tape(G)
    assert np.allclose(img_t, img, rtol=1e-13, atol=0)
    tol = 1e-10 if prec == "fp64" else 1e-5
    for a, b in zip(got, ref):
        assert np.abs(a - b).max() <= tol * np.abs(b).max()


def test_destroy_releases_the_tape(orc, galaxy):
    # a context's crossing lists (here ~150 MB: the rays ten times over) go
    # back to the device when the context is destroyed
    import torch
    from paper_2001_11252_amd import rmc
    pb = galaxy
    orig, x, w, G = _rays(pb)
    orig, x, w = np.tile(orig, (10, 1)), np.tile(x, 10), np.tile(w, 10)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for _ in range(3):
        ctx = rmc.Context.from_problem(pb, "fp64", sources=False)
        ctx.raycast_image_tape(0, orig, x, w)
        ctx.raycast_image_backward_tape(G)
        ctx.close()
    torch.cuda.synchronize()
    assert free0 - torch.cuda.mem_get_info()[0] < (64 << 20)


def test_autograd_falls_back_to_replay(orc, galaxy):
    # a second forward call records its own tape; the backward of the first
    # then sets the first call's gas again and replays its rays
    import torch
    from paper_2001_11252_amd import rmc
    pb = galaxy
    orig, x, w, G = _rays(pb)
    dev = torch.device("cuda:0")
    ctx = rmc.Context.from_problem(pb, "fp64", sources=False)
    fn = rmc.raycast_image_fn()
    t = lambda a, grad=False: torch.tensor(a, dtype=torch.float64, device=dev, requires_grad=grad)
    n1, k1, v1 = t(pb.gas.n_hi, True), t(pb.gas.kappa_d, True), t(pb.gas.v, True)
    n2, k2, v2 = t(1.3 * pb.gas.n_hi, True), t(pb.gas.kappa_d, True), t(pb.gas.v, True)
    args = (ctx, pb.gas.T, 0, t(orig), t(x), t(w))
    img1 = fn.apply(n1, k1, v1, *args)
    img2 = fn.apply(n2, k2, v2, *args)
    assert not torch.allclose(img1, img2)
    (img1 * t(G)).sum().backward()
    ctx.set_gas(pb.gas.n_hi, pb.gas.T, pb.gas.v, pb.gas.kappa_d)
    gn, gk, gv = ctx.raycast_image_backward(0, orig, x, w, G)
    assert np.allclose(n1.grad.cpu().numpy(), gn, rtol=1e-12, atol=1e-300)
    assert np.allclose(k1.grad.cpu().numpy(), gk, rtol=1e-12, atol=1e-300)
    assert np.allclose(v1.grad.cpu().numpy()[:, 2], gv, rtol=1e-12, atol=1e-300)



def test_fp64_gradients_per_element_at_1e12(orc, galaxy):
    # every term of each gradient entry has one sign (G > 0; x_ext far
    # enough in the blue wing that the gas-frame x stays > 0, where
    # dH/dx < 0), so the per-entry sums do not cancel and the double path
    # must give the oracle's exact gradient to 1e-12 per element
    from paper_2001_11252_amd import rmc
    pb = galaxy
    orig, _, w, G = _rays(pb)
    rng = np.random.default_rng(12)
    vth = orc.line_quantities(W.LYA, 1e4)["vth"]
    umax = np.abs(pb.gas.v[:, 2]).max() / vth
    x = rng.uniform(umax + 1.0, umax + 8.0, len(w))
    Gp = np.abs(G) + 0.5
    img_o, gn_o, gk_o, gv_o = orc.raycast_image(pb, pb.observers[0], orig, x, w, Gp)
    ctx = rmc.Context.from_problem(pb, "fp64", sources=False)
    img = ctx.raycast_image(0, orig, x, w)
    nz = img_o > 0
    assert np.max(np.abs(img[nz] / img_o[nz] - 1)) <= 1e-12
    for name, got in (("replay", ctx.raycast_image_backward(0, orig, x, w, Gp)),
                      ("tape", (ctx.raycast_image_tape(0, orig, x, w), ctx.raycast_image_backward_tape(Gp))[1])):
        for a, b, what in zip(got, (gn_o, gk_o, gv_o), ("n_hi", "kappa_d", "v_los")):
            big = np.abs(b) > 1e-6 * np.abs(b).max()
            assert big.sum() > 100, (name, what)
            assert np.all(np.sign(a[big]) == np.sign(b[big]))
            rel = np.abs(a[big] / b[big] - 1)
            assert rel.max() <= 1e-12, (name, what, rel.max())


def test_central_differences_on_100_random_crossed_cells(orc, galaxy):
    # d L / d theta_c of the replaying backward against central differences
    # (FP64 forward) at 100 random leaves that rays cross, for n_HI, kappa_d
    # (relative step 1e-4) and v_los (10 m/s along the observer direction).
    # Only rays crossing leaf c depend on its gas, so each difference uses
    # those rays alone (L over the others cancels exactly).
    from paper_2001_11252_amd import rmc
    pb = galaxy
    orig, x, w, G = _rays(pb)
    g = pb.gas
    ctx = rmc.Context.from_problem(pb, "fp64", sources=False)
    gn, gk, gv = ctx.raycast_image_backward(0, orig, x, w, G)
    kz = np.tile([0.0, 0.0, 1.0], (len(x), 1))
    leaf, seg, cnt = ctx.trace_cells(orig, kz, 512)
    assert cnt.max() < 512
    valid = np.arange(512)[None, :] < cnt[:, None]
    rows = np.repeat(np.arange(len(x)), cnt)
    cells = leaf[valid]
    assert cells.min() >= 0 and len(cells) == len(rows)
    crossed = np.unique(cells)
    cand = crossed[(gn[crossed] != 0) & (gk[crossed] != 0)]
    rng = np.random.default_rng(100)
    pick = rng.choice(cand, size=100, replace=False)
    vth = orc.line_quantities(W.LYA, 1e4)["vth"]
    b = vth / 2.99792458e10
    kink = np.sqrt(0.855)

    def loss(sel):
        ctx.set_gas(g.n_hi, g.T, g.v, g.kappa_d)
        img = ctx.raycast_image(0, orig[sel], x[sel], w[sel])
        return (img * G).sum(), (np.abs(img) * np.abs(G)).sum()

    checked_v = 0
    for c in pick:
        sel = np.unique(rows[cells == c])
        L0, Labs = loss(sel)
        for arr, grad in ((g.n_hi, gn), (g.kappa_d, gk)):
            old = arr[c]
            h = 1e-4 * old
            arr[c] = old + h
            Lp, _ = loss(sel)
            arr[c] = old - h
            Lm, _ = loss(sel)
            arr[c] = old
            fd = (Lp - Lm) / (2 * h)
            assert abs(fd - grad[c]) <= 1e-5 * abs(grad[c]) + 1e-14 * Labs / h, (c, fd, grad[c])
        # v_los: skip leaves where a ray's gas-frame x sits at the kink of
        # the production H (x^2 = 0.855), where H' jumps
        u = g.v[c, 2] / vth
        xc = (x[sel] - u) / (1 + b * u)
        if np.min(np.abs(np.abs(xc) - kink)) < 5e-3:
            continue
        old = g.v[c, 2]
        h = 1e3
        g.v[c, 2] = old + h
        Lp, _ = loss(sel)
        g.v[c, 2] = old - h
        Lm, _ = loss(sel)
        g.v[c, 2] = old
        fd = (Lp - Lm) / (2 * h)
        assert abs(fd - gv[c]) <= 1e-4 * abs(gv[c]) + 1e-13 * Labs / h, (c, fd, gv[c])
        checked_v += 1
    assert checked_v >= 50
    ctx.set_gas(g.n_hi, g.T, g.v, g.kappa_d)


@pytest.mark.parametrize("dt", ["float64", "float32"])
def test_device_gas_equals_host_gas(orc, galaxy, dt):
    # rmc_set_gas with device tensors (RMC_DEVICE, float or double) builds
    # the same leaf records as host arrays with the same values: identical
    # images and gradients; the library's velocity gradient is g_vlos k_obs
    import torch
    from paper_2001_11252_amd import rmc
    pb = galaxy
    orig, x, w, G = _rays(pb)
    g = pb.gas
    tdt = getattr(torch, dt)
    cast = lambda a: np.asarray(a, dtype=dt).astype(np.float64)
    h = rmc.Context.from_problem(pb, "fp64", sources=False)
    h.set_gas(cast(g.n_hi), cast(g.T), cast(g.v), cast(g.kappa_d))
    img_h = h.raycast_image(0, orig, x, w)
    gh = h.raycast_image_backward(0, orig, x, w, G, with_v=True)
    d = rmc.Context.from_problem(pb, "fp64", sources=False)
    dev = torch.device("cuda:0")
    t = lambda a: torch.tensor(np.asarray(a), dtype=tdt, device=dev)
    d.set_gas(t(g.n_hi), t(g.T), t(g.v), t(g.kappa_d))
    img_d = d.raycast_image(0, orig, x, w)
    gd = d.raycast_image_backward(0, orig, x, w, G, with_v=True)
    assert np.allclose(img_d, img_h, rtol=1e-14, atol=0)
    for a, b_ in zip(gd, gh):
        assert np.allclose(a, b_, rtol=1e-12, atol=1e-300)
    assert np.array_equal(gh[3], gh[2][:, None] * np.array([0.0, 0.0, 1.0])[None, :])
    # a non-finite device value is refused and names its leaf; the gas in
    # place is kept
    bad = t(g.n_hi)
    bad[17] = float("nan")
    with pytest.raises(rmc.RmcError, match="leaf 17"):
        d.set_gas(bad, t(g.T), t(g.v), t(g.kappa_d))
    assert np.allclose(d.raycast_image(0, orig, x, w), img_h, rtol=1e-14, atol=0)
    # wrongly typed or placed tensors never reach the library
    with pytest.raises(TypeError):
        d.set_gas(t(g.n_hi), t(g.T).to(torch.int32), t(g.v), t(g.kappa_d))
    with pytest.raises(ValueError):
        d.set_gas(t(g.n_hi), t(g.T), t(g.v).t(), t(g.kappa_d))
    with pytest.raises(ValueError):
        d.set_gas(t(g.n_hi)[:-1], t(g.T)[:-1], t(g.v)[:-1], t(g.kappa_d)[:-1])


def test_autograd_on_device_float32_fields(orc, galaxy):
    # the C5 form: float32 gas tensors on the GPU, passed in place; the
    # gradients equal the library's for the same (float-rounded) gas
    import torch
    from paper_2001_11252_amd import rmc
    pb = galaxy
    orig, x, w, G = _rays(pb)
    dev = torch.device("cuda:0")
    ctx = rmc.Context.from_problem(pb, "fp32", sources=False)
    fn = rmc.raycast_image_fn()
    f = lambda a, grad=False: torch.tensor(np.asarray(a), dtype=torch.float32, device=dev, requires_grad=grad)
    n_hi, kd, v = f(pb.gas.n_hi, True), f(pb.gas.kappa_d, True), f(pb.gas.v, True)
    d64 = lambda a: torch.tensor(a, dtype=torch.float64, device=dev)
    img = fn.apply(n_hi, kd, v, ctx, pb.gas.T, 0, d64(orig), d64(x), d64(w))
    (img * d64(G)).sum().backward()
    assert n_hi.grad.dtype == torch.float32 and v.grad.shape == v.shape
    r = lambda a: np.asarray(a, dtype=np.float32).astype(np.float64)
    ref = rmc.Context.from_problem(pb, "fp32", sources=False)
    ref.set_gas(r(pb.gas.n_hi), r(pb.gas.T), r(pb.gas.v), r(pb.gas.kappa_d))
    gn, gk, gvl, g3 = ref.raycast_image_backward(0, orig, x, w, G, with_v=True)
    for a, b_ in ((n_hi.grad, gn), (kd.grad, gk), (v.grad, g3)):
        a = a.cpu().numpy().astype(np.float64)
        assert np.abs(a - b_).max() <= 1e-5 * np.abs(b_).max()
