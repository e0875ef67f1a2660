"""GPU adjoint (sf_project_backward behind torch.autograd.Function) against autograd through
the FP64 oracle and against central finite differences."""
import numpy as np
import pytest
import torch

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def P():
    import paper_2501_19042_amd as P
    torch.cuda.set_device(0)
    return P


def problem(n=4, S=2, H=20, degree=8, seed=3, sigma=0.3, box=1.0, T=6.0):
    cfg = W.SwarmConfig(n_robots=n, dims=3, degree=degree, horizon=H, t_final=T, safety_a=0.3, safety_b=0.3,
                        vmax=1.0, amax=1.0)
    rng = np.random.default_rng(seed)
    st = W.box_starts(rng, n, (-box, -box, -0.3), (box, box, 0.3), 0.4)
    gl = st[rng.permutation(n)]
    xi = W.sample_coeffs(rng, st, gl, degree, S, sigma)
    return cfg, xi, W.boundary_values(st, gl), rng


def loss_fn(xi_k, xi_bar, res):
    return ((xi_k - xi_bar) ** 2).sum() + res.sum()


def oracle_grads(cfg, xi_bar, b, lam0, iters):
    s = O.build_system(cfg)
    xb = torch.tensor(xi_bar, requires_grad=True)
    x0 = torch.tensor(xi_bar, requires_grad=True)
    l0 = torch.tensor(lam0, requires_grad=True)
    xk, _, r = O.sf_project(s, xb, torch.tensor(b), iters, xi0=x0, lam0=l0)
    L = loss_fn(xk, xb.detach(), r[:, 0])
    gx0, gl0 = torch.autograd.grad(L, (x0, l0))
    # gradient with respect to xi_bar as the SF target only (xi0 held fixed)
    xb2 = torch.tensor(xi_bar, requires_grad=True)
    xk2, _, r2 = O.sf_project(s, xb2, torch.tensor(b), iters, xi0=torch.tensor(xi_bar), lam0=torch.tensor(lam0))
    L2 = ((xk2 - torch.tensor(xi_bar)) ** 2).sum() + r2[:, 0].sum()
    (gxb,) = torch.autograd.grad(L2, (xb2,))
    return gx0, gl0, gxb


def gpu_grads(P, cfg, xi_bar, b, lam0, iters, ce, precision):
    dt = torch.float64 if precision == "fp64" else torch.float32
    sf = P.SafetyFilter([cfg])
    xb = torch.tensor(xi_bar, dtype=dt, device="cuda")
    x0 = xb.clone().requires_grad_(True)
    l0 = torch.tensor(lam0, dtype=dt, device="cuda").requires_grad_(True)
    xbr = xb.clone().requires_grad_(True)
    bv = torch.tensor(b, dtype=dt, device="cuda")
    xk, lk, res, _ = P.project_differentiable(sf, xbr, bv, iters, xi0=x0, lam0=l0, ckpt_every=ce, precision=precision)
    L = loss_fn(xk, xb, res)
    gx0, gl0, gxb = torch.autograd.grad(L, (x0, l0, xbr))
    torch.cuda.synchronize()
    return gx0.cpu().double(), gl0.cpu().double(), gxb.cpu().double(), sf, bv


def rel_err(a, b):
    return ((a - b).abs().max() / b.abs().max().clamp_min(1e-12)).item()


@pytest.mark.parametrize("iters,ce", [(25, 10), (12, 4), (1, 10)])
def test_adjoint_fp64_matches_oracle_autograd(P, iters, ce):
    cfg, xi, b, rng = problem()
    lam0 = rng.normal(size=xi.shape) * 0.1
    og = oracle_grads(cfg, xi, b, lam0, iters)
    gg = gpu_grads(P, cfg, xi, b, lam0, iters, ce, "fp64")
    for nm, a, r in zip(("xi0", "lam0", "xi_bar"), gg[:3], og):
        assert rel_err(a, r) <= 1e-8, (nm, rel_err(a, r))


def test_adjoint_fp32_matches_oracle_autograd(P):
    cfg, xi, b, rng = problem(n=6, S=3, H=30, seed=5)
    lam0 = rng.normal(size=xi.shape) * 0.1
    og = oracle_grads(cfg, xi, b, lam0, 30)
    gg = gpu_grads(P, cfg, xi, b, lam0, 30, 10, "fp32")
    for nm, a, r in zip(("xi0", "lam0", "xi_bar"), gg[:3], og):
        assert rel_err(a, r) <= 2e-3, (nm, rel_err(a, r))


def test_adjoint_fp64_central_differences(P):
    cfg, xi, b, rng = problem(n=5, S=2, H=24, seed=8)
    lam0 = rng.normal(size=xi.shape) * 0.1
    gx0, gl0, _, sf, bv = gpu_grads(P, cfg, xi, b, lam0, 20, 10, "fp64")
    xb = torch.tensor(xi, device="cuda")

    def L(dx, dl):
        out = sf.project(xb, bv, 20, precision="fp64", xi0=(xb + dx).contiguous(),
                         lam0=(torch.tensor(lam0, device="cuda") + dl).contiguous(), generic=True)
        return loss_fn(out.xi, xb, out.resid[:, 0]).item()
    # The map is piecewise smooth (a pair enters or leaves collision at ||s|| = 1), so the step
    # must stay below the distance to the nearest kink: 1e-6 moves positions by ~1e-6 m.
    h = 1e-6
    for _ in range(8):
        dx = torch.tensor(rng.normal(size=xi.shape), device="cuda")
        dl = torch.tensor(rng.normal(size=xi.shape), device="cuda")
        fd = (L(h * dx, h * dl) - L(-h * dx, -h * dl)) / (2 * h)
        an = (gx0 * dx.cpu()).sum().item() + (gl0 * dl.cpu()).sum().item()
        assert abs(fd - an) <= 1e-4 * max(1.0, abs(an)), (fd, an)


def test_adjoint_diff16_full_size(P):
    """512 samples, 16 robots, 100 unrolled FP32 iterations, checkpoints every 10: directional
    derivatives against FP32 central differences (step 1e-3) on 8 random directions, and two
    samples against autograd through the oracle."""
    wl = W.diff16()
    p = wl.problems[0]
    sf = P.SafetyFilter([p.cfg])
    xb = torch.tensor(p.xi_bar, dtype=torch.float32, device="cuda")
    bv = torch.tensor(p.bvals, dtype=torch.float32, device="cuda")
    rng = np.random.default_rng(11)
    lam0 = torch.zeros_like(xb)
    x0 = xb.clone().requires_grad_(True)
    l0 = lam0.clone().requires_grad_(True)
    xk, lk, res, _ = P.project_differentiable(sf, xb, bv, wl.iters, xi0=x0, lam0=l0, ckpt_every=wl.ckpt_every)
    L = loss_fn(xk, xb, res)
    gx0, gl0 = torch.autograd.grad(L, (x0, l0))
    assert torch.isfinite(gx0).all() and torch.isfinite(gl0).all()

    def Lf(dx, dl):
        out = sf.project(xb, bv, wl.iters, precision="fp32", xi0=(xb + dx).contiguous(),
                         lam0=(lam0 + dl).contiguous(), generic=True)
        return loss_fn(out.xi.double(), xb.double(), out.resid[:, 0].double()).item()
    h = 1e-3
    errs = []
    for _ in range(8):
        dx = torch.tensor(rng.normal(size=p.xi_bar.shape), dtype=torch.float32, device="cuda") * 0.1
        dl = torch.tensor(rng.normal(size=p.xi_bar.shape), dtype=torch.float32, device="cuda") * 0.1
        fd = (Lf(h * dx, h * dl) - Lf(-h * dx, -h * dl)) / (2 * h)
        an = (gx0.double() * dx.double()).sum().item() + (gl0.double() * dl.double()).sum().item()
        errs.append(abs(fd - an) / max(1.0, abs(an)))
    assert max(errs) <= 2e-2, errs
    # per-sample gradients of two samples against autograd through the oracle
    idx = [0, 400]
    og = oracle_grads(p.cfg, p.xi_bar[idx], p.bvals, np.zeros_like(p.xi_bar[idx]), wl.iters)
    for nm, a, r in zip(("xi0", "lam0"), (gx0[idx].cpu().double(), gl0[idx].cpu().double()), og[:2]):
        assert rel_err(a, r) <= 5e-3, (nm, rel_err(a, r))


@pytest.mark.parametrize("iters,ce", [(12, 5), (7, 10)])
def test_fixed_point_residual_term_matches_oracle(P, iters, ce):
    """The first term of eq. (NN_loss), w sum_k ||z^{k+1} - z^k||^2 with z = (xi, lambda): its
    value (SF_FP_RESIDUAL) and its gradients through the adjoint, against autograd through the
    oracle's iterations taken one at a time (the oracle solves the exact KKT system each step, so
    chained single steps equal one longer run)."""
    cfg, xi_bar, b, rng = problem(seed=12)
    lam0 = rng.normal(size=xi_bar.shape) * 0.1
    w = 0.7
    s = O.build_system(cfg)
    xb = torch.tensor(xi_bar)
    x0 = torch.tensor(xi_bar + rng.normal(size=xi_bar.shape) * 0.05, requires_grad=True)
    l0 = torch.tensor(lam0, requires_grad=True)
    xi, lam = x0, l0
    fsum = torch.zeros(xi_bar.shape[0], dtype=torch.float64)
    for _ in range(iters):
        xn, ln, _ = O.sf_project(s, xb, torch.tensor(b), 1, xi0=xi, lam0=lam)
        fsum = fsum + ((xn - xi) ** 2).sum((1, 2, 3)) + ((ln - lam) ** 2).sum((1, 2, 3))
        xi, lam = xn, ln
    L = w * fsum.sum() + ((xi - xb) ** 2).sum()
    gx0, gl0 = torch.autograd.grad(L, (x0, l0))
    _say(f"case nn_loss fixed-point term fp64 iters={iters} ckpt_every={ce}")
    sf = P.SafetyFilter([cfg])
    xbd = xb.cuda()
    x0d = x0.detach().cuda().requires_grad_(True)
    l0d = l0.detach().cuda().requires_grad_(True)
    xk, _, _, fpr = P.project_differentiable(sf, xbd, torch.tensor(b).cuda(), iters, xi0=x0d, lam0=l0d,
                                             ckpt_every=ce, precision="fp64")
    assert torch.allclose(fpr.cpu(), fsum.detach(), rtol=1e-9, atol=1e-12), (fpr, fsum)
    Lg = w * fpr.sum() + ((xk - xbd) ** 2).sum()
    g0, g1 = torch.autograd.grad(Lg, (x0d, l0d))
    torch.cuda.synchronize()
    assert rel_err(g0.cpu().double(), gx0) <= 1e-8
    assert rel_err(g1.cpu().double(), gl0) <= 1e-8


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_fixed_point_residual_sum_on_the_mfma_kernel(P, prec):
    """SF_FP_RESIDUAL on the MFMA kernels: the per-sample sum matches the generic FP64 kernel's, the
    checkpoints the differentiable forward writes are unchanged by the flag, and so are the
    iterates."""
    p = W.small3d(n_robots=16, n_samples=6, degree=10, horizon=100, seed=21,
                  box=((-3.0, -3.0, -1.0), (3.0, 3.0, 1.0)), t_final=10.0)
    sf = P.SafetyFilter([p.cfg])
    xb = torch.tensor(p.xi_bar, dtype=torch.float32, device="cuda")
    bv = torch.tensor(p.bvals, dtype=torch.float32, device="cuda")
    _say(f"case fixed-point residual MFMA {prec}")
    a = sf.project(xb, bv, 40, precision=prec, fp_residual=True, ckpt_every=10)
    b = sf.project(xb, bv, 40, precision=prec, ckpt_every=10)
    r64 = sf.project(xb.double(), bv.double(), 40, precision="fp64", fp_residual=True)
    torch.cuda.synchronize()
    assert torch.equal(a.xi, b.xi) and torch.equal(a.lam, b.lam) and torch.equal(a.ckpt, b.ckpt)
    assert torch.equal(a.resid[:, :2], b.resid)
    e = ((a.resid[:, 2].double() - r64.resid[:, 2]).abs() / r64.resid[:, 2]).max().item()
    _say(f"  fixed-point residual sum rel err {e:.2e}")
    assert e <= (1e-4 if prec == "fp32" else 2e-3)


def oracle_chained(cfg, xi_bar, b, xi0, lam0, iters, w):
    """Autograd through the oracle's iterations taken one at a time, with the loss
    w sum_k ||z^{k+1} - z^k||^2 + ||xi^K - xi_bar||^2 + ||r_p^K||^2."""
    s = O.build_system(cfg)
    xb = torch.tensor(xi_bar, requires_grad=True)
    x0 = torch.tensor(xi0, requires_grad=True)
    l0 = torch.tensor(lam0, requires_grad=True)
    xi, lam = x0, l0
    fsum = torch.zeros(xi_bar.shape[0], dtype=torch.float64)
    r = None
    for _ in range(iters):
        xn, ln, r = O.sf_project(s, xb, torch.tensor(b), 1, xi0=xi, lam0=lam)
        fsum = fsum + ((xn - xi) ** 2).sum((1, 2, 3)) + ((ln - lam) ** 2).sum((1, 2, 3))
        xi, lam = xn, ln
    L = w * fsum.sum() + ((xi - torch.tensor(xi_bar)) ** 2).sum() + r[:, 0].sum()
    return torch.autograd.grad(L, (x0, l0, xb))


@pytest.mark.parametrize("n,H,degree,iters,ce,prec", [(6, 30, 8, 17, 5, "fp32"), (16, 100, 10, 20, 10, "fp32"),
                                                      (16, 100, 10, 20, 10, "bf16"), (11, 45, 13, 9, 4, "fp32")])
def test_mfma_adjoint_matches_oracle_autograd(P, n, H, degree, iters, ce, prec):
    """The reverse mode on the matrix cores (recompute with the forward MFMA kernel, reverse sweep
    per checkpoint segment) with every loss term: the projected coefficients, the final residual
    and the fixed-point residual sum, against autograd through the oracle; segments that do not
    divide the iterations, degrees 8 to 13 and the bf16 forward."""
    cfg, xi, b, rng = problem(n=n, S=3, H=H, degree=degree, seed=40 + n, box=2.0 if n > 8 else 1.0, T=8.0)
    xi0 = xi + rng.normal(size=xi.shape) * 0.05
    lam0 = rng.normal(size=xi.shape) * 0.1
    w = 0.3
    ref = oracle_chained(cfg, xi, b, xi0, lam0, iters, w)
    _say(f"case MFMA adjoint n={n} H={H} degree={degree} iters={iters} ckpt_every={ce} {prec}")
    sf = P.SafetyFilter([cfg])
    dt = torch.float32
    xbg = torch.tensor(xi, dtype=dt, device="cuda").requires_grad_(True)
    x0g = torch.tensor(xi0, dtype=dt, device="cuda").requires_grad_(True)
    l0g = torch.tensor(lam0, dtype=dt, device="cuda").requires_grad_(True)
    xk, _, res, fpr = P.project_differentiable(sf, xbg, torch.tensor(b, dtype=dt, device="cuda"), iters, xi0=x0g,
                                               lam0=l0g, ckpt_every=ce, precision=prec)
    L = w * fpr.sum() + ((xk - xbg.detach()) ** 2).sum() + res.sum()
    got = torch.autograd.grad(L, (x0g, l0g, xbg))
    torch.cuda.synchronize()
    tol = 2e-3 if prec == "fp32" else 1e-2
    for nm, a, r in zip(("xi0", "lam0", "xi_bar"), got, ref):
        e = rel_err(a.cpu().double(), r)
        _say(f"  {nm}: rel err {e:.2e}")
        assert e <= tol, (nm, e)


def test_mfma_adjoint_ragged_batch_equals_per_problem(P):
    """A batch of two swarm sizes through the MFMA adjoint equals per-problem calls."""
    probs = [problem(n=n, S=S, H=40, degree=9, seed=60 + n, box=1.5) for n, S in ((5, 3), (12, 2))]
    cfgs = [p[0] for p in probs]
    sf = P.SafetyFilter(cfgs)
    batch = P.Batch([(0, 3), (1, 2)])
    xb = torch.cat([torch.tensor(p[1], dtype=torch.float32).reshape(-1) for p in probs]).cuda()
    bv = torch.cat([torch.tensor(p[2], dtype=torch.float32).reshape(-1) for p in probs]).cuda()
    iters, ce = 12, 5
    _say("case MFMA adjoint ragged batch")
    out = sf.project(xb, bv, iters, batch=batch, ckpt_every=ce, fp_residual=True)
    g_xi = torch.ones_like(xb)
    g_res = torch.ones((5,), dtype=torch.float32, device="cuda")
    w = torch.full((5,), 0.5, dtype=torch.float32, device="cuda")
    g = sf.project_backward(xb, bv, iters, out.ckpt, ce, g_xi_out=g_xi, g_resid=g_res, w_fpr=w, batch=batch)
    torch.cuda.synchronize()
    o = r0 = 0
    for k, (cfg, xi, b, _) in enumerate(probs):
        one = P.SafetyFilter([cfg])
        x1 = torch.tensor(xi, dtype=torch.float32).cuda()
        b1 = torch.tensor(b, dtype=torch.float32).cuda()
        o1 = one.project(x1, b1, iters, ckpt_every=ce, fp_residual=True)
        S = xi.shape[0]
        g1 = one.project_backward(x1, b1, iters, o1.ckpt, ce, g_xi_out=torch.ones_like(x1),
                                  g_resid=g_res[r0:r0 + S].contiguous(), w_fpr=w[r0:r0 + S].contiguous())
        torch.cuda.synchronize()
        for key in ("xi0", "lam0", "xi_bar"):
            assert torch.allclose(g[key][o:o + xi.size].reshape(g1[key].shape), g1[key], rtol=1e-5, atol=1e-6), key
        o += xi.size
        r0 += S


@pytest.mark.parametrize("precision,n,tol", [("fp64", 40, 1e-8), ("fp32", 64, 2e-3)])
def test_adjoint_at_its_size_limits(P, precision, n, tol):
    """The most robots the adjoint's LDS plan takes at degree 10 (FP64: 40 robots in 150 KB; FP32:
    64 robots in 118 KB), both with a one-step time tile, against autograd through the oracle."""
    cfg, xi, b, rng = problem(n=n, S=1, H=40, degree=10, seed=30 + n, box=4.0)
    lam0 = rng.normal(size=xi.shape) * 0.1
    og = oracle_grads(cfg, xi, b, lam0, 6)
    _say(f"case adjoint limits {precision} n={n} degree=10 H=40 iters=6 ckpt_every=4")
    gg = gpu_grads(P, cfg, xi, b, lam0, 6, 4, precision)
    for nm, a, r in zip(("xi0", "lam0", "xi_bar"), gg[:3], og):
        assert rel_err(a, r) <= tol, (nm, rel_err(a, r))


def test_adjoint_refuses_shapes_past_its_lds_bound(P):
    from paper_2501_19042_amd import _native as N
    cfg, xi, b, rng = problem(n=44, S=1, H=40, degree=10, seed=74, box=4.0)
    _say("case adjoint limits refusal fp64 n=44")
    with pytest.raises(N.SfError):
        gpu_grads(P, cfg, xi, b, np.zeros_like(xi), 4, 4, "fp64")
