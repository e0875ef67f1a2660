"""GPU parity of the workspace rows (the F_w block of eq. (f_e), eq. (workspace_polar)) against
the FP64 oracle, through the C ABI: the generic kernel in FP64 and FP32, the MFMA kernels in FP32
and the 16-bit forms, ragged batches that mix configs with and without a workspace, the
violation report and the adjoint through the workspace rows.

Tolerances as for the other constraints: FP64 elementwise |gpu - oracle| <= 1e-9 (1 + |oracle|);
FP32 per sample max|gpu - oracle| / max|oracle| <= 1e-4; bf16 2e-3 and fp16 2e-4.
"""
import sys
from dataclasses import replace

import numpy as np
import pytest
import torch

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-9
FP32_TOL = 1e-4
BOUND = {"fp16": 2e-4, "bf16": 2e-3}


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def P():
    import paper_2501_19042_amd as P
    torch.cuda.set_device(0)
    return P


def ws_problem(n, S, H, seed, ws=(1.6, 0.55), centre=(0.1, -0.05, 0.05), rho_ws=0.8, box=None):
    """The small 3D instance (x, y in [-1.2, 1.2], z in [-0.5, 0.5]) inside an off-centre
    spheroid tight enough that part of most trajectories lies outside it."""
    kw = {} if box is None else {"box": box, "t_final": 10.0}
    p = W.small3d(n_robots=n, n_samples=S, horizon=H, seed=seed, **kw)
    cfg = replace(p.cfg, ws_a=ws[0], ws_b=ws[1], ws_x=centre[0], ws_y=centre[1], ws_z=centre[2],
                  rho_ws=rho_ws)
    return cfg, p.xi_bar, p.bvals


def oracle(cfg, xi_bar, bvals, iters):
    s = O.build_system(cfg)
    return O.sf_project(s, torch.as_tensor(xi_bar, dtype=torch.float64),
                        torch.as_tensor(bvals, dtype=torch.float64), iters)


def run(P, cfg, xi_bar, bvals, iters, precision, **kw):
    dt = torch.float64 if precision == "fp64" else torch.float32
    sf = P.SafetyFilter([cfg])
    xb = torch.as_tensor(xi_bar, dtype=dt).cuda().contiguous()
    bv = torch.as_tensor(bvals, dtype=dt).cuda().contiguous()
    out = sf.project(xb, bv, iters, precision=precision, **kw)
    torch.cuda.synchronize()
    return sf, out, bv


def rel(gpu, ref):
    g = gpu.detach().cpu().double().reshape(gpu.shape[0], -1)
    r = torch.as_tensor(ref).double().reshape(ref.shape[0], -1)
    return ((g - r).abs().amax(1) / r.abs().amax(1)).numpy()


def test_workspace_is_active_in_these_cases():
    # the cases below exercise the rows: the sampled trajectories leave the spheroid
    cfg, xb, bv = ws_problem(5, 4, 40, 11)
    f = O.feasibility(O.build_system(cfg), torch.as_tensor(xb), torch.as_tensor(bv)).numpy()
    assert (f[:, 4] > 0.05).all(), f[:, 4]


@pytest.mark.parametrize("D", [2, 3])
def test_fp64_workspace_matches_oracle(P, D):
    if D == 3:
        cfg, xb, bv = ws_problem(5, 4, 40, 11)
    else:
        p = W.tiny2d(4).problems[0]
        cfg = replace(p.cfg, ws_a=1.8, ws_x=0.2, ws_y=-0.1, rho_ws=1.3)
        xb, bv = p.xi_bar, p.bvals
    for k in (1, 60):
        _say(f"case workspace fp64 D={D} k={k}")
        _, out, _ = run(P, cfg, xb, bv, k, "fp64")
        rx, rl, rr = oracle(cfg, xb, bv, k)
        for got, ref, nm in ((out.xi, rx, "xi"), (out.lam, rl, "lambda")):
            g = got.cpu().double()
            err = ((g - ref).abs() / (1.0 + ref.abs())).max().item()
            assert err <= FP64_TOL, (nm, k, err)
        assert torch.allclose(out.resid.cpu(), rr, rtol=1e-7, atol=1e-12)


@pytest.mark.parametrize("generic", [False, True])
def test_fp32_workspace_matches_oracle(P, generic):
    """MFMA kernel (3D, 6 robots, 45 grid times: three tiles and a ragged tail) and the generic
    kernel, against the oracle at 10 and 60 iterations; the residual report too."""
    cfg, xb, bv = ws_problem(6, 8, 45, 13)
    for k in (10, 60):
        _say(f"case workspace fp32 generic={generic} k={k}")
        _, out, _ = run(P, cfg, xb, bv, k, "fp32", generic=generic)
        rx, _, rr = oracle(cfg, xb, bv, k)
        e = rel(out.xi, rx)
        assert e.max() <= FP32_TOL, (k, e)
        res = out.resid.cpu().double()
        assert torch.allclose(res[:, 0], rr[:, 0], rtol=2e-3, atol=1e-9), (res, rr)
        assert torch.allclose(res[:, 1], rr[:, 1], rtol=2e-3, atol=1e-5), (res, rr)


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
def test_16bit_forms_with_workspace(P, prec):
    cfg, xb, bv = ws_problem(16, 3, 100, 216, ws=(4.0, 1.2), box=((-3.0, -3.0, -1.0), (3.0, 3.0, 1.0)))
    for k in (10, 60):
        _say(f"case workspace {prec} k={k}")
        _, out, _ = run(P, cfg, xb, bv, k, prec)
        rx, _, _ = oracle(cfg, xb, bv, k)
        e = rel(out.xi, rx)
        assert e.max() <= BOUND[prec], (prec, k, e)


def test_ragged_batch_mixing_workspace_and_plain_configs(P):
    """One persistent MFMA launch over problems of 5, 12 and 20 robots, two of them with a
    workspace: each problem against the oracle."""
    probs = []
    for n, S, seed, ws in ((5, 3, 31, True), (12, 2, 32, False), (20, 2, 33, True)):
        p = W.small3d(n_robots=n, n_samples=S, horizon=30, seed=seed,
                      box=((-2.5, -2.5, -0.8), (2.5, 2.5, 0.8)), t_final=8.0)
        cfg = replace(p.cfg, ws_a=2.6, ws_b=0.7, ws_x=0.1) if ws else p.cfg
        probs.append((cfg, p.xi_bar, p.bvals))
    sf = P.SafetyFilter([c for c, _, _ in probs])
    batch = P.Batch([(i, xb.shape[0]) for i, (_, xb, _) in enumerate(probs)])
    xb = torch.cat([torch.as_tensor(x, dtype=torch.float32).reshape(-1) for _, x, _ in probs]).cuda()
    bv = torch.cat([torch.as_tensor(b, dtype=torch.float32).reshape(-1) for _, _, b in probs]).cuda()
    _say("case workspace ragged fp32")
    out = sf.project(xb, bv, 40, batch=batch, precision="fp32")
    torch.cuda.synchronize()
    o = 0
    for cfg, x, b in probs:
        nel = x.size
        rx, _, _ = oracle(cfg, x, b, 40)
        e = rel(out.xi[o:o + nel].reshape(x.shape), rx)
        assert e.max() <= FP32_TOL, (cfg.n_robots, e)
        o += nel


def test_full_size_workspace_workload_sampled(P):
    """The 16-robot workload with its workspace (1024 samples, 300 iterations) in the launch the
    benchmark times; sampled outputs against the oracle."""
    wl = W.swarm16ws()
    p = wl.problems[0]
    idx = [0, 517, 1023]
    for k in (10, 50):
        _say(f"case swarm16ws fp32 full size k={k}")
        _, out, _ = run(P, p.cfg, p.xi_bar, p.bvals, k, "fp32")
        rx, _, _ = oracle(p.cfg, p.xi_bar[idx], p.bvals, k)
        e = rel(out.xi[idx], rx)
        assert e.max() <= FP32_TOL, (k, e)
        assert torch.isfinite(out.xi).all()


def test_violation_report_includes_workspace(P):
    cfg, xb, bv = ws_problem(5, 4, 40, 11)
    sf, out, bvd = run(P, cfg, xb, bv, 80, "fp64")
    s = O.build_system(cfg)
    for x in (torch.as_tensor(xb, dtype=torch.float64).cuda(), out.xi):
        v = sf.feasibility(x, bvd, precision="fp64").cpu()
        ref = O.feasibility(s, x.cpu(), torch.as_tensor(bv, dtype=torch.float64))
        assert torch.allclose(v[:, [0, 3, 4]], ref[:, [0, 3, 4]], atol=1e-12, rtol=1e-10)
        assert torch.allclose(v[:, 1:3], ref[:, 1:3], atol=1e-12, rtol=1e-10)
    # without a workspace the fifth column is zero
    p = W.small3d(n_robots=3, n_samples=2, horizon=12)
    sf2 = P.SafetyFilter([p.cfg])
    v = sf2.feasibility(torch.as_tensor(p.xi_bar).cuda(), torch.as_tensor(p.bvals).cuda(), precision="fp64")
    assert (v[:, 4] == 0).all()


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-8), ("fp32", 2e-3)])
def test_adjoint_with_workspace_matches_oracle_autograd(P, prec, tol):
    """The reverse mode through the workspace rows (their projection's 3x3 Jacobian, weight rho_ws)
    and through their share of the final primal residual: gradients of ||xi^K - xi_bar||^2 +
    ||r_p^K||^2 with respect to xi0, lambda0 and xi_bar against autograd through the oracle."""
    cfg, xb, bv = ws_problem(4, 2, 20, 7)
    rng = np.random.default_rng(9)
    lam0 = rng.normal(size=xb.shape) * 0.1
    iters, ce = 14, 5
    s = O.build_system(cfg)
    x0 = torch.tensor(xb, requires_grad=True)
    l0 = torch.tensor(lam0, requires_grad=True)
    xbo = torch.tensor(xb, requires_grad=True)
    xk, _, r = O.sf_project(s, xbo, torch.tensor(bv), iters, xi0=x0, lam0=l0)
    # the workspace is active in this case (some target differs from its position)
    L = ((xk - torch.tensor(xb)) ** 2).sum() + r[:, 0].sum()
    ref = torch.autograd.grad(L, (x0, l0, xbo))
    _say(f"case adjoint with workspace {prec}")
    dt = torch.float64 if prec == "fp64" else torch.float32
    sf = P.SafetyFilter([cfg])
    xg = torch.tensor(xb, dtype=dt, device="cuda")
    x0g = xg.clone().requires_grad_(True)
    l0g = torch.tensor(lam0, dtype=dt, device="cuda").requires_grad_(True)
    xbg = xg.clone().requires_grad_(True)
    out = P.project_differentiable(sf, xbg, torch.tensor(bv, dtype=dt, device="cuda"), iters, xi0=x0g, lam0=l0g,
                                   ckpt_every=ce, precision=prec)
    Lg = ((out[0] - xg) ** 2).sum() + out[2].sum()
    got = torch.autograd.grad(Lg, (x0g, l0g, xbg))
    torch.cuda.synchronize()
    for nm, a, b in zip(("xi0", "lam0", "xi_bar"), got, ref):
        e = ((a.cpu().double() - b).abs().max() / b.abs().max()).item()
        _say(f"  {nm}: rel err {e:.2e}")
        assert e <= tol, (nm, e)
