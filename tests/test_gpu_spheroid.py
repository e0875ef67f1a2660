"""GPU parity for spheroidal robots (a != b in the collision rows, the scaled projection of the
Appendix's polar form, reading R4) against the FP64 oracle, through the C ABI: generic kernel in
FP64, MFMA kernel in FP32 and bf16, the full-size workload sampled, and the tie-break of
coincident robots, whose target is (0, 0, b).  (The oracle's side of the reading is pinned by
the closed form of the scaled radial projection in the oracle pins.)
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
BF16_TOL = 2e-3


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def P():
    import paper_2501_19042_amd as P
    torch.cuda.set_device(0)
    return P


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
    return out


def rel(gpu, ref):
    g = gpu.detach().cpu().double().reshape(gpu.shape[0], -1)
    r = torch.as_tensor(ref).double().reshape(ref.shape[0], -1)
    return ((g - r).abs().amax(1) / r.abs().amax(1)).numpy()


def spheroid_case(n=6, S=6, H=45, seed=41, b=0.55):
    p = W.small3d(n_robots=n, n_samples=S, horizon=H, seed=seed)
    return replace(p.cfg, safety_b=b), p.xi_bar, p.bvals


def test_collisions_are_active_in_these_cases():
    cfg, xb, bv = spheroid_case()
    f = O.feasibility(O.build_system(cfg), torch.as_tensor(xb), torch.as_tensor(bv)).numpy()
    assert (f[:, 0] > 0.02).any(), f[:, 0]


def test_fp64_spheroid_matches_oracle(P):
    cfg, xb, bv = spheroid_case()
    for k in (1, 50):
        _say(f"case spheroid fp64 k={k}")
        out = run(P, cfg, xb, bv, k, "fp64")
        rx, rl, rr = oracle(cfg, xb, bv, k)
        for got, ref, nm in ((out.xi, rx, "xi"), (out.lam, rl, "lambda")):
            g = got.cpu().double()
            err = ((g - ref).abs() / (1.0 + ref.abs())).max().item()
            assert err <= FP64_TOL, (nm, k, err)
        assert torch.allclose(out.resid.cpu(), rr, rtol=1e-7, atol=1e-12)


@pytest.mark.parametrize("prec,tol", [("fp32", FP32_TOL), ("bf16", BF16_TOL)])
def test_mfma_spheroid_matches_oracle(P, prec, tol):
    cfg, xb, bv = spheroid_case(n=16, S=3, H=100, seed=43)
    cfg = replace(cfg, t_final=10.0)
    for k in (10, 60):
        _say(f"case spheroid {prec} k={k}")
        out = run(P, cfg, xb, bv, k, prec)
        rx, _, _ = oracle(cfg, xb, bv, k)
        e = rel(out.xi, rx)
        assert e.max() <= tol, (prec, k, e)


def test_full_size_spheroid_workload_sampled(P):
    wl = W.swarm16sph()
    p = wl.problems[0]
    idx = [0, 400, 1023]
    for k in (10, 50):
        _say(f"case swarm16sph fp32 full size k={k}")
        out = run(P, p.cfg, p.xi_bar, p.bvals, k, "fp32")
        rx, _, _ = oracle(p.cfg, p.xi_bar[idx], p.bvals, k)
        e = rel(out.xi[idx], rx)
        assert e.max() <= FP32_TOL, (k, e)


def test_coincident_spheroidal_robots(P):
    # robots 0 and 1 rest at the origin (all coefficients exactly 0), so r = 0 exactly at every
    # grid time and the atan2(0, 0) tie-break sends the pair along z towards (0, 0, b), b != a
    cfg = W.SwarmConfig(n_robots=3, dims=3, degree=8, horizon=20, t_final=5.0, safety_a=0.3,
                        safety_b=0.45, vmax=1.5, amax=2.0)
    st = np.zeros((3, 3)); gl = np.zeros((3, 3))
    st[2, :2] = (1.0, 1.0); gl[2, :2] = (-1.0, 1.0)
    xi = W.straight_line_coeffs(st, gl, 8)[None]
    b = W.boundary_values(st, gl)
    _say("case coincident spheroidal fp64")
    out = run(P, cfg, xi, b, 30, "fp64")
    rx, _, _ = oracle(cfg, xi, b, 30)
    g = out.xi.cpu()
    assert ((g - rx).abs() / (1 + rx.abs())).max().item() <= FP64_TOL
    assert (rx[0, 0, 2, 3:-3] > 0).all() and (rx[0, 1, 2, 3:-3] < 0).all()
