"""Precision form: S1 basis products in bf16 / fp16 MFMA with the rounding residuals of both
factors fed back as correction terms (fp32 accumulation, fp32 state).  Per-sample error against
the FP64 oracle is reported and bounded; converged fractions match the FP32 solver."""
import numpy as np
import pytest
import torch

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

BOUND = {"fp16": 2e-4, "bf16": 2e-3}


@pytest.fixture(scope="module")
def P():
    import paper_2501_19042_amd as P
    torch.cuda.set_device(0)
    return P


def rel(gpu, ref):
    g = gpu.detach().cpu().double().reshape(gpu.shape[0], -1)
    r = torch.as_tensor(ref).double().reshape(ref.shape[0], -1)
    return ((g - r).abs().amax(1) / r.abs().amax(1)).numpy()


def run(P, cfg, xi_bar, bvals, iters, prec):
    sf = P.SafetyFilter([cfg])
    xb = torch.as_tensor(xi_bar, dtype=torch.float32).cuda()
    bv = torch.as_tensor(bvals, dtype=torch.float32).cuda()
    out = sf.project(xb, bv, iters, precision=prec)
    torch.cuda.synchronize()
    return sf, out, bv


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
@pytest.mark.parametrize("n,degree,H", [(16, 10, 100), (32, 12, 120), (7, 10, 45)])
def test_precision_form_against_oracle(P, prec, n, degree, H):
    p = W.small3d(n_robots=n, n_samples=3, degree=degree, horizon=H, seed=200 + n,
                  box=((-3.0, -3.0, -1.0), (3.0, 3.0, 1.0)), t_final=10.0)
    s = O.build_system(p.cfg)
    for k in (10, 60):
        _, out, _ = run(P, p.cfg, p.xi_bar, p.bvals, k, prec)
        rx, _, _ = O.sf_project(s, torch.tensor(p.xi_bar), torch.tensor(p.bvals), k)
        e = rel(out.xi, rx)
        print(f"{prec} n={n} k={k} per-sample rel error {e}", flush=True)
        assert e.max() <= BOUND[prec], (prec, n, k, e)


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
def test_precision_form_full_size_swarm32(P, prec):
    """32 robots, degree 12, H 120, 4096 samples, 300 iterations: converged fraction equal to
    the FP32 solver's (within 0.5%), sampled outputs against the oracle."""
    wl = W.swarm32()
    p = wl.problems[0]
    sf, out, bv = run(P, p.cfg, p.xi_bar, p.bvals, wl.iters, prec)
    _, ref32, _ = run(P, p.cfg, p.xi_bar, p.bvals, wl.iters, "fp32")
    tol = 1e-3
    f16 = sf.feasibility(out.xi, bv).cpu()
    f32 = sf.feasibility(ref32.xi, bv).cpu()
    c16 = ((f16[:, :3] <= tol).all(1) & (f16[:, 3] <= tol)).double().mean().item()
    c32 = ((f32[:, :3] <= tol).all(1) & (f32[:, 3] <= tol)).double().mean().item()
    print(f"{prec} converged {c16:.4f} vs fp32 {c32:.4f}", flush=True)
    assert c16 >= c32 - 0.005
    idx = [0, 1000, 4095]
    s = O.build_system(p.cfg)
    rx, _, _ = O.sf_project(s, torch.tensor(p.xi_bar[idx]), torch.tensor(p.bvals), wl.iters)
    e = rel(out.xi[idx], rx)
    e32 = rel(ref32.xi[idx], rx)
    print(f"{prec} full-size per-sample rel error {e} (fp32 {e32})", flush=True)
    assert torch.isfinite(out.xi).all()
    assert e.max() <= BOUND[prec], (e, e32)
