"""GPU parity at the size limits of the C ABI, against the FP64 oracle.

The generic kernel accepts up to 64 robots, degree 30 and horizon 4096 as long as one sample's
state fits the 160 KB of LDS of a workgroup (with a time tile of one step when it needs more than
80 KB); the MFMA kernel takes up to 32 robots, 16 coefficients and horizon 256.  Each case runs
the largest shape of one limit and checks it against the oracle; shapes past the LDS bound must be
refused with an error before any launch.

Tolerances: FP64 elementwise |gpu - oracle| <= 1e-9 (1 + |oracle|); FP32 per sample
max|gpu - oracle| / max|oracle| <= 1e-4 on the coefficients.
"""
import sys

import numpy as np
import pytest
import torch

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-9
FP32_TOL = 1e-4
BOX = ((-4.0, -4.0, -1.0), (4.0, 4.0, 1.0))


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def P():
    import paper_2501_19042_amd as P
    torch.cuda.set_device(0)
    return P


def problem(n, degree, H, S):
    return W.small3d(n_robots=n, n_samples=S, degree=degree, horizon=H, seed=200 + n, box=BOX, t_final=10.0)


def oracle_run(p, iters):
    s = O.build_system(p.cfg)
    return O.sf_project(s, torch.as_tensor(p.xi_bar), torch.as_tensor(p.bvals), iters)


def gpu_run(P, p, iters, precision):
    dt = torch.float64 if precision == "fp64" else torch.float32
    sf = P.SafetyFilter([p.cfg])
    xb = torch.as_tensor(p.xi_bar, dtype=dt).cuda()
    bv = torch.as_tensor(p.bvals, dtype=dt).cuda()
    out = sf.project(xb, bv, iters, precision=precision)
    torch.cuda.synchronize()
    return out


def fp64_err(gpu, ref):
    g = gpu.detach().cpu().double()
    return ((g - ref).abs() / (1.0 + ref.abs())).max().item()


# (robots, degree, horizon): 64 robots (largest count; 129 KB of LDS, one-step time tile),
# degree 30 with the most robots that fit (28 robots, 151 KB), horizon 4096 (largest horizon).
@pytest.mark.parametrize("n,degree,H", [(64, 10, 60), (28, 30, 40), (4, 30, 4096)])
def test_generic_fp64_at_the_limits(P, n, degree, H):
    p = problem(n, degree, H, 2)
    iters = 6
    _say(f"case limits fp64 n={n} degree={degree} H={H} iters={iters}")
    out = gpu_run(P, p, iters, "fp64")
    rx, rl, rr = oracle_run(p, iters)
    assert rr[:, 0].min().item() > 0                      # constraints active, not a pass-through
    assert fp64_err(out.xi, rx) <= FP64_TOL
    assert fp64_err(out.lam, rl) <= FP64_TOL
    assert torch.allclose(out.resid.cpu(), rr, rtol=1e-7, atol=1e-12)


def test_mfma_fp32_at_its_limit(P):
    """32 robots, degree 15 (16 coefficients), horizon 256: sixteen time tiles of 16 steps."""
    p = problem(32, 15, 256, 2)
    iters = 8
    _say(f"case limits fp32 n=32 degree=15 H=256 iters={iters}")
    out = gpu_run(P, p, iters, "fp32")
    rx, rl, rr = oracle_run(p, iters)
    g = out.xi.cpu().double().reshape(2, -1)
    r = rx.reshape(2, -1)
    e = ((g - r).abs().amax(1) / r.abs().amax(1)).numpy()
    assert e.max() <= FP32_TOL, e
    assert torch.allclose(out.resid.cpu().double(), rr, rtol=2e-2, atol=1e-6)


def test_generic_fp32_at_the_limits(P):
    """64 robots at degree 16 fit in FP32 (96 KB, one-step time tile) but not in FP64."""
    p = problem(64, 16, 60, 2)
    iters = 6
    _say(f"case limits fp32 generic n=64 degree=16 H=60 iters={iters}")
    out = gpu_run(P, p, iters, "fp32")
    rx, rl, rr = oracle_run(p, iters)
    g = out.xi.cpu().double().reshape(2, -1)
    r = rx.reshape(2, -1)
    e = ((g - r).abs().amax(1) / r.abs().amax(1)).numpy()
    assert e.max() <= FP32_TOL, e
    assert torch.allclose(out.resid.cpu().double(), rr, rtol=2e-2, atol=1e-6)


@pytest.mark.parametrize("precision,n,degree", [("fp64", 64, 30), ("fp64", 32, 30), ("fp64", 64, 16),
                                                ("fp32", 64, 30)])
def test_shapes_past_the_lds_bound_are_refused(P, precision, n, degree):
    from paper_2501_19042_amd import _native as N
    p = problem(n, degree, 40, 1)
    _say(f"case limits refusal {precision} n={n} degree={degree}")
    with pytest.raises(N.SfError):
        gpu_run(P, p, 2, precision)


def _flat(probs, dt=torch.float32):
    xb = torch.cat([torch.as_tensor(p.xi_bar, dtype=dt).reshape(-1) for p in probs]).cuda()
    bv = torch.cat([torch.as_tensor(p.bvals, dtype=dt).reshape(-1) for p in probs]).cuda()
    return xb, bv


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_batch_mixing_covered_and_uncovered_shapes(P, precision):
    """One call over a 64-robot problem (outside the MFMA kernels' shapes) and a 16- and a 20-robot
    problem (inside them): the covered problems run on the MFMA kernels (a persistent launch over
    their two robot-tile classes) in the requested precision, the 64-robot one on the generic
    kernel in FP32 with the one-step time tile it needs.  Every problem matches the oracle, and
    each part is bit for bit the call over that part alone."""
    probs = [problem(64, 10, 60, 2), problem(16, 10, 100, 3), problem(20, 10, 100, 2)]
    sf = P.SafetyFilter([p.cfg for p in probs])
    batch = P.Batch([(i, p.xi_bar.shape[0]) for i, p in enumerate(probs)])
    xb, bv = _flat(probs)
    iters = 6
    _say(f"case limits mixed batch {precision} n=64+16+20 iters={iters}")
    out = sf.project(xb, bv, iters, batch=batch, precision=precision, want_status=True)
    torch.cuda.synchronize()
    from paper_2501_19042_amd import _native as N
    assert ((out.status.cpu() & (N.SF_SAMPLE_NONFINITE | N.SF_SAMPLE_NONFINITE_INPUT)) == 0).all()
    tol = FP32_TOL if precision == "fp32" else 2e-3
    o = 0
    parts = []
    for p in probs:
        S = p.xi_bar.shape[0]
        rx, _, _ = oracle_run(p, iters)
        g = out.xi[o:o + p.xi_bar.size]
        parts.append(g)
        r = rx.reshape(S, -1)
        e = ((g.cpu().double().reshape(S, -1) - r).abs().amax(1) / r.abs().amax(1)).numpy()
        assert e.max() <= tol, e
        o += p.xi_bar.size
    # the covered part alone (MFMA kernels, same precision) and the uncovered problem alone (generic, FP32)
    sf_c = P.SafetyFilter([probs[1].cfg, probs[2].cfg])
    xc, bc = _flat(probs[1:])
    oc = sf_c.project(xc, bc, iters, batch=P.Batch([(0, 3), (1, 2)]), precision=precision)
    og = gpu_run(P, probs[0], iters, "fp32")
    torch.cuda.synchronize()
    assert torch.equal(torch.cat(parts[1:]), oc.xi)
    assert torch.equal(parts[0], og.xi.reshape(-1))
