"""GPU parity of the equality-only QP layer (sf_qp_equality, its reverse mode) against the FP64
oracle's definition xi_in - A^T (A A^T)^{-1} (A xi_in - b), through the C ABI.

Tolerances: FP64 |gpu - oracle| <= 1e-12 (1 + |oracle|) (a 6 x 6 solve and a pass-through);
FP32 <= 1e-6 relative to the largest |value| per sample.  The pass-through coefficients must be
bit-identical to the input in every precision.
"""
import sys

import numpy as np
import pytest
import torch

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def P():
    import paper_2501_19042_amd as P
    torch.cuda.set_device(0)
    return P


def decoder_like(n, S, degree, seed, D=3):
    """Unconstrained decoder outputs: a noisy line whose end coefficients miss the boundary values."""
    p = W.small3d(n_robots=n, n_samples=S, degree=degree, horizon=degree + 15, seed=seed) if D == 3 else None
    if p is None:
        p = W.tiny2d(S).problems[0]
    rng = np.random.default_rng(seed)
    return p.cfg, p.xi_bar + rng.normal(size=p.xi_bar.shape) * 0.3, p.bvals


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("n,S,degree,D", [(5, 6, 10, 3), (16, 40, 10, 3), (3, 4, 5, 3), (4, 8, 10, 2)])
def test_forward_matches_oracle(P, prec, n, S, degree, D):
    cfg, xi, bv = decoder_like(n, S, degree, seed=50 + n, D=D)
    dt = torch.float64 if prec == "fp64" else torch.float32
    sf = P.SafetyFilter([cfg])
    x = torch.as_tensor(xi, dtype=dt).cuda()
    b = torch.as_tensor(bv, dtype=dt).cuda()
    _say(f"case qp_equality {prec} n={n} S={S} degree={degree} D={D}")
    out = P.qp_equality(sf, x, b, precision=prec)
    torch.cuda.synchronize()
    ref = O.qp_equality(O.build_system(cfg), torch.as_tensor(xi), torch.as_tensor(bv))
    got = out.cpu().double()
    if prec == "fp64":
        assert ((got - ref).abs() / (1 + ref.abs())).max().item() <= 1e-12
    else:
        rel = ((got - ref).abs().reshape(S, -1).amax(1) / ref.abs().reshape(S, -1).amax(1))
        assert rel.max().item() <= 1e-6, rel
    assert torch.equal(out[..., 3:-3].cpu(), x[..., 3:-3].cpu())


def test_in_place_and_ragged_batch(P):
    """A batch of problems of different shapes, many samples per problem (several sample chunks
    each), written in place; each problem against the oracle."""
    probs = [decoder_like(n, S, deg, seed=60 + n) for n, S, deg in ((5, 300, 10), (16, 130, 12), (8, 1, 7))]
    sf = P.SafetyFilter([c for c, _, _ in probs])
    batch = P.Batch([(i, xi.shape[0]) for i, (_, xi, _) in enumerate(probs)])
    x = torch.cat([torch.as_tensor(xi).reshape(-1) for _, xi, _ in probs]).cuda()
    b = torch.cat([torch.as_tensor(bv).reshape(-1) for _, _, bv in probs]).cuda()
    _say("case qp_equality ragged in place fp64")
    out = P.qp_equality(sf, x, b, batch=batch, precision="fp64", out=x)
    torch.cuda.synchronize()
    assert out.data_ptr() == x.data_ptr()
    o = 0
    for cfg, xi, bv in probs:
        ref = O.qp_equality(O.build_system(cfg), torch.as_tensor(xi), torch.as_tensor(bv))
        got = out[o:o + xi.size].cpu().reshape(xi.shape)
        assert ((got - ref).abs() / (1 + ref.abs())).max().item() <= 1e-12
        o += xi.size


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_reverse_mode_matches_oracle_autograd(P, prec):
    """Gradients of a weighted sum through the layer: g_xi_in and g_bvals (summed over the
    problem's samples, in a fixed order, so two runs agree bit for bit) against autograd
    through the oracle."""
    cfg, xi, bv = decoder_like(16, 200, 10, seed=71)
    dt = torch.float64 if prec == "fp64" else torch.float32
    sf = P.SafetyFilter([cfg])
    rng = np.random.default_rng(72)
    wts = rng.normal(size=xi.shape)
    x = torch.as_tensor(xi, dtype=dt).cuda().requires_grad_(True)
    b = torch.as_tensor(bv, dtype=dt).cuda().requires_grad_(True)
    _say(f"case qp_equality backward {prec}")
    y = P.qp_equality_differentiable(sf, x, b, precision=prec)
    (y * torch.as_tensor(wts, dtype=dt).cuda()).sum().backward()
    gx1, gb1 = x.grad.clone(), b.grad.clone()
    x.grad = None
    b.grad = None
    y = P.qp_equality_differentiable(sf, x, b, precision=prec)
    (y * torch.as_tensor(wts, dtype=dt).cuda()).sum().backward()
    assert torch.equal(gb1, b.grad) and torch.equal(gx1, x.grad)
    xo = torch.as_tensor(xi).requires_grad_(True)
    bo = torch.as_tensor(bv).requires_grad_(True)
    (O.qp_equality(O.build_system(cfg), xo, bo) * torch.as_tensor(wts)).sum().backward()
    tol = 1e-12 if prec == "fp64" else 2e-5
    assert ((gx1.cpu().double() - xo.grad).abs().max() / xo.grad.abs().max()).item() <= tol
    assert ((gb1.cpu().double() - bo.grad).abs().max() / bo.grad.abs().max()).item() <= tol


def test_reverse_mode_optional_outputs(P):
    cfg, xi, bv = decoder_like(5, 3, 10, seed=81)
    sf = P.SafetyFilter([cfg])
    import ctypes
    from paper_2501_19042_amd import _native as N
    g = torch.ones(xi.shape, dtype=torch.float64).cuda()
    batch = sf._batch(None, g)
    # only g_bvals, then only g_xi_in (in place on g_out)
    gb = torch.empty(bv.shape, dtype=torch.float64).cuda()
    N.check(N.lib().sf_qp_equality_backward(sf._h, ctypes.byref(batch.c), N.SF_FP64, g.data_ptr(), None,
                                            gb.data_ptr(), None))
    N.check(N.lib().sf_qp_equality_backward(sf._h, ctypes.byref(batch.c), N.SF_FP64, g.data_ptr(), g.data_ptr(),
                                            None, None))
    torch.cuda.synchronize()
    assert (g[..., :3] == 0).all() and (g[..., -3:] == 0).all() and (g[..., 3:-3] == 1).all()
    xo = torch.as_tensor(xi).requires_grad_(True)
    bo = torch.as_tensor(bv).requires_grad_(True)
    O.qp_equality(O.build_system(cfg), xo, bo).sum().backward()
    assert torch.allclose(gb.cpu(), bo.grad, atol=1e-12, rtol=1e-12)
    with pytest.raises(N.SfError):
        N.check(N.lib().sf_qp_equality_backward(sf._h, ctypes.byref(batch.c), N.SF_FP64, None, None, None, None))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_largest_shape(P, prec):
    """64 robots, degree 30 (31 coefficients, an odd row length), 20 samples: forward and reverse
    mode against the oracle."""
    p = W.small3d(n_robots=64, n_samples=20, degree=30, horizon=45, seed=90,
                  box=((-4.0, -4.0, -1.0), (4.0, 4.0, 1.0)))
    rng = np.random.default_rng(91)
    xi = p.xi_bar + rng.normal(size=p.xi_bar.shape) * 0.3
    wts = rng.normal(size=xi.shape)
    dt = torch.float64 if prec == "fp64" else torch.float32
    sf = P.SafetyFilter([p.cfg])
    x = torch.as_tensor(xi, dtype=dt).cuda().requires_grad_(True)
    b = torch.as_tensor(p.bvals, dtype=dt).cuda().requires_grad_(True)
    _say(f"case qp_equality largest shape {prec} n=64 degree=30 S=20")
    y = P.qp_equality_differentiable(sf, x, b, precision=prec)
    (y * torch.as_tensor(wts, dtype=dt).cuda()).sum().backward()
    torch.cuda.synchronize()
    xo = torch.as_tensor(xi).requires_grad_(True)
    bo = torch.as_tensor(p.bvals).requires_grad_(True)
    ref = O.qp_equality(O.build_system(p.cfg), xo, bo)
    (ref * torch.as_tensor(wts)).sum().backward()
    got = y.detach().cpu().double()
    ref = ref.detach()
    if prec == "fp64":
        assert ((got - ref).abs() / (1 + ref.abs())).max().item() <= 1e-12
    else:
        rel = (got - ref).abs().reshape(20, -1).amax(1) / ref.abs().reshape(20, -1).amax(1)
        assert rel.max().item() <= 1e-6, rel
    assert torch.equal(y.detach()[..., 3:-3].cpu(), x.detach()[..., 3:-3].cpu())
    tol = 1e-12 if prec == "fp64" else 2e-5
    assert ((x.grad.cpu().double() - xo.grad).abs().max() / xo.grad.abs().max()).item() <= tol
    assert ((b.grad.cpu().double() - bo.grad).abs().max() / bo.grad.abs().max()).item() <= tol
