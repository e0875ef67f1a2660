"""GPU parity of the HIP safety filter against the FP64 oracle, through the C ABI.

Tolerances: FP64 elementwise |gpu - oracle| <= 1e-9 (1 + |oracle|); FP32 per sample
max|gpu - oracle| / max|oracle| <= 1e-4 on the coefficients.
"""
import math
import sys

import numpy as np
import pytest
import torch

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-9
FP32_TOL = 1e-4


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def lib():
    from paper_2501_19042_amd import SafetyFilter, Batch  # noqa: F401
    import paper_2501_19042_amd as P
    torch.cuda.set_device(0)
    return P


def run_oracle(cfg, xi_bar, bvals, iters, xi0=None, lam0=None, record=False):
    s = O.build_system(cfg)
    t = lambda a: None if a is None else torch.as_tensor(a, dtype=torch.float64)
    return O.sf_project(s, t(xi_bar), t(bvals), iters, xi0=t(xi0), lam0=t(lam0), record=record)


def assert_fp64(gpu, ref, what):
    g = gpu.detach().cpu().double()
    err = ((g - ref).abs() / (1.0 + ref.abs())).max().item()
    assert err <= FP64_TOL, f"{what}: FP64 error {err:.3e}"
    return err


def per_sample_rel(gpu, ref):
    g = gpu.detach().cpu().double().reshape(gpu.shape[0], -1)
    r = ref.reshape(ref.shape[0], -1)
    return ((g - r).abs().amax(1) / r.abs().amax(1)).numpy()


def gpu_run(P, cfg, xi_bar, bvals, iters, precision, **kw):
    dt = torch.float64 if precision == "fp64" else torch.float32
    sf = P.SafetyFilter([cfg])
    xb = torch.as_tensor(xi_bar, dtype=dt).cuda().contiguous()
    bv = torch.as_tensor(bvals, dtype=dt).cuda().contiguous()
    for k in ("xi0", "lam0"):
        if kw.get(k) is not None:
            kw[k] = torch.as_tensor(kw[k], dtype=dt).cuda().contiguous()
    out = sf.project(xb, bv, iters, precision=precision, **kw)
    torch.cuda.synchronize()
    return out


# ----------------------------------------------------------------------------------
# FP64: the generic kernel against the oracle
# ----------------------------------------------------------------------------------

def test_fp64_tiny2d_matches_oracle(lib):
    wl = W.tiny2d()
    p = wl.problems[0]
    _say(f"case tiny2d fp64 S={p.xi_bar.shape[0]} iters={wl.iters}")
    out = gpu_run(lib, p.cfg, p.xi_bar, p.bvals, wl.iters, "fp64")
    rx, rl, rr = run_oracle(p.cfg, p.xi_bar, p.bvals, wl.iters)
    assert_fp64(out.xi, rx, "xi")
    assert_fp64(out.lam, rl, "lambda")
    res = out.resid.cpu()
    assert torch.allclose(res, rr, rtol=1e-7, atol=1e-12)


def test_fp64_small3d_tiles_tail_and_warm_start(lib):
    p = W.small3d(n_robots=5, n_samples=6, horizon=40)          # tile 32 + ragged tail 8
    rng = np.random.default_rng(3)
    xi0 = p.xi_bar + rng.normal(size=p.xi_bar.shape) * 0.05
    lam0 = rng.normal(size=p.xi_bar.shape) * 0.1
    _say("case small3d fp64 n=5 H=40 warm start")
    out = gpu_run(lib, p.cfg, p.xi_bar, p.bvals, 60, "fp64", xi0=xi0, lam0=lam0)
    rx, rl, rr = run_oracle(p.cfg, p.xi_bar, p.bvals, 60, xi0=xi0, lam0=lam0)
    assert_fp64(out.xi, rx, "xi")
    assert_fp64(out.lam, rl, "lambda")
    assert torch.allclose(out.resid.cpu(), rr, rtol=1e-7, atol=1e-12)


def test_fp64_history_and_checkpoints(lib):
    p = W.small3d(n_robots=4, n_samples=3, horizon=33, seed=12)
    iters, ce = 25, 10
    _say("case history+ckpt fp64")
    out = gpu_run(lib, p.cfg, p.xi_bar, p.bvals, iters, "fp64", history=True, ckpt_every=ce)
    _, _, hist = run_oracle(p.cfg, p.xi_bar, p.bvals, iters, record=True)
    assert out.resid.shape == (3, iters, 2)
    assert torch.allclose(out.resid.cpu(), hist, rtol=1e-7, atol=1e-12)
    ck = out.ckpt.cpu()
    assert ck.shape[0] == math.ceil(iters / ce)
    for j in range(ck.shape[0]):
        k = j * ce
        if k == 0:
            rx = torch.as_tensor(p.xi_bar)
            rl = torch.zeros_like(rx)
        else:
            rx, rl, _ = run_oracle(p.cfg, p.xi_bar, p.bvals, k)
        assert_fp64(ck[j, 0].reshape(rx.shape), rx, f"ckpt xi {k}")
        assert_fp64(ck[j, 1].reshape(rx.shape), rl, f"ckpt lambda {k}")


@pytest.mark.parametrize("D", [2, 3])
def test_fp64_coincident_robots_tie_break(lib, D):
    # robots 0 and 1 rest at the origin (all coefficients exactly 0), so r = 0 exactly at every
    # time in any summation order and the atan2(0, 0) tie-break decides the first push
    cfg = W.SwarmConfig(n_robots=3, dims=D, degree=8, horizon=20, t_final=5.0, safety_a=0.3, safety_b=0.3,
                        vmax=1.5, amax=2.0)
    st = np.zeros((3, D)); gl = np.zeros((3, D))
    st[2, :2] = (1.0, 1.0); gl[2, :2] = (-1.0, 1.0)
    xi = W.straight_line_coeffs(st, gl, 8)[None]
    b = W.boundary_values(st, gl)
    _say(f"case coincident fp64 D={D}")
    out = gpu_run(lib, cfg, xi, b, 30, "fp64")
    rx, rl, _ = run_oracle(cfg, xi, b, 30)
    assert_fp64(out.xi, rx, "xi")
    # The two robots also share their pinned start and end points, where no iterate can move
    # them apart: there the oracle's r is LU rounding noise (~1e-17) and the target direction
    # is not unique.  Those rows touch only the pinned coefficients (basis weight 0 elsewhere),
    # so xi and the free multipliers are unique and compared; the pinned multipliers are not.
    assert_fp64(out.lam[..., 3:-3], rl[..., 3:-3], "lambda (free coefficients)")
    # the pair separated along the tie-break axis (z in 3D, x in 2D): X_0 - X_1 moves
    # towards the target (0, 0, b) or (a, 0), so robot 0 goes up that axis
    ax = 2 if D == 3 else 0
    assert (rx[0, 0, ax, 3:-3] > 0).all() and (rx[0, 1, ax, 3:-3] < 0).all()


@pytest.mark.parametrize("degree,n,D", [(5, 2, 3), (6, 2, 2), (12, 3, 3)])
def test_fp64_degenerate_shapes(lib, degree, n, D):
    cfg = W.SwarmConfig(n_robots=n, dims=D, degree=degree, horizon=degree + 4, t_final=3.0,
                        safety_a=0.3, safety_b=0.3, vmax=1.5, amax=2.0)
    rng = np.random.default_rng(degree * 10 + n)
    st = rng.uniform(-0.4, 0.4, size=(n, D))
    gl = rng.uniform(-0.4, 0.4, size=(n, D))    # not antipodal: no exact mid-course coincidence
    xi = W.sample_coeffs(rng, st, gl, degree, 2, 0.3)
    b = W.boundary_values(st, gl)
    _say(f"case degenerate degree={degree} n={n} D={D}")
    out = gpu_run(lib, cfg, xi, b, 20, "fp64")
    rx, rl, rr = run_oracle(cfg, xi, b, 20)
    assert_fp64(out.xi, rx, "xi")
    assert_fp64(out.lam, rl, "lambda")


def test_zero_iterations_returns_initial_state(lib):
    p = W.small3d(n_robots=3, n_samples=2, horizon=12)
    rng = np.random.default_rng(1)
    lam0 = rng.normal(size=p.xi_bar.shape)
    for prec in ("fp64", "fp32"):
        out = gpu_run(lib, p.cfg, p.xi_bar, p.bvals, 0, prec, lam0=lam0)
        dt = torch.float64 if prec == "fp64" else torch.float32
        assert torch.equal(out.xi.cpu(), torch.as_tensor(p.xi_bar, dtype=dt))
        assert torch.equal(out.lam.cpu(), torch.as_tensor(lam0, dtype=dt))
        assert (out.resid.cpu() == 0).all()


def test_feasibility_check_matches_oracle(lib):
    wl = W.tiny2d()
    p = wl.problems[0]
    xb = torch.as_tensor(p.xi_bar).cuda()
    bv = torch.as_tensor(p.bvals).cuda()
    sf = lib.SafetyFilter([p.cfg])
    out = sf.project(xb, bv, 100, precision="fp64")
    v = sf.feasibility(out.xi, bv, precision="fp64").cpu()
    s = O.build_system(p.cfg)
    ref = O.feasibility(s, out.xi.cpu(), bv.cpu())
    assert torch.allclose(v, ref, atol=1e-12, rtol=1e-10)
    v0 = sf.feasibility(xb, bv, precision="fp64").cpu()
    assert torch.allclose(v0, O.feasibility(s, xb.cpu(), bv.cpu()), atol=1e-12, rtol=1e-10)


# ----------------------------------------------------------------------------------
# FP32
# ----------------------------------------------------------------------------------

def test_fp32_tiny2d(lib):
    wl = W.tiny2d()
    p = wl.problems[0]
    _say("case tiny2d fp32")
    out = gpu_run(lib, p.cfg, p.xi_bar, p.bvals, wl.iters, "fp32")
    rx, _, _ = run_oracle(p.cfg, p.xi_bar, p.bvals, wl.iters)
    err = per_sample_rel(out.xi, rx)
    assert err.max() <= FP32_TOL, err


def test_fp32_small3d(lib):
    p = W.small3d(n_robots=6, n_samples=8, horizon=45)
    _say("case small3d fp32")
    for k in (10, 50, 150):
        out = gpu_run(lib, p.cfg, p.xi_bar, p.bvals, k, "fp32")
        rx, _, _ = run_oracle(p.cfg, p.xi_bar, p.bvals, k)
        err = per_sample_rel(out.xi, rx)
        assert err.max() <= FP32_TOL, (k, err)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_zero_initialisation_matches_oracle(lib, prec):
    """xi0 = 0, lambda0 = 0 (the zero warm start of the study): the first step's correction then
    carries the whole boundary jump."""
    p = W.small3d(n_robots=6, n_samples=4, horizon=45, seed=17)
    z = np.zeros_like(p.xi_bar)
    for k in (1, 40):
        _say(f"case zero init {prec} k={k}")
        out = gpu_run(lib, p.cfg, p.xi_bar, p.bvals, k, prec, xi0=z, lam0=z)
        rx, rl, _ = run_oracle(p.cfg, p.xi_bar, p.bvals, k, xi0=z, lam0=z)
        if prec == "fp64":
            assert_fp64(out.xi, rx, "xi")
            assert_fp64(out.lam, rl, "lambda")
        else:
            err = per_sample_rel(out.xi, rx)
            assert err.max() <= FP32_TOL, (k, err)


def test_ragged_batch_equals_separate_calls(lib):
    P = lib
    probs = [W.small3d(n_robots=n, n_samples=s, horizon=30, seed=20 + n) for n, s in ((3, 2), (5, 3), (4, 1))]
    cfgs = [p.cfg for p in probs]
    for prec, dt in (("fp64", torch.float64), ("fp32", torch.float32)):
        sf = P.SafetyFilter(cfgs)
        batch = P.Batch([(i, p.xi_bar.shape[0]) for i, p in enumerate(probs)])
        xb = torch.cat([torch.as_tensor(p.xi_bar, dtype=dt).reshape(-1) for p in probs]).cuda()
        bv = torch.cat([torch.as_tensor(p.bvals, dtype=dt).reshape(-1) for p in probs]).cuda()
        out = sf.project(xb, bv, 30, batch=batch, precision=prec, generic=True)
        torch.cuda.synchronize()
        o = 0
        r0 = 0
        for i, p in enumerate(probs):
            single = gpu_run(P, p.cfg, p.xi_bar, p.bvals, 30, prec, generic=True)
            nel = p.xi_bar.size
            assert torch.equal(out.xi[o:o + nel].cpu(), single.xi.reshape(-1).cpu())
            S = p.xi_bar.shape[0]
            assert torch.equal(out.resid[r0:r0 + S].cpu(), single.resid.cpu())
            o += nel
            r0 += S


def test_deterministic(lib):
    p = W.small3d(n_robots=5, n_samples=4, horizon=30)
    a = gpu_run(lib, p.cfg, p.xi_bar, p.bvals, 40, "fp32")
    b = gpu_run(lib, p.cfg, p.xi_bar, p.bvals, 40, "fp32")
    assert torch.equal(a.xi, b.xi) and torch.equal(a.lam, b.lam) and torch.equal(a.resid, b.resid)


def test_fp32_swarm16_full_size_sampled(lib):
    """Full 16-robot workload (1024 samples, 300 iterations) in the configuration the
    benchmark times; sampled outputs against the oracle, strict at k = 10 and 50."""
    wl = W.swarm16()
    p = wl.problems[0]
    idx = [0, 311, 1023]
    for k in (10, 50, wl.iters):
        _say(f"case swarm16 fp32 full size k={k}")
        out = gpu_run(lib, p.cfg, p.xi_bar, p.bvals, k, "fp32")
        rx, _, _ = run_oracle(p.cfg, p.xi_bar[idx], p.bvals, k)
        err = per_sample_rel(out.xi[idx], rx)
        assert err.max() <= FP32_TOL, (k, err)
        assert torch.isfinite(out.xi).all()


def test_errors_surface_as_exceptions(lib):
    P = lib
    p = W.small3d(n_robots=3, n_samples=2, horizon=12)
    sf = P.SafetyFilter([p.cfg])
    xb = torch.as_tensor(p.xi_bar, dtype=torch.float32).cuda()
    bv = torch.as_tensor(p.bvals, dtype=torch.float32).cuda()
    with pytest.raises(ValueError):
        sf.project(xb.double(), bv, 5, precision="fp32")
    from paper_2501_19042_amd._native import SfError
    with pytest.raises(SfError):
        sf.project_backward(xb, bv, 5, None, 0)


def test_flag_combinations_are_checked(lib):
    """SF_FP_RESIDUAL needs resid_out and excludes SF_RESID_HISTORY; unknown flags are refused; the
    fixed-point residual column matches across precisions of the generic kernel."""
    import ctypes
    from paper_2501_19042_amd import _native as N
    P = lib
    p = W.small3d(n_robots=3, n_samples=2, horizon=12)
    sf = P.SafetyFilter([p.cfg])
    xb = torch.as_tensor(p.xi_bar, dtype=torch.float64).cuda()
    bv = torch.as_tensor(p.bvals, dtype=torch.float64).cuda()
    out = torch.empty_like(xb)
    res = torch.empty((2, 3), dtype=torch.float64).cuda()
    batch = sf._batch(None, xb)
    call = lambda flags, r: N.lib().sf_project(sf._h, ctypes.byref(batch.c), N.SF_FP64, xb.data_ptr(), bv.data_ptr(),
                                               None, None, 5, out.data_ptr(), None, r, None, flags, None, 0, None)
    assert call(N.SF_FP_RESIDUAL, None) == N.SF_EINVAL
    assert call(N.SF_FP_RESIDUAL | N.SF_RESID_HISTORY, res.data_ptr()) == N.SF_EINVAL
    assert call(1 << 20, res.data_ptr()) == N.SF_EINVAL
    assert call(N.SF_FP_RESIDUAL, res.data_ptr()) == N.SF_OK
    torch.cuda.synchronize()
    r32 = sf.project(xb.float(), bv.float(), 5, precision="fp32", fp_residual=True).resid.cpu().double()
    assert torch.allclose(res.cpu()[:, 2], r32[:, 2], rtol=1e-4)
    assert (res.cpu()[:, 2] > 0).all()


def test_empty_batches_are_refused(lib):
    """A batch without problems, or with a problem of zero samples, is an SF_EINVAL error on every
    entry point (checked before any launch); the Python layer refuses an empty problem table."""
    import ctypes
    from paper_2501_19042_amd import _native as N
    P = lib
    p = W.small3d(n_robots=3, n_samples=2, horizon=12)
    sf = P.SafetyFilter([p.cfg])
    xb = torch.as_tensor(p.xi_bar, dtype=torch.float64).cuda()
    bv = torch.as_tensor(p.bvals, dtype=torch.float64).cuda()
    out = torch.empty_like(xb)
    viol = torch.empty((2, 5), dtype=torch.float64).cuda()
    gb = torch.empty_like(bv)
    slots = (ctypes.c_int32 * 1)(0)
    zero = (ctypes.c_int32 * 1)(0)
    two = (ctypes.c_int32 * 1)(2)
    as_p = lambda a: ctypes.cast(a, ctypes.POINTER(ctypes.c_int32))
    L = N.lib()
    _say("case empty batches")
    for b in (N.SfBatch(0, as_p(slots), as_p(two)), N.SfBatch(1, as_p(slots), as_p(zero))):
        assert L.sf_project(sf._h, ctypes.byref(b), N.SF_FP64, xb.data_ptr(), bv.data_ptr(), None, None, 5,
                            out.data_ptr(), None, None, None, 0, None, 0, None) == N.SF_EINVAL
        assert len(L.sf_last_error()) > 0
        assert L.sf_feasibility(sf._h, ctypes.byref(b), N.SF_FP64, xb.data_ptr(), bv.data_ptr(),
                                viol.data_ptr(), None) == N.SF_EINVAL
        assert L.sf_qp_equality(sf._h, ctypes.byref(b), N.SF_FP64, xb.data_ptr(), bv.data_ptr(),
                                out.data_ptr(), None) == N.SF_EINVAL
        assert L.sf_qp_equality_backward(sf._h, ctypes.byref(b), N.SF_FP64, xb.data_ptr(), None,
                                         gb.data_ptr(), None) == N.SF_EINVAL
    with pytest.raises(ValueError):
        P.Batch([])
    with pytest.raises(N.SfError):
        sf.project(xb[:0], bv, 5, precision="fp64")
    # the handle still works after the refusals
    good = sf.project(xb, bv, 5, precision="fp64")
    torch.cuda.synchronize()
    rx, _, _ = run_oracle(p.cfg, p.xi_bar, p.bvals, 5)
    assert_fp64(good.xi, rx, "xi")


def test_symmetric_head_on_keeps_its_symmetry_on_the_gpu(lib):
    """The exactly symmetric 2-robot head-on (2D, generic kernel, FP64; and its 3D lift on the MFMA
    kernel in fp32): the output keeps x_2 = -x_1 and stays on the line, and matches the oracle."""
    cfg = W.SwarmConfig(n_robots=2, dims=2, degree=7, horizon=16, t_final=4.0, safety_a=0.3,
                        safety_b=0.3, vmax=3.0, amax=6.0)
    st = np.array([[-1.0, 0.0], [1.0, 0.0]])
    xi_bar = W.straight_line_coeffs(st, -st, cfg.degree)[None]
    b = W.boundary_values(st, -st)
    _say("case symmetric head-on fp64 generic")
    out = gpu_run(lib, cfg, xi_bar, b, 200, "fp64")
    x = out.xi.cpu().double()[0]
    assert (x[0] + x[1]).abs().max().item() < 1e-12
    assert x[:, 1].abs().max().item() < 1e-12
    rx, _, _ = run_oracle(cfg, xi_bar, b, 200)
    assert_fp64(out.xi, rx, "symmetric head-on")
    # 3D, MFMA kernel: the same pair in the plane z = 0
    cfg3 = W.SwarmConfig(n_robots=2, dims=3, degree=7, horizon=16, t_final=4.0, safety_a=0.3,
                         safety_b=0.3, vmax=3.0, amax=6.0)
    st3 = np.array([[-1.0, 0.0, 0.0], [1.0, 0.0, 0.0]])
    xi3 = W.straight_line_coeffs(st3, -st3, cfg3.degree)[None]
    b3 = W.boundary_values(st3, -st3)
    _say("case symmetric head-on fp32 mfma")
    o3 = gpu_run(lib, cfg3, xi3, b3, 200, "fp32")
    x3 = o3.xi.cpu().double()[0]
    assert (x3[0] + x3[1]).abs().max().item() < 1e-6
    assert x3[:, 1:].abs().max().item() < 1e-6
    r3, _, _ = run_oracle(cfg3, xi3, b3, 200)
    assert per_sample_rel(o3.xi, r3).max() <= FP32_TOL
