"""Per-sample status as data: NaN and infinite inputs, infeasible problems and non-convergence are
reported in status_out (and the outputs of a sample with a non-finite input are NaN), while every
other sample of the batch is computed exactly as without the flagged ones."""
from dataclasses import replace

import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu

NF_IN, NF, NOT_CONV = 1, 2, 4
KERNELS = [("fp32", False), ("bf16", False), ("fp32", True), ("fp64", True)]


@pytest.fixture(scope="module")
def P():
    import paper_2501_19042_amd as P
    torch.cuda.set_device(0)
    return P


def _say(msg):
    print(msg, flush=True)


def problem():
    return W.small3d(n_robots=16, n_samples=8, degree=10, horizon=100, seed=77,
                     box=((-3.0, -3.0, -1.0), (3.0, 3.0, 1.0)), t_final=10.0)


@pytest.mark.parametrize("prec,generic", KERNELS)
def test_nonfinite_inputs_are_flagged_and_isolated(P, prec, generic):
    p = problem()
    dt = torch.float64 if prec == "fp64" else torch.float32
    sf = P.SafetyFilter([p.cfg])
    clean = torch.tensor(p.xi_bar, dtype=dt).cuda()
    bv = torch.tensor(p.bvals, dtype=dt).cuda()
    xb = clean.clone()
    xb[2, 3, 1, 5] = float("nan")
    xb[5, 0, 2, 0] = float("inf")
    lam0 = torch.zeros_like(xb)
    lam0[6, 9, 0, 4] = -float("inf")
    _say(f"case status nonfinite inputs {prec} generic={generic}")
    iters = 60
    ref = sf.project(clean, bv, iters, precision=prec, generic=generic, want_status=True)
    out = sf.project(xb, bv, iters, precision=prec, generic=generic, lam0=lam0, want_status=True)
    torch.cuda.synchronize()
    st = out.status.cpu().numpy()
    bad = [2, 5, 6]
    assert (st[bad] == NF_IN).all(), st
    for s in bad:
        assert torch.isnan(out.xi[s]).all() and torch.isnan(out.lam[s]).all() and torch.isnan(out.resid[s]).all()
    good = [s for s in range(8) if s not in bad]
    assert torch.equal(out.xi[good], ref.xi[good]) and torch.equal(out.lam[good], ref.lam[good])
    assert torch.equal(out.resid[good], ref.resid[good])
    assert (st[good] == ref.status.cpu().numpy()[good]).all()
    # the convergence bit follows the final residual's largest block norm, judged in the kernel's precision
    r = ref.resid[:, 1].cpu()
    conv = (r <= torch.tensor(1e-3, dtype=r.dtype)).numpy()
    assert ((ref.status.cpu().numpy() & NOT_CONV) == 0).tolist() == conv.tolist()
    assert (ref.status.cpu().numpy() & (NF | NF_IN) == 0).all()


@pytest.mark.parametrize("prec,generic", KERNELS)
def test_nonfinite_boundary_values_flag_their_problem(P, prec, generic):
    p = problem()
    q = W.small3d(n_robots=16, n_samples=3, degree=10, horizon=100, seed=78,
                  box=((-3.0, -3.0, -1.0), (3.0, 3.0, 1.0)), t_final=10.0)
    dt = torch.float64 if prec == "fp64" else torch.float32
    sf = P.SafetyFilter([p.cfg])
    batch = P.Batch([(0, 8), (0, 3)])
    xb = torch.cat([torch.tensor(p.xi_bar, dtype=dt).reshape(-1), torch.tensor(q.xi_bar, dtype=dt).reshape(-1)]).cuda()
    bq = torch.tensor(q.bvals, dtype=dt)
    bq[4, 1, 3] = float("nan")
    bv = torch.cat([torch.tensor(p.bvals, dtype=dt).reshape(-1), bq.reshape(-1)]).cuda()
    _say(f"case status nonfinite boundary values {prec} generic={generic}")
    out = sf.project(xb, bv, 30, batch=batch, precision=prec, generic=generic, want_status=True)
    solo = sf.project(xb[:p.xi_bar.size].reshape(p.xi_bar.shape), bv[:p.bvals.size], 30, precision=prec,
                      generic=generic, want_status=True)
    torch.cuda.synchronize()
    st = out.status.cpu().numpy()
    assert (st[8:] == NF_IN).all() and (st[:8] & NF_IN == 0).all(), st
    assert torch.isnan(out.xi[p.xi_bar.size:]).all()
    assert torch.equal(out.xi[:p.xi_bar.size], solo.xi.reshape(-1))
    assert (st[:8] == solo.status.cpu().numpy()).all()


@pytest.mark.parametrize("prec,generic", KERNELS)
def test_infeasible_problem_reports_non_convergence(P, prec, generic):
    """A problem whose speed bound cannot reach its goals in time (vmax 0.05 m/s for goals metres
    away over 10 s) keeps the not-converged bit; a feasible problem in the same batch is solved
    as on its own."""
    p = problem()
    slow = replace(p.cfg, vmax=0.05)
    dt = torch.float64 if prec == "fp64" else torch.float32
    sf = P.SafetyFilter([p.cfg, slow])
    batch = P.Batch([(0, 8), (1, 4)])
    x = torch.tensor(p.xi_bar, dtype=dt)
    xb = torch.cat([x.reshape(-1), x[:4].reshape(-1)]).cuda()
    b = torch.tensor(p.bvals, dtype=dt).reshape(-1)
    bv = torch.cat([b, b]).cuda()
    _say(f"case status infeasible problem {prec} generic={generic}")
    out = sf.project(xb, bv, 200, batch=batch, precision=prec, generic=generic, want_status=True)
    solo = P.SafetyFilter([p.cfg]).project(x.cuda(), b.cuda(), 200, precision=prec, generic=generic,
                                           want_status=True)
    torch.cuda.synchronize()
    st = out.status.cpu().numpy()
    assert (st[8:] == NOT_CONV).all(), st
    assert torch.isfinite(out.xi).all()
    assert torch.equal(out.xi[:x.numel()], solo.xi.reshape(-1))
    assert (st[:8] == solo.status.cpu().numpy()).all()
    viol = sf.feasibility(out.xi, bv, batch=batch, precision=prec).cpu()
    assert (viol[8:, 1] > 1e-2).all()      # the speed bound stays violated


@pytest.mark.parametrize("prec,generic", KERNELS)
def test_status_without_residual_output(P, prec, generic):
    """status_out alone (resid_out NULL) runs the final residual pass for the convergence bit and
    gives the same bits and iterates as with resid_out."""
    p = problem()
    dt = torch.float64 if prec == "fp64" else torch.float32
    sf = P.SafetyFilter([p.cfg])
    xb = torch.tensor(p.xi_bar, dtype=dt).cuda()
    bv = torch.tensor(p.bvals, dtype=dt).cuda()
    a = sf.project(xb, bv, 80, precision=prec, generic=generic, want_status=True)
    b = sf.project(xb, bv, 80, precision=prec, generic=generic, want_status=True, want_resid=False)
    torch.cuda.synchronize()
    assert b.resid is None
    assert torch.equal(a.status, b.status) and torch.equal(a.xi, b.xi)
    assert set(np.unique(a.status.cpu().numpy())) <= {0, NOT_CONV}
