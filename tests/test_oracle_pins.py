"""Pins of the FP64 oracle against facts that do not come from the oracle itself.

Each test checks the oracle against a closed form, a textbook routine, an
independent construction, brute force on a tiny input, or an invariant of the
method, so that a dropped term, a wrong sign or index, or a transposed operand
in the oracle fails at least one of them.
"""
import math
from fractions import Fraction

from dataclasses import replace

import numpy as np
import pytest
import scipy.linalg
import scipy.optimize
import torch

import oracle as O
import workloads as W

DT = torch.float64


# --------------------------------------------------------------------------
# independent helpers (not shared with the oracle)
# --------------------------------------------------------------------------

def de_casteljau(ctrl, tau):
    """Evaluate a Bernstein curve with control points ctrl[..., m] at tau by repeated
    linear interpolation (de Casteljau's algorithm)."""
    c = np.array(ctrl, dtype=np.float64)
    while c.shape[-1] > 1:
        c = (1.0 - tau) * c[..., :-1] + tau * c[..., 1:]
    return c[..., 0]


def curve_on_grid(xi, H, T):
    """Positions, velocities, accelerations of [B, n, D, m] coefficient arrays at the grid
    tau_h = h/(H-1), via de Casteljau and the hodograph (differences of control points)."""
    xi = np.asarray(xi, dtype=np.float64)
    N = xi.shape[-1] - 1
    d1 = N * np.diff(xi, axis=-1) / T
    d2 = (N - 1) * np.diff(d1, axis=-1) / T
    taus = np.arange(H) / (H - 1)
    X = np.stack([de_casteljau(xi, t) for t in taus], axis=-1)
    V = np.stack([de_casteljau(d1, t) for t in taus], axis=-1)
    A = np.stack([de_casteljau(d2, t) for t in taus], axis=-1)
    return X, V, A


def independent_F(n, P, Pd, Pdd, vel=True, acc=True, ws=False):
    """One axis block of F built row by row: pair (i<j) rows are P at robot i and -P at
    robot j; then velocity and acceleration rows per robot; then (ws) position rows per
    robot for the workspace (the F_w block of eq. (f_e))."""
    H, m = P.shape
    rows = []
    for i in range(n):
        for j in range(i + 1, n):
            blk = np.zeros((H, n * m))
            blk[:, i * m:(i + 1) * m] = P
            blk[:, j * m:(j + 1) * m] = -P
            rows.append(blk)
    for on, M in ((vel, Pd), (acc, Pdd), (ws, P)):
        if on:
            for i in range(n):
                blk = np.zeros((H, n * m))
                blk[:, i * m:(i + 1) * m] = M
                rows.append(blk)
    return np.concatenate(rows, axis=0)


def closest_point_outside(r, a):
    """Closest point to r in {x : ||x|| >= a} (a sphere of radius a); ties at r = 0 are
    not unique and are excluded by the callers."""
    nr = np.linalg.norm(r, axis=-1, keepdims=True)
    return np.where(nr >= a, r, a * r / nr)


def closest_point_inside(v, R):
    nv = np.linalg.norm(v, axis=-1, keepdims=True)
    return np.where(nv <= R, v, R * v / np.maximum(nv, 1e-300))


def small_cfg(n=3, D=3, degree=7, H=12, T=4.0, a=0.3, vmax=1.5, amax=2.0, rho=(1.0, 1.0, 1.0),
              ws=(0.0, 0.0), rho_ws=1.0, ws_c=(0.0, 0.0, 0.0)):
    return W.SwarmConfig(n_robots=n, dims=D, degree=degree, horizon=H, t_final=T,
                         safety_a=a, safety_b=a, vmax=vmax, amax=amax,
                         rho_coll=rho[0], rho_vel=rho[1], rho_acc=rho[2],
                         ws_a=ws[0], ws_b=ws[1], rho_ws=rho_ws, ws_x=ws_c[0], ws_y=ws_c[1], ws_z=ws_c[2])


# --------------------------------------------------------------------------
# Basis, eq. (poly)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("N,H,T", [(10, 100, 5.0), (12, 120, 10.0), (5, 7, 1.0)])
def test_bernstein_partition_endpoints_and_exact_values(N, H, T):
    P, Pd, Pdd = O.basis_matrices(N, H, T)
    assert torch.allclose(P.sum(1), torch.ones(H, dtype=DT), atol=1e-14)
    assert torch.allclose(Pd.sum(1), torch.zeros(H, dtype=DT), atol=1e-12)
    assert torch.allclose(Pdd.sum(1), torch.zeros(H, dtype=DT), atol=1e-11)
    e0 = torch.zeros(N + 1, dtype=DT); e0[0] = 1
    eN = torch.zeros(N + 1, dtype=DT); eN[N] = 1
    assert torch.equal(P[0], e0) and torch.equal(P[H - 1], eN)
    # endpoint derivatives: p'(0) = N (c1 - c0)/T, p''(0) = N (N-1)(c2 - 2 c1 + c0)/T^2
    d0 = torch.zeros(N + 1, dtype=DT); d0[0], d0[1] = -N / T, N / T
    dd0 = torch.zeros(N + 1, dtype=DT)
    dd0[0], dd0[1], dd0[2] = N * (N - 1) / T**2, -2 * N * (N - 1) / T**2, N * (N - 1) / T**2
    assert torch.allclose(Pd[0], d0, atol=1e-12)
    assert torch.allclose(Pdd[0], dd0, atol=1e-11)
    # mirror symmetry B_{N,k}(tau) = B_{N,N-k}(1 - tau); derivative rows flip sign once
    assert torch.allclose(P.flip(0), P.flip(1), atol=1e-14)
    assert torch.allclose(Pd.flip(0), -Pd.flip(1), atol=1e-12)
    assert torch.allclose(Pdd.flip(0), Pdd.flip(1), atol=1e-10)


def test_bernstein_matches_exact_rational_values():
    # B_{N,k}(p/q) computed with exact fractions
    N = 10
    for tau in (Fraction(1, 3), Fraction(1, 2), Fraction(7, 9)):
        got = O.bernstein(N, torch.tensor([float(tau)], dtype=DT))[0]
        for k in range(N + 1):
            exact = math.comb(N, k) * tau**k * (1 - tau)**(N - k)
            assert abs(float(exact) - got[k].item()) < 1e-15


@pytest.mark.parametrize("N", [6, 10, 12])
def test_basis_agrees_with_de_casteljau_and_finite_differences(N):
    H, T = 23, 3.0
    P, Pd, Pdd = O.basis_matrices(N, H, T)
    rng = np.random.default_rng(0)
    c = rng.normal(size=(4, N + 1))
    X, V, A = curve_on_grid(c[None, :, None, :], H, T)
    assert np.allclose(c @ P.numpy().T, X[0, :, 0], atol=1e-13)
    assert np.allclose(c @ Pd.numpy().T, V[0, :, 0], atol=1e-12)
    assert np.allclose(c @ Pdd.numpy().T, A[0, :, 0], atol=1e-11)
    # central differences in time of the position curve, at interior grid points
    h = 1e-4
    for hh in (3, 11, 19):
        t = hh / (H - 1)
        fp = de_casteljau(c, t + h / T)
        fm = de_casteljau(c, t - h / T)
        f0 = de_casteljau(c, t)
        assert np.allclose((fp - fm) / (2 * h), c @ Pd[hh].numpy(), rtol=1e-6, atol=1e-7)
        assert np.allclose((fp - 2 * f0 + fm) / h**2, c @ Pdd[hh].numpy(), rtol=1e-4, atol=1e-4)


# --------------------------------------------------------------------------
# F and the pair incidence (Appendix, F_o and F_{o,i})
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n", [2, 3, 5, 16])
def test_pair_incidence_structure(n):
    Dp = O.pair_incidence(n)
    assert Dp.shape == (n * (n - 1) // 2, n)
    r = 0
    for i in range(n):
        for j in range(i + 1, n):
            expect = torch.zeros(n, dtype=DT); expect[i] = 1; expect[j] = -1
            assert torch.equal(Dp[r], expect)
            r += 1
    # D^T D is the Laplacian of the complete graph
    assert torch.allclose(Dp.T @ Dp, n * torch.eye(n, dtype=DT) - torch.ones(n, n, dtype=DT))


def test_F_matches_row_by_row_construction():
    cfg = small_cfg(n=4, D=3, degree=8, H=9)
    s = O.build_system(cfg)
    Fi = independent_F(4, s.P.numpy(), s.Pd.numpy(), s.Pdd.numpy())
    assert np.array_equal(s.F.numpy(), Fi)
    # with the workspace rows (eq. (f_e)): block diagonal P after the bound rows, weighted rho_ws
    cfg = small_cfg(n=4, D=3, degree=8, H=9, ws=(2.0, 1.0), rho_ws=0.6)
    s = O.build_system(cfg)
    Fi = independent_F(4, s.P.numpy(), s.Pd.numpy(), s.Pdd.numpy(), ws=True)
    assert np.array_equal(s.F.numpy(), Fi)
    assert np.array_equal(s.w.numpy()[-4 * 9:], np.full(4 * 9, 0.6))


# --------------------------------------------------------------------------
# alpha/beta/d steps == projection onto the constraint set (eqs. (alpha_step)-(d_step))
# --------------------------------------------------------------------------

def test_collision_target_is_closest_point_outside_sphere():
    rng = np.random.default_rng(1)
    a = 0.3
    r = rng.normal(size=(2000, 3)) * rng.uniform(0.01, 0.6, size=(2000, 1))
    e = O.project_collision(torch.tensor(r), a, a).numpy()
    assert np.allclose(e, closest_point_outside(r, a), atol=1e-14)
    r2 = rng.normal(size=(2000, 2)) * rng.uniform(0.01, 0.6, size=(2000, 1))
    e2 = O.project_collision(torch.tensor(r2), a, a).numpy()
    assert np.allclose(e2, closest_point_outside(r2, a), atol=1e-14)


def test_ball_target_is_closest_point_inside_ball():
    rng = np.random.default_rng(2)
    for D in (2, 3):
        v = rng.normal(size=(2000, D)) * 2.0
        e = O.project_ball(torch.tensor(v), 1.5).numpy()
        assert np.allclose(e, closest_point_inside(v, 1.5), atol=1e-14)


def test_collision_target_brute_force_over_angles():
    """argmin over (alpha, beta, d >= 1) of ||r - d u(alpha, beta)||^2 by a dense grid plus
    a local polish; the closed forms must reach the same minimum."""
    rng = np.random.default_rng(3)
    a = 0.3
    for _ in range(6):
        r = rng.normal(size=3) * 0.2

        def f(z):
            al, be, d = z
            d = max(d, 1.0)
            u = np.array([a * np.cos(al) * np.sin(be), a * np.sin(al) * np.sin(be), a * np.cos(be)])
            return np.sum((r - d * u) ** 2)
        best = None
        for al in np.linspace(-np.pi, np.pi, 37):
            for be in np.linspace(0, np.pi, 19):
                for d in (1.0, 1.5, 2.5):
                    v = f((al, be, d))
                    if best is None or v < best[0]:
                        best = (v, (al, be, d))
        res = scipy.optimize.minimize(f, best[1], method="Nelder-Mead",
                                      options=dict(xatol=1e-12, fatol=1e-16, maxiter=20000))
        e = O.project_collision(torch.tensor(r[None]), a, a).numpy()[0]
        assert abs(np.sum((r - e) ** 2) - res.fun) < 1e-10
        assert np.sum((r - e) ** 2) <= res.fun + 1e-14


def test_spheroid_target_is_radial_projection_in_scaled_frame():
    # reading for a != b: alpha, beta are the angles of s = M^{-1} r, and the least-squares
    # d equals ||s||, so e = M s/||s|| * max(1, ||s||).
    rng = np.random.default_rng(4)
    a, b = 0.3, 0.5
    r = rng.normal(size=(500, 3)) * 0.3
    e = O.project_collision(torch.tensor(r), a, b).numpy()
    Mi = np.array([1 / a, 1 / a, 1 / b])
    s = r * Mi
    ns = np.linalg.norm(s, axis=1, keepdims=True)
    expect = (s / ns) * np.maximum(1.0, ns) / Mi
    assert np.allclose(e, expect, atol=1e-13)


def test_workspace_target_is_radial_projection_in_scaled_frame():
    # eq. (workspace_polar) about the centre p_w: with the least-squares d = ||s||, s = M_w^{-1}
    # (p - p_w), the target is p_w + M_w s min(1, 1/||s||): points inside stay, points outside
    # are scaled back onto the spheroid along the ray from the centre in the scaled frame
    rng = np.random.default_rng(14)
    a, b = 2.0, 0.7
    c = np.array([0.5, -0.25, 0.3])
    p = c + rng.normal(size=(800, 3)) * np.array([2.0, 2.0, 0.8])
    e = O.project_workspace(torch.tensor(p), a, b, torch.tensor(c)).numpy()
    Mi = np.array([1 / a, 1 / a, 1 / b])
    s_ = (p - c) * Mi
    ns = np.linalg.norm(s_, axis=1, keepdims=True)
    expect = c + (s_ * np.minimum(1.0, 1.0 / ns)) / Mi
    assert np.allclose(e, expect, atol=1e-13)
    inside = ns[:, 0] <= 1.0
    assert inside.any() and (~inside).any()
    assert np.allclose(e[inside], p[inside], atol=1e-15)
    # on a ball (a = b) it is the closest point inside, in 2D and 3D; the centre maps to itself
    for D in (2, 3):
        q = rng.normal(size=(500, D)) * 1.5
        cc = c[:D]
        e2 = O.project_workspace(torch.tensor(cc + q), 1.2, 1.2, torch.tensor(cc)).numpy()
        assert np.allclose(e2, cc + closest_point_inside(q, 1.2), atol=1e-13)
        e0 = O.project_workspace(torch.tensor(cc[None]), 1.2, 1.2, torch.tensor(cc)).numpy()
        assert np.allclose(e0, cc[None], atol=0)


def test_coincident_robots_tie_break():
    # atan2(0, 0) = 0: alpha = beta = 0, so the target is (0, 0, b) in 3D and (a, 0) in 2D
    e3 = O.project_collision(torch.zeros(1, 3, dtype=DT), 0.3, 0.4).numpy()[0]
    assert np.array_equal(e3, [0.0, 0.0, 0.4])
    e2 = O.project_collision(torch.zeros(1, 2, dtype=DT), 0.3, 0.3).numpy()[0]
    assert np.array_equal(e2, [0.3, 0.0])
    v = O.project_ball(torch.zeros(1, 3, dtype=DT), 1.5).numpy()[0]
    assert np.array_equal(v, [0.0, 0.0, 0.0])


# --------------------------------------------------------------------------
# one full iteration against an independent implementation of the same step
# --------------------------------------------------------------------------

def _one_step_independent(cfg, xi_bar, bvals, xi0, lam0):
    """Projection by closest points, lambda step with the minus sign, and the xi step as
    an equality-constrained least squares solved on the null space of A (scipy).  A
    workspace, if any, must be a ball (a_w = b_w), whose projection is the closest point."""
    s = O.build_system(cfg)
    n, D, m, H = cfg.n_robots, cfg.dims, cfg.degree + 1, cfg.horizon
    P, Pd, Pdd = s.P.numpy(), s.Pd.numpy(), s.Pdd.numpy()
    ws = cfg.ws_a > 0
    assert not ws or cfg.ws_a == cfg.ws_b
    F = independent_F(n, P, Pd, Pdd, ws=ws)
    Np = n * (n - 1) // 2
    w = np.concatenate([np.full(Np * H, cfg.rho_coll), np.full(n * H, cfg.rho_vel), np.full(n * H, cfg.rho_acc)]
                       + ([np.full(n * H, cfg.rho_ws)] if ws else []))
    wc = np.array([cfg.ws_x, cfg.ws_y, cfg.ws_z])[:D]
    A1 = np.stack([P[0], Pd[0], Pdd[0], P[-1], Pd[-1], Pdd[-1]])
    A = np.kron(np.eye(n), A1)
    out_xi = np.zeros_like(xi0)
    out_lam = np.zeros_like(lam0)
    for bidx in range(xi0.shape[0]):
        Y = np.stack([F @ xi0[bidx, :, d, :].reshape(-1) for d in range(D)], axis=-1)  # [rows, D]
        E = np.empty_like(Y)
        E[:Np * H] = closest_point_outside(Y[:Np * H], cfg.safety_a)
        E[Np * H:Np * H + n * H] = closest_point_inside(Y[Np * H:Np * H + n * H], cfg.vmax)
        E[Np * H + n * H:Np * H + 2 * n * H] = closest_point_inside(Y[Np * H + n * H:Np * H + 2 * n * H], cfg.amax)
        if ws:
            E[Np * H + 2 * n * H:] = wc + closest_point_inside(Y[Np * H + 2 * n * H:] - wc, cfg.ws_a)
        for d in range(D):
            lam = lam0[bidx, :, d, :].reshape(-1) - F.T @ (w * (Y[:, d] - E[:, d]))
            target = xi_bar[bidx, :, d, :].reshape(-1) + lam
            # min 1/2||x - target||^2 + 1/2 sum w (F x - E)^2  s.t.  A x = b
            bvec = bvals[:, d, :].reshape(-1)
            x_p = np.linalg.lstsq(A, bvec, rcond=None)[0]
            Z = scipy.linalg.null_space(A)
            M = np.concatenate([Z, np.sqrt(w)[:, None] * (F @ Z)], axis=0)
            rhs = np.concatenate([target - x_p, np.sqrt(w) * (E[:, d] - F @ x_p)])
            z = np.linalg.lstsq(M, rhs, rcond=None)[0]
            out_xi[bidx, :, d, :] = (x_p + Z @ z).reshape(n, m)
            out_lam[bidx, :, d, :] = lam.reshape(n, m)
    return out_xi, out_lam


@pytest.mark.parametrize("D,ws", [(2, False), (3, False), (2, True), (3, True)])
def test_one_iteration_matches_independent_step(D, ws):
    # with the workspace: a ball of radius 0.35 about an off-origin centre, so that part of
    # every trajectory lies outside it
    cfg = small_cfg(n=3, D=D, degree=7, H=12, rho=(1.0, 0.7, 1.3),
                    ws=(0.35, 0.35) if ws else (0.0, 0.0), rho_ws=0.8, ws_c=(0.05, -0.1, 0.02))
    rng = np.random.default_rng(5)
    st = rng.uniform(-0.4, 0.4, size=(3, D))
    gl = -st
    xi_bar = W.sample_coeffs(rng, st, gl, cfg.degree, 3, 0.5)
    bvals = W.boundary_values(st, gl)
    xi0 = xi_bar + rng.normal(size=xi_bar.shape) * 0.1
    lam0 = rng.normal(size=xi_bar.shape) * 0.2
    s = O.build_system(cfg)
    xi1, lam1, _ = O.sf_project(s, torch.tensor(xi_bar), torch.tensor(bvals), 1,
                                xi0=torch.tensor(xi0), lam0=torch.tensor(lam0))
    exi, elam = _one_step_independent(cfg, xi_bar, bvals, xi0, lam0)
    assert np.allclose(lam1.numpy(), elam, atol=1e-11, rtol=1e-11)
    assert np.allclose(xi1.numpy(), exi, atol=1e-10, rtol=1e-10)


# --------------------------------------------------------------------------
# invariants of the whole iteration
# --------------------------------------------------------------------------

def _feasible_line_instance(n=4, D=3):
    """Straight lines far apart, slow, with boundary velocities consistent with the line."""
    cfg = small_cfg(n=n, D=D, degree=10, H=30, T=10.0)
    st = np.zeros((n, D)); gl = np.zeros((n, D))
    for i in range(n):
        st[i, 0] = 1.5 * i; gl[i, 0] = 1.5 * i
        st[i, 1] = -1.0; gl[i, 1] = 1.0
    xi = W.straight_line_coeffs(st, gl, cfg.degree)[None]
    b = W.boundary_values(st, gl)
    b[:, :, 1] = (gl - st) / cfg.t_final
    b[:, :, 4] = (gl - st) / cfg.t_final
    return cfg, xi, b


@pytest.mark.parametrize("ws", [False, True])
def test_feasible_input_is_a_fixed_point(ws):
    cfg, xi, b = _feasible_line_instance()
    if ws:   # a workspace spheroid that holds every line (x in [0, 4.5], y in [-1, 1], z = 0)
        cfg = replace(cfg, ws_a=3.0, ws_b=0.5, ws_x=2.25)
    s = O.build_system(cfg)
    out, lam, res = O.sf_project(s, torch.tensor(xi), torch.tensor(b), 50)
    assert np.abs(out.numpy() - xi).max() < 1e-12
    assert np.abs(lam.numpy()).max() < 1e-12
    assert res[0, 0].item() < 1e-24


def test_workspace_pulls_trajectories_inside():
    # lines that leave a spheroid workspace are brought inside it (to the R16 tolerance) while
    # the ends, pinned inside, stay put; the report agrees with a de Casteljau evaluation
    cfg, xi, b = _feasible_line_instance(n=3)
    cfg = replace(cfg, ws_a=2.2, ws_b=0.5, ws_x=1.5, ws_y=0.0, vmax=0.0, amax=0.0)
    xi_bar = xi.copy()
    xi_bar[:, :, 2, 3:-3] += 0.8     # middle coefficients lifted 0.8 m in z, out of the spheroid (b_w = 0.5)
    s = O.build_system(cfg)
    f0 = O.feasibility(s, torch.tensor(xi_bar), torch.tensor(b)).numpy()
    assert f0[0, 4] > 0.3
    out, _, _ = O.sf_project(s, torch.tensor(xi_bar), torch.tensor(b), 400)
    f = O.feasibility(s, out, torch.tensor(b)).numpy()
    assert f[0, 4] <= 1e-3 and f[0, 3] < 1e-12
    X, _, _ = curve_on_grid(out.numpy(), cfg.horizon, cfg.t_final)
    q = ((X[0, :, 0] - 1.5) / 2.2) ** 2 + (X[0, :, 1] / 2.2) ** 2 + (X[0, :, 2] / 0.5) ** 2
    assert abs(2.2 * (np.sqrt(q.max()) - 1.0) - f[0, 4]) < 1e-12


def test_equality_only_limit_is_the_affine_projection():
    # no bound rows, robots far apart: every projection is inactive, lambda stays 0 and the
    # iteration is a proximal-point method converging to the projection of xi_bar on {A xi = b}
    cfg = small_cfg(n=3, D=2, degree=8, H=12, T=3.0, vmax=0.0, amax=0.0, rho=(0.05, 1, 1))
    rng = np.random.default_rng(6)
    st = np.array([[0.0, 0.0], [5.0, 0.0], [10.0, 0.0]])
    gl = st + np.array([0.0, 1.0])
    xi_bar = W.straight_line_coeffs(st, gl, cfg.degree)[None] + rng.normal(size=(1, 3, 2, 9)) * 0.05
    b = W.boundary_values(st, gl)
    s = O.build_system(cfg)
    out, lam, _ = O.sf_project(s, torch.tensor(xi_bar), torch.tensor(b), 400)
    P, Pd, Pdd = s.P.numpy(), s.Pd.numpy(), s.Pdd.numpy()
    A1 = np.stack([P[0], Pd[0], Pdd[0], P[-1], Pd[-1], Pdd[-1]])
    for i in range(3):
        for d in range(2):
            c = xi_bar[0, i, d]
            proj = c - A1.T @ np.linalg.solve(A1 @ A1.T, A1 @ c - b[i, d])
            assert np.allclose(out[0, i, d].numpy(), proj, atol=1e-10)
    assert np.abs(lam.numpy()).max() < 1e-12     # the trig closed forms rebuild r to rounding


# --------------------------------------------------------------------------
# equality-only QP layer of the decoders (the QP of eq. (sf_form) without inequalities)
# --------------------------------------------------------------------------

def test_qp_equality_is_the_orthogonal_projection_onto_the_boundary_conditions():
    # the minimiser of 1/2||xi - xi_in||^2 on {A xi = b} is the unique point of that affine set
    # whose offset from xi_in lies in the row space of A: check both with scipy's null space,
    # idempotence, and that only the three first and last coefficients move
    cfg = small_cfg(n=3, D=3, degree=9, H=15, T=4.0)
    s = O.build_system(cfg)
    rng = np.random.default_rng(21)
    xi_in = rng.normal(size=(4, 3, 3, 10))
    b = rng.normal(size=(3, 3, 6))
    out = O.qp_equality(s, torch.tensor(xi_in), torch.tensor(b)).numpy()
    A1 = s.A.numpy()[:6, :10]
    assert np.allclose(np.einsum("rk,bidk->bidr", A1, out), b[None], atol=1e-10)
    Z = scipy.linalg.null_space(A1)
    assert np.abs(np.einsum("kz,bidk->bidz", Z, xi_in - out)).max() < 1e-11
    again = O.qp_equality(s, torch.tensor(out), torch.tensor(b)).numpy()
    assert np.allclose(again, out, atol=1e-11)
    assert np.allclose(out[..., 3:-3], xi_in[..., 3:-3], atol=1e-12)
    # against a generic equality-constrained least-squares solve (scipy lstsq on the KKT system)
    K = np.block([[np.eye(10), A1.T], [A1, np.zeros((6, 6))]])
    for bi in range(2):
        for i in range(3):
            for d in range(3):
                sol = np.linalg.lstsq(K, np.concatenate([xi_in[bi, i, d], b[i, d]]), rcond=None)[0][:10]
                assert np.allclose(out[bi, i, d], sol, atol=1e-10)


def test_qp_equality_is_the_sf_limit_without_active_inequalities():
    # with every inequality inactive the SF iteration converges to the same projection
    cfg = small_cfg(n=3, D=2, degree=8, H=12, T=3.0, vmax=0.0, amax=0.0, rho=(0.05, 1, 1))
    rng = np.random.default_rng(6)
    st = np.array([[0.0, 0.0], [5.0, 0.0], [10.0, 0.0]])
    gl = st + np.array([0.0, 1.0])
    xi_bar = W.straight_line_coeffs(st, gl, cfg.degree)[None] + rng.normal(size=(1, 3, 2, 9)) * 0.05
    b = W.boundary_values(st, gl)
    s = O.build_system(cfg)
    out, _, _ = O.sf_project(s, torch.tensor(xi_bar), torch.tensor(b), 400)
    q = O.qp_equality(s, torch.tensor(xi_bar), torch.tensor(b))
    assert torch.allclose(out, q, atol=1e-10)


def test_qp_equality_gradient_matches_central_differences():
    cfg = small_cfg(n=2, D=3, degree=7, H=10)
    s = O.build_system(cfg)
    rng = np.random.default_rng(22)
    xi = torch.tensor(rng.normal(size=(2, 2, 3, 8)), requires_grad=True)
    b = torch.tensor(rng.normal(size=(2, 3, 6)), requires_grad=True)
    w = torch.tensor(rng.normal(size=(2, 2, 3, 8)))
    loss = (O.qp_equality(s, xi, b) * w).sum()
    gx, gb = torch.autograd.grad(loss, (xi, b))
    for _ in range(3):
        dx = torch.tensor(rng.normal(size=xi.shape))
        db = torch.tensor(rng.normal(size=b.shape))
        h = 1e-6
        f = lambda t: (O.qp_equality(s, xi.detach() + t * dx, b.detach() + t * db) * w).sum().item()
        fd = (f(h) - f(-h)) / (2 * h)
        assert abs(fd - ((gx * dx).sum() + (gb * db).sum()).item()) < 1e-7 * (1 + abs(fd))


def test_boundary_conditions_hold_after_each_iteration():
    wl = W.tiny2d(3)
    p = wl.problems[0]
    s = O.build_system(p.cfg)
    for k in (1, 5):
        xi, _, _ = O.sf_project(s, torch.tensor(p.xi_bar), torch.tensor(p.bvals), k)
        X, V, A = curve_on_grid(xi.numpy(), p.cfg.horizon, p.cfg.t_final)
        assert np.allclose(X[..., 0], p.bvals[None, :, :, 0], atol=1e-12)
        assert np.allclose(V[..., 0], 0.0, atol=1e-11) and np.allclose(A[..., 0], 0.0, atol=1e-10)
        assert np.allclose(X[..., -1], p.bvals[None, :, :, 3], atol=1e-12)
        assert np.allclose(V[..., -1], 0.0, atol=1e-11) and np.allclose(A[..., -1], 0.0, atol=1e-10)


def test_converged_outputs_are_feasible_tiny2d():
    wl = W.tiny2d()
    p = wl.problems[0]
    s = O.build_system(p.cfg)
    xi, _, _ = O.sf_project(s, torch.tensor(p.xi_bar), torch.tensor(p.bvals), wl.iters)
    X, V, A = curve_on_grid(xi.numpy(), p.cfg.horizon, p.cfg.t_final)
    tol = 1e-3
    n = p.cfg.n_robots
    for i in range(n):
        for j in range(i + 1, n):
            dist = np.linalg.norm(X[:, i] - X[:, j], axis=1)        # [B, H]
            assert dist.min() >= p.cfg.safety_a - tol
    assert np.linalg.norm(V, axis=2).max() <= p.cfg.vmax + tol
    assert np.linalg.norm(A, axis=2).max() <= p.cfg.amax + tol
    # the sampled (uncorrected) trajectories were not feasible
    X0, V0, A0 = curve_on_grid(p.xi_bar, p.cfg.horizon, p.cfg.t_final)
    assert np.linalg.norm(A0, axis=2).max() > p.cfg.amax + 0.5
    # and the oracle's own feasibility report agrees with the de Casteljau evaluation
    f = O.feasibility(s, xi, torch.tensor(p.bvals)).numpy()
    assert (f[:, :3] <= tol).all() and (f[:, 3] < 1e-12).all()


def test_residual_block_max_is_non_increasing():
    wl = W.tiny2d()
    p = wl.problems[0]
    s = O.build_system(p.cfg)
    _, _, hist = O.sf_project(s, torch.tensor(p.xi_bar), torch.tensor(p.bvals), 200, record=True)
    h = hist[:, :, 0].numpy()
    blocks = np.stack([h[:, i:i + 25].max(1) for i in range(0, 200, 25)], axis=1)
    assert (np.diff(blocks, axis=1) <= 0).all()
    assert (h[:, -1] < 1e-4 * h[:, 0]).all()


def test_printed_lambda_sign_diverges():
    # Reading of eq. (lambda_step): with the printed "+" the residual blows up; with "-" it
    # converges (test plants the printed sign in the oracle, on the CPU).
    wl = W.tiny2d(2)
    p = wl.problems[0]
    s = O.build_system(p.cfg)
    _, _, good = O.sf_project(s, torch.tensor(p.xi_bar), torch.tensor(p.bvals), 100)
    _, _, bad = O.sf_project(s, torch.tensor(p.xi_bar), torch.tensor(p.bvals), 100, lambda_sign=+1.0)
    assert (good[:, 0] < 1e-2).all()
    assert (bad[:, 0] > 1e3).all() or not torch.isfinite(bad[:, 0]).all()


def test_resume_equals_uninterrupted_run():
    wl = W.tiny2d(3)
    p = wl.problems[0]
    s = O.build_system(p.cfg)
    xb, bv = torch.tensor(p.xi_bar), torch.tensor(p.bvals)
    x1, l1, _ = O.sf_project(s, xb, bv, 30)
    x2, l2, _ = O.sf_project(s, xb, bv, 20, xi0=x1, lam0=l1)
    x3, l3, _ = O.sf_project(s, xb, bv, 50)
    assert torch.equal(x2, x3) and torch.equal(l2, l3)


def test_residual_definition_uses_previous_targets():
    # eq. (primal_residual): r_p = F xi^{k+1} - e^{k+1}, with e^{k+1} from xi^k
    wl = W.tiny2d(2)
    p = wl.problems[0]
    s = O.build_system(p.cfg)
    xb, bv = torch.tensor(p.xi_bar), torch.tensor(p.bvals)
    x9, _, _ = O.sf_project(s, xb, bv, 9)
    x10, _, r10 = O.sf_project(s, xb, bv, 10)
    X9, _, _ = curve_on_grid(x9.numpy(), p.cfg.horizon, p.cfg.t_final)
    X10, V10, A10 = curve_on_grid(x10.numpy(), p.cfg.horizon, p.cfg.t_final)
    _, V9, A9 = curve_on_grid(x9.numpy(), p.cfg.horizon, p.cfg.t_final)
    tot = np.zeros(2)
    mx = np.zeros(2)
    n = p.cfg.n_robots
    for i in range(n):
        for j in range(i + 1, n):
            q9 = np.moveaxis(X9[:, i] - X9[:, j], 1, 2)
            q10 = np.moveaxis(X10[:, i] - X10[:, j], 1, 2)
            rp = q10 - closest_point_outside(q9, p.cfg.safety_a)
            tot += (rp**2).sum((1, 2)); mx = np.maximum(mx, np.linalg.norm(rp, axis=2).max(1))
    for Z9, Z10, lim in ((V9, V10, p.cfg.vmax), (A9, A10, p.cfg.amax)):
        z9 = np.moveaxis(Z9, 2, 3); z10 = np.moveaxis(Z10, 2, 3)
        rp = z10 - closest_point_inside(z9, lim)
        tot += (rp**2).sum((1, 2, 3)); mx = np.maximum(mx, np.linalg.norm(rp, axis=3).max((1, 2)))
    assert np.allclose(r10[:, 0].numpy(), tot, rtol=1e-10)
    assert np.allclose(r10[:, 1].numpy(), mx, rtol=1e-10)


# --------------------------------------------------------------------------
# brute-force comparator (scipy SLSQP) -- one-sided, the SF is not the exact minimiser
# --------------------------------------------------------------------------

def test_two_robot_head_on_against_slsqp():
    cfg = small_cfg(n=2, D=2, degree=7, H=16, T=4.0, vmax=3.0, amax=6.0)
    st = np.array([[-1.0, 0.0], [1.0, 0.0]])
    gl = -st
    rng = np.random.default_rng(7)
    xi_bar = W.straight_line_coeffs(st, gl, cfg.degree)[None] + rng.normal(size=(1, 2, 2, 8)) * 0.05
    b = W.boundary_values(st, gl)
    s = O.build_system(cfg)
    out, _, _ = O.sf_project(s, torch.tensor(xi_bar), torch.tensor(b), 3000)
    sf = out.numpy()[0]
    P, Pd, Pdd = s.P.numpy(), s.Pd.numpy(), s.Pdd.numpy()
    A1 = np.stack([P[0], Pd[0], Pdd[0], P[-1], Pd[-1], Pdd[-1]])

    def unpack(z):
        return z.reshape(2, 2, 8)

    def cost(z):
        return 0.5 * np.sum((z - xi_bar[0].reshape(-1)) ** 2)

    def eq(z):
        c = unpack(z)
        return np.concatenate([A1 @ c[i, d] - b[i, d] for i in range(2) for d in range(2)])

    def ineq(z):
        c = unpack(z)
        X = np.einsum("hk,idk->idh", P, c)
        V = np.einsum("hk,idk->idh", Pd, c)
        A = np.einsum("hk,idk->idh", Pdd, c)
        dist2 = np.sum((X[0] - X[1]) ** 2, axis=0)
        return np.concatenate([dist2 - cfg.safety_a**2,
                               cfg.vmax**2 - np.sum(V**2, axis=1).ravel(),
                               cfg.amax**2 - np.sum(A**2, axis=1).ravel()])
    assert eq(sf.reshape(-1)).__abs__().max() < 1e-10
    assert ineq(sf.reshape(-1)).min() > -1e-3                 # SF output feasible
    res = scipy.optimize.minimize(cost, sf.reshape(-1), method="SLSQP",
                                  constraints=[dict(type="eq", fun=eq), dict(type="ineq", fun=ineq)],
                                  options=dict(maxiter=500, ftol=1e-14))
    assert res.success
    assert cost(sf.reshape(-1)) >= res.fun - 1e-9           # SF is no better than a local optimum
    assert cost(sf.reshape(-1)) <= 3.0 * res.fun + 1e-6     # and within a small factor of it
    # the robots pass each other: separation is attained, not violated
    X = np.einsum("hk,idk->idh", P, sf)
    assert np.sqrt(np.sum((X[0] - X[1]) ** 2, axis=0)).min() >= cfg.safety_a - 1e-3


def test_symmetric_head_on_keeps_its_symmetry():
    """Exactly symmetric head-on (two robots swapping places on a line, no noise): the iteration is
    equivariant under the point reflection that swaps the robots, so the output keeps x_2 = -x_1
    and never leaves the line (no lateral avoidance develops; only a perturbation breaks the tie,
    as in the head-on case above).  The separation at the grid times grows towards the safety
    distance without reaching it in a finite run: the behaviour is pinned, not feasibility."""
    cfg = small_cfg(n=2, D=2, degree=7, H=16, T=4.0, vmax=3.0, amax=6.0)
    st = np.array([[-1.0, 0.0], [1.0, 0.0]])
    gl = -st
    xi_bar = W.straight_line_coeffs(st, gl, cfg.degree)[None]
    b = W.boundary_values(st, gl)
    s = O.build_system(cfg)
    P = s.P.numpy()
    dmins = []
    for K in (200, 800):
        out, _, _ = O.sf_project(s, torch.tensor(xi_bar), torch.tensor(b), K)
        x = out.numpy()[0]
        assert np.abs(x[0] + x[1]).max() < 1e-12            # point symmetry x_2 = -x_1
        X = np.einsum("hk,idk->idh", P, x)
        assert np.abs(X[:, 1]).max() < 1e-12                 # stays on the line
        dmins.append(np.sqrt(((X[0] - X[1]) ** 2).sum(0)).min())
    assert dmins[0] < dmins[1] < cfg.safety_a


def test_three_robot_crossing_against_slsqp():
    """Three robots in 2D on a unit circle crossing through its centre to the antipodes: the SF
    output is feasible, and its cost is no lower than the local optimum scipy's SLSQP reaches from
    it (and from xi_bar: the same optimum) and within a small factor of it (one-sided: the SF
    converges to a feasible point near xi_bar, not to the minimiser of eq. sf_form)."""
    n = 3
    cfg = small_cfg(n=n, D=2, degree=7, H=16, T=4.0, vmax=3.0, amax=6.0)
    th = 2 * np.pi * np.arange(n) / n + 0.1
    st = np.stack([np.cos(th), np.sin(th)], 1)
    gl = -st
    rng = np.random.default_rng(17)
    xi_bar = W.straight_line_coeffs(st, gl, cfg.degree)[None] + rng.normal(size=(1, n, 2, 8)) * 0.05
    b = W.boundary_values(st, gl)
    s = O.build_system(cfg)
    out, _, _ = O.sf_project(s, torch.tensor(xi_bar), torch.tensor(b), 3000)
    sf = out.numpy()[0].reshape(-1)
    P, Pd, Pdd = s.P.numpy(), s.Pd.numpy(), s.Pdd.numpy()
    A1 = np.stack([P[0], Pd[0], Pdd[0], P[-1], Pd[-1], Pdd[-1]])

    def cost(z):
        return 0.5 * np.sum((z - xi_bar[0].reshape(-1)) ** 2)

    def eq(z):
        c = z.reshape(n, 2, 8)
        return np.concatenate([A1 @ c[i, d] - b[i, d] for i in range(n) for d in range(2)])

    def ineq(z):
        c = z.reshape(n, 2, 8)
        X = np.einsum("hk,idk->idh", P, c)
        V = np.einsum("hk,idk->idh", Pd, c)
        A = np.einsum("hk,idk->idh", Pdd, c)
        pairs = [np.sum((X[i] - X[j]) ** 2, axis=0) - cfg.safety_a ** 2 for i in range(n) for j in range(i + 1, n)]
        return np.concatenate(pairs + [cfg.vmax ** 2 - np.sum(V ** 2, axis=1).ravel(),
                                       cfg.amax ** 2 - np.sum(A ** 2, axis=1).ravel()])
    assert np.abs(eq(sf)).max() < 1e-10
    assert ineq(sf).min() > -1e-3                       # SF output feasible
    cons = [dict(type="eq", fun=eq), dict(type="ineq", fun=ineq)]
    opts = dict(maxiter=500, ftol=1e-14)
    res = scipy.optimize.minimize(cost, sf, method="SLSQP", constraints=cons, options=opts)
    res_bar = scipy.optimize.minimize(cost, xi_bar[0].reshape(-1), method="SLSQP", constraints=cons, options=opts)
    assert res.success and res_bar.success
    assert abs(res.fun - res_bar.fun) <= 1e-8 * res.fun
    assert cost(sf) >= res.fun - 1e-9
    assert cost(sf) <= 3.0 * res.fun + 1e-6
    X = np.einsum("hk,idk->idh", P, out.numpy()[0])
    dmin = min(np.sqrt(np.sum((X[i] - X[j]) ** 2, axis=0)).min() for i in range(n) for j in range(i + 1, n))
    assert dmin >= cfg.safety_a - 1e-3


# --------------------------------------------------------------------------
# autograd through the oracle (reference gradients) against central differences
# --------------------------------------------------------------------------

def test_oracle_autograd_matches_central_differences():
    cfg = small_cfg(n=3, D=3, degree=7, H=12)
    rng = np.random.default_rng(8)
    st = rng.uniform(-0.3, 0.3, size=(3, 3))
    xi_bar = torch.tensor(W.sample_coeffs(rng, st, -st, 7, 2, 0.3))
    b = torch.tensor(W.boundary_values(st, -st))
    s = O.build_system(cfg)
    lam0 = torch.tensor(rng.normal(size=xi_bar.shape) * 0.1)

    def loss(x0, l0):
        xo, _, r = O.sf_project(s, xi_bar, b, 8, xi0=x0, lam0=l0)
        return ((xo - xi_bar) ** 2).sum() + r[:, 0].sum()
    x0 = xi_bar.clone().requires_grad_(True)
    l0 = lam0.clone().requires_grad_(True)
    L = loss(x0, l0)
    gx, gl = torch.autograd.grad(L, (x0, l0))
    h = 1e-5
    for k in range(4):
        dx = torch.tensor(rng.normal(size=xi_bar.shape))
        dl = torch.tensor(rng.normal(size=xi_bar.shape))
        fd = (loss(xi_bar + h * dx, lam0 + h * dl) - loss(xi_bar - h * dx, lam0 - h * dl)) / (2 * h)
        an = (gx * dx).sum() + (gl * dl).sum()
        assert abs(fd.item() - an.item()) <= 1e-5 * max(1.0, abs(an.item()))
