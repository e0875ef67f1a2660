"""Plain FP64 CPU oracle of the batched safety filter (SF).

TEST INFRASTRUCTURE ONLY -- only tests/, the entry module's smoke check and the
benchmark's CPU-baseline leg may use it.  It is deliberately slow and literal:
the constraint matrix F is built densely from the Kronecker construction of the
Appendix, the alpha/beta/d steps use the trigonometric closed forms, and the
xi-step solves the full KKT system of eq. (xi_step) with a library LU
factorisation.  Everything is float64 PyTorch on the CPU, so autograd through
this module gives reference gradients.

Readings of the paper taken here, where it is silent, ambiguous or garbled:
  * lambda step: lambda <- lambda - rho F^T (F xi - e).  The printed "+" in
    eq. (lambda_step) contradicts the -<lambda, xi> term of eq. (aug_lag) and the
    +lambda of eta; with "+" the iteration diverges.
  * eq. (fixed_point) prints lambda^{k+1} on the right; the state is (xi^k, lambda^k).
  * eq. (xi_step) prints M = [.]^{-1} and then M^{-1} eta; xi is the first block
    of K^{-1} [eta_1; b] with K the KKT matrix.
  * beta step for a != b: beta = atan2((r_x cos a + r_y sin a)/a, r_z/b), the
    angle in the axis-scaled frame (the paper cites closed forms it does not print).
  * velocity/acceleration bounds are not in the paper; they are modelled as
    origin-centred balls in the polar form of eq. (workspace_polar), d in [0, 1].
  * the workspace constraint (eqs. (workspace_con), (workspace_polar)) is off unless
    its semi-axes are given; its angles are those of the axis-scaled offset from the
    centre, as for the collision spheroid.
  * polynomial basis: Bernstein of the given degree on tau = t/T, uniform grid
    tau_h = h/(H-1) including both endpoints.
  * goal boundary conditions are (p, v, a) at t = T (eq. (boundary_con) lists the
    acceleration twice).
  * rho may differ per constraint block (collision, velocity, acceleration); the
    paper uses a single rho, which is the default of 1 for every block.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Optional

import torch

DT = torch.float64


# ---------------------------------------------------------------------------
# Polynomial parametrisation, eq. (poly)
# ---------------------------------------------------------------------------

def bernstein(degree: int, tau: torch.Tensor) -> torch.Tensor:
    """B_{N,k}(tau) = C(N,k) tau^k (1-tau)^(N-k), k = 0..N.  Returns [len(tau), N+1]."""
    tau = tau.to(DT)
    cols = []
    for k in range(degree + 1):
        cols.append(math.comb(degree, k) * tau ** k * (1.0 - tau) ** (degree - k))
    return torch.stack(cols, dim=1)


def _bern_padded(degree: int, tau: torch.Tensor, shift: int, m: int) -> torch.Tensor:
    """Columns k = 0..m-1 holding B_{degree, k-shift}(tau), zero outside 0..degree."""
    out = torch.zeros(tau.shape[0], m, dtype=DT)
    if degree < 0:
        return out
    b = bernstein(degree, tau)
    for k in range(m):
        j = k - shift
        if 0 <= j <= degree:
            out[:, k] = b[:, j]
    return out


def basis_matrices(degree: int, horizon: int, t_final: float):
    """Position, velocity and acceleration basis matrices W, W-dot, W-ddot of eq. (poly).

    P[h, k] = B_{N,k}(tau_h); time derivatives follow from the Bernstein derivative
    identity dB_{N,k}/dtau = N (B_{N-1,k-1} - B_{N-1,k}) and d/dt = (1/T) d/dtau.
    Returns three [H, N+1] float64 tensors."""
    N, m = degree, degree + 1
    tau = torch.arange(horizon, dtype=DT) / (horizon - 1)
    P = bernstein(N, tau)
    Pd = (N / t_final) * (_bern_padded(N - 1, tau, 1, m) - _bern_padded(N - 1, tau, 0, m))
    Pdd = (N * (N - 1) / t_final ** 2) * (_bern_padded(N - 2, tau, 2, m)
                                          - 2.0 * _bern_padded(N - 2, tau, 1, m)
                                          + _bern_padded(N - 2, tau, 0, m))
    return P, Pd, Pdd


# ---------------------------------------------------------------------------
# Constraint matrices (Appendix, "Reformulated Problem")
# ---------------------------------------------------------------------------

def pair_incidence(n: int) -> torch.Tensor:
    """Stacked F_{o,i} = [F_i, -I] for i = 1..n-1 (the Appendix's F_o before the Kronecker
    product with P).  F_i is (n-i) x i with a column of ones in column i.  Row order is
    the lexicographic pair order (i, j), i < j.  Returns [n(n-1)/2, n]."""
    blocks = []
    for i in range(1, n):
        Fi = torch.zeros(n - i, i, dtype=DT)
        Fi[:, i - 1] = 1.0
        blocks.append(torch.cat([Fi, -torch.eye(n - i, dtype=DT)], dim=1))
    return torch.cat(blocks, dim=0)


@dataclass
class OracleSystem:
    n: int
    D: int
    m: int
    H: int
    a: float
    b: float
    vmax: float
    amax: float
    P: torch.Tensor
    Pd: torch.Tensor
    Pdd: torch.Tensor
    F: torch.Tensor          # one axis block of F: [rows, n*m]
    w: torch.Tensor          # per-row rho
    A: torch.Tensor          # one axis block of A: [6n, n*m]
    kkt_lu: tuple            # LU factors of the per-axis KKT matrix
    n_pairs: int
    vel_on: bool
    acc_on: bool
    ws_on: bool = False
    ws_a: float = 0.0
    ws_b: float = 0.0
    ws_c: Optional[torch.Tensor] = None    # workspace centre [D]

    @property
    def nm(self) -> int:
        return self.n * self.m


def build_system(cfg) -> OracleSystem:
    """Dense per-axis F, A and the factorised KKT matrix of eq. (xi_step).

    F is block diagonal over the axes with identical blocks (eq. (f_e)), and so are A
    (boundary rows of eq. (boundary_con) per robot and axis) and the KKT matrix; the
    oracle stores one block and applies it to each axis."""
    n, D, N, H = cfg.n_robots, cfg.dims, cfg.degree, cfg.horizon
    m = N + 1
    P, Pd, Pdd = basis_matrices(N, H, cfg.t_final)
    Dp = pair_incidence(n)
    rows = [torch.kron(Dp, P)]
    w = [torch.full((Dp.shape[0] * H,), float(cfg.rho_coll), dtype=DT)]
    vel_on = cfg.vmax > 0
    acc_on = cfg.amax > 0
    eye_n = torch.eye(n, dtype=DT)
    if vel_on:
        rows.append(torch.kron(eye_n, Pd))
        w.append(torch.full((n * H,), float(cfg.rho_vel), dtype=DT))
    if acc_on:
        rows.append(torch.kron(eye_n, Pdd))
        w.append(torch.full((n * H,), float(cfg.rho_acc), dtype=DT))
    ws_a, ws_b = float(getattr(cfg, "ws_a", 0.0)), float(getattr(cfg, "ws_b", 0.0))
    ws_on = ws_a > 0
    if ws_on:
        # workspace rows, eq. (workspace_con): every robot position at every grid time
        rows.append(torch.kron(eye_n, P))
        w.append(torch.full((n * H,), float(cfg.rho_ws), dtype=DT))
    F = torch.cat(rows, dim=0)
    w = torch.cat(w)
    A1 = torch.stack([P[0], Pd[0], Pdd[0], P[H - 1], Pd[H - 1], Pdd[H - 1]])
    A = torch.kron(eye_n, A1)
    nm = n * m
    K = torch.zeros(nm + 6 * n, nm + 6 * n, dtype=DT)
    K[:nm, :nm] = torch.eye(nm, dtype=DT) + F.T @ (w[:, None] * F)
    K[:nm, nm:] = A.T
    K[nm:, :nm] = A
    lu = torch.linalg.lu_factor(K)
    return OracleSystem(n=n, D=D, m=m, H=H, a=float(cfg.safety_a), b=float(cfg.safety_b),
                        vmax=float(cfg.vmax), amax=float(cfg.amax), P=P, Pd=Pd, Pdd=Pdd,
                        F=F, w=w, A=A, kkt_lu=lu, n_pairs=Dp.shape[0],
                        vel_on=vel_on, acc_on=acc_on, ws_on=ws_on, ws_a=ws_a,
                        ws_b=ws_b if ws_on else 0.0,
                        ws_c=torch.tensor([float(getattr(cfg, k, 0.0)) for k in ("ws_x", "ws_y", "ws_z")][:D],
                                          dtype=DT))


# ---------------------------------------------------------------------------
# Layout conversion: [sample, robot, axis, coeff]  <->  paper order (axis, robot, coeff)
# ---------------------------------------------------------------------------

def to_paper_order(x: torch.Tensor) -> torch.Tensor:
    """[B, n, D, m] -> [B, D, n*m]; per axis the paper stacks c_{1,x}, ..., c_{n,x}."""
    B, n, D, m = x.shape
    return x.permute(0, 2, 1, 3).reshape(B, D, n * m)


def from_paper_order(x: torch.Tensor, n: int, m: int) -> torch.Tensor:
    B, D, _ = x.shape
    return x.reshape(B, D, n, m).permute(0, 2, 1, 3).contiguous()


# ---------------------------------------------------------------------------
# alpha / beta / d steps, eqs. (alpha_step)-(d_step) with the polar forms
# eq. (inter_agent_polar) and eq. (workspace_polar)
# ---------------------------------------------------------------------------

def _polar_target(r: torch.Tensor, a: float, b: float, d_min: float, d_max: float) -> torch.Tensor:
    """e = d * u(alpha, beta) for r = [..., D], D in {2, 3}.

    alpha = atan2(r_y, r_x); beta = atan2((r_x cos alpha + r_y sin alpha)/a, r_z/b);
    u = (a cos(alpha) sin(beta), a sin(alpha) sin(beta), b cos(beta)); d is the least-squares
    length <r, u>/<u, u> clipped to [d_min, d_max].  In 2D, u = a (cos alpha, sin alpha)."""
    if r.shape[-1] == 2:
        al = torch.atan2(r[..., 1], r[..., 0])
        u = torch.stack([a * torch.cos(al), a * torch.sin(al)], dim=-1)
    else:
        al = torch.atan2(r[..., 1], r[..., 0])
        be = torch.atan2((r[..., 0] * torch.cos(al) + r[..., 1] * torch.sin(al)) / a, r[..., 2] / b)
        u = torch.stack([a * torch.cos(al) * torch.sin(be),
                         a * torch.sin(al) * torch.sin(be),
                         b * torch.cos(be)], dim=-1)
    d = (r * u).sum(-1) / (u * u).sum(-1)
    d = torch.clamp(d, min=d_min, max=d_max)
    return d[..., None] * u


def project_collision(r: torch.Tensor, a: float, b: float) -> torch.Tensor:
    """Targets for the pair rows: d in [1, inf) (eq. (inter_agent_polar))."""
    return _polar_target(r, a, b, 1.0, math.inf)


def project_ball(v: torch.Tensor, radius: float) -> torch.Tensor:
    """Targets for an origin-centred ball of the given radius: d in [0, 1]."""
    return _polar_target(v, radius, radius, 0.0, 1.0)


def project_workspace(p: torch.Tensor, a: float, b: float, centre=None) -> torch.Tensor:
    """Targets for the workspace rows (the F_w block of eq. (f_e)): p_w + d u(alpha_w, beta_w)
    with the spheroid (a, a, b) of eq. (workspace_polar), d in [0, 1]."""
    c = torch.zeros(p.shape[-1], dtype=DT) if centre is None else torch.as_tensor(centre, dtype=DT)
    return c + _polar_target(p - c, a, b, 0.0, 1.0)


def _targets(sys: OracleSystem, Y: torch.Tensor) -> torch.Tensor:
    """e for all rows of all axes.  Y = F xi per axis: [B, D, rows] -> e of the same shape."""
    B, D, _ = Y.shape
    n, H, Np = sys.n, sys.H, sys.n_pairs
    o = 0
    parts = []
    r = Y[:, :, o:o + Np * H].reshape(B, D, Np, H).permute(0, 2, 3, 1)        # [B, Np, H, D]
    e = project_collision(r, sys.a, sys.b)
    parts.append(e.permute(0, 3, 1, 2).reshape(B, D, Np * H))
    o += Np * H
    for on, lim in ((sys.vel_on, sys.vmax), (sys.acc_on, sys.amax)):
        if not on:
            continue
        v = Y[:, :, o:o + n * H].reshape(B, D, n, H).permute(0, 2, 3, 1)        # [B, n, H, D]
        ev = project_ball(v, lim)
        parts.append(ev.permute(0, 3, 1, 2).reshape(B, D, n * H))
        o += n * H
    if sys.ws_on:
        p = Y[:, :, o:o + n * H].reshape(B, D, n, H).permute(0, 2, 3, 1)        # [B, n, H, D]
        ep = project_workspace(p, sys.ws_a, sys.ws_b, sys.ws_c)
        parts.append(ep.permute(0, 3, 1, 2).reshape(B, D, n * H))
        o += n * H
    return torch.cat(parts, dim=2)


def _block_norm_max(sys: OracleSystem, r: torch.Tensor) -> torch.Tensor:
    """Largest Euclidean norm of one constraint's residual (a pair-time or a robot-time
    block across the axes).  r: [B, D, rows] -> [B]."""
    sq = (r * r).sum(1)                       # [B, rows]
    return sq.max(dim=1).values.sqrt()


# ---------------------------------------------------------------------------
# The fixed-point iteration, eqs. (alpha_step)-(xi_step) and (primal_residual)
# ---------------------------------------------------------------------------

def sf_project(sys: OracleSystem, xi_bar: torch.Tensor, bvals: torch.Tensor, iters: int,
               xi0: Optional[torch.Tensor] = None, lam0: Optional[torch.Tensor] = None,
               record: bool = False, lambda_sign: float = -1.0):
    """Run `iters` SF iterations.

    xi_bar, xi0, lam0: [B, n, D, m]; bvals: [n, D, 6] = (p0, v0, a0, pH, vH, aH).
    Defaults: xi0 = xi_bar, lam0 = 0.
    Returns (xi_K, lam_K, resid) with resid [B, 2] = (||r_p||_2^2, largest block norm) of
    eq. (primal_residual) after the last iteration, or [B, iters, 2] when record=True.
    lambda_sign = +1 reproduces the sign printed in eq. (lambda_step) (used only to show
    that reading diverges)."""
    n, D, m = sys.n, sys.D, sys.m
    xb = to_paper_order(xi_bar.to(DT))                           # [B, D, nm]
    xi = xb.clone() if xi0 is None else to_paper_order(xi0.to(DT))
    lam = torch.zeros_like(xb) if lam0 is None else to_paper_order(lam0.to(DT))
    bvec = bvals.to(DT).permute(1, 0, 2).reshape(D, n * 6)       # per axis: (robot, 6)
    F, w = sys.F, sys.w
    B = xb.shape[0]
    nm = sys.nm
    hist = []
    Y = xi @ F.T                                                 # F xi^k, [B, D, rows]
    rp = None
    for _ in range(iters):
        e = _targets(sys, Y)                                     # e^{k+1} from xi^k
        lam = lam + lambda_sign * ((w * (Y - e)) @ F)            # lambda step
        eta1 = (w * e) @ F + lam + xb
        rhs = torch.cat([eta1, bvec.unsqueeze(0).expand(B, D, n * 6)], dim=2)
        sol = torch.linalg.lu_solve(*sys.kkt_lu, rhs.reshape(B * D, -1, 1)).reshape(B, D, -1)
        xi = sol[:, :, :nm]                                      # xi step
        Y = xi @ F.T
        rp = Y - e                                               # primal residual
        if record:
            hist.append(_resid_pair(sys, rp))
    if record:
        resid = torch.stack(hist, dim=1) if hist else torch.zeros(B, 0, 2, dtype=DT)
    elif rp is None:
        resid = torch.zeros(B, 2, dtype=DT)
    else:
        resid = _resid_pair(sys, rp)
    return from_paper_order(xi, n, m), from_paper_order(lam, n, m), resid


def qp_equality(sys: OracleSystem, xi_in: torch.Tensor, bvals: torch.Tensor) -> torch.Tensor:
    """Equality-only QP layer of the decoders (Sec. IV: the QP of eq. (sf_form) without its
    inequality rows): argmin 1/2 ||xi - xi_in||^2 subject to the boundary rows A xi = b of
    eq. (boundary_con), per robot-axis, by its definition xi_in - A^T (A A^T)^{-1} (A xi_in - b).
    xi_in [B, n, D, m], bvals [n, D, 6] -> [B, n, D, m] float64 (differentiable)."""
    A1 = sys.A[:6, :sys.m]                                            # one robot-axis block
    xi = xi_in.to(DT)
    r = torch.einsum("rk,bidk->bidr", A1, xi) - bvals.to(DT)[None]
    mu = torch.linalg.solve(A1 @ A1.T, r.unsqueeze(-1)).squeeze(-1)
    return xi - torch.einsum("rk,bidr->bidk", A1, mu)


def _resid_pair(sys: OracleSystem, rp: torch.Tensor) -> torch.Tensor:
    return torch.stack([(rp * rp).sum((1, 2)), _block_norm_max(sys, rp)], dim=1)


def feasibility(sys: OracleSystem, xi: torch.Tensor, bvals: torch.Tensor) -> torch.Tensor:
    """Constraint violations at the grid times, [B, 5] float64:
    (collision: a * (1 - min ||M_a^{-1}(p_i - p_j)||), max ||v|| - vmax, max ||acc|| - amax,
     max |A xi - b|, workspace: a_w * (max ||M_w^{-1} p_i|| - 1), 0 when it is off).
    Positive means violated."""
    xi = xi.to(DT)
    X = torch.einsum("hk,bidk->bidh", sys.P, xi)
    V = torch.einsum("hk,bidk->bidh", sys.Pd, xi)
    Acc = torch.einsum("hk,bidk->bidh", sys.Pdd, xi)
    n = sys.n
    ii, jj = torch.triu_indices(n, n, offset=1)
    r = X[:, ii] - X[:, jj]                                      # [B, Np, D, H]
    scale = torch.full((sys.D,), sys.a, dtype=DT)
    if sys.D == 3:
        scale[2] = sys.b
    s = (r / scale[None, None, :, None]).pow(2).sum(2).sqrt()
    coll = sys.a * (1.0 - s.amin(dim=(1, 2)))
    vel = V.pow(2).sum(2).sqrt().amax(dim=(1, 2)) - sys.vmax
    acc = Acc.pow(2).sum(2).sqrt().amax(dim=(1, 2)) - sys.amax
    A1 = sys.A[:6, :sys.m]
    bnd = (torch.einsum("rk,bidk->bidr", A1, xi) - bvals.to(DT)[None]).abs().amax(dim=(1, 2, 3))
    if sys.ws_on:
        sw = torch.full((sys.D,), sys.ws_a, dtype=DT)
        if sys.D == 3:
            sw[2] = sys.ws_b
        q = ((X - sys.ws_c[None, None, :, None]) / sw[None, None, :, None]).pow(2).sum(2).sqrt()
        ws = sys.ws_a * (q.amax(dim=(1, 2)) - 1.0)
    else:
        ws = torch.zeros_like(bnd)
    return torch.stack([coll, vel, acc, bnd, ws], dim=1)
