"""Python binding of the safety-filter library: device buffers and streams from PyTorch,
every step of the solve in the HIP kernels behind include/swarmsf.h."""
from __future__ import annotations

import ctypes
import math
from collections import namedtuple
from typing import Iterable, Optional, Sequence, Tuple

import torch

from . import _native as N

ProjectResult = namedtuple("ProjectResult", ["xi", "lam", "resid", "ckpt", "status"], defaults=(None,))


def _ptr(t: Optional[torch.Tensor]):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream_ptr(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Batch:
    """Problem table of a call: a sequence of (config slot, sample count)."""

    def __init__(self, entries: Iterable[Tuple[int, int]]):
        entries = [(int(s), int(c)) for s, c in entries]
        if not entries:
            raise ValueError("empty batch")
        P = len(entries)
        self.entries = entries
        self._slots = (ctypes.c_int32 * P)(*[s for s, _ in entries])
        self._counts = (ctypes.c_int32 * P)(*[c for _, c in entries])
        self.c = N.SfBatch(P, ctypes.cast(self._slots, ctypes.POINTER(ctypes.c_int32)),
                           ctypes.cast(self._counts, ctypes.POINTER(ctypes.c_int32)))

    @property
    def n_samples(self) -> int:
        return sum(c for _, c in self.entries)


class SafetyFilter:
    """Handle on sf_setup's factors for one or more problem shapes (configs)."""

    def __init__(self, configs: Sequence):
        self.configs = list(configs)
        arr = (N.SfConfig * len(self.configs))(*[N.make_config(c) for c in self.configs])
        h = ctypes.c_void_p()
        N.check(N.lib().sf_setup(arr, len(self.configs), ctypes.byref(h)))
        self._h = h
        self.device = torch.device("cuda", torch.cuda.current_device())

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            N.lib().sf_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- sizes of a batch ---------------------------------------------------------
    def sizes(self, batch: Batch):
        coef = bnd = 0
        for slot, cnt in batch.entries:
            c = self.configs[slot]
            per = c.n_robots * c.dims * (c.degree + 1)
            coef += cnt * per
            bnd += c.n_robots * c.dims * 6
        return batch.n_samples, coef, bnd

    def _batch(self, batch, xi_bar):
        if batch is None:
            if len(self.configs) != 1 or xi_bar.dim() != 4:
                raise ValueError("pass a Batch unless there is one config and xi_bar is [S, n, D, m]")
            batch = Batch([(0, xi_bar.shape[0])])
        return batch

    def _check(self, t, name, dtype, numel):
        if t is None:
            return
        if not t.is_cuda or t.device != self.device:
            raise ValueError(f"{name} must be on {self.device}")
        if t.dtype != dtype:
            raise ValueError(f"{name} must be {dtype}")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        if t.numel() != numel:
            raise ValueError(f"{name} has {t.numel()} elements, expected {numel}")

    def project(self, xi_bar: torch.Tensor, bvals: torch.Tensor, iters: int, batch: Optional[Batch] = None,
                precision: str = "fp32", xi0: Optional[torch.Tensor] = None, lam0: Optional[torch.Tensor] = None,
                want_lam: bool = True, want_resid: bool = True, history: bool = False,
                ckpt_every: int = 0, generic: bool = False, graph: bool = False, autotune: bool = False,
                persistent: bool = False, fp_residual: bool = False, want_status: bool = False,
                out: Optional[ProjectResult] = None, stream=None) -> ProjectResult:
        """sf_project on device tensors.  With want_status, `status` holds per-sample int32 bits
        (SF_SAMPLE_NONFINITE_INPUT, SF_SAMPLE_NONFINITE, SF_SAMPLE_NOT_CONVERGED; 0 = finite and
        converged)."""
        prec = N.PRECISIONS[precision]
        dtype = torch.float64 if prec == N.SF_FP64 else torch.float32
        batch = self._batch(batch, xi_bar)
        S, coef, bnd = self.sizes(batch)
        for t, nm, ne in ((xi_bar, "xi_bar", coef), (bvals, "bvals", bnd), (xi0, "xi0", coef), (lam0, "lam0", coef)):
            self._check(t, nm, dtype, ne)
        if out is not None:           # caller-provided outputs (fixed addresses, e.g. for graph replay)
            xi_out, lam_out, resid, ckpt, status = out
        else:
            status = torch.empty((S,), dtype=torch.int32, device=self.device) if want_status else None
            xi_out = torch.empty_like(xi_bar)
            lam_out = torch.empty_like(xi_bar) if want_lam else None
            resid = None
            if want_resid:
                resid = torch.empty((S, iters, 2) if history else (S, 3 if fp_residual else 2), dtype=dtype,
                                    device=self.device)
            ckpt = None
            if ckpt_every:
                nck = max(1, math.ceil(iters / ckpt_every))
                ckpt = torch.empty((nck, 2, coef), dtype=dtype, device=self.device)
        flags = ((N.SF_RESID_HISTORY if history else 0) | (N.SF_GENERIC_KERNEL if generic else 0)
                 | (N.SF_USE_GRAPH if graph else 0) | (N.SF_AUTOTUNE if autotune else 0)
                 | (N.SF_PERSISTENT if persistent else 0) | (N.SF_FP_RESIDUAL if fp_residual else 0))
        N.check(N.lib().sf_project(self._h, ctypes.byref(batch.c), prec, _ptr(xi_bar), _ptr(bvals), _ptr(xi0),
                                   _ptr(lam0), int(iters), _ptr(xi_out), _ptr(lam_out), _ptr(resid), _ptr(status),
                                   flags, _ptr(ckpt), int(ckpt_every), _stream_ptr(stream)))
        return ProjectResult(xi_out, lam_out, resid, ckpt, status)

    def project_backward(self, xi_bar, bvals, iters, ckpt, ckpt_every, g_xi_out=None, g_lam_out=None,
                         g_resid=None, batch: Optional[Batch] = None, precision: str = "fp32",
                         want=("xi0", "lam0", "xi_bar"), w_fpr=None, stream=None):
        prec = N.PRECISIONS[precision]
        dtype = torch.float64 if prec == N.SF_FP64 else torch.float32
        batch = self._batch(batch, xi_bar)
        S, coef, bnd = self.sizes(batch)
        for t, nm, ne in ((xi_bar, "xi_bar", coef), (bvals, "bvals", bnd), (g_xi_out, "g_xi_out", coef),
                          (g_lam_out, "g_lam_out", coef), (g_resid, "g_resid", S), (w_fpr, "w_fpr", S)):
            self._check(t, nm, dtype, ne)
        out = {k: (torch.empty_like(xi_bar) if k in want else None) for k in ("xi0", "lam0", "xi_bar")}
        N.check(N.lib().sf_project_backward(self._h, ctypes.byref(batch.c), prec, _ptr(xi_bar), _ptr(bvals),
                                            int(iters), _ptr(ckpt), int(ckpt_every), _ptr(g_xi_out),
                                            _ptr(g_lam_out), _ptr(g_resid), _ptr(w_fpr), _ptr(out["xi0"]),
                                            _ptr(out["lam0"]),
                                            _ptr(out["xi_bar"]), _stream_ptr(stream)))
        return out

    def feasibility(self, xi: torch.Tensor, bvals: torch.Tensor, batch: Optional[Batch] = None,
                    precision: str = "fp32", stream=None) -> torch.Tensor:
        prec = N.PRECISIONS[precision]
        dtype = torch.float64 if prec == N.SF_FP64 else torch.float32
        batch = self._batch(batch, xi)
        S, coef, bnd = self.sizes(batch)
        self._check(xi, "xi", dtype, coef)
        self._check(bvals, "bvals", dtype, bnd)
        viol = torch.empty((S, 5), dtype=torch.float64, device=self.device)
        N.check(N.lib().sf_feasibility(self._h, ctypes.byref(batch.c), prec, _ptr(xi), _ptr(bvals), _ptr(viol),
                                       _stream_ptr(stream)))
        return viol


def _eq_dtype(precision):
    return torch.float64 if N.PRECISIONS[precision] == N.SF_FP64 else torch.float32


def qp_equality(sf: "SafetyFilter", xi_in: torch.Tensor, bvals: torch.Tensor, batch: Optional[Batch] = None,
                precision: str = "fp32", out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """Equality-only QP layer (sf_qp_equality): xi_in with the boundary conditions imposed."""
    prec = N.PRECISIONS[precision]
    batch = sf._batch(batch, xi_in)
    S, coef, bnd = sf.sizes(batch)
    sf._check(xi_in, "xi_in", _eq_dtype(precision), coef)
    sf._check(bvals, "bvals", _eq_dtype(precision), bnd)
    xo = torch.empty_like(xi_in) if out is None else out
    N.check(N.lib().sf_qp_equality(sf._h, ctypes.byref(batch.c), prec, _ptr(xi_in), _ptr(bvals), _ptr(xo),
                                   _stream_ptr(stream)))
    return xo


class _QPEquality(torch.autograd.Function):
    """sf_qp_equality forward, sf_qp_equality_backward reverse."""

    @staticmethod
    def forward(ctx, xi_in, bvals, sf, batch, precision):
        ctx.cfg = (sf, batch, precision, bvals.shape)
        return qp_equality(sf, xi_in.detach().contiguous(), bvals.detach().contiguous(), batch, precision)

    @staticmethod
    def backward(ctx, g_out):
        sf, batch, precision, bshape = ctx.cfg
        g_out = g_out.contiguous()
        g_in = torch.empty_like(g_out) if ctx.needs_input_grad[0] else None
        g_b = torch.empty(bshape, dtype=g_out.dtype, device=g_out.device) if ctx.needs_input_grad[1] else None
        N.check(N.lib().sf_qp_equality_backward(sf._h, ctypes.byref(sf._batch(batch, g_out).c),
                                                N.PRECISIONS[precision], _ptr(g_out), _ptr(g_in), _ptr(g_b),
                                                _stream_ptr(None)))
        return g_in, g_b, None, None, None


def qp_equality_differentiable(sf: "SafetyFilter", xi_in: torch.Tensor, bvals: torch.Tensor,
                               batch: Optional[Batch] = None, precision: str = "fp32") -> torch.Tensor:
    """The decoders' QP layer as an autograd function: gradients flow to xi_in and bvals."""
    return _QPEquality.apply(xi_in, bvals, sf, batch, precision)


def factor_table(cfg):
    """Host FP64 factor table of one config (no GPU needed); see sf_factor_table."""
    c = N.make_config(cfg)
    need = ctypes.c_int64()
    N.check(N.lib().sf_factor_table(ctypes.byref(c), None, 0, ctypes.byref(need)))
    buf = (ctypes.c_double * need.value)()
    N.check(N.lib().sf_factor_table(ctypes.byref(c), buf, need.value, ctypes.byref(need)))
    vals = list(buf)
    hdr, tab = vals[:16], vals[16:]
    m, mf, H, n = (int(x) for x in hdr[:4])
    offs = [int(x) for x in hdr[4:10]]
    import numpy as np
    t = np.array(tab)
    return {
        "basis": t[offs[0]:offs[0] + 3 * H * m].reshape(3, H, m),
        "X1": t[offs[1]:offs[1] + mf * mf].reshape(mf, mf),
        "X01": t[offs[2]:offs[2] + mf * mf].reshape(mf, mf),
        "Bmap": t[offs[3]:offs[3] + 36].reshape(6, 6),
        "Gfx": t[offs[4]:offs[4] + 6 * mf].reshape(mf, 6),
        "Rfx": t[offs[5]:offs[5] + 6 * mf].reshape(mf, 6),
        "m": m, "mf": mf, "H": H, "n": n,
    }


class _SFProject(torch.autograd.Function):
    """sf_project in the forward pass, sf_project_backward (hand-written adjoint through the
    unrolled iterations, with checkpoints) in the backward pass."""

    @staticmethod
    def forward(ctx, xi0, lam0, xi_bar, bvals, sf, batch, iters, ckpt_every, precision):
        out = sf.project(xi_bar.detach(), bvals.detach(), iters, batch=batch, precision=precision,
                         xi0=xi0.detach(), lam0=lam0.detach(), ckpt_every=ckpt_every, fp_residual=True)
        ctx.save_for_backward(xi_bar.detach(), bvals.detach(), out.ckpt)
        ctx.cfg = (sf, batch, iters, ckpt_every, precision)
        return out.xi, out.lam, out.resid[:, 0].contiguous(), out.resid[:, 2].contiguous()

    @staticmethod
    def backward(ctx, g_xi, g_lam, g_res, g_fpr):
        xi_bar, bvals, ckpt = ctx.saved_tensors
        sf, batch, iters, ckpt_every, precision = ctx.cfg
        c = lambda t: None if t is None else t.contiguous()
        g = sf.project_backward(xi_bar, bvals, iters, ckpt, ckpt_every, g_xi_out=c(g_xi), g_lam_out=c(g_lam),
                                g_resid=c(g_res), w_fpr=c(g_fpr), batch=batch, precision=precision)
        return g["xi0"], g["lam0"], g["xi_bar"], None, None, None, None, None, None


def project_differentiable(sf: SafetyFilter, xi_bar: torch.Tensor, bvals: torch.Tensor, iters: int,
                           xi0: Optional[torch.Tensor] = None, lam0: Optional[torch.Tensor] = None,
                           ckpt_every: int = 10, batch: Optional[Batch] = None, precision: str = "fp32"):
    """Differentiable SF: returns (xi_K, lambda_K, ||r_p^K||^2 per sample, and the fixed-point
    residual sum_k ||z^{k+1} - z^k||^2 per sample, the first term of eq. (NN_loss)); gradients
    flow to xi0, lam0 and xi_bar through the adjoint kernel.  xi0 = None starts from xi_bar (its
    gradient then adds to xi_bar's), lam0 = None starts from zero."""
    if xi0 is None:
        xi0 = xi_bar
    if lam0 is None:
        lam0 = torch.zeros_like(xi_bar)
    return _SFProject.apply(xi0, lam0, xi_bar, bvals, sf, batch, int(iters), int(ckpt_every), precision)
