"""Stored oracle results under tests/golden/ (written by tests/golden/make_golden.py).

CPU: the oracle still reproduces its stored results (a guard against silent change of its
arithmetic).  GPU: both HIP kernels reproduce them through the C ABI without an oracle run
(FP64 generic kernel elementwise within 1e-9 (1 + |ref|); FP32 MFMA kernel per sample
max|d| / max|ref| <= 1e-4).
"""
import glob
import json
import os

import numpy as np
import pytest
import torch

import oracle as O
import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
FILES = sorted(glob.glob(os.path.join(HERE, "golden", "oracle_*.json")))


def load(path):
    with open(path) as f:
        d = json.load(f)
    cfg = W.SwarmConfig(**d["cfg"])
    arr = {k: torch.tensor(d[k], dtype=torch.float64) for k in ("xi_bar", "bvals", "xi", "lam", "resid", "viol")}
    return d["name"], cfg, d["iters"], arr


def test_golden_files_present():
    assert len(FILES) >= 3


@pytest.mark.parametrize("path", FILES, ids=[os.path.basename(f) for f in FILES])
def test_oracle_reproduces_golden(path):
    name, cfg, iters, g = load(path)
    s = O.build_system(cfg)
    xi, lam, resid = O.sf_project(s, g["xi_bar"], g["bvals"], iters)
    # same arithmetic on a possibly different BLAS thread count: rounding-order differences only
    assert ((xi - g["xi"]).abs() / (1 + g["xi"].abs())).max() < 1e-11
    assert ((lam - g["lam"]).abs() / (1 + g["lam"].abs())).max() < 1e-11
    assert torch.allclose(resid, g["resid"], rtol=1e-8, atol=1e-14)
    viol = O.feasibility(s, xi, g["bvals"])
    nv = g["viol"].shape[1]           # fixtures without the workspace hold its first 4 columns
    assert torch.allclose(viol[:, :nv], g["viol"], rtol=1e-8, atol=1e-12)
    if not s.ws_on:
        assert (viol[:, 4] == 0).all()


@pytest.mark.gpu
@pytest.mark.parametrize("path", FILES, ids=[os.path.basename(f) for f in FILES])
def test_gpu_fp64_matches_golden(path):
    import paper_2501_19042_amd as P
    name, cfg, iters, g = load(path)
    print(f"case golden fp64 {name}", flush=True)
    sf = P.SafetyFilter([cfg])
    out = sf.project(g["xi_bar"].cuda(), g["bvals"].cuda(), iters, precision="fp64")
    torch.cuda.synchronize()
    for k in ("xi", "lam"):
        got = getattr(out, k).cpu()
        err = ((got - g[k]).abs() / (1 + g[k].abs())).max().item()
        assert err <= 1e-9, f"{name} {k}: {err:.3e}"
    assert torch.allclose(out.resid.cpu(), g["resid"], rtol=1e-7, atol=1e-12)
    viol = sf.feasibility(out.xi, g["bvals"].cuda(), precision="fp64").cpu()
    nv = g["viol"].shape[1]
    assert torch.allclose(viol[:, :nv], g["viol"], rtol=1e-6, atol=1e-9)


@pytest.mark.gpu
@pytest.mark.parametrize("path", [f for f in FILES if "small3d" in f],
                         ids=[os.path.basename(f) for f in FILES if "small3d" in f])
def test_gpu_fp32_mfma_matches_golden(path):
    import paper_2501_19042_amd as P
    name, cfg, iters, g = load(path)
    print(f"case golden fp32 mfma {name}", flush=True)
    sf = P.SafetyFilter([cfg])
    out = sf.project(g["xi_bar"].float().cuda(), g["bvals"].float().cuda(), iters, precision="fp32")
    torch.cuda.synchronize()
    got = out.xi.cpu().double().reshape(out.xi.shape[0], -1)
    ref = g["xi"].reshape(got.shape[0], -1)
    rel = ((got - ref).abs().amax(1) / ref.abs().amax(1)).numpy()
    assert np.all(rel <= 1e-4), f"{name}: per-sample rel {rel}"
