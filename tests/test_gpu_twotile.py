"""The MFMA kernel with two robot tiles (17-32 robots) at every waves-per-sample choice, against the
FP64 oracle, on shapes that exercise its LDS plan: robot counts that leave phantom robots in the
second tile, degree 15 (every entry of the 16-bit operand rows in use), and horizons whose time
tiles fill each wave's share unevenly (one tile per wave, and a last wave with fewer tiles), so the
boxes of a wave's last tile run past its pair lists and the pair table is rewritten into those
regions for the final residual."""
import numpy as np
import pytest
import torch

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

BOUND = {"fp32": 1e-4, "bf16": 2e-3, "fp16": 2e-4}


@pytest.fixture(scope="module")
def P():
    import paper_2501_19042_amd as P
    torch.cuda.set_device(0)
    return P


@pytest.mark.parametrize("n,degree,H", [(17, 12, 30), (25, 15, 70), (32, 10, 130)])
def test_two_tile_shapes_match_oracle(P, tmp_path, monkeypatch, n, degree, H):
    S, iters = 3, 40
    p = W.small3d(n_robots=n, n_samples=S, degree=degree, horizon=H, seed=500 + n,
                  box=((-3.0, -3.0, -1.0), (3.0, 3.0, 1.0)), t_final=10.0)
    s = O.build_system(p.cfg)
    rx, _, rr = O.sf_project(s, torch.tensor(p.xi_bar), torch.tensor(p.bvals), iters)
    xb = torch.tensor(p.xi_bar, dtype=torch.float32).cuda()
    bv = torch.tensor(p.bvals, dtype=torch.float32).cuda()
    cache = tmp_path / "tune.jsonl"
    monkeypatch.setenv("SWARMSF_TUNE_CACHE", str(cache))
    for prec in ("fp32", "bf16", "fp16"):
        cache.write_text("")
        P.SafetyFilter([p.cfg]).project(xb, bv, 5, precision=prec, autotune=True)
        torch.cuda.synchronize()
        key = [l for l in cache.read_text().splitlines() if '"key"' in l][-1].split('"key": "')[1].split('"')[0]
        for w in (2, 3, 4):
            cache.write_text('{"key": "%s", "waves": %d, "grid": 0, "ms": 1.0}\n' % (key, w))
            print(f"case two-tile n={n} deg={degree} H={H} {prec} W={w}", flush=True)
            out = P.SafetyFilter([p.cfg]).project(xb, bv, iters, precision=prec, autotune=True)
            torch.cuda.synchronize()
            g = out.xi.cpu().double().reshape(S, -1)
            e = ((g - rx.reshape(S, -1)).abs().amax(1) / rx.reshape(S, -1).abs().amax(1)).numpy()
            print(f"  max rel err {e.max():.2e}", flush=True)
            assert e.max() <= BOUND[prec], (prec, w, e)
            # the final residual (pair table rewritten into the pair-list regions) against the
            # oracle's; the 16-bit forms' iterates differ by up to their bound, so their residuals
            # get a proportionally looser tolerance
            tol = dict(rtol=2e-2, atol=1e-6) if prec == "fp32" else dict(rtol=0.25, atol=1e-4)
            assert torch.allclose(out.resid.cpu().double(), rr, **tol), (prec, w, out.resid, rr)


def test_two_tile_persistent_class_mixed_shapes(P, tmp_path, monkeypatch):
    """One persistent launch over 17-32-robot problems of different degrees and horizons (so each
    work item has its own LDS plan inside the class kernel), at three and four waves per sample
    pinned through the autotuner's cache, against the oracle."""
    probs = [W.small3d(n_robots=n, n_samples=S, degree=deg, horizon=H, seed=600 + k,
                       box=((-3.0, -3.0, -1.0), (3.0, 3.0, 1.0)), t_final=10.0)
             for k, (n, deg, H, S) in enumerate([(20, 8, 40, 2), (32, 12, 100, 2), (27, 15, 130, 1)])]
    iters = 30
    refs = []
    for p in probs:
        s = O.build_system(p.cfg)
        refs.append(O.sf_project(s, torch.tensor(p.xi_bar), torch.tensor(p.bvals), iters)[0])
    xb = torch.cat([torch.tensor(p.xi_bar, dtype=torch.float32).reshape(-1) for p in probs]).cuda()
    bv = torch.cat([torch.tensor(p.bvals, dtype=torch.float32).reshape(-1) for p in probs]).cuda()
    batch = P.Batch([(i, p.xi_bar.shape[0]) for i, p in enumerate(probs)])
    cache = tmp_path / "tune.jsonl"
    monkeypatch.setenv("SWARMSF_TUNE_CACHE", str(cache))
    for prec in ("fp32", "bf16"):
        cache.write_text("")
        P.SafetyFilter([p.cfg for p in probs]).project(xb, bv, 5, batch=batch, precision=prec, autotune=True)
        torch.cuda.synchronize()
        keys = sorted({l.split('"key": "')[1].split('"')[0] for l in cache.read_text().splitlines()})
        assert len(keys) == 1 and keys[0].endswith(":c0"), keys
        for w in (3, 4):
            cache.write_text('{"key": "%s", "waves": %d, "grid": 0, "ms": 1.0}\n' % (keys[0], w))
            print(f"case two-tile persistent {prec} W={w}", flush=True)
            out = P.SafetyFilter([p.cfg for p in probs]).project(xb, bv, iters, batch=batch, precision=prec,
                                                                 autotune=True)
            torch.cuda.synchronize()
            assert len(cache.read_text().splitlines()) == 1
            o = 0
            for p, rx in zip(probs, refs):
                S = p.xi_bar.shape[0]
                g = out.xi[o:o + p.xi_bar.size].reshape(rx.shape).cpu().double()
                e = ((g - rx).abs().reshape(S, -1).amax(1) / rx.abs().reshape(S, -1).amax(1)).numpy()
                print(f"  n={p.cfg.n_robots} deg={p.cfg.degree} H={p.cfg.horizon}: max rel err {e.max():.2e}", flush=True)
                assert e.max() <= BOUND[prec], (prec, w, p.cfg.n_robots, e)
                o += p.xi_bar.size


def test_two_tile_workspace_rows_match_oracle(P, tmp_path, monkeypatch):
    """The two-tile workspace instances (two and three waves per sample), whose boxes share the
    pair-list region while the workspace residuals go to the tile accumulator, against the oracle."""
    from dataclasses import replace
    S, iters = 2, 40
    p = W.small3d(n_robots=25, n_samples=S, degree=10, horizon=50, seed=700,
                  box=((-2.5, -2.5, -0.8), (2.5, 2.5, 0.8)), t_final=8.0)
    cfg = replace(p.cfg, ws_a=2.6, ws_b=0.7, ws_x=0.1)
    s = O.build_system(cfg)
    rx, _, _ = O.sf_project(s, torch.tensor(p.xi_bar), torch.tensor(p.bvals), iters)
    xb = torch.tensor(p.xi_bar, dtype=torch.float32).cuda()
    bv = torch.tensor(p.bvals, dtype=torch.float32).cuda()
    cache = tmp_path / "tune.jsonl"
    monkeypatch.setenv("SWARMSF_TUNE_CACHE", str(cache))
    for prec in ("fp32", "bf16"):
        cache.write_text("")
        P.SafetyFilter([cfg]).project(xb, bv, 5, precision=prec, autotune=True)
        torch.cuda.synchronize()
        key = [l for l in cache.read_text().splitlines() if '"key"' in l][-1].split('"key": "')[1].split('"')[0]
        for w in (2, 3):
            cache.write_text('{"key": "%s", "waves": %d, "grid": 0, "ms": 1.0}\n' % (key, w))
            print(f"case two-tile workspace {prec} W={w}", flush=True)
            out = P.SafetyFilter([cfg]).project(xb, bv, iters, precision=prec, autotune=True)
            torch.cuda.synchronize()
            g = out.xi.cpu().double().reshape(S, -1)
            e = ((g - rx.reshape(S, -1)).abs().amax(1) / rx.reshape(S, -1).abs().amax(1)).numpy()
            print(f"  max rel err {e.max():.2e}", flush=True)
            assert e.max() <= BOUND[prec], (prec, w, e)
