"""Run time against iterations and throughput against batch size (the paper reports run time
linear in the iteration count and good scaling with the batch, Sec. V-C).

* Time per call of the MFMA kernel on 16 robots x 1024 samples at K = 60 .. 300: a straight-line
  fit in K explains it (R^2 > 0.99), in fp32 and bf16.
* Throughput at 256 .. 4096 samples (100 iterations): while the GPU is under-filled (fewer samples
  than it holds at once) the time per call grows far less than the batch, so throughput grows with
  it (1024 samples at least twice the rate of 256); past that it stays level (no collapse for large
  batches).
Timings are printed; the bounds leave room for run-to-run noise.
"""
import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_2501_19042_amd as P
    torch.cuda.set_device(0)
    return P


def timed(sf, xb, bv, iters, prec, reps=3, rounds=5):
    """Time per call: the fastest of `rounds` back-to-back groups of `reps` calls (the minimum is the
    figure least disturbed by clock changes and other work on the device)."""
    for _ in range(2):
        sf.project(xb, bv, iters, precision=prec)
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(rounds):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            sf.project(xb, bv, iters, precision=prec)
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1) / reps)
    return best


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_time_is_linear_in_iterations(P, prec):
    p = W.swarm16().problems[0]
    sf = P.SafetyFilter([p.cfg])
    xb = torch.tensor(p.xi_bar, dtype=torch.float32, device="cuda")
    bv = torch.tensor(p.bvals, dtype=torch.float32, device="cuda")
    ks = np.array([60, 120, 180, 240, 300], dtype=float)
    ts = np.array([timed(sf, xb, bv, int(k), prec) for k in ks])
    slope, icept = np.polyfit(ks, ts, 1)
    r2 = 1.0 - ((ts - (slope * ks + icept)) ** 2).sum() / ((ts - ts.mean()) ** 2).sum()
    print(f"{prec}: ms at K {ks.tolist()} = {np.round(ts, 4).tolist()}; {slope * 1e3:.3f} us per iteration, "
          f"intercept {icept:.4f} ms, R^2 {r2:.5f}", flush=True)
    assert slope > 0 and r2 > 0.99, (ts, r2)


def test_throughput_grows_with_the_batch_and_stays_level(P):
    sizes = [256, 512, 1024, 2048, 4096]
    thr = {}
    for S in sizes:
        p = W.swarm16(n_samples=S).problems[0]
        sf = P.SafetyFilter([p.cfg])
        xb = torch.tensor(p.xi_bar, dtype=torch.float32, device="cuda")
        bv = torch.tensor(p.bvals, dtype=torch.float32, device="cuda")
        ms = timed(sf, xb, bv, 100, "bf16")
        thr[S] = S / (ms / 1e3)
        print(f"bf16, {S} samples, 100 iterations: {ms:.4f} ms, {thr[S]:.0f} samples/s", flush=True)
    assert thr[1024] >= 2.0 * thr[256], thr        # 4x the work in less than twice the time
    assert thr[4096] >= 0.8 * thr[1024], thr       # level once the GPU is full
