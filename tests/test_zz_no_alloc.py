"""The allocation-free entry point sf_qp_equality_backward_noalloc against sf_qp_equality_backward,
through the C ABI: bit for bit (both are deterministic and share the kernels and the chunking), on
two calls in a row (the second with a smaller batch, which must not see the first call's leftovers
in the shared array), in FP32 and FP64; and batches past its limits are refused before any launch,
leaving the handle usable."""
import ctypes
from dataclasses import replace

import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_2501_19042_amd as P
    torch.cuda.set_device(0)
    return P


def _say(msg):
    print(msg, flush=True)


def configs():
    a = W.cfg_swarm(16)
    b = replace(W.cfg_swarm(8), degree=12)
    c = replace(W.cfg_swarm(5), degree=7, horizon=40)
    return [a, b, c]


def sizes(cfgs, entries):
    coef = sum(cnt * cfgs[s].n_robots * cfgs[s].dims * (cfgs[s].degree + 1) for s, cnt in entries)
    bnd = sum(cfgs[s].n_robots * cfgs[s].dims * 6 for s, _ in entries)
    return coef, bnd


def both(P, sf, cfgs, entries, prec, seed):
    from paper_2501_19042_amd import _native as N
    dt = torch.float64 if prec == "fp64" else torch.float32
    coef, bnd = sizes(cfgs, entries)
    g = torch.Generator(device="cuda").manual_seed(seed)
    gout = torch.randn(coef, generator=g, dtype=dt, device="cuda")
    batch = P.Batch(entries)
    res = []
    for fn in (N.lib().sf_qp_equality_backward, N.lib().sf_qp_equality_backward_noalloc):
        gin = torch.full((coef,), float("nan"), dtype=dt, device="cuda")
        gb = torch.full((bnd,), float("nan"), dtype=dt, device="cuda")
        N.check(fn(sf._h, ctypes.byref(batch.c), N.PRECISIONS[prec], gout.data_ptr(), gin.data_ptr(), gb.data_ptr(),
                   None))
        torch.cuda.synchronize()
        res.append((gin, gb))
    return res


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_noalloc_equals_allocating_entry_point(P, prec):
    cfgs = configs()
    sf = P.SafetyFilter(cfgs)
    first = [(0, 3000), (1, 517), (2, 9), (0, 70)]      # about 90 chunks over four problems
    second = [(2, 3), (0, 40)]                          # smaller: fewer problems and chunks
    for k, entries in enumerate((first, second)):
        _say(f"case no-alloc {prec} call {k + 1} batch {entries}")
        (gi_a, gb_a), (gi_b, gb_b) = both(P, sf, cfgs, entries, prec, seed=11 + k)
        assert torch.isfinite(gb_a).all() and torch.isfinite(gi_a).all()
        assert torch.equal(gi_a, gi_b)
        assert torch.equal(gb_a, gb_b)


def test_noalloc_refuses_past_its_limits(P):
    from paper_2501_19042_amd import _native as N
    cfgs = configs()
    sf = P.SafetyFilter(cfgs)
    L = N.lib()
    buf = torch.zeros(64, dtype=torch.float32, device="cuda")
    _say("case no-alloc limits")
    # 65 problems
    many = P.Batch([(2, 1)] * 65)
    assert L.sf_qp_equality_backward_noalloc(sf._h, ctypes.byref(many.c), N.SF_FP32, buf.data_ptr(), buf.data_ptr(),
                                             buf.data_ptr(), None) == N.SF_EUNSUPPORTED
    assert b"64 problems" in L.sf_last_error()
    # tables and partial sums past 16 MiB: 2^20 samples of 16 robots (refused before reading anything)
    big = P.Batch([(0, 1 << 20)])
    assert L.sf_qp_equality_backward_noalloc(sf._h, ctypes.byref(big.c), N.SF_FP32, buf.data_ptr(), buf.data_ptr(),
                                             buf.data_ptr(), None) == N.SF_EUNSUPPORTED
    assert b"scratch" in L.sf_last_error()
    # the handle still works
    (gi_a, gb_a), (gi_b, gb_b) = both(P, sf, cfgs, [(1, 33)], "fp32", seed=5)
    assert torch.equal(gi_a, gi_b) and torch.equal(gb_a, gb_b)
