"""Host logic of the benchmark (no GPU): the algorithmic work counts, the roofline formula and the
equal-residual search."""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402
import workloads as W  # noqa: E402


def test_work_counts_of_the_benchmarked_shapes():
    # 16 robots, 3D, degree 10, 100 steps: contractions / elementwise / reciprocal square roots
    assert bench.flops_split(W.cfg_swarm(16)) == (509_760, 291_600, 15_200)
    # 32 robots, degree 12, 120 steps
    assert bench.flops_split(W.cfg_swarm(32, degree=12, horizon=120)) == (1_718_400, 1_345_440, 67_200)
    # every term written out for a small shape: n = 3, D = 3, m = 8 (m_f = 2), H = 10, N_p = 3
    c = W.SwarmConfig(n_robots=3, dims=3, degree=7, horizon=10, t_final=1.0, safety_a=0.3, safety_b=0.3,
                      vmax=1.0, amax=1.0)
    dense = 6 * 3 * 3 * 10 * 8 + 6 * 3 * 3 * 10 * 2 + 4 * 3 * 3 * 8 * 2 + 2 * 3 * (3 * 2) ** 2
    elem = 15 * 3 * 10 + 24 * 3 * 10 + 2 * 3 * 10 * 3 + 5 * 3 * 3 * 2
    assert bench.flops_split(c) == (dense, elem, 3 * 10 + 2 * 3 * 10)


def test_roofline_takes_the_binding_term():
    c = W.cfg_swarm(16)
    # bf16: the vector term binds (0.688 ms floor at 1024 x 300), the MFMA term needs 0.063 ms
    r = bench.roofline([(c, 1024)], 300, 1.376, "bf16", None)
    assert r["bound"] == "alu" and r["peak"] == 157.3
    assert r["frac"] == pytest.approx(0.5, abs=1e-3)
    assert r["terms"]["mfma"]["frac"] < r["frac"]
    # fp32: the fp32-MFMA term binds (0.995 ms floor)
    r = bench.roofline([(c, 1024)], 300, 1.99, "fp32", None)
    assert r["bound"] == "mfma" and r["frac"] == pytest.approx(0.5, abs=1e-3)
    # the generic kernel and FP64 put everything on the vector ALUs
    r = bench.roofline([(c, 1024)], 300, 100.0, "fp64", None)
    assert list(r["terms"]) == ["valu"] and r["peak"] == 78.6


def test_equal_residual_search_takes_the_first_k_meeting_every_criterion(monkeypatch):
    """K from k0 upward; each K must reach the reference's converged count and stay at or below
    its p99 and maximum violation."""
    import types
    trials = {300: (990, 2e-3, 6e-3), 301: (995, 1e-3, 6e-3), 302: (995, 1e-3, 5e-3), 303: (999, 1e-4, 1e-4)}

    class Out:
        def __init__(self, k):
            self.xi = k

    class SF:
        def project(self, xb, bv, K, precision, want_lam):
            return Out(K)
    monkeypatch.setattr(bench, "feasibility_stats", lambda sf, xi, bv, prec: trials[xi])
    fake_torch = types.SimpleNamespace(cuda=types.SimpleNamespace(synchronize=lambda: None))
    monkeypatch.setitem(sys.modules, "torch", fake_torch)
    k, crit, first, tried = bench.equal_residual_iters(SF(), None, None, "bf16", 300, (995, 1e-3, 5e-3), 310)
    assert k == 302 and all(crit.values()) and first.xi == 300 and len(tried) == 3
    k, crit, _, _ = bench.equal_residual_iters(SF(), None, None, "bf16", 300, (1000, 0.0, 0.0), 303)
    assert k is None and not crit["converged"]


def test_counter_and_traffic_summaries_count_only_for_the_current_source(tmp_path, monkeypatch):
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "fast_project_counters_swarm16.txt").write_text(
        "# header\nkernel_source_sha256: abc\n\n## k<1>: bf16 operands, K = 319\nvalu_busy_pct: 64.8\n"
        "mfma_busy_pct: 5.6\nlds_bank_conflict_pct_of_cu_cycles: 15.8\n\n## k<0>: fp32 operands, K = 300\n"
        "valu_busy_pct: 57.1\nmfma_busy_pct: 13.4\nlds_bank_conflict_pct_of_cu_cycles: 13.2\n")
    (tmp_path / "profiles" / "fast_project_traffic_swarm16_bf16.txt").write_text(
        "# c\nkernel_source_sha256: abc\nfetch_kib_per_dispatch: 10\nwrite_kib_per_dispatch: 4\n"
        "fetch_scale: 2.0\nwrite_scale: 1.0\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_digest", lambda: "abc")
    c = bench.measured_counters("swarm16", "fp32")
    assert c["valu_busy_pct"] == 57.1 and c["mfma_busy_pct"] == 13.4
    assert bench.measured_counters("swarm16", "bf16")["lds_bank_conflict_pct_of_cu_cycles"] == 15.8
    assert bench.measured_traffic("swarm16", "bf16") == 24 * 1024
    monkeypatch.setattr(bench, "kernel_source_digest", lambda: "other")
    assert bench.measured_counters("swarm16", "fp32") is None
    assert bench.measured_traffic("swarm16", "bf16") is None


def test_bench_functions_use_no_undefined_names():
    """Static check (the GPU legs cannot run here): every global name a function of bench.py reads
    is defined at module level or a builtin."""
    import builtins
    import symtable
    src = open(os.path.join(ROOT, "bench.py")).read()
    top = symtable.symtable(src, "bench.py", "exec")
    defined = set(top.get_identifiers())
    missing = []

    def walk(t):
        for ch in t.get_children():
            if ch.get_type() == "function":
                for s in ch.get_symbols():
                    nm = s.get_name()
                    if s.is_global() and not s.is_assigned() and nm not in defined and not hasattr(builtins, nm):
                        missing.append((ch.get_name(), nm))
            walk(ch)
    walk(top)
    assert not missing, missing
