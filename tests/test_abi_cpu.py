"""CPU tests of the C ABI: the library loads, exports every symbol the header declares,
and its host-side FP64 factorisation agrees with the oracle's dense KKT matrix."""
import ctypes
import os
import re

import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from paper_2501_19042_amd import _native as N
from paper_2501_19042_amd import factor_table

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "swarmsf.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:sf_status|void|const char\*)\s+(sf_\w+)\s*\(", src, flags=re.M)))


def test_library_exports_every_declared_symbol():
    names = declared_functions()
    assert set(names) == set(N.EXPORTED)
    lib = N.lib()
    for nm in names:
        assert hasattr(lib, nm), nm


def test_header_struct_layout_matches_binding():
    assert ctypes.sizeof(N.SfConfig) == 4 * 4 + 14 * 8
    assert N.SfConfig.t_final.offset == 16
    assert N.SfConfig.ws_a.offset == 16 + 8 * 8 and N.SfConfig.ws_z.offset == 16 + 13 * 8


CFGS = [
    W.cfg_tiny2d(),
    W.cfg_swarm(16),
    W.cfg_swarm(32, degree=12, horizon=120),
    W.SwarmConfig(n_robots=3, dims=3, degree=7, horizon=12, t_final=4.0, safety_a=0.3, safety_b=0.5,
                  vmax=1.5, amax=0.0, rho_coll=0.7, rho_vel=1.3, rho_acc=1.0),
    W.SwarmConfig(n_robots=4, dims=3, degree=9, horizon=20, t_final=6.0, safety_a=0.3, safety_b=0.3,
                  vmax=1.5, amax=2.0, rho_coll=0.8, rho_vel=1.0, rho_acc=1.1,
                  ws_a=2.0, ws_b=0.8, rho_ws=0.6, ws_x=0.3, ws_y=-0.2, ws_z=0.1),
]


@pytest.mark.parametrize("cfg", CFGS, ids=["tiny2d", "n16", "n32deg12", "spheroid_novacc", "workspace"])
def test_factor_table_matches_dense_kkt(cfg):
    ft = factor_table(cfg)
    s = O.build_system(cfg)
    m, mf, n = ft["m"], ft["mf"], cfg.n_robots
    # basis rows: independent C++ and Python constructions of the Bernstein matrices
    assert np.allclose(ft["basis"][0], s.P.numpy(), atol=1e-15)
    assert np.allclose(ft["basis"][1], s.Pd.numpy(), atol=1e-12)
    assert np.allclose(ft["basis"][2], s.Pdd.numpy(), atol=1e-11)
    # free-coefficient block of the inverse KKT matrix
    nm = n * m
    K = torch.zeros(nm + 6 * n, nm + 6 * n, dtype=torch.float64)
    K[:nm, :nm] = torch.eye(nm, dtype=torch.float64) + s.F.T @ (s.w[:, None] * s.F)
    K[:nm, nm:] = s.A.T
    K[nm:, :nm] = s.A
    Kinv = torch.linalg.inv(K).numpy()[:nm, :nm]
    free = [i * m + 3 + f for i in range(n) for f in range(mf)]
    S_dense = Kinv[np.ix_(free, free)]
    J = np.full((n, n), 1.0 / n)
    S_struct = np.kron(J, ft["X1"] + ft["X01"]) + np.kron(np.eye(n) - J, ft["X1"])
    assert np.allclose(S_dense, S_struct, atol=1e-12, rtol=1e-10)
    # K^-1 is zero on pinned rows (the boundary rows fix them completely)
    fixed = [i * m + k for i in range(n) for k in (0, 1, 2, m - 3, m - 2, m - 1)]
    assert np.abs(Kinv[np.ix_(fixed, fixed)]).max() < 1e-12
    # pinned coefficients from boundary values
    A1 = s.A.numpy()[:6, :m]
    fx = [0, 1, 2, m - 3, m - 2, m - 1]
    assert np.allclose(ft["Bmap"] @ A1[:, fx], np.eye(6), atol=1e-10)
    # free x pinned coupling of F^T W F: diagonal robot blocks rho_c (n-1) G + Rm, others -rho_c G
    G = (s.F.T @ (s.w[:, None] * s.F)).numpy()
    rc = cfg.rho_coll
    for i in (0, n - 1):
        for j in (0, 1):
            blk = G[np.ix_([i * m + 3 + f for f in range(mf)], [j * m + k for k in fx])]
            expect = (rc * n * ((i == j) - 1.0 / n)) * ft["Gfx"] + (i == j) * ft["Rfx"]
            assert np.allclose(blk, expect, atol=1e-10, rtol=1e-12)


@pytest.mark.parametrize("field,value,code", [
    ("n_robots", 1, N.SF_EINVAL), ("dims", 4, N.SF_EINVAL), ("degree", 4, N.SF_EINVAL),
    ("horizon", 5, N.SF_EINVAL), ("t_final", 0.0, N.SF_EINVAL), ("safety_a", 0.0, N.SF_EINVAL),
    ("rho_coll", 0.0, N.SF_EINVAL), ("n_robots", 65, N.SF_EUNSUPPORTED), ("degree", 31, N.SF_EUNSUPPORTED),
    ("horizon", 4097, N.SF_EUNSUPPORTED),
])
def test_factor_table_rejects_bad_configs(field, value, code):
    c = N.make_config(W.cfg_swarm(16))
    setattr(c, field, value)
    need = ctypes.c_int64()
    rc = N.lib().sf_factor_table(ctypes.byref(c), None, 0, ctypes.byref(need))
    assert rc == code
    assert len(N.lib().sf_last_error()) > 0


@pytest.mark.parametrize("field,value", [("ws_b", 0.0), ("rho_ws", 0.0), ("ws_x", float("nan"))])
def test_factor_table_rejects_bad_workspace(field, value):
    base = N.make_config(CFGS[-1])
    need = ctypes.c_int64()
    assert N.lib().sf_factor_table(ctypes.byref(base), None, 0, ctypes.byref(need)) == N.SF_OK
    setattr(base, field, value)
    assert N.lib().sf_factor_table(ctypes.byref(base), None, 0, ctypes.byref(need)) == N.SF_EINVAL
    # with the workspace off (ws_a <= 0) its other fields are ignored
    base.ws_a = 0.0
    assert N.lib().sf_factor_table(ctypes.byref(base), None, 0, ctypes.byref(need)) == N.SF_OK


def test_factor_table_capacity_check():
    c = N.make_config(W.cfg_tiny2d())
    need = ctypes.c_int64()
    assert N.lib().sf_factor_table(ctypes.byref(c), None, 0, ctypes.byref(need)) == N.SF_OK
    buf = (ctypes.c_double * 4)()
    assert N.lib().sf_factor_table(ctypes.byref(c), buf, 4, ctypes.byref(need)) == N.SF_EINVAL


def test_null_arguments_are_errors_not_crashes():
    L = N.lib()
    assert L.sf_setup(None, 0, None) == N.SF_EINVAL
    assert L.sf_project(None, None, 1, None, None, None, None, 1, None, None, None, None, 0, None, 0, None) == N.SF_EINVAL
    assert L.sf_feasibility(None, None, 1, None, None, None, None) == N.SF_EINVAL
    L.sf_destroy(None)


@pytest.mark.parametrize("source", ["sf_generic.hip", "sf_fast_p1_w0.hip"])
def test_sample_status_logic_on_the_host(tmp_path, source):
    """The per-sample status bits (non-finite input, non-finite result, not converged against the
    tolerance) and the NaN/infinity bit tests the kernels use, compiled for the host with the
    optimisation and floating-point flags of each kernel source (the MFMA kernels assume no NaNs,
    under which a plain bit test for NaN can be folded away) and run."""
    import subprocess
    from paper_2501_19042_amd import build as B
    exe = tmp_path / "status_logic"
    csrc = os.path.join(ROOT, "paper_2501_19042_amd", "csrc")
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    flags = [f for f in B.FLAGS if f not in ("-fPIC",)] + B.FILE_FLAGS.get(source, [])
    subprocess.run([hipcc] + flags + ["-I", os.path.join(ROOT, "include"), "-I", csrc,
                    "-o", str(exe), os.path.join(ROOT, "tests", "status_logic.cpp")], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    assert r.returncode == 0 and r.stdout.strip().splitlines()[-1] == "0", r.stdout
