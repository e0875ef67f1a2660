"""Writes the stored expected values under tests/golden/ from the FP64 oracle alone.

The paper prints no worked numeric example of the safety filter, so every stored value here
is the oracle's, produced by this script (which calls nothing but `oracle/` and the seeded
input generators).  The fixtures guard the oracle against silent change and give the GPU
tests a reference that needs no oracle run.

    python tests/golden/make_golden.py            # writes the fixtures that are missing
    python tests/golden/make_golden.py --force    # rewrites all of them
"""
import json
import os
import sys
from dataclasses import replace

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import torch  # noqa: E402

import oracle as O  # noqa: E402
import workloads as W  # noqa: E402


def cases():
    """(name, cfg, xi_bar, bvals, iters): small cases the oracle finishes in well under a second."""
    t2 = W.tiny2d(2).problems[0]
    yield "tiny2d_2x60", t2.cfg, t2.xi_bar[:2], t2.bvals, 60
    s3 = W.small3d(n_robots=5, n_samples=2, degree=10, horizon=40, seed=11)
    yield "small3d_n5_2x40", s3.cfg, s3.xi_bar, s3.bvals, 40
    s6 = W.small3d(n_robots=6, n_samples=1, degree=7, horizon=24, seed=23)
    yield "small3d_n6_deg7_1x25", s6.cfg, s6.xi_bar, s6.bvals, 25
    # the workspace rows of eq. (f_e): an off-centre spheroid that the sampled trajectories leave
    cw = replace(s3.cfg, ws_a=1.6, ws_b=0.55, ws_x=0.1, ws_y=-0.05, ws_z=0.05, rho_ws=0.8)
    yield "small3d_n5_ws_2x40", cw, s3.xi_bar, s3.bvals, 40


def cfg_dict(cfg):
    keys = ["n_robots", "dims", "degree", "horizon", "t_final", "safety_a", "safety_b", "vmax", "amax",
            "rho_coll", "rho_vel", "rho_acc"]
    if cfg.ws_a > 0:
        keys += ["ws_a", "ws_b", "rho_ws", "ws_x", "ws_y", "ws_z"]
    return {k: getattr(cfg, k) for k in keys}


def main():
    torch.set_num_threads(1)
    force = "--force" in sys.argv[1:]
    for name, cfg, xb, bv, iters in cases():
        path = os.path.join(HERE, f"oracle_{name}.json")
        if os.path.exists(path) and not force:
            continue
        s = O.build_system(cfg)
        xbt = torch.as_tensor(xb, dtype=torch.float64)
        bvt = torch.as_tensor(bv, dtype=torch.float64)
        xi, lam, resid = O.sf_project(s, xbt, bvt, iters)
        viol = O.feasibility(s, xi, bvt)
        out = {
            "source": "FP64 CPU oracle (oracle/sf_oracle.py), written by tests/golden/make_golden.py",
            "name": name, "cfg": cfg_dict(cfg), "iters": iters,
            "xi_bar": xbt.tolist(), "bvals": bvt.tolist(),
            "xi": xi.tolist(), "lam": lam.tolist(), "resid": resid.tolist(), "viol": viol.tolist(),
        }
        with open(path, "w") as f:
            json.dump(out, f, separators=(",", ":"))
        print(path, os.path.getsize(path), "bytes")


if __name__ == "__main__":
    main()
