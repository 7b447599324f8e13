"""Writes stored expected values by calling the CPU oracle only.

    python tests/golden/make_golden.py elastic3d_spheres_128

Each fixture records the seeded input it was computed from (generator name,
seed, size, SHA-256 of the phase grid), the oracle's homogenized tensor and
its PCG iteration counts.  Nothing here touches the GPU library.
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from oracle.assembly import Problem  # noqa: E402
from synth import workload  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def sha(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def elastic3d_spheres(n=128, seed=0, eta=1e-10):
    t0 = time.time()
    wl = workload("elastic3d_spheres", seed=seed, n=n)
    prob = Problem((n,) * 3, "elastic", "hex8", phase=wl["phase"], mat=wl["mat"])
    H, sols, res = oracle.homogenize(prob, wl["loads"], eta)
    out = dict(workload="elastic3d_spheres", n=n, seed=seed, eta=eta,
               phase_sha256=sha(wl["phase"]), vf=wl["vf"],
               Cref=oracle.mean_material(prob).tolist(), C_hom=H.tolist(),
               iterations=[r.iterations for r in res],
               final_rel=[r.history[-1] if r.history else 0.0 for r in res],
               u_rms=[float(np.sqrt(np.mean(s * s))) for s in sols],
               oracle_seconds=time.time() - t0,
               source="oracle.homogenize (assembled CSR K, naive-DFT Kref pseudo-inverse, PCG)")
    path = os.path.join(HERE, f"elastic3d_spheres_{n}_seed{seed}.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path, out["iterations"], flush=True)


if __name__ == "__main__":
    what = sys.argv[1] if len(sys.argv) > 1 else "elastic3d_spheres_128"
    if what == "elastic3d_spheres_128":
        elastic3d_spheres(128, 0)
    elif what == "elastic3d_spheres_64":
        elastic3d_spheres(64, 0)
    else:
        raise SystemExit(f"unknown fixture {what}")
