"""Writes stored expected values by calling the CPU oracle only.

    python tests/golden/make_golden.py elastic3d_spheres_128
    python tests/golden/make_golden.py conduction3d_grf_256

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


def conduction3d_grf(seed=0, eta=1e-8, nsample=256):
    """256^3 heat conduction, k = exp of a periodic Gaussian random field, 3
    unit gradients, PCG to eta = 1e-8.  The assembled CSR K (about 5 GB) is
    the operator; the preconditioner is the oracle's FFT form (Alg. 2 symbol
    from the impulse response of Kref, numpy FFT as the transform), which the
    pins tie to the dense-DFT form on small grids.  Besides C_hom and the
    iteration counts, the fluctuation of every load is stored at `nsample`
    seeded nodes."""
    from oracle.precond import FFTPreconditioner
    t0 = time.time()
    wl = workload("conduction3d_grf", seed=seed)
    n = tuple(wl["n"][:3])
    prob = Problem(n, "scalar", "hex8", kfield=wl["kfield"])
    Cref = oracle.mean_material(prob)
    print("assemble", flush=True)
    K = oracle.assemble_stiffness(prob)
    print("symbol", time.time() - t0, flush=True)
    M = FFTPreconditioner(prob, Cref)
    print("solve", time.time() - t0, flush=True)
    H, sols, res = oracle.homogenize(prob, wl["loads"], eta, Cref=Cref, K=K, M=M)
    nodes = np.sort(np.random.default_rng(17).choice(prob.N, nsample, replace=False))
    out = dict(workload="conduction3d_grf", n=list(n), seed=seed, eta=eta,
               kfield_sha256=sha(np.asarray(wl["kfield"], dtype=np.float64)),
               Cref=Cref.tolist(), C_hom=H.tolist(),
               iterations=[r.iterations for r in res],
               final_rel=[r.history[-1] if r.history else 0.0 for r in res],
               u_rms=[float(np.sqrt(np.mean(s * s))) for s in sols],
               sample_nodes=nodes.tolist(),
               u_samples=[s[nodes].tolist() for s in sols],
               oracle_seconds=time.time() - t0,
               source="oracle.homogenize (assembled CSR K, FFT-form Kref pseudo-inverse, PCG)")
    path = os.path.join(HERE, f"conduction3d_grf_256_seed{seed}.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path, out["iterations"], flush=True)


if __name__ == "__main__":
    what = sys.argv[1] if len(sys.argv) > 1 else "elastic3d_spheres_128"
    if what == "elastic3d_spheres_128":
        elastic3d_spheres(128, 0)
    elif what == "elastic3d_spheres_64":
        elastic3d_spheres(64, 0)
    elif what == "conduction3d_grf_256":
        conduction3d_grf(0)
    else:
        raise SystemExit(f"unknown fixture {what}")
