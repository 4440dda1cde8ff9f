"""Write the FP64 oracle's full two-level solve of the head-sized workload
(512x512x70, 40 views, 512x384 detector, seeded random-ellipsoid head,
Poisson I0 = 5e4, mu = 1e-3, 20 + 20 iterations), for the GPU parity test
at full size:

  head40_fbs.json    beta and inner counts per level (the oracle's own:
                     30 power-iteration steps), the energies of the result,
                     its norm, the L2 norm and the sum of every z plane, and
                     the result at 4096 seeded voxels of the field of view
                     where the phantom is not air;
  head40_slices.npz  whole axial planes z = 0, 10, 35, 60, 69 of the result
                     (float32), the first and last planes included.

Calls only oracle/ and the seeded input generators.

    OMP_NUM_THREADS=8 python tests/golden/make_head_fbs.py   (~80 min on 8 cores)
"""

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from workloads import head_case, fov_mask  # noqa: E402

N_SAMPLES = 4096
SAMPLE_SEED = 4242
SLICES = (0, 10, 35, 60, 69)
JSON_NAME = "head40_fbs.json"
SLICE_NAME = "head40_slices.npz"


def sample_indices(case):
    """Seeded voxel indices (flat, x fastest) inside the field of view where
    the voxelised phantom is not air."""
    g = case.geom
    mask = (fov_mask(g) & (case.voxelised() > 0.0)).ravel()
    idx = np.nonzero(mask)[0]
    rng = np.random.default_rng(SAMPLE_SEED)
    return np.sort(rng.choice(idx, size=N_SAMPLES, replace=False))


def main():
    t0 = time.time()
    case = head_case(40, iters=(20, 20))
    g = case.geom
    Y32 = case.Y.astype(np.float32).astype(np.float64)  # what the GPU receives
    out = oracle.fbs_solve(g, Y32, case.mu, list(case.iters), eps=case.eps)
    f = out["f"].reshape(g.vol_shape)
    idx = sample_indices(case)
    res = {
        "workload": "head 512x512x70 @0.88x0.88x2.5, 40 views, 512x384 @0.776, "
                    "SAD/SDD 1000/1500, random-ellipsoid head seed 1001, Poisson I0=5e4 "
                    "seed 2001, mu=1e-3, eps=1e-3, 20+20 iterations",
        "beta": [float(b) for b in out["used_beta"]],
        "n_inner": [int(k) for k in out["used_inner"]],
        "E": float(out["report"][0]),
        "E_eps": float(out["report"][1]),
        "E1": float(out["report"][2]),
        "E2": float(out["report"][3]),
        "sample_seed": SAMPLE_SEED,
        "samples": [float(v) for v in f.ravel()[idx]],
        "f_norm": float(np.linalg.norm(f)),
        "plane_norm": [float(np.linalg.norm(f[k])) for k in range(g.nz)],
        "plane_sum": [float(f[k].sum()) for k in range(g.nz)],
        "slices": list(SLICES),
        "oracle_threads": oracle.threads(),
        "oracle_seconds": time.time() - t0,
    }
    np.savez_compressed(os.path.join(HERE, SLICE_NAME),
                        **{"z%d" % k: f[k].astype(np.float32) for k in SLICES})
    with open(os.path.join(HERE, JSON_NAME), "w") as fh:
        json.dump(res, fh)
    print("wrote %s and %s in %.0f s" % (JSON_NAME, SLICE_NAME, time.time() - t0))


if __name__ == "__main__":
    main()
