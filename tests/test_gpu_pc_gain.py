"""What the trained network gains: flexible CG with the learned preconditioner
against Jacobi-PCG and plain CG on held-out Gauss-Newton systems of the
workload it was trained on (the committed parameters): fewer iterations; the
wall time of each solver is measured and reported beside them (the network's
application costs more than an Hv at this size, so fewer iterations need not
mean less time)."""
import os

import numpy as np
import pytest

from gpu_cases import DEV
from paper_1804_10541_amd import pc_train

pytestmark = pytest.mark.gpu


def test_trained_network_needs_fewer_cg_iterations_than_jacobi():
    print("[gpu-case] learned preconditioner gain, held-out seeds 210-211, 8 Gauss-Newton systems each", flush=True)
    assert os.path.exists(pc_train.WEIGHTS), "trained parameters are part of the package"
    params = np.load(pc_train.WEIGHTS)
    rows = pc_train.evaluate(params, [210, 211], gn_iters=8, mix=False, device=DEV)
    s = pc_train.summarize(rows)
    print(f"[gpu-case] {s}", flush=True)
    assert s["not_converged"] == 0
    for r in rows:
        print(f"[gpu-case] seed {r['seed']} GN {r['gn']}: Jacobi {r['jacobi_iters']}, learned {r['learned_iters']}, "
              f"CG {r['cg_iters']}", flush=True)
    print(f"[gpu-case] wall time over {s['systems']} solves: Jacobi-PCG {1e3 * s['jacobi_s']:.1f} ms, "
          f"learned {1e3 * s['learned_s']:.1f} ms, plain CG {1e3 * s['cg_s']:.1f} ms; "
          f"learned / Jacobi {s['learned_s'] / s['jacobi_s']:.2f}x", flush=True)
    assert s["learned_iters_mean"] < s["jacobi_iters_mean"]
    assert s["learned_iters_mean"] < s["cg_iters_mean"]
    assert all(np.isfinite(s[k]) and s[k] > 0 for k in ("jacobi_s", "learned_s", "cg_s"))
