"""What the trained network gains: flexible CG with the learned preconditioner
against Jacobi-PCG and plain CG on held-out Gauss-Newton systems of the
workload it was trained on (the committed parameters)."""
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
    assert s["learned_iters_mean"] < s["jacobi_iters_mean"]
    assert s["learned_iters_mean"] < s["cg_iters_mean"]
