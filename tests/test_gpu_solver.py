"""Gauss-Newton step and multilevel driver on the GPU, checked against the
oracle at the GPU's own iterates (trajectories themselves depend on rounding,
so parity is asserted per iterate: the oracle evaluates J at every u the GPU
produces)."""
import numpy as np
import pytest
import torch

from gpu_cases import DEV, ct_case, rel_l2, to_dev
from oracle import Grid, solver
from paper_1804_10541_amd import mfr
from synth import GridSpec, config_c2

pytestmark = pytest.mark.gpu


def test_gn_steps_decrease_J_and_match_oracle_per_iterate():
    print("[gpu-case] gn steps 64x64x48", flush=True)
    spec, R, T, u, _ = ct_case(2, (64, 64, 48), (17, 17, 13), amp=0.0, n_probes=0)
    ctx = mfr.Context(spec, DEV)
    ctx.set_images(to_dev(R), to_dev(T))
    tu = to_dev(u)
    prob = solver.Problem(Grid.from_spec(spec), R.astype(np.float64), T.astype(np.float64))
    Js = []
    for k in range(4):
        info = ctx.gn_step(tu, pcg_max=30, pcg_rtol=1e-3, precond=1)
        assert info["accepted"] == 1
        assert info["J_after"] < info["J_before"]
        assert info["slope"] < 0
        Jo = prob.objective(tu.cpu().numpy().astype(np.float64))[0]
        assert abs(info["J_after"] - Jo) <= 1e-5 * abs(Jo), (k, info["J_after"], Jo)
        Js.append(info["J_after"])
    assert all(Js[i + 1] < Js[i] for i in range(len(Js) - 1))
    # gradient parity at the last iterate
    g, _ = ctx.gradient(tu)
    go = prob.gradient(tu.cpu().numpy().astype(np.float64))[1]
    assert rel_l2(g.cpu().numpy(), go) <= 1e-4


def test_multilevel_config2_monotone_and_final_objective_parity():
    print("[gpu-case] multilevel config 2 (128x128x96, 3 levels)", flush=True)
    c = config_c2(0)
    spec = c["spec"]
    R = c["R"].contiguous()
    T = c["T"].contiguous()
    u, rep = mfr.register_multilevel(spec, R.to(DEV), T.to(DEV), levels=3, gn_iters=10, pcg_max=50,
                                     pcg_rtol=1e-3, precond=1)
    torch.cuda.synchronize()
    assert all(n >= 1 for n in rep["gn_done"]), rep
    prob = solver.Problem(Grid.from_spec(spec), R.numpy().astype(np.float64), T.numpy().astype(np.float64))
    u64 = u.cpu().numpy().astype(np.float64)
    Jo = prob.objective(u64)[0]
    assert abs(rep["J_final"] - Jo) <= 1e-5 * abs(Jo)
    J0 = prob.objective(np.zeros_like(u64))[0]
    assert Jo < J0
    # the registration recovers the displacement that aligns the pair where the images
    # determine it: along the edge normals.  Elsewhere no bound holds: in the air around
    # the body both images are constant, and in homogeneous tissue only the noise
    # differs, so NGF carries no information there (the body-voxel error is reported)
    from synth import alignment_errors

    g = Grid.from_spec(spec)
    uf = u64.reshape(3, -1)
    err = alignment_errors(0, spec.m, R.numpy(), lambda idx: (g.P_rows(idx) @ uf.T))
    (n0, n1, ne), (b0, b1, nb) = err["edges"], err["body"]
    print(f"[gpu-case] J {J0:.4e} -> {Jo:.4e}; edge-normal error {n0:.3f} -> {n1:.3f} voxels ({ne} edge voxels), "
          f"body error {b0:.3f} -> {b1:.3f} ({nb} body voxels)", flush=True)
    assert n1 <= 0.6 * n0   # measured ratios 0.50-0.51 (trajectories vary with the tile configuration)
