"""The batched path at the full ten-pair workload: CT-like pairs of 256x256 and
512x512 voxels by 94..136 planes with quarter-resolution deformation grids, one
batch.  The batched Hessian-vector products must equal the single-pair path
bit for bit for every pair (the single-pair path is held to the oracle), and
two pairs are also compared with the oracle's exact single-node evaluation at
sampled nodes."""
import numpy as np
import pytest
import torch

from gpu_cases import rel_l2
from oracle import Grid, curvature, ngf
from paper_1804_10541_amd import mfr
from synth import GridSpec, config_c4_sizes, ct_pair, quarter_nodes, smooth_field

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


def test_ten_pair_workload_batched_hv():
    print("[gpu-case] ten-pair batched Hv, sizes 256^2/512^2 x 94..136, seeds 0-9", flush=True)
    specs, Rs, Ts, us, ps = [], [], [], [], []
    gen = torch.Generator(device=DEV).manual_seed(21)
    for k, m in enumerate(config_c4_sizes()):
        spec = GridSpec(m=m, h=(1.0, 1.0, 1.0), my=quarter_nodes(m), tau=50.0, rho=50.0, alpha=0.1)
        R, T, _, rng = ct_pair(k, m, device=DEV)
        specs.append(spec)
        Rs.append(R)
        Ts.append(T)
        us.append(torch.from_numpy(smooth_field(rng, spec.my, 1.0).astype("float32")).to(DEV))
        ps.append(torch.randn(us[-1].shape, generator=gen, device=DEV, dtype=torch.float32))
    b = mfr.Batch(specs, levels=1, device=DEV)
    b.set_images(Rs, Ts)
    qb = [q.cpu().numpy() for q in b.hess_vec(us, ps)]
    b.close()
    for k, spec in enumerate(specs):
        ctx = mfr.Context(spec, DEV)
        ctx.set_images(Rs[k], Ts[k])
        q1 = ctx.hess_vec(us[k], ps[k]).cpu().numpy()
        ctx.close()
        assert np.array_equal(q1, qb[k]), f"pair {k} {spec.m}: batched and single-pair Hv differ"
    rng = np.random.default_rng(4)
    for k in (0, 9):
        grid = Grid.from_spec(specs[k])
        R64, T64 = Rs[k].cpu().numpy().astype(np.float64), Ts[k].cpu().numpy().astype(np.float64)
        u64, p64 = us[k].cpu().numpy().astype(np.float64), ps[k].cpu().numpy().astype(np.float64)
        nx, ny, nz = grid.my
        nodes = [0, grid.nbar - 1] + [int(grid.node_id(rng.integers(0, nx), rng.integers(0, ny), rng.integers(0, nz)))
                                      for _ in range(8)]
        ref = []
        for node in nodes:
            _, hD, _ = ngf.node_outputs(grid, R64, T64, u64, p64, node)
            _, hS, _ = curvature.node_outputs(grid, u64, p64, node)
            ref.append(hD + grid.alpha * hS)
        e = rel_l2(qb[k].reshape(3, -1)[:, nodes], np.array(ref).T)
        print(f"[gpu-case] pair {k} {specs[k].m}: sampled Hv rel-L2 {e:.2e}", flush=True)
        assert e <= 1e-4
