"""Sampled parity at the full bench workload: the 512x512x900 CT-like pair with
129x129x225 deformation nodes, in the launch configuration the bench times
(32x16 work-groups, split target 4096).  The gradient, a Hessian-vector
product and the Jacobi diagonal computed on the GPU over the whole grid are
compared at sampled nodes (corners, faces, tile and z-chunk borders, random
interior nodes) with the oracle's exact single-node evaluation, which builds
only the Jacobian rows and regulariser rows that touch each node.  Cases: NGF with
curvature (the bench's), the sum of squared differences with curvature, and NGF with
the diffusive and the linear-elastic regularisers."""
import numpy as np
import pytest
import torch

from gpu_cases import rel_l2
from oracle import Grid, curvature, diffusive, elastic, ngf, ssd
from paper_1804_10541_amd import mfr
from synth import GridSpec, ct_pair, smooth_field

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


def sample_nodes(grid, rng, n_random=12):
    nx, ny, nz = grid.my
    picks = [(0, 0, 0), (nx - 1, ny - 1, nz - 1), (nx - 1, 0, nz // 2), (0, ny - 1, 1), (nx // 2, ny // 2, 0),
             (7, 3, 37), (14, 7, 38), (21, 21, 112), (64, 0, 75), (128, 64, 150)]
    picks += [tuple(int(v) for v in (rng.integers(0, nx), rng.integers(0, ny), rng.integers(0, nz)))
              for _ in range(n_random)]
    return [int(grid.node_id(a, b, c)) for a, b, c in picks]


@pytest.mark.parametrize("distance,regulariser", [("ngf", "curvature"), ("ssd", "curvature"), ("ngf", "diffusive"),
                                                   ("ngf", "elastic")])
def test_bench_workload_sampled_nodes(distance, regulariser):
    print(f"[gpu-case] {distance} {regulariser} 512x512x900 / 129x129x225, tile 32x16 target 4096, seed 0", flush=True)
    m, my = (512, 512, 900), (129, 129, 225)
    spec = GridSpec(m=m, h=(1.0, 1.0, 1.0), my=my, tau=50.0, rho=50.0, alpha=0.1, distance=distance,
                    regulariser=regulariser, lame_mu=1.0, lame_lambda=1.0)
    dist = ssd if distance == "ssd" else ngf
    reg = {"diffusive": diffusive, "elastic": elastic}.get(regulariser, curvature)
    R, T, _, rng = ct_pair(0, m, device=DEV)
    u = torch.from_numpy(smooth_field(rng, my, 0.5).astype("float32")).to(DEV)
    gen = torch.Generator(device=DEV).manual_seed(11)
    p = torch.randn(u.shape, generator=gen, device=DEV, dtype=torch.float32)
    prev = mfr.get_tile_config()
    mfr.set_tile_config(32, 16, 0, 4096)
    try:
        ctx = mfr.Context(spec, DEV)
        ctx.set_images(R, T)
        g, _ = ctx.gradient(u)
        hv = ctx.hess_vec(u, p)
        dg = ctx.jacobi_diag(u)
        torch.cuda.synchronize()
        g, hv, dg = (x.cpu().numpy().reshape(3, -1) for x in (g, hv, dg))
        ctx.close()
    finally:
        mfr.set_tile_config(**prev)
    R64 = R.cpu().numpy().astype(np.float64)
    T64 = T.cpu().numpy().astype(np.float64)
    u64 = u.cpu().numpy().astype(np.float64)
    p64 = p.cpu().numpy().astype(np.float64)
    del R, T, u, p
    torch.cuda.empty_cache()
    grid = Grid.from_spec(spec)
    nodes = sample_nodes(grid, np.random.default_rng(3))
    og, oh, od = [], [], []
    for node in nodes:
        gD, hD, dD = dist.node_outputs(grid, R64, T64, u64, p64, node)
        gS, hS, dS = reg.node_outputs(grid, u64, p64, node)
        og.append(gD + grid.alpha * gS)
        oh.append(hD + grid.alpha * hS)
        od.append(dD + grid.alpha * dS)
    og, oh, od = (np.array(x).T for x in (og, oh, od))   # (3, samples)
    e_g, e_h, e_d = rel_l2(g[:, nodes], og), rel_l2(hv[:, nodes], oh), rel_l2(dg[:, nodes], od)
    print(f"[gpu-case] sampled rel-L2: gradient {e_g:.2e}, Hv {e_h:.2e}, diagonal {e_d:.2e}", flush=True)
    assert e_g <= 1e-4 and e_h <= 1e-4 and e_d <= 1e-4
    assert np.all(dg > 0)
