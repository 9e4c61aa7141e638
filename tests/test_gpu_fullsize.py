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


def sample_nodes(grid, rng, n_random=12, structured=0):
    """Corners, faces, tile and z-chunk borders of the 32x16 / split-4096 launch
    (own tile widths 30 x 14 voxels, z chunks of 129 planes: node indices near
    7.5 k, 3.5 k and 32.1 k) and random interior nodes."""
    nx, ny, nz = grid.my
    picks = [(0, 0, 0), (nx - 1, ny - 1, nz - 1), (nx - 1, 0, nz // 2), (0, ny - 1, 1), (nx // 2, ny // 2, 0),
             (7, 3, 37), (14, 7, 38), (21, 21, 112), (64, 0, 75), (128, 64, 150)]
    if structured:
        xs = [0, 1, 7, 8, 15, 22, 23, 60, 67, 68, 127, 128]
        ys = [0, 1, 3, 4, 7, 10, 11, 63, 66, 127, 128]
        zs = [0, 1, 32, 33, 64, 65, 96, 97, 129, 161, 193, 223, 224]
        for a in (0, nx - 1):   # the eight corners and the centres of the six faces
            for b in (0, ny - 1):
                for c in (0, nz - 1):
                    picks.append((a, b, c))
        picks += [(0, ny // 2, nz // 3), (nx - 1, ny // 3, nz // 2), (nx // 2, 0, nz // 4), (nx // 3, ny - 1, nz // 5),
                  (nx // 4, ny // 5, 0), (nx // 5, ny // 4, nz - 1)]
        picks += [(int(rng.choice(xs)), int(rng.choice(ys)), int(rng.choice(zs))) for _ in range(structured)]
    picks += [tuple(int(v) for v in (rng.integers(0, nx), rng.integers(0, ny), rng.integers(0, nz)))
              for _ in range(n_random)]
    return sorted({int(grid.node_id(a, b, c)) for a, b, c in picks})


@pytest.mark.parametrize("distance,regulariser", [("ngf", "curvature"), ("ssd", "curvature"), ("ngf", "diffusive"),
                                                   ("ngf", "elastic")])
def test_bench_workload_sampled_nodes(distance, regulariser):
    print(f"[gpu-case] {distance} {regulariser} 512x512x900 / 129x129x225, tile 32x16 target 4096, seed 0", flush=True)
    m, my = (512, 512, 900), (129, 129, 225)
    spec = GridSpec(m=m, h=(1.0, 1.0, 1.0), my=my, tau=50.0, rho=50.0, alpha=0.1, distance=distance,
                    regulariser=regulariser, lame_mu=1.0, lame_lambda=1.0)
    dist = ssd if distance == "ssd" else ngf
    reg = {"diffusive": diffusive, "elastic": elastic}.get(regulariser, curvature)
    # the bench's own case: two Hessian-vector probes and about 100 nodes of every class
    full = distance == "ngf" and regulariser == "curvature"
    n_probes = 2 if full else 1
    R, T, _, rng = ct_pair(0, m, device=DEV)
    u = torch.from_numpy(smooth_field(rng, my, 0.5).astype("float32")).to(DEV)
    gen = torch.Generator(device=DEV).manual_seed(11)
    ps = [torch.randn(u.shape, generator=gen, device=DEV, dtype=torch.float32) for _ in range(n_probes)]
    prev = mfr.get_tile_config()
    mfr.set_tile_config(32, 16, 0, 4096)
    try:
        ctx = mfr.Context(spec, DEV)
        ctx.set_images(R, T)
        g, _ = ctx.gradient(u)
        hvs = [ctx.hess_vec(u, p).cpu().numpy().reshape(3, -1) for p in ps]
        dg = ctx.jacobi_diag(u)
        torch.cuda.synchronize()
        g, dg = (x.cpu().numpy().reshape(3, -1) for x in (g, dg))
        ctx.close()
    finally:
        mfr.set_tile_config(**prev)
    R64 = R.cpu().numpy().astype(np.float64)
    T64 = T.cpu().numpy().astype(np.float64)
    u64 = u.cpu().numpy().astype(np.float64)
    p64s = [p.cpu().numpy().astype(np.float64) for p in ps]
    del R, T, u, ps
    torch.cuda.empty_cache()
    grid = Grid.from_spec(spec)
    nodes = sample_nodes(grid, np.random.default_rng(3), n_random=44 if full else 12, structured=30 if full else 0)
    og, od = [], []
    ohs = [[] for _ in p64s]
    for node in nodes:
        for k, p64 in enumerate(p64s):
            gD, hD, dD = dist.node_outputs(grid, R64, T64, u64, p64, node)
            gS, hS, dS = reg.node_outputs(grid, u64, p64, node)
            ohs[k].append(hD + grid.alpha * hS)
        og.append(gD + grid.alpha * gS)
        od.append(dD + grid.alpha * dS)
    og, od = (np.array(x).T for x in (og, od))   # (3, samples)
    e_g, e_d = rel_l2(g[:, nodes], og), rel_l2(dg[:, nodes], od)
    e_h = [rel_l2(hv[:, nodes], np.array(oh).T) for hv, oh in zip(hvs, ohs)]
    print(f"[gpu-case] {len(nodes)} sampled nodes, rel-L2: gradient {e_g:.2e}, Hv {e_h}, diagonal {e_d:.2e}",
          flush=True)
    assert e_g <= 1e-4 and max(e_h) <= 1e-4 and e_d <= 1e-4
    assert np.all(dg > 0)


_SLAB = {}


def _slab_sum(z0z1):
    """Oracle sum of 1 - r_i^2 over the voxels of planes [z0, z1) (runs in a
    forked worker; reads the problem from the module-level table)."""
    z0, z1 = z0z1
    grid, R64, T64, u64 = _SLAB["args"]
    plane = grid.m[0] * grid.m[1]
    vox = np.arange(z0 * plane, z1 * plane, dtype=np.int64)
    r = ngf.residual_parts(grid, R64, T64, u64, vox)["r"]
    return float(np.sum(1.0 - r * r))


def test_bench_workload_objective_matches_slab_streamed_oracle():
    """Objective of the 512x512x900 / 129x129x225 workload (NGF + curvature), in
    the launch configuration the bench times, against the float64 oracle
    evaluated slab by slab (planes of voxels with their clamped neighbours, the
    per-slab sums of 1 - r_i^2 added in plane order) on the host's cores."""
    import multiprocessing as mp
    import os

    print("[gpu-case] objective 512x512x900 / 129x129x225, tile 32x16 target 4096, seed 0", flush=True)
    m, my = (512, 512, 900), (129, 129, 225)
    spec = GridSpec(m=m, h=(1.0, 1.0, 1.0), my=my, tau=50.0, rho=50.0, alpha=0.1)
    R, T, _, rng = ct_pair(0, m, device=DEV)
    u = torch.from_numpy(smooth_field(rng, my, 0.5).astype("float32")).to(DEV)
    prev = mfr.get_tile_config()
    mfr.set_tile_config(32, 16, 0, 4096)
    try:
        ctx = mfr.Context(spec, DEV)
        ctx.set_images(R, T)
        J, D, S = ctx.objective(u)
        ctx.close()
    finally:
        mfr.set_tile_config(**prev)
    grid = Grid.from_spec(spec)
    R64 = R.cpu().numpy().astype(np.float64)
    T64 = T.cpu().numpy().astype(np.float64)
    u64 = u.cpu().numpy().astype(np.float64)
    del R, T, u
    torch.cuda.empty_cache()
    So = curvature.energy(grid, u64)
    _SLAB["args"] = (grid, R64, T64, u64)
    slabs = [(z, min(z + 6, m[2])) for z in range(0, m[2], 6)]
    workers = max(1, min(16, os.cpu_count() or 1))
    print(f"[gpu-case] oracle: {len(slabs)} slabs on {workers} worker processes", flush=True)
    with mp.get_context("fork").Pool(workers) as pool:
        parts = pool.map(_slab_sum, slabs, chunksize=1)
    _SLAB.clear()
    Do = grid.hbar * float(np.sum(parts))
    Jo = Do + grid.alpha * So
    print(f"[gpu-case] J {J:.10e} / {Jo:.10e}, D {D:.10e} / {Do:.10e}, S {S:.6e} / {So:.6e}", flush=True)
    assert abs(D - Do) <= 1e-5 * abs(Do)
    assert abs(S - So) <= 1e-5 * abs(So)
    assert abs(J - Jo) <= 1e-5 * abs(Jo)
