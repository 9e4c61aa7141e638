"""GPU path (through the C ABI) against the float64 oracle on the same inputs.

Tolerances: objective values 1e-5 relative, gradients / Hessian-vector
products / Jacobi diagonals 1e-4 relative L2 (float32 arithmetic with
float64 sums against float64 throughout).
"""
import os

import numpy as np
import pytest
import torch

from gpu_cases import DEV, assert_parity, blob_case, ct_case, gpu_eval, oracle_eval, rel_l2, to_dev
from oracle import solver
from paper_1804_10541_amd import mfr
from synth import config_c1

pytestmark = pytest.mark.gpu


def _announce(name):
    print(f"[gpu-case] {name}", flush=True)


def test_config1_objective_gradient_ten_hv():
    _announce("config1 32^3 / 17^3, 10 probes")
    c = config_c1(0)
    f32 = lambda a: np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    R, T, u, probes = f32(c["R"]), f32(c["T"]), f32(c["u0"]), f32(c["probes"])
    gpu = gpu_eval(c["spec"], R, T, u, probes)
    ora = oracle_eval(c["spec"], R, T, u, probes)
    assert_parity(gpu, ora)


CASES = [
    # name, m, my, h, tau, rho, alpha, amp
    ("ragged-noninteger", (61, 37, 29), (16, 13, 11), (1.0, 1.3, 0.8), 0.2, 0.35, 0.5, 0.7),
    ("ratio-one", (20, 14, 10), (21, 15, 11), (1.0, 1.0, 1.0), 0.1, 0.1, 1.0, 0.4),
    ("ratio-four", (64, 40, 24), (17, 11, 7), (1.0, 1.0, 1.0), 0.1, 0.1, 0.3, 0.6),
    ("tiny-2x2x2", (2, 2, 2), (2, 2, 2), (1.0, 1.0, 1.0), 0.1, 0.1, 1.0, 0.3),
    ("tiny-3x5x2", (3, 5, 2), (2, 3, 3), (0.7, 1.0, 1.4), 0.3, 0.2, 1.0, 0.3),
    ("large-displacement", (20, 20, 20), (6, 6, 6), (1.0, 1.0, 1.0), 0.1, 0.1, 0.1, 8.0),
    # u = 0: every voxel centre on a template sample, where the derivative takes the floor cell
    ("zero-displacement", (24, 20, 16), (9, 8, 7), (1.0, 1.0, 1.0), 0.1, 0.1, 1.0, 0.0),
    # node supports wider than the diagonal kernel's 32-column blocks: the one-thread-per-node diagonal
    ("coarse-nodes", (70, 40, 20), (3, 2, 3), (1.0, 1.0, 1.0), 0.1, 0.1, 0.5, 0.8),
]


@pytest.mark.parametrize("name,m,my,h,tau,rho,alpha,amp", CASES, ids=[c[0] for c in CASES])
def test_parity_grid_cases(name, m, my, h, tau, rho, alpha, amp):
    _announce(name)
    spec, R, T, u, probes = blob_case(3, m, my, h, tau, rho, alpha, amp)
    assert_parity(gpu_eval(spec, R, T, u, probes), oracle_eval(spec, R, T, u, probes))


def test_parity_separate_template_grid():
    _announce("separate template grid")
    spec, R, T, u, probes = blob_case(5, (24, 18, 14), (9, 7, 6), (1.0, 1.0, 1.0), 0.1, 0.1, 1.0, 0.5,
                                      mT=(27, 22, 12), hT=(0.9, 0.8, 1.1))
    assert_parity(gpu_eval(spec, R, T, u, probes), oracle_eval(spec, R, T, u, probes))


def test_parity_ct_like():
    _announce("ct-like 64x64x48 / 33x33x25")
    spec, R, T, u, probes = ct_case(1, (64, 64, 48), (33, 33, 25), amp=1.5)
    assert_parity(gpu_eval(spec, R, T, u, probes), oracle_eval(spec, R, T, u, probes))


@pytest.mark.parametrize("tile", ["64x8", "32x32", "64x16"])
def test_parity_other_tile_shapes_and_chunks(tile):
    _announce(f"tile {tile}")
    bx, by = (int(k) for k in tile.split("x"))
    prev = mfr.get_tile_config()
    mfr.set_tile_config(bx, by, chunk_len=7)
    try:
        spec, R, T, u, probes = blob_case(4, (70, 45, 33), (24, 16, 12), (1.0, 1.0, 1.0), 0.15, 0.15, 0.8, 0.6)
        assert_parity(gpu_eval(spec, R, T, u, probes), oracle_eval(spec, R, T, u, probes))
    finally:
        mfr.set_tile_config(**prev)


@pytest.mark.parametrize("distance", ["ngf", "ssd"])
def test_parity_chunk_longer_than_the_lds_tables(distance):
    # a requested z chunk of 400 planes is capped at the 252 planes whose tables a group
    # keeps in LDS: 300 planes become chunks of 252 and 48
    _announce(f"{distance} chunk cap, 300 planes")
    prev = mfr.get_tile_config()
    mfr.set_tile_config(32, 16, chunk_len=400)
    try:
        spec, R, T, u, probes = blob_case(7, (20, 18, 300), (6, 5, 76), (1.0, 1.0, 1.0), 0.1, 0.1, 0.5, 0.6,
                                          n_probes=2, distance=distance)
        assert_parity(gpu_eval(spec, R, T, u, probes), oracle_eval(spec, R, T, u, probes))
    finally:
        mfr.set_tile_config(**prev)


def test_hessian_symmetric_psd_and_deterministic():
    _announce("symmetry / determinism")
    spec, R, T, u, probes = blob_case(6, (40, 36, 30), (14, 13, 11), (1.0, 1.0, 1.0), 0.1, 0.1, 0.5, 0.5)
    ctx = mfr.Context(spec, DEV)
    ctx.set_images(to_dev(R), to_dev(T))
    tu, a, b = to_dev(u), to_dev(probes[0]), to_dev(probes[1])
    Ha, Hb = ctx.hess_vec(tu, a), ctx.hess_vec(tu, b)
    Ha2 = ctx.hess_vec(tu, a)
    torch.cuda.synchronize()
    assert torch.equal(Ha, Ha2), "Hessian-vector product is not bitwise reproducible"
    x = float(torch.sum(a.double() * Hb.double()))
    y = float(torch.sum(b.double() * Ha.double()))
    assert abs(x - y) <= 1e-5 * max(abs(x), abs(y))
    assert float(torch.sum(a.double() * Ha.double())) > 0
    g1, _ = ctx.gradient(tu)
    g2, _ = ctx.gradient(tu)
    torch.cuda.synchronize()
    assert torch.equal(g1, g2)


def test_pcg_first_iterates_match_oracle():
    _announce("pcg iterates")
    spec, R, T, u, probes = blob_case(8, (36, 30, 26), (13, 11, 10), (1.0, 1.0, 1.0), 0.1, 0.1, 1.0, 0.5)
    ora = oracle_eval(spec, R, T, u, probes[:0])
    prob, Jac = ora["prob"], ora["Jac"]
    u64 = u.astype(np.float64)
    b = -ora["grad"]
    diag = prob.jacobi_diag(u64, Jac)
    ctx = mfr.Context(spec, DEV)
    ctx.set_images(to_dev(R), to_dev(T))
    tu, tb = to_dev(u), to_dev(b.astype(np.float32))
    b32 = b.astype(np.float32).astype(np.float64)
    for k in (1, 2, 3):
        s_gpu, info = ctx.pcg_solve(tu, tb, max_iter=k, rtol=0.0, precond=1)
        s_ora, info_o = solver.pcg(lambda p: prob.hess_vec(u64, p, Jac), b32, diag, k, 0.0)
        assert info["iters"] == k == info_o["iters"]
        e = rel_l2(s_gpu.cpu().numpy(), s_ora)
        assert e <= 1e-4, f"iterate {k}: rel-L2 {e:.3e}"
        assert abs(info["relres"] - info_o["relres"]) <= 1e-3 * info_o["relres"]
    # a converged solve reaches the requested tolerance
    s, info = ctx.pcg_solve(tu, tb, max_iter=200, rtol=1e-3, precond=1)
    assert info["flag"] == 0 and info["relres"] <= 1e-3
    r = tb - ctx.hess_vec(tu, s)
    assert float(torch.linalg.norm(r.double()) / torch.linalg.norm(tb.double())) <= 2e-3


def test_pcg_without_regulariser_zero_diagonal_entries():
    # alpha = 0 and a template that is zero (flat) in most of the domain: nodes that
    # no row of dr reaches with a non-zero template derivative get a zero diagonal
    _announce("pcg, alpha 0, zero Jacobi entries")
    m = (24, 20, 16)
    spec, R, T, u, probes = blob_case(9, m, (9, 8, 7), (1.0, 1.0, 1.0), 0.1, 0.1, 0.0, 0.0)
    T = np.zeros_like(T)
    T[4:10, 5:11, 6:12] = 1.0
    ora = oracle_eval(spec, R, T, u, probes[:0])
    prob, Jac = ora["prob"], ora["Jac"]
    u64 = u.astype(np.float64)
    diag = prob.jacobi_diag(u64, Jac)
    assert np.any(diag == 0.0) and np.any(diag > 0.0)
    b32 = (-ora["grad"]).astype(np.float32)
    ctx = mfr.Context(spec, DEV)
    ctx.set_images(to_dev(R), to_dev(T))
    tu, tb = to_dev(u), to_dev(b32)
    dg = ctx.jacobi_diag(tu).cpu().numpy()
    z_o, z_g = diag == 0.0, dg == 0.0
    print(f"[gpu-case] zero diagonal entries: oracle {int(z_o.sum())}, GPU {int(z_g.sum())}, GPU max where "
          f"oracle is 0: {float(np.abs(dg[z_o]).max()):.3e}, oracle max where GPU is 0: "
          f"{float(np.abs(diag[z_g]).max()) if z_g.any() else 0.0:.3e}", flush=True)
    assert z_g.any() and np.all(np.abs(dg[z_o]) <= 1e-6 * float(diag.max()))
    assert rel_l2(dg, diag) <= 1e-4
    for k in (1, 2, 4):
        s_gpu, info = ctx.pcg_solve(tu, tb, max_iter=k, rtol=0.0, precond=1)
        s_ora, info_o = solver.pcg(lambda p: prob.hess_vec(u64, p, Jac), b32.astype(np.float64), diag, k, 0.0)
        assert info["iters"] == k == info_o["iters"]
        s_gpu = s_gpu.cpu().numpy()
        assert np.all(np.isfinite(s_gpu))
        e = rel_l2(s_gpu, s_ora)
        assert e <= 1e-4, f"iterate {k}: rel-L2 {e:.3e}"
    ctx.close()
