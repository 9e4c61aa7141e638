"""The two-dimensional case (d = 2) of the path on the GPU against the 2D
oracle (oracle.plane): objective, gradient, Gauss-Newton products and the
Jacobi diagonal on grids that span several work-group columns, several row
chunks and ragged tails, with integer and non-integer grid ratios, a separate
template grid and zero displacement; PCG iterates, Gauss-Newton steps and the
coarse-to-fine path; sampled nodes at the 4096 x 4096 / 2049 x 2049 workload.
(The paper's GPU experiments of Sec. 6.3 are two-dimensional.)"""
import numpy as np
import pytest
import torch

from gpu_cases import DEV, rel_l2
from oracle import plane, solver
from paper_1804_10541_amd import mfr
from synth import GridSpec, section_pair, smooth_field_2d

pytestmark = pytest.mark.gpu


def plane_case(seed, m, my, amp=0.5, n_probes=2, h=(1.0, 1.0), eps=0.05, alpha=1.0, mT=None, hT=None,
               zero_u=False):
    spec = GridSpec(m=(m[0], m[1], 1), h=(h[0], h[1], 1.0), my=(my[0], my[1], 1), tau=eps, rho=eps, alpha=alpha,
                    mT=None if mT is None else (mT[0], mT[1], 1), hT=None if hT is None else (hT[0], hT[1], 1.0))
    R, T, _, rng = section_pair(seed, m)
    if mT is not None:
        _, T, _, _ = section_pair(seed + 1000, mT)
    u = smooth_field_2d(rng, my, amp).astype(np.float32)
    if zero_u:
        u[:] = 0.0
    probes = rng.standard_normal((n_probes, 2, my[1], my[0])).astype(np.float32)
    return spec, R, T, u, probes


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def gpu_eval(spec, R, T, u, probes):
    ctx = mfr.Context(spec, DEV)
    ctx.set_images(to_dev(R), to_dev(T))
    tu = to_dev(u)
    J, D, S = ctx.objective(tu)
    g, Jg = ctx.gradient(tu)
    hv = [ctx.hess_vec(tu, to_dev(p)).cpu().numpy() for p in probes]
    dg = ctx.jacobi_diag(tu).cpu().numpy()
    torch.cuda.synchronize()
    out = dict(J=J, D=D, S=S, Jg=Jg, grad=g.cpu().numpy(), hv=hv, diag=dg, shape=tuple(g.shape))
    ctx.close()
    return out


def oracle_eval(spec, R, T, u, probes):
    g = plane.Grid2.from_spec(spec)
    prob = plane.Problem2(g, R.astype(np.float64), T.astype(np.float64))
    u64 = u.astype(np.float64)
    J, D, S = prob.objective(u64)
    _, grad = prob.gradient(u64)
    Jac = prob.jacobian(u64)
    hv = [prob.hess_vec(u64, p.astype(np.float64), Jac) for p in probes]
    return dict(J=J, D=D, S=S, grad=grad, hv=hv, diag=prob.jacobi_diag(u64, Jac), prob=prob, Jac=Jac)


def assert_parity(gp, og):
    assert gp["shape"] == og["grad"].shape
    for k in ("J", "D", "S"):
        assert abs(gp[k] - og[k]) <= 1e-5 * max(abs(og[k]), 1e-12 * abs(og["J"])), (k, gp[k], og[k])
    assert abs(gp["Jg"] - og["J"]) <= 1e-5 * abs(og["J"])
    assert rel_l2(gp["grad"], og["grad"]) <= 1e-4, rel_l2(gp["grad"], og["grad"])
    for a, b in zip(gp["hv"], og["hv"]):
        assert rel_l2(a, b) <= 1e-4, rel_l2(a, b)
    assert rel_l2(gp["diag"], og["diag"]) <= 1e-4, rel_l2(gp["diag"], og["diag"])


CASES = {
    # one work-group column, grid ratio 2
    "single-column-ratio2": dict(seed=1, m=(40, 33), my=(21, 17)),
    # three work-group columns (254 own pixel columns each), non-integer ratios, ragged row chunks
    "three-columns-ragged": dict(seed=2, m=(600, 97), my=(151, 40)),
    # as many nodes as the image allows (ratio 1)
    "ratio-one": dict(seed=3, m=(64, 48), my=(65, 49)),
    # coarse deformation grid: long node support
    "coarse-nodes": dict(seed=4, m=(300, 70), my=(9, 5)),
    # anisotropic spacing
    "anisotropic": dict(seed=5, m=(130, 90), my=(33, 31), h=(0.8, 1.3)),
    # zero displacement: pixel centres exactly on template samples (floor cell derivative)
    "zero-displacement": dict(seed=6, m=(270, 40), my=(136, 21), zero_u=True),
    # large displacement: samples in the template's zero border
    "large-displacement": dict(seed=7, m=(80, 60), my=(21, 16), amp=9.0),
}


@pytest.mark.parametrize("name", list(CASES))
def test_plane_parity(name):
    print(f"[gpu-case] plane {name}", flush=True)
    spec, R, T, u, probes = plane_case(**CASES[name])
    assert_parity(gpu_eval(spec, R, T, u, probes), oracle_eval(spec, R, T, u, probes))


def test_plane_parity_separate_template_grid():
    print("[gpu-case] plane separate template grid", flush=True)
    spec, R, T, u, probes = plane_case(8, (90, 70), (31, 24), mT=(61, 83), hT=(1.45, 0.8))
    assert_parity(gpu_eval(spec, R, T, u, probes), oracle_eval(spec, R, T, u, probes))


@pytest.mark.parametrize("chunk_len", [1, 5, 13])
def test_plane_parity_short_row_chunks(chunk_len):
    """Row chunks shorter than a node spacing and of odd length: node rows
    gathered from several chunks."""
    print(f"[gpu-case] plane chunk_len {chunk_len}", flush=True)
    saved = mfr.get_tile_config()
    mfr.set_tile_config(saved["bx"], saved["by"], chunk_len, saved["target_groups"])
    try:
        spec, R, T, u, probes = plane_case(9, (300, 61), (101, 31))
        gp = gpu_eval(spec, R, T, u, probes)
    finally:
        mfr.set_tile_config(**saved)
    assert_parity(gp, oracle_eval(spec, R, T, u, probes))


def test_plane_hessian_symmetric_psd_deterministic():
    spec, R, T, u, probes = plane_case(10, (257, 130), (65, 33), n_probes=3)
    ctx = mfr.Context(spec, DEV)
    ctx.set_images(to_dev(R), to_dev(T))
    tu = to_dev(u)
    P = [to_dev(p) for p in probes]
    Q = [ctx.hess_vec(tu, p) for p in P]
    Q2 = ctx.hess_vec(tu, P[0])
    torch.cuda.synchronize()
    assert torch.equal(Q[0], Q2)
    a = float(torch.dot(P[0].flatten().double(), Q[1].flatten().double()))
    b = float(torch.dot(P[1].flatten().double(), Q[0].flatten().double()))
    assert abs(a - b) <= 1e-5 * (abs(a) + abs(b))
    for p, q in zip(P, Q):
        assert float(torch.dot(p.flatten().double(), q.flatten().double())) > 0
    ctx.close()


def test_plane_pcg_iterates_and_gauss_newton_steps():
    spec, R, T, u, _ = plane_case(11, (200, 150), (51, 38))
    g = plane.Grid2.from_spec(spec)
    prob = plane.Problem2(g, R.astype(np.float64), T.astype(np.float64))
    ctx = mfr.Context(spec, DEV)
    ctx.set_images(to_dev(R), to_dev(T))
    tu = to_dev(u)
    grad, _ = ctx.gradient(tu)
    b = (-grad).contiguous()
    b64 = b.cpu().numpy().astype(np.float64)
    u64 = u.astype(np.float64)
    Jac = prob.jacobian(u64)
    diag = prob.jacobi_diag(u64, Jac)
    for k in (1, 2, 3):
        s, info = ctx.pcg_solve(tu, b, max_iter=k, rtol=0.0, precond=1)
        so, oi = solver.pcg(lambda p: prob.hess_vec(u64, p, Jac), b64, diag, max_iter=k, rtol=0.0)
        assert info["iters"] == k == oi["iters"]
        assert rel_l2(s.cpu().numpy(), so) <= 1e-4
    uu = tu.clone()
    for k in range(3):
        info = ctx.gn_step(uu, pcg_max=30, pcg_rtol=1e-3, precond=1, armijo_c1=1e-4, armijo_max=10)
        Jo = prob.objective(uu.cpu().numpy().astype(np.float64))[0]
        print(f"[gpu-case] plane GN step {k}: J {info['J_after']:.8e} / {Jo:.8e}", flush=True)
        assert info["accepted"] == 1
        assert abs(info["J_after"] - Jo) <= 1e-5 * abs(Jo)
        assert info["J_after"] < info["J_before"]
    ctx.close()


def test_plane_pyramid_and_prolongation_match_oracle():
    spec = GridSpec(m=(301, 190, 1), h=(1.0, 1.25, 1.0), my=(76, 48, 1), tau=0.05, rho=0.05, alpha=1.0)
    levels = 3
    want = [plane.Grid2.from_spec(spec)]
    for _ in range(levels - 1):
        want.append(plane.coarse_grid(want[-1]))
    want = want[::-1]
    rng = np.random.default_rng(12)
    for lv in range(levels):
        cg = mfr.ml_level_grid(spec, levels, lv)
        w = want[lv]
        assert (cg.m[0], cg.m[1], cg.m[2]) == (w.m[0], w.m[1], 1)
        assert (cg.my[0], cg.my[1], cg.my[2]) == (w.my[0], w.my[1], 1)
        assert (cg.h[0], cg.h[1]) == w.h
        if lv + 1 < levels:
            fg = mfr.ml_level_grid(spec, levels, lv + 1)
            uc = rng.standard_normal((2, cg.my[1], cg.my[0])).astype(np.float32)
            got = mfr.prolong(to_dev(uc), cg, fg).cpu().numpy()
            ref = plane.prolong(uc.astype(np.float64), w, want[lv + 1])
            assert got.shape == ref.shape
            assert np.abs(got - ref).max() <= 1e-6 * np.abs(ref).max()
    img = (np.random.default_rng(13).standard_normal((1, 37, 51)) + 3.0).astype(np.float32)
    got = mfr.restrict_image(to_dev(img)).cpu().numpy()[0]
    ref = plane.restrict_image(img[0].astype(np.float64))
    assert got.shape == ref.shape
    assert np.abs(got - ref).max() <= 1e-6 * np.abs(ref).max()


def test_plane_multilevel_objective_per_level():
    """Three-level registration of a 512 x 384 section pair: the oracle's
    objective agrees with the GPU's at the start and end of every level (on the
    oracle's pyramid of the same float32 images), and each level improves."""
    m, my = (512, 384), (257, 193)
    spec = GridSpec(m=(m[0], m[1], 1), h=(1.0, 1.0, 1.0), my=(my[0], my[1], 1), tau=0.05, rho=0.05, alpha=1.0)
    R, T, _, _ = section_pair(14, m)
    u, rep = mfr.register_multilevel(spec, to_dev(R), to_dev(T), levels=3, gn_iters=4, pcg_max=30, pcg_rtol=1e-3,
                                     armijo_c1=1e-4, armijo_max=10, precond=1)
    assert tuple(u.shape) == (2, my[1], my[0])
    print(f"[gpu-case] plane multilevel J start {rep['J_start']} end {rep['J_level']} gn {rep['gn_done']}",
          flush=True)
    g = plane.Grid2.from_spec(spec)
    pyr = [(g, R.astype(np.float64), T.astype(np.float64))]
    for _ in range(2):
        gg, r, t = pyr[-1]
        pyr.append((plane.coarse_grid(gg), plane.restrict_image(r), plane.restrict_image(t)))
    gf, Rf, Tf = pyr[0]
    prob = plane.Problem2(gf, Rf, Tf)
    Jo = prob.objective(u.cpu().numpy().astype(np.float64))[0]
    assert abs(rep["J_final"] - Jo) <= 1e-5 * abs(Jo)
    for lv in range(3):
        gl, r, t = pyr[2 - lv]
        J0 = plane.Problem2(gl, r, t).objective(np.zeros(gl.node_shape()))[0]
        if lv == 0:
            assert abs(rep["J_start"][0] - J0) <= 1e-5 * abs(J0)
        assert rep["J_level"][lv] < rep["J_start"][lv]
        assert rep["gn_done"][lv] >= 1


def test_plane_full_size_sampled_nodes():
    """4096 x 4096 pixels, 2049 x 2049 nodes, in the launch configuration the
    bench times: gradient, one Hv and the diagonal at nodes of every border,
    corner, work-group-column and interior class, the NGF part from the
    oracle's exact single-node rows, the curvature part from the oracle's
    assembled regulariser over the whole field."""
    from synth import config_section

    print("[gpu-case] plane 4096x4096 / 2049x2049 sampled nodes, seed 0", flush=True)
    c = config_section(0, n_probes=1)
    spec, R, T, u, p = c["spec"], c["R"], c["T"], c["u0"], c["probes"][0]
    ctx = mfr.Context(spec, DEV)
    ctx.set_images(to_dev(R), to_dev(T))
    tu = to_dev(u)
    grad, _ = ctx.gradient(tu)
    hv = ctx.hess_vec(tu, to_dev(p))
    dg = ctx.jacobi_diag(tu)
    torch.cuda.synchronize()
    grad, hv, dg = (x.cpu().numpy().reshape(2, -1) for x in (grad, hv, dg))
    ctx.close()
    g = plane.Grid2.from_spec(spec)
    nx, ny = g.my
    rng = np.random.default_rng(15)
    picks = [(0, 0), (nx - 1, 0), (0, ny - 1), (nx - 1, ny - 1), (0, ny // 2), (nx - 1, 77), (1000, 0),
             (1234, ny - 1), (127, 1), (128, 2), (129, 1000), (254, 600), (255, 601)]
    picks += [tuple(int(v) for v in rng.integers(0, (nx, ny))) for _ in range(25)]
    nodes = [int(g.node_id(i, j)) for i, j in picks]
    R64, T64, u64, p64 = R.astype(np.float64), T.astype(np.float64), u.astype(np.float64), p.astype(np.float64)
    L = plane.laplacian(g)
    cg = g.alpha * plane.curvature_gradient(g, u64, L).reshape(2, -1)
    ch = g.alpha * plane.curvature_gradient(g, p64, L).reshape(2, -1)
    cd = g.alpha * plane.curvature_diag(g, L).reshape(2, -1)
    og, oh, od = [], [], []
    for n in nodes:
        gD, hD, dD = plane.node_outputs(g, R64, T64, u64, p64, n)
        og.append(gD + cg[:, n])
        oh.append(hD + ch[:, n])
        od.append(dD + cd[:, n])
    og, oh, od = (np.array(x).T for x in (og, oh, od))
    e_g, e_h, e_d = rel_l2(grad[:, nodes], og), rel_l2(hv[:, nodes], oh), rel_l2(dg[:, nodes], od)
    print(f"[gpu-case] sampled rel-L2: gradient {e_g:.2e}, Hv {e_h:.2e}, diagonal {e_d:.2e}", flush=True)
    assert e_g <= 1e-4 and e_h <= 1e-4 and e_d <= 1e-4
    assert np.all(dg > 0)


H0_PLANE_CASES = [
    # name, m, my, h, alpha, gamma
    ("ragged", (61, 37), (16, 13), (1.0, 1.3), 0.5, 0.2),
    ("ratio-one", (20, 14), (21, 15), (1.0, 1.0), 1.0, 1.0),
    ("two-nodes", (5, 4), (2, 2), (1.0, 1.0), 1.0, 0.5),
    ("long-axis", (300, 30), (301, 9), (1.0, 1.0), 0.1, 0.05),
    ("no-regulariser", (24, 20), (9, 8), (1.0, 1.0), 0.0, 2.0),
]


@pytest.mark.parametrize("name,m,my,h,alpha,gamma", H0_PLANE_CASES, ids=[c[0] for c in H0_PLANE_CASES])
def test_plane_h0_solve_matches_oracle(name, m, my, h, alpha, gamma):
    """L-BFGS initial-matrix solve (Sec. 2.3.2) with two cosine axes against the
    oracle's solve of (2 alpha hbar^y L^T L + gamma I) x = v (5-point L)."""
    from oracle import lbfgs

    print(f"[gpu-case] plane h0 {name} {m} / {my}", flush=True)
    spec, R, T, u, probes = plane_case(2, m, my, n_probes=2, h=h, alpha=alpha)
    ctx = mfr.Context(spec, DEV)
    g = plane.Grid2.from_spec(spec)
    h0 = lbfgs.H0Solver(g, gamma, plane.laplacian(g))
    for p in probes:
        want = h0.apply(p.astype(np.float64))
        x = ctx.h0_solve(to_dev(p), gamma).cpu().numpy()
        assert x.shape == p.shape
        assert rel_l2(x, want) <= 1e-4, rel_l2(x, want)
        t = to_dev(p)
        ctx.h0_solve(t, gamma, out=t)   # in place
        assert rel_l2(t.cpu().numpy(), want) <= 1e-4
    ctx.close()


def test_plane_lbfgs_first_iterate_and_objective_per_iterate():
    """The two-dimensional L-BFGS run (the optimiser of the paper's 2D GPU
    registrations): the first step from the same start against the oracle's
    (two-loop recursion with an empty memory, Armijo backtracking), then six
    iterations whose final J the oracle re-evaluates at the GPU's iterate;
    bitwise repeatable."""
    from oracle import lbfgs

    print("[gpu-case] plane lbfgs 192x160 / 49x41", flush=True)
    spec, R, T, u0, _ = plane_case(7, (192, 160), (49, 41), amp=0.0, n_probes=0)
    prob = plane.Problem2(plane.Grid2.from_spec(spec), R.astype(np.float64), T.astype(np.float64))
    gamma = 1e2
    ctx = mfr.Context(spec, DEV)
    ctx.set_images(to_dev(R), to_dev(T))
    tu = to_dev(u0)
    rep = ctx.lbfgs(tu, iters=1, mem=5, gamma=gamma)
    assert rep["iters"] == 1 and rep["status"] == 0, rep
    uo, hist = lbfgs.lbfgs(prob, u0.astype(np.float64), iters=1, mem=5, gamma=gamma)
    e = rel_l2(tu.cpu().numpy().astype(np.float64) - u0, uo - u0)
    print(f"[gpu-case] first step rel-L2 {e:.2e}, eta {hist[0]['eta']}", flush=True)
    assert e <= 1e-4
    assert abs(rep["J_initial"] - hist[0]["J"]) <= 1e-5 * abs(hist[0]["J"])
    tu = to_dev(u0)
    rep = ctx.lbfgs(tu, iters=6, mem=3, gamma=gamma)
    assert rep["status"] == 0 and rep["iters"] == 6, rep
    assert rep["J_final"] < rep["J_initial"]
    Jo = prob.objective(tu.cpu().numpy().astype(np.float64))[0]
    assert abs(rep["J_final"] - Jo) <= 1e-5 * abs(Jo), (rep["J_final"], Jo)
    tu2 = to_dev(u0)
    ctx.lbfgs(tu2, iters=6, mem=3, gamma=gamma)
    assert torch.equal(tu, tu2)
    ctx.close()


def test_plane_lbfgs_pure_regulariser_closed_form_first_step():
    """Zero images: D = 0 and J = alpha S, whose Hessian A = 2 alpha hbar^y L^T L
    (5-point L); the first step from u0 is -(A + gamma I)^{-1} A u0."""
    print("[gpu-case] plane lbfgs closed form", flush=True)
    spec, R, T, u0, _ = plane_case(4, (30, 24), (11, 9), amp=0.7, n_probes=0, alpha=0.6)
    Z = np.zeros_like(R)
    ctx = mfr.Context(spec, DEV)
    ctx.set_images(to_dev(Z), to_dev(Z))
    gamma = 0.05
    tu = to_dev(u0)
    rep = ctx.lbfgs(tu, iters=1, mem=2, gamma=gamma)
    assert rep["iters"] == 1, rep
    g = plane.Grid2.from_spec(spec)
    L = plane.laplacian(g).toarray()
    A = 2.0 * g.alpha * g.hybar * (L.T @ L)
    M = A + gamma * np.eye(g.nbar)
    u64 = u0.astype(np.float64)
    want = np.stack([u64[d].ravel() - np.linalg.solve(M, A @ u64[d].ravel()) for d in range(2)]).reshape(u0.shape)
    e = rel_l2(tu.cpu().numpy() - u64, want - u64)
    assert e <= 1e-4, f"closed-form step rel-L2 {e:.3e}"
    ctx.close()
