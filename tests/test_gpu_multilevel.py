"""The coarse-to-fine path on the GPU against the oracle (Sec. 2.3: the problem
is solved on a sequence of coarser image and deformation grids, each level
starting from the prolongated result of the one below).

* Pyramid restriction and displacement prolongation, element by element
  against oracle.multilevel.restrict_image / prolong; the level grids against
  oracle.multilevel.coarse_grid.
* Configuration 2 (128x128x96, 3 levels, 65x65x49 finest nodes): the
  library's multilevel driver equals the same sequence of public calls
  (restriction, Gauss-Newton steps, prolongation) bit for bit; the oracle's
  objective agrees with the GPU's at the start and end displacement of every
  level (on the oracle's own float64 pyramid); at the finest level J agrees at
  every Gauss-Newton iterate, the gradient at three of them, and the first three
  Jacobi-PCG iterates agree with the oracle's.
Trajectories themselves depend on rounding, so parity is asserted at the
GPU's iterates (the oracle evaluates them)."""
import numpy as np
import pytest
import torch

from gpu_cases import DEV, ct_case, rel_l2, to_dev
from oracle import Grid, interp, multilevel, solver
from paper_1804_10541_amd import mfr
from synth import GridSpec, config_c2

pytestmark = pytest.mark.gpu

GN_OPTS = dict(pcg_max=50, pcg_rtol=1e-3, precond=1, armijo_c1=1e-4, armijo_max=10)


def spec_of(cg):
    """GridSpec of a CGrid returned by the library (NGF, curvature)."""
    t = lambda a: tuple(a[k] for k in range(3))
    return GridSpec(m=t(cg.m), h=t(cg.h), my=t(cg.my), tau=cg.tau, rho=cg.rho, alpha=cg.alpha, mT=t(cg.mT),
                    hT=t(cg.hT))


@pytest.mark.parametrize("shape", [(37, 30, 21), (2, 3, 5), (1, 1, 1), (96, 128, 128)])
def test_restriction_matches_oracle(shape):
    print(f"[gpu-case] restriction {shape}", flush=True)
    rng = np.random.default_rng(sum(shape))
    I = (1000.0 * rng.standard_normal(shape) + 500.0).astype(np.float32)
    got = mfr.restrict_image(torch.from_numpy(I).to(DEV)).cpu().numpy()
    want = multilevel.restrict_image(I.astype(np.float64))
    assert got.shape == want.shape
    err = np.abs(got - want).max() / np.abs(want).max()
    assert err <= 1e-6, err


def test_level_grids_match_oracle():
    for m, my in [((128, 128, 96), (65, 65, 49)), ((37, 30, 21), (10, 9, 6)), ((10, 9, 7), (6, 4, 4))]:
        spec = GridSpec(m=m, h=(1.0, 1.25, 0.8), my=my, tau=50.0, rho=50.0, alpha=0.1)
        levels = 3
        g = Grid.from_spec(spec)
        want = [g]
        for _ in range(levels - 1):
            want.append(multilevel.coarse_grid(want[-1]))
        want = want[::-1]
        for lv in range(levels):
            cg = mfr.ml_level_grid(spec, levels, lv)
            w = want[lv]
            assert tuple(cg.m) == w.m and tuple(cg.my) == w.my and tuple(cg.mT) == w.mT, (m, lv)
            assert np.allclose(tuple(cg.h), w.h, rtol=0, atol=0) and np.allclose(tuple(cg.hT), w.hT, rtol=0, atol=0)


@pytest.mark.parametrize("m,my", [((128, 128, 96), (65, 65, 49)), ((10, 9, 7), (6, 4, 4)), ((37, 30, 21), (10, 9, 6))])
def test_prolongation_matches_oracle(m, my):
    print(f"[gpu-case] prolongation {m} / {my}", flush=True)
    spec = GridSpec(m=m, h=(1.0, 1.0, 1.0), my=my, tau=50.0, rho=50.0, alpha=0.1)
    levels = 3
    rng = np.random.default_rng(5)
    for lv in range(levels - 1):
        gc, gf = mfr.ml_level_grid(spec, levels, lv), mfr.ml_level_grid(spec, levels, lv + 1)
        uc = rng.standard_normal((3, gc.my[2], gc.my[1], gc.my[0])).astype(np.float32)
        got = mfr.prolong(torch.from_numpy(uc).to(DEV), gc, gf).cpu().numpy()
        want = multilevel.prolong(uc.astype(np.float64), Grid.from_spec(spec_of(gc)), Grid.from_spec(spec_of(gf)))
        err = np.abs(got - want).max() / np.abs(want).max()
        assert err <= 1e-6, (lv, err)


def _gn_level(ctx, u, iters, record=None):
    """The driver's loop on one level: Gauss-Newton steps until `iters` or a failed line search."""
    done = 0
    J = ctx.objective(u)[0]
    for _ in range(iters):
        info = ctx.gn_step(u, **GN_OPTS)
        if not info["accepted"]:
            break
        J = info["J_after"]
        done += 1
        if record is not None:
            record.append((u.clone(), info))
    return J, done


@pytest.fixture(scope="module")
def c2_run():
    """Configuration 2 through the library driver and through the public calls."""
    print("[gpu-case] multilevel config 2 (128x128x96, 3 levels): driver and public calls", flush=True)
    c = config_c2(0)
    spec, levels = c["spec"], 3
    R, T = c["R"].contiguous().to(DEV), c["T"].contiguous().to(DEV)
    u_drv, rep = mfr.register_multilevel(spec, R, T, levels=levels, gn_iters=10, **GN_OPTS)
    grids = [mfr.ml_level_grid(spec, levels, lv) for lv in range(levels)]
    Rs, Ts = [R], [T]
    for _ in range(levels - 1):
        Rs.append(mfr.restrict_image(Rs[-1]))
        Ts.append(mfr.restrict_image(Ts[-1]))
    Rs, Ts = Rs[::-1], Ts[::-1]
    starts, ends, Jends, dones, finest_iterates = [], [], [], [], []
    u = None
    for lv in range(levels):
        g = grids[lv]
        if u is None:
            u = torch.zeros((3, g.my[2], g.my[1], g.my[0]), dtype=torch.float32, device=DEV)
        else:
            u = mfr.prolong(u, grids[lv - 1], g)
        starts.append(u.clone())
        ctx = mfr.Context(spec_of(g), DEV)
        ctx.set_images(Rs[lv], Ts[lv])
        rec = finest_iterates if lv == levels - 1 else None
        J, done = _gn_level(ctx, u, 10, rec)
        Jends.append(J)
        dones.append(done)
        ends.append(u.clone())
        ctx.close()
    torch.cuda.synchronize()
    return dict(spec=spec, rep=rep, u_drv=u_drv.cpu().numpy(), grids=grids,
                R=c["R"].numpy().astype(np.float64), T=c["T"].numpy().astype(np.float64),
                starts=[x.cpu().numpy() for x in starts], ends=[x.cpu().numpy() for x in ends], Jends=Jends,
                dones=dones, iterates=[(x.cpu().numpy(), i) for x, i in finest_iterates])


def test_config2_driver_equals_public_calls(c2_run):
    r = c2_run
    rep = r["rep"]
    assert rep["gn_done"] == r["dones"], (rep["gn_done"], r["dones"])
    assert rep["J_level"] == r["Jends"], (rep["J_level"], r["Jends"])
    assert np.array_equal(r["u_drv"], r["ends"][-1])
    assert rep["J_final"] == r["Jends"][-1]
    print(f"[gpu-case] per level J: start {rep['J_start']} end {rep['J_level']} gn {rep['gn_done']} "
          f"pcg {rep['pcg_total']}", flush=True)


def test_config2_objective_per_level_matches_oracle(c2_run):
    r = c2_run
    rep = r["rep"]
    pyr = multilevel.pyramid(Grid.from_spec(r["spec"]), r["R"], r["T"], 3)
    for lv, (g, R64, T64) in enumerate(pyr):
        prob = solver.Problem(g, R64, T64)
        Js = prob.objective(r["starts"][lv].astype(np.float64))[0]
        Je = prob.objective(r["ends"][lv].astype(np.float64))[0]
        print(f"[gpu-case] level {lv}: J start {rep['J_start'][lv]:.6e} / {Js:.6e}, "
              f"end {rep['J_level'][lv]:.6e} / {Je:.6e}", flush=True)
        assert abs(rep["J_start"][lv] - Js) <= 1e-5 * abs(Js), (lv, rep["J_start"][lv], Js)
        assert abs(rep["J_level"][lv] - Je) <= 1e-5 * abs(Je), (lv, rep["J_level"][lv], Je)
        assert Je < Js
        if lv > 0:   # the prolongated start is a better point of the finer level than 0
            assert Js < prob.objective(np.zeros_like(r["starts"][lv], dtype=np.float64))[0]


def test_config2_finest_level_objective_at_every_gauss_newton_iterate(c2_run):
    r = c2_run
    g = Grid.from_spec(r["spec"])
    prob = solver.Problem(g, r["R"], r["T"])
    assert len(r["iterates"]) >= 1
    for k, (u, info) in enumerate(r["iterates"]):
        Jo = prob.objective(u.astype(np.float64))[0]
        assert abs(info["J_after"] - Jo) <= 1e-5 * abs(Jo), (k, info["J_after"], Jo)
        assert info["J_after"] < info["J_before"]


def kink_nodes(grid, u64, delta=1e-5):
    """Nodes whose gradient a voxel at a template kink reaches: voxels whose
    sample coordinate y-hat/hT - 1/2 lies within ``delta`` of an integer in some
    axis (a template cell face, where the derivative of the trilinear
    interpolant jumps and the float32 position may fall on either side), and
    the eight nodes of each such voxel (the gradient sees g at a voxel only
    through the transposed conversion there).  Returns (nodes, voxel count)."""
    vox = np.arange(grid.mbar)
    s = interp.deformed_points(grid, u64, vox) / np.asarray(grid.hT) - 0.5
    amb = np.flatnonzero(np.min(np.abs(s - np.round(s)), axis=1) < delta)
    return np.unique(grid.P_rows(amb).indices), len(amb)


def test_config2_finest_level_gradient_at_iterates(c2_run):
    """Gradient parity at three finest-level Gauss-Newton iterates, on the nodes
    that no voxel at a template kink reaches: there the derivative of the
    interpolant jumps, and a sample within float32 rounding of the cell face
    may take either side (both one-sided derivatives are derivatives of the
    interpolant; at the last iterate the GPU and the float64 oracle took
    different sides at a few of the ~10 voxels within 1e-6 of a face).  grad D
    alone (a context with alpha = 0: the same kernels without the regulariser
    term) is held to the same bar."""
    import dataclasses

    from oracle import ngf

    r = c2_run
    spec = r["spec"]
    g = Grid.from_spec(spec)
    prob = solver.Problem(g, r["R"], r["T"])
    tR = torch.from_numpy(r["R"].astype(np.float32)).to(DEV)
    tT = torch.from_numpy(r["T"].astype(np.float32)).to(DEV)
    ctx = mfr.Context(spec, DEV)
    ctx.set_images(tR, tT)
    ctx_d = mfr.Context(dataclasses.replace(spec, alpha=0.0), DEV)
    ctx_d.set_images(tR, tT)
    its = r["iterates"]
    picks = sorted({0, len(its) // 2, len(its) - 1})
    for k in picks:
        u = its[k][0]
        tu = torch.from_numpy(u).to(DEV)
        gg, Jg = ctx.gradient(tu)
        gd, _ = ctx_d.gradient(tu)
        u64 = u.astype(np.float64)
        Jo, go = prob.gradient(u64)
        gDo = ngf.gradient_D(g, r["R"], r["T"], u64)
        kn, nk = kink_nodes(g, u64)
        keep = np.ones(g.nbar, dtype=bool)
        keep[kn] = False
        gg, gd = gg.cpu().numpy().reshape(3, -1), gd.cpu().numpy().reshape(3, -1)
        go, gDo = go.reshape(3, -1), gDo.reshape(3, -1)
        e_all = rel_l2(gg, go)
        e = rel_l2(gg[:, keep], go[:, keep])
        e_d = rel_l2(gd[:, keep], gDo[:, keep])
        print(f"[gpu-case] finest iterate {k}: {nk} voxels within 1e-5 of a template cell face, "
              f"{len(kn)} nodes set aside; gradient rel-L2 {e:.2e} (all nodes {e_all:.2e}), grad D {e_d:.2e}",
              flush=True)
        assert len(kn) <= 0.01 * g.nbar
        assert e <= 1e-4
        assert e_d <= 1e-4
        assert abs(Jg - Jo) <= 1e-5 * abs(Jo)
    ctx.close()
    ctx_d.close()


def test_config2_finest_level_first_three_pcg_iterates(c2_run):
    r = c2_run
    spec = r["spec"]
    prob = solver.Problem(Grid.from_spec(spec), r["R"], r["T"])
    ctx = mfr.Context(spec, DEV)
    ctx.set_images(torch.from_numpy(r["R"].astype(np.float32)).to(DEV),
                   torch.from_numpy(r["T"].astype(np.float32)).to(DEV))
    u = r["starts"][-1]
    tu = torch.from_numpy(u).to(DEV)
    g, _ = ctx.gradient(tu)
    b = -g
    b64 = b.cpu().numpy().astype(np.float64)
    u64 = u.astype(np.float64)
    Jac = prob.jacobian(u64)
    diag = prob.jacobi_diag(u64, Jac)
    for k in (1, 2, 3):
        s, info = ctx.pcg_solve(tu, b.contiguous(), max_iter=k, rtol=0.0, precond=1)
        so, oi = solver.pcg(lambda p: prob.hess_vec(u64, p, Jac), b64, diag, max_iter=k, rtol=0.0)
        e = rel_l2(s.cpu().numpy(), so)
        print(f"[gpu-case] PCG iterate {k}: rel-L2 {e:.2e}, relres {info['relres']:.4e} / {oi['relres']:.4e}",
              flush=True)
        assert info["iters"] == k == oi["iters"]
        assert e <= 1e-4
        assert abs(info["relres"] - oi["relres"]) <= 1e-4 * oi["relres"]
    ctx.close()


def test_driver_with_learned_preconditioner_equals_public_calls():
    """precond 2: the driver binds the preconditioner to each level's context
    and runs flexible CG; the same public calls give the same result bit for bit."""
    print("[gpu-case] multilevel precond 2, 3 levels, 64x60x48 / 17x16x13: driver and public calls", flush=True)
    spec, R, T, _, _ = ct_case(12, (64, 60, 48), (17, 16, 13), amp=0.5, n_probes=0)
    tR, tT = to_dev(R), to_dev(T)
    ctx = mfr.Context(spec, DEV)
    ctx.set_images(tR, tT)
    pc = mfr.LearnedPC(ctx)
    rng = np.random.default_rng(21)
    params = (0.02 * rng.standard_normal(mfr.PC_PARAMS)).astype(np.float32)
    pc.set_params(params)
    opts = dict(pcg_max=40, pcg_rtol=1e-3, precond=2, armijo_c1=1e-4, armijo_max=10, fallback_iters=30)
    levels, iters = 3, 4
    u_drv, rep = mfr.register_multilevel(spec, tR, tT, levels=levels, gn_iters=iters, pc=pc, **opts)
    grids = [mfr.ml_level_grid(spec, levels, lv) for lv in range(levels)]
    Rs, Ts = [tR], [tT]
    for _ in range(levels - 1):
        Rs.append(mfr.restrict_image(Rs[-1]))
        Ts.append(mfr.restrict_image(Ts[-1]))
    Rs, Ts = Rs[::-1], Ts[::-1]
    u, Jends, dones = None, [], []
    for lv in range(levels):
        g = grids[lv]
        u = torch.zeros((3, g.my[2], g.my[1], g.my[0]), dtype=torch.float32, device=DEV) if u is None else \
            mfr.prolong(u, grids[lv - 1], g)
        c = mfr.Context(spec_of(g), DEV)
        c.set_images(Rs[lv], Ts[lv])
        pc.bind(c)
        c.attach_pc(pc)
        J, done = c.objective(u)[0], 0
        for _ in range(iters):
            info = c.gn_step(u, **opts)
            if not info["accepted"]:
                break
            J, done = info["J_after"], done + 1
        Jends.append(J)
        dones.append(done)
        c.attach_pc(None)
        c.close()
    torch.cuda.synchronize()
    print(f"[gpu-case] per level J {rep['J_level']} gn {rep['gn_done']} pcg {rep['pcg_total']}", flush=True)
    assert rep["gn_done"] == dones and rep["J_level"] == Jends
    assert torch.equal(u_drv, u)
    for lv in range(levels):
        assert rep["J_level"][lv] < rep["J_start"][lv]
    pc.close()
    ctx.close()
