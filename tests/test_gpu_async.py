"""Graph-capturable twins of the objective, gradient, CG solve and Gauss-Newton step (results
written by the device into caller memory): equal to the synchronous calls bit
for bit, and HIP graphs captured from them (with the Hessian-vector product and
the Jacobi diagonal) replay to the results of the same calls run eagerly."""
import numpy as np
import pytest
import torch

from gpu_cases import DEV, ct_case, to_dev
from paper_1804_10541_amd import mfr

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("regulariser", ["curvature", "elastic"])
def test_async_scalars_equal_synchronous_calls(regulariser):
    print(f"[gpu-case] async objective / gradient 40x36x28, {regulariser}", flush=True)
    spec, R, T, u, _ = ct_case(3, (40, 36, 28), (11, 10, 8), amp=0.5, n_probes=0, regulariser=regulariser,
                               lame=(0.7, 0.3))
    ctx = mfr.Context(spec, DEV)
    ctx.set_images(to_dev(R), to_dev(T))
    tu = to_dev(u)
    J, D, S = ctx.objective(tu)
    out = ctx.objective_async(tu)
    assert out.cpu().tolist() == [J, D, S]
    g_sync, Jg = ctx.gradient(tu)
    Jd = torch.full((1,), np.nan, dtype=torch.float64, device=DEV)
    g_async = ctx.gradient_async(tu, J=Jd)
    assert Jd.item() == Jg
    assert torch.equal(g_async, g_sync)
    ctx.gradient_async(tu, out=g_async)   # J may be left out
    assert torch.equal(g_async, g_sync)
    ctx.close()


def test_captured_graph_replays_to_eager_results():
    print("[gpu-case] graph capture of objective + gradient + Hv + diagonal 40x36x28", flush=True)
    spec, R, T, u, probes = ct_case(4, (40, 36, 28), (11, 10, 8), amp=0.5, n_probes=3)
    s = torch.cuda.Stream(DEV)
    with torch.cuda.stream(s):
        ctx = mfr.Context(spec, DEV)   # the library enqueues on the stream current at creation
        ctx.set_images(to_dev(R), to_dev(T))
        tu, tp = to_dev(u), to_dev(probes[0])
        sc = torch.empty(4, dtype=torch.float64, device=DEV)
        g = torch.empty_like(tu)
        q = torch.empty_like(tu)
        d = torch.empty_like(tu)
        # warm-up outside the capture (first launches of each kernel)
        ctx.objective_async(tu, out=sc[:3])
        ctx.gradient_async(tu, out=g, J=sc[3:])
        ctx.hess_vec(tu, tp, out=q)
        ctx.jacobi_diag(tu, out=d)
    s.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=s):
        ctx.objective_async(tu, out=sc[:3])
        ctx.gradient_async(tu, out=g, J=sc[3:])
        ctx.hess_vec(tu, tp, out=q)
        ctx.jacobi_diag(tu, out=d)
    rng = np.random.default_rng(9)
    for k in range(4):
        # new inputs in place, then one replay; eager reference of the same calls
        with torch.cuda.stream(s):
            tu.copy_(to_dev(u * (1.0 + 0.1 * k)))
            tp.copy_(to_dev(probes[k % 3] + 0.01 * rng.standard_normal(probes[0].shape).astype(np.float32)))
            sc.fill_(np.nan)
            # on the context's stream: a replay on another stream would race with
            # the eager calls below for the context's workspace
            graph.replay()
            got = (sc.clone(), g.clone(), q.clone(), d.clone())
        s.synchronize()
        with torch.cuda.stream(s):
            J, D, S = ctx.objective(tu)
            g_ref, Jg = ctx.gradient(tu)
            q_ref = ctx.hess_vec(tu, tp)
            d_ref = ctx.jacobi_diag(tu)
        s.synchronize()
        assert got[0].cpu().tolist() == [J, D, S, Jg], k
        assert torch.equal(got[1], g_ref) and torch.equal(got[2], q_ref) and torch.equal(got[3], d_ref), k
    ctx.close()


@pytest.mark.parametrize("precond", [0, 1])
def test_captured_cg_solve_replays_to_the_synchronous_solve(precond):
    print(f"[gpu-case] graph capture of a CG solve (precond {precond}) 40x36x28", flush=True)
    spec, R, T, u, probes = ct_case(5, (40, 36, 28), (11, 10, 8), amp=0.5, n_probes=3)
    s = torch.cuda.Stream(DEV)
    with torch.cuda.stream(s):
        ctx = mfr.Context(spec, DEV)
        ctx.set_images(to_dev(R), to_dev(T))
        tu, tb = to_dev(u), to_dev(probes[0])
        x = torch.empty_like(tu)
        info = torch.empty(3, dtype=torch.float64, device=DEV)
        # eager twin against the synchronous solve
        x_ref, inf = ctx.pcg_solve(tu, tb, max_iter=60, rtol=1e-3, precond=precond)
        ctx.pcg_solve_async(tu, tb, max_iter=60, rtol=1e-3, precond=precond, out=x, info=info)
    s.synchronize()
    assert torch.equal(x, x_ref)
    assert info.cpu().tolist() == [inf["iters"], inf["relres"], inf["flag"]]
    assert inf["flag"] == 0 and inf["iters"] < 60   # converged: the later launches did nothing
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=s):
        ctx.pcg_solve_async(tu, tb, max_iter=60, rtol=1e-3, precond=precond, out=x, info=info)
    for k in range(3):
        with torch.cuda.stream(s):
            tb.copy_(to_dev(probes[k]))
            info.fill_(np.nan)
            graph.replay()
            got_x, got_i = x.clone(), info.clone()
            x_ref, inf = ctx.pcg_solve(tu, tb, max_iter=60, rtol=1e-3, precond=precond)
        s.synchronize()
        assert torch.equal(got_x, x_ref), k
        assert got_i.cpu().tolist() == [inf["iters"], inf["relres"], inf["flag"]], k
    ctx.close()


GN_FIELDS = ("J_before", "J_after", "eta", "slope", "pcg_iters", "pcg_relres", "pcg_flag", "accepted", "ls_trials")


@pytest.mark.parametrize("precond", [0, 1])
def test_captured_gauss_newton_steps_equal_the_synchronous_steps(precond):
    print(f"[gpu-case] graph capture of a Gauss-Newton step (precond {precond}) 40x36x28", flush=True)
    spec, R, T, u, _ = ct_case(6, (40, 36, 28), (11, 10, 8), amp=0.5, n_probes=0)
    opts = dict(pcg_max=30, pcg_rtol=1e-3, precond=precond, armijo_c1=1e-4, armijo_max=6)
    s = torch.cuda.Stream(DEV)
    with torch.cuda.stream(s):
        ctx = mfr.Context(spec, DEV)
        ctx.set_images(to_dev(R), to_dev(T))
        u_sync, u_async = to_dev(u), to_dev(u)
        info = torch.empty(9, dtype=torch.float64, device=DEV)
        # eager twin against the synchronous step
        ref = ctx.gn_step(u_sync, **opts)
        ctx.gn_step_async(u_async, info=info, **opts)
    s.synchronize()
    assert torch.equal(u_async, u_sync)
    assert info.cpu().tolist() == [float(ref[k]) for k in GN_FIELDS]
    assert ref["accepted"] == 1
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=s):
        ctx.gn_step_async(u_async, info=info, **opts)
    # the capture ran nothing: u_async is still the state after one step
    for k in range(3):
        with torch.cuda.stream(s):
            info.fill_(np.nan)
            graph.replay()
            got = info.clone()
            ref = ctx.gn_step(u_sync, **opts)
        s.synchronize()
        assert torch.equal(u_async, u_sync), k
        assert got.cpu().tolist() == [float(ref[k2]) for k2 in GN_FIELDS], k
    ctx.close()
