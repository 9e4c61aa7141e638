"""Shared helpers for the GPU parity tests: seeded inputs, evaluation through
the C ABI, evaluation by the oracle on the very same float32 inputs."""
import numpy as np
import torch

from oracle import Grid, ngf, solver
from paper_1804_10541_amd import mfr
from synth import GridSpec, blob_pair, ct_pair, smooth_field

DEV = torch.device("cuda:0")


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def blob_case(seed, m, my, h=(1.0, 1.0, 1.0), tau=0.1, rho=0.1, alpha=1.0, amp=0.5, n_probes=3, mT=None,
              hT=None, T_override=None, distance="ngf", regulariser="curvature", lame=(1.0, 0.0)):
    """Gaussian-blob pair + smooth displacement + N(0,1) probes, all float32."""
    spec = GridSpec(m=tuple(m), h=tuple(h), my=tuple(my), tau=tau, rho=rho, alpha=alpha, mT=mT, hT=hT,
                    distance=distance, regulariser=regulariser, lame_mu=lame[0], lame_lambda=lame[1])
    R, T, rng = blob_pair(seed, spec.m)
    if mT is not None:
        _, T, rng = blob_pair(seed, tuple(mT))
    u0 = smooth_field(rng, spec.my, amp)
    probes = rng.standard_normal((n_probes,) + u0.shape)
    f32 = lambda a: np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    return spec, f32(R), f32(T if T_override is None else T_override), f32(u0), f32(probes)


def ct_case(seed, m, my, amp=0.5, n_probes=3, alpha=0.1, eps=50.0, distance="ngf", regulariser="curvature",
            lame=(1.0, 0.0)):
    spec = GridSpec(m=tuple(m), h=(1.0, 1.0, 1.0), my=tuple(my), tau=eps, rho=eps, alpha=alpha, distance=distance,
                    regulariser=regulariser, lame_mu=lame[0], lame_lambda=lame[1])
    R, T, _, rng = ct_pair(seed, spec.m)
    u0 = smooth_field(rng, spec.my, amp)
    probes = rng.standard_normal((n_probes,) + u0.shape)
    f32 = lambda a: np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    return spec, f32(R.numpy()), f32(T.numpy()), f32(u0), f32(probes)


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def gpu_eval(spec, R, T, u, probes, diag=True):
    ctx = mfr.Context(spec, DEV)
    ctx.set_images(to_dev(R), to_dev(T))
    tu = to_dev(u)
    J, D, S = ctx.objective(tu)
    g, Jg = ctx.gradient(tu)
    hv = [ctx.hess_vec(tu, to_dev(p)).cpu().numpy() for p in probes]
    dg = ctx.jacobi_diag(tu).cpu().numpy() if diag else None
    torch.cuda.synchronize()
    out = dict(J=J, D=D, S=S, Jg=Jg, grad=g.cpu().numpy(), hv=hv, diag=dg)
    ctx.close()
    return out


def oracle_eval(spec, R, T, u, probes, diag=True):
    grid = Grid.from_spec(spec)
    prob = solver.Problem(grid, R.astype(np.float64), T.astype(np.float64))
    u64 = u.astype(np.float64)
    J, D, S = prob.objective(u64)
    _, g = prob.gradient(u64)
    Jac = prob.jacobian(u64)
    hv = [prob.hess_vec(u64, p.astype(np.float64), Jac) for p in probes]
    dg = prob.jacobi_diag(u64, Jac) if diag else None
    return dict(J=J, D=D, S=S, grad=g, hv=hv, diag=dg, prob=prob, Jac=Jac)


def assert_parity(gpu, ora, tol_obj=1e-5, tol_vec=1e-4, check_diag=True):
    assert abs(gpu["J"] - ora["J"]) <= tol_obj * abs(ora["J"]), (gpu["J"], ora["J"])
    assert abs(gpu["D"] - ora["D"]) <= tol_obj * abs(ora["D"]), (gpu["D"], ora["D"])
    assert abs(gpu["S"] - ora["S"]) <= tol_obj * max(abs(ora["S"]), 1e-12 * abs(ora["J"])), (gpu["S"], ora["S"])
    assert abs(gpu["Jg"] - ora["J"]) <= tol_obj * abs(ora["J"])
    e = rel_l2(gpu["grad"], ora["grad"])
    assert e <= tol_vec, f"gradient rel-L2 {e:.3e}"
    for k, (a, b) in enumerate(zip(gpu["hv"], ora["hv"])):
        e = rel_l2(a, b)
        assert e <= tol_vec, f"Hv[{k}] rel-L2 {e:.3e}"
    if check_diag and gpu["diag"] is not None:
        e = rel_l2(gpu["diag"], ora["diag"])
        assert e <= tol_vec, f"diag rel-L2 {e:.3e}"
