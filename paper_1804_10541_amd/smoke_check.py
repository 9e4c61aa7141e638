"""One small objective / gradient / Hessian-vector evaluation on cuda:0,
checked against the float64 oracle (used by __graft_entry__.smoke())."""
import numpy as np
import torch


def run():
    from synth import GridSpec, blob_pair, smooth_field
    from oracle import Grid, solver

    from . import mfr

    if not torch.cuda.is_available():
        raise RuntimeError("smoke test needs a GPU")
    spec = GridSpec(m=(20, 18, 16), h=(1.0, 1.0, 1.0), my=(11, 10, 9), tau=0.1, rho=0.1, alpha=1.0)
    R, T, rng = blob_pair(7, spec.m)
    R, T = R.numpy(), T.numpy()
    u0 = smooth_field(rng, spec.my, 0.5)
    p = rng.standard_normal(u0.shape)
    # both sides get the same float32-representable inputs
    R32, T32, u32, p32 = (a.astype(np.float32) for a in (R, T, u0, p))
    dev = torch.device("cuda:0")
    ctx = mfr.Context(spec, dev)
    tR, tT = torch.from_numpy(R32).to(dev), torch.from_numpy(T32).to(dev)
    tu, tp = torch.from_numpy(u32).to(dev), torch.from_numpy(p32).to(dev)
    ctx.set_images(tR, tT)
    J, _, _ = ctx.objective(tu)
    g, _ = ctx.gradient(tu)
    q = ctx.hess_vec(tu, tp)
    torch.cuda.synchronize()
    prob = solver.Problem(Grid.from_spec(spec), R32.astype(np.float64), T32.astype(np.float64))
    u64 = u32.astype(np.float64)
    Jo = prob.objective(u64)[0]
    go = prob.gradient(u64)[1]
    qo = prob.hess_vec(u64, p32.astype(np.float64))
    rel = lambda a, b: float(np.linalg.norm(a - b) / np.linalg.norm(b))
    eJ = abs(J - Jo) / abs(Jo)
    eg = rel(g.cpu().numpy().astype(np.float64), go)
    eq = rel(q.cpu().numpy().astype(np.float64), qo)
    print(f"smoke: J rel err {eJ:.2e}, grad rel-L2 {eg:.2e}, Hv rel-L2 {eq:.2e}")
    if not (eJ <= 1e-5 and eg <= 1e-4 and eq <= 1e-4):
        raise AssertionError(f"GPU result disagrees with the oracle: {eJ:.2e} {eg:.2e} {eq:.2e}")
