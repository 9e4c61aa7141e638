"""Training and evaluation of the learned preconditioner on Gauss-Newton
systems that the registration itself produces.

Systems: for every seed, a CT-like pair of the 128 x 128 x 96 multilevel
workload (65 x 65 x 49 deformation nodes, eps 50, alpha 0.1) for even seeds
and of one of the ten batched sizes (256^2 / 512^2 x 94..136, quarter-resolution
grids) for odd seeds; a Gauss-Newton
trajectory from u = 0 with Jacobi-PCG; at every iterate u_k the system
(H + alpha nabla^2 S) s = -grad J(u_k).  Training runs Jacobi-PCG on each
system and takes an Adam step on residuals sampled along it (the library's
mfr_pc_train_system).  Evaluation solves held-out systems to relative
residual 1e-3 with Jacobi-PCG and with flexible CG + the network, and reports
iterations and wall time of both.

    python -m paper_1804_10541_amd.pc_train --train 0:40 --eval 200:205 \\
        --out paper_1804_10541_amd/weights/pc_ct128.npy
    python -m paper_1804_10541_amd.pc_train --c2-only --eval 210:212 --gn-iters 8 \\
        --eval-only paper_1804_10541_amd/weights/pc_ct128.npy
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_1804_10541_amd import mfr  # noqa: E402

WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights", "pc_ct128.npy")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def workload_spec(m=(128, 128, 96), my=(65, 65, 49)):
    from synth import GridSpec

    return GridSpec(m=m, h=(1.0, 1.0, 1.0), my=my, tau=50.0, rho=50.0, alpha=0.1)


def init_params(seed=0, scale_last=0.1):
    """He-style initialisation (fan-in 27 x 16) of the four layers; the last
    layer scaled down so the start is close to the Jacobi direction."""
    rng = np.random.default_rng(seed)
    out = []
    for l in range(4):
        W = rng.standard_normal((27, 16, 16)) * np.sqrt(2.0 / (27 * 16))
        b = np.zeros(16)
        if l == 3:
            W *= scale_last
            W[:, :, 3:] = 0.0
        out.append(np.concatenate([W.ravel(), b]))
    return np.concatenate(out).astype(np.float32)


def parse_range(s):
    a, b = (int(k) for k in s.split(":"))
    return list(range(a, b))


def c4_specs():
    from synth import GridSpec, config_c4_sizes, quarter_nodes

    return [GridSpec(m=m, h=(1.0, 1.0, 1.0), my=quarter_nodes(m), tau=50.0, rho=50.0, alpha=0.1)
            for m in config_c4_sizes()]


def seed_spec(seed, mix=True):
    """Workload of a seed: even seeds the 128 x 128 x 96 multilevel workload,
    odd seeds cycle through the ten batched sizes (mix=False: always the former)."""
    if not mix or seed % 2 == 0:
        return workload_spec()
    return c4_specs()[(seed // 2) % 10]


class Systems:
    """Gauss-Newton systems along registration trajectories, one context per grid size."""

    def __init__(self, device):
        self.device = torch.device(device)
        self.ctxs = {}

    def ctx(self, spec, R=None, T=None):
        """Context of this grid size, created with the tile configuration the
        autotuner picks for it (timed on R, T when given)."""
        key = (tuple(spec.m), tuple(spec.my))
        if key not in self.ctxs:
            if R is not None:
                from paper_1804_10541_amd import autotune

                u0 = torch.zeros((3, spec.my[2], spec.my[1], spec.my[0]), dtype=torch.float32, device=self.device)
                autotune.apply(spec, R, T, u0, device=self.device)
            self.ctxs[key] = mfr.Context(spec, self.device)
        return self.ctxs[key]

    def trajectory(self, seed, spec, gn_iters, pcg_max=50, pcg_rtol=1e-3):
        from synth import ct_pair

        R, T, _, _ = ct_pair(seed, spec.m, device=self.device)
        ctx = self.ctx(spec, R, T)
        ctx.set_images(R, T)
        self._images = (R, T)
        u = torch.zeros(ctx.node_shape(), dtype=torch.float32, device=self.device)
        for k in range(gn_iters):
            g, _ = ctx.gradient(u)
            b = torch.neg(g)
            yield ctx, k, u, b
            info = ctx.gn_step(u, pcg_max=pcg_max, pcg_rtol=pcg_rtol, precond=1)
            if not info["accepted"]:
                break

    def close(self):
        for c in self.ctxs.values():
            c.close()
        self.ctxs = {}


def val_iterations(params, systems, device="cuda:0"):
    """Mean flexible-CG iterations to relative residual 1e-3 on validation systems
    [(ctx, u, b)] (no fallback)."""
    its = []
    for ctx, u, b in systems:
        pc = mfr.LearnedPC(ctx)
        pc.set_params(params)
        ctx.attach_pc(pc)
        _, info = ctx.pcg_solve(u, b, max_iter=300, rtol=1e-3, precond=2)
        its.append(info["iters"])
        ctx.attach_pc(None)
        pc.close()
    return float(np.mean(its))


def train(seeds, epochs=2, gn_iters=10, lr=1e-3, pcg_iters=24, sample_every=3, params=None, device="cuda:0",
          mix=True, log_every=10, val_seeds=(), val_every=10):
    """Adam on the relative-energy loss over the systems of `seeds`.  With
    val_seeds, every val_every seeds the flexible-CG iteration count on the
    validation systems is measured and the best parameters so far are kept
    (the one-step loss alone does not track CG convergence)."""
    src = Systems(device)
    specs = [workload_spec()] + (c4_specs() if mix else [])
    pc = None
    history = []
    val = []
    if val_seeds:
        vsrc = Systems(device)
        for vs in val_seeds:
            for ctx, k, u, b in vsrc.trajectory(vs, seed_spec(vs, mix), 3):
                val.append((ctx, u.clone(), b.clone()))
    best = (float("inf"), None)
    if val:
        p0 = init_params() if params is None else params
        best = (val_iterations(p0, val, device), p0)
        log(f"[train] validation at start: {best[0]:.2f} iterations")
    count = 0
    for ep in range(epochs):
        for i, seed in enumerate(seeds):
            for ctx, k, u, b in src.trajectory(seed, seed_spec(seed, mix), gn_iters):
                if pc is None:
                    pc = mfr.LearnedPC(ctx, train=True, capacity=specs)
                    pc.set_params(init_params() if params is None else params)
                elif pc.ctx is not ctx:
                    pc.bind(ctx)
                info = pc.train_system(u, b, lr=lr, pcg_iters=pcg_iters, sample_every=sample_every)
                history.append(info["loss_mean"])
            count += 1
            if val and count % val_every == 0:
                cur = pc.get_params()
                it = val_iterations(cur, val, device)
                if it < best[0]:
                    best = (it, cur)
                log(f"[train] epoch {ep} seed {seed}: validation {it:.2f} iterations (best {best[0]:.2f})")
            if (i + 1) % log_every == 0 or i + 1 == len(seeds):
                recent = history[-gn_iters * log_every:]
                log(f"[train] epoch {ep} seed {seed}: mean loss {np.mean(recent):.4f} over {len(recent)} systems")
    params = pc.get_params()
    pc.close()
    src.close()
    if val:
        it = val_iterations(params, val, device)
        if it < best[0]:
            best = (it, params)
        params = best[1]
        log(f"[train] kept parameters with {best[0]:.2f} validation iterations")
        vsrc.close()
    return params, history


def evaluate(params, seeds, gn_iters=10, rtol=1e-3, max_iter=500, device="cuda:0", spec=None, mix=True,
             fallback=True):
    """Per system: iterations and wall time of Jacobi-PCG and of flexible CG with
    the network (Jacobi fallback after twice the Jacobi count), and of plain CG,
    on the same systems."""
    src = Systems(device)
    rows = []
    pcs = {}
    for seed in seeds:
        sp = spec or seed_spec(seed, mix)
        for ctx, k, u, b in src.trajectory(seed, sp, gn_iters):
            if id(ctx) not in pcs:
                pcs[id(ctx)] = mfr.LearnedPC(ctx)
                pcs[id(ctx)].set_params(params)
            ctx.attach_pc(pcs[id(ctx)])
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, ij = ctx.pcg_solve(u, b, max_iter=max_iter, rtol=rtol, precond=1)
            torch.cuda.synchronize()
            tj = time.perf_counter() - t0
            fb = 2 * ij["iters"] if fallback else 0
            t0 = time.perf_counter()
            _, il = ctx.pcg_solve(u, b, max_iter=max_iter, rtol=rtol, precond=2, fallback_iters=fb)
            torch.cuda.synchronize()
            tl = time.perf_counter() - t0
            t0 = time.perf_counter()
            _, ic = ctx.pcg_solve(u, b, max_iter=max_iter, rtol=rtol, precond=0)
            torch.cuda.synchronize()
            tc = time.perf_counter() - t0
            rows.append(dict(seed=seed, m=list(sp.m), gn=k, jacobi_iters=ij["iters"], jacobi_s=tj,
                             learned_iters=il["iters"], learned_s=tl, learned_flag=il["flag"],
                             fallback=il["used_fallback"], cg_iters=ic["iters"], cg_s=tc))
    for ctx in src.ctxs.values():
        ctx.attach_pc(None)
    for pc in pcs.values():
        pc.close()
    src.close()
    return rows


def summarize(rows):
    J = np.array([r["jacobi_iters"] for r in rows], dtype=float)
    L = np.array([r["learned_iters"] for r in rows], dtype=float)
    C = np.array([r["cg_iters"] for r in rows], dtype=float)
    tj = sum(r["jacobi_s"] for r in rows)
    tl = sum(r["learned_s"] for r in rows)
    tc = sum(r["cg_s"] for r in rows)
    return dict(systems=len(rows), jacobi_iters_mean=float(J.mean()), learned_iters_mean=float(L.mean()),
                cg_iters_mean=float(C.mean()), jacobi_s=tj, learned_s=tl, cg_s=tc,
                iter_gain_vs_jacobi=float(J.sum() / max(L.sum(), 1)), time_gain_vs_jacobi=tj / tl,
                time_gain_vs_cg=tc / tl, fallbacks=int(sum(r["fallback"] for r in rows)),
                not_converged=int(sum(r["learned_flag"] != 0 for r in rows)))


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--train", default="0:40")
    ap.add_argument("--eval", default="200:205")
    ap.add_argument("--epochs", type=int, default=2)
    ap.add_argument("--gn-iters", type=int, default=10)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--pcg-iters", type=int, default=24)
    ap.add_argument("--sample-every", type=int, default=3)
    ap.add_argument("--init", default=None, help="start from these parameters (.npy)")
    ap.add_argument("--c2-only", action="store_true", help="train on the 128 x 128 x 96 workload only")
    ap.add_argument("--val", default="150:152", help="validation seeds (early stopping on CG iterations)")
    ap.add_argument("--val-every", type=int, default=10)
    ap.add_argument("--out", default=WEIGHTS)
    ap.add_argument("--eval-only", metavar="PARAMS", default=None,
                    help="skip training: evaluate these parameters (.npy) on the --eval seeds")
    args = ap.parse_args()
    import json

    if args.eval_only:
        rows = evaluate(np.load(args.eval_only), parse_range(args.eval), args.gn_iters, mix=not args.c2_only)
        for r in rows:
            log(f"[eval] seed {r['seed']} GN {r['gn']}: Jacobi {r['jacobi_iters']} ({1e3 * r['jacobi_s']:.2f} ms), "
                f"learned {r['learned_iters']} ({1e3 * r['learned_s']:.2f} ms), CG {r['cg_iters']}")
        print(json.dumps(summarize_by_workload(rows)), flush=True)
        return
    init = np.load(args.init) if args.init else None
    t0 = time.perf_counter()
    params, hist = train(parse_range(args.train), args.epochs, args.gn_iters, args.lr, args.pcg_iters,
                         args.sample_every, init, mix=not args.c2_only, val_seeds=parse_range(args.val),
                         val_every=args.val_every)
    log(f"[train] {len(hist)} systems in {time.perf_counter() - t0:.1f} s; "
        f"loss {np.mean(hist[:10]):.4f} -> {np.mean(hist[-10:]):.4f}")
    os.makedirs(os.path.dirname(args.out), exist_ok=True)
    np.save(args.out, params)
    t0 = time.perf_counter()
    rows = evaluate(params, parse_range(args.eval), args.gn_iters, mix=not args.c2_only)
    log(f"[eval] {len(rows)} systems in {time.perf_counter() - t0:.1f} s")
    print(json.dumps(summarize_by_workload(rows)), flush=True)


def summarize_by_workload(rows):
    """summarize() over all rows and per image size."""
    out = {"all": summarize(rows)}
    for m in sorted({tuple(r["m"]) for r in rows}):
        out["x".join(map(str, m))] = summarize([r for r in rows if tuple(r["m"]) == m])
    return out


if __name__ == "__main__":
    main()
