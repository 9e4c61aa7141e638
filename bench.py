#!/usr/bin/env python3
"""Benchmark of the matrix-free NGF + curvature Gauss-Newton step on one MI355X.

Workload (default): the large single-level Gauss-Newton step -- a 512 x 512 x
900 CT-like float32 volume pair, deformation grid 129 x 129 x 225 nodes, eps
50 HU, alpha 0.1, smooth initial displacement of max 0.5 voxel.  One step is
one call of the library's Gauss-Newton step: objective and gradient, exact
Jacobi diagonal, Jacobi-PCG with exactly 20 Hessian-vector products
(rtol 0), Armijo line search (one or more objective evaluations) and the
update.  All inputs are synthetic and resident in HBM before timing starts.

Output: one JSON line.  ``value`` = voxel-Hessian-vector products per second
over whole steps (image voxels x 20 / step time, in Gvoxel/s).  ``roofline``
refers to the dominant kernel (the voxel-tile kernel in Hessian-vector mode),
timed with HIP events on the stream it runs on.  ``cpu_baseline`` times the
float64 oracle on a bounded crop of the same volume on the host.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HV_PER_STEP = 20
HBM_PEAK_GBS = 8000.0            # MI355X HBM3E, 8 TB/s
FP32_VECTOR_PEAK_TFLOPS = 157.3  # MI355X fp32 vector (256 CU x 2.4 GHz)

# Algorithmic work of one Hessian-vector product (per image voxel / per node).
# Flops: the per-voxel arithmetic of the fused matrix-free scheme for one
# output voxel (grid conversion of u and p, trilinear template value and
# gradient, six short differences of T and R, residual and the rho-hat row,
# dr a, the column gather of dr^T, g w, transposed conversion), FMA = 2 flops,
# no halo recomputation counted.  Bytes: R and T read once (8 B/voxel); u, p
# read and q written once (36 B/node).
HV_FLOP_PER_VOXEL = 217
HV_BYTES_PER_VOXEL = 8
HV_BYTES_PER_NODE = 36
# The same product for the sum-of-squared-differences distance (dr/dT = identity):
# the NGF-only arithmetic (differences of T and R, the three weighted sums, norms and
# residual, the rho-hat row, dr a, the dr^T gather: 119 flop) drops out, and so does
# the reference image (its Gauss-Newton matrix does not depend on R): T once per voxel.
SSD_HV_FLOP_PER_VOXEL = 98
SSD_HV_BYTES_PER_VOXEL = 4

# HBM bytes per launch of the Hessian-vector tile kernel at the 512x512x900 workload come
# from the committed rocprofv3 summary (FETCH_SIZE and WRITE_SIZE, each scaled by what the
# counter reads for a plain copy kernel).  The summary records a hash of the kernel's
# sources and the tile configuration it was taken with; for other sources or another
# configuration the traffic is reported as null.
HV_PROFILE = os.path.join(ROOT, "profiles", "ngf_tile_hv_512x512x900.md")


def profiled_traffic(tile_cfg):
    """Measured HBM bytes per launch of the Hessian-vector kernel from the committed
    profile summary, if it was taken with the current kernel sources and tile
    configuration; else None."""
    import re

    if not tile_cfg or not os.path.exists(HV_PROFILE):
        return None
    text = open(HV_PROFILE).read()
    m_hash = re.search(r"Kernel sources \(sha256, 16 hex\): `([0-9a-f]+)`", text)
    m_tile = re.search(r"Tile configuration: (\d+)x(\d+), split target (\d+)", text)
    m_bytes = re.search(r"HBM traffic per launch: ([0-9,]+) bytes", text)
    from paper_1804_10541_amd.profsum import kernel_source_hash

    if not (m_hash and m_tile and m_bytes) or m_hash.group(1) != kernel_source_hash():
        return None
    if (tile_cfg["bx"], tile_cfg["by"], tile_cfg["target_groups"]) != tuple(int(g) for g in m_tile.groups()):
        return None
    return int(m_bytes.group(1).replace(",", ""))


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def workload_spec(name):
    from synth import GridSpec

    if name == "c3":
        return GridSpec(m=(512, 512, 900), h=(1.0, 1.0, 1.0), my=(129, 129, 225), tau=50.0, rho=50.0, alpha=0.1)
    if name == "c3-half":
        return GridSpec(m=(512, 512, 450), h=(1.0, 1.0, 1.0), my=(129, 129, 113), tau=50.0, rho=50.0, alpha=0.1)
    if name == "small":
        return GridSpec(m=(128, 128, 96), h=(1.0, 1.0, 1.0), my=(33, 33, 25), tau=50.0, rho=50.0, alpha=0.1)
    raise ValueError(name)


def c4_specs():
    """Ten CT-like pairs of uneven sizes (256^2 and 512^2 in-plane, 94-136
    slices), quarter-resolution deformation grids ceil(m/4) + 1."""
    from synth import GridSpec, config_c4_sizes, quarter_nodes

    return [GridSpec(m=s, h=(1.0, 1.0, 1.0), my=quarter_nodes(s), tau=50.0, rho=50.0, alpha=0.1)
            for s in config_c4_sizes()]


def batch_leg(dev, tune):
    """Multilevel registration of the ten uneven pairs: the batched path (one
    persistent launch per phase for all pairs, CG iterations replayed from
    captured HIP graphs) against per-pair runs of the single-pair path, and a
    check that both return the same displacements bit for bit."""
    import torch

    from paper_1804_10541_amd import autotune, mfr
    from synth import ct_pair

    specs = c4_specs()
    pairs = [ct_pair(k, s.m, device=dev)[:2] for k, s in enumerate(specs)]
    torch.cuda.synchronize()
    big = max(range(len(specs)), key=lambda k: specs[k].voxels)
    cfg = None
    if tune:
        ub = torch.zeros((3,) + tuple(reversed(specs[big].my)), dtype=torch.float32, device=dev)
        cfg = autotune.apply(specs[big], pairs[big][0], pairs[big][1], ub, device=dev)
    opts = dict(gn_iters=10, pcg_max=50, pcg_rtol=1e-3, precond=1)
    b = mfr.Batch(specs, levels=3, device=dev)
    b.set_images([p[0] for p in pairs], [p[1] for p in pairs])
    b.register(use_graph=True, gn_iters=1, pcg_max=8, pcg_rtol=1e-3, precond=1)   # warm-up and graph capture
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ub_list, rep = b.register(use_graph=True, **opts)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    log(f"[bench] batched: {t_batch:.3f} s, gn {rep['gn_done']}, pcg {rep['pcg_total']}, "
        f"graph replays {rep['graph_launches']}")
    for k, s in enumerate(specs[:1]):   # warm-up of the single-pair path
        mfr.register_multilevel(s, pairs[k][0], pairs[k][1], levels=3, gn_iters=1, pcg_max=8, pcg_rtol=1e-3)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    seq = [mfr.register_multilevel(s, pairs[k][0], pairs[k][1], levels=3, **opts) for k, s in enumerate(specs)]
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    same = all(torch.equal(seq[k][0], ub_list[k]) for k in range(len(specs)))
    log(f"[bench] sequential: {t_seq:.3f} s; identical displacements: {same}")
    b.close()
    vox = sum(s.voxels for s in specs)
    return {"workload": f"{len(specs)} CT-like pairs, " + ", ".join("x".join(map(str, s.m)) for s in specs)
                        + "; 3 levels, 10 Gauss-Newton steps per level, Jacobi-PCG <= 50 at rtol 1e-3",
            "pairs": len(specs), "voxels": vox, "nodes": sum(s.nodes for s in specs),
            "batched_s": round(t_batch, 4), "sequential_s": round(t_seq, 4), "speedup": round(t_seq / t_batch, 3),
            "graph_replays": rep["graph_launches"], "gn_steps": rep["gn_done"], "pcg_iters": rep["pcg_total"],
            "identical_to_sequential": bool(same), "tile_config": cfg}


def ssd_leg(dev, spec, R, T, u0, reps=20):
    """Hessian-vector products and the Jacobi diagonal with the sum-of-squared-
    differences distance on the same pair, displacement and tile configuration
    as the headline step (HIP-event kernel timings on the context's stream)."""
    import dataclasses

    import torch

    from paper_1804_10541_amd import mfr

    s = dataclasses.replace(spec, distance="ssd")
    ctx = mfr.Context(s, dev)
    ctx.set_images(R, T)
    gen = torch.Generator(device=dev).manual_seed(5)
    p = torch.randn(u0.shape, generator=gen, device=dev, dtype=torch.float32)
    q = torch.empty_like(p)
    diag = torch.empty_like(p)
    for _ in range(3):
        ctx.hess_vec(u0, p, out=q)
    ctx.jacobi_diag(u0, out=diag)
    torch.cuda.synchronize()
    ctx.profile(True)
    ctx.profile_read(reset=True)
    t0 = time.perf_counter()
    for _ in range(reps):
        ctx.hess_vec(u0, p, out=q)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ctx.jacobi_diag(u0, out=diag)
    torch.cuda.synchronize()
    prof = ctx.profile_read(reset=True)
    ctx.profile(False)
    ctx.close()
    mbar, nbar = s.voxels, s.nodes
    hv_n, hv_ms = prof["tile_hv"]
    np_n, np_ms = prof["node_pass"]
    hv_avg = hv_ms / max(hv_n, 1)
    np_avg = np_ms / max(np_n, 1)
    tflops = SSD_HV_FLOP_PER_VOXEL * mbar / (hv_avg * 1e-3) / 1e12
    gbs = (SSD_HV_BYTES_PER_VOXEL * mbar + HV_BYTES_PER_NODE * nbar) / (hv_avg * 1e-3) / 1e9
    out = {"workload": "the headline pair and displacement with the sum-of-squared-differences distance",
           "kernel": "ngf_tile_kernel<HV, SSD>", "avg_ms": round(hv_avg, 4), "launches": hv_n,
           "kernel_gvoxel_s": round(mbar / (hv_avg * 1e-3) / 1e9, 2),
           "with_node_pass_gvoxel_s": round(mbar / ((hv_avg + np_avg) * 1e-3) / 1e9, 2),
           "wall_gvoxel_s": round(mbar * reps / dt / 1e9, 2),
           "alu_tflops": round(tflops, 3), "alu_frac": round(tflops / FP32_VECTOR_PEAK_TFLOPS, 4),
           "flop_per_voxel": SSD_HV_FLOP_PER_VOXEL,
           "hbm_algorithmic_gbs": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
           "jacobi_diag_ms": round(prof["jacobi_diag"][1] / max(prof["jacobi_diag"][0], 1), 3)}
    log(f"[bench] ssd: {out}")
    return out


def regulariser_leg(dev, spec, R, T, u0, regulariser, steps=2, **lame):
    """Gauss-Newton steps with another regulariser on the headline pair and start
    (same step as the headline: 20 Jacobi-PCG iterations, rtol 0), with the
    node-pass and Jacobi-diagonal kernel times (events on the context's stream)."""
    import dataclasses

    import torch

    from paper_1804_10541_amd import mfr

    s = dataclasses.replace(spec, regulariser=regulariser, **lame)
    ctx = mfr.Context(s, dev)
    ctx.set_images(R, T)
    u = u0.clone()
    gn = dict(pcg_max=HV_PER_STEP, pcg_rtol=0.0, precond=1, armijo_c1=1e-4, armijo_max=10)
    ctx.gn_step(u, **gn)   # warm-up
    torch.cuda.synchronize()
    ctx.profile(True)
    ctx.profile_read(reset=True)
    t0 = time.perf_counter()
    infos = [ctx.gn_step(u, **gn) for _ in range(steps)]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = ctx.profile_read(reset=True)
    ctx.profile(False)
    ctx.close()
    avg = lambda k: round(prof[k][1] / max(prof[k][0], 1), 4)
    n_hv = sum(i["pcg_iters"] for i in infos)
    out = {"workload": f"the headline Gauss-Newton step with the {regulariser} regulariser"
                       + (f" (lame_mu {lame['lame_mu']:g}, lame_lambda {lame['lame_lambda']:g})" if lame else ""),
           "ms_per_step": round(dt * 1e3 / steps, 3), "gvoxel_s": round(s.voxels * n_hv / dt / 1e9, 3),
           "J": [round(i["J_after"], 1) for i in infos],
           "tile_hv_ms": avg("tile_hv"), "node_pass_ms": avg("node_pass"), "jacobi_diag_ms": avg("jacobi_diag")}
    log(f"[bench] {regulariser}: {out}")
    return out


def lbfgs_leg(dev, spec, R, T, u0, iters=3, gamma=100.0):
    """L-BFGS iterations (two-loop recursion, H_0 = alpha nabla^2 S + gamma I
    solved in the cosine basis, Armijo steps) on the headline pair from the same
    start, and the time of one H_0 solve (events on the context's stream)."""
    import torch

    from paper_1804_10541_amd import mfr

    ctx = mfr.Context(spec, dev)
    ctx.set_images(R, T)
    v = torch.randn(u0.shape, generator=torch.Generator(device=dev).manual_seed(9), device=dev)
    x = torch.empty_like(v)
    for _ in range(2):
        ctx.h0_solve(v, gamma, out=x)
    torch.cuda.synchronize()
    reps = 10
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        ctx.h0_solve(v, gamma, out=x)
    e1.record()
    torch.cuda.synchronize()
    h0_ms = e0.elapsed_time(e1) / reps
    u = u0.clone()
    ctx.lbfgs(u.clone(), iters=1, mem=5, gamma=gamma)   # warm-up
    torch.cuda.synchronize()
    rep = ctx.lbfgs(u, iters=iters, mem=5, gamma=gamma)
    ctx.close()
    nb = spec.nodes
    h0_flop = 4.0 * 3 * nb * sum(spec.my)   # forward and inverse cosine transforms along x, y, z
    out = {"workload": f"the headline pair and start, {iters} L-BFGS iterations, memory 5, gamma {gamma:g}",
           "iters": rep["iters"], "status": rep["status"], "evals": rep["evals"],
           "J_initial": rep["J_initial"], "J_final": rep["J_final"],
           "s_per_iter": round(rep["seconds"] / max(rep["iters"], 1), 4),
           "h0_solve_ms": round(h0_ms, 3), "h0_solve_tflops": round(h0_flop / (h0_ms * 1e-3) / 1e12, 2)}
    log(f"[bench] lbfgs: {out}")
    return out


def pc_leg(dev):
    """PCG solve time to relative residual 1e-3, flexible CG with the learned
    preconditioner (Jacobi fallback after twice the Jacobi count) against
    Jacobi-PCG on the same held-out Gauss-Newton systems."""
    import numpy as np

    from paper_1804_10541_amd import pc_train

    if not os.path.exists(pc_train.WEIGHTS):
        return {"skipped": f"no trained weights at {os.path.relpath(pc_train.WEIGHTS, ROOT)}"}
    params = np.load(pc_train.WEIGHTS)
    out = {"weights": os.path.relpath(pc_train.WEIGHTS, ROOT), "rtol": 1e-3}
    out["network_vs_hv"] = network_vs_hv(dev, params)
    for name, seeds, spec in (("128x128x96", [200], pc_train.workload_spec()),
                              ("512x512x128", [201], pc_train.c4_specs()[8])):
        rows = pc_train.evaluate(params, seeds, gn_iters=4, spec=spec, device=dev)
        summ = pc_train.summarize(rows)
        out[name] = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in summ.items()}
        log(f"[bench] learned preconditioner {name}: {out[name]}")
    return out


def network_vs_hv(dev, params, reps=50):
    """One application of the learned preconditioner's network (its convolutions,
    the input features computed by the first) against one Hessian-vector product
    (voxel tiles and node pass) on the 128 x 128 x 96 / 65 x 65 x 49 workload:
    mean times from HIP events on the context's stream (the library's timing)."""
    import torch

    from paper_1804_10541_amd import mfr, pc_train
    from synth import ct_pair, smooth_field

    spec = pc_train.workload_spec()
    R, T, _, rng = ct_pair(210, spec.m, device=dev)
    ctx = mfr.Context(spec, dev)
    ctx.set_images(R, T)
    pc = mfr.LearnedPC(ctx)
    pc.set_params(params)
    u = torch.from_numpy(smooth_field(rng, spec.my, 0.5).astype("float32")).to(dev)
    r = torch.randn(u.shape, generator=torch.Generator(device=dev).manual_seed(3), device=dev)
    z, q = torch.empty_like(r), torch.empty_like(r)
    for _ in range(3):
        pc.apply(u, r, out=z)
        ctx.hess_vec(u, r, out=q)
    ctx.profile(True)
    ctx.profile_read(reset=True)
    for _ in range(reps):
        pc.apply(u, r, out=z)
    for _ in range(reps):
        ctx.hess_vec(u, r, out=q)
    pr = ctx.profile_read(reset=True)
    ctx.profile(False)
    net_us = 1e3 * pr["pc_network"][1] / max(pr["pc_network"][0], 1)
    hv_us = 1e3 * (pr["tile_hv"][1] + pr["node_pass"][1]) / reps
    out = {"nodes": list(spec.my), "network_us": round(net_us, 2), "hv_us": round(hv_us, 2),
           "network_per_hv": round(net_us / hv_us, 3)}
    pc.close()
    ctx.close()
    log(f"[bench] learned preconditioner network vs Hv: {out}")
    return out


def device_leg(dev):
    """The device as the runtime reports it, and the bandwidth of a plain
    streaming kernel measured on it (torch's neg over 1 GiB: 1 GiB read and
    1 GiB written per launch, HIP events over 10 launches): the measured
    counterpart of the 8 TB/s datasheet figure the roofline uses."""
    import torch

    props = torch.cuda.get_device_properties(dev)
    src = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
    dst = torch.empty_like(src)
    for _ in range(3):
        torch.neg(src, out=dst)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        torch.neg(src, out=dst)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 10
    del src, dst
    out = {"name": props.name, "gcn_arch": getattr(props, "gcnArchName", None),
           "compute_units": props.multi_processor_count, "memory_bytes": int(props.total_memory),
           "copy_kernel_gbs": round(2 * (1 << 30) / (ms * 1e-3) / 1e9, 1), "copy_kernel_ms": round(ms, 4)}
    log(f"[bench] device: {out}")
    return out


def memory_leg():
    """Device memory of the library at 512 x 512 x 900 and 512 x 512 x 450 voxels
    (same 129 x 129 node grid in x, y; 225 / 113 node planes): the workspace of
    a context (exact size query) split into the zero-bordered template copy,
    which grows with the voxels, and the rest (tables, transposed-conversion
    partials, reductions and the node vectors of CG / Gauss-Newton: the
    derivative memory, independent of the voxel count), beside the images."""
    from paper_1804_10541_amd import mfr

    out = {}
    for name in ("c3", "c3-half"):
        s = workload_spec(name)
        ws = mfr.workspace_size(s)
        tpl = 4 * (s.m[0] + 4) * (s.m[1] + 4) * (s.m[2] + 4)
        out[name] = {"voxels": s.voxels, "nodes": s.nodes, "images_bytes": 8 * s.voxels, "workspace_bytes": ws,
                     "template_copy_bytes": tpl, "derivative_bytes": ws - tpl,
                     "derivative_bytes_per_node": round((ws - tpl) / s.nodes, 1)}
    log(f"[bench] memory: {out}")
    return out


def plane_leg(dev, levels=3):
    """The two-dimensional path at 4096 x 4096 pixels / 2049 x 2049 nodes (the
    largest size of the paper's two-dimensional GPU table): kernel times of the
    objective, gradient and Hessian-vector product (HIP events on the context's
    stream), a Gauss-Newton step with 20 Hessian-vector products, and a
    three-level registration (10 Gauss-Newton steps per level, Jacobi-PCG <= 50
    at rtol 1e-3)."""
    import torch

    from paper_1804_10541_amd import mfr
    from synth import config_section

    c = config_section(0, n_probes=1)
    spec = c["spec"]
    R, T = torch.from_numpy(c["R"]).to(dev), torch.from_numpy(c["T"]).to(dev)
    u0 = torch.from_numpy(c["u0"]).to(dev)
    p = torch.from_numpy(c["probes"][0]).to(dev)
    ctx = mfr.Context(spec, dev)
    ctx.set_images(R, T)
    q = torch.empty_like(p)
    for _ in range(3):
        ctx.objective(u0)
        ctx.gradient(u0)
        ctx.hess_vec(u0, p, out=q)
    torch.cuda.synchronize()
    reps = 20
    ctx.profile(True)
    ctx.profile_read(reset=True)
    t0 = time.perf_counter()
    for _ in range(reps):
        ctx.gradient(u0)   # objective value included (one synchronisation)
    torch.cuda.synchronize()
    t_grad = (time.perf_counter() - t0) / reps
    for _ in range(reps):
        ctx.objective(u0)
        ctx.hess_vec(u0, p, out=q)
    ctx.jacobi_diag(u0)
    torch.cuda.synchronize()
    prof = ctx.profile_read(reset=True)
    ctx.profile(False)
    u = u0.clone()
    gn = dict(pcg_max=HV_PER_STEP, pcg_rtol=0.0, precond=1, armijo_c1=1e-4, armijo_max=10)
    ctx.gn_step(u, **gn)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    info = ctx.gn_step(u, **gn)
    torch.cuda.synchronize()
    t_gn = time.perf_counter() - t0
    ctx.close()
    avg = lambda k: round(prof[k][1] / max(prof[k][0], 1), 4)
    mbar, nbar = spec.m[0] * spec.m[1], spec.my[0] * spec.my[1]
    hv_ms = avg("tile_hv")
    ml_opts = dict(levels=levels, gn_iters=10, pcg_max=50, pcg_rtol=1e-3, armijo_c1=1e-4, armijo_max=10, precond=1)
    mfr.register_multilevel(spec, R, T, **dict(ml_opts, gn_iters=1))   # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, rep = mfr.register_multilevel(spec, R, T, **ml_opts)
    torch.cuda.synchronize()
    t_ml = time.perf_counter() - t0
    out = {"workload": f"two-dimensional section pair {spec.m[0]}x{spec.m[1]} pixels, {spec.my[0]}x{spec.my[1]} "
                       "nodes, eps 0.05, alpha 1",
           "pixels": mbar, "nodes": nbar,
           "gradient_call_ms": round(t_grad * 1e3, 4),
           "kernel_ms": {k: avg(k) for k in ("tile_obj", "tile_grad", "tile_hv", "jacobi_diag", "node_pass")},
           "hv_kernel_gpixel_s": round(mbar / (hv_ms * 1e-3) / 1e9, 2),
           "hv_hbm_algorithmic_gbs": round((8 * mbar + 24 * nbar) / (hv_ms * 1e-3) / 1e9, 1),
           "gn_step_ms": round(t_gn * 1e3, 3), "gn_step_J": [info["J_before"], info["J_after"]],
           "registration_s": round(t_ml, 4), "registration_gn_steps": rep["gn_done"],
           "registration_pcg_iters": rep["pcg_total"], "registration_J": [rep["J_start"][0], rep["J_final"]],
           "paper_context": "GTX 980, float32: gradient 35.3 ms, full three-level L-BFGS registration 1.51 s "
                            "(Table objfunGradRuntime_CUDA, Fig. multiLevelRuntime_CUDA; another GPU and "
                            "another optimiser)"}
    log(f"[bench] plane: {out}")
    return out


def _stats_ms(xs):
    import numpy as np

    a = np.array(xs) * 1e3
    return {"median": round(float(np.median(a)), 4), "min": round(float(a.min()), 4), "max": round(float(a.max()), 4),
            "reps": len(xs)}


def ops_leg(dev, reps=30, warm=3):
    """Per-operation times at configuration 1 (32^3 voxels / 17^3 nodes, blobs, eps 0.1,
    alpha 1) and configuration 2's finest level (128x128x96 CT-like / 65x65x49 nodes):
    each library call (objective, gradient, Hessian-vector product, Jacobi diagonal)
    timed by host wall clock around the call with the device synchronised before and
    after, 3 warm-ups then 30 repetitions (median, min, max); and the float64 oracle's
    same operations (single-thread worker process) at configuration 1, 30 repetitions,
    and at configuration 2, one."""
    import subprocess

    import numpy as np
    import torch

    from paper_1804_10541_amd import mfr
    from synth import GridSpec, config_c1, ct_pair, smooth_field

    out = {}
    c1 = config_c1(0, n_probes=1)
    s2 = GridSpec(m=(128, 128, 96), h=(1.0, 1.0, 1.0), my=(65, 65, 49), tau=50.0, rho=50.0, alpha=0.1)
    R2, T2, _, rng2 = ct_pair(0, s2.m, device=dev)
    u2 = torch.from_numpy(smooth_field(rng2, s2.my, 0.5).astype("float32")).to(dev)
    cases = {
        "configuration 1: 32x32x32 / 17x17x17": (
            c1["spec"], torch.from_numpy(c1["R"].astype("float32")).to(dev),
            torch.from_numpy(c1["T"].astype("float32")).to(dev), torch.from_numpy(c1["u0"].astype("float32")).to(dev)),
        "configuration 2, finest level: 128x128x96 / 65x65x49": (s2, R2, T2, u2),
    }
    for name, (spec, R, T, u) in cases.items():
        ctx = mfr.Context(spec, dev)
        ctx.set_images(R, T)
        p = torch.randn(u.shape, generator=torch.Generator(device=dev).manual_seed(3), device=dev)
        q, g, d = torch.empty_like(p), torch.empty_like(p), torch.empty_like(p)
        calls = {"objective": lambda: ctx.objective(u), "gradient": lambda: ctx.gradient(u, out=g),
                 "hess_vec": lambda: ctx.hess_vec(u, p, out=q), "jacobi_diag": lambda: ctx.jacobi_diag(u, out=d)}
        res = {}
        for op, call in calls.items():
            for _ in range(warm):
                call()
            torch.cuda.synchronize()
            ts = []
            for _ in range(reps):
                t0 = time.perf_counter()
                call()
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
            res[op] = _stats_ms(ts)
        ctx.close()
        out[name] = {"voxels": spec.voxels, "nodes": spec.nodes, "gpu_call_ms": res}
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    for name, which, n in (("configuration 1: 32x32x32 / 17x17x17", "c1", reps),
                           ("configuration 2, finest level: 128x128x96 / 65x65x49", "c2", 1)):
        pr = subprocess.run([sys.executable, os.path.abspath(__file__), "--ops-worker", which, str(n)],
                            stdout=subprocess.PIPE, env=env, timeout=600)
        if pr.returncode == 0:
            out[name]["oracle_ms"] = json.loads(pr.stdout.decode().strip().splitlines()[-1])
            out[name]["oracle_threads"] = 1
    log(f"[bench] ops: {out}")
    return out


def _ops_worker(which, reps):
    """The oracle's per-operation times (float64, assembled sparse Jacobian, one
    thread): objective, gradient, Jacobian assembly, Hessian-vector product with the
    assembled Jacobian, Jacobi diagonal; prints one JSON line."""
    import numpy as np

    from oracle import Grid, solver
    from synth import GridSpec, config_c1, ct_pair, smooth_field

    if which == "c1":
        c = config_c1(0, n_probes=1)
        spec, R, T, u = c["spec"], c["R"], c["T"], c["u0"]
    else:
        spec = GridSpec(m=(128, 128, 96), h=(1.0, 1.0, 1.0), my=(65, 65, 49), tau=50.0, rho=50.0, alpha=0.1)
        R, T, _, rng = ct_pair(0, spec.m)
        u = smooth_field(rng, spec.my, 0.5)
        R, T = R.double().numpy(), T.double().numpy()
    prob = solver.Problem(Grid.from_spec(spec), np.asarray(R, dtype=np.float64), np.asarray(T, dtype=np.float64))
    u = np.asarray(u, dtype=np.float64)
    p = np.random.default_rng(3).standard_normal(u.shape)
    Jac = prob.jacobian(u)
    ops = {"objective": lambda: prob.objective(u), "gradient": lambda: prob.gradient(u),
           "jacobian_assembly": lambda: prob.jacobian(u), "hess_vec": lambda: prob.hess_vec(u, p, Jac),
           "jacobi_diag": lambda: prob.jacobi_diag(u, Jac)}
    res = {}
    for op, call in ops.items():
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            call()
            ts.append(time.perf_counter() - t0)
        res[op] = _stats_ms(ts)
    print(json.dumps(res), flush=True)


CPU_CROP = (128, 128, 64)   # voxels of one oracle sample (x, y, z)
CPU_CROP_NODES = (33, 33, 17)


def _oracle_crop_work(Rc, Tc, spec, seed, budget_s):
    """One sample of the cpu_baseline: the float64 oracle's derivative work of a
    Gauss-Newton step on a crop (spec: the crop's grid; objective, gradient,
    Jacobi diagonal and up to HV_PER_STEP Hessian-vector products with the
    assembled Jacobian).  Returns (Hessian-vector products done, seconds)."""
    import numpy as np

    from oracle import Grid, solver
    from synth import smooth_field

    u = smooth_field(np.random.default_rng(seed), spec.my, 0.5)
    g = Grid(spec.m, spec.h, spec.my, spec.tau, spec.rho, spec.alpha)
    t0 = time.perf_counter()
    prob = solver.Problem(g, Rc, Tc)
    prob.objective(u)
    _, grad = prob.gradient(u)
    Jac = prob.jacobian(u)
    prob.jacobi_diag(u, Jac)
    p = -grad
    n_hv = 0
    for _ in range(HV_PER_STEP):
        p = prob.hess_vec(u, p, Jac)
        p /= np.linalg.norm(p)
        n_hv += 1
        if time.perf_counter() - t0 > budget_s:
            break
    return n_hv, time.perf_counter() - t0


def _cpu_worker(path, seed, budget_s, min_s):
    """Entry of a cpu_baseline worker process (never touches the GPU): loads its
    crop from ``path``, repeats the step's derivative work on it (a new
    displacement each time) until ``min_s`` seconds have passed (at most four
    times) and prints one JSON line."""
    import numpy as np

    from synth import GridSpec

    d = np.load(path)
    spec = GridSpec(m=tuple(d["m"]), h=tuple(d["h"]), my=tuple(d["my"]), tau=float(d["eps"]), rho=float(d["eps"]),
                    alpha=float(d["alpha"]))
    n, t, reps = 0, 0.0, 0
    while True:
        n_hv, dt = _oracle_crop_work(d["R"], d["T"], spec, seed + 100 * reps, budget_s)
        n, t, reps = n + n_hv, t + dt, reps + 1
        if t >= min_s or reps >= 4:
            break
    print(json.dumps({"n_hv": n, "seconds": t, "reps": reps}), flush=True)


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(R, T, u0, spec, budget_s=25.0, max_workers=16):
    """The float64 oracle, as it stands (scipy.sparse, one thread per process),
    on crops of the same volume: single-thread on rank 0 at N = 1, and on all
    host cores as independent worker processes, one crop each (the oracle has
    no parallel path of its own).  Crops of 128 x 128 x 64 voxels / 33 x 33 x 17
    nodes (the workload's grid ratio), centred and shifted along z per worker."""
    import subprocess
    import tempfile

    import numpy as np

    mx, my_, mz = spec.m
    cm = CPU_CROP

    def crop(k):
        x0, y0 = (mx - cm[0]) // 2, (my_ - cm[1]) // 2
        z0 = min(max((mz - cm[2]) // 2 + (k - 8) * cm[2] // 2, 0), mz - cm[2])
        sl = (slice(z0, z0 + cm[2]), slice(y0, y0 + cm[1]), slice(x0, x0 + cm[0]))
        return R[sl].double().cpu().numpy(), T[sl].double().cpu().numpy()

    vox = cm[0] * cm[1] * cm[2]
    cores = os.cpu_count() or 1
    workers = max(1, min(cores, max_workers))
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")

    def launch(path, seed, min_s):
        return subprocess.Popen([sys.executable, os.path.abspath(__file__), "--cpu-worker", path, str(seed),
                                 str(budget_s), str(min_s)], stdout=subprocess.PIPE, env=env)

    def result(pr):
        outp, _ = pr.communicate()
        return json.loads(outp.decode().strip().splitlines()[-1]) if pr.returncode == 0 else None

    with tempfile.TemporaryDirectory() as tmp:
        files = []
        for k in range(workers):
            Rk, Tk = crop(k)
            path = os.path.join(tmp, f"crop{k}.npz")
            np.savez(path, R=Rk, T=Tk, m=np.array(cm), h=np.array(spec.h), my=np.array(CPU_CROP_NODES),
                     eps=spec.tau, alpha=spec.alpha)
            files.append(path)
        # one thread: one worker process alone, the centre crop, about 10 s of work
        one = result(launch(files[8 % workers], 1, 10.0))
        # all host cores: one worker per core at once, one pass each
        procs = [launch(path, k + 1, 0.0) for k, path in enumerate(files)]
        res = [r for r in (result(pr) for pr in procs) if r is not None]
    # the workers' timed sections overlap (all start after the same imports): the
    # longest one is the wall time of the concurrent work
    wall = max((r["seconds"] for r in res), default=0.0)
    n_all = sum(r["n_hv"] for r in res)
    single = vox * one["n_hv"] / one["seconds"] / 1e9 if one else None
    allc = vox * n_all / wall / 1e9 if res else None
    return {"value": single, "unit": "Gvoxel/s", "cores": 1, "kind": "oracle",
            "sample": f"crop {cm[0]}x{cm[1]}x{cm[2]} voxels / {CPU_CROP_NODES[0]}x{CPU_CROP_NODES[1]}x"
                      f"{CPU_CROP_NODES[2]} nodes of the same volume, one worker process with one thread; "
                      f"{one['reps'] if one else 0} x (objective + gradient + Jacobi diagonal + "
                      f"{HV_PER_STEP} Hessian-vector products with the assembled float64 Jacobian, scipy.sparse): "
                      f"{one['n_hv'] if one else 0} Hessian-vector products in "
                      f"{one['seconds'] if one else 0.0:.1f} s",
            "all_cores": {"value": allc, "unit": "Gvoxel/s", "processes": len(res), "host_cpus": cores,
                          "sample": f"{len(res)} single-thread worker processes at once, one crop each (z-shifted), "
                                    f"one step's work per crop; {n_all} Hessian-vector products, longest worker {wall:.1f} s"},
            "cpu_model": _cpu_model()}


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c3", choices=["c3", "c3-half", "small"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the ten-pair batched registration leg")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default tile configuration")
    ap.add_argument("--no-pc", action="store_true", help="skip the learned-preconditioner leg")
    ap.add_argument("--no-ssd", action="store_true", help="skip the sum-of-squared-differences leg")
    ap.add_argument("--no-lbfgs", action="store_true", help="skip the L-BFGS leg")
    ap.add_argument("--no-regularisers", action="store_true", help="skip the diffusive and elastic legs")
    ap.add_argument("--no-plane", action="store_true", help="skip the two-dimensional leg")
    ap.add_argument("--plane-only", action="store_true",
                    help="run only the two-dimensional leg (for profiling it) and print its result")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (reference for HBM byte counters)")
    ap.add_argument("--no-ops", action="store_true", help="skip the per-operation times at configurations 1 and 2")
    ap.add_argument("--cpu-worker", nargs=4, metavar=("CROP", "SEED", "BUDGET", "MIN_S"), help=argparse.SUPPRESS)
    ap.add_argument("--ops-worker", nargs=2, metavar=("CONFIG", "REPS"), help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.cpu_worker:   # a cpu_baseline worker process: oracle only, no GPU
        _cpu_worker(args.cpu_worker[0], int(args.cpu_worker[1]), float(args.cpu_worker[2]), float(args.cpu_worker[3]))
        return
    if args.ops_worker:   # oracle per-operation times, no GPU
        _ops_worker(args.ops_worker[0], int(args.ops_worker[1]))
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1804_10541_amd import mfr
    from synth import ct_pair, smooth_field

    dev = torch.device("cuda:0")
    if args.plane_only:
        if args.copy_calibration:
            src = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
            dst = torch.empty_like(src)
            for _ in range(3):
                torch.neg(src, out=dst)
            torch.cuda.synchronize()
            del src, dst
        print(json.dumps({"plane": plane_leg(dev)}), flush=True)
        return
    spec = workload_spec(args.workload)
    log(f"[bench] generating {args.workload}: {spec.m} voxels, {spec.my} nodes")
    t0 = time.perf_counter()
    R, T, _, rng = ct_pair(0, spec.m, device=dev)
    u0 = torch.from_numpy(smooth_field(rng, spec.my, 0.5).astype("float32")).to(dev)
    torch.cuda.synchronize()
    log(f"[bench] inputs ready in {time.perf_counter() - t0:.1f} s")

    if args.copy_calibration:
        # a plain streaming kernel of known size: 1 GiB read, 1 GiB written (torch's neg kernel)
        src = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.neg(src, out=dst)
        torch.cuda.synchronize()
        del src, dst

    tile_cfg = None
    if not args.no_autotune:
        from paper_1804_10541_amd import autotune

        tile_cfg = autotune.apply(spec, R, T, u0, device=dev)
        log(f"[bench] tile configuration {tile_cfg}")
    ctx = mfr.Context(spec, dev)
    ctx.set_images(R, T)
    u = u0.clone()
    gn = dict(pcg_max=HV_PER_STEP, pcg_rtol=0.0, precond=1, armijo_c1=1e-4, armijo_max=10)
    for i in range(args.warmup):
        info = ctx.gn_step(u, **gn)
        log(f"[bench] warmup {i}: J {info['J_before']:.6e} -> {info['J_after']:.6e}, eta {info['eta']}")
    torch.cuda.synchronize()
    ctx.profile(True)
    ctx.profile_read(reset=True)
    infos = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        infos.append(ctx.gn_step(u, **gn))
        log(f"[bench] step {i}: J {infos[-1]['J_before']:.6e} -> {infos[-1]['J_after']:.6e}, "
            f"pcg {infos[-1]['pcg_iters']} relres {infos[-1]['pcg_relres']:.3e}")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = ctx.profile_read(reset=True)
    ctx.profile(False)
    peak_mem = torch.cuda.max_memory_allocated(dev)

    mbar = spec.voxels
    nbar = spec.nodes
    n_hv = sum(i["pcg_iters"] for i in infos)
    ms_step = dt * 1e3 / args.steps
    value = mbar * n_hv / dt / 1e9
    hv_launches, hv_ms = prof["tile_hv"]
    np_launches, np_ms = prof["node_pass"]
    hv_avg_ms = hv_ms / max(hv_launches, 1)
    flops = HV_FLOP_PER_VOXEL * mbar
    achieved_tflops = flops / (hv_avg_ms * 1e-3) / 1e12
    alg_bytes = HV_BYTES_PER_VOXEL * mbar + HV_BYTES_PER_NODE * nbar
    hv_hbm_gbs = alg_bytes / (hv_avg_ms * 1e-3) / 1e9
    traffic = profiled_traffic(tile_cfg) if args.workload == "c3" else None
    out = {
        "metric": "GN Hessian-vector Gvoxel/s + % HBM peak; PCG solve time, learned vs Jacobi",
        "value": round(value, 3),
        "unit": "Gvoxel/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"large single-level Gauss-Newton step, {spec.m[0]}x{spec.m[1]}x{spec.m[2]} "
                               f"CT-like float32 pair, {spec.my[0]}x{spec.my[1]}x{spec.my[2]} nodes, "
                               f"{HV_PER_STEP} Hessian-vector products per step (Jacobi-PCG, rtol 0)",
                   "voxels": mbar, "nodes": nbar, "hv_per_step": HV_PER_STEP},
        "roofline": {"bound": "alu", "achieved": round(achieved_tflops, 3), "peak": FP32_VECTOR_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(achieved_tflops / FP32_VECTOR_PEAK_TFLOPS, 4),
                     "traffic": traffic,
                     "kernel": "ngf_tile_kernel<HV>", "avg_ms": round(hv_avg_ms, 4), "launches": hv_launches,
                     "flop_per_voxel": HV_FLOP_PER_VOXEL},
        "hv": {"kernel_gvoxel_s": round(mbar / (hv_avg_ms * 1e-3) / 1e9, 2),
               "with_node_pass_gvoxel_s": round(mbar / ((hv_avg_ms + np_ms / max(np_launches, 1)) * 1e-3) / 1e9, 2),
               "hbm_algorithmic_gbs": round(hv_hbm_gbs, 1),
               "hbm_frac": round(hv_hbm_gbs / HBM_PEAK_GBS, 4)},
        "kernel_ms": {k: (v[0], round(v[1] / max(v[0], 1), 4)) for k, v in prof.items()},
        "peak_device_bytes": int(peak_mem),
        "workspace_bytes": int(ctx.ws_bytes),
        "memory": memory_leg(),
        "tile_config": tile_cfg,
        "device": device_leg(dev),
    }
    if not args.no_cpu_baseline:
        log("[bench] timing the float64 oracle on a crop (cpu_baseline)")
        out["cpu_baseline"] = cpu_baseline(R, T, u0, spec)
    del ctx
    if not args.no_ssd:
        log("[bench] sum-of-squared-differences distance")
        out["ssd"] = ssd_leg(dev, spec, R, T, u0)
    if not args.no_lbfgs:
        log("[bench] L-BFGS")
        out["lbfgs"] = lbfgs_leg(dev, spec, R, T, u0)
    if not args.no_regularisers:
        log("[bench] diffusive and elastic regularisers")
        out["diffusive"] = regulariser_leg(dev, spec, R, T, u0, "diffusive")
        out["elastic"] = regulariser_leg(dev, spec, R, T, u0, "elastic", lame_mu=1.0, lame_lambda=1.0)
    del R, T
    if not args.no_plane:
        log("[bench] two-dimensional path")
        out["plane"] = plane_leg(dev)
    if not args.no_ops and args.workload == "c3":
        log("[bench] per-operation times at configurations 1 and 2")
        out["ops"] = ops_leg(dev)
    if not args.no_batch and args.workload != "small":
        log("[bench] ten-pair batched registration")
        out["batch"] = batch_leg(dev, not args.no_autotune)
    if not args.no_pc and args.workload != "small":
        log("[bench] learned preconditioner vs Jacobi")
        out["pcg_learned_vs_jacobi"] = pc_leg(dev)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
