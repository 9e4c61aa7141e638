"""Batched path (several independent pairs of different sizes advanced
together): every result must equal the single-pair path bit for bit, and the
single-pair path is held to the oracle elsewhere; the Hessian-vector products
are also checked against the oracle directly."""
import numpy as np
import pytest
import torch

from gpu_cases import DEV, blob_case, ct_case, oracle_eval, rel_l2, to_dev
from paper_1804_10541_amd import mfr

pytestmark = pytest.mark.gpu

# uneven pairs: ragged tiles in x, y and z, different node grids and parameters
PAIRS = [
    dict(seed=11, m=(40, 28, 21), my=(11, 8, 6)),
    dict(seed=12, m=(64, 48, 40), my=(17, 13, 11)),
    dict(seed=13, m=(33, 70, 17), my=(9, 18, 5)),
]


def _blob_pairs(amp=0.5):
    return [blob_case(p["seed"], p["m"], p["my"], amp=amp, n_probes=1) for p in PAIRS]


def _ct_pairs(sizes, seed0=40):
    out = []
    for i, (m, my) in enumerate(sizes):
        out.append(ct_case(seed0 + i, m, my, amp=0.0, n_probes=0))
    return out


def test_batch_hess_vec_equals_single_and_matches_oracle():
    print("[gpu-case] batch hess_vec, 3 uneven blob pairs", flush=True)
    cases = _blob_pairs()
    specs = [c[0] for c in cases]
    b = mfr.Batch(specs, levels=1, device=DEV)
    b.set_images([to_dev(c[1]) for c in cases], [to_dev(c[2]) for c in cases])
    us = [to_dev(c[3]) for c in cases]
    ps = [to_dev(c[4][0]) for c in cases]
    qs = [q.cpu().numpy() for q in b.hess_vec(us, ps)]
    for k, (spec, R, T, u, probes) in enumerate(cases):
        ctx = mfr.Context(spec, DEV)
        ctx.set_images(to_dev(R), to_dev(T))
        q1 = ctx.hess_vec(to_dev(u), to_dev(probes[0])).cpu().numpy()
        same = bool(np.array_equal(q1, qs[k]))
        assert same, f"pair {k}: batched and single-pair Hv differ"
        ref = oracle_eval(spec, R, T, u, probes, diag=False)
        e = rel_l2(qs[k], ref["hv"][0])
        assert e <= 1e-4, f"pair {k}: Hv rel-L2 {e:.3e}"
        ctx.close()
    b.close()


@pytest.mark.parametrize("use_graph", [False, True])
def test_batch_register_equals_single_pair_register(use_graph):
    print(f"[gpu-case] batch register, 3 uneven CT pairs, 2 levels, graph={use_graph}", flush=True)
    sizes = [((48, 40, 36), (13, 11, 10)), ((64, 64, 30), (17, 17, 8)), ((40, 56, 44), (11, 15, 12))]
    cases = _ct_pairs(sizes)
    specs = [c[0] for c in cases]
    opts = dict(gn_iters=4, pcg_max=12, pcg_rtol=1e-2, precond=1)
    b = mfr.Batch(specs, levels=2, device=DEV)
    b.set_images([to_dev(c[1]) for c in cases], [to_dev(c[2]) for c in cases])
    ub, rep = b.register(use_graph=use_graph, **opts)
    torch.cuda.synchronize()
    print(f"[gpu-case] batch report {rep}", flush=True)
    if use_graph:
        assert rep["graph_launches"] > 0
    for k, (spec, R, T, _, _) in enumerate(cases):
        u1, r1 = mfr.register_multilevel(spec, to_dev(R), to_dev(T), levels=2, **opts)
        torch.cuda.synchronize()
        same = bool(np.array_equal(u1.cpu().numpy(), ub[k].cpu().numpy()))
        assert same, f"pair {k}: displacements differ (J {r1['J_final']!r} vs {rep['J_final'][k]!r})"
        assert r1["J_final"] == rep["J_final"][k], (k, r1["J_final"], rep["J_final"][k])
        assert sum(r1["gn_done"]) == rep["gn_done"][k]
        assert sum(r1["pcg_total"]) == rep["pcg_total"][k]
        assert rep["gn_done"][k] >= 1
    b.close()


def test_batch_graph_replay_equals_direct_launches_twice():
    """Two calls in a row on one batch (graph captured by the first, replayed
    by the second) against direct launches."""
    print("[gpu-case] batch register graph reuse, 2 blob pairs", flush=True)
    cases = _blob_pairs(amp=0.0)[:2]
    specs = [c[0] for c in cases]
    opts = dict(gn_iters=3, pcg_max=10, pcg_rtol=1e-3, precond=1)
    res = {}
    for use_graph in (False, True):
        b = mfr.Batch(specs, levels=1, device=DEV)
        b.set_images([to_dev(c[1]) for c in cases], [to_dev(c[2]) for c in cases])
        runs = [b.register(use_graph=use_graph, **opts) for _ in range(2)]
        torch.cuda.synchronize()
        res[use_graph] = [[u.cpu().numpy() for u in r[0]] for r in runs]
        b.close()
    for run in range(2):
        for k in range(len(cases)):
            same = bool(np.array_equal(res[False][run][k], res[True][run][k]))
            assert same, (run, k)
            same = bool(np.array_equal(res[True][0][k], res[True][run][k]))
            assert same, (run, k)
