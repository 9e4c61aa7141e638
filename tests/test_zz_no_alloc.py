"""mfr_hess_vec_noalloc (the Hessian-vector product for callers that cannot
allocate device memory) against mfr_hess_vec on a caller workspace: the same
kernels on the same inputs give the same floats.  Two calls in a row on the
library's one scratch array, the second with a smaller problem, so the second
call must not depend on anything the first left behind; the first problem is
checked again afterwards.  Also checked against the oracle."""
import numpy as np
import pytest
import torch

from gpu_cases import DEV, blob_case, ct_case, oracle_eval, rel_l2
from paper_1804_10541_amd import mfr

pytestmark = pytest.mark.gpu

CASES = [
    ("ct 128x128x96 / 65x65x49", lambda: ct_case(11, (128, 128, 96), (65, 65, 49), n_probes=1), False),
    ("blob 37x30x26 / 12x11x9", lambda: blob_case(3, (37, 30, 26), (12, 11, 9), n_probes=1), True),
]


def _run_pair(spec, R, T, u, p):
    tR, tT, tu, tp = (torch.from_numpy(a).to(DEV) for a in (R, T, u, p))
    ctx = mfr.Context(spec, DEV)
    ctx.set_images(tR, tT)
    want = ctx.hess_vec(tu, tp)
    got = torch.full_like(want, float("nan"))
    mfr.hess_vec_noalloc(spec, tR, tT, tu, tp, got)
    torch.cuda.synchronize()
    ctx.close()
    return got.cpu().numpy(), want.cpu().numpy()


def test_noalloc_hess_vec_equals_workspace_path_twice_in_a_row():
    results = []
    for name, make, check_oracle in CASES:
        print(f"[gpu-case] noalloc hess_vec {name}", flush=True)
        spec, R, T, u, probes = make()
        got, want = _run_pair(spec, R, T, u, probes[0])
        assert np.isfinite(got).all()
        assert np.array_equal(got, want), rel_l2(got, want)
        if check_oracle:
            qo = oracle_eval(spec, R, T, u, probes[:1], diag=False)["hv"][0]
            assert rel_l2(got, qo) <= 1e-4
        results.append((spec, R, T, u, probes[0], want))
    # the larger problem again, after the smaller one overwrote the array's start
    spec, R, T, u, p, want = results[0]
    print("[gpu-case] noalloc hess_vec first case again", flush=True)
    got, _ = _run_pair(spec, R, T, u, p)
    assert np.array_equal(got, want)
