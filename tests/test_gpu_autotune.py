"""Tile autotuner on the device: it times real launches, caches the winner,
and a context built under the tuned configuration still meets parity."""
import pytest

from gpu_cases import DEV, assert_parity, blob_case, gpu_eval, oracle_eval, to_dev
from paper_1804_10541_amd import autotune, mfr

pytestmark = pytest.mark.gpu


@pytest.fixture
def restore_tiles():
    prev = mfr.get_tile_config()
    yield
    mfr.set_tile_config(**prev)


def test_autotune_caches_winner_and_keeps_parity(tmp_path, restore_tiles):
    print("[gpu-case] autotune 60x44x30", flush=True)
    spec, R, T, u, probes = blob_case(21, (60, 44, 30), (16, 12, 9), n_probes=2)
    path = str(tmp_path / "tiles.json")
    configs = [dict(bx=32, by=16, chunk_len=0, target_groups=2048), dict(bx=64, by=8, chunk_len=0, target_groups=1024),
               dict(bx=32, by=32, chunk_len=0, target_groups=4096)]
    res = autotune.tune(spec, to_dev(R), to_dev(T), to_dev(u), device=DEV, reps=3, configs=configs, path=path)
    assert res["config"] in configs
    assert all(t > 0 for t, _ in res["timings"])
    assert res["ms"] == min(t for t, _ in res["timings"])
    assert autotune.lookup(spec, DEV, path) == res["config"]
    assert mfr.get_tile_config() == res["config"]
    # apply() takes the cached entry without timing again
    mfr.set_tile_config(32, 16)
    assert autotune.apply(spec, None, None, None, device=DEV, path=path) == res["config"]
    gpu = gpu_eval(spec, R, T, u, probes)
    assert_parity(gpu, oracle_eval(spec, R, T, u, probes))
