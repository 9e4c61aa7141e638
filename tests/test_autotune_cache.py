"""Host-side logic of the tile autotuner: candidate set, cache keys and the
JSON cache round trip (no GPU needed)."""
import json

from paper_1804_10541_amd import autotune
from synth import GridSpec


def test_candidates_cover_every_shape_and_split():
    c = autotune.candidates()
    assert len(c) == len(autotune.SHAPES) * (len(autotune.GROUP_TARGETS) + len(autotune.CHUNK_LENS))
    assert {d["chunk_len"] for d in c} == {0, *autotune.CHUNK_LENS}
    assert {(d["bx"], d["by"]) for d in c} == set(autotune.SHAPES)
    assert all((d["chunk_len"] == 0) != (d["target_groups"] == 0) for d in c)


def test_cache_round_trip(tmp_path, monkeypatch):
    monkeypatch.setattr(autotune, "arch", lambda device: "gfx950")
    path = str(tmp_path / "sub" / "tiles.json")
    spec = GridSpec(m=(64, 48, 40), h=(1.0, 1.0, 1.0), my=(17, 13, 11), tau=1.0, rho=1.0, alpha=0.1)
    other = GridSpec(m=(64, 48, 41), h=(1.0, 1.0, 1.0), my=(17, 13, 11), tau=1.0, rho=1.0, alpha=0.1)
    assert autotune.lookup(spec, "cuda:0", path) is None
    best = dict(bx=64, by=8, chunk_len=0, target_groups=4096)
    autotune._store(path, {autotune.cache_key("cuda:0", spec): {"config": best, "ms": 1.0, "timings": []}})
    assert autotune.lookup(spec, "cuda:0", path) == best
    assert autotune.lookup(other, "cuda:0", path) is None
    key = autotune.cache_key("cuda:0", spec)
    assert key.startswith("gfx950|tile_hv|m=64x48x40/my=17x13x11")
    with open(path) as f:
        assert key in json.load(f)


def test_corrupt_cache_reads_as_empty(tmp_path):
    p = tmp_path / "tiles.json"
    p.write_text("{not json")
    assert autotune._load(str(p)) == {}
