"""Host-side behaviour of the autotuner cache (no device needed)."""
import json

from paper_1908_01682_amd import autotune as A
from paper_1908_01682_amd import inputs as I


def test_signature_is_stable_and_discriminating():
    a = I.batched_waves(n_inst=8, n_min=500, n_max=900, seed=1)
    b = I.batched_waves(n_inst=8, n_min=500, n_max=900, seed=1)
    c = I.batched_waves(n_inst=9, n_min=500, n_max=900, seed=1)
    assert A.signature("gfx950", a, 0) == A.signature("gfx950", b, 0)
    assert A.signature("gfx950", a, 0) != A.signature("gfx950", c, 0)
    assert A.signature("gfx950", a, 0) != A.signature("gfx950", a, 1)
    assert A.signature("gfx950", a, 0) != A.signature("other", a, 0)


def test_cache_roundtrip(tmp_path, monkeypatch):
    path = tmp_path / "sub" / "cache.json"
    monkeypatch.setenv("TFSPH_AUTOTUNE_CACHE", str(path))
    assert A.load_cache() == {}
    A.store("k1", {"block": 512})
    A.store("k2", {"block": 1024})
    data = json.loads(path.read_text())
    assert data == {"k1": {"block": 512}, "k2": {"block": 1024}}
    path.write_text("not json")
    assert A.load_cache() == {}


class _FakeSim:
    """What plain_signature reads of a Simulation."""

    class _Ph:
        def __init__(self, n):
            self.n = n

    def __init__(self, prob, precision=0):
        self.prob = prob
        self.precision = precision
        self.gas, self.dust = self._Ph(prob.gas.n), self._Ph(prob.dust.n)


def test_plain_signature_is_stable_and_discriminating():
    a = _FakeSim(I.dusty_box(n_side=8, cells_per_axis=4, regions_per_axis=1))
    b = _FakeSim(I.dusty_box(n_side=8, cells_per_axis=4, regions_per_axis=1))
    c = _FakeSim(I.dusty_box(n_side=8, cells_per_axis=2, regions_per_axis=1))
    d = _FakeSim(I.dusty_box(n_side=10, cells_per_axis=4, regions_per_axis=1))
    assert A.plain_signature("gfx950", a) == A.plain_signature("gfx950", b)
    assert len({A.plain_signature("gfx950", s) for s in (a, c, d)}) == 3
    assert A.plain_signature("gfx950", a) != A.plain_signature("gfx950", _FakeSim(a.prob, 1))
    assert A.plain_signature("gfx950", a) != A.signature("gfx950", [a.prob], 0)
