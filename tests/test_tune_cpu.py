"""Host-side logic of the launch-shape cache (no GPU): keys and the
fallback of a pool with aligned rebuilds to the plain key."""
import json
import types

from paper_0912_3824_amd import tune


class FakePool:
    def __init__(self, sizes, precision=1, rebuild_every=0):
        self.sizes = dict(enumerate(sizes))
        self.cfg = types.SimpleNamespace(precision=precision, rebuild_every=rebuild_every)
        self.applied = None

    def set_launch(self, **kw):
        self.applied = kw


def test_keys_name_precision_size_replicas_and_aligned_period():
    assert tune.key_of(FakePool([1_000_000])) == f"p1_b{tune.bucket(1_000_000)}_r1"
    assert tune.key_of(FakePool([2000] * 4, precision=3)) == f"p3_b{tune.bucket(8000)}_r4"
    assert tune.key_of(FakePool([2000] * 4, rebuild_every=16)).endswith("_r4_a16")


def test_aligned_pool_prefers_its_own_entry_and_falls_back(tmp_path):
    plain = FakePool([3000, 4000])
    aligned = FakePool([3000, 4000], rebuild_every=16)
    cache = tmp_path / "cache.json"
    cache.write_text(json.dumps({tune.key_of(plain): {"shape": {"build_block": 512}, "us_per_step": 1.0}}))
    assert tune.apply_cached(aligned, str(cache)) == {"build_block": 512}
    data = json.loads(cache.read_text())
    data[tune.key_of(aligned)] = {"shape": {"build_block": 320}, "us_per_step": 1.0}
    cache.write_text(json.dumps(data))
    assert tune.apply_cached(aligned, str(cache)) == {"build_block": 320}
    assert aligned.applied == {"build_block": 320}
    assert tune.apply_cached(plain, str(cache)) == {"build_block": 512}
    assert tune.apply_cached(FakePool([10]), str(cache)) is None


def test_aligned_pools_also_try_the_bulk_build():
    plain = tune.space_for(FakePool([3000, 4000]))
    aligned = tune.space_for(FakePool([3000, 4000], rebuild_every=16))
    assert "build_bulk" not in plain
    assert 0 in aligned["build_bulk"] and max(aligned["build_bulk"]) > 0
    assert {k: v for k, v in aligned.items() if k != "build_bulk"} == plain
