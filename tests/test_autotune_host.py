"""Host-side logic of the work-item autotuner (no GPU): cache keys and the JSON cache."""
import json

from paper_2111_14317_amd import autotune


class _FakeBatch:
    def __init__(self, ns, mmax):
        self.ns, self.mmax, self.num_sys = ns, mmax, len(ns)


def test_signature_depends_on_shape_precision_and_device():
    b = _FakeBatch([6, 10, 24], [8, 12, 64])
    idx = [0] * 100 + [1] * 250 + [2] * 40
    k = autotune.signature(b, idx, 1, "gpu-a")
    assert k == autotune.signature(b, idx, 1, "gpu-a")
    assert k != autotune.signature(b, idx, 0, "gpu-a")          # precision
    assert k != autotune.signature(b, idx, 1, "gpu-b")          # device
    assert k != autotune.signature(_FakeBatch([6, 10, 20], [8, 12, 64]), idx, 1, "gpu-a")  # n
    assert k != autotune.signature(b, [0] * 100 + [1] * 400 + [2] * 40, 1, "gpu-a")  # counts
    # path counts enter with two significant digits: a few paths more or less share the key
    assert k == autotune.signature(b, [0] * 101 + [1] * 250 + [2] * 40, 1, "gpu-a")


def test_cache_roundtrip(tmp_path):
    path = str(tmp_path / "sub" / "tiles.json")
    assert autotune._load(path) == {}
    autotune._store(path, {"k": {"tile": 4, "ms": {"4": 1.5}}})
    assert autotune._load(path) == {"k": {"tile": 4, "ms": {"4": 1.5}}}
    with open(path, "w") as f:
        f.write("{not json")
    assert autotune._load(path) == {}
    json.dumps(autotune.CANDIDATES)
