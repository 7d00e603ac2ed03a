"""Host-side logic of the autotuner: signatures and the JSON cache."""
import json

import paper_1807_03249_amd.autotune as at


class _S:
    def __init__(self, fmt, sw=512, sh=512):
        self.fmt, self.sw, self.sh = fmt, sw, sh


class _J:
    def __init__(self, w, h, fmt, p):
        self.w, self.h, self.style, self.params = w, h, _S(fmt), p


def test_signatures_are_order_insensitive_and_shape_sensitive():
    import paper_1807_03249_amd as sb

    p = sb.params(4, 8, 32, 3)
    q = sb.params(5, 8, 4096, 3)
    a = [_J(640, 480, 0, p), _J(1920, 1080, 1, q)]
    assert at.batch_signature(a) == at.batch_signature(a[::-1])
    assert at.batch_signature(a) != at.batch_signature([_J(640, 480, 0, p), _J(1920, 1080, 1, p)])
    assert at.frame_signature(_S(0), 1920, 1080, p) != at.frame_signature(_S(0), 1920, 1080, q)
    assert at.frame_signature(_S(0), 1920, 1080, p) != at.frame_signature(_S(1), 1920, 1080, p)


def test_cache_round_trip(tmp_path):
    path = str(tmp_path / "sub" / "tune.json")
    at._store(path, {"k": {"tune": [4, 16, 2], "ms": 0.05}})
    assert at._load(path) == {"k": {"tune": [4, 16, 2], "ms": 0.05}}
    with open(path, "w") as f:
        f.write("{not json")
    assert at._load(path) == {}
    assert at._load(str(tmp_path / "missing.json")) == {}
    assert at._tparse(at._tkey((2, 8, 4))) == [2, 8, 4]
    json.dumps(at._load(path))
