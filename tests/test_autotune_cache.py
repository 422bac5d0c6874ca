"""Host logic of the SpMV shape autotuner's JSON cache (paper_1807_09467_amd/autotune.py), on the CPU
with a stand-in for a sequence: the first sequence of a size is timed and its fastest shape stored,
later ones reuse the stored shape without timing, a corrupt cache is treated as empty, `retune`
times again, and no cache path keeps nothing."""
import json
import types

import pytest

from paper_1807_09467_amd import autotune

SHAPES = [  # as rsolve_tune_spmv returns them, fastest first
    {"format": "banded", "lanes_per_row": 4, "vec": 8, "xcd_remap": 0, "us": 75.8},
    {"format": "banded", "lanes_per_row": 2, "vec": 8, "xcd_remap": 0, "us": 85.0},
    {"format": "csr", "lanes_per_row": 8, "vec": 4, "xcd_remap": 0, "us": 120.0},
]


class FakeSeq:
    def __init__(self, n=1000, precision=1):
        self.device = "cuda:0"
        self.n = n
        self.cfg = types.SimpleNamespace(precision=precision)
        self.tuned = 0
        self.applied = []
        self.shape = {"format": "csr", "lanes_per_row": 8, "vec": 4, "xcd_remap": 0}

    def tune_spmv(self, row_ptr, col_idx, val, reps=20):
        self.tuned += 1
        return [dict(s) for s in SHAPES]

    def set_spmv_shape(self, lanes_per_row, vec, xcd_remap, fmt):
        self.applied.append((lanes_per_row, vec, xcd_remap, fmt))

    def spmv_shape(self):
        return dict(self.shape, us=0.0, user_set=False)


class FakeVal:
    def __init__(self, nnz):
        self._nnz = nnz

    def numel(self):
        return self._nnz


@pytest.fixture(autouse=True)
def device_name(monkeypatch):
    import torch
    monkeypatch.setattr(torch.cuda, "get_device_name", lambda dev=None: "MI355X")


def test_first_sequence_timed_then_cached(tmp_path):
    path = tmp_path / "shapes.json"
    a = FakeSeq()
    best, src, res = autotune.tune_sequence(a, None, None, FakeVal(5000), cache_path=str(path))
    assert src == "timed" and a.tuned == 1 and len(res) == len(SHAPES)
    assert a.applied == [(4, 8, 0, "banded")]
    assert best["default_us"] == 120.0            # the library's own choice, timed among the others
    table = json.loads(path.read_text())
    assert list(table) == ["MI355X|fp32|n=1000|nnz=5000"]
    b = FakeSeq()
    best_b, src_b, res_b = autotune.tune_sequence(b, None, None, FakeVal(5000), cache_path=str(path))
    assert src_b == "cache" and b.tuned == 0 and res_b == []
    assert b.applied == [(4, 8, 0, "banded")] and best_b["us"] == 75.8


def test_keys_separate_size_and_precision(tmp_path):
    path = str(tmp_path / "shapes.json")
    autotune.tune_sequence(FakeSeq(), None, None, FakeVal(5000), cache_path=path)
    for seq, nnz in ((FakeSeq(precision=0), 5000), (FakeSeq(n=2000), 5000), (FakeSeq(), 6000)):
        _, src, _ = autotune.tune_sequence(seq, None, None, FakeVal(nnz), cache_path=path)
        assert src == "timed"
    assert len(json.loads(open(path).read())) == 4


def test_corrupt_cache_is_ignored_and_rewritten(tmp_path):
    path = tmp_path / "shapes.json"
    path.write_text("{not json")
    seq = FakeSeq()
    _, src, _ = autotune.tune_sequence(seq, None, None, FakeVal(10), cache_path=str(path))
    assert src == "timed" and json.loads(path.read_text())


def test_retune_and_no_cache(tmp_path):
    path = str(tmp_path / "shapes.json")
    autotune.tune_sequence(FakeSeq(), None, None, FakeVal(7), cache_path=path)
    seq = FakeSeq()
    _, src, _ = autotune.tune_sequence(seq, None, None, FakeVal(7), cache_path=path, retune=True)
    assert src == "timed" and seq.tuned == 1
    seq2 = FakeSeq()
    _, src2, _ = autotune.tune_sequence(seq2, None, None, FakeVal(7), cache_path=None)
    assert src2 == "timed" and seq2.tuned == 1
    assert sorted(p.name for p in tmp_path.iterdir()) == ["shapes.json"]   # nothing else written
