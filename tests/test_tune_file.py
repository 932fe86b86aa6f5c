"""The autotuner's table file (ils_tune_save / ils_tune_load): JSON that
round-trips, and malformed files rejected.  Host-only: no GPU needed."""
import json

import pytest

import paper_2203_15340_amd as ils


def _lib():
    try:
        return ils.load_library()
    except ils.ILSError:
        pytest.skip("libils.so not built")


def test_roundtrip(tmp_path):
    _lib()
    ils.tune_clear()
    src = tmp_path / "in.json"
    src.write_text('{"version": 1, "entries": [\n'
                   '  {"kernel": "gram", "precision": 0, "n_bucket": 10, "k_bucket": 15, "tile": 128, "workgroups": 1024},\n'
                   '  {"kernel": "gram", "precision": 1, "n_bucket": 7, "k_bucket": 12, "tile": 64, "workgroups": 256}\n'
                   ']}\n')
    ils.tune_load(src)
    out = tmp_path / "out.json"
    ils.tune_save(out)
    d = json.loads(out.read_text())
    got = sorted((e["precision"], e["n_bucket"], e["k_bucket"], e["tile"], e["workgroups"]) for e in d["entries"])
    assert got == [(0, 10, 15, 128, 1024), (1, 7, 12, 64, 256)]
    ils.tune_clear()
    ils.tune_save(out)
    assert json.loads(out.read_text())["entries"] == []


@pytest.mark.parametrize("text", [
    '{"version": 2, "entries": []}\n',
    '{"version": 1, "entries": [\n  {"kernel": "gram", "precision": 0, "n_bucket": 10, "k_bucket": 15, "tile": 96, "workgroups": 512}\n]}\n',
    '{"version": 1, "entries": [\n  {"kernel": "gram", "precision": 5, "n_bucket": 10, "k_bucket": 15, "tile": 64, "workgroups": 512}\n]}\n',
    '{"version": 1, "entries": [\n  {"kernel": "gram", "precision": 0}\n]}\n',
])
def test_malformed_rejected(tmp_path, text):
    _lib()
    ils.tune_clear()
    f = tmp_path / "bad.json"
    f.write_text(text)
    with pytest.raises(ils.ILSError):
        ils.tune_load(f)
    out = tmp_path / "out.json"
    ils.tune_save(out)
    assert json.loads(out.read_text())["entries"] == []


def test_missing_file(tmp_path):
    _lib()
    with pytest.raises(ils.ILSError):
        ils.tune_load(tmp_path / "nope.json")
