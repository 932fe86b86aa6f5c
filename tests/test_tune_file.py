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
    # the persistent kind: 64-tiles, 4 workgroups per CU
    '{"version": 1, "entries": [\n  {"kernel": "gram", "precision": 0, "n_bucket": 10, "k_bucket": 15, "tile": 64, "workgroups": 8, "kind": 1}\n]}\n',
    '{"version": 1, "entries": [\n  {"kernel": "gram", "precision": 0, "n_bucket": 10, "k_bucket": 15, "tile": 128, "workgroups": 4, "kind": 1}\n]}\n',
    '{"version": 1, "entries": [\n  {"kernel": "gram", "precision": 0, "n_bucket": 10, "k_bucket": 15, "tile": 64, "workgroups": 512, "kind": 2}\n]}\n',
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


def test_kind_roundtrip(tmp_path):
    """Entries with and without the "kind" field (absent: split-K) load, and
    save writes the kind of every entry."""
    _lib()
    ils.tune_clear()
    src = tmp_path / "in.json"
    src.write_text('{"version": 1, "entries": [\n'
                   '  {"kernel": "gram", "precision": 0, "n_bucket": 10, "k_bucket": 15, "tile": 64, "workgroups": 4, "kind": 1},\n'
                   '  {"kernel": "gram", "precision": 0, "n_bucket": 10, "k_bucket": 11, "tile": 64, "workgroups": 8192}\n'
                   ']}\n')
    try:
        ils.tune_load(src)
        out = tmp_path / "out.json"
        ils.tune_save(out)
        got = sorted((e["k_bucket"], e["tile"], e["workgroups"], e["kind"]) for e in json.loads(out.read_text())["entries"])
        assert got == [(11, 64, 8192, ils.GRAM_SPLITK), (15, 64, 4, ils.GRAM_PERSISTENT)]
    finally:
        ils.tune_clear()


def test_batched_and_residual_entries_roundtrip(tmp_path):
    """Launch choices of the batched solver and of the residual share the
    file with the Gram entries."""
    _lib()
    ils.tune_clear()
    src = tmp_path / "in.json"
    src.write_text('{"version": 1, "entries": [\n'
                   '  {"kernel": "gram", "precision": 0, "n_bucket": 10, "k_bucket": 15, "tile": 64, "workgroups": 4, "kind": 1},\n'
                   '  {"kernel": "batched", "precision": 1, "form": 1, "n_bucket": 8, "k_bucket": 12, "tile": 16, "workgroups": 2, "kind": 1},\n'
                   '  {"kernel": "residual", "precision": 0, "form": 0, "n_bucket": 10, "k_bucket": 15, "tile": 16, "workgroups": 512, "kind": 0}\n'
                   ']}\n')
    try:
        ils.tune_load(src)
        out = tmp_path / "out.json"
        ils.tune_save(out)
        d = json.loads(out.read_text())["entries"]
        got = sorted((e["kernel"], e["tile"], e["workgroups"], e["kind"]) for e in d)
        assert got == [("batched", 16, 2, 1), ("gram", 64, 4, 1), ("residual", 16, 512, 0)]
        b = [e for e in d if e["kernel"] == "batched"][0]
        assert (b["precision"], b["form"], b["n_bucket"], b["k_bucket"]) == (1, 1, 8, 12)
        ils.tune_clear()
        ils.tune_save(out)
        assert json.loads(out.read_text())["entries"] == []
    finally:
        ils.tune_clear()


@pytest.mark.parametrize("line", [
    '{"kernel": "batched", "precision": 0, "form": 0, "n_bucket": 8, "k_bucket": 12, "tile": 48, "workgroups": 2, "kind": 0}',
    '{"kernel": "batched", "precision": 0, "form": 0, "n_bucket": 8, "k_bucket": 12, "tile": 32, "workgroups": 3, "kind": 0}',
    '{"kernel": "batched", "precision": 0, "form": 2, "n_bucket": 8, "k_bucket": 12, "tile": 32, "workgroups": 2, "kind": 0}',
    '{"kernel": "batched", "precision": 0, "n_bucket": 8, "k_bucket": 12, "tile": 32, "workgroups": 2, "kind": 0}',
    '{"kernel": "residual", "precision": 0, "form": 0, "n_bucket": 10, "k_bucket": 15, "tile": 16, "workgroups": 8, "kind": 0}',
    '{"kernel": "residual", "precision": 0, "form": 0, "n_bucket": 10, "k_bucket": 15, "tile": 16, "workgroups": 256, "kind": 3}',
    '{"kernel": "residual", "precision": 1, "form": 0, "n_bucket": 10, "k_bucket": 15, "tile": 16, "workgroups": 256, "kind": 0}',
])
def test_bad_batched_residual_entries(tmp_path, line):
    _lib()
    ils.tune_clear()
    f = tmp_path / "bad.json"
    f.write_text('{"version": 1, "entries": [\n  ' + line + '\n]}\n')
    with pytest.raises(ils.ILSError):
        ils.tune_load(f)


def test_missing_file(tmp_path):
    _lib()
    with pytest.raises(ils.ILSError):
        ils.tune_load(tmp_path / "nope.json")
