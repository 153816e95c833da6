"""Autotuner cache (host side): save / load / clear round trip and the
error path for a malformed cache file.  No GPU call."""
import pytest

import paper_2511_11890_amd as h


def test_tune_cache_round_trip(tmp_path):
    h.tune_clear()
    assert h.tune_entries() == 0
    src = tmp_path / "in.txt"
    src.write_text("harpia-tune 1\n00000000000000ab 0 0 4\n00000000000000cd 64 8 128\n")
    h.tune_load(src)
    assert h.tune_entries() == 2
    dst = tmp_path / "out.txt"
    h.tune_save(dst)
    lines = dst.read_text().split("\n")
    assert lines[0] == "harpia-tune 1"
    assert sorted(l for l in lines[1:] if l) == ["00000000000000ab 0 0 4", "00000000000000cd 64 8 128"]
    h.tune_clear()
    assert h.tune_entries() == 0
    h.tune_load(dst)
    assert h.tune_entries() == 2
    h.tune_clear()


@pytest.mark.parametrize("text", ["", "other 1\n", "harpia-tune 2\n", "harpia-tune 1\n12 1 2\n", "harpia-tune 1\nzz 1 2 3\n"])
def test_tune_cache_rejects_malformed(tmp_path, text):
    h.tune_clear()
    p = tmp_path / "bad.txt"
    p.write_text(text)
    with pytest.raises(h.HarpiaError):
        h.tune_load(p)
    assert h.tune_entries() == 0


def test_tune_cache_missing_file(tmp_path):
    with pytest.raises(h.HarpiaError):
        h.tune_load(tmp_path / "absent.txt")
