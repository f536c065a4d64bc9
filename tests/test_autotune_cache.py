"""The library's autotune cache on the host (no device calls): a file that
mg_autotune_cache_save writes is read back by mg_autotune_cache_load and
written again unchanged; malformed files and NULL paths are rejected and
merge nothing."""
import pytest

import paper_2207_09776_amd as mg

LINES = [
    "gfx950 128 128 0 2 0 0 0 2 1 0 1 8 128 0 2 16 8",
    "gfx950 256 256 0 3 0 0 0 2 1 1 2 12 256 1 1 0 0",
]


@pytest.fixture(scope="module")
def lib():
    return mg.load_library()


def test_cache_round_trip(lib, tmp_path):
    src = tmp_path / "in.txt"
    src.write_text("mg-autotune-cache 1\n" + "\n".join(LINES) + "\n")
    assert mg.autotune_cache_load(str(src)) == 2
    out = tmp_path / "out.txt"
    n = mg.autotune_cache_save(str(out))
    got = out.read_text().splitlines()
    assert got[0] == "mg-autotune-cache 1" and len(got) == n + 1
    for line in LINES:
        assert line in got
    # a second load of the saved file changes nothing
    assert mg.autotune_cache_load(str(out)) == n
    again = tmp_path / "again.txt"
    assert mg.autotune_cache_save(str(again)) == n
    assert again.read_text() == out.read_text()


def test_cache_rejects_malformed_files(lib, tmp_path):
    before = tmp_path / "before.txt"
    n = mg.autotune_cache_save(str(before))
    for text in ("not a cache\n" + LINES[0] + "\n",
                 "mg-autotune-cache 1\ngfx950 1 2 3\n",
                 "mg-autotune-cache 1\n" + LINES[0].replace(" 0 2 16 8", " 7 2 16 8") + "\n"):
        bad = tmp_path / "bad.txt"
        bad.write_text(text)
        with pytest.raises(mg.MagnusError) as ex:
            mg.autotune_cache_load(str(bad))
        assert ex.value.code == mg.MG_EINVAL
    after = tmp_path / "after.txt"
    assert mg.autotune_cache_save(str(after)) == n
    assert after.read_text() == before.read_text()
    with pytest.raises(mg.MagnusError):
        mg.autotune_cache_load(str(tmp_path / "missing.txt"))
