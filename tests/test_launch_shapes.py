"""Launch-shape cache (host only, no GPU): tile plans and population-
annealing groups saved by one context and loaded by another, the file
format's checks, and loading as all or nothing."""
import ctypes

import pytest

mcs = pytest.importorskip("paper_1709_04394_amd")


def _ctx():
    h = ctypes.c_void_p()
    assert mcs._lib.mc_ctx_create(ctypes.byref(h), 0) == 0
    return h


def _plan(h, g):
    H, K, T = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    assert mcs._lib.mc_get_tile_plan(h, ctypes.byref(g), ctypes.byref(H), ctypes.byref(K), ctypes.byref(T)) == 0
    return H.value, K.value, T.value


def _group(h, L):
    G = ctypes.c_int32()
    assert mcs._lib.mc_get_pa_group(h, L, ctypes.byref(G)) == 0
    return G.value


@pytest.fixture
def pair():
    a, b = _ctx(), _ctx()
    yield a, b
    mcs._lib.mc_ctx_destroy(a)
    mcs._lib.mc_ctx_destroy(b)


def test_round_trip(pair, tmp_path):
    a, b = pair
    g2, g3 = mcs.make_geom(2, 4096, count=3), mcs.make_geom(3, 256)
    assert mcs._lib.mc_set_tile_plan(a, ctypes.byref(g2), 16, 4, 512) == 0
    assert mcs._lib.mc_set_tile_plan(a, ctypes.byref(g3), 8, 4, 256) == 0
    assert mcs._lib.mc_set_pa_group(a, 32, 16) == 0
    assert mcs._lib.mc_set_pa_group(a, 128, 4) == 0
    path = str(tmp_path / "shapes.txt").encode()
    assert mcs._lib.mc_tuning_save(a, path) == 0
    text = open(path).read().splitlines()
    assert text[0] == "libmcspin-launch-shapes 1"
    assert "tile 2 4096 4096 1 3 16 4 512" in text and "pa 128 4" in text
    assert not (tmp_path / "shapes.txt.tmp").exists()
    before = _plan(b, g2)
    assert before != (16, 4, 512)
    assert mcs._lib.mc_tuning_load(b, path) == 0
    assert _plan(b, g2) == (16, 4, 512) and _plan(b, g3) == (8, 4, 256)
    assert _group(b, 32) == 16 and _group(b, 128) == 4 and _group(b, 64) == 4  # 64: built-in, not in the file


def test_comments_and_blank_lines(pair, tmp_path):
    _, b = pair
    p = tmp_path / "s.txt"
    p.write_text("# tuned on one device\n\nlibmcspin-launch-shapes 1   # version\n  pa 16 32  \n\n# end\n")
    assert mcs._lib.mc_tuning_load(b, str(p).encode()) == 0
    assert _group(b, 16) == 32


@pytest.mark.parametrize("body,code,where", [
    ("", mcs.MC_E_INVAL, b"no header"),
    ("pa 16 32\n", mcs.MC_E_INVAL, b":1:"),                                   # header missing
    ("libmcspin-launch-shapes 2\n", mcs.MC_E_INVAL, b":1:"),                  # other version
    ("libmcspin-launch-shapes 1\npa 16 32\nfoo 1 2\n", mcs.MC_E_INVAL, b":3:"),
    ("libmcspin-launch-shapes 1\npa 16 32 7\n", mcs.MC_E_INVAL, b":2:"),     # trailing field
    ("libmcspin-launch-shapes 1\npa 16 32\npa 16 0\n", mcs.MC_E_RANGE, b":3:"),
    ("libmcspin-launch-shapes 1\npa 16 32\npa 16 65\n", mcs.MC_E_RANGE, b":3:"),
    ("libmcspin-launch-shapes 1\npa 16 32\npa 12 1\n", mcs.MC_E_SHAPE, b":3:"),
    ("libmcspin-launch-shapes 1\npa 16 32\ntile 2 4096 4096 1 3 16 4 96\n", mcs.MC_E_RANGE, b":3:"),
    ("libmcspin-launch-shapes 1\npa 16 32\ntile 2 5 8 1 1 4 1 64\n", mcs.MC_E_SHAPE, b":3:"),
    ("libmcspin-launch-shapes 1\npa 16 32\n" + "#" * 300 + "\n", mcs.MC_E_INVAL, b"too long"),
    ("libmcspin-launch-shapes 1\npa 16 32\npa 99999999999 1\n", mcs.MC_E_INVAL, b":3:"),     # beyond int32
    ("libmcspin-launch-shapes 1\npa 16 32\npa 16 4x\n", mcs.MC_E_INVAL, b":3:"),
    ("libmcspin-launch-shapes 1\npa 16 32\npa16 4\n", mcs.MC_E_INVAL, b":3:"),
    ("libmcspin-launch-shapes 1\npa 16 32\ntile 2 64 64 1 1 16 2\n", mcs.MC_E_INVAL, b":3:"),  # 7 numbers
])
def test_rejected_files_change_nothing(pair, tmp_path, body, code, where):
    _, b = pair
    p = tmp_path / "bad.txt"
    p.write_text(body)
    assert mcs._lib.mc_tuning_load(b, str(p).encode()) == code
    assert where in mcs._lib.mc_ctx_last_error(b)
    assert _group(b, 16) == 16  # the valid "pa 16 32" before the bad line was not applied


def test_io_errors(pair, tmp_path):
    a, _ = pair
    assert mcs._lib.mc_tuning_load(a, str(tmp_path / "missing.txt").encode()) == mcs.MC_E_IO
    assert mcs._lib.mc_tuning_save(a, str(tmp_path / "no" / "such" / "dir.txt").encode()) == mcs.MC_E_IO
    assert mcs._lib.mc_tuning_save(a, b"") == mcs.MC_E_INVAL
    assert mcs._lib.mc_tuning_load(a, None) == mcs.MC_E_INVAL
    assert mcs._lib.mc_tuning_save(None, b"x") == mcs.MC_E_INVAL
    assert "file" in mcs.strerror(mcs.MC_E_IO)


def test_binding_methods(tmp_path):
    ctx = mcs.Context(0)  # host state only: no GPU needed
    ctx.set_pa_group(64, 8)
    ctx.save_launch_shapes(tmp_path / "s.txt")
    other = mcs.Context(0)
    other.load_launch_shapes(tmp_path / "s.txt")
    assert other.get_pa_group(64) == 8
    with pytest.raises(mcs.MCError):
        other.load_launch_shapes(tmp_path / "absent.txt")
