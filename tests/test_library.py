"""Host-side checks of the C ABI library (CPU only, no kernel launches)."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in sorted(os.listdir(os.path.join(ROOT, "include")))
           if h.endswith(".h")]
LIB = os.path.join(ROOT, "paper_2412_03451_amd", "libplanesplat.so")


def declared_functions():
    names = []
    for h in HEADERS:
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names += re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([a-z_][a-z0-9_]*)\s*\(", text,
                            flags=re.M)
    return sorted(set(names))


def test_header_declares_the_six_calls():
    names = declared_functions()
    for n in ("plane_project", "tile_bin", "plane_render_fwd", "plane_render_bwd", "loss_depth_normal",
              "adam_step_planes"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    names = declared_functions()
    assert len(names) >= 10
    for n in names:
        assert hasattr(lib, n), n


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_binding_covers_header():
    from paper_2412_03451_amd import _lib
    assert set(_lib.exported_names()) == set(declared_functions())


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_layout_and_argument_errors():
    from paper_2412_03451_amd import _lib
    lib = _lib.load()
    S = 2
    slots = (_lib.PsSlot * S)()
    for i in range(S):
        slots[i].plane_begin, slots[i].plane_end, slots[i].cam = 0, 10, i
        slots[i].width, slots[i].height, slots[i].tile_w, slots[i].tile_h = 100, 75, 16, 16
    L = _lib.PsLayout()
    assert lib.ps_layout_init(slots, S, 4096, ctypes.byref(L)) == 0
    assert L.n_records == 20 and L.n_tiles == 2 * 7 * 5 and L.n_items == 4 * L.n_tiles
    assert L.n_pixels == 2 * 7500 and slots[1].pix_off == 7500 and slots[1].rec_begin == 10
    assert lib.ps_workspace_bytes(ctypes.byref(L)) == L.ws_bytes > 0
    offs = [L.region[i] for i in range(_lib.PS_NUM_REGIONS)]
    assert offs == sorted(offs) and all(o % 256 == 0 for o in offs)
    slots[0].tile_w = 12
    assert lib.ps_layout_init(slots, S, 4096, ctypes.byref(L)) == _lib.PS_ERR_INVALID
    assert b"tile" in lib.ps_last_error()
    slots[0].tile_w = 16
    assert lib.ps_layout_init(slots, S, 0, ctypes.byref(L)) == _lib.PS_ERR_INVALID
    # null workspace is rejected before any launch
    prm = _lib.PsParams(30, 1e-4, 0.01, 0, 1, 0)
    assert lib.ps_layout_init(slots, S, 4096, ctypes.byref(L)) == 0
    rc = lib.plane_render_fwd(ctypes.byref(L), None, None, 1, None, ctypes.byref(prm), None, None, None, None,
                              None)
    assert rc == _lib.PS_ERR_INVALID
    rc = lib.adam_step_planes(None, None, None, None, None, None, None, None, 5, None, 1e-3, 1e-3, 1e-3,
                              0.9, 0.999, 1e-8, 1e-4, None)
    assert rc == _lib.PS_ERR_INVALID


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_valu_probe_argument_errors():
    """Rejected on the host before any launch: a kind other than 0 or 1, or
    a sink smaller than blocks * 256 values."""
    from paper_2412_03451_amd import _lib
    lib = _lib.load()
    dummy = ctypes.c_void_p(256)
    assert lib.ps_valu_probe(2, 1, 1, dummy, 1 << 20, None) == _lib.PS_ERR_INVALID
    assert lib.ps_valu_probe(0, 2, 1, dummy, 2 * 256 * 4 - 1, None) == _lib.PS_ERR_INVALID
    assert lib.ps_valu_probe(1, 1, 1, dummy, 256 * 8 - 1, None) == _lib.PS_ERR_INVALID
    assert lib.ps_valu_probe(0, 1, 0, dummy, 1 << 20, None) == _lib.PS_ERR_INVALID


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_check_finite_argument_errors():
    """Rejected on the host before any launch."""
    from paper_2412_03451_amd import _lib
    lib = _lib.load()
    dummy = ctypes.c_void_p(256)
    assert lib.ps_check_finite(dummy, -1, dummy, None, None) == _lib.PS_ERR_INVALID
    assert lib.ps_check_finite(dummy, 10, None, None, None) == _lib.PS_ERR_INVALID
    assert lib.ps_check_finite(None, 10, dummy, None, None) == _lib.PS_ERR_INVALID


def test_every_hot_path_call_cites_the_paper():
    """The comment in front of each of the six calls of the splatting path
    names the passage it follows (a Sec. or an Eq. of the paper)."""
    text = open(os.path.join(ROOT, "include", "planesplat.h")).read()
    for n in ("plane_project", "tile_bin", "plane_render_fwd", "plane_render_bwd", "loss_depth_normal",
              "adam_step_planes"):
        m = re.search(r"/\*((?:(?!\*/).)*?)\*/\s*int\s+" + n + r"\s*\(", text, flags=re.S)
        assert m, n
        assert re.search(r"\b(Sec\.|Eq\.)\s*\d", m.group(1)), n


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_noalloc_rejects_sizes_beyond_its_scratch():
    """plane_render_fwd_noalloc checks its fixed regions against the static
    scratch before touching the device (no launch, no device query)."""
    from paper_2412_03451_amd import _lib
    lib = _lib.load()
    dummy = ctypes.c_void_p(256)
    prm = _lib.PsParams(30, 1e-4, 0.01, 0, 1, 0)
    rc = lib.plane_render_fwd_noalloc(dummy, dummy, dummy, 200000, dummy, 640, 480, 16, 16, dummy,
                                      ctypes.byref(prm), dummy, dummy, None, None)
    assert rc == _lib.PS_ERR_INVALID and b"static" in lib.ps_last_error()
    rc = lib.plane_render_fwd_noalloc(dummy, dummy, dummy, 10, dummy, 640, 480, 12, 16, dummy,
                                      ctypes.byref(prm), dummy, dummy, None, None)
    assert rc == _lib.PS_ERR_INVALID
