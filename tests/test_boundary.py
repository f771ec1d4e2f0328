"""C-ABI boundary checks that need no GPU: the library loads, exports every
entry point the header declares, and validates footprints on the host."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", f) for f in os.listdir(os.path.join(ROOT, "include"))
           if f.endswith(".h")]


def _lib():
    import paper_2605_29663_amd as pkg
    if not os.path.exists(pkg.LIB_PATH):
        from paper_2605_29663_amd import build
        build.build()
    return pkg, pkg.load()


def _declared():
    names = []
    for h in HEADERS:
        txt = open(h).read()
        names += re.findall(r"MPPI_API\s+[\w\s\*]+?\b(\w+)\s*\(", txt)
    return names


def test_header_declares_entry_points():
    names = _declared()
    for n in ("mppi_create", "mppi_destroy", "mppi_last_error", "set_footprint", "set_points",
              "sdf_polygon", "sdf_rectcover", "sdf_min_poses", "mppi_step", "mppi_rollout",
              "mppi_check_footprint"):
        assert n in names


def _declared_returns():
    """(return type text, name) of every declaration."""
    out = []
    for h in HEADERS:
        txt = open(h).read()
        out += re.findall(r"MPPI_API\s+([\w\s\*]+?)\s*\b(\w+)\s*\(", txt)
    return [(" ".join(r.split()), n) for r, n in out]


def test_binding_return_types_match_header():
    """A pointer returned through a 32-bit int would be truncated: the ctypes
    return type of every binding must match the header's."""
    pkg, L = _lib()
    want = {"int": ctypes.c_int, "const char*": ctypes.c_char_p, "const char *": ctypes.c_char_p,
            "long long": ctypes.c_longlong, "mppi_batch": ctypes.c_void_p}
    for ret, name in _declared_returns():
        if name not in pkg.EXPORTS:
            continue
        assert ret in want, (ret, name)
        assert getattr(L, name).restype is want[ret], (name, ret, getattr(L, name).restype)
    assert set(pkg.EXPORTS) == set(n for _, n in _declared_returns())


def test_library_exports_every_declared_symbol():
    pkg, L = _lib()
    for n in _declared():
        assert hasattr(L, n), n
    assert set(pkg.EXPORTS) <= set(_declared())


def test_params_struct_layout_matches_header():
    """The ctypes mirror of mppi_params has the C layout: 5 ints, 3 floats,
    3x3 float arrays, 5 floats, 3 floats, 2 floats, 2 ints, 1 float."""
    import paper_2605_29663_amd as pkg
    assert ctypes.sizeof(pkg.MppiParams) == 4 * (5 + 3 + 9 + 5 + 3 + 2 + 2 + 1)
    assert pkg.MppiParams.w_path.offset == 4 * (5 + 3 + 9 + 5 + 3 + 2 + 2)
    assert pkg.MppiParams.goal.offset == 4 * (5 + 3 + 9 + 5 + 3)
    assert ctypes.sizeof(pkg.MppiDiag) == 10 * 8
    # mppi_hybrid_params: float, int32, 4 floats
    assert ctypes.sizeof(pkg.HybridParams) == 6 * 4
    assert pkg.HybridParams.v_min.offset == 8


@pytest.mark.parametrize("poly,code", [
    ([(0, 0), (1, 0), (1, 1), (0, 1)], 0),
    ([(0, 0), (1, 0), (0.5, 0.0), (0.5, 1)], -2),           # fold-back onto an edge
    ([(0, 0), (1, 1), (1, 0), (0, 1)], -2),                 # bow tie (self-crossing)
    ([(0, 0), (1, 0), (1, 0), (0, 1)], -2),                 # zero-length edge
    ([(0, 0), (1, 0), (2, 0)], -2),                         # zero area
    ([(0, 0), (1, 0), (np.nan, 1)], -2),                    # non-finite
    ([(0, 0), (1, 0)], -4),                                 # too few vertices
    ([(0, 0), (2, 0), (2, 2), (1, 0.0), (0, 2)], -2),       # vertex touching an edge
    ([(0, 0), (2, 0), (2, 1), (1, 1), (1, 2), (0, 2)], 0),  # concave L
    ([(0, 0), (1, 0), (2, 0), (2, 1), (0, 1)], 0),          # collinear vertex allowed
])
def test_check_polygon(poly, code):
    pkg, _ = _lib()
    rc, msg = pkg.check_footprint(pkg.POLYGON, poly)
    assert rc == code, msg
    if code:
        assert msg


def test_check_polygon_capacity_and_scene_shapes():
    pkg, _ = _lib()
    from paper_2605_29663_amd import scenes
    a = np.linspace(0, 2 * np.pi, 66)[:-1]                  # 65 vertices: above the capacity
    assert pkg.check_footprint(pkg.POLYGON, np.stack([np.cos(a), np.sin(a)], 1))[0] == -4
    a = np.linspace(0, 2 * np.pi, 65)[:-1]                  # 64 vertices: the capacity
    assert pkg.check_footprint(pkg.POLYGON, np.stack([np.cos(a), np.sin(a)], 1))[0] == 0
    for V in [scenes.FOOTPRINT_L8, scenes.FOOTPRINT_TOWED16, scenes.RECTS_4_BOUNDARY,
              scenes.FOOTPRINT_GAP_L] + [scenes.SHAPES_LTF[k][0] for k in "LTF"]:
        assert pkg.check_footprint(pkg.POLYGON, V)[0] == 0
    rng = np.random.default_rng(0)
    for B in range(3, 65):
        assert pkg.check_footprint(pkg.POLYGON, scenes.star_polygon(rng, B))[0] == 0


@pytest.mark.parametrize("rects,code", [
    ([(0, 0, 1, 1)], 0),
    ([(0, 0, 1, 0)], -2),
    ([(0, 0, -1, 1)], -2),
    ([(0, np.inf, 1, 1)], -2),
    (np.zeros((0, 4)), -4),
    (np.tile([0.0, 0.0, 1.0, 1.0], (33, 1)), -4),
])
def test_check_rects(rects, code):
    pkg, _ = _lib()
    assert pkg.check_footprint(pkg.RECTS, rects)[0] == code


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    import paper_2605_29663_amd as pkg
    monkeypatch.setattr(pkg, "_lib", None)
    monkeypatch.setattr(pkg, "LIB_PATH", str(tmp_path / "nope.so"))
    with pytest.raises(RuntimeError, match="no CPU fallback"):
        pkg.load()
