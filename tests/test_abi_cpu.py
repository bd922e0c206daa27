"""The C ABI library loads and exports every declared symbol; host-side
argument validation answers without touching a GPU."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "swift.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(swift_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_1612_04787_amd import swift as S
    if not os.path.exists(S.LIB_PATH):
        pytest.fail("libswift.so is not built; run __graft_entry__.build()")
    return S.load_library()


def test_header_declares_the_boundary():
    fns = declared_functions()
    for f in ("swift_match_batch", "swift_project", "swift_snr", "swift_match_backward", "swift_pyramid",
              "swift_create", "swift_destroy", "swift_workspace_size", "swift_last_error"):
        assert f in fns


def test_library_exports_every_declared_symbol(lib):
    for f in declared_functions():
        assert hasattr(lib, f), f


def test_binding_declares_every_entry_point():
    from paper_1612_04787_amd import swift as S
    assert sorted(S.exported_symbols()) == declared_functions()


def test_binding_struct_layouts_match_header():
    from paper_1612_04787_amd import swift as S
    assert C.sizeof(S.Image) == 32
    assert C.sizeof(S.Params) == 32
    assert S.REC_BYTES == 64


def test_validation_without_gpu(lib):
    from paper_1612_04787_amd import swift as S
    pr = S.Pairs()
    pa = S.make_params()
    ws = C.c_size_t()
    assert lib.swift_workspace_size(None, C.byref(pr), C.byref(pa), C.byref(ws), None) == -1
    assert b"ctx" in lib.swift_last_error()
    assert lib.swift_plan(None, 512, 0, 0, -1, None, None, None) == -1
    assert lib.swift_autotune(None, None, 0, 0, None) == -1
    assert lib.swift_match_batch(None, None, 0, C.byref(pr), C.byref(pa), None, None, None, None, 0, None) == -1
    assert lib.swift_match_graph(None, None, 0, C.byref(pr), C.byref(pa), None, None, None, None, 0, None) == -1
    assert lib.swift_project(None, None, 1, 1, 1, 1, 1, None, 3, None, 1, 1, None) == -1
    assert lib.swift_snr(None, None, 64, 1, C.byref(pa), None, None) == -1
    assert lib.swift_pyramid(None, None, None, None) == -1
    assert lib.swift_centroid_jacobian(None, None, 0, C.byref(pr), C.byref(pa), None, None, None, 0, None) == -1
    assert lib.swift_refine_update(None, 1, None, None, None, 0, 0.5, None, None) == -1
    assert lib.swift_render(None, None, 1, 1, 1, 1, 1, None, 0, None, 1, 1, 1, 1, None) == -1
    assert lib.swift_stack_windows(None, 1, None, 0, 8, 64, 64, 0, 1, None, None, None, None, None) == -1
    assert lib.swift_fit_sections(None, 1, 64, None, None, None, 0, 6.0, None, None, None) == -1
    assert lib.swift_render_mesh(None, None, 1, 1, 1, 1, 1, None, 8, 0, None, 1, 1, 1, 1, None) == -1
    assert lib.swift_mesh_windows(None, 1, None, 0, 8, 64, 64, 0, 1, None, None, None, None, None) == -1
    assert lib.swift_fit_mesh(None, 1, 8, None, None, None, 0, 6.0, None, None, None, None) == -1
    assert lib.swift_project_side(None, None, 1, 1, 1, 1, 1, None, 3, -1, None, 1, 1, None) == -1
    assert lib.swift_blend_span(None, 4, 1, 2, None, None, None, None) == -1
    assert lib.swift_join_break(None, 4, 1, None, None, None, None) == -1
    assert lib.swift_search_keep(None, 4, 1, None, None, 0, 15.0, None, None, None, None) == -1
    assert lib.swift_search_next(None, 4, None, 0.0, 0.0, None, None, None, None, None, None, None, None, None, None,
                                 None) == -1
    assert b"ctx" in lib.swift_last_error()


def test_spiral_offsets_order():
    # host logic of the search driver: the origin, then each ring row-major
    from paper_1612_04787_amd.search import spiral_offsets
    o = spiral_offsets(10.0, 2).tolist()
    assert len(o) == 25 and o[0] == [0.0, 0.0]
    assert o[1:9] == [[-10, -10], [0, -10], [10, -10], [-10, 0], [10, 0], [-10, 10], [0, 10], [10, 10]]
    assert sorted(map(tuple, o)) == sorted((10.0 * i, 10.0 * j) for i in range(-2, 3) for j in range(-2, 3))
    assert all(max(abs(x), abs(y)) == 20 for x, y in o[9:])
