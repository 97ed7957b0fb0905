"""CPU checks of the C-ABI library: it loads without a GPU and exports every
function include/knn.h declares; the Python binding has the same names."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "knn.h")
LIB = os.path.join(ROOT, "paper_1607_08220_amd", "libknn.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\*?\s+\*?(knn_\w+)\s*\(", src, flags=re.M)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("knn_build", "knn_query", "knn_build_ex", "knn_query_ex", "knn_tree_free",
                     "knn_tree_info", "knn_tree_export", "knn_last_error"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libknn.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libknn.so not built")
def test_binding_names_match_header():
    import paper_1607_08220_amd as knn
    for n in declared_functions():
        assert hasattr(knn, n), n
    assert set(knn.EXPORTED) == set(declared_functions())


@pytest.mark.skipif(not os.path.exists(LIB), reason="libknn.so not built")
def test_argument_errors_need_no_device():
    """Validation is host logic: bad arguments are rejected before any HIP call."""
    import paper_1607_08220_amd as knn
    lib = knn.load_library()
    out = ctypes.c_void_p()
    assert lib.knn_build(None, 10, 3, 32, None, ctypes.byref(out)) == knn.KNN_EINVAL
    assert lib.knn_build(ctypes.c_void_p(16), 0, 3, 32, None, ctypes.byref(out)) == knn.KNN_EINVAL
    assert lib.knn_build(ctypes.c_void_p(16), 10, 17, 32, None, ctypes.byref(out)) == knn.KNN_EINVAL
    assert lib.knn_build(ctypes.c_void_p(16), 10, 0, 32, None, ctypes.byref(out)) == knn.KNN_EINVAL
    assert lib.knn_build(ctypes.c_void_p(16), 10, 3, -1, None, ctypes.byref(out)) == knn.KNN_EINVAL
    assert lib.knn_build(ctypes.c_void_p(16), (1 << 30) + 1, 3, 32, None,
                         ctypes.byref(out)) == knn.KNN_EINVAL
    assert "n must be" in knn.knn_last_error()
    assert lib.knn_query(None, None, 1, 5, None, None, None) == knn.KNN_EINVAL
    assert lib.knn_tree_free(None) == knn.KNN_OK
    assert lib.knn_tree_info(None, None) == knn.KNN_EINVAL


@pytest.mark.skipif(not os.path.exists(LIB), reason="libknn.so not built")
def test_strerror_and_tree_errors_without_device():
    import paper_1607_08220_amd as knn
    lib = knn.load_library()
    names = {c: knn.knn_strerror(c) for c in (0, -1, -2, -3, -4, -5)}
    assert names == {0: "KNN_OK", -1: "KNN_EINVAL", -2: "KNN_ENOMEM", -3: "KNN_EDEVICE",
                     -4: "KNN_EDEPTH", -5: "KNN_ENOTFINITE"}
    assert knn.knn_strerror(7) == "unknown"
    assert lib.knn_tree_errors(None, None, None) == knn.KNN_EINVAL


@pytest.mark.skipif(not os.path.exists(LIB), reason="libknn.so not built")
def test_build_plan_argument_errors_need_no_device():
    import paper_1607_08220_amd as knn
    lib = knn.load_library()
    out = ctypes.c_void_p()
    I64 = ctypes.c_int64 * 3
    assert lib.knn_build_plan_create(0, 3, None, 1, None, None, ctypes.byref(out)) == knn.KNN_EINVAL
    assert lib.knn_build_plan_create(10, 17, None, 1, None, None, ctypes.byref(out)) == knn.KNN_EINVAL
    assert lib.knn_build_plan_create(10, 3, None, 2, None, None, ctypes.byref(out)) == knn.KNN_EINVAL
    bad_end = I64(0, 4, 9)  # offsets[trees] != n
    assert lib.knn_build_plan_create(10, 3, bad_end, 2, None, None,
                                     ctypes.byref(out)) == knn.KNN_EINVAL
    empty_tree = I64(0, 4, 4)
    assert lib.knn_build_plan_create(4, 3, empty_tree, 2, None, None,
                                     ctypes.byref(out)) == knn.KNN_EINVAL
    assert lib.knn_build_plan_create(10, 3, None, 1, None, None, None) == knn.KNN_EINVAL
    assert not out.value
    assert lib.knn_build_plan_run(None, ctypes.c_void_p(16), None) == knn.KNN_EINVAL
    assert lib.knn_build_plan_finish(None, None, None) == knn.KNN_EINVAL
    assert lib.knn_build_plan_tree(None) is None
    assert lib.knn_build_plan_destroy(None) == knn.KNN_OK
