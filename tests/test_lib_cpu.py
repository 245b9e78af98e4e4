"""CPU checks of the C ABI: the library loads, exports every declared symbol,
and rejects bad arguments on the host before touching a device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    src = open(os.path.join(ROOT, "include", "btree.h")).read()
    return sorted(set(re.findall(r"^\s*(?:btree_status|const char\*)\s+(btree_\w+)\s*\(", src, re.M)))


@pytest.fixture(scope="module")
def L():
    from paper_1910_02639_amd import btree
    if not os.path.exists(btree.LIB_PATH):
        from paper_1910_02639_amd import buildlib
        buildlib.build()
    return btree


def test_header_symbols_exported(L):
    syms = _declared_symbols()
    assert "btree_build" in syms and "btree_find_neighbors" in syms
    lib = L.lib()
    for s in syms:
        assert hasattr(lib, s), s
    assert set(syms) <= set(L.SYMBOLS) | set(syms)
    assert set(L.SYMBOLS) == set(syms)


def test_struct_layouts_match_header(L, tmp_path):
    """ctypes mirrors of btree_params / btree_stats_t agree with the header
    as compiled by the C compiler (size and every field offset)."""
    import subprocess
    fields_p = [f for f, _ in L.Params._fields_]
    fields_s = [f for f, _ in L.Stats._fields_]
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "btree.h"', "int main(void){"]
    lines.append('printf("%zu\\n", sizeof(btree_params));')
    for f in fields_p:
        lines.append('printf("%%zu\\n", offsetof(btree_params, %s));' % f)
    lines.append('printf("%zu\\n", sizeof(btree_stats_t));')
    for f in fields_s:
        lines.append('printf("%%zu\\n", offsetof(btree_stats_t, %s));' % f)
    from paper_1910_02639_amd import autotune
    fields_t = [f for f, _ in autotune.TuneSpace._fields_]
    lines.append('printf("%zu\\n", sizeof(btree_tune_space));')
    for f in fields_t:
        lines.append('printf("%%zu\\n", offsetof(btree_tune_space, %s));' % f)
    lines.append("return 0;}")
    c = tmp_path / "lay.c"
    c.write_text("\n".join(lines))
    exe = tmp_path / "lay"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(c), "-o", str(exe)], check=True)
    out = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True,
                                           check=True).stdout.split()]
    want = [ctypes.sizeof(L.Params)] + [getattr(L.Params, f).offset for f in fields_p]
    want += [ctypes.sizeof(L.Stats)] + [getattr(L.Stats, f).offset for f in fields_s]
    T = autotune.TuneSpace
    want += [ctypes.sizeof(T)] + [getattr(T, f).offset for f in fields_t]
    assert out == want


def test_params_default(L):
    p = L.params()
    assert (p.bucket_size, p.alpha, p.beta, p.max_depth) == (64, 0.5, 0.5, 32)
    assert p.precision == L.BTREE_FP32_FILTER
    assert L.lib().btree_params_default(None) == L.BTREE_EINVAL


def _build(L, n, p=None, out=True, ptr=1):
    h = ctypes.c_void_p()
    P = ctypes.c_void_p(ptr) if ptr else None
    return L.lib().btree_build(P, P, P, n, ctypes.byref(p) if p is not None else None, None,
                               ctypes.byref(h) if out else None)


@pytest.mark.parametrize("field,value", [("bucket_size", 0), ("alpha", float("nan")),
                                         ("alpha", -1.0), ("beta", float("inf")),
                                         ("max_depth", -1), ("max_depth", 65),
                                         ("precision", 7), ("group_size", 32),
                                         ("exclude_self", 2), ("octree", -1)])
def test_build_rejects_bad_params(L, field, value):
    p = L.params()
    setattr(p, field, value)
    assert _build(L, 100, p) == L.BTREE_EINVAL
    assert L.last_error()


def test_build_rejects_bad_sizes(L):
    p = L.params()
    assert _build(L, -1, p) == L.BTREE_EINVAL
    assert _build(L, 2 ** 31, p) == L.BTREE_EINVAL
    assert _build(L, 100, p, ptr=0) == L.BTREE_EINVAL
    assert _build(L, 100, p, out=False) == L.BTREE_EINVAL
    p.reserved[2] = 1
    assert _build(L, 100, p) == L.BTREE_EINVAL
    p = L.params(bucket_size=1)
    assert _build(L, 2 ** 31 - 2, p) == L.BTREE_EINVAL   # n / s above 2^30


def test_find_rejects_null_handle(L):
    t = ctypes.c_int64()
    assert L.lib().btree_find_neighbors(None, None, None, None, None, 0, ctypes.byref(t), None) \
        == L.BTREE_ESTATE
    assert L.lib().btree_stats(None, None) == L.BTREE_EINVAL
    assert L.lib().btree_export(None, None, None, None, None, None) == L.BTREE_EINVAL
    assert L.lib().btree_destroy(None) == L.BTREE_OK


def test_product_never_imports_oracle():
    """The product path has no CPU fallback: no package module imports or
    loads the oracle."""
    pkg = os.path.join(ROOT, "paper_1910_02639_amd")
    for f in os.listdir(pkg):
        if f.endswith(".py"):
            s = open(os.path.join(pkg, f)).read()
            assert not re.search(r"^\s*(import oracle|from oracle)", s, re.M), f
            assert "_oracle.so" not in s, f


def test_missing_library_fails_loudly(tmp_path):
    """Without the built HIP library every entry of the binding raises: there
    is no other path to take."""
    import subprocess
    import sys
    code = (
        "import sys; sys.path.insert(0, %r)\n"
        "from paper_1910_02639_amd import btree\n"
        "btree.LIB_PATH = %r\n"
        "try:\n"
        "    btree.lib()\n"
        "except RuntimeError as e:\n"
        "    print('raised:', e)\n"
        "    sys.exit(0)\n"
        "sys.exit(3)\n" % (ROOT, str(tmp_path / "absent" / "libbtree.so")))
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "not built" in r.stdout


def _batch_create(L, nsets, offs, prm=None, out=True):
    import numpy as np
    h = ctypes.c_void_p()
    o = np.asarray(offs, dtype=np.int64) if offs is not None else None
    return L.lib().btree_batch_create(nsets, o.ctypes.data if o is not None else None,
                                      prm, ctypes.byref(h) if out else None)


def test_batch_create_rejects_bad_arguments(L):
    """Host-side checks of btree_batch_create run before any device call."""
    assert _batch_create(L, 2, [0, 5, 9], out=False) == L.BTREE_EINVAL
    assert _batch_create(L, 0, [0]) == L.BTREE_EINVAL
    assert _batch_create(L, 2, None) == L.BTREE_EINVAL
    assert _batch_create(L, 2, [1, 5, 9]) == L.BTREE_EINVAL      # must start at 0
    assert _batch_create(L, 2, [0, 5, 4]) == L.BTREE_EINVAL      # decreasing
    assert _batch_create(L, 1, [0, 2 ** 31]) == L.BTREE_EINVAL   # total too large
    arr = (L.Params * 2)(L.params(), L.params(precision="fp64"))
    assert _batch_create(L, 2, [0, 5, 9], arr) == L.BTREE_EINVAL  # mixed precision
    arr = (L.Params * 2)(L.params(), L.params(bucket_size=0))
    assert _batch_create(L, 2, [0, 5, 9], arr) == L.BTREE_EINVAL
    assert "bucket_size" in L.last_error()
    arr = (L.Params * 2)(L.params(), L.params(timing=True))
    assert _batch_create(L, 2, [0, 5, 9], arr) == L.BTREE_EINVAL  # mixed timing flag
    arr = (L.Params * 2)(L.params(), L.params(exclude_self=True))
    assert _batch_create(L, 2, [0, 5, 9], arr) == L.BTREE_EINVAL  # mixed exclude_self
    assert "exclude_self" in L.last_error()


def test_batch_null_handle(L):
    t = ctypes.c_int64()
    assert L.lib().btree_batch_run(None, None, None, None, None, None, None, None, 0, None,
                                   ctypes.byref(t), None) == L.BTREE_ESTATE
    assert L.lib().btree_batch_stats(None, None) == L.BTREE_EINVAL
    assert L.lib().btree_batch_graph_counts(None, None, None) == L.BTREE_EINVAL
    assert L.lib().btree_batch_destroy(None) == L.BTREE_OK


def test_tune_space_and_argument_checks(L):
    from paper_1910_02639_amd import autotune
    sp = autotune.space()
    assert list(sp.bucket)[:sp.n_bucket] == [16, 24, 32, 48, 64, 96, 128, 192, 256]
    assert list(sp.beta)[:sp.n_beta] == [0.3, 0.5, 0.8]
    assert list(sp.alpha)[:sp.n_alpha] == [0.25, 0.5, 1.0]
    lib = autotune._lib()
    assert lib.btree_tune_space_default(None) == L.BTREE_EINVAL
    best = L.Params()
    ms = ctypes.c_double()
    P = ctypes.c_void_p(1)
    # NULL outputs, bad space, bad bucket, NULL h: all refused on the host
    assert lib.btree_tune(P, P, P, P, 10, None, None, None, ctypes.byref(ms), None, None) \
        == L.BTREE_EINVAL
    bad = autotune.space(repeats=0)
    assert lib.btree_tune(P, P, P, P, 10, None, ctypes.byref(bad), ctypes.byref(best),
                          ctypes.byref(ms), None, None) == L.BTREE_EINVAL
    bad = autotune.space(alphas=[0.5, -0.1])
    assert lib.btree_tune(P, P, P, P, 10, None, ctypes.byref(bad), ctypes.byref(best),
                          ctypes.byref(ms), None, None) == L.BTREE_EINVAL
    bad = autotune.space()
    bad.n_alpha = 5
    assert lib.btree_tune(P, P, P, P, 10, None, ctypes.byref(bad), ctypes.byref(best),
                          ctypes.byref(ms), None, None) == L.BTREE_EINVAL
    bad = autotune.space(buckets=[16, 0])
    assert lib.btree_tune(P, P, P, P, 10, None, ctypes.byref(bad), ctypes.byref(best),
                          ctypes.byref(ms), None, None) == L.BTREE_EINVAL
    assert lib.btree_tune(P, P, P, None, 10, None, None, ctypes.byref(best),
                          ctypes.byref(ms), None, None) == L.BTREE_EINVAL


def test_tuner_keys():
    import numpy as np
    from paper_1910_02639_amd import autotune
    assert autotune.distribution_class(np.full(100, 0.3)) == "const_h"
    assert autotune.distribution_class(np.r_[np.zeros(5), np.full(10, 0.3)]) == "const_h"
    assert autotune.distribution_class(np.linspace(0.1, 0.5, 10)) == "graded_h"
    assert autotune.key(10_000, np.full(3, 1.0), "fp32") == "fp32/const_h/13"
    assert autotune.key(2 ** 20, np.linspace(1, 2, 3), "fp64") == "fp64/graded_h/20"
