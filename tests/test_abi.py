"""C-ABI checks that need no GPU: the library loads, exports every declared entry
point, and host-side argument errors are reported before any device work."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    with open(os.path.join(ROOT, "include", "ttsparse.h")) as f:
        txt = f.read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(tt_[a-z0-9_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    from paper_1908_02721_amd import _lib

    return _lib.load()


def test_exports_every_declared_symbol(lib):
    names = _declared()
    assert "tt_sparse_decompose" in names and "tt_eval_entries_backward" in names
    for n in names:
        assert hasattr(lib, n), n
    from paper_1908_02721_amd import _lib

    assert sorted(_lib.EXPORTS) == names


def _call(lib, d, dims, nnz, idx, val, eps, opt=None):
    from paper_1908_02721_amd import _lib

    o = _lib.tt_options()
    lib.tt_options_default(ctypes.byref(o))
    if opt:
        for k, v in opt.items():
            setattr(o, k, v)
    dims_a = (ctypes.c_int64 * max(1, len(dims)))(*dims)
    h = ctypes.c_void_p(123)
    st = lib.tt_sparse_decompose(d, dims_a, nnz, idx, val, eps, ctypes.byref(o), None, ctypes.byref(h))
    return st, h.value


def test_host_argument_errors(lib):
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: every call below fails on the host
    cases = [
        ((1, [4], 1, fake, fake, 0.1), 1),              # d < 2
        ((65, [2] * 65, 1, fake, fake, 0.1), 1),        # d > 64
        ((2, [4, 0], 1, fake, fake, 0.1), 1),           # n_k < 1
        ((2, [4, 4], 1, None, fake, 0.1), 1),           # idx NULL
        ((2, [4, 4], 1, fake, None, 0.1), 1),           # val NULL
        ((2, [4, 4], 1, fake, fake, 1.0), 1),           # eps >= 1
        ((2, [4, 4], 1, fake, fake, -0.1), 1),          # eps < 0
        ((2, [4, 4], 1, fake, fake, float("nan")), 1),  # eps NaN
        ((2, [4, 4], -1, fake, fake, 0.1), 1),          # nnz < 0
        ((2, [4, 4], 0, fake, fake, 0.1), 5),           # nothing given -> EMPTY
        ((8, [1 << 30] * 8, 1, fake, fake, 0.1), 6),    # packed key > 63 bits
    ]
    for args, expect in cases:
        st, h = _call(lib, *args)
        assert st == expect, (args, st)
        assert h is None
        assert len(lib.tt_last_error()) > 0
    st, _ = _call(lib, 2, [4, 4], 1, fake, fake, 0.1, {"precision": 7})
    assert st == 1
    st, _ = _call(lib, 2, [4, 4], 1, fake, fake, 0.1, {"max_rank": -2})
    assert st == 1
    for kb in (-1, 53):
        st, _ = _call(lib, 2, [4, 4], 1, fake, fake, 0.1, {"key_bits": kb})
        assert st == 1


def test_status_strings(lib):
    from paper_1908_02721_amd import _lib

    for code, name in _lib.STATUS.items():
        assert lib.tt_status_string(code).decode() == name


def test_null_handles(lib):
    lib.tt_free(None)
    r = (ctypes.c_int64 * 4)()
    assert lib.tt_get_ranks(None, r) == 1
    assert lib.tt_get_core(None, 1, ctypes.byref(ctypes.c_void_p()), None) == 1
    assert lib.tt_get_bond_delta(None, 1, ctypes.byref(ctypes.c_double())) == 1


def test_matrix_to_tensor_host_argument_errors(lib):
    fake = ctypes.c_void_p(0x1000)  # never dereferenced

    def call(d, m, n, nnz=4, rows=fake, cols=fake, idx=fake):
        ma = (ctypes.c_int64 * max(1, len(m)))(*m)
        na = (ctypes.c_int64 * max(1, len(n)))(*n)
        return lib.tt_matrix_to_tensor(d, ma, na, nnz, rows, cols, idx, None)

    assert call(0, [2], [2]) == 1                      # d < 1
    assert call(65, [2] * 65, [2] * 65) == 1           # d > 64
    assert call(2, [2, 0], [2, 2]) == 1                # m_k < 1
    assert call(2, [2, 2], [2, -1]) == 1               # n_k < 1
    assert call(2, [1 << 16, 2], [1 << 15, 2]) == 1    # m_k n_k > 2^31 - 1
    assert call(2, [2, 2], [2, 2], nnz=-1) == 1
    assert call(2, [2, 2], [2, 2], rows=None) == 1
    assert call(2, [2, 2], [2, 2], idx=None) == 1
    assert call(2, [1 << 31, 2], [1, 1]) == 1          # m_k above 2^31 - 1
    assert call(3, [1 << 30, 1 << 30, 1 << 30], [1, 1, 1]) == 6  # M above 2^63
    assert len(lib.tt_last_error()) > 0
    assert call(2, [2, 2], [2, 2], nnz=0, rows=None, cols=None, idx=None) == 0  # nothing to do


def test_fasttt_host_argument_errors(lib):
    from paper_1908_02721_amd import _lib

    fake = ctypes.c_void_p(0x1000)  # never dereferenced

    def call(d, dims, nnz, p, opt=None, eps=0.1):
        o = _lib.tt_options()
        lib.tt_options_default(ctypes.byref(o))
        for k, v in (opt or {}).items():
            setattr(o, k, v)
        a = (ctypes.c_int64 * len(dims))(*dims)
        h = ctypes.c_void_p(123)
        st = lib.tt_fasttt_decompose(d, a, nnz, fake, fake, eps, p, ctypes.byref(o), None, ctypes.byref(h))
        assert h.value is None
        return st

    assert call(3, [4, 4, 4], 5, -1) == 1
    assert call(3, [4, 4, 4], 5, 4) == 1
    assert call(3, [4, 4, 4], 5, 2, {"precision": 7}) == 1
    assert call(3, [4, 4, 4], 5, 2, {"key_bits": 30}) == 1
    assert call(3, [4, 4, 4], 5, 2, {"keep_intermediates": 1}) == 1
    assert call(3, [4, 4, 4], 5, 2, eps=1.0) == 1
    assert call(1, [4], 5, 1) == 1
    assert call(3, [4, 4, 4], 0, 2) == 5
    assert lib.tt_get_fasttt_info(None, None, None) == 1
    pp = ctypes.c_int32()
    a = (ctypes.c_int64 * 3)(4, 4, 4)
    assert lib.tt_fasttt_select_p(3, a, 0, fake, fake, None, ctypes.byref(pp), None) == 1


def test_options_layout_matches_header(tmp_path):
    """The ctypes mirror of tt_options has the C struct's size and field offsets."""
    import shutil
    import subprocess

    from paper_1908_02721_amd import _lib

    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    fields = [f for f, _ in _lib.tt_options._fields_]
    src = tmp_path / "layout.c"
    src.write_text("#include <stdio.h>\n#include <stddef.h>\n#include \"ttsparse.h\"\nint main(void) {\n"
                   + "".join(f'  printf("%zu\\n", offsetof(tt_options, {f}));\n' for f in fields)
                   + '  printf("%zu\\n", sizeof(tt_options));\n  return 0;\n}\n')
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()]
    want = [getattr(_lib.tt_options, f).offset for f in fields] + [ctypes.sizeof(_lib.tt_options)]
    assert got == want


def test_eval_host_argument_errors(lib):
    """Argument errors of the evaluation calls are reported on the host, each with its own message."""
    fake = ctypes.c_void_p(0x1000)  # never dereferenced
    d = 2
    cores = (ctypes.c_void_p * d)(fake, fake)
    grads = (ctypes.c_void_p * d)(fake, fake)

    def ev(dims, ranks, dtype=0, m=4, idx=fake, y=fake):
        a = (ctypes.c_int64 * d)(*dims)
        r = (ctypes.c_int64 * (d + 1))(*ranks)
        return lib.tt_eval_entries(d, a, r, cores, dtype, m, idx, y, None)

    def bw(dims, ranks, dtype=0, m=4):
        a = (ctypes.c_int64 * d)(*dims)
        r = (ctypes.c_int64 * (d + 1))(*ranks)
        return lib.tt_eval_entries_backward(d, a, r, cores, dtype, m, fake, fake, grads, None)

    cases = [
        (lambda: ev([4, 4], [1, 300, 1]), "rank"),
        (lambda: ev([4, 4], [2, 3, 1]), "ranks[0]"),
        (lambda: ev([4, 0], [1, 3, 1]), "mode size"),
        (lambda: ev([4, 4], [1, 3, 1], dtype=5), "dtype"),
        (lambda: ev([4, 4], [1, 3, 1], m=-1), "m must"),
        (lambda: ev([4, 4], [1, 3, 1], y=None), "y_out"),
        (lambda: bw([4, 4], [1, 300, 1]), "rank"),
    ]
    for call, word in cases:
        assert call() == 1
        assert word in lib.tt_last_error().decode(), lib.tt_last_error()


def test_eval_plan_host_argument_errors(lib):
    """The plan calls check their arguments on the host before any device work."""
    fake = ctypes.c_void_p(0x1000)  # never dereferenced
    d = 2
    dims = (ctypes.c_int64 * d)(4, 4)
    plan = ctypes.c_void_p()
    assert lib.tt_eval_plan_create(d, dims, 4, fake, None, None) == 1
    assert "plan" in lib.tt_last_error().decode()
    assert lib.tt_eval_plan_create(0, dims, 4, fake, None, ctypes.byref(plan)) == 1
    assert "d must" in lib.tt_last_error().decode()
    assert plan.value is None
    assert lib.tt_eval_plan_create(d, dims, -1, fake, None, ctypes.byref(plan)) == 1
    assert "m must" in lib.tt_last_error().decode()
    assert lib.tt_eval_plan_create(d, dims, 4, None, None, ctypes.byref(plan)) == 1
    bad = (ctypes.c_int64 * d)(4, 0)
    assert lib.tt_eval_plan_create(d, bad, 4, fake, None, ctypes.byref(plan)) == 1
    assert "mode size" in lib.tt_last_error().decode()
    ranks = (ctypes.c_int64 * (d + 1))(1, 3, 1)
    cores = (ctypes.c_void_p * d)(fake, fake)
    assert lib.tt_eval_plan_forward(None, ranks, cores, 0, fake, 1, None) == 1
    assert lib.tt_eval_plan_backward(None, ranks, cores, 0, fake, cores, 1, None) == 1
    lib.tt_eval_plan_free(None)
