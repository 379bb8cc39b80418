"""Host-side checks of the C ABI that need no GPU: the library loads and
exports every entry point declared in include/*.h, and argument validation
rejects bad input with the documented status codes."""
import os
import re

import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for f in os.listdir(os.path.join(ROOT, "include")):
        if f.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", f)).read()
            names |= set(re.findall(r"^\s*(?:rfd_status|const char\*|int)\s+(rfd_\w+)\s*\(", txt, re.M))
    return names


def _lib():
    import paper_1711_09487_amd as R
    if not os.path.exists(R.LIB_PATH):
        pytest.skip("library not built")
    return R


def test_library_exports_every_declared_symbol():
    R = _lib()
    names = _declared()
    assert {"rfd_create_pencil", "rfd_set_partition", "rfd_set_interval_and_poles",
            "rfd_filter_interface", "rfd_solve_interior", "rfd_rayleigh_ritz"} <= names
    L = R.lib()
    for nm in sorted(names):
        assert hasattr(L, nm), nm


def test_create_pencil_validation():
    R = _lib()
    A = W.laplacian((5, 5))
    M = sp.identity(25, format="csr")
    h = R.rfd_create_pencil(A, M)
    R.rfd_destroy_pencil(h)
    Ab = A.tolil()
    Ab[0, 1] = 5.0                       # not symmetric
    with pytest.raises(R.RfdError) as e:
        R.rfd_create_pencil(Ab.tocsr(), M)
    assert e.value.code == 1
    Mb = sp.diags(np.r_[-1.0, np.ones(24)]).tocsr()
    with pytest.raises(R.RfdError) as e:
        R.rfd_create_pencil(A, Mb)
    assert e.value.code == 1


def test_partition_and_interval_validation():
    R = _lib()
    A = W.laplacian((7, 7))
    M = sp.identity(49, format="csr")
    h = R.rfd_create_pencil(A, M)
    try:
        bad = np.zeros(49, dtype=np.int32)
        bad[25:] = 1                     # subdomains touch directly
        with pytest.raises(R.RfdError) as e:
            R.rfd_set_partition(h, 2, bad)
        assert e.value.code == 1
        with pytest.raises(R.RfdError):
            R.rfd_set_partition(h, 2, np.full(49, 5, dtype=np.int32))
        with pytest.raises(R.RfdError) as e:
            R.rfd_set_interval_and_poles(h, 1.0, 0.5, 4)
        assert e.value.code == 1
        with pytest.raises(R.RfdError):
            R.rfd_set_interval_and_poles(h, 0.0, 1.0, 0)
        with pytest.raises(R.RfdError):
            R.rfd_set_precision(h, 7)
        with pytest.raises(R.RfdError) as e:
            R.rfd_solve_interior(h, 0.1, 4, 2, stream=0)
        assert e.value.code == 6        # before set_partition
        assert R.rfd_last_error() != ""
    finally:
        R.rfd_destroy_pencil(h)


def test_destroy_null_is_ok():
    R = _lib()
    assert R.lib().rfd_destroy_pencil(None) == 0


def test_job_and_result_layout_match_the_header(tmp_path):
    """The ctypes mirrors of rfd_job / rfd_result have the C layout (offset of
    every field and the size), checked with the host C compiler."""
    import ctypes as C
    import shutil
    import subprocess
    import paper_1711_09487_amd as R
    if shutil.which("gcc") is None:
        pytest.skip("no host C compiler")
    lines = []
    for st in (R.rfd_job, R.rfd_result):
        name = st.__name__
        lines.append(f'printf("{name} size %zu\\n", sizeof({name}));')
        for f, _ in st._fields_:
            lines.append(f'printf("{name}.{f} %zu\\n", offsetof({name}, {f}));')
    src = tmp_path / "layout.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "rfd.h"\nint main(void){'
                   + "".join(lines) + "return 0;}\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    out = dict(l.rsplit(" ", 1) for l in subprocess.run([str(exe)], capture_output=True,
                                                        text=True, check=True).stdout.split("\n") if l)
    for st in (R.rfd_job, R.rfd_result):
        name = st.__name__
        assert int(out[f"{name} size"]) == C.sizeof(st)
        for f, _ in st._fields_:
            assert int(out[f"{name}.{f}"]) == getattr(st, f).offset, (name, f)


def test_batch_and_server_argument_validation():
    R = _lib()
    L = R.lib()
    import ctypes as C
    assert L.rfd_batch_run(0, None, None, None, 0, 0) == 1
    res = R.rfd_result()
    assert L.rfd_server_poll(None, 1, 0, C.byref(res)) == 1
    assert L.rfd_server_submit(None, None, None, None) == 1
    assert L.rfd_server_destroy(None) == 0


def test_gemm_entry_points_reject_bad_operands_before_launching():
    """Both product entry points refuse null operand planes, and the
    allocation-free one refuses outputs beyond half its 64 MiB scratch, before
    any device work (so these run without a GPU)."""
    R = _lib()
    L = R.lib()
    for fn in (L.rfd_test_gemm, L.rfd_test_gemm_static):
        code = fn(1, 0, 0, 64, 64, 64, 1.0, 0.0, None, None, 64, 0, None, None, 64, 0, None, None,
                  64, 0, 1, None)
        assert code == 1 and "null" in R.rfd_last_error()
    fake = 1 << 20          # never dereferenced: the size check comes first
    code = L.rfd_test_gemm_static(1, 0, 0, 2048, 2048, 64, 1.0, 0.0, fake, fake, 2048, 0, fake, fake,
                                  64, 0, fake, fake, 2048, 0, 1, None)
    assert code == 1 and "at most" in R.rfd_last_error()


def test_interior_solver_needs_a_partition():
    """rfd_set_interior_solver before rfd_set_partition: RFD_ESTATE (no device
    work happens on this path)."""
    R = _lib()
    A = W.laplacian((5, 5))
    M = sp.identity(25, format="csr")
    h = R.rfd_create_pencil(A, M)
    try:
        with pytest.raises(R.RfdError) as e:
            R.rfd_set_interior_solver(h, R.RFD_INTERIOR_SPECTRAL)
        assert e.value.code == 6
    finally:
        R.rfd_destroy_pencil(h)


def test_gemm_tuning_table_validation():
    """rfd_set_gemm_tuning takes rows of 9 int32 and rejects a malformed row
    (unknown variant, the 128-wide tile for a complex or FP64 class, the
    large-tile FP64 kernel for FP32, a log2 out of range) with RFD_EINVAL,
    leaving the table as it was; an empty table restores the built-in rules.
    The forced-variant hook refuses unknown variants before any device work."""
    R = _lib()
    good = [[1, 0, 1, 0, 13, 11, 17, 0, 3], [0, 0, 0, 0, 12, 12, 10, 0, 2],
            [1, 1, 0, 0, 12, 12, 12, 3, 1]]
    R.rfd_set_gemm_tuning(good)
    for bad in ([1, 0, 0, 0, 10, 10, 10, 0, 4], [1, 1, 0, 0, 10, 10, 10, 0, 2],
                [0, 1, 0, 0, 10, 10, 10, 0, 2], [0, 0, 0, 0, 10, 10, 10, 0, 3],
                [1, 0, 2, 0, 10, 10, 10, 0, 1], [1, 0, 0, 0, 63, 10, 10, 0, 1],
                [1, 0, 0, 0, 10, 10, -1, 0, 1]):
        with pytest.raises(R.RfdError) as e:
            R.rfd_set_gemm_tuning(good + [bad])
        assert e.value.code == 1 and "malformed" in str(e.value)
    R.rfd_set_gemm_tuning(np.zeros((0, 9), dtype=np.int32))
    L = R.lib()
    fake = 1 << 20
    for v in (0, 4):
        code = L.rfd_test_gemm_variant(v, 1, 0, 0, 64, 64, 64, 1.0, 0.0, fake, None, 64, 0, fake,
                                       None, 64, 0, fake, None, 64, 0, 1, None)
        assert code == 1 and "variant" in R.rfd_last_error()
