"""C-ABI checks that need no GPU: the library loads, exports every function the
header declares, and rejects malformed arguments on the host before any HIP
call (wrapped handles over dummy pointers are never dereferenced here)."""
import ctypes as C

import numpy as np
import pytest

from paper_2102_08505_amd import ellsp2 as E
from paper_2102_08505_amd import synth

DUMMY = 0x1000  # never dereferenced: every call below fails validation first


def test_library_exports_every_declared_function():
    L = E.load()
    names = E.header_functions()
    expected = {"ellpack_check_host", "ellpack_alloc", "ellpack_wrap", "ellpack_free", "ellpack_info",
                "ellpack_upload", "ellpack_download", "ellpack_x2_threshold", "ellpack_x2_step",
                "ellpack_trace", "sp2_solve", "sp2_solve_batched", "dense_sp2_solve", "dense_x2",
                "ellpack_strerror", "ellpack_last_device_error"}
    assert expected <= set(names)
    for n in names:
        assert hasattr(L, n), n


def test_strerror_covers_every_status():
    for s in [E.ELL_OK, E.ELL_EINVAL, E.ELL_ENOMEM, E.ELL_EOVERFLOW, E.ELL_ENOCONV, E.ELL_EDEVICE,
              E.ELL_ENODEV, E.ELL_ENONFINITE, E.ELL_EDEGENERATE]:
        assert E.ellpack_strerror(s) != "unknown status"
    assert E.ellpack_strerror(12345) == "unknown status"


def test_check_host_accepts_generator_output():
    nnz, idx, val, M = synth.banded_hamiltonian(100, 4)
    assert E.ellpack_check_host(100, M, nnz, idx, val) == E.ELL_OK


@pytest.mark.parametrize("case", ["N0", "M0", "nnz_neg", "nnz_big", "col_neg", "col_big", "unsorted",
                                  "duplicate", "nan", "inf", "M_too_big"])
def test_check_host_rejects(case):
    N, M = 4, 3
    nnz = np.array([2, 1, 0, 3], np.int32)
    idx = np.array([0, 2, -1, 1, -1, -1, -1, -1, -1, 0, 1, 3], np.int32)
    val = np.ones(N * M)
    expect = E.ELL_EINVAL
    if case == "N0":
        N = 0
    elif case == "M0":
        M = 0
    elif case == "nnz_neg":
        nnz[2] = -1
    elif case == "nnz_big":
        nnz[1] = 4
    elif case == "col_neg":
        idx[0] = -2
    elif case == "col_big":
        idx[11] = 4
    elif case == "unsorted":
        idx[0], idx[1] = 2, 0
    elif case == "duplicate":
        idx[10] = 0
    elif case == "nan":
        val[3] = np.nan
        expect = E.ELL_ENONFINITE
    elif case == "inf":
        val[9] = -np.inf
        expect = E.ELL_ENONFINITE
    elif case == "M_too_big":
        assert E.ellpack_check_host(4, 65537, np.zeros(4, np.int32), np.zeros(4 * 65537, np.int32)) == E.ELL_EINVAL
        return
    assert E.ellpack_check_host(N, M, nnz, idx, val) == expect


def test_alloc_argument_errors_need_no_device():
    assert E.ellpack_alloc(0, 4)[0] == E.ELL_EINVAL
    assert E.ellpack_alloc(4, 0)[0] == E.ELL_EINVAL
    assert E.ellpack_alloc(4, 4, prec=7)[0] == E.ELL_EINVAL


def wrap(N, M, prec=E.ELL_F64, base=DUMMY):
    rc, h = E.ellpack_wrap(N, M, prec, base, base + 0x100, base + 0x200)
    assert rc == E.ELL_OK
    return h


def test_wrap_and_info_without_device():
    h = wrap(10, 8, E.ELL_F32)
    assert E.ellpack_info(h) == (E.ELL_OK, 10, 8, E.ELL_F32)
    assert E.ellpack_free(h) == E.ELL_OK
    assert E.ellpack_free(None) == E.ELL_OK
    assert E.ellpack_wrap(10, 8, E.ELL_F64, 0, DUMMY, DUMMY)[0] == E.ELL_EINVAL
    assert E.ellpack_wrap(10, 0, E.ELL_F64, DUMMY, DUMMY, DUMMY)[0] == E.ELL_EINVAL


def test_x2_argument_errors_before_device():
    X = wrap(10, 8, base=0x10000)
    Y = wrap(10, 8, base=0x20000)
    Z = wrap(11, 8, base=0x30000)
    F = wrap(10, 8, E.ELL_F32, base=0x40000)
    assert E.ellpack_x2_threshold(X, X, 0.0)[0] == E.ELL_EINVAL          # aliasing
    assert E.ellpack_x2_threshold(X, Z, 0.0)[0] == E.ELL_EINVAL          # N mismatch
    assert E.ellpack_x2_threshold(X, F, 0.0)[0] == E.ELL_EINVAL          # precision mismatch
    assert E.ellpack_x2_threshold(X, Y, -1e-5)[0] == E.ELL_EINVAL        # negative tau
    assert E.ellpack_x2_threshold(X, Y, float("nan"))[0] == E.ELL_EINVAL
    assert E.ellpack_x2_threshold(None, Y, 0.0)[0] == E.ELL_EINVAL
    assert E.ellpack_x2_step(X, Y, X, 0.0)[0] == E.ELL_EINVAL           # U aliases X
    assert E.ellpack_x2_step(X, Y, Y, 0.0)[0] == E.ELL_EINVAL           # U aliases X2
    Yalias = wrap(10, 8, base=0x10000)                                   # same storage as X
    assert E.ellpack_x2_threshold(X, Yalias, 0.0)[0] == E.ELL_EINVAL
    for h in (X, Y, Z, F, Yalias):
        E.ellpack_free(h)


def test_upload_validates_host_arrays_first():
    h = wrap(4, 3)
    nnz = np.array([1, 1, 1, 5], np.int32)
    assert E.ellpack_upload(h, nnz, np.zeros(12, np.int32), np.zeros(12)) == E.ELL_EINVAL
    nnz = np.array([1, 1, 1, 1], np.int32)
    v = np.zeros(12)
    v[0] = np.inf
    assert E.ellpack_upload(h, nnz, np.array([0, 0, 0, 1, 0, 0, 2, 0, 0, 3, 0, 0], np.int32), v) == E.ELL_ENONFINITE
    E.ellpack_free(h)


def test_sp2_argument_errors_before_device():
    H = wrap(10, 8, base=0x10000)
    D = wrap(10, 8, base=0x20000)
    Hf = wrap(10, 8, E.ELL_F32, base=0x30000)
    good = E.sp2_params(2.5, 0.0, 1e-8)
    assert E.sp2_solve(H, H, good)[0] == E.ELL_EINVAL
    assert E.sp2_solve(Hf, D, good)[0] == E.ELL_EINVAL
    for bad in [E.sp2_params(2.5, -1.0, 1e-8), E.sp2_params(2.5, 0.0, -1.0), E.sp2_params(2.5, 0.0, 1e-8, max_iter=0),
                E.sp2_params(2.5, 0.0, 1e-8, precision=5), E.sp2_params(float("nan"), 0.0, 1e-8),
                E.sp2_params(2.5, 0.0, 1e-8, precision=E.SP2_MIXED, tau_fp32=-1.0),
                E.sp2_params(2.5, 0.0, 1e-8, fp64_tail_steps=-1)]:
        assert E.sp2_solve(H, D, bad)[0] == E.ELL_EINVAL
    for h in (H, D, Hf):
        E.ellpack_free(h)


def test_struct_layouts_match_header(tmp_path):
    """Offsets of the ctypes mirrors equal the ones gcc gives the header's structs."""
    import os
    import subprocess
    src = tmp_path / "layout.c"
    fields_p = [f for f, _ in E.SP2Params._fields_]
    fields_r = [f for f, _ in E.SP2Report._fields_]
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "ellsp2.h"', 'int main(void) {',
             'printf("%zu %zu\\n", sizeof(sp2_params_t), sizeof(sp2_report_t));']
    lines += [f'printf("%zu\\n", offsetof(sp2_params_t, {f}));' for f in fields_p]
    lines += [f'printf("%zu\\n", offsetof(sp2_report_t, {f}));' for f in fields_r]
    lines += ['return 0; }']
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    inc = os.path.join(os.path.dirname(E.HEADER))
    subprocess.run(["gcc", "-I", inc, "-o", str(exe), str(src)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()
    vals = [int(x) for x in out]
    assert vals[0] == C.sizeof(E.SP2Params) and vals[1] == C.sizeof(E.SP2Report)
    offs = vals[2:]
    assert offs[: len(fields_p)] == [getattr(E.SP2Params, f).offset for f in fields_p]
    assert offs[len(fields_p):] == [getattr(E.SP2Report, f).offset for f in fields_r]
