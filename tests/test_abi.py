"""The C-ABI library loads, exports every function include/lyap.h declares,
and its struct layouts agree with the Python binding.  CPU only: no compute
calls (argument validation returns before any device work)."""
import ctypes as ct
import os
import re
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "include", "lyap.h")


def _declared_functions():
    src = open(HDR).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[\w\s\*]+?\b(\w+)\s*\(", src, flags=re.M)
    return sorted({n for n in names if n.startswith(("lyap_", "sylv_")) and not n.endswith("_fn")})


@pytest.fixture(scope="module")
def lib():
    from paper_1602_05033_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        from paper_1602_05033_amd import build
        build.build()
    return binding.load()


def test_every_declared_symbol_is_exported(lib):
    from paper_1602_05033_amd import binding
    names = _declared_functions()
    assert "lyap_solve" in names and "sylv_solve" in names and "lyap_ctri" in names
    for n in names:
        assert hasattr(lib, n), n
    assert set(binding.EXPORTS) <= set(names)


def test_struct_layouts_match_header(lib):
    from paper_1602_05033_amd import binding as b
    code = r"""
#include <stdio.h>
#include <stddef.h>
#include "lyap.h"
int main(void) {
  printf("%zu %zu %zu %zu\n", sizeof(lyap_op), sizeof(lyap_opts), sizeof(lyap_result), sizeof(sylv_result));
  printf("%zu %zu %zu %zu\n", offsetof(lyap_op, shift), offsetof(lyap_opts, verbose),
         offsetof(lyap_result, owns_Z), offsetof(sylv_result, n_checks));
  return 0;
}
"""
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        exe = os.path.join(d, "t")
        open(c, "w").write(code)
        subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe])
        out = subprocess.check_output([exe]).decode().split()
    sizes = list(map(int, out[:4]))
    offs = list(map(int, out[4:]))
    assert sizes == [ct.sizeof(b.LyapOp), ct.sizeof(b.LyapOpts), ct.sizeof(b.LyapResult), ct.sizeof(b.SylvResult)]
    assert offs == [b.LyapOp.shift.offset, b.LyapOpts.verbose.offset, b.LyapResult.owns_Z.offset,
                    b.SylvResult.n_checks.offset]


def test_defaults(lib):
    from paper_1602_05033_amd import binding as b
    o = b.LyapOpts()
    lib.lyap_opts_default(ct.byref(o))
    assert o.tol == 1e-8 and o.two_pass == 1 and o.storage == b.STORE_F64 and o.check_every == 0


def test_argument_errors_without_device_work(lib):
    from paper_1602_05033_amd import binding as b
    r = b.LyapResult()
    # NULL operator
    st = lib.lyap_solve(None, ct.c_void_p(1), 1, 10, None, ct.byref(r))
    assert st == b.E_ARG and b"NULL" in lib.lyap_last_error()
    # inconsistent stencil
    op = b.LyapOp()
    op.kind, op.nx, op.ny, op.n = b.OP_STENCIL5, 4, 4, 15
    st = lib.lyap_solve(ct.byref(op), ct.c_void_p(1), 1, 15, None, ct.byref(r))
    assert st == b.E_ARG and b"stencil5" in lib.lyap_last_error()
    # s out of range / ldc too small / bad tol
    op.n = 16
    assert lib.lyap_solve(ct.byref(op), ct.c_void_p(1), 9, 16, None, ct.byref(r)) == b.E_ARG
    assert lib.lyap_solve(ct.byref(op), ct.c_void_p(1), 1, 8, None, ct.byref(r)) == b.E_ARG
    o = b.LyapOpts()
    lib.lyap_opts_default(ct.byref(o))
    o.tol = 0.0
    assert lib.lyap_solve(ct.byref(op), ct.c_void_p(1), 1, 16, ct.byref(o), ct.byref(r)) == b.E_ARG
    assert r.status == b.E_ARG
    # NULL C
    assert lib.lyap_solve(ct.byref(op), None, 1, 16, None, ct.byref(r)) == b.E_ARG
    # component entry points
    assert lib.lyap_op_apply(ct.byref(op), 0, None, None, 1, None) == b.E_ARG
    res = ct.c_double()
    assert lib.lyap_ctri(None, 1, 4, None, None, ct.byref(res), None, None) == b.E_ARG
    lib.lyap_result_free(ct.byref(r))       # safe on an error result


def test_pcnet_init_matches_oracle():
    """Host-side SplitMix64 weight initialisation of the library = the oracle's
    (the same published generator implemented twice), rounded to FP32."""
    import numpy as np
    from paper_1602_05033_amd import binding as b
    from oracle import cnn as N
    for C, seed, scale in ((4, 0x5eed, 0.05), (2, 7, 0.3), (8, 12345, 1.0)):
        W = b.pcnet_init(C, seed, scale)
        ref = N.init_net(C, seed, scale).flat().astype(np.float32)
        assert np.array_equal(W, ref)
