"""The C ABI library without a GPU: it loads, exports every function that
include/chfsi.h declares, and rejects bad arguments before any device work
(chfsi_plan needs no device)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "chfsi.h")
LIB = os.environ.get("CHFSI_LIBRARY") or os.path.join(ROOT, "paper_2605_30128_amd", "libchfsi.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(chfsi_[A-Za-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2605_30128_amd import build
        build.build()
    return C.CDLL(LIB)


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert len(names) >= 17
    for n in names:
        assert hasattr(lib, n), n
    from paper_2605_30128_amd import binding
    assert set(binding.SYMBOLS) <= set(names)


def _mesh(binding, ncell=(4, 4, 4), h=(2.0, 2.0, 2.0), degree=4, nq=0):
    return binding._Mesh((C.c_int64 * 3)(*ncell), (C.c_double * 3)(*h), degree, nq)


def test_plan_sizes_and_validation(lib):
    from paper_2605_30128_amd import binding
    L = binding.load()
    pb, sb = C.c_size_t(), C.c_size_t()
    m = _mesh(binding)
    assert L.chfsi_plan(C.byref(m), None, 32, C.byref(pb), C.byref(sb)) == 0
    # two recurrence blocks of 2M x 32 complex128 at least
    assert sb.value >= 2 * 2 * 4096 * 32 * 16
    pb2, sb2 = C.c_size_t(), C.c_size_t()
    assert L.chfsi_plan(C.byref(m), None, 64, C.byref(pb2), C.byref(sb2)) == 0
    assert sb2.value > sb.value and pb2.value == pb.value
    bad = [
        _mesh(binding, ncell=(3, 4, 4)),      # odd cell count: colouring impossible
        _mesh(binding, ncell=(0, 4, 4)),
        _mesh(binding, h=(2.0, -1.0, 2.0)),
        _mesh(binding, degree=0),
        _mesh(binding, degree=8),
        _mesh(binding, nq=9),
    ]
    for mb in bad:
        assert L.chfsi_plan(C.byref(mb), None, 32, C.byref(pb), C.byref(sb)) == binding.E_ARG
        assert len(L.chfsi_last_error(None)) > 0
    assert L.chfsi_plan(C.byref(m), None, 0, C.byref(pb), C.byref(sb)) == binding.E_ARG
    assert L.chfsi_plan(None, None, 32, C.byref(pb), C.byref(sb)) == binding.E_ARG


def test_plan_ex_filter_blocks(lib):
    """chfsi_plan_ex: the recurrence area follows filter_block and the
    filter's complex type; chfsi_plan is the FP64 plan of max_nvec columns."""
    from paper_2605_30128_amd import binding
    L = binding.load()
    m = _mesh(binding)
    rows = 2 * 4096

    def plan(opts):
        pb, sb = C.c_size_t(), C.c_size_t()
        rc = L.chfsi_plan_ex(C.byref(m), None, C.byref(opts), C.byref(pb), C.byref(sb))
        return rc, pb.value, sb.value

    rc, pb0, sb0 = plan(binding.PlanOpts(64, 0, binding.FP64))
    assert rc == 0
    pbp, sbp = C.c_size_t(), C.c_size_t()
    assert L.chfsi_plan(C.byref(m), None, 64, C.byref(pbp), C.byref(sbp)) == 0
    assert (pbp.value, sbp.value) == (pb0, sb0)
    rc, pb1, sb1 = plan(binding.PlanOpts(64, 0, binding.BF16))
    assert rc == 0 and pb1 == pb0
    # complex64 recurrence blocks: 2 x rows x 64 x 8 bytes less
    assert sb0 - sb1 == 2 * rows * 64 * 8
    rc, _, sb2 = plan(binding.PlanOpts(64, 16, binding.FP64))
    assert rc == 0 and sb0 - sb2 == 2 * rows * (64 - 16) * 16
    assert plan(binding.PlanOpts(64, 65, binding.FP64))[0] == binding.E_ARG
    assert plan(binding.PlanOpts(0, 0, binding.FP64))[0] == binding.E_ARG
    assert plan(binding.PlanOpts(64, 0, 7))[0] == binding.E_ARG


def test_plan_rejects_bad_projectors(lib):
    from paper_2605_30128_amd import binding
    L = binding.load()
    m = _mesh(binding)
    ptr = np.array([0, 2, 1], np.int64)          # not monotone
    cell = np.array([0, 1], np.int64)
    phi = np.zeros(2 * 125 * 2 * 4, np.complex128)
    delta = np.zeros(2 * 16, np.complex128)
    pr = binding._Proj(2, 4, ptr.ctypes.data, cell.ctypes.data, phi.ctypes.data, delta.ctypes.data)
    pb, sb = C.c_size_t(), C.c_size_t()
    assert L.chfsi_plan(C.byref(m), C.byref(pr), 8, C.byref(pb), C.byref(sb)) == binding.E_ARG
    ptr = np.array([0, 1, 2], np.int64)
    cell = np.array([0, 64], np.int64)           # cell out of range
    pr = binding._Proj(2, 4, ptr.ctypes.data, cell.ctypes.data, phi.ctypes.data, delta.ctypes.data)
    assert L.chfsi_plan(C.byref(m), C.byref(pr), 8, C.byref(pb), C.byref(sb)) == binding.E_ARG
    pr = binding._Proj(2, 17, ptr.ctypes.data, cell.ctypes.data, phi.ctypes.data, delta.ctypes.data)
    assert L.chfsi_plan(C.byref(m), C.byref(pr), 8, C.byref(pb), C.byref(sb)) == binding.E_ARG
    cell = np.array([0, 1], np.int64)
    pr = binding._Proj(2, 4, ptr.ctypes.data, cell.ctypes.data, phi.ctypes.data, delta.ctypes.data)
    assert L.chfsi_plan(C.byref(m), C.byref(pr), 8, C.byref(pb), C.byref(sb)) == 0


def test_null_context_calls_fail_cleanly(lib):
    from paper_2605_30128_amd import binding
    L = binding.load()
    assert L.chfsi_apply_H(None, 0, None, None, 1, 1, None) == binding.E_ARG
    assert L.chfsi_filter(None, 0, 5, None, None, None, None, None, 1, 1, None) == binding.E_ARG
    assert L.chfsi_solve(None, 1, None, None, 2, 2, None, None, None, None, None, 0, None) == binding.E_ARG
    assert L.chfsi_apply_K(None, None, None, None) == binding.E_ARG
    assert L.chfsi_poisson_precond(None, 5, 0.1, 2.0, None, None, None) == binding.E_ARG
    assert L.chfsi_poisson_solve(None, None, None, None, None, None) == binding.E_ARG
    L.chfsi_destroy(None)


def test_bfp_sizes_and_argument_checks(lib):
    """The codec entry points size the stream and reject bad arguments
    before any device work (an empty stream launches nothing)."""
    from paper_2605_30128_amd import binding
    L = binding.load()
    out = C.c_int64()
    for nbits, per4 in ((16, 8), (12, 6), (10, 5)):
        assert L.chfsi_bfp_bytes(nbits, 4096, C.byref(out)) == 0
        assert out.value == 1024 * per4
    assert L.chfsi_bfp_bytes(14, 8, C.byref(out)) == -1
    assert L.chfsi_bfp_bytes(16, 6, C.byref(out)) == -1
    assert L.chfsi_bfp_bytes(16, -4, C.byref(out)) == -1
    assert L.chfsi_bfp_encode(16, None, 0, None, None) == 0
    assert L.chfsi_bfp_decode(12, None, 0, None, None) == 0
    assert L.chfsi_bfp_encode(16, None, 8, None, None) == -1
    assert L.chfsi_bfp_decode(10, None, 4, None, None) == -1
    assert b"NULL" in L.chfsi_last_error(None)
