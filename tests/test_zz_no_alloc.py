"""qtt_dot_noalloc (the entry point for callers that cannot allocate)
against qtt_dot on the same operands, through the C ABI: two calls in a
row, the second with smaller operands, so the shared scratch holds the
first call's contents when the second starts; and an oversized request is
refused before any device work."""
import ctypes as C

import numpy as np
import pytest

import workloads as W
from oracle import assembly as A
from oracle import qtt as T

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2501_07778_amd as P
    return P


def test_dot_noalloc_equals_dot_on_two_calls(P):
    # call 1: a rank-40 train against a level-8 product (ranks up to 1000):
    # the chip-wide GEMM path of the inner product
    Kq, _ = A.assemble_qtt(W.cantilever_traction(8))
    modes = [2] * 17
    x = P.tt_from_cores(W.random_tt_cores(71, modes, W.capped_ranks(modes, 40)))
    y = P.tt_from_cores(T.matvec(Kq, W.random_tt_cores(72, modes, W.capped_ranks(modes, 40))))
    print("noalloc call 1: ranks %d x %d" % (max(x.ranks), max(y.ranks)), flush=True)
    ref1 = P.dot(x, y)
    got1 = P.dot_noalloc(x, y)
    assert got1 == pytest.approx(ref1, rel=1e-13, abs=1e-300)
    # call 2: smaller operands (one-workgroup path) on the same scratch
    modes = [2] * 9
    u = P.tt_from_cores(W.random_tt_cores(73, modes, W.capped_ranks(modes, 5)))
    v = P.tt_from_cores(W.random_tt_cores(74, modes, W.capped_ranks(modes, 7)))
    print("noalloc call 2: ranks %d x %d" % (max(u.ranks), max(v.ranks)), flush=True)
    ref2 = P.dot(u, v)
    got2 = P.dot_noalloc(u, v)
    assert got2 == pytest.approx(ref2, rel=1e-13, abs=1e-300)
    oracle2 = T.dot(P.tt_to_cores(u), P.tt_to_cores(v))
    assert got2 == pytest.approx(oracle2, rel=1e-12)


def test_dot_noalloc_refuses_oversized_operands(P):
    # ranks 2048 against 2048 at one bond need 2 * 2048^2 doubles > 2^21
    # (host-only check: the descriptors' device pointers are never used)
    L = P.lib()
    D = 3
    nrow = (C.c_int32 * D)(2, 2, 2)
    big = (C.c_int32 * (D + 1))(1, 2, 2048, 1)
    x = P._lib._TT(D, nrow, None, big, 4096, 1 << 30)
    y = P._lib._TT(D, nrow, None, big, 4096, 1 << 30)
    out = C.c_double()
    st = L.qtt_dot_noalloc(C.byref(x), C.byref(y), C.byref(out), None)
    assert st == -3 and b"scratch" in L.qtt_last_error()
