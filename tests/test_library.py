"""Host-side checks of the C-ABI library: it loads without a GPU and exports
every function declared in include/qtt.h; host validation rejects bad input
before any device work."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2501_07778_amd", "libqtt.so")


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(qtt_[a-z_0-9]+)\s*\(", txt))
    return names


def test_header_declares_the_four_calls():
    d = _declared()
    for n in ("qtt_assemble_stiffness", "qtt_matvec", "qtt_round", "qtt_solve"):
        assert n in d


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.skip("libqtt.so not built")
    lib = C.CDLL(LIB)
    for n in sorted(_declared()):
        assert hasattr(lib, n), n


def test_host_validation_without_gpu():
    if not os.path.exists(LIB):
        pytest.skip("libqtt.so not built")
    import paper_2501_07778_amd as P
    L = P.lib()
    # NULL operands and bad shapes are rejected on the host with a message
    assert L.qtt_matvec(None, None, None, 0, None, 0, None) == -1
    assert b"NULL" in L.qtt_last_error()
    nrow = (C.c_int32 * 2)(2, 2)
    ranks = (C.c_int32 * 3)(1, 3, 2)    # last rank must be 1
    t = P._lib._TT(2, nrow, None, ranks, None, 100)
    need = C.c_size_t()
    assert L.qtt_round(C.byref(t), 1e-8, 0, None, None, None, 0, None) == -2
    assert b"boundary" in L.qtt_last_error()
    ranks[2] = 1
    t.capacity = 3                      # needs 1*2*3 + 3*2*1 = 12
    t.data = 12345                      # never dereferenced: validation fails first
    assert L.qtt_round(C.byref(t), 1e-8, 0, None, None, None, 0, None) == -3
    t.capacity = 12
    assert L.qtt_round_workspace(C.byref(t), 0, C.byref(need)) == 0 and need.value > 0
    # a workspace that is too small is reported, not used
    assert L.qtt_round(C.byref(t), 1e-8, 0, None, None, None, 16, None) == -3
    # storage other than FP64 is refused before any launch
    t.dtype = 1
    assert L.qtt_round(C.byref(t), 1e-8, 0, None, None, None, 16, None) == -7
    assert b"dtype" in L.qtt_last_error()
    t.dtype = 0
    assert L.qtt_version().startswith(b"qtt")


def test_problem_coupling_and_gamma_validation():
    """The coupling field takes QTT_COUPLING_PAPER (0) or
    QTT_COUPLING_SYMMETRIC (1); a NaN gamma is refused (host checks only)."""
    if not os.path.exists(LIB):
        pytest.skip("libqtt.so not built")
    import paper_2501_07778_amd as P
    import workloads as W
    L = P.lib()
    prob = P._lib.problem_from_workload(W.l_shape(3))
    assert prob.c.coupling == 1 and prob.c.gamma == 0.0
    need, kc, fc = C.c_size_t(), C.c_int64(), C.c_int64()
    assert L.qtt_assemble_workspace(C.byref(prob.c), C.byref(need), C.byref(kc), C.byref(fc)) == 0
    prob.c.coupling = 2
    assert L.qtt_assemble_workspace(C.byref(prob.c), C.byref(need), C.byref(kc), C.byref(fc)) == -1
    prob.c.coupling = 0
    prob.c.gamma = float("nan")
    assert L.qtt_assemble_workspace(C.byref(prob.c), C.byref(need), C.byref(kc), C.byref(fc)) == -1
    assert b"gamma" in L.qtt_last_error()


def test_als_options_and_workspace_on_the_host():
    """The ALS method's option checks and workspace query (host only: the
    descriptors' device pointers are never dereferenced).  The workspace
    holds one dense local matrix, 8 (r n r)^2 bytes at the widest core."""
    if not os.path.exists(LIB):
        pytest.skip("libqtt.so not built")
    import paper_2501_07778_amd as P
    L = P.lib()
    D = 21
    nrow = (C.c_int32 * D)(*([2] * D))
    kr = [1, 4, 14, 23] + [25] * 14 + [20, 16, 4, 1]
    fr = [1, 2, 4, 8] + [12] * 14 + [8, 4, 2, 1]
    kranks = (C.c_int32 * (D + 1))(*kr)
    franks = (C.c_int32 * (D + 1))(*fr)
    K = P._lib._TT(D, nrow, nrow, kranks, 4096, 1 << 30)
    f = P._lib._TT(D, nrow, None, franks, 8192, 1 << 30)

    def ws(**kw):
        o = P.SolveOpts(method="als", **kw).c()
        need = C.c_size_t()
        st = L.qtt_solve_workspace(C.byref(K), C.byref(f), C.byref(o), C.byref(need))
        return st, need.value

    st64, b64 = ws(rmax=64, maxit_out=8)
    st32, b32 = ws(rmax=32, maxit_out=8)
    assert st64 == 0 and st32 == 0
    assert b64 >= 8 * (64 * 2 * 64) ** 2          # the local matrix at N = 8192
    # the local matrix grows as (r n r)^2 (the residual check's trains as r)
    assert b64 - b32 >= 8 * ((64 * 2 * 64) ** 2 - (32 * 2 * 32) ** 2)
    assert ws(rmax=64, maxit_out=0)[0] == -1       # no sweeps
    assert ws(rmax=1000, maxit_out=8)[0] == -1     # rank beyond the supported cap
    assert ws(rmax=64, maxit_out=8, compute="f32")[0] == -7   # local solves are FP64
    assert b"FP64" in L.qtt_last_error()


def test_solve_rejects_malformed_trains_before_any_launch():
    """qtt_solve validates K, f, x0 and u on the host: an undersized or
    mis-shaped start vector, or an undersized operand, is an error code
    before any device work (the descriptors' device pointers are fake)."""
    if not os.path.exists(LIB):
        pytest.skip("libqtt.so not built")
    import paper_2501_07778_amd as P
    L = P.lib()
    D = 5
    nrow = (C.c_int32 * D)(*([2] * D))
    kranks = (C.c_int32 * (D + 1))(1, 3, 3, 3, 3, 1)
    franks = (C.c_int32 * (D + 1))(1, 2, 2, 2, 2, 1)
    K = P._lib._TT(D, nrow, nrow, kranks, 4096, 1 << 20)
    f = P._lib._TT(D, nrow, None, franks, 8192, 1 << 20)
    u = P._lib._TT(D, nrow, None, (C.c_int32 * (D + 1))(*([1] * (D + 1))), 16384, 1 << 20)
    o = P.SolveOpts(method="als", rmax=4, maxit_out=4).c()
    rep = P._lib._SolveReport()

    def solve(x0):
        return L.qtt_solve(C.byref(K), C.byref(f), C.byref(x0) if x0 is not None else None,
                           C.byref(o), C.byref(u), C.byref(rep), 24680, 1 << 20, None)

    # x0 whose packed size exceeds its capacity
    x0 = P._lib._TT(D, nrow, None, (C.c_int32 * (D + 1))(1, 2, 2, 2, 2, 1), 32768, 8)
    assert solve(x0) == -3 and b"x0" in L.qtt_last_error()
    # x0 with other modes than K
    nrow3 = (C.c_int32 * D)(*([3] * D))
    x0 = P._lib._TT(D, nrow3, None, (C.c_int32 * (D + 1))(1, 2, 2, 2, 2, 1), 32768, 1 << 20)
    assert solve(x0) == -2 and b"modes" in L.qtt_last_error()
    # x0 with a boundary rank other than 1
    x0 = P._lib._TT(D, nrow, None, (C.c_int32 * (D + 1))(2, 2, 2, 2, 2, 1), 32768, 1 << 20)
    assert solve(x0) == -2 and b"boundary" in L.qtt_last_error()
    # K whose capacity is below its packed size
    K.capacity = 10
    assert solve(None) == -3 and b"K" in L.qtt_last_error()


def test_graph_create_validates_on_the_host():
    """qtt_matvec_round_graph_create refuses bad arguments, an output whose
    capacity is below the ranks the rounding may leave, and a branch
    workspace that is too small, before it creates a stream or captures."""
    if not os.path.exists(LIB):
        pytest.skip("libqtt.so not built")
    import paper_2501_07778_amd as P
    L = P.lib()
    T = P._lib._TT
    D = 3
    nrow = (C.c_int32 * D)(2, 2, 2)
    ncol = (C.c_int32 * D)(2, 2, 2)
    ra = (C.c_int32 * (D + 1))(1, 3, 3, 1)
    rx = (C.c_int32 * (D + 1))(1, 2, 2, 1)
    ry = (C.c_int32 * (D + 1))(1, 1, 1, 1)
    A = T(D, nrow, ncol, ra, 4096, 3 * 4 + 9 * 4 + 3 * 4)
    x = T(D, nrow, None, rx, 8192, 2 * 2 + 4 * 2 + 2 * 2)
    y = T(D, nrow, None, ry, 12288, 6 * 2 + 36 * 2 + 6 * 2)   # product ranks 6: enough
    case = (P._lib._MVRCase * 1)()
    case[0].A, case[0].x, case[0].y = C.pointer(A), C.pointer(x), C.pointer(y)
    case[0].compute, case[0].ell, case[0].seed, case[0].eps, case[0].rmax = 0, 0, 1, 1e-8, 0
    need = C.c_size_t()
    assert L.qtt_matvec_round_workspace(C.byref(A), C.byref(x), 0, C.byref(need)) == 0
    ws = (C.c_void_p * 1)(1 << 20)          # never dereferenced: validation fails first
    wsb = (C.c_size_t * 1)(need.value)
    aux_n = C.c_size_t()
    assert L.qtt_matvec_round_graph_aux_bytes(1, C.byref(aux_n)) == 0 and aux_n.value > 0
    h = C.c_void_p()
    create = L.qtt_matvec_round_graph_create
    assert create(0, case, 1, ws, wsb, 1 << 21, aux_n.value, 0, C.byref(h)) == -1
    assert create(1, case, 0, ws, wsb, 1 << 21, aux_n.value, 0, C.byref(h)) == -1
    assert create(1, case, 1, ws, wsb, 1 << 21, aux_n.value, 2, C.byref(h)) == -1
    assert create(1, case, 1, ws, wsb, None, aux_n.value, 0, C.byref(h)) == -3
    assert create(1, case, 1, ws, wsb, (1 << 21) + 8, aux_n.value, 0, C.byref(h)) == -3
    y.capacity = 6 * 2 + 36 * 2 + 6 * 2 - 1
    assert create(1, case, 1, ws, wsb, 1 << 21, aux_n.value, 0, C.byref(h)) == -3
    assert b"capacity" in L.qtt_last_error()
    y.capacity += 1
    wsb[0] = need.value // 2
    assert create(1, case, 1, ws, wsb, 1 << 21, aux_n.value, 0, C.byref(h)) == -3
    assert b"branch workspace" in L.qtt_last_error()
    assert not h.value
    assert L.qtt_matvec_round_graph_destroy(None) == 0
