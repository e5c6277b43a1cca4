"""The C-ABI library without a GPU: it loads, exports every function declared in
include/tkmi.h, validates arguments before touching the device, and answers
workspace-size queries.  No compute call is made here."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tkmi.h")

from paper_2603_21379_amd import binding as B  # noqa: E402

FAKE = 0x10000  # a non-NULL address; never dereferenced by validation or size queries


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\(", text, flags=re.M)))


def test_library_exports_every_declared_function():
    L = B.lib()
    names = declared_functions()
    assert "tucker_sketch_all_modes" in names and "htucker_decompose" in names
    for n in names:
        assert hasattr(L, n), n
    assert set(B.EXPORTS) <= set(names)
    assert B.version().startswith("tkmi")


def _tensor(dims, dtype=B.TK_F32, data=FAKE):
    t = B.TkTensor()
    t.order = len(dims)
    t.dtype = dtype
    for k, n in enumerate(dims):
        t.dims[k] = n
    t.data = data
    return t


def _sk(s, ell, idx=FAKE, om=FAKE, reserved=0):
    k = B.TkSketch()
    k.s, k.ell, k.reserved, k.idx, k.omega = s, ell, reserved, idx, om
    return k


def _query(fn, *args):
    n = C.c_size_t(0)
    st = getattr(B.lib(), fn)(*args, None, C.byref(n), None)
    return st, n.value, B.lib().tk_last_error().decode()


def _ptrs(n):
    return (C.c_void_p * n)(*([FAKE] * n))


def test_sketch_validation_and_query():
    X = _tensor((8, 9, 10))
    sks = (B.TkSketch * 3)(_sk(20, 5), _sk(30, 5), _sk(40, 5))
    st, n, _ = _query("tucker_sketch_all_modes", C.byref(X), sks, _ptrs(3), None)
    assert st == 0 and n > 0
    # ell > s
    bad = (B.TkSketch * 3)(_sk(4, 5), _sk(30, 5), _sk(40, 5))
    st, _, msg = _query("tucker_sketch_all_modes", C.byref(X), bad, _ptrs(3), None)
    assert st == 1 and "mode 0" in msg
    # s larger than the number of columns (9*10 = 90)
    bad = (B.TkSketch * 3)(_sk(91, 5), _sk(30, 5), _sk(40, 5))
    assert _query("tucker_sketch_all_modes", C.byref(X), bad, _ptrs(3), None)[0] == 1
    # dense sketch must sample every column
    bad = (B.TkSketch * 3)(_sk(50, 5, idx=None), _sk(30, 5), _sk(40, 5))
    assert _query("tucker_sketch_all_modes", C.byref(X), bad, _ptrs(3), None)[0] == 1
    ok = (B.TkSketch * 3)(_sk(90, 5, idx=None), _sk(30, 5), _sk(40, 5))
    assert _query("tucker_sketch_all_modes", C.byref(X), ok, _ptrs(3), None)[0] == 0
    # reserved field, NULL omega, ell beyond the rows, NULL data
    assert _query("tucker_sketch_all_modes", C.byref(X),
                  (B.TkSketch * 3)(_sk(20, 5, reserved=1), _sk(30, 5), _sk(40, 5)), _ptrs(3), None)[0] == 1
    assert _query("tucker_sketch_all_modes", C.byref(X),
                  (B.TkSketch * 3)(_sk(20, 5, om=None), _sk(30, 5), _sk(40, 5)), _ptrs(3), None)[0] == 1
    assert _query("tucker_sketch_all_modes", C.byref(X),
                  (B.TkSketch * 3)(_sk(20, 9), _sk(30, 5), _sk(40, 5)), _ptrs(3), None)[0] == 1
    X0 = _tensor((8, 9, 10), data=None)
    assert _query("tucker_sketch_all_modes", C.byref(X0), sks, _ptrs(3), None)[0] == 1
    # widths above 64 take the wide QR path (up to 192); beyond it: unsupported
    big = _tensor((100, 100))
    assert _query("tucker_sketch_all_modes", C.byref(big),
                  (B.TkSketch * 2)(_sk(100, 65), _sk(100, 5)), _ptrs(2), None)[0] == 0
    huge = _tensor((200, 200))
    assert _query("tucker_sketch_all_modes", C.byref(huge),
                  (B.TkSketch * 2)(_sk(200, 193), _sk(100, 5)), _ptrs(2), None)[0] == 5


def test_noalloc_sketch_validates_and_rejects_oversize_before_launch():
    """The no-allocation sketch shares the workspace entry point's validation,
    and a call whose partial sketches exceed the fixed 64 MiB scratch is
    refused on the host (nothing enqueued, no device touched)."""
    L = B.lib()
    X = _tensor((8, 9, 10))
    bad = (B.TkSketch * 3)(_sk(4, 5), _sk(30, 5), _sk(40, 5))
    assert L.tucker_sketch_all_modes_noalloc(C.byref(X), bad, _ptrs(3), None, None) == 1
    # 33 chunks of 32 fibers x 4096 rows x 64 columns of FP64 partials > 64 MiB
    big = _tensor((4096, 2048))
    sks = (B.TkSketch * 2)(_sk(1056, 64), _sk(1056, 64))
    st = L.tucker_sketch_all_modes_noalloc(C.byref(big), sks, _ptrs(2), None, None)
    assert st == 5 and "fixed" in L.tk_last_error().decode()


def test_projection_loss_vjp_validation_and_query():
    """The projection-loss backward answers its size query without a GPU;
    without an X output its workspace also holds the X-sized adjoint; a call
    with no output or an unsupported dtype is refused."""
    L = B.lib()
    dims, cols_ = (16, 20, 40, 132), (4, 5, 31, 32)
    X = _tensor(dims)
    cols = (C.c_int32 * 4)(*cols_)
    F = _ptrs(4)
    n1, n2 = C.c_size_t(0), C.c_size_t(0)
    assert L.tucker_projection_loss_vjp(C.byref(X), F, cols, C.c_void_p(FAKE), None, C.c_void_p(FAKE), F,
                                        None, C.byref(n1), None) == 0
    assert L.tucker_projection_loss_vjp(C.byref(X), F, cols, C.c_void_p(FAKE), None, None, F,
                                        None, C.byref(n2), None) == 0
    assert n2.value >= n1.value + 16 * 20 * 40 * 132 * 4
    assert L.tucker_projection_loss_vjp(C.byref(X), F, cols, C.c_void_p(FAKE), None, None, None,
                                        None, C.byref(n1), None) == 1
    Xb = _tensor(dims, dtype=B.TK_BF16)
    assert L.tucker_projection_loss_vjp(C.byref(Xb), F, cols, C.c_void_p(FAKE), None, C.c_void_p(FAKE), F,
                                        None, C.byref(n1), None) == 5


def test_workspace_too_small_is_rejected_before_launch():
    X = _tensor((8, 9, 10))
    sks = (B.TkSketch * 3)(_sk(20, 5), _sk(30, 5), _sk(40, 5))
    n = C.c_size_t(16)
    st = B.lib().tucker_sketch_all_modes(C.byref(X), sks, _ptrs(3), None, C.c_void_p(FAKE),
                                          C.byref(n), None)
    assert st == 2 and "workspace" in B.lib().tk_last_error().decode()


def test_qr_validation():
    m = (C.c_int64 * 2)(10, 20)
    ell = (C.c_int32 * 2)(4, 25)
    st, _, msg = _query("tucker_qr", 2, m, ell, _ptrs(2), None, 0, None, None, None, 0, None)
    assert st == 1 and "ell[1]" in msg
    ell = (C.c_int32 * 2)(4, 5)
    st, n, _ = _query("tucker_qr", 2, m, ell, _ptrs(2), None, 0, None, None, None, 0, None)
    assert st == 0 and n > 0
    s = (C.c_int64 * 2)(30, 40)
    r = (C.c_int32 * 2)(4, 6)
    st, _, msg = _query("tucker_qr", 2, m, ell, _ptrs(2), _ptrs(2), B.TK_F32, s, r, _ptrs(2),
                        B.TK_F32, None)
    assert st == 1 and "r[1]" in msg
    r = (C.c_int32 * 2)(4, 5)
    assert _query("tucker_qr", 2, m, ell, _ptrs(2), _ptrs(2), B.TK_F32, s, r, _ptrs(2), B.TK_BF16,
                  None)[0] == 1
    assert _query("tucker_qr", 2, m, ell, _ptrs(2), _ptrs(2), B.TK_F32, s, r, _ptrs(2), B.TK_F32,
                  None)[0] == 0
    assert _query("tucker_qr", -1, m, ell, _ptrs(2), None, 0, None, None, None, 0, None)[0] == 1
    # a wide sketch (ell = 160 of 270 rows, s = 2700) next to a narrow one: the
    # wide plan holds its own Gram partials, M^T (s x ell), the Jacobi matrix,
    # V and the rotations of a sweep on top of the narrow plan
    m = (C.c_int64 * 2)(270, 20)
    s = (C.c_int64 * 2)(2700, 40)
    r = (C.c_int32 * 2)(150, 5)
    ell = (C.c_int32 * 2)(160, 5)
    st, n_wide, _ = _query("tucker_qr", 2, m, ell, _ptrs(2), _ptrs(2), B.TK_F32, s, r, _ptrs(2),
                           B.TK_F32, None)
    assert st == 0 and n_wide > 8 * (2700 * 160 + 3 * 160 * 160)
    ell = (C.c_int32 * 2)(193, 5)
    st, _, msg = _query("tucker_qr", 2, m, ell, _ptrs(2), _ptrs(2), B.TK_F32, s, r, _ptrs(2),
                        B.TK_F32, None)
    assert st == 5 and "ell[0]" in msg


def test_core_and_reconstruct_validation():
    X = _tensor((8, 9, 10))
    cols = (C.c_int32 * 3)(3, 4, 5)
    st, n, _ = _query("tucker_core", C.byref(X), _ptrs(3), cols, C.c_void_p(FAKE))
    assert st == 0 and n > 0
    bad = (C.c_int32 * 3)(3, 10, 5)
    st, _, msg = _query("tucker_core", C.byref(X), _ptrs(3), bad, C.c_void_p(FAKE))
    assert st == 1 and "cols[1]" in msg
    F = _ptrs(3)
    F[2] = None
    assert _query("tucker_core", C.byref(X), F, cols, C.c_void_p(FAKE))[0] == 1
    assert _query("tucker_core", C.byref(X), _ptrs(3), cols, None)[0] == 1
    dims = (C.c_int64 * 3)(8, 9, 10)
    # neither output requested
    assert _query("tucker_reconstruct", 3, dims, B.TK_F32, C.c_void_p(FAKE), _ptrs(3), cols, None,
                  None, None)[0] == 1
    # residual without reference
    assert _query("tucker_reconstruct", 3, dims, B.TK_F32, C.c_void_p(FAKE), _ptrs(3), cols, None,
                  None, C.c_void_p(FAKE))[0] == 1
    # factor dtype mismatch with the reference
    X64 = _tensor((8, 9, 10), dtype=B.TK_F64)
    assert _query("tucker_reconstruct", 3, dims, B.TK_F32, C.c_void_p(FAKE), _ptrs(3), cols,
                  C.byref(X64), None, C.c_void_p(FAKE))[0] == 1
    st, n, _ = _query("tucker_reconstruct", 3, dims, B.TK_F32, C.c_void_p(FAKE), _ptrs(3), cols,
                      C.byref(X), None, C.c_void_p(FAKE))
    assert st == 0 and n > 0


def test_htucker_validation():
    import synthgen
    X = _tensor((4, 4, 4, 4))
    tr = synthgen.balanced_tree(4)
    td = B.tree_desc(tr)
    nn = tr.num_nodes
    rk = (C.c_int32 * nn)(*([0] + [2] * (nn - 1)))
    sks = (B.TkSketch * nn)(*([_sk(1, 1)] + [_sk(8, 3)] * (nn - 1)))
    st, n, msg = _query("htucker_decompose", C.byref(X), C.byref(td), rk, sks, _ptrs(nn), _ptrs(nn),
                        None)
    assert st == 0 and n > 0, msg
    # a tree that is not the balanced heap tree
    tr.left[0], tr.right[0] = tr.right[0], tr.left[0]
    td2 = B.tree_desc(tr)
    st, _, msg = _query("htucker_decompose", C.byref(X), C.byref(td2), rk, sks, _ptrs(nn), _ptrs(nn),
                        None)
    assert st == 1 and "balanced" in msg
    # rank above ell
    rk2 = (C.c_int32 * nn)(*([0] + [4] * (nn - 1)))
    assert _query("htucker_decompose", C.byref(X), C.byref(td), rk2, sks, _ptrs(nn), _ptrs(nn),
                  None)[0] == 1


def test_status_codes_in_header_match_binding():
    text = open(HEADER).read()
    for code, name in B.STATUS.items():
        assert re.search(rf"\b{name}\s*=\s*{code}\b", text), name


def test_info_bits_in_header_match_binding():
    """Every bit of the device info words, the eigensolver's non-convergence
    bit included, is defined in the header with the binding's value."""
    text = open(HEADER).read()
    for bit, name in B.INFO_BITS.items():
        assert re.search(rf"#define\s+{name}\s+{bit}\b", text), name
    assert sorted(B.INFO_BITS) == [1, 2, 4, 8]


def test_batch_plan_validation_and_query():
    L = B.lib()
    f = L.tucker_batch_plan_create
    dims = (20, 30, 40)
    X = (B.TkTensor * 1)()
    X[0] = _tensor(dims)
    ranks = (C.c_int32 * 3)(3, 4, 5)
    sk = (B.TkSketch * 3)()
    for k, n in enumerate(dims):
        sk[k].s = 10 * n
        sk[k].ell = ranks[k] + 5
        sk[k].idx = FAKE
        sk[k].omega = FAKE
    U = (C.c_void_p * 3)(FAKE, FAKE, FAKE)
    G = (C.c_void_p * 1)(FAKE)
    n = C.c_size_t(0)
    assert f(1, X, ranks, sk, U, G, None, None, None, C.byref(n), None, None) == 0
    assert n.value > 0
    # the residual's tables (expansion steps, its chunk schedule) add to the workspace
    n_r = C.c_size_t(0)
    assert f(1, X, ranks, sk, U, G, None, C.c_void_p(FAKE), None, C.byref(n_r), None, None) == 0
    assert n_r.value > n.value
    # FP64 tensors, order 2 and wide trailing modes are outside the batch form
    X[0] = _tensor(dims, dtype=B.TK_F64)
    assert f(1, X, ranks, sk, U, G, None, None, None, C.byref(n), None, None) == 5
    X[0] = _tensor((20, 300, 40))
    assert f(1, X, ranks, sk, U, G, None, None, None, C.byref(n), None, None) == 5
    X[0] = _tensor(dims)
    ranks[2] = 11    # above ell
    assert f(1, X, ranks, sk, U, G, None, None, None, C.byref(n), None, None) == 1
    ranks[2] = 5
    G[0] = None
    assert f(1, X, ranks, sk, U, G, None, None, None, C.byref(n), None, None) == 1
    assert f(0, X, ranks, sk, U, G, None, None, None, C.byref(n), None, None) == 1


def test_batch_schedule_entry_points_validate():
    L = B.lib()
    a, b, c = C.c_int32(0), C.c_int32(0), C.c_int64(0)
    assert L.tucker_batch_get_schedule(None, C.byref(a), C.byref(b), C.byref(c)) == 1
    assert L.tucker_batch_set_schedule(None, 1, 2, 1 << 20, None) == 1


def test_batch_shape_class_key():
    """Stored schedules are keyed by the multiset of per-tensor classes: the
    order of the tensors does not matter, a size in another 16-wide bucket
    does."""
    dims = [(20, 30, 40), (16, 16, 16, 16), (50, 60, 70)]
    ells = [8, 9, 10, 6, 6, 6, 6, 12, 12, 13]
    k1 = B.batch_shape_class(dims, ells)
    k2 = B.batch_shape_class([dims[2], dims[0], dims[1]], ells[7:] + ells[:3] + ells[3:7])
    assert k1 == k2 and k1.startswith("n3-")
    assert B.batch_shape_class([(20, 30, 41)] + dims[1:], ells) == k1     # same buckets
    assert B.batch_shape_class([(20, 30, 49)] + dims[1:], ells) != k1     # trailing size bucket
    assert B.batch_shape_class(dims, [8, 9, 17] + ells[3:]) != k1        # sketch width bucket


def _ht_args(dims, rank_of):
    import synthgen
    tr = synthgen.balanced_tree(len(dims))
    nn = tr.num_nodes
    td = B.tree_desc(tr)
    rk = (C.c_int32 * nn)(*([0] + [rank_of(t) for t in range(1, nn)]))
    dd = (C.c_int64 * len(dims))(*dims)
    return tr, td, rk, dd, nn


def test_htucker_reconstruct_validation_and_query():
    dims = (5, 6, 4, 7)
    tr, td, rk, dd, nn = _ht_args(dims, lambda t: 2)
    X = _tensor(dims)
    ok = _query("htucker_reconstruct", 4, dd, C.byref(td), rk, _ptrs(nn), _ptrs(nn), C.byref(X),
                C.c_void_p(FAKE), B.TK_F32, C.c_void_p(FAKE))
    assert ok[0] == 0 and ok[1] > 0, ok[2]
    # neither output; a residual without a reference; an output dtype other than F32/F64
    assert _query("htucker_reconstruct", 4, dd, C.byref(td), rk, _ptrs(nn), _ptrs(nn), C.byref(X),
                  None, 0, None)[0] == 1
    assert _query("htucker_reconstruct", 4, dd, C.byref(td), rk, _ptrs(nn), _ptrs(nn), None,
                  None, 0, C.c_void_p(FAKE))[0] == 1
    assert _query("htucker_reconstruct", 4, dd, C.byref(td), rk, _ptrs(nn), _ptrs(nn), None,
                  C.c_void_p(FAKE), B.TK_BF16, None)[0] == 1
    # a reference of other dims
    X2 = _tensor((5, 6, 4, 8))
    assert _query("htucker_reconstruct", 4, dd, C.byref(td), rk, _ptrs(nn), _ptrs(nn), C.byref(X2),
                  None, 0, C.c_void_p(FAKE))[0] == 1
    # a missing leaf basis
    U = _ptrs(nn)
    U[nn - 1] = None
    st, _, msg = _query("htucker_reconstruct", 4, dd, C.byref(td), rk, U, _ptrs(nn), None,
                        C.c_void_p(FAKE), B.TK_F64, None)
    assert st == 1 and "leaf" in msg
    # the rank of the root's right child above 64
    rk2 = (C.c_int32 * nn)(*rk)
    rk2[tr.right[0]] = 65
    assert _query("htucker_reconstruct", 4, dd, C.byref(td), rk2, _ptrs(nn), _ptrs(nn), None,
                  C.c_void_p(FAKE), B.TK_F64, None)[0] == 5
    # a tree that is not the balanced heap tree
    tr.left[0], tr.right[0] = tr.right[0], tr.left[0]
    td2 = B.tree_desc(tr)
    st, _, msg = _query("htucker_reconstruct", 4, dd, C.byref(td2), rk, _ptrs(nn), _ptrs(nn), None,
                        C.c_void_p(FAKE), B.TK_F64, None)
    assert st == 1 and "balanced" in msg


def test_htucker_reconstruct_vjp_validation_and_query():
    dims = (5, 6, 4, 7, 3)
    tr, td, rk, dd, nn = _ht_args(dims, lambda t: 3)
    ok = _query("htucker_reconstruct_vjp", 5, dd, C.byref(td), rk, _ptrs(nn), _ptrs(nn),
                C.c_void_p(FAKE), B.TK_F32, _ptrs(nn), _ptrs(nn))
    assert ok[0] == 0 and ok[1] > 0, ok[2]
    assert _query("htucker_reconstruct_vjp", 5, dd, C.byref(td), rk, _ptrs(nn), _ptrs(nn),
                  C.c_void_p(FAKE), B.TK_F16, _ptrs(nn), _ptrs(nn))[0] == 1
    assert _query("htucker_reconstruct_vjp", 5, dd, C.byref(td), rk, _ptrs(nn), _ptrs(nn),
                  None, B.TK_F32, _ptrs(nn), _ptrs(nn))[0] == 1
    Bb = _ptrs(nn)
    Bb[0] = None
    st, _, msg = _query("htucker_reconstruct_vjp", 5, dd, C.byref(td), rk, _ptrs(nn), _ptrs(nn),
                        C.c_void_p(FAKE), B.TK_F32, Bb, _ptrs(nn))
    assert st == 1 and "Bbar[0]" in msg


def test_htucker_dense_root_children_need_no_unfolding_copy():
    """Every column of the root's children sampled (idx NULL): the workspace
    holds no copy of those unfoldings, so it is far smaller than the same
    call with the columns listed explicitly (which gathers them)."""
    import synthgen
    dims = (30, 30, 30, 30)
    tr = synthgen.balanced_tree(4)
    nn = tr.num_nodes
    td = B.tree_desc(tr)
    X = _tensor(dims)
    rk = (C.c_int32 * nn)(*([0] + [3] * (nn - 1)))
    ncols = {t: 30 ** 4 // 30 ** tr.count[t] for t in range(1, nn)}

    def sketches(dense_idx):
        return (B.TkSketch * nn)(*([_sk(1, 1)] + [
            _sk(ncols[t], 5, idx=dense_idx) if t in (1, 2) else _sk(60, 5) for t in range(1, nn)]))
    st_d, n_dense, msg = _query("htucker_decompose", C.byref(X), C.byref(td), rk, sketches(None),
                                _ptrs(nn), _ptrs(nn), None)
    st_g, n_gather, _ = _query("htucker_decompose", C.byref(X), C.byref(td), rk, sketches(FAKE),
                               _ptrs(nn), _ptrs(nn), None)
    assert st_d == 0 and st_g == 0, msg
    # the gathered form stores the two 900 x 900 FP32 unfoldings; the dense
    # form's own buffers (products with X, split partials) are much smaller
    assert n_gather - n_dense >= 2 * 900 * 900 * 4 * 0.8


def test_draw_sketches_rejects_bad_arguments_before_launch():
    L = B.lib()
    i64 = lambda *v: (C.c_int64 * len(v))(*v)  # noqa: E731
    i32 = lambda *v: (C.c_int32 * len(v))(*v)  # noqa: E731
    pp = (C.c_void_p * 1)(FAKE)
    ip = C.cast(pp, C.POINTER(C.c_void_p))
    cases = [
        (0, i64(10), i32(5), i32(2), B.TK_F64),        # no units
        (1, i64(10), i32(11), i32(2), B.TK_F64),       # s > ncols
        (1, i64(10 ** 6), i32(4097), i32(2), B.TK_F64),  # s above the draw limit
        (1, i64(10), i32(5), i32(0), B.TK_F64),        # ell < 1
        (1, i64(10), i32(5), i32(2), B.TK_BF16),       # Omega dtype
    ]
    for n, nc, s, ell, dt in cases:
        assert L.tucker_draw_sketches(n, nc, s, ell, 1, pp, pp, dt, None) == 1
    null = (C.c_void_p * 1)(None)
    assert L.tucker_draw_sketches(1, i64(10), i32(5), i32(2), 1, null, pp, B.TK_F64, None) == 1
    del ip
