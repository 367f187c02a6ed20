"""Python binding of libbmm.so: exact packed bit-matrix products on MI355X.

Argument marshalling only: every step of every product runs in the HIP
kernels of ``libbmm.so``.  Importing this package raises if the library is
not built; there is no CPU fallback.

Matrices are torch.int64 CUDA tensors holding packed rows (shape rows x ld,
bit j of a row at bit j % 64 of word j // 64).  Calls are asynchronous on the
tensor device's current stream.  The names mirror the C entry points declared
in ``include/bmm.h``.
"""
import ctypes
import os

from . import build as _build

__all__ = [
    "BmmError", "Options", "GF2", "BOOLEAN", "LEAF_AUTO", "LEAF_VALU", "LEAF_MFMA_I8",
    "LEAF_MFMA_F4",
    "FLAG_ACCUMULATE", "FLAG_B_TRANSPOSED", "FLAG_ALT_BASIS_IO", "FLAG_HOST_OPERANDS",
    "FLAG_OOC_BLOCK_ORDER",
    "SCHEME_SELF_INVERSE", "SCHEME_CHAINING", "SCHEME_WINOGRAD",
    "words", "bmm_gf2", "bmm_boolean", "bmm_gf2_strassen", "bmm_gf2_strassen_workspace",
    "bmm_batched", "BatchedPlan", "bmm_transpose", "bmm_basis_change", "bmm_expand",
    "bmm_compress", "bmm_ooc", "bmm_autotune_cubic", "bmm_autotune_leaf",
    "bmm_autotune_strassen", "bmm_autotune_set", "bmm_autotune_batched", "bmm_autotune_save",
    "bmm_autotune_load", "bmm_leaf_tiles", "bmm_leaf_tile_shape", "bmm_leaf_choice", "bmm_version",
    "bmm_finalize", "library_path", "bmm_calibrate_valu", "bmm_cubic_noalloc",
    "bmm_ooc_last_transfers", "bmm_debug_fail_allocations",
]

GF2, BOOLEAN = 0, 1
LEAF_AUTO, LEAF_VALU, LEAF_MFMA_I8, LEAF_MFMA_F4 = 0, 1, 2, 3
FLAG_ACCUMULATE = 0x1
FLAG_B_TRANSPOSED = 0x2
FLAG_ALT_BASIS_IO = 0x4
FLAG_HOST_OPERANDS = 0x8
FLAG_OOC_BLOCK_ORDER = 0x10
FLAG_INPLACE_BASIS = 0x20
FLAG_LEAN_WORKSPACE = 0x40
SCHEME_SELF_INVERSE, SCHEME_CHAINING, SCHEME_WINOGRAD = 0, 1, 2

_STATUS = {0: "ok", -1: "invalid argument", -2: "unsupported", -3: "workspace too small",
           -4: "out of memory", -5: "device error"}


class BmmError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{_STATUS.get(status, status)}: {message}")
        self.status = status


# BMM_LIBRARY names another build of the library (the host-only sanitized build of
# build_sanitized.py, for CPU tests of the host logic); the default is the product build.
_SO = os.environ.get("BMM_LIBRARY") or _build.SO


def library_path():
    return _SO


if not os.path.exists(_SO):
    raise ImportError(f"{_SO} is not built; run __graft_entry__.build() "
                      "(python -m paper_1909_01554_amd.build)")

_lib = ctypes.CDLL(_SO)
_i64 = ctypes.c_int64
_vp = ctypes.c_void_p
_int = ctypes.c_int


class Options(ctypes.Structure):
    """bmm_options: leaf, tile, depth_serial, depth_parallel, block, flags, scheme, shift,
    k_panel."""
    _fields_ = [("leaf", _int), ("tile", _int), ("depth_serial", _int),
                ("depth_parallel", _int), ("block", _i64), ("flags", ctypes.c_uint32),
                ("scheme", _int), ("shift", _int), ("k_panel", _i64)]

    def __init__(self, leaf=LEAF_AUTO, tile=0, depth_serial=-1, depth_parallel=-1, block=0,
                 flags=0, scheme=0, shift=-1, k_panel=0):
        super().__init__(leaf, tile, depth_serial, depth_parallel, block, flags, scheme, shift,
                         k_panel)


class Problem(ctypes.Structure):
    _fields_ = [("semiring", _int), ("m", _i64), ("k", _i64), ("n", _i64), ("A", _vp),
                ("B", _vp), ("C", _vp), ("lda", _i64), ("ldb", _i64), ("ldc", _i64),
                ("b_transposed", _int)]


def _sig(name, args, res=_int):
    f = getattr(_lib, name)
    f.argtypes = args
    f.restype = res
    return f


_prod_args = [_vp, _i64, _vp, _i64, _vp, _i64, _i64, _i64, _i64, ctypes.POINTER(Options), _vp]
_c_gf2 = _sig("bmm_gf2", _prod_args)
_c_boolean = _sig("bmm_boolean", _prod_args)
_c_noalloc = _sig("bmm_cubic_noalloc", [_int] + _prod_args)
NOALLOC_SCRATCH_BYTES = 32 << 20  # BMM_NOALLOC_SCRATCH_BYTES
_c_strassen = _sig("bmm_gf2_strassen", [_vp, _i64, _vp, _i64, _vp, _i64, _i64, _i64, _i64, _int,
                                        _vp, ctypes.c_size_t, ctypes.POINTER(Options), _vp])
_c_strassen_ws = _sig("bmm_gf2_strassen_workspace",
                      [_i64, _i64, _i64, _int, ctypes.POINTER(Options),
                       ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(_int),
                       ctypes.POINTER(_int)])
_c_batched = _sig("bmm_batched", [ctypes.POINTER(Problem), _i64, ctypes.POINTER(Options), _vp])
_c_leaf_choice = _sig("bmm_leaf_choice", [_int, _i64, _i64, _i64, _i64, ctypes.POINTER(Options),
                                          ctypes.POINTER(_int), ctypes.POINTER(_int)])
_c_tune_batched = _sig("bmm_autotune_batched", [ctypes.POINTER(Problem), _i64,
                                                ctypes.POINTER(_int), ctypes.POINTER(_int),
                                                ctypes.POINTER(ctypes.c_double)])
_c_plan_create = _sig("bmm_batched_plan_create", [ctypes.POINTER(Problem), _i64,
                                                  ctypes.POINTER(Options), ctypes.POINTER(_vp)])
_c_plan_launch = _sig("bmm_batched_plan_launch", [_vp, _vp])
_c_plan_destroy = _sig("bmm_batched_plan_destroy", [_vp], None)
_c_transpose = _sig("bmm_transpose", [_vp, _i64, _vp, _i64, _i64, _i64, _vp])
_c_basis = _sig("bmm_basis_change", [_vp, _i64, _i64, _i64, _int, _int, _int, _int, _vp])
_c_expand = _sig("bmm_expand", [_int, _int, _int, _vp, _i64, _i64, _vp, _i64, _i64, _i64, _vp])
_c_compress = _sig("bmm_compress", [_int, _int, _vp, _vp, _i64, _i64, _i64, _i64, _i64, _vp])
_c_ooc = _sig("bmm_ooc", [_int, _vp, _i64, _vp, _i64, _vp, _i64, _i64, _i64, _i64, _i64,
                          ctypes.POINTER(Options), ctypes.POINTER(ctypes.c_double)])
_c_tune = _sig("bmm_autotune_cubic", [_int, _i64, _i64, _i64, ctypes.POINTER(_int),
                                      ctypes.POINTER(_int), ctypes.POINTER(ctypes.c_double)])
_c_tune_set = _sig("bmm_autotune_set", [_int, _i64, _i64, _i64, _i64, _int, _int])
_c_tune_leaf = _sig("bmm_autotune_leaf", [_int, _i64, _i64, _i64, _i64, ctypes.POINTER(_int),
                                          ctypes.POINTER(_int), ctypes.POINTER(ctypes.c_double)])
_c_tune_strassen = _sig("bmm_autotune_strassen",
                        [_vp, _i64, _vp, _i64, _vp, _i64, _i64, _i64, _i64, _vp,
                         ctypes.c_size_t, ctypes.POINTER(Options), ctypes.POINTER(_int),
                         ctypes.POINTER(_int), ctypes.POINTER(_int),
                         ctypes.POINTER(ctypes.c_double)])
_c_tune_kpanel = _sig("bmm_autotune_k_panel",
                      [_int, _vp, _i64, _vp, _i64, _vp, _i64, _i64, _i64, _i64,
                       ctypes.POINTER(Options), ctypes.POINTER(_i64), _int, ctypes.POINTER(_i64),
                       ctypes.POINTER(ctypes.c_double)])
_c_tune_save = _sig("bmm_autotune_save", [ctypes.c_char_p])
_c_tune_load = _sig("bmm_autotune_load", [ctypes.c_char_p])
_c_tiles = _sig("bmm_leaf_tiles", [_int, ctypes.POINTER(_int)])
_c_tile_shape = _sig("bmm_leaf_tile_shape", [_int, _int, ctypes.POINTER(_int),
                                             ctypes.POINTER(_int)])
_c_calib = _sig("bmm_calibrate_valu", [_int, _i64] + [ctypes.POINTER(ctypes.c_double)] * 4)
_c_ooc_xfer = _sig("bmm_ooc_last_transfers", [ctypes.POINTER(ctypes.c_double)] * 4)
_c_fail_allocs = _sig("bmm_debug_fail_allocations", [_i64])
_c_last_error = _sig("bmm_last_error", [], ctypes.c_char_p)
_c_version = _sig("bmm_version", [], ctypes.c_char_p)
_c_finalize = _sig("bmm_finalize", [], None)


def _check(rc):
    if rc != 0:
        raise BmmError(rc, _c_last_error().decode(errors="replace"))


def words(bits):
    return (int(bits) + 63) // 64


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(t, stream):
    if stream is not None:
        return ctypes.c_void_p(int(stream))
    import torch
    if not t.is_cuda:  # host operands: the current device's current stream
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return ctypes.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def _ld(t):
    if t.dim() != 2 or t.stride(1) != 1:
        raise ValueError("matrices must be 2-D with contiguous rows")
    return t.stride(0)


def _is_tensor(t):
    try:
        import torch
    except ImportError:
        return False
    return isinstance(t, torch.Tensor)


def _span(t):
    """64-bit words addressable from t.data_ptr() to the end of its storage."""
    return t.untyped_storage().nbytes() // 8 - t.storage_offset()


def _mat(t, name, rows, cols_bits, device=True):
    """Check a packed matrix operand before its pointer crosses the C ABI: an
    8-byte integer tensor, 2-D with contiguous rows, at least rows x
    words(cols_bits) words, on a GPU (device=False: page-locked host memory).
    The library sees only a pointer and a pitch, so a tensor smaller than the
    sizes claim would otherwise be read or written out of bounds."""
    if not _is_tensor(t):
        raise TypeError(f"{name} must be a torch tensor")
    if t.element_size() != 8 or t.is_floating_point() or t.is_complex():
        raise ValueError(f"{name} must hold 64-bit words (torch.int64 or torch.uint64), "
                         f"not {t.dtype}")
    if t.dim() != 2 or t.stride(1) != 1:
        raise ValueError(f"{name} must be 2-D with contiguous rows")
    if rows > 0 and cols_bits > 0:
        if t.shape[0] < rows or t.shape[1] < words(cols_bits):
            raise ValueError(f"{name} has shape {tuple(t.shape)}; the sizes need at least "
                             f"{rows} x {words(cols_bits)} words")
    if device is True and not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if device is False and t.is_cuda:
        raise ValueError(f"{name} must be in (page-locked) host memory")
    return t


def _sizes(m, k, n):
    for v, nm in ((m, "m"), (k, "k"), (n, "n")):
        if int(v) < 0:
            raise ValueError(f"{nm} = {v} is negative")


def _operands(A, B, C, m, k, n, b_transposed, device=True):
    """Shapes and types of all three operands first, then where they live."""
    _sizes(m, k, n)
    mats = [(C, "C", m, n)]
    if m > 0 and n > 0 and k > 0:
        mats = [(A, "A", m, k), (B, "B (transposed)", n, k) if b_transposed else
                (B, "B", k, n)] + mats
    for t, name, r, c in mats:
        _mat(t, name, r, c, device=None)
    for t, name, r, c in mats:
        _mat(t, name, r, c, device=device)


def _opts(options, flags):
    o = Options()
    if options is not None:
        for name, _ in Options._fields_:
            setattr(o, name, getattr(options, name))
    o.flags |= flags
    return o


def _product(fn, A, B, C, m, k, n, options, flags, stream):
    o = _opts(options, flags)
    _operands(A, B, C, m, k, n, bool(o.flags & FLAG_B_TRANSPOSED),
              device=not (o.flags & FLAG_HOST_OPERANDS))
    _check(fn(_ptr(A), _ld(A), _ptr(B), _ld(B), _ptr(C), _ld(C), m, k, n, ctypes.byref(o),
              _stream(C, stream)))
    return C


def bmm_gf2(A, B, C, m, k, n, options=None, b_transposed=False, accumulate=False, stream=None,
            host_operands=False):
    """C = AB (or C ^= AB) over GF(2) by the cubic method.  host_operands: A, B, C
    are page-locked CPU tensors streamed through HBM (synchronous)."""
    flags = ((FLAG_B_TRANSPOSED if b_transposed else 0) | (FLAG_ACCUMULATE if accumulate else 0)
             | (FLAG_HOST_OPERANDS if host_operands else 0))
    return _product(_c_gf2, A, B, C, m, k, n, options, flags, stream)


def bmm_boolean(A, B, C, m, k, n, options=None, b_transposed=False, accumulate=False,
                stream=None, host_operands=False):
    """C = AB (or C |= AB) over the Boolean algebra by the cubic method."""
    flags = ((FLAG_B_TRANSPOSED if b_transposed else 0) | (FLAG_ACCUMULATE if accumulate else 0)
             | (FLAG_HOST_OPERANDS if host_operands else 0))
    return _product(_c_boolean, A, B, C, m, k, n, options, flags, stream)


def bmm_cubic_noalloc(semiring, A, B, C, m, k, n, options=None, b_transposed=False,
                      accumulate=False, stream=None):
    """C = AB (or C ^= / |= AB) by the cubic method with B^T staged in the library's
    fixed device array (no allocation; n * words(k) * 8 <= NOALLOC_SCRATCH_BYTES
    unless B is given transposed)."""
    flags = (FLAG_B_TRANSPOSED if b_transposed else 0) | (FLAG_ACCUMULATE if accumulate else 0)
    fn = lambda *a: _c_noalloc(semiring, *a)
    return _product(fn, A, B, C, m, k, n, options, flags, stream)


def bmm_gf2_strassen_workspace(m, k, n, depth=-1, options=None, alt_basis_io=False,
                               b_transposed=False, inplace_basis=False):
    """(bytes, depth_serial, depth_parallel) of the Strassen product's workspace."""
    o = _opts(options, (FLAG_ALT_BASIS_IO if alt_basis_io else 0)
              | (FLAG_B_TRANSPOSED if b_transposed else 0)
              | (FLAG_INPLACE_BASIS if inplace_basis else 0))
    nbytes = ctypes.c_size_t(0)
    ds = _int(0)
    dp = _int(0)
    _check(_c_strassen_ws(m, k, n, depth, ctypes.byref(o), ctypes.byref(nbytes),
                          ctypes.byref(ds), ctypes.byref(dp)))
    return nbytes.value, ds.value, dp.value


def bmm_gf2_strassen(A, B, C, m, k, n, workspace, depth=-1, options=None, b_transposed=False,
                     alt_basis_io=False, accumulate=False, inplace_basis=False, stream=None,
                     host_operands=False):
    """C = AB (or C ^= AB) over GF(2) by the self-inverse alternative-basis recursion.
    host_operands: A, B, C are page-locked CPU tensors, streamed through HBM by the
    out-of-core pipeline (synchronous; workspace and depth are not used)."""
    o = _opts(options, (FLAG_B_TRANSPOSED if b_transposed else 0)
              | (FLAG_ALT_BASIS_IO if alt_basis_io else 0)
              | (FLAG_ACCUMULATE if accumulate else 0)
              | (FLAG_INPLACE_BASIS if inplace_basis else 0)
              | (FLAG_HOST_OPERANDS if host_operands else 0))
    host = bool(o.flags & FLAG_HOST_OPERANDS)
    _operands(A, B, C, m, k, n, b_transposed, device=not host)
    if host:
        ws, nbytes = None, 0
    else:
        if not _is_tensor(workspace) or not workspace.is_cuda or not workspace.is_contiguous():
            raise ValueError("the workspace must be a contiguous GPU tensor")
        ws, nbytes = _ptr(workspace), workspace.numel() * workspace.element_size()
    _check(_c_strassen(_ptr(A), _ld(A), _ptr(B), _ld(B), _ptr(C), _ld(C), m, k, n, depth,
                       ws, nbytes, ctypes.byref(o), _stream(C, stream)))
    return C


def _problems(problems):
    arr = (Problem * len(problems))()
    for i, p in enumerate(problems):
        try:
            _operands(p["A"], p["B"], p["C"], p["m"], p["k"], p["n"],
                      bool(p.get("b_transposed")))
        except (TypeError, ValueError) as e:
            raise type(e)(f"problem {i}: {e}") from None
        arr[i] = Problem(p["semiring"], p["m"], p["k"], p["n"], p["A"].data_ptr(),
                         p["B"].data_ptr(), p["C"].data_ptr(), _ld(p["A"]), _ld(p["B"]),
                         _ld(p["C"]), 1 if p.get("b_transposed") else 0)
    return arr


def bmm_batched(problems, options=None, stream=None):
    """Independent products (dicts with semiring, m, k, n, A, B, C[, b_transposed])
    in one persistent launch."""
    if not problems:
        return
    arr = _problems(problems)
    o = _opts(options, 0)
    _check(_c_batched(arr, len(problems), ctypes.byref(o),
                      _stream(problems[0]["C"], stream)))


class BatchedPlan:
    """bmm_batched_plan_*: a device-resident problem table for repeated launches
    (capturable into a HIP graph).  Every problem must be b_transposed."""

    def __init__(self, problems, options=None):
        self._keep = problems
        arr = _problems(problems)
        o = _opts(options, 0)
        h = _vp()
        _check(_c_plan_create(arr, len(problems), ctypes.byref(o), ctypes.byref(h)))
        self._h = h

    def launch(self, stream=None):
        if stream is None:
            import torch
            stream = torch.cuda.current_stream().cuda_stream
        _check(_c_plan_launch(self._h, ctypes.c_void_p(int(stream))))

    def destroy(self):
        if self._h:
            _c_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def bmm_autotune_batched(problems):
    """Time every batched (leaf, tile) candidate on these problems (outputs are
    overwritten) and record the fastest for later AUTO plans; returns
    (leaf, tile, seconds)."""
    arr = _problems(problems)
    leaf = _int(0)
    tile = _int(0)
    secs = ctypes.c_double(0.0)
    _check(_c_tune_batched(arr, len(problems), ctypes.byref(leaf), ctypes.byref(tile),
                           ctypes.byref(secs)))
    return leaf.value, tile.value, secs.value


def bmm_transpose(src, dst, rows, cols, stream=None):
    _sizes(rows, cols, 0)
    if rows > 0 and cols > 0:
        for dev in (None, True):
            _mat(src, "src", rows, cols, device=dev)
            _mat(dst, "dst", cols, rows, device=dev)
    _check(_c_transpose(_ptr(src), _ld(src), _ptr(dst), _ld(dst), rows, cols,
                        _stream(dst, stream)))
    return dst


def bmm_basis_change(X, rows, row_words, depth, inverse=False, scheme=SCHEME_SELF_INVERSE,
                     transposed=False, stream=None):
    _sizes(rows, row_words, 0)
    if depth > 0:
        _mat(X, "X", rows, 64 * row_words)
    _check(_c_basis(_ptr(X), _ld(X), rows, row_words, depth, 1 if inverse else 0, scheme,
                    1 if transposed else 0, _stream(X, stream)))
    return X


def _extent(t, name, parents, stride, rows, ld, row_words, device=None):
    """The C call addresses words [0, (parents-1)*stride + (rows-1)*ld + row_words) from
    t.data_ptr(): t's storage must hold them (and t must be an 8-byte GPU tensor)."""
    if not _is_tensor(t) or t.element_size() != 8 or t.is_floating_point():
        raise ValueError(f"{name} must be a tensor of 64-bit words")
    if device and not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if parents > 0 and rows > 0 and row_words > 0:
        need = (parents - 1) * stride + (rows - 1) * ld + row_words
        if stride < 0 or ld < row_words or need > _span(t):
            raise ValueError(f"{name} holds {_span(t)} words from its start; the sizes "
                             f"address {need}")


def bmm_expand(side, levels, src, ldp, stride_p, dst, rows, words_, parents,
               scheme=SCHEME_SELF_INVERSE, stream=None):
    _sizes(rows, words_, parents)
    if rows > 0 and words_ > 0 and parents > 0 and levels in (1, 2):
        c = 7 ** levels
        cw = (rows >> levels) * (words_ >> levels)
        for dev in (None, True):
            _extent(src, "src", parents, stride_p, rows, ldp, words_, dev)
            _extent(dst, "dst", 1, 0, 1, cw * c * parents, cw * c * parents, dev)
    _check(_c_expand(side, levels, scheme, _ptr(src), ldp, stride_p, _ptr(dst), rows, words_,
                     parents, _stream(dst, stream)))
    return dst


def bmm_compress(levels, src, dst, ldp, stride_p, rows, words_, parents,
                 scheme=SCHEME_SELF_INVERSE, stream=None):
    _sizes(rows, words_, parents)
    if rows > 0 and words_ > 0 and parents > 0 and levels in (1, 2):
        c = 7 ** levels
        cw = (rows >> levels) * (words_ >> levels)
        for dev in (None, True):
            _extent(src, "src", 1, 0, 1, cw * c * parents, cw * c * parents, dev)
            _extent(dst, "dst", parents, stride_p, rows, ldp, words_, dev)
    _check(_c_compress(levels, scheme, _ptr(src), _ptr(dst), ldp, stride_p, rows, words_,
                       parents, _stream(dst, stream)))
    return dst


def bmm_ooc(semiring, A, B, C, m, k, n, block=0, options=None):
    """Out-of-core product of page-locked host matrices (numpy or pinned torch
    CPU tensors) streamed through HBM.  Synchronous; returns the seconds spent."""
    def hptr(t, name, rows, cols):
        if _is_tensor(t):
            _mat(t, name, rows, cols, device=False)
            return ctypes.c_void_p(t.data_ptr()), t.stride(0)
        if (getattr(t, "ndim", 0) != 2 or t.itemsize != 8 or t.dtype.kind not in "iu"
                or t.strides[1] != 8):
            raise ValueError(f"{name} must be a 2-D array of 64-bit words with contiguous rows")
        if rows > 0 and cols > 0 and (t.shape[0] < rows or t.shape[1] < words(cols)):
            raise ValueError(f"{name} has shape {t.shape}; the sizes need at least "
                             f"{rows} x {words(cols)} words")
        return ctypes.c_void_p(t.ctypes.data), t.strides[0] // 8
    _sizes(m, k, n)
    o = _opts(options, FLAG_HOST_OPERANDS)
    a, lda = hptr(A, "A", m, k)
    b, ldb = hptr(B, "B", k, n)
    c, ldc = hptr(C, "C", m, n)
    secs = ctypes.c_double(0.0)
    _check(_c_ooc(semiring, a, lda, b, ldb, c, ldc, m, k, n, block, ctypes.byref(o),
                  ctypes.byref(secs)))
    return secs.value


def bmm_debug_fail_allocations(count):
    """Make the library's next `count` device allocations fail (0 disarms)."""
    _check(_c_fail_allocs(count))


def bmm_ooc_last_transfers():
    """(h2d_bytes, h2d_seconds, d2h_bytes, d2h_seconds) of this thread's last bmm_ooc."""
    out = [ctypes.c_double(0.0) for _ in range(4)]
    _check(_c_ooc_xfer(*[ctypes.byref(v) for v in out]))
    return tuple(v.value for v in out)


def bmm_autotune_cubic(semiring, m, k, n):
    leaf = _int(0)
    tile = _int(0)
    secs = ctypes.c_double(0.0)
    _check(_c_tune(semiring, m, k, n, ctypes.byref(leaf), ctypes.byref(tile),
                   ctypes.byref(secs)))
    return leaf.value, tile.value, secs.value


def bmm_autotune_leaf(semiring, m, k, n, batch=1):
    """Time every leaf kernel and tile on `batch` products; returns (leaf, tile, seconds)."""
    leaf = _int(0)
    tile = _int(0)
    secs = ctypes.c_double(0.0)
    _check(_c_tune_leaf(semiring, m, k, n, batch, ctypes.byref(leaf), ctypes.byref(tile),
                        ctypes.byref(secs)))
    return leaf.value, tile.value, secs.value


def bmm_autotune_strassen(A, B, C, m, k, n, workspace, options=None):
    """Time the admissible Strassen depths (plain and shifted leaf level) on these
    operands; returns (depth, depth_serial, shift, seconds) and records them for
    depth -1."""
    o = _opts(options, 0)
    _operands(A, B, C, m, k, n, False)
    if not _is_tensor(workspace) or not workspace.is_cuda or not workspace.is_contiguous():
        raise ValueError("the workspace must be a contiguous GPU tensor")
    d = _int(0)
    ds = _int(0)
    sh = _int(0)
    secs = ctypes.c_double(0.0)
    nbytes = workspace.numel() * workspace.element_size()
    _check(_c_tune_strassen(_ptr(A), _ld(A), _ptr(B), _ld(B), _ptr(C), _ld(C), m, k, n,
                            _ptr(workspace), nbytes, ctypes.byref(o), ctypes.byref(d),
                            ctypes.byref(ds), ctypes.byref(sh), ctypes.byref(secs)))
    return d.value, ds.value, sh.value, secs.value


def bmm_autotune_k_panel(semiring, A, B, C, m, k, n, options=None, candidates=None,
                         b_transposed=False):
    """Time the cubic product on these operands with each k-panel length (bits;
    default: one panel and the powers of two from 8192 below k); returns
    (panel_bits, seconds) and records the choice for k_panel = 0.  C holds the product."""
    o = _opts(options, FLAG_B_TRANSPOSED if b_transposed else 0)
    _operands(A, B, C, m, k, n, bool(o.flags & FLAG_B_TRANSPOSED))
    cand = list(candidates or [])
    arr = (_i64 * max(1, len(cand)))(*cand)
    bits = _i64(0)
    secs = ctypes.c_double(0.0)
    _check(_c_tune_kpanel(semiring, _ptr(A), _ld(A), _ptr(B), _ld(B), _ptr(C), _ld(C), m, k, n,
                          ctypes.byref(o), arr, len(cand), ctypes.byref(bits),
                          ctypes.byref(secs)))
    return bits.value, secs.value


def bmm_autotune_set(semiring, m, k, n, leaf, tile, batch=1):
    _check(_c_tune_set(semiring, m, k, n, batch, leaf, tile))


def bmm_autotune_save(path):
    _check(_c_tune_save(path.encode()))


def bmm_autotune_load(path):
    _check(_c_tune_load(path.encode()))


def bmm_leaf_tiles(leaf):
    c = _int(0)
    _check(_c_tiles(leaf, ctypes.byref(c)))
    return c.value


def bmm_leaf_choice(semiring, m, k, n, batch=1, options=None):
    """(leaf, tile) that a product of this shape would run with these options."""
    o = _opts(options, 0)
    leaf = _int(0)
    tile = _int(0)
    _check(_c_leaf_choice(semiring, m, k, n, batch, ctypes.byref(o), ctypes.byref(leaf),
                          ctypes.byref(tile)))
    return leaf.value, tile.value


def bmm_leaf_tile_shape(leaf, tile):
    r = _int(0)
    c = _int(0)
    _check(_c_tile_shape(leaf, tile, ctypes.byref(r), ctypes.byref(c)))
    return r.value, c.value


def bmm_calibrate_valu(waves_per_simd=2, rounds=1 << 20):
    """Measured v_bitop3_b32 issue rate (bmm_calibrate_valu): dict with
    lane_ops_per_clk_cu, clock_ghz, seconds and aggregate_bops."""
    out = [ctypes.c_double(0.0) for _ in range(4)]
    _check(_c_calib(waves_per_simd, rounds, *[ctypes.byref(v) for v in out]))
    return dict(zip(("lane_ops_per_clk_cu", "clock_ghz", "seconds", "aggregate_bops"),
                    (v.value for v in out)))


def bmm_version():
    return _c_version().decode()


def bmm_finalize():
    _c_finalize()
