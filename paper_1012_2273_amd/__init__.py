"""MI355X-native dense matrix product C = A*B (Hasta and Mutiara, arXiv 1012.2273).

Thin Python binding over ``libgemm_mi355x.so``: every function marshals torch
device tensors into the C ABI (``include/gemm_mi355x.h``) and launches on
torch's current stream. Every arithmetic step runs in the HIP kernels; there
is no CPU or PyTorch fallback, and a missing library raises.

Names follow the C ABI: ``gemm_plain``, ``gemm_split``, ``gemm_split_convert``,
``gemm_backward``, ``gemm_grouped`` (plus :class:`GroupedPlan` for the
captured, replayable form) and :class:`GemmFn`, an autograd function whose
backward calls ``gemm_backward``.
"""
from __future__ import annotations

import ctypes

from . import _lib
from ._lib import (GEMM_BF16, GEMM_F32, GEMM_F64, GEMM_PLAN_AUTOTUNE, GEMM_PLAN_NO_GRAPH,
                   GEMM_PLAN_NO_PACK, GemmArgError, GemmError)

__all__ = [
    "gemm_plain", "gemm_split", "gemm_split_convert", "gemm_split_workspace_size",
    "gemm_split3", "gemm_split3_convert", "gemm_split3_workspace_size", "split_one_launch",
    "gemm_backward", "gemm_grouped", "GroupedPlan", "GemmFn", "matmul", "load",
    "GemmError", "GemmArgError", "GEMM_F64", "GEMM_F32", "GEMM_BF16",
    "tile_configs", "force_tile_config", "gemm_plain_ksplit", "gemm_plain_ksplit_workspace_size",
    "force_ksplit", "force_split_form",
]


def load():
    """Load the HIP library (raises RuntimeError if it has not been built)."""
    return _lib.load()


def _torch():
    import torch
    return torch


def _dtype_code(t):
    torch = _torch()
    if t.dtype == torch.float64:
        return GEMM_F64
    if t.dtype == torch.float32:
        return GEMM_F32
    if t.dtype == torch.bfloat16:
        return GEMM_BF16
    raise GemmArgError(_lib.GEMM_EUNSUPPORTED, "dtype", f"unsupported dtype {t.dtype}")


def _out_dtype(code):
    torch = _torch()
    return torch.float64 if code == GEMM_F64 else torch.float32


def _mat(t, name):
    """(ptr, ld) of a row-major 2-D device tensor (unit column stride); the
    pointer as a plain int (0 for an empty matrix), which ctypes passes as a
    void pointer. Each tensor attribute is read once: at small N the
    binding's own time is most of a call's."""
    shape = t.shape
    if len(shape) != 2:
        raise GemmArgError(_lib.GEMM_EINVAL, name, "expected a 2-D tensor")
    if not t.is_cuda:
        raise GemmArgError(_lib.GEMM_EINVAL, name, "expected a device tensor")
    r, c = shape
    if r == 0 or c == 0:
        return 0, int(max(c, 1))
    s0, s1 = t.stride()
    if c > 1 and s1 != 1:
        raise GemmArgError(_lib.GEMM_ELD, name, "columns must be contiguous (stride 1)")
    return t.data_ptr(), int(s0 if r > 1 else c)


_raw_stream = None   # the current-stream query, chosen on first use


def _stream(t):
    """The current stream of t's device as a raw pointer (torch's C-level
    query when it has one: a tenth of a microsecond against about two for
    building a Stream object)."""
    global _raw_stream
    if _raw_stream is None:
        torch = _torch()
        raw = getattr(torch._C, "_cuda_getCurrentRawStream", None)
        if raw is not None:
            _raw_stream = lambda dev: raw(dev.index if dev.index is not None
                                          else torch.cuda.current_device())
        else:
            _raw_stream = lambda dev: torch.cuda.current_stream(dev).cuda_stream
    return _raw_stream(t.device)


def _check_out(C, shape, dtype, like, where, name="C"):
    """A caller-supplied output must have the product's shape, the output
    dtype of the call and live on the inputs' device: the kernels write
    shape[0] x shape[1] elements of that dtype through its pointer."""
    if tuple(C.shape) != tuple(shape):
        raise GemmArgError(_lib.GEMM_EINVAL, where,
                           f"{name} has shape {tuple(C.shape)}, expected {tuple(shape)}")
    if C.dtype != dtype:
        raise GemmArgError(_lib.GEMM_EINVAL, where, f"{name} has dtype {C.dtype}, expected {dtype}")
    if C.device != like.device:
        raise GemmArgError(_lib.GEMM_EINVAL, where,
                           f"{name} is on {C.device}, the inputs on {like.device}")


def _workspace(ws, need, like, where):
    """(pointer, size in bytes) of a caller workspace, allocated when absent.
    It must be a contiguous device tensor on the inputs' device."""
    torch = _torch()
    if ws is None:
        ws = torch.empty(max(int(need), 1), dtype=torch.uint8, device=like.device)
    if not ws.is_cuda or ws.device != like.device:
        raise GemmArgError(_lib.GEMM_EINVAL, where,
                           f"workspace must be a device tensor on {like.device}")
    if not ws.is_contiguous():
        raise GemmArgError(_lib.GEMM_EINVAL, where, "workspace must be contiguous")
    return ws, ctypes.c_void_p(ws.data_ptr()), int(ws.numel() * ws.element_size())


def gemm_plain(A, B, C=None):
    """C = A @ B on the matrix cores. float64, float32, or bfloat16 inputs
    (bfloat16 gives a float32 C). Writes into ``C`` if given."""
    torch = _torch()
    code = _dtype_code(A)
    if B.dtype != A.dtype:
        raise GemmArgError(_lib.GEMM_EINVAL, "gemm_plain", "A and B dtypes differ")
    m, k = A.shape
    k2, n = B.shape
    if k2 != k:
        raise GemmArgError(_lib.GEMM_EINVAL, "gemm_plain", f"shape mismatch {tuple(A.shape)} x {tuple(B.shape)}")
    if C is None:
        C = torch.empty((m, n), dtype=_out_dtype(code), device=A.device)
    else:
        _check_out(C, (m, n), _out_dtype(code), A, "gemm_plain")
    pa, lda = _mat(A, "A")
    pb, ldb = _mat(B, "B")
    pc, ldc = _mat(C, "C")
    lib = _lib.load()
    _lib.check(lib.gemm_plain(code, m, n, k, pa, lda, pb, ldb, pc, ldc, _stream(A)), "gemm_plain")
    return C


def gemm_plain_ksplit_workspace_size(dtype_code, m, n, k) -> int:
    return int(_lib.load().gemm_plain_ksplit_workspace_size(int(dtype_code), int(m), int(n), int(k)))


def gemm_plain_ksplit(A, B, C=None, workspace=None):
    """C = A @ B like gemm_plain, with the K loop split over workgroups when
    the product has too few output tiles to occupy the device (partial
    products in ``workspace``, then added in K order)."""
    torch = _torch()
    code = _dtype_code(A)
    if B.dtype != A.dtype:
        raise GemmArgError(_lib.GEMM_EINVAL, "gemm_plain_ksplit", "A and B dtypes differ")
    m, k = A.shape
    k2, n = B.shape
    if k2 != k:
        raise GemmArgError(_lib.GEMM_EINVAL, "gemm_plain_ksplit",
                           f"shape mismatch {tuple(A.shape)} x {tuple(B.shape)}")
    if C is None:
        C = torch.empty((m, n), dtype=_out_dtype(code), device=A.device)
    else:
        _check_out(C, (m, n), _out_dtype(code), A, "gemm_plain_ksplit")
    need = gemm_plain_ksplit_workspace_size(code, m, n, k) if workspace is None else 0
    workspace, pw, wbytes = _workspace(workspace, need, A, "gemm_plain_ksplit")
    pa, lda = _mat(A, "A")
    pb, ldb = _mat(B, "B")
    pc, ldc = _mat(C, "C")
    lib = _lib.load()
    _lib.check(lib.gemm_plain_ksplit(code, m, n, k, pa, lda, pb, ldb, pc, ldc, pw, wbytes,
                                     _stream(A)), "gemm_plain_ksplit")
    return C


def gemm_plain_ksplit_noalloc(A, B, C):
    """gemm_plain_ksplit without a workspace, for callers that cannot
    allocate device memory: the partial products go to the library's
    per-device scratch array (``_lib.NOALLOC_SCRATCH_BYTES``). ``C`` is the
    caller's output; the call allocates nothing. Calls that overlap on one
    device race on the shared array."""
    code = _dtype_code(A)
    if B.dtype != A.dtype:
        raise GemmArgError(_lib.GEMM_EINVAL, "gemm_plain_ksplit_noalloc", "A and B dtypes differ")
    m, k = A.shape
    k2, n = B.shape
    if k2 != k:
        raise GemmArgError(_lib.GEMM_EINVAL, "gemm_plain_ksplit_noalloc",
                           f"shape mismatch {tuple(A.shape)} x {tuple(B.shape)}")
    _check_out(C, (m, n), _out_dtype(code), A, "gemm_plain_ksplit_noalloc")
    pa, lda = _mat(A, "A")
    pb, ldb = _mat(B, "B")
    pc, ldc = _mat(C, "C")
    lib = _lib.load()
    _lib.check(lib.gemm_plain_ksplit_noalloc(code, m, n, k, pa, lda, pb, ldb, pc, ldc,
                                             _stream(A)), "gemm_plain_ksplit_noalloc")
    return C


def force_split_form(form: int):
    """Make this thread's gemm_split / gemm_split3 calls use one form: 0 split
    step and plane product, 1 one launch splitting fragments in registers, 2
    one launch whose loader waves split tiles into LDS (-1: automatic). A
    tuning knob for tests and tools; every form gives the same bits."""
    _lib.check(_lib.load().gemm_tuning_force_split_form(int(form)),
               "gemm_tuning_force_split_form")


def force_ksplit(parts: int):
    """Split the K loop of this thread's gemm_plain_ksplit calls into
    ``parts`` chunks (-1: automatic). A tuning knob for tests and tools."""
    _lib.check(_lib.load().gemm_tuning_force_ksplit_parts(int(parts)),
               "gemm_tuning_force_ksplit_parts")


def gemm_split_workspace_size(m, n, k) -> int:
    return int(_lib.load().gemm_split_workspace_size(int(m), int(n), int(k)))


def gemm_split3_workspace_size(m, n, k) -> int:
    return int(_lib.load().gemm_split3_workspace_size(int(m), int(n), int(k)))


def _split_product(name, size_fn, A, B, C, workspace):
    torch = _torch()
    if A.dtype != torch.float32 or B.dtype != torch.float32:
        raise GemmArgError(_lib.GEMM_EUNSUPPORTED, name, "float32 inputs required")
    m, k = A.shape
    k2, n = B.shape
    if k2 != k:
        raise GemmArgError(_lib.GEMM_EINVAL, name, "shape mismatch")
    if C is None:
        C = torch.empty((m, n), dtype=torch.float32, device=A.device)
    else:
        _check_out(C, (m, n), torch.float32, A, name)
    need = size_fn(m, n, k) if workspace is None else 0
    workspace, pw, wbytes = _workspace(workspace, need, A, name)
    pa, lda = _mat(A, "A")
    pb, ldb = _mat(B, "B")
    pc, ldc = _mat(C, "C")
    lib = _lib.load()
    _lib.check(getattr(lib, name)(m, n, k, pa, lda, pb, ldb, pc, ldc, pw, wbytes,
                                  _stream(A)), name)
    return C


def split_one_launch(A, B):
    """True if gemm_split on these operands runs as one launch that splits
    each fragment in registers (small products, and up to one 128 x 128 tile
    per CU on the loader-wave tile), False if it runs the split step and then
    the plane product (gemm_split3 takes the in-register form only for the
    small products; see gemm_split_one_launch in the C header)."""
    m, k = A.shape
    n = B.shape[1]
    if m == 0 or n == 0:
        return False
    pa, lda = _mat(A, "A")
    pb, ldb = _mat(B, "B")
    return bool(_lib.load().gemm_split_one_launch(m, n, k, pa, lda, pb, ldb))


def gemm_split(A, B, C=None, workspace=None):
    """float32 C ~= A @ B via the two-way bfloat16 split of A and B and three
    bfloat16 products accumulated in float32."""
    return _split_product("gemm_split", gemm_split_workspace_size, A, B, C, workspace)


def gemm_split3(A, B, C=None, workspace=None):
    """float32 C ~= A @ B via the three-way bfloat16 split of A and B and six
    bfloat16 products accumulated in float32 (binary32 accuracy)."""
    return _split_product("gemm_split3", gemm_split3_workspace_size, A, B, C, workspace)


def _split_convert(name, planes, X, transpose):
    torch = _torch()
    if X.dtype != torch.float32:
        raise GemmArgError(_lib.GEMM_EUNSUPPORTED, name, "float32 input required")
    r, c = X.shape
    shape = (c, r) if transpose else (r, c)
    outs = [torch.empty(shape, dtype=torch.int16, device=X.device) for _ in range(planes)]
    px, ldx = _mat(X, "X")
    ldo = shape[1] if shape[1] > 0 else 1
    lib = _lib.load()
    ptrs = [ctypes.c_void_p(t.data_ptr() if t.numel() else 0) for t in outs]
    _lib.check(getattr(lib, name)(r, c, px, ldx, int(bool(transpose)), *ptrs, ldo, _stream(X)), name)
    return tuple(outs)


def gemm_split_convert(X, transpose=False):
    """(hi, lo) int16 tensors holding the bfloat16 patterns of X's split;
    shape X.shape, or transposed when ``transpose``."""
    return _split_convert("gemm_split_convert", 2, X, transpose)


def gemm_split3_convert(X, transpose=False):
    """(hi, mid, lo) int16 tensors holding the bfloat16 patterns of X's
    three-way split; shape X.shape, or transposed when ``transpose``."""
    return _split_convert("gemm_split3_convert", 3, X, transpose)


def gemm_backward(A, B, dC, need_dA=True, need_dB=True):
    """(dA, dB) = (dC @ B^T, A^T @ dC) with transposed-operand tiles."""
    torch = _torch()
    code = _dtype_code(A)
    m, k = A.shape
    n = B.shape[1]
    if B.shape[0] != k or tuple(dC.shape) != (m, n):
        raise GemmArgError(_lib.GEMM_EINVAL, "gemm_backward", "shape mismatch")
    if B.dtype != A.dtype or dC.dtype != A.dtype:
        raise GemmArgError(_lib.GEMM_EINVAL, "gemm_backward", "dtypes differ")
    od = _out_dtype(code)
    dA = torch.empty((m, k), dtype=od, device=A.device) if need_dA else None
    dB = torch.empty((k, n), dtype=od, device=A.device) if need_dB else None
    pa, lda = _mat(A, "A")
    pb, ldb = _mat(B, "B")
    pd, lddc = _mat(dC, "dC")
    pda, ldda = _mat(dA, "dA") if dA is not None else (ctypes.c_void_p(0), 0)
    pdb, lddb = _mat(dB, "dB") if dB is not None else (ctypes.c_void_p(0), 0)
    lib = _lib.load()
    rc = lib.gemm_backward(code, m, n, k, pa, lda, pb, ldb, pd, lddc,
                           pda if dA is not None else None, ldda,
                           pdb if dB is not None else None, lddb, _stream(A))
    _lib.check(rc, "gemm_backward")
    return dA, dB


def _check_group(As, Bs, Cs, where):
    """Every problem's operands agree in dtype and inner size, and every C has
    the problem's output shape, the operands' dtype and device."""
    if not (len(As) == len(Bs) == len(Cs)):
        raise GemmArgError(_lib.GEMM_EINVAL, where, "list lengths differ")
    for i, (A, B, C) in enumerate(zip(As, Bs, Cs)):
        if A.dim() != 2 or B.dim() != 2 or A.shape[1] != B.shape[0] or \
                A.dtype != As[0].dtype or B.dtype != As[0].dtype:
            raise GemmArgError(_lib.GEMM_EINVAL, where, f"shape or dtype mismatch (problem {i})")
        _check_out(C, (A.shape[0], B.shape[1]), A.dtype, A, where, name=f"C[{i}]")


def _problems(As, Bs, Cs):
    arr = (_lib.GemmProblem * len(As))()
    for i, (A, B, C) in enumerate(zip(As, Bs, Cs)):
        pa, lda = _mat(A, "A")
        pb, ldb = _mat(B, "B")
        pc, ldc = _mat(C, "C")
        arr[i] = _lib.GemmProblem(A.shape[0], B.shape[1], A.shape[1], pa, pb, pc, lda, ldb, ldc)
    return arr


class GroupedPlan:
    """A captured persistent launch of independent products C_i = A_i @ B_i.

    ``autotune=True`` times candidate tile policies on the given data once
    (overwriting the C_i); ``tune_cache`` is a JSON path for the chosen policy.
    ``pack=False`` reads every operand where it is instead of copying those
    whose rows are not 16-byte vectors into padded plan-owned buffers.
    ``run()`` replays the captured hipGraph on torch's current stream.
    """

    def __init__(self, As, Bs, Cs=None, autotune=False, tune_cache=None, graph=True,
                 pack=True):
        torch = _torch()
        if not (len(As) == len(Bs)):
            raise GemmArgError(_lib.GEMM_EINVAL, "GroupedPlan", "list lengths differ")
        code = _dtype_code(As[0]) if As else GEMM_F64
        if Cs is None:
            Cs = [torch.empty((A.shape[0], B.shape[1]), dtype=A.dtype, device=A.device)
                  for A, B in zip(As, Bs)]
        _check_group(As, Bs, Cs, "GroupedPlan")
        self.As, self.Bs, self.Cs = list(As), list(Bs), list(Cs)
        self._arr = _problems(self.As, self.Bs, self.Cs)
        self.device = As[0].device if As else torch.device("cuda:0")
        flags = ((GEMM_PLAN_AUTOTUNE if autotune else 0) | (0 if graph else GEMM_PLAN_NO_GRAPH)
                 | (0 if pack else GEMM_PLAN_NO_PACK))
        lib = _lib.load()
        h = ctypes.c_void_p()
        stream = ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)
        _lib.check(lib.gemm_grouped_plan_create(
            ctypes.byref(h), code, self._arr, len(self.As),
            tune_cache.encode() if tune_cache else None, flags, stream), "gemm_grouped_plan_create")
        self._h = h

    def run(self):
        torch = _torch()
        lib = _lib.load()
        _lib.check(lib.gemm_grouped_run(
            self._h, ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)),
            "gemm_grouped_run")
        return self.Cs

    def update(self, As, Bs, Cs):
        """Point the plan at new tensors of identical shapes (no re-capture)."""
        torch = _torch()
        _check_group(As, Bs, Cs, "GroupedPlan.update")
        torch.cuda.current_stream(self.device).synchronize()
        arr = _problems(As, Bs, Cs)
        _lib.check(_lib.load().gemm_grouped_plan_update(self._h, arr, len(As)),
                   "gemm_grouped_plan_update")
        self.As, self.Bs, self.Cs, self._arr = list(As), list(Bs), list(Cs), arr

    def info(self):
        tiles = ctypes.c_int64()
        pol = (ctypes.c_int32 * 7)()
        _lib.check(_lib.load().gemm_grouped_plan_info(self._h, ctypes.byref(tiles), pol, 7),
                   "gemm_grouped_plan_info")
        return int(tiles.value), [tile_configs()[c] for c in pol]

    def close(self):
        if getattr(self, "_h", None):
            _lib.load().gemm_grouped_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def gemm_grouped(As, Bs, Cs=None):
    """Uncaptured convenience form: one persistent launch, then synchronise."""
    torch = _torch()
    if Cs is None:
        Cs = [torch.empty((A.shape[0], B.shape[1]), dtype=A.dtype, device=A.device)
              for A, B in zip(As, Bs)]
    if not As:
        return Cs
    code = _dtype_code(As[0])
    _check_group(As, Bs, Cs, "gemm_grouped")
    arr = _problems(As, Bs, Cs)
    _lib.check(_lib.load().gemm_grouped(code, arr, len(As), _stream(As[0])), "gemm_grouped")
    return Cs


def tile_configs():
    lib = _lib.load()
    return [lib.gemm_tile_config_name(i).decode() for i in range(lib.gemm_tile_config_count())]


def force_tile_config(cfg_id: int):
    """Use tile config ``cfg_id`` for this thread's single-product launches
    (-1: automatic). A tuning knob for tests and tools."""
    _lib.check(_lib.load().gemm_tuning_force_tile_config(int(cfg_id)),
               "gemm_tuning_force_tile_config")


def _gemm_fn():
    torch = _torch()

    class GemmFn(torch.autograd.Function):
        """C = A @ B with the hand-written backward (dA = dC B^T, dB = A^T dC)."""

        @staticmethod
        def forward(ctx, A, B):
            ctx.save_for_backward(A, B)
            return gemm_plain(A.contiguous(), B.contiguous())

        @staticmethod
        def backward(ctx, dC):
            A, B = ctx.saved_tensors
            dC = dC.to(A.dtype).contiguous()
            dA, dB = gemm_backward(A.contiguous(), B.contiguous(), dC,
                                   need_dA=ctx.needs_input_grad[0],
                                   need_dB=ctx.needs_input_grad[1])
            return dA, dB

    return GemmFn


_GemmFn = None


def __getattr__(name):
    global _GemmFn
    if name == "GemmFn":
        if _GemmFn is None:
            _GemmFn = _gemm_fn()
        return _GemmFn
    raise AttributeError(name)


def matmul(A, B):
    """Differentiable C = A @ B through :class:`GemmFn`."""
    return __getattr__("GemmFn").apply(A, B)
