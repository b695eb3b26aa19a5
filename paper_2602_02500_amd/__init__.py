"""Python binding of libifnso (IFNSO on MI355X / gfx950).

Argument marshalling only: every step of the computation runs in the library's HIP
kernels. The functions take torch tensors for device memory and use torch's current
HIP stream; the C ABI itself (include/ifnso.h) takes raw device pointers.
"""
from __future__ import annotations

import ctypes
import os
import re
from typing import Optional, Sequence

__all__ = [
    "load", "LIB_PATH", "HEADER_PATH", "IfnsoError", "Plan", "SchedulePlan", "classical_ns",
    "classical_ns_workspace_bytes", "ns_schedule",
    "orth_error", "F32", "BF16", "COMPUTE_F32", "COMPUTE_BF16", "COMPUTE_FP8", "BASIS_GRAM",
    "BASIS_COMPLEMENT", "NORM_FROBENIUS", "NORM_GRAM_FROBENIUS", "NORM_NONE", "FLAG_ENFORCE_SUM_ONE",
    "FLAG_SPLIT_BF16", "FLAG_DETERMINISTIC", "FLAG_SPLIT_P",
    "header_functions", "STATUS", "orth_error_workspace_bytes", "MLP_NUM_PARAMS", "STATS_PER_PROBLEM",
    "mlp_features", "mlp_forward", "mlp_train_step", "mlp_train_workspace_bytes", "StageConfig",
    "quantize_e4m3", "quantize_e4m3_workspace_bytes", "STAGE_GRAM", "STAGE_SQUARE", "STAGE_PRODUCT",
    "MuonParams", "STATIC_SCRATCH_BYTES",
]

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libifnso.so")
HEADER_PATH = os.path.join(os.path.dirname(_PKG), "include", "ifnso.h")

F32, BF16 = 0, 1
COMPUTE_F32, COMPUTE_BF16, COMPUTE_FP8 = 0, 1, 2
BASIS_GRAM, BASIS_COMPLEMENT = 0, 1
NORM_FROBENIUS, NORM_GRAM_FROBENIUS, NORM_NONE = 0, 1, 2
COEFF_FIXED, COEFF_LEARNED = 0, 1
FLAG_ENFORCE_SUM_ONE = 1
FLAG_DETERMINISTIC = 2
FLAG_SPLIT_P = 4
FLAG_SPLIT_BF16 = 8
STATS_PER_PROBLEM = 26
STATIC_SCRATCH_BYTES = 64 << 20  # IFNSO_STATIC_SCRATCH_BYTES
MLP_NUM_PARAMS = 5126
STATUS = {0: "OK", 1: "INVALID_ARGUMENT", 2: "UNSUPPORTED", 3: "WORKSPACE_TOO_SMALL", 4: "HIP", 5: "INTERNAL"}

_BASIS = {"gram": BASIS_GRAM, "complement": BASIS_COMPLEMENT}
_NORM = {"frobenius": NORM_FROBENIUS, "gram_frobenius": NORM_GRAM_FROBENIUS, "none": NORM_NONE}
_COMPUTE = {"f32": COMPUTE_F32, "bf16": COMPUTE_BF16, "fp8": COMPUTE_FP8}


class IfnsoError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


STAGE_GRAM, STAGE_SQUARE, STAGE_PRODUCT = 0, 1, 2


class MuonParams(ctypes.Structure):
    """Hyper-parameters of one Muon step (see ifnso_muon_params)."""
    _fields_ = [("lr", ctypes.c_double), ("momentum", ctypes.c_double), ("weight_decay", ctypes.c_double),
                ("nesterov", ctypes.c_int32)]


class StageConfig(ctypes.Structure):
    """Schedule of a 256-tile stage (see ifnso_stage_config)."""
    _fields_ = [("xcd_sched", ctypes.c_int32), ("group", ctypes.c_int32), ("block_rows", ctypes.c_int32),
                ("block_cols", ctypes.c_int32), ("wg_per_xcd", ctypes.c_int32)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class PolyDesc(ctypes.Structure):
    _fields_ = [
        ("num_terms", ctypes.c_int32),
        ("exponents", ctypes.POINTER(ctypes.c_int32)),
        ("coeffs", ctypes.POINTER(ctypes.c_double)),
        ("basis", ctypes.c_int32),
        ("norm", ctypes.c_int32),
        ("compute", ctypes.c_int32),
        ("coeff_mode", ctypes.c_int32),
        ("mlp_params", ctypes.POINTER(ctypes.c_float)),
        ("mlp_params_len", ctypes.c_size_t),
        ("flags", ctypes.c_uint32),
    ]


_lib = None


def load() -> ctypes.CDLL:
    """Loads the in-tree libifnso.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2602_02500_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    P64 = ctypes.POINTER(ctypes.c_int64)
    L.ifnso_plan.argtypes = [ctypes.POINTER(PolyDesc), i32, P64, P64, i32, i32, i32, ctypes.POINTER(vp)]
    L.ifnso_plan_workspace_bytes.argtypes = [vp, ctypes.POINTER(sz)]
    L.ifnso_plan_destroy.argtypes = [vp]
    L.ifnso_orthogonalize.argtypes = [vp, vp, i64, vp, i64, vp, sz, vp]
    L.ifnso_orthogonalize_batched.argtypes = [vp, ctypes.POINTER(vp), P64, ctypes.POINTER(vp), P64, vp, sz, vp]
    L.ifnso_orthogonalize_static.argtypes = [vp, vp, i64, vp, i64, vp]
    L.ifnso_orthogonalize_static.restype = ctypes.c_int
    L.ifnso_muon_workspace_bytes.argtypes = [vp, ctypes.POINTER(sz)]
    L.ifnso_muon_step.argtypes = [vp, ctypes.POINTER(MuonParams), ctypes.POINTER(vp), P64, ctypes.POINTER(vp), P64,
                                  ctypes.POINTER(vp), P64, vp, sz, vp]
    L.ifnso_classical_ns.argtypes = [vp, i64, i64, i64, i32, vp, i64, i32, ctypes.POINTER(ctypes.c_double), i32,
                                     vp, sz, vp]
    L.ifnso_ns_schedule.argtypes = [vp, i64, i64, i64, i32, vp, i64, i32, ctypes.POINTER(ctypes.c_double), i32, i32,
                                    vp, sz, vp]
    L.ifnso_schedule_plan.argtypes = [ctypes.POINTER(ctypes.c_double), i32, i32, i32, P64, P64, i32, i32, i32,
                                      ctypes.POINTER(vp)]
    L.ifnso_schedule_plan.restype = ctypes.c_int
    L.ifnso_schedule_plan_workspace_bytes.argtypes = [vp, ctypes.POINTER(sz)]
    L.ifnso_schedule_plan_workspace_bytes.restype = ctypes.c_int
    L.ifnso_schedule_plan_destroy.argtypes = [vp]
    L.ifnso_schedule_plan_destroy.restype = ctypes.c_int
    L.ifnso_schedule_orthogonalize_batched.argtypes = [vp, ctypes.POINTER(vp), P64, ctypes.POINTER(vp), P64, vp, sz,
                                                       vp]
    L.ifnso_schedule_orthogonalize_batched.restype = ctypes.c_int
    L.ifnso_classical_ns_workspace_bytes.argtypes = [i64, i64, i32]
    L.ifnso_classical_ns_workspace_bytes.restype = sz
    L.ifnso_orth_error.argtypes = [i32, ctypes.POINTER(vp), P64, P64, P64, i32, vp, vp, sz, vp]
    L.ifnso_orth_error_workspace_bytes.argtypes = [i32]
    L.ifnso_orth_error_workspace_bytes.restype = sz
    L.ifnso_plan_num_launches.argtypes = [vp]
    L.ifnso_plan_num_launches.restype = i32
    L.ifnso_plan_launch_info.argtypes = [vp, i32, ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_double)]
    L.ifnso_plan_launch_info.restype = ctypes.c_int
    L.ifnso_plan_launch_events.argtypes = [vp, ctypes.POINTER(vp), i32]
    L.ifnso_plan_launch_events.restype = ctypes.c_int
    L.ifnso_plan_stats.argtypes = [vp, ctypes.POINTER(ctypes.c_double), vp]
    L.ifnso_plan_stats.restype = ctypes.c_int
    L.ifnso_mlp_features.argtypes = [i32, vp, vp, i32, vp, vp]
    L.ifnso_mlp_features.restype = ctypes.c_int
    L.ifnso_mlp_forward.argtypes = [i32, vp, vp, vp, vp]
    L.ifnso_mlp_forward.restype = ctypes.c_int
    fl = ctypes.c_float
    L.ifnso_mlp_train_step.argtypes = [i32, vp, vp, vp, i32, vp, vp, vp, i32, fl, fl, fl, fl, vp, vp, vp, sz, vp]
    L.ifnso_mlp_train_step.restype = ctypes.c_int
    L.ifnso_mlp_train_workspace_bytes.argtypes = [i32]
    L.ifnso_mlp_train_workspace_bytes.restype = sz
    L.ifnso_plan_get_config.argtypes = [vp, i32, ctypes.POINTER(StageConfig)]
    L.ifnso_plan_get_config.restype = ctypes.c_int
    L.ifnso_plan_set_config.argtypes = [vp, i32, ctypes.POINTER(StageConfig)]
    L.ifnso_plan_set_config.restype = ctypes.c_int
    L.ifnso_quantize_e4m3.argtypes = [vp, i64, i64, i64, vp, i64, vp, vp, sz, vp]
    L.ifnso_quantize_e4m3.restype = ctypes.c_int
    L.ifnso_quantize_e4m3_workspace_bytes.argtypes = [i64, i64]
    L.ifnso_quantize_e4m3_workspace_bytes.restype = sz
    L.ifnso_last_error.restype = ctypes.c_char_p
    for name in ("ifnso_plan", "ifnso_plan_workspace_bytes", "ifnso_plan_destroy", "ifnso_orthogonalize",
                 "ifnso_orthogonalize_batched", "ifnso_classical_ns", "ifnso_orth_error"):
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def header_functions():
    """Names of the functions declared in include/ifnso.h."""
    src = open(HEADER_PATH).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ifnso_[a-z0-9_]+)\s*\(", src)))


def _check(status: int):
    if status != 0:
        raise IfnsoError(status, load().ifnso_last_error().decode())


def _stream(stream) -> Optional[int]:
    if stream is not None:
        return int(stream)
    import torch
    return torch.cuda.current_stream().cuda_stream


def _ptr(t) -> int:
    return t if isinstance(t, int) else t.data_ptr()


def _dtype_code(t) -> int:
    import torch
    if t.dtype == torch.float32:
        return F32
    if t.dtype == torch.bfloat16:
        return BF16
    raise TypeError(f"unsupported dtype {t.dtype}")


WORKSPACE_ALIGN = 256  # bytes; every workspace of the library starts at such an address
_DTYPE_NAME = {F32: "float32", BF16: "bfloat16"}


def check_matrix(t, name: str, shape, dtype: int, device: int) -> None:
    """Raises unless `t` is a torch tensor that the library can read or write as a row-major
    `shape` matrix of `dtype` (F32 or BF16) on GPU `device`: dtype, then shape, then unit
    column stride and a row stride of at least the column count, then the device. Nothing
    reaches the C ABI before every tensor of a call has passed."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name}: expected a torch tensor, got {type(t).__name__}")
    want = torch.float32 if dtype == F32 else torch.bfloat16
    if t.dtype != want:
        raise TypeError(f"{name}: dtype {t.dtype}, the plan needs {_DTYPE_NAME[dtype]}")
    if t.dim() != 2 or tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name}: shape {tuple(t.shape)}, the plan needs {tuple(shape)}")
    if t.stride(1) != 1 or t.stride(0) < max(1, shape[1]):
        raise ValueError(f"{name}: strides {t.stride()} are not a row-major layout (unit column stride, "
                         f"row stride >= {shape[1]})")
    if t.device.type != "cuda" or t.device.index != device:
        raise ValueError(f"{name}: on {t.device}, the plan runs on cuda:{device}")


def check_workspace(ws, need: int, device: int) -> int:
    """Raises unless `ws` is a contiguous tensor of at least `need` bytes on GPU `device`,
    starting at a WORKSPACE_ALIGN-byte address; returns its size in bytes."""
    import torch
    if not isinstance(ws, torch.Tensor):
        raise TypeError(f"workspace: expected a torch tensor, got {type(ws).__name__}")
    nb = ws.numel() * ws.element_size()
    if nb < need:
        raise ValueError(f"workspace: {nb} bytes, the call needs {need}")
    if not ws.is_contiguous():
        raise ValueError("workspace: not contiguous")
    if ws.device.type != "cuda" or ws.device.index != device:
        raise ValueError(f"workspace: on {ws.device}, the plan runs on cuda:{device}")
    if ws.data_ptr() % WORKSPACE_ALIGN:
        raise ValueError(f"workspace: address not {WORKSPACE_ALIGN}-byte aligned")
    return nb


class Plan:
    """A plan over problems of the given (rows, cols) shapes (ifnso_plan)."""

    def __init__(self, exponents: Sequence[int], coeffs: Sequence[float], shapes, basis="gram",
                 norm="frobenius", compute="bf16", in_dtype=None, out_dtype=None, device: int = 0,
                 flags: int = 0, mlp_params=None):
        """mlp_params: host float sequence of MLP_NUM_PARAMS values selects the learned mode."""
        L = load()
        self._L = L
        K = len(exponents)
        self._e = (ctypes.c_int32 * K)(*[int(x) for x in exponents])
        self._c = (ctypes.c_double * K)(*[float(x) for x in coeffs])
        comp = _COMPUTE[compute] if isinstance(compute, str) else int(compute)
        mode, mp, mlen = COEFF_FIXED, None, 0
        if mlp_params is not None:
            self._mp = (ctypes.c_float * len(mlp_params))(*[float(x) for x in mlp_params])
            mode, mp, mlen = COEFF_LEARNED, self._mp, len(mlp_params)
        d = PolyDesc(K, self._e, self._c, _BASIS[basis] if isinstance(basis, str) else int(basis),
                     _NORM[norm] if isinstance(norm, str) else int(norm), comp, mode, mp, mlen, int(flags))
        self.shapes = [(int(r), int(c)) for r, c in shapes]
        n = len(self.shapes)
        rows = (ctypes.c_int64 * n)(*[r for r, _ in self.shapes])
        cols = (ctypes.c_int64 * n)(*[c for _, c in self.shapes])
        if in_dtype is None:
            in_dtype = F32 if comp == COMPUTE_F32 else BF16
        if out_dtype is None:
            out_dtype = in_dtype
        self.in_dtype, self.out_dtype = int(in_dtype), int(out_dtype)
        self.device = int(device)
        h = ctypes.c_void_p()
        _check(L.ifnso_plan(ctypes.byref(d), n, rows, cols, self.in_dtype, self.out_dtype, int(device),
                            ctypes.byref(h)))
        self._h = h
        b = ctypes.c_size_t()
        _check(L.ifnso_plan_workspace_bytes(h, ctypes.byref(b)))
        self.workspace_bytes = b.value
        _check(L.ifnso_muon_workspace_bytes(h, ctypes.byref(b)))
        self.muon_workspace_bytes = b.value

    def check_io(self, Ms, Ys) -> None:
        """Raises unless Ms and Ys are the plan's problems in order: dtype, shape, layout and
        device (check_matrix)."""
        if len(Ms) != len(self.shapes) or len(Ys) != len(self.shapes):
            raise ValueError(f"{len(Ms)} inputs and {len(Ys)} outputs for a plan of {len(self.shapes)} problems")
        for i, (m, y, s) in enumerate(zip(Ms, Ys, self.shapes)):
            check_matrix(m, f"M[{i}]", s, self.in_dtype, self.device)
            check_matrix(y, f"Y[{i}]", s, self.out_dtype, self.device)

    def orthogonalize(self, M, Y, workspace, stream=None):
        if len(self.shapes) != 1:
            raise ValueError("orthogonalize takes a single-problem plan; use orthogonalize_batched")
        self.check_io([M], [Y])
        nb = check_workspace(workspace, self.workspace_bytes, self.device)
        _check(self._L.ifnso_orthogonalize(self._h, _ptr(M), int(M.stride(0)), _ptr(Y), int(Y.stride(0)),
                                           _ptr(workspace), nb, _stream(stream)))

    def orthogonalize_static(self, M, Y, stream=None):
        """ifnso_orthogonalize_static: the single problem with the library's fixed scratch area
        (STATIC_SCRATCH_BYTES per GPU) instead of a workspace; allocates nothing. Calls that
        overlap on one GPU race on that area."""
        if len(self.shapes) != 1:
            raise ValueError("orthogonalize_static takes a single-problem plan")
        self.check_io([M], [Y])
        _check(self._L.ifnso_orthogonalize_static(self._h, _ptr(M), int(M.stride(0)), _ptr(Y), int(Y.stride(0)),
                                                  _stream(stream)))

    def orthogonalize_batched(self, Ms, Ys, workspace, stream=None):
        self.check_io(Ms, Ys)
        nb = check_workspace(workspace, self.workspace_bytes, self.device)
        n = len(Ms)
        mp = (ctypes.c_void_p * n)(*[_ptr(m) for m in Ms])
        yp = (ctypes.c_void_p * n)(*[_ptr(y) for y in Ys])
        ldm = (ctypes.c_int64 * n)(*[int(m.stride(0)) for m in Ms])
        ldy = (ctypes.c_int64 * n)(*[int(y.stride(0)) for y in Ys])
        _check(self._L.ifnso_orthogonalize_batched(self._h, mp, ldm, yp, ldy, _ptr(workspace), nb, _stream(stream)))

    def muon_step(self, Ws, Gs, Bs, workspace, lr, momentum, weight_decay=0.0, nesterov=True, stream=None):
        """One Muon step (ifnso_muon_step): Ws, Bs float32 weights and momentum (updated in place),
        Gs gradients in the plan's input type, workspace of muon_workspace_bytes."""
        n = len(Ws)
        if not (len(Gs) == len(Bs) == n == len(self.shapes)):
            raise ValueError(f"{n} weights, {len(Gs)} gradients, {len(Bs)} momenta for a plan of "
                             f"{len(self.shapes)} problems")
        for i, s in enumerate(self.shapes):
            check_matrix(Ws[i], f"W[{i}]", s, F32, self.device)
            check_matrix(Gs[i], f"G[{i}]", s, self.in_dtype, self.device)
            check_matrix(Bs[i], f"B[{i}]", s, F32, self.device)
        nb = check_workspace(workspace, self.muon_workspace_bytes, self.device)
        wp = (ctypes.c_void_p * n)(*[_ptr(w) for w in Ws])
        gp = (ctypes.c_void_p * n)(*[_ptr(g) for g in Gs])
        bp = (ctypes.c_void_p * n)(*[_ptr(b) for b in Bs])
        ldw = (ctypes.c_int64 * n)(*[int(w.stride(0)) for w in Ws])
        ldg = (ctypes.c_int64 * n)(*[int(g.stride(0)) for g in Gs])
        ldb = (ctypes.c_int64 * n)(*[int(b.stride(0)) for b in Bs])
        hp = MuonParams(float(lr), float(momentum), float(weight_decay), 1 if nesterov else 0)
        _check(self._L.ifnso_muon_step(self._h, ctypes.byref(hp), wp, ldw, gp, ldg, bp, ldb, _ptr(workspace), nb,
                                       _stream(stream)))

    @property
    def num_launches(self) -> int:
        return int(self._L.ifnso_plan_num_launches(self._h))

    def launch_info(self, i: int):
        """(stage, algorithmic flops) of launch slot i; stage 0 Gram, 1 squaring, 2 product."""
        st, fl = ctypes.c_int32(), ctypes.c_double()
        _check(self._L.ifnso_plan_launch_info(self._h, int(i), ctypes.byref(st), ctypes.byref(fl)))
        return int(st.value), float(fl.value)

    def get_config(self, stage: int) -> dict:
        c = StageConfig()
        _check(self._L.ifnso_plan_get_config(self._h, int(stage), ctypes.byref(c)))
        return c.as_dict()

    def set_config(self, stage: int, cfg: dict):
        c = StageConfig(**{k: int(v) for k, v in cfg.items()})
        _check(self._L.ifnso_plan_set_config(self._h, int(stage), ctypes.byref(c)))

    def launch_events(self, events):
        """Events (raw hipEvent_t handles) for the next call: one before each slot and one after."""
        n = len(events)
        arr = (ctypes.c_void_p * max(n, 1))(*[int(e) for e in events])
        _check(self._L.ifnso_plan_launch_events(self._h, arr, n))

    def stats(self, stream=None):
        """Per-problem statistics of the last call (see ifnso_plan_stats), as a list of lists."""
        n = len(self.shapes)
        buf = (ctypes.c_double * (n * STATS_PER_PROBLEM))()
        _check(self._L.ifnso_plan_stats(self._h, buf, _stream(stream)))
        return [list(buf[i * STATS_PER_PROBLEM:(i + 1) * STATS_PER_PROBLEM]) for i in range(n)]

    def destroy(self):
        if getattr(self, "_h", None):
            self._L.ifnso_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


class SchedulePlan:
    """Newton-Schulz step schedules over a batch (ifnso_schedule_plan): step k,
    X <- a_k X + b_k (XX^T) X + c_k (XX^T)^2 X, on the batched path; the first step scales the
    input by ||A||_F (gelfand_q = 0) or ||AA^T||_F^(1/2) (gelfand_q = 1), the others not at
    all. The iterates between steps live in the workspace (workspace_bytes)."""

    def __init__(self, schedule, shapes, gelfand_q: int = 0, compute="bf16", device: int = 0):
        L = load()
        self._L = L
        self.schedule = [tuple(float(v) for v in abc) for abc in schedule]
        flat = [v for abc in self.schedule for v in abc]
        if not self.schedule or len(flat) != 3 * len(self.schedule):
            raise ValueError("schedule entries must be (a, b, c) triples")
        self.shapes = [(int(r), int(c)) for r, c in shapes]
        n = len(self.shapes)
        comp = _COMPUTE[compute] if isinstance(compute, str) else int(compute)
        self.dtype = F32 if comp == COMPUTE_F32 else BF16
        self.device = int(device)
        abc_c = (ctypes.c_double * len(flat))(*flat)
        rows = (ctypes.c_int64 * n)(*[r for r, _ in self.shapes])
        cols = (ctypes.c_int64 * n)(*[c for _, c in self.shapes])
        h = ctypes.c_void_p()
        _check(L.ifnso_schedule_plan(abc_c, len(self.schedule), int(gelfand_q), n, rows, cols, self.dtype, comp,
                                     self.device, ctypes.byref(h)))
        self._h = h
        b = ctypes.c_size_t()
        _check(L.ifnso_schedule_plan_workspace_bytes(h, ctypes.byref(b)))
        self.workspace_bytes = b.value

    def orthogonalize_batched(self, Ms, Ys, workspace, stream=None):
        if len(Ms) != len(self.shapes) or len(Ys) != len(self.shapes):
            raise ValueError(f"{len(Ms)} inputs and {len(Ys)} outputs for a schedule of {len(self.shapes)} problems")
        for i, (m, y, s) in enumerate(zip(Ms, Ys, self.shapes)):
            check_matrix(m, f"M[{i}]", s, self.dtype, self.device)
            check_matrix(y, f"Y[{i}]", s, self.dtype, self.device)
        nb = check_workspace(workspace, self.workspace_bytes, self.device)
        n = len(Ms)
        mp = (ctypes.c_void_p * n)(*[_ptr(m) for m in Ms])
        yp = (ctypes.c_void_p * n)(*[_ptr(y) for y in Ys])
        ldm = (ctypes.c_int64 * n)(*[int(m.stride(0)) for m in Ms])
        ldy = (ctypes.c_int64 * n)(*[int(y.stride(0)) for y in Ys])
        _check(self._L.ifnso_schedule_orthogonalize_batched(self._h, mp, ldm, yp, ldy, _ptr(workspace), nb,
                                                            _stream(stream)))

    def destroy(self):
        if getattr(self, "_h", None):
            self._L.ifnso_schedule_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def classical_ns_workspace_bytes(rows: int, cols: int, compute="bf16") -> int:
    comp = _COMPUTE[compute] if isinstance(compute, str) else int(compute)
    return int(load().ifnso_classical_ns_workspace_bytes(rows, cols, comp))


def _ns_args(M, Y, compute, workspace):
    """Checks M, Y (same dtype, shape and GPU, row-major) and the workspace of a single-matrix
    Newton-Schulz call; allocates the workspace (classical_ns_workspace_bytes on M's device)
    when None is passed. Returns (rows, cols, workspace, its size in bytes)."""
    import torch
    if not isinstance(M, torch.Tensor) or M.dim() != 2:
        raise TypeError("M: expected a 2-d torch tensor")
    rows, cols = (int(x) for x in M.shape)
    dt = _dtype_code(M)
    dev = M.device.index if M.device.type == "cuda" else -1
    check_matrix(M, "M", (rows, cols), dt, dev)
    check_matrix(Y, "Y", (rows, cols), dt, dev)
    need = classical_ns_workspace_bytes(rows, cols, compute)
    if workspace is None:
        workspace = torch.empty(need, dtype=torch.uint8, device=M.device)
    return rows, cols, workspace, check_workspace(workspace, need, dev)


def classical_ns(M, Y, steps: int, abc, compute="bf16", workspace=None, stream=None):
    L = load()
    comp = _COMPUTE[compute] if isinstance(compute, str) else int(compute)
    rows, cols, workspace, nb = _ns_args(M, Y, comp, workspace)
    abc_c = (ctypes.c_double * 3)(*[float(x) for x in abc])
    _check(L.ifnso_classical_ns(_ptr(M), rows, cols, int(M.stride(0)), _dtype_code(M), _ptr(Y), int(Y.stride(0)),
                                int(steps), abc_c, comp, _ptr(workspace), nb, _stream(stream)))


def ns_schedule(M, Y, schedule, gelfand_q: int = 0, compute="bf16", workspace=None, stream=None):
    """Newton-Schulz with one (a, b, c) per step (``schedule``: a sequence of triples) and the
    input scaled by ||A||_F (gelfand_q = 0) or by ||(AA^T)^q||_F^(1/(2q)) (q = 1, 2).
    Workspace: classical_ns_workspace_bytes(rows, cols, compute) bytes (allocated here when
    None is passed)."""
    L = load()
    comp = _COMPUTE[compute] if isinstance(compute, str) else int(compute)
    rows, cols, workspace, nb = _ns_args(M, Y, comp, workspace)
    flat = [float(x) for abc in schedule for x in abc]
    if len(flat) != 3 * len(schedule):
        raise ValueError("schedule entries must be (a, b, c) triples")
    abc_c = (ctypes.c_double * max(len(flat), 3))(*flat)
    _check(L.ifnso_ns_schedule(_ptr(M), rows, cols, int(M.stride(0)), _dtype_code(M), _ptr(Y), int(Y.stride(0)),
                               len(schedule), abc_c, int(gelfand_q), comp, _ptr(workspace), nb, _stream(stream)))


def quantize_e4m3_workspace_bytes(rows: int, cols: int) -> int:
    return int(load().ifnso_quantize_e4m3_workspace_bytes(int(rows), int(cols)))


def quantize_e4m3(M, Q, out3, workspace, stream=None):
    """e4m3 copy of A (M, or M^T when tall) into the uint8 matrix Q (h x ldq), with
    out3 (float64, 3) = (||A||_F^2, max |A|, scale)."""
    L = load()
    rows, cols = M.shape
    nb = workspace.numel() * workspace.element_size()
    _check(L.ifnso_quantize_e4m3(_ptr(M), rows, cols, int(M.stride(0)), _ptr(Q), int(Q.stride(0)), _ptr(out3),
                                 _ptr(workspace), nb, _stream(stream)))


def orth_error(Ys, out, workspace, stream=None):
    """float64 ||Z Z^T - I||_F of each matrix (Z in the h <= w orientation) into `out`."""
    L = load()
    n = len(Ys)
    yp = (ctypes.c_void_p * n)(*[_ptr(y) for y in Ys])
    rows = (ctypes.c_int64 * n)(*[y.shape[0] for y in Ys])
    cols = (ctypes.c_int64 * n)(*[y.shape[1] for y in Ys])
    ld = (ctypes.c_int64 * n)(*[int(y.stride(0)) for y in Ys])
    nb = workspace.numel() * workspace.element_size()
    _check(L.ifnso_orth_error(n, yp, rows, cols, ld, _dtype_code(Ys[0]), _ptr(out), _ptr(workspace), nb,
                              _stream(stream)))


def orth_error_workspace_bytes(count: int) -> int:
    return int(load().ifnso_orth_error_workspace_bytes(int(count)))


def mlp_features(sig, nsig, feats_out, stream=None):
    """Device features (n x 8) of zero-padded spectra sig (n x smax float32) with counts nsig."""
    _check(load().ifnso_mlp_features(int(sig.shape[0]), _ptr(sig), _ptr(nsig), int(sig.shape[1]), _ptr(feats_out),
                                     _stream(stream)))


def mlp_forward(feats, params, coeffs_out, stream=None):
    _check(load().ifnso_mlp_forward(int(feats.shape[0]), _ptr(feats), _ptr(params), _ptr(coeffs_out), _stream(stream)))


def mlp_train_workspace_bytes(n: int) -> int:
    return int(load().ifnso_mlp_train_workspace_bytes(int(n)))


def mlp_train_step(feats, sig, nsig, params, adam_m, adam_v, t, lr, workspace, beta1=0.9, beta2=0.999, eps=1e-8,
                   grad_out=None, loss_out=None, stream=None):
    n = int(feats.shape[0])
    nb = workspace.numel() * workspace.element_size()
    _check(load().ifnso_mlp_train_step(n, _ptr(feats), _ptr(sig), _ptr(nsig), int(sig.shape[1]), _ptr(params),
                                       _ptr(adam_m), _ptr(adam_v), int(t), float(lr), float(beta1), float(beta2),
                                       float(eps), _ptr(grad_out) if grad_out is not None else None,
                                       _ptr(loss_out) if loss_out is not None else None, _ptr(workspace), nb,
                                       _stream(stream)))
