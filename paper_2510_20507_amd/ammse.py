"""Python binding of libammse (argument marshalling only).

Every function here forwards to the C ABI declared in ``include/ammse.h``;
all arithmetic of the method runs in the library's HIP kernels.  PyTorch is
used for device memory and the current stream.  There is no fallback: if the
shared library is missing or no GPU is present, the calls raise.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libammse.so")

AMMSE_OK = 0
STATUS_NAMES = {0: "OK", 1: "ERR_NULL", 2: "ERR_SHAPE", 3: "ERR_OPTION", 4: "ERR_WORKSPACE",
                5: "ERR_HIP", 6: "ERR_UNSUPPORTED", 7: "ERR_ALLOC"}
PREC_FP64 = 0
PREC_FP32 = 1
PREC_BF16 = 2
PATH_AUTO = 0
PATH_GENERAL = 1
ALGO_AMMMSE = 0
ALGO_WMMSE = 1
ALGO_MMMSE = 2
ALGO_BCGD = 3
STEP_BOUND = 0
STEP_FROZEN = 1
INST_NONFINITE = 1
INST_CHOLESKY = 2
INST_ZERO_POWER = 4

EXPORTED = ("ammse_version", "ammse_status_string", "ammse_default_options", "ammse_validate",
            "ammse_plan_create", "ammse_plan_workspace_size", "ammse_plan_destroy",
            "ammse_solve", "ammse_wsr", "ammse_plan_info", "ammse_unrolled_workspace_size",
            "ammse_unrolled_forward", "ammse_unrolled_backward", "ammse_autotune",
            "ammse_solve_noalloc")
SCRATCH_BYTES = 64 << 20   # AMMSE_SCRATCH_BYTES
KERNEL_LDS_MFMA = 0
KERNEL_GENERAL = 1


class AmmseInstance(ctypes.Structure):
    _fields_ = [("C", ctypes.c_int32), ("U", ctypes.c_int32), ("M", ctypes.c_int32),
                ("N", ctypes.c_int32), ("d", ctypes.c_int32), ("cell_off", ctypes.c_int32),
                ("h_off", ctypes.c_int64), ("v_off", ctypes.c_int64),
                ("user_off", ctypes.c_int64), ("bs_off", ctypes.c_int64)]


class AmmseOptions(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("max_iters", ctypes.c_int32),
                ("T_c", ctypes.c_int32), ("warm_start", ctypes.c_int32),
                ("extrapolate", ctypes.c_int32), ("rearm_at_switch", ctypes.c_int32),
                ("force_switch_iter", ctypes.c_int32), ("lanczos_steps", ctypes.c_int32),
                ("path", ctypes.c_int32), ("refine_iters", ctypes.c_int32),
                ("algorithm", ctypes.c_int32), ("tile", ctypes.c_int32),
                ("step_rule", ctypes.c_int32), ("eps1", ctypes.c_double),
                ("eps2", ctypes.c_double), ("gamma_c", ctypes.c_double)]


class AmmseError(RuntimeError):
    def __init__(self, code: int, where: str):
        super().__init__(f"{where}: {STATUS_NAMES.get(code, code)} ({_status_text(code)})")
        self.code = code


_lib = None


def lib() -> ctypes.CDLL:
    """Load libammse.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    # torch first: the library must bind to the HIP runtime torch has loaded
    # (loaded before torch it would pull in a second runtime, and device
    # pointers from torch would be invalid in it)
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    P = ctypes.POINTER
    L.ammse_version.restype = i32
    L.ammse_version.argtypes = []
    L.ammse_status_string.restype = ctypes.c_char_p
    L.ammse_status_string.argtypes = [i32]
    L.ammse_default_options.restype = None
    L.ammse_default_options.argtypes = [P(AmmseOptions)]
    L.ammse_validate.restype = i32
    L.ammse_validate.argtypes = [P(AmmseInstance), P(i32), i32, P(AmmseOptions), P(i64), P(i64),
                                 P(i64), P(i64)]
    L.ammse_plan_create.restype = i32
    L.ammse_plan_create.argtypes = [P(vp), i32, P(AmmseInstance), P(i32), i32, P(AmmseOptions)]
    L.ammse_plan_workspace_size.restype = i32
    L.ammse_plan_workspace_size.argtypes = [vp, P(sz)]
    L.ammse_plan_info.restype = i32
    L.ammse_plan_info.argtypes = [vp, P(i32), P(sz)]
    L.ammse_plan_destroy.restype = i32
    L.ammse_plan_destroy.argtypes = [vp]
    L.ammse_solve.restype = i32
    L.ammse_solve.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, sz, vp]
    L.ammse_solve_noalloc.restype = i32
    L.ammse_solve_noalloc.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    L.ammse_wsr.restype = i32
    L.ammse_wsr.argtypes = [vp, vp, vp, vp, vp, vp, vp, sz, vp]
    L.ammse_autotune.restype = i32
    L.ammse_autotune.argtypes = [vp, vp, vp, vp, vp, vp, vp, sz, P(i32), vp]
    L.ammse_unrolled_workspace_size.restype = i32
    L.ammse_unrolled_workspace_size.argtypes = [vp, i32, P(sz), P(sz)]
    L.ammse_unrolled_forward.restype = i32
    L.ammse_unrolled_forward.argtypes = [vp, vp, vp, vp, vp, vp, vp, i32, vp, vp, vp, vp, vp, vp,
                                         vp, sz, vp]
    L.ammse_unrolled_backward.restype = i32
    L.ammse_unrolled_backward.argtypes = [vp, vp, vp, vp, vp, vp, i32, vp, vp, vp, vp, vp, vp,
                                          sz, vp]
    _lib = L
    return L


def _status_text(code: int) -> str:
    try:
        return lib().ammse_status_string(int(code)).decode()
    except Exception:  # library not loadable: plain name only
        return STATUS_NAMES.get(code, "?")


def _check(code: int, where: str) -> None:
    if code != AMMSE_OK:
        raise AmmseError(code, where)


@dataclasses.dataclass
class Options:
    """Mirror of ammse_options_t (defaults: the paper's settings, FP32)."""
    precision: int = PREC_FP32
    max_iters: int = 100
    T_c: int = 3
    warm_start: int = 1
    extrapolate: int = 1
    rearm_at_switch: int = 1
    force_switch_iter: int = -1
    lanczos_steps: int = 0
    path: int = 0
    refine_iters: int = 10
    algorithm: int = ALGO_AMMMSE
    tile: int = 0            # 0: plan's (autotuned) tile shapes; v + 1: force shape v
    step_rule: int = 0       # STEP_BOUND (stage-II step 1/Lhat) or STEP_FROZEN
    eps1: float = 0.1
    eps2: float = 0.0
    gamma_c: float = 0.0

    def to_c(self) -> AmmseOptions:
        o = AmmseOptions()
        for f in dataclasses.fields(self):
            setattr(o, f.name, getattr(self, f.name))
        return o


def make_table(batch) -> tuple:
    """ammse_instance_t array and cell_users (int32) from a synth.Batch."""
    B = batch.batch
    table = (AmmseInstance * B)()
    for i in range(B):
        t = table[i]
        t.C, t.U, t.M, t.N, t.d = (int(batch.C[i]), int(batch.U[i]), int(batch.M[i]),
                                   int(batch.N[i]), int(batch.d[i]))
        t.cell_off = int(batch.cell_off[i])
        t.h_off, t.v_off = int(batch.h_off[i]), int(batch.v_off[i])
        t.user_off, t.bs_off = int(batch.user_off[i]), int(batch.bs_off[i])
    cu = np.ascontiguousarray(batch.cell_users, np.int32)
    return table, cu


def validate(table, cell_users: np.ndarray, options: Optional[Options] = None) -> tuple:
    """ammse_validate: returns the minimum lengths (H, V, users, BSs)."""
    L = lib()
    out = [ctypes.c_int64() for _ in range(4)]
    opt = (options or Options()).to_c()
    cu = np.ascontiguousarray(cell_users, np.int32)
    n = len(table)
    code = L.ammse_validate(table if n else None,
                            cu.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)) if n else None,
                            n, ctypes.byref(opt), *[ctypes.byref(x) for x in out])
    _check(code, "ammse_validate")
    return tuple(int(x.value) for x in out)


def _ptr(t) -> Optional[int]:
    return None if t is None else int(t.data_ptr())


class Plan:
    """A plan on one device for a fixed instance table (ammse_plan_create)."""

    def __init__(self, table, cell_users: np.ndarray, options: Options, device: int = 0):
        L = lib()
        self.options = options
        self.batch = len(table)
        self.device = device
        self._table = table
        cu = np.ascontiguousarray(cell_users, np.int32)
        self._handle = ctypes.c_void_p()
        opt = options.to_c()
        code = L.ammse_plan_create(ctypes.byref(self._handle), device, table,
                                   cu.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                   self.batch, ctypes.byref(opt))
        _check(code, "ammse_plan_create")
        ws = ctypes.c_size_t()
        _check(L.ammse_plan_workspace_size(self._handle, ctypes.byref(ws)),
               "ammse_plan_workspace_size")
        self.workspace_bytes = int(ws.value)
        kern, lds = ctypes.c_int32(), ctypes.c_size_t()
        _check(L.ammse_plan_info(self._handle, ctypes.byref(kern), ctypes.byref(lds)),
               "ammse_plan_info")
        self.kernel = int(kern.value)
        self.lds_bytes = int(lds.value)

    def close(self):
        if getattr(self, "_handle", None) is not None and self._handle.value:
            lib().ammse_plan_destroy(self._handle)
            self._handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def workspace(self):
        import torch
        # 256-byte alignment is guaranteed by the caching allocator (512 B blocks)
        return torch.empty(self.workspace_bytes, dtype=torch.uint8, device=f"cuda:{self.device}")

    def solve(self, H, sigma2, alpha, P, V, wsr, iters=None, switch_iter=None, status=None,
              trace=None, force_switch=None, workspace=None, stream=None):
        """ammse_solve on device tensors (V is updated in place)."""
        import torch
        if workspace is None:
            workspace = self.workspace()
        if stream is None:
            stream = torch.cuda.current_stream(self.device).cuda_stream
        code = lib().ammse_solve(self._handle, _ptr(H), _ptr(sigma2), _ptr(alpha), _ptr(P),
                                 _ptr(V), _ptr(wsr), _ptr(iters), _ptr(switch_iter),
                                 _ptr(status), _ptr(trace), _ptr(force_switch), _ptr(workspace),
                                 workspace.numel() * workspace.element_size(), stream)
        _check(code, "ammse_solve")

    def solve_noalloc(self, H, sigma2, alpha, P, V, wsr, iters=None, switch_iter=None,
                      status=None, trace=None, force_switch=None, stream=None):
        """ammse_solve_noalloc on device tensors: as solve(), with the library's
        static workspace array instead of a caller workspace."""
        import torch
        if stream is None:
            stream = torch.cuda.current_stream(self.device).cuda_stream
        code = lib().ammse_solve_noalloc(self._handle, _ptr(H), _ptr(sigma2), _ptr(alpha),
                                         _ptr(P), _ptr(V), _ptr(wsr), _ptr(iters),
                                         _ptr(switch_iter), _ptr(status), _ptr(trace),
                                         _ptr(force_switch), stream)
        _check(code, "ammse_solve_noalloc")

    def unrolled_sizes(self, ckpt_every: int) -> tuple:
        """(workspace bytes, checkpoint bytes) of the unrolled solver."""
        ws, ck = ctypes.c_size_t(), ctypes.c_size_t()
        _check(lib().ammse_unrolled_workspace_size(self._handle, int(ckpt_every), ctypes.byref(ws),
                                                   ctypes.byref(ck)),
               "ammse_unrolled_workspace_size")
        return int(ws.value), int(ck.value)

    def unrolled_forward(self, H, sigma2, alpha, P, V, gamma, ckpt_every, wsr, switch_iter, ckpt,
                         workspace, status=None, trace=None, force_switch=None, stream=None):
        """ammse_unrolled_forward on device tensors (V: in V^0, out V^T)."""
        import torch
        if stream is None:
            stream = torch.cuda.current_stream(self.device).cuda_stream
        code = lib().ammse_unrolled_forward(
            self._handle, _ptr(H), _ptr(sigma2), _ptr(alpha), _ptr(P), _ptr(V), _ptr(gamma),
            int(ckpt_every), _ptr(wsr), _ptr(switch_iter), _ptr(status), _ptr(trace),
            _ptr(force_switch), _ptr(ckpt), _ptr(workspace),
            workspace.numel() * workspace.element_size(), stream)
        _check(code, "ammse_unrolled_forward")

    def unrolled_backward(self, H, sigma2, alpha, P, gamma, ckpt_every, switch_iter, ckpt, dwsr,
                          dH, dgamma, workspace, stream=None):
        """ammse_unrolled_backward on device tensors."""
        import torch
        if stream is None:
            stream = torch.cuda.current_stream(self.device).cuda_stream
        code = lib().ammse_unrolled_backward(
            self._handle, _ptr(H), _ptr(sigma2), _ptr(alpha), _ptr(P), _ptr(gamma),
            int(ckpt_every), _ptr(switch_iter), _ptr(ckpt), _ptr(dwsr), _ptr(dH), _ptr(dgamma),
            _ptr(workspace), workspace.numel() * workspace.element_size(), stream)
        _check(code, "ammse_unrolled_backward")

    def autotune(self, H, sigma2, alpha, P, V, workspace=None, stream=None) -> list:
        """ammse_autotune on device tensors (V is only read); returns the tile
        shape picked per shape class (-1: class absent or nothing to tune)."""
        import torch
        if workspace is None:
            workspace = self.workspace()
        if stream is None:
            stream = torch.cuda.current_stream(self.device).cuda_stream
        choice = (ctypes.c_int32 * 3)()
        code = lib().ammse_autotune(self._handle, _ptr(H), _ptr(sigma2), _ptr(alpha), _ptr(P),
                                    _ptr(V), _ptr(workspace),
                                    workspace.numel() * workspace.element_size(), choice, stream)
        _check(code, "ammse_autotune")
        return [int(c) for c in choice]

    def wsr(self, H, sigma2, alpha, V, wsr, workspace=None, stream=None):
        """ammse_wsr on device tensors."""
        import torch
        if workspace is None:
            workspace = self.workspace()
        if stream is None:
            stream = torch.cuda.current_stream(self.device).cuda_stream
        code = lib().ammse_wsr(self._handle, _ptr(H), _ptr(sigma2), _ptr(alpha), _ptr(V),
                               _ptr(wsr), _ptr(workspace),
                               workspace.numel() * workspace.element_size(), stream)
        _check(code, "ammse_wsr")


@dataclasses.dataclass
class DeviceBatch:
    """A synth.Batch resident in device memory in the library's layout."""
    H: "object"
    sigma2: "object"
    alpha: "object"
    P: "object"
    V0: "object"
    table: "object"
    cell_users: np.ndarray
    precision: int


def to_device(batch, precision: int = PREC_FP32, device: int = 0) -> DeviceBatch:
    import torch
    cdt = torch.complex128 if precision == PREC_FP64 else torch.complex64   # BF16 mode: float I/O
    dev = f"cuda:{device}"
    table, cu = make_table(batch)
    return DeviceBatch(
        H=torch.from_numpy(batch.H).to(dev, cdt).contiguous(),
        sigma2=torch.from_numpy(batch.sigma2).to(dev, torch.float64),
        alpha=torch.from_numpy(batch.alpha).to(dev, torch.float64),
        P=torch.from_numpy(batch.P).to(dev, torch.float64),
        V0=torch.from_numpy(batch.V0).to(dev, cdt).contiguous(),
        table=table, cell_users=cu, precision=precision)


@dataclasses.dataclass
class Result:
    V: np.ndarray
    wsr: np.ndarray
    iters: np.ndarray
    switch_iter: np.ndarray
    status: np.ndarray
    trace: Optional[np.ndarray]


def solve(batch, options: Optional[Options] = None, device: int = 0, want_trace: bool = False,
          force_switch: Optional[np.ndarray] = None, autotune: bool = False) -> Result:
    """Convenience wrapper: upload a synth.Batch, run ammse_solve, download
    (with ``autotune``, ammse_autotune picks the plan's tile shapes first)."""
    import torch
    options = options or Options()
    db = to_device(batch, options.precision, device)
    plan = Plan(db.table, db.cell_users, options, device)
    dev = f"cuda:{device}"
    B = batch.batch
    V = db.V0.clone()
    wsr = torch.empty(B, dtype=torch.float64, device=dev)
    iters = torch.empty(B, dtype=torch.int32, device=dev)
    sw = torch.empty(B, dtype=torch.int32, device=dev)
    st = torch.empty(B, dtype=torch.int32, device=dev)
    trace = (torch.empty((B, options.max_iters + 1), dtype=torch.float64, device=dev)
             if want_trace else None)
    fs = (torch.from_numpy(np.ascontiguousarray(force_switch, np.int32)).to(dev)
          if force_switch is not None else None)
    if autotune:
        plan.autotune(db.H, db.sigma2, db.alpha, db.P, V)
    plan.solve(db.H, db.sigma2, db.alpha, db.P, V, wsr, iters, sw, st, trace, fs)
    torch.cuda.synchronize(device)
    out = Result(V=V.cpu().numpy().astype(np.complex128), wsr=wsr.cpu().numpy(),
                 iters=iters.cpu().numpy(), switch_iter=sw.cpu().numpy(), status=st.cpu().numpy(),
                 trace=trace.cpu().numpy() if trace is not None else None)
    plan.close()
    return out


def wsr(batch, V: Optional[np.ndarray] = None, precision: int = PREC_FP32,
        device: int = 0) -> np.ndarray:
    """Convenience wrapper around ammse_wsr (V defaults to the batch's V0)."""
    import torch
    db = to_device(batch, precision, device)
    opt = Options(precision=precision, max_iters=0)
    plan = Plan(db.table, db.cell_users, opt, device)
    dev = f"cuda:{device}"
    cdt = torch.complex128 if precision == PREC_FP64 else torch.complex64   # BF16 mode: float I/O
    Vt = db.V0 if V is None else torch.from_numpy(np.asarray(V)).to(dev, cdt).contiguous()
    out = torch.empty(batch.batch, dtype=torch.float64, device=dev)
    plan.wsr(db.H, db.sigma2, db.alpha, Vt, out)
    torch.cuda.synchronize(device)
    plan.close()
    return out.cpu().numpy()
