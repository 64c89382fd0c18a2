"""Thin Python binding of the C ABI in include/lbm.h (argument marshalling only).

Every step of the method runs in the HIP library ``liblbm.so``; PyTorch is
used only to allocate the device workspace and to supply the HIP stream.
There is no CPU fallback: if the library is missing this module raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "liblbm.so")

LBM_OK, LBM_EINVAL, LBM_ENOMEM, LBM_EDEVICE, LBM_ENONFINITE, LBM_ESTATE = 0, -1, -2, -3, -4, -5
FLOWS = {"ns": 0, "prescribed": 1}
PRECISIONS = {"fp64": 0, "fp32": 1, "fp16dev": 2}
EOS = {"linear": 0, "langmuir": 1}


class LbmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{msg} (status {status})")
        self.status = status


class NonFiniteError(LbmError):
    pass


class lbm_params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("walls_y", ctypes.c_int32), ("eos", ctypes.c_int32),
        ("precision", ctypes.c_int32), ("flow", ctypes.c_int32),
        ("u_wall_bot", ctypes.c_double), ("u_wall_top", ctypes.c_double),
        ("phiA", ctypes.c_double), ("phiB", ctypes.c_double),
        ("W", ctypes.c_double), ("M", ctypes.c_double), ("D", ctypes.c_double),
        ("r", ctypes.c_double), ("rhoA", ctypes.c_double), ("rhoB", ctypes.c_double),
        ("muA", ctypes.c_double), ("muB", ctypes.c_double),
        ("sigma0", ctypes.c_double), ("beta", ctypes.c_double),
        ("gx", ctypes.c_double), ("gy", ctypes.c_double),
        ("s_free", (ctypes.c_double * 3) * 3),
        ("fp16_scale", ctypes.c_double * 3),
    ]


class lbm_moments_t(ctypes.Structure):
    _fields_ = [("step", ctypes.c_int64), ("sum_phi", ctypes.c_double),
                ("sum_psi", ctypes.c_double), ("mom_x", ctypes.c_double),
                ("mom_y", ctypes.c_double), ("kinetic", ctypes.c_double),
                ("max_u", ctypes.c_double), ("nonfinite", ctypes.c_int32),
                ("pad", ctypes.c_int32)]


class lbm_shape_t(ctypes.Structure):
    _fields_ = [(k, ctypes.c_double) for k in
                ("area", "cx", "cy", "Ixx", "Ixy", "Iyy", "length", "taylor_D", "angle")]


class lbm_schedule(ctypes.Structure):
    """Tile-to-wavefront schedule of a batch (see include/lbm.h)."""
    _fields_ = [("rows", ctypes.c_int32), ("grid_waves", ctypes.c_int32),
                ("chunk", ctypes.c_int32), ("reserved", ctypes.c_int32)]


EXPORTS = ("lbm_workspace_bytes", "lbm_create", "lbm_init_fields", "lbm_step",
           "lbm_read_fields", "lbm_moments", "lbm_moments_async", "lbm_state_bytes",
           "lbm_get_state",
           "lbm_set_state", "lbm_destroy", "lbm_last_error", "lbm_set_tile_rows",
           "lbm_get_tile_plan", "lbm_step_kernel_name")

_lib = None


def load(path: str = LIB_PATH):
    """Load liblbm.so and declare the signatures.  Raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with "
                          "`python -m paper_2408_15654_amd.build`")
    # torch first: its HIP runtime (soname libamdhip64.so.7) is then the one
    # the library binds to.  Loaded the other way round, torch would load a
    # second runtime under another file name and the two would not share
    # device memory.
    import torch  # noqa: F401

    lib = ctypes.CDLL(path)
    P = ctypes.POINTER(lbm_params)
    vp, dp, H = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_void_p
    lib.lbm_workspace_bytes.argtypes = [P]
    lib.lbm_workspace_bytes.restype = ctypes.c_size_t
    lib.lbm_create.argtypes = [P, vp, ctypes.c_size_t, vp, ctypes.POINTER(H)]
    lib.lbm_init_fields.argtypes = [H, dp, dp, dp, dp]
    lib.lbm_step.argtypes = [H, ctypes.c_int64]
    lib.lbm_read_fields.argtypes = [H, dp, dp, dp, dp, dp]
    lib.lbm_moments.argtypes = [H, ctypes.POINTER(lbm_moments_t)]
    lib.lbm_moments_async.argtypes = [H, vp]
    lib.lbm_state_bytes.argtypes = [H]
    lib.lbm_state_bytes.restype = ctypes.c_size_t
    lib.lbm_get_state.argtypes = [H, vp, ctypes.c_size_t]
    lib.lbm_set_state.argtypes = [H, vp, ctypes.c_size_t]
    lib.lbm_destroy.argtypes = [H]
    lib.lbm_destroy.restype = None
    lib.lbm_last_error.argtypes = [H]
    lib.lbm_last_error.restype = ctypes.c_char_p
    lib.lbm_set_tile_rows.argtypes = [H, ctypes.c_int32]
    lib.lbm_get_tile_plan.argtypes = [H, ctypes.POINTER(ctypes.c_int32)]
    lib.lbm_step_kernel_name.argtypes = [H]
    lib.lbm_step_kernel_name.restype = ctypes.c_char_p
    for name in ("lbm_create", "lbm_init_fields", "lbm_step", "lbm_read_fields",
                 "lbm_moments", "lbm_moments_async", "lbm_get_state", "lbm_set_state",
                 "lbm_set_tile_rows", "lbm_get_tile_plan"):
        getattr(lib, name).restype = ctypes.c_int
    # batches
    B, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    S = ctypes.POINTER(lbm_schedule)
    lib.lbm_batch_instance_bytes.argtypes = [P]
    lib.lbm_batch_instance_bytes.restype = ctypes.c_size_t
    lib.lbm_batch_overhead_bytes.argtypes = [i32]
    lib.lbm_batch_overhead_bytes.restype = ctypes.c_size_t
    lib.lbm_batch_create.argtypes = [i32, vp, ctypes.c_size_t, vp, ctypes.POINTER(B)]
    lib.lbm_batch_submit.argtypes = [B, P, dp, dp, dp, dp, i64, ctypes.POINTER(i32)]
    lib.lbm_batch_step.argtypes = [B, i64]
    lib.lbm_batch_remaining.argtypes = [B, i32, ctypes.POINTER(i64)]
    lib.lbm_batch_read_fields.argtypes = [B, i32, dp, dp, dp, dp, dp]
    lib.lbm_batch_moments.argtypes = [B, i32, ctypes.POINTER(lbm_moments_t)]
    lib.lbm_batch_retire.argtypes = [B, i32]
    lib.lbm_batch_free_bytes.argtypes = [B]
    lib.lbm_batch_free_bytes.restype = ctypes.c_size_t
    lib.lbm_batch_set_schedule.argtypes = [B, S]
    lib.lbm_batch_get_schedule.argtypes = [B, S]
    lib.lbm_batch_autotune.argtypes = [B, i64, S]
    lib.lbm_shape.argtypes = [H, ctypes.POINTER(lbm_shape_t)]
    lib.lbm_shape.restype = ctypes.c_int
    lib.lbm_batch_shape.argtypes = [B, i32, ctypes.POINTER(lbm_shape_t)]
    lib.lbm_batch_shape.restype = ctypes.c_int
    lib.lbm_batch_destroy.argtypes = [B]
    lib.lbm_batch_destroy.restype = None
    lib.lbm_batch_last_error.argtypes = [B]
    lib.lbm_batch_last_error.restype = ctypes.c_char_p
    for name in ("lbm_batch_create", "lbm_batch_submit", "lbm_batch_step",
                 "lbm_batch_remaining", "lbm_batch_read_fields", "lbm_batch_moments",
                 "lbm_batch_retire", "lbm_batch_set_schedule", "lbm_batch_get_schedule",
                 "lbm_batch_autotune"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def to_c_params(p: dict) -> lbm_params:
    c = lbm_params()
    c.nx, c.ny = int(p["nx"]), int(p["ny"])
    c.walls_y = int(bool(p.get("walls_y", 0)))
    c.eos = EOS[p.get("eos", "linear")] if isinstance(p.get("eos", "linear"), str) else int(p["eos"])
    prec = p.get("precision", "fp64")
    c.precision = PRECISIONS[prec] if isinstance(prec, str) else int(prec)
    fl = p.get("flow", "ns")
    c.flow = FLOWS[fl] if isinstance(fl, str) else int(fl)
    c.u_wall_bot = float(p.get("u_wall_bot", 0.0))
    c.u_wall_top = float(p.get("u_wall_top", 0.0))
    c.phiA = float(p.get("phiA", 1.0))
    c.phiB = float(p.get("phiB", 0.0))
    for k in ("W", "M", "D", "r", "rhoA", "rhoB", "muA", "muB", "sigma0", "beta"):
        setattr(c, k, float(p[k]))
    c.gx = float(p.get("gx", 0.0))
    c.gy = float(p.get("gy", 0.0))
    sf = np.asarray(p.get("s_free", np.ones((3, 3))), dtype=np.float64).reshape(3, 3)
    for a in range(3):
        for b in range(3):
            c.s_free[a][b] = float(sf[a, b])
    fs = p.get("fp16_scale", (0.0, 0.0, 0.0))
    for a in range(3):
        c.fp16_scale[a] = float(fs[a])
    return c


def _dptr(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class Simulation:
    """One simulation on one GPU: workspace, handle and stream."""

    def __init__(self, params: dict, device: str = "cuda:0", stream=None):
        import torch

        self.lib = load()
        self.params = dict(params)
        self._c = to_c_params(params)
        self.nx, self.ny = self._c.nx, self._c.ny
        nbytes = self.lib.lbm_workspace_bytes(ctypes.byref(self._c))
        if nbytes == 0:
            self._handle = None
            raise LbmError(LBM_EINVAL, "invalid parameters")
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        with torch.cuda.device(self.device):
            self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self._handle = ctypes.c_void_p()
        st = self.lib.lbm_create(ctypes.byref(self._c), ctypes.c_void_p(self.workspace.data_ptr()),
                                 nbytes, ctypes.c_void_p(self.stream.cuda_stream),
                                 ctypes.byref(self._handle))
        if st != LBM_OK:
            msg = self.lib.lbm_last_error(None).decode()
            self._handle = None
            raise LbmError(st, msg)

    # --------------------------------------------------------------- api
    def _check(self, st: int):
        if st == LBM_OK:
            return
        msg = self.lib.lbm_last_error(self._handle).decode()
        if st == LBM_ENONFINITE:
            raise NonFiniteError(st, msg)
        raise LbmError(st, msg)

    def _field(self, a):
        a = np.ascontiguousarray(a, dtype=np.float64)
        if a.size != self.nx * self.ny:
            raise ValueError("field has the wrong size")
        return a

    def init_fields(self, phi, psi, ux, uy):
        arrs = [self._field(a) for a in (phi, psi, ux, uy)]
        self._check(self.lib.lbm_init_fields(self._handle, *[_dptr(a) for a in arrs]))

    def step(self, n: int = 1):
        self._check(self.lib.lbm_step(self._handle, int(n)))

    def read_fields(self) -> dict:
        out = {k: np.empty((self.ny, self.nx)) for k in ("phi", "psi", "ux", "uy", "P")}
        self._check(self.lib.lbm_read_fields(self._handle, *[_dptr(out[k]) for k in
                                                            ("phi", "psi", "ux", "uy", "P")]))
        return out

    def moments(self) -> dict:
        m = lbm_moments_t()
        self._check(self.lib.lbm_moments(self._handle, ctypes.byref(m)))
        return {k: getattr(m, k) for k, _ in lbm_moments_t._fields_ if k != "pad"}

    MOMENTS_ASYNC = ("sum_phi", "sum_psi", "mom_x", "mom_y", "kinetic", "max_u", "nonfinite")

    def moments_async(self, out):
        """lbm_moments_async: the float64 sums, in the order of
        MOMENTS_ASYNC, written to the float64 device tensor `out` (7 or more
        elements, on this simulation's device) on the simulation's stream;
        nothing is allocated and nothing waits."""
        import torch

        if (not isinstance(out, torch.Tensor) or out.dtype != torch.float64
                or out.device != self.device or out.numel() < 7 or not out.is_contiguous()):
            raise ValueError("out must be a contiguous float64 tensor of >= 7 elements "
                             "on the simulation's device")
        self._check(self.lib.lbm_moments_async(self._handle, ctypes.c_void_p(out.data_ptr())))

    def shape(self) -> dict:
        """Shape diagnostics of fluid A (area, centroid, moments, interface
        length, Taylor deformation, orientation), reduced on the device."""
        sh = lbm_shape_t()
        self._check(self.lib.lbm_shape(self._handle, ctypes.byref(sh)))
        return {k: getattr(sh, k) for k, _ in lbm_shape_t._fields_}

    def state_bytes(self) -> int:
        return int(self.lib.lbm_state_bytes(self._handle))

    def get_state(self) -> bytes:
        buf = ctypes.create_string_buffer(self.state_bytes())
        self._check(self.lib.lbm_get_state(self._handle, buf, len(buf)))
        return buf.raw

    def set_state(self, data: bytes):
        buf = ctypes.create_string_buffer(data, len(data))
        self._check(self.lib.lbm_set_state(self._handle, buf, len(data)))

    def set_tile_rows(self, rows: int):
        self._check(self.lib.lbm_set_tile_rows(self._handle, int(rows)))

    def tile_plan(self) -> tuple[int, int, int]:
        """(tile height, rows per XCD band in short tiles, their height)."""
        plan = (ctypes.c_int32 * 3)()
        self._check(self.lib.lbm_get_tile_plan(self._handle, plan))
        return tuple(plan)

    def step_kernel_name(self) -> str:
        return self.lib.lbm_step_kernel_name(self._handle).decode()

    def close(self):
        if getattr(self, "_handle", None):
            self.lib.lbm_destroy(self._handle)
            self._handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many independent simulations advanced together on one GPU.

    The workspace (the HBM budget) is one torch tensor of `budget_bytes`;
    simulations are admitted into it with submit() while others run and
    leave with retire().  Every step() advances all of them by up to n
    steps (each stops at its own step count)."""

    def __init__(self, budget_bytes: int, max_instances: int = 1024, device: str = "cuda:0",
                 stream=None):
        import torch

        self.lib = load()
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        with torch.cuda.device(self.device):
            self.workspace = torch.empty(int(budget_bytes), dtype=torch.uint8, device=self.device)
        self._b = ctypes.c_void_p()
        st = self.lib.lbm_batch_create(int(max_instances),
                                       ctypes.c_void_p(self.workspace.data_ptr()),
                                       int(budget_bytes), ctypes.c_void_p(self.stream.cuda_stream),
                                       ctypes.byref(self._b))
        if st != LBM_OK:
            self._b = None
            raise LbmError(st, self.lib.lbm_batch_last_error(None).decode())
        self.shapes = {}

    @staticmethod
    def instance_bytes(params: dict) -> int:
        lib = load()
        c = to_c_params(params)
        return int(lib.lbm_batch_instance_bytes(ctypes.byref(c)))

    @staticmethod
    def overhead_bytes(max_instances: int) -> int:
        return int(load().lbm_batch_overhead_bytes(int(max_instances)))

    def _check(self, st: int):
        if st == LBM_OK:
            return
        msg = self.lib.lbm_batch_last_error(self._b).decode()
        if st == LBM_ENONFINITE:
            raise NonFiniteError(st, msg)
        raise LbmError(st, msg)

    def submit(self, params: dict, phi, psi, ux, uy, nsteps: int) -> int:
        """Admit a simulation; returns its id.  Raises LbmError with status
        LBM_ENOMEM when it does not fit now."""
        c = to_c_params(params)
        n = c.nx * c.ny
        arrs = []
        for a in (phi, psi, ux, uy):
            a = np.ascontiguousarray(a, dtype=np.float64)
            if a.size != n:
                raise ValueError("field has the wrong size")
            arrs.append(a)
        i = ctypes.c_int32()
        self._check(self.lib.lbm_batch_submit(self._b, ctypes.byref(c), *[_dptr(a) for a in arrs],
                                              int(nsteps), ctypes.byref(i)))
        self.shapes[i.value] = (c.ny, c.nx)
        return i.value

    def try_submit(self, params: dict, phi, psi, ux, uy, nsteps: int):
        """submit(), or None when the batch has no room for it now."""
        try:
            return self.submit(params, phi, psi, ux, uy, nsteps)
        except LbmError as e:
            if e.status == LBM_ENOMEM:
                return None
            raise

    def step(self, n: int = 1):
        self._check(self.lib.lbm_batch_step(self._b, int(n)))

    def remaining(self, i: int) -> int:
        r = ctypes.c_int64()
        self._check(self.lib.lbm_batch_remaining(self._b, int(i), ctypes.byref(r)))
        return r.value

    def read_fields(self, i: int) -> dict:
        ny, nx = self.shapes[i]
        out = {k: np.empty((ny, nx)) for k in ("phi", "psi", "ux", "uy", "P")}
        self._check(self.lib.lbm_batch_read_fields(self._b, int(i), *[_dptr(out[k]) for k in
                                                                     ("phi", "psi", "ux", "uy", "P")]))
        return out

    def moments(self, i: int) -> dict:
        m = lbm_moments_t()
        self._check(self.lib.lbm_batch_moments(self._b, int(i), ctypes.byref(m)))
        return {k: getattr(m, k) for k, _ in lbm_moments_t._fields_ if k != "pad"}

    def shape(self, i: int) -> dict:
        sh = lbm_shape_t()
        self._check(self.lib.lbm_batch_shape(self._b, int(i), ctypes.byref(sh)))
        return {k: getattr(sh, k) for k, _ in lbm_shape_t._fields_}

    def retire(self, i: int):
        self._check(self.lib.lbm_batch_retire(self._b, int(i)))
        self.shapes.pop(i, None)

    def free_bytes(self) -> int:
        return int(self.lib.lbm_batch_free_bytes(self._b))

    def set_schedule(self, rows=0, grid_waves=0, chunk=32):
        s = lbm_schedule(int(rows), int(grid_waves), int(chunk), 0)
        self._check(self.lib.lbm_batch_set_schedule(self._b, ctypes.byref(s)))

    def schedule(self) -> dict:
        s = lbm_schedule()
        self._check(self.lib.lbm_batch_get_schedule(self._b, ctypes.byref(s)))
        return {"rows": s.rows, "grid_waves": s.grid_waves, "chunk": s.chunk}

    def autotune(self, probe_steps: int) -> dict:
        s = lbm_schedule()
        self._check(self.lib.lbm_batch_autotune(self._b, int(probe_steps), ctypes.byref(s)))
        return {"rows": s.rows, "grid_waves": s.grid_waves, "chunk": s.chunk}

    def close(self):
        if getattr(self, "_b", None):
            self.lib.lbm_batch_destroy(self._b)
            self._b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
