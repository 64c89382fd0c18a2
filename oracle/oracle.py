"""ctypes shim over the FP64 C oracle (``lbm_oracle.c``).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark use it; the library never does.  It takes the same plain
parameter dictionary as the HIP binding (keys listed in ``PARAM_KEYS``) and
plain float64 arrays of shape (ny, nx), x fastest.

State layout (numpy, float64): ``f``, ``g``, ``h`` of shape (9, ny, nx) hold
the post-collision populations of the previous step; ``aux`` of shape
(6, ny, nx) holds (phi, psi, ux, uy, Sx, Sy) of the previous time level.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import time

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
# A prebuilt copy elsewhere (used to check that the pins catch planted
# mistakes in a modified copy of the oracle source).
_LIB_OVERRIDE = os.environ.get("LBM_ORACLE_LIB")

PARAM_KEYS = ("nx", "ny", "walls_y", "eos", "flow", "u_wall_bot", "u_wall_top", "phiA",
              "phiB", "W", "M", "D", "r", "rhoA", "rhoB", "muA", "muB",
              "sigma0", "beta", "gx", "gy", "s_free")


class _Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("walls_y", ctypes.c_int32), ("eos", ctypes.c_int32),
        ("flow", ctypes.c_int32), ("pad", ctypes.c_int32),
        ("u_wall_bot", ctypes.c_double), ("u_wall_top", ctypes.c_double),
        ("phiA", ctypes.c_double), ("phiB", ctypes.c_double),
        ("W", ctypes.c_double), ("M", ctypes.c_double),
        ("D", ctypes.c_double), ("r", ctypes.c_double),
        ("rhoA", ctypes.c_double), ("rhoB", ctypes.c_double),
        ("muA", ctypes.c_double), ("muB", ctypes.c_double),
        ("sigma0", ctypes.c_double), ("beta", ctypes.c_double),
        ("gx", ctypes.c_double), ("gy", ctypes.c_double),
        ("s_free", (ctypes.c_double * 3) * 3),
        ("s0", ctypes.c_double), ("rho0", ctypes.c_double),
    ]


SITE_FIELDS = ("phi", "psi", "rho", "ux", "uy", "Sx", "Sy", "P", "delta", "nx",
               "ny", "a", "gpsix", "gpsiy", "dphiux", "dphiuy", "dpsiux",
               "dpsiuy", "dTxx", "dTxy", "dTyy", "grhox", "grhoy", "Fx", "Fy")


class Site(ctypes.Structure):
    _fields_ = [(k, ctypes.c_double) for k in SITE_FIELDS]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (no fused multiply-add, no fast math)."""
    if _LIB_OVERRIDE and not force:
        return _LIB_OVERRIDE
    if (force or not os.path.exists(_LIB)
            or os.path.getmtime(_LIB) < os.path.getmtime(_SRC)):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC",
                               "-ffp-contract=off", "-shared", "-o", tmp, _SRC,
                               "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        dp = ctypes.POINTER(ctypes.c_double)
        pp = ctypes.POINTER(_Params)
        _lib.or_init.argtypes = [pp, dp, dp, dp, dp, dp, dp, dp, dp]
        _lib.or_step.argtypes = [pp, dp, dp, dp, dp, ctypes.c_int64]
        _lib.or_macros.argtypes = [pp, dp, dp, dp, dp, dp, dp, dp, dp, dp]
        _lib.or_site_fields.argtypes = [pp, dp, dp, dp, dp, ctypes.POINTER(Site)]
        _lib.or_stencils.argtypes = [pp, dp, dp, dp, dp]
        _lib.or_site_distributions.argtypes = [pp, ctypes.POINTER(Site)] + [dp] * 6
        _lib.or_collide.argtypes = [dp] * 5
        _lib.or_matrices.argtypes = [dp, dp]
        assert _lib.or_sizeof_site() == ctypes.sizeof(Site)
        assert _lib.or_sizeof_params() == ctypes.sizeof(_Params)
    return _lib


def make_params(p: dict) -> _Params:
    """Plain parameter dict -> C struct (defaults for optional keys)."""
    c = _Params()
    c.nx, c.ny = int(p["nx"]), int(p["ny"])
    c.walls_y = int(bool(p.get("walls_y", 0)))
    eos = p.get("eos", "linear")
    c.eos = {"linear": 0, "langmuir": 1, 0: 0, 1: 1}[eos]
    flow = p.get("flow", "ns")
    c.flow = {"ns": 0, "prescribed": 1, 0: 0, 1: 1}[flow]
    for k in ("u_wall_bot", "u_wall_top", "gx", "gy"):
        setattr(c, k, float(p.get(k, 0.0)))
    c.phiA = float(p.get("phiA", 1.0))
    c.phiB = float(p.get("phiB", 0.0))
    for k in ("W", "M", "D", "r", "rhoA", "rhoB", "muA", "muB", "sigma0", "beta"):
        setattr(c, k, float(p[k]))
    sf = np.asarray(p.get("s_free", np.ones((3, 3))), dtype=np.float64).reshape(3, 3)
    for a in range(3):
        for b in range(3):
            c.s_free[a][b] = float(sf[a, b])
    c.s0 = float(p.get("s0", 1.0))
    c.rho0 = float(p.get("rho0", 0.0))
    return c


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class OracleSim:
    """The oracle's state for one problem, advanced in place."""

    def __init__(self, params: dict, phi0, psi0, ux0, uy0):
        self.params = dict(params)
        self.cp = make_params(params)
        ny, nx = self.cp.ny, self.cp.nx
        self.shape = (ny, nx)
        self.f = np.zeros((9, ny, nx))
        self.g = np.zeros((9, ny, nx))
        self.h = np.zeros((9, ny, nx))
        self.aux = np.zeros((6, ny, nx))
        self.step_count = 0
        arrs = [np.ascontiguousarray(a, dtype=np.float64).reshape(ny, nx)
                for a in (phi0, psi0, ux0, uy0)]
        rc = lib().or_init(ctypes.byref(self.cp), *[_ptr(a) for a in arrs],
                           _ptr(self.f), _ptr(self.g), _ptr(self.h), _ptr(self.aux))
        if rc != 0:
            raise ValueError(f"oracle init rejected the problem (rc={rc})")

    def step(self, n: int = 1) -> None:
        rc = lib().or_step(ctypes.byref(self.cp), _ptr(self.f), _ptr(self.g),
                           _ptr(self.h), _ptr(self.aux), int(n))
        if rc != 0:
            raise RuntimeError(f"oracle step failed (rc={rc})")
        self.step_count += n

    def fields(self) -> dict:
        """phi, psi, ux, uy, P of the current time level."""
        out = {k: np.zeros(self.shape) for k in ("phi", "psi", "ux", "uy", "P")}
        rc = lib().or_macros(ctypes.byref(self.cp), _ptr(self.f), _ptr(self.g),
                             _ptr(self.h), _ptr(self.aux),
                             *[_ptr(out[k]) for k in ("phi", "psi", "ux", "uy", "P")])
        if rc != 0:
            raise RuntimeError("oracle macros failed")
        return out

    def site_fields(self) -> dict:
        """All per-site macroscopic quantities of the current level."""
        n = self.shape[0] * self.shape[1]
        arr = (Site * n)()
        rc = lib().or_site_fields(ctypes.byref(self.cp), _ptr(self.f), _ptr(self.g),
                                  _ptr(self.h), _ptr(self.aux), arr)
        if rc != 0:
            raise RuntimeError("oracle site_fields failed")
        raw = np.ctypeslib.as_array(ctypes.cast(arr, ctypes.POINTER(ctypes.c_double)),
                                    shape=(n, len(SITE_FIELDS))).copy()
        return {k: raw[:, i].reshape(self.shape) for i, k in enumerate(SITE_FIELDS)}

    def moments(self) -> dict:
        """Domain sums of the current level (FP64)."""
        fl = self.fields()
        p = self.params
        phiA, phiB = p.get("phiA", 1.0), p.get("phiB", 0.0)
        rho = (fl["phi"] - phiB) / (phiA - phiB) * (p["rhoA"] - p["rhoB"]) + p["rhoB"]
        umag = np.hypot(fl["ux"], fl["uy"])
        return {"sum_phi": float(fl["phi"].sum()), "sum_psi": float(fl["psi"].sum()),
                "mom_x": float((rho * fl["ux"]).sum()),
                "mom_y": float((rho * fl["uy"]).sum()),
                "kinetic": float((0.5 * rho * umag ** 2).sum()),
                "max_u": float(umag.max())}


def stencils(params: dict, a: np.ndarray):
    cp = make_params(params)
    a = np.ascontiguousarray(a, dtype=np.float64)
    gx, gy, lp = (np.zeros_like(a) for _ in range(3))
    lib().or_stencils(ctypes.byref(cp), _ptr(a), _ptr(gx), _ptr(gy), _ptr(lp))
    return gx, gy, lp


def site_distributions(params: dict, site: dict):
    """feq, F, geq, G, heq, H (each length 9) for one site's inputs."""
    cp = make_params(params)
    s = Site(**{k: float(site.get(k, 0.0)) for k in SITE_FIELDS})
    outs = [np.zeros(9) for _ in range(6)]
    lib().or_site_distributions(ctypes.byref(cp), ctypes.byref(s), *[_ptr(o) for o in outs])
    return outs


def collide(f, feq, F, S):
    out = np.zeros(9)
    arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (f, feq, F, S)]
    lib().or_collide(*[_ptr(a) for a in arrs], _ptr(out))
    return out


def matrices():
    M = np.zeros(81)
    Mi = np.zeros(81)
    lib().or_matrices(_ptr(M), _ptr(Mi))
    return M.reshape(9, 9), Mi.reshape(9, 9)


def time_mlups(params: dict, fields0, nsteps: int, threads: int | None = None):
    """Wall-clock MLUPS of the oracle on a problem (CPU baseline)."""
    if threads is not None:
        lib().or_set_threads(int(threads))
    sim = OracleSim(params, *fields0)
    t0 = time.perf_counter()
    sim.step(nsteps)
    dt = time.perf_counter() - t0
    return sim.shape[0] * sim.shape[1] * nsteps / dt / 1e6, dt


def threads() -> int:
    return int(lib().or_get_threads())
