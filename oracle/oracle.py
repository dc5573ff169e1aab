"""Python front of the FP64 CPU oracle (oracle/lbcg_oracle.c).

TEST INFRASTRUCTURE ONLY. The oracle is the plain, slow reference that the GPU library is
checked against; only the test suite, the smoke check and the benchmark's CPU-baseline leg use
it. Nothing here is imported by the product package, and nothing here imports it.

Parameters are passed as a plain dict with the keys of ``PARAM_KEYS``; arrays are float64 numpy
arrays in the C layout: populations (q, nz, ny, nx), scalar fields (nz, ny, nx).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbcg_oracle.so")
SRC_PATH = os.path.join(HERE, "lbcg_oracle.c")

PARAM_KEYS = ("dim", "nx", "ny", "nz", "flow", "xbc", "W0", "tau0", "lam", "D", "eps", "nu",
              "h_drag", "u_in", "U0", "U_in", "seed_c", "seed_R", "grad_eps2")


class OrcParams(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("nz", ctypes.c_int32), ("flow", ctypes.c_int32), ("xbc", ctypes.c_int32),
        ("W0", ctypes.c_double), ("tau0", ctypes.c_double), ("lam", ctypes.c_double),
        ("D", ctypes.c_double), ("eps", ctypes.c_double),
        ("nu", ctypes.c_double), ("h_drag", ctypes.c_double), ("u_in", ctypes.c_double),
        ("U0", ctypes.c_double), ("U_in", ctypes.c_double),
        ("seed_c", ctypes.c_double * 3), ("seed_R", ctypes.c_double),
        ("grad_eps2", ctypes.c_double),
        ("wall", ctypes.c_void_p),
        ("seed_shape", ctypes.c_int32),
        ("seed_tilt", ctypes.c_double),
        ("collision", ctypes.c_int32),
        ("omega_bulk", ctypes.c_double),
        ("solute_source", ctypes.c_int32),
    ]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C11, FP64, OpenMP, no FMA contraction)."""
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC_PATH):
        cmd = ["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
               SRC_PATH, "-o", LIB_PATH + ".tmp", "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        pp = ctypes.POINTER(OrcParams)
        L.orc_lattice.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                  ctypes.POINTER(ctypes.c_int), dp, dp]
        L.orc_aniso.argtypes = [ctypes.c_double, ctypes.c_double, dp, dp, dp]
        L.orc_aniso.restype = None
        L.orc_init.argtypes = [pp, dp, dp, dp, dp]
        L.orc_flow_equilibrium.argtypes = [pp, dp, dp, dp, dp, dp]
        L.orc_step.argtypes = [pp, dp, dp, dp, dp, ctypes.c_int64]
        L.orc_fields.argtypes = [pp, dp, dp, dp, dp, dp, dp, dp, dp, dp]
        L.orc_measure.argtypes = [pp, dp, dp, dp, dp, ctypes.c_int, dp, dp, dp]
        L.orc_raymarch.argtypes = [pp, dp, ctypes.c_int, dp, dp]
        L.orc_num_threads.argtypes = []
        L.orc_set_num_threads.argtypes = [ctypes.c_int]
        L.orc_seed_distance.argtypes = [ctypes.POINTER(OrcParams), ctypes.c_double, ctypes.c_double, ctypes.c_double]
        L.orc_seed_distance.restype = ctypes.c_double
        L.orc_set_num_threads.restype = None
        _lib = L
    return _lib


def _dp(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def make_params(p: dict) -> OrcParams:
    s = OrcParams()
    for k in PARAM_KEYS:
        v = p[k]
        if k == "seed_c":
            for d in range(3):
                s.seed_c[d] = float(v[d])
        elif k in ("dim", "nx", "ny", "nz", "flow", "xbc"):
            setattr(s, k, int(v))
        else:
            setattr(s, k, float(v))
    s.seed_shape = int(p.get("seed_shape", 0))
    s.seed_tilt = float(p.get("seed_tilt", 0.0))
    s.collision = int(p.get("collision", 0))
    s.omega_bulk = float(p.get("omega_bulk", 1.0))
    s.solute_source = int(p.get("solute_source", 0))
    return s


def lattice(kind: int):
    """kind 0 D2Q5, 1 D3Q7, 2 D2Q9, 3 D3Q19 -> (c [q,3] int, w [q], cs2)."""
    q = ctypes.c_int()
    c = (ctypes.c_int * 57)()
    w = np.zeros(19)
    cs2 = ctypes.c_double()
    rc = lib().orc_lattice(kind, ctypes.byref(q), c, _dp(w), ctypes.byref(cs2))
    assert rc == 0
    n = q.value
    return np.array(c[: 3 * n], dtype=np.int64).reshape(n, 3), w[:n].copy(), cs2.value


def aniso(eps: float, p, grad_eps2: float = 1e-12):
    pv = np.ascontiguousarray(np.asarray(p, dtype=np.float64).reshape(3))
    a = ctypes.c_double()
    N = np.zeros(3)
    lib().orc_aniso(eps, grad_eps2, _dp(pv), ctypes.byref(a), _dp(N))
    return a.value, N


def num_threads() -> int:
    return int(lib().orc_num_threads())


def seed_distance(p: dict, dx: float, dy: float, dz: float = 0.0) -> float:
    cp = make_params(p)
    return float(lib().orc_seed_distance(ctypes.byref(cp), dx, dy, dz))


def set_num_threads(n: int):
    lib().orc_set_num_threads(int(n))


class Sim:
    """One oracle simulation: owns the FP64 state arrays."""

    def __init__(self, p: dict, init: bool = True):
        self.p = dict(p)
        self.cp = make_params(self.p)
        self.shape = (int(p["nz"]), int(p["ny"]), int(p["nx"]))
        self.qs = 5 if p["dim"] == 2 else 7
        self.qf = 9 if p["dim"] == 2 else 19
        self.h = np.zeros((self.qs,) + self.shape)
        self.g = np.zeros((self.qs,) + self.shape)
        self.f = np.zeros((self.qf,) + self.shape) if p["flow"] else None
        self.phi_prev = np.zeros(self.shape)
        self.nstep = 0
        if init:
            rc = lib().orc_init(ctypes.byref(self.cp), _dp(self.h), _dp(self.g), _dp(self.f),
                                _dp(self.phi_prev))
            if rc != 0:
                raise ValueError("oracle rejected the parameters")

    def set_walls(self, mask):
        """Solid wall nodes (nonzero entries of a (nz, ny, nx) mask), or None for none."""
        if mask is None:
            self.wall = None
            self.cp.wall = None
            return
        self.wall = np.ascontiguousarray(np.broadcast_to(mask, self.shape), dtype=np.uint8)
        self.cp.wall = self.wall.ctypes.data

    def set_flow_equilibrium(self, rho, ux, uy, uz=None):
        arrs = [np.ascontiguousarray(np.broadcast_to(np.asarray(a, dtype=np.float64), self.shape))
                for a in (rho, ux, uy, 0.0 if uz is None else uz)]
        rc = lib().orc_flow_equilibrium(ctypes.byref(self.cp), *[_dp(a) for a in arrs], _dp(self.f))
        assert rc == 0

    def step(self, n: int = 1):
        rc = lib().orc_step(ctypes.byref(self.cp), _dp(self.h), _dp(self.g), _dp(self.f),
                            _dp(self.phi_prev), int(n))
        if rc != 0:
            raise ValueError("oracle step failed")
        self.nstep += n

    def fields(self) -> dict:
        out = {k: np.zeros(self.shape) for k in ("phi", "U", "rho", "ux", "uy", "uz")}
        rc = lib().orc_fields(ctypes.byref(self.cp), _dp(self.h), _dp(self.g), _dp(self.f),
                              *[_dp(out[k]) for k in ("phi", "U", "rho", "ux", "uy", "uz")])
        assert rc == 0
        return out

    def measure(self, dirs=None):
        """Returns (L [ndirs], mass dict)."""
        dirs = np.zeros((0, 3)) if dirs is None else np.ascontiguousarray(dirs, dtype=np.float64)
        nd = dirs.shape[0]
        L = np.zeros(max(nd, 1))
        m = np.zeros(6)
        rc = lib().orc_measure(ctypes.byref(self.cp), _dp(self.h), _dp(self.g), _dp(self.f),
                               _dp(self.phi_prev), nd, _dp(dirs) if nd else None, _dp(L), _dp(m))
        assert rc == 0
        mass = dict(sumU=m[0], sumPhiPrev=m[1], Vs=m[2], Mprime=m[3], umax=m[4], nonfinite=m[5])
        return L[:nd], mass


def raymarch(p: dict, phi: np.ndarray, dirs) -> np.ndarray:
    cp = make_params(p)
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    dirs = np.ascontiguousarray(dirs, dtype=np.float64)
    L = np.zeros(dirs.shape[0])
    lib().orc_raymarch(ctypes.byref(cp), _dp(phi), dirs.shape[0], _dp(dirs), _dp(L))
    return L
