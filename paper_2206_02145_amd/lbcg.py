"""ctypes binding of liblbcg.so (include/lbcg.h): argument marshalling only.

Every step of the solver runs in the HIP kernels of the library; PyTorch provides the device
workspace and the stream. There is no CPU fallback: without the built library or a HIP device
these functions raise.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbcg.so")

LBCG_OK = 0
STATUS = {0: "OK", -1: "EINVAL", -2: "EUNSTABLE", -3: "ENOMEM", -4: "EDEVICE", -5: "ENONFINITE",
          -6: "ESTATE"}
PRECISION = {"fp64": 0, "fp32": 1, "fp16shift": 2}
FIELD = {"phi": 0, "U": 1, "rho": 2, "ux": 3, "uy": 4, "uz": 5, "phi_prev": 6, "raw_h": 7,
         "raw_g": 8, "raw_f": 9}
DTYPE = {np.float64: 0, np.float32: 1}


class lbcg_params(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("nz", ctypes.c_int32), ("flow", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("xbc", ctypes.c_int32), ("walls", ctypes.c_int32),
        ("W0", ctypes.c_double), ("tau0", ctypes.c_double), ("lambda_", ctypes.c_double),
        ("D", ctypes.c_double), ("eps_aniso", ctypes.c_double), ("nu", ctypes.c_double),
        ("h_drag", ctypes.c_double), ("u_inlet", ctypes.c_double), ("U0", ctypes.c_double),
        ("U_inlet", ctypes.c_double), ("seed_center", ctypes.c_double * 3),
        ("seed_radius", ctypes.c_double), ("grad_eps2", ctypes.c_double),
        ("seed_shape", ctypes.c_int32), ("collision", ctypes.c_int32), ("seed_tilt", ctypes.c_double),
        ("omega_bulk", ctypes.c_double), ("solute_source", ctypes.c_int32),
    ]


class LbcgError(RuntimeError):
    def __init__(self, code: int, where: str, msg: str):
        super().__init__(f"{where}: {STATUS.get(code, code)}: {msg}")
        self.code = code
        self.status = STATUS.get(code, str(code))


_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run `python -c 'import __graft_entry__ as g; g.build()'`")
        L = ctypes.CDLL(LIB_PATH)
        L.lbcg_source_hash.argtypes = []
        L.lbcg_source_hash.restype = ctypes.c_char_p
        from . import build as _build
        built, now = L.lbcg_source_hash().decode(), _build.source_hash()
        if built != now:
            raise RuntimeError(f"{LIB_PATH} was built from other sources (built {built}, sources {now}); "
                               "rebuild it: python -c 'import __graft_entry__ as g; g.build()'")
        vp, i32, i64, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_size_t
        dp = ctypes.POINTER(ctypes.c_double)
        pp = ctypes.POINTER(lbcg_params)
        L.lbcg_workspace_bytes.argtypes = [pp]
        L.lbcg_workspace_bytes.restype = sz
        L.lbcg_create.argtypes = [pp, vp, sz, vp, ctypes.POINTER(vp)]
        L.lbcg_step.argtypes = [vp, i64]
        L.lbcg_step_count.argtypes = [vp]
        L.lbcg_step_count.restype = i64
        L.lbcg_read_field.argtypes = [vp, i32, vp, sz, i32, i32]
        L.lbcg_write_field.argtypes = [vp, i32, vp, sz, i32, i32]
        L.lbcg_measure.argtypes = [vp, i32, dp, dp, dp]
        L.lbcg_measure_noalloc.argtypes = [vp, i32, dp, dp, dp]
        L.lbcg_run.argtypes = [vp, i64, i64, i32, dp, dp, dp]
        L.lbcg_growth_rates.argtypes = [vp, dp, dp, dp]
        L.lbcg_destroy.argtypes = [vp]
        L.lbcg_set_walls.argtypes = [vp, vp, sz, i32]
        L.lbcg_state_bytes.argtypes = [vp]
        L.lbcg_state_bytes.restype = sz
        L.lbcg_state_save.argtypes = [vp, vp, sz, i32]
        L.lbcg_state_load.argtypes = [vp, vp, sz, i32]
        L.lbcg_variant_count.argtypes = [vp]
        L.lbcg_variant_current.argtypes = [vp]
        L.lbcg_variant_name.argtypes = [vp, i32, ctypes.c_char_p, sz]
        L.lbcg_variant_select.argtypes = [vp, i32]
        L.lbcg_variant_time.argtypes = [vp, i32, i32, dp]
        L.lbcg_autotune.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_int), dp]
        L.lbcg_batch_workspace_bytes.argtypes = [i32, pp]
        L.lbcg_batch_workspace_bytes.restype = sz
        L.lbcg_batch_create.argtypes = [i32, pp, vp, sz, vp, ctypes.POINTER(vp)]
        L.lbcg_batch_run.argtypes = [vp, i64, i64, i32, dp, dp, i32]
        L.lbcg_batch_measure.argtypes = [vp, i32, dp, dp]
        L.lbcg_batch_read_field.argtypes = [vp, i32, i32, vp, sz, i32, i32]
        L.lbcg_batch_step_count.argtypes = [vp]
        L.lbcg_batch_step_count.restype = i64
        L.lbcg_batch_destroy.argtypes = [vp]
        L.lbcg_batch_variant_count.argtypes = [vp]
        L.lbcg_batch_variant_current.argtypes = [vp]
        L.lbcg_batch_variant_name.argtypes = [vp, i32, ctypes.c_char_p, sz]
        L.lbcg_batch_variant_select.argtypes = [vp, i32]
        L.lbcg_batch_variant_time.argtypes = [vp, i32, i32, dp]
        L.lbcg_batch_autotune.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_int), dp, dp]
        L.lbcg_tune_cache_clear.argtypes = []
        L.lbcg_mlp_workspace_bytes.argtypes = [i32, ctypes.POINTER(ctypes.c_int), i32]
        L.lbcg_mlp_workspace_bytes.restype = sz
        L.lbcg_mlp_create.argtypes = [i32, ctypes.POINTER(ctypes.c_int), i32, vp, sz, vp, ctypes.POINTER(vp)]
        L.lbcg_mlp_num_params.argtypes = [vp]
        L.lbcg_mlp_num_params.restype = i64
        fp = ctypes.POINTER(ctypes.c_float)
        L.lbcg_mlp_set_params.argtypes = [vp, fp]
        L.lbcg_mlp_get_params.argtypes = [vp, fp]
        L.lbcg_mlp_forward.argtypes = [vp, i32, vp, vp]
        L.lbcg_mlp_grads.argtypes = [vp, i32, vp, vp, vp, i32, fp, fp]
        L.lbcg_mlp_train_step.argtypes = [vp, i32, vp, vp, vp, i32, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                          ctypes.c_float, fp]
        L.lbcg_mlp_destroy.argtypes = [vp]
        L.lbcg_last_error.argtypes = []
        L.lbcg_last_error.restype = ctypes.c_char_p
        for name in ("lbcg_create", "lbcg_step", "lbcg_read_field", "lbcg_write_field",
                     "lbcg_measure", "lbcg_measure_noalloc", "lbcg_growth_rates", "lbcg_destroy", "lbcg_variant_name",
                     "lbcg_variant_select", "lbcg_variant_time", "lbcg_autotune", "lbcg_variant_count",
                     "lbcg_variant_current", "lbcg_batch_create", "lbcg_batch_run", "lbcg_batch_measure",
                     "lbcg_batch_read_field", "lbcg_batch_destroy", "lbcg_mlp_create", "lbcg_mlp_set_params",
                     "lbcg_mlp_get_params", "lbcg_mlp_forward", "lbcg_mlp_grads", "lbcg_mlp_train_step",
                     "lbcg_mlp_destroy", "lbcg_state_save", "lbcg_state_load", "lbcg_set_walls",
                     "lbcg_batch_variant_count", "lbcg_batch_variant_current", "lbcg_batch_variant_name",
                     "lbcg_batch_variant_select", "lbcg_batch_variant_time", "lbcg_batch_autotune",
                     "lbcg_tune_cache_clear"):
            getattr(L, name).restype = i32
        _lib = L
    return _lib


def check(code: int, where: str):
    if code != LBCG_OK:
        raise LbcgError(code, where, lib().lbcg_last_error().decode())


def make_params(p: dict, precision: str = "fp32") -> lbcg_params:
    """lbcg_params from a parameter dict (keys as in paper_2206_02145_amd.workloads)."""
    s = lbcg_params()
    s.dim, s.nx, s.ny, s.nz = int(p["dim"]), int(p["nx"]), int(p["ny"]), int(p["nz"])
    s.flow, s.xbc, s.walls = int(p["flow"]), int(p["xbc"]), int(p.get("walls", 0))
    s.precision = PRECISION[precision]
    s.W0, s.tau0, s.lambda_, s.D = p["W0"], p["tau0"], p["lam"], p["D"]
    s.eps_aniso, s.nu, s.h_drag = p["eps"], p["nu"], p["h_drag"]
    s.u_inlet, s.U0, s.U_inlet = p["u_in"], p["U0"], p["U_in"]
    for d in range(3):
        s.seed_center[d] = float(p["seed_c"][d])
    s.seed_radius, s.grad_eps2 = p["seed_R"], p["grad_eps2"]
    s.seed_shape, s.seed_tilt = int(p.get("seed_shape", 0)), float(p.get("seed_tilt", 0.0))
    s.collision, s.omega_bulk = int(p.get("collision", 0)), float(p.get("omega_bulk", 1.0))
    s.solute_source = int(p.get("solute_source", 0))
    return s


def lbcg_workspace_bytes(params: lbcg_params) -> int:
    return int(lib().lbcg_workspace_bytes(ctypes.byref(params)))


def _dptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class Solver:
    """One grid: owns a torch device workspace and a library handle."""

    def __init__(self, p: dict, precision: str = "fp32", stream=None, ws_fill: int | None = None):
        """ws_fill: if given, the byte every workspace byte holds before lbcg_create (the library
        must not depend on the workspace's prior contents)."""
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("the lbcg solver needs a HIP device")
        self.p = dict(p)
        self.precision = precision
        self.params = make_params(p, precision)
        nbytes = lbcg_workspace_bytes(self.params)
        if nbytes == 0:
            # reproduce the validation error message through lbcg_create
            h = ctypes.c_void_p()
            check(lib().lbcg_create(ctypes.byref(self.params), None, 0, None, ctypes.byref(h)), "lbcg_create")
        if ws_fill is None:
            self.ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        else:
            self.ws = torch.full((nbytes,), int(ws_fill), dtype=torch.uint8, device="cuda")
            torch.cuda.synchronize()
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.handle = ctypes.c_void_p()
        check(lib().lbcg_create(ctypes.byref(self.params), ctypes.c_void_p(self.ws.data_ptr()), nbytes,
                                ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(self.handle)),
              "lbcg_create")
        self.shape = (int(p["nz"]), int(p["ny"]), int(p["nx"]))
        self.qs = 5 if p["dim"] == 2 else 7
        self.qf = 9 if p["dim"] == 2 else 19

    def step(self, n: int = 1):
        check(lib().lbcg_step(self.handle, int(n)), "lbcg_step")

    @property
    def nstep(self) -> int:
        return int(lib().lbcg_step_count(self.handle))

    def _planes(self, field: str) -> int:
        return {"raw_h": self.qs, "raw_g": self.qs, "raw_f": self.qf}.get(field, 1)

    def read(self, field: str, dtype=np.float64) -> np.ndarray:
        """Field as a host numpy array: (nz, ny, nx), or (q, nz, ny, nx) for raw_*."""
        k = self._planes(field)
        shape = ((k,) if k > 1 or field.startswith("raw") else ()) + self.shape
        out = np.empty(shape, dtype=dtype)
        check(lib().lbcg_read_field(self.handle, FIELD[field], out.ctypes.data, out.nbytes, 0,
                                    DTYPE[np.dtype(dtype).type]), "lbcg_read_field")
        return out

    def read_device(self, field: str, dtype=None):
        """Field into a new torch tensor on the device."""
        import torch
        dtype = dtype or torch.float64
        k = self._planes(field)
        shape = ((k,) if field.startswith("raw") else ()) + self.shape
        out = torch.empty(shape, dtype=dtype, device="cuda")
        code = 0 if dtype == torch.float64 else 1
        check(lib().lbcg_read_field(self.handle, FIELD[field], ctypes.c_void_p(out.data_ptr()),
                                    out.numel() * out.element_size(), 1, code), "lbcg_read_field")
        return out

    def write(self, field: str, arr: np.ndarray):
        arr = np.ascontiguousarray(arr)
        if arr.dtype not in (np.float64, np.float32):
            arr = arr.astype(np.float64)
        check(lib().lbcg_write_field(self.handle, FIELD[field], arr.ctypes.data, arr.nbytes, 0,
                                     DTYPE[arr.dtype.type]), "lbcg_write_field")

    def set_walls(self, mask):
        """Solid wall nodes: nonzero entries of a (nz, ny, nx) mask (the solver needs walls=1)."""
        m = np.ascontiguousarray(np.broadcast_to(np.asarray(mask) != 0, self.shape), dtype=np.uint8)
        check(lib().lbcg_set_walls(self.handle, m.ctypes.data, m.nbytes, 0), "lbcg_set_walls")

    # ---- checkpoints ----
    def save_state(self, device: bool = False):
        """The stored state and step count as a uint8 numpy array (host) or torch tensor (device)."""
        n = int(lib().lbcg_state_bytes(self.handle))
        if device:
            import torch
            out = torch.empty(n, dtype=torch.uint8, device="cuda")
            check(lib().lbcg_state_save(self.handle, ctypes.c_void_p(out.data_ptr()), n, 1), "lbcg_state_save")
            return out
        out = np.empty(n, dtype=np.uint8)
        check(lib().lbcg_state_save(self.handle, out.ctypes.data, n, 0), "lbcg_state_save")
        return out

    def load_state(self, blob):
        """Restore a state written by save_state (numpy array or device tensor)."""
        if isinstance(blob, np.ndarray):
            blob = np.ascontiguousarray(blob, dtype=np.uint8)
            check(lib().lbcg_state_load(self.handle, blob.ctypes.data, blob.nbytes, 0), "lbcg_state_load")
        else:
            check(lib().lbcg_state_load(self.handle, ctypes.c_void_p(blob.data_ptr()), blob.numel(), 1),
                  "lbcg_state_load")

    def measure(self, dirs=None, raise_nonfinite: bool = True):
        """(L [ndirs], mass dict) -- see lbcg_measure."""
        dirs = np.zeros((0, 3)) if dirs is None else np.ascontiguousarray(dirs, dtype=np.float64)
        nd = dirs.shape[0]
        L = np.zeros(max(nd, 1))
        m = np.zeros(6)
        code = lib().lbcg_measure(self.handle, nd, _dptr(dirs) if nd else None, _dptr(L), _dptr(m))
        if code != -5 or raise_nonfinite:
            check(code, "lbcg_measure")
        mass = dict(sumU=m[0], sumPhiPrev=m[1], Vs=m[2], Mprime=m[3], umax=m[4], nonfinite=m[5])
        return L[:nd], mass

    def measure_noalloc(self, dirs=None, raise_nonfinite: bool = True):
        """As measure, through lbcg_measure_noalloc (the library's static device scratch)."""
        dirs = np.zeros((0, 3)) if dirs is None else np.ascontiguousarray(dirs, dtype=np.float64)
        nd = dirs.shape[0]
        L = np.zeros(max(nd, 1))
        m = np.zeros(6)
        code = lib().lbcg_measure_noalloc(self.handle, nd, _dptr(dirs) if nd else None, _dptr(L), _dptr(m))
        if code != -5 or raise_nonfinite:
            check(code, "lbcg_measure_noalloc")
        mass = dict(sumU=m[0], sumPhiPrev=m[1], Vs=m[2], Mprime=m[3], umax=m[4], nonfinite=m[5])
        return L[:nd], mass

    def run(self, nsteps: int, measure_every: int, dirs=None, raise_nonfinite: bool = True):
        """nsteps steps with the diagnostics every measure_every steps, kept on the device and copied
        back once (lbcg_run). Returns (L_hist [samples, ndirs], mass_hist [samples] of dicts)."""
        dirs = np.zeros((0, 3)) if dirs is None else np.ascontiguousarray(dirs, dtype=np.float64)
        nd = dirs.shape[0]
        ns = int(nsteps) // int(measure_every) if int(measure_every) > 0 and int(nsteps) > 0 else 0
        L = np.zeros((max(ns, 1), max(nd, 1)))
        M = np.zeros((max(ns, 1), 6))
        code = lib().lbcg_run(self.handle, int(nsteps), int(measure_every), nd, _dptr(dirs) if nd else None,
                              _dptr(L) if nd else None, _dptr(M))
        if code != -5 or raise_nonfinite:
            check(code, "lbcg_run")
        keys = ("sumU", "sumPhiPrev", "Vs", "Mprime", "umax", "nonfinite")
        return L[:ns, :nd], [dict(zip(keys, row)) for row in M[:ns]]

    def growth_rates(self, ndirs: int):
        G = np.zeros(ndirs)
        R2 = np.zeros(ndirs)
        Ga = ctypes.c_double()
        check(lib().lbcg_growth_rates(self.handle, _dptr(G), _dptr(R2), ctypes.byref(Ga)), "lbcg_growth_rates")
        return G, R2, Ga.value

    # ---- kernel variants / autotuning ----
    def variants(self):
        n = lib().lbcg_variant_count(self.handle)
        out = []
        buf = ctypes.create_string_buffer(128)
        for i in range(n):
            check(lib().lbcg_variant_name(self.handle, i, buf, 128), "lbcg_variant_name")
            out.append(buf.value.decode())
        return out

    @property
    def variant(self) -> int:
        return int(lib().lbcg_variant_current(self.handle))

    def select_variant(self, idx: int):
        check(lib().lbcg_variant_select(self.handle, int(idx)), "lbcg_variant_select")

    def time_variant(self, idx: int, launches: int = 20) -> float:
        """Microseconds per step of variant idx over `launches` real steps (the state advances by
        launches + 1 steps)."""
        us = ctypes.c_double()
        check(lib().lbcg_variant_time(self.handle, int(idx), int(launches), ctypes.byref(us)), "lbcg_variant_time")
        return us.value

    def autotune(self, launches: int = 20):
        """Select the fastest variant (two timing rounds); the state advances by 2 (launches + 1)
        steps per variant."""
        best = ctypes.c_int()
        us = ctypes.c_double()
        check(lib().lbcg_autotune(self.handle, int(launches), ctypes.byref(best), ctypes.byref(us)), "lbcg_autotune")
        return best.value, us.value

    def close(self):
        if getattr(self, "handle", None):
            lib().lbcg_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many independent grids of one kind (same dim, flow, precision) stepped together."""

    def __init__(self, plist, precision: str = "fp32", stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("the lbcg solver needs a HIP device")
        self.plist = [dict(p) for p in plist]
        self.n = len(plist)
        arr = (lbcg_params * self.n)(*[make_params(p, precision) for p in plist])
        self._params = arr
        nbytes = int(lib().lbcg_batch_workspace_bytes(self.n, arr))
        if nbytes == 0:
            h = ctypes.c_void_p()
            check(lib().lbcg_batch_create(self.n, arr, None, 0, None, ctypes.byref(h)), "lbcg_batch_create")
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        # a stream of its own (default priority): graph capture needs a non-null stream
        self.stream = stream if stream is not None else torch.cuda.Stream()
        self.handle = ctypes.c_void_p()
        torch.cuda.synchronize()
        check(lib().lbcg_batch_create(self.n, arr, ctypes.c_void_p(self.ws.data_ptr()), nbytes,
                                      ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(self.handle)),
              "lbcg_batch_create")

    def run(self, nsteps: int, measure_every: int = 0, dirs=None, use_graph: bool = True):
        """Returns L_hist [samples, n, ndirs] (None without measurements)."""
        dirs = np.zeros((0, 3)) if dirs is None else np.ascontiguousarray(dirs, dtype=np.float64)
        nd = dirs.shape[0]
        ns = nsteps // measure_every if (measure_every > 0 and nd > 0) else 0
        L = np.zeros((max(ns, 1), self.n, max(nd, 1)))
        check(lib().lbcg_batch_run(self.handle, int(nsteps), int(measure_every), nd, _dptr(dirs) if nd else None,
                                   _dptr(L), 1 if use_graph else 0), "lbcg_batch_run")
        return L[:ns, :, :nd] if ns else None

    def variants(self):
        """Names of the batched step's tilings (index 0 is the default)."""
        out = []
        buf = ctypes.create_string_buffer(128)
        for k in range(lib().lbcg_batch_variant_count(self.handle)):
            check(lib().lbcg_batch_variant_name(self.handle, k, buf, 128), "lbcg_batch_variant_name")
            out.append(buf.value.decode())
        return out

    @property
    def variant(self) -> int:
        return int(lib().lbcg_batch_variant_current(self.handle))

    def select_variant(self, idx: int):
        check(lib().lbcg_batch_variant_select(self.handle, int(idx)), "lbcg_batch_variant_select")

    def time_variant(self, idx: int, launches: int = 20) -> float:
        us = ctypes.c_double()
        check(lib().lbcg_batch_variant_time(self.handle, int(idx), int(launches), ctypes.byref(us)),
              "lbcg_batch_variant_time")
        return us.value

    def autotune(self, launches: int = 20):
        """(best index, its microseconds per step, every tiling's microseconds); the choice is cached."""
        best, us = ctypes.c_int(), ctypes.c_double()
        all_us = np.zeros(max(1, lib().lbcg_batch_variant_count(self.handle)))
        check(lib().lbcg_batch_autotune(self.handle, int(launches), ctypes.byref(best), ctypes.byref(us),
                                        _dptr(all_us)), "lbcg_batch_autotune")
        return best.value, us.value, all_us

    def measure(self, dirs):
        dirs = np.ascontiguousarray(dirs, dtype=np.float64)
        L = np.zeros((self.n, dirs.shape[0]))
        check(lib().lbcg_batch_measure(self.handle, dirs.shape[0], _dptr(dirs), _dptr(L)), "lbcg_batch_measure")
        return L

    def read(self, i: int, field: str, dtype=np.float64) -> np.ndarray:
        p = self.plist[i]
        shape = (int(p["nz"]), int(p["ny"]), int(p["nx"]))
        qs = 5 if p["dim"] == 2 else 7
        qf = 9 if p["dim"] == 2 else 19
        k = {"raw_h": qs, "raw_g": qs, "raw_f": qf}.get(field)
        out = np.empty(((k,) if k else ()) + shape, dtype=dtype)
        check(lib().lbcg_batch_read_field(self.handle, int(i), FIELD[field], out.ctypes.data, out.nbytes, 0,
                                          DTYPE[np.dtype(dtype).type]), "lbcg_batch_read_field")
        return out

    @property
    def nstep(self) -> int:
        return int(lib().lbcg_batch_step_count(self.handle))

    def close(self):
        if getattr(self, "handle", None):
            lib().lbcg_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def tune_cache_clear():
    """Forget the autotuner's cached choices of this process."""
    check(lib().lbcg_tune_cache_clear(), "lbcg_tune_cache_clear")


def _fptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


class MLP:
    """The surrogate network on the GPU (lbcg_mlp_*): bf16 MFMA GEMMs, fp32 master weights, Adam."""

    def __init__(self, widths, max_batch: int, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("the lbcg MLP needs a HIP device")
        self.widths = [int(w) for w in widths]
        self.nl = len(self.widths) - 1
        self._w = (ctypes.c_int * len(self.widths))(*self.widths)
        self.max_batch = int(max_batch)
        nbytes = int(lib().lbcg_mlp_workspace_bytes(self.nl, self._w, self.max_batch))
        if nbytes == 0:
            raise ValueError("invalid MLP shape")
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.handle = ctypes.c_void_p()
        check(lib().lbcg_mlp_create(self.nl, self._w, self.max_batch, ctypes.c_void_p(self.ws.data_ptr()), nbytes,
                                    ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(self.handle)),
              "lbcg_mlp_create")
        self.n_params = int(lib().lbcg_mlp_num_params(self.handle))

    def set_params(self, flat):
        flat = np.ascontiguousarray(flat, dtype=np.float32)
        assert flat.size == self.n_params
        check(lib().lbcg_mlp_set_params(self.handle, _fptr(flat)), "lbcg_mlp_set_params")

    def get_params(self) -> np.ndarray:
        out = np.empty(self.n_params, dtype=np.float32)
        check(lib().lbcg_mlp_get_params(self.handle, _fptr(out)), "lbcg_mlp_get_params")
        return out

    def forward(self, x_dev, y_dev=None):
        """x_dev: torch float32 (B, widths[0]) on the device; returns y (B, widths[-1])."""
        import torch
        B = int(x_dev.shape[0])
        if y_dev is None:
            y_dev = torch.empty((B, self.widths[-1]), dtype=torch.float32, device="cuda")
        check(lib().lbcg_mlp_forward(self.handle, B, ctypes.c_void_p(x_dev.data_ptr()),
                                     ctypes.c_void_p(y_dev.data_ptr())), "lbcg_mlp_forward")
        return y_dev

    def grads(self, X_dev, T_dev, idx_dev):
        g = np.empty(self.n_params, dtype=np.float32)
        loss = ctypes.c_float()
        check(lib().lbcg_mlp_grads(self.handle, int(idx_dev.shape[0]), ctypes.c_void_p(X_dev.data_ptr()),
                                   ctypes.c_void_p(T_dev.data_ptr()), ctypes.c_void_p(idx_dev.data_ptr()),
                                   int(X_dev.shape[0]), _fptr(g), ctypes.byref(loss)), "lbcg_mlp_grads")
        return g, loss.value

    def train_step(self, X_dev, T_dev, idx_dev, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, want_loss=True):
        """One Adam step on the rows idx_dev of (X_dev, T_dev); returns the batch loss, or None
        without synchronising when want_loss is False."""
        loss = ctypes.c_float()
        check(lib().lbcg_mlp_train_step(self.handle, int(idx_dev.shape[0]), ctypes.c_void_p(X_dev.data_ptr()),
                                        ctypes.c_void_p(T_dev.data_ptr()), ctypes.c_void_p(idx_dev.data_ptr()),
                                        int(X_dev.shape[0]), lr, beta1, beta2, eps,
                                        ctypes.byref(loss) if want_loss else None),
              "lbcg_mlp_train_step")
        return loss.value if want_loss else None

    def close(self):
        if getattr(self, "handle", None):
            lib().lbcg_mlp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
