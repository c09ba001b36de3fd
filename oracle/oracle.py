"""ctypes binding of the FP64 CPU oracle (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py``
may import this module. The HIP product path never does.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle_wmc.so")
SOURCES = ["wo_tables.c", "wo_sweep.c"]

BOND = {"none": 0, "fene": 1, "harmonic": 2}
MAX_LEVELS = 16
K_SHELLS = 16
ACCEPT = {"metropolis": 0, "glauber": 1}
WAVELET_MAP = {"linear": 0, "rotation": 1}
CENTRING = {"anchor": 0, "uniform": 1}


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (contraction off so the schedule arithmetic is IEEE-plain)."""
    stale = not os.path.exists(LIB_PATH) or any(
        os.path.getmtime(os.path.join(HERE, f)) > os.path.getmtime(LIB_PATH) for f in SOURCES + ["wmc_oracle.h", "wo_internal.h"])
    if force or stale:
        cmd = ["gcc", "-O3", "-std=gnu11", "-ffp-contract=off", "-fPIC", "-shared", "-o", LIB_PATH]
        cmd += [os.path.join(HERE, s) for s in SOURCES] + ["-lm"]
        subprocess.run(cmd, check=True)
    return LIB_PATH


class Params(C.Structure):
    _fields_ = [
        ("periodic", C.c_int32), ("plane_waves", C.c_int32), ("wavelets", C.c_int32), ("pad0", C.c_int32),
        ("box_L", C.c_double), ("lambda_min", C.c_double), ("lambda_max", C.c_double),
        ("band_ratio", C.c_double), ("A0", C.c_double), ("kT", C.c_double),
        ("bond_type", C.c_int32), ("wca", C.c_int32),
        ("k_bond", C.c_double), ("R0", C.c_double), ("sigma", C.c_double), ("eps", C.c_double),
        ("r_int_harmonic", C.c_double),
        ("n_layers", C.c_int32), ("retry_cap", C.c_int32),
        ("seed", C.c_uint64),
        ("accept_rule", C.c_int32), ("wavelet_map", C.c_int32), ("centring", C.c_int32), ("pad1", C.c_int32),
    ]


class Obs(C.Structure):
    _fields_ = [("sweeps", C.c_int64)] + [
        (name, C.c_int64 * MAX_LEVELS)
        for name in ("trials", "hits", "attempts", "accepts", "caps", "redraws", "bead_updates")
    ] + [(name, C.c_int64) for name in (
        "pw_chains", "pw_attempts", "pw_accepts", "pw_k0", "pw_caps", "pw_bead_updates",
        "violations", "accepted_total", "accepted_bead_updates")] + [
        ("pw_shell_attempts", C.c_int64 * K_SHELLS), ("pw_shell_accepts", C.c_int64 * K_SHELLS)]


class TraceRec(C.Structure):
    _fields_ = [(n, C.c_int32) for n in (
        "kind", "system", "sweep", "level", "cell", "trial", "retry", "n", "accepted", "extra")
    ] + [("dU", C.c_double), ("thr", C.c_double)]


class LevelInfo(C.Structure):
    _fields_ = [("lo", C.c_double), ("hi", C.c_double), ("p", C.c_double), ("T", C.c_double),
                ("h", C.c_double), ("ncell", C.c_int32), ("pad", C.c_int32), ("r_int", C.c_double)]


class SystemInfo(C.Structure):
    _fields_ = [(n, C.c_double) for n in (
        "P_F", "R", "N_k", "P_cube", "W_cube", "W_cont", "W_corner", "P_k0", "dt")
    ] + [("n_levels", C.c_int32), ("n_modes", C.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, dp = C.c_void_p, C.c_int32, C.c_int64, C.POINTER(C.c_double)
        L.wo_init.argtypes = [C.POINTER(vp), C.POINTER(Params), i32, C.POINTER(C.c_int64), dp, dp,
                              i64, C.POINTER(C.c_int64), dp, i64]
        L.wo_init.restype = C.c_int
        L.wo_sweep.argtypes = [vp, i64]
        L.wo_positions.argtypes = [vp, dp]
        L.wo_set_positions.argtypes = [vp, dp]
        L.wo_set_sweep.argtypes = [vp, i64]
        L.wo_observables.argtypes = [vp, C.POINTER(Obs)]
        L.wo_system_tau.argtypes = [vp, dp]
        L.wo_chain_rg2.argtypes = [vp, dp]
        L.wo_chain_com.argtypes = [vp, dp]
        L.wo_inf_table.argtypes = [vp, i32, dp, i32]
        L.wo_inf_k_of_v.argtypes = [vp, i32, C.c_double]
        L.wo_inf_k_of_v.restype = C.c_double
        L.wo_G.argtypes = [C.c_double]
        L.wo_G.restype = C.c_double
        L.wo_trace.argtypes = [vp, C.POINTER(TraceRec), i64]
        L.wo_trace.restype = i64
        L.wo_get_level_info.argtypes = [vp, i32, C.POINTER(LevelInfo), i32]
        L.wo_get_system_info.argtypes = [vp, i32, C.POINTER(SystemInfo)]
        L.wo_cell_ids.argtypes = [vp, i32, i64, i32, C.POINTER(C.c_int32)]
        L.wo_cube_weights.argtypes = [vp, i32, dp]
        L.wo_shell_table.argtypes = [vp, i32, dp, i32]
        L.wo_last_error.argtypes = [vp]
        L.wo_last_error.restype = C.c_char_p
        L.wo_free.argtypes = [vp]
        L.wo_philox4x32_10.argtypes = [C.POINTER(C.c_uint32)] * 3
        for name in ("wo_inv_cbrt", "wo_phit", "wo_I", "wo_J6"):
            getattr(L, name).argtypes = [C.c_double]
            getattr(L, name).restype = C.c_double
        L.wo_M.argtypes = [C.c_int]
        L.wo_M.restype = C.c_double
        L.wo_wavelet.argtypes = [dp, dp, dp]
        L.wo_u_fene.argtypes = [C.c_double] * 3
        L.wo_u_fene.restype = C.c_double
        L.wo_u_wca.argtypes = [C.c_double] * 3
        L.wo_u_wca.restype = C.c_double
        L.wo_stream_doubles.argtypes = [C.c_uint64, i32, i64, i32, i64, i64, i32, i32, i32, dp, dp]
        L.wo_draw_lambda.argtypes = [C.c_double] * 3
        L.wo_draw_lambda.restype = C.c_double
        _lib = L
    return _lib


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def make_params(d: dict) -> Params:
    p = Params()
    p.periodic = int(d.get("periodic", 1))
    p.plane_waves = int(d.get("plane_waves", 1))
    p.wavelets = int(d.get("wavelets", 1))
    p.box_L = float(d.get("box_L", 0.0))
    p.lambda_min = float(d["lambda_min"])
    p.lambda_max = float(d["lambda_max"])
    p.band_ratio = float(d.get("band_ratio", 2.0))
    p.A0 = float(d.get("A0", 0.5))
    p.kT = float(d.get("kT", 1.0))
    bt = d.get("bond_type", "fene")
    p.bond_type = BOND[bt] if isinstance(bt, str) else int(bt)
    p.wca = int(d.get("wca", 1))
    p.k_bond = float(d.get("k_bond", 30.0))
    p.R0 = float(d.get("R0", 1.5))
    p.sigma = float(d.get("sigma", 1.0))
    p.eps = float(d.get("eps", 1.0))
    p.r_int_harmonic = float(d.get("r_int_harmonic", 0.0))
    p.n_layers = int(d.get("n_layers", 15))
    p.retry_cap = int(d.get("retry_cap", 64))
    p.seed = int(d.get("seed", 1))
    p.accept_rule = ACCEPT[d.get("accept", "metropolis")]
    p.wavelet_map = WAVELET_MAP[d.get("wavelet_map", "linear")]
    p.centring = CENTRING[d.get("centring", "anchor")]
    return p


class Oracle:
    """One oracle context: n systems, chains, FP64 positions [N, 3]."""

    def __init__(self, params: dict, sys_bead_offset, chain_offset, pos, sys_box_L=None,
                 sys_lambda_max=None, trace_capacity: int = 0):
        L = lib()
        self.params = dict(params)
        self.sys_off = np.ascontiguousarray(sys_bead_offset, dtype=np.int64)
        self.chain_off = np.ascontiguousarray(chain_offset, dtype=np.int64)
        pos = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1, 3)
        self.N = pos.shape[0]
        self.n_systems = len(self.sys_off) - 1
        self.n_chains = len(self.chain_off) - 1
        self._p = make_params(params)
        bl = None if sys_box_L is None else np.ascontiguousarray(sys_box_L, dtype=np.float64)
        lm = None if sys_lambda_max is None else np.ascontiguousarray(sys_lambda_max, dtype=np.float64)
        self._keep = (bl, lm)
        h = C.c_void_p()
        rc = L.wo_init(C.byref(h), C.byref(self._p), self.n_systems,
                       self.sys_off.ctypes.data_as(C.POINTER(C.c_int64)),
                       _dptr(bl) if bl is not None else None, _dptr(lm) if lm is not None else None,
                       self.n_chains, self.chain_off.ctypes.data_as(C.POINTER(C.c_int64)),
                       _dptr(pos), int(trace_capacity))
        self._h = h
        if rc != 0:
            msg = L.wo_last_error(h).decode()
            L.wo_free(h)
            self._h = None
            raise RuntimeError(f"oracle init failed ({rc}): {msg}")

    def __del__(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            _lib.wo_free(self._h)
            self._h = None

    def sweep(self, n: int = 1):
        lib().wo_sweep(self._h, int(n))

    def positions(self) -> np.ndarray:
        out = np.empty((self.N, 3), dtype=np.float64)
        lib().wo_positions(self._h, _dptr(out))
        return out

    def set_positions(self, pos):
        pos = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1, 3)
        lib().wo_set_positions(self._h, _dptr(pos))

    def set_sweep(self, s: int):
        lib().wo_set_sweep(self._h, int(s))

    def observables(self) -> dict:
        o = Obs()
        lib().wo_observables(self._h, C.byref(o))
        d = {"sweeps": o.sweeps}
        for name in ("trials", "hits", "attempts", "accepts", "caps", "redraws", "bead_updates"):
            d[name] = np.array(getattr(o, name)[:], dtype=np.int64)
        for name in ("pw_chains", "pw_attempts", "pw_accepts", "pw_k0", "pw_caps", "pw_bead_updates",
                     "violations", "accepted_total", "accepted_bead_updates"):
            d[name] = getattr(o, name)
        for name in ("pw_shell_attempts", "pw_shell_accepts"):
            d[name] = np.array(getattr(o, name)[:], dtype=np.int64)
        return d

    def tau(self) -> np.ndarray:
        out = np.empty(self.n_systems, dtype=np.float64)
        lib().wo_system_tau(self._h, _dptr(out))
        return out

    def chain_rg2(self) -> np.ndarray:
        out = np.empty(self.n_chains, dtype=np.float64)
        lib().wo_chain_rg2(self._h, _dptr(out))
        return out

    def chain_com(self) -> np.ndarray:
        out = np.empty((self.n_chains, 3), dtype=np.float64)
        lib().wo_chain_com(self._h, _dptr(out))
        return out

    def inf_table(self, system: int = 0) -> np.ndarray:
        out = np.empty(8193, dtype=np.float64)
        n = lib().wo_inf_table(self._h, system, _dptr(out), 8193)
        if n < 0:
            raise RuntimeError("no infinite-system plane-wave table")
        return out[:n].copy()

    def inf_x_of_v(self, v: float, system: int = 0) -> float:
        return lib().wo_inf_k_of_v(self._h, system, float(v))

    def trace(self, max_records: int = 1 << 22) -> np.ndarray:
        buf = (TraceRec * max_records)()
        n = lib().wo_trace(self._h, buf, max_records)
        arr = np.ctypeslib.as_array(buf)[:n].copy()
        return arr

    def level_info(self, system: int = 0) -> list:
        buf = (LevelInfo * MAX_LEVELS)()
        n = lib().wo_get_level_info(self._h, system, buf, MAX_LEVELS)
        return [{f: getattr(buf[i], f) for f, _ in LevelInfo._fields_ if f != "pad"} for i in range(n)]

    def system_info(self, system: int = 0) -> dict:
        s = SystemInfo()
        lib().wo_get_system_info(self._h, system, C.byref(s))
        return {f: getattr(s, f) for f, _ in SystemInfo._fields_}

    def cell_ids(self, system: int, sweep: int, level: int) -> np.ndarray:
        n = int(self.sys_off[system + 1] - self.sys_off[system])
        out = np.empty(n, dtype=np.int32)
        lib().wo_cell_ids(self._h, system, int(sweep), level, out.ctypes.data_as(C.POINTER(C.c_int32)))
        return out

    def cube_weights(self, system: int = 0) -> np.ndarray:
        nl = self._p.n_layers
        out = np.empty((2 * nl + 1) ** 3, dtype=np.float64)
        rc = lib().wo_cube_weights(self._h, system, _dptr(out))
        if rc < 0:
            raise RuntimeError("no plane-wave tables")
        return out

    def shell_table(self, system: int = 0) -> np.ndarray:
        out = np.empty(8193, dtype=np.float64)
        n = lib().wo_shell_table(self._h, system, _dptr(out), 8193)
        if n < 0:
            raise RuntimeError("no plane-wave tables")
        return out[:n].copy()


# --- building blocks for the pins -----------------------------------------------------

def philox(ctr, key):
    c = (C.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (C.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (C.c_uint32 * 4)()
    lib().wo_philox4x32_10(c, k, o)
    return [int(v) for v in o]


def inv_cbrt(x: float) -> float:
    return lib().wo_inv_cbrt(float(x))


def phit(q: float) -> float:
    return lib().wo_phit(float(q))


def I(x: float) -> float:
    return lib().wo_I(float(x))


def J6(x: float) -> float:
    return lib().wo_J6(float(x))


def moment(m: int) -> float:
    return lib().wo_M(int(m))


def wavelet(x, p) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float64)
    p = np.ascontiguousarray(p, dtype=np.float64)
    out = np.empty(3)
    lib().wo_wavelet(_dptr(x), _dptr(p), _dptr(out))
    return out


def u_fene(r2, k, R0):
    return lib().wo_u_fene(float(r2), float(k), float(R0))


def u_wca(r2, sigma, eps):
    return lib().wo_u_wca(float(r2), float(sigma), float(eps))


def stream_doubles(seed, system, sweep, tag, cell, t, r, j, n):
    co = np.empty(n)
    oc = np.empty(n)
    lib().wo_stream_doubles(int(seed), system, sweep, tag, cell, t, r, j, n, _dptr(co), _dptr(oc))
    return co, oc


def G(x: float) -> float:
    return lib().wo_G(float(x))


def draw_lambda(u, lo, hi):
    return lib().wo_draw_lambda(float(u), float(lo), float(hi))
