"""Python binding of libwmc (include/wmc.h): argument marshalling only.

Every step of the sweep runs in the HIP kernels of libwmc.so; torch supplies the device
arena (one uint8 tensor) and the stream. Importing this module on a machine without the
built library raises immediately: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libwmc.so")

MAX_LEVELS = 16
K_SHELLS = 16
BOND = {"none": 0, "fene": 1, "harmonic": 2}
PRECISION = {"fp64": 0, "mixed": 1}
ACCEPT = {"metropolis": 0, "glauber": 1}
WAVELET_MAP = {"linear": 0, "rotation": 1}
CENTRING = {"anchor": 0, "uniform": 1}
# return codes of include/wmc.h
ECAPACITY, ESCHEDULE = -5, -6


class Params(C.Structure):
    _fields_ = [
        ("periodic", C.c_int32), ("plane_waves", C.c_int32), ("wavelets", C.c_int32), ("precision", C.c_int32),
        ("box_L", C.c_double), ("lambda_min", C.c_double), ("lambda_max", C.c_double),
        ("band_ratio", C.c_double), ("A0", C.c_double), ("kT", C.c_double),
        ("bond_type", C.c_int32), ("wca", C.c_int32),
        ("k_bond", C.c_double), ("R0", C.c_double), ("sigma", C.c_double), ("eps", C.c_double),
        ("r_int_harmonic", C.c_double),
        ("n_layers", C.c_int32), ("retry_cap", C.c_int32),
        ("seed", C.c_uint64),
        ("accept_rule", C.c_int32), ("wavelet_map", C.c_int32), ("centring", C.c_int32), ("mixed_verify", C.c_int32),
    ]


class Obs(C.Structure):
    _fields_ = [("sweeps", C.c_int64)] + [
        (name, C.c_int64 * MAX_LEVELS)
        for name in ("trials", "hits", "attempts", "accepts", "caps", "redraws", "bead_updates")
    ] + [(name, C.c_int64) for name in (
        "pw_chains", "pw_attempts", "pw_accepts", "pw_k0", "pw_caps", "pw_bead_updates",
        "violations", "accepted_total", "rechecks", "overflows", "grid_rebuilds", "wait_timeouts",
        "fallback_cells", "accepted_bead_updates")] + [
        ("pw_shell_attempts", C.c_int64 * K_SHELLS), ("pw_shell_accepts", C.c_int64 * K_SHELLS),
        ("member_rechecks", C.c_int64), ("margin_checks", C.c_int64), ("margin_fails", C.c_int64),
        ("margin_max_ratio", C.c_double)]


class TraceRec(C.Structure):
    _fields_ = [(n, C.c_int32) for n in (
        "kind", "system", "sweep", "level", "cell", "trial", "retry", "n", "accepted", "extra")
    ] + [("dU", C.c_double), ("thr", C.c_double)]


_lib = None


def lib():
    """Load libwmc.so; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1611_09160_amd/build.py")
        # torch's bundled HIP runtime must be the one loaded into the process: loading the
        # library first would bind it (and torch) to the system runtime under the same soname.
        import torch  # noqa: F401

        L = C.CDLL(LIB_PATH)
        vp, i32, i64, dp, lp = C.c_void_p, C.c_int32, C.c_int64, C.POINTER(C.c_double), C.POINTER(C.c_int64)
        L.wmc_arena_bytes.argtypes = [C.POINTER(Params), i32, lp, dp, dp, i64, lp, i64, C.POINTER(C.c_size_t)]
        L.wmc_init.argtypes = [C.POINTER(vp), C.POINTER(Params), i32, lp, dp, dp, i64, lp, dp, i64, vp, C.c_size_t, vp]
        L.wmc_init_static.argtypes = [C.POINTER(vp), C.POINTER(Params), i32, lp, dp, dp, i64, lp, dp, i64, vp]
        L.wmc_launch_plan.argtypes = [C.POINTER(Params), i32, lp, dp, dp, i64, lp, dp, i32, i32, i32, i32, C.c_char_p,
                                      C.c_size_t]
        L.wmc_sweep.argtypes = [vp, i64, vp]
        L.wmc_positions.argtypes = [vp, dp, i32, vp]
        L.wmc_set_state.argtypes = [vp, dp, i64, vp]
        L.wmc_observables.argtypes = [vp, C.POINTER(Obs)]
        L.wmc_system_tau.argtypes = [vp, dp]
        L.wmc_chain_rg2.argtypes = [vp, dp]
        L.wmc_chain_com.argtypes = [vp, dp]
        L.wmc_chain_msd.argtypes = [vp, dp]
        L.wmc_trace.argtypes = [vp, C.POINTER(TraceRec), i64, lp]
        L.wmc_system_info.argtypes = [vp, i32, dp, C.POINTER(C.c_int32), dp]
        L.wmc_cell_ids.argtypes = [vp, i32, i64, i32, C.POINTER(C.c_int32)]
        L.wmc_philox.argtypes = [C.POINTER(C.c_uint32), C.POINTER(C.c_uint32), i64, C.POINTER(C.c_uint32), vp,
                                 C.c_size_t, vp]
        L.wmc_set_timing.argtypes = [vp, i32]
        L.wmc_kernel_times.argtypes = [vp, dp, lp]
        L.wmc_tune.argtypes = [vp, i32, C.c_char_p, C.c_size_t]
        L.wmc_set_tuning.argtypes = [vp, C.c_char_p]
        L.wmc_get_tuning.argtypes = [vp, C.c_char_p, C.c_size_t]
        L.wmc_last_error.argtypes = [vp]
        L.wmc_last_error.restype = C.c_char_p
        L.wmc_free.argtypes = [vp]
        for f in ("wmc_arena_bytes", "wmc_launch_plan", "wmc_init", "wmc_init_static", "wmc_sweep", "wmc_positions", "wmc_set_state", "wmc_observables",
                  "wmc_system_tau", "wmc_chain_rg2", "wmc_chain_com", "wmc_chain_msd", "wmc_trace", "wmc_system_info", "wmc_cell_ids", "wmc_philox",
                  "wmc_set_timing", "wmc_kernel_times", "wmc_tune", "wmc_set_tuning", "wmc_get_tuning"):
            getattr(L, f).restype = C.c_int
        _lib = L
    return _lib


def make_params(d: dict) -> Params:
    p = Params()
    p.periodic = int(d.get("periodic", 1))
    p.plane_waves = int(d.get("plane_waves", 1))
    p.wavelets = int(d.get("wavelets", 1))
    prec = d.get("precision", "fp64")
    p.precision = PRECISION[prec] if isinstance(prec, str) else int(prec)
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
    p.mixed_verify = int(d.get("mixed_verify", 0))
    return p


def _dp(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_double))


def _lp(a):
    return a.ctypes.data_as(C.POINTER(C.c_int64))


def _stream(stream):
    import torch

    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


class WMC:
    """A set of systems advanced by libwmc on the current GPU."""

    def __init__(self, params: dict, sys_bead_offset, chain_offset, pos, sys_box_L=None, sys_lambda_max=None,
                 trace_capacity: int = 0, stream=None, device="cuda", static_arena: bool = False):
        """static_arena: place the context in the library-held device arena (wmc_init_static)
        instead of a torch tensor; nothing is allocated on the device then."""
        import torch

        L = lib()
        self.params = dict(params)
        self._p = make_params(params)
        self.sys_off = np.ascontiguousarray(sys_bead_offset, dtype=np.int64)
        self.chain_off = np.ascontiguousarray(chain_offset, dtype=np.int64)
        pos = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1, 3)
        self.N = pos.shape[0]
        self.n_systems = len(self.sys_off) - 1
        self.n_chains = len(self.chain_off) - 1
        self.sys_box_L = None if sys_box_L is None else np.ascontiguousarray(sys_box_L, dtype=np.float64)
        self.sys_lambda_max = None if sys_lambda_max is None else np.ascontiguousarray(sys_lambda_max, dtype=np.float64)
        if static_arena:
            self.arena = None
            h = C.c_void_p()
            rc = L.wmc_init_static(C.byref(h), C.byref(self._p), self.n_systems, _lp(self.sys_off),
                                   _dp(self.sys_box_L), _dp(self.sys_lambda_max), self.n_chains, _lp(self.chain_off),
                                   _dp(pos), int(trace_capacity), _stream(stream))
            self._h = h
            if rc != 0:
                msg = L.wmc_last_error(h).decode()
                L.wmc_free(h)
                self._h = None
                raise RuntimeError(f"wmc_init_static failed ({rc}): {msg}")
            return
        nbytes = C.c_size_t()
        rc = L.wmc_arena_bytes(C.byref(self._p), self.n_systems, _lp(self.sys_off), _dp(self.sys_box_L),
                               _dp(self.sys_lambda_max), self.n_chains, _lp(self.chain_off), int(trace_capacity),
                               C.byref(nbytes))
        if rc != 0:
            raise ValueError(f"wmc_arena_bytes failed ({rc}): invalid parameters")
        self.arena = torch.empty(int(nbytes.value) + 256, dtype=torch.uint8, device=device)
        h = C.c_void_p()
        rc = L.wmc_init(C.byref(h), C.byref(self._p), self.n_systems, _lp(self.sys_off), _dp(self.sys_box_L),
                        _dp(self.sys_lambda_max), self.n_chains, _lp(self.chain_off), _dp(pos), int(trace_capacity),
                        C.c_void_p(self.arena.data_ptr()), int(self.arena.numel()), _stream(stream))
        self._h = h
        if rc != 0:
            msg = L.wmc_last_error(h).decode()
            L.wmc_free(h)
            self._h = None
            raise RuntimeError(f"wmc_init failed ({rc}): {msg}")

    def _check(self, rc, what):
        if rc != 0:
            raise RuntimeError(f"{what} failed ({rc}): {lib().wmc_last_error(self._h).decode()}")

    def close(self):
        if getattr(self, "_h", None) is not None:
            lib().wmc_free(self._h)
            self._h = None

    def __del__(self):
        # at interpreter shutdown the HIP runtime may already be gone: leave the context to the
        # process exit instead of calling into it (close() contexts explicitly before exiting)
        if sys.is_finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    def sweep(self, n: int = 1, stream=None):
        self._check(lib().wmc_sweep(self._h, int(n), _stream(stream)), "wmc_sweep")

    def positions(self) -> np.ndarray:
        out = np.empty((self.N, 3), dtype=np.float64)
        self._check(lib().wmc_positions(self._h, _dp(out), 0, _stream(None)), "wmc_positions")
        return out

    def positions_into(self, tensor, stream=None):
        """Copy positions into a CUDA float64 tensor of shape [N, 3] (asynchronous)."""
        self._check(lib().wmc_positions(self._h, C.cast(C.c_void_p(tensor.data_ptr()), C.POINTER(C.c_double)), 1,
                                        _stream(stream)), "wmc_positions")

    def set_state(self, pos, sweep: int):
        pos = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1, 3)
        self._check(lib().wmc_set_state(self._h, _dp(pos), int(sweep), _stream(None)), "wmc_set_state")

    def observables(self, check: bool = True) -> dict:
        """Counters; with check=False an overflow or wait time-out is reported in the counters
        (overflows, wait_timeouts) instead of raising."""
        o = Obs()
        rc = lib().wmc_observables(self._h, C.byref(o))
        if check or rc not in (ECAPACITY, ESCHEDULE):
            self._check(rc, "wmc_observables")
        d = {"sweeps": o.sweeps}
        for name in ("trials", "hits", "attempts", "accepts", "caps", "redraws", "bead_updates"):
            d[name] = np.array(getattr(o, name)[:], dtype=np.int64)
        for name in ("pw_chains", "pw_attempts", "pw_accepts", "pw_k0", "pw_caps", "pw_bead_updates", "violations",
                     "accepted_total", "rechecks", "overflows", "grid_rebuilds", "wait_timeouts", "fallback_cells",
                     "accepted_bead_updates", "member_rechecks", "margin_checks", "margin_fails",
                     "margin_max_ratio"):
            d[name] = getattr(o, name)
        for name in ("pw_shell_attempts", "pw_shell_accepts"):
            d[name] = np.array(getattr(o, name)[:], dtype=np.int64)
        return d

    def tau(self) -> np.ndarray:
        out = np.empty(self.n_systems)
        self._check(lib().wmc_system_tau(self._h, _dp(out)), "wmc_system_tau")
        return out

    def chain_rg2(self) -> np.ndarray:
        out = np.empty(self.n_chains)
        self._check(lib().wmc_chain_rg2(self._h, _dp(out)), "wmc_chain_rg2")
        return out

    def chain_com(self) -> np.ndarray:
        out = np.empty((self.n_chains, 3))
        self._check(lib().wmc_chain_com(self._h, _dp(out)), "wmc_chain_com")
        return out

    def chain_msd(self) -> np.ndarray:
        out = np.empty(self.n_chains)
        self._check(lib().wmc_chain_msd(self._h, _dp(out)), "wmc_chain_msd")
        return out

    def trace(self, max_records: int = 1 << 22) -> np.ndarray:
        buf = (TraceRec * max_records)()
        n = C.c_int64()
        self._check(lib().wmc_trace(self._h, buf, max_records, C.byref(n)), "wmc_trace")
        return np.ctypeslib.as_array(buf)[: n.value].copy()

    def system_info(self, system: int = 0) -> dict:
        lv = np.zeros(6 * MAX_LEVELS)
        pw = np.zeros(6)
        n = C.c_int32()
        self._check(lib().wmc_system_info(self._h, system, _dp(lv), C.byref(n), _dp(pw)), "wmc_system_info")
        levels = [dict(zip(("lo", "hi", "p", "T", "h", "ncell"), lv[6 * i: 6 * i + 6])) for i in range(n.value)]
        return {"levels": levels, **dict(zip(("P_F", "R", "N_k", "P_cube", "P_k0", "dt"), pw))}

    def set_timing(self, enable: bool = True):
        self._check(lib().wmc_set_timing(self._h, int(enable)), "wmc_set_timing")

    def kernel_times(self) -> dict:
        """Per kernel class: summed milliseconds and launch count since timing was switched on."""
        ms = np.zeros(18)
        n = np.zeros(18, dtype=np.int64)
        self._check(lib().wmc_kernel_times(self._h, _dp(ms), _lp(n)), "wmc_kernel_times")
        names = ["grid"] + [f"level{l}" for l in range(MAX_LEVELS)] + ["plane_waves"]
        return {names[i]: (float(ms[i]), int(n[i])) for i in range(18) if n[i] > 0}

    def tune(self, trial_sweeps: int = 3) -> dict:
        """Time each launch choice per level from the current state, keep the fastest, restore the
        state (wmc_tune); returns the chosen settings with their times."""
        import json

        buf = C.create_string_buffer(1 << 16)
        self._check(lib().wmc_tune(self._h, int(trial_sweeps), buf, len(buf)), "wmc_tune")
        return json.loads(buf.value.decode())

    def set_tuning(self, settings):
        """Apply launch settings (a dict as tune() returns, or its JSON text)."""
        import json

        text = settings if isinstance(settings, str) else json.dumps(settings)
        self._check(lib().wmc_set_tuning(self._h, text.encode()), "wmc_set_tuning")

    def get_tuning(self) -> dict:
        import json

        buf = C.create_string_buffer(1 << 16)
        self._check(lib().wmc_get_tuning(self._h, buf, len(buf)), "wmc_get_tuning")
        return json.loads(buf.value.decode())

    def cell_ids(self, system: int, sweep: int, level: int) -> np.ndarray:
        n = int(self.sys_off[system + 1] - self.sys_off[system])
        out = np.empty(n, dtype=np.int32)
        self._check(lib().wmc_cell_ids(self._h, system, int(sweep), level, out.ctypes.data_as(C.POINTER(C.c_int32))),
                    "wmc_cell_ids")
        return out


def launch_plan(cfg: dict, cell_blocks: int, pw_blocks: int, cell_launch_max: int, pw_launch_max: int):
    """Host-only check of the launch plan of a workload for given co-residency limits
    (wmc_launch_plan): returns (return code, report)."""
    p = make_params(cfg["params"])
    so = np.ascontiguousarray(cfg["sys_offset"], dtype=np.int64)
    co = np.ascontiguousarray(cfg["chain_offset"], dtype=np.int64)
    pos = np.ascontiguousarray(cfg["pos"], dtype=np.float64).reshape(-1, 3)
    bl = cfg.get("sys_box_L")
    lm = cfg.get("sys_lambda_max")
    bl = None if bl is None else np.ascontiguousarray(bl, dtype=np.float64)
    lm = None if lm is None else np.ascontiguousarray(lm, dtype=np.float64)
    buf = C.create_string_buffer(1024)
    rc = lib().wmc_launch_plan(C.byref(p), len(so) - 1, _lp(so), _dp(bl), _dp(lm), len(co) - 1, _lp(co), _dp(pos),
                               int(cell_blocks), int(pw_blocks), int(cell_launch_max), int(pw_launch_max), buf, 1024)
    return rc, buf.value.decode()


def philox(ctr, key, n: int = 1) -> np.ndarray:
    """Philox4x32-10 evaluated on the GPU for counters ctr, ctr+1, ... (first word incremented)."""
    import torch

    scratch = torch.empty(16 * n, dtype=torch.uint8, device="cuda")
    c = (C.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (C.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    out = np.empty((n, 4), dtype=np.uint32)
    rc = lib().wmc_philox(c, k, n, out.ctypes.data_as(C.POINTER(C.c_uint32)), C.c_void_p(scratch.data_ptr()),
                          scratch.numel(), _stream(None))
    if rc != 0:
        raise RuntimeError(f"wmc_philox failed ({rc})")
    return out
