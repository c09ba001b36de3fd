"""Helpers shared by the GPU parity tests: run the HIP path and the oracle on the same seeded
inputs and compare traces, counters and positions."""
import numpy as np

KEY = ("kind", "system", "sweep", "level", "cell", "trial", "retry")

# Mixed precision against the FP64 oracle. Decisions must be identical (a decision within the FP32
# error bound is re-evaluated in FP64). The reported dU of a test that was not re-evaluated is the
# FP32 sum: its terms come from FP32 tile offsets (absolute error ~eps times the tile half-width,
# so a WCA term near contact is off by up to ~1e-3). Positions carry the FP32 displacements: per
# accepted move about eps (He/lambda) A of error, summed over the moves of one sweep.
MIXED_DU_TOL = dict(dU_rtol=1e-3, dU_atol=1e-3, dU_atol_member=2e-3)
MIXED_POS_RTOL = 1e-6


def tolerances(precision):
    """(trace tolerance kwargs, position rtol) of a parity comparison at this precision."""
    if precision == "mixed":
        return MIXED_DU_TOL, MIXED_POS_RTOL
    return {}, 1e-10


def build_pair(cfg, trace=1_000_000, precision="fp64", **over):
    from oracle import oracle as O
    from paper_1611_09160_amd import wmc

    params = dict(cfg["params"], precision=precision, **over)
    kw = {}
    if "sys_box_L" in cfg:
        kw = dict(sys_box_L=cfg["sys_box_L"], sys_lambda_max=cfg["sys_lambda_max"])
    g = wmc.WMC(params, cfg["sys_offset"], cfg["chain_offset"], cfg["pos"], trace_capacity=trace, **kw)
    o = O.Oracle(params, cfg["sys_offset"], cfg["chain_offset"], cfg["pos"], trace_capacity=trace, **kw)
    return g, o


def sort_trace(t):
    order = np.lexsort(tuple(t[k] for k in reversed(KEY)))
    return t[order]


def compare_traces(tg, to, dU_rtol=1e-9, dU_atol=1e-8, dU_atol_member=0.0):
    """Same records (keys, n, anchors, decisions); energies within tolerance. Returns stats.

    The energy tolerance of a test is dU_atol + dU_rtol |dU| + dU_atol_member n (n = beads
    moved): FP32 energy terms round each bond and pair term of every moved bead separately."""
    tg, to = sort_trace(tg), sort_trace(to)
    assert len(tg) == len(to), (len(tg), len(to))
    for k in KEY + ("n", "extra"):
        bad = np.nonzero(tg[k] != to[k])[0]
        assert len(bad) == 0, (k, bad[:5], tg[bad[:5]], to[bad[:5]])
    moves = to["kind"] != 1
    d = np.abs(tg["dU"][moves] - to["dU"][moves])
    fin = np.isfinite(to["dU"][moves])
    assert np.all(np.isfinite(tg["dU"][moves]) == fin)
    tol = dU_atol + dU_rtol * np.abs(to["dU"][moves]) + dU_atol_member * to["n"][moves]
    if not np.all(d[fin] <= tol[fin]):
        i = np.nonzero(moves)[0][np.nonzero(fin)[0][np.argmax(d[fin] - tol[fin])]]
        raise AssertionError(f"dU differs by {abs(tg['dU'][i] - to['dU'][i]):.3e} (tolerance "
                             f"{dU_atol + dU_rtol * abs(to['dU'][i]) + dU_atol_member * to['n'][i]:.3e}) "
                             f"at record {to[i]} (GPU dU {tg['dU'][i]!r})")
    thr = np.abs(tg["thr"][moves] - to["thr"][moves])
    assert np.all(thr <= 1e-12 * (1 + np.abs(to["thr"][moves])))
    acc_bad = np.nonzero(tg["accepted"] != to["accepted"])[0]
    assert len(acc_bad) == 0, (acc_bad[:5], tg[acc_bad[:5]], to[acc_bad[:5]])
    return dict(records=len(to), moves=int(moves.sum()), max_dU_diff=float(d.max()) if len(d) else 0.0)


def compare_positions(pg, po, rtol=1e-10):
    scale = 1.0 + np.abs(po)
    err = np.abs(pg - po) / scale
    assert err.max() <= rtol, (err.max(), np.unravel_index(np.argmax(err), err.shape))
    return float(err.max())


def compare_counters(og, oo):
    for k in ("trials", "hits", "attempts", "accepts", "caps", "redraws", "bead_updates"):
        np.testing.assert_array_equal(og[k], oo[k], err_msg=k)
    for k in ("pw_chains", "pw_attempts", "pw_accepts", "pw_k0", "pw_caps", "pw_bead_updates", "violations",
              "accepted_total", "accepted_bead_updates"):
        assert og[k] == oo[k], (k, og[k], oo[k])
    for k in ("pw_shell_attempts", "pw_shell_accepts"):
        np.testing.assert_array_equal(og[k], oo[k], err_msg=k)
    assert og["overflows"] == 0
    assert og.get("wait_timeouts", 0) == 0
