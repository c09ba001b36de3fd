"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the same seeded
inputs. Bar: identical integer schedule (cells, reach-list sizes, trial counts, anchors, member
counts, accept decisions, counters), energies within 1e-9 relative + 1e-8 absolute, positions
within 1e-10 relative per sweep (transcendentals and summation order differ by a few ulp). Mixed
precision: the same integer schedule and decisions, energies and positions within the FP32
bounds of tests/parity_util.py."""
import numpy as np
import pytest

from tests.parity_util import build_pair, compare_counters, compare_positions, compare_traces, tolerances

pytestmark = pytest.mark.gpu


def _workload(index, scale, seed=None):
    from paper_1611_09160_amd import workloads as W

    return W.config(index, scale=scale, seed=seed)


def test_philox_bit_exact(oracle_mod):
    from paper_1611_09160_amd import wmc

    rng = np.random.default_rng(0)
    for _ in range(3):
        ctr = [int(v) for v in rng.integers(0, 2 ** 32, 4)]
        key = [int(v) for v in rng.integers(0, 2 ** 32, 2)]
        g = wmc.philox(ctr, key, 4096)
        for i in (0, 1, 777, 4095):
            c = [(ctr[0] + i) & 0xFFFFFFFF] + ctr[1:]
            assert list(g[i]) == oracle_mod.philox(c, key)
    assert list(wmc.philox([0, 0, 0, 0], [0, 0], 1)[0]) == [0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8]


@pytest.mark.parametrize("index,scale", [(1, 1.0), (2, 0.25), (3, 0.0625), (4, 0.01)])
def test_schedule_constants_match(index, scale):
    cfg = _workload(index, scale)
    g, o = build_pair(cfg, trace=0)
    for s in range(min(3, g.n_systems)):
        gi, oi = g.system_info(s), o.system_info(s)
        ol = o.level_info(s)
        assert len(gi["levels"]) == len(ol)
        for a, b in zip(gi["levels"], ol):
            for k in ("lo", "hi", "p", "T", "h"):
                assert a[k] == pytest.approx(b[k], rel=1e-12), k
            if cfg["params"]["periodic"]:
                assert int(a["ncell"]) == b["ncell"]
        for k in ("P_F", "dt"):
            assert gi[k] == pytest.approx(oi[k], rel=1e-11, abs=1e-300), k


@pytest.mark.parametrize("index,scale", [(1, 1.0), (2, 0.25), (3, 0.0625), (4, 0.01)])
def test_cell_ids_bit_exact(index, scale):
    cfg = _workload(index, scale)
    g, o = build_pair(cfg, trace=0)
    for s in range(min(3, g.n_systems)):
        nl = len(o.level_info(s))
        for sweep in (0, 7, 123456):
            for level in range(nl):
                np.testing.assert_array_equal(g.cell_ids(s, sweep, level), o.cell_ids(s, sweep, level))


@pytest.mark.parametrize("index,scale,sweeps", [(1, 1.0, 3), (2, 0.25, 2), (3, 0.0625, 2), (3, 0.25, 2), (4, 0.01, 1)])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_sweep_parity(index, scale, sweeps, precision):
    cfg = _workload(index, scale)
    g, o = build_pair(cfg, precision=precision)
    for s in range(sweeps):
        start = o.positions()
        g.set_state(start, s)
        o.set_sweep(s)
        g.sweep(1)
        o.sweep(1)
        # mixed mode reports FP32-accurate energies; its decisions are rechecked in FP64 near
        # the threshold, so they must still match exactly
        tol, prt = tolerances(precision)
        stats = compare_traces(g.trace(), o.trace(), **tol)
        assert stats["moves"] > 0
        compare_positions(g.positions(), o.positions(), rtol=prt)
    compare_counters(g.observables(), o.observables())
    np.testing.assert_allclose(g.tau(), o.tau(), rtol=1e-12)
    np.testing.assert_allclose(g.chain_rg2(), o.chain_rg2(), rtol=1e-10 if precision == "fp64" else 1e-5)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batched_copies_parity(precision):
    """Three 8192-bead semi-dilute systems in one batch: every colour phase of the top levels and
    the plane waves run as several cooperative groups in one launch."""
    from paper_1611_09160_amd import workloads as W

    cfg = W.replicas(3, 3, 0.25)
    g, o = build_pair(cfg, precision=precision, trace=2_000_000)
    g.sweep(1)
    o.sweep(1)
    tol, prt = tolerances(precision)
    stats = compare_traces(g.trace(2_000_000), o.trace(2_000_000), **tol)
    assert stats["moves"] > 0
    compare_positions(g.positions(), o.positions(), rtol=prt)
    compare_counters(g.observables(), o.observables())
    np.testing.assert_allclose(g.tau(), o.tau(), rtol=1e-12)


@pytest.mark.parametrize("verify", [0, 1])
def test_mixed_rechecks_near_threshold(verify):
    """An adversarial state for the FP32 energy terms: every bond stretched to 1.45 (R0 = 1.5, where
    the FENE term is steep) and beads packed to within 0.85 sigma (steep WCA). Decisions near the
    threshold are re-evaluated in FP64 (rechecks > 0) and every decision equals the oracle's. With
    mixed_verify every FP32-tile test is evaluated in FP64 too: the FP32 error never exceeds the
    recheck margin (and the decisions are the same as without it)."""
    from paper_1611_09160_amd import workloads as W

    # box 24: the level-0 cells (side 6) run on FP32 LDS tiles, the coarser levels on the global path
    sysd = W.make_solution(n_chains=162, n_beads=32, box_L=24.0, seed=77, bond=1.45, min_dist=0.85)
    params = dict(W.KG, periodic=1, plane_waves=1, box_L=24.0, lambda_max=4.0, seed=78, mixed_verify=verify)
    cfg = dict(params=params, pos=sysd["pos"], chain_offset=sysd["chain_offset"],
               sys_offset=np.array([0, len(sysd["pos"])]))
    g, o = build_pair(cfg, precision="mixed")
    g.sweep(1)
    o.sweep(1)
    # the reported dU carries FP32 errors of terms up to ~1e3 here; the decisions are exact
    stats = compare_traces(g.trace(), o.trace(), dU_rtol=1e-3, dU_atol=1e-2, dU_atol_member=1e-2)
    compare_positions(g.positions(), o.positions(), rtol=tolerances("mixed")[1])
    ob = g.observables()
    assert ob["rechecks"] > 0, ob["rechecks"]
    assert ob["rechecks"] < 0.2 * stats["moves"]
    compare_counters(ob, o.observables())
    print(f"moves {stats['moves']} rechecks {ob['rechecks']} member rechecks {ob['member_rechecks']} "
          f"margin checks {ob['margin_checks']} max |dU32 - dU64| / margin {ob['margin_max_ratio']:.3g}")
    if verify:
        assert ob["margin_checks"] > 0.3 * stats["moves"], (ob["margin_checks"], stats["moves"])
        assert ob["margin_fails"] == 0 and ob["margin_max_ratio"] < 1.0, (ob["margin_fails"], ob["margin_max_ratio"])
    else:
        assert ob["margin_checks"] == 0


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_forced_caps_and_infinite_energies(precision):
    """Large moves (A0 = 5) with a retry cap of 2 on the semi-dilute solution: many tests stretch a
    FENE bond past R0 (an infinite dU, always rejected) and many chains end at the cap; the trace,
    the infinite records and the counters equal the oracle's."""
    cfg = _workload(3, 0.0625)
    g, o = build_pair(cfg, precision=precision, A0=5.0, retry_cap=2)
    g.sweep(1)
    o.sweep(1)
    tg, to = g.trace(), o.trace()
    tol, prt = tolerances(precision)
    compare_traces(tg, to, **tol)
    moves = to["kind"] != 1
    assert np.isinf(to["dU"][moves]).sum() > 0
    assert np.isinf(tg["dU"][tg["kind"] != 1]).sum() == np.isinf(to["dU"][moves]).sum()
    ob = o.observables()
    assert ob["caps"].sum() > 0, ob["caps"]
    compare_counters(g.observables(), ob)
    compare_positions(g.positions(), o.positions(), rtol=prt)


def test_mixed_margin_on_semidilute():
    """mixed_verify on the semi-dilute solution (64 x 128 beads): every FP32-tile test's FP32 error
    stays within its recheck margin, and the decisions still equal the oracle's."""
    cfg = _workload(3, 0.25)
    g, o = build_pair(cfg, precision="mixed", mixed_verify=1)
    g.sweep(1)
    o.sweep(1)
    tol, prt = tolerances("mixed")
    stats = compare_traces(g.trace(), o.trace(), **tol)
    compare_positions(g.positions(), o.positions(), rtol=prt)
    ob = g.observables()
    compare_counters(ob, o.observables())
    print(f"tests {stats['moves']} verified {ob['margin_checks']} rechecks {ob['rechecks']} support rechecks "
          f"{ob['member_rechecks']} max |dU32 - dU64| / margin {ob['margin_max_ratio']:.3g}")
    assert ob["margin_checks"] > 0.3 * stats["moves"], (ob["margin_checks"], stats["moves"])
    assert ob["margin_fails"] == 0 and ob["margin_max_ratio"] < 1.0, (ob["margin_fails"], ob["margin_max_ratio"])


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_full_size_semidilute_one_sweep(precision):
    """The benchmark workload (256 x 128 beads, L = 84) for one sweep against the oracle."""
    cfg = _workload(3, 1.0)
    g, o = build_pair(cfg, trace=4_000_000, precision=precision)
    g.sweep(1)
    o.sweep(1)
    tol, prt = tolerances(precision)
    stats = compare_traces(g.trace(4_000_000), o.trace(4_000_000), **tol)
    err = compare_positions(g.positions(), o.positions(), rtol=prt)
    compare_counters(g.observables(), o.observables())
    print(f"{precision}: {stats['moves']} tests, max |dU - dU_oracle| {stats['max_dU_diff']:.3g}, "
          f"max position error / (1 + |x|) {err:.3g}")


def test_full_size_after_equilibration():
    """The benchmark workload after 150 GPU sweeps (dense regions, large member lists appear):
    no list overflows, then one more sweep from the GPU state against the oracle."""
    cfg = _workload(3, 1.0)
    g, _ = build_pair(cfg, trace=0)
    g.sweep(150)
    ob = g.observables()
    assert ob["overflows"] == 0 and ob["violations"] == 0, (ob["overflows"], ob["violations"])
    pos = g.positions()
    g.close()
    g2, o = build_pair(dict(cfg, pos=pos), trace=4_000_000)
    g2.set_state(pos, 150)
    o.set_sweep(150)
    g2.sweep(1)
    o.sweep(1)
    compare_traces(g2.trace(4_000_000), o.trace(4_000_000))
    compare_positions(g2.positions(), o.positions())
    assert g2.observables()["overflows"] == 0


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_resume_is_bit_exact(precision):
    """A run is determined by (positions, sweep counter, seed): 6 sweeps in one go equal 3 sweeps,
    a fresh context started from those positions at sweep 3, and 3 more sweeps."""
    cfg = _workload(3, 0.0625)
    a, _ = build_pair(cfg, precision=precision, trace=0)
    a.sweep(6)
    full = a.positions()
    b, _ = build_pair(cfg, precision=precision, trace=0)
    b.sweep(3)
    mid = b.positions()
    c, _ = build_pair(dict(cfg, pos=mid), precision=precision, trace=0)
    c.set_state(mid, 3)
    c.sweep(3)
    np.testing.assert_array_equal(c.positions(), full)


def test_full_size_dilute_chain_one_sweep():
    """The dilute workload (one 1024-bead chain, L = 128) for one sweep against the oracle."""
    cfg = _workload(2, 1.0)
    g, o = build_pair(cfg, trace=1_000_000)
    g.sweep(1)
    o.sweep(1)
    compare_traces(g.trace(1_000_000), o.trace(1_000_000))
    compare_positions(g.positions(), o.positions())
    compare_counters(g.observables(), o.observables())


# --------------------------------------------------------------- variants of the method
VARIANTS = {
    "glauber": dict(accept="glauber"),
    "rotation": dict(wavelet_map="rotation"),
    "uniform-centres": dict(centring="uniform"),
    "all-three": dict(accept="glauber", wavelet_map="rotation", centring="uniform"),
}


@pytest.mark.parametrize("name", list(VARIANTS))
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_variant_parity(name, precision):
    """Glauber acceptance, the exact-rotation map and uniform centres on the semi-dilute solution
    (64 x 32 beads: LDS-tile levels, global-list cell groups and plane waves)."""
    cfg = _workload(3, 0.25)
    g, o = build_pair(cfg, precision=precision, **VARIANTS[name])
    tol, prt = tolerances(precision)
    for s in range(2):
        start = o.positions()
        g.set_state(start, s)
        o.set_sweep(s)
        g.sweep(1)
        o.sweep(1)
        stats = compare_traces(g.trace(), o.trace(), **tol)
        assert stats["moves"] > 0
        compare_positions(g.positions(), o.positions(), rtol=prt)
    compare_counters(g.observables(), o.observables())
    np.testing.assert_allclose(g.tau(), o.tau(), rtol=1e-12)


@pytest.mark.parametrize("over", [dict(), dict(wavelet_map="rotation", accept="glauber")])
def test_infinite_plane_waves_parity(over):
    """The ideal chain (64 beads, infinite system) with infinite-system plane waves, and a dilute
    FENE + WCA chain in an infinite system with them (every pair in the plane-wave energy)."""
    cfg = _workload(1, 1.0)
    # lambda 1..3: P_F = 1/27, about 2.4 plane waves per sweep of the 64 beads
    g, o = build_pair(cfg, plane_waves=1, lambda_max=3.0, **over)
    for s in range(4):
        start = o.positions()
        g.set_state(start, s)
        o.set_sweep(s)
        g.sweep(1)
        o.sweep(1)
        compare_traces(g.trace(), o.trace())
        compare_positions(g.positions(), o.positions())
    ob = g.observables()
    assert ob["pw_attempts"] > 0
    compare_counters(ob, o.observables())
    gi, oi = g.system_info(0), o.system_info(0)
    assert gi["P_F"] == pytest.approx(oi["P_F"], rel=1e-15) and gi["dt"] == pytest.approx(oi["dt"], rel=1e-12)
    # dilute FENE + WCA chain, infinite system
    from paper_1611_09160_amd import workloads as W

    sysd = W.make_solution(1, 256, 1000.0, seed=5, periodic=False)
    params = dict(W.KG, periodic=0, plane_waves=1, lambda_max=4.0, seed=6, **over)
    cfg2 = dict(params=params, pos=sysd["pos"], chain_offset=sysd["chain_offset"], sys_offset=np.array([0, 256]))
    g2, o2 = build_pair(cfg2)
    for s in range(4):
        start = o2.positions()
        g2.set_state(start, s)
        o2.set_sweep(s)
        g2.sweep(1)
        o2.sweep(1)
        compare_traces(g2.trace(), o2.trace())
        compare_positions(g2.positions(), o2.positions())
    ob2 = g2.observables()
    assert ob2["pw_attempts"] > 0
    compare_counters(ob2, o2.observables())


def test_centre_of_mass_observables():
    """Chain centres of mass (Sec. VI.B) and their squared displacement since the start."""
    cfg = _workload(3, 0.0625)
    g, o = build_pair(cfg, trace=0)
    com0 = o.chain_com()
    np.testing.assert_allclose(g.chain_com(), com0, rtol=1e-13, atol=1e-12)
    assert np.all(g.chain_msd() == 0.0)
    g.sweep(3)
    o.sweep(3)
    com = o.chain_com()
    np.testing.assert_allclose(g.chain_com(), com, rtol=1e-10, atol=1e-10)
    np.testing.assert_allclose(g.chain_msd(), np.sum((com - com0) ** 2, 1), rtol=1e-8, atol=1e-14)


def test_repeated_runs_are_bit_identical():
    """Two runs of the same state give identical positions and identical counters, including the
    cells that fell back from the LDS tile (the drift bound a cell uses no longer depends on the
    timing of cells it does not wait for)."""
    from paper_1611_09160_amd import workloads as W

    cfg = W.replicas(3, 3, 0.25)
    res = []
    for _ in range(2):
        g, _ = build_pair(cfg, trace=0, precision="mixed")
        g.sweep(4)
        res.append((g.positions(), g.observables()))
        g.close()
    np.testing.assert_array_equal(res[0][0], res[1][0])
    for k in ("fallback_cells", "rechecks", "grid_rebuilds", "accepted_total", "overflows", "wait_timeouts"):
        assert res[0][1][k] == res[1][1][k], k
    np.testing.assert_array_equal(res[0][1]["attempts"], res[1][1]["attempts"])
