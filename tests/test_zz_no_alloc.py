"""The allocation-free entry point wmc_init_static (library-held device arena) against wmc_init
with a caller-allocated arena, on the same seeded inputs: identical accept decisions and
counters, positions within 1e-10 relative. Two contexts in a row, the second on a smaller
problem, so the second reuses the array the first left behind."""
import numpy as np
import pytest

from tests.parity_util import compare_counters, compare_positions, compare_traces

pytestmark = pytest.mark.gpu


def _pair(cfg, sweeps):
    from paper_1611_09160_amd import wmc

    kw = {}
    if "sys_box_L" in cfg:
        kw = dict(sys_box_L=cfg["sys_box_L"], sys_lambda_max=cfg["sys_lambda_max"])
    ref = wmc.WMC(cfg["params"], cfg["sys_offset"], cfg["chain_offset"], cfg["pos"], trace_capacity=100_000, **kw)
    ref.sweep(sweeps)
    st = wmc.WMC(cfg["params"], cfg["sys_offset"], cfg["chain_offset"], cfg["pos"], trace_capacity=100_000,
                 static_arena=True, **kw)
    assert st.arena is None
    st.sweep(sweeps)
    compare_traces(st.trace(), ref.trace())
    compare_positions(st.positions(), ref.positions())
    compare_counters(st.observables(), ref.observables())
    np.testing.assert_array_equal(st.tau(), ref.tau())
    ref.close()
    st.close()


def test_static_arena_matches_caller_arena_twice():
    from paper_1611_09160_amd import workloads as W

    print("no-alloc: semi-dilute 64 x 32 beads, 2 sweeps", flush=True)
    _pair(W.config(3, 0.25), 2)
    print("no-alloc: semi-dilute 16 x 32 beads (smaller), 2 sweeps", flush=True)
    _pair(W.config(3, 0.0625), 2)


def test_static_arena_rejects_oversize_and_second_context():
    from paper_1611_09160_amd import wmc
    from paper_1611_09160_amd import workloads as W

    # 400,000 free beads: their arena exceeds the library-held one (checked before any device work)
    n, box = 400_000, 150.0
    pos = np.random.default_rng(1).uniform(0.0, box, (n, 3))
    params = dict(W.KG, periodic=1, plane_waves=1, box_L=box, lambda_max=box / 4, seed=5)
    with pytest.raises(RuntimeError, match=r"wmc_init_static failed \(-3\)"):
        wmc.WMC(params, [0, n], np.arange(n + 1), pos, static_arena=True)
    cfg = W.config(3, 0.0625)
    a = wmc.WMC(cfg["params"], cfg["sys_offset"], cfg["chain_offset"], cfg["pos"], static_arena=True)
    with pytest.raises(RuntimeError, match="in use"):
        wmc.WMC(cfg["params"], cfg["sys_offset"], cfg["chain_offset"], cfg["pos"], static_arena=True)
    a.close()
    b = wmc.WMC(cfg["params"], cfg["sys_offset"], cfg["chain_offset"], cfg["pos"], static_arena=True)
    b.sweep(1)
    assert b.observables()["overflows"] == 0
    b.close()
