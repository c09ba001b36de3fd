"""Launch tuning (wmc_tune, wmc_set_tuning): the tuner leaves the state exactly as it found it,
each launch choice keeps the oracle's results, and settings applied to a second context reproduce
the first context's sweep bit for bit."""
import numpy as np
import pytest

from tests.parity_util import build_pair, compare_counters, compare_positions, compare_traces

pytestmark = pytest.mark.gpu

NL = 6


def _cfg():
    from paper_1611_09160_amd import workloads as W

    return W.config(3, scale=0.25)  # 64 x 128 beads: tile levels, cell groups, plane waves


def test_tune_restores_state_and_keeps_parity():
    cfg = _cfg()
    g, o = build_pair(cfg)
    g.sweep(2)
    o.sweep(2)
    g.trace()
    o.trace()
    pos0, ob0, tau0 = g.positions(), g.observables(), g.tau()
    tuned = g.tune(2)
    print(tuned)
    np.testing.assert_array_equal(g.positions(), pos0)
    np.testing.assert_array_equal(g.tau(), tau0)
    ob1 = g.observables()
    for k, v in ob0.items():
        np.testing.assert_array_equal(np.asarray(ob1[k]), np.asarray(v), err_msg=k)
    assert len(g.trace()) == 0  # the trial sweeps left no records
    assert {lv["level"] for lv in tuned["levels"]} == set(range(len(tuned["levels"])))
    assert all(lv["ms_per_sweep"] > 0 for lv in tuned["levels"])
    assert g.get_tuning()["levels"] == [{k: v for k, v in lv.items() if k != "ms_per_sweep"} for lv in tuned["levels"]]
    # the tuned launches against the oracle, then a second context with the same settings
    g.sweep(1)
    o.sweep(1)
    compare_traces(g.trace(), o.trace())
    compare_positions(g.positions(), o.positions())
    compare_counters(g.observables(), o.observables())
    g2, _ = build_pair(dict(cfg, pos=pos0), trace=0)
    g2.set_state(pos0, 2)
    g2.set_tuning(tuned)
    g2.sweep(1)
    np.testing.assert_array_equal(g2.positions(), g.positions())


@pytest.mark.parametrize("settings", [
    {"levels": [{"level": l, "pass": "colours"} for l in range(NL)]},
    {"levels": [{"level": l, "variant": "V1024", "groups": "off"} for l in range(NL)], "plane_wave_groups": "off"},
    {"levels": [{"level": l, "variant": "V64", "width": 64} for l in range(NL)]},
    {"levels": [{"level": l, "variant": "V256", "pass": "colours"} for l in range(NL)]},
], ids=["colours", "v1024-no-groups", "width64", "v256-colours"])
def test_launch_choices_keep_parity(settings):
    cfg = _cfg()
    g, o = build_pair(cfg, precision="fp64")
    g.set_tuning(settings)
    for s in range(2):
        start = o.positions()
        g.set_state(start, s)
        o.set_sweep(s)
        g.sweep(1)
        o.sweep(1)
        compare_traces(g.trace(), o.trace())
        compare_positions(g.positions(), o.positions())
    compare_counters(g.observables(), o.observables())


def test_set_tuning_rejects_bad_settings():
    from paper_1611_09160_amd import wmc

    cfg = _cfg()
    g = wmc.WMC(cfg["params"], cfg["sys_offset"], cfg["chain_offset"], cfg["pos"])
    before = g.get_tuning()
    for bad in ('{"levels": [{"level": 0, "pass": "sideways"}]}', '{"levels": [{"level": 99}]}',
                '{"nothing": 1}', '{"levels": [{"level": 1, "variant": "V2048"}]}'):
        with pytest.raises(RuntimeError):
            g.set_tuning(bad)
    assert g.get_tuning() == before
    g.close()
