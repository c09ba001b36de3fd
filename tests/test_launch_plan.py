"""Launch plans checked on the host (CPU only, no device): wmc_launch_plan builds the plan wmc_init
would make for given co-residency limits and checks every index the kernels derive from it
(block maps, cooperative group tables, per-workgroup result slots, barrier words, list slices,
global list slots, cell flags)."""
import os

import pytest

from tests.conftest import ROOT


@pytest.fixture(scope="module")
def wmc_mod():
    from paper_1611_09160_amd import wmc

    if not os.path.exists(wmc.LIB_PATH):
        pytest.skip("libwmc.so not built")
    wmc.lib()
    return wmc


# (cell-group co-residency, plane-wave co-residency, cell launch cap, plane-wave launch cap): the
# limits of the library (two cell groups and three plane-wave workgroups per CU on 256 CUs, caps
# 256 and 512), and wider ones up to a full 1024-workgroup launch of both kinds
LIMITS = [(512, 768, 256, 512), (512, 768, 1024, 1024), (1024, 1024, 1024, 1024), (64, 64, 64, 64)]


@pytest.mark.parametrize("limits", LIMITS)
def test_plan_of_the_512_system_batch(wmc_mod, batch512, limits):
    """The lognormal batch of 512 systems (724,725 beads, boxes 16..108)."""
    for precision in ("fp64", "mixed"):
        cfg = dict(batch512, params=dict(batch512["params"], precision=precision))
        rc, report = wmc_mod.launch_plan(cfg, *limits)
        assert rc == 0 and report.startswith("ok"), report
        assert "systems 512 beads 724725" in report


@pytest.fixture(scope="module")
def batch512():
    from paper_1611_09160_amd import workloads as W

    return W.config(4)


@pytest.mark.parametrize("index,scale", [(2, 1.0), (3, 1.0), (3, 0.25), (5, 0.0625)])
def test_plan_of_single_systems(wmc_mod, index, scale):
    from paper_1611_09160_amd import workloads as W

    rc, report = wmc_mod.launch_plan(W.config(index, scale), *LIMITS[0])
    assert rc == 0 and report.startswith("ok"), report


def test_plan_of_copies(wmc_mod):
    from paper_1611_09160_amd import workloads as W

    rc, report = wmc_mod.launch_plan(W.replicas(3, 3, 0.25), *LIMITS[0])
    assert rc == 0 and "cell-group launches" in report, report
