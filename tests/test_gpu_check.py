"""usp_check through the C ABI: NaN and infinite values in a state, and
injections dropped for lack of capacity, become the statuses USP_ENUMERIC
and USP_ECAPACITY; a cell whose sums are not finite is not collided and
does not spread its values to its neighbours."""
import sys

import numpy as np
import pytest

import usp_workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

OK, ECAPACITY, ENUMERIC = 0, -3, -4


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_clean_state_checks_ok():
    from paper_2508_05642_amd import usp
    prob = W.poiseuille(kn=0.05, cells=16, ppc=60, f32=True)
    parts = W.particles_for(prob)
    _say(f"[check] clean channel n={parts['n']}")
    st = usp.DeviceState(prob, parts)
    st.step(0, 2)
    status, found = st.check()
    assert (status, found) == (OK, 0)
    assert st.cnt()["NONFINITE"] == 0


@pytest.mark.parametrize("bad", [float("nan"), float("inf")])
def test_nonfinite_velocity_is_reported_and_contained(bad):
    """One particle with a non-finite velocity: the scan finds it before a
    step; after a step its cell is counted, not collided, and every particle
    of the other cells stays finite."""
    from paper_2508_05642_amd import usp
    prob = W.poiseuille(kn=0.05, cells=16, ppc=60, f32=True)
    parts = W.particles_for(prob)
    k = 7
    parts["cx"][k] = bad
    _say(f"[check] channel with cx[{k}] = {bad}, n={parts['n']}")
    st = usp.DeviceState(prob, parts)
    status, found = usp.usp_check(st.grid, st.p, None, None, st.counters)
    assert (status, found) == (ENUMERIC, 1)
    st.counters.zero_()
    st.step(0, 1)
    s = st.state()
    assert st.cnt()["NONFINITE"] == 1
    bad_pid = int(parts["pid"][k])
    i = int(np.nonzero(s["pid"] == bad_pid)[0][0])
    c = int(s["cell"][i])
    cs = st.cellstate()
    from paper_2508_05642_amd import usp as U
    assert cs[U.names("cs").index("COLLIDE"), c] == 0.0
    others = s["cell"] != c
    for f in ("y", "cx", "cy", "cz", "erot"):
        assert np.all(np.isfinite(s[f][others])), f
    status, found = st.check()
    assert status == ENUMERIC and found >= 1


def test_nonfinite_position_is_reported():
    from paper_2508_05642_amd import usp
    prob = W.poiseuille(kn=0.05, cells=16, ppc=60, f32=True)
    parts = W.particles_for(prob)
    parts["y"][3] = np.nan
    _say(f"[check] channel with y[3] = nan, n={parts['n']}")
    st = usp.DeviceState(prob, parts)
    status, found = usp.usp_check(st.grid, st.p, None, None, st.counters)
    assert (status, found) == (ENUMERIC, 1)


def test_dropped_injections_report_capacity():
    """A cylinder state whose buffers have no free slot: the first step's
    injection is dropped and counted, and usp_check returns USP_ECAPACITY."""
    from paper_2508_05642_amd import usp
    prob = W.cylinder(scale=0.05, f32=True)
    parts = W.particles_for(prob)
    n = int(parts["n"])
    _say(f"[check] cylinder scale 0.05 at capacity n={n}")
    st = usp.DeviceState(prob, parts, capacity=n)
    st.step(0, 1)
    assert st.cnt()["CAPACITY"] > 0
    status, found = st.check()
    assert (status, found) == (ECAPACITY, 0)
