"""GPU (FP32 HIP kernel through the C ABI of include/link.h) against the
FP64 oracle of the full-resolution link, per the substep protocol of
tests/link_parity.py: index work bit for bit; positions 1e-5, velocities
and multipliers 1e-4 relative per block type."""
import numpy as np
import pytest

import oracle.link as OL
import workloads as W
from link_parity import (advance_both, assert_parity, compare, gpu_state, load_gpu, load_oracle,
                         state_after)

pytestmark = pytest.mark.gpu
LK = pytest.importorskip("paper_1904_02833_amd.link")


@pytest.mark.parametrize("n_links,ground", [(4, True), (1, True), (3, False)])
def test_link_index_bit_exact(n_links, ground):
    wl = W.make_link(2, n_links=n_links)
    flags = 0 if ground else OL.NO_GROUND
    o = OL.LinkOracle(wl, flags=flags)
    ix = o.index()
    sim = LK.LinkSim(wl, flags=flags)
    got = {k: sim.index(k) for k in LK.INDEX}
    sim.close()
    assert np.array_equal(got["dist_i"], ix["dist_i"])
    assert np.array_equal(got["dist_j"], ix["dist_j"])
    assert np.array_equal(got["dist_kind"], ix["dist_kind"])
    assert np.array_equal(got["degree_particle"], ix["degree_particle"])
    assert np.array_equal(got["degree_frame"], ix["degree_frame"])


def test_link_initial_state_matches_oracle():
    wl = W.make_link(3, n_links=2)
    o = OL.LinkOracle(wl)
    sim = LK.LinkSim(wl)
    g = gpu_state(sim)
    sim.close()
    assert np.array_equal(g["x"], o.x.astype(np.float32).astype(np.float64))
    assert np.array_equal(g["fx"], o.fx.astype(np.float32).astype(np.float64))
    assert np.array_equal(g["fq"], o.fq)


@pytest.mark.parametrize("steps", [0, 6])
def test_link_substep_parity(steps):
    """Four snakes of four links: one substep of 20 iterations from the
    oracle's state after `steps` steps of drawn commands (0: at rest on the
    ground, the first substep of a drop onto the contacts)."""
    wl = W.make_link(4, n_links=4)
    st = state_after(wl, steps)
    o, g = advance_both(wl, st)
    assert np.array_equal(np.asarray(g["iters"]), o.iters)
    assert_parity(f"link substep after {steps} steps", compare(o, g), wl.particles * wl.n_snakes)
