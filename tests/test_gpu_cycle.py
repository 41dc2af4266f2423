"""The whole control cycle (Alg. 2) on the GPU against the CPU oracle, and
HIP-graph replays of it against eager runs."""
import numpy as np
import pytest
import torch

from paper_2407_02363_amd import inputs
from paper_2407_02363_amd.cycle import ControlCycle
from tests.gpu_util import say

pytestmark = pytest.mark.gpu


def oracle_cycle(oracle_lib, ci, k, centres):
    g = ci.grid
    q = ci.joint_states[k % len(ci.joint_states)]
    occ_s = np.zeros(g.shape, np.uint8)
    oracle_lib.insert_links(g, occ_s, ci.link_pts, ci.link_off, ci.robot.poses12(q), 0xFF)
    occ_e = np.zeros(g.shape, np.uint8)
    oracle_lib.insert_points(g, occ_e, ci.frames[k % len(ci.frames)], ci.T_map_cam, exclude=occ_s)
    d2e, se = oracle_lib.edt(occ_e)
    d2s, ss = oracle_lib.edt(occ_s)
    c = centres[k % len(ci.joint_states)]
    return (occ_s, occ_e, d2e, se, d2s, ss,
            oracle_lib.query_spheres(g, d2e, se, c, ci.sphere_radii),
            oracle_lib.query_spheres(g, d2s, ss, c, ci.sphere_radii))


def gpu_state(cyc):
    sh = cyc.grid.shape
    return (cyc.occ_self.cpu().numpy().reshape(sh), cyc.occ_env.cpu().numpy().reshape(sh),
            cyc.d2_env.cpu().numpy().reshape(sh), cyc.site_env.cpu().numpy().reshape(sh),
            cyc.d2_self.cpu().numpy().reshape(sh), cyc.site_self.cpu().numpy().reshape(sh),
            cyc.out_env.cpu().numpy().view(np.uint32), cyc.out_self.cpu().numpy().view(np.uint32))


NAMES = ["occ_self", "occ_env", "d2_env", "site_env", "d2_self", "site_self", "q_env", "q_self"]


@pytest.mark.parametrize("variant", ["many", "per_map", "batched", "two_streams"])
def test_cycle_matches_oracle(oracle_lib, variant):
    ci = inputs.cycle_inputs(4, n_frames=2, n_states=3)
    cyc = ControlCycle(ci, "cuda:0", edt_mode="per_map" if variant == "two_streams" else variant,
                       two_streams=variant == "two_streams")
    for k in range(3):
        say(f"[cycle] k={k} {variant}")
        cyc.run(k)
        torch.cuda.synchronize()
        got = gpu_state(cyc)
        ref = oracle_cycle(oracle_lib, ci, k, cyc.centres_host)
        for name, a, b in zip(NAMES, got, ref):
            assert np.array_equal(a, b), f"cycle {k}: {name} differs"


@pytest.mark.parametrize("variant", ["many", "two_streams"])
def test_graph_replays_match_eager(variant):
    ci = inputs.cycle_inputs(5, n_frames=2, n_states=2)
    cyc = ControlCycle(ci, "cuda:0", edt_mode="per_map" if variant == "two_streams" else variant,
                       two_streams=variant == "two_streams")
    say("[cycle graph] capture")
    graphs = cyc.capture_graphs(2)
    eager = []
    for k in range(2):
        cyc.run(k)
        torch.cuda.synchronize()
        eager.append(gpu_state(cyc))
    # replay several times, with eager work and synchronisations in between
    for rep in range(4):
        for k in (1, 0):
            say(f"[cycle graph] replay {rep} slot {k}")
            graphs[k].replay()
            torch.cuda.synchronize()
            got = gpu_state(cyc)
            for name, a, b in zip(NAMES, got, eager[k]):
                assert np.array_equal(a, b), f"replay {rep} slot {k}: {name} differs"
            cyc.run(1 - k)
            torch.cuda.synchronize()


def test_split_graph_replays_match_eager():
    """The two-stream cycle replayed from three graphs per slot gives the
    eager cycle's bytes, replay after replay."""
    ci = inputs.cycle_inputs(6, n_frames=2, n_states=2)
    cyc = ControlCycle(ci, "cuda:0", edt_mode="per_map")
    eager = []
    for k in range(2):
        cyc.run(k)
        torch.cuda.synchronize()
        eager.append(gpu_state(cyc))
    say("[cycle split graphs] capture")
    cyc.capture_split_graphs(2)
    for rep in range(3):
        for k in (1, 0):
            say(f"[cycle split graphs] replay {rep} slot {k}")
            cyc.replay_split(k)
            torch.cuda.synchronize()
            for name, a, b in zip(NAMES, gpu_state(cyc), eager[k]):
                assert np.array_equal(a, b), f"replay {rep} slot {k}: {name} differs"
