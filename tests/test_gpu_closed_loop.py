"""The closed loop of Alg. 2 and Sec. III-F on the GPU: a ball flying
through the arm hits it when the arm only holds its pose, and the
task-priority controller fed by the exact-EDT sphere queries keeps every
sphere clear of it."""
import numpy as np
import pytest

from paper_2407_02363_amd import inputs
from paper_2407_02363_amd.closed_loop import ARM_GRID, ClosedLoop, fly_through
from tests.gpu_util import say

pytestmark = pytest.mark.gpu


def test_avoidance_keeps_the_arm_clear():
    ci = inputs.cycle_inputs(0, n_frames=1, n_states=4)
    q0 = np.array([0.3, 0.6, -0.2, -0.9, 0.1, 0.5, 0.0])
    C = inputs.sphere_centres(ci.robot, q0, ci.sphere_links, ci.sphere_local)
    top = np.array([ARM_GRID.nx, ARM_GRID.ny, ARM_GRID.nz]) * ARM_GRID.voxel
    assert (C > 0.2).all() and (C < top - 0.2).all()    # the whole arm, and the ball, in the map
    loop = ClosedLoop(ci)
    obstacle = fly_through(ci, q0)
    steps = 750
    say("[closed loop] holding only")
    hold, _, _ = loop.run(q0, obstacle, steps, avoid=False)
    say("[closed loop] with avoidance")
    avoid, traj, dt = loop.run(q0, obstacle, steps, avoid=True)
    say(f"[closed loop] min clearance hold {hold.min():.3f} m, avoid {avoid.min():.3f} m, "
        f"{1e3 * dt:.3f} ms per step")
    assert hold.min() < -0.02                  # the ball passes through the arm
    assert avoid.min() > 0.0                   # no sphere ever touches it
    assert np.isfinite(traj).all()
