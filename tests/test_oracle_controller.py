"""Pins of the controller oracle (Sec. III-F, Alg. 3): the activation by
hand, a one-joint worked example, the classic pseudo-inverse solution it
reduces to with every task active and no regularisation, the lower-priority
velocity passing through untouched when no task is active, and the position
Jacobian against finite differences of the arm's forward kinematics; then
the library's tp_step against the oracle."""
import numpy as np
import pytest

from oracle import controller_ref as T
from paper_2407_02363_amd import inputs


def test_activation_by_hand():
    a = T.activation([0.05, 0.1, 0.11, 0.12, 0.13], 0.1, 0.02)
    assert a[0] == 1.0 and a[1] == 1.0 and abs(a[2] - 0.5) < 1e-12 and a[3] == 0.0 and a[4] == 0.0
    xs = np.linspace(0.09, 0.13, 401)
    assert (np.diff(T.activation(xs, 0.1, 0.02)) <= 1e-15).all()   # non-increasing, continuous


def test_one_joint_worked_example():
    # a joint about z at the origin; the sphere at (1, 0, 0); the obstacle
    # 0.1 m away along +y: J = (0, -1, 0) . (z x (1, 0, 0)) = -1; with
    # x_M = 0.2 the task is active, xdot = 2 (0.25 - 0.1) = 0.3, so
    # qdot = J^-1 xdot = -0.3 (turn towards -y), whatever qdot0 wants
    q, A, x = T.step([[0, 0, 1]], [[0, 0, 0]], [1], [[1, 0, 0]], [[1, 0.1, 0]], [0.2], qdot0=[5.0],
                     buffer=0.02, target_offset=0.05, gain=2.0, reg_max=0.0)
    assert abs(x[0] - 0.1) < 1e-15 and A[0] == 1.0 and abs(q[0] + 0.3) < 1e-12


def random_case(seed, active):
    g = inputs.rng(seed)
    robot = inputs.make_robot(seed)
    qs = inputs.random_joint_states(1, seed)[0]
    axes, origins = robot.joint_frames(qs)
    f = robot.fk(qs)
    m = 10
    links = g.integers(1, 8, m)
    C = np.array([f[l][:, 3] + f[l][:, :3] @ np.array([0, 0, g.uniform(0, robot.lengths[l])])
                  for l in links])
    dirs = g.normal(size=(m, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    dist = g.uniform(0.02, 0.3, m)
    O = C + dirs * dist[:, None]
    x_m = dist + (0.01 if active else -0.05)          # active: x < x_M; inactive: x >= x_M + b
    return axes, origins, links, C, O, x_m, g.normal(size=7)


def test_all_active_unregularised_is_the_classic_solution():
    axes, origins, links, C, O, x_m, q0 = random_case(3, True)
    q, A, x = T.step(axes, origins, links, C, O, x_m, qdot0=q0, reg_max=0.0, pinv_tol=1e-10)
    assert (A == 1.0).all()
    _, J = T.task_jacobian(axes, origins, links, C, O)
    xdot = 2.0 * (x_m + 0.05 - x)
    Jp = np.linalg.pinv(J, rcond=1e-10)
    ref = Jp @ xdot + (np.eye(7) - Jp @ J) @ q0
    assert np.allclose(q, ref, rtol=1e-8, atol=1e-10)


def test_inactive_tasks_pass_qdot0_through():
    axes, origins, links, C, O, x_m, q0 = random_case(4, False)
    q, A, _ = T.step(axes, origins, links, C, O, x_m, qdot0=q0)
    assert (A == 0.0).all() and np.allclose(q, q0, rtol=0, atol=1e-12)


def test_position_jacobian_by_finite_differences():
    robot = inputs.make_robot(5)
    q = inputs.random_joint_states(1, 6)[0]
    axes, origins = robot.joint_frames(q)
    for link in (1, 4, 7):
        local = np.array([0.0, 0.0, 0.6 * robot.lengths[link]])
        point = lambda qq: robot.fk(qq)[link][:, :3] @ local + robot.fk(qq)[link][:, 3]
        C = point(q)
        O = C + np.array([0.05, -0.02, 0.03])
        x, J = T.task_jacobian(axes, origins, [link], [C], [O])
        h = 1e-6
        num = np.zeros(7)
        for j in range(7):
            dq = np.zeros(7)
            dq[j] = h
            xp = np.linalg.norm(O - point(q + dq))
            xm = np.linalg.norm(O - point(q - dq))
            num[j] = (xp - xm) / (2 * h)
        assert np.allclose(J[0], num, atol=1e-7), (link, J[0], num)


@pytest.mark.parametrize("seed,active", [(7, True), (8, False), (9, None)])
def test_library_matches_oracle(seed, active):
    from paper_2407_02363_amd import controller as TC
    axes, origins, links, C, O, x_m, q0 = random_case(seed, bool(active))
    if active is None:   # a mix: some active, some in transition, some off
        x_m = np.linalg.norm(O - C, axis=1) + inputs.rng(seed).uniform(-0.03, 0.01, len(links))
    args = dict(buffer=0.02, target_offset=0.05, gain=2.0, reg_max=1e-3, reg_width=1e-2, pinv_tol=1e-12)
    ql, Al, xl = TC.tp_step(axes, origins, links, C, O, x_m, qdot0=q0, **args)
    qr, Ar, xr = T.step(axes, origins, links, C, O, x_m, qdot0=q0, **args)
    assert np.array_equal(xl, xr) or np.allclose(xl, xr, rtol=1e-15, atol=0)
    assert np.allclose(Al, Ar, rtol=0, atol=1e-14)
    scale = np.abs(qr).max() + 1e-12
    assert np.allclose(ql, qr, rtol=0, atol=1e-8 * scale), (ql, qr)


def test_library_rejects_bad_arguments():
    from paper_2407_02363_amd import controller as TC
    from paper_2407_02363_amd.edt import EdtError
    with pytest.raises(EdtError):
        TC.tp_step(np.zeros((0, 3)), np.zeros((0, 3)), [], np.zeros((0, 3)), np.zeros((0, 3)), [])
    with pytest.raises(EdtError):
        TC.tp_step([[0, 0, 1]], [[0, 0, 0]], [2], [[1, 0, 0]], [[1, 0.1, 0]], [0.2])
    with pytest.raises(EdtError):
        TC.tp_step([[0, 0, 1]], [[0, 0, 0]], [1], [[1, 0, 0]], [[1, 0.1, 0]], [0.2], buffer=0.0)
