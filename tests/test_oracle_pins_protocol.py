"""CPU pins of the oracle's grasp-validation controls (Sec. III-D):

* contact forces between tagged bodies: antisymmetric (the force on a from b is minus the force on b from
  a), and for a block resting on the ground they balance its weight (the ground pushes the block up by
  m g);
* a held kinematic group keeps the target of its hold row: a plate stopped mid-press stays exactly there
  while the schedule would have moved it further;
* a gravity override replaces the schedule: free fall along +x follows the implicit-Euler closed form
  x_n = x_0 + h^2 g n (n + 1) / 2, and releasing the override restores the schedule.
"""
import numpy as np
import pytest

import oracle as O
from paper_2503_05020_amd import scenes as S


def test_contact_forces_balance_the_weight_at_rest():
    sc = S.soft_cube_drop(cells=2, edge=0.02, height=0.0005)
    o = O.Scene(sc)
    for _ in range(60):
        assert o.step(1)[0] == 0
    pos, vel = o.state()
    assert np.abs(vel[sc["kin_group"] < 0]).max() < 1e-3
    tags = sc["body"]  # 0 the cube, 1 the ground
    F = o.contact_forces(pos, tags, 2)
    m = o.mass()[sc["kin_group"] < 0].sum()
    assert np.allclose(F[0, 1], -F[1, 0], rtol=0, atol=1e-15 * m * 9.81)
    assert F[0, 1][2] == pytest.approx(m * 9.81, rel=2e-3)
    # the vertex jitter tilts the contact normals slightly: the horizontal parts nearly cancel
    assert abs(F[0, 1][0]) < 1e-3 * m * 9.81 and abs(F[0, 1][1]) < 1e-3 * m * 9.81
    assert np.all(F[0, 0] == 0) and np.all(F[1, 1] == 0)
    # tags outside the range are ignored
    assert np.all(o.contact_forces(pos, np.full_like(tags, -1), 2) == 0)


def test_hold_group_keeps_the_target_of_its_row():
    sc = S.press_block(steps=8, speed=0.05)
    o = O.Scene(sc, pcg_rel_tol=1e-8)
    kin = sc["kin_group"]
    X = sc["rest_pos"]
    for _ in range(3):
        assert o.step(1)[0] == 0
    o.hold_group(1, 3)  # the plate stays at the target of motion row 3 from now on
    row3 = X[kin == 1, 2] + sc["motion"][3, 1, 11]
    for k in range(3):
        assert o.step(1)[0] == 0
        pos, _ = o.state()
        assert np.array_equal(pos[kin == 1, 2], row3)
    # the schedule would have moved it on: releasing the hold resumes it
    o.hold_group(1, -1)
    assert o.step(1)[0] == 0
    pos, _ = o.state()
    assert np.array_equal(pos[kin == 1, 2], X[kin == 1, 2] + sc["motion"][7, 1, 11])


def test_gravity_override_free_fall_closed_form():
    sc = S.free_block(cells=1, gravity=(0.0, 0.0, 0.0))
    o = O.Scene(sc, linear_solver=1)
    g = np.array([9.8, 0.0, 0.0])
    o.set_gravity(g)
    x0 = sc["rest_pos"].copy()
    h = sc["dt"]
    for n in range(1, 6):
        assert o.step(1)[0] == 0
        pos, _ = o.state()
        ref = x0 + h * h * g * n * (n + 1) / 2.0
        assert np.abs(pos - ref).max() < 1e-12
    o.set_gravity(None)  # back to the schedule (no gravity): the block coasts at its velocity
    _, v = o.state()
    before, _ = o.state()
    assert o.step(1)[0] == 0
    after, _ = o.state()
    assert np.abs(after - before - h * v).max() < 1e-12
