"""Pins of the raycast contact-depth oracle (App. A.1, raycast backend).

- A box face, probes on its normal axis: outside at height h the depth is R - h (the sphere
  test), inside at depth h' it is R + h' (the ray test leaving through the face), i.e. R - phi with
  phi the box's exact SDF, on both sides; the normal is the face's outward normal.
- An axis tilted by theta from the face normal, probe inside at depth h': the ray leaves after
  h' / cos(theta), so the depth is R + h' / cos(theta); outside the tilt changes nothing.
- A finely tessellated sphere against the analytic sphere: outside probes within the mesh's
  sagitta of R - phi, inside probes along the radius likewise.
- A filler probe (R = 0) and a probe beyond R of every face read zero; rigid motion of link and
  object together changes nothing.
Poses enter as FP32, as the library's inputs do, so closed forms hold to the rounding of the
probe position (2e-9 m).
"""
import numpy as np
import pytest

import oracle
from paper_2606_22332_amd import synth


def one_probe(x, n, R, mesh, q=(1, 0, 0, 0), p=(0, 0, 0), obj=None):
    """One link with one taxel at link-frame origin-less pose: the link pose puts the taxel at x
    with axis n (world frame, identity rotation unless q given)."""
    off = np.array([0, 1], np.int32)
    pos = np.zeros((1, 3), np.float32)
    nrm = np.asarray(n, np.float32).reshape(1, 3)
    rad = np.array([R], np.float32)
    ls = np.zeros((1, 13, 1), np.float32)
    ls[0, 0:3, 0] = x
    ls[0, 3:7, 0] = q
    oid = np.zeros((1, 1), np.int32)
    d, nm, t = oracle.raycast_run(off, pos, nrm, rad, [mesh], ls, oid, obj)
    return d[0, 0, 0], nm[0, :, 0, 0], t[0, 0, 0]


def box_mesh(b=(0.05, 0.05, 0.01)):
    return synth.shape_mesh({"family": "box", "extent": 0.1, "b": np.asarray(b, float)})


@pytest.mark.parametrize("h", [0.0, 2e-4, 7e-4, 0.99e-3, 1.5e-3])
def test_box_face_outside(h):
    R = 1e-3
    d, n, t = one_probe((0.01, -0.02, 0.01 + h), (0, 0, -1), R, box_mesh())
    assert d == pytest.approx(max(0.0, R - h), abs=2e-9)     # (the pose is FP32)
    if R - h > 0:
        np.testing.assert_allclose(n, [0, 0, 1], atol=1e-12)


@pytest.mark.parametrize("hin", [1e-4, 5e-4, 3e-3])
def test_box_face_inside_is_r_minus_sdf(hin):
    R = 1e-3
    b = (0.05, 0.05, 0.01)
    x = np.array([0.01, -0.02, 0.01 - hin])
    d, n, t = one_probe(x, (0, 0, -1), R, box_mesh(b))
    phi = synth.shape_sdf({"family": "box", "b": np.asarray(b)}, x)
    assert d == pytest.approx(R - phi, abs=1e-9)
    np.testing.assert_allclose(n, [0, 0, 1], atol=1e-12)


def test_tilted_axis():
    R, hin, th = 1e-3, 5e-4, 0.4
    a = (np.sin(th), 0.0, -np.cos(th))
    d, n, t = one_probe((0.0, 0.0, 0.01 - hin), a, R, box_mesh())
    assert d == pytest.approx(R + hin / np.cos(th), rel=1e-6)
    d2, _, _ = one_probe((0.0, 0.0, 0.01 + 3e-4), a, R, box_mesh())
    assert d2 == pytest.approx(R - 3e-4, abs=2e-9)


def test_tessellated_sphere_against_the_analytic_sphere():
    r = 0.02
    v, tr = synth.shape_mesh({"family": "sphere", "extent": 2 * r, "r": r}, detail=4)
    vv = v.astype(float)
    cen = (vv[tr[:, 0]] + vv[tr[:, 1]] + vv[tr[:, 2]]) / 3
    nrm = np.cross(vv[tr[:, 1]] - vv[tr[:, 0]], vv[tr[:, 2]] - vv[tr[:, 0]])
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    sag = r - np.min(np.sum(cen * nrm, axis=1))           # deepest face plane below the sphere
    rng = np.random.default_rng(1)
    R = 1e-3
    for _ in range(40):
        u = rng.normal(size=3); u /= np.linalg.norm(u)
        for rad in (r + 6e-4, r - 4e-4, r - 2e-3):
            d, n, t = one_probe(u * rad, -u, R, (v, tr))
            want = R - (rad - r)
            assert abs(d - want) <= sag * 1.001 + 1e-9, (rad, d, want, sag)
            assert np.dot(n, u) > 0.99


def test_filler_and_far_probes_read_zero():
    d, n, t = one_probe((0, 0, 0.0), (0, 0, -1), 0.0, box_mesh())
    assert d == 0 and t == -1 and np.all(n == 0)
    d, n, t = one_probe((0, 0, 0.0115), (0, 0, -1), 1e-3, box_mesh())
    assert d == 0 and t == -1


def test_rigid_motion_invariance():
    rng = np.random.default_rng(5)
    mesh = synth.shape_mesh({"family": "torus", "extent": 0.04, "R": 0.015, "r": 0.005})
    x = np.array([0.0148, 0.0013, 0.0042])               # off the mesh's symmetry lines
    base = one_probe(x, (0, 0, -1), 1e-3, mesh)
    q = rng.normal(size=4); q /= np.linalg.norm(q)
    t = np.array([0.1, 0.2, -0.3])
    Rq = oracle_R(q)
    obj = np.zeros((1, 13, 1), np.float32)
    obj[0, 0:3, 0] = t
    obj[0, 3:7, 0] = q
    moved = one_probe(Rq @ x + t, (0, 0, -1), 1e-3, mesh, q=q, p=(0, 0, 0), obj=obj)
    # the taxel's axis is along the link's z; with the link rotated by q, the world axis is R_q (0,0,-1)
    assert moved[0] == pytest.approx(base[0], abs=2e-8)
    np.testing.assert_allclose(moved[1], base[1], atol=1e-6)


def oracle_R(q):
    w, x, y, z = q
    return np.array([[1-2*(y*y+z*z), 2*(x*y-w*z), 2*(x*z+w*y)], [2*(x*y+w*z), 1-2*(x*x+z*z), 2*(y*z-w*x)],
                     [2*(x*z-w*y), 2*(y*z+w*x), 1-2*(x*x+y*y)]])


def test_a_ray_entering_the_object_is_no_penetration():
    """Outside, facing away: the ray along -a enters the box after 3 mm; that is not a contact."""
    d, n, t = one_probe((0.0, 0.0, 0.013), (0, 0, 1), 1e-3, box_mesh())
    assert d == 0 and t == -1


def test_the_first_exit_counts_on_a_non_convex_object():
    """Inside a torus tube with the ray across the hole: it leaves the tube after about r, then
    crosses the other side of the ring 20-30 mm on; the first exit sets the depth."""
    mesh = synth.shape_mesh({"family": "torus", "extent": 0.04, "R": 0.015, "r": 0.005}, detail=4)
    x = np.array([0.0149, 0.0011, 0.0003])
    d, n, t = one_probe(x, (1, 0, 0), 1e-3, mesh)
    rho = np.hypot(x[0] - 0.0, 0.0)                       # the ray runs along -x at y, z fixed
    # exit: the smallest t with (sqrt((x0 - t)^2 + y^2) - R)^2 + z^2 = r^2
    ts = np.linspace(0, 0.01, 200001)
    g = (np.sqrt((x[0] - ts) ** 2 + x[1] ** 2) - 0.015) ** 2 + x[2] ** 2 - 0.005 ** 2
    t_exit = ts[np.argmax(g > 0)]
    assert d == pytest.approx(1e-3 + t_exit, abs=2e-4)    # within the tessellation
    assert n[0] < -0.9                                     # the inner wall faces the hole
