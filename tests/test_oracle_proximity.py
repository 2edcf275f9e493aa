"""Pins of the ProximityTaxel oracle (App. A.6) against closed forms and invariants.

Each case is small enough to work out by hand: a single point on or off the taxel axis, a plane of
points (whose penetration sum has a closed form), sliding and spinning objects and links, and the
invariances the definition implies (rigid motion of the whole scene, the density normalisation).
A swapped cross product, a dropped normal projection, a wrong lever arm or velocity origin, or a
density scale without the point count each fail at least one of them.
"""
import numpy as np
import pytest

import oracle

K, KS, DENS = 300.0, 10.0, 100.0


def quat_of(axis, angle):
    axis = np.asarray(axis, np.float64)
    axis = axis / np.linalg.norm(axis)
    return np.concatenate([[np.cos(angle / 2)], np.sin(angle / 2) * axis])


def R_of(q):
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def state13(p=(0, 0, 0), q=(1, 0, 0, 0), v=(0, 0, 0), w=(0, 0, 0)):
    return np.concatenate([p, q, v, w]).astype(np.float64)


def run(taxels, clouds, link, obj=None, radius=0.01, oid=0, **kw):
    """One env, one link; taxels: list of (x_j, n_j); link/obj: 13-vectors."""
    pos = np.array([t[0] for t in taxels], np.float32)
    nrm = np.array([t[1] for t in taxels], np.float32)
    T = len(taxels)
    ls = np.asarray(link, np.float32).reshape(1, 13, 1)
    ost = None if obj is None else np.asarray(obj, np.float32).reshape(1, 13, 1)
    ft, mass = oracle.prox_run([0, T], pos, nrm, np.full(T, radius, np.float32), clouds, ls,
                               np.array([[oid]], np.int32), ost, **kw)
    return ft[0, :, 0, :].T, mass[0, 0]          # [T][6], [T]


def plane(h, spacing, half_width, z_axis=2):
    """Points on a square grid in the plane z = -h (object frame)."""
    g = np.arange(-half_width, half_width + spacing / 2, spacing)
    X, Y = np.meshgrid(g, g, indexing="ij")
    pts = np.stack([X.ravel(), Y.ravel(), np.full(X.size, -h)], axis=1)
    return pts.astype(np.float32)


def test_single_point_on_the_axis():
    d = 4e-3
    cloud = [np.array([[0, 0, d]], np.float32)]                # point 4 mm in front of the taxel
    ft, m = run([((0, 0, 0), (0, 0, 1))], cloud, state13())
    rho = DENS / 1.0
    np.testing.assert_allclose(ft[0, :3], [0, 0, K * rho * (0.01 - d)], rtol=1e-6, atol=1e-12)
    np.testing.assert_allclose(ft[0, 3:], 0, atol=1e-12)       # (p - q) parallel to a: no torque
    assert m[0] == pytest.approx(0.01 - d, rel=1e-6)


def test_single_point_off_the_axis_gives_r_cross_a():
    p = np.array([3e-3, -2e-3, 5e-3], np.float32)
    cloud = [p[None]]
    ft, m = run([((0, 0, 0), (0, 0, 1))], cloud, state13())
    P = 0.01 - np.linalg.norm(p.astype(np.float64))
    rho = DENS
    a = np.array([0, 0, 1.0])
    np.testing.assert_allclose(ft[0, :3], K * rho * P * a, rtol=1e-6)
    np.testing.assert_allclose(ft[0, 3:], K * rho * P * np.cross(p.astype(np.float64), a), rtol=1e-6)
    # tau = (p - q) x a, not a x (p - q): the x component is -2e-3 * 1 for (p - q) = (3, -2, 5) mm
    assert ft[0, 3] < 0 and ft[0, 4] < 0
    # the lever arm is taken from the probe centre q_j, not from the link origin: a taxel away from
    # the origin of a translated link sees the same point through q_j = p_L + x_j
    xj, pL = np.array([2e-3, 1e-3, 0.0], np.float32), np.array([-1e-3, 4e-3, 2e-3], np.float32)
    ft2, _ = run([(tuple(xj), (0, 0, 1))], [(p + pL + xj)[None]], state13(p=pL))
    np.testing.assert_allclose(ft2[0, 3:], ft[0, 3:], rtol=1e-5)


def test_points_outside_the_sphere_do_not_count():
    cloud = [np.array([[0, 0, 0.0101], [0.011, 0, 0], [0, 0, -0.02]], np.float32)]
    ft, m = run([((0, 0, 0), (0, 0, 1))], cloud, state13())
    assert np.all(ft == 0) and m[0] == 0


@pytest.mark.parametrize("h", [0.0, 3e-3, 7e-3])
def test_plane_penetration_sum_matches_the_cap_integral(h):
    """A plane of areal density s at distance h from the centre: sum_i P_ij tends to
    s * integral over the disc of radius sqrt(R^2 - h^2) of (R - sqrt(h^2 + r^2)) = s pi (R - h)^2 (R + 2h) / 3."""
    R, dx = 0.01, 1e-4
    cloud = [plane(h, dx, 0.012)]
    ft, m = run([((0, 0, 0), (0, 0, -1))], cloud, state13(), radius=R)
    s = 1.0 / dx ** 2
    want = s * np.pi * (R - h) ** 2 * (R + 2 * h) / 3.0
    assert m[0] == pytest.approx(want, rel=2e-3)
    rho = DENS / cloud[0].shape[0]
    np.testing.assert_allclose(ft[0, :3], [0, 0, -K * rho * m[0]], rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(ft[0, 3:], 0, atol=1e-9 * K * rho * m[0] * R)   # symmetric: no torque


def test_density_scale_divides_by_the_point_count():
    """Every point listed twice: the sums double and rho_b halves, so nothing changes."""
    cloud = plane(2e-3, 5e-4, 0.012)
    link = state13(p=(1e-3, 0, 0), q=quat_of((1, 2, 3), 0.2), v=(0.01, 0, 0), w=(0, 0.5, 0))
    a, _ = run([((0, 0, 0), (0, 0, -1)), ((2e-3, 1e-3, 0), (0, 0, -1))], [cloud], link)
    b, _ = run([((0, 0, 0), (0, 0, -1)), ((2e-3, 1e-3, 0), (0, 0, -1))], [np.concatenate([cloud, cloud])], link)
    np.testing.assert_allclose(a, b, rtol=1e-10, atol=1e-15)


def test_sliding_object_gives_the_tangential_slip_only():
    """The object slides under a static taxel with velocity v: the slip term is k_s rho sum P
    times the part of v normal to the taxel axis; a purely normal velocity adds nothing."""
    cloud = [plane(2e-3, 5e-4, 0.012)]
    rho = DENS / cloud[0].shape[0]
    base, m = run([((0, 0, 0), (0, 0, -1))], cloud, state13())
    v = np.array([0.02, -0.01, 0.03])
    ft, _ = run([((0, 0, 0), (0, 0, -1))], cloud, state13(), obj=state13(v=v))
    v32 = v.astype(np.float32).astype(np.float64)               # the inputs are FP32
    np.testing.assert_allclose(ft[0, :3] - base[0, :3], KS * rho * m[0] * np.array([v32[0], v32[1], 0.0]), rtol=1e-9)
    np.testing.assert_allclose(ft[0, 3:], base[0, 3:], atol=1e-12)
    # the link moving with -v instead: the same relative velocity, the same reading
    ft2, _ = run([((0, 0, 0), (0, 0, -1))], cloud, state13(v=-v))
    np.testing.assert_allclose(ft2, ft, rtol=1e-9, atol=1e-12)
    normal_only, _ = run([((0, 0, 0), (0, 0, -1))], cloud, state13(), obj=state13(v=(0, 0, 0.05)))
    np.testing.assert_allclose(normal_only, base, rtol=1e-12, atol=1e-12)


def test_spinning_link_moves_an_off_centre_taxel():
    """Link spinning about z at w through its origin; taxel at x = (r, 0, 0) facing -z: the taxel
    moves with w x x = (0, w r, 0), so the slip force is -k_s rho sum P (0, w r, 0)."""
    r, w = 4e-3, 3.0
    cloud = [plane(2e-3, 5e-4, 0.02)]
    rho = DENS / cloud[0].shape[0]
    base, m = run([((r, 0, 0), (0, 0, -1))], cloud, state13())
    ft, _ = run([((r, 0, 0), (0, 0, -1))], cloud, state13(w=(0, 0, w)))
    r32 = float(np.float32(r))
    np.testing.assert_allclose(ft[0, :3] - base[0, :3], [0, -KS * rho * m[0] * w * r32, 0], rtol=1e-9, atol=1e-12)


def test_spinning_object_uses_each_points_velocity_about_the_object_origin():
    """The object (origin at c, away from the taxel) spins about z: each point moves with
    w x (p_i - c).  Summed over the symmetric cap under the taxel the tangential part is
    w x (q - c) times sum P (the in-plane offsets cancel), against the hand value."""
    w = 2.0
    c = np.array([0.01, 0.005, 0.0])
    cloud_world = plane(2e-3, 5e-4, 0.02).astype(np.float64)
    cloud_obj = (cloud_world - c).astype(np.float32)           # object frame: origin at c
    rho = DENS / cloud_obj.shape[0]
    base, m = run([((0, 0, 0), (0, 0, -1))], [cloud_obj], state13(), obj=state13(p=c))
    ft, _ = run([((0, 0, 0), (0, 0, -1))], [cloud_obj], state13(), obj=state13(p=c, w=(0, 0, w)))
    vt = np.cross([0, 0, w], -c.astype(np.float32).astype(np.float64))   # w x (q - c), q = 0; in-plane already
    np.testing.assert_allclose(ft[0, :3] - base[0, :3], KS * rho * m[0] * vt, rtol=1e-6, atol=1e-12)


def test_rigid_motion_of_the_whole_scene_leaves_link_frame_readings_unchanged():
    rng = np.random.default_rng(3)
    cloud = rng.normal(0, 6e-3, (400, 3)).astype(np.float32)
    taxels = [((0, 0, 0), (0, 0, 1)), ((3e-3, -2e-3, 0), (0, 0, 1)), ((-4e-3, 1e-3, 0), (0.6, 0, 0.8))]
    link = state13(p=(0.002, -0.001, 0.004), q=quat_of((0.3, -1, 0.2), 0.7), v=(0.03, -0.02, 0.01), w=(1.0, -2.0, 0.5))
    obj = state13(p=(0.001, 0.002, -0.003), q=quat_of((1, 1, 0), 0.4), v=(-0.01, 0.02, 0.0), w=(0.2, 0.1, -0.7))
    a, _ = run(taxels, [cloud], link, obj=obj)
    # move everything by a rigid transform G = (Rg, tg): poses, velocities and spins transform alike
    Rg, tg = R_of(quat_of((2, -1, 3), 1.1)), np.array([0.05, -0.02, 0.1])

    def moved(s):
        p, q, v, w = s[:3], s[3:7], s[7:10], s[10:]
        qg = quat_of((2, -1, 3), 1.1)
        w0, x0, y0, z0 = qg
        w1, x1, y1, z1 = q
        qn = np.array([w0 * w1 - x0 * x1 - y0 * y1 - z0 * z1, w0 * x1 + x0 * w1 + y0 * z1 - z0 * y1,
                       w0 * y1 - x0 * z1 + y0 * w1 + z0 * x1, w0 * z1 + x0 * y1 - y0 * x1 + z0 * w1])
        return np.concatenate([Rg @ p + tg, qn, Rg @ v, Rg @ w])

    b, _ = run(taxels, [cloud], moved(link), obj=moved(obj))
    np.testing.assert_allclose(b, a, rtol=1e-4, atol=1e-6 * np.abs(a).max())


def test_no_object_and_radius_noise():
    cloud = [plane(2e-3, 5e-4, 0.012)]
    taxel = [((0, 0, 0), (0, 0, -1))]
    ft, m = run(taxel, cloud, state13(), oid=-1)
    assert np.all(ft == 0) and np.all(m == 0)
    base, m0 = run(taxel, cloud, state13(), seed=7, radius_rho=0.0)
    same, _ = run(taxel, cloud, state13(), seed=7, radius_rho=0.0)
    assert np.array_equal(base, same)
    # radius noise of at most rho: the penetration sum lies between those of R - rho and R + rho
    lo, mlo = run(taxel, cloud, state13(), radius=0.009)
    hi, mhi = run(taxel, cloud, state13(), radius=0.011)
    noisy = [run(taxel, cloud, state13(), seed=s, radius_rho=1e-3)[1][0] for s in range(8)]
    assert all(mlo[0] <= v <= mhi[0] for v in noisy) and len(set(noisy)) > 1


def test_gain_scales_every_channel():
    cloud = [plane(2e-3, 5e-4, 0.012)]
    taxel = [((1e-3, 0, 0), (0, 0, -1))]
    link = state13(v=(0.01, 0.02, 0), w=(0, 0, 1.0))
    a, _ = run(taxel, cloud, link)
    b, _ = run(taxel, cloud, link, gain=np.array([[1.25]], np.float32))
    np.testing.assert_allclose(b, 1.25 * a, rtol=1e-12)
