"""Pins of the ElastomerTaxel oracle (App. A.7): dilation and anchored shear.

Dilation (one source probe of penetration h, markers on a line through it):
- peak normalisation: with c = 1 the in-plane displacement peaks at s_d h where |r| = 1/sqrt(2 lambda_d);
  with c = 0 it peaks at s_d h where |r| = eps, and it decays as 1/|r| far out;
- the in-plane part is linear in h and the normal part goes as h^alpha;
- only the tangential offset counts: a source lifted along the marker normal moves nothing;
- two sources symmetric about a marker cancel in-plane and add along the normal; superposition.
Shear (one tracked point):
- the anchor state machine: no anchor at a depth of half eta_enter, an anchor beyond eta_enter;
  the anchor holds until the pad SDF rises above eta_exit; at first contact the shear is zero;
- a slide by delta in the pad plane gives a shear along delta, linear in delta and in the depth,
  Gaussian in the marker's distance (ratio of two markers = exp(-lambda_s (d1^2 - d2^2)));
- a change of the env's object clears the anchors;
- rotating and moving the link and the object together changes nothing (the sensor frame).
"""
import numpy as np
import pytest

import oracle

P = oracle.ELASTOMER_DEFAULTS


def line_layout(n=41, pitch=5e-4, radius=0.0):
    x = (np.arange(n) - n // 2) * pitch
    pos = np.stack([x, np.zeros(n), np.zeros(n)], 1).astype(np.float32)
    nrm = np.tile(np.array([0, 0, 1], np.float32), (n, 1))
    return np.array([0, n], np.int32), pos, nrm, np.full(n, radius, np.float32)


def ident_state(S, E=1, L=1, p=(0, 0, 0), q=(1, 0, 0, 0)):
    ls = np.zeros((S, 13, E * L), np.float32)
    ls[:, 0:3] = np.asarray(p, np.float32)[None, :, None]
    ls[:, 3:7] = np.asarray(q, np.float32)[None, :, None]
    return ls


PAD_C = np.array([[0, 0, -1e-3]], np.float32)
PAD_H = np.array([[0.05, 0.05, 1e-3]], np.float32)


def dilation(h_of, n=41, pitch=5e-4, **prm):
    off, pos, nrm, rad = line_layout(n, pitch)
    depth = np.zeros((1, 1, n), np.float32)
    for i, h in h_of.items():
        depth[0, 0, i] = h
    oid = np.full((1, 1), -1, np.int32)
    d, a, _ = oracle.elastomer_run(off, pos, nrm, rad, [0], PAD_C, PAD_H, [], ident_state(1), oid, None, depth, **prm)
    return d[0, :, 0, :].T, pos                           # [n][3]


@pytest.mark.parametrize("c", [1.0, 0.0])
def test_peak_normalisation(c):
    n, pitch = 401, 5e-5                                  # 0.05 mm steps out to 10 mm
    h = 1e-3
    y, pos = dilation({n // 2: h}, n, pitch, c=c)
    inplane = np.abs(y[:, 0])
    r = np.abs(pos[:, 0])
    k = np.argmax(inplane)
    assert inplane[k] == pytest.approx(P["s_d"] * h, rel=2e-3)
    r_peak = 1 / np.sqrt(2 * P["lambda_d"]) if c == 1.0 else P["eps"]
    assert abs(r[k] - r_peak) <= pitch


def test_inverse_distance_far_field():
    n, pitch = 801, 1e-3
    y, pos = dilation({n // 2: 1e-3}, n, pitch, c=0.0)
    r = np.abs(pos[:, 0])
    i1 = np.argmin(np.abs(r - 0.1)); i2 = np.argmin(np.abs(r - 0.2))        # 50 eps and 100 eps
    assert abs(y[i1, 0] / y[i2, 0]) == pytest.approx(2.0, rel=2e-3)


def test_depth_laws():
    y1, _ = dilation({20: 1e-3})
    y2, _ = dilation({20: 2e-3})
    np.testing.assert_allclose(y2[:, 0], 2.0 * y1[:, 0], rtol=1e-12, atol=0)
    np.testing.assert_allclose(y2[:, 2], 2.0 ** P["alpha"] * y1[:, 2], rtol=1e-12, atol=0)
    assert np.all(y1[:, 1] == 0)


def test_only_the_tangential_offset_counts():
    off, pos, nrm, rad = line_layout()
    depth = np.zeros((1, 1, 41), np.float32)
    depth[0, 0, 20] = 1e-3
    args = ([0], PAD_C, PAD_H, [], ident_state(1), np.full((1, 1), -1, np.int32), None, depth)
    d0, _, _ = oracle.elastomer_run(off, pos, nrm, rad, *args)
    pos2 = pos.copy()
    pos2[20, 2] = 3e-3                                    # the source lifted along the normal
    d1, _, _ = oracle.elastomer_run(off, pos2, nrm, rad, *args)
    mask = np.arange(41) != 20
    np.testing.assert_allclose(d1[0, :, 0, mask], d0[0, :, 0, mask], rtol=1e-12, atol=1e-18)


def test_symmetric_sources_and_superposition():
    yb, _ = dilation({16: 1e-3, 24: 1e-3})
    assert abs(yb[20, 0]) < 1e-12 * np.abs(yb[:, 0]).max()
    ya, _ = dilation({16: 1e-3})
    yc, _ = dilation({24: 1e-3})
    np.testing.assert_allclose(yb, ya + yc, rtol=1e-12, atol=1e-18)
    assert yb[20, 2] == pytest.approx(2 * ya[20, 2], rel=1e-12)


def test_probe_radius_is_subtracted():
    off, pos, nrm, _ = line_layout()
    rad = np.full(41, 1e-3, np.float32)
    depth = np.zeros((1, 1, 41), np.float32)
    depth[0, 0, 20] = 2e-3                                 # d = R + h with h = 1 mm
    args = ([0], PAD_C, PAD_H, [], ident_state(1), np.full((1, 1), -1, np.int32), None, depth)
    d1, _, _ = oracle.elastomer_run(off, pos, nrm, rad, *args)
    y0, _ = dilation({20: 1e-3})
    np.testing.assert_allclose(d1[0, :, 0, :].T, y0, rtol=1e-6)
    depth[0, 0, 20] = 1e-3                                  # d = R: no penetration
    d2, _, _ = oracle.elastomer_run(off, pos, nrm, rad, *args)
    assert np.all(d2 == 0)


def shear_run(zs, obj_ids=None, **kw):
    """One tracked point at object-frame origin, moved to the link-frame positions zs[s] by the
    object's translation (identity link pose)."""
    off, pos, nrm, rad = line_layout()
    S = len(zs)
    ost = np.zeros((S, 13, 1), np.float32)
    ost[:, 0:3, 0] = np.asarray(zs, np.float32)
    ost[:, 3, 0] = 1.0
    oid = np.zeros((S, 1), np.int32) if obj_ids is None else np.asarray(obj_ids, np.int32).reshape(S, 1)
    clouds = [np.zeros((1, 3), np.float32), np.zeros((1, 3), np.float32)]
    depth = np.zeros((S, 1, 41), np.float32)
    d, a, st = oracle.elastomer_run(off, pos, nrm, rad, [0], PAD_C, PAD_H, clouds, ident_state(S), oid, ost, depth, **kw)
    return d[:, :, 0, :].transpose(0, 2, 1), pos, st       # [S][n][3]


def test_anchor_state_machine():
    e_in, e_out = P["eta_enter"], P["eta_exit"]
    # half of eta_enter deep: never anchored, however far it slides
    y, _, st = shear_run([(0, 0, -0.5 * e_in), (2e-3, 0, -0.5 * e_in)])
    assert np.all(y == 0) and st["active"].sum() == 0
    # between eta_enter and eta_exit deep: anchored (the entry threshold is eta_enter)
    y, _, st = shear_run([(0, 0, -0.5 * e_out), (1e-3, 0, -0.5 * e_out)])
    assert st["active"].sum() == 1 and np.abs(y[1]).max() > 0
    # beyond eta_enter: anchored at first contact with zero shear, then a slide shears
    zs = [(0, 0, -2e-4), (1e-3, 0, -2e-4), (1e-3, 0, 0.5 * e_out), (2e-3, 0, 0.5 * e_out), (2e-3, 0, -2e-4),
          (2e-3, 0, 2 * e_out), (3e-3, 0, -2e-4)]
    y, pos, st = shear_run(zs)
    assert np.all(y[0] == 0)
    assert np.abs(y[1]).max() > 0
    assert np.all(y[2] == 0) and np.all(y[3] == 0)        # above the pad: no penetration, anchor kept
    # back in at x = 2 mm: still anchored at x = 0, so the shear is that of a 2 mm slide
    j = 20
    h = 2e-4
    expect = P["s_s"] * 2e-3 * h * np.exp(-P["lambda_s"] * (pos[j, 0] - 2e-3) ** 2)
    assert y[4, j, 0] == pytest.approx(expect, rel=1e-6)
    assert np.all(y[5] == 0)                              # out beyond eta_exit: anchor cleared
    assert np.all(y[6] == 0)                              # re-anchored at x = 3 mm: zero shear


def test_slide_laws():
    y1, pos, _ = shear_run([(0, 0, -2e-4), (1e-3, 0, -2e-4)])
    y2, _, _ = shear_run([(0, 0, -2e-4), (2e-3, 0, -2e-4)])
    y3, _, _ = shear_run([(0, 0, -4e-4), (1e-3, 0, -4e-4)])
    s1 = y1[1]
    assert np.all(s1[:, 1] == 0) and np.all(s1[:, 2] == 0) and np.all(s1[:, 0] > 0)
    np.testing.assert_allclose(y3[1], 2 * s1, rtol=1e-6)                   # linear in the depth
    # Gaussian in the marker's distance from the point (x = 1 mm) and linear in the slide
    d1, d2 = pos[20, 0] - 1e-3, pos[30, 0] - 1e-3
    assert s1[20, 0] / s1[30, 0] == pytest.approx(np.exp(-P["lambda_s"] * (d1 ** 2 - d2 ** 2)), rel=1e-6)
    d1b, d2b = pos[20, 0] - 2e-3, pos[30, 0] - 2e-3
    r = y2[1][20, 0] / s1[20, 0]
    assert r == pytest.approx(2.0 * np.exp(-P["lambda_s"] * (d1b ** 2 - d1 ** 2)), rel=1e-6)


def test_object_change_clears_anchors():
    zs = [(0, 0, -2e-4), (1e-3, 0, -2e-4), (1e-3, 0, -2e-4)]
    y, _, _ = shear_run(zs, obj_ids=[0, 0, 1])
    assert np.abs(y[1]).max() > 0 and np.all(y[2] == 0)


def test_sensor_frame_invariance():
    rng = np.random.default_rng(3)
    off, pos, nrm, rad = line_layout()
    S = 3
    cloud = [rng.uniform(-2e-3, 2e-3, (30, 3)).astype(np.float32)]
    ost = np.zeros((S, 13, 1), np.float32)
    ost[:, 3, 0] = 1.0
    ost[:, 0, 0] = [0.0, 1e-3, 1.5e-3]
    ost[:, 2, 0] = -1e-3
    depth = rng.uniform(0, 1e-3, (S, 1, 41)).astype(np.float32)
    oid = np.zeros((S, 1), np.int32)
    d0, _, st0 = oracle.elastomer_run(off, pos, nrm, rad, [0], PAD_C, PAD_H, cloud, ident_state(S), oid, ost, depth)
    assert st0["active"].sum() > 0 and np.abs(d0).max() > 0
    # the same scene under a rigid motion (rotation by quaternion qg, translation tg) of link and object
    qg = np.array([0.9, 0.1, -0.3, 0.2]); qg /= np.linalg.norm(qg)
    tg = np.array([0.1, -0.2, 0.05])
    def R(q):
        w, x, y, z = q
        return np.array([[1-2*(y*y+z*z), 2*(x*y-w*z), 2*(x*z+w*y)], [2*(x*y+w*z), 1-2*(x*x+z*z), 2*(y*z-w*x)],
                         [2*(x*z-w*y), 2*(y*z+w*x), 1-2*(x*x+y*y)]])
    def qmul(a, b):
        w1, x1, y1, z1 = a; w2, x2, y2, z2 = b
        return np.array([w1*w2-x1*x2-y1*y2-z1*z2, w1*x2+x1*w2+y1*z2-z1*y2, w1*y2-x1*z2+y1*w2+z1*x2, w1*z2+x1*y2-y1*x2+z1*w2])
    ls = ident_state(S, p=tg, q=qg)
    ost2 = ost.copy()
    for s in range(S):
        ost2[s, 0:3, 0] = R(qg) @ ost[s, 0:3, 0].astype(np.float64) + tg
        ost2[s, 3:7, 0] = qmul(qg, ost[s, 3:7, 0].astype(np.float64))
    d1, _, st1 = oracle.elastomer_run(off, pos, nrm, rad, [0], PAD_C, PAD_H, cloud, ls, oid, ost2, depth)
    np.testing.assert_array_equal(st1["active"], st0["active"])
    np.testing.assert_allclose(d1, d0, rtol=0, atol=2e-4 * np.abs(d0).max())
