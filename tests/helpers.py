"""Small hand-built scenes for closed-form pins (input construction only)."""
from __future__ import annotations

import numpy as np

from paper_2606_22332_amd import synth


def layout_from(points, links=None, radius=1e-3, normals=None):
    pts = np.asarray(points, dtype=np.float64).reshape(-1, 3)
    T = pts.shape[0]
    if links is None:
        links = [T]
    off = np.zeros(len(links) + 1, dtype=np.int32)
    off[1:] = np.cumsum(links)
    nrm = np.zeros((T, 3)); nrm[:, 2] = 1
    if normals is not None:
        nrm = np.asarray(normals, dtype=np.float64).reshape(-1, 3)
    rad = np.full(T, radius) if np.isscalar(radius) else np.asarray(radius)
    return synth.Layout(off, pts.astype(np.float32), nrm.astype(np.float32), rad.astype(np.float32))


def grid_from(fn, n=32, side=0.1, center=(0.0, 0.0, 0.0)):
    o = np.asarray(center) - side / 2
    h = side / (n - 1)
    ax = np.arange(n) * h
    Z, Y, X = np.meshgrid(o[2] + ax, o[1] + ax, o[0] + ax, indexing="ij")
    vals = fn(np.stack([X, Y, Z], axis=-1)).astype(np.float32)
    return synth.Grid(n, o.astype(np.float32), np.float32(h), np.ascontiguousarray(vals), "custom", {})


def plane_grid(normal=(0, 0, 1), offset=0.0, n=32, side=0.1):
    nn = np.asarray(normal, dtype=np.float64)
    nn = nn / np.linalg.norm(nn)
    return grid_from(lambda P: P @ nn - offset, n, side)


def sphere_grid(r=0.03, n=32, side=0.1):
    return grid_from(lambda P: np.linalg.norm(P, axis=-1) - r, n, side)


def scene(layout, grids, num_envs=1, force=None, noise=None, name="custom"):
    return synth.Scene(name, num_envs, 1, layout, grids, force or synth.ForceParams(),
                       noise or synth.NoiseParams(), 0.005)


def quat_axis_angle(axis, ang):
    a = np.asarray(axis, dtype=np.float64)
    a = a / np.linalg.norm(a)
    return np.concatenate([[np.cos(ang / 2)], np.sin(ang / 2) * a])


def rot_of_quat(q):
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def inputs(poses, obj_ids=None, obj_state=None, step0=0):
    """poses: array [S, E*L, 13] (p, q(wxyz), v, w) -> synth.Inputs."""
    P = np.asarray(poses, dtype=np.float64)
    while P.ndim < 3:
        P = P[None]
    S, EL, _ = P.shape
    ls = np.ascontiguousarray(np.transpose(P, (0, 2, 1))).astype(np.float32)
    if obj_ids is None:
        obj_ids = np.zeros((S, 1), dtype=np.int32)
    oid = np.asarray(obj_ids, dtype=np.int32)
    if oid.ndim == 1:
        oid = np.repeat(oid[None], S, axis=0)
    ost = None
    if obj_state is not None:
        O = np.asarray(obj_state, dtype=np.float64)
        if O.ndim == 2:
            O = O[None]
        ost = np.ascontiguousarray(np.transpose(O, (0, 2, 1))).astype(np.float32)
    return synth.Inputs(ls, oid, ost, step0)


def pose(p=(0, 0, 0), q=(1, 0, 0, 0), v=(0, 0, 0), w=(0, 0, 0)):
    return np.concatenate([p, q, v, w]).astype(np.float64)
