"""Seeded synthetic scenes shaped like the paper's tactile workloads.

This module is input generation only.  It builds taxel layouts, object SDF
grids and link trajectories in FP64 with numpy, rounds them once to FP32, and
hands them to whoever asks (the HIP path and the CPU oracle alike).  It does
none of the readout arithmetic: no pose transform of taxels, no grid lookup,
no force law, no noise.

Shapes follow the paper: probes on planar patches rigidly attached to links
(App. A.1), hand layouts sized like the probe-count table (App. B, "Tactile
Placement and Probe Counts"), and objects like the cube/cylinder sets used in
training (App. B, tasks).  The paper's assets are not available, so primitive
and convex-hull objects stand in for them.

Configurations (sizes, seeds):
  c1  64 envs x 5 links x 20 taxels, one 3 cm sphere on a 32^3 grid, random
      poses within 4 cm of the centre, 10 steps, noise off.
  c2  4096 envs x 16 links (uneven 8..40 taxels, 200 total), 8 objects on 64^3
      grids, sinusoidal trajectories, 100 steps, drift + lag + dead + banded
      crosstalk.
  c3  20480 envs x 16 links (16..128 taxels, 1024 total), 32 objects, 64
      steps, dense crosstalk.
  c4  the c3 hand with 256 objects, 16 steps, noise off (neural-SDF workload).
  c5  the c2 hand at dt = 1 ms for 500 steps (thermal workload).
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass, field, replace
from typing import List, Optional

import numpy as np

MASTER_SEED = 260622332
PITCH = 2.0e-3          # taxel pitch on every patch [m]
TAXEL_RADIUS = 1.0e-3   # probe radius R_j [m]
FAMILIES = ["sphere", "box", "capsule", "torus", "hull", "box", "capsule", "hull"]

C2_LINKS = [40, 20, 16, 16, 16, 12] + [8] * 10
C3_LINKS = [128, 117, 101, 93, 85, 71, 66, 60, 54, 49, 43, 37, 32, 29, 25, 34]


# ----------------------------------------------------------------------------------------------
# data containers
# ----------------------------------------------------------------------------------------------
@dataclass
class Layout:
    """Taxels of one robot, shared by every env; taxels are sorted by link."""
    link_offset: np.ndarray   # int32 [L+1]
    pos: np.ndarray           # float32 [T,3] link-frame centre x_j
    normal: np.ndarray        # float32 [T,3] link-frame unit normal n_j
    radius: np.ndarray        # float32 [T]   R_j (0 = inactive filler)

    @property
    def num_links(self) -> int:
        return int(self.link_offset.shape[0] - 1)

    @property
    def num_taxels(self) -> int:
        return int(self.pos.shape[0])

    def link_of_taxel(self) -> np.ndarray:
        return np.repeat(np.arange(self.num_links, dtype=np.int32), np.diff(self.link_offset))


@dataclass
class Grid:
    """Node-centred SDF grid in the object frame: N nodes per axis over [o, o+(N-1)h]."""
    n: int
    origin: np.ndarray        # float32 [3]
    spacing: np.float32
    values: np.ndarray        # float32 [N,N,N] indexed [z,y,x] (x fastest in memory)
    family: str = ""
    shape: dict = field(default_factory=dict)


@dataclass
class ForceParams:
    k_n: float = 2000.0
    c_n: float = 5.0
    alpha: float = 1.0
    k_t: float = 2.0
    k_w: float = 2.0
    mu: float = 0.8
    prox_range: float = 0.01
    eta_on: float = 5.0e-4
    spring_only: bool = False


@dataclass
class NoiseParams:
    enabled: bool = False
    seed: int = 0
    drift_sigma: float = 0.0
    white_sigma: float = 0.0
    bias: float = 0.0
    quant_step: float = 0.0
    hyst_mode: int = 0            # 0 off, 1 asymmetric first-order lag, 2 Maxwell element
    tau_load_steps: float = 0.0
    tau_unload_steps: float = 0.0
    maxwell_beta: float = 0.0
    maxwell_tau_s: float = 0.0
    dt_s: float = 0.005
    p_dead: float = 0.0
    stuck_lo: float = 0.0
    stuck_hi: float = 0.0
    radius_rho: float = 0.0
    gain_lo: float = 1.0
    gain_hi: float = 1.0
    xtalk_kind: int = 0           # 0 none, 1 banded, 2 dense per-link matrix
    xtalk_chi: float = 0.0
    xtalk_sigma: float = 0.0
    eta_off: float = 5.0e-4


@dataclass
class ThermalParams:
    """Voxel temperature fields on some links (one n^3 block per env and link, link frame)."""
    field_links: List[int]
    T_obj: np.ndarray                     # float32 [E] object temperature per env [degC]
    n: int = 16
    dx: float = 1e-3
    origin: tuple = (-8e-3, -8e-3, -16e-3)   # outer corner of voxel (0,0,0); top face at z = 0
    dt: float = 1e-3
    k_sensor: float = 0.2
    rho_cp: float = 2.0e6
    emissivity: float = 0.85
    k_object: float = 10.0
    d_w: float = 1.0
    T0: float = 22.0
    T_amb: float = 22.0
    P_gen: float = 0.1
    solver: int = 0                       # 0 explicit 7-point step, 1 the paper's spectral step
    h_conv: float = 0.0                   # convection coefficient [W/m^2K] (solver 1)
    lag_tau: float = 0.0                  # sensor element time constant [s] (solver 1; 0 = none)


@dataclass
class Scene:
    name: str
    num_envs: int
    num_steps: int
    layout: Layout
    grids: List[Grid]
    force: ForceParams
    noise: NoiseParams
    dt: float = 0.005
    geom_seed: int = MASTER_SEED
    thermal: Optional[ThermalParams] = None


@dataclass
class Inputs:
    """Per-step device-shaped inputs (host copies)."""
    link_state: np.ndarray            # float32 [S,13,E*L]: p(3) q=(w,x,y,z)(4) v(3) omega(3)
    obj_id: np.ndarray                # int32 [S,E]
    obj_state: Optional[np.ndarray]   # float32 [S,13,E] or None (object static at the env origin)
    step0: int = 0


# ----------------------------------------------------------------------------------------------
# layouts
# ----------------------------------------------------------------------------------------------
def patch(n: int, pitch: float = PITCH) -> np.ndarray:
    """n taxel centres on a near-square grid at `pitch` in the link z=0 plane; last row partial."""
    cols = int(math.ceil(math.sqrt(n)))
    rows = int(math.ceil(n / cols))
    pts = []
    for r in range(rows):
        for c in range(cols):
            if len(pts) == n:
                break
            pts.append(((c - (cols - 1) / 2.0) * pitch, (r - (rows - 1) / 2.0) * pitch, 0.0))
    return np.asarray(pts, dtype=np.float64)


def make_layout(counts: List[int], radius: float = TAXEL_RADIUS) -> Layout:
    pos = np.concatenate([patch(n) for n in counts], axis=0)
    T = pos.shape[0]
    normal = np.zeros((T, 3)); normal[:, 2] = 1.0
    off = np.zeros(len(counts) + 1, dtype=np.int32)
    off[1:] = np.cumsum(counts)
    return Layout(off, pos.astype(np.float32), normal.astype(np.float32),
                  np.full(T, radius, dtype=np.float32))


# ----------------------------------------------------------------------------------------------
# object shapes (FP64 analytic signed distances, used only to fill grids and place trajectories)
# ----------------------------------------------------------------------------------------------
_hull_lib = None


def _load_hull_lib():
    global _hull_lib
    if _hull_lib is None:
        path = os.path.join(os.path.dirname(__file__), "_synth_hull.so")
        if not os.path.exists(path):
            build_hull_lib()
        lib = ctypes.CDLL(path)
        lib.hull_sdf_points.restype = None
        lib.hull_sdf_points.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                        ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        _hull_lib = lib
    return _hull_lib


def build_hull_lib() -> str:
    import subprocess
    here = os.path.dirname(os.path.abspath(__file__))
    src = os.path.join(here, "synth_hull.c")
    out = os.path.join(here, "_synth_hull.so")
    subprocess.check_call(["gcc", "-O2", "-shared", "-fPIC", "-o", out, src, "-lm"])
    return out


def make_shape(family: str, extent: float, rng: np.random.Generator) -> dict:
    s = {"family": family, "extent": extent}
    if family == "sphere":
        s["r"] = extent / 2
    elif family == "box":
        a = rng.uniform(0.5, 1.0, size=2)
        s["b"] = np.array([extent / 2, extent / 2 * a[0], extent / 2 * a[1]])
    elif family == "capsule":
        r = extent * rng.uniform(1 / 6, 1 / 4)
        s["r"] = r
        s["hl"] = extent / 2 - r
    elif family == "torus":
        s["R"] = extent * 3 / 8
        s["r"] = extent / 8
    elif family == "hull":
        from scipy.spatial import ConvexHull
        d = rng.normal(size=(32, 3))
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        scale = np.array([1.0, rng.uniform(0.6, 1.0), rng.uniform(0.6, 1.0)]) * extent / 2
        v = d * scale
        h = ConvexHull(v)
        planes = h.equations.copy()          # a.x + b.y + c.z + d <= 0 inside; normals unit
        s["verts"] = v
        s["tris"] = h.simplices.astype(np.int32)
        s["planes"] = np.concatenate([planes[:, :3], -planes[:, 3:4]], axis=1)  # n.x - off
    else:
        raise ValueError(family)
    return s


def shape_sdf(s: dict, p: np.ndarray) -> np.ndarray:
    """Exact FP64 signed distance of shape `s` at points p [...,3] (object frame)."""
    p = np.asarray(p, dtype=np.float64)
    f = s["family"]
    if f == "sphere":
        return np.linalg.norm(p, axis=-1) - s["r"]
    if f == "box":
        q = np.abs(p) - s["b"]
        return np.linalg.norm(np.maximum(q, 0), axis=-1) + np.minimum(q.max(axis=-1), 0)
    if f == "capsule":
        z = np.clip(p[..., 2], -s["hl"], s["hl"])
        d = p.copy(); d[..., 2] -= z
        return np.linalg.norm(d, axis=-1) - s["r"]
    if f == "torus":
        qx = np.hypot(p[..., 0], p[..., 1]) - s["R"]
        return np.hypot(qx, p[..., 2]) - s["r"]
    if f == "hull":
        lib = _load_hull_lib()
        flat = np.ascontiguousarray(p.reshape(-1, 3))
        out = np.empty(flat.shape[0])
        v = np.ascontiguousarray(s["verts"]); t = np.ascontiguousarray(s["tris"])
        pl = np.ascontiguousarray(s["planes"])
        lib.hull_sdf_points(flat.shape[0], flat.ctypes.data, v.shape[0], v.ctypes.data, t.shape[0],
                            t.ctypes.data, pl.ctypes.data, out.ctypes.data)
        return out.reshape(p.shape[:-1])
    raise ValueError(f)


def shape_grad(s: dict, p: np.ndarray, h: float = 1e-6) -> np.ndarray:
    g = np.zeros(p.shape)
    for k in range(3):
        e = np.zeros(3); e[k] = h
        g[..., k] = (shape_sdf(s, p + e) - shape_sdf(s, p - e)) / (2 * h)
    return g


def sample_grid(s: dict, n: int, side: float) -> Grid:
    o = -side / 2
    h = side / (n - 1)
    ax = o + h * np.arange(n)
    Z, Y, X = np.meshgrid(ax, ax, ax, indexing="ij")
    P = np.stack([X, Y, Z], axis=-1)
    vals = shape_sdf(s, P).astype(np.float32)
    return Grid(n, np.full(3, o, dtype=np.float32), np.float32(h), np.ascontiguousarray(vals),
                s["family"], s)


def make_objects(n_obj: int, rng: np.random.Generator, n: int = 64, margin: float = 0.04) -> List[Grid]:
    grids = []
    for k in range(n_obj):
        fam = FAMILIES[k % len(FAMILIES)]
        extent = rng.uniform(0.02, 0.06)
        s = make_shape(fam, extent, rng)
        grids.append(sample_grid(s, n, extent + margin))
    return grids


# ----------------------------------------------------------------------------------------------
# rotations (input generation only)
# ----------------------------------------------------------------------------------------------
def quat_mul(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    w1, x1, y1, z1 = np.moveaxis(a, -1, 0)
    w2, x2, y2, z2 = np.moveaxis(b, -1, 0)
    return np.stack([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2,
                     w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                     w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2,
                     w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2], axis=-1)


def matrix_to_quat(R: np.ndarray) -> np.ndarray:
    from scipy.spatial.transform import Rotation
    xyzw = Rotation.from_matrix(R.reshape(-1, 3, 3)).as_quat()
    q = np.concatenate([xyzw[:, 3:4], xyzw[:, :3]], axis=1)
    return q.reshape(R.shape[:-2] + (4,))


def random_unit(rng: np.random.Generator, n: int) -> np.ndarray:
    d = rng.normal(size=(n, 3))
    return d / np.linalg.norm(d, axis=1, keepdims=True)


# ----------------------------------------------------------------------------------------------
# configurations
# ----------------------------------------------------------------------------------------------
def c2_noise(seed: int) -> NoiseParams:
    return NoiseParams(enabled=True, seed=seed, drift_sigma=1e-3, hyst_mode=1, tau_load_steps=2.0,
                       tau_unload_steps=6.0, p_dead=0.02, xtalk_kind=1, xtalk_chi=0.05, eta_off=2e-4)


def make_scene(cfg: str, num_envs: Optional[int] = None, num_steps: Optional[int] = None) -> Scene:
    k = int(cfg[1])
    rng = np.random.default_rng(MASTER_SEED + k)
    key = MASTER_SEED + 100 * k
    if cfg == "c1":
        layout = make_layout([20] * 5)
        s = {"family": "sphere", "extent": 0.06, "r": 0.03}
        grids = [sample_grid(s, 32, 0.10)]
        sc = Scene("c1", 64, 10, layout, grids, ForceParams(), NoiseParams(seed=key))
    elif cfg == "c2":
        layout = make_layout(C2_LINKS)
        sc = Scene("c2", 4096, 100, layout, make_objects(8, rng), ForceParams(), c2_noise(key))
    elif cfg == "c3":
        layout = make_layout(C3_LINKS)
        nz = c2_noise(key)
        nz.xtalk_kind, nz.xtalk_chi, nz.xtalk_sigma = 2, 0.1, 2e-3
        sc = Scene("c3", 20480, 64, layout, make_objects(32, rng), ForceParams(), nz)
    elif cfg == "c4":
        layout = make_layout(C3_LINKS)
        sc = Scene("c4", 20480, 16, layout, make_objects(256, rng), ForceParams(), NoiseParams(seed=key))
    elif cfg == "c5":
        layout = make_layout(C2_LINKS)
        sc = Scene("c5", 4096, 500, layout, make_objects(8, rng), ForceParams(), c2_noise(key), dt=0.001)
        sc.noise.dt_s = 0.001
    else:
        raise ValueError(cfg)
    sc.geom_seed = MASTER_SEED + k
    if num_envs is not None:
        sc.num_envs = num_envs
    if num_steps is not None:
        sc.num_steps = num_steps
    if cfg == "c5":        # fingertips are links 1..5 of the hand; object temperature U(10, 60) degC
        trng = np.random.default_rng(MASTER_SEED + 50)
        sc.thermal = ThermalParams([1, 2, 3, 4, 5], trng.uniform(10.0, 60.0, sc.num_envs).astype(np.float32))
    return sc


def make_inputs(sc: Scene, num_steps: Optional[int] = None, step0: int = 0) -> Inputs:
    """Trajectories for every env and link.  Random draws depend on (config seed, env count)."""
    S = sc.num_steps if num_steps is None else num_steps
    E, L = sc.num_envs, sc.layout.num_links
    rng = np.random.default_rng(sc.geom_seed + 7919)
    n_obj = len(sc.grids)
    obj = rng.integers(0, n_obj, size=E).astype(np.int32)
    link_state = np.empty((S, 13, E * L), dtype=np.float32)
    if sc.name == "c1":
        # independent uniform poses in a 4 cm ball around the sphere centre, every step
        for t in range(S):
            r = 0.04 * rng.uniform(size=E * L) ** (1 / 3)
            p = random_unit(rng, E * L) * r[:, None]
            q = rng.normal(size=(E * L, 4)); q /= np.linalg.norm(q, axis=1, keepdims=True)
            v = rng.normal(0, 0.05, size=(E * L, 3))
            w = rng.normal(0, 0.05, size=(E * L, 3))
            link_state[t] = np.concatenate([p, q, v, w], axis=1).T.astype(np.float32)
        return Inputs(link_state, np.repeat(obj[None], S, axis=0), None, step0)

    # smooth sinusoidal trajectories around a base pose near the object surface
    EL = E * L
    env_obj = np.repeat(obj, L)
    base_p = np.empty((EL, 3)); base_n = np.empty((EL, 3))
    for g in range(n_obj):
        idx = np.nonzero(env_obj == g)[0]
        if idx.size == 0:
            continue
        s = sc.grids[g].shape
        x = random_unit(rng, idx.size) * s["extent"]
        for _ in range(3):   # project onto the surface along the exact SDF gradient
            d = shape_sdf(s, x)
            gr = shape_grad(s, x)
            gr /= np.maximum(np.linalg.norm(gr, axis=1, keepdims=True), 1e-12)
            x = x - d[:, None] * gr
        base_p[idx] = x
        base_n[idx] = gr
    off = rng.uniform(-3e-3, 8e-3, size=EL)
    c = base_p + off[:, None] * base_n
    zax = -base_n
    tmp = random_unit(rng, EL)
    xax = tmp - (tmp * zax).sum(1, keepdims=True) * zax
    xax /= np.linalg.norm(xax, axis=1, keepdims=True)
    yax = np.cross(zax, xax)
    Rb = np.stack([xax, yax, zax], axis=2)          # columns = link axes in the world
    qb = matrix_to_quat(Rb)
    A = rng.uniform(0, 5e-3, size=(EL, 3))
    f = rng.uniform(0.5, 3.0, size=(EL, 3))
    ph = rng.uniform(0, 2 * np.pi, size=(EL, 3))
    ax = random_unit(rng, EL)
    fr = rng.uniform(0.5, 3.0, size=EL)
    phr = rng.uniform(0, 2 * np.pi, size=EL)
    ax_w = np.einsum("nij,nj->ni", Rb, ax)
    for t in range(S):
        tt = (step0 + t) * sc.dt
        arg = 2 * np.pi * f * tt + ph
        p = c + A * np.sin(arg)
        v = A * 2 * np.pi * f * np.cos(arg)
        th = 0.3 * np.sin(2 * np.pi * fr * tt + phr)
        thd = 0.3 * 2 * np.pi * fr * np.cos(2 * np.pi * fr * tt + phr)
        qa = np.concatenate([np.cos(th / 2)[:, None], np.sin(th / 2)[:, None] * ax], axis=1)
        q = quat_mul(qb, qa)
        q /= np.linalg.norm(q, axis=1, keepdims=True)
        w = ax_w * thd[:, None]
        link_state[t, 0:3] = p.T
        link_state[t, 3:7] = q.T
        link_state[t, 7:10] = v.T
        link_state[t, 10:13] = w.T
    return Inputs(link_state, np.repeat(obj[None], S, axis=0), None, step0)


def random_object_state(sc: Scene, S: int, rng_seed: int = 1) -> np.ndarray:
    """Optional moving-object inputs [S,13,E] (pose near the origin, small velocities)."""
    rng = np.random.default_rng(rng_seed)
    E = sc.num_envs
    out = np.empty((S, 13, E), dtype=np.float32)
    for t in range(S):
        p = rng.normal(0, 2e-3, size=(E, 3))
        q = rng.normal(size=(E, 4)); q[:, 0] += 6.0
        q /= np.linalg.norm(q, axis=1, keepdims=True)
        v = rng.normal(0, 0.05, size=(E, 3))
        w = rng.normal(0, 0.5, size=(E, 3))
        out[t] = np.concatenate([p, q, v, w], axis=1).T
    return out


def subset_envs(inp: Inputs, envs: np.ndarray, L: int) -> Inputs:
    """Inputs restricted to the env indices `envs` (for sampled oracle checks)."""
    envs = np.asarray(envs)
    cols = (envs[:, None] * L + np.arange(L)[None, :]).reshape(-1)
    ls = np.ascontiguousarray(inp.link_state[:, :, cols])
    oid = np.ascontiguousarray(inp.obj_id[:, envs])
    os_ = None if inp.obj_state is None else np.ascontiguousarray(inp.obj_state[:, :, envs])
    return Inputs(ls, oid, os_, inp.step0)


# ----------------------------------------------------------------------------------------------
# neural-SDF training inputs: random initial weights and sample points (targets are computed
# from the grids by the library / the oracle)
# ----------------------------------------------------------------------------------------------
NSDF_NUM_PARAMS = 15681
NSDF_FAN_INS = (48, 64, 64, 64)      # the four hidden layers; the output layer has fan-in 64


def nsdf_init(n_obj: int, seed: int) -> np.ndarray:
    """He-uniform weights U(-sqrt(6/fan_in), +sqrt(6/fan_in)), zero biases: float32 [n_obj, 15681]
    in the flat order W1[64][48], b1, W2[64][64], b2, W3, b3, W4, b4, w5[64], b5."""
    rng = np.random.default_rng(seed)
    P = np.zeros((n_obj, NSDF_NUM_PARAMS), dtype=np.float64)
    o = 0
    for fan_in in NSDF_FAN_INS:
        lim = np.sqrt(6.0 / fan_in)
        P[:, o:o + 64 * fan_in] = rng.uniform(-lim, lim, (n_obj, 64 * fan_in))
        o += 64 * fan_in + 64
    P[:, o:o + 64] = rng.uniform(-np.sqrt(6.0 / 64), np.sqrt(6.0 / 64), (n_obj, 64))
    return P.astype(np.float32)


def surface_clouds(grids: List[Grid], n: int, seed: int) -> List[np.ndarray]:
    """The tracked surface point cloud of each object (ProximityTaxel, App. A.6): n area-uniform
    points on the analytic surface, object frame, generated in FP64 and rounded once to FP32."""
    rng = np.random.default_rng(seed)
    return [np.ascontiguousarray(_surface_points(g.shape, n, rng).astype(np.float32)) for g in grids]


def _surface_points(s: dict, n: int, rng: np.random.Generator) -> np.ndarray:
    """n area-uniform points on the surface of analytic shape s (object frame, FP64)."""
    f = s["family"]
    if f == "sphere":
        return random_unit(rng, n) * s["r"]
    if f == "box":
        b = s["b"]
        areas = np.array([b[1] * b[2], b[1] * b[2], b[0] * b[2], b[0] * b[2], b[0] * b[1], b[0] * b[1]])
        face = rng.choice(6, size=n, p=areas / areas.sum())
        p = rng.uniform(-1, 1, (n, 3)) * b
        ax = face // 2
        p[np.arange(n), ax] = np.where(face % 2 == 0, -1.0, 1.0) * b[ax]
        return p
    if f == "capsule":
        r, hl = s["r"], s["hl"]
        a_cyl, a_cap = 2 * np.pi * r * 2 * hl, 4 * np.pi * r * r
        cyl = rng.uniform(size=n) < a_cyl / (a_cyl + a_cap)
        th = rng.uniform(0, 2 * np.pi, n)
        p = np.stack([r * np.cos(th), r * np.sin(th), rng.uniform(-hl, hl, n)], axis=1)
        d = random_unit(rng, n) * r
        d[:, 2] += np.where(d[:, 2] >= 0, hl, -hl)
        return np.where(cyl[:, None], p, d)
    if f == "torus":
        R, r = s["R"], s["r"]
        out = np.empty((0, 3))
        while out.shape[0] < n:
            m = 2 * (n - out.shape[0]) + 16
            u, v = rng.uniform(0, 2 * np.pi, m), rng.uniform(0, 2 * np.pi, m)
            keep = rng.uniform(size=m) < (R + r * np.cos(v)) / (R + r)
            u, v = u[keep], v[keep]
            rho = R + r * np.cos(v)
            out = np.concatenate([out, np.stack([rho * np.cos(u), rho * np.sin(u), r * np.sin(v)], axis=1)])
        return out[:n]
    if f == "hull":
        v, t = s["verts"], s["tris"]
        a, b, c = v[t[:, 0]], v[t[:, 1]], v[t[:, 2]]
        area = 0.5 * np.linalg.norm(np.cross(b - a, c - a), axis=1)
        k = rng.choice(t.shape[0], size=n, p=area / area.sum())
        u1, u2 = rng.uniform(size=n), rng.uniform(size=n)
        su = np.sqrt(u1)
        return (1 - su)[:, None] * a[k] + (su * (1 - u2))[:, None] * b[k] + (su * u2)[:, None] * c[k]
    raise ValueError(f)


def nsdf_points(grids: List[Grid], n: int, seed: int, sigma: float = 2e-3) -> np.ndarray:
    """Training points float32 [n_obj, n, 3] (object frame): the first n//2 are area-uniform surface
    points of the analytic shape plus an isotropic N(0, sigma^2) offset, the rest are uniform in
    the grid box.  Points are clamped into the box."""
    rng = np.random.default_rng(seed)
    out = np.empty((len(grids), n, 3), dtype=np.float32)
    for o, g in enumerate(grids):
        lo = g.origin.astype(np.float64)
        hi = lo + (g.n - 1) * float(g.spacing)
        ns = n // 2
        near = _surface_points(g.shape, ns, rng) + rng.normal(0.0, sigma, (ns, 3))
        uni = rng.uniform(lo, hi, (n - ns, 3))
        out[o] = np.clip(np.concatenate([near, uni]), lo, hi)
    return out


def nsdf_pairs(points: np.ndarray, delta: float, seed: int) -> np.ndarray:
    """Pairs for the pair term of the training loss: float32 [n_obj, 2n, 3] with point i at 2i and
    a partner at 2i+1, delta away in a uniformly random direction (object frame, not clamped;
    the targets clamp into the box)."""
    rng = np.random.default_rng(seed)
    n_obj, n, _ = points.shape
    out = np.empty((n_obj, 2 * n, 3), dtype=np.float32)
    out[:, 0::2] = points
    out[:, 1::2] = (points.astype(np.float64) + delta * random_unit(rng, n_obj * n).reshape(n_obj, n, 3)).astype(np.float32)
    return out


# ---------------------------------------------------------------------------------------------
# Contact-audio inputs: material banks and taxel excitations
# ---------------------------------------------------------------------------------------------
# Preset banks from the textbook modes of a simply supported rectangular plate (a x b x h):
#   f_mn = (pi / 2) sqrt(D / (rho h)) ((m / a)^2 + (n / b)^2),  D = E h^3 / (12 (1 - nu^2)),
# Rayleigh damping d = (alpha + beta w^2) / 2 and gains sin(m pi x0 / a) sin(n pi y0 / b) at a
# strike point; the lowest modes below the Nyquist frequency of the sample rate are kept.
AUDIO_PRESETS = {   # Young's modulus [Pa], density [kg/m^3], Poisson ratio, Rayleigh alpha [1/s], beta [s]
    "wood": (10e9, 600.0, 0.30, 60.0, 2e-7),
    "metal": (200e9, 7800.0, 0.29, 4.0, 1e-9),
    "glass": (70e9, 2500.0, 0.22, 10.0, 5e-9),
}


def audio_material(name: str, n_modes: int, fs: float, plate=(0.30, 0.20, 0.003), strike=(0.37, 0.41)):
    E_y, rho, nu, alpha, beta = AUDIO_PRESETS[name]
    a, b, h = plate
    D = E_y * h ** 3 / (12.0 * (1.0 - nu * nu))
    c = 0.5 * np.pi * np.sqrt(D / (rho * h))
    modes = sorted((c * ((m / a) ** 2 + (n / b) ** 2), m, n) for m in range(1, 40) for n in range(1, 40))
    modes = [x for x in modes if x[0] < 0.45 * fs][:n_modes]
    f = np.array([x[0] for x in modes])
    w = 2.0 * np.pi * f
    d = 0.5 * (alpha + beta * w * w)
    g = np.array([np.sin(m * np.pi * strike[0]) * np.sin(n * np.pi * strike[1]) for _, m, n in modes])
    return f, d, g


def audio_materials(n_modes: int = 16, fs: float = 48000.0):
    return [audio_material(k, n_modes, fs) for k in ("wood", "metal", "glass")]


def audio_excitation(num_steps: int, num_envs: int, num_taxels: int, seed: int, contact_frac: float = 0.3,
                     mu: float = 0.5):
    """Taxel forces and contact normals with the structure of the kinematic law: where a taxel is
    in contact, f = F_n m + f_t with m a unit normal, f_t normal to m and |f_t| <= mu F_n; elsewhere
    f = 0 and m = 0.  F_n follows a clipped sinusoid per taxel, so contacts rise, hold and release.
    The torque channels hold a marker (99) where in contact.
    Returns (ft [S][6][E][T], normal [S][3][E][T]), float32."""
    rng = np.random.default_rng(seed)
    S, E, T = num_steps, num_envs, num_taxels
    f32 = np.float32
    m = rng.normal(size=(3, E, T)).astype(f32)
    m /= np.linalg.norm(m, axis=0, keepdims=True)
    amp = rng.uniform(0.5, 3.0, (E, T)).astype(f32)
    ph = rng.uniform(0, 2 * np.pi, (E, T)).astype(f32)
    w = rng.uniform(0.2, 1.5, (E, T)).astype(f32)
    bias = (rng.uniform(-1.0, 1.0, (E, T)) + (contact_frac - 0.5) * 2.0).astype(f32)
    # a tangent direction per taxel normal to m, turning with the step
    a = rng.normal(size=(3, E, T)).astype(f32)
    a -= np.sum(a * m, axis=0, keepdims=True) * m
    a /= np.maximum(np.linalg.norm(a, axis=0, keepdims=True), f32(1e-12))
    b = np.cross(m, a, axis=0)
    ft = np.zeros((S, 6, E, T), f32)
    normal = np.zeros((S, 3, E, T), f32)
    for s in range(S):
        fn = np.maximum(f32(0), amp * np.sin(w * f32(s) + ph) + bias * amp)
        inc = fn > 0
        ang = rng.uniform(0, 2 * np.pi, (E, T)).astype(f32)
        tm = f32(mu) * fn * rng.uniform(0.0, 1.0, (E, T)).astype(f32)
        f = fn * m + tm * (np.cos(ang) * a + np.sin(ang) * b)
        ft[s, 0:3] = np.where(inc, f, f32(0))
        ft[s, 3:6] = np.where(inc, f32(99.0), f32(0))
        normal[s] = np.where(inc, m, f32(0))
    return ft, normal


def elastomer_pads(layout, links, margin: float = 1e-3, thickness: float = 2e-3):
    """Pad boxes of the ElastomerTaxel sensor links: the footprint of each link's markers grown by
    `margin` in the marker plane, `thickness` deep below it (link frame, markers on z = 0 facing
    +z).  Returns (centre [Ls][3], half extents [Ls][3]), float32."""
    c = np.zeros((len(links), 3))
    h = np.zeros((len(links), 3))
    for i, l in enumerate(links):
        x = np.asarray(layout.pos[layout.link_offset[l]:layout.link_offset[l + 1]], np.float64)
        lo, hi = x.min(0), x.max(0)
        c[i, :2] = 0.5 * (lo[:2] + hi[:2])
        h[i, :2] = 0.5 * (hi[:2] - lo[:2]) + margin
        c[i, 2] = -0.5 * thickness
        h[i, 2] = 0.5 * thickness
    return c.astype(np.float32), h.astype(np.float32)


# ---------------------------------------------------------------------------------------------
# Triangle meshes of the objects (the raycast depth backend's collision meshes)
# ---------------------------------------------------------------------------------------------
def _orient_outward(v: np.ndarray, t: np.ndarray, inside: np.ndarray) -> np.ndarray:
    """Flip triangles whose normal points toward `inside` (a point inside the solid near them is
    given per triangle), so every face normal points out."""
    a, b, c = v[t[:, 0]], v[t[:, 1]], v[t[:, 2]]
    n = np.cross(b - a, c - a)
    flip = np.sum(n * (a - inside), axis=1) < 0
    t = t.copy()
    t[flip] = t[flip][:, [0, 2, 1]]
    return t


def _grid_tris(nu: int, nv: int, wrap_v: bool) -> np.ndarray:
    """Triangles of an nu x nv vertex grid (u wraps; v wraps if wrap_v), vertex index u * nv + v."""
    tris = []
    for i in range(nu):
        i2 = (i + 1) % nu
        for j in range(nv if wrap_v else nv - 1):
            j2 = (j + 1) % nv
            a, b, c, d = i * nv + j, i2 * nv + j, i2 * nv + j2, i * nv + j2
            tris += [(a, b, c), (a, c, d)]
    return np.array(tris, np.int32)


def shape_mesh(s: dict, detail: int = 3):
    """A closed, outward-oriented triangle mesh of shape `s` (object frame): (verts [n][3] f32,
    tris [m][3] i32).  Vertices lie on the exact surface."""
    f = s["family"]
    if f == "sphere":
        t0 = (1 + 5 ** 0.5) / 2
        v = np.array([[-1, t0, 0], [1, t0, 0], [-1, -t0, 0], [1, -t0, 0], [0, -1, t0], [0, 1, t0], [0, -1, -t0],
                      [0, 1, -t0], [t0, 0, -1], [t0, 0, 1], [-t0, 0, -1], [-t0, 0, 1]], np.float64)
        t = np.array([[0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11], [1, 5, 9], [5, 11, 4], [11, 10, 2],
                      [10, 7, 6], [7, 1, 8], [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9], [4, 9, 5],
                      [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1]], np.int64)
        verts = [x / np.linalg.norm(x) for x in v]
        for _ in range(detail):
            mid = {}
            def m(i, j):
                k = (min(i, j), max(i, j))
                if k not in mid:
                    p = verts[i] + verts[j]
                    verts.append(p / np.linalg.norm(p))
                    mid[k] = len(verts) - 1
                return mid[k]
            nt = []
            for a, b, c in t:
                ab, bc, ca = m(a, b), m(b, c), m(c, a)
                nt += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
            t = np.array(nt, np.int64)
        v = np.array(verts) * s["r"]
        t = _orient_outward(v, t.astype(np.int32), np.zeros((len(t), 3)))
    elif f == "box":
        b = s["b"]
        v = np.array([[x, y, z] for x in (-1, 1) for y in (-1, 1) for z in (-1, 1)], np.float64) * b
        t = np.array([[0, 1, 3], [0, 3, 2], [4, 6, 7], [4, 7, 5], [0, 4, 5], [0, 5, 1], [2, 3, 7], [2, 7, 6],
                      [0, 2, 6], [0, 6, 4], [1, 5, 7], [1, 7, 3]], np.int32)
        t = _orient_outward(v, t, np.zeros((12, 3)))
    elif f == "capsule":
        r, hl = s["r"], s["hl"]
        nu, nr = 8 * (2 ** detail) // 2, 2 ** detail + 1      # around the axis; rings per hemisphere
        rows = [(r * np.sin(th), hl + r * np.cos(th)) for th in 0.5 * np.pi * np.arange(1, nr + 1) / nr]
        rows += [(r * np.sin(th), -hl + r * np.cos(th)) for th in 0.5 * np.pi * (1 + np.arange(0, nr) / nr)]
        phi = 2 * np.pi * np.arange(nu) / nu
        ring = np.array([[rr * np.cos(p), rr * np.sin(p), z] for p in phi for (rr, z) in rows])
        nv = len(rows)
        t = _grid_tris(nu, nv, wrap_v=False)
        top, bot = len(ring), len(ring) + 1
        v = np.concatenate([ring, [[0, 0, hl + r], [0, 0, -hl - r]]])
        caps = []
        for i in range(nu):
            i2 = (i + 1) % nu
            caps += [(top, i2 * nv, i * nv), (bot, i * nv + nv - 1, i2 * nv + nv - 1)]
        t = np.concatenate([t, np.array(caps, np.int32)])
        ctr = v[t].mean(axis=1)
        inside = np.zeros_like(ctr)
        inside[:, 2] = np.clip(ctr[:, 2], -hl, hl)
        t = _orient_outward(v, t, inside)
    elif f == "torus":
        R, r = s["R"], s["r"]
        nu, nv = 12 * 2 ** detail // 2, 6 * 2 ** detail // 2
        u = 2 * np.pi * np.arange(nu) / nu
        w = 2 * np.pi * np.arange(nv) / nv
        v = np.array([[(R + r * np.cos(b)) * np.cos(a), (R + r * np.cos(b)) * np.sin(a), r * np.sin(b)]
                      for a in u for b in w])
        t = _grid_tris(nu, nv, wrap_v=True)
        ctr = v[t].mean(axis=1)
        ang = np.arctan2(ctr[:, 1], ctr[:, 0])
        inside = np.stack([R * np.cos(ang), R * np.sin(ang), np.zeros(len(t))], 1)
        t = _orient_outward(v, t, inside)
    elif f == "hull":
        v = np.asarray(s["verts"], np.float64)
        t = _orient_outward(v, np.asarray(s["tris"], np.int32), np.tile(v.mean(0), (len(s["tris"]), 1)))
    else:
        raise ValueError(f)
    return np.ascontiguousarray(v, np.float32), np.ascontiguousarray(t, np.int32)


def object_meshes(grids, detail: int = 3):
    return [shape_mesh(g.shape, detail) for g in grids]
