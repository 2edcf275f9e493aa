"""ctypes marshalling for the C oracle (oracle.c).  TEST INFRASTRUCTURE ONLY."""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Dict, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle (contraction off, no fast-math, OpenMP)."""
    srcs = [os.path.join(_HERE, f) for f in ("oracle.c", "oracle_impl.h", "oracle.h", "nsdf.c", "thermal.c",
                                              "proximity.c", "elastomer.c", "raycast.c")]
    srcs = [s for s in srcs if os.path.exists(s)]
    if not force and os.path.exists(_LIB) and all(os.path.getmtime(_LIB) >= os.path.getmtime(s) for s in srcs):
        return _LIB
    cfiles = [s for s in srcs if s.endswith(".c")]
    tmp = _LIB + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
                           "-shared", "-fPIC", "-o", tmp] + cfiles + ["-lm"])
    os.replace(tmp, _LIB)
    return _LIB


class OrGrid(C.Structure):
    _fields_ = [("n", C.c_int32), ("origin", C.c_float * 3), ("spacing", C.c_float),
                ("values", C.c_void_p), ("sphere_c", C.c_double * 3), ("sphere_r", C.c_double)]


class OrProblem(C.Structure):
    _fields_ = [("num_envs", C.c_int32), ("env_index", C.c_void_p),
                ("num_links", C.c_int32), ("num_taxels", C.c_int32), ("num_objects", C.c_int32),
                ("link_offset", C.c_void_p), ("taxel_pos", C.c_void_p), ("taxel_normal", C.c_void_p),
                ("taxel_radius", C.c_void_p), ("grids", C.c_void_p),
                ("k_n", C.c_float), ("c_n", C.c_float), ("alpha", C.c_float), ("k_t", C.c_float),
                ("k_w", C.c_float), ("mu", C.c_float), ("prox_range", C.c_float), ("eta_on", C.c_float),
                ("spring_only", C.c_int32), ("noise_on", C.c_int32), ("seed", C.c_uint64),
                ("drift_sigma", C.c_float), ("white_sigma", C.c_float), ("bias", C.c_float),
                ("quant_step", C.c_float), ("hyst_mode", C.c_int32), ("tau_load", C.c_float),
                ("tau_unload", C.c_float), ("maxwell_beta", C.c_float), ("maxwell_tau", C.c_float),
                ("dt", C.c_float), ("p_dead", C.c_float), ("stuck_lo", C.c_float), ("stuck_hi", C.c_float),
                ("radius_rho", C.c_float), ("gain_lo", C.c_float), ("gain_hi", C.c_float),
                ("xtalk_kind", C.c_int32), ("xtalk_chi", C.c_float), ("xtalk_sigma", C.c_float),
                ("eta_off", C.c_float), ("sdf_mode", C.c_int32), ("nsdf_band", C.c_float),
                ("nsdf_params", C.c_void_p)]


class OrInputs(C.Structure):
    _fields_ = [("link_state", C.c_void_p), ("obj_id", C.c_void_p), ("obj_state", C.c_void_p),
                ("step0", C.c_int64), ("num_steps", C.c_int32)]


class OrOutputs(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in ("bit", "bit_noisy", "depth", "prox", "surfdist", "ft", "ft_noisy",
                                         "normal", "link_sums", "link_sums_noisy", "xtalk_scale", "xhat")]


class OrState(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in ("drift", "hyst", "hyst_prev", "schmitt", "dead", "stuck", "gain")]


def _load():
    global _lib
    if _lib is None:
        build()
        lib = C.CDLL(_LIB)
        lib.or_philox4x32_10.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        for n in ("or_run_f32", "or_run_f64"):
            getattr(lib, n).argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int]
            getattr(lib, n).restype = C.c_int
        for n in ("or_reset_f32", "or_reset_f64"):
            getattr(lib, n).argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64]
            getattr(lib, n).restype = C.c_int
        lib.or_dense_xtalk_f64.argtypes = [C.c_void_p, C.c_void_p]
        lib.or_bf16_round.argtypes = [C.c_float]
        lib.or_bf16_round.restype = C.c_float
        _lib = lib
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


def philox4x32_10(ctr, key) -> np.ndarray:
    lib = _load()
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    o = np.zeros(4, dtype=np.uint32)
    lib.or_philox4x32_10(c.ctypes.data, k.ctypes.data, o.ctypes.data)
    return o


def u01(x):
    x = np.asarray(x, dtype=np.uint64)
    return (2 * (x >> 9) + 1).astype(np.float64) * 2.0 ** -24


def bf16_round(x: float) -> float:
    return float(_load().or_bf16_round(float(x)))


class Oracle:
    """Holds one marshalled problem (a scene restricted to a set of envs) and its noise state."""

    def __init__(self, scene, envs: Optional[np.ndarray] = None, precision: str = "f32",
                 grids_override=None, nsdf_params=None, nsdf_band: float = 1e-3):
        self.lib = _load()
        self.sc = scene
        self.prec = precision
        lay = scene.layout
        self.E = scene.num_envs if envs is None else len(envs)
        self.T, self.L = lay.num_taxels, lay.num_links
        self.env_index = (np.arange(self.E, dtype=np.int32) if envs is None
                          else np.ascontiguousarray(envs, dtype=np.int32))
        self._keep = []
        grids = grids_override if grids_override is not None else scene.grids
        garr = (OrGrid * max(1, len(grids)))()
        for i, g in enumerate(grids):
            if isinstance(g, dict):          # analytic sphere (pins)
                garr[i].n = 0
                garr[i].sphere_c[:] = list(g["c"])
                garr[i].sphere_r = g["r"]
                continue
            v = np.ascontiguousarray(g.values, dtype=np.float32)
            self._keep.append(v)
            garr[i].n = g.n
            garr[i].origin[:] = [float(x) for x in g.origin]
            garr[i].spacing = float(g.spacing)
            garr[i].values = v.ctypes.data
        self._keep.append(garr)
        self.arrs = dict(off=np.ascontiguousarray(lay.link_offset, dtype=np.int32),
                         pos=np.ascontiguousarray(lay.pos, dtype=np.float32),
                         nrm=np.ascontiguousarray(lay.normal, dtype=np.float32),
                         rad=np.ascontiguousarray(lay.radius, dtype=np.float32))
        f, nz = scene.force, scene.noise
        P = OrProblem()
        P.num_envs, P.env_index = self.E, self.env_index.ctypes.data
        P.num_links, P.num_taxels, P.num_objects = self.L, self.T, len(grids)
        P.link_offset, P.taxel_pos = self.arrs["off"].ctypes.data, self.arrs["pos"].ctypes.data
        P.taxel_normal, P.taxel_radius = self.arrs["nrm"].ctypes.data, self.arrs["rad"].ctypes.data
        P.grids = C.addressof(garr)
        P.k_n, P.c_n, P.alpha, P.k_t, P.k_w, P.mu = f.k_n, f.c_n, f.alpha, f.k_t, f.k_w, f.mu
        P.prox_range, P.eta_on, P.spring_only = f.prox_range, f.eta_on, int(f.spring_only)
        P.noise_on, P.seed = int(nz.enabled), nz.seed
        P.drift_sigma, P.white_sigma, P.bias, P.quant_step = nz.drift_sigma, nz.white_sigma, nz.bias, nz.quant_step
        P.hyst_mode, P.tau_load, P.tau_unload = nz.hyst_mode, nz.tau_load_steps, nz.tau_unload_steps
        P.maxwell_beta, P.maxwell_tau, P.dt = nz.maxwell_beta, nz.maxwell_tau_s, nz.dt_s
        P.p_dead, P.stuck_lo, P.stuck_hi = nz.p_dead, nz.stuck_lo, nz.stuck_hi
        P.radius_rho, P.gain_lo, P.gain_hi = nz.radius_rho, nz.gain_lo, nz.gain_hi
        P.xtalk_kind, P.xtalk_chi, P.xtalk_sigma, P.eta_off = nz.xtalk_kind, nz.xtalk_chi, nz.xtalk_sigma, nz.eta_off
        if nsdf_params is not None:      # neural backend: FP32 parameters held as FP64 copies
            prm = np.ascontiguousarray(np.asarray(nsdf_params, np.float32).astype(np.float64))
            assert prm.shape == (len(grids), 15681)
            self._keep.append(prm)
            P.sdf_mode, P.nsdf_band, P.nsdf_params = 1, float(nsdf_band), prm.ctypes.data
        self.P = P
        E, T = self.E, self.T
        self.state = dict(drift=np.zeros((6, E, T)), hyst=np.zeros((6, E, T)), hyst_prev=np.zeros((6, E, T)),
                          schmitt=np.zeros((E, T), np.uint8), dead=np.zeros((E, T), np.uint8),
                          stuck=np.zeros((E, T)), gain=np.ones((E, T)))
        self.St = OrState(**{k: v.ctypes.data for k, v in self.state.items()})
        self.reset(None, 0)

    def reset(self, env_mask: Optional[np.ndarray], step: int):
        m = None if env_mask is None else np.ascontiguousarray(env_mask, dtype=np.uint8)
        fn = self.lib.or_reset_f32 if self.prec == "f32" else self.lib.or_reset_f64
        fn(C.byref(self.P), C.byref(self.St), _ptr(m), int(step))

    def run(self, inp, threads: int = 0, want=("bit", "bit_noisy", "depth", "prox", "surfdist", "ft", "ft_noisy",
                                                "normal", "link_sums", "link_sums_noisy", "xtalk_scale")) -> Dict[str, np.ndarray]:
        S = inp.link_state.shape[0]
        E, T, L = self.E, self.T, self.L
        ls = np.ascontiguousarray(inp.link_state, dtype=np.float32)
        oid = np.ascontiguousarray(inp.obj_id, dtype=np.int32)
        ost = None if inp.obj_state is None else np.ascontiguousarray(inp.obj_state, dtype=np.float32)
        assert ls.shape == (S, 13, E * L) and oid.shape == (S, E)
        shapes = dict(bit=((S, E, T), np.uint8), bit_noisy=((S, E, T), np.uint8), depth=((S, E, T), np.float64),
                      prox=((S, E, T), np.float64), surfdist=((S, E, T), np.float64),
                      ft=((S, 6, E, T), np.float64), ft_noisy=((S, 6, E, T), np.float64),
                      normal=((S, 3, E, T), np.float64), link_sums=((S, 11, E, L), np.float64),
                      link_sums_noisy=((S, 11, E, L), np.float64), xtalk_scale=((S, 6, E, T), np.float64),
                      xhat=((S, 3, E, T), np.float64))
        out = {k: np.zeros(*shapes[k]) for k in want}
        O = OrOutputs(**{k: v.ctypes.data for k, v in out.items()})
        I = OrInputs(ls.ctypes.data, oid.ctypes.data, _ptr(ost), int(inp.step0), S)
        fn = self.lib.or_run_f32 if self.prec == "f32" else self.lib.or_run_f64
        rc = fn(C.byref(self.P), C.byref(I), C.byref(O), C.byref(self.St), int(threads or os.cpu_count() or 1))
        assert rc == 0
        return out


def run_readout(scene, inp, envs=None, precision="f32", threads=0, nsdf_params=None, nsdf_band=1e-3, **kw):
    """Convenience: fresh oracle (reset at inp.step0) over `envs`, run every step of `inp`."""
    o = Oracle(scene, envs, precision, nsdf_params=nsdf_params, nsdf_band=nsdf_band)
    o.reset(None, inp.step0)
    return o.run(inp, threads=threads, **kw)


def dense_xtalk(scene) -> list:
    """The FP64 per-link crosstalk blocks the oracle uses (row-major, one per link)."""
    o = Oracle(scene, np.arange(1), "f64")
    lay = scene.layout
    n = np.diff(lay.link_offset)
    buf = np.zeros(int((n * n).sum()))
    o.lib.or_dense_xtalk_f64(C.byref(o.P), buf.ctypes.data)
    out, off = [], 0
    for k in n:
        out.append(buf[off:off + k * k].reshape(k, k).copy())
        off += k * k
    return out


# ------------------------------------------------------------------------------------------------
# neural SDF surrogate (nsdf.c)
# ------------------------------------------------------------------------------------------------
def _nsdf_lib():
    lib = _load()
    if not getattr(lib, "_nsdf_ready", False):
        lib.or_nsdf_num_params.restype = C.c_int
        lib.or_nsdf_forward.argtypes = [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int]
        lib.or_nsdf_loss_grad.argtypes = [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int,
                                          C.c_double]
        lib.or_nsdf_loss_grad.restype = C.c_double
        lib.or_nsdf_adam.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_int, C.c_double,
                                     C.c_double, C.c_double, C.c_double]
        lib.or_nsdf_targets.argtypes = [C.c_int32, C.c_void_p, C.c_float, C.c_void_p, C.c_int64, C.c_void_p,
                                        C.c_void_p]
        lib.or_nsdf_targets2.argtypes = [C.c_int32, C.c_void_p, C.c_float, C.c_void_p, C.c_int64, C.c_void_p,
                                         C.c_void_p, C.c_void_p]
        lib.or_nsdf_loss_grad2.argtypes = [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                           C.c_int, C.c_double, C.c_double]
        lib.or_nsdf_loss_grad2.restype = C.c_double
        lib.or_nsdf_dirderiv.argtypes = [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int]
        lib.or_nsdf_forward_trace.argtypes = [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                              C.c_void_p, C.c_int]
        lib._nsdf_ready = True
    return lib


def nsdf_num_params() -> int:
    return int(_nsdf_lib().or_nsdf_num_params())


def nsdf_forward(P, x, grad=False, bf16=False):
    lib = _nsdf_lib()
    P = np.ascontiguousarray(P, np.float64)
    x = np.ascontiguousarray(x, np.float64).reshape(-1, 3)
    out = np.zeros(x.shape[0])
    gx = np.zeros_like(x) if grad else None
    lib.or_nsdf_forward(P.ctypes.data, x.shape[0], x.ctypes.data, out.ctypes.data, _ptr(gx), int(bf16))
    return (out, gx) if grad else out


def nsdf_loss_grad(P, x, target, bf16=False, pair_lambda=0.0, gtarget=None, grad_lambda=0.0):
    """Loss and its parameter gradient: mean L1 on the value; pair_lambda > 0 adds the pair term
    over points (2i, 2i+1); grad_lambda > 0 with gtarget [n][3] adds the L1 term on the input
    gradient (see or_nsdf_loss_grad2)."""
    lib = _nsdf_lib()
    P = np.ascontiguousarray(P, np.float64)
    x = np.ascontiguousarray(x, np.float64).reshape(-1, 3)
    t = np.ascontiguousarray(target, np.float64)
    if pair_lambda > 0 and x.shape[0] % 2:
        raise ValueError("the pair term needs an even number of points")
    gt = None
    if grad_lambda > 0:
        gt = np.ascontiguousarray(gtarget, np.float64).reshape(-1, 3)
        assert gt.shape == x.shape
    g = np.zeros_like(P)
    loss = lib.or_nsdf_loss_grad2(P.ctypes.data, x.shape[0], x.ctypes.data, t.ctypes.data, _ptr(gt), g.ctypes.data,
                                   int(bf16), float(pair_lambda), float(grad_lambda))
    return loss, g


def nsdf_forward_trace(P, x, bf16=True):
    """The BF16 rounding record of the forward pass at x[n][3]: encoding features before rounding
    [n][48], layer sums before rounding [n][4][64], after it [n][4][64], and the sum of the
    absolute values of each layer sum's terms [n][4][64]."""
    lib = _nsdf_lib()
    P = np.ascontiguousarray(P, np.float64)
    x = np.ascontiguousarray(x, np.float64).reshape(-1, 3)
    n = x.shape[0]
    feat = np.zeros((n, 48))
    zw, zb, sabs = np.zeros((n, 4, 64)), np.zeros((n, 4, 64)), np.zeros((n, 4, 64))
    lib.or_nsdf_forward_trace(P.ctypes.data, n, x.ctypes.data, feat.ctypes.data, zw.ctypes.data, zb.ctypes.data,
                              sabs.ctypes.data, int(bf16))
    return feat, zw, zb, sabs


def nsdf_dirderiv(P, x, u, bf16=False):
    """Directional derivative of the network output along u[n][3] at x[n][3] by the forward-mode
    tangent pass."""
    lib = _nsdf_lib()
    P = np.ascontiguousarray(P, np.float64)
    x = np.ascontiguousarray(x, np.float64).reshape(-1, 3)
    u = np.ascontiguousarray(u, np.float64).reshape(-1, 3)
    dd = np.zeros(x.shape[0])
    lib.or_nsdf_dirderiv(P.ctypes.data, x.shape[0], x.ctypes.data, u.ctypes.data, dd.ctypes.data, int(bf16))
    return dd


def nsdf_adam(P, m, v, g, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    lib = _nsdf_lib()
    for a in (P, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    g = np.ascontiguousarray(g, np.float64)
    lib.or_nsdf_adam(P.ctypes.data, m.ctypes.data, v.ctypes.data, g.ctypes.data, P.size, int(t), lr, b1, b2, eps)


def nsdf_targets(grid, points, grad=False):
    """FP64 training records {x_hat, phi/e} of object-frame points for one grid (synth.Grid); with
    grad=True also the grid's d phi / d q [n][3] at the clamped points."""
    lib = _nsdf_lib()
    pts = np.ascontiguousarray(points, np.float32).reshape(-1, 3)
    vals = np.ascontiguousarray(grid.values, np.float32)
    org = np.ascontiguousarray(grid.origin, np.float32)
    rec = np.zeros((pts.shape[0], 4))
    gr = np.zeros((pts.shape[0], 3)) if grad else None
    lib.or_nsdf_targets2(int(grid.n), org.ctypes.data, float(grid.spacing), vals.ctypes.data,
                         pts.shape[0], pts.ctypes.data, rec.ctypes.data, _ptr(gr))
    return (rec, gr) if grad else rec


# ------------------------------------------------------------------------------------------------
# thermal fields (thermal.c)
# ------------------------------------------------------------------------------------------------
class OrThermal(C.Structure):
    _fields_ = [("num_fields", C.c_int32), ("field_link", C.c_void_p), ("n", C.c_int32), ("dx", C.c_float),
                ("origin", C.c_float * 3), ("dt", C.c_float), ("k_sensor", C.c_float), ("rho_cp", C.c_float),
                ("emissivity", C.c_float), ("k_object", C.c_float), ("d_w", C.c_float), ("T0", C.c_float),
                ("T_amb", C.c_float), ("P_gen", C.c_float), ("T_obj", C.c_void_p)]


class OrThermalConsts(C.Structure):
    _fields_ = [(k, C.c_double) for k in ("alpha", "r", "h_r", "rho_f", "g", "k_eff", "kappa")]


def _thermal_lib():
    lib = _load()
    if not getattr(lib, "_th_ready", False):
        lib.or_thermal_constants.argtypes = [C.c_void_p, C.c_void_p]
        lib.or_thermal_voxel.argtypes = [C.c_void_p, C.c_void_p]
        lib.or_thermal_voxel.restype = C.c_int
        lib.or_thermal_stable.argtypes = [C.c_void_p, C.c_double, C.c_int32]
        lib.or_thermal_stable.restype = C.c_int
        for nm in ("or_thermal_run_f32", "or_thermal_run_f64"):
            getattr(lib, nm).argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                                         C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]
            getattr(lib, nm).restype = C.c_int
        lib._th_ready = True
    return lib


def _thermal_struct(th, keep):
    links = np.ascontiguousarray(th.field_links, np.int32)
    tobj = np.ascontiguousarray(th.T_obj, np.float32)
    keep += [links, tobj]
    s = OrThermal()
    s.num_fields, s.field_link, s.n, s.dx = len(links), links.ctypes.data, th.n, th.dx
    s.origin[:] = [float(x) for x in th.origin]
    s.dt, s.k_sensor, s.rho_cp, s.emissivity = th.dt, th.k_sensor, th.rho_cp, th.emissivity
    s.k_object, s.d_w, s.T0, s.T_amb, s.P_gen = th.k_object, th.d_w, th.T0, th.T_amb, th.P_gen
    s.T_obj = tobj.ctypes.data
    return s


def thermal_constants(th) -> dict:
    keep = []
    s = _thermal_struct(th, keep)
    K = OrThermalConsts()
    _thermal_lib().or_thermal_constants(C.byref(s), C.byref(K))
    return {k: getattr(K, k) for k, _ in K._fields_}


def thermal_voxel(th, x) -> int:
    keep = []
    s = _thermal_struct(th, keep)
    xx = np.ascontiguousarray(x, np.float32)
    return int(_thermal_lib().or_thermal_voxel(C.byref(s), xx.ctypes.data))


def thermal_stable(th, delta_max: float, taxels_per_voxel_max: int) -> bool:
    keep = []
    s = _thermal_struct(th, keep)
    return bool(_thermal_lib().or_thermal_stable(C.byref(s), float(delta_max), int(taxels_per_voxel_max)))


def thermal_run(th, layout, depth, fields=None, precision="f64"):
    """Integrate the fields over the steps of `depth` ([S][E][T] clean depths).  fields: [E][F][n][n][n]
    initial state (default: T0 everywhere), updated in place.  Returns (fields, taxel_temp [S][E][T],
    ledger [S][E][F][2] = (stored energy change, source energy) in J)."""
    lib = _thermal_lib()
    keep = []
    s = _thermal_struct(th, keep)
    depth = np.ascontiguousarray(depth, np.float64)
    S, E, T = depth.shape
    F, n = len(th.field_links), th.n
    dt = np.float32 if precision == "f32" else np.float64
    if fields is None:
        fields = np.full((E, F, n, n, n), th.T0, dtype=dt)
    assert fields.dtype == dt and fields.flags.c_contiguous and fields.shape == (E, F, n, n, n)
    off = np.ascontiguousarray(layout.link_offset, np.int32)
    pos = np.ascontiguousarray(layout.pos, np.float32)
    tt = np.zeros((S, E, T))
    led = np.zeros((S, E, F, 2))
    fn = lib.or_thermal_run_f32 if precision == "f32" else lib.or_thermal_run_f64
    rc = fn(C.byref(s), E, T, off.ctypes.data, pos.ctypes.data, depth.ctypes.data, S, fields.ctypes.data,
            tt.ctypes.data, led.ctypes.data)
    assert rc == 0
    return fields, tt, led


# ------------------------------------------------------------------------------------------------
# ProximityTaxel (proximity.c)
# ------------------------------------------------------------------------------------------------
class OrProxProblem(C.Structure):
    _fields_ = [("num_envs", C.c_int32), ("num_links", C.c_int32), ("num_taxels", C.c_int32),
                ("num_objects", C.c_int32), ("link_offset", C.c_void_p), ("taxel_pos", C.c_void_p),
                ("taxel_normal", C.c_void_p), ("taxel_radius", C.c_void_p), ("cloud_offset", C.c_void_p),
                ("cloud", C.c_void_p), ("k", C.c_double), ("k_s", C.c_double), ("density", C.c_double),
                ("seed", C.c_uint64), ("radius_rho", C.c_double)]


def prox_run(link_offset, taxel_pos, taxel_normal, taxel_radius, clouds, link_state, obj_id, obj_state=None,
             step0=0, k=300.0, k_s=10.0, density=100.0, seed=0, radius_rho=0.0, gain=None, threads=0,
             with_count=False):
    """ProximityTaxel channels in FP64 by brute force over every point (App. A.6).
    link_state [S][13][E*L], obj_id [S][E], obj_state [S][13][E] or None, clouds: list of [n_o][3]
    object-frame points.  Returns (ft [S][6][E][T] link frame, mass [S][E][T] = sum_i P_ij), and
    with with_count the number of points inside each sphere [S][E][T] as a third value."""
    lib = _load()
    if not getattr(lib, "_prox_ready", False):
        lib.or_prox_run.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_int32, C.c_void_p,
                                    C.c_void_p, C.c_void_p, C.c_void_p, C.c_int]
        lib._prox_ready = True
    off = np.ascontiguousarray(link_offset, np.int32)
    pos = np.ascontiguousarray(taxel_pos, np.float32).reshape(-1, 3)
    nrm = np.ascontiguousarray(taxel_normal, np.float32).reshape(-1, 3)
    rad = np.ascontiguousarray(taxel_radius, np.float32).reshape(-1)
    T, L = pos.shape[0], off.size - 1
    coff = np.zeros(len(clouds) + 1, np.int32)
    coff[1:] = np.cumsum([len(c) for c in clouds])
    cloud = np.ascontiguousarray(np.concatenate([np.asarray(c, np.float32).reshape(-1, 3) for c in clouds])
                                 if clouds else np.zeros((0, 3), np.float32))
    ls = np.ascontiguousarray(link_state, np.float32)
    oid = np.ascontiguousarray(obj_id, np.int32)
    S, E = oid.shape
    assert ls.shape == (S, 13, E * L)
    ost = None if obj_state is None else np.ascontiguousarray(obj_state, np.float32)
    gn = None if gain is None else np.ascontiguousarray(gain, np.float32).reshape(E, T)
    Pb = OrProxProblem(E, L, T, len(clouds), off.ctypes.data, pos.ctypes.data, nrm.ctypes.data, rad.ctypes.data,
                       coff.ctypes.data, cloud.ctypes.data, float(k), float(k_s), float(density), int(seed),
                       float(radius_rho))
    ft = np.zeros((S, 6, E, T))
    mass = np.zeros((S, E, T))
    cnt = np.zeros((S, E, T)) if with_count else None
    lib.or_prox_run(C.byref(Pb), ls.ctypes.data, oid.ctypes.data, _ptr(ost), int(step0), S, _ptr(gn),
                    ft.ctypes.data, mass.ctypes.data, _ptr(cnt), int(threads or os.cpu_count() or 1))
    return (ft, mass, cnt) if with_count else (ft, mass)


# ---------------------------------------------------------------------------------------------
# ElastomerTaxel (elastomer.c)
# ---------------------------------------------------------------------------------------------
class OrElastProblem(C.Structure):
    _fields_ = [("num_envs", C.c_int32), ("num_links", C.c_int32), ("num_taxels", C.c_int32),
                ("num_objects", C.c_int32), ("link_offset", C.c_void_p), ("taxel_pos", C.c_void_p),
                ("taxel_normal", C.c_void_p), ("taxel_radius", C.c_void_p), ("num_sensor_links", C.c_int32),
                ("sensor_links", C.c_void_p), ("pad_center", C.c_void_p), ("pad_half", C.c_void_p),
                ("cloud_offset", C.c_void_p), ("cloud", C.c_void_p), ("s_d", C.c_double), ("s_s", C.c_double),
                ("lambda_d", C.c_double), ("lambda_s", C.c_double), ("alpha", C.c_double), ("c", C.c_double),
                ("eps", C.c_double), ("eta_enter", C.c_float), ("eta_exit", C.c_float), ("max_points", C.c_int32)]


class OrElastState(C.Structure):
    _fields_ = [("anchor", C.c_void_p), ("active", C.c_void_p), ("last_oid", C.c_void_p)]


ELASTOMER_DEFAULTS = dict(s_d=100.0, s_s=100.0, lambda_d=8000.0, lambda_s=2000.0, alpha=1.2, c=1.0, eps=2e-3,
                          eta_enter=1e-5, eta_exit=1e-4)


def elastomer_new_state(num_envs, num_sensor_links, max_points):
    return {"anchor": np.zeros((num_envs, num_sensor_links, max_points, 3), np.float32),
            "active": np.zeros((num_envs, num_sensor_links, max_points), np.uint8),
            "last_oid": np.full((num_envs, num_sensor_links), -2, np.int32)}


def elastomer_run(link_offset, taxel_pos, taxel_normal, taxel_radius, sensor_links, pad_center, pad_half, clouds,
                  link_state, obj_id, obj_state, depth, state=None, threads=0, **params):
    """ElastomerTaxel marker displacements (App. A.7).  link_state [S][13][E*L], obj_id [S][E],
    obj_state [S][13][E] or None, depth [S][E][T] (the readout's clean depth, float32), clouds:
    list of [n_o][3] object-frame points.  state (elastomer_new_state(...) or None: no anchors) is
    updated in place.  Returns (disp [S][3][E][T] link frame, absum [S][E][T], state); entries of
    taxels outside the sensor links are 0."""
    lib = _load()
    if not getattr(lib, "_elast_ready", False):
        lib.or_elast_run.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                     C.c_int32, C.c_void_p, C.c_void_p, C.c_int]
        lib._elast_ready = True
    prm = dict(ELASTOMER_DEFAULTS)
    prm.update(params)
    off = np.ascontiguousarray(link_offset, np.int32)
    pos = np.ascontiguousarray(taxel_pos, np.float32).reshape(-1, 3)
    nrm = np.ascontiguousarray(taxel_normal, np.float32).reshape(-1, 3)
    rad = np.ascontiguousarray(taxel_radius, np.float32).reshape(-1)
    T, L = pos.shape[0], off.size - 1
    sl = np.ascontiguousarray(sensor_links, np.int32)
    pc = np.ascontiguousarray(pad_center, np.float32).reshape(-1, 3)
    ph = np.ascontiguousarray(pad_half, np.float32).reshape(-1, 3)
    coff = np.zeros(len(clouds) + 1, np.int32)
    coff[1:] = np.cumsum([len(c) for c in clouds])
    cloud = np.ascontiguousarray(np.concatenate([np.asarray(c, np.float32).reshape(-1, 3) for c in clouds])
                                 if clouds else np.zeros((0, 3), np.float32))
    NP = max([len(c) for c in clouds] + [1])
    ls = np.ascontiguousarray(link_state, np.float32)
    oid = np.ascontiguousarray(obj_id, np.int32)
    S, E = oid.shape
    assert ls.shape == (S, 13, E * L)
    ost = None if obj_state is None else np.ascontiguousarray(obj_state, np.float32)
    dep = np.ascontiguousarray(depth, np.float32).reshape(S, E, T)
    if state is None:
        state = elastomer_new_state(E, sl.size, NP)
    assert state["anchor"].shape == (E, sl.size, NP, 3)
    Pb = OrElastProblem(E, L, T, len(clouds), off.ctypes.data, pos.ctypes.data, nrm.ctypes.data, rad.ctypes.data,
                        sl.size, sl.ctypes.data, pc.ctypes.data, ph.ctypes.data, coff.ctypes.data, cloud.ctypes.data,
                        prm["s_d"], prm["s_s"], prm["lambda_d"], prm["lambda_s"], prm["alpha"], prm["c"], prm["eps"],
                        prm["eta_enter"], prm["eta_exit"], NP)
    St = OrElastState(state["anchor"].ctypes.data, state["active"].ctypes.data, state["last_oid"].ctypes.data)
    disp = np.zeros((S, 3, E, T))
    absum = np.zeros((S, E, T))
    lib.or_elast_run(C.byref(Pb), C.byref(St), ls.ctypes.data, oid.ctypes.data, _ptr(ost), dep.ctypes.data, S,
                     disp.ctypes.data, absum.ctypes.data, int(threads or os.cpu_count() or 1))
    return disp, absum, state


# ---------------------------------------------------------------------------------------------
# Raycast contact-depth backend (raycast.c)
# ---------------------------------------------------------------------------------------------
class OrRayProblem(C.Structure):
    _fields_ = [("num_envs", C.c_int32), ("num_links", C.c_int32), ("num_taxels", C.c_int32),
                ("num_objects", C.c_int32), ("link_offset", C.c_void_p), ("taxel_pos", C.c_void_p),
                ("taxel_normal", C.c_void_p), ("taxel_radius", C.c_void_p), ("vert_offset", C.c_void_p),
                ("verts", C.c_void_p), ("tri_offset", C.c_void_p), ("tris", C.c_void_p)]


def raycast_run(link_offset, taxel_pos, taxel_normal, taxel_radius, meshes, link_state, obj_id, obj_state=None,
                tri_query=None, threads=0):
    """Raycast contact depth (App. A.1) by brute force over every triangle, FP64.  meshes: list of
    (verts [n][3] f32, tris [m][3] i32) per object, outward faces.  Returns (depth [S][E][T],
    normal [S][3][E][T] link frame, tri [S][E][T] winning triangle or -1) and, with tri_query
    [S][E][T], a fourth value: the penetration of each queried triangle alone."""
    lib = _load()
    if not getattr(lib, "_ray_ready", False):
        lib.or_ray_run.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p,
                                   C.c_void_p, C.c_void_p, C.c_void_p, C.c_int]
        lib._ray_ready = True
    off = np.ascontiguousarray(link_offset, np.int32)
    pos = np.ascontiguousarray(taxel_pos, np.float32).reshape(-1, 3)
    nrm = np.ascontiguousarray(taxel_normal, np.float32).reshape(-1, 3)
    rad = np.ascontiguousarray(taxel_radius, np.float32).reshape(-1)
    T, L = pos.shape[0], off.size - 1
    voff = np.zeros(len(meshes) + 1, np.int32)
    toff = np.zeros(len(meshes) + 1, np.int32)
    voff[1:] = np.cumsum([len(m[0]) for m in meshes])
    toff[1:] = np.cumsum([len(m[1]) for m in meshes])
    verts = np.ascontiguousarray(np.concatenate([np.asarray(m[0], np.float32).reshape(-1, 3) for m in meshes])
                                 if meshes else np.zeros((0, 3), np.float32))
    tris = np.ascontiguousarray(np.concatenate([np.asarray(m[1], np.int32).reshape(-1, 3) for m in meshes])
                                if meshes else np.zeros((0, 3), np.int32))
    ls = np.ascontiguousarray(link_state, np.float32)
    oid = np.ascontiguousarray(obj_id, np.int32)
    S, E = oid.shape
    assert ls.shape == (S, 13, E * L)
    ost = None if obj_state is None else np.ascontiguousarray(obj_state, np.float32)
    Pb = OrRayProblem(E, L, T, len(meshes), off.ctypes.data, pos.ctypes.data, nrm.ctypes.data, rad.ctypes.data,
                      voff.ctypes.data, verts.ctypes.data, toff.ctypes.data, tris.ctypes.data)
    depth = np.zeros((S, E, T))
    normal = np.zeros((S, 3, E, T))
    tri = np.zeros((S, E, T), np.int32)
    tq = None if tri_query is None else np.ascontiguousarray(tri_query, np.int32).reshape(S, E, T)
    tp = None if tri_query is None else np.zeros((S, E, T))
    lib.or_ray_run(C.byref(Pb), ls.ctypes.data, oid.ctypes.data, _ptr(ost), S, depth.ctypes.data, normal.ctypes.data,
                   tri.ctypes.data, _ptr(tq), _ptr(tp), int(threads or os.cpu_count() or 1))
    return (depth, normal, tri) if tri_query is None else (depth, normal, tri, tp)
