"""Thin ctypes binding of the tg_readout C ABI (include/tg_readout.h).

Argument marshalling only: every step of the readout runs in the HIP library.  PyTorch
provides device memory and the current stream.  There is no fallback: if the compiled
library is missing, loading raises.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Dict, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtg_readout.so")
ABI_VERSION = 1

TG_OUT_BITS, TG_OUT_DEPTH, TG_OUT_PROX, TG_OUT_FT = 1, 2, 4, 8
TG_OUT_NOISY, TG_OUT_NORMAL, TG_OUT_SURFDIST, TG_OUT_LINK_SUMS = 16, 32, 64, 128
TG_OUT_TEMP = 256
TG_DEVERR_BAD_OBJECT_ID = 1  # device error flag: an object id outside [-1, num_objects) was read
OUT_ALL = 255                 # every readout output (TG_OUT_TEMP is added when the scene has fields)
NSDF_NUM_PARAMS = 15681


class TgError(RuntimeError):
    pass


class TgSdfGrid(C.Structure):
    _fields_ = [("n", C.c_int32), ("origin", C.c_float * 3), ("spacing", C.c_float), ("values", C.c_void_p)]


class TgNoiseDesc(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("drift_sigma", C.c_float), ("white_sigma", C.c_float), ("bias", C.c_float),
                ("quant_step", C.c_float), ("hyst_mode", C.c_int32), ("tau_load_steps", C.c_float),
                ("tau_unload_steps", C.c_float), ("maxwell_beta", C.c_float), ("maxwell_tau_s", C.c_float),
                ("dt_s", C.c_float), ("p_dead", C.c_float), ("stuck_lo", C.c_float), ("stuck_hi", C.c_float),
                ("radius_rho", C.c_float), ("gain_lo", C.c_float), ("gain_hi", C.c_float),
                ("xtalk_kind", C.c_int32), ("xtalk_chi", C.c_float), ("xtalk_sigma", C.c_float),
                ("eta_off", C.c_float)]


class TgThermalDesc(C.Structure):
    _fields_ = [("num_fields", C.c_int32), ("field_links", C.c_void_p), ("n", C.c_int32), ("dx", C.c_float),
                ("origin", C.c_float * 3), ("dt", C.c_float), ("k_sensor", C.c_float), ("rho_cp", C.c_float),
                ("emissivity", C.c_float), ("k_object", C.c_float), ("d_w", C.c_float), ("T0", C.c_float),
                ("T_amb", C.c_float), ("P_gen", C.c_float), ("T_obj", C.c_void_p), ("solver", C.c_int32),
                ("h_conv", C.c_float), ("lag_tau", C.c_float)]


class TgReadoutConfig(C.Structure):
    _fields_ = [("abi_version", C.c_uint32), ("num_envs", C.c_int32), ("num_links", C.c_int32),
                ("num_taxels", C.c_int32), ("num_objects", C.c_int32), ("link_taxel_offset", C.c_void_p),
                ("taxel_pos", C.c_void_p), ("taxel_normal", C.c_void_p), ("taxel_radius", C.c_void_p),
                ("grids", C.c_void_p), ("k_n", C.c_float), ("c_n", C.c_float), ("alpha", C.c_float),
                ("k_t", C.c_float), ("k_w", C.c_float), ("mu", C.c_float), ("prox_range", C.c_float),
                ("eta_on", C.c_float), ("ft_spring_only", C.c_int32), ("noise_enabled", C.c_int32),
                ("noise", TgNoiseDesc), ("output_mask", C.c_uint32), ("sdf_mode", C.c_int32),
                ("nsdf_band", C.c_float), ("nsdf_params", C.c_void_p), ("thermal", C.c_void_p)]


class TgStepInputs(C.Structure):
    _fields_ = [("link_state", C.c_void_p), ("obj_state", C.c_void_p), ("obj_id", C.c_void_p), ("step", C.c_int64)]


class TgStepOutputs(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in ("contact_bits", "contact_bits_noisy", "depth", "prox", "surfdist", "ft",
                                         "ft_noisy", "normal", "link_sums", "link_sums_noisy", "temperature")]


_lib = None


def load() -> C.CDLL:
    """Load the compiled HIP library; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise TgError(f"HIP library not built: {LIB_PATH} (run python -m paper_2606_22332_amd.build)")
    lib = C.CDLL(LIB_PATH)
    P = C.c_void_p
    sig = {
        "tg_readout_create": ([P, P], C.c_int),
        "tg_readout_step": ([P, P, P, P], C.c_int),
        "tg_readout_rollout": ([P, P, P, C.c_int32, P], C.c_int),
        "tg_readout_reset": ([P, P, C.c_int64, P], C.c_int),
        "tg_readout_state_size": ([P, P], C.c_int),
        "tg_readout_get_state": ([P, P, C.c_size_t, P], C.c_int),
        "tg_readout_set_state": ([P, P, C.c_size_t, P], C.c_int),
        "tg_readout_launch_shape": ([P, P, P], C.c_int),
        "tg_readout_poll_errors": ([P, P], C.c_int),
        "tg_readout_set_graph": ([P, C.c_int32], C.c_int),
        "tg_readout_autotune": ([P, P, P, C.c_int32, P, P, P], C.c_int),
        "tg_readout_set_work_plan": ([P, C.c_int32], C.c_int),
        "tg_readout_destroy": ([P], C.c_int),
        "tg_readout_last_error": ([P], C.c_char_p),
        "tg_status_string": ([C.c_int], C.c_char_p),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _check(lib, h, rc, what):
    if rc != 0:
        msg = lib.tg_readout_last_error(h).decode()
        raise TgError(f"{what}: {lib.tg_status_string(rc).decode()} ({rc}): {msg}")


def _stream_ptr(stream) -> Optional[int]:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def make_config(scene, output_mask: int = OUT_ALL, keep: Optional[list] = None, nsdf_params=None,
                nsdf_band: float = 1e-3) -> TgReadoutConfig:
    """Marshal a synthetic scene (paper_2606_22332_amd.synth.Scene) into tg_readout_config.
    Host arrays are kept alive in `keep` until create has copied them."""
    keep = [] if keep is None else keep
    lay = scene.layout
    arrs = dict(off=np.ascontiguousarray(lay.link_offset, np.int32), pos=np.ascontiguousarray(lay.pos, np.float32),
                nrm=np.ascontiguousarray(lay.normal, np.float32), rad=np.ascontiguousarray(lay.radius, np.float32))
    keep.append(arrs)
    grids = (TgSdfGrid * len(scene.grids))()
    for i, g in enumerate(scene.grids):
        v = np.ascontiguousarray(g.values, np.float32)
        keep.append(v)
        grids[i].n = g.n
        grids[i].origin[:] = [float(x) for x in g.origin]
        grids[i].spacing = float(g.spacing)
        grids[i].values = v.ctypes.data
    keep.append(grids)
    f, nz = scene.force, scene.noise
    cfg = TgReadoutConfig()
    cfg.abi_version = ABI_VERSION
    cfg.num_envs, cfg.num_links = scene.num_envs, lay.num_links
    cfg.num_taxels, cfg.num_objects = lay.num_taxels, len(scene.grids)
    cfg.link_taxel_offset, cfg.taxel_pos = arrs["off"].ctypes.data, arrs["pos"].ctypes.data
    cfg.taxel_normal, cfg.taxel_radius = arrs["nrm"].ctypes.data, arrs["rad"].ctypes.data
    cfg.grids = C.addressof(grids)
    cfg.k_n, cfg.c_n, cfg.alpha, cfg.k_t, cfg.k_w, cfg.mu = f.k_n, f.c_n, f.alpha, f.k_t, f.k_w, f.mu
    cfg.prox_range, cfg.eta_on, cfg.ft_spring_only = f.prox_range, f.eta_on, int(f.spring_only)
    cfg.noise_enabled = int(nz.enabled)
    n = cfg.noise
    n.seed, n.drift_sigma, n.white_sigma, n.bias, n.quant_step = nz.seed, nz.drift_sigma, nz.white_sigma, nz.bias, nz.quant_step
    n.hyst_mode, n.tau_load_steps, n.tau_unload_steps = nz.hyst_mode, nz.tau_load_steps, nz.tau_unload_steps
    n.maxwell_beta, n.maxwell_tau_s, n.dt_s = nz.maxwell_beta, nz.maxwell_tau_s, nz.dt_s
    n.p_dead, n.stuck_lo, n.stuck_hi = nz.p_dead, nz.stuck_lo, nz.stuck_hi
    n.radius_rho, n.gain_lo, n.gain_hi = nz.radius_rho, nz.gain_lo, nz.gain_hi
    n.xtalk_kind, n.xtalk_chi, n.xtalk_sigma, n.eta_off = nz.xtalk_kind, nz.xtalk_chi, nz.xtalk_sigma, nz.eta_off
    if not nz.enabled:
        output_mask &= ~TG_OUT_NOISY
    cfg.output_mask = output_mask
    th = getattr(scene, "thermal", None)
    if th is not None:
        links = np.ascontiguousarray(th.field_links, np.int32)
        tobj = np.ascontiguousarray(th.T_obj, np.float32)
        assert tobj.shape == (scene.num_envs,)
        td = TgThermalDesc()
        td.num_fields, td.field_links, td.n, td.dx = len(links), links.ctypes.data, th.n, th.dx
        td.origin[:] = [float(x) for x in th.origin]
        td.dt, td.k_sensor, td.rho_cp, td.emissivity = th.dt, th.k_sensor, th.rho_cp, th.emissivity
        td.k_object, td.d_w, td.T0, td.T_amb, td.P_gen = th.k_object, th.d_w, th.T0, th.T_amb, th.P_gen
        td.T_obj = tobj.ctypes.data
        td.solver, td.h_conv, td.lag_tau = int(th.solver), float(th.h_conv), float(th.lag_tau)
        keep += [links, tobj, td]
        cfg.thermal = C.addressof(td)
        cfg.output_mask |= TG_OUT_TEMP
    if nsdf_params is not None:      # torch float32 [num_objects, 15681] on the device
        assert nsdf_params.is_cuda and nsdf_params.is_contiguous()
        assert tuple(nsdf_params.shape) == (len(scene.grids), NSDF_NUM_PARAMS)
        cfg.sdf_mode, cfg.nsdf_band, cfg.nsdf_params = 1, float(nsdf_band), nsdf_params.data_ptr()
    return cfg


@dataclass
class DeviceInputs:
    link_state: "object"          # torch float32 [S,13,E*L] on cuda
    obj_id: "object"              # torch int32 [S,E]
    obj_state: "object" = None    # torch float32 [S,13,E] or None
    step0: int = 0


def to_device(inp, device="cuda") -> DeviceInputs:
    import torch
    ls = torch.from_numpy(np.ascontiguousarray(inp.link_state, np.float32)).to(device)
    oid = torch.from_numpy(np.ascontiguousarray(inp.obj_id, np.int32)).to(device)
    ost = None
    if inp.obj_state is not None:
        ost = torch.from_numpy(np.ascontiguousarray(inp.obj_state, np.float32)).to(device)
    return DeviceInputs(ls, oid, ost, int(inp.step0))


class Readout:
    """A tg_readout handle plus torch-allocated output buffers for up to `max_steps` steps."""

    def __init__(self, scene, output_mask: int = OUT_ALL, device: str = "cuda", nsdf_params=None,
                 nsdf_band: float = 1e-3):
        import torch
        self.lib = load()
        self.scene = scene
        keep: list = []
        cfg = make_config(scene, output_mask, keep, nsdf_params, nsdf_band)
        self.mask = cfg.output_mask
        h = C.c_void_p()
        rc = self.lib.tg_readout_create(C.byref(cfg), C.byref(h))
        _check(self.lib, None, rc, "tg_readout_create")
        self.h = h
        self.device = device
        self.E, self.L, self.T = scene.num_envs, scene.layout.num_links, scene.layout.num_taxels
        self.W = (self.T + 63) // 64
        self._torch = torch
        self.out: Dict[str, "object"] = {}
        self._out_steps = 0

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            self.lib.tg_readout_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def poll_errors(self) -> int:
        """Device error flags since the last poll (TG_DEVERR_*); waits for the device."""
        f = C.c_uint32()
        _check(self.lib, self.h, self.lib.tg_readout_poll_errors(self.h, C.byref(f)), "poll_errors")
        return f.value

    def launch_shape(self):
        eb, th = C.c_int32(), C.c_int32()
        _check(self.lib, self.h, self.lib.tg_readout_launch_shape(self.h, C.byref(eb), C.byref(th)), "launch_shape")
        return eb.value, th.value

    def alloc_outputs(self, steps: int):
        torch = self._torch
        E, T, L, W, m = self.E, self.T, self.L, self.W, self.mask
        dev = self.device
        f32 = dict(dtype=torch.float32, device=dev)
        o = {}
        if m & TG_OUT_BITS:
            o["bits"] = torch.zeros((steps, E, W), dtype=torch.int64, device=dev)
        if m & TG_OUT_DEPTH:
            o["depth"] = torch.zeros((steps, E, T), **f32)
        if m & TG_OUT_PROX:
            o["prox"] = torch.zeros((steps, E, T), **f32)
        if m & TG_OUT_SURFDIST:
            o["surfdist"] = torch.zeros((steps, E, T), **f32)
        if m & TG_OUT_FT:
            o["ft"] = torch.zeros((steps, 6, E, T), **f32)
        if m & TG_OUT_NOISY:
            o["ft_noisy"] = torch.zeros((steps, 6, E, T), **f32)
            o["bits_noisy"] = torch.zeros((steps, E, W), dtype=torch.int64, device=dev)
        if m & TG_OUT_NORMAL:
            o["normal"] = torch.zeros((steps, 3, E, T), **f32)
        if m & TG_OUT_LINK_SUMS:
            # the library writes [S][11][L][E]; exposed as a [S][11][E][L] view
            o["link_sums"] = torch.zeros((steps, 11, L, E), **f32).permute(0, 1, 3, 2)
            if m & TG_OUT_NOISY:
                o["link_sums_noisy"] = torch.zeros((steps, 11, L, E), **f32).permute(0, 1, 3, 2)
        if m & TG_OUT_TEMP:
            o["temperature"] = torch.zeros((steps, E, T), **f32)
        self.out = o
        self._out_steps = steps
        return o

    def _outputs_struct(self, out, s0: int) -> TgStepOutputs:
        def ptr(k):
            t = out.get(k)
            return None if t is None else t[s0].data_ptr()
        return TgStepOutputs(ptr("bits"), ptr("bits_noisy"), ptr("depth"), ptr("prox"), ptr("surfdist"), ptr("ft"),
                             ptr("ft_noisy"), ptr("normal"), ptr("link_sums"), ptr("link_sums_noisy"),
                             ptr("temperature"))

    def rollout(self, dinp: DeviceInputs, n_steps: Optional[int] = None, s_in: int = 0, s_out: int = 0,
                out=None, stream=None):
        """Steps s_in .. s_in+n-1 of the device inputs into output slots s_out .., one launch."""
        S = dinp.link_state.shape[0] if n_steps is None else n_steps
        out = self.out if out is None else out
        ist = TgStepInputs(dinp.link_state[s_in].data_ptr(),
                           None if dinp.obj_state is None else dinp.obj_state[s_in].data_ptr(),
                           dinp.obj_id[s_in].data_ptr(), dinp.step0 + s_in)
        ost = self._outputs_struct(out, s_out)
        rc = self.lib.tg_readout_rollout(self.h, C.byref(ist), C.byref(ost), int(S), _stream_ptr(stream))
        _check(self.lib, self.h, rc, "tg_readout_rollout")

    def step(self, dinp: DeviceInputs, s: int, s_out: Optional[int] = None, stream=None):
        out = self.out
        ist = TgStepInputs(dinp.link_state[s].data_ptr(),
                           None if dinp.obj_state is None else dinp.obj_state[s].data_ptr(),
                           dinp.obj_id[s].data_ptr(), dinp.step0 + s)
        ost = self._outputs_struct(out, s if s_out is None else s_out)
        rc = self.lib.tg_readout_step(self.h, C.byref(ist), C.byref(ost), _stream_ptr(stream))
        _check(self.lib, self.h, rc, "tg_readout_step")

    def reset(self, env_mask=None, step: int = 0, stream=None):
        ptr = None if env_mask is None else env_mask.data_ptr()
        rc = self.lib.tg_readout_reset(self.h, ptr, int(step), _stream_ptr(stream))
        _check(self.lib, self.h, rc, "tg_readout_reset")

    def state_size(self) -> int:
        n = C.c_size_t()
        _check(self.lib, self.h, self.lib.tg_readout_state_size(self.h, C.byref(n)), "state_size")
        return n.value

    def get_state(self, buf, stream=None):
        _check(self.lib, self.h, self.lib.tg_readout_get_state(self.h, buf.data_ptr(), buf.numel() * buf.element_size(),
                                                               _stream_ptr(stream)), "get_state")

    def set_state(self, buf, stream=None):
        _check(self.lib, self.h, self.lib.tg_readout_set_state(self.h, buf.data_ptr(), buf.numel() * buf.element_size(),
                                                               _stream_ptr(stream)), "set_state")

    def set_graph(self, enable: bool):
        _check(self.lib, self.h, self.lib.tg_readout_set_graph(self.h, int(bool(enable))), "set_graph")

    def set_work_plan(self, readouts_per_workgroup: int):
        _check(self.lib, self.h, self.lib.tg_readout_set_work_plan(self.h, int(readouts_per_workgroup)),
               "set_work_plan")

    def autotune(self, dinp: DeviceInputs, n_steps: Optional[int] = None, stream=None):
        """Time the candidate work plans on these inputs (outputs are overwritten, state restored);
        returns (readouts per workgroup, ms of the best rollout)."""
        S = dinp.link_state.shape[0] if n_steps is None else n_steps
        ist = TgStepInputs(dinp.link_state[0].data_ptr(),
                           None if dinp.obj_state is None else dinp.obj_state[0].data_ptr(),
                           dinp.obj_id[0].data_ptr(), dinp.step0)
        ost = self._outputs_struct(self.out, 0)
        best, ms = C.c_int32(), C.c_float()
        rc = self.lib.tg_readout_autotune(self.h, C.byref(ist), C.byref(ost), int(S), _stream_ptr(stream),
                                          C.byref(best), C.byref(ms))
        _check(self.lib, self.h, rc, "tg_readout_autotune")
        return best.value, ms.value

    def thermal_fields(self):
        """Copy of the temperature fields, torch float32 [E, F, 16, 16, 16] (z, y, x), or None."""
        th = getattr(self.scene, "thermal", None)
        if th is None:
            return None
        torch = self._torch
        buf = torch.empty(self.state_size(), dtype=torch.uint8, device=self.device)
        self.get_state(buf)
        nb = self.E * len(th.field_links) * 16 ** 3 * 4
        # the fields end the state, but for the sensor-lag readings [E][T] of the spectral solver
        tail = self.E * self.T * 4 if getattr(th, "solver", 0) == 1 and getattr(th, "lag_tau", 0.0) > 0 else 0
        end = buf.numel() - tail
        return buf[end - nb:end].view(torch.float32).reshape(self.E, len(th.field_links), 16, 16, 16).clone()


def unpack_bits(words: np.ndarray, T: int) -> np.ndarray:
    """[..., W] int64/uint64 words -> [..., T] uint8 (bit j%64 of word j/64)."""
    w = np.ascontiguousarray(words).view(np.uint64)
    b = np.unpackbits(w.view(np.uint8).reshape(w.shape + (8,)), axis=-1, bitorder="little")
    return b.reshape(w.shape[:-1] + (w.shape[-1] * 64,))[..., :T]


# ------------------------------------------------------------------------------------------------
# neural SDF surrogate (include/tg_nsdf.h)
# ------------------------------------------------------------------------------------------------


class TgNsdfConfig(C.Structure):
    _fields_ = [("abi_version", C.c_uint32), ("num_objects", C.c_int32), ("grids", C.c_void_p)]


class TgNsdfTrainParams(C.Structure):
    _fields_ = [("lr", C.c_float), ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float),
                ("batch", C.c_int32), ("seed", C.c_uint64), ("pair_lambda", C.c_float), ("grad_lambda", C.c_float)]


_nsdf_ready = False


def _nsdf_lib() -> C.CDLL:
    global _nsdf_ready
    lib = load()
    if not _nsdf_ready:
        P, I64 = C.c_void_p, C.c_int64
        sig = {
            "tg_nsdf_create": ([P, P], C.c_int),
            "tg_nsdf_destroy": ([P], C.c_int),
            "tg_nsdf_last_error": ([P], C.c_char_p),
            "tg_nsdf_targets": ([P, P, I64, P, P, P], C.c_int),
            "tg_nsdf_grad": ([P, P, P, P, I64, C.c_float, C.c_float, P, P, P], C.c_int),
            "tg_nsdf_adam": ([P, P, P, P, I64, I64, P, P], C.c_int),
            "tg_nsdf_train": ([P, P, P, P, P, P, I64, I64, C.c_int32, P, P, P], C.c_int),
            "tg_nsdf_query": ([P, P, P, I64, P, P, P, P], C.c_int),
            "tg_nsdf_query_noalloc": ([P, P, P, I64, P, P, P, P], C.c_int),
            "tg_nsdf_query_trace": ([P, P, P, I64, P, P, P, P, P], C.c_int),
        }
        for name, (args, res) in sig.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = res
        _nsdf_ready = True
    return lib


def train_params(lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, batch=16384, seed=0,
                 pair_lambda=0.0, grad_lambda=0.0) -> TgNsdfTrainParams:
    return TgNsdfTrainParams(lr, beta1, beta2, eps, batch, seed, pair_lambda, grad_lambda)


class Nsdf:
    """Per-object neural SDF networks over the grids of a scene (or a list of synth.Grid).

    Parameters, Adam moments, samples and outputs are torch tensors on the current device;
    this class only passes their pointers to the library."""

    def __init__(self, grids):
        self.lib = _nsdf_lib()
        self.n_obj = len(grids)
        keep = []
        arr = (TgSdfGrid * self.n_obj)()
        for i, g in enumerate(grids):
            v = np.ascontiguousarray(g.values, np.float32)
            keep.append(v)
            arr[i].n = g.n
            arr[i].origin[:] = [float(x) for x in g.origin]
            arr[i].spacing = float(g.spacing)
            arr[i].values = v.ctypes.data
        cfg = TgNsdfConfig(ABI_VERSION, self.n_obj, C.cast(arr, C.c_void_p).value)
        h = C.c_void_p()
        rc = self.lib.tg_nsdf_create(C.byref(cfg), C.byref(h))
        if rc != 0:
            raise TgError(f"tg_nsdf_create: {self.lib.tg_nsdf_last_error(None).decode()}")
        self.h = h

    def _chk(self, rc, what):
        if rc != 0:
            raise TgError(f"{what}: {self.lib.tg_status_string(rc).decode()}: "
                          f"{self.lib.tg_nsdf_last_error(self.h).decode()}")

    def targets(self, points, samples=None, stream=None, grad=False):
        """points: float32 [n_obj, n, 3] object-frame positions -> float32 [n_obj, n, 4] records;
        grad=True: also the gradient records [n_obj, n, 4] {d phi / d q, 0}."""
        import torch
        assert points.is_cuda and points.dtype == torch.float32 and points.is_contiguous()
        n = points.shape[1]
        if samples is None:
            samples = torch.empty((self.n_obj, n, 4), dtype=torch.float32, device=points.device)
        gs = torch.empty((self.n_obj, n, 4), dtype=torch.float32, device=points.device) if grad else None
        self._chk(self.lib.tg_nsdf_targets(self.h, points.data_ptr(), n, samples.data_ptr(),
                                           gs.data_ptr() if grad else None, _stream_ptr(stream)), "tg_nsdf_targets")
        return (samples, gs) if grad else samples

    def grad(self, params, samples, pair_lambda=0.0, stream=None, grad_samples=None, grad_lambda=0.0):
        import torch
        n = samples.shape[1]
        g = torch.empty_like(params)
        loss = torch.empty(self.n_obj, dtype=torch.float32, device=params.device)
        gp = grad_samples.data_ptr() if grad_samples is not None else None
        self._chk(self.lib.tg_nsdf_grad(self.h, params.data_ptr(), samples.data_ptr(), gp, n, float(pair_lambda),
                                        float(grad_lambda), g.data_ptr(), loss.data_ptr(), _stream_ptr(stream)),
                  "tg_nsdf_grad")
        return loss, g

    def adam(self, params, m, v, grad, t, hp: TgNsdfTrainParams, stream=None):
        self._chk(self.lib.tg_nsdf_adam(params.data_ptr(), m.data_ptr(), v.data_ptr(), grad.data_ptr(),
                                        params.numel(), int(t), C.byref(hp), _stream_ptr(stream)), "tg_nsdf_adam")

    def train(self, params, m, v, samples, step0, n_steps, hp: TgNsdfTrainParams, loss=None, stream=None,
              grad_samples=None):
        n = samples.shape[1]
        lp = loss.data_ptr() if loss is not None else None
        gp = grad_samples.data_ptr() if grad_samples is not None else None
        self._chk(self.lib.tg_nsdf_train(self.h, params.data_ptr(), m.data_ptr(), v.data_ptr(), samples.data_ptr(),
                                         gp, n, int(step0), int(n_steps), C.byref(hp), lp, _stream_ptr(stream)),
                  "tg_nsdf_train")

    def query(self, params, offsets, xhat, grad=True, stream=None, noalloc=False, out=None, grad_out=None):
        """offsets: int64 list/array [n_obj+1] (points grouped by object); xhat: float32 [n, 3] on device.
        noalloc: call tg_nsdf_query_noalloc (images in the library's static device array) instead of
        tg_nsdf_query.  out / grad_out: caller-provided result tensors ([n], [n, 3])."""
        import torch
        offs = np.asarray(offsets, np.int64)
        d_off = torch.from_numpy(offs).to(xhat.device)
        n = xhat.shape[0]
        if out is None:
            out = torch.empty(n, dtype=torch.float32, device=xhat.device)
        g = grad_out
        if grad and g is None:
            g = torch.empty((n, 3), dtype=torch.float32, device=xhat.device)
        self._keep = d_off
        fn = self.lib.tg_nsdf_query_noalloc if noalloc else self.lib.tg_nsdf_query
        name = "tg_nsdf_query_noalloc" if noalloc else "tg_nsdf_query"
        self._chk(fn(self.h, params.data_ptr(), d_off.data_ptr(), int(np.diff(offs).max()) if offs.size > 1 else 0,
                     xhat.data_ptr(), out.data_ptr(), g.data_ptr() if grad else None, _stream_ptr(stream)), name)
        return (out, g) if grad else out

    def query_trace(self, params, offsets, xhat, stream=None):
        """tg_nsdf_query_trace: (out [n], grad [n, 3], trace int16 [n, 5, 64] of BF16 bit patterns:
        row 0 the encoding features, rows 1..4 the hidden layers' pre-activations)."""
        import torch
        offs = np.asarray(offsets, np.int64)
        d_off = torch.from_numpy(offs).to(xhat.device)
        n = xhat.shape[0]
        out = torch.empty(n, dtype=torch.float32, device=xhat.device)
        g = torch.empty((n, 3), dtype=torch.float32, device=xhat.device)
        tr = torch.zeros((n, 5, 64), dtype=torch.int16, device=xhat.device)
        self._keep = d_off
        self._chk(self.lib.tg_nsdf_query_trace(self.h, params.data_ptr(), d_off.data_ptr(),
                                               int(np.diff(offs).max()) if offs.size > 1 else 0, xhat.data_ptr(),
                                               out.data_ptr(), g.data_ptr(), tr.data_ptr(), _stream_ptr(stream)),
                  "tg_nsdf_query_trace")
        return out, g, tr

    def close(self):
        if getattr(self, "h", None):
            self.lib.tg_nsdf_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------------------------------------
# ProximityTaxel readout (include/tg_proximity.h)
# ------------------------------------------------------------------------------------------------
class TgPointCloud(C.Structure):
    _fields_ = [("num_points", C.c_int32), ("points", C.c_void_p)]


class TgProxConfig(C.Structure):
    _fields_ = [("abi_version", C.c_uint32), ("num_envs", C.c_int32), ("num_links", C.c_int32),
                ("num_taxels", C.c_int32), ("num_objects", C.c_int32), ("link_taxel_offset", C.c_void_p),
                ("taxel_pos", C.c_void_p), ("taxel_normal", C.c_void_p), ("sensing_radius", C.c_void_p),
                ("clouds", C.c_void_p), ("k", C.c_float), ("k_s", C.c_float), ("density", C.c_float),
                ("seed", C.c_uint64), ("radius_rho", C.c_float)]


_prox_ready = False


def _prox_lib() -> C.CDLL:
    global _prox_ready
    lib = load()
    if not _prox_ready:
        P = C.c_void_p
        sig = {"tg_prox_create": ([P, P], C.c_int), "tg_prox_destroy": ([P], C.c_int),
               "tg_prox_last_error": ([P], C.c_char_p),
               "tg_prox_rollout": ([P, P, P, P, P, C.c_int32, P], C.c_int)}
        for name, (args, res) in sig.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = res
        _prox_ready = True
    return lib


class Proximity:
    """ProximityTaxel readout of a scene's hand over per-object surface point clouds (list of
    float32 [n][3], object frame).  Inputs and outputs are torch tensors on the current device; this
    class only passes their pointers to the library."""

    def __init__(self, scene, clouds, radius=0.01, k=300.0, k_s=10.0, density=100.0, seed=0, radius_rho=0.0):
        import torch
        self._torch = torch
        self.lib = _prox_lib()
        lay = scene.layout
        self.E, self.T, self.L = scene.num_envs, lay.num_taxels, lay.num_links
        keep = [np.ascontiguousarray(lay.link_offset, np.int32), np.ascontiguousarray(lay.pos, np.float32),
                np.ascontiguousarray(lay.normal, np.float32), np.full(self.T, radius, np.float32)]
        pcs = (TgPointCloud * len(clouds))()
        for i, c in enumerate(clouds):
            a = np.ascontiguousarray(c, np.float32).reshape(-1, 3)
            keep.append(a)
            pcs[i].num_points = a.shape[0]
            pcs[i].points = a.ctypes.data
        cfg = TgProxConfig(ABI_VERSION, self.E, self.L, self.T, len(clouds), keep[0].ctypes.data, keep[1].ctypes.data,
                           keep[2].ctypes.data, keep[3].ctypes.data, C.cast(pcs, C.c_void_p).value, float(k),
                           float(k_s), float(density), int(seed), float(radius_rho))
        h = C.c_void_p()
        rc = self.lib.tg_prox_create(C.byref(cfg), C.byref(h))
        if rc != 0:
            raise TgError(f"tg_prox_create: {self.lib.tg_prox_last_error(None).decode()}")
        self.h = h

    def rollout(self, dinp: DeviceInputs, n_steps: Optional[int] = None, s_in: int = 0, ft=None, mass=None,
                gain=None, want_mass: bool = True, stream=None):
        """Steps s_in .. s_in+n-1 of the device inputs, one launch.  Returns (ft [n][6][E][T],
        mass [n][E][T] or None)."""
        torch = self._torch
        S = dinp.link_state.shape[0] - s_in if n_steps is None else n_steps
        dev = dinp.link_state.device
        if ft is None:
            ft = torch.empty((S, 6, self.E, self.T), dtype=torch.float32, device=dev)
        if mass is None and want_mass:
            mass = torch.empty((S, self.E, self.T), dtype=torch.float32, device=dev)
        ist = TgStepInputs(dinp.link_state[s_in].data_ptr(),
                           None if dinp.obj_state is None else dinp.obj_state[s_in].data_ptr(),
                           dinp.obj_id[s_in].data_ptr(), dinp.step0 + s_in)
        rc = self.lib.tg_prox_rollout(self.h, C.byref(ist), ft.data_ptr(), None if mass is None else mass.data_ptr(),
                                      None if gain is None else gain.data_ptr(), int(S), _stream_ptr(stream))
        if rc != 0:
            raise TgError(f"tg_prox_rollout: {self.lib.tg_status_string(rc).decode()}: "
                          f"{self.lib.tg_prox_last_error(self.h).decode()}")
        return ft, mass

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            self.lib.tg_prox_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class TgAudioMaterial(C.Structure):
    _fields_ = [("num_modes", C.c_int32), ("freq", C.c_void_p), ("decay", C.c_void_p), ("gain", C.c_void_p)]


class TgAudioConfig(C.Structure):
    _fields_ = [("abi_version", C.c_uint32), ("num_envs", C.c_int32), ("num_taxels", C.c_int32),
                ("num_sensor_links", C.c_int32), ("sensor_taxel_begin", C.c_void_p),
                ("sensor_taxel_end", C.c_void_p), ("num_materials", C.c_int32), ("materials", C.c_void_p),
                ("slots", C.c_int32), ("samples_per_step", C.c_int32), ("dt", C.c_double), ("g_imp", C.c_double),
                ("g_scr", C.c_double), ("seed", C.c_uint64), ("lanes_per_pair", C.c_int32)]


_audio_ready = False


def _audio_lib() -> C.CDLL:
    global _audio_ready
    lib = load()
    if not _audio_ready:
        P = C.c_void_p
        sig = {"tg_audio_create": ([P, P], C.c_int), "tg_audio_destroy": ([P], C.c_int),
               "tg_audio_last_error": ([P], C.c_char_p), "tg_audio_reset": ([P, P], C.c_int),
               "tg_audio_rollout": ([P, P, P, P, C.c_int64, C.c_int32, P, P], C.c_int)}
        for name, (args, res) in sig.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = res
        _audio_ready = True
    return lib


class Audio:
    """Contact-audio sensor on the sensor links of a taxel layout.  materials: list of (freq, decay,
    gain) arrays; sensor_ranges: list of (first taxel, one past the last).  Buffers are torch
    tensors on the current device; this class only passes their pointers to the library."""

    def __init__(self, num_envs, num_taxels, sensor_ranges, materials, slots, samples_per_step, dt,
                 g_imp=1.0, g_scr=1.0, seed=0, lanes_per_pair=0):
        import torch
        self._torch = torch
        self.lib = _audio_lib()
        self.E, self.T, self.K = int(num_envs), int(num_taxels), int(samples_per_step)
        self.Ls = len(sensor_ranges)
        begin = np.ascontiguousarray([r[0] for r in sensor_ranges], np.int32)
        end = np.ascontiguousarray([r[1] for r in sensor_ranges], np.int32)
        keep = [begin, end]
        mats = (TgAudioMaterial * max(len(materials), 1))()
        for i, (f, d, g) in enumerate(materials):
            arrs = [np.ascontiguousarray(x, np.float64).reshape(-1) for x in (f, d, g)]
            keep += arrs
            mats[i].num_modes = arrs[0].shape[0]
            mats[i].freq, mats[i].decay, mats[i].gain = (a.ctypes.data for a in arrs)
        cfg = TgAudioConfig(ABI_VERSION, self.E, self.T, self.Ls, begin.ctypes.data, end.ctypes.data, len(materials),
                            C.cast(mats, C.c_void_p).value, int(slots), self.K, float(dt), float(g_imp), float(g_scr),
                            int(seed), int(lanes_per_pair))
        h = C.c_void_p()
        rc = self.lib.tg_audio_create(C.byref(cfg), C.byref(h))
        if rc != 0:
            raise TgError(f"tg_audio_create: {self.lib.tg_status_string(rc).decode()}: "
                          f"{self.lib.tg_audio_last_error(None).decode()}")
        self.h = h

    def rollout(self, ft, normal, material, step0=0, out=None, stream=None):
        """ft [S][6][E][T], normal [S][3][E][T] (float32), material [E] (int32), all on the device.
        Returns the samples [S][E][Ls][K]."""
        torch = self._torch
        S = ft.shape[0]
        if out is None:
            out = torch.empty((S, self.E, self.Ls, self.K), dtype=torch.float32, device=ft.device)
        rc = self.lib.tg_audio_rollout(self.h, ft.data_ptr(), normal.data_ptr(), material.data_ptr(), int(step0),
                                       int(S), out.data_ptr(), _stream_ptr(stream))
        if rc != 0:
            raise TgError(f"tg_audio_rollout: {self.lib.tg_status_string(rc).decode()}: "
                          f"{self.lib.tg_audio_last_error(self.h).decode()}")
        return out

    def reset(self, stream=None):
        rc = self.lib.tg_audio_reset(self.h, _stream_ptr(stream))
        if rc != 0:
            raise TgError(f"tg_audio_reset: {self.lib.tg_audio_last_error(self.h).decode()}")

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            self.lib.tg_audio_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class TgElastConfig(C.Structure):
    _fields_ = [("abi_version", C.c_uint32), ("num_envs", C.c_int32), ("num_links", C.c_int32),
                ("num_taxels", C.c_int32), ("num_objects", C.c_int32), ("link_taxel_offset", C.c_void_p),
                ("taxel_pos", C.c_void_p), ("taxel_normal", C.c_void_p), ("taxel_radius", C.c_void_p),
                ("num_sensor_links", C.c_int32), ("sensor_links", C.c_void_p), ("pad_center", C.c_void_p),
                ("pad_half", C.c_void_p), ("clouds", C.c_void_p), ("s_d", C.c_float), ("s_s", C.c_float),
                ("lambda_d", C.c_float), ("lambda_s", C.c_float), ("alpha", C.c_float), ("c", C.c_float),
                ("eps", C.c_float), ("eta_enter", C.c_float), ("eta_exit", C.c_float)]


_elast_ready = False


def _elast_lib() -> C.CDLL:
    global _elast_ready
    lib = load()
    if not _elast_ready:
        P = C.c_void_p
        sig = {"tg_elast_create": ([P, P], C.c_int), "tg_elast_destroy": ([P], C.c_int),
               "tg_elast_last_error": ([P], C.c_char_p), "tg_elast_reset": ([P, P], C.c_int),
               "tg_elast_rollout": ([P, P, P, P, C.c_int32, P], C.c_int)}
        for name, (args, res) in sig.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = res
        _elast_ready = True
    return lib


ELASTOMER_PARAMS = dict(s_d=100.0, s_s=100.0, lambda_d=8000.0, lambda_s=2000.0, alpha=1.2, c=1.0, eps=2e-3,
                        eta_enter=1e-5, eta_exit=1e-4)


class Elastomer:
    """ElastomerTaxel on the sensor links of a scene's layout: pads (centre, half extents) per
    sensor link, surface clouds per object (float32 [n][3], object frame).  Buffers are torch
    tensors on the current device; this class only passes their pointers to the library."""

    def __init__(self, scene, clouds, sensor_links, pad_center, pad_half, **params):
        import torch
        self._torch = torch
        self.lib = _elast_lib()
        lay = scene.layout
        self.E, self.T, self.L = scene.num_envs, lay.num_taxels, lay.num_links
        prm = dict(ELASTOMER_PARAMS)
        prm.update(params)
        keep = [np.ascontiguousarray(lay.link_offset, np.int32), np.ascontiguousarray(lay.pos, np.float32),
                np.ascontiguousarray(lay.normal, np.float32), np.ascontiguousarray(lay.radius, np.float32),
                np.ascontiguousarray(sensor_links, np.int32), np.ascontiguousarray(pad_center, np.float32),
                np.ascontiguousarray(pad_half, np.float32)]
        pcs = (TgPointCloud * max(len(clouds), 1))()
        for i, c in enumerate(clouds):
            a = np.ascontiguousarray(c, np.float32).reshape(-1, 3)
            keep.append(a)
            pcs[i].num_points = a.shape[0]
            pcs[i].points = a.ctypes.data
        cfg = TgElastConfig(ABI_VERSION, self.E, self.L, self.T, len(clouds), *[k.ctypes.data for k in keep[:4]],
                            keep[4].size, keep[4].ctypes.data, keep[5].ctypes.data, keep[6].ctypes.data,
                            C.cast(pcs, C.c_void_p).value,
                            *[float(prm[k]) for k in ("s_d", "s_s", "lambda_d", "lambda_s", "alpha", "c", "eps",
                                                      "eta_enter", "eta_exit")])
        h = C.c_void_p()
        rc = self.lib.tg_elast_create(C.byref(cfg), C.byref(h))
        if rc != 0:
            raise TgError(f"tg_elast_create: {self.lib.tg_status_string(rc).decode()}: "
                          f"{self.lib.tg_elast_last_error(None).decode()}")
        self.h = h

    def rollout(self, dinp: DeviceInputs, depth, n_steps: Optional[int] = None, s_in: int = 0, disp=None,
                stream=None):
        """Steps s_in .. s_in+n-1 of the device inputs with the readout's clean depth of the same
        steps (depth [n][E][T]), one launch.  Returns disp [n][3][E][T] (zeros off the pads when
        the buffer is allocated here)."""
        torch = self._torch
        S = dinp.link_state.shape[0] - s_in if n_steps is None else n_steps
        if disp is None:
            disp = torch.zeros((S, 3, self.E, self.T), dtype=torch.float32, device=dinp.link_state.device)
        ist = TgStepInputs(dinp.link_state[s_in].data_ptr(),
                           None if dinp.obj_state is None else dinp.obj_state[s_in].data_ptr(),
                           dinp.obj_id[s_in].data_ptr(), dinp.step0 + s_in)
        rc = self.lib.tg_elast_rollout(self.h, C.byref(ist), depth.data_ptr(), disp.data_ptr(), int(S),
                                       _stream_ptr(stream))
        if rc != 0:
            raise TgError(f"tg_elast_rollout: {self.lib.tg_status_string(rc).decode()}: "
                          f"{self.lib.tg_elast_last_error(self.h).decode()}")
        return disp

    def reset(self, stream=None):
        rc = self.lib.tg_elast_reset(self.h, _stream_ptr(stream))
        if rc != 0:
            raise TgError(f"tg_elast_reset: {self.lib.tg_elast_last_error(self.h).decode()}")

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            self.lib.tg_elast_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class TgMesh(C.Structure):
    _fields_ = [("num_verts", C.c_int32), ("verts", C.c_void_p), ("num_tris", C.c_int32), ("tris", C.c_void_p)]


class TgRayConfig(C.Structure):
    _fields_ = [("abi_version", C.c_uint32), ("num_envs", C.c_int32), ("num_links", C.c_int32),
                ("num_taxels", C.c_int32), ("num_objects", C.c_int32), ("link_taxel_offset", C.c_void_p),
                ("taxel_pos", C.c_void_p), ("taxel_normal", C.c_void_p), ("taxel_radius", C.c_void_p),
                ("meshes", C.c_void_p)]


_ray_ready = False


def _ray_lib() -> C.CDLL:
    global _ray_ready
    lib = load()
    if not _ray_ready:
        P = C.c_void_p
        sig = {"tg_ray_create": ([P, P], C.c_int), "tg_ray_destroy": ([P], C.c_int),
               "tg_ray_last_error": ([P], C.c_char_p),
               "tg_ray_rollout": ([P, P, P, P, P, C.c_int32, P], C.c_int)}
        for name, (args, res) in sig.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = res
        _ray_ready = True
    return lib


class Raycast:
    """The raycast contact-depth backend over per-object triangle meshes (list of (verts [n][3]
    f32, tris [m][3] i32), outward faces).  Buffers are torch tensors on the current device; this
    class only passes their pointers to the library."""

    def __init__(self, scene, meshes):
        import torch
        self._torch = torch
        self.lib = _ray_lib()
        lay = scene.layout
        self.E, self.T, self.L = scene.num_envs, lay.num_taxels, lay.num_links
        keep = [np.ascontiguousarray(lay.link_offset, np.int32), np.ascontiguousarray(lay.pos, np.float32),
                np.ascontiguousarray(lay.normal, np.float32), np.ascontiguousarray(lay.radius, np.float32)]
        ms = (TgMesh * max(len(meshes), 1))()
        for i, (v, t) in enumerate(meshes):
            va = np.ascontiguousarray(v, np.float32).reshape(-1, 3)
            tb = np.ascontiguousarray(t, np.int32).reshape(-1, 3)
            keep += [va, tb]
            ms[i].num_verts, ms[i].verts, ms[i].num_tris, ms[i].tris = va.shape[0], va.ctypes.data, tb.shape[0], tb.ctypes.data
        cfg = TgRayConfig(ABI_VERSION, self.E, self.L, self.T, len(meshes), *[k.ctypes.data for k in keep[:4]],
                          C.cast(ms, C.c_void_p).value)
        h = C.c_void_p()
        rc = self.lib.tg_ray_create(C.byref(cfg), C.byref(h))
        if rc != 0:
            raise TgError(f"tg_ray_create: {self.lib.tg_status_string(rc).decode()}: "
                          f"{self.lib.tg_ray_last_error(None).decode()}")
        self.h = h

    def rollout(self, dinp: DeviceInputs, n_steps: Optional[int] = None, s_in: int = 0, depth=None, normal=None,
                tri=None, want_normal: bool = True, want_tri: bool = True, stream=None):
        """Steps s_in .. s_in+n-1, one launch.  Returns (depth [n][E][T], normal [n][3][E][T] or None,
        tri [n][E][T] or None)."""
        torch = self._torch
        S = dinp.link_state.shape[0] - s_in if n_steps is None else n_steps
        dev = dinp.link_state.device
        if depth is None:
            depth = torch.empty((S, self.E, self.T), dtype=torch.float32, device=dev)
        if normal is None and want_normal:
            normal = torch.empty((S, 3, self.E, self.T), dtype=torch.float32, device=dev)
        if tri is None and want_tri:
            tri = torch.empty((S, self.E, self.T), dtype=torch.int32, device=dev)
        ist = TgStepInputs(dinp.link_state[s_in].data_ptr(),
                           None if dinp.obj_state is None else dinp.obj_state[s_in].data_ptr(),
                           dinp.obj_id[s_in].data_ptr(), dinp.step0 + s_in)
        rc = self.lib.tg_ray_rollout(self.h, C.byref(ist), depth.data_ptr(),
                                     None if normal is None else normal.data_ptr(),
                                     None if tri is None else tri.data_ptr(), int(S), _stream_ptr(stream))
        if rc != 0:
            raise TgError(f"tg_ray_rollout: {self.lib.tg_status_string(rc).decode()}: "
                          f"{self.lib.tg_ray_last_error(self.h).decode()}")
        return depth, normal, tri

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            self.lib.tg_ray_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
