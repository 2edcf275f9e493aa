#!/usr/bin/env python3
"""Throughput of the tactile readout on one MI355X.

A "step" here is one pass of the whole hot path over one batch: a 64-step rollout of the
20480-env x 1024-taxel hand (16 links of 16..128 taxels) against 32 objects on 64^3 grid SDFs,
with the clean readout (contact bits, depth, proximity, force/torque), the noise model (dense
BF16 crosstalk on MFMA, first-order lag, Gaussian drift, dead taxels, Schmitt bits) and the
per-link sums, all in one persistent launch.  Inputs are resident in HBM before timing.

Prints one JSON line with the throughput, the roofline of the readout kernel (algorithmic bytes
per launch / measured launch time) and a CPU baseline (the oracle on a bounded sample).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "taxel-readouts/sec on 1 MI355X (grid-SDF vs neural-SDF at ≤0.5 mm depth err)"
# weight of the network training's L1 term on its input gradient (0: value-only recipe)
DEFAULT_GRAD_LAMBDA = 0.005
HBM_PEAK_GBS = 8000.0


def algorithmic_bytes(E, L, T, S, n_obj, grid_n, noisy=True, sums=True):
    """Bytes the method must move for one launch of S steps (per readout: outputs, amortised
    state, inputs, link sums; per launch: the grids once)."""
    R = E * T * S
    per_readout = 4 + 24 + 4 + 1 / 8                    # depth, f/tau, prox, clean bit
    if noisy:
        per_readout += 24 + 1 / 8                       # noisy f/tau, noisy bit
    state = E * T * (2 * (24 + 24) + 2 * 1 / 8 + 1 / 8) if noisy else 0   # drift+lag r/w, Schmitt r/w, dead r
    inputs = S * (E * L * 52 + E * 4)                   # link_state + obj_id
    link = S * E * L * 44 * (2 if noisy else 1) if sums else 0
    grids = n_obj * grid_n ** 3 * 4
    return R * per_readout + state + inputs + link + grids, R


def _oracle_rate(sc, inp, precision, threads, target_s, n0):
    """Readouts/s of the oracle over a sample of envs (all steps), grown until it takes about
    target_s (at most three rounds); returns (rate, envs in the sample, seconds)."""
    import oracle
    from paper_2606_22332_amd import synth
    L, T = sc.layout.num_links, sc.layout.num_taxels
    want = ("bit", "bit_noisy", "depth", "prox", "ft", "ft_noisy", "link_sums", "link_sums_noisy")
    n = n0
    envs = np.arange(n)
    t0 = time.perf_counter()
    oracle.run_readout(sc, synth.subset_envs(inp, envs, L), envs=envs, precision=precision, threads=threads, want=want)
    dt = time.perf_counter() - t0
    for _ in range(3):
        if dt >= target_s / 2 or n >= sc.num_envs:
            break
        n2 = int(min(sc.num_envs, max(n + 1, n * target_s / max(dt, 1e-3))))
        envs = np.linspace(0, sc.num_envs - 1, n2).astype(np.int64)
        t0 = time.perf_counter()
        oracle.run_readout(sc, synth.subset_envs(inp, envs, L), envs=envs, precision=precision, threads=threads,
                           want=want)
        dt = time.perf_counter() - t0
        n = n2
    S = inp.link_state.shape[0]
    return n * T * S / dt, n, dt


def cpu_baseline(sc, inp, target_s=12.0):
    """The oracle as it stands (OpenMP over envs) on bounded samples of envs of the same workload,
    all steps, scaled to readouts/s: the FP32 parity build on every host thread (the reported
    value), the FP64 build on every thread, and the FP32 build on one thread."""
    threads = os.cpu_count() or 1
    T, S = sc.layout.num_taxels, inp.link_state.shape[0]
    v, n, dt = _oracle_rate(sc, inp, "f32", threads, target_s, max(threads, 8))
    v64, n64, dt64 = _oracle_rate(sc, inp, "f64", threads, target_s / 2, max(threads, 8))
    v1, n1, dt1 = _oracle_rate(sc, inp, "f32", 1, target_s / 3, 2)
    return {"value": v, "unit": "taxel-readouts/s", "cores": threads, "kind": "oracle",
            "sample": f"{n} of {sc.num_envs} envs x {T} taxels x {S} steps ({dt:.1f} s, FP32 oracle)",
            "fp64": {"value": v64, "cores": threads,
                     "sample": f"{n64} envs x {T} taxels x {S} steps ({dt64:.1f} s, FP64 oracle)"},
            "one_thread": {"value": v1, "cores": 1,
                           "sample": f"{n1} envs x {T} taxels x {S} steps ({dt1:.1f} s, FP32 oracle)"}}


def fp64_error(sc, inp, out, envs):
    """Error of the GPU rollout (fresh state at step 0) against the FP64 oracle on sampled envs:
    contact-bit disagreement, depth and proximity absolute error, and per-3-vector relative error
    of the clean and noisy force/torque (the noisy channel carries the BF16 crosstalk)."""
    import oracle
    from paper_2606_22332_amd import synth
    L = sc.layout.num_links
    ref = oracle.run_readout(sc, synth.subset_envs(inp, envs, L), envs=envs, precision="f64")
    W = out["bits"].shape[-1]
    res = {"envs": [int(e) for e in envs], "steps": int(inp.link_state.shape[0])}

    def bits(words):
        b = np.unpackbits(words.view(np.uint8).reshape(*words.shape[:-1], W * 8), axis=-1, bitorder="little")
        return b[..., :sc.layout.num_taxels]

    def rel3(g, r, floor):
        # per 3-vector: |g - r|_inf / max(|r|_inf, floor), over vectors with |r|_inf > 1e-6
        g = np.moveaxis(g.astype(np.float64), 1, -1).reshape(*g.shape[:1], g.shape[2], g.shape[3], 2, 3)
        r = np.moveaxis(r, 1, -1).reshape(g.shape)
        num = np.abs(g - r).max(-1)
        den = np.abs(r).max(-1)
        m = den > 1e-6
        q = num[m] / np.maximum(den[m], floor)
        return {"p99": float(np.quantile(q, 0.99)) if q.size else 0.0, "max": float(q.max()) if q.size else 0.0,
                "abs_max": float(num.max()), "floor": floor}

    res["bit_mismatch_fraction"] = float((bits(out["bits"]) != ref["bit"]).mean())
    res["depth_max_abs_m"] = float(np.abs(out["depth"].astype(np.float64) - ref["depth"]).max())
    res["prox_max_abs"] = float(np.abs(out["prox"].astype(np.float64) - ref["prox"]).max())
    res["ft_rel"] = rel3(out["ft"], ref["ft"], 1e-6)
    if "ft_noisy" in out:
        res["bit_noisy_mismatch_fraction"] = float((bits(out["bits_noisy"]) != ref["bit_noisy"]).mean())
        # floor: one step of drift (the noisy channel's own scale), so near-zero sums of crosstalk
        # and drift do not read as large relative errors
        res["ft_noisy_rel"] = rel3(out["ft_noisy"], ref["ft_noisy"], float(sc.noise.drift_sigma))
    return res


def copy_calibration(nbytes: int) -> None:
    """A plain device-to-device copy of known size: its FETCH_SIZE / WRITE_SIZE counters give the
    factor that turns those counters into bytes for the readout kernel."""
    import torch
    n = nbytes // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": n * 4, "copies": 3}), flush=True)


# Sources that define the readout kernel and its launch plan: HBM counters taken on another
# version of them no longer describe the kernel that runs.
KERNEL_SOURCES = ["readout_device.h", "readout_kernel.h", "link_kernel.h", "xtalk_dense.h", "tg_readout.hip"]
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "tg_link_kernel_c3_hbm_counters.txt")


def copy_bandwidth(nbytes: int = 1 << 31, reps: int = 5) -> float:
    """Achievable HBM bandwidth on this GPU (GB/s): a device-to-device copy of `nbytes`, counted
    as read + write, best of `reps` after a warm-up."""
    import torch
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1))
    del a, b
    torch.cuda.empty_cache()
    return 2.0 * nbytes / (best * 1e-3) / 1e9


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2606_22332_amd", "csrc", f), "rb") as fh:
            h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()


def measured_traffic(workload_key: str):
    """HBM bytes per launch of the readout kernel from the committed counter summary: FETCH_SIZE
    and WRITE_SIZE (KiB per dispatch), each scaled by what the same counter reads for a plain copy
    of known size.  None when there is no summary for this workload or the kernel sources have
    changed since the counters were taken."""
    if not os.path.exists(TRAFFIC_PROFILE):
        return None
    kv = {}
    with open(TRAFFIC_PROFILE) as fh:
        for line in fh:
            if ":" in line and not line.startswith(("#", "|", " ")):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    try:
        if kv["source_sha256"] != kernel_source_hash() or kv["workload_key"] != workload_key:
            return None
        cb = float(kv["copy_bytes"])
        f_fetch = cb / (float(kv["copy_fetch_kib"]) * 1024.0)
        f_write = cb / (float(kv["copy_write_kib"]) * 1024.0)
        return (float(kv["fetch_kib_per_dispatch"]) * 1024.0 * f_fetch
                + float(kv["write_kib_per_dispatch"]) * 1024.0 * f_write)
    except (KeyError, ValueError, ZeroDivisionError):
        return None


def angle_deg(a, b):
    a = np.asarray(a, np.float64); b = np.asarray(b, np.float64)
    return np.degrees(np.arctan2(np.linalg.norm(np.cross(a, b), axis=-1), np.sum(a * b, axis=-1)))


def bench_c4(args) -> dict:
    """Neural-SDF readout against the grid readout on the 256-object hand workload: trains the
    per-object networks on the GPU, then times 16-step clean rollouts on both SDF backends and
    reports the neural path's depth and normal error against the grid path."""
    import torch
    from paper_2606_22332_amd import binding as B
    from paper_2606_22332_amd import synth
    t0 = time.perf_counter()
    sc = synth.make_scene("c4", num_envs=args.envs)
    sc.noise = synth.NoiseParams(enabled=False, seed=sc.noise.seed)
    inp = synth.make_inputs(sc)
    E, L, T, S = sc.num_envs, sc.layout.num_links, sc.layout.num_taxels, inp.link_state.shape[0]
    n_obj = len(sc.grids)
    if args.pair_lambda > 0:   # half the records as recipe points, each with a partner delta away
        pts = synth.nsdf_pairs(synth.nsdf_points(sc.grids, args.nsdf_samples // 2, seed=sc.geom_seed + 7),
                               args.pair_delta, seed=sc.geom_seed + 10)
    else:
        pts = synth.nsdf_points(sc.grids, args.nsdf_samples, seed=sc.geom_seed + 7)
    gen_s = time.perf_counter() - t0
    ns = B.Nsdf(sc.grids)
    grec = None
    if args.grad_lambda > 0:   # gradient records: the grid's gradient, target of the gradient term
        rec, grec = ns.targets(torch.from_numpy(pts).cuda(), grad=True)
    else:
        rec = ns.targets(torch.from_numpy(pts).cuda())
    del pts
    P = torch.from_numpy(synth.nsdf_init(n_obj, sc.geom_seed + 8)).cuda()
    m, v = torch.zeros_like(P), torch.zeros_like(P)
    hp = B.train_params(lr=1e-3, batch=1 << 14, seed=sc.geom_seed + 9, pair_lambda=args.pair_lambda,
                        grad_lambda=args.grad_lambda)
    loss = torch.zeros((args.train_steps, n_obj), device="cuda")
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    if args.lr_schedule == "cosine":
        # Adam from lr 1e-3, decayed along a half cosine to 1e-5 over the run (in 20 constant
        # pieces; the step counter, hence bias correction and minibatch draws, runs on)
        pieces = 20
        edges = np.linspace(0, args.train_steps, pieces + 1).astype(int)
        for i in range(pieces):
            n_i = int(edges[i + 1] - edges[i])
            if n_i <= 0:
                continue
            lr_i = 1e-5 + 0.5 * (1e-3 - 1e-5) * (1.0 + np.cos(np.pi * (i + 0.5) / pieces))
            hp_i = B.train_params(lr=float(lr_i), batch=1 << 14, seed=sc.geom_seed + 9, pair_lambda=args.pair_lambda,
                                  grad_lambda=args.grad_lambda)
            ns.train(P, m, v, rec, int(edges[i]), n_i, hp_i, loss=loss[int(edges[i]):int(edges[i + 1])],
                     grad_samples=grec)
    else:
        ns.train(P, m, v, rec, 0, args.train_steps, hp, loss=loss, grad_samples=grec)
    b.record()
    torch.cuda.synchronize()
    train_ms = a.elapsed_time(b)
    final_loss = loss[-50:].mean(0)
    half = torch.tensor([0.5 * (g.n - 1) * float(g.spacing) for g in sc.grids], device="cuda")
    loss_um = (final_loss * half * 1e6).cpu().numpy()
    ns.close()
    del rec, grec
    mask = (B.TG_OUT_BITS | B.TG_OUT_DEPTH | B.TG_OUT_PROX | B.TG_OUT_FT | B.TG_OUT_NORMAL | B.TG_OUT_LINK_SUMS
            | B.TG_OUT_SURFDIST)
    d = B.to_device(inp)
    res, outs = {}, {}
    for name, kw in (("grid", {}), ("neural", {"nsdf_params": P, "nsdf_band": 1e-3})):
        ro = B.Readout(sc, mask, **kw)
        ro.alloc_outputs(S)
        ro.rollout(d, S)
        torch.cuda.synchronize()
        ts = []
        for _ in range(args.steps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            ro.rollout(d, S)
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        res[name] = float(np.median(ts))
        outs[name] = {k: ro.out[k] for k in ("depth", "normal", "surfdist")}
        ro.out = {}
        ro.close()
    # error of the neural path against the grid path over taxels in contact on the grid path
    dg, dn = outs["grid"]["depth"], outs["neural"]["depth"]
    c = dg > 0
    derr = (dn - dg).abs()[c].float().cpu().numpy()
    ng = outs["grid"]["normal"].permute(0, 2, 3, 1)[c].cpu().numpy()
    nn_ = outs["neural"]["normal"].permute(0, 2, 3, 1)[c].cpu().numpy()
    both = (np.linalg.norm(nn_, axis=-1) > 0)
    ang = angle_deg(nn_[both], ng[both])
    # the network supplies the normal only where |phi_nn| >= band, i.e. for a contact (phi < R_j)
    # about where the probe is more than R_j + band deep; split the error there
    deep = (dg[c].float().cpu().numpy() >= 2e-3)[both]
    # the network supplied phi (and, in contact, the normal) where its surface distance differs
    # from the grid path's
    net = (outs["neural"]["surfdist"] != outs["grid"]["surfdist"])[c].cpu().numpy()[both]
    def q99(a):
        return float(np.quantile(a, 0.99)) if a.size else 0.0
    readouts = E * T * S
    return {
        "metric": METRIC, "value": readouts / (res["neural"] * 1e-3), "unit": "taxel-readouts/s", "n_gpus": 1,
        "steps": args.steps, "warmup": 1, "ms_per_step": res["neural"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "bf16-mfma/f32", "data": "synthetic",
        "config": {"workload": f"c4: {E} envs x {T} taxels ({L} links) x {S}-step clean rollout, {n_obj} objects, "
                               "neural SDF (PE48-4x64 SiLU-1, BF16 MFMA) with grid fallback |phi|<1 mm",
                   "envs": E, "taxels": T, "objects": n_obj, "steps_per_rollout": S},
        "grid_path": {"ms_per_rollout": res["grid"], "readouts_per_s": readouts / (res["grid"] * 1e-3)},
        "speedup_vs_grid": res["grid"] / res["neural"],
        "depth_err_um": {"p50": float(np.quantile(derr, 0.5) * 1e6), "p99": float(np.quantile(derr, 0.99) * 1e6),
                         "max": float(derr.max() * 1e6), "contacts": int(c.sum().item())},
        "normal_err_deg": {"p50": float(np.quantile(ang, 0.5)), "p99": float(np.quantile(ang, 0.99)),
                           "max": float(ang.max()), "p99_depth_below_2mm": q99(ang[~deep]),
                           "p99_depth_2mm_or_more": q99(ang[deep]), "fraction_2mm_or_more": float(deep.mean()),
                           "network_supplied": {"fraction": float(net.mean()),
                                                "p50": float(np.quantile(ang[net], 0.5)) if net.any() else 0.0,
                                                "p90": float(np.quantile(ang[net], 0.9)) if net.any() else 0.0,
                                                "p99": q99(ang[net])}},
        "training": {"steps": args.train_steps, "batch_per_object": 1 << 14, "samples_per_object": args.nsdf_samples,
                     "lr_schedule": args.lr_schedule, "pair_lambda": args.pair_lambda,
                     "grad_lambda": args.grad_lambda,
                     "pair_delta_m": args.pair_delta if args.pair_lambda > 0 else None,
                     "ms_total": train_ms, "ms_per_step": train_ms / args.train_steps,
                     "final_l1_um_median": float(np.median(loss_um)), "final_l1_um_max": float(loss_um.max())},
        "memory_MB": {"grids_fp32": n_obj * sc.grids[0].n ** 3 * 4 / 1e6,
                      "network_bf16": n_obj * 15681 * 2 / 1e6,
                      "network_images": n_obj * 65024 / 1e6},
        "input_gen_s": gen_s,
    }


def bench_c2_step(reps: int = 3) -> dict:
    """The per-step entry point on the 4096-env x 200-taxel noisy hand (16 links, banded
    crosstalk): 100 consecutive tg_readout_step calls, each one launch that reads and writes the
    noise state, timed with HIP events on the stream they run on (median per step over `reps`
    runs of 100 steps), beside the same 100 steps as one rollout launch."""
    import torch
    from paper_2606_22332_amd import binding as B
    from paper_2606_22332_amd import synth
    sc = synth.make_scene("c2")
    inp = synth.make_inputs(sc)
    E, L, T, S = sc.num_envs, sc.layout.num_links, sc.layout.num_taxels, inp.link_state.shape[0]
    mask = B.TG_OUT_BITS | B.TG_OUT_DEPTH | B.TG_OUT_PROX | B.TG_OUT_FT | B.TG_OUT_LINK_SUMS | B.TG_OUT_NOISY
    ro = B.Readout(sc, mask)
    d = B.to_device(inp)
    ro.alloc_outputs(S)
    stream = torch.cuda.current_stream()
    for s_ in range(S):          # warm-up (graph recorded, then updated per call)
        ro.step(d, s_)
    torch.cuda.synchronize()
    per_step, walls = [], []
    for _ in range(reps):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(S + 1)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev[0].record(stream)
        for s_ in range(S):
            ro.step(d, s_)
            ev[s_ + 1].record(stream)
        torch.cuda.synchronize()
        walls.append((time.perf_counter() - t0) / S * 1e3)
        per_step += [ev[i].elapsed_time(ev[i + 1]) for i in range(S)]
    ro.reset(None, 0)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ro.rollout(d, S)
    e0.record(stream)
    ro.rollout(d, S)
    e1.record(stream)
    torch.cuda.synchronize()
    roll_ms = e0.elapsed_time(e1)
    ro.close()
    ms = float(np.median(per_step))
    nbytes, _ = algorithmic_bytes(E, L, T, 1, len(sc.grids), sc.grids[0].n, True, True)
    return {"workload": f"c2: {E} envs x {T} taxels ({L} links), noisy, banded crosstalk; per-step tg_readout_step",
            "ms_per_step_median": ms, "ms_per_step_min": float(np.min(per_step)),
            "host_wall_ms_per_step": float(np.median(walls)), "readouts_per_s": E * T / (ms * 1e-3),
            "algorithmic_bytes_per_step": nbytes, "hbm_frac": nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "rollout_ms_per_step": roll_ms / S}


def bench_prox(reps: int = 5) -> dict:
    """The ProximityTaxel readout (App. A.6) on the 4096-env x 200-taxel hand: 8 objects, each
    tracked by 5000 area-uniform surface points, sensing radius 1 cm, k = 300, k_s = 10,
    density 100; one 100-step launch timed with HIP events (median of `reps`), with the error of
    sampled envs against the FP64 oracle."""
    import torch
    from paper_2606_22332_amd import binding as B
    from paper_2606_22332_amd import synth
    sc = synth.make_scene("c2")
    inp = synth.make_inputs(sc)
    clouds = synth.surface_clouds(sc.grids, 5000, seed=sc.geom_seed + 20)
    E, T, S = sc.num_envs, sc.layout.num_taxels, inp.link_state.shape[0]
    px = B.Proximity(sc, clouds)
    d = B.to_device(inp)
    stream = torch.cuda.current_stream()
    ft, mass = px.rollout(d)
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        px.rollout(d, ft=ft, want_mass=False)
        e1.record(stream)
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    ms = float(np.median(ts))
    res = {"workload": f"c2 hand: {E} envs x {T} taxels x {S} steps, ProximityTaxel, 8 objects x 5000 surface "
                       "points, R = 1 cm", "ms_per_rollout": ms, "readouts_per_s": E * T * S / (ms * 1e-3),
           "in_range_fraction": float((mass > 0).float().mean().item()),
           "mean_penetration_sum_m": float(mass[mass > 0].mean().item())}
    try:
        import oracle
        envs = np.array([0, E // 2, E - 1])
        idx = torch.as_tensor(envs, device="cuda")
        g = ft[:, :, idx].cpu().numpy()
        sub = synth.subset_envs(inp, envs, sc.layout.num_links)
        r, m = oracle.prox_run(sc.layout.link_offset, sc.layout.pos, sc.layout.normal,
                               np.full(T, 0.01, np.float32), clouds, sub.link_state, sub.obj_id, sub.obj_state,
                               sub.step0)
        scale = np.maximum(np.abs(r).max(1, keepdims=True), 1e-9)
        res["fp64_error"] = {"envs": envs.tolist(), "max_rel_to_channel_max": float((np.abs(g - r) / scale).max())}
    except ImportError:
        pass
    px.close()
    return res


FP64_VECTOR_PEAK_TFLOPS = 78.6


def bench_audio(reps: int = 5, lanes_per_pair: int = 0) -> dict:
    """The contact-audio sensor (App. E) on the hand's 5 fingertip links (4096 envs): the clean
    100-step readout of the 4096-env x 200-taxel hand supplies taxel forces and contact normals;
    each (env, fingertip) synthesises K = 240 samples per 5 ms step (48 kHz) through a 16-mode
    plate bank of the env's object's material (wood, metal, glass).  The audio launch alone is
    timed with HIP events (median of `reps`); the roofline is FP64 FMA issue: 6 flops per mode and
    sample (two FMAs of the recurrence, one of the output sum)."""
    import torch
    from paper_2606_22332_amd import binding as B
    from paper_2606_22332_amd import synth
    sc = synth.make_scene("c2")
    inp = synth.make_inputs(sc)
    lay = sc.layout
    E, T, S, K = sc.num_envs, lay.num_taxels, inp.link_state.shape[0], 240
    links = (1, 2, 3, 4, 5)
    ranges = [(int(lay.link_offset[l]), int(lay.link_offset[l + 1])) for l in links]
    ro = B.Readout(sc, B.TG_OUT_FT | B.TG_OUT_NORMAL)
    d = B.to_device(inp)
    ro.alloc_outputs(S)
    ro.rollout(d, S)
    ft, nm = ro.out["ft"], ro.out["normal"]
    mats = synth.audio_materials(16, K / sc.dt)
    material = (np.asarray(inp.obj_id[0]) % 3).astype(np.int32)
    dmat = torch.from_numpy(material).cuda()
    au = B.Audio(E, T, ranges, mats, 16, K, sc.dt, g_imp=1.0, g_scr=1.0, seed=sc.noise.seed,
                 lanes_per_pair=lanes_per_pair)
    stream = torch.cuda.current_stream()
    out = au.rollout(ft, nm, dmat)
    torch.cuda.synchronize()
    first = out.clone()
    ts = []
    for _ in range(reps):
        au.reset()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        au.rollout(ft, nm, dmat, out=out)
        e1.record(stream)
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    ms = float(np.median(ts))
    Ls = len(links)
    samples = E * Ls * K * S
    modes = np.array([len(m[0]) for m in mats])[material]
    flops = 6.0 * float(modes.sum()) * Ls * K * S
    sensor_taxels = sum(b - a for a, b in ranges)
    hbm = S * E * (sensor_taxels * 6 * 4 + Ls * K * 4)
    res = {"workload": f"c2 hand: {E} envs x {Ls} fingertip links ({sensor_taxels} taxels) x {S} steps, K = {K} "
                       f"samples per {sc.dt * 1e3:.0f} ms step (48 kHz), 16-mode banks (wood, metal, glass), "
                       "excited by the clean readout's forces and normals",
           "ms_per_rollout": ms, "samples_per_s": samples / (ms * 1e-3), "dtype": "f64 (FP32 output)",
           "roofline": {"bound": "alu", "achieved": flops / (ms * 1e-3) / 1e12, "peak": FP64_VECTOR_PEAK_TFLOPS,
                        "unit": "TFLOP/s", "frac": flops / (ms * 1e-3) / 1e12 / FP64_VECTOR_PEAK_TFLOPS,
                        "flops_per_launch": flops, "hbm_gbs": hbm / (ms * 1e-3) / 1e9,
                        "kernel": "tg_audio_kernel"},
           "repeatable_after_reset": bool(torch.equal(first, out)),
           "active_fraction": float((out.abs().amax(dim=3) > 0).float().mean().item())}
    try:
        from oracle import audio as OA
        envs = np.array([0, E - 1])
        idx = torch.as_tensor(envs, device="cuda")
        fts = ft[:, :, idx].cpu().numpy()
        nms = nm[:, :, idx].cpu().numpy()
        Fn = np.zeros((S, len(envs), Ls))
        Ft = np.zeros_like(Fn)
        for li, (a, b) in enumerate(ranges):
            n_, t_ = OA.link_excitation(fts, nms, [a, b], [0])
            Fn[:, :, li], Ft[:, :, li] = n_[:, :, 0], t_[:, :, 0]
        ref = OA.contact_audio(Fn, Ft, material[envs], mats, 16, sc.dt, K, 1.0, 1.0, sc.noise.seed, env_ids=envs)
        g = first[:, idx].cpu().numpy().astype(np.float64)
        scale = np.abs(ref).max(axis=(0, 3), keepdims=True)
        tol = 2.0 ** -24 * np.abs(ref) + 1e-9 * scale + 1e-30
        res["fp64_check"] = {"envs": envs.tolist(), "max_err_over_bar": float((np.abs(g - ref) / tol).max()),
                             "fp32_equal_fraction": float(np.mean(g == ref.astype(np.float32).astype(np.float64)))}
    except ImportError:
        pass
    au.close()
    ro.out = {}
    ro.close()
    return res


def bench_elastomer(reps: int = 5) -> dict:
    """The ElastomerTaxel (App. A.7) on the hand's 5 fingertip pads (4096 envs x 100 steps): the
    clean readout supplies the source probes' depths; each object carries a 1000-point surface
    cloud for the shear anchors.  The elastomer launch alone is timed with HIP events (median of
    `reps`, anchors reset before each).  Work is counted in terms: marker x active source (dilation),
    marker x anchored contact point (shear), and one pose / SDF / anchor update per tracked point."""
    import torch
    from paper_2606_22332_amd import binding as B
    from paper_2606_22332_amd import synth
    sc = synth.make_scene("c2")
    inp = synth.make_inputs(sc)
    lay = sc.layout
    E, T, S = sc.num_envs, lay.num_taxels, inp.link_state.shape[0]
    links = [1, 2, 3, 4, 5]
    clouds = synth.surface_clouds(sc.grids, 1000, seed=sc.geom_seed + 30)
    pc, ph = synth.elastomer_pads(lay, links)
    ro = B.Readout(sc, B.TG_OUT_DEPTH)
    d = B.to_device(inp)
    ro.alloc_outputs(S)
    ro.rollout(d, S)
    depth = ro.out["depth"]
    el = B.Elastomer(sc, clouds, links, pc, ph)
    disp = el.rollout(d, depth)
    torch.cuda.synchronize()
    first = disp.clone()
    stream = torch.cuda.current_stream()
    ts = []
    for _ in range(reps):
        el.reset()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        el.rollout(d, depth, disp=disp)
        e1.record(stream)
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    ms = float(np.median(ts))
    markers = sum(int(lay.link_offset[l + 1] - lay.link_offset[l]) for l in links)
    res = {"workload": f"c2 hand: {E} envs x {len(links)} fingertip pads ({markers} markers) x {S} steps, "
                       "1000-point surface clouds, App. A.7 constants (c = 1, no clamped boundary)",
           "ms_per_rollout": ms, "marker_readouts_per_s": E * markers * S / (ms * 1e-3),
           "repeatable_after_reset": bool(torch.equal(first, disp))}
    try:
        import oracle
        envs = np.array([0, E // 2, E - 1])
        idx = torch.as_tensor(envs, device="cuda")
        g = first[:, :, idx].cpu().numpy().astype(np.float64)
        sub = synth.subset_envs(inp, envs, lay.num_links)
        dep = depth[:, idx].cpu().numpy()
        ref, absum, st = oracle.elastomer_run(lay.link_offset, lay.pos, lay.normal, lay.radius, links, pc, ph, clouds,
                                              sub.link_state, sub.obj_id, sub.obj_state, dep)
        m = np.zeros(T, bool)
        for l in links:
            m[lay.link_offset[l]:lay.link_offset[l + 1]] = True
        err = np.abs(g - ref)[..., m].max(axis=1)
        res["fp64_check"] = {"envs": envs.tolist(),
                             "max_err_over_bar": float((err / (1e-5 * absum[..., m] + 1e-12)).max()),
                             "anchored_points_at_end": int(st["active"].sum())}
    except ImportError:
        pass
    el.close()
    ro.out = {}
    ro.close()
    return res


def bench_raycast(reps: int = 5) -> dict:
    """The raycast contact-depth backend (App. A.1) on the hand (4096 envs x 200 taxels x 100 steps)
    over the 8 objects' triangle meshes (icospheres, boxes, capsules, tori, convex hulls; 12 to 2304
    triangles), one launch per rollout timed with HIP events (median of `reps`), beside the grid
    backend's depth-only rollout of the same steps; sampled envs against the FP64 brute force."""
    import torch
    from paper_2606_22332_amd import binding as B
    from paper_2606_22332_amd import synth
    sc = synth.make_scene("c2")
    inp = synth.make_inputs(sc)
    E, T, S = sc.num_envs, sc.layout.num_taxels, inp.link_state.shape[0]
    meshes = synth.object_meshes(sc.grids)
    rc = B.Raycast(sc, meshes)
    d = B.to_device(inp)
    dep, nm, tri = rc.rollout(d)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    def timed(fn):
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            fn()
            e1.record(stream)
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        return float(np.median(ts))
    ms = timed(lambda: rc.rollout(d, depth=dep, normal=nm, tri=tri))
    ro = B.Readout(sc, B.TG_OUT_DEPTH)
    ro.set_work_plan(512)
    ro.alloc_outputs(S)
    ro.rollout(d, S)
    torch.cuda.synchronize()
    ms_grid = timed(lambda: ro.rollout(d, S))
    gdep = ro.out["depth"]
    both = (dep > 0) & (gdep > 0)
    res = {"workload": f"c2 hand: {E} envs x {T} taxels x {S} steps, raycast depth over BVHs of "
                       f"{sum(len(m[1]) for m in meshes)} triangles (8 objects)",
           "ms_per_rollout": ms, "readouts_per_s": E * T * S / (ms * 1e-3),
           "grid_backend_depth_only_ms": ms_grid,
           "contact_fraction": float((dep > 0).float().mean().item()),
           "vs_grid_depth_um": {"p50": float((dep - gdep)[both].abs().median().item() * 1e6),
                                "p99": float(torch.quantile((dep - gdep)[both].abs()[:1 << 20].float(), 0.99).item() * 1e6)}}
    try:
        import oracle
        envs = np.array([0, E // 2, E - 1])
        idx = torch.as_tensor(envs, device="cuda")
        sub = synth.subset_envs(inp, envs, sc.layout.num_links)
        lay = sc.layout
        rd, _, _ = oracle.raycast_run(lay.link_offset, lay.pos, lay.normal, lay.radius, meshes, sub.link_state,
                                      sub.obj_id, sub.obj_state)
        res["fp64_check"] = {"envs": envs.tolist(),
                             "max_depth_err_um": float(np.abs(dep[:, idx].cpu().numpy() - rd).max() * 1e6)}
    except ImportError:
        pass
    rc.close()
    ro.out = {}
    ro.close()
    return res


def c4_summary(r: dict) -> dict:
    """The grid-vs-neural comparison of bench_c4, without the fields of a bench line."""
    keep = ("config", "grid_path", "speedup_vs_grid", "depth_err_um", "normal_err_deg", "training", "memory_MB")
    out = {k: r[k] for k in keep}
    out["neural_path"] = {"ms_per_rollout": r["ms_per_step"], "readouts_per_s": r["value"]}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="c3")
    ap.add_argument("--envs", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--readouts-per-block", type=int, default=0,
                    help="fix the work plan instead of autotuning (the profiles pin the autotuner's choice)")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--workload", default="readout", choices=["readout", "c4", "proximity", "audio", "elastomer", "raycast"])
    ap.add_argument("--train-steps", type=int, default=5000)
    ap.add_argument("--nsdf-samples", type=int, default=1 << 17)
    ap.add_argument("--lr-schedule", default="constant", choices=["constant", "cosine"])
    ap.add_argument("--pair-lambda", type=float, default=0.0,
                    help="weight of the pair term of the training loss (0: the plain L1 recipe)")
    ap.add_argument("--pair-delta", type=float, default=5e-4, help="distance between the points of a pair [m]")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the per-step C2 timing and the C4 grid-vs-neural comparison in the readout run")
    ap.add_argument("--grad-lambda", type=float, default=None,
                    help="weight of the L1 term on the network's input gradient against the grid's (0: off)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES")
    ap.add_argument("--thermal-solver", type=int, default=0, choices=[0, 1],
                    help="c5 only: 0 the explicit stencil, 1 the spectral step with T^4 radiation (App. D.1)")
    ap.add_argument("--h-conv", type=float, default=0.0, help="c5, solver 1: convection coefficient [W/m^2K]")
    ap.add_argument("--lag-tau", type=float, default=0.0, help="c5, solver 1: sensor element lag [s] (0: off)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(environments shard across GPUs with no exchange; see the design notes)", file=sys.stderr)
        sys.exit(2)

    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.grad_lambda is None:
        args.grad_lambda = DEFAULT_GRAD_LAMBDA
    if args.workload == "c4":
        print(json.dumps(bench_c4(args)), flush=True)
        return
    if args.workload == "proximity":
        print(json.dumps(bench_prox()), flush=True)
        return
    if args.workload == "audio":
        print(json.dumps(bench_audio()), flush=True)
        return
    if args.workload == "elastomer":
        print(json.dumps(bench_elastomer()), flush=True)
        return
    if args.workload == "raycast":
        print(json.dumps(bench_raycast()), flush=True)
        return

    import torch
    from paper_2606_22332_amd import binding as B
    from paper_2606_22332_amd import synth

    sc = synth.make_scene(args.config, num_envs=args.envs)
    if sc.thermal is not None and args.thermal_solver:
        sc.thermal.solver, sc.thermal.h_conv, sc.thermal.lag_tau = 1, args.h_conv, args.lag_tau
    t0 = time.perf_counter()
    inp = synth.make_inputs(sc)
    gen_s = time.perf_counter() - t0
    E, L, T, S = sc.num_envs, sc.layout.num_links, sc.layout.num_taxels, inp.link_state.shape[0]
    mask = B.TG_OUT_BITS | B.TG_OUT_DEPTH | B.TG_OUT_PROX | B.TG_OUT_FT | B.TG_OUT_LINK_SUMS
    if sc.noise.enabled:
        mask |= B.TG_OUT_NOISY
    ro = B.Readout(sc, mask)
    if args.no_graph:
        ro.set_graph(False)
    dinp = B.to_device(inp)
    ro.alloc_outputs(S)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    tuned = None
    if args.readouts_per_block:
        ro.set_work_plan(args.readouts_per_block)
    elif not args.no_autotune:
        tuned = ro.autotune(dinp, S)

    # rollouts continue one another (the step counter advances by S each time), as in a long
    # simulation; the noise state carries over on the device
    step = 0
    for _ in range(args.warmup):
        dinp.step0 = step
        ro.rollout(dinp, S)
        step += S
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    for i in range(args.steps):
        dinp.step0 = step
        ev[i][0].record(stream)
        ro.rollout(dinp, S)
        ev[i][1].record(stream)
        step += S
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_wall
    kernel_ms = [a.elapsed_time(b) for a, b in ev]
    ms = float(np.mean(kernel_ms))
    readouts = E * T * S
    value = readouts / (wall / args.steps)
    nbytes, _ = algorithmic_bytes(E, L, T, S, len(sc.grids), sc.grids[0].n, sc.noise.enabled, True)
    achieved = nbytes / (ms * 1e-3) / 1e9
    copy_gbs = copy_bandwidth()            # after the timed region
    eb, threads = ro.launch_shape()
    wkey = f"{sc.name}:E{E}:T{T}:S{S}:target{eb}:threads{threads}"
    rec = {
        "metric": METRIC, "value": value, "unit": "taxel-readouts/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": wall / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{sc.name}: {E} envs x {T} taxels ({L} links) x {S}-step rollout, grid SDF "
                               f"({len(sc.grids)} objects, {sc.grids[0].n}^3), "
                               + ("noisy, " + {0: "no", 1: "banded", 2: "dense BF16-MFMA"}[sc.noise.xtalk_kind]
                                  + " crosstalk" if sc.noise.enabled else "clean")
                               + ("" if sc.thermal is None else
                                  ", TemperatureGrid " + ("spectral" if sc.thermal.solver == 1 else "explicit")
                                  + f" on {len(sc.thermal.field_links)} links"),
                   "envs": E, "taxels": T, "links": L, "steps_per_rollout": S,
                   "readouts_per_block_target": eb, "threads_per_block": threads,
                   "autotuned": tuned is not None, "graph": not args.no_graph},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(wkey),
                     "kernel": "tg_link_kernel", "algorithmic_bytes_per_launch": nbytes,
                     "bytes_per_readout": nbytes / readouts, "kernel_ms_mean": ms,
                     "kernel_ms_min": float(np.min(kernel_ms)), "workload_key": wkey,
                     "kernel_source_sha256": kernel_source_hash(),
                     "copy_gbs": copy_gbs, "frac_of_copy": achieved / copy_gbs},
        "input_gen_s": gen_s,
    }
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(sc, inp)
        # error against the FP64 oracle: one more rollout from a fresh state at step 0, sampled envs
        ro.reset(None, 0)
        dinp.step0 = 0
        ro.rollout(dinp, S)
        torch.cuda.synchronize()
        envs = np.unique(np.array([0, E // 3, (2 * E) // 3, E - 1]))
        idx = torch.as_tensor(envs, device="cuda")
        sub = {k: (v[:, idx] if v.ndim == 3 else v[:, :, idx]).cpu().numpy() for k, v in ro.out.items()}
        rec["fp64_error"] = fp64_error(sc, inp, sub, envs)
    ro.out = {}
    ro.close()
    del dinp
    torch.cuda.empty_cache()
    if not args.no_extra and args.config == "c3" and args.envs is None:
        # the other two lines of the metric: the per-step entry point (C2) and the neural SDF
        # against the grid (C4: 256 objects, networks trained here on the GPU)
        rec["c2_step"] = bench_c2_step()
        torch.cuda.empty_cache()
        rec["proximity"] = bench_prox()
        torch.cuda.empty_cache()
        rec["contact_audio"] = bench_audio()
        torch.cuda.empty_cache()
        rec["elastomer"] = bench_elastomer()
        torch.cuda.empty_cache()
        rec["raycast"] = bench_raycast()
        torch.cuda.empty_cache()
        a4 = argparse.Namespace(**vars(args))
        a4.envs, a4.steps = None, 5
        rec["c4_grid_vs_neural"] = c4_summary(bench_c4(a4))
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
