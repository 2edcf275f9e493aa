"""Neural-SDF kernels (include/tg_nsdf.h) against the CPU oracle, through the C ABI.

Inputs: seeded He-uniform weights and sample points from the scene generator; training
records (x_hat, phi/e) come from the oracle's FP64 grid interpolation, never from the GPU.
Bars: training targets within FP32 rounding of the FP64 records; network output within 20 um
(phi = e * out) of the BF16-emulating oracle and its input gradient within 0.1 deg; the loss
gradient within 1e-2 (norm-wise per layer) of FP64 backprop and tighter against the
BF16-emulating backprop; Adam within FP32 rounding of the FP64 update.

Both sides round the same operands to BF16, but the values rounded differ in their last FP32
bits (FP32 MFMA sums and hardware sin/cos against FP64): where a value sits that close to a BF16
rounding tie the two round apart by one BF16 ulp (2^-8 relative), and that step travels through
the rest of the network.  Such points are rare, so the per-point bars are quantiles with a
bounded maximum: phi p99.9 <= 20 um (max 200 um), gradient angle p99 <= 0.1 deg (max 1 deg).
"""
import math

import numpy as np
import pytest

import oracle
from paper_2606_22332_amd import synth

pytestmark = pytest.mark.gpu

NP = 15681
LAYERS = {"W1": (0, 3072), "b1": (3072, 3136), "W2": (3136, 7232), "b2": (7232, 7296), "W3": (7296, 11392),
          "b3": (11392, 11456), "W4": (11456, 15552), "b4": (15552, 15616), "w5": (15616, 15680),
          "b5": (15680, 15681)}


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def grids():
    return synth.make_scene("c2", num_envs=4, num_steps=2).grids


def half_extent(g):
    return 0.5 * (g.n - 1) * float(g.spacing)


def init_params(n_obj, seed, bias_sigma=0.1):
    P = synth.nsdf_init(n_obj, seed).astype(np.float64)
    rng = np.random.default_rng(seed + 1)
    for name in ("b1", "b2", "b3", "b4", "b5"):
        a, b = LAYERS[name]
        P[:, a:b] = rng.normal(0, bias_sigma, (n_obj, b - a))
    return P.astype(np.float32)


def records(grids, n, seed):
    pts = synth.nsdf_points(grids, n, seed)
    return np.stack([oracle.nsdf_targets(g, p) for g, p in zip(grids, pts)]).astype(np.float32)


def test_targets_match_oracle(torch_cuda, grids):
    torch = torch_cuda
    from paper_2606_22332_amd import binding as B
    n = 1000
    pts = synth.nsdf_points(grids, n, 11)
    rng = np.random.default_rng(12)
    for o, g in enumerate(grids):            # some points outside the box exercise the clamp
        lo = g.origin.astype(np.float64); hi = lo + (g.n - 1) * float(g.spacing)
        pts[o, :40] = rng.uniform(lo - 0.01, hi + 0.01, (40, 3))
    ns = B.Nsdf(grids)
    rec, grec = ns.targets(torch.from_numpy(pts).cuda(), grad=True)
    rec2 = ns.targets(torch.from_numpy(pts).cuda())
    rec, grec, rec2 = rec.cpu().numpy(), grec.cpu().numpy(), rec2.cpu().numpy()
    ns.close()
    assert np.array_equal(rec, rec2)
    for o, g in enumerate(grids):
        ref, gref = oracle.nsdf_targets(g, pts[o], grad=True)
        np.testing.assert_allclose(rec[o, :, :3], ref[:, :3], atol=2e-6, rtol=0)
        np.testing.assert_allclose(rec[o, :, 3], ref[:, 3], atol=1e-6, rtol=0)
        assert np.all(np.abs(rec[o, :, :3]) <= 1.0)
        # the gradient: corner differences of FP32 values over h ~ 1 mm, so FP32 rounding of the
        # corner values (|phi| up to a few cm) sets the scale: 2^-24 * 5 cm / 1 mm ~ 3e-6 per term
        np.testing.assert_allclose(grec[o, :, :3], gref, atol=5e-5, rtol=0)
        assert np.all(grec[o, :, 3] == 0.0)


def angle_deg(a, b):
    """Angle between rows of a and b in FP64 (atan2 form: accurate for tiny angles)."""
    a = np.asarray(a, np.float64); b = np.asarray(b, np.float64)
    return np.degrees(np.arctan2(np.linalg.norm(np.cross(a, b), axis=-1), np.sum(a * b, axis=-1)))


@pytest.mark.parametrize("counts", [[1, 37, 3000], [0, 64, 2049]])
def test_query_matches_bf16_oracle(torch_cuda, grids, counts):
    torch = torch_cuda
    from paper_2606_22332_amd import binding as B
    gs = grids[:len(counts)]
    P = init_params(len(gs), 21)
    rng = np.random.default_rng(22)
    xs = [rng.uniform(-1, 1, (c, 3)).astype(np.float32) for c in counts]
    if counts[-1] >= 8:
        xs[-1][:8] = np.array([[sx, sy, sz] for sx in (-1, 1) for sy in (-1, 1) for sz in (-1, 1)], np.float32)
    offs = np.concatenate([[0], np.cumsum(counts)])
    X = np.concatenate(xs)
    ns = B.Nsdf(gs)
    dP = torch.from_numpy(P).cuda()
    out, gx = ns.query(dP, offs, torch.from_numpy(X).cuda(), grad=True)
    out2 = ns.query(dP, offs, torch.from_numpy(X).cuda(), grad=False)
    torch.cuda.synchronize()
    out, gx, out2 = out.cpu().numpy(), gx.cpu().numpy(), out2.cpu().numpy()
    ns.close()
    assert np.array_equal(out, out2)
    errs, angs, rels = [], [], []
    for o, g in enumerate(gs):
        sl = slice(offs[o], offs[o + 1])
        if counts[o] == 0:
            continue
        ref, rg = oracle.nsdf_forward(P[o].astype(np.float64), X[sl].astype(np.float64), grad=True, bf16=True)
        errs.append(np.abs(out[sl] - ref) * half_extent(g) * 1e6)
        angs.append(angle_deg(gx[sl], rg))
        nr = np.linalg.norm(rg, axis=1)
        rels.append(np.abs(np.linalg.norm(gx[sl].astype(np.float64), axis=1) - nr) / np.maximum(nr, 1e-30))
    err_um, ang, rel = np.concatenate(errs), np.concatenate(angs), np.concatenate(rels)
    stats = dict(n=len(ang), phi_p999_um=np.quantile(err_um, 0.999), phi_max_um=err_um.max(),
                 ang_p99=np.quantile(ang, 0.99), ang_max=ang.max(), gnorm_rel_p99=np.quantile(rel, 0.99))
    print(stats)
    assert stats["phi_p999_um"] <= 20.0 and stats["phi_max_um"] <= 200.0, stats
    assert stats["ang_p99"] <= 0.1 and stats["ang_max"] <= 1.0, stats
    assert stats["gnorm_rel_p99"] <= 1e-2, stats


def layer_rel(a, b):
    return {k: np.linalg.norm(a[s:e] - b[s:e]) / max(np.linalg.norm(b[s:e]), 1e-30) for k, (s, e) in LAYERS.items()}


@pytest.mark.parametrize("lam", [0.0, 0.5])
def test_grad_matches_oracle(torch_cuda, grids, lam):
    """Full-batch loss gradient against the oracle (FP64 and BF16-emulating), with and without
    the pair term (records 2i and 2i+1 paired)."""
    torch = torch_cuda
    from paper_2606_22332_amd import binding as B
    gs = grids[:3]
    n = 200                                   # 12.5 tiles of 16: ragged tail
    P = init_params(len(gs), 31)
    S = records(gs, n, 32)
    ns = B.Nsdf(gs)
    loss, G = ns.grad(torch.from_numpy(P).cuda(), torch.from_numpy(S).cuda(), pair_lambda=lam)
    torch.cuda.synchronize()
    loss, G = loss.cpu().numpy(), G.cpu().numpy()
    ns.close()
    for o in range(len(gs)):
        x, t = S[o, :, :3].astype(np.float64), S[o, :, 3].astype(np.float64)
        l64, g64 = oracle.nsdf_loss_grad(P[o].astype(np.float64), x, t, pair_lambda=lam)
        lbf, gbf = oracle.nsdf_loss_grad(P[o].astype(np.float64), x, t, bf16=True, pair_lambda=lam)
        r64 = layer_rel(G[o].astype(np.float64), g64)
        rbf = layer_rel(G[o].astype(np.float64), gbf)
        print(dict(obj=o, loss_gpu=float(loss[o]), loss_bf=lbf, loss_64=l64, vs64=r64, vsbf=rbf))
        # the loss is a mean of |out - t| (plus lam |r_odd - r_even| per pair): it moves by at most
        # the forward tolerance (20 um / e) per point, times (1 + 2 lam / 2) with the pair term
        assert abs(loss[o] - lbf) <= (1 + lam) * 20e-6 / half_extent(gs[o])
        assert max(r64.values()) <= 1e-2, r64
        assert max(rbf.values()) <= 5e-3, rbf


def decisive_records(gs, n, seed, P, margin=0.02):
    """Records with their grid-gradient records, kept only where every component of the BF16
    oracle's input-gradient error g - gt is farther than `margin` (relative to |g|) from zero:
    the gradient term's sign(g - gt) is then the same on both sides whatever their last-bit
    differences."""
    out_s, out_g = [], []
    for o, g in enumerate(gs):
        pts = synth.nsdf_points([g], 4 * n, seed + o)[0]
        rec, grad = oracle.nsdf_targets(g, pts, grad=True)
        _, gx = oracle.nsdf_forward(P[o].astype(np.float64), rec[:, :3], grad=True, bf16=True)
        e = gx - grad
        ok = np.all(np.abs(e) > margin * np.maximum(np.linalg.norm(gx, axis=1, keepdims=True), 1e-3), axis=1)
        idx = np.flatnonzero(ok)[:n]
        assert idx.size == n
        out_s.append(rec[idx])
        out_g.append(np.concatenate([grad[idx], np.zeros((n, 1))], axis=1))
    return np.stack(out_s).astype(np.float32), np.stack(out_g).astype(np.float32)


@pytest.mark.parametrize("lam,glam", [(0.0, 0.25), (0.5, 0.05)])
def test_grad_with_gradient_term_matches_oracle(torch_cuda, grids, lam, glam):
    """Full-batch loss gradient with the L1 term on the network's input gradient (a tangent pass
    along sign(g - gt), differentiated in reverse mode) against the oracle's FP64 and
    BF16-emulating backprop of the same loss; ragged tail, with and without the pair term."""
    torch = torch_cuda
    from paper_2606_22332_amd import binding as B
    gs = grids[:3]
    n = 200
    P = init_params(len(gs), 33)
    S, G = decisive_records(gs, n, 34, P)
    ns = B.Nsdf(gs)
    loss, Gr = ns.grad(torch.from_numpy(P).cuda(), torch.from_numpy(S).cuda(), pair_lambda=lam,
                       grad_samples=torch.from_numpy(G).cuda(), grad_lambda=glam)
    loss0, Gr0 = ns.grad(torch.from_numpy(P).cuda(), torch.from_numpy(S).cuda(), pair_lambda=lam)
    torch.cuda.synchronize()
    loss, Gr, loss0, Gr0 = loss.cpu().numpy(), Gr.cpu().numpy(), loss0.cpu().numpy(), Gr0.cpu().numpy()
    ns.close()
    for o in range(len(gs)):
        x, t, gt = S[o, :, :3].astype(np.float64), S[o, :, 3].astype(np.float64), G[o, :, :3].astype(np.float64)
        l64, g64 = oracle.nsdf_loss_grad(P[o].astype(np.float64), x, t, pair_lambda=lam, gtarget=gt, grad_lambda=glam)
        lbf, gbf = oracle.nsdf_loss_grad(P[o].astype(np.float64), x, t, bf16=True, pair_lambda=lam, gtarget=gt,
                                         grad_lambda=glam)
        _, gv = oracle.nsdf_loss_grad(P[o].astype(np.float64), x, t, bf16=True, pair_lambda=lam)
        r64 = layer_rel(Gr[o].astype(np.float64), g64)
        rbf = layer_rel(Gr[o].astype(np.float64), gbf)
        # the gradient term changes the gradient: its share of it, layer by layer
        share = layer_rel(gbf, gv)
        print(dict(obj=o, loss_gpu=float(loss[o]), loss_bf=lbf, loss_64=l64, vs64=r64, vsbf=rbf, term_share=share))
        # the value part moves by the forward tolerance; the gradient part by the gradient's
        # (p99 0.1 deg and 1% in norm, on |g| ~ 1..100 per x_hat unit)
        _, gx = oracle.nsdf_forward(P[o].astype(np.float64), x, grad=True, bf16=True)
        gnorm = float(np.linalg.norm(gx, axis=1).mean())
        assert abs(loss[o] - lbf) <= (1 + lam) * 20e-6 / half_extent(gs[o]) + glam * 3 * 1e-2 * gnorm
        assert loss[o] > loss0[o]
        # Against the BF16-emulating oracle only: the records are chosen so that its sign(g - gt)
        # decisions are clear of the GPU's rounding, but the FP64 network's input gradient and
        # output differ from the BF16 network's by more than that margin at a few records, so its
        # L1 terms take other signs there (vs64 is printed, not asserted; the FP64 backprop of this
        # loss is pinned by central differences on the CPU)
        assert max(rbf.values()) <= 2e-3, rbf
        assert min(share[k] for k in ("W1", "W2", "W3", "W4")) > 0.05, share


def test_adam_matches_oracle(torch_cuda):
    torch = torch_cuda
    from paper_2606_22332_amd import binding as B
    rng = np.random.default_rng(41)
    n = 2 * NP + 7
    P = rng.normal(0, 0.3, n).astype(np.float32)
    m = rng.normal(0, 1e-3, n).astype(np.float32)
    v = rng.uniform(0, 1e-5, n).astype(np.float32)
    g = rng.normal(0, 1e-2, n).astype(np.float32)
    hp = B.train_params(lr=1e-3)
    ns = B.Nsdf(synth.make_scene("c1", num_envs=1, num_steps=1).grids)
    dP, dm, dv, dg = (torch.from_numpy(a).cuda() for a in (P, m, v, g))
    ns.adam(dP, dm, dv, dg, 7, hp)
    torch.cuda.synchronize()
    ns.close()
    P64, m64, v64 = P.astype(np.float64), m.astype(np.float64), v.astype(np.float64)
    # the library holds the hyperparameters in FP32: give the oracle the same values
    b1, b2, lr, eps = (float(np.float32(x)) for x in (0.9, 0.999, 1e-3, 1e-8))
    oracle.nsdf_adam(P64, m64, v64, g.astype(np.float64), 7, lr=lr, b1=b1, b2=b2, eps=eps)
    # FP32 against FP64: each result within a few FP32 ulps of the magnitude of what was summed
    sm = b1 * np.abs(m) + (1 - b1) * np.abs(g)
    sv = b2 * np.abs(v) + (1 - b2) * g.astype(np.float64) ** 2
    assert np.all(np.abs(dm.cpu().numpy() - m64) <= 4e-7 * sm + 1e-30)
    assert np.all(np.abs(dv.cpu().numpy() - v64) <= 4e-7 * sv + 1e-30)
    step = np.abs(P64 - P.astype(np.float64))
    assert np.all(np.abs(dP.cpu().numpy() - P64) <= 4e-7 * np.abs(P64) + 1e-5 * step + 1e-12)


def minibatch_indices(o, step, batch, n, seed):
    """Record indices of one object's minibatch: Philox4x32-10 with key (seed lo, seed hi) and
    counter (object, step, j / 4, 8), word j % 4, index = (word * n) >> 32 (oracle's generator)."""
    key = [seed & 0xffffffff, seed >> 32]
    idx = np.empty(batch, np.int64)
    for q in range(batch // 4):
        w = oracle.philox4x32_10([o, step, q, 8], key)
        idx[4 * q:4 * q + 4] = (w.astype(np.uint64) * np.uint64(n)) >> np.uint64(32)
    return idx


@pytest.mark.parametrize("glam", [0.0, 0.1])
def test_fused_training_equals_grad_then_adam(torch_cuda, grids, glam):
    torch = torch_cuda
    from paper_2606_22332_amd import binding as B
    gs = grids[:2]
    n, batch, steps, seed = 3000, 128, 3, 0x1234_0000_0042
    P0 = init_params(len(gs), 51)
    pts = synth.nsdf_points(gs, n, 52)
    ns = B.Nsdf(gs)
    dS, dG = ns.targets(torch.from_numpy(pts).cuda(), grad=True)
    hp = B.train_params(lr=1e-3, batch=batch, seed=seed, grad_lambda=glam)
    Pf = torch.from_numpy(P0).cuda(); mf = torch.zeros_like(Pf); vf = torch.zeros_like(Pf)
    lf = torch.zeros((steps, len(gs)), device="cuda")
    ns.train(Pf, mf, vf, dS, 0, steps, hp, loss=lf, grad_samples=dG if glam > 0 else None)
    Pc = torch.from_numpy(P0).cuda(); mc = torch.zeros_like(Pc); vc = torch.zeros_like(Pc)
    lc = []
    for t in range(1, steps + 1):
        idx = np.stack([minibatch_indices(o, t, batch, n, seed) for o in range(len(gs))])
        sub = torch.stack([dS[o, torch.from_numpy(idx[o]).cuda()] for o in range(len(gs))]).contiguous()
        gsub = torch.stack([dG[o, torch.from_numpy(idx[o]).cuda()] for o in range(len(gs))]).contiguous()
        loss, G = ns.grad(Pc, sub, grad_samples=gsub if glam > 0 else None, grad_lambda=glam)
        ns.adam(Pc, mc, vc, G, t, hp)
        lc.append(loss.cpu().numpy())
    torch.cuda.synchronize()
    ns.close()
    np.testing.assert_allclose(lf.cpu().numpy(), np.stack(lc), rtol=1e-5)
    dPf, dPc = (Pf.cpu().numpy() - P0), (Pc.cpu().numpy() - P0)
    for o in range(len(gs)):
        assert np.linalg.norm(dPf[o] - dPc[o]) <= 1e-3 * np.linalg.norm(dPc[o])


def test_training_fits_a_sphere(torch_cuda):
    """Fused GPU training on the sphere grid cuts the L1 loss several-fold in 400 steps and the
    trained network's surface error falls well below the initial one."""
    torch = torch_cuda
    from paper_2606_22332_amd import binding as B
    gs = synth.make_scene("c1", num_envs=1, num_steps=1).grids
    n = 1 << 15
    S = records(gs, n, 61)
    P0 = synth.nsdf_init(1, 62)
    hp = B.train_params(lr=1e-3, batch=1024, seed=63)
    ns = B.Nsdf(gs)
    P = torch.from_numpy(P0).cuda(); m = torch.zeros_like(P); v = torch.zeros_like(P)
    L = torch.zeros((400, 1), device="cuda")
    ns.train(P, m, v, torch.from_numpy(S).cuda(), 0, 400, hp, loss=L)
    x = torch.from_numpy(np.ascontiguousarray(S[0, :2000, :3])).cuda()
    out0 = ns.query(torch.from_numpy(P0).cuda(), [0, 2000], x, grad=False)
    out1 = ns.query(P, [0, 2000], x, grad=False)
    torch.cuda.synchronize()
    ns.close()
    L = L.cpu().numpy()[:, 0]
    assert L[-20:].mean() < 0.2 * L[:5].mean(), (L[:5], L[-20:])
    e = half_extent(gs[0])
    err0 = np.abs(out0.cpu().numpy() - S[0, :2000, 3]) * e
    err1 = np.abs(out1.cpu().numpy() - S[0, :2000, 3]) * e
    assert math.isfinite(float(np.median(err1)))
    assert np.median(err1) < 0.2 * np.median(err0), (np.median(err0), np.median(err1))


def train_decayed(B, ns, P, m, v, S, steps, batch, seed, pieces=10):
    """Adam with the learning rate decayed along a half cosine from 1e-3 to 1e-5 in `pieces`
    constant pieces (the step counter runs on across pieces)."""
    edges = np.linspace(0, steps, pieces + 1).astype(int)
    for i in range(pieces):
        lr = 1e-5 + 0.5 * (1e-3 - 1e-5) * (1.0 + np.cos(np.pi * (i + 0.5) / pieces))
        ns.train(P, m, v, S, int(edges[i]), int(edges[i + 1] - edges[i]),
                 B.train_params(lr=float(lr), batch=batch, seed=seed))


@pytest.mark.parametrize("family_index", [3, 4])     # torus, convex hull of the C2 objects
def test_trained_network_against_a_grid_of_equal_size(torch_cuda, family_index):
    """What the learned SDF buys: a network trained on the GPU (15,681 parameters, 3000 steps
    with a decayed learning rate) against a grid of the same number of values (25^3 = 15,625)
    on the same box, both judged on near-surface points (|phi| < 3 mm, where contacts happen)
    against the object's 64^3 reference grid; both error distributions are printed.
    - torus (curved everywhere): the network beats the equal-size grid clearly, at the median
      and at p99;
    - convex hull (flat faces, sharp edges): the grid keeps the lead at the median, since away
      from edges the signed distance to a face is affine, which trilinear interpolation
      reproduces exactly while the network's smooth fit does not; at p99, where the error sits
      at edges and vertices, the two are on par.
    Training is bitwise repeatable, so the outcome is fixed for a given build; over four
    initialisation seeds the margins asserted here held with room (torus median 51-57 um vs 167,
    p99 241-250 vs 428; hull p99 533-571 vs 544)."""
    torch = torch_cuda
    from paper_2606_22332_amd import binding as B
    grids = synth.make_scene("c2", num_envs=2, num_steps=1).grids
    g = grids[family_index]
    n_train = 1 << 16
    S = records([g], n_train, 71)
    P0 = synth.nsdf_init(1, 72)
    ns = B.Nsdf([g])
    P = torch.from_numpy(P0).cuda(); m = torch.zeros_like(P); v = torch.zeros_like(P)
    train_decayed(B, ns, P, m, v, torch.from_numpy(S).cuda(), 3000, 4096, 73)
    # held-out near-surface points
    pts = synth.nsdf_points([g], 8192, 74, sigma=1e-3)[0, :4096]
    ref = oracle.nsdf_targets(g, pts)                       # 64^3 reference grid, FP64
    e = half_extent(g)
    near = np.abs(ref[:, 3] * e) < 3e-3
    x = torch.from_numpy(np.ascontiguousarray(ref[near, :3].astype(np.float32))).cuda()
    out = ns.query(P, [0, int(near.sum())], x, grad=False)
    torch.cuda.synchronize()
    ns.close()
    err_nn = np.abs(out.cpu().numpy() - ref[near, 3]) * e
    side = (g.n - 1) * float(g.spacing)
    coarse = synth.sample_grid(g.shape, 25, side)
    err_grid = np.abs(oracle.nsdf_targets(coarse, pts[near])[:, 3] * e - ref[near, 3] * e)
    stats = dict(family=g.family, points=int(near.sum()), nn_median_um=float(np.median(err_nn) * 1e6),
                 nn_p99_um=float(np.quantile(err_nn, 0.99) * 1e6), grid25_median_um=float(np.median(err_grid) * 1e6),
                 grid25_p99_um=float(np.quantile(err_grid, 0.99) * 1e6))
    print(stats)
    q_nn, q_grid = np.quantile(err_nn, 0.99), np.quantile(err_grid, 0.99)
    if g.family == "torus":
        assert np.median(err_nn) < 0.5 * np.median(err_grid) and q_nn < 0.8 * q_grid, stats
    else:
        assert np.median(err_grid) < np.median(err_nn) and q_nn < 1.1 * q_grid, stats


@pytest.mark.parametrize("glam", [0.0, 0.1])
def test_training_is_bitwise_repeatable(torch_cuda, grids, glam):
    """Two trainings from the same start give the same parameters, moments and loss trace bit for
    bit: the minibatches come from a counter-based generator and every reduction of a step adds
    its terms in a fixed order (with and without the gradient term)."""
    torch = torch_cuda
    from paper_2606_22332_amd import binding as B
    pts = torch.from_numpy(synth.nsdf_points(grids, 4096, 81)).cuda()
    runs = []
    for _ in range(2):
        ns = B.Nsdf(grids)
        S, G = ns.targets(pts, grad=True)
        P = torch.from_numpy(synth.nsdf_init(len(grids), 82)).cuda(); m = torch.zeros_like(P); v = torch.zeros_like(P)
        loss = torch.zeros((300, len(grids)), device="cuda")
        ns.train(P, m, v, S, 0, 300, B.train_params(lr=1e-3, batch=1024, seed=83, grad_lambda=glam), loss=loss,
                 grad_samples=G)
        torch.cuda.synchronize()
        ns.close()
        runs.append([t.cpu().numpy() for t in (P, m, v, loss)])
    for a, b in zip(*runs):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("family_index", [3, 1])     # torus, box of the C2 objects
def test_gradient_term_improves_the_network_normal(torch_cuda, family_index):
    """What the gradient term buys: the same network trained from the same start with and without
    the L1 term on its input gradient (grid gradient as the target, weight 0.01),
    judged on held-out points 1-8 mm from the surface (where the neural readout takes the normal
    from the network: outside the 1 mm fallback band) by the angle between the network's gradient
    and the 64^3 grid's, and by the value error there."""
    torch = torch_cuda
    from paper_2606_22332_amd import binding as B
    grids = synth.make_scene("c2", num_envs=2, num_steps=1).grids
    g = grids[family_index]
    ns = B.Nsdf([g])
    S, G = ns.targets(torch.from_numpy(synth.nsdf_points([g], 1 << 16, 91)).cuda(), grad=True)
    pts = synth.nsdf_points([g], 1 << 14, 92, sigma=4e-3)[0]
    ref, gref = oracle.nsdf_targets(g, pts, grad=True)
    e = half_extent(g)
    band = (np.abs(ref[:, 3] * e) >= 1e-3) & (np.abs(ref[:, 3] * e) <= 8e-3) & (np.linalg.norm(gref, axis=1) > 0.5)
    x = torch.from_numpy(np.ascontiguousarray(ref[band, :3].astype(np.float32))).cuda()
    res = {}
    for glam in (0.0, 0.01):
        P = torch.from_numpy(synth.nsdf_init(1, 93)).cuda(); m = torch.zeros_like(P); v = torch.zeros_like(P)
        ns.train(P, m, v, S, 0, 3000, B.train_params(lr=1e-3, batch=4096, seed=94, grad_lambda=glam), grad_samples=G)
        out, gx = ns.query(P, [0, int(band.sum())], x, grad=True)
        torch.cuda.synchronize()
        ang = angle_deg(gx.cpu().numpy(), gref[band])
        err = np.abs(out.cpu().numpy() - ref[band, 3]) * e * 1e6
        res[glam] = dict(ang_p50=float(np.median(ang)), ang_p90=float(np.quantile(ang, 0.9)),
                         ang_p99=float(np.quantile(ang, 0.99)), phi_p50_um=float(np.median(err)),
                         phi_p99_um=float(np.quantile(err, 0.99)))
    ns.close()
    print(dict(family=g.family, points=int(band.sum()), **{f"lambda={k}": v for k, v in res.items()}))
    a, b = res[0.0], res[0.01]
    assert b["ang_p50"] < 0.8 * a["ang_p50"] and b["ang_p90"] < 0.9 * a["ang_p90"], res
    assert b["phi_p50_um"] < 2.0 * a["phi_p50_um"] + 20.0, res
