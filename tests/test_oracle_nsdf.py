"""Pins of the neural-SDF oracle (positional encoding -> 4 x 64 SiLU -> 1): backprop against
central finite differences, closed forms of degenerate networks, the first Adam step, and a small
fit that converges."""
import math

import numpy as np
import pytest

import oracle

NP = 15681
H, F = 64, 48


def he_init(rng):
    P = np.zeros(NP)
    o = 0
    for fan_in, fan_out in ((F, H), (H, H), (H, H), (H, H)):
        lim = math.sqrt(6.0 / fan_in)
        P[o:o + fan_in * fan_out] = rng.uniform(-lim, lim, fan_in * fan_out)
        o += fan_in * fan_out + fan_out
    lim = math.sqrt(6.0 / H)
    P[o:o + H] = rng.uniform(-lim, lim, H)
    return P


def offsets():
    o, out = 0, []
    for fan_in in (F, H, H, H):
        out.append((o, o + fan_in * H))          # (W, b) offsets
        o += fan_in * H + H
    out.append((o, o + H))                       # (w5, b5)
    return out


def silu(z):
    return z / (1 + np.exp(-z))


def test_parameter_count():
    assert oracle.nsdf_num_params() == NP == 48 * 64 + 64 + 3 * (64 * 64 + 64) + 64 + 1


@pytest.mark.parametrize("lam", [0.0, 0.7])
def test_loss_gradient_matches_central_differences(lam):
    """The loss gradient against central differences of the loss; with lam > 0 the loss is
    also checked against its definition, mean |r| plus lam times the mean over the points of
    |r_2i+1 - r_2i| counted once per pair, from the plain forward pass."""
    rng = np.random.default_rng(0)
    P = he_init(rng)
    P[offsets()[0][1]:offsets()[0][1] + H] = rng.normal(0, 0.1, H)     # nonzero biases too
    x = rng.uniform(-1, 1, (16, 3))
    t = rng.normal(0, 0.3, 16)
    loss, g = oracle.nsdf_loss_grad(P, x, t, pair_lambda=lam)
    r = oracle.nsdf_forward(P, x) - t
    assert loss == pytest.approx((np.abs(r).sum() + lam * np.abs(r[1::2] - r[0::2]).sum()) / 16, rel=1e-12)
    idx = np.concatenate([rng.choice(NP, 200, replace=False), [NP - 1, NP - 2, 0]])
    h = 1e-6
    for i in idx:
        Pp, Pm = P.copy(), P.copy()
        Pp[i] += h
        Pm[i] -= h
        fd = (oracle.nsdf_loss_grad(Pp, x, t, pair_lambda=lam)[0] - oracle.nsdf_loss_grad(Pm, x, t, pair_lambda=lam)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])), (i, fd, g[i])


@pytest.mark.parametrize("lam", [0.0, 0.7])
def test_gradient_term_matches_its_definition_and_central_differences(lam):
    """With the L1 term on the input gradient (grad_lambda > 0): the loss equals its definition,
    mean |r| (plus the pair term) plus grad_lambda times the mean over the points of
    sum_d |g_d - gt_d| with g from the plain reverse pass; its parameter gradient (through the
    tangent pass and the second derivative of SiLU) matches central differences of that loss."""
    rng = np.random.default_rng(5)
    P = he_init(rng)
    for w, b in offsets()[:4]:
        P[b:b + H] = rng.normal(0, 0.1, H)
    P[NP - 1] = 0.05
    n = 16
    x = rng.uniform(-1, 1, (n, 3))
    t = rng.normal(0, 0.3, n)
    gt = rng.normal(0, 1.0, (n, 3))
    gl = 0.3
    loss, g = oracle.nsdf_loss_grad(P, x, t, pair_lambda=lam, gtarget=gt, grad_lambda=gl)
    out, gx = oracle.nsdf_forward(P, x, grad=True)
    r = out - t
    expect = (np.abs(r).sum() + lam * np.abs(r[1::2] - r[0::2]).sum() + gl * np.abs(gx - gt).sum()) / n
    assert loss == pytest.approx(expect, rel=1e-12)
    # the gradient term changes the parameter gradient in every layer
    _, g0 = oracle.nsdf_loss_grad(P, x, t, pair_lambda=lam)
    for w, b in offsets():
        assert np.linalg.norm(g[w:b] - g0[w:b]) > 1e-3 * np.linalg.norm(g0[w:b])
    lossf = lambda Q: oracle.nsdf_loss_grad(Q, x, t, pair_lambda=lam, gtarget=gt, grad_lambda=gl)[0]
    idx = np.concatenate([rng.choice(NP, 200, replace=False), [NP - 1, NP - 2, 0]] +
                         [np.arange(b, b + 3) for _, b in offsets()[:4]])
    h = 1e-6
    for i in idx:
        Pp, Pm = P.copy(), P.copy()
        Pp[i] += h
        Pm[i] -= h
        fd = (lossf(Pp) - lossf(Pm)) / (2 * h)
        assert abs(fd - g[i]) <= 2e-6 * max(1.0, abs(g[i])), (i, fd, g[i])


def test_tangent_pass_is_the_directional_derivative():
    """The forward-mode tangent pass along u gives u . (d out / d x_hat) of the reverse pass, and
    the fourth-order central difference of the output along u."""
    rng = np.random.default_rng(6)
    P = he_init(rng)
    x = rng.uniform(-1, 1, (30, 3))
    u = rng.normal(0, 1, (30, 3))
    dd = oracle.nsdf_dirderiv(P, x, u)
    _, gx = oracle.nsdf_forward(P, x, grad=True)
    np.testing.assert_allclose(dd, (gx * u).sum(1), rtol=1e-11, atol=1e-12)
    h = 1e-5
    f = lambda y: oracle.nsdf_forward(P, y)
    fd = (-f(x + 2 * h * u) + 8 * f(x + h * u) - 8 * f(x - h * u) + f(x - 2 * h * u)) / (12 * h)
    np.testing.assert_allclose(dd, fd, rtol=1e-6, atol=1e-7)
    # BF16 emulation of the same pass stays within BF16 noise of the exact one
    dbf = oracle.nsdf_dirderiv(P, x, u, bf16=True)
    assert np.quantile(np.abs(dbf - dd) / np.maximum(np.abs(dd), 1e-3), 0.9) < 0.1


def test_grid_gradient_targets():
    """The grid gradient of the training targets: a linear field's gradient is its normal wherever
    the point lies (trilinear interpolation reproduces it), and for a generic field the analytic
    gradient equals the central difference of the interpolated value inside a cell."""
    from helpers import grid_from, plane_grid
    nrm = np.array([0.3, -0.5, 0.81])
    nrm /= np.linalg.norm(nrm)
    g = plane_grid(nrm, 0.004, n=16, side=0.06)
    rng = np.random.default_rng(7)
    pts = rng.uniform(-0.029, 0.029, (300, 3)).astype(np.float32)
    rec, gr = oracle.nsdf_targets(g, pts, grad=True)
    np.testing.assert_allclose(gr, np.broadcast_to(nrm, gr.shape), atol=2e-6)
    g2 = grid_from(lambda P: np.sin(40 * P[..., 0]) * np.cos(30 * P[..., 1]) + 20 * P[..., 2] ** 2, n=16, side=0.06)
    h = float(g2.spacing)
    o = g2.origin.astype(np.float64)
    # cell-centre neighbourhoods: the stencil stays inside one cell
    cells = rng.integers(0, 15, (200, 3))
    base = o + (cells + rng.uniform(0.3, 0.7, (200, 3))) * h
    pts = base.astype(np.float32)
    p64 = pts.astype(np.float64)
    _, gr = oracle.nsdf_targets(g2, pts, grad=True)
    e = 0.5 * (g2.n - 1) * h
    for d in range(3):
        step = np.zeros(3)
        step[d] = 0.05 * h
        hi = oracle.nsdf_targets(g2, (p64 + step).astype(np.float32))
        lo = oracle.nsdf_targets(g2, (p64 - step).astype(np.float32))
        dx = (hi[:, d] - lo[:, d]) * e          # the clamped points actually used, x_hat -> q
        fd = (hi[:, 3] - lo[:, 3]) * e / dx
        np.testing.assert_allclose(gr[:, d], fd, rtol=1e-6, atol=1e-6)


def test_input_gradient_matches_central_differences():
    rng = np.random.default_rng(1)
    P = he_init(rng)
    x = rng.uniform(-1, 1, (40, 3))
    _, gx = oracle.nsdf_forward(P, x, grad=True)
    h = 1e-5      # fourth-order stencil: the encoding reaches 2^7 pi, so second-order FD is too coarse
    f = lambda y: oracle.nsdf_forward(P, y)
    for d in range(3):
        e = np.zeros(3); e[d] = h
        fd = (-f(x + 2 * e) + 8 * f(x + e) - 8 * f(x - e) + f(x - 2 * e)) / (12 * h)
        np.testing.assert_allclose(gx[:, d], fd, rtol=1e-6, atol=1e-7)


def test_single_path_network_closed_form():
    """Only feature f* feeds hidden unit 0, which is passed on unit 0 to the output: out = silu^4(feat)."""
    ofs = offsets()
    for k, s, d in ((0, 0, 0), (3, 1, 2), (7, 0, 1)):
        P = np.zeros(NP)
        f = 6 * k + 3 * s + d                   # [sin xyz, cos xyz] per frequency
        P[ofs[0][0] + 0 * F + f] = 1.0
        for l in (1, 2, 3):
            P[ofs[l][0] + 0] = 1.0              # W_l[0][0]
        P[ofs[4][0]] = 1.0                      # w5[0]
        x = np.random.default_rng(2).uniform(-1, 1, (20, 3))
        feat = (np.sin if s == 0 else np.cos)(2 ** k * math.pi * x[:, d])
        expect = silu(silu(silu(silu(feat))))
        np.testing.assert_allclose(oracle.nsdf_forward(P, x), expect, rtol=1e-13, atol=1e-15)


def test_input_independent_network():
    """With every weight zero the hidden layers see only their biases: out = b5 + w5 . silu(b4)."""
    rng = np.random.default_rng(3)
    P = np.zeros(NP)
    ofs = offsets()
    b4 = rng.normal(size=H); w5 = rng.normal(size=H)
    P[ofs[3][1]:ofs[3][1] + H] = b4
    P[ofs[4][0]:ofs[4][0] + H] = w5
    P[ofs[4][1]] = 0.25
    out, gx = oracle.nsdf_forward(P, rng.uniform(-1, 1, (5, 3)), grad=True)
    np.testing.assert_allclose(out, 0.25 + w5 @ silu(b4), rtol=1e-14)
    assert np.all(gx == 0)


def test_first_adam_step_is_signed_lr():
    """From zero moments, bias correction makes the first step lr * g / (|g| + eps)."""
    rng = np.random.default_rng(4)
    P = rng.normal(size=100); m = np.zeros(100); v = np.zeros(100)
    g = rng.normal(size=100)
    P0 = P.copy()
    oracle.nsdf_adam(P, m, v, g, 1, lr=1e-3)
    np.testing.assert_allclose(P0 - P, 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12)


def test_bf16_forward_tracks_fp64():
    rng = np.random.default_rng(5)
    P = he_init(rng)
    x = rng.uniform(-1, 1, (200, 3))
    a = oracle.nsdf_forward(P, x)
    b = oracle.nsdf_forward(P, x, bf16=True)
    err = np.abs(a - b) / (np.abs(a).mean() + 1e-12)
    assert err.max() < 0.05 and err.mean() < 0.01


def test_small_fit_converges_on_a_sphere():
    """A few hundred Adam steps on the normalised SDF of a sphere cut the L1 loss several-fold."""
    rng = np.random.default_rng(6)
    P = he_init(rng)
    m = np.zeros(NP); v = np.zeros(NP)
    losses = []
    for t in range(1, 301):
        x = rng.uniform(-1, 1, (64, 3))
        target = np.linalg.norm(x, axis=1) - 0.5
        loss, g = oracle.nsdf_loss_grad(P, x, target)
        oracle.nsdf_adam(P, m, v, g, t, lr=1e-3)
        losses.append(loss)
    assert np.mean(losses[-20:]) < 0.25 * np.mean(losses[:5])


def test_bf16_loss_gradient_tracks_fp64():
    """The BF16-emulating backprop stays within a few BF16 ulps of exact backprop, layer by layer."""
    rng = np.random.default_rng(7)
    P = he_init(rng)
    x = rng.uniform(-1, 1, (64, 3))
    t = rng.normal(0, 0.3, 64)
    l64, g64 = oracle.nsdf_loss_grad(P, x, t)
    lbf, gbf = oracle.nsdf_loss_grad(P, x, t, bf16=True)
    assert abs(lbf - l64) < 0.02 * l64
    for (a, b) in offsets()[:4]:
        w = slice(a, b)
        assert np.linalg.norm(gbf[w] - g64[w]) < 2e-2 * np.linalg.norm(g64[w])


def test_targets_reproduce_a_plane_and_clamp_to_the_box():
    """Trilinear interpolation reproduces a linear field exactly (up to rounding of the FP32 grid);
    points outside the box are clamped onto it before the lookup."""
    import sys, os
    sys.path.insert(0, os.path.dirname(__file__))
    import helpers
    nrm = np.array([0.3, -0.5, 0.8]); nrm /= np.linalg.norm(nrm)
    g = helpers.plane_grid(normal=nrm, offset=0.004, n=16, side=0.08)
    rng = np.random.default_rng(8)
    pts = rng.uniform(-0.06, 0.06, (500, 3)).astype(np.float32)
    rec = oracle.nsdf_targets(g, pts)
    lo = g.origin.astype(np.float64); hi = lo + 15 * float(g.spacing)
    q = np.clip(pts.astype(np.float64), lo, hi)
    e = 0.5 * 15 * float(g.spacing)
    np.testing.assert_allclose(rec[:, :3], (q - (lo + e)) / e, atol=1e-14)
    np.testing.assert_allclose(rec[:, 3] * e, q @ nrm - 0.004, atol=2e-8)
    assert np.all(np.abs(rec[:, :3]) <= 1 + 1e-12)


def test_generated_surface_points_lie_on_the_shapes():
    from paper_2606_22332_amd import synth
    grids = synth.make_scene("c2", num_envs=2, num_steps=1).grids
    rng = np.random.default_rng(9)
    for g in grids:
        p = synth._surface_points(g.shape, 500, rng)
        assert np.abs(synth.shape_sdf(g.shape, p)).max() < 1e-12, g.family
    P = synth.nsdf_init(3, 10)
    assert P.shape == (3, NP) and P.dtype == np.float32
    W1 = P[:, :F * H]
    assert abs(W1.std() - math.sqrt(6 / F) / math.sqrt(3)) < 0.01
    assert np.all(P[:, F * H:F * H + H] == 0)
