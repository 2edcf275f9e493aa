"""ProximityTaxel readout (include/tg_proximity.h) against the FP64 oracle, through the C ABI.

The oracle visits every point of the cloud and forms each term of App. A.6 per point in FP64; the
GPU visits the cells around each probe and forms the channels from two FP32 moments of the
penetration (sum P and sum P (p - q)).  Both are exact up to rounding.  What rounding allows: the
GPU's probe centre is FP32 arithmetic on FP32 poses, off the FP64 one by about 1e-8 m, which moves
each point's P by as much, so with n the number of points inside the sphere
  |d sum P| <= 1e-5 sum P + n * 2e-8,
  |df|_inf <= 1e-5 fs + (k rho + k_s rho v) n * 2e-8,   fs = (k rho + k_s rho v) sum P,
  |dtau|_inf <= 1e-5 ts + k rho (n * 2e-8 * R + sum P * 2e-8),   ts = k rho sum P R,
per taxel, with v an upper bound of the relative point speed.  Points at the edge of a sensing
sphere contribute P ~ 0 whichever side of it rounding puts them.

Scenes: the 16-link hand (4096 envs in the benchmark; fewer here) and its 8 objects, each with an
area-uniform surface cloud of 5000 points, sensing radius 1 cm; trajectories as in the readout
workloads; static and moving objects; envs without an object; radius noise; per-probe gain.
"""
import numpy as np
import pytest

import oracle
from paper_2606_22332_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def run_gpu(sc, clouds, inp, **kw):
    import torch
    from paper_2606_22332_amd import binding as B
    gain = kw.pop("gain", None)
    px = B.Proximity(sc, clouds, **kw)
    d = B.to_device(inp)
    g = None if gain is None else torch.from_numpy(np.ascontiguousarray(gain, np.float32)).cuda()
    ft, mass = px.rollout(d, gain=g)
    torch.cuda.synchronize()
    px.close()
    return ft.cpu().numpy(), mass.cpu().numpy()


def run_oracle(sc, clouds, inp, envs=None, radius=0.01, k=300.0, k_s=10.0, density=100.0, seed=0, radius_rho=0.0,
               gain=None):
    lay = sc.layout
    L = lay.num_links
    if envs is not None:
        inp = synth.subset_envs(inp, np.asarray(envs), L)
        if gain is not None:
            gain = gain[envs]
    return oracle.prox_run(lay.link_offset, lay.pos, lay.normal, np.full(lay.num_taxels, radius, np.float32), clouds,
                           inp.link_state, inp.obj_id, inp.obj_state, inp.step0, k=k, k_s=k_s, density=density,
                           seed=seed, radius_rho=radius_rho, gain=gain, with_count=True)


def velocity_scale(inp, sc, envs=None):
    """Per (step, env, taxel): an upper bound of |v_p - v_tax| over the sensing sphere, from the
    link and object speeds and spins (lever arms of at most 10 cm)."""
    L = sc.layout.num_links
    ls = inp.link_state
    S, E = inp.obj_id.shape
    vl = np.linalg.norm(ls[:, 7:10], axis=1).reshape(S, E, L)
    wl = np.linalg.norm(ls[:, 10:13], axis=1).reshape(S, E, L)
    link_of = np.repeat(np.arange(L), np.diff(sc.layout.link_offset))
    v = vl[..., link_of] + 0.1 * wl[..., link_of]
    if inp.obj_state is not None:
        v = v + (np.linalg.norm(inp.obj_state[:, 7:10], axis=1) + 0.1 * np.linalg.norm(inp.obj_state[:, 10:13], axis=1))[..., None]
    if envs is not None:
        v = v[:, envs]
    return v


def check(g_ft, g_m, ref, vscale, radius=0.01, k=300.0, k_s=10.0, density=100.0, n_pts=5000, gain=None):
    r_ft, r_m, cnt = ref
    rho = density / n_pts
    gmul = 1.0 if gain is None else np.abs(gain)[None]
    dq = 2e-8
    kf = k * rho + k_s * rho * vscale
    fs = kf * r_m * gmul
    ts = k * rho * r_m * radius * gmul
    f_tol = (1e-5 * fs + kf * cnt * dq * gmul) + 1e-12
    t_tol = (1e-5 * ts + k * rho * (cnt * dq * radius + r_m * dq) * gmul) + 1e-15
    m_tol = 1e-5 * r_m + cnt * dq + 1e-15
    f_err = np.abs(g_ft[:, :3] - r_ft[:, :3]).max(1)
    t_err = np.abs(g_ft[:, 3:] - r_ft[:, 3:]).max(1)
    m_err = np.abs(g_m - r_m)
    info = dict(f_ratio=float((f_err / f_tol).max()), t_ratio=float((t_err / t_tol).max()),
                m_ratio=float((m_err / m_tol).max()), in_range=float((r_m > 0).mean()),
                points_in_sphere_mean=float(cnt[cnt > 0].mean()) if (cnt > 0).any() else 0.0)
    assert np.all(f_err <= f_tol), info
    assert np.all(t_err <= t_tol), info
    assert np.all(m_err <= m_tol), info
    return info


def scene(E, S, moving=False, seed_shift=0):
    sc = synth.make_scene("c2", num_envs=E, num_steps=S)
    inp = synth.make_inputs(sc)
    if moving:
        inp.obj_state = synth.random_object_state(sc, S)
    clouds = synth.surface_clouds(sc.grids, 5000, seed=sc.geom_seed + 20 + seed_shift)
    return sc, inp, clouds


@pytest.mark.parametrize("moving", [False, True])
def test_hand_parity(torch_cuda, moving):
    sc, inp, clouds = scene(37, 3, moving)
    oid = inp.obj_id.copy()
    oid[:, 2] = -1                     # no object
    oid[:, 5] = 99                     # out of range: no object
    inp.obj_id = oid
    g_ft, g_m = run_gpu(sc, clouds, inp)
    ref = run_oracle(sc, clouds, inp)
    info = check(g_ft, g_m, ref, velocity_scale(inp, sc))
    print(dict(moving=moving, **info))
    assert info["in_range"] > 0.2
    assert np.all(g_ft[:, :, [2, 5]] == 0) and np.all(g_m[:, [2, 5]] == 0)


def test_radius_noise_and_gain(torch_cuda):
    sc, inp, clouds = scene(24, 4)
    gain = np.random.default_rng(5).uniform(0.8, 1.2, (sc.num_envs, sc.layout.num_taxels)).astype(np.float32)
    kw = dict(seed=0x5EED_0001_0002, radius_rho=1e-3)
    g_ft, g_m = run_gpu(sc, clouds, inp, gain=gain, **kw)
    ref = run_oracle(sc, clouds, inp, gain=gain, **kw)
    info = check(g_ft, g_m, ref, velocity_scale(inp, sc), radius=0.011, gain=gain)
    # the noise moves the radius, and with it the sums, from step to step
    g0, m0 = run_gpu(sc, clouds, inp)
    assert not np.array_equal(m0, g_m)
    print(info)


def test_small_radius_and_sparse_cloud(torch_cuda):
    """Radius 3 mm and 300 points per object: most probes see no point at all, the rest a few."""
    sc, inp, _ = scene(20, 2)
    clouds = synth.surface_clouds(sc.grids, 300, seed=77)
    g_ft, g_m = run_gpu(sc, clouds, inp, radius=3e-3)
    ref = run_oracle(sc, clouds, inp, radius=3e-3)
    info = check(g_ft, g_m, ref, velocity_scale(inp, sc), radius=3e-3, n_pts=300)
    assert 0 < info["in_range"] < 0.5
    print(info)


def test_full_size_sampled(torch_cuda):
    """The benchmark's launch (4096 envs x 200 taxels x 100 steps) checked on sampled envs."""
    import torch
    from paper_2606_22332_amd import binding as B
    sc = synth.make_scene("c2")
    inp = synth.make_inputs(sc)
    clouds = synth.surface_clouds(sc.grids, 5000, seed=sc.geom_seed + 20)
    px = B.Proximity(sc, clouds)
    ft, mass = px.rollout(B.to_device(inp))
    torch.cuda.synchronize()
    envs = np.array([0, 1, 1365, 2730, 4095])
    g_ft = ft[:, :, torch.as_tensor(envs, device="cuda")].cpu().numpy()
    g_m = mass[:, torch.as_tensor(envs, device="cuda")].cpu().numpy()
    px.close()
    ref = run_oracle(sc, clouds, inp, envs=envs)
    info = check(g_ft, g_m, ref, velocity_scale(inp, sc, envs))
    print(info)


def test_rejects_bad_configurations(torch_cuda):
    from paper_2606_22332_amd import binding as B
    sc, inp, clouds = scene(4, 1)
    with pytest.raises(B.TgError):
        B.Proximity(sc, clouds, radius=-1.0)
    bad = [c.copy() for c in clouds]
    bad[1][3, 0] = np.nan
    with pytest.raises(B.TgError):
        B.Proximity(sc, bad)
