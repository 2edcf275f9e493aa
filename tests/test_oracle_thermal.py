"""Pins of the thermal-field oracle (explicit 7-point voxel solver with generation, linearised
radiation and contact conduction), checked against closed forms and conservation:

- the lowest cosine mode of the insulated block decays by exactly (1 - 4 r sin^2(pi/2n)) per step
  (the eigenvalue of the mirrored discrete Laplacian), along x, y or z, and that rate matches the
  continuous exp(-alpha (pi/L)^2 t) to O(dx^2);
- energy balance: the stored energy change equals dt * (P_gen + P_contact - P_rad) each step,
  because mirrored diffusion moves heat without creating it;
- a uniform field with radiation only loses rho_f * (faces) * (T - T_amb) per voxel in one step,
  so corners lose 3 faces' worth, edges 2, faces 1 and the interior nothing;
- generation only: T rises by exactly P_gen dt / (rho c_p V) per step;
- contact: a conductance of one (kappa * depth = 1) takes the voxel to T_obj in one step;
- the constants match the configuration's figures (alpha = 1e-7, r = 1e-4, h_r ~ 4.96 W/m^2K);
- the stability bound accepts the configuration and rejects r > 1/6 or an over-unity contact step.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2606_22332_amd import synth


def f32(x):
    return float(np.float32(x))


def params(**kw):
    E = kw.pop("E", 1)
    th = synth.ThermalParams(field_links=[0], T_obj=np.full(E, 40.0, np.float32))
    for k, v in kw.items():
        setattr(th, k, v)
    return th


def one_link_layout(points):
    pts = np.asarray(points, np.float64).reshape(-1, 3)
    off = np.array([0, pts.shape[0]], np.int32)
    nrm = np.zeros_like(pts); nrm[:, 2] = 1
    return synth.Layout(off, pts.astype(np.float32), nrm.astype(np.float32), np.full(pts.shape[0], 1e-3, np.float32))


def test_constants_of_the_configuration():
    K = oracle.thermal_constants(params())          # inputs are FP32: figures to ~1e-7
    assert K["alpha"] == pytest.approx(1e-7, rel=1e-6)
    assert K["r"] == pytest.approx(1e-4, rel=1e-6)
    assert K["h_r"] == pytest.approx(4 * 0.85 * 5.670374419e-8 * 295.15 ** 3, rel=1e-6)
    assert 4.9 < K["h_r"] < 5.0
    assert K["k_eff"] == pytest.approx(2 * 0.2 * 10 / 10.2, rel=1e-6)


def test_source_rates_of_the_configuration_worked_by_hand():
    """The per-step source coefficients of the configuration (dt = dx = 1 mm units, rho c_p = 2e6 J/m^3K),
    worked out by hand from the thermal model's definitions and written here as numbers:
      radiation  h_r = 4 * 0.85 * 5.6704e-8 W/m^2K^4 * (295.15 K)^3 = 4.9570 W/m^2K,
                 rho_f = dt h_r / (rho c_p dx) = 1e-3 * 4.9570 / (2e6 * 1e-3) = 2.4785e-6 per face,
      contact    k_eff = 2 * 0.2 * 10 / 10.2 = 0.39216 W/mK,
                 kappa = dt pi d_w k_eff / (rho c_p dx^3) = 1e-3 * 3.14159 * 0.39216 / 2e-3 = 0.61600 per m of depth,
      generation g = dt P_gen / (16^3 rho c_p dx^3) = 1e-4 / 8.192 = 1.2207e-5 K per step.
    A dropped dx (area instead of volume), a missing pi or the wrong temperature scale moves them by far
    more than the 1e-4 these figures are held to."""
    K = oracle.thermal_constants(params())
    assert K["h_r"] == pytest.approx(4.9570, rel=1e-4)
    assert K["rho_f"] == pytest.approx(2.4785e-6, rel=1e-4)
    assert K["k_eff"] == pytest.approx(0.39216, rel=1e-4)
    assert K["kappa"] == pytest.approx(0.61600, rel=1e-4)
    assert K["g"] == pytest.approx(1.2207e-5, rel=1e-4)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_cosine_mode_decays_at_the_discrete_eigenvalue(axis):
    n, steps = 16, 300
    th = params(P_gen=0.0, emissivity=0.0, dt=0.5)                # r = 0.05
    K = oracle.thermal_constants(th)
    i = np.arange(n)
    mode = 5.0 * np.cos(np.pi * (i + 0.5) / n)
    shape = [1, 1, 1]
    shape[2 - axis] = n                                            # field index [z][y][x]
    f = np.broadcast_to(22.0 + mode.reshape(shape), (n, n, n)).astype(np.float64).copy()
    fields = f.reshape(1, 1, n, n, n).copy()
    lay = one_link_layout([[0.0, 0.0, 0.0]])
    depth = np.zeros((steps, 1, 1))
    fields, _, _ = oracle.thermal_run(th, lay, depth, fields)
    lam = 1.0 - 4.0 * K["r"] * math.sin(math.pi / (2 * n)) ** 2
    expect = 22.0 + (lam ** steps) * mode.reshape(shape)
    np.testing.assert_allclose(fields[0, 0], np.broadcast_to(expect, (n, n, n)), rtol=0, atol=1e-11)
    # the continuous slab: amplitude exp(-alpha (pi / L)^2 t), L = n dx; O(dx^2) apart per unit time
    L = n * th.dx
    cont = -K["alpha"] * (math.pi / L) ** 2
    disc = math.log(lam) / th.dt
    assert abs(disc - cont) <= (math.pi / n) ** 2 / 12 * abs(cont) * 1.05


def test_energy_balance_with_every_source():
    n, S, E = 16, 40, 3
    rng = np.random.default_rng(1)
    th = params(E=E, dt=0.05)
    th.T_obj = rng.uniform(10, 60, E).astype(np.float32)
    pts = [[x, y, 0.0] for x in (-3e-3, -1e-3, 1e-3, 3e-3) for y in (-4e-3, -2e-3, 0.0, 2e-3, 4e-3)]
    lay = one_link_layout(pts)
    depth = rng.uniform(0, 1.5e-3, (S, E, len(pts))) * (rng.uniform(size=(S, E, len(pts))) < 0.6)
    fields = 22.0 + rng.normal(0, 2.0, (E, 1, n, n, n))
    f0 = fields.copy()
    fields, tt, led = oracle.thermal_run(th, lay, depth, fields)
    np.testing.assert_allclose(led[..., 0], led[..., 1], rtol=1e-10, atol=1e-14)
    cap = f32(th.rho_cp) * f32(th.dx) ** 3
    np.testing.assert_allclose(cap * (fields - f0).sum(axis=(1, 2, 3, 4)), led[..., 0].sum(axis=(0, 2)), rtol=1e-9)
    # taxel temperatures are the top-layer voxels under the taxels
    v = [oracle.thermal_voxel(th, p) for p in lay.pos]
    top = fields[:, 0, n - 1].reshape(E, n * n)
    np.testing.assert_array_equal(tt[-1], top[:, v])


def test_radiation_counts_exposed_faces():
    n = 16
    th = params(P_gen=0.0, T_amb=22.0)
    K = oracle.thermal_constants(th)
    fields = np.full((1, 1, n, n, n), 30.0)
    fields, _, _ = oracle.thermal_run(th, one_link_layout([[0, 0, 0]]), np.zeros((1, 1, 1)), fields)
    d = fields[0, 0] - 30.0
    faces = np.zeros((n, n, n))
    for ax in range(3):
        idx = [slice(None)] * 3
        idx[ax] = 0
        faces[tuple(idx)] += 1
        idx[ax] = n - 1
        faces[tuple(idx)] += 1
    np.testing.assert_allclose(d, -K["rho_f"] * faces * 8.0, rtol=1e-12, atol=1e-13)
    assert d[0, 0, 0] == pytest.approx(3 * d[0, 5, 5]) and d[0, 0, 5] == pytest.approx(2 * d[0, 5, 5])
    assert d[5, 5, 5] == 0.0


def test_generation_raises_temperature_uniformly():
    n, S = 16, 25
    th = params(emissivity=0.0)
    fields, _, led = oracle.thermal_run(th, one_link_layout([[0, 0, 0]]), np.zeros((S, 1, 1)))
    rise = S * f32(th.P_gen) * f32(th.dt) / (f32(th.rho_cp) * (n * f32(th.dx)) ** 3)
    np.testing.assert_allclose(fields - f32(th.T0), rise, rtol=1e-9)
    np.testing.assert_allclose(led[:, 0, 0, 1], f32(th.P_gen) * f32(th.dt), rtol=1e-12)


def test_unit_contact_conductance_reaches_object_temperature():
    n = 16
    th = params(P_gen=0.0, emissivity=0.0)
    K = oracle.thermal_constants(th)
    lay = one_link_layout([[0.5e-3, -3.2e-3, 0.0]])
    assert oracle.thermal_voxel(th, lay.pos[0]) == 4 * n + 8
    depth = np.full((1, 1, 1), 1.0 / K["kappa"])                    # kappa * depth = 1
    fields, tt, _ = oracle.thermal_run(th, lay, depth)
    assert fields[0, 0, n - 1, 4, 8] == pytest.approx(40.0, abs=1e-9)
    assert tt[0, 0, 0] == fields[0, 0, n - 1, 4, 8]
    rest = fields[0, 0].copy(); rest[n - 1, 4, 8] = 22.0
    assert np.all(rest == 22.0)


def test_stability_bound():
    th = params()
    assert oracle.thermal_stable(th, delta_max=0.031, taxels_per_voxel_max=2)
    assert not oracle.thermal_stable(params(dt=1.7), 0.0, 1)            # r = 0.17 > 1/6
    K = oracle.thermal_constants(th)
    assert not oracle.thermal_stable(th, delta_max=1.01 / K["kappa"], taxels_per_voxel_max=1)


def test_float_build_tracks_double():
    n, S = 16, 30
    rng = np.random.default_rng(3)
    th = params(E=2, dt=0.05)
    pts = [[x, y, 0.0] for x in (-1e-3, 1e-3) for y in (-2e-3, 0.0, 2e-3)]
    lay = one_link_layout(pts)
    depth = rng.uniform(0, 1e-3, (S, 2, len(pts)))
    a64, _, _ = oracle.thermal_run(th, lay, depth)
    a32, _, _ = oracle.thermal_run(th, lay, depth, precision="f32")
    assert np.abs(a32 - a64).max() < 1e-4
