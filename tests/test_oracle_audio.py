"""Pins of the contact-audio oracle (App. E, contact audio: source-filter modal synthesis).

- Closed form of the two-pole resonator: after an impulse A at sample 0 from rest, a mode reads
  y[k] = A r^k sin((k + 1) theta) / sin(theta), theta = 2 pi f dt_sub, across block boundaries (the
  states carry over); a wrong sign of a2, a missing factor 2 in a1, or dropped state fails it.
- Only a rise of the normal force pings the bank: a hold or a fall adds nothing, a rise adds exactly
  g_imp times the rise.
- Superposition: the output is linear in the excitation (impact + scrape = impact alone + scrape
  alone), and a bank's output is the gain-weighted sum of its single-mode banks.
- Scrape noise: uniform on (-1, 1) (Kolmogorov-Smirnov), exact in FP32, one stream per (env, link,
  step); a noise-driven mode settles at the AR(2) variance sigma^2 (1 + a2) / ((1 - a2)((1 + a2)^2 - a1^2)).
- The ring-down's zero crossings repeat at half the mode's period.
- Excitation: a taxel force 3 m + 4 t (t a unit vector normal to the contact normal m) gives
  F_n = 3 and F_t = 4; tangential parts add as magnitudes; only the sensor link's taxels count.
- Silent slots and out-of-range materials.
"""
import numpy as np
import pytest
from scipy import stats

from oracle import audio as A


def run(Fn, Ft, banks, dt, K, g_imp, g_scr, seed=0, material=None, slots=None, **kw):
    Fn = np.asarray(Fn, float)
    E = Fn.shape[1]
    material = np.zeros(E, int) if material is None else material
    slots = max(len(b[0]) for b in banks) if slots is None else slots
    return A.contact_audio(Fn, Ft, material, banks, slots, dt, K, g_imp, g_scr, seed, **kw)


def single(f, d, g=1.0):
    return (np.array([f], float), np.array([d], float), np.array([g], float))


def step_force(S, rise_at=0, F=2.0):
    Fn = np.zeros((S, 1, 1))
    Fn[rise_at:] = F
    return Fn, np.zeros_like(Fn)


@pytest.mark.parametrize("f,d", [(440.0, 30.0), (3000.0, 200.0), (11000.0, 5.0)])
def test_impulse_response_closed_form(f, d):
    dt, K, S = 0.005, 240, 3
    out = run(*step_force(S, F=1.5), [single(f, d, 0.7)], dt, K, g_imp=2.0, g_scr=0.0)
    dts = dt / K
    r, th = np.exp(-d * dts), 2 * np.pi * f * dts
    k = np.arange(S * K)
    want = 0.7 * 2.0 * 1.5 * r ** k * np.sin((k + 1) * th) / np.sin(th)
    np.testing.assert_allclose(out.reshape(-1), want, rtol=0, atol=1e-9 * np.abs(want).max())


def test_only_a_rise_of_the_normal_force_pings():
    dt, K = 0.004, 64
    Fn = np.array([0.0, 3.0, 3.0, 1.0, 4.0])[:, None, None]          # rise 3, hold, fall, rise 3
    m = [single(800.0, 50.0)]
    out = run(Fn, np.zeros_like(Fn), m, dt, K, 1.0, 0.0).reshape(5, K)
    base = run(*step_force(5, rise_at=1, F=3.0), m, dt, K, 1.0, 0.0).reshape(5, K)
    np.testing.assert_allclose(out[:4], base[:4], rtol=0, atol=1e-12)
    late = run(*step_force(5, rise_at=4, F=3.0), m, dt, K, 1.0, 0.0).reshape(5, K)
    np.testing.assert_allclose(out[4], base[4] + late[4], rtol=0, atol=1e-12)
    assert np.all(out[0] == 0)


def test_superposition_and_gain_weighted_sum():
    rng = np.random.default_rng(7)
    S, E, Ls, K, dt = 4, 2, 2, 48, 0.005
    Fn, Ft = rng.uniform(0, 2, (S, E, Ls)), rng.uniform(0, 1, (S, E, Ls))
    banks = [(np.array([500.0, 1700.0, 4100.0]), np.array([20.0, 80.0, 300.0]), np.array([1.0, -0.5, 0.25])),
             (np.array([900.0]), np.array([10.0]), np.array([2.0]))]
    mat = np.array([0, 1])
    both = run(Fn, Ft, banks, dt, K, 0.8, 0.3, seed=11, material=mat)
    imp = run(Fn, Ft, banks, dt, K, 0.8, 0.0, seed=11, material=mat)
    scr = run(Fn, Ft, banks, dt, K, 0.0, 0.3, seed=11, material=mat)
    np.testing.assert_allclose(both, imp + scr, rtol=0, atol=1e-12)
    b0 = banks[0]
    per_mode = sum(run(Fn[:, :1], Ft[:, :1], [(b0[0][i:i + 1], b0[1][i:i + 1], b0[2][i:i + 1])], dt, K, 0.8, 0.3,
                       seed=11) for i in range(3))
    np.testing.assert_allclose(both[:, :1], per_mode, rtol=0, atol=1e-12)


def test_scrape_noise_is_uniform_exact_and_per_stream():
    xi = np.concatenate([A.noise_block(0x1234_5678_9ABC, e, l, t, 64) for e in range(4) for l in range(3)
                         for t in range(20)])
    assert stats.kstest(xi, "uniform", args=(-1, 2)).pvalue > 1e-3
    assert np.array_equal(xi.astype(np.float32).astype(np.float64), xi)
    assert np.all(np.abs(xi) < 1)
    a, b, c = A.noise_block(5, 0, 0, 0, 8), A.noise_block(5, 0, 0, 1, 8), A.noise_block(5, 0, 1, 0, 8)
    assert not np.allclose(a, b) and not np.allclose(a, c)
    assert np.array_equal(A.noise_block(5, 0, 0, 0, 6), a[:6])          # a ragged block is a prefix


def test_noise_driven_mode_settles_at_the_ar2_variance():
    f, d, dt, K, S = 2000.0, 400.0, 0.005, 240, 150
    Ft = np.ones((S, 1, 1))
    out = run(np.zeros_like(Ft), Ft, [single(f, d)], dt, K, 0.0, 1.0, seed=3).reshape(-1)
    dts = dt / K
    r = np.exp(-d * dts)
    a1, a2 = 2 * r * np.cos(2 * np.pi * f * dts), r * r
    var = (1.0 / 3.0) * (1 + a2) / ((1 - a2) * ((1 + a2) ** 2 - a1 ** 2))
    assert np.var(out[K * 20:]) == pytest.approx(var, rel=0.1)          # past the 1 / d settling time


def test_ring_down_zero_crossings():
    f, dt, K = 1000.0, 0.01, 480                                        # 48 kHz: 48 samples a period
    out = run(*step_force(1), [single(f, 5.0)], dt, K, 1.0, 0.0).reshape(-1)
    z = np.nonzero(np.sign(out[:-1]) != np.sign(out[1:]))[0]
    assert np.all(np.abs(np.diff(z) - 24) <= 1)


def test_link_excitation_splits_the_force_law():
    S, E, T = 1, 2, 5
    link_offset = [0, 2, 5]
    ft = np.zeros((S, 6, E, T))
    nm = np.zeros((S, 3, E, T))
    m = np.array([0.0, 0.6, 0.8])
    t = np.array([1.0, 0.0, 0.0])
    t2 = np.array([0.0, 0.8, -0.6])                                     # also normal to m
    for j, (fm, tt) in zip([2, 3], [(3.0, 4.0 * t), (1.0, -4.0 * t)]):
        ft[0, 0:3, 0, j] = fm * m + tt
        nm[0, :, 0, j] = m
    ft[0, 0:3, 0, 4] = 2.0 * m + 1.5 * t2
    nm[0, :, 0, 4] = m
    ft[0, 0:3, 0, 0] = 7.0 * m                                          # link 0: not a sensor link
    nm[0, :, 0, 0] = m
    ft[0, 3:6] = 99.0                                                   # torques are not read
    Fn, Ft = A.link_excitation(ft, nm, link_offset, [1])
    assert Fn[0, 0, 0] == pytest.approx(6.0, abs=1e-12)
    assert Ft[0, 0, 0] == pytest.approx(9.5, abs=1e-12)                 # magnitudes add: 4 + 4 + 1.5
    assert Fn[0, 1, 0] == 0 and Ft[0, 1, 0] == 0


def test_silent_slots_and_out_of_range_material():
    rng = np.random.default_rng(2)
    Fn, Ft = rng.uniform(0, 1, (3, 3, 1)), rng.uniform(0, 1, (3, 3, 1))
    banks = [single(700.0, 40.0)]
    out = run(Fn, Ft, banks, 0.005, 32, 1.0, 1.0, seed=4, material=np.array([-1, 0, 5]), slots=4)
    assert np.all(out[:, 0] == 0) and np.all(out[:, 2] == 0) and np.any(out[:, 1] != 0)
    # padding the bank with silent slots changes nothing audible
    one = run(Fn, Ft, banks, 0.005, 32, 1.0, 1.0, seed=4, material=np.array([-1, 0, 5]), slots=1)
    np.testing.assert_allclose(out, one, rtol=0, atol=1e-15)


def test_env_subset_keeps_its_noise_streams():
    rng = np.random.default_rng(9)
    Fn, Ft = rng.uniform(0, 1, (2, 5, 1)), rng.uniform(0, 1, (2, 5, 1))
    banks = [single(900.0, 30.0)]
    full = run(Fn, Ft, banks, 0.005, 16, 1.0, 1.0, seed=2)
    envs = np.array([1, 4])
    sub = run(Fn[:, envs], Ft[:, envs], banks, 0.005, 16, 1.0, 1.0, seed=2, env_ids=envs)
    np.testing.assert_array_equal(sub, full[:, envs])
