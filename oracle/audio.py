"""Oracle of the contact-audio sensor: source-filter modal synthesis driven by the contacts of a
sensor link (App. E, contact audio).  TEST INFRASTRUCTURE ONLY.  FP64 numpy, sample by sample.

Each physics step of length dt emits K samples at dt_sub = dt / K.  A material is a bank of modes
(f_i, d_i, g_i); mode i is the two-pole resonator
  y_i[k] = a1_i y_i[k-1] - a2_i y_i[k-2] + u[k],   a1_i = 2 r_i cos(2 pi f_i dt_sub),  a2_i = r_i^2,
  r_i = exp(-d_i dt_sub),
and the emitted sample is s[k] = sum_i g_i y_i[k].  Readings where the paper leaves the form open:
  - the excitation of a sensor link comes from its taxels' kinematic force law: with f_j the taxel
    force and m_j its contact normal (both link frame, as the readout reports them), the normal force
    is F_n = sum_j f_j . m_j and the friction F_t = sum_j |f_j - (f_j . m_j) m_j| (the tangential
    part, which the law scales with the slip velocity and caps by mu F_n);
  - impact: a rise of F_n since the previous step adds g_imp * max(0, F_n(t) - F_n(t-1)) to the
    block's first sample;
  - scrape: F_t drives white noise g_scr * F_t * xi[k] over the whole block, xi uniform on (-1, 1):
    xi[k] = 2 u - 1 with u = (2 (w >> 9) + 1) 2^-24 from word k mod 4 of Philox4x32-10 at counter
    (env, 2^31 + sensor link, step, k / 4);
  - the bank has a fixed number of slots; a material with fewer modes fills the rest with silent
    slots (a1 = a2 = g = 0, so y = u there), and an env whose material id is out of range has every
    slot silent.  Slot states carry over from step to step and across calls.
"""
from __future__ import annotations

import numpy as np

from . import oracle as _o


def link_excitation(ft, normal, link_offset, sensor_links):
    """ft [S][6][E][T] taxel force/torque and normal [S][3][E][T] contact normals (link frame).
    Returns (F_n, F_t), each [S][E][Ls]."""
    ft = np.asarray(ft, np.float64)
    normal = np.asarray(normal, np.float64)
    S, _, E, _ = ft.shape
    Ls = len(sensor_links)
    Fn, Ft = np.zeros((S, E, Ls)), np.zeros((S, E, Ls))
    for li, l in enumerate(sensor_links):
        for j in range(link_offset[l], link_offset[l + 1]):
            f = ft[:, 0:3, :, j]                       # [S][3][E]
            m = normal[:, :, :, j]
            fn = np.sum(f * m, axis=1)                  # [S][E]
            t = f - fn[:, None, :] * m
            Fn[:, :, li] += fn
            Ft[:, :, li] += np.sqrt(np.sum(t * t, axis=1))
    return Fn, Ft


def bank_coefficients(banks, slots, dt_sub):
    """banks: list of (f, d, g) arrays.  Returns (a1, a2, g), each [len(banks)][slots], zero-padded."""
    nb = len(banks)
    a1, a2, g = np.zeros((nb, slots)), np.zeros((nb, slots)), np.zeros((nb, slots))
    for b, (f, d, gg) in enumerate(banks):
        f, d, gg = (np.asarray(x, np.float64) for x in (f, d, gg))
        n = len(f)
        if n > slots:
            raise ValueError("more modes than slots")
        r = np.exp(-d * dt_sub)
        a1[b, :n] = 2.0 * r * np.cos(2.0 * np.pi * f * dt_sub)
        a2[b, :n] = r * r
        g[b, :n] = gg
    return a1, a2, g


def noise_block(seed, env, link, step, K):
    """xi[0..K) of one block, uniform on (-1, 1), exact in FP32."""
    key = [seed & 0xffffffff, (seed >> 32) & 0xffffffff]
    out = np.zeros(K)
    for c in range((K + 3) // 4):
        w = _o.philox4x32_10([env, 0x80000000 + link, step, c], key)
        for i in range(4):
            k = 4 * c + i
            if k < K:
                out[k] = 2.0 * _o.u01(int(w[i])) - 1.0
    return out


def new_state(E, Ls, slots):
    return {"y1": np.zeros((E, Ls, slots)), "y2": np.zeros((E, Ls, slots)), "fn": np.zeros((E, Ls))}


def contact_audio(Fn, Ft, material, banks, slots, dt, K, g_imp, g_scr, seed, step0=0, state=None, env_ids=None):
    """Fn, Ft [S][E][Ls] link excitations; material [E] bank index per env (out of range: silent);
    banks: list of (f, d, g).  state (new_state(...) or None: at rest) is updated in place.
    env_ids [E]: the env index of each row in the noise counter (default 0..E-1, for a subset of
    envs their indices in the full batch).  Returns the samples [S][E][Ls][K]."""
    Fn = np.asarray(Fn, np.float64)
    Ft = np.asarray(Ft, np.float64)
    S, E, Ls = Fn.shape
    if state is None:
        state = new_state(E, Ls, slots)
    if env_ids is None:
        env_ids = np.arange(E)
    dts = dt / K
    A1, A2, G = bank_coefficients(banks, slots, dts)
    zero = np.zeros(slots)
    out = np.zeros((S, E, Ls, K))
    for e in range(E):
        m = int(material[e])
        ok = 0 <= m < len(banks)
        a1, a2, g = (A1[m], A2[m], G[m]) if ok else (zero, zero, zero)
        for l in range(Ls):
            y1, y2 = state["y1"][e, l].copy(), state["y2"][e, l].copy()
            fn_prev = state["fn"][e, l]
            for s in range(S):
                xi = noise_block(seed, int(env_ids[e]), l, step0 + s, K)
                imp = g_imp * max(0.0, Fn[s, e, l] - fn_prev)
                amp = g_scr * Ft[s, e, l]
                for k in range(K):
                    u = amp * xi[k] + (imp if k == 0 else 0.0)
                    y = a1 * y1 - a2 * y2 + u
                    y2, y1 = y1, y
                    out[s, e, l, k] = float(np.dot(g, y))
                fn_prev = Fn[s, e, l]
            state["y1"][e, l], state["y2"][e, l] = y1, y2
            state["fn"][e, l] = fn_prev
    return out
