"""Oracle of the paper's TemperatureGrid step with its spectral diffusion and sensor element lag
(App. D.1).  TEST INFRASTRUCTURE ONLY.  FP64 numpy; the FFT is numpy's.

Per field (one n^3 voxel block per env and thermal link, link frame, index [z][y][x], top layer
z = n - 1), per step, in the paper's order:
  1. diffusion, semi-implicit and spectral with zero-flux walls: the block is mirror-padded to 2n
     along each axis, transformed by a real FFT, every mode divided by 1 + alpha dt k^2 (k the
     wavenumber vector of the padded grid, k^2 floored at eps), transformed back and cropped;
  2. the internal source: dT = g in every voxel (the configured power spread over the block);
  3. contact conduction into the top-layer voxel under each taxel: dT = c_v (T_obj - T),
     c_v = kappa * (sum of the clean depths of the taxels over the voxel);
  4. radiation (grey body, Stefan-Boltzmann, in kelvin) and convection (Newton) from every voxel
     on the block surface, per exposed face: dT = -dt faces (eps sigma (T_K^4 - T_amb,K^4)
     + h (T - T_amb)) / (rho c_p dx);
  5. the measured reading of each taxel, T_meas <- T_meas + (dt / tau) (T_voxel - T_meas), tau <= 0
     reporting T_voxel itself.
g, kappa and the face count are those of the explicit solver (thermal.c): the two solvers differ in
the diffusion step, the radiation law (full T^4 here, linearised there) and the lag.
"""
from __future__ import annotations

import numpy as np

SIGMA_SB = 5.670374419e-8


def spectral_diffusion(T, alpha, dt, dx, eps=1e-12):
    """One implicit spectral diffusion step of the n^3 block T[z][y][x] with zero-flux walls."""
    T = np.asarray(T, np.float64)
    n = T.shape
    P = T
    for ax in range(3):
        P = np.concatenate([P, np.flip(P, axis=ax)], axis=ax)
    F = np.fft.rfftn(P)
    kz = 2 * np.pi * np.fft.fftfreq(2 * n[0], d=dx)
    ky = 2 * np.pi * np.fft.fftfreq(2 * n[1], d=dx)
    kx = 2 * np.pi * np.fft.rfftfreq(2 * n[2], d=dx)
    k2 = kz[:, None, None] ** 2 + ky[None, :, None] ** 2 + kx[None, None, :] ** 2
    F = F / (1.0 + alpha * dt * np.maximum(k2, eps))
    return np.fft.irfftn(F, s=P.shape, axes=(0, 1, 2))[:n[0], :n[1], :n[2]]


def surface_faces(n):
    """Exposed faces of each voxel of an n^3 block, [z][y][x]."""
    i = np.arange(n)
    e = (i == 0).astype(np.int64) + (i == n - 1)
    return e[:, None, None] + e[None, :, None] + e[None, None, :]


def spectral_run(th, layout, depth, fields=None, h_conv=0.0, tau=0.0, t_meas=None, eps=1e-12):
    """S steps of every field (S, E, T from depth [S][E][T], the clean depths).  th: synth.ThermalParams;
    g, kappa and the top-layer voxel of each taxel are the explicit solver's (thermal.c).
    fields [E][F][n][n][n] initial state (default T0 everywhere) and t_meas [E][T] (default T0) are
    updated in place.  Returns (fields, measured taxel temperatures [S][E][T], 0 off the fields)."""
    from . import oracle as _o
    depth = np.asarray(depth, np.float64)
    S, E, T = depth.shape
    n, dx, dt = th.n, float(np.float32(th.dx)), float(np.float32(th.dt))
    rc, em, Ta = float(np.float32(th.rho_cp)), float(np.float32(th.emissivity)), float(np.float32(th.T_amb))
    K = _o.thermal_constants(th)
    F = len(th.field_links)
    if fields is None:
        fields = np.full((E, F, n, n, n), float(np.float32(th.T0)))
    if t_meas is None:
        t_meas = np.full((E, T), float(np.float32(th.T0)))
    faces = surface_faces(n).astype(np.float64)
    off = layout.link_offset
    vox = {j: _o.thermal_voxel(th, layout.pos[j]) for l in th.field_links for j in range(off[l], off[l + 1])}
    tobj = np.asarray(th.T_obj, np.float32).astype(np.float64)
    out = np.zeros((S, E, T))
    for s in range(S):
        for e in range(E):
            for f, l in enumerate(th.field_links):
                Tf = spectral_diffusion(fields[e, f], K["alpha"], dt, dx, eps)
                Tf = Tf + K["g"]
                cv = np.zeros(n * n)
                for j in range(off[l], off[l + 1]):
                    cv[vox[j]] += K["kappa"] * depth[s, e, j]
                top = Tf[n - 1].reshape(-1)
                Tf[n - 1] = (top + cv * (tobj[e] - top)).reshape(n, n)
                TK, TaK = Tf + 273.15, Ta + 273.15
                q = em * SIGMA_SB * (TK ** 4 - TaK ** 4) + h_conv * (Tf - Ta)
                Tf = Tf - dt * faces * q / (rc * dx)
                fields[e, f] = Tf
                top = Tf[n - 1].reshape(-1)
                for j in range(off[l], off[l + 1]):
                    if tau > 0:
                        t_meas[e, j] = t_meas[e, j] + (dt / tau) * (top[vox[j]] - t_meas[e, j])
                        out[s, e, j] = t_meas[e, j]
                    else:
                        out[s, e, j] = top[vox[j]]
    return fields, out
