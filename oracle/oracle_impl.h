/* Oracle body, included twice by oracle.c: once with REAL = float (the parity
 * oracle, following the written FP32 operation sequence) and once with
 * REAL = double (the FP64 reference).  TEST INFRASTRUCTURE ONLY.
 *
 * Macros expected: REAL, SFX(name), FMA, SQRT, FLOOR, POW, RINT.
 * Every equation cited below is from the paper (App. A: "Probe geometry and
 * contact-depth query", "ContactProbe", "KinematicTaxel", "ProximityTaxel",
 * "Sensor Noise Model"; App. B: "Tactile Observation Types").
 */

typedef struct {
  REAL R[3][3], p[3], v[3], w[3];
} SFX(pose);

/* Rotation matrix of a Hamilton unit quaternion (w,x,y,z), used as given. */
static void SFX(quat_to_R)(REAL w, REAL x, REAL y, REAL z, REAL R[3][3]) {
  REAL xx = x * x, yy = y * y, zz = z * z, xy = x * y, xz = x * z, yz = y * z;
  REAL wx = w * x, wy = w * y, wz = w * z;
  R[0][0] = (REAL)1 - (REAL)2 * (yy + zz);
  R[0][1] = (REAL)2 * (xy - wz);
  R[0][2] = (REAL)2 * (xz + wy);
  R[1][0] = (REAL)2 * (xy + wz);
  R[1][1] = (REAL)1 - (REAL)2 * (xx + zz);
  R[1][2] = (REAL)2 * (yz - wx);
  R[2][0] = (REAL)2 * (xz - wy);
  R[2][1] = (REAL)2 * (yz + wx);
  R[2][2] = (REAL)1 - (REAL)2 * (xx + yy);
}

static void SFX(load_pose)(const float* st, int64_t stride, int64_t idx, SFX(pose) * P) {
  REAL v[13];
  for (int c = 0; c < 13; ++c) v[c] = (REAL)st[c * stride + idx];
  SFX(quat_to_R)(v[3], v[4], v[5], v[6], P->R);
  for (int i = 0; i < 3; ++i) {
    P->p[i] = v[i];
    P->v[i] = v[7 + i];
    P->w[i] = v[10 + i];
  }
}

/* y = R x, each row as fma(R_i2, x2, fma(R_i1, x1, R_i0 * x0)) */
static void SFX(matvec)(REAL R[3][3], const REAL x[3], REAL y[3]) {
  for (int i = 0; i < 3; ++i) y[i] = FMA(R[i][2], x[2], FMA(R[i][1], x[1], R[i][0] * x[0]));
}
/* y = R^T x */
static void SFX(matTvec)(REAL R[3][3], const REAL x[3], REAL y[3]) {
  for (int i = 0; i < 3; ++i) y[i] = FMA(R[2][i], x[2], FMA(R[1][i], x[1], R[0][i] * x[0]));
}
static void SFX(cross)(const REAL a[3], const REAL b[3], REAL c[3]) {
  c[0] = FMA(a[1], b[2], -(a[2] * b[1]));
  c[1] = FMA(a[2], b[0], -(a[0] * b[2]));
  c[2] = FMA(a[0], b[1], -(a[1] * b[0]));
}
static REAL SFX(lerp)(REAL t, REAL a, REAL b) { return FMA(t, b - a, a); }

typedef struct {
  int active;      /* object present and R_j > 0 */
  int far;         /* query outside the grid box */
  REAL phi;        /* SDF at the probe centre (valid when active && !far) */
  REAL depth;      /* clean depth d */
  REAL prox, surf;
  REAL f[3], tau[3], mb[3];
  int nn;          /* the neural backend evaluated the network at xh */
  double xh[3];
} SFX(taxel_out);

/* One clean readout: App. A.1 probe transform and SDF depth, ContactDepthProbe,
 * KinematicTaxel force/torque, and the proximity scalar. */
static void SFX(readout)(const or_problem* P, const SFX(pose) * L, const SFX(pose) * O, int oid, int j,
                         SFX(taxel_out) * o) {
  memset(o, 0, sizeof(*o));
  o->surf = (REAL)FLT_MAX;
  const REAL Rj = (REAL)P->taxel_radius[j];
  if (oid < 0 || oid >= P->num_objects || !(Rj > 0)) return;   /* filler / no object: zeros */
  o->active = 1;
  REAL xj[3], nj[3], q[3], qo[3];
  for (int i = 0; i < 3; ++i) {
    xj[i] = (REAL)P->taxel_pos[3 * j + i];
    nj[i] = (REAL)P->taxel_normal[3 * j + i];
  }
  /* q_j = p_L + R_L x_j */
  for (int i = 0; i < 3; ++i) q[i] = FMA(L->R[i][2], xj[2], FMA(L->R[i][1], xj[1], FMA(L->R[i][0], xj[0], L->p[i])));
  /* object frame */
  if (O) {
    REAL dq[3] = {q[0] - O->p[0], q[1] - O->p[1], q[2] - O->p[2]};
    SFX(matTvec)((REAL(*)[3])O->R, dq, qo);
  } else {
    for (int i = 0; i < 3; ++i) qo[i] = q[i];
  }
  const or_grid* g = &P->grids[oid];
  REAL phi, grad[3];
  if (g->n == 0) { /* analytic sphere (pins) */
    REAL d[3];
    for (int i = 0; i < 3; ++i) d[i] = qo[i] - (REAL)g->sphere_c[i];
    REAL r = SQRT(FMA(d[2], d[2], FMA(d[1], d[1], d[0] * d[0])));
    phi = r - (REAL)g->sphere_r;
    for (int i = 0; i < 3; ++i) grad[i] = d[i];
    o->far = 0;
    o->surf = phi;
  } else {
    const int N = g->n;
    const REAL hinv = (REAL)1 / (REAL)g->spacing;
    const REAL nm1 = (REAL)(N - 1);
    REAL u[3];
    for (int i = 0; i < 3; ++i) u[i] = (qo[i] - (REAL)g->origin[i]) * hinv;
    int far = 0;
    for (int i = 0; i < 3; ++i)
      if (!(u[i] >= 0 && u[i] <= nm1)) far = 1;
    int ii[3];
    REAL t[3];
    REAL uc[3];
    for (int i = 0; i < 3; ++i) {
      uc[i] = far ? (u[i] > 0 ? (u[i] < nm1 ? u[i] : nm1) : (REAL)0) : u[i];
      int k = (int)FLOOR(uc[i]);
      if (k > N - 2) k = N - 2;
      ii[i] = k;
      t[i] = uc[i] - (REAL)k;
    }
    REAL c[2][2][2]; /* c[a][b][cz]: x offset a, y offset b, z offset cz */
    for (int cz = 0; cz < 2; ++cz)
      for (int b = 0; b < 2; ++b)
        for (int a = 0; a < 2; ++a)
          c[a][b][cz] = (REAL)g->values[((int64_t)(ii[2] + cz) * N + (ii[1] + b)) * N + (ii[0] + a)];
    REAL l00 = SFX(lerp)(t[0], c[0][0][0], c[1][0][0]);
    REAL l10 = SFX(lerp)(t[0], c[0][1][0], c[1][1][0]);
    REAL l01 = SFX(lerp)(t[0], c[0][0][1], c[1][0][1]);
    REAL l11 = SFX(lerp)(t[0], c[0][1][1], c[1][1][1]);
    REAL m0 = SFX(lerp)(t[1], l00, l10);
    REAL m1 = SFX(lerp)(t[1], l01, l11);
    phi = SFX(lerp)(t[2], m0, m1);
    if (far) {
      /* SurfaceDistanceProbe outside the box: value at the clamped point plus the
       * distance to it (an upper bound on the true distance). */
      REAL du[3];
      for (int i = 0; i < 3; ++i) du[i] = u[i] - uc[i];
      REAL dist = SQRT(FMA(du[2], du[2], FMA(du[1], du[1], du[0] * du[0]))) * (REAL)g->spacing;
      o->far = 1;
      o->surf = phi + dist;
      return;
    }
    o->surf = phi;
    if (P->sdf_mode == 1) {
      /* neural surrogate: x_hat = (q_o - c) / e over the grid box (c = centre, e = half extent,
       * both rounded to FP32 as the library does), phi_nn = e * out(x_hat); the grid stays in
       * charge inside the band |phi_nn| < nsdf_band */
      const float half = 0.5f * ((float)(N - 1) * g->spacing);
      const float einv = 1.0f / half;
      double xh[3], out, gxh[3];
      for (int i = 0; i < 3; ++i) {
        const REAL c = (REAL)(g->origin[i] + half);
        xh[i] = (double)((qo[i] - c) * (REAL)einv);
      }
      or_nsdf_forward(P->nsdf_params + (int64_t)oid * 15681, 1, xh, &out, gxh, 1);
      o->nn = 1;
      for (int i = 0; i < 3; ++i) o->xh[i] = xh[i];
      const REAL phin = (REAL)half * (REAL)out;
      if (!(FABS(phin) < (REAL)P->nsdf_band)) {
        phi = phin;
        o->surf = phi;
        for (int i = 0; i < 3; ++i) grad[i] = (REAL)gxh[i];
        goto have_sdf;
      }
    }
    /* analytic gradient of the same trilinear interpolant (direction only) */
    REAL gx = SFX(lerp)(t[2], SFX(lerp)(t[1], c[1][0][0] - c[0][0][0], c[1][1][0] - c[0][1][0]),
                        SFX(lerp)(t[1], c[1][0][1] - c[0][0][1], c[1][1][1] - c[0][1][1]));
    REAL gy = SFX(lerp)(t[2], SFX(lerp)(t[0], c[0][1][0] - c[0][0][0], c[1][1][0] - c[1][0][0]),
                        SFX(lerp)(t[0], c[0][1][1] - c[0][0][1], c[1][1][1] - c[1][0][1]));
    REAL gz = SFX(lerp)(t[1], SFX(lerp)(t[0], c[0][0][1] - c[0][0][0], c[1][0][1] - c[1][0][0]),
                        SFX(lerp)(t[0], c[0][1][1] - c[0][1][0], c[1][1][1] - c[1][1][0]));
    grad[0] = gx; grad[1] = gy; grad[2] = gz;
  }
have_sdf:
  o->phi = phi;
  /* depth d = [R_j - phi]_+ (App. A.1, SDF backend) */
  REAL diff = Rj - phi;
  REAL d = diff > 0 ? diff : (REAL)0;
  o->depth = d;
  /* proximity: normalised in-sphere point sum of a locally flat surface,
   * p = w^2 (3 - 2w) with w = clamp((R_p - phi)/R_p, 0, 1) */
  {
    const REAL Rp = (REAL)P->prox_range;
    const REAL rpinv = (REAL)1 / Rp;
    REAL w = (Rp - phi) * rpinv;
    w = w > 0 ? (w < 1 ? w : (REAL)1) : (REAL)0;
    o->prox = (w * w) * ((REAL)3 - (REAL)2 * w);
  }
  if (!(d > 0)) return;
  /* contact normal: normalised SDF gradient, world frame, then link frame */
  REAL m[3], mb[3];
  REAL n2 = FMA(grad[2], grad[2], FMA(grad[1], grad[1], grad[0] * grad[0]));
  if (n2 > 0) {
    REAL inv = (REAL)1 / SQRT(n2);
    REAL mh[3] = {grad[0] * inv, grad[1] * inv, grad[2] * inv};
    if (O) SFX(matvec)((REAL(*)[3])O->R, mh, m);
    else for (int i = 0; i < 3; ++i) m[i] = mh[i];
    SFX(matTvec)((REAL(*)[3])L->R, m, mb);
  } else {
    REAL a[3];
    SFX(matvec)((REAL(*)[3])L->R, nj, a);
    for (int i = 0; i < 3; ++i) {
      m[i] = -a[i];
      mb[i] = -nj[i];
    }
  }
  /* relative point velocity, link frame */
  REAL rL[3], cw[3], vLq[3], dv[3], dw[3], vr[3];
  for (int i = 0; i < 3; ++i) rL[i] = q[i] - L->p[i];
  SFX(cross)(L->w, rL, cw);
  for (int i = 0; i < 3; ++i) vLq[i] = L->v[i] + cw[i];
  if (O) {
    REAL rO[3], cwo[3];
    for (int i = 0; i < 3; ++i) rO[i] = q[i] - O->p[i];
    SFX(cross)(O->w, rO, cwo);
    for (int i = 0; i < 3; ++i) {
      dv[i] = (O->v[i] + cwo[i]) - vLq[i];
      dw[i] = O->w[i] - L->w[i];
    }
  } else {
    for (int i = 0; i < 3; ++i) {
      dv[i] = -vLq[i];
      dw[i] = -L->w[i];
    }
  }
  SFX(matTvec)((REAL(*)[3])L->R, dv, vr);
  /* KinematicTaxel force and torque with a Coulomb cap on the tangential part */
  REAL s = (P->alpha == 1.0f) ? d : POW(d, (REAL)P->alpha);
  REAL f[3], tau[3], cx[3];
  if (P->spring_only) {
    REAL Fn = (REAL)P->k_n * s;
    for (int i = 0; i < 3; ++i) f[i] = Fn * mb[i];
    SFX(cross)(xj, f, tau);
  } else {
    REAL vn = FMA(vr[2], mb[2], FMA(vr[1], mb[1], vr[0] * mb[0]));
    REAL vt[3], ft[3];
    for (int i = 0; i < 3; ++i) vt[i] = FMA(-vn, mb[i], vr[i]);
    REAL ks = (REAL)P->k_n * s, cs = (REAL)P->c_n * s;
    REAL Fn = FMA(cs, vn, ks);
    Fn = Fn > 0 ? Fn : (REAL)0;
    const REAL nkt = -(REAL)P->k_t;
    for (int i = 0; i < 3; ++i) ft[i] = nkt * vt[i];
    REAL ftn2 = FMA(ft[2], ft[2], FMA(ft[1], ft[1], ft[0] * ft[0]));
    REAL lim = (REAL)P->mu * Fn;
    if (ftn2 > lim * lim) {
      REAL sc = lim / SQRT(ftn2);
      for (int i = 0; i < 3; ++i) ft[i] = ft[i] * sc;
    }
    for (int i = 0; i < 3; ++i) f[i] = FMA(Fn, mb[i], ft[i]);
    REAL tw = FMA(dw[2], m[2], FMA(dw[1], m[1], dw[0] * m[0]));
    REAL kt = (REAL)P->k_w * tw;
    SFX(cross)(xj, f, cx);
    for (int i = 0; i < 3; ++i) tau[i] = FMA(-kt, mb[i], cx[i]);
  }
  for (int i = 0; i < 3; ++i) {
    o->f[i] = f[i];
    o->tau[i] = tau[i];
    o->mb[i] = mb[i];
  }
}

/* Six Gaussian deviates for (env, taxel, step t) of one stream (purpose base p0: 0 = drift,
 * 2 = white noise).  Box-Muller on pairs of uniforms from Philox4x32-10:
 *   call (env, taxel, t, p0)        -> (x0,x1) -> ch0, ch1;  (x2,x3) -> ch2, ch3
 *   call (env, taxel, t >> 1, p0+1) -> even t: (y0,y1) -> ch4, ch5;  odd t: (y2,y3) -> ch4, ch5
 * i.e. 1.5 generator calls per step; the paper fixes only the distributions. */
static void SFX(gauss6)(uint64_t seed, uint32_t env, uint32_t taxel, int64_t t, uint32_t p0, REAL g[6]) {
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t x[4], y[4];
  uint32_t c0[4] = {env, taxel, (uint32_t)t, p0};
  uint32_t c1[4] = {env, taxel, (uint32_t)(t >> 1), p0 + 1u};
  or_philox4x32_10(c0, key, x);
  or_philox4x32_10(c1, key, y);
  const int h = (int)(t & 1);
  const uint32_t pr[3][2] = {{x[0], x[1]}, {x[2], x[3]}, {y[2 * h], y[2 * h + 1]}};
  for (int i = 0; i < 3; ++i) {
    double ua = or_u01(pr[i][0]), ub = or_u01(pr[i][1]);
    double r = sqrt(-2.0 * log(ua));
    g[2 * i] = (REAL)(r * cos(2.0 * M_PI * ub));
    g[2 * i + 1] = (REAL)(r * sin(2.0 * M_PI * ub));
  }
}

int SFX(or_reset)(const or_problem* P, or_state* st, const uint8_t* env_mask, int64_t reset_step) {
  const int E = P->num_envs, T = P->num_taxels;
  const uint64_t thr64 = (uint64_t)floor((double)P->p_dead * 4294967296.0);
  uint32_t key[2] = {(uint32_t)P->seed, (uint32_t)(P->seed >> 32)};
  for (int e = 0; e < E; ++e) {
    if (env_mask && !env_mask[e]) continue;
    uint32_t ge = P->env_index ? (uint32_t)P->env_index[e] : (uint32_t)e;
    for (int j = 0; j < T; ++j) {
      int64_t k = (int64_t)e * T + j;
      for (int c = 0; c < 6; ++c) {
        if (st->drift) st->drift[(int64_t)c * E * T + k] = 0;
        if (st->hyst) st->hyst[(int64_t)c * E * T + k] = 0;
        if (st->hyst_prev) st->hyst_prev[(int64_t)c * E * T + k] = 0;
      }
      if (st->schmitt) st->schmitt[k] = 0;
      uint32_t ctr[4] = {ge, (uint32_t)j, (uint32_t)reset_step, 7u};
      uint32_t x[4];
      or_philox4x32_10(ctr, key, x);
      /* dead taxels (Bernoulli), stuck value and per-probe gain, all drawn at reset */
      if (st->dead) st->dead[k] = (uint8_t)((uint64_t)x[0] < thr64);
      REAL us = (REAL)or_u01(x[1]), ug = (REAL)or_u01(x[2]);
      if (st->stuck) st->stuck[k] = (double)FMA(us, (REAL)P->stuck_hi - (REAL)P->stuck_lo, (REAL)P->stuck_lo);
      if (st->gain) st->gain[k] = (double)FMA(ug, (REAL)P->gain_hi - (REAL)P->gain_lo, (REAL)P->gain_lo);
    }
  }
  return 0;
}

static REAL SFX(bf16)(REAL x) { return (REAL)or_bf16_round((float)x); }

int SFX(or_run)(const or_problem* P, const or_inputs* in, or_outputs* out, or_state* st, int threads) {
  const int E = P->num_envs, T = P->num_taxels, L = P->num_links;
  const int64_t ET = (int64_t)E * T, EL = (int64_t)E * L;
  double* dense = NULL;
  int64_t* dense_off = NULL;
  if (P->noise_on && P->xtalk_kind == 2) {
    int64_t tot = 0;
    dense_off = (int64_t*)malloc(sizeof(int64_t) * (L + 1));
    for (int l = 0; l < L; ++l) {
      dense_off[l] = tot;
      int64_t n = P->link_offset[l + 1] - P->link_offset[l];
      tot += n * n;
    }
    dense_off[L] = tot;
    dense = (double*)malloc(sizeof(double) * (tot > 0 ? tot : 1));
    or_dense_xtalk_f64(P, dense);
  }
  int* link_of = (int*)malloc(sizeof(int) * (T > 0 ? T : 1));
  for (int l = 0; l < L; ++l)
    for (int j = P->link_offset[l]; j < P->link_offset[l + 1]; ++j) link_of[j] = l;
  const REAL kload = (REAL)1 / (REAL)(P->tau_load > 0 ? P->tau_load : 1);
  const REAL kunload = (REAL)1 / (REAL)(P->tau_unload > 0 ? P->tau_unload : 1);
  const REAL decay = (REAL)exp(-(double)P->dt / (double)(P->maxwell_tau > 0 ? P->maxwell_tau : 1));
  const REAL qinv = P->quant_step > 0 ? (REAL)1 / (REAL)P->quant_step : (REAL)0;

  for (int s = 0; s < in->num_steps; ++s) {
    const int64_t t = in->step0 + s;
    const float* ls = in->link_state + (int64_t)s * 13 * EL;
    const int32_t* oids = in->obj_id + (int64_t)s * E;
    const float* os = in->obj_state ? in->obj_state + (int64_t)s * 13 * E : NULL;
#pragma omp parallel for num_threads(threads) schedule(dynamic, 4)
    for (int e = 0; e < E; ++e) {
      const uint32_t ge = P->env_index ? (uint32_t)P->env_index[e] : (uint32_t)e;
      SFX(pose) Opose;
      if (os) SFX(load_pose)(os, E, e, &Opose);
      const int oid = oids[e];
      REAL* z = (REAL*)malloc(sizeof(REAL) * 6 * (T > 0 ? T : 1));   /* clean F/T (x gain) per channel */
      REAL* zt = (REAL*)malloc(sizeof(REAL) * 6 * (T > 0 ? T : 1));
      REAL* fno = (REAL*)malloc(sizeof(REAL) * 6 * (T > 0 ? T : 1));
      REAL* dn = (REAL*)malloc(sizeof(REAL) * (T > 0 ? T : 1));
      uint8_t* bn = (uint8_t*)malloc(T > 0 ? T : 1);
      SFX(taxel_out)* tx = (SFX(taxel_out)*)malloc(sizeof(SFX(taxel_out)) * (T > 0 ? T : 1));
      for (int l = 0; l < L; ++l) {
        SFX(pose) Lp;
        SFX(load_pose)(ls, EL, (int64_t)e * L + l, &Lp);
        for (int j = P->link_offset[l]; j < P->link_offset[l + 1]; ++j) {
          SFX(readout)(P, &Lp, os ? &Opose : NULL, oid, j, &tx[j]);
        }
      }
      for (int j = 0; j < T; ++j) {
        const int64_t k = (int64_t)e * T + j;
        const int64_t ok = (int64_t)s * ET + k;
        SFX(taxel_out)* o = &tx[j];
        const int bit = o->depth > (REAL)P->eta_on;
        if (out->bit) out->bit[ok] = (uint8_t)bit;
        if (out->depth) out->depth[ok] = (double)o->depth;
        if (out->prox) out->prox[ok] = (double)o->prox;
        if (out->surfdist) out->surfdist[ok] = (double)o->surf;
        if (out->xhat)
          for (int c = 0; c < 3; ++c) out->xhat[(int64_t)s * 3 * ET + (int64_t)c * ET + k] = o->nn ? o->xh[c] : NAN;
        for (int c = 0; c < 3; ++c) {
          if (out->ft) {
            out->ft[(int64_t)s * 6 * ET + (int64_t)c * ET + k] = (double)o->f[c];
            out->ft[(int64_t)s * 6 * ET + (int64_t)(c + 3) * ET + k] = (double)o->tau[c];
          }
          if (out->normal) out->normal[(int64_t)s * 3 * ET + (int64_t)c * ET + k] = (double)o->mb[c];
        }
      }
      if (P->noise_on) {
        /* 1. per-probe gain, drawn at reset */
        for (int j = 0; j < T; ++j) {
          const int64_t k = (int64_t)e * T + j;
          REAL gn = st->gain ? (REAL)st->gain[k] : (REAL)1;
          for (int c = 0; c < 3; ++c) {
            z[c * T + j] = gn * tx[j].f[c];
            z[(c + 3) * T + j] = gn * tx[j].tau[c];
          }
        }
        /* 2. spatial crosstalk within each link */
        for (int l = 0; l < L; ++l) {
          const int a = P->link_offset[l], b = P->link_offset[l + 1], n = b - a;
          for (int c = 0; c < 6; ++c) {
            const REAL* zc = z + c * T;
            REAL* ztc = zt + c * T;
            for (int jj = 0; jj < n; ++jj) {
              const int j = a + jj;
              double scale = 0;
              if (P->xtalk_kind == 1) {
                const REAL chi = (REAL)P->xtalk_chi;
                int deg = (jj > 0) + (jj < n - 1);
                REAL acc = ((REAL)1 - chi * (REAL)deg) * zc[j];
                if (jj > 0) acc = FMA(chi, zc[j - 1], acc);
                if (jj < n - 1) acc = FMA(chi, zc[j + 1], acc);
                ztc[j] = acc;
                scale = fabs((double)(((REAL)1 - chi * (REAL)deg) * zc[j])) +
                        (jj > 0 ? fabs((double)chi * (double)zc[j - 1]) : 0) +
                        (jj < n - 1 ? fabs((double)chi * (double)zc[j + 1]) : 0);
              } else if (P->xtalk_kind == 2) {
                const double* Cl = dense + dense_off[l] + (int64_t)jj * n;
                double acc = 0;
                for (int kk = 0; kk < n; ++kk) {
                  double cw, zv;
                  if (sizeof(REAL) == 4) { /* BF16 operands, exact products, wide accumulation */
                    cw = (double)or_bf16_round((float)Cl[kk]);
                    zv = (double)SFX(bf16)(zc[a + kk]);
                  } else {
                    cw = Cl[kk];
                    zv = (double)zc[a + kk];
                  }
                  acc += cw * zv;
                  scale += fabs(cw) * fabs(zv);
                }
                ztc[j] = (REAL)acc;
              } else {
                ztc[j] = zc[j];
                scale = fabs((double)zc[j]);
              }
              if (out->xtalk_scale) out->xtalk_scale[(int64_t)s * 6 * ET + (int64_t)c * ET + (int64_t)e * T + j] = scale;
            }
          }
        }
        /* 3. hysteresis, 4. bias + white + drift, 5. quantisation, 6. dead overwrite */
        for (int j = 0; j < T; ++j) {
          const int64_t k = (int64_t)e * T + j;
          const int dead = st->dead ? st->dead[k] : 0;
          REAL gd[6] = {0, 0, 0, 0, 0, 0}, gw[6] = {0, 0, 0, 0, 0, 0};
          if (P->drift_sigma != 0) SFX(gauss6)(P->seed, ge, (uint32_t)j, t, 0u, gd);
          if (P->white_sigma != 0) SFX(gauss6)(P->seed, ge, (uint32_t)j, t, 2u, gw);
          for (int c = 0; c < 6; ++c) {
            const int64_t sk = (int64_t)c * ET + k;
            REAL x = zt[c * T + j];
            REAL h = x;
            if (P->hyst_mode == 1) {
              REAL y = (REAL)st->hyst[sk];
              REAL kap = (FABS(x) > FABS(y)) ? kload : kunload;
              y = FMA(kap, x - y, y);
              st->hyst[sk] = (double)y;
              h = y;
            } else if (P->hyst_mode == 2) {
              REAL xi = (REAL)st->hyst[sk], xp = (REAL)st->hyst_prev[sk];
              xi = FMA(decay, xi, x - xp);
              st->hyst[sk] = (double)xi;
              st->hyst_prev[sk] = (double)x;
              h = FMA((REAL)P->maxwell_beta, xi, x);
            }
            REAL o = h;
            if (P->bias != 0) o = o + (REAL)P->bias;
            if (P->white_sigma != 0) o = FMA((REAL)P->white_sigma, gw[c], o);
            if (P->drift_sigma != 0) {
              REAL D = FMA((REAL)P->drift_sigma, gd[c], (REAL)st->drift[sk]);
              st->drift[sk] = (double)D;
              o = o + D;
            }
            if (P->quant_step > 0) o = (REAL)P->quant_step * RINT(o * qinv);
            if (dead) o = (REAL)st->stuck[k];
            fno[c * T + j] = o;
            if (out->ft_noisy) out->ft_noisy[(int64_t)s * 6 * ET + sk] = (double)o;
          }
          /* noisy contact bit: radius noise, Schmitt hysteresis, dead overwrite */
          SFX(taxel_out)* o = &tx[j];
          REAL dd = o->depth;
          if (P->radius_rho > 0) {
            dd = 0;
            if (o->active && !o->far) {
              uint32_t key[2] = {(uint32_t)P->seed, (uint32_t)(P->seed >> 32)};
              uint32_t ctr[4] = {ge, (uint32_t)j, (uint32_t)t, 6u}, x[4];
              or_philox4x32_10(ctr, key, x);
              REAL u = (REAL)or_u01(x[0]);
              REAL rho = (REAL)P->radius_rho;
              REAL Rn = (REAL)P->taxel_radius[j] + FMA(u, (REAL)2 * rho, -rho);
              Rn = Rn > 0 ? Rn : (REAL)0;
              REAL df = Rn - o->phi;
              dd = df > 0 ? df : (REAL)0;
            }
          }
          int prev = st->schmitt[k];
          int nb = (dd > (REAL)P->eta_on) || (prev && dd > (REAL)P->eta_off);
          if (dead) {
            nb = 0;
            dd = 0;
          }
          st->schmitt[k] = (uint8_t)nb;
          bn[j] = (uint8_t)nb;
          dn[j] = dd;
          if (out->bit_noisy) out->bit_noisy[(int64_t)s * ET + k] = (uint8_t)nb;
        }
      }
      /* per-link observations (App. B): force/torque sums, contact count, agg_bool, agg_force */
      for (int pass = 0; pass < 2; ++pass) {
        double* dst = pass == 0 ? out->link_sums : out->link_sums_noisy;
        if (!dst || (pass == 1 && !P->noise_on)) continue;
        for (int l = 0; l < L; ++l) {
          REAL acc[11];
          for (int c = 0; c < 11; ++c) acc[c] = 0;
          int cnt = 0;
          for (int j = P->link_offset[l]; j < P->link_offset[l + 1]; ++j) {
            for (int c = 0; c < 6; ++c)
              acc[c] += pass == 0 ? (c < 3 ? tx[j].f[c] : tx[j].tau[c - 3]) : fno[c * T + j];
            REAL dj = pass == 0 ? tx[j].depth : dn[j];
            int bj = pass == 0 ? (tx[j].depth > (REAL)P->eta_on) : bn[j];
            cnt += bj;
            acc[8] += dj * (REAL)P->taxel_normal[3 * j + 2];
            acc[9] += dj * (REAL)P->taxel_normal[3 * j + 1];
            acc[10] += dj * (REAL)P->taxel_normal[3 * j + 0];
          }
          int64_t base = (int64_t)s * 11 * EL + (int64_t)e * L + l;
          for (int c = 0; c < 6; ++c) dst[base + (int64_t)c * EL] = (double)acc[c];
          dst[base + 6 * EL] = (double)cnt;
          dst[base + 7 * EL] = cnt > 2 ? 1.0 : 0.0;
          for (int c = 8; c < 11; ++c) dst[base + (int64_t)c * EL] = 1.0e4 * (double)acc[c];
        }
      }
      free(z); free(zt); free(fno); free(dn); free(bn); free(tx);
    }
  }
  free(link_of);
  free(dense);
  free(dense_off);
  return 0;
}
