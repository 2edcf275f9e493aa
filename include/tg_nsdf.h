/* tg_nsdf — per-object neural signed-distance surrogate on one MI355X (gfx950).
 *
 * The network stands in for an object's SDF grid (App. A.1, sdf backend: the readout only
 * needs phi and grad phi at the probe centres).  Per object:
 *   x_hat = (q_o - c) / e, the object-frame point mapped from the grid box (centre c,
 *           half extent e = (n-1)*spacing/2) to [-1,1]^3
 *   features: sin(2^k pi x_hat_d), cos(2^k pi x_hat_d), k = 0..7, ordered
 *           [sin k=0 (x,y,z), cos k=0 (x,y,z), sin k=1 (x,y,z), ...]      (48)
 *   4 hidden layers of width 64 with SiLU, then one linear output "out";  phi = e * out.
 * Parameters, FP32, flat and per object (TG_NSDF_NUM_PARAMS = 15681 floats):
 *   W1[64][48], b1[64], W2[64][64], b2[64], W3[64][64], b3[64], W4[64][64], b4[64], w5[64], b5.
 * The hidden layers run on BF16 MFMA with FP32 accumulation: weights and layer inputs are
 * rounded to BF16, pre-activations are rounded to BF16 before SiLU, the output layer is FP32.
 *
 * Training sample record (device, FP32, 16 bytes): { x_hat[3], phi / e }; optional gradient
 * record (16 bytes): { d phi / d q [3], 0 }, the grid's gradient at the same point, which is also
 * d(phi / e) / d x_hat.
 * Training loss: mean |out - phi/e| over the minibatch (L1), optionally plus a pair term and a
 * gradient term (below); optimiser Adam (Kingma & Ba) with bias correction, FP32 master weights
 * and moments owned by the caller.
 *
 * Conventions are those of tg_readout.h: device pointers are caller-owned HIP memory valid
 * until the queued work finishes; host pointers are read during the call; entry points
 * return a tg_status, launch nothing on error, never synchronise and never throw.
 */
#ifndef TG_NSDF_H
#define TG_NSDF_H
#include <stddef.h>
#include <stdint.h>

#include "tg_readout.h"

#ifdef __cplusplus
extern "C" {
#endif

#define TG_NSDF_NUM_PARAMS 15681

typedef struct tg_nsdf tg_nsdf; /* opaque handle: device copies of the grids + packed weights */

typedef struct {
  uint32_t abi_version;     /* TG_ABI_VERSION */
  int32_t num_objects;      /* >= 1 */
  const tg_sdf_grid* grids; /* host [num_objects]; deep-copied (targets, box of each object) */
} tg_nsdf_config;

typedef struct {
  float lr, beta1, beta2, eps; /* Adam; e.g. 1e-3, 0.9, 0.999, 1e-8 */
  int32_t batch;               /* samples per object per step, a multiple of 64 */
  uint64_t seed;               /* Philox4x32-10 key of the minibatch draw */
  float pair_lambda;           /* 0: plain L1 loss.  > 0: records 2i and 2i+1 form a pair (n even)
                                  and the loss adds pair_lambda * |r_2i+1 - r_2i| per pair, the
                                  error of the difference across the pair (a first-order hold on
                                  the slope between nearby points), divided by the batch */
  float grad_lambda;           /* 0: no gradient term.  > 0: the loss adds grad_lambda * sum_d
                                  |g_d - gt_d| per record, divided by the batch, where g = d out /
                                  d x_hat is the network's input gradient (the normal source of
                                  App. A.1) and gt the record's gradient record; the training call
                                  then needs grad_samples.  Its parameter gradient runs a
                                  forward-mode tangent pass along sign(g - gt) and differentiates
                                  it in reverse mode (second derivatives of SiLU enter) */
} tg_nsdf_train_params;

/* Create / destroy.  create copies the grids to the device and allocates one packed BF16
 * weight image per object (about 64 KiB each). */
tg_status tg_nsdf_create(const tg_nsdf_config* cfg, tg_nsdf** out);
tg_status tg_nsdf_destroy(tg_nsdf* h); /* NULL is OK */
const char* tg_nsdf_last_error(const tg_nsdf* h);

/* Training targets from the grids.  points: device [num_objects][n][3] object-frame
 * positions [m]; each is clamped into its object's grid box, then samples[o][i] receives
 * { x_hat, phi_grid / e } with phi_grid the trilinear value of the grid (App. A.1), and
 * grad_samples[o][i] (device [num_objects][n][4], or NULL to skip) receives { d phi_grid / d q, 0 },
 * the analytic gradient of the same interpolant at the clamped point.
 * samples: device [num_objects][n][4].  Both 16-byte aligned. */
tg_status tg_nsdf_targets(tg_nsdf* h, const float* points, int64_t n, float* samples, float* grad_samples,
                          void* hip_stream);

/* Full-batch loss gradient: for every object o, grad[o] = d/dP of the loss over the n records
 * samples[o][0..n) and loss[o] = that loss: mean_i |out(x_i) - t_i|, plus, for pair_lambda > 0
 * (n even), pair_lambda * sum over pairs |r_2i+1 - r_2i| / n, plus, for grad_lambda > 0,
 * grad_lambda * sum_i sum_d |g_i,d - gt_i,d| / n with gt from grad_samples[o][0..n) (device
 * [num_objects][n][4], or NULL when grad_lambda = 0).  params: device [num_objects][15681]; grad:
 * device [num_objects][15681] (written); loss: device [num_objects] or NULL.
 * TG_ERR_INVALID_ARGUMENT for a negative lambda, an odd n with pair_lambda > 0, or grad_lambda > 0
 * without grad_samples. */
tg_status tg_nsdf_grad(tg_nsdf* h, const float* params, const float* samples, const float* grad_samples, int64_t n,
                       float pair_lambda, float grad_lambda, float* grad, float* loss, void* hip_stream);

/* One Adam step over count contiguous parameters at step number t (>= 1):
 *   m = b1 m + (1-b1) g;  v = b2 v + (1-b2) g^2;  p -= lr (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps). */
tg_status tg_nsdf_adam(float* params, float* m, float* v, const float* grad, int64_t count, int64_t t,
                       const tg_nsdf_train_params* hp, void* hip_stream);

/* n_steps fused training steps (steps step0+1 .. step0+n_steps), all objects at once, one
 * workgroup per object.  Each step draws hp->batch record indices per object uniformly from
 * [0, n): Philox4x32-10 with key (seed low, seed high) and counter (object, step, j / 4, 8),
 * word j % 4, index = (word * n) >> 32; with hp->pair_lambda > 0 it draws pairs instead: counter
 * (object, step, j / 8, 8), word (j / 2) % 4, pair = (word * n/2) >> 32, index = 2 pair + j % 2
 * (n even).  Then forward, backward, Adam.  params, m, v: device
 * [num_objects][15681], updated in place.  grad_samples: device [num_objects][n][4] gradient
 * records, read when hp->grad_lambda > 0 (else may be NULL).  loss: device
 * [n_steps][num_objects] (each step's minibatch loss) or NULL. */
tg_status tg_nsdf_train(tg_nsdf* h, float* params, float* m, float* v, const float* samples,
                        const float* grad_samples, int64_t n, int64_t step0, int32_t n_steps,
                        const tg_nsdf_train_params* hp, float* loss, void* hip_stream);

/* Network evaluation at normalised points grouped by object: object o owns points
 * [offsets[o], offsets[o+1]) of xhat (device [n][3]).  offsets: device [num_objects+1],
 * non-decreasing from 0; max_count: host, at least the largest offsets[o+1] - offsets[o]
 * (it sizes the launch; points beyond it are not evaluated).  out: device [n] (the network
 * output, phi / e); grad: device [n][3] (d out / d x_hat) or NULL.  params: device
 * [num_objects][15681]; the call packs them into the handle's BF16 image first. */
tg_status tg_nsdf_query(tg_nsdf* h, const float* params, const int64_t* offsets, int64_t max_count,
                        const float* xhat, float* out, float* grad, void* hip_stream);

/* tg_nsdf_query that also records, per point, the BF16 values the network rounded on its way:
 * trace: device [n][5][64] uint16 (BF16 bit patterns), row 0 the 48 encoding features in the
 * encoding's order (entries 48..63 unused), rows 1..4 the pre-activations of hidden layers 1..4
 * (the layer sums, bias included, rounded to BF16 before SiLU) in unit order.  Outputs and kernels
 * are those of tg_nsdf_query, bit for bit.  For the diagnosis of BF16 rounding ties: where two
 * evaluations of the network differ, the first of these values that differs tells where. */
tg_status tg_nsdf_query_trace(tg_nsdf* h, const float* params, const int64_t* offsets, int64_t max_count,
                              const float* xhat, float* out, float* grad, uint16_t* trace, void* hip_stream);

/* Allocation-free evaluation, for callers that cannot allocate device memory while they run:
 * code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments, results and kernels as tg_nsdf_query, bit for bit; the difference is where the
 * packed BF16 images live.  tg_nsdf_query packs them into the handle's own buffer; this call
 * packs them into one static device array per GPU (TG_NSDF_QUERY_NOALLOC_SCRATCH_BYTES, about
 * 4 MB, reserved on each GPU that runs it until the process ends) and calls no hipMalloc,
 * hipFree or other allocating routine.  Its device address is looked up once per device, at
 * the first call on that device.
 *   - The handle's num_objects must be <= TG_NSDF_QUERY_NOALLOC_MAX_OBJECTS, else
 *     TG_ERR_INVALID_ARGUMENT (nothing launched; use tg_nsdf_query).
 *   - The current device must be the one the handle was created on, else
 *     TG_ERR_INVALID_ARGUMENT.
 *   - Every call on a GPU shares that GPU's array, which keeps the last call's images.  Each
 *     call rewrites the images of all its objects before reading them, so nothing needs
 *     clearing, but calls that overlap in time on one GPU (two streams, two threads) race on
 *     the array: order them, for instance on one stream. */
#define TG_NSDF_QUERY_NOALLOC_MAX_OBJECTS 64
#define TG_NSDF_QUERY_NOALLOC_SCRATCH_BYTES (64 * 65024) /* max objects x bytes per image */
tg_status tg_nsdf_query_noalloc(tg_nsdf* h, const float* params, const int64_t* offsets, int64_t max_count,
                                const float* xhat, float* out, float* grad, void* hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* TG_NSDF_H */
