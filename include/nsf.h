/*
 * nsf.h - C ABI of the MI355X (gfx950) latent-space time step for reduced-order MPM with
 * neural deformation, stress and affine fields (Zong et al., "Neural Stress Fields for
 * Reduced-order Elastoplasticity and Fracture", SIGGRAPH Asia 2023).
 *
 * The problem, as the paper states it: given trained fields g (deformation, Sec. 4.2),
 * h (Kirchhoff stress, Sec. 4.3) and l (affine momentum, Sec. 4.4), reference positions
 * X_p (Sec. 3.2), a latent z_0, MPM constants (dt, dx, gravity, boundaries; Sec. 3.3) and
 * sample / integration particle sets (Sec. 5.4):
 *   - advance the latent z_n -> z_{n+1} by inference, one MPM step on the integration
 *     particles, and Gauss-Newton network inversion (Sec. 5.1-5.3);
 *   - decode positions x = X + u(X, z_n) at any reference point (Sec. 5.1; Sec. 6
 *     resolution boost).
 *
 * Conventions
 *   - Every call returns nsf_status (0 = NSF_OK). No exception crosses the ABI; the
 *     message of the last failure on the calling thread is nsf_last_error().
 *   - "host" pointers are read during the call only and may be freed afterwards.
 *     "device" pointers are HIP device addresses on the current device.
 *   - Stream arguments are hipStream_t passed as void* (NULL = the legacy default
 *     stream). Calls marked async only enqueue work on that stream.
 *   - Points are structure-of-arrays float32: X[3][n] means X[c * n + p].
 *   - A sim is not thread-safe. Distinct sims may be stepped on distinct streams.
 */
#ifndef NSF_H
#define NSF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  NSF_OK = 0,
  NSF_EINVAL = -1,       /* invalid argument or descriptor                                */
  NSF_ENOMEM = -2,       /* arena too small / workspace too small                         */
  NSF_EHIP = -3,         /* a HIP runtime call failed                                     */
  NSF_ENODEV = -4,       /* no gfx950 device is visible                                   */
  NSF_EDOMAIN = -5,      /* sticky: a particle stencil left the grid                      */
  NSF_ESINGULAR = -6,    /* sticky: Gauss-Newton normal matrix had a pivot <= 0           */
  NSF_ENONFINITE = -7,   /* sticky: the latent or the residual became non-finite          */
  NSF_ECAPACITY = -8     /* sticky: a closure integration set outgrew n_integration       */
} nsf_status;

/* NSF_FP32: every field layer on FP32 MFMA. NSF_BF16: hidden layers of every field on BF16
 * MFMA with FP32 accumulation (layer 1 and the output layer FP32). NSF_BF16_MIXED: BF16
 * hidden layers for the stress and affine fields (h, l) and the decode of all particles;
 * the deformation field where the inversion reads it (inference at the integration
 * particles, its latent Jacobian at the samples, the Gauss-Newton iterate) in FP32, with
 * the step's exact differences (sim steps only; the MLP calls take FP32 or BF16). */
typedef enum { NSF_FP32 = 0, NSF_BF16 = 1, NSF_BF16_MIXED = 2 } nsf_precision;

/* sticky device status bits, see nsf_status_flags */
enum { NSF_FLAG_DOMAIN = 1u, NSF_FLAG_NONFINITE = 2u, NSF_FLAG_SINGULAR = 4u,
       NSF_FLAG_CAPACITY = 8u };

/* How the integration particles N of each step are chosen (Sec. 5.4).
 * NSF_INTEGRATION_PLAN: step n integrates row (n mod plan_steps) of sample_plan, whose first
 *   n_sample entries are S. Particle volumes are body_volume / n_integration.
 * NSF_INTEGRATION_CLOSURE: S is fixed (sample_plan holds one row of n_sample distinct
 *   indices), and each step N is the closure of S's stencils: I = the grid nodes in the
 *   3 x 3 x 3 B-spline stencil of some p in S, N = S followed by every other particle whose
 *   in-grid stencil meets I, by ascending index, both at the decoded positions
 *   x = X + u(X, z_n). Then the MPM step on N gives S the result of a full-order step on
 *   all particles (Sec. 5.2). n_integration is the capacity of N: a closure that
 *   outgrows it is truncated and raises NSF_FLAG_CAPACITY. Particle volumes are
 *   body_volume / n_particles. Requires decode_every_step = 1 (the closure reads the
 *   decoded positions) and steps alone (not in nsf_step_batch). */
typedef enum { NSF_INTEGRATION_PLAN = 0, NSF_INTEGRATION_CLOSURE = 1 } nsf_integration;

/* Fields and their output widths (supplementary "Network architecture"): g -> 3
 * (displacement u, x = X + u), h -> 6 (Kirchhoff stress, Voigt xx yy zz yz xz xy),
 * l -> 9 (affine matrix C, row-major). */
enum { NSF_FIELD_G = 0, NSF_FIELD_H = 1, NSF_FIELD_L = 2 };

/* A moving blade imposed as a grid velocity boundary condition: after gravity and the
 * sticky walls, every node i with |normal . x_i - offset| <= half_thickness and
 * x_i.z >= edge_z0 - edge_speed * t_{n+1} takes `velocity`. */
typedef struct {
  int32_t enabled;
  double normal[3];
  double offset;
  double half_thickness;
  double edge_z0;
  double edge_speed;
  double velocity[3];
} nsf_knife;

/* Everything a reduced simulation needs. Read once by nsf_create_sim.
 *
 * weights[f] (host, float32) holds field f's six affine layers back to back, each as
 * W (row-major, out x in) followed by b (out):
 *   W1 [width x (3 + r)], b1 [width], W2..W5 [width x width] + b, W6 [d x width], b6 [d]
 * with d = 3, 6, 9 for g, h, l. The network input is [X; z] and ELU (alpha = 1) follows
 * layers 1-5. The physical value is out_scale[f][c] * y_c + out_shift[f][c]
 * (de-normalisation of data normalised to mean 0, variance 1; supplementary
 * "Training Details"). */
typedef struct {
  int32_t r;                   /* latent dimension, 1 <= r <= 32                          */
  int32_t width;               /* hidden width: 64 or 128                                 */
  int32_t n_hidden;            /* must be 5                                               */
  nsf_precision precision;     /* FP32, BF16 or BF16_MIXED (see nsf_precision)            */
  const float *weights[3];     /* host, see above                                         */
  double out_scale[3][9];
  double out_shift[3][9];
  int64_t n_particles;         /* |P|                                                     */
  const float *X;              /* host, [3][n_particles] reference positions              */
  double rho;                  /* density; m_p = rho V_p                                  */
  double body_volume;          /* V_p = body_volume / n_integration                       */
  int32_t grid_n;              /* nodes per axis, x_i = i dx, 8 <= grid_n <= 256          */
  double dx, dt;
  double gravity[3];
  int32_t wall_nodes;          /* sticky band: nodes with any index < b or >= n - b       */
  nsf_knife knife;
  int32_t n_integration;       /* |N| per step (closure integration: the capacity of N)   */
  int32_t n_sample;            /* |S| <= |N|; S = first n_sample entries of the step list */
  int32_t plan_steps;          /* rows in sample_plan; step n uses row n mod plan_steps   */
  const int32_t *sample_plan;  /* host, [plan_steps][n_integration] indices into P
                                  (closure integration: plan_steps = 1, [n_sample] = S)  */
  int32_t gn_iters;            /* Gauss-Newton iterations per step, 1..4 (paper: 2-3)     */
  int32_t decode_every_step;   /* 0: no decode in the step. 1: each step ends by decoding
                                  all P into the decoded-position buffer (nsf_sim_buffer
                                  NSF_BUF_XDEC) at the new latent. 2 (pipelined): each step
                                  decodes the latent it starts from, on a side stream,
                                  concurrently with its MPM step and inversion, so after a
                                  step the buffer holds the positions one step behind the
                                  latent; nsf_refresh decodes the current latent       */
  const double *z0;            /* host [r]                                                */
  const double *z_prev;        /* host [r] or NULL (then z_{-1} = z_0, zero velocity)     */
  double gn_damping;           /* lambda >= 0 (at most 1e6): every Gauss-Newton iteration
                                  solves (J^T J + lambda diag(J^T J)) delta = -J^T r, the
                                  Levenberg-Marquardt step with Marquardt's scaling, for
                                  ill-conditioned Jacobians. 0: the plain Gauss-Newton
                                  step of Sec. 5.3; with gn_iters = 1 that is the
                                  first-order (linearised) projection Sec. 5.3 offers as a
                                  speed-up: one solve with the Jacobian at z_n          */
  int32_t integration;         /* nsf_integration (0: plan rows, 1: closure of S)         */
  int32_t n_mu;                /* problem parameters mu (Sec. 4.3: a stress field may
                                  depend on a parameter of the return mapping), 0..4:
                                  h takes [X; z; mu] and its W1 is
                                  [width x (3 + r + n_mu)]; r + n_mu <= 32              */
  double mu[4];                /* their values (finite)                                   */
} nsf_sim_desc;

typedef struct nsf_sim nsf_sim;  /* opaque, owned by the library */

/* Bytes of device memory nsf_create_sim needs for this descriptor (0 if invalid). This
 * is the unit of HBM-budget admission. */
size_t nsf_sim_bytes(const nsf_sim_desc *d);

/* Validate d, carve `arena` (device, >= nsf_sim_bytes(d) bytes, 256-byte aligned, owned
 * by the caller and kept alive until nsf_destroy_sim), copy every input into it and
 * pack the weights for the MFMA kernels. Work is enqueued on `stream`; the call returns
 * after that work completes. Validation: r in 1..32, width in {64, 128}, n_hidden == 5,
 * n_sample >= ceil(r / 3) (well-posedness of the inversion, Sec. 5.4),
 * 1 <= n_sample <= n_integration <= n_particles, plan indices in range.
 * NSF_ENODEV without a gfx950 device. */
nsf_status nsf_create_sim(const nsf_sim_desc *d, void *arena, size_t arena_bytes,
                          void *stream, nsf_sim **out);

/* Advance n_steps latent steps (Sec. 5.1-5.3), async. The first call on a stream captures
 * one step into a HIP graph; later calls replay it. No device-to-host transfer occurs. */
nsf_status nsf_step(nsf_sim *s, int32_t n_steps, void *stream);

/* Advance several sims together, async: each kernel of the step runs once over the
 * union of the sims' work (fields of every sim in one launch, P2G of every sim in one
 * launch, ...). Sims keep private grids and latents, and every reduction in the step has
 * a fixed order (P2G gathers per node in a sorted particle order, the Gauss-Newton sums
 * reduce in a fixed tree), so each sim's result is bit for bit the one it gets stepped
 * alone. All sims must share width and precision. The launch shape is planned for this
 * set of sims on first use; when the set changes, the work tables are rewritten and the
 * captured graph is replayed unchanged (it is re-captured only when the tables outgrow
 * their capacity). At most 1024 sims per call (NSF_EINVAL beyond). */
nsf_status nsf_step_batch(nsf_sim *const *sims, int32_t n, int32_t n_steps, void *stream);

/* The MPM stage of the current step alone (Sec. 5.2, with the algorithm of Sec. 3.3),
 * async: P2G of the integration particles with APIC and the stress impulse, the grid
 * update (gravity, walls, knife) and G2P of the new velocity at the samples, from the
 * field inference the step starts from (run first if the sims do not hold it yet, as
 * after create or nsf_set_latent). It writes NSF_BUF_GRID and NSF_BUF_VNEW and the first
 * Gauss-Newton partial sums, exactly as the step's own MPM kernels do; it advances
 * neither the latent nor the step counter, so repeated calls recompute the same values
 * (the way to time the transfers alone). sims: host array of n distinct sims; n > 1
 * runs one launch per kernel over the union of their work under the same rules as
 * nsf_step_batch. */
nsf_status nsf_mpm_stage(nsf_sim *const *sims, int32_t n, void *stream);

/* Evaluate the fields at the current latent in one launch, async: decode all particles
 * into the decoded-position buffer (when decode_every_step is 1 or 2) and the field inference the
 * next step starts from (Sec. 5.1). nsf_step ends every step with this launch; call it
 * directly to refresh the decoded positions after nsf_set_latent, or to time it. */
nsf_status nsf_refresh(nsf_sim *s, void *stream);

/* Decode x = X + u(X, z_n) (Sec. 5.1), async. X: device [3][n] or NULL for the sim's own
 * reference positions (then n must equal n_particles). x_out: device [3][n]. */
nsf_status nsf_decode(nsf_sim *s, const float *X, int64_t n, float *x_out, void *stream);

/* Copy the latent state to host (synchronises the stream). z, z_prev: host [r] or NULL;
 * step: host or NULL. This is the whole dynamic state (checkpoint). */
nsf_status nsf_get_latent(nsf_sim *s, double *z, double *z_prev, int64_t *step, void *stream);

/* Restore a latent state (host arrays, z_prev NULL -> z), async. Clears sticky flags. */
nsf_status nsf_set_latent(nsf_sim *s, const double *z, const double *z_prev, int64_t step,
                          void *stream);

/* Closure integration (Sec. 5.4; the paper's cake halves its sample set half-way): keep
 * only the first n_sample entries of the sample list from the next step on, async.
 * 1 <= n_sample <= the n_sample given at creation, 3 n_sample >= r. The next nsf_step
 * first recomputes the integration set and the field inference for the smaller S at the
 * current latent. NSF_EINVAL for a plan sim. */
nsf_status nsf_set_sample_count(nsf_sim *s, int32_t n_sample, void *stream);

/* Problem parameters of the stress field h(X, z, mu) (Sec. 4.3), host [n_mu], async: the
 * next nsf_step first re-evaluates the field inference with the new values. NSF_EINVAL
 * if n_mu differs from the descriptor's or a value is not finite. */
nsf_status nsf_set_parameters(nsf_sim *s, const double *mu, int32_t n_mu, void *stream);

/* Read the sticky device flags (synchronises). Returns NSF_OK with *flags = 0, or, with
 * *flags set, the status of the first set condition in the order NONFINITE, SINGULAR,
 * DOMAIN, CAPACITY (a non-finite latent also throws particles off the grid). */
nsf_status nsf_status_flags(nsf_sim *s, uint32_t *flags, void *stream);

/* Inspect a per-step device buffer of the sim (read-only views for tests and callers
 * that consume the step's intermediates). *ptr receives the device address and *count
 * the number of elements (float unless noted).
 *   NSF_BUF_U       u(X_N, z_n)          [3][n_integration]
 *   NSF_BUF_UPREV   u(X_N, z_{n-1})      [3][n_integration]; with BF16 precision the
 *                   velocity itself, J((z_n + z_{n-1})/2) (z_n - z_{n-1}) / dt
 *   NSF_BUF_TAU     h(X_N, z_n)          [6][n_integration]
 *   NSF_BUF_C       l(X_N, z_n)          [9][n_integration]
 *   NSF_BUF_JAC     du/dz at z_n on S    [3 r][n_sample], row c*r + j = du_c/dz_j
 *   NSF_BUF_VNEW    G2P velocity on S    [3][n_sample]
 *   NSF_BUF_XDEC    decoded positions    [3][n_particles]
 *   NSF_BUF_GRID    grid after the grid update, float4 (v_x, v_y, v_z, m) per node,
 *                   node (i, j, k) at (i grid_n + j) grid_n + k; valid on the node blocks
 *                   the step's particles reach (others hold older values)
 *   NSF_BUF_Z       double [3][r]: z_{n-1}, z_n, last Gauss-Newton iterate
 *   NSF_BUF_NLIST   int32 integration lists: [plan_steps][n_integration] (plan), or the
 *                   current list [n_integration] (closure; entries past its live length
 *                   are stale)
 *   NSF_BUF_NLIVE   int32 [1]: live length of the closure list (closure only)
 * Buffers hold the values of the last completed step; with closure integration the
 * per-particle buffers (U, UPREV, TAU, C) follow the current list. */
enum { NSF_BUF_U = 0, NSF_BUF_UPREV, NSF_BUF_TAU, NSF_BUF_C, NSF_BUF_JAC, NSF_BUF_VNEW,
       NSF_BUF_XDEC, NSF_BUF_GRID, NSF_BUF_Z, NSF_BUF_NLIST, NSF_BUF_NLIVE };
nsf_status nsf_sim_buffer(nsf_sim *s, int32_t which, void **ptr, int64_t *count);

/* Release host-side state and any captured graphs. The arena stays the caller's. */
nsf_status nsf_destroy_sim(nsf_sim *s);

/* Message of the last failed call on this thread ("" if none). */
const char *nsf_last_error(void);

/* Number of visible gfx950 devices (0 without a GPU). Does not create a context on
 * machines without HIP devices. */
int32_t nsf_device_count(void);

/* ---- Field fitting (differentiation form) ------------------------------------------
 * One MLP as above (in = 3 + r, width, out = d, 6 layers), weights in the same layout
 * as nsf_sim_desc.weights but on the device. Per-point latents: the input of point p is
 * [X_p ; z_rows[p]] with z_rows device float32 [n][r] row-major. Training data for the
 * fields is fitted by minimising squared error (Sec. 4.5).
 *
 * nsf_mlp_forward: out device [d][n] (SoA); saved device float32 of nsf_mlp_saved_floats
 *   (width, n) elements, receiving the five hidden pre-activations for the backward in
 *   the kernels' internal format (scaled by log2 e; NULL = inference only). With NSF_BF16
 *   they are stored rounded to BF16 and fill the first half of the buffer.
 * nsf_mlp_backward: given dout [d][n] = dLoss/dout, accumulate (+=) dW (device, same
 *   layout and size as the weights), write dz device [n][r] = dLoss/dz_rows and dX device
 *   [3][n] = dLoss/dX (SoA like X), each NULL to skip. Requires `saved` from the forward
 *   of the same weights and inputs.
 * Precision: NSF_FP32 (also used by the finite-difference check) or NSF_BF16 (hidden
 * layers on BF16 MFMA with FP32 accumulation, forward and backward; the backward's deltas
 * and the saved pre-activations are BF16, dz and dX are formed in FP32). */
typedef struct {
  int32_t r, width, d;
  nsf_precision precision;
  const float *weights;        /* device, layout as nsf_sim_desc.weights                  */
} nsf_mlp;

size_t nsf_mlp_param_count(int32_t r, int32_t width, int32_t d);
size_t nsf_mlp_saved_floats(int32_t width, int64_t n);
size_t nsf_mlp_workspace_bytes(const nsf_mlp *m, int64_t n);
nsf_status nsf_mlp_forward(const nsf_mlp *m, const float *X, const float *z_rows, int64_t n,
                           float *out, float *saved, void *workspace, size_t workspace_bytes,
                           void *stream);
nsf_status nsf_mlp_backward(const nsf_mlp *m, const float *X, const float *z_rows, int64_t n,
                            const float *saved, const float *dout, float *dW, float *dz,
                            float *dX, void *workspace, size_t workspace_bytes, void *stream);

/* One Adam step (Sec. 4.5 trains the fields with Adam) over n FP32 parameters on the
 * device: m and v are the first and second moment buffers (device, n each, zero before
 * the first step), step counts from 1. With g = grad, in PyTorch's order of operations:
 * m = beta1 m + (1 - beta1) g; v = beta2 v + (1 - beta2) g^2;
 * w -= (lr / (1 - beta1^step)) m / (sqrt(v) / sqrt(1 - beta2^step) + eps).
 * NSF_EINVAL for NULL buffers, n < 1, step < 1 or betas outside [0, 1), eps <= 0. */
nsf_status nsf_adam_step(float *w, const float *grad, float *m, float *v, int64_t n, double lr,
                         double beta1, double beta2, double eps, int64_t step, void *stream);

/* The latent rows of a minibatch whose (particle, snapshot) pairs are grouped by snapshot
 * (the per-snapshot latents of Sec. 4.5): segment s covers rows [offsets[s], offsets[s+1])
 * of a row-major [n][width] FP32 device array, offsets device int64 [segments + 1],
 * non-decreasing from 0. nsf_rows_expand writes out[i][:] = table[s][:] for every row i
 * of segment s (table [segments][width]); nsf_rows_segment_sum, its adjoint, writes
 * out[s][:] = the sum of rows[i][:] over segment s, added in a fixed order. width 1..256;
 * NSF_EINVAL for NULL buffers or widths out of range. */
nsf_status nsf_rows_expand(const float *table, const int64_t *offsets, int32_t segments, int32_t width,
                           float *out, void *stream);
nsf_status nsf_rows_segment_sum(const float *rows, const int64_t *offsets, int32_t segments,
                                int32_t width, float *out, void *stream);

/* The fitting objective of one minibatch (Sec. 4.5 fits each field by least squares to the
 * snapshots' values) and its gradient, in one pass. With e = out[c n + i] - Y[c ldy + q_i]
 * and q_i = rows[i] P + cols[i] (pair i's snapshot and particle):
 *   loss[0] = (sum over c < d, i < n of e^2) / (d n),   grad[c n + i] = e * (2 / (d n)),
 * the factor 2 / (d n) rounded to FP32 once. out: device, d x n floats (output-major, as
 * nsf_mlp_forward writes them); Y: device, d rows of ldy floats, every q_i < ldy; rows,
 * cols: device, n int64 each; loss: device, 1 float; grad: device, d x n floats (may be
 * out itself); workspace: device, NSF_SQERR_WORKSPACE_BYTES bytes, owned by the caller.
 * The squares are summed in FP64 in a fixed order, so the loss is the same bits on every
 * run. NSF_EINVAL for NULL pointers, d < 1, n < 1, P < 1 or ldy < 1; NSF_EHIP for a
 * failed launch. */
#define NSF_SQERR_WORKSPACE_BYTES 4096
nsf_status nsf_squared_error(const float *out, int32_t d, int64_t n, const float *Y, int64_t ldy,
                             const int64_t *rows, const int64_t *cols, int64_t P, float *loss,
                             float *grad, void *workspace, void *stream);

/* nsf_mlp_forward without a workspace argument, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc). It allocates nothing: the packed weights go to a library-owned device array
 * of 1 MiB per GPU (enough for any nsf_mlp this header accepts: width 128, r = 32, d = 9
 * packs to ~0.7 MB), resolved once per device on that device's first call. Arguments,
 * layouts and results are those of nsf_mlp_forward. Returns NSF_EINVAL for an invalid m
 * or NULL X / z_rows / out, NSF_ENOMEM if the packed weights would exceed the array,
 * NSF_EHIP if the array's address cannot be resolved. Every call on one GPU shares its
 * array and the array keeps the last call's packed weights: calls that overlap on one GPU
 * (different streams, or threads) race and must be serialised by the caller. */
nsf_status nsf_mlp_forward_noalloc(const nsf_mlp *m, const float *X, const float *z_rows,
                                   int64_t n, float *out, float *saved, void *stream);

/* ---- Full-order MLS-MPM (the model the reduced step is measured against) -------------
 * Every particle is integrated (Sec. 3.3): P2G with APIC and the MLS stress impulse, grid
 * update with gravity, sticky walls and a separating ground (the bottom wall_nodes layers
 * keep v_z >= 0), G2P of v and C, F_trial = (I + dt C) F^E, then one of three return maps
 * and its elasticity (supplementary "Elasticity and plasticity details"). With
 * F_trial = U S V^T, eps = log S, eps_hat = eps - mean(eps):
 *   NSF_FO_VON_MISES: dgamma = |eps_hat| - tau_y / (2 mu); if dgamma > 0,
 *     eps -= dgamma eps_hat / |eps_hat|; F^E = U exp(eps) V^T; fixed corotated stress
 *     tau = 2 mu (F^E - R) F^E^T + lambda (J - 1) J I, R = U V^T.
 *   NSF_FO_DRUCKER_PRAGER: dgamma = |eps_hat| + alpha (3 lambda + 2 mu) sum(eps) / (2 mu),
 *     alpha = sqrt(2/3) 2 sin(phi_f) / (3 - sin(phi_f)); sum(eps) > 0 gives F^E = U V^T,
 *     dgamma <= 0 leaves F_trial, otherwise eps -= dgamma eps_hat / |eps_hat|; StVK stress
 *     in log strain tau = U diag(2 mu eps + lambda sum(eps)) U^T.
 *   NSF_FO_HERSCHEL_BULKLEY (h = 1): with bbar = J^(-2/3) S^2 and s_t = mu |dev(bbar)|, if
 *     s_t > sqrt(2/3) tau_y the deviator is scaled to
 *     s = s_t - (s_t - sqrt(2/3) tau_y) / (1 + viscosity / (2 mu dt)) and bbar becomes
 *     (s / s_t) dev(bbar) + c I with det(bbar) = 1 (volume and rotations kept), so
 *     F^E = U J^(1/3) sqrt(bbar) V^T; stress tau = kappa/2 (J^2 - 1) I + mu dev(bbar)
 *     (kappa = E / (3 (1 - 2 nu))).
 * Positions, velocities and C are FP32 and F^E FP64; each particle's SVD comes from a
 * Jacobi eigen-decomposition of F^T F in FP64. Particle volume body_volume / n_particles.
 * All particles start with velocity v0, C = 0 and F^E = I. */
enum { NSF_FO_VON_MISES = 0, NSF_FO_DRUCKER_PRAGER = 1, NSF_FO_HERSCHEL_BULKLEY = 2 };
typedef struct {
  int64_t n_particles;
  const float *X;              /* host [3][n_particles] initial positions                 */
  double v0[3];                /* initial velocity                                        */
  double rho, body_volume;
  double youngs, poisson;      /* E, nu: mu = E / (2 (1 + nu)), lambda = E nu / ((1 + nu)(1 - 2 nu)) */
  double yield_stress;         /* tau_y of von Mises and Herschel-Bulkley (> 0; unused by
                                  Drucker-Prager)                                       */
  int32_t grid_n;              /* nodes per axis, 8..256, dx = 1 / grid_n                 */
  double dt;
  double gravity[3];
  int32_t wall_nodes;          /* wall band; its bottom layers are the separating ground  */
  int32_t plasticity;          /* NSF_FO_VON_MISES, NSF_FO_DRUCKER_PRAGER or
                                  NSF_FO_HERSCHEL_BULKLEY                              */
  double friction_angle;       /* Drucker-Prager phi_f in degrees, 0 <= phi_f < 90        */
  double viscosity;            /* Herschel-Bulkley eta >= 0                               */
} nsf_fo_desc;

typedef struct nsf_fo nsf_fo;

/* Device bytes of the full-order sim's arena (0 if d is invalid). */
size_t nsf_fo_bytes(const nsf_fo_desc *d);
/* Create in a caller-owned arena (device, 256-byte aligned, >= nsf_fo_bytes); the call
 * returns after the set-up work on `stream` completes. */
nsf_status nsf_fo_create(const nsf_fo_desc *d, void *arena, size_t arena_bytes, void *stream,
                         nsf_fo **out);
/* Advance n_steps full-order steps, async (a captured graph after the first call). */
nsf_status nsf_fo_step(nsf_fo *f, int32_t n_steps, void *stream);
/* Device views: NSF_FO_U displacement x - X [3][P], NSF_FO_V velocity [3][P], NSF_FO_C
 * affine C [9][P] (row-major), NSF_FO_TAU Kirchhoff stress, Voigt [6][P] (all float),
 * NSF_FO_F elastic F^E, double [9][P]. */
enum { NSF_FO_U = 0, NSF_FO_V, NSF_FO_C, NSF_FO_TAU, NSF_FO_F };
nsf_status nsf_fo_buffer(nsf_fo *f, int32_t which, void **ptr, int64_t *count);
/* Sticky flags as nsf_status_flags (DOMAIN if a particle leaves the grid). */
nsf_status nsf_fo_flags(nsf_fo *f, uint32_t *flags, void *stream);
nsf_status nsf_fo_destroy(nsf_fo *f);

#ifdef __cplusplus
}
#endif
#endif /* NSF_H */
