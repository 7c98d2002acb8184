/*
 * smppi.h -- C ABI of the MI355X (gfx950) Shield-MPPI sampled-rollout library.
 *
 * Paper: Yin, Dawson, Fan, Tsiotras, "Shield Model Predictive Path Integral: A
 * Computationally Efficient Robust MPC Method Using Control Barrier Functions"
 * (arXiv 2302.11719).  Notation: K samples per problem, T horizon steps, B
 * independent problems (the paper writes M for samples and K for the horizon).
 *
 * Conventions for every call
 *  - Pointers marked "device" are caller-owned device memory on the ctx's device
 *    (for instance torch tensors' data pointers), contiguous, of the element type
 *    named; "dtype" means float for SMPPI_F32 and double for SMPPI_F64.  The
 *    library never frees or retains caller memory beyond the call (plans keep the
 *    pointers they were created with, see smppi_plan_create).
 *  - Struct arguments are host memory, read during the call only.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).  Work is
 *    enqueued on it and the call returns without synchronising.  Validation
 *    errors are detected before anything is enqueued.  Faults inside kernels
 *    surface at the caller's next synchronisation.
 *  - Scratch memory is owned by the ctx and sized by smppi_reserve_batch (or
 *    by a plan at creation).  No call that enqueues work allocates device
 *    memory: a call whose batch needs more scratch than the ctx holds returns
 *    SMPPI_ERR_SHAPE before enqueueing anything.  A ctx is not thread-safe, and
 *    calls made on one ctx must be ordered on one stream: they share the ctx's
 *    scratch.
 *  - The library never aborts and never prints; smppi_last_error() describes the
 *    last non-OK status of a ctx.
 *
 * Layouts (per problem b, with K_b = k_off[b+1]-k_off[b], T_b = t_off[b+1]-t_off[b]):
 *  - state x: 6 values (p_x, p_y, psi, v_x, v_y, omega); x0 is [B][6].
 *  - control sequence V: 2*T_b values at offset 2*t_off[b], steer row first:
 *    V[2*t_off[b] + d*T_b + t], d = 0 steer, d = 1 throttle.
 *  - per-sample arrays (S, w, grad_S) are indexed by k_off[b] + m.
 */
#ifndef SMPPI_H
#define SMPPI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SMPPI_ABI_VERSION 7

typedef enum {
  SMPPI_OK = 0,
  SMPPI_ERR_INVALID_ARGUMENT = 1, /* null pointer, bad parameter value */
  SMPPI_ERR_SHAPE = 2,            /* sizes inconsistent or beyond a supported bound */
  SMPPI_ERR_DTYPE = 3,            /* dtype not supported by this call */
  SMPPI_ERR_NO_DEVICE = 4,        /* no HIP device (or not the one asked for) */
  SMPPI_ERR_HIP = 5,              /* a HIP runtime call failed; see smppi_last_error */
  SMPPI_ERR_UNSUPPORTED = 6,      /* valid request this build does not implement */
  SMPPI_ERR_NONFINITE = 7         /* reserved: non-finite input detected on the host */
} smppi_status;

typedef enum { SMPPI_F32 = 0, SMPPI_F64 = 1 } smppi_dtype;

typedef struct smppi_ctx_s* smppi_ctx;
typedef struct smppi_plan_s* smppi_plan;

/* Dynamics x_{k+1} = f(x_k, u_k) of eq. (1), realised as a six-state dynamic
 * single-track vehicle with linear tyres integrated by classic RK4 over dt with
 * the control held:
 *   dp_x = v_x cos(psi) - v_y sin(psi),   dp_y = v_x sin(psi) + v_y cos(psi),
 *   dpsi = omega,
 *   dv_x = a_max tau - c_v v_x - F_f sin(delta)/m + v_y omega,
 *   dv_y = (F_f cos(delta) + F_r)/m - v_x omega,
 *   domega = (l_f F_f cos(delta) - l_r F_r)/I_z,
 *   F_f = C_f (delta - (v_y + l_f omega)/v~),  F_r = -C_r (v_y - l_r omega)/v~,
 *   v~ = max(v_x, v_min).
 * Sampled controls are clipped to [u_lo, u_hi] (steer, throttle). */
typedef struct {
  double m, lf, lr, Iz, Cf, Cr, a_max, c_v, v_min, dt;
  double u_lo[2], u_hi[2];
} smppi_model;

/* Trajectory cost (Algorithm 2; eqs. (8), (12), (17)-(20), (23)-(25)):
 *   S~ = sum_{k<T} [ q(x_k) + lambda_u sum_d v_{k,d} u_{k,d} / sigma_d^2 ]
 *        + phi_w q(x_T) + sum_{k=0}^{T} C_cbf(z_k),
 *   q(x) = q_v (v_x - v_g)^2 + q_ey e_y^2 + C_obs [x outside the safe region],
 *   C_cbf(z_k) = C_cbf sum_j max(alpha h_j(x_{k-1}) - h_j(x_k), 0), x_{-1} = x_0,
 *   alpha = 1 - gamma (gamma is the class-kappa slope of eq. (15)).
 * Barriers: h_0 = w^2 - e_y^2 (eq. (23)); per obstacle h_i = |p - c_i|^2 - r_eff_i^2.
 * "Outside" = h_0 < 0 or inside any obstacle's physical radius.
 * sigma also scales the sampled noise: eps = sigma (.) z, z ~ N(0, I). */
typedef struct {
  double v_g, q_v, q_ey, C_obs, phi_w;
  double lambda_u;
  double sigma[2];
  double C_cbf, gamma;
} smppi_cost;

/* Noise: Philox4x32-10 (Salmon et al., SC'11) with key (seed, 0) and counter
 * (t>>1, m, pid_base + b, iter[b]); words (0,1) feed step 2j and (2,3) step 2j+1
 * through u = ((x>>8)+1) 2^-24 and Box-Muller (first normal steers).
 * nominal != 0 replaces every sample's noise by zero (nominal rollouts). */
typedef struct {
  uint32_t seed;
  int32_t nominal;
} smppi_noise;

/* A batch of B independent problems in CSR form. */
typedef struct {
  int32_t n_problems;   /* B >= 1 */
  int32_t k_max;        /* host: max K_b (launch sizing); every K_b <= k_max */
  int32_t t_max;        /* host: max T_b; every T_b <= t_max, 1 <= T_b */
  int32_t pid_base;     /* problem id of problem 0 in the noise counter */
  smppi_dtype dtype;
  const int64_t* k_off; /* device [B+1], k_off[0] = 0, non-decreasing */
  const int32_t* t_off; /* device [B+1], t_off[0] = 0, strictly increasing */
} smppi_batch;

/* Per-problem track: a circle (when the problem has no polyline vertices) or a
 * closed polyline; e_y^2 is the squared distance to the nearest segment, found
 * by a global search at x_0 and afterwards within +-window segments of the
 * previous step's segment (offsets visited 0, -1, +1, -2, ...; first strict
 * minimum wins). */
typedef struct {
  const int32_t* poly_off;  /* device [B+1] vertex offsets */
  const void* poly;         /* device [sum N][5] dtype: a_x, a_y, d_x, d_y, 1/|d|^2 */
  const void* circle;       /* device [B][3] dtype: c_x, c_y, R (used when N_b = 0) */
  const void* half_width;   /* device [B] dtype: w */
  const int32_t* obs_off;   /* device [B+1] obstacle offsets, or NULL for none */
  const void* obs;          /* device [sum O][4] dtype: c_x, c_y, r_eff^2, r^2 */
  int32_t window;           /* search half width, 1 <= window, 2*window+1 <= N_b */
  int32_t poly_max;         /* host: max N_b (<= 4096) */
  int32_t obs_max;          /* host: max O_b (<= 64) */
} smppi_track;

/* Per-problem curvature table of the curvilinear model (Sec. VI-A: the vehicle
 * state is expressed along the track as progress s, lateral error e_y and
 * heading error e_psi, so the track barrier h = w^2 - e_y^2 of eq. (23) needs no
 * projection).  kappa(s) is periodic: table entry j at s = j*ds, linear in
 * between; left turns positive. */
typedef struct {
  const int32_t* kappa_off; /* device [B+1] table offsets (N_b >= 2) */
  const void* kappa;        /* device [sum N][1] dtype */
  const void* ds;           /* device [B] dtype: grid spacing (> 0) */
  const void* half_width;   /* device [B] dtype: w */
  int32_t n_max;            /* host: max N_b (<= 8192) */
} smppi_curv_track;

/* Wheels of the eight-state curvilinear model (Sec. VI-A names the state
 * x = (v_x, v_y, r, omega_F, omega_R, e_psi, e_y, s): body velocities, yaw rate,
 * front and rear wheel speeds, heading error, lateral deviation, progress; the
 * paper prints no equations, so the library's reading is):
 *   F_yF = C_f (delta - (v_y + l_f r)/v~),  F_yR = C_r (l_r r - v_y)/v~,  v~ = max(v_x, v_min),
 *   F_xF = C_x (r_w omega_F - v_x cos(delta) - (v_y + l_f r) sin(delta))/v~,
 *   F_xR = C_x (r_w omega_R - v_x)/v~,
 *   v_x' = (F_xR + F_xF cos(delta) - F_yF sin(delta))/m - c_v v_x + v_y r,
 *   v_y' = (F_yR + F_xF sin(delta) + F_yF cos(delta))/m - v_x r,
 *   r'   = (l_f (F_xF sin(delta) + F_yF cos(delta)) - l_r F_yR)/I_z,
 *   omega_F' = -r_w F_xF / I_w,  omega_R' = (m a_max r_w T - r_w F_xR)/I_w,
 *   s' = (v_x cos(e_psi) - v_y sin(e_psi))/(1 - kappa(s) e_y),
 *   e_y' = v_x sin(e_psi) + v_y cos(e_psi),  e_psi' = r - kappa(s) s',
 * with the smppi_model constants; at the wheels' equilibrium speeds the body
 * equations are the six-state model's. */
typedef struct {
  double r_w;  /* wheel radius (m) */
  double I_w;  /* wheel inertia per axle (kg m^2) */
  double C_x;  /* longitudinal slip stiffness per axle (N) */
} smppi_wheels;

/* Differentiated objective of one trajectory (used by the adjoint and repair):
 *   L = w_S S~' + w_sq sum_{j,t<T} viol_{j,t}^2 + w_lin sum_{j, t<n_lin} viol_{j,t},
 *   viol_{j,t} = max(alpha h_j(x_t) - h_j(x_{t+1}), 0),
 * S~' = S~ without the (piecewise constant) collision indicator.  The shield of
 * Algorithm 1 / eq. (22) is w_S = w_sq = 0, w_lin = 1, n_lin = N+1. */
typedef struct {
  double w_S, w_sq, w_lin;
  int32_t n_lin;
} smppi_objective;

/* Safety shield on the objective evaluated on the nominal trajectory from x0.
 * method 0 (Algorithm 1): n_steps times V <- clip(V - step * dL/dV, u_lo, u_hi).
 * method 1 (the quasi-Newton optimiser the text of Sec. IV-B names): projected
 * limited-memory BFGS, V <- clip(V - H dL/dV), H from the two-loop recursion
 * over the last `memory` (1..16) pairs (s, y) of iterate and gradient
 * differences kept when s.y > 0.01 |s| |y|, H_0 = (s.y / y.y) I of the newest
 * pair, or step * I when none is kept.  Both stop early when the gradient is
 * zero. */
typedef struct {
  int32_t n_steps;
  double step;
  smppi_objective objective;
  int32_t method;
  int32_t memory;
} smppi_repair_opts;

/* ---- context ---------------------------------------------------------------- */

/* Create a ctx bound to HIP device `device`.  SMPPI_ERR_NO_DEVICE when no GPU. */
smppi_status smppi_create(int device, smppi_ctx* out);
void smppi_destroy(smppi_ctx ctx);
const char* smppi_last_error(smppi_ctx ctx);
const char* smppi_status_string(smppi_status s);
int smppi_abi_version(void);
/* Size the ctx's scratch for the plain calls on any batch within the host
 * bounds of `batch` (n_problems, k_max, t_max, dtype; its device arrays are not
 * read): the update's and the adjoint's per-workgroup partials
 * (dtype bytes x B x ceil(k_max / workgroup samples) x 2 x t_max), the padded
 * obstacle slots of FP32 rollouts (B x 64 x 16 bytes) and B ticket counters.
 * Allocates (and synchronises) only when the ctx holds less; the scratch never
 * shrinks.  Call it before smppi_rollout (FP32 with obstacles), smppi_update
 * and smppi_rollout_backward, outside timed or captured regions. */
smppi_status smppi_reserve_batch(smppi_ctx ctx, const smppi_batch* batch);
/* Synchronise the device, return (and clear) the OR of the input-bound errors
 * kernels detected on device data since the last call: 1 = some T_b outside
 * [1, t_max], 2 = some K_b outside [0, k_max], 4 = some polyline longer than
 * poly_max or shorter than 2*window+1, 8 = more than obs_max obstacles.
 * Problems with such data are skipped (their outputs are left unwritten).
 * 16 = a wave of the shield gave up waiting for another wave of its workgroup
 * (a bounded wait that correct inputs never exhaust; that problem's V_safe is
 * then invalid). */
smppi_status smppi_device_errors(smppi_ctx ctx, uint32_t* flags);

/* ---- the sampled-rollout step ---------------------------------------------- */

/* Sampling and cost of Algorithm 2's inner loop (eqs. (8), (12), (20)): for every
 * problem b and sample m < K_b, draw eps, clip u = v + eps, integrate f over T_b
 * steps from x0[b] and write S~ to S[k_off[b]+m] (dtype).
 * x0: device [B][6] dtype.  V: device control sequences (layout above).
 * iter: device [B] uint32 iteration counters (noise counter word 3).
 * eps_out: NULL, or device [sum K][t_max][2] dtype receiving the effective
 *   noise u - v of every step (debug/test; rows beyond T_b untouched).
 * FP32 with obstacles: a small kernel first copies every problem's obstacles
 * into padded slots in the ctx scratch (B * 64 * 16 bytes, see
 * smppi_reserve_batch), which the rollout kernel reads through the scalar
 * cache. */
smppi_status smppi_rollout(smppi_ctx ctx, const smppi_batch* batch, const smppi_model* model,
                           const smppi_cost* cost, const smppi_noise* noise, const smppi_track* track,
                           const void* x0, const void* V, const uint32_t* iter, void* S, void* eps_out,
                           void* stream);

/* The sampled rollout of smppi_rollout for the eight-state curvilinear model
 * (smppi_wheels): x0 device [B][8] dtype in the state order
 * (v_x, v_y, r, omega_F, omega_R, e_psi, e_y, s); S~ as in smppi_rollout with
 * q = q_v (v_x - v_g)^2 + q_ey e_y^2 + C_obs [|e_y| > w] and the DCBF penalty on
 * h = w^2 - e_y^2 (no obstacles).  V, iter, S, eps_out and the noise as in
 * smppi_rollout; smppi_weights and smppi_update apply unchanged. */
smppi_status smppi_rollout_curvilinear(smppi_ctx ctx, const smppi_batch* batch, const smppi_model* model,
                                       const smppi_wheels* wheels, const smppi_cost* cost, const smppi_noise* noise,
                                       const smppi_curv_track* track, const void* x0, const void* V,
                                       const uint32_t* iter, void* S, void* eps_out, void* stream);

/* Adjoint of smppi_rollout_curvilinear (as smppi_rollout_backward, with the
 * barrier read from e_y): grad_V = sum_m grad_S[m] dL_m/dV, states recomputed
 * from per-sample checkpoints.  Scratch as smppi_rollout_backward
 * (smppi_reserve_batch). */
smppi_status smppi_rollout_backward_curvilinear(smppi_ctx ctx, const smppi_batch* batch, const smppi_model* model,
                                                const smppi_wheels* wheels, const smppi_cost* cost,
                                                const smppi_noise* noise, const smppi_curv_track* track,
                                                const void* x0, const void* V, const uint32_t* iter,
                                                const void* grad_S, const smppi_objective* objective, void* grad_V,
                                                void* stream);

/* Safety shield (Algorithm 1, eq. (22)) on the curvilinear model: method 0 of
 * smppi_repair_opts only (SMPPI_ERR_UNSUPPORTED otherwise).  V_safe may equal
 * V_plus. */
smppi_status smppi_shield_repair_curvilinear(smppi_ctx ctx, const smppi_batch* batch, const smppi_model* model,
                                             const smppi_wheels* wheels, const smppi_cost* cost,
                                             const smppi_curv_track* track, const void* x0, const void* V_plus,
                                             const smppi_repair_opts* opts, void* V_safe, void* stream);

/* Execute and warm start on the curvilinear model (as smppi_execute): x [B][8]
 * <- RK4(x, clipped first control of V_exec) + (0, dist_vy, dist_r, 0, ...),
 * V <- V_plus shifted one step, iter += 1. */
smppi_status smppi_execute_curvilinear(smppi_ctx ctx, const smppi_batch* batch, const smppi_model* model,
                                       const smppi_wheels* wheels, const smppi_curv_track* track, const void* V_exec,
                                       const void* V_plus, const void* dist, int32_t n_dist, void* x, void* V,
                                       uint32_t* iter, void* stream);

/* Path-integral weights (eqs. (7), (9), (11)): w_m = exp(-(S_m - min S)/lambda)
 * / sum, per problem, with non-finite S_m given weight 0.
 * w: device [sum K] dtype.  stats: device [B][4] dtype = (min S, log sum_m
 * exp(-(S_m - min S)/lambda), effective sample size 1/sum w^2, number of
 * non-finite costs); when every cost is non-finite all weights are 0.
 * lambda > 0. */
smppi_status smppi_weights(smppi_ctx ctx, const smppi_batch* batch, const void* S, double lambda, void* w,
                           void* stats, void* stream);

/* Update law (eq. (10) with the per-trajectory weights of eq. (11)):
 * V+ = V + sum_m w_m (clip(V + eps_m) - V), the noise regenerated from the same
 * counters as smppi_rollout.  V_plus may equal V (in place). */
smppi_status smppi_update(smppi_ctx ctx, const smppi_batch* batch, const smppi_model* model,
                          const smppi_cost* cost, const smppi_noise* noise, const void* V, const void* w,
                          const uint32_t* iter, void* V_plus, void* stream);

/* Adjoint rollout: grad_V = sum_m grad_S[m] dL_m/dV for the objective above,
 * where sample m's trajectory uses the same noise as smppi_rollout.  States are
 * recomputed from per-sample checkpoints (every min(ceil(sqrt(t_max)), 12)
 * steps, in the ctx scratch, with each step's window segment) instead of being
 * stored.  Every 64 samples write a partial; a second small kernel adds them in a fixed order
 * (the result does not depend on scheduling).  grad_V has the
 * layout of V (dtype).  Gradients pass through the clip where it is inactive and
 * through the hinge where it is active (one-sided at ties). */
smppi_status smppi_rollout_backward(smppi_ctx ctx, const smppi_batch* batch, const smppi_model* model,
                                    const smppi_cost* cost, const smppi_noise* noise,
                                    const smppi_track* track, const void* x0, const void* V,
                                    const uint32_t* iter, const void* grad_S,
                                    const smppi_objective* objective, void* grad_V, void* stream);

/* smppi_rollout_backward for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): same arguments, same kernels and results, but the ticket
 * counters and per-workgroup partials live in a fixed scratch array that each
 * GPU holds for the life of the process (looked up at smppi_create), so no
 * smppi_reserve_batch is needed and nothing is allocated.  Limits: at most 4096
 * ticket counters (B x ceil(2 t_max / 64)) and at most 64 MiB of partials,
 * slice sums, per-lane checkpoints and window indices (about B x n x (2 t_max x
 * dtype bytes + 64 x (ceil(t_max / s) x (8 dtype bytes + 4) + 4 t_max)) bytes,
 * n = ceil(k_max / 64), s = min(ceil(sqrt(t_max)), 12); K = 65536 at T = 100
 * needs about 51 MB), else SMPPI_ERR_SHAPE before anything is enqueued.  Every call on a
 * GPU shares that GPU's array (the counters are cleared by a kernel at the
 * start of each call): calls that overlap on one GPU, from any ctx or thread,
 * race and must be ordered by the caller. */
smppi_status smppi_rollout_backward_noalloc(smppi_ctx ctx, const smppi_batch* batch, const smppi_model* model,
                                            const smppi_cost* cost, const smppi_noise* noise,
                                            const smppi_track* track, const void* x0, const void* V,
                                            const uint32_t* iter, const void* grad_S,
                                            const smppi_objective* objective, void* grad_V, void* stream);

/* Safety shield (Algorithm 1, eq. (22)): V_safe = repair of V_plus from x0 (see
 * smppi_repair_opts).  V_safe may equal V_plus. */
smppi_status smppi_shield_repair(smppi_ctx ctx, const smppi_batch* batch, const smppi_model* model,
                                 const smppi_cost* cost, const smppi_track* track, const void* x0,
                                 const void* V_plus, const smppi_repair_opts* opts, void* V_safe,
                                 void* stream);

/* Execute and warm start (Algorithm 2, last two lines; disturbed plant of eq.
 * (26)): x[b] <- RK4(x[b], first control of V_exec) + (0,0,0,0,dist_vy,dist_om),
 * V[b] <- V_plus[b] shifted one step (last step repeated), iter[b] += 1.
 * dist: NULL or device [n_dist][B][2] dtype; row iter[b] (before the increment)
 * is used when iter[b] < n_dist, otherwise no disturbance. */
smppi_status smppi_execute(smppi_ctx ctx, const smppi_batch* batch, const smppi_model* model,
                           const void* V_exec, const void* V_plus, const void* dist, int32_t n_dist,
                           void* x, void* V, uint32_t* iter, void* stream);

/* ---- batched plan: one persistent fused launch, captured in a HIP graph ------ */

typedef struct {
  double lambda;             /* softmax temperature */
  int32_t repair;            /* nonzero: run the shield after the update */
  smppi_repair_opts repair_opts;
  int32_t execute;           /* nonzero: run smppi_execute after (V_exec = V_safe or V_plus) */
  const void* dist;          /* as smppi_execute */
  int32_t n_dist;
  int32_t block;             /* threads per workgroup (64, 128, 256 or 512); 0 = 256 */
  int32_t tile;              /* samples per tile (multiple of block); 0 = 2 block when the
                                batch has at least 16 block samples per CU, else block */
  int32_t grid;              /* persistent workgroups; 0 = chosen from occupancy */
  int32_t use_graph;         /* nonzero: capture into a hipGraph at creation when a launch
                                has more than one kernel (one kernel is launched directly) */
  int32_t pipeline;          /* 1: latency mode (64-sample tiles, four specialised waves
                                pipelining noise, dynamics and cost); -1: off; 0: on when
                                the batch has at most 2*64 samples per compute unit and
                                no obstacles */
  int32_t fuse_shield;       /* 1: run the shield (and execute) of each problem inside the
                                fused launch, in the workgroup that combines the problem,
                                when its workgroups have at least three waves and the LDS
                                fits; 0: the same in latency mode, a separate shield kernel
                                otherwise (measured faster for tile-mode batches); -1:
                                always a separate shield kernel.  The results are the same
                                bit for bit. */
} smppi_plan_opts;

/* Buffers a plan reads and writes on every launch (device pointers, dtype F32):
 * x0 [B][6] (state; advanced in place when execute is set), V (controls; replaced
 * by the warm start when execute is set, else read only), iter [B] (incremented
 * when execute is set), S [sum K] out, V_plus out, stats [B][4] out, V_safe out
 * (NULL when repair is off). */
typedef struct {
  void* x0;
  void* V;
  uint32_t* iter;
  void* S;
  void* V_plus;
  void* stats;
  void* V_safe;
} smppi_plan_buffers;

/* Build a plan for `batch` (which must stay valid, with its device arrays, for
 * the plan's life): tile list in longest-first order, per-problem ticket
 * counters, and (use_graph) the captured graph.  The batch's offsets (k_off,
 * t_off; with one problem also the track's poly_off and obs_off) are read once,
 * here: later changes to them are not seen by the plan's launches (the rows
 * they point to, x0, V and iter are read on every launch).  The first launch
 * of a plan resets nothing the caller owns. */
smppi_status smppi_plan_create(smppi_ctx ctx, const smppi_batch* batch, const smppi_model* model,
                               const smppi_cost* cost, const smppi_noise* noise, const smppi_track* track,
                               const smppi_plan_opts* opts, const smppi_plan_buffers* bufs,
                               smppi_plan* out);
/* One MPPI iteration of every problem: rollout, weights and update fused in one
 * persistent launch, then (optionally) the shield and the execute/warm start.
 * With obstacles outside latency mode, a small kernel first copies the current
 * obstacles into padded slots the plan owns (one slot per lane of each wave
 * of the rollouts). */
smppi_status smppi_plan_launch(smppi_plan plan, void* stream);
void smppi_plan_destroy(smppi_plan plan);
/* Profiling: the same work as smppi_plan_launch, enqueued without the graph and
 * with HIP events recorded between the stages on `stream`; smppi_plan_stage_ms
 * waits for the last profiled launch and returns its stage durations (ms):
 * reset + fused rollout/weights/update, shield repair, execute/warm start. */
smppi_status smppi_plan_launch_profiled(smppi_plan plan, void* stream);
smppi_status smppi_plan_stage_ms(smppi_plan plan, float* fused_ms, float* repair_ms, float* execute_ms);
/* Kernel-only durations (ms) of the last profiled launch: the fused
 * rollout/weights/update kernel and the shield kernel, from events stamped with
 * each kernel's own start and end (no launch gaps); 0 for a stage the plan does
 * not run.  Waits for the last profiled launch; INVALID_ARGUMENT before one. */
smppi_status smppi_plan_kernel_ms(smppi_plan plan, float* fused_ms, float* repair_ms);
/* Launch geometry the plan uses (any output pointer may be NULL). */
smppi_status smppi_plan_info(smppi_plan plan, int32_t* grid, int32_t* block, int32_t* tile, int32_t* n_tiles);

/* ---- launch-geometry autotuner (plan helper) ---------------------------------
 * The fused plan kernel has four knobs: the four-wave latency mode, the
 * workgroup size, the samples per tile and the number of persistent
 * workgroups.  Which is fastest depends on the batch shape (a few thousand
 * samples are bound by each wave's per-step chain, hundreds of thousands by
 * VALU issue, ragged batches by the tail of the tile queue), so the tuner
 * times candidates on the caller's own batch. */
typedef struct {
  int32_t pipeline;  /* 1: latency mode (block, tile ignored); -1: tile mode */
  int32_t block;     /* tile mode: 64, 128, 256 or 512 */
  int32_t tile;      /* tile mode: samples per tile, a multiple of block */
  int32_t grid;      /* persistent workgroups; 0 = from occupancy */
  float kernel_ms;   /* output: median fused-kernel time; negative when the
                        candidate could not be built for this batch */
} smppi_tune_entry;

/* The default candidate set for n_cu compute units (host only, no device):
 * latency mode, then block {64,128,256,512} x samples per thread {1,2,4}
 * (block x samples <= 1024) x grid {occupancy, 1, 2, 4 per CU}.  Writes up to
 * cap entries to out (may be NULL with cap 0) and returns the set's size. */
int32_t smppi_autotune_candidates(int32_t n_cu, smppi_tune_entry* out, int32_t cap);

/* Shape key under which a tuning result is cached (host only, no device):
 * "B<n>-sk<round(8 log2 sum K)>-kmax<K>-tmax<T>-tmean<mean T, 1 decimal>-obs<0|1>-cu<n_cu>"
 * from host copies of the batch's CSR offsets (k_off_host [B+1], t_off_host
 * [B+1]).  INVALID_ARGUMENT on NULL pointers, B < 1 or a key longer than cap - 1. */
smppi_status smppi_autotune_key(int32_t n_problems, const int64_t* k_off_host, const int32_t* t_off_host,
                                int32_t has_obstacles, int32_t n_cu, char* out, int32_t cap);

/* Times each candidate (cands [n_cands] host, or the default set when cands is
 * NULL) on this batch: a plan with the shield, execute and graph off, warmup +
 * reps profiled launches, the median of the fused kernel's own duration.
 * table (host, table_cap entries, may be NULL) receives the candidates, the
 * timed ones fastest first, then those that cannot be built for this batch
 * (kernel_ms = -1); *n_table their count (entries beyond table_cap are
 * dropped); *best the fastest.  bufs as for a plan
 * (V_safe unused); x0, V and iter are only read, S, V_plus and stats are
 * overwritten.  With cache_path (host string, may be NULL): a result stored
 * under the batch's shape key is returned without timing, *cached = 1 (table
 * then holds that one entry), unless force; a new result replaces the key's line
 * of the file (text, one "key pipeline block tile grid kernel_ms" line per key,
 * written to a temporary file in the same directory and renamed; the directory
 * must exist).  Not for hot loops: it creates plans (device allocations),
 * synchronises the device and does file I/O.  Errors: as smppi_plan_create for
 * the batch; SMPPI_ERR_SHAPE when no candidate can be built; SMPPI_ERR_HIP on
 * cache I/O failure (the timing result is still returned). */
smppi_status smppi_autotune(smppi_ctx ctx, const smppi_batch* batch, const smppi_model* model,
                            const smppi_cost* cost, const smppi_noise* noise, const smppi_track* track,
                            double lambda, const smppi_plan_buffers* bufs, const smppi_tune_entry* cands,
                            int32_t n_cands, int32_t reps, int32_t warmup, const char* cache_path, int32_t force,
                            smppi_tune_entry* best, int32_t* cached, smppi_tune_entry* table, int32_t table_cap,
                            int32_t* n_table, void* stream);

/* ---- test hooks: the device generator, evaluated on its own ---------------- */

/* out[4*i + j] = word j of Philox4x32-10(ctr[4*i .. 4*i+3], key = key[0..1]).
 * ctr: device [n][4] uint32; out: device [n][4] uint32. */
smppi_status smppi_debug_philox(smppi_ctx ctx, const uint32_t* ctr, const uint32_t* key_host, int64_t n,
                                uint32_t* out, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* SMPPI_H */
