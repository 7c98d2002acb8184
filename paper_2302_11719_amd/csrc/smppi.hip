// Host side of the C ABI: context, validation, scratch, dispatch of the plain
// (one call per stage) path.  The batched persistent plan lives in plan.hip.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/smppi.h"
#include "common.hpp"
#include "kernels.hpp"
#include "curv8.hpp"

using namespace smppi;

// ------------------------------------------------------------------ helpers
smppi_status smppi::fail(smppi_ctx ctx, smppi_status s, const char* fmt, ...) {
  if (ctx) {  // formatted into the ctx's fixed buffer: error paths allocate nothing either
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(ctx->last, sizeof(ctx->last), fmt, ap);
    va_end(ap);
  }
  return s;
}

smppi_status smppi::hip_fail(smppi_ctx ctx, hipError_t e, const char* what) {
  return fail(ctx, SMPPI_ERR_HIP, "%s: %s (%d)", what, hipGetErrorString(e), (int)e);
}

smppi_status smppi::ensure_scratch(smppi_ctx ctx, size_t bytes) {
  if (bytes <= ctx->scratch_bytes) return SMPPI_OK;
  size_t want = bytes + bytes / 2 + (1u << 20);
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, want);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipMalloc(scratch)");
  // In-flight work may still read the old buffer: keep it until destroy.
  if (ctx->scratch) ctx->retired.push_back(ctx->scratch);
  ctx->scratch = p;
  ctx->scratch_bytes = want;
  return SMPPI_OK;
}

smppi_status smppi::ensure_tickets(smppi_ctx ctx, int n) {
  if (n <= ctx->n_tickets) return SMPPI_OK;
  int want = n + n / 2 + 64;
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, sizeof(uint32_t) * want);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipMalloc(tickets)");
  e = hipMemset(p, 0, sizeof(uint32_t) * want);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipMemset(tickets)");
  if (ctx->tickets) ctx->retired.push_back(ctx->tickets);
  ctx->tickets = static_cast<uint32_t*>(p);
  ctx->n_tickets = want;
  return SMPPI_OK;
}

// The adjoint's scratch for a batch: per-workgroup partials [B][nblk][2][t_max],
// slice sums [B][ceil(nblk / SUM_SLICE)][2][t_max] (dtype) and ticket counters
// [B][ceil(2 t_max / 64)] for the sum kernel.
AdjScratch smppi::adjoint_scratch(const smppi_batch* b) {
  AdjScratch a;
  a.r = b->dtype == SMPPI_F32 ? sizeof(float) : sizeof(double);
  a.nblk = std::max(1, (std::max(0, b->k_max) + WAVE - 1) / WAVE);
  a.n_slices = (a.nblk + SUM_SLICE - 1) / SUM_SLICE;
  a.n_chunks = (2 * b->t_max + WAVE - 1) / WAVE;
  const size_t row = a.r * 2 * (size_t)b->t_max;
  a.part_bytes = row * b->n_problems * a.nblk;
  // slice sums, then the per-problem validity flags (16-byte aligned)
  a.slice_bytes = ((row * b->n_problems * a.n_slices + 15) & ~(size_t)15) + sizeof(uint32_t) * b->n_problems;
  // checkpoints (8 state components covers both models), 256-byte aligned
  const int seg = adj_seg_len(b->t_max);
  a.ck_off = (a.part_bytes + a.slice_bytes + 255) & ~(size_t)255;
  // (8 components and the per-step window indices cover both models' layouts)
  a.ck_bytes = (size_t)b->n_problems * a.nblk *
               (a.r == sizeof(float) ? adj_ck_bytes_per_wg<float>(b->t_max, seg, 8, true)
                                     : adj_ck_bytes_per_wg<double>(b->t_max, seg, 8, true));
  // padded obstacle slots of the FP32 adjoint ([B][64] float4), after the checkpoints
  a.pad_off = (a.ck_off + a.ck_bytes + 255) & ~(size_t)255;
  a.pad_bytes = b->dtype == SMPPI_F32 ? sizeof(float4) * (size_t)b->n_problems * kMaxObs : 0;
  a.tickets = (size_t)b->n_problems * a.n_chunks;
  a.n_problems = b->n_problems;
  return a;
}

// Scratch of the plain calls for a batch within these host bounds: the
// update's per-workgroup partials [B][workgroups][2][t_max], the adjoint's
// (adjoint_scratch) and, for FP32 rollouts with obstacles, the padded obstacle
// slots [B][64].
size_t smppi::batch_scratch_bytes(const smppi_batch* b) {
  const size_t r = b->dtype == SMPPI_F32 ? sizeof(float) : sizeof(double);
  const size_t B = (size_t)b->n_problems, k = (size_t)std::max(0, b->k_max), t = (size_t)b->t_max;
  const size_t upd = r * B * std::max<size_t>(1, (k + UPD_BLOCK - 1) / UPD_BLOCK) * 2 * t;
  const AdjScratch adj = adjoint_scratch(b);
  const size_t bwd = adj.pad_off + adj.pad_bytes;
  const size_t pad = b->dtype == SMPPI_F32 ? sizeof(float4) * B * kMaxObs : 0;
  return std::max(upd, std::max(bwd, pad));
}

smppi_status smppi::need_scratch(smppi_ctx ctx, size_t bytes, int tickets, const char* what) {
  if (bytes <= ctx->scratch_bytes && tickets <= ctx->n_tickets) return SMPPI_OK;
  return fail(ctx, SMPPI_ERR_SHAPE,
              "%s needs %zu B of scratch and %d tickets, the ctx holds %zu B and %d: size it with "
              "smppi_reserve_batch for this batch first",
              what, bytes, tickets, ctx->scratch_bytes, ctx->n_tickets);
}

smppi_status smppi::check_launch(smppi_ctx ctx, const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(ctx, e, what);
  return SMPPI_OK;
}

smppi_status smppi::validate_batch(smppi_ctx ctx, const smppi_batch* b) {
  if (!b) return fail(ctx, SMPPI_ERR_INVALID_ARGUMENT, "batch is NULL");
  if (b->n_problems < 1) return fail(ctx, SMPPI_ERR_SHAPE, "n_problems must be >= 1 (got %d)", b->n_problems);
  if (b->n_problems > 65535) return fail(ctx, SMPPI_ERR_SHAPE, "n_problems must be <= 65535");
  if (b->k_max < 0) return fail(ctx, SMPPI_ERR_SHAPE, "k_max must be >= 0");
  if (b->t_max < 1 || b->t_max > kMaxT) return fail(ctx, SMPPI_ERR_SHAPE, "t_max must be in [1, %d]", kMaxT);
  if (b->pid_base < 0) return fail(ctx, SMPPI_ERR_INVALID_ARGUMENT, "pid_base must be >= 0");
  if (b->dtype != SMPPI_F32 && b->dtype != SMPPI_F64) return fail(ctx, SMPPI_ERR_DTYPE, "unknown dtype");
  if (!b->k_off || !b->t_off) return fail(ctx, SMPPI_ERR_INVALID_ARGUMENT, "k_off/t_off must be device pointers");
  return SMPPI_OK;
}

smppi_status smppi::validate_model(smppi_ctx ctx, const smppi_model* m) {
  if (!m) return fail(ctx, SMPPI_ERR_INVALID_ARGUMENT, "model is NULL");
  const double pos[] = {m->m, m->lf, m->lr, m->Iz, m->Cf, m->Cr, m->dt, m->v_min};
  for (double v : pos)
    if (!(v > 0.0) || !std::isfinite(v))
      return fail(ctx, SMPPI_ERR_INVALID_ARGUMENT, "model: m, lf, lr, Iz, Cf, Cr, dt, v_min must be > 0");
  if (!std::isfinite(m->a_max) || !std::isfinite(m->c_v))
    return fail(ctx, SMPPI_ERR_INVALID_ARGUMENT, "model: a_max, c_v must be finite");
  for (int d = 0; d < 2; ++d)
    if (!(m->u_lo[d] < m->u_hi[d])) return fail(ctx, SMPPI_ERR_INVALID_ARGUMENT, "model: u_lo must be < u_hi");
  return SMPPI_OK;
}

smppi_status smppi::validate_cost(smppi_ctx ctx, const smppi_cost* c) {
  if (!c) return fail(ctx, SMPPI_ERR_INVALID_ARGUMENT, "cost is NULL");
  if (!(c->sigma[0] > 0.0) || !(c->sigma[1] > 0.0))
    return fail(ctx, SMPPI_ERR_INVALID_ARGUMENT, "cost: sigma must be > 0");
  if (!(c->gamma > 0.0 && c->gamma < 1.0))
    return fail(ctx, SMPPI_ERR_INVALID_ARGUMENT, "cost: gamma must be in (0, 1)");
  const double fin[] = {c->v_g, c->q_v, c->q_ey, c->C_obs, c->phi_w, c->lambda_u, c->C_cbf};
  for (double v : fin)
    if (!std::isfinite(v)) return fail(ctx, SMPPI_ERR_INVALID_ARGUMENT, "cost: parameters must be finite");
  return SMPPI_OK;
}

smppi_status smppi::validate_track(smppi_ctx ctx, const smppi_track* t, smppi_dtype dt, int t_max) {
  if (!t) return fail(ctx, SMPPI_ERR_INVALID_ARGUMENT, "track is NULL");
  if (!t->poly_off || !t->circle || !t->half_width)
    return fail(ctx, SMPPI_ERR_INVALID_ARGUMENT, "track: poly_off, circle, half_width are required");
  if (t->poly_max < 0 || t->poly_max > kMaxPoly)
    return fail(ctx, SMPPI_ERR_SHAPE, "track: poly_max must be in [0, %d]", kMaxPoly);
  if (t->poly_max > 0 && !t->poly) return fail(ctx, SMPPI_ERR_INVALID_ARGUMENT, "track: poly is NULL");
  if (t->obs_max < 0 || t->obs_max > kMaxObs)
    return fail(ctx, SMPPI_ERR_SHAPE, "track: obs_max must be in [0, %d]", kMaxObs);
  if (t->obs_max > 0 && (!t->obs || !t->obs_off))
    return fail(ctx, SMPPI_ERR_INVALID_ARGUMENT, "track: obs/obs_off are NULL with obs_max > 0");
  if (t->poly_max > 0 && (t->window < 1 || 2 * t->window + 1 > t->poly_max))
    return fail(ctx, SMPPI_ERR_INVALID_ARGUMENT, "track: window must satisfy 1 <= window, 2*window+1 <= poly_max");
  const int slots = obs_slots(t);
  const size_t lds = dt == SMPPI_F32 ? stage_lds_bytes<float>(t->poly_max, t_max, slots)
                                     : stage_lds_bytes<double>(t->poly_max, t_max, slots);
  if (lds > (size_t)kMaxStageLds)
    return fail(ctx, SMPPI_ERR_SHAPE, "track: polyline + control staging needs %zu B of LDS (max %d)", lds,
                kMaxStageLds);
  return SMPPI_OK;
}

template <class R>
DevModel<R> smppi::dev_model(const smppi_model* m) {
  DevModel<R> d;
  d.lf = (R)m->lf;
  d.lr = (R)m->lr;
  d.Cf = (R)m->Cf;
  d.Cr = (R)m->Cr;
  d.a_max = (R)m->a_max;
  d.c_v = (R)m->c_v;
  d.v_min = (R)m->v_min;
  d.dt = (R)m->dt;
  d.inv_m = (R)(1.0 / m->m);
  d.lr_Iz = (R)(m->lr / m->Iz);
  d.lf_Iz = (R)(m->lf / m->Iz);
  for (int i = 0; i < 2; ++i) {
    d.u_lo[i] = (R)m->u_lo[i];
    d.u_hi[i] = (R)m->u_hi[i];
  }
  return d;
}

template <class R>
DevCost<R> smppi::dev_cost(const smppi_cost* c) {
  DevCost<R> d;
  d.v_g = (R)c->v_g;
  d.q_v = (R)c->q_v;
  d.q_ey = (R)c->q_ey;
  d.C_obs = (R)c->C_obs;
  d.phi_w = (R)c->phi_w;
  for (int i = 0; i < 2; ++i) {
    d.ctrl_w[i] = (R)(c->lambda_u / (c->sigma[i] * c->sigma[i]));
    d.sigma[i] = (R)c->sigma[i];
  }
  d.C_cbf = (R)c->C_cbf;
  d.alpha = (R)(1.0 - c->gamma);
  return d;
}

template <class R>
DevObjective<R> smppi::dev_objective(const smppi_objective* o) {
  DevObjective<R> d;
  d.w_S = (R)o->w_S;
  d.w_sq = (R)o->w_sq;
  d.w_lin = (R)o->w_lin;
  d.n_lin = o->n_lin;
  return d;
}

template DevModel<float> smppi::dev_model<float>(const smppi_model*);
template DevCost<float> smppi::dev_cost<float>(const smppi_cost*);
template DevObjective<float> smppi::dev_objective<float>(const smppi_objective*);

template <class R>
ProblemArgs<R> smppi::problem_args(smppi_ctx ctx, const smppi_batch* b, const smppi_track* t,
                                   const smppi_noise* n, const void* x0, const uint32_t* iter) {
  ProblemArgs<R> p;
  p.k_off = b->k_off;
  p.t_off = b->t_off;
  p.poly_off = t ? t->poly_off : nullptr;
  p.poly = t ? static_cast<const R*>(t->poly) : nullptr;
  p.circle = t ? static_cast<const R*>(t->circle) : nullptr;
  p.half_width = t ? static_cast<const R*>(t->half_width) : nullptr;
  p.obs_off = (t && t->obs_max > 0) ? t->obs_off : nullptr;
  p.obs = (t && t->obs_max > 0) ? static_cast<const R*>(t->obs) : nullptr;
  p.x0 = static_cast<const R*>(x0);
  p.iter = iter;
  p.k_max = b->k_max;
  p.t_max = b->t_max;
  p.poly_max = t ? t->poly_max : 0;
  p.obs_max = t ? obs_slots(t) : 0;
  p.window = t ? t->window : 1;
  p.pid_base = b->pid_base;
  p.seed = n ? n->seed : 0u;
  p.nominal = n ? n->nominal : 1;
  p.err = ctx->err;
  return p;
}

template ProblemArgs<float> smppi::problem_args<float>(smppi_ctx, const smppi_batch*, const smppi_track*,
                                                       const smppi_noise*, const void*, const uint32_t*);

// Steps per recomputed segment of the adjoint: ceil(sqrt(t_max)) (fewest
// checkpoint plus segment slots), at most 12 so that the segment held in LDS
// (13 slots) leaves room for four workgroups per CU beside a 512-segment track;
// longer horizons only keep more checkpoints in the global scratch.
int smppi::adj_seg_len(int t_max) {
  int s = (int)std::ceil(std::sqrt((double)t_max));
  return s < 1 ? 1 : (s > ADJ_SEG_MAX ? ADJ_SEG_MAX : s);
}

// ------------------------------------------------------------------ context
extern "C" int smppi_abi_version(void) { return SMPPI_ABI_VERSION; }

extern "C" const char* smppi_status_string(smppi_status s) {
  switch (s) {
    case SMPPI_OK: return "ok";
    case SMPPI_ERR_INVALID_ARGUMENT: return "invalid argument";
    case SMPPI_ERR_SHAPE: return "shape";
    case SMPPI_ERR_DTYPE: return "dtype";
    case SMPPI_ERR_NO_DEVICE: return "no device";
    case SMPPI_ERR_HIP: return "hip error";
    case SMPPI_ERR_UNSUPPORTED: return "unsupported";
    case SMPPI_ERR_NONFINITE: return "non-finite";
  }
  return "unknown status";
}

static smppi_status noalloc_setup(smppi_ctx ctx);

extern "C" smppi_status smppi_create(int device, smppi_ctx* out) {
  if (!out) return SMPPI_ERR_INVALID_ARGUMENT;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) return SMPPI_ERR_NO_DEVICE;
  if (device < 0 || device >= n) return SMPPI_ERR_NO_DEVICE;
  smppi_ctx ctx = new smppi_ctx_s();
  ctx->device = device;
  if (hipSetDevice(device) != hipSuccess) {
    delete ctx;
    return SMPPI_ERR_NO_DEVICE;
  }
  (void)hipDeviceGetAttribute(&ctx->n_cu, hipDeviceAttributeMultiprocessorCount, device);
  (void)hipDeviceGetAttribute(&ctx->max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device);
  void* e = nullptr;
  if (hipMalloc(&e, sizeof(uint32_t)) != hipSuccess || hipMemset(e, 0, sizeof(uint32_t)) != hipSuccess) {
    delete ctx;
    return SMPPI_ERR_HIP;
  }
  ctx->err = static_cast<uint32_t*>(e);
  if (noalloc_setup(ctx) != SMPPI_OK) {
    (void)hipFree(ctx->err);
    delete ctx;
    return SMPPI_ERR_HIP;
  }
  *out = ctx;
  return SMPPI_OK;
}

extern "C" void smppi_destroy(smppi_ctx ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  for (void* p : ctx->retired) (void)hipFree(p);
  if (ctx->scratch) (void)hipFree(ctx->scratch);
  if (ctx->tickets) (void)hipFree(ctx->tickets);
  if (ctx->err) (void)hipFree(ctx->err);
  delete ctx;
}

extern "C" const char* smppi_last_error(smppi_ctx ctx) { return ctx ? ctx->last : "no ctx"; }

extern "C" smppi_status smppi_reserve_batch(smppi_ctx ctx, const smppi_batch* batch) {
  if (!ctx) return SMPPI_ERR_INVALID_ARGUMENT;
  smppi_status st;
  if ((st = validate_batch(ctx, batch))) return st;
  (void)hipSetDevice(ctx->device);
  if ((st = ensure_scratch(ctx, batch_scratch_bytes(batch)))) return st;
  return ensure_tickets(ctx, (int)std::max<size_t>(batch->n_problems, adjoint_scratch(batch).tickets));
}

extern "C" smppi_status smppi_device_errors(smppi_ctx ctx, uint32_t* flags) {
  if (!ctx || !flags) return SMPPI_ERR_INVALID_ARGUMENT;
  (void)hipSetDevice(ctx->device);
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(ctx, e, "hipDeviceSynchronize");
  uint32_t v = 0;
  e = hipMemcpy(&v, ctx->err, sizeof(v), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipMemcpy(err)");
  e = hipMemset(ctx->err, 0, sizeof(uint32_t));
  if (e != hipSuccess) return hip_fail(ctx, e, "hipMemset(err)");
  *flags = v;
  return SMPPI_OK;
}

// ------------------------------------------------------------------ rollout
template <class R, int NOBS>
static smppi_status launch_rollout(smppi_ctx ctx, const smppi_batch* b, const RolloutArgs<R>& a, hipStream_t s) {
  const int blk = 256;
  const int gx = b->k_max > 0 ? (b->k_max + blk - 1) / blk : 0;
  if (gx == 0) return SMPPI_OK;
  const size_t lds = stage_lds_bytes<R>(a.p.poly_max, a.p.t_max, a.p.obs_max);
  RolloutArgs<R> ra = a;
  ra.obs_pad = nullptr;
  if (NOBS > 0 && sizeof(R) == 4) {
    // FP32 obstacles are evaluated per wave from padded slots in the scratch buffer
    smppi_status st = need_scratch(ctx, sizeof(float4) * (size_t)b->n_problems * NOBS, 0, "smppi_rollout");
    if (st) return st;
    float4* pad = static_cast<float4*>(ctx->scratch);
    hipLaunchKernelGGL(k_pad_obs, dim3(b->n_problems), dim3(64), 0, s, a.p.obs_off,
                       reinterpret_cast<const float*>(a.p.obs), a.p.obs_max, NOBS, (float)a.C.alpha, pad);
    if ((st = check_launch(ctx, "k_pad_obs"))) return st;
    ra.obs_pad = pad;
  }
  hipLaunchKernelGGL((k_rollout<R, NOBS>), dim3(gx, b->n_problems), dim3(blk), lds, s, ra);
  return check_launch(ctx, "k_rollout");
}

template <class R>
static smppi_status rollout_t(smppi_ctx ctx, const smppi_batch* b, const smppi_model* m, const smppi_cost* c,
                              const smppi_noise* n, const smppi_track* t, const void* x0, const void* V,
                              const uint32_t* iter, void* S, void* eps_out, hipStream_t s) {
  RolloutArgs<R> a;
  a.p = problem_args<R>(ctx, b, t, n, x0, iter);
  a.M = dev_model<R>(m);
  a.C = dev_cost<R>(c);
  a.V = static_cast<const R*>(V);
  a.S = static_cast<R*>(S);
  a.eps_out = static_cast<R*>(eps_out);
  if (t->obs_max > 0) return launch_rollout<R, kMaxObs>(ctx, b, a, s);
  return launch_rollout<R, 0>(ctx, b, a, s);
}

extern "C" smppi_status smppi_rollout(smppi_ctx ctx, const smppi_batch* batch, const smppi_model* model,
                                      const smppi_cost* cost, const smppi_noise* noise, const smppi_track* track,
                                      const void* x0, const void* V, const uint32_t* iter, void* S, void* eps_out,
                                      void* stream) {
  if (!ctx) return SMPPI_ERR_INVALID_ARGUMENT;
  smppi_status st;
  if ((st = validate_batch(ctx, batch)) || (st = validate_model(ctx, model)) || (st = validate_cost(ctx, cost)) ||
      (st = validate_track(ctx, track, batch->dtype, batch->t_max)))
    return st;
  if (!noise) return fail(ctx, SMPPI_ERR_INVALID_ARGUMENT, "noise is NULL");
  if (!x0 || !V || !iter || !S) return fail(ctx, SMPPI_ERR_INVALID_ARGUMENT, "x0, V, iter, S are required");
  (void)hipSetDevice(ctx->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (batch->dtype == SMPPI_F32)
    return rollout_t<float>(ctx, batch, model, cost, noise, track, x0, V, iter, S, eps_out, s);
  return rollout_t<double>(ctx, batch, model, cost, noise, track, x0, V, iter, S, eps_out, s);
}

// The per-problem validity flags at the end of the adjoint scratch.
static uint32_t* adjoint_valid(const AdjScratch& as, void* scratch) {
  return reinterpret_cast<uint32_t*>(static_cast<unsigned char*>(scratch) + as.part_bytes + as.slice_bytes) -
         as.n_problems;
}

// The sum of the adjoint's per-workgroup partials into grad_V (k_sum_partials):
// part and slice sums in `scratch` (adjoint_scratch layout), counters zero on entry.
template <class R>
static smppi_status launch_sum_partials(smppi_ctx ctx, const smppi_batch* b, const AdjScratch& as, void* scratch,
                                        uint32_t* tickets, void* gV, hipStream_t s) {
  SumArgs<R> sa;
  sa.k_off = b->k_off;
  sa.t_off = b->t_off;
  sa.t_max = b->t_max;
  sa.nblk_max = as.nblk;
  sa.n_slices_max = as.n_slices;
  sa.n_chunks = as.n_chunks;
  sa.part = static_cast<const R*>(scratch);
  sa.slice = reinterpret_cast<R*>(static_cast<unsigned char*>(scratch) + as.part_bytes);
  sa.valid = adjoint_valid(as, scratch);
  sa.tickets = tickets;
  sa.out = static_cast<R*>(gV);
  hipLaunchKernelGGL((k_sum_partials<R>), dim3(as.n_chunks, b->n_problems, as.n_slices), dim3(WAVE), 0, s, sa);
  return check_launch(ctx, "k_sum_partials");
}

// ------------------------------------------------------------------ curvilinear model
static smppi_status validate_curv(smppi_ctx ctx, const smppi_wheels* wh, const smppi_curv_track* t) {
  if (!wh) return fail(ctx, SMPPI_ERR_INVALID_ARGUMENT, "wheels are required");
  if (!(wh->r_w > 0.0) || !(wh->I_w > 0.0) || !(wh->C_x > 0.0) || !std::isfinite(wh->r_w) ||
      !std::isfinite(wh->I_w) || !std::isfinite(wh->C_x))
    return fail(ctx, SMPPI_ERR_INVALID_ARGUMENT, "wheels: r_w, I_w, C_x must be finite and > 0");
  if (!t) return fail(ctx, SMPPI_ERR_INVALID_ARGUMENT, "track is required");
  if (!t->kappa_off || !t->kappa || !t->ds || !t->half_width)
    return fail(ctx, SMPPI_ERR_INVALID_ARGUMENT, "curvature track arrays are required");
  if (t->n_max < 2 || t->n_max > 8192) return fail(ctx, SMPPI_ERR_SHAPE, "n_max must be in [2, 8192]");
  return SMPPI_OK;
}

template <class R>
static C8Args<R> c8_args(smppi_ctx ctx, const smppi_batch* b, const smppi_model* m, const smppi_wheels* wh,
                         const smppi_cost* c, const smppi_noise* n, const smppi_curv_track* t, const void* x0,
                         const void* V, const uint32_t* iter) {
  C8Args<R> a;
  a.k_off = b->k_off;
  a.t_off = b->t_off;
  a.kappa_off = t->kappa_off;
  a.kappa = static_cast<const R*>(t->kappa);
  a.ds = static_cast<const R*>(t->ds);
  a.half_width = static_cast<const R*>(t->half_width);
  a.x0 = static_cast<const R*>(x0);
  a.iter = iter;
  a.V = static_cast<const R*>(V);
  a.M = dev_model<R>(m);
  a.Wh.r_w = (R)wh->r_w;
  a.Wh.C_x = (R)wh->C_x;
  a.Wh.rw_Iw = (R)(wh->r_w / wh->I_w);
  a.Wh.drive_Iw = (R)(m->m * m->a_max * wh->r_w / wh->I_w);
  a.C = dev_cost<R>(c);
  a.B = b->n_problems;
  a.k_max = b->k_max;
  a.t_max = b->t_max;
  a.n_max = t->n_max;
  a.pid_base = b->pid_base;
  a.seed = n ? n->seed : 0u;
  a.nominal = n ? n->nominal : 1;
  a.err = ctx->err;
  return a;
}

template <class R>
static smppi_status rollout_c8_t(smppi_ctx ctx, const smppi_batch* b, const C8Args<R>& a, void* S, void* eps_out,
                                 hipStream_t s) {
  const int blk = 256;
  const int gx = b->k_max > 0 ? (b->k_max + blk - 1) / blk : 0;
  if (gx == 0) return SMPPI_OK;
  const size_t lds = c8_stage_bytes<R>(a.n_max, a.t_max);
  if (lds > (size_t)ctx->max_lds)
    return fail(ctx, SMPPI_ERR_SHAPE, "curvilinear rollout needs %zu B of LDS per workgroup (device max %d)", lds,
                ctx->max_lds);
  hipLaunchKernelGGL((k_rollout_c8<R>), dim3(gx, b->n_problems), dim3(blk), lds, s, a, static_cast<R*>(S),
                     static_cast<R*>(eps_out));
  return check_launch(ctx, "k_rollout_c8");
}

extern "C" smppi_status smppi_rollout_curvilinear(smppi_ctx ctx, const smppi_batch* batch, const smppi_model* model,
                                                  const smppi_wheels* wheels, const smppi_cost* cost,
                                                  const smppi_noise* noise, const smppi_curv_track* track,
                                                  const void* x0, const void* V, const uint32_t* iter, void* S,
                                                  void* eps_out, void* stream) {
  if (!ctx) return SMPPI_ERR_INVALID_ARGUMENT;
  smppi_status st;
  if ((st = validate_batch(ctx, batch)) || (st = validate_model(ctx, model)) || (st = validate_cost(ctx, cost)) ||
      (st = validate_curv(ctx, wheels, track)))
    return st;
  if (!noise) return fail(ctx, SMPPI_ERR_INVALID_ARGUMENT, "noise is NULL");
  if (!x0 || !V || !iter || !S) return fail(ctx, SMPPI_ERR_INVALID_ARGUMENT, "x0, V, iter, S are required");
  (void)hipSetDevice(ctx->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (batch->dtype == SMPPI_F32)
    return rollout_c8_t<float>(ctx, batch, c8_args<float>(ctx, batch, model, wheels, cost, noise, track, x0, V, iter),
                               S, eps_out, s);
  return rollout_c8_t<double>(ctx, batch, c8_args<double>(ctx, batch, model, wheels, cost, noise, track, x0, V, iter),
                              S, eps_out, s);
}

template <class R>
static smppi_status backward_c8_t(smppi_ctx ctx, const smppi_batch* b, const C8Args<R>& a,
                                  const smppi_objective* ob, const void* gS, void* gV, hipStream_t s) {
  C8BackwardArgs<R> g;
  g.a = a;
  g.ob = dev_objective<R>(ob);
  g.grad_S = static_cast<const R*>(gS);
  g.grad_V = static_cast<R*>(gV);
  const AdjScratch as = adjoint_scratch(b);
  g.nblk_max = as.nblk;
  g.seg_len = adj_seg_len(b->t_max);
  smppi_status st;
  if ((st = need_scratch(ctx, as.ck_off + as.ck_bytes, (int)as.tickets, "smppi_rollout_backward_curvilinear")))
    return st;
  g.part = static_cast<R*>(ctx->scratch);
  g.valid = adjoint_valid(as, ctx->scratch);
  g.ck = static_cast<unsigned char*>(ctx->scratch) + as.ck_off;
  const size_t lds = c8_stage_bytes<R>(a.n_max, a.t_max) + c8_adj_lds_bytes<R>(a.t_max, g.seg_len);
  if (lds > (size_t)ctx->max_lds)
    return fail(ctx, SMPPI_ERR_SHAPE, "curvilinear adjoint needs %zu B of LDS per workgroup (device max %d)", lds,
                ctx->max_lds);
  hipLaunchKernelGGL((k_backward_c8<R>), dim3(g.nblk_max, b->n_problems), dim3(WAVE), lds, s, g);
  if ((st = check_launch(ctx, "k_backward_c8"))) return st;
  return launch_sum_partials<R>(ctx, b, as, ctx->scratch, ctx->tickets, gV, s);
}

extern "C" smppi_status smppi_rollout_backward_curvilinear(
    smppi_ctx ctx, const smppi_batch* batch, const smppi_model* model, const smppi_wheels* wheels,
    const smppi_cost* cost, const smppi_noise* noise, const smppi_curv_track* track, const void* x0, const void* V,
    const uint32_t* iter, const void* grad_S, const smppi_objective* objective, void* grad_V, void* stream) {
  if (!ctx) return SMPPI_ERR_INVALID_ARGUMENT;
  smppi_status st;
  if ((st = validate_batch(ctx, batch)) || (st = validate_model(ctx, model)) || (st = validate_cost(ctx, cost)) ||
      (st = validate_curv(ctx, wheels, track)) || (st = validate_objective(ctx, objective)))
    return st;
  if (!noise) return fail(ctx, SMPPI_ERR_INVALID_ARGUMENT, "noise is NULL");
  if (!x0 || !V || !iter || !grad_S || !grad_V)
    return fail(ctx, SMPPI_ERR_INVALID_ARGUMENT, "x0, V, iter, grad_S, grad_V are required");
  (void)hipSetDevice(ctx->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (batch->dtype == SMPPI_F32)
    return backward_c8_t<float>(ctx, batch,
                                c8_args<float>(ctx, batch, model, wheels, cost, noise, track, x0, V, iter), objective,
                                grad_S, grad_V, s);
  return backward_c8_t<double>(ctx, batch,
                               c8_args<double>(ctx, batch, model, wheels, cost, noise, track, x0, V, iter), objective,
                               grad_S, grad_V, s);
}

template <class R>
static smppi_status repair_c8_t(smppi_ctx ctx, const smppi_batch* b, const C8Args<R>& a,
                                const smppi_repair_opts* o, const void* Vp, void* Vs, hipStream_t s) {
  C8RepairArgs<R> r;
  r.a = a;
  r.ob = dev_objective<R>(&o->objective);
  r.V_plus = static_cast<const R*>(Vp);
  r.V_safe = static_cast<R*>(Vs);
  r.n_steps = o->n_steps;
  r.step = (R)o->step;
  const size_t lds = c8_repair_lds_bytes<R>(a.n_max, a.t_max);
  if (lds > (size_t)ctx->max_lds)
    return fail(ctx, SMPPI_ERR_SHAPE, "curvilinear shield needs %zu B of LDS per workgroup (device max %d)", lds,
                ctx->max_lds);
  hipLaunchKernelGGL((k_repair_c8<R>), dim3(b->n_problems), dim3(C8_REP_BLK), lds, s, r);
  return check_launch(ctx, "k_repair_c8");
}

extern "C" smppi_status smppi_shield_repair_curvilinear(smppi_ctx ctx, const smppi_batch* batch,
                                                        const smppi_model* model, const smppi_wheels* wheels,
                                                        const smppi_cost* cost, const smppi_curv_track* track,
                                                        const void* x0, const void* V_plus,
                                                        const smppi_repair_opts* opts, void* V_safe, void* stream) {
  if (!ctx) return SMPPI_ERR_INVALID_ARGUMENT;
  smppi_status st;
  if ((st = validate_batch(ctx, batch)) || (st = validate_model(ctx, model)) || (st = validate_cost(ctx, cost)) ||
      (st = validate_curv(ctx, wheels, track)) || (st = validate_repair(ctx, opts)))
    return st;
  if (opts->method != 0)
    return fail(ctx, SMPPI_ERR_UNSUPPORTED, "the curvilinear shield implements Algorithm 1 (method 0) only");
  if (!x0 || !V_plus || !V_safe) return fail(ctx, SMPPI_ERR_INVALID_ARGUMENT, "x0, V_plus, V_safe are required");
  (void)hipSetDevice(ctx->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (batch->dtype == SMPPI_F32)
    return repair_c8_t<float>(
        ctx, batch, c8_args<float>(ctx, batch, model, wheels, cost, nullptr, track, x0, V_plus, nullptr), opts, V_plus,
        V_safe, s);
  return repair_c8_t<double>(
      ctx, batch, c8_args<double>(ctx, batch, model, wheels, cost, nullptr, track, x0, V_plus, nullptr), opts, V_plus,
      V_safe, s);
}

template <class R>
static smppi_status execute_c8_t(smppi_ctx ctx, const smppi_batch* b, const C8Args<R>& a, const void* Ve,
                                 const void* Vp, const void* dist, int32_t n_dist, void* x, void* V, uint32_t* iter,
                                 hipStream_t s) {
  C8ExecArgs<R> e;
  e.a = a;
  e.V_exec = static_cast<const R*>(Ve);
  e.V_plus = static_cast<const R*>(Vp);
  e.dist = static_cast<const R*>(dist);
  e.n_dist = n_dist;
  e.x = static_cast<R*>(x);
  e.V = static_cast<R*>(V);
  e.iter = iter;
  hipLaunchKernelGGL((k_execute_c8<R>), dim3(b->n_problems), dim3(WAVE), sizeof(R) * 2 * b->t_max, s, e);
  return check_launch(ctx, "k_execute_c8");
}

extern "C" smppi_status smppi_execute_curvilinear(smppi_ctx ctx, const smppi_batch* batch, const smppi_model* model,
                                                  const smppi_wheels* wheels, const smppi_curv_track* track,
                                                  const void* V_exec, const void* V_plus, const void* dist,
                                                  int32_t n_dist, void* x, void* V, uint32_t* iter, void* stream) {
  if (!ctx) return SMPPI_ERR_INVALID_ARGUMENT;
  smppi_status st;
  if ((st = validate_batch(ctx, batch)) || (st = validate_model(ctx, model)) ||
      (st = validate_curv(ctx, wheels, track)))
    return st;
  if (!V_exec || !V_plus || !x || !V || !iter)
    return fail(ctx, SMPPI_ERR_INVALID_ARGUMENT, "V_exec, V_plus, x, V, iter are required");
  if (dist && n_dist < 0) return fail(ctx, SMPPI_ERR_INVALID_ARGUMENT, "n_dist must be >= 0");
  (void)hipSetDevice(ctx->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  smppi_cost dummy{};
  dummy.sigma[0] = dummy.sigma[1] = 1.0;
  if (batch->dtype == SMPPI_F32)
    return execute_c8_t<float>(ctx, batch,
                               c8_args<float>(ctx, batch, model, wheels, &dummy, nullptr, track, x, V_plus, nullptr),
                               V_exec, V_plus, dist, n_dist, x, V, iter, s);
  return execute_c8_t<double>(ctx, batch,
                              c8_args<double>(ctx, batch, model, wheels, &dummy, nullptr, track, x, V_plus, nullptr),
                              V_exec, V_plus, dist, n_dist, x, V, iter, s);
}

// ------------------------------------------------------------------ weights
extern "C" smppi_status smppi_weights(smppi_ctx ctx, const smppi_batch* batch, const void* S, double lambda, void* w,
                                      void* stats, void* stream) {
  if (!ctx) return SMPPI_ERR_INVALID_ARGUMENT;
  smppi_status st;
  if ((st = validate_batch(ctx, batch))) return st;
  if (!(lambda > 0.0) || !std::isfinite(lambda)) return fail(ctx, SMPPI_ERR_INVALID_ARGUMENT, "lambda must be > 0");
  if (!S || !w || !stats) return fail(ctx, SMPPI_ERR_INVALID_ARGUMENT, "S, w, stats are required");
  (void)hipSetDevice(ctx->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (batch->dtype == SMPPI_F32)
    hipLaunchKernelGGL((k_weights<float>), dim3(batch->n_problems), dim3(256), 0, s, batch->k_off,
                       static_cast<const float*>(S), (float)(1.0 / lambda), static_cast<float*>(w),
                       static_cast<float*>(stats));
  else
    hipLaunchKernelGGL((k_weights<double>), dim3(batch->n_problems), dim3(256), 0, s, batch->k_off,
                       static_cast<const double*>(S), 1.0 / lambda, static_cast<double*>(w),
                       static_cast<double*>(stats));
  return check_launch(ctx, "k_weights");
}

// ------------------------------------------------------------------ update
template <class R>
static smppi_status update_t(smppi_ctx ctx, const smppi_batch* b, const smppi_model* m, const smppi_cost* c,
                             const smppi_noise* n, const void* V, const void* w, const uint32_t* iter, void* Vp,
                             hipStream_t s) {
  UpdateArgs<R> a;
  a.p = problem_args<R>(ctx, b, nullptr, n, nullptr, iter);
  a.M = dev_model<R>(m);
  a.C = dev_cost<R>(c);
  a.V = static_cast<const R*>(V);
  a.w = static_cast<const R*>(w);
  a.V_plus = static_cast<R*>(Vp);
  a.nblk_max = std::max(1, (b->k_max + UPD_BLOCK - 1) / UPD_BLOCK);
  smppi_status st;
  if ((st = need_scratch(ctx, sizeof(R) * (size_t)b->n_problems * a.nblk_max * 2 * b->t_max, b->n_problems,
                         "smppi_update")))
    return st;
  a.part = static_cast<R*>(ctx->scratch);
  a.tickets = ctx->tickets;
  hipLaunchKernelGGL((k_update<R>), dim3(a.nblk_max, b->n_problems), dim3(UPD_BLOCK), 0, s, a);
  return check_launch(ctx, "k_update");
}

extern "C" smppi_status smppi_update(smppi_ctx ctx, const smppi_batch* batch, const smppi_model* model,
                                     const smppi_cost* cost, const smppi_noise* noise, const void* V, const void* w,
                                     const uint32_t* iter, void* V_plus, void* stream) {
  if (!ctx) return SMPPI_ERR_INVALID_ARGUMENT;
  smppi_status st;
  if ((st = validate_batch(ctx, batch)) || (st = validate_model(ctx, model)) || (st = validate_cost(ctx, cost)))
    return st;
  if (!noise) return fail(ctx, SMPPI_ERR_INVALID_ARGUMENT, "noise is NULL");
  if (!V || !w || !iter || !V_plus) return fail(ctx, SMPPI_ERR_INVALID_ARGUMENT, "V, w, iter, V_plus are required");
  (void)hipSetDevice(ctx->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (batch->dtype == SMPPI_F32) return update_t<float>(ctx, batch, model, cost, noise, V, w, iter, V_plus, s);
  return update_t<double>(ctx, batch, model, cost, noise, V, w, iter, V_plus, s);
}

// ------------------------------------------------------------------ adjoint
template <class R, int NOBS>
static smppi_status launch_backward(smppi_ctx ctx, const smppi_batch* b, const BackwardArgs<R>& a, hipStream_t s) {
  const size_t lds = stage_lds_bytes<R>(a.p.poly_max, a.p.t_max, a.p.obs_max) + adj_lds_bytes<R>(a.p.t_max, a.seg_len);
  if (lds > (size_t)ctx->max_lds)
    return fail(ctx, SMPPI_ERR_SHAPE, "adjoint needs %zu B of LDS per workgroup (device max %d)", lds, ctx->max_lds);
  hipLaunchKernelGGL((k_backward<R, NOBS>), dim3(a.nblk_max, b->n_problems), dim3(WAVE), lds, s, a);
  return check_launch(ctx, "k_backward");
}

// The adjoint launch with its scratch given (adjoint_scratch layout: partials
// then slice sums; counters zero on entry, reset by the sum kernel).
template <class R>
static smppi_status backward_launch(smppi_ctx ctx, const smppi_batch* b, const smppi_model* m, const smppi_cost* c,
                                    const smppi_noise* n, const smppi_track* t, const void* x0, const void* V,
                                    const uint32_t* iter, const void* gS, const smppi_objective* ob, void* gV,
                                    void* scratch, uint32_t* tickets, hipStream_t s) {
  const AdjScratch as = adjoint_scratch(b);
  BackwardArgs<R> a;
  a.p = problem_args<R>(ctx, b, t, n, x0, iter);
  a.M = dev_model<R>(m);
  a.C = dev_cost<R>(c);
  a.ob = dev_objective<R>(ob);
  a.V = static_cast<const R*>(V);
  a.grad_S = static_cast<const R*>(gS);
  a.grad_V = static_cast<R*>(gV);
  a.nblk_max = as.nblk;
  a.seg_len = adj_seg_len(b->t_max);
  a.part = static_cast<R*>(scratch);
  a.valid = adjoint_valid(as, scratch);
  a.ck = static_cast<unsigned char*>(scratch) + as.ck_off;
  a.obs_pad = nullptr;
  smppi_status st;
  if (t->obs_max > 0 && sizeof(R) == sizeof(float)) {
    // FP32 obstacles per wave, from padded slots (as the rollout)
    float4* pad = reinterpret_cast<float4*>(static_cast<unsigned char*>(scratch) + as.pad_off);
    hipLaunchKernelGGL(k_pad_obs, dim3(b->n_problems), dim3(64), 0, s, a.p.obs_off,
                       reinterpret_cast<const float*>(a.p.obs), a.p.obs_max, kMaxObs, (float)a.C.alpha, pad);
    if ((st = check_launch(ctx, "k_pad_obs"))) return st;
    a.obs_pad = pad;
  }
  st = t->obs_max > 0 ? launch_backward<R, kMaxObs>(ctx, b, a, s) : launch_backward<R, 0>(ctx, b, a, s);
  if (st) return st;
  return launch_sum_partials<R>(ctx, b, as, scratch, tickets, gV, s);
}

template <class R>
static smppi_status backward_t(smppi_ctx ctx, const smppi_batch* b, const smppi_model* m, const smppi_cost* c,
                               const smppi_noise* n, const smppi_track* t, const void* x0, const void* V,
                               const uint32_t* iter, const void* gS, const smppi_objective* ob, void* gV,
                               hipStream_t s) {
  smppi_status st;
  const AdjScratch as = adjoint_scratch(b);
  if ((st = need_scratch(ctx, as.pad_off + as.pad_bytes, (int)as.tickets, "smppi_rollout_backward")))
    return st;
  return backward_launch<R>(ctx, b, m, c, n, t, x0, V, iter, gS, ob, gV, ctx->scratch, ctx->tickets, s);
}

smppi_status smppi::validate_objective(smppi_ctx ctx, const smppi_objective* o) {
  if (!o) return fail(ctx, SMPPI_ERR_INVALID_ARGUMENT, "objective is NULL");
  if (!std::isfinite(o->w_S) || !std::isfinite(o->w_sq) || !std::isfinite(o->w_lin))
    return fail(ctx, SMPPI_ERR_INVALID_ARGUMENT, "objective weights must be finite");
  return SMPPI_OK;
}

static smppi_status validate_backward(smppi_ctx ctx, const smppi_batch* batch, const smppi_model* model,
                                      const smppi_cost* cost, const smppi_noise* noise, const smppi_track* track,
                                      const void* x0, const void* V, const uint32_t* iter, const void* grad_S,
                                      const smppi_objective* objective, const void* grad_V) {
  smppi_status st;
  if ((st = validate_batch(ctx, batch)) || (st = validate_model(ctx, model)) || (st = validate_cost(ctx, cost)) ||
      (st = validate_track(ctx, track, batch->dtype, batch->t_max)) || (st = validate_objective(ctx, objective)))
    return st;
  if (!noise) return fail(ctx, SMPPI_ERR_INVALID_ARGUMENT, "noise is NULL");
  if (!x0 || !V || !iter || !grad_S || !grad_V)
    return fail(ctx, SMPPI_ERR_INVALID_ARGUMENT, "x0, V, iter, grad_S, grad_V are required");
  return SMPPI_OK;
}

extern "C" smppi_status smppi_rollout_backward(smppi_ctx ctx, const smppi_batch* batch, const smppi_model* model,
                                               const smppi_cost* cost, const smppi_noise* noise,
                                               const smppi_track* track, const void* x0, const void* V,
                                               const uint32_t* iter, const void* grad_S,
                                               const smppi_objective* objective, void* grad_V, void* stream) {
  if (!ctx) return SMPPI_ERR_INVALID_ARGUMENT;
  smppi_status st;
  if ((st = validate_backward(ctx, batch, model, cost, noise, track, x0, V, iter, grad_S, objective, grad_V)))
    return st;
  (void)hipSetDevice(ctx->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (batch->dtype == SMPPI_F32)
    return backward_t<float>(ctx, batch, model, cost, noise, track, x0, V, iter, grad_S, objective, grad_V, s);
  return backward_t<double>(ctx, batch, model, cost, noise, track, x0, V, iter, grad_S, objective, grad_V, s);
}

// ------------------------------------------------------------------ adjoint without allocation
// For callers that cannot allocate device memory: the adjoint's ticket
// counters and per-workgroup partials live in one fixed file-scope device
// array.  Each GPU the library runs on holds its own copy until the process
// ends; host code reaches it only through the address hipGetSymbolAddress
// returned for that device at smppi_create (the array's name is a host-side
// stand-in, not a device address).  Every call on a GPU shares that GPU's
// copy: calls that overlap on one GPU race.
namespace {
constexpr size_t kNoAllocTicketBytes = 16384;  // 4096 problems
constexpr size_t kNoAllocBytes = (64u << 20) + kNoAllocTicketBytes;
constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mu;
void* g_noalloc_ptr[kMaxDevices] = {};
}  // namespace

static __device__ __align__(256) unsigned char noalloc_scratch[kNoAllocBytes];

namespace smppi {
__global__ void k_zero_u32(uint32_t* __restrict__ p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}
}  // namespace smppi

// The array's device address on ctx->device (that device current): looked up
// once per device, kept for the life of the process.
static smppi_status noalloc_setup(smppi_ctx ctx) {
  ctx->noalloc = nullptr;
  if (ctx->device >= kMaxDevices) return SMPPI_OK;  // the entry point then reports UNSUPPORTED
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  if (!g_noalloc_ptr[ctx->device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(noalloc_scratch));
    if (e != hipSuccess || !p) return hip_fail(ctx, e, "hipGetSymbolAddress(noalloc_scratch)");
    g_noalloc_ptr[ctx->device] = p;
  }
  ctx->noalloc = g_noalloc_ptr[ctx->device];
  return SMPPI_OK;
}

extern "C" smppi_status smppi_rollout_backward_noalloc(smppi_ctx ctx, const smppi_batch* batch,
                                                       const smppi_model* model, const smppi_cost* cost,
                                                       const smppi_noise* noise, const smppi_track* track,
                                                       const void* x0, const void* V, const uint32_t* iter,
                                                       const void* grad_S, const smppi_objective* objective,
                                                       void* grad_V, void* stream) {
  if (!ctx) return SMPPI_ERR_INVALID_ARGUMENT;
  smppi_status st;
  if ((st = validate_backward(ctx, batch, model, cost, noise, track, x0, V, iter, grad_S, objective, grad_V)))
    return st;
  if (!ctx->noalloc) return fail(ctx, SMPPI_ERR_UNSUPPORTED, "no fixed scratch on device %d", ctx->device);
  const AdjScratch as = adjoint_scratch(batch);
  const size_t part = as.pad_off + as.pad_bytes;
  if (as.tickets * sizeof(uint32_t) > kNoAllocTicketBytes || part > kNoAllocBytes - kNoAllocTicketBytes)
    return fail(ctx, SMPPI_ERR_SHAPE,
                "smppi_rollout_backward_noalloc: the batch needs %zu ticket counters (B x ceil(2 t_max / 64); "
                "max %zu) and %zu B of partials, slice sums and checkpoints (about dtype bytes x B x n x "
                "(2 t_max + 9 t_max / seg) + 4 B, n = ceil(k_max / 64), seg = ceil(sqrt(t_max)); max %zu)",
                as.tickets, kNoAllocTicketBytes / sizeof(uint32_t), part, kNoAllocBytes - kNoAllocTicketBytes);
  (void)hipSetDevice(ctx->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  unsigned char* base = static_cast<unsigned char*>(ctx->noalloc);
  uint32_t* tickets = reinterpret_cast<uint32_t*>(base);
  // the counters must start at zero: cleared by a kernel (capturable; no memset node)
  const int nt = (int)as.tickets;
  hipLaunchKernelGGL(k_zero_u32, dim3((nt + 255) / 256), dim3(256), 0, s, tickets, nt);
  if ((st = check_launch(ctx, "k_zero_u32"))) return st;
  void* pp = base + kNoAllocTicketBytes;
  if (batch->dtype == SMPPI_F32)
    return backward_launch<float>(ctx, batch, model, cost, noise, track, x0, V, iter, grad_S, objective, grad_V, pp,
                                  tickets, s);
  return backward_launch<double>(ctx, batch, model, cost, noise, track, x0, V, iter, grad_S, objective, grad_V, pp,
                                 tickets, s);
}

// ------------------------------------------------------------------ repair
template <class R, int NOBS>
static smppi_status launch_repair(smppi_ctx ctx, const smppi_batch* b, const RepairArgs<R>& a, hipStream_t s,
                                  hipEvent_t e0, hipEvent_t e1) {
  const size_t lds = stage_lds_bytes<R>(a.p.poly_max, a.p.t_max, a.p.obs_max) +
                     repair_lds_bytes<R>(a.p.t_max, a.memory, a.par_rev != 0, true);
  if (lds > (size_t)ctx->max_lds)
    return fail(ctx, SMPPI_ERR_SHAPE, "repair needs %zu B of LDS per workgroup (device max %d)", lds, ctx->max_lds);
  // the wider workgroup only for Algorithm 1 with at most one problem per
  // compute unit (L-BFGS's many workgroup dot products, and two workgroups per
  // compute unit, measured slower with it)
  const int nt = (a.method == 0 && b->n_problems <= ctx->n_cu) ? rep_blk<R, NOBS>() : REP_BLK;
  if (e0 && e1)  // events stamped with the kernel's own start and end
    hipExtLaunchKernelGGL((k_repair<R, NOBS>), dim3(b->n_problems), dim3(nt), (uint32_t)lds, s, e0, e1, 0u, a);
  else
    hipLaunchKernelGGL((k_repair<R, NOBS>), dim3(b->n_problems), dim3(nt), lds, s, a);
  return check_launch(ctx, "k_repair");
}

template <class R>
RepairArgs<R> smppi::repair_args(smppi_ctx ctx, const smppi_batch* b, const smppi_model* m, const smppi_cost* c,
                                 const smppi_track* t, const void* x0, const void* Vp, const smppi_repair_opts* o,
                                 void* Vs, const ExecFuse* ex) {
  RepairArgs<R> a;
  a.p = problem_args<R>(ctx, b, t, nullptr, x0, nullptr);
  a.M = dev_model<R>(m);
  a.C = dev_cost<R>(c);
  a.ob = dev_objective<R>(&o->objective);
  a.V_plus = static_cast<const R*>(Vp);
  a.V_safe = static_cast<R*>(Vs);
  a.n_steps = o->n_steps;
  a.step = (R)o->step;
  a.seg_len = adj_seg_len(b->t_max);
  a.method = o->method;
  a.memory = o->method == 1 ? o->memory : 0;
  // the parallel reverse sweep when its per-step Jacobians fit in LDS
  a.par_rev = stage_lds_bytes<R>(a.p.poly_max, a.p.t_max, a.p.obs_max) +
                      repair_lds_bytes<R>(a.p.t_max, a.memory, true, true) <=
                  (size_t)ctx->max_lds;
  a.exec = ex != nullptr;
  a.ex = ExecuteArgs<R>{};
  if (ex) {
    a.ex.t_off = b->t_off;
    a.ex.B = b->n_problems;
    a.ex.t_max = b->t_max;
    a.ex.M = a.M;
    a.ex.V_exec = static_cast<const R*>(Vs);
    a.ex.V_plus = static_cast<const R*>(Vp);
    a.ex.dist = static_cast<const R*>(ex->dist);
    a.ex.n_dist = ex->n_dist;
    a.ex.x = static_cast<R*>(ex->x);
    a.ex.V = static_cast<R*>(ex->V);
    a.ex.iter = ex->iter;
    a.ex.err = ctx->err;
  }
  return a;
}
template RepairArgs<float> smppi::repair_args<float>(smppi_ctx, const smppi_batch*, const smppi_model*,
                                                     const smppi_cost*, const smppi_track*, const void*, const void*,
                                                     const smppi_repair_opts*, void*, const ExecFuse*);

template <class R>
smppi_status smppi::repair_t(smppi_ctx ctx, const smppi_batch* b, const smppi_model* m, const smppi_cost* c,
                             const smppi_track* t, const void* x0, const void* Vp, const smppi_repair_opts* o,
                             void* Vs, hipStream_t s, hipEvent_t e0, hipEvent_t e1, const ExecFuse* ex) {
  const RepairArgs<R> a = repair_args<R>(ctx, b, m, c, t, x0, Vp, o, Vs, ex);
  if (t->obs_max > 0) return launch_repair<R, kMaxObs>(ctx, b, a, s, e0, e1);
  return launch_repair<R, 0>(ctx, b, a, s, e0, e1);
}
template smppi_status smppi::repair_t<float>(smppi_ctx, const smppi_batch*, const smppi_model*, const smppi_cost*,
                                             const smppi_track*, const void*, const void*, const smppi_repair_opts*,
                                             void*, hipStream_t, hipEvent_t, hipEvent_t, const ExecFuse*);

smppi_status smppi::validate_repair(smppi_ctx ctx, const smppi_repair_opts* o) {
  if (!o) return fail(ctx, SMPPI_ERR_INVALID_ARGUMENT, "repair opts are NULL");
  if (o->n_steps < 0 || o->n_steps > 100000) return fail(ctx, SMPPI_ERR_INVALID_ARGUMENT, "n_steps out of range");
  if (!std::isfinite(o->step)) return fail(ctx, SMPPI_ERR_INVALID_ARGUMENT, "step must be finite");
  if (o->method != 0 && o->method != 1) return fail(ctx, SMPPI_ERR_INVALID_ARGUMENT, "method must be 0 or 1");
  if (o->method == 1 && (o->memory < 1 || o->memory > kMaxMemory))
    return fail(ctx, SMPPI_ERR_INVALID_ARGUMENT, "memory must be in [1, %d]", kMaxMemory);
  return validate_objective(ctx, &o->objective);
}

extern "C" smppi_status smppi_shield_repair(smppi_ctx ctx, const smppi_batch* batch, const smppi_model* model,
                                            const smppi_cost* cost, const smppi_track* track, const void* x0,
                                            const void* V_plus, const smppi_repair_opts* opts, void* V_safe,
                                            void* stream) {
  if (!ctx) return SMPPI_ERR_INVALID_ARGUMENT;
  smppi_status st;
  if ((st = validate_batch(ctx, batch)) || (st = validate_model(ctx, model)) || (st = validate_cost(ctx, cost)) ||
      (st = validate_track(ctx, track, batch->dtype, batch->t_max)) || (st = validate_repair(ctx, opts)))
    return st;
  if (!x0 || !V_plus || !V_safe) return fail(ctx, SMPPI_ERR_INVALID_ARGUMENT, "x0, V_plus, V_safe are required");
  (void)hipSetDevice(ctx->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (batch->dtype == SMPPI_F32) return repair_t<float>(ctx, batch, model, cost, track, x0, V_plus, opts, V_safe, s);
  return repair_t<double>(ctx, batch, model, cost, track, x0, V_plus, opts, V_safe, s);
}

// ------------------------------------------------------------------ execute
template <class R>
smppi_status smppi::execute_t(smppi_ctx ctx, const smppi_batch* b, const smppi_model* m, const void* Ve,
                              const void* Vp, const void* dist, int32_t n_dist, void* x, void* V, uint32_t* iter,
                              hipStream_t s) {
  ExecuteArgs<R> a;
  a.t_off = b->t_off;
  a.B = b->n_problems;
  a.t_max = b->t_max;
  a.M = dev_model<R>(m);
  a.V_exec = static_cast<const R*>(Ve);
  a.V_plus = static_cast<const R*>(Vp);
  a.dist = static_cast<const R*>(dist);
  a.n_dist = n_dist;
  a.x = static_cast<R*>(x);
  a.V = static_cast<R*>(V);
  a.iter = iter;
  a.err = ctx->err;
  hipLaunchKernelGGL((k_execute<R>), dim3(b->n_problems), dim3(WAVE), sizeof(R) * 2 * b->t_max, s, a);
  return check_launch(ctx, "k_execute");
}
template smppi_status smppi::execute_t<float>(smppi_ctx, const smppi_batch*, const smppi_model*, const void*,
                                              const void*, const void*, int32_t, void*, void*, uint32_t*, hipStream_t);

extern "C" smppi_status smppi_execute(smppi_ctx ctx, const smppi_batch* batch, const smppi_model* model,
                                      const void* V_exec, const void* V_plus, const void* dist, int32_t n_dist,
                                      void* x, void* V, uint32_t* iter, void* stream) {
  if (!ctx) return SMPPI_ERR_INVALID_ARGUMENT;
  smppi_status st;
  if ((st = validate_batch(ctx, batch)) || (st = validate_model(ctx, model))) return st;
  if (!V_exec || !V_plus || !x || !V || !iter)
    return fail(ctx, SMPPI_ERR_INVALID_ARGUMENT, "V_exec, V_plus, x, V, iter are required");
  if (dist && n_dist < 0) return fail(ctx, SMPPI_ERR_INVALID_ARGUMENT, "n_dist must be >= 0");
  (void)hipSetDevice(ctx->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (batch->dtype == SMPPI_F32)
    return execute_t<float>(ctx, batch, model, V_exec, V_plus, dist, n_dist, x, V, iter, s);
  return execute_t<double>(ctx, batch, model, V_exec, V_plus, dist, n_dist, x, V, iter, s);
}

// ------------------------------------------------------------------ debug
namespace smppi {
// ============================================================== debug: generator
__global__ void k_debug_philox(const uint32_t* __restrict__ ctr, uint32_t k0, uint32_t k1, int64_t n,
                               uint32_t* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint32_t c0 = ctr[4 * i], c1 = ctr[4 * i + 1], c2 = ctr[4 * i + 2], c3 = ctr[4 * i + 3];
  philox4x32_10(c0, c1, c2, c3, k0, k1);
  out[4 * i] = c0;
  out[4 * i + 1] = c1;
  out[4 * i + 2] = c2;
  out[4 * i + 3] = c3;
}

}  // namespace smppi

extern "C" smppi_status smppi_debug_philox(smppi_ctx ctx, const uint32_t* ctr, const uint32_t* key_host, int64_t n,
                                           uint32_t* out, void* stream) {
  if (!ctx) return SMPPI_ERR_INVALID_ARGUMENT;
  if (!ctr || !key_host || !out || n < 0) return fail(ctx, SMPPI_ERR_INVALID_ARGUMENT, "bad debug_philox arguments");
  if (n == 0) return SMPPI_OK;
  (void)hipSetDevice(ctx->device);
  const int blk = 256;
  const int64_t g = (n + blk - 1) / blk;
  if (g > 0x7fffffff) return fail(ctx, SMPPI_ERR_SHAPE, "n too large");
  hipLaunchKernelGGL(k_debug_philox, dim3((unsigned)g), dim3(blk), 0, static_cast<hipStream_t>(stream), ctr,
                     key_host[0], key_host[1], n, out);
  return check_launch(ctx, "k_debug_philox");
}
