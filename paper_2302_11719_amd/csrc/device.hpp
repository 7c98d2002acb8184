// Device building blocks of the Shield-MPPI sampled-rollout step for gfx950.
//
// Everything here runs per lane with the state in registers: the counter-based
// noise generator, the vehicle model and its RK4 step, the track/obstacle
// barriers, the trajectory cost of Algorithm 2 (eqs. (8), (12), (17)-(20),
// (23)-(25)) and the reverse (adjoint) sweep that differentiates it.
// Templates take the arithmetic type R (float or double) and NOBS, the
// compile-time bound on obstacles per problem (0 or 64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace smppi {

constexpr int WAVE = 64;

// ---------------------------------------------------------------- parameters
template <class R>
struct DevModel {
  R lf, lr, Cf, Cr, a_max, c_v, v_min, dt, inv_m, lr_Iz, lf_Iz;
  R u_lo[2], u_hi[2];
};

template <class R>
struct DevCost {
  R v_g, q_v, q_ey, C_obs, phi_w;
  R ctrl_w[2];  // lambda_u / sigma_d^2
  R sigma[2];
  R C_cbf, alpha;
};

template <class R>
struct DevObjective {
  R w_S, w_sq, w_lin;
  int n_lin;
};

// ---------------------------------------------------------------- math shims
// FP32 uses the hardware transcendental units directly: v_sin/v_cos take their
// argument in revolutions, so an angle is first scaled by 1/(2 pi) and reduced
// to [0, 1) with v_fract (exact), v_rcp/v_sqrt/v_log are the single-instruction
// approximations (about 1 ulp).  FP64 uses the correctly rounded library calls.
__device__ __forceinline__ void sincos_r(float x, float* s, float* c) {
  const float r = __builtin_amdgcn_fractf(x * 0.15915494309189535f);
  *s = __builtin_amdgcn_sinf(r);
  *c = __builtin_amdgcn_cosf(r);
}
__device__ __forceinline__ void sincos_r(double x, double* s, double* c) { sincos(x, s, c); }
__device__ __forceinline__ float rcp_r(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp_r(double x) { return 1.0 / x; }
__device__ __forceinline__ float sqrt_r(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double sqrt_r(double x) { return sqrt(x); }
__device__ __forceinline__ float exp_r(float x) { return __builtin_amdgcn_exp2f(x * 1.4426950408889634f); }
__device__ __forceinline__ double exp_r(double x) { return exp(x); }
template <class R> __device__ __forceinline__ R clamp_r(R x, R lo, R hi) { return fmin(fmax(x, lo), hi); }
// Fused multiply-add written out: the model's arithmetic below pairs every
// product with its sum explicitly, so the compiler has no contraction choices
// left and every kernel that integrates the model rounds it the same way.
__device__ __forceinline__ float fma_r(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_r(double a, double b, double c) { return __builtin_fma(a, b, c); }
// single v_med3_f32 (lo <= hi)
template <> __device__ __forceinline__ float clamp_r<float>(float x, float lo, float hi) {
  return __builtin_amdgcn_fmed3f(x, lo, hi);
}

// ---------------------------------------------------------------- noise
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 32x32 -> 64-bit products with a Weyl-sequence key schedule.
__device__ __forceinline__ void philox4x32_10(uint32_t& c0, uint32_t& c1, uint32_t& c2, uint32_t& c3,
                                              uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    // one 32x32 -> 64-bit product per multiplier (v_mad_u64_u32)
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
    const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
    const uint32_t n0 = hi1 ^ c1 ^ k0;
    const uint32_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

// Uniform in (0, 1] from the top 24 bits (exact in FP32), then Box-Muller.
__device__ __forceinline__ void box_muller(uint32_t a, uint32_t b, float& z0, float& z1) {
  const float ua = (float)((a >> 8) + 1u) * 0x1p-24f;
  const float ub = (float)((b >> 8) + 1u) * 0x1p-24f;
  // -2 ln u = -2 ln 2 * log2 u; v_sin/v_cos of ub in revolutions give sin/cos(2 pi ub)
  const float r = __builtin_amdgcn_sqrtf(-1.3862943611198906f * __builtin_amdgcn_logf(ua));
  z0 = r * __builtin_amdgcn_cosf(ub);
  z1 = r * __builtin_amdgcn_sinf(ub);
}
__device__ __forceinline__ void box_muller(uint32_t a, uint32_t b, double& z0, double& z1) {
  const double ua = (double)((a >> 8) + 1u) * 0x1p-24;
  const double ub = (double)((b >> 8) + 1u) * 0x1p-24;
  const double r = sqrt(-2.0 * log(ua));
  double s, c;
  sincospi(2.0 * ub, &s, &c);
  z0 = r * c;
  z1 = r * s;
}

// Four standard normals for steps 2j and 2j+1 of sample m: counter
// (j, m, pid, it), key (seed, 0).
template <class R>
__device__ __forceinline__ void normals4(uint32_t seed, uint32_t j, uint32_t m, uint32_t pid, uint32_t it,
                                         R z[4]) {
  uint32_t c0 = j, c1 = m, c2 = pid, c3 = it;
  philox4x32_10(c0, c1, c2, c3, seed, 0u);
  box_muller(c0, c1, z[0], z[1]);
  box_muller(c2, c3, z[2], z[3]);
}

// Per-step noise of one sample: one Philox call covers the pair of steps
// (2j, 2j+1).  gen(t) regenerates the pair containing t; get(t) reads it.
template <class R>
struct NoiseStream {
  uint32_t seed, m, pid, it;
  bool nominal;
  R z[4];
  __device__ __forceinline__ void gen(int t) {
    if (!nominal) normals4<R>(seed, (uint32_t)(t >> 1), m, pid, it, z);
  }
  __device__ __forceinline__ void get(int t, R sig0, R sig1, R& e0, R& e1) const {
    if (nominal) {
      e0 = R(0);
      e1 = R(0);
      return;
    }
    // selects rather than a computed index keep z in registers
    const bool odd = (t & 1) != 0;
    e0 = sig0 * (odd ? z[2] : z[0]);
    e1 = sig1 * (odd ? z[3] : z[1]);
  }
  // Sequential access (t = 0, 1, 2, ...): regenerates on even steps.
  __device__ __forceinline__ void at(int t, R sig0, R sig1, R& e0, R& e1) {
    if ((t & 1) == 0) gen(t);
    get(t, sig0, sig1, e0, e1);
  }
};

// ---------------------------------------------------------------- dynamics
// Per-step constants of the held control (steer delta, throttle tau).
template <class R>
struct StepCtl {
  R delta, sd_m, cd_m, lfcd_Iz, a_tau, sd, cd;
};

template <class R>
__device__ __forceinline__ StepCtl<R> step_ctl(const DevModel<R>& M, R delta, R tau) {
  StepCtl<R> c;
  R sd, cd;
  sincos_r(delta, &sd, &cd);
  c.delta = delta;
  c.sd = sd;
  c.cd = cd;
  c.sd_m = sd * M.inv_m;
  c.cd_m = cd * M.inv_m;
  c.lfcd_Iz = cd * M.lf_Iz;
  c.a_tau = M.a_max * tau;
  return c;
}

// f of the six-state single-track model.  The velocities (v_x, v_y, omega)
// evolve on their own (body-frame forces depend on neither position nor
// heading); (p_x, p_y, psi) integrate them.  The two parts are separate
// functions so that a step can be split across waves with the same arithmetic.
template <class R>
__device__ __forceinline__ void vel_deriv(const DevModel<R>& M, const StepCtl<R>& c, R vx, R vy, R om, R& dvx,
                                          R& dvy, R& dom) {
  const R vt = fmax(vx, M.v_min);
  const R inv = rcp_r(vt);
  const R Ff = M.Cf * fma_r(-fma_r(M.lf, om, vy), inv, c.delta);  // C_f (delta - (v_y + l_f om) / v)
  const R Fr = M.Cr * (fma_r(M.lr, om, -vy) * inv);               // C_r (l_r om - v_y) / v
  dvx = fma_r(vy, om, fma_r(-Ff, c.sd_m, fma_r(-M.c_v, vx, c.a_tau)));
  dvy = fma_r(-vx, om, fma_r(Ff, c.cd_m, Fr * M.inv_m));
  dom = fma_r(Ff, c.lfcd_Iz, -(Fr * M.lr_Iz));
}

template <class R>
__device__ __forceinline__ void pose_deriv(R psi, R vx, R vy, R& dpx, R& dpy) {
  R sp, cp;
  sincos_r(psi, &sp, &cp);
  dpx = fma_r(vx, cp, -(vy * sp));
  dpy = fma_r(vx, sp, vy * cp);
}

template <class R>
__device__ __forceinline__ void deriv(const DevModel<R>& M, const StepCtl<R>& c, R psi, R vx, R vy, R om,
                                      R& dpx, R& dpy, R& dvx, R& dvy, R& dom) {
  vel_deriv(M, c, vx, vy, om, dvx, dvy, dom);
  pose_deriv(psi, vx, vy, dpx, dpy);
}

template <class R>
struct State {
  R px, py, psi, vx, vy, om;
};

// Velocities at the four RK4 stages of one step (stage 1 = the step's start).
template <class R>
struct VelStages {
  R vx[4], vy[4], om[4];
};

// Velocity part of a classic RK4 step over dt with the control held: advances
// (v_x, v_y, omega) and returns the stage velocities the pose part needs.
template <class R>
__device__ __forceinline__ void rk4_vel(const DevModel<R>& M, const StepCtl<R>& c, R& vx, R& vy, R& om,
                                        VelStages<R>& g) {
  const R h = M.dt, h2 = R(0.5) * M.dt, h6 = M.dt * R(1.0 / 6.0);
  R a3, a4, a5, b3, b4, b5, c3, c4, c5, d3, d4, d5;
  g.vx[0] = vx;
  g.vy[0] = vy;
  g.om[0] = om;
  vel_deriv(M, c, vx, vy, om, a3, a4, a5);
  g.vx[1] = fma_r(h2, a3, vx);
  g.vy[1] = fma_r(h2, a4, vy);
  g.om[1] = fma_r(h2, a5, om);
  vel_deriv(M, c, g.vx[1], g.vy[1], g.om[1], b3, b4, b5);
  g.vx[2] = fma_r(h2, b3, vx);
  g.vy[2] = fma_r(h2, b4, vy);
  g.om[2] = fma_r(h2, b5, om);
  vel_deriv(M, c, g.vx[2], g.vy[2], g.om[2], c3, c4, c5);
  g.vx[3] = fma_r(h, c3, vx);
  g.vy[3] = fma_r(h, c4, vy);
  g.om[3] = fma_r(h, c5, om);
  vel_deriv(M, c, g.vx[3], g.vy[3], g.om[3], d3, d4, d5);
  vx = fma_r(h6, fma_r(R(2), b3 + c3, a3) + d3, vx);
  vy = fma_r(h6, fma_r(R(2), b4 + c4, a4) + d4, vy);
  om = fma_r(h6, fma_r(R(2), b5 + c5, a5) + d5, om);
}

// Pose part of the same step from the stage velocities.
template <class R>
__device__ __forceinline__ void rk4_pose(const DevModel<R>& M, const VelStages<R>& g, R& px, R& py, R& psi) {
  const R h = M.dt, h2 = R(0.5) * M.dt, h6 = M.dt * R(1.0 / 6.0);
  R a0, a1, b0, b1, c0, c1, d0, d1;
  pose_deriv(psi, g.vx[0], g.vy[0], a0, a1);
  pose_deriv(fma_r(h2, g.om[0], psi), g.vx[1], g.vy[1], b0, b1);
  pose_deriv(fma_r(h2, g.om[1], psi), g.vx[2], g.vy[2], c0, c1);
  pose_deriv(fma_r(h, g.om[2], psi), g.vx[3], g.vy[3], d0, d1);
  px = fma_r(h6, fma_r(R(2), b0 + c0, a0) + d0, px);
  py = fma_r(h6, fma_r(R(2), b1 + c1, a1) + d1, py);
  psi = fma_r(h6, fma_r(R(2), g.om[1] + g.om[2], g.om[0]) + g.om[3], psi);
}

// Classic RK4 over dt with the control held.
template <class R>
__device__ __forceinline__ void rk4(const DevModel<R>& M, const StepCtl<R>& c, State<R>& x) {
  VelStages<R> g;
  rk4_vel(M, c, x.vx, x.vy, x.om, g);
  rk4_pose(M, g, x.px, x.py, x.psi);
}

// ---------------------------------------------------------------- curvilinear model
// Track of the curvilinear model: the periodic curvature table kappa(j ds)
// (LDS or global), its length, spacing and the half width squared.
template <class R>
struct CurvView {
  const R* kappa;
  int n;
  R ds, w2;
  R inv_ds, rn, inv_n;  // 1/ds, n and 1/n (the cell lookup multiplies instead of dividing)
};

template <class R>
__device__ __forceinline__ CurvView<R> curv_view(const R* kappa, int n, R ds, R w2) {
  CurvView<R> cv;
  cv.kappa = kappa;
  cv.n = n;
  cv.ds = ds;
  cv.w2 = w2;
  cv.inv_ds = R(1) / ds;
  cv.rn = R(n);
  cv.inv_n = R(1) / R(n);
  return cv;
}

// ---------------------------------------------------------------- track
// Polyline segments are staged in LDS as (a_x, a_y, d_x, d_y) plus 1/|d|^2.
template <class R> struct Vec4 { R x, y, z, w; };
template <> struct Vec4<float> { float4 v; };

// Wrapped copies kept on each side of the staged polyline (bounds the window
// half width of the unwrapped search).
constexpr int SEG_PAD = 8;

template <class R>
struct TrackView {
  int n;                  // polyline segments (0: circle)
  int window;
  const R* seg;           // LDS [n][4], valid for indices -SEG_PAD .. n+SEG_PAD-1
  const R* il2;           // LDS [n], same index range
  R cx, cy, rad;          // circle
  R w2;                   // half width squared
  const R* obs;           // LDS [obstacle slots][4]
  int n_obs;
  int idx0;               // nearest segment to the problem's start state
};

// One circular obstacle: centre, inflated radius squared (barrier), radius
// squared (collision indicator).  LDS slots are 16-byte aligned for FP32.
template <class R> struct Obs { R cx, cy, re2, r2; };
template <class R>
__device__ __forceinline__ Obs<R> obs_at(const TrackView<R>& tr, int i) {
  return Obs<R>{tr.obs[4 * i], tr.obs[4 * i + 1], tr.obs[4 * i + 2], tr.obs[4 * i + 3]};
}
template <>
__device__ __forceinline__ Obs<float> obs_at<float>(const TrackView<float>& tr, int i) {
  const float4 v = reinterpret_cast<const float4*>(tr.obs)[i];
  return Obs<float>{v.x, v.y, v.z, v.w};
}

// Squared distance from (px, py) to the segment a + lam d, lam in [0, 1]
// (il2 = 1/|d|^2); the error vector in (*rx_o, *ry_o) when requested.
template <class R>
__device__ __forceinline__ R seg_dist2_row(R ax, R ay, R dx, R dy, R il2, R px, R py, R* rx_o = nullptr,
                                           R* ry_o = nullptr) {
  const R rx = px - ax, ry = py - ay;
  R lam = (rx * dx + ry * dy) * il2;
  lam = clamp_r(lam, R(0), R(1));
  const R ex = rx - lam * dx, ey = ry - lam * dy;
  if (rx_o) {
    *rx_o = ex;
    *ry_o = ey;
  }
  return ex * ex + ey * ey;
}
template <class R>
__device__ __forceinline__ R seg_dist2(const TrackView<R>& tr, int i, R px, R py, R* rx_o = nullptr,
                                       R* ry_o = nullptr) {
  return seg_dist2_row(tr.seg[4 * i + 0], tr.seg[4 * i + 1], tr.seg[4 * i + 2], tr.seg[4 * i + 3], tr.il2[i], px,
                       py, rx_o, ry_o);
}

// Global nearest segment (first strict minimum: lowest index on ties).
template <class R>
__device__ int global_argmin(const TrackView<R>& tr, R px, R py) {
  int best = 0;
  R bd = seg_dist2(tr, 0, px, py);
  for (int i = 1; i < tr.n; ++i) {
    const R d = seg_dist2(tr, i, px, py);
    if (d < bd) {
      bd = d;
      best = i;
    }
  }
  return best;
}

// Window rule around `c`: offsets 0, -1, +1, -2, +2, ... (first strict minimum wins).
template <class R>
__device__ __forceinline__ R window_min(const TrackView<R>& tr, int& c, R px, R py) {
  int best = c;
  R bd = seg_dist2(tr, c, px, py);
  for (int k = 1; k <= tr.window; ++k) {
    int i = c - k;
    if (i < 0) i += tr.n;
    int j = c + k;
    if (j >= tr.n) j -= tr.n;
    const R di = seg_dist2(tr, i, px, py);
    if (di < bd) {
      bd = di;
      best = i;
    }
    const R dj = seg_dist2(tr, j, px, py);
    if (dj < bd) {
      bd = dj;
      best = j;
    }
  }
  c = best;
  return bd;
}

// The same rule with the half width fixed at compile time: all 2W+1 segments
// are read from LDS first (one latency for the whole window), then compared
// in the rule's order.
template <int W, class R>
__device__ __forceinline__ R window_min_fixed(const TrackView<R>& tr, int& c, R px, R py) {
  static_assert(W <= SEG_PAD, "window wider than the staged wrap-around");
  constexpr int NS = 2 * W + 1;
  // slots c-W .. c+W are consecutive in the padded copy: one base address,
  // immediate offsets, no index wrapping
  const R* sg = tr.seg + 4 * (c - W);
  const R* il = tr.il2 + (c - W);
  R d2[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const R rx = px - sg[4 * s + 0], ry = py - sg[4 * s + 1];
    const R dx = sg[4 * s + 2], dy = sg[4 * s + 3];
    const R lam = clamp_r((rx * dx + ry * dy) * il[s], R(0), R(1));
    const R ex = rx - lam * dx, ey = ry - lam * dy;
    d2[s] = ex * ex + ey * ey;
  }
  // the rule's order: offsets 0, -1, +1, -2, +2, ...; first strict minimum wins
  R bd = d2[W];
  int off = 0;
#pragma unroll
  for (int k = 1; k <= W; ++k) {
    if (d2[W - k] < bd) {
      bd = d2[W - k];
      off = -k;
    }
    if (d2[W + k] < bd) {
      bd = d2[W + k];
      off = k;
    }
  }
  int i = c + off;
  i += (i < 0) ? tr.n : 0;
  i -= (i >= tr.n) ? tr.n : 0;
  c = i;
  return bd;
}

// e_y^2 at (px, py); for the polyline `idx` is the window centre in/out
// (negative: global search).
template <class R>
__device__ __forceinline__ R lateral_sq(const TrackView<R>& tr, R px, R py, int& idx) {
  if (tr.n == 0) {
    const R dx = px - tr.cx, dy = py - tr.cy;
    const R e = sqrt_r(dx * dx + dy * dy) - tr.rad;
    return e * e;
  }
  if (idx < 0) idx = global_argmin(tr, px, py);
  if (tr.window == 4) return window_min_fixed<4>(tr, idx, px, py);
  return window_min(tr, idx, px, py);
}

// Gradient of e_y^2 with respect to (px, py) at a fixed segment (envelope of
// the projection) or for the circle.
template <class R>
__device__ __forceinline__ void lateral_sq_grad(const TrackView<R>& tr, R px, R py, int idx, R& gx, R& gy) {
  if (tr.n == 0) {
    const R dx = px - tr.cx, dy = py - tr.cy;
    const R rho = sqrt_r(dx * dx + dy * dy);
    const R f = R(2) * (rho - tr.rad) / rho;
    gx = f * dx;
    gy = f * dy;
    return;
  }
  R ex, ey;
  seg_dist2(tr, idx, px, py, &ex, &ey);
  gx = R(2) * ex;
  gy = R(2) * ey;
}

// ---------------------------------------------------------------- obstacles
// Circular-obstacle barriers of eqs. (17)-(20) per step: h_i = |p - c_i|^2 -
// (r_i + margin)^2, penalty sum_i max(alpha h_i(x_t) - h_i(x_{t+1}), 0), and the
// collision indicator of eq. (25) (|p - c_i| < r_i for some i).  Two sources of
// the obstacle table, same arithmetic up to rounding order:
//
// LdsObstacles: the staged table in LDS, read per lane (broadcast reads), any
// arithmetic type.  Used by the plain per-call kernels and the FP64 path.
template <class R>
struct LdsObstacles {
  const TrackView<R>* tr;
  // hob[i] = h_i at (px, py); collision of the point
  template <int NOBS>
  __device__ __forceinline__ void init(R px, R py, R /*alpha*/, R* hob, bool& outside) const {
#pragma unroll
    for (int i = 0; i < NOBS; ++i) {
      const Obs<R> o = obs_at(*tr, i);
      const R ox = px - o.cx, oy = py - o.cy;
      const R d2 = ox * ox + oy * oy;
      hob[i] = d2 - o.re2;
      outside = outside || (d2 < o.r2);
    }
  }
  // one transition to (px, py): pen += sum_i max(alpha hob_i - h_i, 0); hob_i = h_i
  template <int NOBS>
  __device__ __forceinline__ void step(R px, R py, R alpha, R* hob, R& pen, bool& outside) const {
#pragma unroll
    for (int i = 0; i < NOBS; ++i) {
      const Obs<R> o = obs_at(*tr, i);
      const R ox = px - o.cx, oy = py - o.cy;
      const R d2 = ox * ox + oy * oy;
      const R hi = d2 - o.re2;
      pen += fmax(alpha * hob[i] - hi, R(0));
      hob[i] = hi;
      outside = outside || (d2 < o.r2);
    }
  }
};

// ---------------------------------------------------------------- wave reductions
// Whole-wave reductions; every lane gets the result.
template <class R>
__device__ __forceinline__ R wave_sum(R v) {
#pragma unroll
  for (int o = WAVE / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
  return v;
}
template <class R>
__device__ __forceinline__ R wave_min(R v) {
#pragma unroll
  for (int o = WAVE / 2; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, WAVE));
  return v;
}
// FP32 (the whole wave active): within each 16-lane row, partners lane^1 and
// lane^2 (quad permutations), then the other quad of the half row and the
// other half of the row (mirrors; after the first two steps every lane of a
// quad holds the same value, so a mirror reaches the same partner value as
// lane^4 and lane^8 would); the four row results then meet as
// (row0 + row1) + (row2 + row3) through readlane.  Every lane gets the same
// value, and each kernel reduces in this one order.
template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, false));
}
__device__ __forceinline__ float lane_f(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
template <>
__device__ __forceinline__ float wave_sum<float>(float v) {
  v += dpp_f<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_f<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_f<0x141>(v);  // row_half_mirror
  v += dpp_f<0x140>(v);  // row_mirror
  return (lane_f(v, 0) + lane_f(v, 16)) + (lane_f(v, 32) + lane_f(v, 48));
}
template <>
__device__ __forceinline__ float wave_min<float>(float v) {
  v = fminf(v, dpp_f<0xB1>(v));
  v = fminf(v, dpp_f<0x4E>(v));
  v = fminf(v, dpp_f<0x141>(v));
  v = fminf(v, dpp_f<0x140>(v));
  return fminf(fminf(lane_f(v, 0), lane_f(v, 16)), fminf(lane_f(v, 32), lane_f(v, 48)));
}

// Unsigned minimum / maximum over a wave, in every lane (the whole wave active):
// four DPP row rotations, then a scalar combine of the four rows.
__device__ __forceinline__ unsigned wave_min_u32(unsigned m) {
  m = min(m, (unsigned)__builtin_amdgcn_mov_dpp((int)m, 0x128, 0xF, 0xF, false));  // row_ror:8
  m = min(m, (unsigned)__builtin_amdgcn_mov_dpp((int)m, 0x124, 0xF, 0xF, false));  // row_ror:4
  m = min(m, (unsigned)__builtin_amdgcn_mov_dpp((int)m, 0x122, 0xF, 0xF, false));  // row_ror:2
  m = min(m, (unsigned)__builtin_amdgcn_mov_dpp((int)m, 0x121, 0xF, 0xF, false));  // row_ror:1
  const unsigned r0 = (unsigned)__builtin_amdgcn_readlane((int)m, 0), r1 = (unsigned)__builtin_amdgcn_readlane((int)m, 16);
  const unsigned r2 = (unsigned)__builtin_amdgcn_readlane((int)m, 32), r3 = (unsigned)__builtin_amdgcn_readlane((int)m, 48);
  return min(min(r0, r1), min(r2, r3));
}
__device__ __forceinline__ unsigned wave_max_u32(unsigned m) {
  m = max(m, (unsigned)__builtin_amdgcn_mov_dpp((int)m, 0x128, 0xF, 0xF, false));  // row_ror:8
  m = max(m, (unsigned)__builtin_amdgcn_mov_dpp((int)m, 0x124, 0xF, 0xF, false));  // row_ror:4
  m = max(m, (unsigned)__builtin_amdgcn_mov_dpp((int)m, 0x122, 0xF, 0xF, false));  // row_ror:2
  m = max(m, (unsigned)__builtin_amdgcn_mov_dpp((int)m, 0x121, 0xF, 0xF, false));  // row_ror:1
  const unsigned r0 = (unsigned)__builtin_amdgcn_readlane((int)m, 0), r1 = (unsigned)__builtin_amdgcn_readlane((int)m, 16);
  const unsigned r2 = (unsigned)__builtin_amdgcn_readlane((int)m, 32), r3 = (unsigned)__builtin_amdgcn_readlane((int)m, 48);
  return max(max(r0, r1), max(r2, r3));
}
// Order-preserving map between FP32 values (not NaN) and unsigned keys: the sign
// bit set for non-negative values, all bits flipped for negative ones.
__device__ __forceinline__ unsigned f32_key(float f) {
  const unsigned b = __float_as_uint(f);
  return b ^ ((unsigned)((int)b >> 31) | 0x80000000u);
}
__device__ __forceinline__ float key_f32(unsigned k) { return __uint_as_float(k ^ (((k >> 31) - 1u) | 0x80000000u)); }

// WaveObstacles: the FP32 obstacle barriers of a whole wave of samples of one
// problem.  The table holds one slot per obstacle, (c_x, c_y, r^2, kappa) with
// kappa = (1 - alpha) ((r + margin)^2 - r^2), unused slots inert
// ((0, 0, -1e30, 0)); lane j keeps slot j in registers.  With g_i(p) =
// |p - c_i|^2 - r_i^2 (collision iff g_i < 0) and h_i = g_i - delta_i,
// delta_i = (r + margin)^2 - r^2, the DCBF transition term of eqs. (17)-(20) is
//   alpha h_i(x_t) - h_i(x_{t+1}) = alpha g_i(p) + kappa_i - g_i(q),
// p, q the positions at t and t+1.
//
// Most obstacles are far from every sample of a wave, and for those the term is
// exactly zero: with a = |q - c| and s = |q - p|, |p - c| <= a + s gives
//   alpha g(p) + kappa - g(q) <= F(a) = -(1 - alpha) a^2 + 2 alpha s a + alpha s^2
//                                     + (1 - alpha) r^2 + kappa,
// which decreases in a beyond alpha s / (1 - alpha).  So once per transition the
// wave takes the bounding box of its q's and its largest step s (wave
// reductions), each lane j bounds a from below for obstacle j by its distance to
// the box, and obstacle j is skipped when F at that bound, with the largest step,
// is below minus a rounding margin (then also g(q) > 0: no collision either).
// The remaining obstacles are evaluated for every lane, in index order, with the
// same FP32 operations as a full sweep, so the sums are the same bits (a skipped
// term would have added exactly zero).  The whole wave must be active.
struct WaveObstacles {
  float4 mine;  // slot of obstacle `lane` (inert beyond the table)

  __device__ __forceinline__ WaveObstacles() : mine(make_float4(0.f, 0.f, -1e30f, 0.f)) {}
  __device__ __forceinline__ WaveObstacles(const float4* slots, int n_slots) {
    const int lane = threadIdx.x % WAVE;
    mine = lane < n_slots ? slots[lane] : make_float4(0.f, 0.f, -1e30f, 0.f);
  }

  // Obstacles that may contribute to some lane's transition into a point of the
  // per-lane box [xlo, xhi] x [ylo, yhi] (order-preserving keys) by a step of at
  // most sqrt(s2) (bit i).  The wave reductions take the box of all lanes and the
  // largest step; a NaN coordinate widens the box or the step, which only keeps
  // more obstacles.
  __device__ __forceinline__ uint64_t live_box(unsigned kxlo, unsigned kxhi, unsigned kylo, unsigned kyhi, float s2l,
                                               float alpha) const {
    const float lox = key_f32(wave_min_u32(kxlo)), hix = key_f32(wave_max_u32(kxhi));
    const float loy = key_f32(wave_min_u32(kylo)), hiy = key_f32(wave_max_u32(kyhi));
    const float s2 = __uint_as_float(wave_max_u32(__float_as_uint(s2l)));
    // lower bound of the distance from obstacle `lane` to any q, upper bound of
    // any step (a relative 2^-20 and 1e-6 absolute cover the FP32 rounding and
    // the hardware square root's error)
    const float ex = fmaxf(fmaxf(lox - mine.x, mine.x - hix), 0.f);
    const float ey = fmaxf(fmaxf(loy - mine.y, mine.y - hiy), 0.f);
    const float A = __builtin_amdgcn_sqrtf(fmaf(ex, ex, ey * ey)) * (1.f - 0x1p-20f);
    const float S = __builtin_amdgcn_sqrtf(s2) * (1.f + 0x1p-20f) + 1e-6f;
    const float om = 1.f - alpha;
    const float F = fmaf(-om * A, A, fmaf(2.f * alpha * S, A, fmaf(alpha * S, S, fmaf(om, mine.z, mine.w))));
    const float AS = A + S;
    const bool skip = alpha > 0.f && om > 0.f && om * A >= alpha * S && F + fmaf(1e-4f * AS, AS, 1e-4f) <= 0.f;
    // a non-finite bound (a lane that diverged to infinity) keeps every obstacle
    return __ballot(!skip);
  }

  // Obstacles that may contribute to the transition p -> q of some lane (bit i).
  __device__ __forceinline__ uint64_t live(float ppx, float ppy, float qpx, float qpy, float alpha) const {
    const float dsx = qpx - ppx, dsy = qpy - ppy;
    const unsigned kx = f32_key(qpx), ky = f32_key(qpy);
    return live_box(kx, kx, ky, ky, fmaf(dsx, dsx, dsy * dsy), alpha);
  }

  // pen += sum_i max(alpha g_i(p) + kappa_i - g_i(q), 0); outside |= min_i g_i(q) < 0.
  __device__ __forceinline__ void step(float ppx, float ppy, float qpx, float qpy, float alpha, float& pen,
                                       bool& outside) const {
    uint64_t m = live(ppx, ppy, qpx, qpy, alpha);
    float mo = INFINITY;
    while (m) {
      const int i = (int)__builtin_ctzll(m);
      m &= m - 1;
      const float cx = lane_f(mine.x, i), cy = lane_f(mine.y, i), r2 = lane_f(mine.z, i), kap = lane_f(mine.w, i);
      const float ax = ppx - cx, ay = ppy - cy;
      const float g0 = fmaf(ax, ax, fmaf(ay, ay, -r2));
      const float bx = qpx - cx, by = qpy - cy;
      const float g1 = fmaf(bx, bx, fmaf(by, by, -r2));
      pen += fmaxf(fmaf(alpha, g0, kap) - g1, 0.f);
      mo = fminf(mo, g1);
    }
    outside = outside || (mo < 0.f);
  }

  // step for two consecutive transitions p -> q (pen0, out1) and q -> r (pen1,
  // out2) with one live set: the box of the q's and r's and the larger step bound
  // both transitions, so every obstacle either transition needs is in it; an
  // obstacle kept only for the other transition adds exactly +0 and has g > 0.
  // Each sum is taken in index order, as step takes it.
  __device__ __forceinline__ void step2(float ppx, float ppy, float qpx, float qpy, float rpx, float rpy, float alpha,
                                        float& pen0, bool& out1, float& pen1, bool& out2) const {
    const unsigned kqx = f32_key(qpx), kqy = f32_key(qpy), krx = f32_key(rpx), kry = f32_key(rpy);
    const float d0x = qpx - ppx, d0y = qpy - ppy, d1x = rpx - qpx, d1y = rpy - qpy;
    // squared steps compared as bit patterns (non-negative, so ordered; NaN wins)
    const float s2 = __uint_as_float(max(__float_as_uint(fmaf(d0x, d0x, d0y * d0y)),
                                         __float_as_uint(fmaf(d1x, d1x, d1y * d1y))));
    uint64_t m = live_box(min(kqx, krx), max(kqx, krx), min(kqy, kry), max(kqy, kry), s2, alpha);
    float mo1 = INFINITY, mo2 = INFINITY;
    while (m) {
      const int i = (int)__builtin_ctzll(m);
      m &= m - 1;
      const float cx = lane_f(mine.x, i), cy = lane_f(mine.y, i), r2 = lane_f(mine.z, i), kap = lane_f(mine.w, i);
      const float ax = ppx - cx, ay = ppy - cy;
      const float g0 = fmaf(ax, ax, fmaf(ay, ay, -r2));
      const float bx = qpx - cx, by = qpy - cy;
      const float g1 = fmaf(bx, bx, fmaf(by, by, -r2));
      pen0 += fmaxf(fmaf(alpha, g0, kap) - g1, 0.f);
      mo1 = fminf(mo1, g1);
      const float cx2 = rpx - cx, cy2 = rpy - cy;
      const float g2 = fmaf(cx2, cx2, fmaf(cy2, cy2, -r2));
      pen1 += fmaxf(fmaf(alpha, g1, kap) - g2, 0.f);
      mo2 = fminf(mo2, g2);
    }
    out1 = out1 || (mo1 < 0.f);
    out2 = out2 || (mo2 < 0.f);
  }

  // Adjoint of step: with r_i = alpha g_i(p) + kappa_i - g_i(q), where r_i > 0 its
  // cotangent is base + w_sq2 r_i (base = w_S C + w_lin [t < n_lin], w_sq2 =
  // 2 w_sq), and dr/dq = -2 (q - c), dr/dp = 2 alpha (p - c).  Adds the q part to
  // (lqx, lqy) and the p part to (lpx, lpy).
  __device__ __forceinline__ void grad(float ppx, float ppy, float qpx, float qpy, float alpha, float base,
                                       float w_sq2, float& lqx, float& lqy, float& lpx, float& lpy) const {
    uint64_t m = live(ppx, ppy, qpx, qpy, alpha);
    while (m) {
      const int i = (int)__builtin_ctzll(m);
      m &= m - 1;
      const float cx = lane_f(mine.x, i), cy = lane_f(mine.y, i), r2 = lane_f(mine.z, i), kap = lane_f(mine.w, i);
      const float ax = ppx - cx, ay = ppy - cy, bx = qpx - cx, by = qpy - cy;
      const float gp = fmaf(ax, ax, fmaf(ay, ay, -r2));
      const float gq = fmaf(bx, bx, fmaf(by, by, -r2));
      const float r = fmaf(alpha, gp, kap) - gq;
      const float k2 = r > 0.f ? 2.f * fmaf(w_sq2, r, base) : 0.f;
      lqx = fmaf(-k2, bx, lqx);
      lqy = fmaf(-k2, by, lqy);
      const float k2a = k2 * alpha;
      lpx = fmaf(k2a, ax, lpx);
      lpy = fmaf(k2a, ay, lpy);
    }
  }
};

// ---------------------------------------------------------------- one sample
// The model and cost constants are the same for every lane; a rollout keeps
// them in VGPRs (an empty asm statement hides their uniformity), which leaves
// the SGPRs to the addresses and loop state of the large fused kernels (whose
// SGPR spills otherwise cost a readlane per reload inside the step loop) and
// lifts the one-scalar-operand limit of a VALU instruction.
template <class R>
__device__ __forceinline__ void in_vgprs(R& x) {}
template <>
__device__ __forceinline__ void in_vgprs<float>(float& x) {
  asm volatile("" : "+v"(x));
}
template <class R>
__device__ __forceinline__ DevModel<R> model_in_vgprs(const DevModel<R>& M) {
  DevModel<R> v = M;
  in_vgprs(v.lf); in_vgprs(v.lr); in_vgprs(v.Cf); in_vgprs(v.Cr); in_vgprs(v.a_max); in_vgprs(v.c_v);
  in_vgprs(v.v_min); in_vgprs(v.dt); in_vgprs(v.inv_m); in_vgprs(v.lr_Iz); in_vgprs(v.lf_Iz);
  in_vgprs(v.u_lo[0]); in_vgprs(v.u_lo[1]); in_vgprs(v.u_hi[0]); in_vgprs(v.u_hi[1]);
  return v;
}
template <class R>
__device__ __forceinline__ DevCost<R> cost_in_vgprs(const DevCost<R>& C) {
  DevCost<R> v = C;
  in_vgprs(v.v_g); in_vgprs(v.q_v); in_vgprs(v.q_ey); in_vgprs(v.C_obs); in_vgprs(v.phi_w);
  in_vgprs(v.ctrl_w[0]); in_vgprs(v.ctrl_w[1]); in_vgprs(v.sigma[0]); in_vgprs(v.sigma[1]);
  in_vgprs(v.C_cbf); in_vgprs(v.alpha);
  return v;
}

// Modified trajectory cost S~ of one sample (Algorithm 2 inner loop):
//   S~ = sum_{t<T} [q(x_t) + lambda_u v_t^T Sigma^-1 u_t] + phi_w q(x_T) + sum_{t=0}^{T} C_cbf(z_t).
// V is [2][T] (steer row, throttle row), read from LDS or global.  Obstacles
// come from `os` (LdsObstacles, or WaveObstacles: FP32, the whole wave active).
template <class R, int NOBS, class OS>
__device__ R rollout_sample(const DevModel<R>& Mg, const DevCost<R>& Cg, const TrackView<R>& tr, const State<R>& x0,
                            const R* __restrict__ V, int T, NoiseStream<R>& ns, R* eps_out, const OS& os) {
  // (with obstacles: the kernels run one wave per SIMD, so the VGPRs are free;
  // without, the copies would cost occupancy)
  DevModel<R> Mv;
  DevCost<R> Cv;
  if constexpr (NOBS > 0) {
    Mv = model_in_vgprs(Mg);
    Cv = cost_in_vgprs(Cg);
  }
  const DevModel<R>& M = NOBS > 0 ? Mv : Mg;
  const DevCost<R>& C = NOBS > 0 ? Cv : Cg;
  State<R> x = x0;
  // the window around the global nearest segment of x0 returns that segment
  int idx = tr.idx0;
  R ey2 = lateral_sq(tr, x.px, x.py, idx);
  R h0 = tr.w2 - ey2;
  bool outside = h0 < R(0);
  constexpr bool WV = std::is_same<OS, WaveObstacles>::value;  // FP32 wave-level obstacles
  R hob[NOBS > 0 && !WV ? NOBS : 1];
  // z_0 = (x_0, x_0): C max((alpha - 1) h(x_0), 0) per barrier, i.e. the
  // transition penalty with both ends at x_0.
  R S = C.C_cbf * fmax((C.alpha - R(1)) * h0, R(0));
  if constexpr (NOBS > 0 && WV) {
    R pen0 = R(0);
    os.step(x.px, x.py, x.px, x.py, C.alpha, pen0, outside);
    S += C.C_cbf * pen0;
  } else if constexpr (NOBS > 0) {
    os.template init<NOBS>(x.px, x.py, C.alpha, hob, outside);
    R pen0 = R(0);
    bool dummy = false;
    os.template step<NOBS>(x.px, x.py, C.alpha, hob, pen0, dummy);
    S += C.C_cbf * pen0;
  }
  int t = 0;
  if constexpr (NOBS > 0 && WV) {
    // Steps in pairs with one obstacle live set per pair (WaveObstacles::step2):
    // the second step's dynamics run before the first transition's obstacle
    // terms; S receives the same terms in the same order as the loop below.
    for (; t + 1 < T; t += 2) {
      const R v0 = V[t], v1 = V[T + t];
      R e0, e1;
      ns.at(t, C.sigma[0], C.sigma[1], e0, e1);
      const R u0 = clamp_r(v0 + e0, M.u_lo[0], M.u_hi[0]);
      const R u1 = clamp_r(v1 + e1, M.u_lo[1], M.u_hi[1]);
      if (eps_out) {
        eps_out[2 * t] = u0 - v0;
        eps_out[2 * t + 1] = u1 - v1;
      }
      const R dv = x.vx - C.v_g;
      R q = C.q_v * dv * dv + C.q_ey * ey2;
      if (outside) q += C.C_obs;
      S += q + (C.ctrl_w[0] * v0 * u0 + C.ctrl_w[1] * v1 * u1);
      const StepCtl<R> sc = step_ctl(M, u0, u1);
      const R p0x = x.px, p0y = x.py;
      rk4(M, sc, x);
      ey2 = lateral_sq(tr, x.px, x.py, idx);
      R h1 = tr.w2 - ey2;
      R pen0 = fmax(C.alpha * h0 - h1, R(0));
      h0 = h1;
      bool out1 = h1 < R(0);
      // step t + 1; its collision constant waits for transition t's obstacles
      const R w0 = V[t + 1], w1 = V[T + t + 1];
      ns.at(t + 1, C.sigma[0], C.sigma[1], e0, e1);
      const R y0 = clamp_r(w0 + e0, M.u_lo[0], M.u_hi[0]);
      const R y1 = clamp_r(w1 + e1, M.u_lo[1], M.u_hi[1]);
      if (eps_out) {
        eps_out[2 * t + 2] = y0 - w0;
        eps_out[2 * t + 3] = y1 - w1;
      }
      const R dv1 = x.vx - C.v_g;
      R q1 = C.q_v * dv1 * dv1 + C.q_ey * ey2;
      const R ctl1 = C.ctrl_w[0] * w0 * y0 + C.ctrl_w[1] * w1 * y1;
      const StepCtl<R> sc1 = step_ctl(M, y0, y1);
      const R p1x = x.px, p1y = x.py;
      rk4(M, sc1, x);
      ey2 = lateral_sq(tr, x.px, x.py, idx);
      h1 = tr.w2 - ey2;
      R pen1 = fmax(C.alpha * h0 - h1, R(0));
      h0 = h1;
      outside = h1 < R(0);
      os.step2(p0x, p0y, p1x, p1y, x.px, x.py, C.alpha, pen0, out1, pen1, outside);
      S += C.C_cbf * pen0;
      if (out1) q1 += C.C_obs;
      S += q1 + ctl1;
      S += C.C_cbf * pen1;
    }
  }
  for (; t < T; ++t) {
    const R v0 = V[t], v1 = V[T + t];
    R e0, e1;
    ns.at(t, C.sigma[0], C.sigma[1], e0, e1);
    const R u0 = clamp_r(v0 + e0, M.u_lo[0], M.u_hi[0]);
    const R u1 = clamp_r(v1 + e1, M.u_lo[1], M.u_hi[1]);
    if (eps_out) {
      eps_out[2 * t] = u0 - v0;
      eps_out[2 * t + 1] = u1 - v1;
    }
    const R dv = x.vx - C.v_g;
    R q = C.q_v * dv * dv + C.q_ey * ey2;
    if (outside) q += C.C_obs;
    S += q + (C.ctrl_w[0] * v0 * u0 + C.ctrl_w[1] * v1 * u1);
    const StepCtl<R> sc = step_ctl(M, u0, u1);
    const R ppx = x.px, ppy = x.py;
    rk4(M, sc, x);
    ey2 = lateral_sq(tr, x.px, x.py, idx);
    const R h1 = tr.w2 - ey2;
    R pen = fmax(C.alpha * h0 - h1, R(0));
    h0 = h1;
    outside = h1 < R(0);
    if constexpr (NOBS > 0 && WV) os.step(ppx, ppy, x.px, x.py, C.alpha, pen, outside);
    else if constexpr (NOBS > 0) os.template step<NOBS>(x.px, x.py, C.alpha, hob, pen, outside);
    S += C.C_cbf * pen;
  }
  const R dv = x.vx - C.v_g;
  R q = C.q_v * dv * dv + C.q_ey * ey2;
  if (outside) q += C.C_obs;
  S += C.phi_w * q;
  return S;
}

template <class R, int NOBS>
__device__ R rollout_sample(const DevModel<R>& M, const DevCost<R>& C, const TrackView<R>& tr, const State<R>& x0,
                            const R* __restrict__ V, int T, NoiseStream<R>& ns, R* eps_out) {
  return rollout_sample<R, NOBS>(M, C, tr, x0, V, T, ns, eps_out, LdsObstacles<R>{&tr});
}

// ---------------------------------------------------------------- adjoint
// Vector-Jacobian product of one derivative evaluation: given the cotangent
// (gpx, gpy, gpsi, gvx, gvy, gom) of f's output at (psi, vx, vy, om) with the
// step control, accumulate d/d(psi, vx, vy, om) into o* and d/d(delta, tau)
// into gd, gt.
template <class R>
__device__ __forceinline__ void deriv_vjp(const DevModel<R>& M, const StepCtl<R>& c, R psi, R vx, R vy, R om,
                                          R gpx, R gpy, R gpsi, R gvx, R gvy, R gom, R& opsi, R& ovx, R& ovy,
                                          R& oom, R& gd, R& gt) {
  const bool above = vx >= M.v_min;
  const R vt = fmax(vx, M.v_min);
  const R inv = rcp_r(vt);
  const R Ff = M.Cf * (c.delta - (vy + M.lf * om) * inv);
  const R Fr = M.Cr * ((M.lr * om - vy) * inv);
  R sp, cp;
  sincos_r(psi, &sp, &cp);
  // kinematics
  const R dpx = vx * cp - vy * sp, dpy = vx * sp + vy * cp;
  opsi += gpy * dpx - gpx * dpy;
  ovx += gpx * cp + gpy * sp;
  ovy += gpy * cp - gpx * sp;
  oom += gpsi;
  // v_x equation
  ovx += -M.c_v * gvx - om * gvy;
  ovy += om * gvx;
  oom += vy * gvx - vx * gvy;
  gt += M.a_max * gvx;
  // tyre forces
  const R gFf = -c.sd_m * gvx + c.cd_m * gvy + c.lfcd_Iz * gom;
  const R gFr = M.inv_m * gvy - M.lr_Iz * gom;
  gd += -Ff * c.cd * M.inv_m * gvx - Ff * c.sd * M.inv_m * gvy - Ff * c.sd * M.lf_Iz * gom;
  const R gaf = M.Cf * gFf, gar = M.Cr * gFr;
  gd += gaf;
  ovy += -inv * (gaf + gar);
  oom += inv * (M.lr * gar - M.lf * gaf);
  const R ginv = -(vy + M.lf * om) * gaf + (M.lr * om - vy) * gar;
  if (above) ovx += -inv * inv * ginv;
}

// Reverse of one RK4 step from x (stage states recomputed): given lam =
// dL/dx_{t+1}, returns dL/dx_t in lam and accumulates dL/du into gd, gt.
template <class R>
__device__ __forceinline__ void rk4_vjp(const DevModel<R>& M, const StepCtl<R>& c, const State<R>& x, R lam[6],
                                        R& gd, R& gt) {
  const R h = M.dt, h2 = R(0.5) * M.dt, h6 = M.dt * R(1.0 / 6.0);
  R a0, a1, a3, a4, a5, b0, b1, b3, b4, b5, c0, c1, c3, c4, c5;
  deriv(M, c, x.psi, x.vx, x.vy, x.om, a0, a1, a3, a4, a5);
  const R a2 = x.om;
  const R X2psi = x.psi + h2 * a2, X2vx = x.vx + h2 * a3, X2vy = x.vy + h2 * a4, X2om = x.om + h2 * a5;
  deriv(M, c, X2psi, X2vx, X2vy, X2om, b0, b1, b3, b4, b5);
  const R b2 = X2om;
  const R X3psi = x.psi + h2 * b2, X3vx = x.vx + h2 * b3, X3vy = x.vy + h2 * b4, X3om = x.om + h2 * b5;
  deriv(M, c, X3psi, X3vx, X3vy, X3om, c0, c1, c3, c4, c5);
  const R c2 = X3om;
  const R X4psi = x.psi + h * c2, X4vx = x.vx + h * c3, X4vy = x.vy + h * c4, X4om = x.om + h * c5;
  // cotangents of the stage derivatives k1..k4: (h/6, h/3, h/3, h/6) * lam
  R gk4[6], gk3[6], gk2[6], gk1[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    gk4[i] = h6 * lam[i];
    gk3[i] = R(2) * h6 * lam[i];
    gk2[i] = R(2) * h6 * lam[i];
    gk1[i] = h6 * lam[i];
  }
  // k4 = f(X4): X4 = x + h k3 (p components of k feed only the output)
  R o[4] = {R(0), R(0), R(0), R(0)};
  deriv_vjp(M, c, X4psi, X4vx, X4vy, X4om, gk4[0], gk4[1], gk4[2], gk4[3], gk4[4], gk4[5], o[0], o[1], o[2],
            o[3], gd, gt);
  // psi component of k is omega of the stage state: dpsi_dot/dom = 1 (inside deriv_vjp via gpsi)
  lam[2] += o[0];
  lam[3] += o[1];
  lam[4] += o[2];
  lam[5] += o[3];
  gk3[2] += h * o[0];
  gk3[3] += h * o[1];
  gk3[4] += h * o[2];
  gk3[5] += h * o[3];
  o[0] = o[1] = o[2] = o[3] = R(0);
  deriv_vjp(M, c, X3psi, X3vx, X3vy, X3om, gk3[0], gk3[1], gk3[2], gk3[3], gk3[4], gk3[5], o[0], o[1], o[2],
            o[3], gd, gt);
  lam[2] += o[0];
  lam[3] += o[1];
  lam[4] += o[2];
  lam[5] += o[3];
  gk2[2] += h2 * o[0];
  gk2[3] += h2 * o[1];
  gk2[4] += h2 * o[2];
  gk2[5] += h2 * o[3];
  o[0] = o[1] = o[2] = o[3] = R(0);
  deriv_vjp(M, c, X2psi, X2vx, X2vy, X2om, gk2[0], gk2[1], gk2[2], gk2[3], gk2[4], gk2[5], o[0], o[1], o[2],
            o[3], gd, gt);
  lam[2] += o[0];
  lam[3] += o[1];
  lam[4] += o[2];
  lam[5] += o[3];
  gk1[2] += h2 * o[0];
  gk1[3] += h2 * o[1];
  gk1[4] += h2 * o[2];
  gk1[5] += h2 * o[3];
  o[0] = o[1] = o[2] = o[3] = R(0);
  deriv_vjp(M, c, x.psi, x.vx, x.vy, x.om, gk1[0], gk1[1], gk1[2], gk1[3], gk1[4], gk1[5], o[0], o[1], o[2],
            o[3], gd, gt);
  lam[2] += o[0];
  lam[3] += o[1];
  lam[4] += o[2];
  lam[5] += o[3];
  (void)a0; (void)a1; (void)b0; (void)b1; (void)c0; (void)c1;
}

// Barrier values at a state, given the segment index at that state.
template <class R, int NOBS>
__device__ __forceinline__ R track_h_at(const TrackView<R>& tr, const State<R>& x, int idx) {
  R e2;
  if (tr.n == 0) {
    int dummy = 0;
    e2 = lateral_sq(tr, x.px, x.py, dummy);
  } else {
    e2 = seg_dist2(tr, idx, x.px, x.py);
  }
  return tr.w2 - e2;
}

// Adds dP/dx for the transition penalty between x_t (prev) and x_{t+1} (next):
// r_j = alpha h_j(x_t) - h_j(x_{t+1}); dL/dr_j = w_S C + 2 w_sq r_j + w_lin [t < n_lin]
// when r_j > 0.  lam_next gets the x_{t+1} part, g_prev the x_t part (p only).
template <class R, int NOBS>
__device__ __forceinline__ void penalty_grad(const DevCost<R>& C, const DevObjective<R>& ob, const TrackView<R>& tr,
                                             const State<R>& xp, int ip, const State<R>& xn, int in_, int t,
                                             R lam_next[6], R& gpx_prev, R& gpy_prev) {
  const R lin = (t < ob.n_lin) ? ob.w_lin : R(0);
  {
    const R hp = track_h_at<R, NOBS>(tr, xp, ip), hn = track_h_at<R, NOBS>(tr, xn, in_);
    const R r = C.alpha * hp - hn;
    if (r > R(0)) {
      const R g = ob.w_S * C.C_cbf + R(2) * ob.w_sq * r + lin;
      R gx, gy;
      // dh/dp = -d(e^2)/dp
      lateral_sq_grad(tr, xn.px, xn.py, in_, gx, gy);
      lam_next[0] += g * gx;
      lam_next[1] += g * gy;
      lateral_sq_grad(tr, xp.px, xp.py, ip, gx, gy);
      gpx_prev -= g * C.alpha * gx;
      gpy_prev -= g * C.alpha * gy;
    }
  }
#pragma unroll
  for (int i = 0; i < NOBS; ++i) {
    const Obs<R> o = obs_at(tr, i);
    const R pxp = xp.px - o.cx, pyp = xp.py - o.cy, pxn = xn.px - o.cx, pyn = xn.py - o.cy;
    const R hp = pxp * pxp + pyp * pyp - o.re2, hn = pxn * pxn + pyn * pyn - o.re2;
    const R r = C.alpha * hp - hn;
    const R g = r > R(0) ? ob.w_S * C.C_cbf + R(2) * ob.w_sq * r + lin : R(0);
    lam_next[0] -= g * R(2) * pxn;
    lam_next[1] -= g * R(2) * pyn;
    gpx_prev += g * C.alpha * R(2) * pxp;
    gpy_prev += g * C.alpha * R(2) * pyp;
  }
}

// d q'(x)/dx (q' = q without the indicator): speed term and lateral term.
template <class R>
__device__ __forceinline__ void stage_grad(const DevCost<R>& C, const TrackView<R>& tr, const State<R>& x, int idx,
                                           R scale, R lam[6]) {
  lam[3] += scale * R(2) * C.q_v * (x.vx - C.v_g);
  R gx, gy;
  lateral_sq_grad(tr, x.px, x.py, idx, gx, gy);
  lam[0] += scale * C.q_ey * gx;
  lam[1] += scale * C.q_ey * gy;
}

}  // namespace smppi
