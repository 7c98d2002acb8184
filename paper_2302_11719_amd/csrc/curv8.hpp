// The curvilinear eight-state vehicle model (Sec. VI-A: body velocities, yaw
// rate, front and rear wheel speeds, heading error, lateral deviation and
// progress along the centre line) on the device: its derivative, RK4 step and
// the hand-written vector-Jacobian products of both; the sampled rollout, the
// K-sample adjoint with recomputed states, the shield of Algorithm 1 and the
// plant step.  The track barrier of eq. (23), h = w^2 - e_y^2, is read from the
// state; the track enters only through the curvature table kappa(s).
//
// Model (the paper names the states and a single-track bicycle model but prints
// no equations; this is the reading the library documents):
//   F_yF = C_f (delta - (v_y + l_f r) / v~),  F_yR = C_r (l_r r - v_y) / v~,  v~ = max(v_x, v_min)
//   F_xF = C_x (r_w omega_F - v_wF) / v~,  v_wF = v_x cos(delta) + (v_y + l_f r) sin(delta)
//   F_xR = C_x (r_w omega_R - v_x) / v~
//   v_x' = (F_xR + F_xF cos(delta) - F_yF sin(delta)) / m - c_v v_x + v_y r
//   v_y' = (F_yR + F_xF sin(delta) + F_yF cos(delta)) / m - v_x r
//   r'   = (l_f (F_xF sin(delta) + F_yF cos(delta)) - l_r F_yR) / I_z
//   omega_F' = -r_w F_xF / I_w,   omega_R' = (m a_max r_w T - r_w F_xR) / I_w
//   s' = (v_x cos(e_psi) - v_y sin(e_psi)) / (1 - kappa(s) e_y)
//   e_y' = v_x sin(e_psi) + v_y cos(e_psi),   e_psi' = r - kappa(s) s'
// With both wheels at their equilibrium speeds the body equations are the
// six-state model's (drive m a_max T on the body, no front longitudinal force).
#pragma once

#include "kernels.hpp"

namespace smppi {

template <class R>
struct DevWheels {
  R r_w, C_x, rw_Iw, drive_Iw;  // wheel radius, slip stiffness, r_w / I_w, m a_max r_w / I_w
};

// State in the paper's order.
template <class R>
struct C8 {
  R vx, vy, r, wF, wR, ep, ey, s;
};

// Held control of one step: steer and its sine/cosine, throttle.
template <class R>
struct Ctl8 {
  R delta, sd, cd, thr;
};

template <class R>
__device__ __forceinline__ Ctl8<R> ctl8(R delta, R thr) {
  Ctl8<R> c;
  sincos_r(delta, &c.sd, &c.cd);
  c.delta = delta;
  c.thr = thr;
  return c;
}

// kappa(s) of the periodic table (linear between grid points) and its slope in
// the cell holding s.  The cell index floor(s/ds) mod n is formed in floating
// point with multiplications by 1/ds and 1/n (no division on the chain; exact
// while |s/ds| < 2^24 in FP32, and a rounding of the quotient by n that leaves
// -1 or n is folded back); non-finite s, or s beyond that range, maps to cell 0.
template <class R>
__device__ __forceinline__ R kappa_cell(const CurvView<R>& cv, R s, R& slope) {
  const R q = s * cv.inv_ds;
  const R jf = floor(q);
  const R f = q - jf;
  R jw = fma_r(-cv.rn, floor(jf * cv.inv_n), jf);
  jw += jw < R(0) ? cv.rn : R(0);
  jw -= jw >= cv.rn ? cv.rn : R(0);
  const int j = (jw >= R(0) && jw < cv.rn) ? (int)jw : 0;
  const int j1 = j + 1 == cv.n ? 0 : j + 1;
  const R k0 = cv.kappa[j], k1 = cv.kappa[j1];
  slope = (k1 - k0) * cv.inv_ds;
  return k0 * (R(1) - f) + k1 * f;
}

// Body part of f: (v_x, v_y, r, omega_F, omega_R) from themselves and the control
// (the tyre forces depend on neither the path coordinates nor the curvature).
template <class R>
__device__ __forceinline__ void deriv_c8_body(const DevModel<R>& M, const DevWheels<R>& Wh, const Ctl8<R>& c,
                                              const C8<R>& x, C8<R>& d) {
  const R vt = fmax(x.vx, M.v_min);
  const R inv = rcp_r(vt);
  const R a = fma_r(M.lf, x.r, x.vy);
  const R FyF = M.Cf * fma_r(-a, inv, c.delta);
  const R FyR = M.Cr * (fma_r(M.lr, x.r, -x.vy) * inv);
  const R vwF = fma_r(x.vx, c.cd, a * c.sd);
  const R FxF = Wh.C_x * (fma_r(Wh.r_w, x.wF, -vwF) * inv);
  const R FxR = Wh.C_x * (fma_r(Wh.r_w, x.wR, -x.vx) * inv);
  d.vx = fma_r(FxR + fma_r(FxF, c.cd, -(FyF * c.sd)), M.inv_m, fma_r(-M.c_v, x.vx, x.vy * x.r));
  d.vy = fma_r(FyR + fma_r(FxF, c.sd, FyF * c.cd), M.inv_m, -(x.vx * x.r));
  d.r = fma_r(M.lf_Iz, fma_r(FxF, c.sd, FyF * c.cd), -(M.lr_Iz * FyR));
  d.wF = -(Wh.rw_Iw * FxF);
  d.wR = fma_r(Wh.drive_Iw, c.thr, -(Wh.rw_Iw * FxR));
}

// Path part of f: (e_psi, e_y, s) from themselves, (v_x, v_y, r) and kappa(s).
template <class R>
__device__ __forceinline__ void deriv_c8_path(const CurvView<R>& cv, const C8<R>& x, C8<R>& d) {
  R slope;
  const R k = kappa_cell(cv, x.s, slope);
  R se, ce;
  sincos_r(x.ep, &se, &ce);
  const R sdot = fma_r(x.vx, ce, -(x.vy * se)) * rcp_r(fma_r(-k, x.ey, R(1)));
  d.ep = fma_r(-k, sdot, x.r);
  d.ey = fma_r(x.vx, se, x.vy * ce);
  d.s = sdot;
}

template <class R>
__device__ __forceinline__ void deriv_c8(const DevModel<R>& M, const DevWheels<R>& Wh, const CurvView<R>& cv,
                                         const Ctl8<R>& c, const C8<R>& x, C8<R>& d) {
  deriv_c8_body(M, Wh, c, x, d);
  deriv_c8_path(cv, x, d);
}

// y = x + h k
template <class R>
__device__ __forceinline__ C8<R> axpy8(R h, const C8<R>& k, const C8<R>& x) {
  return C8<R>{fma_r(h, k.vx, x.vx), fma_r(h, k.vy, x.vy), fma_r(h, k.r, x.r),   fma_r(h, k.wF, x.wF),
               fma_r(h, k.wR, x.wR), fma_r(h, k.ep, x.ep), fma_r(h, k.ey, x.ey), fma_r(h, k.s, x.s)};
}

// Classic RK4 over dt with the control held.
template <class R>
__device__ __forceinline__ void rk4_c8(const DevModel<R>& M, const DevWheels<R>& Wh, const CurvView<R>& cv,
                                       const Ctl8<R>& c, C8<R>& x) {
  const R h = M.dt, h2 = R(0.5) * M.dt, h6 = M.dt * R(1.0 / 6.0);
  C8<R> k1, k2, k3, k4;
  deriv_c8(M, Wh, cv, c, x, k1);
  deriv_c8(M, Wh, cv, c, axpy8(h2, k1, x), k2);
  deriv_c8(M, Wh, cv, c, axpy8(h2, k2, x), k3);
  deriv_c8(M, Wh, cv, c, axpy8(h, k3, x), k4);
  auto comb = [&](R a1, R a2, R a3, R a4, R xv) { return fma_r(h6, fma_r(R(2), a2 + a3, a1) + a4, xv); };
  x.vx = comb(k1.vx, k2.vx, k3.vx, k4.vx, x.vx);
  x.vy = comb(k1.vy, k2.vy, k3.vy, k4.vy, x.vy);
  x.r = comb(k1.r, k2.r, k3.r, k4.r, x.r);
  x.wF = comb(k1.wF, k2.wF, k3.wF, k4.wF, x.wF);
  x.wR = comb(k1.wR, k2.wR, k3.wR, k4.wR, x.wR);
  x.ep = comb(k1.ep, k2.ep, k3.ep, k4.ep, x.ep);
  x.ey = comb(k1.ey, k2.ey, k3.ey, k4.ey, x.ey);
  x.s = comb(k1.s, k2.s, k3.s, k4.s, x.s);
}

// Vector-Jacobian product of deriv_c8 at x: given the cotangent g of the
// derivative, accumulates d/dx into o and d/d(delta, T) into gd, gt.
template <class R>
__device__ __forceinline__ void deriv_c8_vjp(const DevModel<R>& M, const DevWheels<R>& Wh, const CurvView<R>& cv,
                                             const Ctl8<R>& c, const C8<R>& x, const C8<R>& g, C8<R>& o, R& gd,
                                             R& gt) {
  // forward intermediates
  const bool above = x.vx >= M.v_min;
  const R vt = fmax(x.vx, M.v_min);
  const R inv = rcp_r(vt);
  const R a = fma_r(M.lf, x.r, x.vy);
  const R z = fma_r(M.lr, x.r, -x.vy);
  const R FyF = M.Cf * fma_r(-a, inv, c.delta);
  const R FyR = M.Cr * (z * inv);
  const R vwF = fma_r(x.vx, c.cd, a * c.sd);
  const R p = fma_r(Wh.r_w, x.wF, -vwF), q = fma_r(Wh.r_w, x.wR, -x.vx);
  const R FxF = Wh.C_x * (p * inv);
  const R FxR = Wh.C_x * (q * inv);
  R slope;
  const R k = kappa_cell(cv, x.s, slope);
  R se, ce;
  sincos_r(x.ep, &se, &ce);
  const R rden = rcp_r(fma_r(-k, x.ey, R(1)));
  const R sdot = fma_r(x.vx, ce, -(x.vy * se)) * rden;
  // cotangents of the tyre forces
  const R gFxF = M.inv_m * (g.vx * c.cd + g.vy * c.sd) + M.lf_Iz * c.sd * g.r - Wh.rw_Iw * g.wF;
  const R gFxR = M.inv_m * g.vx - Wh.rw_Iw * g.wR;
  const R gFyF = M.inv_m * (g.vy * c.cd - g.vx * c.sd) + M.lf_Iz * c.cd * g.r;
  const R gFyR = M.inv_m * g.vy - M.lr_Iz * g.r;
  // terms of the outputs that are direct in the state
  o.vx += -M.c_v * g.vx - x.r * g.vy + se * g.ey;
  o.vy += x.r * g.vx + ce * g.ey;
  o.r += x.vy * g.vx - x.vx * g.vy + g.ep;
  gt += Wh.drive_Iw * g.wR;
  R gcd = M.inv_m * (g.vx * FxF + g.vy * FyF) + M.lf_Iz * FyF * g.r;
  R gsd = M.inv_m * (g.vy * FxF - g.vx * FyF) + M.lf_Iz * FxF * g.r;
  // Frenet kinematics: s' = num / den, e_psi' = r - k s', e_y' = v_x se + v_y ce
  const R gsdot = g.s - k * g.ep;
  const R gnum = gsdot * rden;
  const R gden = -gsdot * sdot * rden;
  const R gk = -sdot * g.ep - x.ey * gden;
  o.vx += ce * gnum;
  o.vy += -se * gnum;
  const R gce = x.vx * gnum + x.vy * g.ey;
  const R gse = -x.vy * gnum + x.vx * g.ey;
  o.ey += -k * gden;
  o.ep += ce * gse - se * gce;
  o.s += slope * gk;
  // longitudinal forces
  const R gq = Wh.C_x * inv * gFxR;
  R ginv = Wh.C_x * q * gFxR;
  o.wR += Wh.r_w * gq;
  o.vx -= gq;
  const R gp = Wh.C_x * inv * gFxF;
  ginv += Wh.C_x * p * gFxF;
  o.wF += Wh.r_w * gp;
  o.vx -= c.cd * gp;  // v_wF = v_x cos(delta) + a sin(delta), p = r_w omega_F - v_wF
  R ga = -c.sd * gp;
  gcd += -x.vx * gp;
  gsd += -a * gp;
  // lateral forces
  const R gz = M.Cr * inv * gFyR;
  ginv += M.Cr * z * gFyR;
  o.r += M.lr * gz;
  o.vy -= gz;
  gd += M.Cf * gFyF;
  ga += -M.Cf * inv * gFyF;
  ginv += -M.Cf * a * gFyF;
  o.vy += ga;
  o.r += M.lf * ga;
  if (above) o.vx += -inv * inv * ginv;
  gd += c.cd * gsd - c.sd * gcd;
}

template <class R>
__device__ __forceinline__ void scale_add8(C8<R>& y, R h, const C8<R>& x) {
  y.vx = fma_r(h, x.vx, y.vx); y.vy = fma_r(h, x.vy, y.vy); y.r = fma_r(h, x.r, y.r); y.wF = fma_r(h, x.wF, y.wF);
  y.wR = fma_r(h, x.wR, y.wR); y.ep = fma_r(h, x.ep, y.ep); y.ey = fma_r(h, x.ey, y.ey); y.s = fma_r(h, x.s, y.s);
}
template <class R>
__device__ __forceinline__ C8<R> scaled8(R h, const C8<R>& x) {
  return C8<R>{h * x.vx, h * x.vy, h * x.r, h * x.wF, h * x.wR, h * x.ep, h * x.ey, h * x.s};
}
template <class R>
__device__ __forceinline__ C8<R> zero8() {
  return C8<R>{R(0), R(0), R(0), R(0), R(0), R(0), R(0), R(0)};
}

// Reverse of one RK4 step from x (stage states recomputed): lam = dL/dx_{t+1}
// in, dL/dx_t out; dL/du accumulated into gd, gt.
template <class R>
__device__ __forceinline__ void rk4_c8_vjp(const DevModel<R>& M, const DevWheels<R>& Wh, const CurvView<R>& cv,
                                           const Ctl8<R>& c, const C8<R>& x, C8<R>& lam, R& gd, R& gt) {
  const R h = M.dt, h2 = R(0.5) * M.dt, h6 = M.dt * R(1.0 / 6.0);
  C8<R> k1, k2, k3;
  deriv_c8(M, Wh, cv, c, x, k1);
  const C8<R> X2 = axpy8(h2, k1, x);
  deriv_c8(M, Wh, cv, c, X2, k2);
  const C8<R> X3 = axpy8(h2, k2, x);
  deriv_c8(M, Wh, cv, c, X3, k3);
  const C8<R> X4 = axpy8(h, k3, x);
  // x_{t+1} = x + h6 (k1 + 2 k2 + 2 k3 + k4); stage k_i = f(X_i)
  C8<R> gk3 = scaled8(R(2) * h6, lam), gk2 = gk3, gk1 = scaled8(h6, lam);
  C8<R> o = zero8<R>();
  deriv_c8_vjp(M, Wh, cv, c, X4, scaled8(h6, lam), o, gd, gt);  // X4 = x + h k3
  scale_add8(lam, R(1), o);
  scale_add8(gk3, h, o);
  o = zero8<R>();
  deriv_c8_vjp(M, Wh, cv, c, X3, gk3, o, gd, gt);  // X3 = x + h2 k2
  scale_add8(lam, R(1), o);
  scale_add8(gk2, h2, o);
  o = zero8<R>();
  deriv_c8_vjp(M, Wh, cv, c, X2, gk2, o, gd, gt);  // X2 = x + h2 k1
  scale_add8(lam, R(1), o);
  scale_add8(gk1, h2, o);
  o = zero8<R>();
  deriv_c8_vjp(M, Wh, cv, c, x, gk1, o, gd, gt);
  scale_add8(lam, R(1), o);
}

// Running cost gradient (without the indicator): speed and lateral terms.
template <class R>
__device__ __forceinline__ void stage_grad_c8(const DevCost<R>& C, const C8<R>& x, R scale, C8<R>& lam) {
  lam.vx += scale * R(2) * C.q_v * (x.vx - C.v_g);
  lam.ey += scale * R(2) * C.q_ey * x.ey;
}

// Transition t (x_t = xp -> x_{t+1} = xn) of the track barrier h = w^2 - e_y^2:
// when r = alpha h(x_t) - h(x_{t+1}) > 0, dL/dr = w_S C + 2 w_sq r + w_lin [t < n_lin];
// adds the x_{t+1} part to lam_next, returns the x_t part (an e_y cotangent).
template <class R>
__device__ __forceinline__ R penalty_grad_c8(const DevCost<R>& C, const DevObjective<R>& ob, R w2, const C8<R>& xp,
                                             const C8<R>& xn, int t, C8<R>& lam_next) {
  const R hp = w2 - xp.ey * xp.ey, hn = w2 - xn.ey * xn.ey;
  const R r = C.alpha * hp - hn;
  if (!(r > R(0))) return R(0);
  const R g = ob.w_S * C.C_cbf + R(2) * ob.w_sq * r + ((t < ob.n_lin) ? ob.w_lin : R(0));
  lam_next.ey += g * R(2) * xn.ey;
  return -g * C.alpha * R(2) * xp.ey;
}

// Sampled cost S~ of one trajectory (Algorithm 2 inner loop, eqs. (17)-(20),
// (23)-(25)), as rollout_sample with the barrier read from e_y.
template <class R>
__device__ R rollout_sample_c8(const DevModel<R>& M, const DevWheels<R>& Wh, const DevCost<R>& C,
                               const CurvView<R>& cv, C8<R> x, const R* __restrict__ V, int T, NoiseStream<R>& ns,
                               R* eps_out) {
  R h0 = cv.w2 - x.ey * x.ey;
  bool outside = h0 < R(0);
  R S = C.C_cbf * fmax((C.alpha - R(1)) * h0, R(0));
  for (int t = 0; t < T; ++t) {
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
    R q = C.q_v * dv * dv + C.q_ey * (x.ey * x.ey);
    if (outside) q += C.C_obs;
    S += q + (C.ctrl_w[0] * v0 * u0 + C.ctrl_w[1] * v1 * u1);
    rk4_c8(M, Wh, cv, ctl8(u0, u1), x);
    const R h1 = cv.w2 - x.ey * x.ey;
    S += C.C_cbf * fmax(C.alpha * h0 - h1, R(0));
    h0 = h1;
    outside = h1 < R(0);
  }
  const R dv = x.vx - C.v_g;
  R q = C.q_v * dv * dv + C.q_ey * (x.ey * x.ey);
  if (outside) q += C.C_obs;
  S += C.phi_w * q;
  return S;
}

template <class R>
__device__ __forceinline__ C8<R> load_c8(const R* p) {
  return C8<R>{p[0], p[1], p[2], p[3], p[4], p[5], p[6], p[7]};
}
template <class R>
__device__ __forceinline__ void store_c8(R* p, const C8<R>& x) {
  p[0] = x.vx; p[1] = x.vy; p[2] = x.r; p[3] = x.wF; p[4] = x.wR; p[5] = x.ep; p[6] = x.ey; p[7] = x.s;
}
// Lane-strided LDS slot [8][64]: component i of lane at base[i * WAVE + lane].
template <class R>
__device__ __forceinline__ void store_c8_lane(R* base, int lane, const C8<R>& x) {
  base[0 * WAVE + lane] = x.vx; base[1 * WAVE + lane] = x.vy; base[2 * WAVE + lane] = x.r;
  base[3 * WAVE + lane] = x.wF; base[4 * WAVE + lane] = x.wR; base[5 * WAVE + lane] = x.ep;
  base[6 * WAVE + lane] = x.ey; base[7 * WAVE + lane] = x.s;
}
template <class R>
__device__ __forceinline__ C8<R> load_c8_lane(const R* base, int lane) {
  return C8<R>{base[0 * WAVE + lane], base[1 * WAVE + lane], base[2 * WAVE + lane], base[3 * WAVE + lane],
               base[4 * WAVE + lane], base[5 * WAVE + lane], base[6 * WAVE + lane], base[7 * WAVE + lane]};
}

// ---------------------------------------------------------------- kernels
template <class R>
struct C8Args {
  const int64_t* k_off;
  const int32_t* t_off;
  const int32_t* kappa_off;
  const R* kappa;
  const R* ds;
  const R* half_width;
  const R* x0;  // [B][8]
  const uint32_t* iter;
  const R* V;
  DevModel<R> M;
  DevWheels<R> Wh;
  DevCost<R> C;
  int32_t B, k_max, t_max, n_max, pid_base;
  uint32_t seed;
  int32_t nominal;
  uint32_t* err;
};

struct C8Dims {
  int64_t k0;
  int K, t0, T, c0, n;
};

// Problem b's sizes; false (flag raised) when device data breaks a bound the
// kernels rely on.
template <class R>
__device__ __forceinline__ bool c8_dims(const C8Args<R>& a, int b, C8Dims& d) {
  d.k0 = a.k_off[b];
  const int64_t K = a.k_off[b + 1] - d.k0;
  d.t0 = a.t_off[b];
  d.T = a.t_off[b + 1] - d.t0;
  d.c0 = a.kappa_off[b];
  d.n = a.kappa_off[b + 1] - d.c0;
  uint32_t e = 0;
  if (d.T < 1 || d.T > a.t_max) e |= DERR_T;
  if (K < 0 || K > a.k_max) e |= DERR_K;
  if (d.n < 2 || d.n > a.n_max) e |= DERR_POLY;
  d.K = (int)K;
  if (e) {
    if (threadIdx.x == 0 && blockIdx.x == 0) atomicOr(a.err, e);
    return false;
  }
  return true;
}

// The curvature table [n_max] and V [2][t_max] of problem b staged in LDS.
template <class R>
__device__ __forceinline__ CurvView<R> c8_stage(const C8Args<R>& a, int b, const C8Dims& d, R* lds, R** Vs) {
  R* kap = lds;
  R* v = kap + a.n_max;
  for (int i = threadIdx.x; i < d.n; i += blockDim.x) kap[i] = a.kappa[d.c0 + i];
  for (int i = threadIdx.x; i < 2 * d.T; i += blockDim.x) v[i] = a.V[2 * (size_t)d.t0 + i];
  const R w = a.half_width[b];
  *Vs = v;
  return curv_view(static_cast<const R*>(kap), d.n, a.ds[b], w * w);
}

template <class R>
__host__ __device__ inline size_t c8_stage_bytes(int n_max, int t_max) {
  return (sizeof(R) * ((size_t)n_max + 2 * (size_t)t_max) + 15) & ~(size_t)15;
}

template <class R>
__device__ __forceinline__ NoiseStream<R> c8_noise(const C8Args<R>& a, int b, int m) {
  NoiseStream<R> ns;
  ns.seed = a.seed;
  ns.m = (uint32_t)m;
  ns.pid = (uint32_t)(a.pid_base + b);
  ns.it = a.iter[b];
  ns.nominal = a.nominal != 0;
  return ns;
}

// Sampled costs: one sample per lane, grid (ceil(k_max / 256), B).
template <class R>
__global__ __launch_bounds__(256) void k_rollout_c8(C8Args<R> a, R* S, R* eps_out) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int b = blockIdx.y;
  C8Dims d;
  if (!c8_dims(a, b, d)) return;
  const int m_base = blockIdx.x * blockDim.x;
  if (m_base >= d.K) return;
  R* Vs;
  const CurvView<R> cv = c8_stage(a, b, d, reinterpret_cast<R*>(smem), &Vs);
  __syncthreads();
  const int m = m_base + threadIdx.x;
  if (m >= d.K) return;
  NoiseStream<R> ns = c8_noise(a, b, m);
  R* eo = eps_out ? eps_out + ((size_t)(d.k0 + m)) * a.t_max * 2 : nullptr;
  S[d.k0 + m] = rollout_sample_c8(a.M, a.Wh, a.C, cv, load_c8(a.x0 + 8 * (size_t)b), Vs, d.T, ns, eo);
}

// Reverse sweep of one lane's trajectory with checkpoints every seg_len steps
// (ck [n_ck][8][64], global scratch of the workgroup) and one recomputed
// segment (sx [seg_len+1][8][64], LDS); sink(t, dL/dv_t0, dL/dv_t1) for t
// descending.
template <class R, class Sink>
__device__ void adjoint_lane_c8(const DevModel<R>& M, const DevWheels<R>& Wh, const DevCost<R>& C,
                                const DevObjective<R>& ob, const CurvView<R>& cv, const C8<R>& x0, const R* V, int T,
                                NoiseStream<R>& ns, R* ck, R* sx, int seg_len, int lane, Sink& sink) {
  C8<R> x = x0;
  for (int t = 0; t < T; ++t) {
    if (t % seg_len == 0) store_c8_lane(ck + (size_t)(t / seg_len) * 8 * WAVE, lane, x);
    R e0, e1;
    ns.at(t, C.sigma[0], C.sigma[1], e0, e1);
    const R u0 = clamp_r(V[t] + e0, M.u_lo[0], M.u_hi[0]);
    const R u1 = clamp_r(V[T + t] + e1, M.u_lo[1], M.u_hi[1]);
    rk4_c8(M, Wh, cv, ctl8(u0, u1), x);
  }
  C8<R> lam = zero8<R>();
  stage_grad_c8(C, x, ob.w_S * C.phi_w, lam);
  const int n_seg = (T + seg_len - 1) / seg_len;
  for (int c = n_seg - 1; c >= 0; --c) {
    const int t0 = c * seg_len, t1 = min(T, t0 + seg_len);
    C8<R> xs = load_c8_lane(ck + (size_t)c * 8 * WAVE, lane);
    store_c8_lane(sx, lane, xs);
    for (int t = t0; t < t1; ++t) {
      R e0, e1;
      if (t == t0 || (t & 1) == 0) ns.gen(t);
      ns.get(t, C.sigma[0], C.sigma[1], e0, e1);
      const R u0 = clamp_r(V[t] + e0, M.u_lo[0], M.u_hi[0]);
      const R u1 = clamp_r(V[T + t] + e1, M.u_lo[1], M.u_hi[1]);
      rk4_c8(M, Wh, cv, ctl8(u0, u1), xs);
      store_c8_lane(sx + (size_t)(t - t0 + 1) * 8 * WAVE, lane, xs);
    }
    for (int t = t1 - 1; t >= t0; --t) {
      const C8<R> xp = load_c8_lane(sx + (size_t)(t - t0) * 8 * WAVE, lane);
      const C8<R> xn = load_c8_lane(sx + (size_t)(t - t0 + 1) * 8 * WAVE, lane);
      const R gey_prev = penalty_grad_c8(C, ob, cv.w2, xp, xn, t, lam);
      R e0, e1;
      if ((t & 1) == 1 || t == t1 - 1) ns.gen(t);
      ns.get(t, C.sigma[0], C.sigma[1], e0, e1);
      const R v0 = V[t], v1 = V[T + t];
      const R r0 = v0 + e0, r1 = v1 + e1;
      const R u0 = clamp_r(r0, M.u_lo[0], M.u_hi[0]);
      const R u1 = clamp_r(r1, M.u_lo[1], M.u_hi[1]);
      const bool pass0 = (r0 >= M.u_lo[0]) && (r0 <= M.u_hi[0]);
      const bool pass1 = (r1 >= M.u_lo[1]) && (r1 <= M.u_hi[1]);
      R gd = R(0), gt = R(0);
      rk4_c8_vjp(M, Wh, cv, ctl8(u0, u1), xp, lam, gd, gt);
      lam.ey += gey_prev;
      stage_grad_c8(C, xp, ob.w_S, lam);
      const R gu0 = gd + ob.w_S * C.ctrl_w[0] * v0;
      const R gu1 = gt + ob.w_S * C.ctrl_w[1] * v1;
      const R gv0 = (pass0 ? gu0 : R(0)) + ob.w_S * C.ctrl_w[0] * u0;
      const R gv1 = (pass1 ? gu1 : R(0)) + ob.w_S * C.ctrl_w[1] * u1;
      sink(t, gv0, gv1);
    }
  }
}

template <class R>
__host__ __device__ inline size_t c8_adj_lds_bytes(int /*t_max*/, int seg_len) {
  return (size_t)(seg_len + 1) * 8 * WAVE * sizeof(R);
}

template <class R>
struct C8BackwardArgs {
  C8Args<R> a;
  DevObjective<R> ob;
  const R* grad_S;
  R* grad_V;
  R* part;            // [B][nblk_max][2][t_max]: per-workgroup partials, summed by k_sum_partials
  uint32_t* valid;    // [B]: 1 when the problem's sizes are valid (written by workgroup 0)
  unsigned char* ck;  // [B][nblk_max] blocks of adj_ck_bytes_per_wg(t_max, seg_len, 8): checkpoints
  int nblk_max;
  int seg_len;
};

// grad_V = sum_m grad_S[m] dL_m/dV: one 64-lane workgroup per 64 samples, grid
// (nblk_max, B); each workgroup writes its partial (k_sum_partials adds them).
template <class R>
__global__ __launch_bounds__(WAVE) void k_backward_c8(C8BackwardArgs<R> g) {
  extern __shared__ __align__(16) unsigned char smem[];
  const C8Args<R>& a = g.a;
  const int b = blockIdx.y;
  C8Dims d;
  const bool ok = c8_dims(a, b, d);
  if (blockIdx.x == 0 && threadIdx.x == 0) g.valid[b] = ok ? 1u : 0u;
  if (!ok) return;
  R* gVb = g.grad_V + 2 * (size_t)d.t0;
  if (d.K == 0) {
    if (blockIdx.x == 0)
      for (int i = threadIdx.x; i < 2 * d.T; i += blockDim.x) gVb[i] = R(0);
    return;
  }
  const int nblk = (d.K + WAVE - 1) / WAVE;
  if ((int)blockIdx.x >= nblk) return;
  R* Vs;
  const CurvView<R> cv = c8_stage(a, b, d, reinterpret_cast<R*>(smem), &Vs);
  R* sx = reinterpret_cast<R*>(smem + c8_stage_bytes<R>(a.n_max, a.t_max));
  R* ck = reinterpret_cast<R*>(g.ck + ((size_t)b * g.nblk_max + blockIdx.x) *
                                          adj_ck_bytes_per_wg<R>(a.t_max, g.seg_len, 8, false));
  __syncthreads();
  const int lane = threadIdx.x;
  const int m = blockIdx.x * WAVE + lane;
  NoiseStream<R> ns = c8_noise(a, b, m);
  ReduceSink<R> sink;
  sink.g = (m < d.K) ? g.grad_S[d.k0 + m] : R(0);
  sink.gp = g.part + ((size_t)b * g.nblk_max + blockIdx.x) * 2 * a.t_max;
  sink.T = d.T;
  sink.lane = lane;
  adjoint_lane_c8(a.M, a.Wh, a.C, g.ob, cv, load_c8(a.x0 + 8 * (size_t)b), Vs, d.T, ns, ck, sx, g.seg_len, lane,
                  sink);
}

template <class R>
struct C8RepairArgs {
  C8Args<R> a;
  DevObjective<R> ob;
  const R* V_plus;
  R* V_safe;
  int n_steps;
  R step;
};

// The repair's workgroup: the forward chain runs on one lane, the reverse sweep
// on all threads.
constexpr int C8_REP_BLK = 4 * WAVE;
// Per step of the parallel reverse sweep: the rows [J_t^T | B_t^T] of the RK4
// step's Jacobians for the eight unit cotangents (8 x 10), the barrier gradient
// at x_{t+1} (an e_y value), the local gradient at x_t (v_x and e_y values) and
// the control gradient (2), padded.
constexpr int C8_PAR = 88;

template <class R>
__host__ __device__ inline size_t c8_repair_lds_bytes(int n_max, int t_max) {
  return c8_stage_bytes<R>(n_max, t_max) + sizeof(R) * 8 * ((size_t)t_max + 1) + sizeof(R) * C8_PAR * (size_t)t_max;
}

// Component j of x (selects: no dynamic index into the struct).
template <class R>
__device__ __forceinline__ R c8_comp(const C8<R>& x, int j) {
  R v = x.vx;
  v = j == 1 ? x.vy : v;
  v = j == 2 ? x.r : v;
  v = j == 3 ? x.wF : v;
  v = j == 4 ? x.wR : v;
  v = j == 5 ? x.ep : v;
  v = j == 6 ? x.ey : v;
  v = j == 7 ? x.s : v;
  return v;
}

// Algorithm 1 on the curvilinear model, one workgroup per problem.  Per
// iteration: the nominal trajectory from x0 under clip(V) on one lane (stored in
// LDS), and the last transition whose objective term has a non-zero derivative;
// then the reverse sweep from there.  The adjoint recursion is linear once the
// trajectory is fixed,
//   lam_t = J_t^T (lam_{t+1} + dn_t) + dc_t,   g_t = B_t^T (lam_{t+1} + dn_t),
// so the Jacobian rows (one vector-Jacobian product per unit cotangent) and the
// local gradients of every step are computed in parallel, the recursion runs as
// 8 x 10 matrix-vector products on ten lanes (lam broadcast by readlane), and the
// projected step V <- clip(V - step g) is applied to every step in parallel;
// later steps only get the projection.  Stops early when no transition is
// active (the gradient is then zero).
template <class R>
__global__ __launch_bounds__(C8_REP_BLK) void k_repair_c8(C8RepairArgs<R> r) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int s_last, s_step;
  const C8Args<R>& a = r.a;
  const int b = blockIdx.x;
  C8Dims d;
  if (!c8_dims(a, b, d)) return;
  R* Vs;
  C8Args<R> av = a;
  av.V = r.V_plus;
  const CurvView<R> cv = c8_stage(av, b, d, reinterpret_cast<R*>(smem), &Vs);
  R* xs = reinterpret_cast<R*>(smem + c8_stage_bytes<R>(a.n_max, a.t_max));
  R* Wp = xs + 8 * ((size_t)a.t_max + 1);
  __syncthreads();
  const int T = d.T;
  const DevModel<R>& M = a.M;
  const DevCost<R>& C = a.C;
  const DevObjective<R>& ob = r.ob;
  const bool cost_terms = ob.w_S != R(0);
  const int w = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
  const R h = M.dt, h2 = R(0.5) * M.dt, h6 = M.dt * R(1.0 / 6.0);
  auto comb = [&](R a1, R a2, R a3, R a4, R xv) { return fma_r(h6, fma_r(R(2), a2 + a3, a1) + a4, xv); };
  for (int s = 0; s < r.n_steps; ++s) {
    if (threadIdx.x == 0) {
      store_c8(xs, load_c8(a.x0 + 8 * (size_t)b));
      s_step = 0;
    }
    __syncthreads();
    // nominal trajectory: the body states on one lane of wave 0, publishing each
    // step's stage values of (v_x, v_y, r) ([t][12] in the reverse sweep's
    // buffer, free until then), the path states and the barrier activity on one
    // lane of wave 1 as the steps are published (the classic RK4 of the model,
    // the same operations as rk4_c8)
    if (w == 0 && lane == 0) {
      C8<R> x = load_c8(xs);
      for (int t = 0; t < T; ++t) {
        const R u0 = clamp_r(Vs[t], M.u_lo[0], M.u_hi[0]);
        const R u1 = clamp_r(Vs[T + t], M.u_lo[1], M.u_hi[1]);
        const Ctl8<R> c = ctl8(u0, u1);
        C8<R> k1 = zero8<R>(), k2 = zero8<R>(), k3 = zero8<R>(), k4 = zero8<R>();
        deriv_c8_body(M, a.Wh, c, x, k1);
        const C8<R> X2 = axpy8(h2, k1, x);
        deriv_c8_body(M, a.Wh, c, X2, k2);
        const C8<R> X3 = axpy8(h2, k2, x);
        deriv_c8_body(M, a.Wh, c, X3, k3);
        const C8<R> X4 = axpy8(h, k3, x);
        deriv_c8_body(M, a.Wh, c, X4, k4);
        R* g = Wp + 12 * (size_t)t;
        g[0] = x.vx; g[1] = X2.vx; g[2] = X3.vx; g[3] = X4.vx;
        g[4] = x.vy; g[5] = X2.vy; g[6] = X3.vy; g[7] = X4.vy;
        g[8] = x.r;  g[9] = X2.r;  g[10] = X3.r; g[11] = X4.r;
        x.vx = comb(k1.vx, k2.vx, k3.vx, k4.vx, x.vx);
        x.vy = comb(k1.vy, k2.vy, k3.vy, k4.vy, x.vy);
        x.r = comb(k1.r, k2.r, k3.r, k4.r, x.r);
        x.wF = comb(k1.wF, k2.wF, k3.wF, k4.wF, x.wF);
        x.wR = comb(k1.wR, k2.wR, k3.wR, k4.wR, x.wR);
        R* o = xs + 8 * (t + 1);
        o[0] = x.vx; o[1] = x.vy; o[2] = x.r; o[3] = x.wF; o[4] = x.wR;
        wave_publish(&s_step, t + 1);
        // the next step's chain starts after the counter store
        asm volatile("" : "+v"(x.vx), "+v"(x.vy), "+v"(x.r), "+v"(x.wF), "+v"(x.wR)::"memory");
      }
    } else if (w == 1 && lane == 0) {
      C8<R> x = load_c8(xs);
      int last = -1, seen = 0;
      R hp = cv.w2 - x.ey * x.ey;
      for (int t = 0; t < T; ++t) {
        wave_wait(&s_step, t, seen, a.err);
        const R* g = Wp + 12 * (size_t)t;
        C8<R> k1 = zero8<R>(), k2 = zero8<R>(), k3 = zero8<R>(), k4 = zero8<R>();
        C8<R> X = x;
        X.vx = g[0]; X.vy = g[4]; X.r = g[8];
        deriv_c8_path(cv, X, k1);
        X.vx = g[1]; X.vy = g[5]; X.r = g[9];
        X.ep = fma_r(h2, k1.ep, x.ep); X.ey = fma_r(h2, k1.ey, x.ey); X.s = fma_r(h2, k1.s, x.s);
        deriv_c8_path(cv, X, k2);
        X.vx = g[2]; X.vy = g[6]; X.r = g[10];
        X.ep = fma_r(h2, k2.ep, x.ep); X.ey = fma_r(h2, k2.ey, x.ey); X.s = fma_r(h2, k2.s, x.s);
        deriv_c8_path(cv, X, k3);
        X.vx = g[3]; X.vy = g[7]; X.r = g[11];
        X.ep = fma_r(h, k3.ep, x.ep); X.ey = fma_r(h, k3.ey, x.ey); X.s = fma_r(h, k3.s, x.s);
        deriv_c8_path(cv, X, k4);
        x.ep = comb(k1.ep, k2.ep, k3.ep, k4.ep, x.ep);
        x.ey = comb(k1.ey, k2.ey, k3.ey, k4.ey, x.ey);
        x.s = comb(k1.s, k2.s, k3.s, k4.s, x.s);
        R* o = xs + 8 * (t + 1);
        o[5] = x.ep; o[6] = x.ey; o[7] = x.s;
        const R hn = cv.w2 - x.ey * x.ey;
        if (dcbf_active(C.alpha, hp, hn) && (ob.w_sq != R(0) || (ob.w_lin != R(0) && t < ob.n_lin))) last = t;
        hp = hn;
      }
      s_last = last;
    }
    __syncthreads();
    const int t_end = cost_terms ? T - 1 : s_last;
    for (int t = t_end + 1 + (int)threadIdx.x; t < T; t += blockDim.x) {
      Vs[t] = clamp_r(Vs[t], M.u_lo[0], M.u_hi[0]);
      Vs[T + t] = clamp_r(Vs[T + t], M.u_lo[1], M.u_hi[1]);
    }
    if (t_end < 0) break;  // uniform: every thread read the same s_last
    // Jacobian rows and local gradients of every step
    for (int k = threadIdx.x; k < 8 * (t_end + 1); k += blockDim.x) {
      const int t = k >> 3, i = k & 7;
      const C8<R> xp = load_c8(xs + 8 * t);
      const R u0 = clamp_r(Vs[t], M.u_lo[0], M.u_hi[0]);
      const R u1 = clamp_r(Vs[T + t], M.u_lo[1], M.u_hi[1]);
      C8<R> lam = zero8<R>();
      lam.vx = i == 0 ? R(1) : R(0);
      lam.vy = i == 1 ? R(1) : R(0);
      lam.r = i == 2 ? R(1) : R(0);
      lam.wF = i == 3 ? R(1) : R(0);
      lam.wR = i == 4 ? R(1) : R(0);
      lam.ep = i == 5 ? R(1) : R(0);
      lam.ey = i == 6 ? R(1) : R(0);
      lam.s = i == 7 ? R(1) : R(0);
      R gd = R(0), gt = R(0);
      rk4_c8_vjp(M, a.Wh, cv, ctl8(u0, u1), xp, lam, gd, gt);
      R* q = Wp + (size_t)C8_PAR * t + 10 * i;
      store_c8(q, lam);
      q[8] = gd;
      q[9] = gt;
      if (i == 0) {
        const C8<R> xn = load_c8(xs + 8 * (t + 1));
        C8<R> dn = zero8<R>(), dc = zero8<R>();
        dc.ey = penalty_grad_c8(C, ob, cv.w2, xp, xn, t, dn);
        if (cost_terms) stage_grad_c8(C, xp, ob.w_S, dc);
        R* qq = Wp + (size_t)C8_PAR * t;
        qq[80] = dn.ey;
        qq[81] = dc.vx;
        qq[82] = dc.ey;
      }
    }
    __syncthreads();
    if (threadIdx.x < WAVE) {
      // lane j < 10 holds component j: lam_j for j < 8, the control gradient for j = 8, 9
      const int j = threadIdx.x < 10 ? (int)threadIdx.x : 9;
      R lam = R(0);
      if (cost_terms) {
        C8<R> l = zero8<R>();
        stage_grad_c8(C, load_c8(xs + 8 * T), ob.w_S * C.phi_w, l);
        lam = j < 8 ? c8_comp(l, j) : R(0);
      }
      for (int t = t_end; t >= 0; --t) {
        const R* q = Wp + (size_t)C8_PAR * t;
        if (j == 6) lam += q[80];
        R l[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) l[i] = lane_bcast(lam, i);
        const R nl = ((l[0] * q[j] + l[1] * q[10 + j]) + (l[2] * q[20 + j] + l[3] * q[30 + j])) +
                     ((l[4] * q[40 + j] + l[5] * q[50 + j]) + (l[6] * q[60 + j] + l[7] * q[70 + j]));
        if (j < 8)
          lam = nl + (j == 0 ? q[81] : (j == 6 ? q[82] : R(0)));
        else if (threadIdx.x < 10)
          Wp[(size_t)C8_PAR * t + 83 + (j - 8)] = nl;
      }
    }
    __syncthreads();
    for (int t = threadIdx.x; t <= t_end; t += blockDim.x) {
      const R* g = Wp + (size_t)C8_PAR * t + 83;
      const R v0 = Vs[t], v1 = Vs[T + t];
      const R u0 = clamp_r(v0, M.u_lo[0], M.u_hi[0]);
      const R u1 = clamp_r(v1, M.u_lo[1], M.u_hi[1]);
      const bool pass0 = (v0 >= M.u_lo[0]) && (v0 <= M.u_hi[0]);
      const bool pass1 = (v1 >= M.u_lo[1]) && (v1 <= M.u_hi[1]);
      const R gu0 = g[0] + ob.w_S * C.ctrl_w[0] * v0;
      const R gu1 = g[1] + ob.w_S * C.ctrl_w[1] * v1;
      const R gv0 = (pass0 ? gu0 : R(0)) + ob.w_S * C.ctrl_w[0] * u0;
      const R gv1 = (pass1 ? gu1 : R(0)) + ob.w_S * C.ctrl_w[1] * u1;
      Vs[t] = clamp_r(v0 - r.step * gv0, M.u_lo[0], M.u_hi[0]);
      Vs[T + t] = clamp_r(v1 - r.step * gv1, M.u_lo[1], M.u_hi[1]);
    }
    __syncthreads();
  }
  __syncthreads();
  R* out = r.V_safe + 2 * (size_t)d.t0;
  for (int i = threadIdx.x; i < 2 * T; i += blockDim.x) out[i] = Vs[i];
}

template <class R>
struct C8ExecArgs {
  C8Args<R> a;
  const R* V_exec;
  const R* V_plus;
  const R* dist;  // [n_dist][B][2] on (v_y, r), or null
  int32_t n_dist;
  R* x;           // [B][8], advanced in place
  R* V;           // warm start out
  uint32_t* iter;
};

// Plant step and warm start (Algorithm 2, last two lines): x <- RK4(x, clip(v_0))
// + disturbance on (v_y, r); V <- V+ shifted one step, last step repeated.
template <class R>
__global__ __launch_bounds__(WAVE) void k_execute_c8(C8ExecArgs<R> e) {
  extern __shared__ __align__(16) unsigned char smem[];
  const C8Args<R>& a = e.a;
  const int b = blockIdx.x;
  const int t0 = a.t_off[b], T = a.t_off[b + 1] - t0;
  const int c0 = a.kappa_off[b], n = a.kappa_off[b + 1] - c0;
  if (T < 1 || T > a.t_max || n < 2 || n > a.n_max) {
    if (threadIdx.x == 0) atomicOr(a.err, (T < 1 || T > a.t_max) ? DERR_T : DERR_POLY);
    return;
  }
  R* buf = reinterpret_cast<R*>(smem);
  const R* Vp = e.V_plus + 2 * (size_t)t0;
  for (int i = threadIdx.x; i < 2 * T; i += blockDim.x) buf[i] = Vp[i];
  __syncthreads();
  if (threadIdx.x == 0) {
    const CurvView<R> cv = curv_view(a.kappa + c0, n, a.ds[b], R(0));
    const R* Ve = e.V_exec + 2 * (size_t)t0;
    const R u0 = clamp_r(Ve[0], a.M.u_lo[0], a.M.u_hi[0]);
    const R u1 = clamp_r(Ve[T], a.M.u_lo[1], a.M.u_hi[1]);
    C8<R> x = load_c8(e.x + 8 * (size_t)b);
    rk4_c8(a.M, a.Wh, cv, ctl8(u0, u1), x);
    const uint32_t it = e.iter[b];
    if (e.dist && (int64_t)it < (int64_t)e.n_dist) {
      x.vy += e.dist[2 * ((size_t)it * a.B + b)];
      x.r += e.dist[2 * ((size_t)it * a.B + b) + 1];
    }
    store_c8(e.x + 8 * (size_t)b, x);
    e.iter[b] = it + 1u;
  }
  R* Vo = e.V + 2 * (size_t)t0;
  for (int i = threadIdx.x; i < 2 * T; i += blockDim.x) {
    const int dd = i / T, t = i % T;
    Vo[i] = buf[dd * T + min(t + 1, T - 1)];
  }
}

}  // namespace smppi
