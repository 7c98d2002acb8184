// Shield-MPPI sampled-rollout oracle: plain, slow, FP64, scalar C++17.
//
// TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes or
// calls this file; only the test suite, the smoke check and the CPU-baseline
// leg of the benchmark load it.  It shares no source, header or generated table
// with the GPU path: the only thing both sides consume in common is input data
// (track polyline, obstacles, initial states, disturbances) produced by the
// seeded workload generator, and the published definition of Philox4x32-10.
//
// Paper: Yin, Dawson, Fan, Tsiotras, "Shield Model Predictive Path Integral:
// A Computationally Efficient Robust MPC Method Using Control Barrier
// Functions" (arXiv 2302.11719).  Notation: K samples, T horizon steps (the
// paper writes M samples and horizon K).  Every function below cites the
// passage it follows.  Where the paper is silent or garbled, the reading taken
// is stated in one line where it is applied.
//
// Built with: g++ -O2 -std=c++17 -ffp-contract=off -fPIC -shared (no SIMD
// intrinsics, no fast-math), so every expression rounds as written.

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <thread>
#include <vector>

namespace {

// ---------------------------------------------------------------------------
// Forward-mode dual numbers (value + one tangent).  Used only to obtain an
// exact gradient of the rollout objective, independent of any hand-derived
// adjoint.  Discrete decisions (clamps, hinges, argmins) compare values.
// ---------------------------------------------------------------------------
struct Dual {
  double v, d;
  Dual(double a = 0.0, double b = 0.0) : v(a), d(b) {}
};
inline Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
inline Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
inline Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
inline Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
inline Dual operator/(Dual a, Dual b) {
  return Dual(a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v));
}
inline Dual& operator+=(Dual& a, Dual b) { a = a + b; return a; }
inline Dual sin(Dual a) { return Dual(std::sin(a.v), std::cos(a.v) * a.d); }
inline Dual cos(Dual a) { return Dual(std::cos(a.v), -std::sin(a.v) * a.d); }
inline Dual sqrt(Dual a) {
  double s = std::sqrt(a.v);
  return Dual(s, a.d / (2.0 * s));
}
inline double val(double a) { return a; }
inline double val(Dual a) { return a.v; }
using std::cos;
using std::sin;
using std::sqrt;

template <class R> inline R rmax(R a, R b) { return val(a) >= val(b) ? a : b; }
template <class R> inline R clampr(R x, double lo, double hi) {
  if (val(x) < lo) return R(lo);
  if (val(x) > hi) return R(hi);
  return x;
}

// ---------------------------------------------------------------------------
// Philox4x32-10 counter-based generator, from its published definition
// (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3",
// SC'11): 10 rounds of two 32x32->64 multiplies with the Weyl key schedule.
// ---------------------------------------------------------------------------
void philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; ++r) {
    uint64_t p0 = (uint64_t)M0 * (uint64_t)c0;
    uint64_t p1 = (uint64_t)M1 * (uint64_t)c2;
    uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    uint32_t n1 = (uint32_t)p1;
    uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    uint32_t n3 = (uint32_t)p0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    k0 += W0;
    k1 += W1;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

// Uniform on (0, 1]: top 24 bits plus one, times 2^-24 (exact in FP32/FP64,
// never zero, so the logarithm below is finite).
double uniform01(uint32_t x) { return ((double)(x >> 8) + 1.0) * (1.0 / 16777216.0); }

// Box-Muller transform (Box and Muller 1958): two uniforms -> two standard normals.
void box_muller(uint32_t xa, uint32_t xb, double* z0, double* z1) {
  const double two_pi = 6.283185307179586476925286766559;
  double r = std::sqrt(-2.0 * std::log(uniform01(xa)));
  double ang = two_pi * uniform01(xb);
  *z0 = r * std::cos(ang);
  *z1 = r * std::sin(ang);
}

// Control noise of sample m at step t (Section II: u_k ~ N(v_k, Sigma_eps) with
// diagonal Sigma_eps; Algorithm 2 samples one noise sequence per trajectory).
// Counter (t/2, m, problem id, iteration), key (seed, stream 0).  Words 0,1
// give step 2j, words 2,3 give step 2j+1; first normal steers, second throttles.
void step_normals(uint32_t seed, uint32_t pid, uint32_t it, uint32_t m, int t, double z[2]) {
  uint32_t ctr[4] = {(uint32_t)(t >> 1), m, pid, it};
  uint32_t key[2] = {seed, 0u};
  uint32_t w[4];
  philox4x32_10(ctr, key, w);
  if ((t & 1) == 0) box_muller(w[0], w[1], &z[0], &z[1]);
  else              box_muller(w[2], w[3], &z[0], &z[1]);
}

// ---------------------------------------------------------------------------
// Parameters (flattened double arrays so that the Python wrapper needs no
// struct layout).  Model: six-state dynamic single-track vehicle with linear
// tyres (the paper's eq. (1) system f; the paper's own vehicle is a calibrated
// eight-state model whose constants it does not print).
// ---------------------------------------------------------------------------
struct Model {
  double m, lf, lr, Iz, Cf, Cr, a_max, c_v, v_min, dt;
  double u_lo[2], u_hi[2];
};
enum { MODEL_NPARAM = 14 };
Model model_from(const double* p) {
  Model M;
  M.m = p[0]; M.lf = p[1]; M.lr = p[2]; M.Iz = p[3]; M.Cf = p[4]; M.Cr = p[5];
  M.a_max = p[6]; M.c_v = p[7]; M.v_min = p[8]; M.dt = p[9];
  M.u_lo[0] = p[10]; M.u_lo[1] = p[11]; M.u_hi[0] = p[12]; M.u_hi[1] = p[13];
  return M;
}

// Cost: running cost of eq. (24) on (v_x, e_y) with collision indicator eq.
// (25); control term of eq. (8)/Algorithm 2; DCBF penalty eq. (17)-(20) with
// alpha = 1 - beta (beta is the class-kappa slope of eq. (15)).
struct Cost {
  double v_g, q_v, q_ey, C_obs, phi_w, lambda_u, sigma[2], C_cbf, beta;
};
enum { COST_NPARAM = 10 };
Cost cost_from(const double* p) {
  Cost C;
  C.v_g = p[0]; C.q_v = p[1]; C.q_ey = p[2]; C.C_obs = p[3]; C.phi_w = p[4];
  C.lambda_u = p[5]; C.sigma[0] = p[6]; C.sigma[1] = p[7]; C.C_cbf = p[8]; C.beta = p[9];
  return C;
}

// Track: either a circle (centre, radius) or a closed polyline of n segments,
// segment i from (ax, ay) along (dx, dy), with 1/|d|^2 given; half width w;
// optional circular obstacles (cx, cy, inflated radius^2, radius^2).
struct Track {
  int kind;  // 0 circle, 1 polyline
  double cx, cy, R;
  const double* poly;  // [n][5]: ax, ay, dx, dy, inv_len2
  int n;
  double w;
  const double* obs;  // [n_obs][4]: cx, cy, r_eff^2, r^2
  int n_obs;
  int window;
};

// ---------------------------------------------------------------------------
// Dynamics f(x, u) (eq. (1)); x = (px, py, psi, vx, vy, omega), u = (steer, throttle).
// Classic linear single-track model: slip angles from body velocities, lateral
// tyre forces linear in slip, longitudinal drive a_max*throttle minus linear drag.
// ---------------------------------------------------------------------------
template <class R>
void deriv(const Model& M, const R x[6], const R u[2], R dx[6]) {
  R psi = x[2], vx = x[3], vy = x[4], om = x[5];
  R delta = u[0], tau = u[1];
  R vt = rmax(vx, R(M.v_min));
  R alpha_f = delta - (vy + R(M.lf) * om) / vt;
  R alpha_r = R(0.0) - (vy - R(M.lr) * om) / vt;
  R Fyf = R(M.Cf) * alpha_f;
  R Fyr = R(M.Cr) * alpha_r;
  R c = cos(psi), s = sin(psi);
  R cd = cos(delta), sd = sin(delta);
  dx[0] = vx * c - vy * s;
  dx[1] = vx * s + vy * c;
  dx[2] = om;
  dx[3] = R(M.a_max) * tau - R(M.c_v) * vx - Fyf * sd / R(M.m) + vy * om;
  dx[4] = (Fyf * cd + Fyr) / R(M.m) - vx * om;
  dx[5] = (R(M.lf) * Fyf * cd - R(M.lr) * Fyr) / R(M.Iz);
}

// Classic fourth-order Runge-Kutta step of length dt with the control held.
template <class R>
void rk4_step(const Model& M, const R x[6], const R u[2], double dt, R out[6]) {
  R k1[6], k2[6], k3[6], k4[6], xs[6];
  deriv(M, x, u, k1);
  for (int i = 0; i < 6; ++i) xs[i] = x[i] + R(0.5 * dt) * k1[i];
  deriv(M, xs, u, k2);
  for (int i = 0; i < 6; ++i) xs[i] = x[i] + R(0.5 * dt) * k2[i];
  deriv(M, xs, u, k3);
  for (int i = 0; i < 6; ++i) xs[i] = x[i] + R(dt) * k3[i];
  deriv(M, xs, u, k4);
  for (int i = 0; i < 6; ++i)
    out[i] = x[i] + R(dt / 6.0) * (k1[i] + R(2.0) * k2[i] + R(2.0) * k3[i] + k4[i]);
}

// ---------------------------------------------------------------------------
// Lateral deviation e_y^2 from the centreline (the quantity in eq. (23)).
// ---------------------------------------------------------------------------
template <class R>
R seg_dist2(const Track& tr, int i, R px, R py) {
  const double* s = tr.poly + 5 * i;
  R rx = px - R(s[0]), ry = py - R(s[1]);
  R lam = (rx * R(s[2]) + ry * R(s[3])) * R(s[4]);
  lam = clampr(lam, 0.0, 1.0);
  R ex = rx - lam * R(s[2]), ey = ry - lam * R(s[3]);
  return ex * ex + ey * ey;
}

// Global nearest segment; ties go to the lowest index.
int global_argmin(const Track& tr, double px, double py) {
  int best = 0;
  double bd = seg_dist2<double>(tr, 0, px, py);
  for (int i = 1; i < tr.n; ++i) {
    double d = seg_dist2<double>(tr, i, px, py);
    if (d < bd) { bd = d; best = i; }
  }
  return best;
}

// Windowed nearest segment around the previous index: offsets visited in the
// order 0, -1, +1, -2, +2, ...; the first strict minimum wins ties.
int window_argmin(const Track& tr, int prev, double px, double py) {
  int best = prev;
  double bd = seg_dist2<double>(tr, prev, px, py);
  for (int k = 1; k <= tr.window; ++k) {
    for (int sgn = -1; sgn <= 1; sgn += 2) {
      int i = ((prev + sgn * k) % tr.n + tr.n) % tr.n;
      double d = seg_dist2<double>(tr, i, px, py);
      if (d < bd) { bd = d; best = i; }
    }
  }
  return best;
}

// e_y^2 at (px, py); for the polyline, *idx carries the window centre in and
// the chosen segment out (*idx < 0 requests the global search, used at x_0).
template <class R>
R lateral_sq(const Track& tr, R px, R py, int* idx) {
  if (tr.kind == 0) {
    R dx = px - R(tr.cx), dy = py - R(tr.cy);
    R e = sqrt(dx * dx + dy * dy) - R(tr.R);
    return e * e;
  }
  int i = (*idx < 0) ? global_argmin(tr, val(px), val(py)) : window_argmin(tr, *idx, val(px), val(py));
  *idx = i;
  return seg_dist2<R>(tr, i, px, py);
}

// All barrier values at one state: h_0 = w^2 - e_y^2 (eq. (23)), then
// h_i = |p - c_i|^2 - r_eff_i^2 for each obstacle.  Also reports whether the
// state is inside the track and clear of every obstacle (eq. (25)), and the
// smallest distance of any indicator test from its switching point.
template <class R>
void barriers(const Track& tr, const R x[6], int* idx, R* h, R* ey2, bool* inside, double* margin) {
  R e2 = lateral_sq<R>(tr, x[0], x[1], idx);
  *ey2 = e2;
  h[0] = R(tr.w * tr.w) - e2;
  bool in = val(h[0]) >= 0.0;
  double mg = std::fabs(val(h[0]));
  for (int i = 0; i < tr.n_obs; ++i) {
    const double* o = tr.obs + 4 * i;
    R ddx = x[0] - R(o[0]), ddy = x[1] - R(o[1]);
    R d2 = ddx * ddx + ddy * ddy;
    h[1 + i] = d2 - R(o[2]);
    double gap = val(d2) - o[3];
    if (gap < 0.0) in = false;
    mg = std::min(mg, std::fabs(gap));
  }
  *inside = in;
  *margin = mg;
}

// Running cost q(x) of eq. (24) restricted to the states this model has
// (target speed v_g and lateral deviation), plus C_obs outside the safe region
// (eq. (25)).  The indicator is dropped (with_indicator = false) when the cost
// is differentiated: it is piecewise constant.
template <class R>
R stage_cost(const Cost& C, const R x[6], R ey2, bool inside, bool with_indicator) {
  R dv = x[3] - R(C.v_g);
  R q = R(C.q_v) * dv * dv + R(C.q_ey) * ey2;
  if (with_indicator && !inside) q = q + R(C.C_obs);
  return q;
}

// ---------------------------------------------------------------------------
// One sampled trajectory (Algorithm 2, inner loop; eqs. (8), (12), (17)-(20)).
// Returns the modified cost S~ and, through `obj`, the objective used for
// differentiation:
//   w_S * (S~ without the indicator) + w_sq * sum viol^2 + w_lin * sum_{t<N} viol
// with viol_{j,t} = max(alpha h_j(x_t) - h_j(x_{t+1}), 0).
// ---------------------------------------------------------------------------
struct Objective {
  double w_S, w_sq, w_lin;
  int n_lin;
};

struct SampleOut {
  double S;        // modified trajectory cost S~ (with indicator)
  double margin;   // smallest indicator margin along the trajectory
  uint64_t sig;    // hash of every discrete decision (kink detector)
};

inline uint64_t mix(uint64_t h, uint64_t v) {
  h ^= v + 0x9E3779B97F4A7C15ull + (h << 6) + (h >> 2);
  return h;
}

template <class R>
R rollout_one(const Model& M, const Cost& C, const Track& tr, const double x0[6],
              const R* V, int T, const double* eps,  // eps: [T][2] raw noise sigma*z (or null = zero)
              double* eps_eff,                        // out: [T][2] clip(v+eps)-v (nullable)
              const Objective* ob, R* obj_out, SampleOut* so) {
  const double alpha = 1.0 - C.beta;
  const int nb = 1 + tr.n_obs;
  std::vector<R> h_prev(nb), h_cur(nb);
  R x[6];
  for (int i = 0; i < 6; ++i) x[i] = R(x0[i]);
  int idx = -1;
  R ey2;
  bool inside;
  double mg, margin = 1e300;
  uint64_t sig = 0;
  barriers<R>(tr, x, &idx, h_cur.data(), &ey2, &inside, &mg);
  margin = std::min(margin, mg);
  sig = mix(sig, (uint64_t)idx);
  // z_0 = (x_0, x_0): the paper sets x_{-1} = x_0 (text after eq. (20)).
  for (int j = 0; j < nb; ++j) h_prev[j] = h_cur[j];

  R S = R(0.0), S_noind = R(0.0), obj_extra = R(0.0);
  for (int t = 0; t <= T; ++t) {
    // C_cbf(z_t) = C max(-h(x_t) + alpha h(x_{t-1}), 0), eq. (17)/(19), summed over barriers.
    R pen = R(0.0);
    for (int j = 0; j < nb; ++j) {
      R r = R(alpha) * h_prev[j] - h_cur[j];
      bool act = val(r) > 0.0;
      sig = mix(sig, act);
      if (act) {
        pen = pen + R(C.C_cbf) * r;
        if (t >= 1) {  // violations of the transitions x_{t-1} -> x_t
          obj_extra = obj_extra + R(ob ? ob->w_sq : 0.0) * r * r;
          if (ob && t - 1 < ob->n_lin) obj_extra = obj_extra + R(ob->w_lin) * r;
        }
      }
    }
    if (t < T) {
      // u_t = v_t + eps_t, held inside the control box.
      R u[2], ctrl = R(0.0);
      for (int d = 0; d < 2; ++d) {
        R v = V[2 * t + d];
        R raw = v + R(eps ? eps[2 * t + d] : 0.0);
        bool lo = val(raw) < M.u_lo[d], hi = val(raw) > M.u_hi[d];
        sig = mix(sig, (uint64_t)(lo + 2 * hi));
        u[d] = clampr(raw, M.u_lo[d], M.u_hi[d]);
        if (eps_eff) eps_eff[2 * t + d] = val(u[d]) - val(v);
        // lambda v^T Sigma^{-1} u, diagonal Sigma (eq. (8), Algorithm 2).
        ctrl = ctrl + R(C.lambda_u) * v * u[d] / R(C.sigma[d] * C.sigma[d]);
      }
      R qv = stage_cost<R>(C, x, ey2, inside, true);
      R qn = stage_cost<R>(C, x, ey2, inside, false);
      S = S + (qv + ctrl + pen);
      S_noind = S_noind + (qn + ctrl + pen);
      sig = mix(sig, val(x[3]) > M.v_min);
      R xn[6];
      rk4_step<R>(M, x, u, M.dt, xn);
      for (int i = 0; i < 6; ++i) x[i] = xn[i];
      for (int j = 0; j < nb; ++j) h_prev[j] = h_cur[j];
      barriers<R>(tr, x, &idx, h_cur.data(), &ey2, &inside, &mg);
      margin = std::min(margin, mg);
      sig = mix(sig, (uint64_t)idx);
    } else {
      // Terminal cost phi = phi_w * q (the paper prints no phi; reading: phi = q).
      R qv = stage_cost<R>(C, x, ey2, inside, true);
      R qn = stage_cost<R>(C, x, ey2, inside, false);
      S = S + (R(C.phi_w) * qv + pen);
      S_noind = S_noind + (R(C.phi_w) * qn + pen);
    }
  }
  if (so) { so->S = val(S); so->margin = margin; so->sig = sig; }
  if (obj_out) *obj_out = R(ob ? ob->w_S : 0.0) * S_noind + obj_extra;
  return S;
}

// ---------------------------------------------------------------------------
// Curvilinear eight-state model (Sec. VI-A): the vehicle's state is
// x = (v_x, v_y, r, omega_F, omega_R, e_psi, e_y, s) -- body velocities, yaw
// rate, front and rear wheel speeds, heading error, lateral deviation and
// progress along the centre line -- and the track barrier of eq. (23),
// h = w^2 - e_y^2, is read from the state.  The paper names these states and a
// single-track bicycle model but prints neither equations nor constants.  The
// reading taken here:
//  - lateral tyre forces as in the six-state model, linear in slip angle;
//  - longitudinal tyre forces linear in wheel slip,
//      F_x = C_x (r_w omega - v_w) / v~,   v~ = max(v_x, v_min),
//    v_w the wheel centre's speed along its rolling direction (front:
//    v_x cos(delta) + (v_y + l_f r) sin(delta); rear: v_x);
//  - the throttle drives the rear axle with torque m a_max r_w T, so that with
//    both wheels at their equilibrium speeds (F_xF = 0, F_xR = m a_max T) the
//    body equations are exactly the six-state model's:
//      I_w omega_F' = -r_w F_xF,   I_w omega_R' = m a_max r_w T - r_w F_xR;
//  - body equations with the front axle's forces rotated by the steering angle:
//      v_x' = (F_xR + F_xF cos(delta) - F_yF sin(delta)) / m - c_v v_x + v_y r,
//      v_y' = (F_yR + F_xF sin(delta) + F_yF cos(delta)) / m - v_x r,
//      r'   = (l_f (F_xF sin(delta) + F_yF cos(delta)) - l_r F_yR) / I_z;
//  - Frenet kinematics along a path of curvature kappa(s):
//      s' = (v_x cos(e_psi) - v_y sin(e_psi)) / (1 - kappa(s) e_y),
//      e_y' = v_x sin(e_psi) + v_y cos(e_psi),   e_psi' = r - kappa(s) s'.
// kappa(s): periodic table on a uniform grid s_j = j ds, linear in between.
// ---------------------------------------------------------------------------
struct Wheels {
  double r_w, I_w, C_x;
};
Wheels wheels_from(const double* p) { return Wheels{p[0], p[1], p[2]}; }

struct CurvTrack {
  const double* kappa;
  int n;
  double ds, w;
};

template <class R>
R kappa_at(const CurvTrack& ct, R s) {
  const double jf = std::floor(val(s) / ct.ds);
  R f = s / R(ct.ds) - R(jf);
  long j = (long)jf;
  long j0 = ((j % ct.n) + ct.n) % ct.n, j1 = (j0 + 1) % ct.n;
  return R(ct.kappa[j0]) * (R(1.0) - f) + R(ct.kappa[j1]) * f;
}

template <class R>
void deriv_c8(const Model& M, const Wheels& Wh, const CurvTrack& ct, const R x[8], const R u[2], R dx[8]) {
  R vx = x[0], vy = x[1], r = x[2], wF = x[3], wR = x[4], epsi = x[5], ey = x[6], s = x[7];
  R delta = u[0], thr = u[1];
  R vt = rmax(vx, R(M.v_min));
  R cd = cos(delta), sd = sin(delta);
  R FyF = R(M.Cf) * (delta - (vy + R(M.lf) * r) / vt);
  R FyR = R(M.Cr) * ((R(M.lr) * r - vy) / vt);
  R vwF = vx * cd + (vy + R(M.lf) * r) * sd;
  R FxF = R(Wh.C_x) * (R(Wh.r_w) * wF - vwF) / vt;
  R FxR = R(Wh.C_x) * (R(Wh.r_w) * wR - vx) / vt;
  R k = kappa_at<R>(ct, s);
  R ce = cos(epsi), se = sin(epsi);
  R sdot = (vx * ce - vy * se) / (R(1.0) - k * ey);
  dx[0] = (FxR + FxF * cd - FyF * sd) / R(M.m) - R(M.c_v) * vx + vy * r;
  dx[1] = (FyR + FxF * sd + FyF * cd) / R(M.m) - vx * r;
  dx[2] = (R(M.lf) * (FxF * sd + FyF * cd) - R(M.lr) * FyR) / R(M.Iz);
  dx[3] = R(0.0) - R(Wh.r_w) * FxF / R(Wh.I_w);
  dx[4] = (R(M.m * M.a_max * Wh.r_w) * thr - R(Wh.r_w) * FxR) / R(Wh.I_w);
  dx[5] = r - k * sdot;
  dx[6] = vx * se + vy * ce;
  dx[7] = sdot;
}

template <class R>
void rk4_step_c8(const Model& M, const Wheels& Wh, const CurvTrack& ct, const R x[8], const R u[2], double dt,
                 R out[8]) {
  R k1[8], k2[8], k3[8], k4[8], xs[8];
  deriv_c8(M, Wh, ct, x, u, k1);
  for (int i = 0; i < 8; ++i) xs[i] = x[i] + R(0.5 * dt) * k1[i];
  deriv_c8(M, Wh, ct, xs, u, k2);
  for (int i = 0; i < 8; ++i) xs[i] = x[i] + R(0.5 * dt) * k2[i];
  deriv_c8(M, Wh, ct, xs, u, k3);
  for (int i = 0; i < 8; ++i) xs[i] = x[i] + R(dt) * k3[i];
  deriv_c8(M, Wh, ct, xs, u, k4);
  for (int i = 0; i < 8; ++i)
    out[i] = x[i] + R(dt / 6.0) * (k1[i] + R(2.0) * k2[i] + R(2.0) * k3[i] + k4[i]);
}

// One sampled trajectory of the curvilinear model (Algorithm 2 inner loop):
// S~ with the running cost of eq. (24) on (v_x, e_y), the indicator of eq. (25)
// for |e_y| > w, the control term and the DCBF penalty of eqs. (17)-(20) on the
// track barrier (z_0 term included), as rollout_one; the objective for
// differentiation likewise.
template <class R>
R rollout_one_c8(const Model& M, const Wheels& Wh, const Cost& C, const CurvTrack& ct, const double x0[8],
                 const R* V, int T, const double* eps, double* eps_eff, const Objective* ob, R* obj_out,
                 SampleOut* so) {
  const double alpha = 1.0 - C.beta;
  R x[8];
  for (int i = 0; i < 8; ++i) x[i] = R(x0[i]);
  R h_cur = R(ct.w * ct.w) - x[6] * x[6], h_prev = h_cur;
  double margin = std::fabs(val(h_cur));
  uint64_t sig = 0;
  R S = R(0.0), S_noind = R(0.0), obj_extra = R(0.0);
  for (int t = 0; t <= T; ++t) {
    R pen = R(0.0);
    R rr = R(alpha) * h_prev - h_cur;
    bool act = val(rr) > 0.0;
    sig = mix(sig, act);
    if (act) {
      pen = R(C.C_cbf) * rr;
      if (t >= 1) {
        obj_extra = obj_extra + R(ob ? ob->w_sq : 0.0) * rr * rr;
        if (ob && t - 1 < ob->n_lin) obj_extra = obj_extra + R(ob->w_lin) * rr;
      }
    }
    const bool inside = val(h_cur) >= 0.0;
    R dv = x[0] - R(C.v_g);
    R qn = R(C.q_v) * dv * dv + R(C.q_ey) * x[6] * x[6];
    R qv = inside ? qn : qn + R(C.C_obs);
    if (t < T) {
      R u[2], ctrl = R(0.0);
      for (int d = 0; d < 2; ++d) {
        R v = V[2 * t + d];
        R raw = v + R(eps ? eps[2 * t + d] : 0.0);
        bool lo = val(raw) < M.u_lo[d], hi = val(raw) > M.u_hi[d];
        sig = mix(sig, (uint64_t)(lo + 2 * hi));
        u[d] = clampr(raw, M.u_lo[d], M.u_hi[d]);
        if (eps_eff) eps_eff[2 * t + d] = val(u[d]) - val(v);
        ctrl = ctrl + R(C.lambda_u) * v * u[d] / R(C.sigma[d] * C.sigma[d]);
      }
      S = S + (qv + ctrl + pen);
      S_noind = S_noind + (qn + ctrl + pen);
      sig = mix(sig, val(x[0]) > M.v_min);
      sig = mix(sig, (uint64_t)(int64_t)std::floor(val(x[7]) / ct.ds));
      R xn[8];
      rk4_step_c8<R>(M, Wh, ct, x, u, M.dt, xn);
      for (int i = 0; i < 8; ++i) x[i] = xn[i];
      h_prev = h_cur;
      h_cur = R(ct.w * ct.w) - x[6] * x[6];
      margin = std::min(margin, std::fabs(val(h_cur)));
    } else {
      S = S + (R(C.phi_w) * qv + pen);
      S_noind = S_noind + (R(C.phi_w) * qn + pen);
    }
  }
  if (so) { so->S = val(S); so->margin = margin; so->sig = sig; }
  if (obj_out) *obj_out = R(ob ? ob->w_S : 0.0) * S_noind + obj_extra;
  return S;
}

Track track_from(int kind, const double* circle, const double* poly, int n_poly, double half_width,
                 const double* obs, int n_obs, int window) {
  Track tr;
  tr.kind = kind;
  tr.cx = circle ? circle[0] : 0.0;
  tr.cy = circle ? circle[1] : 0.0;
  tr.R = circle ? circle[2] : 0.0;
  tr.poly = poly;
  tr.n = n_poly;
  tr.w = half_width;
  tr.obs = obs;
  tr.n_obs = n_obs;
  tr.window = window;
  return tr;
}

// Raw noise sigma*z for every step of sample m (zero when nominal).
void sample_noise(const Cost& C, uint32_t seed, uint32_t pid, uint32_t it, uint32_t m, int T,
                  int nominal, double* eps) {
  for (int t = 0; t < T; ++t) {
    double z[2] = {0.0, 0.0};
    if (!nominal) step_normals(seed, pid, it, m, t, z);
    eps[2 * t + 0] = C.sigma[0] * z[0];
    eps[2 * t + 1] = C.sigma[1] * z[1];
  }
}

}  // namespace

// ===========================================================================
// C ABI for the Python test wrapper.  Control sequences are [T][2] (time
// major) here; the wrapper converts to and from the library's layout.
// ===========================================================================
extern "C" {

int or_abi_version(void) { return 7; }

void or_philox(const uint32_t* ctr, const uint32_t* key, uint32_t* out) { philox4x32_10(ctr, key, out); }

void or_normals(uint32_t seed, uint32_t pid, uint32_t it, uint32_t m, int T, double* z /*[T][2]*/) {
  for (int t = 0; t < T; ++t) step_normals(seed, pid, it, m, t, z + 2 * t);
}

void or_deriv(const double* mp, const double* x, const double* u, double* dx) {
  Model M = model_from(mp);
  deriv<double>(M, x, u, dx);
}

void or_rk4(const double* mp, const double* x, const double* u, double dt, int n_steps, double* out) {
  Model M = model_from(mp);
  double a[6], b[6];
  for (int i = 0; i < 6; ++i) a[i] = x[i];
  for (int s = 0; s < n_steps; ++s) {
    rk4_step<double>(M, a, u, dt, b);
    for (int i = 0; i < 6; ++i) a[i] = b[i];
  }
  for (int i = 0; i < 6; ++i) out[i] = a[i];
}

// Lateral e_y^2: global search (idx_in < 0) or the window rule around idx_in.
double or_lateral_sq(int kind, const double* circle, const double* poly, int n_poly, int window,
                     double px, double py, int idx_in, int* idx_out) {
  Track tr = track_from(kind, circle, poly, n_poly, 1.0, nullptr, 0, window);
  int idx = idx_in;
  double e2 = lateral_sq<double>(tr, px, py, &idx);
  if (idx_out) *idx_out = idx;
  return e2;
}

// Rollout of K samples of one problem (Algorithm 2, inner loop).
//   V: [T][2]; S: [K]; eps_eff: [K][T][2] or null; margin: [K] or null;
//   ms: null (samples 0..K-1) or the K sample indices to evaluate.
void or_rollout(const double* mp, const double* cp, int kind, const double* circle, const double* poly,
                int n_poly, double half_width, const double* obs, int n_obs, int window,
                const double* x0, const double* V, int K, int T, uint32_t seed, uint32_t pid,
                uint32_t it, int nominal, const uint32_t* ms, double* S, double* eps_eff, double* margin,
                int n_threads) {
  Model M = model_from(mp);
  Cost C = cost_from(cp);
  Track tr = track_from(kind, circle, poly, n_poly, half_width, obs, n_obs, window);
  auto work = [&](int m0, int m1) {
    std::vector<double> eps(2 * T);
    for (int m = m0; m < m1; ++m) {
      // output slot m holds sample ms[m] when a sample list is given
      sample_noise(C, seed, pid, it, ms ? ms[m] : (uint32_t)m, T, nominal, eps.data());
      SampleOut so;
      rollout_one<double>(M, C, tr, x0, V, T, eps.data(), eps_eff ? eps_eff + (size_t)2 * T * m : nullptr,
                          nullptr, nullptr, &so);
      S[m] = so.S;
      if (margin) margin[m] = so.margin;
    }
  };
  if (n_threads <= 1) {
    work(0, K);
  } else {
    std::vector<std::thread> th;
    int chunk = (K + n_threads - 1) / n_threads;
    for (int i = 0; i < n_threads; ++i) {
      int a = i * chunk, b = std::min(K, a + chunk);
      if (a < b) th.emplace_back(work, a, b);
    }
    for (auto& t : th) t.join();
  }
}

// ---- curvilinear eight-state model.  x: [8] (v_x, v_y, r, omega_F, omega_R,
// e_psi, e_y, s); wp: (r_w, I_w, C_x); kappa: periodic table with spacing ds.
void or_deriv_c8(const double* mp, const double* wp, const double* kappa, int n_kappa, double ds, const double* x,
                 const double* u, double* dx) {
  CurvTrack ct{kappa, n_kappa, ds, 0.0};
  deriv_c8<double>(model_from(mp), wheels_from(wp), ct, x, u, dx);
}

// Sampled costs (same noise streams as or_rollout).
void or_rollout_c8(const double* mp, const double* wp, const double* cp, const double* kappa, int n_kappa, double ds,
                   double half_width, const double* x0, const double* V, int K, int T, uint32_t seed, uint32_t pid,
                   uint32_t it, int nominal, double* S, double* eps_eff, double* margin, int n_threads) {
  Model M = model_from(mp);
  Wheels Wh = wheels_from(wp);
  Cost C = cost_from(cp);
  CurvTrack ct{kappa, n_kappa, ds, half_width};
  auto work = [&](int m0, int m1) {
    std::vector<double> eps(2 * T);
    for (int m = m0; m < m1; ++m) {
      sample_noise(C, seed, pid, it, (uint32_t)m, T, nominal, eps.data());
      SampleOut so;
      rollout_one_c8<double>(M, Wh, C, ct, x0, V, T, eps.data(),
                             eps_eff ? eps_eff + (size_t)2 * T * m : nullptr, nullptr, nullptr, &so);
      S[m] = so.S;
      if (margin) margin[m] = so.margin;
    }
  };
  if (n_threads <= 1) {
    work(0, K);
  } else {
    std::vector<std::thread> th;
    int chunk = (K + n_threads - 1) / n_threads;
    for (int i = 0; i < n_threads; ++i) {
      int a = i * chunk, b = std::min(K, a + chunk);
      if (a < b) th.emplace_back(work, a, b);
    }
    for (auto& t : th) t.join();
  }
}

// Trajectory under V (+ raw noise eps, or nominal), states [T+1][8].
void or_trajectory_c8(const double* mp, const double* wp, const double* kappa, int n_kappa, double ds,
                      const double* x0, const double* V, int T, const double* eps, double* xs) {
  Model M = model_from(mp);
  Wheels Wh = wheels_from(wp);
  CurvTrack ct{kappa, n_kappa, ds, 0.0};
  double x[8];
  for (int i = 0; i < 8; ++i) x[i] = xs[i] = x0[i];
  for (int t = 0; t < T; ++t) {
    double u[2], xn[8];
    for (int d = 0; d < 2; ++d) u[d] = clampr(V[2 * t + d] + (eps ? eps[2 * t + d] : 0.0), M.u_lo[d], M.u_hi[d]);
    rk4_step_c8<double>(M, Wh, ct, x, u, M.dt, xn);
    for (int i = 0; i < 8; ++i) x[i] = xs[8 * (t + 1) + i] = xn[i];
  }
}

double or_objective_c8(const double* mp, const double* wp, const double* cp, const double* kappa, int n_kappa,
                       double ds, double half_width, const double* x0, const double* V, int T, const double* eps,
                       double w_S, double w_sq, double w_lin, int n_lin, uint64_t* sig) {
  CurvTrack ct{kappa, n_kappa, ds, half_width};
  Objective ob{w_S, w_sq, w_lin, n_lin};
  double L;
  SampleOut so;
  rollout_one_c8<double>(model_from(mp), wheels_from(wp), cost_from(cp), ct, x0, V, T, eps, nullptr, &ob, &L,
                         &so);
  if (sig) *sig = so.sig;
  return L;
}

// Exact gradient of the objective with respect to V ([T][2]) by dual numbers.
void or_gradient_dual_c8(const double* mp, const double* wp, const double* cp, const double* kappa, int n_kappa,
                         double ds, double half_width, const double* x0, const double* V, int T, const double* eps,
                         double w_S, double w_sq, double w_lin, int n_lin, double* grad) {
  Model M = model_from(mp);
  Wheels Wh = wheels_from(wp);
  Cost C = cost_from(cp);
  CurvTrack ct{kappa, n_kappa, ds, half_width};
  Objective ob{w_S, w_sq, w_lin, n_lin};
  std::vector<Dual> Vd(2 * T);
  for (int i = 0; i < 2 * T; ++i) {
    for (int k = 0; k < 2 * T; ++k) Vd[k] = Dual(V[k], k == i ? 1.0 : 0.0);
    Dual L;
    rollout_one_c8<Dual>(M, Wh, C, ct, x0, Vd.data(), T, eps, nullptr, &ob, &L, nullptr);
    grad[i] = L.d;
  }
}

// Central differences with the kink detector (as or_gradient_fd).
void or_gradient_fd_c8(const double* mp, const double* wp, const double* cp, const double* kappa, int n_kappa,
                       double ds, double half_width, const double* x0, const double* V, int T, const double* eps,
                       double w_S, double w_sq, double w_lin, int n_lin, double h, double* grad, int* valid) {
  std::vector<double> Vp(V, V + 2 * T);
  uint64_t s0, sp, sm;
  or_objective_c8(mp, wp, cp, kappa, n_kappa, ds, half_width, x0, V, T, eps, w_S, w_sq, w_lin, n_lin, &s0);
  for (int i = 0; i < 2 * T; ++i) {
    Vp[i] = V[i] + h;
    double Lp = or_objective_c8(mp, wp, cp, kappa, n_kappa, ds, half_width, x0, Vp.data(), T, eps, w_S, w_sq,
                                w_lin, n_lin, &sp);
    Vp[i] = V[i] - h;
    double Lm = or_objective_c8(mp, wp, cp, kappa, n_kappa, ds, half_width, x0, Vp.data(), T, eps, w_S, w_sq,
                                w_lin, n_lin, &sm);
    Vp[i] = V[i];
    grad[i] = (Lp - Lm) / (2.0 * h);
    valid[i] = (sp == s0 && sm == s0) ? 1 : 0;
  }
}

// Safety shield (Algorithm 1) on the curvilinear model: n_s times
// V <- clip(V - delta grad L(V)) on the nominal trajectory from x0.
void or_repair_c8(const double* mp, const double* wp, const double* cp, const double* kappa, int n_kappa,
                  double ds, double half_width, const double* x0, const double* V_plus, int T, int n_steps,
                  double delta, double w_S, double w_sq, double w_lin, int n_lin, double* V_safe) {
  Model M = model_from(mp);
  std::vector<double> g(2 * T);
  for (int i = 0; i < 2 * T; ++i) V_safe[i] = V_plus[i];
  for (int s = 0; s < n_steps; ++s) {
    or_gradient_dual_c8(mp, wp, cp, kappa, n_kappa, ds, half_width, x0, V_safe, T, nullptr, w_S, w_sq, w_lin, n_lin,
                        g.data());
    for (int t = 0; t < T; ++t)
      for (int d = 0; d < 2; ++d) {
        double v = V_safe[2 * t + d] - delta * g[2 * t + d];
        V_safe[2 * t + d] = std::min(std::max(v, M.u_lo[d]), M.u_hi[d]);
      }
  }
}

double or_kappa_at(const double* kappa, int n_kappa, double ds, double s) {
  CurvTrack ct{kappa, n_kappa, ds, 0.0};
  return kappa_at<double>(ct, s);
}

// Path-integral weights (eqs. (7), (9), (11)): omega = exp(-(S - min S)/lambda),
// w = omega / sum(omega).  Non-finite costs get omega = 0.
// stats: [S_min, log(sum omega), ESS = 1/sum w^2, number of non-finite costs].
void or_weights(const double* S, int K, double lambda, double* w, double* stats) {
  double smin = INFINITY;
  int nonfin = 0;
  for (int m = 0; m < K; ++m) {
    if (std::isfinite(S[m])) smin = std::min(smin, S[m]);
    else ++nonfin;
  }
  double eta = 0.0;
  for (int m = 0; m < K; ++m) {
    w[m] = std::isfinite(S[m]) ? std::exp(-(S[m] - smin) / lambda) : 0.0;
    eta += w[m];
  }
  double sq = 0.0;
  for (int m = 0; m < K; ++m) {
    w[m] = eta > 0.0 ? w[m] / eta : 0.0;
    sq += w[m] * w[m];
  }
  stats[0] = smin;
  stats[1] = std::log(eta);
  stats[2] = sq > 0.0 ? 1.0 / sq : 0.0;
  stats[3] = (double)nonfin;
}

// Update law (eq. (10) with the per-trajectory weight of eq. (11)):
// V+ = V + sum_m w_m eps'_m, eps' = clip(V + eps) - V.   eps_eff: [K][T][2].
void or_update(const double* V, const double* w, const double* eps_eff, int K, int T, double* Vp) {
  for (int i = 0; i < 2 * T; ++i) {
    double acc = 0.0;
    for (int m = 0; m < K; ++m) acc += w[m] * eps_eff[(size_t)2 * T * m + i];
    Vp[i] = V[i] + acc;
  }
}

// Objective of one trajectory and its discrete-decision signature.
//   eps: [T][2] raw noise (null: nominal).
double or_objective(const double* mp, const double* cp, int kind, const double* circle, const double* poly,
                    int n_poly, double half_width, const double* obs, int n_obs, int window,
                    const double* x0, const double* V, int T, const double* eps, double w_S,
                    double w_sq, double w_lin, int n_lin, uint64_t* sig) {
  Model M = model_from(mp);
  Cost C = cost_from(cp);
  Track tr = track_from(kind, circle, poly, n_poly, half_width, obs, n_obs, window);
  Objective ob{w_S, w_sq, w_lin, n_lin};
  double L;
  SampleOut so;
  rollout_one<double>(M, C, tr, x0, V, T, eps, nullptr, &ob, &L, &so);
  if (sig) *sig = so.sig;
  return L;
}

// Exact gradient of the objective with respect to V ([T][2]) by forward-mode
// dual numbers: one pass per control component.
void or_gradient_dual(const double* mp, const double* cp, int kind, const double* circle,
                      const double* poly, int n_poly, double half_width, const double* obs, int n_obs,
                      int window, const double* x0, const double* V, int T, const double* eps,
                      double w_S, double w_sq, double w_lin, int n_lin, double* grad) {
  Model M = model_from(mp);
  Cost C = cost_from(cp);
  Track tr = track_from(kind, circle, poly, n_poly, half_width, obs, n_obs, window);
  Objective ob{w_S, w_sq, w_lin, n_lin};
  std::vector<Dual> Vd(2 * T);
  for (int i = 0; i < 2 * T; ++i) {
    for (int k = 0; k < 2 * T; ++k) Vd[k] = Dual(V[k], k == i ? 1.0 : 0.0);
    Dual L;
    rollout_one<Dual>(M, C, tr, x0, Vd.data(), T, eps, nullptr, &ob, &L, nullptr);
    grad[i] = L.d;
  }
}

// Central differences of the objective, step h; valid[i] = 0 when any discrete
// decision differs between V - h e_i, V and V + h e_i (a kink inside the stencil).
void or_gradient_fd(const double* mp, const double* cp, int kind, const double* circle, const double* poly,
                    int n_poly, double half_width, const double* obs, int n_obs, int window,
                    const double* x0, const double* V, int T, const double* eps, double w_S, double w_sq,
                    double w_lin, int n_lin, double h, double* grad, int* valid) {
  std::vector<double> Vp(V, V + 2 * T);
  uint64_t s0, sp, sm;
  or_objective(mp, cp, kind, circle, poly, n_poly, half_width, obs, n_obs, window, x0, V, T, eps, w_S,
               w_sq, w_lin, n_lin, &s0);
  for (int i = 0; i < 2 * T; ++i) {
    Vp[i] = V[i] + h;
    double Lp = or_objective(mp, cp, kind, circle, poly, n_poly, half_width, obs, n_obs, window, x0,
                             Vp.data(), T, eps, w_S, w_sq, w_lin, n_lin, &sp);
    Vp[i] = V[i] - h;
    double Lm = or_objective(mp, cp, kind, circle, poly, n_poly, half_width, obs, n_obs, window, x0,
                             Vp.data(), T, eps, w_S, w_sq, w_lin, n_lin, &sm);
    Vp[i] = V[i];
    grad[i] = (Lp - Lm) / (2.0 * h);
    valid[i] = (sp == s0 && sm == s0) ? 1 : 0;
  }
}

// Safety shield (Algorithm 1, with the gradient taken at the current iterate
// and the step projected onto the control box): n_s times
//   V <- clip(V - delta * grad L(V)),
// where L is the objective above evaluated on the nominal (noise-free)
// trajectory from x0.  With w_lin = 1 and the other weights 0 this is ascent
// on sum_k min(h(x_{k+1}) - alpha h(x_k), 0) of eq. (22).
void or_repair(const double* mp, const double* cp, int kind, const double* circle, const double* poly,
               int n_poly, double half_width, const double* obs, int n_obs, int window, const double* x0,
               const double* V_plus, int T, int n_steps, double delta, double w_S, double w_sq,
               double w_lin, int n_lin, double* V_safe) {
  Model M = model_from(mp);
  std::vector<double> g(2 * T);
  for (int i = 0; i < 2 * T; ++i) V_safe[i] = V_plus[i];
  for (int s = 0; s < n_steps; ++s) {
    or_gradient_dual(mp, cp, kind, circle, poly, n_poly, half_width, obs, n_obs, window, x0, V_safe, T,
                     nullptr, w_S, w_sq, w_lin, n_lin, g.data());
    for (int t = 0; t < T; ++t)
      for (int d = 0; d < 2; ++d) {
        double v = V_safe[2 * t + d] - delta * g[2 * t + d];
        V_safe[2 * t + d] = std::min(std::max(v, M.u_lo[d]), M.u_hi[d]);
      }
  }
}

// Quasi-Newton direction d = -H g of limited-memory BFGS by the two-loop
// recursion (Nocedal & Wright, Numerical Optimization, Algorithm 7.4): pairs
// S[i], Y[i] ([n_pairs][n], oldest first), initial inverse Hessian gamma I.
void or_lbfgs_direction(const double* g, const double* S, const double* Y, int n_pairs, int n, double gamma,
                        double* d) {
  std::vector<double> q(g, g + n), alpha(n_pairs), rho(n_pairs);
  for (int i = n_pairs - 1; i >= 0; --i) {
    const double* s = S + (size_t)i * n;
    const double* y = Y + (size_t)i * n;
    double sy = 0.0, sq = 0.0;
    for (int k = 0; k < n; ++k) sy += s[k] * y[k];
    rho[i] = 1.0 / sy;
    for (int k = 0; k < n; ++k) sq += s[k] * q[k];
    alpha[i] = rho[i] * sq;
    for (int k = 0; k < n; ++k) q[k] -= alpha[i] * y[k];
  }
  for (int k = 0; k < n; ++k) q[k] *= gamma;
  for (int i = 0; i < n_pairs; ++i) {
    const double* s = S + (size_t)i * n;
    const double* y = Y + (size_t)i * n;
    double yr = 0.0;
    for (int k = 0; k < n; ++k) yr += y[k] * q[k];
    const double beta = rho[i] * yr;
    for (int k = 0; k < n; ++k) q[k] += s[k] * (alpha[i] - beta);
  }
  for (int k = 0; k < n; ++k) d[k] = -q[k];
}

// Safety shield with the quasi-Newton optimiser the paper's text names
// (Sec. IV-B) in place of Algorithm 1's plain gradient step; limited-memory
// BFGS with projection onto the control box (reading: the paper gives no
// details).  Per iteration k, with g_k = grad L(V_k) of the objective above:
//   stop when g_k = 0 (V is then only projected);
//   for k > 0 the pair s = V_k - V_{k-1}, y = g_k - g_{k-1} is kept (at most
//   `memory` pairs, oldest dropped) when s.y > 1e-2 |s| |y|;
//   d = -H g_k by the two-loop recursion with H_0 = gamma I, gamma = s.y / y.y
//   of the newest kept pair, or delta when none is kept (then the step is
//   Algorithm 1's);  V_{k+1} = clip(V_k + d).
// memory = 0 is Algorithm 1 exactly.
void or_repair_lbfgs(const double* mp, const double* cp, int kind, const double* circle, const double* poly,
                     int n_poly, double half_width, const double* obs, int n_obs, int window, const double* x0,
                     const double* V_plus, int T, int n_steps, double delta, double w_S, double w_sq,
                     double w_lin, int n_lin, int memory, double* V_safe) {
  Model M = model_from(mp);
  const int n = 2 * T;
  std::vector<double> V(V_plus, V_plus + n), g(n), Vp(n), gp(n), d(n), S, Y;
  int n_pairs = 0;
  auto clip_all = [&](std::vector<double>& v) {
    for (int t = 0; t < T; ++t)
      for (int c = 0; c < 2; ++c) v[2 * t + c] = std::min(std::max(v[2 * t + c], M.u_lo[c]), M.u_hi[c]);
  };
  for (int k = 0; k < n_steps; ++k) {
    or_gradient_dual(mp, cp, kind, circle, poly, n_poly, half_width, obs, n_obs, window, x0, V.data(), T,
                     nullptr, w_S, w_sq, w_lin, n_lin, g.data());
    bool zero = true;
    for (int i = 0; i < n; ++i) zero = zero && g[i] == 0.0;
    if (zero) {
      clip_all(V);
      break;
    }
    if (k > 0 && memory > 0) {
      std::vector<double> s(n), y(n);
      double sy = 0.0, ss = 0.0, yy = 0.0;
      for (int i = 0; i < n; ++i) {
        s[i] = V[i] - Vp[i];
        y[i] = g[i] - gp[i];
        sy += s[i] * y[i];
        ss += s[i] * s[i];
        yy += y[i] * y[i];
      }
      if (sy > 1e-2 * std::sqrt(ss) * std::sqrt(yy)) {
        if (n_pairs == memory) {
          S.erase(S.begin(), S.begin() + n);
          Y.erase(Y.begin(), Y.begin() + n);
          --n_pairs;
        }
        S.insert(S.end(), s.begin(), s.end());
        Y.insert(Y.end(), y.begin(), y.end());
        ++n_pairs;
      }
    }
    double gamma = delta;
    if (n_pairs > 0) {
      const double* s = S.data() + (size_t)(n_pairs - 1) * n;
      const double* y = Y.data() + (size_t)(n_pairs - 1) * n;
      double sy = 0.0, yy = 0.0;
      for (int i = 0; i < n; ++i) {
        sy += s[i] * y[i];
        yy += y[i] * y[i];
      }
      gamma = sy / yy;
    }
    or_lbfgs_direction(g.data(), S.data(), Y.data(), n_pairs, n, gamma, d.data());
    Vp = V;
    gp = g;
    for (int i = 0; i < n; ++i) V[i] += d[i];
    clip_all(V);
  }
  for (int i = 0; i < n; ++i) V_safe[i] = V[i];
}

// Nominal trajectory x_0..x_T ([T+1][6]) and barrier values ([T+1][1+n_obs]).
void or_trajectory(const double* mp, const double* cp, int kind, const double* circle, const double* poly,
                   int n_poly, double half_width, const double* obs, int n_obs, int window,
                   const double* x0, const double* V, int T, const double* eps, double* xs, double* hs) {
  Model M = model_from(mp);
  Cost C = cost_from(cp);
  (void)C;
  Track tr = track_from(kind, circle, poly, n_poly, half_width, obs, n_obs, window);
  const int nb = 1 + n_obs;
  double x[6], xn[6];
  for (int i = 0; i < 6; ++i) x[i] = x0[i];
  int idx = -1;
  double ey2, mg;
  bool inside;
  for (int t = 0; t <= T; ++t) {
    for (int i = 0; i < 6; ++i) xs[6 * t + i] = x[i];
    barriers<double>(tr, x, &idx, hs + (size_t)nb * t, &ey2, &inside, &mg);
    if (t == T) break;
    double u[2];
    for (int d = 0; d < 2; ++d)
      u[d] = std::min(std::max(V[2 * t + d] + (eps ? eps[2 * t + d] : 0.0), M.u_lo[d]), M.u_hi[d]);
    rk4_step<double>(M, x, u, M.dt, xn);
    for (int i = 0; i < 6; ++i) x[i] = xn[i];
  }
}

}  // extern "C"
