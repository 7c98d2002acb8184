// Batched plan: hundreds of independent MPPI problems of uneven K and T in one
// persistent launch.  Workgroups take (problem, sample-tile) items ordered
// longest-horizon first (workgroup g starts with item g, then pops the rest
// from a queue); each tile runs its rollouts, reduces them to a
// split softmax partial (tile min cost, sum of weights, sum of squared weights,
// weighted noise sums per step) and takes a ticket on its problem; the tile
// that takes the last ticket combines the partials in tile order (streaming
// log-sum-exp rescale) and writes V+ and the weight statistics; when the grid
// is smaller than the tile list, the last workgroup to leave re-arms the
// queue (a grid as large as the list never touches it).  With the shield, the combining
// workgroup then runs it on the problem (Algorithm 1 or L-BFGS) and, when the
// plan executes, the plant step and warm start, all in the same launch (a
// separate shield kernel when the workgroup has fewer than three waves or its
// LDS does not fit; a separate execute kernel without the shield).  A launch
// of several kernels (obstacle slots, empty problems, separate shield or
// execute) is captured once into a HIP graph; a single kernel is launched
// directly.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <numeric>
#include <string>
#include <vector>

#include "common.hpp"

using namespace smppi;

namespace {

constexpr int PART_HDR = 4;  // tile min, sum w, sum w^2, non-finite count
// Row stride of the tile partials: the header, then the 2 t_max noise sums
// padded to a multiple of four floats (16-byte rows for the combine's wide loads).
__host__ __device__ constexpr int part_stride(int t_max) { return PART_HDR + ((2 * t_max + 3) & ~3); }

struct FusedArgs {
  ProblemArgs<float> p;
  DevModel<float> M;
  DevCost<float> C;
  const float* V;
  float* S;
  float* V_plus;
  float* stats;
  float inv_lambda;
  const int2* tiles;         // [n_tiles] (problem, tile index within problem)
  const int32_t* tile_off;   // [B+1] first tile of each problem
  int n_tiles;
  int tile;                  // samples per tile
  float* part;               // [n_tiles][part_stride(t_max)]
  uint32_t* queue;           // [1] next tile
  uint32_t* tickets;         // [B] finished tiles per problem
  uint32_t* exits;           // [1] workgroups that have left the tile loop
  int repair;                // nonzero: the combining workgroup also runs the shield (and execute)
  RepairArgs<float> rep;
  const float4* obs_pad;     // [B][kMaxObs] obstacle slots (WaveObstacles; NOBS > 0, tile mode)
  // One-problem plans: problem 0's dimensions, taken from the offsets at plan
  // creation (checked there); tile k is then (0, k), and a workgroup reads
  // neither the tile list nor the offsets before staging.
  int one;
  ProblemDims d1;
};

// ---------------------------------------------------------------------------
// Latency mode: one tile = 64 samples handled by four specialised waves (one
// per SIMD) that run the same trajectories as a pipeline, step by step:
//   wave 0: noise, clipped controls, control cost, and per step the
//           coefficients of the velocity part of the RK4 step (shield_vel_row:
//           the stage factors and tyre stiffnesses folded in, so that each RK4
//           stage is three FMA chains on the next wave's chain),
//   wave 1: the RK4 chain (velocity part as shield_vel_step, pose part as
//           rk4_pose: the classic RK4 of the model, in another evaluation
//           order), writing (p_x, p_y, v_x) of every new state,
//   waves 2-3: two lanes per sample: the lateral offset window split between
//           the pair, running cost, DCBF penalties, obstacles (split between
//           the pair), collision indicator.
// Steps pass through rings of PIPE_R slots in LDS with step counters (the
// producer publishes a step once its slot is written, and reuses a slot once
// its consumers have counted the step read), so the pipeline fills in a few
// steps and runs at its slowest wave's rate.  A launch with fewer waves than
// SIMDs is bound by each wave's per-step chain; splitting the step four ways
// shortens it.  Same arithmetic as rollout_sample, summed in partial sums
// (control terms, state terms of each half) instead of one.
constexpr int PIPE_R = 8;
constexpr int PIPE_BLK = 4 * WAVE;

struct PipeLds {
  float2 ctl[PIPE_R][7][WAVE];  // the 13 values of shield_vel_row for the step (pairs; the last one padded)
  float pos[PIPE_R][3][WAVE];  // p_x, p_y, v_x of x_{t+1}
  float part[2][WAVE];
  int cnt[4];  // steps published by wave 0 (controls) and wave 1 (states); steps read by waves 2 and 3
};

// Swap with the neighbouring lane (DPP quad_perm [1,0,3,2]).
__device__ __forceinline__ float pair_swap(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF, false));
}
__device__ __forceinline__ int pair_swap(int v) { return __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xF, 0xF, false); }

// The five polyline rows a lane of the pair reads for a window centred on c
// (half 0: slots c-2..c+2 as c-2, c-1, c and c+1, c+2; half 1: c-4..c-2 and
// c+3, c+4).  They depend on c alone, so they are read before the wave waits
// for the next position.
struct PairRows {
  float s[5][4];
  float il[5];
};
__device__ __forceinline__ PairRows pair_rows(const TrackView<float>& tr, int c, int half) {
  const int bA = half ? -4 : -2, bB = half ? 3 : 1;
  const float* sa = tr.seg + 4 * (c + bA);  // padded copy: no wrap needed
  const float* sb = tr.seg + 4 * (c + bB);
  PairRows r;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
#pragma unroll
    for (int q = 0; q < 4; ++q) r.s[k][q] = sa[4 * k + q];
    r.il[k] = tr.il2[c + bA + k];
  }
#pragma unroll
  for (int k = 0; k < 2; ++k) {
#pragma unroll
    for (int q = 0; q < 4; ++q) r.s[3 + k][q] = sb[4 * k + q];
    r.il[3 + k] = tr.il2[c + bB + k];
  }
  return r;
}

// The window rule with half width 4 on a pair of lanes, from the rows of
// pair_rows.  Half 0 evaluates the offsets 0, -1, +1, -2, +2 (slots c-2..c+2),
// half 1 the offsets -3, +3, -4, +4 (slots c-4, c-3, c+3, c+4; its fifth slot,
// c-2, is excluded), each half in the rule's order; all of half 0's offsets
// precede half 1's in the rule, so the pair keeps half 1's result only when it
// is strictly smaller.  Both lanes return the same e_y^2 and centre.  The whole
// wave must be active.
__device__ __forceinline__ float pair_window4(const TrackView<float>& tr, const PairRows& r, int& c, float px,
                                              float py, int half) {
  auto d2 = [&](int k) {
    const float rx = px - r.s[k][0], ry = py - r.s[k][1];
    const float dx = r.s[k][2], dy = r.s[k][3];
    const float lam = clamp_r((rx * dx + ry * dy) * r.il[k], 0.f, 1.f);
    const float ex = rx - lam * dx, ey = ry - lam * dy;
    return ex * ex + ey * ey;
  };
  const float a0 = d2(0), a1 = d2(1), a2 = d2(2);
  const float b0 = d2(3), b1 = d2(4);
  const int m1 = 1 + 2 * half, m2 = 2 + 2 * half;
  float bd = half ? INFINITY : a2;  // offset 0 (half 1: excluded slot)
  int off = 0;
  if (a1 < bd) { bd = a1; off = -m1; }
  if (b0 < bd) { bd = b0; off = m1; }
  if (a0 < bd) { bd = a0; off = -m2; }
  if (b1 < bd) { bd = b1; off = m2; }
  const float obd = pair_swap(bd);
  const int ooff = pair_swap(off);
  const float bd0 = half ? obd : bd, bd1 = half ? bd : obd;
  const int off0 = half ? ooff : off, off1 = half ? off : ooff;
  const bool take1 = bd1 < bd0;
  int i = c + (take1 ? off1 : off0);
  i += (i < 0) ? tr.n : 0;
  i -= (i >= tr.n) ? tr.n : 0;
  c = i;
  return take1 ? bd1 : bd0;
}

template <int NOBS>
__device__ float rollout_pipe(const FusedArgs& a, const TrackView<float>& tr, const State<float>& x0,
                              const float* Vs, const ProblemDims& d, int m, uint32_t pid, uint32_t it,
                              PipeLds& P) {
  constexpr int NH = NOBS > 0 ? (NOBS + 1) / 2 : 1;  // obstacles per half
  const int w = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
  const int T = d.T;
  const DevModel<float> M = model_in_vgprs(a.M);
  const DevCost<float> C = cost_in_vgprs(a.C);
  // wave 0
  NoiseStream<float> ns;
  ns.seed = a.p.seed;
  ns.m = (uint32_t)m;
  ns.pid = pid;
  ns.it = it;
  ns.nominal = a.p.nominal != 0;
  float Sc = 0.f;
  // wave 1
  State<float> x = x0;
  // waves 2-3: sample j = lane pair, half h
  const int tt = threadIdx.x - 2 * WAVE, j = tt >> 1, half = tt & 1;
  int idx = tr.idx0;
  float ey2 = 0.f, hp = 0.f, vxp = x0.vx, S2 = 0.f;
  bool outside = false;
  float hob[NH];
  if (w >= 2) {
    if (tr.n > 0) {
      ey2 = seg_dist2(tr, idx, x0.px, x0.py);  // the window around the global nearest segment returns it
    } else {
      int dummy = 0;
      ey2 = lateral_sq(tr, x0.px, x0.py, dummy);
    }
    hp = tr.w2 - ey2;
    outside = hp < 0.f;
    float pen0 = half ? 0.f : fmaxf((C.alpha - 1.f) * hp, 0.f);
    bool oo = false;
#pragma unroll
    for (int k = 0; k < NH; ++k) {
      const int i = 2 * k + half;
      hob[k] = 0.f;
      if (i < NOBS) {
        const Obs<float> o = obs_at(tr, i);
        const float ox = x0.px - o.cx, oy = x0.py - o.cy;
        const float dd = ox * ox + oy * oy;
        hob[k] = dd - o.re2;
        oo = oo || (dd < o.r2);
        pen0 += fmaxf((C.alpha - 1.f) * hob[k], 0.f);
      }
    }
    if (NOBS > 0) {
      // the partner lane's hits, exchanged with the whole wave active (inside a
      // short-circuit the exchange would run only on the lanes without a hit of
      // their own, and a lane whose partner had one would read a stale value)
      const bool po = pair_swap((int)oo) != 0;
      outside = outside || oo || po;
    }
    S2 = C.C_cbf * pen0;
  }
  if (threadIdx.x == 0) P.cnt[0] = P.cnt[1] = P.cnt[2] = P.cnt[3] = 0;
  __syncthreads();
  if (w == 0) {
    int seen = 0;
    for (int t = 0; t < T; ++t) {
      const float v0 = Vs[t], v1 = Vs[T + t];
      float e0, e1;
      ns.at(t, C.sigma[0], C.sigma[1], e0, e1);
      const float u0 = clamp_r(v0 + e0, M.u_lo[0], M.u_hi[0]);
      const float u1 = clamp_r(v1 + e1, M.u_lo[1], M.u_hi[1]);
      Sc += C.ctrl_w[0] * v0 * u0 + C.ctrl_w[1] * v1 * u1;
      float cr[14];
      shield_vel_row(M, u0, u1, cr);
      cr[13] = 0.f;
      if (t >= PIPE_R) wave_wait(&P.cnt[1], t - PIPE_R, seen, a.p.err);  // slot read by wave 1
      float2(*c)[WAVE] = P.ctl[t % PIPE_R];
#pragma unroll
      for (int k = 0; k < 7; ++k) c[k][lane] = make_float2(cr[2 * k], cr[2 * k + 1]);
      wave_publish(&P.cnt[0], t + 1);
    }
  } else if (w == 1) {
    const ShieldVel<float> kv = shield_vel(M);
    int seen = 0, seen2 = 0, seen3 = 0;
    for (int t = 0; t < T; ++t) {
      wave_wait(&P.cnt[0], t, seen, a.p.err);
      const float2(*c)[WAVE] = P.ctl[t % PIPE_R];
      float cr[14];
#pragma unroll
      for (int k = 0; k < 7; ++k) {
        const float2 v = c[k][lane];
        cr[2 * k] = v.x;
        cr[2 * k + 1] = v.y;
      }
      VelStages<float> g;
      shield_vel_step(kv, cr, x.vx, x.vy, x.om, g);
      rk4_pose(M, g, x.px, x.py, x.psi);
      if (t >= PIPE_R) {  // slot read by waves 2 and 3
        wave_wait(&P.cnt[2], t - PIPE_R, seen2, a.p.err);
        wave_wait(&P.cnt[3], t - PIPE_R, seen3, a.p.err);
      }
      float(*o)[WAVE] = P.pos[t % PIPE_R];
      o[0][lane] = x.px;
      o[1][lane] = x.py;
      o[2][lane] = x.vx;
      wave_publish(&P.cnt[1], t + 1);
    }
  } else {
    int seen = 0;
    const bool w4 = tr.n > 0 && tr.window == 4;
    PairRows rows;
    if (w4) rows = pair_rows(tr, idx, half);
    for (int t = 0; t < T; ++t) {
      const float dv = vxp - C.v_g;
      float q = C.q_v * dv * dv + C.q_ey * ey2;
      if (outside) q += C.C_obs;
      S2 += half ? 0.f : q;
      wave_wait(&P.cnt[1], t, seen, a.p.err);
      const float(*qp)[WAVE] = P.pos[t % PIPE_R];
      const float px = qp[0][j], py = qp[1][j];
      vxp = qp[2][j];
      // counted as read once the reads are issued (the LDS performs this wave's
      // operations in order, so the slot's next store lands after them)
      wave_publish(&P.cnt[w], t + 1);
      if (w4) {
        ey2 = pair_window4(tr, rows, idx, px, py, half);
        rows = pair_rows(tr, idx, half);  // the next step's window, read before its wait
      } else {
        ey2 = lateral_sq(tr, px, py, idx);
      }
      const float h1 = tr.w2 - ey2;
      float pen = half ? 0.f : fmaxf(C.alpha * hp - h1, 0.f);
      hp = h1;
      outside = h1 < 0.f;
      bool oo = false;
#pragma unroll
      for (int k = 0; k < NH; ++k) {
        const int i = 2 * k + half;
        if (i < NOBS) {
          const Obs<float> o = obs_at(tr, i);
          const float ox = px - o.cx, oy = py - o.cy;
          const float dd = ox * ox + oy * oy;
          const float hi = dd - o.re2;
          pen += fmaxf(C.alpha * hob[k] - hi, 0.f);
          hob[k] = hi;
          oo = oo || (dd < o.r2);
        }
      }
      if (NOBS > 0) {
        const bool po = pair_swap((int)oo) != 0;  // whole wave active (see above)
        outside = outside || oo || po;
      }
      S2 += C.C_cbf * pen;
    }
  }
  __syncthreads();
  if (w >= 2) {
    const float dv = vxp - C.v_g;
    float q = C.q_v * dv * dv + C.q_ey * ey2;
    if (outside) q += C.C_obs;
    const float mine = S2 + (half ? 0.f : C.phi_w * q);
    const float other = pair_swap(mine);
    if (half == 0) P.part[1][j] = mine + other;
  }
  if (w == 0) P.part[0][lane] = Sc;
  __syncthreads();
  return P.part[0][lane] + P.part[1][lane];
}

// FUSE: the shield (and execute) code is compiled in (plans that run the shield
// inside the launch); without it the kernel needs far fewer registers, which
// raises the occupancy of plans without the shield.
template <int NOBS, int BLK, int SPT, bool PIPE, bool FUSE>
__global__ __launch_bounds__(BLK) void k_fused(FusedArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  // block reductions: minima in red[0, waves), sums in red[waves, 4 waves); a
  // tile and a combine each take one minimum then the sums, and every pair is
  // separated from the next by the ticket barriers, so neither needs its
  // leading barrier
  __shared__ float red[4 * (BLK / WAVE)];
  float* const red_sum = red + BLK / WAVE;
  __shared__ NoiseSumLds<float, BLK, SPT> L;
  __shared__ int s_tile;
  __shared__ uint32_t s_ticket;
  __shared__ int s_last;
  const int tid = threadIdx.x;
  const int pstride = part_stride(a.p.t_max);
  int staged_b = -1;
  float* Vs = nullptr;
  TrackView<float> tr;
  ProblemDims d;
  // Workgroup g takes tile g first (no queue round trip before the first
  // rollout; the grid never exceeds the tile count), then tiles gridDim.x + q
  // for q popped from the queue.  A grid as large as the tile list never uses
  // the queue (which then stays armed), so a workgroup leaves without the two
  // atomic round trips of a final pop and the exit count.
  const bool queued = (int)gridDim.x < a.n_tiles;
  bool first = true;
  for (;;) {
    int tile;
    if (first) {
      tile = blockIdx.x;
      first = false;
    } else {
      if (!queued) break;
      if (tid == 0) s_tile = (int)gridDim.x + (int)atomicAdd(a.queue, 1u);
      __syncthreads();
      tile = __builtin_amdgcn_readfirstlane(s_tile);
      __syncthreads();
    }
    if (tile >= a.n_tiles) break;
    int b, kb;
    if (a.one) {
      b = 0;
      kb = tile;
      d = a.d1;
    } else {
      const int2 tk = a.tiles[tile];
      b = __builtin_amdgcn_readfirstlane(tk.x);
      kb = __builtin_amdgcn_readfirstlane(tk.y);
      if (!load_dims(a.p, b, d)) continue;
    }
    if (b != staged_b) {
      tr = stage_problem(a.p, b, d, a.V, smem, &Vs);
      staged_b = b;
      __syncthreads();
    }
    const uint32_t pid = (uint32_t)(a.p.pid_base + b), it = a.p.iter[b];
    const State<float> x0 = load_state(a.p.x0 + 6 * (size_t)b);
    // ---- rollouts: sample ms[j] of this tile, owned by this thread when own[j]
    float s[SPT];
    int ms[SPT];
    bool own[SPT];
    float mn = INFINITY;
    if constexpr (PIPE) {
      __shared__ PipeLds PL;
      ms[0] = kb * a.tile + tid % WAVE;
      own[0] = tid < WAVE && ms[0] < d.K;
      const float sv = rollout_pipe<NOBS>(a, tr, x0, Vs, d, ms[0], pid, it, PL);
      s[0] = own[0] ? sv : INFINITY;
      if (own[0]) a.S[d.k0 + ms[0]] = sv;
      if (isfinite(s[0])) mn = s[0];
    } else {
      // (with obstacles every lane of a wave that has samples runs: the wave-level
      // obstacle evaluation needs the whole wave; lanes past K copy the last sample)
      const WaveObstacles wob = NOBS > 0 ? WaveObstacles(a.obs_pad + (size_t)b * NOBS, NOBS) : WaveObstacles();
#pragma unroll
      for (int j = 0; j < SPT; ++j) {
        ms[j] = kb * a.tile + j * BLK + tid;
        own[j] = ms[j] < d.K;
        s[j] = INFINITY;
        const bool run = NOBS > 0 ? (ms[j] - (int)(tid % WAVE) < d.K) : own[j];
        if (run) {
          NoiseStream<float> ns;
          ns.seed = a.p.seed;
          ns.m = (uint32_t)(own[j] ? ms[j] : d.K - 1);
          ns.pid = pid;
          ns.it = it;
          ns.nominal = a.p.nominal != 0;
          float sv;
          if constexpr (NOBS > 0)
            sv = rollout_sample<float, NOBS>(a.M, a.C, tr, x0, Vs, d.T, ns, nullptr, wob);
          else
            sv = rollout_sample<float, NOBS>(a.M, a.C, tr, x0, Vs, d.T, ns, nullptr);
          if (own[j]) {
            s[j] = sv;
            a.S[d.k0 + ms[j]] = sv;
          }
        }
        if (isfinite(s[j])) mn = fminf(mn, s[j]);
      }
    }
    // ---- tile-local softmax partial
    mn = block_min<float, false>(mn, red);
    float om[SPT], z = 0.f, q = 0.f, nf = 0.f;
#pragma unroll
    for (int j = 0; j < SPT; ++j) {
      om[j] = isfinite(s[j]) ? exp_r(-(s[j] - mn) * a.inv_lambda) : 0.f;
      z += om[j];
      q += om[j] * om[j];
      if (own[j] && !isfinite(s[j])) nf += 1.f;
    }
    block_sum3<float, false>(z, q, nf, red_sum);
    const int toff_b = a.one ? 0 : a.tile_off[b];  // first tile of problem b
    float* P = a.part + (size_t)(toff_b + kb) * pstride;
    block_noise_sums<float, BLK, SPT, PIPE>(a.M, a.C, a.p.seed, pid, it, a.p.nominal != 0, Vs, d.T, ms, om, L,
                                      P + PART_HDR);
    if (tid == 0) {
      P[0] = mn;
      P[1] = z;
      P[2] = q;
      P[3] = nf;
    }
    // ---- ticket; the last tile of problem b combines
    ticket_release();
    __syncthreads();
    const int ntb = (d.K + a.tile - 1) / a.tile;
    if (tid == 0) s_ticket = atomicAdd(&a.tickets[b], 1u);
    __syncthreads();
    if (s_ticket == (uint32_t)(ntb - 1)) {
      ticket_acquire();
      // Streaming log-sum-exp combine: tile k's sums are rescaled by
      // exp(-(min_k - min)/lambda).  The partials were written by other
      // workgroups (other XCDs), so every pass is a round trip to memory: the
      // tile headers are read once into registers and the scales kept in LDS
      // when the problem has at most BLK*SPT tiles; the V+ pass keeps NB loads
      // in flight per thread.
      const float* P0 = a.part + (size_t)toff_b * pstride;
      float* s_sc = L.w;
      float gmin, Z, Q, NF;
      const bool one_pass = ntb <= BLK * SPT;
      if (one_pass) {
        float mk[SPT], zk[SPT], qk[SPT];
        float mn_l = INFINITY, nf_l = 0.f;
#pragma unroll
        for (int j = 0; j < SPT; ++j) {
          const int k = tid + j * BLK;
          mk[j] = INFINITY;
          zk[j] = qk[j] = 0.f;
          if (k < ntb) {
            const float* Pk = P0 + (size_t)k * pstride;
            mk[j] = Pk[0];
            zk[j] = Pk[1];
            qk[j] = Pk[2];
            nf_l += Pk[3];
            mn_l = fminf(mn_l, mk[j]);
          }
        }
        gmin = block_min<float, false>(mn_l, red);
        float z_l = 0.f, q_l = 0.f;
#pragma unroll
        for (int j = 0; j < SPT; ++j) {
          const int k = tid + j * BLK;
          if (k < ntb) {
            const float sc = isfinite(mk[j]) ? exp_r(-(mk[j] - gmin) * a.inv_lambda) : 0.f;
            s_sc[k] = sc;
            z_l += sc * zk[j];
            q_l += sc * sc * qk[j];
          }
        }
        block_sum3<float, false>(z_l, q_l, nf_l, red_sum);
        Z = z_l;
        Q = q_l;
        NF = nf_l;
      } else {
        float mn_l = INFINITY;
        for (int k = tid; k < ntb; k += BLK) mn_l = fminf(mn_l, P0[(size_t)k * pstride]);
        gmin = block_min<float, false>(mn_l, red);
        float z_l = 0.f, q_l = 0.f, nf_l = 0.f;
        for (int k = tid; k < ntb; k += BLK) {
          const float* Pk = P0 + (size_t)k * pstride;
          const float mk = Pk[0];
          const float sc = isfinite(mk) ? exp_r(-(mk - gmin) * a.inv_lambda) : 0.f;
          z_l += sc * Pk[1];
          q_l += sc * sc * Pk[2];
          nf_l += Pk[3];
        }
        block_sum3<float, false>(z_l, q_l, nf_l, red_sum);
        Z = z_l;
        Q = q_l;
        NF = nf_l;
      }
      const float iZ = Z > 0.f ? 1.f / Z : 0.f;
      const float* Vb = a.V + 2 * (size_t)d.t0;
      float* Vpb = a.V_plus + 2 * (size_t)d.t0;
      // V+ pass: thread (g, il) sums tiles g, g+G, ... of output i0 + il (NB
      // loads in flight); the G group sums are then added in group order.
      const int nI = min(2 * d.T, BLK), G = one_pass ? BLK / nI : 1;
      const int g = tid / nI, il = tid % nI;
      float* s_red = &L.red4[0][0];
      // Many tiles (tile mode): thread (g4, i4) sums tiles g4, g4 + G4, ... of the
      // four outputs 4 i4 .. 4 i4 + 3 with 16-byte loads (a quarter of the load
      // round trips; the columns past 2T of the last group are never used).
      const int n4 = (2 * d.T + 3) >> 2;
      const bool wide = !PIPE && one_pass && n4 <= BLK && ntb > 16 * G;
      if (wide) {
        constexpr int NB4 = 8;  // loads in flight (no more registers than the rollout needs)
        const int G4 = BLK / n4, g4 = tid / n4, i4 = tid % n4;
        float a4[4] = {0.f, 0.f, 0.f, 0.f};
        if (g4 < G4) {
          const float* Pi = P0 + PART_HDR + 4 * i4;
          for (int k0 = g4; k0 < ntb; k0 += NB4 * G4) {
            float4 v[NB4];
            float sc[NB4];
#pragma unroll
            for (int u = 0; u < NB4; ++u) {
              const int kk = k0 + u * G4;
              const bool in = kk < ntb;
              v[u] = in ? *reinterpret_cast<const float4*>(Pi + (size_t)kk * pstride) : make_float4(0.f, 0.f, 0.f, 0.f);
              sc[u] = in ? s_sc[kk] : 0.f;
            }
#pragma unroll
            for (int u = 0; u < NB4; ++u) {
              a4[0] += sc[u] * v[u].x;
              a4[1] += sc[u] * v[u].y;
              a4[2] += sc[u] * v[u].z;
              a4[3] += sc[u] * v[u].w;
            }
          }
#pragma unroll
          for (int q = 0; q < 4; ++q) L.red4[q][tid] = a4[q];
        }
        __syncthreads();
        for (int i = tid; i < 2 * d.T; i += BLK) {
          const int j4 = i >> 2, q = i & 3;
          float acc = 0.f;
          for (int gg = 0; gg < G4; ++gg) acc += L.red4[q][gg * n4 + j4];
          const float vp = Vb[i] + acc * iZ;
          Vpb[i] = vp;
          if (BLK >= 3 * WAVE && a.repair) Vs[i] = vp;
        }
      }
      for (int i0 = 0; i0 < (wide ? 0 : 2 * d.T); i0 += (one_pass ? nI : BLK)) {
        const int i = one_pass ? i0 + il : i0 + tid;
        float acc = 0.f;
        if (one_pass) {
          if (g < G && i < 2 * d.T) {
            const float* Pi = P0 + PART_HDR + i;
            constexpr int NB = PIPE ? 32 : 16;  // loads in flight (latency mode: one batch covers 64 tiles)
            for (int k0 = g; k0 < ntb; k0 += NB * G) {
              float v[NB], sc[NB];
#pragma unroll
              for (int u = 0; u < NB; ++u) {
                const int kk = k0 + u * G;
                const bool in = kk < ntb;
                v[u] = in ? Pi[(size_t)kk * pstride] : 0.f;
                sc[u] = in ? s_sc[kk] : 0.f;
              }
#pragma unroll
              for (int u = 0; u < NB; ++u) acc += sc[u] * v[u];
            }
          }
          if (G > 1) {
            s_red[tid] = acc;
            __syncthreads();
            if (g == 0)
              for (int gg = 1; gg < G; ++gg) acc += s_red[gg * nI + il];
            if (i0 + nI < 2 * d.T) __syncthreads();  // s_red is written again (the last chunk: the barrier below)
          }
          if (g != 0) continue;
        } else {
          for (int k0 = 0; k0 < ntb; k0 += BLK) {
            __syncthreads();
            if (k0 + tid < ntb) {
              const float mk = P0[(size_t)(k0 + tid) * pstride];
              s_sc[tid] = isfinite(mk) ? exp_r(-(mk - gmin) * a.inv_lambda) : 0.f;
            }
            __syncthreads();
            const int kn = min(BLK, ntb - k0);
            if (i < 2 * d.T) {
              const float* Pi = P0 + (size_t)k0 * pstride + PART_HDR + i;
#pragma unroll 8
              for (int kk = 0; kk < kn; ++kk) acc += s_sc[kk] * Pi[(size_t)kk * pstride];
            }
          }
        }
        if (i < 2 * d.T) {
          const float vp = Vb[i] + acc * iZ;
          Vpb[i] = vp;
          // no tile of problem b is left: its staged V becomes the shield's V+
          if (BLK >= 3 * WAVE && a.repair) Vs[i] = vp;
        }
      }
      __syncthreads();
      if (tid == 0) {
        a.stats[4 * b + 0] = gmin;
        a.stats[4 * b + 1] = logf(Z);
        a.stats[4 * b + 2] = Q > 0.f ? Z * Z / Q : 0.f;
        a.stats[4 * b + 3] = NF;
        a.tickets[b] = 0u;
      }
      if constexpr (FUSE && BLK >= 3 * WAVE) {
        if (a.repair) {
          // the barrier above published Vs; since then only thread 0 wrote (global memory)
          unsigned char* rl = smem + stage_lds_bytes<float>(a.p.poly_max, a.p.t_max, a.p.obs_max);
          repair_problem<float, NOBS, PIPE>(a.rep, b, d, tr, Vs, rl, &s_last);
          float* out = a.rep.V_safe + 2 * (size_t)d.t0;
          for (int i = tid; i < 2 * d.T; i += BLK) out[i] = Vs[i];
          if (a.rep.exec) execute_problem(a.rep.ex, b, d.t0, d.T, Vs, reinterpret_cast<float*>(rl));
          __syncthreads();
          staged_b = -1;  // Vs no longer holds problem b's V
        }
      }
    }
  }
  // The last workgroup to leave re-arms the queue for the next launch (every
  // other workgroup has taken its final, out-of-range, tile by then).
  if (queued && tid == 0 && atomicAdd(a.exits, 1u) == gridDim.x - 1) {
    atomicExch(a.queue, 0u);
    atomicExch(a.exits, 0u);
  }
}

// Problems with K_b = 0 still need V+ = V.
__global__ void k_copy_empty(const int64_t* k_off, const int32_t* t_off, const float* V, float* V_plus,
                             float* stats) {
  const int b = blockIdx.x;
  if (k_off[b + 1] != k_off[b]) return;
  const int t0 = t_off[b], T = t_off[b + 1] - t0;
  for (int i = threadIdx.x; i < 2 * T; i += blockDim.x) V_plus[2 * (size_t)t0 + i] = V[2 * (size_t)t0 + i];
  if (threadIdx.x == 0) {
    stats[4 * b + 0] = INFINITY;
    stats[4 * b + 1] = -INFINITY;
    stats[4 * b + 2] = 0.f;
    stats[4 * b + 3] = 0.f;
  }
}


using FusedFn = void (*)(FusedArgs);

// Tile-mode kernel for (block, samples per thread); with fuse, the variant with
// the shield compiled in (blocks of at least three waves only).
template <int NOBS>
FusedFn pick_fused(int blk, int spt, bool fuse) {
#define SMPPI_CASE(BL, SP) \
  if (blk == BL && spt == SP) return k_fused<NOBS, BL, SP, false, false>;
#define SMPPI_CASE_F(BL, SP) \
  if (blk == BL && spt == SP) return fuse ? k_fused<NOBS, BL, SP, false, true> : k_fused<NOBS, BL, SP, false, false>;
  SMPPI_CASE(64, 1) SMPPI_CASE(64, 2) SMPPI_CASE(64, 4)
  SMPPI_CASE(128, 1) SMPPI_CASE(128, 2) SMPPI_CASE(128, 4)
  SMPPI_CASE_F(256, 1) SMPPI_CASE_F(256, 2) SMPPI_CASE_F(256, 4)
  SMPPI_CASE_F(512, 1) SMPPI_CASE_F(512, 2)
#undef SMPPI_CASE
#undef SMPPI_CASE_F
  return nullptr;
}

template <int NOBS>
FusedFn pick_pipe(bool fuse) {
  return fuse ? k_fused<NOBS, PIPE_BLK, 1, true, true> : k_fused<NOBS, PIPE_BLK, 1, true, false>;
}

}  // namespace

struct smppi_plan_s {
  smppi_ctx ctx = nullptr;
  smppi_batch batch{};
  smppi_model model{};
  smppi_cost cost{};
  smppi_noise noise{};
  smppi_track track{};
  smppi_plan_opts opts{};
  smppi_plan_buffers bufs{};
  FusedArgs fa{};
  FusedFn fn = nullptr;
  int grid = 0, block = 256, lds = 0;
  bool any_empty = false;
  bool fused_shield = false;  // shield (+ execute) run inside k_fused
  // device allocations owned by the plan
  int2* tiles = nullptr;
  int32_t* tile_off = nullptr;
  float* part = nullptr;
  uint32_t* counters = nullptr;  // [0] queue, [1..B] tickets, [B+1] exits
  float4* obs_pad = nullptr;     // [B][kMaxObs] obstacle slots (tile mode with obstacles)
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  hipEvent_t ek[4] = {nullptr, nullptr, nullptr, nullptr};  // k_fused, k_repair start/stop
};

static smppi_status ensure_events(smppi_plan p, hipEvent_t* e, int n) {
  for (int i = 0; i < n; ++i)
    if (!e[i]) {
      hipError_t r = hipEventCreate(&e[i]);
      if (r != hipSuccess) return hip_fail(p->ctx, r, "hipEventCreate");
    }
  return SMPPI_OK;
}

static smppi_status mark(smppi_plan p, hipStream_t s, int i, bool profiled) {
  if (!profiled) return SMPPI_OK;
  smppi_status st = ensure_events(p, p->ev + i, 1);
  if (st) return st;
  hipError_t e = hipEventRecord(p->ev[i], s);
  if (e != hipSuccess) return hip_fail(p->ctx, e, "hipEventRecord");
  return SMPPI_OK;
}

// Records event i of a profiled launch (no-op for ordinary launches).
static smppi_status mark(smppi_plan p, hipStream_t s, int i, bool profiled);

static smppi_status plan_enqueue(smppi_plan p, hipStream_t s, bool profiled = false) {
  smppi_ctx ctx = p->ctx;
  const int B = p->batch.n_problems;
  smppi_status st0 = mark(p, s, 0, profiled);
  if (st0) return st0;
  if (profiled && (st0 = ensure_events(p, p->ek, 4))) return st0;
  smppi_status st = SMPPI_OK;
  if (p->any_empty) {
    hipLaunchKernelGGL(k_copy_empty, dim3(B), dim3(64), 0, s, p->batch.k_off, p->batch.t_off,
                       static_cast<const float*>(p->bufs.V), static_cast<float*>(p->bufs.V_plus),
                       static_cast<float*>(p->bufs.stats));
    if ((st = check_launch(ctx, "k_copy_empty"))) return st;
  }
  if (p->obs_pad && p->fa.n_tiles > 0) {
    hipLaunchKernelGGL(k_pad_obs, dim3(B), dim3(kMaxObs), 0, s, static_cast<const int32_t*>(p->track.obs_off),
                       static_cast<const float*>(p->track.obs), p->fa.p.obs_max, kMaxObs, p->fa.C.alpha, p->obs_pad);
    if ((st = check_launch(ctx, "k_pad_obs"))) return st;
  }
  if (p->fa.n_tiles > 0) {
    if (profiled)  // events stamped with the kernel's own start and end
      hipExtLaunchKernelGGL(p->fn, dim3(p->grid), dim3(p->block), (uint32_t)p->lds, s, p->ek[0], p->ek[1], 0u, p->fa);
    else
      hipLaunchKernelGGL(p->fn, dim3(p->grid), dim3(p->block), p->lds, s, p->fa);
    if ((st = check_launch(ctx, "k_fused"))) return st;
  }
  if ((st = mark(p, s, 1, profiled))) return st;
  if (p->opts.repair && !p->fused_shield) {
    // with execute on, the shield kernel also runs the plant step and warm start
    const ExecFuse ef{p->opts.dist, p->opts.n_dist, p->bufs.x0, p->bufs.V, p->bufs.iter};
    if ((st = repair_t<float>(ctx, &p->batch, &p->model, &p->cost, &p->track, p->bufs.x0, p->bufs.V_plus,
                              &p->opts.repair_opts, p->bufs.V_safe, s, profiled ? p->ek[2] : nullptr,
                              profiled ? p->ek[3] : nullptr, p->opts.execute ? &ef : nullptr)))
      return st;
  }
  if ((st = mark(p, s, 2, profiled))) return st;
  if (p->opts.execute && !p->opts.repair) {  // (with the shield, it runs the plant step)
    const void* V_exec = p->bufs.V_plus;
    if ((st = execute_t<float>(ctx, &p->batch, &p->model, V_exec, p->bufs.V_plus, p->opts.dist, p->opts.n_dist,
                               p->bufs.x0, p->bufs.V, p->bufs.iter, s)))
      return st;
  }
  return mark(p, s, 3, profiled);
}

extern "C" void smppi_plan_destroy(smppi_plan p) {
  if (!p) return;
  (void)hipSetDevice(p->ctx->device);
  (void)hipDeviceSynchronize();
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
  for (hipEvent_t e : p->ev)
    if (e) (void)hipEventDestroy(e);
  for (hipEvent_t e : p->ek)
    if (e) (void)hipEventDestroy(e);
  if (p->tiles) (void)hipFree(p->tiles);
  if (p->tile_off) (void)hipFree(p->tile_off);
  if (p->part) (void)hipFree(p->part);
  if (p->counters) (void)hipFree(p->counters);
  if (p->obs_pad) (void)hipFree(p->obs_pad);
  delete p;
}

extern "C" smppi_status smppi_plan_create(smppi_ctx ctx, const smppi_batch* batch, const smppi_model* model,
                                          const smppi_cost* cost, const smppi_noise* noise,
                                          const smppi_track* track, const smppi_plan_opts* opts,
                                          const smppi_plan_buffers* bufs, smppi_plan* out) {
  if (!ctx || !out) return SMPPI_ERR_INVALID_ARGUMENT;
  *out = nullptr;
  smppi_status st;
  if ((st = validate_batch(ctx, batch)) || (st = validate_model(ctx, model)) || (st = validate_cost(ctx, cost)) ||
      (st = validate_track(ctx, track, batch->dtype, batch->t_max)))
    return st;
  if (batch->dtype != SMPPI_F32) return fail(ctx, SMPPI_ERR_DTYPE, "plans run in FP32 only");
  if (!noise || !opts || !bufs) return fail(ctx, SMPPI_ERR_INVALID_ARGUMENT, "noise, opts, bufs are required");
  if (!(opts->lambda > 0.0) || !std::isfinite(opts->lambda))
    return fail(ctx, SMPPI_ERR_INVALID_ARGUMENT, "opts.lambda must be > 0");
  if (!bufs->x0 || !bufs->V || !bufs->iter || !bufs->S || !bufs->V_plus || !bufs->stats)
    return fail(ctx, SMPPI_ERR_INVALID_ARGUMENT, "plan buffers x0, V, iter, S, V_plus, stats are required");
  if (opts->repair && ((st = validate_repair(ctx, &opts->repair_opts)))) return st;
  if (opts->repair && !bufs->V_safe) return fail(ctx, SMPPI_ERR_INVALID_ARGUMENT, "V_safe required with repair");
  if (opts->execute && opts->dist && opts->n_dist < 0)
    return fail(ctx, SMPPI_ERR_INVALID_ARGUMENT, "n_dist must be >= 0");
  if (opts->fuse_shield < -1 || opts->fuse_shield > 1)
    return fail(ctx, SMPPI_ERR_INVALID_ARGUMENT, "fuse_shield must be -1, 0 or 1");
  if (opts->pipeline < -1 || opts->pipeline > 1)
    return fail(ctx, SMPPI_ERR_INVALID_ARGUMENT, "pipeline must be -1, 0 or 1");
  (void)hipSetDevice(ctx->device);
  const int B = batch->n_problems;

  // Host copies of the CSR offsets for the tile list (creation-time only).
  std::vector<int64_t> koff(B + 1);
  std::vector<int32_t> toff(B + 1);
  hipError_t e = hipMemcpy(koff.data(), batch->k_off, sizeof(int64_t) * (B + 1), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipMemcpy(k_off)");
  e = hipMemcpy(toff.data(), batch->t_off, sizeof(int32_t) * (B + 1), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipMemcpy(t_off)");
  // Latency mode when the whole batch gives at most two sample-waves per CU:
  // then each wave's per-step chain, not the VALU throughput, bounds the launch.
  // (Obstacles: the latency-mode kernel with 64 obstacle slots spills
  // registers, so it is used only when asked for.)
  const bool pipe = opts->pipeline == 1 ||
                    (opts->pipeline == 0 && track->obs_max == 0 &&
                     koff[B] <= (int64_t)2 * WAVE * std::max(ctx->n_cu, 1));
  const int block = pipe ? PIPE_BLK : (opts->block ? opts->block : 256);
  // Two samples per thread once the batch has at least 8 two-sample tiles per CU
  // (halves the tile partials the combine reads; measured faster on large ragged
  // batches); one otherwise, so that smaller batches still fill every CU.
  const bool two = koff[B] >= (int64_t)16 * block * std::max(ctx->n_cu, 1);
  const int tile = pipe ? WAVE : (opts->tile ? opts->tile : (two ? 2 * block : block));
  if (!pipe && block != 64 && block != 128 && block != 256 && block != 512)
    return fail(ctx, SMPPI_ERR_INVALID_ARGUMENT, "block must be 64, 128, 256 or 512");
  if (!pipe && tile % block != 0)
    return fail(ctx, SMPPI_ERR_INVALID_ARGUMENT, "tile must be a multiple of block");
  const int spt = tile / block;
  // the shield inside the launch when the workgroup has three waves (the LDS check
  // below may still turn it off): by default only in latency mode.  A tile-mode
  // launch with the shield compiled in needs more registers in every tile (fewer
  // waves per SIMD for the whole batch), and its shield shares a compute unit with
  // rollout tiles (chunk barriers instead of step counters); there the separate
  // shield kernel was measured faster (64 x K = 4096: 0.224 -> 0.157 ms, 512
  // problems: 1.17 -> 0.87 ms), in latency mode the fused one (8 problems: 0.075 vs
  // 0.079 ms; the headline launch).
  const bool want_fuse = opts->repair && block >= 3 * WAVE &&
                         (opts->fuse_shield == 1 || (opts->fuse_shield == 0 && pipe));
  auto pick = [&](bool fuse) -> FusedFn {
    if (pipe) return track->obs_max > 0 ? pick_pipe<kMaxObs>(fuse) : pick_pipe<0>(fuse);
    return track->obs_max > 0 ? pick_fused<kMaxObs>(block, spt, fuse) : pick_fused<0>(block, spt, fuse);
  };
  FusedFn fn = pick(false);
  if (!fn) return fail(ctx, SMPPI_ERR_UNSUPPORTED, "no fused kernel for block %d, tile %d", block, tile);
  std::vector<int32_t> ntile(B), tile_off(B + 1, 0);
  bool any_empty = false;
  for (int b = 0; b < B; ++b) {
    const int64_t K = koff[b + 1] - koff[b];
    const int T = toff[b + 1] - toff[b];
    if (K < 0 || K > batch->k_max || T < 1 || T > batch->t_max)
      return fail(ctx, SMPPI_ERR_SHAPE, "problem %d: K=%lld T=%d outside k_max/t_max", b, (long long)K, T);
    ntile[b] = (int)((K + tile - 1) / tile);
    tile_off[b + 1] = tile_off[b] + ntile[b];
    any_empty = any_empty || K == 0;
  }
  const int n_tiles = tile_off[B];
  // Longest-processing-time order: problems by T (tile cost ~ tile * T), descending.
  std::vector<int> order(B);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
    return (toff[x + 1] - toff[x]) > (toff[y + 1] - toff[y]);
  });
  std::vector<int2> tl;
  tl.reserve(n_tiles);
  for (int b : order)
    for (int k = 0; k < ntile[b]; ++k) tl.push_back(make_int2(b, k));

  smppi_plan p = new smppi_plan_s();
  p->ctx = ctx;
  p->batch = *batch;
  p->model = *model;
  p->cost = *cost;
  p->noise = *noise;
  p->track = *track;
  p->opts = *opts;
  p->bufs = *bufs;
  p->block = block;
  p->fn = fn;
  p->any_empty = any_empty;
  auto bail = [&](smppi_status s2) {
    smppi_plan_destroy(p);
    return s2;
  };
  const int pstride = part_stride(batch->t_max);
  if ((e = hipMalloc(&p->tiles, sizeof(int2) * std::max(1, n_tiles))) != hipSuccess ||
      (e = hipMalloc(&p->tile_off, sizeof(int32_t) * (B + 1))) != hipSuccess ||
      (e = hipMalloc(&p->part, sizeof(float) * (size_t)std::max(1, n_tiles) * pstride)) != hipSuccess ||
      (e = hipMalloc(&p->counters, sizeof(uint32_t) * (B + 2))) != hipSuccess)
    return bail(hip_fail(ctx, e, "hipMalloc(plan)"));
  if (n_tiles > 0 && (e = hipMemcpy(p->tiles, tl.data(), sizeof(int2) * n_tiles, hipMemcpyHostToDevice)) != hipSuccess)
    return bail(hip_fail(ctx, e, "hipMemcpy(tiles)"));
  if ((e = hipMemcpy(p->tile_off, tile_off.data(), sizeof(int32_t) * (B + 1), hipMemcpyHostToDevice)) != hipSuccess)
    return bail(hip_fail(ctx, e, "hipMemcpy(tile_off)"));
  if ((e = hipMemset(p->counters, 0, sizeof(uint32_t) * (B + 2))) != hipSuccess)
    return bail(hip_fail(ctx, e, "hipMemset(counters)"));
  // tile mode with obstacles reads them from padded slots (one per lane of each wave)
  if (!pipe && obs_slots(track) > 0 &&
      (e = hipMalloc(&p->obs_pad, sizeof(float4) * (size_t)B * kMaxObs)) != hipSuccess)
    return bail(hip_fail(ctx, e, "hipMalloc(obs_pad)"));

  FusedArgs& a = p->fa;
  a.p = problem_args<float>(ctx, &p->batch, &p->track, &p->noise, bufs->x0, bufs->iter);
  a.M = dev_model<float>(model);
  a.C = dev_cost<float>(cost);
  a.V = static_cast<const float*>(bufs->V);
  a.S = static_cast<float*>(bufs->S);
  a.V_plus = static_cast<float*>(bufs->V_plus);
  a.stats = static_cast<float*>(bufs->stats);
  a.inv_lambda = (float)(1.0 / opts->lambda);
  a.tiles = p->tiles;
  a.one = 0;
  if (B == 1) {
    // problem 0's dimensions for the one-problem path, checked as load_dims does
    // (an invalid problem keeps the general path, whose kernels flag it)
    int32_t po[2] = {0, 0}, oo[2] = {0, 0};
    if (track->poly_off && (e = hipMemcpy(po, track->poly_off, sizeof(po), hipMemcpyDeviceToHost)) != hipSuccess)
      return bail(hip_fail(ctx, e, "hipMemcpy(poly_off)"));
    if (track->obs_off && (e = hipMemcpy(oo, track->obs_off, sizeof(oo), hipMemcpyDeviceToHost)) != hipSuccess)
      return bail(hip_fail(ctx, e, "hipMemcpy(obs_off)"));
    ProblemDims& d = a.d1;
    d.k0 = koff[0];
    d.K = (int)(koff[1] - koff[0]);
    d.t0 = toff[0];
    d.T = toff[1] - toff[0];
    d.p0 = po[0];
    d.np = po[1] - po[0];
    d.o0 = oo[0];
    d.no = oo[1] - oo[0];
    const bool ok = d.T >= 1 && d.T <= batch->t_max && koff[1] - koff[0] >= 0 && koff[1] - koff[0] <= batch->k_max &&
                    d.np >= 0 && d.np <= track->poly_max && !(d.np > 0 && 2 * track->window + 1 > d.np) &&
                    d.no >= 0 && d.no <= track->obs_max;
    a.one = ok ? 1 : 0;
  }
  a.tile_off = p->tile_off;
  a.n_tiles = n_tiles;
  a.tile = tile;
  a.part = p->part;
  a.queue = p->counters;
  a.tickets = p->counters + 1;
  a.exits = p->counters + 1 + B;
  a.obs_pad = p->obs_pad;
  p->lds = (int)stage_lds_bytes<float>(track->poly_max, batch->t_max, obs_slots(track));
  hipFuncAttributes fattr{};
  if ((e = hipFuncGetAttributes(&fattr, reinterpret_cast<const void*>(fn))) != hipSuccess)
    return bail(hip_fail(ctx, e, "hipFuncGetAttributes"));
  if (fattr.sharedSizeBytes + p->lds > (size_t)ctx->max_lds)
    return bail(fail(ctx, SMPPI_ERR_SHAPE, "fused kernel needs %zu B of LDS per workgroup (device max %d)",
                     fattr.sharedSizeBytes + p->lds, ctx->max_lds));
  // The shield (and execute) inside the fused launch: the workgroup that
  // combines a problem runs Algorithm 1 on it right away.
  a.repair = 0;
  a.rep = RepairArgs<float>{};
  const int mem = opts->repair_opts.method == 1 ? opts->repair_opts.memory : 0;
  size_t lds_static = fattr.sharedSizeBytes;
  bool fuse = false;
  if (want_fuse) {
    // the variant with the shield compiled in, when its LDS fits
    const FusedFn fn_f = pick(true);
    hipFuncAttributes fa2{};
    if ((e = hipFuncGetAttributes(&fa2, reinterpret_cast<const void*>(fn_f))) != hipSuccess)
      return bail(hip_fail(ctx, e, "hipFuncGetAttributes"));
    if (fa2.sharedSizeBytes + p->lds + repair_lds_bytes<float>(batch->t_max, mem, false, pipe) <= (size_t)ctx->max_lds) {
      fn = fn_f;
      p->fn = fn;
      lds_static = fa2.sharedSizeBytes;
      fuse = true;
    }
  }
  if (fuse) {
    const ExecFuse ef{opts->dist, opts->n_dist, bufs->x0, bufs->V, bufs->iter};
    a.repair = 1;
    a.rep = repair_args<float>(ctx, &p->batch, model, cost, &p->track, bufs->x0, bufs->V_plus, &opts->repair_opts,
                               bufs->V_safe, opts->execute ? &ef : nullptr);
    // the parallel reverse sweep only when its tables fit beside the fused kernel's LDS
    a.rep.par_rev = lds_static + p->lds + repair_lds_bytes<float>(batch->t_max, mem, true, pipe) <= (size_t)ctx->max_lds;
    p->lds += (int)repair_lds_bytes<float>(batch->t_max, mem, a.rep.par_rev != 0, pipe);
  }
  p->fused_shield = a.repair != 0;
  int per_cu = 0;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, block, p->lds);
  if (e != hipSuccess || per_cu < 1) per_cu = 1;
  int grid = opts->grid > 0 ? opts->grid : ctx->n_cu * per_cu;
  grid = std::max(1, std::min(grid, std::max(1, n_tiles)));
  p->grid = grid;
  // A graph only pays when the launch has several kernels; a single kernel is
  // launched directly (measured: the one-node graph adds about 4 us per launch).
  const int n_kernels = (any_empty ? 1 : 0) + (n_tiles > 0 ? (p->obs_pad ? 2 : 1) : 0) + (opts->repair && !p->fused_shield ? 1 : 0) +
                        (opts->execute && !opts->repair ? 1 : 0);
  if (opts->use_graph && n_kernels > 1) {
    if ((e = hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking)) != hipSuccess)
      return bail(hip_fail(ctx, e, "hipStreamCreate"));
    if ((e = hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal)) != hipSuccess)
      return bail(hip_fail(ctx, e, "hipStreamBeginCapture"));
    st = plan_enqueue(p, p->cap_stream);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(p->cap_stream, &g);
    if (st) {
      if (g) (void)hipGraphDestroy(g);
      return bail(st);
    }
    if (e != hipSuccess) return bail(hip_fail(ctx, e, "hipStreamEndCapture"));
    p->graph = g;
    if ((e = hipGraphInstantiate(&p->exec, g, nullptr, nullptr, 0)) != hipSuccess)
      return bail(hip_fail(ctx, e, "hipGraphInstantiate"));
  }
  *out = p;
  return SMPPI_OK;
}

extern "C" smppi_status smppi_plan_launch(smppi_plan p, void* stream) {
  if (!p) return SMPPI_ERR_INVALID_ARGUMENT;
  (void)hipSetDevice(p->ctx->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (p->exec) {
    hipError_t e = hipGraphLaunch(p->exec, s);
    if (e != hipSuccess) return hip_fail(p->ctx, e, "hipGraphLaunch");
    return SMPPI_OK;
  }
  return plan_enqueue(p, s);
}

extern "C" smppi_status smppi_plan_launch_profiled(smppi_plan p, void* stream) {
  if (!p) return SMPPI_ERR_INVALID_ARGUMENT;
  (void)hipSetDevice(p->ctx->device);
  return plan_enqueue(p, static_cast<hipStream_t>(stream), true);
}

extern "C" smppi_status smppi_plan_stage_ms(smppi_plan p, float* fused_ms, float* repair_ms, float* execute_ms) {
  if (!p || !p->ev[3]) return p ? smppi::fail(p->ctx, SMPPI_ERR_INVALID_ARGUMENT, "no profiled launch yet")
                                : SMPPI_ERR_INVALID_ARGUMENT;
  hipError_t e = hipEventSynchronize(p->ev[3]);
  if (e != hipSuccess) return hip_fail(p->ctx, e, "hipEventSynchronize");
  float t[3] = {0.f, 0.f, 0.f};
  for (int i = 0; i < 3; ++i) {
    e = hipEventElapsedTime(&t[i], p->ev[i], p->ev[i + 1]);
    if (e != hipSuccess) return hip_fail(p->ctx, e, "hipEventElapsedTime");
  }
  if (fused_ms) *fused_ms = t[0];
  if (repair_ms) *repair_ms = t[1];
  if (execute_ms) *execute_ms = t[2];
  return SMPPI_OK;
}

extern "C" smppi_status smppi_plan_kernel_ms(smppi_plan p, float* fused_ms, float* repair_ms) {
  if (!p || !p->ev[3]) return p ? smppi::fail(p->ctx, SMPPI_ERR_INVALID_ARGUMENT, "no profiled launch yet")
                                : SMPPI_ERR_INVALID_ARGUMENT;
  hipError_t e = hipEventSynchronize(p->ev[3]);
  if (e != hipSuccess) return hip_fail(p->ctx, e, "hipEventSynchronize");
  float f = 0.f, r = 0.f;
  if (p->fa.n_tiles > 0 && (e = hipEventElapsedTime(&f, p->ek[0], p->ek[1])) != hipSuccess)
    return hip_fail(p->ctx, e, "hipEventElapsedTime");
  if (p->opts.repair && !p->fused_shield && (e = hipEventElapsedTime(&r, p->ek[2], p->ek[3])) != hipSuccess)
    return hip_fail(p->ctx, e, "hipEventElapsedTime");
  if (fused_ms) *fused_ms = f;
  if (repair_ms) *repair_ms = r;
  return SMPPI_OK;
}

// Launch geometry actually used by a plan: grid, block, tile, tiles.
extern "C" smppi_status smppi_plan_info(smppi_plan p, int32_t* grid, int32_t* block, int32_t* tile,
                                        int32_t* n_tiles) {
  if (!p) return SMPPI_ERR_INVALID_ARGUMENT;
  if (grid) *grid = p->grid;
  if (block) *block = p->block;
  if (tile) *tile = p->fa.tile;
  if (n_tiles) *n_tiles = p->fa.n_tiles;
  return SMPPI_OK;
}

// ---------------------------------------------------------------------------
// Launch-geometry autotuner.

namespace {

constexpr int kTuneBlocks[] = {64, 128, 256, 512};
constexpr int kTuneSpt[] = {1, 2, 4};
constexpr int kTuneGridPerCu[] = {0, 1, 2, 4};  // 0: occupancy-derived

std::vector<smppi_tune_entry> default_candidates(int n_cu) {
  std::vector<smppi_tune_entry> c;
  c.push_back(smppi_tune_entry{1, 0, 0, 0, 0.f});
  for (int block : kTuneBlocks)
    for (int spt : kTuneSpt) {
      if (block * spt > 1024) continue;
      for (int g : kTuneGridPerCu) c.push_back(smppi_tune_entry{-1, block, block * spt, g * n_cu, 0.f});
    }
  return c;
}

// The cache file: one "key pipeline block tile grid kernel_ms" line per key.
bool cache_lookup(const char* path, const std::string& key, smppi_tune_entry* e) {
  FILE* f = std::fopen(path, "r");
  if (!f) return false;
  char k[256];
  smppi_tune_entry t{};
  bool found = false;
  while (std::fscanf(f, "%255s %d %d %d %d %f", k, &t.pipeline, &t.block, &t.tile, &t.grid, &t.kernel_ms) == 6)
    if (key == k) {
      *e = t;
      found = true;
    }
  std::fclose(f);
  return found;
}

bool cache_store(const char* path, const std::string& key, const smppi_tune_entry& e) {
  std::vector<std::string> keep;
  if (FILE* f = std::fopen(path, "r")) {
    char line[512];
    while (std::fgets(line, sizeof line, f)) {
      char k[256];
      if (std::sscanf(line, "%255s", k) == 1 && key != k) keep.emplace_back(line);
    }
    std::fclose(f);
  }
  const std::string tmp = std::string(path) + ".tmp";
  FILE* f = std::fopen(tmp.c_str(), "w");
  if (!f) return false;
  bool ok = true;
  for (const std::string& l : keep) ok = ok && std::fputs(l.c_str(), f) >= 0;
  ok = ok && std::fprintf(f, "%s %d %d %d %d %.6g\n", key.c_str(), e.pipeline, e.block, e.tile, e.grid,
                          (double)e.kernel_ms) > 0;
  ok = (std::fclose(f) == 0) && ok;
  if (!ok || std::rename(tmp.c_str(), path) != 0) {
    std::remove(tmp.c_str());
    return false;
  }
  return true;
}

}  // namespace

extern "C" int32_t smppi_autotune_candidates(int32_t n_cu, smppi_tune_entry* out, int32_t cap) {
  const std::vector<smppi_tune_entry> c = default_candidates(std::max(0, n_cu));
  for (int i = 0; out && i < cap && i < (int)c.size(); ++i) out[i] = c[i];
  return (int32_t)c.size();
}

extern "C" smppi_status smppi_autotune_key(int32_t n_problems, const int64_t* k_off_host, const int32_t* t_off_host,
                                           int32_t has_obstacles, int32_t n_cu, char* out, int32_t cap) {
  if (n_problems < 1 || !k_off_host || !t_off_host || !out || cap < 1) return SMPPI_ERR_INVALID_ARGUMENT;
  int64_t sum_k = 0, k_max = 0;
  int32_t t_max = 0;
  double t_sum = 0.0;
  for (int b = 0; b < n_problems; ++b) {
    const int64_t K = k_off_host[b + 1] - k_off_host[b];
    const int32_t T = t_off_host[b + 1] - t_off_host[b];
    sum_k += K;
    k_max = std::max(k_max, K);
    t_max = std::max(t_max, T);
    t_sum += T;
  }
  const long octave = sum_k > 0 ? std::lround(8.0 * std::log2((double)sum_k)) : -1;
  const int n = std::snprintf(out, (size_t)cap, "B%d-sk%ld-kmax%lld-tmax%d-tmean%.1f-obs%d-cu%d", n_problems, octave,
                              (long long)k_max, t_max, t_sum / n_problems, has_obstacles ? 1 : 0, n_cu);
  return (n < 0 || n >= cap) ? SMPPI_ERR_INVALID_ARGUMENT : SMPPI_OK;
}

extern "C" smppi_status smppi_autotune(smppi_ctx ctx, const smppi_batch* batch, const smppi_model* model,
                                       const smppi_cost* cost, const smppi_noise* noise, const smppi_track* track,
                                       double lambda, const smppi_plan_buffers* bufs, const smppi_tune_entry* cands,
                                       int32_t n_cands, int32_t reps, int32_t warmup, const char* cache_path,
                                       int32_t force, smppi_tune_entry* best, int32_t* cached,
                                       smppi_tune_entry* table, int32_t table_cap, int32_t* n_table, void* stream) {
  if (!ctx) return SMPPI_ERR_INVALID_ARGUMENT;
  if (!best || !bufs || !batch || !track) return fail(ctx, SMPPI_ERR_INVALID_ARGUMENT, "batch, track, bufs, best are required");
  if (cands && n_cands < 1) return fail(ctx, SMPPI_ERR_INVALID_ARGUMENT, "n_cands must be >= 1 with cands");
  if (reps < 1 || warmup < 0) return fail(ctx, SMPPI_ERR_INVALID_ARGUMENT, "reps must be >= 1, warmup >= 0");
  if (table_cap < 0 || (table_cap > 0 && !table)) return fail(ctx, SMPPI_ERR_INVALID_ARGUMENT, "table_cap without table");
  smppi_status st = validate_batch(ctx, batch);
  if (st) return st;
  if (cached) *cached = 0;
  if (n_table) *n_table = 0;
  (void)hipSetDevice(ctx->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int B = batch->n_problems;
  std::vector<int64_t> koff(B + 1);
  std::vector<int32_t> toff(B + 1);
  hipError_t e = hipMemcpy(koff.data(), batch->k_off, sizeof(int64_t) * (B + 1), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipMemcpy(k_off)");
  e = hipMemcpy(toff.data(), batch->t_off, sizeof(int32_t) * (B + 1), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipMemcpy(t_off)");
  char keybuf[256];
  if ((st = smppi_autotune_key(B, koff.data(), toff.data(), track->obs_max > 0, ctx->n_cu, keybuf, sizeof keybuf)))
    return fail(ctx, st, "batch shape key");
  const std::string key(keybuf);
  if (cache_path && !force) {
    smppi_tune_entry hit{};
    if (cache_lookup(cache_path, key, &hit)) {
      *best = hit;
      if (cached) *cached = 1;
      if (table && table_cap > 0) table[0] = hit;
      if (n_table) *n_table = 1;
      return SMPPI_OK;
    }
  }
  const std::vector<smppi_tune_entry> cand =
      cands ? std::vector<smppi_tune_entry>(cands, cands + n_cands) : default_candidates(ctx->n_cu);
  smppi_plan_opts o{};
  o.lambda = lambda;
  o.use_graph = 0;
  o.fuse_shield = -1;
  smppi_plan_buffers pb = *bufs;
  pb.V_safe = nullptr;
  std::vector<smppi_tune_entry> done, skipped;
  std::vector<float> ms;
  for (smppi_tune_entry c : cand) {
    o.pipeline = c.pipeline == 1 ? 1 : -1;
    o.block = c.pipeline == 1 ? 0 : c.block;
    o.tile = c.pipeline == 1 ? 0 : c.tile;
    o.grid = c.grid;
    smppi_plan p = nullptr;
    if (smppi_plan_create(ctx, batch, model, cost, noise, track, &o, &pb, &p) != SMPPI_OK) {
      c.kernel_ms = -1.f;  // not buildable for this batch (block, LDS)
      skipped.push_back(c);
      continue;
    }
    ms.clear();
    for (int i = 0; i < warmup + reps && st == SMPPI_OK; ++i) {
      float f = 0.f;
      if ((st = smppi_plan_launch_profiled(p, s)) == SMPPI_OK && (st = smppi_plan_kernel_ms(p, &f, nullptr)) == SMPPI_OK &&
          i >= warmup)
        ms.push_back(f);
    }
    smppi_plan_destroy(p);
    if (st) return st;
    std::nth_element(ms.begin(), ms.begin() + ms.size() / 2, ms.end());
    c.kernel_ms = ms[ms.size() / 2];
    done.push_back(c);
  }
  if (done.empty()) return fail(ctx, SMPPI_ERR_SHAPE, "no candidate geometry can be built for this batch");
  std::stable_sort(done.begin(), done.end(),
                   [](const smppi_tune_entry& x, const smppi_tune_entry& y) { return x.kernel_ms < y.kernel_ms; });
  *best = done[0];
  done.insert(done.end(), skipped.begin(), skipped.end());
  for (int i = 0; table && i < table_cap && i < (int)done.size(); ++i) table[i] = done[i];
  if (n_table) *n_table = (int32_t)done.size();
  if (cache_path && !cache_store(cache_path, key, done[0]))
    return fail(ctx, SMPPI_ERR_HIP, "could not write the tuning cache %s", cache_path);
  return SMPPI_OK;
}
