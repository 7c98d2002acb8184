// gfx950 kernels of the plain (one call per stage) sampled-rollout path, and
// the device functions the batched plan shares with it (problem staging, block
// reductions, noise sums, the shield of Algorithm 1 and its L-BFGS variant,
// the plant step).
#pragma once

#include "device.hpp"

namespace smppi {

// Device-side input errors (bounds a kernel relies on); OR-ed into ctx->err.
enum : uint32_t {
  DERR_T = 1u,        // T_b outside [1, t_max]
  DERR_K = 2u,        // K_b outside [0, k_max]
  DERR_POLY = 4u,     // N_b > poly_max or window too wide for N_b
  DERR_OBS = 8u,      // O_b > obs_max
  DERR_WAIT = 16u,    // a wave's wait for another wave of its workgroup exceeded its bound
};

template <class R>
struct ProblemArgs {
  const int64_t* k_off;
  const int32_t* t_off;
  const int32_t* poly_off;
  const R* poly;
  const R* circle;
  const R* half_width;
  const int32_t* obs_off;
  const R* obs;
  const R* x0;
  const uint32_t* iter;
  int32_t k_max, t_max, poly_max, obs_max, window, pid_base;
  uint32_t seed;
  int32_t nominal;
  uint32_t* err;
};

struct ProblemDims {
  int64_t k0;
  int K, t0, T, p0, np, o0, no;
};

template <class R>
__device__ __forceinline__ bool load_dims(const ProblemArgs<R>& a, int b, ProblemDims& d) {
  d.k0 = a.k_off[b];
  const int64_t K = a.k_off[b + 1] - d.k0;
  d.t0 = a.t_off[b];
  d.T = a.t_off[b + 1] - d.t0;
  d.p0 = a.poly_off ? a.poly_off[b] : 0;
  d.np = a.poly_off ? a.poly_off[b + 1] - d.p0 : 0;
  d.o0 = a.obs_off ? a.obs_off[b] : 0;
  d.no = a.obs_off ? a.obs_off[b + 1] - d.o0 : 0;
  uint32_t e = 0;
  if (d.T < 1 || d.T > a.t_max) e |= DERR_T;
  if (K < 0 || K > a.k_max) e |= DERR_K;
  if (d.np < 0 || d.np > a.poly_max || (d.np > 0 && 2 * a.window + 1 > d.np)) e |= DERR_POLY;
  if (d.no < 0 || d.no > a.obs_max) e |= DERR_OBS;
  d.K = (int)K;
  if (e) {
    if (threadIdx.x == 0) atomicOr(a.err, e);
    return false;
  }
  return true;
}

// Lexicographic minimum of (distance, index) over a wave, in every lane (the
// whole wave active; an infinite or NaN distance never wins, as in a scan with
// a strict "<").  FP64: butterfly shuffles.  FP32: distances are non-negative,
// so their bit patterns order like their values; two integer minima (distance,
// then the index among the lanes holding it), each four DPP row rotations and
// a scalar minimum over the four rows.
template <class R>
__device__ __forceinline__ void wave_argmin(R& bd, int& bi) {
#pragma unroll
  for (int o = WAVE / 2; o > 0; o >>= 1) {
    const R od = __shfl_xor(bd, o, WAVE);
    const int oi = __shfl_xor(bi, o, WAVE);
    if (od < bd || (od == bd && oi < bi)) {
      bd = od;
      bi = oi;
    }
  }
}
template <>
__device__ __forceinline__ void wave_argmin<float>(float& bd, int& bi) {
  const unsigned key = bd < INFINITY ? __float_as_uint(bd) : 0xFFFFFFFFu;
  const unsigned m = wave_min_u32(key);
  const unsigned mi = wave_min_u32(key == m ? (unsigned)bi : 0x7fffffffu);
  const bool none = m == 0xFFFFFFFFu;
  bd = none ? INFINITY : __uint_as_float(m);
  bi = none ? 0x7fffffff : (int)mi;
}

// Stages problem b's polyline, obstacles and control sequence in LDS; returns
// the track view.  LDS layout: seg [poly_max][4] | obs [obs_max][4] |
// il2 [poly_max] | V [2][t_max].
//
// The staging is one memory round trip for the usual sizes: every thread
// issues its loads (start position, first V element, first obstacle word, up to
// STAGE_U polyline rows) before the first LDS store.
constexpr int STAGE_U = 4;
template <class R>
__device__ TrackView<R> stage_problem(const ProblemArgs<R>& a, int b, const ProblemDims& d, const R* __restrict__ Vg,
                                      unsigned char* smem, R** Vs_out) {
  // The closed polyline is stored with SEG_PAD wrapped copies on each side, so
  // a window around any segment reads consecutive slots without index wrapping.
  const int ns = a.poly_max + 2 * SEG_PAD;
  R* seg = reinterpret_cast<R*>(smem);
  R* obs = seg + 4 * ns;
  R* il2 = obs + 4 * a.obs_max;
  R* Vs = il2 + ns;
  const int tid = threadIdx.x, nt = blockDim.x;
  // start position (for the nearest segment below), loaded with the rest
  const R px = a.x0[6 * (size_t)b], py = a.x0[6 * (size_t)b + 1];
  // Obstacle slots beyond the problem's own count hold an inert barrier
  // (h = |p|^2 + 1e30 > 0 everywhere, never violated, never hit), so the
  // per-step loops run a fixed count without per-obstacle branches.
  auto obs_word = [&](int i) { return i < 4 * d.no ? a.obs[4 * (size_t)d.o0 + i] : ((i & 3) >= 2 ? R(-1e30) : R(0)); };
  const R v_first = tid < 2 * d.T ? Vg[2 * (size_t)d.t0 + tid] : R(0);
  const R o_first = tid < 4 * a.obs_max ? obs_word(tid) : R(0);
  // Polyline rows (a_x, a_y, d_x, d_y, 1/|d|^2): the np rows in batches of
  // STAGE_U per thread, and the 2 SEG_PAD wrapped copies on threads below
  // 2 SEG_PAD, loaded beside the first batch.
  const bool pad_t = d.np > 0 && tid < 2 * SEG_PAD;
  const int pad_slot = tid < SEG_PAD ? tid : d.np + tid;  // slot in the padded copy
  R prow[5];
  if (pad_t) {
    const int src = ((pad_slot - SEG_PAD) % d.np + d.np) % d.np;
    const R* sp = a.poly + 5 * (size_t)(d.p0 + src);
#pragma unroll
    for (int c = 0; c < 5; ++c) prow[c] = sp[c];
  }
  // Nearest segment to the start position (global search, lowest index on
  // ties): each thread tracks the first strict minimum over the rows it stages
  // (increasing index), computed from the rows in registers.
  R bd = R(INFINITY);
  int bi = 0x7fffffff;
  for (int r0 = 0; r0 < d.np; r0 += STAGE_U * nt) {
    R row[STAGE_U][5];
#pragma unroll
    for (int u = 0; u < STAGE_U; ++u) {
      const int k = r0 + u * nt + tid;
      if (k < d.np) {
        const R* sp = a.poly + 5 * (size_t)(d.p0 + k);
#pragma unroll
        for (int c = 0; c < 5; ++c) row[u][c] = sp[c];
      }
    }
#pragma unroll
    for (int u = 0; u < STAGE_U; ++u) {
      const int k = r0 + u * nt + tid, i = k + SEG_PAD;
      if (k < d.np) {
        seg[4 * i + 0] = row[u][0];
        seg[4 * i + 1] = row[u][1];
        seg[4 * i + 2] = row[u][2];
        seg[4 * i + 3] = row[u][3];
        il2[i] = row[u][4];
        const R dd = seg_dist2_row(row[u][0], row[u][1], row[u][2], row[u][3], row[u][4], px, py);
        if (dd < bd) {
          bd = dd;
          bi = k;
        }
      }
    }
  }
  if (pad_t) {
    seg[4 * pad_slot + 0] = prow[0];
    seg[4 * pad_slot + 1] = prow[1];
    seg[4 * pad_slot + 2] = prow[2];
    seg[4 * pad_slot + 3] = prow[3];
    il2[pad_slot] = prow[4];
  }
  if (tid < 2 * d.T) Vs[tid] = v_first;
  for (int i = tid + nt; i < 2 * d.T; i += nt) Vs[i] = Vg[2 * (size_t)d.t0 + i];
  if (tid < 4 * a.obs_max) obs[tid] = o_first;
  for (int i = tid + nt; i < 4 * a.obs_max; i += nt) obs[i] = obs_word(i);
  TrackView<R> tr;
  tr.n = d.np;
  tr.window = a.window;
  tr.seg = seg + 4 * SEG_PAD;
  tr.il2 = il2 + SEG_PAD;
  tr.cx = a.circle[3 * b + 0];
  tr.cy = a.circle[3 * b + 1];
  tr.rad = a.circle[3 * b + 2];
  const R w = a.half_width[b];
  tr.w2 = w * w;
  tr.obs = obs;
  tr.n_obs = d.no;
  tr.idx0 = 0;
  *Vs_out = Vs;
  // The start segment is shared by every sample: the waves' minima meet in LDS
  // (the barrier also publishes the staged rows; every caller synchronises
  // again before the staged problem is used, which also guards s_bd and s_bi
  // against the next staging).
  if (d.np > 0) {
    __shared__ R s_bd[32];
    __shared__ int s_bi[32];
    wave_argmin(bd, bi);
    if (tid % WAVE == 0) {
      s_bd[tid / WAVE] = bd;
      s_bi[tid / WAVE] = bi;
    }
    __syncthreads();
    bd = s_bd[0];
    bi = s_bi[0];
    for (int k = 1; k < nt / WAVE; ++k)
      if (s_bd[k] < bd || (s_bd[k] == bd && s_bi[k] < bi)) {
        bd = s_bd[k];
        bi = s_bi[k];
      }
    tr.idx0 = bi == 0x7fffffff ? 0 : bi;
  }
  return tr;
}

template <class R>
__host__ __device__ inline size_t stage_lds_bytes(int poly_max, int t_max, int obs_max) {
  // rounded up to 16 bytes: LDS placed after the staged problem starts aligned
  const size_t n = sizeof(R) * (5 * ((size_t)poly_max + 2 * SEG_PAD) + 2 * (size_t)t_max + 4 * (size_t)obs_max);
  return (n + 15) & ~(size_t)15;
}

template <class R>
__device__ __forceinline__ State<R> load_state(const R* x) {
  State<R> s;
  s.px = x[0];
  s.py = x[1];
  s.psi = x[2];
  s.vx = x[3];
  s.vy = x[4];
  s.om = x[5];
  return s;
}

// Block-wide reductions in a fixed order (lane tree, then waves in index order).
template <class R>
__device__ R block_sum(R v, R* red) {
  const int lane = threadIdx.x % WAVE, wv = threadIdx.x / WAVE, nw = blockDim.x / WAVE;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) red[wv] = v;
  __syncthreads();
  R s = R(0);
  for (int i = 0; i < nw; ++i) s += red[i];
  return s;
}
// Three block sums with one exchange (same order as block_sum); red: 3 * waves.
// LEAD = false drops the leading barrier, which only guards `red` against
// readers of its previous use: for callers that have passed a barrier since.
template <class R, bool LEAD = true>
__device__ void block_sum3(R& a, R& b, R& c, R* red) {
  const int lane = threadIdx.x % WAVE, wv = threadIdx.x / WAVE, nw = blockDim.x / WAVE;
  a = wave_sum(a);
  b = wave_sum(b);
  c = wave_sum(c);
  if (LEAD) __syncthreads();
  if (lane == 0) {
    red[wv] = a;
    red[nw + wv] = b;
    red[2 * nw + wv] = c;
  }
  __syncthreads();
  a = b = c = R(0);
  for (int i = 0; i < nw; ++i) {
    a += red[i];
    b += red[nw + i];
    c += red[2 * nw + i];
  }
}
template <class R, bool LEAD = true>
__device__ R block_min(R v, R* red) {
  const int lane = threadIdx.x % WAVE, wv = threadIdx.x / WAVE, nw = blockDim.x / WAVE;
  v = wave_min(v);
  if (LEAD) __syncthreads();
  if (lane == 0) red[wv] = v;
  __syncthreads();
  R s = red[0];
  for (int i = 1; i < nw; ++i) s = fmin(s, red[i]);
  return s;
}

// ============================================================== rollout
template <class R>
struct RolloutArgs {
  ProblemArgs<R> p;
  DevModel<R> M;
  DevCost<R> C;
  const R* V;
  R* S;
  R* eps_out;
  const float4* obs_pad;  // FP32 with obstacles: [B][NOBS] slots from k_pad_obs (WaveObstacles)
};

// Obstacle slots of every problem for the FP32 rollouts and adjoint
// (WaveObstacles): (c_x, c_y, r^2, (1 - alpha) ((r + margin)^2 - r^2)) for
// the problem's obstacles, the inert slot (0, 0, -1e30, 0) after them, n_slots
// per problem.  Runs before every launch that reads them, so obstacles the caller
// moves between launches are seen.  A problem whose obstacle count is out of
// range gets inert slots only (the rollout kernels flag and skip it).
// Grid: one workgroup per problem.
static __global__ void k_pad_obs(const int32_t* __restrict__ obs_off, const float* __restrict__ obs, int obs_max,
                          int n_slots, float alpha, float4* __restrict__ out) {
  const int b = blockIdx.x;
  const int o0 = obs_off ? obs_off[b] : 0, no = obs_off ? obs_off[b + 1] - o0 : 0;
  const bool ok = no >= 0 && no <= obs_max;
  for (int i = threadIdx.x; i < n_slots; i += blockDim.x) {
    float4 v = make_float4(0.f, 0.f, -1e30f, 0.f);
    if (ok && i < no) {
      const float* o = obs + 4 * ((size_t)o0 + i);
      v = make_float4(o[0], o[1], o[3], (1.f - alpha) * (o[2] - o[3]));
    }
    out[(size_t)b * n_slots + i] = v;
  }
}

template <class R, int NOBS>
__global__ __launch_bounds__(256) void k_rollout(RolloutArgs<R> a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int b = blockIdx.y;
  ProblemDims d;
  if (!load_dims(a.p, b, d)) return;
  const int m_base = blockIdx.x * blockDim.x;
  if (m_base >= d.K) return;
  R* Vs;
  const TrackView<R> tr = stage_problem(a.p, b, d, a.V, smem, &Vs);
  __syncthreads();
  const int m = m_base + threadIdx.x;
  constexpr bool WV = NOBS > 0 && sizeof(R) == 4;
  // The wave-level obstacle evaluation needs every lane of a wave: lanes past K
  // in a wave that has samples run a copy of the last sample and store nothing.
  if (WV ? (m - (int)(threadIdx.x % WAVE) >= d.K) : (m >= d.K)) return;
  const bool own = m < d.K;
  const int mr = own ? m : d.K - 1;
  NoiseStream<R> ns;
  ns.seed = a.p.seed;
  ns.m = (uint32_t)mr;
  ns.pid = (uint32_t)(a.p.pid_base + b);
  ns.it = a.p.iter[b];
  ns.nominal = a.p.nominal != 0;
  const State<R> x0 = load_state(a.p.x0 + 6 * (size_t)b);
  R* eo = (a.eps_out && own) ? a.eps_out + (size_t)(d.k0 + m) * a.p.t_max * 2 : nullptr;
  R s;
  if constexpr (WV)
    s = rollout_sample<R, NOBS>(a.M, a.C, tr, x0, Vs, d.T, ns, eo, WaveObstacles(a.obs_pad + (size_t)b * NOBS, NOBS));
  else
    s = rollout_sample<R, NOBS>(a.M, a.C, tr, x0, Vs, d.T, ns, eo);
  if (own) a.S[d.k0 + m] = s;
}

// ============================================================== weights
template <class R>
__global__ __launch_bounds__(256) void k_weights(const int64_t* __restrict__ k_off, const R* __restrict__ S,
                                                 R inv_lambda, R* __restrict__ w, R* __restrict__ stats) {
  __shared__ R red[256 / WAVE];
  const int b = blockIdx.x;
  const int64_t k0 = k_off[b];
  const int K = (int)(k_off[b + 1] - k0);
  R mn = R(INFINITY), nf = R(0);
  for (int m = threadIdx.x; m < K; m += blockDim.x) {
    const R s = S[k0 + m];
    if (isfinite(s)) mn = fmin(mn, s);
    else nf += R(1);
  }
  mn = block_min(mn, red);
  nf = block_sum(nf, red);
  R z = R(0), q = R(0);
  for (int m = threadIdx.x; m < K; m += blockDim.x) {
    const R s = S[k0 + m];
    const R om = isfinite(s) ? exp_r(-(s - mn) * inv_lambda) : R(0);
    z += om;
    q += om * om;
  }
  z = block_sum(z, red);
  q = block_sum(q, red);
  const R iz = z > R(0) ? R(1) / z : R(0);
  for (int m = threadIdx.x; m < K; m += blockDim.x) {
    const R s = S[k0 + m];
    const R om = isfinite(s) ? exp_r(-(s - mn) * inv_lambda) : R(0);
    w[k0 + m] = om * iz;
  }
  if (threadIdx.x == 0) {
    stats[4 * b + 0] = mn;
    stats[4 * b + 1] = log(z);
    stats[4 * b + 2] = q > R(0) ? z * z / q : R(0);
    stats[4 * b + 3] = nf;
  }
}

// ============================================================== update
// Per-step reduction of sum_m w_m eps'_{m,t} over a block's samples, written as
// block partials; the last block of each problem (ticket) sums the partials in
// block order and writes V+ = V + sum.
template <class R>
struct UpdateArgs {
  ProblemArgs<R> p;
  DevModel<R> M;
  DevCost<R> C;
  const R* V;
  const R* w;
  R* V_plus;
  R* part;            // [B][nblk_max][2][t_max]
  uint32_t* tickets;  // [B], zero between calls
  int nblk_max;
};

constexpr int UPD_BLOCK = 256;
constexpr int UPD_TCHUNK = 64;

// Release (every writer, before its ticket increment) and acquire (the last
// ticket holder, before it reads the partials) halves of the ticket protocol,
// at device scope.  A full __threadfence on the reader side would also write
// back the reader's L2, which costs microseconds and is not needed there.
__device__ __forceinline__ void ticket_release() { __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent"); }
__device__ __forceinline__ void ticket_acquire() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }

template <class R, int BLK, int SPT>
struct NoiseSumLds {
  int m[BLK * SPT];
  R w[BLK * SPT];
  int cnt[BLK / WAVE];
  R wpart[BLK / WAVE][2][UPD_TCHUNK];
  R red4[4][BLK];
};

// Weighted sums of a workgroup's effective noise, P[d*T + t] = sum_m w_m
// eps'_{m,t,d}, for the SPT samples (ms, ws) each thread holds.  Samples with
// a zero weight (most of them: exp(-(S - min S)/lambda) underflows) contribute
// nothing, so they are first compacted in ascending sample order; when few
// remain, each thread owns a time step and regenerates only the live samples'
// noise (no cross-lane reduction); otherwise every lane keeps its own sample
// and the per-step sums go through wave reductions.  Both orders are fixed.
template <class R, int BLK, int SPT, bool VG = false>
__device__ void block_noise_sums(const DevModel<R>& Mg, const DevCost<R>& Cg, uint32_t seed, uint32_t pid, uint32_t it,
                                 bool nominal, const R* V, int T, const int (&ms)[SPT], const R (&ws)[SPT],
                                 NoiseSumLds<R, BLK, SPT>& L, R* P) {
  // VG: model and cost constants in VGPRs (for kernels whose occupancy does
  // not depend on the VGPR count)
  DevModel<R> Mv;
  DevCost<R> Cv;
  if constexpr (VG) {
    Mv = model_in_vgprs(Mg);
    Cv = cost_in_vgprs(Cg);
  }
  const DevModel<R>& M = VG ? Mv : Mg;
  const DevCost<R>& C = VG ? Cv : Cg;
  constexpr int NW = BLK / WAVE;
  const int tid = threadIdx.x, lane = tid % WAVE, wv = tid / WAVE;
  int n_live = 0;
#pragma unroll
  for (int j = 0; j < SPT; ++j) {
    const bool f = ws[j] != R(0);
    const unsigned long long bal = __ballot(f);
    if (lane == 0) L.cnt[wv] = __popcll(bal);
    __syncthreads();
    int base = n_live, tot = 0;
    for (int i = 0; i < NW; ++i) {
      base += (i < wv) ? L.cnt[i] : 0;
      tot += L.cnt[i];
    }
    if (f) {
      const int pos = base + __popcll(bal & ((1ull << lane) - 1ull));
      L.m[pos] = ms[j];
      L.w[pos] = ws[j];
    }
    n_live += tot;
    __syncthreads();
  }
  // Sparse path: thread (g, j) owns the step pair (2j, 2j+1) (one Philox call
  // per live sample gives both steps) for the live samples i = g, g+G, ...;
  // the G partial sums of a pair are then added in g order.
  const int npairs = (T + 1) / 2;
  const int G = npairs >= BLK ? 1 : BLK / npairs;
  if (n_live <= G * T) {
    for (int j0 = 0; j0 < npairs; j0 += BLK / G) {
      const int j = j0 + tid % (BLK / G), g = tid / (BLK / G);
      R acc[4] = {R(0), R(0), R(0), R(0)};
      if (g < G && j < npairs) {
        const int ta = 2 * j, tb = min(2 * j + 1, T - 1);
        const R va0 = V[ta], va1 = V[T + ta], vb0 = V[tb], vb1 = V[T + tb];
        for (int i = g; i < n_live; i += G) {
          R z[4] = {R(0), R(0), R(0), R(0)};
          if (!nominal) normals4<R>(seed, (uint32_t)j, (uint32_t)L.m[i], pid, it, z);
          const R wi = L.w[i];
          acc[0] += wi * (clamp_r(va0 + C.sigma[0] * z[0], M.u_lo[0], M.u_hi[0]) - va0);
          acc[1] += wi * (clamp_r(va1 + C.sigma[1] * z[1], M.u_lo[1], M.u_hi[1]) - va1);
          acc[2] += wi * (clamp_r(vb0 + C.sigma[0] * z[2], M.u_lo[0], M.u_hi[0]) - vb0);
          acc[3] += wi * (clamp_r(vb1 + C.sigma[1] * z[3], M.u_lo[1], M.u_hi[1]) - vb1);
        }
      }
      const int per = BLK / G, jn = min(per, npairs - j0);
      if (g < G && j < npairs)
#pragma unroll
        for (int q = 0; q < 4; ++q) L.red4[q][g * per + tid % per] = acc[q];
      __syncthreads();
      for (int e = tid; e < 4 * jn; e += BLK) {
        const int q = e / jn, jj = e % jn;
        R s = R(0);
        for (int gg = 0; gg < G; ++gg) s += L.red4[q][gg * per + jj];
        const int t = 2 * (j0 + jj) + (q >> 1);
        if (t < T) P[(q & 1) * T + t] = s;
      }
      if (j0 + BLK / G < npairs) __syncthreads();  // red4 is written again
    }
    return;
  }
  NoiseStream<R> ns[SPT];
#pragma unroll
  for (int j = 0; j < SPT; ++j) {
    ns[j].seed = seed;
    ns[j].m = (uint32_t)ms[j];
    ns[j].pid = pid;
    ns[j].it = it;
    ns[j].nominal = nominal;
  }
  for (int tc = 0; tc < T; tc += UPD_TCHUNK) {
    const int tn = min(UPD_TCHUNK, T - tc);
    for (int tt = 0; tt < tn; ++tt) {
      const int t = tc + tt;
      const R v0 = V[t], v1 = V[T + t];
      R p0 = R(0), p1 = R(0);
#pragma unroll
      for (int j = 0; j < SPT; ++j) {
        if (ws[j] != R(0)) {
          R e0, e1;
          ns[j].at(t, C.sigma[0], C.sigma[1], e0, e1);
          p0 += ws[j] * (clamp_r(v0 + e0, M.u_lo[0], M.u_hi[0]) - v0);
          p1 += ws[j] * (clamp_r(v1 + e1, M.u_lo[1], M.u_hi[1]) - v1);
        }
      }
      p0 = wave_sum(p0);
      p1 = wave_sum(p1);
      if (lane == 0) {
        L.wpart[wv][0][tt] = p0;
        L.wpart[wv][1][tt] = p1;
      }
    }
    __syncthreads();
    for (int e = tid; e < 2 * tn; e += BLK) {
      const int dd = e / tn, tt = e % tn;
      R acc = R(0);
      for (int i = 0; i < NW; ++i) acc += L.wpart[i][dd][tt];
      P[dd * T + tc + tt] = acc;
    }
    __syncthreads();
  }
}

template <class R>
__global__ __launch_bounds__(UPD_BLOCK) void k_update(UpdateArgs<R> a) {
  __shared__ NoiseSumLds<R, UPD_BLOCK, 1> L;
  __shared__ uint32_t s_ticket;
  const int b = blockIdx.y;
  ProblemDims d;
  if (!load_dims(a.p, b, d)) return;
  const R* Vb = a.V + 2 * (size_t)d.t0;
  R* Vpb = a.V_plus + 2 * (size_t)d.t0;
  if (d.K == 0) {
    if (blockIdx.x == 0)
      for (int i = threadIdx.x; i < 2 * d.T; i += blockDim.x) Vpb[i] = Vb[i];
    return;
  }
  const int nblk = (d.K + UPD_BLOCK - 1) / UPD_BLOCK;
  if ((int)blockIdx.x >= nblk) return;
  const int m = blockIdx.x * UPD_BLOCK + threadIdx.x;
  const int ms[1] = {m};
  const R ws[1] = {(m < d.K) ? a.w[d.k0 + m] : R(0)};
  R* gp = a.part + ((size_t)b * a.nblk_max + blockIdx.x) * 2 * a.p.t_max;
  block_noise_sums<R, UPD_BLOCK, 1>(a.M, a.C, a.p.seed, (uint32_t)(a.p.pid_base + b), a.p.iter[b],
                                    a.p.nominal != 0, Vb, d.T, ms, ws, L, gp);
  ticket_release();
  __syncthreads();
  if (threadIdx.x == 0) s_ticket = atomicAdd(&a.tickets[b], 1u);
  __syncthreads();
  if (s_ticket == (uint32_t)(nblk - 1)) {
    ticket_acquire();
    const R* g0 = a.part + (size_t)b * a.nblk_max * 2 * a.p.t_max;
    for (int i = threadIdx.x; i < 2 * d.T; i += blockDim.x) {
      R acc = R(0);
#pragma unroll 8
      for (int k = 0; k < nblk; ++k) acc += g0[(size_t)k * 2 * a.p.t_max + i];
      Vpb[i] = Vb[i] + acc;
    }
    if (threadIdx.x == 0) a.tickets[b] = 0u;
  }
}

// ============================================================== adjoint
// Per-lane reverse sweep with checkpoints every `seg_len` steps (global scratch
// of the workgroup: written once, read once per segment) and the states of one
// segment recomputed into LDS (layout [slot][component][lane]).  Keeping only
// the segment in LDS leaves room for enough workgroups per CU that the large
// batches run in one wave of workgroups.
template <class R>
struct AdjLds {
  R* ck;      // global [n_ck][6][64]
  int* cki;   // global [n_ck][64]
  int* sti;   // global [t_max][64]: window segment of x_{t+1}, from the forward pass
  R* sx;      // LDS [seg_len+1][6][64]
  int* sxi;   // LDS [seg_len+1][64]
};

// Global checkpoint storage of the adjoint: per (problem, workgroup) n_ck slots
// of `comp` values and one index per lane, and with step_idx the window
// segment of every step per lane (the recomputation then skips the window
// search).
template <class R>
__host__ __device__ inline size_t adj_ck_bytes_per_wg(int t_max, int seg_len, int comp, bool step_idx) {
  const int n_ck = (t_max + seg_len - 1) / seg_len;
  return (size_t)n_ck * WAVE * (comp * sizeof(R) + sizeof(int)) + (step_idx ? (size_t)t_max * WAVE * sizeof(int) : 0);
}
// Longest checkpoint segment (the recomputation copies a segment's stored
// window indices through registers).
constexpr int ADJ_SEG_MAX = 12;

template <class R>
__device__ __forceinline__ void adj_store(R* base, int* ibase, int slot, int lane, const State<R>& x, int idx) {
  R* p = base + (size_t)slot * 6 * WAVE + lane;
  p[0 * WAVE] = x.px;
  p[1 * WAVE] = x.py;
  p[2 * WAVE] = x.psi;
  p[3 * WAVE] = x.vx;
  p[4 * WAVE] = x.vy;
  p[5 * WAVE] = x.om;
  ibase[slot * WAVE + lane] = idx;
}
template <class R>
__device__ __forceinline__ void adj_store_state(R* base, int slot, int lane, const State<R>& x) {
  R* p = base + (size_t)slot * 6 * WAVE + lane;
  p[0 * WAVE] = x.px;
  p[1 * WAVE] = x.py;
  p[2 * WAVE] = x.psi;
  p[3 * WAVE] = x.vx;
  p[4 * WAVE] = x.vy;
  p[5 * WAVE] = x.om;
}
template <class R>
__device__ __forceinline__ State<R> adj_load(const R* base, const int* ibase, int slot, int lane, int& idx) {
  const R* p = base + (size_t)slot * 6 * WAVE + lane;
  State<R> x;
  x.px = p[0 * WAVE];
  x.py = p[1 * WAVE];
  x.psi = p[2 * WAVE];
  x.vx = p[3 * WAVE];
  x.vy = p[4 * WAVE];
  x.om = p[5 * WAVE];
  idx = ibase[slot * WAVE + lane];
  return x;
}

template <class R>
__host__ __device__ inline size_t adj_lds_bytes(int /*t_max*/, int seg_len) {
  return (size_t)(seg_len + 1) * WAVE * (6 * sizeof(R) + sizeof(int));
}

// Reverse sweep of one lane's trajectory.  `V` is [2][T] in LDS.  For every t
// (descending) calls sink(t, dL/dv_{t,0}, dL/dv_{t,1}); the sink may modify V[t]
// (the repair does), which is safe because V[t'] for t' >= t is never read again.
// FP32 with obstacles: `slots` (k_pad_obs) gives the obstacle transitions
// for the whole wave (WaveObstacles::grad) instead of the LDS table.
template <class R, int NOBS, class Sink>
__device__ void adjoint_lane(const DevModel<R>& M, const DevCost<R>& C, const DevObjective<R>& ob,
                             const TrackView<R>& tr, const State<R>& x0, R* V, int T, NoiseStream<R>& ns,
                             const AdjLds<R>& L, int seg_len, int lane, Sink& sink, const float4* slots = nullptr) {
  WaveObstacles wob;  // FP32 with obstacles: this lane's slot, read once
  if constexpr (NOBS > 0 && sizeof(R) == sizeof(float)) wob = WaveObstacles(slots, NOBS);
  // forward with checkpoints
  State<R> x = x0;
  int idx = tr.idx0;
  (void)lateral_sq(tr, x.px, x.py, idx);
  for (int t = 0; t < T; ++t) {
    if (t % seg_len == 0) adj_store(L.ck, L.cki, t / seg_len, lane, x, idx);
    R e0, e1;
    ns.at(t, C.sigma[0], C.sigma[1], e0, e1);
    const R u0 = clamp_r(V[t] + e0, M.u_lo[0], M.u_hi[0]);
    const R u1 = clamp_r(V[T + t] + e1, M.u_lo[1], M.u_hi[1]);
    rk4(M, step_ctl(M, u0, u1), x);
    (void)lateral_sq(tr, x.px, x.py, idx);
    L.sti[(size_t)t * WAVE + lane] = idx;
  }
  // terminal cost gradient
  R lam[6] = {R(0), R(0), R(0), R(0), R(0), R(0)};
  stage_grad(C, tr, x, idx, ob.w_S * C.phi_w, lam);
  const int n_seg = (T + seg_len - 1) / seg_len;
  for (int c = n_seg - 1; c >= 0; --c) {
    const int t0 = c * seg_len, t1 = min(T, t0 + seg_len);
    int ci;
    State<R> xs = adj_load(L.ck, L.cki, c, lane, ci);
    adj_store(L.sx, L.sxi, 0, lane, xs, ci);
    // the segment's window indices from the forward pass (all loads first)
    int iv[ADJ_SEG_MAX];
#pragma unroll
    for (int k = 0; k < ADJ_SEG_MAX; ++k) iv[k] = k < t1 - t0 ? L.sti[(size_t)(t0 + k) * WAVE + lane] : 0;
#pragma unroll
    for (int k = 0; k < ADJ_SEG_MAX; ++k)
      if (k < t1 - t0) L.sxi[(k + 1) * WAVE + lane] = iv[k];
    for (int t = t0; t < t1; ++t) {
      R e0, e1;
      if (t == t0 || (t & 1) == 0) ns.gen(t);
      ns.get(t, C.sigma[0], C.sigma[1], e0, e1);
      const R u0 = clamp_r(V[t] + e0, M.u_lo[0], M.u_hi[0]);
      const R u1 = clamp_r(V[T + t] + e1, M.u_lo[1], M.u_hi[1]);
      rk4(M, step_ctl(M, u0, u1), xs);
      adj_store_state(L.sx, t - t0 + 1, lane, xs);
    }
    for (int t = t1 - 1; t >= t0; --t) {
      int ip, in_;
      const State<R> xp = adj_load(L.sx, L.sxi, t - t0, lane, ip);
      const State<R> xn = adj_load(L.sx, L.sxi, t - t0 + 1, lane, in_);
      R gpx = R(0), gpy = R(0);
      if constexpr (NOBS > 0 && sizeof(R) == sizeof(float)) {
        // track barrier as usual, obstacles for the whole wave from the slots
        penalty_grad<R, 0>(C, ob, tr, xp, ip, xn, in_, t, lam, gpx, gpy);
        const R base = ob.w_S * C.C_cbf + ((t < ob.n_lin) ? ob.w_lin : R(0));
        wob.grad(xp.px, xp.py, xn.px, xn.py, C.alpha, base, R(2) * ob.w_sq, lam[0], lam[1], gpx, gpy);
      } else {
        penalty_grad<R, NOBS>(C, ob, tr, xp, ip, xn, in_, t, lam, gpx, gpy);
      }
      R e0, e1;
      // descending: the pair (t-1, t) is regenerated at odd t or at the segment's last step
      if ((t & 1) == 1 || t == t1 - 1) ns.gen(t);
      ns.get(t, C.sigma[0], C.sigma[1], e0, e1);
      const R v0 = V[t], v1 = V[T + t];
      const R r0 = v0 + e0, r1 = v1 + e1;
      const R u0 = clamp_r(r0, M.u_lo[0], M.u_hi[0]);
      const R u1 = clamp_r(r1, M.u_lo[1], M.u_hi[1]);
      const bool pass0 = (r0 >= M.u_lo[0]) && (r0 <= M.u_hi[0]);
      const bool pass1 = (r1 >= M.u_lo[1]) && (r1 <= M.u_hi[1]);
      R gd = R(0), gt = R(0);
      rk4_vjp(M, step_ctl(M, u0, u1), xp, lam, gd, gt);
      lam[0] += gpx;
      lam[1] += gpy;
      stage_grad(C, tr, xp, ip, ob.w_S, lam);
      // control term w_S * lambda_u * v^T Sigma^-1 u: direct in v, and through u
      const R gu0 = gd + ob.w_S * C.ctrl_w[0] * v0;
      const R gu1 = gt + ob.w_S * C.ctrl_w[1] * v1;
      const R gv0 = (pass0 ? gu0 : R(0)) + ob.w_S * C.ctrl_w[0] * u0;
      const R gv1 = (pass1 ? gu1 : R(0)) + ob.w_S * C.ctrl_w[1] * u1;
      sink(t, gv0, gv1);
    }
  }
}

template <class R>
struct BackwardArgs {
  ProblemArgs<R> p;
  DevModel<R> M;
  DevCost<R> C;
  DevObjective<R> ob;
  const R* V;
  const R* grad_S;
  R* grad_V;
  R* part;            // [B][nblk_max][2][t_max]: per-workgroup partials, summed by k_sum_partials
  uint32_t* valid;    // [B]: 1 when the problem's sizes are valid (written by workgroup 0)
  unsigned char* ck;  // [B][nblk_max] blocks of adj_ck_bytes_per_wg(t_max, seg_len, 6): checkpoints
  const float4* obs_pad;  // FP32 with obstacles: [B][NOBS] slots from k_pad_obs (WaveObstacles)
  int nblk_max;
  int seg_len;
};

template <class R>
struct ReduceSink {
  R g;
  R* gp;  // this block's partial [2][T]
  int T;
  int lane;
  // A sample with zero upstream weight (lanes past K, non-finite costs given
  // weight 0) contributes exactly zero, even when its own adjoint diverged.
  __device__ __forceinline__ void operator()(int t, R gv0, R gv1) {
    const R s0 = wave_sum(g != R(0) ? g * gv0 : R(0));
    const R s1 = wave_sum(g != R(0) ? g * gv1 : R(0));
    if (lane == 0) {
      gp[t] = s0;
      gp[T + t] = s1;
    }
  }
};

template <class R, int NOBS>
__global__ __launch_bounds__(WAVE) void k_backward(BackwardArgs<R> a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int b = blockIdx.y;
  ProblemDims d;
  const bool ok = load_dims(a.p, b, d);
  if (blockIdx.x == 0 && threadIdx.x == 0) a.valid[b] = ok ? 1u : 0u;
  if (!ok) return;
  R* gVb = a.grad_V + 2 * (size_t)d.t0;
  if (d.K == 0) {
    if (blockIdx.x == 0)
      for (int i = threadIdx.x; i < 2 * d.T; i += blockDim.x) gVb[i] = R(0);
    return;
  }
  const int nblk = (d.K + WAVE - 1) / WAVE;
  if ((int)blockIdx.x >= nblk) return;
  R* Vs;
  const TrackView<R> tr = stage_problem(a.p, b, d, a.V, smem, &Vs);
  unsigned char* rest = smem + stage_lds_bytes<R>(a.p.poly_max, a.p.t_max, a.p.obs_max);
  const int n_ck = (a.p.t_max + a.seg_len - 1) / a.seg_len;
  AdjLds<R> L;
  L.sx = reinterpret_cast<R*>(rest);
  L.sxi = reinterpret_cast<int*>(L.sx + (size_t)(a.seg_len + 1) * 6 * WAVE);
  unsigned char* ckb =
      a.ck + ((size_t)b * a.nblk_max + blockIdx.x) * adj_ck_bytes_per_wg<R>(a.p.t_max, a.seg_len, 6, true);
  L.ck = reinterpret_cast<R*>(ckb);
  L.cki = reinterpret_cast<int*>(L.ck + (size_t)n_ck * 6 * WAVE);
  L.sti = L.cki + (size_t)n_ck * WAVE;
  __syncthreads();
  const int lane = threadIdx.x;
  const int m = blockIdx.x * WAVE + lane;
  NoiseStream<R> ns;
  ns.seed = a.p.seed;
  ns.m = (uint32_t)m;
  ns.pid = (uint32_t)(a.p.pid_base + b);
  ns.it = a.p.iter[b];
  ns.nominal = a.p.nominal != 0;
  ReduceSink<R> sink;
  sink.g = (m < d.K) ? a.grad_S[d.k0 + m] : R(0);
  sink.gp = a.part + ((size_t)b * a.nblk_max + blockIdx.x) * 2 * a.p.t_max;
  sink.T = d.T;
  sink.lane = lane;
  const State<R> x0 = load_state(a.p.x0 + 6 * (size_t)b);
  adjoint_lane<R, NOBS>(a.M, a.C, a.ob, tr, x0, Vs, d.T, ns, L, a.seg_len, lane, sink,
                        a.obs_pad ? a.obs_pad + (size_t)b * NOBS : nullptr);
}

// Sum of the adjoint's per-workgroup partials: out[2 t0_b + i] = sum over the
// problem's nblk_b = ceil(K_b / 64) rows of part[b][k][i], i < 2 T_b, in a fixed
// order (each slice of SUM_SLICE consecutive rows in row order, then the slices
// in order), so the result does not depend on scheduling.  Grid (n_chunks, B,
// n_slices) of 64 threads, chunk = 64 consecutive outputs: every workgroup sums
// one slice of one chunk; with more than one slice the last workgroup of a
// (problem, chunk) to finish (ticket, zero on entry and reset on exit) adds the
// slice sums.  Problems with K_b = 0 (the adjoint wrote zeros) or invalid sizes
// (flagged by the adjoint) are skipped.
constexpr int SUM_SLICE = 32;

template <class R>
struct SumArgs {
  const int64_t* k_off;
  const int32_t* t_off;
  int t_max, nblk_max, n_slices_max, n_chunks;
  const R* part;      // [B][nblk_max][2][t_max]
  const uint32_t* valid;  // [B]: the adjoint processed the problem
  R* slice;           // [B][n_slices_max][2][t_max]
  uint32_t* tickets;  // [B][n_chunks]
  R* out;             // [sum 2T]
};

template <class R>
__global__ __launch_bounds__(WAVE) void k_sum_partials(SumArgs<R> a) {
  __shared__ uint32_t s_ticket;
  const int b = blockIdx.y, chunk = blockIdx.x, sl = blockIdx.z;
  const int64_t K = a.k_off[b + 1] - a.k_off[b];
  const int t0 = a.t_off[b], T = a.t_off[b + 1] - t0;
  if (!a.valid[b] || K <= 0 || T < 1 || T > a.t_max || (K + WAVE - 1) / WAVE > a.nblk_max) return;
  const int nblk = (int)((K + WAVE - 1) / WAVE);
  const int ns = (nblk + SUM_SLICE - 1) / SUM_SLICE;
  if (sl >= ns || chunk * WAVE >= 2 * T) return;
  const int i = chunk * WAVE + threadIdx.x;
  const bool valid = i < 2 * T;
  const int k0 = sl * SUM_SLICE, k1 = min(nblk, k0 + SUM_SLICE);
  const size_t row = 2 * (size_t)a.t_max;
  R acc = R(0);
  if (valid) {
    const R* p = a.part + ((size_t)b * a.nblk_max + k0) * row + i;
#pragma unroll 8
    for (int k = 0; k < k1 - k0; ++k) acc += p[(size_t)k * row];
  }
  if (ns == 1) {
    if (valid) a.out[2 * (size_t)t0 + i] = acc;
    return;
  }
  if (valid) a.slice[((size_t)b * a.n_slices_max + sl) * row + i] = acc;
  ticket_release();
  __syncthreads();
  uint32_t* tk = a.tickets + (size_t)b * a.n_chunks + chunk;
  if (threadIdx.x == 0) s_ticket = atomicAdd(tk, 1u);
  __syncthreads();
  if (s_ticket == (uint32_t)(ns - 1)) {
    ticket_acquire();
    if (valid) {
      const R* q = a.slice + (size_t)b * a.n_slices_max * row + i;
      R tot = R(0);
      for (int k = 0; k < ns; ++k) tot += q[(size_t)k * row];
      a.out[2 * (size_t)t0 + i] = tot;
    }
    if (threadIdx.x == 0) *tk = 0u;
  }
}

// ============================================================== repair
// ============================================================== execute / warm start
template <class R>
struct ExecuteArgs {
  const int32_t* t_off;
  int32_t B, t_max;
  DevModel<R> M;
  const R* V_exec;
  const R* V_plus;
  const R* dist;
  int32_t n_dist;
  R* x;
  R* V;
  uint32_t* iter;
  uint32_t* err;
};

// Plant step and warm start of problem b by one workgroup (Alg. 2, last two
// lines): x <- RK4(x, clip(v_0)) + disturbance on (v_y, omega); V <- V+ shifted
// by one step, last step repeated.  Vexec points at the problem's executed
// sequence (global or LDS); buf is 2T values of LDS.
template <class R>
__device__ void execute_problem(const ExecuteArgs<R>& a, int b, int t0, int T, const R* Vexec, R* buf) {
  const R* Vp = a.V_plus + 2 * (size_t)t0;
  for (int i = threadIdx.x; i < 2 * T; i += blockDim.x) buf[i] = Vp[i];
  __syncthreads();
  if (threadIdx.x == 0) {
    const R u0 = clamp_r(Vexec[0], a.M.u_lo[0], a.M.u_hi[0]);
    const R u1 = clamp_r(Vexec[T], a.M.u_lo[1], a.M.u_hi[1]);
    State<R> x = load_state(a.x + 6 * (size_t)b);
    rk4(a.M, step_ctl(a.M, u0, u1), x);
    const uint32_t it = a.iter[b];
    if (a.dist && (int64_t)it < (int64_t)a.n_dist) {
      x.vy += a.dist[(2 * ((size_t)it * a.B + b))];
      x.om += a.dist[(2 * ((size_t)it * a.B + b)) + 1];
    }
    R* xo = a.x + 6 * (size_t)b;
    xo[0] = x.px;
    xo[1] = x.py;
    xo[2] = x.psi;
    xo[3] = x.vx;
    xo[4] = x.vy;
    xo[5] = x.om;
    a.iter[b] = it + 1u;
  }
  R* Vo = a.V + 2 * (size_t)t0;
  for (int i = threadIdx.x; i < 2 * T; i += blockDim.x) {
    const int dd = i / T, t = i % T;
    Vo[i] = buf[dd * T + min(t + 1, T - 1)];
  }
}

template <class R>
struct RepairArgs {
  ProblemArgs<R> p;
  DevModel<R> M;
  DevCost<R> C;
  DevObjective<R> ob;
  const R* V_plus;
  R* V_safe;
  int n_steps;
  R step;
  int seg_len;
  int method;           // 0: Algorithm 1; 1: projected L-BFGS
  int memory;           // L-BFGS pairs (0 with method 0)
  int par_rev;          // nonzero: reverse sweep with per-step Jacobians computed in parallel
  int exec;             // nonzero: also run the plant step and warm start (ex)
  ExecuteArgs<R> ex;
};

constexpr int REP_C = 4;  // shield: control rows read ahead, segment indices stored, per chunk of steps
// Parallel reverse sweep: per step the transposed Jacobian of the RK4 step with
// respect to (x, u) (6 x 8), the local barrier/cost gradients (8) and the
// control gradient (2).
constexpr int REP_PAR_PER_STEP = 48 + 8 + 2;
// Per-step constants of the shield's forward pass, one 16-byte aligned row per
// step: the 13 values of shield_vel_row, 3 unused.
constexpr int REP_CTL = 16;

// The shield's nominal trajectory runs on one lane, where every instruction of
// the RK4 chain costs an issue slot, so its velocity part takes its per-step
// constants precomputed (by all threads, in parallel, before the pass) in the
// form that needs the fewest instructions per stage.  With the lateral tyre
// forces F_f = C_f t1, F_r = C_r t2, t1 = delta - (v_y + l_f om) / v,
// t2 = (l_r om - v_y) / v (v = max(v_x, v_min)), each RK4 stage value
// y_k = y_0 + f_k F(y_{k-1}) (f = h/2, h/2, h) is three FMA chains whose
// coefficients carry f_k and the tyre stiffnesses, with y_0 folded into the
// innermost addend; the last stage gives K = (h/6) F(y_3), and the step is
// y_0 + (h/6)(k_1 + 2 k_2 + 2 k_3 + k_4) = (y_1 + 2 y_2 + y_3 - y_0)/3 + K.
// (The classic RK4 of the model, evaluated in another order.)
template <class R>
struct ShieldVel {
  R v_min, lf, lr;
  R f[3];    // h/2, h, h/6
  R cv[3];   // -f c_v
  R crm[3];  // f C_r / m
  R crl[3];  // -f C_r l_r / I_z
};

template <class R>
__device__ __forceinline__ ShieldVel<R> shield_vel(const DevModel<R>& M) {
  ShieldVel<R> k;
  k.v_min = M.v_min;
  k.lf = M.lf;
  k.lr = M.lr;
  k.f[0] = R(0.5) * M.dt;
  k.f[1] = M.dt;
  k.f[2] = M.dt * R(1.0 / 6.0);
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    k.cv[i] = -(k.f[i] * M.c_v);
    k.crm[i] = k.f[i] * (M.Cr * M.inv_m);
    k.crl[i] = -(k.f[i] * (M.Cr * M.lr_Iz));
  }
  return k;
}

// Row of a step with the held control (delta, tau): delta; f a_max tau for
// f = h/2, h, h/6; then per f: -f C_f sin(delta)/m, f C_f cos(delta)/m,
// f C_f l_f cos(delta)/I_z.
template <class R>
__device__ __forceinline__ void shield_vel_row(const DevModel<R>& M, R delta, R tau, R* cr) {
  const StepCtl<R> c = step_ctl(M, delta, tau);
  const R f[3] = {R(0.5) * M.dt, M.dt, M.dt * R(1.0 / 6.0)};
  cr[0] = c.delta;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const R g = f[i] * M.Cf;
    cr[1 + i] = f[i] * c.a_tau;
    cr[4 + 3 * i] = -(g * c.sd_m);
    cr[5 + 3 * i] = g * c.cd_m;
    cr[6 + 3 * i] = g * c.lfcd_Iz;
  }
}

// max(x, v_min) on the velocity chain, v_min > 0.  FP32: one integer max of
// the bit patterns (fmax first quiets a possible signalling NaN in x with a
// second instruction on the chain): non-negative floats order like their bits
// as signed integers, and every negative x (sign bit set) is below v_min's
// positive pattern, so the value is fmax's for every x that is not a NaN.
template <class R>
__device__ __forceinline__ R shield_vmax(R x, R v_min) { return fmax(x, v_min); }
template <>
__device__ __forceinline__ float shield_vmax<float>(float x, float v_min) {
  return __int_as_float(max(__float_as_int(x), __float_as_int(v_min)));
}

// f_i F(x, y, o) added to (ax, ay, ao), coefficients of factor i.
template <class R, int I>
__device__ __forceinline__ void shield_vel_inc(const ShieldVel<R>& k, const R* cr, R x, R y, R o, R ax, R ay, R ao,
                                               R& ox, R& oy, R& oo) {
  const R inv = rcp_r(shield_vmax(x, k.v_min));
  const R t1 = fma_r(-fma_r(k.lf, o, y), inv, cr[0]);
  const R t2 = fma_r(k.lr, o, -y) * inv;
  const R oh = o * k.f[I];
  ox = fma_r(y, oh, fma_r(t1, cr[4 + 3 * I], fma_r(k.cv[I], x, ax)));
  oy = fma_r(-x, oh, fma_r(t1, cr[5 + 3 * I], fma_r(t2, k.crm[I], ay)));
  oo = fma_r(t1, cr[6 + 3 * I], fma_r(t2, k.crl[I], ao));
}

// One RK4 step of (v_x, v_y, om) from a row of shield_vel_row; the stage
// velocities (stage 1 = the step's start) for the pose part.
template <class R>
__device__ __forceinline__ void shield_vel_step(const ShieldVel<R>& k, const R* cr, R& vx, R& vy, R& om,
                                                VelStages<R>& g) {
  const R x0 = vx, y0 = vy, o0 = om;
  g.vx[0] = x0;
  g.vy[0] = y0;
  g.om[0] = o0;
  const R p2 = x0 + cr[1], p1 = x0 + cr[2];
  shield_vel_inc<R, 0>(k, cr, x0, y0, o0, p2, y0, o0, g.vx[1], g.vy[1], g.om[1]);
  shield_vel_inc<R, 0>(k, cr, g.vx[1], g.vy[1], g.om[1], p2, y0, o0, g.vx[2], g.vy[2], g.om[2]);
  shield_vel_inc<R, 1>(k, cr, g.vx[2], g.vy[2], g.om[2], p1, y0, o0, g.vx[3], g.vy[3], g.om[3]);
  R kx, ky, ko;
  shield_vel_inc<R, 2>(k, cr, g.vx[3], g.vy[3], g.om[3], cr[3], R(0), R(0), kx, ky, ko);
  const R third = R(1.0 / 3.0), two_thirds = R(2.0 / 3.0);
  vx = fma_r(two_thirds, g.vx[2], fma_r(third, g.vx[1] + g.vx[3], fma_r(-third, x0, kx)));
  vy = fma_r(two_thirds, g.vy[2], fma_r(third, g.vy[1] + g.vy[3], fma_r(-third, y0, ky)));
  om = fma_r(two_thirds, g.om[2], fma_r(third, g.om[1] + g.om[3], fma_r(-third, o0, ko)));
}

// LDS of the shield beyond the staged problem: states x_0..x_T, their e_y^2,
// segment indices, the per-step constants (REP_CTL per step) and two chunks of RK4
// stage velocities (12 per step) passed from the velocity wave to the pose wave;
// with L-BFGS (memory > 0) also the gradient, the previous iterate and
// gradient, the two-loop vector, memory + 1 pair slots (s, y) of 2 t_max
// values, four scalars per slot and a reduction buffer.
template <class R>
__host__ __device__ inline size_t repair_lds_bytes(int t_max, int memory, bool par_rev, bool stepwise) {
  // stage velocities: every step for the step-by-step hand-over, else a ring of two chunks
  const size_t vst_rows = stepwise ? (size_t)t_max : (size_t)2 * REP_C;
  size_t n = (size_t)(t_max + 1) * (7 * sizeof(R) + sizeof(int)) + (size_t)REP_CTL * (t_max + 2) * sizeof(R) +
             (size_t)12 * vst_rows * sizeof(R) + 16;
  if (memory > 0) n += ((size_t)(4 + 2 * (memory + 1)) * 2 * t_max + 4 * (memory + 1) + 16) * sizeof(R);
  if (par_rev) n += (size_t)REP_PAR_PER_STEP * t_max * sizeof(R);
  return n;
}

// Algorithm 1 for one problem on one workgroup of three (or more) waves.  The
// nominal trajectory is short (T+1 states), so every state is kept in LDS and
// the reverse sweep reads it back instead of recomputing it.  The forward pass
// is pipelined step by step through LDS counters (wave 0: velocity part of the
// RK4 chain; wave 2: pose part, one RK4 stage per lane; wave 1: the
// lateral-offset window, one segment per lane with the rule's first minimum
// picked by ballot, and the obstacle barriers, one obstacle per lane),
// recording the segment indices and the last transition whose objective term
// has a non-zero derivative (without obstacles: found after the pass from the
// stored e_y^2).  The reverse
// sweep starts at that transition (everything later has a zero gradient, so
// those controls only get the box projection), and the iteration stops as
// soon as no such transition is left: the gradient is then exactly zero and
// every remaining step would be the identity after the projection already
// applied.
constexpr int REP_BLK = 3 * WAVE;
// Largest workgroup of the shield kernel: the three pipeline waves, plus three
// more for the FP32 kernel without obstacles (its registers leave room for two
// waves per SIMD), so that the parallel reverse sweep's per-step Jacobian rows
// (six per step) take one round instead of two for horizons up to 64.  The
// extra waves only join the workgroup's barriers during the forward pass; the
// launch chooses between this and REP_BLK.
template <class R, int NOBS>
constexpr int rep_blk() {
  return (sizeof(R) == 4 && NOBS == 0) ? 2 * REP_BLK : REP_BLK;
}

// Row-rotate of a value across the 16 lanes of each row (DPP row_ror:N).
template <int N>
__device__ __forceinline__ float row_ror(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x120 + N, 0xF, 0xF, false));
}
template <int N>
__device__ __forceinline__ double row_ror(double v) {
  const long long bits = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)bits, 0x120 + N, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(bits >> 32), 0x120 + N, 0xF, 0xF, false);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// Minimum over the 16 lanes of each row (four DPP rotations).  FP32 values
// here are squared distances (non-negative, or +inf): their bit patterns order
// like unsigned integers, so the reduction runs on integers (no NaN
// canonicalisation before each min) and the rotation can fold into the min.
template <class R>
__device__ __forceinline__ R row_min(R m) {
  m = fmin(m, row_ror<8>(m));
  m = fmin(m, row_ror<4>(m));
  m = fmin(m, row_ror<2>(m));
  return fmin(m, row_ror<1>(m));
}
template <>
__device__ __forceinline__ float row_min<float>(float v) {
  unsigned m = __float_as_uint(v);
  m = min(m, (unsigned)__builtin_amdgcn_mov_dpp((int)m, 0x128, 0xF, 0xF, false));
  m = min(m, (unsigned)__builtin_amdgcn_mov_dpp((int)m, 0x124, 0xF, 0xF, false));
  m = min(m, (unsigned)__builtin_amdgcn_mov_dpp((int)m, 0x122, 0xF, 0xF, false));
  m = min(m, (unsigned)__builtin_amdgcn_mov_dpp((int)m, 0x121, 0xF, 0xF, false));
  return __uint_as_float(m);
}

// The window rule on the lanes of a row (half width <= 7; the whole wave must
// be active and c, px, py uniform): lane r of each row holds the r-th offset of
// the rule's order (0, -1, +1, -2, ...), the row minimum comes from four DPP
// rotations, and the first offset in the rule's order attaining it is the
// lowest set bit of the ballot; that lane's wrapped segment index is the new c
// (one v_readlane).  Returns e_y^2; c (uniform) in/out.
template <class R>
__device__ R row_window(const TrackView<R>& tr, int& c, R px, R py) {
  const int r = threadIdx.x & 15;
  const int off = r == 0 ? 0 : ((r & 1) ? -((r + 1) >> 1) : (r >> 1));
  // the slot's segment wrapped onto 0 .. n-1 (the padded copy is read at c + off)
  int iw = c + off;
  iw += (iw < 0) ? tr.n : 0;
  iw -= (iw >= tr.n) ? tr.n : 0;
  R dd = R(INFINITY);
  if (r < 2 * tr.window + 1) dd = seg_dist2(tr, c + off, px, py);
  const R m = row_min(dd);
  const unsigned long long bal = __ballot(dd == m) & 0xFFFFull;
  // the first slot attaining the minimum; slot 0 (offset 0) if none does (NaN)
  const int rr = bal ? __ffsll((long long)bal) - 1 : 0;
  c = __builtin_amdgcn_readlane(iw, rr);
  return m;
}

template <class R>
__device__ __forceinline__ R circle_e2(const TrackView<R>& tr, R px, R py) {
  const R dx = px - tr.cx, dy = py - tr.cy;
  const R e = sqrt_r(dx * dx + dy * dy) - tr.rad;
  return e * e;
}

// Reverse sweep of the shield objective on the stored nominal trajectory,
// t = t_end .. 0: applies the projected gradient step to V in place, or, with
// gout, writes the gradient dL/dV there and leaves V unchanged.
template <class R, int NOBS>
__device__ void repair_reverse(const DevModel<R>& M, const DevCost<R>& C, const DevObjective<R>& ob,
                               const TrackView<R>& tr, R* V, int T, int t_end, R step, const R* xs, const int* is,
                               R* gout) {
  const bool cost_terms = ob.w_S != R(0);
  R lam[6] = {R(0), R(0), R(0), R(0), R(0), R(0)};
  if (cost_terms) {
    State<R> xT;
    const R* pT = xs + 6 * T;
    xT.px = pT[0]; xT.py = pT[1]; xT.psi = pT[2]; xT.vx = pT[3]; xT.vy = pT[4]; xT.om = pT[5];
    stage_grad(C, tr, xT, is[T], ob.w_S * C.phi_w, lam);
  }
  for (int t = t_end; t >= 0; --t) {
    const R* pp = xs + 6 * t;
    const R* pn = pp + 6;
    State<R> xp, xn;
    xp.px = pp[0]; xp.py = pp[1]; xp.psi = pp[2]; xp.vx = pp[3]; xp.vy = pp[4]; xp.om = pp[5];
    xn.px = pn[0]; xn.py = pn[1]; xn.psi = pn[2]; xn.vx = pn[3]; xn.vy = pn[4]; xn.om = pn[5];
    const int ip = is[t], in_ = is[t + 1];
    R gpx = R(0), gpy = R(0);
    penalty_grad<R, NOBS>(C, ob, tr, xp, ip, xn, in_, t, lam, gpx, gpy);
    const R v0 = V[t], v1 = V[T + t];
    const R u0 = clamp_r(v0, M.u_lo[0], M.u_hi[0]);
    const R u1 = clamp_r(v1, M.u_lo[1], M.u_hi[1]);
    const bool pass0 = (v0 >= M.u_lo[0]) && (v0 <= M.u_hi[0]);
    const bool pass1 = (v1 >= M.u_lo[1]) && (v1 <= M.u_hi[1]);
    R gd = R(0), gt = R(0);
    rk4_vjp(M, step_ctl(M, u0, u1), xp, lam, gd, gt);
    lam[0] += gpx;
    lam[1] += gpy;
    if (cost_terms) stage_grad(C, tr, xp, ip, ob.w_S, lam);
    const R gu0 = gd + ob.w_S * C.ctrl_w[0] * v0;
    const R gu1 = gt + ob.w_S * C.ctrl_w[1] * v1;
    const R gv0 = (pass0 ? gu0 : R(0)) + ob.w_S * C.ctrl_w[0] * u0;
    const R gv1 = (pass1 ? gu1 : R(0)) + ob.w_S * C.ctrl_w[1] * u1;
    if (gout) {  // gradient only (quasi-Newton shield)
      gout[t] = gv0;
      gout[T + t] = gv1;
    } else {
      V[t] = clamp_r(v0 - step * gv0, M.u_lo[0], M.u_hi[0]);
      V[T + t] = clamp_r(v1 - step * gv1, M.u_lo[1], M.u_hi[1]);
    }
  }
}

// Value of lane i of the wave (uniform result).
__device__ __forceinline__ float lane_bcast(float v, int i) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), i));
}
__device__ __forceinline__ double lane_bcast(double v, int i) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, i), hi = __builtin_amdgcn_readlane((int)(b >> 32), i);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// Value of lane Q of each quad (DPP quad_perm [Q, Q, Q, Q]).
template <int Q>
__device__ __forceinline__ float quad_get(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), Q * 0x55, 0xF, 0xF, false));
}
template <int Q>
__device__ __forceinline__ double quad_get(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)b, Q * 0x55, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), Q * 0x55, 0xF, 0xF, false);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// The same reverse sweep by the whole workgroup (every thread must call it).
// The adjoint recursion is linear once the nominal trajectory is fixed:
//   lam_t = J_t^T (lam_{t+1} + dn_t) + dc_t,   g_t = B_t^T (lam_{t+1} + dn_t),
// with J_t, B_t the RK4 step's Jacobians with respect to x_t and u_t, dn_t / dc_t
// the barrier (and cost) gradients of transition t at x_{t+1} / x_t.  Phase A
// computes [J_t^T; B_t^T] (six vector-Jacobian products with unit cotangents,
// one per thread) and dn_t, dc_t for every step in parallel; phase B runs the
// recursion as 6 x 8 matrix-vector products on eight lanes of the first wave
// (lane j forms component j from the lam_i broadcast by readlane); phase C applies the
// projected step (or writes the gradient) for every step in parallel.
// W: [t_max][REP_PAR_PER_STEP] LDS.
template <class R, int NOBS>
__device__ void repair_reverse_par(const DevModel<R>& M, const DevCost<R>& C, const DevObjective<R>& ob,
                                   const TrackView<R>& tr, R* V, int T, int t_end, R step, const R* xs,
                                   const int* is, R* gout, R* W) {
  constexpr int P = REP_PAR_PER_STEP;
  const bool cost_terms = ob.w_S != R(0);
  const int n_pen = t_end + 1, nit = 6 * n_pen;
  // barrier and cost gradients of every step (dn_t, dc_t)
  auto pen_task = [&](int t) {
    const R* pp = xs + 6 * t;
    State<R> xp, xn;
    xp.px = pp[0]; xp.py = pp[1]; xp.psi = pp[2]; xp.vx = pp[3]; xp.vy = pp[4]; xp.om = pp[5];
    const R* pn = pp + 6;
    xn.px = pn[0]; xn.py = pn[1]; xn.psi = pn[2]; xn.vx = pn[3]; xn.vy = pn[4]; xn.om = pn[5];
    R dn[6] = {R(0), R(0), R(0), R(0), R(0), R(0)};
    R gpx = R(0), gpy = R(0);
    penalty_grad<R, NOBS>(C, ob, tr, xp, is[t], xn, is[t + 1], t, dn, gpx, gpy);
    R dc[6] = {gpx, gpy, R(0), R(0), R(0), R(0)};
    if (cost_terms) stage_grad(C, tr, xp, is[t], ob.w_S, dc);
    R* dd = W + (size_t)P * t + 48;
    dd[0] = dn[0];
    dd[1] = dn[1];
#pragma unroll
    for (int j = 0; j < 6; ++j) dd[2 + j] = dc[j];
  };
  // The gradient tasks take waves of their own when the Jacobian rows then need
  // no more rounds (else each wave would run both kinds of task in turn).
  const int nt = blockDim.x, pw = WAVE * ((n_pen + WAVE - 1) / WAVE), nv = nt - pw;
  const bool own = nv > 0 && (nit + nv - 1) / nv <= (nit + nt - 1) / nt;
  const int nvt = own ? nv : nt;
  for (int k = threadIdx.x; k < nit && (int)threadIdx.x < nvt; k += nvt) {
    const int t = k / 6, i = k % 6;
    const R* pp = xs + 6 * t;
    State<R> xp;
    xp.px = pp[0]; xp.py = pp[1]; xp.psi = pp[2]; xp.vx = pp[3]; xp.vy = pp[4]; xp.om = pp[5];
    const R u0 = clamp_r(V[t], M.u_lo[0], M.u_hi[0]);
    const R u1 = clamp_r(V[T + t], M.u_lo[1], M.u_hi[1]);
    R lam[6] = {R(0), R(0), R(0), R(0), R(0), R(0)};
    lam[i] = R(1);
    R gd = R(0), gt = R(0);
    rk4_vjp(M, step_ctl(M, u0, u1), xp, lam, gd, gt);
    R* q = W + (size_t)P * t + 8 * i;
#pragma unroll
    for (int j = 0; j < 6; ++j) q[j] = lam[j];
    q[6] = gd;
    q[7] = gt;
    if (!own && i == 0) pen_task(t);
  }
  if (own && (int)threadIdx.x >= nv)
    for (int t = threadIdx.x - nv; t < n_pen; t += pw) pen_task(t);
  __syncthreads();
  if (threadIdx.x < WAVE) {
    // lane j < 8 holds component j: lam_j for j < 6, the control gradient for j = 6, 7;
    // each step broadcasts lam_0..5 from their lanes and forms column j of Q^T lam
    const int j = threadIdx.x & 7;
    R lam = R(0);
    if (cost_terms) {
      State<R> xT;
      const R* pT = xs + 6 * T;
      xT.px = pT[0]; xT.py = pT[1]; xT.psi = pT[2]; xT.vx = pT[3]; xT.vy = pT[4]; xT.om = pT[5];
      R l6[6] = {R(0), R(0), R(0), R(0), R(0), R(0)};
      stage_grad(C, tr, xT, is[T], ob.w_S * C.phi_w, l6);
#pragma unroll
      for (int i = 0; i < 6; ++i) lam = j == i ? l6[i] : lam;
    }
    for (int t = t_end; t >= 0; --t) {
      const R* q = W + (size_t)P * t;
      if (j < 2) lam += q[48 + j];
      R l[6];
#pragma unroll
      for (int i = 0; i < 6; ++i) l[i] = lane_bcast(lam, i);
      const R nl = ((l[0] * q[j] + l[1] * q[8 + j]) + (l[2] * q[16 + j] + l[3] * q[24 + j])) +
                   (l[4] * q[32 + j] + l[5] * q[40 + j]);
      if (j < 6) {
        lam = nl + q[50 + j];
      } else if (threadIdx.x < 8) {
        W[(size_t)P * t + 56 + (j - 6)] = nl;
      }
    }
  }
  __syncthreads();
  for (int t = threadIdx.x; t <= t_end; t += blockDim.x) {
    const R* g = W + (size_t)P * t + 56;
    const R v0 = V[t], v1 = V[T + t];
    const R u0 = clamp_r(v0, M.u_lo[0], M.u_hi[0]);
    const R u1 = clamp_r(v1, M.u_lo[1], M.u_hi[1]);
    const bool pass0 = (v0 >= M.u_lo[0]) && (v0 <= M.u_hi[0]);
    const bool pass1 = (v1 >= M.u_lo[1]) && (v1 <= M.u_hi[1]);
    const R gu0 = g[0] + ob.w_S * C.ctrl_w[0] * v0;
    const R gu1 = g[1] + ob.w_S * C.ctrl_w[1] * v1;
    const R gv0 = (pass0 ? gu0 : R(0)) + ob.w_S * C.ctrl_w[0] * u0;
    const R gv1 = (pass1 ? gu1 : R(0)) + ob.w_S * C.ctrl_w[1] * u1;
    if (gout) {
      gout[t] = gv0;
      gout[T + t] = gv1;
    } else {
      V[t] = clamp_r(v0 - step * gv0, M.u_lo[0], M.u_hi[0]);
      V[T + t] = clamp_r(v1 - step * gv1, M.u_lo[1], M.u_hi[1]);
    }
  }
}

// Block-wide dot product of two LDS vectors of n values (fixed order).
template <class R>
__device__ R block_dot(const R* x, const R* y, int n, R* red) {
  R v = R(0);
  for (int i = threadIdx.x; i < n; i += blockDim.x) v += x[i] * y[i];
  return block_sum(v, red);
}

// One projected L-BFGS step of the shield by the whole workgroup, given the
// gradient g at V (LDS): keeps the pair (V - V_prev, g - g_prev) when
// `have_prev` and its curvature s.y exceeds 0.01 |s| |y|, computes q = H g by
// the two-loop recursion (H_0 = (s.y / y.y) I of the newest pair, or step * I
// with no pair), and sets V_prev = V, g_prev = g, V = clip(V - q).
template <class R>
__device__ void lbfgs_step(const DevModel<R>& M, R* V, int T, const R* g, R* gprev, R* vprev, R* q, R* Sp, R* Yp,
                           R* rho, R* alpha, R* psy, R* pyy, R* red, int mem, int stride, R step, bool have_prev,
                           int& n_pairs, int& head) {
  const int n = 2 * T;
  const int cap = mem + 1;  // ring slots: at most `mem` kept pairs plus the candidate
  if (have_prev && mem > 0) {
    // candidate pair into the free slot after the newest kept pair
    const int slot = (head + n_pairs) % cap;
    R* s = Sp + (size_t)slot * stride;
    R* y = Yp + (size_t)slot * stride;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
      s[i] = V[i] - vprev[i];
      y[i] = g[i] - gprev[i];
    }
    __syncthreads();
    const R sy = block_dot(s, y, n, red), ss = block_dot(s, s, n, red), yy = block_dot(y, y, n, red);
    if (sy > R(0.01) * sqrt(ss) * sqrt(yy)) {
      if (threadIdx.x == 0) {
        rho[slot] = R(1) / sy;
        psy[slot] = sy;
        pyy[slot] = yy;
      }
      if (n_pairs == mem) head = (head + 1) % cap;  // drop the oldest
      else ++n_pairs;
    }
    __syncthreads();
  }
  R gamma = step;
  if (n_pairs > 0) {
    const int nw = (head + n_pairs - 1) % cap;
    gamma = psy[nw] / pyy[nw];
  }
  for (int i = threadIdx.x; i < n; i += blockDim.x) q[i] = g[i];
  __syncthreads();
  for (int k = n_pairs - 1; k >= 0; --k) {
    const int sl = (head + k) % cap;
    const R al = rho[sl] * block_dot(Sp + (size_t)sl * stride, q, n, red);
    if (threadIdx.x == 0) alpha[sl] = al;
    const R* y = Yp + (size_t)sl * stride;
    for (int i = threadIdx.x; i < n; i += blockDim.x) q[i] -= al * y[i];
    __syncthreads();
  }
  for (int i = threadIdx.x; i < n; i += blockDim.x) q[i] *= gamma;
  __syncthreads();
  for (int k = 0; k < n_pairs; ++k) {
    const int sl = (head + k) % cap;
    const R be = rho[sl] * block_dot(Yp + (size_t)sl * stride, q, n, red);
    const R* s = Sp + (size_t)sl * stride;
    const R coef = alpha[sl] - be;
    for (int i = threadIdx.x; i < n; i += blockDim.x) q[i] += s[i] * coef;
    __syncthreads();
  }
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    vprev[i] = V[i];
    gprev[i] = g[i];
    // bounds selected, not indexed (a dynamic index into a local copy of the
    // model would put it in scratch memory)
    const bool thr = i >= T;
    V[i] = clamp_r(V[i] - q[i], thr ? M.u_lo[1] : M.u_lo[0], thr ? M.u_hi[1] : M.u_hi[0]);
  }
  __syncthreads();
}

// The DCBF condition of one transition fails: alpha h(x_t) > h(x_{t+1}), i.e.
// alpha h(x_t) - h(x_{t+1}) > 0 (a difference of two floats is zero only when
// they are equal).  One definition for every place that decides it.
template <class R>
__device__ __forceinline__ bool dcbf_active(R alpha, R h_t, R h_t1) {
  return alpha * h_t > h_t1;
}

// Step counters between the waves of one workgroup (LDS only).  The LDS
// performs the operations of one wave in the order the wave issues them, so a
// counter stored after a step's LDS rows lands after those rows, and a wave
// that has read the new counter value issues its row reads after that: the
// producer does not have to wait for its row stores to complete before it
// stores the counter (a release store would, one LDS round trip per step on
// the producer's dependency chain).  The empty asm statements keep the
// compiler from moving LDS accesses across the counter accesses.
__device__ __forceinline__ void wave_publish(int* c, int v) {
  asm volatile("" ::: "memory");
  __hip_atomic_store(c, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Waits until the step counter *c (wave_publish by another wave of the
// workgroup) exceeds t; `seen` keeps the last value read, so a wave that trails
// its producer polls only when it has caught up.  Polls back to back: a poll
// is one LDS read, a compare and a branch, and the wave sleeps in the read's
// wait.  The wait is bounded: after 2^22 polls
// the wave flags DERR_WAIT and stops waiting (its results are then wrong, but
// the workgroup finishes).
__device__ __forceinline__ void wave_wait(const int* c, int t, int& seen, uint32_t* err) {
  for (int n = 0; seen <= t; ++n) {
    seen = __hip_atomic_load(c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    if (seen > t) break;
    if (n >= (1 << 22)) {
      if (threadIdx.x % WAVE == 0) atomicOr(err, DERR_WAIT);
      seen = 0x7fffffff;
      break;
    }
  }
  asm volatile("" ::: "memory");
}

// Algorithm 1 for problem b by one workgroup of at least three waves (threads
// beyond the first three waves only join the barriers).  Vs (LDS) holds V+ on
// entry and V_safe on exit; tr is the staged problem; `lds` is
// repair_lds_bytes of LDS.  Per iteration: every thread computes the control
// constants of its share of the steps; then a pipeline over the steps: wave 0
// runs the velocity part of the RK4 chain on one lane, wave 2 the pose part
// (with VG on four lanes, one RK4 stage each; else on one lane), and wave 1
// evaluates the window (one segment per lane), the obstacles (one per lane) and
// the barrier activity of each new position (with VG and no obstacles the
// activity is evaluated after the pass by all threads).  With VG the waves hand
// over step by step through LDS step counters; without (the workgroup shares
// its compute unit with rollout tiles), chunk by chunk of REP_C steps between
// workgroup barriers.  The reverse sweep starts at the last active transition,
// and the iteration loop stops when no transition is active (zero gradient).
// VG: model and cost constants in VGPRs (kernels whose occupancy does not
// depend on the VGPR count: the shield kernel, the latency-mode fused kernel).
template <class R, int NOBS, bool VG = true>
__device__ void repair_problem(const RepairArgs<R>& a, int b, const ProblemDims& d, const TrackView<R>& tr, R* Vs,
                               unsigned char* lds, int* s_last) {
  // 16-byte aligned rows first (lds is 16-byte aligned): ctl [t_max + 2][REP_CTL]
  // (two padding rows for the velocity wave's reads ahead),
  // vst stage velocities ([t_max][12] with VG, else a ring [2][REP_C][12]), 16
  // bytes of step counters; then states xs [t_max+1][6], e_y^2 of each state
  // e2s [t_max+1], segment indices is [t_max+1]
  R* ctl = static_cast<R*>(__builtin_assume_aligned(reinterpret_cast<R*>(lds), 16));
  R* vst = static_cast<R*>(__builtin_assume_aligned(ctl + REP_CTL * ((size_t)a.p.t_max + 2), 16));
  // steps published by the velocity wave [0] and the pose wave [1] (16 bytes)
  int* flg = reinterpret_cast<int*>(vst + 12 * (size_t)(VG ? a.p.t_max : 2 * REP_C));
  R* xs = reinterpret_cast<R*>(flg + 4);
  R* e2s = xs + 6 * (size_t)(a.p.t_max + 1);
  int* is = reinterpret_cast<int*>(e2s + (a.p.t_max + 1));
  // L-BFGS state (memory > 0): gradient, previous iterate and gradient, two-loop
  // vector, pairs in a ring of memory + 1 slots (kept pair i at (head + i) %
  // (memory + 1), i = 0 oldest; the next slot takes the candidate), per pair
  // rho = 1/s.y, alpha, s.y, y.y; reduction buffer
  const int tm2 = 2 * a.p.t_max, mem = a.memory;
  R* gq = reinterpret_cast<R*>(is + (a.p.t_max + 1));
  R* gprev = gq + tm2;
  R* vprev = gprev + tm2;
  R* qv = vprev + tm2;
  R* Sp = qv + tm2;
  R* Yp = Sp + (size_t)(mem + 1) * tm2;
  R* prho = Yp + (size_t)(mem + 1) * tm2;
  R* palpha = prho + (mem + 1);
  R* psy = palpha + (mem + 1);
  R* pyy = psy + (mem + 1);
  R* red = pyy + (mem + 1);
  R* wpar = mem > 0 ? red + 16 : gq;  // parallel reverse sweep: [t_max][REP_PAR_PER_STEP]
  int n_pairs = 0, head = 0;
  const int w = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
  DevModel<R> Mv;
  DevCost<R> Cv;
  if constexpr (VG) {
    Mv = model_in_vgprs(a.M);
    Cv = cost_in_vgprs(a.C);
  }
  const DevModel<R>& M = VG ? Mv : a.M;  // without VG: the arguments themselves, no copy
  const DevCost<R>& C = VG ? Cv : a.C;
  const DevObjective<R>& ob = a.ob;
  const bool cost_terms = ob.w_S != R(0);
  const int T = d.T, nch = (T + REP_C - 1) / REP_C;
  const State<R> x0 = load_state(a.p.x0 + 6 * (size_t)b);
  // segment and offset at x0 do not change over the iterations
  const int idx0 = tr.idx0;
  const R e20 = tr.n > 0 ? seg_dist2(tr, idx0, x0.px, x0.py) : circle_e2(tr, x0.px, x0.py);
  for (int s = 0; s < a.n_steps; ++s) {
    for (int t = threadIdx.x; t < T; t += blockDim.x)
      shield_vel_row(M, clamp_r(Vs[t], M.u_lo[0], M.u_hi[0]), clamp_r(Vs[T + t], M.u_lo[1], M.u_hi[1]),
                     ctl + REP_CTL * t);
    if (threadIdx.x == 0) {
      flg[0] = 0;
      flg[1] = 0;
      *s_last = -1;
      e2s[0] = e20;
    }
    State<R> x = x0;
    int idx = idx0, last = -1;
    R hp = tr.w2 - e20, hob = R(0);
    if (w == 1) {
      if (lane < NOBS) {
        const Obs<R> o = obs_at(tr, lane);
        const R ox = x0.px - o.cx, oy = x0.py - o.cy;
        hob = ox * ox + oy * oy - o.re2;
      }
      if (lane == 0) {
        xs[0] = x0.px; xs[1] = x0.py; xs[2] = x0.psi; xs[3] = x0.vx; xs[4] = x0.vy; xs[5] = x0.om;
        is[0] = idx0;
      }
    }
    // one DCBF transition of the nominal trajectory (window wave): track
    // barrier from e2, obstacle barriers on the lanes; records the last
    // active transition
    auto transition = [&](int t, R px, R py, R e2) {
      const R h = tr.w2 - e2;
      bool act = dcbf_active(C.alpha, hp, h);
      hp = h;
      if (NOBS > 0) {
        bool ao = false;
        if (lane < NOBS) {
          const Obs<R> o = obs_at(tr, lane);
          const R ox = px - o.cx, oy = py - o.cy;
          const R hi = ox * ox + oy * oy - o.re2;
          ao = dcbf_active(C.alpha, hob, hi);
          hob = hi;
        }
        const bool any_ob = __ballot(ao) != 0ull;  // with every lane active
        act = act || any_ob;
      }
      if (act && (ob.w_sq != R(0) || (ob.w_lin != R(0) && t < ob.n_lin))) last = t;
    };
    if constexpr (VG) {
      // (kernels with one workgroup per compute unit: the shield kernel, the
      // latency-mode plan) step by step through the LDS step counters
      __syncthreads();
      if (w == 0 && lane == 0) {
        // velocity wave: the RK4 chain of (v_x, v_y, omega), publishing each step.
        // Each step's control row is read one step ahead: the read completes
        // during the previous step's chain, and the stores and counters in
        // between never wait for it (the counter store waits for nothing).
        // Written out for two steps per iteration, so the two rows alternate
        // between two register sets instead of being copied, with the first
        // step peeled: the loop is entered with the same LDS operations in
        // flight as on its back edge (reads of the next row, stores of the last
        // step, reads of the row after), so every step waits only for its own
        // row.  The empty asm statements keep the reads and stores where they are
        // issued.
        const ShieldVel<R> kv = shield_vel(M);
        auto load_row = [&](R* cc, int t) {
          // rows T and T + 1 (padding) are read at the end and never used
          const R* cr = static_cast<const R*>(__builtin_assume_aligned(ctl + REP_CTL * t, 16));
  #pragma unroll
          for (int c = 0; c < 13; ++c) cc[c] = cr[c];
          // (tied to the state, so the reads are issued before the next step's chain)
          asm volatile("" : "+v"(x.vx), "+v"(x.vy), "+v"(x.om)::"memory");
        };
        auto vel_step = [&](const R* cc, int t) {
          VelStages<R> g;
          shield_vel_step(kv, cc, x.vx, x.vy, x.om, g);
          R* gt = static_cast<R*>(__builtin_assume_aligned(vst + 12 * (size_t)t, 16));
  #pragma unroll
          for (int q = 0; q < 4; ++q) {
            gt[q] = g.vx[q];
            gt[4 + q] = g.vy[q];
            gt[8 + q] = g.om[q];
          }
          // (the velocities of x_{t+1} are the next row's first stage: copied
          // into the states after the pass)
          wave_publish(flg, t + 1);
          // the next step's chain starts after the counter store (the
          // compiler would otherwise hoist it above the stores and publish
          // each step a step late)
          asm volatile("" : "+v"(x.vx), "+v"(x.vy), "+v"(x.om)::"memory");
        };
        R ca[13], cb[13];
        load_row(ca, 0);
        load_row(cb, 1);
        if (T > 0) vel_step(ca, 0);
        load_row(ca, 2);
        int t = 1;
        for (; t + 1 < T; t += 2) {
          vel_step(cb, t);
          load_row(cb, t + 2);
          vel_step(ca, t + 1);
          load_row(ca, t + 3);
        }
        if (t < T) vel_step(cb, t);
        if (T > 0) {
          R* o = xs + 6 * T;
          o[3] = x.vx; o[4] = x.vy; o[5] = x.om;
        }
      } else if (w == 2 && lane < 4) {
        // pose wave: (p_x, p_y, psi) from the stage velocities, step by step as
        // they are published, one RK4 stage per lane (lane q: the heading of
        // stage q and its position derivative, one sine and cosine per lane);
        // the four stages meet through quad broadcasts and every lane forms the
        // same sums in the same order as the one-lane step (rk4_pose)
        const int q = lane;
        const R h = M.dt, h2 = R(0.5) * M.dt, h6 = M.dt * R(1.0 / 6.0);
        int seen = 0;
        for (int t = 0; t < T; ++t) {
          wave_wait(flg, t, seen, a.p.err);
          const R* gt = static_cast<const R*>(__builtin_assume_aligned(vst + 12 * (size_t)t, 16));
          const R vq = gt[q], wq = gt[4 + q];
          const R o0 = gt[8], o1 = gt[9], o2 = gt[10], o3 = gt[11];
          const R psq = q == 0 ? x.psi : fma_r(q == 3 ? h : h2, q == 1 ? o0 : (q == 2 ? o1 : o2), x.psi);
          R ex, ey;
          pose_deriv(psq, vq, wq, ex, ey);
          const R a0 = quad_get<0>(ex), b0 = quad_get<1>(ex), c0 = quad_get<2>(ex), d0 = quad_get<3>(ex);
          const R a1 = quad_get<0>(ey), b1 = quad_get<1>(ey), c1 = quad_get<2>(ey), d1 = quad_get<3>(ey);
          x.px = fma_r(h6, fma_r(R(2), b0 + c0, a0) + d0, x.px);
          x.py = fma_r(h6, fma_r(R(2), b1 + c1, a1) + d1, x.py);
          x.psi = fma_r(h6, fma_r(R(2), o1 + o2, o0) + o3, x.psi);
          R* o = xs + 6 * (t + 1);
          o[0] = x.px; o[1] = x.py; o[2] = x.psi;  // the same values from all four lanes
          wave_publish(flg + 1, t + 1);
          asm volatile("" : "+v"(x.px), "+v"(x.py), "+v"(x.psi)::"memory");
        }
      } else if (w == 1) {
        // window wave: e_y^2, obstacle barriers and activity of each new position.
        // A chunk's segment indices collect on lanes 0 .. REP_C-1 and are stored
        // once after the chunk (a store on every step made the next step wait for
        // it, inside the chain through idx).
        int seen = 0;
        for (int t0 = 0; t0 < T; t0 += REP_C) {
          const int t1 = min(T, t0 + REP_C);
          int ic = 0;
          R ec = R(0);
          auto chunk = [&](auto track_e2) {
            for (int t = t0; t < t1; ++t) {
              wave_wait(flg + 1, t, seen, a.p.err);
              const R px = xs[6 * (t + 1)], py = xs[6 * (t + 1) + 1];
              const R e2 = track_e2(px, py);
              const bool mine = lane == t - t0;
              ic = mine ? idx : ic;
              // without obstacles the activity of every transition is found
              // after the pass, in parallel, from the stored e_y^2
              if constexpr (NOBS > 0)
                transition(t, px, py, e2);
              else
                ec = mine ? e2 : ec;
            }
          };
          // window segments on the lanes of a row, min by DPP (no LDS round trip
          // on the chain through idx); wider windows: one lane, sequential rule
          if (tr.n == 0)
            chunk([&](R px, R py) { return circle_e2(tr, px, py); });
          else if (tr.window <= 7)
            chunk([&](R px, R py) { return row_window(tr, idx, px, py); });
          else
            chunk([&](R px, R py) { return window_min(tr, idx, px, py); });
          if (lane < t1 - t0) {
            is[t0 + 1 + lane] = ic;
            e2s[t0 + 1 + lane] = ec;
          }
        }
      }
      __syncthreads();
      // velocities of x_1 .. x_{T-1}: the first stage of the next step's row
      // (read after the barrier below)
      for (int t = (int)threadIdx.x + 1; t < T; t += blockDim.x) {
        const R* gt = vst + 12 * (size_t)t;
        R* o = xs + 6 * t;
        o[3] = gt[0]; o[4] = gt[4]; o[5] = gt[8];
      }
    } else {
      // (workgroups that share their compute unit with rollout tiles) chunk by
      // chunk between workgroup barriers: waiting waves then sit in the
      // barrier instead of polling (measured faster there)
      __syncthreads();
      for (int st = 0; st <= nch + 1; ++st) {
        if (w == 0 && lane == 0 && st < nch) {
          const int t0 = st * REP_C, t1 = min(T, t0 + REP_C);
          R* gb = vst + (st & 1) * (REP_C * 12);
          // the chunk's control rows are read before its first store: LDS
          // returns in order, so a row read after a step's stores would wait for
          // them inside the RK4 chain
          R cc[REP_C][13];
  #pragma unroll
          for (int k = 0; k < REP_C; ++k) {
            const R* cr = static_cast<const R*>(__builtin_assume_aligned(ctl + REP_CTL * min(t0 + k, t1 - 1), 16));
  #pragma unroll
            for (int c = 0; c < 13; ++c) cc[k][c] = cr[c];
          }
          const ShieldVel<R> kv = shield_vel(M);
  #pragma unroll
          for (int j = 0; j < REP_C; ++j) {
            const int t = t0 + j;
            if (t >= t1) break;
            VelStages<R> g;
            shield_vel_step(kv, cc[j], x.vx, x.vy, x.om, g);
            R* gt = static_cast<R*>(__builtin_assume_aligned(gb + 12 * (t - t0), 16));
  #pragma unroll
            for (int k = 0; k < 4; ++k) {
              gt[k] = g.vx[k];
              gt[4 + k] = g.vy[k];
              gt[8 + k] = g.om[k];
            }
            R* o = xs + 6 * (t + 1);
            o[3] = x.vx; o[4] = x.vy; o[5] = x.om;
          }
        } else if (w == 2 && lane == 0 && st >= 1 && st <= nch) {
          const int t0 = (st - 1) * REP_C, t1 = min(T, t0 + REP_C);
          const R* gb = vst + ((st - 1) & 1) * (REP_C * 12);
          // the chunk's stage velocities are read before its first store (as
          // the control rows in the velocity wave)
          VelStages<R> gc[REP_C];
  #pragma unroll
          for (int j = 0; j < REP_C; ++j) {
            const R* gt = static_cast<const R*>(__builtin_assume_aligned(gb + 12 * min(j, t1 - t0 - 1), 16));
  #pragma unroll
            for (int k = 0; k < 4; ++k) {
              gc[j].vx[k] = gt[k];
              gc[j].vy[k] = gt[4 + k];
              gc[j].om[k] = gt[8 + k];
            }
          }
  #pragma unroll
          for (int j = 0; j < REP_C; ++j) {
            const int t = t0 + j;
            if (t >= t1) break;
            rk4_pose(M, gc[j], x.px, x.py, x.psi);
            R* o = xs + 6 * (t + 1);
            o[0] = x.px; o[1] = x.py; o[2] = x.psi;
          }
        } else if (w == 1 && st >= 2) {
          const int t0 = (st - 2) * REP_C, t1 = min(T, t0 + REP_C);
          // The chunk's segment indices collect on lanes 0 .. REP_C-1 and are
          // stored once after the chunk (a store on every step made the next
          // step wait for it, inside the chain through idx).  The kind of window
          // is chosen once, outside the step loop.
          int ic = 0;
          auto chunk = [&](auto track_e2) {
            for (int t = t0; t < t1; ++t) {
              const R px = xs[6 * (t + 1)], py = xs[6 * (t + 1) + 1];
              const R e2 = track_e2(px, py);
              ic = lane == t - t0 ? idx : ic;
              transition(t, px, py, e2);
            }
          };
          // window segments on the lanes of a row, min by DPP (no LDS round trip
          // on the chain through idx); wider windows: one lane, sequential rule
          if (tr.n == 0)
            chunk([&](R px, R py) { return circle_e2(tr, px, py); });
          else if (tr.window <= 7)
            chunk([&](R px, R py) { return row_window(tr, idx, px, py); });
          else
            chunk([&](R px, R py) { return window_min(tr, idx, px, py); });
          if (lane < t1 - t0) is[t0 + 1 + lane] = ic;
        }
        __syncthreads();
      }
    }
    if constexpr (VG && NOBS == 0) {
      // the last transition t whose DCBF condition fails, from e_y^2 of x_t and
      // x_{t+1} (the same comparison as on the window wave)
      const int t_lim = ob.w_sq != R(0) ? T : (ob.w_lin != R(0) ? min(ob.n_lin, T) : 0);
      int lt = -1;
      for (int t = threadIdx.x; t < t_lim; t += blockDim.x)
        if (dcbf_active(C.alpha, tr.w2 - e2s[t], tr.w2 - e2s[t + 1])) lt = t;
      if (lt >= 0) atomicMax(s_last, lt);
    } else {
      if (w == 1 && lane == 0) *s_last = last;
    }
    __syncthreads();
    const int t_end = cost_terms ? T - 1 : *s_last;
    if (a.method == 1 && t_end >= 0) {
      // gradient (zero after the last active transition), then the L-BFGS step
      for (int t = t_end + 1 + (int)threadIdx.x; t < T; t += blockDim.x) gq[t] = gq[T + t] = R(0);
      if (a.par_rev)
        repair_reverse_par<R, NOBS>(M, C, ob, tr, Vs, T, t_end, a.step, xs, is, gq, wpar);
      else if (w == 0 && lane == 0)
        repair_reverse<R, NOBS>(M, C, ob, tr, Vs, T, t_end, a.step, xs, is, gq);
      __syncthreads();
      lbfgs_step(M, Vs, T, gq, gprev, vprev, qv, Sp, Yp, prho, palpha, psy, pyy, red, mem, tm2, a.step, s > 0,
                 n_pairs, head);
      continue;
    }
    // steps after the last active transition have zero gradient: projection only
    for (int t = t_end + 1 + (int)threadIdx.x; t < T; t += blockDim.x) {
      Vs[t] = clamp_r(Vs[t], M.u_lo[0], M.u_hi[0]);
      Vs[T + t] = clamp_r(Vs[T + t], M.u_lo[1], M.u_hi[1]);
    }
    if (a.par_rev) {
      if (t_end >= 0) repair_reverse_par<R, NOBS>(M, C, ob, tr, Vs, T, t_end, a.step, xs, is, (R*)nullptr, wpar);
    } else if (w == 0 && lane == 0 && t_end >= 0) {
      repair_reverse<R, NOBS>(M, C, ob, tr, Vs, T, t_end, a.step, xs, is, (R*)nullptr);
    }
    __syncthreads();
    if (t_end < 0) break;
  }
}

// One workgroup per problem (rep_blk threads: three waves, or six).
template <class R, int NOBS>
__global__ __launch_bounds__((rep_blk<R, NOBS>())) void k_repair(RepairArgs<R> a) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int s_last;
  const int b = blockIdx.x;
  ProblemDims d;
  if (!load_dims(a.p, b, d)) return;
  R* Vs;
  const TrackView<R> tr = stage_problem(a.p, b, d, a.V_plus, smem, &Vs);
  unsigned char* lds = smem + stage_lds_bytes<R>(a.p.poly_max, a.p.t_max, a.p.obs_max);
  __syncthreads();
  repair_problem<R, NOBS>(a, b, d, tr, Vs, lds, &s_last);
  R* out = a.V_safe + 2 * (size_t)d.t0;
  for (int i = threadIdx.x; i < 2 * d.T; i += blockDim.x) out[i] = Vs[i];
  if (a.exec) execute_problem(a.ex, b, d.t0, d.T, Vs, reinterpret_cast<R*>(lds));
}

// The plant step and warm start as a kernel of their own.
template <class R>
__global__ __launch_bounds__(WAVE) void k_execute(ExecuteArgs<R> a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int b = blockIdx.x;
  const int t0 = a.t_off[b], T = a.t_off[b + 1] - t0;
  if (T < 1 || T > a.t_max) {
    if (threadIdx.x == 0) atomicOr(a.err, DERR_T);
    return;
  }
  execute_problem(a, b, t0, T, a.V_exec + 2 * (size_t)t0, reinterpret_cast<R*>(smem));
}

}  // namespace smppi
