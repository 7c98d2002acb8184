// Host-side declarations shared by the translation units of libsmppi.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/smppi.h"
#include "kernels.hpp"

struct smppi_ctx_s {
  int device = 0;
  int n_cu = 0;
  int max_lds = 65536;
  void* scratch = nullptr;
  size_t scratch_bytes = 0;
  uint32_t* tickets = nullptr;
  int n_tickets = 0;
  uint32_t* err = nullptr;
  void* noalloc = nullptr;  // device address of the fixed scratch of the no-allocation entry point
  std::vector<void*> retired;
  char last[512] = {0};  // message of the last non-OK status
};

extern "C" smppi_status smppi_device_errors(smppi_ctx ctx, uint32_t* flags);

namespace smppi {

constexpr int kMaxT = 4096;
constexpr int kMaxPoly = 4096;
constexpr int kMaxObs = 64;
constexpr int kMaxMemory = 16;  // L-BFGS pairs of the shield
constexpr int kMaxStageLds = 65536;

// Obstacle slots staged per problem: kernels with obstacles run a fixed count
// of kMaxObs barriers (unused slots hold an inert barrier).
inline int obs_slots(const smppi_track* t) { return t->obs_max > 0 ? kMaxObs : 0; }

smppi_status fail(smppi_ctx ctx, smppi_status s, const char* fmt, ...);
smppi_status hip_fail(smppi_ctx ctx, hipError_t e, const char* what);
smppi_status ensure_scratch(smppi_ctx ctx, size_t bytes);
smppi_status ensure_tickets(smppi_ctx ctx, int n);
struct AdjScratch {
  size_t r;            // dtype bytes
  int nblk;            // adjoint workgroups per problem (ceil(k_max / 64))
  int n_slices;        // slices of the partial sum (ceil(nblk / SUM_SLICE))
  int n_chunks;        // 64-output chunks of a control sequence (ceil(2 t_max / 64))
  size_t part_bytes, slice_bytes, tickets;  // slice_bytes includes the [B] validity flags at its end
  size_t ck_off, ck_bytes;                   // checkpoint region: offset in the scratch, size
  size_t pad_off, pad_bytes;                 // FP32 obstacle slots: offset, size
  int n_problems;
};
AdjScratch adjoint_scratch(const smppi_batch* b);
size_t batch_scratch_bytes(const smppi_batch* b);
smppi_status need_scratch(smppi_ctx ctx, size_t bytes, int tickets, const char* what);
smppi_status check_launch(smppi_ctx ctx, const char* what);
smppi_status validate_batch(smppi_ctx ctx, const smppi_batch* b);
smppi_status validate_model(smppi_ctx ctx, const smppi_model* m);
smppi_status validate_cost(smppi_ctx ctx, const smppi_cost* c);
smppi_status validate_track(smppi_ctx ctx, const smppi_track* t, smppi_dtype dt, int t_max);
smppi_status validate_objective(smppi_ctx ctx, const smppi_objective* o);
smppi_status validate_repair(smppi_ctx ctx, const smppi_repair_opts* o);
int adj_seg_len(int t_max);

template <class R> DevModel<R> dev_model(const smppi_model* m);
template <class R> DevCost<R> dev_cost(const smppi_cost* c);
template <class R> DevObjective<R> dev_objective(const smppi_objective* o);
template <class R>
ProblemArgs<R> problem_args(smppi_ctx ctx, const smppi_batch* b, const smppi_track* t, const smppi_noise* n,
                            const void* x0, const uint32_t* iter);
// Plant step + warm start fused into the shield kernel (plans with both).
struct ExecFuse {
  const void* dist;
  int32_t n_dist;
  void* x;
  void* V;
  uint32_t* iter;
};

template <class R>
RepairArgs<R> repair_args(smppi_ctx ctx, const smppi_batch* b, const smppi_model* m, const smppi_cost* c,
                          const smppi_track* t, const void* x0, const void* Vp, const smppi_repair_opts* o, void* Vs,
                          const ExecFuse* ex);
template <class R>
smppi_status repair_t(smppi_ctx ctx, const smppi_batch* b, const smppi_model* m, const smppi_cost* c,
                      const smppi_track* t, const void* x0, const void* Vp, const smppi_repair_opts* o, void* Vs,
                      hipStream_t s, hipEvent_t kernel_start = nullptr, hipEvent_t kernel_stop = nullptr,
                      const ExecFuse* ex = nullptr);
template <class R>
smppi_status execute_t(smppi_ctx ctx, const smppi_batch* b, const smppi_model* m, const void* Ve, const void* Vp,
                       const void* dist, int32_t n_dist, void* x, void* V, uint32_t* iter, hipStream_t s);

}  // namespace smppi
