// Many control loops in one launch per tick.
//
// The (loop, tile) work items of every loop are ordered longest-processing-
// time first on the host, and the launch runs one workgroup per item: the
// hardware dispatcher hands workgroups to compute units in index order as
// they free up, which serves the list longest-first without a work counter.
// Each tile publishes its arg-min keys into its loop's slot; the workgroup
// completing a loop's last tile writes that loop's selection and advances
// the loop's tick counter.
//
// Everything the kernel reads per item is behind read-only kernel arguments:
// the loop table (the advancing tick counters live in an array of their own)
// and the plan's copy of each distinct packed model.  Every per-loop and
// per-model field is then a scalar load the compiler may re-issue instead of
// holding it, and with no loop around the item the register budget goes to
// the prediction itself, as in the single-loop tick.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "mpmi_device.hpp"
#include "mpmi_launch.hpp"
#include "mpmi_tick_common.hpp"

namespace mpmi {

struct WorkItem {
  uint32_t loop;
  uint32_t tile;
  uint32_t model;  // index into the plan's model snapshot
  uint32_t pad;
};

// RECHECK (precision FP32_RECHECK64): near-band candidates go to the plan's
// FP64 re-roll list and each tile publishes without a ticket; the re-roll
// launch that follows finalises every loop and advances the tick counters.
template <bool NOISE, bool RECHECK>
__global__ void __launch_bounds__(1024)
multi_kernel(const mpmi_loop_desc* __restrict__ loops, const ModelDev* __restrict__ models,
             const int* __restrict__ n_tiles, const WorkItem* __restrict__ work, Slot* __restrict__ slots,
             uint64_t* __restrict__ ticks, MultiRecheck* __restrict__ rl) {
  __shared__ float4 sK[kLdsKFloat4];
  const WorkItem w = work[blockIdx.x];
  const mpmi_loop_desc* L = &loops[w.loop];
  const ModelDev* md = models + w.model;
  const int basis = md->sys.basis;
  if (basis == MPMI_BASIS_RACE_CAR) stage_K<MPMI_BASIS_RACE_CAR>(md, sK);
  else if (basis == MPMI_BASIS_BALANCE_BOT) stage_K<MPMI_BASIS_BALANCE_BOT>(md, sK);
  else stage_K<MPMI_BASIS_LINEAR>(md, sK);
  GenParams gp;
  gp.seed = L->seed;
  // Written below by the workgroup that completes this loop's tick; every
  // tile of the loop reads it before that (the completing workgroup is the
  // last of the loop's tiles to publish).
  const uint64_t tk = ticks[w.loop];
  gp.tick = ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(tk >> 32)) << 32) |
            (uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)tk);
  gp.loop = (int32_t)w.loop;
  gp.gen = L->gen;
  gp.n_cand = L->n_cand;
  gp.n_seg = L->n_seg;
#pragma unroll
  for (int j = 0; j < MPMI_MAX_INPUT; ++j) gp.grid[j] = L->grid[j] > 0 ? L->grid[j] : 1;
  const int H = L->horizon;
  const int c = (int)w.tile * (int)blockDim.x + (int)threadIdx.x;
  CandResult r;
  if (basis == MPMI_BASIS_RACE_CAR)
    r = evaluate_candidate<MPMI_BASIS_RACE_CAR, NOISE, kMaxHarm, RECHECK>(md, sK, gp, H, L->x_t, L->u_user, L->cand,
                                                                         c, L->first_violation, nullptr, 0);
  else if (basis == MPMI_BASIS_BALANCE_BOT)
    r = evaluate_candidate<MPMI_BASIS_BALANCE_BOT, NOISE, kMaxHarm, RECHECK>(md, sK, gp, H, L->x_t, L->u_user,
                                                                            L->cand, c, L->first_violation, nullptr, 0);
  else
    r = evaluate_candidate<MPMI_BASIS_LINEAR, NOISE, kMaxHarm, RECHECK>(md, sK, gp, H, L->x_t, L->u_user, L->cand, c,
                                                                       L->first_violation, nullptr, 0);
  Slot* slot = &slots[w.loop];
  if constexpr (RECHECK) {
    wave_append(&rl->count, rl->e, r.near, make_uint4(w.loop, (unsigned int)c, w.model, r.safe32 ? 1u : 0u));
    publish_partial(r.ks, r.kf, (unsigned int)__popcll(__ballot(r.safe_counted)),
                    (unsigned int)__popcll(__ballot(r.near)), slot, w.tile);
    return;
  }
  if (reduce_and_publish(r.ks, r.kf, r.safe_counted, slot, (unsigned int)n_tiles[w.loop], w.tile) &&
      threadIdx.x == 0) {
    finalize<MPMI_MAX_INPUT>(md, gp, L->cand, L->u_user, H, slot, L->out);
    ticks[w.loop] = gp.tick + 1;
    __threadfence();
  }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
static double unit_cost(int basis) {
  // Relative per-step cost, for ordering only (race car ~ 4.7x balance bot).
  return basis == MPMI_BASIS_RACE_CAR ? 4.7 : 1.0;
}

hipError_t multi_alloc(MultiPlan& p) {
  size_t cap = 0;
  for (const auto& l : p.host) cap += ((size_t)l.n_cand + 1 + 63) / 64;
  p.work_capacity = cap;
  hipError_t e;
  if ((e = hipMalloc(&p.d_loops, sizeof(mpmi_loop_desc) * p.n_loops)) != hipSuccess) return e;
  if ((e = hipMalloc(&p.d_ntiles, sizeof(int) * p.n_loops)) != hipSuccess) return e;
  if ((e = hipMalloc(&p.d_work, sizeof(WorkItem) * (cap > 0 ? cap : 1))) != hipSuccess) return e;
  if ((e = hipMalloc(&p.d_slots, sizeof(Slot) * p.n_loops)) != hipSuccess) return e;
  if ((e = hipMalloc(&p.d_ticks, sizeof(uint64_t) * p.n_loops)) != hipSuccess) return e;
  p.model_of_loop.assign(p.n_loops, 0);
  p.model_src.clear();
  for (int l = 0; l < p.n_loops; ++l) {
    const void* m = p.host[l].model;
    int k = 0;
    while (k < (int)p.model_src.size() && p.model_src[k] != m) ++k;
    if (k == (int)p.model_src.size()) p.model_src.push_back(m);
    p.model_of_loop[l] = k;
  }
  if ((e = hipMalloc(&p.d_models, sizeof(ModelDev) * p.model_src.size())) != hipSuccess) return e;
  // FP64 re-roll list: room for every candidate of every loop; count and
  // ticket start at zero (the re-roll launch leaves them at zero).
  size_t total = 0;
  for (const auto& l : p.host) total += (size_t)l.n_cand + 1;
  if ((e = hipMalloc(&p.d_recheck, multi_recheck_bytes(total))) != hipSuccess) return e;
  if ((e = hipMemset(p.d_recheck, 0, 256)) != hipSuccess) return e;
  if ((e = hipMalloc(&p.d_model_idx, sizeof(int) * p.n_loops)) != hipSuccess) return e;
  if ((e = hipMemcpy(p.d_model_idx, p.model_of_loop.data(), sizeof(int) * p.n_loops, hipMemcpyHostToDevice)) !=
      hipSuccess)
    return e;
  std::vector<uint64_t> tk(p.n_loops);
  for (int l = 0; l < p.n_loops; ++l) tk[l] = p.host[l].tick;
  if ((e = hipMemcpy(p.d_ticks, tk.data(), sizeof(uint64_t) * p.n_loops, hipMemcpyHostToDevice)) != hipSuccess)
    return e;
  if ((e = hipMemcpy(p.d_loops, p.host.data(), sizeof(mpmi_loop_desc) * p.n_loops, hipMemcpyHostToDevice)) !=
      hipSuccess)
    return e;
  std::vector<unsigned char> s(sizeof(Slot) * p.n_loops);
  slot_reset_image(s.data(), p.n_loops);
  return hipMemcpy(p.d_slots, s.data(), s.size(), hipMemcpyHostToDevice);
}

void multi_free(MultiPlan& p) {
  if (p.d_loops) (void)hipFree(p.d_loops);
  if (p.d_ntiles) (void)hipFree(p.d_ntiles);
  if (p.d_work) (void)hipFree(p.d_work);
  if (p.d_slots) (void)hipFree(p.d_slots);
  if (p.d_ticks) (void)hipFree(p.d_ticks);
  if (p.d_models) (void)hipFree(p.d_models);
  if (p.d_recheck) (void)hipFree(p.d_recheck);
  if (p.d_model_idx) (void)hipFree(p.d_model_idx);
  p.d_recheck = nullptr;
  p.d_model_idx = nullptr;
  p.d_loops = nullptr;
  p.d_ntiles = nullptr;
  p.d_work = nullptr;
  p.d_slots = nullptr;
  p.d_ticks = nullptr;
  p.d_models = nullptr;
}

int device_cu_count() {
  int dev = 0, ncu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 1;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 1;
  return ncu > 0 ? ncu : 1;
}

// Builds the longest-first work list for `block`, uploads it and re-takes the
// model snapshot (synchronous).
hipError_t multi_plan(MultiPlan& p, int block) {
  // The work list may be in use by launches still queued on any stream.
  hipError_t e0 = hipDeviceSynchronize();
  if (e0 != hipSuccess) return e0;
  std::vector<int> nt(p.n_loops);
  std::vector<int> order(p.n_loops);
  size_t total = 0;
  for (int l = 0; l < p.n_loops; ++l) {
    nt[l] = (p.host[l].n_cand + 1 + block - 1) / block;
    total += nt[l];
    order[l] = l;
  }
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    return p.host[a].horizon * unit_cost(p.basis[a]) > p.host[b].horizon * unit_cost(p.basis[b]);
  });
  std::vector<WorkItem> items;
  items.reserve(total);
  for (int l : order)
    for (int t = 0; t < nt[l]; ++t) items.push_back(WorkItem{(uint32_t)l, (uint32_t)t, (uint32_t)p.model_of_loop[l], 0u});
  // Snapshot of the packed models (re-taken at every re-plan).
  for (size_t k = 0; k < p.model_src.size(); ++k) {
    e0 = hipMemcpy(p.d_models + k, p.model_src[k], sizeof(ModelDev), hipMemcpyDeviceToDevice);
    if (e0 != hipSuccess) return e0;
  }
  hipError_t e = hipMemcpy(p.d_work, items.data(), sizeof(WorkItem) * items.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) return e;
  e = hipMemcpy(p.d_ntiles, nt.data(), sizeof(int) * p.n_loops, hipMemcpyHostToDevice);
  if (e != hipSuccess) return e;
  p.n_work = (int)items.size();
  p.block = block;
  return hipDeviceSynchronize();
}

hipError_t multi_launch(const MultiPlan& p, hipStream_t st) {
  MultiRecheck* rl = (MultiRecheck*)p.d_recheck;
  const bool re = p.precision == MPMI_PREC_FP32_RECHECK64;
  if (p.noisy && re)
    multi_kernel<true, true><<<p.n_work, p.block, 0, st>>>(p.d_loops, p.d_models, p.d_ntiles, p.d_work, p.d_slots,
                                                           p.d_ticks, rl);
  else if (p.noisy)
    multi_kernel<true, false><<<p.n_work, p.block, 0, st>>>(p.d_loops, p.d_models, p.d_ntiles, p.d_work, p.d_slots,
                                                            p.d_ticks, rl);
  else if (re)
    multi_kernel<false, true><<<p.n_work, p.block, 0, st>>>(p.d_loops, p.d_models, p.d_ntiles, p.d_work, p.d_slots,
                                                            p.d_ticks, rl);
  else
    multi_kernel<false, false><<<p.n_work, p.block, 0, st>>>(p.d_loops, p.d_models, p.d_ntiles, p.d_work, p.d_slots,
                                                             p.d_ticks, rl);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !re) return e;
  return launch_multi_recheck64(p.d_loops, p.d_models, p.d_model_idx, p.d_slots, p.d_ticks, p.d_recheck, p.n_loops,
                                device_cu_count() * 4, st);
}

}  // namespace mpmi
