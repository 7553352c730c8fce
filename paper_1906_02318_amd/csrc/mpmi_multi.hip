// Many control loops in one persistent launch per tick.
//
// The (loop, tile) work items of every loop are ordered longest-processing-
// time first on the host and taken from an atomic counter by a grid sized to
// fill the chip.  A workgroup keeps the K of the loop it served last in LDS
// and restages only when the next item belongs to another model.  Each tile
// publishes its arg-min keys into its loop's slot; the workgroup completing a
// loop's last tile writes that loop's selection and advances its tick
// counter; the last workgroup to leave resets the work counter, so the next
// launch (or graph replay) starts clean without a memset.
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
};

struct MultiState {
  unsigned int next;    // next work item
  unsigned int exited;  // workgroups that found the list empty
  unsigned int pad[62];
};

__global__ void __launch_bounds__(1024)
multi_kernel(mpmi_loop_desc* __restrict__ loops, const int* __restrict__ n_tiles,
             const WorkItem* __restrict__ work, int n_work, MultiState* __restrict__ st,
             Slot* __restrict__ slots) {
  __shared__ float4 sK[kLdsKFloat4];
  __shared__ int s_item;
  const ModelDev* cached = nullptr;
  for (;;) {
    if (threadIdx.x == 0) s_item = (int)atomicAdd(&st->next, 1u);
    __syncthreads();
    const int it = s_item;
    __syncthreads();
    if (it >= n_work) break;
    const WorkItem w = work[it];
    mpmi_loop_desc* L = &loops[w.loop];
    const ModelDev* md = (const ModelDev*)L->model;
    const int basis = md->sys.basis;
    if (md != cached) {
      if (basis == MPMI_BASIS_RACE_CAR) stage_K<MPMI_BASIS_RACE_CAR>(md, sK);
      else if (basis == MPMI_BASIS_BALANCE_BOT) stage_K<MPMI_BASIS_BALANCE_BOT>(md, sK);
      else stage_K<MPMI_BASIS_LINEAR>(md, sK);
      cached = md;
    }
    GenParams gp;
    gp.seed = L->seed;
    gp.tick = L->tick;
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
      r = evaluate_candidate<MPMI_BASIS_RACE_CAR>(md, sK, gp, H, L->x_t, L->u_user, L->cand, c,
                                                  L->first_violation, nullptr);
    else if (basis == MPMI_BASIS_BALANCE_BOT)
      r = evaluate_candidate<MPMI_BASIS_BALANCE_BOT>(md, sK, gp, H, L->x_t, L->u_user, L->cand, c,
                                                     L->first_violation, nullptr);
    else
      r = evaluate_candidate<MPMI_BASIS_LINEAR>(md, sK, gp, H, L->x_t, L->u_user, L->cand, c,
                                                L->first_violation, nullptr);
    Slot* slot = &slots[w.loop];
    if (reduce_and_publish(r.ks, r.kf, r.safe_counted, slot, (unsigned int)n_tiles[w.loop]) &&
        threadIdx.x == 0) {
      finalize<MPMI_MAX_INPUT>(md, gp, L->cand, L->u_user, H, slot, L->out);
      L->tick = gp.tick + 1;
      __threadfence();
    }
  }
  if (threadIdx.x == 0) {
    __threadfence();
    if (atomicAdd(&st->exited, 1u) == gridDim.x - 1) {
      st->next = 0u;
      st->exited = 0u;
      __threadfence();
    }
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
  if ((e = hipMalloc(&p.d_state, sizeof(MultiState))) != hipSuccess) return e;
  if ((e = hipMalloc(&p.d_slots, sizeof(Slot) * p.n_loops)) != hipSuccess) return e;
  if ((e = hipMemcpy(p.d_loops, p.host.data(), sizeof(mpmi_loop_desc) * p.n_loops, hipMemcpyHostToDevice)) !=
      hipSuccess)
    return e;
  if ((e = hipMemset(p.d_state, 0, sizeof(MultiState))) != hipSuccess) return e;
  std::vector<Slot> s(p.n_loops);
  for (auto& x : s) {
    x.key_safe = kKeyNone;
    x.key_fb = kKeyNone;
    x.n_safe = x.done = x.n_recheck = x.pad = 0;
  }
  return hipMemcpy(p.d_slots, s.data(), sizeof(Slot) * p.n_loops, hipMemcpyHostToDevice);
}

void multi_free(MultiPlan& p) {
  if (p.d_loops) (void)hipFree(p.d_loops);
  if (p.d_ntiles) (void)hipFree(p.d_ntiles);
  if (p.d_work) (void)hipFree(p.d_work);
  if (p.d_state) (void)hipFree(p.d_state);
  if (p.d_slots) (void)hipFree(p.d_slots);
  p.d_loops = nullptr;
  p.d_ntiles = nullptr;
  p.d_work = nullptr;
  p.d_state = nullptr;
  p.d_slots = nullptr;
}

int multi_max_blocks_per_cu(int block) {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, multi_kernel, block, 0) != hipSuccess) return 1;
  return nb > 0 ? nb : 1;
}

int device_cu_count() {
  int dev = 0, ncu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 1;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 1;
  return ncu > 0 ? ncu : 1;
}

// Builds the longest-first work list for `block` and uploads it (synchronous).
hipError_t multi_plan(MultiPlan& p, int block, int grid) {
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
    for (int t = 0; t < nt[l]; ++t) items.push_back(WorkItem{(uint32_t)l, (uint32_t)t});
  hipError_t e = hipMemcpy(p.d_work, items.data(), sizeof(WorkItem) * items.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) return e;
  e = hipMemcpy(p.d_ntiles, nt.data(), sizeof(int) * p.n_loops, hipMemcpyHostToDevice);
  if (e != hipSuccess) return e;
  p.n_work = (int)items.size();
  p.block = block;
  const int full = device_cu_count() * multi_max_blocks_per_cu(block);
  p.grid = grid > 0 ? grid : full;
  if (p.grid > p.n_work) p.grid = p.n_work > 0 ? p.n_work : 1;
  return hipDeviceSynchronize();
}

hipError_t multi_launch(const MultiPlan& p, hipStream_t st) {
  multi_kernel<<<p.grid, p.block, 0, st>>>(p.d_loops, p.d_ntiles, p.d_work, p.n_work, p.d_state, p.d_slots);
  return hipGetLastError();
}

}  // namespace mpmi
