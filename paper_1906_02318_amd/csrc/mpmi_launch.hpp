// Host-side launch wrappers shared between the C-ABI layer and the kernel
// translation units (no validation here: the C-ABI layer validates first).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <vector>

#include "../../include/mpmi.h"

namespace mpmi {

// Custom-basis ticks use at most this many threads per workgroup (each lane
// keeps its w and atoms in LDS).
constexpr int kCustomBlock = 256;

size_t model_bytes();
size_t slot_bytes();
// Host image of n slots in their reset state (keys all-ones, counters zero).
void slot_reset_image(unsigned char* dst, int n);

hipError_t launch_pack(const mpmi_system& sys, int dim, int state_feat0, const double* K, void* model,
                       hipStream_t st);
// Process noise is drawn when a state component has a positive sigma (the
// packed model's has_noise flag follows the same rule).
inline bool system_noisy(const mpmi_system& s) {
  for (int j = 0; j < s.n_state && j < 8; ++j)
    if (s.noise_sigma[j] > 0.0f) return true;
  return false;
}

// Highest harmonic of the track (degree of its centreline polynomial in
// cos phi); 0 without a track.
inline int track_degree(const mpmi_system& s) {
  int h = 0;
  if (s.has_track)
    for (int q = 0; q < s.track_n && q < 4; ++q) h = s.track_freq[q] > h ? s.track_freq[q] : h;
  return h;
}

// With `recheck` non-NULL (FP32_RECHECK64): the FP32 tick lists near-band
// candidates there, then the FP64 re-roll launch (recheck_grid workgroups)
// completes the selection.
hipError_t launch_tick(const mpmi_system& sys, const void* model, const mpmi_tick_desc& d, const float* x_t,
                       const float* u_user, const float* cand, void* slot, mpmi_selection* out,
                       int16_t* fv, float* traj, long long traj_ld, hipStream_t st,
                       const mpmi_selection* gate = nullptr, void* recheck = nullptr, int recheck_capacity = 0,
                       int recheck_grid = 0);
// Filter and FP64 re-roll of a tick's listed candidates, and the selection
// (mpmi_recheck64.hip); with `gate` set, nothing is finalised when the gate
// record already holds a safe choice.
hipError_t launch_recheck64(const mpmi_system& sys, const void* model, const mpmi_tick_desc& d, const float* x_t,
                            const float* u_user, const float* cand, void* slot, mpmi_selection* out, int16_t* fv,
                            void* recheck, int capacity, int grid, hipStream_t st,
                            const mpmi_selection* gate = nullptr);
size_t multi_recheck_bytes(size_t capacity);
hipError_t launch_multi_recheck64(const mpmi_loop_desc* loops, const void* models, const int* model_of_loop,
                                  void* slots, uint64_t* ticks, void* recheck, int n_loops, int grid, hipStream_t st);
hipError_t launch_rollout(int basis, const void* model, int Nc, int S, int H, const float* x0,
                          const float* cand, float* traj, long long traj_ld, hipStream_t st);
hipError_t launch_mask(int basis, const void* model, int Nc, int H, const float* traj, long long traj_ld,
                       int16_t* fv, float* mm, uint32_t* near_bits, hipStream_t st);
hipError_t launch_select(const void* model, int Nc, int S, int H, const float* cand, const int16_t* fv,
                         const float* u_user, int loop, void* slot, mpmi_selection* out, hipStream_t st);
hipError_t launch_gen(const void* model, const mpmi_tick_desc& d, const float* u_user, const float* cand,
                      float* cand_out, hipStream_t st);

// Koopman fit (FP64): Gram accumulation, reduction, Cholesky solve.
size_t fit_workspace_bytes();
size_t fit_info_offset();  // {int32 status, int32 pad, double cond} of the last solve
hipError_t launch_fit(const mpmi_system& sys, int dim, const double* X, const double* U, const double* Y,
                      int64_t T, double ridge, double* K_out, void* work, hipStream_t st);
// Lifted operator (dim x dim) with targets psi(Y_t, U_t).
hipError_t launch_fit_lifted(const mpmi_system& sys, int dim, const double* X, const double* U, const double* Y,
                             int64_t T, double ridge, double* K_out, void* work, hipStream_t st);

// Basis selection (mpmi_select.hip): workspace bytes for n_gamma penalties,
// and the synchronous selection.
size_t select_workspace_bytes(int n_gamma);
hipError_t launch_select_basis(const mpmi_library& lib, const double* X, const double* U, const double* Y, int64_t T,
                               const double* gammas_host, int n_gamma, double rho, int iters, double* B_out,
                               uint8_t* support, double* resid_host, void* work, hipStream_t st);

// Lifted whole-horizon tick (mpmi_lifted.hip).
size_t lifted_bytes(int h_max);
void lifted_layout(int basis, int n, int m, int D, int* feat_g, int* feat_phi, int* n_phi, int* n_g);
// Host-side pack (synchronous); *n_safe_slots < 0 when more than four state
// components are constrained (then nothing is written).
hipError_t lifted_pack(const mpmi_system& sys, int D, int state_feat0, const void* model, const double* K_dev,
                       int h_max, void* lifted, int* n_safe_slots);
hipError_t launch_tick_lifted(const mpmi_system& sys, void* lifted, int h_max, const mpmi_tick_desc& d,
                              const float* x_t, const float* u_user, const float* cand, void* slot,
                              mpmi_selection* out, int16_t* fv, float* traj, long long traj_ld, int grid_per_cu,
                              hipStream_t st);

// Latency form of the tick (mpmi_split.hip).
hipError_t launch_tick_split(const mpmi_system& sys, int split, const void* model, const mpmi_tick_desc& d,
                             const float* x_t, const float* u_user, const float* cand, void* slot,
                             mpmi_selection* out, int16_t* fv, hipStream_t st);

// BF16X3 race-car tick + FP32 recheck (mpmi_bf16.hip).
constexpr int kRecheckCapacity = 1 << 22;
size_t recheck_bytes(int capacity);
hipError_t launch_rollout_bf16(const void* model, int Nc, int S, int H, const float* x0, const float* cand,
                               float* traj, long long traj_ld, hipStream_t st);
hipError_t launch_tick_bf16(const mpmi_system& sys, const void* model, const mpmi_tick_desc& d, const float* x_t,
                            const float* u_user, const float* cand, void* slot, mpmi_selection* out, int16_t* fv,
                            void* recheck, int capacity, int recheck_grid, hipStream_t st);

// Proposal network (mpmi_mlp.hip).
size_t mlp_workspace_bytes(int B);
hipError_t launch_mlp_forward(const uint16_t* w16, const float* w32, const float* mean, const float* stdv,
                              const float* X, int B, float* Y, void* work, hipStream_t st);
hipError_t launch_mlp_grad(const uint16_t* w16, const float* w32, const float* mean, const float* stdv,
                           const float* X, const float* T, int B, float* grad, float* loss, void* work,
                           hipStream_t st);
hipError_t launch_mlp_adam(float* w32, uint16_t* w16, float* m, float* v, const float* grad, int step, float lr,
                           hipStream_t st);
hipError_t launch_mdn_sample(const void* model, const float* Yrow, int P, uint64_t seed, uint64_t tick, int loop,
                             float* cand, hipStream_t st);
// Forward pass of the one row [x_t; u_user] and P > 0 draws from its head
// into cand (EXPLICIT layout), in one launch; the head goes to head_out, or to
// the workspace's head buffer when head_out is NULL.  w16 16-byte aligned.
hipError_t launch_mlp_row_forward(const float* x_t, const float* u_user, const uint16_t* w16, const float* w32,
                                  const float* mean, const float* stdv, void* work, float* head_out, float** head,
                                  const void* model, int P, uint64_t seed, uint64_t tick, int loop, float* cand,
                                  hipStream_t st);
hipError_t launch_gemm_test(const uint16_t* A, const uint16_t* B, int M, int N, int K, int ta, int tb, float* C,
                            hipStream_t st);

// Device ceiling diagnostics (mpmi_diag.hip): non-packed FP32 FMA rate,
// TFLOP/s; `sink` is any device buffer of >= 4 bytes (never written in
// practice).
hipError_t measure_fma_rate(float* sink, double* tflops);
// Write ceilings on buf (rows * Nc floats, overwritten): the trajectory
// store's pattern and a contiguous stream, GB/s.
hipError_t measure_write_rates(void* buf, int Nc, long long ld, int rows, double* pattern_gbs, double* stream_gbs);
hipError_t measure_read_rates(const void* buf, int Nc, long long ld, int rows, double* pattern_gbs,
                              double* stream_gbs);
// The FP64 re-roll's sin and cos of n doubles (device arrays).
hipError_t launch_sincos64(const double* x, double* sn, double* cs, int n, hipStream_t st);

// Many-loop tick (mpmi_multi.hip).
struct WorkItem;
struct Slot;
struct ModelDev;
struct MultiPlan {
  int n_loops = 0;
  mpmi_loop_desc* d_loops = nullptr;  // device copy of the loop table
  int* d_ntiles = nullptr;            // tiles per loop for the current block size
  WorkItem* d_work = nullptr;         // ordered (loop, tile) items
  Slot* d_slots = nullptr;            // one selection slot per loop
  uint64_t* d_ticks = nullptr;        // per-loop tick counters (advanced on the device)
  ModelDev* d_models = nullptr;       // copy of each distinct packed model
  std::vector<const void*> model_src; // the packed models the copies were taken from
  std::vector<int> model_of_loop;     // loop -> index into d_models
  size_t work_capacity = 0;
  int n_work = 0;
  int block = 256;
  int precision = MPMI_PREC_FP32;     // or MPMI_PREC_FP32_RECHECK64
  void* d_recheck = nullptr;          // MultiRecheck list, one entry per candidate of all loops
  int* d_model_idx = nullptr;         // loop -> index into d_models
  std::vector<mpmi_loop_desc> host;
  std::vector<int> basis;
  bool noisy = false;  // some loop's model draws process noise
};
hipError_t multi_alloc(MultiPlan& p);
void multi_free(MultiPlan& p);
hipError_t multi_plan(MultiPlan& p, int block);
hipError_t multi_launch(const MultiPlan& p, hipStream_t st);
int device_cu_count();

}  // namespace mpmi
