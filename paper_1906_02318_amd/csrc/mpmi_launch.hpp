// Host-side launch wrappers shared between the C-ABI layer and the kernel
// translation units (no validation here: the C-ABI layer validates first).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/mpmi.h"

namespace mpmi {

size_t model_bytes();
size_t slot_bytes();

hipError_t launch_pack(const mpmi_system& sys, int dim, int state_feat0, const double* K, void* model,
                       hipStream_t st);
hipError_t launch_tick(int basis, const void* model, const mpmi_tick_desc& d, const float* x_t,
                       const float* u_user, const float* cand, void* slot, mpmi_selection* out,
                       int16_t* fv, float* traj, hipStream_t st);
hipError_t launch_rollout(int basis, const void* model, int Nc, int S, int H, const float* x0,
                          const float* cand, float* traj, hipStream_t st);
hipError_t launch_mask(int basis, const void* model, int Nc, int H, const float* traj, int16_t* fv,
                       float* mm, hipStream_t st);
hipError_t launch_select(const void* model, int Nc, int S, int H, const float* cand, const int16_t* fv,
                         const float* u_user, int loop, void* slot, mpmi_selection* out, hipStream_t st);
hipError_t launch_gen(const void* model, const mpmi_tick_desc& d, const float* u_user, const float* cand,
                      float* cand_out, hipStream_t st);

// Koopman fit (FP64): Gram accumulation, reduction, Cholesky solve.
size_t fit_workspace_bytes();
hipError_t launch_fit(const mpmi_system& sys, int dim, const double* X, const double* U, const double* Y,
                      int64_t T, double ridge, double* K_out, void* work, hipStream_t st);

}  // namespace mpmi
