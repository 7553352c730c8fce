// Kernels of the control tick: fused tick (generate -> predict with early exit
// -> safety -> selection, one launch), and the separable stages rollout_batch,
// safe_mask, select_min_intervention, candidate generation and model packing.
//
// Work decomposition: one candidate per lane (candidates are independent,
// Alg. 2's parallel loop), the state kept in VGPRs across the whole horizon,
// K staged once per workgroup in LDS and read with broadcast loads, so the
// contraction is VALU FMAs fed from LDS with no HBM traffic.  The
// arg-min is a 64-bit key reduced across the wave with shuffles, across the
// workgroup in LDS, and across workgroups with one atomicMin per workgroup;
// the last workgroup to finish decodes the key (no second launch; an
// FP32_RECHECK64 tick adds the filter and FP64 re-roll launches of
// mpmi_recheck64.hip, whose last workgroup decodes it instead).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "mpmi_device.hpp"
#include "mpmi_launch.hpp"
#include "mpmi_tick_common.hpp"

namespace mpmi {

// ---------------------------------------------------------------------------
// Fused tick, FP32
// ---------------------------------------------------------------------------
// RECHECK (precision FP32_RECHECK64): candidates with a checked margin within
// the FP32 band are appended to the recheck list (with their FP32 verdict)
// instead of publishing, and the workgroup publishes without a ticket; the
// filter and FP64 re-roll launches that follow complete the slot.
template <int BASIS, bool NOISE, int DEG, bool RECHECK>
__global__ void __launch_bounds__(1024)
tick_fp32_kernel(const ModelDev* __restrict__ md, GenParams gp, int H, const float* __restrict__ x_t,
                 const float* __restrict__ u_user, const float* __restrict__ cand,
                 Slot* __restrict__ slot, mpmi_selection* __restrict__ out,
                 int16_t* __restrict__ fv_out, float* __restrict__ traj, long long traj_ld,
                 const mpmi_selection* __restrict__ gate, RecheckList* __restrict__ rl) {
  constexpr int MS = Dims<BASIS>::M;
  // Gated form (fallback after a proposal tick): nothing to do if the gate
  // selection already found a safe candidate.  Uniform across the grid.
  if (gate && gate->status == MPMI_OK) return;
  __shared__ float4 sK[kLdsKFloat4];
  stage_K<BASIS>(md, sK);
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  const CandResult r = evaluate_candidate<BASIS, NOISE, DEG, RECHECK>(md, sK, gp, H, x_t, u_user, cand, c, fv_out,
                                                                      traj, (size_t)traj_ld);
  if constexpr (RECHECK) {
    wave_append(&rl->count, rl->idx, r.near, (c << 1) | (r.safe32 ? 1 : 0));
    publish_partial(r.ks, r.kf, (unsigned int)__popcll(__ballot(r.safe_counted)),
                    (unsigned int)__popcll(__ballot(r.near)), slot, blockIdx.x);
  } else {
    if (reduce_and_publish(r.ks, r.kf, r.safe_counted, slot, gridDim.x, blockIdx.x) && threadIdx.x == 0)
      finalize<MS>(md, gp, cand, u_user, H, slot, out);
  }
}

// ---------------------------------------------------------------------------
// Separable stages
// ---------------------------------------------------------------------------
template <int BASIS>
__global__ void __launch_bounds__(1024)
rollout_fp32_kernel(const ModelDev* __restrict__ md, int Nc, int S, int H, const float* __restrict__ x0,
                    const float* __restrict__ cand, float* __restrict__ traj, long long traj_ld) {
  constexpr int NS = Dims<BASIS>::N, MS = Dims<BASIS>::M;
  __shared__ float4 sK[kLdsKFloat4];
  stage_K<BASIS>(md, sK);
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= Nc) return;
  const int n = md->n, m = md->m;
  float x[NS], u[MS];
#pragma unroll
  for (int j = 0; j < NS; ++j) x[j] = (j < n) ? x0[j] : 0.0f;
  int gcur = -1;
  Stepper<BASIS> stp;
  for (int s = 1; s <= H; ++s) {
    const int g = ((s - 1) * S) / H;
    if (g != gcur) {
      gcur = g;
#pragma unroll
      for (int j = 0; j < MS; ++j) u[j] = (j < m) ? cand[((size_t)g * m + j) * (size_t)Nc + c] : 0.0f;
      stp.set_input(md, sK, u);
    }
    stp.step(md, sK, x);
    settle_state<NS>(x);
#pragma unroll
    for (int j = 0; j < NS; ++j)
      if (j < n) __builtin_nontemporal_store(x[j], &traj[((size_t)(s - 1) * n + j) * (size_t)traj_ld + c]);
  }
}

// Safety of stored trajectories (Alg. 2's check over predicted states), one
// candidate per lane.  The states of kMaskChunk steps are loaded before any
// of them is checked, so a lane keeps that many steps' loads in flight
// instead of one memory round trip per step; they are then checked in step
// order, so the first violation and the least margin up to it are those of
// a step-by-step scan.  At most kMaskChunk - 1 steps past the first violation
// are read and ignored.
constexpr int kMaskChunk = 4;

// NEAR: also the near-boundary bitmask (bit c % 32 of word c / 32 set when
// some checked state of candidate c has a margin within its FP32 band), one
// ballot per wave.  Blocks are whole waves; lanes past Nc take part in the
// ballot only.
template <int NS, bool NEAR>
__global__ void __launch_bounds__(1024)
mask_kernel(const ModelDev* __restrict__ md, int Nc, int H, const float* __restrict__ traj, long long traj_ld,
            int16_t* __restrict__ fv_out, float* __restrict__ mm_out, uint32_t* __restrict__ near_bits) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = c < Nc;
  const int cc = valid ? c : Nc - 1;  // lanes past the end scan a valid candidate and store nothing
  const int n = md->n;
  int fv = H + 1;
  float least = INFINITY;
  bool near = false;
  for (int s0 = 1; s0 <= H && fv > H; s0 += kMaskChunk) {
    float x[kMaskChunk][NS];
    // Every load is issued: a step past the horizon rereads the last one
    // (never checked) and a component past n rereads component n - 1 (then
    // zeroed), so no load sits behind a branch that waits for it.
#pragma unroll
    for (int k = 0; k < kMaskChunk; ++k) {
      const int s = min(s0 + k, H);
#pragma unroll
      for (int j = 0; j < NS; ++j) {
        const int jj = j < n ? j : n - 1;
        const float v = traj[((size_t)(s - 1) * n + jj) * (size_t)traj_ld + cc];
        x[k][j] = j < n ? v : 0.0f;
      }
    }
#pragma unroll
    for (int k = 0; k < kMaskChunk; ++k) {
      if (s0 + k > H) break;
      const float mg = NEAR ? min_margin_near<NS>(md, x[k], &near) : min_margin<NS>(md, x[k]);
      least = (mg != mg) ? mg : fminf(least, mg);
      if (!(mg > 0.0f)) {
        fv = s0 + k;
        break;
      }
    }
  }
  if (valid) {
    fv_out[c] = (int16_t)fv;
    if (mm_out) mm_out[c] = least;
  }
  if (NEAR) {
    const unsigned long long b = __ballot(valid && near);
    const int lane = threadIdx.x & 63;
    const int c0 = c - lane;
    if (lane == 0 && c0 < Nc) near_bits[c0 >> 5] = (uint32_t)b;
    if (lane == 32 && c0 + 32 < Nc) near_bits[(c0 >> 5) + 1] = (uint32_t)(b >> 32);
  }
}

// Selection over given first violations (Alg. 2's arg-min).  A pass of a
// workgroup covers kSelectPer * kSelectBlock candidates, kSelectPer per lane
// (lane t takes base + q * kSelectBlock + t, so each load stays coalesced),
// all of a lane's loads issued before its keys are formed; passes repeat over
// at most kSelectParts workgroups.  A workgroup per 256 candidates would make
// the parts' slot atomics, not the ten bytes read per candidate, the cost at
// a million candidates.  The keys carry the candidate index, so the minimum
// does not depend on which part saw which candidate.
constexpr int kSelectBlock = 1024, kSelectPer = 4;
constexpr unsigned int kSelectParts = 256;

template <int MS>
__global__ void __launch_bounds__(kSelectBlock)
select_kernel(const ModelDev* __restrict__ md, GenParams gp, int H, const float* __restrict__ cand,
              const int16_t* __restrict__ fv_in, const float* __restrict__ u_user,
              Slot* __restrict__ slot, mpmi_selection* __restrict__ out) {
  const int Nc = gp.n_cand + 1;
  const int m = md->m;
  const long long pass = (long long)gridDim.x * kSelectBlock * kSelectPer;
  // The cost with unused components weighted zero: the same sum as the
  // tick's (each skipped term adds 0 * 0 to a non-negative sum), with no
  // branch for the compiler to sink a candidate load into.
  float uu[MS], hw[MS];
#pragma unroll
  for (int j = 0; j < MS; ++j) {
    uu[j] = j < m ? u_user[j] : 0.0f;
    hw[j] = j < m ? md->half_inv[j] : 0.0f;
  }
  unsigned long long ks = kKeyNone, kf = kKeyNone;
  unsigned int n_safe = 0;  // uniform across the wave
  for (long long base = (long long)blockIdx.x * kSelectBlock * kSelectPer; base < Nc; base += pass) {
    float u0[kSelectPer][MS];
    int fv[kSelectPer];
    // Lanes past the end read the last candidate (in bounds) and drop it.
#pragma unroll
    for (int q = 0; q < kSelectPer; ++q) {
      const int cc = (int)min(base + q * kSelectBlock + threadIdx.x, (long long)Nc - 1);
#pragma unroll
      for (int j = 0; j < MS; ++j) u0[q][j] = cand[(size_t)(j < m ? j : m - 1) * (size_t)Nc + cc];
      fv[q] = fv_in[cc];
    }
    // One wait for all of them: the empty statement takes every loaded value,
    // so no key arithmetic is scheduled between the loads.
    static_assert(kSelectPer == 4 && MS == 4, "operand list below");
    asm volatile("" : "+v"(u0[0][0]), "+v"(u0[0][1]), "+v"(u0[0][2]), "+v"(u0[0][3]), "+v"(u0[1][0]),
                      "+v"(u0[1][1]), "+v"(u0[1][2]), "+v"(u0[1][3]), "+v"(u0[2][0]), "+v"(u0[2][1]),
                      "+v"(u0[2][2]), "+v"(u0[2][3]), "+v"(u0[3][0]), "+v"(u0[3][1]), "+v"(u0[3][2]),
                      "+v"(u0[3][3]), "+v"(fv[0]), "+v"(fv[1]), "+v"(fv[2]), "+v"(fv[3]));
#pragma unroll
    for (int q = 0; q < kSelectPer; ++q)
#pragma unroll
      for (int j = 1; j < MS; ++j) u0[q][j] = j < m ? u0[q][j] : 0.0f;  // m >= 1
#pragma unroll
    for (int q = 0; q < kSelectPer; ++q) {
      const int c = (int)(base + q * kSelectBlock + threadIdx.x);
      const bool valid = base + q * kSelectBlock + threadIdx.x < Nc;
      float cst = 0.0f;
#pragma unroll
      for (int j = 0; j < MS; ++j) {
        const float d = (u0[q][j] - uu[j]) * hw[j];
        cst = fmaf(d, d, cst);
      }
      const bool safe = valid && fv[q] == H + 1;
      const unsigned long long a = safe ? safe_key(cst, c) : kKeyNone;
      const unsigned long long b =
          (valid && !safe) ? fallback_key(fv[q] < 1 ? 1 : (fv[q] > H ? H : fv[q]), cst, c) : kKeyNone;
      ks = a < ks ? a : ks;
      kf = b < kf ? b : kf;
      n_safe += (unsigned int)__popcll(__ballot(safe && c > 0));
    }
  }
  if (publish_wave_counted(ks, kf, n_safe, slot, gridDim.x, blockIdx.x) && threadIdx.x == 0)
    finalize<MS>(md, gp, cand, u_user, H, slot, out);
}

__global__ void gen_kernel(const ModelDev* __restrict__ md, GenParams gp, const float* __restrict__ u_user,
                           const float* __restrict__ cand, float* __restrict__ cand_out) {
  const int Nc = gp.n_cand + 1;
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= Nc) return;
  const int m = md->m;
  for (int g = 0; g < gp.n_seg; ++g)
    for (int j = 0; j < m; ++j)
      cand_out[((size_t)g * m + j) * (size_t)Nc + c] = cand_value(gp, md, cand, u_user, c, g, j);
}

// ---------------------------------------------------------------------------
// Model packing
// ---------------------------------------------------------------------------
__global__ void pack_kernel(mpmi_system sys, int dim, int state_feat0, const double* __restrict__ K,
                            ModelDev* __restrict__ md) {
  const int t = threadIdx.x;
  const int n = sys.n_state;
  // FP32 K, zero-padded to 8 columns and MPMI_MAX_DIM rows.
  for (int e = t; e < MPMI_MAX_DIM * 8; e += blockDim.x) {
    const int f = e >> 3, j = e & 7;
    md->K[f][j] = (f < dim && j < n) ? (float)K[(size_t)f * n + j] : 0.0f;
  }
  // FP64 K for the re-roll, and (race car) its step rows in step order.
  for (int e = t; e < MPMI_MAX_DIM * 8; e += blockDim.x) {
    const int f = e >> 3, j = e & 7;
    md->m64.K[f][j] = (f < dim && j < n) ? K[(size_t)f * n + j] : 0.0;
  }
  for (int e = t; e < kRcStepRows * 8; e += blockDim.x) {
    const int q = e >> 3, j = e & 7;
    md->m64.Kstep[q][j] = (sys.basis == MPMI_BASIS_RACE_CAR && j < n) ? K[(size_t)rc_step_row(q) * n + j] : 0.0;
  }
  // Race-car step table (the rows the per-step contraction reads, in order).
  for (int e = t; e < kStepWords; e += blockDim.x) {
    const int q = e / 6, j = e % 6;
    md->Kstep[e] = (sys.basis == MPMI_BASIS_RACE_CAR && q < kRcStepRows && j < n)
                       ? (float)K[(size_t)rc_step_row(q) * n + j]
                       : 0.0f;
  }
  // Residual R = K - E as BF16 hi/lo splits in B-operand order of a 16x16x32
  // MFMA: lane l holds column (l & 15), rows kb*32 + (l >> 4)*8 + [0..8).
  for (int e = t; e < 2 * 64 * 8; e += blockDim.x) {
    const int kb = e >> 9, lane = (e >> 3) & 63, q = e & 7;
    const int col = lane & 15, row = kb * 32 + (lane >> 4) * 8 + q;
    double r = 0.0;
    if (row < dim && col < n) {
      r = K[(size_t)row * n + col];
      if (row == state_feat0 + col) r -= 1.0;
    }
    const float rf = (float)r;
    const uint32_t hi = bf16_bits_rne_u(rf);
    const float lo = rf - __uint_as_float(hi << 16);
    const uint32_t lob = bf16_bits_rne_u(lo);
    const int word = (kb * 64 + lane) * 4 + (q >> 1);
    const int sh = (q & 1) * 16;
    atomicOr(&md->Rhi[word], hi << sh);
    atomicOr(&md->Rlo[word], lob << sh);
  }
  if (t == 0) {
    md->sys = sys;
    md->magic = kModelMagic;
    md->dim = dim;
    md->n = n;
    md->m = sys.n_input;
    md->state_feat0 = state_feat0;
    for (int b = 0; b < MPMI_MAX_BOX; ++b)
      md->safe.bb_lim[b] = (b < sys.n_box) ? (float)((double)sys.box_bound[b] - (double)sys.box_infl[b]) : 0.0f;
    for (int b = 0; b < MPMI_MAX_BOX; ++b) md->safe.box_index[b] = (b < sys.n_box) ? sys.box_index[b] : 0;
    int cmask = 0;
    for (int k = 0; k < MPMI_MAX_STATE; ++k) md->safe.comp_lim[k] = INFINITY;
    for (int b = 0; b < sys.n_box; ++b) {
      const int k = sys.box_index[b];
      cmask |= 1 << k;
      md->safe.comp_lim[k] = fminf(md->safe.comp_lim[k], md->safe.bb_lim[b]);
    }
    md->safe.comp_mask = cmask;
    // FP32 bands: per component the band of its binding (least-limit) box.
    for (int k = 0; k < MPMI_MAX_STATE; ++k) md->safe.comp_eps[k] = 0.0f;
    for (int b = 0; b < sys.n_box; ++b) {
      const int k = sys.box_index[b];
      if (md->safe.bb_lim[b] == md->safe.comp_lim[k]) md->safe.comp_eps[k] = fmaxf(md->safe.comp_eps[k], sys.eps32_box[b]);
    }
    md->safe.trk_eps = sys.has_track ? sys.eps32_track : 0.0f;
    md->safe.n_box = sys.n_box;
    md->safe.has_track = sys.has_track;
    md->safe.trk_lim = (float)((double)sys.track_half - (double)sys.track_infl);
    // r_c(phi) = r0 + sum_k a_k sin(f_k phi + p_k)
    //          = r0 + sum_k a_k [cos p_k sin(f_k phi) + sin p_k cos(f_k phi)]
    //          = r0 + sum_k a_k [cos p_k sin(phi) U_{f_k-1}(c) + sin p_k T_{f_k}(c)],  c = cos phi,
    // collected into monomials of c in FP64: P (cos terms + r0), Q (sin terms).
    double T[kMaxHarm + 1][kMaxHarm + 1], U[kMaxHarm + 1][kMaxHarm + 1];
    for (int h = 0; h <= kMaxHarm; ++h)
      for (int k = 0; k <= kMaxHarm; ++k) T[h][k] = U[h][k] = 0.0;
    T[0][0] = 1.0;
    T[1][1] = 1.0;
    U[0][0] = 1.0;
    U[1][1] = 2.0;
    for (int h = 1; h < kMaxHarm; ++h)
      for (int k = 0; k <= kMaxHarm; ++k) {
        T[h + 1][k] = (k > 0 ? 2.0 * T[h][k - 1] : 0.0) - T[h - 1][k];
        U[h + 1][k] = (k > 0 ? 2.0 * U[h][k - 1] : 0.0) - U[h - 1][k];
      }
    double P[kMaxHarm + 1], Q[kMaxHarm];
    for (int k = 0; k <= kMaxHarm; ++k) P[k] = 0.0;
    for (int k = 0; k < kMaxHarm; ++k) Q[k] = 0.0;
    int hmax = 0;
    if (sys.has_track) {
      P[0] = sys.track_r0;
      for (int q = 0; q < sys.track_n; ++q) {
        const int f = sys.track_freq[q];
        const double a = sys.track_amp[q], ph = sys.track_phase[q];
        for (int k = 0; k <= f; ++k) P[k] += a * sin(ph) * T[f][k];
        if (f >= 1)
          for (int k = 0; k < f; ++k) Q[k] += a * cos(ph) * U[f - 1][k];
        hmax = f > hmax ? f : hmax;
      }
    }
    for (int k = 0; k <= kMaxHarm; ++k) md->safe.trk_p[k] = (float)P[k];
    for (int k = 0; k < kMaxHarm; ++k) md->safe.trk_q[k] = (float)Q[k];
    md->safe.hmax = hmax;
    // The FP64 re-roll's safety set, noise and basis description.
    Model64* m = &md->m64;
    m->comp_mask = cmask;
    for (int k = 0; k < MPMI_MAX_STATE; ++k) m->comp_lim[k] = INFINITY;
    for (int b = 0; b < sys.n_box; ++b) {
      const int k = sys.box_index[b];
      const double lim = (double)sys.box_bound[b] - (double)sys.box_infl[b];
      m->comp_lim[k] = lim < m->comp_lim[k] ? lim : m->comp_lim[k];
    }
    m->has_track = sys.has_track;
    m->trk_lim = (double)sys.track_half - (double)sys.track_infl;
    for (int k = 0; k <= kMaxHarm; ++k) m->trk_p[k] = P[k];
    for (int k = 0; k < kMaxHarm; ++k) m->trk_q[k] = Q[k];
    for (int j = 0; j < MPMI_MAX_STATE; ++j) m->sigma[j] = j < n ? (double)sys.noise_sigma[j] : 0.0;
    m->n_atoms = sys.n_atoms;
    for (int q = 0; q < MPMI_MAX_ATOMS; ++q) {
      m->atom_kind[q] = sys.atom_kind[q];
      m->atom_var[q] = sys.atom_var[q];
    }
    for (int f = 0; f < MPMI_MAX_DIM; ++f) {
      m->feat_a[f] = sys.feat_a[f];
      m->feat_b[f] = sys.feat_b[f];
    }
    int noisy = 0;
    for (int j = 0; j < 8; ++j) noisy |= (j < n && sys.noise_sigma[j] > 0.0f) ? 1 : 0;
    md->has_noise = noisy;
    for (int j = 0; j < MPMI_MAX_INPUT; ++j)
      md->half_inv[j] = (j < sys.n_input) ? (float)(2.0 / ((double)sys.u_hi[j] - (double)sys.u_lo[j])) : 0.0f;
  }
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------
static GenParams make_gen(const mpmi_tick_desc& d) {
  GenParams gp;
  gp.seed = d.seed;
  gp.tick = d.tick;
  gp.loop = d.loop;
  gp.gen = d.gen;
  gp.n_cand = d.n_cand;
  gp.n_seg = d.n_seg;
  for (int j = 0; j < MPMI_MAX_INPUT; ++j) gp.grid[j] = d.grid[j] > 0 ? d.grid[j] : 1;
  return gp;
}

static inline unsigned blocks_for(long long n, int block) { return (unsigned)((n + block - 1) / block); }

hipError_t launch_pack(const mpmi_system& sys, int dim, int state_feat0, const double* K, void* model,
                       hipStream_t st) {
  hipError_t e = hipMemsetAsync(model, 0, sizeof(ModelDev), st);
  if (e != hipSuccess) return e;
  pack_kernel<<<1, 256, 0, st>>>(sys, dim, state_feat0, K, (ModelDev*)model);
  return hipGetLastError();
}

template <int BASIS, int DEG>
static void tick_dispatch(bool noisy, unsigned grid, int block, hipStream_t st, const ModelDev* md,
                          const GenParams& gp, int H, const float* x_t, const float* u_user, const float* cand,
                          Slot* sl, mpmi_selection* out, int16_t* fv, float* traj, long long ld,
                          const mpmi_selection* gate, RecheckList* rl) {
  if (rl) {
    if (noisy)
      tick_fp32_kernel<BASIS, true, DEG, true>
          <<<grid, block, 0, st>>>(md, gp, H, x_t, u_user, cand, sl, out, fv, traj, ld, gate, rl);
    else
      tick_fp32_kernel<BASIS, false, DEG, true>
          <<<grid, block, 0, st>>>(md, gp, H, x_t, u_user, cand, sl, out, fv, traj, ld, gate, rl);
  } else {
    if (noisy)
      tick_fp32_kernel<BASIS, true, DEG, false>
          <<<grid, block, 0, st>>>(md, gp, H, x_t, u_user, cand, sl, out, fv, traj, ld, gate, rl);
    else
      tick_fp32_kernel<BASIS, false, DEG, false>
          <<<grid, block, 0, st>>>(md, gp, H, x_t, u_user, cand, sl, out, fv, traj, ld, gate, rl);
  }
}

hipError_t launch_tick(const mpmi_system& sys, const void* model, const mpmi_tick_desc& d, const float* x_t,
                       const float* u_user, const float* cand, void* slot, mpmi_selection* out,
                       int16_t* fv, float* traj, long long traj_ld, hipStream_t st, const mpmi_selection* gate,
                       void* recheck, int recheck_capacity, int recheck_grid) {
  const GenParams gp = make_gen(d);
  const int block = d.block > 0 ? d.block : 256;
  const unsigned grid = blocks_for((long long)d.n_cand + 1, block);
  const ModelDev* md = (const ModelDev*)model;
  Slot* sl = (Slot*)slot;
  const bool noisy = system_noisy(sys);
  RecheckList* rl = (RecheckList*)recheck;
  switch (sys.basis) {
    case MPMI_BASIS_LINEAR:
      tick_dispatch<MPMI_BASIS_LINEAR, kMaxHarm>(noisy, grid, block, st, md, gp, d.horizon, x_t, u_user, cand, sl,
                                                 out, fv, traj, traj_ld, gate, rl);
      break;
    case MPMI_BASIS_BALANCE_BOT:
      tick_dispatch<MPMI_BASIS_BALANCE_BOT, kMaxHarm>(noisy, grid, block, st, md, gp, d.horizon, x_t, u_user, cand,
                                                      sl, out, fv, traj, traj_ld, gate, rl);
      break;
    case MPMI_BASIS_CUSTOM:
      tick_dispatch<MPMI_BASIS_CUSTOM, kMaxHarm>(noisy, grid, block, st, md, gp, d.horizon, x_t, u_user, cand, sl,
                                                 out, fv, traj, traj_ld, gate, rl);
      break;
    default:
      if (track_degree(sys) <= kSmallTrackDeg)
        tick_dispatch<MPMI_BASIS_RACE_CAR, kSmallTrackDeg>(noisy, grid, block, st, md, gp, d.horizon, x_t, u_user,
                                                           cand, sl, out, fv, traj, traj_ld, gate, rl);
      else
        tick_dispatch<MPMI_BASIS_RACE_CAR, kMaxHarm>(noisy, grid, block, st, md, gp, d.horizon, x_t, u_user, cand,
                                                     sl, out, fv, traj, traj_ld, gate, rl);
      break;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !rl) return e;
  return launch_recheck64(sys, model, d, x_t, u_user, cand, slot, out, fv, recheck, recheck_capacity, recheck_grid,
                          st, gate);
}

hipError_t launch_rollout(int basis, const void* model, int Nc, int S, int H, const float* x0,
                          const float* cand, float* traj, long long traj_ld, hipStream_t st) {
  const int block = 256;
  const unsigned grid = blocks_for(Nc, block);
  const ModelDev* md = (const ModelDev*)model;
  switch (basis) {
    case MPMI_BASIS_LINEAR:
      rollout_fp32_kernel<MPMI_BASIS_LINEAR><<<grid, block, 0, st>>>(md, Nc, S, H, x0, cand, traj, traj_ld);
      break;
    case MPMI_BASIS_BALANCE_BOT:
      rollout_fp32_kernel<MPMI_BASIS_BALANCE_BOT><<<grid, block, 0, st>>>(md, Nc, S, H, x0, cand, traj, traj_ld);
      break;
    case MPMI_BASIS_CUSTOM:
      rollout_fp32_kernel<MPMI_BASIS_CUSTOM><<<grid, block, 0, st>>>(md, Nc, S, H, x0, cand, traj, traj_ld);
      break;
    default:
      rollout_fp32_kernel<MPMI_BASIS_RACE_CAR><<<grid, block, 0, st>>>(md, Nc, S, H, x0, cand, traj, traj_ld);
      break;
  }
  return hipGetLastError();
}

template <int NS>
static void mask_dispatch(unsigned grid, int block, hipStream_t st, const ModelDev* md, int Nc, int H,
                          const float* traj, long long traj_ld, int16_t* fv, float* mm, uint32_t* nb) {
  if (nb) mask_kernel<NS, true><<<grid, block, 0, st>>>(md, Nc, H, traj, traj_ld, fv, mm, nb);
  else mask_kernel<NS, false><<<grid, block, 0, st>>>(md, Nc, H, traj, traj_ld, fv, mm, nb);
}

hipError_t launch_mask(int basis, const void* model, int Nc, int H, const float* traj, long long traj_ld,
                       int16_t* fv, float* mm, uint32_t* near_bits, hipStream_t st) {
  const int block = 256;
  const unsigned grid = blocks_for(Nc, block);
  const ModelDev* md = (const ModelDev*)model;
  switch (basis) {
    case MPMI_BASIS_LINEAR:
    case MPMI_BASIS_CUSTOM:
      mask_dispatch<MPMI_MAX_STATE>(grid, block, st, md, Nc, H, traj, traj_ld, fv, mm, near_bits);
      break;
    case MPMI_BASIS_BALANCE_BOT:
      mask_dispatch<4>(grid, block, st, md, Nc, H, traj, traj_ld, fv, mm, near_bits);
      break;
    default:
      mask_dispatch<6>(grid, block, st, md, Nc, H, traj, traj_ld, fv, mm, near_bits);
      break;
  }
  return hipGetLastError();
}

hipError_t launch_select(const void* model, int Nc, int S, int H, const float* cand, const int16_t* fv,
                         const float* u_user, int loop, void* slot, mpmi_selection* out, hipStream_t st) {
  GenParams gp{};
  gp.gen = kGenFull;
  gp.n_cand = Nc - 1;
  gp.n_seg = S;
  gp.loop = loop;
  for (int j = 0; j < MPMI_MAX_INPUT; ++j) gp.grid[j] = 1;
  const unsigned grid = std::min(blocks_for(Nc, kSelectBlock * kSelectPer), kSelectParts);
  select_kernel<MPMI_MAX_INPUT><<<grid, kSelectBlock, 0, st>>>(
      (const ModelDev*)model, gp, H, cand, fv, u_user, (Slot*)slot, out);
  return hipGetLastError();
}

hipError_t launch_gen(const void* model, const mpmi_tick_desc& d, const float* u_user, const float* cand,
                      float* cand_out, hipStream_t st) {
  const GenParams gp = make_gen(d);
  const int block = 256;
  gen_kernel<<<blocks_for((long long)d.n_cand + 1, block), block, 0, st>>>((const ModelDev*)model, gp, u_user,
                                                                            cand, cand_out);
  return hipGetLastError();
}

size_t model_bytes() { return sizeof(ModelDev); }
size_t slot_bytes() { return sizeof(Slot); }

void slot_reset_image(unsigned char* dst, int n) {
  Slot r;
  std::memset(&r, 0, sizeof(r));
  for (int i = 0; i < kSubSlots; ++i) r.sub[i].key_safe = r.sub[i].key_fb = r.sub[i].key_safe64 = kKeyNone;
  for (int l = 0; l < n; ++l) std::memcpy(dst + (size_t)l * sizeof(Slot), &r, sizeof(Slot));
}

}  // namespace mpmi
