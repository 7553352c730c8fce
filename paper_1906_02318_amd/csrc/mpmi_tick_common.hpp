// Device code shared by the single-loop and many-loop ticks: candidate
// values, cost, one candidate's prediction with early exit, and the
// workgroup/cross-workgroup arg-min with its last-workgroup finalisation.
#pragma once

#include "mpmi_device.hpp"

namespace mpmi {

// Candidates of one tick left to a re-roll launch, in context-owned device
// memory: BF16X3 lists candidate indices (FP32 re-roll); FP32_RECHECK64
// lists (candidate << 1) | FP32 verdict (1 = safe) (FP64 re-roll), and its
// filter launch copies the entries that can still change the selection to a
// second array of capacity entries after the first (n_keep of them).
struct RecheckList {
  unsigned int count;
  unsigned int n_keep;
  unsigned int pad[62];
  int idx[1];  // capacity entries follow, then (FP32_RECHECK64) capacity kept entries
};

// Candidates of a many-loop tick left to the FP64 re-roll: {loop, candidate,
// model index, FP32 verdict (1 = safe)}; the last workgroup of the re-roll
// launch (ticket `done`) finalises every loop.
struct MultiRecheck {
  unsigned int count;
  unsigned int done;
  unsigned int pad[62];
  uint4 e[1];  // capacity entries follow
};

// Candidate source modes: the three public generators plus FULL (an explicit
// array that already holds candidate 0 in column 0).
constexpr int kGenFull = 3;

__device__ __forceinline__ float cand_value(const GenParams& gp, const ModelDev* __restrict__ md,
                                            const float* __restrict__ cand,
                                            const float* __restrict__ u_user, int c, int g, int j) {
  if (gp.gen == kGenFull) return cand[(size_t)(g * md->m + j) * (size_t)(gp.n_cand + 1) + (size_t)c];
  if (c == 0) return u_user[j];
  return gen_value(gp, md, cand, c, g, j);
}

template <int MS>
__device__ __forceinline__ float cost_of(const ModelDev* __restrict__ md, const float* u0,
                                         const float* __restrict__ u_user) {
  float cst = 0.0f;
#pragma unroll
  for (int j = 0; j < MS; ++j) {
    if (j < md->m) {
      const float d = (u0[j] - u_user[j]) * md->half_inv[j];
      cst = fmaf(d, d, cst);
    }
  }
  return cst;
}

// Workgroup reduction of the two keys and the waves' safe counts (cnt is the
// wave's count, uniform across it), then the part's atomics on its sub-slot
// (part < n_parts; n_parts parts serve this slot in this launch); returns
// true in every thread of the workgroup that completes the slot.  Up to
// kOneLevelParts parts take their ticket on the slot itself (contention stays
// small); more parts take one on their sub-slot first, and the last of each
// sub-slot one on the slot.
constexpr unsigned int kOneLevelParts = 128;
template <bool SAFE64 = false>  // the FP64 re-roll's safe keys go to key_safe64
__device__ __forceinline__ bool publish_wave_counted(unsigned long long ks, unsigned long long kf,
                                                     unsigned int cnt, Slot* __restrict__ slot,
                                                     unsigned int n_parts, unsigned int part) {
  __shared__ unsigned long long s_ks[16], s_kf[16];
  __shared__ unsigned int s_cnt[16];
  __shared__ int s_last;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  ks = wave_min_u64(ks);
  kf = wave_min_u64(kf);
  if (lane == 0) {
    s_ks[wave] = ks;
    s_kf[wave] = kf;
    s_cnt[wave] = cnt;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) >> 6;
    unsigned long long bks = kKeyNone, bkf = kKeyNone;
    unsigned int bcnt = 0;
    for (int w = 0; w < nw; ++w) {
      bks = s_ks[w] < bks ? s_ks[w] : bks;
      bkf = s_kf[w] < bkf ? s_kf[w] : bkf;
      bcnt += s_cnt[w];
    }
    const unsigned int sidx = part % kSubSlots;
    SubSlot* ss = &slot->sub[sidx];
    if (bks != kKeyNone) atomicMin(SAFE64 ? &ss->key_safe64 : &ss->key_safe, bks);
    if (bkf != kKeyNone) atomicMin(&ss->key_fb, bkf);
    bool last = false;
    if (n_parts <= kOneLevelParts) {
      // Few parts: the count needs no ticket, and one ticket on the slot
      // saves a round trip to memory on the completing part's path.
      if (bcnt) atomicAdd(&ss->count, (unsigned long long)bcnt);
      __threadfence();
      last = atomicAdd(&slot->done, 1u) == n_parts - 1;
    } else {
      __threadfence();
      // parts p < n_parts with p % kSubSlots == sidx
      const unsigned int in_sub = (n_parts - sidx + kSubSlots - 1) / kSubSlots;
      const unsigned long long prev = atomicAdd(&ss->count, (1ull << 32) | (unsigned long long)bcnt);
      if ((unsigned int)(prev >> 32) == in_sub - 1) {
        __threadfence();
        last = atomicAdd(&slot->done, 1u) == (unsigned int)kSubSlots - 1;
      }
    }
    s_last = last;
  }
  __syncthreads();
  return s_last != 0;
}

// The same for one candidate per lane: the wave's count is its number of
// lanes with safe_counted set.
__device__ __forceinline__ bool reduce_and_publish(unsigned long long ks, unsigned long long kf,
                                                   bool safe_counted, Slot* __restrict__ slot,
                                                   unsigned int n_parts, unsigned int part) {
  return publish_wave_counted(ks, kf, (unsigned int)__popcll(__ballot(safe_counted)), slot, n_parts, part);
}

// Decodes the slot into the selection and resets the slot (one thread, in
// the part whose ticket completed the slot).  Every slot read is an atomic
// exchange with the reset value, performed where the other parts' atomics
// were: it sees the values they left (their tickets followed their keys) and
// restores the reset state in one step, so no fence is needed here; the other
// inputs were written before the launch, and the selection is read after it.
template <int MS>
__device__ void finalize(const ModelDev* __restrict__ md, const GenParams& gp,
                         const float* __restrict__ cand, const float* __restrict__ u_user, int H,
                         Slot* __restrict__ slot, mpmi_selection* __restrict__ out) {
  unsigned long long ks = kKeyNone, kf = kKeyNone;
  unsigned int n_safe = 0, n_re = 0;
#pragma unroll
  for (int i = 0; i < kSubSlots; ++i) {
    SubSlot* ss = &slot->sub[i];
    const unsigned long long a0 = atomicExch(&ss->key_safe, kKeyNone);
    const unsigned long long a1 = atomicExch(&ss->key_safe64, kKeyNone);
    const unsigned long long a = a0 < a1 ? a0 : a1;
    const unsigned long long b = atomicExch(&ss->key_fb, kKeyNone);
    const unsigned long long n = atomicExch(&ss->count, 0ull);
    const unsigned int r = atomicExch(&ss->n_recheck, 0u);
    ks = a < ks ? a : ks;
    kf = b < kf ? b : kf;
    n_safe += (unsigned int)(n & 0xffffffffull);
    n_re += r;
  }
  (void)atomicExch(&slot->done, 0u);
  int idx, status, fv;
  float cost;
  if (ks != kKeyNone) {
    idx = (int)(ks & 0xffffffffull);
    cost = __uint_as_float((unsigned int)(ks >> 32));
    status = MPMI_OK;
    fv = H + 1;
  } else {
    idx = (int)(kf & 0x1ffffffull);
    cost = __uint_as_float((unsigned int)((kf >> 25) & 0x7fffffffull));
    status = MPMI_NO_SAFE;
    fv = 255 - (int)(kf >> 56);
  }
  mpmi_selection sel;
  sel.idx = idx;
  sel.status = status;
  sel.n_safe = (int)n_safe;
  sel.n_recheck = (int)n_re;
  float dev2 = 0.0f;
#pragma unroll
  for (int j = 0; j < MPMI_MAX_INPUT; ++j) {
    float v = 0.0f;
    if (j < md->m) {
      v = cand_value(gp, md, cand, u_user, idx, 0, j);
      const float d = v - u_user[j];
      dev2 = fmaf(d, d, dev2);
    }
    sel.u_r[j] = v;
  }
  sel.cost = cost;
  sel.deviation = sqrtf(dev2);
  sel.first_violation = fv;
  sel.n_cand = gp.n_cand + 1;
  *out = sel;
}

struct CandResult {
  unsigned long long ks, kf;
  bool safe_counted;
  bool near;    // NEAR instances: some checked state lies within the FP32 band of a constraint
  bool safe32;  // the FP32 verdict: every state safe (valid candidates)
};

// Publishes a workgroup's keys and counts (cnt: the wave's safe count, n_re:
// the wave's re-rolled count, both uniform across the wave) into sub-slot
// part % kSubSlots without taking a ticket: a later launch completes the
// slot.  Every thread of the workgroup calls it.
__device__ __forceinline__ void publish_partial(unsigned long long ks, unsigned long long kf, unsigned int cnt,
                                                unsigned int n_re, Slot* __restrict__ slot, unsigned int part) {
  __shared__ unsigned long long s_ks[16], s_kf[16];
  __shared__ unsigned int s_cnt[16], s_re[16];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  ks = wave_min_u64(ks);
  kf = wave_min_u64(kf);
  if (lane == 0) {
    s_ks[wave] = ks;
    s_kf[wave] = kf;
    s_cnt[wave] = cnt;
    s_re[wave] = n_re;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) >> 6;
    unsigned long long bks = kKeyNone, bkf = kKeyNone;
    unsigned int bcnt = 0, bre = 0;
    for (int w = 0; w < nw; ++w) {
      bks = s_ks[w] < bks ? s_ks[w] : bks;
      bkf = s_kf[w] < bkf ? s_kf[w] : bkf;
      bcnt += s_cnt[w];
      bre += s_re[w];
    }
    SubSlot* ss = &slot->sub[part % kSubSlots];
    if (bks != kKeyNone) atomicMin(&ss->key_safe, bks);
    if (bkf != kKeyNone) atomicMin(&ss->key_fb, bkf);
    if (bcnt) atomicAdd(&ss->count, (unsigned long long)bcnt);
    if (bre) atomicAdd(&ss->n_recheck, bre);
  }
}

// Appends value v of every lane with `flag` set to list[] (one atomic on
// *count per wave; the lanes' order within the wave is kept).  Called by
// every lane of the wave.
template <typename T>
__device__ __forceinline__ void wave_append(unsigned int* __restrict__ count, T* __restrict__ list, bool flag, T v) {
  const unsigned long long b = __ballot(flag);
  if (b == 0ull) return;  // uniform
  const int lane = threadIdx.x & 63;
  const int leader = __ffsll((long long)b) - 1;
  unsigned int base = 0;
  if (lane == leader) base = atomicAdd(count, (unsigned int)__popcll(b));
  base = (unsigned int)__shfl((int)base, leader, 64);
  if (flag) list[base + (unsigned int)__popcll(b & ((1ull << lane) - 1ull))] = v;
}

// Prediction of candidate c with early exit at the first unsafe state
// (Alg. 2 inner loop), then its selection keys.  Lanes with c >= Nc return
// empty keys.  fv_out / traj are optional; traj rows are traj_ld floats apart.  NOISE compiles the process-noise
// draw in (models with a positive sigma); noise-free instances carry none of
// its registers (a noisy instance still skips the draw for a noise-free model).
// DEG is the track polynomial's degree (>= the model's highest harmonic).
//
// NEAR instances also track whether some checked state (steps 1 .. first
// violation) has a margin within its constraint's FP32 band: such a
// candidate is left to the FP64 re-roll, so it gets no keys here (its FP32
// first violation is stored; the re-roll overwrites it when it predicts the
// candidate again).
template <int BASIS, bool NOISE, int DEG = kMaxHarm, bool NEAR = false>
__device__ __forceinline__ CandResult evaluate_candidate(const ModelDev* __restrict__ md, const float4* sK,
                                                         const GenParams& gp, int H,
                                                         const float* __restrict__ x_t,
                                                         const float* __restrict__ u_user,
                                                         const float* __restrict__ cand, int c,
                                                         int16_t* __restrict__ fv_out, float* __restrict__ traj,
                                                         size_t traj_ld) {
  constexpr int NS = Dims<BASIS>::N, MS = Dims<BASIS>::M;
  const int Nc = gp.n_cand + 1;
  const bool valid = c < Nc;
  const int n = md->n, S = gp.n_seg;
  float x[NS], u[MS];
#pragma unroll
  for (int j = 0; j < NS; ++j) x[j] = (j < n) ? x_t[j] : 0.0f;
#pragma unroll
  for (int j = 0; j < MS; ++j) u[j] = (valid && j < md->m) ? cand_value(gp, md, cand, u_user, c, 0, j) : 0.0f;
  // The cost needs only the first segment's input: taken now, so a single
  // float instead of the input vector stays live across the horizon.
  const float cst = valid ? cost_of<MS>(md, u, u_user) : 0.0f;
  Stepper<BASIS> stp;
  stp.set_input(md, sK, u);
  int fv = H + 1;
  bool near = false;
  if (valid) {
    const bool noisy = NOISE && md->has_noise != 0;
    const uint64_t nprefix = noisy ? hash_prefix(gp.seed, gp.tick, (uint64_t)(uint32_t)gp.loop, (uint64_t)c) : 0ull;
    int gcur = 0;
    for (int s = 1; s <= H; ++s) {
      const int g = ((s - 1) * S) / H;
      if (g != gcur) {
        gcur = g;
#pragma unroll
        for (int j = 0; j < MS; ++j) u[j] = (j < md->m) ? cand_value(gp, md, cand, u_user, c, g, j) : 0.0f;
        stp.set_input(md, sK, u);
      }
      stp.step(md, sK, x);
      settle_state<NS>(x);
      if (noisy) add_process_noise<NS>(md->sys.noise_sigma, nprefix, s, n, x);
      if (traj) {
        // Streaming stores: the cloud is written once, for a later reader.
#pragma unroll
        for (int j = 0; j < NS; ++j)
          if (j < n) __builtin_nontemporal_store(x[j], &traj[((size_t)(s - 1) * n + j) * traj_ld + c]);
      }
      const float mg = NEAR ? min_margin_near<NS, DEG>(md, x, &near) : min_margin<NS, DEG>(md, x);
      if (!(mg > 0.0f)) {
        fv = s;
        break;
      }
    }
    if (fv_out) fv_out[c] = (int16_t)fv;
  }
  const bool pub = valid && !(NEAR && near);
  const bool safe = pub && fv == H + 1;
  CandResult r;
  r.ks = safe ? safe_key(cst, c) : kKeyNone;
  r.kf = (pub && !safe) ? fallback_key(fv, cst, c) : kKeyNone;
  r.safe_counted = safe && c > 0;
  r.near = NEAR && valid && near;
  r.safe32 = valid && fv == H + 1;
  return r;
}

// Cost of candidate c (FP32, from its first-segment input, as in the tick).
__device__ __forceinline__ float cost_at(const ModelDev* __restrict__ md, const GenParams& gp,
                                         const float* __restrict__ cand, const float* __restrict__ u_user, int c) {
  float u0[MPMI_MAX_INPUT];
#pragma unroll
  for (int j = 0; j < MPMI_MAX_INPUT; ++j) u0[j] = (j < md->m) ? cand_value(gp, md, cand, u_user, c, 0, j) : 0.0f;
  return cost_of<MPMI_MAX_INPUT>(md, u0, u_user);
}

// K*: the least safe key the FP32 tick published into a slot (key_safe; the
// FP64 re-roll's own keys go to key_safe64), or kKeyNone.
__device__ __forceinline__ unsigned long long published_best(const Slot* __restrict__ slot) {
  unsigned long long k = kKeyNone;
#pragma unroll
  for (int i = 0; i < kSubSlots; ++i) {
    const unsigned long long v = __atomic_load_n(&slot->sub[i].key_safe, __ATOMIC_RELAXED);
    k = v < k ? v : k;
  }
  return k;
}

}  // namespace mpmi
