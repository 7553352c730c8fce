// Race-car tick with the shared-coefficient part of the contraction on BF16
// matrix cores (precision MPMI_PREC_BF16X3), plus the FP32 recheck of every
// candidate that comes within eps of a constraint.
//
// Per step, each lane (one candidate) forms the 27 features made of state
// alone (21 quadratics and sin/cos psi x (vx, vy, r)) whose K rows are shared
// by every candidate; the input-dependent terms stay folded into per-lane FP32
// coefficients as in the FP32 path.  The 27 features are split into BF16
// hi + lo parts and written to LDS; each wave then runs, for its four groups
// of 16 candidates, hi*Khi + hi*Klo + lo*Khi on v_mfma_f32_16x16x32_bf16 with
// FP32 accumulation (about 16 mantissa bits per product), and reads its own
// six outputs back.  The horizon loop is wave-uniform (a matrix instruction
// needs every lane), and a lane that left the safe set keeps its state frozen.
//
// A candidate whose margin to some constraint is below that constraint's eps
// at some step up to its first violation is appended to a recheck list
// instead of publishing; a second launch re-rolls the listed candidates in
// FP32, publishes them, and its last workgroup finalises the selection.
#include <hip/hip_runtime.h>

#include "mpmi_device.hpp"
#include "mpmi_launch.hpp"
#include "mpmi_tick_common.hpp"

namespace mpmi {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

constexpr int kWaves = 4;            // waves per workgroup (256 threads)
constexpr int kArow = 40;            // bf16 per LDS feature row (32 + 8 pad = 80 B)

// Safety verdict of x (min_margin's rule: every checked margin positive, a
// NaN margin unsafe) and whether some constraint margin is within its eps of
// zero (either side), with the track's centreline evaluated once.
template <int DEG>
__device__ __forceinline__ bool check_rc(const ModelDev* __restrict__ md, const float* x, bool* near) {
  const ConstSafety* sc = safety_of(md);
  float mm = INFINITY;
  bool nan = false, nr = false;
  const int mask = sc->comp_mask;
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    if (mask & (1 << k)) {
      const float mg = sc->comp_lim[k] - fabsf(x[k]);
      nan |= (mg != mg);
      mm = fminf(mm, mg);
    }
  }
  const int nb = sc->n_box;
#pragma unroll
  for (int b = 0; b < MPMI_MAX_BOX; ++b) {
    if (b < nb) {
      // x[box_index] by bit masks: a select chain on a run-time index is
      // turned into an indexed stack load, which would keep x in memory.
      const int bi = sc->box_index[b];
      uint32_t xb = 0u;
#pragma unroll
      for (int k = 0; k < 6; ++k) xb |= __float_as_uint(x[k]) & (bi == k ? 0xffffffffu : 0u);
      const float mg = sc->bb_lim[b] - fabsf(__uint_as_float(xb));
      nr |= fabsf(mg) < md->sys.eps_box[b];
    }
  }
  if (sc->has_track) {
    float rho;
    const float rc = track_centre<DEG>(sc, x, &rho);
    const float mg = sc->trk_lim - fabsf(rho - rc);
    nan |= (mg != mg);
    mm = fminf(mm, mg);
    nr |= fabsf(mg) < md->sys.eps_track;
  }
  *near = nr;
  return !nan && mm > 0.0f;
}

typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));

// hi = RNE_bf16(v) and lo = RNE_bf16(v - hi) for two features at once
// (v_cvt_pk_bf16_f32), packed two per 32-bit word.
__device__ __forceinline__ void split_pair(float a, float b, uint32_t* hi, uint32_t* lo) {
  bf16x2_t h;
  h[0] = (__bf16)a;
  h[1] = (__bf16)b;
  const uint32_t hb = __builtin_bit_cast(uint32_t, h);
  bf16x2_t l;
  l[0] = (__bf16)(a - __uint_as_float(hb << 16));
  l[1] = (__bf16)(b - __uint_as_float(hb & 0xffff0000u));
  *hi = hb;
  *lo = __builtin_bit_cast(uint32_t, l);
}

__device__ __forceinline__ uint16_t bf16_hi(float v) { return (uint16_t)bf16_bits_rne_u(v); }

// The 32 shared-coefficient features of the race-car step, zero-padded:
// f < 21: x_k x_l in (k <= l) order; 21..23: sin psi (vx, vy, r); 24..26:
// cos psi (vx, vy, r).  Nested unrolled loops keep every index a compile-time
// constant (the state stays in registers).
__device__ __forceinline__ void rc_shared_features(const float* x, float sp, float cp, float* f) {
  int q = 0;
#pragma unroll
  for (int k = 0; k < 6; ++k)
#pragma unroll
    for (int l = k; l < 6; ++l) f[q++] = x[k] * x[l];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    f[21 + r] = sp * x[3 + r];
    f[24 + r] = cp * x[3 + r];
  }
#pragma unroll
  for (int r = 27; r < 32; ++r) f[r] = 0.0f;
}

// B operand of the step: the 27 shared K rows (k) x 6 outputs (n) as BF16
// hi/lo splits, zero-padded to 32 x 16.
__device__ __forceinline__ void rc_b_operand(const float4* sK, int lane, bf16x8_t* bhi, bf16x8_t* blo) {
  const float* Ks = reinterpret_cast<const float*>(sK) + kRcStepOff;
  const int n = lane & 15, k0 = (lane >> 4) * 8;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int k = k0 + i;
    const float v = (n < 6 && k < kRcStepRows) ? Ks[k * 6 + n] : 0.0f;
    const uint16_t h = bf16_hi(v);
    const float vh = __uint_as_float((uint32_t)h << 16);
    const uint16_t l = bf16_hi(v - vh);
    (*bhi)[i] = __builtin_bit_cast(__bf16, h);
    (*blo)[i] = __builtin_bit_cast(__bf16, l);
  }
}

// One BF16X3 prediction step of a wave (every lane takes part: the matrix
// instructions need the whole wave): y = folded input terms (FP32) + the
// shared-coefficient contraction on the matrix cores, for this lane's state x.
__device__ __forceinline__ void rc_bf16x3_step(const Stepper<MPMI_BASIS_RACE_CAR>& stp, const float* x,
                                               bf16x8_t bhi, bf16x8_t blo, uint16_t (*sAw)[64][kArow],
                                               float (*sDw)[64], int lane, float* y) {
  // The FP32 path's hardware sine and cosine (the recheck re-rolls with it).
  const float sp = __sinf(x[2]), cp = __cosf(x[2]);
  // Per-step shared-coefficient features, split into BF16 hi/lo, to LDS,
  // eight at a time.
  float feat[32];
  rc_shared_features(x, sp, cp, feat);
#pragma unroll
  for (int k8 = 0; k8 < 4; ++k8) {
    uint32_t h[4], l[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) split_pair(feat[k8 * 8 + 2 * i], feat[k8 * 8 + 2 * i + 1], &h[i], &l[i]);
    *reinterpret_cast<uint4*>(&sAw[0][lane][k8 * 8]) = make_uint4(h[0], h[1], h[2], h[3]);
    *reinterpret_cast<uint4*>(&sAw[1][lane][k8 * 8]) = make_uint4(l[0], l[1], l[2], l[3]);
  }
  __builtin_amdgcn_wave_barrier();
  // Four groups of 16 candidates: D = Ahi Bhi + Ahi Blo + Alo Bhi.  Lane
  // (col, quarter) holds outputs col of four consecutive candidates.
#pragma unroll
  for (int rb = 0; rb < 4; ++rb) {
    const int row = rb * 16 + (lane & 15), k0 = (lane >> 4) * 8;
    const bf16x8_t ah = *reinterpret_cast<const bf16x8_t*>(&sAw[0][row][k0]);
    const bf16x8_t al = *reinterpret_cast<const bf16x8_t*>(&sAw[1][row][k0]);
    f32x4_t acc = {0.f, 0.f, 0.f, 0.f};
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bhi, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, blo, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bhi, acc, 0, 0, 0);
    const int col = lane & 15;
    if (col < 6)
      *reinterpret_cast<float4*>(&sDw[col][rb * 16 + (lane >> 4) * 4]) = make_float4(acc[0], acc[1], acc[2], acc[3]);
  }
  __builtin_amdgcn_wave_barrier();
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    float v = fmaf(stp.Tc[j], cp, fmaf(stp.Ts[j], sp, stp.cu[j]));
#pragma unroll
    for (int k = 0; k < 6; ++k) v = fmaf(stp.L[k][j], x[k], v);
    y[j] = v + sDw[j][lane];
  }
  __builtin_amdgcn_wave_barrier();
}

template <int DEG>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 4)))
tick_bf16_race_car_kernel(const ModelDev* __restrict__ md, GenParams gp, int H, const float* __restrict__ x_t,
                          const float* __restrict__ u_user, const float* __restrict__ cand,
                          Slot* __restrict__ slot, int16_t* __restrict__ fv_out, RecheckList* __restrict__ rl,
                          int capacity) {
  __shared__ float4 sK[kLdsKFloat4];
  __shared__ __attribute__((aligned(16))) uint16_t sA[kWaves][2][64][kArow];  // [wave][hi/lo][cand][k]
  __shared__ __attribute__((aligned(16))) float sD[kWaves][8][64];            // [wave][output][cand]
  stage_K<MPMI_BASIS_RACE_CAR>(md, sK);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int Nc = gp.n_cand + 1;
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = c < Nc;

  bf16x8_t bhi, blo;
  rc_b_operand(sK, lane, &bhi, &blo);

  float x[6], u[2], u0[2];
#pragma unroll
  for (int j = 0; j < 6; ++j) x[j] = x_t[j];
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    u0[j] = valid ? cand_value(gp, md, cand, u_user, c, 0, j) : 0.0f;
    u[j] = u0[j];
  }
  Stepper<MPMI_BASIS_RACE_CAR> stp;  // folded per-lane coefficients (FP32)
  stp.set_input(md, sK, u);
  bool alive = valid, near = false;
  int fv = H + 1;
  const int S = gp.n_seg;
  int gcur = 0;
  int nxt = (H + S - 1) / S;  // first s - 1 of the next segment
  for (int s = 1; s <= H; ++s) {
    if (!__any(alive)) break;  // wave-uniform
    if (s - 1 >= nxt) {
      gcur = ((s - 1) * S) / H;
      nxt = ((gcur + 1) * H + S - 1) / S;
#pragma unroll
      for (int j = 0; j < 2; ++j) u[j] = valid ? cand_value(gp, md, cand, u_user, c, gcur, j) : 0.0f;
      stp.set_input(md, sK, u);
    }
    float y[6];
    rc_bf16x3_step(stp, x, bhi, blo, sA[wave], sD[wave], lane, y);
    if (alive) {
#pragma unroll
      for (int j = 0; j < 6; ++j) x[j] = y[j];
      bool nr;
      const bool ok = check_rc<DEG>(md, x, &nr);
      near |= nr;
      if (!ok) {
        fv = s;
        alive = false;
      }
    }
  }
  // Near-boundary candidates go to the FP32 recheck; the rest publish now.
  bool listed = false;
  if (valid && near) {
    const unsigned int at = atomicAdd(&rl->count, 1u);
    if ((int)at < capacity) {
      rl->idx[at] = c;
      listed = true;
    }
  }
  if (valid && !listed && fv_out) fv_out[c] = (int16_t)fv;
  const bool pub = valid && !listed;
  const float cst = pub ? cost_of<2>(md, u0, u_user) : 0.0f;
  const bool safe = pub && fv == H + 1;
  const unsigned long long ks = safe ? safe_key(cst, c) : kKeyNone;
  const unsigned long long kf = (pub && !safe) ? fallback_key(fv, cst, c) : kKeyNone;
  // Publish without completing the slot (the recheck launch finalises).
  __shared__ unsigned long long s_ks[kWaves], s_kf[kWaves];
  __shared__ unsigned int s_cnt[kWaves], s_re[kWaves];
  const unsigned long long wks = wave_min_u64(ks), wkf = wave_min_u64(kf);
  const unsigned int wcnt = (unsigned int)__popcll(__ballot(safe && c > 0));
  const unsigned int wre = (unsigned int)__popcll(__ballot(listed));
  if (lane == 0) {
    s_ks[wave] = wks;
    s_kf[wave] = wkf;
    s_cnt[wave] = wcnt;
    s_re[wave] = wre;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long bks = kKeyNone, bkf = kKeyNone;
    unsigned int bcnt = 0, bre = 0;
    for (int w = 0; w < kWaves; ++w) {
      bks = s_ks[w] < bks ? s_ks[w] : bks;
      bkf = s_kf[w] < bkf ? s_kf[w] : bkf;
      bcnt += s_cnt[w];
      bre += s_re[w];
    }
    SubSlot* ss = &slot->sub[blockIdx.x % kSubSlots];
    if (bks != kKeyNone) atomicMin(&ss->key_safe, bks);
    if (bkf != kKeyNone) atomicMin(&ss->key_fb, bkf);
    if (bcnt) atomicAdd(&ss->count, (unsigned long long)bcnt);
    if (bre) atomicAdd(&ss->n_recheck, bre);
  }
}

// FP32 re-roll of the listed candidates, then the selection.  Every workgroup
// publishes (possibly empty keys) so the last one can finalise.
template <int DEG>
__global__ void __launch_bounds__(256)
recheck_race_car_kernel(const ModelDev* __restrict__ md, GenParams gp, int H, const float* __restrict__ x_t,
                        const float* __restrict__ u_user, const float* __restrict__ cand,
                        Slot* __restrict__ slot, mpmi_selection* __restrict__ out,
                        int16_t* __restrict__ fv_out, RecheckList* __restrict__ rl, int capacity) {
  __shared__ float4 sK[kLdsKFloat4];
  stage_K<MPMI_BASIS_RACE_CAR>(md, sK);
  const unsigned int cnt_raw = rl->count;
  const int count = (int)(cnt_raw < (unsigned int)capacity ? cnt_raw : (unsigned int)capacity);
  unsigned long long ks = kKeyNone, kf = kKeyNone;
  unsigned int n_safe_local = 0;
  const int stride = gridDim.x * blockDim.x;
  for (int e0 = blockIdx.x * blockDim.x; e0 < count; e0 += stride) {
    const int e = e0 + threadIdx.x;
    const int c = e < count ? rl->idx[e] : gp.n_cand + 1;  // past the end: an invalid lane
    const CandResult r = evaluate_candidate<MPMI_BASIS_RACE_CAR, false, DEG>(md, sK, gp, H, x_t, u_user, cand, c,
                                                                      fv_out, nullptr, 0);
    ks = r.ks < ks ? r.ks : ks;
    kf = r.kf < kf ? r.kf : kf;
    n_safe_local += r.safe_counted ? 1u : 0u;
  }
  // A lane may have served several listed candidates: add its safe count to
  // the slot directly (reduce_and_publish counts one flag per lane).
  unsigned int wsum = n_safe_local;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) wsum += __shfl_xor(wsum, off, 64);
  if ((threadIdx.x & 63) == 0 && wsum) atomicAdd(&slot->sub[blockIdx.x % kSubSlots].count, (unsigned long long)wsum);
  if (reduce_and_publish(ks, kf, false, slot, gridDim.x, blockIdx.x) && threadIdx.x == 0) {
    finalize<2>(md, gp, cand, u_user, H, slot, out);
    rl->count = 0u;
    __threadfence();
  }
}

// Full-horizon BF16X3 rollout (rollout_batch with MPMI_PREC_BF16X3): the
// tick's step without safety checks, every state stored.  Lanes past Nc
// take part in the wave's matrix instructions and store nothing.
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 4)))
rollout_bf16_race_car_kernel(const ModelDev* __restrict__ md, int Nc, int S, int H, const float* __restrict__ x0,
                             const float* __restrict__ cand, float* __restrict__ traj, long long traj_ld) {
  __shared__ float4 sK[kLdsKFloat4];
  __shared__ __attribute__((aligned(16))) uint16_t sA[kWaves][2][64][kArow];
  __shared__ __attribute__((aligned(16))) float sD[kWaves][8][64];
  stage_K<MPMI_BASIS_RACE_CAR>(md, sK);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = c < Nc;
  const int cc = valid ? c : Nc - 1;  // lanes past the end read a valid candidate
  bf16x8_t bhi, blo;
  rc_b_operand(sK, lane, &bhi, &blo);
  float x[6], u[2];
#pragma unroll
  for (int j = 0; j < 6; ++j) x[j] = x0[j];
  Stepper<MPMI_BASIS_RACE_CAR> stp;
  int gcur = -1;
  for (int s = 1; s <= H; ++s) {
    const int g = ((s - 1) * S) / H;
    if (g != gcur) {
      gcur = g;
#pragma unroll
      for (int j = 0; j < 2; ++j) u[j] = cand[((size_t)g * 2 + j) * (size_t)Nc + cc];
      stp.set_input(md, sK, u);
    }
    float y[6];
    rc_bf16x3_step(stp, x, bhi, blo, sA[wave], sD[wave], lane, y);
#pragma unroll
    for (int j = 0; j < 6; ++j) x[j] = y[j];
    if (valid) {
#pragma unroll
      for (int j = 0; j < 6; ++j)
        __builtin_nontemporal_store(x[j], &traj[((size_t)(s - 1) * 6 + j) * (size_t)traj_ld + c]);
    }
  }
}

hipError_t launch_rollout_bf16(const void* model, int Nc, int S, int H, const float* x0, const float* cand,
                               float* traj, long long traj_ld, hipStream_t st) {
  const unsigned grid = (unsigned)(((long long)Nc + 255) / 256);
  rollout_bf16_race_car_kernel<<<grid, 256, 0, st>>>((const ModelDev*)model, Nc, S, H, x0, cand, traj, traj_ld);
  return hipGetLastError();
}

// Room for both arrays of the list (the FP64 re-roll's kept entries follow the listed ones).
size_t recheck_bytes(int capacity) { return sizeof(RecheckList) + 2 * sizeof(int) * (size_t)capacity; }

template <int DEG>
static hipError_t bf16_dispatch(const ModelDev* md, const GenParams& gp, int H, const float* x_t, const float* u_user,
                                const float* cand, Slot* sl, mpmi_selection* out, int16_t* fv, RecheckList* rl,
                                int capacity, int recheck_grid, hipStream_t st) {
  const unsigned grid = (unsigned)(((long long)gp.n_cand + 1 + 255) / 256);
  tick_bf16_race_car_kernel<DEG><<<grid, 256, 0, st>>>(md, gp, H, x_t, u_user, cand, sl, fv, rl, capacity);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  recheck_race_car_kernel<DEG><<<recheck_grid, 256, 0, st>>>(md, gp, H, x_t, u_user, cand, sl, out, fv, rl, capacity);
  return hipGetLastError();
}

hipError_t launch_tick_bf16(const mpmi_system& sys, const void* model, const mpmi_tick_desc& d, const float* x_t,
                            const float* u_user, const float* cand, void* slot, mpmi_selection* out, int16_t* fv,
                            void* recheck, int capacity, int recheck_grid, hipStream_t st) {
  GenParams gp;
  gp.seed = d.seed;
  gp.tick = d.tick;
  gp.loop = d.loop;
  gp.gen = d.gen;
  gp.n_cand = d.n_cand;
  gp.n_seg = d.n_seg;
  for (int j = 0; j < MPMI_MAX_INPUT; ++j) gp.grid[j] = d.grid[j] > 0 ? d.grid[j] : 1;
  const ModelDev* md = (const ModelDev*)model;
  if (track_degree(sys) <= kSmallTrackDeg)
    return bf16_dispatch<kSmallTrackDeg>(md, gp, d.horizon, x_t, u_user, cand, (Slot*)slot, out, fv,
                                         (RecheckList*)recheck, capacity, recheck_grid, st);
  return bf16_dispatch<kMaxHarm>(md, gp, d.horizon, x_t, u_user, cand, (Slot*)slot, out, fv, (RecheckList*)recheck,
                                 capacity, recheck_grid, st);
}

}  // namespace mpmi
