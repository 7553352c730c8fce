// Device-side building blocks of the MPMI-SC tick: packed model layout,
// basis evaluation + Koopman step, safety margins, counter-based candidate
// generation and the orderable selection keys.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/mpmi.h"
#include "mpmi_launch.hpp"

namespace mpmi {

constexpr uint32_t kModelMagic = 0x4d504d49u;  // "MPMI"
constexpr int kMaxHarm = 8;
constexpr int kStepWords = 168;  // per-step K table (race car: 27 rows x 6)                     // highest track frequency
constexpr uint64_t kGoldenGamma = 0x9E3779B97F4A7C15ull;

// BF16X3 operand tiles of the residual operator R = K - E (E copies the state
// features of the basis into x'): 64 feature rows x 16 output columns, stored
// per 32-row k-block in the lane order of a 16x16x32 MFMA B operand, hi and lo
// splits side by side.
constexpr int kRTileWords = 2 /*k-blocks*/ * 64 /*lanes*/ * 4 /*u32 = 8 bf16*/;

// Proposal network shape (fixed).
constexpr int kMlpIn = 8, kMlpHid = 256, kMlpComp = 16, kMlpOut = 5 * kMlpComp;
constexpr int kMlpParams = kMlpIn * kMlpHid + kMlpHid + 2 * (kMlpHid * kMlpHid + kMlpHid) + kMlpHid * kMlpOut + kMlpOut;
constexpr float kLogSigMin = -7.0f, kLogSigMax = 2.0f;
constexpr float kLog2Pi = 1.8378770664093453f;

// FP32 -> BF16 bits, round to nearest even (NaN stays NaN).
__host__ __device__ inline uint32_t bf16_bits_rne_u(float f) {
  uint32_t b;
  __builtin_memcpy(&b, &f, 4);
  if ((b & 0x7fffffffu) > 0x7f800000u) return 0x7fc0u;
  return (b + 0x7fffu + ((b >> 16) & 1u)) >> 16;
}

// Constraint constants read at every prediction step (Sec. IV-B checks with
// the Sec. V-C-1 inflation), contiguous so that a step fetches them with two
// scalar loads.  Track coefficients above the model's highest harmonic are 0.
struct SafetyConsts {
  float comp_lim[MPMI_MAX_STATE];    // per state component: least box_bound - box_infl over its boxes
  int32_t comp_mask;                 // bit k set if component k has a box
  float bb_lim[MPMI_MAX_BOX];        // box_bound - box_infl
  int32_t box_index[MPMI_MAX_BOX];   // state component of each box constraint
  int32_t n_box;
  int32_t has_track;
  int32_t hmax;                      // highest track harmonic (degree of P)
  float trk_lim;                     // track_half - track_infl
  float trk_p[kMaxHarm + 1];         // r_c = P(cos phi) + sin phi * Q(cos phi): P coefficients
  float trk_q[kMaxHarm];             // Q coefficients (monomial, ascending powers)
  // FP32 rounding bands (MPMI_PREC_FP32_RECHECK64): a state whose margin to a
  // constraint is within its band of zero sends the candidate to the FP64
  // re-roll.  Per component: the band of the binding (least-limit) box.
  float comp_eps[MPMI_MAX_STATE];
  float trk_eps;
};

// What the FP64 re-roll reads (MPMI_PREC_FP32_RECHECK64): K (and the race
// car's step rows in step order) and the safety set in FP64, and the basis as
// atoms and features (filled for the fixed families too, from their
// descriptions).  Limits are (double)bound - (double)inflation; the track's
// centreline radius is the FP32 tick's Chebyshev form P(cos phi) +
// sin phi Q(cos phi) with the FP64 coefficients.
struct Model64 {
  double K[MPMI_MAX_DIM][8];        // row = feature, col = state component
  double comp_lim[MPMI_MAX_STATE];  // least limit over the boxes on a component; +inf if none
  double trk_lim;
  double trk_p[kMaxHarm + 1];       // r_c = P(cos phi) + sin phi * Q(cos phi), FP64 monomial coefficients
  double trk_q[kMaxHarm];
  double sigma[MPMI_MAX_STATE];     // process-noise deviations
  double Kstep[27][8];              // race car: the rows of K the step reads, in its order (rc_step_row)
  int32_t has_track, comp_mask, n_atoms, pad;
  int8_t atom_kind[MPMI_MAX_ATOMS];
  int8_t atom_var[MPMI_MAX_ATOMS];
  int8_t feat_a[MPMI_MAX_DIM];
  int8_t feat_b[MPMI_MAX_DIM];
};

// Packed model: everything a rollout reads, in one device blob.
struct alignas(256) ModelDev {
  mpmi_system sys;
  uint32_t magic;
  int32_t dim;          // D
  int32_t n;            // state size
  int32_t m;            // input size
  int32_t state_feat0;  // index of feature w_0 = x_0 in psi (E's first row)
  int32_t has_noise;    // any noise_sigma > 0
  int32_t pad0;
  int32_t pad1;
  alignas(64) SafetyConsts safe;
  float half_inv[MPMI_MAX_INPUT]; // 2 / (u_hi - u_lo)
  float K[MPMI_MAX_DIM][8];       // FP32 K, row = feature, col = state component
  float Kstep[kStepWords];        // race car: the rows of K the step reads, in its order
  uint32_t Rhi[kRTileWords];      // BF16 hi split of R, MFMA B-operand order
  uint32_t Rlo[kRTileWords];      // BF16 lo split of R
  alignas(256) Model64 m64;       // the FP64 re-roll's copy
};

// Per-loop selection slot (context-owned device memory).  The memory-side
// atomic unit performs atomics on one address one after another, so the
// workgroups ("parts") of a launch publish into kSubSlots sub-slots, part p
// into sub-slot p % kSubSlots: keys by 64-bit atomicMin, and the safe count
// (with, for launches of many parts, a per-sub-slot ticket in its high half)
// by one 64-bit atomicAdd.  Tickets on the slot find the part that completes
// it; that part decodes the keys of all sub-slots, writes the mpmi_selection
// and restores the reset state (keys all-ones, counters zero).
constexpr int kSubSlots = 8;
struct alignas(64) SubSlot {
  unsigned long long key_safe;    // (cost bits << 32) | idx  over safe candidates
  unsigned long long key_fb;      // ((255 - fv) << 56) | (cost bits << 25) | idx
  unsigned long long count;       // low 32 bits: safe count; high 32: parts published
  unsigned int n_recheck;
  unsigned int pad0;
  unsigned long long key_safe64;  // safe keys of the FP64 re-roll (kept apart from key_safe,
                                  // whose least value the re-roll compares against)
  unsigned int pad[6];
};
struct alignas(64) Slot {
  SubSlot sub[kSubSlots];
  unsigned int done;  // sub-slots whose parts have all published
  unsigned int pad[15];
};
static_assert(sizeof(SubSlot) == 64 && sizeof(Slot) == 64 * (kSubSlots + 1), "slot layout");
constexpr unsigned long long kKeyNone = ~0ull;

// ---------------------------------------------------------------------------
// Counter-based generator (SplitMix64 output function, Steele et al. 2014)
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Chain over (seed, tick, loop, idx); hash_counter finishes it with the slot.
__device__ __forceinline__ uint64_t hash_prefix(uint64_t seed, uint64_t tick, uint64_t loop, uint64_t idx) {
  uint64_t h = seed;
  h = mix64((h ^ tick) + kGoldenGamma);
  h = mix64((h ^ loop) + kGoldenGamma);
  h = mix64((h ^ idx) + kGoldenGamma);
  return h;
}

__device__ __forceinline__ uint64_t hash_finish(uint64_t prefix, uint64_t slot) {
  return mix64((prefix ^ slot) + kGoldenGamma);
}

__device__ __forceinline__ uint64_t hash_counter(uint64_t seed, uint64_t tick, uint64_t loop,
                                                 uint64_t idx, uint64_t slot) {
  return hash_finish(hash_prefix(seed, tick, loop, idx), slot);
}

constexpr uint64_t kNoiseSlot = 65536;

// Process noise after step s (Alg. 2's z_i): pairs of components from one
// 64-bit draw, Box-Muller in FP32.
template <int NS>
__device__ __forceinline__ void add_process_noise(const float* sigma, uint64_t prefix, int s, int n, float* x) {
#pragma unroll
  for (int q = 0; q < (NS + 1) / 2; ++q) {
    if (2 * q < n) {
      const uint64_t h = hash_finish(prefix, kNoiseSlot + 4ull * (uint64_t)(s - 1) + (uint64_t)q);
      const float u1 = (float)((h >> 40) + 1ull) * 0x1p-24f;
      const float u2 = (float)((h >> 16) & 0xFFFFFFull) * 0x1p-24f;
      const float r = sqrtf(-2.0f * logf(u1));
      float sn, cs;
      sincosf(6.283185307179586f * u2, &sn, &cs);
      x[2 * q] = fmaf(sigma[2 * q], r * cs, x[2 * q]);
      if (2 * q + 1 < n) x[2 * q + 1] = fmaf(sigma[2 * q + 1], r * sn, x[2 * q + 1]);
    }
  }
}

// Value of a UNIFORM candidate input: lo + (hi - lo) * r in FP64, r = top 24
// bits / 2^24, rounded to FP32.  (hi - lo) and its product with r are exact
// in FP64, so the only rounding is the final sum and the cast.
__device__ __forceinline__ float uniform_value(float lo, float hi, uint64_t h) {
  const double r = (double)(h >> 40) * 0x1p-24;
  const double d = (double)hi - (double)lo;
  return (float)((double)lo + d * r);
}

// Value of a GRID candidate input: lo + (k + 1/2) * ((hi - lo) / G) in FP64,
// evaluated in exactly that order without fused multiply-add, rounded to FP32.
__device__ __forceinline__ float grid_value(float lo, float hi, int k, int G) {
#pragma clang fp contract(off)
  const double step = ((double)hi - (double)lo) / (double)G;
  const double t = ((double)k + 0.5) * step;
  return (float)((double)lo + t);
}

// Input j of segment g of candidate c (c >= 1) for a generated tick.
struct GenParams {
  uint64_t seed, tick;
  int32_t loop, gen, n_cand, n_seg;
  int32_t grid[MPMI_MAX_INPUT];
};

__device__ __forceinline__ float gen_value(const GenParams& gp, const ModelDev* __restrict__ md,
                                           const float* __restrict__ cand, int c, int g, int j) {
  const float lo = md->sys.u_lo[j], hi = md->sys.u_hi[j];
  if (gp.gen == MPMI_GEN_GRID) {
    int k = c - 1;
    for (int q = 0; q < j; ++q) k /= gp.grid[q];
    return grid_value(lo, hi, k % gp.grid[j], gp.grid[j]);
  }
  if (gp.gen == MPMI_GEN_UNIFORM) {
    return uniform_value(lo, hi, hash_counter(gp.seed, gp.tick, (uint64_t)(uint32_t)gp.loop,
                                              (uint64_t)c, (uint64_t)(g * md->m + j)));
  }
  return cand[(size_t)(g * md->m + j) * (size_t)gp.n_cand + (size_t)(c - 1)];
}

// ---------------------------------------------------------------------------
// Koopman step x' = psi(x, u)^T K (Sec. IV-A), FP32.
//
// K is staged once per workgroup in LDS and read inside every step with
// 16-byte broadcast loads; an opaque zero offset added to the LDS base at
// every step keeps the compiler from hoisting those loads out of the horizon
// loop (hoisted, the race-car coefficients overflow the scalar register file).
//
// The input is constant within a segment, so every feature that involves the
// input (input-only terms and state x input products) is folded once per
// segment into per-lane coefficients: a constant c_u, a linear map L on the
// state and, for the race car, the coefficients of sin/cos of the heading.
// A step then evaluates only the features made of state alone.  This is an
// exact regrouping of psi^T K in real arithmetic.
// ---------------------------------------------------------------------------
template <int BASIS>
struct Dims;
template <>
struct Dims<MPMI_BASIS_LINEAR> { static constexpr int N = MPMI_MAX_STATE, M = MPMI_MAX_INPUT; };
template <>
struct Dims<MPMI_BASIS_BALANCE_BOT> { static constexpr int N = 4, M = 1; };
template <>
struct Dims<MPMI_BASIS_RACE_CAR> { static constexpr int N = 6, M = 2; };
template <>
struct Dims<MPMI_BASIS_CUSTOM> { static constexpr int N = MPMI_MAX_STATE, M = MPMI_MAX_INPUT; };


// Index of the quadratic feature w_k w_l (k <= l) in a basis [1, w_0..w_{nw-1}, w_k w_l ...].
__host__ __device__ constexpr int quad_index(int k, int l, int nw) {
  return 1 + nw + (k * nw - (k * (k - 1)) / 2) + (l - k);
}

// LDS layout of the staged K (float offsets):
//   LINEAR       rows padded to 8 floats                           [0, 8 D)
//   BALANCE_BOT  all 21 rows, 4 floats each                        [0, 84)
//                the 10 state-state quadratic rows (k <= l < 4)    [84, 124)
//   RACE_CAR     all 64 rows, 6 floats each                        [0, 384)
//                the 21 state-state quadratic rows (k <= l < 6), then
//                sp*vx, sp*vy, sp*r, cp*vx, cp*vy, cp*r, 6 floats each  [384, 546)
constexpr int kBbStepOff = 84;
constexpr int kRcStepOff = 384;
constexpr int kRcStepRows = 27;
static_assert(sizeof(Model64::Kstep) == sizeof(double) * 8 * kRcStepRows, "FP64 step table");
constexpr int kLdsKFloat4 = 137;  // 546 floats rounded up to float4

// Row of K feeding row q of the race-car step table: the 21 state-state
// quadratic features (k <= l < 6), then sp*vx, sp*vy, sp*r, cp*vx, cp*vy, cp*r.
__host__ __device__ inline int rc_step_row(int q) {
  if (q < 21) {
    int k = 0, r = q;
    while (r >= 6 - k) { r -= 6 - k; ++k; }
    return quad_index(k, k + r, 8);
  }
  const int trig_rows[6] = {49, 50, 51, 53, 54, 55};
  return trig_rows[q - 21];
}

template <int BASIS>
__device__ __forceinline__ void stage_K(const ModelDev* __restrict__ md, float4* sK) {
  float* f = reinterpret_cast<float*>(sK);
  const int t = threadIdx.x, nt = blockDim.x;
  if constexpr (BASIS == MPMI_BASIS_LINEAR || BASIS == MPMI_BASIS_CUSTOM) {
    for (int e = t; e < md->dim * 8; e += nt) f[e] = md->K[e >> 3][e & 7];
  } else if constexpr (BASIS == MPMI_BASIS_BALANCE_BOT) {
    for (int e = t; e < 21 * 4; e += nt) f[e] = md->K[e >> 2][e & 3];
    for (int e = t; e < 10 * 4; e += nt) {
      const int q = e >> 2, j = e & 3;
      int k = 0, r = q;
      while (r >= 4 - k) { r -= 4 - k; ++k; }
      f[kBbStepOff + e] = md->K[quad_index(k, k + r, 5)][j];
    }
  } else {
    for (int e = t; e < 64 * 6; e += nt) f[e] = md->K[e / 6][e % 6];
    for (int e = t; e < kRcStepRows * 6; e += nt) f[kRcStepOff + e] = md->Kstep[e];
  }
  __syncthreads();
}

// Read-only model data seen through the constant address space, so uniform
// loads from it become scalar loads whose results feed VALU operands directly.
typedef const __attribute__((address_space(4))) float ConstF;
typedef const __attribute__((address_space(4))) SafetyConsts ConstSafety;

__device__ __forceinline__ const float4* opaque_lds(const float4* sK) {
  int off = 0;
  asm volatile("" : "+s"(off));
  return sK + off;
}

// Marks every component of the new state as computed at this point (no
// instruction is emitted).  Without it the compiler may sink the step's
// per-component contractions into the branches of the safety check that use
// them, holding all the step coefficients live across those branches.
template <int NS>
__device__ __forceinline__ void settle_state(float* x) {
#pragma unroll
  for (int j = 0; j < NS; ++j) asm volatile("" : "+v"(x[j]));
}

template <int BASIS>
struct Stepper;

// psi = w = [x; u] with run-time n, m (identity basis; used for checks).
template <>
struct Stepper<MPMI_BASIS_LINEAR> {
  float u[MPMI_MAX_INPUT];
  __device__ __forceinline__ void set_input(const ModelDev* __restrict__, const float4*, const float* uin) {
#pragma unroll
    for (int j = 0; j < MPMI_MAX_INPUT; ++j) u[j] = uin[j];
  }
  __device__ __forceinline__ void step(const ModelDev* __restrict__ md, const float4* sK, float* x) {
    constexpr int NM = MPMI_MAX_STATE, MM = MPMI_MAX_INPUT;
    const int n = md->n, m = md->m;
    const float4* k = opaque_lds(sK);
    float y[NM];
#pragma unroll
    for (int j = 0; j < NM; ++j) y[j] = 0.0f;
#pragma unroll
    for (int f = 0; f < NM + MM; ++f) {
      const bool on = (f < NM) ? (f < n) : (f - NM < m);
      if (on) {
        const int row = (f < NM) ? f : n + (f - NM);
        const float w = (f < NM) ? x[f] : u[f - NM];
        const float4 a = k[2 * row], b = k[2 * row + 1];
        y[0] = fmaf(w, a.x, y[0]); y[1] = fmaf(w, a.y, y[1]); y[2] = fmaf(w, a.z, y[2]); y[3] = fmaf(w, a.w, y[3]);
        y[4] = fmaf(w, b.x, y[4]); y[5] = fmaf(w, b.y, y[5]); y[6] = fmaf(w, b.z, y[6]); y[7] = fmaf(w, b.w, y[7]);
      }
    }
#pragma unroll
    for (int j = 0; j < NM; ++j) x[j] = (j < n) ? y[j] : 0.0f;
  }
};

// A basis given as data (MPMI_BASIS_CUSTOM): per step, w = [x; u] and the
// atoms go to this lane's column of two LDS tables (atom-major, so a wave's
// accesses hit 64 consecutive words), then every feature is the product of
// two atoms read back at wave-uniform rows, contracted with its K row (LDS
// broadcast).  The descriptor is read by scalar loads.  Sine and cosine are
// the hardware ones, as in the race-car step.
template <>
struct Stepper<MPMI_BASIS_CUSTOM> {
  float u[MPMI_MAX_INPUT];
  __device__ __forceinline__ void set_input(const ModelDev* __restrict__, const float4*, const float* uin) {
#pragma unroll
    for (int j = 0; j < MPMI_MAX_INPUT; ++j) u[j] = uin[j];
  }
  __device__ __forceinline__ void step(const ModelDev* __restrict__ md, const float4* sK, float* x) {
    __shared__ float sW[MPMI_MAX_STATE + MPMI_MAX_INPUT][kCustomBlock];
    __shared__ float sAt[MPMI_MAX_ATOMS][kCustomBlock];
    const int t = threadIdx.x;
    const int n = md->n, m = md->m;
#pragma unroll
    for (int j = 0; j < MPMI_MAX_STATE; ++j) sW[j][t] = x[j];
#pragma unroll
    for (int j = 0; j < MPMI_MAX_INPUT; ++j) sW[MPMI_MAX_STATE + j][t] = u[j];
    const int na = md->sys.n_atoms;
    for (int q = 0; q < na; ++q) {
      const int kd = md->sys.atom_kind[q], v = md->sys.atom_var[q];
      const float w = sW[v < n ? v : MPMI_MAX_STATE + (v - n)][t];
      float a = 1.0f;
      if (kd == MPMI_ATOM_VAR) a = w;
      else if (kd == MPMI_ATOM_SIN) a = __sinf(w);
      else if (kd == MPMI_ATOM_COS) a = __cosf(w);
      sAt[q][t] = a;
    }
    (void)m;
    const float4* k = opaque_lds(sK);
    float y[MPMI_MAX_STATE];
#pragma unroll
    for (int j = 0; j < MPMI_MAX_STATE; ++j) y[j] = 0.0f;
    const int D = md->dim;
    for (int f = 0; f < D; ++f) {
      const float p = sAt[md->sys.feat_a[f]][t] * sAt[md->sys.feat_b[f]][t];
      const float4 a = k[2 * f], b = k[2 * f + 1];
      y[0] = fmaf(p, a.x, y[0]); y[1] = fmaf(p, a.y, y[1]); y[2] = fmaf(p, a.z, y[2]); y[3] = fmaf(p, a.w, y[3]);
      y[4] = fmaf(p, b.x, y[4]); y[5] = fmaf(p, b.y, y[5]); y[6] = fmaf(p, b.z, y[6]); y[7] = fmaf(p, b.w, y[7]);
    }
#pragma unroll
    for (int j = 0; j < MPMI_MAX_STATE; ++j) x[j] = (j < n) ? y[j] : 0.0f;
  }
};

// Balance bot: [1, w_0..w_4, w_k w_l (k <= l)], w = [p, pd, th, thd, u].
template <>
struct Stepper<MPMI_BASIS_BALANCE_BOT> {
  float cu[4];     // 1, u, u^2 terms
  float L[4][4];   // x_k and x_k u terms
  __device__ __forceinline__ void set_input(const ModelDev* __restrict__, const float4* sK, const float* uin) {
    const float* K = reinterpret_cast<const float*>(sK);
    const float u = uin[0];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      cu[j] = fmaf(u * u, K[quad_index(4, 4, 5) * 4 + j], fmaf(u, K[5 * 4 + j], K[j]));
#pragma unroll
      for (int k = 0; k < 4; ++k) L[k][j] = fmaf(u, K[quad_index(k, 4, 5) * 4 + j], K[(1 + k) * 4 + j]);
    }
  }
  // Nested form of the linear + quadratic part:
  //   y_j = c_j + sum_k x_k (L_kj + sum_{l >= k} Q_klj x_l),
  // the same polynomial as the plain feature sum with no feature products;
  // each coefficient row (one LDS broadcast read) feeds all four outputs.
  __device__ __forceinline__ void step(const ModelDev* __restrict__, const float4* sK, float* x) {
    const float4* kk = opaque_lds(sK) + kBbStepOff / 4;
    float y[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) y[j] = cu[j];
    int q = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      float t[4] = {L[k][0], L[k][1], L[k][2], L[k][3]};
#pragma unroll
      for (int l = k; l < 4; ++l, ++q) {
        const float4 a = kk[q];
        t[0] = fmaf(a.x, x[l], t[0]); t[1] = fmaf(a.y, x[l], t[1]);
        t[2] = fmaf(a.z, x[l], t[2]); t[3] = fmaf(a.w, x[l], t[3]);
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) y[j] = fmaf(x[k], t[j], y[j]);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) x[j] = y[j];
  }
};

// Race car: w = [x, y, psi, vx, vy, r, delta, a].
template <>
struct Stepper<MPMI_BASIS_RACE_CAR> {
  float cu[6];     // 1, delta, a, delta^2, delta a, a^2, sin/cos delta, a sin delta terms
  float L[6][6];   // x_k, x_k delta, x_k a, and sin/cos delta * (vx, vy, r) terms
  float Ts[6];     // sin psi and a sin psi terms
  float Tc[6];     // cos psi and a cos psi terms
  __device__ __forceinline__ void set_input(const ModelDev* __restrict__, const float4* sK, const float* uin) {
    const float* K = reinterpret_cast<const float*>(sK);
    const float d = uin[0], a = uin[1];
    float sd, cd;
    sincosf(d, &sd, &cd);
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      float c = K[j];
      c = fmaf(d, K[7 * 6 + j], c);
      c = fmaf(a, K[8 * 6 + j], c);
      c = fmaf(d * d, K[quad_index(6, 6, 8) * 6 + j], c);
      c = fmaf(d * a, K[quad_index(6, 7, 8) * 6 + j], c);
      c = fmaf(a * a, K[quad_index(7, 7, 8) * 6 + j], c);
      c = fmaf(sd, K[47 * 6 + j], c);
      c = fmaf(cd, K[48 * 6 + j], c);
      c = fmaf(a * sd, K[63 * 6 + j], c);
      cu[j] = c;
#pragma unroll
      for (int k = 0; k < 6; ++k)
        L[k][j] = fmaf(a, K[quad_index(k, 7, 8) * 6 + j], fmaf(d, K[quad_index(k, 6, 8) * 6 + j], K[(1 + k) * 6 + j]));
      L[3][j] = fmaf(cd, K[60 * 6 + j], fmaf(sd, K[57 * 6 + j], L[3][j]));
      L[4][j] = fmaf(cd, K[61 * 6 + j], fmaf(sd, K[58 * 6 + j], L[4][j]));
      L[5][j] = fmaf(cd, K[62 * 6 + j], fmaf(sd, K[59 * 6 + j], L[5][j]));
      Ts[j] = fmaf(a, K[52 * 6 + j], K[45 * 6 + j]);
      Tc[j] = fmaf(a, K[56 * 6 + j], K[46 * 6 + j]);
    }
  }
  __device__ __forceinline__ void step(const ModelDev* __restrict__, const float4* sK, float* x) {
    // Hardware sine/cosine (argument scaled to revolutions): about 1e-6
    // absolute error for headings within a few hundred turns, well inside
    // the FP32 rollout tolerance, at a tenth of the instructions of sincosf.
    const float sp = __sinf(x[2]), cp = __cosf(x[2]);
    float p[kRcStepRows + 1];
    int q = 0;
#pragma unroll
    for (int k = 0; k < 6; ++k)
#pragma unroll
      for (int l = k; l < 6; ++l) p[q++] = x[k] * x[l];
    p[21] = sp * x[3]; p[22] = sp * x[4]; p[23] = sp * x[5];
    p[24] = cp * x[3]; p[25] = cp * x[4]; p[26] = cp * x[5];
    p[27] = 0.0f;
    float y[6];
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      float v = fmaf(Tc[j], cp, fmaf(Ts[j], sp, cu[j]));
#pragma unroll
      for (int k = 0; k < 6; ++k) v = fmaf(L[k][j], x[k], v);
      y[j] = v;
    }
    const float4* kk = opaque_lds(sK) + kRcStepOff / 4;
#pragma unroll
    for (int r = 0; r < 13; ++r) {
      const float4 a = kk[3 * r], b = kk[3 * r + 1], c = kk[3 * r + 2];
      const float p0 = p[2 * r], p1 = p[2 * r + 1];
      y[0] = fmaf(p0, a.x, y[0]); y[1] = fmaf(p0, a.y, y[1]); y[2] = fmaf(p0, a.z, y[2]);
      y[3] = fmaf(p0, a.w, y[3]); y[4] = fmaf(p0, b.x, y[4]); y[5] = fmaf(p0, b.y, y[5]);
      y[0] = fmaf(p1, b.z, y[0]); y[1] = fmaf(p1, b.w, y[1]); y[2] = fmaf(p1, c.x, y[2]);
      y[3] = fmaf(p1, c.y, y[3]); y[4] = fmaf(p1, c.z, y[4]); y[5] = fmaf(p1, c.w, y[5]);
    }
    const float4 a = kk[39];
    const float2 b = *reinterpret_cast<const float2*>(kk + 40);
    const float p0 = p[26];
    y[0] = fmaf(p0, a.x, y[0]); y[1] = fmaf(p0, a.y, y[1]); y[2] = fmaf(p0, a.z, y[2]);
    y[3] = fmaf(p0, a.w, y[3]); y[4] = fmaf(p0, b.x, y[4]); y[5] = fmaf(p0, b.y, y[5]);
#pragma unroll
    for (int j = 0; j < 6; ++j) x[j] = y[j];
  }
};

// a * b + c, one rounding, as the three-address v_fma_f64.  For an addend
// that stays live (a polynomial coefficient held across a loop) the compiler
// picks the two-address form, whose destination is the addend, and copies
// the coefficient into a fresh register before every use; this form needs
// no copy.  CS: the addend is wave-uniform and lives in scalar registers.
__device__ __forceinline__ double fma3(double a, double b, double c) {
  double d;
  asm("v_fma_f64 %0, %1, %2, %3" : "=v"(d) : "v"(a), "v"(b), "v"(c));
  return d;
}
__device__ __forceinline__ double fma3s(double a, double b, double c) {
  double d;
  asm("v_fma_f64 %0, %1, %2, %3" : "=v"(d) : "v"(a), "v"(b), "s"(c));
  return d;
}

// ---------------------------------------------------------------------------
// sin and cos of a double, for the FP64 re-roll's heading.
//
// Cody and Waite's reduction by pi/2 in two FMA steps: k = rint(x 2/pi) and
// r = (x - k P1) - k P2, with P1 the double nearest pi/2 and P2 the double
// nearest pi/2 - P1 (each step one rounding; the part of pi/2 below P2 adds
// at most |k| 2^-107).  On |r| <= pi/4 (+ rounding) the Taylor series of
// sin through r^17 and of cos through r^16, in z = r^2 (the first omitted
// terms, r^19/19! and r^18/18!, are below 2^-62 and 2^-57 of the result),
// then the quadrant k mod 4 swaps and negates.  About an ulp from the
// correctly rounded values; |x| >= 2^20 (and NaN, +-inf) take the library's
// sincos, whose reduction holds for any argument.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void sincos_rr64(double x, double* sn, double* cs) {
  if (!(fabs(x) < 0x1p20)) {
    sincos(x, sn, cs);
    return;
  }
  constexpr double kTwoOverPi = 0x1.45f306dc9c883p-1;
  constexpr double kP1 = 0x1.921fb54442d18p+0;
  constexpr double kP2 = 0x1.1a62633145c07p-54;
  const double k = rint(x * kTwoOverPi);
  const double r = fma(-k, kP2, fma(-k, kP1, x));
  const double z = r * r;
  // (-1)^n / (2n + 1)!, n = 8 .. 1, and (-1)^n / (2n)!, n = 8 .. 2
  double ps = fma3(1.0 / 355687428096000.0, z, -1.0 / 1307674368000.0);
  ps = fma3(ps, z, 1.0 / 6227020800.0);
  ps = fma3(ps, z, -1.0 / 39916800.0);
  ps = fma3(ps, z, 1.0 / 362880.0);
  ps = fma3(ps, z, -1.0 / 5040.0);
  ps = fma3(ps, z, 1.0 / 120.0);
  ps = fma3(ps, z, -1.0 / 6.0);
  double pc = fma3(1.0 / 20922789888000.0, z, -1.0 / 87178291200.0);
  pc = fma3(pc, z, 1.0 / 479001600.0);
  pc = fma3(pc, z, -1.0 / 3628800.0);
  pc = fma3(pc, z, 1.0 / 40320.0);
  pc = fma3(pc, z, -1.0 / 720.0);
  pc = fma3(pc, z, 1.0 / 24.0);
  const double s = fma(r * z, ps, r);                   // r + r z (-1/6 + ...)
  const double c = fma(z * z, pc, fma(-0.5, z, 1.0));   // 1 - z/2 + z^2 (1/24 + ...)
  const int q = (int)k;  // |k| < 2^20
  const bool swap = (q & 1) != 0;
  const double sv = swap ? c : s, cv = swap ? s : c;
  *sn = (q & 2) ? -sv : sv;
  *cs = ((q + 1) & 2) ? -cv : cv;
}

// ---------------------------------------------------------------------------
// Safety margins (Sec. IV-B geometric checks, Sec. V-C-1 inflation)
// ---------------------------------------------------------------------------
template <int NS>
__device__ __forceinline__ float pick(const float* x, int idx) {
  float v = x[0];
#pragma unroll
  for (int k = 1; k < NS; ++k) v = (idx == k) ? x[k] : v;
  return v;
}

// Centreline radius r_c(phi) at the polar angle of (x[0], x[1]), and rho.
// sin(h phi + p) expands into Chebyshev polynomials of cos phi (T_h, and
// sin phi * U_{h-1}), so r_c = P(cos phi) + sin phi * Q(cos phi) with
// coefficients formed once per model in FP64; cos phi and sin phi come from
// one reciprocal square root (rho = 0 or an infinite coordinate gives NaN,
// i.e. unsafe; the centreline radius exceeds the half-width there anyway).
// Horner runs over a fixed DEG (>= the model's highest harmonic, chosen on
// the host): the zero coefficients above the model's degree leave every
// partial sum exactly as it is, and the fixed trip count lets all the
// coefficients arrive in one scalar-load batch.
constexpr int kSmallTrackDeg = 5;  // the paper's track: harmonics 2..5
template <int DEG = kMaxHarm, class SC>
__device__ __forceinline__ float track_centre(const SC* sc, const float* x, float* rho) {
  static_assert(DEG >= 1 && DEG <= kMaxHarm, "track degree");
  const float r2 = fmaf(x[0], x[0], x[1] * x[1]);
  const float inv = __builtin_amdgcn_rsqf(r2);
  *rho = r2 * inv;
  const float c1 = x[0] * inv, s1 = x[1] * inv;
  float P = sc->trk_p[DEG];
#pragma unroll
  for (int k = DEG - 1; k >= 0; --k) P = fmaf(P, c1, sc->trk_p[k]);
  float Q = sc->trk_q[DEG - 1];
#pragma unroll
  for (int k = DEG - 2; k >= 0; --k) Q = fmaf(Q, c1, sc->trk_q[k]);
  return fmaf(s1, Q, P);
}

// The model's constraint constants as scalar-load operands, re-fetched at
// each call (not held in registers across the horizon).
__device__ __forceinline__ const ConstSafety* safety_of(const ModelDev* __restrict__ md) {
  int off = 0;
  asm volatile("" : "+s"(off));
  return (const ConstSafety*)(uintptr_t)&md->safe + off;
}

// Least margin over all constraints of state x (NaN if any margin is NaN, so
// that "safe" = (margin > 0) rejects NaN states).
// Boxes are taken per state component (wave-uniform branches on the mask,
// compile-time register indices): several boxes on one component reduce to
// the least limit, which gives the same least margin.
template <int NS, int DEG = kMaxHarm>
__device__ __forceinline__ float min_margin(const ModelDev* __restrict__ md, const float* x);

// The same over constants the caller holds (SC: SafetyConsts in registers, or
// the model's constant-space copy).
template <int NS, int DEG = kMaxHarm, class SC>
__device__ __forceinline__ float min_margin_of(const SC* sc, const float* x) {
  float mm = INFINITY;
  bool nan = false;
  const int mask = sc->comp_mask;
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    if (mask & (1 << k)) {
      const float mg = sc->comp_lim[k] - fabsf(x[k]);
      nan |= (mg != mg);
      mm = fminf(mm, mg);
    }
  }
  if (sc->has_track) {
    float rho;
    const float rc = track_centre<DEG>(sc, x, &rho);
    const float mg = sc->trk_lim - fabsf(rho - rc);
    nan |= (mg != mg);
    mm = fminf(mm, mg);
  }
  return nan ? NAN : mm;
}

template <int NS, int DEG>
__device__ __forceinline__ float min_margin(const ModelDev* __restrict__ md, const float* x) {
  return min_margin_of<NS, DEG>(safety_of(md), x);
}

// The verdict alone: min_margin(x) > 0, i.e. every margin positive.  A NaN
// margin fails its comparison, so no NaN bookkeeping and no minimum are
// needed; the tests combine bitwise (each a compare into a lane mask, no
// branch, no short circuit).  Used by the lifted tick; in the FP32 tick's
// step loop the least-margin form measured faster (0.405 against 0.447 ms
// on the 1M tick).
template <int NS, int DEG = kMaxHarm, class SC>
__device__ __forceinline__ bool all_safe_of(const SC* sc, const float* x) {
  bool ok = true;
  const int mask = sc->comp_mask;
#pragma unroll
  for (int k = 0; k < NS; ++k) ok &= !((mask >> k) & 1) | (sc->comp_lim[k] - fabsf(x[k]) > 0.0f);
  if (sc->has_track) {
    float rho;
    const float rc = track_centre<DEG>(sc, x, &rho);
    ok &= sc->trk_lim - fabsf(rho - rc) > 0.0f;
  }
  return ok;
}

// min_margin, also OR-ing into *near whether some constraint's margin lies
// within that constraint's FP32 band of zero (either side; a NaN margin is
// unsafe and not near).
template <int NS, int DEG = kMaxHarm>
__device__ __forceinline__ float min_margin_near(const ModelDev* __restrict__ md, const float* x, bool* near) {
  const ConstSafety* sc = safety_of(md);
  float mm = INFINITY;
  bool nan = false, nr = false;
  const int mask = sc->comp_mask;
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    if (mask & (1 << k)) {
      const float mg = sc->comp_lim[k] - fabsf(x[k]);
      nan |= (mg != mg);
      mm = fminf(mm, mg);
      nr |= fabsf(mg) < sc->comp_eps[k];
    }
  }
  if (sc->has_track) {
    float rho;
    const float rc = track_centre<DEG>(sc, x, &rho);
    const float mg = sc->trk_lim - fabsf(rho - rc);
    nan |= (mg != mg);
    mm = fminf(mm, mg);
    nr |= fabsf(mg) < sc->trk_eps;
  }
  *near |= nr;
  return nan ? NAN : mm;
}

// ---------------------------------------------------------------------------
// Selection keys
// ---------------------------------------------------------------------------
__device__ __forceinline__ unsigned long long safe_key(float cost, int idx) {
  return ((unsigned long long)__float_as_uint(cost) << 32) | (unsigned long long)(uint32_t)idx;
}
__device__ __forceinline__ unsigned long long fallback_key(int fv, float cost, int idx) {
  const unsigned long long cb = (unsigned long long)(__float_as_uint(cost) & 0x7fffffffu);
  return ((unsigned long long)(255 - fv) << 56) | (cb << 25) | (unsigned long long)(uint32_t)idx;
}

// One step of a DPP min-reduction: v against the value CTRL selects (rows
// and banks outside the masks, and sources outside the row, read all-ones,
// the identity of min).
template <int CTRL, int ROW_MASK, int BANK_MASK>
__device__ __forceinline__ unsigned long long dpp_min_u64(unsigned long long v) {
  const int lo = __builtin_amdgcn_update_dpp(-1, (int)(uint32_t)v, CTRL, ROW_MASK, BANK_MASK, false);
  const int hi = __builtin_amdgcn_update_dpp(-1, (int)(uint32_t)(v >> 32), CTRL, ROW_MASK, BANK_MASK, false);
  const unsigned long long o = ((unsigned long long)(uint32_t)hi << 32) | (uint32_t)lo;
  return o < v ? o : v;
}

// Minimum of v over the wave (every lane active), in every lane: within each
// row of 16, shifts by 1, 2, 4, 8 leave lane 15 with the row's minimum; the
// row broadcasts of lanes 15 and 31 carry it to lane 63, read back as a
// scalar.  No LDS round trip (a shuffle butterfly is six ds_bpermute waits).
__device__ __forceinline__ unsigned long long wave_min_u64(unsigned long long v) {
  v = dpp_min_u64<0x111, 0xF, 0xF>(v);  // row_shr:1
  v = dpp_min_u64<0x112, 0xF, 0xF>(v);  // row_shr:2
  v = dpp_min_u64<0x114, 0xF, 0xF>(v);  // row_shr:4
  v = dpp_min_u64<0x118, 0xF, 0xF>(v);  // row_shr:8
  v = dpp_min_u64<0x142, 0xA, 0xF>(v);  // row_bcast:15 into rows 1 and 3
  v = dpp_min_u64<0x143, 0xC, 0xF>(v);  // row_bcast:31 into rows 2 and 3
  const uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)v, 63);
  const uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), 63);
  return ((unsigned long long)hi << 32) | lo;
}

}  // namespace mpmi
