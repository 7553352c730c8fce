// Device-side building blocks of the MPMI-SC tick: packed model layout,
// basis evaluation + Koopman step, safety margins, counter-based candidate
// generation and the orderable selection keys.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/mpmi.h"

namespace mpmi {

constexpr uint32_t kModelMagic = 0x4d504d49u;  // "MPMI"
constexpr int kMaxHarm = 8;                     // highest track frequency
constexpr uint64_t kGoldenGamma = 0x9E3779B97F4A7C15ull;

// BF16X3 operand tiles of the residual operator R = K - E (E copies the state
// features of the basis into x'): 64 feature rows x 16 output columns, stored
// per 32-row k-block in the lane order of a 16x16x32 MFMA B operand, hi and lo
// splits side by side.
constexpr int kRTileWords = 2 /*k-blocks*/ * 64 /*lanes*/ * 4 /*u32 = 8 bf16*/;

// Packed model: everything a rollout reads, in one device blob.
struct alignas(256) ModelDev {
  mpmi_system sys;
  uint32_t magic;
  int32_t dim;          // D
  int32_t n;            // state size
  int32_t m;            // input size
  int32_t state_feat0;  // index of feature w_0 = x_0 in psi (E's first row)
  int32_t hmax;         // highest track harmonic used (0 = no track)
  int32_t pad0[2];
  float bb_lim[MPMI_MAX_BOX];     // box_bound - box_infl
  float trk_lim;                  // track_half - track_infl
  float trk_r0;                   // r0 plus the constant (frequency 0) terms
  float trk_s[kMaxHarm + 1];      // coefficient of sin(h phi)
  float trk_c[kMaxHarm + 1];      // coefficient of cos(h phi)
  float half_inv[MPMI_MAX_INPUT]; // 2 / (u_hi - u_lo)
  float K[MPMI_MAX_DIM][8];       // FP32 K, row = feature, col = state component
  uint32_t Rhi[kRTileWords];      // BF16 hi split of R, MFMA B-operand order
  uint32_t Rlo[kRTileWords];      // BF16 lo split of R
};

// Per-loop selection slot (context-owned device memory).  Keys are reduced
// with 64-bit atomicMin; the last workgroup of a launch decodes them, writes
// the mpmi_selection and restores the slot to its reset state.
struct Slot {
  unsigned long long key_safe;  // (cost bits << 32) | idx  over safe candidates
  unsigned long long key_fb;    // ((255 - fv) << 56) | (cost bits << 25) | idx
  unsigned int n_safe;
  unsigned int done;
  unsigned int n_recheck;
  unsigned int pad;
};
constexpr unsigned long long kKeyNone = ~0ull;

// ---------------------------------------------------------------------------
// Counter-based generator (SplitMix64 output function, Steele et al. 2014)
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__device__ __forceinline__ uint64_t hash_counter(uint64_t seed, uint64_t tick, uint64_t loop,
                                                 uint64_t idx, uint64_t slot) {
  uint64_t h = seed;
  h = mix64((h ^ tick) + kGoldenGamma);
  h = mix64((h ^ loop) + kGoldenGamma);
  h = mix64((h ^ idx) + kGoldenGamma);
  h = mix64((h ^ slot) + kGoldenGamma);
  return h;
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
// Koopman step x' = psi(x, u)^T K (Sec. IV-A), FP32, K read as uniform values.
// ---------------------------------------------------------------------------
template <int BASIS>
struct Dims;
template <>
struct Dims<MPMI_BASIS_LINEAR> { static constexpr int N = MPMI_MAX_STATE, M = MPMI_MAX_INPUT; };
template <>
struct Dims<MPMI_BASIS_BALANCE_BOT> { static constexpr int N = 4, M = 1; };
template <>
struct Dims<MPMI_BASIS_RACE_CAR> { static constexpr int N = 6, M = 2; };

template <int BASIS>
__device__ __forceinline__ void koopman_step(const ModelDev* __restrict__ md, float* x, const float* u);

// psi = w = [x; u] with run-time n, m.
template <>
__device__ __forceinline__ void koopman_step<MPMI_BASIS_LINEAR>(const ModelDev* __restrict__ md,
                                                                float* x, const float* u) {
  constexpr int NM = MPMI_MAX_STATE, MM = MPMI_MAX_INPUT;
  const int n = md->n, m = md->m;
  float y[NM];
#pragma unroll
  for (int j = 0; j < NM; ++j) y[j] = 0.0f;
#pragma unroll
  for (int f = 0; f < NM; ++f) {
    if (f < n) {
#pragma unroll
      for (int j = 0; j < NM; ++j) y[j] = fmaf(x[f], md->K[f][j], y[j]);
    }
  }
#pragma unroll
  for (int f = 0; f < MM; ++f) {
    if (f < m) {
#pragma unroll
      for (int j = 0; j < NM; ++j) y[j] = fmaf(u[f], md->K[n + f][j], y[j]);
    }
  }
#pragma unroll
  for (int j = 0; j < NM; ++j) x[j] = (j < n) ? y[j] : 0.0f;
}

// [1, w_0..w_4, w_k w_l (k <= l)], w = [p, pd, th, thd, u].
template <>
__device__ __forceinline__ void koopman_step<MPMI_BASIS_BALANCE_BOT>(const ModelDev* __restrict__ md,
                                                                     float* x, const float* u) {
  const float w[5] = {x[0], x[1], x[2], x[3], u[0]};
  float y[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) y[j] = md->K[0][j];
#pragma unroll
  for (int k = 0; k < 5; ++k) {
#pragma unroll
    for (int j = 0; j < 4; ++j) y[j] = fmaf(w[k], md->K[1 + k][j], y[j]);
  }
  int f = 6;
#pragma unroll
  for (int k = 0; k < 5; ++k) {
#pragma unroll
    for (int l = k; l < 5; ++l) {
      const float p = w[k] * w[l];
#pragma unroll
      for (int j = 0; j < 4; ++j) y[j] = fmaf(p, md->K[f][j], y[j]);
      ++f;
    }
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) x[j] = y[j];
}

// Race-car basis; sd, cd = sin/cos of the steering input (constant within a
// segment, so the caller evaluates them once per segment).
__device__ __forceinline__ void race_car_step(const ModelDev* __restrict__ md, float* x,
                                              const float* u, float sd, float cd) {
  const float w[8] = {x[0], x[1], x[2], x[3], x[4], x[5], u[0], u[1]};
  float sp, cp;
  sincosf(x[2], &sp, &cp);
  float y[6];
#pragma unroll
  for (int j = 0; j < 6; ++j) y[j] = md->K[0][j];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
#pragma unroll
    for (int j = 0; j < 6; ++j) y[j] = fmaf(w[k], md->K[1 + k][j], y[j]);
  }
  int f = 9;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
#pragma unroll
    for (int l = k; l < 8; ++l) {
      const float p = w[k] * w[l];
#pragma unroll
      for (int j = 0; j < 6; ++j) y[j] = fmaf(p, md->K[f][j], y[j]);
      ++f;
    }
  }
  const float vx = w[3], vy = w[4], r = w[5], a = w[7];
  const float extra[19] = {sp,      cp,      sd,      cd,      sp * vx, sp * vy, sp * r,
                           sp * a,  cp * vx, cp * vy, cp * r,  cp * a,  sd * vx, sd * vy,
                           sd * r,  cd * vx, cd * vy, cd * r,  a * sd};
#pragma unroll
  for (int e = 0; e < 19; ++e) {
#pragma unroll
    for (int j = 0; j < 6; ++j) y[j] = fmaf(extra[e], md->K[45 + e][j], y[j]);
  }
#pragma unroll
  for (int j = 0; j < 6; ++j) x[j] = y[j];
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

// Least margin over all constraints of state x (NaN if any margin is NaN, so
// that "safe" = (margin > 0) rejects NaN states).
template <int NS>
__device__ __forceinline__ float min_margin(const ModelDev* __restrict__ md, const float* x) {
  float mm = INFINITY;
  bool nan = false;
  const int nb = md->sys.n_box;
  for (int b = 0; b < nb; ++b) {
    const float mg = md->bb_lim[b] - fabsf(pick<NS>(x, md->sys.box_index[b]));
    nan |= (mg != mg);
    mm = fminf(mm, mg);
  }
  if (md->hmax >= 0 && md->sys.has_track) {
    const float rho = sqrtf(x[0] * x[0] + x[1] * x[1]);
    float c1 = 1.0f, s1 = 0.0f;
    if (rho > 0.0f) {
      const float inv = 1.0f / rho;
      c1 = x[0] * inv;
      s1 = x[1] * inv;
    }
    float rc = md->trk_r0;
    float ch = 1.0f, sh = 0.0f;
    const int hmax = md->hmax;
    for (int h = 1; h <= hmax; ++h) {
      const float cn = ch * c1 - sh * s1;
      const float sn = sh * c1 + ch * s1;
      ch = cn;
      sh = sn;
      rc = fmaf(md->trk_s[h], sh, rc);
      rc = fmaf(md->trk_c[h], ch, rc);
    }
    const float mg = md->trk_lim - fabsf(rho - rc);
    nan |= (mg != mg);
    mm = fminf(mm, mg);
  }
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

__device__ __forceinline__ unsigned long long wave_min_u64(unsigned long long v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const unsigned long long o = __shfl_xor(v, off, 64);
    v = o < v ? o : v;
  }
  return v;
}

}  // namespace mpmi
