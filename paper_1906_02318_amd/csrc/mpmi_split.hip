// Latency form of the fused tick: each candidate spread over SPLIT lanes.
//
// With few candidates per tick a wave's 60-step serial chain, not the chip's
// throughput, sets the tick time: a wave issues one instruction per four
// cycles, so the step's instruction count is its latency.  Here lane h of a
// group of SPLIT computes output columns [h J, h J + J) of every step
// (J = ceil(n / SPLIT)) from the full feature set, and the group rebuilds the
// full next state with cross-lane permutes, so each lane's contraction is
// J / n of the one-lane form, at the price of redundant feature and safety
// work.  The autotuner picks SPLIT (1, 2, 4 or 8) and the workgroup size per
// workload.
#include <hip/hip_runtime.h>

#include "mpmi_device.hpp"
#include "mpmi_launch.hpp"
#include "mpmi_tick_common.hpp"

namespace mpmi {

// LDS rows of 8 floats; column j of a row sits at (j / J) * A + (j % J), A = 4
// when J = 3 (so a lane's three columns are one aligned float4), else J.
template <int J>
struct SplitLayout {
  static constexpr int A = (J == 3) ? 4 : J;
  static __device__ __forceinline__ int pos(int j) { return (j / J) * A + (j % J); }
};

constexpr int kSplitRows = 64 + 27;  // full rows + per-step rows (race car is the larger)

// Row r of the table: K row r (r < D), or the per-step row r - D (the
// quadratic state features, then for the race car the heading terms).
template <int BASIS>
__device__ __forceinline__ int split_row(int r) {
  constexpr int D = (BASIS == MPMI_BASIS_RACE_CAR) ? 64 : 21;
  if (r < D) return r;
  const int q = r - D;
  if (BASIS == MPMI_BASIS_RACE_CAR) {
    if (q < 21) {
      int k = 0, t = q;
      while (t >= 6 - k) { t -= 6 - k; ++k; }
      return quad_index(k, k + t, 8);
    }
    constexpr int trig_rows[6] = {49, 50, 51, 53, 54, 55};
    return trig_rows[q - 21];
  }
  int k = 0, t = q;
  while (t >= 4 - k) { t -= 4 - k; ++k; }
  return quad_index(k, k + t, 5);
}

// One pass over the table: every entry is written once, with its K value or
// zero (positions no column maps to), so one barrier suffices; D and R are
// the basis' constants, so the loads start without a round trip.
template <int BASIS, int J>
__device__ __forceinline__ void stage_K_split(const ModelDev* __restrict__ md, float* sK8) {
  constexpr int NS = Dims<BASIS>::N;
  constexpr int D = (BASIS == MPMI_BASIS_RACE_CAR) ? 64 : 21;
  constexpr int R = (BASIS == MPMI_BASIS_RACE_CAR) ? kRcStepRows : 10;
  constexpr int A = SplitLayout<J>::A;
  for (int e = threadIdx.x; e < (D + R) * 8; e += blockDim.x) {
    const int r = e >> 3, p = e & 7;
    const int j = (p / A) * J + (p % A);  // the column at position p, if p % A < J
    float v = 0.0f;
    if (p % A < J && j < NS) v = md->K[split_row<BASIS>(r)][j];
    sK8[e] = v;
  }
  __syncthreads();
}

// Loads J consecutive floats at an aligned LDS position.
template <int J>
__device__ __forceinline__ void ldsJ(const float* p, float* out) {
  if constexpr (J == 3 || J == 4) {
    const float4 v = *reinterpret_cast<const float4*>(p);
    out[0] = v.x; out[1] = v.y; out[2] = v.z;
    if constexpr (J == 4) out[3] = v.w;
  } else if constexpr (J == 2) {
    const float2 v = *reinterpret_cast<const float2*>(p);
    out[0] = v.x; out[1] = v.y;
  } else {
    out[0] = p[0];
  }
}

// Folded per-lane coefficients for this lane's J columns (LDS position p0).
template <int BASIS, int J>
struct SplitFold {
  static constexpr int NS = Dims<BASIS>::N;
  float cu[J], L[NS][J], Ts[J], Tc[J];
  __device__ __forceinline__ void fold(const float* sK8, int p0, const float* uu) {
    float sd = 0.0f, cd = 1.0f;
    if (BASIS == MPMI_BASIS_RACE_CAR) sincosf(uu[0], &sd, &cd);
#pragma unroll
    for (int jj = 0; jj < J; ++jj) {
      const float* Kc = sK8 + p0 + jj;  // column jj of this lane: Kc[f * 8]
      if (BASIS == MPMI_BASIS_RACE_CAR) {
        const float d = uu[0], a = uu[1];
        float v = Kc[0];
        v = fmaf(d, Kc[7 * 8], v);
        v = fmaf(a, Kc[8 * 8], v);
        v = fmaf(d * d, Kc[quad_index(6, 6, 8) * 8], v);
        v = fmaf(d * a, Kc[quad_index(6, 7, 8) * 8], v);
        v = fmaf(a * a, Kc[quad_index(7, 7, 8) * 8], v);
        v = fmaf(sd, Kc[47 * 8], v);
        v = fmaf(cd, Kc[48 * 8], v);
        v = fmaf(a * sd, Kc[63 * 8], v);
        cu[jj] = v;
#pragma unroll
        for (int k = 0; k < 6; ++k)
          L[k][jj] = fmaf(a, Kc[quad_index(k, 7, 8) * 8], fmaf(d, Kc[quad_index(k, 6, 8) * 8], Kc[(1 + k) * 8]));
        L[3][jj] = fmaf(cd, Kc[60 * 8], fmaf(sd, Kc[57 * 8], L[3][jj]));
        L[4][jj] = fmaf(cd, Kc[61 * 8], fmaf(sd, Kc[58 * 8], L[4][jj]));
        L[5][jj] = fmaf(cd, Kc[62 * 8], fmaf(sd, Kc[59 * 8], L[5][jj]));
        Ts[jj] = fmaf(a, Kc[52 * 8], Kc[45 * 8]);
        Tc[jj] = fmaf(a, Kc[56 * 8], Kc[46 * 8]);
      } else {
        const float uv = uu[0];
        cu[jj] = fmaf(uv * uv, Kc[quad_index(4, 4, 5) * 8], fmaf(uv, Kc[5 * 8], Kc[0]));
#pragma unroll
        for (int k = 0; k < NS; ++k) L[k][jj] = fmaf(uv, Kc[quad_index(k, 4, 5) * 8], Kc[(1 + k) * 8]);
        Ts[jj] = Tc[jj] = 0.0f;
      }
    }
  }
};

// This lane's columns of the per-step rows (quadratic state features, and for
// the race car the six heading cross terms), held in registers for the whole
// horizon: at one or two waves per SIMD nothing hides LDS latency, and a wave
// of this kernel has the register file to itself.
template <int BASIS, int J>
struct SplitRows {
  static constexpr int NQ = (BASIS == MPMI_BASIS_RACE_CAR) ? 21 : 10;
  static constexpr int NT = (BASIS == MPMI_BASIS_RACE_CAR) ? 6 : 0;
  float q[NQ][J], t[NT > 0 ? NT : 1][J];
  __device__ __forceinline__ void load(const float* sK8, int D, int colpos) {
#pragma unroll
    for (int r = 0; r < NQ; ++r) ldsJ<J>(&sK8[(D + r) * 8 + colpos], q[r]);
#pragma unroll
    for (int r = 0; r < NT; ++r) ldsJ<J>(&sK8[(D + NQ + r) * 8 + colpos], t[r]);
  }
};

// The constraint constants in registers, loaded once per launch, and the
// safety verdict of a state.  safe(x) equals min_margin(x) > 0: every margin
// lim - |v| is positive and none is NaN exactly when |v| < lim holds for each
// (with denormals kept, the difference of two distinct finite floats is never
// rounded to zero, and a NaN fails either comparison).  The track's
// centreline radius takes track_centre's operations in its order.  TRACK is
// the model's has_track flag, fixed per kernel instance; the float constants
// are pinned to vector registers (the scalar file is too small to hold them
// beside the loop's own state).
template <int NS, int DEG, bool TRACK>
struct SafetyRegs {
  float lim[NS], p[DEG + 1], q[DEG], trk_lim;
  bool chk[NS];
  __device__ __forceinline__ void load(const ModelDev* __restrict__ md) {
    const ConstSafety* sc = (const ConstSafety*)(uintptr_t)&md->safe;
    const int mask = sc->comp_mask;
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      chk[k] = (mask >> k) & 1;
      lim[k] = sc->comp_lim[k];
      asm volatile("" : "+v"(lim[k]));
    }
    if constexpr (TRACK) {
      trk_lim = sc->trk_lim;
      asm volatile("" : "+v"(trk_lim));
#pragma unroll
      for (int k = 0; k <= DEG; ++k) {
        p[k] = sc->trk_p[k];
        asm volatile("" : "+v"(p[k]));
      }
#pragma unroll
      for (int k = 0; k < DEG; ++k) {
        q[k] = sc->trk_q[k];
        asm volatile("" : "+v"(q[k]));
      }
    }
  }
  // Bitwise, not short-circuit, combination: each test is one compare into a
  // lane mask, with no branch.
  __device__ __forceinline__ bool safe(const float* x) const {
    bool ok = true;
#pragma unroll
    for (int k = 0; k < NS; ++k) ok &= (fabsf(x[k]) < lim[k]) | !chk[k];
    if constexpr (TRACK) {
      const float r2 = fmaf(x[0], x[0], x[1] * x[1]);
      const float inv = __builtin_amdgcn_rsqf(r2);
      const float rho = r2 * inv;
      const float c1 = x[0] * inv, s1 = x[1] * inv;
      float P = p[DEG];
#pragma unroll
      for (int k = DEG - 1; k >= 0; --k) P = fmaf(P, c1, p[k]);
      float Q = q[DEG - 1];
#pragma unroll
      for (int k = DEG - 2; k >= 0; --k) Q = fmaf(Q, c1, q[k]);
      ok &= fabsf(rho - fmaf(s1, Q, P)) < trk_lim;
    }
    return ok;
  }
};

// Value of v in lane `SRC` of this lane's group, with DPP permutes (no LDS
// round trip).  Groups of 2 or 4 lanes sit inside one quad: one quad_perm.
// A group of 8 is two quads of one row half: a quad_perm broadcasts lane
// SRC % 4 of every quad, then the quad that does not hold SRC takes the value
// of the quad beside it (row_shr:4 into banks 1 and 3, or row_shl:4 into
// banks 0 and 2; the other banks keep the broadcast).
template <int SPLIT, int SRC>
__device__ __forceinline__ float group_lane(float v) {
  const int iv = __builtin_bit_cast(int, v);
  if constexpr (SPLIT == 8) {
    const int b = __builtin_amdgcn_mov_dpp(iv, (SRC & 3) * 0x55, 0xF, 0xF, true);
    constexpr int shift = SRC < 4 ? 0x114 : 0x104;      // row_shr:4 / row_shl:4
    constexpr int banks = SRC < 4 ? 0xA : 0x5;          // the quads that take the neighbour's value
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(b, b, shift, 0xF, banks, false));
  } else {
    constexpr int ctrl = (SPLIT == 4) ? SRC * 0x55 : (SRC == 0 ? 0xA0 : 0xF5);  // quad_perm selectors
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(iv, ctrl, 0xF, 0xF, true));
  }
}

template <int NS, int J, int SPLIT, int JJ = 0>
__device__ __forceinline__ void rebuild_state(const float* y, float* x) {
  if constexpr (JJ < NS) {
    x[JJ] = group_lane<SPLIT, JJ / J>(y[JJ % J]);
    rebuild_state<NS, J, SPLIT, JJ + 1>(y, x);
  }
}

template <int BASIS, int SPLIT, int DEG, bool TRACK>
__global__ void __launch_bounds__(256)
tick_split_kernel(const ModelDev* __restrict__ md, GenParams gp, int H, const float* __restrict__ x_t,
                  const float* __restrict__ u_user, const float* __restrict__ cand, Slot* __restrict__ slot,
                  mpmi_selection* __restrict__ out, int16_t* __restrict__ fv_out) {
  constexpr int NS = Dims<BASIS>::N, MS = Dims<BASIS>::M;
  constexpr int J = (NS + SPLIT - 1) / SPLIT;
  constexpr int D = (BASIS == MPMI_BASIS_RACE_CAR) ? 64 : 21;
  static_assert(SPLIT == 2 || SPLIT == 4 || SPLIT == 8, "groups of 2, 4 or 8 lanes (one row half)");
  __shared__ __attribute__((aligned(16))) float sK8[kSplitRows * 8];
  // A group never straddles a quad (2, 4) or a row half (8): the launch
  // uses a block that is a multiple of 64, so lane l of a wave holds gid with
  // gid % 64 == l.
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  const int c = gid / SPLIT, h = gid % SPLIT;
  const int Nc = gp.n_cand + 1;
  const bool valid = c < Nc;
  const int colpos = h * SplitLayout<J>::A;

  // State and candidate loads first: their latency overlaps the staging of K.
  float x[NS], u[MS], u0[MS];
#pragma unroll
  for (int j = 0; j < NS; ++j) x[j] = x_t[j];
#pragma unroll
  for (int j = 0; j < MS; ++j) {
    u0[j] = valid ? cand_value(gp, md, cand, u_user, c, 0, j) : 0.0f;
    u[j] = u0[j];
  }
  stage_K_split<BASIS, J>(md, sK8);
  SplitFold<BASIS, J> F;
  F.fold(sK8, colpos, u);
  SplitRows<BASIS, J> Kr;
  Kr.load(sK8, D, colpos);
  SafetyRegs<NS, DEG, TRACK> sr;
  sr.load(md);
  // The cost needs only the first segment's input: taken now, so its loads
  // are not on the path after the horizon.
  const bool lead = valid && h == 0;
  const float cst = lead ? cost_of<MS>(md, u0, u_user) : 0.0f;
  // Every register above is loaded before the horizon starts, so the loop
  // carries no wait for them.
  __syncthreads();
  int fv = H + 1;
  if (valid) {
    const int S = gp.n_seg;
    // Segment g covers steps s with floor((s - 1) S / H) == g; the next
    // boundary is the least s - 1 >= ceil((g + 1) H / S).
    int gcur = 0;
    int nxt = (H + S - 1) / S;
    for (int s = 1; s <= H; ++s) {
      if (s - 1 >= nxt) {
        gcur = ((s - 1) * S) / H;
        nxt = ((gcur + 1) * H + S - 1) / S;
#pragma unroll
        for (int j = 0; j < MS; ++j) u[j] = cand_value(gp, md, cand, u_user, c, gcur, j);
        F.fold(sK8, colpos, u);
      }
      // Each form in the one-lane kernel's operation order, so the two give
      // bit-identical states: race car as the feature sum, balance bot nested.
      float y[J];
      if constexpr (BASIS == MPMI_BASIS_RACE_CAR) {
        const float sp = __sinf(x[2]), cp = __cosf(x[2]);
#pragma unroll
        for (int jj = 0; jj < J; ++jj) {
          float v = fmaf(F.Tc[jj], cp, fmaf(F.Ts[jj], sp, F.cu[jj]));
#pragma unroll
          for (int k = 0; k < NS; ++k) v = fmaf(F.L[k][jj], x[k], v);
          y[jj] = v;
        }
        int q = 0;
#pragma unroll
        for (int k = 0; k < NS; ++k)
#pragma unroll
          for (int l = k; l < NS; ++l, ++q) {
            const float p = x[k] * x[l];
#pragma unroll
            for (int jj = 0; jj < J; ++jj) y[jj] = fmaf(p, Kr.q[q][jj], y[jj]);
          }
        const float tp[6] = {sp * x[3], sp * x[4], sp * x[5], cp * x[3], cp * x[4], cp * x[5]};
#pragma unroll
        for (int r = 0; r < 6; ++r)
#pragma unroll
          for (int jj = 0; jj < J; ++jj) y[jj] = fmaf(tp[r], Kr.t[r][jj], y[jj]);
      } else {
        // y = c + sum_k x_k (L_k + sum_{l >= k} Q_kl x_l) per output column.
#pragma unroll
        for (int jj = 0; jj < J; ++jj) y[jj] = F.cu[jj];
        int q = 0;
#pragma unroll
        for (int k = 0; k < NS; ++k) {
          float t[J];
#pragma unroll
          for (int jj = 0; jj < J; ++jj) t[jj] = F.L[k][jj];
#pragma unroll
          for (int l = k; l < NS; ++l, ++q)
#pragma unroll
            for (int jj = 0; jj < J; ++jj) t[jj] = fmaf(Kr.q[q][jj], x[l], t[jj]);
#pragma unroll
          for (int jj = 0; jj < J; ++jj) y[jj] = fmaf(x[k], t[jj], y[jj]);
        }
      }
      // The group's lanes hold identical states (same values, same
      // operations), so they leave the loop at the same step.
      rebuild_state<NS, J, SPLIT>(y, x);
      settle_state<NS>(x);
      if (!sr.safe(x)) {
        fv = s;
        break;
      }
    }
    if (fv_out && h == 0) fv_out[c] = (int16_t)fv;
  }
  const bool safe = lead && fv == H + 1;
  const unsigned long long ks = safe ? safe_key(cst, c) : kKeyNone;
  const unsigned long long kf = (lead && !safe) ? fallback_key(fv, cst, c) : kKeyNone;
  if (reduce_and_publish(ks, kf, safe && c > 0, slot, gridDim.x, blockIdx.x) && threadIdx.x == 0)
    finalize<MS>(md, gp, cand, u_user, H, slot, out);
}

template <int BASIS, int DEG, bool TRACK>
static void split_dispatch(int split, unsigned grid, int block, hipStream_t st, const ModelDev* md, const GenParams& gp,
                           int H, const float* x_t, const float* u_user, const float* cand, Slot* sl,
                           mpmi_selection* out, int16_t* fv) {
  if (split == 2)
    tick_split_kernel<BASIS, 2, DEG, TRACK><<<grid, block, 0, st>>>(md, gp, H, x_t, u_user, cand, sl, out, fv);
  else if (split == 4)
    tick_split_kernel<BASIS, 4, DEG, TRACK><<<grid, block, 0, st>>>(md, gp, H, x_t, u_user, cand, sl, out, fv);
  else
    tick_split_kernel<BASIS, 8, DEG, TRACK><<<grid, block, 0, st>>>(md, gp, H, x_t, u_user, cand, sl, out, fv);
}

hipError_t launch_tick_split(const mpmi_system& sys, int split, const void* model, const mpmi_tick_desc& d,
                             const float* x_t, const float* u_user, const float* cand, void* slot,
                             mpmi_selection* out, int16_t* fv, hipStream_t st) {
  GenParams gp;
  gp.seed = d.seed;
  gp.tick = d.tick;
  gp.loop = d.loop;
  gp.gen = d.gen;
  gp.n_cand = d.n_cand;
  gp.n_seg = d.n_seg;
  for (int j = 0; j < MPMI_MAX_INPUT; ++j) gp.grid[j] = d.grid[j] > 0 ? d.grid[j] : 1;
  const int block = d.block > 0 ? d.block : 256;
  const unsigned grid = (unsigned)((((long long)d.n_cand + 1) * split + block - 1) / block);
  const ModelDev* md = (const ModelDev*)model;
  Slot* sl = (Slot*)slot;
  const int H = d.horizon;
  const bool small = track_degree(sys) <= kSmallTrackDeg;
  if (sys.basis == MPMI_BASIS_RACE_CAR) {
    if (!sys.has_track)
      split_dispatch<MPMI_BASIS_RACE_CAR, 1, false>(split, grid, block, st, md, gp, H, x_t, u_user, cand, sl, out, fv);
    else if (small)
      split_dispatch<MPMI_BASIS_RACE_CAR, kSmallTrackDeg, true>(split, grid, block, st, md, gp, H, x_t, u_user, cand,
                                                                sl, out, fv);
    else
      split_dispatch<MPMI_BASIS_RACE_CAR, kMaxHarm, true>(split, grid, block, st, md, gp, H, x_t, u_user, cand, sl,
                                                          out, fv);
  } else {
    if (!sys.has_track)
      split_dispatch<MPMI_BASIS_BALANCE_BOT, 1, false>(split, grid, block, st, md, gp, H, x_t, u_user, cand, sl, out,
                                                       fv);
    else
      split_dispatch<MPMI_BASIS_BALANCE_BOT, kMaxHarm, true>(split, grid, block, st, md, gp, H, x_t, u_user, cand, sl,
                                                             out, fv);
  }
  return hipGetLastError();
}

}  // namespace mpmi
