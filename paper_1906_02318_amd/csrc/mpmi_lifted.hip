// Lifted whole-horizon form of the prediction (Sec. IV-A).
//
// The paper reads batched prediction in the Koopman representation as one
// matrix-matrix product: the lifted state z = psi(x_t, u_i) of every
// candidate advances by z <- z K with the full lifted operator K (D x D,
// fitted with the input held over a step), and the predicted state is read
// off z's state coordinates.  For a candidate's constant input this is
// exactly
//   x_s(u) = psi(x_t, u)^T M_s,   M_s = K^s C   (C picks the state columns),
// and every feature of the bases here is a product of a function of the
// state and a function of the input, psi_f(x, u) = g_{k_f}(u) phi_{r_f}(x).
// Collecting terms gives an exact regrouping,
//   x_s[j](u) = sum_k g_k(u) Q_s[k][j],
//   Q_s[k][j] = sum_r P_s[k][j][r] phi_r(x_t),
//   P_s[k][j][r] = sum of M_s[f][j] over the features f with (k_f, r_f) = (k, r),
// so a tick is:
//   1. P, once per model, in FP64 on the host (mpmi_lifted_pack);
//   2. Q, once per tick, by a small prologue launch (one workgroup per step);
//   3. every candidate's whole horizon as one product [candidates x kp] by
//      [kp x H * 4 output slots] on the FP32 matrix cores
//      (v_mfma_f32_16x16x4_f32), each 16 x 16 output tile checked for safety
//      as it leaves the accumulator, then the arg-min of the fused tick.
//
// Tile mapping.  A: rows = (step, slot) pairs, 4 steps x 4 slots per row tile;
// columns k = input functions (kp = 4, 8 or 12: one to three MFMAs).  B: k x 16
// candidates.  The 16 x 16 result leaves lane l holding rows 4 (l >> 4) .. +3
// of column l & 15: all four output slots of one step of one candidate, so the
// safety check of that candidate-step runs in one lane with no exchange.
// Output slots 0..3 hold the constrained state components (the track's x and
// y first), slots 4..7 the others, needed only when trajectories are stored.
// A wave owns 64 candidates as four column tiles; after the horizon the four
// lanes of a candidate combine their least unsafe step, and lane l keeps
// candidate 16 (l >> 4) + (l & 15) = l of the wave, as in the fused tick.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "mpmi_device.hpp"
#include "mpmi_launch.hpp"
#include "mpmi_tick_common.hpp"

namespace mpmi {

typedef float f32x4_t __attribute__((ext_vector_type(4)));

constexpr int kLiftPhiMax = 36;  // state functions phi (race car: 36)
constexpr int kLiftKMax = 12;    // input functions g, padded to a multiple of 4 (race car: 9 -> 12)
constexpr int kLiftSlots = 8;    // two groups of four output slots
constexpr int kLiftBlock = 256;  // four waves, 256 candidates per pass
constexpr int kLiftHPad = 256;   // horizon rounded up to whole row tiles of 4 steps
constexpr uint32_t kLiftMagic = 0x4c494654u;  // "LIFT"

// Packed lifted model.  md is a copy of the packed model with the safety
// constants remapped from state components to output slots 0..3, so the
// usual margin code reads an accumulator fragment directly.  P (pack time)
// and Q (per tick) follow the header at fixed offsets.
struct alignas(256) LiftedDev {
  ModelDev md;
  uint32_t magic;
  int32_t basis, h_max, kp, n_phi, n_slots, n_safe_slots, pad0;
  int32_t slot_comp[kLiftSlots];  // state component held in output slot i, -1 for none
};
constexpr size_t kLiftPFloats = (size_t)kLiftKMax * kLiftSlots * kLiftPhiMax;  // per step
constexpr size_t kLiftQFloats = (size_t)2 * kLiftHPad * kLiftKMax * 4;        // per tick

__host__ __device__ inline size_t lifted_p_offset() { return sizeof(LiftedDev); }
__host__ __device__ inline size_t lifted_q_offset(int h_max) {
  return sizeof(LiftedDev) + (size_t)h_max * kLiftPFloats * sizeof(float);
}

size_t lifted_bytes(int h_max) { return lifted_q_offset(h_max) + kLiftQFloats * sizeof(float); }

template <int BASIS>
struct LiftShape;
template <>
struct LiftShape<MPMI_BASIS_LINEAR> { static constexpr int KP = 8; };
template <>
struct LiftShape<MPMI_BASIS_BALANCE_BOT> { static constexpr int KP = 4; };
template <>
struct LiftShape<MPMI_BASIS_RACE_CAR> { static constexpr int KP = 12; };

// ---------------------------------------------------------------------------
// The decomposition psi_f(x, u) = g_{k_f}(u) phi_{r_f}(x) of each basis.
//   LINEAR       phi = [1, x_0 .. x_{n-1}]                     g = [1, u_0 .. u_{m-1}]
//   BALANCE_BOT  phi = [1, x_0..x_3, x_k x_l (k <= l < 4)]     g = [1, u, u^2]
//   RACE_CAR     phi = [1, x_0..x_5, x_k x_l (k <= l < 6), sin psi, cos psi,
//                       sin psi (vx, vy, r), cos psi (vx, vy, r)]       (36)
//                g = [1, delta, a, delta^2, delta a, a^2, sin delta, cos delta, a sin delta]
// (products in k-outer order, as in the bases themselves).
// ---------------------------------------------------------------------------
__host__ __device__ constexpr int tri_index(int k, int l, int nv) { return k * nv - (k * (k - 1)) / 2 + (l - k); }

static void decompose(int basis, int n, int m, int D, std::vector<int>& kf, std::vector<int>& rf, int* n_phi,
                      int* n_g) {
  kf.assign(D, 0);
  rf.assign(D, 0);
  if (basis == MPMI_BASIS_LINEAR) {
    for (int f = 0; f < n; ++f) { kf[f] = 0; rf[f] = 1 + f; }
    for (int j = 0; j < m; ++j) { kf[n + j] = 1 + j; rf[n + j] = 0; }
    *n_phi = 1 + n;
    *n_g = 1 + m;
    return;
  }
  if (basis == MPMI_BASIS_BALANCE_BOT) {
    kf[0] = 0; rf[0] = 0;
    for (int k = 0; k < 4; ++k) { kf[1 + k] = 0; rf[1 + k] = 1 + k; }
    kf[5] = 1; rf[5] = 0;
    for (int k = 0; k < 5; ++k)
      for (int l = k; l < 5; ++l) {
        const int f = quad_index(k, l, 5);
        if (l < 4) { kf[f] = 0; rf[f] = 5 + tri_index(k, l, 4); }
        else if (k < 4) { kf[f] = 1; rf[f] = 1 + k; }
        else { kf[f] = 2; rf[f] = 0; }
      }
    *n_phi = 15;
    *n_g = 3;
    return;
  }
  // race car, w = [x, y, psi, vx, vy, r, delta, a]
  kf[0] = 0; rf[0] = 0;
  for (int k = 0; k < 6; ++k) { kf[1 + k] = 0; rf[1 + k] = 1 + k; }
  kf[7] = 1; rf[7] = 0;
  kf[8] = 2; rf[8] = 0;
  for (int k = 0; k < 8; ++k)
    for (int l = k; l < 8; ++l) {
      const int f = quad_index(k, l, 8);
      if (l < 6) { kf[f] = 0; rf[f] = 7 + tri_index(k, l, 6); }
      else if (k < 6) { kf[f] = (l == 6) ? 1 : 2; rf[f] = 1 + k; }
      else if (l == 6) { kf[f] = 3; rf[f] = 0; }        // delta^2
      else if (k == 6) { kf[f] = 4; rf[f] = 0; }        // delta a
      else { kf[f] = 5; rf[f] = 0; }                    // a^2
    }
  const int tail_k[19] = {0, 0, 6, 7, 0, 0, 0, 2, 0, 0, 0, 2, 6, 6, 6, 7, 7, 7, 8};
  const int tail_r[19] = {28, 29, 0, 0, 30, 31, 32, 28, 33, 34, 35, 29, 4, 5, 6, 4, 5, 6, 0};
  for (int q = 0; q < 19; ++q) { kf[45 + q] = tail_k[q]; rf[45 + q] = tail_r[q]; }
  *n_phi = 36;
  *n_g = 9;
}

template <int BASIS>
__device__ __forceinline__ void phi_eval(const float* __restrict__ x, int n, float* phi) {
  phi[0] = 1.0f;
  if constexpr (BASIS == MPMI_BASIS_LINEAR) {
    for (int k = 0; k < n; ++k) phi[1 + k] = x[k];
  } else if constexpr (BASIS == MPMI_BASIS_BALANCE_BOT) {
    for (int k = 0; k < 4; ++k) phi[1 + k] = x[k];
    for (int k = 0; k < 4; ++k)
      for (int l = k; l < 4; ++l) phi[5 + tri_index(k, l, 4)] = x[k] * x[l];
  } else {
    for (int k = 0; k < 6; ++k) phi[1 + k] = x[k];
    for (int k = 0; k < 6; ++k)
      for (int l = k; l < 6; ++l) phi[7 + tri_index(k, l, 6)] = x[k] * x[l];
    float sp, cp;
    sincosf(x[2], &sp, &cp);
    phi[28] = sp; phi[29] = cp;
    phi[30] = sp * x[3]; phi[31] = sp * x[4]; phi[32] = sp * x[5];
    phi[33] = cp * x[3]; phi[34] = cp * x[4]; phi[35] = cp * x[5];
  }
}

// g(u), padded with zeros to KP entries.
template <int BASIS>
__device__ __forceinline__ void g_eval(const float* u, int m, float* g) {
  constexpr int KP = LiftShape<BASIS>::KP;
#pragma unroll
  for (int k = 0; k < KP; ++k) g[k] = 0.0f;
  g[0] = 1.0f;
  if constexpr (BASIS == MPMI_BASIS_LINEAR) {
#pragma unroll
    for (int j = 0; j < MPMI_MAX_INPUT; ++j) g[1 + j] = j < m ? u[j] : 0.0f;
  } else if constexpr (BASIS == MPMI_BASIS_BALANCE_BOT) {
    g[1] = u[0];
    g[2] = u[0] * u[0];
  } else {
    const float d = u[0], a = u[1];
    float sd, cd;
    sincosf(d, &sd, &cd);
    g[1] = d; g[2] = a; g[3] = d * d; g[4] = d * a; g[5] = a * a;
    g[6] = sd; g[7] = cd; g[8] = a * sd;
  }
}

// ---------------------------------------------------------------------------
// Per-tick prologue: Q_s[k][slot] = sum_r P_s[k][slot][r] phi_r(x_t), one
// workgroup per step s < Hpad (steps past H are zero), written as
// Qt[group][s][k][slot & 3], the order the tick stages into LDS.
// ---------------------------------------------------------------------------
template <int BASIS>
__global__ void __launch_bounds__(128)
lifted_prologue_kernel(const LiftedDev* __restrict__ ld, int H, int hpad, const float* __restrict__ x_t,
                       float* __restrict__ Qt) {
  constexpr int KP = LiftShape<BASIS>::KP;
  __shared__ float phi[kLiftPhiMax];
  const int n = ld->md.n;
  if (threadIdx.x == 0) {
    float x[MPMI_MAX_STATE];
    for (int k = 0; k < MPMI_MAX_STATE; ++k) x[k] = k < n ? x_t[k] : 0.0f;
    for (int r = 0; r < kLiftPhiMax; ++r) phi[r] = 0.0f;
    phi_eval<BASIS>(x, n, phi);
  }
  __syncthreads();
  const int s = blockIdx.x, t = threadIdx.x;
  const int k = t / kLiftSlots, slot = t % kLiftSlots;
  if (k >= KP) return;
  float q = 0.0f;
  if (s < H && k < ld->kp && slot < ld->n_slots) {
    const float* P = (const float*)((const char*)ld + lifted_p_offset()) + (size_t)s * kLiftPFloats +
                     ((size_t)k * kLiftSlots + slot) * kLiftPhiMax;
    const int nphi = ld->n_phi;
    for (int r = 0; r < nphi; ++r) q = fmaf(P[r], phi[r], q);
  }
  Qt[(((size_t)(slot >> 2) * hpad + s) * KP + k) * 4 + (slot & 3)] = q;
}

// ---------------------------------------------------------------------------
// The tick.  Persistent: workgroup b takes 256-candidate passes b, b + grid,
// ... and publishes its arg-min keys once.  TRAJ also computes slots 4..7 and
// stores the predicted states of the steps it evaluates (every step up to
// each candidate's first violation, some after it).
// ---------------------------------------------------------------------------
template <int BASIS, int DEG, bool TRAJ>
__global__ void __launch_bounds__(kLiftBlock)
lifted_tick_kernel(const LiftedDev* __restrict__ ld, GenParams gp, int H, int hpad,
                   const float* __restrict__ u_user, const float* __restrict__ cand, const float* __restrict__ Qt,
                   Slot* __restrict__ slot, mpmi_selection* __restrict__ out, int16_t* __restrict__ fv_out,
                   float* __restrict__ traj, long long traj_ld) {
  constexpr int KP = LiftShape<BASIS>::KP, KC = KP / 4, MS = Dims<BASIS>::M, G = TRAJ ? 2 : 1;
  extern __shared__ float sQ[];  // [G][hpad][KP][4]
  const ModelDev* __restrict__ md = &ld->md;
  // The constraint constants held in registers for the whole launch (a call
  // per output tile re-fetching them by scalar loads stalled on each fetch).
  const SafetyConsts sc = md->safe;
  {
    const float4* src = reinterpret_cast<const float4*>(Qt);
    float4* dst = reinterpret_cast<float4*>(sQ);
    for (int e = threadIdx.x; e < hpad * KP; e += kLiftBlock) dst[e] = src[e];
    if (TRAJ)
      for (int e = threadIdx.x; e < hpad * KP; e += kLiftBlock) dst[hpad * KP + e] = src[hpad * KP + e];
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = lane & 15, quarter = lane >> 4;
  const int Nc = gp.n_cand + 1;
  const int n = md->n;
  const int nrt = hpad >> 2;
  // this lane's A-operand address within a row tile: row (col) = 4 * step + slot
  const int a_off = ((col >> 2) * KP + quarter) * 4 + (col & 3);
  unsigned long long ks = kKeyNone, kf = kKeyNone;
  unsigned int n_safe = 0;  // uniform across the wave
  const int n_pass = (Nc + kLiftBlock - 1) / kLiftBlock;
  for (int pass = blockIdx.x; pass < n_pass; pass += gridDim.x) {
    const int wbase = pass * kLiftBlock + wave * 64;
    float B[4][KC];
    float own_u[MS];
    int fvm[4];
    unsigned int dead = 0, inval[4];
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) {
      const int c = wbase + 16 * ct + col;
      const bool valid = c < Nc;
      float u[MS], g[KP];
#pragma unroll
      for (int j = 0; j < MS; ++j) u[j] = (valid && j < md->m) ? cand_value(gp, md, cand, u_user, c, 0, j) : 0.0f;
      g_eval<BASIS>(u, md->m, g);
#pragma unroll
      for (int i = 0; i < KC; ++i) {
        // register values: the selection stays a chain of selects instead of
        // becoming an indexed scratch load of g
        float g0 = g[4 * i], g1 = g[4 * i + 1], g2 = g[4 * i + 2], g3 = g[4 * i + 3];
        asm volatile("" : "+v"(g0), "+v"(g1), "+v"(g2), "+v"(g3));
        float v = quarter == 1 ? g1 : g0;
        v = quarter == 2 ? g2 : v;
        v = quarter == 3 ? g3 : v;
        B[ct][i] = v;
      }
      if (quarter == ct) {
#pragma unroll
        for (int j = 0; j < MS; ++j) own_u[j] = u[j];
      }
      fvm[ct] = H + 1;
      const unsigned long long b = __ballot(!valid);
      inval[ct] = (unsigned int)((b | (b >> 16) | (b >> 32) | (b >> 48)) & 0xffffull);
      if (inval[ct] == 0xffffu) dead |= 1u << ct;
    }
    for (int rt = 0; rt < nrt && dead != 0xfu; ++rt) {
      float A[G][KC];
#pragma unroll
      for (int gi = 0; gi < G; ++gi)
#pragma unroll
        for (int i = 0; i < KC; ++i) A[gi][i] = sQ[(size_t)(gi * hpad + 4 * rt) * KP * 4 + a_off + 16 * i];
      const int s = 4 * rt + quarter + 1;  // this lane's step
      // Every live tile's products first (independent accumulators, issued
      // back to back), then the checks: one tile's MFMA latency overlaps the
      // next tile's issue and the checks of the tiles before it.
      f32x4_t acc[4], acc1[4];
#pragma unroll
      for (int ct = 0; ct < 4; ++ct) {
        acc[ct] = f32x4_t{0.0f, 0.0f, 0.0f, 0.0f};
        acc1[ct] = f32x4_t{0.0f, 0.0f, 0.0f, 0.0f};
        if (dead & (1u << ct)) continue;  // uniform
#pragma unroll
        for (int i = 0; i < KC; ++i)
          acc[ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(A[0][i], B[ct][i], acc[ct], 0, 0, 0);
        if constexpr (TRAJ) {
#pragma unroll
          for (int i = 0; i < KC; ++i)
            acc1[ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(A[G - 1][i], B[ct][i], acc1[ct], 0, 0, 0);
        }
      }
#pragma unroll
      for (int ct = 0; ct < 4; ++ct) {
        if (dead & (1u << ct)) continue;  // uniform
        const float x4[4] = {acc[ct][0], acc[ct][1], acc[ct][2], acc[ct][3]};
        if constexpr (TRAJ) {
          const int c = wbase + 16 * ct + col;
          if (s <= H && c < Nc) {
            const float v8[8] = {acc[ct][0], acc[ct][1], acc[ct][2], acc[ct][3],
                                 acc1[ct][0], acc1[ct][1], acc1[ct][2], acc1[ct][3]};
#pragma unroll
            for (int i = 0; i < kLiftSlots; ++i) {
              const int comp = ld->slot_comp[i];
              if (comp >= 0)
                __builtin_nontemporal_store(v8[i], &traj[((size_t)(s - 1) * n + comp) * (size_t)traj_ld + c]);
            }
          }
        }
        const bool unsafe = !all_safe_of<4, DEG>(&sc, x4);
        fvm[ct] = (s <= H && unsafe) ? min(fvm[ct], s) : fvm[ct];
      }
#pragma unroll
      for (int ct = 0; ct < 4; ++ct) {
        const unsigned long long b = __ballot(fvm[ct] <= H);
        const unsigned int f16 = (unsigned int)((b | (b >> 16) | (b >> 32) | (b >> 48)) & 0xffffull);
        if ((f16 | inval[ct]) == 0xffffu) dead |= 1u << ct;
      }
    }
    // first violation of each candidate: least over its four lanes; lane l
    // keeps column tile l >> 4, i.e. candidate wbase + l
    int fv = H + 1;
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) {
      int v = fvm[ct];
      v = min(v, __shfl_xor(v, 16));
      v = min(v, __shfl_xor(v, 32));
      if (quarter == ct) fv = v;
    }
    const int c = wbase + lane;
    const bool valid = c < Nc;
    if (valid && fv_out) fv_out[c] = (int16_t)fv;
    const float cst = valid ? cost_of<MS>(md, own_u, u_user) : 0.0f;
    const bool safe = valid && fv == H + 1;
    const unsigned long long a = safe ? safe_key(cst, c) : kKeyNone;
    const unsigned long long b = (valid && !safe) ? fallback_key(fv, cst, c) : kKeyNone;
    ks = a < ks ? a : ks;
    kf = b < kf ? b : kf;
    n_safe += (unsigned int)__popcll(__ballot(safe && c > 0));
  }
  if (publish_wave_counted(ks, kf, n_safe, slot, gridDim.x, blockIdx.x) && threadIdx.x == 0)
    finalize<MS>(md, gp, cand, u_user, H, slot, out);
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
void lifted_layout(int basis, int n, int m, int D, int* feat_g, int* feat_phi, int* n_phi, int* n_g) {
  std::vector<int> kf, rf;
  decompose(basis, n, m, D, kf, rf, n_phi, n_g);
  for (int f = 0; f < D; ++f) {
    feat_g[f] = kf[f];
    feat_phi[f] = rf[f];
  }
}

// Output slots: the constrained components first (x and y first when there is
// a track), then the others; returns the count of constrained ones, or -1 if
// more than four components are constrained.
static int assign_slots(const mpmi_system& sys, int* slot_comp) {
  const int n = sys.n_state;
  bool used[MPMI_MAX_STATE] = {};
  int ns = 0;
  if (sys.has_track) {
    slot_comp[ns++] = 0;
    slot_comp[ns++] = 1;
    used[0] = used[1] = true;
  }
  for (int b = 0; b < sys.n_box; ++b) {
    const int k = sys.box_index[b];
    if (used[k]) continue;
    if (ns == 4) return -1;
    used[k] = true;
    slot_comp[ns++] = k;
  }
  const int n_safe = ns;
  for (int k = 0; k < kLiftSlots; ++k)
    if (k >= ns) slot_comp[k] = -1;
  // the rest: slots n_safe .. 3, then 4 ..
  int next = n_safe;
  for (int k = 0; k < n; ++k) {
    if (used[k]) continue;
    if (next < kLiftSlots) slot_comp[next++] = k;
  }
  return n_safe;
}

hipError_t lifted_pack(const mpmi_system& sys, int D, int state_feat0, const void* model, const double* K_dev,
                       int h_max, void* lifted, int* n_safe_slots) {
  const int n = sys.n_state, m = sys.n_input;
  LiftedDev hdr;
  std::memset(&hdr, 0, sizeof hdr);
  hipError_t e = hipMemcpy(&hdr.md, model, sizeof(ModelDev), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return e;
  std::vector<double> K((size_t)D * D);
  e = hipMemcpy(K.data(), K_dev, K.size() * sizeof(double), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return e;
  int slot_comp[kLiftSlots];
  const int ns = assign_slots(sys, slot_comp);
  *n_safe_slots = ns;
  if (ns < 0) return hipErrorInvalidValue;
  // Safety constants from components to slots 0..3 (the track reads slots 0, 1).
  const SafetyConsts sc = hdr.md.safe;
  int cmask = 0;
  for (int i = 0; i < MPMI_MAX_STATE; ++i) hdr.md.safe.comp_lim[i] = INFINITY;
  for (int i = 0; i < 4; ++i) {
    const int k = slot_comp[i];
    if (i < ns && k >= 0 && (sc.comp_mask & (1 << k))) {
      hdr.md.safe.comp_lim[i] = sc.comp_lim[k];
      cmask |= 1 << i;
    }
  }
  hdr.md.safe.comp_mask = cmask;
  for (int b = 0; b < sys.n_box; ++b)
    for (int i = 0; i < 4; ++i)
      if (slot_comp[i] == sys.box_index[b]) hdr.md.safe.box_index[b] = i;
  std::vector<int> kf, rf;
  int n_phi = 0, n_g = 0;
  decompose(sys.basis, n, m, D, kf, rf, &n_phi, &n_g);
  hdr.magic = kLiftMagic;
  hdr.basis = sys.basis;
  hdr.h_max = h_max;
  hdr.kp = n_g;
  hdr.n_phi = n_phi;
  hdr.n_slots = n < kLiftSlots ? n : kLiftSlots;
  hdr.n_safe_slots = ns;
  for (int i = 0; i < kLiftSlots; ++i) hdr.slot_comp[i] = slot_comp[i];
  // M_s = K^s C in FP64 (rows: features; C picks the state columns), s = 1 .. h_max.
  std::vector<double> M((size_t)D * n), Mn((size_t)D * n);
  for (int f = 0; f < D; ++f)
    for (int j = 0; j < n; ++j) M[(size_t)f * n + j] = K[(size_t)f * D + state_feat0 + j];
  std::vector<float> P((size_t)h_max * kLiftPFloats, 0.0f);
  std::vector<double> acc(kLiftPFloats);
  for (int s = 0; s < h_max; ++s) {
    if (s > 0) {
      for (int f = 0; f < D; ++f)
        for (int j = 0; j < n; ++j) {
          double v = 0.0;
          for (int q = 0; q < D; ++q) v += K[(size_t)f * D + q] * M[(size_t)q * n + j];
          Mn[(size_t)f * n + j] = v;
        }
      M.swap(Mn);
    }
    std::fill(acc.begin(), acc.end(), 0.0);
    for (int f = 0; f < D; ++f)
      for (int i = 0; i < kLiftSlots; ++i) {
        const int j = slot_comp[i];
        if (j < 0) continue;
        acc[((size_t)kf[f] * kLiftSlots + i) * kLiftPhiMax + rf[f]] += M[(size_t)f * n + j];
      }
    float* Ps = P.data() + (size_t)s * kLiftPFloats;
    for (size_t q = 0; q < kLiftPFloats; ++q) Ps[q] = (float)acc[q];
  }
  e = hipMemcpy(lifted, &hdr, sizeof hdr, hipMemcpyHostToDevice);
  if (e != hipSuccess) return e;
  e = hipMemcpy((char*)lifted + lifted_p_offset(), P.data(), P.size() * sizeof(float), hipMemcpyHostToDevice);
  if (e != hipSuccess) return e;
  return hipMemset((char*)lifted + lifted_q_offset(h_max), 0, kLiftQFloats * sizeof(float));
}

template <int BASIS, int DEG>
static void lifted_dispatch(bool traj, unsigned grid, size_t lds, hipStream_t st, const LiftedDev* ld,
                            const GenParams& gp, int H, int hpad, const float* u_user, const float* cand,
                            const float* Qt, Slot* sl, mpmi_selection* out, int16_t* fv, float* tr, long long trl) {
  if (traj)
    lifted_tick_kernel<BASIS, DEG, true>
        <<<grid, kLiftBlock, lds, st>>>(ld, gp, H, hpad, u_user, cand, Qt, sl, out, fv, tr, trl);
  else
    lifted_tick_kernel<BASIS, DEG, false>
        <<<grid, kLiftBlock, lds, st>>>(ld, gp, H, hpad, u_user, cand, Qt, sl, out, fv, tr, trl);
}

hipError_t launch_tick_lifted(const mpmi_system& sys, void* lifted, int h_max, const mpmi_tick_desc& d,
                              const float* x_t, const float* u_user, const float* cand, void* slot,
                              mpmi_selection* out, int16_t* fv, float* traj, long long traj_ld, int grid_per_cu,
                              hipStream_t st) {
  const LiftedDev* ld = (const LiftedDev*)lifted;
  float* Qt = (float*)((char*)lifted + lifted_q_offset(h_max));
  const int H = d.horizon;
  const int hpad = (H + 3) & ~3;
  GenParams gp{};
  gp.seed = d.seed;
  gp.tick = d.tick;
  gp.loop = d.loop;
  gp.gen = d.gen;
  gp.n_cand = d.n_cand;
  gp.n_seg = 1;
  for (int j = 0; j < MPMI_MAX_INPUT; ++j) gp.grid[j] = d.grid[j] > 0 ? d.grid[j] : 1;
  const long long Nc = (long long)d.n_cand + 1;
  const long long passes = (Nc + kLiftBlock - 1) / kLiftBlock;
  const long long cap = (long long)device_cu_count() * grid_per_cu;
  const unsigned grid = (unsigned)std::min(passes, cap);
  const bool tr = traj != nullptr;
  Slot* sl = (Slot*)slot;
  int kp = 4;
  switch (sys.basis) {
    case MPMI_BASIS_LINEAR:
      kp = LiftShape<MPMI_BASIS_LINEAR>::KP;
      lifted_prologue_kernel<MPMI_BASIS_LINEAR><<<hpad, 128, 0, st>>>(ld, H, hpad, x_t, Qt);
      break;
    case MPMI_BASIS_BALANCE_BOT:
      kp = LiftShape<MPMI_BASIS_BALANCE_BOT>::KP;
      lifted_prologue_kernel<MPMI_BASIS_BALANCE_BOT><<<hpad, 128, 0, st>>>(ld, H, hpad, x_t, Qt);
      break;
    default:
      kp = LiftShape<MPMI_BASIS_RACE_CAR>::KP;
      lifted_prologue_kernel<MPMI_BASIS_RACE_CAR><<<hpad, 128, 0, st>>>(ld, H, hpad, x_t, Qt);
      break;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const size_t lds = (size_t)(tr ? 2 : 1) * hpad * kp * 4 * sizeof(float);
  switch (sys.basis) {
    case MPMI_BASIS_LINEAR:
      lifted_dispatch<MPMI_BASIS_LINEAR, kMaxHarm>(tr, grid, lds, st, ld, gp, H, hpad, u_user, cand, Qt, sl, out, fv,
                                                   traj, traj_ld);
      break;
    case MPMI_BASIS_BALANCE_BOT:
      lifted_dispatch<MPMI_BASIS_BALANCE_BOT, kMaxHarm>(tr, grid, lds, st, ld, gp, H, hpad, u_user, cand, Qt, sl,
                                                        out, fv, traj, traj_ld);
      break;
    default:
      if (track_degree(sys) <= kSmallTrackDeg)
        lifted_dispatch<MPMI_BASIS_RACE_CAR, kSmallTrackDeg>(tr, grid, lds, st, ld, gp, H, hpad, u_user, cand, Qt,
                                                             sl, out, fv, traj, traj_ld);
      else
        lifted_dispatch<MPMI_BASIS_RACE_CAR, kMaxHarm>(tr, grid, lds, st, ld, gp, H, hpad, u_user, cand, Qt, sl,
                                                       out, fv, traj, traj_ld);
      break;
  }
  return hipGetLastError();
}

}  // namespace mpmi
