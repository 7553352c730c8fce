// Learned proposal network: forward, mixture loss, backward, Adam and the
// mixture sampler, all hand-written for gfx950.
//
// Shape (fixed): 8 standardised inputs -> 256 -> 256 -> 256 -> 80, GELU (tanh
// form) on the hidden layers; the 80 outputs are 16 x {logit, mu_0, mu_1,
// log sigma_0, log sigma_1} of a diagonal-Gaussian mixture over the input
// normalised to [-1, 1]^2.  Weights are BF16 (FP32 master copy for Adam);
// every product accumulates in FP32.
//
// The dense products run on BF16 matrix cores (v_mfma_f32_16x16x32_bf16):
// a 256-thread workgroup computes a 64 x 64 tile of C = op(A) op(B), each wave
// a 32 x 32 quarter as 2 x 2 MFMA blocks, with 64 x 32 slices of A and B
// staged through LDS per k-step (transposed operands are transposed while
// staging, so one kernel serves the forward product and both backward ones).
#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>

#include "mpmi_device.hpp"
#include "mpmi_launch.hpp"

namespace mpmi {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

constexpr int kGelu = 1, kLinear = 2, kGeluBack = 3, kPlain = 4;
constexpr float kGeluC = 0.7978845608028654f;  // sqrt(2/pi)
constexpr float kGeluA = 0.044715f;

__device__ __forceinline__ uint16_t f2bf(float f) { return (uint16_t)bf16_bits_rne_u(f); }
__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

__device__ __forceinline__ float gelu_f(float z) {
  return 0.5f * z * (1.0f + tanhf(kGeluC * fmaf(kGeluA * z * z, z, z)));
}
__device__ __forceinline__ float gelu_grad_f(float z) {
  const float t = tanhf(kGeluC * fmaf(kGeluA * z * z, z, z));
  return 0.5f * (1.0f + t) + 0.5f * z * (1.0f - t * t) * kGeluC * fmaf(3.0f * kGeluA, z * z, 1.0f);
}

struct GemmArgs {
  const uint16_t* A;  // bf16
  const uint16_t* B;  // bf16
  int M, N, K;
  int lda, ldb;
  int ta, tb;          // A(m,k) = ta ? A[k*lda+m] : A[m*lda+k]; B(k,n) = tb ? B[n*ldb+k] : B[k*ldb+n]
  const float* bias;   // [N] or NULL
  const float* zin;    // kGeluBack: pre-activation [M][N] FP32
  float* out_f32;      // [M][N] or NULL
  uint16_t* out_bf16;  // [M][N] or NULL
  uint16_t* out_bf16_t;  // the BF16 output transposed, [N][ldt], or NULL
  int ldt;
  // Split-K (kPlain only): gridDim.z parts of ksplit rows of K each write
  // FP32 partial products to part[z][M][N]; colsum (or NULL), an FP32
  // [K][N] matrix whose column sums over each part's K range go to
  // part_cs[z][N] (the bias gradient of a dW product).
  int ksplit;
  float* part;
  const float* colsum;
  float* part_cs;
  bool vec_a, vec_b;   // 16-byte loads allowed (leading dimension a multiple of 8, 16-byte aligned base)
  bool vec_t;          // 8-byte transposed stores allowed (ldt a multiple of 4, 8-byte aligned base)
};

// C = op(A) op(B) on v_mfma_f32_16x16x32_bf16.  A 256-thread workgroup owns a
// 64 x 64 tile of C, each wave a 32 x 32 quarter as 2 x 2 MFMA blocks.  Per
// 32-wide k step every thread moves one 16-byte chunk (8 BF16) of A and one
// of B from global memory into LDS, in the operand order the MFMA reads (row
// or column, then k): a chunk along k (row-major A, transposed B) is stored
// as one 16-byte LDS write, a chunk along m or n as eight 2-byte writes.  The
// next stage's chunks (several k steps) are loaded into registers while the
// current stage's MFMAs run (see gemm_bf16_kernel).  Chunks that are contiguous, aligned and wholly inside the matrix take one
// 16-byte load; others (ragged edges, odd leading dimensions) load element by
// element.
constexpr int kGemmKP = 40;  // padded k extent of an LDS row (80 B, keeps 16-B alignment)

struct GemmChunk {
  uint4 a, b;
};

// Eight BF16 values p[0], p[s], ..., p[7 s], those with index >= lim zero,
// packed as a 16-byte chunk; one 16-byte load when all eight are in range
// and contiguous and aligned (vec).
__device__ __forceinline__ uint4 load_chunk(const uint16_t* __restrict__ p, size_t s, int idx, int lim, bool vec) {
  if (vec && idx + 8 <= lim) return *reinterpret_cast<const uint4*>(p);
  uint32_t w[4] = {0u, 0u, 0u, 0u};
#pragma unroll
  for (int i = 0; i < 8; ++i)
    if (idx + i < lim) w[i >> 1] |= (uint32_t)p[(size_t)i * s] << ((i & 1) * 16);
  return make_uint4(w[0], w[1], w[2], w[3]);
}

// This thread's chunks of the k step at k0: A row-major -- row t / 4, k
// (t % 4) * 8 .. +8; A transposed -- k t / 8, rows (t % 8) * 8 .. +8; B
// transposed -- column t / 4, k (t % 4) * 8 .. +8; B row-major -- k t / 8,
// columns (t % 8) * 8 .. +8.  Values outside the matrix (or past kend) are 0.
__device__ __forceinline__ void gemm_load(const GemmArgs& g, int m0, int n0, int k0, int kend, GemmChunk* c) {
  const int t = threadIdx.x;
  c->a = make_uint4(0u, 0u, 0u, 0u);
  c->b = make_uint4(0u, 0u, 0u, 0u);
  if (!g.ta) {
    const int m = m0 + (t >> 2), k = k0 + (t & 3) * 8;
    if (m < g.M && k < kend) c->a = load_chunk(g.A + (size_t)m * g.lda + k, 1, k, kend, g.vec_a);
  } else {
    const int k = k0 + (t >> 3), m = m0 + (t & 7) * 8;
    if (m < g.M && k < kend) c->a = load_chunk(g.A + (size_t)k * g.lda + m, 1, m, g.M, g.vec_a);
  }
  if (g.tb) {
    const int n = n0 + (t >> 2), k = k0 + (t & 3) * 8;
    if (n < g.N && k < kend) c->b = load_chunk(g.B + (size_t)n * g.ldb + k, 1, k, kend, g.vec_b);
  } else {
    const int k = k0 + (t >> 3), n = n0 + (t & 7) * 8;
    if (n < g.N && k < kend) c->b = load_chunk(g.B + (size_t)k * g.ldb + n, 1, n, g.N, g.vec_b);
  }
}

__device__ __forceinline__ void gemm_store(const GemmArgs& g, const GemmChunk& c, uint16_t (*As)[kGemmKP],
                                           uint16_t (*Bs)[kGemmKP]) {
  const int t = threadIdx.x;
  const uint32_t wa[4] = {c.a.x, c.a.y, c.a.z, c.a.w};
  const uint32_t wb[4] = {c.b.x, c.b.y, c.b.z, c.b.w};
  if (!g.ta) {
    *reinterpret_cast<uint4*>(&As[t >> 2][(t & 3) * 8]) = c.a;
  } else {
    const int k = t >> 3, m = (t & 7) * 8;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      As[m + 2 * i][k] = (uint16_t)(wa[i] & 0xffffu);
      As[m + 2 * i + 1][k] = (uint16_t)(wa[i] >> 16);
    }
  }
  if (g.tb) {
    *reinterpret_cast<uint4*>(&Bs[t >> 2][(t & 3) * 8]) = c.b;
  } else {
    const int k = t >> 3, n = (t & 7) * 8;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      Bs[n + 2 * i][k] = (uint16_t)(wb[i] & 0xffffu);
      Bs[n + 2 * i + 1][k] = (uint16_t)(wb[i] >> 16);
    }
  }
}

// A stage is kGemmSub k-steps of 32 (128 values of k): every thread issues
// the loads of the whole next stage (kGemmSub 16-byte chunks of A and of B)
// into registers before the MFMAs of the current one, so a product with
// K = 256 takes two memory round trips instead of eight (a single stage of
// 256, one round trip, measured the same at batch 4,096: launch and epilogue
// latency, not the round trips, bound those products).  One LDS buffer
// (40 KB, several workgroups per CU): the registers are stored into it
// after a barrier that ends the current stage's reads.
constexpr int kGemmSub = 4;

template <int EPI>
__global__ void __launch_bounds__(256) gemm_bf16_kernel(GemmArgs g) {
  __shared__ __attribute__((aligned(16))) uint16_t As[kGemmSub][64][kGemmKP];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[kGemmSub][64][kGemmKP];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
  const int kbeg = blockIdx.z * g.ksplit;
  const int kend = min(g.K, kbeg + g.ksplit);
  constexpr int kStage = 32 * kGemmSub;
  f32x4_t acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4_t{0.f, 0.f, 0.f, 0.f};
  GemmChunk c[kGemmSub];
#pragma unroll
  for (int q = 0; q < kGemmSub; ++q) gemm_load(g, m0, n0, kbeg + 32 * q, kend, &c[q]);
#pragma unroll
  for (int q = 0; q < kGemmSub; ++q) gemm_store(g, c[q], As[q], Bs[q]);
  __syncthreads();
  for (int k0 = kbeg; k0 < kend; k0 += kStage) {
    const bool more = k0 + kStage < kend;
    if (more) {
#pragma unroll
      for (int q = 0; q < kGemmSub; ++q) gemm_load(g, m0, n0, k0 + kStage + 32 * q, kend, &c[q]);
    }
    const int kq = (lane >> 4) * 8;
#pragma unroll
    for (int q = 0; q < kGemmSub; ++q) {
      if (k0 + 32 * q >= kend) break;  // uniform: a ragged last stage
      bf16x8_t af[2], bfr[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        af[i] = *reinterpret_cast<const bf16x8_t*>(&As[q][wm * 32 + i * 16 + (lane & 15)][kq]);
        bfr[i] = *reinterpret_cast<const bf16x8_t*>(&Bs[q][wn * 32 + i * 16 + (lane & 15)][kq]);
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfr[j], acc[i][j], 0, 0, 0);
    }
    if (more) {  // uniform
      __syncthreads();  // the stage's reads are done
#pragma unroll
      for (int q = 0; q < kGemmSub; ++q) gemm_store(g, c[q], As[q], Bs[q]);
      __syncthreads();
    }
  }
  // Bias-gradient partial column sums over this part's K range (dW products:
  // the workgroups of the first tile row).  Thread t sums rows
  // kbeg + (t >> 6) + 4 i of column n0 + (t & 63) into four interleaved
  // accumulators (independent loads in flight); the four row groups are then
  // added in a fixed order.
  if (EPI == kPlain && g.colsum && blockIdx.y == 0) {  // uniform across the workgroup
    __shared__ float cs[4][64];
    const int col = t & 63, rg = t >> 6;
    const int n = n0 + col;
    float a[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    if (n < g.N) {
      int k = kbeg + rg;
      for (; k + 12 < kend; k += 16) {
#pragma unroll
        for (int q = 0; q < 4; ++q) a[q] += g.colsum[(size_t)(k + 4 * q) * g.N + n];
      }
      for (int q = 0; k < kend; k += 4, ++q) a[q & 3] += g.colsum[(size_t)k * g.N + n];
    }
    cs[rg][col] = (a[0] + a[1]) + (a[2] + a[3]);
    __syncthreads();
    if (t < 64 && n0 + t < g.N)
      g.part_cs[(size_t)blockIdx.z * g.N + n0 + t] = (cs[0][t] + cs[1][t]) + (cs[2][t] + cs[3][t]);
  }
  // D fragment: lane holds column (lane & 15), rows (lane >> 4) * 4 + r.  The
  // transposed BF16 copy (when asked for) takes the lane's four rows of one
  // column as one 8-byte store.
  float* dst = (EPI == kPlain && g.part) ? g.part + (size_t)blockIdx.z * g.M * g.N : nullptr;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int mb = m0 + wm * 32 + i * 16 + (lane >> 4) * 4;
      const int n = n0 + wn * 32 + j * 16 + (lane & 15);
      uint16_t hb[4] = {0, 0, 0, 0};
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = mb + r;
        if (m >= g.M || n >= g.N) continue;
        float v = acc[i][j][r];
        const size_t o = (size_t)m * g.N + n;
        if (dst) {
          dst[o] = v;
        } else if (EPI == kGelu) {
          v += g.bias[n];
          if (g.out_f32) g.out_f32[o] = v;
          hb[r] = f2bf(gelu_f(v));
          g.out_bf16[o] = hb[r];
        } else if (EPI == kLinear) {
          v += g.bias[n];
          if (g.out_f32) g.out_f32[o] = v;
          hb[r] = f2bf(v);
          if (g.out_bf16) g.out_bf16[o] = hb[r];
        } else if (EPI == kGeluBack) {
          v *= gelu_grad_f(g.zin[o]);
          if (g.out_f32) g.out_f32[o] = v;
          hb[r] = f2bf(v);
          g.out_bf16[o] = hb[r];
        } else {
          if (g.out_f32) g.out_f32[o] = v;
          hb[r] = f2bf(v);
          if (g.out_bf16) g.out_bf16[o] = hb[r];
        }
      }
      if (!dst && g.out_bf16_t && n < g.N) {
        uint16_t* tp = g.out_bf16_t + (size_t)n * g.ldt + mb;
        if (g.vec_t && mb + 3 < g.M) {
          *reinterpret_cast<uint2*>(tp) =
              make_uint2((uint32_t)hb[0] | ((uint32_t)hb[1] << 16), (uint32_t)hb[2] | ((uint32_t)hb[3] << 16));
        } else {
#pragma unroll
          for (int r = 0; r < 4; ++r)
            if (mb + r < g.M) tp[r] = hb[r];
        }
      }
    }
}

// Split-K reduction: out[e] = sum over parts z (in order) of part[z][e],
// e < M N; then cs_out[n] = sum over z of part_cs[z][n] when cs_out is set.
__global__ void splitk_reduce_kernel(const float* __restrict__ part, int parts, int MN, float* __restrict__ out,
                                     const float* __restrict__ part_cs, int N, float* __restrict__ cs_out) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < MN) {
    float s = 0.0f;
    for (int z = 0; z < parts; ++z) s += part[(size_t)z * MN + e];
    out[e] = s;
  } else if (cs_out && e < MN + N) {
    const int n = e - MN;
    float s = 0.0f;
    for (int z = 0; z < parts; ++z) s += part_cs[(size_t)z * N + n];
    cs_out[n] = s;
  }
}

// Launches op(A) op(B) in `splits` parts of the K range (rounded to 32-row
// steps; *parts_out receives the number of parts launched).
template <int EPI>
static hipError_t gemm(GemmArgs g, hipStream_t st, int splits = 1, int* parts_out = nullptr) {
  g.vec_a = g.lda % 8 == 0 && ((uintptr_t)g.A & 15) == 0;
  g.vec_b = g.ldb % 8 == 0 && ((uintptr_t)g.B & 15) == 0;
  g.vec_t = g.ldt % 4 == 0 && ((uintptr_t)g.out_bf16_t & 7) == 0;
  if (splits < 1) splits = 1;
  g.ksplit = (((g.K + splits - 1) / splits) + 31) / 32 * 32;
  splits = (g.K + g.ksplit - 1) / g.ksplit;
  if (parts_out) *parts_out = splits;
  dim3 grid((g.N + 63) / 64, (g.M + 63) / 64, splits);
  gemm_bf16_kernel<EPI><<<grid, 256, 0, st>>>(g);
  return hipGetLastError();
}

// Standardised inputs, BF16: X [B][8] -> H0 [B][8], and H0T [8][B] when set.
__global__ void mlp_input_kernel(const float* __restrict__ X, const float* __restrict__ mean,
                                 const float* __restrict__ stdv, int B, uint16_t* __restrict__ H0,
                                 uint16_t* __restrict__ H0T) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= B * kMlpIn) return;
  const int j = e % kMlpIn;
  const uint16_t h = f2bf((X[e] - mean[j]) / stdv[j]);
  H0[e] = h;
  if (H0T) H0T[(size_t)j * B + e / kMlpIn] = h;
}

// The weights of every layer transposed: W_l [din][dout] -> Wt_l [dout][din],
// at the same offsets of the flat vector (the forward product's B operand
// then runs along k).  One thread per parameter; biases are skipped.
__global__ void mlp_weights_t_kernel(const uint16_t* __restrict__ w16, uint16_t* __restrict__ w16t) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int dims[5] = {kMlpIn, kMlpHid, kMlpHid, kMlpHid, kMlpOut};
  int o = 0;
#pragma unroll
  for (int l = 0; l < 4; ++l) {
    const int din = dims[l], dout = dims[l + 1], nw = din * dout;
    if (e >= o && e < o + nw) {
      const int k = (e - o) / dout, n = (e - o) % dout;
      w16t[o + n * din + k] = w16[e];
    }
    o += nw + dout;
  }
}

// Mixture negative log-likelihood of targets T [B][2] under heads Y [B][80]:
// per-sample NLL (FP32) and dNLL/dY / B as FP32 and BF16 ([B][80], and the
// BF16 values again as [80][B]).  One lane per (sample, component): the 16
// lanes of a sample form the two log-sum-exps by shuffles within their group
// (a wave holds four samples), so a sample's work is 16 lanes wide instead of
// a loop over its components.
__device__ __forceinline__ float group16_max(float v) {
#pragma unroll
  for (int o = 8; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 16));
  return v;
}
__device__ __forceinline__ float group16_sum(float v) {
#pragma unroll
  for (int o = 8; o > 0; o >>= 1) v += __shfl_xor(v, o, 16);
  return v;
}

__global__ void __launch_bounds__(256)
mdn_loss_kernel(const float* __restrict__ Y, const float* __restrict__ T, int B, float* __restrict__ nll,
                float* __restrict__ dY32, uint16_t* __restrict__ dY16, uint16_t* __restrict__ dY16T,
                float* __restrict__ loss_sum) {
  static_assert(kMlpComp == 16, "one 16-lane group per sample");
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  const int b = gid >> 4, k = gid & 15;
  const bool valid = b < B;  // uniform across each 16-lane group
  const int bb = valid ? b : 0;
  const float* y = Y + (size_t)bb * kMlpOut + 5 * k;
  const float logit = y[0];
  const float lse_logit = [&] {
    const float lmax = group16_max(logit);
    return lmax + logf(group16_sum(expf(logit - lmax)));
  }();
  const float t0 = T[2 * bb], t1 = T[2 * bb + 1];
  const float r0 = y[3], r1 = y[4];
  const float l0 = fminf(fmaxf(r0, kLogSigMin), kLogSigMax);
  const float l1 = fminf(fmaxf(r1, kLogSigMin), kLogSigMax);
  const float is0 = expf(-l0), is1 = expf(-l1);
  const float d0 = (t0 - y[1]) * is0;
  const float d1 = (t1 - y[2]) * is1;
  const float lp = logit - lse_logit;
  const float a = lp - (0.5f * (d0 * d0 + d1 * d1) + l0 + l1 + kLog2Pi);
  const float amax = group16_max(a);
  const float lse = amax + logf(group16_sum(expf(a - amax)));
  const float contrib = (valid && k == 0) ? -lse : 0.0f;
  if (valid) {
    if (k == 0) nll[b] = -lse;
    const float inv_b = 1.0f / (float)B;
    const float gam = expf(a - lse);
    const float pi = expf(lp);
    float gk[5];
    gk[0] = pi - gam;
    gk[1] = -gam * d0 * is0;
    gk[2] = -gam * d1 * is1;
    gk[3] = (r0 > kLogSigMin && r0 < kLogSigMax) ? gam * (1.0f - d0 * d0) : 0.0f;
    gk[4] = (r1 > kLogSigMin && r1 < kLogSigMax) ? gam * (1.0f - d1 * d1) : 0.0f;
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      const float v = gk[q] * inv_b;
      const uint16_t h = f2bf(v);
      dY32[(size_t)b * kMlpOut + 5 * k + q] = v;
      dY16[(size_t)b * kMlpOut + 5 * k + q] = h;
      dY16T[(size_t)(5 * k + q) * B + b] = h;  // [80][B]: the dW product's B operand
    }
  }
  // Workgroup sum of the NLL, one atomic per workgroup (reported loss only).
  __shared__ float red[256];
  red[threadIdx.x] = contrib;
  __syncthreads();
  for (int st = blockDim.x / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0 && loss_sum) atomicAdd(loss_sum, red[0] / (float)B);
}

// Adam (Kingma & Ba 2015) with bias correction on the FP32 master weights,
// refreshing the BF16 copy used by the products.
__global__ void adam_kernel(float* __restrict__ w, uint16_t* __restrict__ w16, float* __restrict__ mom,
                            float* __restrict__ vel, const float* __restrict__ grad, int n, float lr, float b1,
                            float b2, float omb1, float omb2, float eps, float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float g = grad[i];
  const float m = b1 * mom[i] + omb1 * g;
  const float v = b2 * vel[i] + omb2 * g * g;
  mom[i] = m;
  vel[i] = v;
  const float wi = w[i] - lr * (m / c1) / (sqrtf(v / c2) + eps);
  w[i] = wi;
  w16[i] = f2bf(wi);
}

// The mixture of one head in the form the draws use, built once per
// workgroup in LDS: cdf[k] = (sum_{i<=k} e_i) / (sum_i e_i) with e_i =
// exp(logit_i - max logit), summed in component order, and sig = exp of the
// clamped log sigmas.
struct MdnTable {
  float e[kMlpComp], w[kMlpComp], cdf[kMlpComp], sig[kMlpComp][2], acc;
};

// Called by every thread of the workgroup (three barriers); head is readable
// by all of them.
__device__ __forceinline__ void mdn_table_build(const float* head, MdnTable* t) {
  const int j = threadIdx.x;
  if (j < kMlpComp) {
    float lmax = -INFINITY;
    for (int k = 0; k < kMlpComp; ++k) lmax = fmaxf(lmax, head[5 * k]);
    t->e[j] = expf(head[5 * j] - lmax);
  } else if (j < 3 * kMlpComp) {
    const int k = (j - kMlpComp) >> 1, q = (j - kMlpComp) & 1;
    t->sig[k][q] = expf(fminf(fmaxf(head[5 * k + 3 + q], kLogSigMin), kLogSigMax));
  }
  __syncthreads();
  if (j == 0) {
    float acc = 0.0f;
    for (int k = 0; k < kMlpComp; ++k) {
      acc += t->e[k];
      t->w[k] = acc;
    }
    t->acc = acc;
  }
  __syncthreads();
  if (j < kMlpComp) t->cdf[j] = t->w[j] / t->acc;
  __syncthreads();
}

// Proposal p: component by inverse CDF at r0, Box-Muller normals from r1,
// r2, mu + sigma z clipped to [-1, 1], mapped to the input box.  Writes cand
// [1][m][P] (EXPLICIT layout, m = 2).
__device__ __forceinline__ void mdn_draw(const ModelDev* __restrict__ md, const float* head, const MdnTable* t,
                                         int P, int p, uint64_t seed, uint64_t tick, int loop,
                                         float* __restrict__ cand) {
  const uint64_t pre = hash_prefix(seed, tick, (uint64_t)(uint32_t)loop, (uint64_t)p);
  const uint64_t h0 = hash_finish(pre, 0), h1 = hash_finish(pre, 1), h2 = hash_finish(pre, 2);
  const float r0 = (float)((double)(h0 >> 40) * 0x1p-24);
  int kc = 0;
#pragma unroll
  for (int k = 0; k < kMlpComp; ++k) kc += (t->cdf[k] <= r0) ? 1 : 0;
  kc = kc < kMlpComp ? kc : kMlpComp - 1;
  const float r1 = (float)(((double)(h1 >> 40) + 1.0) * 0x1p-24);
  const float r2 = (float)((double)(h2 >> 40) * 0x1p-24);
  const float rad = sqrtf(-2.0f * logf(r1));
  float sn, cs;
  sincosf(6.283185307179586f * r2, &sn, &cs);
  const float z[2] = {rad * cs, rad * sn};
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    float un = fmaf(t->sig[kc][j], z[j], head[5 * kc + 1 + j]);
    un = fminf(fmaxf(un, -1.0f), 1.0f);
    const float lo = md->sys.u_lo[j], hi = md->sys.u_hi[j];
    cand[(size_t)j * P + p] = fmaf(0.5f * (hi - lo), un, 0.5f * (lo + hi));
  }
}

__global__ void __launch_bounds__(256)
mdn_sample_kernel(const ModelDev* __restrict__ md, const float* __restrict__ Yrow, int P, uint64_t seed,
                  uint64_t tick, int loop, float* __restrict__ cand) {
  __shared__ MdnTable tab;
  mdn_table_build(Yrow, &tab);
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < P) mdn_draw(md, Yrow, &tab, P, p, seed, tick, loop, cand);
}

// Offsets of (W_l, b_l) in the flat parameter vector (per layer W[in][out]
// then b[out]), as plain constants: device code must not call a recursive
// function (it would need a call stack of unbounded depth).
constexpr size_t kMlpW0 = 0;
constexpr size_t kMlpB0 = kMlpW0 + (size_t)kMlpIn * kMlpHid;
constexpr size_t kMlpW1 = kMlpB0 + kMlpHid;
constexpr size_t kMlpB1 = kMlpW1 + (size_t)kMlpHid * kMlpHid;
constexpr size_t kMlpW2 = kMlpB1 + kMlpHid;
constexpr size_t kMlpB2 = kMlpW2 + (size_t)kMlpHid * kMlpHid;
constexpr size_t kMlpW3 = kMlpB2 + kMlpHid;
constexpr size_t kMlpB3 = kMlpW3 + (size_t)kMlpHid * kMlpOut;
static_assert(kMlpB3 + kMlpOut == MPMI_MLP_PARAMS, "parameter layout");

// Forward pass of the one row [x_t; u_user] in a workgroup of 1,024
// threads, then draws from its head: each of the launch's workgroups runs the
// same forward (bit-identical; workgroup 0 stores the head) and draws its
// share of the P proposals, kRowDraws per workgroup and pass.  The arithmetic rules are the
// batched path's (standardised input and activations rounded to BF16, BF16
// weights, FP32 accumulation, FP32 bias added last).  In a layer of DIN
// inputs and DOUT units, thread t takes units [8g, 8g + 8) (g = t % (DOUT/8))
// over inputs [8s, 8s + 8) (s = t / (DOUT/8)): eight 16-byte weight loads and
// 64 FMAs; its eight partial sums go to LDS, where one thread per unit adds
// the DIN/8 partials in order.  Each layer's weight loads are issued before
// the previous layer's reduction, so their latency overlaps it.  A serving
// tick needs one row, for which a GEMM tile per layer is mostly idle.
constexpr int kRowThreads = 1024;
constexpr int kRowDraws = 256;
constexpr int kRowMaxGroups = 64;

// Workgroup barrier over LDS only: waits for this wave's LDS accesses, not
// for its global loads (__syncthreads' fence also drains the vector-memory
// counter, which would retire the next layer's weight prefetch at once).
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

template <int DIN, int DOUT>
struct RowSlice {
  static constexpr int G = DOUT / 8, S = DIN / 8;
  static_assert(DOUT % 8 == 0 && DIN % 8 == 0 && G * S <= kRowThreads, "row layer shape");
  uint4 w[8];
  __device__ __forceinline__ bool active() const { return (int)threadIdx.x < G * S; }
  __device__ __forceinline__ void load(const uint16_t* __restrict__ W) {
    if (!active()) return;
    const int g = threadIdx.x % G, sl = threadIdx.x / G;
#pragma unroll
    for (int r = 0; r < 8; ++r) w[r] = *reinterpret_cast<const uint4*>(W + (size_t)(8 * sl + r) * DOUT + 8 * g);
  }
  // red[s][DOUT]: this thread's eight partial sums.
  __device__ __forceinline__ void partial(const float* hin, float* red) const {
    if (!active()) return;
    const int g = threadIdx.x % G, sl = threadIdx.x / G;
    float acc[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) acc[u] = 0.0f;
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const float h = hin[8 * sl + r];
      const uint32_t q[4] = {w[r].x, w[r].y, w[r].z, w[r].w};
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        acc[2 * u] = fmaf(h, __uint_as_float(q[u] << 16), acc[2 * u]);
        acc[2 * u + 1] = fmaf(h, __uint_as_float(q[u] & 0xffff0000u), acc[2 * u + 1]);
      }
    }
    float4* dst = reinterpret_cast<float4*>(red + (size_t)sl * DOUT + 8 * g);
    dst[0] = make_float4(acc[0], acc[1], acc[2], acc[3]);
    dst[1] = make_float4(acc[4], acc[5], acc[6], acc[7]);
  }
};

// Unit j's pre-activation: the DIN/8 partials in order, then the bias.
template <int DIN, int DOUT>
__device__ __forceinline__ float row_unit(const float* red, float bias, int j) {
  float v = 0.0f;
#pragma unroll 8
  for (int sl = 0; sl < DIN / 8; ++sl) v += red[sl * DOUT + j];
  return v + bias;
}

__global__ void __launch_bounds__(kRowThreads)
mlp_row_forward_kernel(const float* __restrict__ x_t, const float* __restrict__ u_user,
                       const uint16_t* __restrict__ w16, const float* __restrict__ w32,
                       const float* __restrict__ mean, const float* __restrict__ stdv,
                       float* __restrict__ Y, const ModelDev* __restrict__ md, int P, uint64_t seed,
                       uint64_t tick, int loop, float* __restrict__ cand) {
  __shared__ __attribute__((aligned(16))) float red[(kMlpHid / 8) * kMlpHid];
  __shared__ __attribute__((aligned(16))) float bufA[kMlpHid], bufB[kMlpHid], head[kMlpOut];
  const int j = threadIdx.x;
  // Global loads in the order they are consumed (the vector-memory counter
  // retires loads in issue order): input row and biases, then the weights of
  // layers 0 and 1; layer l + 2's weights are issued before layer l + 1's
  // products.
  float xin = 0.0f, b0 = 0.0f, b1 = 0.0f, b2 = 0.0f, b3 = 0.0f;
  float xm = 0.0f, xs = 1.0f;
  if (j < kMlpIn) {
    xin = j < 6 ? x_t[j] : u_user[j - 6];
    xm = mean[j];
    xs = stdv[j];
  }
  if (j < kMlpHid) {
    b0 = w32[kMlpB0 + j];
    b1 = w32[kMlpB1 + j];
    b2 = w32[kMlpB2 + j];
  }
  if (j < kMlpOut) b3 = w32[kMlpB3 + j];
  RowSlice<kMlpIn, kMlpHid> s0;
  RowSlice<kMlpHid, kMlpHid> s1;
  s0.load(w16 + kMlpW0);
  s1.load(w16 + kMlpW1);
  if (j < kMlpIn) bufA[j] = bf2f(f2bf((xin - xm) / xs));
  lds_barrier();
  s0.partial(bufA, red);
  lds_barrier();
  if (j < kMlpHid) bufB[j] = bf2f(f2bf(gelu_f(row_unit<kMlpIn, kMlpHid>(red, b0, j))));
  lds_barrier();
  RowSlice<kMlpHid, kMlpHid> s2;
  s2.load(w16 + kMlpW2);
  s1.partial(bufB, red);
  lds_barrier();
  if (j < kMlpHid) bufA[j] = bf2f(f2bf(gelu_f(row_unit<kMlpHid, kMlpHid>(red, b1, j))));
  lds_barrier();
  RowSlice<kMlpHid, kMlpOut> s3;
  s3.load(w16 + kMlpW3);
  s2.partial(bufA, red);
  lds_barrier();
  if (j < kMlpHid) bufB[j] = bf2f(f2bf(gelu_f(row_unit<kMlpHid, kMlpHid>(red, b2, j))));
  lds_barrier();
  s3.partial(bufB, red);
  lds_barrier();
  if (j < kMlpOut) {
    const float v = row_unit<kMlpHid, kMlpOut>(red, b3, j);
    head[j] = v;
    if (blockIdx.x == 0) Y[j] = v;
  }
  if (P <= 0) return;
  __shared__ MdnTable tab;
  lds_barrier();
  mdn_table_build(head, &tab);
  for (int p = blockIdx.x * kRowDraws + j; j < kRowDraws && p < P; p += gridDim.x * kRowDraws)
    mdn_draw(md, head, &tab, P, p, seed, tick, loop, cand);
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------
static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Split-K parts of the weight-gradient products (batch rows split into at
// most kMlpSplits ranges of at least kMlpSplitRows rows): batch 4,096 runs 16
// parts, 256 workgroups for a 256 x 256 product; batch 16,384 and more run 64
// parts (1,024 workgroups), each part a chain of at most B / 2,048 k-steps.
constexpr int kMlpSplits = 64, kMlpSplitRows = 256;

// Activations and their gradients are kept batch-major ([B][width]) for the
// forward products and the dX products, and batch-minor ([width][B], the "T"
// copies, written by the same epilogues) for the weight-gradient products,
// whose contraction runs over the batch: every product then stages operands
// whose k index is contiguous in memory.
struct MlpWork {
  uint16_t *h0, *h1, *h2, *h3, *dY16, *dz16;
  uint16_t *w16t, *h0T, *h1T, *h2T, *h3T, *dY16T, *dz16T;
  float *z1, *z2, *z3, *Y, *dY32, *dz32, *nll, *loss, *row, *part, *part_cs;
};

static MlpWork carve(void* base, int B) {
  char* p = (char*)base;
  MlpWork w;
  auto take = [&](size_t bytes) { char* r = p; p += align256(bytes); return (void*)r; };
  w.h0 = (uint16_t*)take((size_t)B * kMlpIn * 2);
  w.h1 = (uint16_t*)take((size_t)B * kMlpHid * 2);
  w.h2 = (uint16_t*)take((size_t)B * kMlpHid * 2);
  w.h3 = (uint16_t*)take((size_t)B * kMlpHid * 2);
  w.dY16 = (uint16_t*)take((size_t)B * kMlpOut * 2);
  w.dz16 = (uint16_t*)take((size_t)B * kMlpHid * 2 * 2);  // two ping-pong halves
  w.w16t = (uint16_t*)take((size_t)kMlpParams * 2);
  w.h0T = (uint16_t*)take((size_t)B * kMlpIn * 2);
  w.h1T = (uint16_t*)take((size_t)B * kMlpHid * 2);
  w.h2T = (uint16_t*)take((size_t)B * kMlpHid * 2);
  w.h3T = (uint16_t*)take((size_t)B * kMlpHid * 2);
  w.dY16T = (uint16_t*)take((size_t)B * kMlpOut * 2);
  w.dz16T = (uint16_t*)take((size_t)B * kMlpHid * 2 * 2);
  w.z1 = (float*)take((size_t)B * kMlpHid * 4);
  w.z2 = (float*)take((size_t)B * kMlpHid * 4);
  w.z3 = (float*)take((size_t)B * kMlpHid * 4);
  w.Y = (float*)take((size_t)B * kMlpOut * 4);
  w.dY32 = (float*)take((size_t)B * kMlpOut * 4);
  w.dz32 = (float*)take((size_t)B * kMlpHid * 4 * 2);
  w.nll = (float*)take((size_t)B * 4);
  w.loss = (float*)take(4);
  w.row = (float*)take(kMlpIn * 4);
  w.part = (float*)take((size_t)kMlpSplits * kMlpHid * kMlpHid * 4);
  w.part_cs = (float*)take((size_t)kMlpSplits * kMlpHid * 4);
  return w;
}

size_t mlp_workspace_bytes(int B) {
  char* base = nullptr;
  MlpWork w = carve((void*)base, B);
  return (size_t)((char*)w.part_cs - base) + align256((size_t)kMlpSplits * kMlpHid * 4);
}

// Offsets of (W_l, b_l) in the flat parameter vector.
static void layer_offsets(size_t* ow, size_t* ob) {
  const int dims[5] = {kMlpIn, kMlpHid, kMlpHid, kMlpHid, kMlpOut};
  size_t o = 0;
  for (int l = 0; l < 4; ++l) {
    ow[l] = o;
    o += (size_t)dims[l] * dims[l + 1];
    ob[l] = o;
    o += dims[l + 1];
  }
}

// The forward products read the transposed weights (w.w16t, formed first);
// with `with_t` the hidden activations are also written batch-minor.
static hipError_t forward_into(const uint16_t* w16, const float* bias32, const float* mean, const float* stdv,
                               const float* X, int B, const MlpWork& w, float* Y, bool with_t, hipStream_t st) {
  size_t ow[4], ob[4];
  layer_offsets(ow, ob);
  mlp_weights_t_kernel<<<(kMlpParams + 255) / 256, 256, 0, st>>>(w16, w.w16t);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  mlp_input_kernel<<<(B * kMlpIn + 255) / 256, 256, 0, st>>>(X, mean, stdv, B, w.h0, with_t ? w.h0T : nullptr);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const uint16_t* hin[4] = {w.h0, w.h1, w.h2, w.h3};
  uint16_t* hout[3] = {w.h1, w.h2, w.h3};
  uint16_t* hout_t[3] = {w.h1T, w.h2T, w.h3T};
  float* zout[3] = {w.z1, w.z2, w.z3};
  const int din[4] = {kMlpIn, kMlpHid, kMlpHid, kMlpHid};
  for (int l = 0; l < 3; ++l) {
    GemmArgs g{};
    g.A = hin[l]; g.B = w.w16t + ow[l]; g.tb = 1; g.M = B; g.N = kMlpHid; g.K = din[l];
    g.lda = din[l]; g.ldb = din[l]; g.bias = bias32 + ob[l]; g.out_f32 = zout[l]; g.out_bf16 = hout[l];
    if (with_t) {
      g.out_bf16_t = hout_t[l];
      g.ldt = B;
    }
    if ((e = gemm<kGelu>(g, st)) != hipSuccess) return e;
  }
  GemmArgs g{};
  g.A = w.h3; g.B = w.w16t + ow[3]; g.tb = 1; g.M = B; g.N = kMlpOut; g.K = kMlpHid;
  g.lda = kMlpHid; g.ldb = kMlpHid; g.bias = bias32 + ob[3]; g.out_f32 = Y;
  return gemm<kLinear>(g, st);
}

// Biases are kept in FP32 (they add to FP32 accumulators): the FP32 master
// vector is passed alongside the BF16 weights.
hipError_t launch_mlp_forward(const uint16_t* w16, const float* w32, const float* mean, const float* stdv,
                              const float* X, int B, float* Y, void* work, hipStream_t st) {
  const MlpWork w = carve(work, B);
  return forward_into(w16, w32, mean, stdv, X, B, w, Y, false, st);
}

hipError_t launch_mlp_grad(const uint16_t* w16, const float* w32, const float* mean, const float* stdv,
                           const float* X, const float* T, int B, float* grad, float* loss, void* work,
                           hipStream_t st) {
  const MlpWork w = carve(work, B);
  hipError_t e = hipMemsetAsync(w.loss, 0, sizeof(float), st);
  if (e != hipSuccess) return e;
  if ((e = forward_into(w16, w32, mean, stdv, X, B, w, w.Y, true, st)) != hipSuccess) return e;
  mdn_loss_kernel<<<(B * kMlpComp + 255) / 256, 256, 0, st>>>(w.Y, T, B, w.nll, w.dY32, w.dY16, w.dY16T, w.loss);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  size_t ow[4], ob[4];
  layer_offsets(ow, ob);
  const int dims[5] = {kMlpIn, kMlpHid, kMlpHid, kMlpHid, kMlpOut};
  const uint16_t* hin_t[4] = {w.h0T, w.h1T, w.h2T, w.h3T};
  const float* zin[4] = {nullptr, w.z1, w.z2, w.z3};
  // dz of the current layer (output width dims[l+1]): FP32 for bias sums,
  // BF16 as operand, batch-major and batch-minor.
  const float* dz32 = w.dY32;
  const uint16_t* dz16 = w.dY16;
  const uint16_t* dz16t = w.dY16T;
  for (int l = 3; l >= 0; --l) {
    const int kin = dims[l], nout = dims[l + 1];
    // dW_l = h_{l-1}^T dz  ([kin][nout]) from the batch-minor copies
    // (h^T [kin][B] as A, dz^T [nout][B] as the transposed B), split over the
    // batch, with the bias gradient db_l = column sums of dz (FP32) in the
    // same parts; both reduced over the parts in order.
    GemmArgs gw{};
    gw.A = hin_t[l]; gw.lda = B;
    gw.B = dz16t; gw.tb = 1; gw.ldb = B;
    gw.M = kin; gw.N = nout; gw.K = B;
    gw.part = w.part; gw.colsum = dz32; gw.part_cs = w.part_cs;
    int splits = B / kMlpSplitRows;
    splits = splits < 1 ? 1 : (splits > kMlpSplits ? kMlpSplits : splits);
    int parts = 1;
    if ((e = gemm<kPlain>(gw, st, splits, &parts)) != hipSuccess) return e;
    splitk_reduce_kernel<<<(kin * nout + nout + 255) / 256, 256, 0, st>>>(w.part, parts, kin * nout, grad + ow[l],
                                                                          w.part_cs, nout, grad + ob[l]);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (l == 0) break;
    // dz_{l-1} = (dz W_l^T) * gelu'(z_{l-1})  ([B][kin])
    const int half = (l % 2) * B * kMlpHid;
    GemmArgs gd{};
    gd.A = dz16; gd.lda = nout;
    gd.B = w16 + ow[l]; gd.tb = 1; gd.ldb = nout;
    gd.M = B; gd.N = kin; gd.K = nout;
    gd.zin = zin[l]; gd.out_f32 = w.dz32 + half; gd.out_bf16 = w.dz16 + half;
    gd.out_bf16_t = w.dz16T + half; gd.ldt = B;
    if ((e = gemm<kGeluBack>(gd, st)) != hipSuccess) return e;
    dz32 = w.dz32 + half;
    dz16 = w.dz16 + half;
    dz16t = w.dz16T + half;
  }
  if (loss) {
    e = hipMemcpyAsync(loss, w.loss, sizeof(float), hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_mlp_adam(float* w32, uint16_t* w16, float* m, float* v, const float* grad, int step, float lr,
                           hipStream_t st) {
  // Constants and their complements rounded once from FP64 (1 - 0.999f in
  // FP32 would carry a 1e-5 relative error into the second moment).
  const double b1 = 0.9, b2 = 0.999;
  const float c1 = (float)(1.0 - pow(b1, step)), c2 = (float)(1.0 - pow(b2, step));
  adam_kernel<<<(kMlpParams + 255) / 256, 256, 0, st>>>(w32, w16, m, v, grad, kMlpParams, lr, (float)b1, (float)b2,
                                                        (float)(1.0 - b1), (float)(1.0 - b2), 1e-8f, c1, c2);
  return hipGetLastError();
}

hipError_t launch_mdn_sample(const void* model, const float* Yrow, int P, uint64_t seed, uint64_t tick, int loop,
                             float* cand, hipStream_t st) {
  mdn_sample_kernel<<<(P + 255) / 256, 256, 0, st>>>((const ModelDev*)model, Yrow, P, seed, tick, loop, cand);
  return hipGetLastError();
}

hipError_t launch_mlp_row_forward(const float* x_t, const float* u_user, const uint16_t* w16, const float* w32,
                                  const float* mean, const float* stdv, void* work, float* head_out, float** head,
                                  const void* model, int P, uint64_t seed, uint64_t tick, int loop, float* cand,
                                  hipStream_t st) {
  const MlpWork w = carve(work, 1);
  *head = head_out ? head_out : w.Y;
  int groups = P > 0 ? (P + kRowDraws - 1) / kRowDraws : 1;
  groups = groups < kRowMaxGroups ? groups : kRowMaxGroups;
  mlp_row_forward_kernel<<<groups, kRowThreads, 0, st>>>(x_t, u_user, w16, w32, mean, stdv, *head,
                                                         (const ModelDev*)model, P, seed, tick, loop, cand);
  return hipGetLastError();
}

hipError_t launch_gemm_test(const uint16_t* A, const uint16_t* B, int M, int N, int K, int ta, int tb, float* C,
                            hipStream_t st) {
  GemmArgs g{};
  g.A = A; g.B = B; g.M = M; g.N = N; g.K = K; g.ta = ta; g.tb = tb;
  g.lda = ta ? M : K;
  g.ldb = tb ? K : N;
  g.out_f32 = C;
  return gemm<kPlain>(g, st);
}

}  // namespace mpmi
