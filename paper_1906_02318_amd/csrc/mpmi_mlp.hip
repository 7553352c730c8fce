// Learned proposal network: forward, mixture loss, backward, Adam and the
// mixture sampler, all hand-written for gfx950.
//
// Shape (fixed): 8 standardised inputs -> 256 -> 256 -> 256 -> 80, GELU (tanh
// form) on the hidden layers; the 80 outputs are 16 x {logit, mu_0, mu_1,
// log sigma_0, log sigma_1} of a diagonal-Gaussian mixture over the input
// normalised to [-1, 1]^2.  Weights are BF16 (FP32 master copy for Adam);
// every product accumulates in FP32.
//
// The dense products run on BF16 matrix cores (v_mfma_f32_16x16x32_bf16).
// The forward and the backward dX products run layer after layer inside two
// fused row-block kernels (activations in LDS).  The weight-gradient
// products, contractions over the batch, run as split-K tiles: a 256-thread
// workgroup computes a 64 x 64 tile of C = op(A) op(B), each wave a 32 x 32
// quarter as 2 x 2 MFMA blocks, with 64 x 32 slices of A and B staged through
// LDS per k-step (transposed operands are transposed while staging).
#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>

#include <algorithm>

#include "mpmi_device.hpp"
#include "mpmi_launch.hpp"

namespace mpmi {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

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
  float* out_f32;      // [M][N] (single part)
  // Split-K: gridDim.z parts of ksplit rows of K each write FP32 partial
  // products to part[z][M][N].
  int ksplit;
  float* part;
  bool vec_a, vec_b;   // 16-byte loads allowed (leading dimension a multiple of 8, 16-byte aligned base)
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

// One 64 x 64 output tile (bx, by) of K part bz; every thread of the
// workgroup calls it.
__device__ __forceinline__ void gemm_tile(const GemmArgs& g, int bx, int by, int bz) {
  __shared__ __attribute__((aligned(16))) uint16_t As[kGemmSub][64][kGemmKP];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[kGemmSub][64][kGemmKP];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int m0 = by * 64, n0 = bx * 64;
  const int kbeg = bz * g.ksplit;
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
  // D fragment: lane holds column (lane & 15), rows (lane >> 4) * 4 + r.
  float* dst = g.part ? g.part + (size_t)bz * g.M * g.N : g.out_f32;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int mb = m0 + wm * 32 + i * 16 + (lane >> 4) * 4;
      const int n = n0 + wn * 32 + j * 16 + (lane & 15);
#pragma unroll
      for (int r = 0; r < 4; ++r)
        if (mb + r < g.M && n < g.N) dst[(size_t)(mb + r) * g.N + n] = acc[i][j][r];
    }
}

__global__ void __launch_bounds__(256) gemm_bf16_kernel(GemmArgs g) { gemm_tile(g, blockIdx.x, blockIdx.y, blockIdx.z); }

// Several independent products in one launch (the weight gradients of every
// layer): member i owns the grid's z range [zbase[i], zbase[i + 1]) as its
// K parts; the grid's x and y cover the largest member, and a workgroup past
// its member's tiles returns at once.
constexpr int kGemmGroupMax = 4;
struct GemmGroup {
  GemmArgs g[kGemmGroupMax];
  int zbase[kGemmGroupMax + 1];
  int n;
};

__global__ void __launch_bounds__(256) gemm_group_kernel(GemmGroup gg) {
  int i = 0;
  while (i + 1 < gg.n && (int)blockIdx.z >= gg.zbase[i + 1]) ++i;  // uniform
  const GemmArgs& g = gg.g[i];
  if ((int)blockIdx.x * 64 >= g.N || (int)blockIdx.y * 64 >= g.M) return;  // uniform
  gemm_tile(g, blockIdx.x, blockIdx.y, blockIdx.z - gg.zbase[i]);
}

// The split-K reductions of a GemmGroup in one launch.  The grid's first
// wblocks workgroups take the weight elements, one thread each: member i
// owns elements [wbase[i], wbase[i + 1]), out[e] = sum over parts z, in
// order, of part[z][e].  The rest take the bias columns, one wave each:
// member i owns columns [cbase[i], cbase[i + 1]), cs_out[n] = sum over row
// blocks r of cs_part[r cs_ld + n], lane l summing blocks l, l + 64, ... in
// order and the lanes then combined by a fixed butterfly.
struct ReduceGroup {
  const float* part[kGemmGroupMax];
  const float* cs_part[kGemmGroupMax];
  float* out[kGemmGroupMax];
  float* cs_out[kGemmGroupMax];
  int parts[kGemmGroupMax], cs_parts[kGemmGroupMax], cs_ld[kGemmGroupMax];
  int wbase[kGemmGroupMax + 1], cbase[kGemmGroupMax + 1];
  int wblocks, n;
};

__global__ void __launch_bounds__(256) splitk_reduce_group_kernel(ReduceGroup rg) {
  if ((int)blockIdx.x < rg.wblocks) {
    const int e0 = blockIdx.x * blockDim.x + threadIdx.x;
    if (e0 >= rg.wbase[rg.n]) return;
    int i = 0;
    while (i + 1 < rg.n && e0 >= rg.wbase[i + 1]) ++i;
    const int e = e0 - rg.wbase[i], MN = rg.wbase[i + 1] - rg.wbase[i], parts = rg.parts[i];
    float s = 0.0f;
    for (int z = 0; z < parts; ++z) s += rg.part[i][(size_t)z * MN + e];
    rg.out[i][e] = s;
    return;
  }
  const int c0 = ((int)blockIdx.x - rg.wblocks) * 4 + (int)(threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (c0 >= rg.cbase[rg.n]) return;  // uniform per wave
  int i = 0;
  while (i + 1 < rg.n && c0 >= rg.cbase[i + 1]) ++i;
  const int n = c0 - rg.cbase[i], ld = rg.cs_ld[i], cp = rg.cs_parts[i];
  float s = 0.0f;
  for (int r = lane; r < cp; r += 64) s += rg.cs_part[i][(size_t)r * ld + n];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if (lane == 0) rg.cs_out[i][n] = s;
}

// Sets a product's derived fields (16-byte load flags, K part size for
// `splits` parts rounded to 32-row steps) and returns the number of parts.
static int gemm_prepare(GemmArgs& g, int splits) {
  g.vec_a = g.lda % 8 == 0 && ((uintptr_t)g.A & 15) == 0;
  g.vec_b = g.ldb % 8 == 0 && ((uintptr_t)g.B & 15) == 0;
  if (splits < 1) splits = 1;
  g.ksplit = (((g.K + splits - 1) / splits) + 31) / 32 * 32;
  return (g.K + g.ksplit - 1) / g.ksplit;
}

// Launches op(A) op(B) in `splits` parts of the K range (rounded to 32-row
// steps; *parts_out receives the number of parts launched).
static hipError_t gemm(GemmArgs g, hipStream_t st, int splits = 1, int* parts_out = nullptr) {
  splits = gemm_prepare(g, splits);
  if (parts_out) *parts_out = splits;
  dim3 grid((g.N + 63) / 64, (g.M + 63) / 64, splits);
  gemm_bf16_kernel<<<grid, 256, 0, st>>>(g);
  return hipGetLastError();
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

// Max and sum over a 16-lane group (one sample's mixture components).
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

// ---------------------------------------------------------------------------
// Fused row-block passes of the training step.  A workgroup owns a block of
// 16 or 32 batch rows and takes them through every layer with the
// activations in LDS, so a pass is one launch instead of a launch per layer:
// the forward (inputs standardised, three GELU layers, the linear head) and
// the backward (the mixture loss, then the three dX products with GELU').
// Each product is the block's activations [rows x K] (BF16, LDS) times B
// (K x N) on v_mfma_f32_16x16x32_bf16, B read from global memory (L2) as
// 8-value k-chunks straight into the operand registers, wave w of the 16
// taking the output column tile w (16 columns); per output tile the k-steps
// run in the order the one-product kernel uses, so results equal the
// layer-by-layer products.  The weight-gradient products (a contraction over
// the batch) stay separate.
// ---------------------------------------------------------------------------
// Block height: 16 rows while the batch has too few 32-row blocks to fill
// the chip (twice the workgroups, each half the serial work), 32 above (half
// the weight reads from L2).
__host__ __device__ constexpr int fuse_rows(int B) { return B < 16384 ? 16 : 32; }
constexpr int kFuseLd = 264;  // LDS row stride in BF16: 256 + 8, rows 16 B apart in bank order
constexpr int kFuseWaves = 16;  // one 16-column output tile per wave for the 256-wide layers
constexpr int kFuseThreads = 64 * kFuseWaves;

// acc[i][jt] = A[16 i .. 16 i + 15][0 .. K) B[0 .. K)[tile j = wave + 16 jt],
// Bk(n, k) at W[n * ldw + k] (k-chunks of 8 with k + 8 <= K or k >= K, zero
// past K); tiles j >= NT are skipped.  A's columns [K, K rounded up to 32)
// must hold zeros.  Every B chunk of the product is loaded before the first
// MFMA (one memory round trip per layer; the registers are there, a pass
// runs few waves per SIMD), then the k-steps run in order.
template <int RT, int K, int NTW>
__device__ __forceinline__ void rowblock_product(const uint16_t (*A)[kFuseLd], const uint16_t* __restrict__ W,
                                                 int ldw, int NT, f32x4_t (&acc)[RT][NTW]) {
  constexpr int KS = (K + 31) / 32;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int kq = (lane >> 4) * 8;
  uint4 bv[KS][NTW];
#pragma unroll
  for (int ks = 0; ks < KS; ++ks)
#pragma unroll
    for (int jt = 0; jt < NTW; ++jt) {
      const int j = wave + kFuseWaves * jt, k = ks * 32 + kq;
      const int n = j * 16 + (lane & 15);
      bv[ks][jt] = (j < NT && k < K) ? *reinterpret_cast<const uint4*>(W + (size_t)n * ldw + k)
                                     : make_uint4(0u, 0u, 0u, 0u);
    }
#pragma unroll
  for (int i = 0; i < RT; ++i)
#pragma unroll
    for (int jt = 0; jt < NTW; ++jt) acc[i][jt] = f32x4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) {
    bf16x8_t af[RT];
#pragma unroll
    for (int i = 0; i < RT; ++i)
      af[i] = *reinterpret_cast<const bf16x8_t*>(&A[i * 16 + (lane & 15)][ks * 32 + kq]);
#pragma unroll
    for (int jt = 0; jt < NTW; ++jt) {
      if (wave + kFuseWaves * jt >= NT) break;  // uniform across the wave
      const bf16x8_t bf = __builtin_bit_cast(bf16x8_t, bv[ks][jt]);
#pragma unroll
      for (int i = 0; i < RT; ++i) acc[i][jt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bf, acc[i][jt], 0, 0, 0);
    }
  }
}

// Four BF16 values of consecutive batch rows b0 .. b0 + 3 (those < B) into
// a batch-minor row: one 8-byte store when all four are in range and aligned.
__device__ __forceinline__ void store_rows4(uint16_t* __restrict__ p, int b0, int B, const uint16_t* h) {
  if (b0 + 3 < B && ((uintptr_t)p & 7) == 0) {
    *reinterpret_cast<uint2*>(p) =
        make_uint2((uint32_t)h[0] | ((uint32_t)h[1] << 16), (uint32_t)h[2] | ((uint32_t)h[3] << 16));
  } else {
#pragma unroll
    for (int r = 0; r < 4; ++r)
      if (b0 + r < B) p[r] = h[r];
  }
}

// One hidden layer of the forward pass (KIN inputs, the transposed weights
// Wt [256][KIN]): z = h W + b to zout (FP32, [B][256]), GELU(z) in BF16 to
// the next LDS buffer and, with hT set, batch-minor [256][B].
template <int RT, int KIN>
__device__ __forceinline__ void fwd_hidden_layer(const uint16_t (*hin)[kFuseLd], uint16_t (*hout)[kFuseLd],
                                                 const uint16_t* __restrict__ Wt, const float* __restrict__ bias,
                                                 int r0, int B, float* __restrict__ zout, uint16_t* __restrict__ hT) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  constexpr int NTW = kMlpHid / 16 / kFuseWaves;
  f32x4_t acc[RT][NTW];
  rowblock_product<RT, KIN, NTW>(hin, Wt, KIN, kMlpHid / 16, acc);
#pragma unroll
  for (int jt = 0; jt < NTW; ++jt) {
    const int n = (wave + kFuseWaves * jt) * 16 + (lane & 15);
    const float bn = bias[n];
#pragma unroll
    for (int i = 0; i < RT; ++i) {
      const int rb = i * 16 + (lane >> 4) * 4;
      uint16_t hb[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int b = r0 + rb + r;
        const float v = acc[i][jt][r] + bn;
        if (b < B) zout[(size_t)b * kMlpHid + n] = v;
        hb[r] = f2bf(gelu_f(v));
        hout[rb + r][n] = hb[r];
      }
      if (hT) store_rows4(hT + (size_t)n * B + r0 + rb, r0 + rb, B, hb);
    }
  }
  __syncthreads();
}

// Forward pass of a block of ROWS rows: z1..z3 (FP32 pre-activations, [B][256]) and Y
// ([B][80]); with hT set, the BF16 activations h0..h3 batch-minor too (the
// weight-gradient products' operands).  loss_zero (optional): zeroed by the
// first workgroup, for the backward pass to accumulate into.
template <int ROWS>
__global__ void __launch_bounds__(kFuseThreads)
mlp_forward_fused_kernel(const uint16_t* __restrict__ w16t, const float* __restrict__ bias32,
                         const float* __restrict__ mean, const float* __restrict__ stdv, const float* __restrict__ X,
                         int B, float* __restrict__ z1, float* __restrict__ z2, float* __restrict__ z3,
                         float* __restrict__ Y, uint16_t* __restrict__ h0T, uint16_t* __restrict__ h1T,
                         uint16_t* __restrict__ h2T, uint16_t* __restrict__ h3T, float* __restrict__ loss_zero) {
  constexpr int RT = ROWS / 16;
  __shared__ __attribute__((aligned(16))) uint16_t hs[2][ROWS][kFuseLd];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int r0 = blockIdx.x * ROWS;
  if (loss_zero && blockIdx.x == 0 && t == 0) *loss_zero = 0.0f;
  // standardised inputs, k 8 .. 31 zero (the first product's K step)
  for (int e = t; e < ROWS * 32; e += kFuseThreads) {
    const int r = e >> 5, k = e & 31, b = r0 + r;
    uint16_t v = 0;
    if (k < kMlpIn && b < B) {
      v = f2bf((X[(size_t)b * kMlpIn + k] - mean[k]) / stdv[k]);
      if (h0T) h0T[(size_t)k * B + b] = v;
    }
    hs[0][r][k] = v;
  }
  __syncthreads();
  fwd_hidden_layer<RT, kMlpIn>(hs[0], hs[1], w16t + kMlpW0, bias32 + kMlpB0, r0, B, z1, h1T);
  fwd_hidden_layer<RT, kMlpHid>(hs[1], hs[0], w16t + kMlpW1, bias32 + kMlpB1, r0, B, z2, h2T);
  fwd_hidden_layer<RT, kMlpHid>(hs[0], hs[1], w16t + kMlpW2, bias32 + kMlpB2, r0, B, z3, h3T);
  // the head: 80 outputs, five column tiles (waves 0-4), linear
  f32x4_t acc[RT][1];
  rowblock_product<RT, kMlpHid, 1>(hs[1], w16t + kMlpW3, kMlpHid, kMlpOut / 16, acc);
#pragma unroll
  for (int jt = 0; jt < 1; ++jt) {
    const int j = wave + kFuseWaves * jt;
    if (j >= kMlpOut / 16) break;
    const int n = j * 16 + (lane & 15);
    const float bias = bias32[kMlpB3 + n];
#pragma unroll
    for (int i = 0; i < RT; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int b = r0 + i * 16 + (lane >> 4) * 4 + r;
        if (b < B) Y[(size_t)b * kMlpOut + n] = acc[i][jt][r] + bias;
      }
  }
}

// One dX product of the backward pass: layer l with NOUT outputs (W_l
// [256][NOUT], row-major), dz_{l-1} = (dz_l W_l^T) * gelu'(z_l) from the BF16
// dz_l in LDS, written BF16 batch-minor [256][B] (o16t) and to the next LDS
// buffer, and the block's FP32 column sums of dz_{l-1} (its part of the bias
// gradient of layer l - 1) to csum[256]: per column, the lane's rows in
// order, then the four lane groups by two butterfly steps.
template <int RT, int NOUT>
__device__ __forceinline__ void bwd_layer(const uint16_t (*din)[kFuseLd], uint16_t (*dout)[kFuseLd],
                                          const uint16_t* __restrict__ Wl, const float* __restrict__ zl, int r0,
                                          int B, uint16_t* __restrict__ o16t, float* __restrict__ csum) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  constexpr int NTW = kMlpHid / 16 / kFuseWaves;
  f32x4_t acc[RT][NTW];
  rowblock_product<RT, NOUT, NTW>(din, Wl, NOUT, kMlpHid / 16, acc);
#pragma unroll
  for (int jt = 0; jt < NTW; ++jt) {
    const int n = (wave + kFuseWaves * jt) * 16 + (lane & 15);
    float cs = 0.0f;
#pragma unroll
    for (int i = 0; i < RT; ++i) {
      const int rb = i * 16 + (lane >> 4) * 4;
      uint16_t hb[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int b = r0 + rb + r;
        float v = 0.0f;
        if (b < B) v = acc[i][jt][r] * gelu_grad_f(zl[(size_t)b * kMlpHid + n]);
        cs += v;
        hb[r] = f2bf(v);
        dout[rb + r][n] = hb[r];
      }
      store_rows4(o16t + (size_t)n * B + r0 + rb, r0 + rb, B, hb);
    }
    cs += __shfl_xor(cs, 16);
    cs += __shfl_xor(cs, 32);
    if (lane < 16) csum[n] = cs;
  }
  __syncthreads();
}

// Backward pass of a block of ROWS rows: the mixture negative log-likelihood of T [B][2]
// under Y (per-sample NLL, and its sum / B added into *loss_sum), dNLL/dY / B
// (BF16 batch-minor [80][B]), then for layers 3, 2, 1 dz_{l-1} = (dz_l W_l^T)
// * gelu'(z_l), BF16 batch-minor [256][B] at slot l - 1 of dz16T (dz_3 =
// dNLL/dY).  The block's FP32 column sums of each gradient, its parts of
// the bias gradients, go to bsum: layer l's ([256], or [80] for l = 3) at
// bsum + (l nblk + block) 256.  The loss takes one lane per (sample,
// component): the 16 lanes of a sample form the two log-sum-exps by shuffles
// within their group.
template <int ROWS>
__global__ void __launch_bounds__(kFuseThreads)
mlp_backward_fused_kernel(const uint16_t* __restrict__ w16, const float* __restrict__ Y, const float* __restrict__ T,
                          int B, const float* __restrict__ z1, const float* __restrict__ z2,
                          const float* __restrict__ z3, float* __restrict__ nll, uint16_t* __restrict__ dY16T,
                          uint16_t* __restrict__ dz16T, float* __restrict__ bsum, float* __restrict__ loss_sum) {
  static_assert(kMlpComp == 16, "one 16-lane group per sample");
  constexpr int RT = ROWS / 16;
  __shared__ __attribute__((aligned(16))) uint16_t ds[2][ROWS][kFuseLd];
  __shared__ float red[kFuseThreads];
  __shared__ float dys[ROWS][kMlpOut];  // FP32 dNLL/dY of the block, for its column sums
  const int t = threadIdx.x;
  const int r0 = blockIdx.x * ROWS;
  const float inv_b = 1.0f / (float)B;
  float contrib = 0.0f;
  static_assert(ROWS * kMlpComp <= kFuseThreads, "one lane per (sample, component)");
  if (t < ROWS * kMlpComp) {  // uniform per wave
    const int sl = t >> 4, k = t & 15;
    const int b = r0 + sl;
    const bool valid = b < B;  // uniform across each 16-lane group
    const int bb = valid ? b : 0;
    const float* y = Y + (size_t)bb * kMlpOut + 5 * k;
    const float logit = y[0];
    const float lmax0 = group16_max(logit);
    const float lse_logit = lmax0 + logf(group16_sum(expf(logit - lmax0)));
    const float t0 = T[2 * bb], t1 = T[2 * bb + 1];
    const float q0 = y[3], q1 = y[4];
    const float l0 = fminf(fmaxf(q0, kLogSigMin), kLogSigMax);
    const float l1 = fminf(fmaxf(q1, kLogSigMin), kLogSigMax);
    const float is0 = expf(-l0), is1 = expf(-l1);
    const float d0 = (t0 - y[1]) * is0;
    const float d1 = (t1 - y[2]) * is1;
    const float lp = logit - lse_logit;
    const float a = lp - (0.5f * (d0 * d0 + d1 * d1) + l0 + l1 + kLog2Pi);
    const float amax = group16_max(a);
    const float lse = amax + logf(group16_sum(expf(a - amax)));
    contrib += (valid && k == 0) ? -lse : 0.0f;
    float gk[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
    if (valid) {
      if (k == 0) nll[b] = -lse;
      const float gam = expf(a - lse);
      const float pi = expf(lp);
      gk[0] = pi - gam;
      gk[1] = -gam * d0 * is0;
      gk[2] = -gam * d1 * is1;
      gk[3] = (q0 > kLogSigMin && q0 < kLogSigMax) ? gam * (1.0f - d0 * d0) : 0.0f;
      gk[4] = (q1 > kLogSigMin && q1 < kLogSigMax) ? gam * (1.0f - d1 * d1) : 0.0f;
    }
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      const float v = gk[q] * inv_b;
      const uint16_t h = f2bf(v);
      if (valid) dY16T[(size_t)(5 * k + q) * B + b] = h;  // [80][B]: the dW product's B operand
      ds[0][sl][5 * k + q] = valid ? h : (uint16_t)0;
      dys[sl][5 * k + q] = valid ? v : 0.0f;
    }
  }
  // the head's K runs to 96 (three k-steps): its last 16 columns are zero
  for (int e = t; e < ROWS * 16; e += kFuseThreads) ds[0][e >> 4][kMlpOut + (e & 15)] = 0;
  red[t] = contrib;
  __syncthreads();
  for (int st = kFuseThreads / 2; st > 0; st >>= 1) {
    if (t < st) red[t] += red[t + st];
    __syncthreads();
  }
  if (t == 0 && loss_sum) atomicAdd(loss_sum, red[0] / (float)B);
  const size_t nblk = gridDim.x;
  if (t < kMlpOut) {  // the head's bias gradient part: rows in order
    float cs = 0.0f;
    for (int r = 0; r < ROWS; ++r) cs += dys[r][t];
    bsum[(3 * nblk + blockIdx.x) * kMlpHid + t] = cs;
  }
  const size_t slot = (size_t)B * kMlpHid;
  bwd_layer<RT, kMlpOut>(ds[0], ds[1], w16 + kMlpW3, z3, r0, B, dz16T + 2 * slot, bsum + (2 * nblk + blockIdx.x) * kMlpHid);
  bwd_layer<RT, kMlpHid>(ds[1], ds[0], w16 + kMlpW2, z2, r0, B, dz16T + slot, bsum + (nblk + blockIdx.x) * kMlpHid);
  bwd_layer<RT, kMlpHid>(ds[0], ds[1], w16 + kMlpW1, z1, r0, B, dz16T, bsum + blockIdx.x * kMlpHid);
}

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

// The fused passes keep a row block's activations in LDS; what leaves them
// is what later launches read: the FP32 pre-activations z (GELU' of the
// backward pass), and the BF16 activations and gradients batch-minor
// ([width][B], the "T" copies) for the weight-gradient products, whose
// contraction runs over the batch, so their operands' k index is contiguous
// in memory.  The gradients dz_0, dz_1, dz_2 of the hidden layers (index l:
// the input side of layer l + 1) all stay alive until those products, which
// run together after the backward pass; each layer has its own split-K
// partial buffers.
struct MlpWork {
  uint16_t *w16t, *h0T, *h1T, *h2T, *h3T, *dY16T, *dz16T;
  float *z1, *z2, *z3, *Y, *nll, *loss, *row, *bsum;
  float* part[4];
};

constexpr int kMlpDims[5] = {kMlpIn, kMlpHid, kMlpHid, kMlpHid, kMlpOut};

static MlpWork carve(void* base, int B) {
  char* p = (char*)base;
  MlpWork w;
  auto take = [&](size_t bytes) { char* r = p; p += align256(bytes); return (void*)r; };
  w.w16t = (uint16_t*)take((size_t)kMlpParams * 2);
  w.h0T = (uint16_t*)take((size_t)B * kMlpIn * 2);
  w.h1T = (uint16_t*)take((size_t)B * kMlpHid * 2);
  w.h2T = (uint16_t*)take((size_t)B * kMlpHid * 2);
  w.h3T = (uint16_t*)take((size_t)B * kMlpHid * 2);
  w.dY16T = (uint16_t*)take((size_t)B * kMlpOut * 2);
  w.dz16T = (uint16_t*)take((size_t)B * kMlpHid * 2 * 3);  // dz_0, dz_1, dz_2
  w.z1 = (float*)take((size_t)B * kMlpHid * 4);
  w.z2 = (float*)take((size_t)B * kMlpHid * 4);
  w.z3 = (float*)take((size_t)B * kMlpHid * 4);
  w.Y = (float*)take((size_t)B * kMlpOut * 4);
  w.nll = (float*)take((size_t)B * 4);
  w.loss = (float*)take(4);
  w.row = (float*)take(kMlpIn * 4);
  // bias-gradient parts: four layers x row blocks x 256 (the head uses 80)
  w.bsum = (float*)take((size_t)4 * ((B + 15) / 16) * kMlpHid * 4);  // blocks of at least 16 rows
  for (int l = 0; l < 4; ++l) w.part[l] = (float*)take((size_t)kMlpSplits * kMlpDims[l] * kMlpDims[l + 1] * 4);
  return w;
}

size_t mlp_workspace_bytes(int B) {
  char* base = nullptr;
  MlpWork w = carve((void*)base, B);
  return (size_t)((char*)w.part[3] - base) + align256((size_t)kMlpSplits * kMlpHid * kMlpOut * 4);
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

// The forward pass reads the transposed weights (w.w16t, formed first);
// with `with_t` the activations are also written batch-minor, and loss_zero
// (optional) is zeroed for the backward pass.
static hipError_t forward_into(const uint16_t* w16, const float* bias32, const float* mean, const float* stdv,
                               const float* X, int B, const MlpWork& w, float* Y, bool with_t, float* loss_zero,
                               hipStream_t st) {
  mlp_weights_t_kernel<<<(kMlpParams + 255) / 256, 256, 0, st>>>(w16, w.w16t);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int rows = fuse_rows(B);
  auto kern = rows == 16 ? mlp_forward_fused_kernel<16> : mlp_forward_fused_kernel<32>;
  kern<<<(B + rows - 1) / rows, kFuseThreads, 0, st>>>(w.w16t, bias32, mean, stdv, X, B, w.z1, w.z2, w.z3, Y,
                                                       with_t ? w.h0T : nullptr, with_t ? w.h1T : nullptr,
                                                       with_t ? w.h2T : nullptr, with_t ? w.h3T : nullptr, loss_zero);
  return hipGetLastError();
}

// Biases are kept in FP32 (they add to FP32 accumulators): the FP32 master
// vector is passed alongside the BF16 weights.
hipError_t launch_mlp_forward(const uint16_t* w16, const float* w32, const float* mean, const float* stdv,
                              const float* X, int B, float* Y, void* work, hipStream_t st) {
  const MlpWork w = carve(work, B);
  return forward_into(w16, w32, mean, stdv, X, B, w, Y, false, nullptr, st);
}

// One gradient: weights transposed, the fused forward and backward passes,
// every layer's weight gradient in one launch and their split-K reductions
// in another.  The loss accumulates straight into *loss (or the workspace).
hipError_t launch_mlp_grad(const uint16_t* w16, const float* w32, const float* mean, const float* stdv,
                           const float* X, const float* T, int B, float* grad, float* loss, void* work,
                           hipStream_t st) {
  const MlpWork w = carve(work, B);
  float* const lossp = loss ? loss : w.loss;
  hipError_t e = forward_into(w16, w32, mean, stdv, X, B, w, w.Y, true, lossp, st);
  if (e != hipSuccess) return e;
  const int rows = fuse_rows(B);
  auto bkern = rows == 16 ? mlp_backward_fused_kernel<16> : mlp_backward_fused_kernel<32>;
  bkern<<<(B + rows - 1) / rows, kFuseThreads, 0, st>>>(w16, w.Y, T, B, w.z1, w.z2, w.z3, w.nll, w.dY16T, w.dz16T,
                                                        w.bsum, lossp);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  size_t ow[4], ob[4];
  layer_offsets(ow, ob);
  const uint16_t* hin_t[4] = {w.h0T, w.h1T, w.h2T, w.h3T};
  // dz of each layer's output, BF16 batch-minor (the operand); layer 3's is
  // dNLL/dY.
  const uint16_t* dz16t[4];
  for (int l = 0; l < 3; ++l) dz16t[l] = w.dz16T + (size_t)l * B * kMlpHid;
  dz16t[3] = w.dY16T;
  const int nblk = (B + rows - 1) / rows;
  // Every layer's weight gradient in one launch: dW_l = h_l^T dz_l
  // ([kin][nout]) from the batch-minor copies (h^T [kin][B] as A, dz^T
  // [nout][B] as the transposed B), split over the batch; then one launch
  // reduces every layer's parts in order, and its bias gradient (db_l =
  // column sums of dz_l) from the backward pass's per-block FP32 sums.
  int splits = B / kMlpSplitRows;
  splits = splits < 1 ? 1 : (splits > kMlpSplits ? kMlpSplits : splits);
  GemmGroup gg{};
  ReduceGroup rg{};
  gg.n = rg.n = 4;
  int mt = 1, nt = 1;
  for (int l = 0; l < 4; ++l) {
    const int kin = kMlpDims[l], nout = kMlpDims[l + 1];
    GemmArgs& gw = gg.g[l];
    gw.A = hin_t[l]; gw.lda = B;
    gw.B = dz16t[l]; gw.tb = 1; gw.ldb = B;
    gw.M = kin; gw.N = nout; gw.K = B;
    gw.part = w.part[l];
    const int parts = gemm_prepare(gw, splits);
    gg.zbase[l + 1] = gg.zbase[l] + parts;
    mt = std::max(mt, (kin + 63) / 64);
    nt = std::max(nt, (nout + 63) / 64);
    rg.part[l] = w.part[l]; rg.cs_part[l] = w.bsum + (size_t)l * nblk * kMlpHid;
    rg.out[l] = grad + ow[l]; rg.cs_out[l] = grad + ob[l];
    rg.parts[l] = parts; rg.cs_parts[l] = nblk; rg.cs_ld[l] = kMlpHid;
    rg.wbase[l + 1] = rg.wbase[l] + kin * nout;
    rg.cbase[l + 1] = rg.cbase[l] + nout;
  }
  rg.wblocks = (rg.wbase[4] + 255) / 256;
  gemm_group_kernel<<<dim3(nt, mt, gg.zbase[4]), 256, 0, st>>>(gg);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  splitk_reduce_group_kernel<<<rg.wblocks + (rg.cbase[4] + 3) / 4, 256, 0, st>>>(rg);
  return hipGetLastError();
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
  return gemm(g, st);
}

}  // namespace mpmi
