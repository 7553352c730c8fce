// Device ceiling diagnostics.
//
// The fused tick's step is VALU-bound: its work is FP32 FMAs and products
// issued one wave64 instruction per four cycles per SIMD (packed FP32 is
// disabled in every kernel of the library).  fma_rate_kernel measures the
// rate such instructions reach on the part: registers only, 16 independent
// FMA chains per lane, 8 workgroups of 256 lanes per compute unit.
// sincos64_kernel exposes the FP64 re-roll's sin/cos for accuracy checks.
#include <hip/hip_runtime.h>

#include "mpmi_device.hpp"
#include "mpmi_launch.hpp"

namespace mpmi {

constexpr int kFmaChains = 16;

__global__ void __launch_bounds__(256) fma_rate_kernel(float* __restrict__ sink, int iters, float a, float b) {
  float v[kFmaChains];
#pragma unroll
  for (int k = 0; k < kFmaChains; ++k) v[k] = (float)threadIdx.x * 1e-3f + (float)k;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int k = 0; k < kFmaChains; ++k) v[k] = fmaf(v[k], a, b);
  }
  float s = 0.0f;
#pragma unroll
  for (int k = 0; k < kFmaChains; ++k) s += v[k];
  // Data-dependent store (never taken for the arguments used) keeps the
  // chains live without writing memory.
  if (s == -1.0f) sink[0] = s;
}

hipError_t measure_fma_rate(float* sink, double* tflops) {
  const int ncu = device_cu_count();
  const int block = 256, grid = ncu * 8, iters = 20000;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  float best = 1e30f;
  for (int rep = 0; rep < 3 && e == hipSuccess; ++rep) {
    fma_rate_kernel<<<grid, block, 0, 0>>>(sink, iters, 0.999f, 0.001f);  // warm
    if ((e = hipEventRecord(e0, 0)) != hipSuccess) break;
    fma_rate_kernel<<<grid, block, 0, 0>>>(sink, iters, 0.999f, 0.001f);
    if ((e = hipGetLastError()) != hipSuccess) break;
    if ((e = hipEventRecord(e1, 0)) != hipSuccess) break;
    if ((e = hipEventSynchronize(e1)) != hipSuccess) break;
    float ms = 0.0f;
    if ((e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) break;
    best = ms < best ? ms : best;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (e != hipSuccess) return e;
  const double flops = 2.0 * kFmaChains * (double)iters * (double)grid * (double)block;
  *tflops = flops / ((double)best * 1e-3) / 1e12;
  return hipSuccess;
}

// HBM write ceilings for the trajectory store: the store pattern of
// traj[H][n][ld] alone (rows ld floats apart; lane c < Nc writes element c
// of each of the H * n rows, no compute), and a contiguous stream of
// 16-byte stores of the same number of bytes.
__global__ void __launch_bounds__(256) traj_pattern_kernel(float* __restrict__ traj, int Nc, long long ld,
                                                           int rows) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= Nc) return;
  float v = (float)c;
  for (int r = 0; r < rows; ++r) {
    v = fmaf(v, 1.0001f, 1.0f);
    __builtin_nontemporal_store(v, &traj[(size_t)r * (size_t)ld + c]);
  }
}

__global__ void __launch_bounds__(256) write_stream_kernel(float4* __restrict__ out, size_t n4) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride)
    out[i] = make_float4(1.0f, 2.0f, 3.0f, (float)i);
}

hipError_t measure_write_rates(void* buf, int Nc, long long ld, int rows, double* pattern_gbs, double* stream_gbs) {
  const size_t bytes = (size_t)rows * (size_t)Nc * sizeof(float);
  const size_t n4 = bytes / 16;
  const int block = 256;
  const unsigned grid_p = (unsigned)((Nc + block - 1) / block);
  const unsigned grid_s = (unsigned)(device_cu_count() * 16);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  float best_p = 1e30f, best_s = 1e30f;
  for (int rep = 0; rep < 3 && e == hipSuccess; ++rep) {
    for (int kind = 0; kind < 2 && e == hipSuccess; ++kind) {
      if (kind == 0) traj_pattern_kernel<<<grid_p, block, 0, 0>>>((float*)buf, Nc, ld, rows);  // warm
      else write_stream_kernel<<<grid_s, block, 0, 0>>>((float4*)buf, n4);
      if ((e = hipEventRecord(e0, 0)) != hipSuccess) break;
      if (kind == 0) traj_pattern_kernel<<<grid_p, block, 0, 0>>>((float*)buf, Nc, ld, rows);
      else write_stream_kernel<<<grid_s, block, 0, 0>>>((float4*)buf, n4);
      if ((e = hipGetLastError()) != hipSuccess) break;
      if ((e = hipEventRecord(e1, 0)) != hipSuccess) break;
      if ((e = hipEventSynchronize(e1)) != hipSuccess) break;
      float ms = 0.0f;
      if ((e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) break;
      if (kind == 0) best_p = ms < best_p ? ms : best_p;
      else best_s = ms < best_s ? ms : best_s;
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (e != hipSuccess) return e;
  *pattern_gbs = (double)bytes / ((double)best_p * 1e-3) / 1e9;
  *stream_gbs = (double)(n4 * 16) / ((double)best_s * 1e-3) / 1e9;
  return hipSuccess;
}

// HBM read ceilings for the safety check over stored trajectories: the load
// pattern of traj[rows][ld] alone (lane c < Nc reads element c of every row,
// no compute) and a contiguous stream of 16-byte loads of the same number of
// bytes.  The sums feed an empty asm statement, so the loads stay and
// nothing is written.
__global__ void __launch_bounds__(256) traj_read_kernel(const float* __restrict__ traj, int Nc, long long ld,
                                                        int rows) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= Nc) return;
  float acc = 0.0f;
#pragma unroll 4
  for (int r = 0; r < rows; ++r) acc += traj[(size_t)r * (size_t)ld + c];
  asm volatile("" ::"v"(acc));
}

__global__ void __launch_bounds__(256) read_stream_kernel(const float4* __restrict__ in, size_t n4) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  float acc = 0.0f;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride) {
    const float4 v = in[i];
    acc += (v.x + v.y) + (v.z + v.w);
  }
  asm volatile("" ::"v"(acc));
}

hipError_t measure_read_rates(const void* buf, int Nc, long long ld, int rows, double* pattern_gbs,
                              double* stream_gbs) {
  const size_t bytes = (size_t)rows * (size_t)Nc * sizeof(float);
  const size_t n4 = bytes / 16;
  const int block = 256;
  const unsigned grid_p = (unsigned)((Nc + block - 1) / block);
  const unsigned grid_s = (unsigned)(device_cu_count() * 16);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  float best_p = 1e30f, best_s = 1e30f;
  for (int rep = 0; rep < 3 && e == hipSuccess; ++rep) {
    for (int kind = 0; kind < 2 && e == hipSuccess; ++kind) {
      if ((e = hipEventRecord(e0, 0)) != hipSuccess) break;
      if (kind == 0) traj_read_kernel<<<grid_p, block, 0, 0>>>((const float*)buf, Nc, ld, rows);
      else read_stream_kernel<<<grid_s, block, 0, 0>>>((const float4*)buf, n4);
      if ((e = hipGetLastError()) != hipSuccess) break;
      if ((e = hipEventRecord(e1, 0)) != hipSuccess) break;
      if ((e = hipEventSynchronize(e1)) != hipSuccess) break;
      float ms = 0.0f;
      if ((e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) break;
      if (kind == 0) best_p = ms < best_p ? ms : best_p;
      else best_s = ms < best_s ? ms : best_s;
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (e != hipSuccess) return e;
  *pattern_gbs = (double)bytes / ((double)best_p * 1e-3) / 1e9;
  *stream_gbs = (double)(n4 * 16) / ((double)best_s * 1e-3) / 1e9;
  return hipSuccess;
}

// The FP64 re-roll's sin and cos (sincos_rr64) of n doubles.
__global__ void __launch_bounds__(256) sincos64_kernel(const double* __restrict__ x, double* __restrict__ sn,
                                                       double* __restrict__ cs, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) sincos_rr64(x[i], &sn[i], &cs[i]);
}

hipError_t launch_sincos64(const double* x, double* sn, double* cs, int n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  sincos64_kernel<<<(n + 255) / 256, 256, 0, st>>>(x, sn, cs, n);
  return hipGetLastError();
}

}  // namespace mpmi
