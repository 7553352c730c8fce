// Koopman fit in FP64 (Sec. IV-A: the model is learned from transition data;
// least squares as in extended DMD).  Three launches:
//   1. gram:   every workgroup lifts tiles of 64 rows into LDS (psi computed on
//              the fly, never materialised in HBM) and accumulates its share
//              of Z^T Z restricted to the first D rows, Z = [Psi | Y];
//   2. reduce: partial sums added in a fixed order (deterministic);
//   3. solve:  one workgroup: RMS column scaling, ridge, Cholesky of the
//              scaled Gram matrix in LDS, then, one wave per task, the two
//              triangular solves per right-hand side, unscaling, and power /
//              inverse iteration for the condition number.
#include <hip/hip_runtime.h>

#include "mpmi_launch.hpp"

namespace mpmi {

constexpr int kFitRows = 64;       // rows per LDS tile
constexpr int kFitBlocks = 256;    // maximum partial-sum workgroups
constexpr int kFitCols = MPMI_MAX_DIM + MPMI_MAX_STATE;  // D + n <= 72
constexpr int kFitThreads = 256;
constexpr int kFitPerThread = (MPMI_MAX_DIM * kFitCols + kFitThreads - 1) / kFitThreads;  // 18

struct FitInfo {
  int32_t status;
  int32_t pad;
  double cond;
};

// psi(x, u) in FP64, same feature order as the FP32 path.
__device__ void lift_f64(int basis, int n, int m, const double* x, const double* u, double* psi) {
  if (basis == MPMI_BASIS_LINEAR) {
    for (int k = 0; k < n; ++k) psi[k] = x[k];
    for (int k = 0; k < m; ++k) psi[n + k] = u[k];
    return;
  }
  if (basis == MPMI_BASIS_BALANCE_BOT) {
    const double w[5] = {x[0], x[1], x[2], x[3], u[0]};
    int f = 0;
    psi[f++] = 1.0;
    for (int k = 0; k < 5; ++k) psi[f++] = w[k];
    for (int k = 0; k < 5; ++k)
      for (int l = k; l < 5; ++l) psi[f++] = w[k] * w[l];
    return;
  }
  const double w[8] = {x[0], x[1], x[2], x[3], x[4], x[5], u[0], u[1]};
  int f = 0;
  psi[f++] = 1.0;
  for (int k = 0; k < 8; ++k) psi[f++] = w[k];
  for (int k = 0; k < 8; ++k)
    for (int l = k; l < 8; ++l) psi[f++] = w[k] * w[l];
  const double sp = sin(w[2]), cp = cos(w[2]), sd = sin(w[6]), cd = cos(w[6]);
  const double vx = w[3], vy = w[4], r = w[5], a = w[7];
  psi[f++] = sp; psi[f++] = cp; psi[f++] = sd; psi[f++] = cd;
  psi[f++] = sp * vx; psi[f++] = sp * vy; psi[f++] = sp * r; psi[f++] = sp * a;
  psi[f++] = cp * vx; psi[f++] = cp * vy; psi[f++] = cp * r; psi[f++] = cp * a;
  psi[f++] = sd * vx; psi[f++] = sd * vy; psi[f++] = sd * r;
  psi[f++] = cd * vx; psi[f++] = cd * vy; psi[f++] = cd * r;
  psi[f++] = a * sd;
}

__global__ void __launch_bounds__(kFitThreads)
gram_kernel(int basis, int n, int m, int D, const double* __restrict__ X, const double* __restrict__ U,
            const double* __restrict__ Y, long long T, double* __restrict__ part) {
  __shared__ double Z[kFitRows][kFitCols + 1];
  const int C = D + n;
  const int E = D * C;
  double acc[kFitPerThread];
  int ea[kFitPerThread], eb[kFitPerThread];
#pragma unroll
  for (int k = 0; k < kFitPerThread; ++k) {
    acc[k] = 0.0;
    const int e = threadIdx.x + k * kFitThreads;
    ea[k] = e < E ? e / C : 0;
    eb[k] = e < E ? e % C : 0;
  }
  const long long ntiles = (T + kFitRows - 1) / kFitRows;
  for (long long tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const long long r0 = tile * kFitRows;
    if (threadIdx.x < kFitRows) {
      const long long r = r0 + threadIdx.x;
      double psi[MPMI_MAX_DIM];
      double x[MPMI_MAX_STATE], u[MPMI_MAX_INPUT];
      if (r < T) {
        for (int k = 0; k < n; ++k) x[k] = X[r * n + k];
        for (int k = 0; k < m; ++k) u[k] = U[r * m + k];
        lift_f64(basis, n, m, x, u, psi);
        for (int k = 0; k < D; ++k) Z[threadIdx.x][k] = psi[k];
        for (int k = 0; k < n; ++k) Z[threadIdx.x][D + k] = Y[r * n + k];
      } else {
        for (int k = 0; k < C; ++k) Z[threadIdx.x][k] = 0.0;
      }
    }
    __syncthreads();
    for (int rr = 0; rr < kFitRows; ++rr) {
#pragma unroll
      for (int k = 0; k < kFitPerThread; ++k) acc[k] = fma(Z[rr][ea[k]], Z[rr][eb[k]], acc[k]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int k = 0; k < kFitPerThread; ++k) {
    const int e = threadIdx.x + k * kFitThreads;
    if (e < E) part[(size_t)blockIdx.x * E + e] = acc[k];
  }
}

__global__ void reduce_kernel(int nparts, int E, const double* __restrict__ part, double* __restrict__ tot) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= E) return;
  double s = 0.0;
  for (int p = 0; p < nparts; ++p) s += part[(size_t)p * E + e];
  tot[e] = s;
}

// Value of x in lane k (k wave-uniform), to every lane of the wave.
__device__ __forceinline__ double lane_bcast(double x, int k) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(x);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, k);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), k);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Sum over the 64 lanes (butterfly, the same order in every lane).
__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}

// L z = b with the Cholesky factor in the lower triangle of Lf (diagonal
// included): lane i holds b_i and returns z_i (lanes >= D hold 0).  Column
// by column: z_k = r_k / L_kk once lane k's residual r_k is complete, then
// every later row subtracts L_ik z_k.
template <int LD>
__device__ __forceinline__ double wave_lower_solve(const double (&Lf)[MPMI_MAX_DIM][LD], int D, int lane, double b) {
  double r = b, z = 0.0;
  for (int k = 0; k < D; ++k) {
    const double zk = lane_bcast(r, k) / Lf[k][k];
    if (lane == k) z = zk;
    if (lane > k && lane < D) r = fma(-Lf[lane][k], zk, r);
  }
  return z;
}

// L^T y = z, the same way from the last row up.
template <int LD>
__device__ __forceinline__ double wave_upper_solve(const double (&Lf)[MPMI_MAX_DIM][LD], int D, int lane, double z) {
  double r = z, y = 0.0;
  for (int k = D - 1; k >= 0; --k) {
    const double yk = lane_bcast(r, k) / Lf[k][k];
    if (lane == k) y = yk;
    if (lane < k) r = fma(-Lf[k][lane], yk, r);
  }
  return y;
}

// One workgroup.  tot holds [D][C]: G = columns 0..D-1, A = columns D..D+n-1.
__global__ void __launch_bounds__(kFitThreads)
solve_kernel(int n, int D, long long T, double ridge, const double* __restrict__ tot, double* __restrict__ K,
             FitInfo* __restrict__ info) {
  __shared__ double L[MPMI_MAX_DIM][MPMI_MAX_DIM + 1];
  __shared__ double B[MPMI_MAX_DIM][MPMI_MAX_STATE];
  __shared__ double sc[MPMI_MAX_DIM];
  __shared__ int bad;
  const int t = threadIdx.x;
  const int C = D + n;
  if (t == 0) bad = 0;
  for (int f = t; f < D; f += blockDim.x) {
    const double g = tot[(size_t)f * C + f];
    const double s = sqrt(g / (double)T);
    sc[f] = s > 0.0 ? s : 1.0;
  }
  __syncthreads();
  for (int e = t; e < D * D; e += blockDim.x) {
    const int i = e / D, j = e % D;
    double g = tot[(size_t)i * C + j] / (sc[i] * sc[j]);
    if (i == j) g += ridge;
    L[i][j] = g;
  }
  for (int e = t; e < D * n; e += blockDim.x) {
    const int i = e / n, j = e % n;
    B[i][j] = tot[(size_t)i * C + D + j] / sc[i];
  }
  __syncthreads();
  // Keep the scaled Gram matrix's upper triangle (i < j) for the condition
  // estimate; the factor goes to the lower triangle and the diagonal.
  const double pivot_floor = 1e-14 * (double)T;
  for (int k = 0; k < D; ++k) {
    if (t == 0) {
      double d = L[k][k];
      if (!(d > pivot_floor)) {
        bad = 1;
        d = 1.0;
      }
      L[k][k] = sqrt(d);
    }
    __syncthreads();
    for (int i = k + 1 + t; i < D; i += blockDim.x) L[i][k] /= L[k][k];
    __syncthreads();
    for (int e = t; e < (D - k - 1) * (D - k - 1); e += blockDim.x) {
      const int i = k + 1 + e / (D - k - 1), j = k + 1 + e % (D - k - 1);
      if (j <= i) L[i][j] -= L[i][k] * L[j][k];
    }
    __syncthreads();
  }
  // Triangular solves and the condition estimate run one wave per task: lane
  // i owns row i (D <= 64), the wave's lockstep orders the steps, and the
  // values a step needs from another lane arrive by lane broadcast, so no
  // workgroup barrier is involved.  The factor is read-only from here on.
  const int lane = t & 63, wave = t >> 6;
  const bool own = lane < D;
  // K: wave q solves the right-hand sides q, q + 4 (n <= 8 columns).
  for (int c = wave; c < n; c += kFitThreads / 64) {
    const double z = wave_lower_solve(L, D, lane, own ? B[lane][c] : 0.0);
    const double k = wave_upper_solve(L, D, lane, z);
    if (own) K[(size_t)lane * n + c] = k / sc[lane];
  }
  // Condition estimate of the scaled Gram matrix G_s (wave 0): power
  // iteration for the largest eigenvalue (G_s from its upper triangle and
  // the diagonal of L L^T), inverse iteration through the Cholesky factor
  // for the smallest.
  if (wave == 0) {
    double diag = 0.0;
    if (own)
      for (int k = 0; k <= lane; ++k) diag += L[lane][k] * L[lane][k];
    double v = own ? 1.0 + 0.01 * lane : 0.0;
    double lmax = 0.0;
    for (int it = 0; it < 60; ++it) {
      double w = 0.0;
      for (int j = 0; j < D; ++j) {
        const double vj = lane_bcast(v, j);
        const double g = lane == j ? diag : (lane < j ? L[lane][j] : L[j][lane]);
        w = own ? fma(g, vj, w) : 0.0;
      }
      const double nn = sqrt(wave_sum(w * w));
      lmax = wave_sum(w * v);
      v = w / nn;
    }
    v = own ? 1.0 - 0.01 * lane : 0.0;
    double lmin_inv = 0.0;
    for (int it = 0; it < 60; ++it) {
      const double w = wave_upper_solve(L, D, lane, wave_lower_solve(L, D, lane, v));
      const double nn = sqrt(wave_sum(w * w));
      lmin_inv = wave_sum(w * v);
      v = w / nn;
    }
    if (lane == 0) {
      info->status = bad ? MPMI_ESINGULAR : MPMI_OK;
      const double cg = lmax * lmin_inv;
      info->cond = cg > 0.0 ? sqrt(cg) : INFINITY;
    }
  }
}

size_t fit_workspace_bytes() {
  const size_t E = (size_t)MPMI_MAX_DIM * kFitCols;
  return (size_t)(kFitBlocks + 1) * E * sizeof(double) + 256;
}

hipError_t launch_fit(const mpmi_system& sys, int dim, const double* X, const double* U, const double* Y,
                      int64_t T, double ridge, double* K_out, void* work, hipStream_t st) {
  const int n = sys.n_state, m = sys.n_input;
  const int E = dim * (dim + n);
  long long ntiles = (T + kFitRows - 1) / kFitRows;
  const int nparts = (int)(ntiles < kFitBlocks ? ntiles : kFitBlocks);
  double* part = (double*)work;
  double* tot = part + (size_t)kFitBlocks * MPMI_MAX_DIM * kFitCols;
  FitInfo* info = (FitInfo*)(tot + (size_t)MPMI_MAX_DIM * kFitCols);
  gram_kernel<<<nparts, kFitThreads, 0, st>>>(sys.basis, n, m, dim, X, U, Y, (long long)T, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  reduce_kernel<<<(E + 255) / 256, 256, 0, st>>>(nparts, E, part, tot);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  solve_kernel<<<1, kFitThreads, 0, st>>>(n, dim, (long long)T, ridge, tot, K_out, info);
  return hipGetLastError();
}

}  // namespace mpmi
