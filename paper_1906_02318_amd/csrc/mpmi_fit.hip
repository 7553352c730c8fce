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
constexpr int kFitThreads = 256;  // four waves: the solve kernel gives each a task
static_assert(kFitThreads == 4 * 64, "solve_kernel assigns tasks to exactly four waves");
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

// tot[e] = sum over the parts of part[p][e], in a fixed order: the four
// threads of element e sum parts p = q, q + 4, ... (q = 0..3), then add the
// four quarters in order.  A workgroup covers kReduceElems elements.
constexpr int kReduceElems = 64;
__global__ void __launch_bounds__(4 * kReduceElems)
reduce_kernel(int nparts, int E, const double* __restrict__ part, double* __restrict__ tot) {
  __shared__ double q4[4][kReduceElems];
  const int el = threadIdx.x % kReduceElems, q = threadIdx.x / kReduceElems;
  const int e = blockIdx.x * kReduceElems + el;
  double s = 0.0;
  if (e < E)
    for (int p = q; p < nparts; p += 4) s += part[(size_t)p * E + e];
  q4[q][el] = s;
  __syncthreads();
  if (q == 0 && e < E) tot[e] = ((q4[0][el] + q4[1][el]) + q4[2][el]) + q4[3][el];
}

// Value of x in lane k (k wave-uniform), to every lane of the wave.
__device__ __forceinline__ double lane_bcast(double x, int k) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(x);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, k);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), k);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// One step of a DPP sum: x plus the value CTRL selects (0 where the source
// is outside the row or the row and bank masks).
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_add(double x) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, ROW_MASK, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, ROW_MASK, 0xF, false);
  return x + __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// Sum over the 64 lanes (every lane active), the same value in every lane:
// shifts by 1, 2, 4, 8 within each row of 16, the row broadcasts of lanes 15
// and 31, then lane 63's total read back.  A fixed order; no LDS round trip.
__device__ __forceinline__ double wave_sum(double x) {
  x = dpp_add<0x111, 0xF>(x);  // row_shr:1
  x = dpp_add<0x112, 0xF>(x);  // row_shr:2
  x = dpp_add<0x114, 0xF>(x);  // row_shr:4
  x = dpp_add<0x118, 0xF>(x);  // row_shr:8
  x = dpp_add<0x142, 0xA>(x);  // row_bcast:15 into rows 1 and 3
  x = dpp_add<0x143, 0xC>(x);  // row_bcast:31 into rows 2 and 3
  return lane_bcast(x, 63);
}

// L z = b with the Cholesky factor in the lower triangle of Lf (diagonal
// included): lane i holds b_i and 1 / L_ii (rinv) and returns z_i (lanes >= D
// hold 0).  Column by column: z_k = r_k / L_kk once lane k's residual r_k is
// complete (lane k forms the quotient, the wave reads it back), then every
// later row subtracts L_ik z_k.  No division in the serial chain.
template <int LD>
__device__ __forceinline__ double wave_lower_solve(const double (&Lf)[MPMI_MAX_DIM][LD], int D, int lane, double rinv,
                                                   double b) {
  double r = b, z = 0.0;
#pragma unroll 4
  for (int k = 0; k < D; ++k) {
    const double zk = lane_bcast(r * rinv, k);
    if (lane == k) z = zk;
    if (lane > k && lane < D) r = fma(-Lf[lane][k], zk, r);
  }
  return z;
}

// L^T y = z, the same way from the last row up.
template <int LD>
__device__ __forceinline__ double wave_upper_solve(const double (&Lf)[MPMI_MAX_DIM][LD], int D, int lane, double rinv,
                                                   double z) {
  double r = z, y = 0.0;
#pragma unroll 4
  for (int k = D - 1; k >= 0; --k) {
    const double yk = lane_bcast(r * rinv, k);
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
  // Triangular solves and the condition estimate run one wave per task, the
  // tasks concurrently: lane i owns row i (D <= 64), the wave's lockstep
  // orders the steps, and the values a step needs from another lane arrive
  // by lane broadcast, so no workgroup barrier is involved.  The factor is
  // read-only from here on.
  const int lane = t & 63, wave = t >> 6;
  const bool own = lane < D;
  const double rinv = own ? 1.0 / L[lane][lane] : 0.0;
  __shared__ double s_lmax, s_lmin_inv;
  if (wave >= 2) {
    // K: waves 2 and 3 solve the right-hand sides c = wave - 2, wave, ...
    for (int c = wave - 2; c < n; c += 2) {
      const double z = wave_lower_solve(L, D, lane, rinv, own ? B[lane][c] : 0.0);
      const double k = wave_upper_solve(L, D, lane, rinv, z);
      if (own) K[(size_t)lane * n + c] = k / sc[lane];
    }
  } else if (wave == 1) {
    // Largest eigenvalue of the scaled Gram matrix G_s by power iteration
    // (G_s from its upper triangle and the diagonal of L L^T).  Lane i holds
    // row i of G_s in registers; the loops run over the 64-row maximum with
    // compile-time indices (rows and columns past D are zero).
    double diag = 0.0;
    if (own)
      for (int k = 0; k <= lane; ++k) diag += L[lane][k] * L[lane][k];
    double grow[MPMI_MAX_DIM];
#pragma unroll
    for (int j = 0; j < MPMI_MAX_DIM; ++j)
      grow[j] = (own && j < D) ? (lane == j ? diag : (lane < j ? L[lane][j] : L[j][lane])) : 0.0;
    double v = own ? 1.0 + 0.01 * lane : 0.0;
    double lmax = 0.0;
    for (int it = 0; it < 60; ++it) {
      double w = 0.0;
#pragma unroll
      for (int j = 0; j < MPMI_MAX_DIM; ++j) w = fma(grow[j], lane_bcast(v, j), w);
      const double nn = sqrt(wave_sum(w * w));
      lmax = wave_sum(w * v);
      v = w / nn;
    }
    if (lane == 0) s_lmax = lmax;
  } else {
    // Smallest eigenvalue by inverse iteration through the Cholesky factor.
    // Lane i holds m[k] = L_ik for k < i (its row) and L_ki for k > i (its
    // column) in registers.  The forward solve uses lane i's residual only up
    // to step i and the backward solve only down to step i, so each may
    // subtract the other half's entries after that point: a solve step is a
    // multiply, a broadcast and an FMA.
    double m[MPMI_MAX_DIM];
#pragma unroll
    for (int k = 0; k < MPMI_MAX_DIM; ++k)
      m[k] = (own && k < D && k != lane) ? (k < lane ? L[lane][k] : L[k][lane]) : 0.0;
    double v = own ? 1.0 - 0.01 * lane : 0.0;
    double lmin_inv = 0.0;
    for (int it = 0; it < 60; ++it) {
      double r = v, z = 0.0;
#pragma unroll
      for (int k = 0; k < MPMI_MAX_DIM; ++k) {  // L z = v
        const double zk = lane_bcast(r * rinv, k);
        z = lane == k ? zk : z;
        r = fma(-m[k], zk, r);
      }
      double y = 0.0;
      r = z;
#pragma unroll
      for (int k = MPMI_MAX_DIM - 1; k >= 0; --k) {  // L^T y = z
        const double yk = lane_bcast(r * rinv, k);
        y = lane == k ? yk : y;
        r = fma(-m[k], yk, r);
      }
      const double nn = sqrt(wave_sum(y * y));
      lmin_inv = wave_sum(y * v);
      v = y / nn;
    }
    if (lane == 0) s_lmin_inv = lmin_inv;
  }
  __syncthreads();
  if (t == 0) {
    info->status = bad ? MPMI_ESINGULAR : MPMI_OK;
    const double cg = s_lmax * s_lmin_inv;
    info->cond = cg > 0.0 ? sqrt(cg) : INFINITY;
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
  reduce_kernel<<<(E + kReduceElems - 1) / kReduceElems, 4 * kReduceElems, 0, st>>>(nparts, E, part, tot);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  solve_kernel<<<1, kFitThreads, 0, st>>>(n, dim, (long long)T, ridge, tot, K_out, info);
  return hipGetLastError();
}

}  // namespace mpmi
