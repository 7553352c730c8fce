// Koopman fit in FP64 (Sec. IV-A: the model is learned from transition data;
// least squares as in extended DMD).  Three launches:
//   1. gram:   every workgroup lifts tiles of 64 rows into LDS (psi computed on
//              the fly, never materialised in HBM) and accumulates its share
//              of Z^T Z restricted to the first D rows, Z = [Psi | Y], in
//              4 x 6 register blocks, one wave lifting the next tile while
//              three accumulate the current one;
//   2. reduce: partial sums added in a fixed order (deterministic);
//   3. solve:  one workgroup: RMS column scaling, ridge, Cholesky of the
//              scaled Gram matrix in registers, then, one wave per task, the two
//              triangular solves per right-hand side and unscaling, power
//              iteration on the Gram matrix and, after all four waves form
//              its inverse from the factor's inverse, on that, for the
//              condition number.
#include <hip/hip_runtime.h>

#include "mpmi_launch.hpp"

namespace mpmi {

constexpr int kFitRows = 64;       // rows per LDS tile
constexpr int kFitBlocks = 256;    // maximum partial-sum workgroups
constexpr int kFitCols = MPMI_MAX_DIM + MPMI_MAX_STATE;  // D + n <= 72
constexpr int kFitThreads = 256;  // four waves: the solve kernel gives each a task
static_assert(kFitThreads == 4 * 64, "solve_kernel assigns tasks to exactly four waves");

struct FitInfo {
  int32_t status;
  int32_t pad;
  double cond;
};

// psi(x, u) of one transition in FP64, the FP32 path's feature order,
// written to z (an LDS row) from the row's state xr[n] and input ur[m].  The
// fixed bases take their atoms into registers by constant index.
// Atom q of a custom basis at w = [xr; ur], FP64.
__device__ __forceinline__ double custom_atom(const mpmi_system& sys, int q, const double* __restrict__ xr,
                                              const double* __restrict__ ur) {
  const int kd = sys.atom_kind[q], v = sys.atom_var[q];
  const double w = v < sys.n_state ? xr[v] : ur[v - sys.n_state];
  if (kd == MPMI_ATOM_VAR) return w;
  if (kd == MPMI_ATOM_SIN) return sin(w);
  if (kd == MPMI_ATOM_COS) return cos(w);
  return 1.0;
}

__device__ __forceinline__ void lift_row(const mpmi_system& sys, const double* __restrict__ xr,
                                         const double* __restrict__ ur, double* z) {
  const int basis = sys.basis, n = sys.n_state, m = sys.n_input;
  if (basis == MPMI_BASIS_CUSTOM) {
    for (int f = 0; f < sys.dim; ++f)
      z[f] = custom_atom(sys, sys.feat_a[f], xr, ur) * custom_atom(sys, sys.feat_b[f], xr, ur);
    return;
  }
  if (basis == MPMI_BASIS_LINEAR) {
    for (int k = 0; k < n; ++k) z[k] = xr[k];
    for (int k = 0; k < m; ++k) z[n + k] = ur[k];
    return;
  }
  if (basis == MPMI_BASIS_BALANCE_BOT) {
    const double w[5] = {xr[0], xr[1], xr[2], xr[3], ur[0]};
    int f = 0;
    z[f++] = 1.0;
#pragma unroll
    for (int k = 0; k < 5; ++k) z[f++] = w[k];
#pragma unroll
    for (int k = 0; k < 5; ++k)
#pragma unroll
      for (int l = k; l < 5; ++l) z[f++] = w[k] * w[l];
    return;
  }
  const double w[8] = {xr[0], xr[1], xr[2], xr[3], xr[4], xr[5], ur[0], ur[1]};
  int f = 0;
  z[f++] = 1.0;
#pragma unroll
  for (int k = 0; k < 8; ++k) z[f++] = w[k];
#pragma unroll
  for (int k = 0; k < 8; ++k)
#pragma unroll
    for (int l = k; l < 8; ++l) z[f++] = w[k] * w[l];
  const double sp = sin(w[2]), cp = cos(w[2]), sd = sin(w[6]), cd = cos(w[6]);
  const double vx = w[3], vy = w[4], r = w[5], a = w[7];
  z[f++] = sp; z[f++] = cp; z[f++] = sd; z[f++] = cd;
  z[f++] = sp * vx; z[f++] = sp * vy; z[f++] = sp * r; z[f++] = sp * a;
  z[f++] = cp * vx; z[f++] = cp * vy; z[f++] = cp * r; z[f++] = cp * a;
  z[f++] = sd * vx; z[f++] = sd * vy; z[f++] = sd * r;
  z[f++] = cd * vx; z[f++] = cd * vy; z[f++] = cd * r;
  z[f++] = a * sd;
}

// Register blocks of the accumulation: thread t of waves 1..3 owns rows
// a0 .. a0 + 3 by columns b0 .. b0 + 5 of Z^T Z, so a tile row costs it 10
// LDS reads for 24 FMAs; the 16 x 12 blocks fill those three waves exactly.
// Wave 0 lifts the next tile into the other LDS buffer meanwhile, so a tile
// costs the longer of the lift and the accumulation, not their sum.  Each
// entry still sums the rows in their order.
constexpr int kGa = 4, kGb = 6;
constexpr int kGaBlocks = MPMI_MAX_DIM / kGa;            // 16
constexpr int kGbBlocks = (kFitCols + kGb - 1) / kGb;    // 12
constexpr int kZCols = kGbBlocks * kGb;                  // 72: every block's columns lie in the row
constexpr int kZStride = kZCols + 2;                     // 16-byte aligned rows
static_assert(kGaBlocks * kGbBlocks == kFitThreads - 64, "one register block per thread of waves 1..3");
static_assert(MPMI_MAX_DIM % kGa == 0, "feature blocks");
static_assert(kFitRows == 64, "wave 0 lifts one row per lane");

// Right-hand sides: ny columns, either Y itself (yc0 < 0; ny = n) or, for the
// lifted operator, features yc0 .. yc0 + ny - 1 of psi(Y_t, U_t) (the input
// held over the step), lifted on the fly like the rows of Psi.
__global__ void __launch_bounds__(kFitThreads)
gram_kernel(mpmi_system sys, int D, int ny, int yc0, const double* __restrict__ X, const double* __restrict__ U,
            const double* __restrict__ Y, long long T, double* __restrict__ part) {
  __shared__ __attribute__((aligned(16))) double Z[2][kFitRows][kZStride];
  const int n = sys.n_state, m = sys.n_input;
  const int C = D + ny;
  const int E = D * C;
  const bool lifter = threadIdx.x < 64;
  const int blk = (int)threadIdx.x - 64;
  const int ab = blk / kGbBlocks, bb = blk % kGbBlocks;
  const int a0 = ab * kGa, b0 = bb * kGb;
  const bool active = !lifter && a0 < D && b0 < C;
  double acc[kGa][kGb];
#pragma unroll
  for (int i = 0; i < kGa; ++i)
#pragma unroll
    for (int j = 0; j < kGb; ++j) acc[i][j] = 0.0;
  const long long ntiles = (T + kFitRows - 1) / kFitRows;
  // This workgroup's tiles: blockIdx.x + k * gridDim.x, k = 0 .. count - 1.
  const long long count = blockIdx.x < ntiles ? (ntiles - 1 - blockIdx.x) / gridDim.x + 1 : 0;
  auto lift_tile = [&](long long k, int buf) {
    const long long r = (blockIdx.x + k * gridDim.x) * kFitRows + threadIdx.x;
    double* z = Z[buf][threadIdx.x];
    if (r < T) {
      if (yc0 >= 0) {
        // psi(Y_t, U_t) into the row first, its chunk moved past the D features
        lift_row(sys, Y + r * n, U + r * m, z);
        for (int q = 0; q < ny; ++q) z[D + q] = z[yc0 + q];
      } else {
        for (int q = 0; q < ny; ++q) z[D + q] = Y[r * n + q];
      }
      lift_row(sys, X + r * n, U + r * m, z);
    } else {
      for (int q = 0; q < C; ++q) z[q] = 0.0;
    }
    for (int q = C; q < kZCols; ++q) z[q] = 0.0;
  };
  if (lifter && count > 0) lift_tile(0, 0);
  __syncthreads();
  for (long long k = 0; k < count; ++k) {
    if (lifter) {
      if (k + 1 < count) lift_tile(k + 1, (int)((k + 1) & 1));
    } else if (active) {
      const int buf = (int)(k & 1);
#pragma unroll 4
      for (int rr = 0; rr < kFitRows; ++rr) {
        double av[kGa], bv[kGb];
#pragma unroll
        for (int i = 0; i < kGa; ++i) av[i] = Z[buf][rr][a0 + i];
#pragma unroll
        for (int j = 0; j < kGb; ++j) bv[j] = Z[buf][rr][b0 + j];
#pragma unroll
        for (int i = 0; i < kGa; ++i)
#pragma unroll
          for (int j = 0; j < kGb; ++j) acc[i][j] = fma(av[i], bv[j], acc[i][j]);
      }
    }
    __syncthreads();
  }
  if (!active) return;
  double* out = part + (size_t)blockIdx.x * E;
#pragma unroll
  for (int i = 0; i < kGa; ++i)
#pragma unroll
    for (int j = 0; j < kGb; ++j)
      if (a0 + i < D && b0 + j < C) out[(a0 + i) * C + b0 + j] = acc[i][j];
}

// tot[e] = sum over the parts of part[p][e], in a fixed order: the
// kReduceWays threads of element e sum parts p = q, q + kReduceWays, ...
// (q = 0 .. kReduceWays - 1), then one of them adds the partial sums in q
// order.  A workgroup covers kReduceElems elements (lanes of one q read
// consecutive elements); the grid spreads the ~4,500 elements of the race
// car over ~280 workgroups.
constexpr int kReduceElems = 16, kReduceWays = 16;
__global__ void __launch_bounds__(kReduceElems * kReduceWays)
reduce_kernel(int nparts, int E, const double* __restrict__ part, double* __restrict__ tot) {
  __shared__ double qs[kReduceWays][kReduceElems];
  const int el = threadIdx.x % kReduceElems, q = threadIdx.x / kReduceElems;
  const int e = blockIdx.x * kReduceElems + el;
  double s = 0.0;
  if (e < E) {
#pragma unroll 4
    for (int p = q; p < nparts; p += kReduceWays) s += part[(size_t)p * E + e];
  }
  qs[q][el] = s;
  __syncthreads();
  if (q == 0 && e < E) {
    double t = qs[0][el];
#pragma unroll
    for (int k = 1; k < kReduceWays; ++k) t += qs[k][el];
    tot[e] = t;
  }
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

// The factor as lane i keeps it in registers: m[k] = L_ik for k < i (its
// row) and L_ki for k > i (its column), zero past D.  The forward solve uses
// lane i's residual only up to step i and the backward solve only down to
// step i, so each may subtract the other half's entries after that point; a
// solve step is then a multiply, a broadcast and an FMA, with no memory
// access in the serial chain.
__device__ __forceinline__ void load_packed_factor(const double (&L)[MPMI_MAX_DIM][MPMI_MAX_DIM + 1], int D, int lane,
                                                   double (&m)[MPMI_MAX_DIM]) {
  const bool own = lane < D;
#pragma unroll
  for (int k = 0; k < MPMI_MAX_DIM; ++k)
    m[k] = (own && k < D && k != lane) ? (k < lane ? L[lane][k] : L[k][lane]) : 0.0;
}

// L L^T y = b: lane i holds b_i and rinv = 1 / L_ii (0 past D) and returns
// y_i.  Step k of the forward solve fixes z_k = r_k / L_kk once lane k's
// residual is complete; the backward solve runs from the last row up.
__device__ __forceinline__ double packed_cholesky_solve(const double (&m)[MPMI_MAX_DIM], int lane, double rinv,
                                                        double b) {
  double r = b, z = 0.0;
#pragma unroll
  for (int k = 0; k < MPMI_MAX_DIM; ++k) {  // L z = b
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
  return y;
}

// Orders this wave's LDS accesses before and after it (the lanes of a wave
// exchange values through LDS with no workgroup barrier).
__device__ __forceinline__ void wave_lds_sync() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }

// Largest eigenvalue of the symmetric matrix whose row `lane` the lane holds
// in a[] (rows and columns past D zero) by 60 steps of power iteration from
// v0: the Rayleigh quotient (w . v) / (v . v), w = A v, of the last step.
// The iterate reaches every lane through vb (this wave's 64 doubles of LDS)
// as broadcast reads.  Between steps it is rescaled by the hardware's
// reciprocal square root of w . w: the quotient does not depend on the
// scale, so no exact square root or division sits in the steps' chain.
__device__ __forceinline__ double power_rayleigh(const double (&a)[MPMI_MAX_DIM], bool own, int lane, double v0,
                                                 double* vb) {
  double v = own ? v0 : 0.0, w = 0.0;
  for (int it = 0; it < 60; ++it) {
    vb[lane] = v;
    wave_lds_sync();
    double w0 = 0.0, w1 = 0.0, w2 = 0.0, w3 = 0.0;
#pragma unroll
    for (int j = 0; j < MPMI_MAX_DIM; j += 4) {
      w0 = fma(a[j], vb[j], w0);
      w1 = fma(a[j + 1], vb[j + 1], w1);
      w2 = fma(a[j + 2], vb[j + 2], w2);
      w3 = fma(a[j + 3], vb[j + 3], w3);
    }
    w = (w0 + w1) + (w2 + w3);
    if (it + 1 < 60) v = w * __builtin_amdgcn_rsq(wave_sum(w * w));
  }
  return wave_sum(w * v) / wave_sum(v * v);
}

// One workgroup.  tot holds [D][C]: G = columns 0..D-1, A = columns D..D+n-1.
__global__ void __launch_bounds__(kFitThreads)
solve_kernel(int n, int D, long long T, double ridge, const double* __restrict__ tot, double* __restrict__ K,
             FitInfo* __restrict__ info) {
  __shared__ double L[MPMI_MAX_DIM][MPMI_MAX_DIM + 1];
  __shared__ __attribute__((aligned(16))) double Lt[MPMI_MAX_DIM][MPMI_MAX_DIM + 2];  // (L^-1)^T (wave 0)
  __shared__ __attribute__((aligned(16))) double Lz[MPMI_MAX_DIM][MPMI_MAX_DIM + 2];  // strictly lower L, then G_s^-1
  __shared__ double B[MPMI_MAX_DIM][MPMI_MAX_STATE];
  __shared__ double sc[MPMI_MAX_DIM], srinv[MPMI_MAX_DIM], piv[MPMI_MAX_DIM];
  __shared__ __attribute__((aligned(16))) double vbuf[2][MPMI_MAX_DIM];
  __shared__ int bad;
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int C = D + n;
  if (t == 0) bad = 0;
  for (int f = t; f < D; f += blockDim.x) {
    const double g = tot[(size_t)f * C + f];
    const double s = sqrt(g / (double)T);
    sc[f] = s > 0.0 ? s : 1.0;
  }
  __syncthreads();
  // Thread (wave w, lane j) holds entries (w + 4r, j), r = 0..15, of G_s in
  // registers through the factorisation; G_s itself also goes to L, whose
  // upper triangle the condition estimate reads.  Loads use clamped (valid)
  // indices so that none waits behind a branch.
  constexpr int kRowsPerWave = MPMI_MAX_DIM / 4;
  double a[kRowsPerWave];
  {
    const int jc = min(lane, D - 1);
#pragma unroll
    for (int r = 0; r < kRowsPerWave; ++r) a[r] = tot[(size_t)min(wave + 4 * r, D - 1) * C + jc];
#pragma unroll
    for (int r = 0; r < kRowsPerWave; ++r) {
      const int i = wave + 4 * r;
      a[r] = (i < D && lane < D) ? a[r] / (sc[i] * sc[lane]) + (i == lane ? ridge : 0.0) : 0.0;
      if (i < D && lane < D) L[i][lane] = a[r];
    }
  }
  for (int e = t; e < D * n; e += blockDim.x) {
    const int i = e / n, j = e % n;
    B[i][j] = tot[(size_t)i * C + D + j] / sc[i];
  }
  // Cholesky, right-looking, on the register copy; one barrier per two
  // columns.  With c_k column k before its own step (entries not yet
  // scaled) and d_k its pivot, step k subtracts c_ik c_jk / d_k from every
  // entry (i, j) with j > k (entries above the diagonal become garbage and
  // are never read).  Columns k and k + 1 as they stand before step k are
  // published in LDS by their owners, the threads of lanes k and k + 1, as
  // col[.][0 or 1][w][r] = entry (w + 4r, column).  Each thread then applies
  // steps k and k + 1 itself, forming the step-k update of column k + 1 that
  // it needs exactly as lane k + 1 forms it (so the factor is the
  // one-column-per-step factor, bit for bit); the threads of lanes k + 2 and
  // k + 3 publish the next pair.  The pair buffers alternate.  The pivots
  // are kept, and each column is scaled into the factor (L_ik = c_i /
  // sqrt(d_k), L_kk = sqrt(d_k)) after the loop, off the steps' chain.
  __shared__ __attribute__((aligned(16))) double col[2][2][4][kRowsPerWave];
  if (lane < 2)
#pragma unroll
    for (int r = 0; r < kRowsPerWave; ++r) col[0][lane][wave][r] = a[r];
  __syncthreads();
  const double pivot_floor = 1e-14 * (double)T;
  // A pivot below the floor marks the fit singular and is replaced by 1.
  auto pivot = [&](double d) {
    if (!(d > pivot_floor)) {
      if (t == 0) bad = 1;
      d = 1.0;
    }
    return d;
  };
  // 1 / d: the hardware estimate and two Newton steps (d > 0, normal).
  auto recip = [](double d) {
    double rd = __builtin_amdgcn_rcp(d);
    rd = fma(rd, fma(-d, rd, 1.0), rd);
    return fma(rd, fma(-d, rd, 1.0), rd);
  };
  int k = 0;
  for (; k + 1 < D; k += 2) {
    const double(*c0)[kRowsPerWave] = col[(k >> 1) & 1][0];
    const double(*c1)[kRowsPerWave] = col[(k >> 1) & 1][1];
    const int k1 = k + 1;
    const double d0 = pivot(c0[k & 3][k >> 2]);
    const double r0 = recip(d0);
    const double t01 = c0[k1 & 3][k1 >> 2] * r0;  // step k's multiplier of column k + 1
    const double d1 = pivot(fma(-c0[k1 & 3][k1 >> 2], t01, c1[k1 & 3][k1 >> 2]));
    if (t == 0) {
      piv[k] = d0;
      piv[k1] = d1;
    }
    if (lane > k) {
      const double tj0 = c0[lane & 3][lane >> 2] * r0;
#pragma unroll
      for (int r = 0; r < kRowsPerWave; ++r) a[r] = fma(-c0[wave][r], tj0, a[r]);
    }
    if (lane > k1) {
      const double r1 = recip(d1);
      const double tj1 = fma(-c0[lane & 3][lane >> 2], t01, c1[lane & 3][lane >> 2]) * r1;
#pragma unroll
      for (int r = 0; r < kRowsPerWave; ++r) a[r] = fma(-fma(-c0[wave][r], t01, c1[wave][r]), tj1, a[r]);
    }
    if (lane == k + 2 || lane == k + 3)
#pragma unroll
      for (int r = 0; r < kRowsPerWave; ++r) col[((k >> 1) + 1) & 1][lane - k - 2][wave][r] = a[r];
    __syncthreads();
  }
  if (k < D && t == 0) piv[k] = pivot(col[(k >> 1) & 1][0][k & 3][k >> 2]);  // odd D: the last column
  __syncthreads();
  if (lane < D) {
    const double lkk = sqrt(piv[lane]), rs = 1.0 / lkk;
#pragma unroll
    for (int r = 0; r < kRowsPerWave; ++r) {
      const int i = wave + 4 * r;
      a[r] = i == lane ? lkk : a[r] * rs;
    }
  }
  // The factor to L (lower triangle and diagonal; G_s stays above), and its
  // strictly lower part, zero elsewhere, to Lz for the inverse.
#pragma unroll
  for (int r = 0; r < kRowsPerWave; ++r) {
    const int i = wave + 4 * r;
    if (i < D && lane <= i) L[i][lane] = a[r];
    Lz[i][lane] = (i < D && lane < i) ? a[r] : 0.0;
  }
  __syncthreads();
  // Triangular solves and the condition estimate run one wave per task, the
  // tasks concurrently: lane i owns row i (D <= 64), the wave's lockstep
  // orders the steps, and the values a step needs from another lane arrive
  // by lane broadcast or through LDS written by the same wave, so no
  // workgroup barrier is involved until the inverse is complete.  The factor
  // is read-only from here on.
  const bool own = lane < D;
  const double rinv = own ? 1.0 / L[lane][lane] : 0.0;
  __shared__ double s_lmax, s_lmin_inv;
  if (wave >= 2) {
    // K: waves 2 and 3 solve the right-hand sides c = wave - 2, wave, ...
    double m[MPMI_MAX_DIM];
    load_packed_factor(L, D, lane, m);
    for (int c = wave - 2; c < n; c += 2) {
      const double k = packed_cholesky_solve(m, lane, rinv, own ? B[lane][c] : 0.0);
      if (own) K[(size_t)lane * n + c] = k / sc[lane];
    }
  } else if (wave == 1) {
    // Largest eigenvalue of the scaled Gram matrix G_s (from its upper
    // triangle and the diagonal of L L^T); lane i holds row i.
    double diag = 0.0;
    if (own)
      for (int k = 0; k <= lane; ++k) diag += L[lane][k] * L[lane][k];
    double grow[MPMI_MAX_DIM];
#pragma unroll
    for (int j = 0; j < MPMI_MAX_DIM; ++j)
      grow[j] = (own && j < D) ? (lane == j ? diag : (lane < j ? L[lane][j] : L[j][lane])) : 0.0;
    const double lmax = power_rayleigh(grow, own, lane, 1.0 + 0.01 * lane, vbuf[1]);
    if (lane == 0) s_lmax = lmax;
  } else {
    // Smallest eigenvalue of G_s as 1 / the largest of G_s^-1 = L^-T L^-1
    // (power iteration on G_s^-1 from the start vector is the inverse
    // iteration on G_s through the factor).  Here lane c forms column c of
    // L^-1 by forward substitution into row c of Lt = (L^-1)^T: row k is a
    // dot product of the strictly lower row k of L with the entries found
    // so far, over blocks of 16 up to k.  Loops, not unrolled code, so the
    // task stays in the instruction cache beside the other waves'.
    srinv[lane] = rinv;
#pragma unroll
    for (int k = 0; k < MPMI_MAX_DIM; ++k) Lt[lane][k] = 0.0;
    wave_lds_sync();
    for (int k = 0; k < D; ++k) {
      double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
      for (int j0 = 0; j0 < k; j0 += 16) {
#pragma unroll
        for (int j = j0; j < j0 + 16; j += 4) {
          s0 = fma(Lz[k][j], Lt[lane][j], s0);
          s1 = fma(Lz[k][j + 1], Lt[lane][j + 1], s1);
          s2 = fma(Lz[k][j + 2], Lt[lane][j + 2], s2);
          s3 = fma(Lz[k][j + 3], Lt[lane][j + 3], s3);
        }
      }
      Lt[lane][k] = ((k == lane ? 1.0 : 0.0) - ((s0 + s1) + (s2 + s3))) * srinv[k];
    }
  }
  __syncthreads();
  // G_s^-1 into Lz (no longer needed), its rows spread over the four waves:
  // (G_s^-1)_ji = sum_{k >= j} (L^-1)_ki (L^-1)_kj, lane i of row j, the
  // entries of L^-1 above the diagonal being zero.
  for (int j = wave; j < D; j += 4) {
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    for (int k0 = j & ~15; k0 < MPMI_MAX_DIM; k0 += 16) {
#pragma unroll
      for (int k = k0; k < k0 + 16; k += 4) {
        s0 = fma(Lt[lane][k], Lt[j][k], s0);
        s1 = fma(Lt[lane][k + 1], Lt[j][k + 1], s1);
        s2 = fma(Lt[lane][k + 2], Lt[j][k + 2], s2);
        s3 = fma(Lt[lane][k + 3], Lt[j][k + 3], s3);
      }
    }
    Lz[j][lane] = (s0 + s1) + (s2 + s3);
  }
  __syncthreads();
  if (wave == 0) {
    double gi[MPMI_MAX_DIM];
#pragma unroll
    for (int j = 0; j < MPMI_MAX_DIM; ++j) gi[j] = (own && j < D) ? Lz[j][lane] : 0.0;
    const double lmin_inv = power_rayleigh(gi, own, lane, 1.0 - 0.01 * lane, vbuf[0]);
    if (lane == 0) s_lmin_inv = lmin_inv;
  }
  __syncthreads();
  if (t == 0) {
    info->status = bad ? MPMI_ESINGULAR : MPMI_OK;
    const double cg = s_lmax * s_lmin_inv;
    info->cond = cg > 0.0 ? sqrt(cg) : INFINITY;
  }
}

// Workspace: partial sums, totals, the info record (256 bytes at
// fit_info_offset()), then a [D][MPMI_MAX_STATE] chunk of the lifted solution.
size_t fit_info_offset() { return (size_t)(kFitBlocks + 1) * MPMI_MAX_DIM * kFitCols * sizeof(double); }
size_t fit_workspace_bytes() { return fit_info_offset() + 256 + (size_t)MPMI_MAX_DIM * MPMI_MAX_STATE * 8; }

// One least-squares solve with ny right-hand sides (see gram_kernel).
static hipError_t fit_columns(const mpmi_system& sys, int dim, int ny, int yc0, const double* X, const double* U,
                              const double* Y, int64_t T, double ridge, double* K_out, void* work, hipStream_t st) {
  const int E = dim * (dim + ny);
  long long ntiles = (T + kFitRows - 1) / kFitRows;
  const int nparts = (int)(ntiles < kFitBlocks ? ntiles : kFitBlocks);
  double* part = (double*)work;
  double* tot = part + (size_t)kFitBlocks * MPMI_MAX_DIM * kFitCols;
  FitInfo* info = (FitInfo*)(tot + (size_t)MPMI_MAX_DIM * kFitCols);
  gram_kernel<<<nparts, kFitThreads, 0, st>>>(sys, dim, ny, yc0, X, U, Y, (long long)T, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  reduce_kernel<<<(E + kReduceElems - 1) / kReduceElems, kReduceElems * kReduceWays, 0, st>>>(nparts, E, part, tot);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  solve_kernel<<<1, kFitThreads, 0, st>>>(ny, dim, (long long)T, ridge, tot, K_out, info);
  return hipGetLastError();
}

hipError_t launch_fit(const mpmi_system& sys, int dim, const double* X, const double* U, const double* Y,
                      int64_t T, double ridge, double* K_out, void* work, hipStream_t st) {
  return fit_columns(sys, dim, sys.n_state, -1, X, U, Y, T, ridge, K_out, work, st);
}

// The lifted operator K (dim x dim, targets psi(Y_t, U_t)): the same scaled
// least-squares problem solved for MPMI_MAX_STATE target columns at a time;
// each chunk's [dim][ny] solution goes from the workspace into its columns of
// K_out.  Every chunk recomputes the Gram matrix (a set-up call: the cost is
// dim / 8 fits).  The status and condition estimate left in the workspace
// are those of the last chunk (the Gram matrix, and so both, are the same).
hipError_t launch_fit_lifted(const mpmi_system& sys, int dim, const double* X, const double* U, const double* Y,
                             int64_t T, double ridge, double* K_out, void* work, hipStream_t st) {
  double* Kc = (double*)((char*)work + fit_info_offset() + 256);
  for (int c0 = 0; c0 < dim; c0 += MPMI_MAX_STATE) {
    const int ny = dim - c0 < MPMI_MAX_STATE ? dim - c0 : MPMI_MAX_STATE;
    hipError_t e = fit_columns(sys, dim, ny, c0, X, U, Y, T, ridge, Kc, work, st);
    if (e != hipSuccess) return e;
    e = hipMemcpy2DAsync(K_out + c0, (size_t)dim * sizeof(double), Kc, (size_t)ny * sizeof(double),
                         (size_t)ny * sizeof(double), (size_t)dim, hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace mpmi
