// Sparsity-promoting basis selection (Sec. IV-A and Sec. V-C-3: from a
// library of random basis functions, keep the ones most relevant to the
// dynamics, by the ADMM of Jovanovic, Schmid and Nichols 2014, a basis
// function's row of coefficients being the unit kept or dropped), FP64.
//
// Four launches, then one synchronous read-back:
//   1. Gram of the augmented data Z = [Psi | Y] (T x (L + n)), the library
//      functions lifted on the fly from (X, U) into LDS tiles of 32 rows;
//      thread b of a workgroup owns one 8 x 8 block of the upper block
//      triangle in registers (at most 21 x 22 / 2 = 231 blocks), each
//      workgroup a set of row tiles, partial sums per workgroup;
//   2. fixed-order reduction of the partials (deterministic);
//   3. one workgroup: RMS scaling of the columns, G_s = Psi_s' Psi_s / T and
//      A_s = Psi_s' Y_s / T, and the inverse M = (G_s + rho/2 I)^-1 by
//      in-place Gauss-Jordan elimination in global memory (G_s + rho/2 I is
//      symmetric positive definite, so no pivoting);
//   4. the ADMM, one workgroup per penalty gamma (a whole penalty path in one
//      launch): K <- M (A + rho/2 (B - Lam/rho)), B <- row-wise block soft
//      threshold of K + Lam/rho at gamma/rho, Lam <- Lam + rho (K - B), for a
//      fixed number of iterations; B, K, Lam live in LDS, M is read from L2.
#include <hip/hip_runtime.h>

#include "mpmi_device.hpp"
#include "mpmi_launch.hpp"

namespace mpmi {

constexpr int kSelCols = MPMI_MAX_LIBRARY + MPMI_MAX_STATE;  // augmented columns
constexpr int kSelRows = 32;                                 // rows per LDS tile
constexpr int kSelBlk = 8;                                   // register block side
constexpr int kSelNB = (kSelCols + kSelBlk - 1) / kSelBlk;   // 21 block rows
constexpr int kSelThreads = 256;
constexpr int kSelParts = 128;                               // Gram workgroups
constexpr int kSelLdsPitch = kSelCols + 1;                   // LDS row pitch (doubles)
static_assert(kSelNB * (kSelNB + 1) / 2 <= kSelThreads, "one upper block per thread");

struct SelLibrary {
  int32_t n, m, na, L;
  int8_t kind[MPMI_MAX_ATOMS], var[MPMI_MAX_ATOMS];
  uint8_t fa[MPMI_MAX_LIBRARY], fb[MPMI_MAX_LIBRARY];
};

// Upper block (bi, bj), bi <= bj, of block index b in row-major order over
// the upper triangle of an nb x nb block grid.
__device__ __forceinline__ void upper_block(int b, int nb, int* bi, int* bj) {
  int i = 0, rem = b;
  while (rem >= nb - i) {
    rem -= nb - i;
    ++i;
  }
  *bi = i;
  *bj = i + rem;
}

__global__ void __launch_bounds__(kSelThreads)
sel_gram_kernel(SelLibrary lib, const double* __restrict__ X, const double* __restrict__ U,
                const double* __restrict__ Y, long long T, double* __restrict__ part) {
  __shared__ double Z[kSelRows][kSelLdsPitch];
  __shared__ double At[kSelRows][MPMI_MAX_ATOMS];
  const int t = threadIdx.x;
  const int n = lib.n, m = lib.m, na = lib.na, L = lib.L, C = L + n;
  const int nb = (C + kSelBlk - 1) / kSelBlk;
  const int nblocks = nb * (nb + 1) / 2;
  int bi = 0, bj = 0;
  if (t < nblocks) upper_block(t, nb, &bi, &bj);
  double acc[kSelBlk][kSelBlk];
#pragma unroll
  for (int i = 0; i < kSelBlk; ++i)
#pragma unroll
    for (int j = 0; j < kSelBlk; ++j) acc[i][j] = 0.0;
  const long long ntiles = (T + kSelRows - 1) / kSelRows;
  for (long long tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const long long r0 = tile * kSelRows;
    // atoms of each row (rows past T are zero everywhere below)
    for (int e = t; e < kSelRows * na; e += kSelThreads) {
      const int r = e / na, q = e - r * na;
      const long long row = r0 + r;
      double a = 0.0;
      if (row < T) {
        const int v = lib.var[q], kd = lib.kind[q];
        const double w = v < n ? X[row * n + v] : U[row * m + (v - n)];
        a = kd == MPMI_ATOM_VAR ? w : kd == MPMI_ATOM_SIN ? sin(w) : kd == MPMI_ATOM_COS ? cos(w) : 1.0;
      }
      At[r][q] = a;
    }
    __syncthreads();
    for (int e = t; e < kSelRows * kSelCols; e += kSelThreads) {
      const int r = e / kSelCols, c = e - r * kSelCols;
      const long long row = r0 + r;
      double z = 0.0;
      if (row < T) {
        if (c < L) z = At[r][lib.fa[c]] * At[r][lib.fb[c]];
        else if (c < C) z = Y[row * n + (c - L)];
      }
      Z[r][c] = z;
    }
    __syncthreads();
    if (t < nblocks) {
      for (int r = 0; r < kSelRows; ++r) {
        double a[kSelBlk], b[kSelBlk];
#pragma unroll
        for (int i = 0; i < kSelBlk; ++i) {
          a[i] = Z[r][bi * kSelBlk + i];
          b[i] = Z[r][bj * kSelBlk + i];
        }
#pragma unroll
        for (int i = 0; i < kSelBlk; ++i)
#pragma unroll
          for (int j = 0; j < kSelBlk; ++j) acc[i][j] = fma(a[i], b[j], acc[i][j]);
      }
    }
    __syncthreads();
  }
  if (t < nblocks) {
    double* P = part + (size_t)blockIdx.x * kSelCols * kSelCols;
#pragma unroll
    for (int i = 0; i < kSelBlk; ++i)
#pragma unroll
      for (int j = 0; j < kSelBlk; ++j) P[(size_t)(bi * kSelBlk + i) * kSelCols + bj * kSelBlk + j] = acc[i][j];
  }
}

// Sum of the parts' upper blocks, parts in order (deterministic).
__global__ void sel_reduce_kernel(const double* __restrict__ part, int nparts, int C, double* __restrict__ G) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= kSelCols * kSelCols) return;
  const int i = e / kSelCols, j = e - i * kSelCols;
  if (i >= C || j >= C || i / kSelBlk > j / kSelBlk) return;
  double s = 0.0;
  for (int p = 0; p < nparts; ++p) s += part[(size_t)p * kSelCols * kSelCols + e];
  G[e] = s;
}

// Entry (i, j) of the symmetric Gram from its stored upper blocks.
__device__ __forceinline__ double gram_at(const double* __restrict__ G, int i, int j) {
  return (i / kSelBlk <= j / kSelBlk) ? G[(size_t)i * kSelCols + j] : G[(size_t)j * kSelCols + i];
}

// Scaling, the scaled problem and M = (G_s + rho/2 I)^-1 (one workgroup).
// W: L x L work/result; As: L x n; sc: L + n column scales.
__global__ void __launch_bounds__(1024)
sel_prepare_kernel(const double* __restrict__ G, int L, int n, long long T, double rho, double* __restrict__ W,
                   double* __restrict__ MT, double* __restrict__ As, double* __restrict__ sc) {
  __shared__ double s[kSelCols];
  __shared__ double pinv_s;
  const int t = threadIdx.x, nt = blockDim.x;
  const int C = L + n;
  const double Td = (double)T;
  for (int c = t; c < C; c += nt) {
    const double v = sqrt(gram_at(G, c, c) / Td);
    s[c] = v > 0.0 ? v : 1.0;
    sc[c] = s[c];
  }
  __syncthreads();
  for (int e = t; e < L * L; e += nt) {
    const int i = e / L, j = e - i * L;
    W[e] = gram_at(G, i, j) / (s[i] * s[j] * Td) + (i == j ? 0.5 * rho : 0.0);
  }
  for (int e = t; e < L * n; e += nt) {
    const int f = e / n, k = e - f * n;
    As[e] = gram_at(G, f, L + k) / (s[f] * s[L + k] * Td);
  }
  __threadfence_block();
  __syncthreads();
  // In-place Gauss-Jordan: after step k, column k holds the inverse's column.
  for (int k = 0; k < L; ++k) {
    if (t == 0) pinv_s = 1.0 / W[(size_t)k * L + k];
    __syncthreads();
    const double pinv = pinv_s;
    for (int j = t; j < L; j += nt) W[(size_t)k * L + j] = (j == k) ? pinv : W[(size_t)k * L + j] * pinv;
    __threadfence_block();
    __syncthreads();
    for (int e = t; e < L * L; e += nt) {
      const int i = e / L, j = e - i * L;
      if (i != k && j != k) W[e] = fma(-W[(size_t)i * L + k], W[(size_t)k * L + j], W[e]);
    }
    __threadfence_block();
    __syncthreads();
    for (int i = t; i < L; i += nt)
      if (i != k) W[(size_t)i * L + k] = -W[(size_t)i * L + k] * pinv;
    __threadfence_block();
    __syncthreads();
  }
  // M transposed, so that the ADMM's row-per-thread products read it with
  // coalesced loads (MT[q][f] = M[f][q]).
  for (int e = t; e < L * L; e += nt) {
    const int i = e / L, j = e - i * L;
    MT[(size_t)j * L + i] = W[e];
  }
}

// ADMM for penalty gamma[blockIdx.x]; B_out unscaled (B_s[f][j] s_y[j] / s_f).
__global__ void __launch_bounds__(kSelThreads)
sel_admm_kernel(const double* __restrict__ MT, const double* __restrict__ As, const double* __restrict__ sc,
                const double* __restrict__ gammas, int L, int n, double rho, int iters, double* __restrict__ B_out,
                uint8_t* __restrict__ support, double* __restrict__ resid) {
  __shared__ double B[MPMI_MAX_LIBRARY][MPMI_MAX_STATE], Lam[MPMI_MAX_LIBRARY][MPMI_MAX_STATE];
  __shared__ double K[MPMI_MAX_LIBRARY][MPMI_MAX_STATE], R[MPMI_MAX_LIBRARY][MPMI_MAX_STATE];
  __shared__ double red_p[kSelThreads], red_d[kSelThreads];
  const int t = threadIdx.x;
  const int g = blockIdx.x;
  const double kappa = gammas[g] / rho;
  for (int e = t; e < MPMI_MAX_LIBRARY * MPMI_MAX_STATE; e += kSelThreads) {
    (&B[0][0])[e] = 0.0;
    (&Lam[0][0])[e] = 0.0;
  }
  __syncthreads();
  double prim = 0.0, dual = 0.0;
  for (int it = 0; it < iters; ++it) {
    for (int e = t; e < L * n; e += kSelThreads) {
      const int f = e / n, j = e - f * n;
      R[f][j] = As[e] + 0.5 * rho * (B[f][j] - Lam[f][j] / rho);
    }
    __syncthreads();
    if (t < L) {
      double y[MPMI_MAX_STATE];
#pragma unroll
      for (int j = 0; j < MPMI_MAX_STATE; ++j) y[j] = 0.0;
      for (int q = 0; q < L; ++q) {
        const double mq = MT[(size_t)q * L + t];
#pragma unroll
        for (int j = 0; j < MPMI_MAX_STATE; ++j)
          if (j < n) y[j] = fma(mq, R[q][j], y[j]);
      }
#pragma unroll
      for (int j = 0; j < MPMI_MAX_STATE; ++j)
        if (j < n) K[t][j] = y[j];
    }
    __syncthreads();
    prim = dual = 0.0;
    if (t < L) {
      double v[MPMI_MAX_STATE], nrm2 = 0.0;
#pragma unroll
      for (int j = 0; j < MPMI_MAX_STATE; ++j) {
        v[j] = j < n ? K[t][j] + Lam[t][j] / rho : 0.0;
        nrm2 = fma(v[j], v[j], nrm2);
      }
      const double nrm = sqrt(nrm2);
      const double fac = nrm > kappa ? 1.0 - kappa / nrm : 0.0;
#pragma unroll
      for (int j = 0; j < MPMI_MAX_STATE; ++j) {
        if (j < n) {
          const double bn = v[j] * fac;
          const double dp = K[t][j] - bn, dd = bn - B[t][j];
          prim = fma(dp, dp, prim);
          dual = fma(dd, dd, dual);
          Lam[t][j] = Lam[t][j] + rho * dp;
          B[t][j] = bn;
        }
      }
    }
    __syncthreads();
  }
  if (t < L) {
    bool any = false;
#pragma unroll
    for (int j = 0; j < MPMI_MAX_STATE; ++j) {
      if (j < n) {
        B_out[((size_t)g * L + t) * n + j] = B[t][j] * sc[L + j] / sc[t];
        any |= B[t][j] != 0.0;
      }
    }
    support[(size_t)g * L + t] = any ? 1 : 0;
  }
  red_p[t] = prim;
  red_d[t] = dual;
  __syncthreads();
  if (t == 0) {
    double p = 0.0, d = 0.0;
    for (int i = 0; i < kSelThreads; ++i) {
      p += red_p[i];
      d += red_d[i];
    }
    resid[2 * g] = sqrt(p);
    resid[2 * g + 1] = rho * sqrt(d);
  }
}

// Workspace layout (doubles): parts [kSelParts][kSelCols^2], Gram
// [kSelCols^2], W and MT [L^2] each, As [L n], scales [kSelCols], gammas
// [n_gamma], resid [2 n_gamma].
size_t select_workspace_bytes(int n_gamma) {
  return sizeof(double) * ((size_t)(kSelParts + 1) * kSelCols * kSelCols +
                           2 * (size_t)MPMI_MAX_LIBRARY * MPMI_MAX_LIBRARY + (size_t)MPMI_MAX_LIBRARY * MPMI_MAX_STATE +
                           kSelCols + 3 * (size_t)n_gamma);
}

hipError_t launch_select_basis(const mpmi_library& lib, const double* X, const double* U, const double* Y, int64_t T,
                               const double* gammas_host, int n_gamma, double rho, int iters, double* B_out,
                               uint8_t* support, double* resid_host, void* work, hipStream_t st) {
  SelLibrary sl;
  sl.n = lib.n_state;
  sl.m = lib.n_input;
  sl.na = lib.n_atoms;
  sl.L = lib.n_feat;
  for (int q = 0; q < MPMI_MAX_ATOMS; ++q) {
    sl.kind[q] = lib.atom_kind[q];
    sl.var[q] = lib.atom_var[q];
  }
  for (int f = 0; f < MPMI_MAX_LIBRARY; ++f) {
    sl.fa[f] = lib.feat_a[f];
    sl.fb[f] = lib.feat_b[f];
  }
  const int L = sl.L, n = sl.n, C = L + n;
  double* part = (double*)work;
  double* Gm = part + (size_t)kSelParts * kSelCols * kSelCols;
  double* W = Gm + (size_t)kSelCols * kSelCols;
  double* MT = W + (size_t)MPMI_MAX_LIBRARY * MPMI_MAX_LIBRARY;
  double* As = MT + (size_t)MPMI_MAX_LIBRARY * MPMI_MAX_LIBRARY;
  double* sc = As + (size_t)MPMI_MAX_LIBRARY * MPMI_MAX_STATE;
  double* gam = sc + kSelCols;
  double* res = gam + n_gamma;
  hipError_t e = hipMemcpyAsync(gam, gammas_host, sizeof(double) * n_gamma, hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return e;
  const long long ntiles = (T + kSelRows - 1) / kSelRows;
  const int nparts = (int)(ntiles < kSelParts ? ntiles : kSelParts);
  sel_gram_kernel<<<nparts, kSelThreads, 0, st>>>(sl, X, U, Y, (long long)T, part);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  sel_reduce_kernel<<<(kSelCols * kSelCols + 255) / 256, 256, 0, st>>>(part, nparts, C, Gm);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  sel_prepare_kernel<<<1, 1024, 0, st>>>(Gm, L, n, (long long)T, rho, W, MT, As, sc);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  sel_admm_kernel<<<n_gamma, kSelThreads, 0, st>>>(MT, As, sc, gam, L, n, rho, iters, B_out, support, res);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (resid_host) {
    e = hipMemcpyAsync(resid_host, res, sizeof(double) * 2 * n_gamma, hipMemcpyDeviceToHost, st);
    if (e != hipSuccess) return e;
  }
  return hipStreamSynchronize(st);
}

}  // namespace mpmi
