// FP64 re-roll of the candidates an FP32 tick left in its rounding band
// (precision MPMI_PREC_FP32_RECHECK64).
//
// A minimal-intervention choice lies on the boundary of the safe input set
// whenever the user's own input is unsafe, so the candidate the selection
// picks is often one whose predicted margin is within FP32 rounding of zero.
// The FP32 tick therefore lists every candidate with such a margin at some
// checked step (with its FP32 verdict) instead of publishing it.  Outside the
// band the FP32 verdicts are exact, so the least key K* the tick published is
// the FP64 selection's unless a listed candidate of smaller key is safe in
// FP64.  A filter launch keeps the listed candidates whose key precedes K*
// (every listed one when nothing outside the band is safe, so that the
// fallback order is exact too); the others keep their FP32 verdicts.  The
// re-roll launch predicts each kept candidate again, from
// x_t with K, the basis, the process noise and the margins in FP64 (Sec.
// IV-A's prediction and Sec. IV-B's checks), writes its first violation and
// publishes its keys.  The last workgroup finalises the selection, which is
// then that of an FP64 rollout whenever the bands cover the FP32 margin error.
//
// The launch is latency-bound: a tick keeps from none to a few thousand
// candidates, each a serial H-step FP64 prediction.  The race car spreads one
// candidate over eight lanes (one output component each, the step's
// coefficients read from LDS) and holds eight per 64-lane workgroup; the
// described bases run one candidate per lane, the atoms going through a
// per-lane column of LDS.  The many-loop form lists (loop, candidate, model)
// entries and prunes by each loop's K* itself.
#include <hip/hip_runtime.h>

#include "mpmi_device.hpp"
#include "mpmi_launch.hpp"
#include "mpmi_tick_common.hpp"

namespace mpmi {

constexpr int kR64Block = 64;

// The coefficient pointer behind an opaque zero offset, taken at every step:
// without it the compiler hoists the loop-invariant coefficient loads out of
// the horizon loop, and the 162 doubles of the race-car step overflow the
// register file.
__device__ __forceinline__ const double* opaque_coeffs(const double* p) {
  int off = 0;
  asm volatile("" : "+s"(off));
  return p + off;
}

// First step s (1-based) of input segment g >= 1: the least s with
// ((s - 1) S) / H >= g, i.e. ceil(g H / S) + 1 (H + 1 when g >= S).  The
// horizon loop compares the step with it instead of dividing at every step.
__device__ __forceinline__ int segment_start(int g, int S, int H) { return (g * H + S - 1) / S + 1; }

// The safety set's FP64 constants, read in one batch (every component's
// limit, masked afterwards, rather than one load behind each component's
// test) so that the step can issue the reads early and wait once.
template <int NS, int DEG>
struct Safety64 {
  double lim[NS];
  double trk_lim, P[DEG + 1], Q[DEG];
  int mask, has_track;
};
template <int NS, int DEG>
__device__ __forceinline__ Safety64<NS, DEG> safety64(const Model64* __restrict__ m) {
  Safety64<NS, DEG> sc;
#pragma unroll
  for (int k = 0; k < NS; ++k) sc.lim[k] = m->comp_lim[k];
  sc.trk_lim = m->trk_lim;
#pragma unroll
  for (int k = 0; k <= DEG; ++k) sc.P[k] = m->trk_p[k];
#pragma unroll
  for (int k = 0; k < DEG; ++k) sc.Q[k] = m->trk_q[k];
  sc.mask = m->comp_mask;
  sc.has_track = m->has_track;
  return sc;
}

// Safety verdict of x in FP64: every boxed component strictly inside its
// limit and the track margin positive.  This is "least margin > 0" with
// the least margin NaN when a boxed component's or the track's margin is
// NaN: lim - |v| > 0 exactly when |v| < lim (the difference of two distinct
// doubles is never rounded to zero), and a NaN fails either comparison.  The
// tests are combined bitwise (a compare each, no branch).  The centreline
// radius r_c(phi) is the FP32 tick's Chebyshev form in FP64,
// P(cos phi) + sin phi * Q(cos phi) with the model's FP64 monomial
// coefficients, (cos phi, sin phi) = (x0, x1) / rho; Horner runs over a fixed
// DEG >= the model's highest harmonic (zero coefficients above it leave each
// partial sum unchanged).  NS: the components that can carry a box (6 for
// the race car, MPMI_MAX_STATE for the described bases).
template <int NS, int DEG>
__device__ __forceinline__ bool track_ok64(const Safety64<NS, DEG>& sc, const double* x) {
  if (!sc.has_track) return true;
  // 1 / rho by the hardware reciprocal square root and two Newton steps
  // (each at least doubles the correct bits), rho = r2 / rho: a shorter
  // dependent chain than a square root followed by a division.  r2 = 0 or
  // an infinite coordinate gives NaN (unsafe), as in the FP32 tick.
  const double r2 = fma(x[0], x[0], x[1] * x[1]);
  double inv = __builtin_amdgcn_rsq(r2);
  inv = inv * fma(-0.5 * r2, inv * inv, 1.5);
  inv = inv * fma(-0.5 * r2, inv * inv, 1.5);
  const double rho = r2 * inv;
  const double c1 = x[0] * inv, s1 = x[1] * inv;
  double P = sc.P[DEG];
#pragma unroll
  for (int k = DEG - 1; k >= 0; --k) P = fma3s(P, c1, sc.P[k]);
  double Q = sc.Q[DEG - 1];
#pragma unroll
  for (int k = DEG - 2; k >= 0; --k) Q = fma3s(Q, c1, sc.Q[k]);
  return fabs(rho - fma(s1, Q, P)) < sc.trk_lim;
}

// track_ok64 with no branch on has_track: the test is formed either way
// and a model without a track takes true.
template <int NS, int DEG>
__device__ __forceinline__ bool track_ok64_nb(const Safety64<NS, DEG>& sc, const double* x) {
  const double r2 = fma(x[0], x[0], x[1] * x[1]);
  double inv = __builtin_amdgcn_rsq(r2);
  inv = inv * fma(-0.5 * r2, inv * inv, 1.5);
  inv = inv * fma(-0.5 * r2, inv * inv, 1.5);
  const double rho = r2 * inv;
  const double c1 = x[0] * inv, s1 = x[1] * inv;
  double P = sc.P[DEG];
#pragma unroll
  for (int k = DEG - 1; k >= 0; --k) P = fma3s(P, c1, sc.P[k]);
  double Q = sc.Q[DEG - 1];
#pragma unroll
  for (int k = DEG - 2; k >= 0; --k) Q = fma3s(Q, c1, sc.Q[k]);
  return !sc.has_track | (fabs(rho - fma(s1, Q, P)) < sc.trk_lim);
}

template <int NS, int DEG>
__device__ __forceinline__ bool safe64(const Safety64<NS, DEG>& sc, const double* x) {
  bool ok = true;
#pragma unroll
  for (int k = 0; k < NS; ++k) ok &= (fabs(x[k]) < sc.lim[k]) | !((sc.mask >> k) & 1);
  return ok & track_ok64(sc, x);
}

// Alg. 2's z_i for step s: the FP32 tick's draws (same counter hash), the
// Box-Muller transform in FP64.
__device__ __forceinline__ void add_noise64(const Model64* __restrict__ m, uint64_t pre, int s, int n, double* x) {
#pragma unroll
  for (int q = 0; q < MPMI_MAX_STATE / 2; ++q) {
    if (2 * q < n) {
      const uint64_t h = hash_finish(pre, kNoiseSlot + 4ull * (uint64_t)(s - 1) + (uint64_t)q);
      const double u1 = ((double)(h >> 40) + 1.0) * 0x1p-24;
      const double u2 = (double)((h >> 16) & 0xFFFFFFull) * 0x1p-24;
      const double r = sqrt(-2.0 * log(u1));
      const double ang = 6.283185307179586 * u2;
      x[2 * q] = x[2 * q] + m->sigma[2 * q] * (r * cos(ang));
      if (2 * q + 1 < n) x[2 * q + 1] = x[2 * q + 1] + m->sigma[2 * q + 1] * (r * sin(ang));
    }
  }
}

// A basis given by its description: atoms of w = [x; u] into this lane's LDS
// column (stride kR64Block), then x' = sum_f atom[a_f] atom[b_f] K[f].
__device__ __forceinline__ void step64_described(const Model64* __restrict__ m, const double* __restrict__ K, int n,
                                                 int D, const double* u, double* x, double* at) {
  const int na = m->n_atoms;
  for (int q = 0; q < na; ++q) {
    const int kd = m->atom_kind[q], v = m->atom_var[q];
    double w = 0.0;
#pragma unroll
    for (int k = 0; k < MPMI_MAX_STATE; ++k) w = (v == k) ? x[k] : w;
#pragma unroll
    for (int j = 0; j < MPMI_MAX_INPUT; ++j) w = (v == n + j) ? u[j] : w;
    double a = 1.0;
    if (kd == MPMI_ATOM_VAR) a = w;
    else if (kd == MPMI_ATOM_SIN) a = sin(w);
    else if (kd == MPMI_ATOM_COS) a = cos(w);
    at[q * kR64Block] = a;
  }
  double y[MPMI_MAX_STATE];
#pragma unroll
  for (int j = 0; j < MPMI_MAX_STATE; ++j) y[j] = 0.0;
  K = opaque_coeffs(K);
  for (int f = 0; f < D; ++f) {
    const double p = at[m->feat_a[f] * kR64Block] * at[m->feat_b[f] * kR64Block];
#pragma unroll
    for (int j = 0; j < MPMI_MAX_STATE; ++j) y[j] = fma(p, K[f * 8 + j], y[j]);
  }
#pragma unroll
  for (int j = 0; j < MPMI_MAX_STATE; ++j) x[j] = (j < n) ? y[j] : 0.0;
}

// Race car, w = [x, y, psi, vx, vy, r, delta, a]: the input terms of output
// column j folded once per segment (K row stride 8): the constant cu, the
// coefficients L[k] of x_k, and Ts, Tc of sin psi, cos psi.
__device__ __forceinline__ void fold_column64(const double* __restrict__ K, int j, double d, double a, double sd,
                                              double cd, double* cu, double* L, double* Ts, double* Tc) {
  double c = K[0 * 8 + j];
  c = fma(d, K[7 * 8 + j], c);
  c = fma(a, K[8 * 8 + j], c);
  c = fma(d * d, K[quad_index(6, 6, 8) * 8 + j], c);
  c = fma(d * a, K[quad_index(6, 7, 8) * 8 + j], c);
  c = fma(a * a, K[quad_index(7, 7, 8) * 8 + j], c);
  c = fma(sd, K[47 * 8 + j], c);
  c = fma(cd, K[48 * 8 + j], c);
  c = fma(a * sd, K[63 * 8 + j], c);
  *cu = c;
#pragma unroll
  for (int k = 0; k < 6; ++k)
    L[k] = fma(a, K[quad_index(k, 7, 8) * 8 + j], fma(d, K[quad_index(k, 6, 8) * 8 + j], K[(1 + k) * 8 + j]));
  L[3] = fma(cd, K[60 * 8 + j], fma(sd, K[57 * 8 + j], L[3]));
  L[4] = fma(cd, K[61 * 8 + j], fma(sd, K[58 * 8 + j], L[4]));
  L[5] = fma(cd, K[62 * 8 + j], fma(sd, K[59 * 8 + j], L[5]));
  *Ts = fma(a, K[52 * 8 + j], K[45 * 8 + j]);
  *Tc = fma(a, K[56 * 8 + j], K[46 * 8 + j]);
}

// Output column j of the race car's FP64 step, x'_j, from the column's 27
// step rows kc[r * STRIDE] (the step-ordered table: the 21 quadratic rows
// (k, l >= k) in order, then sin psi (vx, vy, r) and cos psi (vx, vy, r)) and
// its folded input terms, in nested form:
//   x'_j = cu + sin psi (Ts + sum_i kc[21 + i] x_{3+i}) + cos psi (Tc + sum_i kc[24 + i] x_{3+i})
//        + sum_k x_k (L_k + sum_{l >= k} kc[q(k, l)] x_l).
// The same polynomial as the sum over the step's features, with no feature
// products: 37 operations in place of 67.  The inner sums are independent
// chains; the outer one is split in two, starting from the shortest.
template <int STRIDE>
__device__ __forceinline__ double rc_column64(const double* kc, double cu, const double* L, double Ts, double Tc,
                                              double sp, double cp, const double* x) {
  const double ts = fma(kc[23 * STRIDE], x[5], fma(kc[22 * STRIDE], x[4], fma(kc[21 * STRIDE], x[3], Ts)));
  const double tc = fma(kc[26 * STRIDE], x[5], fma(kc[25 * STRIDE], x[4], fma(kc[24 * STRIDE], x[3], Tc)));
  const double y0 = fma(cp, tc, fma(sp, ts, cu));
  double t[6];
  int q = 0;
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    t[k] = L[k];
#pragma unroll
    for (int l = k; l < 6; ++l, ++q) t[k] = fma(kc[q * STRIDE], x[l], t[k]);
  }
  const double ya = fma(x[1], t[1], fma(x[3], t[3], x[5] * t[5]));
  const double yb = fma(x[0], t[0], fma(x[2], t[2], x[4] * t[4]));
  return (y0 + ya) + yb;
}

// Race car, one candidate per lane: the FP32 tick's folded input terms, and
// the step's six columns in the nested form, in FP64.
struct Stepper64RaceCar {
  double cu[6], L[6][6], Ts[6], Tc[6];  // L[j][k]: column j's coefficient of x_k
  __device__ __forceinline__ void set_input(const double* __restrict__ Kin, const double* u) {
    const double* K = opaque_coeffs(Kin);
    const double sd = sin(u[0]), cd = cos(u[0]);
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      double Lj[6];
      fold_column64(K, j, u[0], u[1], sd, cd, &cu[j], Lj, &Ts[j], &Tc[j]);
#pragma unroll
      for (int k = 0; k < 6; ++k) L[j][k] = Lj[k];
    }
  }
  // Ks: the step rows in step order (Model64::Kstep).
  __device__ __forceinline__ void step(const double* __restrict__ Ksin, double* x) {
    const double* Ks = opaque_coeffs(Ksin);
    double sp, cp;
    sincos_rr64(x[2], &sp, &cp);
    double y[6];
#pragma unroll
    for (int j = 0; j < 6; ++j) y[j] = rc_column64<8>(Ks + j, cu[j], L[j], Ts[j], Tc[j], sp, cp, x);
#pragma unroll
    for (int j = 0; j < 6; ++j) x[j] = y[j];
  }
};

// First violation (1..H, or H + 1) of candidate c (c < Nc) predicted in FP64
// from x_t, one lane.  K: the model's FP64 K (LDS copy or the blob's); Ks:
// the race car's step rows in step order; at: this lane's LDS column for the
// described bases.
template <bool RC, int DEG>
__device__ int evaluate64(const ModelDev* __restrict__ md, const double* __restrict__ K,
                          const double* __restrict__ Ks, const GenParams& gp, int H,
                          const float* __restrict__ x_t, const float* __restrict__ u_user,
                          const float* __restrict__ cand, int c, double* at) {
  const Model64* m = &md->m64;
  const int n = md->n, mi = md->m, S = gp.n_seg, D = md->dim;
  double x[MPMI_MAX_STATE], u[MPMI_MAX_INPUT];
#pragma unroll
  for (int j = 0; j < MPMI_MAX_STATE; ++j) x[j] = (j < n) ? (double)x_t[j] : 0.0;
#pragma unroll
  for (int j = 0; j < MPMI_MAX_INPUT; ++j) u[j] = (j < mi) ? (double)cand_value(gp, md, cand, u_user, c, 0, j) : 0.0;
  Stepper64RaceCar stp;
  if constexpr (RC) stp.set_input(K, u);
  const bool noisy = md->has_noise != 0;
  const uint64_t pre = noisy ? hash_prefix(gp.seed, gp.tick, (uint64_t)(uint32_t)gp.loop, (uint64_t)c) : 0ull;
  int snext = segment_start(1, S, H);
  for (int s = 1; s <= H; ++s) {
    if (s == snext) {
      const int g = ((s - 1) * S) / H;
      snext = segment_start(g + 1, S, H);
#pragma unroll
      for (int j = 0; j < MPMI_MAX_INPUT; ++j)
        u[j] = (j < mi) ? (double)cand_value(gp, md, cand, u_user, c, g, j) : 0.0;
      if constexpr (RC) stp.set_input(K, u);
    }
    const Safety64<MPMI_MAX_STATE, DEG> sc = safety64<MPMI_MAX_STATE, DEG>(m);
    if constexpr (RC) stp.step(Ks, x);
    else step64_described(m, K, n, D, u, x, at);
    if (noisy) add_noise64(m, pre, s, n, x);
    if (!safe64(sc, x)) return s;
  }
  return H + 1;
}

// Race car, one candidate over the 8 lanes of an aligned lane group: lane j
// (< 6) holds output column j's coefficients in registers and forms x'_j, the
// group exchanges the six new components, and every lane then holds the same
// state (the same bits, so the same verdict and the same exit step).  Lanes 6
// and 7 repeat column 5.  The heading's sine and cosine, the noise draws and
// the track margin are formed by every lane; lane j tests component j's box.  Returns the first violation (1..H, or
// H + 1).

template <int DEG>
__device__ int evaluate64_rc8(const ModelDev* __restrict__ md, const double* __restrict__ K,
                              const double* __restrict__ Ks, const GenParams& gp, int H,
                              const float* __restrict__ x_t, const float* __restrict__ u_user,
                              const float* __restrict__ cand, int c) {
  const Model64* m = &md->m64;
  const int lane = threadIdx.x & 63;
  const int j = (lane & 7) < 6 ? (lane & 7) : 5;
  const int base = lane & ~7;
  const int S = gp.n_seg;
  double x[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) x[k] = (double)x_t[k];
  double cu, L[6], Ts, Tc;
  {
    const double d = (double)cand_value(gp, md, cand, u_user, c, 0, 0);
    const double a = (double)cand_value(gp, md, cand, u_user, c, 0, 1);
    fold_column64(K, j, d, a, sin(d), cos(d), &cu, L, &Ts, &Tc);
  }
  // Lane j's box: the limit of component j and whether it is boxed.
  const double lim_j = m->comp_lim[j];
  const bool box_j = (m->comp_mask >> j) & 1;
  const bool noisy = md->has_noise != 0;
  const uint64_t pre = noisy ? hash_prefix(gp.seed, gp.tick, (uint64_t)(uint32_t)gp.loop, (uint64_t)c) : 0ull;
  // Iteration s forms x_s from x_{s-1} and, beside it, the verdict of
  // x_{s-1} (the two are independent, so their chains overlap); an unsafe
  // x_{s-1} ends the rollout at s - 1 and the step formed with it is dropped.
  double own = 0.0;  // component j of the state being checked
  int snext = segment_start(1, S, H);
  for (int s = 1; s <= H; ++s) {
    if (s == snext) {
      const int g = ((s - 1) * S) / H;
      snext = segment_start(g + 1, S, H);
      const double d = (double)cand_value(gp, md, cand, u_user, c, g, 0);
      const double a = (double)cand_value(gp, md, cand, u_user, c, g, 1);
      fold_column64(K, j, d, a, sin(d), cos(d), &cu, L, &Ts, &Tc);
    }
    // The step rows of column j (the step-ordered table), read from LDS at
    // every step (held in registers across the horizon they spill), all
    // issued here and awaited together before the contraction: left to the
    // scheduler, the reads go one round trip per pair of FMAs.
    double kc[kRcStepRows];
    {
      const double* Kc = opaque_coeffs(Ks) + j;
#pragma unroll
      for (int r = 0; r < kRcStepRows; ++r) kc[r] = Kc[r * 8];
    }
    const Safety64<6, DEG> sc = safety64<6, DEG>(m);
    double sp, cp;
    sincos_rr64(x[2], &sp, &cp);
#pragma unroll
    for (int r = 0; r < kRcStepRows; ++r) asm volatile("" : "+v"(kc[r]));
    const double y = rc_column64<1>(kc, cu, L, Ts, Tc, sp, cp, x);
    // The boxes: lane j tests component j, and the group's eight tests are
    // combined from one ballot (the group's lanes are all active: they hold
    // the same state and exit together).  safe64's verdict, split over the
    // group.  x_0, the current state, is not checked.
    const unsigned long long okm = __ballot((fabs(own) < lim_j) | !box_j);
    const bool ok = (((okm >> base) & 0xFFull) == 0xFFull) & track_ok64_nb(sc, x);
    double xn[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) xn[k] = __shfl(y, base + k, 64);
    if (s > 1 && !ok) return s - 1;
#pragma unroll
    for (int k = 0; k < 6; ++k) x[k] = xn[k];
    own = y;
    if (noisy) {
      add_noise64(m, pre, s, 6, x);
      own = x[0];
#pragma unroll
      for (int k = 1; k < 6; ++k) own = (j == k) ? x[k] : own;
    }
  }
  {
    const Safety64<6, DEG> sc = safety64<6, DEG>(m);
    const unsigned long long okm = __ballot((fabs(own) < lim_j) | !box_j);
    if (!((((okm >> base) & 0xFFull) == 0xFFull) & track_ok64_nb(sc, x))) return H;
  }
  return H + 1;
}

// ---------------------------------------------------------------------------
// Single loop: re-roll the context's list, publish, finalise.
// ---------------------------------------------------------------------------

// The end of a re-roll workgroup: the wave's keys and safe count published,
// and the last workgroup finalises the selection and empties the list.
__device__ __forceinline__ void recheck_publish(const ModelDev* __restrict__ md, const GenParams& gp, int H,
                                                const float* __restrict__ u_user, const float* __restrict__ cand,
                                                Slot* __restrict__ slot, mpmi_selection* __restrict__ out,
                                                RecheckList* __restrict__ rl, unsigned long long ks,
                                                unsigned long long kf, unsigned int n_safe, unsigned int n_parts) {
  unsigned int wsum = n_safe;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) wsum += __shfl_xor(wsum, off, 64);
  if (publish_wave_counted<true>(ks, kf, wsum, slot, n_parts, blockIdx.x) && threadIdx.x == 0) {
    finalize<MPMI_MAX_INPUT>(md, gp, cand, u_user, H, slot, out);
    rl->count = 0u;
    rl->n_keep = 0u;
    __threadfence();
  }
}

// Filter: K* is final once the FP32 tick has completed (every candidate
// outside the band published), so a listed candidate can change the selection
// only if its key precedes K* (every listed one when nothing outside the band
// is safe).  Those are copied to the kept array; the others keep their FP32
// verdicts and their safe ones are added to the safe count.  One entry per
// lane; workgroups past the list's end return at once.
constexpr int kFilterBlock = 256;
__global__ void __launch_bounds__(kFilterBlock)
recheck64_filter_kernel(const ModelDev* __restrict__ md, GenParams gp, const float* __restrict__ u_user,
                        const float* __restrict__ cand, Slot* __restrict__ slot, RecheckList* __restrict__ rl,
                        int capacity) {
  __shared__ unsigned int s_w[kFilterBlock / 64];
  const unsigned int cnt_raw = rl->count;
  const int count = (int)(cnt_raw < (unsigned int)capacity ? cnt_raw : (unsigned int)capacity);
  if ((int)blockIdx.x * kFilterBlock >= count) return;  // uniform
  const unsigned long long kstar = published_best(slot);
  int* keep = rl->idx + capacity;
  const int t = threadIdx.x;
  unsigned int kept_safe = 0;
  for (int e0 = blockIdx.x * kFilterBlock; e0 < count; e0 += gridDim.x * kFilterBlock) {  // uniform
    const int e = e0 + t;
    bool want = false;
    int entry = 0;
    if (e < count) {
      entry = rl->idx[e];
      const int c = entry >> 1;
      if (kstar != kKeyNone && safe_key(cost_at(md, gp, cand, u_user, c), c) > kstar)
        kept_safe += ((entry & 1) && c > 0) ? 1u : 0u;
      else
        want = true;
    }
    wave_append(&rl->n_keep, keep, want, entry);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) kept_safe += __shfl_xor(kept_safe, o, 64);
  if ((t & 63) == 0) s_w[t >> 6] = kept_safe;
  __syncthreads();
  if (t == 0) {
    unsigned int tot = 0;
#pragma unroll
    for (int w = 0; w < kFilterBlock / 64; ++w) tot += s_w[w];
    if (tot) atomicAdd(&slot->sub[blockIdx.x % kSubSlots].count, (unsigned long long)tot);
  }
}

// Re-roll of the kept entries.  With none kept, the first workgroup
// finalises and the others return at once; otherwise only the workgroups
// that own kept entries take part (and count the tickets).
__device__ __forceinline__ bool recheck_nothing_kept(const ModelDev* __restrict__ md, const GenParams& gp, int H,
                                                     const float* __restrict__ u_user,
                                                     const float* __restrict__ cand, Slot* __restrict__ slot,
                                                     mpmi_selection* __restrict__ out, RecheckList* __restrict__ rl,
                                                     int n_keep) {
  if (n_keep > 0) return false;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    finalize<MPMI_MAX_INPUT>(md, gp, cand, u_user, H, slot, out);
    rl->count = 0u;
    rl->n_keep = 0u;
    __threadfence();
  }
  return true;
}

// Described bases: one kept candidate per lane.
template <int DEG>
__global__ void __launch_bounds__(kR64Block)
recheck64_kernel(const ModelDev* __restrict__ md, GenParams gp, int H, const float* __restrict__ x_t,
                 const float* __restrict__ u_user, const float* __restrict__ cand, Slot* __restrict__ slot,
                 mpmi_selection* __restrict__ out, int16_t* __restrict__ fv_out, RecheckList* __restrict__ rl,
                 int capacity, const mpmi_selection* __restrict__ gate) {
  __shared__ double sK[MPMI_MAX_DIM * 8];
  __shared__ double sAt[MPMI_MAX_ATOMS * kR64Block];
  // Gated tick (a fallback after a proposal tick): nothing ran, nothing to finalise.
  if (gate && gate->status == MPMI_OK) return;
  const unsigned int kn = rl->n_keep;
  const int n_keep = (int)(kn < (unsigned int)capacity ? kn : (unsigned int)capacity);
  if (recheck_nothing_kept(md, gp, H, u_user, cand, slot, out, rl, n_keep)) return;
  const int parts = min((int)gridDim.x, (n_keep + kR64Block - 1) / kR64Block);
  if ((int)blockIdx.x >= parts) return;  // uniform
  const int* keep = rl->idx + capacity;
  const int lane = threadIdx.x;
  unsigned long long ks = kKeyNone, kf = kKeyNone;
  unsigned int n_safe = 0;
  const double* Kg = &md->m64.K[0][0];
  for (int e = lane; e < MPMI_MAX_DIM * 8; e += kR64Block) sK[e] = Kg[e];
  __syncthreads();
  for (int e = blockIdx.x * kR64Block + lane; e < n_keep; e += parts * kR64Block) {
    const int c = keep[e] >> 1;
    const int fv = evaluate64<false, DEG>(md, sK, nullptr, gp, H, x_t, u_user, cand, c, sAt + lane);
    if (fv_out) fv_out[c] = (int16_t)fv;
    const float cst = cost_at(md, gp, cand, u_user, c);
    const bool safe = fv == H + 1;
    const unsigned long long a = safe ? safe_key(cst, c) : kKeyNone;
    const unsigned long long b = safe ? kKeyNone : fallback_key(fv, cst, c);
    ks = a < ks ? a : ks;
    kf = b < kf ? b : kf;
    n_safe += (safe && c > 0) ? 1u : 0u;
  }
  recheck_publish(md, gp, H, u_user, cand, slot, out, rl, ks, kf, n_safe, (unsigned int)parts);
}

// Race car: one kept candidate per 8-lane group (evaluate64_rc8), eight per
// workgroup.
template <int DEG>
__global__ void __launch_bounds__(kR64Block, 2)
recheck64_rc_kernel(const ModelDev* __restrict__ md, GenParams gp, int H, const float* __restrict__ x_t,
                    const float* __restrict__ u_user, const float* __restrict__ cand, Slot* __restrict__ slot,
                    mpmi_selection* __restrict__ out, int16_t* __restrict__ fv_out, RecheckList* __restrict__ rl,
                    int capacity, const mpmi_selection* __restrict__ gate) {
  static_assert(kR64Block == 64, "one wave per workgroup");
  constexpr int kPer = kR64Block / 8;  // candidates per workgroup pass
  __shared__ double sK[MPMI_MAX_DIM * 8];
  __shared__ double sKs[kRcStepRows * 8];
  // Gated tick (a fallback after a proposal tick): nothing ran, nothing to finalise.
  if (gate && gate->status == MPMI_OK) return;
  const unsigned int kn = rl->n_keep;
  const int n_keep = (int)(kn < (unsigned int)capacity ? kn : (unsigned int)capacity);
  if (recheck_nothing_kept(md, gp, H, u_user, cand, slot, out, rl, n_keep)) return;
  const int parts = min((int)gridDim.x, (n_keep + kPer - 1) / kPer);
  if ((int)blockIdx.x >= parts) return;  // uniform
  const int* keep = rl->idx + capacity;
  const int lane = threadIdx.x;
  unsigned long long ks = kKeyNone, kf = kKeyNone;
  unsigned int n_safe = 0;
  const double* Kg = &md->m64.K[0][0];
  for (int e = lane; e < MPMI_MAX_DIM * 8; e += kR64Block) sK[e] = Kg[e];
  for (int e = lane; e < kRcStepRows * 8; e += kR64Block) sKs[e] = (&md->m64.Kstep[0][0])[e];
  __syncthreads();
  for (int q = blockIdx.x * kPer + (lane >> 3); q < n_keep; q += parts * kPer) {  // uniform per 8-lane group
    const int c = keep[q] >> 1;
    const int fv = evaluate64_rc8<DEG>(md, sK, sKs, gp, H, x_t, u_user, cand, c);
    if ((lane & 7) == 0) {
      if (fv_out) fv_out[c] = (int16_t)fv;
      const float cst = cost_at(md, gp, cand, u_user, c);
      const bool safe = fv == H + 1;
      const unsigned long long a = safe ? safe_key(cst, c) : kKeyNone;
      const unsigned long long b = safe ? kKeyNone : fallback_key(fv, cst, c);
      ks = a < ks ? a : ks;
      kf = b < kf ? b : kf;
      n_safe += (safe && c > 0) ? 1u : 0u;
    }
  }
  recheck_publish(md, gp, H, u_user, cand, slot, out, rl, ks, kf, n_safe, (unsigned int)parts);
}

hipError_t launch_recheck64(const mpmi_system& sys, const void* model, const mpmi_tick_desc& d, const float* x_t,
                            const float* u_user, const float* cand, void* slot, mpmi_selection* out, int16_t* fv,
                            void* recheck, int capacity, int grid, hipStream_t st, const mpmi_selection* gate) {
  GenParams gp;
  gp.seed = d.seed;
  gp.tick = d.tick;
  gp.loop = d.loop;
  gp.gen = d.gen;
  gp.n_cand = d.n_cand;
  gp.n_seg = d.n_seg;
  for (int j = 0; j < MPMI_MAX_INPUT; ++j) gp.grid[j] = d.grid[j] > 0 ? d.grid[j] : 1;
  const ModelDev* md = (const ModelDev*)model;
  Slot* sl = (Slot*)slot;
  RecheckList* rl = (RecheckList*)recheck;
  const bool small = track_degree(sys) <= kSmallTrackDeg;
  recheck64_filter_kernel<<<grid, kFilterBlock, 0, st>>>(md, gp, u_user, cand, sl, rl, capacity);
  if (sys.basis == MPMI_BASIS_RACE_CAR) {
    // Windows of 8 entries, one wave per workgroup, up to three waves per
    // SIMD: 16 workgroups per compute unit cover 32,768 entries per pass.
    if (small)
      recheck64_rc_kernel<kSmallTrackDeg><<<grid * 4, kR64Block, 0, st>>>(md, gp, d.horizon, x_t, u_user, cand, sl,
                                                                          out, fv, rl, capacity, gate);
    else
      recheck64_rc_kernel<kMaxHarm><<<grid * 4, kR64Block, 0, st>>>(md, gp, d.horizon, x_t, u_user, cand, sl, out,
                                                                    fv, rl, capacity, gate);
  } else if (small) {
    recheck64_kernel<kSmallTrackDeg><<<grid, kR64Block, 0, st>>>(md, gp, d.horizon, x_t, u_user, cand, sl, out, fv,
                                                                 rl, capacity, gate);
  } else {
    recheck64_kernel<kMaxHarm><<<grid, kR64Block, 0, st>>>(md, gp, d.horizon, x_t, u_user, cand, sl, out, fv, rl,
                                                           capacity, gate);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Many loops: re-roll every loop's listed candidates (each entry names its
// loop and model), publish per lane into the loop's slot, then the last
// workgroup finalises every loop and advances the tick counters.
// ---------------------------------------------------------------------------
__device__ __forceinline__ GenParams loop_gen(const mpmi_loop_desc* __restrict__ L, uint64_t tick, int loop) {
  GenParams gp;
  gp.seed = L->seed;
  gp.tick = tick;
  gp.loop = loop;
  gp.gen = L->gen;
  gp.n_cand = L->n_cand;
  gp.n_seg = L->n_seg;
#pragma unroll
  for (int j = 0; j < MPMI_MAX_INPUT; ++j) gp.grid[j] = L->grid[j] > 0 ? L->grid[j] : 1;
  return gp;
}

__global__ void __launch_bounds__(kR64Block)
multi_recheck64_kernel(const mpmi_loop_desc* __restrict__ loops, const ModelDev* __restrict__ models,
                       const int* __restrict__ model_of_loop, Slot* __restrict__ slots, uint64_t* __restrict__ ticks,
                       MultiRecheck* __restrict__ rl, int n_loops) {
  __shared__ double sAt[MPMI_MAX_ATOMS * kR64Block];
  __shared__ int s_last;
  const int lane = threadIdx.x;
  const int count = (int)rl->count;
  for (int e0 = blockIdx.x * kR64Block; e0 < count; e0 += gridDim.x * kR64Block) {
    const int e = e0 + lane;
    if (e < count) {
      const uint4 en = rl->e[e];
      const int loop = (int)en.x, c = (int)en.y;
      const mpmi_loop_desc* L = &loops[loop];
      const ModelDev* md = models + en.z;
      const GenParams gp = loop_gen(L, ticks[loop], loop);
      const int H = L->horizon;
      // The loop's K* is complete: the many-loop launch before this one
      // published every tile of every loop.
      const unsigned long long kstar = published_best(&slots[loop]);
      const float cst = cost_at(md, gp, L->cand, L->u_user, c);
      SubSlot* ss = &slots[loop].sub[c % kSubSlots];
      if (kstar != kKeyNone && safe_key(cst, c) > kstar) {
        if (en.w && c > 0) atomicAdd(&ss->count, 1ull);  // FP32 verdict stands
      } else {
        const int fv = md->sys.basis == MPMI_BASIS_RACE_CAR
                           ? evaluate64<true, kMaxHarm>(md, &md->m64.K[0][0], &md->m64.Kstep[0][0], gp, H,
                                                        L->x_t, L->u_user, L->cand, c, sAt + lane)
                           : evaluate64<false, kMaxHarm>(md, &md->m64.K[0][0], nullptr, gp, H, L->x_t, L->u_user,
                                                         L->cand, c, sAt + lane);
        if (L->first_violation) L->first_violation[c] = (int16_t)fv;
        const bool safe = fv == H + 1;
        if (safe) atomicMin(&ss->key_safe64, safe_key(cst, c));
        else atomicMin(&ss->key_fb, fallback_key(fv, cst, c));
        if (safe && c > 0) atomicAdd(&ss->count, 1ull);
      }
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    s_last = atomicAdd(&rl->done, 1u) == gridDim.x - 1;
  }
  __syncthreads();
  if (!s_last) return;
  __threadfence();
  for (int l = lane; l < n_loops; l += kR64Block) {
    const mpmi_loop_desc* L = &loops[l];
    const ModelDev* md = models + model_of_loop[l];
    const GenParams gp = loop_gen(L, ticks[l], l);
    finalize<MPMI_MAX_INPUT>(md, gp, L->cand, L->u_user, L->horizon, &slots[l], L->out);
    ticks[l] = gp.tick + 1;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    rl->count = 0u;
    rl->done = 0u;
    __threadfence();
  }
}

size_t multi_recheck_bytes(size_t capacity) { return sizeof(MultiRecheck) + sizeof(uint4) * capacity; }

hipError_t launch_multi_recheck64(const mpmi_loop_desc* loops, const void* models, const int* model_of_loop,
                                  void* slots, uint64_t* ticks, void* recheck, int n_loops, int grid, hipStream_t st) {
  multi_recheck64_kernel<<<grid, kR64Block, 0, st>>>(loops, (const ModelDev*)models, model_of_loop, (Slot*)slots,
                                                     ticks, (MultiRecheck*)recheck, n_loops);
  return hipGetLastError();
}

}  // namespace mpmi
