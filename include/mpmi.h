/*
 * mpmi.h -- C ABI of the MI355X library for model-predictive minimal
 * intervention shared control (MPMI-SC).
 *
 * The library evaluates, once per control tick, a large batch of candidate
 * user inputs against a learned Koopman model and a safety set, and returns
 * the safe candidate closest to the user's own input (Algorithm 2, Sec. IV-C
 * of the paper).  Every entry point below names the passage of the paper that
 * defines the operation.
 *
 * Conventions shared by every entry point
 *  - Pointers are DEVICE pointers (memory of the GPU the context was created
 *    on) unless the parameter is marked "host".  The caller owns and allocates
 *    every buffer it passes; the library owns only what mpmi_create()
 *    allocates (per-loop selection slots and the fit workspace).
 *  - Arrays are dense and row-major in the order their shape is written, the
 *    LAST index fastest: cand[S][m][Nc] stores candidate c of input j in
 *    segment g at cand[(g*m + j)*Nc + c].
 *  - `stream` is a hipStream_t (NULL = the null stream).  Apart from
 *    koopman_fit, calls only enqueue work and return at once; results are
 *    ready when the stream reaches them.
 *  - Arguments are validated on the host before anything is enqueued.  A bad
 *    argument returns MPMI_EINVAL (or MPMI_EUNSUPPORTED for a valid but
 *    unimplemented combination) and enqueues nothing; mpmi_last_error()
 *    then holds a message.  A failed launch returns MPMI_EDEVICE.
 *  - "No candidate is safe" is not an error: it is reported per tick in
 *    mpmi_selection.status (device memory), because the host has returned
 *    before the kernels run.
 *  - One context may be used by one host thread at a time.  Calls on one
 *    context that share a `loop` slot must be ordered on one stream, and so
 *    must all BF16X3 and FP32_RECHECK64 ticks of a context (they share its
 *    recheck list).
 *  - Set-up calls (mpmi_create, mpmi_model_pack, koopman_fit,
 *    mpmi_multi_create / _set_config / _autotune / _graph) may allocate or
 *    synchronise and are not meant for stream capture; tick calls allocate
 *    nothing and do not synchronise.
 *  - A model pointer is valid only on the context that packed it.
 */
#ifndef MPMI_H
#define MPMI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MPMI_ABI_VERSION 7

/* Size limits (checked on the host). */
#define MPMI_MAX_STATE 8      /* n */
#define MPMI_MAX_INPUT 4      /* m */
#define MPMI_MAX_DIM 64       /* D, basis size */
#define MPMI_MAX_BOX 4        /* box constraints per system */
#define MPMI_MAX_HORIZON 255  /* H, prediction steps */
#define MPMI_MAX_SEGMENTS 8   /* S, piecewise-constant input segments */
#define MPMI_MAX_CAND 33554431 /* Nc = N + 1 <= 2^25 - 1 */
#define MPMI_MAX_LOOPS 4096   /* selection slots per context */
#define MPMI_MAX_ATOMS 32     /* atoms of a custom basis */
#define MPMI_MAX_LIBRARY 160  /* candidate functions of a basis-selection library */

typedef int32_t mpmi_status;
enum {
  MPMI_OK = 0,
  MPMI_NO_SAFE = 1, /* informational: only ever stored in mpmi_selection.status */
  MPMI_EINVAL = -1,
  MPMI_ENOMEM = -2,
  MPMI_EDEVICE = -3,
  MPMI_EUNSUPPORTED = -4,
  MPMI_ESINGULAR = -5
};

/* Basis families psi(w), w = [x; u] (Sec. IV-A: the Koopman operator acts on
 * functions of the state; the functions used here are fixed families).
 *  LINEAR       psi = w                                    D = n + m
 *  BALANCE_BOT  n = 4, m = 1: [1, w_0..w_4, w_k w_l for 0 <= k <= l <= 4,
 *               k outer, l inner]                           D = 21
 *  RACE_CAR     n = 6, m = 2, w = [x, y, psi, vx, vy, r, delta, a]:
 *               [1, w_0..w_7, w_k w_l (0 <= k <= l <= 7, k outer),
 *                sin psi, cos psi, sin delta, cos delta,
 *                sin psi * (vx, vy, r, a), cos psi * (vx, vy, r, a),
 *                sin delta * (vx, vy, r), cos delta * (vx, vy, r),
 *                a sin delta]                               D = 64        */
enum { MPMI_BASIS_LINEAR = 0, MPMI_BASIS_BALANCE_BOT = 1, MPMI_BASIS_RACE_CAR = 2, MPMI_BASIS_CUSTOM = 3 };

/* Atoms of a custom basis (functions of one component of w = [x; u]). */
enum { MPMI_ATOM_ONE = 0, MPMI_ATOM_VAR = 1, MPMI_ATOM_SIN = 2, MPMI_ATOM_COS = 3 };

/* Arithmetic of the prediction step.
 *  FP32    states, features and K in FP32, FP32 accumulation.
 *  FP32_RECHECK64  the FP32 tick; every candidate that has a checked state
 *          (steps 1 .. its first violation) whose margin to some constraint
 *          lies within that constraint's FP32 band (eps32_box, eps32_track)
 *          of zero is listed instead of ranked (n_recheck counts them).
 *          Two more launches on the same stream keep the listed candidates
 *          whose selection key precedes the least key ranked outside the
 *          band -- every listed one when no candidate outside the band is
 *          safe -- and predict each again from x_t, with K, the features,
 *          noise and margins in FP64 (Sec. IV-A and IV-B in double
 *          precision); its FP64 first violation replaces the FP32 one.  The
 *          other listed candidates cannot change the selection and keep
 *          their FP32 verdicts.  With bands at least the
 *          FP32 rollout's margin error, the selection is that of an FP64
 *          rollout, and so is every first violation outside the band (and
 *          every one, when nothing is safe).  One lane per candidate in the
 *          FP32 tick; ticks of at most 2^22 candidates (MPMI_EUNSUPPORTED
 *          otherwise);
 *          trajectories, when stored, are the FP32 states.
 *  BF16X3  the contraction runs on BF16 matrix cores as three products of
 *          hi/lo BF16 splits of the features and of (K - E) in residual form
 *          x' = x + psi^T (K - E), FP32 accumulation; every candidate whose
 *          margin comes within the system's eps band of a constraint is then
 *          re-rolled in FP32 and the FP32 verdict is kept.  Race-car models,
 *          ticks of at most 2^22 candidates (the recheck list holds them all;
 *          larger ticks return MPMI_EUNSUPPORTED).                          */
enum { MPMI_PREC_FP32 = 0, MPMI_PREC_BF16X3 = 1, MPMI_PREC_FP32_RECHECK64 = 2 };

/* How a tick obtains candidates 1..N (candidate 0 is always the user's input,
 * held over all segments; Sec. III-D: a safe user input passes unchanged).
 *  EXPLICIT  read from a caller array cand[S][m][N] (candidate i at column i-1)
 *  GRID      cell-centred grid (Sec. IV-B, equally spaced samples): index
 *            k = i - 1 = k_0 + G_0 (k_1 + G_1 (...)), value of input j is
 *            (float)(lo_j + (k_j + 0.5) * ((hi_j - lo_j) / G_j)) evaluated in
 *            FP64 in that order; S must be 1
 *  UNIFORM   counter-based uniform draws (Alg. 2's sampling step): for input
 *            j of segment g, h = seed; h = mix((h ^ w) + G) for w in (tick,
 *            loop, i, g*m + j), mix the SplitMix64 output function and G its
 *            golden gamma 0x9E3779B97F4A7C15; r = (h >> 40) * 2^-24; value =
 *            (float)(lo_j + (hi_j - lo_j) * r) in FP64.                     */
enum { MPMI_GEN_EXPLICIT = 0, MPMI_GEN_GRID = 1, MPMI_GEN_UNIFORM = 2 };

/* A controlled system: basis, safety set and input box (host struct, copied).
 * Safety (Sec. IV-B predictive safety; inflated barrier of Sec. V-C-1): a
 * predicted state x is safe iff every margin is > 0 (a NaN margin is not):
 *   box j   : (box_bound[j] - box_infl[j]) - |x[box_index[j]]|
 *   track   : (track_half - track_infl) - |rho - r_c(phi)|, (rho, phi) the
 *             polar coordinates of (x[0], x[1]) and
 *             r_c(phi) = track_r0 + sum_k track_amp[k] sin(track_freq[k] phi + track_phase[k])
 * eps_box / eps_track: in BF16X3 mode, a candidate whose margin at some step
 * falls below eps is re-rolled in FP32.  eps32_box / eps32_track: the FP32
 * bands of MPMI_PREC_FP32_RECHECK64 (a margin within them sends the candidate
 * to the FP64 re-roll); several boxes on one component use the band of the
 * one with the least limit.
 * noise_sigma: process noise of the fused tick (Alg. 2 adds a Gaussian z_i to
 * every predicted state): after step s, component j of candidate i's state
 * gains noise_sigma[j] * z_j.  z comes in pairs (components 2q, 2q+1) from
 * one 64-bit draw h = hash(seed, tick, loop, i, 65536 + 4 (s-1) + q) of the
 * MPMI_GEN_UNIFORM generator: u1 = ((h >> 40) + 1) 2^-24, u2 = ((h >> 16) &
 * 0xFFFFFF) 2^-24, z_2q = sqrt(-2 ln u1) cos(2 pi u2), z_2q+1 = sqrt(-2 ln u1)
 * sin(2 pi u2).  All zero = a deterministic model.                          */
typedef struct mpmi_system {
  int32_t basis;          /* MPMI_BASIS_* */
  int32_t n_state;        /* n (LINEAR: 1..8; fixed 4 / 6 for the others) */
  int32_t n_input;        /* m (LINEAR: 1..4; fixed 1 / 2 for the others) */
  int32_t n_box;          /* number of box constraints used, 0..4 */
  int32_t box_index[4];   /* state index of box constraint j */
  float box_bound[4];
  float box_infl[4];
  float eps_box[4];
  int32_t has_track;      /* 0 or 1; needs n >= 2 */
  int32_t track_n;        /* number of sinusoids used, 0..4 */
  int32_t track_freq[4];  /* integer frequencies, 0..8 */
  float track_amp[4];
  float track_phase[4];
  float track_r0;
  float track_half;
  float track_infl;
  float eps_track;
  float u_lo[4];          /* input box; cost divides input j by (u_hi-u_lo)/2 */
  float u_hi[4];
  float noise_sigma[8];   /* per state component, >= 0 */
  /* MPMI_BASIS_CUSTOM only (a basis given as data, Sec. IV-A's functions of
   * state chosen by the caller, e.g. by basis selection): feature f is
   * psi_f(w) = atom[feat_a[f]](w) * atom[feat_b[f]](w), atom q being 1
   * (ONE), w[atom_var[q]] (VAR), sin w[atom_var[q]] (SIN) or cos w[atom_var[q]]
   * (COS), with w = [x; u].  Ignored for the fixed families.               */
  int32_t n_atoms;        /* 1..MPMI_MAX_ATOMS */
  int32_t dim;            /* D, 1..MPMI_MAX_DIM */
  int8_t atom_kind[MPMI_MAX_ATOMS];
  int8_t atom_var[MPMI_MAX_ATOMS];  /* 0 .. n + m - 1 */
  int8_t feat_a[MPMI_MAX_DIM];      /* 0 .. n_atoms - 1 */
  int8_t feat_b[MPMI_MAX_DIM];
  float eps32_box[4];     /* FP32_RECHECK64 bands, >= 0 */
  float eps32_track;
  int32_t pad_eps;
} mpmi_system;

/* Fills the custom-basis fields of *sys with the atoms and features of a
 * fixed family (LINEAR with n_state, n_input; BALANCE_BOT; RACE_CAR), and
 * sets sys->basis = MPMI_BASIS_CUSTOM, n_state and n_input; other fields are
 * left as they are.  Host only.  MPMI_EINVAL for an unknown family or sizes. */
int32_t mpmi_basis_describe(int32_t family, int32_t n_state, int32_t n_input, mpmi_system* sys /* host */);

/* The fixed family whose features, in order, are those of a custom basis
 * (its fast kernels compute the same functions), or MPMI_BASIS_CUSTOM if
 * none is; for a fixed family, that family.  Host only.  A caller switches
 * to the fast path by setting sys->basis to the result.                     */
int32_t mpmi_basis_match(const mpmi_system* sys /* host */);

/* Result of one tick (device memory, written by the library).
 * Selection (Alg. 2 selection step, Sec. IV-D): among candidates whose H
 * predicted states are all safe, the least cost
 *   cost_i = sum_j ((u_ij - u_h,j) / ((u_hi_j - u_lo_j)/2))^2
 * on the first segment, ties to the lowest index.  If none is safe: the
 * latest first violation, then least cost, then lowest index, with
 * status = MPMI_NO_SAFE.                                                     */
typedef struct mpmi_selection {
  int32_t idx;             /* chosen candidate; 0 = the user's own input */
  int32_t status;          /* MPMI_OK or MPMI_NO_SAFE */
  int32_t n_safe;          /* safe candidates other than candidate 0 */
  int32_t n_recheck;       /* candidates re-rolled in FP32 (BF16X3) */
  float u_r[4];            /* applied input: first segment of candidate idx */
  float cost;              /* cost of idx (FP32) */
  float deviation;         /* Euclidean norm of u_r - u_h (Sec. VI-D-1) */
  int32_t first_violation; /* of idx: 1..H, or H+1 when its rollout is safe */
  int32_t n_cand;          /* Nc = N + 1 candidates evaluated */
} mpmi_selection;

/* One control tick's candidate set and horizon (host struct, copied). */
typedef struct mpmi_tick_desc {
  uint64_t seed;          /* UNIFORM: generator seed */
  uint64_t tick;          /* UNIFORM: tick counter */
  int32_t loop;           /* selection slot 0..MPMI_MAX_LOOPS-1; also an RNG word */
  int32_t gen;            /* MPMI_GEN_* */
  int32_t n_cand;         /* N, candidates besides candidate 0 (>= 0) */
  int32_t grid[4];        /* GRID: points per input, product == N */
  int32_t n_seg;          /* S, 1..8; step s (1..H) uses segment floor((s-1)S/H) */
  int32_t horizon;        /* H, 1..255 */
  int32_t precision;      /* MPMI_PREC_* */
  int32_t block;          /* threads per workgroup: 0 (library default) or 64..1024, multiple of 64 */
  int32_t lanes_per_cand; /* FP32 ticks: 0 or 1 (one lane per candidate), or 2 / 4 / 8 lanes per
                             candidate, each lane computing a share of the state (lower latency at
                             small N; block <= 256); the same operations in the same order as one
                             lane, so the same selection */
} mpmi_tick_desc;

typedef struct mpmi_ctx_s* mpmi_ctx;

/* Version of this header the library was built from. */
int32_t mpmi_abi_version(void);

/* Creates a context on HIP device `device` (makes it current on the calling
 * thread) and allocates its slots and workspace.  *out is NULL on failure.  */
mpmi_status mpmi_create(mpmi_ctx* out, int32_t device);
void mpmi_destroy(mpmi_ctx ctx);
/* Message of the last failed call on ctx (never NULL; "" after success);
 * with ctx NULL, of the last failed call made without a context
 * (mpmi_tick_noalloc) on the calling thread.                              */
const char* mpmi_last_error(mpmi_ctx ctx);

/* Size in bytes of a packed model (device blob read by every rollout).      */
size_t mpmi_model_bytes(void);

/* Packs a system and its fitted K (device FP64 [D][n], row f = feature f,
 * column j = next-state component j; Sec. IV-A) into `model` (device,
 * mpmi_model_bytes() bytes, 256-byte aligned): FP32 K, the residual K - E
 * split into BF16 hi/lo operand tiles, and the safety constants.            */
mpmi_status mpmi_model_pack(mpmi_ctx ctx, const mpmi_system* sys /* host */,
                            const double* K, void* model, void* stream);

/* Learns K from transitions (Sec. IV-A: the Koopman model is learned from
 * data; least squares as in extended DMD).  X [T][n], U [T][m], Y [T][n] are
 * device FP64 with Y[t] the successor of (X[t], U[t]).  Solves
 *   min || Psi_s K_s - Y ||^2 + ridge || K_s ||^2,  Psi_s = Psi diag(1/s),
 * s_f the RMS of feature f over the T rows, by an FP64 Gram accumulation,
 * a Cholesky factorisation and two triangular solves; writes K = diag(1/s) K_s
 * to K_out (device FP64 [D][n]) and, if cond_out is not NULL, an estimate of
 * the 2-norm condition number of Psi_s to *cond_out (host).  Synchronous:
 * returns after the result is in K_out.  MPMI_ESINGULAR when the scaled Gram
 * matrix is not numerically positive definite.  T >= D required.           */
mpmi_status koopman_fit(mpmi_ctx ctx, const mpmi_system* sys /* host */,
                        const double* X, const double* U, const double* Y, int64_t T,
                        double ridge, double* K_out, double* cond_out /* host */,
                        void* stream);

/* Predicts every candidate over the full horizon, without early exit
 * (Alg. 2 prediction loop; Fig. 1's cloud of trajectories): from x0 [n],
 * x_s = psi(x_{s-1}, u_c(seg(s)))^T K for s = 1..H.  cand [S][m][Nc];
 * traj [H][n][traj_ld] receives x_1..x_H (candidate fastest; row stride
 * traj_ld >= Nc floats, columns past Nc untouched).  precision FP32, or
 * BF16X3 for race-car models (the BF16X3 tick's step, its states stored
 * unchecked: the precision's own rollout error can be measured).
 *
 * Trajectory rows and write rate (this call, mpmi_tick, safe_mask): rows
 * that start on 256-byte boundaries (traj 256-byte aligned, traj_ld a
 * multiple of 64) are stored as whole memory lines.  With traj_ld = Nc =
 * N + 1 each row starts 4 bytes further past a 256-byte boundary than the
 * last, every wave's store straddles lines, and the store runs at about half
 * the rate (measured on MI355X).
 * MPMI_EINVAL for traj_ld < Nc.                                              */
mpmi_status rollout_batch(mpmi_ctx ctx, const void* model, int32_t precision,
                          const float* x0, const float* cand, int32_t Nc, int32_t S,
                          int32_t H, float* traj, int64_t traj_ld, void* stream);

/* Safety verdicts of stored trajectories (Sec. IV-B; Alg. 2 safety check):
 * traj [H][n][traj_ld] (traj_ld >= Nc); first_violation[c] = first step s in
 * 1..H whose state traj[s-1][.][c] is unsafe, or H+1.  near_bits (optional,
 * may be NULL) [ceil(Nc/32)]: bit c % 32 of word c / 32 is set when some state
 * of steps 1..min(first_violation, H) has a margin within its constraint's
 * FP32 band (eps32_box / eps32_track of the packed system) of zero -- the
 * candidates whose verdict FP32 rounding could decide.  min_margin (optional,
 * may be NULL) [Nc] = the least margin over all constraints and over steps
 * 1..min(first_violation, H).                                                */
mpmi_status safe_mask(mpmi_ctx ctx, const void* model, const float* traj, int64_t traj_ld,
                      int32_t Nc, int32_t H, int16_t* first_violation, uint32_t* near_bits,
                      float* min_margin, void* stream);

/* Minimal-intervention choice (Alg. 2 selection step; Sec. III-D; Sec. IV-D)
 * over candidates cand [S][m][Nc] with verdicts first_violation [Nc]
 * (safe = H+1); candidate 0 is taken to be the user's input u_user [m] for
 * n_safe.  Writes *out (device).  `loop` picks the selection slot.           */
mpmi_status select_min_intervention(mpmi_ctx ctx, const void* model, const float* cand,
                                    int32_t Nc, int32_t S, const int16_t* first_violation,
                                    int32_t H, const float* u_user, int32_t loop,
                                    mpmi_selection* out, void* stream);

/* One fused control tick (Alg. 2 entire): candidates generated per desc,
 * prediction with early exit at the first unsafe state, selection, in one
 * kernel launch.  x_t [n] and u_user [m] device FP32.  cand: EXPLICIT only,
 * [S][m][N].  Optional outputs (NULL to skip): first_violation [N+1];
 * traj [H][n][traj_ld], traj_ld >= N+1 (states after a candidate's first
 * violation are left unwritten; traj_ld is ignored when traj is NULL).
 * *out receives the selection.                                               */
mpmi_status mpmi_tick(mpmi_ctx ctx, const void* model, const mpmi_tick_desc* desc /* host */,
                      const float* x_t, const float* u_user, const float* cand,
                      mpmi_selection* out, int16_t* first_violation, float* traj,
                      int64_t traj_ld, void* stream);

/* The tick of mpmi_tick for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): no context, nothing allocated or freed, no synchronisation.
 * The tick's scratch -- the selection slots of loops 0..63 and an FP64
 * re-roll list of 65,536 entries and as many kept entries (about 548 KiB in
 * all) -- is a file-scope
 * device array of the library, one copy per GPU, held until the process
 * ends; its load-time image is the reset state and every tick leaves it so.
 * sys (host) must be the system `model` was packed from (mpmi_model_pack);
 * the tick runs on the current device.  desc as for mpmi_tick with loop
 * 0..63, precision FP32 (any launch shape) or FP32_RECHECK64 (at most 65,536
 * candidates); MPMI_EINVAL / MPMI_EUNSUPPORTED beyond these limits, with the
 * message in mpmi_last_error(NULL) (thread-local).  Calls on one GPU share
 * the array: calls that overlap in time on that GPU (other streams, other
 * threads) race; order them on one stream.  The record and first violations
 * equal mpmi_tick's for the same inputs.                                  */
mpmi_status mpmi_tick_noalloc(const mpmi_system* sys /* host */, const void* model,
                              const mpmi_tick_desc* desc /* host */, const float* x_t, const float* u_user,
                              const float* cand, mpmi_selection* out, int16_t* first_violation, void* stream);

/* ---------------------------------------------------------------------------
 * Basis selection (Sec. IV-A: the basis is chosen from data by the
 * sparsity-promoting method of Jovanovic, Schmid and Nichols 2014; Sec.
 * V-C-3: a library of random basis functions is reduced to the relevant few).
 * ------------------------------------------------------------------------- */

/* A library of candidate functions (host struct): function f is
 * atom[feat_a[f]](w) * atom[feat_b[f]](w), w = [x; u], atoms as in
 * mpmi_system's custom basis. */
typedef struct mpmi_library {
  int32_t n_state;   /* n, 1..MPMI_MAX_STATE */
  int32_t n_input;   /* m, 1..MPMI_MAX_INPUT */
  int32_t n_atoms;   /* 1..MPMI_MAX_ATOMS */
  int32_t n_feat;    /* L, 1..MPMI_MAX_LIBRARY */
  int8_t atom_kind[MPMI_MAX_ATOMS];
  int8_t atom_var[MPMI_MAX_ATOMS];
  uint8_t feat_a[MPMI_MAX_LIBRARY];
  uint8_t feat_b[MPMI_MAX_LIBRARY];
} mpmi_library;

/* Selects basis functions from transitions X [T][n], U [T][m] -> Y [T][n]
 * (device FP64), for each penalty gamma[g] (host, g < n_gamma, >= 0) at
 * once.  With Psi_s the library's values divided by each function's RMS over
 * the T rows and Y_s the targets divided by each component's RMS, and
 * G = Psi_s' Psi_s / T, A = Psi_s' Y_s / T, it minimises
 *   tr(B' G B) - 2 tr(B' A) + gamma sum_f ||B_f||
 * over L x n coefficients B (one row per library function) by `iters`
 * iterations of ADMM from B = Lam = 0 with penalty rho > 0:
 *   K <- (G + rho/2 I)^-1 (A + rho/2 (B - Lam/rho)),
 *   B <- rows of K + Lam/rho shrunk by max(0, 1 - (gamma/rho)/||row||),
 *   Lam <- Lam + rho (K - B)
 * (FP64 throughout).  Writes B_out [n_gamma][L][n] (device FP64, unscaled:
 * B_s[f][j] * rms(Y_j) / rms(psi_f)), support [n_gamma][L] (device, 1 where
 * row f of B is nonzero: the selected functions) and, if resid is not NULL,
 * resid [n_gamma][2] (host) = the last iteration's primal ||K - B||_F and
 * dual rho ||B - B_prev||_F residuals.  The selected functions' model is then
 * fitted (the method's polishing step) by koopman_fit on a custom basis of
 * them.  Synchronous; a set-up call (allocates and frees its workspace).
 * MPMI_EINVAL for a bad library, T < L, n_gamma out of 1..1024, rho <= 0, a
 * negative gamma or iters out of 1..1000000. */
mpmi_status koopman_select_basis(mpmi_ctx ctx, const mpmi_library* lib /* host */, const double* X,
                                 const double* U, const double* Y, int64_t T, const double* gamma /* host */,
                                 int32_t n_gamma, double rho, int32_t iters, double* B_out, uint8_t* support,
                                 double* resid /* host, may be NULL */, void* stream);

/* ---------------------------------------------------------------------------
 * Lifted whole-horizon form (Sec. IV-A: in the Koopman representation a
 * prediction step is one matrix-vector product and a batch of trajectories one
 * matrix-matrix product).  Instead of re-lifting the predicted state at every
 * step, a candidate's lifted state z = psi(x_t, u) advances by z <- z K with
 * the full lifted operator K (D x D, row f = feature f), and the predicted
 * state is read off z's state coordinates (features state_feat0 ..
 * state_feat0 + n - 1: 0 for LINEAR, 1 otherwise).  Inputs are held over the
 * horizon (one segment).  The predictions differ from the re-lifting model's
 * from the second step on; the safety check, cost and selection are those of
 * mpmi_tick.
 * ------------------------------------------------------------------------- */

/* Fits the lifted operator: min || Psi_s K_s - Psi' ||^2 + ridge || K_s ||^2
 * over transitions (X[t], U[t]) -> Y[t], with Psi' rows psi(Y[t], U[t]) (the
 * input held over the step) and the scaling and FP64 solver of koopman_fit;
 * K_out device FP64 [D][D].  Its state columns solve koopman_fit's problem.
 * Synchronous; errors as koopman_fit.                                       */
mpmi_status koopman_fit_lifted(mpmi_ctx ctx, const mpmi_system* sys /* host */, const double* X, const double* U,
                               const double* Y, int64_t T, double ridge, double* K_out, double* cond_out /* host */,
                               void* stream);

/* Bytes of a packed lifted model for horizons up to h_max (0 if h_max is out
 * of 1..MPMI_MAX_HORIZON).                                                 */
size_t mpmi_lifted_bytes(int32_t h_max);

/* The factorisation the lifted tick runs on (host only, no device needed):
 * every feature is psi_f(x, u) = g[feat_g[f]](u) * phi[feat_phi[f]](x), with
 *   LINEAR       phi = [1, x_0 .. x_{n-1}]                  g = [1, u_0 .. u_{m-1}]
 *   BALANCE_BOT  phi = [1, x_0..x_3, x_k x_l (k <= l < 4)]  g = [1, u, u^2]
 *   RACE_CAR     phi = [1, x_0..x_5, x_k x_l (k <= l < 6), sin psi, cos psi,
 *                       sin psi (vx, vy, r), cos psi (vx, vy, r)]
 *                g = [1, delta, a, delta^2, delta a, a^2, sin delta, cos delta,
 *                     a sin delta]
 * (products k outer, l inner).  feat_g, feat_phi: host [D]; *n_phi, *n_g
 * receive the lengths of phi and g.  MPMI_EINVAL for an invalid basis/size. */
mpmi_status mpmi_lifted_layout(int32_t basis, int32_t n_state, int32_t n_input, int32_t* feat_g /* host */,
                               int32_t* feat_phi /* host */, int32_t* n_phi /* host */, int32_t* n_g /* host */);

/* Packs a lifted model for horizons up to h_max from a model packed by
 * mpmi_model_pack (its system, safety set and input box) and the lifted
 * operator K_full (device FP64 [D][D]) into `lifted` (device,
 * mpmi_lifted_bytes(h_max) bytes, 256-byte aligned).  With the input held,
 * x_s[j](u) = sum_k g_k(u) Q_s[k][j], Q_s[k][j] = sum_r P_s[k][j][r] phi_r(x_t),
 * P_s[k][j][r] = sum over features f with (feat_g, feat_phi) = (k, r) of
 * (K^s)[f][state_feat0 + j]; the powers and P are formed here in FP64 on the
 * host and stored in FP32.  Synchronous.  MPMI_EUNSUPPORTED when more than
 * four state components are constrained.  The lifted blob also holds the
 * per-tick table Q: lifted ticks on one blob must be ordered on one stream.  */
mpmi_status mpmi_lifted_pack(mpmi_ctx ctx, const void* model, const double* K_full, int32_t h_max, void* lifted,
                             void* stream);

/* One tick with lifted predictions (Alg. 2 with Sec. IV-A's matrix-product
 * prediction): a prologue launch forms Q for x_t, then one launch evaluates
 * every candidate's horizon as a product [candidates x g] by [g x H * slots]
 * on the FP32 matrix cores with the safety check on each output tile, the
 * first violation, and the selection of mpmi_tick.  desc as for mpmi_tick
 * with n_seg 1, precision FP32, block 0 or 256, lanes_per_cand 0 or 1,
 * horizon <= the blob's h_max.  Optional first_violation [N+1] and traj
 * [H][n][traj_ld] (every state up to a candidate's first violation is
 * written; some later ones may be).                                         */
mpmi_status mpmi_tick_lifted(mpmi_ctx ctx, void* lifted, const mpmi_tick_desc* desc /* host */, const float* x_t,
                             const float* u_user, const float* cand, mpmi_selection* out, int16_t* first_violation,
                             float* traj, int64_t traj_ld, void* stream);

/* Tick autotuner: times `reps` ticks of *desc for every launch shape in the
 * library's search space (block 64..512; lanes_per_cand 1, 2, 4, 8 for FP32, 1
 * for FP32_RECHECK64; other precisions MPMI_EUNSUPPORTED)
 * and writes the fastest into desc->block and desc->lanes_per_cand (host);
 * *best_ms (host, may be NULL) receives its mean tick time.  The timed ticks
 * are real ticks writing *out. */
mpmi_status mpmi_tick_autotune(mpmi_ctx ctx, const void* model, mpmi_tick_desc* desc /* host, in/out */,
                               const float* x_t, const float* u_user, const float* cand, mpmi_selection* out,
                               int32_t reps, float* best_ms /* host */, void* stream);

/* Writes the candidates a tick with `desc` evaluates, cand_out [S][m][N+1]
 * (column 0 = u_user), so generated candidates can be inspected.           */
mpmi_status mpmi_generate_candidates(mpmi_ctx ctx, const void* model,
                                     const mpmi_tick_desc* desc /* host */,
                                     const float* u_user, const float* cand,
                                     float* cand_out, void* stream);


/* Diagnostic: the device's non-packed FP32 FMA issue rate (TFLOP/s, host
 * *tflops), measured by a register-only kernel with 16 independent FMA
 * chains per lane and 8 workgroups of 256 lanes per compute unit; the best
 * of three timed launches.  It is the ceiling of the tick's VALU-bound step.
 * Synchronous (default stream, about 15 ms); allocates nothing. */
mpmi_status mpmi_fp32_fma_rate(mpmi_ctx ctx, double* tflops /* host */);

/* Diagnostic: the sine and cosine the FP64 re-roll of MPMI_PREC_FP32_RECHECK64
 * applies to the race car's heading (the prediction of Sec. IV-A in FP64),
 * of n doubles: sn[i], cs[i] = sin, cos of x[i] (all device, n entries,
 * caller-owned).  Cody and Waite's reduction by pi/2 and the Taylor series
 * on [-pi/4, pi/4], about an ulp from the correctly rounded values for
 * |x| < 2^20; larger, infinite and NaN arguments take the HIP library's
 * sincos.  Asynchronous on `stream`; allocates nothing.  MPMI_EINVAL for
 * NULL pointers with n > 0 or n < 0. */
mpmi_status mpmi_sincos64(mpmi_ctx ctx, const double* x, double* sn, double* cs, int32_t n, void* stream);

/* Diagnostic: HBM write ceilings of the trajectory store (GB/s, host), on a
 * caller buffer buf of rows * ld floats (device, 16-byte aligned; contents
 * overwritten): *pattern_gbs for the store pattern of traj[rows][ld] alone
 * (lane c < Nc writes element c of every row, streaming stores, no
 * compute), *stream_gbs for contiguous 16-byte stores of rows * Nc floats;
 * best of three timed launches each.  Synchronous (default stream);
 * allocates nothing.  MPMI_EINVAL for NULL pointers, misalignment, Nc or
 * rows < 1, ld < Nc, or more than 2^33 elements. */
mpmi_status mpmi_write_rates(mpmi_ctx ctx, float* buf, int32_t Nc, int64_t ld, int32_t rows,
                             double* pattern_gbs /* host */, double* stream_gbs /* host */);

/* Diagnostic: HBM read ceilings of the safety check over stored
 * trajectories (GB/s, host), on a caller buffer buf of rows * ld floats
 * (device, 16-byte aligned; read only): *pattern_gbs for the load pattern of
 * traj[rows][ld] alone (lane c < Nc reads element c of every row, no
 * compute), *stream_gbs for contiguous 16-byte loads of rows * Nc floats;
 * best of three timed launches each.  Synchronous (default stream);
 * allocates nothing.  MPMI_EINVAL as for mpmi_write_rates. */
mpmi_status mpmi_read_rates(mpmi_ctx ctx, const float* buf, int32_t Nc, int64_t ld, int32_t rows,
                            double* pattern_gbs /* host */, double* stream_gbs /* host */);

/* ---------------------------------------------------------------------------
 * Many concurrent control loops in one launch per tick.
 *
 * Each loop runs Alg. 2 on its own model, state, user input, candidate count
 * and horizon.  The (loop, tile) work items of all loops, ordered
 * longest-processing-time first (horizon x per-step cost), run as one
 * workgroup each, which the hardware dispatches in list order; each loop's
 * selection is finalised by the workgroup that completes its last tile.  Nothing is allocated and no
 * host synchronisation happens per tick, so a tick can be captured once in a
 * HIP graph (mpmi_multi_graph) and replayed.
 * ------------------------------------------------------------------------- */

/* One loop (host struct, copied into device memory by mpmi_multi_create;
 * every pointer must stay valid for the life of the mpmi_multi).  The
 * mpmi_multi keeps its own copy of each distinct packed model, taken at
 * mpmi_multi_create and again at every re-plan (mpmi_multi_set_config,
 * mpmi_multi_autotune): a model re-packed in place is seen by the loops from
 * the next re-plan on. */
typedef struct mpmi_loop_desc {
  const void* model;          /* packed model on this context */
  const float* x_t;           /* device [n]: current state, read every tick */
  const float* u_user;        /* device [m]: user input, read every tick */
  const float* cand;          /* EXPLICIT only: device [S][m][N] */
  mpmi_selection* out;        /* device: selection written every tick */
  int16_t* first_violation;   /* optional device [N+1] */
  uint64_t seed;              /* UNIFORM: generator seed */
  uint64_t tick;              /* UNIFORM: tick counter of the first tick; the
                                 device adds one after every completed tick */
  int32_t gen;                /* MPMI_GEN_* */
  int32_t n_cand;             /* N */
  int32_t grid[4];            /* GRID: points per input, product == N */
  int32_t n_seg;              /* S */
  int32_t horizon;            /* H */
} mpmi_loop_desc;

/* Launch shape: `block` threads per workgroup = candidates per tile
 * (64..1024, multiple of 64).  `grid` must be 0 on input; on output
 * (mpmi_multi_get_config, mpmi_multi_autotune) it is the launch's workgroup
 * count, one per work item. */
typedef struct mpmi_multi_config {
  int32_t block;
  int32_t grid;
  int32_t precision;  /* MPMI_PREC_FP32, or MPMI_PREC_FP32_RECHECK64: one more
                         launch per tick re-rolls every loop's near-band
                         candidates in FP64 and then finalises all loops */
} mpmi_multi_config;

typedef struct mpmi_multi_s* mpmi_multi;

/* Validates the loops, copies them to device memory, builds the ordered
 * work list for `cfg` (NULL = block 256) and allocates the per-loop
 * selection slots.  Synchronous. */
mpmi_status mpmi_multi_create(mpmi_ctx ctx, const mpmi_loop_desc* loops /* host */, int32_t n_loops,
                              const mpmi_multi_config* cfg /* host, may be NULL */, mpmi_multi* out);
void mpmi_multi_destroy(mpmi_multi multi);

/* Re-plans the work list for a new launch shape and precision (synchronous,
 * no allocation). */
mpmi_status mpmi_multi_set_config(mpmi_ctx ctx, mpmi_multi multi, const mpmi_multi_config* cfg /* host */);

/* Current launch shape and work-list size (host outputs, may be NULL). */
mpmi_status mpmi_multi_get_config(mpmi_multi multi, mpmi_multi_config* cfg, int32_t* n_work_items);

/* Current device tick counters of the loops, ticks[n_loops] (host).
 * Synchronous (waits for the device). */
mpmi_status mpmi_multi_get_ticks(mpmi_ctx ctx, mpmi_multi multi, uint64_t* ticks /* host */);

/* One tick of every loop: one kernel launch on `stream`. */
mpmi_status mpmi_multi_tick(mpmi_ctx ctx, mpmi_multi multi, void* stream);

/* Autotuner: times `reps` ticks (HIP events on `stream`) for each block size
 * in 64, 128, 256, 512, 1024, keeps the fastest, and reports it in *best and
 * its mean tick time in *best_ms (host, may be NULL).  The timed ticks are real ticks:
 * they write selections and advance tick counters. */
mpmi_status mpmi_multi_autotune(mpmi_ctx ctx, mpmi_multi multi, int32_t reps, mpmi_multi_config* best /* host */,
                                float* best_ms /* host */, void* stream);

/* Captures one mpmi_multi_tick into an instantiated HIP graph (*graph_exec,
 * a hipGraphExec_t).  Replays read x_t / u_user at the loops' fixed
 * pointers, so the caller updates those buffers between replays.  The graph
 * holds the launch shape of the plan at capture: after mpmi_multi_set_config
 * or mpmi_multi_autotune, destroy it and capture again. */
mpmi_status mpmi_multi_graph(mpmi_ctx ctx, mpmi_multi multi, void** graph_exec);
/* Captures one mpmi_tick (all of its launches: the FP32 tick, or the tick
 * and its re-roll for BF16X3 / FP32_RECHECK64) with these arguments into an
 * instantiated HIP graph (*graph_exec).  Replays read x_t, u_user (and cand)
 * at the same addresses and write out and first_violation, so the caller
 * updates the inputs between replays; the descriptor is fixed at capture (a
 * UNIFORM tick replays the same draws: capture again, or use GRID /
 * EXPLICIT candidates, for fresh ones).  No trajectory store.  Destroy with
 * mpmi_graph_destroy. */
mpmi_status mpmi_tick_graph(mpmi_ctx ctx, const void* model, const mpmi_tick_desc* desc /* host */,
                            const float* x_t, const float* u_user, const float* cand, mpmi_selection* out,
                            int16_t* first_violation, void** graph_exec);
mpmi_status mpmi_graph_launch(mpmi_ctx ctx, void* graph_exec, void* stream);
void mpmi_graph_destroy(void* graph_exec);

/* ---------------------------------------------------------------------------
 * Learned proposal (race car).  A small network maps (state, user input) to
 * a mixture over inputs near the safe minimal-intervention choice, so a tick
 * can evaluate a few thousand proposals instead of an exhaustive grid; the
 * exhaustive sampler of Sec. IV-B remains the fallback whenever no proposal
 * (and not the user's own input) is safe.
 *
 * Network: 8 inputs [x (6); u_user (2)], standardised by in_mean / in_std,
 * three hidden layers of 256 with GELU 0.5 z (1 + tanh(sqrt(2/pi)(z + 0.044715 z^3))),
 * 80 outputs = 16 x {logit, mu_0, mu_1, log sigma_0, log sigma_1} of a
 * diagonal-Gaussian mixture over the input mapped to [-1, 1]^2; log sigma is
 * clamped to [-7, 2].  Parameters: one flat vector of MPMI_MLP_PARAMS values,
 * per layer W [in][out] row-major then b [out], layers in order.  Products
 * use the BF16 copy of the weights with FP32 accumulation; biases and the
 * Adam state are FP32; w_bf16 16-byte aligned (the products read it in
 * 16-byte chunks; MPMI_EINVAL otherwise).  Workspace: caller-allocated
 * device memory of mlp_workspace_bytes(B) bytes (256-byte aligned).
 * ------------------------------------------------------------------------- */
#define MPMI_MLP_IN 8
#define MPMI_MLP_HIDDEN 256
#define MPMI_MLP_COMP 16
#define MPMI_MLP_OUT 80
#define MPMI_MLP_PARAMS 154448
#define MPMI_MLP_MAX_BATCH 65536

size_t mlp_workspace_bytes(int32_t batch);

/* Y [B][80] = network(X [B][8]).  w_bf16 / w_f32: the parameters in BF16
 * (products) and FP32 (biases). */
mpmi_status mlp_forward(mpmi_ctx ctx, const uint16_t* w_bf16, const float* w_f32, const float* in_mean,
                        const float* in_std, const float* X, int32_t B, float* Y, void* work,
                        size_t work_bytes, void* stream);

/* Mean mixture negative log-likelihood of targets T [B][2] (inputs mapped
 * to [-1, 1]) and its gradient grad [MPMI_MLP_PARAMS] (FP32) with respect
 * to the parameters; *loss (device FP32) receives the mean NLL. */
mpmi_status mlp_grad(mpmi_ctx ctx, const uint16_t* w_bf16, const float* w_f32, const float* in_mean,
                     const float* in_std, const float* X, const float* T, int32_t B, float* grad, float* loss,
                     void* work, size_t work_bytes, void* stream);

/* One Adam step (Kingma & Ba 2015; beta 0.9 / 0.999, eps 1e-8, bias
 * correction with step >= 1) on the FP32 master weights; refreshes w_bf16. */
mpmi_status mlp_adam(mpmi_ctx ctx, float* w_f32, uint16_t* w_bf16, float* adam_m, float* adam_v,
                     const float* grad, int32_t step, float lr, void* stream);

/* P proposals from one mixture head (80 floats, device): component by the
 * inverse CDF of the FP32 mixture weights at r0, two Box-Muller normals from
 * r1 in (0, 1] and r2 in [0, 1), mu + sigma z clipped to [-1, 1], mapped to
 * the model's input box; r_s = top 24 bits of the counter hash of (seed,
 * tick, loop, p, s) as in MPMI_GEN_UNIFORM (r1 adds one unit first).
 * cand [1][m][P] (EXPLICIT layout). */
mpmi_status mdn_sample(mpmi_ctx ctx, const void* model, const float* head, int32_t P, uint64_t seed,
                       uint64_t tick, int32_t loop, float* cand, void* stream);

/* A learned-proposal tick: network on [x_t; u_user] and P = prop->n_cand
 * proposals drawn from its head as mdn_sample draws them, with (prop->seed,
 * prop->tick, prop->loop), in one launch (the rounding rules
 * of mlp_forward; each unit sums FP32 partials over blocks of 8 inputs, the
 * blocks in input order), then a fused tick over {u_user} + proposals (EXPLICIT; block and
 * lanes_per_cand as in mpmi_tick) into *out, then the exhaustive fallback
 * tick described by *fallback (GRID or UNIFORM), which runs only if *out
 * holds MPMI_NO_SAFE and then overwrites it (out->n_cand tells which
 * candidate set decided).  Each of the two ticks is FP32 or FP32_RECHECK64
 * (its descriptor's precision; the latter with one lane per candidate and at
 * most 2^22 candidates, and sharing the context's recheck list, so ordered
 * on one stream with the context's other such ticks).  cand_work [1][2][P]
 * device; head_out [80] device or NULL; w_bf16 16-byte aligned (MPMI_EINVAL
 * otherwise).  Race-car models only. */
mpmi_status mpmi_proposal_tick(mpmi_ctx ctx, const void* model, const uint16_t* w_bf16, const float* w_f32,
                               const float* in_mean, const float* in_std, const float* x_t,
                               const float* u_user, const mpmi_tick_desc* prop /* host */,
                               const mpmi_tick_desc* fallback /* host */, float* cand_work, float* head_out,
                               mpmi_selection* out, void* work, size_t work_bytes, void* stream);

/* C = op(A) op(B) on the BF16 matrix-core path (test hook): A, B BF16,
 * op transposes when ta / tb is 1, C [M][N] FP32. */
mpmi_status mpmi_gemm_bf16(mpmi_ctx ctx, const uint16_t* A, const uint16_t* B, int32_t M, int32_t N, int32_t K,
                           int32_t ta, int32_t tb, float* C, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* MPMI_H */
