// C-ABI layer of libmpmi: context management, host-side argument validation
// and dispatch to the kernel launchers.  Nothing here computes any part of
// the method; every step runs in the HIP kernels.
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstddef>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/mpmi.h"
#include "mpmi_launch.hpp"
#include "mpmi_tick_common.hpp"

struct mpmi_ctx_s {
  int device = 0;
  void* slots = nullptr;       // MPMI_MAX_LOOPS selection slots
  void* fit_work = nullptr;    // fit partial sums, totals and info
  void* recheck = nullptr;     // BF16X3 recheck list (count + indices)
  std::unordered_map<const void*, mpmi_system> models;  // packed models, by device address
  struct Lifted {
    mpmi_system sys;
    int32_t h_max;
  };
  std::unordered_map<const void*, Lifted> lifted;      // packed lifted models, by device address
  std::string err;
};

namespace {

// Message of the last failed call made without a context on this thread
// (mpmi_tick_noalloc and the validation it shares).
thread_local std::string g_noctx_err;

mpmi_status fail(mpmi_ctx ctx, mpmi_status code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (ctx) ctx->err = buf;
  else g_noctx_err = buf;
  return code;
}

mpmi_status ok(mpmi_ctx ctx) {
  ctx->err.clear();
  return MPMI_OK;
}

mpmi_status check_hip(mpmi_ctx ctx, hipError_t e, const char* what) {
  if (e == hipSuccess) return ok(ctx);
  return fail(ctx, MPMI_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

bool aligned(const void* p, size_t a) { return ((uintptr_t)p % a) == 0; }

int basis_dim(const mpmi_system& s) {
  switch (s.basis) {
    case MPMI_BASIS_LINEAR: return s.n_state + s.n_input;
    case MPMI_BASIS_BALANCE_BOT: return 21;
    case MPMI_BASIS_RACE_CAR: return 64;
    case MPMI_BASIS_CUSTOM: return s.dim;
    default: return -1;
  }
}

// Atoms and features of a fixed family, in its feature order (the custom
// form of the same functions).  Returns false for an unknown family.
bool family_descriptor(int family, int n, int m, mpmi_system* s) {
  int na = 0, d = 0;
  auto atom = [&](int kind, int var) { s->atom_kind[na] = (int8_t)kind; s->atom_var[na] = (int8_t)var; return na++; };
  auto feat = [&](int a, int b) { s->feat_a[d] = (int8_t)a; s->feat_b[d] = (int8_t)b; ++d; };
  if (family == MPMI_BASIS_LINEAR) {
    if (n < 1 || n > MPMI_MAX_STATE || m < 1 || m > MPMI_MAX_INPUT) return false;
    const int one = atom(MPMI_ATOM_ONE, 0);
    for (int k = 0; k < n + m; ++k) feat(atom(MPMI_ATOM_VAR, k), one);
  } else if (family == MPMI_BASIS_BALANCE_BOT || family == MPMI_BASIS_RACE_CAR) {
    const int nw = family == MPMI_BASIS_BALANCE_BOT ? 5 : 8;
    n = family == MPMI_BASIS_BALANCE_BOT ? 4 : 6;
    m = nw - n;
    const int one = atom(MPMI_ATOM_ONE, 0);
    int w[8];
    for (int k = 0; k < nw; ++k) w[k] = atom(MPMI_ATOM_VAR, k);
    feat(one, one);
    for (int k = 0; k < nw; ++k) feat(w[k], one);
    for (int k = 0; k < nw; ++k)
      for (int l = k; l < nw; ++l) feat(w[k], w[l]);
    if (family == MPMI_BASIS_RACE_CAR) {
      const int sp = atom(MPMI_ATOM_SIN, 2), cp = atom(MPMI_ATOM_COS, 2);
      const int sd = atom(MPMI_ATOM_SIN, 6), cd = atom(MPMI_ATOM_COS, 6);
      feat(sp, one); feat(cp, one); feat(sd, one); feat(cd, one);
      for (int k : {3, 4, 5, 7}) feat(sp, w[k]);
      for (int k : {3, 4, 5, 7}) feat(cp, w[k]);
      for (int k : {3, 4, 5}) feat(sd, w[k]);
      for (int k : {3, 4, 5}) feat(cd, w[k]);
      feat(w[7], sd);
    }
  } else {
    return false;
  }
  s->basis = MPMI_BASIS_CUSTOM;
  s->n_state = n;
  s->n_input = m;
  s->n_atoms = na;
  s->dim = d;
  for (int q = na; q < MPMI_MAX_ATOMS; ++q) s->atom_kind[q] = s->atom_var[q] = 0;
  for (int f = d; f < MPMI_MAX_DIM; ++f) s->feat_a[f] = s->feat_b[f] = 0;
  return true;
}

// The value of atom q of s as (kind, variable) with the variable ignored for ONE.
inline int atom_code(const mpmi_system& s, int q) {
  return s.atom_kind[q] == MPMI_ATOM_ONE ? -1 : s.atom_kind[q] * 64 + s.atom_var[q];
}

// Index in psi of feature w_0 = x_0 (the state features are contiguous).
int state_feat0(const mpmi_system& s) { return s.basis == MPMI_BASIS_LINEAR ? 0 : 1; }

mpmi_status validate_system(mpmi_ctx ctx, const mpmi_system* s) {
  if (!s) return fail(ctx, MPMI_EINVAL, "system descriptor is NULL");
  switch (s->basis) {
    case MPMI_BASIS_LINEAR:
      if (s->n_state < 1 || s->n_state > MPMI_MAX_STATE || s->n_input < 1 || s->n_input > MPMI_MAX_INPUT)
        return fail(ctx, MPMI_EINVAL, "LINEAR basis needs 1 <= n <= %d and 1 <= m <= %d (got n=%d m=%d)",
                    MPMI_MAX_STATE, MPMI_MAX_INPUT, s->n_state, s->n_input);
      break;
    case MPMI_BASIS_BALANCE_BOT:
      if (s->n_state != 4 || s->n_input != 1)
        return fail(ctx, MPMI_EINVAL, "BALANCE_BOT basis needs n=4, m=1 (got n=%d m=%d)", s->n_state, s->n_input);
      break;
    case MPMI_BASIS_RACE_CAR:
      if (s->n_state != 6 || s->n_input != 2)
        return fail(ctx, MPMI_EINVAL, "RACE_CAR basis needs n=6, m=2 (got n=%d m=%d)", s->n_state, s->n_input);
      break;
    case MPMI_BASIS_CUSTOM: {
      if (s->n_state < 1 || s->n_state > MPMI_MAX_STATE || s->n_input < 1 || s->n_input > MPMI_MAX_INPUT)
        return fail(ctx, MPMI_EINVAL, "CUSTOM basis needs 1 <= n <= %d and 1 <= m <= %d (got n=%d m=%d)",
                    MPMI_MAX_STATE, MPMI_MAX_INPUT, s->n_state, s->n_input);
      if (s->n_atoms < 1 || s->n_atoms > MPMI_MAX_ATOMS)
        return fail(ctx, MPMI_EINVAL, "n_atoms=%d out of 1..%d", s->n_atoms, MPMI_MAX_ATOMS);
      if (s->dim < 1 || s->dim > MPMI_MAX_DIM) return fail(ctx, MPMI_EINVAL, "dim=%d out of 1..%d", s->dim, MPMI_MAX_DIM);
      for (int q = 0; q < s->n_atoms; ++q) {
        if (s->atom_kind[q] < MPMI_ATOM_ONE || s->atom_kind[q] > MPMI_ATOM_COS)
          return fail(ctx, MPMI_EINVAL, "atom_kind[%d]=%d is not an atom kind", q, s->atom_kind[q]);
        if (s->atom_var[q] < 0 || s->atom_var[q] >= s->n_state + s->n_input)
          return fail(ctx, MPMI_EINVAL, "atom_var[%d]=%d is not a component of w = [x; u]", q, s->atom_var[q]);
      }
      for (int f = 0; f < s->dim; ++f)
        if (s->feat_a[f] < 0 || s->feat_a[f] >= s->n_atoms || s->feat_b[f] < 0 || s->feat_b[f] >= s->n_atoms)
          return fail(ctx, MPMI_EINVAL, "feature %d names an atom outside 0..%d", f, s->n_atoms - 1);
      break;
    }
    default:
      return fail(ctx, MPMI_EINVAL, "unknown basis %d", s->basis);
  }
  if (s->n_box < 0 || s->n_box > MPMI_MAX_BOX) return fail(ctx, MPMI_EINVAL, "n_box=%d out of 0..%d", s->n_box, MPMI_MAX_BOX);
  for (int b = 0; b < s->n_box; ++b) {
    if (s->box_index[b] < 0 || s->box_index[b] >= s->n_state)
      return fail(ctx, MPMI_EINVAL, "box_index[%d]=%d is not a state index", b, s->box_index[b]);
    if (!(s->box_infl[b] >= 0.0f)) return fail(ctx, MPMI_EINVAL, "box_infl[%d] must be >= 0", b);
  }
  if (s->has_track != 0 && s->has_track != 1) return fail(ctx, MPMI_EINVAL, "has_track must be 0 or 1");
  if (s->has_track) {
    if (s->n_state < 2) return fail(ctx, MPMI_EINVAL, "track constraint needs n >= 2");
    if (s->track_n < 0 || s->track_n > 4) return fail(ctx, MPMI_EINVAL, "track_n=%d out of 0..4", s->track_n);
    for (int k = 0; k < s->track_n; ++k)
      if (s->track_freq[k] < 0 || s->track_freq[k] > 8)
        return fail(ctx, MPMI_EINVAL, "track_freq[%d]=%d out of 0..8", k, s->track_freq[k]);
    if (!(s->track_infl >= 0.0f)) return fail(ctx, MPMI_EINVAL, "track_infl must be >= 0");
  }
  for (int j = 0; j < 8; ++j)
    if (!(s->noise_sigma[j] >= 0.0f) || s->noise_sigma[j] > 1e30f)
      return fail(ctx, MPMI_EINVAL, "noise_sigma[%d] must be finite and >= 0", j);
  for (int b = 0; b < MPMI_MAX_BOX; ++b)
    if (!(s->eps32_box[b] >= 0.0f) || s->eps32_box[b] > 1e30f)
      return fail(ctx, MPMI_EINVAL, "eps32_box[%d] must be finite and >= 0", b);
  if (!(s->eps32_track >= 0.0f) || s->eps32_track > 1e30f)
    return fail(ctx, MPMI_EINVAL, "eps32_track must be finite and >= 0");
  for (int j = 0; j < s->n_input; ++j)
    if (!(s->u_hi[j] > s->u_lo[j]))
      return fail(ctx, MPMI_EINVAL, "input box %d is empty (lo=%g hi=%g)", j, (double)s->u_lo[j], (double)s->u_hi[j]);
  return MPMI_OK;
}

// Host copy of the descriptor of a model packed by this context, so calls
// that take only the model validate and dispatch without touching the device.
mpmi_status model_system(mpmi_ctx ctx, const void* model, mpmi_system* out, hipStream_t) {
  if (!model) return fail(ctx, MPMI_EINVAL, "model is NULL");
  auto it = ctx->models.find(model);
  if (it == ctx->models.end())
    return fail(ctx, MPMI_EINVAL, "model %p was not packed by mpmi_model_pack on this context", model);
  *out = it->second;
  return MPMI_OK;
}

}  // namespace

extern "C" {

int32_t mpmi_abi_version(void) { return MPMI_ABI_VERSION; }

int32_t mpmi_basis_describe(int32_t family, int32_t n_state, int32_t n_input, mpmi_system* sys) {
  if (!sys) return MPMI_EINVAL;
  mpmi_system t = *sys;
  if (!family_descriptor(family, n_state, n_input, &t)) return MPMI_EINVAL;
  *sys = t;
  return MPMI_OK;
}

int32_t mpmi_basis_match(const mpmi_system* sys) {
  if (!sys) return MPMI_EINVAL;
  if (sys->basis != MPMI_BASIS_CUSTOM) return sys->basis;
  // only the descriptor matters here (not the safety set or the input box)
  if (sys->n_atoms < 1 || sys->n_atoms > MPMI_MAX_ATOMS || sys->dim < 1 || sys->dim > MPMI_MAX_DIM)
    return MPMI_BASIS_CUSTOM;
  for (int f = 0; f < sys->dim; ++f)
    if (sys->feat_a[f] < 0 || sys->feat_a[f] >= sys->n_atoms || sys->feat_b[f] < 0 || sys->feat_b[f] >= sys->n_atoms)
      return MPMI_BASIS_CUSTOM;
  for (int fam : {MPMI_BASIS_LINEAR, MPMI_BASIS_BALANCE_BOT, MPMI_BASIS_RACE_CAR}) {
    mpmi_system t = *sys;
    if (!family_descriptor(fam, sys->n_state, sys->n_input, &t)) continue;
    if (t.n_state != sys->n_state || t.n_input != sys->n_input || t.dim != sys->dim) continue;
    bool same = true;
    for (int f = 0; f < t.dim && same; ++f) {
      // the same product of the same two functions, in either order
      const int a = atom_code(t, t.feat_a[f]), b = atom_code(t, t.feat_b[f]);
      const int c = atom_code(*sys, sys->feat_a[f]), d = atom_code(*sys, sys->feat_b[f]);
      same = (a == c && b == d) || (a == d && b == c);
    }
    if (same) return fam;
  }
  return MPMI_BASIS_CUSTOM;
}

size_t mpmi_model_bytes(void) { return mpmi::model_bytes(); }

mpmi_status mpmi_create(mpmi_ctx* out, int32_t device) {
  if (!out) return MPMI_EINVAL;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count == 0) return MPMI_EDEVICE;
  if (device < 0 || device >= count) return MPMI_EINVAL;
  mpmi_ctx ctx = new (std::nothrow) mpmi_ctx_s();
  if (!ctx) return MPMI_ENOMEM;
  ctx->device = device;
  if (hipSetDevice(device) != hipSuccess) {
    delete ctx;
    return MPMI_EDEVICE;
  }
  const size_t slot_bytes = (size_t)MPMI_MAX_LOOPS * mpmi::slot_bytes();
  if (hipMalloc(&ctx->slots, slot_bytes) != hipSuccess ||
      hipMalloc(&ctx->fit_work, mpmi::fit_workspace_bytes()) != hipSuccess ||
      hipMalloc(&ctx->recheck, mpmi::recheck_bytes(mpmi::kRecheckCapacity)) != hipSuccess) {
    mpmi_destroy(ctx);
    return MPMI_ENOMEM;
  }
  // All slots in their reset state (one copy of a host image).
  std::vector<unsigned char> image(slot_bytes, 0);
  mpmi::slot_reset_image(image.data(), MPMI_MAX_LOOPS);
  if (hipMemcpy(ctx->slots, image.data(), slot_bytes, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(ctx->recheck, 0, 256) != hipSuccess) {
    mpmi_destroy(ctx);
    return MPMI_EDEVICE;
  }
  if (hipDeviceSynchronize() != hipSuccess) {
    mpmi_destroy(ctx);
    return MPMI_EDEVICE;
  }
  *out = ctx;
  return MPMI_OK;
}

void mpmi_destroy(mpmi_ctx ctx) {
  if (!ctx) return;
  if (ctx->slots) (void)hipFree(ctx->slots);
  if (ctx->fit_work) (void)hipFree(ctx->fit_work);
  if (ctx->recheck) (void)hipFree(ctx->recheck);
  delete ctx;
}

const char* mpmi_last_error(mpmi_ctx ctx) { return ctx ? ctx->err.c_str() : g_noctx_err.c_str(); }

mpmi_status mpmi_model_pack(mpmi_ctx ctx, const mpmi_system* sys, const double* K, void* model, void* stream) {
  if (!ctx) return MPMI_EINVAL;
  mpmi_status s = validate_system(ctx, sys);
  if (s != MPMI_OK) return s;
  if (!K) return fail(ctx, MPMI_EINVAL, "K is NULL");
  if (!model) return fail(ctx, MPMI_EINVAL, "model is NULL");
  if (!aligned(model, 256)) return fail(ctx, MPMI_EINVAL, "model must be 256-byte aligned");
  if (!aligned(K, 8)) return fail(ctx, MPMI_EINVAL, "K must be 8-byte aligned");
  // The FP64 re-roll evaluates every basis from its atom/feature description.
  mpmi_system packed = *sys;
  if (packed.basis != MPMI_BASIS_CUSTOM) {
    if (mpmi_basis_describe(sys->basis, sys->n_state, sys->n_input, &packed) != MPMI_OK)
      return fail(ctx, MPMI_EINVAL, "no description of basis %d", sys->basis);
    packed.basis = sys->basis;
  }
  s = check_hip(ctx, mpmi::launch_pack(packed, basis_dim(*sys), state_feat0(*sys), K, model, (hipStream_t)stream),
                "mpmi_model_pack launch");
  if (s == MPMI_OK) ctx->models[model] = *sys;
  return s;
}

mpmi_status koopman_fit(mpmi_ctx ctx, const mpmi_system* sys, const double* X, const double* U, const double* Y,
                        int64_t T, double ridge, double* K_out, double* cond_out, void* stream) {
  if (!ctx) return MPMI_EINVAL;
  mpmi_status s = validate_system(ctx, sys);
  if (s != MPMI_OK) return s;
  const int D = basis_dim(*sys);
  if (!X || !U || !Y || !K_out) return fail(ctx, MPMI_EINVAL, "X, U, Y and K_out must be non-NULL");
  if (T < D) return fail(ctx, MPMI_EINVAL, "T=%lld rows cannot determine D=%d features", (long long)T, D);
  if (T > (int64_t)1 << 40) return fail(ctx, MPMI_EINVAL, "T=%lld too large", (long long)T);
  if (!(ridge >= 0.0)) return fail(ctx, MPMI_EINVAL, "ridge must be >= 0");
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = mpmi::launch_fit(*sys, D, X, U, Y, T, ridge, K_out, ctx->fit_work, st);
  if (e != hipSuccess) return fail(ctx, MPMI_EDEVICE, "koopman_fit launch: %s", hipGetErrorString(e));
  e = hipStreamSynchronize(st);
  if (e != hipSuccess) return fail(ctx, MPMI_EDEVICE, "koopman_fit: %s", hipGetErrorString(e));
  struct { int32_t status, pad; double cond; } info;
  const size_t info_off = mpmi::fit_info_offset();
  e = hipMemcpy(&info, (char*)ctx->fit_work + info_off, sizeof info, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return fail(ctx, MPMI_EDEVICE, "koopman_fit readback: %s", hipGetErrorString(e));
  if (cond_out) *cond_out = info.cond;
  if (info.status != MPMI_OK)
    return fail(ctx, MPMI_ESINGULAR, "scaled Gram matrix is not numerically positive definite");
  return ok(ctx);
}

static mpmi_status validate_desc(mpmi_ctx ctx, const mpmi_system& sys, const mpmi_tick_desc* d);

mpmi_status koopman_fit_lifted(mpmi_ctx ctx, const mpmi_system* sys, const double* X, const double* U,
                               const double* Y, int64_t T, double ridge, double* K_out, double* cond_out,
                               void* stream) {
  if (!ctx) return MPMI_EINVAL;
  mpmi_status s = validate_system(ctx, sys);
  if (s != MPMI_OK) return s;
  const int D = basis_dim(*sys);
  if (!X || !U || !Y || !K_out) return fail(ctx, MPMI_EINVAL, "X, U, Y and K_out must be non-NULL");
  if (T < D) return fail(ctx, MPMI_EINVAL, "T=%lld rows cannot determine D=%d features", (long long)T, D);
  if (T > (int64_t)1 << 40) return fail(ctx, MPMI_EINVAL, "T=%lld too large", (long long)T);
  if (!(ridge >= 0.0)) return fail(ctx, MPMI_EINVAL, "ridge must be >= 0");
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = mpmi::launch_fit_lifted(*sys, D, X, U, Y, T, ridge, K_out, ctx->fit_work, st);
  if (e != hipSuccess) return fail(ctx, MPMI_EDEVICE, "koopman_fit_lifted launch: %s", hipGetErrorString(e));
  e = hipStreamSynchronize(st);
  if (e != hipSuccess) return fail(ctx, MPMI_EDEVICE, "koopman_fit_lifted: %s", hipGetErrorString(e));
  struct { int32_t status, pad; double cond; } info;
  e = hipMemcpy(&info, (char*)ctx->fit_work + mpmi::fit_info_offset(), sizeof info, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return fail(ctx, MPMI_EDEVICE, "koopman_fit_lifted readback: %s", hipGetErrorString(e));
  if (cond_out) *cond_out = info.cond;
  if (info.status != MPMI_OK)
    return fail(ctx, MPMI_ESINGULAR, "scaled Gram matrix is not numerically positive definite");
  return ok(ctx);
}

mpmi_status koopman_select_basis(mpmi_ctx ctx, const mpmi_library* lib, const double* X, const double* U,
                                 const double* Y, int64_t T, const double* gamma, int32_t n_gamma, double rho,
                                 int32_t iters, double* B_out, uint8_t* support, double* resid, void* stream) {
  if (!ctx) return MPMI_EINVAL;
  if (!lib) return fail(ctx, MPMI_EINVAL, "library is NULL");
  const int n = lib->n_state, m = lib->n_input, na = lib->n_atoms, L = lib->n_feat;
  if (n < 1 || n > MPMI_MAX_STATE || m < 1 || m > MPMI_MAX_INPUT)
    return fail(ctx, MPMI_EINVAL, "library needs 1 <= n <= %d and 1 <= m <= %d", MPMI_MAX_STATE, MPMI_MAX_INPUT);
  if (na < 1 || na > MPMI_MAX_ATOMS) return fail(ctx, MPMI_EINVAL, "n_atoms=%d out of 1..%d", na, MPMI_MAX_ATOMS);
  if (L < 1 || L > MPMI_MAX_LIBRARY) return fail(ctx, MPMI_EINVAL, "n_feat=%d out of 1..%d", L, MPMI_MAX_LIBRARY);
  for (int q = 0; q < na; ++q) {
    if (lib->atom_kind[q] < MPMI_ATOM_ONE || lib->atom_kind[q] > MPMI_ATOM_COS)
      return fail(ctx, MPMI_EINVAL, "atom_kind[%d]=%d is not an atom kind", q, lib->atom_kind[q]);
    if (lib->atom_var[q] < 0 || lib->atom_var[q] >= n + m)
      return fail(ctx, MPMI_EINVAL, "atom_var[%d]=%d is not a component of w = [x; u]", q, lib->atom_var[q]);
  }
  for (int f = 0; f < L; ++f)
    if (lib->feat_a[f] >= na || lib->feat_b[f] >= na)
      return fail(ctx, MPMI_EINVAL, "library function %d names an atom outside 0..%d", f, na - 1);
  if (!X || !U || !Y || !gamma || !B_out || !support)
    return fail(ctx, MPMI_EINVAL, "X, U, Y, gamma, B_out and support must be non-NULL");
  if (T < L) return fail(ctx, MPMI_EINVAL, "T=%lld rows cannot determine L=%d functions", (long long)T, L);
  if (T > (int64_t)1 << 40) return fail(ctx, MPMI_EINVAL, "T=%lld too large", (long long)T);
  if (n_gamma < 1 || n_gamma > 1024) return fail(ctx, MPMI_EINVAL, "n_gamma=%d out of 1..1024", n_gamma);
  for (int g = 0; g < n_gamma; ++g)
    if (!(gamma[g] >= 0.0) || gamma[g] > 1e300) return fail(ctx, MPMI_EINVAL, "gamma[%d] must be finite and >= 0", g);
  if (!(rho > 0.0) || rho > 1e300) return fail(ctx, MPMI_EINVAL, "rho must be finite and > 0");
  if (iters < 1 || iters > 1000000) return fail(ctx, MPMI_EINVAL, "iters=%d out of 1..1000000", iters);
  void* work = nullptr;
  hipError_t e = hipMalloc(&work, mpmi::select_workspace_bytes(n_gamma));
  if (e != hipSuccess) return fail(ctx, MPMI_ENOMEM, "koopman_select_basis workspace: %s", hipGetErrorString(e));
  e = mpmi::launch_select_basis(*lib, X, U, Y, T, gamma, n_gamma, rho, iters, B_out, support, resid, work,
                                (hipStream_t)stream);
  const hipError_t ef = hipFree(work);
  if (e != hipSuccess) return fail(ctx, MPMI_EDEVICE, "koopman_select_basis: %s", hipGetErrorString(e));
  if (ef != hipSuccess) return fail(ctx, MPMI_EDEVICE, "koopman_select_basis free: %s", hipGetErrorString(ef));
  return ok(ctx);
}

size_t mpmi_lifted_bytes(int32_t h_max) {
  if (h_max < 1 || h_max > MPMI_MAX_HORIZON) return 0;
  return mpmi::lifted_bytes(h_max);
}

mpmi_status mpmi_lifted_layout(int32_t basis, int32_t n_state, int32_t n_input, int32_t* feat_g, int32_t* feat_phi,
                               int32_t* n_phi, int32_t* n_g) {
  mpmi_system s;
  std::memset(&s, 0, sizeof s);
  s.basis = basis;
  s.n_state = n_state;
  s.n_input = n_input;
  for (int j = 0; j < n_input && j < MPMI_MAX_INPUT; ++j) s.u_hi[j] = 1.0f;
  if (validate_system(nullptr, &s) != MPMI_OK) return MPMI_EINVAL;
  if (!feat_g || !feat_phi || !n_phi || !n_g) return MPMI_EINVAL;
  int a = 0, b = 0;
  mpmi::lifted_layout(basis, n_state, n_input, basis_dim(s), feat_g, feat_phi, &a, &b);
  *n_phi = a;
  *n_g = b;
  return MPMI_OK;
}

mpmi_status mpmi_lifted_pack(mpmi_ctx ctx, const void* model, const double* K_full, int32_t h_max, void* lifted,
                             void* stream) {
  if (!ctx) return MPMI_EINVAL;
  mpmi_system sys;
  mpmi_status s = model_system(ctx, model, &sys, (hipStream_t)stream);
  if (s != MPMI_OK) return s;
  if (!K_full || !lifted) return fail(ctx, MPMI_EINVAL, "K_full and lifted must be non-NULL");
  if (sys.basis == MPMI_BASIS_CUSTOM)
    return fail(ctx, MPMI_EUNSUPPORTED, "the lifted form runs the fixed bases (see mpmi_basis_match)");
  if (!aligned(lifted, 256)) return fail(ctx, MPMI_EINVAL, "lifted must be 256-byte aligned");
  if (!aligned(K_full, 8)) return fail(ctx, MPMI_EINVAL, "K_full must be 8-byte aligned");
  if (h_max < 1 || h_max > MPMI_MAX_HORIZON)
    return fail(ctx, MPMI_EINVAL, "h_max=%d out of 1..%d", h_max, MPMI_MAX_HORIZON);
  hipError_t e = hipStreamSynchronize((hipStream_t)stream);
  if (e != hipSuccess) return fail(ctx, MPMI_EDEVICE, "mpmi_lifted_pack: %s", hipGetErrorString(e));
  int n_safe = 0;
  e = mpmi::lifted_pack(sys, basis_dim(sys), state_feat0(sys), model, K_full, h_max, lifted, &n_safe);
  if (n_safe < 0)
    return fail(ctx, MPMI_EUNSUPPORTED, "the lifted form checks at most four constrained state components");
  if (e != hipSuccess) return fail(ctx, MPMI_EDEVICE, "mpmi_lifted_pack: %s", hipGetErrorString(e));
  ctx->lifted[lifted] = mpmi_ctx_s::Lifted{sys, h_max};
  return ok(ctx);
}

mpmi_status mpmi_tick_lifted(mpmi_ctx ctx, void* lifted, const mpmi_tick_desc* desc, const float* x_t,
                             const float* u_user, const float* cand, mpmi_selection* out, int16_t* first_violation,
                             float* traj, int64_t traj_ld, void* stream) {
  if (!ctx) return MPMI_EINVAL;
  if (!lifted) return fail(ctx, MPMI_EINVAL, "lifted is NULL");
  auto it = ctx->lifted.find(lifted);
  if (it == ctx->lifted.end())
    return fail(ctx, MPMI_EINVAL, "lifted model %p was not packed by mpmi_lifted_pack on this context", lifted);
  const mpmi_system& sys = it->second.sys;
  mpmi_status s = validate_desc(ctx, sys, desc);
  if (s != MPMI_OK) return s;
  if (!x_t || !u_user || !out) return fail(ctx, MPMI_EINVAL, "x_t, u_user and out must be non-NULL");
  if (desc->horizon > it->second.h_max)
    return fail(ctx, MPMI_EINVAL, "horizon=%d beyond the lifted model's h_max=%d", desc->horizon, it->second.h_max);
  if (desc->n_seg != 1) return fail(ctx, MPMI_EUNSUPPORTED, "lifted ticks hold each input over the horizon (n_seg 1)");
  if (desc->precision != MPMI_PREC_FP32) return fail(ctx, MPMI_EUNSUPPORTED, "lifted ticks are FP32");
  if (desc->block != 0 && desc->block != 256) return fail(ctx, MPMI_EUNSUPPORTED, "lifted ticks use 256-thread workgroups");
  if (desc->lanes_per_cand > 1) return fail(ctx, MPMI_EUNSUPPORTED, "lifted ticks use one candidate per lane");
  if (desc->gen == MPMI_GEN_EXPLICIT && desc->n_cand > 0 && !cand)
    return fail(ctx, MPMI_EINVAL, "EXPLICIT candidates need cand");
  if (traj && traj_ld < (int64_t)desc->n_cand + 1)
    return fail(ctx, MPMI_EINVAL, "traj_ld=%lld below N+1=%d", (long long)traj_ld, desc->n_cand + 1);
  void* slot = (char*)ctx->slots + (size_t)desc->loop * mpmi::slot_bytes();
  return check_hip(ctx, mpmi::launch_tick_lifted(sys, lifted, it->second.h_max, *desc, x_t, u_user, cand, slot, out,
                                                 first_violation, traj, traj ? traj_ld : 0, 4, (hipStream_t)stream),
                   "mpmi_tick_lifted launch");
}

mpmi_status rollout_batch(mpmi_ctx ctx, const void* model, int32_t precision, const float* x0, const float* cand,
                          int32_t Nc, int32_t S, int32_t H, float* traj, int64_t traj_ld, void* stream) {
  if (!ctx) return MPMI_EINVAL;
  if (precision != MPMI_PREC_FP32 && precision != MPMI_PREC_BF16X3)
    return fail(ctx, MPMI_EINVAL, "unknown precision %d", precision);
  if (Nc < 1 || Nc > MPMI_MAX_CAND) return fail(ctx, MPMI_EINVAL, "Nc=%d out of 1..%d", Nc, MPMI_MAX_CAND);
  if (S < 1 || S > MPMI_MAX_SEGMENTS) return fail(ctx, MPMI_EINVAL, "S=%d out of 1..%d", S, MPMI_MAX_SEGMENTS);
  if (H < 1 || H > MPMI_MAX_HORIZON) return fail(ctx, MPMI_EINVAL, "H=%d out of 1..%d", H, MPMI_MAX_HORIZON);
  if (!x0 || !cand || !traj) return fail(ctx, MPMI_EINVAL, "x0, cand and traj must be non-NULL");
  if (traj_ld < Nc) return fail(ctx, MPMI_EINVAL, "traj_ld=%lld below Nc=%d", (long long)traj_ld, Nc);
  mpmi_system sys;
  mpmi_status s = model_system(ctx, model, &sys, (hipStream_t)stream);
  if (s != MPMI_OK) return s;
  if (precision == MPMI_PREC_BF16X3) {
    if (sys.basis != MPMI_BASIS_RACE_CAR)
      return fail(ctx, MPMI_EUNSUPPORTED, "BF16X3 is implemented for race-car models");
    return check_hip(ctx, mpmi::launch_rollout_bf16(model, Nc, S, H, x0, cand, traj, traj_ld, (hipStream_t)stream),
                     "rollout_batch (BF16X3) launch");
  }
  return check_hip(ctx, mpmi::launch_rollout(sys.basis, model, Nc, S, H, x0, cand, traj, traj_ld, (hipStream_t)stream),
                   "rollout_batch launch");
}

mpmi_status safe_mask(mpmi_ctx ctx, const void* model, const float* traj, int64_t traj_ld, int32_t Nc, int32_t H,
                      int16_t* first_violation, uint32_t* near_bits, float* min_margin, void* stream) {
  if (!ctx) return MPMI_EINVAL;
  if (Nc < 1 || Nc > MPMI_MAX_CAND) return fail(ctx, MPMI_EINVAL, "Nc=%d out of 1..%d", Nc, MPMI_MAX_CAND);
  if (H < 1 || H > MPMI_MAX_HORIZON) return fail(ctx, MPMI_EINVAL, "H=%d out of 1..%d", H, MPMI_MAX_HORIZON);
  if (!traj || !first_violation) return fail(ctx, MPMI_EINVAL, "traj and first_violation must be non-NULL");
  if (traj_ld < Nc) return fail(ctx, MPMI_EINVAL, "traj_ld=%lld below Nc=%d", (long long)traj_ld, Nc);
  mpmi_system sys;
  mpmi_status s = model_system(ctx, model, &sys, (hipStream_t)stream);
  if (s != MPMI_OK) return s;
  return check_hip(ctx, mpmi::launch_mask(sys.basis, model, Nc, H, traj, traj_ld, first_violation, min_margin,
                                          near_bits, (hipStream_t)stream),
                   "safe_mask launch");
}

mpmi_status select_min_intervention(mpmi_ctx ctx, const void* model, const float* cand, int32_t Nc, int32_t S,
                                    const int16_t* first_violation, int32_t H, const float* u_user, int32_t loop,
                                    mpmi_selection* out, void* stream) {
  if (!ctx) return MPMI_EINVAL;
  if (Nc < 1 || Nc > MPMI_MAX_CAND) return fail(ctx, MPMI_EINVAL, "Nc=%d out of 1..%d", Nc, MPMI_MAX_CAND);
  if (S < 1 || S > MPMI_MAX_SEGMENTS) return fail(ctx, MPMI_EINVAL, "S=%d out of 1..%d", S, MPMI_MAX_SEGMENTS);
  if (H < 1 || H > MPMI_MAX_HORIZON) return fail(ctx, MPMI_EINVAL, "H=%d out of 1..%d", H, MPMI_MAX_HORIZON);
  if (loop < 0 || loop >= MPMI_MAX_LOOPS) return fail(ctx, MPMI_EINVAL, "loop=%d out of 0..%d", loop, MPMI_MAX_LOOPS - 1);
  if (!cand || !first_violation || !u_user || !out)
    return fail(ctx, MPMI_EINVAL, "cand, first_violation, u_user and out must be non-NULL");
  mpmi_system sys;
  mpmi_status s = model_system(ctx, model, &sys, (hipStream_t)stream);
  if (s != MPMI_OK) return s;
  void* slot = (char*)ctx->slots + (size_t)loop * mpmi::slot_bytes();
  return check_hip(ctx, mpmi::launch_select(model, Nc, S, H, cand, first_violation, u_user, loop, slot, out,
                                            (hipStream_t)stream),
                   "select_min_intervention launch");
}

static mpmi_status validate_desc(mpmi_ctx ctx, const mpmi_system& sys, const mpmi_tick_desc* d) {
  if (!d) return fail(ctx, MPMI_EINVAL, "tick descriptor is NULL");
  if (d->n_cand < 0 || d->n_cand > MPMI_MAX_CAND - 1)
    return fail(ctx, MPMI_EINVAL, "n_cand=%d out of 0..%d", d->n_cand, MPMI_MAX_CAND - 1);
  if (d->horizon < 1 || d->horizon > MPMI_MAX_HORIZON)
    return fail(ctx, MPMI_EINVAL, "horizon=%d out of 1..%d", d->horizon, MPMI_MAX_HORIZON);
  if (d->n_seg < 1 || d->n_seg > MPMI_MAX_SEGMENTS)
    return fail(ctx, MPMI_EINVAL, "n_seg=%d out of 1..%d", d->n_seg, MPMI_MAX_SEGMENTS);
  if (d->loop < 0 || d->loop >= MPMI_MAX_LOOPS)
    return fail(ctx, MPMI_EINVAL, "loop=%d out of 0..%d", d->loop, MPMI_MAX_LOOPS - 1);
  if (d->block != 0 && (d->block < 64 || d->block > 1024 || d->block % 64 != 0))
    return fail(ctx, MPMI_EINVAL, "block=%d must be 0 or a multiple of 64 in 64..1024", d->block);
  if (d->precision != MPMI_PREC_FP32 && d->precision != MPMI_PREC_BF16X3 && d->precision != MPMI_PREC_FP32_RECHECK64)
    return fail(ctx, MPMI_EINVAL, "unknown precision %d", d->precision);
  if (d->lanes_per_cand != 0 && d->lanes_per_cand != 1 && d->lanes_per_cand != 2 && d->lanes_per_cand != 4 &&
      d->lanes_per_cand != 8)
    return fail(ctx, MPMI_EINVAL, "lanes_per_cand=%d must be 0, 1, 2, 4 or 8", d->lanes_per_cand);
  if (d->lanes_per_cand > 1 &&
      (d->precision != MPMI_PREC_FP32 || sys.basis == MPMI_BASIS_LINEAR || sys.basis == MPMI_BASIS_CUSTOM))
    return fail(ctx, MPMI_EUNSUPPORTED, "several lanes per candidate: FP32 ticks of the fixed bases only");
  if (sys.basis == MPMI_BASIS_CUSTOM && d->block > mpmi::kCustomBlock)
    return fail(ctx, MPMI_EUNSUPPORTED, "custom-basis ticks use at most %d threads per workgroup", mpmi::kCustomBlock);
  switch (d->gen) {
    case MPMI_GEN_EXPLICIT:
    case MPMI_GEN_UNIFORM:
      break;
    case MPMI_GEN_GRID: {
      if (d->n_seg != 1) return fail(ctx, MPMI_EINVAL, "GRID candidates need n_seg == 1");
      long long prod = 1;
      for (int j = 0; j < sys.n_input; ++j) {
        if (d->grid[j] < 1) return fail(ctx, MPMI_EINVAL, "grid[%d]=%d must be >= 1", j, d->grid[j]);
        prod *= d->grid[j];
      }
      if (prod != d->n_cand)
        return fail(ctx, MPMI_EINVAL, "grid product %lld != n_cand %d", prod, d->n_cand);
      break;
    }
    default:
      return fail(ctx, MPMI_EINVAL, "unknown candidate generator %d", d->gen);
  }
  return MPMI_OK;
}

mpmi_status mpmi_tick(mpmi_ctx ctx, const void* model, const mpmi_tick_desc* desc, const float* x_t,
                      const float* u_user, const float* cand, mpmi_selection* out, int16_t* first_violation,
                      float* traj, int64_t traj_ld, void* stream) {
  if (!ctx) return MPMI_EINVAL;
  mpmi_system sys;
  mpmi_status s = model_system(ctx, model, &sys, (hipStream_t)stream);
  if (s != MPMI_OK) return s;
  s = validate_desc(ctx, sys, desc);
  if (s != MPMI_OK) return s;
  if (!x_t || !u_user || !out) return fail(ctx, MPMI_EINVAL, "x_t, u_user and out must be non-NULL");
  if (desc->gen == MPMI_GEN_EXPLICIT && desc->n_cand > 0 && !cand)
    return fail(ctx, MPMI_EINVAL, "EXPLICIT candidates need cand");
  if (traj && traj_ld < (int64_t)desc->n_cand + 1)
    return fail(ctx, MPMI_EINVAL, "traj_ld=%lld below N+1=%d", (long long)traj_ld, desc->n_cand + 1);
  void* slot = (char*)ctx->slots + (size_t)desc->loop * mpmi::slot_bytes();
  if (desc->lanes_per_cand > 1) {
    if (traj) return fail(ctx, MPMI_EUNSUPPORTED, "several lanes per candidate: no trajectory store");
    if (desc->block > 256) return fail(ctx, MPMI_EUNSUPPORTED, "several lanes per candidate: block <= 256");
    if (mpmi::system_noisy(sys))
      return fail(ctx, MPMI_EUNSUPPORTED, "several lanes per candidate: noise-free models only");
    return check_hip(ctx, mpmi::launch_tick_split(sys, desc->lanes_per_cand, model, *desc, x_t, u_user, cand,
                                                  slot, out, first_violation, (hipStream_t)stream),
                     "mpmi_tick (split) launch");
  }
  if (desc->precision == MPMI_PREC_BF16X3) {
    if (sys.basis != MPMI_BASIS_RACE_CAR)
      return fail(ctx, MPMI_EUNSUPPORTED, "BF16X3 is implemented for race-car models");
    if (traj) return fail(ctx, MPMI_EUNSUPPORTED, "BF16X3 ticks do not store trajectories");
    if (mpmi::system_noisy(sys)) return fail(ctx, MPMI_EUNSUPPORTED, "BF16X3 ticks are noise-free");
    if (desc->block != 0 && desc->block != 256)
      return fail(ctx, MPMI_EUNSUPPORTED, "BF16X3 ticks use 256-thread workgroups");
    if ((long long)desc->n_cand + 1 > mpmi::kRecheckCapacity)
      return fail(ctx, MPMI_EUNSUPPORTED,
                  "BF16X3 ticks take at most %d candidates (the FP32 recheck list holds every one)",
                  mpmi::kRecheckCapacity);
    return check_hip(ctx, mpmi::launch_tick_bf16(sys, model, *desc, x_t, u_user, cand, slot, out, first_violation,
                                                 ctx->recheck, mpmi::kRecheckCapacity,
                                                 mpmi::device_cu_count() * 4, (hipStream_t)stream),
                     "mpmi_tick (BF16X3) launch");
  }
  if (desc->precision == MPMI_PREC_FP32_RECHECK64) {
    if ((long long)desc->n_cand + 1 > mpmi::kRecheckCapacity)
      return fail(ctx, MPMI_EUNSUPPORTED,
                  "FP32_RECHECK64 ticks take at most %d candidates (the FP64 recheck list holds every one)",
                  mpmi::kRecheckCapacity);
    return check_hip(ctx, mpmi::launch_tick(sys, model, *desc, x_t, u_user, cand, slot, out, first_violation, traj,
                                            traj ? traj_ld : 0, (hipStream_t)stream, nullptr, ctx->recheck,
                                            mpmi::kRecheckCapacity, mpmi::device_cu_count() * 4),
                     "mpmi_tick (FP32_RECHECK64) launch");
  }
  return check_hip(ctx, mpmi::launch_tick(sys, model, *desc, x_t, u_user, cand, slot, out, first_violation,
                                          traj, traj ? traj_ld : 0, (hipStream_t)stream),
                   "mpmi_tick launch");
}

mpmi_status mpmi_tick_autotune(mpmi_ctx ctx, const void* model, mpmi_tick_desc* desc, const float* x_t,
                               const float* u_user, const float* cand, mpmi_selection* out, int32_t reps,
                               float* best_ms, void* stream) {
  if (!ctx) return MPMI_EINVAL;
  if (!desc) return fail(ctx, MPMI_EINVAL, "desc is NULL");
  if (reps < 1 || reps > 100000) return fail(ctx, MPMI_EINVAL, "reps=%d out of 1..100000", reps);
  if (desc->precision != MPMI_PREC_FP32 && desc->precision != MPMI_PREC_FP32_RECHECK64)
    return fail(ctx, MPMI_EUNSUPPORTED, "the tick autotuner times FP32 and FP32_RECHECK64 ticks");
  mpmi_system sys;
  mpmi_status s = model_system(ctx, model, &sys, nullptr);
  if (s != MPMI_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return fail(ctx, MPMI_EDEVICE, "hipEventCreate failed");
  mpmi_tick_desc d = *desc;
  float bms = 1e30f;
  int bblock = 256, blanes = 1;
  for (int lanes : {1, 2, 4, 8}) {
    if (lanes > 1 && (sys.basis == MPMI_BASIS_LINEAR || sys.basis == MPMI_BASIS_CUSTOM || mpmi::system_noisy(sys) ||
                      desc->precision != MPMI_PREC_FP32))
      continue;
    for (int block : {64, 128, 256, 512}) {
      if (sys.basis == MPMI_BASIS_CUSTOM && block > mpmi::kCustomBlock) continue;
      if (lanes > 1 && block > 256) continue;
      d.block = block;
      d.lanes_per_cand = lanes;
      for (int w = 0; w < 2 && s == MPMI_OK; ++w)
        s = mpmi_tick(ctx, model, &d, x_t, u_user, cand, out, nullptr, nullptr, 0, stream);
      if (s == MPMI_OK && hipEventRecord(e0, st) != hipSuccess) s = MPMI_EDEVICE;
      for (int r = 0; r < reps && s == MPMI_OK; ++r)
        s = mpmi_tick(ctx, model, &d, x_t, u_user, cand, out, nullptr, nullptr, 0, stream);
      float ms = 0.0f;
      if (s == MPMI_OK && (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                           hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
        s = MPMI_EDEVICE;
      if (s != MPMI_OK) break;
      ms /= (float)reps;
      if (ms < bms) {
        bms = ms;
        bblock = block;
        blanes = lanes;
      }
    }
    if (s != MPMI_OK) break;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (s != MPMI_OK) return s;
  desc->block = bblock;
  desc->lanes_per_cand = blanes;
  if (best_ms) *best_ms = bms;
  return ok(ctx);
}

mpmi_status mpmi_fp32_fma_rate(mpmi_ctx ctx, double* tflops) {
  if (!ctx) return MPMI_EINVAL;
  if (!tflops) return fail(ctx, MPMI_EINVAL, "tflops is NULL");
  return check_hip(ctx, mpmi::measure_fma_rate((float*)ctx->fit_work, tflops), "mpmi_fp32_fma_rate");
}

mpmi_status mpmi_sincos64(mpmi_ctx ctx, const double* x, double* sn, double* cs, int32_t n, void* stream) {
  if (!ctx) return MPMI_EINVAL;
  if (n < 0) return fail(ctx, MPMI_EINVAL, "n=%d must be >= 0", n);
  if (n > 0 && (!x || !sn || !cs)) return fail(ctx, MPMI_EINVAL, "x, sn and cs must be non-NULL");
  return check_hip(ctx, mpmi::launch_sincos64(x, sn, cs, n, (hipStream_t)stream), "mpmi_sincos64");
}

mpmi_status mpmi_write_rates(mpmi_ctx ctx, float* buf, int32_t Nc, int64_t ld, int32_t rows, double* pattern_gbs,
                             double* stream_gbs) {
  if (!ctx) return MPMI_EINVAL;
  if (!buf || !pattern_gbs || !stream_gbs) return fail(ctx, MPMI_EINVAL, "buf, pattern_gbs and stream_gbs must be non-NULL");
  if (!aligned(buf, 16)) return fail(ctx, MPMI_EINVAL, "buf must be 16-byte aligned");
  if (Nc < 1 || rows < 1 || ld < Nc || (long long)ld * rows > (1ll << 33))
    return fail(ctx, MPMI_EINVAL, "Nc=%d ld=%lld rows=%d out of range", Nc, (long long)ld, rows);
  return check_hip(ctx, mpmi::measure_write_rates(buf, Nc, (long long)ld, rows, pattern_gbs, stream_gbs),
                   "mpmi_write_rates");
}

mpmi_status mpmi_read_rates(mpmi_ctx ctx, const float* buf, int32_t Nc, int64_t ld, int32_t rows, double* pattern_gbs,
                            double* stream_gbs) {
  if (!ctx) return MPMI_EINVAL;
  if (!buf || !pattern_gbs || !stream_gbs) return fail(ctx, MPMI_EINVAL, "buf, pattern_gbs and stream_gbs must be non-NULL");
  if (!aligned(buf, 16)) return fail(ctx, MPMI_EINVAL, "buf must be 16-byte aligned");
  if (Nc < 1 || rows < 1 || ld < Nc || (long long)ld * rows > (1ll << 33))
    return fail(ctx, MPMI_EINVAL, "Nc=%d ld=%lld rows=%d out of range", Nc, (long long)ld, rows);
  return check_hip(ctx, mpmi::measure_read_rates(buf, Nc, (long long)ld, rows, pattern_gbs, stream_gbs),
                   "mpmi_read_rates");
}

mpmi_status mpmi_generate_candidates(mpmi_ctx ctx, const void* model, const mpmi_tick_desc* desc,
                                     const float* u_user, const float* cand, float* cand_out, void* stream) {
  if (!ctx) return MPMI_EINVAL;
  mpmi_system sys;
  mpmi_status s = model_system(ctx, model, &sys, (hipStream_t)stream);
  if (s != MPMI_OK) return s;
  s = validate_desc(ctx, sys, desc);
  if (s != MPMI_OK) return s;
  if (!u_user || !cand_out) return fail(ctx, MPMI_EINVAL, "u_user and cand_out must be non-NULL");
  if (desc->gen == MPMI_GEN_EXPLICIT && desc->n_cand > 0 && !cand)
    return fail(ctx, MPMI_EINVAL, "EXPLICIT candidates need cand");
  return check_hip(ctx, mpmi::launch_gen(model, *desc, u_user, cand, cand_out, (hipStream_t)stream),
                   "mpmi_generate_candidates launch");
}

struct mpmi_multi_s {
  mpmi::MultiPlan plan;
};

mpmi_status mpmi_multi_create(mpmi_ctx ctx, const mpmi_loop_desc* loops, int32_t n_loops,
                              const mpmi_multi_config* cfg, mpmi_multi* out) {
  if (!ctx) return MPMI_EINVAL;
  if (!out) return fail(ctx, MPMI_EINVAL, "out is NULL");
  *out = nullptr;
  if (!loops) return fail(ctx, MPMI_EINVAL, "loops is NULL");
  if (n_loops < 1 || n_loops > MPMI_MAX_LOOPS)
    return fail(ctx, MPMI_EINVAL, "n_loops=%d out of 1..%d", n_loops, MPMI_MAX_LOOPS);
  const int block = cfg ? cfg->block : 256;
  const int grid = cfg ? cfg->grid : 0;
  const int prec = cfg ? cfg->precision : MPMI_PREC_FP32;
  if (block < 64 || block > 1024 || block % 64 != 0)
    return fail(ctx, MPMI_EINVAL, "block=%d must be a multiple of 64 in 64..1024", block);
  if (grid != 0) return fail(ctx, MPMI_EINVAL, "grid=%d must be 0 (one workgroup per work item)", grid);
  if (prec != MPMI_PREC_FP32 && prec != MPMI_PREC_FP32_RECHECK64)
    return fail(ctx, MPMI_EUNSUPPORTED, "many-loop ticks run FP32 or FP32_RECHECK64 (precision=%d)", prec);
  mpmi_multi m = new (std::nothrow) mpmi_multi_s();
  if (!m) return fail(ctx, MPMI_ENOMEM, "out of host memory");
  m->plan.n_loops = n_loops;
  m->plan.precision = prec;
  for (int l = 0; l < n_loops; ++l) {
    const mpmi_loop_desc& L = loops[l];
    mpmi_system sys;
    mpmi_status s = model_system(ctx, L.model, &sys, nullptr);
    if (s != MPMI_OK) {
      delete m;
      return fail(ctx, s, "loop %d: %s", l, ctx->err.c_str());
    }
    if (sys.basis == MPMI_BASIS_CUSTOM) {
      delete m;
      return fail(ctx, MPMI_EUNSUPPORTED, "loop %d: many-loop ticks serve the fixed bases (see mpmi_basis_match)", l);
    }
    mpmi_tick_desc d{};
    d.seed = L.seed;
    d.tick = L.tick;
    d.loop = 0;
    d.gen = L.gen;
    d.n_cand = L.n_cand;
    for (int j = 0; j < 4; ++j) d.grid[j] = L.grid[j];
    d.n_seg = L.n_seg;
    d.horizon = L.horizon;
    d.precision = MPMI_PREC_FP32;
    s = validate_desc(ctx, sys, &d);
    if (s != MPMI_OK) {
      delete m;
      return fail(ctx, s, "loop %d: %s", l, ctx->err.c_str());
    }
    if (!L.x_t || !L.u_user || !L.out || (L.gen == MPMI_GEN_EXPLICIT && L.n_cand > 0 && !L.cand)) {
      delete m;
      return fail(ctx, MPMI_EINVAL, "loop %d: x_t, u_user, out (and cand for EXPLICIT) must be non-NULL", l);
    }
    m->plan.host.push_back(L);
    m->plan.basis.push_back(sys.basis);
    m->plan.noisy = m->plan.noisy || mpmi::system_noisy(sys);
  }
  hipError_t e = mpmi::multi_alloc(m->plan);
  if (e == hipSuccess) e = mpmi::multi_plan(m->plan, block);
  if (e != hipSuccess) {
    mpmi::multi_free(m->plan);
    delete m;
    return fail(ctx, e == hipErrorOutOfMemory ? MPMI_ENOMEM : MPMI_EDEVICE, "mpmi_multi_create: %s",
                hipGetErrorString(e));
  }
  *out = m;
  return ok(ctx);
}

void mpmi_multi_destroy(mpmi_multi m) {
  if (!m) return;
  mpmi::multi_free(m->plan);
  delete m;
}

mpmi_status mpmi_multi_set_config(mpmi_ctx ctx, mpmi_multi m, const mpmi_multi_config* cfg) {
  if (!ctx) return MPMI_EINVAL;
  if (!m || !cfg) return fail(ctx, MPMI_EINVAL, "multi and cfg must be non-NULL");
  if (cfg->block < 64 || cfg->block > 1024 || cfg->block % 64 != 0)
    return fail(ctx, MPMI_EINVAL, "block=%d must be a multiple of 64 in 64..1024", cfg->block);
  if (cfg->grid != 0) return fail(ctx, MPMI_EINVAL, "grid=%d must be 0 (one workgroup per work item)", cfg->grid);
  if (cfg->precision != MPMI_PREC_FP32 && cfg->precision != MPMI_PREC_FP32_RECHECK64)
    return fail(ctx, MPMI_EUNSUPPORTED, "many-loop ticks run FP32 or FP32_RECHECK64 (precision=%d)", cfg->precision);
  mpmi_status s = check_hip(ctx, mpmi::multi_plan(m->plan, cfg->block), "mpmi_multi_set_config");
  if (s == MPMI_OK) m->plan.precision = cfg->precision;
  return s;
}

mpmi_status mpmi_multi_get_config(mpmi_multi m, mpmi_multi_config* cfg, int32_t* n_work_items) {
  if (!m) return MPMI_EINVAL;
  if (cfg) {
    cfg->block = m->plan.block;
    cfg->grid = m->plan.n_work;
    cfg->precision = m->plan.precision;
  }
  if (n_work_items) *n_work_items = m->plan.n_work;
  return MPMI_OK;
}

mpmi_status mpmi_multi_get_ticks(mpmi_ctx ctx, mpmi_multi m, uint64_t* ticks) {
  if (!ctx) return MPMI_EINVAL;
  if (!m || !ticks) return fail(ctx, MPMI_EINVAL, "multi and ticks must be non-NULL");
  hipError_t e = hipDeviceSynchronize();
  if (e == hipSuccess)
    e = hipMemcpy(ticks, m->plan.d_ticks, sizeof(uint64_t) * (size_t)m->plan.n_loops, hipMemcpyDeviceToHost);
  return check_hip(ctx, e, "mpmi_multi_get_ticks");
}

mpmi_status mpmi_multi_tick(mpmi_ctx ctx, mpmi_multi m, void* stream) {
  if (!ctx) return MPMI_EINVAL;
  if (!m) return fail(ctx, MPMI_EINVAL, "multi is NULL");
  return check_hip(ctx, mpmi::multi_launch(m->plan, (hipStream_t)stream), "mpmi_multi_tick launch");
}

mpmi_status mpmi_multi_autotune(mpmi_ctx ctx, mpmi_multi m, int32_t reps, mpmi_multi_config* best,
                                float* best_ms, void* stream) {
  if (!ctx) return MPMI_EINVAL;
  if (!m) return fail(ctx, MPMI_EINVAL, "multi is NULL");
  if (reps < 1 || reps > 100000) return fail(ctx, MPMI_EINVAL, "reps=%d out of 1..100000", reps);
  hipStream_t st = (hipStream_t)stream;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return fail(ctx, MPMI_EDEVICE, "hipEventCreate failed");
  float bms = 1e30f;
  int bblock = m->plan.block;
  hipError_t e = hipSuccess;
  for (int block : {64, 128, 256, 512, 1024}) {
    if ((e = mpmi::multi_plan(m->plan, block)) != hipSuccess) break;
    for (int w = 0; w < 2 && e == hipSuccess; ++w) e = mpmi::multi_launch(m->plan, st);
    if (e == hipSuccess) e = hipEventRecord(e0, st);
    for (int r = 0; r < reps && e == hipSuccess; ++r) e = mpmi::multi_launch(m->plan, st);
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e != hipSuccess) break;
    ms /= (float)reps;
    if (ms < bms) {
      bms = ms;
      bblock = block;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess) return fail(ctx, MPMI_EDEVICE, "mpmi_multi_autotune: %s", hipGetErrorString(e));
  e = mpmi::multi_plan(m->plan, bblock);
  if (e != hipSuccess) return fail(ctx, MPMI_EDEVICE, "mpmi_multi_autotune: %s", hipGetErrorString(e));
  if (best) {
    best->block = m->plan.block;
    best->grid = m->plan.n_work;
    best->precision = m->plan.precision;
  }
  if (best_ms) *best_ms = bms;
  return ok(ctx);
}

mpmi_status mpmi_multi_graph(mpmi_ctx ctx, mpmi_multi m, void** graph_exec) {
  if (!ctx) return MPMI_EINVAL;
  if (!m || !graph_exec) return fail(ctx, MPMI_EINVAL, "multi and graph_exec must be non-NULL");
  *graph_exec = nullptr;
  hipStream_t s = nullptr;
  hipGraph_t g = nullptr;
  hipGraphExec_t ge = nullptr;
  hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    hipError_t el = mpmi::multi_launch(m->plan, s);
    e = hipStreamEndCapture(s, &g);
    if (el != hipSuccess) e = el;
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
  if (g) (void)hipGraphDestroy(g);
  if (s) (void)hipStreamDestroy(s);
  if (e != hipSuccess) return fail(ctx, MPMI_EDEVICE, "mpmi_multi_graph: %s", hipGetErrorString(e));
  *graph_exec = (void*)ge;
  return ok(ctx);
}

mpmi_status mpmi_tick_graph(mpmi_ctx ctx, const void* model, const mpmi_tick_desc* desc, const float* x_t,
                            const float* u_user, const float* cand, mpmi_selection* out, int16_t* first_violation,
                            void** graph_exec) {
  if (!ctx) return MPMI_EINVAL;
  if (!graph_exec) return fail(ctx, MPMI_EINVAL, "graph_exec is NULL");
  *graph_exec = nullptr;
  hipStream_t s = nullptr;
  hipGraph_t g = nullptr;
  hipGraphExec_t ge = nullptr;
  mpmi_status st = MPMI_OK;
  hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    st = mpmi_tick(ctx, model, desc, x_t, u_user, cand, out, first_violation, nullptr, 0, (void*)s);
    e = hipStreamEndCapture(s, &g);
  }
  if (st == MPMI_OK && e == hipSuccess) e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
  if (g) (void)hipGraphDestroy(g);
  if (s) (void)hipStreamDestroy(s);
  if (st != MPMI_OK) return st;  // mpmi_tick's own message stays in ctx
  if (e != hipSuccess) return fail(ctx, MPMI_EDEVICE, "mpmi_tick_graph: %s", hipGetErrorString(e));
  *graph_exec = (void*)ge;
  return ok(ctx);
}

mpmi_status mpmi_graph_launch(mpmi_ctx ctx, void* graph_exec, void* stream) {
  if (!ctx) return MPMI_EINVAL;
  if (!graph_exec) return fail(ctx, MPMI_EINVAL, "graph_exec is NULL");
  return check_hip(ctx, hipGraphLaunch((hipGraphExec_t)graph_exec, (hipStream_t)stream), "mpmi_graph_launch");
}

void mpmi_graph_destroy(void* graph_exec) {
  if (graph_exec) (void)hipGraphExecDestroy((hipGraphExec_t)graph_exec);
}

size_t mlp_workspace_bytes(int32_t batch) {
  if (batch < 1 || batch > MPMI_MLP_MAX_BATCH) return 0;
  return mpmi::mlp_workspace_bytes(batch);
}

static mpmi_status check_mlp_common(mpmi_ctx ctx, const void* w16, const void* w32, const void* mean,
                                    const void* stdv, int32_t B, void* work, size_t work_bytes) {
  if (!w16 || !w32 || !mean || !stdv) return fail(ctx, MPMI_EINVAL, "weights, in_mean and in_std must be non-NULL");
  if (!aligned(w16, 16)) return fail(ctx, MPMI_EINVAL, "w_bf16 must be 16-byte aligned");
  if (B < 1 || B > MPMI_MLP_MAX_BATCH) return fail(ctx, MPMI_EINVAL, "batch %d out of 1..%d", B, MPMI_MLP_MAX_BATCH);
  if (!work || !aligned(work, 256)) return fail(ctx, MPMI_EINVAL, "workspace must be non-NULL and 256-byte aligned");
  if (work_bytes < mpmi::mlp_workspace_bytes(B))
    return fail(ctx, MPMI_EINVAL, "workspace of %zu bytes < mlp_workspace_bytes(%d) = %zu", work_bytes, B,
                mpmi::mlp_workspace_bytes(B));
  return MPMI_OK;
}

mpmi_status mlp_forward(mpmi_ctx ctx, const uint16_t* w_bf16, const float* w_f32, const float* in_mean,
                        const float* in_std, const float* X, int32_t B, float* Y, void* work, size_t work_bytes,
                        void* stream) {
  if (!ctx) return MPMI_EINVAL;
  mpmi_status s = check_mlp_common(ctx, w_bf16, w_f32, in_mean, in_std, B, work, work_bytes);
  if (s != MPMI_OK) return s;
  if (!X || !Y) return fail(ctx, MPMI_EINVAL, "X and Y must be non-NULL");
  return check_hip(ctx, mpmi::launch_mlp_forward(w_bf16, w_f32, in_mean, in_std, X, B, Y, work, (hipStream_t)stream),
                   "mlp_forward launch");
}

mpmi_status mlp_grad(mpmi_ctx ctx, const uint16_t* w_bf16, const float* w_f32, const float* in_mean,
                     const float* in_std, const float* X, const float* T, int32_t B, float* grad, float* loss,
                     void* work, size_t work_bytes, void* stream) {
  if (!ctx) return MPMI_EINVAL;
  mpmi_status s = check_mlp_common(ctx, w_bf16, w_f32, in_mean, in_std, B, work, work_bytes);
  if (s != MPMI_OK) return s;
  if (!X || !T || !grad) return fail(ctx, MPMI_EINVAL, "X, T and grad must be non-NULL");
  return check_hip(ctx, mpmi::launch_mlp_grad(w_bf16, w_f32, in_mean, in_std, X, T, B, grad, loss, work,
                                              (hipStream_t)stream),
                   "mlp_grad launch");
}

mpmi_status mlp_adam(mpmi_ctx ctx, float* w_f32, uint16_t* w_bf16, float* adam_m, float* adam_v, const float* grad,
                     int32_t step, float lr, void* stream) {
  if (!ctx) return MPMI_EINVAL;
  if (!w_f32 || !w_bf16 || !adam_m || !adam_v || !grad) return fail(ctx, MPMI_EINVAL, "NULL argument");
  if (step < 1) return fail(ctx, MPMI_EINVAL, "step=%d must be >= 1", step);
  if (!(lr > 0.0f)) return fail(ctx, MPMI_EINVAL, "lr must be > 0");
  return check_hip(ctx, mpmi::launch_mlp_adam(w_f32, w_bf16, adam_m, adam_v, grad, step, lr, (hipStream_t)stream),
                   "mlp_adam launch");
}

mpmi_status mdn_sample(mpmi_ctx ctx, const void* model, const float* head, int32_t P, uint64_t seed, uint64_t tick,
                       int32_t loop, float* cand, void* stream) {
  if (!ctx) return MPMI_EINVAL;
  mpmi_system sys;
  mpmi_status s = model_system(ctx, model, &sys, nullptr);
  if (s != MPMI_OK) return s;
  if (sys.n_input != 2) return fail(ctx, MPMI_EUNSUPPORTED, "the proposal head is over 2 inputs");
  if (!head || !cand) return fail(ctx, MPMI_EINVAL, "head and cand must be non-NULL");
  if (P < 1 || P > MPMI_MAX_CAND - 1) return fail(ctx, MPMI_EINVAL, "P=%d out of range", P);
  return check_hip(ctx, mpmi::launch_mdn_sample(model, head, P, seed, tick, loop, cand, (hipStream_t)stream),
                   "mdn_sample launch");
}

mpmi_status mpmi_proposal_tick(mpmi_ctx ctx, const void* model, const uint16_t* w_bf16, const float* w_f32,
                               const float* in_mean, const float* in_std, const float* x_t, const float* u_user,
                               const mpmi_tick_desc* prop, const mpmi_tick_desc* fallback, float* cand_work,
                               float* head_out, mpmi_selection* out, void* work, size_t work_bytes, void* stream) {
  if (!ctx) return MPMI_EINVAL;
  mpmi_system sys;
  mpmi_status s = model_system(ctx, model, &sys, nullptr);
  if (s != MPMI_OK) return s;
  if (sys.basis != MPMI_BASIS_RACE_CAR) return fail(ctx, MPMI_EUNSUPPORTED, "the proposal network serves race-car models");
  s = check_mlp_common(ctx, w_bf16, w_f32, in_mean, in_std, 1, work, work_bytes);
  if (s != MPMI_OK) return s;
  if (!prop || !fallback) return fail(ctx, MPMI_EINVAL, "prop and fallback descriptors must be non-NULL");
  mpmi_tick_desc pd = *prop;
  pd.gen = MPMI_GEN_EXPLICIT;
  if ((s = validate_desc(ctx, sys, &pd)) != MPMI_OK) return s;
  if ((s = validate_desc(ctx, sys, fallback)) != MPMI_OK) return s;
  if (pd.n_cand < 1 || pd.n_seg != 1) return fail(ctx, MPMI_EINVAL, "proposals need n_cand >= 1 and n_seg == 1");
  if (fallback->gen == MPMI_GEN_EXPLICIT) return fail(ctx, MPMI_EINVAL, "the fallback must be GRID or UNIFORM");
  const bool r64 = pd.precision == MPMI_PREC_FP32_RECHECK64, fb64 = fallback->precision == MPMI_PREC_FP32_RECHECK64;
  if ((pd.precision != MPMI_PREC_FP32 && !r64) || (fallback->precision != MPMI_PREC_FP32 && !fb64))
    return fail(ctx, MPMI_EUNSUPPORTED, "proposal ticks are FP32 or FP32_RECHECK64");
  if (r64 && pd.lanes_per_cand > 1)
    return fail(ctx, MPMI_EUNSUPPORTED, "FP32_RECHECK64 proposal ticks run one lane per candidate");
  if ((r64 && (long long)pd.n_cand + 1 > mpmi::kRecheckCapacity) ||
      (fb64 && (long long)fallback->n_cand + 1 > mpmi::kRecheckCapacity))
    return fail(ctx, MPMI_EUNSUPPORTED, "FP32_RECHECK64 ticks take at most %d candidates", mpmi::kRecheckCapacity);
  if (!x_t || !u_user || !cand_work || !out) return fail(ctx, MPMI_EINVAL, "x_t, u_user, cand_work, out must be non-NULL");
  if (!aligned(w_bf16, 16)) return fail(ctx, MPMI_EINVAL, "w_bf16 must be 16-byte aligned");
  if (pd.lanes_per_cand > 1 && mpmi::system_noisy(sys))
    return fail(ctx, MPMI_EUNSUPPORTED, "several lanes per candidate: noise-free models only");
  hipStream_t st = (hipStream_t)stream;
  float* head = nullptr;
  hipError_t e = mpmi::launch_mlp_row_forward(x_t, u_user, w_bf16, w_f32, in_mean, in_std, work, head_out, &head,
                                              model, pd.n_cand, pd.seed, pd.tick, pd.loop, cand_work, st);
  void* slot = (char*)ctx->slots + (size_t)pd.loop * mpmi::slot_bytes();
  if (e == hipSuccess) {
    if (pd.lanes_per_cand > 1)
      e = mpmi::launch_tick_split(sys, pd.lanes_per_cand, model, pd, x_t, u_user, cand_work, slot, out, nullptr,
                                  st);
    else if (r64)
      e = mpmi::launch_tick(sys, model, pd, x_t, u_user, cand_work, slot, out, nullptr, nullptr, 0, st, nullptr,
                            ctx->recheck, mpmi::kRecheckCapacity, mpmi::device_cu_count() * 4);
    else
      e = mpmi::launch_tick(sys, model, pd, x_t, u_user, cand_work, slot, out, nullptr, nullptr, 0, st);
  }
  void* slot2 = (char*)ctx->slots + (size_t)fallback->loop * mpmi::slot_bytes();
  if (e == hipSuccess) {
    if (fb64)
      e = mpmi::launch_tick(sys, model, *fallback, x_t, u_user, nullptr, slot2, out, nullptr, nullptr, 0, st, out,
                            ctx->recheck, mpmi::kRecheckCapacity, mpmi::device_cu_count() * 4);
    else
      e = mpmi::launch_tick(sys, model, *fallback, x_t, u_user, nullptr, slot2, out, nullptr, nullptr, 0, st, out);
  }
  return check_hip(ctx, e, "mpmi_proposal_tick launch");
}

mpmi_status mpmi_gemm_bf16(mpmi_ctx ctx, const uint16_t* A, const uint16_t* B, int32_t M, int32_t N, int32_t K,
                           int32_t ta, int32_t tb, float* C, void* stream) {
  if (!ctx) return MPMI_EINVAL;
  if (!A || !B || !C) return fail(ctx, MPMI_EINVAL, "NULL argument");
  if (M < 1 || N < 1 || K < 1 || (ta != 0 && ta != 1) || (tb != 0 && tb != 1))
    return fail(ctx, MPMI_EINVAL, "bad GEMM shape or transpose flag");
  return check_hip(ctx, mpmi::launch_gemm_test(A, B, M, N, K, ta, tb, C, (hipStream_t)stream), "mpmi_gemm_bf16");
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Allocation-free tick (mpmi_tick_noalloc).  The tick's scratch -- the
// selection slots of kScratchLoops loops and one FP64 re-roll list of
// kScratchRecheck entries (and as many kept entries) -- is one file-scope
// device object, `scratch`, whose load-time image is already the reset state
// (keys all-ones, counts zero): the workgroup that finalises a tick (of the
// tick launch, or of the re-roll launch) leaves it in that state again, so no
// call ever has to clear it.  Every device the library
// runs on holds its own copy until the process ends; its address on a device
// is taken once, with that device current, by hipGetSymbolAddress, and only
// that address is passed to kernels.
// ---------------------------------------------------------------------------
namespace {

constexpr int kScratchLoops = 64;
constexpr int kScratchRecheck = 1 << 16;
constexpr int kScratchDevices = 64;

struct alignas(64) ScratchSubSlot {
  unsigned long long key_safe = ~0ull, key_fb = ~0ull, count = 0ull;
  unsigned int n_recheck = 0u, pad0 = 0u;
  unsigned long long key_safe64 = ~0ull;
  unsigned int pad[6] = {};
};
struct alignas(64) ScratchSlot {
  ScratchSubSlot sub[mpmi::kSubSlots];
  unsigned int done = 0u;
  unsigned int pad[15] = {};
};
struct alignas(256) ScratchImage {
  ScratchSlot slots[kScratchLoops];
  unsigned int count = 0u;  // the re-roll list: a RecheckList of kScratchRecheck entries
  unsigned int n_keep = 0u;
  unsigned int pad[62] = {};
  int idx[kScratchRecheck] = {};
  int keep[kScratchRecheck] = {};
};
static_assert(sizeof(ScratchSlot) == sizeof(mpmi::Slot) && sizeof(ScratchSubSlot) == sizeof(mpmi::SubSlot) &&
                  offsetof(ScratchSubSlot, key_fb) == offsetof(mpmi::SubSlot, key_fb) &&
                  offsetof(ScratchSubSlot, count) == offsetof(mpmi::SubSlot, count) &&
                  offsetof(ScratchSubSlot, n_recheck) == offsetof(mpmi::SubSlot, n_recheck) &&
                  offsetof(ScratchSubSlot, key_safe64) == offsetof(mpmi::SubSlot, key_safe64) &&
                  offsetof(ScratchSlot, done) == offsetof(mpmi::Slot, done),
              "scratch slots have the library's slot layout");
static_assert(offsetof(ScratchImage, count) == (size_t)kScratchLoops * sizeof(mpmi::Slot) &&
                  offsetof(ScratchImage, n_keep) - offsetof(ScratchImage, count) ==
                      offsetof(mpmi::RecheckList, n_keep) &&
                  offsetof(ScratchImage, idx) - offsetof(ScratchImage, count) == offsetof(mpmi::RecheckList, idx) &&
                  offsetof(ScratchImage, keep) == offsetof(ScratchImage, idx) + sizeof(int) * kScratchRecheck,
              "scratch list has the recheck list's layout");

static __device__ __align__(256) ScratchImage scratch[1];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kScratchDevices] = {};

// This device's address of `scratch` (taken on the first call on the device).
mpmi_status scratch_address(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(nullptr, MPMI_EDEVICE, "mpmi_tick_noalloc: hipGetDevice: %s", hipGetErrorString(e));
  if (dev < 0 || dev >= kScratchDevices)
    return fail(nullptr, MPMI_EUNSUPPORTED, "mpmi_tick_noalloc: device %d beyond the %d the library serves", dev,
                kScratchDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(nullptr, MPMI_EDEVICE, "mpmi_tick_noalloc: hipGetSymbolAddress: %s", hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return MPMI_OK;
}

}  // namespace

extern "C" mpmi_status mpmi_tick_noalloc(const mpmi_system* sys, const void* model, const mpmi_tick_desc* desc,
                                         const float* x_t, const float* u_user, const float* cand,
                                         mpmi_selection* out, int16_t* first_violation, void* stream) {
  mpmi_status s = validate_system(nullptr, sys);
  if (s != MPMI_OK) return s;
  s = validate_desc(nullptr, *sys, desc);
  if (s != MPMI_OK) return s;
  if (!model || !aligned(model, 256)) return fail(nullptr, MPMI_EINVAL, "model must be non-NULL and 256-byte aligned");
  if (!x_t || !u_user || !out) return fail(nullptr, MPMI_EINVAL, "x_t, u_user and out must be non-NULL");
  if (desc->gen == MPMI_GEN_EXPLICIT && desc->n_cand > 0 && !cand)
    return fail(nullptr, MPMI_EINVAL, "EXPLICIT candidates need cand");
  if (desc->loop >= kScratchLoops)
    return fail(nullptr, MPMI_EINVAL, "loop=%d: the allocation-free tick has %d selection slots", desc->loop,
                kScratchLoops);
  if (desc->precision == MPMI_PREC_BF16X3)
    return fail(nullptr, MPMI_EUNSUPPORTED, "the allocation-free tick runs FP32 and FP32_RECHECK64 ticks");
  if (desc->precision == MPMI_PREC_FP32_RECHECK64 && (long long)desc->n_cand + 1 > kScratchRecheck)
    return fail(nullptr, MPMI_EUNSUPPORTED,
                "FP32_RECHECK64 ticks without allocation take at most %d candidates (N+1=%lld)", kScratchRecheck,
                (long long)desc->n_cand + 1);
  if (desc->lanes_per_cand > 1) {
    if (desc->block > 256) return fail(nullptr, MPMI_EUNSUPPORTED, "several lanes per candidate: block <= 256");
    if (mpmi::system_noisy(*sys))
      return fail(nullptr, MPMI_EUNSUPPORTED, "several lanes per candidate: noise-free models only");
  }
  void* base = nullptr;
  s = scratch_address(&base);
  if (s != MPMI_OK) return s;
  void* slot = (char*)base + (size_t)desc->loop * sizeof(mpmi::Slot);
  void* list = (char*)base + offsetof(ScratchImage, count);
  const hipStream_t st = (hipStream_t)stream;
  hipError_t e;
  if (desc->lanes_per_cand > 1)
    e = mpmi::launch_tick_split(*sys, desc->lanes_per_cand, model, *desc, x_t, u_user, cand, slot, out,
                                first_violation, st);
  else if (desc->precision == MPMI_PREC_FP32_RECHECK64)
    e = mpmi::launch_tick(*sys, model, *desc, x_t, u_user, cand, slot, out, first_violation, nullptr, 0, st, nullptr,
                          list, kScratchRecheck, mpmi::device_cu_count() * 4);
  else
    e = mpmi::launch_tick(*sys, model, *desc, x_t, u_user, cand, slot, out, first_violation, nullptr, 0, st);
  if (e != hipSuccess) return fail(nullptr, MPMI_EDEVICE, "mpmi_tick_noalloc launch: %s", hipGetErrorString(e));
  g_noctx_err.clear();
  return MPMI_OK;
}
