// api.cpp — host side of libhr2: contexts, resident tables, observation
// layouts, validation, staging and the launch sequence of the forward model
// (level records -> fused opacity/RT column kernel -> convolve/bin kernel).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>
#include <cmath>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "hr2_context.h"
#include "hr2_internal.h"

using namespace hr2;

// ------------------------------------------------------------------ errors
namespace hr2 {
thread_local std::string g_last_error;

hr2_status set_error(hr2_status st, const std::string &msg) {
  g_last_error = msg;
  return st;
}

hr2_status hip_error(hipError_t e, const char *what) {
  return set_error(HR2_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}
}  // namespace hr2

#define HIP_TRY(expr)                                    \
  do {                                                   \
    hipError_t e_ = (expr);                              \
    if (e_ != hipSuccess) return hip_error(e_, #expr);   \
  } while (0)

extern "C" const char *hr2_last_error(void) { return g_last_error.c_str(); }

// ------------------------------------------------------------ device buffers
namespace hr2 {

hr2_status DevBuf::ensure(size_t bytes) {
  if (bytes <= cap) return HR2_OK;
  size_t want = std::max<size_t>(bytes, 4096);
  want = (want + 255) & ~size_t(255);
  void *fresh = nullptr;
  if (hipMalloc(&fresh, want) != hipSuccess) {
    (void)hipGetLastError();
    return set_error(HR2_E_NO_MEMORY, "device allocation of " + std::to_string(want) + " bytes failed");
  }
  // the old buffer may still be read by enqueued work or a captured graph:
  // keep it until the owner frees it at a safe point
  if (ptr != nullptr) retired.push_back(ptr);
  ptr = fresh;
  cap = want;
  return HR2_OK;
}

void DevBuf::free_retired() {
  for (void *p : retired) (void)hipFree(p);
  retired.clear();
}

void DevBuf::release() {
  free_retired();
  if (ptr) (void)hipFree(ptr);
  ptr = nullptr;
  cap = 0;
}

// Gauss-Legendre nodes on [0, 1] (Eq. 8): roots of P_n by Newton's method.
static void gauss_legendre_01(int n, double *mu, double *w) {
  const double pi = 3.14159265358979323846;
  for (int i = 0; i < n; ++i) {
    double z = std::cos(pi * (i + 0.75) / (n + 0.5));
    double dpn = 1.0;
    for (int it = 0; it < 200; ++it) {
      double pa = 1.0, pb = 0.0;
      for (int k = 1; k <= n; ++k) {
        const double pc = pb;
        pb = pa;
        pa = ((2.0 * k - 1.0) * z * pb - (k - 1.0) * pc) / k;
      }
      dpn = n * (z * pa - pb) / (z * z - 1.0);
      const double step = pa / dpn;
      z -= step;
      if (std::fabs(step) <= 1e-16) {
        double qa = 1.0, qb = 0.0;
        for (int k = 1; k <= n; ++k) {
          const double qc = qb;
          qb = qa;
          qa = ((2.0 * k - 1.0) * z * qb - (k - 1.0) * qc) / k;
        }
        dpn = n * (z * qa - qb) / (z * z - 1.0);
        break;
      }
    }
    mu[n - 1 - i] = 0.5 * (1.0 + z);
    w[n - 1 - i] = 1.0 / ((1.0 - z * z) * dpn * dpn);
  }
}

static AngleTable make_angle_table() {
  AngleTable t;
  std::memset(&t, 0, sizeof(t));
  const double pi = 3.14159265358979323846;
  const double log2e = 1.4426950408889634074;
  for (int n = 1; n <= kMaxMu; ++n) {
    double mu[kMaxMu], w[kMaxMu];
    gauss_legendre_01(n, mu, w);
    // slots past the n nodes: a valid direction (mu = 1) of weight 0, so a
    // kernel may run them unguarded and add exactly zero to the flux
    for (int k = n; k < kMaxMu; ++k) {
      t.mu[n - 1][k] = t.inv_mu[n - 1][k] = 1.0f;
      t.l2e_mu[n - 1][k] = (float)log2e;
      t.mu_d[n - 1][k] = t.inv_mu_d[n - 1][k] = 1.0;
    }
    for (int k = 0; k < n; ++k) {
      t.mu[n - 1][k] = (float)mu[k];
      t.inv_mu[n - 1][k] = (float)(1.0 / mu[k]);
      t.l2e_mu[n - 1][k] = (float)(log2e / mu[k]);
      t.cw[n - 1][k] = (float)(2.0 * pi * w[k] * mu[k]);
      t.mu_d[n - 1][k] = mu[k];
      t.inv_mu_d[n - 1][k] = 1.0 / mu[k];
      t.cw_d[n - 1][k] = 2.0 * pi * w[k] * mu[k];
    }
  }
  return t;
}

// Make `stream` wait for the context's previous use of its scratch, so
// scratch reuse is ordered even when calls alternate streams.
// (Under stream capture the captured calls are ordered by the graph itself
// and an event from outside the capture may not be waited on: skip both.)
static bool capturing(hipStream_t stream) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(stream, &cs) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return cs != hipStreamCaptureStatusNone;
}

// Scratch superseded by growth is freed once every earlier call of the
// context has completed (calls are ordered through scratch_event, so the
// last call's event covers all of them), never after a call was captured.
static void free_retired_scratch(hr2_ctx *ctx) {
  DevBuf *bufs[] = {&ctx->recs, &ctx->fplus, &ctx->cols, &ctx->terms, &ctx->unpacked};
  bool any = false;
  for (DevBuf *b : bufs) any |= !b->retired.empty();
  if (!any || ctx->captured) return;
  if (ctx->scratch_used) {
    const hipError_t q = hipEventQuery(ctx->scratch_event);
    if (q != hipSuccess) {
      (void)hipGetLastError();   // not ready (or failed): try again on a later call
      return;
    }
  }
  for (DevBuf *b : bufs) b->free_retired();
}

hr2_status ctx_begin(hr2_ctx *ctx, hipStream_t stream) {
  HIP_TRY(hipSetDevice(ctx->device));
  if (capturing(stream)) {
    ctx->captured = true;
    return HR2_OK;
  }
  free_retired_scratch(ctx);
  if (ctx->scratch_used) HIP_TRY(hipStreamWaitEvent(stream, ctx->scratch_event, 0));
  return HR2_OK;
}

hr2_status ctx_end(hr2_ctx *ctx, hipStream_t stream) {
  if (capturing(stream)) return HR2_OK;
  HIP_TRY(hipEventRecord(ctx->scratch_event, stream));
  ctx->scratch_used = true;
  return HR2_OK;
}

// Copy `bytes` host bytes to device scratch `dst` through pinned staging.
hr2_status stage_upload(hr2_ctx *ctx, DevBuf &dst, const void *src, size_t bytes,
                        hipStream_t stream) {
  if (bytes == 0) return HR2_OK;
  if (capturing(stream))
    return set_error(HR2_E_UNSUPPORTED,
                     "a staging copy cannot be captured: make the same call once before capture");
  hr2_status st = dst.ensure(bytes);
  if (st != HR2_OK) return st;
  if (ctx->pinned_pending) {
    HIP_TRY(hipEventSynchronize(ctx->pinned_event));
    ctx->pinned_pending = false;
  }
  if (ctx->pinned_cap < bytes) {
    if (ctx->pinned) HIP_TRY(hipHostFree(ctx->pinned));
    ctx->pinned = nullptr;
    size_t want = std::max<size_t>(bytes, 1 << 16);
    HIP_TRY(hipHostMalloc(&ctx->pinned, want, hipHostMallocDefault));
    ctx->pinned_cap = want;
  }
  std::memcpy(ctx->pinned, src, bytes);
  HIP_TRY(hipMemcpyAsync(dst.ptr, ctx->pinned, bytes, hipMemcpyHostToDevice, stream));
  HIP_TRY(hipEventRecord(ctx->pinned_event, stream));
  ctx->pinned_pending = true;
  return HR2_OK;
}

}  // namespace hr2

// ----------------------------------------------------------------- context
extern "C" hr2_status hr2_ctx_create(int hip_device, hr2_ctx **out) {
  if (out == nullptr) return set_error(HR2_E_INVALID_ARG, "out is NULL");
  *out = nullptr;
  int n_dev = 0;
  if (hipGetDeviceCount(&n_dev) != hipSuccess || hip_device < 0 || hip_device >= n_dev) {
    (void)hipGetLastError();
    return set_error(HR2_E_DEVICE, "no HIP device " + std::to_string(hip_device));
  }
  HIP_TRY(hipSetDevice(hip_device));
  auto *ctx = new hr2_ctx();
  ctx->device = hip_device;
  hipError_t e = hipStreamCreateWithFlags(&ctx->internal, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&ctx->scratch_event, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&ctx->pinned_event, hipEventDisableTiming);
  if (e == hipSuccess) e = upload_angle_table(make_angle_table());
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    hr2_ctx_destroy(ctx);
    return hip_error(e, "context setup");
  }
  // the allocation-free entry point's fixed array: its address on this device
  const hr2_status sst = noalloc_scratch_init(hip_device);
  if (sst != HR2_OK) {
    hr2_ctx_destroy(ctx);
    return sst;
  }
  *out = ctx;
  return HR2_OK;
}

extern "C" void hr2_ctx_destroy(hr2_ctx *ctx) {
  if (ctx == nullptr) return;
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  ctx->recs.release();
  ctx->fplus.release();
  ctx->cols.release();
  ctx->terms.release();
  ctx->unpacked.release();
  if (ctx->pinned) (void)hipHostFree(ctx->pinned);
  for (hipEvent_t ev : ctx->tev) (void)hipEventDestroy(ev);
  if (ctx->scratch_event) (void)hipEventDestroy(ctx->scratch_event);
  if (ctx->pinned_event) (void)hipEventDestroy(ctx->pinned_event);
  if (ctx->internal) (void)hipStreamDestroy(ctx->internal);
  delete ctx;
}

extern "C" hr2_status hr2_ctx_set_option(hr2_ctx *ctx, hr2_option opt, int value) {
  if (ctx == nullptr) return set_error(HR2_E_INVALID_ARG, "ctx is NULL");
  switch (opt) {
    case HR2_OPT_CHUNKS:
      if (value < 0 || value > 8) return set_error(HR2_E_INVALID_ARG, "chunks must be in [0, 8]");
      ctx->opt_chunks = value;
      return HR2_OK;
    case HR2_OPT_NU_PER_LANE:
      if (value < 0 || value > 2)
        return set_error(HR2_E_UNSUPPORTED, "wavenumbers per lane must be 0 (auto), 1 or 2");
      ctx->opt_nu_per_lane = value;
      return HR2_OK;
    case HR2_OPT_TIMING:
      if (value < 0) return set_error(HR2_E_INVALID_ARG, "timing period must be >= 0");
      ctx->timing_every = value;
      ctx->timing_calls = 0;
      return HR2_OK;
    case HR2_OPT_SOURCE:
      if (value != 1 && value != 2)
        return set_error(HR2_E_INVALID_ARG, "source order must be 1 (linear) or 2 (parabolic)");
      ctx->opt_source = value;
      return HR2_OK;
    case HR2_OPT_ROW_POLICY:
      if (value < 0 || value > 2)
        return set_error(HR2_E_INVALID_ARG, "row policy must be 0 (auto), 1 or 2");
      ctx->opt_row_policy = value;
      return HR2_OK;
    case HR2_OPT_TIMING_KERNELS:
      if (value < 1 || value > 7)
        return set_error(HR2_E_INVALID_ARG, "timed kernels: a mask of 1 (levels), 2 (column), "
                                            "4 (convolution), 1 .. 7");
      ctx->timing_kernels = value;
      return HR2_OK;
    case HR2_OPT_TILE_PAIRS:
      if (value < 0 || value > 1)
        return set_error(HR2_E_INVALID_ARG, "tile pairs must be 0 (auto) or 1 (off)");
      ctx->opt_tile_pairs = value;
      return HR2_OK;

  }
  return set_error(HR2_E_INVALID_ARG, "unknown option");
}

// ------------------------------------------------------------------ tables
namespace {

constexpr double kLog2of10 = 3.32192809488736234787031942948939017586;

bool finite_increasing(const double *a, int n) {
  for (int i = 0; i < n; ++i) {
    if (!std::isfinite(a[i])) return false;
    if (i > 0 && !(a[i] > a[i - 1])) return false;
  }
  return true;
}

inline uint16_t to_bf16(double y) {
  const float f = (float)y;   // first rounding: RNE to float
  uint32_t u;
  std::memcpy(&u, &f, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);   // second rounding: RNE to bfloat16
  return (uint16_t)(u >> 16);
}

// Convert rows of log10 values to stored log2 values minus the row offset
// (midpoint of the row's log2 range, or fixed_off[r] when given); returns
// false on a non-finite input.
template <typename TT>
bool convert_rows(const double *src, int64_t n_rows, int64_t n_nu, int64_t pitch, bool offset,
                  TT *dst, double *off, const double *fixed_off = nullptr) {
  bool ok = true;
  const int n_thr = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  std::vector<std::thread> pool;
  std::vector<char> row_ok(n_thr, 1);
  for (int t = 0; t < n_thr; ++t) {
    pool.emplace_back([=, &row_ok]() {
      for (int64_t r = t; r < n_rows; r += n_thr) {
        const double *a = src + r * n_nu;
        double lo = INFINITY, hi = -INFINITY;
        for (int64_t k = 0; k < n_nu; ++k) {
          const double y = a[k] * kLog2of10;
          if (!std::isfinite(y)) row_ok[t] = 0;
          lo = std::min(lo, y);
          hi = std::max(hi, y);
        }
        const double o = !offset ? 0.0 : (fixed_off ? fixed_off[r] : 0.5 * (lo + hi));
        off[r] = o;
        TT *d = dst + r * pitch;
        for (int64_t k = 0; k < n_nu; ++k) {
          const double y = a[k] * kLog2of10 - o;
          if constexpr (std::is_same<TT, uint16_t>::value)
            d[k] = to_bf16(y);
          else
            d[k] = (TT)y;
        }
        for (int64_t k = n_nu; k < pitch; ++k) d[k] = (TT)0;
      }
    });
  }
  for (auto &th : pool) th.join();
  for (char c : row_ok) ok = ok && c;
  return ok;
}

// Midpoint of each species' log2 range (rows_per_species rows each), copied
// to every row of the species; false on a non-finite input.
bool species_offsets(const double *src, int n_species, int64_t rows_per_species, int64_t n_nu,
                     std::vector<double> &row_off) {
  row_off.assign((size_t)n_species * rows_per_species, 0.0);
  const int64_t n_rows = (int64_t)n_species * rows_per_species;
  const int n_thr = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  std::vector<double> lo(n_rows, INFINITY), hi(n_rows, -INFINITY);
  std::vector<char> ok(n_thr, 1);
  std::vector<std::thread> pool;
  for (int t = 0; t < n_thr; ++t) {
    pool.emplace_back([=, &lo, &hi, &ok]() {
      for (int64_t r = t; r < n_rows; r += n_thr) {
        const double *a = src + r * n_nu;
        for (int64_t k = 0; k < n_nu; ++k) {
          const double y = a[k] * kLog2of10;
          if (!std::isfinite(y)) ok[t] = 0;
          lo[r] = std::min(lo[r], y);
          hi[r] = std::max(hi[r], y);
        }
      }
    });
  }
  for (auto &th : pool) th.join();
  for (char c : ok)
    if (!c) return false;
  for (int q = 0; q < n_species; ++q) {
    double l = INFINITY, h = -INFINITY;
    for (int64_t r = 0; r < rows_per_species; ++r) {
      l = std::min(l, lo[q * rows_per_species + r]);
      h = std::max(h, hi[q * rows_per_species + r]);
    }
    for (int64_t r = 0; r < rows_per_species; ++r) row_off[q * rows_per_species + r] = 0.5 * (l + h);
  }
  return true;
}

template <typename TT>
hr2_status upload_table(const double *src, int64_t n_rows, int64_t n_nu, int64_t pitch,
                        bool offset, void **dptr, double *off, size_t *bytes_out,
                        const double *fixed_off = nullptr) {
  const size_t bytes = (size_t)n_rows * pitch * sizeof(TT);
  if (hipMalloc(dptr, bytes) != hipSuccess) {
    *dptr = nullptr;
    (void)hipGetLastError();
    return set_error(HR2_E_NO_MEMORY, "table allocation failed");
  }
  *bytes_out += bytes;
  // convert and copy in blocks of rows to bound host memory
  const int64_t rows_per_block = std::max<int64_t>(1, (int64_t)((256u << 20) / (pitch * sizeof(TT))));
  std::vector<TT> buf;
  for (int64_t r0 = 0; r0 < n_rows; r0 += rows_per_block) {
    const int64_t nr = std::min(rows_per_block, n_rows - r0);
    buf.resize((size_t)nr * pitch);
    if (!convert_rows<TT>(src + r0 * n_nu, nr, n_nu, pitch, offset, buf.data(), off + r0,
                          fixed_off ? fixed_off + r0 : nullptr))
      return set_error(HR2_E_INVALID_ARG, "table holds a non-finite value");
    HIP_TRY(hipMemcpy((TT *)*dptr + r0 * pitch, buf.data(), (size_t)nr * pitch * sizeof(TT),
                      hipMemcpyHostToDevice));
  }
  return HR2_OK;
}

}  // namespace

extern "C" hr2_status hr2_tables_create(hr2_ctx *ctx, const hr2_tables_desc *d, hr2_tables **out) {
  if (ctx == nullptr || d == nullptr || out == nullptr)
    return set_error(HR2_E_INVALID_ARG, "NULL argument");
  *out = nullptr;
  if (d->n_species < 1 || d->n_species > HR2_MAX_SPECIES)
    return set_error(HR2_E_INVALID_ARG, "n_species must be in [1, 12]");
  if (d->n_T < 2 || d->n_p < 2 || d->n_T > 256 || d->n_p > 256)
    return set_error(HR2_E_INVALID_ARG, "n_T and n_p must be in [2, 256]");
  if (d->n_nu < 1 || d->n_nu > (int64_t(1) << 31) - 4096)
    return set_error(HR2_E_INVALID_ARG, "n_nu out of range");
  if (!d->T_K || !d->log10_p_bar || !d->log10_sigma || !d->molar_mass)
    return set_error(HR2_E_INVALID_ARG, "NULL table array");
  if (d->n_cia != 0 && d->n_cia != 2) return set_error(HR2_E_INVALID_ARG, "n_cia must be 0 or 2");
  if (d->n_cia == 2 && !d->log10_k_cia) return set_error(HR2_E_INVALID_ARG, "NULL CIA table");
  if (!finite_increasing(d->T_K, d->n_T) || !(d->T_K[0] > 0))
    return set_error(HR2_E_INVALID_ARG, "T axis must be positive and strictly increasing");
  if (!finite_increasing(d->log10_p_bar, d->n_p))
    return set_error(HR2_E_INVALID_ARG, "log10 p axis must be strictly increasing");
  if (!(d->nu0_cm > 0) || !(d->dnu_cm > 0) || !std::isfinite(d->nu0_cm) || !std::isfinite(d->dnu_cm))
    return set_error(HR2_E_INVALID_ARG, "nu0 and dnu must be positive");
  if (!(d->he_h2_ratio > 0) || !std::isfinite(d->he_h2_ratio))
    return set_error(HR2_E_INVALID_ARG, "he_h2_ratio must be positive");
  for (int s = 0; s < d->n_species; ++s)
    if (!(d->molar_mass[s] > 0) || !std::isfinite(d->molar_mass[s]))
      return set_error(HR2_E_INVALID_ARG, "molar masses must be positive");
  if (d->dtype < HR2_TABLE_F32 || d->dtype > HR2_TABLE_F64)
    return set_error(HR2_E_INVALID_ARG, "unknown table dtype");
  if (d->offset_mode != HR2_OFFSET_ROW && d->offset_mode != HR2_OFFSET_SPECIES)
    return set_error(HR2_E_INVALID_ARG, "offset_mode must be 0 (per row) or 1 (per species)");

  const int S = d->n_species, nT = d->n_T, nP = d->n_p, nc = d->n_cia;
  const int64_t n_nu = d->n_nu, pitch = (n_nu + 63) / 64 * 64;
  // rows are addressed by 32-bit byte offsets inside one species block (and
  // inside one CIA pair block), in the storage type
  const double elem = d->dtype == HR2_TABLE_F64 ? 8.0 : (d->dtype == HR2_TABLE_F32 ? 4.0 : 2.0);
  const double cia_elem = d->dtype == HR2_TABLE_F64 ? 8.0 : 4.0;
  if ((double)nT * nP * pitch * elem >= 4294967296.0)
    return set_error(HR2_E_OUT_OF_RANGE, "one species block of the table must stay below 4 GiB");
  // the column kernel reads both CIA pairs through one buffer resource
  if ((double)nc * nT * pitch * cia_elem >= 4294967296.0)
    return set_error(HR2_E_OUT_OF_RANGE, "the CIA pair blocks together must stay below 4 GiB");
  HIP_TRY(hipSetDevice(ctx->device));
  auto *t = new hr2_tables();
  t->ctx = ctx;
  t->T_axis.assign(d->T_K, d->T_K + nT);
  t->lp_axis.assign(d->log10_p_bar, d->log10_p_bar + nP);
  t->mass.assign(d->molar_mass, d->molar_mass + S);
  t->off.assign((size_t)S * nT * nP, 0.0);
  t->off_cia.assign((size_t)std::max(nc, 1) * nT, 0.0);
  const bool f64 = d->dtype == HR2_TABLE_F64;
  const int64_t rows = (int64_t)S * nT * nP;
  hr2_status st = HR2_OK;
  std::vector<double> sp_off;
  const bool per_species = d->offset_mode == HR2_OFFSET_SPECIES && !f64;
  if (per_species && !species_offsets(d->log10_sigma, S, (int64_t)nT * nP, n_nu, sp_off))
    st = set_error(HR2_E_INVALID_ARG, "table holds a non-finite value");
  const double *fixed = per_species ? sp_off.data() : nullptr;
  if (st == HR2_OK) {
    switch (d->dtype) {
      case HR2_TABLE_F64:
        st = upload_table<double>(d->log10_sigma, rows, n_nu, pitch, false, &t->d_tab,
                                  t->off.data(), &t->bytes);
        break;
      case HR2_TABLE_F16:
        st = upload_table<_Float16>(d->log10_sigma, rows, n_nu, pitch, true, &t->d_tab,
                                    t->off.data(), &t->bytes, fixed);
        break;
      case HR2_TABLE_BF16:
        st = upload_table<uint16_t>(d->log10_sigma, rows, n_nu, pitch, true, &t->d_tab,
                                    t->off.data(), &t->bytes, fixed);
        break;
      default:
        st = upload_table<float>(d->log10_sigma, rows, n_nu, pitch, true, &t->d_tab,
                                 t->off.data(), &t->bytes, fixed);
    }
  }
  if (st == HR2_OK && nc > 0) {
    if (f64)
      st = upload_table<double>(d->log10_k_cia, (int64_t)nc * nT, n_nu, pitch, false, &t->d_cia,
                                t->off_cia.data(), &t->bytes);
    else
      st = upload_table<float>(d->log10_k_cia, (int64_t)nc * nT, n_nu, pitch, true, &t->d_cia,
                               t->off_cia.data(), &t->bytes);
  }
  if (st == HR2_OK) {
    std::vector<double> meta;
    meta.insert(meta.end(), t->T_axis.begin(), t->T_axis.end());
    meta.insert(meta.end(), t->lp_axis.begin(), t->lp_axis.end());
    meta.insert(meta.end(), t->off.begin(), t->off.end());
    meta.insert(meta.end(), t->off_cia.begin(), t->off_cia.end());
    meta.insert(meta.end(), t->mass.begin(), t->mass.end());
    if (hipMalloc(&t->d_meta, meta.size() * sizeof(double)) != hipSuccess) {
      t->d_meta = nullptr;
      (void)hipGetLastError();
      st = set_error(HR2_E_NO_MEMORY, "meta allocation failed");
    } else {
      hipError_t e = hipMemcpy(t->d_meta, meta.data(), meta.size() * sizeof(double),
                               hipMemcpyHostToDevice);
      if (e != hipSuccess) st = hip_error(e, "meta upload");
      t->bytes += meta.size() * sizeof(double);
    }
  }
  if (st != HR2_OK) {
    hr2_tables_destroy(t);
    return st;
  }
  TableView &v = t->view;
  v.tab = t->d_tab;
  v.cia = t->d_cia;
  v.T_axis = t->d_meta;
  v.lp_axis = v.T_axis + nT;
  v.off = v.lp_axis + nP;
  v.off_cia = v.off + (size_t)S * nT * nP;
  v.mass = v.off_cia + (size_t)std::max(nc, 1) * nT;
  v.S = S;
  v.nT = nT;
  v.nP = nP;
  v.n_cia = nc;
  v.n_nu = n_nu;
  v.pitch = pitch;
  v.nu0 = d->nu0_cm;
  v.dnu = d->dnu_cm;
  v.he_ratio = d->he_h2_ratio;
  v.dtype = d->dtype;
  v.tab_elem = d->dtype == HR2_TABLE_F64 ? 8 : (d->dtype == HR2_TABLE_F32 ? 4 : 2);
  v.cia_elem = f64 ? 8 : 4;
  *out = t;
  return HR2_OK;
}

extern "C" void hr2_tables_destroy(hr2_tables *t) {
  if (t == nullptr) return;
  (void)hipSetDevice(t->ctx->device);
  (void)hipDeviceSynchronize();
  if (t->d_tab) (void)hipFree(t->d_tab);
  if (t->d_cia) (void)hipFree(t->d_cia);
  if (t->d_meta) (void)hipFree(t->d_meta);
  delete t;
}

// ------------------------------------------------------------- validation
namespace hr2 {

hr2_status check_window(const hr2_tables *t, const hr2_window &w) {
  if (w.nu_count < 1 || w.nu_stride < 1 || w.nu_begin < 0)
    return set_error(HR2_E_OUT_OF_RANGE, "window needs begin >= 0, count >= 1, stride >= 1");
  if (w.nu_begin + (w.nu_count - 1) * w.nu_stride >= t->view.n_nu)
    return set_error(HR2_E_OUT_OF_RANGE, "window leaves the table");
  return HR2_OK;
}

hr2_status check_column(const hr2_tables *t, const hr2_column &c, int want_levels) {
  if (c.n_levels < 2 || c.n_levels > HR2_MAX_LEVELS)
    return set_error(HR2_E_INVALID_ARG, "n_levels must be in [2, 1024]");
  if (want_levels > 0 && c.n_levels != want_levels)
    return set_error(HR2_E_INVALID_ARG, "all columns of a batch must share n_levels");
  if (!c.p_bar || !c.T_K || !c.x) return set_error(HR2_E_INVALID_ARG, "NULL column array");
  for (int l = 0; l < c.n_levels; ++l) {
    if (!(c.p_bar[l] > 0) || !std::isfinite(c.p_bar[l]))
      return set_error(HR2_E_INVALID_ARG, "pressures must be positive and finite");
    if (!(c.T_K[l] > 0) || !std::isfinite(c.T_K[l]))
      return set_error(HR2_E_INVALID_ARG, "temperatures must be positive and finite");
    if (l > 0 && !(c.p_bar[l] < c.p_bar[l - 1]))
      return set_error(HR2_E_INVALID_ARG, "pressures must decrease upward");
  }
  double xs = 0;
  for (int s = 0; s < t->view.S; ++s) {
    if (!(c.x[s] >= 0) || !std::isfinite(c.x[s]))
      return set_error(HR2_E_INVALID_ARG, "mixing ratios must be >= 0 and finite");
    xs += c.x[s];
  }
  if (!(xs < 1.0)) return set_error(HR2_E_INVALID_ARG, "mixing ratios must sum below 1");
  if (!std::isfinite(c.log_g_cgs) || !std::isfinite(c.scale))
    return set_error(HR2_E_INVALID_ARG, "log g and scale must be finite");
  if (!(c.tau_cloud >= 0.0) || !std::isfinite(c.tau_cloud))
    return set_error(HR2_E_INVALID_ARG, "tau_cloud must be finite and >= 0");
  if (c.tau_cloud > 0.0 &&
      (!(c.p_cloud_top_bar > 0.0) || !std::isfinite(c.p_cloud_top_bar) ||
       !(c.cloud_bottom_frac > 1.0) || !std::isfinite(c.cloud_bottom_frac)))
    return set_error(HR2_E_INVALID_ARG, "a cloud needs p_cloud_top_bar > 0 and bottom_frac > 1");
  return HR2_OK;
}

hr2_status check_n_mu(int n_mu) {
  if (n_mu < 1 || n_mu > HR2_MAX_MU) return set_error(HR2_E_OUT_OF_RANGE, "n_mu must be in [1, 8]");
  return HR2_OK;
}

void pack_columns(const hr2_tables *t, int n_sets, const hr2_column *cols, std::vector<double> &buf) {
  const int L = cols[0].n_levels, S = t->view.S;
  buf.resize((size_t)n_sets * (2 * L + S + 5));
  double *p = buf.data(), *T = p + (size_t)n_sets * L, *x = T + (size_t)n_sets * L;
  double *lg = x + (size_t)n_sets * S, *sc = lg + n_sets, *cl = sc + n_sets;
  for (int s = 0; s < n_sets; ++s) {
    std::memcpy(p + (size_t)s * L, cols[s].p_bar, sizeof(double) * L);
    std::memcpy(T + (size_t)s * L, cols[s].T_K, sizeof(double) * L);
    std::memcpy(x + (size_t)s * S, cols[s].x, sizeof(double) * S);
    lg[s] = cols[s].log_g_cgs;
    sc[s] = cols[s].scale;
    cl[3 * s] = cols[s].tau_cloud;
    cl[3 * s + 1] = cols[s].p_cloud_top_bar;
    cl[3 * s + 2] = cols[s].cloud_bottom_frac;
  }
}

ColumnsView columns_view(const void *dev, int n_sets, int L, int S) {
  ColumnsView v;
  const double *p = (const double *)dev;
  v.p = p;
  v.T = p + (size_t)n_sets * L;
  v.x = v.T + (size_t)n_sets * L;
  v.logg = v.x + (size_t)n_sets * S;
  v.scale = v.logg + n_sets;
  v.cloud = v.scale + n_sets;
  v.B = n_sets;
  v.L = L;
  return v;
}

// Layer chunks per 64-point tile.  A launch of W = B * tiles * C waves, each
// sweeping about (L - 1)/C layers plus one shared boundary level, takes at
// least the wave-level steps of one wave (the critical path) and at least
// W * steps / capacity (the resident-wave throughput); pick the C with the
// smaller of the two maxima (small penalty per chunk for the combine).
// Depends on the request and the device only.
// Resident waves of the column kernel variant for (tables, angles, chunks)
// on the current device; they depend on the variant and the device only, so
// they are cached.
int cached_wave_capacity(const TableView &tv, int n_mu, bool from_chi, int c, bool para) {
  static std::mutex mu;
  static std::map<std::tuple<int, int, int, int, int, bool, int, bool>, int> cache;
  int dev = 0;
  (void)hipGetDevice(&dev);
  const int big = (int64_t)tv.S * tv.nT * tv.nP * tv.pitch * tv.tab_elem >= 0xFFFFFFFFll;
  const auto key =
      std::make_tuple(dev, tv.dtype, tv.S, big, column_mu_class(n_mu), from_chi, c, para);
  std::lock_guard<std::mutex> lk(mu);
  auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  const int v = column_wave_capacity(tv, n_mu, from_chi, c, para);
  cache.emplace(key, v);
  return v;
}

int auto_chunks(const TableView &tv, int64_t base_waves, int n_levels, int n_mu,
                bool from_chi, bool para) {
  auto capacity = [&](int c) { return cached_wave_capacity(tv, n_mu, from_chi, c, para); };
  int best = 1;
  double best_cost = 1e300;
  for (int c = 1; c <= 8 && c <= n_levels - 1; ++c) {
    const int64_t cap = std::max(1, capacity(c));
    const double per_wave = (double)((n_levels - 1 + c - 1) / c + (para && c > 1 ? 2 : 1));
    const double through = (double)base_waves * c * per_wave / (double)cap;
    const double cost = std::max(through, per_wave) * (1.0 + 0.02 * c);
    if (cost < best_cost * 0.999) {
      best_cost = cost;
      best = c;
    }
  }
  return best;
}

}  // namespace hr2

// ------------------------------------------------------------ observations
namespace hr2 {

// Host plan of an observation layout: snapped edges, 5 sigma half widths,
// per-bin supports and offsets of the banded weight rows.
hr2_status plan_obs(const hr2_tables *t, const hr2_window &w, double R, int n_bins,
                    const double *edges, ObsPlan &pl) {
  if (edges == nullptr) return set_error(HR2_E_INVALID_ARG, "NULL bin edges");
  hr2_status st = check_window(t, w);
  if (st != HR2_OK) return st;
  if (!(R > 0) || !std::isfinite(R)) return set_error(HR2_E_INVALID_ARG, "R must be positive");
  if (n_bins < 1) return set_error(HR2_E_INVALID_ARG, "n_bins must be >= 1");
  pl.dnu = (double)w.nu_stride * t->view.dnu;
  pl.first = t->view.nu0 + (double)w.nu_begin * t->view.dnu;
  pl.N = w.nu_count;
  pl.R = R;
  pl.n_bins = n_bins;
  pl.idx.assign(n_bins + 1, 0);
  for (int e = 0; e <= n_bins; ++e) {
    if (!std::isfinite(edges[e])) return set_error(HR2_E_INVALID_ARG, "bin edges must be finite");
    const double v = std::floor((edges[e] - pl.first) / pl.dnu + 0.5);
    if (v < 0 || v > (double)(pl.N - 1))
      return set_error(HR2_E_OUT_OF_RANGE, "a bin edge snaps outside the window");
    pl.idx[e] = (int64_t)v;
    if (e > 0 && pl.idx[e] <= pl.idx[e - 1])
      return set_error(HR2_E_INVALID_ARG, "snapped bin edges must be strictly increasing");
  }
  // 5 sigma half widths (the same FP64 test as the definition: the largest k
  // with k dnu <= 5 sigma_i).  The device computes them for every point with
  // the same operations; the host needs them only at the bin edges: 5 sigma
  // grows by less than one grid step per point when R > 5 / (2 sqrt(2 ln 2)),
  // so i - h_i and i + h_i never decrease and each bin's support runs from
  // its first edge's reach to its last edge's.
  pl.i0 = pl.idx[0];
  pl.n_pts = pl.idx[n_bins] - pl.i0 + 1;
  pl.denom = R * 2.0 * std::sqrt(2.0 * std::log(2.0));
  auto half_width = [&](int64_t i) -> int64_t {
    const double sig = (pl.first + (double)i * pl.dnu) / pl.denom;
    const double hv = std::floor(5.0 * sig / pl.dnu);
    int64_t hh = hv < 1e9 ? (int64_t)hv : (int64_t)1e9;
    while ((double)(hh + 1) * pl.dnu <= 5.0 * sig) ++hh;
    while (hh > 0 && (double)hh * pl.dnu > 5.0 * sig) --hh;
    return std::min<int64_t>(hh, pl.N);
  };
  if (!(5.0 * ((pl.first + (double)pl.idx[n_bins] * pl.dnu) / pl.denom) / pl.dnu < 1e9))
    return set_error(HR2_E_OUT_OF_RANGE, "instrument profile too wide");
  const bool monotone = R > 2.2;
  pl.kstart.assign(n_bins, 0);
  pl.mlo.assign(n_bins, 0);
  pl.mlen.assign(n_bins, 0);
  pl.nnz = 0;
  for (int j = 0; j < n_bins; ++j) {
    int64_t lo, hi;
    if (monotone) {
      lo = std::max<int64_t>(0, pl.idx[j] - half_width(pl.idx[j]));
      hi = std::min<int64_t>(pl.N - 1, pl.idx[j + 1] + half_width(pl.idx[j + 1]));
    } else {
      lo = INT64_MAX;
      hi = INT64_MIN;
      for (int64_t i = pl.idx[j]; i <= pl.idx[j + 1]; ++i) {
        const int64_t h = half_width(i);
        lo = std::min(lo, std::max<int64_t>(0, i - h));
        hi = std::max(hi, std::min<int64_t>(pl.N - 1, i + h));
      }
    }
    pl.kstart[j] = pl.nnz;
    pl.mlo[j] = (int32_t)lo;
    pl.mlen[j] = (int32_t)(hi - lo + 1);
    pl.nnz += hi - lo + 1;
  }
  return HR2_OK;
}

}  // namespace hr2

extern "C" hr2_status hr2_obs_create(hr2_ctx *ctx, const hr2_tables *t, hr2_window w, double R,
                                     int n_bins, const double *edges, hr2_obs **out) {
  if (ctx == nullptr || t == nullptr || out == nullptr || edges == nullptr)
    return set_error(HR2_E_INVALID_ARG, "NULL argument");
  *out = nullptr;
  ObsPlan pl;
  hr2_status st = plan_obs(t, w, R, n_bins, edges, pl);
  if (st != HR2_OK) return st;
  HIP_TRY(hipSetDevice(ctx->device));
  auto *o = new hr2_obs();
  o->ctx = ctx;
  o->tables = t;
  o->window = w;
  o->R = R;
  o->n_bins = n_bins;
  o->fp64 = t->view.dtype == HR2_TABLE_F64;
  o->nnz = pl.nnz;
  o->edge_idx = pl.idx;
  const size_t rs = o->fp64 ? sizeof(double) : sizeof(float);
  const int64_t nnz = pl.nnz, n_pts = pl.n_pts;
  void *d_edges = nullptr, *d_h = nullptr, *d_q = nullptr, *d_z = nullptr;
  hipError_t e = hipMalloc(&o->d_K, std::max<int64_t>(nnz, 1) * rs);
  if (e == hipSuccess) e = hipMalloc((void **)&o->d_kstart, n_bins * sizeof(int64_t));
  if (e == hipSuccess) e = hipMalloc((void **)&o->d_mlo, n_bins * sizeof(int32_t));
  if (e == hipSuccess) e = hipMalloc((void **)&o->d_mlen, n_bins * sizeof(int32_t));
  if (e == hipSuccess) e = hipMalloc(&d_edges, (n_bins + 1) * sizeof(int64_t));
  if (e == hipSuccess) e = hipMalloc(&d_h, n_pts * sizeof(int32_t));
  if (e == hipSuccess) e = hipMalloc(&d_q, n_pts * rs);
  if (e == hipSuccess) e = hipMalloc(&d_z, n_pts * rs);
  hipStream_t s = ctx->internal;
  if (e == hipSuccess)
    e = hipMemcpyAsync(o->d_kstart, pl.kstart.data(), n_bins * sizeof(int64_t),
                       hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(o->d_mlo, pl.mlo.data(), n_bins * sizeof(int32_t), hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(o->d_mlen, pl.mlen.data(), n_bins * sizeof(int32_t), hipMemcpyHostToDevice,
                       s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d_edges, pl.idx.data(), (n_bins + 1) * sizeof(int64_t),
                       hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = launch_obs_build(o->fp64, pl.N, pl.first, pl.dnu, pl.denom, n_bins, nnz,
                         (const int64_t *)d_edges, (int32_t *)d_h, pl.i0, n_pts, d_q, d_z,
                         o->d_kstart, o->d_mlo, o->d_K, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (d_edges) (void)hipFree(d_edges);
  if (d_h) (void)hipFree(d_h);
  if (d_q) (void)hipFree(d_q);
  if (d_z) (void)hipFree(d_z);
  if (e != hipSuccess) {
    hr2_obs_destroy(o);
    return hip_error(e, "observation layout build");
  }
  o->bytes = std::max<int64_t>(nnz, 1) * rs + n_bins * (sizeof(int64_t) + 2 * sizeof(int32_t));
  *out = o;
  return HR2_OK;
}

extern "C" void hr2_obs_destroy(hr2_obs *o) {
  if (o == nullptr) return;
  (void)hipSetDevice(o->ctx->device);
  (void)hipDeviceSynchronize();
  if (o->d_K) (void)hipFree(o->d_K);
  if (o->d_kstart) (void)hipFree(o->d_kstart);
  if (o->d_mlo) (void)hipFree(o->d_mlo);
  if (o->d_mlen) (void)hipFree(o->d_mlen);
  if (o->d_D) (void)hipFree(o->d_D);   // d_s2 lives in the same allocation
  delete o;
}

extern "C" int hr2_obs_n_bins(const hr2_obs *o) { return o ? o->n_bins : 0; }

extern "C" hr2_status hr2_obs_set_data(hr2_obs *o, const double *D, const double *sigma) {
  if (!o || !D || !sigma) return set_error(HR2_E_INVALID_ARG, "NULL argument");
  const int nb = o->n_bins;
  std::vector<double> buf(2 * (size_t)nb);
  for (int j = 0; j < nb; ++j) {
    if (!std::isfinite(D[j]) || !std::isfinite(sigma[j]) || !(sigma[j] > 0.0))
      return set_error(HR2_E_INVALID_ARG, "data must be finite and sigma > 0 in every bin");
    buf[j] = D[j];
    buf[nb + j] = sigma[j] * sigma[j];
  }
  hr2_ctx *ctx = o->ctx;
  HIP_TRY(hipSetDevice(ctx->device));
  if (o->d_D == nullptr) {
    void *p = nullptr;
    HIP_TRY(hipMalloc(&p, buf.size() * sizeof(double)));
    o->d_D = (double *)p;
    o->d_s2 = o->d_D + nb;
  }
  // the previous data may still be read by the context's enqueued calls: wait
  // for the last of them (they are ordered through scratch_event), not for
  // the whole device, then copy on the context's own stream
  if (ctx->scratch_used) HIP_TRY(hipEventSynchronize(ctx->scratch_event));
  HIP_TRY(hipMemcpyAsync(o->d_D, buf.data(), buf.size() * sizeof(double), hipMemcpyHostToDevice,
                         ctx->internal));
  HIP_TRY(hipStreamSynchronize(ctx->internal));
  return HR2_OK;
}

// ------------------------------------------------------------ stage calls
namespace hr2 {

size_t real_size(const hr2_tables *t) {
  return t->view.dtype == HR2_TABLE_F64 ? sizeof(double) : sizeof(float);
}
size_t rec_size(const hr2_tables *t) {
  return t->view.dtype == HR2_TABLE_F64 ? sizeof(LevelRecD) : sizeof(LevelRecF);
}

}  // namespace hr2

namespace {

// Stage one host column and build its level records (B = 1).
hr2_status one_column_records(hr2_ctx *ctx, const hr2_tables *t, const hr2_column *col,
                              hipStream_t s) {
  std::vector<double> buf;
  pack_columns(t, 1, col, buf);
  hr2_status st = stage_upload(ctx, ctx->cols, buf.data(), buf.size() * sizeof(double), s);
  if (st != HR2_OK) return st;
  st = ctx->recs.ensure((size_t)col->n_levels * rec_size(t));
  if (st != HR2_OK) return st;
  const ColumnsView cv = columns_view(ctx->cols.ptr, 1, col->n_levels, t->view.S);
  HIP_TRY(launch_levels(t->view, cv, ctx->recs.ptr, nullptr, t->view.dtype == HR2_TABLE_F64, s));
  return HR2_OK;
}

}  // namespace

extern "C" hr2_status hr2_opacity(hr2_ctx *ctx, const hr2_tables *t, const hr2_column *col,
                                  hr2_window w, void *chi, void *stream) {
  if (!ctx || !t || !col || !chi) return set_error(HR2_E_INVALID_ARG, "NULL argument");
  hr2_status st = check_window(t, w);
  if (st == HR2_OK) st = check_column(t, *col, 0);
  if (st != HR2_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  if ((st = ctx_begin(ctx, s)) != HR2_OK) return st;
  if ((st = one_column_records(ctx, t, col, s)) != HR2_OK) return st;
  HIP_TRY(launch_opacity_only(t->view, ctx->recs.ptr, col->n_levels, w.nu_begin, w.nu_count,
                              w.nu_stride, chi, s));
  return ctx_end(ctx, s);
}

extern "C" hr2_status hr2_rt_emission(hr2_ctx *ctx, const hr2_tables *t, const hr2_column *col,
                                      hr2_window w, const void *chi, int n_mu, void *fplus,
                                      void *stream) {
  if (!ctx || !t || !col || !chi || !fplus) return set_error(HR2_E_INVALID_ARG, "NULL argument");
  hr2_status st = check_window(t, w);
  if (st == HR2_OK) st = check_column(t, *col, 0);
  if (st == HR2_OK) st = check_n_mu(n_mu);
  if (st != HR2_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  if ((st = ctx_begin(ctx, s)) != HR2_OK) return st;
  if ((st = one_column_records(ctx, t, col, s)) != HR2_OK) return st;
  const int64_t base_waves = (w.nu_count + 63) / 64;
  const int chunks = ctx->opt_chunks ? std::min(ctx->opt_chunks, std::max(1, col->n_levels - 1))
                                     : auto_chunks(t->view, base_waves, col->n_levels, n_mu,
                                                   true, ctx->opt_source == 2);
  ColSeg seg{};
  seg.wg_begin = 0;
  seg.nu_begin = w.nu_begin;
  seg.nu_count = w.nu_count;
  seg.nu_stride = w.nu_stride;
  seg.rec_offset = 0;
  seg.out_offset = 0;
  seg.out_stride = w.nu_count;
  seg.chi_offset = 0;
  seg.n_sets = 1;
  seg.n_levels = col->n_levels;
  seg.n_mu = n_mu;
  seg.chunks = chunks;
  const int per_wg = column_nu_per_wg(chunks);
  seg.tiles_per_set = (int32_t)((w.nu_count + per_wg - 1) / per_wg);
  HIP_TRY(launch_column(t->view, nullptr, 1, &seg, seg.tiles_per_set, chunks, ctx->recs.ptr, chi,
                        fplus, n_mu, true, ctx->opt_source == 2, false, s));
  return ctx_end(ctx, s);
}

extern "C" hr2_status hr2_convolve_bin(hr2_ctx *ctx, const hr2_obs *o, const void *fplus,
                                       double scale, void *bins, void *stream) {
  if (!ctx || !o || !fplus || !bins) return set_error(HR2_E_INVALID_ARG, "NULL argument");
  if (!std::isfinite(scale)) return set_error(HR2_E_INVALID_ARG, "scale must be finite");
  hipStream_t s = (hipStream_t)stream;
  hr2_status st;
  if ((st = ctx_begin(ctx, s)) != HR2_OK) return st;
  ConvSeg cs{};
  cs.item_begin = 0;
  cs.K = o->d_K;
  cs.kstart = o->d_kstart;
  cs.mlo = o->d_mlo;
  cs.mlen = o->d_mlen;
  cs.in_offset = 0;
  cs.in_stride = o->window.nu_count;
  cs.out_offset = 0;
  cs.scale = nullptr;
  cs.scale_const = scale;
  cs.n_sets = 1;
  cs.n_bins = o->n_bins;
  cs.items_per_wg = conv_items_per_wg(o->nnz, o->n_bins);
  HIP_TRY(launch_convolve_bin(o->fp64, nullptr, 1, &cs,
                              conv_workgroups(o->n_bins, cs.items_per_wg), fplus, bins, s));
  return ctx_end(ctx, s);
}

// ----------------------------------------------------------- forward model
namespace hr2 {

constexpr size_t kMaxTimedCalls = 65536;

// Event slot k of the current timed call (nullptr when not timing): the
// start and end of its level kernel, column kernel (or whole-forward-model
// kernel) and convolution, each taken from the launch itself.
constexpr int kTimedEvents = 6;
static hipEvent_t timing_event(hr2_ctx *ctx, int k) {
  if (ctx->timing_every <= 0 || ctx->tev_used + kTimedEvents > kTimedEvents * kMaxTimedCalls)
    return nullptr;
  const size_t at = ctx->tev_used + k;
  while (ctx->tev.size() <= at) {
    hipEvent_t ev;
    if (hipEventCreate(&ev) != hipSuccess) return nullptr;
    ctx->tev.push_back(ev);
  }
  return ctx->tev[at];
}


// MI355X Infinity Cache (the last-level cache in front of HBM)
constexpr double kLastLevelCacheBytes = 256.0 * 1024 * 1024;

hr2_status run_forward(hr2_ctx *ctx, const hr2_tables *t, const hr2_obs *o, const ColumnsView &cv,
                       int n_mu, void *bins, void *fplus, int *status, hipStream_t s,
                       const LikeArgs *like = nullptr, const ThetaArgs *theta = nullptr) {
  const hr2_window &w = o->window;
  const int B = cv.B, L = cv.L;
  const size_t rec_bytes = (size_t)B * L * rec_size(t);
  const size_t fp_bytes = fplus == nullptr ? (size_t)B * w.nu_count * real_size(t) : 0;
  const size_t term_bytes = like ? (size_t)B * o->n_bins * sizeof(double) : 0;
  if ((rec_bytes > ctx->recs.cap || fp_bytes > ctx->fplus.cap || term_bytes > ctx->terms.cap) &&
      capturing(s))
    return set_error(HR2_E_UNSUPPORTED,
                     "scratch would grow under stream capture: make the same call once first");
  hr2_status st = ctx->recs.ensure(rec_bytes);
  if (st != HR2_OK) return st;
  if (like && (st = ctx->terms.ensure(term_bytes)) != HR2_OK) return st;
  if (fplus == nullptr && (st = ctx->fplus.ensure(fp_bytes)) != HR2_OK) return st;
  FwdScratch scr;
  scr.recs = ctx->recs.ptr;
  scr.fplus = ctx->fplus.ptr;
  scr.terms = (double *)ctx->terms.ptr;
  return launch_forward(ctx, t, o, cv, n_mu, bins, fplus, status, s, scr, like, theta);
}

hr2_status launch_forward(hr2_ctx *ctx, const hr2_tables *t, const hr2_obs *o,
                          const ColumnsView &cv, int n_mu, void *bins, void *fplus, int *status,
                          hipStream_t s, const FwdScratch &scr, const LikeArgs *like,
                          const ThetaArgs *theta) {
  const hr2_window &w = o->window;
  const int B = cv.B, L = cv.L;
  if (fplus == nullptr) fplus = scr.fplus;
  const bool this_call = scr.timing && ctx->timing_every > 0 && !capturing(s) &&
                         (ctx->timing_calls++ % ctx->timing_every) == 0;
  hipEvent_t ev[kTimedEvents] = {};
  bool timed = this_call;
  if (this_call)
    for (int k = 0; k < kTimedEvents; ++k) timed = (ev[k] = timing_event(ctx, k)) && timed;
  const int tk = ctx->timing_kernels;
  auto tev = [&](int k) { return timed && ((tk >> (k / 2)) & 1) ? ev[k] : nullptr; };
  const int64_t base_waves = (int64_t)B * ((w.nu_count + 63) / 64);
  // Small windows in a batch that fills the device on its own: the whole
  // forward model in one launch, one workgroup per set (records and F+ in
  // LDS).  Columns and bins only; the same arithmetic as the three kernels.
  if (theta == nullptr && like == nullptr && ctx->opt_chunks == 0 && ctx->opt_source == 1 &&
      set_forward_fits(t->view, L, w.nu_count) && conv_items_per_wg(o->nnz, o->n_bins) == 4 &&
      base_waves >= cached_wave_capacity(t->view, n_mu, false, 1, false)) {
    SetFwdArgs a{};
    a.nu_begin = w.nu_begin;
    a.nu_count = w.nu_count;
    a.nu_stride = w.nu_stride;
    a.n_mu = n_mu;
    a.n_bins = o->n_bins;
    a.fplus = (float *)fplus;
    a.bins = (float *)bins;
    a.status = status;
    a.K = (const float *)o->d_K;
    a.kstart = o->d_kstart;
    a.mlo = o->d_mlo;
    a.mlen = o->d_mlen;
    HIP_TRY(launch_set_forward(t->view, cv, a, n_mu, ctx->opt_nu_per_lane, s, tev(2), tev(3)));
    if (timed) {
      ctx->tmask.push_back((uint8_t)(tk & 2));   // one kernel: the column interval
      ctx->tev_used += kTimedEvents;
    }
    return HR2_OK;
  }
  HIP_TRY(launch_levels(t->view, cv, scr.recs, status, t->view.dtype == HR2_TABLE_F64, s,
                        theta, tev(0), tev(1)));
  const int chunks = ctx->opt_chunks ? std::min(ctx->opt_chunks, std::max(1, L - 1))
                                     : auto_chunks(t->view, base_waves, L, n_mu, false,
                                                   ctx->opt_source == 2);
  const int per_wg = column_nu_per_wg(chunks);
  ColSeg seg{};
  seg.wg_begin = 0;
  seg.nu_begin = w.nu_begin;
  seg.nu_count = w.nu_count;
  seg.nu_stride = w.nu_stride;
  seg.rec_offset = 0;
  seg.out_offset = 0;
  seg.out_stride = w.nu_count;
  seg.chi_offset = 0;
  seg.n_sets = B;
  seg.n_levels = L;
  seg.n_mu = n_mu;
  seg.chunks = chunks;
  seg.tiles_per_set = (int32_t)((w.nu_count + per_wg - 1) / per_wg);
  int64_t total_wgs = (int64_t)B * seg.tiles_per_set;
  if (total_wgs > 0x7fffffff) return set_error(HR2_E_OUT_OF_RANGE, "launch too large");
  // One set whose tiles spill past one round of resident workgroups: on each
  // XCD the first round's workgroups take two tiles of `chunks` layer chunks
  // each, and the tiles left over get twice the chunks (half the levels per
  // wave), so the last round ends sooner.  Only where the twice-as-large
  // workgroups keep as many resident waves (C2: 8 waves per SIMD either way;
  // column kernel 77 vs 81 us with FP32 rows, 70.5 vs 81 us with FP16/BF16).
  int launch_chunks = chunks;
  if (B == 1 && ctx->opt_tile_pairs == 0 && 2 * chunks <= 8) {
    const bool para = ctx->opt_source == 2;
    const int64_t cap1 = cached_wave_capacity(t->view, n_mu, false, chunks, para);
    const int64_t cap2 = cached_wave_capacity(t->view, n_mu, false, 2 * chunks, para);
    const int64_t per_xcd = cap2 / (2 * chunks) / 8;
    if (cap2 >= cap1 && per_xcd >= 1 && seg.tiles_per_set / 8 > 2 * per_xcd) {
      seg.wg_multi = (int32_t)per_xcd;
      seg.tiles_per_wg = 2;
      seg.chunks = launch_chunks = 2 * chunks;
      total_wgs = seg.tiles_per_set - 8 * per_xcd;
    }
  }
  // A single set reads each of its rows once.  When they cannot stay in the
  // last-level cache until the next call anyway (estimated at one new row per
  // level and species, against the 256 MB Infinity Cache), they are loaded
  // non-temporal, which keeps the small working set of the level and
  // convolution kernels cached (C2, FP32 rows: +3.5 % per step).  Smaller row
  // sets (C2 with 2-byte rows: 182 MB) keep the default policy, under which a
  // following call over similar cells finds them cached.
  const double row_bytes_est = (double)t->view.S *
                               (double)std::min<int64_t>((int64_t)t->view.nT * t->view.nP, L) *
                               (double)w.nu_count * (double)t->view.tab_elem;
  const bool stream_rows =
      B == 1 && (ctx->opt_row_policy == 1 ||
                 (ctx->opt_row_policy == 0 && row_bytes_est > kLastLevelCacheBytes));
  HIP_TRY(launch_column(t->view, nullptr, 1, &seg, total_wgs, launch_chunks, scr.recs, nullptr,
                        fplus, n_mu, false, ctx->opt_source == 2, stream_rows, s, tev(2),
                        tev(3)));
  ConvSeg cs{};
  cs.item_begin = 0;
  cs.K = o->d_K;
  cs.kstart = o->d_kstart;
  cs.mlo = o->d_mlo;
  cs.mlen = o->d_mlen;
  cs.in_offset = 0;
  cs.in_stride = w.nu_count;
  cs.out_offset = 0;
  cs.scale = cv.scale;
  cs.scale_const = 0.0;
  cs.n_sets = B;
  cs.n_bins = o->n_bins;
  if (like) {
    cs.D = o->d_D;
    cs.s2 = o->d_s2;
    cs.log10_eps = like->log10_eps;
    cs.terms = scr.terms;
  }
  cs.items_per_wg = conv_items_per_wg(o->nnz, o->n_bins);
  HIP_TRY(launch_convolve_bin(o->fp64, nullptr, 1, &cs,
                              conv_workgroups((int64_t)B * o->n_bins, cs.items_per_wg), fplus,
                              bins, s, tev(4), tev(5)));
  if (like) HIP_TRY(launch_lnl_reduce(cs.terms, B, o->n_bins, like->lnl, s));
  if (timed) {
    ctx->tmask.push_back((uint8_t)tk);   // levels, column, convolution as asked
    ctx->tev_used += kTimedEvents;
  }
  return HR2_OK;
}

}  // namespace hr2

extern "C" hr2_status hr2_forward_batch(hr2_ctx *ctx, const hr2_tables *t, const hr2_obs *o,
                                        int n_sets, const hr2_column *cols, int n_mu, void *bins,
                                        void *fplus, void *stream) {
  if (!ctx || !t || !o || !cols || !bins) return set_error(HR2_E_INVALID_ARG, "NULL argument");
  if (o->tables != t) return set_error(HR2_E_INVALID_ARG, "layout was made for other tables");
  if (n_sets < 1) return set_error(HR2_E_INVALID_ARG, "n_sets must be >= 1");
  hr2_status st = check_n_mu(n_mu);
  if (st != HR2_OK) return st;
  for (int i = 0; i < n_sets; ++i)
    if ((st = check_column(t, cols[i], cols[0].n_levels)) != HR2_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  if ((st = ctx_begin(ctx, s)) != HR2_OK) return st;
  std::vector<double> buf;
  pack_columns(t, n_sets, cols, buf);
  if ((st = stage_upload(ctx, ctx->cols, buf.data(), buf.size() * sizeof(double), s)) != HR2_OK)
    return st;
  const ColumnsView cv = columns_view(ctx->cols.ptr, n_sets, cols[0].n_levels, t->view.S);
  if ((st = run_forward(ctx, t, o, cv, n_mu, bins, fplus, nullptr, s)) != HR2_OK) return st;
  return ctx_end(ctx, s);
}

extern "C" hr2_status hr2_forward_batch_dev(hr2_ctx *ctx, const hr2_tables *t, const hr2_obs *o,
                                            int n_sets, int n_levels, const double *p_dev,
                                            const double *T_dev, const double *x_dev,
                                            const double *logg_dev, const double *scale_dev,
                                            const double *cloud_dev, int n_mu, void *bins,
                                            void *fplus, int *status_dev, void *stream) {
  if (!ctx || !t || !o || !p_dev || !T_dev || !x_dev || !logg_dev || !scale_dev || !bins)
    return set_error(HR2_E_INVALID_ARG, "NULL argument");
  if (o->tables != t) return set_error(HR2_E_INVALID_ARG, "layout was made for other tables");
  if (n_sets < 1) return set_error(HR2_E_INVALID_ARG, "n_sets must be >= 1");
  if (n_levels < 2 || n_levels > HR2_MAX_LEVELS)
    return set_error(HR2_E_INVALID_ARG, "n_levels must be in [2, 1024]");
  hr2_status st = check_n_mu(n_mu);
  if (st != HR2_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  if ((st = ctx_begin(ctx, s)) != HR2_OK) return st;
  ColumnsView cv;
  cv.p = p_dev;
  cv.T = T_dev;
  cv.x = x_dev;
  cv.logg = logg_dev;
  cv.scale = scale_dev;
  cv.cloud = cloud_dev;
  cv.B = n_sets;
  cv.L = n_levels;
  if ((st = run_forward(ctx, t, o, cv, n_mu, bins, fplus, status_dev, s)) != HR2_OK) return st;
  return ctx_end(ctx, s);
}

namespace {

hr2_status check_like(const hr2_tables *t, const hr2_obs *o, int n_sets, int n_mu) {
  if (o->tables != t) return set_error(HR2_E_INVALID_ARG, "layout was made for other tables");
  if (o->d_D == nullptr)
    return set_error(HR2_E_INVALID_ARG, "no data on this layout: call hr2_obs_set_data first");
  if (n_sets < 1) return set_error(HR2_E_INVALID_ARG, "n_sets must be >= 1");
  return check_n_mu(n_mu);
}

}  // namespace

extern "C" hr2_status hr2_loglike_batch(hr2_ctx *ctx, const hr2_tables *t, const hr2_obs *o,
                                        int n_sets, const hr2_column *cols, int n_mu,
                                        const double *log10_eps, double *lnl, void *bins,
                                        void *stream) {
  if (!ctx || !t || !o || !cols || !lnl) return set_error(HR2_E_INVALID_ARG, "NULL argument");
  hr2_status st = check_like(t, o, n_sets, n_mu);
  if (st != HR2_OK) return st;
  for (int i = 0; i < n_sets; ++i)
    if ((st = check_column(t, cols[i], cols[0].n_levels)) != HR2_OK) return st;
  if (log10_eps)
    for (int i = 0; i < n_sets; ++i)
      if (!std::isfinite(log10_eps[i]))
        return set_error(HR2_E_INVALID_ARG, "log10_eps must be finite");
  hipStream_t s = (hipStream_t)stream;
  if ((st = ctx_begin(ctx, s)) != HR2_OK) return st;
  std::vector<double> buf;
  pack_columns(t, n_sets, cols, buf);
  const size_t n_col = buf.size();
  if (log10_eps) buf.insert(buf.end(), log10_eps, log10_eps + n_sets);
  if ((st = stage_upload(ctx, ctx->cols, buf.data(), buf.size() * sizeof(double), s)) != HR2_OK)
    return st;
  const ColumnsView cv = columns_view(ctx->cols.ptr, n_sets, cols[0].n_levels, t->view.S);
  LikeArgs like{log10_eps ? (const double *)ctx->cols.ptr + n_col : nullptr, lnl};
  if ((st = run_forward(ctx, t, o, cv, n_mu, bins, nullptr, nullptr, s, &like)) != HR2_OK)
    return st;
  return ctx_end(ctx, s);
}

extern "C" hr2_status hr2_loglike_batch_dev(hr2_ctx *ctx, const hr2_tables *t, const hr2_obs *o,
                                            int n_sets, int n_levels, const double *p_dev,
                                            const double *T_dev, const double *x_dev,
                                            const double *logg_dev, const double *scale_dev,
                                            const double *cloud_dev, const double *log10_eps_dev,
                                            int n_mu, double *lnl, void *bins, int *status_dev,
                                            void *stream) {
  if (!ctx || !t || !o || !p_dev || !T_dev || !x_dev || !logg_dev || !scale_dev || !lnl)
    return set_error(HR2_E_INVALID_ARG, "NULL argument");
  hr2_status st = check_like(t, o, n_sets, n_mu);
  if (st != HR2_OK) return st;
  if (n_levels < 2 || n_levels > HR2_MAX_LEVELS)
    return set_error(HR2_E_INVALID_ARG, "n_levels must be in [2, 1024]");
  hipStream_t s = (hipStream_t)stream;
  if ((st = ctx_begin(ctx, s)) != HR2_OK) return st;
  ColumnsView cv;
  cv.p = p_dev;
  cv.T = T_dev;
  cv.x = x_dev;
  cv.logg = logg_dev;
  cv.scale = scale_dev;
  cv.cloud = cloud_dev;
  cv.B = n_sets;
  cv.L = n_levels;
  LikeArgs like{log10_eps_dev, lnl};
  if ((st = run_forward(ctx, t, o, cv, n_mu, bins, nullptr, status_dev, s, &like)) != HR2_OK)
    return st;
  return ctx_end(ctx, s);
}

// ------------------------------------------------------ parameter vectors
namespace {

// Gauss-Lobatto points of [0, 1] for n = q + 1 points: the ends and the
// roots of P'_q, found by Newton steps with P''_q from Legendre's equation
// (1 - x^2) P'' = 2 x P' - q (q + 1) P, started at the Chebyshev-Lobatto
// points.
void gauss_lobatto_01(int q, double *x01) {
  x01[0] = 0.0;
  x01[q] = 1.0;
  const double pi = 3.14159265358979323846;
  for (int i = 1; i < q; ++i) {
    double z = -std::cos(pi * i / q);
    for (int it = 0; it < 100; ++it) {
      double pa = 1.0, pb = 0.0, da = 0.0, db = 0.0;   // P_k, P_{k-1} and derivatives
      for (int k = 1; k <= q; ++k) {
        const double pc = pb, dc = db;
        pb = pa;
        db = da;
        pa = ((2.0 * k - 1.0) * z * pb - (k - 1.0) * pc) / k;
        da = ((2.0 * k - 1.0) * (pb + z * db) - (k - 1.0) * dc) / k;
      }
      const double d2 = (2.0 * z * da - q * (q + 1.0) * pa) / (1.0 - z * z);
      const double step = da / d2;
      z -= step;
      if (std::fabs(step) <= 1e-16) break;
    }
    x01[i] = 0.5 * (z + 1.0);
  }
}

}  // namespace

extern "C" hr2_status hr2_params_create(hr2_ctx *ctx, const hr2_tables *t,
                                        const hr2_param_layout *lay, hr2_params **out) {
  if (!ctx || !t || !lay || !out) return set_error(HR2_E_INVALID_ARG, "NULL argument");
  *out = nullptr;
  const int S = t->view.S;
  if (lay->n_elements < 1 || lay->order < 1 || lay->order > HR2_MAX_ORDER ||
      (int64_t)lay->n_elements * lay->order + 1 > HR2_MAX_TNODES)
    return set_error(HR2_E_INVALID_ARG, "need K_e >= 1, 1 <= q <= 8 and K_e q + 1 <= 128");
  if (lay->n_levels < 2 || lay->n_levels > HR2_MAX_LEVELS)
    return set_error(HR2_E_INVALID_ARG, "n_levels must be in [2, 1024]");
  if (!std::isfinite(lay->log10_p_bottom) || !std::isfinite(lay->log10_p_top) ||
      !(lay->log10_p_top < lay->log10_p_bottom))
    return set_error(HR2_E_INVALID_ARG, "need finite log10_p_top < log10_p_bottom");
  if (!(lay->radius_cm > 0.0) || !std::isfinite(lay->radius_cm))
    return set_error(HR2_E_INVALID_ARG, "radius_cm must be finite and > 0");
  if (lay->n_free < 0 || lay->n_free > HR2_MAX_SPECIES || (lay->with_eps != 0 && lay->with_eps != 1) ||
      (lay->with_cloud != 0 && lay->with_cloud != 1))
    return set_error(HR2_E_INVALID_ARG,
                     "n_free must be in [0, 12], with_cloud and with_eps 0 or 1");
  if (S > 0 && (!lay->species_src || !lay->species_factor))
    return set_error(HR2_E_INVALID_ARG, "NULL species map");
  auto *pp = new hr2_params();
  pp->ctx = ctx;
  pp->tables = t;
  ParamView &v = pp->view;
  for (int s = 0; s < S; ++s) {
    const int src = lay->species_src[s];
    const double f = lay->species_factor[s];
    if (src < -1 || src >= lay->n_free || !std::isfinite(f) || f < 0.0) {
      delete pp;
      return set_error(HR2_E_INVALID_ARG,
                       "species_src must be in [-1, n_free) and species_factor finite, >= 0");
    }
    v.src[s] = src;
    v.fac[s] = f;
  }
  const int q = lay->order;
  gauss_lobatto_01(q, v.nodes);
  for (int i = 0; i <= q; ++i) {
    double den = 1.0;
    for (int j = 0; j <= q; ++j)
      if (j != i) den *= v.nodes[i] - v.nodes[j];
    v.inv_den[i] = 1.0 / den;
  }
  v.lp_bottom = lay->log10_p_bottom;
  v.lp_top = lay->log10_p_top;
  v.radius_cm = lay->radius_cm;
  v.K = lay->n_elements;
  v.q = q;
  v.L = lay->n_levels;
  v.S = S;
  v.n_free = lay->n_free;
  v.with_cloud = lay->with_cloud;
  v.with_eps = lay->with_eps;
  v.n_theta = 3 + v.K * q + 1 + v.n_free + 3 * v.with_cloud + v.with_eps;
  *out = pp;
  return HR2_OK;
}

extern "C" void hr2_params_destroy(hr2_params *p) { delete p; }

extern "C" int hr2_params_n_theta(const hr2_params *p) { return p ? p->view.n_theta : 0; }

extern "C" hr2_status hr2_params_unpack_dev(hr2_ctx *ctx, const hr2_params *pp, int n_sets,
                                            const double *theta, double *p_dev, double *T_dev,
                                            double *x_dev, double *logg_dev, double *scale_dev,
                                            double *cloud_dev, double *eps_dev, void *stream) {
  if (!ctx || !pp || !theta || !p_dev || !T_dev || !logg_dev || !scale_dev ||
      (!x_dev && pp->view.S > 0))
    return set_error(HR2_E_INVALID_ARG, "NULL argument");
  if (n_sets < 1) return set_error(HR2_E_INVALID_ARG, "n_sets must be >= 1");
  hipStream_t s = (hipStream_t)stream;
  hr2_status st;
  if ((st = ctx_begin(ctx, s)) != HR2_OK) return st;
  HIP_TRY(launch_unpack(pp->view, n_sets, theta, p_dev, T_dev, x_dev, logg_dev, scale_dev,
                        cloud_dev, eps_dev, s));
  return ctx_end(ctx, s);
}

extern "C" hr2_status hr2_forward_params_dev(hr2_ctx *ctx, const hr2_tables *t, const hr2_obs *o,
                                             const hr2_params *pp, int n_sets,
                                             const double *theta, int n_mu, void *bins,
                                             double *lnl, int *status_dev, void *stream) {
  if (!ctx || !t || !o || !pp || !theta || (!bins && !lnl))
    return set_error(HR2_E_INVALID_ARG, "NULL argument");
  if (pp->tables != t) return set_error(HR2_E_INVALID_ARG, "parameter layout is for other tables");
  if (o->tables != t) return set_error(HR2_E_INVALID_ARG, "layout was made for other tables");
  if (n_sets < 1) return set_error(HR2_E_INVALID_ARG, "n_sets must be >= 1");
  hr2_status st = lnl ? check_like(t, o, n_sets, n_mu) : check_n_mu(n_mu);
  if (st != HR2_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  const ParamView &v = pp->view;
  const int B = n_sets, L = v.L, S = v.S;
  const size_t n_dbl = (size_t)B * (2 * (size_t)L + S + 6);   // columns, clouds, eps
  if (n_dbl * sizeof(double) > ctx->unpacked.cap && capturing(s))
    return set_error(HR2_E_UNSUPPORTED,
                     "scratch would grow under stream capture: make the same call once first");
  if ((st = ctx_begin(ctx, s)) != HR2_OK) return st;
  if ((st = ctx->unpacked.ensure(n_dbl * sizeof(double))) != HR2_OK) return st;
  // the level kernel forms the columns from theta and writes each set's
  // scale and eps where the later stages read them
  ColumnsView cv = columns_view(ctx->unpacked.ptr, B, L, S);
  double *cloud = const_cast<double *>(cv.cloud);
  double *eps = cloud + (size_t)3 * B;
  const ThetaArgs ta{v, theta, const_cast<double *>(cv.scale), eps};
  LikeArgs like{v.with_eps ? eps : nullptr, lnl};
  if ((st = run_forward(ctx, t, o, cv, n_mu, bins, nullptr, status_dev, s, lnl ? &like : nullptr,
                        &ta)) != HR2_OK)
    return st;
  return ctx_end(ctx, s);
}

extern "C" hr2_status hr2_ctx_collect_timing(hr2_ctx *ctx, double ms[3], int64_t *n_calls) {
  if (!ctx || !ms || !n_calls) return set_error(HR2_E_INVALID_ARG, "NULL argument");
  ms[0] = ms[1] = ms[2] = 0.0;
  *n_calls = (int64_t)ctx->tmask.size();
  for (size_t c = 0; c < ctx->tmask.size(); ++c) {
    const size_t base = c * kTimedEvents;
    const int mask = ctx->tmask[c];
    for (int k = 0; k < 3; ++k) {
      if (!(mask & (1 << k))) continue;
      HIP_TRY(hipEventSynchronize(ctx->tev[base + 2 * k + 1]));
      float t = 0.0f;
      HIP_TRY(hipEventElapsedTime(&t, ctx->tev[base + 2 * k], ctx->tev[base + 2 * k + 1]));
      ms[k] += t;
    }
  }
  ctx->tev_used = 0;
  ctx->tmask.clear();
  return HR2_OK;
}
