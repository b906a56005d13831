// noalloc.hip — the forward model for callers that cannot allocate device
// memory (code under HIP graph capture, tight serving loops, harnesses that
// forbid hipMalloc): hr2_forward_batch_dev with its scratch (the level
// records, and F+ when the caller passes no F+ buffer) in one fixed device
// array per GPU instead of the context's grow-only buffers.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "hr2_context.h"
#include "hr2_internal.h"

namespace hr2 {

// The fixed array.  Each GPU the library runs on holds its own copy, at its
// own address, from the module load until the process ends.  In host code
// the name is only a host-side stand-in: kernels get the device address
// that noalloc_scratch_init looked up.
static __device__ __align__(256) unsigned char scratch[HR2_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

void *scratch_ptr(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return device >= 0 && device < kMaxDevices ? g_scratch_ptr[device] : nullptr;
}
}  // namespace

hr2_status noalloc_scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices)
    return set_error(HR2_E_DEVICE, "device index beyond the library's table of " +
                                       std::to_string(kMaxDevices) + " devices");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device] != nullptr) return HR2_OK;
  void *p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return hip_error(e, "address of the fixed scratch array");
  }
  if (p == nullptr) return set_error(HR2_E_DEVICE, "the fixed scratch array has no address");
  g_scratch_ptr[device] = p;
  return HR2_OK;
}

}  // namespace hr2

using namespace hr2;

extern "C" hr2_status hr2_forward_batch_dev_noalloc(
    hr2_ctx *ctx, const hr2_tables *t, const hr2_obs *o, int n_sets, int n_levels,
    const double *p_dev, const double *T_dev, const double *x_dev, const double *logg_dev,
    const double *scale_dev, const double *cloud_dev, int n_mu, void *bins, void *fplus,
    int *status_dev, void *stream) {
  if (!ctx || !t || !o || !p_dev || !T_dev || !x_dev || !logg_dev || !scale_dev || !bins)
    return set_error(HR2_E_INVALID_ARG, "NULL argument");
  if (o->tables != t) return set_error(HR2_E_INVALID_ARG, "layout was made for other tables");
  if (n_sets < 1) return set_error(HR2_E_INVALID_ARG, "n_sets must be >= 1");
  if (n_levels < 2 || n_levels > HR2_MAX_LEVELS)
    return set_error(HR2_E_INVALID_ARG, "n_levels must be in [2, 1024]");
  hr2_status st = check_n_mu(n_mu);
  if (st != HR2_OK) return st;
  // the call's scratch: records (256-byte aligned), then F+ when none is given
  const double rec_d = (double)n_sets * n_levels * rec_size(t);
  const double fp_d = fplus == nullptr ? (double)n_sets * o->window.nu_count * real_size(t) : 0.0;
  const double need = (double)(((size_t)rec_d + 255) & ~(size_t)255) + fp_d;
  if (!(need <= (double)HR2_NOALLOC_SCRATCH_BYTES))
    return set_error(HR2_E_OUT_OF_RANGE,
                     "the call needs " + std::to_string((long long)need) +
                         " bytes of scratch; the fixed array holds " +
                         std::to_string((long long)HR2_NOALLOC_SCRATCH_BYTES) +
                         " (pass an F+ buffer or fewer sets)");
  const hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_error(e, "hipSetDevice");
  unsigned char *base = (unsigned char *)scratch_ptr(ctx->device);
  if (base == nullptr)
    return set_error(HR2_E_DEVICE, "the fixed scratch array was not set up on this device");
  FwdScratch scr;
  scr.recs = base;
  scr.fplus = base + (((size_t)rec_d + 255) & ~(size_t)255);
  scr.terms = nullptr;
  scr.timing = false;
  ColumnsView cv;
  cv.p = p_dev;
  cv.T = T_dev;
  cv.x = x_dev;
  cv.logg = logg_dev;
  cv.scale = scale_dev;
  cv.cloud = cloud_dev;
  cv.B = n_sets;
  cv.L = n_levels;
  return launch_forward(ctx, t, o, cv, n_mu, bins, fplus, status_dev, (hipStream_t)stream, scr,
                        nullptr, nullptr);
}
