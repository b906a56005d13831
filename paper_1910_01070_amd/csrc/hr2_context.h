// hr2_context.h — the context object and host helpers shared by api.cpp and
// serve.cpp.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "hr2_internal.h"

namespace hr2 {

// Grow-only device buffer.  Growing allocates the new buffer first and keeps
// the superseded one in `retired` (enqueued work or a captured graph may
// still read it); free_retired() frees those once the owner knows that
// nothing can read them any more.  Nothing here synchronises the device.
struct DevBuf {
  void *ptr = nullptr;
  size_t cap = 0;
  std::vector<void *> retired;
  hr2_status ensure(size_t bytes);
  void free_retired();
  void release();
};

hr2_status set_error(hr2_status st, const std::string &msg);
hr2_status hip_error(hipError_t e, const char *what);

}  // namespace hr2

struct hr2_ctx {
  int device = 0;
  hipStream_t internal = nullptr;   // layout builds
  hipEvent_t scratch_event = nullptr;
  bool scratch_used = false;
  hipEvent_t pinned_event = nullptr;
  bool pinned_pending = false;
  void *pinned = nullptr;
  size_t pinned_cap = 0;
  int opt_chunks = 0;
  int opt_source = 1;              // 1 linear, 2 parabolic short characteristics
  int opt_row_policy = 0;          // one-set calls: 0 auto, 1 non-temporal, 2 cached
  int opt_tile_pairs = 0;          // one-set calls: 0 auto, 1 off
  int opt_nu_per_lane = 0;         // per-set launches: 0 auto, 1 or 2 wavenumbers per lane
  int timing_every = 0;            // time every n-th forward call (0 = off)
  int timing_kernels = 7;          // of those calls: 1 levels, 2 column, 4 convolution
  int64_t timing_calls = 0;
  std::vector<hipEvent_t> tev;     // 6 events per timed call (start, end of 3 kernels)
  std::vector<uint8_t> tmask;      // per timed call: which of the 3 intervals it has
  size_t tev_used = 0;             // events recorded since the last collection
  bool captured = false;           // a call on this context ran under stream capture: a
                                   // graph may hold its scratch, so superseded scratch
                                   // is kept until hr2_ctx_destroy
  hr2::DevBuf recs, fplus, cols, terms, unpacked;
};

namespace hr2 {

hr2_status ctx_begin(hr2_ctx *ctx, hipStream_t stream);
hr2_status ctx_end(hr2_ctx *ctx, hipStream_t stream);
hr2_status stage_upload(hr2_ctx *ctx, DevBuf &dst, const void *src, size_t bytes,
                        hipStream_t stream);
hr2_status check_window(const hr2_tables *t, const hr2_window &w);
hr2_status check_column(const hr2_tables *t, const hr2_column &c, int want_levels);
hr2_status check_n_mu(int n_mu);
void pack_columns(const hr2_tables *t, int n_sets, const hr2_column *cols,
                  std::vector<double> &buf);
ColumnsView columns_view(const void *dev, int n_sets, int L, int S);
int auto_chunks(const TableView &tv, int64_t base_waves, int n_levels, int n_mu, bool from_chi,
                bool para);
int cached_wave_capacity(const TableView &tv, int n_mu, bool from_chi, int chunks, bool para);

// Likelihood outputs of a forward call (NULL: bins only).
struct LikeArgs {
  const double *log10_eps;   // device [B] or NULL
  double *lnl;               // device [B]
};

// Device scratch of one forward call: level records, F+ (used when the
// caller passes none) and the likelihood's per-bin terms.
struct FwdScratch {
  void *recs = nullptr;
  void *fplus = nullptr;
  double *terms = nullptr;
  bool timing = true;   // the call may record timing events (event creation)
};

// Bytes of one level record for these tables, and of one spectrum element.
size_t rec_size(const hr2_tables *t);
size_t real_size(const hr2_tables *t);

// The launch sequence of the forward model (levels -> column -> convolve/bin
// [-> ln L]) on the given scratch; allocates nothing itself (timing events
// are created only when scr.timing is set).
hr2_status launch_forward(hr2_ctx *ctx, const hr2_tables *t, const hr2_obs *o,
                          const ColumnsView &cv, int n_mu, void *bins, void *fplus, int *status,
                          hipStream_t s, const FwdScratch &scr, const LikeArgs *like,
                          const ThetaArgs *theta);

// The fixed device array of the allocation-free entry point: looks up its
// address on `device` (which must be current) once per device.
hr2_status noalloc_scratch_init(int device);

struct ObsPlan {
  int64_t N = 0, i0 = 0, n_pts = 0, nnz = 0;
  double first = 0, dnu = 0, R = 0;
  int n_bins = 0;
  std::vector<int64_t> idx;      // snapped edges [n_bins + 1]
  double denom = 0;              // R 2 sqrt(2 ln 2): sigma_i = nu_i / denom
  std::vector<int64_t> kstart;   // [n_bins]
  std::vector<int32_t> mlo, mlen;
};
hr2_status plan_obs(const hr2_tables *t, const hr2_window &w, double R, int n_bins,
                    const double *edges, ObsPlan &plan);

}  // namespace hr2
