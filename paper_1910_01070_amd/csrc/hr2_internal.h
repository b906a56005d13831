// hr2_internal.h — structures shared by the host side (api.cpp, serve.cpp)
// and the kernels (kernels.hip) of libhr2.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "hr2.h"

namespace hr2 {

// ---------------------------------------------------------------- level records
// One record per (set, level), written by the level kernel and read with
// scalar loads by the column kernels.  The four "slots" hold the four
// table rows of the bilinear cell (Sect. 2.3 reading: bilinear in
// (T, log10 p)); a slot keeps its row across levels when the next level's
// cell still needs that row, so only rows new to the column are fetched.
// The CIA (linear in T) uses two slots the same way.
constexpr int kMaxSpecies = HR2_MAX_SPECIES;
constexpr int kMaxMu = HR2_MAX_MU;

struct alignas(16) LevelRecF {
  float w[4];            // slot weights (bilinear corner weights)
  uint32_t rowb[4];      // byte offset of each slot's row in a species block: (iT n_p + ip) pitch b
  int32_t mask;          // bit k < 4: species slot k changes here (coming from level l-1);
                         // bit 4 + q: CIA slot q; bits 8 + k, 12 + q: the slot's weight is
                         // nonzero; bits 16 + k, 20 + q: as bits k, 4 + q coming from l+1
  uint32_t cia_rowb[2];  // byte offset of each CIA slot's row (T node) in a pair block
  float cia_w[2];        // CIA slot weights
  float a_cia[2];        // n_H2^2 2^{c}, n_H2 n_He 2^{c'} (c: interpolated row offsets)
  float hdz;             // dz_l / 2 of layer l -> l+1 (0 at the top level)
  float pl_hi, pl_lo;    // c2 log2(e) / T_l as an unevaluated float sum
  float a_s[kMaxSpecies];  // n_s 2^{c_s}
  float dtc;             // gray-cloud optical depth of layer l -> l+1
  float pad;
};
static_assert(sizeof(LevelRecF) == 128, "LevelRecF must be 128 bytes");

struct alignas(16) LevelRecD {
  double w[4];
  uint32_t rowb[4];
  int32_t mask;
  uint32_t cia_rowb[2];
  int32_t pad0;
  double cia_w[2];
  double a_cia[2];
  double hdz;
  double T;               // level temperature (Planck in FP64)
  double a_s[kMaxSpecies];
  double dtc;             // gray-cloud optical depth of layer l -> l+1
  double pad[5];
};
static_assert(sizeof(LevelRecD) == 256, "LevelRecD must be 256 bytes");

template <typename Real> struct RecOf;
template <> struct RecOf<float> { using type = LevelRecF; };
template <> struct RecOf<double> { using type = LevelRecD; };

// --------------------------------------------------------------- table meta
// Device view of a resident table set.
struct TableView {
  const void *tab;          // [S][nT][nP][pitch] storage elements
  const void *cia;          // [n_cia][nT][pitch] float (double for F64)
  const double *T_axis;     // [nT]
  const double *lp_axis;    // [nP]
  const double *off;        // [S][nT][nP] log2 offsets of the rows
  const double *off_cia;    // [n_cia][nT]
  const double *mass;       // [S] g/mol
  int S, nT, nP, n_cia;
  int64_t n_nu, pitch;
  double nu0, dnu, he_ratio;
  int dtype;                // hr2_table_dtype
  int tab_elem, cia_elem;   // bytes per stored entry
};

// Packed device columns of one batch (FP64).
struct ColumnsView {
  const double *p;      // [B][L]
  const double *T;      // [B][L]
  const double *x;      // [B][S]
  const double *logg;   // [B]
  const double *scale;  // [B]
  const double *cloud = nullptr;  // [B][3] (tau_c, p_top_bar, bottom_frac) or NULL: clear sky
  int B, L;
};

// One segment of a level-kernel launch: the sets of one batch (a request
// when serving) and where their records go.
struct LevelSeg {
  int64_t wg_begin;        // first workgroup of the segment
  int64_t rec_offset;      // records of set s: recs + rec_offset + s * n_levels
  ColumnsView cv;
  int32_t blocks_per_set;  // workgroups per set (from level_blocks_per_set)
  int32_t pad;
};

// One segment of an observation-layout build (one layout per segment).
struct ObsSeg {
  int64_t norm_wg_begin;     // first workgroup of the segment in the normalisation launch
  int64_t weight_wg_begin;   // first workgroup in the weights launch
  int64_t N, i0, n_pts, nnz;
  double nu_first, dnu, denom;
  int32_t n_bins, pad;
  const int64_t *edge_idx;   // [n_bins + 1] snapped edges
  const int64_t *kstart;     // [n_bins]
  const int32_t *mlo;        // [n_bins]
  int32_t *h;                // [n_pts] 5 sigma half widths (written)
  void *q, *invz;            // [n_pts] scratch (Real)
  void *K;                   // [nnz] weights (Real, written)
};

// One segment of a column-kernel launch: a batch of sets sharing levels and
// a wavenumber window (a forward_batch call, or one request when serving).
struct ColSeg {
  int64_t wg_begin;        // first workgroup of the segment
  int64_t nu_begin, nu_count, nu_stride;
  int64_t rec_offset;      // records of set s: recs + rec_offset + s * n_levels
  int64_t out_offset;      // F+ of set s: out + out_offset + s * out_stride
  int64_t out_stride;
  int64_t chi_offset;      // stage call only: chi + chi_offset + l * nu_count
  int32_t n_sets, n_levels, tiles_per_set, n_mu;
  int32_t chunks;          // layer chunks per 64-point tile, 1..8 (= waves per workgroup)
  // Tile groups (one set, the launch's only segment): workgroup blockIdx
  // = x + 8 k runs on XCD x (round-robin dispatch) and covers XCD x's
  // contiguous share of the tiles; its first wg_multi workgroups take
  // tiles_per_wg tiles of chunks / tiles_per_wg layer chunks each, the rest
  // one tile of `chunks`, so the tiles left for the last round of waves
  // finish in a fraction of the levels.  wg_multi = 0: one tile per
  // workgroup (segment lists, batches).
  int32_t wg_multi, tiles_per_wg;
};

// One segment of a convolve/bin launch: n_sets spectra against one layout.
struct ConvSeg {
  int64_t item_begin;       // first workgroup of the segment
  int32_t items_per_wg;     // 1: a (set, bin) per workgroup of four waves;
                            // 4: one per wave (short supports)
  const void *K;            // weights (Real)
  const int64_t *kstart;    // [n_bins]
  const int32_t *mlo;       // [n_bins] first window point of the support
  const int32_t *mlen;      // [n_bins] support length
  int64_t in_offset, in_stride;    // F+ of set s
  int64_t out_offset;              // bins of set s: out + out_offset + s * n_bins
  const double *scale;      // [n_sets] or NULL
  double scale_const;       // used when scale == NULL
  int32_t n_sets, n_bins;
  // Likelihood (Eq. 19, Eq. 22-23); all NULL when only the bins are wanted.
  const double *D;          // [n_bins] observed binned flux
  const double *s2;         // [n_bins] sigma_j^2
  const double *log10_eps;  // [n_sets] error inflation exponent, or NULL
  double *terms;            // [n_sets][n_bins] per-bin terms of ln L
};

// Arguments of the whole-forward-model-per-set launch (small windows).
struct SetFwdArgs {
  int64_t nu_begin, nu_count, nu_stride;
  int32_t n_mu, n_bins;
  float *fplus;             // [B][nu_count] unscaled F+ (written)
  float *bins;              // [B][n_bins] (written)
  int *status;              // [B] or NULL
  const float *K;           // layout weights
  const int64_t *kstart;    // [n_bins]
  const int32_t *mlo;       // [n_bins]
  const int32_t *mlen;      // [n_bins]
};

// Angular quadrature constants for n_mu = 1..8 (Eq. 8): row n-1.
struct AngleTable {
  float mu[kMaxMu][kMaxMu];
  float l2e_mu[kMaxMu][kMaxMu];   // log2(e) / mu
  float inv_mu[kMaxMu][kMaxMu];
  float cw[kMaxMu][kMaxMu];       // 2 pi w mu
  double mu_d[kMaxMu][kMaxMu];
  double inv_mu_d[kMaxMu][kMaxMu];
  double cw_d[kMaxMu][kMaxMu];
};

// Parameter-vector layout (finite-element temperature, free chemistry,
// Eq. 9 scale), passed to the unpack kernel by value.
constexpr int kMaxOrder = HR2_MAX_ORDER;
constexpr int kMaxTNodes = HR2_MAX_TNODES;
struct ParamView {
  double nodes[kMaxOrder + 1];     // Gauss-Lobatto points on [0, 1]
  double inv_den[kMaxOrder + 1];   // 1 / prod_{j != i} (x_i - x_j)
  double fac[kMaxSpecies];
  int32_t src[kMaxSpecies];
  double lp_bottom, lp_top, radius_cm;
  int32_t K, q, L, S, n_free, with_cloud, with_eps, n_theta;
};

// ----------------------------------------------------------------- launchers
// All launchers enqueue on `stream` and return hipSuccess or the launch error.
hipError_t upload_angle_table(const AngleTable &t);

// Level records straight from parameter vectors: the level kernel forms
// each set's column from theta (the same arithmetic as launch_unpack) and
// writes the per-set scale and error-inflation exponent the later stages
// read.  theta == nullptr: the columns come from the ColumnsView.
struct ThetaArgs {
  ParamView pv;
  const double *theta;   // [B][n_theta]
  double *scale;         // [B] out
  double *eps;           // [B] out, or NULL
};

hipError_t launch_levels(const TableView &tv, const ColumnsView &cv, void *recs,
                         int *status, bool fp64, hipStream_t stream,
                         const ThetaArgs *theta = nullptr, hipEvent_t t_start = nullptr,
                         hipEvent_t t_stop = nullptr);
// Workgroups per set of the segmented level launch for columns of L levels.
int level_blocks_per_set(const TableView &tv, int L);
// Several batches in one launch: segs_dev[n_segs] in device memory (ascending
// wg_begin, blocks_per_set from level_blocks_per_set), records relative to
// recs_base; total_wgs = the workgroups of all segments.
hipError_t launch_levels_segs(const TableView &tv, const LevelSeg *segs_dev, int n_segs,
                              int64_t total_wgs, void *recs_base, bool fp64, hipStream_t stream);

// One workgroup = `chunks` waves = one 64-point tile of one set; every
// segment of the launch must use that chunk count.
// para: parabolic source (else linear).
// seg0_host: a launch of one segment passes it by value (segs_dev unused).
// stream_rows: load the table rows non-temporal (a launch of one set, whose
// rows nothing reads again); ignored when the opacity comes from memory.
// t_start / t_stop (optional, here and on the other launch helpers): events
// that take the kernel's own start and end times (the launch's profiling
// timestamps, not markers in the stream).
hipError_t launch_column(const TableView &tv, const ColSeg *segs_dev, int n_segs,
                         const ColSeg *seg0_host, int64_t total_wgs, int chunks, const void *recs,
                         const void *chi_in, void *out, int max_mu, bool opacity_from_memory,
                         bool para, bool stream_rows, hipStream_t stream,
                         hipEvent_t t_start = nullptr, hipEvent_t t_stop = nullptr);
int column_nu_per_wg(int chunks);
// Waves of the column kernel (with this chunk count) the device holds at once.
// Largest angle count of the column kernel variant a request of n_mu angles
// runs (requests of one class share a launch).
int column_mu_class(int n_mu);
int column_wave_capacity(const TableView &tv, int max_mu, bool opacity_from_memory, int chunks,
                         bool para);

// The whole forward model in one launch, one workgroup per set: for FP32,
// FP16 and BF16 tables of one species (below 4 GiB), columns of at most 64
// levels and windows of at most 4096 points (set_forward_fits), a linear
// source and a layout with short supports (one wave per bin).  Same
// arithmetic as the level, column (one chunk) and convolve/bin kernels.
// nu_per_lane: 0 = automatic (two wavenumbers per lane up to three angles,
// one above), 1 or 2; set_forward_nu_per_lane says which the launch uses.
bool set_forward_fits(const TableView &tv, int n_levels, int64_t nu_count);
int set_forward_nu_per_lane(const TableView &tv, int requested, int max_mu);
hipError_t launch_set_forward(const TableView &tv, const ColumnsView &cv, const SetFwdArgs &args,
                              int max_mu, int nu_per_lane, hipStream_t stream,
                              hipEvent_t t_start = nullptr, hipEvent_t t_stop = nullptr);

hipError_t launch_opacity_only(const TableView &tv, const void *recs, int n_levels,
                               int64_t nu_begin, int64_t nu_count, int64_t nu_stride,
                               void *chi, hipStream_t stream);

// Items per convolution workgroup for a layout whose n_bins supports hold
// nnz weights in total (the choice depends on the layout alone), and the
// workgroups that n_items (set, bin) items of it take.
int conv_items_per_wg(int64_t nnz, int n_bins);
int64_t conv_workgroups(int64_t n_items, int items_per_wg);

// total_wgs: the workgroups of all segments.
hipError_t launch_convolve_bin(bool fp64, const ConvSeg *segs_dev, int n_segs,
                               const ConvSeg *seg0_host, int64_t total_wgs, const void *in,
                               void *out, hipStream_t stream, hipEvent_t t_start = nullptr,
                               hipEvent_t t_stop = nullptr);
// ln L per set: the sum over bins of the terms k_convolve_bin wrote.
hipError_t launch_lnl_reduce(const double *terms, int n_sets, int n_bins, double *lnl,
                             hipStream_t stream);

// Parameter vectors -> FP64 columns (p, T [B][L], x [B][S], log g, scale
// [B], cloud [B][3], eps [B]; cloud and eps may be NULL).
hipError_t launch_unpack(const ParamView &pv, int n_sets, const double *theta, double *p,
                         double *T, double *x, double *logg, double *scale, double *cloud,
                         double *eps, hipStream_t stream);

// Observation layout build: the 5 sigma half widths h_i (written to h_dev),
// Z_i and q_i for window points [i0, i0 + n_pts), then the nnz banded
// per-bin weights.  sigma_i = nu_i / denom.
hipError_t launch_obs_build(bool fp64, int64_t N, double nu_first, double dnu_eff, double denom,
                            int n_bins, int64_t nnz, const int64_t *edge_idx_dev, int32_t *h_dev,
                            int64_t i0, int64_t n_pts, void *q_scratch, void *invz_scratch,
                            const int64_t *kstart_dev, const int32_t *mlo_dev, void *K_dev,
                            hipStream_t stream);
// Workgroups of one layout in the normalisation and the weights launches.
int64_t obs_norm_workgroups(bool fp64, int64_t n_pts);
int64_t obs_weight_workgroups(int64_t nnz);
// Several layouts in two launches: segs_dev[n_segs] in device memory
// (ascending workgroup offsets from the two functions above).
hipError_t launch_obs_build_segs(bool fp64, const ObsSeg *segs_dev, int n_segs,
                                 int64_t norm_wgs, int64_t weight_wgs, hipStream_t stream);

}  // namespace hr2

// ------------------------------------------------------------- handle types
struct hr2_tables {
  hr2_ctx *ctx = nullptr;
  hr2::TableView view{};
  void *d_tab = nullptr, *d_cia = nullptr;
  double *d_meta = nullptr;
  std::vector<double> T_axis, lp_axis, off, off_cia, mass;
  size_t bytes = 0;
};

struct hr2_obs {
  hr2_ctx *ctx = nullptr;
  const hr2_tables *tables = nullptr;
  hr2_window window{};
  double R = 0;
  int n_bins = 0;
  bool fp64 = false;
  int64_t nnz = 0;
  std::vector<int64_t> edge_idx;     // [n_bins + 1]
  void *d_K = nullptr;               // Real[nnz]
  int64_t *d_kstart = nullptr;       // [n_bins]
  int32_t *d_mlo = nullptr, *d_mlen = nullptr;
  size_t bytes = 0;
  double *d_D = nullptr, *d_s2 = nullptr;   // [n_bins] data and sigma^2 (hr2_obs_set_data)
};

struct hr2_params {
  hr2_ctx *ctx = nullptr;
  const hr2_tables *tables = nullptr;
  hr2::ParamView view{};
};
