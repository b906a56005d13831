// kernels.hip — gfx950 kernels of libhr2: level records, the fused
// opacity + short-characteristics column kernel, the stage-1 opacity kernel,
// the observation-layout build and the convolve/bin kernel.
//
// Paper: Kitzmann et al. 2020 (arXiv:1910.01070), Sect. 2.1-2.3, 2.7, 2.8,
// Eq. 2, 4-9, 17.  Design: wavefronts of 64 lanes own 64 consecutive window
// points each (coalesced table rows); all per-level quantities are uniform
// across the workgroup and arrive through scalar loads of a 128-byte record;
// the table rows of the bilinear cell stay in registers between levels; the
// layer recurrence may be split into up to eight chunks whose affine maps
// I_out = exp(-tau_c / mu) I_in + B_c are combined through LDS.
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <type_traits>

#include "hr2_internal.h"

namespace hr2 {

// CODATA 2018 exact constants (cgs) and the atomic mass constant.
constexpr double kH = 6.62607015e-27;
constexpr double kC = 2.99792458e10;
constexpr double kKB = 1.380649e-16;
constexpr double kAMU = 1.66053906660e-24;
constexpr double kMH2 = 2.016;
constexpr double kMHe = 4.0026;
constexpr double kC2 = kH * kC / kKB;          // second radiation constant, cm K
constexpr double kC1 = 2.0 * kH * kC * kC;     // 2 h c^2
constexpr double kLog2e = 1.4426950408889634074;
constexpr double kTwoPi = 6.283185307179586477;
constexpr double kParsecCm = 3.0856775814913673e18;   // IAU 2015 parsec
constexpr float kLn2f = 0.69314718055994530942f;

__constant__ AngleTable c_ang;

hipError_t upload_angle_table(const AngleTable &t) {
  return hipMemcpyToSymbol(HIP_SYMBOL(c_ang), &t, sizeof(AngleTable), 0, hipMemcpyHostToDevice);
}

// ------------------------------------------------------------ small helpers

// Workgroups are dispatched round-robin over the eight XCDs; hand each XCD a
// contiguous range of logical work items so that the sets of one wavenumber
// tile (which read the same table rows) share that XCD's L2.
__device__ __forceinline__ int64_t xcd_remap(int64_t g, int64_t n) {
  const int64_t x = g & 7, k = g >> 3;
  const int64_t q = n >> 3, r = n & 7;
  return x * q + (x < r ? x : r) + k;
}

template <typename TT> __device__ __forceinline__ float to_float(TT v);
template <> __device__ __forceinline__ float to_float<float>(float v) { return v; }
template <> __device__ __forceinline__ float to_float<_Float16>(_Float16 v) { return (float)v; }
template <> __device__ __forceinline__ float to_float<uint16_t>(uint16_t v) {
  return __uint_as_float(((uint32_t)v) << 16);   // bfloat16 -> float is exact
}

// Table reads go through buffer resources (base + byte size in SGPRs, the
// lane's 32-bit byte offset in a VGPR): one address add per load, and the
// hardware returns 0 for any offset past the resource instead of faulting.
using rsrc_t = __amdgpu_buffer_rsrc_t;
__device__ __forceinline__ rsrc_t make_rsrc(const void *base, int64_t bytes) {
  const uint32_t n = bytes >= 0xFFFFFFFFll ? 0xFFFFFFFFu : (uint32_t)bytes;
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)n,
                                           0x00020000);
}
// soff: a uniform byte offset added by the hardware (scalar operand).
// CPOL: the load's cache-policy bits (0, or kCpolStream for rows read once).
constexpr int kCpolStream = 2;   // nt: non-temporal
template <typename TT, int CPOL = 0>
__device__ __forceinline__ TT buf_load(rsrc_t r, uint32_t off, uint32_t soff) {
  if constexpr (std::is_same<TT, float>::value) {
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, off, soff, CPOL));
  } else if constexpr (std::is_same<TT, _Float16>::value) {
    const unsigned short u = __builtin_amdgcn_raw_buffer_load_b16(r, off, soff, CPOL);
    return __builtin_bit_cast(_Float16, u);
  } else if constexpr (std::is_same<TT, uint16_t>::value) {
    return __builtin_amdgcn_raw_buffer_load_b16(r, off, soff, CPOL);
  } else {
    static_assert(std::is_same<TT, double>::value, "table element type");
    const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, off, soff, CPOL);
    return __builtin_bit_cast(double, v);
  }
}

// The lane's byte offset in a CIA row (FP32 or FP64 elements, like the
// sweep) from its byte offset in a table row (TT elements): formed at each
// CIA fetch when the two element sizes differ, by an opaque shift that the
// compiler cannot hoist, so that no register holds it across the sweep.
template <typename TT, typename Real = float>
__device__ __forceinline__ uint32_t cia_offset_from_row_offset(uint32_t kb) {
  if constexpr (sizeof(TT) == sizeof(Real)) {
    return kb;
  } else {
    static_assert(sizeof(Real) == 2 * sizeof(TT), "FP32 sweep over 16-bit rows");
    uint32_t r;
    asm volatile("v_lshlrev_b32 %0, 1, %1" : "=v"(r) : "v"(kb));
    return r;
  }
}

__device__ __forceinline__ float fexp2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }

// A launch with start/stop events takes the kernel's own timestamps
// (hipExtLaunchKernel); without events it is a plain launch (which stream
// capture records).
template <typename F, typename... Args>
static void launch_timed(F kernel, dim3 grid, dim3 block, uint32_t shmem, hipStream_t stream,
                         hipEvent_t t_start, hipEvent_t t_stop, Args... args) {
  if (t_start || t_stop)
    hipExtLaunchKernelGGL(kernel, grid, block, shmem, stream, t_start, t_stop, 0u, args...);
  else
    hipLaunchKernelGGL(kernel, grid, block, shmem, stream, args...);
}

// ------------------------------------------------------------ level records
// Each workgroup stages one set (inputs and axes in LDS, every level's cell)
// and runs independent items: per level, one for the cell, rows, weights and
// masks, one for the layer above it, and one per species and CIA pair.
// Everything here is FP64; the column kernel gets FP32 (FP64 for F64
// tables) per-level constants:
//   n = p / (k_B T); n_s = x_s n; x_H2 = (1 - sum x)/(1 + r), x_He = r x_H2;
//   mubar; dz_l = k_B (T_l + T_l+1)/2 / (mubar m_u g) ln(p_l / p_l+1)
//   (Sect. 2, 2.4, 5.2 and the hydrostatic reading of the optical depths);
// the bilinear cell of (T, log10 p) and its corner weights, the corner rows
// assigned to slots by node parity (slot = (row_T & 1) * 2 + (row_p & 1)),
// so a row shared by consecutive levels keeps its slot and is not reloaded.
struct CellW {
  int iT, ip;
  double wT, wp;
};

// slot k <-> corner (a, b) of the cell with row parity k
__device__ __forceinline__ void slot_corner(const CellW &c, int k, int nP, int &row, double &w) {
  const int a = ((k >> 1) ^ c.iT) & 1;
  const int b = ((k & 1) ^ c.ip) & 1;
  row = (c.iT + a) * nP + (c.ip + b);
  w = (a ? c.wT : 1.0 - c.wT) * (b ? c.wp : 1.0 - c.wp);
}

__device__ __forceinline__ void cia_slot(const CellW &c, int k, int &row, double &w) {
  const int a = (k ^ c.iT) & 1;
  row = c.iT + a;
  w = a ? c.wT : 1.0 - c.wT;
}

constexpr int kMaxAxis = 256;

// Axis lookup (reading of Sect. 2.3): lower node = the largest index with
// a[i] <= v (v clamped to the axis), at most n-2, and w = (v - a_i)/(a_{i+1}
// - a_i); binary search over the LDS copy of the axis
__device__ __forceinline__ void locate_lds(const double *a, int n, double v, int &i, double &w) {
  v = v < a[0] ? a[0] : v;
  v = v > a[n - 1] ? a[n - 1] : v;
  int lo = 0, hi = n - 1;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (a[mid] <= v) lo = mid;
    else hi = mid;
  }
  i = lo;
  w = (v - a[lo]) / (a[lo + 1] - a[lo]);
}

// ------------------------------------------------- parameter vector pieces
// Layout of theta (Table 1 order): log g, f, d [pc], T1, b_1..b_{NT-1}, the
// free mixing ratios, then (tau_c, p_top, bottom_frac) with a cloud and eps
// last.  Node temperatures T_0 = T1, T_n = b_n T_{n-1} (Sect. 2.5.1); the
// return value says whether the vector is invalid.
__device__ bool theta_nodes(const ParamView &pv, const double *th, double *Tn) {
  const int NT = pv.K * pv.q + 1;
  bool bad = !isfinite(th[0]) || !(th[1] > 0.0) || !isfinite(th[1]) || !(th[2] > 0.0) ||
             !isfinite(th[2]);
  double t = th[3];
  bad |= !(t > 0.0) || !isfinite(t);
  Tn[0] = t;
  for (int n = 1; n < NT; ++n) {
    const double b = th[3 + n];
    bad |= !(b > 0.0) || !isfinite(b);
    t *= b;
    Tn[n] = t;
  }
  for (int k = 0; k < pv.n_free; ++k) {
    const double xf = th[3 + NT + k];
    bad |= !(xf >= 0.0) || !isfinite(xf);
  }
  if (pv.with_cloud) {
    const double *c = th + 3 + NT + pv.n_free;
    bad |= !(c[0] >= 0.0) || !isfinite(c[0]);
    if (c[0] > 0.0)
      bad |= !(c[1] > 0.0) || !isfinite(c[1]) || !(c[2] > 1.0) || !isfinite(c[2]);
  }
  if (pv.with_eps) bad |= !isfinite(th[3 + NT + pv.n_free + 3 * pv.with_cloud]);
  return bad;
}

// Level l sits at u = l K / (L - 1) element widths above the bottom (levels
// and elements both equidistant in log p over the same range), in element
// k = min(floor(u), K - 1) at local coordinate xi = u - k, where
// T = sum_i T_{kq+i} l_i(xi) (Eq. 12-13); NaN for an invalid vector.
__device__ void theta_level(const ParamView &pv, const double *Tn, int l, bool bad, double &p,
                            double &T) {
  const int L = pv.L;
  const double step = (pv.lp_top - pv.lp_bottom) / (double)(L - 1);
  const double lp = l == L - 1 ? pv.lp_top : pv.lp_bottom + (double)l * step;
  p = exp10(lp);
  const double u = (double)l * (double)pv.K / (double)(L - 1);
  int k = (int)floor(u);
  k = k < 0 ? 0 : (k > pv.K - 1 ? pv.K - 1 : k);
  const double xi = u - (double)k;
  double acc = 0.0;
  for (int i = 0; i <= pv.q; ++i) {
    double li = pv.inv_den[i];
    for (int j = 0; j <= pv.q; ++j)
      if (j != i) li *= xi - pv.nodes[j];
    acc += Tn[k * pv.q + i] * li;
  }
  T = bad ? __builtin_nan("") : acc;
}

__device__ double theta_x(const ParamView &pv, const double *th, int sp) {
  const int src = pv.src[sp];
  return src >= 0 ? pv.fac[sp] * th[3 + pv.K * pv.q + 1 + src] : 0.0;
}

// f (R/d)^2 (Eq. 9), d in parsec
__device__ double theta_scale(const ParamView &pv, const double *th) {
  const double rd = pv.radius_cm / (th[2] * kParsecCm);
  return th[1] * rd * rd;
}

// the cloud triple (with a cloud) and eps follow the free mixing ratios
__device__ const double *theta_tail(const ParamView &pv, const double *th) {
  return th + 3 + pv.K * pv.q + 1 + pv.n_free;
}

// 128-thread workgroups, each staging its set: at C2 (101 levels, 12 items
// per level) ten per set; shorter barriers and more CUs per set than larger
// workgroups (per C2 spectrum: 1024 threads 10.1 us, 256 threads 7.7 us,
// 128 threads 7.0-7.3 us; 64 threads 8.3-8.4 us)
constexpr int kLevelThreads = 128;

// A double that every lane of the wave holds (loaded from one address, or
// formed from the same LDS values): moved to scalar registers, so that it
// costs no vector registers while the level items run.
__device__ __forceinline__ double wave_uniform(double v) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)u);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(u >> 32));
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// The level records of set s, written to recs_set[0 .. L-1] (global or LDS
// memory): the items of that set that fall to this workgroup, which is
// workgroup `part` of the blocks_per_set ones sharing the set.  Every thread
// of the workgroup calls it (it has barriers).
template <typename Real>
__device__ void level_records(const TableView &tv, const ColumnsView &cv, int s, int part,
                              int blocks_per_set, typename RecOf<Real>::type *recs_set,
                              int *status, const ThetaArgs &ta) {
  using Rec = typename RecOf<Real>::type;
  __shared__ double s_T[kMaxAxis], s_lp[kMaxAxis];
  __shared__ double s_pl[HR2_MAX_LEVELS], s_Tl[HR2_MAX_LEVELS];
  __shared__ double s_x[kMaxSpecies], s_m[kMaxSpecies];
  __shared__ CellW s_cell[HR2_MAX_LEVELS];
  const int L = cv.L;
  const int S = tv.S;
  // one coalesced pass over the set's inputs and the axes
  for (int i = threadIdx.x; i < tv.nT; i += blockDim.x) s_T[i] = tv.T_axis[i];
  for (int i = threadIdx.x; i < tv.nP; i += blockDim.x) s_lp[i] = tv.lp_axis[i];
  if (threadIdx.x < S) s_m[threadIdx.x] = tv.mass[threadIdx.x];
  double logg, scale;
  // gray cloud (App. B): tau_c >= 0; with tau_c > 0 a top pressure > 0 and a
  // bottom at bottom_frac > 1 times the top
  double tau_c = 0.0, c_top = 1.0, c_frac = 2.0;
  if (ta.theta != nullptr) {
    // the column from the set's parameter vector
    __shared__ double s_Tn[kMaxTNodes];
    __shared__ int s_badt;
    const double *th = ta.theta + (int64_t)s * ta.pv.n_theta;
    if (threadIdx.x == 0) s_badt = theta_nodes(ta.pv, th, s_Tn) ? 1 : 0;
    __syncthreads();
    const bool badt = s_badt != 0;
    for (int l = threadIdx.x; l < L; l += blockDim.x)
      theta_level(ta.pv, s_Tn, l, badt, s_pl[l], s_Tl[l]);
    if (threadIdx.x < S) s_x[threadIdx.x] = theta_x(ta.pv, th, threadIdx.x);
    logg = th[0];
    scale = theta_scale(ta.pv, th);
    const double *c = theta_tail(ta.pv, th);
    if (ta.pv.with_cloud) {
      tau_c = c[0];
      c_top = c[1];
      c_frac = c[2];
    }
    if (part == 0 && threadIdx.x == 0) {
      ta.scale[s] = scale;
      if (ta.eps) ta.eps[s] = ta.pv.with_eps ? c[3 * ta.pv.with_cloud] : 0.0;
    }
  } else {
    for (int l = threadIdx.x; l < L; l += blockDim.x) {
      s_pl[l] = cv.p[(int64_t)s * L + l];
      s_Tl[l] = cv.T[(int64_t)s * L + l];
    }
    if (threadIdx.x < S) s_x[threadIdx.x] = cv.x[(int64_t)s * S + threadIdx.x];
    logg = cv.logg[s];
    scale = cv.scale[s];
    if (cv.cloud) {
      tau_c = cv.cloud[(int64_t)s * 3];
      c_top = cv.cloud[(int64_t)s * 3 + 1];
      c_frac = cv.cloud[(int64_t)s * 3 + 2];
    }
  }
  __syncthreads();

  // column-wide quantities and validity (Sect. 5.2 filler gas, Table 1 inputs)
  bool bad = false;
  double xs = 0.0, mm = 0.0;
  for (int q = 0; q < S; ++q) {
    bad |= !(s_x[q] >= 0.0) || !isfinite(s_x[q]);
    xs += s_x[q];
    mm += s_x[q] * s_m[q];
  }
  logg = wave_uniform(logg);
  scale = wave_uniform(scale);
  tau_c = wave_uniform(tau_c);
  c_top = wave_uniform(c_top);
  c_frac = wave_uniform(c_frac);
  xs = wave_uniform(xs);
  mm = wave_uniform(mm);
  bad |= !(xs < 1.0) || !isfinite(logg) || !isfinite(scale);
  bad |= !(tau_c >= 0.0) || !isfinite(tau_c);
  if (tau_c > 0.0)
    bad |= !(c_top > 0.0) || !isfinite(c_top) || !(c_frac > 1.0) || !isfinite(c_frac);
  for (int l = threadIdx.x; l < L; l += blockDim.x) {
    bad |= !(s_pl[l] > 0.0) || !isfinite(s_pl[l]) || !(s_Tl[l] > 0.0) || !isfinite(s_Tl[l]);
    if (l + 1 < L) bad |= !(s_pl[l] > s_pl[l + 1]);
  }
  // every level's table cell, once per workgroup (independent of the
  // validity checks: invalid inputs give NaN weights and NaN hdz records)
  for (int l = threadIdx.x; l < L; l += blockDim.x) {
    CellW c;
    locate_lds(s_T, tv.nT, s_Tl[l], c.iT, c.wT);
    locate_lds(s_lp, tv.nP, log10(s_pl[l]), c.ip, c.wp);
    s_cell[l] = c;
  }
  bad = __syncthreads_or(bad);
  if (status != nullptr && threadIdx.x == 0 && part == 0)
    status[s] = bad ? (int)HR2_E_INVALID_ARG : 0;

  const double h2 = (1.0 - xs) / (1.0 + tv.he_ratio);
  const double he = tv.he_ratio * h2;
  mm += h2 * kMH2 + he * kMHe;
  const int64_t rows_per_species = (int64_t)tv.nT * tv.nP;
  const uint32_t row_bytes = (uint32_t)(tv.pitch * tv.tab_elem);
  const uint32_t cia_row_bytes = (uint32_t)(tv.pitch * tv.cia_elem);
  auto cell_of = [&](int l) { return s_cell[l]; };

  // Items: first one per level (everything but the species factors), then
  // one per (level, species or CIA pair); no item waits for another, so the
  // table offsets are fetched while the level items run.  Items write
  // disjoint fields of the records.
  const int per_level = S + tv.n_cia;
  const int n_items = L * (2 + per_level);
  // every launch gives each item a thread of its own (blocks_per_set
  // workgroups of blockDim.x threads cover n_items), so a thread runs at most
  // one item: a branch, not a loop, whose invariant FP64 polynomial constants
  // the compiler would keep in (and spill from) vector registers
  const int t = part * blockDim.x + threadIdx.x;
  if (t < n_items) {
    if (t >= L && t < 2 * L) {
      // the layer above level l: half thickness and cloud optical depth
      const int l = t - L;
      Rec *r = recs_set + l;
      double hdz = 0.0, dtc = 0.0;
      if (l + 1 < L) {
        const double tbar = 0.5 * (s_Tl[l] + s_Tl[l + 1]);
        const double lr = log(s_pl[l] / s_pl[l + 1]);
        hdz = 0.5 * kKB * tbar / (mm * kAMU * exp10(logg)) * lr;
        // the cloud's optical depth, spread uniformly in ln p over
        // [p_top, p_top bottom_frac]: this layer's share of that range
        if (tau_c > 0.0) {
          const double lc_top = log(c_top), lc_bot = log(c_top * c_frac);
          const double hi = fmin(log(s_pl[l]), lc_bot), lo = fmax(log(s_pl[l + 1]), lc_top);
          if (hi > lo) dtc = tau_c * (hi - lo) / (lc_bot - lc_top);
        }
      }
      if (bad) hdz = __builtin_nan("");
      r->hdz = (Real)hdz;
      r->dtc = (Real)dtc;
    } else if (t < L) {
      const int l = t;
      Rec *r = recs_set + l;
      const CellW c = cell_of(l);
      const bool has_prev = l > 0, has_next = l + 1 < L;
      const CellW cp = has_prev ? cell_of(l - 1) : c;
      const CellW cn = has_next ? cell_of(l + 1) : c;
      int mask = 0;
      for (int k = 0; k < 4; ++k) {
        int row, rowp, rown;
        double w, wp, wn;
        slot_corner(c, k, tv.nP, row, w);
        slot_corner(cp, k, tv.nP, rowp, wp);
        slot_corner(cn, k, tv.nP, rown, wn);
        r->w[k] = (Real)w;
        r->rowb[k] = (uint32_t)row * row_bytes;
        const bool nz = w != 0.0;
        const bool kept = has_prev && wp != 0.0 && rowp == row;
        const bool kept_dn = has_next && wn != 0.0 && rown == row;
        if (nz) mask |= 1 << (8 + k);
        if (nz && !kept) mask |= 1 << k;
        if (nz && !kept_dn) mask |= 1 << (16 + k);
      }
      for (int k = 0; k < 2; ++k) {
        int row, rowp, rown;
        double w, wp, wn;
        cia_slot(c, k, row, w);
        cia_slot(cp, k, rowp, wp);
        cia_slot(cn, k, rown, wn);
        r->cia_rowb[k] = (uint32_t)row * cia_row_bytes;
        r->cia_w[k] = (Real)w;
        const bool nz = w != 0.0 && tv.n_cia > 0;
        const bool kept = has_prev && wp != 0.0 && rowp == row;
        const bool kept_dn = has_next && wn != 0.0 && rown == row;
        if (nz) mask |= 1 << (12 + k);
        if (nz && !kept) mask |= 1 << (4 + k);
        if (nz && !kept_dn) mask |= 1 << (20 + k);
      }
      r->mask = mask;
      for (int q = S; q < kMaxSpecies; ++q) r->a_s[q] = (Real)0;
      if (tv.n_cia == 0) r->a_cia[0] = r->a_cia[1] = (Real)0;
      if constexpr (std::is_same<Real, float>::value) {
        const double pl = kC2 * kLog2e / s_Tl[l];
        const float hi = (float)pl;
        r->pl_hi = hi;
        r->pl_lo = (float)(pl - (double)hi);
        r->pad = 0.0f;
      } else {
        r->T = s_Tl[l];
        r->pad0 = 0;
        for (int q = 0; q < 5; ++q) r->pad[q] = 0.0;
      }
    } else {
      // n_s 2^{interpolated row offset} (and the CIA pairs' n_a n_b 2^{...}):
      // the column kernel exponentiates only the stored offset-free part,
      // keeping its exp2 argument small.
      const int u = t - 2 * L;
      const int l = u / per_level, q = u - l * per_level;
      Rec *r = recs_set + l;
      const CellW c = cell_of(l);
      const double n = s_pl[l] * 1.0e6 / (kKB * s_Tl[l]);
      if (q < S) {
        double off[4], w[4];
        for (int k = 0; k < 4; ++k) {
          int row;
          slot_corner(c, k, tv.nP, row, w[k]);
          off[k] = tv.off[q * rows_per_species + row];
        }
        const double cq = w[0] * off[0] + w[1] * off[1] + w[2] * off[2] + w[3] * off[3];
        r->a_s[q] = (Real)(s_x[q] * n * exp2(cq));
      } else {
        const int qc = q - S;
        double cq = 0.0;
        for (int k = 0; k < 2; ++k) {
          int row;
          double w;
          cia_slot(c, k, row, w);
          cq += w * tv.off_cia[qc * tv.nT + row];
        }
        const double nh2 = h2 * n, nhe = he * n;
        r->a_cia[qc] = (Real)((qc == 0 ? nh2 * nh2 : nh2 * nhe) * exp2(cq));
      }
    }
  }
}

// n_segs == 0: one batch, passed by value in seg0; otherwise the segment
// holding this workgroup (the last one with wg_begin <= blockIdx.x)
template <typename Real>
__global__ __launch_bounds__(kLevelThreads) void k_levels(TableView tv, const LevelSeg *segs,
                                                int n_segs, LevelSeg seg0,
                                                typename RecOf<Real>::type *recs_base,
                                                int *status, ThetaArgs ta) {
  int sg = 0;
  for (int lo = 0, hi = n_segs; hi - lo > 1;) {
    const int mid = (lo + hi) >> 1;
    if (segs[mid].wg_begin <= (int64_t)blockIdx.x) lo = mid;
    else hi = mid;
    sg = lo;
  }
  const LevelSeg d = n_segs == 0 ? seg0 : segs[sg];
  const int blocks_per_set = d.blocks_per_set;
  // blocks_per_set workgroups share one set's items; each stages the set
  const int64_t local = (int64_t)blockIdx.x - d.wg_begin;
  const int s = (int)(local / blocks_per_set);
  const int part = (int)(local - (int64_t)s * blocks_per_set);
  level_records<Real>(tv, d.cv, s, part, blocks_per_set,
                      recs_base + d.rec_offset + (int64_t)s * d.cv.L, status, ta);
}

hipError_t launch_levels(const TableView &tv, const ColumnsView &cv, void *recs, int *status,
                         bool fp64, hipStream_t stream, const ThetaArgs *theta,
                         hipEvent_t t_start, hipEvent_t t_stop) {
  ThetaArgs ta{};
  if (theta) ta = *theta;
  // one workgroup per kLevelThreads items of a set: every item runs at once
  const int64_t items = (int64_t)cv.L * (2 + tv.S + tv.n_cia);
  const int threads = (int)std::min<int64_t>(kLevelThreads, (items + 63) / 64 * 64);
  const int per_set = (int)((items + threads - 1) / threads);
  const dim3 grid((unsigned)((int64_t)cv.B * per_set));
  LevelSeg seg0{};
  seg0.wg_begin = 0;
  seg0.rec_offset = 0;
  seg0.cv = cv;
  seg0.blocks_per_set = per_set;
  if (fp64)
    launch_timed(k_levels<double>, grid, dim3(threads), 0u, stream, t_start, t_stop, tv,
                 (const LevelSeg *)nullptr, 0, seg0, (LevelRecD *)recs, status, ta);
  else
    launch_timed(k_levels<float>, grid, dim3(threads), 0u, stream, t_start, t_stop, tv,
                 (const LevelSeg *)nullptr, 0, seg0, (LevelRecF *)recs, status, ta);
  return hipGetLastError();
}

int level_blocks_per_set(const TableView &tv, int L) {
  const int64_t items = (int64_t)L * (2 + tv.S + tv.n_cia);
  return (int)((items + kLevelThreads - 1) / kLevelThreads);
}

hipError_t launch_levels_segs(const TableView &tv, const LevelSeg *segs_dev, int n_segs,
                              int64_t total_wgs, void *recs_base, bool fp64, hipStream_t stream) {
  if (total_wgs <= 0) return hipSuccess;
  const ThetaArgs ta{};
  const LevelSeg seg0{};
  if (fp64)
    hipLaunchKernelGGL(k_levels<double>, dim3((unsigned)total_wgs), dim3(kLevelThreads), 0,
                       stream, tv, segs_dev, n_segs, seg0, (LevelRecD *)recs_base, nullptr, ta);
  else
    hipLaunchKernelGGL(k_levels<float>, dim3((unsigned)total_wgs), dim3(kLevelThreads), 0,
                       stream, tv, segs_dev, n_segs, seg0, (LevelRecF *)recs_base, nullptr, ta);
  return hipGetLastError();
}

// --------------------------------------------------------------- RT pieces

// Planck source, Eq. 2 (wavenumber form), FP32: x = c2 nu / T is formed as
// an unevaluated float sum (pl_hi + pl_lo)(nu_hi + nu_lo) in log2 units so
// that exp stays accurate for large x; expm1 by its series below x = 1/2.
// Above, B = c1 nu^3 g / (1 - g) with g = e^{-x} <= e^{-1/2}: no overflow for
// any x (g underflows to 0, and B with it, once x passes ~87).
__device__ __forceinline__ float planck_f(float nu_hi, float nu_lo, float c1nu3, float pl_hi,
                                          float pl_lo) {
  const float p_hi = pl_hi * nu_hi;
  const float p_err = fmaf(pl_hi, nu_hi, -p_hi);
  const float p_lo = fmaf(pl_hi, nu_lo, fmaf(pl_lo, nu_hi, p_err));
  const float xl2 = p_hi + p_lo;
  if (xl2 < 0.72134752044448170f) {   // x < 1/2
    const float x = xl2 * kLn2f;
    float t = 1.0f / 40320.0f;
    t = fmaf(t, x, 1.0f / 5040.0f);
    t = fmaf(t, x, 1.0f / 720.0f);
    t = fmaf(t, x, 1.0f / 120.0f);
    t = fmaf(t, x, 1.0f / 24.0f);
    t = fmaf(t, x, 1.0f / 6.0f);
    t = fmaf(t, x, 0.5f);
    t = fmaf(t, x, 1.0f);
    return c1nu3 * frcp(t * x);
  }
  const float g = fexp2(-p_hi) * fmaf(-p_lo, kLn2f, 1.0f);
  return c1nu3 * g * frcp(1.0f - g);
}

__device__ __forceinline__ double planck_d(double nu, double c1nu3, double T) {
  return c1nu3 / expm1(kC2 * nu / T);
}

// One layer of Eq. 4-7 for one angle (FP32).  Linear source, alpha = 0,
// attenuation e = exp(-Delta), Delta = dtau / mu, u = (1 - e)/Delta:
//   I_new = e I + (1 - u) S1 + (u - e) S0 = S1 + e (I - S0) + u (S0 - S1).
// D = S0 - S1 and rD = D / dtau are per layer.  Below Delta = 1/20, u comes
// from its series to Delta^3 (truncation < 1e-7) and e = 1 - Delta u, which
// avoids the cancellation in 1 - e; above, u D = (1 - e) mu rD.
__device__ __forceinline__ void sc_coef_f(float dtau, float rD, float D, float inv_mu,
                                          float l2e_mu, float mu, float &e, float &uD) {
  const float d = dtau * inv_mu;
  if (d < 0.05f) {
    float u = fmaf(d, -1.0f / 24.0f, 1.0f / 6.0f);
    u = fmaf(d, u, -0.5f);
    u = fmaf(d, u, 1.0f);
    e = fmaf(-d, u, 1.0f);
    uD = u * D;
  } else {
    e = fexp2(-dtau * l2e_mu);
    const float m = mu * rD;
    uD = fmaf(-e, m, m);
  }
}

__device__ __forceinline__ float sc_step_f(float I, float dtau, float rD, float S1, float S0,
                                           float D, float inv_mu, float l2e_mu, float mu) {
  float e, uD;
  sc_coef_f(dtau, rD, D, inv_mu, l2e_mu, mu, e, uD);
  return fmaf(e, I - S0, S1) + uD;
}

// The same step with the weights beta = 1 - u, gamma = u - e formed
// explicitly (FP32): I_new = e I + beta S1 + gamma S0.  Below Delta = 1/2,
// beta comes from its series and gamma = Delta (1 - beta) - beta,
// e = 1 - Delta (1 - beta).  Used by the parabolic sweep for its linear
// steps, where it needs no per-layer source difference in registers.
__device__ __forceinline__ void sc_weights_coef_f(float dtau, float rdt, float S1, float S0,
                                                  float inv_mu, float l2e_mu, float mu, float &e,
                                                  float &c) {
  const float d = dtau * inv_mu;
  float beta, gamma;
  if (d < 0.5f) {
    float b = -1.0f / 362880.0f;
    b = fmaf(b, d, 1.0f / 40320.0f);
    b = fmaf(b, d, -1.0f / 5040.0f);
    b = fmaf(b, d, 1.0f / 720.0f);
    b = fmaf(b, d, -1.0f / 120.0f);
    b = fmaf(b, d, 1.0f / 24.0f);
    b = fmaf(b, d, -1.0f / 6.0f);
    b = fmaf(b, d, 0.5f);
    beta = b * d;
    const float ome = d * (1.0f - beta);
    gamma = ome - beta;
    e = 1.0f - ome;
  } else {
    e = fexp2(-dtau * l2e_mu);
    const float u = (1.0f - e) * (rdt * mu);
    beta = 1.0f - u;
    gamma = u - e;
  }
  c = fmaf(beta, S1, gamma * S0);
}

__device__ __forceinline__ float sc_step_weights_f(float I, float dtau, float rdt, float S1,
                                                   float S0, float inv_mu, float l2e_mu, float mu) {
  float e, c;
  sc_weights_coef_f(dtau, rdt, S1, S0, inv_mu, l2e_mu, mu, e, c);
  return fmaf(e, I, c);
}

// The layer as an affine map I -> e I + c (FP64), for sweeps that compose
// maps from the top down.
__device__ __forceinline__ void sc_coef_d(double dtau, double S1, double S0, double mu, double &e,
                                          double &c) {
  const double d = dtau / mu;
  e = exp(-d);
  const double u = d > 0.0 ? -expm1(-d) / d : 1.0;
  c = (1.0 - u) * S1 + (u - e) * S0;
}

__device__ __forceinline__ double sc_step_d(double I, double dtau, double S1, double S0,
                                            double mu) {
  const double d = dtau / mu;
  const double e = exp(-d);
  const double u = d > 0.0 ? -expm1(-d) / d : 1.0;
  const double beta = 1.0 - u, gamma = u - e;
  return e * I + beta * S1 + gamma * S0;
}

// One parabolic step (the higher-order interpolant of Eq. 4-7, after Olson
// & Kunasz 1987): the source on the upwind layer is the quadratic through
// the upwind, local and downwind levels.  With path lengths du, dd (optical
// depths over mu of the upwind and downwind layers) and the moments
// w_n = int_0^du x^n e^{-x} dx,
//   I_new = e^{-du} I + w0 S_loc + gamma (S_up - S_loc) + alpha (S_dn - S_loc)
//   gamma = (w2 + dd w1) / (du (du + dd)),  alpha = (w2 - du w1) / (dd (du + dd))
// (alpha + beta + gamma = w0 written with differences of S).  FP32: below
// du = 1/2 the moments come from their series, q0 = w0/du,
// q1 = w1/du^2 and q21 = (w2 - du w1)/du^3, free of cancellation; dd > 0.
// r_s = 1/(dtau_u + dtau_d) and r_d = 1/dtau_d, r_u = 1/dtau_u are shared
// by the angles.
__device__ __forceinline__ void sc_para_coef_f(float dtau_u, float dtau_d, float r_u, float r_d,
                                               float r_s, float S_up, float S_loc, float S_dn,
                                               float inv_mu, float l2e_mu, float mu, float &e,
                                               float &c) {
  const float du = dtau_u * inv_mu, dd = dtau_d * inv_mu;
  const float i_s = mu * r_s;   // 1 / (du + dd)
  float w0, gam, alp;
  if (du < 0.5f) {
    // Horner in -du; coefficients 1/(m+1)!, 1/(m! (m+2)), -1/(m! (m+2)(m+3)), m = 9 .. 0
    const float x = -du;
    float q0 = 2.755731922e-07f, q1 = 2.505210839e-07f, q21 = -2.087675699e-08f;
    q0 = fmaf(q0, x, 2.755731922e-06f);
    q1 = fmaf(q1, x, 2.480158730e-06f);
    q21 = fmaf(q21, x, -2.254689755e-07f);
    q0 = fmaf(q0, x, 2.480158730e-05f);
    q1 = fmaf(q1, x, 2.204585538e-05f);
    q21 = fmaf(q21, x, -2.204585538e-06f);
    q0 = fmaf(q0, x, 1.984126984e-04f);
    q1 = fmaf(q1, x, 1.736111111e-04f);
    q21 = fmaf(q21, x, -1.929012346e-05f);
    q0 = fmaf(q0, x, 1.388888889e-03f);
    q1 = fmaf(q1, x, 1.190476190e-03f);
    q21 = fmaf(q21, x, -1.488095238e-04f);
    q0 = fmaf(q0, x, 8.333333333e-03f);
    q1 = fmaf(q1, x, 6.944444444e-03f);
    q21 = fmaf(q21, x, -9.920634921e-04f);
    q0 = fmaf(q0, x, 4.166666667e-02f);
    q1 = fmaf(q1, x, 3.333333333e-02f);
    q21 = fmaf(q21, x, -5.555555556e-03f);
    q0 = fmaf(q0, x, 1.666666667e-01f);
    q1 = fmaf(q1, x, 1.250000000e-01f);
    q21 = fmaf(q21, x, -2.500000000e-02f);
    q0 = fmaf(q0, x, 5.000000000e-01f);
    q1 = fmaf(q1, x, 3.333333333e-01f);
    q21 = fmaf(q21, x, -8.333333333e-02f);
    q0 = fmaf(q0, x, 1.000000000e+00f);
    q1 = fmaf(q1, x, 5.000000000e-01f);
    q21 = fmaf(q21, x, -1.666666667e-01f);
    w0 = du * q0;
    e = 1.0f - w0;
    gam = du * fmaf(du, q1 + q21, dd * q1) * i_s;
    alp = du * du * du * q21 * (mu * r_d) * i_s;
  } else {
    e = fexp2(-dtau_u * l2e_mu);
    w0 = 1.0f - e;
    const float w1 = fmaf(-du, e, w0);
    const float w2 = fmaf(-du * du, e, 2.0f * w1);
    gam = fmaf(dd, w1, w2) * (mu * r_u) * i_s;
    alp = fmaf(-du, w1, w2) * (mu * r_d) * i_s;
  }
  c = fmaf(w0, S_loc, fmaf(gam, S_up - S_loc, alp * (S_dn - S_loc)));
}

__device__ __forceinline__ float sc_para_f(float I, float dtau_u, float dtau_d, float r_u,
                                           float r_d, float r_s, float S_up, float S_loc,
                                           float S_dn, float inv_mu, float l2e_mu, float mu) {
  float e, c;
  sc_para_coef_f(dtau_u, dtau_d, r_u, r_d, r_s, S_up, S_loc, S_dn, inv_mu, l2e_mu, mu, e, c);
  return fmaf(e, I, c);
}

__device__ __forceinline__ void sc_para_coef_d(double dtau_u, double dtau_d, double S_up,
                                               double S_loc, double S_dn, double mu, double &e,
                                               double &c) {
  if (dtau_u == 0.0) {
    e = 1.0;
    c = 0.0;
    return;
  }
  const double du = dtau_u / mu, dd = dtau_d / mu;
  double w0, gam, alp;
  if (du < 0.5) {
    // the series of the FP32 step, to m = 16 (FP64 accuracy at du = 1/2)
    const double x = -du;
    double q0 = 2.81145725434552060e-15, q1 = 2.65526518465965852e-15, q21 = -1.39750799192613615e-16;
    q0 = fma(q0, x, 4.77947733238738525e-14);
    q1 = fma(q1, x, 4.49833160695283296e-14);
    q21 = fma(q21, x, -2.49907311497379604e-15);
    q0 = fma(q0, x, 7.64716373181981641e-13);
    q1 = fma(q1, x, 7.16921599858107782e-13);
    q21 = fma(q21, x, -4.21718588151828129e-14);
    q0 = fma(q0, x, 1.14707455977297245e-11);
    q1 = fma(q1, x, 1.07060292245477428e-11);
    q21 = fma(q21, x, -6.69126826534233923e-13);
    q0 = fma(q0, x, 1.60590438368216133e-10);
    q1 = fma(q1, x, 1.49119692770486430e-10);
    q21 = fma(q21, x, -9.94131285136576102e-12);
    q0 = fma(q0, x, 2.08767569878681002e-09);
    q1 = fma(q1, x, 1.92708526041859370e-09);
    q21 = fma(q21, x, -1.37648947172756701e-10);
    q0 = fma(q0, x, 2.50521083854417202e-08);
    q1 = fma(q1, x, 2.29644326866549102e-08);
    q21 = fma(q21, x, -1.76649482205037760e-09);
    q0 = fma(q0, x, 2.75573192239858883e-07);
    q1 = fma(q1, x, 2.50521083854417176e-07);
    q21 = fma(q21, x, -2.08767569878681002e-08);
    q0 = fma(q0, x, 2.75573192239858925e-06);
    q1 = fma(q1, x, 2.48015873015873016e-06);
    q21 = fma(q21, x, -2.25468975468975469e-07);
    q0 = fma(q0, x, 2.48015873015873016e-05);
    q1 = fma(q1, x, 2.20458553791887140e-05);
    q21 = fma(q21, x, -2.20458553791887106e-06);
    q0 = fma(q0, x, 1.98412698412698413e-04);
    q1 = fma(q1, x, 1.73611111111111118e-04);
    q21 = fma(q21, x, -1.92901234567901231e-05);
    q0 = fma(q0, x, 1.38888888888888894e-03);
    q1 = fma(q1, x, 1.19047619047619058e-03);
    q21 = fma(q21, x, -1.48809523809523823e-04);
    q0 = fma(q0, x, 8.33333333333333322e-03);
    q1 = fma(q1, x, 6.94444444444444406e-03);
    q21 = fma(q21, x, -9.92063492063492008e-04);
    q0 = fma(q0, x, 4.16666666666666644e-02);
    q1 = fma(q1, x, 3.33333333333333329e-02);
    q21 = fma(q21, x, -5.55555555555555577e-03);
    q0 = fma(q0, x, 1.66666666666666657e-01);
    q1 = fma(q1, x, 1.25000000000000000e-01);
    q21 = fma(q21, x, -2.50000000000000014e-02);
    q0 = fma(q0, x, 5.00000000000000000e-01);
    q1 = fma(q1, x, 3.33333333333333315e-01);
    q21 = fma(q21, x, -8.33333333333333287e-02);
    q0 = fma(q0, x, 1.00000000000000000e+00);
    q1 = fma(q1, x, 5.00000000000000000e-01);
    q21 = fma(q21, x, -1.66666666666666657e-01);
    w0 = du * q0;
    e = exp(-du);
    gam = du * (du * (q1 + q21) + dd * q1) / (du + dd);
    alp = du * du * du * q21 / (dd * (du + dd));
  } else {
    e = exp(-du);
    w0 = -expm1(-du);
    const double w1 = w0 - du * e;
    const double w2 = 2.0 * w1 - du * du * e;
    gam = (w2 + dd * w1) / (du * (du + dd));
    alp = (w2 - du * w1) / (dd * (du + dd));
  }
  c = w0 * S_loc + gam * (S_up - S_loc) + alp * (S_dn - S_loc);
}

__device__ __forceinline__ double sc_para_d(double I, double dtau_u, double dtau_d, double S_up,
                                            double S_loc, double S_dn, double mu) {
  double e, c;
  sc_para_coef_d(dtau_u, dtau_d, S_up, S_loc, S_dn, mu, e, c);
  return e * I + c;
}

// ------------------------------------------------------------ column kernel
// Angle tiers compiled: up to 3 angles (registers for exactly 3), else up
// to 8.  A request runs the kernel of its tier.
constexpr int kMuTierSmall = 3;

// Occupancy floor per instantiation: the FP32 parabolic sweep with an exact
// species count and the small angle tier fits in 72 VGPRs (7 waves per SIMD)
// without spilling when asked to, where the compiler otherwise takes 73-74
// (6 waves).  The linear sweep over exactly 8 species in the small angle tier
// takes 62-63 VGPRs but 102 SGPRs, which holds it to 7 waves per SIMD (SGPRs
// are allocated in blocks of 16 from 800 per SIMD); asked for 8 it fits in
// 78 SGPRs without spilling, so that four 8-wave workgroups of tile pairs fit
// on a CU.  Everything else keeps the compiler's choice.
template <typename Real, int NSS, int MAXMU, bool PARA>
constexpr int column_min_waves() {
  if (std::is_same<Real, double>::value || NSS >= 0 || MAXMU > kMuTierSmall) return 1;
  if (PARA) return 7;
  return NSS == -8 ? 8 : 1;
}


// Workgroup = C waves over one 64-point tile of one set; wave c sweeps layer
// chunk c: stage 1 (opacity, Sect. 2.3) from the slot registers, dtau
// (trapezoid over the layer), Planck, and the recurrence for every angle.
// Even chunks go bottom to top; odd chunks compose their layers' maps top
// down, so neighbouring chunks read the rows of their shared boundary level
// at about the same time.  Then the chunks' affine maps are combined through
// LDS and Eq. 8 applied.
// BIG: the table spans 4 GiB or more, so each species gets its own buffer
// resource; otherwise one resource covers the table and the species offset
// rides in the scalar offset operand.
// NS: species slots compiled; a negative NS means exactly -NS species (no
// per-species guards), otherwise tv.S <= NS species with uniform guards.
// PARA: parabolic source (each step also needs the downwind level, so a
// chunk below the top reads one level past its end).
// STREAM: the table rows are loaded non-temporal.  For launches of one set,
// whose rows are read once: the row stream (376 MB at C2) then no longer
// flushes the small working set of the neighbouring kernels (records, layout
// weights, F+) from the caches.  Batches share rows across sets through the
// caches and keep the default policy.
template <typename Real, typename TT, int NSS, int MAXMU, bool FROM_CHI, bool BIG, bool PARA,
          bool STREAM>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(
    column_min_waves<Real, NSS, MAXMU, PARA>()))) void k_column(TableView tv, const ColSeg *__restrict__ segs,
                                                int n_segs, ColSeg seg0, int64_t total_wgs,
                                                const void *__restrict__ recs_v,
                                                const void *__restrict__ chi_in_v,
                                                void *__restrict__ out_v) {
  using Rec = typename RecOf<Real>::type;
  constexpr bool kF64 = std::is_same<Real, double>::value;
  constexpr int NS = NSS < 0 ? -NSS : NSS;
  constexpr bool kExact = NSS < 0;
  // small angle tier: every one of the MAXMU slots runs (the angle table
  // pads a row past its n_mu nodes with mu = 1 and weight 0, so the extra
  // slots add exactly zero to F), and the loops carry no per-angle guards
  constexpr bool kAllMu = MAXMU <= kMuTierSmall;
  const Rec *__restrict__ recs = (const Rec *)recs_v;
  const Real *__restrict__ chi_in = (const Real *)chi_in_v;
  Real *__restrict__ out = (Real *)out_v;
  // chunk c's affine map (per angle: B, then the chunk's optical depth)
  extern __shared__ unsigned char sh_raw[];
  Real *sh = (Real *)sh_raw;

  const int64_t g = xcd_remap(blockIdx.x, total_wgs);
  // n_segs == 0: the launch is the one segment passed by value; otherwise
  // the segment holding workgroup g: last one with wg_begin <= g (ascending)
  int sg = 0;
  for (int lo = 0, hi = n_segs; hi - lo > 1;) {
    const int mid = (lo + hi) >> 1;
    if (segs[mid].wg_begin <= g) lo = mid;
    else hi = mid;
    sg = lo;
  }
  const ColSeg d = n_segs == 0 ? seg0 : segs[sg];
  const int n_sets = d.n_sets;
  // the wave index is uniform across a wavefront; say so, so that everything
  // derived from it (chunk, levels, records, load masks) stays scalar
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  int C = blockDim.x >> 6;   // one wave per layer chunk (the segment's chunks)
  int chunk = wave, grp = 0;
  int64_t t;
  int s;
  if (n_segs == 0 && d.wg_multi > 0) {
    // tile groups (one set): XCD x's tiles are [t0, t0 + q + (x < r))
    const int x = blockIdx.x & 7;
    const int64_t k = blockIdx.x >> 3;
    const int64_t q = d.tiles_per_set >> 3, r = d.tiles_per_set & 7;
    const int64_t t0 = x * q + (x < r ? x : r);
    const int G = d.tiles_per_wg;
    if (k < d.wg_multi) {
      C /= G;
      grp = wave / C;
      chunk = wave - grp * C;
      t = t0 + G * k + grp;
    } else {
      t = t0 + (int64_t)(G - 1) * d.wg_multi + k;
    }
    s = 0;
  } else {
    const int64_t local = g - d.wg_begin;
    t = local / n_sets;
    s = (int)(local - t * n_sets);
  }
  // this wave's tile group in the combine area
  sh += grp * C * (MAXMU + 1) * 64;
  const int lane = threadIdx.x & 63;
  const int L = d.n_levels, nlay = L - 1;
  const int m = (nlay + C - 1) / C;
  const int l0 = chunk * m;
  const int l1 = min(l0 + m, nlay);
  const int64_t nu_count = d.nu_count;
  const int64_t j = t * 64 + lane;
  const bool active = j < nu_count;
  const int64_t jj = active ? j : nu_count - 1;
  const int64_t kidx = d.nu_begin + jj * d.nu_stride;
  const uint32_t kk = (uint32_t)kidx;
  const Rec *rec = recs + d.rec_offset + (int64_t)s * L;
  const int nmu = d.n_mu;

  const double nu_d = tv.nu0 + (double)kidx * tv.dnu;
  const double c1nu3_d = kC1 * nu_d * nu_d * nu_d;
  const float nu_hi = (float)nu_d;
  const float nu_lo = (float)(nu_d - (double)nu_hi);
  // FP32: the sweep carries source and intensities in units of the lane's
  // Planck prefactor c1 nu^3 (the transfer is linear in them), which
  // multiplies the flux once at the end: one multiply and one register fewer
  // per level

  // per-species and per-pair base pointers (uniform) and this lane's byte
  // offset in a row: each load is base + (row offset + lane offset)
  const int64_t sp_bytes = (int64_t)tv.nT * tv.nP * tv.pitch * (int64_t)sizeof(TT);
  const int64_t pair_bytes = (int64_t)tv.nT * tv.pitch * (int64_t)sizeof(Real);
  const char *tab = (const char *)tv.tab;
  const char *cia = (const char *)tv.cia;
  rsrc_t rs[BIG ? NS : 1];
  if constexpr (BIG) {
#pragma unroll
    for (int q = 0; q < NS; ++q) rs[q] = make_rsrc(tab + q * sp_bytes, sp_bytes);
  } else {
    rs[0] = make_rsrc(tab, sp_bytes * tv.S);
  }
  const rsrc_t rc = make_rsrc(cia, 2 * pair_bytes);
  const uint32_t kb = kk * (uint32_t)sizeof(TT);
  const int S = kExact ? NS : tv.S;
  const bool has_cia = tv.n_cia > 0;

  Real slot[NS][4];
  Real cslot[2][2];
#pragma unroll
  for (int q = 0; q < NS; ++q)
#pragma unroll
    for (int k = 0; k < 4; ++k) slot[q][k] = (Real)0;
#pragma unroll
  for (int q = 0; q < 2; ++q) cslot[q][0] = cslot[q][1] = (Real)0;

  Real I[MAXMU];
  float a_mu[MAXMU], a_inv[MAXMU], a_l2e[MAXMU];
  double a_mud[MAXMU];
#pragma unroll
  for (int k = 0; k < MAXMU; ++k) {
    I[k] = (Real)0;
    a_mu[k] = c_ang.mu[nmu - 1][k];
    a_inv[k] = c_ang.inv_mu[nmu - 1][k];
    a_l2e[k] = c_ang.l2e_mu[nmu - 1][k];
    a_mud[k] = kF64 ? c_ang.mu_d[nmu - 1][k] : 0.0;
  }
  // a chunk's first level is the boundary it shares with the chunk that
  // starts there too (odd chunks sweep down, even ones up): its rows load
  // with the default policy, so the second wave's read finds them in the
  // cache.  So do the rows of the sweep's last kCachedTail levels: the
  // chunk that ends at the same boundary from the other side reaches rows
  // of the same (T, p) grid points at about the same time.  The levels
  // before follow the launch's policy (non-temporal for one-set launches
  // whose rows overflow the cache); caching every level was slower.  Only
  // such launches split the sweep in two loops: where both policies are the
  // default one the split only cost time (2-byte rows lost 20-30 %, although
  // both copies compiled to loops of the same length without spills).
  using kLoopPol = std::integral_constant<int, STREAM ? kCpolStream : 0>;
  using kFirstPol = std::integral_constant<int, 0>;
  constexpr int kCachedTail = 16;
  Real tau = (Real)0, chi_prev = (Real)0, S_prev = (Real)0, hdz_prev = (Real)0,
       dtc_prev = (Real)0;
  Real S_pp = (Real)0, dtau_last = (Real)0;   // parabolic: level l-2, layer l-2 -> l-1
  // last level visited: the chunk's top, or one more for the parabolic
  // step's downwind level when the chunk is not the topmost
  const int l_end = (PARA && l1 < nlay) ? l1 + 1 : l1;

  // Fetch the rows a level needs that the slots do not hold yet.  The rows
  // of level l+1 are requested right after level l's opacity is formed (its
  // slot values are no longer needed), so the loads are in flight while
  // level l's Planck function and RT update run.
  auto fetch = [&](const Rec &rr, int mask, auto pol) {
    constexpr int kPol = decltype(pol)::value;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (mask & (1 << k)) {
        const uint32_t off = rr.rowb[k] + kb;
#pragma unroll
        for (int q = 0; q < NS; ++q) {
          if (q < S) {
            const TT v = BIG ? buf_load<TT, kPol>(rs[BIG ? q : 0], off, 0)
                             : buf_load<TT, kPol>(rs[0], off, (uint32_t)(q * sp_bytes));
            if constexpr (kF64)
              slot[q][k] = (Real)v;
            else
              slot[q][k] = to_float<TT>(v);
          }
        }
      }
    }
    if (has_cia) {
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        if (mask & (16 << k)) {
          const uint32_t off = rr.cia_rowb[k] + cia_offset_from_row_offset<TT, Real>(kb);
          cslot[0][k] = buf_load<Real>(rc, off, 0);
          cslot[1][k] = buf_load<Real>(rc, off, (uint32_t)pair_bytes);
        }
      }
    }
  };

  // stage 1 at one level: chi from the slot rows (or read back from memory)
  auto opacity = [&](const Rec &r, int l) -> Real {
    if constexpr (FROM_CHI) {
      return chi_in[d.chi_offset + (int64_t)l * nu_count + jj];
    } else {
      Real chi = (Real)0;
#pragma unroll
      for (int q = 0; q < NS; ++q) {
        if (q < S) {
          const Real y = r.w[0] * slot[q][0] + r.w[1] * slot[q][1] + r.w[2] * slot[q][2] +
                         r.w[3] * slot[q][3];
          if constexpr (kF64)
            chi += r.a_s[q] * exp2(y);
          else
            chi = fmaf(r.a_s[q], fexp2(y), chi);
        }
      }
      if (has_cia) {
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          const Real y = r.cia_w[0] * cslot[q][0] + r.cia_w[1] * cslot[q][1];
          if constexpr (kF64)
            chi += r.a_cia[q] * exp2(y);
          else
            chi = fmaf(r.a_cia[q], fexp2(y), chi);
        }
      }
      return chi;
    }
  };
  auto source = [&](const Rec &r) -> Real {
    if constexpr (kF64)
      return planck_d(nu_d, c1nu3_d, r.T);
    else
      return planck_f(nu_hi, nu_lo, 1.0f, r.pl_hi, r.pl_lo);
  };

  // Odd chunks compose their layers' maps from the top down, so that the
  // rows at each chunk boundary are read by the two chunks that share it at
  // about the same time (the second read is an L2 hit) instead of at
  // opposite ends of the sweep.  With the parabolic source the sweep starts
  // at l_end, the downwind level of the chunk's top layer.
  const bool down = (chunk & 1) != 0;
  if (down && l0 < nlay) {
    if constexpr (!FROM_CHI) fetch(rec[l_end], rec[l_end].mask >> 8, kFirstPol{});
    Real A[MAXMU];   // transmission of the layers composed so far
#pragma unroll
    for (int k = 0; k < MAXMU; ++k) A[k] = (Real)1;
    // the sweep's cached tail runs in a loop of its own
    auto down_level = [&](int l, auto pol) {
      const Rec r = rec[l];
      const Real chi = opacity(r, l);
      if constexpr (!FROM_CHI) {
        if (l > l0) {
          const Rec &rn = rec[l - 1];
          asm volatile("" ::: "memory");
          fetch(rn, rn.mask >> 16, pol);
        }
      }
      const Real Sl = source(r);
      if (l < l_end) {
        // layer l -> l+1: lower level l (S0 = Sl), upper level l+1 (S1 = S_prev)
        const Real dtau = (chi + chi_prev) * r.hdz + r.dtc;
        if constexpr (!PARA) {
          tau += dtau;
          if constexpr (kF64) {
#pragma unroll
            for (int k = 0; k < MAXMU; ++k)
              if (kAllMu || k < nmu) {
                double e, c;
                sc_coef_d(dtau, S_prev, Sl, a_mud[k], e, c);
                I[k] = fma(A[k], c, I[k]);
                A[k] *= e;
              }
          } else {
            const float D = Sl - S_prev, rD = D * frcp(dtau);
#pragma unroll
            for (int k = 0; k < MAXMU; ++k)
              if (kAllMu || k < nmu) {
                float e, uD;
                sc_coef_f(dtau, rD, D, a_inv[k], a_l2e[k], a_mu[k], e, uD);
                I[k] = fmaf(A[k], fmaf(-e, Sl, S_prev) + uD, I[k]);
                A[k] *= e;
              }
          }
        } else {
          if (l < l1) {
            tau += dtau;
            // upwind level l, local l+1, downwind l+2 (S_pp, across the layer
            // of optical depth dtau_last) once the sweep has been there; a
            // transparent downwind layer leaves the linear coefficients
            const bool has_dn = l + 2 <= l_end;
            if constexpr (kF64) {
#pragma unroll
              for (int k = 0; k < MAXMU; ++k)
                if (kAllMu || k < nmu) {
                  double e, c;
                  if (has_dn && dtau_last > 0.0)
                    sc_para_coef_d(dtau, dtau_last, Sl, S_prev, S_pp, a_mud[k], e, c);
                  else
                    sc_coef_d(dtau, S_prev, Sl, a_mud[k], e, c);
                  I[k] = fma(A[k], c, I[k]);
                  A[k] *= e;
                }
            } else {
              const float r_u = frcp(dtau), r_d = frcp(dtau_last),
                          r_s = frcp(dtau + dtau_last);
              const bool para = has_dn && dtau_last > 0.0f;
#pragma unroll
              for (int k = 0; k < MAXMU; ++k)
                if (kAllMu || k < nmu) {
                  float e, c;
                  if (para)
                    sc_para_coef_f(dtau, dtau_last, r_u, r_d, r_s, Sl, S_prev, S_pp, a_inv[k],
                                   a_l2e[k], a_mu[k], e, c);
                  else
                    sc_weights_coef_f(dtau, r_u, S_prev, Sl, a_inv[k], a_l2e[k], a_mu[k], e, c);
                  I[k] = fmaf(A[k], c, I[k]);
                  A[k] *= e;
                }
            }
          }
          S_pp = S_prev;
          dtau_last = dtau;
        }
      }
      chi_prev = chi;
      S_prev = Sl;
    };
    int l = l_end;
    if constexpr (STREAM)
      for (; l >= l0 + kCachedTail; --l) down_level(l, kLoopPol{});
    for (; l >= l0; --l) down_level(l, kFirstPol{});
  } else if (l0 < nlay) {
    if constexpr (!FROM_CHI) fetch(rec[l0], rec[l0].mask >> 8, kFirstPol{});
    auto up_level = [&](int l, auto pol) {
      const Rec r = rec[l];
      const Real chi = opacity(r, l);
      if constexpr (!FROM_CHI) {
        if (l < l_end) {
          const Rec &rn = rec[l + 1];
          // keeps this fetch here, after the opacity, instead of being merged
          // with the chunk's first fetch at the top of the loop
          asm volatile("" ::: "memory");
          fetch(rn, rn.mask, pol);
        }
      }
      const Real S = source(r);
      if (l == l0) {
#pragma unroll
        for (int k = 0; k < MAXMU; ++k) I[k] = (chunk == 0) ? S : (Real)0;
      } else {
        // trapezoid of chi over the layer, plus its share of a gray cloud
        const Real dtau = (chi_prev + chi) * hdz_prev + dtc_prev;
        if constexpr (!PARA) {
          tau += dtau;
          if constexpr (kF64) {
#pragma unroll
            for (int k = 0; k < MAXMU; ++k)
              if (kAllMu || k < nmu) I[k] = sc_step_d(I[k], dtau, S, S_prev, a_mud[k]);
          } else {
            const float D = S_prev - S, rD = D * frcp(dtau);
#pragma unroll
            for (int k = 0; k < MAXMU; ++k)
              if (kAllMu || k < nmu)
                I[k] = sc_step_f(I[k], dtau, rD, S, S_prev, D, a_inv[k], a_l2e[k], a_mu[k]);
          }
        } else {
          if (l <= l1) tau += dtau;
          // the step l-2 -> l-1 now has its downwind level l; a transparent
          // downwind layer leaves the linear coefficients
          if (l >= l0 + 2) {
            if constexpr (kF64) {
#pragma unroll
              for (int k = 0; k < MAXMU; ++k)
                if (kAllMu || k < nmu)
                  I[k] = dtau > 0.0 ? sc_para_d(I[k], dtau_last, dtau, S_pp, S_prev, S, a_mud[k])
                                    : sc_step_d(I[k], dtau_last, S_prev, S_pp, a_mud[k]);
            } else {
              const float r_u = frcp(dtau_last), r_d = frcp(dtau), r_s = frcp(dtau_last + dtau);
#pragma unroll
              for (int k = 0; k < MAXMU; ++k)
                if (kAllMu || k < nmu)
                  I[k] = dtau > 0.0f
                             ? sc_para_f(I[k], dtau_last, dtau, r_u, r_d, r_s, S_pp, S_prev, S,
                                         a_inv[k], a_l2e[k], a_mu[k])
                             : sc_step_weights_f(I[k], dtau_last, r_u, S_prev, S_pp, a_inv[k],
                                                 a_l2e[k], a_mu[k]);
            }
          }
          S_pp = S_prev;
          dtau_last = dtau;
        }
      }
      chi_prev = chi;
      S_prev = S;
      hdz_prev = r.hdz;
      dtc_prev = r.dtc;
    };
    int l = l0;
    if constexpr (STREAM)
      for (; l + kCachedTail <= l_end; ++l) up_level(l, kLoopPol{});
    for (; l <= l_end; ++l) up_level(l, kFirstPol{});
    if constexpr (PARA) {
      // the topmost chunk's last step has no downwind level: linear
      if (l_end == l1 && l1 > l0) {
        if constexpr (kF64) {
#pragma unroll
          for (int k = 0; k < MAXMU; ++k)
            if (kAllMu || k < nmu) I[k] = sc_step_d(I[k], dtau_last, S_prev, S_pp, a_mud[k]);
        } else {
          const float r_u = frcp(dtau_last);
#pragma unroll
          for (int k = 0; k < MAXMU; ++k)
            if (kAllMu || k < nmu)
              I[k] = sc_step_weights_f(I[k], dtau_last, r_u, S_prev, S_pp, a_inv[k], a_l2e[k],
                                       a_mu[k]);
        }
      }
    }
  }

  // the lane id again (no register carries it across the sweep)
  const int lane_e = __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
  Real F = (Real)0;
  if (C == 1) {
#pragma unroll
    for (int k = 0; k < MAXMU; ++k)
      if (kAllMu || k < nmu) {
        if constexpr (kF64)
          F += c_ang.cw_d[nmu - 1][k] * I[k];
        else
          F = fmaf(c_ang.cw[nmu - 1][k], I[k], F);
      }
  } else {
    // layout (from the tile group's base): sh[(c * (MAXMU + 1) + k) * 64 + lane_e],
    // k = MAXMU holds tau
    sh[(chunk * (MAXMU + 1) + MAXMU) * 64 + lane_e] = tau;
#pragma unroll
    for (int k = 0; k < MAXMU; ++k) sh[(chunk * (MAXMU + 1) + k) * 64 + lane_e] = I[k];
    __syncthreads();
    if (chunk == C - 1) {
#pragma unroll
      for (int k = 0; k < MAXMU; ++k)
        if (kAllMu || k < nmu) {
          Real acc = sh[k * 64 + lane_e];
          for (int c = 1; c < C; ++c) {
            const Real tc = sh[(c * (MAXMU + 1) + MAXMU) * 64 + lane_e];
            Real tr;
            if constexpr (kF64)
              tr = exp(-tc / a_mud[k]);
            else
              tr = fexp2(-tc * a_l2e[k]);
            acc = tr * acc + sh[(c * (MAXMU + 1) + k) * 64 + lane_e];
          }
          if constexpr (kF64)
            F += c_ang.cw_d[nmu - 1][k] * acc;
          else
            F = fmaf(c_ang.cw[nmu - 1][k], acc, F);
        }
    }
  }
  // the lane's point again, from uniform values and the lane id
  const int64_t je = t * 64 + lane_e;
  if constexpr (!kF64) {
    const int64_t jje = je < nu_count ? je : nu_count - 1;
    const double nu_e = tv.nu0 + (double)(d.nu_begin + jje * d.nu_stride) * tv.dnu;
    F *= (float)(kC1 * nu_e * nu_e * nu_e);
  }
  if (je < nu_count && chunk == C - 1) out[d.out_offset + (int64_t)s * d.out_stride + je] = F;
}

int column_nu_per_wg(int) { return 64; }

using ColumnFn = void (*)(TableView, const ColSeg *, int, ColSeg, int64_t, const void *,
                          const void *, void *);
struct ColumnKernel {
  ColumnFn fn;
  int max_mu;
  int real_bytes;
};

template <typename Real, typename TT, int NS, int MAXMU, bool FROM_CHI, bool PARA, bool STREAM,
          bool BIG = false>
static ColumnKernel ck() {
  return ColumnKernel{&k_column<Real, TT, NS, MAXMU, FROM_CHI, BIG, PARA, STREAM>, MAXMU,
                      (int)sizeof(Real)};
}

int column_mu_class(int n_mu) { return n_mu > kMuTierSmall ? 8 : kMuTierSmall; }

template <typename Real, typename TT, bool FROM_CHI, bool PARA, bool STREAM>
static ColumnKernel pick_ns(const TableView &tv, int max_mu) {
  const int S = tv.S;
  if constexpr (FROM_CHI) {
    if (max_mu <= kMuTierSmall) return ck<Real, TT, 1, kMuTierSmall, true, PARA, false>();
    return ck<Real, TT, 1, 8, true, PARA, false>();
  } else {
    const int64_t table_bytes = (int64_t)tv.S * tv.nT * tv.nP * tv.pitch * (int64_t)sizeof(TT);
    if (table_bytes >= 0xFFFFFFFFll)
      return ck<Real, TT, kMaxSpecies, 8, false, PARA, false, true>();
    if (max_mu <= kMuTierSmall) {
      if (S <= 1) return ck<Real, TT, -1, kMuTierSmall, false, PARA, STREAM>();
      if (S == 8) return ck<Real, TT, -8, kMuTierSmall, false, PARA, STREAM>();
      if (S <= 8) return ck<Real, TT, 8, kMuTierSmall, false, PARA, STREAM>();
      return ck<Real, TT, kMaxSpecies, kMuTierSmall, false, PARA, STREAM>();
    }
    if (S <= 1) return ck<Real, TT, -1, 8, false, PARA, STREAM>();
    if (S <= 8) return ck<Real, TT, 8, 8, false, PARA, STREAM>();
    return ck<Real, TT, kMaxSpecies, 8, false, PARA, STREAM>();
  }
}

template <bool PARA, bool STREAM>
static ColumnKernel pick_dtype(const TableView &tv, int max_mu, bool from_chi) {
  if (from_chi) {
    if (tv.dtype == HR2_TABLE_F64) return pick_ns<double, double, true, PARA, false>(tv, max_mu);
    return pick_ns<float, float, true, PARA, false>(tv, max_mu);
  }
  switch (tv.dtype) {
    case HR2_TABLE_F64: return pick_ns<double, double, false, PARA, STREAM>(tv, max_mu);
    case HR2_TABLE_F16: return pick_ns<float, _Float16, false, PARA, STREAM>(tv, max_mu);
    case HR2_TABLE_BF16: return pick_ns<float, uint16_t, false, PARA, STREAM>(tv, max_mu);
    default: return pick_ns<float, float, false, PARA, STREAM>(tv, max_mu);
  }
}

// stream_rows: non-temporal row loads (from_chi reads no table rows)
static ColumnKernel pick_column(const TableView &tv, int max_mu, bool from_chi, bool para,
                                bool stream_rows) {
  if (stream_rows && !from_chi)
    return para ? pick_dtype<true, true>(tv, max_mu, false)
                : pick_dtype<false, true>(tv, max_mu, false);
  return para ? pick_dtype<true, false>(tv, max_mu, from_chi)
              : pick_dtype<false, false>(tv, max_mu, from_chi);
}

static size_t column_shmem(const ColumnKernel &k, int chunks) {
  return chunks > 1 ? (size_t)chunks * (k.max_mu + 1) * 64 * k.real_bytes : 0;
}

hipError_t launch_column(const TableView &tv, const ColSeg *segs_dev, int n_segs,
                         const ColSeg *seg0_host, int64_t total_wgs, int chunks, const void *recs,
                         const void *chi_in, void *out, int max_mu, bool opacity_from_memory,
                         bool para, bool stream_rows, hipStream_t stream, hipEvent_t t_start,
                         hipEvent_t t_stop) {
  if (total_wgs <= 0) return hipSuccess;
  const ColumnKernel k = pick_column(tv, max_mu, opacity_from_memory, para, stream_rows);
  const ColSeg seg0 = seg0_host ? *seg0_host : ColSeg{};
  const int ns = seg0_host ? 0 : n_segs;
  launch_timed(k.fn, dim3((unsigned)total_wgs), dim3(64 * chunks),
               (uint32_t)column_shmem(k, chunks), stream, t_start, t_stop, tv, segs_dev, ns, seg0,
               total_wgs, recs, chi_in, out);
  return hipGetLastError();
}

int column_wave_capacity(const TableView &tv, int max_mu, bool opacity_from_memory, int chunks,
                         bool para) {
  // the streaming variants differ only in the loads' cache policy
  const ColumnKernel k = pick_column(tv, max_mu, opacity_from_memory, para, false);
  int blocks = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, (const void *)k.fn, 64 * chunks,
                                                   column_shmem(k, chunks)) != hipSuccess ||
      blocks < 1) {
    (void)hipGetLastError();
    blocks = 1;
  }
  int dev = 0, n_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      n_cu < 1) {
    (void)hipGetLastError();
    n_cu = 1;
  }
  return blocks * chunks * n_cu;
}

// ------------------------------------------------------- stage 1 on its own
// chi_l(nu) for every (level, window point): one thread each, the four
// corner rows of the level's cell read directly (Sect. 2.3).
template <typename Real, typename TT>
__global__ __launch_bounds__(256) void k_opacity_only(TableView tv,
                                                      const typename RecOf<Real>::type *recs,
                                                      int64_t nu_begin, int64_t nu_count,
                                                      int64_t nu_stride, Real *chi) {
  constexpr bool kF64 = std::is_same<Real, double>::value;
  const int l = blockIdx.y;
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= nu_count) return;
  const auto &r = recs[l];
  const uint32_t kk = (uint32_t)(nu_begin + j * nu_stride);
  const int64_t sp_bytes = (int64_t)tv.nT * tv.nP * tv.pitch * (int64_t)sizeof(TT);
  const char *tab = (const char *)tv.tab;
  Real c = (Real)0;
  for (int q = 0; q < tv.S; ++q) {
    const char *base = tab + q * sp_bytes;
    Real y = (Real)0;
    for (int k = 0; k < 4; ++k) {
      const TT e = *(const TT *)(base + r.rowb[k] + kk * (uint32_t)sizeof(TT));
      Real v;
      if constexpr (kF64)
        v = (Real)e;
      else
        v = to_float<TT>(e);
      y += r.w[k] * v;
    }
    if constexpr (kF64)
      c += r.a_s[q] * exp2(y);
    else
      c = fmaf(r.a_s[q], fexp2(y), c);
  }
  const char *cia = (const char *)tv.cia;
  const int64_t pair_bytes = (int64_t)tv.nT * tv.pitch * (int64_t)sizeof(Real);
  for (int q = 0; q < tv.n_cia; ++q) {
    const char *cbase = cia + q * pair_bytes;
    const uint32_t kc = kk * (uint32_t)sizeof(Real);
    const Real y = r.cia_w[0] * *(const Real *)(cbase + r.cia_rowb[0] + kc) +
                   r.cia_w[1] * *(const Real *)(cbase + r.cia_rowb[1] + kc);
    if constexpr (kF64)
      c += r.a_cia[q] * exp2(y);
    else
      c = fmaf(r.a_cia[q], fexp2(y), c);
  }
  chi[(int64_t)l * nu_count + j] = c;
}

hipError_t launch_opacity_only(const TableView &tv, const void *recs, int n_levels,
                               int64_t nu_begin, int64_t nu_count, int64_t nu_stride, void *chi,
                               hipStream_t stream) {
  const dim3 grid((unsigned)((nu_count + 255) / 256), (unsigned)n_levels);
  switch (tv.dtype) {
    case HR2_TABLE_F64:
      hipLaunchKernelGGL((k_opacity_only<double, double>), grid, dim3(256), 0, stream, tv,
                         (const LevelRecD *)recs, nu_begin, nu_count, nu_stride, (double *)chi);
      break;
    case HR2_TABLE_F16:
      hipLaunchKernelGGL((k_opacity_only<float, _Float16>), grid, dim3(256), 0, stream, tv,
                         (const LevelRecF *)recs, nu_begin, nu_count, nu_stride, (float *)chi);
      break;
    case HR2_TABLE_BF16:
      hipLaunchKernelGGL((k_opacity_only<float, uint16_t>), grid, dim3(256), 0, stream, tv,
                         (const LevelRecF *)recs, nu_begin, nu_count, nu_stride, (float *)chi);
      break;
    default:
      hipLaunchKernelGGL((k_opacity_only<float, float>), grid, dim3(256), 0, stream, tv,
                         (const LevelRecF *)recs, nu_begin, nu_count, nu_stride, (float *)chi);
  }
  return hipGetLastError();
}

// ------------------------------------------------------ convolution + bins
// bin_j = scale * sum_m K_j[m] F+[m] over the bin's support (Eq. 9, 17 and
// the binning, composed into one banded row per bin).  A layout whose
// supports average 512 points or more gets four waves per (set, bin), a
// shorter one one wave per (set, bin) (four per workgroup).  Either way
// lane-strided partial sums then a fixed butterfly, and the scheme depends
// on the layout alone: a bin's value does not depend on what else is in the
// launch.
int conv_items_per_wg(int64_t nnz, int n_bins) {
  return n_bins > 0 && nnz < (int64_t)512 * n_bins ? 4 : 1;
}

int64_t conv_workgroups(int64_t n_items, int items_per_wg) {
  return (n_items + items_per_wg - 1) / items_per_wg;
}

// One thread's share of a support of len points: the item's WIDTH threads
// stride it, four independent partial sums per thread so that a round's
// loads are in flight together.
template <typename Real, int WIDTH>
__device__ __forceinline__ Real conv_partial(const Real *__restrict__ K,
                                             const Real *__restrict__ F, int len, int q) {
  Real a0 = (Real)0, a1 = (Real)0, a2 = (Real)0, a3 = (Real)0;
  for (; q + 3 * WIDTH < len; q += 4 * WIDTH) {
    const Real k0 = K[q], k1 = K[q + WIDTH], k2 = K[q + 2 * WIDTH], k3 = K[q + 3 * WIDTH];
    const Real f0 = F[q], f1 = F[q + WIDTH], f2 = F[q + 2 * WIDTH], f3 = F[q + 3 * WIDTH];
    a0 += k0 * f0;
    a1 += k1 * f1;
    a2 += k2 * f2;
    a3 += k3 * f3;
  }
  if (q < len) a0 += K[q] * F[q];
  if (q + WIDTH < len) a1 += K[q + WIDTH] * F[q + WIDTH];
  if (q + 2 * WIDTH < len) a2 += K[q + 2 * WIDTH] * F[q + 2 * WIDTH];
  return (a0 + a1) + (a2 + a3);
}

template <typename Real>
__global__ __launch_bounds__(256) void k_convolve_bin(const ConvSeg *__restrict__ segs,
                                                      int n_segs, ConvSeg seg0,
                                                      int64_t total_wgs,
                                                      const Real *__restrict__ in,
                                                      Real *__restrict__ out) {
  __shared__ Real part[4];
  const int64_t g = blockIdx.x;
  int sg = 0;
  for (int lo = 0, hi = n_segs; hi - lo > 1;) {
    const int mid = (lo + hi) >> 1;
    if (segs[mid].item_begin <= g) lo = mid;
    else hi = mid;
    sg = lo;
  }
  const ConvSeg d = n_segs == 0 ? seg0 : segs[sg];   // n_segs == 0: the one segment by value
  const bool per_wave = d.items_per_wg == 4;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int64_t local = per_wave ? (g - d.item_begin) * 4 + wave : g - d.item_begin;
  if (per_wave && local >= (int64_t)d.n_sets * d.n_bins) return;
  const int s = (int)(local / d.n_bins);
  const int jb = (int)(local - (int64_t)s * d.n_bins);
  const Real *K = (const Real *)d.K + d.kstart[jb];
  const int len = d.mlen[jb];
  const Real *F = in + d.in_offset + (int64_t)s * d.in_stride + d.mlo[jb];
  // what the storing thread needs after the reduction, requested now so
  // that it arrives with the data
  const bool storer = per_wave ? lane == 0 : threadIdx.x == 0;
  double sc = d.scale_const, Dj = 0.0, s2 = 0.0, l10e = 0.0;
  if (storer) {
    if (d.scale) sc = d.scale[s];
    if (d.terms) {
      Dj = d.D[jb];
      s2 = d.s2[jb];
      if (d.log10_eps) l10e = d.log10_eps[s];
    }
  }
  Real acc = per_wave ? conv_partial<Real, 64>(K, F, len, lane)
                      : conv_partial<Real, 256>(K, F, len, (int)threadIdx.x);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if (!per_wave) {
    if (lane == 0) part[wave] = acc;
    __syncthreads();
    acc = (part[0] + part[1]) + (part[2] + part[3]);
  }
  if (storer) {
    const Real v = acc * (Real)sc;
    if (out) out[d.out_offset + (int64_t)s * d.n_bins + jb] = v;
    if (d.terms) {
      // Eq. 19 term of bin j in FP64; with Eq. 22 the variance gains 10^eps
      if (d.log10_eps) s2 += exp10(l10e);
      const double r = Dj - (double)v;
      d.terms[(int64_t)s * d.n_bins + jb] = -r * r / (2.0 * s2) - 0.5 * log(kTwoPi * s2);
    }
  }
}

hipError_t launch_convolve_bin(bool fp64, const ConvSeg *segs_dev, int n_segs,
                               const ConvSeg *seg0_host, int64_t total_wgs, const void *in,
                               void *out, hipStream_t stream, hipEvent_t t_start,
                               hipEvent_t t_stop) {
  if (total_wgs <= 0) return hipSuccess;
  const dim3 grid((unsigned)total_wgs);
  const ConvSeg seg0 = seg0_host ? *seg0_host : ConvSeg{};
  const int ns = seg0_host ? 0 : n_segs;
  if (fp64)
    launch_timed(k_convolve_bin<double>, grid, dim3(256), 0u, stream, t_start, t_stop, segs_dev,
                 ns, seg0, total_wgs, (const double *)in, (double *)out);
  else
    launch_timed(k_convolve_bin<float>, grid, dim3(256), 0u, stream, t_start, t_stop, segs_dev,
                 ns, seg0, total_wgs, (const float *)in, (float *)out);
  return hipGetLastError();
}

// ------------------------------------------- whole forward model per set
// Small windows in large batches (the sampler's many live points on a short
// spectral range): one workgroup per set runs the whole forward model in
// one launch.  It builds the set's level records in LDS (the same items as
// k_levels), sweeps every 64-point tile of the window with the fused
// opacity + short-characteristics recurrence (one layer chunk; waves take
// tiles in turn), keeps F+ in LDS (and writes it out), then forms the set's
// bins one wave per bin from LDS.  The arithmetic is that of k_column with
// one chunk and of k_convolve_bin's one-wave-per-bin scheme, step for step.
constexpr int kSetThreads = 1024;
constexpr int kSetMaxLevels = 64;
// one thread per level item (one species, up to two CIA pairs)
static_assert(kSetMaxLevels * (2 + 1 + HR2_MAX_CIA) <= kSetThreads, "level items per thread");
constexpr int kSetMaxNu = 4096;

// NU wavenumbers per lane (1 or 2): a wave's tile is 64 NU points, lane j
// holding points j, j + 64, ...; the NU recurrences of a lane are
// independent, which gives the wave more work between its row loads.
template <typename TT, int NSS, int MAXMU, int NU>
__global__ __launch_bounds__(kSetThreads) __attribute__((amdgpu_waves_per_eu(8))) void k_set_forward(
    TableView tv, ColumnsView cv, SetFwdArgs a) {
  using Rec = LevelRecF;
  constexpr int NS = NSS < 0 ? -NSS : NSS;
  constexpr bool kExact = NSS < 0;
  __shared__ Rec s_rec[kSetMaxLevels];
  __shared__ float s_fp[kSetMaxNu];
  __shared__ float s_scale;   // the set's scale, for the bins (kept out of registers)
  const int s = blockIdx.x;
  const int L = cv.L;
  if (threadIdx.x == 0) s_scale = (float)cv.scale[s];
  level_records<float>(tv, cv, s, 0, 1, s_rec, a.status, ThetaArgs{});
  __syncthreads();

  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int n_waves = blockDim.x >> 6;
  const int64_t nu_count = a.nu_count;
  const int tiles = (int)((nu_count + 64 * NU - 1) / (64 * NU));
  const int nmu = a.n_mu;
  const int64_t sp_bytes = (int64_t)tv.nT * tv.nP * tv.pitch * (int64_t)sizeof(TT);
  const int64_t pair_bytes = (int64_t)tv.nT * tv.pitch * (int64_t)sizeof(float);
  const rsrc_t rs = make_rsrc(tv.tab, sp_bytes * tv.S);
  const rsrc_t rc = make_rsrc(tv.cia, 2 * pair_bytes);
  const int S = kExact ? NS : tv.S;
  const bool has_cia = tv.n_cia > 0;
  float a_mu[MAXMU], a_inv[MAXMU], a_l2e[MAXMU];
#pragma unroll
  for (int k = 0; k < MAXMU; ++k) {
    a_mu[k] = c_ang.mu[nmu - 1][k];
    a_inv[k] = c_ang.inv_mu[nmu - 1][k];
    a_l2e[k] = c_ang.l2e_mu[nmu - 1][k];
  }

  for (int t = wave; t < tiles; t += n_waves) {
    float nu_hi[NU], nu_lo[NU];
    uint32_t kb[NU];
#pragma unroll
    for (int u = 0; u < NU; ++u) {
      const int64_t j = (int64_t)t * (64 * NU) + u * 64 + lane;
      const int64_t jj = j < nu_count ? j : nu_count - 1;
      const int64_t kidx = a.nu_begin + jj * a.nu_stride;
      const uint32_t kk = (uint32_t)kidx;
      const double nu_d = tv.nu0 + (double)kidx * tv.dnu;
      nu_hi[u] = (float)nu_d;
      nu_lo[u] = (float)(nu_d - (double)nu_hi[u]);
      kb[u] = kk * (uint32_t)sizeof(TT);
    }
    float slot[NU][NS][4];
    float cslot[NU][2][2];
#pragma unroll
    for (int u = 0; u < NU; ++u) {
#pragma unroll
      for (int q = 0; q < NS; ++q)
#pragma unroll
        for (int k = 0; k < 4; ++k) slot[u][q][k] = 0.0f;
#pragma unroll
      for (int q = 0; q < 2; ++q) cslot[u][q][0] = cslot[u][q][1] = 0.0f;
    }
    auto fetch = [&](const Rec &rr, int mask) {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        if (mask & (1 << k)) {
#pragma unroll
          for (int u = 0; u < NU; ++u) {
            const uint32_t off = rr.rowb[k] + kb[u];
#pragma unroll
            for (int q = 0; q < NS; ++q)
              if (q < S)
                slot[u][q][k] = to_float<TT>(buf_load<TT>(rs, off, (uint32_t)(q * sp_bytes)));
          }
        }
      }
      if (has_cia) {
#pragma unroll
        for (int k = 0; k < 2; ++k) {
          if (mask & (16 << k)) {
#pragma unroll
            for (int u = 0; u < NU; ++u) {
              const uint32_t off = rr.cia_rowb[k] + cia_offset_from_row_offset<TT>(kb[u]);
              cslot[u][0][k] = buf_load<float>(rc, off, 0);
              cslot[u][1][k] = buf_load<float>(rc, off, (uint32_t)pair_bytes);
            }
          }
        }
      }
    };
    auto opacity = [&](const Rec &r, int u) -> float {
      float chi = 0.0f;
#pragma unroll
      for (int q = 0; q < NS; ++q) {
        if (q < S) {
          const float y = r.w[0] * slot[u][q][0] + r.w[1] * slot[u][q][1] +
                          r.w[2] * slot[u][q][2] + r.w[3] * slot[u][q][3];
          chi = fmaf(r.a_s[q], fexp2(y), chi);
        }
      }
      if (has_cia) {
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          const float y = r.cia_w[0] * cslot[u][q][0] + r.cia_w[1] * cslot[u][q][1];
          chi = fmaf(r.a_cia[q], fexp2(y), chi);
        }
      }
      return chi;
    };
    float I[NU][MAXMU];
    float chi_prev[NU], S_prev[NU];
    float hdz_prev = 0.0f, dtc_prev = 0.0f;
#pragma unroll
    for (int u = 0; u < NU; ++u) chi_prev[u] = S_prev[u] = 0.0f;
    fetch(s_rec[0], __builtin_amdgcn_readfirstlane(s_rec[0].mask) >> 8);
    for (int l = 0; l < L; ++l) {
      const Rec r = s_rec[l];
      float chi[NU];
#pragma unroll
      for (int u = 0; u < NU; ++u) chi[u] = opacity(r, u);
      if (l + 1 < L) {
        const Rec &rn = s_rec[l + 1];
        asm volatile("" ::: "memory");
        fetch(rn, __builtin_amdgcn_readfirstlane(rn.mask));
      }
#pragma unroll
      for (int u = 0; u < NU; ++u) {
        // in units of c1 nu^3, as in k_column
        const float Sl = planck_f(nu_hi[u], nu_lo[u], 1.0f, r.pl_hi, r.pl_lo);
        if (l == 0) {
#pragma unroll
          for (int k = 0; k < MAXMU; ++k) I[u][k] = Sl;
        } else {
          // trapezoid of chi over the layer, plus its share of a gray cloud
          const float dtau = (chi_prev[u] + chi[u]) * hdz_prev + dtc_prev;
          const float D = S_prev[u] - Sl, rD = D * frcp(dtau);
#pragma unroll
          for (int k = 0; k < MAXMU; ++k)
            if (k < nmu)
              I[u][k] = sc_step_f(I[u][k], dtau, rD, Sl, S_prev[u], D, a_inv[k], a_l2e[k], a_mu[k]);
        }
        chi_prev[u] = chi[u];
        S_prev[u] = Sl;
      }
      hdz_prev = r.hdz;
      dtc_prev = r.dtc;
    }
    // the lane's points again, from the tile and the lane id (no register
    // carries them across the sweep)
    const int lane_e = __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
#pragma unroll
    for (int u = 0; u < NU; ++u) {
      float F = 0.0f;
#pragma unroll
      for (int k = 0; k < MAXMU; ++k)
        if (k < nmu) F = fmaf(c_ang.cw[nmu - 1][k], I[u][k], F);
      const int64_t j = (int64_t)t * (64 * NU) + u * 64 + lane_e;
      {
        const int64_t jj = j < nu_count ? j : nu_count - 1;
        const double nu_d = tv.nu0 + (double)(a.nu_begin + jj * a.nu_stride) * tv.dnu;
        F *= (float)(kC1 * nu_d * nu_d * nu_d);
      }
      if (j < nu_count) {
        s_fp[j] = F;
        a.fplus[(int64_t)s * nu_count + j] = F;
      }
    }
  }
  __syncthreads();

  // Eq. 17 and the binning: one wave per bin, as k_convolve_bin's short-
  // support scheme, from the F+ in LDS
  const float sc = s_scale;
  for (int jb = wave; jb < a.n_bins; jb += n_waves) {
    float acc = conv_partial<float, 64>(a.K + a.kstart[jb], s_fp + a.mlo[jb], a.mlen[jb], lane);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if (lane == 0) a.bins[(int64_t)s * a.n_bins + jb] = acc * sc;
  }
}

// Variants: one species (C1-like tables), one or two wavenumbers per lane.
// With more species the sweep's slot rows and the record items no longer
// fit the 64 registers of two 1,024-thread workgroups per CU without
// spilling inside the sweep, so those batches keep the three kernels.
template <typename TT, int MAXMU>
static bool set_forward_kernel(int S, int nu_per_lane,
                               void (**fn)(TableView, ColumnsView, SetFwdArgs)) {
  if (S != 1) return false;
  if (nu_per_lane == 2) *fn = &k_set_forward<TT, -1, MAXMU, 2>;
  else *fn = &k_set_forward<TT, -1, MAXMU, 1>;
  return true;
}

// Automatic: two per lane in the small angle tier; one in the large tier,
// where two would not fit the registers without spilling.
int set_forward_nu_per_lane(const TableView &, int requested, int max_mu) {
  if (requested == 1 || requested == 2) return requested;
  return max_mu <= kMuTierSmall ? 2 : 1;
}

bool set_forward_fits(const TableView &tv, int n_levels, int64_t nu_count) {
  return tv.dtype != HR2_TABLE_F64 && tv.S == 1 && n_levels <= kSetMaxLevels &&
         nu_count <= kSetMaxNu &&
         (int64_t)tv.nT * tv.nP * tv.pitch * tv.tab_elem * tv.S < 0xFFFFFFFFll;
}

hipError_t launch_set_forward(const TableView &tv, const ColumnsView &cv, const SetFwdArgs &args,
                              int max_mu, int nu_per_lane, hipStream_t stream, hipEvent_t t_start,
                              hipEvent_t t_stop) {
  if (cv.B <= 0) return hipSuccess;
  void (*fn)(TableView, ColumnsView, SetFwdArgs) = nullptr;
  bool ok;
  const bool small = max_mu <= kMuTierSmall;
  const int nl = set_forward_nu_per_lane(tv, nu_per_lane, max_mu);
  switch (tv.dtype) {
    case HR2_TABLE_F16:
      ok = small ? set_forward_kernel<_Float16, kMuTierSmall>(tv.S, nl, &fn)
                 : set_forward_kernel<_Float16, 8>(tv.S, nl, &fn);
      break;
    case HR2_TABLE_BF16:
      ok = small ? set_forward_kernel<uint16_t, kMuTierSmall>(tv.S, nl, &fn)
                 : set_forward_kernel<uint16_t, 8>(tv.S, nl, &fn);
      break;
    case HR2_TABLE_F32:
      ok = small ? set_forward_kernel<float, kMuTierSmall>(tv.S, nl, &fn)
                 : set_forward_kernel<float, 8>(tv.S, nl, &fn);
      break;
    default:
      ok = false;
  }
  if (!ok) return hipErrorInvalidValue;
  launch_timed(fn, dim3((unsigned)cv.B), dim3(kSetThreads), 0u, stream, t_start, t_stop, tv, cv,
               args);
  return hipGetLastError();
}

// ln L of set s = the sum of its n_bins terms, in a fixed order (strided
// per-thread sums, wave butterfly, then the four waves), so repeated calls
// give identical results.
__global__ __launch_bounds__(256) void k_lnl_reduce(const double *__restrict__ terms,
                                                    int n_bins, double *__restrict__ lnl) {
  __shared__ double part[4];
  const int s = blockIdx.x;
  const double *t = terms + (int64_t)s * n_bins;
  double acc = 0.0;
  for (int j = threadIdx.x; j < n_bins; j += 256) acc += t[j];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) lnl[s] = (part[0] + part[1]) + (part[2] + part[3]);
}

hipError_t launch_lnl_reduce(const double *terms, int n_sets, int n_bins, double *lnl,
                             hipStream_t stream) {
  if (n_sets <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_lnl_reduce, dim3((unsigned)n_sets), dim3(256), 0, stream, terms, n_bins,
                     lnl);
  return hipGetLastError();
}

// ------------------------------------------------------ parameter unpack
// One workgroup per parameter vector, writing the columns out (the fused
// path forms them inside the level kernel with the same functions).
__global__ __launch_bounds__(256) void k_unpack(ParamView pv, const double *__restrict__ theta,
                                                double *__restrict__ p, double *__restrict__ T,
                                                double *__restrict__ x, double *__restrict__ logg,
                                                double *__restrict__ scale,
                                                double *__restrict__ cloud,
                                                double *__restrict__ eps) {
  __shared__ double Tn[kMaxTNodes];
  __shared__ int bad_s;
  const int s = blockIdx.x;
  const double *th = theta + (int64_t)s * pv.n_theta;
  if (threadIdx.x == 0) bad_s = theta_nodes(pv, th, Tn) ? 1 : 0;
  __syncthreads();
  const bool bad = bad_s != 0;
  const int L = pv.L;
  for (int l = threadIdx.x; l < L; l += blockDim.x)
    theta_level(pv, Tn, l, bad, p[(int64_t)s * L + l], T[(int64_t)s * L + l]);
  for (int sp = threadIdx.x; sp < pv.S; sp += blockDim.x)
    x[(int64_t)s * pv.S + sp] = theta_x(pv, th, sp);
  if (threadIdx.x == 0) {
    logg[s] = th[0];
    scale[s] = theta_scale(pv, th);
    const double *c = theta_tail(pv, th);
    if (cloud)
      for (int k = 0; k < 3; ++k) cloud[(int64_t)s * 3 + k] = pv.with_cloud ? c[k] : 0.0;
    if (eps) eps[s] = pv.with_eps ? c[3 * pv.with_cloud] : 0.0;
  }
}

hipError_t launch_unpack(const ParamView &pv, int n_sets, const double *theta, double *p,
                         double *T, double *x, double *logg, double *scale, double *cloud,
                         double *eps, hipStream_t stream) {
  if (n_sets <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_unpack, dim3((unsigned)n_sets), dim3(256), 0, stream, pv, theta, p, T, x,
                     logg, scale, cloud, eps);
  return hipGetLastError();
}

// ------------------------------------------------ observation layout build
// Eq. 17 with the 5 sigma cut: for window point i, sigma_i = nu_i / (R 2
// sqrt(2 ln 2)), h_i = the largest k with k dnu <= 5 sigma_i (found here with
// the host plan's operations, written out for the weights kernel),
// g_i(k) = exp(-(k dnu)^2 / (2 sigma_i^2)), Z_i = sum of g_i over the
// window.  Then per bin j with edges a < b: K_j(x) = 1/(b - a) *
// sum_{i=a}^{b} c_i g_i(x - i) / Z_i, c_i = 1/2 at i = a, b and 1 inside
// (trapezoid rule over the bin's points, divided by its width).
// Each launch covers one or more layouts: n_segs == 0 means the single
// layout passed by value in seg0, otherwise the segment of the workgroup is
// the last one whose first workgroup (norm_wg_begin / weight_wg_begin) is at
// or below it.
__device__ __forceinline__ ObsSeg obs_seg(const ObsSeg *segs, int n_segs, const ObsSeg &seg0,
                                          bool weights) {
  if (n_segs == 0) return seg0;
  const int64_t g = blockIdx.x;
  int lo = 0;
  for (int hi = n_segs; hi - lo > 1;) {
    const int mid = (lo + hi) >> 1;
    if ((weights ? segs[mid].weight_wg_begin : segs[mid].norm_wg_begin) <= g) lo = mid;
    else hi = mid;
  }
  return segs[lo];
}

// The 5 sigma cut decides which taps exist: the same FP64 operations as the
// host's plan (no contraction into fused multiply-adds), so both find the
// same largest k with k dnu <= 5 sigma_i.
__device__ __forceinline__ int obs_half_width(const ObsSeg &d, int64_t i, double &sig) {
#pragma clang fp contract(off)
  sig = (d.nu_first + (double)i * d.dnu) / d.denom;
  const double lim = 5.0 * sig;
  const double hv = floor(lim / d.dnu);
  int64_t hh = hv < 1e9 ? (int64_t)hv : (int64_t)1e9;
  while ((double)(hh + 1) * d.dnu <= lim) ++hh;
  while (hh > 0 && (double)hh * d.dnu > lim) --hh;
  return (int)(hh < d.N ? hh : d.N);
}

// FP64 layouts: the direct sums, one wave per window point (four per
// workgroup).
__global__ __launch_bounds__(256) void k_obs_norm_f64(const ObsSeg *segs, int n_segs,
                                                      ObsSeg seg0) {
  const ObsSeg d = obs_seg(segs, n_segs, seg0, false);
  // lanes split the 2h+1 taps, fixed butterfly sum
  const int64_t t = ((int64_t)blockIdx.x - d.norm_wg_begin) * 4 +
                    __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (t >= d.n_pts) return;
  const int64_t i = d.i0 + t;
  double sig;
  const int hi = obs_half_width(d, i, sig);
  if (lane == 0) d.h[t] = hi;
  int64_t klo = -hi, khi = hi;
  if (i + klo < 0) klo = -i;
  if (i + khi > d.N - 1) khi = d.N - 1 - i;
  double z = 0.0;
  for (int64_t k = klo + lane; k <= khi; k += 64) {
    const double dx = (double)(k < 0 ? -k : k) * d.dnu;
    z += exp(-dx * dx / (2.0 * sig * sig));
  }
  const double q = 1.0 / (2.0 * sig * sig);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) z += __shfl_xor(z, off, 64);
  if (lane == 0) {
    ((double *)d.q)[t] = q;
    ((double *)d.invz)[t] = 1.0 / z;
  }
}

// Z = sum_{k=a}^{b} exp(-k^2 / (2 s^2)) (a <= 0 <= b integers) by the
// Euler-Maclaurin formula: the integral (erf) plus the endpoint terms of f
// and of its first, third and fifth derivatives.  Against the direct sum:
// relative error below 1e-9 for s >= 4 and below 5e-12 for s >= 8, also for
// ranges cut short by the window's ends (the aliasing error of the
// trapezoid sum, ~exp(-2 pi^2 s^2), is nil there).
__device__ double gauss_sum_em(double s, double a, double b) {
  const double is2 = 1.0 / (s * s);
  const double r = 0.70710678118654752 / s;   // 1 / (s sqrt 2)
  const double fa = exp(-0.5 * a * a * is2), fb = exp(-0.5 * b * b * is2);
  // odd derivatives, with u = x^2 / s^2: d1 = -x/s^2 f,
  // d3 = x/s^4 (3 - u) f, d5 = x/s^6 (-15 + 10 u - u^2) f
  auto odd = [&](double x, double fx, double &d1, double &d3, double &d5) {
    const double u = x * x * is2, xs = x * is2;
    d1 = -xs * fx;
    d3 = xs * is2 * (3.0 - u) * fx;
    d5 = xs * is2 * is2 * (-15.0 + u * (10.0 - u)) * fx;
  };
  double a1, a3, a5, b1, b3, b5;
  odd(a, fa, a1, a3, a5);
  odd(b, fb, b1, b3, b5);
  return s * 1.2533141373155003 * (erf(b * r) - erf(a * r)) + 0.5 * (fa + fb) +
         (b1 - a1) / 12.0 - (b3 - a3) / 720.0 + (b5 - a5) / 30240.0;
}

// FP32 layouts: one thread per window point.  Z_i in closed form once the
// profile spans s = sigma_i / dnu >= 4 grid steps, else the direct sum of
// its at most 41 taps.
__global__ __launch_bounds__(256) void k_obs_norm_f32(const ObsSeg *segs, int n_segs,
                                                      ObsSeg seg0) {
  const ObsSeg d = obs_seg(segs, n_segs, seg0, false);
  const int64_t t = ((int64_t)blockIdx.x - d.norm_wg_begin) * blockDim.x + threadIdx.x;
  if (t >= d.n_pts) return;
  const int64_t i = d.i0 + t;
  double sig;
  const int hi = obs_half_width(d, i, sig);
  d.h[t] = hi;
  int64_t klo = -hi, khi = hi;
  if (i + klo < 0) klo = -i;
  if (i + khi > d.N - 1) khi = d.N - 1 - i;
  const float q = (float)(d.dnu * d.dnu * kLog2e / (2.0 * sig * sig));
  const double s = sig / d.dnu;
  double z;
  if (s >= 4.0) {
    z = gauss_sum_em(s, (double)klo, (double)khi);
  } else {
    float zf = 0.0f;
    for (int64_t k = klo; k <= khi; ++k) {
      const float kf = (float)k;
      zf += fexp2(-(kf * kf) * q);
    }
    z = zf;
  }
  ((float *)d.q)[t] = q;
  ((float *)d.invz)[t] = (float)(1.0 / z);
}

// k_obs_weights: workgroup size and lanes per stored weight
constexpr int kObsWeightThreads = 256;
constexpr int kObsLanes = 4;

template <typename Real>
__global__ __launch_bounds__(kObsWeightThreads) void k_obs_weights(const ObsSeg *segs,
                                                                   int n_segs, ObsSeg seg0) {
  const ObsSeg d = obs_seg(segs, n_segs, seg0, true);
  const double dnu = d.dnu;
  const int32_t *h = d.h;
  const Real *q = (const Real *)d.q, *invz = (const Real *)d.invz;
  const int64_t i0 = d.i0, nnz = d.nnz;
  // four lanes per stored weight: find its bin, then each lane sums every
  // fourth of the bin's Gaussians that reach this point (in the order of i),
  // and a fixed two-step butterfly adds the four partial sums
  const int64_t e_raw = ((int64_t)blockIdx.x - d.weight_wg_begin) *
                            (kObsWeightThreads / kObsLanes) +
                        (threadIdx.x / kObsLanes);
  const int part = threadIdx.x % kObsLanes;
  const bool live = e_raw < nnz;
  const int64_t e = live ? e_raw : nnz - 1;   // spare lanes still join the butterfly
  int lo = 0, hi = d.n_bins;   // largest j with kstart[j] <= e
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (d.kstart[mid] <= e) lo = mid;
    else hi = mid;
  }
  const int jb = lo;
  const int64_t a = d.edge_idx[jb], b = d.edge_idx[jb + 1];
  const int64_t x = d.mlo[jb] + (e - d.kstart[jb]);
  const int hmax = h[b - i0] > h[a - i0] ? h[b - i0] : h[a - i0];
  int64_t ia = x - hmax, ib = x + hmax;
  if (ia < a) ia = a;
  if (ib > b) ib = b;
  // point i's term; a point whose cut ends before x adds an exact zero
  auto term = [&](int64_t i, Real acc) -> Real {
    const int64_t k = x - i;
    const int64_t ak = k < 0 ? -k : k;
    const int hi_i = h[i - i0];
    const Real qi = q[i - i0], zi = invz[i - i0];
    const Real ci = (i == a || i == b) ? (Real)0.5 : (Real)1;
    Real gk;
    if constexpr (std::is_same<Real, double>::value) {
      const double dx = (double)ak * dnu;
      gk = exp(-dx * dx * qi);
    } else {
      const float kf = (float)ak;
      gk = fexp2(-(kf * kf) * qi);
    }
    return fma(ci * gk, ak <= hi_i ? zi : (Real)0, acc);
  };
  // four of this lane's points' loads and exponentials are issued together
  Real acc = (Real)0;
  int64_t i = ia + part;
  for (; i + 3 * kObsLanes <= ib; i += 4 * kObsLanes) {
#pragma unroll
    for (int u = 0; u < 4; ++u) acc = term(i + u * kObsLanes, acc);
  }
  for (; i <= ib; i += kObsLanes) acc = term(i, acc);
#pragma unroll
  for (int off = 1; off < kObsLanes; off <<= 1) acc += __shfl_xor(acc, off, 64);
  if (!live || part != 0) return;
  ((Real *)d.K)[e] = acc * (Real)(1.0 / (double)(b - a));
}

int64_t obs_norm_workgroups(bool fp64, int64_t n_pts) {
  return fp64 ? (n_pts + 3) / 4 : (n_pts + 255) / 256;
}

int64_t obs_weight_workgroups(int64_t nnz) {
  const int64_t per_wg = kObsWeightThreads / kObsLanes;
  return (nnz + per_wg - 1) / per_wg;
}

static hipError_t obs_launches(bool fp64, const ObsSeg *segs, int n_segs, const ObsSeg &seg0,
                               int64_t norm_wgs, int64_t weight_wgs, hipStream_t stream) {
  if (norm_wgs <= 0 || weight_wgs <= 0) return hipSuccess;
  if (fp64) {
    hipLaunchKernelGGL(k_obs_norm_f64, dim3((unsigned)norm_wgs), dim3(256), 0, stream, segs,
                       n_segs, seg0);
    hipLaunchKernelGGL(k_obs_weights<double>, dim3((unsigned)weight_wgs),
                       dim3(kObsWeightThreads), 0, stream, segs, n_segs, seg0);
  } else {
    hipLaunchKernelGGL(k_obs_norm_f32, dim3((unsigned)norm_wgs), dim3(256), 0, stream, segs,
                       n_segs, seg0);
    hipLaunchKernelGGL(k_obs_weights<float>, dim3((unsigned)weight_wgs),
                       dim3(kObsWeightThreads), 0, stream, segs, n_segs, seg0);
  }
  return hipGetLastError();
}

hipError_t launch_obs_build(bool fp64, int64_t N, double nu_first, double dnu_eff, double denom,
                            int n_bins, int64_t nnz, const int64_t *edge_idx_dev, int32_t *h_dev,
                            int64_t i0, int64_t n_pts, void *q_scratch, void *invz_scratch,
                            const int64_t *kstart_dev, const int32_t *mlo_dev, void *K_dev,
                            hipStream_t stream) {
  ObsSeg d{};
  d.norm_wg_begin = 0;
  d.weight_wg_begin = 0;
  d.N = N;
  d.i0 = i0;
  d.n_pts = n_pts;
  d.nnz = nnz;
  d.nu_first = nu_first;
  d.dnu = dnu_eff;
  d.denom = denom;
  d.n_bins = n_bins;
  d.edge_idx = edge_idx_dev;
  d.kstart = kstart_dev;
  d.mlo = mlo_dev;
  d.h = h_dev;
  d.q = q_scratch;
  d.invz = invz_scratch;
  d.K = K_dev;
  return obs_launches(fp64, nullptr, 0, d, obs_norm_workgroups(fp64, n_pts),
                      obs_weight_workgroups(nnz), stream);
}

hipError_t launch_obs_build_segs(bool fp64, const ObsSeg *segs_dev, int n_segs,
                                 int64_t norm_wgs, int64_t weight_wgs, hipStream_t stream) {
  const ObsSeg seg0{};
  return obs_launches(fp64, segs_dev, n_segs, seg0, norm_wgs, weight_wgs, stream);
}

}  // namespace hr2
