// serve.cpp — continuous batching of uneven forward-model requests.
//
// A scheduler thread owns two streams and a device arena of the server's
// byte budget.  Requests are admitted first-in first-out while their
// footprint fits the arena and a slot is free; each step launches the work
// of every admitted, not yet launched request as a handful of launches over
// all of them (one segment per request): one upload of their columns and
// bin plans, ONE level-record launch, ONE pair of layout-build launches, ONE
// column-kernel launch per kernel variant, ONE convolve/bin launch, and one
// download of all their bins to pinned host memory.  Up to two steps are in
// flight, one per stream, so a step admitted while another runs overlaps it
// on the device.  Per-set arithmetic does not depend on the other requests
// of a step (the layer-chunk count is a function of the request alone), so
// a result is bit-identical alone and in the mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <ctime>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "hr2_context.h"
#include "hr2_internal.h"
#include "serve_sched.h"

using namespace hr2;

namespace {

double now_s() {
  timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

struct Req {
  uint64_t ticket = 0;
  hr2_request_info info{};
  hr2_window window{};
  int n_bins = 0, n_sets = 0, L = 0, n_mu = 0, chunks = 1;
  std::vector<double> cols;   // packed p, T, x, log g, scale
  ObsPlan plan;
  // byte offsets inside the request's device block (arena)
  size_t o_h = 0, o_recs = 0, o_fplus = 0, o_K = 0, o_q = 0, o_z = 0, bytes = 0;
  size_t bins_bytes = 0;
  // byte offsets inside the stage of the step that launches the request
  size_t st_cols = 0, st_kstart = 0, st_mlo = 0, st_mlen = 0, st_edges = 0, st_bins = 0;
  size_t dev_off = 0;
  bool admitted = false;
  std::vector<unsigned char> result;
};

// One of the two step streams with its stage: descriptors and the inputs of
// the step's requests (uploaded at once), then their bins (downloaded at
// once), in device memory and in a pinned host image of the same layout.
struct StepSlot {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  DevBuf stage;
  void *pinned = nullptr;
  size_t pinned_cap = 0;
  std::vector<Req *> reqs;
  bool busy = false;
  uint64_t seq = 0;
};

}  // namespace

struct hr2_server {
  hr2_ctx *ctx = nullptr;
  const hr2_tables *tables = nullptr;
  size_t budget = 0;
  int max_slots = 1;
  void *arena_dev = nullptr;
  Arena dev;
  StepSlot slots[2];
  uint64_t step_seq = 0;

  std::mutex mu;
  std::condition_variable cv_work;   // wakes the scheduler
  std::condition_variable cv_done;   // wakes waiters
  std::deque<Req *> pending;         // submitted, not admitted
  std::vector<Req *> admitted;       // admitted, not launched
  std::unordered_map<uint64_t, std::unique_ptr<Req>> all;
  uint64_t next_ticket = 1;
  int n_admitted = 0;                // admitted and not finished
  bool stop = false;
  bool fail_next = false;
  bool hold = false;
  bool para = false;                 // parabolic source (the context's option at creation)
  hr2_serve_stats stats{};
  std::thread thr;

  void run();
  void finish_step(StepSlot &sl);
  void release(Req *r);
  bool launch_step(StepSlot &sl, std::vector<Req *> &reqs);
};

namespace {

size_t real_bytes(const hr2_tables *t) {
  return t->view.dtype == HR2_TABLE_F64 ? sizeof(double) : sizeof(float);
}
size_t rec_bytes(const hr2_tables *t) {
  return t->view.dtype == HR2_TABLE_F64 ? sizeof(LevelRecD) : sizeof(LevelRecF);
}

// The request's device block: half widths, level records, F+, layout
// weights and the layout build's scratch.
void layout_request(const hr2_tables *t, Req &r) {
  const size_t rs = real_bytes(t);
  size_t o = 0;
  auto take = [&o](size_t n) {
    const size_t at = o;
    o += round256(std::max<size_t>(n, 1));
    return at;
  };
  r.o_h = take(r.plan.n_pts * sizeof(int32_t));   // written by the layout build
  r.o_recs = take((size_t)r.n_sets * r.L * rec_bytes(t));
  r.o_fplus = take((size_t)r.n_sets * r.window.nu_count * rs);
  r.o_K = take((size_t)r.plan.nnz * rs);
  r.o_q = take((size_t)r.plan.n_pts * rs);
  r.o_z = take((size_t)r.plan.n_pts * rs);
  r.bytes = o;
  r.bins_bytes = (size_t)r.n_sets * r.n_bins * rs;
}

}  // namespace

// ------------------------------------------------------------- scheduler
void hr2_server::release(Req *r) {
  if (r->admitted) {
    dev.release(r->dev_off, r->bytes);
    r->admitted = false;
    --n_admitted;
  }
}

bool hr2_server::launch_step(StepSlot &sl, std::vector<Req *> &reqs) {
  const TableView &tv = tables->view;
  const bool fp64 = tv.dtype == HR2_TABLE_F64;
  const size_t rs = real_bytes(tables), rb = rec_bytes(tables);
  hipStream_t s = sl.stream;
  unsigned char *base = (unsigned char *)arena_dev;
  if (hipSetDevice(ctx->device) != hipSuccess) return false;
  // column launches group the requests by chunk count (= workgroup size)
  // and by angle class (kernel variant), so each request runs exactly the
  // code it would run alone
  std::stable_sort(reqs.begin(), reqs.end(), [](const Req *a, const Req *b) {
    const int ka = a->chunks * 16 + column_mu_class(a->n_mu);
    const int kb = b->chunks * 16 + column_mu_class(b->n_mu);
    return ka < kb;
  });
  const size_t n = reqs.size();
  // stage layout: descriptors, then each request's inputs, then the bins
  size_t o = 0;
  auto take = [&o](size_t bytes) {
    const size_t at = o;
    o += round256(std::max<size_t>(bytes, 1));
    return at;
  };
  const size_t o_lv = take(n * sizeof(LevelSeg)), o_ob = take(n * sizeof(ObsSeg));
  const size_t o_cs = take(n * sizeof(ColSeg)), o_vs = take(n * sizeof(ConvSeg));
  for (Req *r : reqs) {
    r->st_cols = take(r->cols.size() * sizeof(double));
    r->st_kstart = take(r->n_bins * sizeof(int64_t));
    r->st_mlo = take(r->n_bins * sizeof(int32_t));
    r->st_mlen = take(r->n_bins * sizeof(int32_t));
    r->st_edges = take((r->n_bins + 1) * sizeof(int64_t));
  }
  const size_t o_bins = o;
  for (Req *r : reqs) r->st_bins = take(r->bins_bytes);
  const size_t total = o;
  // this slot's previous step has completed, so nothing reads its old stage
  sl.stage.free_retired();
  if (sl.stage.ensure(total) != HR2_OK) return false;
  if (sl.pinned_cap < total) {
    if (sl.pinned) (void)hipHostFree(sl.pinned);
    sl.pinned = nullptr;
    sl.pinned_cap = 0;
    if (hipHostMalloc(&sl.pinned, total, hipHostMallocDefault) != hipSuccess) return false;
    sl.pinned_cap = total;
  }
  unsigned char *img = (unsigned char *)sl.pinned;
  unsigned char *dst = (unsigned char *)sl.stage.ptr;
  LevelSeg *lv = (LevelSeg *)(img + o_lv);
  ObsSeg *ob = (ObsSeg *)(img + o_ob);
  ColSeg *cs = (ColSeg *)(img + o_cs);
  ConvSeg *vs = (ConvSeg *)(img + o_vs);
  struct Group {
    size_t first, count;
    int64_t wgs;
    int chunks, max_mu;
  };
  std::vector<Group> groups;
  int64_t wg = 0, conv_wgs = 0, lev_wgs = 0, norm_wgs = 0, weight_wgs = 0;
  for (size_t i = 0; i < n; ++i) {
    Req &r = *reqs[i];
    std::memcpy(img + r.st_cols, r.cols.data(), r.cols.size() * sizeof(double));
    std::memcpy(img + r.st_kstart, r.plan.kstart.data(), r.n_bins * sizeof(int64_t));
    std::memcpy(img + r.st_mlo, r.plan.mlo.data(), r.n_bins * sizeof(int32_t));
    std::memcpy(img + r.st_mlen, r.plan.mlen.data(), r.n_bins * sizeof(int32_t));
    std::memcpy(img + r.st_edges, r.plan.idx.data(), (r.n_bins + 1) * sizeof(int64_t));
    unsigned char *blk = base + r.dev_off;
    const ColumnsView cv = columns_view(dst + r.st_cols, r.n_sets, r.L, tv.S);
    LevelSeg &l = lv[i];
    std::memset(&l, 0, sizeof(l));
    l.wg_begin = lev_wgs;
    l.rec_offset = (int64_t)((r.dev_off + r.o_recs) / rb);
    l.cv = cv;
    l.blocks_per_set = level_blocks_per_set(tv, r.L);
    lev_wgs += (int64_t)r.n_sets * l.blocks_per_set;
    ObsSeg &b = ob[i];
    std::memset(&b, 0, sizeof(b));
    b.norm_wg_begin = norm_wgs;
    b.weight_wg_begin = weight_wgs;
    b.N = r.plan.N;
    b.i0 = r.plan.i0;
    b.n_pts = r.plan.n_pts;
    b.nnz = r.plan.nnz;
    b.nu_first = r.plan.first;
    b.dnu = r.plan.dnu;
    b.denom = r.plan.denom;
    b.n_bins = r.n_bins;
    b.edge_idx = (const int64_t *)(dst + r.st_edges);
    b.kstart = (const int64_t *)(dst + r.st_kstart);
    b.mlo = (const int32_t *)(dst + r.st_mlo);
    b.h = (int32_t *)(blk + r.o_h);
    b.q = blk + r.o_q;
    b.invz = blk + r.o_z;
    b.K = blk + r.o_K;
    norm_wgs += obs_norm_workgroups(fp64, r.plan.n_pts);
    weight_wgs += obs_weight_workgroups(r.plan.nnz);
    const int mu_class = column_mu_class(r.n_mu);
    if (groups.empty() || groups.back().chunks != r.chunks || groups.back().max_mu != mu_class) {
      groups.push_back(Group{i, 0, 0, r.chunks, mu_class});
      wg = 0;
    }
    ColSeg &c = cs[i];
    std::memset(&c, 0, sizeof(c));
    const int per_wg = column_nu_per_wg(r.chunks);
    c.wg_begin = wg;
    c.nu_begin = r.window.nu_begin;
    c.nu_count = r.window.nu_count;
    c.nu_stride = r.window.nu_stride;
    c.rec_offset = l.rec_offset;
    c.out_offset = (int64_t)((r.dev_off + r.o_fplus) / rs);
    c.out_stride = r.window.nu_count;
    c.n_sets = r.n_sets;
    c.n_levels = r.L;
    c.n_mu = r.n_mu;
    c.chunks = r.chunks;
    c.tiles_per_set = (int32_t)((r.window.nu_count + per_wg - 1) / per_wg);
    wg += (int64_t)r.n_sets * c.tiles_per_set;
    groups.back().count += 1;
    groups.back().wgs = wg;
    if (wg > 0x7fffffff || lev_wgs > 0x7fffffff || norm_wgs > 0x7fffffff ||
        weight_wgs > 0x7fffffff)
      return false;
    ConvSeg &v = vs[i];
    std::memset(&v, 0, sizeof(v));
    v.item_begin = conv_wgs;
    v.K = blk + r.o_K;
    v.kstart = b.kstart;
    v.mlo = b.mlo;
    v.mlen = (const int32_t *)(dst + r.st_mlen);
    v.in_offset = c.out_offset;
    v.in_stride = r.window.nu_count;
    v.out_offset = (int64_t)(r.st_bins / rs);
    v.scale = cv.scale;
    v.n_sets = r.n_sets;
    v.n_bins = r.n_bins;
    v.items_per_wg = conv_items_per_wg(r.plan.nnz, r.n_bins);
    conv_wgs += conv_workgroups((int64_t)r.n_sets * r.n_bins, v.items_per_wg);
  }
  if (conv_wgs > 0x7fffffff) return false;
  if (hipMemcpyAsync(dst, img, o_bins, hipMemcpyHostToDevice, s) != hipSuccess) return false;
  if (launch_levels_segs(tv, (const LevelSeg *)(dst + o_lv), (int)n, lev_wgs, base, fp64, s) !=
      hipSuccess)
    return false;
  if (launch_obs_build_segs(fp64, (const ObsSeg *)(dst + o_ob), (int)n, norm_wgs, weight_wgs,
                            s) != hipSuccess)
    return false;
  const ColSeg *dcs = (const ColSeg *)(dst + o_cs);
  for (const Group &gq : groups)
    if (launch_column(tv, dcs + gq.first, (int)gq.count, nullptr, gq.wgs, gq.chunks, base,
                      nullptr, base, gq.max_mu, false, para, false, s) != hipSuccess)
      return false;
  if (launch_convolve_bin(fp64, (const ConvSeg *)(dst + o_vs), (int)n, nullptr, conv_wgs, base,
                          dst, s) != hipSuccess)
    return false;
  if (hipMemcpyAsync(img + o_bins, dst + o_bins, total - o_bins, hipMemcpyDeviceToHost, s) !=
      hipSuccess)
    return false;
  return hipEventRecord(sl.done, s) == hipSuccess;
}

void hr2_server::finish_step(StepSlot &sl) {
  // called with mu held, after sl.done completed
  const hipError_t e = hipEventQuery(sl.done);
  const double t = now_s();
  for (Req *r : sl.reqs) {
    if (e == hipSuccess) {
      const unsigned char *src = (const unsigned char *)sl.pinned + r->st_bins;
      r->result.assign(src, src + r->bins_bytes);
      r->info.state = HR2_REQ_DONE;
      r->info.error = HR2_OK;
      ++stats.requests_done;
    } else {
      r->info.state = HR2_REQ_ERROR;
      r->info.error = HR2_E_DEVICE;
      ++stats.requests_failed;
    }
    r->info.t_done = t;
    release(r);
  }
  sl.reqs.clear();
  sl.busy = false;
  cv_done.notify_all();
}

void hr2_server::run() {
  (void)hipSetDevice(ctx->device);
  std::unique_lock<std::mutex> lk(mu);
  for (;;) {
    // retire finished steps, oldest first
    for (;;) {
      StepSlot *oldest = nullptr;
      for (auto &sl : slots)
        if (sl.busy && (!oldest || sl.seq < oldest->seq)) oldest = &sl;
      if (!oldest) break;
      const hipError_t q = hipEventQuery(oldest->done);
      if (q == hipErrorNotReady) break;
      finish_step(*oldest);
    }
    if (stop) {
      for (Req *r : pending) {
        r->info.state = HR2_REQ_CANCELLED;
        r->info.error = HR2_E_CANCELLED;
        r->info.t_done = now_s();
      }
      pending.clear();
      for (Req *r : admitted) {
        r->info.state = HR2_REQ_CANCELLED;
        r->info.error = HR2_E_CANCELLED;
        r->info.t_done = now_s();
        release(r);
      }
      admitted.clear();
      cv_done.notify_all();
      bool any = false;
      for (auto &sl : slots) any |= sl.busy;
      if (!any) break;
    }
    // admit first-in first-out while memory and slots allow
    if (!stop)
      admit_fifo(
          pending, dev, max_slots, n_admitted, [](const Req *r) { return r->bytes; },
          [this](Req *r, size_t off) {
            r->dev_off = off;
            r->admitted = true;
            stats.peak_bytes = std::max(stats.peak_bytes, dev.used());
            stats.max_inflight = std::max<uint64_t>(stats.max_inflight, (uint64_t)n_admitted);
            r->info.t_admit = now_s();
            r->info.state = HR2_REQ_RUNNING;
            admitted.push_back(r);
          });
    // launch a step on a free slot
    StepSlot *free_slot = nullptr;
    for (auto &sl : slots)
      if (!sl.busy) free_slot = &sl;
    if (!stop && !hold && !admitted.empty() && free_slot) {
      std::vector<Req *> reqs;
      reqs.swap(admitted);
      StepSlot &sl = *free_slot;
      sl.busy = true;
      sl.seq = ++step_seq;
      sl.reqs = reqs;
      ++stats.steps;
      stats.max_step_requests = std::max<uint64_t>(stats.max_step_requests, reqs.size());
      if (fail_next) {
        // injected failure: nothing is enqueued for this step
        fail_next = false;
        const double t = now_s();
        for (Req *r : reqs) {
          r->info.state = HR2_REQ_ERROR;
          r->info.error = HR2_E_DEVICE;
          r->info.t_done = t;
          ++stats.requests_failed;
          release(r);
        }
        sl.reqs.clear();
        sl.busy = false;
        cv_done.notify_all();
        continue;
      }
      lk.unlock();
      const bool ok = launch_step(sl, reqs);
      if (!ok) {
        (void)hipGetLastError();
        (void)hipStreamSynchronize(sl.stream);
      }
      lk.lock();
      if (!ok) {
        const double t = now_s();
        for (Req *r : sl.reqs) {
          r->info.state = HR2_REQ_ERROR;
          r->info.error = HR2_E_DEVICE;
          r->info.t_done = t;
          ++stats.requests_failed;
          release(r);
        }
        sl.reqs.clear();
        sl.busy = false;
        cv_done.notify_all();
      }
      continue;
    }
    // nothing to launch: wait for a submission or for the device
    bool any_busy = false;
    for (auto &sl : slots) any_busy |= sl.busy;
    if (any_busy) {
      StepSlot *oldest = nullptr;
      for (auto &sl : slots)
        if (sl.busy && (!oldest || sl.seq < oldest->seq)) oldest = &sl;
      if (!free_slot || (pending.empty() && admitted.empty())) {
        // block on the device (no new step could start anyway)
        hipEvent_t ev = oldest->done;
        lk.unlock();
        (void)hipEventSynchronize(ev);
        lk.lock();
      } else {
        cv_work.wait_for(lk, std::chrono::microseconds(50));
      }
    } else if (hold && !stop) {
      cv_work.wait_for(lk, std::chrono::milliseconds(1));
    } else if (!stop) {
      cv_work.wait(lk, [this] { return stop || hold || !pending.empty() || !admitted.empty(); });
    }
  }
}

// ------------------------------------------------------------------ C ABI
extern "C" hr2_status hr2_serve_create(hr2_ctx *ctx, const hr2_tables *t, size_t budget,
                                       int max_slots, hr2_server **out) {
  if (!ctx || !t || !out) return set_error(HR2_E_INVALID_ARG, "NULL argument");
  *out = nullptr;
  if (budget < 4096) return set_error(HR2_E_INVALID_ARG, "budget must be at least 4096 bytes");
  if (max_slots < 1) return set_error(HR2_E_INVALID_ARG, "max_slots must be >= 1");
  if (hipSetDevice(ctx->device) != hipSuccess) return set_error(HR2_E_DEVICE, "hipSetDevice");
  auto *srv = new hr2_server();
  srv->ctx = ctx;
  srv->para = ctx->opt_source == 2;
  srv->tables = t;
  srv->budget = round256(budget);
  srv->max_slots = max_slots;
  hipError_t e = hipMalloc(&srv->arena_dev, srv->budget);
  for (auto &sl : srv->slots) {
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    if (srv->arena_dev) (void)hipFree(srv->arena_dev);
    for (auto &sl : srv->slots) {
      if (sl.stream) (void)hipStreamDestroy(sl.stream);
      if (sl.done) (void)hipEventDestroy(sl.done);
    }
    delete srv;
    return set_error(e == hipErrorOutOfMemory ? HR2_E_NO_MEMORY : HR2_E_DEVICE,
                     std::string("server setup: ") + hipGetErrorString(e));
  }
  srv->dev.reset(srv->budget);
  srv->thr = std::thread([srv] { srv->run(); });
  *out = srv;
  return HR2_OK;
}

extern "C" hr2_status hr2_serve_submit(hr2_server *srv, const hr2_request *q, uint64_t *ticket) {
  if (!srv || !q || !ticket) return set_error(HR2_E_INVALID_ARG, "NULL argument");
  const hr2_tables *t = srv->tables;
  if (q->n_sets < 1 || !q->cols) return set_error(HR2_E_INVALID_ARG, "request needs columns");
  hr2_status st = check_n_mu(q->n_mu);
  if (st != HR2_OK) return st;
  for (int i = 0; i < q->n_sets; ++i)
    if ((st = check_column(t, q->cols[i], q->cols[0].n_levels)) != HR2_OK) return st;
  auto r = std::make_unique<Req>();
  if ((st = plan_obs(t, q->window, q->resolving_power, q->n_bins, q->bin_edges_cm, r->plan)) !=
      HR2_OK)
    return st;
  r->window = q->window;
  r->n_bins = q->n_bins;
  r->n_sets = q->n_sets;
  r->L = q->cols[0].n_levels;
  r->n_mu = q->n_mu;
  {
    // chunking depends on the request alone, so its result does not depend on the mix
    (void)hipSetDevice(srv->ctx->device);
    r->chunks = auto_chunks(t->view, (int64_t)r->n_sets * ((r->window.nu_count + 63) / 64), r->L,
                            r->n_mu, false, srv->para);
  }
  pack_columns(t, q->n_sets, q->cols, r->cols);
  layout_request(t, *r);
  if (r->bytes > srv->budget)
    return set_error(HR2_E_NO_MEMORY, "request needs " + std::to_string(r->bytes) +
                                          " device bytes, budget is " + std::to_string(srv->budget));
  r->info.state = HR2_REQ_PENDING;
  r->info.t_submit = now_s();
  r->info.n_bins = r->n_bins;
  r->info.n_sets = r->n_sets;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    if (srv->stop) return set_error(HR2_E_CANCELLED, "server is shutting down");
    r->ticket = srv->next_ticket++;
    *ticket = r->ticket;
    srv->pending.push_back(r.get());
    srv->all.emplace(r->ticket, std::move(r));
  }
  srv->cv_work.notify_one();
  return HR2_OK;
}

extern "C" hr2_status hr2_serve_submit_packed(hr2_server *srv, hr2_window window, double R,
                                              int n_bins, const double *edges, int n_sets,
                                              int n_levels, const double *p, const double *T,
                                              const double *x, const double *log_g,
                                              const double *scale, int n_mu, uint64_t *ticket) {
  if (!srv || !p || !T || !x || !log_g || !scale || !ticket)
    return set_error(HR2_E_INVALID_ARG, "NULL argument");
  if (n_sets < 1) return set_error(HR2_E_INVALID_ARG, "n_sets must be >= 1");
  const int S = srv->tables->view.S;
  std::vector<hr2_column> cols(n_sets);
  for (int i = 0; i < n_sets; ++i) {
    cols[i].n_levels = n_levels;
    cols[i].p_bar = p + (size_t)i * n_levels;
    cols[i].T_K = T + (size_t)i * n_levels;
    cols[i].x = x + (size_t)i * S;
    cols[i].log_g_cgs = log_g[i];
    cols[i].scale = scale[i];
  }
  hr2_request q;
  q.window = window;
  q.resolving_power = R;
  q.n_bins = n_bins;
  q.bin_edges_cm = edges;
  q.n_sets = n_sets;
  q.cols = cols.data();
  q.n_mu = n_mu;
  return hr2_serve_submit(srv, &q, ticket);
}

static hr2_status poll_locked(hr2_server *srv, uint64_t ticket, void *bins, size_t cap,
                              hr2_request_info *info) {
  auto it = srv->all.find(ticket);
  if (it == srv->all.end()) return set_error(HR2_E_NOT_FOUND, "unknown or released ticket");
  Req &r = *it->second;
  if (info) *info = r.info;
  switch (r.info.state) {
    case HR2_REQ_PENDING:
    case HR2_REQ_RUNNING:
      return HR2_NOT_READY;
    case HR2_REQ_DONE: {
      const size_t elems = (size_t)r.n_sets * r.n_bins;
      if (bins == nullptr || cap < elems)
        return set_error(HR2_E_INVALID_ARG, "result buffer too small: need " + std::to_string(elems));
      std::memcpy(bins, r.result.data(), r.result.size());
      srv->all.erase(it);
      return HR2_OK;
    }
    default: {
      const hr2_status e = r.info.error;
      srv->all.erase(it);
      return set_error(e, e == HR2_E_CANCELLED ? "request cancelled" : "request failed");
    }
  }
}

extern "C" hr2_status hr2_serve_poll(hr2_server *srv, uint64_t ticket, void *bins, size_t cap,
                                     hr2_request_info *info) {
  if (!srv) return set_error(HR2_E_INVALID_ARG, "NULL server");
  std::lock_guard<std::mutex> lk(srv->mu);
  return poll_locked(srv, ticket, bins, cap, info);
}

extern "C" hr2_status hr2_serve_wait(hr2_server *srv, uint64_t ticket, double timeout_s,
                                     void *bins, size_t cap, hr2_request_info *info) {
  if (!srv) return set_error(HR2_E_INVALID_ARG, "NULL server");
  std::unique_lock<std::mutex> lk(srv->mu);
  const auto until = std::chrono::steady_clock::now() +
                     std::chrono::duration_cast<std::chrono::steady_clock::duration>(
                         std::chrono::duration<double>(std::max(0.0, timeout_s)));
  srv->cv_done.wait_until(lk, until, [&] {
    auto it = srv->all.find(ticket);
    return it == srv->all.end() || it->second->info.state >= HR2_REQ_DONE;
  });
  return poll_locked(srv, ticket, bins, cap, info);
}

extern "C" hr2_status hr2_serve_debug_fail_next_step(hr2_server *srv) {
  if (!srv) return set_error(HR2_E_INVALID_ARG, "NULL server");
  std::lock_guard<std::mutex> lk(srv->mu);
  srv->fail_next = true;
  return HR2_OK;
}

extern "C" hr2_status hr2_serve_debug_hold(hr2_server *srv, int hold) {
  if (!srv) return set_error(HR2_E_INVALID_ARG, "NULL server");
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->hold = hold != 0;
  }
  srv->cv_work.notify_all();
  return HR2_OK;
}

extern "C" hr2_status hr2_serve_get_stats(hr2_server *srv, hr2_serve_stats *out) {
  if (!srv || !out) return set_error(HR2_E_INVALID_ARG, "NULL argument");
  std::lock_guard<std::mutex> lk(srv->mu);
  *out = srv->stats;
  return HR2_OK;
}

extern "C" void hr2_serve_destroy(hr2_server *srv) {
  if (!srv) return;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->stop = true;
  }
  srv->cv_work.notify_all();
  if (srv->thr.joinable()) srv->thr.join();
  (void)hipSetDevice(srv->ctx->device);
  for (auto &sl : srv->slots) {
    if (sl.stream) {
      (void)hipStreamSynchronize(sl.stream);
      (void)hipStreamDestroy(sl.stream);
    }
    if (sl.done) (void)hipEventDestroy(sl.done);
    sl.stage.release();
    if (sl.pinned) (void)hipHostFree(sl.pinned);
  }
  if (srv->arena_dev) (void)hipFree(srv->arena_dev);
  delete srv;
}
