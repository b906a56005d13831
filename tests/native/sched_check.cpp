// Checks of the serving scheduler's host policy (serve_sched.h) against a
// reference model, driven by seeded random operations: the first-fit arena
// (no overlap, lowest fitting offset, exact byte accounting, full
// coalescing) and the first-in first-out admission under a byte budget and a
// slot cap with simulated step completions.  Exit status 0 = all passed.
#include <cstdint>
#include <cstdio>
#include <deque>
#include <random>
#include <vector>

#include "serve_sched.h"

using hr2::Arena;

static int g_fail = 0;
#define CHECK(c, ...)                                            \
  do {                                                           \
    if (!(c)) {                                                  \
      ++g_fail;                                                  \
      std::fprintf(stderr, "FAIL %s:%d: ", __FILE__, __LINE__); \
      std::fprintf(stderr, __VA_ARGS__);                         \
      std::fprintf(stderr, "\n");                                \
      if (g_fail > 20) return;                                   \
    }                                                            \
  } while (0)

// lowest unit index where `n` free units start in the reference bitmap, or -1
static long first_fit(const std::vector<char> &used, size_t n) {
  size_t run = 0;
  for (size_t u = 0; u < used.size(); ++u) {
    run = used[u] ? 0 : run + 1;
    if (run == n) return (long)(u + 1 - n);
  }
  return -1;
}

static void arena_random(uint64_t seed, size_t units, int ops) {
  std::mt19937_64 rng(seed);
  Arena a(units * 256);
  std::vector<char> ref(units, 0);
  struct Blk { size_t off, bytes; };
  std::vector<Blk> live;
  size_t ref_used = 0;
  for (int op = 0; op < ops; ++op) {
    const bool do_alloc = live.empty() || (rng() % 100) < 55;
    if (do_alloc) {
      // sizes from one byte to a quarter of the arena, some exact multiples
      size_t bytes = 1 + rng() % (units * 64);
      if (rng() % 4 == 0) bytes = (bytes + 255) / 256 * 256;
      const size_t n = (bytes + 255) / 256;
      const long want = first_fit(ref, n);
      size_t off = 0;
      const bool ok = a.alloc(bytes, &off);
      CHECK(ok == (want >= 0), "seed %llu op %d: alloc(%zu) ok=%d, reference %ld",
            (unsigned long long)seed, op, bytes, (int)ok, want);
      if (!ok) continue;
      CHECK(off % 256 == 0 && off / 256 == (size_t)want,
            "seed %llu op %d: alloc(%zu) at %zu, first fit at unit %ld",
            (unsigned long long)seed, op, bytes, off, want);
      for (size_t u = off / 256; u < off / 256 + n; ++u) {
        CHECK(u < units && !ref[u], "seed %llu op %d: unit %zu overlaps or leaves the arena",
              (unsigned long long)seed, op, u);
        if (u < units) ref[u] = 1;
      }
      live.push_back({off, bytes});
      ref_used += n * 256;
    } else {
      const size_t k = rng() % live.size();
      const Blk b = live[k];
      live[k] = live.back();
      live.pop_back();
      a.release(b.off, b.bytes);
      for (size_t u = b.off / 256; u < b.off / 256 + (b.bytes + 255) / 256; ++u) ref[u] = 0;
      ref_used -= (b.bytes + 255) / 256 * 256;
    }
    CHECK(a.used() == ref_used, "seed %llu op %d: used %zu, reference %zu",
          (unsigned long long)seed, op, a.used(), ref_used);
  }
  for (const Blk &b : live) a.release(b.off, b.bytes);
  CHECK(a.used() == 0 && a.free_blocks() == 1, "seed %llu: after releasing all, used %zu, %zu free blocks",
        (unsigned long long)seed, a.used(), a.free_blocks());
  size_t off = 1;
  CHECK(a.alloc(units * 256, &off) && off == 0, "seed %llu: the whole arena is not one block",
        (unsigned long long)seed);
}

struct MockReq {
  int id;
  size_t bytes;
  size_t off;
  int done_after;   // steps the request stays admitted
};

// A mock executor: requests arrive in bursts, each step admits what the
// policy allows and every admitted request completes after its own number
// of steps (releasing its block).
static void admission_random(uint64_t seed, size_t cap, int max_slots, int n_req) {
  std::mt19937_64 rng(seed);
  Arena arena(cap);
  std::vector<MockReq> all(n_req);
  for (int i = 0; i < n_req; ++i) {
    size_t b = 256 + rng() % (cap / 3);
    if (rng() % 10 == 0) b = cap - rng() % 512;   // some nearly fill the arena alone
    all[i] = {i, b, 0, 1 + (int)(rng() % 4)};
  }
  std::deque<MockReq *> pending;
  std::vector<MockReq *> admitted;
  std::vector<int> order;
  int next = 0, n_admitted = 0, steps = 0;
  while ((next < n_req || !pending.empty() || !admitted.empty()) && steps < 100000) {
    ++steps;
    const int burst = (int)(rng() % 5);
    for (int k = 0; k < burst && next < n_req; ++k) pending.push_back(&all[next++]);
    const size_t head_before = pending.empty() ? 0 : pending.front()->bytes;
    const int before = n_admitted;
    const int k = hr2::admit_fifo(
        pending, arena, max_slots, n_admitted, [](const MockReq *r) { return r->bytes; },
        [&](MockReq *r, size_t off) {
          r->off = off;
          order.push_back(r->id);
          admitted.push_back(r);
        });
    CHECK(n_admitted == before + k, "seed %llu step %d: admitted count", (unsigned long long)seed,
          steps);
    CHECK(n_admitted <= max_slots, "seed %llu step %d: %d admitted > %d slots",
          (unsigned long long)seed, steps, n_admitted, max_slots);
    CHECK(arena.used() <= cap, "seed %llu step %d: %zu bytes used > budget %zu",
          (unsigned long long)seed, steps, arena.used(), cap);
    // the head left waiting either does not fit now or the slots are full
    if (!pending.empty() && k == 0 && n_admitted < max_slots) {
      size_t off;
      Arena probe = arena;
      CHECK(!probe.alloc(pending.front()->bytes, &off),
            "seed %llu step %d: head of %zu bytes waits though it fits",
            (unsigned long long)seed, steps, head_before);
    }
    // the admitted blocks never overlap
    for (size_t i = 0; i < admitted.size(); ++i)
      for (size_t j = i + 1; j < admitted.size(); ++j) {
        const MockReq *a = admitted[i], *b = admitted[j];
        const size_t ae = a->off + hr2::round256(a->bytes), be = b->off + hr2::round256(b->bytes);
        CHECK(ae <= b->off || be <= a->off, "seed %llu step %d: blocks of %d and %d overlap",
              (unsigned long long)seed, steps, a->id, b->id);
      }
    // completions
    for (size_t i = 0; i < admitted.size();) {
      if (--admitted[i]->done_after <= 0) {
        arena.release(admitted[i]->off, admitted[i]->bytes);
        --n_admitted;
        admitted[i] = admitted.back();
        admitted.pop_back();
      } else {
        ++i;
      }
    }
  }
  CHECK((int)order.size() == n_req, "seed %llu: %zu of %d requests admitted in %d steps",
        (unsigned long long)seed, order.size(), n_req, steps);
  for (int i = 0; i < (int)order.size(); ++i)
    CHECK(order[i] == i, "seed %llu: admission %d was request %d (not first in, first out)",
          (unsigned long long)seed, i, order[i]);
  CHECK(arena.used() == 0, "seed %llu: %zu bytes still held", (unsigned long long)seed,
        arena.used());
}

int main() {
  for (uint64_t seed = 1; seed <= 40; ++seed) arena_random(seed, 64 + seed * 7, 3000);
  arena_random(1001, 1, 200);   // a one-unit arena
  for (uint64_t seed = 1; seed <= 40; ++seed)
    admission_random(seed, (size_t)(4096 + seed * 1000) * 256, 1 + (int)(seed % 9), 400);
  admission_random(2001, 256 * 1024, 1, 200);   // one slot: strictly one at a time
  if (g_fail) {
    std::fprintf(stderr, "%d check(s) failed\n", g_fail);
    return 1;
  }
  std::printf("scheduler policy checks passed\n");
  return 0;
}
