// Unit test of the serving loop's host-side scheduling (batching.h): the
// first-fit arena, FIFO admission and batch selection, single-threaded and
// under concurrent submitters, completers and a scheduler thread. Built and
// run by tests/test_host_sanitizers.py with AddressSanitizer + UBSan and
// with ThreadSanitizer (g++, host code only).

#include <atomic>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <mutex>
#include <random>
#include <thread>
#include <utility>
#include <vector>

#include "batching.h"

using sand::Arena;

#define CHECK(c)                                                        \
  do {                                                                  \
    if (!(c)) {                                                         \
      std::fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #c); \
      std::exit(1);                                                     \
    }                                                                   \
  } while (0)

struct Req {
  size_t bytes = 0, off = 0;
  int64_t n = 0;
  int key = 0;
  int id = 0;
};

// Free ranges always tile [0, size) minus the allocated ranges, sorted and
// coalesced (no two adjacent free ranges touch).
static void check_invariant(const Arena& a, size_t size,
                            const std::vector<std::pair<size_t, size_t>>& live) {
  auto fr = a.free_ranges();
  size_t free_total = 0;
  for (size_t i = 0; i < fr.size(); ++i) {
    free_total += fr[i].second;
    CHECK(fr[i].second > 0);
    if (i) CHECK(fr[i - 1].first + fr[i - 1].second < fr[i].first);
  }
  size_t used = 0;
  for (auto& l : live) used += l.second;
  CHECK(used == a.used);
  CHECK(free_total + used == size);
  for (auto& l : live)
    for (auto& f : fr) CHECK(l.first + l.second <= f.first || f.first + f.second <= l.first);
}

static void test_arena_basic() {
  Arena a;
  a.init(1000);
  size_t o1, o2, o3, o4;
  CHECK(a.alloc(100, &o1) && o1 == 0);
  CHECK(a.alloc(200, &o2) && o2 == 100);
  CHECK(a.alloc(300, &o3) && o3 == 300);
  CHECK(a.used == 600 && a.peak == 600);
  CHECK(!a.alloc(401, &o4));                      // 400 left
  a.release(o2, 200);                             // hole [100, 300)
  CHECK(a.used == 400 && a.peak == 600);
  CHECK(a.alloc(150, &o4) && o4 == 100);          // first fit takes the hole
  a.release(o1, 100);
  a.release(o4, 150);                             // [0, 300) free again, one range
  auto fr = a.free_ranges();
  CHECK(fr.size() == 2 && fr[0].first == 0 && fr[0].second == 300);
  a.release(o3, 300);                             // everything coalesces
  fr = a.free_ranges();
  CHECK(fr.size() == 1 && fr[0].first == 0 && fr[0].second == 1000);
  CHECK(a.used == 0 && a.peak == 600);
  CHECK(!a.alloc(0, &o1));                        // a zero-size request takes nothing
  CHECK(a.alloc(1000, &o1) && o1 == 0 && !a.alloc(1, &o2));
  a.release(o1, 1000);
  a.init(64);
  CHECK(a.used == 0 && a.peak == 0);
}

static void test_arena_random() {
  const size_t size = 1 << 20;
  Arena a;
  a.init(size);
  std::mt19937_64 rng(7);
  std::vector<std::pair<size_t, size_t>> live;
  for (int it = 0; it < 20000; ++it) {
    if (live.empty() || rng() % 3 != 0) {
      const size_t n = 1 + rng() % 40000;
      size_t off;
      if (a.alloc(n, &off)) live.emplace_back(off, n);
    } else {
      const size_t k = rng() % live.size();
      a.release(live[k].first, live[k].second);
      live[k] = live.back();
      live.pop_back();
    }
    if (it % 97 == 0) check_invariant(a, size, live);
  }
  for (auto& l : live) a.release(l.first, l.second);
  live.clear();
  check_invariant(a, size, live);
  CHECK(a.free_ranges().size() == 1);
}

static void test_fifo_and_batches() {
  Arena a;
  a.init(1000);
  std::vector<Req> rs(6);
  const size_t bytes[6] = {400, 500, 50, 100, 300, 10};
  const int keys[6] = {1, 2, 1, 1, 2, 1};
  std::deque<Req*> pending, admitted;
  for (int i = 0; i < 6; ++i) {
    rs[i].bytes = bytes[i];
    rs[i].n = (int64_t)bytes[i];
    rs[i].key = keys[i];
    rs[i].id = i;
    pending.push_back(&rs[i]);
  }
  // 400 + 500 fit; 50 would fit too but must not overtake... it is behind
  // them in order, so it is admitted; 100 does not fit (950 used) and stops
  // the queue, even though 10 would fit
  CHECK(sand::admit_fifo(pending, admitted, a) == 3);
  CHECK(pending.size() == 3 && pending.front()->id == 3);
  CHECK(admitted.size() == 3);
  auto key = [](const Req* r) { return r->key; };
  // the head's key is 1: requests 0 and 2 form the batch, 1 (key 2) waits
  auto b = sand::take_batch(admitted, 1 << 20, 1024, key);
  CHECK(b.size() == 2 && b[0]->id == 0 && b[1]->id == 2);
  CHECK(admitted.size() == 1 && admitted.front()->id == 1);
  for (Req* r : b) a.release(r->off, r->bytes);
  CHECK(sand::admit_fifo(pending, admitted, a) == 3);
  // point cap: the head always goes, then only what fits under the cap
  b = sand::take_batch(admitted, 320, 1024, key);
  CHECK(b.size() == 1 && b[0]->id == 1);
  b = sand::take_batch(admitted, 110, 1024, key);
  CHECK(b.size() == 2 && b[0]->id == 3 && b[1]->id == 5);
  b = sand::take_batch(admitted, 1, 1024, key);
  CHECK(b.size() == 1 && b[0]->id == 4 && admitted.empty());
  CHECK(sand::take_batch(admitted, 1, 1024, key).empty());
}

// Submitters push requests, a scheduler admits and batches them under one
// mutex, completer threads release them, as the serving loop does with its
// HIP callbacks. Checks that every request completes once and the arena
// ends empty; ThreadSanitizer checks the locking.
static void test_threaded() {
  struct Srv {
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Req*> pending, admitted;
    std::deque<std::vector<Req*>> running;
    Arena arena;
    int submitted = 0, completed = 0, callbacks = 0;
    bool stopping = false;
  } s;
  const int kSubmitters = 4, kPerSubmitter = 500;
  s.arena.init(1 << 16);
  std::vector<Req> reqs(kSubmitters * kPerSubmitter);
  std::thread sched([&] {
    std::unique_lock<std::mutex> lk(s.mu);
    for (;;) {
      sand::admit_fifo(s.pending, s.admitted, s.arena);
      if (!s.admitted.empty()) {
        auto b = sand::take_batch(s.admitted, 5000, 16, [](const Req* r) { return r->key; });
        s.running.push_back(std::move(b));
        ++s.callbacks;
        s.cv_done.notify_all();
        continue;
      }
      if (s.stopping && s.pending.empty() && s.running.empty() && s.callbacks == 0) break;
      s.cv_work.wait(lk);
    }
  });
  std::vector<std::thread> completers;
  std::atomic<bool> done_all{false};
  for (int c = 0; c < 2; ++c)
    completers.emplace_back([&] {
      std::unique_lock<std::mutex> lk(s.mu);
      for (;;) {
        s.cv_done.wait(lk, [&] { return !s.running.empty() || done_all.load(); });
        if (s.running.empty()) break;
        std::vector<Req*> b = std::move(s.running.front());
        s.running.pop_front();
        for (Req* r : b) {
          s.arena.release(r->off, r->bytes);
          ++s.completed;
        }
        --s.callbacks;
        s.cv_work.notify_all();
        s.cv_done.notify_all();
      }
    });
  std::vector<std::thread> subs;
  for (int t = 0; t < kSubmitters; ++t)
    subs.emplace_back([&, t] {
      std::mt19937 rng(100 + t);
      for (int i = 0; i < kPerSubmitter; ++i) {
        Req& r = reqs[t * kPerSubmitter + i];
        r.n = 1 + rng() % 4000;
        r.bytes = (size_t)r.n * 4;
        r.key = (int)(rng() % 3);
        {
          std::lock_guard<std::mutex> lk(s.mu);
          s.pending.push_back(&r);
          ++s.submitted;
        }
        s.cv_work.notify_all();
      }
    });
  for (auto& t : subs) t.join();
  {
    std::unique_lock<std::mutex> lk(s.mu);
    s.stopping = true;
    s.cv_work.notify_all();
    s.cv_done.wait(lk, [&] { return s.completed == s.submitted; });
  }
  sched.join();
  {
    std::lock_guard<std::mutex> lk(s.mu);
    done_all = true;
    s.cv_done.notify_all();
  }
  for (auto& t : completers) t.join();
  CHECK(s.completed == kSubmitters * kPerSubmitter);
  CHECK(s.arena.used == 0 && s.arena.free_ranges().size() == 1);
  CHECK(s.arena.peak <= (size_t)(1 << 16));
}

int main() {
  test_arena_basic();
  test_arena_random();
  test_fifo_and_batches();
  test_threaded();
  std::printf("batching tests passed\n");
  return 0;
}
