// Unit tests of the serving loop's device-memory bookkeeping (ih_admission):
// first-fit placement and merging, admission with eviction and retry,
// never-fits detection, retention and readers.  Host-only; built and run by
// tests/test_host_checks.py, also under AddressSanitizer, UBSan and
// ThreadSanitizer.
#include "ih_admission.h"

#include <cstdio>
#include <cstdlib>
#include <random>
#include <thread>
#include <vector>

#define CHECK(c)                                                                   \
    do {                                                                           \
        if (!(c)) {                                                                \
            std::fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #c); \
            std::exit(1);                                                          \
        }                                                                          \
    } while (0)

using ih::Admit;
using ih::Arena;
using ih::Residency;
using ih::Retained;

static void arena_first_fit_and_merge()
{
    Arena a(256);
    a.reset(4096);
    size_t x, y, z;
    CHECK(a.alloc(1, &x) && x == 0);
    CHECK(a.alloc(300, &y) && y == 256);         // rounded to 512
    CHECK(a.alloc(1024, &z) && z == 768);
    CHECK(a.used() == 256 + 512 + 1024);
    a.release(y, 300);
    size_t w;
    CHECK(a.alloc(512, &w) && w == 256);         // first fit reuses the hole
    a.release(w, 512);
    a.release(x, 1);
    a.release(z, 1024);
    CHECK(a.used() == 0 && a.largest_free() == 4096);   // all merged back
    CHECK(a.peak() == 256 + 512 + 1024);
    CHECK(!a.alloc(4097, &w));
}

static void fragmentation_is_resolved_by_eviction()
{
    // budget 10 units; two retained histograms split the free space so that
    // neither hole holds the request's histogram, though the total would
    Residency r;
    r.reset(10 * 256);
    size_t a, b, c, d, e;
    CHECK(r.reserve(2 * 256, 256, false, &a, &b) == Admit::kOk);       // stream 1: [0,2) + [2,3)
    CHECK(r.reserve(2 * 256, 256, false, &c, &d) == Admit::kOk);       // stream 2: [3,5) + [5,6)
    r.release(b, 256);
    r.release(d, 256);
    r.retain(1, Retained{1, 1, 1, 1, a, 2 * 256, 0});
    r.retain(2, Retained{2, 1, 1, 1, c, 2 * 256, 0});
    // free: [2,3) and [5,10): a 5-unit histogram fits only the big hole, and
    // then the 2-unit work block does not fit what is left
    CHECK(r.reserve(5 * 256, 2 * 256, false, &e, &b) == Admit::kOk);
    CHECK(r.retained_count() < 2);                                      // something was evicted for it
    // the oldest (stream 1) went first
    Retained h;
    CHECK(!r.acquire(1, &h));
}

static void wait_and_never()
{
    Residency r;
    r.reset(8 * 256);
    size_t a, b;
    CHECK(r.reserve(4 * 256, 2 * 256, false, &a, &b) == Admit::kOk);
    size_t c, d;
    // does not fit beside the admitted request: wait while it is in flight
    CHECK(r.reserve(4 * 256, 2 * 256, true, &c, &d) == Admit::kWait);
    // with nothing in flight and nothing retained, it can never fit
    CHECK(r.reserve(6 * 256, 3 * 256, false, &c, &d) == Admit::kNever);
    r.release(a, 4 * 256);
    r.release(b, 2 * 256);
    CHECK(r.arena().used() == 0);
    CHECK(r.reserve(6 * 256, 2 * 256, false, &c, &d) == Admit::kOk);
}

static void readers_block_eviction()
{
    Residency r;
    r.reset(8 * 256);
    size_t a, b;
    CHECK(r.reserve(4 * 256, 256, false, &a, &b) == Admit::kOk);
    r.release(b, 256);
    r.retain(7, Retained{70, 1, 1, 1, a, 4 * 256, 0});
    Retained h;
    CHECK(r.acquire(7, &h) && h.ticket == 70);
    size_t c, d;
    // the histogram being read is not evicted: wait, not never
    CHECK(r.reserve(6 * 256, 256, false, &c, &d) == Admit::kWait);
    CHECK(r.retained_count() == 1);
    // a newer histogram replaces it; the old one is freed by its last reader
    size_t e, f;
    CHECK(r.reserve(2 * 256, 256, false, &e, &f) == Admit::kOk);
    r.release(f, 256);
    r.retain(7, Retained{71, 1, 1, 1, e, 2 * 256, 0});
    CHECK(r.arena().used() == 6 * 256);                                 // old one still held
    r.release_reader(7, 70);
    CHECK(r.arena().used() == 2 * 256);
    // reserve_one keeps the stream being read
    Retained g;
    CHECK(r.acquire(7, &g) && g.ticket == 71);
    size_t q;
    CHECK(r.reserve_one(7 * 256, false, 7, &q) == Admit::kWait);
    r.release_reader(7, 71);
    CHECK(r.reserve_one(7 * 256, false, 7, &q) == Admit::kNever);       // kept stream, nothing else to free
    // free space is [0,4) and [6,8) around the kept histogram: 4 units fit, 6 never
    CHECK(r.reserve_one(6 * 256, false, 7, &q) == Admit::kNever);
    CHECK(r.reserve_one(4 * 256, false, 7, &q) == Admit::kOk && q == 0);
}

static void fifo_budget_model()
{
    // random requests admitted first-in first-out under a budget: used bytes
    // never exceed it and every request is eventually admitted
    std::mt19937 rng(5);
    Residency r;
    const size_t budget = 1 << 20;
    r.reset(budget);
    struct Held { size_t a, na, b, nb; };
    std::vector<Held> running;
    int admitted = 0;
    for (int i = 0; i < 2000;) {
        const size_t na = 256 * (1 + rng() % 1024), nb = 256 * (1 + rng() % 64);
        size_t a, b;
        Admit ad;
        while ((ad = r.reserve(na, nb, !running.empty(), &a, &b)) == Admit::kWait) {
            const Held h = running.front();
            running.erase(running.begin());
            r.release(h.b, h.nb);
            if (rng() % 2) r.retain((int32_t)(rng() % 8), Retained{(uint64_t)i, 1, 1, 1, h.a, h.na, 0});
            else r.release(h.a, h.na);
        }
        CHECK(ad == Admit::kOk);
        CHECK(r.arena().used() <= budget);
        running.push_back(Held{a, na, b, nb});
        ++admitted;
        ++i;
    }
    CHECK(admitted == 2000);
}

static void arena_threads()
{
    // concurrent callers (the pinned staging pool is shared by submitting and
    // polling threads)
    Arena a(256);
    a.reset(64 << 20);
    std::vector<std::thread> th;
    for (int t = 0; t < 8; ++t)
        th.emplace_back([&a, t] {
            std::mt19937 rng(t);
            std::vector<std::pair<size_t, size_t>> mine;
            for (int i = 0; i < 4000; ++i) {
                if (mine.empty() || rng() % 3) {
                    size_t off, n = 1 + rng() % 100000;
                    if (a.alloc(n, &off)) mine.push_back({off, n});
                } else {
                    a.release(mine.back().first, mine.back().second);
                    mine.pop_back();
                }
            }
            for (auto& m : mine) a.release(m.first, m.second);
        });
    for (auto& t : th) t.join();
    CHECK(a.used() == 0 && a.largest_free() == a.size());
}

int main()
{
    arena_first_fit_and_merge();
    fragmentation_is_resolved_by_eviction();
    wait_and_never();
    readers_block_eviction();
    fifo_budget_model();
    arena_threads();
    std::printf("admission tests passed\n");
    return 0;
}
