// The serving loop's host paths through the C ABI, from several threads at
// once: argument validation, the whole-budget rejection, queued work on a
// device that cannot start (the scheduler fails it), latest-histogram
// queries, holds, statistics, polling and shutdown with work still queued.
// Built against a host-only build of the library (no device code, so nothing
// can reach a kernel) under ThreadSanitizer or AddressSanitizer by
// tests/test_host_checks.py.
#include "ih.h"

#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <thread>
#include <vector>

#define CHECK(c)                                                                   \
    do {                                                                           \
        if (!(c)) {                                                                \
            std::fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #c); \
            std::exit(1);                                                          \
        }                                                                          \
    } while (0)

int main()
{
    ih_server_config bad{1000, 4, 2, 4, 0, 0};
    ih_server* s = nullptr;
    CHECK(ih_server_create(&bad, &s) == IH_ERR_INVALID_ARG && s == nullptr);
    ih_server_config cfg{64u << 20, 8, 2, 4, 1, 16u << 20};
    CHECK(ih_server_create(&cfg, &s) == IH_OK && s != nullptr);

    std::vector<uint8_t> frame(64 * 80, 7), big(1024 * 1024, 1);
    const ih_rect good{0, 0, 79, 63}, outside{0, 0, 80, 0};
    std::atomic<int> done{0};
    std::vector<std::thread> th;
    std::vector<uint64_t> tickets[4];
    for (int t = 0; t < 4; ++t)
        th.emplace_back([&, t] {
            for (int i = 0; i < 25; ++i) {
                uint64_t tk = 0;
                CHECK(ih_submit(s, t, frame.data(), 64, 80, 0, &good, 1, &tk) == IH_ERR_INVALID_ARG);
                CHECK(ih_submit(s, t, frame.data(), 64, 80, 16, &outside, 1, &tk) == IH_ERR_INVALID_ARG);
                CHECK(ih_submit(s, t, big.data(), 1024, 1024, 64, nullptr, 0, &tk) == IH_ERR_BUDGET);
                const ih_status st = ih_submit(s, t, frame.data(), 64, 80, 16, &good, 1, &tk);
                CHECK(st == IH_OK);
                tickets[t].push_back(tk);
                uint32_t h[256];
                uint64_t ft = 0;
                const ih_status q = ih_server_query_latest(s, t, &good, 1, h, &ft);
                CHECK(q != IH_OK || ft != 0);
                ih_server_counters c;
                CHECK(ih_server_stats(s, &c) == IH_OK);
            }
            done += 1;
        });
    std::thread holder([&] {
        for (int i = 0; i < 20; ++i) {
            CHECK(ih_server_hold(s, i % 2) == IH_OK);
            std::this_thread::yield();
        }
        CHECK(ih_server_hold(s, 0) == IH_OK);
    });
    for (auto& x : th) x.join();
    holder.join();
    // every request either finished (on a machine without a usable device,
    // with the error the scheduler recorded) or is still queued; poll them
    int finished = 0;
    for (int t = 0; t < 4; ++t)
        for (uint64_t tk : tickets[t]) {
            uint32_t h[16];
            ih_timing tm;
            const ih_status st = ih_poll(s, tk, h, &tm);
            CHECK(st != IH_ERR_UNKNOWN_TICKET);
            if (st != IH_NOT_READY) {
                ++finished;
                CHECK(ih_poll(s, tk, h, &tm) == IH_ERR_UNKNOWN_TICKET);   // collected once
            }
        }
    // shut down with whatever is still queued
    CHECK(ih_server_destroy(s) == IH_OK);
    std::printf("server paths passed (%d of 100 requests finished before shutdown)\n", finished);
    return 0;
}
