// Host test of the serving pool (paper_1910_02611_amd/csrc/serve_pool.hpp):
// batch layouts, the first-fit allocator, and admission by device bytes
// against a fake budget in a simulated serving loop.  Exits 0 when every
// check holds.
#include <cstdio>
#include <deque>
#include <random>
#include <vector>

#include "serve_pool.hpp"

using namespace rambo_pool;

#define CHECK(c)                                                                \
    do {                                                                        \
        if (!(c)) {                                                             \
            std::fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
            return 1;                                                           \
        }                                                                       \
    } while (0)

int main()
{
    // layouts: every part starts 256-aligned and after the previous one
    for (uint64_t n : {1ull, 7ull, 1000ull})
        for (uint64_t b : {0ull, 150ull, 5000ull}) {
            const BatchLayout l = batch_layout(n, b, 4 * n * 197);
            CHECK(l.hdr == 0 && l.chars >= 8 * (n + 2) && l.state >= l.chars + b && l.total >= l.state + 4 * n * 197);
            CHECK(l.chars % kAlign == 0 && l.state % kAlign == 0 && l.total % kAlign == 0);
            CHECK(l.total < 8 * (n + 2) + b + 4 * n * 197 + 3 * kAlign);
        }

    // allocator: fill, free in another order, merge back to one block
    {
        Pool p(10 * kAlign);
        uint64_t a = p.alloc(3 * kAlign), b = p.alloc(1), c = p.alloc(4 * kAlign);
        CHECK(a == 0 && b == 3 * kAlign && c == 4 * kAlign && p.used() == 8 * kAlign);
        CHECK(p.alloc(3 * kAlign) == kNone && p.largest_free() == 2 * kAlign);
        p.release(b, 1);
        CHECK(p.free_blocks() == 2 && p.largest_free() == 2 * kAlign);
        p.release(a, 3 * kAlign);
        CHECK(p.free_blocks() == 2 && p.largest_free() == 4 * kAlign);
        CHECK(p.alloc(4 * kAlign) == 0);
        p.release(0, 4 * kAlign);
        p.release(c, 4 * kAlign);
        CHECK(p.free_blocks() == 1 && p.largest_free() == 10 * kAlign && p.used() == 0 && p.peak() == 8 * kAlign);
    }

    // admission: a serving loop over a fake budget; batches take requests in
    // order while their bytes fit the largest free region, and finish in a
    // random order
    const uint64_t rsw = 192;
    const auto need = [&](uint64_t n, uint64_t b) { return batch_layout(n, b, 4 * (n * (rsw + 4) + n + 2)).total; };
    std::mt19937_64 rng(7);
    struct Req {
        uint64_t reads, bytes;
        bool barrier;
    };
    std::deque<Req> queue;
    size_t n_req = 0;
    for (int i = 0; i < 5000; ++i) {
        const uint64_t n = 1 + rng() % 64;
        queue.push_back({n, n * (150 + rng() % 4850), i % 997 == 996});
        n_req += 1;
    }
    const uint64_t budget = 4 * need(64, 64 * 5000);   // room for about four of the largest requests
    Pool pool(budget);
    struct Run {
        uint64_t off, size, reqs;
    };
    std::vector<Run> running;
    const size_t max_slots = 6;
    uint64_t served = 0, waits = 0, peak_running = 0, served_barriers = 0;
    while (!queue.empty() || !running.empty()) {
        // start batches while slots and room allow
        while (running.size() < max_slots && !queue.empty()) {
            if (queue.front().barrier) {
                if (!running.empty())
                    break;   // an insert runs alone, after every earlier batch
                queue.pop_front();
                ++served;
                ++served_barriers;
                continue;
            }
            uint64_t reads = 0, bytes = 0;
            const auto at = [&](size_t i) { return Queued{queue[i].barrier, queue[i].reads, queue[i].bytes}; };
            const size_t take = batch_take(queue.size(), at, need, 8192, 8ull << 20, pool.largest_free(),
                                           budget / max_slots, reads, bytes);
            if (take == 0) {
                ++waits;
                CHECK(!running.empty());   // only a running batch can free room
                break;
            }
            const uint64_t size = need(reads, bytes);
            CHECK(size <= pool.largest_free());
            const uint64_t off = pool.alloc(size);
            CHECK(off != kNone && off + size <= budget);
            running.push_back({off, size, take});
            for (size_t i = 0; i < take; ++i)
                queue.pop_front();
            CHECK(pool.used() <= budget);
            peak_running = running.size() > peak_running ? running.size() : peak_running;
        }
        if (running.empty())
            continue;
        const size_t k = rng() % running.size();
        pool.release(running[k].off, running[k].size);
        served += running[k].reqs;
        running.erase(running.begin() + (long)k);
    }
    CHECK(served == n_req && served_barriers == 5);
    CHECK(pool.used() == 0 && pool.free_blocks() == 1 && pool.largest_free() == pool.size());
    CHECK(waits > 0 && peak_running >= 2 && pool.peak() <= budget);
    // a request larger than the whole pool never fits
    uint64_t r = 0, b = 0;
    const auto big = [&](size_t) { return Queued{false, 64, 64 * 5000}; };
    CHECK(batch_take(1, big, need, 8192, 8ull << 20, need(64, 64 * 5000) - kAlign, ~0ull, r, b) == 0);
    // past the first request a batch keeps to its share; the first may exceed it
    const auto small = [&](size_t) { return Queued{false, 4, 600}; };
    CHECK(batch_take(100, small, need, 8192, 8ull << 20, ~0ull, need(8, 1200), r, b) == 2 && r == 8);
    CHECK(batch_take(100, small, need, 8192, 8ull << 20, ~0ull, 1, r, b) == 1 && r == 4);
    std::printf("serve pool ok: %llu requests, %llu waits for room, peak %llu of %llu bytes\n",
                (unsigned long long)served, (unsigned long long)waits, (unsigned long long)pool.peak(),
                (unsigned long long)budget);
    return 0;
}
