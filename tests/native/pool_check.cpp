// Randomised check of the server's device-budget allocator (RegionPool)
// against a byte-occupancy model: granted ranges never overlap, lie inside
// the region and are the lowest that fit; the free list stays sorted,
// disjoint and merged; the accounting adds up; freeing everything restores
// one free range.  Exit status 0 when every check holds.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "pool.h"

using wmd::RegionPool;

static int failures = 0;
#define CHECK(c)                                                             \
    do {                                                                     \
        if (!(c)) {                                                          \
            std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            ++failures;                                                      \
        }                                                                    \
    } while (0)

struct Grant {
    size_t off, bytes;
};

// lowest offset at which `need` free bytes start, in the occupancy model
static long long first_fit(const std::vector<char>& used, size_t need) {
    size_t run = 0;
    for (size_t i = 0; i < used.size(); ++i) {
        run = used[i] ? 0 : run + 1;
        if (run == need) return (long long)(i + 1 - need);
    }
    return -1;
}

static void check_free_list(const RegionPool& p, const std::vector<char>& used) {
    size_t prev_end = 0, total = 0, largest = 0;
    bool first = true;
    for (const auto& f : p.free_ranges()) {
        CHECK(f.second > 0);
        CHECK(f.first + f.second <= p.capacity());
        if (!first) CHECK(f.first > prev_end);   // sorted, disjoint, never adjacent
        for (size_t i = f.first; i < f.first + f.second; i += RegionPool::kAlign) CHECK(!used[i / RegionPool::kAlign]);
        prev_end = f.first + f.second;
        total += f.second;
        if (f.second > largest) largest = f.second;
        first = false;
    }
    CHECK(total + p.used() == p.capacity());
    CHECK(largest == p.largest_free());
}

int main() {
    const size_t units = 512;
    RegionPool p(units * RegionPool::kAlign + 100);   // the tail below one unit is not usable
    CHECK(p.capacity() == units * RegionPool::kAlign);
    CHECK(RegionPool::rounded(0) == RegionPool::kAlign);
    CHECK(RegionPool::rounded(1) == RegionPool::kAlign);
    CHECK(RegionPool::rounded(256) == 256 && RegionPool::rounded(257) == 512);
    std::vector<char> used(units, 0);
    std::vector<Grant> live;
    std::mt19937_64 rng(12345);
    for (int step = 0; step < 200000; ++step) {
        const bool do_alloc = live.empty() || (rng() % 100) < 55;
        if (do_alloc) {
            const size_t bytes = 1 + rng() % (RegionPool::kAlign * (1 + rng() % 64));
            const size_t need = RegionPool::rounded(bytes) / RegionPool::kAlign;
            const long long want = first_fit(used, need);
            size_t off = 0;
            const bool ok = p.alloc(bytes, &off);
            CHECK(ok == (want >= 0));
            if (ok) {
                CHECK(off % RegionPool::kAlign == 0);
                CHECK((long long)(off / RegionPool::kAlign) == want);
                for (size_t i = 0; i < need; ++i) {
                    CHECK(!used[off / RegionPool::kAlign + i]);
                    used[off / RegionPool::kAlign + i] = 1;
                }
                live.push_back({off, bytes});
            }
        } else {
            const size_t k = rng() % live.size();
            const Grant g = live[k];
            live[k] = live.back();
            live.pop_back();
            p.release(g.off, g.bytes);
            for (size_t i = 0; i < RegionPool::rounded(g.bytes) / RegionPool::kAlign; ++i)
                used[g.off / RegionPool::kAlign + i] = 0;
        }
        if (step % 97 == 0) check_free_list(p, used);
        if (failures > 20) break;
    }
    for (const Grant& g : live) p.release(g.off, g.bytes);
    CHECK(p.used() == 0);
    CHECK(p.free_ranges().size() == 1);
    CHECK(p.largest_free() == p.capacity());
    // an empty region grants nothing
    RegionPool z(100);
    size_t off = 0;
    CHECK(!z.alloc(1, &off));
    CHECK(z.largest_free() == 0);
    std::printf("pool checks: %d failures\n", failures);
    return failures == 0 ? 0 : 1;
}
