// CPU checks of the driver's host-side pieces (paper_2504_18943_amd/csrc/ltlf_host.h):
// the scheduler's region allocator against a granule-by-granule model, the
// workspace size model's invariants, and the staging-block search against
// brute force.  Prints "ok" and exits 0, or names
// the first failure and exits 1.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "../../paper_2504_18943_amd/csrc/ltlf_host.h"

using namespace ltlf;

static int fails = 0;
#define CHECK(c, ...)                                      \
    do {                                                   \
        if (!(c)) {                                        \
            std::printf("FAIL %s:%d: ", __FILE__, __LINE__); \
            std::printf(__VA_ARGS__);                      \
            std::printf("\n");                             \
            if (++fails > 10) std::exit(1);                \
        }                                                  \
    } while (0)

// Allocator: random alloc / alloc_high / alloc_at / release against a
// bitmap of 256-byte granules; every returned range lies in [lo, hi), is
// 256-aligned, was free, and the free list stays sorted, coalesced and
// equal to the bitmap's free granules.
static void arena_random(uint64_t seed) {
    std::mt19937_64 rng(seed);
    const uint64_t G = 256, n = 4096, lo = 1024 * G;
    Arena a;
    a.init(lo, lo + n * G);
    std::vector<int> used(n, 0);
    std::vector<std::pair<uint64_t, uint64_t>> live;
    for (int step = 0; step < 20000; ++step) {
        const int kind = (int)(rng() % 4);
        if (kind < 3) {
            const uint64_t bytes = 1 + rng() % (64 * G);
            const uint64_t g = (bytes + G - 1) / G;
            uint64_t off = 0;
            bool ok = false;
            if (kind == 0) ok = a.alloc(bytes, off);
            else if (kind == 1) ok = a.alloc_high(bytes, off);
            else {
                off = lo + (rng() % n) * G;
                ok = off + g * G <= lo + n * G && a.alloc_at(off, bytes);
                if (!ok) {  // alloc_at must refuse exactly when the range is not wholly free
                    bool free_all = off + g * G <= lo + n * G;
                    for (uint64_t i = 0; free_all && i < g; ++i) free_all = !used[(off - lo) / G + i];
                    CHECK(!free_all, "alloc_at refused a free range at %llu", (unsigned long long)off);
                    continue;
                }
            }
            if (!ok) {  // first-fit / top-fit refuse only when no run of g free granules exists
                uint64_t run = 0, best = 0;
                for (uint64_t i = 0; i < n; ++i) {
                    run = used[i] ? 0 : run + 1;
                    best = std::max(best, run);
                }
                CHECK(best < g, "alloc refused %llu granules with a run of %llu free", (unsigned long long)g,
                      (unsigned long long)best);
                continue;
            }
            CHECK(off >= lo && off + g * G <= lo + n * G && off % G == 0, "range out of the arena");
            for (uint64_t i = 0; i < g; ++i) {
                CHECK(!used[(off - lo) / G + i], "granule handed out twice");
                used[(off - lo) / G + i] = 1;
            }
            if (kind == 0) {  // first fit: no free run of g granules below off
                uint64_t run = 0;
                for (uint64_t i = 0; i < (off - lo) / G; ++i) {
                    run = used[i] ? 0 : run + 1;
                    CHECK(run < g, "first fit skipped a lower free run");
                }
            }
            live.push_back({off, bytes});
        } else if (!live.empty()) {
            const size_t k = rng() % live.size();
            const auto r = live[k];
            live.erase(live.begin() + (long)k);
            a.release(r.first, r.second);
            for (uint64_t i = 0; i < (r.second + G - 1) / G; ++i) used[(r.first - lo) / G + i] = 0;
        }
        // the free list equals the bitmap's free runs, sorted and coalesced
        uint64_t fb = 0;
        for (uint64_t i = 0; i < n; ++i) fb += used[i] ? 0 : G;
        CHECK(a.free_bytes() == fb, "free bytes %llu, model %llu", (unsigned long long)a.free_bytes(),
              (unsigned long long)fb);
        for (size_t i = 0; i < a.free_.size(); ++i) {
            const auto& f = a.free_[i];
            CHECK(f.second > 0 && f.second % G == 0 && f.first % G == 0, "bad free range");
            if (i) CHECK(a.free_[i - 1].first + a.free_[i - 1].second < f.first, "free list not sorted and coalesced");
            for (uint64_t j = 0; j < f.second / G; ++j) CHECK(!used[(f.first - lo) / G + j], "free range overlaps a live one");
        }
        CHECK(a.empty() == (fb == n * G), "empty() disagrees");
    }
}

// Size model: the pieces of a workspace of `bytes` fit in it in the carve-up
// order (deferral lists, table of two slots per row, rows, records), the row
// capacity grows with the workspace and never passes 2^31 - 16, and a
// region's row store never starts beyond a larger workspace's (so a region
// can be placed with its rows where the larger layout puts them).
static void size_model(uint64_t seed) {
    std::mt19937_64 rng(seed);
    for (int t = 0; t < 20000; ++t) {
        const uint64_t fixed = align_up(4096 + rng() % (64ull << 20), 256);
        const uint64_t Wp = 4 * (1 + rng() % 512);
        const uint64_t bytes = fixed + (1ull << 20) + rng() % (256ull << 30);
        const uint64_t cap = row_capacity(fixed, Wp, bytes);
        uint64_t d0, d1;
        deferral_records(bytes - fixed, d0, d1);
        CHECK(d0 >= 65536 && d0 <= kDeferMax && d1 >= 4096 && d1 >= d0 / 16, "deferral list sizes");
        CHECK(cap <= (1ull << 31) - 16, "capacity above the limit");
        if (cap) {
            const uint64_t ro = rows_offset(fixed, Wp, bytes);
            const uint64_t table = align_up(align_up(fixed + 16 * d0, 256) + 16 * d1, 256);
            CHECK(ro == align_up(table + 16 * cap, 256), "row store offset");
            const uint64_t meta = align_up(ro + 4 * Wp * cap, 256);
            CHECK(meta + 16 * cap <= bytes, "records pass the end of the workspace");
            CHECK(ro % 256 == 0, "row store not aligned");
            const uint64_t bigger = bytes + rng() % (256ull << 30);
            const uint64_t cap2 = row_capacity(fixed, Wp, bigger);
            CHECK(cap2 >= cap, "capacity not monotone");
            CHECK(rows_offset(fixed, Wp, bigger) >= ro, "a larger workspace's rows start earlier");
        }
    }
}

// Staging-block search: against every 256-aligned start in a small range,
// free_spot finds a block exactly when one exists, and what it returns lies
// in the range, is aligned and overlaps no interval to avoid.
static void spot_random(uint64_t seed) {
    std::mt19937_64 rng(seed);
    const uint64_t G = 256;
    for (int t = 0; t < 20000; ++t) {
        const uint64_t lo = (rng() % 8) * 100 + (rng() % 2) * G * 4, hi = lo + (8 + rng() % 56) * G + rng() % G;
        const uint64_t need = 1 + rng() % (24 * G);
        std::vector<std::pair<uint64_t, uint64_t>> avoid;
        for (uint64_t k = 0, m = rng() % 6; k < m; ++k) {
            const uint64_t a = lo + rng() % (hi - lo + 512), b = a + 1 + rng() % (8 * G);
            avoid.push_back({a, b});
        }
        auto clear = [&](uint64_t x) {
            if (x < lo || x + need > hi) return false;
            for (const auto& iv : avoid)
                if (x < iv.second && iv.first < x + need) return false;
            return true;
        };
        bool any = false;
        for (uint64_t x = align_up(lo, G); x + need <= hi && !any; x += G) any = clear(x);
        const uint64_t got = free_spot(lo, hi, need, avoid);
        CHECK(any == (got != UINT64_MAX), "free_spot %s a block (need %llu in [%llu, %llu))",
              any ? "missed" : "invented", (unsigned long long)need, (unsigned long long)lo,
              (unsigned long long)hi);
        if (got != UINT64_MAX) CHECK(got % G == 0 && clear(got), "free_spot returned a bad block");
    }
}

int main() {
    arena_random(1);
    arena_random(2);
    size_model(3);
    spot_random(4);
    if (fails) return 1;
    std::printf("ok\n");
    return 0;
}
