// Host-side pieces of the driver that touch no device: the workspace size
// model (how a workspace of a given size is carved into deferral lists, hash
// table, row store and derivation records) and the region allocator of the
// scheduler.  Plain C++ (the CPU tests compile it on its own).
#pragma once

#include <cstddef>
#include <cstdint>
#include <utility>
#include <vector>
#include <algorithm>

namespace ltlf {

inline uint64_t align_up(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }

// Largest deferral list 0 (records of 16 bytes; the list gets 1/1024 of the
// workspace up to this)
#ifndef LTLF_DEFER_MAX
#define LTLF_DEFER_MAX (1ull << 27)
#endif
constexpr uint64_t kDeferMax = LTLF_DEFER_MAX;

// Sizes of the workspace carve-up (the driver's plan_memory follows them),
// for a workspace whose fixed regions (specification, masks, atoms,
// counters, digests, witness tokens, staging; each 256-byte aligned) take
// `fixed` bytes and whose rows have Wp words ...
// ... the deferral lists (records) of what follows them ...
inline void deferral_records(uint64_t rest, uint64_t& d0, uint64_t& d1) {
    d0 = std::min<uint64_t>(std::max<uint64_t>(rest / 64 / 16, 1ull << 16), kDeferMax);
    d1 = std::max<uint64_t>(d0 / 16, 4096);
}
// ... and the rows that fit a workspace of `bytes` (0: none).  Each row takes
// 4 Wp bytes, a 16-byte derivation record and two 8-byte table slots.
inline uint64_t row_capacity(uint64_t fixed, uint64_t Wp, uint64_t bytes) {
    if (fixed >= bytes) return 0;
    uint64_t d0, d1;
    deferral_records(bytes - fixed, d0, d1);
    if ((d0 + d1) * 16 + 4096 >= bytes - fixed) return 0;
    const uint64_t off = align_up(align_up(fixed + 16 * d0, 256) + 16 * d1, 256);
    if (off + 3 * 256 >= bytes) return 0;
    return std::min<uint64_t>((bytes - off - 3 * 256) / (4 * Wp + 32), (1ull << 31) - 16);
}

// ... and the offset of the row store in a workspace of `bytes` (after the
// deferral lists and the table).
inline uint64_t rows_offset(uint64_t fixed, uint64_t Wp, uint64_t bytes) {
    uint64_t d0, d1;
    deferral_records(bytes - fixed, d0, d1);
    const uint64_t table = align_up(align_up(fixed + 16 * d0, 256) + 16 * d1, 256);
    return align_up(table + 16 * row_capacity(fixed, Wp, bytes), 256);
}


// First-fit allocator over [lo, hi) of the workspace (offsets), 256-byte
// granules.
struct Arena {
    uint64_t lo = 0, hi = 0;
    std::vector<std::pair<uint64_t, uint64_t>> free_;  // (offset, bytes), sorted by offset
    void init(uint64_t a, uint64_t b) {
        lo = a;
        hi = b;
        free_.assign(1, {a, b - a});
    }
    uint64_t total() const { return hi - lo; }
    uint64_t free_bytes() const {
        uint64_t f = 0;
        for (const auto& r : free_) f += r.second;
        return f;
    }
    bool empty() const { return free_bytes() == total(); }
    bool alloc(uint64_t bytes, uint64_t& off) {
        bytes = align_up(bytes, 256);
        for (size_t i = 0; i < free_.size(); ++i) {
            if (free_[i].second >= bytes) {
                off = free_[i].first;
                free_[i].first += bytes;
                free_[i].second -= bytes;
                if (free_[i].second == 0) free_.erase(free_.begin() + (long)i);
                return true;
            }
        }
        return false;
    }
    // the top of the highest free range that fits (regions that are not
    // aligned stay clear of the bottom of the large area, where aligned ones go)
    bool alloc_high(uint64_t bytes, uint64_t& off) {
        bytes = align_up(bytes, 256);
        for (size_t i = free_.size(); i-- > 0;) {
            if (free_[i].second >= bytes) {
                free_[i].second -= bytes;
                off = free_[i].first + free_[i].second;
                if (free_[i].second == 0) free_.erase(free_.begin() + (long)i);
                return true;
            }
        }
        return false;
    }
    // [off, off + bytes) if it is free
    bool alloc_at(uint64_t off, uint64_t bytes) {
        bytes = align_up(bytes, 256);
        for (size_t i = 0; i < free_.size(); ++i) {
            const uint64_t o = free_[i].first, b = free_[i].second;
            if (o > off || off + bytes > o + b) continue;
            const uint64_t tail = o + b - (off + bytes);
            if (off > o) {
                free_[i].second = off - o;
                if (tail) free_.insert(free_.begin() + (long)i + 1, {off + bytes, tail});
            } else if (tail) {
                free_[i] = {off + bytes, tail};
            } else {
                free_.erase(free_.begin() + (long)i);
            }
            return true;
        }
        return false;
    }
    void release(uint64_t off, uint64_t bytes) {
        bytes = align_up(bytes, 256);
        auto it = std::lower_bound(free_.begin(), free_.end(), std::make_pair(off, (uint64_t)0));
        it = free_.insert(it, {off, bytes});
        if (it + 1 != free_.end() && it->first + it->second == (it + 1)->first) {
            it->second += (it + 1)->second;
            free_.erase(it + 1);
        }
        if (it != free_.begin() && (it - 1)->first + (it - 1)->second == it->first) {
            (it - 1)->second += it->second;
            free_.erase(it);
        }
    }
};

// Start of a 256-aligned block of `need` bytes in [lo, hi) that overlaps none
// of the intervals [first, second) in `avoid`; UINT64_MAX if there is none.
// Candidates: the start of the range and the end of each interval (a block
// that fits anywhere still fits after sliding down to one of them), and the
// end of the range.
inline uint64_t free_spot(uint64_t lo, uint64_t hi, uint64_t need,
                          const std::vector<std::pair<uint64_t, uint64_t>>& avoid) {
    std::vector<uint64_t> at = {align_up(lo, 256)};
    if (hi >= need) at.push_back((hi - need) & ~255ull);
    for (const auto& iv : avoid) at.push_back(align_up(iv.second, 256));
    for (const uint64_t x : at) {
        if (x < lo || x + need > hi) continue;
        bool clear = true;
        for (const auto& iv : avoid) clear = clear && (x + need <= iv.first || iv.second <= x);
        if (clear) return x;
    }
    return UINT64_MAX;
}

}  // namespace ltlf
