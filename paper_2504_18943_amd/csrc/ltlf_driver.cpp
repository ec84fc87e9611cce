// Host driver and C ABI of the LTLf synthesiser (see include/ltlf.h).
//
// The driver owns the level loop of the bottom-up enumeration (paper,
// "Program synthesis": language cache by size, every level built from the
// cheaper ones) and everything around the kernels: validation, the device
// memory plan, the per-level block lists, launch chunking, deferral
// resolution, table growth, and witness reconstruction.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "../../include/ltlf.h"
#include "ltlf_internal.h"
#include "ltlf_host.h"

using namespace ltlf;

namespace {

constexpr uint64_t kMinWorkspace = 64ull << 20;
constexpr uint64_t kDefaultBudget = 2ull << 30;
constexpr uint32_t kMaxBound = 1024;
constexpr uint32_t kMaxTokens = kMaxBound + 1;
constexpr uint64_t kStagingBytes = 8ull << 20;
constexpr uint64_t kMinTableSlots = 1ull << 12;
constexpr uint64_t kLookaheadTiles = 1ull << 30;  // tiles per look-ahead launch (grid limit)
// Candidates per launch of the one-block-per-tile kernels (at most the
// deferral list): a candidate that meets a row of its own launch is
// deferred and verified afterwards, so smaller launches defer fewer.
#ifndef LTLF_LAUNCH_CANDIDATES
#define LTLF_LAUNCH_CANDIDATES (1ull << 27)
#endif
constexpr uint64_t kLaunchCandidates = LTLF_LAUNCH_CANDIDATES;
// Candidates per launch of the persistent kernels (a level larger than this
// runs as several launches, for the same reason)
#ifndef LTLF_PERSISTENT_CANDIDATES
#define LTLF_PERSISTENT_CANDIDATES (1ull << 25)
#endif
constexpr uint64_t kPersistentCandidates = LTLF_PERSISTENT_CANDIDATES;
// Share of the resident block slots (eighths) the large region's persistent
// launches take while small problems are on the device
#ifndef LTLF_BUSY_EIGHTHS
#define LTLF_BUSY_EIGHTHS 7
#endif
constexpr uint32_t kBusyEighths = LTLF_BUSY_EIGHTHS;

inline uint64_t pow2_ceil(uint64_t x) {
    uint64_t p = 1;
    while (p < x) p <<= 1;
    return p;
}

// One class of the kernel tuning table: rows of about `chunks` 16-byte
// chunks generate fastest with kernel `kind` (KERNEL_*), and the wave kernel
// there with pair tiles of side `wtile` (0: the built-in side).
struct TuneClass {
    uint32_t chunks, kind, wtile;
};

}  // namespace

struct ltlf_ctx {
    int device = 0;
    uint64_t budget = kDefaultBudget;
    char* ws = nullptr;
    uint64_t ws_bytes = 0;
    bool own_ws = false;

    // loaded specification
    bool loaded = false;
    uint32_t n_props = 0, n_traces = 0;
    uint64_t n_pos = 0;   // sum of lengths
    uint64_t n_bits = 0;  // sum of (length + 1)
    uint32_t Wp = 0;

    // device regions
    uint32_t *d_letters = nullptr, *d_lengths = nullptr, *d_pos_off = nullptr, *d_seg_off = nullptr;
    uint8_t* d_positive = nullptr;
    uint32_t* d_canon = nullptr;
    uint32_t *d_V = nullptr, *d_S = nullptr, *d_P0 = nullptr, *d_atoms = nullptr;
    unsigned long long* d_ctr = nullptr;
    unsigned long long* d_digest = nullptr;  // level digests, kMaxBound + 1 entries
    uint32_t* d_tokens = nullptr;
    uint64_t* d_stage = nullptr;
    Store st{};
    uint64_t table_max = 0;  // slots available
    uint64_t plan_cap = 0;   // rows that fit the workspace
    uint64_t row_limit = 0;  // caller's limit (0 = none)
    uint64_t lds_limit = 0;  // largest dynamic LDS per workgroup on the device

    // host mirrors
    unsigned long long* h_ctr = nullptr;  // pinned
    uint32_t* h_tokens = nullptr;         // pinned
    unsigned long long* h_dig = nullptr;  // pinned, level digests (kMaxBound + 1)
    // the scheduler's loads: pinned image of the input regions, the event
    // after its last copy, and whether that copy may still be in flight
    uint8_t* h_load = nullptr;
    uint64_t h_load_cap = 0;
    hipEvent_t ev_load = nullptr;
    bool h_load_busy = false;
    // events around a whole run (created with the context, so a run creates
    // no runtime objects)
    hipEvent_t ev0 = nullptr, ev1 = nullptr;    // ltlf_run
    hipEvent_t evb0 = nullptr, evb1 = nullptr;  // ltlf_solve_batch (whose problems may run ltlf_run)

    // last run
    bool ran = false;
    uint32_t levels_done = 0;
    std::vector<uint64_t> lstart, lcount;

    // description of the last failure (empty after a successful call)
    std::string err;

    // set by ltlf_ctx_cancel from any thread; taken (and cleared) by the
    // level loop of ltlf_run / ltlf_solve_batch between levels
    std::atomic<bool> cancel{false};

    // batched solving: export staging of this context (sub-contexts of a
    // batch need none), and the pooled sub-contexts with their pinned mirror
    uint64_t staging_bytes = kStagingBytes;
    std::vector<ltlf_ctx*> subs;
    unsigned long long* h_batch = nullptr;  // pinned, h_batch_cap counters
    uint64_t h_batch_cap = 0;

    // measured kernel choice per row-width class; empty = the built-in rule
    std::vector<TuneClass> tune;
    uint32_t wave_tile_force = 0;  // autotune's timed runs: this wave tile (0: the table's)
};

namespace {

// Failure helpers: every error path records what failed in ctx->err.
ltlf_status fail(ltlf_ctx* c, ltlf_status s, const char* what, hipError_t e = hipSuccess) {
    if (c) {
        c->err = what;
        if (e != hipSuccess) {
            c->err += ": ";
            c->err += hipGetErrorString(e);
        }
    }
    return s;
}
#define TRY_HIP(x)                                                   \
    do {                                                             \
        const hipError_t e_ = (x);                                   \
        if (e_ != hipSuccess) return fail(c, LTLF_EDEVICE, #x, e_);  \
    } while (0)
#define TRY(x)                                \
    do {                                      \
        ltlf_status s_ = (x);                 \
        if (s_ != LTLF_OK) return s_;         \
    } while (0)


// Bytes of the fixed regions of the workspace carve-up (plan_memory_impl
// follows them), each 256-byte aligned, for a specification of n_pos
// positions over T traces with m propositions and rows of Wp words; the rest
// of the size model (deferral lists, table, row store) is in ltlf_host.h.
uint64_t fixed_bytes(uint64_t n_pos, uint64_t T, uint64_t Wp, uint64_t m, uint64_t staging) {
    uint64_t off = 0;
    const uint64_t sizes[] = {4 * n_pos, 4 * T, 4 * (T + 1), 4 * (T + 1), T, 4 * n_pos, 4 * Wp, 4 * Wp, 4 * Wp,
                              4 * Wp * m, (uint64_t)8 * C_NUM, (uint64_t)8 * (kMaxBound + 1),
                              (uint64_t)4 * (1 + kMaxTokens + 3 * (kMaxTokens + 1)), staging};
    for (const uint64_t b : sizes)
        off = align_up(off, 256) + b;
    return align_up(off, 256);
}
// Carves the workspace.  Fixed regions first, then deferral lists, then the
// row store and the table, which take what is left.
ltlf_status plan_memory_impl(ltlf_ctx* c);
ltlf_status plan_memory(ltlf_ctx* c) {
    const ltlf_status s = plan_memory_impl(c);
    if (s != LTLF_OK) return fail(c, s, "workspace too small for this specification");
    return s;
}
ltlf_status plan_memory_impl(ltlf_ctx* c) {
    const uint64_t T = c->n_traces, Wp = c->Wp;
    uint64_t off = 0;
    auto take = [&](uint64_t bytes) {
        const uint64_t o = align_up(off, 256);
        off = o + bytes;
        return c->ws + o;
    };
    c->d_letters = reinterpret_cast<uint32_t*>(take(4 * c->n_pos));
    c->d_lengths = reinterpret_cast<uint32_t*>(take(4 * T));
    c->d_pos_off = reinterpret_cast<uint32_t*>(take(4 * (T + 1)));
    c->d_seg_off = reinterpret_cast<uint32_t*>(take(4 * (T + 1)));
    c->d_positive = reinterpret_cast<uint8_t*>(take(T));
    c->d_canon = reinterpret_cast<uint32_t*>(take(4 * c->n_pos));
    c->d_V = reinterpret_cast<uint32_t*>(take(4 * Wp));
    c->d_S = reinterpret_cast<uint32_t*>(take(4 * Wp));
    c->d_P0 = reinterpret_cast<uint32_t*>(take(4 * Wp));
    c->d_atoms = reinterpret_cast<uint32_t*>(take(4 * Wp * c->n_props));
    c->d_ctr = reinterpret_cast<unsigned long long*>(take(8 * C_NUM));
    c->d_digest = reinterpret_cast<unsigned long long*>(take(8 * (kMaxBound + 1)));
    c->d_tokens = reinterpret_cast<uint32_t*>(take(4 * (1 + kMaxTokens + 3 * (kMaxTokens + 1))));
    c->d_stage = reinterpret_cast<uint64_t*>(take(c->staging_bytes));
    off = align_up(off, 256);
    if (off >= c->ws_bytes) return LTLF_ENOMEM;
    uint64_t rest = c->ws_bytes - off;

    uint64_t d0, d1;
    deferral_records(rest, d0, d1);
    if ((d0 + d1) * 16 + 4096 >= rest) return LTLF_ENOMEM;
    c->st.def0 = reinterpret_cast<uint4*>(take(16 * d0));
    c->st.def1 = reinterpret_cast<uint4*>(take(16 * d1));
    c->st.def0_cap = d0;
    c->st.def1_cap = d1;
    off = align_up(off, 256);
    if (off >= c->ws_bytes) return LTLF_ENOMEM;
    rest = c->ws_bytes - off;

    // two table slots (16 bytes) per row; the table holds at most 2^32 slots
    const uint64_t per_row = 4 * Wp + 16;
    uint64_t cap = (rest - 3 * 256) / (per_row + 16);
    cap = std::min<uint64_t>(cap, (1ull << 31) - 16);
    const uint64_t slots = 2 * cap;
    if (cap < c->n_props + 16 || slots < kMinTableSlots) return LTLF_ENOMEM;
    c->st.table = reinterpret_cast<uint64_t*>(take(8 * slots));
    c->st.rows = reinterpret_cast<uint32_t*>(take(4 * Wp * cap));
    c->st.meta = reinterpret_cast<uint4*>(take(16 * cap));
    if (off > c->ws_bytes) return LTLF_ENOMEM;
    if (cap != row_capacity(fixed_bytes(c->n_pos, T, Wp, c->n_props, c->staging_bytes), Wp, c->ws_bytes))
        return LTLF_EDEVICE;  // the size model disagrees with the carve-up
    c->table_max = slots;
    c->plan_cap = cap;
    c->st.cap = cap;
    c->st.V = c->d_V;
    c->st.S = c->d_S;
    c->st.P0 = c->d_P0;
    c->st.atoms = c->d_atoms;
    c->st.ctr = c->d_ctr;
    c->st.Wp = c->Wp;
    c->st.n_props = c->n_props;
    c->st.hmask = ~0ull;
    return LTLF_OK;
}

ltlf_status ensure_workspace(ltlf_ctx* c) {
    if (c->ws) return LTLF_OK;
    TRY_HIP(hipSetDevice(c->device));
    void* p = nullptr;
    if (hipMalloc(&p, c->budget) != hipSuccess) {
        (void)hipGetLastError();
        return fail(c, LTLF_ENOMEM, "hipMalloc of the workspace failed");
    }
    c->ws = static_cast<char*>(p);
    c->ws_bytes = c->budget;
    c->own_ws = true;
    return LTLF_OK;
}

const char* op_token(uint32_t op) {
    switch (op) {
    case OP_NOT: return "!";
    case OP_X: return "X";
    case OP_F: return "F";
    case OP_G: return "G";
    case OP_AND: return "&";
    case OP_OR: return "|";
    case OP_U: return "U";
    default: return "?";
    }
}

// Runs the formula kernel from a root derivation (operator in bits 0..7 of
// op) and copies its prefix tokens to c->h_tokens on s; read them with
// decode_formula once s has been synchronised.
ltlf_status enqueue_formula(ltlf_ctx* c, uint32_t op, uint32_t a, uint32_t b, hipStream_t s) {
    TRY_HIP(launch_formula(c->st.meta, op & 0xFFu, a, b, kMaxTokens, c->d_tokens, s));
    TRY_HIP(hipMemcpyAsync(c->h_tokens, c->d_tokens, 4 * (1 + kMaxTokens), hipMemcpyDeviceToHost, s));
    return LTLF_OK;
}

// Renders the tokens in c->h_tokens.  Bits 8.. of op name a unary operator
// applied on top (a look-ahead witness).
ltlf_status decode_formula(ltlf_ctx* c, uint32_t op, std::string& out) {
    const uint32_t outer = op >> 8;
    const uint32_t n = c->h_tokens[0];
    if (n > kMaxTokens) return fail(c, LTLF_EDEVICE, "witness formula longer than the token buffer");
    out.clear();
    if (outer) out = std::string(op_token(outer)) + " ";
    for (uint32_t i = 0; i < n; ++i) {
        const uint32_t t = c->h_tokens[1 + i];
        const uint32_t top = t >> 24;
        if (i) out.push_back(' ');
        if (top == OP_ATOM) {
            out += "p" + std::to_string(t & 0xFFFFFFu);
        } else {
            out += op_token(top);
        }
    }
    return LTLF_OK;
}

// Witness formula of a root derivation, rendered (synchronises s).
ltlf_status render_formula(ltlf_ctx* c, uint32_t op, uint32_t a, uint32_t b, hipStream_t s,
                           std::string& out) {
    TRY(enqueue_formula(c, op, a, b, s));
    TRY_HIP(hipStreamSynchronize(s));
    return decode_formula(c, op, out);
}

struct LevelPlan {
    std::vector<Seg> segs;
    std::vector<uint64_t> cand_per_tile;
    uint64_t cand_ub = 0;
};

// Blocks of level c: atoms, unary operators over U_{c-k}, and for every pair
// of levels i <= j the binary operators whose cost closes the sum to c.  The
// larger operand level goes to the lanes; a pair (a, b) yields a&b, a|b,
// aUb and bUa, so each unordered pair of representatives is visited once.
LevelPlan plan_level(const ltlf_ctx* c, const ltlf_costs* k, uint32_t lev, const TileShape& ts) {
    LevelPlan p;
    auto cnt = [&](uint32_t i) -> uint64_t { return i < c->lcount.size() ? c->lcount[i] : 0; };
    auto ceil_div = [](uint64_t a, uint64_t b) { return (a + b - 1) / b; };
    if (lev == k->atom_cost) {
        Seg g{};
        g.kind = SEG_ATOM;
        g.nb = c->n_props;
        g.tiles = 1;
        p.segs.push_back(g);
        p.cand_per_tile.push_back(c->n_props);
    }
    // unary: group operators by source level
    const uint32_t umask[4] = {M_NOT, M_X, M_F, M_G};
    for (uint32_t src = 1; src < lev; ++src) {
        uint32_t mask = 0;
        for (int o = 0; o < 4; ++o)
            if (k->op_cost[o] && k->op_cost[o] + src == lev) mask |= umask[o];
        if (!mask || cnt(src) == 0) continue;
        Seg g{};
        g.kind = SEG_UNARY;
        g.opmask = mask;
        g.b0 = c->lstart[src];
        g.nb = cnt(src);
        g.tiles = ceil_div(g.nb, ts.tu);
        p.segs.push_back(g);
        p.cand_per_tile.push_back((uint64_t)std::min<uint64_t>(ts.tu, g.nb) * __builtin_popcount(mask));
    }
    // binary
    for (uint32_t i = 1; i < lev; ++i) {
        for (uint32_t j = i; i + j < lev; ++j) {
            uint32_t mask = 0;
            if (k->op_cost[LTLF_AND] && i + j + k->op_cost[LTLF_AND] == lev) mask |= M_AND;
            if (k->op_cost[LTLF_OR] && i + j + k->op_cost[LTLF_OR] == lev) mask |= M_OR;
            if (k->op_cost[LTLF_U] && i + j + k->op_cost[LTLF_U] == lev) mask |= M_UAB | M_UBA;
            if (!mask || cnt(i) == 0 || cnt(j) == 0) continue;
            Seg g{};
            g.kind = SEG_PAIR;
            g.opmask = mask;
            if (i == j) {
                const uint64_t n = cnt(i);
                if (n < 2) continue;
                g.tri = 1;
                g.a0 = g.b0 = c->lstart[i];
                g.na = g.nb = n;
                if (ts.square_tri) {
                    const uint64_t T = ceil_div(n, ts.ta);
                    g.tiles = T * (T + 1) / 2;
                } else {  // b-tile column k holds R(k+1) a-tiles, R = tb / ta
                    const uint64_t K = ceil_div(n, ts.tb);
                    g.tiles = (uint64_t)(ts.tb / ts.ta / 2) * (K - 1) * K + ceil_div(n, ts.ta);
                }
            } else {
                // lanes (the right operand) take the larger level
                uint32_t la = i, lb = j;
                if (cnt(i) > cnt(j)) std::swap(la, lb);
                g.a0 = c->lstart[la];
                g.na = cnt(la);
                g.b0 = c->lstart[lb];
                g.nb = cnt(lb);
                g.tiles = ceil_div(g.na, ts.ta) * ceil_div(g.nb, ts.tb);
            }
            p.segs.push_back(g);
            p.cand_per_tile.push_back(std::min<uint64_t>(ts.ta, g.na) * std::min<uint64_t>(ts.tb, g.nb) *
                                      __builtin_popcount(mask));
        }
    }
    for (size_t s = 0; s < p.segs.size(); ++s) p.cand_ub += p.segs[s].tiles * p.cand_per_tile[s];
    return p;
}

// Grows the table (clear + re-insert every stored row) so that it keeps at
// least two slots per row after `extra` more rows.  A growth re-inserts every
// stored row, so it goes at least to twice the size, and to room for `ahead`
// more rows (the rows expected before the next growth would otherwise come).
ltlf_status ensure_table(ltlf_ctx* c, uint64_t rows, uint64_t extra, hipStream_t s, uint64_t ahead = 0) {
    const uint64_t want = std::max<uint64_t>(2 * (rows + extra), kMinTableSlots);
    if (want <= c->st.tsize || c->st.tsize == c->table_max) return LTLF_OK;
    const uint64_t need = std::min<uint64_t>(
        std::max<uint64_t>(std::max<uint64_t>(want, 2 * (rows + ahead)), 2 * c->st.tsize), c->table_max);
    c->st.tsize = need;
    TRY_HIP(launch_fill_u64(c->st.table, need, ~0ull, s));
    TRY_HIP(launch_rehash(c->st, rows, s));
    return LTLF_OK;
}

ltlf_status read_counters(ltlf_ctx* c, hipStream_t s) {
    TRY_HIP(hipMemcpyAsync(c->h_ctr, c->d_ctr, 8 * C_NUM, hipMemcpyDeviceToHost, s));
    TRY_HIP(hipStreamSynchronize(s));
    return LTLF_OK;
}

// Events around generation/verification launches: mark() records one event;
// collect() adds the gaps (gen = mark0..mark1, verify = mark1..mark2, per
// launch triple) after the stream has been synchronised.
struct Profiler {
    ltlf_ctx* c = nullptr;
    std::vector<hipEvent_t> ev;
    size_t used = 0;
    ltlf_status mark(hipStream_t s) {
        if (used == ev.size()) {
            hipEvent_t e;
            TRY_HIP(hipEventCreate(&e));
            ev.push_back(e);
        }
        TRY_HIP(hipEventRecord(ev[used++], s));
        return LTLF_OK;
    }
    ltlf_status collect(double& gen_ms, double& ver_ms) {
        for (size_t i = 0; i + 2 < used; i += 3) {
            float a = 0.f, b = 0.f;
            TRY_HIP(hipEventElapsedTime(&a, ev[i], ev[i + 1]));
            TRY_HIP(hipEventElapsedTime(&b, ev[i + 1], ev[i + 2]));
            gen_ms += a;
            ver_ms += b;
        }
        used = 0;
        return LTLF_OK;
    }
    ~Profiler() {
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    }
};

uint32_t tuned_wave_tile(const ltlf_ctx* c);

// Start of a run: per-level bookkeeping, store settings, and on the stream
// (a1) encoding of the atoms and masks, counters reset, initial table.
ltlf_status begin_run(ltlf_ctx* c, uint32_t bound, uint32_t flags, uint32_t kernel, hipStream_t s) {
    c->ran = false;
    c->lstart.assign(bound + 1, 0);
    c->lcount.assign(bound + 1, 0);
    c->st.cap = c->plan_cap;  // the row limit is applied to live rows per level
    c->st.hmask = (flags & LTLF_FLAG_DEBUG_WEAK_HASH) ? 0x3Full : ~0ull;
    c->st.kernel = kernel;
    c->st.wtile = tuned_wave_tile(c);  // for any wave launch of the run (the look-ahead's too)
    TRY_HIP(launch_encode(c->d_letters, c->d_lengths, c->d_pos_off, c->d_seg_off, c->d_positive,
                          c->n_traces, c->n_props, c->Wp, c->d_V, c->d_S, c->d_P0, c->d_atoms, s));
    TRY_HIP(launch_fill_u64(reinterpret_cast<uint64_t*>(c->d_ctr), C_NUM, 0, s));
    if (flags & LTLF_FLAG_DIGEST)
        TRY_HIP(launch_fill_u64(reinterpret_cast<uint64_t*>(c->d_digest), kMaxBound + 1, 0, s));
    const uint64_t slots0 = std::min<uint64_t>(pow2_ceil(std::max<uint64_t>(4ull * c->n_props, kMinTableSlots)),
                                               c->table_max);
    c->st.tsize = slots0;
    TRY_HIP(launch_fill_u64(c->st.table, slots0, ~0ull, s));
    return LTLF_OK;
}

void reset_result(ltlf_result* res, uint32_t row_bytes) {
    res->status = LTLF_NOT_FOUND;
    res->min_cost = 0;
    res->levels_done = 0;
    res->overflow_level = 0;
    res->checked_level = 0;
    res->formula_len = 0;
    res->candidates = 0;
    res->unique_total = 0;
    res->deferred = 0;
    res->row_bytes = row_bytes;
    res->gen_launches = 0;
    res->verify_launches = 0;
    res->enum_ms = 0.0;
    res->gen_ms = 0.0;
    res->verify_ms = 0.0;
    res->dead_rows = 0;
}

// Level digests of levels 1..levels_done into out[0..len) (0 elsewhere);
// zeros when they were not computed.  take_digests reads them from c->h_dig
// (copied there on s, and s synchronised); copy_digests copies and waits.
void take_digests(const ltlf_ctx* c, uint32_t levels_done, bool computed, uint64_t* out, uint32_t len) {
    for (uint32_t i = 0; i < len; ++i)
        out[i] = (computed && i >= 1 && i <= levels_done && i <= kMaxBound) ? c->h_dig[i] : 0;
}
ltlf_status copy_digests(ltlf_ctx* c, uint32_t levels_done, bool computed, uint64_t* out, uint32_t len,
                         hipStream_t s) {
    if (computed) {
        TRY_HIP(hipMemcpyAsync(c->h_dig, c->d_digest, 8 * (kMaxBound + 1), hipMemcpyDeviceToHost, s));
        TRY_HIP(hipStreamSynchronize(s));
    }
    take_digests(c, levels_done, computed, out, len);
    return LTLF_OK;
}

// Copies the witness formula (or an empty string), the level counts and
// digests of a finished run into the caller's buffers.
ltlf_status finish_result(ltlf_ctx* c, ltlf_result* res, ltlf_status status, uint32_t wit_op, uint32_t wit_a,
                          uint32_t wit_b, bool digests, hipStream_t s) {
    uint64_t uniq = 0;
    for (uint32_t lev = 1; lev <= res->levels_done; ++lev) uniq += c->lcount[lev];
    res->unique_total = uniq;
    res->checked_level = std::max({res->checked_level, res->levels_done, res->overflow_level});
    if (res->level_counts) {
        for (uint32_t i = 0; i < res->level_counts_len; ++i)
            res->level_counts[i] = (i <= res->levels_done && i < c->lcount.size()) ? c->lcount[i] : 0;
    }
    if (res->level_digests) TRY(copy_digests(c, res->levels_done, digests, res->level_digests,
                                            res->level_counts_len, s));
    res->status = status;
    if (status == LTLF_OK) {
        std::string f;
        TRY(render_formula(c, wit_op, wit_a, wit_b, s, f));
        res->formula_len = f.size() + 1;
        if (res->formula) {
            if (res->formula_cap < f.size() + 1) return LTLF_EBUFSZ;
            std::memcpy(res->formula, f.c_str(), f.size() + 1);
        }
    } else if (res->formula && res->formula_cap) {
        res->formula[0] = 0;
        res->formula_len = 1;
    }
    return LTLF_OK;
}

ltlf_status validate_spec(const ltlf_spec* sp) {
    if (!sp || !sp->lengths || !sp->letters || !sp->positive) return LTLF_EINVAL;
    if (sp->n_props < 1 || sp->n_props > 32 || sp->n_traces < 1) return LTLF_EINVAL;
    uint64_t total = 0;
    for (uint32_t t = 0; t < sp->n_traces; ++t) {
        if (sp->lengths[t] < 1) return LTLF_EINVAL;
        total += sp->lengths[t];
    }
    const uint32_t bad = sp->n_props == 32 ? 0u : ~((1u << sp->n_props) - 1u);
    for (uint64_t i = 0; i < total; ++i)
        if (sp->letters[i] & bad) return LTLF_EINVAL;
    return LTLF_OK;
}

// Sizes of specification sp recorded in c and the workspace carved for it
// (nothing is copied yet; c is not loaded afterwards).
ltlf_status load_layout(ltlf_ctx* c, const ltlf_spec* sp) {
    TRY(validate_spec(sp));
    TRY_HIP(hipSetDevice(c->device));
    TRY(ensure_workspace(c));
    const uint32_t T = sp->n_traces;
    uint64_t n_pos = 0;
    for (uint32_t t = 0; t < T; ++t) n_pos += sp->lengths[t];
    c->loaded = false;
    c->ran = false;
    c->n_props = sp->n_props;
    c->n_traces = T;
    c->n_pos = n_pos;
    c->n_bits = n_pos + T;
    c->Wp = (uint32_t)align_up((c->n_bits + 31) / 32, 4);
    return plan_memory(c);
}

// Bytes of the input regions (raw letters, lengths, position and segment
// offsets, labels, canonical bit map), which the carve-up lays out one after
// another from d_letters.
uint64_t input_bytes(const ltlf_ctx* c) {
    return (uint64_t)(reinterpret_cast<const char*>(c->d_canon) - reinterpret_cast<const char*>(c->d_letters)) +
           4 * c->n_pos;
}

// The device image of the input regions of sp (after load_layout) written to
// img[0, input_bytes(c)): the raw traces, per-trace position offsets, segment
// offsets (length + 1 bits per trace, guard bit included), labels, and the
// map from canonical bit (trace t, position k) to the packed bit of that
// position.
void fill_inputs(const ltlf_ctx* c, const ltlf_spec* sp, uint8_t* img) {
    const char* base = reinterpret_cast<const char*>(c->d_letters);
    auto at = [&](const void* d) { return img + (reinterpret_cast<const char*>(d) - base); };
    const uint32_t T = c->n_traces;
    std::memset(img, 0, input_bytes(c));
    std::memcpy(img, sp->letters, 4 * c->n_pos);
    std::memcpy(at(c->d_lengths), sp->lengths, 4ull * T);
    std::memcpy(at(c->d_positive), sp->positive, T);
    uint32_t* pos_off = reinterpret_cast<uint32_t*>(at(c->d_pos_off));
    uint32_t* seg_off = reinterpret_cast<uint32_t*>(at(c->d_seg_off));
    uint32_t* canon = reinterpret_cast<uint32_t*>(at(c->d_canon));
    pos_off[0] = seg_off[0] = 0;
    for (uint32_t t = 0; t < T; ++t) {
        const uint32_t n = sp->lengths[t];
        pos_off[t + 1] = pos_off[t] + n;
        seg_off[t + 1] = seg_off[t] + n + 1;
        for (uint32_t k = 0; k < n; ++k) canon[pos_off[t] + k] = seg_off[t] + (n - 1 - k);
    }
}

// Load for the scheduler's sub-contexts: the image goes through the
// context's pinned buffer in one copy on s, without waiting for it (work on
// the region is ordered after it on s; callers that hand the region to
// another stream synchronise s first).  The buffer is rewritten only after
// the previous copy from it has completed.
ltlf_status load_staged(ltlf_ctx* c, const ltlf_spec* sp, hipStream_t s) {
    TRY(load_layout(c, sp));
    const uint64_t bytes = input_bytes(c);
    if (c->h_load_busy) {
        TRY_HIP(hipEventSynchronize(c->ev_load));
        c->h_load_busy = false;
    }
    if (!c->ev_load) TRY_HIP(hipEventCreateWithFlags(&c->ev_load, hipEventDisableTiming));
    if (bytes > c->h_load_cap) {
        if (c->h_load) (void)hipHostFree(c->h_load);
        c->h_load = nullptr;
        c->h_load_cap = 0;
        const uint64_t cap = align_up(bytes, 1ull << 16);
        TRY_HIP(hipHostMalloc(reinterpret_cast<void**>(&c->h_load), cap, hipHostMallocDefault));
        c->h_load_cap = cap;
    }
    fill_inputs(c, sp, c->h_load);
    TRY_HIP(hipMemcpyAsync(c->d_letters, c->h_load, bytes, hipMemcpyHostToDevice, s));
    TRY_HIP(hipEventRecord(c->ev_load, s));
    c->h_load_busy = true;
    c->loaded = true;
    return LTLF_OK;
}


// Built-in choice: the lane kernel wherever one of its tiles (256 or 128
// lanes) fits the LDS, else the group kernel up to 64 chunks, else the wave
// kernel (measured: the 128-lane form beats group and wave by 1.5..2x at
// 38..64 chunks).
constexpr uint32_t kBuiltinPref = KERNEL_LANE;

// The measured kernel for the loaded row width: the tuning class nearest to
// it on a log scale; the built-in choice without a table.
const TuneClass* tuned_class(const ltlf_ctx* c) {
    if (c->tune.empty()) return nullptr;
    const double w = std::log((double)std::max<uint32_t>(1, c->Wp / 4));
    double best = 1e300;
    const TuneClass* pick = nullptr;
    for (const auto& t : c->tune) {
        const double d = std::fabs(std::log((double)t.chunks) - w);
        if (d < best) {
            best = d;
            pick = &t;
        }
    }
    return pick;
}
uint32_t tuned_kernel(const ltlf_ctx* c) {
    const TuneClass* t = tuned_class(c);
    return t ? t->kind : kBuiltinPref;
}

// The wave kernel's pair-tile side for the loaded row width (the tuning
// class's, else the built-in one), and the generation kernel and tile shape
// for preference pref with it.  Every plan and every launch of a run takes
// the wave tile from here (the store carries it to the kernels).
uint32_t tuned_wave_tile(const ltlf_ctx* c) {
    if (c->wave_tile_force) return c->wave_tile_force;
    const TuneClass* t = tuned_class(c);
    return t && wave_tile_ok(t->wtile) ? t->wtile : kWaveTileBuiltin;
}
TileShape shape_of(const ltlf_ctx* c, uint32_t pref) {
    return tile_shape(c->Wp, c->lds_limit, pref, tuned_wave_tile(c));
}

// One single-problem run, level by level: the level loop of ltlf_run, also
// used by the scheduler for resident problems whose levels are large (they
// keep the single-problem kernels and table sizing).
struct LevelRun {
    ltlf_ctx* c = nullptr;
    const ltlf_costs* k = nullptr;
    uint32_t bound = 0, flags = 0;
    bool exhaust = false, profile = false;
    TileShape shape{};
    Profiler prof;
    ltlf_result* res = nullptr;
    uint64_t rows = 0, candidates = 0;
    ltlf_status status = LTLF_NOT_FOUND;
    uint32_t wit_op = 0, wit_a = 0, wit_b = 0;
    bool stop = false;  // the run ended: a separating level without EXHAUST, or an overflow
    uint32_t grid_eighths = 8;  // share of the resident blocks a persistent launch takes
    // Set by the scheduler when the store is a region sized by forecast: a
    // level that overflows it is dropped (overflowed = true, nothing of it
    // kept, the run's state as the previous level left it) to be run again
    // in a larger region, instead of ending the run.
    bool redo_overflow = false, overflowed = false;

    ltlf_status begin(ltlf_ctx* ctx, const ltlf_costs* costs, uint32_t cost_bound, uint32_t run_flags,
                      ltlf_result* result, hipStream_t s) {
        c = ctx;
        k = costs;
        bound = cost_bound;
        flags = run_flags;
        exhaust = (flags & LTLF_FLAG_EXHAUST) != 0;
        profile = (flags & LTLF_FLAG_PROFILE) != 0;
        res = result;
        prof.c = c;
        const uint32_t pref = (flags & LTLF_FLAG_KERNEL_WAVE)    ? KERNEL_WAVE
                              : (flags & LTLF_FLAG_KERNEL_GROUP) ? KERNEL_GROUP
                              : (flags & LTLF_FLAG_KERNEL_LANE)  ? KERNEL_LANE
                                                                 : tuned_kernel(c);
        shape = shape_of(c, pref);
        rows = 0;
        candidates = 0;
        status = LTLF_NOT_FOUND;
        stop = false;
        return begin_run(c, bound, flags, shape.kind, s);
    }

    // Continues a run whose levels up to the last closed one are stored in
    // ctx (moved there from another region, see Scheduler::migrate): the
    // store, its counters and the level bookkeeping are as that level left
    // them; rows_now rows are stored, cand_now candidates were generated.
    void resume(ltlf_ctx* ctx, const ltlf_costs* costs, uint32_t cost_bound, uint32_t run_flags, ltlf_result* result,
                uint64_t rows_now, uint64_t cand_now, ltlf_status status_now, uint32_t wo, uint32_t wa,
                uint32_t wb) {
        c = ctx;
        k = costs;
        bound = cost_bound;
        flags = run_flags;
        exhaust = (flags & LTLF_FLAG_EXHAUST) != 0;
        profile = (flags & LTLF_FLAG_PROFILE) != 0;
        res = result;
        prof.c = c;
        shape = shape_of(c, tuned_kernel(c));
        c->st.kernel = shape.kind;
        c->st.wtile = tuned_wave_tile(c);
        rows = rows_now;
        candidates = cand_now;
        status = status_now;
        wit_op = wo;
        wit_a = wa;
        wit_b = wb;
        stop = false;
    }

    // The level after `lev`, which overflowed with no separating candidate,
    // checked without storing anything.  Its candidates over stored levels
    // (binary operators, unary operators of cost >= 2: every operand level is
    // below lev) run through the generation kernels with the overflow flag
    // set, so each is only checked; those over level lev (unary operators of
    // cost 1) through the look-ahead kernel, which generates every candidate
    // of lev again and checks the operators' images of it.
    ltlf_status lookahead(uint32_t lev, hipStream_t s) {
        const uint32_t next = lev + 1;
        TRY_HIP(launch_set_counter(c->d_ctr, C_OVERFLOW, 1, s));
        auto launch_groups = [&](const LevelPlan& p, auto&& launch) -> ltlf_status {
            for (size_t g0 = 0; g0 < p.segs.size(); g0 += kMaxSegs) {
                const size_t g1 = std::min(p.segs.size(), g0 + kMaxSegs);
                SegTable t{};
                t.n = (uint32_t)(g1 - g0);
                for (size_t q = g0; q < g1; ++q) {
                    t.seg[q - g0] = p.segs[q];
                    t.first[q - g0 + 1] = t.first[q - g0] + p.segs[q].tiles;
                }
                TRY(launch(t, t.first[t.n]));
            }
            return LTLF_OK;
        };
        // lcount[lev] is 0 now: the plan of the next level has no operand in lev
        const LevelPlan p = plan_level(c, k, next, shape);
        TRY(launch_groups(p, [&](SegTable& t, uint64_t total) -> ltlf_status {
            if (shape.kind == KERNEL_GROUP || shape.kind == KERNEL_WAVE) {
                uint64_t blocks = 0;
                TRY_HIP(generate_blocks(c->st, total, blocks));
                t.tile_begin = 0;
                t.tile_end = total;
                t.tile_stop = total;
                t.def_margin = t.row_margin = 0;
                t.row_budget = ~0ull;
                TRY_HIP(launch_set_counter(c->d_ctr, C_TILE, 0, s));
                TRY_HIP(launch_generate(c->st, t, blocks, s));
                ++res->gen_launches;
                return LTLF_OK;
            }
            for (uint64_t tile = 0; tile < total; tile += kLookaheadTiles) {
                t.tile_begin = tile;
                t.tile_end = std::min<uint64_t>(total, tile + kLookaheadTiles);
                TRY_HIP(launch_generate(c->st, t, 0, s));
                ++res->gen_launches;
            }
            return LTLF_OK;
        }));
        uint32_t omask = 0;
        for (uint32_t o = 0; o < 4; ++o)
            if (k->op_cost[o] == 1) omask |= 1u << o;
        if (omask) {
            const LevelPlan q = plan_level(c, k, lev, shape_of(c, KERNEL_WAVE));
            TRY(launch_groups(q, [&](SegTable& t, uint64_t total) -> ltlf_status {
                for (uint64_t tile = 0; tile < total; tile += kLookaheadTiles) {
                    t.tile_begin = tile;
                    t.tile_end = std::min<uint64_t>(total, tile + kLookaheadTiles);
                    TRY_HIP(launch_lookahead(c->st, t, omask, s));
                    ++res->gen_launches;
                }
                return LTLF_OK;
            }));
        }
        TRY(read_counters(c, s));
        res->checked_level = next;
        if (c->h_ctr[C_FOUND]) {
            status = LTLF_OK;
            res->min_cost = next;
            wit_op = (uint32_t)c->h_ctr[C_WIT_OP];
            wit_a = (uint32_t)c->h_ctr[C_WIT_A];
            wit_b = (uint32_t)c->h_ctr[C_WIT_B];
        }
        return LTLF_OK;
    }

    // Level `lev` (levels are run in order from 1): generation, dedup, check,
    // close.  Sets `stop` when the run ends at this level.
    ltlf_status level(uint32_t lev, hipStream_t s) {
        c->lstart[lev] = rows;
        const uint64_t cand_before = candidates;
        LevelPlan p = plan_level(c, k, lev, shape);
        if (p.segs.empty()) {
            res->levels_done = lev;
            return LTLF_OK;
        }
        // Size the table for this level from the growth of the previous
        // levels (1.5x margin, never above the candidate bound); the guard
        // below keeps >= 2 slots per row that can exist after the next chunk
        // whatever the estimate, growing the table between chunks if needed.
        // rows_ub is an upper bound on the rows stored so far (kept without
        // a sync).
        // A growth is sized for the next level too (same growth ratio), so
        // the largest stored rows are not re-inserted twice.
        uint64_t ahead = 0;
        {
            uint64_t est = p.cand_ub;
            if (lev >= 3 && c->lcount[lev - 1] && c->lcount[lev - 2]) {
                const double ratio = (double)c->lcount[lev - 1] / (double)c->lcount[lev - 2];
                est = std::min<uint64_t>(est, (uint64_t)(1.5 * ratio * (double)c->lcount[lev - 1]) + 4096);
                if (lev < bound) ahead = est + (uint64_t)(ratio * (double)est);
            }
            ahead = std::min<uint64_t>(std::max(ahead, est), c->st.cap - rows);
            TRY(ensure_table(c, rows, std::min<uint64_t>(est, c->st.cap - rows), s, ahead));
        }
        uint64_t rows_ub = rows;
        TRY_HIP(launch_set_counter(c->d_ctr, C_DEAD, 0, s));
        const bool persistent = shape.kind == KERNEL_GROUP || shape.kind == KERNEL_WAVE;
        // launch in groups of at most kMaxSegs segments
        for (size_t g0 = 0; g0 < p.segs.size(); g0 += kMaxSegs) {
            const size_t g1 = std::min(p.segs.size(), g0 + kMaxSegs);
            SegTable t{};
            t.n = (uint32_t)(g1 - g0);
            t.first[0] = 0;
            for (size_t q = g0; q < g1; ++q) {
                t.seg[q - g0] = p.segs[q];
                t.first[q - g0 + 1] = t.first[q - g0] + p.segs[q].tiles;
            }
            const uint64_t total = t.first[t.n];
            if (persistent) {
                // persistent group kernel: resident blocks pull tiles from a
                // cursor and stop while the deferral list or the table could
                // not take every candidate of the tiles in flight (one per
                // block, plus each wave's allocation chunk); the host empties
                // the list, grows the table if needed, and launches again
                uint64_t per_tile = 0;
                for (size_t q = g0; q < g1; ++q) per_tile = std::max(per_tile, p.cand_per_tile[q]);
                const uint64_t per_block = per_tile + (kLanes / 64) * kAllocChunk;
                uint64_t blocks = 0;
                TRY_HIP(generate_blocks(c->st, total, blocks));
                blocks = std::max<uint64_t>(1, blocks * grid_eighths / 8);
                blocks = std::max<uint64_t>(1, std::min<uint64_t>(blocks, c->st.def0_cap / (2 * per_block)));
                const uint64_t margin = blocks * per_block;
                const uint64_t share = std::max<uint64_t>(1, kPersistentCandidates / std::max<uint64_t>(per_tile, 1));
                t.tile_begin = 0;
                t.tile_end = total;
                t.def_margin = margin;
                t.row_margin = margin;
                TRY_HIP(launch_set_counter(c->d_ctr, C_TILE, 0, s));
                uint64_t taken = 0, ctr_rows = rows_ub;
                for (;;) {
                    if (2 * (ctr_rows + margin) > c->st.tsize && c->st.tsize < c->table_max) {
                        // room for the margin, and for the rest of the group at
                        // the yield seen so far
                        uint64_t extra = margin;
                        if (taken > 0 && ctr_rows > rows)
                            extra = std::max<uint64_t>(
                                extra, (uint64_t)(1.25 * (double)(ctr_rows - rows) / (double)taken *
                                                  (double)(total - taken)));
                        const uint64_t stored = std::min<uint64_t>(ctr_rows, c->st.cap);
                        TRY(ensure_table(c, stored, extra + (ctr_rows - stored), s));
                    }
                    t.row_budget = c->st.tsize < c->table_max ? c->st.tsize / 2 : ~0ull;
                    t.tile_stop = std::min<uint64_t>(total, taken + share);
                    if (profile) TRY(prof.mark(s));
                    TRY_HIP(launch_generate(c->st, t, blocks, s));
                    if (profile) TRY(prof.mark(s));
                    TRY_HIP(launch_verify_deferred(c->st, s));
                    if (profile) TRY(prof.mark(s));
                    ++res->gen_launches;
                    ++res->verify_launches;
                    TRY_HIP(launch_between(c->d_ctr, s));
                    TRY(read_counters(c, s));
                    const uint64_t now_taken = std::min<uint64_t>(c->h_ctr[C_TILE], total);
                    ctr_rows = c->h_ctr[C_ROWS];
                    if (now_taken >= total) break;
                    if (now_taken == taken) {  // not expected: the table was sized for the margin
                        if (c->st.tsize >= c->table_max)
                            return fail(c, LTLF_EDEVICE, "generation made no progress");
                        const uint64_t stored = std::min<uint64_t>(ctr_rows, c->st.cap);
                        TRY(ensure_table(c, stored, c->st.tsize, s));
                    }
                    taken = now_taken;
                }
                rows_ub = std::min<uint64_t>(ctr_rows, c->st.cap);
                continue;
            }
            // one block per tile: split into launches whose candidates fit
            // the deferral list
            uint64_t tile = 0;
            while (tile < total) {
                const uint64_t launch_cap = std::min<uint64_t>(c->st.def0_cap, kLaunchCandidates);
                uint64_t budget = launch_cap, end = tile;
                uint32_t si = 0;
                while (end < total) {
                    while (t.first[si + 1] <= end) ++si;
                    const uint64_t per = p.cand_per_tile[g0 + si];
                    const uint64_t seg_end = t.first[si + 1];
                    const uint64_t fit = budget / per;
                    if (fit == 0) break;
                    const uint64_t take = std::min<uint64_t>(fit, seg_end - end);
                    end += take;
                    budget -= take * per;
                }
                if (end == tile) return fail(c, LTLF_EDEVICE, "a tile exceeds the deferral list");
                const uint64_t chunk = launch_cap - budget;  // candidates, upper bound
                if (2 * (rows_ub + chunk) > c->st.tsize) {
                    TRY(read_counters(c, s));
                    rows_ub = std::min<uint64_t>(c->h_ctr[C_ROWS], c->st.cap);
                    TRY(ensure_table(c, rows_ub, std::min<uint64_t>(chunk, c->st.cap - rows_ub), s,
                                     ahead > rows_ub - rows ? ahead - (rows_ub - rows) : 0));
                }
                rows_ub = std::min<uint64_t>(rows_ub + chunk, c->st.cap);
                t.tile_begin = tile;
                t.tile_end = end;
                if (profile) TRY(prof.mark(s));
                TRY_HIP(launch_generate(c->st, t, 0, s));
                if (profile) TRY(prof.mark(s));
                TRY_HIP(launch_verify_deferred(c->st, s));
                if (profile) TRY(prof.mark(s));
                ++res->gen_launches;
                ++res->verify_launches;
                TRY_HIP(launch_between(c->d_ctr, s));
                tile = end;
            }
        }
        TRY(read_counters(c, s));
        if (profile) TRY(prof.collect(res->gen_ms, res->verify_ms));
        // rare: deferred candidates that were new after all.  Every round
        // inserts or resolves at least one record (a record is deferred again
        // only after meeting a row that another record of the same round
        // inserted), so the loop ends within n0 rounds.
        const uint64_t n0 = c->h_ctr[C_DEF1];
        for (uint64_t round = 0; c->h_ctr[C_DEF1] > 0 && !c->h_ctr[C_DEF_OVF]; ++round) {
            if (round > n0 + 16) return fail(c, LTLF_EDEVICE, "re-insertion rounds made no progress");
            const uint64_t n = c->h_ctr[C_DEF1];
            const uint64_t now_rows = std::min<uint64_t>(c->h_ctr[C_ROWS], c->st.cap);
            TRY(ensure_table(c, now_rows, std::min<uint64_t>(n, c->st.cap - now_rows), s));
            TRY_HIP(launch_reinsert(c->st, n, s));
            TRY_HIP(launch_set_counter(c->d_ctr, C_DEF1, 0, s));
            TRY_HIP(launch_verify_deferred(c->st, s));
            TRY_HIP(launch_between(c->d_ctr, s));
            TRY(read_counters(c, s));
        }
        if (c->h_ctr[C_DEF_OVF]) return fail(c, LTLF_EDEVICE, "deferral list overflow");
        const uint64_t now = std::min<uint64_t>(c->h_ctr[C_ROWS], c->st.cap);
        const uint64_t dead = c->h_ctr[C_DEAD];
        res->dead_rows += dead;
        if (dead > now - rows) return fail(c, LTLF_EDEVICE, "dead row count exceeds the level");
        const uint64_t live_end = now - dead;
        candidates = c->h_ctr[C_CAND];
        // the caller's row limit counts live rows only (unused allocation
        // tails do not count against it)
        const bool overflow = c->h_ctr[C_OVERFLOW] != 0 || (c->row_limit && live_end > c->row_limit);
        if (redo_overflow && c->h_ctr[C_OVERFLOW]) {
            c->lcount[lev] = 0;
            candidates = cand_before;
            overflowed = true;
            stop = true;
            return LTLF_OK;
        }
        if (!overflow && dead) {
            // move the live rows above live_end into the holes below it, in
            // rounds of at most `lcap` (the deferral list is free now)
            const uint64_t lcap = 2 * c->st.def0_cap;
            uint32_t* holes = reinterpret_cast<uint32_t*>(c->st.def0);
            for (uint64_t done = 0; done < dead; done += lcap) {
                TRY_HIP(launch_set_counter(c->d_ctr, C_NH, 0, s));
                TRY_HIP(launch_set_counter(c->d_ctr, C_NM, 0, s));
                TRY_HIP(launch_compact(c->st, rows, live_end, now, holes, holes + lcap, lcap, s));
            }
            // the next level allocates from the compacted end, and its first
            // launch treats exactly the rows below it as written before it
            TRY_HIP(launch_set_counter(c->d_ctr, C_ROWS, live_end, s));
            TRY_HIP(launch_set_counter(c->d_ctr, C_SNAP, live_end, s));
        }
        c->lcount[lev] = live_end - rows;
        if (!overflow && (flags & LTLF_FLAG_DIGEST))
            TRY_HIP(launch_digest(c->st.rows, c->Wp, rows, live_end - rows, c->d_digest + lev, s));
        rows = live_end;
        if (c->h_ctr[C_FOUND] && status != LTLF_OK) {
            status = LTLF_OK;
            res->min_cost = lev;
            wit_op = (uint32_t)c->h_ctr[C_WIT_OP];
            wit_a = (uint32_t)c->h_ctr[C_WIT_A];
            wit_b = (uint32_t)c->h_ctr[C_WIT_B];
        }
        if (overflow) {
            if (status != LTLF_OK) status = LTLF_CAPACITY;
            res->overflow_level = lev;
            c->lcount[lev] = 0;
            stop = true;
            if (status == LTLF_CAPACITY && lev < bound && !(flags & LTLF_FLAG_NO_LOOKAHEAD)) TRY(lookahead(lev, s));
            return LTLF_OK;
        }
        res->levels_done = lev;
        if (status == LTLF_OK && !exhaust) stop = true;
        return LTLF_OK;
    }
};

// ------------------------------------------------------------ scheduler --
// Many problems on one device at once (batched solving and the request
// server).  The workspace holds a control region, a small pool and a large
// area, each carved into regions by a first-fit allocator.  A job (one
// problem) owns one region, used as an ordinary sub-context (row store,
// derivations, table, deferral lists, counters, digests), and is either
//   small: its levels are small (at most kBigLevel candidates); one step of
//     the scheduler advances every small job by one level with one batched
//     generation launch (the wave kernel's tile body over pieces of every
//     job's level plan), one verification launch per deferral budget and one
//     transfer of all counters; or
//   large: it runs the single-problem level loop (LevelRun, the loop of
//     ltlf_run) on a worker thread with a stream of its own while the main
//     thread keeps stepping the small jobs; several large jobs run at once
//     when their regions fit the large area.
// A job starts with a region for the first few thousand rows.  Before each
// level a small job's region must hold the level's worst case (every
// candidate a new row), a large job's the level's forecast (the growth ratio
// of the levels before it, with a margin).  Otherwise the job moves to a
// larger region: its stored levels (rows, derivation records, digests) are
// copied to the same indices there and its table is rebuilt from the records,
// so no level is enumerated twice (a small job whose next level is large
// moves into the large area the same way).  A large level that overflows a
// region sized by forecast is dropped and run again in a region sized for
// its worst case.  A job that needs more than half the large area for its
// next level, or is expected to for the level after it, waits for the whole
// area; the first such job that holds a region keeps it and takes the whole
// area with its stored levels (in place where its region lines up with the
// whole area's layout, else through a staging block), the others start over
// there.  The large area is a request's capacity, and every result equals
// ltlf_solve's with a workspace of the large area's size (status, minimal
// cost, levels, overflow level, counts and sets), hence ltlf_solve's on the
// same context whenever the run does not overflow it.

struct Job {
    enum Mode : uint32_t { QUEUED, SMALL, LARGE, FINISHED };
    uint64_t ticket = 0;
    uint32_t n_props = 0;
    std::vector<uint32_t> lengths, letters;
    std::vector<uint8_t> positive;
    ltlf_costs costs{};
    uint32_t bound = 0, flags = 0, wp = 0;
    uint64_t n_pos = 0;
    uint64_t want = 0;  // caller's first region in bytes (0: the forecast)
    Mode mode = QUEUED;
    bool done = false;
    ltlf_ctx* sub = nullptr;  // sub-context on the region
    Arena* arena = nullptr;   // owner of the region (nullptr: none)
    uint64_t off = 0, bytes = 0;
    bool full = false;  // the region is the whole large area
    bool aligned = false;  // the region's rows sit where the whole area's layout puts them
    uint32_t lev = 0;   // last closed level
    uint64_t rows = 0, next_tile = 0, total = 0;
    uint64_t need_rows = 0;  // rows the next level may need (a request for a larger region)
    uint32_t redo_level = 0;  // a level that overflowed a region sized by forecast
    bool early_full = false;  // asked for the whole area a level ahead (big_loop)
    LevelPlan plan;
    ltlf_status status = LTLF_NOT_FOUND;
    uint32_t wit_op = 0, wit_a = 0, wit_b = 0;
    ltlf_result res{};
    std::vector<uint64_t> counts, digests;
    std::string formula;
    std::unique_ptr<LevelRun> run;  // large jobs
    // the large job's worker (running, stop and grow are guarded by Scheduler::mu)
    std::thread worker;
    hipStream_t stream = nullptr;
    bool running = false, stop = false, grow = false;
    ltlf_status wstatus = LTLF_OK;
    ltlf_spec spec() const {
        return ltlf_spec{n_props, (uint32_t)lengths.size(), lengths.data(), letters.data(), positive.data()};
    }
};

struct Scheduler {
    ltlf_ctx* c = nullptr;
    uint32_t max_resident = 0;
    uint64_t base = 0;
    Arena small, large;
    std::deque<Job*> queue;        // not started
    std::deque<Job*> grow_queue;   // waiting for a larger region in the large area (region kept)
    std::deque<Job*> full_queue;   // waiting for the whole large area (to start there)
    std::deque<Job*> solo_queue;   // fixed regions beyond the large area: the whole workspace
    std::vector<Job*> resident;    // small jobs
    std::vector<Job*> bigs;        // large jobs with a worker (running, or finished and not yet reaped)
    std::map<uint64_t, Job*> jobs;
    std::vector<ltlf_ctx*> used;   // sub-contexts held by jobs
    std::vector<hipStream_t> streams;  // one per large job slot, reused
    uint64_t next_ticket = 1;
    Store* d_stores = nullptr;
    BSeg* d_segs = nullptr;
    unsigned long long* d_gather = nullptr;
    uint32_t launches = 0;
    // the small pool's batched launch: replayed as a graph, or (LTLF_NO_GRAPH
    // set) the same launches issued one by one
    StepGraphs graphs;
    bool use_graphs = true;
    hipStream_t graph_stream = nullptr;  // where the graph was last replayed
    bool graph_launched = false;
    bool trace = false;  // LTLF_TRACE set: one line per job event on stderr
    // small-pool statistics (reported with the trace): steps with small jobs,
    // their batched launches, wall time in those steps and, within it, time
    // waiting for the device
    uint64_t small_steps = 0;
    double small_step_s = 0.0, small_wait_s = 0.0, admit_s = 0.0, plan_s = 0.0, close_s = 0.0;
    double forecast_margin = 1.5;  // LTLF_FORECAST_SCALE: margin of the large jobs' forecasts
    bool always_stage = false;     // LTLF_PROMOTE_STAGED: promote() stages even aligned regions
    bool early_full = true;        // LTLF_EARLY_FULL=0: big_loop asks for the whole area only when due
    std::chrono::steady_clock::time_point t0;
    std::mutex mu;
    std::condition_variable cv;
    std::atomic<uint32_t> big_running{0};
    std::atomic<bool> small_busy{false};
    static constexpr uint64_t kSegs = 1ull << 16;
    static constexpr uint64_t kMinSlice = 16ull << 20;
    static constexpr uint64_t kBigLevel = 1ull << 20;  // candidates of a level that runs on its own
    static constexpr uint64_t kFirstRows = 1ull << 12;  // rows of a first region
    static constexpr uint64_t kSubStaging = 4096;

    ~Scheduler() {
        if (trace)  // the batch's or the server's small-pool summary
            std::fprintf(stderr,
                         "[ltlf] small pool: %llu steps, %u batched launches, %.1f ms in those steps (planning and "
                         "moves %.1f, level close and finish %.1f), %.1f ms of it waiting for the device; admission "
                         "%.1f ms\n",
                         (unsigned long long)small_steps, launches, 1e3 * small_step_s, 1e3 * plan_s, 1e3 * close_s,
                         1e3 * small_wait_s, 1e3 * admit_s);
        // a step that failed part-way may have left a replay in flight
        if (graph_launched) (void)hipStreamSynchronize(graph_stream);
        free_step_graphs(graphs);
        for (Job* j : bigs) stop_worker(j);
        for (hipStream_t st : streams) {
            (void)hipStreamSynchronize(st);
            (void)hipStreamDestroy(st);
        }
        for (auto& kv : jobs) delete kv.second;
    }

    // -------------------------------------------------------------- set-up
    ltlf_status init(ltlf_ctx* ctx, uint32_t max_res) {
        c = ctx;
        max_resident = max_res;
        const char* tr = std::getenv("LTLF_TRACE");
        trace = tr && *tr && *tr != '0';
        // a test hook: a small margin makes forecasts fall short, so that
        // levels are dropped and run again in larger regions
        const char* fm = std::getenv("LTLF_FORECAST_SCALE");
        if (fm && *fm) {
            const double v = std::atof(fm);
            if (v > 0.0 && v <= 1e6) forecast_margin = v;
        }
        // a test hook: a job that takes the whole area with its stored levels
        // stages them even where they already sit in place
        const char* ps = std::getenv("LTLF_PROMOTE_STAGED");
        always_stage = ps && *ps && *ps != '0';
        // a test hook: jobs ask for the whole area only for the level that
        // needs it, not a level ahead
        const char* ef = std::getenv("LTLF_EARLY_FULL");
        early_full = !(ef && *ef == '0');
        t0 = std::chrono::steady_clock::now();
        TRY(ensure_workspace(c));
        c->loaded = false;  // the workspace is carved below
        c->ran = false;
        const uint64_t off_segs = align_up(sizeof(Store) * (uint64_t)max_res, 256);
        const uint64_t off_gather = off_segs + align_up(sizeof(BSeg) * kSegs, 256);
        base = off_gather + align_up(8ull * C_NUM * max_res, 256);
        if (base + 4 * kMinSlice > c->ws_bytes) return fail(c, LTLF_ENOMEM, "workspace too small for the scheduler");
        const uint64_t region = c->ws_bytes - base;
        // the small pool is kept small: the large area is a request's
        // capacity, so it should be nearly all of the workspace
        const uint64_t pool = std::max<uint64_t>(region / 32, std::min<uint64_t>(region / 2, 256ull << 20));
        const uint64_t small_end = base + pool / 256 * 256;
        small.init(base, small_end);
        large.init(small_end, small_end + (c->ws_bytes - small_end) / 256 * 256);
        d_stores = reinterpret_cast<Store*>(c->ws);
        d_segs = reinterpret_cast<BSeg*>(c->ws + off_segs);
        d_gather = reinterpret_cast<unsigned long long*>(c->ws + off_gather);
        if (c->h_batch_cap < (uint64_t)C_NUM * max_res) {
            if (c->h_batch) (void)hipHostFree(c->h_batch);
            c->h_batch = nullptr;
            c->h_batch_cap = 0;
            TRY_HIP(hipHostMalloc(reinterpret_cast<void**>(&c->h_batch), 8ull * C_NUM * max_res,
                                  hipHostMallocDefault));
            c->h_batch_cap = (uint64_t)C_NUM * max_res;
        }
        const char* ng = std::getenv("LTLF_NO_GRAPH");
        use_graphs = !(ng && *ng && *ng != '0');
        if (use_graphs) {
            graphs.d_stores = d_stores;
            graphs.d_segs = d_segs;
            const hipError_t ge = make_step_graphs(graphs);
            if (ge != hipSuccess) {
                free_step_graphs(graphs);
                return fail(c, LTLF_EDEVICE, "building the batched step's graphs", ge);
            }
        }
        // one sub-context per resident job, plus the targets of moves
        while (c->subs.size() < (size_t)max_res + 2) {
            ltlf_ctx* sub = nullptr;
            TRY(ltlf_ctx_create(c->device, 0, &sub));
            sub->staging_bytes = kSubStaging;
            c->subs.push_back(sub);
        }
        return LTLF_OK;
    }
    uint64_t small_pool() const { return small.total(); }

    ltlf_status submit(const ltlf_spec* sp, const ltlf_costs* k, uint32_t bound, uint32_t flags, uint64_t want,
                       uint64_t* ticket) {
        if (!k || !ticket) return LTLF_EINVAL;
        TRY(validate_spec(sp));
        if (k->atom_cost == 0 || bound < k->atom_cost || bound > kMaxBound) return LTLF_EINVAL;
        Job* j = new (std::nothrow) Job();
        if (!j) return LTLF_ENOMEM;
        j->ticket = next_ticket++;
        j->n_props = sp->n_props;
        j->lengths.assign(sp->lengths, sp->lengths + sp->n_traces);
        uint64_t total = 0, bits = 0;
        for (uint32_t t = 0; t < sp->n_traces; ++t) {
            total += sp->lengths[t];
            bits += sp->lengths[t] + 1;
        }
        j->n_pos = total;
        j->letters.assign(sp->letters, sp->letters + total);
        j->positive.assign(sp->positive, sp->positive + sp->n_traces);
        j->costs = *k;
        j->bound = bound;
        j->flags = flags & (LTLF_FLAG_EXHAUST | LTLF_FLAG_NO_LOOKAHEAD | LTLF_FLAG_DEBUG_WEAK_HASH | LTLF_FLAG_DIGEST);
        j->wp = (uint32_t)align_up((bits + 31) / 32, 4);
        j->want = want;
        reset_result(&j->res, 4 * j->wp);
        jobs[j->ticket] = j;
        queue.push_back(j);
        *ticket = j->ticket;
        return LTLF_OK;
    }

    // ------------------------------------------------------------ regions
    void note(const Job* j, const char* what) const {
        if (!trace) return;
        const double t = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        std::fprintf(stderr,
                     "[ltlf] %8.3f s job %llu %s: level %u rows %llu status %d | queued %zu small %zu large %zu "
                     "grow %zu full %zu\n",
                     t, (unsigned long long)j->ticket, what, j->lev, (unsigned long long)j->rows, (int)j->status,
                     queue.size(), resident.size(), bigs.size(), grow_queue.size(), full_queue.size());
        std::fflush(stderr);
    }

    // Bytes of a region that holds `rows` rows of job j (see row_capacity);
    // UINT64_MAX if no region of the workspace can (a store holds at most
    // 2^31 - 16 rows).
    uint64_t region_for(const Job* j, uint64_t rows) const {
        if (rows > (1ull << 31) - 16) return UINT64_MAX;
        const uint64_t f = fixed_bytes(j->n_pos, j->lengths.size(), j->wp, j->n_props, kSubStaging);
        const uint64_t per = 4ull * j->wp + 32;
        uint64_t b = align_up(f + rows * per + rows * per / 32 + (2ull << 20), 1ull << 20);
        while (row_capacity(f, j->wp, b) < rows) {
            if (b > c->ws_bytes) return UINT64_MAX;
            b = align_up(b + b / 16, 1ull << 20);
        }
        return b;
    }

    ltlf_ctx* take_sub() {
        for (ltlf_ctx* sub : c->subs)
            if (std::find(used.begin(), used.end(), sub) == used.end()) {
                used.push_back(sub);
                return sub;
            }
        ltlf_ctx* sub = nullptr;  // pooled in the context for later schedulers
        if (ltlf_ctx_create(c->device, 0, &sub) != LTLF_OK) return nullptr;
        sub->staging_bytes = kSubStaging;
        c->subs.push_back(sub);
        used.push_back(sub);
        return sub;
    }
    void give_sub(ltlf_ctx* sub) {
        if (!sub) return;
        sub->loaded = false;
        auto it = std::find(used.begin(), used.end(), sub);
        if (it != used.end()) used.erase(it);
    }

    // A sub-context on region [off, off + bytes) with j's specification
    // loaded on s (the copy is ordered before later work on s; it is not
    // waited for).
    ltlf_status open_sub(Job* j, uint64_t off, uint64_t bytes, hipStream_t s, ltlf_ctx*& out) {
        ltlf_ctx* sub = take_sub();
        if (!sub) return fail(c, LTLF_EDEVICE, "no sub-context free");
        sub->ws = c->ws + off;
        sub->ws_bytes = bytes;
        sub->own_ws = false;
        sub->row_limit = c->row_limit;
        sub->tune = c->tune;
        const ltlf_spec sp = j->spec();
        sub->err.clear();
        const ltlf_status ls = load_staged(sub, &sp, s);
        if (ls != LTLF_OK) {
            give_sub(sub);
            return ls == LTLF_ENOMEM ? ls : fail(c, ls, sub->err.c_str());
        }
        out = sub;
        return LTLF_OK;
    }

    // The job leaves its region (and sub-context).
    void leave_region(Job* j) {
        if (j->arena) j->arena->release(j->off, j->bytes);
        give_sub(j->sub);
        j->sub = nullptr;
        j->arena = nullptr;
        j->off = j->bytes = 0;
        j->full = false;
        j->aligned = false;
    }

    // Moves j's stored levels into sub-context `to` (loaded, on a region
    // disjoint from j's): atoms and masks encoded there, counters reset,
    // then the rows and derivation records of every stored level copied to
    // the same indices, the digests and level bookkeeping carried over, the
    // counters set as the last closed level left them, and the table rebuilt
    // from the records.  The old region may be reused by later work on s;
    // the caller drains s before another stream may write it.
    // in_place: the rows already sit at to's row addresses and the caller
    // restores the digests (promote).
    ltlf_status migrate(Job* j, ltlf_ctx* to, uint32_t kernel, hipStream_t s, bool in_place = false) {
        ltlf_ctx* from = j->sub;
        TRY(begin_run(to, j->bound, j->flags & (LTLF_FLAG_DEBUG_WEAK_HASH | LTLF_FLAG_DIGEST), kernel, s));
        const uint64_t n = j->rows;
        if (n > to->plan_cap) return fail(c, LTLF_EDEVICE, "a moved job does not fit its new region");
        if (n) {
            if (!in_place)
                TRY_HIP(hipMemcpyAsync(to->st.rows, from->st.rows, n * 4ull * j->wp, hipMemcpyDeviceToDevice, s));
            TRY_HIP(hipMemcpyAsync(to->st.meta, from->st.meta, n * sizeof(uint4), hipMemcpyDeviceToDevice, s));
        }
        if ((j->flags & LTLF_FLAG_DIGEST) && !in_place)
            TRY_HIP(hipMemcpyAsync(to->d_digest, from->d_digest, 8ull * (kMaxBound + 1), hipMemcpyDeviceToDevice, s));
        TRY_HIP(launch_set_counter(to->d_ctr, C_ROWS, n, s));
        TRY_HIP(launch_set_counter(to->d_ctr, C_SNAP, n, s));
        TRY_HIP(launch_set_counter(to->d_ctr, C_CAND, j->res.candidates, s));
        TRY_HIP(launch_set_counter(to->d_ctr, C_DEFERRED, j->res.deferred, s));
        to->lstart = from->lstart;
        to->lcount = from->lcount;
        if (n && ensure_table(to, n, n, s) != LTLF_OK) return fail(c, LTLF_EDEVICE, to->err.c_str());
        return LTLF_OK;
    }

    // ------------------------------------------------------------- workers
    hipStream_t take_stream() {
        for (hipStream_t st : streams) {
            bool busy = false;
            for (Job* b : bigs) busy |= b->stream == st;
            for (Job* b : grow_queue) busy |= b->stream == st;
            if (!busy) return st;
        }
        hipStream_t st = nullptr;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) return nullptr;
        streams.push_back(st);
        return st;
    }

    // the large job, level after level, on its worker thread: before each
    // level (unless its region is the whole large area) the region must hold
    // the level's worst case, else the job stops and asks for a larger one
    void big_loop(Job* j) {
        ltlf_status st = hipSetDevice(c->device) == hipSuccess ? LTLF_OK : LTLF_EDEVICE;
        LevelRun& r = *j->run;
        bool grow = false;
        while (st == LTLF_OK) {
            {
                std::lock_guard<std::mutex> g(mu);
                if (j->stop) break;
            }
            const uint32_t lev = j->lev + 1;
            uint64_t worst = 0;
            if (!j->full) {
                const LevelPlan p = plan_level(j->sub, &j->costs, lev, r.shape);
                worst = r.rows + p.cand_ub;
                uint64_t need = r.rows + forecast(j->sub, lev, p.cand_ub, j->redo_level == lev);
                if (c->row_limit) {
                    worst = std::min<uint64_t>(worst, std::max<uint64_t>(c->row_limit, r.rows) + 1);
                    need = std::min<uint64_t>(need, worst);
                }
                // the level after this one expected to need more than half
                // the area: the job asks for the whole area now, where it will
                // be anyway, instead of enumerating this level here first
                const uint64_t next =
                    !early_full || c->row_limit || lev >= j->bound ? 0 : grown(j->sub, lev, need - r.rows);
                if (next && region_for(j, need + next) > large.total() / 2) {
                    j->need_rows = need + next;
                    j->early_full = true;
                    grow = true;
                    break;
                }
                if (need > j->sub->plan_cap) {
                    j->need_rows = std::max<uint64_t>(need, 4 * r.rows);
                    grow = true;
                    break;
                }
            }
            r.redo_overflow = !j->full;
            // persistent launches share the resident block slots with the
            // other large jobs and leave room to the small jobs' launches
            const uint32_t nb = std::max<uint32_t>(1, big_running.load(std::memory_order_relaxed));
            const uint32_t share = small_busy.load(std::memory_order_relaxed) ? kBusyEighths : 8;
            r.grid_eighths = std::max<uint32_t>(1, share / nb);
            st = r.level(lev, j->stream);
            if (st != LTLF_OK) break;
            if (r.overflowed) {  // the forecast fell short: the level again, in a region for its worst case
                r.overflowed = false;
                r.stop = false;
                j->redo_level = lev;
                j->need_rows = std::max<uint64_t>(worst, 4 * r.rows);
                grow = true;
                break;
            }
            j->lev = lev;
            j->res.candidates = r.candidates;
            j->rows = r.rows;
            j->status = r.status;
            j->wit_op = r.wit_op;
            j->wit_a = r.wit_a;
            j->wit_b = r.wit_b;
            if (r.stop || lev == j->bound) break;
        }
        // a level can end with work still queued (the compaction of its dead
        // rows); the main thread reads the sub-context and may hand the
        // region on, so the stream is drained first
        if (hipStreamSynchronize(j->stream) != hipSuccess && st == LTLF_OK) st = LTLF_EDEVICE;
        std::lock_guard<std::mutex> g(mu);
        j->wstatus = st;
        j->grow = grow;
        j->running = false;
        big_running.fetch_sub(1, std::memory_order_relaxed);
        cv.notify_all();
    }

    ltlf_status start_worker(Job* j) {
        j->stream = take_stream();
        if (!j->stream) return fail(c, LTLF_EDEVICE, "cannot create a stream for a large job");
        {
            std::lock_guard<std::mutex> g(mu);
            j->running = true;
            j->stop = false;
            j->grow = false;
            j->wstatus = LTLF_OK;
        }
        big_running.fetch_add(1, std::memory_order_relaxed);
        try {
            j->worker = std::thread([this, j] { big_loop(j); });
        } catch (...) {
            std::lock_guard<std::mutex> g(mu);
            j->running = false;
            big_running.fetch_sub(1, std::memory_order_relaxed);
            return fail(c, LTLF_EDEVICE, "cannot start a large job's worker thread");
        }
        bigs.push_back(j);
        return LTLF_OK;
    }

    // asks j's worker to stop after its current level and waits for it
    void stop_worker(Job* j) {
        {
            std::lock_guard<std::mutex> g(mu);
            j->stop = true;
        }
        if (j->worker.joinable()) j->worker.join();
    }

    // ------------------------------------------------------------ placement
    enum Place { PLACED, WAIT, NEED_FULL };

    // A region of the large area for j's next `rows` rows: j moves there
    // (keeping its stored levels) or, with nothing stored yet, starts there;
    // then its worker starts.  WAIT: no such region is free now; NEED_FULL:
    // only the whole large area would do, or more than half of it (such a
    // region could only be had with the area nearly empty, and while waiting
    // for it the job would hold what it has and be restarted by every job
    // that wants the whole area: it takes the whole area, once).
    ltlf_status place_large(Job* j, uint64_t rows, hipStream_t s, Place& out) {
        out = WAIT;
        const uint64_t bytes = region_for(j, rows);
        if (bytes > large.total() / 2) {
            out = NEED_FULL;
            return LTLF_OK;
        }
        uint64_t off = 0;
        bool aligned = false;
        if (bytes >= large.total() / 16) {
            // a large region goes, if that part of the area is free, where its
            // rows sit at the addresses the whole area's layout gives them, so
            // that the job can later take the whole area without moving them
            const uint64_t f = fixed_bytes(j->n_pos, j->lengths.size(), j->wp, j->n_props, kSubStaging);
            const uint64_t rf = rows_offset(f, j->wp, large.total()), rr = rows_offset(f, j->wp, bytes);
            if (rf >= rr && large.lo + (rf - rr) + bytes <= large.hi && large.alloc_at(large.lo + (rf - rr), bytes)) {
                off = large.lo + (rf - rr);
                aligned = true;
            }
        }
        if (!aligned && !large.alloc_high(bytes, off)) return LTLF_OK;
        ltlf_ctx* sub = nullptr;
        const ltlf_status ls = open_sub(j, off, bytes, s, sub);
        if (ls != LTLF_OK) {
            large.release(off, bytes);
            if (ls == LTLF_ENOMEM) out = NEED_FULL;
            return ls == LTLF_ENOMEM ? LTLF_OK : ls;
        }
        TRY(start_large(j, sub, &large, off, bytes, false, s));
        j->aligned = aligned;
        out = PLACED;
        return LTLF_OK;
    }

    // A job waiting for the whole area that holds a region of it takes the
    // area with its stored levels, and its table is rebuilt there.  If the
    // region is aligned (place_large) its rows stay where they are, its
    // derivation records move to the whole area's layout and its digests go
    // through the host (the whole area's fixed regions overlap the
    // region's).  Otherwise rows, records and digests are first copied to a
    // staging block of the area that overlaps neither the region, nor what
    // the whole area's set-up writes before they are moved in (its fixed
    // regions, deferral lists and the start of its table), nor their
    // destinations; then moved to the whole area's layout as any move does.
    // Starts it over in the whole area when neither works.  Only j holds part
    // of the area.
    ltlf_status promote(Job* j, hipStream_t s) {
        ltlf_ctx* from = j->sub;
        const uint64_t n = j->rows;
        const bool digests = (j->flags & LTLF_FLAG_DIGEST) != 0;
        const uint64_t f = fixed_bytes(j->n_pos, j->lengths.size(), j->wp, j->n_props, kSubStaging);
        const uint64_t total = large.total();
        const uint64_t rf = rows_offset(f, j->wp, total), cap = row_capacity(f, j->wp, total);
        const uint64_t rows_lo = large.lo + rf;
        const uint64_t meta_lo = large.lo + align_up(rf + 4ull * j->wp * cap, 256);
        const uint64_t from_meta = (uint64_t)(reinterpret_cast<char*>(from->st.meta) - c->ws);
        const bool lined_up = !always_stage && reinterpret_cast<char*>(from->st.rows) == c->ws + rows_lo &&
                              n <= cap && from_meta + 16 * n <= meta_lo;
        uint64_t stage = UINT64_MAX;
        const uint64_t rows_b = align_up(n * 4ull * j->wp, 256), meta_b = align_up(16 * n, 256);
        if (!lined_up && n <= cap) {
            // the table (two slots per row) ends where the rows start; the
            // set-up fills its first slots0 slots
            const uint64_t slots0 = pow2_ceil(std::max<uint64_t>(4ull * j->n_props, kMinTableSlots));
            const uint64_t table_lo = rows_lo - 16 * cap;
            stage = free_spot(large.lo, large.hi, rows_b + meta_b + align_up(8ull * (kMaxBound + 1), 256),
                              {{j->off, j->off + j->bytes},
                               {large.lo, table_lo + 8 * slots0 + 256},
                               {rows_lo, rows_lo + 4ull * j->wp * n},
                               {meta_lo, meta_lo + 16 * n}});
        }
        std::vector<uint64_t> dig(kMaxBound + 1, 0);
        if (lined_up && digests) {
            TRY_HIP(hipMemcpyAsync(dig.data(), from->d_digest, 8ull * (kMaxBound + 1), hipMemcpyDeviceToHost, s));
            TRY_HIP(hipStreamSynchronize(s));
        }
        if (stage != UINT64_MAX) {  // queued before anything is written to the area
            char* base = c->ws + stage;
            if (n) {
                TRY_HIP(hipMemcpyAsync(base, from->st.rows, n * 4ull * j->wp, hipMemcpyDeviceToDevice, s));
                TRY_HIP(hipMemcpyAsync(base + rows_b, from->st.meta, 16 * n, hipMemcpyDeviceToDevice, s));
            }
            if (digests)
                TRY_HIP(hipMemcpyAsync(base + rows_b + meta_b, from->d_digest, 8ull * (kMaxBound + 1),
                                       hipMemcpyDeviceToDevice, s));
            // `from` is given back below: its pointers now name the copies
            from->st.rows = reinterpret_cast<uint32_t*>(base);
            from->st.meta = reinterpret_cast<uint4*>(base + rows_b);
            from->d_digest = reinterpret_cast<unsigned long long*>(base + rows_b + meta_b);
        }
        large.release(j->off, j->bytes);
        j->arena = nullptr;  // the region is gone; `from` is still j's sub-context
        uint64_t off = 0;
        if (!large.alloc(total, off)) return fail(c, LTLF_EDEVICE, "the large area is not free");
        ltlf_ctx* to = nullptr;
        const ltlf_status ls = open_sub(j, large.lo, total, s, to);
        if (ls != LTLF_OK) {
            large.release(off, total);
            if (ls != LTLF_ENOMEM) return ls;
            leave_region(j);
            j->lev = 0;
            solo_queue.push_back(j);
            return LTLF_OK;
        }
        if (!lined_up && stage == UINT64_MAX) {
            note(j, "takes the whole area from the start (no room to stage its levels)");
            give_sub(from);
            j->sub = nullptr;
            j->arena = nullptr;
            j->aligned = false;
            j->lev = 0;
            return start_large(j, to, &large, off, total, true, s);
        }
        const uint32_t kind = shape_of(to, tuned_kernel(to)).kind;
        TRY(migrate(j, to, kind, s, lined_up));
        if (lined_up && digests)
            TRY_HIP(hipMemcpyAsync(to->d_digest, dig.data(), 8ull * (kMaxBound + 1), hipMemcpyHostToDevice, s));
        TRY_HIP(hipStreamSynchronize(s));
        give_sub(from);
        j->sub = to;
        j->arena = &large;
        j->off = off;
        j->bytes = total;
        j->full = true;
        j->aligned = false;
        j->mode = Job::LARGE;
        j->run->resume(to, &j->costs, j->bound, j->flags, &j->res, j->rows, j->res.candidates, j->status, j->wit_op,
                       j->wit_a, j->wit_b);
        note(j, lined_up ? "takes the whole area with its stored levels"
                         : "takes the whole area with its stored levels (staged)");
        return start_worker(j);
    }

    // j becomes a large job on sub-context `sub` (region [off, off+bytes) of
    // `ar`): moved there with its stored levels, or started there.
    ltlf_status start_large(Job* j, ltlf_ctx* sub, Arena* ar, uint64_t off, uint64_t bytes, bool full,
                            hipStream_t s) {
        const bool fresh = j->sub == nullptr || j->lev == 0;
        if (!fresh) {
            const uint32_t kind = shape_of(sub, tuned_kernel(sub)).kind;
            TRY(migrate(j, sub, kind, s));
            TRY_HIP(hipStreamSynchronize(s));  // the copies have read the old region
        }
        if (j->mode == Job::SMALL) resident.erase(std::find(resident.begin(), resident.end(), j));
        leave_region(j);
        j->sub = sub;
        j->arena = ar;
        j->off = off;
        j->bytes = bytes;
        j->full = full;
        j->mode = Job::LARGE;
        if (!j->run) j->run.reset(new (std::nothrow) LevelRun());
        if (!j->run) return fail(c, LTLF_ENOMEM, "out of host memory");
        if (fresh) {
            j->lev = 0;
            j->rows = 0;
            j->status = LTLF_NOT_FOUND;
            reset_result(&j->res, 4 * j->wp);
            TRY(j->run->begin(sub, &j->costs, j->bound, j->flags, &j->res, s));
            TRY_HIP(hipStreamSynchronize(s));  // the load and the run's set-up precede its levels
        } else {
            j->run->resume(sub, &j->costs, j->bound, j->flags, &j->res, j->rows, j->res.candidates, j->status,
                           j->wit_op, j->wit_a, j->wit_b);
        }
        note(j, full ? "large (whole area)" : fresh ? "large (fresh)" : "large (moved)");
        return start_worker(j);
    }

    // A small job moves to a region of the small pool for `rows` rows.
    ltlf_status move_small(Job* j, uint64_t rows, hipStream_t s, bool& moved) {
        moved = false;
        const uint64_t bytes = region_for(j, rows);
        uint64_t off = 0;
        if (bytes > small.total() / 4 || !small.alloc(bytes, off)) return LTLF_OK;
        ltlf_ctx* sub = nullptr;
        const ltlf_status ls = open_sub(j, off, bytes, s, sub);
        if (ls != LTLF_OK) {
            small.release(off, bytes);
            return ls == LTLF_ENOMEM ? LTLF_OK : ls;
        }
        // the old region may be handed out again at once: all work on the
        // small pool is on s, so its next use is ordered after these copies
        TRY(migrate(j, sub, KERNEL_WAVE, s));
        const uint32_t lev = j->lev;
        leave_region(j);
        j->sub = sub;
        j->arena = &small;
        j->off = off;
        j->bytes = bytes;
        j->lev = lev;
        moved = true;
        return LTLF_OK;
    }

    ltlf_status start_small(Job* j, hipStream_t s, bool& placed) {
        placed = false;
        const uint64_t bytes = std::max<uint64_t>(j->want ? j->want : region_for(j, kFirstRows), 1ull << 20);
        if (bytes > small.total() / 4) {  // too wide for the small pool: a large job from the start
            queue.erase(std::find(queue.begin(), queue.end(), j));
            j->need_rows = kFirstRows;
            grow_queue.push_back(j);
            placed = true;
            return LTLF_OK;
        }
        uint64_t off = 0;
        if (!small.alloc(bytes, off)) return LTLF_OK;
        ltlf_ctx* sub = nullptr;
        const ltlf_status ls = open_sub(j, off, bytes, s, sub);
        if (ls != LTLF_OK) {
            small.release(off, bytes);
            if (ls != LTLF_ENOMEM) return ls;
            queue.erase(std::find(queue.begin(), queue.end(), j));
            j->need_rows = kFirstRows;
            grow_queue.push_back(j);
            placed = true;
            return LTLF_OK;
        }
        j->sub = sub;
        j->arena = &small;
        j->off = off;
        j->bytes = bytes;
        j->mode = Job::SMALL;
        resident.push_back(j);
        placed = true;
        queue.erase(std::find(queue.begin(), queue.end(), j));
        return begin_run(sub, j->bound, j->flags & (LTLF_FLAG_DEBUG_WEAK_HASH | LTLF_FLAG_DIGEST), KERNEL_WAVE, s);
    }

    // back to the queue, from the start (its device state is discarded)
    void restart(Job* j, bool front) {
        note(j, "restart");
        if (j->mode == Job::SMALL) resident.erase(std::find(resident.begin(), resident.end(), j));
        leave_region(j);
        j->mode = Job::QUEUED;
        j->run.reset();
        j->lev = 0;
        j->rows = 0;
        j->redo_level = 0;
        j->status = LTLF_NOT_FOUND;
        reset_result(&j->res, 4 * j->wp);
        if (front) queue.push_front(j);
        else queue.push_back(j);
    }

    uint32_t holding() const {
        uint32_t n = (uint32_t)(resident.size() + bigs.size());
        for (Job* j : grow_queue) n += j->sub != nullptr;
        for (Job* j : full_queue) n += j->sub != nullptr;
        return n;
    }

    // ------------------------------------------------------------- admission
    ltlf_status admit(hipStream_t s) {
        if (!solo_queue.empty()) return LTLF_OK;  // the whole workspace is wanted: drain first
        // the whole large area, once nothing but the jobs waiting for it holds
        // any of it: the first of them that holds a region takes it with its
        // stored levels (others that hold regions give them up first)
        if (!full_queue.empty() && bigs.empty() && !large.empty()) {
            uint64_t held = 0;
            std::vector<Job*> holders;
            for (Job* w : full_queue)
                if (w->arena == &large) {
                    holders.push_back(w);
                    held += align_up(w->bytes, 256);
                }
            if (!holders.empty() && large.free_bytes() + held == large.total()) {
                for (size_t i = 1; i < holders.size(); ++i) {
                    Job* w = holders[i];
                    leave_region(w);
                    w->run.reset();
                    w->lev = 0;
                    w->rows = 0;
                    w->redo_level = 0;
                    w->status = LTLF_NOT_FOUND;
                    reset_result(&w->res, 4 * w->wp);
                    w->mode = Job::QUEUED;
                }
                Job* h = holders[0];
                full_queue.erase(std::find(full_queue.begin(), full_queue.end(), h));
                TRY(promote(h, s));
            }
        }
        if (!full_queue.empty() && large.empty()) {
            Job* j = full_queue.front();
            full_queue.pop_front();
            ltlf_ctx* sub = nullptr;
            const ltlf_status ls = open_sub(j, large.lo, large.total(), s, sub);
            if (ls == LTLF_ENOMEM) {  // not even the large area: the whole workspace
                solo_queue.push_back(j);
                return LTLF_OK;
            }
            if (ls != LTLF_OK) return ls;
            uint64_t off = 0;
            if (!large.alloc(large.total(), off)) return fail(c, LTLF_EDEVICE, "the large area is not free");
            j->lev = 0;  // from the start
            TRY(start_large(j, sub, &large, off, large.total(), true, s));
        }
        // a waiter that wants more than half the area (see place_large) waits
        // for the whole area holding nothing, wherever it stands in the queue
        for (size_t i = 0; i < grow_queue.size();) {
            Job* w = grow_queue[i];
            if (region_for(w, w->need_rows) > large.total() / 2) {
                grow_queue.erase(grow_queue.begin() + (long)i);
                // it keeps its region and levels if aligned, or if no other
                // job waiting for the whole area holds a region (it will take
                // the area first and keep them)
                bool alone = true;
                for (const Job* o : full_queue) alone = alone && (o->arena != &large);
                full_queue.push_back(w);
                if (w->arena == &large && w->lev > 0 && (w->aligned || alone)) {
                    note(w, w->aligned ? "waits for the whole area, keeping its aligned region"
                                       : "waits for the whole area, keeping its region");
                    continue;
                }
                if (w->mode == Job::SMALL) resident.erase(std::find(resident.begin(), resident.end(), w));
                leave_region(w);
                w->mode = Job::QUEUED;
                note(w, "waits for the whole area");
            } else {
                ++i;
            }
        }
        // larger regions, oldest first.  While a job waits for the whole area
        // the area drains: only jobs that already hold large-area regions are
        // served (they finish, or come to want the whole area themselves);
        // others wait.
        auto eligible = [&](const Job* w) { return full_queue.empty() || w->arena == &large; };
        auto to_full = [&](Job* w) {
            if (w->mode == Job::SMALL) resident.erase(std::find(resident.begin(), resident.end(), w));
            leave_region(w);
            w->mode = Job::QUEUED;
            full_queue.push_back(w);
        };
        for (size_t i = 0; i < grow_queue.size();) {
            Job* j = grow_queue[i];
            if (!eligible(j)) {
                ++i;
                continue;
            }
            Place pl = WAIT;
            TRY(place_large(j, j->need_rows, s, pl));
            if (pl == WAIT) break;
            grow_queue.erase(grow_queue.begin() + (long)i);
            if (pl == NEED_FULL) to_full(j);
        }
        // nothing runs in the large area and the oldest eligible waiter cannot
        // be served (the others hold part of what it needs): the youngest
        // waiters that hold large-area regions start over later, one at a time
        // until it fits; if none helps, it starts over itself in a fresh
        // region.  (With no eligible waiter left the area is empty, and the
        // job that waits for it starts above on the next call.)
        if (big_running.load() == 0 && bigs.empty()) {
            size_t hi = 0;
            while (hi < grow_queue.size() && !eligible(grow_queue[hi])) ++hi;
            if (hi < grow_queue.size()) {
                Job* h = grow_queue[hi];
                bool served = false;
                for (size_t i = grow_queue.size(); i-- > 0 && !served;) {
                    Job* w = grow_queue[i];
                    if (w == h || w->arena != &large) continue;
                    if (i < hi) break;  // only younger waiters
                    grow_queue.erase(grow_queue.begin() + (long)i);
                    restart(w, true);
                    Place pl = WAIT;
                    TRY(place_large(h, h->need_rows, s, pl));
                    if (pl == WAIT) continue;
                    served = true;
                    grow_queue.erase(std::find(grow_queue.begin(), grow_queue.end(), h));
                    if (pl == NEED_FULL) to_full(h);
                }
                if (!served && h->arena == &large) {
                    grow_queue.erase(std::find(grow_queue.begin(), grow_queue.end(), h));
                    const uint64_t need = h->need_rows;
                    restart(h, true);
                    queue.erase(std::find(queue.begin(), queue.end(), h));
                    h->need_rows = need;
                    grow_queue.push_front(h);
                }
            }
        }
        // new jobs into the small pool
        for (size_t i = 0; i < queue.size() && holding() < max_resident;) {
            Job* j = queue[i];
            bool placed = false;
            TRY(start_small(j, s, placed));
            if (!placed) ++i;
        }
        return LTLF_OK;
    }

    // ---------------------------------------------------------------- finish
    // a job ends: its result is kept until polled; its memory is returned
    // (cancelled: the levels it completed stand, its status is CANCELLED)
    ltlf_status finish(Job* j, hipStream_t s, bool cancelled = false) {
        TRY(finish_enqueue(j, s));
        if (j->sub) TRY_HIP(hipStreamSynchronize(s));
        return finish_complete(j, cancelled);
    }
    // finish in two halves, so that the jobs that end together wait for the
    // device once: the digests and the witness tokens are copied to the
    // sub-context's pinned buffers on s, then read once s is synchronised
    ltlf_status finish_enqueue(Job* j, hipStream_t s) {
        ltlf_ctx* sub = j->sub;
        if (!sub) return LTLF_OK;
        if (j->flags & LTLF_FLAG_DIGEST)
            TRY_HIP(hipMemcpyAsync(sub->h_dig, sub->d_digest, 8 * (kMaxBound + 1), hipMemcpyDeviceToHost, s));
        if (j->status == LTLF_OK && enqueue_formula(sub, j->wit_op, j->wit_a, j->wit_b, s) != LTLF_OK)
            return fail(c, LTLF_EDEVICE, sub->err.c_str());
        return LTLF_OK;
    }
    ltlf_status finish_complete(Job* j, bool cancelled) {
        ltlf_ctx* sub = j->sub;
        ltlf_result& r = j->res;
        j->counts.assign(j->bound + 1, 0);
        j->digests.assign(j->bound + 1, 0);
        uint64_t uniq = 0;
        if (sub) {
            for (uint32_t lev = 1; lev <= r.levels_done; ++lev) {
                j->counts[lev] = sub->lcount[lev];
                uniq += sub->lcount[lev];
            }
            take_digests(sub, r.levels_done, (j->flags & LTLF_FLAG_DIGEST) != 0, j->digests.data(), j->bound + 1);
        } else {
            r.levels_done = 0;
        }
        r.unique_total = uniq;
        r.checked_level = std::max({r.checked_level, r.levels_done, r.overflow_level});
        r.status = j->status;
        j->formula.clear();
        if (sub && j->status == LTLF_OK && decode_formula(sub, j->wit_op, j->formula) != LTLF_OK)
            return fail(c, LTLF_EDEVICE, sub->err.c_str());
        r.formula_len = j->formula.size() + 1;
        if (cancelled) r.status = LTLF_CANCELLED;
        j->done = true;
        note(j, "done");
        if (j->mode == Job::SMALL) resident.erase(std::find(resident.begin(), resident.end(), j));
        auto b = std::find(bigs.begin(), bigs.end(), j);
        if (b != bigs.end()) bigs.erase(b);
        leave_region(j);
        j->mode = Job::FINISHED;
        j->run.reset();
        return LTLF_OK;
    }

    // Every unfinished job ends as CANCELLED with the levels it completed:
    // large jobs after their running level (workers are stopped between
    // levels), small jobs at their last closed level, queued ones with none.
    ltlf_status cancel_all(hipStream_t s) {
        for (Job* j : std::vector<Job*>(bigs)) {
            stop_worker(j);
            if (j->wstatus != LTLF_OK) return fail(c, j->wstatus, j->sub->err.c_str());
            TRY(finish(j, s, true));
        }
        for (Job* j : std::vector<Job*>(resident)) TRY(finish(j, s, true));
        for (Job* j : std::vector<Job*>(grow_queue.begin(), grow_queue.end()))
            if (j->sub) TRY(finish(j, s, true));
        for (Job* j : std::vector<Job*>(full_queue.begin(), full_queue.end()))
            if (j->sub) TRY(finish(j, s, true));
        for (std::deque<Job*>* q : {&queue, &grow_queue, &full_queue, &solo_queue}) {
            for (Job* j : *q) {
                if (j->done) continue;
                j->counts.assign(j->bound + 1, 0);
                j->digests.assign(j->bound + 1, 0);
                reset_result(&j->res, 4 * j->wp);
                j->res.status = LTLF_CANCELLED;
                j->formula.clear();
                j->res.formula_len = 1;
                j->done = true;
                j->mode = Job::FINISHED;
            }
            q->clear();
        }
        return LTLF_OK;
    }

    // the whole workspace, through ltlf_solve
    ltlf_status run_solo(Job* j, hipStream_t s) {
        j->counts.assign(j->bound + 1, 0);
        j->digests.assign(j->bound + 1, 0);
        std::vector<char> fbuf(kMaxTokens * 8);
        ltlf_result r{};
        r.level_counts = j->counts.data();
        r.level_counts_len = j->bound + 1;
        r.level_digests = j->digests.data();
        r.formula = fbuf.data();
        r.formula_cap = fbuf.size();
        const ltlf_spec sp = j->spec();
        const ltlf_status st = ltlf_solve(c, &sp, &j->costs, j->bound, j->flags, s, &r);
        c->loaded = false;  // the scheduler's carve-up stands
        if (st < 0) return st;
        j->res = r;
        j->formula = st == LTLF_OK ? std::string(fbuf.data()) : std::string();
        j->res.formula = nullptr;
        j->res.level_counts = nullptr;
        j->res.level_digests = nullptr;
        j->done = true;
        j->mode = Job::FINISHED;
        return LTLF_OK;
    }

    // ------------------------------------------------------------------ step
    ltlf_status reap(hipStream_t s, uint32_t& finished) {
        for (Job* j : std::vector<Job*>(bigs)) {
            bool running;
            {
                std::lock_guard<std::mutex> g(mu);
                running = j->running;
            }
            if (running) continue;
            if (j->worker.joinable()) j->worker.join();
            if (j->wstatus != LTLF_OK) return fail(c, j->wstatus, j->sub ? j->sub->err.c_str() : "large job");
            if (j->grow) {  // wants a larger region: waits for it, keeping its own
                note(j, j->redo_level == j->lev + 1 ? "level dropped (region too small), waits for a larger one"
                        : j->early_full                   ? "expects to need the whole area after the next level"
                                                          : "waits for a larger region");
                j->early_full = false;
                bigs.erase(std::find(bigs.begin(), bigs.end(), j));
                grow_queue.push_back(j);
                continue;
            }
            // an overflow is final only in the whole large area; elsewhere the
            // worst-case check rules it out except through the row limit
            if (j->status != LTLF_OK && j->res.overflow_level) j->status = LTLF_CAPACITY;
            TRY(finish(j, s));
            ++finished;
        }
        return LTLF_OK;
    }

    ltlf_status step(hipStream_t s, uint32_t* n_done) {
        uint32_t finished = 0;
        const auto t_admit = std::chrono::steady_clock::now();
        TRY(reap(s, finished));
        TRY(admit(s));
        admit_s += std::chrono::duration<double>(std::chrono::steady_clock::now() - t_admit).count();
        if (resident.empty() && bigs.empty() && grow_queue.empty() && full_queue.empty() && queue.empty()) {
            if (!solo_queue.empty()) {
                Job* j = solo_queue.front();
                solo_queue.pop_front();
                TRY(run_solo(j, s));
                ++finished;
            }
            if (n_done) *n_done = finished;
            return LTLF_OK;
        }
        // small jobs: plan the next level; one that outgrows its region moves
        const auto t_small = std::chrono::steady_clock::now();
        std::vector<Job*> live;
        for (Job* j : std::vector<Job*>(resident)) {
            if (std::find(grow_queue.begin(), grow_queue.end(), j) != grow_queue.end()) continue;  // waiting
            ltlf_ctx* sub = j->sub;
            const uint32_t lev = j->lev + 1;
            sub->lstart[lev] = j->rows;
            j->plan = plan_level(sub, &j->costs, lev, small_shape(sub));
            j->next_tile = 0;
            j->total = 0;
            for (const Seg& g : j->plan.segs) j->total += g.tiles;
            if (j->total) {
                const uint64_t need = j->rows + j->plan.cand_ub;
                if (j->plan.cand_ub > kBigLevel) {  // a large job from this level: a region by forecast
                    j->need_rows = std::max<uint64_t>(j->rows + forecast(sub, lev, j->plan.cand_ub, false),
                                                      4 * j->rows);
                    grow_queue.push_back(j);
                    continue;
                }
                if (need > sub->plan_cap) {
                    bool moved = false;
                    TRY(move_small(j, std::max<uint64_t>(need, 4 * j->rows), s, moved));
                    if (!moved) {
                        j->need_rows = std::max<uint64_t>(need, 4 * j->rows);
                        grow_queue.push_back(j);
                        continue;
                    }
                    sub = j->sub;
                    sub->lstart[lev] = j->rows;
                    j->plan = plan_level(sub, &j->costs, lev, small_shape(sub));
                }
                if (ensure_table(sub, j->rows, j->plan.cand_ub, s) != LTLF_OK)
                    return fail(c, LTLF_EDEVICE, sub->err.c_str());
            }
            live.push_back(j);
        }
        small_busy.store(!live.empty() || !queue.empty(), std::memory_order_relaxed);
        plan_s += std::chrono::duration<double>(std::chrono::steady_clock::now() - t_small).count();
        // large-area requests raised just now are served at once if they fit
        if (!grow_queue.empty()) TRY(admit(s));
        if (!live.empty()) {
            std::vector<Store> h_stores(live.size());
            for (size_t i = 0; i < live.size(); ++i) h_stores[i] = live[i]->sub->st;
            TRY_HIP(hipMemcpyAsync(d_stores, h_stores.data(), sizeof(Store) * live.size(), hipMemcpyHostToDevice, s));
            // pieces of every job's plan, each job's share of a launch
            // bounded by its deferral list
            std::vector<BSeg> pieces;
            for (;;) {
                pieces.clear();
                uint64_t first = 0;
                for (size_t i = 0; i < live.size() && pieces.size() + kMaxSegs < kSegs; ++i) {
                    Job* j = live[i];
                    uint64_t budget = j->sub->st.def0_cap;
                    uint64_t seg_first = 0;
                    for (size_t g = 0; g < j->plan.segs.size() && j->next_tile < j->total; ++g) {
                        const Seg& sg = j->plan.segs[g];
                        const uint64_t seg_end = seg_first + sg.tiles;
                        if (j->next_tile < seg_end) {
                            const uint64_t per = j->plan.cand_per_tile[g];
                            const uint64_t fit = per ? budget / per : seg_end - j->next_tile;
                            const uint64_t take = std::min<uint64_t>(fit, seg_end - j->next_tile);
                            if (take == 0) break;
                            BSeg b{};
                            b.problem = (uint32_t)i;
                            b.first = first;
                            b.lt0 = j->next_tile - seg_first;
                            b.seg = sg;
                            pieces.push_back(b);
                            first += take;
                            j->next_tile += take;
                            budget -= take * per;
                        }
                        seg_first = seg_end;
                    }
                }
                if (pieces.empty()) break;
                TRY_HIP(hipMemcpyAsync(d_segs, pieces.data(), sizeof(BSeg) * pieces.size(), hipMemcpyHostToDevice, s));
                if (use_graphs) {
                    TRY_HIP(set_step(graphs, (uint32_t)pieces.size(), first, (uint32_t)live.size()));
                    graph_stream = s;
                    graph_launched = true;
                    TRY_HIP(hipGraphLaunch(graphs.exec, s));
                } else {
                    TRY_HIP(launch_generate_batch(d_stores, d_segs, (uint32_t)pieces.size(), 0, first, s));
                    TRY_HIP(launch_verify_batch(d_stores, (uint32_t)live.size(), s));
                    TRY_HIP(launch_between_batch(d_stores, (uint32_t)live.size(), s));
                }
                ++launches;
                {
                    const auto w0 = std::chrono::steady_clock::now();
                    TRY_HIP(hipStreamSynchronize(s));  // `pieces` is reused
                    small_wait_s += std::chrono::duration<double>(std::chrono::steady_clock::now() - w0).count();
                }
            }
            TRY_HIP(launch_gather_ctr(d_stores, (uint32_t)live.size(), d_gather, s));
            TRY_HIP(hipMemcpyAsync(c->h_batch, d_gather, 8ull * C_NUM * live.size(), hipMemcpyDeviceToHost, s));
            const auto w0 = std::chrono::steady_clock::now();
            TRY_HIP(hipStreamSynchronize(s));
            small_wait_s += std::chrono::duration<double>(std::chrono::steady_clock::now() - w0).count();
        }
        const auto t_close = std::chrono::steady_clock::now();
        std::vector<Job*> ending;  // finished at this level: completed together below
        for (size_t i = 0; i < live.size(); ++i) {
            Job* j = live[i];
            ltlf_ctx* sub = j->sub;
            ltlf_result* r = &j->res;
            const uint32_t lev = j->lev + 1;
            j->lev = lev;
            if (j->total == 0) {
                r->levels_done = lev;
                if (lev == j->bound) ending.push_back(j);
                continue;
            }
            std::memcpy(sub->h_ctr, c->h_batch + (uint64_t)i * C_NUM, 8ull * C_NUM);
            // rare: deferred candidates that were new after all (as in ltlf_run)
            const uint64_t n0 = sub->h_ctr[C_DEF1];
            for (uint64_t round = 0; sub->h_ctr[C_DEF1] > 0 && !sub->h_ctr[C_DEF_OVF]; ++round) {
                if (round > n0 + 16) return fail(c, LTLF_EDEVICE, "re-insertion rounds made no progress");
                const uint64_t m = sub->h_ctr[C_DEF1];
                const uint64_t now_rows = std::min<uint64_t>(sub->h_ctr[C_ROWS], sub->st.cap);
                if (ensure_table(sub, now_rows, std::min<uint64_t>(m, sub->st.cap - now_rows), s) != LTLF_OK)
                    return fail(c, LTLF_EDEVICE, sub->err.c_str());
                TRY_HIP(launch_reinsert(sub->st, m, s));
                TRY_HIP(launch_set_counter(sub->d_ctr, C_DEF1, 0, s));
                TRY_HIP(launch_verify_deferred(sub->st, s));
                TRY_HIP(launch_between(sub->d_ctr, s));
                if (read_counters(sub, s) != LTLF_OK) return fail(c, LTLF_EDEVICE, sub->err.c_str());
            }
            const uint64_t now = std::min<uint64_t>(sub->h_ctr[C_ROWS], sub->st.cap);
            r->candidates = sub->h_ctr[C_CAND];
            r->deferred = sub->h_ctr[C_DEFERRED];
            if (sub->h_ctr[C_DEF_OVF] || sub->h_ctr[C_OVERFLOW] || (sub->row_limit && now > sub->row_limit)) {
                // not expected past the worst-case check except through the
                // row limit: the large-area path applies it as ltlf_run does
                restart(j, true);
                queue.erase(std::find(queue.begin(), queue.end(), j));
                j->need_rows = kFirstRows;
                grow_queue.push_back(j);
                continue;
            }
            sub->lcount[lev] = now - j->rows;
            if (j->flags & LTLF_FLAG_DIGEST)
                TRY_HIP(launch_digest(sub->st.rows, sub->Wp, j->rows, now - j->rows, sub->d_digest + lev, s));
            j->rows = now;
            if (sub->h_ctr[C_FOUND] && j->status != LTLF_OK) {
                j->status = LTLF_OK;
                r->min_cost = lev;
                j->wit_op = (uint32_t)sub->h_ctr[C_WIT_OP];
                j->wit_a = (uint32_t)sub->h_ctr[C_WIT_A];
                j->wit_b = (uint32_t)sub->h_ctr[C_WIT_B];
            }
            r->levels_done = lev;
            if ((j->status == LTLF_OK && !(j->flags & LTLF_FLAG_EXHAUST)) || lev == j->bound) {
                r->gen_launches = launches;
                r->verify_launches = launches;
                ending.push_back(j);
            }
        }
        if (!ending.empty()) {
            for (Job* j : ending) TRY(finish_enqueue(j, s));
            TRY_HIP(hipStreamSynchronize(s));
            for (Job* j : ending) TRY(finish_complete(j, false));
            finished += (uint32_t)ending.size();
        }
        close_s += std::chrono::duration<double>(std::chrono::steady_clock::now() - t_close).count();
        if (!live.empty()) {
            ++small_steps;
            small_step_s += std::chrono::duration<double>(std::chrono::steady_clock::now() - t_small).count();
        }
        small_busy.store(!resident.empty() || !queue.empty(), std::memory_order_relaxed);
        // with nothing else to step, wait a little for a large job instead of
        // returning at once
        if (live.empty() && !bigs.empty()) {
            std::unique_lock<std::mutex> lk(mu);
            cv.wait_for(lk, std::chrono::milliseconds(2), [this] {
                for (Job* j : bigs)
                    if (!j->running) return true;
                return false;
            });
        }
        TRY(reap(s, finished));
        if (n_done) *n_done = finished;
        return LTLF_OK;
    }

    // copies a finished job's result into the caller's buffers and forgets it
    ltlf_status collect(uint64_t ticket, ltlf_result* out) {
        auto it = jobs.find(ticket);
        if (it == jobs.end() || !out) return LTLF_EINVAL;
        Job* j = it->second;
        if (!j->done) return LTLF_PENDING;
        uint64_t* lc = out->level_counts;
        uint64_t* ld = out->level_digests;
        const uint32_t lcl = out->level_counts_len;
        char* f = out->formula;
        const uint64_t fc = out->formula_cap;
        *out = j->res;
        out->level_counts = lc;
        out->level_digests = ld;
        if (ld)
            for (uint32_t i = 0; i < lcl; ++i) ld[i] = i < j->digests.size() ? j->digests[i] : 0;
        out->level_counts_len = lcl;
        out->formula = f;
        out->formula_cap = fc;
        if (lc)
            for (uint32_t i = 0; i < lcl; ++i) lc[i] = i < j->counts.size() ? j->counts[i] : 0;
        ltlf_status st = out->status;
        out->formula_len = j->formula.size() + 1;
        if (f && fc) {
            if (fc < j->formula.size() + 1) st = LTLF_EBUFSZ;
            else std::memcpy(f, j->formula.c_str(), j->formula.size() + 1);
        }
        jobs.erase(it);
        delete j;
        return st;
    }

    ltlf_status cancel(uint64_t ticket) {
        auto it = jobs.find(ticket);
        if (it == jobs.end()) return LTLF_EINVAL;
        Job* j = it->second;
        if (std::find(bigs.begin(), bigs.end(), j) != bigs.end()) {
            stop_worker(j);
            bigs.erase(std::find(bigs.begin(), bigs.end(), j));
        }
        if (j->mode == Job::SMALL) resident.erase(std::find(resident.begin(), resident.end(), j));
        for (std::deque<Job*>* q : {&queue, &grow_queue, &full_queue, &solo_queue}) {
            auto f = std::find(q->begin(), q->end(), j);
            if (f != q->end()) q->erase(f);
        }
        leave_region(j);
        jobs.erase(it);
        delete j;
        return LTLF_OK;
    }

    uint32_t waiting() const {
        uint32_t n = (uint32_t)(queue.size() + full_queue.size() + solo_queue.size());
        for (Job* j : grow_queue) n += j->sub == nullptr;
        return n;
    }
    uint32_t on_device() const { return holding(); }
    bool idle() const {
        return queue.empty() && grow_queue.empty() && full_queue.empty() && solo_queue.empty() && resident.empty() &&
               bigs.empty();
    }
    uint64_t free_bytes() const { return small.free_bytes() + large.free_bytes(); }

    // Rows level `lev` of a large job is expected to add: the growth ratio of
    // the two levels before it, with a 1.5x margin (the table sizing's
    // estimate; forecast_margin), never above the candidate bound; the bound
    // itself where that growth is unknown, or after the level overflowed a
    // region sized this way.
    uint64_t forecast(const ltlf_ctx* sub, uint32_t lev, uint64_t cand_ub, bool worst) const {
        if (worst || lev < 3 || lev >= sub->lcount.size()) return cand_ub;
        const uint64_t a = sub->lcount[lev - 1], b = sub->lcount[lev - 2];
        if (!a || !b) return cand_ub;
        const double est = forecast_margin * (double)a / (double)b * (double)a + 4096.0;
        return est >= (double)cand_ub ? cand_ub : (uint64_t)est;
    }

    // Rows the level after `lev` is expected to add when level lev adds
    // `est`: the same growth ratio as forecast's, without a second margin; 0
    // where that growth is unknown.
    static uint64_t grown(const ltlf_ctx* sub, uint32_t lev, uint64_t est) {
        if (lev < 3 || lev >= sub->lcount.size()) return 0;
        const uint64_t a = sub->lcount[lev - 1], b = sub->lcount[lev - 2];
        if (!a || !b) return 0;
        const double g = (double)a / (double)b * (double)est;
        return g >= 1e18 ? (uint64_t)1e18 : (uint64_t)g;
    }

    // Small jobs run the wave kernel's batched form (any row width).
    static TileShape small_shape(const ltlf_ctx* sub) { return shape_of(sub, KERNEL_WAVE); }
};

}  // namespace

extern "C" {

const char* ltlf_status_str(ltlf_status s) {
    switch (s) {
    case LTLF_OK: return "ok";
    case LTLF_NOT_FOUND: return "no separating formula within the cost bound";
    case LTLF_CAPACITY: return "store full before the cost bound";
    case LTLF_PENDING: return "request not finished";
    case LTLF_CANCELLED: return "cancelled";
    case LTLF_EINVAL: return "invalid argument";
    case LTLF_ENOMEM: return "out of device memory";
    case LTLF_EDEVICE: return "HIP runtime error";
    case LTLF_EBUFSZ: return "buffer too small";
    case LTLF_ESTATE: return "call out of order";
    }
    return "unknown status";
}

ltlf_status ltlf_ctx_create(int device, uint64_t hbm_budget_bytes, ltlf_ctx** out) {
    if (!out) return LTLF_EINVAL;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess) return LTLF_EDEVICE;
    if (device < 0 || device >= n) return LTLF_EINVAL;
    if (hipSetDevice(device) != hipSuccess) return LTLF_EDEVICE;
    ltlf_ctx* c = new (std::nothrow) ltlf_ctx();
    if (!c) return LTLF_ENOMEM;
    c->device = device;
    int lds = 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device) != hipSuccess) {
        delete c;
        return LTLF_EDEVICE;
    }
    c->lds_limit = lds > 1024 ? (uint64_t)lds - 1024 : 0;  // room for static LDS
    c->budget = hbm_budget_bytes ? std::max<uint64_t>(hbm_budget_bytes, kMinWorkspace) : kDefaultBudget;
    if (hipHostMalloc(reinterpret_cast<void**>(&c->h_ctr), 8 * C_NUM, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&c->h_tokens), 4 * (1 + kMaxTokens), hipHostMallocDefault) !=
            hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&c->h_dig), 8 * (kMaxBound + 1), hipHostMallocDefault) != hipSuccess ||
        hipEventCreate(&c->ev0) != hipSuccess || hipEventCreate(&c->ev1) != hipSuccess ||
        hipEventCreate(&c->evb0) != hipSuccess || hipEventCreate(&c->evb1) != hipSuccess) {
        if (c->h_ctr) (void)hipHostFree(c->h_ctr);
        if (c->h_tokens) (void)hipHostFree(c->h_tokens);
        if (c->h_dig) (void)hipHostFree(c->h_dig);
        for (hipEvent_t e : {c->ev0, c->ev1, c->evb0, c->evb1})
            if (e) (void)hipEventDestroy(e);
        delete c;
        return LTLF_EDEVICE;
    }
    *out = c;
    return LTLF_OK;
}

ltlf_status ltlf_ctx_set_workspace(ltlf_ctx* c, void* dev_ptr, uint64_t bytes) {
    if (!c || !dev_ptr || (reinterpret_cast<uintptr_t>(dev_ptr) & 255u) || bytes < kMinWorkspace)
        return LTLF_EINVAL;
    if (c->own_ws && c->ws) (void)hipFree(c->ws);
    c->ws = static_cast<char*>(dev_ptr);
    c->ws_bytes = bytes;
    c->own_ws = false;
    c->loaded = false;
    c->ran = false;
    return LTLF_OK;
}

const char* ltlf_ctx_last_error(const ltlf_ctx* c) {
    if (!c) return "null context";
    return c->err.c_str();
}

ltlf_status ltlf_ctx_cancel(ltlf_ctx* c) {
    if (!c) return LTLF_EINVAL;
    c->cancel.store(true, std::memory_order_release);
    return LTLF_OK;
}

ltlf_status ltlf_ctx_set_row_limit(ltlf_ctx* c, uint64_t max_rows) {
    if (!c) return LTLF_EINVAL;
    c->row_limit = max_rows;
    return LTLF_OK;
}

void ltlf_ctx_destroy(ltlf_ctx* c) {
    if (!c) return;
    for (ltlf_ctx* sub : c->subs) ltlf_ctx_destroy(sub);
    c->subs.clear();
    (void)hipSetDevice(c->device);
    if (c->h_batch) (void)hipHostFree(c->h_batch);
    if (c->own_ws && c->ws) (void)hipFree(c->ws);
    if (c->h_ctr) (void)hipHostFree(c->h_ctr);
    if (c->h_tokens) (void)hipHostFree(c->h_tokens);
    if (c->h_dig) (void)hipHostFree(c->h_dig);
    if (c->h_load_busy) (void)hipEventSynchronize(c->ev_load);
    if (c->h_load) (void)hipHostFree(c->h_load);
    for (hipEvent_t e : {c->ev0, c->ev1, c->evb0, c->evb1, c->ev_load})
        if (e) (void)hipEventDestroy(e);
    delete c;
}

ltlf_status ltlf_load(ltlf_ctx* c, const ltlf_spec* sp, void* stream) {
    if (!c) return LTLF_EINVAL;
    c->err.clear();
    TRY(load_layout(c, sp));
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::vector<uint8_t> img(input_bytes(c));
    fill_inputs(c, sp, img.data());
    TRY_HIP(hipMemcpyAsync(c->d_letters, img.data(), img.size(), hipMemcpyHostToDevice, s));
    TRY_HIP(hipStreamSynchronize(s));
    c->loaded = true;
    return LTLF_OK;
}

ltlf_status ltlf_run(ltlf_ctx* c, const ltlf_costs* k, uint32_t bound, uint32_t flags, void* stream,
                     ltlf_result* res) {
    if (!c || !k || !res) return LTLF_EINVAL;
    c->err.clear();
    if (k->atom_cost == 0 || bound < k->atom_cost || bound > kMaxBound) return LTLF_EINVAL;
    if (!c->loaded) return LTLF_ESTATE;
    TRY_HIP(hipSetDevice(c->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    reset_result(res, 4 * c->Wp);

    hipEvent_t e0 = c->ev0, e1 = c->ev1;
    TRY_HIP(hipEventRecord(e0, s));
    LevelRun run;
    TRY(run.begin(c, k, bound, flags, res, s));
    bool cancelled = false;
    for (uint32_t lev = 1; lev <= bound && !run.stop; ++lev) {
        if (c->cancel.exchange(false, std::memory_order_acq_rel)) {
            cancelled = true;
            break;
        }
        TRY(run.level(lev, s));
    }
    TRY_HIP(hipEventRecord(e1, s));
    TRY_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    TRY_HIP(hipEventElapsedTime(&ms, e0, e1));
    res->enum_ms = ms;
    res->candidates = run.candidates;
    res->deferred = c->h_ctr[C_DEFERRED];
    c->levels_done = res->levels_done;
    c->ran = true;
    TRY(finish_result(c, res, run.status, run.wit_op, run.wit_a, run.wit_b, (flags & LTLF_FLAG_DIGEST) != 0, s));
    if (cancelled) res->status = LTLF_CANCELLED;
    return res->status;
}

ltlf_status ltlf_ctx_set_tuning(ltlf_ctx* c, const ltlf_tuning* t) {
    if (!c) return LTLF_EINVAL;
    if (!t) {
        c->tune.clear();
        return LTLF_OK;
    }
    if (t->n_classes > LTLF_TUNE_CLASSES) return LTLF_EINVAL;
    std::vector<TuneClass> tune;
    for (uint32_t i = 0; i < t->n_classes; ++i) {
        const uint32_t f = t->kernel[i];
        const uint32_t kind = f == LTLF_FLAG_KERNEL_LANE    ? KERNEL_LANE
                              : f == LTLF_FLAG_KERNEL_GROUP ? KERNEL_GROUP
                              : f == LTLF_FLAG_KERNEL_WAVE  ? KERNEL_WAVE
                                                            : 0u;
        if (!kind || t->chunks[i] == 0) return LTLF_EINVAL;
        if (t->wave_tile[i] != 0 && !wave_tile_ok(t->wave_tile[i])) return LTLF_EINVAL;
        tune.push_back(TuneClass{t->chunks[i], kind, t->wave_tile[i]});
    }
    c->tune = tune;
    return LTLF_OK;
}

ltlf_status ltlf_autotune(ltlf_ctx* c, void* stream, ltlf_tuning* out) {
    if (!c) return LTLF_EINVAL;
    c->err.clear();
    TRY_HIP(hipSetDevice(c->device));
    TRY(ensure_workspace(c));
    static const uint32_t kClasses[] = {1, 2, 4, 8, 10, 16, 24, 32, 38, 48, 64, 96, 128, 256, 328};
    static_assert(sizeof(kClasses) / sizeof(kClasses[0]) <= LTLF_TUNE_CLASSES, "tuning classes");
    constexpr uint32_t kLen = 15;  // 16 bits per trace with the guard bit
    // a timed run has levels of the size real runs spend their time in: about
    // 2e10 bytes of candidate rows (5e6 .. 1e8 candidates)
    const ltlf_costs k{1, {1, 1, 1, 1, 1, 1, 1}};
    const uint32_t flag_of[3] = {LTLF_FLAG_KERNEL_LANE, LTLF_FLAG_KERNEL_GROUP, LTLF_FLAG_KERNEL_WAVE};
    const uint32_t kind_of[3] = {KERNEL_LANE, KERNEL_GROUP, KERNEL_WAVE};
    ltlf_tuning t{};
    std::vector<TuneClass> tune;
    c->tune.clear();  // the timed runs name their kernel; the search runs use the built-in rule
    struct Unforce {
        ltlf_ctx* c;
        ~Unforce() { c->wave_tile_force = 0; }
    } unforce{c};
    static const uint32_t kTiles[3] = {8, 16, 32};
    uint64_t rng = 0x2504189430ull;
    auto next = [&rng]() {  // splitmix64
        uint64_t z = (rng += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    };
    for (uint32_t ci = 0; ci < sizeof(kClasses) / sizeof(kClasses[0]); ++ci) {
        const uint32_t chunks = kClasses[ci], T = 8 * chunks;
        std::vector<uint32_t> lengths(T, kLen), letters((uint64_t)T * kLen);
        std::vector<uint8_t> positive(T);
        for (auto& l : letters) l = (uint32_t)(next() & 7u);
        for (uint32_t i = 0; i < T; ++i) positive[i] = (uint8_t)(next() & 1u);
        const ltlf_spec sp{3, T, lengths.data(), letters.data(), positive.data()};
        TRY(ltlf_load(c, &sp, stream));
        const uint64_t want = std::min<uint64_t>(100000000ull,
                                                 std::max<uint64_t>(5000000ull, 20000000000ull / (16ull * chunks)));
        // the smallest bound whose run has enough candidates to time
        ltlf_result r{};
        uint32_t bound = 4;
        for (;; ++bound) {
            r = ltlf_result{};
            const ltlf_status st = ltlf_run(c, &k, bound, LTLF_FLAG_EXHAUST, stream, &r);
            if (st < 0) return st;
            if (r.candidates >= want || bound >= 12 || st == LTLF_CAPACITY) break;
        }
        double best = 0;
        uint32_t best_i = 2;
        // the lane kernel's family: 256-lane tiles, or 128-lane tiles where only those fit
        auto family = [](uint32_t kind) { return kind == KERNEL_LANE_HALF ? (uint32_t)KERNEL_LANE : kind; };
        // the wave kernel with each pair-tile side; the built-in side stays
        // unless another is clearly faster
        uint32_t wtile = kWaveTileBuiltin;
        for (uint32_t w = 0; w < 3; ++w) {
            c->wave_tile_force = kTiles[w];
            r = ltlf_result{};
            const ltlf_status st =
                ltlf_run(c, &k, bound, LTLF_FLAG_EXHAUST | LTLF_FLAG_PROFILE | LTLF_FLAG_KERNEL_WAVE, stream, &r);
            if (st < 0) return st;
            t.ns_wave_tile[ci][w] = 1e6 * (r.gen_ms + r.verify_ms) / (double)std::max<uint64_t>(1, r.candidates);
        }
        c->wave_tile_force = 0;
        {
            double wbest = 0;
            for (uint32_t w = 0; w < 3; ++w)
                if (wbest == 0 || t.ns_wave_tile[ci][w] < wbest) {
                    wbest = t.ns_wave_tile[ci][w];
                    wtile = kTiles[w];
                }
            if (t.ns_wave_tile[ci][1] <= 1.05 * wbest) wtile = kWaveTileBuiltin;
        }
        t.wave_tile[ci] = wtile;
        for (uint32_t i = 0; i < 3; ++i) {
            t.ns_per_candidate[ci][i] = 0;
            if (family(tile_shape(c->Wp, c->lds_limit, kind_of[i]).kind) != kind_of[i]) continue;  // does not apply
            double ns = 0;
            if (kind_of[i] == KERNEL_WAVE) {
                ns = t.ns_wave_tile[ci][wtile == 8 ? 0 : wtile == 16 ? 1 : 2];
            } else {
                r = ltlf_result{};
                const ltlf_status st =
                    ltlf_run(c, &k, bound, LTLF_FLAG_EXHAUST | LTLF_FLAG_PROFILE | flag_of[i], stream, &r);
                if (st < 0) return st;
                ns = 1e6 * (r.gen_ms + r.verify_ms) / (double)std::max<uint64_t>(1, r.candidates);
            }
            t.ns_per_candidate[ci][i] = ns;
            t.candidates[ci] = r.candidates;
            if (best == 0 || ns < best) {
                best = ns;
                best_i = i;
            }
        }
        // the built-in choice stays unless another kernel is clearly faster
        // (measurements of near-equal kernels vary by a few percent)
        const uint32_t builtin = family(tile_shape(c->Wp, c->lds_limit, kBuiltinPref).kind);
        for (uint32_t i = 0; i < 3; ++i)
            if (kind_of[i] == builtin && t.ns_per_candidate[ci][i] > 0 && t.ns_per_candidate[ci][i] <= 1.05 * best)
                best_i = i;
        t.chunks[ci] = chunks;
        t.kernel[ci] = flag_of[best_i];
        t.bound[ci] = bound;
        t.n_classes = ci + 1;
        tune.push_back(TuneClass{chunks, kind_of[best_i], wtile});
    }
    c->tune = tune;
    c->loaded = false;
    c->ran = false;
    if (out) *out = t;
    return LTLF_OK;
}

ltlf_status ltlf_solve(ltlf_ctx* c, const ltlf_spec* sp, const ltlf_costs* k, uint32_t bound,
                       uint32_t flags, void* stream, ltlf_result* res) {
    TRY(ltlf_load(c, sp, stream));
    return ltlf_run(c, k, bound, flags, stream, res);
}

ltlf_status ltlf_solve_static(ltlf_ctx* c, const ltlf_spec* sp, const ltlf_costs* k, uint32_t bound,
                              uint32_t flags, void* stream, ltlf_result* res) {
    if (!c || !sp || !k || !res) return LTLF_EINVAL;
    c->err.clear();
    if (flags & LTLF_FLAG_PROFILE) return fail(c, LTLF_EINVAL, "LTLF_FLAG_PROFILE creates events: not available here");
    TRY_HIP(hipSetDevice(c->device));
    void* p = nullptr;
    TRY_HIP(static_workspace(c->device, &p));
    // the context's own workspace is put aside for the call; the problem
    // lives in the static array, so nothing of it stays loaded afterwards
    struct Swap {
        ltlf_ctx* c;
        char* ws;
        uint64_t bytes;
        bool own;
        ~Swap() {
            c->ws = ws;
            c->ws_bytes = bytes;
            c->own_ws = own;
            c->loaded = false;
            c->ran = false;
        }
    } swap{c, c->ws, c->ws_bytes, c->own_ws};
    c->ws = static_cast<char*>(p);
    c->ws_bytes = kStaticWorkspaceBytes;
    c->own_ws = false;
    c->loaded = false;
    const ltlf_status st = ltlf_solve(c, sp, k, bound, flags, stream, res);
    if (st == LTLF_ENOMEM)
        return fail(c, LTLF_ENOMEM, "the specification's fixed regions need more than the 64 MiB static workspace");
    return st;
}

ltlf_status ltlf_solve_batch(ltlf_ctx* c, uint32_t n, const ltlf_spec* specs, const ltlf_costs* k,
                             const uint32_t* bounds, uint32_t flags, void* stream, ltlf_result* results) {
    if (!c || !specs || !k || !bounds || !results || n == 0) return LTLF_EINVAL;
    c->err.clear();
    if (k->atom_cost == 0) return LTLF_EINVAL;
    TRY_HIP(hipSetDevice(c->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    Scheduler sc;
    TRY(sc.init(c, n));
    hipEvent_t e0 = c->evb0, e1 = c->evb1;
    TRY_HIP(hipEventRecord(e0, s));
    std::vector<uint64_t> ticket(n, 0);
    for (uint32_t i = 0; i < n; ++i) {
        const ltlf_status st = sc.submit(&specs[i], k, bounds[i], flags, 0, &ticket[i]);
        if (st == LTLF_EINVAL) {
            reset_result(&results[i], 0);
            results[i].status = LTLF_EINVAL;
            ticket[i] = 0;
        } else if (st != LTLF_OK) {
            return st;
        }
    }
    while (!sc.idle()) {
        if (c->cancel.exchange(false, std::memory_order_acq_rel)) {
            TRY(sc.cancel_all(s));
            break;
        }
        TRY(sc.step(s, nullptr));
    }
    TRY_HIP(hipEventRecord(e1, s));
    TRY_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    TRY_HIP(hipEventElapsedTime(&ms, e0, e1));
    for (uint32_t i = 0; i < n; ++i) {
        if (!ticket[i]) continue;
        const ltlf_status st = sc.collect(ticket[i], &results[i]);
        if (st < 0 && st != LTLF_EBUFSZ) return st;
        results[i].enum_ms = ms;
    }
    c->loaded = false;
    return LTLF_OK;
}

struct ltlf_server {
    Scheduler sched;
};

ltlf_status ltlf_server_create(ltlf_ctx* c, uint32_t max_resident, ltlf_server** out) {
    if (!c || !out || max_resident == 0 || max_resident > 65535) return LTLF_EINVAL;
    *out = nullptr;
    c->err.clear();
    TRY_HIP(hipSetDevice(c->device));
    ltlf_server* sv = new (std::nothrow) ltlf_server();
    if (!sv) return LTLF_ENOMEM;
    const ltlf_status st = sv->sched.init(c, max_resident);
    if (st != LTLF_OK) {
        delete sv;
        return st;
    }
    *out = sv;
    return LTLF_OK;
}

ltlf_status ltlf_server_submit(ltlf_server* sv, const ltlf_spec* sp, const ltlf_costs* k, uint32_t bound,
                               uint32_t flags, uint64_t reserve_bytes, uint64_t* ticket) {
    if (!sv || !ticket) return LTLF_EINVAL;
    return sv->sched.submit(sp, k, bound, flags, reserve_bytes, ticket);
}

ltlf_status ltlf_server_step(ltlf_server* sv, void* stream, uint32_t* n_done) {
    if (!sv) return LTLF_EINVAL;
    ltlf_ctx* c = sv->sched.c;
    TRY_HIP(hipSetDevice(c->device));
    return sv->sched.step(static_cast<hipStream_t>(stream), n_done);
}

ltlf_status ltlf_server_poll(ltlf_server* sv, uint64_t ticket, ltlf_result* res) {
    if (!sv || !res) return LTLF_EINVAL;
    return sv->sched.collect(ticket, res);
}

ltlf_status ltlf_server_cancel(ltlf_server* sv, uint64_t ticket) {
    if (!sv) return LTLF_EINVAL;
    return sv->sched.cancel(ticket);
}

ltlf_status ltlf_server_load(const ltlf_server* sv, uint32_t* queued, uint32_t* resident, uint64_t* free_bytes) {
    if (!sv) return LTLF_EINVAL;
    if (queued) *queued = sv->sched.waiting();
    if (resident) *resident = sv->sched.on_device();
    if (free_bytes) {
        uint64_t f = 0;
        f = sv->sched.free_bytes();
        *free_bytes = f;
    }
    return LTLF_OK;
}

void ltlf_server_destroy(ltlf_server* sv) {
    if (!sv) return;
    if (sv->sched.c) sv->sched.c->loaded = false;
    delete sv;
}

ltlf_status ltlf_export_level(ltlf_ctx* c, uint32_t cost, uint64_t first, uint64_t count,
                              uint64_t* host_buf, uint64_t cap_words, uint64_t* n_cms,
                              uint64_t* words_per_cm) {
    if (!c || !n_cms || !words_per_cm) return LTLF_EINVAL;
    if (!c->ran) return LTLF_ESTATE;
    if (cost == 0 || cost > c->levels_done) return LTLF_EINVAL;
    const uint64_t cw = (c->n_pos + 63) / 64;
    const uint64_t total = c->lcount[cost];
    const uint64_t lo = std::min(first, total);
    const uint64_t n = std::min(count, total - lo);
    *n_cms = n;
    *words_per_cm = cw;
    if (!host_buf) return LTLF_OK;
    if (cap_words < n * cw) return LTLF_EBUFSZ;
    TRY_HIP(hipSetDevice(c->device));
    if (c->staging_bytes < 8 * cw) return LTLF_ESTATE;
    const uint64_t per = std::max<uint64_t>(1, c->staging_bytes / 8 / cw);
    for (uint64_t q = 0; q < n; q += per) {
        const uint64_t m = std::min<uint64_t>(per, n - q);
        TRY_HIP(launch_export(c->st.rows, c->Wp, c->lstart[cost] + lo + q, m, c->d_canon, c->n_pos,
                              c->d_stage, nullptr));
        TRY_HIP(hipMemcpy(host_buf + q * cw, c->d_stage, 8 * m * cw, hipMemcpyDeviceToHost));
    }
    return LTLF_OK;
}

ltlf_status ltlf_formula_of(ltlf_ctx* c, uint32_t cost, uint64_t index, char* buf, uint64_t cap,
                            uint64_t* need) {
    if (!c || !need) return LTLF_EINVAL;
    if (!c->ran) return LTLF_ESTATE;
    if (cost == 0 || cost > c->levels_done || index >= c->lcount[cost]) return LTLF_EINVAL;
    TRY_HIP(hipSetDevice(c->device));
    uint4 m;
    TRY_HIP(hipMemcpy(&m, c->st.meta + c->lstart[cost] + index, sizeof(uint4), hipMemcpyDeviceToHost));
    std::string f;
    TRY(render_formula(c, m.x & 7u, m.y, m.z, nullptr, f));
    *need = f.size() + 1;
    if (!buf || cap < f.size() + 1) return LTLF_EBUFSZ;
    std::memcpy(buf, f.c_str(), f.size() + 1);
    return LTLF_OK;
}

}  // extern "C"
