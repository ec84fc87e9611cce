// Internal declarations shared by the host driver and the HIP kernels of the
// library (both are product code; nothing here is part of the public ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ltlf {

// Operator codes stored in derivation records.  The unary/binary codes follow
// ltlf_op + 1; 0 is an atom.
enum : uint32_t {
    OP_ATOM = 0,
    OP_NOT = 1,
    OP_X = 2,
    OP_F = 3,
    OP_G = 4,
    OP_AND = 5,
    OP_OR = 6,
    OP_U = 7,
};

// Bits of a segment's op mask.
enum : uint32_t {
    M_NOT = 1u << 0,
    M_X = 1u << 1,
    M_F = 1u << 2,
    M_G = 1u << 3,
    M_AND = 1u << 4,
    M_OR = 1u << 5,
    M_UAB = 1u << 6,  // a U b  (a = loop operand, b = lane operand)
    M_UBA = 1u << 7,  // b U a
};

// Slots of the device counter block (uint64 each).
// Device counters (64-bit).  The ones that take atomics all the time (row,
// deferral and tile counters) each have a 128-byte cache line of their own,
// and the read-mostly flags share another: a coherent read of a line that is
// under constant atomic traffic waits behind that traffic.
enum : uint32_t {
    C_ROWS = 0,        // rows allocated (may run past capacity on overflow)
    C_DEF0 = 16,       // records in deferral list 0
    C_TILE = 32,       // persistent kernels: tile cursor, kept over the launches of one segment table
    C_DEF1 = 48,       // records in deferral list 1
    C_CAND = 49,       // candidates generated
    C_DEF_OVF = 50,    // a deferral list ran out of room (internal error)
    C_DEFERRED = 51,   // deferred records verified (statistics)
    C_VERIFY = 52,     // verification reads (statistics)
    C_DEAD = 53,       // rows of the level left unused (retired chunk tails)
    C_NH = 54,         // compaction: holes found
    C_NM = 55,         // compaction: rows to move
    C_SNAP = 64,       // row count when the running inserting launch started
    C_OVERFLOW = 65,   // 1 once a row could not be allocated
    C_FOUND = 66,      // 1 once a separating CM was seen
    C_WIT_OP = 67,     // witness derivation
    C_WIT_A = 68,
    C_WIT_B = 69,
    C_NUM = 80,
};

enum : uint32_t { SEG_ATOM = 0, SEG_UNARY = 1, SEG_PAIR = 2 };

constexpr uint32_t kLanes = 256;   // workgroup size; lane operand tile
constexpr uint32_t kTileA = 16;    // loop operands per pair tile
constexpr uint32_t kMaxSegs = 40;  // segments per launch
constexpr uint32_t kAllocChunk = 64;  // rows / records a wave takes per atomic (group kernel)

struct Seg {
    uint32_t kind;    // SEG_*
    uint32_t opmask;  // M_* bits
    uint32_t tri;     // pair segment over one level: only pairs a < b
    uint32_t pad;
    uint64_t a0, na;  // loop operand rows [a0, a0+na)
    uint64_t b0, nb;  // lane operand rows [b0, b0+nb)
    uint64_t tiles;   // tiles in this segment
};

struct SegTable {
    uint32_t n;
    uint32_t pad;
    uint64_t tile_begin;  // first tile (inclusive) handled by this launch
    uint64_t tile_end;    // last tile (exclusive)
    // persistent group kernel only (tiles [0, tile_end) from the C_TILE
    // cursor): a block takes a tile only while C_DEF0 + def_margin <= the
    // deferral capacity and C_ROWS + row_margin <= row_budget, and while the
    // cursor is below tile_stop (a launch's share of the level; blocks that
    // pass the test together may take a few tiles beyond it)
    uint64_t def_margin, row_margin, row_budget, tile_stop;
    uint64_t first[kMaxSegs + 1];  // prefix sums of tiles
    Seg seg[kMaxSegs];
};

// Piece of a segment in a batched launch: launch tiles [first, first + n)
// are the segment's local tiles [lt0, lt0 + n) of problem `problem` (pieces
// sorted by first, contiguous).
struct BSeg {
    uint32_t problem;
    uint32_t pad;
    uint64_t first, lt0;
    Seg seg;
};


// Device-side view of one loaded problem and its store.
struct Store {
    const uint32_t* V;      // valid-position mask, Wp words
    const uint32_t* S;      // position-0 mask
    const uint32_t* P0;     // position-0 mask of positive traces
    const uint32_t* atoms;  // n_props rows of Wp words
    uint32_t* rows;         // cap rows of Wp words
    uint4* meta;            // per row {op | tag << 3, a, b, low 32 hash bits}
    uint64_t* table;        // open addressing, tsize slots
    uint64_t tsize;         // slots in use (<= 2^32)
    unsigned long long* ctr;  // C_NUM counters
    uint4* def0;            // deferral list written by generation kernels
    uint4* def1;            // records that still need inserting
    uint64_t def0_cap, def1_cap;
    uint64_t cap;           // row capacity
    uint64_t hmask;         // hash mask (all ones; fewer bits force collisions in tests)
    uint32_t Wp;            // words per row (multiple of 4)
    uint32_t n_props;
    uint32_t kernel;        // KERNEL_* generation kernel of the run
    uint32_t wtile;         // wave kernel: side of its square pair tiles (unary tiles: 2 x wtile operands)
};

// Launchers (defined in ltlf_kernels.hip).
hipError_t launch_encode(const uint32_t* letters, const uint32_t* lengths, const uint32_t* pos_off,
                         const uint32_t* seg_off, const uint8_t* positive, uint32_t n_traces,
                         uint32_t n_props, uint32_t Wp, uint32_t* V, uint32_t* S, uint32_t* P0,
                         uint32_t* atoms, hipStream_t st);
hipError_t launch_fill_u64(uint64_t* p, uint64_t n, uint64_t v, hipStream_t st);
// Generation kernel chosen for rows of Wp words, and its tile shape: pair
// tiles of ta left x tb right operands, unary tiles of tu operands; triangular
// (same-level) pair segments use square tiles if square_tri, else columns of
// 16(k+1) left tiles per right tile k.
enum : uint32_t { KERNEL_LANE = 1, KERNEL_GROUP = 2, KERNEL_AUTO = 3, KERNEL_WAVE = 4, KERNEL_LANE_HALF = 5 };
struct TileShape {
    uint32_t kind, ta, tb, tu, square_tri;
};
// Generation kernel and tile for rows of Wp words.  pref: KERNEL_LANE or
// KERNEL_GROUP asks for that kernel where it fits (the lane kernel on
// 128-lane tiles, KERNEL_LANE_HALF, where only those fit), KERNEL_WAVE for
// the wave kernel, anything else is the default (lane kernel where its
// 256-lane tile fits the LDS, else the group kernel for rows of 2..64 chunks,
// else the wave kernel).
// wave_tile: side of the wave kernel's pair tiles (8, 16 or 32; 0: the
// built-in 16).
constexpr uint32_t kWaveTileBuiltin = 16;
TileShape tile_shape(uint32_t Wp, uint64_t lds_limit, uint32_t pref, uint32_t wave_tile = 0);
inline bool wave_tile_ok(uint32_t t) { return t == 8 || t == 16 || t == 32; }
uint64_t lds_bytes(uint32_t Wp, uint32_t lanes);
// Grid of the generation launch: the tile count, or for the persistent group
// kernel the resident block count (at most the tile count).
hipError_t generate_blocks(const Store& s, uint64_t n_tiles, uint64_t& blocks);
hipError_t launch_generate(const Store& s, const SegTable& t, uint64_t blocks, hipStream_t st);
hipError_t launch_verify_deferred(const Store& s, hipStream_t st);
// Batched solving (device arrays of per-problem stores and segments).
// Look-ahead past an overflowed level: tiles [tile_begin, tile_end) of that
// level's plan (wave-kernel tile shape), each candidate with the cost-1 unary
// operators of omask (bits: not, X, F, G) applied and checked; one block per
// tile.
hipError_t launch_lookahead(const Store& s, const SegTable& t, uint32_t omask, hipStream_t st);
hipError_t launch_generate_batch(const Store* d_stores, const BSeg* d_segs, uint32_t nsegs, uint64_t tile0,
                                 uint64_t tiles, hipStream_t st);
hipError_t launch_verify_batch(const Store* d_stores, uint32_t n, hipStream_t st);
hipError_t launch_between_batch(const Store* d_stores, uint32_t n, hipStream_t st);
hipError_t launch_gather_ctr(const Store* d_stores, uint32_t n, unsigned long long* out, hipStream_t st);
// The batched launch (generation over pieces of every problem's plan,
// verification, between-launch reset) as an executable graph, replayed per
// launch with its counts and grids written into it (set_step: nsegs pieces
// at d_segs covering `tiles` launch tiles, n problems at d_stores).
struct StepGraphs {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipGraphNode_t gen = nullptr, ver = nullptr, btw = nullptr;
    const Store* d_stores = nullptr;
    const BSeg* d_segs = nullptr;
};
hipError_t make_step_graphs(StepGraphs& g);
hipError_t set_step(StepGraphs& g, uint32_t nsegs, uint64_t tiles, uint32_t n);
void free_step_graphs(StepGraphs& g);
hipError_t launch_reinsert(const Store& s, uint64_t n, hipStream_t st);
// Sets C_DEF0 = 0 and C_SNAP = C_ROWS; must run between any launch that
// allocates rows and the next inserting launch.
hipError_t launch_between(unsigned long long* ctr, hipStream_t st);
hipError_t launch_set_counter(unsigned long long* ctr, uint32_t which, unsigned long long v,
                              hipStream_t st);
hipError_t launch_rehash(const Store& s, uint64_t n_rows, hipStream_t st);
// Level compaction over [lo, hi) (one round): lists up to `cap` holes below
// new_end and live rows above it (C_NH, C_NM must be zero), then moves rows
// and repoints their table slots.
hipError_t launch_compact(const Store& s, uint64_t lo, uint64_t new_end, uint64_t hi, uint32_t* holes,
                          uint32_t* movers, uint64_t cap, hipStream_t st);
hipError_t launch_export(const uint32_t* rows, uint32_t Wp, uint64_t first, uint64_t n,
                         const uint32_t* canon_bit, uint64_t n_bits, uint64_t* out, hipStream_t st);
// Static scratch workspace of ltlf_solve_static: kStaticWorkspaceBytes of
// device memory per device (a file-scope device array); *ptr receives this
// device's address of it.  The device must be current.
constexpr uint64_t kStaticWorkspaceBytes = 64ull << 20;
constexpr uint32_t kMaxStaticDevices = 64;
hipError_t static_workspace(int device, void** ptr);
// Adds the digest of rows [first, first + n) to *out (see k_digest).
hipError_t launch_digest(const uint32_t* rows, uint32_t Wp, uint64_t first, uint64_t n,
                         unsigned long long* out, hipStream_t st);
// tokens must hold 1 + max_tokens + 3 * (max_tokens + 1) words (list + stack).
hipError_t launch_formula(const uint4* meta, uint32_t root_op, uint32_t root_a, uint32_t root_b,
                          uint32_t max_tokens, uint32_t* tokens, hipStream_t st);

}  // namespace ltlf
