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
enum : uint32_t {
    C_ROWS = 0,       // rows allocated (may run past capacity on overflow)
    C_FOUND = 1,      // 1 once a separating CM was seen
    C_OVERFLOW = 2,   // 1 once a row could not be allocated
    C_DEF0 = 3,       // records in deferral list 0
    C_DEF1 = 4,       // records in deferral list 1
    C_CAND = 5,       // candidates generated
    C_DEF_OVF = 6,    // a deferral list ran out of room (internal error)
    C_WIT_OP = 7,     // witness derivation
    C_WIT_A = 8,
    C_WIT_B = 9,
    C_DEFERRED = 10,  // total deferrals (statistics)
    C_VERIFY = 11,    // verification reads (statistics)
    C_SNAP = 12,      // row count when the running inserting launch started
    C_NUM = 16,
};

enum : uint32_t { SEG_ATOM = 0, SEG_UNARY = 1, SEG_PAIR = 2 };

constexpr uint32_t kLanes = 256;   // workgroup size; lane operand tile
constexpr uint32_t kTileA = 16;    // loop operands per pair tile
constexpr uint32_t kMaxSegs = 40;  // segments per launch

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
    uint64_t first[kMaxSegs + 1];  // prefix sums of tiles
    Seg seg[kMaxSegs];
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
};

// Launchers (defined in ltlf_kernels.hip).
hipError_t launch_encode(const uint32_t* letters, const uint32_t* lengths, const uint32_t* pos_off,
                         const uint32_t* seg_off, const uint8_t* positive, uint32_t n_traces,
                         uint32_t n_props, uint32_t Wp, uint32_t* V, uint32_t* S, uint32_t* P0,
                         uint32_t* atoms, hipStream_t st);
hipError_t launch_fill_u64(uint64_t* p, uint64_t n, uint64_t v, hipStream_t st);
// Dynamic LDS bytes of the LDS-staged generation kernel for rows of Wp words;
// rows needing more than lds_limit use the generic kernel.
uint64_t lds_bytes(uint32_t Wp);
hipError_t launch_generate(const Store& s, const SegTable& t, uint64_t lds_limit, hipStream_t st);
hipError_t launch_verify_deferred(const Store& s, hipStream_t st);
hipError_t launch_reinsert(const Store& s, uint64_t n, hipStream_t st);
// Sets C_DEF0 = 0 and C_SNAP = C_ROWS; must run between any launch that
// allocates rows and the next inserting launch.
hipError_t launch_between(unsigned long long* ctr, hipStream_t st);
hipError_t launch_set_counter(unsigned long long* ctr, uint32_t which, unsigned long long v,
                              hipStream_t st);
hipError_t launch_rehash(const Store& s, uint64_t n_rows, hipStream_t st);
hipError_t launch_export(const uint32_t* rows, uint32_t Wp, uint64_t first, uint64_t n,
                         const uint32_t* canon_bit, uint64_t n_bits, uint64_t* out, hipStream_t st);
// tokens must hold 1 + max_tokens + 3 * (max_tokens + 1) words (list + stack).
hipError_t launch_formula(const uint4* meta, uint32_t root_op, uint32_t root_a, uint32_t root_b,
                          uint32_t max_tokens, uint32_t* tokens, hipStream_t st);

}  // namespace ltlf
