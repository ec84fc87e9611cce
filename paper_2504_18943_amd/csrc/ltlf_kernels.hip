// HIP kernels (gfx950) for bottom-up LTLf semantic enumeration.
//
// Representation (paper, "Parallel enumeration of LTLf formulae on GPUs":
// characteristic sequences/matrices, suffix-contiguity).  All traces of the
// specification are packed into one bit string of 32-bit words.  Trace t
// occupies a segment of n_t + 1 bits; from the low end of the segment upward
// the bits are position n_t-1, ..., position 1, position 0, then one guard
// bit that is always 0.  A row is Wp words (Wp a multiple of 4, so a row is a
// whole number of 16-byte vectors); padding bits are 0.  V marks the valid
// position bits, S the position-0 bits, P0 the position-0 bits of positive
// traces.
//
// Operators on this layout, word by word from the lowest word up:
//   not a      = ~a & V
//   X a        = (a << 1, with the top bit of the next lower word shifted in) & V
//                position k receives position k+1; the guard below each
//                segment feeds 0 into the last position, so X is strong.
//   F a        = a | (V & c),  c = (a + V) ^ a ^ V   (multi-word add)
//                c holds at a bit iff some lower bit of the same segment is
//                set in a (V is all ones inside a segment, so the carry runs
//                up from the lowest set bit); the guard (0 in both a and V)
//                stops every carry at the segment end.  This is the
//                reflexive suffix-OR that the paper computes with log-step
//                shifts, done with one add per word and no length limit.
//   G a        = V & ~F(V & ~a)
//   a and b, a or b: bitwise
//   a U b      = b | (a & c),  c = (b + (a|b)) ^ b ^ (a|b)
//                a carry reaches bit i iff below i there is a bit with b set
//                and every bit between holds a and not b, which is the
//                reflexive until.
//
// Deduplication (paper: observational equivalence; one representative per
// distinct CM, global over all levels).  Open addressing over 2^k 64-bit
// slots: high word = 32-bit tag of the hash, low word = row index; EMPTY is
// all ones, a slot whose low word is 0xFFFFFFFF is reserved but not yet
// published.  A candidate probes linearly from hash & mask.  A slot with a
// matching tag is verified against the stored row only if the row was written
// by an earlier launch (index below the row count at launch start, kept in
// the counter block by a small kernel between launches); rows written by the
// running launch are not read, because on a multi-XCD device they are not
// guaranteed to be visible inside the same launch without cache maintenance.
// Such candidates are appended to a deferral list and verified by the next
// kernel.  Winning a slot (CAS EMPTY -> reserved) gives the candidate the
// right to allocate a row, write it, and publish the index.  Every outcome is
// exact: a candidate is dropped only after a full-row comparison.
#include "ltlf_internal.h"

#include <mutex>

namespace ltlf {

static constexpr uint64_t kEmpty = ~0ull;
static constexpr uint32_t kPending = 0xFFFFFFFFu;
// Derivation record of a row index that was allocated but never used (y),
// and operator code of an unused deferral record.
static constexpr uint32_t kDead = 0xFFFFFFFFu;
static constexpr uint32_t kNoRecord = 0xFu;

// ----------------------------------------------------------- table atomics --
__device__ __forceinline__ uint64_t slot_load(uint64_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t slot_cas(uint64_t* p, uint64_t expect, uint64_t want) {
    __hip_atomic_compare_exchange_strong(p, &expect, want, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT);
    return expect;
}
__device__ __forceinline__ void slot_store(uint64_t* p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The store has overflowed (no more slots are reserved; candidates are only
// checked).  A coherent load: the flag is set by other blocks of the running
// launch, and a launch that kept reserving slots after it was set could fill
// the table.
__device__ __forceinline__ bool store_full(const Store& s) {
    return __hip_atomic_load(&s.ctr[C_OVERFLOW], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
}

// One atomicAdd per wave for every lane that is active at the call site.
__device__ __forceinline__ unsigned long long wave_alloc(unsigned long long* ctr) {
    const uint64_t active = __ballot(1);
    const uint32_t lane = __lane_id();
    const uint32_t leader = (uint32_t)__ffsll((unsigned long long)active) - 1u;
    const uint32_t rank = (uint32_t)__popcll(active & ((1ull << lane) - 1ull));
    unsigned long long base = 0;
    if (lane == leader) base = atomicAdd(ctr, (unsigned long long)__popcll(active));
    base = __shfl(base, (int)leader);
    return base + rank;
}

// ----------------------------------------------------------------- hashing --
// Hash of a CM: the XOR over its 16-byte chunks k of chunk_hash(k, chunk),
// then a 64-bit finaliser.  Chunks are independent, so a group of lanes that
// holds one chunk each combines its parts with shuffles, and every kernel
// (one lane per candidate or one group per candidate) gets the same value.
// Only speed depends on the quality: every match is verified against the
// full row.  chunk_hash is a keyed multiply-add in the manner of NH: the four
// words plus four keys of the chunk index, multiplied in pairs into 64 bits
// (two 32 x 32 -> 64 multiply-adds per chunk).  The keys depend on the chunk
// index only, so the candidates of a work item share them, and a lane that
// walks a row keeps them in scalar registers.
struct ChunkKey {
    uint32_t k0, k1, k2, k3;
};
__device__ __forceinline__ ChunkKey chunk_key(uint32_t k) {
    const uint32_t u = (k + 1u) * 0x9E3779B9u;
    return ChunkKey{u ^ 0x85EBCA6Bu, u + 0xC2B2AE35u, ((u << 13) | (u >> 19)) ^ 0x27D4EB2Fu,
                    ((u << 27) | (u >> 5)) + 0x165667B1u};
}
__device__ __forceinline__ uint64_t chunk_hash(const ChunkKey& K, uint4 r) {
    return (uint64_t)(r.x + K.k0) * (uint64_t)(r.y + K.k1) + (uint64_t)(r.z + K.k2) * (uint64_t)(r.w + K.k3);
}
__device__ __forceinline__ uint64_t chunk_hash(uint32_t k, uint4 r) { return chunk_hash(chunk_key(k), r); }
__device__ __forceinline__ uint64_t hash_fin(uint64_t k) {
    k ^= k >> 33;
    k *= 0xff51afd7ed558ccdull;
    k ^= k >> 33;
    k *= 0xc4ceb9fe1a85ec53ull;
    k ^= k >> 33;
    return k;
}
struct Hash {
    uint64_t acc = 0;
    uint32_t k = 0;
    __device__ __forceinline__ void add4(uint4 r) { acc ^= chunk_hash(k++, r); }
    __device__ __forceinline__ uint64_t fin() const { return hash_fin(acc); }
};

// --------------------------------------------------------------- operators --
__device__ __forceinline__ uint32_t addc(uint32_t x, uint32_t y, uint32_t& carry) {
    const uint64_t s = (uint64_t)x + y + carry;
    carry = (uint32_t)(s >> 32);
    return (uint32_t)s;
}

template <uint32_t OP>
__device__ __forceinline__ uint32_t op_word(uint32_t a, uint32_t b, uint32_t v, uint32_t& st) {
    if constexpr (OP == OP_ATOM) {
        return a;
    } else if constexpr (OP == OP_NOT) {
        return ~a & v;
    } else if constexpr (OP == OP_X) {
        const uint32_t r = ((a << 1) | st) & v;
        st = a >> 31;
        return r;
    } else if constexpr (OP == OP_F) {
        const uint32_t s = addc(a, v, st);
        return a | (v & (s ^ a ^ v));
    } else if constexpr (OP == OP_G) {
        const uint32_t x = v & ~a;
        const uint32_t s = addc(x, v, st);
        return v & ~(x | (v & (s ^ x ^ v)));
    } else if constexpr (OP == OP_AND) {
        return a & b;
    } else if constexpr (OP == OP_OR) {
        return a | b;
    } else {  // OP_U: a U b
        const uint32_t p = a | b;
        const uint32_t s = addc(b, p, st);
        return b | (a & (s ^ b ^ p));
    }
}

template <uint32_t OP>
__device__ __forceinline__ uint4 op_vec(uint4 a, uint4 b, uint4 v, uint32_t& st) {
    uint4 r;
    r.x = op_word<OP>(a.x, b.x, v.x, st);
    r.y = op_word<OP>(a.y, b.y, v.y, st);
    r.z = op_word<OP>(a.z, b.z, v.z, st);
    r.w = op_word<OP>(a.w, b.w, v.w, st);
    return r;
}

// *p if c, else zero.  Written as a branch: the select form `c ? p[i] : z`
// with a zero local becomes a select between p and a stack copy of z, i.e.
// flat (generic) loads even for LDS and global pointers.
__device__ __forceinline__ uint4 load_if(bool c, const uint4* p) {
    uint4 v = make_uint4(0, 0, 0, 0);
    if (c) v = *p;
    return v;
}

__device__ __forceinline__ uint32_t diff4(uint4 a, uint4 b) {
    return (a.x ^ b.x) | (a.y ^ b.y) | (a.z ^ b.z) | (a.w ^ b.w);
}

__device__ __forceinline__ bool is_binary(uint32_t op) { return op >= OP_AND; }

__device__ __forceinline__ const uint32_t* operand(const Store& s, uint32_t op, uint32_t idx) {
    return op == OP_ATOM ? s.atoms + (uint64_t)idx * s.Wp : s.rows + (uint64_t)idx * s.Wp;
}

// Streams the candidate op(L, R) 16 bytes at a time into fn(word_index, r);
// fn returns false to stop early.
template <uint32_t OP, class Fn>
__device__ __forceinline__ void stream_op(const Store& s, const uint32_t* A, const uint32_t* B,
                                          Fn&& fn) {
    uint32_t st = 0;
    const uint4 zero = make_uint4(0, 0, 0, 0);
    for (uint32_t w = 0; w < s.Wp; w += 4) {
        const uint4 a = *reinterpret_cast<const uint4*>(A + w);
        const uint4 b = load_if(is_binary(OP), reinterpret_cast<const uint4*>(B + w));
        const uint4 v = *reinterpret_cast<const uint4*>(s.V + w);
        if (!fn(w, op_vec<OP>(a, b, v, st))) return;
    }
}

template <class Fn>
__device__ __forceinline__ void stream_cm(const Store& s, uint32_t op, uint32_t L, uint32_t R,
                                          Fn&& fn) {
    const uint32_t* A = operand(s, op, L);
    const uint32_t* B = is_binary(op) ? s.rows + (uint64_t)R * s.Wp : nullptr;
    switch (op) {
    case OP_ATOM: stream_op<OP_ATOM>(s, A, B, fn); break;
    case OP_NOT: stream_op<OP_NOT>(s, A, B, fn); break;
    case OP_X: stream_op<OP_X>(s, A, B, fn); break;
    case OP_F: stream_op<OP_F>(s, A, B, fn); break;
    case OP_G: stream_op<OP_G>(s, A, B, fn); break;
    case OP_AND: stream_op<OP_AND>(s, A, B, fn); break;
    case OP_OR: stream_op<OP_OR>(s, A, B, fn); break;
    default: stream_op<OP_U>(s, A, B, fn); break;
    }
}

// An emitter streams one candidate's CM as 16-byte vectors: e(fn) calls
// fn(w, r) for word index w = 0, 4, 8, ... until fn returns false.  The
// generic emitter reads both operands from the row store; the register
// emitters below read them from VGPRs and LDS.
struct GlobalEmit {
    static constexpr bool kChunked = false;
    const Store& s;
    uint32_t op, L, R;
    template <class Fn>
    __device__ __forceinline__ void operator()(Fn&& fn) const {
        stream_cm(s, op, L, R, fn);
    }
};

template <class Emit>
__device__ __forceinline__ uint64_t emit_hash(const Store& s, const Emit& e) {
    Hash h;
    e([&](uint32_t, uint4 r) {
        h.add4(r);
        return true;
    });
    return h.fin() & s.hmask;
}

constexpr uint32_t kVerifyGroup = 8;

// Full comparison of candidate e with stored row `row`.  Emitters that can
// produce chunk q directly (kChunked) compare in groups of kVerifyGroup chunks whose
// loads are issued together, so a row costs ceil(chunks / kVerifyGroup) memory round
// trips instead of one per chunk (the early exit of the streamed form makes
// every load wait for the previous comparison).
template <class Emit>
__device__ __forceinline__ bool emit_equal_row(const Store& s, uint64_t row, const Emit& e) {
    const uint4* M = reinterpret_cast<const uint4*>(s.rows + row * s.Wp);
    if constexpr (Emit::kChunked) {
        const uint32_t nq = s.Wp / 4;
        uint32_t st = 0;
        for (uint32_t q0 = 0; q0 < nq; q0 += kVerifyGroup) {
            uint4 m[kVerifyGroup];
#pragma unroll
            for (uint32_t i = 0; i < kVerifyGroup; ++i) m[i] = load_if(q0 + i < nq, &M[q0 + i]);
            uint32_t d = 0;
#pragma unroll
            for (uint32_t i = 0; i < kVerifyGroup; ++i)
                if (q0 + i < nq) d |= diff4(e.at(q0 + i, st), m[i]);
            if (d != 0) return false;
        }
        return true;
    } else {
        bool eq = true;
        e([&](uint32_t w, uint4 r) {
            const uint4 m = M[w >> 2];
            eq = (r.x == m.x) && (r.y == m.y) && (r.z == m.z) && (r.w == m.w);
            return eq;
        });
        return eq;
    }
}

// Spec check (paper: phi separates (P, N) iff it holds at position 0 of every
// positive trace and of no negative one): ((cm ^ P0) & S) == 0 in every word.
struct Masks {
    const uint4* S;
    const uint4* P;
};
__device__ __forceinline__ uint32_t check_vec(const Masks& m, uint32_t w, uint4 r) {
    const uint4 p = m.P[w >> 2];
    const uint4 q = m.S[w >> 2];
    return ((r.x ^ p.x) & q.x) | ((r.y ^ p.y) & q.y) | ((r.z ^ p.z) & q.z) | ((r.w ^ p.w) & q.w);
}

__device__ __forceinline__ void report_found(const Store& s, uint32_t op, uint32_t L, uint32_t R) {
    if (__hip_atomic_load(&s.ctr[C_FOUND], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0ull &&
        atomicCAS(&s.ctr[C_FOUND], 0ull, 1ull) == 0ull) {
        atomicExch(&s.ctr[C_WIT_OP], (unsigned long long)op);
        atomicExch(&s.ctr[C_WIT_A], (unsigned long long)L);
        atomicExch(&s.ctr[C_WIT_B], (unsigned long long)R);
    }
}

template <class Emit>
__device__ __forceinline__ void emit_check_only(const Store& s, const Masks& m, uint32_t op,
                                                uint32_t L, uint32_t R, const Emit& e) {
    uint32_t acc = 0;
    e([&](uint32_t w, uint4 r) {
        acc |= check_vec(m, w, r);
        return true;
    });
    if (acc == 0) report_found(s, op, L, R);
}

// Slot tag: the top 29 bits of the hash (never all ones, so a reserved slot
// never reads as EMPTY).  The derivation record keeps the tag next to the
// operator code and the low 32 hash bits beside it, so the table can be
// rebuilt from the records alone (table size <= 2^32 slots).
__device__ __forceinline__ uint32_t tag_of(uint64_t h) { return (uint32_t)(h >> 35); }

// Home slot of hash h: the low 32 hash bits scaled to the table size
// (multiply-shift, so the table need not be a power of two); probing walks
// forward and wraps.
__device__ __forceinline__ uint64_t slot_of(const Store& s, uint64_t h) {
    return (uint64_t)__umulhi((uint32_t)h, (uint32_t)s.tsize) | 0ull;
}
__device__ __forceinline__ uint64_t slot_next(const Store& s, uint64_t pos) {
    return pos + 1 == s.tsize ? 0 : pos + 1;
}

// Outcome of probing one candidate.
enum : uint32_t { P_SKIP = 0, P_DUP = 1, P_DEFER = 2, P_WON = 3, P_FULL = 4 };

// Probes candidate e (hash h) from `pos`, whose slot value the caller has
// already loaded (cur0, so that several first probes can be in flight), until
// an equal stored row is found (DUP), a matching slot of the running launch is
// met (DEFER; pos = that slot), or an empty slot is reserved (WON; pos = that
// slot).  FULL: no free slot in the whole table, or the store has already
// overflowed (full_store: the table is not probed at all and the caller only
// checks the candidate against the spec).  An overflowed level is never
// stored, so all it still decides is whether some candidate of the level meets
// the spec; a duplicate of a row of a cheaper level cannot (that level would
// have ended the search), and one of a row of this level has the same answer
// as that row, so skipping the duplicate test changes no outcome.  Rows with
// index >= snap were allocated by the running launch and are not read.
template <class Emit>
__device__ uint32_t probe_reserve(const Store& s, uint64_t h, uint64_t& pos, uint64_t cur0,
                                  uint64_t snap, bool full_store, const Emit& e) {
    if (full_store) return P_FULL;
    const uint32_t tag = tag_of(h);
    const uint64_t hi = (uint64_t)tag << 32;
    uint64_t cur = cur0;
    for (uint64_t steps = 0;; ++steps) {
        if (steps > s.tsize) return P_FULL;
        if (steps) cur = slot_load(&s.table[pos]);
        if (cur == kEmpty) {
            const uint64_t old = slot_cas(&s.table[pos], kEmpty, hi | kPending);
            if (old == kEmpty) return P_WON;
            cur = old;
        }
        const uint32_t cidx = (uint32_t)cur;
        if ((uint32_t)(cur >> 32) == tag) {
            if (cidx == kPending || cidx >= snap) return P_DEFER;
            if (emit_equal_row(s, cidx, e)) return P_DUP;
        }
        pos = slot_next(s, pos);
    }
}

// Writes a candidate whose slot `pos` it reserved into row r (or, past the
// row capacity, only checks it), publishes the slot and runs the spec check.
template <class Emit>
__device__ __forceinline__ void write_row(const Store& s, const Masks& m, uint32_t op, uint32_t L,
                                          uint32_t R, uint64_t h, uint64_t pos, uint64_t r,
                                          const Emit& e) {
    if (r >= s.cap) {  // the slot stays reserved; the level will not be stored
        atomicExch(&s.ctr[C_OVERFLOW], 1ull);
        emit_check_only(s, m, op, L, R, e);
        return;
    }
    uint4* M = reinterpret_cast<uint4*>(s.rows + r * s.Wp);
    uint32_t acc = 0;
    e([&](uint32_t w, uint4 v) {
        M[w >> 2] = v;
        acc |= check_vec(m, w, v);
        return true;
    });
    s.meta[r] = make_uint4(op | (tag_of(h) << 3), L, R, (uint32_t)h);
    slot_store(&s.table[pos], ((uint64_t)tag_of(h) << 32) | (uint32_t)r);
    if (acc == 0) report_found(s, op, L, R);
}

__device__ __forceinline__ void write_defer(const Store& s, unsigned long long d, uint32_t op,
                                            uint32_t L, uint32_t R, uint64_t pos) {
    if (d >= s.def0_cap) {
        atomicExch(&s.ctr[C_DEF_OVF], 1ull);
        return;
    }
    s.def0[d] = make_uint4(op | ((uint32_t)(pos >> 32) << 4), L, R, (uint32_t)pos);
}

// One candidate end to end, operands from the row store (atoms and re-inserted
// records), with per-wave counter aggregation.
template <class Emit>
__device__ void insert_emit(const Store& s, const Masks& m, uint32_t op, uint32_t L, uint32_t R,
                            uint64_t h, uint64_t pos, uint64_t cur0, uint64_t snap, const Emit& e) {
    const bool full = store_full(s);
    const uint32_t o = probe_reserve(s, h, pos, cur0, snap, full, e);
    if (o == P_WON) {
        write_row(s, m, op, L, R, h, pos, wave_alloc(&s.ctr[C_ROWS]), e);
    } else if (o == P_DEFER) {
        write_defer(s, wave_alloc(&s.ctr[C_DEF0]), op, L, R, pos);
    } else if (o == P_FULL) {
        if (!full) atomicExch(&s.ctr[C_OVERFLOW], 1ull);
        emit_check_only(s, m, op, L, R, e);
    }
}

__device__ __forceinline__ Masks global_masks(const Store& s) {
    return Masks{reinterpret_cast<const uint4*>(s.S), reinterpret_cast<const uint4*>(s.P0)};
}

__device__ __forceinline__ void check_only(const Store& s, uint32_t op, uint32_t L, uint32_t R) {
    emit_check_only(s, global_masks(s), op, L, R, GlobalEmit{s, op, L, R});
}

__device__ __forceinline__ void process(const Store& s, uint32_t op, uint32_t L, uint32_t R,
                                        uint64_t snap) {
    const GlobalEmit e{s, op, L, R};
    const uint64_t h = emit_hash(s, e);
    const uint64_t pos = slot_of(s, h);
    insert_emit(s, global_masks(s), op, L, R, h, pos, slot_load(&s.table[pos]), snap, e);
}

__device__ __forceinline__ bool cm_equal_row(const Store& s, uint32_t op, uint32_t L, uint32_t R,
                                             uint64_t row) {
    return emit_equal_row(s, row, GlobalEmit{s, op, L, R});
}

__device__ __forceinline__ uint64_t cm_hash(const Store& s, uint32_t op, uint32_t L, uint32_t R) {
    return emit_hash(s, GlobalEmit{s, op, L, R});
}

// ------------------------------------------------------------ LDS emitters --
// Operators selected at run time (the selector is wave-uniform in the
// generation kernels, so the switch costs scalar branches only).
__device__ __forceinline__ uint4 unary_any(uint32_t op, uint4 a, uint4 v, uint32_t& st) {
    switch (op) {
    case OP_NOT: return op_vec<OP_NOT>(a, a, v, st);
    case OP_X: return op_vec<OP_X>(a, a, v, st);
    case OP_F: return op_vec<OP_F>(a, a, v, st);
    default: return op_vec<OP_G>(a, a, v, st);
    }
}
__device__ __forceinline__ uint4 binary_any(uint32_t op, uint4 a, uint4 b, uint32_t& st) {
    switch (op) {
    case OP_AND: return op_vec<OP_AND>(a, b, b, st);
    case OP_OR: return op_vec<OP_OR>(a, b, b, st);
    default: return op_vec<OP_U>(a, b, b, st);
    }
}

// Unary operator `op` over a row in LDS (v), with V in LDS.
struct LdsUnaryEmit {
    static constexpr bool kChunked = true;
    const uint4* v;
    const uint4* V;
    uint32_t nq, op;
    // chunk q, given the carry state st of chunks < q (updated)
    __device__ __forceinline__ uint4 at(uint32_t q, uint32_t& st) const { return unary_any(op, v[q], V[q], st); }
    template <class Fn>
    __device__ __forceinline__ void operator()(Fn&& fn) const {
        uint32_t st = 0;
        for (uint32_t q = 0; q < nq; ++q) {
            if (!fn(4u * q, unary_any(op, v[q], V[q], st))) return;
        }
    }
};

// Binary operator `op` with left operand l and right operand r (LDS rows).
struct LdsPairEmit {
    static constexpr bool kChunked = true;
    const uint4* l;
    const uint4* r;
    uint32_t nq, op;
    __device__ __forceinline__ uint4 at(uint32_t q, uint32_t& st) const { return binary_any(op, l[q], r[q], st); }
    template <class Fn>
    __device__ __forceinline__ void operator()(Fn&& fn) const {
        uint32_t st = 0;
        for (uint32_t q = 0; q < nq; ++q) {
            if (!fn(4u * q, binary_any(op, l[q], r[q], st))) return;
        }
    }
};

// ------------------------------------------------------------ tile mapping --
// Triangular pair grid with b-tiles R times as wide as a-tiles (R even): b-tile
// column k holds a-tiles [0, R(k+1)) and starts at tile (R/2)k(k+1).
template <uint32_t R>
__device__ __forceinline__ void tri_tile(uint64_t lt, uint64_t& ta, uint64_t& tb) {
    constexpr uint64_t H = R / 2;
    uint64_t k = (uint64_t)((sqrt(1.0 + (double)lt * (8.0 / R)) - 1.0) * 0.5);
    while (H * (k + 1) * (k + 2) <= lt) ++k;
    while (k > 0 && H * k * (k + 1) > lt) --k;
    tb = k;
    ta = lt - H * k * (k + 1);
}

// ------------------------------------------------------------------ kernels --
// Wave-wide allocation of rows and deferral records: every active lane
// brings how many rows (nrow) and records (ndef) it needs (each <= 4); one
// atomic per counter and wave hands out consecutive indices.  No barrier, so
// waves never wait for each other's probe chains.
__device__ __forceinline__ void wave_alloc2(const Store& s, uint32_t nrow, uint32_t ndef,
                                            unsigned long long& rbase,
                                            unsigned long long& dbase) {
    const uint32_t lane = __lane_id();
    const uint32_t mine = nrow | (ndef << 16);
    uint32_t incl = mine;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t t = __shfl_up(incl, d, 64);
        if (lane >= (uint32_t)d) incl += t;
    }
    const uint32_t total = __shfl(incl, 63, 64);
    unsigned long long rb = 0, db = 0;
    if (lane == 0) {
        if (total & 0xFFFFu) rb = atomicAdd(&s.ctr[C_ROWS], (unsigned long long)(total & 0xFFFFu));
        if (total >> 16) db = atomicAdd(&s.ctr[C_DEF0], (unsigned long long)(total >> 16));
    }
    rb = __shfl(rb, 0, 64);
    db = __shfl(db, 0, 64);
    const uint32_t excl = incl - mine;
    rbase = rb + (excl & 0xFFFFu);
    dbase = db + (excl >> 16);
}

// Per-wave allocator used by the persistent group kernel: row indices and
// deferral records are taken from the global counters kAllocChunk at a time,
// so one same-address atomic serves ~kAllocChunk rows (same-address atomics
// serialise).  A request that does not fit the wave's current chunk takes
// its rest and a new chunk, so the only unused indices are the tails the
// waves hold when the launch ends.  Those are retired: rows get a dead
// derivation record (y = kDead) and are counted in C_DEAD (removed at the end
// of the level), records get the empty operator code.
struct WaveAlloc {
    unsigned long long rnext = 0, rend = 0, dnext = 0, dend = 0;
};

__device__ __forceinline__ void retire_rows(const Store& s, unsigned long long lo,
                                            unsigned long long hi) {
    const unsigned long long top = hi < s.cap ? hi : s.cap;
    if (lo >= top) return;
    for (unsigned long long r = lo + __lane_id(); r < top; r += 64) s.meta[r] = make_uint4(0, kDead, 0, 0);
    if (__lane_id() == 0) atomicAdd(&s.ctr[C_DEAD], top - lo);
}

__device__ __forceinline__ void retire_records(const Store& s, unsigned long long lo,
                                               unsigned long long hi) {
    const unsigned long long top = hi < s.def0_cap ? hi : s.def0_cap;
    for (unsigned long long r = lo + __lane_id(); r < top; r += 64) s.def0[r] = make_uint4(kNoRecord, 0, 0, 0);
}

// Wave-uniform: `total` indices are needed, this lane's first is `excl`
// (each lane takes at most one).  Returns the lane's index.
__device__ __forceinline__ unsigned long long chunk_take(unsigned long long* ctr, unsigned long long& next,
                                                         unsigned long long& end, uint32_t total,
                                                         uint32_t excl, uint32_t chunk) {
    if (total == 0) return 0;
    const unsigned long long rem = end - next;
    if (total <= rem) {
        const unsigned long long mine = next + excl;
        next += total;
        return mine;
    }
    const uint32_t need = total - (uint32_t)rem;
    const uint32_t ch = need > chunk ? need : chunk;
    unsigned long long b = 0;
    if (__lane_id() == 0) b = atomicAdd(ctr, (unsigned long long)ch);
    b = __shfl(b, 0, 64);
    const unsigned long long mine = excl < rem ? next + excl : b + (excl - rem);
    next = b + need;
    end = b + ch;
    return mine;
}

// Wave-wide: adds every lane's n to counter `which` with one atomic.
__device__ __forceinline__ void wave_count(const Store& s, uint32_t which, uint32_t n) {
    for (int off = 32; off > 0; off >>= 1) n += __shfl_down(n, off, 64);
    if (__lane_id() == 0 && n) atomicAdd(&s.ctr[which], (unsigned long long)n);
}

// Wave-wide (every lane calls it): lane needs nrow rows and ndef records
// (each 0 or 1); returns its indices.
__device__ __forceinline__ void wave_take(const Store& s, WaveAlloc& wa, uint32_t nrow,
                                          uint32_t ndef, unsigned long long& rbase,
                                          unsigned long long& dbase, uint32_t chunk = kAllocChunk) {
    const uint32_t lane = __lane_id();
    const uint32_t mine = nrow | (ndef << 16);
    uint32_t incl = mine;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t t = __shfl_up(incl, d, 64);
        if (lane >= (uint32_t)d) incl += t;
    }
    const uint32_t total = __shfl(incl, 63, 64);
    const uint32_t excl = incl - mine;
    rbase = chunk_take(&s.ctr[C_ROWS], wa.rnext, wa.rend, total & 0xFFFFu, excl & 0xFFFFu, chunk);
    dbase = chunk_take(&s.ctr[C_DEF0], wa.dnext, wa.dend, total >> 16, excl >> 16, chunk);
}



// Per-candidate state of one iteration.
struct Cand {
    uint64_t h, pos, cur;
    uint32_t out;
};

// Hash pass of one candidate: records the hash and issues the first probe
// (once the store has overflowed: neither, the candidate is only checked),
// unless the candidate is disabled or its CM equals one of its operands
// (A, or B if given) -- a stored, cheaper CM, so a sure duplicate.  P_WON
// here only marks "still to probe".
template <class Emit>
__device__ __forceinline__ void cand_begin(const Store& s, Cand& c, bool enabled, bool check_eq,
                                           bool full_store, const uint4* A, const uint4* B, const Emit& e) {
    c.out = P_SKIP;
    if (!enabled) return;
    if (full_store) {  // only checked: no hash, no duplicate test
        c.out = P_FULL;
        return;
    }
    Hash hs;
    uint32_t ea = 0, eb = 0;
    e([&](uint32_t w, uint4 r) {
        hs.add4(r);
        ea |= diff4(r, A[w >> 2]);
        eb |= diff4(r, B[w >> 2]);
        return true;
    });
    if (check_eq && (ea == 0 || eb == 0)) return;
    c.h = hs.fin() & s.hmask;
    c.pos = slot_of(s, c.h);
    c.cur = slot_load(&s.table[c.pos]);
    c.out = P_WON;
}

template <class Emit>
__device__ __forceinline__ void cand_probe(const Store& s, Cand& c, uint64_t snap, bool full_store,
                                           const Emit& e) {
    if (c.out == P_WON) c.out = probe_reserve(s, c.h, c.pos, c.cur, snap, full_store, e);
}

template <class Emit>
__device__ __forceinline__ void cand_finish(const Store& s, const Masks& m, const Cand& c,
                                            uint32_t op, uint32_t L, uint32_t R,
                                            unsigned long long& rb, unsigned long long& db,
                                            bool full_store, const Emit& e) {
    if (c.out == P_WON) {
        write_row(s, m, op, L, R, c.h, c.pos, rb++, e);
    } else if (c.out == P_DEFER) {
        write_defer(s, db++, op, L, R, c.pos);
    } else if (c.out == P_FULL) {
        if (!full_store) atomicExch(&s.ctr[C_OVERFLOW], 1ull);
        emit_check_only(s, m, op, L, R, e);
    }
}

__host__ __device__ __forceinline__ uint32_t lds_stride(uint32_t nq) { return nq | 1u; }

// Generation with operands staged in LDS, for rows that fit (see
// lds_bytes()).  Pair tiles: the workgroup stages its 16 left operands (read
// by whole waves at one address: broadcast) and each lane its right operand
// (rows padded to an odd number of 16-byte vectors, so the 8 lanes served per
// LDS cycle hit disjoint banks); the masks go to LDS too.  For every pair,
// each enabled operator (a and b, a or b, a U b, b U a) is streamed once to
// hash it and to test it against both operands, the first probes of all
// operators are issued before any is waited on, and rows and deferral records
// are allocated with one atomic per counter, wave and pair.  Unary tiles do
// the same for not, X, F, G over the lane's operand.  LANES (256, or 128 for
// rows whose 256-lane tile does not fit the LDS) is both the workgroup size
// and the width of a pair tile.
template <int BATCH, int LANES>
__device__ __forceinline__ void lds_tile(const Store& s, const Seg& g, uint64_t lt, uint4* dyn) {
    const uint32_t NQ = s.Wp / 4, SB = lds_stride(NQ);
    uint4* sh_b = dyn;
    uint4* sh_a = sh_b + LANES * SB;
    uint4* sh_v = sh_a + kTileA * NQ;
    uint4* sh_s = sh_v + NQ;
    uint4* sh_p = sh_s + NQ;
    const uint64_t snap = s.ctr[C_SNAP];
    const bool full_store = store_full(s);
    const uint32_t tid = threadIdx.x;
    const uint4* rows4 = reinterpret_cast<const uint4*>(s.rows);
    for (uint32_t q = tid; q < NQ; q += LANES) {
        sh_v[q] = reinterpret_cast<const uint4*>(s.V)[q];
        sh_s[q] = reinterpret_cast<const uint4*>(s.S)[q];
        sh_p[q] = reinterpret_cast<const uint4*>(s.P0)[q];
    }
    const Masks m{sh_s, sh_p};
    uint4* mine = sh_b + tid * SB;
    uint32_t count = 0;

    if (g.kind == SEG_ATOM) {
        __syncthreads();
        if (tid < g.nb) {
            process(s, OP_ATOM, tid, 0, snap);
            ++count;
        }
    } else if (g.kind == SEG_UNARY) {
        const uint64_t vl = lt * LANES + tid;
        const bool ok = vl < g.nb;
        const uint32_t vi = (uint32_t)(g.b0 + (ok ? vl : 0));
        for (uint32_t q = 0; q < NQ; ++q) mine[q] = ok ? rows4[(uint64_t)vi * NQ + q] : make_uint4(0, 0, 0, 0);
        __syncthreads();
        const uint32_t vop = ok ? (s.meta[vi].x & 7u) : OP_ATOM;
        // not not a, F F a, G G a are cheaper formulas' CMs: skipped.  A result
        // equal to a (possible for X, F, G) is a sure duplicate.
        constexpr uint32_t ops[4] = {OP_NOT, OP_X, OP_F, OP_G};
        constexpr uint32_t bits[4] = {M_NOT, M_X, M_F, M_G};
#pragma unroll
        for (int j0 = 0; j0 < 4; j0 += BATCH) {
            Cand c[BATCH];
#pragma unroll
            for (int jj = 0; jj < BATCH; ++jj) {
                const int j = j0 + jj;
                const bool en = ok && (g.opmask & bits[j]) && (j == 1 || vop != ops[j]);
                cand_begin(s, c[jj], en, j != 0, full_store, mine, mine, LdsUnaryEmit{mine, sh_v, NQ, ops[j]});
                count += en;
            }
            uint32_t nrow = 0, ndef = 0;
#pragma unroll
            for (int jj = 0; jj < BATCH; ++jj) {
                cand_probe(s, c[jj], snap, full_store, LdsUnaryEmit{mine, sh_v, NQ, ops[j0 + jj]});
                nrow += c[jj].out == P_WON;
                ndef += c[jj].out == P_DEFER;
            }
            unsigned long long rb, db;
            wave_alloc2(s, nrow, ndef, rb, db);
#pragma unroll
            for (int jj = 0; jj < BATCH; ++jj)
                cand_finish(s, m, c[jj], ops[j0 + jj], vi, 0, rb, db, full_store,
                            LdsUnaryEmit{mine, sh_v, NQ, ops[j0 + jj]});
        }
    } else {
        uint64_t ta, tb;
        if (g.tri) {
            tri_tile<LANES / kTileA>(lt, ta, tb);
        } else {
            const uint64_t tiles_b = (g.nb + LANES - 1) / LANES;
            ta = lt / tiles_b;
            tb = lt % tiles_b;
        }
        for (uint32_t idx = tid; idx < kTileA * NQ; idx += LANES) {
            const uint64_t al = ta * kTileA + idx / NQ;
            sh_a[idx] = al < g.na ? rows4[(g.a0 + al) * NQ + idx % NQ] : make_uint4(0, 0, 0, 0);
        }
        const uint64_t bl = tb * LANES + tid;
        const bool valid = bl < g.nb;
        const uint32_t bi = (uint32_t)(g.b0 + (valid ? bl : 0));
        for (uint32_t q = 0; q < NQ; ++q) mine[q] = valid ? rows4[(uint64_t)bi * NQ + q] : make_uint4(0, 0, 0, 0);
        __syncthreads();
        // candidate j: a&b, a|b, a U b, b U a
        constexpr uint32_t ops[4] = {OP_AND, OP_OR, OP_U, OP_U};
        constexpr uint32_t bits[4] = {M_AND, M_OR, M_UAB, M_UBA};
        for (uint32_t i = 0; i < kTileA; ++i) {
            const uint64_t al = ta * kTileA + i;
            if (al >= g.na) break;  // uniform across the block
            const bool ok = valid && !(g.tri && al >= bl);  // pairs a < b only
            const uint32_t ai = (uint32_t)(g.a0 + al);
            const uint4* arow = sh_a + i * NQ;
#pragma unroll
            for (int j0 = 0; j0 < 4; j0 += BATCH) {
                Cand c[BATCH];
#pragma unroll
                for (int jj = 0; jj < BATCH; ++jj) {
                    const int j = j0 + jj;
                    const bool en = ok && (g.opmask & bits[j]);
                    const LdsPairEmit e{j == 3 ? mine : arow, j == 3 ? arow : mine, NQ, ops[j]};
                    cand_begin(s, c[jj], en, true, full_store, arow, mine, e);
                    count += en;
                }
                uint32_t nrow = 0, ndef = 0;
#pragma unroll
                for (int jj = 0; jj < BATCH; ++jj) {
                    const int j = j0 + jj;
                    cand_probe(s, c[jj], snap, full_store,
                               LdsPairEmit{j == 3 ? mine : arow, j == 3 ? arow : mine, NQ, ops[j]});
                    nrow += c[jj].out == P_WON;
                    ndef += c[jj].out == P_DEFER;
                }
                unsigned long long rb, db;
                wave_alloc2(s, nrow, ndef, rb, db);
#pragma unroll
                for (int jj = 0; jj < BATCH; ++jj) {
                    const int j = j0 + jj;
                    cand_finish(s, m, c[jj], ops[j], j == 3 ? bi : ai, j == 3 ? ai : bi, rb, db, full_store,
                                LdsPairEmit{j == 3 ? mine : arow, j == 3 ? arow : mine, NQ, ops[j]});
                }
            }
        }
    }
    unsigned long long cc = count;
    for (int off = 32; off > 0; off >>= 1) cc += __shfl_down(cc, off);
    if (__lane_id() == 0 && cc) atomicAdd(&s.ctr[C_CAND], cc);
}

template <int BATCH, int LANES>
__global__ __launch_bounds__(LANES) void k_generate_lds(Store s, SegTable t) {
    extern __shared__ uint4 dyn[];
    const uint64_t tile = t.tile_begin + blockIdx.x;
    if (tile >= t.tile_end) return;
    uint32_t si = 0;
    while (si + 1 < t.n && t.first[si + 1] <= tile) ++si;
    lds_tile<BATCH, LANES>(s, t.seg[si], tile - t.first[si], dyn);
}

// ------------------------------------------------ one lane group per candidate --
// Rows of 2..64 chunks are handled by groups of G lanes (G = the next power of
// two >= chunks, at least 4): lane k of a group holds chunk k of the operands
// and of the candidate.  Carries of the multi-word adds (F, G, U) cross chunk
// boundaries by carry-lookahead over ballots; the hash, the operand-equality
// test and the spec check are combined across the group; lanes 0..3 own the
// table work of the (up to) four candidates of the group's work item, and the
// whole group verifies and writes rows, so every row access is one coalesced
// 16*NQ-byte transfer.

constexpr uint32_t kGA = 32;  // left operands per pair tile
constexpr uint32_t kGB = 32;  // right operands per pair tile (kGA == kGB: square triangles)
constexpr uint32_t kGU = 64;  // operands per unary tile

// 128-bit add of two chunks with carry-in; *cout receives the carry out.
__device__ __forceinline__ uint4 add128(uint4 x, uint4 y, uint32_t cin, uint32_t& cout) {
    uint32_t c = cin;
    uint4 r;
    r.x = addc(x.x, y.x, c);
    r.y = addc(x.y, y.y, c);
    r.z = addc(x.z, y.z, c);
    r.w = addc(x.w, y.w, c);
    cout = c;
    return r;
}

template <int G>
__device__ __forceinline__ uint64_t group_bits(uint64_t wave_mask, uint32_t base) {
    if constexpr (G == 64) return wave_mask;
    else return (wave_mask >> base) & ((1ull << G) - 1);
}

// True iff `flag` is clear on every lane of the caller's group (wave-wide
// ballot: every lane of the wave must call it).
template <int G>
__device__ __forceinline__ bool group_none(bool flag, uint32_t base) {
    return group_bits<G>(__ballot(flag), base) == 0;
}

// Full multi-chunk sum X + Y for the caller's chunk k of a group: the carry
// into chunk k is 1 iff a lower chunk generates a carry and every chunk in
// between propagates it.  With generate bits g and propagate bits p (one per
// chunk), the carries into all chunks are ((g|p) + g) ^ (g|p) ^ g.
template <int G>
__device__ __forceinline__ uint4 group_add(uint4 x, uint4 y, uint32_t base, uint32_t k) {
    uint32_t co = 0;
    const uint4 s0 = add128(x, y, 0, co);
    const bool gen = co != 0;
    const bool prop = !gen && (s0.x & s0.y & s0.z & s0.w) == 0xFFFFFFFFu;
    const uint64_t g = group_bits<G>(__ballot(gen), base);
    const uint64_t p = group_bits<G>(__ballot(prop), base);
    const uint64_t a = g | p;
    const uint32_t cin = (uint32_t)((((a + g) ^ a ^ g) >> k) & 1u);
    uint32_t dummy;
    return add128(x, y, cin, dummy);
}

// XOR of a 64-bit value over the caller's group.
template <int G>
__device__ __forceinline__ uint64_t group_xor(uint64_t v) {
#pragma unroll
    for (int m = 1; m < G; m <<= 1) {
        const uint32_t lo = __shfl_xor((uint32_t)v, m, 64);
        const uint32_t hi = __shfl_xor((uint32_t)(v >> 32), m, 64);
        v ^= ((uint64_t)hi << 32) | lo;
    }
    return v;
}

__device__ __forceinline__ uint4 select4(int j, uint4 r0, uint4 r1, uint4 r2, uint4 r3) {
    return j == 0 ? r0 : j == 1 ? r1 : j == 2 ? r2 : r3;
}

enum : uint32_t { S_DONE = 0, S_PROBE = 1, S_DUP = 2, S_DEFER = 3, S_WON = 4, S_FULL = 5 };

// Table work of the four candidates of one work item.  Owner lane j (k == j)
// holds candidate j's state; results r0..r3 are this lane's chunks of the
// four candidates.  Every lane of the wave must call it (ballots, shuffles).
template <int G>
__device__ __forceinline__ void group_insert(const Store& s, WaveAlloc& wa, uint32_t NQ,
                                             uint32_t base, uint32_t k,
                                             uint64_t snap, bool full_store, bool active,
                                             uint64_t h, uint32_t op, uint32_t L, uint32_t R,
                                             bool sep, uint4 r0, uint4 r1, uint4 r2, uint4 r3) {
    const uint4* rows4 = reinterpret_cast<const uint4*>(s.rows);
    const uint32_t tag = tag_of(h);
    uint32_t st = active ? (full_store ? S_FULL : S_PROBE) : S_DONE;
    uint64_t pos = 0, cur = 0, steps = 0;
    if (st == S_PROBE) {
        pos = slot_of(s, h);
        cur = slot_load(&s.table[pos]);
    }
    while (__ballot(st == S_PROBE) != 0) {
        bool need_v = false;
        uint32_t vrow = 0;
        if (st == S_PROBE) {
            if (steps++ >= s.tsize) st = S_FULL;
            if (st == S_PROBE && cur == kEmpty) {
                const uint64_t old = slot_cas(&s.table[pos], kEmpty, ((uint64_t)tag << 32) | kPending);
                if (old == kEmpty) st = S_WON;
                else cur = old;
            }
            if (st == S_PROBE) {
                const uint32_t cidx = (uint32_t)cur;
                if ((uint32_t)(cur >> 32) == tag) {
                    if (cidx == kPending || cidx >= snap) st = S_DEFER;
                    else {
                        need_v = true;
                        vrow = cidx;
                    }
                } else {
                    pos = slot_next(s, pos);
                    cur = slot_load(&s.table[pos]);
                }
            }
        }
        // verify the owners' rows with the whole group (coalesced reads)
        const uint64_t nvm = group_bits<G>(__ballot(need_v), base);
        uint4 m[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t vr = __shfl(vrow, (int)(base + j), 64);
            m[j] = load_if(((nvm >> j) & 1u) && k < NQ, &rows4[(uint64_t)vr * NQ + k]);
        }
        bool eq_mine = false;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const bool differ = ((nvm >> j) & 1u) && k < NQ && diff4(m[j], select4(j, r0, r1, r2, r3)) != 0;
            const bool eq = group_none<G>(differ, base);
            if (k == (uint32_t)j) eq_mine = eq;
        }
        if (need_v) {
            if (eq_mine) st = S_DUP;
            else {
                pos = slot_next(s, pos);
                cur = slot_load(&s.table[pos]);
            }
        }
    }
    unsigned long long rb, db;
    wave_take(s, wa, st == S_WON ? 1u : 0u, st == S_DEFER ? 1u : 0u, rb, db);
    const uint64_t wonm = group_bits<G>(__ballot(st == S_WON), base);
    // past the capacity the broadcast index is 0xFFFFFFFF (>= cap): nothing is written
    const uint32_t myrow = st == S_WON && rb < s.cap ? (uint32_t)rb : 0xFFFFFFFFu;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const uint32_t rj = __shfl(myrow, (int)(base + j), 64);
        if (((wonm >> j) & 1u) && rj < s.cap && k < NQ)
            reinterpret_cast<uint4*>(s.rows)[(uint64_t)rj * NQ + k] = select4(j, r0, r1, r2, r3);
    }
    if (st == S_WON) {
        if (rb >= s.cap) {  // the slot stays reserved; the level will not be stored
            atomicExch(&s.ctr[C_OVERFLOW], 1ull);
        } else {
            s.meta[rb] = make_uint4(op | (tag << 3), L, R, (uint32_t)h);
            slot_store(&s.table[pos], ((uint64_t)tag << 32) | (uint32_t)rb);
        }
        if (sep) report_found(s, op, L, R);
    } else if (st == S_DEFER) {
        write_defer(s, db, op, L, R, pos);
    } else if (st == S_FULL) {
        if (!full_store) atomicExch(&s.ctr[C_OVERFLOW], 1ull);
        if (sep) report_found(s, op, L, R);
    }
}

template <int G>
__global__ __launch_bounds__(kLanes) void k_generate_grp(Store s, SegTable t) {
    constexpr uint32_t NG = kLanes / G;  // groups per block
    extern __shared__ uint4 dyn[];
    __shared__ unsigned long long sh_tile;
    const uint32_t NQ = s.Wp / 4;
    uint4* sh_a = dyn;                  // kGA rows (pair tiles)
    uint4* sh_b = sh_a + kGA * NQ;      // kGB rows (pair tiles) or kGU rows (unary tiles)
    uint4* sh_v = sh_b + kGU * NQ;
    uint4* sh_s = sh_v + NQ;
    uint4* sh_p = sh_s + NQ;
    __shared__ uint32_t sh_full;
    const uint64_t snap = s.ctr[C_SNAP];
    bool full_store = false;  // refreshed for every tile
    const uint32_t tid = threadIdx.x;
    const uint32_t lane = __lane_id();
    const uint32_t k = lane % G, base = lane - k, grp = tid / G;
    const uint4* rows4 = reinterpret_cast<const uint4*>(s.rows);
    for (uint32_t q = tid; q < NQ; q += kLanes) {
        sh_v[q] = reinterpret_cast<const uint4*>(s.V)[q];
        sh_s[q] = reinterpret_cast<const uint4*>(s.S)[q];
        sh_p[q] = reinterpret_cast<const uint4*>(s.P0)[q];
    }
    WaveAlloc wa;
    uint32_t count = 0;
    // persistent: the block takes tiles from a cursor that persists across
    // launches, while the deferral list and the table can take every
    // candidate of the tiles that may still be in flight (one per block)
    for (;;) {
    if (tid == 0) {
        unsigned long long tl = ~0ull;
        const unsigned long long d = __hip_atomic_load(&s.ctr[C_DEF0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned long long r = __hip_atomic_load(&s.ctr[C_ROWS], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const bool full = store_full(s);
        const unsigned long long cur = __hip_atomic_load(&s.ctr[C_TILE], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (cur < t.tile_stop && d + t.def_margin <= s.def0_cap && (full || r + t.row_margin <= t.row_budget))
            tl = atomicAdd(&s.ctr[C_TILE], 1ull);
        sh_tile = tl;
        sh_full = full;
    }
    __syncthreads();
    const uint64_t tile = sh_tile;
    full_store = sh_full != 0;
    __syncthreads();
    if (tile >= t.tile_end) break;
    uint32_t si = 0;
    while (si + 1 < t.n && t.first[si + 1] <= tile) ++si;
    const Seg& g = t.seg[si];
    const uint64_t lt = tile - t.first[si];

    if (g.kind == SEG_ATOM) {
        __syncthreads();
        if (tid < g.nb) {
            process(s, OP_ATOM, tid, 0, snap);
            ++count;
        }
    } else if (g.kind == SEG_UNARY) {
        const uint64_t v0 = lt * kGU;
        for (uint32_t idx = tid; idx < kGU * NQ; idx += kLanes) {
            const uint64_t vl = v0 + idx / NQ;
            sh_b[idx] = load_if(vl < g.nb, &rows4[(g.b0 + vl) * NQ + idx % NQ]);
        }
        __syncthreads();
        const uint4 V = load_if(k < NQ, &sh_v[k]);
        const uint4 S = load_if(k < NQ, &sh_s[k]);
        const uint4 P = load_if(k < NQ, &sh_p[k]);
        for (uint32_t iv = grp; iv < kGU; iv += NG) {
            const uint64_t vl = v0 + iv;
            const bool valid = vl < g.nb;
            const uint32_t vi = (uint32_t)(g.b0 + (valid ? vl : 0));
            const uint4 a = load_if(valid && k < NQ, &sh_b[iv * NQ + k]);
            const uint32_t vop = valid ? (s.meta[vi].x & 7u) : OP_ATOM;
            // not not a, F F a, G G a are cheaper formulas' CMs: skipped
            const bool dn = valid && (g.opmask & M_NOT) && vop != OP_NOT;
            const bool dx = valid && (g.opmask & M_X);
            const bool df = valid && (g.opmask & M_F) && vop != OP_F;
            const bool dg = valid && (g.opmask & M_G) && vop != OP_G;
            // not
            const uint4 rn = make_uint4(~a.x & V.x, ~a.y & V.y, ~a.z & V.z, ~a.w & V.w);
            // X: the bit entering this chunk is the top bit of the chunk below
            uint32_t up = __shfl_up(a.w >> 31, 1, 64);
            if (k == 0) up = 0;
            const uint4 rx = make_uint4(((a.x << 1) | up) & V.x, ((a.y << 1) | (a.x >> 31)) & V.y,
                                        ((a.z << 1) | (a.y >> 31)) & V.z, ((a.w << 1) | (a.z >> 31)) & V.w);
            // F: a | (V & carries of a + V)
            const uint4 sf = group_add<G>(a, V, base, k);
            const uint4 rf = make_uint4(a.x | (V.x & (sf.x ^ a.x ^ V.x)), a.y | (V.y & (sf.y ^ a.y ^ V.y)),
                                        a.z | (V.z & (sf.z ^ a.z ^ V.z)), a.w | (V.w & (sf.w ^ a.w ^ V.w)));
            // G: V & ~F(V & ~a)
            const uint4 x = make_uint4(V.x & ~a.x, V.y & ~a.y, V.z & ~a.z, V.w & ~a.w);
            const uint4 sg = group_add<G>(x, V, base, k);
            const uint4 rg = make_uint4(V.x & ~(x.x | (V.x & (sg.x ^ x.x ^ V.x))),
                                        V.y & ~(x.y | (V.y & (sg.y ^ x.y ^ V.y))),
                                        V.z & ~(x.z | (V.z & (sg.z ^ x.z ^ V.z))),
                                        V.w & ~(x.w | (V.w & (sg.w ^ x.w ^ V.w))));
            const bool in = k < NQ;
            // once the store has overflowed, candidates are only checked (the
            // flag is uniform over the block: the group reductions stay whole)
            uint64_t hn = 0, hx = 0, hf = 0, hg = 0;
            bool ex = false, ef = false, eg = false;
            if (!full_store) {
                hn = hash_fin(group_xor<G>(in ? chunk_hash(k, rn) : 0));
                hx = hash_fin(group_xor<G>(in ? chunk_hash(k, rx) : 0));
                hf = hash_fin(group_xor<G>(in ? chunk_hash(k, rf) : 0));
                hg = hash_fin(group_xor<G>(in ? chunk_hash(k, rg) : 0));
                ex = group_none<G>(in && diff4(rx, a) != 0, base);
                ef = group_none<G>(in && diff4(rf, a) != 0, base);
                eg = group_none<G>(in && diff4(rg, a) != 0, base);
            }
            const bool sn = group_none<G>(in && ((rn.x ^ P.x) & S.x | (rn.y ^ P.y) & S.y | (rn.z ^ P.z) & S.z | (rn.w ^ P.w) & S.w) != 0, base);
            const bool sx = group_none<G>(in && ((rx.x ^ P.x) & S.x | (rx.y ^ P.y) & S.y | (rx.z ^ P.z) & S.z | (rx.w ^ P.w) & S.w) != 0, base);
            const bool sf2 = group_none<G>(in && ((rf.x ^ P.x) & S.x | (rf.y ^ P.y) & S.y | (rf.z ^ P.z) & S.z | (rf.w ^ P.w) & S.w) != 0, base);
            const bool sg2 = group_none<G>(in && ((rg.x ^ P.x) & S.x | (rg.y ^ P.y) & S.y | (rg.z ^ P.z) & S.z | (rg.w ^ P.w) & S.w) != 0, base);
            // owner lane j takes candidate j: not, X, F, G
            const uint32_t opj = k == 0 ? OP_NOT : k == 1 ? OP_X : k == 2 ? OP_F : OP_G;
            const bool act = k == 0 ? dn : k == 1 ? (dx && !ex) : k == 2 ? (df && !ef) : k == 3 ? (dg && !eg) : false;
            const uint64_t hj = (k == 0 ? hn : k == 1 ? hx : k == 2 ? hf : hg) & s.hmask;
            const bool sepj = k == 0 ? sn : k == 1 ? sx : k == 2 ? sf2 : sg2;
            group_insert<G>(s, wa, NQ, base, k, snap, full_store, act && k < 4, hj, opj, vi, 0, sepj,
                            rn, rx, rf, rg);
            if (k == 0) count += (uint32_t)dn + dx + df + dg;
        }
    } else {
        uint64_t ta, tb;
        if (g.tri) {  // square tiles, upper triangle ta <= tb, column by column
            tb = (uint64_t)((sqrt(8.0 * (double)lt + 1.0) - 1.0) * 0.5);
            while ((tb + 1) * (tb + 2) / 2 <= lt) ++tb;
            while (tb > 0 && tb * (tb + 1) / 2 > lt) --tb;
            ta = lt - tb * (tb + 1) / 2;
        } else {
            const uint64_t tiles_b = (g.nb + kGB - 1) / kGB;
            ta = lt / tiles_b;
            tb = lt % tiles_b;
        }
        for (uint32_t idx = tid; idx < (kGA + kGB) * NQ; idx += kLanes) {
            if (idx < kGA * NQ) {
                const uint64_t al = ta * kGA + idx / NQ;
                sh_a[idx] = load_if(al < g.na, &rows4[(g.a0 + al) * NQ + idx % NQ]);
            } else {
                const uint32_t j = idx - kGA * NQ;
                const uint64_t bl = tb * kGB + j / NQ;
                sh_b[j] = load_if(bl < g.nb, &rows4[(g.b0 + bl) * NQ + j % NQ]);
            }
        }
        __syncthreads();
        const uint4 S = load_if(k < NQ, &sh_s[k]);
        const uint4 P = load_if(k < NQ, &sh_p[k]);
        const bool mA = (g.opmask & M_AND) != 0, mO = (g.opmask & M_OR) != 0;  // uniform
        const bool mU = (g.opmask & M_UAB) != 0, mV = (g.opmask & M_UBA) != 0;
        for (uint32_t it = grp; it < kGA * kGB; it += NG) {
            const uint32_t ia = it / kGB, ib = it % kGB;
            const uint64_t al = ta * kGA + ia, bl = tb * kGB + ib;
            const bool valid = al < g.na && bl < g.nb && (!g.tri || al < bl);
            const uint32_t ai = (uint32_t)(g.a0 + (valid ? al : 0));
            const uint32_t bi = (uint32_t)(g.b0 + (valid ? bl : 0));
            const bool in = valid && k < NQ;
            const uint4 a = load_if(in, &sh_a[ia * NQ + k]);
            const uint4 b = load_if(in, &sh_b[ib * NQ + k]);
            const uint4 o = make_uint4(a.x | b.x, a.y | b.y, a.z | b.z, a.w | b.w);
            const uint4 rA = make_uint4(a.x & b.x, a.y & b.y, a.z & b.z, a.w & b.w);
            // a U b = b | (a & carries of b + (a|b)); b U a symmetric
            const uint4 s1 = group_add<G>(b, o, base, k);
            const uint4 rU = make_uint4(b.x | (a.x & (s1.x ^ b.x ^ o.x)), b.y | (a.y & (s1.y ^ b.y ^ o.y)),
                                        b.z | (a.z & (s1.z ^ b.z ^ o.z)), b.w | (a.w & (s1.w ^ b.w ^ o.w)));
            const uint4 s2 = group_add<G>(a, o, base, k);
            const uint4 rV = make_uint4(a.x | (b.x & (s2.x ^ a.x ^ o.x)), a.y | (b.y & (s2.y ^ a.y ^ o.y)),
                                        a.z | (b.z & (s2.z ^ a.z ^ o.z)), a.w | (b.w & (s2.w ^ a.w ^ o.w)));
            uint64_t hA = 0, hO = 0, hU = 0, hV = 0;
            bool eA = false, eO = false, eU = false, eV = false;
            if (!full_store) {  // after an overflow candidates are only checked
                hA = hash_fin(group_xor<G>(in ? chunk_hash(k, rA) : 0));
                hO = hash_fin(group_xor<G>(in ? chunk_hash(k, o) : 0));
                hU = hash_fin(group_xor<G>(in ? chunk_hash(k, rU) : 0));
                hV = hash_fin(group_xor<G>(in ? chunk_hash(k, rV) : 0));
                // a result equal to an operand is a stored, cheaper CM (the
                // second test runs on whole groups: the first is group-uniform)
                eA = group_none<G>(in && diff4(rA, a) != 0, base) || group_none<G>(in && diff4(rA, b) != 0, base);
                eO = group_none<G>(in && diff4(o, a) != 0, base) || group_none<G>(in && diff4(o, b) != 0, base);
                eU = group_none<G>(in && diff4(rU, a) != 0, base) || group_none<G>(in && diff4(rU, b) != 0, base);
                eV = group_none<G>(in && diff4(rV, a) != 0, base) || group_none<G>(in && diff4(rV, b) != 0, base);
            }
            const bool sA = group_none<G>(in && ((rA.x ^ P.x) & S.x | (rA.y ^ P.y) & S.y | (rA.z ^ P.z) & S.z | (rA.w ^ P.w) & S.w) != 0, base);
            const bool sO = group_none<G>(in && ((o.x ^ P.x) & S.x | (o.y ^ P.y) & S.y | (o.z ^ P.z) & S.z | (o.w ^ P.w) & S.w) != 0, base);
            const bool sU = group_none<G>(in && ((rU.x ^ P.x) & S.x | (rU.y ^ P.y) & S.y | (rU.z ^ P.z) & S.z | (rU.w ^ P.w) & S.w) != 0, base);
            const bool sV = group_none<G>(in && ((rV.x ^ P.x) & S.x | (rV.y ^ P.y) & S.y | (rV.z ^ P.z) & S.z | (rV.w ^ P.w) & S.w) != 0, base);
            // owner lane j takes candidate j: a&b, a|b, a U b, b U a
            const uint32_t opj = k == 0 ? OP_AND : k == 1 ? OP_OR : OP_U;
            const uint32_t Lj = k == 3 ? bi : ai, Rj = k == 3 ? ai : bi;
            const bool act = valid && (k == 0 ? (mA && !eA) : k == 1 ? (mO && !eO) : k == 2 ? (mU && !eU) :
                                       k == 3 ? (mV && !eV) : false);
            const uint64_t hj = (k == 0 ? hA : k == 1 ? hO : k == 2 ? hU : hV) & s.hmask;
            const bool sepj = k == 0 ? sA : k == 1 ? sO : k == 2 ? sU : sV;
            group_insert<G>(s, wa, NQ, base, k, snap, full_store, act, hj, opj, Lj, Rj, sepj, rA, o, rU, rV);
            if (k == 0 && valid) count += (uint32_t)mA + mO + mU + mV;
        }
    }
    __syncthreads();  // the next tile reuses the LDS tiles
    }
    retire_rows(s, wa.rnext, wa.rend);
    retire_records(s, wa.dnext, wa.dend);
    unsigned long long cc = count;
    for (int off = 32; off > 0; off >>= 1) cc += __shfl_down(cc, off);
    if (__lane_id() == 0 && cc) atomicAdd(&s.ctr[C_CAND], cc);
}

// ---------------------------------------------------- one wave per candidate --
// Rows of any width: a wavefront takes one work item (a pair and its four
// candidates, or an operand and its four unary results) and streams the rows
// in steps of 64 chunks (lane k holds chunk 64*step + k), with every load and
// store a coalesced 1 KB transfer.  Operands are read from global memory (a
// tile's operands stay L2-resident); candidates are recomputed in each pass
// (hash and tests, verification, write) instead of being held.  Carries of
// the multi-word adds cross lanes by ballot carry-lookahead and steps through
// the top lane.

// Pair tile of the wave kernel: Store::wtile left x wtile right operands
// (square: triangular segments use square tiles), unary tiles of 2 x wtile
// operands; the block's four waves share a tile and meet at a barrier
// between tiles.  The side is chosen per row width by the autotuner (8, 16
// or 32), else kWaveTileBuiltin.
constexpr uint32_t kWaveChunk = 8;  // rows / records a wave takes per atomic


// X + Y over a whole row, one step of 64 chunks: `carry` (wave-uniform) is
// the carry into lane 0 on entry and the carry out of lane 63 on return.
__device__ __forceinline__ uint4 wave_add(uint4 x, uint4 y, uint32_t& carry) {
    uint32_t co = 0;
    const uint4 s0 = add128(x, y, 0, co);
    const bool gen = co != 0;
    const bool prop = !gen && (s0.x & s0.y & s0.z & s0.w) == 0xFFFFFFFFu;
    const uint64_t g = __ballot(gen), p = __ballot(prop);
    const uint64_t a = g | p;
    // carries into the lanes: (a + g + carry) ^ a ^ g; out of lane 63: its overflow
    const uint64_t t = a + g;
    const uint64_t sum = t + carry;
    const uint32_t out = (t < a || sum < t) ? 1u : 0u;
    const uint32_t cin = (uint32_t)(((sum ^ a ^ g) >> __lane_id()) & 1u);
    carry = out;
    uint32_t dummy;
    return add128(x, y, cin, dummy);
}

// Top bit of the lower chunk for X: lane k takes lane k-1's, lane 0 the
// carried bit of the previous step; `carry` becomes lane 63's top bit.
__device__ __forceinline__ uint32_t wave_shift_in(uint4 v, uint32_t& carry) {
    const uint32_t top = v.w >> 31;
    uint32_t up = __shfl_up(top, 1, 64);
    if (__lane_id() == 0) up = carry;
    carry = __shfl(top, 63, 64);
    return up;
}

__device__ __forceinline__ uint4 x_chunk(uint4 a, uint32_t up, uint4 V) {
    return make_uint4(((a.x << 1) | up) & V.x, ((a.y << 1) | (a.x >> 31)) & V.y,
                      ((a.z << 1) | (a.y >> 31)) & V.z, ((a.w << 1) | (a.z >> 31)) & V.w);
}

__device__ __forceinline__ uint32_t check_chunk(uint4 r, uint4 P, uint4 S) {
    return ((r.x ^ P.x) & S.x) | ((r.y ^ P.y) & S.y) | ((r.z ^ P.z) & S.z) | ((r.w ^ P.w) & S.w);
}

// Streams the four results of a work item over the row.  Pair (unary ==
// false): a & b, a | b, a U b, b U a of rows A, B.  Unary: not, X, F, G of
// row A.  body(q, in, a, b, r0, r1, r2, r3) runs once per step (a, b: the
// operands' chunks; in: chunk q exists).
template <class Body>
__device__ __forceinline__ void wave_pass(const Store& s, bool unary, const uint4* A, const uint4* B,
                                          uint32_t nq, Body&& body) {
    const uint4* V4 = reinterpret_cast<const uint4*>(s.V);
    uint32_t c0 = 0, c1 = 0, c2 = 0;
    const uint32_t steps = (nq + 63) / 64;
    // the next step's operand chunks are loaded while this step computes
    const uint32_t lane = __lane_id();
    uint4 a_nx = load_if(lane < nq, &A[lane]);
    uint4 b_nx = load_if(lane < nq && !unary, &B[lane]);
    uint4 v_nx = load_if(lane < nq && unary, &V4[lane]);
    for (uint32_t st = 0; st < steps; ++st) {
        const uint32_t q = st * 64 + lane;
        const bool in = q < nq;
        const uint4 a = a_nx, b_cur = b_nx, v_cur = v_nx;
        const uint32_t qn = q + 64;
        const bool in_nx = st + 1 < steps && qn < nq;
        a_nx = load_if(in_nx, &A[qn]);
        b_nx = load_if(in_nx && !unary, &B[qn]);
        v_nx = load_if(in_nx && unary, &V4[qn]);
        if (unary) {
            const uint4 V = v_cur;
            const uint4 rn = make_uint4(~a.x & V.x, ~a.y & V.y, ~a.z & V.z, ~a.w & V.w);
            const uint4 rx = x_chunk(a, wave_shift_in(a, c0), V);
            const uint4 sf = wave_add(a, V, c1);
            const uint4 rf = make_uint4(a.x | (V.x & (sf.x ^ a.x ^ V.x)), a.y | (V.y & (sf.y ^ a.y ^ V.y)),
                                        a.z | (V.z & (sf.z ^ a.z ^ V.z)), a.w | (V.w & (sf.w ^ a.w ^ V.w)));
            const uint4 x = make_uint4(V.x & ~a.x, V.y & ~a.y, V.z & ~a.z, V.w & ~a.w);
            const uint4 sg = wave_add(x, V, c2);
            const uint4 rg = make_uint4(V.x & ~(x.x | (V.x & (sg.x ^ x.x ^ V.x))),
                                        V.y & ~(x.y | (V.y & (sg.y ^ x.y ^ V.y))),
                                        V.z & ~(x.z | (V.z & (sg.z ^ x.z ^ V.z))),
                                        V.w & ~(x.w | (V.w & (sg.w ^ x.w ^ V.w))));
            body(q, in, a, a, rn, rx, rf, rg);
        } else {
            const uint4 b = b_cur;
            const uint4 o = make_uint4(a.x | b.x, a.y | b.y, a.z | b.z, a.w | b.w);
            const uint4 rA = make_uint4(a.x & b.x, a.y & b.y, a.z & b.z, a.w & b.w);
            const uint4 s1 = wave_add(b, o, c1);
            const uint4 rU = make_uint4(b.x | (a.x & (s1.x ^ b.x ^ o.x)), b.y | (a.y & (s1.y ^ b.y ^ o.y)),
                                        b.z | (a.z & (s1.z ^ b.z ^ o.z)), b.w | (a.w & (s1.w ^ b.w ^ o.w)));
            const uint4 s2 = wave_add(a, o, c2);
            const uint4 rV = make_uint4(a.x | (b.x & (s2.x ^ a.x ^ o.x)), a.y | (b.y & (s2.y ^ a.y ^ o.y)),
                                        a.z | (b.z & (s2.z ^ a.z ^ o.z)), a.w | (b.w & (s2.w ^ a.w ^ o.w)));
            body(q, in, a, b, rA, o, rU, rV);
        }
    }
}

__device__ __forceinline__ uint64_t lane_pick4(uint32_t j, uint64_t v0, uint64_t v1, uint64_t v2, uint64_t v3) {
    return j == 0 ? v0 : j == 1 ? v1 : j == 2 ? v2 : v3;
}

// The same stream, specialised: UNARY fixed at compile time, and only the
// results selected by `need` (bit j: result j; wave-uniform, constant over
// the pass, so every carry chain runs on every step or on none) computed,
// the others left zero.  Side loads travel with the operands, one step
// ahead: with ROWS, the step's chunk of the stored row M[j] for every j in
// `need` (verification); with MASKS, the step's chunks of P0 and S (spec
// check).  body(q, in, a, b, r0, r1, r2, r3, m, P, S) runs once per step (b is
// a for unary items; m[j], P, S zero where not loaded).
// Side loads one step ahead (1) or in their own step (0).
#ifndef LTLF_SIDE_PREFETCH
#define LTLF_SIDE_PREFETCH 1
#endif
template <bool UNARY, bool ROWS, bool MASKS, class Body>
__device__ __forceinline__ void wave_pass_t(const Store& s, const uint4* A, const uint4* B, uint32_t nq,
                                            uint32_t need, const uint4* const (&M)[4], Body&& body) {
    const uint4* V4 = reinterpret_cast<const uint4*>(s.V);
    const uint4* P4 = reinterpret_cast<const uint4*>(s.P0);
    const uint4* S4 = reinterpret_cast<const uint4*>(s.S);
    const uint4 zero = make_uint4(0, 0, 0, 0);
    uint32_t c0 = 0, c1 = 0, c2 = 0;
    const uint32_t steps = (nq + 63) / 64;
    const uint32_t lane = __lane_id();
    uint4 a_nx, b_nx = zero, v_nx = zero, p_nx = zero, s_nx = zero;
    uint4 m_nx[4] = {zero, zero, zero, zero};
    auto side = [&](uint32_t qq, bool ok) {
        if constexpr (ROWS) {
#pragma unroll
            for (int j = 0; j < 4; ++j) m_nx[j] = load_if(ok && ((need >> j) & 1u), &M[j][qq]);
        }
        if constexpr (MASKS) {
            p_nx = load_if(ok, &P4[qq]);
            s_nx = load_if(ok, &S4[qq]);
        }
    };
    auto fetch = [&](uint32_t qq, bool ok) {
        a_nx = load_if(ok, &A[qq]);
        if constexpr (UNARY) v_nx = load_if(ok, &V4[qq]);
        else b_nx = load_if(ok, &B[qq]);
        if (LTLF_SIDE_PREFETCH) side(qq, ok);
    };
    fetch(lane, lane < nq);
    for (uint32_t st = 0; st < steps; ++st) {
        const uint32_t q = st * 64 + lane;
        const bool in = q < nq;
        if (!LTLF_SIDE_PREFETCH) side(q, in);
        const uint4 a = a_nx, b = b_nx, V = v_nx, P = p_nx, S = s_nx;
        const uint4 m[4] = {m_nx[0], m_nx[1], m_nx[2], m_nx[3]};
        const uint32_t qn = q + 64;
        fetch(qn, st + 1 < steps && qn < nq);
        uint4 r0 = zero, r1 = zero, r2 = zero, r3 = zero;
        if constexpr (UNARY) {
            if (need & 1u) r0 = make_uint4(~a.x & V.x, ~a.y & V.y, ~a.z & V.z, ~a.w & V.w);
            if (need & 2u) r1 = x_chunk(a, wave_shift_in(a, c0), V);
            if (need & 4u) {
                const uint4 sf = wave_add(a, V, c1);
                r2 = make_uint4(a.x | (V.x & (sf.x ^ a.x ^ V.x)), a.y | (V.y & (sf.y ^ a.y ^ V.y)),
                                a.z | (V.z & (sf.z ^ a.z ^ V.z)), a.w | (V.w & (sf.w ^ a.w ^ V.w)));
            }
            if (need & 8u) {
                const uint4 x = make_uint4(V.x & ~a.x, V.y & ~a.y, V.z & ~a.z, V.w & ~a.w);
                const uint4 sg = wave_add(x, V, c2);
                r3 = make_uint4(V.x & ~(x.x | (V.x & (sg.x ^ x.x ^ V.x))), V.y & ~(x.y | (V.y & (sg.y ^ x.y ^ V.y))),
                                V.z & ~(x.z | (V.z & (sg.z ^ x.z ^ V.z))), V.w & ~(x.w | (V.w & (sg.w ^ x.w ^ V.w))));
            }
            body(q, in, a, a, r0, r1, r2, r3, m, P, S);
        } else {
            const uint4 o = make_uint4(a.x | b.x, a.y | b.y, a.z | b.z, a.w | b.w);
            if (need & 1u) r0 = make_uint4(a.x & b.x, a.y & b.y, a.z & b.z, a.w & b.w);
            if (need & 2u) r1 = o;
            if (need & 4u) {
                const uint4 s1 = wave_add(b, o, c1);
                r2 = make_uint4(b.x | (a.x & (s1.x ^ b.x ^ o.x)), b.y | (a.y & (s1.y ^ b.y ^ o.y)),
                                b.z | (a.z & (s1.z ^ b.z ^ o.z)), b.w | (a.w & (s1.w ^ b.w ^ o.w)));
            }
            if (need & 8u) {
                const uint4 s2 = wave_add(a, o, c2);
                r3 = make_uint4(a.x | (b.x & (s2.x ^ a.x ^ o.x)), a.y | (b.y & (s2.y ^ a.y ^ o.y)),
                                a.z | (b.z & (s2.z ^ a.z ^ o.z)), a.w | (b.w & (s2.w ^ a.w ^ o.w)));
            }
            body(q, in, a, b, r0, r1, r2, r3, m, P, S);
        }
    }
}

// OR over a chunk of x & ~y, accumulated (x within y iff the total is 0).
__device__ __forceinline__ uint32_t andnot4(uint4 x, uint4 y) {
    return (x.x & ~y.x) | (x.y & ~y.y) | (x.z & ~y.z) | (x.w & ~y.w);
}

// Hash, operand-equality tests, spec check and table work of one work item
// (every lane of the wave calls it).  en[j]: candidate j is enabled; op[j],
// L[j], R[j]: its derivation.  Lane j (< 4) owns candidate j.
//
// Passes over the row (each recomputes the candidates from the operands):
//   1. hash of every candidate and its operand-equality tests (a result
//      equal to an operand is a stored, cheaper CM: dropped);
//   2. (only if some owner met its tag) verification against stored rows;
//   3. (only if some candidate won a slot or found the table full) the spec
//      check of those candidates and the row writes of the winners.
// A duplicate cannot separate (its stored equal was checked when written, or
// is a cheaper formula's, which would have ended the search), so only stored
// and check-only candidates are checked.  Once the store has overflowed
// (full_store, uniform) candidates are only checked: one pass, no hash.
template <bool UNARY>
__device__ __forceinline__ void wave_item_t(const Store& s, WaveAlloc& wa, const uint4* A, const uint4* B,
                                            uint32_t nq, uint64_t snap, bool full_store, const bool (&en)[4],
                                            const uint32_t (&op)[4], const uint32_t (&L)[4], const uint32_t (&R)[4],
                                            uint32_t chunk) {
    uint4* rows4 = reinterpret_cast<uint4*>(s.rows);
    const uint4* const kNoRows[4] = {nullptr, nullptr, nullptr, nullptr};
    const uint32_t lane = __lane_id();
    const uint32_t enm = (en[0] ? 1u : 0u) | (en[1] ? 2u : 0u) | (en[2] ? 4u : 0u) | (en[3] ? 8u : 0u);
    if (enm == 0) return;
    if (full_store) {  // check only
        uint32_t ck[4] = {0, 0, 0, 0};
        wave_pass_t<UNARY, false, true>(s, A, B, nq, enm, kNoRows, [&](uint32_t, bool in, uint4, uint4, uint4 r0,
                                                                     uint4 r1, uint4 r2, uint4 r3, const uint4(&)[4],
                                                                     uint4 P, uint4 S) {
            if (!in) return;
            ck[0] |= check_chunk(r0, P, S);
            ck[1] |= check_chunk(r1, P, S);
            ck[2] |= check_chunk(r2, P, S);
            ck[3] |= check_chunk(r3, P, S);
        });
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const bool sep = ((enm >> j) & 1u) && __ballot(ck[j] != 0) == 0;
            if (sep && lane == 0) report_found(s, op[j], L[j], R[j]);
        }
        return;
    }
    // pass 1: hashes and operand-equality tests
    uint64_t h[4] = {0, 0, 0, 0};
    uint32_t e[4] = {0, 0, 0, 0};  // pair: a-b, b-a, aUb vs a|b, bUa vs a|b; unary: X, F, G vs a
    uint32_t f[2] = {0, 0};        // pair: aUb vs b, bUa vs a
    wave_pass_t<UNARY, false, false>(s, A, B, nq, enm, kNoRows, [&](uint32_t q, bool in, uint4 a, uint4 b, uint4 r0,
                                                                  uint4 r1, uint4 r2, uint4 r3, const uint4(&)[4],
                                                                  uint4, uint4) {
        if (!in) return;
        const ChunkKey K = chunk_key(q);
        h[0] ^= chunk_hash(K, r0);
        h[1] ^= chunk_hash(K, r1);
        h[2] ^= chunk_hash(K, r2);
        h[3] ^= chunk_hash(K, r3);
        if constexpr (UNARY) {  // not a never equals a
            e[1] |= diff4(r1, a);
            e[2] |= diff4(r2, a);
            e[3] |= diff4(r3, a);
        } else {
            // a & b and a | b equal an operand iff one operand contains the other
            e[0] |= andnot4(a, b);
            e[1] |= andnot4(b, a);
            // a U b equals b iff it lies within b; equals a iff a U b == a
            f[0] |= andnot4(r2, b);
            e[2] |= diff4(r2, a);
            f[1] |= andnot4(r3, a);
            e[3] |= diff4(r3, b);
        }
    });
    bool act[4];
    uint64_t hj[4];
    {
        bool eq[4];
        if constexpr (UNARY) {
            eq[0] = false;
            eq[1] = __ballot(e[1] != 0) == 0;
            eq[2] = __ballot(e[2] != 0) == 0;
            eq[3] = __ballot(e[3] != 0) == 0;
        } else {
            const bool nest = __ballot(e[0] != 0) == 0 || __ballot(e[1] != 0) == 0;
            eq[0] = eq[1] = nest;
            eq[2] = __ballot(f[0] != 0) == 0 || __ballot(e[2] != 0) == 0;
            eq[3] = __ballot(f[1] != 0) == 0 || __ballot(e[3] != 0) == 0;
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            act[j] = ((enm >> j) & 1u) && !eq[j];
            hj[j] = act[j] ? hash_fin(group_xor<64>(h[j])) & s.hmask : 0;
        }
    }
    // owner lanes 0..3 run the probe; tag matches are verified by the wave
    const bool mine = lane < 4 && (lane == 0 ? act[0] : lane == 1 ? act[1] : lane == 2 ? act[2] : act[3]);
    const uint64_t hh = lane_pick4(lane & 3u, hj[0], hj[1], hj[2], hj[3]);
    const uint32_t tag = tag_of(hh);
    uint32_t st = mine ? S_PROBE : S_DONE;
    uint64_t pos = 0, cur = 0, steps = 0;
    if (st == S_PROBE) {
        pos = slot_of(s, hh);
        cur = slot_load(&s.table[pos]);
    }
    while (__ballot(st == S_PROBE) != 0) {
        bool need_v = false;
        uint32_t vrow = 0;
        if (st == S_PROBE) {
            if (steps++ >= s.tsize) st = S_FULL;
            if (st == S_PROBE && cur == kEmpty) {
                const uint64_t old = slot_cas(&s.table[pos], kEmpty, ((uint64_t)tag << 32) | kPending);
                if (old == kEmpty) st = S_WON;
                else cur = old;
            }
            if (st == S_PROBE) {
                const uint32_t cidx = (uint32_t)cur;
                if ((uint32_t)(cur >> 32) == tag) {
                    if (cidx == kPending || cidx >= snap) st = S_DEFER;
                    else {
                        need_v = true;
                        vrow = cidx;
                    }
                } else {
                    pos = slot_next(s, pos);
                    cur = slot_load(&s.table[pos]);
                }
            }
        }
        const uint32_t nvm = (uint32_t)(__ballot(need_v) & 0xFull);
        if (nvm) {
            const uint4* M[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) M[j] = rows4 + (uint64_t)__shfl(vrow, j, 64) * nq;
            uint32_t d[4] = {0, 0, 0, 0};
            wave_pass_t<UNARY, true, false>(s, A, B, nq, nvm, M, [&](uint32_t, bool in, uint4, uint4, uint4 r0,
                                                                   uint4 r1, uint4 r2, uint4 r3,
                                                                   const uint4(&mr)[4], uint4, uint4) {
                if (!in) return;
                const uint4 r[4] = {r0, r1, r2, r3};
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    if ((nvm >> j) & 1u) d[j] |= diff4(mr[j], r[j]);
            });
            bool eq_mine = false;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const bool eq = __ballot(d[j] != 0) == 0;
                if (lane == (uint32_t)j) eq_mine = eq;
            }
            if (need_v) {
                if (eq_mine) st = S_DUP;
                else {
                    pos = slot_next(s, pos);
                    cur = slot_load(&s.table[pos]);
                }
            }
        }
    }
    unsigned long long rb, dbase;
    // a wave stores at most four rows per work item: small chunks keep the
    // unused tails short
    wave_take(s, wa, st == S_WON ? 1u : 0u, st == S_DEFER ? 1u : 0u, rb, dbase, chunk);
    const uint32_t wonm = (uint32_t)(__ballot(st == S_WON) & 0xFull);
    const uint32_t chkm = (uint32_t)(__ballot(st == S_WON || st == S_FULL) & 0xFull);
    const uint32_t myrow = st == S_WON && rb < s.cap ? (uint32_t)rb : 0xFFFFFFFFu;
    bool sep_mine = false;
    if (chkm) {
        uint32_t wr[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) wr[j] = __shfl(myrow, j, 64);
        uint32_t ck[4] = {0, 0, 0, 0};
        wave_pass_t<UNARY, false, true>(s, A, B, nq, chkm, kNoRows, [&](uint32_t q, bool in, uint4, uint4, uint4 r0,
                                                                      uint4 r1, uint4 r2, uint4 r3,
                                                                      const uint4(&)[4], uint4 P, uint4 S) {
            if (!in) return;
            const uint4 r[4] = {r0, r1, r2, r3};
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                if (!((chkm >> j) & 1u)) continue;
                ck[j] |= check_chunk(r[j], P, S);
                if (((wonm >> j) & 1u) && wr[j] < s.cap) rows4[(uint64_t)wr[j] * nq + q] = r[j];
            }
        });
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const bool sep = __ballot(ck[j] != 0) == 0;
            if (lane == (uint32_t)j) sep_mine = sep;
        }
    }
    if (lane < 4) {
        const uint32_t j = lane;
        const uint32_t opj = op[0] * (j == 0) + op[1] * (j == 1) + op[2] * (j == 2) + op[3] * (j == 3);
        const uint32_t Lj = L[0] * (j == 0) + L[1] * (j == 1) + L[2] * (j == 2) + L[3] * (j == 3);
        const uint32_t Rj = R[0] * (j == 0) + R[1] * (j == 1) + R[2] * (j == 2) + R[3] * (j == 3);
        if (st == S_WON) {
            if (rb >= s.cap) {  // the slot stays reserved; the level will not be stored
                atomicExch(&s.ctr[C_OVERFLOW], 1ull);
            } else {
                s.meta[rb] = make_uint4(opj | (tag << 3), Lj, Rj, (uint32_t)hh);
                slot_store(&s.table[pos], ((uint64_t)tag << 32) | (uint32_t)rb);
            }
            if (sep_mine) report_found(s, opj, Lj, Rj);
        } else if (st == S_DEFER) {
            write_defer(s, dbase, opj, Lj, Rj, pos);
        } else if (st == S_FULL) {
            atomicExch(&s.ctr[C_OVERFLOW], 1ull);
            if (sep_mine) report_found(s, opj, Lj, Rj);
        }
    }
}

// Work items of one wave-kernel tile of a unary or pair segment g (atoms are
// the caller's): item(unary, A, B, en, op, L, R) runs on every lane of the
// wave that owns the item, with the item's operand rows and its four
// candidates (enabled, operator, left, right).  Returns the candidates
// counted by this thread.
template <class Item>
__device__ __forceinline__ uint32_t wave_items(const Store& s, const Seg& g, uint64_t lt, Item&& item) {
    const uint32_t NQ = s.Wp / 4;
    const uint32_t tid = threadIdx.x;
    const uint32_t wave = tid / 64;
    const uint32_t WT = s.wtile, WU = 2 * s.wtile;
    const uint4* rows4 = reinterpret_cast<const uint4*>(s.rows);
    uint32_t count = 0;
    if (g.kind == SEG_UNARY) {
        for (uint32_t iv = wave; iv < WU; iv += kLanes / 64) {
            const uint64_t vl = lt * WU + iv;
            if (vl >= g.nb) break;  // uniform over the wave
            const uint32_t vi = (uint32_t)(g.b0 + vl);
            const uint32_t vop = s.meta[vi].x & 7u;
            // not not a, F F a, G G a are cheaper formulas' CMs: skipped
            const bool en[4] = {(g.opmask & M_NOT) && vop != OP_NOT, (g.opmask & M_X) != 0,
                                (g.opmask & M_F) && vop != OP_F, (g.opmask & M_G) && vop != OP_G};
            const uint32_t op[4] = {OP_NOT, OP_X, OP_F, OP_G};
            const uint32_t L[4] = {vi, vi, vi, vi}, R[4] = {0, 0, 0, 0};
            item(true, rows4 + (uint64_t)vi * NQ, (const uint4*)nullptr, en, op, L, R);
            if (tid % 64 == 0) count += (uint32_t)en[0] + en[1] + en[2] + en[3];
        }
    } else {
        uint64_t ta, tb;
        if (g.tri) {  // square tiles, upper triangle ta <= tb, column by column
            tb = (uint64_t)((sqrt(8.0 * (double)lt + 1.0) - 1.0) * 0.5);
            while ((tb + 1) * (tb + 2) / 2 <= lt) ++tb;
            while (tb > 0 && tb * (tb + 1) / 2 > lt) --tb;
            ta = lt - tb * (tb + 1) / 2;
        } else {
            const uint64_t tiles_b = (g.nb + WT - 1) / WT;
            ta = lt / tiles_b;
            tb = lt % tiles_b;
        }
        const bool mA = (g.opmask & M_AND) != 0, mO = (g.opmask & M_OR) != 0;
        const bool mU = (g.opmask & M_UAB) != 0, mV = (g.opmask & M_UBA) != 0;
        for (uint32_t it = wave; it < WT * WT; it += kLanes / 64) {
            const uint64_t al = ta * WT + it / WT, bl = tb * WT + it % WT;
            if (al >= g.na || bl >= g.nb || (g.tri && al >= bl)) continue;  // uniform over the wave
            const uint32_t ai = (uint32_t)(g.a0 + al), bi = (uint32_t)(g.b0 + bl);
            const bool en[4] = {mA, mO, mU, mV};
            const uint32_t op[4] = {OP_AND, OP_OR, OP_U, OP_U};
            const uint32_t L[4] = {ai, ai, ai, bi}, R[4] = {bi, bi, bi, ai};
            item(false, rows4 + (uint64_t)ai * NQ, rows4 + (uint64_t)bi * NQ, en, op, L, R);
            if (tid % 64 == 0) count += (uint32_t)mA + mO + mU + mV;
        }
    }
    return count;
}

// One tile of the wave kernel (every thread of the block calls it): atoms,
// unary operands or pairs of segment g, rows and records taken per wave with
// `chunk`-sized allocations.  Returns the candidates counted by this thread.
__device__ __forceinline__ uint32_t wave_tile(const Store& s, const Seg& g, uint64_t lt, WaveAlloc& wa,
                                              uint64_t snap, bool full_store, uint32_t chunk) {
    if (g.kind == SEG_ATOM) {
        if (threadIdx.x < g.nb) {
            process(s, OP_ATOM, threadIdx.x, 0, snap);
            return 1;
        }
        return 0;
    }
    const uint32_t NQ = s.Wp / 4;
    return wave_items(s, g, lt,
                      [&](bool unary, const uint4* A, const uint4* B, const bool (&en)[4], const uint32_t (&op)[4],
                          const uint32_t (&L)[4], const uint32_t (&R)[4]) {
                          if (unary) wave_item_t<true>(s, wa, A, B, NQ, snap, full_store, en, op, L, R, chunk);
                          else wave_item_t<false>(s, wa, A, B, NQ, snap, full_store, en, op, L, R, chunk);
                      });
}

// Minimum waves per SIMD asked of the compiler for the wave kernel (0: its
// own choice by register use, 195 VGPRs = 2 waves; 3 costs ~17 spilled
// VGPRs and measured 18% faster on 328-chunk rows).
#ifndef LTLF_WAVE_OCC
#define LTLF_WAVE_OCC 3
#endif
#if LTLF_WAVE_OCC > 0
__global__ __launch_bounds__(kLanes, LTLF_WAVE_OCC) void k_generate_wave(Store s, SegTable t) {
#else
__global__ __launch_bounds__(kLanes) void k_generate_wave(Store s, SegTable t) {
#endif
    __shared__ unsigned long long sh_tile;
    __shared__ uint32_t sh_full;
    const uint64_t snap = s.ctr[C_SNAP];
    const uint32_t tid = threadIdx.x;
    WaveAlloc wa;
    uint32_t count = 0;
    // persistent: tiles from the cursor while the lists can take the tiles in
    // flight; the overflow flag is refreshed for every tile
    for (;;) {
        if (tid == 0) {
            unsigned long long tl = ~0ull;
            const unsigned long long d = __hip_atomic_load(&s.ctr[C_DEF0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const unsigned long long r = __hip_atomic_load(&s.ctr[C_ROWS], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const bool full = store_full(s);
            const unsigned long long cur = __hip_atomic_load(&s.ctr[C_TILE], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (cur < t.tile_stop && d + t.def_margin <= s.def0_cap && (full || r + t.row_margin <= t.row_budget))
                tl = atomicAdd(&s.ctr[C_TILE], 1ull);
            sh_tile = tl;
            sh_full = full;
        }
        __syncthreads();
        const uint64_t tile = sh_tile;
        const bool full_store = sh_full != 0;
        __syncthreads();
        if (tile >= t.tile_end) break;
        uint32_t si = 0;
        while (si + 1 < t.n && t.first[si + 1] <= tile) ++si;
        count += wave_tile(s, t.seg[si], tile - t.first[si], wa, snap, full_store, kWaveChunk);
        __syncthreads();
    }
    retire_rows(s, wa.rnext, wa.rend);
    retire_records(s, wa.dnext, wa.dend);
    wave_count(s, C_CAND, count);
}

// Batched form: tiles of many problems in one launch, one block per tile;
// segs[] sorted by first tile, each naming its problem's store.  Rows and
// records are taken exactly (chunk 1: no unused tails), each problem's
// counters being its own addresses.
__global__ __launch_bounds__(kLanes) void k_generate_wave_batch(const Store* stores, const BSeg* segs, uint32_t nsegs,
                                                                uint64_t tile0) {
    const uint64_t tile = tile0 + blockIdx.x;
    uint32_t lo = 0, hi = nsegs;  // last seg with first <= tile
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) / 2;
        if (segs[mid].first <= tile) lo = mid;
        else hi = mid;
    }
    const BSeg& b = segs[lo];
    const Store s = stores[b.problem];
    const uint64_t snap = s.ctr[C_SNAP];
    const bool full_store = store_full(s);
    WaveAlloc wa;
    const uint32_t count = wave_tile(s, b.seg, b.lt0 + (tile - b.first), wa, snap, full_store, 1);
    wave_count(s, C_CAND, count);
}

// ----------------------------------------------------------- look-ahead --
// The level after an overflowed level c holds candidates whose operand lies
// in level c: the unary operators of cost 1 (omask bits 0..3: not, X, F, G).
// Level c is not stored, so every candidate z of level c is generated again
// from the stored levels below it (level c's tiles, one wave per work item)
// and each such operator is applied to z in the same pass and checked against
// the spec.  Nothing is stored or probed: a candidate z whose CM equals a
// cheaper one has images equal to a cheaper formula's, and every cheaper
// formula has been checked without success, so checking every z is exact.
// A witness is z's derivation with the outer operator in bits 8.. of its
// operator code.
__device__ __forceinline__ void lookahead_item(const Store& s, bool unary, const uint4* A, const uint4* B,
                                               uint32_t nq, uint32_t omask, const bool (&en)[4],
                                               const uint32_t (&op)[4], const uint32_t (&L)[4],
                                               const uint32_t (&R)[4]) {
    const uint4* P4 = reinterpret_cast<const uint4*>(s.P0);
    const uint4* S4 = reinterpret_cast<const uint4*>(s.S);
    const uint4* V4 = reinterpret_cast<const uint4*>(s.V);
    // not over not, F over F and G over G give cheaper formulas' CMs
    uint32_t om[4];
#pragma unroll
    for (int j = 0; j < 4; ++j)
        om[j] = en[j] ? omask & ~(op[j] == OP_NOT ? 1u : op[j] == OP_F ? 4u : op[j] == OP_G ? 8u : 0u) : 0u;
    uint32_t cx[4] = {0, 0, 0, 0}, cf[4] = {0, 0, 0, 0}, cg[4] = {0, 0, 0, 0};
    uint32_t ck[4][4] = {};
    // lanes past the row read zero operands and masks: their chunks are 0
    wave_pass(s, unary, A, B, nq, [&](uint32_t q, bool in, uint4, uint4, uint4 r0, uint4 r1, uint4 r2, uint4 r3) {
        const uint4 V = load_if(in, &V4[q]), P = load_if(in, &P4[q]), S = load_if(in, &S4[q]);
        const uint4 r[4] = {r0, r1, r2, r3};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint4 z = r[j];
            if (om[j] & 1u)
                ck[j][0] |= check_chunk(make_uint4(~z.x & V.x, ~z.y & V.y, ~z.z & V.z, ~z.w & V.w), P, S);
            if (om[j] & 2u) ck[j][1] |= check_chunk(x_chunk(z, wave_shift_in(z, cx[j]), V), P, S);
            if (om[j] & 4u) {
                const uint4 sf = wave_add(z, V, cf[j]);
                ck[j][2] |= check_chunk(make_uint4(z.x | (V.x & (sf.x ^ z.x ^ V.x)), z.y | (V.y & (sf.y ^ z.y ^ V.y)),
                                                   z.z | (V.z & (sf.z ^ z.z ^ V.z)), z.w | (V.w & (sf.w ^ z.w ^ V.w))),
                                        P, S);
            }
            if (om[j] & 8u) {
                const uint4 x = make_uint4(V.x & ~z.x, V.y & ~z.y, V.z & ~z.z, V.w & ~z.w);
                const uint4 sg = wave_add(x, V, cg[j]);
                ck[j][3] |= check_chunk(make_uint4(V.x & ~(x.x | (V.x & (sg.x ^ x.x ^ V.x))),
                                                   V.y & ~(x.y | (V.y & (sg.y ^ x.y ^ V.y))),
                                                   V.z & ~(x.z | (V.z & (sg.z ^ x.z ^ V.z))),
                                                   V.w & ~(x.w | (V.w & (sg.w ^ x.w ^ V.w)))),
                                        P, S);
            }
        }
    });
    constexpr uint32_t outer[4] = {OP_NOT, OP_X, OP_F, OP_G};
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int o = 0; o < 4; ++o)
            if ((om[j] >> o) & 1u) {
                const bool sep = __ballot(ck[j][o] != 0) == 0;
                if (sep && __lane_id() == 0) report_found(s, op[j] | (outer[o] << 8), L[j], R[j]);
            }
}

// One block per tile of level c's plan (wave-kernel tiles), tiles
// [tile_begin, tile_end) of t.
__global__ __launch_bounds__(kLanes) void k_lookahead_wave(Store s, SegTable t, uint32_t omask) {
    const uint64_t tile = t.tile_begin + blockIdx.x;
    if (tile >= t.tile_end) return;
    uint32_t si = 0;
    while (si + 1 < t.n && t.first[si + 1] <= tile) ++si;
    const Seg& g = t.seg[si];
    const uint32_t NQ = s.Wp / 4;
    if (g.kind == SEG_ATOM) {  // level c is the atoms' level: z = p
        const uint4* atoms4 = reinterpret_cast<const uint4*>(s.atoms);
        for (uint32_t ia = threadIdx.x / 64; ia < g.nb; ia += kLanes / 64) {
            const bool en[4] = {true, false, false, false};
            const uint32_t op[4] = {OP_ATOM, OP_ATOM, OP_ATOM, OP_ATOM};
            const uint32_t L[4] = {ia, 0, 0, 0}, R[4] = {0, 0, 0, 0};
            const uint4* a = atoms4 + (uint64_t)ia * NQ;
            lookahead_item(s, false, a, a, NQ, omask, en, op, L, R);  // a & a = a
        }
        return;
    }
    wave_items(s, g, tile - t.first[si],
               [&](bool unary, const uint4* A, const uint4* B, const bool (&en)[4], const uint32_t (&op)[4],
                   const uint32_t (&L)[4], const uint32_t (&R)[4]) {
                   lookahead_item(s, unary, A, B, NQ, omask, en, op, L, R);
               });
}

// Deferred records of wide rows: one wave per record, recomputing the
// candidate step by step (any operator) against the rows it meets.
__device__ __forceinline__ void verify_wave_records(const Store& s, uint64_t first_wave, uint64_t waves) {
    const uint64_t n0 = s.ctr[C_DEF0];
    const uint64_t n = n0 < s.def0_cap ? n0 : s.def0_cap;
    const uint32_t nq = s.Wp / 4, lane = __lane_id();
    uint32_t nrec = 0;  // real records verified (statistics)
    const uint4* rows4 = reinterpret_cast<const uint4*>(s.rows);
    const uint4* atoms4 = reinterpret_cast<const uint4*>(s.atoms);
    const uint4* V4 = reinterpret_cast<const uint4*>(s.V);
    const uint4* P4 = reinterpret_cast<const uint4*>(s.P0);
    const uint4* S4 = reinterpret_cast<const uint4*>(s.S);
    for (uint64_t i = first_wave; i < n; i += waves) {
        const uint4 rec = s.def0[i];
        const uint32_t op = rec.x & 15u, L = rec.y, R = rec.z;
        if (op == kNoRecord) continue;  // uniform over the wave
        nrec += lane == 0;
        uint64_t pos = ((uint64_t)(rec.x >> 4) << 32) | rec.w;
        const uint4* A = (op == OP_ATOM ? atoms4 : rows4) + (uint64_t)L * nq;
        const uint4* B = rows4 + (uint64_t)R * nq;
        // the candidate, step by step: `body(q, in, r)`
        auto pass = [&](auto&& body) {
            uint32_t c0 = 0, c1 = 0;
            const uint32_t steps = (nq + 63) / 64;
            for (uint32_t stp = 0; stp < steps; ++stp) {
                const uint32_t q = stp * 64 + lane;
                const bool in = q < nq;
                const uint4 a = load_if(in, &A[q]);
                const uint4 b = load_if(in && op >= OP_AND, &B[q]);
                const uint4 V = load_if(in, &V4[q]);
                uint4 r;
                switch (op) {
                case OP_ATOM: r = a; break;
                case OP_NOT: r = make_uint4(~a.x & V.x, ~a.y & V.y, ~a.z & V.z, ~a.w & V.w); break;
                case OP_X: r = x_chunk(a, wave_shift_in(a, c0), V); break;
                case OP_F: {
                    const uint4 sf = wave_add(a, V, c1);
                    r = make_uint4(a.x | (V.x & (sf.x ^ a.x ^ V.x)), a.y | (V.y & (sf.y ^ a.y ^ V.y)),
                                   a.z | (V.z & (sf.z ^ a.z ^ V.z)), a.w | (V.w & (sf.w ^ a.w ^ V.w)));
                    break;
                }
                case OP_G: {
                    const uint4 x = make_uint4(V.x & ~a.x, V.y & ~a.y, V.z & ~a.z, V.w & ~a.w);
                    const uint4 sg = wave_add(x, V, c1);
                    r = make_uint4(V.x & ~(x.x | (V.x & (sg.x ^ x.x ^ V.x))), V.y & ~(x.y | (V.y & (sg.y ^ x.y ^ V.y))),
                                   V.z & ~(x.z | (V.z & (sg.z ^ x.z ^ V.z))), V.w & ~(x.w | (V.w & (sg.w ^ x.w ^ V.w))));
                    break;
                }
                case OP_AND: r = make_uint4(a.x & b.x, a.y & b.y, a.z & b.z, a.w & b.w); break;
                case OP_OR: r = make_uint4(a.x | b.x, a.y | b.y, a.z | b.z, a.w | b.w); break;
                default: {
                    const uint4 o = make_uint4(a.x | b.x, a.y | b.y, a.z | b.z, a.w | b.w);
                    const uint4 su = wave_add(b, o, c1);
                    r = make_uint4(b.x | (a.x & (su.x ^ b.x ^ o.x)), b.y | (a.y & (su.y ^ b.y ^ o.y)),
                                   b.z | (a.z & (su.z ^ b.z ^ o.z)), b.w | (a.w & (su.w ^ b.w ^ o.w)));
                    break;
                }
                }
                if (!in) r = make_uint4(0, 0, 0, 0);
                body(q, in, r);
            }
        };
        uint64_t hx = 0;
        uint32_t ck = 0;
        pass([&](uint32_t q, bool in, uint4 r) {
            if (!in) return;
            hx ^= chunk_hash(q, r);
            ck |= check_chunk(r, P4[q], S4[q]);
        });
        const uint64_t h = hash_fin(group_xor<64>(hx)) & s.hmask;
        const bool sep = __ballot(ck != 0) == 0;
        const uint32_t tag = tag_of(h);
        // walk from the slot it met (wave-uniform: every lane follows)
        uint32_t st = S_PROBE;
        for (uint64_t steps = 0; st == S_PROBE; ++steps) {
            const uint64_t cur = slot_load(&s.table[pos]);
            if (steps > s.tsize) {
                st = S_FULL;
            } else if (cur == kEmpty) {
                st = S_WON;  // new after all: re-inserted later
            } else if ((uint32_t)(cur >> 32) == tag) {
                if ((uint32_t)cur == kPending) {
                    st = S_FULL;  // only after a row overflow
                } else {
                    const uint32_t vr = (uint32_t)cur;
                    uint32_t d = 0;
                    pass([&](uint32_t q, bool in, uint4 r) {
                        if (in) d |= diff4(rows4[(uint64_t)vr * nq + q], r);
                    });
                    if (__ballot(d != 0) == 0) st = S_DUP;
                    else pos = slot_next(s, pos);
                }
            } else {
                pos = slot_next(s, pos);
            }
        }
        if (lane == 0) {
            if (st == S_WON) {
                const unsigned long long d = atomicAdd(&s.ctr[C_DEF1], 1ull);
                if (d < s.def1_cap) s.def1[d] = make_uint4(op, L, R, 0);
                else atomicExch(&s.ctr[C_DEF_OVF], 1ull);
            } else if (st == S_FULL) {
                atomicExch(&s.ctr[C_OVERFLOW], 1ull);
                if (sep) report_found(s, op, L, R);
            }
        }
    }
    wave_count(s, C_DEFERRED, nrec);
}

__global__ __launch_bounds__(kLanes) void k_verify_wave(Store s) {
    verify_wave_records(s, ((uint64_t)blockIdx.x * kLanes + threadIdx.x) / 64, (uint64_t)gridDim.x * (kLanes / 64));
}

// Batched form: blockIdx.y is the problem.
__global__ __launch_bounds__(kLanes) void k_verify_wave_batch(const Store* stores) {
    const Store s = stores[blockIdx.y];
    verify_wave_records(s, ((uint64_t)blockIdx.x * kLanes + threadIdx.x) / 64, (uint64_t)gridDim.x * (kLanes / 64));
}

// Between batched launches: every problem's deferral list is emptied and its
// launch snapshot taken (see k_between).
__global__ void k_between_batch(const Store* stores, uint32_t n) {
    const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    unsigned long long* ctr = stores[p].ctr;
    ctr[C_DEF0] = 0;
    ctr[C_SNAP] = ctr[C_ROWS];
}

// Copies every problem's counters to out[p * C_NUM + i] (one transfer to the host).
__global__ void k_gather_ctr(const Store* stores, uint32_t n, unsigned long long* out) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * C_NUM) return;
    out[i] = stores[i / C_NUM].ctr[i % C_NUM];
}

// Verifies deferred candidates against the entries they met (now visible).
// Candidates that turn out to be new go to list 1 for re-insertion.
__global__ __launch_bounds__(kLanes) void k_verify_deferred(Store s) {
    const uint64_t n = s.ctr[C_DEF0];
    const uint64_t lim = n < s.def0_cap ? n : s.def0_cap;
    uint32_t nrec = 0;  // real records verified (statistics)
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < lim;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const uint4 rec = s.def0[i];
        const uint32_t op = rec.x & 15u;
        if (op == kNoRecord) continue;
        ++nrec;
        uint64_t pos = ((uint64_t)(rec.x >> 4) << 32) | rec.w;
        const uint64_t h = cm_hash(s, op, rec.y, rec.z);
        const uint32_t tag = tag_of(h);
        for (uint64_t steps = 0;; ++steps) {
            if (steps > s.tsize) {
                atomicExch(&s.ctr[C_OVERFLOW], 1ull);
                check_only(s, op, rec.y, rec.z);
                break;
            }
            const uint64_t cur = slot_load(&s.table[pos]);
            if (cur == kEmpty) {
                const unsigned long long d = atomicAdd(&s.ctr[C_DEF1], 1ull);
                if (d < s.def1_cap) s.def1[d] = make_uint4(op, rec.y, rec.z, 0);
                else atomicExch(&s.ctr[C_DEF_OVF], 1ull);
                break;
            }
            const uint32_t cidx = (uint32_t)cur;
            if ((uint32_t)(cur >> 32) == tag) {
                if (cidx == kPending) {  // only after a row overflow
                    check_only(s, op, rec.y, rec.z);
                    break;
                }
                if (cm_equal_row(s, op, rec.y, rec.z, cidx)) break;
            }
            pos = slot_next(s, pos);
        }
    }
    wave_count(s, C_DEFERRED, nrec);
}

// Group version of the deferred verification (rows of 2..64 chunks): one
// group of G lanes per record, operands and the compared rows read as
// coalesced chunks.  The operator varies per group, so every group runs the
// same instructions with operator-selected operands (ballots stay uniform).
template <int G>
__global__ __launch_bounds__(kLanes) void k_verify_grp(Store s) {
    const uint64_t n0 = s.ctr[C_DEF0];
    const uint64_t n = n0 < s.def0_cap ? n0 : s.def0_cap;
    const uint32_t NQ = s.Wp / 4;
    const uint32_t lane = __lane_id(), k = lane % G, base = lane - k;
    uint32_t nrec = 0;  // real records verified (statistics)
    const uint64_t gid = ((uint64_t)blockIdx.x * kLanes + threadIdx.x) / G;
    const uint64_t ngroups = (uint64_t)gridDim.x * kLanes / G;
    const uint4* rows4 = reinterpret_cast<const uint4*>(s.rows);
    const uint4* atoms4 = reinterpret_cast<const uint4*>(s.atoms);
    const uint4 zero = make_uint4(0, 0, 0, 0);
    const bool kin = k < NQ;
    const uint4 V = load_if(kin, &reinterpret_cast<const uint4*>(s.V)[k]);
    const uint4 S = load_if(kin, &reinterpret_cast<const uint4*>(s.S)[k]);
    const uint4 P = load_if(kin, &reinterpret_cast<const uint4*>(s.P0)[k]);
    const uint64_t rounds = (n + ngroups - 1) / ngroups;  // uniform over the grid
    for (uint64_t rd = 0; rd < rounds; ++rd) {
        const uint64_t i = gid + rd * ngroups;
        const bool valid = i < n;
        const uint4 rec0 = load_if(valid, &s.def0[i]);
        const bool real = valid && (rec0.x & 15u) != kNoRecord;
        nrec += real && k == 0;
        const uint4 rec = real ? rec0 : make_uint4(OP_AND, 0, 0, 0);
        const uint32_t op = rec.x & 15u, L = rec.y, R = rec.z;
        uint64_t pos = ((uint64_t)(rec.x >> 4) << 32) | rec.w;
        const bool in = real && kin;
        const uint4 a = load_if(in, &(op == OP_ATOM ? atoms4 : rows4)[(uint64_t)L * NQ + k]);
        const uint4 b = load_if(in && op >= OP_AND, &rows4[(uint64_t)R * NQ + k]);
        const uint4 o = make_uint4(a.x | b.x, a.y | b.y, a.z | b.z, a.w | b.w);
        const uint4 ng = make_uint4(V.x & ~a.x, V.y & ~a.y, V.z & ~a.z, V.w & ~a.w);
        // operands of the one multi-chunk add the operator needs
        const uint4 x = op == OP_F ? a : op == OP_G ? ng : op == OP_U ? b : zero;
        const uint4 y = op == OP_F || op == OP_G ? V : op == OP_U ? o : zero;
        const uint4 sm = group_add<G>(x, y, base, k);
        const uint4 c = make_uint4(sm.x ^ x.x ^ y.x, sm.y ^ x.y ^ y.y, sm.z ^ x.z ^ y.z, sm.w ^ x.w ^ y.w);
        uint32_t up = __shfl_up(a.w >> 31, 1, 64);
        if (k == 0) up = 0;
        uint4 r;
        switch (op) {
        case OP_ATOM: r = a; break;
        case OP_NOT: r = make_uint4(~a.x & V.x, ~a.y & V.y, ~a.z & V.z, ~a.w & V.w); break;
        case OP_X:
            r = make_uint4(((a.x << 1) | up) & V.x, ((a.y << 1) | (a.x >> 31)) & V.y,
                           ((a.z << 1) | (a.y >> 31)) & V.z, ((a.w << 1) | (a.z >> 31)) & V.w);
            break;
        case OP_F: r = make_uint4(a.x | (V.x & c.x), a.y | (V.y & c.y), a.z | (V.z & c.z), a.w | (V.w & c.w)); break;
        case OP_G:
            r = make_uint4(V.x & ~(ng.x | (V.x & c.x)), V.y & ~(ng.y | (V.y & c.y)),
                           V.z & ~(ng.z | (V.z & c.z)), V.w & ~(ng.w | (V.w & c.w)));
            break;
        case OP_AND: r = make_uint4(a.x & b.x, a.y & b.y, a.z & b.z, a.w & b.w); break;
        case OP_OR: r = o; break;
        default: r = make_uint4(b.x | (a.x & c.x), b.y | (a.y & c.y), b.z | (a.z & c.z), b.w | (a.w & c.w)); break;
        }
        if (!in) r = zero;
        const uint64_t h = hash_fin(group_xor<G>(in ? chunk_hash(k, r) : 0)) & s.hmask;
        const uint32_t tag = tag_of(h);
        const bool sep = group_none<G>(in && ((r.x ^ P.x) & S.x | (r.y ^ P.y) & S.y | (r.z ^ P.z) & S.z |
                                               (r.w ^ P.w) & S.w) != 0, base);
        // owner (k == 0) walks the table from the slot it met; the group verifies
        uint32_t st = real && k == 0 ? S_PROBE : S_DONE;
        uint64_t steps = 0;
        while (__ballot(st == S_PROBE) != 0) {
            bool need_v = false;
            uint32_t vrow = 0;
            if (st == S_PROBE) {
                const uint64_t cur = slot_load(&s.table[pos]);
                if (steps++ > s.tsize) {
                    st = S_FULL;
                } else if (cur == kEmpty) {
                    st = S_WON;  // new after all: re-inserted later
                } else if ((uint32_t)(cur >> 32) == tag) {
                    if ((uint32_t)cur == kPending) st = S_FULL;  // only after a row overflow
                    else {
                        need_v = true;
                        vrow = (uint32_t)cur;
                    }
                } else {
                    pos = slot_next(s, pos);
                }
            }
            const bool nv = __shfl((int)need_v, (int)base, 64) != 0;
            const uint32_t vr = __shfl(vrow, (int)base, 64);
            const uint4 mrow = load_if(nv && kin, &rows4[(uint64_t)vr * NQ + k]);
            const bool eq = group_none<G>(nv && kin && diff4(mrow, r) != 0, base);
            if (need_v) {
                if (eq) st = S_DUP;
                else pos = slot_next(s, pos);
            }
        }
        if (st == S_WON) {
            const unsigned long long d = atomicAdd(&s.ctr[C_DEF1], 1ull);
            if (d < s.def1_cap) s.def1[d] = make_uint4(op, L, R, 0);
            else atomicExch(&s.ctr[C_DEF_OVF], 1ull);
        } else if (st == S_FULL) {
            atomicExch(&s.ctr[C_OVERFLOW], 1ull);
            if (sep) report_found(s, op, L, R);
        }
    }
    wave_count(s, C_DEFERRED, nrec);
}

// Re-inserts list-1 records (the rare deferred candidates that were new).
__global__ __launch_bounds__(kLanes) void k_reinsert(Store s, uint64_t n) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint64_t snap = s.ctr[C_SNAP];
    const uint4 rec = s.def1[i];
    process(s, rec.x, rec.y, rec.z, snap);
}

// Between launches: empty deferral list 0 and record the row count that the
// next inserting launch treats as "written before me".
__global__ void k_between(unsigned long long* ctr) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        ctr[C_DEF0] = 0;
        ctr[C_SNAP] = ctr[C_ROWS];
    }
}

__global__ void k_set_counter(unsigned long long* ctr, uint32_t which, unsigned long long v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) ctr[which] = v;
}

__global__ void k_fill_u64(uint64_t* p, uint64_t n, uint64_t v) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// Re-inserts every stored row into a freshly cleared (larger) table.
__global__ __launch_bounds__(kLanes) void k_rehash(Store s, uint64_t n_rows) {
    const uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n_rows) return;
    const uint4 mt = s.meta[r];
    if (mt.y == kDead) return;
    const uint64_t want = ((uint64_t)(mt.x >> 3) << 32) | (uint32_t)r;
    uint64_t pos = (uint64_t)__umulhi(mt.w, (uint32_t)s.tsize);
    for (uint64_t steps = 0; slot_cas(&s.table[pos], kEmpty, want) != kEmpty; ++steps) {
        if (steps > s.tsize) {
            atomicExch(&s.ctr[C_OVERFLOW], 1ull);
            return;
        }
        pos = slot_next(s, pos);
    }
}

// Level compaction (after a level kept dead rows): the holes below the new
// end of the level receive the live rows above it.  Scan: list up to `cap`
// of each (unordered; both lists have the same true length).  Move: copy row
// and record, repoint the row's table slot (probing from its home slot), and
// retire the source, so that a further round continues where this one ended.
__device__ __forceinline__ void list_append(unsigned long long* ctr, bool take, uint32_t v, uint32_t* list,
                                            uint64_t cap) {
    const uint64_t m = __ballot(take);
    if (m == 0) return;
    unsigned long long b = 0;
    if (__lane_id() == 0) b = atomicAdd(ctr, (unsigned long long)__popcll(m));
    b = __shfl(b, 0, 64);
    const uint64_t i = b + __popcll(m & ((1ull << __lane_id()) - 1));
    if (take && i < cap) list[i] = v;
}

__global__ __launch_bounds__(kLanes) void k_compact_scan(Store s, uint64_t lo, uint64_t new_end, uint64_t hi,
                                                         uint32_t* holes, uint32_t* movers, uint64_t cap) {
    const uint64_t waves = (uint64_t)gridDim.x * (kLanes / 64);
    const uint64_t wid = ((uint64_t)blockIdx.x * kLanes + threadIdx.x) / 64;
    for (uint64_t r0 = lo + wid * 64; r0 < hi; r0 += waves * 64) {
        const uint64_t r = r0 + __lane_id();
        const bool valid = r < hi;
        const bool dead = valid && s.meta[r].y == kDead;
        list_append(&s.ctr[C_NH], dead && r < new_end, (uint32_t)r, holes, cap);
        list_append(&s.ctr[C_NM], valid && !dead && r >= new_end, (uint32_t)r, movers, cap);
    }
}

__global__ __launch_bounds__(kLanes) void k_compact_move(Store s, const uint32_t* holes, const uint32_t* movers,
                                                         uint64_t cap) {
    const uint64_t nh = s.ctr[C_NH], nm = s.ctr[C_NM];
    uint64_t n = nh < nm ? nh : nm;
    n = n < cap ? n : cap;
    const uint32_t NQ = s.Wp / 4;
    uint4* rows4 = reinterpret_cast<uint4*>(s.rows);
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t src = movers[i], dst = holes[i];
        for (uint32_t q = 0; q < NQ; ++q) rows4[(uint64_t)dst * NQ + q] = rows4[(uint64_t)src * NQ + q];
        const uint4 mt = s.meta[src];
        s.meta[dst] = mt;
        s.meta[src] = make_uint4(0, kDead, 0, 0);
        const uint64_t tagw = (uint64_t)(mt.x >> 3) << 32;
        uint64_t pos = slot_of(s, mt.w);
        for (uint64_t steps = 0; steps <= s.tsize; ++steps) {
            if (s.table[pos] == (tagw | src)) {
                s.table[pos] = tagw | dst;
                break;
            }
            pos = slot_next(s, pos);
        }
    }
}

// Builds atom rows and the masks from the raw specification, one thread per
// word.  letters: trace after trace, position 0 first; seg_off[t] = first bit
// of trace t's segment (sum of n+1 over earlier traces).
__global__ void k_encode(const uint32_t* letters, const uint32_t* lengths, const uint32_t* pos_off,
                         const uint32_t* seg_off, const uint8_t* positive, uint32_t n_traces,
                         uint32_t n_props, uint32_t Wp, uint32_t* V, uint32_t* S, uint32_t* P0,
                         uint32_t* atoms) {
    const uint32_t w = blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= Wp) return;
    const uint64_t lo = 32ull * w, hi = lo + 32;
    // first trace whose segment ends after lo
    uint32_t a = 0, b = n_traces;
    while (a < b) {
        const uint32_t m = (a + b) >> 1;
        if ((uint64_t)seg_off[m + 1] <= lo) a = m + 1;
        else b = m;
    }
    // trace t's positions k = 0..n-1 sit at bits seg_off[t] + n - 1 - k (the
    // guard at seg_off[t] + n stays clear): only the bits inside this word
    // are visited
    uint32_t vw = 0, sw = 0, pw = 0;
    for (uint32_t t = a; t < n_traces && (uint64_t)seg_off[t] < hi; ++t) {
        const uint64_t seg = seg_off[t];
        const uint32_t n = lengths[t];
        const uint64_t b0 = seg > lo ? seg : lo, b1 = seg + n < hi ? seg + n : hi;
        for (uint64_t bit = b0; bit < b1; ++bit) {
            const uint32_t m = 1u << (uint32_t)(bit - lo);
            vw |= m;
            if (bit == seg + n - 1) {  // position 0
                sw |= m;
                if (positive[t]) pw |= m;
            }
        }
    }
    V[w] = vw;
    S[w] = sw;
    P0[w] = pw;
    for (uint32_t p = 0; p < n_props; ++p) {
        uint32_t aw = 0;
        for (uint32_t t = a; t < n_traces && (uint64_t)seg_off[t] < hi; ++t) {
            const uint64_t seg = seg_off[t];
            const uint32_t n = lengths[t];
            const uint64_t b0 = seg > lo ? seg : lo, b1 = seg + n < hi ? seg + n : hi;
            for (uint64_t bit = b0; bit < b1; ++bit) {
                const uint32_t k = (uint32_t)(seg + n - 1 - bit);
                if ((letters[pos_off[t] + k] >> p) & 1u) aw |= 1u << (uint32_t)(bit - lo);
            }
        }
        atoms[(uint64_t)p * Wp + w] = aw;
    }
}

// Canonical export: thread per (row, output word).  canon_bit[g] = packed bit
// index of canonical bit g.
__global__ void k_export(const uint32_t* rows, uint32_t Wp, uint64_t first, uint64_t n,
                         const uint32_t* canon_bit, uint64_t n_bits, uint64_t* out) {
    const uint64_t cw = (n_bits + 63) / 64;
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * cw) return;
    const uint64_t r = i / cw, w = i % cw;
    const uint32_t* M = rows + (first + r) * Wp;
    uint64_t acc = 0;
    for (uint32_t k = 0; k < 64; ++k) {
        const uint64_t g = w * 64 + k;
        if (g >= n_bits) break;
        const uint32_t pb = canon_bit[g];
        acc |= (uint64_t)((M[pb >> 5] >> (pb & 31)) & 1u) << k;
    }
    out[i] = acc;
}

// Level digest (a set fingerprint for comparing runs): the sum mod 2^64, over
// the rows r of a range, of D(r) = dfin(XOR over the row's 16-byte chunks q
// of dmix(q, chunk q)).  A sum does not depend on the order of the rows.  Its
// own functions (not the table hash), so that the table hash can change
// without changing digests.
__device__ __forceinline__ uint64_t dmix(uint32_t q, uint4 r) {
    const uint64_t a = ((uint64_t)r.y << 32) | r.x;
    const uint64_t b = ((uint64_t)r.w << 32) | r.z;
    uint64_t h = (a ^ ((uint64_t)(q + 1) * 0x9E3779B97F4A7C15ull)) * 0xbf58476d1ce4e5b9ull;
    h ^= (b + (h >> 31)) * 0x94d049bb133111ebull;
    return h ^ (h >> 29);
}
__device__ __forceinline__ uint64_t dfin(uint64_t k) {
    k ^= k >> 33;
    k *= 0xff51afd7ed558ccdull;
    k ^= k >> 33;
    k *= 0xc4ceb9fe1a85ec53ull;
    k ^= k >> 33;
    return k;
}

// Groups of G lanes (a power of two <= 64) take one row each, lane k of a
// group the chunks k, k + G, ...; one atomic add per wave.
__global__ __launch_bounds__(256) void k_digest(const uint4* rows, uint32_t nq, uint64_t first, uint64_t n,
                                                uint32_t G, unsigned long long* out) {
    const uint32_t lane = __lane_id();
    const uint32_t sub = lane & (G - 1);
    const uint64_t gid = ((uint64_t)blockIdx.x * 256 + threadIdx.x) / G;
    const uint64_t ngroups = (uint64_t)gridDim.x * (256 / G);
    const uint64_t iters = (n + ngroups - 1) / ngroups;
    unsigned long long sum = 0;
    for (uint64_t it = 0; it < iters; ++it) {  // uniform trip count: every lane reaches the shuffles
        const uint64_t r = it * ngroups + gid;
        uint64_t h = 0;
        if (r < n) {
            const uint4* M = rows + (first + r) * nq;
            for (uint32_t q = sub; q < nq; q += G) h ^= dmix(q, M[q]);
        }
        for (uint32_t m = 1; m < G; m <<= 1) {
            const uint32_t lo = __shfl_xor((uint32_t)h, (int)m, 64);
            const uint32_t hi = __shfl_xor((uint32_t)(h >> 32), (int)m, 64);
            h ^= ((uint64_t)hi << 32) | lo;
        }
        if (sub == 0 && r < n) sum += dfin(h);
    }
    for (int m = 32; m >= 1; m >>= 1) {
        const uint32_t lo = __shfl_xor((uint32_t)sum, m, 64);
        const uint32_t hi = __shfl_xor((uint32_t)(sum >> 32), m, 64);
        sum += ((unsigned long long)hi << 32) | lo;
    }
    if (lane == 0 && sum) atomicAdd(out, sum);
}

// Writes the prefix token list of a formula given its root derivation.
// Token = op code << 24 | payload (atom index for atoms).  tokens[0] holds the
// count (max_tokens + 1 if the formula does not fit); the words after the
// list hold the explicit traversal stack of (op, a, b) triples.
__global__ void k_formula(const uint4* meta, uint32_t root_op, uint32_t root_a, uint32_t root_b,
                          uint32_t max_tokens, uint32_t* tokens) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    uint32_t* stk = tokens + 1 + max_tokens;
    const uint32_t stack_cap = max_tokens + 1;
    uint32_t sp = 0, nt = 0;
    stk[0] = root_op;
    stk[1] = root_a;
    stk[2] = root_b;
    sp = 1;
    while (sp > 0) {
        --sp;
        const uint32_t op = stk[3 * sp], a = stk[3 * sp + 1], b = stk[3 * sp + 2];
        if (nt >= max_tokens || sp + 2 > stack_cap) {
            tokens[0] = max_tokens + 1;
            return;
        }
        tokens[1 + nt++] = (op << 24) | (op == OP_ATOM ? a : 0u);
        if (op == OP_ATOM) continue;
        if (op >= OP_AND) {  // right child below the left child on the stack
            const uint4 rb = meta[b];
            stk[3 * sp] = rb.x & 7u;
            stk[3 * sp + 1] = rb.y;
            stk[3 * sp + 2] = rb.z;
            ++sp;
        }
        const uint4 ra = meta[a];
        stk[3 * sp] = ra.x & 7u;
        stk[3 * sp + 1] = ra.y;
        stk[3 * sp + 2] = ra.z;
        ++sp;
    }
    tokens[0] = nt;
}

// ------------------------------------------------- static scratch workspace --
// The device memory of ltlf_solve_static: a file-scope array that every
// device the library runs on holds until the process ends.  In host code
// the array's name is only a stand-in for it, so its device address is
// looked up once per device (with that device current) and kept; kernels
// receive that address like any other workspace.
static __device__ __align__(256) unsigned char scratch[kStaticWorkspaceBytes];

hipError_t static_workspace(int device, void** ptr) {
    static std::mutex mu;
    static void* addr[kMaxStaticDevices] = {};
    if (device < 0 || device >= (int)kMaxStaticDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> g(mu);
    if (!addr[device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device) return hipErrorInvalidDevice;
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p || (reinterpret_cast<uintptr_t>(p) & 255u)) return hipErrorInvalidValue;
        addr[device] = p;
    }
    *ptr = addr[device];
    return hipSuccess;
}

// ---------------------------------------------------------------- launchers --
static inline uint32_t blocks_for(uint64_t n, uint32_t per) { return (uint32_t)((n + per - 1) / per); }

hipError_t launch_encode(const uint32_t* letters, const uint32_t* lengths, const uint32_t* pos_off,
                         const uint32_t* seg_off, const uint8_t* positive, uint32_t n_traces,
                         uint32_t n_props, uint32_t Wp, uint32_t* V, uint32_t* S, uint32_t* P0,
                         uint32_t* atoms, hipStream_t st) {
    hipLaunchKernelGGL(k_encode, dim3(blocks_for(Wp, 64)), dim3(64), 0, st, letters, lengths,
                       pos_off, seg_off, positive, n_traces, n_props, Wp, V, S, P0, atoms);
    return hipGetLastError();
}

hipError_t launch_fill_u64(uint64_t* p, uint64_t n, uint64_t v, hipStream_t st) {
    if (n == 0) return hipSuccess;
    uint64_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_fill_u64, dim3((uint32_t)blocks), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

// Candidates a lane keeps in flight in the LDS-staged kernel (1, 2 or 4 of a
// pair's or operand's operators between allocation points).
#ifndef LTLF_BATCH
#define LTLF_BATCH 4
#endif
constexpr int kBatch = LTLF_BATCH;

uint64_t lds_bytes(uint32_t Wp, uint32_t lanes) {
    const uint32_t nq = Wp / 4;
    return 16ull * ((uint64_t)lanes * lds_stride(nq) + kTileA * nq + 3ull * nq);
}

static uint64_t grp_lds_bytes(uint32_t Wp) {
    const uint32_t nq = Wp / 4;
    return 16ull * ((uint64_t)(kGA + kGU) * nq + 3ull * nq);
}

static uint32_t group_size(uint32_t nq) {
    uint32_t g = 4;
    while (g < nq) g <<= 1;
    return g;
}

TileShape tile_shape(uint32_t Wp, uint64_t lds_limit, uint32_t pref, uint32_t wave_tile) {
    const uint32_t wt = wave_tile_ok(wave_tile) ? wave_tile : kWaveTileBuiltin;
    const uint32_t nq = Wp / 4;
    const bool group_fits = nq >= 2 && nq <= 64 && grp_lds_bytes(Wp) <= lds_limit;
    const bool lane_fits = lds_bytes(Wp, kLanes) <= lds_limit;
    const bool half_fits = lds_bytes(Wp, kLanes / 2) <= lds_limit;
    const TileShape group{KERNEL_GROUP, kGA, kGB, kGU, 1}, lane{KERNEL_LANE, kTileA, kLanes, kLanes, 0};
    const TileShape half{KERNEL_LANE_HALF, kTileA, kLanes / 2, kLanes / 2, 0};
    const TileShape wave{KERNEL_WAVE, wt, wt, 2 * wt, 1};
    if (pref == KERNEL_WAVE) return wave;
    if (pref == KERNEL_GROUP && group_fits) return group;
    if (lane_fits) return lane;
    if (pref == KERNEL_LANE && half_fits) return half;  // the lane kernel on half-width tiles
    if (group_fits) return group;
    return wave;
}

template <class K>
static hipError_t raise_lds(K kernel, uint64_t lds) {
    if (lds <= 65536) return hipSuccess;
    return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

hipError_t generate_blocks(const Store& s, uint64_t n_tiles, uint64_t& blocks) {
    blocks = n_tiles;
    if (s.kernel != KERNEL_GROUP && s.kernel != KERNEL_WAVE) return hipSuccess;
    const uint64_t lds = grp_lds_bytes(s.Wp);
    int dev = 0, cus = 0, per_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    if (s.kernel == KERNEL_WAVE) {
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_generate_wave, kLanes, 0);
        if (e != hipSuccess) return e;
        const uint64_t resident = (uint64_t)(per_cu > 0 ? per_cu : 1) * (uint64_t)(cus > 0 ? cus : 1);
        blocks = n_tiles < resident ? n_tiles : resident;
        return hipSuccess;
    }
    switch (group_size(s.Wp / 4)) {
#define LTLF_OCC(G)                                                                              \
    case G:                                                                                      \
        e = raise_lds(k_generate_grp<G>, lds);                                                   \
        if (e == hipSuccess)                                                                     \
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_generate_grp<G>, kLanes, lds); \
        break;
        LTLF_OCC(4) LTLF_OCC(8) LTLF_OCC(16) LTLF_OCC(32) LTLF_OCC(64)
#undef LTLF_OCC
    default: return hipErrorInvalidValue;
    }
    if (e != hipSuccess) return e;
    const uint64_t resident = (uint64_t)(per_cu > 0 ? per_cu : 1) * (uint64_t)(cus > 0 ? cus : 1);
    blocks = n_tiles < resident ? n_tiles : resident;
    return hipSuccess;
}

hipError_t launch_generate(const Store& s, const SegTable& t, uint64_t blocks, hipStream_t st) {
    const uint64_t n = t.tile_end - t.tile_begin;
    if (n == 0) return hipSuccess;
    const dim3 grid((uint32_t)n), block(kLanes);
    hipError_t e = hipSuccess;
    if (s.kernel == KERNEL_GROUP) {
        // persistent blocks; the caller sized the grid and the margins
        if (blocks == 0 || blocks > n) return hipErrorInvalidValue;
        const uint64_t lds = grp_lds_bytes(s.Wp);
        switch (group_size(s.Wp / 4)) {
#define LTLF_GRP(G)                                                                             \
    case G:                                                                                     \
        e = raise_lds(k_generate_grp<G>, lds);                                                  \
        if (e != hipSuccess) return e;                                                          \
        hipLaunchKernelGGL(k_generate_grp<G>, dim3((uint32_t)blocks), block, (uint32_t)lds, st, s, t); \
        break;
            LTLF_GRP(4) LTLF_GRP(8) LTLF_GRP(16) LTLF_GRP(32) LTLF_GRP(64)
#undef LTLF_GRP
        default: return hipErrorInvalidValue;
        }
    } else if (s.kernel == KERNEL_WAVE) {
        if (blocks == 0 || blocks > n || !wave_tile_ok(s.wtile)) return hipErrorInvalidValue;
        hipLaunchKernelGGL(k_generate_wave, dim3((uint32_t)blocks), block, 0, st, s, t);
    } else if (s.kernel == KERNEL_LANE) {
        const uint64_t lds = lds_bytes(s.Wp, kLanes);
        e = raise_lds(k_generate_lds<kBatch, kLanes>, lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_generate_lds<kBatch, kLanes>), grid, block, (uint32_t)lds, st, s, t);
    } else if (s.kernel == KERNEL_LANE_HALF) {
        const uint64_t lds = lds_bytes(s.Wp, kLanes / 2);
        e = raise_lds(k_generate_lds<kBatch, kLanes / 2>, lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_generate_lds<kBatch, kLanes / 2>), grid, dim3(kLanes / 2), (uint32_t)lds, st, s, t);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_lookahead(const Store& s, const SegTable& t, uint32_t omask, hipStream_t st) {
    const uint64_t n = t.tile_end - t.tile_begin;
    if (n == 0) return hipSuccess;
    if (n > 0x7FFFFFFFull || omask == 0 || omask > 15 || !wave_tile_ok(s.wtile)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_lookahead_wave, dim3((uint32_t)n), dim3(kLanes), 0, st, s, t, omask);
    return hipGetLastError();
}

hipError_t launch_generate_batch(const Store* d_stores, const BSeg* d_segs, uint32_t nsegs, uint64_t tile0,
                                 uint64_t tiles, hipStream_t st) {
    if (tiles == 0) return hipSuccess;
    if (tiles > 0x7FFFFFFFull) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_generate_wave_batch, dim3((uint32_t)tiles), dim3(kLanes), 0, st, d_stores, d_segs, nsegs,
                       tile0);
    return hipGetLastError();
}

hipError_t launch_verify_batch(const Store* d_stores, uint32_t n, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_verify_wave_batch, dim3(8, n), dim3(kLanes), 0, st, d_stores);
    return hipGetLastError();
}

hipError_t launch_between_batch(const Store* d_stores, uint32_t n, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_between_batch, dim3(blocks_for(n, 256)), dim3(256), 0, st, d_stores, n);
    return hipGetLastError();
}

hipError_t launch_gather_ctr(const Store* d_stores, uint32_t n, unsigned long long* out, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_ctr, dim3(blocks_for((uint64_t)n * C_NUM, 256)), dim3(256), 0, st, d_stores, n,
                       out);
    return hipGetLastError();
}

// The batched launch as a graph (generation, verification, between-launch
// reset), built node by node; set_step writes each replay's counts and grids
// into the executable graph.
static hipKernelNodeParams node_params(const void* fn, dim3 grid, dim3 block, void** args) {
    hipKernelNodeParams p{};
    p.func = const_cast<void*>(fn);
    p.gridDim = grid;
    p.blockDim = block;
    p.sharedMemBytes = 0;
    p.kernelParams = args;
    p.extra = nullptr;
    return p;
}

hipError_t make_step_graphs(StepGraphs& g) {
    hipError_t e = hipGraphCreate(&g.graph, 0);
    if (e != hipSuccess) return e;
    const Store* stores = g.d_stores;
    const BSeg* segs = g.d_segs;
    uint32_t nsegs = 1, n = 1;
    uint64_t tile0 = 0;
    void* ag[] = {&stores, &segs, &nsegs, &tile0};
    void* av[] = {&stores};
    void* ab[] = {&stores, &n};
    hipKernelNodeParams p = node_params(reinterpret_cast<const void*>(k_generate_wave_batch), dim3(1), dim3(kLanes), ag);
    e = hipGraphAddKernelNode(&g.gen, g.graph, nullptr, 0, &p);
    if (e == hipSuccess) {
        p = node_params(reinterpret_cast<const void*>(k_verify_wave_batch), dim3(8, 1), dim3(kLanes), av);
        e = hipGraphAddKernelNode(&g.ver, g.graph, &g.gen, 1, &p);
    }
    if (e == hipSuccess) {
        p = node_params(reinterpret_cast<const void*>(k_between_batch), dim3(1), dim3(256), ab);
        e = hipGraphAddKernelNode(&g.btw, g.graph, &g.ver, 1, &p);
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0);
    return e;
}

hipError_t set_step(StepGraphs& g, uint32_t nsegs, uint64_t tiles, uint32_t n) {
    if (tiles == 0 || tiles > 0x7FFFFFFFull || n == 0) return hipErrorInvalidValue;
    const Store* stores = g.d_stores;
    const BSeg* segs = g.d_segs;
    uint64_t tile0 = 0;
    void* ag[] = {&stores, &segs, &nsegs, &tile0};
    void* av[] = {&stores};
    void* ab[] = {&stores, &n};
    hipKernelNodeParams p =
        node_params(reinterpret_cast<const void*>(k_generate_wave_batch), dim3((uint32_t)tiles), dim3(kLanes), ag);
    hipError_t e = hipGraphExecKernelNodeSetParams(g.exec, g.gen, &p);
    if (e == hipSuccess) {
        p = node_params(reinterpret_cast<const void*>(k_verify_wave_batch), dim3(8, n), dim3(kLanes), av);
        e = hipGraphExecKernelNodeSetParams(g.exec, g.ver, &p);
    }
    if (e == hipSuccess) {
        p = node_params(reinterpret_cast<const void*>(k_between_batch), dim3((uint32_t)blocks_for(n, 256)), dim3(256),
                        ab);
        e = hipGraphExecKernelNodeSetParams(g.exec, g.btw, &p);
    }
    return e;
}

void free_step_graphs(StepGraphs& g) {
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (g.graph) (void)hipGraphDestroy(g.graph);
    g.exec = nullptr;
    g.graph = nullptr;
}


hipError_t launch_verify_deferred(const Store& s, hipStream_t st) {
    // records are the same for every generation kernel; rows of 2..64
    // chunks are verified by lane groups (coalesced row reads)
    const uint32_t nq = s.Wp / 4;
    if (nq > 64) {
        hipLaunchKernelGGL(k_verify_wave, dim3(2048), dim3(kLanes), 0, st, s);
    } else if (nq >= 2) {
        switch (group_size(s.Wp / 4)) {
#define LTLF_VGRP(G) \
    case G: hipLaunchKernelGGL(k_verify_grp<G>, dim3(2048), dim3(kLanes), 0, st, s); break;
            LTLF_VGRP(4) LTLF_VGRP(8) LTLF_VGRP(16) LTLF_VGRP(32) LTLF_VGRP(64)
#undef LTLF_VGRP
        default: return hipErrorInvalidValue;
        }
    } else {
        hipLaunchKernelGGL(k_verify_deferred, dim3(2048), dim3(kLanes), 0, st, s);
    }
    return hipGetLastError();
}

hipError_t launch_reinsert(const Store& s, uint64_t n, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_reinsert, dim3(blocks_for(n, kLanes)), dim3(kLanes), 0, st, s, n);
    return hipGetLastError();
}

hipError_t launch_between(unsigned long long* ctr, hipStream_t st) {
    hipLaunchKernelGGL(k_between, dim3(1), dim3(64), 0, st, ctr);
    return hipGetLastError();
}

hipError_t launch_set_counter(unsigned long long* ctr, uint32_t which, unsigned long long v,
                              hipStream_t st) {
    hipLaunchKernelGGL(k_set_counter, dim3(1), dim3(64), 0, st, ctr, which, v);
    return hipGetLastError();
}

hipError_t launch_compact(const Store& s, uint64_t lo, uint64_t new_end, uint64_t hi, uint32_t* holes,
                          uint32_t* movers, uint64_t cap, hipStream_t st) {
    if (hi <= lo) return hipSuccess;
    const uint64_t b = blocks_for(hi - lo, kLanes);
    hipLaunchKernelGGL(k_compact_scan, dim3((uint32_t)(b < 16384 ? b : 16384)), dim3(kLanes), 0, st, s, lo,
                       new_end, hi, holes, movers, cap);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const uint64_t m = blocks_for(cap < hi - lo ? cap : hi - lo, kLanes);
    hipLaunchKernelGGL(k_compact_move, dim3((uint32_t)(m < 16384 ? m : 16384)), dim3(kLanes), 0, st, s, holes,
                       movers, cap);
    return hipGetLastError();
}

hipError_t launch_rehash(const Store& s, uint64_t n_rows, hipStream_t st) {
    if (n_rows == 0) return hipSuccess;
    hipLaunchKernelGGL(k_rehash, dim3(blocks_for(n_rows, kLanes)), dim3(kLanes), 0, st, s, n_rows);
    return hipGetLastError();
}

hipError_t launch_export(const uint32_t* rows, uint32_t Wp, uint64_t first, uint64_t n,
                         const uint32_t* canon_bit, uint64_t n_bits, uint64_t* out,
                         hipStream_t st) {
    const uint64_t total = n * ((n_bits + 63) / 64);
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(k_export, dim3(blocks_for(total, 256)), dim3(256), 0, st, rows, Wp, first, n,
                       canon_bit, n_bits, out);
    return hipGetLastError();
}

hipError_t launch_digest(const uint32_t* rows, uint32_t Wp, uint64_t first, uint64_t n,
                         unsigned long long* out, hipStream_t st) {
    if (n == 0) return hipSuccess;
    const uint32_t nq = Wp / 4;
    // lanes per row: rows of up to 8 chunks one pass of the next power of
    // two; wider rows the group of 8..64 lanes (128 B or more contiguous per
    // pass) that leaves the fewest lanes idle on a row's last pass (ties: the
    // larger group)
    uint32_t G = 1;
    while (G < nq && G < 8) G <<= 1;
    if (nq > 8) {
        uint64_t best = ~0ull;
        for (uint32_t g = 8; g <= 64; g <<= 1) {
            const uint64_t slots = (uint64_t)g * ((nq + g - 1) / g);
            if (slots <= best) {
                best = slots;
                G = g;
            }
        }
    }
    const uint64_t groups = n;  // one row per group per iteration
    uint64_t blocks = (groups * G + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_digest, dim3((uint32_t)blocks), dim3(256), 0, st,
                       reinterpret_cast<const uint4*>(rows), nq, first, n, G, out);
    return hipGetLastError();
}

hipError_t launch_formula(const uint4* meta, uint32_t root_op, uint32_t root_a, uint32_t root_b,
                          uint32_t max_tokens, uint32_t* tokens, hipStream_t st) {
    hipLaunchKernelGGL(k_formula, dim3(1), dim3(64), 0, st, meta, root_op, root_a, root_b,
                       max_tokens, tokens);
    return hipGetLastError();
}

}  // namespace ltlf
