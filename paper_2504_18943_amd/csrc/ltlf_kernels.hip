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

namespace ltlf {

static constexpr uint64_t kEmpty = ~0ull;
static constexpr uint32_t kPending = 0xFFFFFFFFu;

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
// Per word: three full-rate ops per state word (xor, rotate, add/xor), then
// a 64-bit finaliser.  Only speed depends on the quality: every match is
// verified against the full row.
struct Hash {
    uint32_t x = 0x243F6A88u, y = 0x85A308D3u;
    __device__ __forceinline__ void add(uint32_t w) {
        const uint32_t a = w ^ x;
        x = ((a << 11) | (a >> 21)) + y;
        y = ((y << 7) | (y >> 25)) ^ a;
    }
    __device__ __forceinline__ void add4(uint4 r) {
        add(r.x);
        add(r.y);
        add(r.z);
        add(r.w);
    }
    __device__ __forceinline__ uint64_t fin() const {
        uint64_t k = ((uint64_t)x << 32) | y;
        k ^= k >> 33;
        k *= 0xff51afd7ed558ccdull;
        k ^= k >> 33;
        k *= 0xc4ceb9fe1a85ec53ull;
        k ^= k >> 33;
        return k;
    }
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
        const uint4 b = is_binary(OP) ? *reinterpret_cast<const uint4*>(B + w) : zero;
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

template <class Emit>
__device__ __forceinline__ bool emit_equal_row(const Store& s, uint64_t row, const Emit& e) {
    const uint4* M = reinterpret_cast<const uint4*>(s.rows + row * s.Wp);
    bool eq = true;
    e([&](uint32_t w, uint4 r) {
        const uint4 m = M[w >> 2];
        eq = (r.x == m.x) && (r.y == m.y) && (r.z == m.z) && (r.w == m.w);
        return eq;
    });
    return eq;
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
    if (atomicCAS(&s.ctr[C_FOUND], 0ull, 1ull) == 0ull) {
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
// overflowed (full_store: no more slots are reserved; the caller only checks
// the candidate).  Rows with index >= snap were allocated by the running
// launch and are not read.
template <class Emit>
__device__ uint32_t probe_reserve(const Store& s, uint64_t h, uint64_t& pos, uint64_t cur0,
                                  uint64_t snap, bool full_store, const Emit& e) {
    const uint32_t tag = tag_of(h);
    const uint64_t hi = (uint64_t)tag << 32;
    uint64_t cur = cur0;
    for (uint64_t steps = 0;; ++steps) {
        if (steps > s.tsize) return P_FULL;
        if (steps) cur = slot_load(&s.table[pos]);
        if (cur == kEmpty) {
            if (full_store) return P_FULL;
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

// One candidate end to end, with per-wave counter aggregation (generic path).
template <class Emit>
__device__ void insert_emit(const Store& s, const Masks& m, uint32_t op, uint32_t L, uint32_t R,
                            uint64_t h, uint64_t pos, uint64_t cur0, uint64_t snap, const Emit& e) {
    const uint32_t o = probe_reserve(s, h, pos, cur0, snap, s.ctr[C_OVERFLOW] != 0, e);
    if (o == P_WON) {
        write_row(s, m, op, L, R, h, pos, wave_alloc(&s.ctr[C_ROWS]), e);
    } else if (o == P_DEFER) {
        write_defer(s, wave_alloc(&s.ctr[C_DEF0]), op, L, R, pos);
    } else if (o == P_FULL) {
        atomicExch(&s.ctr[C_OVERFLOW], 1ull);
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
    const uint4* v;
    const uint4* V;
    uint32_t nq, op;
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
    const uint4* l;
    const uint4* r;
    uint32_t nq, op;
    template <class Fn>
    __device__ __forceinline__ void operator()(Fn&& fn) const {
        uint32_t st = 0;
        for (uint32_t q = 0; q < nq; ++q) {
            if (!fn(4u * q, binary_any(op, l[q], r[q], st))) return;
        }
    }
};

// ------------------------------------------------------------ tile mapping --
__device__ __forceinline__ void tri_tile(uint64_t lt, uint64_t& ta, uint64_t& tb) {
    // b-tile column k holds a-tiles [0, 16(k+1)); column k starts at 8k(k+1).
    uint64_t k = (uint64_t)((sqrt(1.0 + (double)lt * 0.5) - 1.0) * 0.5);
    while (8ull * (k + 1) * (k + 2) <= lt) ++k;
    while (k > 0 && 8ull * k * (k + 1) > lt) --k;
    tb = k;
    ta = lt - 8ull * k * (k + 1);
}

// ------------------------------------------------------------------ kernels --
__global__ __launch_bounds__(kLanes) void k_generate(Store s, SegTable t) {
    const uint64_t tile = t.tile_begin + blockIdx.x;
    if (tile >= t.tile_end) return;
    const uint64_t snap = s.ctr[C_SNAP];
    uint32_t si = 0;
    while (si + 1 < t.n && t.first[si + 1] <= tile) ++si;
    const Seg& g = t.seg[si];
    const uint64_t lt = tile - t.first[si];
    const uint32_t tid = threadIdx.x;
    uint32_t count = 0;

    if (g.kind == SEG_ATOM) {
        if (tid < g.nb) {
            process(s, OP_ATOM, tid, 0, snap);
            ++count;
        }
    } else if (g.kind == SEG_UNARY) {
        const uint64_t vl = lt * kLanes + tid;
        if (vl < g.nb) {
            const uint32_t v = (uint32_t)(g.b0 + vl);
            const uint32_t vop = s.meta[v].x & 7u;
            // not not a = a, F F a = F a, G G a = G a: those candidates are
            // cheaper formulas' CMs and are skipped without changing any set.
            if ((g.opmask & M_NOT) && vop != OP_NOT) { process(s, OP_NOT, v, 0, snap); ++count; }
            if (g.opmask & M_X) { process(s, OP_X, v, 0, snap); ++count; }
            if ((g.opmask & M_F) && vop != OP_F) { process(s, OP_F, v, 0, snap); ++count; }
            if ((g.opmask & M_G) && vop != OP_G) { process(s, OP_G, v, 0, snap); ++count; }
        }
    } else {
        uint64_t ta, tb;
        if (g.tri) {
            tri_tile(lt, ta, tb);
        } else {
            const uint64_t tiles_b = (g.nb + kLanes - 1) / kLanes;
            ta = lt / tiles_b;
            tb = lt % tiles_b;
        }
        const uint64_t bl = tb * kLanes + tid;
        if (bl < g.nb) {
            const uint32_t b = (uint32_t)(g.b0 + bl);
            for (uint32_t i = 0; i < kTileA; ++i) {
                const uint64_t al = ta * kTileA + i;
                if (al >= g.na) break;
                if (g.tri && al >= bl) break;  // pairs a < b only; a grows with i
                const uint32_t a = (uint32_t)(g.a0 + al);
                if (g.opmask & M_AND) { process(s, OP_AND, a, b, snap); ++count; }
                if (g.opmask & M_OR) { process(s, OP_OR, a, b, snap); ++count; }
                if (g.opmask & M_UAB) { process(s, OP_U, a, b, snap); ++count; }
                if (g.opmask & M_UBA) { process(s, OP_U, b, a, snap); ++count; }
            }
        }
    }
    // one atomic per wave for the candidate statistics
    unsigned long long c = count;
    for (int off = 32; off > 0; off >>= 1) c += __shfl_down(c, off);
    if (__lane_id() == 0 && c) atomicAdd(&s.ctr[C_CAND], c);
}

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

__device__ __forceinline__ uint32_t diff4(uint4 a, uint4 b) {
    return (a.x ^ b.x) | (a.y ^ b.y) | (a.z ^ b.z) | (a.w ^ b.w);
}

// Per-candidate state of one iteration.
struct Cand {
    uint64_t h, pos, cur;
    uint32_t out;
};

// Hash pass of one candidate: records the hash and issues the first probe,
// unless the candidate is disabled or its CM equals one of its operands
// (A, or B if given) -- a stored, cheaper CM, so a sure duplicate.  P_WON
// here only marks "still to probe".
template <class Emit>
__device__ __forceinline__ void cand_begin(const Store& s, Cand& c, bool enabled, bool check_eq,
                                           const uint4* A, const uint4* B, const Emit& e) {
    c.out = P_SKIP;
    if (!enabled) return;
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
                                            const Emit& e) {
    if (c.out == P_WON) {
        write_row(s, m, op, L, R, c.h, c.pos, rb++, e);
    } else if (c.out == P_DEFER) {
        write_defer(s, db++, op, L, R, c.pos);
    } else if (c.out == P_FULL) {
        atomicExch(&s.ctr[C_OVERFLOW], 1ull);
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
// the same for not, X, F, G over the lane's operand.
template <int BATCH>
__global__ __launch_bounds__(kLanes) void k_generate_lds(Store s, SegTable t) {
    extern __shared__ uint4 dyn[];
    const uint32_t NQ = s.Wp / 4, SB = lds_stride(NQ);
    uint4* sh_b = dyn;
    uint4* sh_a = sh_b + kLanes * SB;
    uint4* sh_v = sh_a + kTileA * NQ;
    uint4* sh_s = sh_v + NQ;
    uint4* sh_p = sh_s + NQ;
    const uint64_t tile = t.tile_begin + blockIdx.x;
    if (tile >= t.tile_end) return;
    const uint64_t snap = s.ctr[C_SNAP];
    const bool full_store = s.ctr[C_OVERFLOW] != 0;
    uint32_t si = 0;
    while (si + 1 < t.n && t.first[si + 1] <= tile) ++si;
    const Seg& g = t.seg[si];
    const uint64_t lt = tile - t.first[si];
    const uint32_t tid = threadIdx.x;
    const uint4* rows4 = reinterpret_cast<const uint4*>(s.rows);
    for (uint32_t q = tid; q < NQ; q += kLanes) {
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
        const uint64_t vl = lt * kLanes + tid;
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
                cand_begin(s, c[jj], en, j != 0, mine, mine, LdsUnaryEmit{mine, sh_v, NQ, ops[j]});
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
                cand_finish(s, m, c[jj], ops[j0 + jj], vi, 0, rb, db,
                            LdsUnaryEmit{mine, sh_v, NQ, ops[j0 + jj]});
        }
    } else {
        uint64_t ta, tb;
        if (g.tri) {
            tri_tile(lt, ta, tb);
        } else {
            const uint64_t tiles_b = (g.nb + kLanes - 1) / kLanes;
            ta = lt / tiles_b;
            tb = lt % tiles_b;
        }
        for (uint32_t idx = tid; idx < kTileA * NQ; idx += kLanes) {
            const uint64_t al = ta * kTileA + idx / NQ;
            sh_a[idx] = al < g.na ? rows4[(g.a0 + al) * NQ + idx % NQ] : make_uint4(0, 0, 0, 0);
        }
        const uint64_t bl = tb * kLanes + tid;
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
                    cand_begin(s, c[jj], en, true, arow, mine, e);
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
                    cand_finish(s, m, c[jj], ops[j], j == 3 ? bi : ai, j == 3 ? ai : bi, rb, db,
                                LdsPairEmit{j == 3 ? mine : arow, j == 3 ? arow : mine, NQ, ops[j]});
                }
            }
        }
    }
    unsigned long long cc = count;
    for (int off = 32; off > 0; off >>= 1) cc += __shfl_down(cc, off);
    if (__lane_id() == 0 && cc) atomicAdd(&s.ctr[C_CAND], cc);
}

// Verifies deferred candidates against the entries they met (now visible).
// Candidates that turn out to be new go to list 1 for re-insertion.
__global__ __launch_bounds__(kLanes) void k_verify_deferred(Store s) {
    const uint64_t n = s.ctr[C_DEF0];
    const uint64_t lim = n < s.def0_cap ? n : s.def0_cap;
    if (blockIdx.x == 0 && threadIdx.x == 0 && lim) atomicAdd(&s.ctr[C_DEFERRED], (unsigned long long)lim);
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < lim;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const uint4 rec = s.def0[i];
        const uint32_t op = rec.x & 15u;
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
    uint32_t vw = 0, sw = 0, pw = 0;
    for (uint32_t t = a; t < n_traces && (uint64_t)seg_off[t] < hi; ++t) {
        const uint32_t n = lengths[t];
        for (uint32_t k = 0; k < n; ++k) {
            const uint64_t bit = (uint64_t)seg_off[t] + (n - 1 - k);
            if (bit < lo || bit >= hi) continue;
            const uint32_t m = 1u << (uint32_t)(bit - lo);
            vw |= m;
            if (k == 0) {
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
            const uint32_t n = lengths[t];
            for (uint32_t k = 0; k < n; ++k) {
                const uint64_t bit = (uint64_t)seg_off[t] + (n - 1 - k);
                if (bit < lo || bit >= hi) continue;
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

uint64_t lds_bytes(uint32_t Wp) {
    const uint32_t nq = Wp / 4;
    return 16ull * (kLanes * lds_stride(nq) + kTileA * nq + 3ull * nq);
}

hipError_t launch_generate(const Store& s, const SegTable& t, uint64_t lds_limit, hipStream_t st) {
    const uint64_t n = t.tile_end - t.tile_begin;
    if (n == 0) return hipSuccess;
    const dim3 grid((uint32_t)n), block(kLanes);
    const uint64_t lds = lds_bytes(s.Wp);
    if (lds <= lds_limit) {
        static uint64_t raised = 0;  // largest dynamic LDS size enabled so far
        if (lds > 65536 && lds > raised) {
            const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_generate_lds<kBatch>),
                                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                                     (int)lds);
            if (e != hipSuccess) return e;
            raised = lds;
        }
        hipLaunchKernelGGL(k_generate_lds<kBatch>, grid, block, (uint32_t)lds, st, s, t);
    } else {
        hipLaunchKernelGGL(k_generate, grid, block, 0, st, s, t);
    }
    return hipGetLastError();
}

hipError_t launch_verify_deferred(const Store& s, hipStream_t st) {
    hipLaunchKernelGGL(k_verify_deferred, dim3(2048), dim3(kLanes), 0, st, s);
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

hipError_t launch_formula(const uint4* meta, uint32_t root_op, uint32_t root_a, uint32_t root_b,
                          uint32_t max_tokens, uint32_t* tokens, hipStream_t st) {
    hipLaunchKernelGGL(k_formula, dim3(1), dim3(64), 0, st, meta, root_op, root_a, root_b,
                       max_tokens, tokens);
    return hipGetLastError();
}

}  // namespace ltlf
