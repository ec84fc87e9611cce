/*
 * ltlf_oracle.c -- CPU oracle for bottom-up LTLf semantic enumeration.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path links, loads or
 * calls this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or helper with
 * the HIP implementation.
 *
 * What it computes (paper, sections "Synthesising linear temporal logic
 * formulae from examples" and "Parallel enumeration of LTLf formulae on
 * GPUs"):
 *   - formulas over p_i, not, and, or, X, F, G, U with integer node costs;
 *   - the characteristic matrix (CM) of a formula: one bit per (trace,
 *     position), bit set iff  tr, k |= phi  (the paper's characteristic
 *     sequences, one per trace, in the caller's trace order);
 *   - U_c: the set of CMs whose cheapest realising formula costs exactly c
 *     ("observational equivalence": one representative per distinct CM,
 *     deduplicated over all levels, over all positions);
 *   - the minimal cost c* of a formula that separates (P, N): holds at
 *     position 0 of every positive trace and fails at position 0 of every
 *     negative one, plus one witness formula of that cost.
 *
 * Algorithm (the generic bottom-up enumeration of the "Program synthesis"
 * section, with complete levels): for c = 1 .. bound, generate every
 * candidate of cost c from the representatives of cheaper levels, in the
 * fixed order atoms, not, X, F, G, and, or, U (binary splits i = 1..), keep a
 * candidate iff its CM has not been seen before, then look for the first
 * separating CM of the completed level.
 *
 * Semantics, evaluated per position by backward loops over each trace
 * (finite-trace LTL; a trace is a non-empty sequence of proposition sets):
 *   not: r[k] = !v[k]
 *   X  : r[k] = (k+1 < n) && v[k+1]             strong next
 *   F  : r[k] = v[k] || r[k+1]                   reflexive eventually
 *   G  : r[k] = v[k] && (k == n-1 || r[k+1])     always (= not F not)
 *   U  : r[k] = psi[k] || (phi[k] && r[k+1])     reflexive until, r[n] = 0
 *
 * Data layout (private to this file): a CM is an array of 64-bit words;
 * trace t owns words [woff[t], woff[t] + ceil(n_t/64)), position k of
 * trace t is bit (k mod 64) of word woff[t] + k/64.
 *
 * Capacity: when storing one more CM would exceed max_rows, the level is
 * finished check-only (candidates not already known are still tested for
 * separation but not stored) and the search stops after that level.  With
 * the look-ahead flag, the level after it is then checked too, without
 * storing anything (see lookahead()).  The paper assumes the levels fit;
 * this capacity behaviour is the library's contract, restated here.
 */
#define _POSIX_C_SOURCE 199309L
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <stdio.h>
#include <time.h>

#define ORC_OK 0
#define ORC_NOT_FOUND 1
#define ORC_CAPACITY 2
#define ORC_EINVAL -1
#define ORC_ENOMEM -2

/* Operator codes (also the order in which a level generates candidates). */
enum { OP_ATOM = 0, OP_NOT, OP_X, OP_F, OP_G, OP_AND, OP_OR, OP_U, N_OPKINDS };

typedef struct {
    uint8_t op;
    uint32_t left;  /* atom index for OP_ATOM, else CM id */
    uint32_t right; /* CM id for binary operators */
} orc_deriv;

typedef struct orc_ctx {
    /* spec */
    uint32_t n_props, n_traces;
    uint32_t *len;   /* n_traces */
    uint32_t *woff;  /* n_traces + 1 */
    uint8_t *pos;    /* n_traces */
    uint32_t nw;     /* words per CM */
    uint64_t **atom; /* n_props CMs */
    /* store */
    uint64_t *cms;   /* rows * nw */
    orc_deriv *der;  /* rows */
    uint32_t *level_of; /* rows */
    uint64_t rows, cap_rows, alloc_rows;
    /* level ranges: ids of level c are [lstart[c], lstart[c] + lcount[c]) */
    uint64_t *lstart, *lcount;
    uint32_t max_cost;
    /* open-addressing set of CM ids keyed by the full CM */
    uint64_t *slots; /* UINT64_MAX = empty */
    uint64_t nslots;
    /* stats */
    uint64_t candidates;
    double seconds;
} orc_ctx;

/* ---- bit access in the private layout ---- */
static inline int getb(const uint64_t *cm, const orc_ctx *o, uint32_t t, uint32_t k) {
    return (int)((cm[o->woff[t] + (k >> 6)] >> (k & 63)) & 1u);
}
static inline void setb(uint64_t *cm, const orc_ctx *o, uint32_t t, uint32_t k, int v) {
    uint64_t m = 1ull << (k & 63);
    if (v) cm[o->woff[t] + (k >> 6)] |= m;
    else cm[o->woff[t] + (k >> 6)] &= ~m;
}

/* ---- the operators, one position at a time ---- */
static void eval_op(const orc_ctx *o, int op, const uint64_t *a, const uint64_t *b, uint64_t *r) {
    memset(r, 0, sizeof(uint64_t) * o->nw);
    for (uint32_t t = 0; t < o->n_traces; ++t) {
        uint32_t n = o->len[t];
        int next = 0; /* r[k+1]; 0 past the end */
        for (uint32_t kk = n; kk-- > 0;) {
            int v = 0;
            switch (op) {
            case OP_NOT: v = !getb(a, o, t, kk); break;
            case OP_X: v = (kk + 1 < n) ? getb(a, o, t, kk + 1) : 0; break;
            case OP_F: v = getb(a, o, t, kk) || next; break;
            case OP_G: v = getb(a, o, t, kk) && (kk == n - 1 || next); break;
            case OP_AND: v = getb(a, o, t, kk) && getb(b, o, t, kk); break;
            case OP_OR: v = getb(a, o, t, kk) || getb(b, o, t, kk); break;
            case OP_U: v = getb(b, o, t, kk) || (getb(a, o, t, kk) && next); break;
            default: break;
            }
            setb(r, o, t, kk, v);
            next = v;
        }
    }
}

/* ---- separation: position-0 bit equals the label on every trace ---- */
static int separates(const orc_ctx *o, const uint64_t *cm) {
    for (uint32_t t = 0; t < o->n_traces; ++t)
        if (getb(cm, o, t, 0) != (o->pos[t] ? 1 : 0)) return 0;
    return 1;
}

/* ---- exact set of CMs ---- */
static uint64_t fnv1a(const uint64_t *cm, uint32_t nw) {
    uint64_t h = 1469598103934665603ull;
    const unsigned char *p = (const unsigned char *)cm;
    for (size_t i = 0; i < (size_t)nw * 8; ++i) {
        h ^= p[i];
        h *= 1099511628211ull;
    }
    return h;
}
static const uint64_t *row(const orc_ctx *o, uint64_t id) { return o->cms + id * o->nw; }

/* returns the id of an equal stored CM, or UINT64_MAX */
static uint64_t lookup(const orc_ctx *o, const uint64_t *cm, uint64_t h) {
    uint64_t mask = o->nslots - 1;
    for (uint64_t p = h & mask;; p = (p + 1) & mask) {
        uint64_t id = o->slots[p];
        if (id == UINT64_MAX) return UINT64_MAX;
        if (memcmp(row(o, id), cm, sizeof(uint64_t) * o->nw) == 0) return id;
    }
}
static void slot_insert(orc_ctx *o, uint64_t id, uint64_t h) {
    uint64_t mask = o->nslots - 1;
    uint64_t p = h & mask;
    while (o->slots[p] != UINT64_MAX) p = (p + 1) & mask;
    o->slots[p] = id;
}
static int grow_slots(orc_ctx *o) {
    uint64_t n2 = o->nslots ? o->nslots * 2 : 1024;
    uint64_t *s = (uint64_t *)malloc(sizeof(uint64_t) * n2);
    if (!s) return -1;
    memset(s, 0xff, sizeof(uint64_t) * n2);
    free(o->slots);
    o->slots = s;
    o->nslots = n2;
    for (uint64_t id = 0; id < o->rows; ++id) slot_insert(o, id, fnv1a(row(o, id), o->nw));
    return 0;
}
static int ensure_rows(orc_ctx *o, uint64_t need) {
    if (need <= o->alloc_rows && o->cms) return 0;
    uint64_t n2 = o->alloc_rows ? o->alloc_rows : 1024;
    while (n2 < need) n2 *= 2;
    uint64_t *c = (uint64_t *)realloc(o->cms, sizeof(uint64_t) * o->nw * n2);
    if (!c) return -1;
    o->cms = c;
    orc_deriv *d = (orc_deriv *)realloc(o->der, sizeof(orc_deriv) * n2);
    if (!d) return -1;
    o->der = d;
    uint32_t *l = (uint32_t *)realloc(o->level_of, sizeof(uint32_t) * n2);
    if (!l) return -1;
    o->level_of = l;
    o->alloc_rows = n2;
    return 0;
}

/* ---- API ---- */
orc_ctx *oracle_create(void) {
    orc_ctx *o = (orc_ctx *)calloc(1, sizeof(orc_ctx));
    return o;
}

static void clear(orc_ctx *o) {
    if (o->atom) {
        for (uint32_t p = 0; p < o->n_props; ++p) free(o->atom[p]);
        free(o->atom);
    }
    free(o->len); free(o->woff); free(o->pos);
    free(o->cms); free(o->der); free(o->level_of);
    free(o->lstart); free(o->lcount); free(o->slots);
    memset(o, 0, sizeof(*o));
}

void oracle_destroy(orc_ctx *o) {
    if (!o) return;
    clear(o);
    free(o);
}

/* Validation rules shared with the library's contract (restated here). */
static int validate(uint32_t n_props, uint32_t n_traces, const uint32_t *lengths,
                    const uint32_t *letters, const uint8_t *positive, uint32_t atom_cost,
                    uint32_t cost_bound) {
    if (!lengths || !letters || !positive) return ORC_EINVAL;
    if (n_props < 1 || n_props > 32 || n_traces < 1) return ORC_EINVAL;
    if (atom_cost < 1 || cost_bound < atom_cost) return ORC_EINVAL;
    uint64_t total = 0;
    for (uint32_t t = 0; t < n_traces; ++t) {
        if (lengths[t] < 1) return ORC_EINVAL;
        total += lengths[t];
    }
    uint32_t bad = n_props == 32 ? 0u : ~((1u << n_props) - 1u);
    for (uint64_t i = 0; i < total; ++i)
        if (letters[i] & bad) return ORC_EINVAL;
    return ORC_OK;
}

typedef struct {
    int32_t status;
    uint32_t min_cost;
    uint32_t levels_done;
    uint32_t overflow_level; /* 0 if none */
    uint32_t checked_level;  /* every candidate of every level <= this was tested */
    uint32_t witness_outer;  /* unary operator over witness_der (kind 3) */
    uint64_t witness_kind;   /* 0 none, 1 stored id, 2 unstored candidate,
                                3 unary operator over an unstored candidate */
    uint64_t witness_id;     /* stored id (kind 1) */
    orc_deriv witness_der;   /* derivation (kinds 2 and 3) */
    uint64_t candidates;
    double seconds;
} orc_result;

static int add_row(orc_ctx *o, const uint64_t *cm, uint64_t h, int op, uint32_t l, uint32_t r,
                   uint32_t c) {
    if (ensure_rows(o, o->rows + 1)) return -1;
    memcpy(o->cms + o->rows * o->nw, cm, sizeof(uint64_t) * o->nw);
    o->der[o->rows].op = (uint8_t)op;
    o->der[o->rows].left = l;
    o->der[o->rows].right = r;
    o->level_of[o->rows] = c;
    o->rows += 1;
    if ((o->rows) * 2 > o->nslots) {
        if (grow_slots(o)) return -1;
    } else {
        slot_insert(o, o->rows - 1, h);
    }
    return 0;
}

/*
 * Look-ahead past level c, which did not fit the store and has no separating
 * candidate: level c + 1 is tested without storing it.  Levels below c are
 * complete.  A candidate of level c + 1 is either
 *   (a) an operator over stored levels: a unary operator of cost >= 2, or a
 *       binary operator (each of its operands costs at most c - 1), or
 *   (b) a unary operator of cost 1 over a formula of cost c.  Level c is not
 *       stored, so every candidate of level c is generated again from the
 *       stored levels (atoms, unary and binary operators, as in the main
 *       loop) and the operator is applied to it.  Candidates of level c that
 *       equal a cheaper CM give an image equal to a cheaper formula's, which
 *       does not separate, so testing them all is exact.
 * Returns 1 with the witness in res if a candidate separates, else 0.
 */
static int lookahead(orc_ctx *o, uint32_t c, const uint32_t *kappa, uint32_t atom_cost,
                     uint64_t *cand, uint64_t *img, orc_result *res) {
    const uint32_t d = c + 1;
    /* (a) unary operators of cost >= 2 over stored levels */
    for (int op = OP_NOT; op <= OP_G; ++op) {
        uint32_t k = kappa[op];
        if (k < 2 || k >= d) continue;
        uint32_t src = d - k;
        for (uint64_t q = 0; q < o->lcount[src]; ++q) {
            uint64_t id = o->lstart[src] + q;
            eval_op(o, op, row(o, id), NULL, cand);
            o->candidates++;
            if (separates(o, cand)) {
                res->witness_kind = 2;
                res->witness_der = (orc_deriv){(uint8_t)op, (uint32_t)id, 0};
                return 1;
            }
        }
    }
    /* (a) binary operators over stored levels */
    for (int op = OP_AND; op <= OP_U; ++op) {
        uint32_t k = kappa[op];
        if (k == 0 || k + 2 > d) continue;
        uint32_t rest = d - k;
        for (uint32_t i = 1; i < rest; ++i) {
            uint32_t j = rest - i;
            for (uint64_t qa = 0; qa < o->lcount[i]; ++qa) {
                for (uint64_t qb = 0; qb < o->lcount[j]; ++qb) {
                    uint64_t ia = o->lstart[i] + qa, ib = o->lstart[j] + qb;
                    eval_op(o, op, row(o, ia), row(o, ib), cand);
                    o->candidates++;
                    if (separates(o, cand)) {
                        res->witness_kind = 2;
                        res->witness_der = (orc_deriv){(uint8_t)op, (uint32_t)ia, (uint32_t)ib};
                        return 1;
                    }
                }
            }
        }
    }
    /* (b) cost-1 unary operators over every candidate of level c */
#define OUTER(OPC, L, R)                                                              \
    do {                                                                              \
        for (int ou = OP_NOT; ou <= OP_G; ++ou) {                                     \
            if (kappa[ou] != 1) continue;                                             \
            eval_op(o, ou, cand, NULL, img);                                          \
            o->candidates++;                                                          \
            if (separates(o, img)) {                                                  \
                res->witness_kind = 3;                                                \
                res->witness_outer = (uint32_t)ou;                                    \
                res->witness_der = (orc_deriv){(uint8_t)(OPC), (L), (R)};             \
                return 1;                                                             \
            }                                                                         \
        }                                                                             \
    } while (0)
    if (c == atom_cost) {
        for (uint32_t p = 0; p < o->n_props; ++p) {
            memcpy(cand, o->atom[p], sizeof(uint64_t) * o->nw);
            OUTER(OP_ATOM, p, 0);
        }
    }
    for (int op = OP_NOT; op <= OP_G; ++op) {
        uint32_t k = kappa[op];
        if (k == 0 || k >= c) continue;
        uint32_t src = c - k;
        for (uint64_t q = 0; q < o->lcount[src]; ++q) {
            uint64_t id = o->lstart[src] + q;
            eval_op(o, op, row(o, id), NULL, cand);
            OUTER(op, (uint32_t)id, 0);
        }
    }
    for (int op = OP_AND; op <= OP_U; ++op) {
        uint32_t k = kappa[op];
        if (k == 0 || k + 2 > c) continue;
        uint32_t rest = c - k;
        for (uint32_t i = 1; i < rest; ++i) {
            uint32_t j = rest - i;
            for (uint64_t qa = 0; qa < o->lcount[i]; ++qa) {
                for (uint64_t qb = 0; qb < o->lcount[j]; ++qb) {
                    uint64_t ia = o->lstart[i] + qa, ib = o->lstart[j] + qb;
                    eval_op(o, op, row(o, ia), row(o, ib), cand);
                    OUTER(op, (uint32_t)ia, (uint32_t)ib);
                }
            }
        }
    }
#undef OUTER
    return 0;
}

/*
 * Solve.  op_cost[0..6] are the costs of not, X, F, G, and, or, U; 0 disables
 * the operator.  max_rows = 0 means unlimited.  flags bit 0 (exhaust): keep
 * enumerating complete levels up to the bound after the first separating
 * level (the reported minimum cost and witness are unchanged).  flags bit 1
 * (look-ahead): after a level that overflowed with no separating candidate,
 * test the next level too (lookahead()).
 */
int oracle_solve(orc_ctx *o, uint32_t n_props, uint32_t n_traces, const uint32_t *lengths,
                 const uint32_t *letters, const uint8_t *positive, uint32_t atom_cost,
                 const uint32_t *op_cost, uint32_t cost_bound, uint64_t max_rows,
                 uint32_t flags, orc_result *res) {
    if (!o || !res || !op_cost) return ORC_EINVAL;
    memset(res, 0, sizeof(*res));
    int v = validate(n_props, n_traces, lengths, letters, positive, atom_cost, cost_bound);
    if (v != ORC_OK) { res->status = v; return v; }
    clear(o);
    struct timespec t0, t1;
    clock_gettime(CLOCK_MONOTONIC, &t0);

    o->n_props = n_props;
    o->n_traces = n_traces;
    o->len = (uint32_t *)malloc(sizeof(uint32_t) * n_traces);
    o->woff = (uint32_t *)malloc(sizeof(uint32_t) * (n_traces + 1));
    o->pos = (uint8_t *)malloc(n_traces);
    o->lstart = (uint64_t *)calloc(cost_bound + 1, sizeof(uint64_t));
    o->lcount = (uint64_t *)calloc(cost_bound + 1, sizeof(uint64_t));
    o->max_cost = cost_bound;
    if (!o->len || !o->woff || !o->pos || !o->lstart || !o->lcount) return ORC_ENOMEM;
    o->woff[0] = 0;
    for (uint32_t t = 0; t < n_traces; ++t) {
        o->len[t] = lengths[t];
        o->pos[t] = positive[t] ? 1 : 0;
        o->woff[t + 1] = o->woff[t] + (lengths[t] + 63) / 64;
    }
    o->nw = o->woff[n_traces];
    o->cap_rows = max_rows ? max_rows : UINT64_MAX;

    /* atoms: bit (t, k) of p is set iff p holds at position k of trace t */
    o->atom = (uint64_t **)calloc(n_props, sizeof(uint64_t *));
    if (!o->atom) return ORC_ENOMEM;
    for (uint32_t p = 0; p < n_props; ++p) {
        o->atom[p] = (uint64_t *)calloc(o->nw, sizeof(uint64_t));
        if (!o->atom[p]) return ORC_ENOMEM;
    }
    uint64_t li = 0;
    for (uint32_t t = 0; t < n_traces; ++t)
        for (uint32_t k = 0; k < lengths[t]; ++k, ++li)
            for (uint32_t p = 0; p < n_props; ++p)
                setb(o->atom[p], o, t, k, (int)((letters[li] >> p) & 1u));

    if (grow_slots(o)) return ORC_ENOMEM;
    uint64_t *cand = (uint64_t *)malloc(sizeof(uint64_t) * o->nw);
    if (!cand) return ORC_ENOMEM;

    int status = ORC_NOT_FOUND;
    uint32_t kappa[N_OPKINDS];
    kappa[OP_ATOM] = atom_cost;
    for (int k = 0; k < 7; ++k) kappa[OP_NOT + k] = op_cost[k];

    for (uint32_t c = 1; c <= cost_bound; ++c) {
        o->lstart[c] = o->rows;
        int overflow = 0;
        int have_unstored = 0;
        orc_deriv first_unstored = {0, 0, 0};
        /* one candidate: look it up, store it if new (or only test it once the
         * store is full); remember the first unstored separating candidate */
#define VISIT(OPC, L, R)                                                              \
    do {                                                                              \
        o->candidates++;                                                              \
        uint64_t h_ = fnv1a(cand, o->nw);                                             \
        if (lookup(o, cand, h_) == UINT64_MAX) {                                      \
            if (!overflow && o->rows + 1 > o->cap_rows) overflow = 1;                 \
            if (!overflow) {                                                          \
                if (add_row(o, cand, h_, (OPC), (L), (R), c)) { free(cand); return ORC_ENOMEM; } \
            } else if (!have_unstored && separates(o, cand)) {                        \
                have_unstored = 1;                                                    \
                first_unstored.op = (uint8_t)(OPC);                                   \
                first_unstored.left = (L);                                            \
                first_unstored.right = (R);                                           \
            }                                                                         \
        }                                                                             \
    } while (0)

        if (c == atom_cost) {
            for (uint32_t p = 0; p < n_props; ++p) {
                memcpy(cand, o->atom[p], sizeof(uint64_t) * o->nw);
                VISIT(OP_ATOM, p, 0);
            }
        }
        for (int op = OP_NOT; op <= OP_G; ++op) {
            uint32_t k = kappa[op];
            if (k == 0 || k >= c) continue;
            uint32_t src = c - k;
            for (uint64_t q = 0; q < o->lcount[src]; ++q) {
                uint64_t id = o->lstart[src] + q;
                eval_op(o, op, row(o, id), NULL, cand);
                VISIT(op, (uint32_t)id, 0);
            }
        }
        for (int op = OP_AND; op <= OP_U; ++op) {
            uint32_t k = kappa[op];
            if (k == 0 || k + 2 > c) continue;
            uint32_t rest = c - k;
            for (uint32_t i = 1; i < rest; ++i) {
                uint32_t j = rest - i;
                for (uint64_t qa = 0; qa < o->lcount[i]; ++qa) {
                    for (uint64_t qb = 0; qb < o->lcount[j]; ++qb) {
                        uint64_t ia = o->lstart[i] + qa, ib = o->lstart[j] + qb;
                        eval_op(o, op, row(o, ia), row(o, ib), cand);
                        VISIT(op, (uint32_t)ia, (uint32_t)ib);
                    }
                }
            }
        }
#undef VISIT
        o->lcount[c] = o->rows - o->lstart[c];
        /* first separating CM of the completed level, in insertion order;
         * an unstored (check-only) candidate only if no stored one separates */
        if (status != ORC_OK) {
            for (uint64_t q = 0; q < o->lcount[c]; ++q) {
                uint64_t id = o->lstart[c] + q;
                if (separates(o, row(o, id))) {
                    res->witness_kind = 1;
                    res->witness_id = id;
                    break;
                }
            }
            if (!res->witness_kind && have_unstored) {
                res->witness_kind = 2;
                res->witness_der = first_unstored;
            }
            if (res->witness_kind) {
                status = ORC_OK;
                res->min_cost = c;
            }
        }
        if (overflow) {
            if (status != ORC_OK) status = ORC_CAPACITY;
            res->levels_done = c - 1;
            res->overflow_level = c;
            res->checked_level = c;
            if (status != ORC_OK && (flags & 2u) && c < cost_bound) {
                uint64_t *img = (uint64_t *)malloc(sizeof(uint64_t) * o->nw);
                if (!img) { free(cand); return ORC_ENOMEM; }
                int found = lookahead(o, c, kappa, atom_cost, cand, img, res);
                free(img);
                res->checked_level = c + 1;
                if (found) {
                    status = ORC_OK;
                    res->min_cost = c + 1;
                }
            }
            break;
        }
        res->levels_done = c;
        res->checked_level = c;
        if (status == ORC_OK && !(flags & 1u)) break;
    }
    free(cand);
    clock_gettime(CLOCK_MONOTONIC, &t1);
    o->seconds = (double)(t1.tv_sec - t0.tv_sec) + 1e-9 * (double)(t1.tv_nsec - t0.tv_nsec);
    res->status = status;
    res->candidates = o->candidates;
    res->seconds = o->seconds;
    return status;
}

uint64_t oracle_level_count(const orc_ctx *o, uint32_t c) {
    if (!o || !o->lcount || c > o->max_cost) return 0;
    return o->lcount[c];
}

/* Words (uint64) of one CM in the canonical export format. */
uint64_t oracle_canon_words(const orc_ctx *o) {
    uint64_t total = 0;
    for (uint32_t t = 0; t < o->n_traces; ++t) total += o->len[t];
    return (total + 63) / 64;
}

/*
 * Canonical export of U_c: for each CM in insertion order, for trace t in the
 * caller's order, positions 0..n_t-1 as consecutive bits, LSB first, packed
 * into uint64 words with the tail zero-padded.  Returns the number of CMs
 * written (0 if the buffer is too small or the level does not exist).
 */
uint64_t oracle_export_level(const orc_ctx *o, uint32_t c, uint64_t *buf, uint64_t cap_words) {
    if (!o || c > o->max_cost) return 0;
    uint64_t cw = oracle_canon_words(o);
    uint64_t n = o->lcount[c];
    if (n * cw > cap_words) return 0;
    memset(buf, 0, sizeof(uint64_t) * n * cw);
    for (uint64_t q = 0; q < n; ++q) {
        const uint64_t *cm = row(o, o->lstart[c] + q);
        uint64_t *out = buf + q * cw;
        uint64_t g = 0;
        for (uint32_t t = 0; t < o->n_traces; ++t)
            for (uint32_t k = 0; k < o->len[t]; ++k, ++g)
                if (getb(cm, o, t, k)) out[g >> 6] |= 1ull << (g & 63);
    }
    return n;
}

/* ---- formula printing (prefix tokens) ---- */
static const char *tok(int op) {
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
static int emit(char *buf, size_t cap, size_t *at, const char *s) {
    size_t n = strlen(s);
    if (*at) {
        if (*at + 1 < cap) buf[*at] = ' ';
        (*at)++;
    }
    for (size_t i = 0; i < n; ++i) {
        if (*at + 1 < cap) buf[*at] = s[i];
        (*at)++;
    }
    return 0;
}
static void print_der(const orc_ctx *o, orc_deriv d, char *buf, size_t cap, size_t *at) {
    char t[16];
    if (d.op == OP_ATOM) {
        snprintf(t, sizeof t, "p%u", d.left);
        emit(buf, cap, at, t);
        return;
    }
    emit(buf, cap, at, tok(d.op));
    print_der(o, o->der[d.left], buf, cap, at);
    if (d.op >= OP_AND) print_der(o, o->der[d.right], buf, cap, at);
}

/* Writes the witness of the last solve; returns bytes needed incl. NUL. */
uint64_t oracle_witness(const orc_ctx *o, const orc_result *res, char *buf, uint64_t cap) {
    size_t at = 0;
    if (!o || !res || !res->witness_kind) {
        if (cap) buf[0] = 0;
        return 1;
    }
    orc_deriv d = res->witness_kind == 1 ? o->der[res->witness_id] : res->witness_der;
    if (res->witness_kind == 3) emit(buf, (size_t)cap, &at, tok((int)res->witness_outer));
    print_der(o, d, buf, (size_t)cap, &at);
    if (cap) buf[at < cap ? at : cap - 1] = 0;
    return (uint64_t)at + 1;
}

/* Formula of stored CM id (for re-evaluation of every stored representative). */
uint64_t oracle_formula_of(const orc_ctx *o, uint64_t id, char *buf, uint64_t cap) {
    size_t at = 0;
    if (!o || id >= o->rows) {
        if (cap) buf[0] = 0;
        return 1;
    }
    print_der(o, o->der[id], buf, (size_t)cap, &at);
    if (cap) buf[at < cap ? at : cap - 1] = 0;
    return (uint64_t)at + 1;
}

uint64_t oracle_level_start(const orc_ctx *o, uint32_t c) {
    if (!o || !o->lstart || c > o->max_cost) return 0;
    return o->lstart[c];
}
