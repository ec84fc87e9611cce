/*
 * ltlf.h -- C ABI of the MI355X LTLf synthesiser.
 *
 * Problem (paper, "Synthesising linear temporal logic formulae from
 * examples"): given finite example traces over atomic propositions
 * p_0..p_{m-1}, each labelled positive or negative, find a formula of minimal
 * cost over p_i, not, and, or, X, F, G, U that holds at position 0 of every
 * positive trace and fails at position 0 of every negative trace
 * ("phi separates (P, N)").  Cost is the sum of node costs; with unit costs it
 * is the formula size.
 *
 * Method (paper, "Program synthesis" and "Parallel enumeration of LTLf
 * formulae on GPUs"): bottom-up enumeration by cost, one level per cost c,
 * over formula semantics instead of syntax.  Each candidate is represented by
 * its characteristic matrix (CM): one bit per (trace, position), set iff the
 * formula holds there.  A CM is kept only if no cheaper or equally cheap
 * formula with the same CM was kept before (observational equivalence), so
 * U_c, the kept CMs of level c, are exactly the CMs whose cheapest formula
 * costs c.
 *
 * Semantics (finite traces): X is strong (false at the last position), F, G
 * and U are reflexive (phi U psi holds at i if psi holds at some j >= i and
 * phi holds on [i, j)).
 *
 * Conventions for every call:
 *   - the return value is an ltlf_status; nothing else signals errors and no
 *     C++ exception crosses this boundary;
 *   - pointers named host_* or documented as host memory are read or written
 *     only during the call; the caller keeps ownership of every buffer it
 *     passes;
 *   - "stream" is a hipStream_t passed as void* (NULL = the null stream); all
 *     device work of a call is enqueued on it, and calls that return host
 *     results synchronise it before returning;
 *   - a context is used by one host thread at a time.
 */
#ifndef LTLF_H
#define LTLF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LTLF_OK = 0,         /* a separating formula of minimal cost was found */
    LTLF_NOT_FOUND = 1,  /* no separating formula of cost <= bound */
    LTLF_CAPACITY = 2,   /* the store filled before the bound; levels_done is exact */
    LTLF_PENDING = 3,    /* server: the request has not finished yet */
    LTLF_CANCELLED = 4,  /* stopped between levels by ltlf_ctx_cancel; levels_done,
                            the level counts and checked_level are exact */
    LTLF_EINVAL = -1,    /* invalid argument (see each call) */
    LTLF_ENOMEM = -2,    /* device memory could not be obtained */
    LTLF_EDEVICE = -3,   /* a HIP runtime call failed */
    LTLF_EBUFSZ = -4,    /* a caller buffer is too small; the needed size is reported */
    LTLF_ESTATE = -5     /* call out of order (e.g. run before load) */
} ltlf_status;

/* Operator indices into ltlf_costs.op_cost. */
typedef enum {
    LTLF_NOT = 0,
    LTLF_X = 1,
    LTLF_F = 2,
    LTLF_G = 3,
    LTLF_AND = 4,
    LTLF_OR = 5,
    LTLF_U = 6,
    LTLF_NUM_OPS = 7
} ltlf_op;

/* Node costs.  atom_cost >= 1; op_cost[k] >= 1 enables operator k with that
 * cost, 0 disables it. */
typedef struct {
    uint32_t atom_cost;
    uint32_t op_cost[LTLF_NUM_OPS];
} ltlf_costs;

/* The specification (P, N), host memory.
 *   n_props  : 1..32 atomic propositions p_0..p_{n_props-1};
 *   n_traces : >= 1; the caller's order fixes the trace order inside a CM;
 *   lengths  : n_traces entries, each >= 1;
 *   letters  : sum(lengths) entries, trace after trace, position 0 first;
 *              bit p of an entry is set iff p holds at that position (bits at
 *              or above n_props must be clear);
 *   positive : n_traces entries; nonzero = P, zero = N. */
typedef struct {
    uint32_t n_props;
    uint32_t n_traces;
    const uint32_t *lengths;
    const uint32_t *letters;
    const uint8_t *positive;
} ltlf_spec;

/* Flags for ltlf_run / ltlf_solve. */
#define LTLF_FLAG_EXHAUST 0x1u /* keep enumerating complete levels up to the
                                  bound after the first separating level; the
                                  minimal cost and witness are unchanged */
#define LTLF_FLAG_PROFILE 0x2u /* time every generation and verification launch
                                  with HIP events on the run's stream and
                                  report the sums (gen_ms, verify_ms) */
#define LTLF_FLAG_KERNEL_LANE 0x4u /* generation with one candidate per lane where
                                  its operand tile (256 or 128 lanes wide) fits
                                  the LDS (the default choice wherever it
                                  fits) */
#define LTLF_FLAG_KERNEL_GROUP 0x8u /* generation with one candidate per group
                                  of lanes (one 16-byte chunk per lane) where
                                  rows have 2..64 chunks;
                                  else the default */
#define LTLF_FLAG_KERNEL_WAVE 0x10u /* generation with one candidate per
                                  wavefront, rows streamed 64 chunks at a time
                                  (the default for rows over 64 chunks).
                                  Results never depend on the kernel: these
                                  three flags exist for testing and tuning */
#define LTLF_FLAG_NO_LOOKAHEAD 0x20u /* stop at a level that overflows the store.
                                  By default, when a level overflows and none
                                  of its candidates separates, the next level
                                  is checked too, without storing it: its
                                  candidates over stored levels directly, and
                                  the cost-1 unary operators over every
                                  candidate of the overflowed level, generated
                                  again.  min_cost is then exact up to
                                  overflow_level + 1 (checked_level) */
#define LTLF_FLAG_DIGEST 0x40u /* compute each stored level's digest (a
                                  fingerprint of the level's set of CMs,
                                  independent of their order; defined at
                                  ltlf_result.level_digests) when the level
                                  closes: one extra read of its rows */
#define LTLF_FLAG_DEBUG_WEAK_HASH 0x100u /* test hook: keep 6 bits of every hash,
                                  so all candidates share a few slots and one
                                  tag; exercises the verify/defer paths */

/* Result of a run.  level_counts and formula are caller buffers (host). */
typedef struct {
    ltlf_status status;       /* OK, NOT_FOUND, CAPACITY or CANCELLED */
    uint32_t min_cost;        /* valid iff status == OK (or CANCELLED after a
                                 completed level that separates) */
    uint32_t levels_done;     /* highest completely enumerated and stored level */
    uint32_t overflow_level;  /* level that did not fit the store, 0 if none */
    uint64_t *level_counts;   /* in: buffer of level_counts_len entries or NULL;
                                 out: entry c = |U_c| for c <= levels_done, 0 above */
    uint32_t level_counts_len;
    char *formula;            /* in: buffer or NULL; out: witness in prefix tokens,
                                 e.g. "! U p1 p0"; tokens p<k>, !, X, F, G, &, |, U */
    uint64_t formula_cap;     /* in: capacity of formula in bytes */
    uint64_t formula_len;     /* out: bytes needed including the NUL */
    uint64_t candidates;      /* out: candidates generated (after pruning) */
    uint64_t unique_total;    /* out: sum of |U_c| over stored levels */
    uint64_t deferred;        /* out: candidates whose check was deferred to the
                                 verification kernel (statistics) */
    uint32_t row_bytes;       /* out: bytes of one stored CM (4 * words) */
    uint32_t gen_launches;    /* out: generation kernel launches */
    uint32_t verify_launches; /* out: verification kernel launches */
    uint32_t checked_level;   /* out: every candidate of every level up to this
                                 one was checked against the specification, so
                                 no formula of this cost or less separates
                                 unless status == OK (then min_cost <= it):
                                 levels_done, overflow_level, or
                                 overflow_level + 1 after the look-ahead */
    double enum_ms;           /* out: stream time of the whole run (events) */
    double gen_ms;            /* out: summed generation kernel time (PROFILE) */
    double verify_ms;         /* out: summed verification kernel time (PROFILE) */
    uint64_t dead_rows;       /* out: row indices taken but left unused (the
                                 allocation tails of the persistent kernels);
                                 each level is compacted at its end (statistics) */
    uint64_t *level_digests;  /* in: buffer of level_counts_len entries or NULL;
                                 out: with LTLF_FLAG_DIGEST, entry c = digest of
                                 U_c for 1 <= c <= levels_done, 0 elsewhere (all
                                 0 without the flag).  digest(U_c) = sum mod 2^64
                                 over the CMs of U_c of D(row), where row is the
                                 CM in the packed layout below, cut into 16-byte
                                 chunks k = 0, 1, ... (little-endian 64-bit
                                 halves a = bytes 0..7, b = bytes 8..15):
                                   m_k = (a ^ (k+1) * 0x9E3779B97F4A7C15) * 0xBF58476D1CE4E5B9
                                   m_k ^= (b + (m_k >> 31)) * 0x94D049BB133111EB
                                   m_k ^= m_k >> 29
                                   D = fmix64(m_0 ^ m_1 ^ ...)  (MurmurHash3's
                                 64-bit finaliser; all arithmetic mod 2^64).
                                 Packed layout: trace t of length n_t occupies
                                 bits o_t .. o_t + n_t of a little-endian bit
                                 string (o_0 = 0, o_{t+1} = o_t + n_t + 1);
                                 position k of trace t is bit o_t + n_t - 1 - k,
                                 bit o_t + n_t is 0; the string is zero-padded
                                 to W = 4 * ceil(ceil(o_T / 32) / 4) 32-bit
                                 words (row_bytes = 4 W).  Equal sets have equal
                                 digests, on any path (single, batched, served) */
} ltlf_result;

typedef struct ltlf_ctx ltlf_ctx;

/* Create a context on HIP device `device`.  hbm_budget_bytes is the device
 * memory the context allocates for itself at the first load (0 = 2 GiB,
 * values below 64 MiB are raised to 64 MiB); it is ignored once a workspace
 * is set.  EINVAL: out == NULL or
 * no such device.  EDEVICE: the device cannot be selected. */
ltlf_status ltlf_ctx_create(int device, uint64_t hbm_budget_bytes, ltlf_ctx **out);

/* Use caller-owned device memory (e.g. a framework allocation) as the
 * context's only workspace instead of allocating.  dev_ptr must be 256-byte
 * aligned device memory on the context's device, valid until the context is
 * destroyed or another workspace is set; the context never frees it.
 * EINVAL: null pointer, misalignment, or bytes < 64 MiB. */
ltlf_status ltlf_ctx_set_workspace(ltlf_ctx *ctx, void *dev_ptr, uint64_t bytes);

/* Limit the store to at most max_rows characteristic matrices (0 = as many
 * as fit in the workspace).  The level that would need more is finished
 * check-only: its candidates are still tested for separation, so a minimal
 * formula of that cost is still found, but the level is not stored and the
 * run ends there (status CAPACITY unless a separating formula was found).
 * Takes effect at the next ltlf_run.  EINVAL: ctx == NULL. */
ltlf_status ltlf_ctx_set_row_limit(ltlf_ctx *ctx, uint64_t max_rows);

/* Ask the context's running (or next) ltlf_run / ltlf_solve /
 * ltlf_solve_batch to stop.  The only call that may be made from another
 * thread while the context is in use.  The level loop takes the request
 * between two levels (a level that has started is completed): the run then
 * returns LTLF_CANCELLED with levels_done, level_counts and checked_level
 * exact for the levels it completed, and min_cost and formula filled if one
 * of them already separates (as for LTLF_OK).  A batch ends every problem
 * that has not finished as LTLF_CANCELLED with the levels it completed
 * (problems that had finished keep their results).  A request that finds no
 * run between levels stays pending for the context's next run, which then
 * stops before its first level; each request stops one run.
 * EINVAL: ctx == NULL. */
ltlf_status ltlf_ctx_cancel(ltlf_ctx *ctx);

/* Destroy a context and free the memory it allocated.  NULL is ignored. */
void ltlf_ctx_destroy(ltlf_ctx *ctx);

/* Validate a specification and copy it to the device (stream-ordered; the
 * call synchronises the stream before returning, so host buffers may be
 * reused at once).  The uploaded specification stays resident for any number
 * of ltlf_run calls.  EINVAL: ctx/spec/arrays NULL, n_props outside 1..32,
 * n_traces == 0, a zero length, or a letter with a bit >= n_props. */
ltlf_status ltlf_load(ltlf_ctx *ctx, const ltlf_spec *spec, void *stream);

/* Enumerate levels c = 1..cost_bound for the loaded specification (encode
 * atoms and masks, seed, and for each level generate, deduplicate and check
 * every candidate), then write the witness formula.  Without
 * LTLF_FLAG_EXHAUST the run stops after the first level that contains a
 * separating formula (that level is still completed).  Returns res->status
 * for OK/NOT_FOUND/CAPACITY.  EINVAL: NULL ctx/costs/res, atom_cost == 0,
 * cost_bound < atom_cost or cost_bound > 1024.  ESTATE: nothing loaded.
 * EBUFSZ: res->formula non-NULL and too small (formula_len reports the need;
 * all other fields are valid). */
ltlf_status ltlf_run(ltlf_ctx *ctx, const ltlf_costs *costs, uint32_t cost_bound, uint32_t flags,
                     void *stream, ltlf_result *res);

/* ltlf_load followed by ltlf_run. */
ltlf_status ltlf_solve(ltlf_ctx *ctx, const ltlf_spec *spec, const ltlf_costs *costs,
                       uint32_t cost_bound, uint32_t flags, void *stream, ltlf_result *res);

/* ltlf_solve without device memory allocation, for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the workspace is a static 64 MiB device array of the
 * library (one per device, held until the process ends) instead of the
 * context's, and the call makes no hipMalloc / hipFree / hipHostMalloc and
 * creates no events.  Results are those of ltlf_solve on a context whose
 * workspace is 64 MiB: levels that do not fit end the run as described at
 * LTLF_CAPACITY.  The context's own workspace and row limit are kept; the
 * context has no loaded problem afterwards (export / formula_of: ESTATE).
 * All calls on one device share the one array and each call overwrites it,
 * so calls that overlap in time on the same device (from several threads or
 * contexts) race and must not be made.
 * EINVAL: as ltlf_solve, or LTLF_FLAG_PROFILE (it creates events).  ENOMEM:
 * the specification's fixed regions (raw traces, masks, atoms, staging) do
 * not fit 64 MiB (ltlf_ctx_last_error says so).  EDEVICE: HIP failure. */
ltlf_status ltlf_solve_static(ltlf_ctx *ctx, const ltlf_spec *spec, const ltlf_costs *costs,
                              uint32_t cost_bound, uint32_t flags, void *stream, ltlf_result *res);

/* Solve n independent problems together: the batched form of ltlf_solve
 * (paper, "Program synthesis": the same bottom-up enumeration, run for many
 * specifications at once), through the request server's scheduler (see
 * ltlf_server_*): all problems are submitted at once, with reservations of
 * the small pool in proportion to their row width, and stepped until every
 * one has finished.  Every result equals that of ltlf_solve on the same
 * problem with the server's large region as capacity: status, minimal cost,
 * levels_done and level counts (the witness may be another formula of the
 * same cost); identical to ltlf_solve on this context unless the store
 * overflows.
 *   specs[i], bounds[i], results[i]: problem i; results[i] as for ltlf_run
 *     (level_counts and formula are caller buffers, or NULL).
 *   costs: shared by all problems.  flags: LTLF_FLAG_EXHAUST,
 *     LTLF_FLAG_NO_LOOKAHEAD and LTLF_FLAG_DEBUG_WEAK_HASH as for ltlf_run
 *     (others are ignored).
 * The context's row limit applies to every problem as in ltlf_solve.
 * Statistics in results[i]: enum_ms is the whole batch's time.  The
 * context's loaded problem is discarded (call ltlf_load again before
 * ltlf_run).  An invalid spec or bound gives results[i].status = EINVAL
 * without stopping the batch.  Returns OK, or EINVAL (null pointers,
 * n == 0, atom_cost == 0), ENOMEM (workspace too small), EDEVICE. */
ltlf_status ltlf_solve_batch(ltlf_ctx *ctx, uint32_t n, const ltlf_spec *specs,
                             const ltlf_costs *costs, const uint32_t *bounds,
                             uint32_t flags, void *hip_stream,
                             ltlf_result *results);

/* Generation-kernel tuning: for each class of row widths, the word tile that
 * generates fastest on this device (one candidate per lane with operands in
 * LDS, per group of lanes with one 16-byte chunk each, or per wavefront with
 * the row streamed 64 chunks at a time; each kernel has its own pair-grid
 * tile, the wave kernel's chosen per class as well).  Results never depend
 * on the choice, only the speed. */
#define LTLF_TUNE_CLASSES 16
typedef struct {
    uint32_t n_classes;                    /* classes filled */
    uint32_t chunks[LTLF_TUNE_CLASSES];    /* row width of the class, 16-byte chunks */
    uint32_t kernel[LTLF_TUNE_CLASSES];    /* choice: LTLF_FLAG_KERNEL_LANE, _GROUP or _WAVE */
    uint32_t bound[LTLF_TUNE_CLASSES];     /* cost bound of the timed runs */
    uint64_t candidates[LTLF_TUNE_CLASSES];  /* candidates of one timed run */
    double ns_per_candidate[LTLF_TUNE_CLASSES][3];  /* generation + verification time per
                                                       candidate of lane, group, wave
                                                       (wave: with its chosen pair tile;
                                                       0: not applicable at this width) */
    uint32_t wave_tile[LTLF_TUNE_CLASSES];  /* the wave kernel's pair-grid tile at this
                                               width: side of its square pair tiles, 8, 16
                                               or 32 (unary tiles: twice as many operands);
                                               0 = the built-in 16 */
    double ns_wave_tile[LTLF_TUNE_CLASSES][3];  /* the wave kernel's time per candidate with
                                                   tiles of side 8, 16, 32 */
} ltlf_tuning;

/* Measures every applicable generation kernel on a synthetic problem per
 * width class (3 propositions, 8 x chunks traces of length 15, letters and
 * labels from a fixed seed; cost bound raised until a run has about 2e10
 * bytes of candidate rows (5e6 .. 1e8 candidates) or reaches 12; every level
 * enumerated), the wave kernel with pair tiles of side 8, 16 and 32, and
 * keeps, per class in the context, the fastest (the built-in choice, and the
 * wave kernel's built-in tile, unless another is more than 5% faster): later
 * runs use the class nearest to their row width (log scale) for the kernel,
 * unless an LTLF_FLAG_KERNEL_* flag names one, and for the wave kernel's
 * tile.  The large region of a
 * batch or server created on the context inherits it.  The context's loaded
 * problem is discarded.  out may be NULL.  Returns OK, EINVAL, ENOMEM,
 * EDEVICE. */
ltlf_status ltlf_autotune(ltlf_ctx *ctx, void *stream, ltlf_tuning *out);

/* Installs a tuning table (e.g. one measured earlier on another context);
 * NULL restores the built-in choice (lane where its 256- or 128-lane tile
 * fits the LDS, up to about 67 chunks, else group up to 64 chunks, else
 * wave; the wave kernel's tile 16).  EINVAL: n_classes > LTLF_TUNE_CLASSES,
 * a chunks entry of 0, a kernel entry that is not one of the three flags, or
 * a wave_tile entry other than 0, 8, 16, 32. */
ltlf_status ltlf_ctx_set_tuning(ltlf_ctx *ctx, const ltlf_tuning *tuning);

/* Result of ltlf_solve_split.  formula is a caller buffer (host) or NULL. */
typedef struct {
    ltlf_status status;      /* OK, or NOT_FOUND / CAPACITY: a part that can no
                                longer be split (at most one positive and one
                                negative trace) has no separating formula
                                within the bound / overflowed the store */
    uint32_t depth;          /* rounds of solving (one batch each) */
    uint32_t parts_solved;   /* parts solved by enumeration (leaves) */
    uint32_t parts_split;    /* parts split */
    uint32_t max_part_cost;  /* largest minimal cost among the leaves */
    uint32_t pad;
    uint64_t cost;           /* cost of formula: separating, not necessarily
                                minimal */
    char *formula;           /* in: buffer or NULL; out: prefix tokens */
    uint64_t formula_cap;    /* in: capacity of formula in bytes */
    uint64_t formula_len;    /* out: bytes needed including the NUL */
    double enum_ms;          /* out: summed time of the batches */
} ltlf_split_result;

/* Divide-and-conquer synthesis (paper, "Parallel enumeration of LTLf formulae
 * on GPUs", paragraph "Divide-and-conquer"), for specifications too large to
 * solve in one go.  A part (P', N') of the specification is split into
 * halves P' = P1 + P2, N' = N1 + N2 (first halves in the caller's trace
 * order, the larger half first), the parts (Pi, Nj) are solved recursively
 * and recombined as (phi11 & phi12) | (phi21 & phi22); a side with one trace
 * is not split (then phi1 & phi2 over the halves of N', or phi1 | phi2 over
 * the halves of P').  A part is split before it is solved if it has more than
 * max_traces traces (0: no limit), and after its solve if that found no
 * formula within cost_bound or overflowed the store.  Each round solves all
 * of its open parts with one ltlf_solve_batch call (exact minimal formulas
 * for the parts).  The combined formula separates the specification but is in
 * general not minimal; & and | are written as their De Morgan forms over the
 * other one and ! where disabled in costs (EINVAL if neither form exists).
 *   flags: LTLF_FLAG_NO_LOOKAHEAD and LTLF_FLAG_DEBUG_WEAK_HASH as for
 *   ltlf_run.  The context's loaded problem is discarded.  Returns the
 *   result's status, or EINVAL (null pointers, invalid spec, costs or
 *   bound), EBUFSZ (formula buffer too small; formula_len says what is
 *   needed), ENOMEM, EDEVICE. */
ltlf_status ltlf_solve_split(ltlf_ctx *ctx, const ltlf_spec *spec, const ltlf_costs *costs,
                             uint32_t cost_bound, uint32_t max_traces, uint32_t flags, void *stream,
                             ltlf_split_result *res);

/* ---------------------------------------------------------------- server --
 * A request loop over one context (continuous batching).  Requests are
 * submitted at any time and advanced by ltlf_server_step.  The workspace is
 * split into a small pool (1/32, at least min(half, 256 MiB)) and one
 * large region.  Requests start in the small pool, each in its own
 * reservation, and every step moves all of them by one cost level with one
 * generation launch, one verification launch and one counter transfer (each
 * at its own level: the batched form of ltlf_solve).  A request whose next
 * level is large (over 2^20 candidates) or might not fit its reservation is
 * restarted, from the start, in the large region, which holds one request at
 * a time and runs one of its levels per step with the single-problem kernels,
 * while the small pool keeps flowing.  The large region is a request's
 * capacity: every result equals that of ltlf_solve with a workspace of the
 * large region's size (status, minimal cost, levels_done, overflow level,
 * level counts; the witness may be another formula of the same cost), so it
 * equals ltlf_solve's on this context whenever the store does not overflow;
 * a request whose fixed regions do not fit the large region is solved with
 * the whole workspace once nothing else is on the device.  While a server
 * exists its context serves it
 * only (no ltlf_load / run / solve / export on the context); the context's
 * row limit applies to every request. */
typedef struct ltlf_server ltlf_server;

/* max_resident: problems on the device at once (1..65535).  EINVAL: null
 * pointers or max_resident out of range; ENOMEM: workspace too small. */
ltlf_status ltlf_server_create(ltlf_ctx *ctx, uint32_t max_resident, ltlf_server **out);

/* Queue a request; the specification is copied.  reserve_bytes: its
 * reservation in the small pool (0 = room for ~2^18 rows, at most an eighth
 * of the pool; at least 16 MiB).  flags: LTLF_FLAG_EXHAUST,
 * LTLF_FLAG_NO_LOOKAHEAD, LTLF_FLAG_DEBUG_WEAK_HASH.  *ticket identifies it
 * in poll / cancel.
 * EINVAL: invalid specification, costs or bound (nothing is queued). */
ltlf_status ltlf_server_submit(ltlf_server *srv, const ltlf_spec *spec, const ltlf_costs *costs,
                               uint32_t cost_bound, uint32_t flags, uint64_t reserve_bytes,
                               uint64_t *ticket);

/* Admit what fits, then advance every request on the device by one level
 * (or run one waiting whole-workspace request); *n_done (may be NULL)
 * receives the number of requests that finished in this step.
 * Synchronises the stream. */
ltlf_status ltlf_server_step(ltlf_server *srv, void *hip_stream, uint32_t *n_done);

/* Result of a finished request, as ltlf_run fills it (level_counts and
 * formula are caller buffers, or NULL); the ticket is then released.
 * Returns the result's status (OK / NOT_FOUND / CAPACITY), PENDING if the
 * request has not finished, EBUFSZ if the formula buffer is too small
 * (formula_len says what is needed; the ticket is released), EINVAL for an
 * unknown ticket. */
ltlf_status ltlf_server_poll(ltlf_server *srv, uint64_t ticket, ltlf_result *result);

/* Drop a queued or running request (its reservation is freed).  EINVAL:
 * unknown ticket. */
ltlf_status ltlf_server_cancel(ltlf_server *srv, uint64_t ticket);

/* Requests waiting, requests on the device, and free bytes of the small
 * pool (each pointer may be NULL). */
ltlf_status ltlf_server_load(const ltlf_server *srv, uint32_t *queued, uint32_t *resident,
                             uint64_t *free_bytes);

/* Destroy a server; unfinished requests are dropped.  NULL is ignored. */
void ltlf_server_destroy(ltlf_server *srv);

/* Export CMs first .. first+count-1 (clipped to |U_cost|) of U_cost from the
 * last run in the canonical layout: per CM, trace by trace in the caller's
 * order, positions 0..n_t-1 as consecutive bits, least significant bit first,
 * packed into uint64 words, tail zero-padded; *words_per_cm =
 * ceil(sum(lengths) / 64).  The order of CMs within a level is unspecified
 * but fixed until the next run.  *n_cms receives the number of CMs exported
 * (or, with host_buf == NULL, that would be exported).  EBUFSZ: cap_words <
 * n_cms * words_per_cm.  EINVAL: cost 0 or above the last run's levels_done.
 * ESTATE: no completed run. */
ltlf_status ltlf_export_level(ltlf_ctx *ctx, uint32_t cost, uint64_t first, uint64_t count,
                              uint64_t *host_buf, uint64_t cap_words, uint64_t *n_cms,
                              uint64_t *words_per_cm);

/* Formula (prefix tokens) of the index-th CM of U_cost in the order used by
 * ltlf_export_level.  *need receives the bytes needed including the NUL.
 * EBUFSZ: buf too small.  EINVAL: cost or index out of range. */
ltlf_status ltlf_formula_of(ltlf_ctx *ctx, uint32_t cost, uint64_t index, char *buf, uint64_t cap,
                            uint64_t *need);

/* Description of the last failure of a call on this context (which step or
 * HIP call failed and the HIP error string); empty after a successful
 * ltlf_load/ltlf_run.  The string is owned by the context and valid until
 * the next call on it.  Never NULL. */
const char *ltlf_ctx_last_error(const ltlf_ctx *ctx);

/* Static description of a status code; never NULL. */
const char *ltlf_status_str(ltlf_status s);

#ifdef __cplusplus
}
#endif

#endif /* LTLF_H */
