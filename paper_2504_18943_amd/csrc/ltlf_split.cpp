// Divide-and-conquer synthesis (paper, "Parallel enumeration of LTLf formulae
// on GPUs", paragraph "Divide-and-conquer"): a specification (P, N) that is
// too large is split into parts (P_i, N_j) with P = P_1 + P_2 and
// N = N_1 + N_2 (disjoint halves), each part is solved, recursively, and the
// parts' formulas are recombined as (phi_11 and phi_12) or (phi_21 and phi_22).
// phi_i1 and phi_i2 hold on all of P_i, and one of them fails on each trace of
// N, so the conjunction separates (P_i, N); the disjunction then separates
// (P, N).  The result is a separating formula, in general not a minimal one.
//
// Built on the public entry points only: every round of splitting solves all
// of its open parts with one ltlf_solve_batch call (the exact, minimal
// enumeration for each part).
#include "ltlf.h"

#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

namespace {

// A part of the specification: the caller's trace indices, positives and
// negatives in the caller's order.
struct Part {
    std::vector<uint32_t> pos, neg;
    enum Kind { OPEN, LEAF, SPLIT_PN, SPLIT_N, SPLIT_P } kind = OPEN;
    std::string formula;  // LEAF
    uint64_t cost = 0;    // LEAF
    uint32_t child[4] = {0, 0, 0, 0};
};

// Prefix-token combinations; with a connective disabled, its De Morgan form
// over the other one and negation.
struct Combiner {
    const ltlf_costs* k;
    bool can_and() const { return k->op_cost[LTLF_AND] || (k->op_cost[LTLF_OR] && k->op_cost[LTLF_NOT]); }
    bool can_or() const { return k->op_cost[LTLF_OR] || (k->op_cost[LTLF_AND] && k->op_cost[LTLF_NOT]); }
    void bin(bool conj, const std::string& a, uint64_t ca, const std::string& b, uint64_t cb, std::string& f,
             uint64_t& c) const {
        const uint32_t direct = k->op_cost[conj ? LTLF_AND : LTLF_OR];
        if (direct) {
            f = std::string(conj ? "& " : "| ") + a + " " + b;
            c = direct + ca + cb;
            return;
        }
        // a and b = not (not a or not b); a or b = not (not a and not b)
        const uint32_t other = k->op_cost[conj ? LTLF_OR : LTLF_AND], neg = k->op_cost[LTLF_NOT];
        f = std::string(conj ? "! | ! " : "! & ! ") + a + " ! " + b;
        c = 3ull * neg + other + ca + cb;
    }
};

ltlf_status check_spec(const ltlf_spec* sp) {
    if (!sp || !sp->lengths || !sp->letters || !sp->positive) return LTLF_EINVAL;
    if (sp->n_props < 1 || sp->n_props > 32 || sp->n_traces < 1) return LTLF_EINVAL;
    for (uint32_t t = 0; t < sp->n_traces; ++t)
        if (sp->lengths[t] < 1) return LTLF_EINVAL;
    return LTLF_OK;
}

}  // namespace

extern "C" ltlf_status ltlf_solve_split(ltlf_ctx* ctx, const ltlf_spec* spec, const ltlf_costs* costs,
                                        uint32_t cost_bound, uint32_t max_traces, uint32_t flags, void* stream,
                                        ltlf_split_result* res) {
    if (!ctx || !costs || !res) return LTLF_EINVAL;
    if (check_spec(spec) != LTLF_OK) return LTLF_EINVAL;
    const Combiner comb{costs};
    if (!comb.can_and() || !comb.can_or()) return LTLF_EINVAL;
    res->status = LTLF_NOT_FOUND;
    res->depth = 0;
    res->parts_solved = 0;
    res->parts_split = 0;
    res->max_part_cost = 0;
    res->cost = 0;
    res->formula_len = 0;
    res->enum_ms = 0.0;

    // offsets of each trace's letters in the caller's array
    std::vector<uint64_t> off(spec->n_traces + 1, 0);
    for (uint32_t t = 0; t < spec->n_traces; ++t) off[t + 1] = off[t] + spec->lengths[t];

    std::vector<Part> parts(1);
    for (uint32_t t = 0; t < spec->n_traces; ++t) (spec->positive[t] ? parts[0].pos : parts[0].neg).push_back(t);

    // Splits part p into halves of P and / or N (only sides with >= 2 traces).
    auto split = [&](uint32_t p) -> bool {
        const bool sp = parts[p].pos.size() >= 2, sn = parts[p].neg.size() >= 2;
        if (!sp && !sn) return false;
        auto halves = [](const std::vector<uint32_t>& v, bool cut) {
            const size_t h = cut ? (v.size() + 1) / 2 : v.size();
            return std::make_pair(std::vector<uint32_t>(v.begin(), v.begin() + h),
                                  std::vector<uint32_t>(v.begin() + h, v.end()));
        };
        const auto P = halves(parts[p].pos, sp), N = halves(parts[p].neg, sn);
        std::vector<std::pair<const std::vector<uint32_t>*, const std::vector<uint32_t>*>> kids;
        if (sp && sn) {
            parts[p].kind = Part::SPLIT_PN;  // (P1,N1) (P1,N2) (P2,N1) (P2,N2)
            kids = {{&P.first, &N.first}, {&P.first, &N.second}, {&P.second, &N.first}, {&P.second, &N.second}};
        } else if (sn) {
            parts[p].kind = Part::SPLIT_N;  // (P,N1) (P,N2)
            kids = {{&P.first, &N.first}, {&P.first, &N.second}};
        } else {
            parts[p].kind = Part::SPLIT_P;  // (P1,N) (P2,N)
            kids = {{&P.first, &N.first}, {&P.second, &N.first}};
        }
        for (size_t i = 0; i < kids.size(); ++i) {
            Part q;
            q.pos = *kids[i].first;
            q.neg = *kids[i].second;
            parts[p].child[i] = (uint32_t)parts.size();
            parts.push_back(std::move(q));
        }
        ++res->parts_split;
        return true;
    };

    std::vector<uint32_t> open = {0};
    const uint64_t fcap = 8ull * cost_bound + 64;  // a formula of cost <= bound has <= bound tokens
    while (!open.empty()) {
        // parts above the size limit are split before any solve
        std::vector<uint32_t> solve;
        for (size_t i = 0; i < open.size(); ++i) {
            const uint32_t p = open[i];
            const size_t n = parts[p].pos.size() + parts[p].neg.size();
            if (max_traces && n > max_traces && split(p)) {
                const uint32_t nk = parts[p].kind == Part::SPLIT_PN ? 4 : 2;
                for (uint32_t j = 0; j < nk; ++j) open.push_back(parts[p].child[j]);
            } else {
                solve.push_back(p);
            }
        }
        open.clear();
        if (solve.empty()) break;
        ++res->depth;
        // one batch for every part of this round
        const uint32_t n = (uint32_t)solve.size();
        std::vector<std::vector<uint32_t>> lens(n), lets(n);
        std::vector<std::vector<uint8_t>> labs(n);
        std::vector<ltlf_spec> specs(n);
        std::vector<uint32_t> bounds(n, cost_bound);
        std::vector<ltlf_result> results(n);
        std::vector<std::vector<char>> fbuf(n, std::vector<char>(fcap));
        for (uint32_t i = 0; i < n; ++i) {
            const Part& q = parts[solve[i]];
            for (int side = 0; side < 2; ++side)
                for (uint32_t t : side == 0 ? q.pos : q.neg) {
                    lens[i].push_back(spec->lengths[t]);
                    lets[i].insert(lets[i].end(), spec->letters + off[t], spec->letters + off[t + 1]);
                    labs[i].push_back(side == 0 ? 1 : 0);
                }
            specs[i] = ltlf_spec{spec->n_props, (uint32_t)lens[i].size(), lens[i].data(), lets[i].data(),
                                 labs[i].data()};
            std::memset(&results[i], 0, sizeof(ltlf_result));
            results[i].formula = fbuf[i].data();
            results[i].formula_cap = fcap;
        }
        const ltlf_status st = ltlf_solve_batch(ctx, n, specs.data(), costs, bounds.data(),
                                                flags & (LTLF_FLAG_NO_LOOKAHEAD | LTLF_FLAG_DEBUG_WEAK_HASH),
                                                stream, results.data());
        if (st != LTLF_OK) return st;
        if (n) res->enum_ms += results[0].enum_ms;
        for (uint32_t i = 0; i < n; ++i) {
            const uint32_t p = solve[i];
            const ltlf_result& r = results[i];
            if (r.status == LTLF_OK) {
                parts[p].kind = Part::LEAF;
                parts[p].formula = fbuf[i].data();
                parts[p].cost = r.min_cost;
                res->max_part_cost = std::max(res->max_part_cost, r.min_cost);
                ++res->parts_solved;
            } else if (r.status == LTLF_NOT_FOUND || r.status == LTLF_CAPACITY) {
                // no formula within the bound, or the store overflowed: split further
                if (!split(p)) {
                    res->status = r.status;
                    if (res->formula && res->formula_cap) res->formula[0] = 0;
                    res->formula_len = 1;
                    return r.status;
                }
                const uint32_t nk = parts[p].kind == Part::SPLIT_PN ? 4 : 2;
                for (uint32_t j = 0; j < nk; ++j) open.push_back(parts[p].child[j]);
            } else {
                return r.status < 0 ? r.status : LTLF_EDEVICE;
            }
        }
    }

    // recombine bottom-up (children always have larger indices than parents)
    for (size_t p = parts.size(); p-- > 0;) {
        Part& q = parts[p];
        if (q.kind == Part::LEAF) continue;
        const Part* c[4] = {&parts[q.child[0]], &parts[q.child[1]], &parts[q.child[2]], &parts[q.child[3]]};
        if (q.kind == Part::SPLIT_PN) {
            std::string a, b;
            uint64_t ca = 0, cb = 0;
            comb.bin(true, c[0]->formula, c[0]->cost, c[1]->formula, c[1]->cost, a, ca);
            comb.bin(true, c[2]->formula, c[2]->cost, c[3]->formula, c[3]->cost, b, cb);
            comb.bin(false, a, ca, b, cb, q.formula, q.cost);
        } else {
            comb.bin(q.kind == Part::SPLIT_N, c[0]->formula, c[0]->cost, c[1]->formula, c[1]->cost, q.formula, q.cost);
        }
        q.kind = Part::LEAF;
    }
    res->status = LTLF_OK;
    res->cost = parts[0].cost;
    res->formula_len = parts[0].formula.size() + 1;
    if (res->formula) {
        if (res->formula_cap < res->formula_len) return LTLF_EBUFSZ;
        std::memcpy(res->formula, parts[0].formula.c_str(), res->formula_len);
    }
    return LTLF_OK;
}
