// queue.hpp -- the work queue of the one-launch batched merge (the task
// queue of Section 6.2.1, scheme (i), as one persistent launch): which work
// items exist, the order in which workers take them, and what each item
// waits for.  Pure host C++: the library builds the plan from it, and a CPU
// model of the workers (tests) runs the same protocol on the same plans.
//
// Items.  Every step of every column is cut into items (a tile, a digit
// range, a slice of a strided pass).  Tickets number the items in PHASE-MAJOR
// order: all items of phase 0 (column 0's, then column 1's, ...), then all
// of phase 1, and so on.  A worker takes the next ticket from one counter,
// finds the item's phase, column and index, waits for the item's
// dependencies, runs it and counts it done.
//
// Dependencies.  A column's phases form a chain: an item of phase p of
// column j needs every item of column j in the phases before p.  One counter
// per column counts its finished items; since an item starts only when all
// earlier items of its column are finished, "counter >= number of the
// column's items before phase p" holds exactly when they are all done.  The
// full-sort fallback is made of global phases (their items stride over maps
// of the columns that need it): the first waits for every column's emit, each
// later one for all items of the global phases before it (one global
// counter, same argument), and a column that needed the fallback waits for
// the whole global chain before its merge.
//
// Progress.  Every dependency of an item has a lower ticket.  Tickets are
// taken in increasing order by workers that are running, so every item an
// item waits for is held by a running worker (or finished); the lowest
// unfinished item has all its dependencies finished and runs.  No worker
// waits for a worker that has not started, so the launch needs no
// residency guarantee: it completes with any number of workers, one
// included.
#pragma once

#include <stdint.h>

#include <vector>

namespace mcq {

// Phases in ticket order.  kHash .. kEmit and kRank .. kRepack are
// per-column phases; kFbPlan .. kFbEmit are the global phases of the
// full-sort fallback (kFbPass0 + 3 * p + k: pass p, k = 0 counts, 1 scan,
// 2 scatter).
constexpr uint32_t kFbPasses = 16;  // digit positions of the widest value (16 bytes)
enum Phase : uint32_t {
    kHash = 0,
    kCompact,
    kHist,
    kHScan,
    kPre0Up,  // prefix slot s: kPre0Up + 3 * s + k, s < 3
    kWin0 = kPre0Up + 9,
    kWin1,
    kEmit,
    kFbPlan,
    kFbPass0,
    kFbEmit = kFbPass0 + 3 * kFbPasses,
    kRank,
    kMPart,
    kMerge,
    kXc,
    kRepack,
    kNumPhases
};
static_assert(kNumPhases <= 128, "two 64-lane rounds find a ticket's phase");

constexpr bool is_global(uint32_t ph) { return ph >= kFbPlan && ph <= kFbEmit; }
// The first phases after Step 1(a): a column whose prefix sort left it
// unsorted waits there for the whole fallback chain.  (constexpr: usable in
// device code too.)
constexpr bool after_fallback(uint32_t ph) { return ph == kRank || ph == kMPart || ph == kMerge; }

// The plan of one batch.  Device copies of base, pmap, cum and gcum are what
// the kernel reads; the host keeps them to size the launch.
struct Plan {
    uint32_t ncols = 0;
    std::vector<uint32_t> base;  // kNumPhases + 1: first ticket of each phase; base[kNumPhases] = total
    std::vector<uint32_t> pmap;  // kNumPhases x (ncols + 1): prefix of the columns' item counts (per-column phases)
    std::vector<uint32_t> cum;   // ncols x kNumPhases: the column's items in per-column phases before ph
    std::vector<uint32_t> gcum;  // kNumPhases: items of global phases before ph
    uint32_t emit_total = 0;     // items of phase kEmit over all columns
    uint32_t fb_total = 0;       // items of all global phases
    uint32_t total() const { return base[kNumPhases]; }
};

// counts: ncols x kNumPhases item counts (entries of global phases ignored);
// gcount: kNumPhases counts of the global phases (others ignored).
// Returns false if the tickets would not fit in 32 bits.
inline bool build_plan(uint32_t ncols, const std::vector<uint32_t> &counts,
                       const std::vector<uint32_t> &gcount, Plan &P) {
    P.ncols = ncols;
    P.base.assign(kNumPhases + 1, 0);
    P.pmap.assign((size_t)kNumPhases * (ncols + 1), 0);
    P.cum.assign((size_t)ncols * kNumPhases, 0);
    P.gcum.assign(kNumPhases, 0);
    P.emit_total = 0;
    P.fb_total = 0;
    uint64_t t = 0, g = 0;
    std::vector<uint64_t> col(ncols, 0);
    for (uint32_t ph = 0; ph < kNumPhases; ph++) {
        P.base[ph] = (uint32_t)t;
        if (is_global(ph)) {
            P.gcum[ph] = (uint32_t)g;
            g += gcount[ph];
            t += gcount[ph];
        } else {
            uint64_t acc = 0;
            for (uint32_t j = 0; j < ncols; j++) {
                const uint32_t n = counts[(size_t)j * kNumPhases + ph];
                P.pmap[(size_t)ph * (ncols + 1) + j] = (uint32_t)acc;
                P.cum[(size_t)j * kNumPhases + ph] = (uint32_t)col[j];
                acc += n;
                col[j] += n;
                if (ph == kEmit) P.emit_total += n;
            }
            P.pmap[(size_t)ph * (ncols + 1) + ncols] = (uint32_t)acc;
            t += acc;
        }
        if (t >= (1ull << 32) - 1) return false;
    }
    P.base[kNumPhases] = (uint32_t)t;
    P.fb_total = (uint32_t)g;
    return true;
}

// What an item needs before it runs: the column counter's target (per-column
// phases), the global counter's target (global phases: kFbPlan waits for
// the emit counter, the others for the fallback counter).
struct Item {
    uint32_t phase, col, index;  // index: the item's number inside its (phase, column), or inside a global phase
};

// Decode ticket k (< total): the phase is the last one whose base is <= k;
// the column is the last one whose prefix entry is <= the offset in the phase.
inline Item decode(const Plan &P, uint32_t k) {
    uint32_t ph = 0;
    while (ph + 1 < kNumPhases && P.base[ph + 1] <= k) ph++;
    // empty phases share their base with the next one: take the last
    // phase whose range contains k
    const uint32_t off = k - P.base[ph];
    if (is_global(ph)) return Item{ph, 0, off};
    const uint32_t *m = &P.pmap[(size_t)ph * (P.ncols + 1)];
    uint32_t lo = 0, hi = P.ncols;  // m[lo] <= off < m[hi]
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) / 2;
        if (m[mid] <= off)
            lo = mid;
        else
            hi = mid;
    }
    return Item{ph, lo, off - m[lo]};
}

}  // namespace mcq
