// queue_model.cpp -- a CPU model of the persistent batched launch's work
// queue (paper_1109_6885_amd/csrc/queue.hpp and kn_persist): host threads
// play the workgroups and run the same protocol -- one ticket counter,
// the same decode (the 64-lane searches of the kernel emulated lane by lane
// and checked against the plain decode), the same wait targets on the same
// counters, relaxed atomics with fences where the kernel fences -- on random
// plans, with random delays between taking a ticket and running it.
//
// Checked: every item runs exactly once; when an item starts, every item it
// depends on has finished (the dependencies are written out here from the
// method's data flow, independently of the counters); the items of the two
// look-back phases (emit, merge) take per-column tickets and wait for the
// lower ones, as the kernel's look-back does; and every run ends (a watchdog
// reports a run that stops making progress as a deadlock).
//
// Usage: queue_model <seed> <plans>   (exit status 0: all plans passed)
#include <stdint.h>
#include <stdio.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <random>
#include <thread>
#include <vector>

#include "queue.hpp"

using mcq::kNumPhases;

namespace {

struct Run {
    const mcq::Plan *P;
    std::vector<uint8_t> unsorted;  // per column
    std::atomic<uint32_t> ticket{0}, emit_done{0}, fb_done{0};
    std::vector<std::atomic<uint32_t>> col_done;
    std::vector<std::atomic<uint32_t>> started, finished;  // per ticket
    // look-back phases: per (column, phase) ticket and per-ticket published flag
    std::vector<std::atomic<uint32_t>> lb_ticket;           // ncols x 2
    std::vector<std::vector<std::atomic<uint8_t>>> lb_pub;  // (ncols x 2) x items
    std::atomic<uint32_t> errors{0};
    std::atomic<uint64_t> progress{0};
    uint64_t delay_seed = 0;
    explicit Run(const mcq::Plan &p)
        : P(&p), col_done(p.ncols), started(p.total()), finished(p.total()), lb_ticket(2 * p.ncols),
          lb_pub(2 * p.ncols) {}
};

// The kernel's decode, lane by lane: the phase is the number of x in
// [1, kNumPhases) with base[x] <= k (two rounds of 64 lanes); the column is
// found by 64-ary narrowing of [lo, hi) over the phase's prefix map.
mcq::Item decode_lanes(const mcq::Plan &P, uint32_t k) {
    uint32_t ph = 0;
    for (uint32_t r = 0; r < 2; r++)
        for (uint32_t lane = 0; lane < 64; lane++) {
            const uint32_t x = r * 64 + lane;
            if (x >= 1 && x < kNumPhases && P.base[x] <= k) ph++;
        }
    const uint32_t off = k - P.base[ph];
    if (mcq::is_global(ph)) return mcq::Item{ph, 0, off};
    const uint32_t *m = &P.pmap[(size_t)ph * (P.ncols + 1)];
    uint32_t lo = 0, hi = P.ncols;
    while (hi - lo > 1) {
        const uint32_t step = (hi - lo + 63) / 64;
        uint32_t cnt = 0;
        for (uint32_t lane = 1; lane < 64; lane++) {
            const uint32_t x = lo + lane * step;
            if (x < hi && m[x] <= off) cnt++;
        }
        lo += cnt * step;
        hi = std::min(hi, lo + step);
    }
    return mcq::Item{ph, lo, off - m[lo]};
}

bool wait_ge(std::atomic<uint32_t> &c, uint32_t target) {
    auto t0 = std::chrono::steady_clock::now();
    while (c.load(std::memory_order_relaxed) < target) {
        std::this_thread::yield();
        if (std::chrono::steady_clock::now() - t0 > std::chrono::seconds(20)) return false;
    }
    std::atomic_thread_fence(std::memory_order_seq_cst);  // the kernel's acquire fence
    return true;
}

// The items item k depends on, by the data flow: for a per-column item, every
// item of its column in an earlier per-column phase (and, after the fallback,
// every global item if the column was unsorted); for a global item, every
// emit item (the first global phase) or every global item of an earlier
// global phase.
bool deps_finished(Run &R, uint32_t k, const mcq::Item &it) {
    const mcq::Plan &P = *R.P;
    const uint32_t total = P.total();
    for (uint32_t q = 0; q < total; q++) {
        if (q == k) continue;
        const mcq::Item d = mcq::decode(P, q);
        bool need = false;
        if (mcq::is_global(it.phase)) {
            if (it.phase == mcq::kFbPlan)
                need = d.phase == mcq::kEmit;
            else
                need = mcq::is_global(d.phase) && d.phase < it.phase;
        } else {
            need = !mcq::is_global(d.phase) && d.col == it.col && d.phase < it.phase;
            if (mcq::is_global(d.phase) && mcq::after_fallback(it.phase) && R.unsorted[it.col])
                need = true;
        }
        if (need && !R.finished[q].load(std::memory_order_relaxed)) return false;
    }
    return true;
}

void worker(Run &R, uint32_t id) {
    const mcq::Plan &P = *R.P;
    std::mt19937_64 rng(R.delay_seed * 7919 + id);
    std::uniform_int_distribution<int> d(0, 9);
    while (true) {
        const uint32_t k = R.ticket.fetch_add(1, std::memory_order_relaxed);
        if (k >= P.total()) break;
        const mcq::Item it = decode_lanes(P, k);
        const mcq::Item ref = mcq::decode(P, k);
        if (it.phase != ref.phase || it.col != ref.col || it.index != ref.index) R.errors++;
        if (d(rng) == 0) std::this_thread::sleep_for(std::chrono::microseconds(d(rng) * 50));
        bool ok = true;
        if (mcq::is_global(it.phase)) {
            ok = it.phase == mcq::kFbPlan ? wait_ge(R.emit_done, P.emit_total)
                                          : wait_ge(R.fb_done, P.gcum[it.phase]);
        } else {
            ok = wait_ge(R.col_done[it.col], P.cum[(size_t)it.col * kNumPhases + it.phase]);
            if (ok && mcq::after_fallback(it.phase) && R.unsorted[it.col])
                ok = wait_ge(R.fb_done, P.fb_total);
        }
        if (!ok) {
            R.errors += 1000;  // a wait that never ended: a deadlock
            return;
        }
        if (!deps_finished(R, k, it)) R.errors++;
        if (R.started[k].fetch_add(1) != 0) R.errors++;
        // the look-back phases: a per-column ticket, then a wait for the
        // predecessor's published prefix (held by a running worker)
        if (!mcq::is_global(it.phase) && (it.phase == mcq::kEmit || it.phase == mcq::kMerge)) {
            const size_t slot = 2 * (size_t)it.col + (it.phase == mcq::kMerge);
            const uint32_t e = R.lb_ticket[slot].fetch_add(1, std::memory_order_relaxed);
            if (e > 0) {
                auto t0 = std::chrono::steady_clock::now();
                while (!R.lb_pub[slot][e - 1].load(std::memory_order_relaxed)) {
                    std::this_thread::yield();
                    if (std::chrono::steady_clock::now() - t0 > std::chrono::seconds(20)) {
                        R.errors += 1000;
                        return;
                    }
                }
            }
            R.lb_pub[slot][e].store(1, std::memory_order_relaxed);
        }
        if (d(rng) < 2) std::this_thread::sleep_for(std::chrono::microseconds(d(rng) * 20));
        R.finished[k].store(1, std::memory_order_relaxed);
        std::atomic_thread_fence(std::memory_order_seq_cst);  // the kernel's release fence
        if (mcq::is_global(it.phase)) {
            R.fb_done.fetch_add(1, std::memory_order_relaxed);
        } else {
            R.col_done[it.col].fetch_add(1, std::memory_order_relaxed);
            if (it.phase == mcq::kEmit) R.emit_done.fetch_add(1, std::memory_order_relaxed);
        }
        R.progress++;
    }
}

// A random plan: columns with or without a delta, hashing or not, some
// unsorted; item counts like the library's (zero where a step does not run).
void random_plan(std::mt19937_64 &rng, mcq::Plan &P, std::vector<uint8_t> &unsorted) {
    const uint32_t ncols = 1 + (uint32_t)(rng() % 40);
    std::vector<uint32_t> counts((size_t)ncols * kNumPhases, 0), gcount(kNumPhases, 0);
    unsorted.assign(ncols, 0);
    uint32_t npass = 0;
    auto r = [&](uint32_t lo, uint32_t hi) { return lo + (uint32_t)(rng() % (hi - lo + 1)); };
    for (uint32_t j = 0; j < ncols; j++) {
        uint32_t *c = &counts[(size_t)j * kNumPhases];
        const bool delta = rng() % 5 != 0, hashed = delta && rng() % 4 == 0;
        if (delta) {
            const uint32_t tiles = r(1, 9);
            if (hashed) c[mcq::kHash] = c[mcq::kCompact] = c[mcq::kRank] = r(1, 6);
            c[mcq::kHist] = r(1, 4);
            c[mcq::kHScan] = 1;
            for (uint32_t k = 0; k < 9; k++) c[mcq::kPre0Up + k] = (k % 3 == 1) ? 4 : tiles;
            c[mcq::kWin0] = c[mcq::kWin1] = tiles;
            c[mcq::kEmit] = r(1, 5);
            unsorted[j] = rng() % 3 == 0;
            npass = std::max(npass, (uint32_t)(4u << (rng() % 3)));
        }
        if (rng() % 3 == 0) c[mcq::kMPart] = r(1, 3);
        c[mcq::kMerge] = r(1, 6);
        c[mcq::kXc] = r(0, 3);
        c[mcq::kRepack] = r(0, 12);
    }
    if (npass) {
        gcount[mcq::kFbPlan] = 2 * npass + 1;
        for (uint32_t p = 0; p < npass; p++)
            for (uint32_t k = 0; k < 3; k++) gcount[mcq::kFbPass0 + 3 * p + k] = r(1, 3);
        gcount[mcq::kFbEmit] = r(1, 3);
    }
    mcq::build_plan(ncols, counts, gcount, P);
}

}  // namespace

int main(int argc, char **argv) {
    const uint64_t seed = argc > 1 ? strtoull(argv[1], nullptr, 10) : 1;
    const int plans = argc > 2 ? atoi(argv[2]) : 50;
    std::mt19937_64 rng(seed);
    const uint32_t worker_counts[] = {1, 2, 3, 5, 16};
    int failures = 0;
    for (int p = 0; p < plans; p++) {
        mcq::Plan P;
        std::vector<uint8_t> unsorted;
        random_plan(rng, P, unsorted);
        for (uint32_t G : worker_counts) {
            Run R(P);
            R.unsorted = unsorted;
            R.delay_seed = seed * 1000003ull + (uint64_t)p * 31 + G;
            for (size_t s = 0; s < R.lb_pub.size(); s++) {
                const uint32_t ph = (s & 1) ? mcq::kMerge : mcq::kEmit;
                const uint32_t j = (uint32_t)(s / 2);
                const size_t n = P.pmap[(size_t)ph * (P.ncols + 1) + j + 1] -
                                 P.pmap[(size_t)ph * (P.ncols + 1) + j];
                R.lb_pub[s] = std::vector<std::atomic<uint8_t>>(n);
            }
            std::vector<std::thread> th;
            for (uint32_t w = 0; w < G; w++) th.emplace_back(worker, std::ref(R), w);
            for (auto &t : th) t.join();
            uint32_t ran = 0;
            for (uint32_t k = 0; k < P.total(); k++) ran += R.started[k].load() == 1;
            if (R.errors.load() || ran != P.total()) {
                fprintf(stderr, "plan %d (ncols %u, items %u) with %u workers: %u errors, %u of %u ran\n",
                        p, P.ncols, P.total(), G, R.errors.load(), ran, P.total());
                failures++;
            }
        }
    }
    printf("queue model: %d plans x %zu worker counts, %d failures\n", plans,
           sizeof(worker_counts) / sizeof(worker_counts[0]), failures);
    return failures ? 1 : 0;
}
