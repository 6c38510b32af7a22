// hash.hpp -- Step 1(a) for large deltas: deduplicate by hashing first, then
// radix-sort only the distinct values (Sections 5.1 and 5.3 ask for the
// sorted unique delta values and every row's index among them; the paper
// gets them from its CSB+ tree, which holds each value once).
//
//   hash_insert_tile   every row finds or claims its value's slot in an
//                      open-addressing table; the claiming row is the
//                      value's representative (rep[row] = representative);
//                      rows first meet their tile's equal values in LDS
//   compact_tile       representatives become the distinct list (dkeys):
//                      each tile reserves a range of it with one atomic add
//                      on *dcount (the list's length); dindex[rep] is a
//                      representative's position in it.  The list's order
//                      does not matter (it is sorted next), so tiles need no
//                      prefix over each other
//   (radix passes over dkeys, count read on the device)
//   emit_distinct_tile sorted position i holds distinct value i of U_D;
//                      drankd[distinct position] = i
//   rank_rows_tile     drank[row] = drankd[dindex[rep[row]]]
//
// The same two kernels keep a delta index up to date as rows are appended
// (rows [hrow0, nd) of the delta, a batch at a time: the table, the
// representatives and the distinct list persist between batches, and the
// batch's new distinct values are added to the list), so that a merge can
// start from the distinct list.
//
// A slot holds (representative row + 1) and is written once, by one
// compare-and-swap from zero.  Slots are read with device-coherent loads:
// the compare-and-swap takes effect beyond the per-XCD L2, so a plain load
// could keep returning a cached zero and send every later row of a frequent
// value into a (serialized) compare-and-swap on the same slot.  Probing is
// linear and bounded by the table size, a power of two of at least twice
// the rows.
#pragma once

#include "sort.hpp"

namespace mc {

__device__ __forceinline__ uint64_t mix64(uint64_t x) {
    // MurmurHash3's 64-bit finalizer "fmix64" (Austin Appleby, public
    // domain): xor-shift / multiply rounds with its published constants
    x ^= x >> 33;
    x *= 0xff51afd7ed558ccdull;
    x ^= x >> 33;
    x *= 0xc4ceb9fe1a85ec53ull;
    x ^= x >> 33;
    return x;
}
__device__ __forceinline__ uint64_t hash_key(uint32_t k) { return mix64(k); }
__device__ __forceinline__ uint64_t hash_key(uint64_t k) { return mix64(k); }
__device__ __forceinline__ uint64_t hash_key(Raw16 k) { return mix64(k.a ^ mix64(k.b)); }

// Delta rows per hashing tile: 1024 (at 2048 the tile's LDS held 3
// workgroups per CU instead of 6, and its global probes, a few random
// round trips each, had less company to hide them: c3 1.072 -> 1.054 ms).
constexpr int kHashItems = 4;
constexpr int kHashTile = kBlock * kHashItems;
constexpr int kLocalSlots = 2 * kHashTile;  // LDS table of the tile's first occurrences

template <class T>
struct HashSmem {
    // the tile's values; once the global probes are done, the same bytes
    // hold the representative row of every first occurrence (u32 each)
    typename T::K keys[kHashTile];
    uint32_t slot[kLocalSlots];  // tile-local index + 1 of a value's first occurrence
    uint16_t lrep[kHashTile];    // first occurrence inside the tile of each row's value
};
static_assert(kHashTile <= 65536, "tile-local indices are 16-bit");

// A slot of the global table changes once, from 0 to its representative's
// row + 1, by an atomic compare-and-swap; a non-zero slot never changes
// again within a merge.  So a slot is read with a plain load, which may hit
// a cache: a non-zero value read anywhere is final, and a zero (perhaps
// stale) only leads to the compare-and-swap, whose returned value is
// authoritative.  (Reading every slot with a device-scope atomic load made
// the probes of a skewed delta's frequent values, which every tile repeats,
// queue on the same few words at the device's coherence point.)

// Find or claim the slot of `key` in the global table, probing from slot h
// on (`done` slots of its probe sequence already seen); returns the
// representative row, or `row` itself if it claimed the slot.
template <class T>
__device__ __forceinline__ uint32_t global_rep(const ColDesc &C, typename T::K key, uint32_t row,
                                               uint64_t h, uint64_t done, bool *ok) {
    for (uint64_t probe = done; probe <= C.hmask; probe++) {
        uint32_t s = C.htab[h];
        if (s == 0) {
            s = atomicCAS(&C.htab[h], 0u, row + 1u);
            if (s == 0) return row;  // claimed: this row represents its value
        }
        const uint32_t r = s - 1u;
        if (T::keq(T::load(C.delta, r), key)) return r;
        h = (h + 1) & C.hmask;
    }
    *ok = false;
    return row;
}

// Rows of one tile: equal values inside the tile first meet in an LDS table,
// so only the first occurrence of each value probes the global table (a
// frequent value then costs one global probe per tile, not one per row).
template <class T>
__device__ __forceinline__ void hash_insert_tile(const ColDesc &C, uint64_t t, char *smem) {
    typedef typename T::K K;
    HashSmem<T> &S = *reinterpret_cast<HashSmem<T> *>(smem);
    const uint64_t r0 = C.hrow0 + t * kHashTile;
    if (r0 >= C.nd) return;
    const uint32_t tn = (uint32_t)min<uint64_t>(kHashTile, C.nd - r0);
    for (uint32_t i = threadIdx.x; i < (uint32_t)kLocalSlots; i += kBlock) S.slot[i] = 0;
    stage_all<kHashItems>(
        tn, [&](uint32_t x) { return T::load(C.delta, r0 + x); },
        [&](uint32_t x, const K &k) { S.keys[x] = k; });
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < tn; i += kBlock) {
        const K key = S.keys[i];
        uint32_t h = (uint32_t)(hash_key(key) >> 20) & (kLocalSlots - 1);
        uint32_t first = i;
        for (int probe = 0; probe < kLocalSlots; probe++) {
            uint32_t sl = S.slot[h];
            if (sl == 0) {
                sl = atomicCAS(&S.slot[h], 0u, i + 1u);
                if (sl == 0) break;  // first occurrence inside the tile
            }
            if (T::keq(S.keys[sl - 1u], key)) {
                first = sl - 1u;
                break;
            }
            h = (h + 1) & (kLocalSlots - 1);
        }
        S.lrep[i] = (uint16_t)first;
    }
    __syncthreads();
    // Global probes of the first occurrences.  A thread's (up to
    // kHashItems) probes advance together, one memory round trip at a time
    // (slot loads, then claims of empty slots, then the representatives'
    // values), so their latencies overlap; the rare probe that meets another
    // value continues alone along its probe sequence.
    bool ok = true;
    K kk[kHashItems];
    uint64_t hh[kHashItems];
    uint32_t sv[kHashItems], res[kHashItems];
    uint32_t live = 0;  // bit j: item j is a first occurrence still probing
#pragma unroll
    for (int j = 0; j < kHashItems; j++) {
        const uint32_t i = j * kBlock + threadIdx.x;
        res[j] = 0;
        if (i < tn && S.lrep[i] == i) {
            kk[j] = S.keys[i];
            hh[j] = hash_key(kk[j]) & C.hmask;
            live |= 1u << j;
        }
    }
#pragma unroll
    for (int j = 0; j < kHashItems; j++)
        if ((live >> j) & 1u) sv[j] = C.htab[hh[j]];  // plain: see the note above global_rep
#pragma unroll
    for (int j = 0; j < kHashItems; j++)
        if (((live >> j) & 1u) && sv[j] == 0)
            sv[j] = atomicCAS(&C.htab[hh[j]], 0u, (uint32_t)(r0 + j * kBlock + threadIdx.x) + 1u);
    // sv[j] == 0 now means the claim succeeded
    K rk[kHashItems];
#pragma unroll
    for (int j = 0; j < kHashItems; j++) {
        if (((live >> j) & 1u) && sv[j] == 0) {
            res[j] = (uint32_t)(r0 + j * kBlock + threadIdx.x);
            live &= ~(1u << j);
        }
    }
#pragma unroll
    for (int j = 0; j < kHashItems; j++)
        if ((live >> j) & 1u) rk[j] = T::load(C.delta, sv[j] - 1u);
#pragma unroll
    for (int j = 0; j < kHashItems; j++) {
        if ((live >> j) & 1u) {
            if (T::keq(rk[j], kk[j])) {
                res[j] = sv[j] - 1u;
            } else {  // another value holds the slot: go on alone
                res[j] = global_rep<T>(C, kk[j], (uint32_t)(r0 + j * kBlock + threadIdx.x),
                                       (hh[j] + 1) & C.hmask, 1, &ok);
            }
        }
    }
    __syncthreads();  // every thread is done reading the values
    uint32_t *grep = reinterpret_cast<uint32_t *>(S.keys);
    uint32_t nrep = 0;  // rows of this thread that became representatives
#pragma unroll
    for (int j = 0; j < kHashItems; j++) {
        const uint32_t i = j * kBlock + threadIdx.x;
        if (i < tn && S.lrep[i] == i) {
            grep[i] = res[j];
            nrep += res[j] == (uint32_t)(r0 + i) ? 1u : 0u;
        }
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < tn; i += kBlock) C.rep[r0 + i] = grep[S.lrep[i]];
    if (!ok) flag_error(C.err, MC_DEVERR_DELTA_RANGE);
    if (C.hcnt) {  // the tile's count of representatives, for the compaction's positions
        nrep = wave_sum(nrep);
        uint32_t *wsum = S.slot;  // the local table is no longer read
        __syncthreads();
        if (lane_id() == 0) wsum[wave_id()] = nrep;
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t tot = 0;
#pragma unroll
            for (int w = 0; w < kWaves; w++) tot += wsum[w];
            C.hcnt[t] = tot;
            if (tot) atomicAdd(&C.hgsum[t / kEmitGroup], tot);
        }
    }
}

struct CompactSmem {
    uint32_t tmp[kWaves];
    uint64_t base;  // the tile's first position in the distinct list
    uint64_t pre;   // representatives of the tiles before it (per-tile counts)
};

// The compaction's tile t covers the rows of hashing tile t, whose count of
// representatives (hcnt[t]) gives it its place in the list.
constexpr int kCompactItems = kHashItems;
constexpr int kCompactTile = kBlock * kCompactItems;
static_assert(kCompactTile == kHashTile, "compaction tile t takes hashing tile t's count");

// With per-tile counts (C.hcnt, a merge's own hashing) the tile's range
// starts after the representatives of the tiles before it, so the list is
// in row order and no workgroup waits on a shared counter (one atomic add
// per tile on a single word serializes the tiles); the last tile writes the
// count.  A delta index appends its batches' values at *dcount with one
// atomic add per tile.  With C.drow the list's payload is each value's
// representative row; else dindex[rep] holds the value's position.
template <class T>
__device__ __forceinline__ void compact_tile(const ColDesc &C, uint64_t t, char *smem) {
    CompactSmem &S = *reinterpret_cast<CompactSmem *>(smem);
    if (C.hcnt) group_prefix(C.hcnt, C.hgsum, (uint32_t)t, kEmitGroup, &S.pre);
    const uint64_t r0 = C.hrow0 + t * kCompactTile + (uint64_t)threadIdx.x * kCompactItems;
    // every load first (clamped, unguarded), then the comparisons: a
    // comparison inside each load's guard waits for that load
    uint32_t rv[kCompactItems];
#pragma unroll
    for (int j = 0; j < kCompactItems; j++) {
        const uint64_t row = r0 + j;
        rv[j] = C.rep[row < C.nd ? row : (uint64_t)C.nd - 1];
    }
    uint32_t flags = 0;
#pragma unroll
    for (int j = 0; j < kCompactItems; j++) {
        const uint64_t row = r0 + j;
        if (row < C.nd && rv[j] == (uint32_t)row) flags |= 1u << j;
    }
    uint32_t tot;
    const uint32_t ex = block_excl_scan((uint32_t)__popc(flags), S.tmp, &tot);  // also publishes S.pre
    if (threadIdx.x == 0) {
        if (C.hcnt) {
            S.base = S.pre;
            if ((t + 1) * kCompactTile >= C.nd - C.hrow0) *C.dcount = S.pre + tot;  // the last tile
        } else {
            S.base = tot ? atomicAdd(reinterpret_cast<unsigned long long *>(C.dcount),
                                     (unsigned long long)tot)
                         : 0;
        }
    }
    __syncthreads();
    uint64_t pos = S.base + ex;
    bool full = false;
    typename T::K kv[kCompactItems];
#pragma unroll
    for (int j = 0; j < kCompactItems; j++)  // the representatives' values, all loads first
        if ((flags >> j) & 1u) kv[j] = T::load(C.delta, r0 + j);
#pragma unroll
    for (int j = 0; j < kCompactItems; j++) {
        if ((flags >> j) & 1u) {
            const uint64_t row = r0 + j;
            if (pos < C.nd_max) {  // the distinct list's capacity
                T::store(C.dkeys, pos, kv[j]);
                if (C.drow)
                    C.drow[pos] = (uint32_t)row;
                else
                    C.dindex[row] = (uint32_t)pos;
            } else {
                full = true;
            }
            pos++;
        }
    }
    if (full) flag_error(C.err, MC_DEVERR_DELTA_RANGE);
}

// After the radix passes over the distinct values: every sorted position
// starts a new value.  again: as for emit_tile (the run after the full LSD
// sort, only when the first run found the order wrong).
template <class T>
__device__ __forceinline__ void emit_distinct_tile(const ColDesc &C, uint64_t t, bool again) {
    if (again && C.sflags[kSfUnsorted] == 0) return;
    const void *keys = C.keys1;  // sorted values (both sorts end in keys1 / vals1)
    const uint32_t *rows = C.vals1;
    const uint64_t n = sort_n(C);
    const uint64_t dlim = C.drow ? C.nd : n;  // payload: a representative row, or a list position
    bool bad = false, unsorted = false;
    typedef typename T::K K;
    K k[kEmitItems], kp[kEmitItems];
    uint32_t d[kEmitItems];
#pragma unroll
    for (int j = 0; j < kEmitItems; j++) {  // every load first
        const uint64_t i = t * kEmitTile + (uint64_t)j * kBlock + threadIdx.x;
        if (i < n) {
            k[j] = T::load(keys, i);
            kp[j] = i > 0 ? T::load(keys, i - 1) : K{};
            d[j] = rows[i];
        }
    }
#pragma unroll
    for (int j = 0; j < kEmitItems; j++) {
        const uint64_t i = t * kEmitTile + (uint64_t)j * kBlock + threadIdx.x;
        if (i >= n) break;
        // distinct values: strictly increasing
        if (i > 0 && !T::lt(T::norm(kp[j]), T::norm(k[j]))) unsorted = true;
        T::store(C.u_d, i, k[j]);
        if (d[j] < dlim)
            C.drankd[d[j]] = (uint32_t)i;
        else
            bad = true;
    }
    if (bad) flag_error(C.err, MC_DEVERR_DELTA_RANGE);
    if (unsorted && !again) C.sflags[kSfUnsorted] = 1u;
    if (t == 0 && threadIdx.x == 0) *C.n_ud = n;
}

// emit_distinct_tile with the windows folded in (window_view): the
// view of tile t is ordered inside its runs of equal prefix in LDS.
template <class T>
__device__ __forceinline__ void emit_distinct_window_tile(const ColDesc &C, uint64_t t, char *smem) {
    typedef typename T::N N;
    EmitWinSmem<T> &S = *reinterpret_cast<EmitWinSmem<T> *>(smem);
    const uint64_t n = sort_n(C);
    const uint64_t tb = t * kEmitTile;
    if (tb >= n) return;  // the launch is sized for every delta row; fewer values are distinct
    const uint64_t vb = tb ? tb - 1 : 0, ve = min<uint64_t>(n, tb + kEmitTile);
    window_view<T>(C, n, vb, ve, S);
    const uint32_t off = tb ? 1u : 0u;  // view index of position tb
    bool bad = false, unsorted = false;
    for (uint32_t r = threadIdx.x; r < (uint32_t)(ve - tb); r += kBlock) {
        const uint64_t i = tb + r;
        const uint32_t v = off + r;
        const N k = S.keys[S.perm[v]];
        // distinct values: strictly increasing
        if (i > 0 && !T::lt(S.keys[S.perm[v - 1]], k)) unsorted = true;
        T::store(C.u_d, i, T::denorm(k));
        const uint32_t d = S.vals[S.perm[v]];
        if (d < (C.drow ? C.nd : n))  // payload: a representative row, or a list position
            C.drankd[d] = (uint32_t)i;
        else
            bad = true;
    }
    if (bad) flag_error(C.err, MC_DEVERR_DELTA_RANGE);
    if (unsorted) C.sflags[kSfUnsorted] = 1u;
    if (t == 0 && threadIdx.x == 0) *C.n_ud = n;
}

__device__ __forceinline__ void rank_rows_tile(const ColDesc &C, uint64_t t) {
    const uint64_t n = sort_n(C);
    bool bad = false;
    if (C.drow) {
        // the emit wrote every distinct value's rank at its representative
        // row: two rounds of gathers (representative, its rank)
        uint32_t v[kHashItems];
#pragma unroll
        for (int j = 0; j < kHashItems; j++) {
            const uint64_t row = t * kHashTile + (uint64_t)j * kBlock + threadIdx.x;
            v[j] = row < C.nd ? C.rep[row] : 0xffffffffu;
        }
#pragma unroll
        for (int j = 0; j < kHashItems; j++) {
            const uint64_t row = t * kHashTile + (uint64_t)j * kBlock + threadIdx.x;
            if (row < C.nd && v[j] >= C.nd) bad = true;
            v[j] = v[j] < C.nd ? C.drankd[v[j]] : 0u;
        }
#pragma unroll
        for (int j = 0; j < kHashItems; j++) {
            const uint64_t row = t * kHashTile + (uint64_t)j * kBlock + threadIdx.x;
            if (row < C.nd) C.drank[row] = v[j];
        }
        if (bad) flag_error(C.err, MC_DEVERR_DELTA_RANGE);
        return;
    }
    // three rounds of gathers (representative, its distinct position, that
    // position's rank), each with all of the thread's loads in flight
    uint32_t v[kHashItems];
#pragma unroll
    for (int j = 0; j < kHashItems; j++) {
        const uint64_t row = t * kHashTile + (uint64_t)j * kBlock + threadIdx.x;
        v[j] = row < C.nd ? C.rep[row] : 0xffffffffu;
    }
#pragma unroll
    for (int j = 0; j < kHashItems; j++) v[j] = v[j] < C.nd ? C.dindex[v[j]] : 0xffffffffu;
#pragma unroll
    for (int j = 0; j < kHashItems; j++) {
        const uint64_t row = t * kHashTile + (uint64_t)j * kBlock + threadIdx.x;
        if (row < C.nd && v[j] >= n) bad = true;
        v[j] = v[j] < n ? C.drankd[v[j]] : 0u;
    }
#pragma unroll
    for (int j = 0; j < kHashItems; j++) {
        const uint64_t row = t * kHashTile + (uint64_t)j * kBlock + threadIdx.x;
        if (row < C.nd) C.drank[row] = v[j];
    }
    if (bad) flag_error(C.err, MC_DEVERR_DELTA_RANGE);
}

}  // namespace mc
