// sort.hpp -- Step 1(a) on the GPU: the delta dictionary U_D and the index
// of every delta row in it (Sections 5.1 and 5.3, modified Step 1(a)).
//
// The paper walks the leaves of a CSB+ tree kept beside the delta; here the
// delta is a plain append-order array, so the sorted order comes from radix
// passes over (value, row) pairs with 8-bit digits, one digit per pass:
//   hist_tile      one read of the delta: histograms of every digit position
//   hist_scan_col  exclusive digit offsets per position; flags positions where
//                  every value has the same digit (those passes only copy);
//                  picks the positions of the prefix passes
//   per pass:  sort_up_tile    per-tile digit counts (digit-major)
//              sort_scan_digit per-digit exclusive scan over tiles
//              sort_down_tile  stable rank inside the tile (wave ballots),
//                              staging through LDS, coalesced scatter
//
// One to three global passes over the most significant varying digits (as
// many as it takes for runs of about 32 values on average, judged from the
// histograms; all three when the top digit shows a few heavily repeated
// values) leave the values ordered by their leading bytes ("prefix"), in
// runs of equal prefix.
// window_sort_tile then sorts every tile in LDS by the whole value: each run
// of equal prefix inside the tile is ordered.  window_seam_tile finishes the
// runs that cross a tile seam: such a run, if it is short, is ranked as a
// whole; if it is long, both of its sides are already ordered and only the
// pair across the seam needs checking.  A tile or seam that meets a long run
// out of order flags it at once, and emit_tile checks every adjacent pair;
// either way (heavy duplicates, clustered values) the full LSD sort over
// every digit runs after the emit (its launches return at once otherwise)
// and emit runs again.
//
// emit_tile marks run heads of the sorted values, numbers them with a
// cross-tile prefix, writes U_D and scatters each row's index (the paper's
// tuple-id update).  Equal values collapse, so row order inside a run is
// irrelevant; the passes are stable anyway, as LSD radix sort needs.
//
// Every function handles one tile of one column (ColDesc) and takes its LDS
// from the caller, so one launch can serve tiles of many columns.
#pragma once

#include "common.hpp"

namespace mc {

template <class T>
struct SortCfg;
template <>
struct SortCfg<TU32> { static constexpr int kItems = 8; };
template <>
struct SortCfg<TU64> { static constexpr int kItems = 8; };
template <>
struct SortCfg<TS16> { static constexpr int kItems = 6; };

template <class T>
__host__ __device__ constexpr int sort_tile() { return kBlock * SortCfg<T>::kItems; }

constexpr int kHistChunk = 4096;  // delta values per workgroup in hist_tile
// Copies of a column's digit histograms that hist_tile's workgroups add
// into (workgroup b into copy b % kGhCopies) and hist_scan_col sums: the
// global atomic adds on each counter then come from 1/kGhCopies of the
// workgroups.
constexpr int kGhCopies = 8;

// Runs of equal prefix longer than this are not ordered by the windows (they
// keep their place if already ordered, else the full sort takes over).
constexpr uint32_t kRunLimit = 256;

// Buffers of pass p (selects, not indexing, so the descriptor stays in registers).
__device__ __forceinline__ void *kbuf(const ColDesc &C, int i) { return (i & 1) ? C.keys1 : C.keys0; }
__device__ __forceinline__ uint32_t *vbuf(const ColDesc &C, int i) { return (i & 1) ? C.vals1 : C.vals0; }
__device__ __forceinline__ const void *pass_src(const ColDesc &C, int p) {
    return p == 0 ? C.sort_src : kbuf(C, p - 1);
}
// Number of values the radix passes sort: the delta rows, or the distinct
// values counted on the device when Step 1(a) hashes first.
__device__ __forceinline__ uint64_t sort_n(const ColDesc &C) {
    return C.sort_n ? min<uint64_t>(*C.sort_n, C.nd) : C.nd;
}

// Source and destination of one radix pass, and its digit position (< 0:
// the pass only copies).
struct PassIO {
    int p;
    const void *src;
    const uint32_t *vsrc;  // null: the rows are the identity
    void *kdst;
    uint32_t *vdst;
};
// Pass p of the full LSD sort (every digit position, least significant first).
__device__ __forceinline__ PassIO lsd_io(const ColDesc &C, int p) {
    PassIO io;
    io.p = C.trivial[p] ? -1 : p;
    io.src = pass_src(C, p);
    io.vsrc = p == 0 ? C.drow : vbuf(C, p - 1);  // pass 0: the payload (null: the position)
    io.kdst = kbuf(C, p);
    io.vdst = vbuf(C, p);
    return io;
}
// Slot s (0 .. kPrefixSlots - 1) of the prefix sort.  Used slots are the
// last ones, their digit positions rising; the last slot ends in the buffers
// the last LSD pass writes (keys1 / vals1) and copies there if no digit
// varies.  An unused slot (p == kPassSkip) does nothing.
constexpr int kPassCopy = -1, kPassSkip = -2;
__device__ __forceinline__ PassIO prefix_io(const ColDesc &C, int s) {
    PassIO io;
    const int p = (int)C.sflags[kSfPrefix + s] - 1;
    const bool first = s == 0 || C.sflags[kSfPrefix + s - 1] == 0;
    const bool to1 = ((kPrefixSlots - 1 - s) & 1) == 0;  // slots alternate, the last into keys1
    io.p = p >= 0 ? p : (s == kPrefixSlots - 1 ? kPassCopy : kPassSkip);
    io.src = first ? C.sort_src : (to1 ? C.keys0 : C.keys1);
    io.vsrc = first ? C.drow : (to1 ? C.vals0 : C.vals1);
    io.kdst = to1 ? C.keys1 : C.keys0;
    io.vdst = to1 ? C.vals1 : C.vals0;
    return io;
}

// ---- LDS layouts -------------------------------------------------------------

template <class T>
struct HistSmem { uint32_t h[T::kBytes * 256]; };

template <class T>
struct DownSmem {
    typename T::K keys[sort_tile<T>()];
    uint32_t vals[sort_tile<T>()];
    uint32_t wcnt[kWaves][256];
    uint32_t dex[256];   // exclusive digit offset inside the tile
    uint32_t gpos[256];  // global position of the digit's first key
    uint32_t tmp[kWaves];
};

// ---- histograms of all digit positions in one read ----------------------

template <class T>
__device__ __forceinline__ void hist_tile(const ColDesc &C, uint32_t blk, char *smem) {
    constexpr int P = T::kBytes;
    HistSmem<T> &S = *reinterpret_cast<HistSmem<T> *>(smem);
    for (int i = threadIdx.x; i < P * 256; i += kBlock) S.h[i] = 0;
    __syncthreads();
    const uint64_t b0 = (uint64_t)blk * kHistChunk;
    const uint64_t n = sort_n(C);
    if (b0 >= n) return;  // past the values (hashing left fewer than the rows)
    // eight loads in flight per thread, then their counts
    constexpr int kBatch = 8;
    static_assert(kHistChunk % (kBatch * kBlock) == 0, "whole batches");
    for (int h = 0; h < kHistChunk / kBlock; h += kBatch) {
        typename T::K k[kBatch];
#pragma unroll
        for (int q = 0; q < kBatch; q++) {  // unguarded (clamped): no load waits for another
            const uint64_t i = b0 + (uint64_t)(h + q) * kBlock + threadIdx.x;
            k[q] = T::load(C.sort_src, i < n ? i : n - 1);
        }
#pragma unroll
        for (int q = 0; q < kBatch; q++) {
            const uint64_t i = b0 + (uint64_t)(h + q) * kBlock + threadIdx.x;
            if (i < n) {
#pragma unroll
                for (int p = 0; p < P; p++) atomicAdd(&S.h[p * 256 + T::digit(k[q], p)], 1u);
            }
        }
    }
    __syncthreads();
    uint32_t *gh = C.gh + (uint64_t)(blk % kGhCopies) * (P * 256);
    for (int i = threadIdx.x; i < P * 256; i += kBlock)
        if (S.h[i]) atomicAdd(&gh[i], S.h[i]);
}

template <class T>
__device__ __forceinline__ void hist_scan_col(const ColDesc &C, char *smem) {
    constexpr int P = T::kBytes;
    uint32_t *tmp = reinterpret_cast<uint32_t *>(smem);
    uint32_t *ndig = tmp + kWaves;  // distinct digits per position
    uint32_t *maxc = ndig + 16;     // count of the most frequent digit per position
    const uint64_t n = sort_n(C);
    // one wave per digit position at a time, lane l holding digits 4l..4l+3:
    // a wave scan and no block barrier per position
    const int lane = lane_id();
    for (int p = wave_id(); p < P; p += kWaves) {
        uint32_t v[4], run = 0, nz = 0, mx = 0;
#pragma unroll
        for (int q = 0; q < 4; q++) {
            v[q] = 0;
#pragma unroll
            for (int c = 0; c < kGhCopies; c++) v[q] += C.gh[(c * P + p) * 256 + 4 * lane + q];
        }
#pragma unroll
        for (int q = 0; q < 4; q++) {
            run += v[q];
            nz += v[q] ? 1u : 0u;
            mx = max(mx, v[q]);
            if (v[q] == n) C.trivial[p] = 1u;
        }
        uint32_t ex = wave_incl_scan(run) - run;
#pragma unroll
        for (int q = 0; q < 4; q++) {
            C.base[p * 256 + 4 * lane + q] = ex;
            ex += v[q];
        }
        nz = wave_sum(nz);
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) mx = max(mx, (uint32_t)__shfl_xor(mx, o, 64));
        if (lane == 0) {
            ndig[p] = nz;
            maxc[p] = mx;
        }
    }
    __syncthreads();  // the flags above, written by other threads of the block
    if (threadIdx.x == 0) {
        // prefix digits: the most significant varying positions, as many as
        // it takes (at most kPrefixSlots) for n / (product of their numbers
        // of distinct digits) <= the wanted run length.  If the top digit is
        // skewed (its most frequent value holds more than kRunLimit values
        // and more than twice the mean), a few values are heavily repeated:
        // a run of equal prefix then holds all copies of such a value, and
        // any other value sharing that prefix leaves a long run out of order
        // (the full sort); every slot is used, so that the prefix almost
        // never covers a second value.
        int pos[kPrefixSlots];
        int k = 0;
        double combos = 1.0;
        bool skewed = false;
        const double run = C.prefix_run ? (double)C.prefix_run : kPrefixRun;
        for (int p = P - 1; p >= 0 && k < kPrefixSlots; p--) {
            if (C.trivial[p]) continue;
            if (k == 0)
                skewed = maxc[p] > kRunLimit && (double)maxc[p] > 2.0 * (double)n / ndig[p];
            pos[k++] = p;
            combos *= (double)ndig[p];
            if ((double)n <= combos * run && !skewed) break;
        }
        for (int s = 0; s < kPrefixSlots; s++) {
            const int from_top = kPrefixSlots - 1 - s;  // the last slot takes the top digit
            C.sflags[kSfPrefix + s] = from_top < k ? (uint32_t)(pos[from_top] + 1) : 0u;
        }
    }
}

// ---- loads of a tile's keys ---------------------------------------------
// Every load of a thread is issued before any loaded value is used: a digit
// or a select computed inside the guard of each load makes the compiler wait
// for that load before it issues the next, one memory round trip per item.

template <class K>
struct KeyVal {
    K k;
    uint32_t v;
};

// Keys (and their payloads) at tile positions base + 64 j, j < ITEMS, of the
// tile starting at b0 with tn values; entries past tn are zero.
template <class T, int ITEMS>
__device__ __forceinline__ void load_keys(const PassIO &io, uint64_t b0, uint32_t tn, uint32_t base,
                                          typename T::K (&key)[ITEMS], uint32_t (&val)[ITEMS]) {
#pragma unroll
    for (int j = 0; j < ITEMS; j++) {
        const uint32_t li = base + j * 64;
        key[j] = typename T::K{};
        if (li < tn) key[j] = T::load(io.src, b0 + li);
    }
    if (io.vsrc) {
#pragma unroll
        for (int j = 0; j < ITEMS; j++) {
            const uint32_t li = base + j * 64;
            val[j] = 0;
            if (li < tn) val[j] = io.vsrc[b0 + li];
        }
    } else {
#pragma unroll
        for (int j = 0; j < ITEMS; j++) val[j] = (uint32_t)(b0 + base + j * 64);
    }
}

// Count the digits p of the tile's values (positions b0 + j * kBlock +
// thread, below n) into the 256 LDS counters h.
template <class T>
__device__ __forceinline__ void count_digits(const PassIO &io, uint64_t b0, uint64_t n, int p, uint32_t *h) {
    constexpr int ITEMS = SortCfg<T>::kItems;
    typename T::K key[ITEMS];
#pragma unroll
    for (int j = 0; j < ITEMS; j++) {
        const uint64_t i = b0 + (uint64_t)j * kBlock + threadIdx.x;
        key[j] = typename T::K{};
        if (i < n) key[j] = T::load(io.src, i);
    }
#pragma unroll
    for (int j = 0; j < ITEMS; j++) {
        const uint64_t i = b0 + (uint64_t)j * kBlock + threadIdx.x;
        if (i < n) atomicAdd(&h[T::digit(key[j], p)], 1u);
    }
}

// ---- one pass: per-tile counts -------------------------------------------

template <class T>
__device__ __forceinline__ void sort_up_tile(const ColDesc &C, const PassIO &io, uint32_t t, char *smem) {
    const int p = io.p;
    if (p < 0) return;
    constexpr int TILE = sort_tile<T>();
    if ((uint64_t)t * TILE >= sort_n(C)) return;  // past the values: never scanned
    uint32_t *h = reinterpret_cast<uint32_t *>(smem);
    h[threadIdx.x] = 0;
    __syncthreads();
    const uint64_t b0 = (uint64_t)t * TILE;
    const uint64_t n = sort_n(C);
    count_digits<T>(io, b0, n, p, h);
    __syncthreads();
    C.tcount[(uint64_t)threadIdx.x * C.sort_tiles + t] = h[threadIdx.x];
}

// ---- one pass: per-digit exclusive scan over the tiles --------------------
// Adds the digit's global base, so tcount then holds the first output
// position of every (digit, tile).

template <class T>
__device__ __forceinline__ void sort_scan_digit(const ColDesc &C, const PassIO &io, uint32_t d, char *smem) {
    const int p = io.p;
    if (p < 0) return;
    uint32_t *tmp = reinterpret_cast<uint32_t *>(smem);
    uint32_t *row = C.tcount + (uint64_t)d * C.sort_tiles;
    uint32_t carry = C.base[p * 256 + d];
    // tiles holding values (fewer than sort_tiles when hashing removed duplicates)
    const uint32_t nt = (uint32_t)min<uint64_t>(C.sort_tiles,
                                                (sort_n(C) + sort_tile<T>() - 1) / sort_tile<T>());
    constexpr int kPer = 8;
    for (uint32_t c0 = 0; c0 < nt; c0 += kBlock * kPer) {
        uint32_t v[kPer];
        uint32_t sum = 0;
        const uint32_t i0 = c0 + threadIdx.x * kPer;
#pragma unroll
        for (int j = 0; j < kPer; j++) {
            v[j] = (i0 + j < nt) ? row[i0 + j] : 0u;
            sum += v[j];
        }
        uint32_t tot;
        uint32_t ex = block_excl_scan(sum, tmp, &tot) + carry;
#pragma unroll
        for (int j = 0; j < kPer; j++) {
            if (i0 + j < nt) row[i0 + j] = ex;
            ex += v[j];
        }
        carry += tot;
    }
}

// The same scan for a column of at most kSmallScanTiles tiles, in
// kSmallScanParts workgroups of 64 digits each: each wave takes 16 of them,
// with its lanes along the tiles (two chunks of 64, coalesced), and issues
// all its loads at once.  A launch then needs 4 workgroups per such column
// instead of 256.
constexpr uint32_t kSmallScanTiles = 128;
constexpr uint32_t kSmallScanParts = 4;

template <class T>
__device__ __forceinline__ void sort_scan_small(const ColDesc &C, const PassIO &io, uint32_t part) {
    const int p = io.p;
    if (p < 0) return;
    const int lane = lane_id(), wv = wave_id();
    const uint32_t nt = (uint32_t)min<uint64_t>(C.sort_tiles,
                                                (sort_n(C) + sort_tile<T>() - 1) / sort_tile<T>());
    constexpr int kRound = 256 / kSmallScanParts / kWaves;  // digits per wave
    const int d0 = (int)part * (256 / kSmallScanParts) + wv;
    {
        uint32_t v0[kRound], v1[kRound];
#pragma unroll
        for (int r = 0; r < kRound; r++) {
            const uint32_t *row = C.tcount + (uint64_t)(d0 + r * kWaves) * C.sort_tiles;
            v0[r] = (uint32_t)lane < nt ? row[lane] : 0u;
            v1[r] = (uint32_t)lane + 64 < nt ? row[lane + 64] : 0u;
        }
#pragma unroll
        for (int r = 0; r < kRound; r++) {
            const int d = d0 + r * kWaves;
            uint32_t *row = C.tcount + (uint64_t)d * C.sort_tiles;
            const uint32_t base = C.base[p * 256 + d];
            const uint32_t i0 = wave_incl_scan(v0[r]);
            const uint32_t tot0 = __shfl(i0, 63, 64);
            const uint32_t i1 = wave_incl_scan(v1[r]);
            if ((uint32_t)lane < nt) row[lane] = base + i0 - v0[r];
            if ((uint32_t)lane + 64 < nt) row[lane + 64] = base + tot0 + i1 - v1[r];
        }
    }
}

// ---- stable rank of a tile's digits ------------------------------------------
// Item j of thread (wave wv, lane) is tile entry wv * 64 * ITEMS + j * 64 +
// lane (each wave owns a contiguous chunk).  Returns in slot[j] the entry's
// position in the tile stably ordered by digit (entries >= tn are ignored),
// and leaves in dex[d] the tile's first position of digit d.  Lanes with the
// same digit find each other by intersecting the ballots of the digit's 8
// bits.  Every thread of the block must call it; it ends with a barrier.
template <int ITEMS>
__device__ __forceinline__ void rank_digits(const uint32_t (&dig)[ITEMS], uint32_t tn,
                                            uint32_t (*wcnt)[256], uint32_t *dex,
                                            uint32_t *tmp, uint32_t (&slot)[ITEMS]) {
    constexpr int WCHUNK = 64 * ITEMS;
    const int lane = lane_id(), wv = wave_id();
#pragma unroll
    for (int x = 0; x < kWaves; x++) wcnt[x][threadIdx.x] = 0;
    __syncthreads();
    uint32_t rank[ITEMS];
    const uint64_t lane_lt = (1ull << lane) - 1ull;
#pragma unroll
    for (int j = 0; j < ITEMS; j++) {
        const bool valid = (uint32_t)(wv * WCHUNK + j * 64 + lane) < tn;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; b++) {
            const bool bit = (dig[j] >> b) & 1u;
            const uint64_t bal = __ballot(bit);
            peers &= bit ? bal : ~bal;
        }
        uint32_t before = 0;
        if (valid) before = wcnt[wv][dig[j]];
        const uint32_t r = __popcll(peers & lane_lt);
        if (valid && r == 0) wcnt[wv][dig[j]] = before + (uint32_t)__popcll(peers);
        rank[j] = before + r;
    }
    __syncthreads();
    {
        // per digit: offsets of the waves (wave-major), then the tile prefix
        const int d = threadIdx.x;
        uint32_t run = 0;
#pragma unroll
        for (int x = 0; x < kWaves; x++) {
            const uint32_t c = wcnt[x][d];
            wcnt[x][d] = run;
            run += c;
        }
        uint32_t all;
        dex[d] = block_excl_scan(run, tmp, &all);
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < ITEMS; j++) slot[j] = dex[dig[j]] + wcnt[wv][dig[j]] + rank[j];
}

// ---- one pass: rank and scatter --------------------------------------------

template <class T>
__device__ __forceinline__ void sort_down_tile(const ColDesc &C, const PassIO &io, uint32_t t, char *smem) {
    typedef typename T::K K;
    constexpr int ITEMS = SortCfg<T>::kItems;
    constexpr int TILE = sort_tile<T>();
    constexpr int WCHUNK = 64 * ITEMS;  // keys per wave, contiguous
    DownSmem<T> &S = *reinterpret_cast<DownSmem<T> *>(smem);

    const uint64_t b0 = (uint64_t)t * TILE;
    const uint64_t n = sort_n(C);
    if (b0 >= n) return;  // only when hashing left fewer values than rows
    const uint32_t tn = (uint32_t)min<uint64_t>(TILE, n - b0);
    const int p = io.p;
    if (p == kPassSkip) return;

    if (p < 0) {
        // every value has the same digit here: the stable order is unchanged
        // (every load of the thread first, then the stores)
        stage_all<ITEMS>(
            tn,
            [&](uint32_t i) {
                return KeyVal<K>{T::load(io.src, b0 + i),
                                 io.vsrc ? io.vsrc[b0 + i] : (uint32_t)(b0 + i)};
            },
            [&](uint32_t i, const KeyVal<K> &e) {
                T::store(io.kdst, b0 + i, e.k);
                io.vdst[b0 + i] = e.v;
            });
        return;
    }

    const int lane = lane_id(), wv = wave_id();
    K key[ITEMS];
    uint32_t val[ITEMS], dig[ITEMS], slot[ITEMS];
    load_keys<T, ITEMS>(io, b0, tn, wv * WCHUNK + lane, key, val);
#pragma unroll
    for (int j = 0; j < ITEMS; j++)
        dig[j] = wv * WCHUNK + j * 64 + lane < tn ? T::digit(key[j], p) : 0u;
    S.gpos[threadIdx.x] = C.tcount[(uint64_t)threadIdx.x * C.sort_tiles + t];
    rank_digits<ITEMS>(dig, tn, S.wcnt, S.dex, S.tmp, slot);

#pragma unroll
    for (int j = 0; j < ITEMS; j++) {
        if ((uint32_t)(wv * WCHUNK + j * 64 + lane) < tn) {
            S.keys[slot[j]] = key[j];
            S.vals[slot[j]] = val[j];
        }
    }
    __syncthreads();

    bool bad = false;
    for (uint32_t i = threadIdx.x; i < tn; i += kBlock) {
        const K k = S.keys[i];
        const uint32_t d = T::digit(k, p);
        const uint64_t pos = (uint64_t)S.gpos[d] + (i - S.dex[d]);
        if (pos < n) {  // always true for consistent counts; never write outside
            T::store(io.kdst, pos, k);
            io.vdst[pos] = S.vals[i];
        } else {
            bad = true;
        }
    }
    if (bad) flag_error(C.err, MC_DEVERR_DELTA_RANGE);
}

// ---- one pass in two launches ------------------------------------------------
// For a single column of at most kP2MaxTiles tiles, a prefix pass runs as
// two launches and no workgroup waits for another: sort_up2_tile writes its
// tile's digit counts (tile-major) and adds them into its group's sums
// (kP2Group consecutive tiles); sort_down2_tile finds every digit's first
// output position from the digit's global offset, the sums of the groups
// before its tile's group and the counts of the group's earlier tiles, then
// ranks and scatters as sort_down_tile.  (The three-launch form scans the
// counts in a launch of its own; the one-launch form chained the tiles by a
// look-back, whose cross-workgroup round trips measured slower than the
// extra launch.)
constexpr uint32_t kP2Group = 32;
constexpr uint32_t kP2MaxTiles = 4096;

__device__ __forceinline__ uint32_t *p2_gsum(const ColDesc &C, int slot) {
    return C.pgsum + (uint64_t)slot * ((C.sort_tiles + kP2Group - 1) / kP2Group) * 256;
}

template <class T>
__device__ __forceinline__ void sort_up2_tile(const ColDesc &C, const PassIO &io, int slot, uint32_t t,
                                              char *smem) {
    const int p = io.p;
    if (p < 0) return;
    constexpr int TILE = sort_tile<T>();
    const uint64_t n = sort_n(C);
    if ((uint64_t)t * TILE >= n) return;  // past the values: never read
    uint32_t *h = reinterpret_cast<uint32_t *>(smem);
    h[threadIdx.x] = 0;
    __syncthreads();
    const uint64_t b0 = (uint64_t)t * TILE;
    count_digits<T>(io, b0, n, p, h);
    __syncthreads();
    const uint32_t c = h[threadIdx.x];
    C.tcount[(uint64_t)t * 256 + threadIdx.x] = c;
    if (c) atomicAdd(&p2_gsum(C, slot)[(t / kP2Group) * 256 + threadIdx.x], c);
}

template <class T>
__device__ __forceinline__ void sort_down2_tile(const ColDesc &C, const PassIO &io, int slot, uint32_t t,
                                                char *smem) {
    typedef typename T::K K;
    constexpr int ITEMS = SortCfg<T>::kItems;
    constexpr int TILE = sort_tile<T>();
    constexpr int WCHUNK = 64 * ITEMS;
    DownSmem<T> &S = *reinterpret_cast<DownSmem<T> *>(smem);
    const int p = io.p;
    if (p < 0) {  // no digit varies (copy) or an unused slot
        sort_down_tile<T>(C, io, t, smem);
        return;
    }
    const uint64_t b0 = (uint64_t)t * TILE;
    const uint64_t n = sort_n(C);
    if (b0 >= n) return;
    const uint32_t tn = (uint32_t)min<uint64_t>(TILE, n - b0);
    const int lane = lane_id(), wv = wave_id();
    K key[ITEMS];
    uint32_t val[ITEMS], dig[ITEMS], slotv[ITEMS];
    load_keys<T, ITEMS>(io, b0, tn, wv * WCHUNK + lane, key, val);
#pragma unroll
    for (int j = 0; j < ITEMS; j++)
        dig[j] = wv * WCHUNK + j * 64 + lane < tn ? T::digit(key[j], p) : 0u;
    {
        // digit d's first position: its global offset, the groups before
        // this tile's group, the group's tiles before this one
        // (eight loads in flight per round: a plain loop would wait for each)
        const uint32_t d = threadIdx.x;
        const uint32_t g = t / kP2Group;
        const uint32_t *gs = p2_gsum(C, slot) + d;
        const uint32_t *tc = C.tcount + (uint64_t)g * kP2Group * 256 + d;
        const uint32_t nt = t - g * kP2Group;  // the group's tiles before t
        uint32_t pos = C.base[p * 256 + d];
        for (uint32_t x0 = 0; x0 < g; x0 += 8) {
            uint32_t v[8];
#pragma unroll
            for (uint32_t k = 0; k < 8; k++) v[k] = x0 + k < g ? gs[(x0 + k) * 256] : 0u;
#pragma unroll
            for (uint32_t k = 0; k < 8; k++) pos += v[k];
        }
        for (uint32_t x0 = 0; x0 < nt; x0 += 8) {
            uint32_t v[8];
#pragma unroll
            for (uint32_t k = 0; k < 8; k++) v[k] = x0 + k < nt ? tc[(x0 + k) * 256] : 0u;
#pragma unroll
            for (uint32_t k = 0; k < 8; k++) pos += v[k];
        }
        S.gpos[d] = pos;
    }
    rank_digits<ITEMS>(dig, tn, S.wcnt, S.dex, S.tmp, slotv);
#pragma unroll
    for (int j = 0; j < ITEMS; j++) {
        if ((uint32_t)(wv * WCHUNK + j * 64 + lane) < tn) {
            S.keys[slotv[j]] = key[j];
            S.vals[slotv[j]] = val[j];
        }
    }
    __syncthreads();
    bool bad = false;
    for (uint32_t i = threadIdx.x; i < tn; i += kBlock) {
        const K k = S.keys[i];
        const uint32_t d = T::digit(k, p);
        const uint64_t pos = (uint64_t)S.gpos[d] + (i - S.dex[d]);
        if (pos < n) {
            T::store(io.kdst, pos, k);
            io.vdst[pos] = S.vals[i];
        } else {
            bad = true;
        }
    }
    if (bad) flag_error(C.err, MC_DEVERR_DELTA_RANGE);
}

// ---- windows sorted in LDS after the prefix passes --------------------------
// window_sort_tile sorts [t*TILE, (t+1)*TILE) in place in keys1 / vals1.  The
// tile is already ordered by prefix, so only runs of equal prefix need
// ordering: a value's place in its run is the number of run members that
// are smaller (or equal and before it).  Runs longer than kRunLimit keep
// their place if already ordered (runs of one repeated value); a long run
// out of order (heavy duplicates among other values, clustered values)
// means the prefix sort cannot finish the job: the tile sets the "out of
// order" flag at once and leaves its values, and the full LSD sort after
// the emit starts over from the unsorted values.  window_seam_tile then
// handles the run crossing seam (t+1)*TILE, if any.

// The prefix of a value: its digits at the used prefix slots (pp[s] < 0: unused).
template <class T>
__device__ __forceinline__ uint32_t prefix_of(const typename T::K &k, const int (&pp)[kPrefixSlots]) {
    uint32_t v = 0;
#pragma unroll
    for (int s = 0; s < kPrefixSlots; s++)
        if (pp[s] >= 0) v = (v << 8) | T::digit(k, pp[s]);
    return v;
}

template <class T>
__device__ __forceinline__ void window_sort_tile(const ColDesc &C, uint32_t t, char *smem) {
    typedef typename T::K K;
    constexpr int ITEMS = SortCfg<T>::kItems;
    constexpr int TILE = sort_tile<T>();
    constexpr int NW = TILE / 64;  // words of the run-head mask
    DownSmem<T> &S = *reinterpret_cast<DownSmem<T> *>(smem);
    uint64_t *heads = reinterpret_cast<uint64_t *>(&S.wcnt[0][0]);  // NW words, counting path only
    const uint64_t n = sort_n(C);
    const uint64_t b0 = (uint64_t)t * TILE;
    if (b0 >= n) return;
    const uint32_t tn = (uint32_t)min<uint64_t>(TILE, n - b0);
    int pp[kPrefixSlots];
#pragma unroll
    for (int s = 0; s < kPrefixSlots; s++) pp[s] = (int)C.sflags[kSfPrefix + s] - 1;
    if (pp[kPrefixSlots - 1] < 0) return;  // no digit varies: every value is the same
    if (threadIdx.x == 0) S.tmp[0] = 0;  // "a long run is out of order"
    struct KV {
        K k;
        uint32_t v;
    };
    stage_all<ITEMS>(
        tn, [&](uint32_t x) { return KV{T::load(C.keys1, b0 + x), C.vals1[b0 + x]}; },
        [&](uint32_t x, const KV &e) {
            S.keys[x] = e.k;
            S.vals[x] = e.v;
        });
    __syncthreads();
    // run heads: bit i set where a run of equal prefix starts (positions past
    // the window count as heads, so every run ends inside the mask)
    const int lane = lane_id(), wv = wave_id();
#pragma unroll
    for (int j = 0; j < ITEMS; j++) {
        const uint32_t i = j * kBlock + wv * 64 + lane;
        bool h = true;
        if (i < tn && i > 0)
            h = prefix_of<T>(S.keys[i], pp) != prefix_of<T>(S.keys[i - 1], pp);
        const uint64_t bal = __ballot(h);
        if (lane == 0) heads[i / 64] = bal;
    }
    __syncthreads();

    uint32_t npos[ITEMS];
    bool disorder = false;
#pragma unroll
    for (int j = 0; j < ITEMS; j++) {
        const uint32_t i = j * kBlock + wv * 64 + lane;
        npos[j] = i;
        if (i >= tn) continue;
        // run [s, e) around i
        uint32_t w = i / 64;
        const uint32_t bit = i & 63u;
        uint64_t m = heads[w] & (bit == 63 ? ~0ull : ((2ull << bit) - 1ull));
        while (m == 0) m = heads[--w];  // position 0 is a head
        const uint32_t s = w * 64 + 63 - (uint32_t)__clzll((long long)m);
        w = i / 64;
        m = bit == 63 ? 0ull : (heads[w] & ~((2ull << bit) - 1ull));
        while (m == 0 && ++w < (uint32_t)NW) m = heads[w];
        const uint32_t e = m ? min<uint32_t>(w * 64 + (uint32_t)(__ffsll((long long)m) - 1), tn) : tn;
        const K k = S.keys[i];
        const typename T::N kn = T::norm(k);
        if (e - s - 1 > kRunLimit) {
            // long run: keeps its place if already in order
            if (i > s && T::lt(kn, T::norm(S.keys[i - 1]))) disorder = true;
            continue;
        }
        // one loop over the run (a wave runs as long as its longest run, once)
        uint32_t rank = 0;
#pragma unroll 4
        for (uint32_t q = s; q < e; q++) {
            const typename T::N o = T::norm(S.keys[q]);
            rank += (q < i ? T::le(o, kn) : T::lt(o, kn)) ? 1u : 0u;
        }
        npos[j] = s + rank;
    }
    if (disorder) S.tmp[0] = 1u;
    __syncthreads();
    if (S.tmp[0] != 0) {
        if (threadIdx.x == 0) C.sflags[kSfUnsorted] = 1u;  // the full sort takes over
        return;
    }
#pragma unroll
    for (int j = 0; j < ITEMS; j++) {
        const uint32_t i = j * kBlock + wv * 64 + lane;
        if (i < tn && npos[j] != i) {
            T::store(C.keys1, b0 + npos[j], S.keys[i]);
            C.vals1[b0 + npos[j]] = S.vals[i];
        }
    }
}

// The run of equal prefix crossing seam B = (t+1)*TILE, after every tile is
// sorted.  Values [B - kRunLimit - 1, B + kRunLimit + 1) are read: a run no
// longer than kRunLimit lies inside them and is ranked as a whole (its two
// sides were sorted separately); a longer run (it may leave the range,
// which then holds more than kRunLimit + 1 of its values) is in order iff
// the pair across the seam is, since each side is ordered or already
// flagged.  Seams are at least 1536 values apart, so the ranges of two
// seams never overlap.
template <class T>
__device__ __forceinline__ void window_seam_tile(const ColDesc &C, uint32_t t, char *smem) {
    typedef typename T::K K;
    constexpr int TILE = sort_tile<T>();
    static_assert(TILE >= 2 * (int)(kRunLimit + 1), "seam ranges must not overlap");
    DownSmem<T> &S = *reinterpret_cast<DownSmem<T> *>(smem);
    const uint64_t n = sort_n(C);
    const uint64_t B = (uint64_t)(t + 1) * TILE;
    if (B >= n) return;  // no seam inside the values
    int pp[kPrefixSlots];
#pragma unroll
    for (int s = 0; s < kPrefixSlots; s++) pp[s] = (int)C.sflags[kSfPrefix + s] - 1;
    if (pp[kPrefixSlots - 1] < 0) return;  // no digit varies: every value is the same
    const uint64_t lo = B - (kRunLimit + 1);  // B >= TILE > kRunLimit + 1
    const uint32_t m = (uint32_t)(min<uint64_t>(n, B + kRunLimit + 1) - lo);
    const uint32_t sb = kRunLimit + 1;  // index of B in the range
    if (threadIdx.x == 0) {
        S.tmp[0] = 0;  // run start: one past the last differing value before the seam
        S.tmp[1] = m;  // run end: the first differing value after it
    }
    struct KV {
        K k;
        uint32_t v;
    };
    constexpr int kSeamSlots = (2 * (kRunLimit + 1) + kBlock - 1) / kBlock;
    stage_all<kSeamSlots>(
        m, [&](uint32_t x) { return KV{T::load(C.keys1, lo + x), C.vals1[lo + x]}; },
        [&](uint32_t x, const KV &e) {
            S.keys[x] = e.k;
            S.vals[x] = e.v;
        });
    __syncthreads();
    const uint32_t pre = prefix_of<T>(S.keys[sb - 1], pp);
    if (prefix_of<T>(S.keys[sb], pp) != pre) return;  // no run crosses the seam (uniform)
    for (uint32_t i = threadIdx.x; i < m; i += kBlock) {
        if (prefix_of<T>(S.keys[i], pp) != pre) {
            if (i < sb)
                atomicMax(&S.tmp[0], i + 1);
            else
                atomicMin(&S.tmp[1], i);
        }
    }
    __syncthreads();
    const uint32_t s = S.tmp[0], e = S.tmp[1];
    if (e - s - 1 > kRunLimit) {
        // long run: its sides are ordered; check the pair across the seam
        if (threadIdx.x == 0 && T::lt(T::norm(S.keys[sb]), T::norm(S.keys[sb - 1])))
            C.sflags[kSfUnsorted] = 1u;
        return;
    }
    for (uint32_t i = s + threadIdx.x; i < e; i += kBlock) {
        const K k = S.keys[i];
        const typename T::N kn = T::norm(k);
        uint32_t rank = 0;
        for (uint32_t q = s; q < e; q++) {
            const typename T::N o = T::norm(S.keys[q]);
            rank += (q < i ? T::le(o, kn) : T::lt(o, kn)) ? 1u : 0u;
        }
        const uint32_t np = s + rank;
        if (np != i) {
            T::store(C.keys1, lo + np, k);
            C.vals1[lo + np] = S.vals[i];
        }
    }
}

// ---- run heads -> U_D and the delta rows' indices ---------------------------

// Sorted positions per thread of an emit tile: 1024 per tile, with the
// windows' 2 x 257 staged neighbours (2048 per tile measured slower: c2
// 0.581 -> 0.575 ms and c3 1.094 -> 1.072 ms at 1024, whose smaller LDS
// keeps more workgroups per CU for the latency-bound run ranking).
constexpr int kEmitItems = 4;
constexpr int kEmitTile = kBlock * kEmitItems;

template <class T>
struct EmitSmem {
    typename T::K keys[kEmitTile + 1];  // keys[0]: the value before the tile
    uint16_t head[kEmitTile];           // LDS slot of the tile's r-th run head
    uint32_t tile;
    uint32_t tmp[kWaves];
    uint64_t lb;  // look-back result
};

// again = false: the emit after the prefix sort, which also checks the
// order; again = true: the emit after the full LSD sort, only when that check
// failed (its own tile counter and prefix words).
template <class T, bool DIRECT = false>
__device__ __forceinline__ void emit_tile_at(const ColDesc &C, char *smem, bool again, uint32_t t);

template <class T>
__device__ __forceinline__ void emit_tile(const ColDesc &C, char *smem, bool again) {
    EmitSmem<T> &S = *reinterpret_cast<EmitSmem<T> *>(smem);
    if (again && C.sflags[kSfUnsorted] == 0) return;
    if (threadIdx.x == 0) S.tile = atomicAdd(&C.sflags[again ? kSfEmitTicket2 : kSfEmitTicket], 1u);
    __syncthreads();
    emit_tile_at<T>(C, smem, again, S.tile);
}

// Emit groups: emit_count_tile adds every tile's count of run heads into
// the sum of its group of kEmitGroup tiles.
constexpr uint32_t kEmitGroup = 64;

// Exclusive prefix of tile t over the per-tile counts cnt, from the sums of
// the groups before t's group (gsum) and the counts of the group's earlier
// tiles, all written by an earlier launch.  Wave 0 computes it into *out.
__device__ __forceinline__ void group_prefix(const uint32_t *cnt, const uint32_t *gsum, uint32_t t,
                                             uint32_t group, uint64_t *out) {
    if (wave_id() != 0) return;
    const uint32_t lane = lane_id(), g = t / group;
    uint64_t v = 0;
    for (uint32_t x = lane; x < g; x += 64) v += gsum[x];
    for (uint32_t j = g * group + lane; j < t; j += 64) v += cnt[j];
    v = wave_sum(v);
    if (lane == 0) *out = v;
}

// Emit tile t.  DIRECT = false: the sorted values are in keys1 / vals1 and t
// is a ticket below the number of emit tiles, taken in order (the tile's
// prefix comes from a look-back).  DIRECT = true: emit_count_tile has
// written the sorted values to keys0 / vals0 and the tiles' run-head counts
// and group sums, and t is the workgroup index.
template <class T, bool DIRECT>
__device__ __forceinline__ void emit_tile_at(const ColDesc &C, char *smem, bool again, uint32_t t) {
    typedef typename T::K K;
    EmitSmem<T> &S = *reinterpret_cast<EmitSmem<T> *>(smem);
    const void *keys = DIRECT ? C.keys0 : C.keys1;
    const uint32_t *rows = DIRECT ? C.vals0 : C.vals1;
    uint64_t *status = again ? C.emit_status2 : C.emit_status;
    if (DIRECT) group_prefix(C.ecnt, C.egsum, t, kEmitGroup, &S.lb);
    const uint64_t tb = (uint64_t)t * kEmitTile;
    // coalesced staging of the tile (and its predecessor value) in LDS: slot
    // x holds sorted position tb + x - 1 (zero where there is none; such
    // slots are never compared)
    constexpr int kStageSlots = (kEmitTile + 1 + kBlock - 1) / kBlock;
    stage_all<kStageSlots>(
        kEmitTile + 1,
        [&](uint32_t x) {  // clamped: the load never waits for a select
            const uint64_t i = tb + x;
            return T::load(keys, i >= 1 ? min<uint64_t>(i - 1, C.nd - 1) : 0);
        },
        [&](uint32_t x, const K &k) {
            const uint64_t i = tb + x;
            S.keys[x] = (i >= 1 && i - 1 < C.nd) ? k : K{};
        });
    __syncthreads();
    const uint64_t i0 = tb + (uint64_t)threadIdx.x * kEmitItems;
    const uint32_t l0 = threadIdx.x * kEmitItems;

    uint32_t head = 0;  // bit j: position i0 + j starts a new value
    bool unsorted = false;
#pragma unroll
    for (int j = 0; j < kEmitItems; j++) {
        const uint64_t i = i0 + j;
        if (i < C.nd) {
            const K k = S.keys[l0 + j + 1], prev = S.keys[l0 + j];
            const bool h = (i == 0) || !T::keq(k, prev);
            head |= (uint32_t)h << j;
            if (i > 0 && T::lt(T::norm(k), T::norm(prev))) unsorted = true;
        }
    }
    if (unsorted && !again && !DIRECT) C.sflags[kSfUnsorted] = 1u;
    const uint32_t cnt = __popc(head);
    uint32_t tot;
    const uint32_t ex = block_excl_scan(cnt, S.tmp, &tot);  // its barriers also publish S.lb
    if (!DIRECT) lookback_publish(status, t, tot);
    {
        uint32_t lo = ex;
#pragma unroll
        for (int j = 0; j < kEmitItems; j++)
            if ((head >> j) & 1u) S.head[lo++] = (uint16_t)(l0 + j + 1);
    }
    const uint64_t tile_prefix = DIRECT ? S.lb : lookback_resolve(status, t, tot, C.err, &S.lb);
    __syncthreads();  // head slots complete
    for (uint32_t r = threadIdx.x; r < tot; r += kBlock) {
        const uint64_t idx = tile_prefix + r;
        if (idx < C.nd) T::store(C.u_d, idx, S.keys[S.head[r]]);
    }
    uint64_t idx = tile_prefix + ex;  // heads seen so far, over the whole array
    bool bad = false;
    uint32_t rowv[kEmitItems];
#pragma unroll
    for (int j = 0; j < kEmitItems; j++) rowv[j] = i0 + j < C.nd ? rows[i0 + j] : 0u;
#pragma unroll
    for (int j = 0; j < kEmitItems; j++) {
        const uint64_t i = i0 + j;
        if (i < C.nd) {
            if ((head >> j) & 1u) idx++;
            const uint32_t row = rowv[j];
            if (row < C.nd && idx - 1 < C.nd)
                C.drank[row] = (uint32_t)(idx - 1);
            else
                bad = true;
        }
    }
    if (bad) flag_error(C.err, MC_DEVERR_DELTA_RANGE);
    const uint64_t tile_end = (uint64_t)(t + 1) * kEmitTile;
    if (threadIdx.x == 0 && tile_end >= C.nd && (uint64_t)t * kEmitTile < C.nd)
        *C.n_ud = tile_prefix + tot;
}

// ---- the windows folded into the emit ----------------------------------------
// The emit after the prefix sort does what window_sort_tile,
// window_seam_tile and emit_tile do one after the other, without a pass of
// its own for the windows.  Emit tile t needs the sorted values at its view,
// positions [tb - 1, tb + kEmitTile) (tb = t * kEmitTile; the first one for
// the run-head test at tb).  It stages the prefix-sorted values of the view
// and kWinPad more on each side, finds the runs of equal prefix among them
// and orders the view: a run of at most kRunLimit + 1 values that meets the
// view lies wholly inside the staged range and is ranked there; a longer run
// (also every run cut off by the staged range's ends, which are then longer
// than that) keeps its place, and the check of adjacent pairs finds it if it
// is out of order (the full sort then takes over).  Neighbouring tiles see
// the same runs around their common position, so they agree on the value
// there.  emit_count_tile (radix route) and emit_distinct_window_tile
// (hashing route) build on window_view.
constexpr int kWinPad = kRunLimit + 1;
constexpr int kEmitView = kEmitTile + 1;
constexpr int kEmitWin = kEmitView + 2 * kWinPad;  // values staged per tile
constexpr int kEmitWinWords = (kEmitWin + 63) / 64 + 1;  // run-head mask (+1: all heads past the end)
static_assert(kEmitWin <= 65536, "staged indices are 16-bit");

template <class T>
struct EmitWinSmem {
    typename T::N keys[kEmitWin];  // normalized: compared without conversion
    uint32_t vals[kEmitWin];
    uint64_t heads[kEmitWinWords];
    uint16_t perm[kEmitView];  // view position -> staged index of the value sorted there
    uint32_t tmp[kWaves];
};

// The prefix of a normalized value (as prefix_of).
template <class T>
__device__ __forceinline__ uint32_t nprefix_of(const typename T::N &k, const int (&pp)[kPrefixSlots]) {
    uint32_t v = 0;
#pragma unroll
    for (int s = 0; s < kPrefixSlots; s++)
        if (pp[s] >= 0) v = (v << 8) | T::ndigit(k, pp[s]);
    return v;
}

// Stage [lo, hi) = [vb - kWinPad, ve + kWinPad) clipped to [0, n) of the
// prefix-sorted values (keys1 / vals1) and order the view [vb, ve) inside
// its runs of equal prefix: perm[v] = staged index of the value at sorted
// position vb + v.  Returns lo.  Ends with a barrier.
template <class T>
__device__ __forceinline__ uint64_t window_view(const ColDesc &C, uint64_t n, uint64_t vb, uint64_t ve,
                                                EmitWinSmem<T> &S) {
    typedef typename T::N N;
    const uint64_t lo = vb > (uint64_t)kWinPad ? vb - kWinPad : 0;
    const uint32_t m = (uint32_t)(min<uint64_t>(n, ve + kWinPad) - lo);
    const uint32_t v0 = (uint32_t)(vb - lo), v1 = (uint32_t)(ve - lo);  // the view, staged indices
    constexpr int kSlots = (kEmitWin + kBlock - 1) / kBlock;
    stage_all<kSlots>(
        m, [&](uint32_t x) { return KeyVal<typename T::K>{T::load(C.keys1, lo + x), C.vals1[lo + x]}; },
        [&](uint32_t x, const KeyVal<typename T::K> &e) {
            S.keys[x] = T::norm(e.k);  // normalized once every load is in flight
            S.vals[x] = e.v;
        });
    int pp[kPrefixSlots];
#pragma unroll
    for (int s = 0; s < kPrefixSlots; s++) pp[s] = (int)C.sflags[kSfPrefix + s] - 1;
    // no digit varies: every value is the same, each one a run of its own
    const bool varies = pp[kPrefixSlots - 1] >= 0;
    __syncthreads();
    const int lane = lane_id();
    for (int w = wave_id(); w < kEmitWinWords; w += kWaves) {
        const uint32_t x = (uint32_t)w * 64 + lane;
        bool h = true;  // staged index 0 and everything past the staged values count as heads
        if (varies && x > 0 && x < m) h = nprefix_of<T>(S.keys[x], pp) != nprefix_of<T>(S.keys[x - 1], pp);
        const uint64_t bal = __ballot(h);
        if (lane == 0) S.heads[w] = bal;
    }
    __syncthreads();
    for (uint32_t x = threadIdx.x; x < m; x += kBlock) {
        uint32_t w = x / 64;
        const uint32_t bit = x & 63u;
        uint64_t hm = S.heads[w] & (bit == 63 ? ~0ull : ((2ull << bit) - 1ull));
        while (hm == 0) hm = S.heads[--w];  // staged index 0 is a head
        const uint32_t s = w * 64 + 63 - (uint32_t)__clzll((long long)hm);
        w = x / 64;
        hm = bit == 63 ? 0ull : (S.heads[w] & ~((2ull << bit) - 1ull));
        while (hm == 0) hm = S.heads[++w];  // the last word is all heads
        const uint32_t e = min<uint32_t>(w * 64 + (uint32_t)(__ffsll((long long)hm) - 1), m);
        if (e <= v0 || s >= v1) continue;  // the run misses the view
        uint32_t dest = x;
        if (e - s - 1 <= kRunLimit) {
            // stable rank in the run: the members before x that are <= it
            // and those after it that are < it, in one loop over the run
            // (its lanes then step through the run together)
            const N kn = S.keys[x];
            uint32_t rank = 0;
#pragma unroll 4
            for (uint32_t q = s; q < e; q++)
                rank += (q < x ? T::le(S.keys[q], kn) : T::lt(S.keys[q], kn)) ? 1u : 0u;
            dest = s + rank;
        }
        if (dest >= v0 && dest < v1) S.perm[dest - v0] = (uint16_t)x;
    }
    __syncthreads();
    return lo;
}

// The first half of the emit after the prefix sort: tile t orders its view
// (window_view), writes its positions' sorted values to keys0 / vals0,
// checks the order of adjacent pairs, counts its run heads and adds the
// count into its group's sum; emit_tile_at<T, true> then numbers the heads.
template <class T>
__device__ __forceinline__ void emit_count_tile(const ColDesc &C, uint32_t t, char *smem) {
    typedef typename T::N N;
    EmitWinSmem<T> &S = *reinterpret_cast<EmitWinSmem<T> *>(smem);
    const uint64_t n = C.nd;
    const uint64_t tb = (uint64_t)t * kEmitTile;
    if (tb >= n) return;  // the launch has one tile per kEmitTile values
    const uint64_t vb = tb ? tb - 1 : 0, ve = min<uint64_t>(n, tb + kEmitTile);
    window_view<T>(C, n, vb, ve, S);
    const uint32_t off = tb ? 1u : 0u;  // view index of position tb
    uint32_t cnt = 0;
    bool unsorted = false;
    for (uint32_t r = threadIdx.x; r < (uint32_t)(ve - tb); r += kBlock) {
        const uint64_t i = tb + r;
        const uint32_t v = off + r;
        const N k = S.keys[S.perm[v]];
        T::store(C.keys0, i, T::denorm(k));
        C.vals0[i] = S.vals[S.perm[v]];
        bool h = true;
        if (i > 0) {
            const N prev = S.keys[S.perm[v - 1]];
            h = !T::eq(k, prev);
            if (T::lt(k, prev)) unsorted = true;
        }
        cnt += h ? 1u : 0u;
    }
    if (unsorted) C.sflags[kSfUnsorted] = 1u;
    uint32_t tot;
    block_excl_scan(cnt, S.tmp, &tot);
    if (threadIdx.x == 0) {
        C.ecnt[t] = tot;
        if (tot) atomicAdd(&C.egsum[t / kEmitGroup], tot);
    }
}

}  // namespace mc
