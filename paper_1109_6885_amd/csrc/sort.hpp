// sort.hpp -- Step 1(a) on the GPU: the delta dictionary U_D and the index
// of every delta row in it (Sections 5.1 and 5.3, modified Step 1(a)).
//
// The paper walks the leaves of a CSB+ tree kept beside the delta; here the
// delta is a plain append-order array, so the sorted order comes from an LSD
// radix sort of (value, row) pairs with 8-bit digits, one digit per pass:
//   hist_tile      one read of the delta: histograms of every digit position
//   hist_scan_col  exclusive digit offsets per position; flags positions where
//                  every value has the same digit (those passes only copy)
//   per pass:  sort_up_tile    per-tile digit counts (digit-major)
//              sort_scan_digit per-digit exclusive scan over tiles
//              sort_down_tile  stable rank inside the tile (wave ballots),
//                              staging through LDS, coalesced scatter
// then emit_tile marks run heads of the sorted values, numbers them with a
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
__device__ void hist_tile(const ColDesc &C, uint32_t blk, char *smem) {
    constexpr int P = T::kBytes;
    HistSmem<T> &S = *reinterpret_cast<HistSmem<T> *>(smem);
    for (int i = threadIdx.x; i < P * 256; i += kBlock) S.h[i] = 0;
    __syncthreads();
    const uint64_t b0 = (uint64_t)blk * kHistChunk;
    const uint64_t n = sort_n(C);
    for (uint32_t j = threadIdx.x; j < kHistChunk; j += kBlock) {
        const uint64_t i = b0 + j;
        if (i < n) {
            typename T::K k = T::load(C.sort_src, i);
#pragma unroll
            for (int p = 0; p < P; p++) atomicAdd(&S.h[p * 256 + T::digit(k, p)], 1u);
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < P * 256; i += kBlock)
        if (S.h[i]) atomicAdd(&C.gh[i], S.h[i]);
}

template <class T>
__device__ void hist_scan_col(const ColDesc &C, char *smem) {
    constexpr int P = T::kBytes;
    uint32_t *tmp = reinterpret_cast<uint32_t *>(smem);
    const uint64_t n = sort_n(C);
    for (int p = 0; p < P; p++) {
        const uint32_t v = C.gh[p * 256 + threadIdx.x];
        uint32_t tot;
        const uint32_t ex = block_excl_scan(v, tmp, &tot);
        C.base[p * 256 + threadIdx.x] = ex;
        if (v == n) C.trivial[p] = 1u;
    }
}

// ---- one pass: per-tile counts -------------------------------------------

template <class T>
__device__ void sort_up_tile(const ColDesc &C, int p, uint32_t t, char *smem) {
    if (C.trivial[p]) return;
    constexpr int TILE = sort_tile<T>();
    if ((uint64_t)t * TILE >= sort_n(C)) return;  // past the values: never scanned
    uint32_t *h = reinterpret_cast<uint32_t *>(smem);
    h[threadIdx.x] = 0;
    __syncthreads();
    const uint64_t b0 = (uint64_t)t * TILE;
    const void *src = pass_src(C, p);
    const uint64_t n = sort_n(C);
#pragma unroll 4
    for (int j = 0; j < SortCfg<T>::kItems; j++) {
        const uint64_t i = b0 + (uint64_t)j * kBlock + threadIdx.x;
        if (i < n) atomicAdd(&h[T::digit(T::load(src, i), p)], 1u);
    }
    __syncthreads();
    C.tcount[(uint64_t)threadIdx.x * C.sort_tiles + t] = h[threadIdx.x];
}

// ---- one pass: per-digit exclusive scan over the tiles --------------------
// Adds the digit's global base, so tcount then holds the first output
// position of every (digit, tile).

template <class T>
__device__ void sort_scan_digit(const ColDesc &C, int p, uint32_t d, char *smem) {
    if (C.trivial[p]) return;
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

// ---- one pass: rank and scatter --------------------------------------------

template <class T>
__device__ void sort_down_tile(const ColDesc &C, int p, uint32_t t, char *smem) {
    typedef typename T::K K;
    constexpr int ITEMS = SortCfg<T>::kItems;
    constexpr int TILE = sort_tile<T>();
    constexpr int WCHUNK = 64 * ITEMS;  // keys per wave, contiguous
    DownSmem<T> &S = *reinterpret_cast<DownSmem<T> *>(smem);

    const uint64_t b0 = (uint64_t)t * TILE;
    const uint64_t n = sort_n(C);
    if (b0 >= n) return;  // only when hashing left fewer values than rows
    const uint32_t tn = (uint32_t)min<uint64_t>(TILE, n - b0);
    const void *src = pass_src(C, p);
    const uint32_t *vsrc = p == 0 ? nullptr : vbuf(C, p - 1);
    void *kdst = kbuf(C, p);
    uint32_t *vdst = vbuf(C, p);

    if (C.trivial[p]) {
        // every value has the same digit here: the stable order is unchanged
        for (uint32_t i = threadIdx.x; i < tn; i += kBlock) {
            T::store(kdst, b0 + i, T::load(src, b0 + i));
            vdst[b0 + i] = vsrc ? vsrc[b0 + i] : (uint32_t)(b0 + i);
        }
        return;
    }

    const int lane = lane_id(), wv = wave_id();
#pragma unroll
    for (int x = 0; x < kWaves; x++) S.wcnt[x][threadIdx.x] = 0;
    __syncthreads();

    K key[ITEMS];
    uint32_t val[ITEMS];
    uint32_t rank[ITEMS];
    uint32_t dig[ITEMS];
    const uint64_t lane_lt = (1ull << lane) - 1ull;
#pragma unroll
    for (int j = 0; j < ITEMS; j++) {
        const uint32_t li = wv * WCHUNK + j * 64 + lane;  // index inside the tile
        const bool valid = li < tn;
        if (valid) {
            key[j] = T::load(src, b0 + li);
            val[j] = vsrc ? vsrc[b0 + li] : (uint32_t)(b0 + li);
            dig[j] = T::digit(key[j], p);
        } else {
            dig[j] = 0;
        }
        // lanes with the same digit: intersect the ballots of its 8 bits
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; b++) {
            const bool bit = (dig[j] >> b) & 1u;
            const uint64_t bal = __ballot(bit);
            peers &= bit ? bal : ~bal;
        }
        uint32_t before = 0;
        if (valid) before = S.wcnt[wv][dig[j]];
        const uint32_t r = __popcll(peers & lane_lt);
        if (valid && r == 0) S.wcnt[wv][dig[j]] = before + (uint32_t)__popcll(peers);
        rank[j] = before + r;
    }
    __syncthreads();

    // per digit: offsets of the waves (wave-major), tile total, tile prefix
    {
        const int d = threadIdx.x;
        uint32_t run = 0;
#pragma unroll
        for (int x = 0; x < kWaves; x++) {
            const uint32_t c = S.wcnt[x][d];
            S.wcnt[x][d] = run;
            run += c;
        }
        uint32_t all;
        const uint32_t ex = block_excl_scan(run, S.tmp, &all);
        S.dex[d] = ex;
        S.gpos[d] = C.tcount[(uint64_t)d * C.sort_tiles + t];
    }
    __syncthreads();

#pragma unroll
    for (int j = 0; j < ITEMS; j++) {
        const uint32_t li = wv * WCHUNK + j * 64 + lane;
        if (li < tn) {
            const uint32_t slot = S.dex[dig[j]] + S.wcnt[wv][dig[j]] + rank[j];
            S.keys[slot] = key[j];
            S.vals[slot] = val[j];
        }
    }
    __syncthreads();

    bool bad = false;
    for (uint32_t i = threadIdx.x; i < tn; i += kBlock) {
        const K k = S.keys[i];
        const uint32_t d = T::digit(k, p);
        const uint64_t pos = (uint64_t)S.gpos[d] + (i - S.dex[d]);
        if (pos < n) {  // always true for consistent counts; never write outside
            T::store(kdst, pos, k);
            vdst[pos] = S.vals[i];
        } else {
            bad = true;
        }
    }
    if (bad) flag_error(C.err, MC_DEVERR_DELTA_RANGE);
}

// ---- run heads -> U_D and the delta rows' indices ---------------------------

constexpr int kEmitItems = 8;
constexpr int kEmitTile = kBlock * kEmitItems;

template <class T>
struct EmitSmem {
    typename T::K keys[kEmitTile + 1];  // keys[0]: the value before the tile
    uint32_t tile;
    uint32_t tmp[kWaves];
    uint64_t lb64[kWaves + 1];
    int lb32[kWaves];
};

template <class T>
__device__ void emit_tile(const ColDesc &C, char *smem) {
    typedef typename T::K K;
    EmitSmem<T> &S = *reinterpret_cast<EmitSmem<T> *>(smem);
    constexpr int P = T::kBytes;
    const void *keys = kbuf(C, P - 1);  // sorted values after the last pass
    const uint32_t *rows = vbuf(C, P - 1);
    if (threadIdx.x == 0) S.tile = atomicAdd(&C.counters[0], 1u);
    __syncthreads();
    const uint32_t t = S.tile;
    const uint64_t tb = (uint64_t)t * kEmitTile;
    // coalesced staging of the tile (and its predecessor value) in LDS
    for (uint32_t x = threadIdx.x; x <= (uint32_t)kEmitTile; x += kBlock) {
        const uint64_t i = tb + x;  // LDS slot x holds sorted position i - 1
        if (i >= 1 && i - 1 < C.nd) S.keys[x] = T::load(keys, i - 1);
    }
    __syncthreads();
    const uint64_t i0 = tb + (uint64_t)threadIdx.x * kEmitItems;
    const uint32_t l0 = threadIdx.x * kEmitItems;

    K k[kEmitItems];
    uint32_t head = 0;  // bit j: position i0 + j starts a new value
#pragma unroll
    for (int j = 0; j < kEmitItems; j++) {
        const uint64_t i = i0 + j;
        if (i < C.nd) {
            k[j] = S.keys[l0 + j + 1];
            const bool h = (i == 0) || !T::keq(k[j], S.keys[l0 + j]);
            head |= (uint32_t)h << j;
        }
    }
    const uint32_t cnt = __popc(head);
    uint32_t tot;
    const uint32_t ex = block_excl_scan(cnt, S.tmp, &tot);
    const uint64_t tile_prefix = lookback_block(C.emit_status, t, tot, C.err, S.lb64, S.lb32);
    uint64_t idx = tile_prefix + ex;  // heads seen so far, over the whole array
    bool bad = false;
#pragma unroll
    for (int j = 0; j < kEmitItems; j++) {
        const uint64_t i = i0 + j;
        if (i < C.nd) {
            if ((head >> j) & 1u) {
                if (idx < C.nd) T::store(C.u_d, idx, k[j]);
                idx++;
            }
            const uint32_t row = rows[i];
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

}  // namespace mc
