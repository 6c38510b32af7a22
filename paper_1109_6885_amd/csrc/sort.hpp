// sort.hpp -- Step 1(a) on the GPU: the delta dictionary U_D and the index
// of every delta row in it (Sections 5.1 and 5.3, modified Step 1(a)).
//
// The paper walks the leaves of a CSB+ tree kept beside the delta; here the
// delta is a plain append-order array, so the sorted order comes from an LSD
// radix sort of (value, row) pairs with 8-bit digits, one digit per pass:
//   k_hist_all   one read of the delta: histograms of every digit position
//   k_hist_scan  exclusive digit offsets per position; flags positions where
//                every value has the same digit (those passes only copy)
//   per pass:  k_sort_up    per-tile digit counts (digit-major)
//              k_sort_scan  per-digit exclusive scan over tiles
//              k_sort_down  stable rank inside the tile (wave ballots),
//                           staging through LDS, coalesced scatter
// then k_emit marks run heads of the sorted values, numbers them with a
// cross-tile prefix, writes U_D and scatters each row's index (the paper's
// tuple-id update).  Equal values collapse, so row order inside a run is
// irrelevant; the passes are stable anyway, as LSD radix sort needs.
#pragma once

#include "common.hpp"

namespace mc {

template <class T>
struct SortCfg;
template <>
struct SortCfg<TU32> { static constexpr int kItems = 16; };
template <>
struct SortCfg<TU64> { static constexpr int kItems = 12; };
template <>
struct SortCfg<TS16> { static constexpr int kItems = 8; };

template <class T>
__host__ __device__ constexpr int sort_tile() { return kBlock * SortCfg<T>::kItems; }

struct SortJob {
    const void *src;    // raw delta values (input of pass 0)
    void *keys[2];      // ping-pong value buffers
    uint32_t *vals[2];  // ping-pong row buffers
    uint32_t n;         // delta rows
    uint32_t ntiles;    // ceil(n / tile)
    uint32_t *gh;       // [passes][256] global digit histograms (zeroed)
    uint32_t *base;     // [passes][256] exclusive digit offsets
    uint32_t *trivial;  // [passes] 1 if every value has the same digit (zeroed)
    uint32_t *tcount;   // [256][ntiles] per-tile digit counts, then offsets
    uint32_t *err;
};

// Buffers of pass p (selects, not indexing, so the job stays in registers).
__device__ __forceinline__ void *kbuf(const SortJob &J, int i) { return (i & 1) ? J.keys[1] : J.keys[0]; }
__device__ __forceinline__ uint32_t *vbuf(const SortJob &J, int i) {
    return (i & 1) ? J.vals[1] : J.vals[0];
}
template <class T>
__device__ __forceinline__ const void *pass_src(const SortJob &J, int p) {
    return p == 0 ? J.src : kbuf(J, p - 1);
}

// ---- histograms of all digit positions in one read ----------------------

template <class T>
__global__ __launch_bounds__(kBlock) void k_hist_all(SortJob J) {
    constexpr int P = T::kBytes;
    __shared__ uint32_t s_h[P * 256];
    for (int i = threadIdx.x; i < P * 256; i += kBlock) s_h[i] = 0;
    __syncthreads();
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < J.n; i += stride) {
        typename T::K k = T::load(J.src, i);
#pragma unroll
        for (int p = 0; p < P; p++) atomicAdd(&s_h[p * 256 + T::digit(k, p)], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < P * 256; i += kBlock)
        if (s_h[i]) atomicAdd(&J.gh[i], s_h[i]);
}

template <class T>
__global__ __launch_bounds__(kBlock) void k_hist_scan(SortJob J) {
    constexpr int P = T::kBytes;
    __shared__ uint32_t s_tmp[kWaves];
    for (int p = 0; p < P; p++) {
        uint32_t v = J.gh[p * 256 + threadIdx.x];
        uint32_t tot;
        uint32_t ex = block_excl_scan(v, s_tmp, &tot);
        J.base[p * 256 + threadIdx.x] = ex;
        if (v == J.n) J.trivial[p] = 1u;
    }
}

// ---- one pass: per-tile counts -------------------------------------------

template <class T>
__global__ __launch_bounds__(kBlock) void k_sort_up(SortJob J, int p) {
    if (J.trivial[p]) return;
    constexpr int TILE = sort_tile<T>();
    __shared__ uint32_t s_h[256];
    s_h[threadIdx.x] = 0;
    __syncthreads();
    const uint32_t t = blockIdx.x;
    const uint64_t b0 = (uint64_t)t * TILE;
    const void *src = pass_src<T>(J, p);
#pragma unroll 4
    for (int j = 0; j < SortCfg<T>::kItems; j++) {
        uint64_t i = b0 + (uint64_t)j * kBlock + threadIdx.x;
        if (i < J.n) atomicAdd(&s_h[T::digit(T::load(src, i), p)], 1u);
    }
    __syncthreads();
    J.tcount[(uint64_t)threadIdx.x * J.ntiles + t] = s_h[threadIdx.x];
}

// ---- one pass: per-digit exclusive scan over the tiles --------------------
// One block per digit; adds the digit's global base so that tcount holds the
// first output position of (digit, tile).

template <class T>
__global__ __launch_bounds__(kBlock) void k_sort_scan(SortJob J, int p) {
    if (J.trivial[p]) return;
    __shared__ uint32_t s_tmp[kWaves];
    const uint32_t d = blockIdx.x;
    uint32_t *row = J.tcount + (uint64_t)d * J.ntiles;
    uint32_t carry = J.base[p * 256 + d];
    constexpr int kPer = 8;
    for (uint32_t c0 = 0; c0 < J.ntiles; c0 += kBlock * kPer) {
        uint32_t v[kPer];
        uint32_t sum = 0;
        const uint32_t i0 = c0 + threadIdx.x * kPer;
#pragma unroll
        for (int j = 0; j < kPer; j++) {
            v[j] = (i0 + j < J.ntiles) ? row[i0 + j] : 0u;
            sum += v[j];
        }
        uint32_t tot;
        uint32_t ex = block_excl_scan(sum, s_tmp, &tot) + carry;
#pragma unroll
        for (int j = 0; j < kPer; j++) {
            if (i0 + j < J.ntiles) row[i0 + j] = ex;
            ex += v[j];
        }
        carry += tot;
    }
}

// ---- one pass: rank and scatter --------------------------------------------

template <class T>
__global__ __launch_bounds__(kBlock) void k_sort_down(SortJob J, int p) {
    typedef typename T::K K;
    constexpr int ITEMS = SortCfg<T>::kItems;
    constexpr int TILE = sort_tile<T>();
    constexpr int WCHUNK = 64 * ITEMS;  // keys per wave, contiguous

    __shared__ K s_keys[TILE];
    __shared__ uint32_t s_vals[TILE];
    __shared__ uint32_t s_wcnt[kWaves][256];
    __shared__ uint32_t s_dex[256];   // exclusive digit offset inside the tile
    __shared__ uint32_t s_gpos[256];  // global position of the digit's first key
    __shared__ uint32_t s_tmp[kWaves];

    const uint32_t t = blockIdx.x;
    const uint64_t b0 = (uint64_t)t * TILE;
    const uint32_t tn = (uint32_t)min<uint64_t>(TILE, J.n - b0);
    const void *src = pass_src<T>(J, p);
    const uint32_t *vsrc = p == 0 ? nullptr : vbuf(J, p - 1);
    void *kdst = kbuf(J, p);
    uint32_t *vdst = vbuf(J, p);

    if (J.trivial[p]) {
        // every value has the same digit here: the stable order is unchanged
        for (uint32_t i = threadIdx.x; i < tn; i += kBlock) {
            T::store(kdst, b0 + i, T::load(src, b0 + i));
            vdst[b0 + i] = vsrc ? vsrc[b0 + i] : (uint32_t)(b0 + i);
        }
        return;
    }

    const int lane = lane_id(), wv = wave_id();
    s_wcnt[0][threadIdx.x] = 0;
    s_wcnt[1][threadIdx.x] = 0;
    s_wcnt[2][threadIdx.x] = 0;
    s_wcnt[3][threadIdx.x] = 0;
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
        if (valid) before = s_wcnt[wv][dig[j]];
        const uint32_t r = __popcll(peers & lane_lt);
        if (valid && r == 0) s_wcnt[wv][dig[j]] = before + (uint32_t)__popcll(peers);
        rank[j] = before + r;
    }
    __syncthreads();

    // per digit: offsets of the waves (wave-major), tile total, tile prefix
    {
        const int d = threadIdx.x;
        uint32_t c0 = s_wcnt[0][d], c1 = s_wcnt[1][d], c2 = s_wcnt[2][d], c3 = s_wcnt[3][d];
        s_wcnt[0][d] = 0;
        s_wcnt[1][d] = c0;
        s_wcnt[2][d] = c0 + c1;
        s_wcnt[3][d] = c0 + c1 + c2;
        const uint32_t tot = c0 + c1 + c2 + c3;
        uint32_t all;
        const uint32_t ex = block_excl_scan(tot, s_tmp, &all);
        s_dex[d] = ex;
        s_gpos[d] = J.tcount[(uint64_t)d * J.ntiles + t];
    }
    __syncthreads();

#pragma unroll
    for (int j = 0; j < ITEMS; j++) {
        const uint32_t li = wv * WCHUNK + j * 64 + lane;
        if (li < tn) {
            const uint32_t slot = s_dex[dig[j]] + s_wcnt[wv][dig[j]] + rank[j];
            s_keys[slot] = key[j];
            s_vals[slot] = val[j];
        }
    }
    __syncthreads();

    bool bad = false;
    for (uint32_t i = threadIdx.x; i < tn; i += kBlock) {
        const K k = s_keys[i];
        const uint32_t d = T::digit(k, p);
        const uint64_t pos = (uint64_t)s_gpos[d] + (i - s_dex[d]);
        if (pos < J.n) {  // always true for consistent counts; never write outside
            T::store(kdst, pos, k);
            vdst[pos] = s_vals[i];
        } else {
            bad = true;
        }
    }
    if (bad) flag_error(J.err, MC_DEVERR_DELTA_RANGE);
}

// ---- run heads -> U_D and the delta rows' indices ---------------------------

struct EmitJob {
    const void *keys;       // sorted values
    const uint32_t *rows;   // their rows
    uint32_t n;
    void *u_d;              // out: sorted unique values
    uint32_t *drank;        // out: index in u_d of every row
    uint64_t *n_ud;         // out: |U_D|
    uint64_t *status;       // per-tile prefix words (zeroed)
    uint32_t *counter;      // tile counter (zeroed)
    uint32_t *err;
};

constexpr int kEmitItems = 8;
constexpr int kEmitTile = kBlock * kEmitItems;

template <class T>
__global__ __launch_bounds__(kBlock) void k_emit(EmitJob J) {
    typedef typename T::K K;
    __shared__ uint32_t s_tile;
    __shared__ uint32_t s_tmp[kWaves];
    __shared__ uint64_t s_prefix;
    if (threadIdx.x == 0) s_tile = atomicAdd(J.counter, 1u);
    __syncthreads();
    const uint32_t t = s_tile;
    const uint64_t i0 = (uint64_t)t * kEmitTile + (uint64_t)threadIdx.x * kEmitItems;

    K k[kEmitItems];
    uint32_t head = 0;  // bit j: position i0 + j starts a new value
    K prev;
    if (i0 > 0 && i0 < J.n) prev = T::load(J.keys, i0 - 1);
#pragma unroll
    for (int j = 0; j < kEmitItems; j++) {
        const uint64_t i = i0 + j;
        if (i < J.n) {
            k[j] = T::load(J.keys, i);
            const bool h = (i == 0) || !T::keq(k[j], prev);
            head |= (uint32_t)h << j;
            prev = k[j];
        }
    }
    const uint32_t cnt = __popc(head);
    uint32_t tot;
    const uint32_t ex = block_excl_scan(cnt, s_tmp, &tot);
    if (wave_id() == 0) {
        const uint64_t pre = lookback_wave(J.status, t, tot, J.err);
        if (lane_id() == 0) s_prefix = pre;
    }
    __syncthreads();
    uint64_t idx = s_prefix + ex;  // heads seen so far, over the whole array
    bool bad = false;
#pragma unroll
    for (int j = 0; j < kEmitItems; j++) {
        const uint64_t i = i0 + j;
        if (i < J.n) {
            if ((head >> j) & 1u) {
                if (idx < J.n) T::store(J.u_d, idx, k[j]);
                idx++;
            }
            const uint32_t row = J.rows[i];
            if (row < J.n && idx - 1 < J.n)
                J.drank[row] = (uint32_t)(idx - 1);
            else
                bad = true;
        }
    }
    if (bad) flag_error(J.err, MC_DEVERR_DELTA_RANGE);
    const uint64_t tile_end = (uint64_t)(t + 1) * kEmitTile;
    if (threadIdx.x == 0 && tile_end >= J.n && (uint64_t)t * kEmitTile < J.n)
        *J.n_ud = s_prefix + tot;
}

}  // namespace mc
