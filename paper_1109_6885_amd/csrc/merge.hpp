// merge.hpp -- Step 1(b) and Step 2(a) on the GPU (Sections 5.1, 5.3 and
// 6.2.1; Eq. 4): merge the sorted unique dictionaries U_M and U_D into U'
// and emit the translation tables X_M and X_D.
//
// The paper splits the merge among threads by quantiles of both inputs,
// merges each part with duplicate removal, counts the unique outputs per
// part, scans the counts and writes the final positions in a third phase.
// Here each workgroup owns a fixed range of the merged sequence (merge
// path: a binary search on the cross diagonal finds how many U_M entries
// fall before the range), merges it out of LDS, counts its unique values
// and gets its output offset from the tiles before it through a
// cross-workgroup prefix instead of a global barrier.
//
// Ties are resolved U_M first, so a value present in both dictionaries
// appears as U_M[i-1] immediately followed by U_D[j].  A merged element is
// new iff it does not equal that predecessor; the U_D copy of a shared value
// takes the index of the U_M copy (the rule "equal values get the same
// index in both tables").
//
// Each thread merges 8 (16-byte values: 4) consecutive merged positions
// once, remembering what every step took; the tile then publishes its count
// of new values, replays the steps into LDS (which input each output comes
// from, tile-relative X entries) while its predecessors finish, and once its
// offset is known writes U', X_M and X_D as contiguous runs (coalesced
// stores).
#pragma once

#include "common.hpp"

namespace mc {

// Merged positions per thread: 8 in the batched merge (many columns, mostly
// small: more, smaller tiles keep more workgroups per CU), 16 in a
// single-column merge of 4- and 8-byte values (one large merge: half the
// tiles, half the look-back; c2's dictionary merge 38 -> 28.5 us, while
// the 300-column batch measured 10.27 -> 10.43 ms with 16).  Half the tile
// for 16-byte values would fit four workgroups in one CU's LDS instead of
// two, but measured slower on a 10M-entry string dictionary (0.33 ms
// against 0.26 ms for the dictionary merge step): more tiles, more
// look-back.
template <class T>
struct MergeCfg {
    static constexpr int kItems = 8;         // batched
    static constexpr int kItemsSingle = 16;  // single column
};
template <>
struct MergeCfg<TS16> {
    static constexpr int kItems = 8;
    static constexpr int kItemsSingle = 8;
};
template <class T, int ITEMS = MergeCfg<T>::kItems>
__host__ __device__ constexpr int merge_tile() { return kBlock * ITEMS; }

constexpr uint32_t kStepA = 0, kStepNew = 1, kStepDup = 2;
constexpr uint32_t kFromB = 0x8000u;  // > any merge tile: marks an index into b

template <class T, int ITEMS = MergeCfg<T>::kItems>
struct MergeSmem {
    // the tile's inputs in one array (a tile holds na + nb <= merge_tile
    // entries): ab[0] = U_M[i0 - 1] (predecessor), ab[1 + x] = U_M[i0 + x]
    // for x < na ("a"), ab[na + 1 + y] = U_D[j0 + y] for y < nb ("b")
    typename T::N ab[merge_tile<T, ITEMS>() + 1];
    uint16_t src[merge_tile<T, ITEMS>()];  // output r of the tile: index in a, or kFromB | index in b
    int16_t xm[merge_tile<T, ITEMS>()];    // tile-relative U' index of a[1 + x]
    int16_t xd[merge_tile<T, ITEMS>()];    // tile-relative U' index of b[y] (-1: the tile before's last)
    uint32_t tile;
    uint32_t tmp[kWaves];
    uint64_t i0, i1;
    uint64_t lb;  // look-back result
};

// Number of U_M entries among the first k merged elements (ties: U_M first).
template <class T, class GetA, class GetB>
__device__ __forceinline__ uint64_t co_rank(uint64_t k, uint64_t a, uint64_t b, GetA A, GetB B) {
    uint64_t lo = k > b ? k - b : 0;
    uint64_t hi = k < a ? k : a;
    while (lo < hi) {
        const uint64_t mid = (lo + hi) >> 1;
        if (T::le(A(mid), B(k - 1 - mid)))
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

// The same co-rank found by one wave in about log64 rounds: each round the
// 64 lanes test 64 evenly spaced candidates of the remaining range at once
// (the predicate "A[i] <= B[k-1-i]" is true below the answer and false from
// it on), and the ballot narrows the range to one step.  Every lane returns
// the answer.  Used for the tile boundaries, where the arrays are in global
// memory and a sequential search would wait on ~20 dependent loads.
template <class T, class GetA, class GetB>
__device__ __forceinline__ uint64_t co_rank_wave(uint64_t k, uint64_t a, uint64_t b, GetA A,
                                                 GetB B) {
    uint64_t lo = k > b ? k - b : 0;
    uint64_t hi = k < a ? k : a;  // answer in [lo, hi]
    const int lane = lane_id();
    while (hi > lo) {
        const uint64_t span = hi - lo;  // candidates lo .. hi-1
        // lane l tests candidate lo + floor(span * (l + 1) / 65)  (< hi)
        const uint64_t step = span / 65, rem = span % 65;
        const uint64_t cand = lo + step * (lane + 1) + (rem * (lane + 1)) / 65;
        bool pred = false;  // true: the answer lies above cand
        if (cand < hi) pred = T::le(A(cand), B(k - 1 - cand));
        const uint64_t yes = __ballot(pred);
        // predicate is monotone in cand: the lanes that say "above" form a prefix
        const int nyes = __popcll(yes);
        const uint64_t new_lo = nyes ? (lo + step * nyes + (rem * nyes) / 65) + 1 : lo;
        const uint64_t new_hi = nyes < 64 ? lo + step * (nyes + 1) + (rem * (nyes + 1)) / 65 : hi;
        lo = new_lo;
        hi = new_hi < hi ? new_hi : hi;
        if (span <= 64) {
            // every candidate was tested: lo is the answer
            hi = lo;
        }
    }
    return lo;
}

// Tile boundaries ahead of the merge: wave q of the launch finds how many
// U_M entries precede merged position q * merge_tile (q = 0 .. tiles), so the
// merge tiles start without a search through global memory.  Each wave
// returns on its own; there is no barrier.
template <class T, int ITEMS = MergeCfg<T>::kItems>
__device__ __forceinline__ void merge_partition(const ColDesc &C, uint32_t blk) {
    const uint64_t q = (uint64_t)blk * kWaves + wave_id();
    const uint64_t a = C.n_um;
    const uint64_t b = min(*C.n_ud_in, C.nd_max);
    const uint64_t total = a + b;
    constexpr uint64_t TILE = merge_tile<T, ITEMS>();
    if (q > (total + TILE - 1) / TILE) return;
    const uint64_t k = min<uint64_t>(q * TILE, total);
    auto gA = [&](uint64_t i) { return T::norm(T::load(C.u_m, i)); };
    auto gB = [&](uint64_t j) { return T::norm(T::load(C.u_d, j)); };
    const uint64_t r = co_rank_wave<T>(k, a, b, gA, gB);
    if (lane_id() == 0) C.mbound[q] = r;
}

template <class T, int ITEMS = MergeCfg<T>::kItems>
__device__ __forceinline__ void merge_tile(const ColDesc &C, char *smem) {
    MergeSmem<T, ITEMS> &S = *reinterpret_cast<MergeSmem<T, ITEMS> *>(smem);
    if (threadIdx.x == 0) S.tile = atomicAdd(&C.counters[1], 1u);
    __syncthreads();
    const uint32_t t = S.tile;
    const uint64_t a = C.n_um;
    const uint64_t b = min(*C.n_ud_in, C.nd_max);  // never read past U_D's buffer
    const uint64_t cap = C.u_new_cap;
    const uint64_t total = a + b;
    const uint64_t k0 = (uint64_t)t * merge_tile<T, ITEMS>();
    if (k0 >= total) {
        if (t == 0 && threadIdx.x == 0) {  // nothing to merge at all
            C.result->new_dict_len = 0;
            C.result->new_bitwidth = 1;
            C.result->new_codes_words = (C.rows_total + 63) / 64;
            C.result->delta_dict_len = b;
        }
        return;
    }
    const uint64_t k1 = min<uint64_t>(k0 + merge_tile<T, ITEMS>(), total);
    auto gA = [&](uint64_t i) { return T::norm(T::load(C.u_m, i)); };
    auto gB = [&](uint64_t j) { return T::norm(T::load(C.u_d, j)); };
    uint64_t i0, i1;
    if (C.mbound) {  // tile boundaries found by merge_partition
        i0 = C.mbound[t];
        i1 = C.mbound[t + 1];
    } else {
        if (wave_id() == 0) {
            const uint64_t r = co_rank_wave<T>(k0, a, b, gA, gB);
            if (lane_id() == 0) S.i0 = r;
        } else if (wave_id() == 1) {
            const uint64_t r = co_rank_wave<T>(k1, a, b, gA, gB);
            if (lane_id() == 0) S.i1 = r;
        }
        __syncthreads();
        i0 = S.i0;
        i1 = S.i1;
    }
    // With both inputs strictly increasing the co-ranks grow with k and the
    // tile holds i1 - i0 U_M and j1 - j0 U_D entries.  Out-of-order inputs
    // can break that; then the tile is left empty (nothing is read or
    // written past the inputs) and the error word says why.
    const bool order_ok = i1 >= i0 && i1 - i0 <= k1 - k0;
    if (!order_ok && threadIdx.x == 0) flag_error(C.err, MC_DEVERR_ORDER);
    const uint64_t j0 = k0 - i0, j1 = order_ok ? k1 - i1 : j0;
    const uint32_t na = order_ok ? (uint32_t)(i1 - i0) : 0u, nb = (uint32_t)(j1 - j0);
    if (order_ok && nb == 0 && na > 0) {
        // U_M entries only (large dictionaries with small deltas are mostly
        // such tiles): U' continues U_M shifted by the tile's offset, X_M
        // counts on from it; no walk and no staging
        lookback_publish(C.merge_status, t, na);
        const uint64_t tile_prefix = lookback_resolve(C.merge_status, t, na, C.err, &S.lb);
        typedef typename T::K K;
        constexpr int kSlots = (merge_tile<T, ITEMS>() + kBlock - 1) / kBlock;
        K v[kSlots];
#pragma unroll
        for (int q = 0; q < kSlots; q++) {
            const uint32_t x = q * kBlock + threadIdx.x;
            if (x < na) v[q] = T::load(C.u_m, i0 + x);
        }
#pragma unroll
        for (int q = 0; q < kSlots; q++) {
            const uint32_t x = q * kBlock + threadIdx.x;
            if (x < na) {
                const uint64_t pos = tile_prefix + x;
                if (pos < cap) T::store(C.u_new, pos, v[q]);
                if (C.x_m) C.x_m[i0 + x] = (uint32_t)pos;
            }
        }
        if (threadIdx.x == 0 && k1 == total) {
            const uint64_t n = tile_prefix + na;
            const uint32_t w = code_width(n);
            C.result->new_dict_len = n;
            C.result->new_bitwidth = w;
            C.result->new_codes_words = (C.rows_total * w + 63) / 64;
            C.result->delta_dict_len = b;
        }
        return;
    }
    // stage a[0] = U_M[i0 - 1] (if any), a[1 + x] = U_M[i0 + x] and
    // b[y] = U_D[j0 + y]: the predecessor by thread 0, the rest as one range
    // of na + nb loads, all in flight before any value is normalized (a
    // normalization or select inside each load's guard makes the compiler
    // wait for that load before it issues the next)
    typedef typename T::N N;
    typedef typename T::K K;
    N *const sa = S.ab, *const sb = S.ab + na + 1;
    // every thread loads the predecessor's address (one request per wave),
    // unguarded so that nothing waits for it here; without a predecessor it
    // reads some valid entry and stores zero
    const K pred = T::load((i0 > 0 || a > 0) ? C.u_m : C.u_d, i0 > 0 ? i0 - 1 : 0);
    stage_all<merge_tile<T, ITEMS>() / kBlock>(
        na + nb,
        [&](uint32_t q) -> K { return q < na ? T::load(C.u_m, i0 + q) : T::load(C.u_d, j0 + (q - na)); },
        [&](uint32_t q, const K &v) { S.ab[q + 1] = T::norm(v); });
    if (threadIdx.x == 0) S.ab[0] = i0 > 0 ? T::norm(pred) : N{};
    __syncthreads();

    // this thread's slice of the tile's merged range
    const uint32_t len = na + nb;
    const uint32_t d0 = min<uint32_t>(threadIdx.x * ITEMS, len);
    const uint32_t d1 = min<uint32_t>(d0 + ITEMS, len);
    auto lA = [&](uint64_t i) { return sa[i + 1]; };
    auto lB = [&](uint64_t j) { return sb[j]; };
    const uint32_t ia0 = (uint32_t)co_rank<T>(d0, na, nb, lA, lB);
    const uint32_t jb0 = d0 - ia0;

    // one merge walk: 2 bits per step (kStepA: U_M element, kStepNew: new U_D
    // element, kStepDup: U_D element equal to its U_M predecessor)
    const uint32_t nsteps = d1 - d0;
    uint32_t steps = 0, cnt = 0;
    {
        uint32_t ia = ia0, jb = jb0;
        for (uint32_t s = 0; s < nsteps; s++) {
            const bool take_a = jb >= nb || (ia < na && T::le(sa[ia + 1], sb[jb]));
            uint32_t kind;
            if (take_a) {
                kind = kStepA;
                ia++;
            } else {
                kind = ((i0 + ia > 0) && T::eq(sa[ia], sb[jb])) ? kStepDup : kStepNew;
                jb++;
            }
            steps |= kind << (2 * s);
            cnt += kind != kStepDup;
        }
    }
    uint32_t tot;
    const uint32_t ex = block_excl_scan(cnt, S.tmp, &tot);
    lookback_publish(C.merge_status, t, tot);

    // replay into LDS with tile-relative output indices
    {
        uint32_t ia = ia0, jb = jb0, lo = ex;
        for (uint32_t s = 0; s < nsteps; s++) {
            const uint32_t kind = (steps >> (2 * s)) & 3u;
            if (kind == kStepA) {
                S.src[lo] = (uint16_t)(ia + 1);
                S.xm[ia] = (int16_t)lo;
                lo++;
                ia++;
            } else if (kind == kStepNew) {
                S.src[lo] = (uint16_t)(kFromB | jb);
                S.xd[jb] = (int16_t)lo;
                lo++;
                jb++;
            } else {
                S.xd[jb] = (int16_t)((int)lo - 1);
                jb++;
            }
        }
    }
    const uint64_t tile_prefix = lookback_resolve(C.merge_status, t, tot, C.err, &S.lb);
    __syncthreads();  // staging complete (the look-back may return without a barrier)

    for (uint32_t r = threadIdx.x; r < tot; r += kBlock) {
        const uint32_t sv = S.src[r];
        const uint64_t pos = tile_prefix + r;
        if (pos < cap) T::store(C.u_new, pos, T::denorm((sv & kFromB) ? sb[sv & ~kFromB] : sa[sv]));
    }
    if (C.x_m)
        for (uint32_t x = threadIdx.x; x < na; x += kBlock)
            C.x_m[i0 + x] = (uint32_t)(tile_prefix + (uint64_t)(int64_t)S.xm[x]);
    if (C.x_d)
        for (uint32_t y = threadIdx.x; y < nb; y += kBlock)
            C.x_d[j0 + y] = (uint32_t)(tile_prefix + (uint64_t)(int64_t)S.xd[y]);
    if (threadIdx.x == 0 && k1 == total) {
        const uint64_t n = tile_prefix + tot;
        const uint32_t w = code_width(n);
        C.result->new_dict_len = n;
        C.result->new_bitwidth = w;
        C.result->new_codes_words = (C.rows_total * w + 63) / 64;
        C.result->delta_dict_len = b;
    }
}

}  // namespace mc
