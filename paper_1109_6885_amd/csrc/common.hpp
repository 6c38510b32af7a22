// common.hpp -- value traits, wave/block scans and the cross-workgroup
// prefix protocol shared by the column-merge kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "colmerge.h"

namespace mc {

constexpr int kBlock = 256;       // threads per workgroup (4 waves of 64)
constexpr int kWaves = kBlock / 64;

// Slots of ColDesc::sflags: the digit positions (+ 1, 0 = unused) of the
// prefix passes, the flag "the prefix sort left the values out of order",
// the tile tickets of the two emits, and the arrival count of the full
// sort's grid-wide barriers.
constexpr int kPrefixSlots = 3;     // at most this many prefix passes
constexpr double kPrefixRun = 32.0;  // default wanted values per run of equal prefix
constexpr int kSfPrefix = 0, kSfUnsorted = kPrefixSlots, kSfEmitTicket = kPrefixSlots + 1,
              kSfEmitTicket2 = kPrefixSlots + 2, kSfGridBar = kPrefixSlots + 3, kSfSlots = 8;

// ---------------------------------------------------------------------------
// Value traits.  Stored values are always the caller's raw bytes.  For
// ordering, a value is mapped to a "normalized" key whose unsigned
// comparison is the column order: identity for integers, the two 8-byte
// halves byte-swapped (big-endian) for 16-byte strings.
// ---------------------------------------------------------------------------

struct alignas(16) Raw16 {
    uint64_t a, b;  // bytes 0..7 and 8..15, little-endian loads
};
struct Norm16 {
    uint64_t hi, lo;  // most / least significant 8 bytes in byte order
};

struct TU32 {
    typedef uint32_t K;
    typedef uint32_t N;
    static constexpr int kBytes = 4;
    __device__ static K load(const void *p, uint64_t i) { return static_cast<const K *>(p)[i]; }
    __device__ static void store(void *p, uint64_t i, K k) { static_cast<K *>(p)[i] = k; }
    // radix digit `d` (0 = least significant byte of the order)
    __device__ static uint32_t digit(K k, int d) { return (k >> (8 * d)) & 0xffu; }
    __device__ static uint32_t ndigit(N k, int d) { return (k >> (8 * d)) & 0xffu; }  // of norm(k)
    __device__ static N norm(K k) { return k; }
    __device__ static K denorm(N n) { return n; }
    __device__ static bool lt(N a, N b) { return a < b; }
    __device__ static bool le(N a, N b) { return a <= b; }
    __device__ static bool eq(N a, N b) { return a == b; }
    __device__ static bool keq(K a, K b) { return a == b; }
};

struct TU64 {
    typedef uint64_t K;
    typedef uint64_t N;
    static constexpr int kBytes = 8;
    __device__ static K load(const void *p, uint64_t i) { return static_cast<const K *>(p)[i]; }
    __device__ static void store(void *p, uint64_t i, K k) { static_cast<K *>(p)[i] = k; }
    __device__ static uint32_t digit(K k, int d) { return (uint32_t)(k >> (8 * d)) & 0xffu; }
    __device__ static uint32_t ndigit(N k, int d) { return (uint32_t)(k >> (8 * d)) & 0xffu; }
    __device__ static N norm(K k) { return k; }
    __device__ static K denorm(N n) { return n; }
    __device__ static bool lt(N a, N b) { return a < b; }
    __device__ static bool le(N a, N b) { return a <= b; }
    __device__ static bool eq(N a, N b) { return a == b; }
    __device__ static bool keq(K a, K b) { return a == b; }
};

struct TS16 {
    typedef Raw16 K;
    typedef Norm16 N;
    static constexpr int kBytes = 16;
    __device__ static K load(const void *p, uint64_t i) { return static_cast<const K *>(p)[i]; }
    __device__ static void store(void *p, uint64_t i, K k) { static_cast<K *>(p)[i] = k; }
    // digit d is byte 15 - d of the string (byte 15 is least significant)
    __device__ static uint32_t digit(K k, int d) {
        int byte = 15 - d;
        uint64_t w = byte >= 8 ? k.b : k.a;
        return (uint32_t)(w >> (8 * (byte & 7))) & 0xffu;
    }
    // digit d of norm(k): byte d of the 128-bit number (lo: bytes 0-7)
    __device__ static uint32_t ndigit(const N &n, int d) {
        return (uint32_t)((d >= 8 ? n.hi >> (8 * (d - 8)) : n.lo >> (8 * d)) & 0xffu);
    }
    __device__ static N norm(K k) {
        N n;
        n.hi = __builtin_bswap64(k.a);
        n.lo = __builtin_bswap64(k.b);
        return n;
    }
    __device__ static K denorm(N n) {
        K k;
        k.a = __builtin_bswap64(n.hi);
        k.b = __builtin_bswap64(n.lo);
        return k;
    }
    __device__ static bool lt(N x, N y) { return x.hi < y.hi || (x.hi == y.hi && x.lo < y.lo); }
    __device__ static bool le(N x, N y) { return x.hi < y.hi || (x.hi == y.hi && x.lo <= y.lo); }
    __device__ static bool eq(N x, N y) { return x.hi == y.hi && x.lo == y.lo; }
    __device__ static bool keq(K x, K y) { return x.a == y.a && x.b == y.b; }
};

// ---------------------------------------------------------------------------
// Wave and block scans (wave64, 256-thread blocks).
// ---------------------------------------------------------------------------

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }
__device__ __forceinline__ int wave_id() { return threadIdx.x >> 6; }

template <class T>
__device__ __forceinline__ T wave_incl_scan(T v) {
    const int lane = lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        T t = __shfl_up(v, o, 64);
        if (lane >= o) v += t;
    }
    return v;
}

template <class T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Exclusive scan over the block; s_tmp must hold kWaves values.  Returns the
// exclusive prefix of v and stores the block total in *total.  Contains two
// barriers; every thread of the block must call it.
template <class T>
__device__ __forceinline__ T block_excl_scan(T v, T *s_tmp, T *total) {
    T inc = wave_incl_scan(v);
    if (lane_id() == 63) s_tmp[wave_id()] = inc;
    __syncthreads();
    T off = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < kWaves; i++) {
        T x = s_tmp[i];
        if (i < wave_id()) off += x;
        tot += x;
    }
    __syncthreads();
    *total = tot;
    return off + inc - v;
}

// ---------------------------------------------------------------------------
// Cross-workgroup prefix ("decoupled look-back").  Tiles take their index
// from an atomic counter in launch order, publish their own aggregate, then
// add the aggregates of earlier tiles until one of them has published an
// inclusive prefix.  A tile only ever waits for tiles that took their index
// earlier, which are resident and never wait for later tiles, so the wait
// ends; it is additionally bounded, and on overrun the error word is set
// and the wave moves on, so every wave exits.
// ---------------------------------------------------------------------------

constexpr uint64_t kFlagAgg = 1ull << 62;
constexpr uint64_t kFlagPre = 2ull << 62;
constexpr uint64_t kValMask = kFlagAgg - 1;
constexpr uint32_t kSpinLimit = 1u << 22;

// Agent-scope relaxed atomics on the look-back status words.  Relaxed is
// enough: a status word carries the value it publishes (flag and count in
// one 64-bit word), so a reader needs no other data ordered with it, and
// agent scope keeps the word coherent across the XCDs' L2 caches.
__device__ __forceinline__ uint64_t ld_relaxed(const uint64_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_relaxed(uint64_t *p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void flag_error(uint32_t *err, uint32_t bit) {
    if (err) atomicOr(err, bit);
}

// ---------------------------------------------------------------------------
// Everything one column's merge reads and writes.  The single-column entry
// points pass it by value as a kernel argument; the batched entry point keeps
// an array of them in device memory and maps every workgroup of a launch to
// (column, tile).
// ---------------------------------------------------------------------------
struct ColDesc {
    int32_t type;              // mc_type
    uint32_t w;                // input code width
    const void *u_m;           // U_M
    uint64_t n_um;
    const uint64_t *main_codes;
    uint64_t n_main;
    const void *delta;         // D (append order)
    uint32_t nd;               // N_D
    uint32_t sort_tiles;       // ceil(N_D / sort tile)
    void *u_new;               // U' (capacity u_new_cap)
    uint64_t u_new_cap;
    uint64_t *out;             // packed result codes (capacity out_cap words)
    uint64_t out_cap;
    uint32_t *x_m;             // X_M (may be null when only Step 1(a) runs)
    uint32_t *x_d;             // X_D
    mc_result *result;         // device result scalars
    uint32_t *err;             // error word (result->error or a scratch word)
    uint64_t rows_total;       // N_M + N_D
    // workspace
    void *keys0, *keys1;       // radix ping-pong values
    uint32_t *vals0, *vals1;   // radix ping-pong rows
    uint32_t *gh;              // [passes][256] digit histograms (zeroed)
    uint32_t *base;            // [passes][256] digit offsets
    uint32_t *trivial;         // [passes] single-digit flags (zeroed)
    uint32_t *tcount;          // [256][sort_tiles] tile counts / offsets
    uint32_t *pgsum;           // [slot][tile group][256] digit counts of the tile groups of
                               // the two-launch prefix passes (zeroed), or null: three
                               // launches per pass
    uint32_t *ecnt;            // run heads of every emit tile (two-launch emit)
    uint32_t *egsum;           // run heads of every group of emit tiles (zeroed)
    uint32_t *counters;        // [1] merge tile counter (zeroed)
    uint32_t *sflags;          // Step 1(a) words, slots kSf* below (zeroed)
    uint64_t *emit_status;     // emit prefix words (zeroed)
    uint64_t *emit_status2;    // prefix words of the emit after the full LSD sort (zeroed)
    uint64_t *merge_status;    // merge prefix words (zeroed)
    uint64_t *mbound;          // U_M entries before each merge tile's start, or null
    uint32_t prefix_run;       // Step 1(a): wanted values per run of equal prefix (0: default)
    uint64_t *n_ud;            // |U_D| as written by Step 1(a) (zeroed)
    const uint64_t *n_ud_in;   // |U_D| as read by Step 1(b)
    uint64_t nd_max;           // capacity of u_d, drank, x_d
    void *u_d;                 // U_D
    uint32_t *drank;           // index in U_D of every delta row
    int16_t *xdev;             // compact X_M (see repack.hpp), n_um entries, or null
    uint4 *xsp;                // sparse X_M records (see repack.hpp), one per 128 codes, or null
    uint32_t *xflag;           // [0] nonzero: a compact entry overflowed, use x_m;
                               // [1] sparse records that overflowed (zeroed)
    // Step 1(a) by hashing first (see hash.hpp); unused when htab is null
    const void *sort_src;      // input of radix pass 0 (delta, or the distinct values)
    const uint64_t *sort_n;    // device count of values to sort, or null for nd
    uint32_t *htab;            // open-addressing table of representative rows + 1 (zeroed)
    uint64_t hmask;            // table size - 1 (power of two >= 2 * nd)
    uint32_t *rep;             // representative row of every delta row
    uint32_t *dindex;          // position of a representative in the distinct list
    void *dkeys;               // distinct values (tiles of representatives in any order)
    uint32_t *drankd;          // rank in U_D of every distinct value (by distinct position)
    uint64_t *dcount;          // number of distinct values listed (zeroed in a merge)
    uint64_t hrow0;            // first delta row of this hashing launch (0 in a merge)
    // single-column merges (else null): the compaction takes its positions
    // from per-tile counts instead of one shared atomic counter, and the
    // sort carries each distinct value's representative row
    uint32_t *hcnt;            // representatives found by every hashing tile
    uint32_t *hgsum;           // ... by every group of kEmitGroup hashing tiles (zeroed)
    uint32_t *drow;            // representative row of every distinct value (sort payload)
};

// Decoupled look-back over the tiles' status words.  One wave looks back:
// each round its 64 lanes read the statuses of the 256 nearest unvisited
// predecessors at once (four per lane), then, 64 at a time and nearest
// first, wait only for the lanes up to the nearest one that holds an
// inclusive prefix (the others are not needed) and sum the aggregates up to
// that one; a tile far from the last published inclusive prefix needs
// (distance / 256) memory round trips.  (All 256 threads polling, each
// waiting for its own predecessor, put four times the agent-scope loads on
// the same few status lines.)  Every thread of the block must call it; every
// thread gets the exclusive prefix (the sum of the aggregates of tiles
// 0 .. tile-1), after a barrier.  s_prefix: one 64-bit word of LDS.
//
// Split in two so that a tile can publish its own total first, do other work
// while its predecessors finish, and only then wait for their prefix.
__device__ inline void lookback_publish(uint64_t *status, uint32_t tile, uint64_t agg) {
    if (threadIdx.x == 0) st_relaxed(&status[tile], (tile == 0 ? kFlagPre : kFlagAgg) | agg);
}
__device__ inline uint64_t lookback_resolve(uint64_t *status, uint32_t tile, uint64_t agg,
                                            uint32_t *err, uint64_t *s_prefix) {
    if (tile == 0) return 0;
    if (wave_id() == 0) {
        // each round reads kLbGroups groups of 64 predecessors at once (one
        // memory round trip for 256 tiles), then consumes them nearest first
        constexpr int kLbGroups = 4;
        const int lane = lane_id();
        uint64_t prefix = 0;
        int64_t base = (int64_t)tile - 1;
        uint32_t spins = 0;
        bool done = false;
        while (!done) {
            uint64_t sg[kLbGroups];
#pragma unroll
            for (int g = 0; g < kLbGroups; g++) {
                const int64_t t = base - 64 * g - lane;  // lane 0: nearest predecessor of the group
                sg[g] = t >= 0 ? ld_relaxed(&status[t]) : kFlagPre;  // before tile 0: zero prefix
            }
#pragma unroll
            for (int g = 0; g < kLbGroups; g++) {
                if (done) break;
                const int64_t t = base - 64 * g - lane;
                uint64_t s = sg[g];
                while (true) {
                    const uint64_t pre = __ballot((s & kFlagPre) != 0);
                    // lanes up to and including the nearest inclusive prefix
                    const uint64_t need = pre ? ((pre & (~pre + 1)) << 1) - 1 : ~0ull;
                    const uint64_t wait = __ballot((s >> 62) == 0) & need;
                    if (!wait) break;
                    if (++spins > kSpinLimit) {  // give up: unpublished statuses count as zero
                        if (lane == 0) flag_error(err, MC_DEVERR_SPIN);
                        if ((s >> 62) == 0) s = kFlagPre;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                    if ((wait >> lane) & 1ull) s = ld_relaxed(&status[t]);
                }
                const uint64_t pre = __ballot((s & kFlagPre) != 0);
                const int stop = pre ? __ffsll((long long)pre) - 1 : 64;
                prefix += wave_sum(lane <= stop ? (s & kValMask) : 0ull);
                if (stop < 64) done = true;
            }
            base -= 64 * kLbGroups;
        }
        if (lane == 0) {
            st_relaxed(&status[tile], kFlagPre | (prefix + agg));
            *s_prefix = prefix;
        }
    }
    __syncthreads();
    return *s_prefix;
}

// Barrier over every workgroup of a launch whose workgroups are all resident
// at once (the caller launches at most one per two compute units).  ctr is a
// zeroed word that only grows: the caller's b-th barrier passes target =
// b * gridDim.x.  The workgroups may sit on different XCDs, whose L2 caches
// are not coherent with each other, so every thread releases its writes to
// the device before arriving and acquires after leaving.  The wait is
// bounded: on overrun the error word gets MC_DEVERR_SPIN and false returns
// (the caller then stops; every workgroup ends the same way, at this or its
// next barrier).  s_ok: one word of LDS.
__device__ inline bool grid_barrier(uint32_t *ctr, uint32_t target, uint32_t *err,
                                    uint32_t *s_ok) {
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        uint32_t spins = 0, ok = 1;
        while (__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (++spins > kSpinLimit) {
                flag_error(err, MC_DEVERR_SPIN);
                ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        *s_ok = ok;
    }
    __syncthreads();
    __threadfence();
    return *s_ok != 0;
}

// Move n (<= SLOTS * kBlock) elements: element x = load(x) goes to
// store(x, value).  Every load of a thread is issued before its first
// store, so the loads are in flight together; a strided load-then-store
// loop would wait for each load in turn (the compiler keeps the order
// because the store may alias the next load).  The loads are not guarded:
// slots past n load element n - 1 again and store nothing.  (With a guard
// per load, the compiler moves work of the store, such as a normalization,
// into the guarded block, and then waits for each load before the next.)
template <int SLOTS, class LoadF, class StoreF>
__device__ __forceinline__ void stage_all(uint32_t n, LoadF load, StoreF store) {
    if (n == 0) return;
    typedef decltype(load(0u)) V;
    V r[SLOTS];
#pragma unroll
    for (int j = 0; j < SLOTS; j++) {
        const uint32_t x = j * kBlock + threadIdx.x;
        r[j] = load(x < n ? x : n - 1);
    }
#pragma unroll
    for (int j = 0; j < SLOTS; j++) {
        const uint32_t x = j * kBlock + threadIdx.x;
        if (x < n) store(x, r[j]);
    }
}

// Code width for a dictionary of n entries: ceil(log2 n), at least 1.
__device__ __host__ inline uint32_t code_width(uint64_t n) {
    uint32_t w = 1;
    while (w < 64 && (1ull << w) < n) w++;
    return w;
}

}  // namespace mc
