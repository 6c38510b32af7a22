// repack.hpp -- Step 2(b) on the GPU (modified Step 2(b) of Section 5.3,
// Eq. 11, parallelized by row ranges as in Section 6.2.2): every main code
// is unpacked at the old width w, translated through X_M and repacked at
// the new width w'; the delta rows follow, translated through X_D.
//
// A workgroup owns CODES consecutive output rows (1024, 2048 or 4096; the
// default 2048, or what the batched autotuner picked).  Because 64 codes of
// width w fill exactly w 64-bit words, a tile of CODES rows starts on an even
// word boundary both in the input (CODES/64*w words) and in the output, so
// tiles never share a word and need no atomics in global memory.  The tile's
// input words are staged in LDS with 128-bit loads; each thread decodes
// CODES/256 consecutive codes, gathers their new codes from X_M (X_D for
// delta rows) and writes them as one run of bits into an LDS copy of the
// tile's output words (an LDS OR, since neighbouring threads share the words
// at the ends of their runs); the words then leave with coalesced 128-bit
// stores.  (Assembling each output word from a code array instead leaves
// only 16*w' threads busy, each with about 64/w' dependent LDS reads: three
// times slower at w' = 4 on a 32M-row column with a 6-entry dictionary.)
#pragma once

#include "common.hpp"

namespace mc {

constexpr int kRepackCodes = 2048;  // default rows per tile (32 groups of 64)
constexpr int kRepackPer = kRepackCodes / kBlock;  // codes per thread at the default

typedef unsigned long long u64x2 __attribute__((ext_vector_type(2)));

template <int CODES>
struct RepackSmemT {
    uint64_t in[CODES / 64 * 32 + 2];
    uint32_t code[CODES];
};
typedef RepackSmemT<kRepackCodes> RepackSmem;
// the re-encode's tile: input words, and the output words (w' <= 32) being built
template <int CODES>
struct RepackOutSmem {
    uint64_t in[CODES / 64 * 32 + 2];
    unsigned long long out[CODES / 64 * 32];
};

// ---------------------------------------------------------------------------
// Compact X_M.  The gathers X_M[c] dominate Step 2(b), and their cost grows
// with the table's footprint, not with the bytes used per entry.  X_M is
// strictly increasing: X_M[c] = c + g(c), where g(c) counts the new delta
// values below U_M[c] (monotone, from 0 to |U'| - |U_M|).  With
// a(c) = floor(c * A / 2^32), A = floor(2^32 * (|U'| - |U_M|) / |U_M|) (a
// fixed-point straight line through g's end points), the table stores the
// exact deviation d(c) = g(c) - a(c) in 16 bits, and X_M[c] = c + a(c) + d(c)
// is recomputed with the same integer formula.  If any deviation leaves
// int16 the flag is set and Step 2(b) gathers from the 32-bit X_M instead.
// The result is bit-identical either way.
// ---------------------------------------------------------------------------

constexpr int kXCompactTile = 4096;

__device__ __forceinline__ uint64_t xm_line_slope(const ColDesc &C) {
    const uint64_t added = C.result->new_dict_len - C.n_um;  // new delta values
    return C.n_um ? (added << 32) / C.n_um : 0;
}
__device__ __forceinline__ uint64_t xm_line(uint64_t c, uint64_t A) {
    const uint64_t lo = c * A, hi = __umul64hi(c, A);
    return (hi << 32) | (lo >> 32);
}

// ---------------------------------------------------------------------------
// Sparse X_M.  When few new delta values fall between neighbouring U_M
// entries (a large main dictionary and a small delta), g(c) = X_M[c] - c is
// nearly constant over runs of codes.  One 16-byte record per block of 128
// codes then holds g at the block's first code (bits 0-29; bit 31 flags an
// overflowed record) and up to 12 insertion offsets, one byte each (unused:
// 0xFF): offset i in 1..127 appears once for every new value between
// U_M[c0 + i - 1] and U_M[c0 + i], where c0 is the block's first code.  Then
// g(c0 + j) = g(c0) + (number of offsets <= j), exactly.  The records take
// n_um / 8 bytes, a sixteenth of the 16-bit deviation table, so the tables of
// dictionaries up to about 256K entries stay in a compute unit's L1 and those
// of about 30M entries in one XCD's L2, where the 16-bit table would need the
// MALL.  A block with more than 12 insertions is flagged, and the re-encode
// reads X_M itself for its codes.
// ---------------------------------------------------------------------------

constexpr int kXspBlock = 128;            // codes per record
constexpr int kXspSlots = 12;             // insertion offsets per record
constexpr uint32_t kXspOver = 1u << 31;   // record flag: more than kXspSlots insertions
constexpr uint64_t kXspMinDict = 1u << 14;  // smaller dictionaries keep the 16-bit table (L1)

// Are the sparse records worth building?  They need a large enough
// dictionary (below kXspMinDict the 16-bit table already sits in L1) and few
// new values per block: at more than 8 on average (c2: about 110) most
// records would overflow, and building them would only cost time.
constexpr uint64_t kXspMaxMean = 8;
__device__ __forceinline__ bool xsp_build(const ColDesc &C) {
    if (!C.xsp || C.n_um < kXspMinDict) return false;
    const uint64_t added = C.result->new_dict_len - C.n_um;  // new delta values
    return added * kXspBlock <= kXspMaxMean * C.n_um;
}
// Does the re-encode of this column read them?  When they were built and at
// most 1 in 32 of them overflowed.
__device__ __forceinline__ bool xsp_use(const ColDesc &C) {
    if (!xsp_build(C)) return false;
    const uint64_t nrec = (C.n_um + kXspBlock - 1) / kXspBlock;
    return (uint64_t)C.xflag[1] * 32u <= nrec;
}

// Number of offset bytes of word x that are <= j, for jj = j * 0x01010101 |
// 0x80808080 and 0 <= j <= 127.  Per byte, (128 + j) - (x & 127) lies in
// [1, 255], so the 32-bit subtraction borrows across no byte; its bit 7 is
// set exactly when x & 127 <= j, and ~x clears it for unused bytes (0xFF).
__device__ __forceinline__ uint32_t xsp_le(uint32_t x, uint32_t jj) {
    return (uint32_t)__popc((jj - (x & 0x7F7F7F7Fu)) & ~x & 0x80808080u);
}
__device__ __forceinline__ uint32_t xsp_lookup(const uint4 &r, uint32_t c) {
    const uint32_t jj = (c & (kXspBlock - 1)) * 0x01010101u | 0x80808080u;
    return c + r.x + xsp_le(r.y, jj) + xsp_le(r.z, jj) + xsp_le(r.w, jj);
}

// LDS of one X_M compaction tile: its X_M entries, one pad word after every
// 128 (entry j at j + j / 128), so that the 32 threads walking the records'
// blocks side by side read 32 different banks.
struct XCompactSmem {
    uint32_t x[kXCompactTile + kXCompactTile / kXspBlock];
    uint32_t slot[kXCompactTile / kXspBlock * 4];  // each record's offset bytes (12 used)
};
__device__ __forceinline__ uint32_t xs_at(uint32_t j) { return j + j / kXspBlock; }

// Both compact forms of one tile of X_M: the 16-bit deviations of every
// entry and, if the column has room for them, the sparse records of the
// tile's 32 blocks.
__device__ __forceinline__ void xcompact_tile(const ColDesc &C, uint64_t t, char *smem) {
    uint32_t *s_x = reinterpret_cast<XCompactSmem *>(smem)->x;
    const uint64_t c0 = t * kXCompactTile;
    if (c0 >= C.n_um) return;
    const uint32_t tn = (uint32_t)min<uint64_t>(kXCompactTile, C.n_um - c0);
    // staging: 16-byte loads of four entries where X_M is so aligned (the
    // library's own tables always are; a caller's may not be), the rest one
    // entry at a time
    const uint32_t n4 = reinterpret_cast<uintptr_t>(C.x_m + c0) % 16 == 0 ? tn / 4 : 0u;
    const uint4 *x4 = reinterpret_cast<const uint4 *>(C.x_m + c0);
    stage_all<kXCompactTile / 4 / kBlock>(
        n4, [&](uint32_t q) { return x4[q]; },
        [&](uint32_t q, const uint4 &v) {
            s_x[xs_at(4 * q)] = v.x;  // four entries of one 128-entry block
            s_x[xs_at(4 * q + 1)] = v.y;
            s_x[xs_at(4 * q + 2)] = v.z;
            s_x[xs_at(4 * q + 3)] = v.w;
        });
    for (uint32_t j = 4 * n4 + threadIdx.x; j < tn; j += kBlock) s_x[xs_at(j)] = C.x_m[c0 + j];
    __syncthreads();
    const uint64_t A = xm_line_slope(C);
    bool bad = false;
    // eight consecutive deviations per thread and round, written as one
    // 16-byte store (the table is the library's, 256-byte aligned, and
    // c0 + j0 is a multiple of 8); a partial group one entry at a time
    for (uint32_t j0 = 8 * threadIdx.x; j0 < tn; j0 += 8 * kBlock) {
        const uint32_t m = min<uint32_t>(8u, tn - j0);
        int16_t d[8];
#pragma unroll
        for (int i = 0; i < 8; i++) {
            const uint64_t c = c0 + j0 + i;
            const int64_t dev = (uint32_t)i < m ? (int64_t)s_x[xs_at(j0 + i)] - (int64_t)c -
                                                      (int64_t)xm_line(c, A)
                                                : 0;
            const bool ok = dev >= -32768 && dev <= 32767;
            bad |= !ok;
            d[i] = ok ? (int16_t)dev : (int16_t)0;
        }
        if (m == 8u) {
            uint4 v;
            v.x = (uint32_t)(uint16_t)d[0] | ((uint32_t)(uint16_t)d[1] << 16);
            v.y = (uint32_t)(uint16_t)d[2] | ((uint32_t)(uint16_t)d[3] << 16);
            v.z = (uint32_t)(uint16_t)d[4] | ((uint32_t)(uint16_t)d[5] << 16);
            v.w = (uint32_t)(uint16_t)d[6] | ((uint32_t)(uint16_t)d[7] << 16);
            *reinterpret_cast<uint4 *>(C.xdev + c0 + j0) = v;
        } else {
#pragma unroll
            for (int i = 0; i < 8; i++)
                if ((uint32_t)i < m) C.xdev[c0 + j0 + i] = d[i];
        }
    }
    if (__ballot(bad) && lane_id() == 0) atomicOr(C.xflag, 1u);
    if (!xsp_build(C)) return;  // the re-encode will not read them
    // 8 threads per record (the tile's 32 records side by side): each takes
    // 16 consecutive entries of the block and counts the new values between
    // them, a prefix over the 8 counts gives each its first slot, and each
    // writes its insertion offsets into the record's slot bytes in LDS.
    uint32_t *s_slot = reinterpret_cast<XCompactSmem *>(smem)->slot;
    for (uint32_t x = threadIdx.x; x < kXCompactTile / kXspBlock * 4; x += kBlock) s_slot[x] = ~0u;
    const uint32_t rb = threadIdx.x / 8, q = threadIdx.x % 8;
    const uint32_t r0 = rb * kXspBlock;                        // the record's first entry
    const uint32_t rn = r0 < tn ? min<uint32_t>(kXspBlock, tn - r0) : 0u;
    const uint32_t i_beg = q ? q * 16 : 1, i_end = min<uint32_t>(q * 16 + 16, rn);
    uint32_t cnt = 0;  // new values before the entries i_beg .. i_end - 1
    for (uint32_t i = i_beg; i < i_end; i++)
        cnt += s_x[xs_at(r0 + i)] - s_x[xs_at(r0 + i - 1)] - 1u;
    uint32_t incl = cnt;
#pragma unroll
    for (int d = 1; d < 8; d <<= 1) {
        const uint32_t v = __shfl_up(incl, d, 8);
        if (q >= (uint32_t)d) incl += v;
    }
    const uint32_t total = __shfl(incl, 7, 8);  // insertions in the whole block
    __syncthreads();  // slots initialised
    if (total <= (uint32_t)kXspSlots && cnt) {
        uint8_t *slot = reinterpret_cast<uint8_t *>(s_slot) + rb * 16;
        uint32_t k = incl - cnt;
        for (uint32_t i = i_beg; i < i_end; i++)
            for (uint32_t g = s_x[xs_at(r0 + i)] - s_x[xs_at(r0 + i - 1)] - 1u; g; g--)
                slot[k++] = (uint8_t)i;
    }
    __syncthreads();
    const bool over = rn && q == 0 && total > (uint32_t)kXspSlots;
    if (rn && q == 0) {
        const uint32_t g0 = s_x[xs_at(r0)] - (uint32_t)(c0 + r0);  // < 2^30: at most N_D new values
        C.xsp[(c0 + r0) / kXspBlock] = make_uint4(g0 | (over ? kXspOver : 0u), s_slot[rb * 4],
                                                  s_slot[rb * 4 + 1], s_slot[rb * 4 + 2]);
    }
    // one count per wave (a column with many new values overflows most records)
    const uint32_t n_over = (uint32_t)__popcll(__ballot(over));
    if (lane_id() == 0 && n_over) atomicAdd(&C.xflag[1], n_over);
}

// Stage the packed main words of the tile starting at row c0 into LDS with
// 128-bit loads (streamed once: non-temporal, so the tables keep the cache).
// A thread's loads (up to CODES / 1024 pairs, at w = 32) are all issued
// before the first LDS store: a strided load-then-store loop waits for each.
template <int CODES = kRepackCodes>
__device__ __forceinline__ void stage_main_words(const ColDesc &C, uint64_t c0, uint64_t *s_in) {
    if (c0 >= C.n_main) return;
    const uint32_t w = C.w;
    const uint64_t win = (C.n_main * w + 63) / 64;  // readable input words
    const uint64_t wbase = (c0 / 64) * w;           // even: c0/64 is a multiple of 16
    const uint32_t nw = (uint32_t)min<uint64_t>(CODES / 64 * (uint64_t)w, win - wbase);
    const uint32_t npair = nw / 2;  // <= CODES / 4 (w <= 32)
    const u64x2 *src2 = reinterpret_cast<const u64x2 *>(C.main_codes + wbase);
    u64x2 *dst2 = reinterpret_cast<u64x2 *>(s_in);
    stage_all<CODES / 1024>(
        npair, [&](uint32_t x) { return __builtin_nontemporal_load(src2 + x); },
        [&](uint32_t x, const u64x2 &v) { dst2[x] = v; });
    if ((nw & 1u) && threadIdx.x == 0)
        s_in[nw - 1] = __builtin_nontemporal_load(C.main_codes + wbase + nw - 1);
}

// Code i (tile-local) of the staged main words.
__device__ __forceinline__ uint32_t decode_code(const uint64_t *s_in, uint32_t i, uint32_t w,
                                                uint64_t mask) {
    const uint32_t bit = i * w;
    const uint32_t wi = bit >> 6, sh = bit & 63u;
    uint64_t v = s_in[wi] >> sh;
    if (sh + w > 64) v |= s_in[wi + 1] << (64 - sh);
    return (uint32_t)(v & mask);
}

// The same without a branch, for rows known to be inside the staged words:
// both words are read (s_in has a spare word past any tile), and the high
// word's bits are shifted in as (hi << 1) << (63 - sh), which is zero for
// sh = 0; bits of hi that the code does not use land at or above bit w and
// are masked off.
__device__ __forceinline__ uint32_t decode_code_nb(const uint64_t *s_in, uint32_t i, uint32_t w,
                                                   uint64_t mask) {
    const uint32_t bit = i * w;
    const uint32_t wi = bit >> 6, sh = bit & 63u;
    const uint64_t v = (s_in[wi] >> sh) | ((s_in[wi + 1] << 1) << (63u - sh));
    return (uint32_t)(v & mask);
}

// Assemble the tile's output words from its new codes (s_code, zero past the
// last row) and store them with 128-bit writes.
template <int CODES = kRepackCodes>
__device__ __forceinline__ void pack_store_tile(const ColDesc &C, uint64_t t, const uint32_t *s_code,
                                       uint32_t wn, uint64_t n_out) {
    // local word k covers tile bits [64k, 64k + 64)
    const uint64_t obase = t * (uint64_t)(CODES / 64) * wn;
    const uint64_t wres = (n_out * wn + 63) / 64;
    const uint64_t wlim = min<uint64_t>(C.out_cap, (wres + 1) & ~1ull);
    const uint32_t nwo = (CODES / 64) * wn;  // words of a full tile (even)
    // floor(x / wn) for x < CODES * 32 <= 2^17 as (x * ceil(2^32 / wn)) >> 32:
    // the reciprocal's rounding error adds less than x / 2^32 <= 2^-15 < 1 / wn
    // to the quotient, so the floor is exact.  The reciprocal is 64-bit: for
    // wn = 1 it is 2^32 itself.
    const uint64_t rcp = (0x100000000ull + wn - 1) / wn;
    for (uint32_t k2 = threadIdx.x; k2 < nwo / 2; k2 += kBlock) {
        uint64_t word[2];
#pragma unroll
        for (int h = 0; h < 2; h++) {
            const uint32_t k = 2 * k2 + h;
            const uint32_t b0 = 64u * k;
            uint32_t q = (uint32_t)(((uint64_t)b0 * rcp) >> 32);
            const uint32_t qe =
                min<uint32_t>((uint32_t)(((uint64_t)(b0 + 63) * rcp) >> 32), CODES - 1);
            uint64_t acc = 0;
            for (; q <= qe; q++) {
                const uint64_t c = s_code[q];
                const int sh = (int)(q * wn) - (int)b0;
                acc |= sh < 0 ? (c >> (-sh)) : (c << sh);
            }
            word[h] = acc;
        }
        const uint64_t gw = obase + 2ull * k2;
        if (gw + 1 < wlim) {
            u64x2 v;
            v.x = word[0];
            v.y = word[1];
            __builtin_nontemporal_store(v, reinterpret_cast<u64x2 *>(C.out + gw));
        } else if (gw < wlim) {
            C.out[gw] = word[0];
        }
    }
}

template <int CODES = kRepackCodes>
__device__ __forceinline__ void repack_tile(const ColDesc &C, uint64_t t, char *smem) {
    constexpr int PER = CODES / kBlock;  // consecutive codes per thread
    RepackOutSmem<CODES> &S = *reinterpret_cast<RepackOutSmem<CODES> *>(smem);
    uint64_t *s_in = S.in;
    unsigned long long *s_out = S.out;

    const uint32_t w = C.w;
    const uint32_t wn = C.result->new_bitwidth;
    const uint64_t n_ud = C.result->delta_dict_len;
    const uint64_t n_out = C.n_main + C.nd;
    const uint64_t c0 = t * CODES;
    if (c0 >= n_out) return;
    const uint32_t tn = (uint32_t)min<uint64_t>(CODES, n_out - c0);
    if (wn - 1u >= 32u) {  // the merge writes 1 <= w' <= 32 (|U'| <= 2^32); never past s_out
        if (threadIdx.x == 0) flag_error(C.err, MC_DEVERR_DELTA_RANGE);
        return;
    }
    const uint32_t nwo = (CODES / 64) * wn;  // output words of a full tile (even)

    for (uint32_t x = threadIdx.x; x < nwo; x += kBlock) s_out[x] = 0ull;
    stage_main_words<CODES>(C, c0, s_in);
    __syncthreads();

    // decode every code of this thread first, then issue all gathers together
    const uint64_t mask = (1ull << w) - 1ull;
    const bool compact = C.xdev != nullptr && *C.xflag == 0;
    const uint64_t A = compact ? xm_line_slope(C) : 0;
    const uint32_t i0 = threadIdx.x * PER;  // tile-local index of the thread's first code
    uint32_t idx[PER];
    uint32_t nc[PER];
    uint32_t bad = 0;
    const bool use_xsp = xsp_use(C);
    if (c0 + CODES <= C.n_main && !use_xsp) {
        // every row of the tile is a main row (most tiles) and reads the
        // 16-bit or the 4-byte table: no branch per row; the codes are
        // range-checked together and an out-of-range one (a data error)
        // reads entry 0 and writes 0.  (The sparse records need a branch
        // per row for overflowed records anyway, and measured faster in the
        // general path below: c3's re-encode 0.40 ms there, 0.43 ms here.)
        uint32_t cmax = 0;
#pragma unroll
        for (int j = 0; j < PER; j++) {
            idx[j] = decode_code_nb(s_in, i0 + j, w, mask);
            cmax = max(cmax, idx[j]);
        }
        uint32_t okm = (uint32_t)((1ull << PER) - 1ull);  // bit j: code j is in range
        if (cmax >= C.n_um) {
            bad |= MC_DEVERR_CODE_RANGE;
#pragma unroll
            for (int j = 0; j < PER; j++) {
                if (idx[j] >= C.n_um) {
                    okm &= ~(1u << j);
                    idx[j] = 0;
                }
            }
        }
        if (compact) {
#pragma unroll
            for (int j = 0; j < PER; j++)
                nc[j] = idx[j] + (uint32_t)xm_line(idx[j], A) + (uint32_t)(int32_t)C.xdev[idx[j]];
        } else {
#pragma unroll
            for (int j = 0; j < PER; j++) nc[j] = C.x_m[idx[j]];
        }
        if (okm != (uint32_t)((1ull << PER) - 1ull)) {
#pragma unroll
            for (int j = 0; j < PER; j++)
                if (!((okm >> j) & 1u)) nc[j] = 0u;
        }
    } else {
        uint32_t mm = 0, dm = 0;  // bit j: row j reads X_M (a main row) / X_D (a delta row)
#pragma unroll
        for (int j = 0; j < PER; j++) {
            const uint32_t i = i0 + j;
            const uint64_t g = c0 + i;
            idx[j] = 0;
            if (i < tn) {
                if (g < C.n_main) {
                    const uint32_t c = decode_code(s_in, i, w, mask);
                    if (c < C.n_um) {
                        mm |= 1u << j;
                        idx[j] = c;
                    } else {
                        bad |= MC_DEVERR_CODE_RANGE;
                    }
                } else {
                    const uint32_t r = C.drank[g - C.n_main];
                    if (r < n_ud) {
                        dm |= 1u << j;
                        idx[j] = r;
                    } else {
                        bad |= MC_DEVERR_DELTA_RANGE;
                    }
                }
            }
        }
        if (use_xsp) {
            // main rows: a 16-byte record per 128 codes (X_M itself for the codes
            // of an overflowed record); delta rows gather X_D.  Groups of 4 rows,
            // so that the records in flight take 16 registers, not 4 * PER.
            constexpr int GRP = PER < 4 ? PER : 4;
#pragma unroll
            for (int j0 = 0; j0 < PER; j0 += GRP) {
                uint4 rec[GRP];
#pragma unroll
                for (int k = 0; k < GRP; k++) {
                    const int j = j0 + k;
                    nc[j] = 0u;
                    if ((mm >> j) & 1u)
                        rec[k] = C.xsp[idx[j] / kXspBlock];
                    else if ((dm >> j) & 1u)
                        nc[j] = C.x_d[idx[j]];
                }
#pragma unroll
                for (int k = 0; k < GRP; k++) {
                    const int j = j0 + k;
                    if ((mm >> j) & 1u)
                        nc[j] = (rec[k].x & kXspOver) ? C.x_m[idx[j]] : xsp_lookup(rec[k], idx[j]);
                }
            }
        } else if (compact) {
            // main rows: X_M[c] = c + a(c) + d(c); delta rows gather X_D
#pragma unroll
            for (int j = 0; j < PER; j++) {
                if ((mm >> j) & 1u)
                    nc[j] = idx[j] + (uint32_t)xm_line(idx[j], A) + (uint32_t)(int32_t)C.xdev[idx[j]];
                else
                    nc[j] = ((dm >> j) & 1u) ? C.x_d[idx[j]] : 0u;
            }
        } else {
#pragma unroll
            for (int j = 0; j < PER; j++)
                nc[j] = ((mm >> j) & 1u) ? C.x_m[idx[j]] : ((dm >> j) & 1u) ? C.x_d[idx[j]] : 0u;
        }
    }
    if (bad) flag_error(C.err, bad);

    // the thread's codes are tile bits [i0 * wn, (i0 + PER) * wn): fill 64-bit
    // words from the low end and OR each finished one into LDS (rows past the
    // tile's end are 0 and add nothing)
    uint32_t wi = (i0 * wn) >> 6, nb = (i0 * wn) & 63u;
    uint64_t cur = 0;
#pragma unroll
    for (int j = 0; j < PER; j++) {
        const uint64_t c = nc[j];
        cur |= c << nb;
        nb += wn;
        if (nb >= 64) {
            atomicOr(&s_out[wi], (unsigned long long)cur);
            wi++;
            nb -= 64;
            cur = nb ? (c >> (wn - nb)) : 0ull;
        }
    }
    if (nb) atomicOr(&s_out[wi], (unsigned long long)cur);
    __syncthreads();

    // coalesced 128-bit stores, cut at the column's last word (and the
    // buffer's capacity)
    const uint64_t obase = t * (uint64_t)nwo;
    const uint64_t wres = (n_out * wn + 63) / 64;
    const uint64_t wlim = min<uint64_t>(C.out_cap, (wres + 1) & ~1ull);
    const u64x2 *src2 = reinterpret_cast<const u64x2 *>(s_out);
    for (uint32_t k2 = threadIdx.x; k2 < nwo / 2; k2 += kBlock) {
        const uint64_t gw = obase + 2ull * k2;
        if (gw + 1 < wlim) {
            __builtin_nontemporal_store(src2[k2], reinterpret_cast<u64x2 *>(C.out + gw));
        } else if (gw < wlim) {
            C.out[gw] = s_out[2 * k2];
        }
    }
}

}  // namespace mc
