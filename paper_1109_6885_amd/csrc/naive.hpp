// naive.hpp -- the unoptimized Step 2(b) of Section 5.2 (cost of Eq. 5), kept
// as the comparison the paper measures its translation tables against
// (Section 7.1, Fig. 7): every main row's code is decoded, its value is read
// from U_M, and its new code is found by binary search in U'; every delta
// value is searched directly.  Same output as repack_tile.
#pragma once

#include "repack.hpp"

namespace mc {

template <class T>
__device__ __forceinline__ void naive_tile(const ColDesc &C, uint64_t t, char *smem) {
    typedef typename T::N N;
    RepackSmem &S = *reinterpret_cast<RepackSmem *>(smem);
    const uint32_t w = C.w;
    const uint32_t wn = C.result->new_bitwidth;
    const uint64_t n_new = min(C.result->new_dict_len, C.u_new_cap);
    const uint64_t n_out = C.n_main + C.nd;
    const uint64_t c0 = t * kRepackCodes;
    if (c0 >= n_out) return;
    const uint32_t tn = (uint32_t)min<uint64_t>(kRepackCodes, n_out - c0);
    stage_main_words(C, c0, S.in);
    __syncthreads();
    const uint64_t mask = (1ull << w) - 1ull;
    uint32_t bad = 0;
    for (int j = 0; j < kRepackPer; j++) {
        const uint32_t i = j * kBlock + threadIdx.x;
        const uint64_t g = c0 + i;
        uint32_t nc = 0;
        if (i < tn) {
            N v;
            bool ok = true;
            if (g < C.n_main) {
                const uint32_t c = decode_code(S.in, i, w, mask);
                if (c < C.n_um)
                    v = T::norm(T::load(C.u_m, c));
                else
                    ok = false;
            } else {
                v = T::norm(T::load(C.delta, g - C.n_main));
            }
            if (ok) {
                uint64_t lo = 0, hi = n_new;  // first entry of U' not below v
                while (lo < hi) {
                    const uint64_t mid = (lo + hi) >> 1;
                    if (T::lt(T::norm(T::load(C.u_new, mid)), v))
                        lo = mid + 1;
                    else
                        hi = mid;
                }
                if (lo < n_new && T::eq(T::norm(T::load(C.u_new, lo)), v))
                    nc = (uint32_t)lo;
                else
                    ok = false;
            }
            if (!ok) bad |= (g < C.n_main) ? MC_DEVERR_CODE_RANGE : MC_DEVERR_DELTA_RANGE;
        }
        S.code[i] = nc;
    }
    if (bad) flag_error(C.err, bad);
    __syncthreads();
    pack_store_tile(C, t, S.code, wn, n_out);
}

}  // namespace mc
