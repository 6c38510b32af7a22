/*
 * colmerge_cpu.h -- the merge of one dictionary-encoded column on the host's
 * cores, parallelized as Section 6.2 of Krueger et al., "Fast Updates on
 * Read-Optimized Databases Using Multi-Core CPUs" (arXiv 1109.6885) does on
 * a multi-core CPU (parallel Step 1(a), the three-phase merge of Step 1(b),
 * row ranges for Step 2(b)).  A measurement baseline beside the GPU library;
 * it shares no code with the GPU library or with the serial oracle.
 *
 * All pointers are HOST pointers; the call is synchronous and uses
 * `threads` threads.  Value types and the packed-code layout are those of the
 * GPU library: u32 / u64 little-endian in numeric order, 16-byte strings in
 * byte order; code i at stream bits [i*w, (i+1)*w), LSB first, 64-bit words.
 *
 * Outputs (caller buffers): u_new (n_um + n_delta values), out
 * (ceil((n_main + n_delta) * 32 / 64) words suffice), x_m (n_um), x_d
 * (n_delta entries, indexed by position in the sorted unique delta values),
 * *n_new = |U'|, *w_new = w' (Eq. 4, at least 1), *n_ud = |U_D|.
 * Returns 0, -1 (argument), -3 (out of memory) or -5 (a main code >= n_um).
 */
#ifndef COLMERGE_CPU_H
#define COLMERGE_CPU_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { CMP_U32 = 0, CMP_U64 = 1, CMP_STR16 = 2 };

int cmp_merge_column(int type, const void *u_m, uint64_t n_um, const uint64_t *codes,
                     uint64_t n_main, uint32_t w, const void *delta, uint64_t n_delta,
                     int threads, void *u_new, uint64_t *out, uint32_t *x_m, uint32_t *x_d,
                     uint64_t *n_new, uint32_t *w_new, uint64_t *n_ud);

#ifdef __cplusplus
}
#endif
#endif /* COLMERGE_CPU_H */
