/*
 * colmerge_oracle.h -- serial CPU oracle for the online merge of a
 * dictionary-encoded column (Krueger et al., "Fast Updates on Read-Optimized
 * Databases Using Multi-Core CPUs", arXiv 1109.6885, Sections 4.1, 5 and 5.3).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU library
 * against a plain, slow, obviously correct implementation.  Only the test
 * suite, the smoke check and the benchmark's CPU-baseline leg may load it.
 * It shares no source, header, table or helper with the GPU library.
 *
 * All pointers are HOST pointers.  All calls are synchronous and
 * single-threaded.  Return value: 0 on success, negative on error
 * (-1 argument error, -3 out of memory, -5 invalid data).
 *
 * Value types (fixed value length E, Section 7):
 *   CMO_U32   E = 4,  unsigned numeric order, little-endian in memory
 *   CMO_U64   E = 8,  unsigned numeric order, little-endian in memory
 *   CMO_STR16 E = 16, raw bytes, order = unsigned lexicographic byte order
 *
 * Packed code layout (the paper only says codes use the needed number of
 * bits, Section 4.1): code i occupies stream bits [i*w, (i+1)*w), least
 * significant bit first; stream bit b is bit (b mod 64) of 64-bit word b/64.
 */
#ifndef COLMERGE_ORACLE_H
#define COLMERGE_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { CMO_U32 = 0, CMO_U64 = 1, CMO_STR16 = 2 };

/* Code width for a dictionary of n entries (Eq. 4): ceil(log2 n) bits,
 * with 1 bit for n = 0 or 1 (Eq. 4 is undefined / zero there). */
uint32_t cmo_width(uint64_t n);

/* Read code i of width w from a packed stream (bit-by-bit). */
uint32_t cmo_unpack(const uint64_t *words, uint64_t i, uint32_t w);

/* OR code c of width w into position i of a packed stream (bit-by-bit). */
void cmo_pack(uint64_t *words, uint64_t i, uint32_t w, uint32_t code);

/* Step 1(a), modified form (Sections 5.1 and 5.3): sorted unique delta
 * values u_d (caller buffer of n_delta * E bytes) and, for every delta row,
 * its index in u_d (drank, n_delta entries).  *n_ud receives |U_D|. */
int cmo_delta_dictionary(int type, const void *delta, uint64_t n_delta,
                         void *u_d, uint32_t *drank, uint64_t *n_ud);

/* Step 1(b), modified form (Sections 5.1 and 5.3): two-pointer merge of the
 * sorted unique dictionaries u_m (n_um entries) and u_d (n_ud entries) into
 * u_new (caller buffer of (n_um + n_ud) * E bytes) with translation tables
 * x_m (n_um entries) and x_d (n_ud entries).  *n_new receives |U'|. */
int cmo_merge_dictionaries(int type, const void *u_m, uint64_t n_um,
                           const void *u_d, uint64_t n_ud, void *u_new,
                           uint32_t *x_m, uint32_t *x_d, uint64_t *n_new);

/* Step 2(b), modified form (Eq. 11): re-encode the main codes through x_m
 * and append the delta codes through x_d, all at width w_new.  out must hold
 * cmo_words(n_main + n_delta, w_new) words; it is zeroed first. */
int cmo_reencode(const uint64_t *main_codes, uint64_t n_main, uint32_t w,
                 const uint32_t *x_m, uint64_t n_um, const uint32_t *drank,
                 uint64_t n_delta, const uint32_t *x_d, uint64_t n_ud,
                 uint32_t w_new, uint64_t *out);

/* Number of 64-bit words that hold n codes of width w. */
uint64_t cmo_words(uint64_t n, uint32_t w);

/* The whole merge for one column (Section 5: Steps 1(a), 1(b), 2(a), 2(b)).
 * Inputs: sorted unique main dictionary u_m (n_um entries), n_main packed
 * main codes at width w, n_delta delta values in append order.
 * Outputs (caller buffers): u_new ((n_um + n_delta) * E bytes), new_codes
 * (cmo_words(n_main + n_delta, 32) words suffice), optional x_m / x_d
 * (n_um / n_delta entries; may be NULL), optional u_d / drank (n_delta
 * entries; may be NULL).  Scalars: |U'|, w', |U_D| and the number of
 * result words W'.  Returns -5 if u_m is not strictly increasing or a main
 * code is >= n_um, -1 for widths outside 1..32 or n_um > 2^w. */
int cmo_merge_column(int type, const void *u_m, uint64_t n_um,
                     const uint64_t *main_codes, uint64_t n_main, uint32_t w,
                     const void *delta, uint64_t n_delta,
                     void *u_new, uint64_t *new_codes,
                     uint32_t *x_m, uint32_t *x_d, void *u_d, uint32_t *drank,
                     uint64_t *n_new, uint32_t *w_new, uint64_t *n_ud,
                     uint64_t *n_words);

/* Naive Step 2(b) (Section 5.2, Eq. 5): decode each main code through u_m
 * and binary-search the value in u_new; the delta values are searched
 * directly.  Same output as cmo_reencode; used to pin the translation-table
 * route against the route the paper starts from. */
int cmo_reencode_naive(int type, const void *u_m, uint64_t n_um,
                       const uint64_t *main_codes, uint64_t n_main,
                       uint32_t w, const void *delta, uint64_t n_delta,
                       const void *u_new, uint64_t n_new, uint32_t w_new,
                       uint64_t *out);

#ifdef __cplusplus
}
#endif
#endif
