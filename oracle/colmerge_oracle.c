/*
 * colmerge_oracle.c -- serial CPU oracle for the online column merge of
 * Krueger et al., arXiv 1109.6885 (Sections 4.1, 5.1, 5.2, 5.3).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test suite, the smoke check and
 * the benchmark's CPU-baseline leg, never by the GPU library.  It is written
 * to be read against the paper, not to be fast: one thread, bit-by-bit code
 * packing, qsort for the delta, a two-pointer merge for the dictionaries.
 *
 * The result of the merge is uniquely defined (Eqs. 2 and 3): the new
 * dictionary is the sorted set U_M united with the delta values, and every
 * output row holds the rank of its value in that set, main rows first, then
 * the delta rows in append order.  The translation-table route of Section
 * 5.3 computes exactly that; the naive route of Section 5.2 is kept beside it
 * as an independent check.
 *
 * Readings where the paper is silent (recorded with the design notes):
 *  - width(n) = ceil(log2 n) for n >= 2 and 1 bit for n <= 1 (Eq. 4);
 *  - codes are packed least significant bit first into 64-bit words;
 *  - 16-byte values compare as unsigned bytes, first byte most significant;
 *  - every U_M entry is kept, referenced or not (Eq. 3 unions with U_M);
 *  - every row is kept (insert-only, Eq. 2).
 */
#include "colmerge_oracle.h"

#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* Values                                                              */
/* ------------------------------------------------------------------ */

static size_t value_len(int type)
{
    switch (type) {
    case CMO_U32: return 4;
    case CMO_U64: return 8;
    case CMO_STR16: return 16;
    default: return 0;
    }
}

/* Three-way compare of two values of the column's type. */
static int value_cmp(int type, const void *a, const void *b)
{
    if (type == CMO_U32) {
        uint32_t x, y;
        memcpy(&x, a, 4);
        memcpy(&y, b, 4);
        return (x > y) - (x < y);
    }
    if (type == CMO_U64) {
        uint64_t x, y;
        memcpy(&x, a, 8);
        memcpy(&y, b, 8);
        return (x > y) - (x < y);
    }
    /* 16-byte strings: unsigned lexicographic byte order. */
    return memcmp(a, b, 16);
}

static const void *value_at(int type, const void *base, uint64_t i)
{
    return (const unsigned char *)base + i * value_len(type);
}

static void value_copy(int type, void *dst_base, uint64_t di,
                       const void *src_base, uint64_t si)
{
    size_t e = value_len(type);
    memcpy((unsigned char *)dst_base + di * e,
           (const unsigned char *)src_base + si * e, e);
}

/* ------------------------------------------------------------------ */
/* Code width and packing                                              */
/* ------------------------------------------------------------------ */

uint32_t cmo_width(uint64_t n)
{
    /* Eq. 4: smallest w with 2^w >= n; at least one bit. */
    uint32_t w = 1;
    while (w < 64 && ((uint64_t)1 << w) < n)
        w++;
    return w;
}

uint64_t cmo_words(uint64_t n, uint32_t w)
{
    return (n * (uint64_t)w + 63) / 64;
}

uint32_t cmo_unpack(const uint64_t *words, uint64_t i, uint32_t w)
{
    uint32_t code = 0;
    for (uint32_t b = 0; b < w; b++) {
        uint64_t bit = i * (uint64_t)w + b;
        uint64_t v = (words[bit / 64] >> (bit % 64)) & 1u;
        code |= (uint32_t)v << b;
    }
    return code;
}

void cmo_pack(uint64_t *words, uint64_t i, uint32_t w, uint32_t code)
{
    for (uint32_t b = 0; b < w; b++) {
        uint64_t bit = i * (uint64_t)w + b;
        uint64_t v = (code >> b) & 1u;
        words[bit / 64] |= v << (bit % 64);
    }
}

/* ------------------------------------------------------------------ */
/* Step 1(a): delta dictionary and delta ranks                         */
/* ------------------------------------------------------------------ */

/* qsort has no user pointer in C99; the oracle is single-threaded, so the
 * column being sorted is held in file scope for the duration of the sort. */
static int g_sort_type;
static const void *g_sort_values;

static int cmp_rows(const void *pa, const void *pb)
{
    uint32_t a = *(const uint32_t *)pa;
    uint32_t b = *(const uint32_t *)pb;
    return value_cmp(g_sort_type, value_at(g_sort_type, g_sort_values, a),
                     value_at(g_sort_type, g_sort_values, b));
}

int cmo_delta_dictionary(int type, const void *delta, uint64_t n_delta,
                         void *u_d, uint32_t *drank, uint64_t *n_ud)
{
    if (value_len(type) == 0 || n_ud == NULL)
        return -1;
    if (n_delta > 0xffffffffull)
        return -1;
    *n_ud = 0;
    if (n_delta == 0)
        return 0;
    if (delta == NULL || u_d == NULL || drank == NULL)
        return -1;

    /* A permutation of the delta rows, sorted by value.  Equal values end
     * up adjacent; their relative order does not matter because they all
     * receive the same index. */
    uint32_t *perm = (uint32_t *)malloc(n_delta * sizeof(uint32_t));
    if (perm == NULL)
        return -3;
    for (uint64_t r = 0; r < n_delta; r++)
        perm[r] = (uint32_t)r;
    g_sort_type = type;
    g_sort_values = delta;
    qsort(perm, n_delta, sizeof(uint32_t), cmp_rows);

    /* Walk the sorted rows once: a new dictionary entry starts whenever the
     * value differs from the previous one, and every row of the current run
     * gets the index of that entry (the paper's tuple-id update). */
    uint64_t count = 0;
    for (uint64_t s = 0; s < n_delta; s++) {
        uint32_t row = perm[s];
        if (s == 0 || value_cmp(type, value_at(type, delta, row),
                                value_at(type, u_d, count - 1)) != 0) {
            value_copy(type, u_d, count, delta, row);
            count++;
        }
        drank[row] = (uint32_t)(count - 1);
    }
    free(perm);
    *n_ud = count;
    return 0;
}

/* ------------------------------------------------------------------ */
/* Step 1(b): dictionary merge with translation tables                 */
/* ------------------------------------------------------------------ */

int cmo_merge_dictionaries(int type, const void *u_m, uint64_t n_um,
                           const void *u_d, uint64_t n_ud, void *u_new,
                           uint32_t *x_m, uint32_t *x_d, uint64_t *n_new)
{
    if (value_len(type) == 0 || n_new == NULL)
        return -1;
    if ((n_um > 0 && (u_m == NULL || x_m == NULL)) ||
        (n_ud > 0 && (u_d == NULL || x_d == NULL)) ||
        (n_um + n_ud > 0 && u_new == NULL))
        return -1;

    uint64_t i = 0, k = 0, n = 0;
    /* Compare the two current values, append the smaller one and advance
     * its pointer; equal values are appended once, both pointers advance
     * and both tables receive the same index. */
    while (i < n_um && k < n_ud) {
        int c = value_cmp(type, value_at(type, u_m, i), value_at(type, u_d, k));
        if (c < 0) {
            value_copy(type, u_new, n, u_m, i);
            x_m[i++] = (uint32_t)n;
        } else if (c > 0) {
            value_copy(type, u_new, n, u_d, k);
            x_d[k++] = (uint32_t)n;
        } else {
            value_copy(type, u_new, n, u_m, i);
            x_m[i++] = (uint32_t)n;
            x_d[k++] = (uint32_t)n;
        }
        n++;
    }
    /* One side is exhausted: append the rest of the other side. */
    while (i < n_um) {
        value_copy(type, u_new, n, u_m, i);
        x_m[i++] = (uint32_t)n;
        n++;
    }
    while (k < n_ud) {
        value_copy(type, u_new, n, u_d, k);
        x_d[k++] = (uint32_t)n;
        n++;
    }
    *n_new = n;
    return 0;
}

/* ------------------------------------------------------------------ */
/* Step 2(b): re-encode through the translation tables (Eq. 11)        */
/* ------------------------------------------------------------------ */

int cmo_reencode(const uint64_t *main_codes, uint64_t n_main, uint32_t w,
                 const uint32_t *x_m, uint64_t n_um, const uint32_t *drank,
                 uint64_t n_delta, const uint32_t *x_d, uint64_t n_ud,
                 uint32_t w_new, uint64_t *out)
{
    if (w < 1 || w > 32 || w_new < 1 || w_new > 32)
        return -1;
    uint64_t n_out = n_main + n_delta;
    uint64_t nw = cmo_words(n_out, w_new);
    if (nw > 0 && out == NULL)
        return -1;
    for (uint64_t j = 0; j < nw; j++)
        out[j] = 0;
    for (uint64_t r = 0; r < n_main; r++) {
        uint32_t c = cmo_unpack(main_codes, r, w);
        if (c >= n_um)
            return -5;
        cmo_pack(out, r, w_new, x_m[c]);
    }
    for (uint64_t r = 0; r < n_delta; r++) {
        uint32_t k = drank[r];
        if (k >= n_ud)
            return -5;
        cmo_pack(out, n_main + r, w_new, x_d[k]);
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Naive Step 2(b) (Section 5.2)                                       */
/* ------------------------------------------------------------------ */

/* Index of value v in the sorted dictionary u (binary search); n if absent. */
static uint64_t search(int type, const void *u, uint64_t n, const void *v)
{
    uint64_t lo = 0, hi = n;
    while (lo < hi) {
        uint64_t mid = lo + (hi - lo) / 2;
        int c = value_cmp(type, value_at(type, u, mid), v);
        if (c == 0)
            return mid;
        if (c < 0)
            lo = mid + 1;
        else
            hi = mid;
    }
    return n;
}

int cmo_reencode_naive(int type, const void *u_m, uint64_t n_um,
                       const uint64_t *main_codes, uint64_t n_main,
                       uint32_t w, const void *delta, uint64_t n_delta,
                       const void *u_new, uint64_t n_new, uint32_t w_new,
                       uint64_t *out)
{
    if (value_len(type) == 0 || w < 1 || w > 32 || w_new < 1 || w_new > 32)
        return -1;
    uint64_t nw = cmo_words(n_main + n_delta, w_new);
    for (uint64_t j = 0; j < nw; j++)
        out[j] = 0;
    for (uint64_t r = 0; r < n_main; r++) {
        uint32_t c = cmo_unpack(main_codes, r, w);
        if (c >= n_um)
            return -5;
        uint64_t p = search(type, u_new, n_new, value_at(type, u_m, c));
        if (p == n_new)
            return -5;
        cmo_pack(out, r, w_new, (uint32_t)p);
    }
    for (uint64_t r = 0; r < n_delta; r++) {
        uint64_t p = search(type, u_new, n_new, value_at(type, delta, r));
        if (p == n_new)
            return -5;
        cmo_pack(out, n_main + r, w_new, (uint32_t)p);
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* The whole merge                                                     */
/* ------------------------------------------------------------------ */

int cmo_merge_column(int type, const void *u_m, uint64_t n_um,
                     const uint64_t *main_codes, uint64_t n_main, uint32_t w,
                     const void *delta, uint64_t n_delta,
                     void *u_new, uint64_t *new_codes,
                     uint32_t *x_m, uint32_t *x_d, void *u_d, uint32_t *drank,
                     uint64_t *n_new, uint32_t *w_new, uint64_t *n_ud,
                     uint64_t *n_words)
{
    size_t e = value_len(type);
    if (e == 0 || n_new == NULL || w_new == NULL || n_ud == NULL ||
        n_words == NULL)
        return -1;
    if (w < 1 || w > 32)
        return -1;
    if (n_um > ((uint64_t)1 << w))
        return -1;
    if (n_um == 0 && n_main > 0)
        return -1;
    if (n_um + n_delta > ((uint64_t)1 << 32))
        return -1;

    /* Step 0: the main dictionary must be sorted and unique (Section 3). */
    for (uint64_t i = 1; i < n_um; i++)
        if (value_cmp(type, value_at(type, u_m, i - 1),
                      value_at(type, u_m, i)) >= 0)
            return -5;

    int rc = 0;
    uint32_t *own_xm = NULL, *own_xd = NULL, *own_drank = NULL;
    void *own_ud = NULL;
    if (x_m == NULL && n_um > 0)
        x_m = own_xm = (uint32_t *)malloc(n_um * sizeof(uint32_t));
    if (x_d == NULL && n_delta > 0)
        x_d = own_xd = (uint32_t *)malloc(n_delta * sizeof(uint32_t));
    if (drank == NULL && n_delta > 0)
        drank = own_drank = (uint32_t *)malloc(n_delta * sizeof(uint32_t));
    if (u_d == NULL && n_delta > 0)
        u_d = own_ud = malloc(n_delta * e);
    if ((n_um > 0 && x_m == NULL) ||
        (n_delta > 0 && (x_d == NULL || drank == NULL || u_d == NULL))) {
        rc = -3;
        goto done;
    }

    /* Step 1(a). */
    rc = cmo_delta_dictionary(type, delta, n_delta, u_d, drank, n_ud);
    if (rc != 0)
        goto done;
    /* Step 1(b). */
    rc = cmo_merge_dictionaries(type, u_m, n_um, u_d, *n_ud, u_new, x_m, x_d,
                                n_new);
    if (rc != 0)
        goto done;
    /* Step 2(a), Eq. 4. */
    *w_new = cmo_width(*n_new);
    if (*w_new > 32) {
        rc = -1;
        goto done;
    }
    /* Step 2(b), Eq. 11. */
    rc = cmo_reencode(main_codes, n_main, w, x_m, n_um, drank, n_delta, x_d,
                      *n_ud, *w_new, new_codes);
    *n_words = cmo_words(n_main + n_delta, *w_new);

done:
    free(own_xm);
    free(own_xd);
    free(own_drank);
    free(own_ud);
    return rc;
}
