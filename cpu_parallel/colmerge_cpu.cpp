// colmerge_cpu.cpp -- the merge of one dictionary-encoded column on the host's
// cores, parallelized the way Section 6.2 of Krueger et al. (arXiv 1109.6885)
// parallelizes it for a multi-core CPU.  A baseline to compare the GPU
// library with (not used by it, and sharing no code with it or with the
// serial oracle):
//
//   Step 1(a)  the delta's (value, row) pairs sorted by a parallel LSD radix
//              sort (per-thread digit counts, one prefix over threads,
//              stable scatter), then run heads counted per thread range,
//              a prefix over the ranges, and U_D and every row's index
//              written in parallel (the paper walks its CSB+ tree on one
//              thread and scatters the tuple ids in parallel, scheme (ii));
//   Step 1(b)  the three-phase merge of Section 6.2.1: every thread finds
//              its range of the merged sequence in both dictionaries (a
//              binary search on the cross diagonal), merges it counting the
//              values that are new (a value equal to its predecessor in the
//              merged order is the same dictionary entry), the counts are
//              prefix-summed, and every thread merges its range again,
//              writing U', X_M and X_D at its offset;
//   Step 2(a)  w' = ceil(log2 |U'|), at least 1 bit (Eq. 4);
//   Step 2(b)  the rows divided evenly among the threads (Section 6.2.2),
//              in ranges of whole 64-row groups so that no two threads
//              write the same output word; each code is unpacked at w,
//              translated through X_M (X_D for delta rows) and packed at w'.
//
// Ties between U_M and U_D resolve U_M first; the packed layout is code i at
// stream bits [i*w, (i+1)*w), least significant bit first, in 64-bit words.
#include "colmerge_cpu.h"

#include <algorithm>
#include <cstring>
#include <functional>
#include <thread>
#include <vector>

namespace {

struct Key16 {
    uint64_t hi, lo;  // the 16 bytes in memory order as a big-endian pair
};

// Value access per type: load as an order-preserving key, store back.
struct U32 {
    typedef uint32_t K;
    static constexpr int kBytes = 4;
    static K load(const void *p, uint64_t i) { return static_cast<const uint32_t *>(p)[i]; }
    static void store(void *p, uint64_t i, K k) { static_cast<uint32_t *>(p)[i] = k; }
    static uint32_t digit(K k, int d) { return (k >> (8 * d)) & 0xffu; }
    static bool lt(K a, K b) { return a < b; }
    static bool eq(K a, K b) { return a == b; }
};
struct U64 {
    typedef uint64_t K;
    static constexpr int kBytes = 8;
    static K load(const void *p, uint64_t i) { return static_cast<const uint64_t *>(p)[i]; }
    static void store(void *p, uint64_t i, K k) { static_cast<uint64_t *>(p)[i] = k; }
    static uint32_t digit(K k, int d) { return (uint32_t)(k >> (8 * d)) & 0xffu; }
    static bool lt(K a, K b) { return a < b; }
    static bool eq(K a, K b) { return a == b; }
};
struct S16 {
    typedef Key16 K;
    static constexpr int kBytes = 16;
    static K load(const void *p, uint64_t i) {
        const unsigned char *b = static_cast<const unsigned char *>(p) + 16 * i;
        K k{0, 0};
        for (int j = 0; j < 8; j++) k.hi = (k.hi << 8) | b[j];
        for (int j = 8; j < 16; j++) k.lo = (k.lo << 8) | b[j];
        return k;
    }
    static void store(void *p, uint64_t i, K k) {
        unsigned char *b = static_cast<unsigned char *>(p) + 16 * i;
        for (int j = 7; j >= 0; j--) {
            b[j] = (unsigned char)(k.hi & 0xffu);
            k.hi >>= 8;
        }
        for (int j = 15; j >= 8; j--) {
            b[j] = (unsigned char)(k.lo & 0xffu);
            k.lo >>= 8;
        }
    }
    // digit d counts from the least significant byte of the (hi, lo) pair
    static uint32_t digit(K k, int d) {
        return d < 8 ? (uint32_t)(k.lo >> (8 * d)) & 0xffu : (uint32_t)(k.hi >> (8 * (d - 8))) & 0xffu;
    }
    static bool lt(K a, K b) { return a.hi < b.hi || (a.hi == b.hi && a.lo < b.lo); }
    static bool eq(K a, K b) { return a.hi == b.hi && a.lo == b.lo; }
};

// Run f(t, lo, hi) on `nt` threads over [0, n) split evenly.
void parallel_ranges(int nt, uint64_t n, const std::function<void(int, uint64_t, uint64_t)> &f) {
    std::vector<std::thread> th;
    for (int t = 0; t < nt; t++) {
        const uint64_t lo = n * t / nt, hi = n * (t + 1) / nt;
        th.emplace_back(f, t, lo, hi);
    }
    for (auto &x : th) x.join();
}

uint32_t width_of(uint64_t n) {
    uint32_t w = 1;
    while (w < 64 && (1ull << w) < n) w++;
    return w;
}

// ---- Step 1(a) -----------------------------------------------------------

template <class T>
void delta_dictionary(int nt, const void *delta, uint64_t nd, std::vector<typename T::K> &u_d,
                      std::vector<uint32_t> &drank) {
    typedef typename T::K K;
    std::vector<K> k0(nd), k1(nd);
    std::vector<uint32_t> v0(nd), v1(nd);
    parallel_ranges(nt, nd, [&](int, uint64_t lo, uint64_t hi) {
        for (uint64_t i = lo; i < hi; i++) {
            k0[i] = T::load(delta, i);
            v0[i] = (uint32_t)i;
        }
    });
    // LSD radix: per pass, per-thread digit counts, one exclusive prefix over
    // (digit, thread), a stable scatter of every thread's range
    std::vector<uint64_t> cnt((size_t)nt * 256);
    for (int p = 0; p < T::kBytes; p++) {
        std::fill(cnt.begin(), cnt.end(), 0);
        parallel_ranges(nt, nd, [&](int t, uint64_t lo, uint64_t hi) {
            uint64_t *c = &cnt[(size_t)t * 256];
            for (uint64_t i = lo; i < hi; i++) c[T::digit(k0[i], p)]++;
        });
        bool trivial = false;
        for (int d = 0; d < 256 && !trivial; d++) {
            uint64_t s = 0;
            for (int t = 0; t < nt; t++) s += cnt[(size_t)t * 256 + d];
            trivial = s == nd;
        }
        if (trivial) continue;  // every value has the same digit here
        uint64_t run = 0;
        for (int d = 0; d < 256; d++)
            for (int t = 0; t < nt; t++) {
                const uint64_t c = cnt[(size_t)t * 256 + d];
                cnt[(size_t)t * 256 + d] = run;
                run += c;
            }
        parallel_ranges(nt, nd, [&](int t, uint64_t lo, uint64_t hi) {
            uint64_t *c = &cnt[(size_t)t * 256];
            for (uint64_t i = lo; i < hi; i++) {
                const uint64_t pos = c[T::digit(k0[i], p)]++;
                k1[pos] = k0[i];
                v1[pos] = v0[i];
            }
        });
        k0.swap(k1);
        v0.swap(v1);
    }
    // run heads per thread range, prefix over ranges, then U_D and indices
    std::vector<uint64_t> heads(nt + 1, 0);
    parallel_ranges(nt, nd, [&](int t, uint64_t lo, uint64_t hi) {
        uint64_t h = 0;
        for (uint64_t i = lo; i < hi; i++) h += (i == 0 || !T::eq(k0[i], k0[i - 1])) ? 1 : 0;
        heads[t + 1] = h;
    });
    for (int t = 0; t < nt; t++) heads[t + 1] += heads[t];
    u_d.resize(heads[nt]);
    drank.resize(nd);
    parallel_ranges(nt, nd, [&](int t, uint64_t lo, uint64_t hi) {
        uint64_t idx = heads[t];  // heads before this range
        for (uint64_t i = lo; i < hi; i++) {
            if (i == 0 || !T::eq(k0[i], k0[i - 1])) u_d[idx++] = k0[i];
            drank[v0[i]] = (uint32_t)(idx - 1);
        }
    });
}

// ---- Step 1(b) -----------------------------------------------------------

// Number of U_M entries among the first k merged elements (ties: U_M first).
template <class T>
uint64_t co_rank(uint64_t k, const std::vector<typename T::K> &a,
                 const std::vector<typename T::K> &b) {
    uint64_t lo = k > b.size() ? k - b.size() : 0, hi = std::min<uint64_t>(k, a.size());
    while (lo < hi) {
        const uint64_t mid = (lo + hi) / 2;
        if (!T::lt(b[k - 1 - mid], a[mid]))  // a[mid] <= b[k-1-mid]
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

template <class T>
void merge_dictionaries(int nt, const std::vector<typename T::K> &a,
                        const std::vector<typename T::K> &b, void *u_new, uint32_t *x_m,
                        uint32_t *x_d, uint64_t *n_new) {
    const uint64_t total = a.size() + b.size();
    std::vector<uint64_t> ks(nt + 1), is(nt + 1), count(nt + 1, 0);
    for (int t = 0; t <= nt; t++) {
        ks[t] = total * t / nt;
        is[t] = co_rank<T>(ks[t], a, b);
    }
    // walk merged positions [k0, k1) of thread t; `emit(is_a, idx, is_new)`
    auto walk = [&](int t, auto &&emit) {
        uint64_t i = is[t], j = ks[t] - is[t];
        for (uint64_t k = ks[t]; k < ks[t + 1]; k++) {
            const bool take_a = j >= b.size() || (i < a.size() && !T::lt(b[j], a[i]));
            if (take_a) {
                emit(true, i, true);
                i++;
            } else {
                // the U_D copy of a value equal to its U_M predecessor is not new
                const bool dup = i > 0 && T::eq(a[i - 1], b[j]);
                emit(false, j, !dup);
                j++;
            }
        }
    };
    // phase 1: count the new values of every range
    parallel_ranges(nt, nt, [&](int, uint64_t t0, uint64_t t1) {
        for (uint64_t t = t0; t < t1; t++) {
            uint64_t c = 0;
            walk((int)t, [&](bool, uint64_t, bool is_new) { c += is_new ? 1 : 0; });
            count[t + 1] = c;
        }
    });
    // phase 2: prefix sum of the counts
    for (int t = 0; t < nt; t++) count[t + 1] += count[t];
    // phase 3: write U', X_M, X_D from every range's offset
    parallel_ranges(nt, nt, [&](int, uint64_t t0, uint64_t t1) {
        for (uint64_t t = t0; t < t1; t++) {
            uint64_t pos = count[t];
            walk((int)t, [&](bool is_a, uint64_t idx, bool is_new) {
                if (is_a) {
                    T::store(u_new, pos, a[idx]);
                    x_m[idx] = (uint32_t)pos;
                    pos++;
                } else if (is_new) {
                    T::store(u_new, pos, b[idx]);
                    x_d[idx] = (uint32_t)pos;
                    pos++;
                } else {
                    x_d[idx] = (uint32_t)(pos - 1);
                }
            });
        }
    });
    *n_new = count[nt];
}

// ---- Step 2(b) -----------------------------------------------------------

inline uint32_t unpack(const uint64_t *words, uint64_t i, uint32_t w) {
    const uint64_t bit = i * w, wi = bit >> 6;
    const uint32_t sh = (uint32_t)(bit & 63);
    uint64_t v = words[wi] >> sh;
    if (sh + w > 64) v |= words[wi + 1] << (64 - sh);
    return (uint32_t)(v & ((1ull << w) - 1));
}

int reencode(int nt, const uint64_t *codes, uint64_t n_main, uint32_t w, uint64_t n_um,
             const uint32_t *x_m, const uint32_t *drank, uint64_t nd, const uint32_t *x_d,
             uint32_t wn, uint64_t *out) {
    const uint64_t rows = n_main + nd, groups = (rows + 63) / 64;
    const uint64_t words = (rows * wn + 63) / 64;
    bool bad = false;
    std::vector<char> bad_t(nt, 0);
    parallel_ranges(nt, groups, [&](int t, uint64_t g0, uint64_t g1) {
        // rows [64 g0, 64 g1): output words [g0 wn, g1 wn), owned by this thread
        const uint64_t w0 = g0 * wn, w1 = std::min<uint64_t>(g1 * wn, words);
        for (uint64_t x = w0; x < w1; x++) out[x] = 0;
        const uint64_t r1 = std::min<uint64_t>(64 * g1, rows);
        for (uint64_t r = 64 * g0; r < r1; r++) {
            uint32_t c;
            if (r < n_main) {
                const uint32_t old = unpack(codes, r, w);
                if (old >= n_um) {
                    bad_t[t] = 1;
                    continue;
                }
                c = x_m[old];
            } else {
                c = x_d[drank[r - n_main]];
            }
            const uint64_t bit = r * wn, wi = bit >> 6;
            const uint32_t sh = (uint32_t)(bit & 63);
            out[wi] |= (uint64_t)c << sh;
            if (sh + wn > 64) out[wi + 1] |= (uint64_t)c >> (64 - sh);
        }
    });
    for (int t = 0; t < nt; t++) bad = bad || bad_t[t];
    return bad ? -5 : 0;
}

template <class T>
int merge_column_t(const void *u_m, uint64_t n_um, const uint64_t *codes, uint64_t n_main,
                   uint32_t w, const void *delta, uint64_t nd, int nt, void *u_new,
                   uint64_t *out, uint32_t *x_m, uint32_t *x_d, uint64_t *n_new, uint32_t *w_new,
                   uint64_t *n_ud) {
    std::vector<typename T::K> a(n_um), u_d;
    std::vector<uint32_t> drank;
    parallel_ranges(nt, n_um, [&](int, uint64_t lo, uint64_t hi) {
        for (uint64_t i = lo; i < hi; i++) a[i] = T::load(u_m, i);
    });
    delta_dictionary<T>(nt, delta, nd, u_d, drank);
    *n_ud = u_d.size();
    merge_dictionaries<T>(nt, a, u_d, u_new, x_m, x_d, n_new);
    *w_new = width_of(*n_new);
    return reencode(nt, codes, n_main, w, n_um, x_m, drank.data(), nd, x_d, *w_new, out);
}

}  // namespace

extern "C" {

int cmp_merge_column(int type, const void *u_m, uint64_t n_um, const uint64_t *codes,
                     uint64_t n_main, uint32_t w, const void *delta, uint64_t n_delta, int threads,
                     void *u_new, uint64_t *out, uint32_t *x_m, uint32_t *x_d, uint64_t *n_new,
                     uint32_t *w_new, uint64_t *n_ud) {
    if (threads < 1 || w < 1 || w > 32 || !n_new || !w_new || !n_ud) return -1;
    if (n_um > 0 && (!u_m || !x_m)) return -1;
    if (n_delta > 0 && (!delta || !x_d)) return -1;
    if ((n_main + n_delta > 0) && !out) return -1;
    if (n_um + n_delta > 0 && !u_new) return -1;
    if (n_delta >= (1ull << 32) || n_um + n_delta > (1ull << 32)) return -1;
    try {
        switch (type) {
            case CMP_U32:
                return merge_column_t<U32>(u_m, n_um, codes, n_main, w, delta, n_delta, threads,
                                           u_new, out, x_m, x_d, n_new, w_new, n_ud);
            case CMP_U64:
                return merge_column_t<U64>(u_m, n_um, codes, n_main, w, delta, n_delta, threads,
                                           u_new, out, x_m, x_d, n_new, w_new, n_ud);
            case CMP_STR16:
                return merge_column_t<S16>(u_m, n_um, codes, n_main, w, delta, n_delta, threads,
                                           u_new, out, x_m, x_d, n_new, w_new, n_ud);
            default:
                return -1;
        }
    } catch (...) {
        return -3;
    }
}

}  // extern "C"
