// colmerge.hip -- host side of the column-merge library: argument checks,
// workspace layout, kernel launches and the extern "C" entry points that
// include/colmerge.h declares.  Kernels live in sort.hpp (Step 1(a)),
// merge.hpp (Steps 1(b), 2(a)) and repack.hpp (Step 2(b)).
#include <hip/hip_runtime.h>

#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <array>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "colmerge.h"
#include "common.hpp"
#include "hash.hpp"
#include "merge.hpp"
#include "naive.hpp"
#include "queue.hpp"
#include "repack.hpp"
#include "sort.hpp"

struct mc_ctx {
    int device = 0;
    uint32_t cus = 0;  // compute units of the device (grid of the one-launch full sort)
    int timing = 0;
    // one set of six events per timed merge since timing was enabled
    std::vector<std::array<hipEvent_t, 6>> ev;
    size_t used = 0;
    // pinned staging of batched descriptors, and the event of its last copy
    void *meta_host = nullptr;
    uint64_t meta_cap = 0;
    hipEvent_t meta_event = nullptr;
    // launch shapes (mc_ctx_set_tuning / mc_autotune_batched)
    mc_tuning tune = {2048u, 32u, 0u, MC_BATCHED_PHASES, 0u, 0u, 0u, 0u};
    // per-class shapes of the batched merge (mc_ctx_set_class_tuning /
    // mc_autotune_batched_classes): repack_codes and prefix_run of the
    // classes that have them
    mc_tuning class_tune[MC_TUNE_CLASSES] = {};
    uint8_t class_set[MC_TUNE_CLASSES] = {};
    // device address of this device's allocation-free workspace
    void *noalloc_scratch = nullptr;
    // validate mode (mc_ctx_set_validate)
    int validate = 0;
};

struct mc_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

// Workspace of mc_merge_column_noalloc: one copy per device, held from the
// library's load until the process ends.  Host code never uses this name as
// an address (on the host it only names the symbol); the device address of
// each device's copy comes from hipGetSymbolAddress in mc_ctx_create.
static __device__ __align__(256) unsigned char noalloc_scratch[MC_NOALLOC_SCRATCH_BYTES];

namespace {

thread_local std::string g_err;

// hipGetSymbolAddress results per device, looked up once per device.
constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mu;
void *g_noalloc_ptr[kMaxDevices] = {};

int fail(int code, const std::string &msg) {
    g_err = msg;
    return code;
}

int hip_fail(hipError_t e, const char *what) {
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return MC_E_HIP;
}

#define MC_HIP(call)                                   \
    do {                                               \
        hipError_t e_ = (call);                        \
        if (e_ != hipSuccess) return hip_fail(e_, #call); \
    } while (0)

#define MC_LAUNCHED(name)                                              \
    do {                                                               \
        hipError_t e_ = hipGetLastError();                             \
        if (e_ != hipSuccess) return hip_fail(e_, "launch " name);     \
    } while (0)

inline uint64_t ceil_div(uint64_t a, uint64_t b) { return (a + b - 1) / b; }
inline uint64_t align_up(uint64_t a, uint64_t b) { return (a + b - 1) / b * b; }

uint32_t value_len(int32_t type) {
    switch (type) {
        case MC_U32: return 4;
        case MC_U64: return 8;
        case MC_STR16: return 16;
        default: return 0;
    }
}

// Merged positions per merge tile: the batched merge's tiles, or a
// single-column merge's (larger for 4- and 8-byte values).
uint32_t merge_tile_of(int32_t type, bool batched) {
    switch (type) {
        case MC_U32:
            return batched ? mc::merge_tile<mc::TU32>()
                           : mc::merge_tile<mc::TU32, mc::MergeCfg<mc::TU32>::kItemsSingle>();
        case MC_U64:
            return batched ? mc::merge_tile<mc::TU64>()
                           : mc::merge_tile<mc::TU64, mc::MergeCfg<mc::TU64>::kItemsSingle>();
        default:
            return batched ? mc::merge_tile<mc::TS16>()
                           : mc::merge_tile<mc::TS16, mc::MergeCfg<mc::TS16>::kItemsSingle>();
    }
}
uint32_t sort_tile_of(int32_t type) {
    switch (type) {
        case MC_U32: return mc::sort_tile<mc::TU32>();
        case MC_U64: return mc::sort_tile<mc::TU64>();
        default: return mc::sort_tile<mc::TS16>();
    }
}

bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }
bool aligned4(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 3u) == 0; }

// ---------------------------------------------------------------------------
// Workspace layout of one column.  Part Z is cleared by a fill kernel at the
// start of every call (tile counters, histograms, prefix words, the sort's
// "same digit" flags, |U_D|, an error word); part B is written before it is
// read.  A single-column call places Z then B in its scratch; a batched call
// places every column's Z first (one contiguous clear) and then every B.
// ---------------------------------------------------------------------------

struct Carver {
    uint64_t off = 0;
    uint64_t take(uint64_t bytes) {
        off = align_up(off, 256);
        uint64_t at = off;
        off += bytes;
        return at;
    }
    uint64_t size() const { return align_up(off, 256); }
};

struct ColLayout {
    // part Z
    uint64_t counters = 0, sflags = 0, n_ud = 0, err = 0, xflag = 0, gh = 0, trivial = 0,
             pgsum = 0, egsum = 0, emit_status = 0, emit_status2 = 0,
             merge_status = 0, mbound = 0, dcount = 0, htab = 0, hgsum = 0, z_size = 0;
    // part B
    uint64_t base = 0, tcount = 0, ecnt = 0, keys0 = 0, keys1 = 0, vals0 = 0, vals1 = 0, u_d = 0,
             drank = 0, x_d = 0, x_m = 0, xdev = 0, xsp = 0, rep = 0, dindex = 0, dkeys = 0,
             drankd = 0, hcnt = 0, drow = 0, b_size = 0;
    uint32_t sort_tiles = 0, emit_tiles = 0, hist_tiles = 0, passes = 0;
    uint64_t merge_tiles = 0, repack_tiles = 0, xc_tiles = 0;
    uint32_t repack_codes = mc::kRepackCodes, prefix_run = 0;  // launch shapes
    bool partitioned = false;  // merge tile boundaries come from merge_partition
    bool two_launch_pass = false;  // prefix passes in two launches each (no waits)
    bool single = false;           // a single-column call (emit in two launches)
    bool hashed = false;       // Step 1(a) deduplicates by hashing first
    bool indexed = false;      // ... with the hashing done by a delta index (mc_delta_index)
    uint64_t hmask = 0;
    uint32_t hash_tiles = 0;
};

// Deltas with at least this many rows take the hashing route of Step 1(a):
// the radix passes then only see distinct values.  Smaller deltas sort
// directly (their passes are latency-bound, and hashing would add work).
constexpr uint64_t kHashMinRows = 1ull << 21;
// A delta of at least kHashMinRowsDict rows with at least hash_dict_ratio
// (default kHashDictRatio) times as many rows as U_M has entries hashes
// first too: if a good share of its rows repeat main values, each of those
// values fills a run of equal prefix thousands of values long, and one
// other value sharing the prefix leaves the run out of order, which costs
// the full LSD sort (16 passes for strings).  Hashing leaves the radix
// passes only the distinct values.  (On the 300-column batch: every one of
// the 16 columns that took the full sort has 6 to 738 dictionary entries
// and 29K to 197K delta rows.)
constexpr uint64_t kHashMinRowsDict = 4096;
constexpr uint64_t kHashDictRatio = 64;
bool many_repeats(uint64_t nd, uint64_t n_um, uint32_t ratio) {
    if (ratio == 0xFFFFFFFFu || n_um == 0 || nd < kHashMinRowsDict) return false;
    return nd >= (ratio ? ratio : kHashDictRatio) * n_um;
}

// Merges of at least this many tiles find the tile boundaries in a launch of
// their own (one wave per boundary, all at once) instead of at the start of
// every tile, where the search's dependent global loads would delay each
// round of resident tiles.  (128 against 512: c2, 489 tiles, 5-9 us faster;
// the 300-column batch 8.40 -> 8.34 ms; 2048 no better than 512.)
constexpr uint64_t kMergePartMinTiles = 128;

// Workgroups of merge_partition: one wave per tile boundary (tiles + 1).
uint64_t merge_part_blocks(uint64_t merge_tiles) { return ceil_div(merge_tiles + 1, mc::kWaves); }

const mc_tuning kDefaultTuning = {2048u, 32u, 0u, MC_BATCHED_PHASES, 0u, 0u, 0u, 0u};
// Tiles per work item of the persistent batched launch (defaults).
constexpr uint32_t kPersistRepack = 4, kPersistMerge = 2;
// Items of each global fallback phase of the persistent launch (they stride
// over the device-built maps of the columns that need the full sort).
constexpr uint32_t kPersistFbItems = 32;
// Queue counters of the persistent launch, after the batch's zeroed parts:
// the ticket, finished emit items, finished fallback items, error bits of the
// fallback chain's waits, then one finished-item count per column.
constexpr int kQTicket = 0, kQEmitDone = 1, kQFbDone = 2, kQErr = 3, kQColDone = 4;

ColLayout col_layout(int32_t type, uint64_t n_um, uint64_t nd, uint64_t n_main,
                     bool allow_hash = true, const mc_tuning &tune = kDefaultTuning,
                     bool indexed = false, bool batched = false) {
    ColLayout L;
    L.repack_codes = tune.repack_codes;
    L.prefix_run = tune.prefix_run;
    const uint32_t E = value_len(type);
    L.indexed = indexed;
    L.hashed = indexed ||
               (allow_hash && (nd >= (tune.hash_min_rows ? tune.hash_min_rows : kHashMinRows) ||
                               many_repeats(nd, n_um, tune.hash_dict_ratio)));
    if (L.hashed) L.hash_tiles = (uint32_t)ceil_div(nd, mc::kHashTile);  // also rank_rows' grid
    if (L.hashed && !L.indexed) {
        uint64_t h = 1024;
        while (h < 2 * nd) h <<= 1;
        L.hmask = h - 1;
    }
    L.passes = E;  // one 8-bit digit per value byte
    L.sort_tiles = (uint32_t)ceil_div(nd, sort_tile_of(type));
    L.emit_tiles = (uint32_t)ceil_div(nd, mc::kEmitTile);
    L.hist_tiles = (uint32_t)ceil_div(nd, mc::kHistChunk);
    L.merge_tiles = ceil_div(n_um + nd, merge_tile_of(type, batched));
    L.repack_tiles = ceil_div(n_main + nd, L.repack_codes);
    L.xc_tiles = n_main ? ceil_div(n_um, mc::kXCompactTile) : 0;
    Carver z;
    L.counters = z.take(16 * 4);
    L.sflags = z.take(mc::kSfSlots * 4);
    L.n_ud = z.take(8);
    L.err = z.take(8);
    L.xflag = z.take(8);
    L.gh = z.take((uint64_t)mc::kGhCopies * L.passes * 256 * 4);
    L.trivial = z.take(16 * 4);
    // the prefix passes in two launches each (counts with group sums, then
    // rank and scatter) for columns of at most kP2MaxTiles sort tiles; not
    // in the persistent batched launch, whose items run the three phases
    L.single = !batched;
    L.two_launch_pass = nd > 0 && L.sort_tiles <= mc::kP2MaxTiles &&
                        !(batched && tune.batched_launch == MC_BATCHED_PERSISTENT);
    if (L.two_launch_pass)
        L.pgsum = z.take((uint64_t)mc::kPrefixSlots * ceil_div(L.sort_tiles, mc::kP2Group) * 256 * 4);
    L.egsum = z.take(ceil_div(L.emit_tiles, mc::kEmitGroup) * 4);
    L.emit_status = z.take((uint64_t)L.emit_tiles * 8);
    L.emit_status2 = z.take((uint64_t)L.emit_tiles * 8);
    L.merge_status = z.take(L.merge_tiles * 8);
    L.partitioned = L.merge_tiles >= kMergePartMinTiles;
    if (L.partitioned) L.mbound = z.take((L.merge_tiles + 1) * 8);
    if (L.hashed && !L.indexed) {
        L.dcount = z.take(8);
        L.htab = z.take((L.hmask + 1) * 4);
        if (L.single) L.hgsum = z.take(ceil_div(L.hash_tiles, mc::kEmitGroup) * 4);
    }
    L.z_size = z.size();
    Carver b;
    L.base = b.take((uint64_t)L.passes * 256 * 4);
    L.tcount = b.take((uint64_t)256 * L.sort_tiles * 4);
    L.ecnt = b.take((uint64_t)L.emit_tiles * 4);
    L.keys0 = b.take(nd * E);
    L.keys1 = b.take(nd * E);
    L.vals0 = b.take(nd * 4);
    L.vals1 = b.take(nd * 4);
    L.u_d = b.take(nd * E);
    L.drank = b.take(nd * 4);
    L.x_d = b.take(nd * 4);
    L.x_m = b.take(n_um * 4);
    L.xdev = b.take(n_um * 2);
    L.xsp = b.take(ceil_div(n_um, mc::kXspBlock) * 16);
    if (L.hashed && !L.indexed) {
        L.rep = b.take(nd * 4);
        L.dkeys = b.take(nd * E);
        if (L.single) {
            L.hcnt = b.take((uint64_t)L.hash_tiles * 4);
            L.drow = b.take(nd * 4);
        } else {
            L.dindex = b.take(nd * 4);
        }
    }
    if (L.hashed) L.drankd = b.take(nd * 4);
    L.b_size = b.size();
    return L;
}

uint64_t single_scratch(const ColLayout &L) { return L.z_size + L.b_size; }

// Step 1(b) alone uses only the zeroed part of a column layout (counters,
// prefix words, tile boundaries).
ColLayout merge_only_layout(int32_t type, uint64_t n_um, uint64_t n_ud_max) {
    return col_layout(type, n_um, n_ud_max, 0, /*allow_hash=*/false);
}

// Step 1(a) fields for the hashing route (or the plain radix route).
void set_hash_fields(mc::ColDesc &C, char *za, char *zb, const ColLayout &L) {
    C.sort_src = C.delta;
    C.sort_n = nullptr;
    if (!L.hashed) return;
    C.drankd = reinterpret_cast<uint32_t *>(zb + L.drankd);
    if (L.indexed) return;  // the index's own buffers are set by the caller
    C.htab = reinterpret_cast<uint32_t *>(za + L.htab);
    C.hmask = L.hmask;
    C.rep = reinterpret_cast<uint32_t *>(zb + L.rep);
    C.dkeys = zb + L.dkeys;
    C.dcount = reinterpret_cast<uint64_t *>(za + L.dcount);
    if (L.single) {  // positions from per-tile counts; the sort carries representative rows
        C.hcnt = reinterpret_cast<uint32_t *>(zb + L.hcnt);
        C.hgsum = reinterpret_cast<uint32_t *>(za + L.hgsum);
        C.drow = reinterpret_cast<uint32_t *>(zb + L.drow);
    } else {
        C.dindex = reinterpret_cast<uint32_t *>(zb + L.dindex);
    }
    C.sort_src = C.dkeys;
    C.sort_n = C.dcount;
}

// Descriptor of one column with its workspace at za (part Z) and zb (part B).
mc::ColDesc make_desc(const mc_column_in *in, const mc_column_out *out, char *za, char *zb,
                      const ColLayout &L) {
    mc::ColDesc C;
    memset(&C, 0, sizeof(C));
    C.type = in->type;
    C.w = in->bitwidth;
    C.u_m = in->main_dict;
    C.n_um = in->main_dict_len;
    C.main_codes = in->main_codes;
    C.n_main = in->main_rows;
    C.delta = in->delta_values;
    C.nd = (uint32_t)in->delta_rows;
    C.sort_tiles = L.sort_tiles;
    C.u_new = out->new_dict;
    C.u_new_cap = out->new_dict_cap;
    C.out = out->new_codes;
    C.out_cap = out->new_codes_cap_words;
    C.x_m = out->x_main ? out->x_main : reinterpret_cast<uint32_t *>(zb + L.x_m);
    C.x_d = out->x_delta ? out->x_delta : reinterpret_cast<uint32_t *>(zb + L.x_d);
    C.result = out->result;
    C.err = &out->result->error;
    C.rows_total = in->main_rows + in->delta_rows;
    C.keys0 = zb + L.keys0;
    C.keys1 = zb + L.keys1;
    C.vals0 = reinterpret_cast<uint32_t *>(zb + L.vals0);
    C.vals1 = reinterpret_cast<uint32_t *>(zb + L.vals1);
    C.gh = reinterpret_cast<uint32_t *>(za + L.gh);
    C.base = reinterpret_cast<uint32_t *>(zb + L.base);
    C.trivial = reinterpret_cast<uint32_t *>(za + L.trivial);
    C.tcount = reinterpret_cast<uint32_t *>(zb + L.tcount);
    C.pgsum = L.two_launch_pass ? reinterpret_cast<uint32_t *>(za + L.pgsum) : nullptr;
    C.egsum = reinterpret_cast<uint32_t *>(za + L.egsum);
    C.ecnt = reinterpret_cast<uint32_t *>(zb + L.ecnt);
    C.counters = reinterpret_cast<uint32_t *>(za + L.counters);
    C.sflags = reinterpret_cast<uint32_t *>(za + L.sflags);
    C.emit_status = reinterpret_cast<uint64_t *>(za + L.emit_status);
    C.emit_status2 = reinterpret_cast<uint64_t *>(za + L.emit_status2);
    C.merge_status = reinterpret_cast<uint64_t *>(za + L.merge_status);
    C.mbound = L.partitioned ? reinterpret_cast<uint64_t *>(za + L.mbound) : nullptr;
    C.prefix_run = L.prefix_run;
    C.n_ud = reinterpret_cast<uint64_t *>(za + L.n_ud);
    C.n_ud_in = C.n_ud;
    C.nd_max = in->delta_rows;
    C.u_d = zb + L.u_d;
    C.drank = reinterpret_cast<uint32_t *>(zb + L.drank);
    C.xdev = L.xc_tiles ? reinterpret_cast<int16_t *>(zb + L.xdev) : nullptr;
    C.xsp = L.xc_tiles ? reinterpret_cast<uint4 *>(zb + L.xsp) : nullptr;
    C.xflag = reinterpret_cast<uint32_t *>(za + L.xflag);
    set_hash_fields(C, za, zb, L);
    return C;
}

// ---------------------------------------------------------------------------
// Delta index (mc_delta_index): the hashing route's table, representatives
// and distinct list, kept up to date by appends instead of built in a merge.
// Layout of its workspace:
//   64: u64 distinct values listed; 80: u32 error word (the rest of the
//   first 128 bytes is unused)
//   then the table (power of two >= 2 * capacity slots, >= 1024), the
//   representative and distinct position of every row, and the distinct
//   values.
// ---------------------------------------------------------------------------

struct IndexLayout {
    uint64_t scal = 0, htab = 0, rep = 0, dindex = 0, dkeys = 0, size = 0;
    uint64_t hmask = 0;
};

IndexLayout index_layout(int32_t type, uint64_t cap) {
    IndexLayout X;
    uint64_t h = 1024;
    while (h < 2 * cap) h <<= 1;
    X.hmask = h - 1;
    Carver c;
    X.scal = c.take(128);
    X.htab = c.take(h * 4);
    X.rep = c.take(cap * 4);
    X.dindex = c.take(cap * 4);
    X.dkeys = c.take(cap * value_len(type));
    X.size = c.size();
    return X;
}

// The index's part of a column descriptor.
void set_index_fields(mc::ColDesc &C, const mc_delta_index *ix) {
    const IndexLayout X = index_layout(ix->type, ix->capacity);
    char *w = static_cast<char *>(ix->workspace);
    C.htab = reinterpret_cast<uint32_t *>(w + X.htab);
    C.hmask = X.hmask;
    C.rep = reinterpret_cast<uint32_t *>(w + X.rep);
    C.dindex = reinterpret_cast<uint32_t *>(w + X.dindex);
    C.dkeys = w + X.dkeys;
    C.dcount = reinterpret_cast<uint64_t *>(w + X.scal + 64);
    C.sort_src = C.dkeys;
    C.sort_n = C.dcount;
}

// ---------------------------------------------------------------------------
// Kernels.  k1_* serve one column (descriptor by value, grid = its tiles);
// kn_* serve a batch: every workgroup finds its column in a per-phase prefix
// of tile counts and runs the same tile function, dispatched on the value
// type, with LDS sized for the largest type.
// ---------------------------------------------------------------------------

template <class A, class B, class C3>
constexpr size_t max3(A a, B b, C3 c) { return a > b ? (a > c ? a : c) : (b > c ? b : c); }

constexpr size_t kSmemHist = sizeof(mc::HistSmem<mc::TS16>);
constexpr size_t kSmemDown = max3(sizeof(mc::DownSmem<mc::TU32>), sizeof(mc::DownSmem<mc::TU64>),
                                  sizeof(mc::DownSmem<mc::TS16>));
static_assert(MC_U32 == 0 && MC_U64 == 1 && MC_STR16 == 2, "merge map slots follow mc_type");
constexpr size_t kSmemSmall = 1024;
constexpr size_t kSmemHash = max3(sizeof(mc::HashSmem<mc::TU32>), sizeof(mc::HashSmem<mc::TU64>),
                                  sizeof(mc::HashSmem<mc::TS16>));
// scan scratch + distinct digits and most frequent digit's count per position
constexpr size_t kSmemHistScan = (mc::kWaves + 32) * 4;

__global__ __launch_bounds__(256) void k_fill_zero(uint32_t *p0, uint64_t n0, uint32_t *p1,
                                                   uint64_t n1) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n0; i += stride)
        p0[i] = 0u;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n1; i += stride)
        p1[i] = 0u;
}

// Validate mode: err |= MC_DEVERR_ORDER unless u[0..n) is strictly increasing.
template <class T>
__global__ __launch_bounds__(256) void k_check_order(const void *u, uint64_t n, uint32_t *err) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    bool bad = false;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x + 1; i < n; i += stride)
        bad |= !T::lt(T::norm(T::load(u, i - 1)), T::norm(T::load(u, i)));
    if (bad) atomicOr(err, MC_DEVERR_ORDER);
}

// err |= *src (an index's error word into a merge's result)
__global__ void k_or_word(uint32_t *err, const uint32_t *src) {
    if (threadIdx.x == 0 && *src) atomicOr(err, *src);
}

// Plain 128-bit copy: the achievable streaming bandwidth on this GPU, and
// the kernel of known traffic that calibrates hardware byte counters.
// One 16-byte non-temporal load and store per thread and one workgroup per
// 4 KiB (measured on a 1 GiB copy: 6.57 TB/s; a grid-stride loop capped at
// 16 workgroups per CU reached 4.6, with 2 to 16 loads per thread in flight
// 5.4 to 6.3).  Past 2^32 work-items a launch cannot be one-shot: then each
// thread strides.
typedef unsigned int v4u32 __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void k_copy16(const v4u32 *__restrict__ src,
                                                v4u32 *__restrict__ dst, uint64_t n16) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride)
        __builtin_nontemporal_store(__builtin_nontemporal_load(&src[i]), &dst[i]);
}

template <class T>
__global__ __launch_bounds__(256) void k1_hist(mc::ColDesc C) {
    __shared__ __attribute__((aligned(16))) char smem[sizeof(mc::HistSmem<T>)];
    mc::hist_tile<T>(C, blockIdx.x, smem);
}
template <class T>
__global__ __launch_bounds__(256) void k1_hist_scan(mc::ColDesc C) {
    __shared__ __attribute__((aligned(16))) char smem[kSmemHistScan];
    mc::hist_scan_col<T>(C, smem);
}
// Radix pass kinds: one of the prefix passes (p = slot), or pass p of
// the full LSD sort, which runs only when the prefix sort left the values
// out of order (otherwise the launch returns at once).
constexpr int kPassPrefix = 0, kPassFull = 1;

__device__ __forceinline__ bool pass_io(const mc::ColDesc &C, int kind, int p, mc::PassIO *io) {
    if (kind == kPassPrefix) {
        *io = mc::prefix_io(C, p);
        return true;
    }
    if (C.sflags[mc::kSfUnsorted] == 0) return false;
    *io = mc::lsd_io(C, p);
    return true;
}

template <class T>
__global__ __launch_bounds__(256) void k1_sort_up(mc::ColDesc C, int kind, int p) {
    __shared__ __attribute__((aligned(16))) char smem[kSmemSmall];
    mc::PassIO io;
    if (pass_io(C, kind, p, &io)) mc::sort_up_tile<T>(C, io, blockIdx.x, smem);
}
template <class T>
__global__ __launch_bounds__(256) void k1_sort_scan(mc::ColDesc C, int kind, int p) {
    __shared__ __attribute__((aligned(16))) char smem[64];
    mc::PassIO io;
    if (!pass_io(C, kind, p, &io)) return;
    if (C.sort_tiles <= mc::kSmallScanTiles)
        mc::sort_scan_small<T>(C, io, blockIdx.x);  // 64 digits per workgroup
    else
        mc::sort_scan_digit<T>(C, io, blockIdx.x, smem);
}
template <class T>
__global__ __launch_bounds__(256) void k1_sort_down(mc::ColDesc C, int kind, int p) {
    __shared__ __attribute__((aligned(16))) char smem[sizeof(mc::DownSmem<T>)];
    mc::PassIO io;
    if (pass_io(C, kind, p, &io)) mc::sort_down_tile<T>(C, io, blockIdx.x, smem);
}
// The full LSD sort (every digit position) in one launch.  It runs only
// when the prefix sort left the values out of order; otherwise every
// workgroup returns at once, where a launch per phase and pass (3 x 4, 8 or
// 16 of them) would each cost a kernel boundary.  The grid has at most one
// workgroup per two compute units, so all are resident together, also beside
// the same kernel of other merges; they stride over the tiles (or digits) of
// each phase, with a grid-wide barrier between phases.  Every pass reads
// what the previous pass wrote, exactly as the per-phase launches do.
//
// The second emit follows in the same launch, after one more barrier: the
// workgroups take emit tiles by ticket until none is left (a tile's
// look-back waits only for lower tickets, held by running workgroups), or,
// on the hashing route, stride over the tiles of the distinct values.
template <class T>
__global__ __launch_bounds__(256) void k1_full_sort(mc::ColDesc C) {
    __shared__ __attribute__((aligned(16)))
    char smem[std::max(sizeof(mc::DownSmem<T>), sizeof(mc::EmitSmem<T>))];
    __shared__ uint32_t s_ok, s_tile;
    if (C.sflags[mc::kSfUnsorted] == 0) return;
    const uint32_t G = gridDim.x;
    const bool small = C.sort_tiles <= mc::kSmallScanTiles;
    const uint32_t scan_units = small ? mc::kSmallScanParts : 256u;
    uint32_t *bar = &C.sflags[mc::kSfGridBar];
    uint32_t target = 0;
    for (int p = 0; p < T::kBytes; p++) {
        const mc::PassIO io = mc::lsd_io(C, p);
        for (uint32_t t = blockIdx.x; t < C.sort_tiles; t += G) {
            mc::sort_up_tile<T>(C, io, t, smem);
            __syncthreads();
        }
        target += G;
        if (!mc::grid_barrier(bar, target, C.err, &s_ok)) return;
        for (uint32_t d = blockIdx.x; d < scan_units; d += G) {
            if (small)
                mc::sort_scan_small<T>(C, io, d);
            else
                mc::sort_scan_digit<T>(C, io, d, smem);
            __syncthreads();
        }
        target += G;
        if (!mc::grid_barrier(bar, target, C.err, &s_ok)) return;
        for (uint32_t t = blockIdx.x; t < C.sort_tiles; t += G) {
            mc::sort_down_tile<T>(C, io, t, smem);
            __syncthreads();
        }
        target += G;
        if (!mc::grid_barrier(bar, target, C.err, &s_ok)) return;
    }
    const uint32_t emit_tiles = (C.nd + mc::kEmitTile - 1) / mc::kEmitTile;
    if (C.sort_n) {  // the hashing route: every sorted position is a distinct value
        for (uint32_t t = blockIdx.x; t < emit_tiles; t += G) {
            mc::emit_distinct_tile<T>(C, t, true);
            __syncthreads();
        }
        return;
    }
    while (true) {
        if (threadIdx.x == 0) s_tile = atomicAdd(&C.sflags[mc::kSfEmitTicket2], 1u);
        __syncthreads();
        const uint32_t t = s_tile;
        __syncthreads();  // everyone has the ticket before thread 0 takes the next
        if (t >= emit_tiles) break;
        mc::emit_tile_at<T>(C, smem, true, t);
        __syncthreads();
    }
}
// One prefix pass (slot) in two launches.
template <class T>
__global__ __launch_bounds__(256) void k1_sort_up2(mc::ColDesc C, int slot) {
    __shared__ __attribute__((aligned(16))) char smem[kSmemSmall];
    mc::sort_up2_tile<T>(C, mc::prefix_io(C, slot), slot, blockIdx.x, smem);
}
template <class T>
__global__ __launch_bounds__(256) void k1_sort_down2(mc::ColDesc C, int slot) {
    __shared__ __attribute__((aligned(16))) char smem[sizeof(mc::DownSmem<T>)];
    mc::sort_down2_tile<T>(C, mc::prefix_io(C, slot), slot, blockIdx.x, smem);
}
// The emit after the prefix sort in two launches: the windows and the run
// heads' counts, then the numbering.
template <class T>
__global__ __launch_bounds__(256) void k1_emit_count(mc::ColDesc C) {
    __shared__ __attribute__((aligned(16))) char smem[sizeof(mc::EmitWinSmem<T>)];
    mc::emit_count_tile<T>(C, blockIdx.x, smem);
}
template <class T>
__global__ __launch_bounds__(256) void k1_emit_write(mc::ColDesc C) {
    __shared__ __attribute__((aligned(16))) char smem[sizeof(mc::EmitSmem<T>)];
    mc::emit_tile_at<T, true>(C, smem, false, blockIdx.x);
}
template <class T>
__global__ __launch_bounds__(256) void k1_emit_distinct_win(mc::ColDesc C) {
    __shared__ __attribute__((aligned(16))) char smem[sizeof(mc::EmitWinSmem<T>)];
    mc::emit_distinct_window_tile<T>(C, blockIdx.x, smem);
}
template <class T>
__global__ __launch_bounds__(256) void k1_hash_insert(mc::ColDesc C) {
    __shared__ __attribute__((aligned(16))) char smem[sizeof(mc::HashSmem<T>)];
    mc::hash_insert_tile<T>(C, blockIdx.x, smem);
}
template <class T>
__global__ __launch_bounds__(256) void k1_compact(mc::ColDesc C) {
    __shared__ __attribute__((aligned(16))) char smem[sizeof(mc::CompactSmem)];
    mc::compact_tile<T>(C, blockIdx.x, smem);
}
__global__ __launch_bounds__(256) void k1_rank_rows(mc::ColDesc C) {
    mc::rank_rows_tile(C, blockIdx.x);
}
template <class T>
__global__ __launch_bounds__(256) void k1_merge_part(mc::ColDesc C) {
    mc::merge_partition<T, mc::MergeCfg<T>::kItemsSingle>(C, blockIdx.x);
}
template <class T>
__global__ __launch_bounds__(256) void k1_merge(mc::ColDesc C) {
    constexpr int kItems = mc::MergeCfg<T>::kItemsSingle;
    __shared__ __attribute__((aligned(16))) char smem[sizeof(mc::MergeSmem<T, kItems>)];
    mc::merge_tile<T, kItems>(C, smem);
}
template <class T>
__global__ __launch_bounds__(256) void k1_naive(mc::ColDesc C) {
    __shared__ __attribute__((aligned(16))) char smem[sizeof(mc::RepackSmem)];
    mc::naive_tile<T>(C, blockIdx.x, smem);
}
__global__ __launch_bounds__(256) void k1_xcompact(mc::ColDesc C) {
    __shared__ __attribute__((aligned(16))) char smem[sizeof(mc::XCompactSmem)];
    mc::xcompact_tile(C, blockIdx.x, smem);
}
template <int CODES>
__global__ __launch_bounds__(256) void k1_repack(mc::ColDesc C) {
    __shared__ __attribute__((aligned(16))) char smem[sizeof(mc::RepackOutSmem<CODES>)];
    mc::repack_tile<CODES>(C, blockIdx.x, smem);
}

// ---- batched ----

struct Batch {
    const mc::ColDesc *cols;
    const uint32_t *map;  // ncols + 1 prefix of tile counts for this phase
    uint32_t ncols;
};

// Column of workgroup b: the j with map[j] <= b < map[j + 1].
__device__ __forceinline__ uint32_t find_col(const Batch &B, uint32_t b) {
    uint32_t lo = 0, hi = B.ncols;  // map[lo] <= b < map[hi]
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (B.map[mid] <= b)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

#define MC_DISPATCH(C, FN, ...)                                     \
    switch ((C).type) {                                             \
        case MC_U32: FN<mc::TU32>(__VA_ARGS__); break;              \
        case MC_U64: FN<mc::TU64>(__VA_ARGS__); break;              \
        default: FN<mc::TS16>(__VA_ARGS__); break;                  \
    }
// out = FN<T>(C) for the column's value type
#define MC_DISPATCH_R(C, OUT, FN)                                   \
    switch ((C).type) {                                             \
        case MC_U32: OUT = FN<mc::TU32>(C); break;                  \
        case MC_U64: OUT = FN<mc::TU64>(C); break;                  \
        default: OUT = FN<mc::TS16>(C); break;                      \
    }

__global__ __launch_bounds__(256) void kn_zero_results(Batch B) {
    for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < B.ncols;
         j += gridDim.x * blockDim.x) {
        mc_result *r = B.cols[j].result;
        r->new_dict_len = 0;
        r->new_codes_words = 0;
        r->delta_dict_len = 0;
        r->new_bitwidth = 0;
        r->error = 0;
    }
}
__global__ __launch_bounds__(256) void kn_hist(Batch B) {
    __shared__ __attribute__((aligned(16))) char smem[kSmemHist];
    const uint32_t j = find_col(B, blockIdx.x);
    const mc::ColDesc &C = B.cols[j];
    MC_DISPATCH(C, mc::hist_tile, C, blockIdx.x - B.map[j], smem);
}
__global__ __launch_bounds__(256) void kn_hist_scan(Batch B) {
    __shared__ __attribute__((aligned(16))) char smem[kSmemHistScan];
    const uint32_t j = find_col(B, blockIdx.x);
    const mc::ColDesc &C = B.cols[j];
    MC_DISPATCH(C, mc::hist_scan_col, C, smem);
}
// One radix pass phase for every column.  Workgroup b of the map takes tile
// (or, for the scan, digit / part) b - map[j] of column j; a launch with fewer
// workgroups than the map's total strides over it (the fallback passes, whose
// maps are built on the device and hold only the columns the prefix sort left
// unsorted, so an unneeded pass is a launch of workgroups that return).
__device__ __forceinline__ uint32_t map_total(const Batch &B) { return B.map[B.ncols]; }

// The bodies stride: workgroup `first` of `count` takes units first,
// first + count, ... of the map (a launch, or the one-launch fallback below).
__device__ __forceinline__ void sort_up_units(const Batch &B, int kind, int p, uint32_t first,
                                              uint32_t count, char *smem) {
    const uint32_t total = map_total(B);
    for (uint32_t b = first; b < total; b += count) {
        if (b != first) __syncthreads();  // the tile before is done with the LDS
        const uint32_t j = find_col(B, b);
        const mc::ColDesc &C = B.cols[j];
        mc::PassIO io;
        if (!pass_io(C, kind, p, &io)) continue;
        if (kind == kPassPrefix && C.pgsum) {  // counts with group sums (slot p)
            MC_DISPATCH(C, mc::sort_up2_tile, C, io, p, b - B.map[j], smem);
        } else {
            MC_DISPATCH(C, mc::sort_up_tile, C, io, b - B.map[j], smem);
        }
    }
}
__device__ __forceinline__ void sort_scan_units(const Batch &B, int kind, int p, uint32_t first,
                                                uint32_t count, char *smem) {
    const uint32_t total = map_total(B);
    for (uint32_t b = first; b < total; b += count) {
        if (b != first) __syncthreads();
        const uint32_t j = find_col(B, b);
        const mc::ColDesc &C = B.cols[j];
        if (kind == kPassPrefix && C.pgsum) continue;  // the scatter sums the counts itself
        mc::PassIO io;
        if (!pass_io(C, kind, p, &io)) continue;
        if (C.sort_tiles <= mc::kSmallScanTiles) {  // 64 digits per workgroup
            MC_DISPATCH(C, mc::sort_scan_small, C, io, b - B.map[j]);
        } else {
            MC_DISPATCH(C, mc::sort_scan_digit, C, io, b - B.map[j], smem);
        }
    }
}
__device__ __forceinline__ void sort_down_units(const Batch &B, int kind, int p, uint32_t first,
                                                uint32_t count, char *smem) {
    const uint32_t total = map_total(B);
    for (uint32_t b = first; b < total; b += count) {
        if (b != first) __syncthreads();
        const uint32_t j = find_col(B, b);
        const mc::ColDesc &C = B.cols[j];
        mc::PassIO io;
        if (!pass_io(C, kind, p, &io)) continue;
        if (kind == kPassPrefix && C.pgsum) {
            MC_DISPATCH(C, mc::sort_down2_tile, C, io, p, b - B.map[j], smem);
        } else {
            MC_DISPATCH(C, mc::sort_down_tile, C, io, b - B.map[j], smem);
        }
    }
}
// emit_tile takes its tile from a per-column ticket (a workgroup holds one
// ticket at a time and waits only on lower ones, all held by running
// workgroups), emit_distinct_tile waits on no other tile.
__device__ __forceinline__ void emit_units(const Batch &B, bool again, uint32_t first,
                                           uint32_t count, char *smem) {
    const uint32_t total = map_total(B);
    for (uint32_t b = first; b < total; b += count) {
        if (b != first) __syncthreads();
        const uint32_t j = find_col(B, b);
        const mc::ColDesc &C = B.cols[j];
        if (C.drankd) {  // hashing route: the sorted values are distinct
            MC_DISPATCH(C, mc::emit_distinct_tile, C, b - B.map[j], again);
        } else {
            MC_DISPATCH(C, mc::emit_tile, C, smem, again);
        }
    }
}

__global__ __launch_bounds__(256) void kn_sort_up(Batch B, int kind, int p) {
    __shared__ __attribute__((aligned(16))) char smem[kSmemSmall];
    sort_up_units(B, kind, p, blockIdx.x, gridDim.x, smem);
}
__global__ __launch_bounds__(256) void kn_sort_scan(Batch B, int kind, int p) {
    __shared__ __attribute__((aligned(16))) char smem[64];
    sort_scan_units(B, kind, p, blockIdx.x, gridDim.x, smem);
}
__global__ __launch_bounds__(256) void kn_sort_down(Batch B, int kind, int p) {
    __shared__ __attribute__((aligned(16))) char smem[kSmemDown];
    sort_down_units(B, kind, p, blockIdx.x, gridDim.x, smem);
}
// The first emit in two launches, as for a single column: the windows
// folded into the emit (order each tile's view inside its runs of equal
// prefix in LDS, count the run heads; the hashing route's distinct values
// are written at once), then the numbering of the heads from the tiles'
// counts and group sums.
// (One launch per value type, each with its own type's LDS, measured
// slower on the 300-column batch: 8.57 -> 8.65 ms.)
__global__ __launch_bounds__(256) void kn_emit_count(Batch B) {
    __shared__ __attribute__((aligned(16))) char smem[sizeof(mc::EmitWinSmem<mc::TS16>)];
    const uint32_t j = find_col(B, blockIdx.x);
    const mc::ColDesc &C = B.cols[j];
    if (C.drankd) {
        MC_DISPATCH(C, mc::emit_distinct_window_tile, C, blockIdx.x - B.map[j], smem);
    } else {
        MC_DISPATCH(C, mc::emit_count_tile, C, blockIdx.x - B.map[j], smem);
    }
}
template <class T>
__device__ __forceinline__ void emit_write_at(const mc::ColDesc &C, char *smem, uint32_t t) {
    mc::emit_tile_at<T, true>(C, smem, false, t);
}
__global__ __launch_bounds__(256) void kn_emit_write(Batch B) {
    __shared__ __attribute__((aligned(16))) char smem[sizeof(mc::EmitSmem<mc::TS16>)];
    const uint32_t j = find_col(B, blockIdx.x);
    const mc::ColDesc &C = B.cols[j];
    if (C.drankd) return;  // the hashing route's emit is done
    MC_DISPATCH(C, emit_write_at, C, smem, blockIdx.x - B.map[j]);
}
// Step 1(a)'s hashing route for the columns whose deltas take it
__global__ __launch_bounds__(256) void kn_hash_insert(Batch B) {
    __shared__ __attribute__((aligned(16))) char smem[kSmemHash];
    const uint32_t j = find_col(B, blockIdx.x);
    const mc::ColDesc &C = B.cols[j];
    MC_DISPATCH(C, mc::hash_insert_tile, C, blockIdx.x - B.map[j], smem);
}
__global__ __launch_bounds__(256) void kn_compact(Batch B) {
    __shared__ __attribute__((aligned(16))) char smem[sizeof(mc::CompactSmem)];
    const uint32_t j = find_col(B, blockIdx.x);
    const mc::ColDesc &C = B.cols[j];
    MC_DISPATCH(C, mc::compact_tile, C, blockIdx.x - B.map[j], smem);
}
__global__ __launch_bounds__(256) void kn_rank_rows(Batch B) {
    const uint32_t j = find_col(B, blockIdx.x);
    mc::rank_rows_tile(B.cols[j], blockIdx.x - B.map[j]);
}
__global__ __launch_bounds__(256) void kn_merge_part(Batch B) {
    const uint32_t j = find_col(B, blockIdx.x);
    const mc::ColDesc &C = B.cols[j];
    MC_DISPATCH(C, mc::merge_partition, C, blockIdx.x - B.map[j]);
}
// One launch per value type (the map covers that type's columns only), so
// that each sizes its LDS for its own type: more workgroups fit a CU for 4-
// and 8-byte values than the 16-byte tiles allow.
template <class T>
__global__ __launch_bounds__(256) void kn_merge(Batch B) {
    __shared__ __attribute__((aligned(16))) char smem[sizeof(mc::MergeSmem<T>)];
    const uint32_t j = find_col(B, blockIdx.x);
    mc::merge_tile<T>(B.cols[j], smem);
}
__global__ __launch_bounds__(256) void kn_xcompact(Batch B) {
    __shared__ __attribute__((aligned(16))) char smem[sizeof(mc::XCompactSmem)];
    const uint32_t j = find_col(B, blockIdx.x);
    mc::xcompact_tile(B.cols[j], blockIdx.x - B.map[j], smem);
}
template <int CODES>
__global__ __launch_bounds__(256) void kn_repack(Batch B) {
    __shared__ __attribute__((aligned(16))) char smem[sizeof(mc::RepackOutSmem<CODES>)];
    const uint32_t j = find_col(B, blockIdx.x);
    mc::repack_tile<CODES>(B.cols[j], blockIdx.x - B.map[j], smem);
}

// Random-gather reference: out[i] = table[idx[i] % n_table] for 4- or
// 2-byte entries, 8 independent gathers in flight per thread.  Measures the
// ceiling of the re-encode's translation-table lookups for a given table
// footprint, beside the streaming ceiling of k_copy16.
template <class E>
__global__ __launch_bounds__(256) void k_gather_ref(const uint32_t *__restrict__ idx, uint64_t n,
                                                    const E *__restrict__ table, uint32_t n_table,
                                                    uint32_t *__restrict__ out) {
    constexpr int kPer = 8;
    const uint64_t base = (uint64_t)blockIdx.x * 256 * kPer + threadIdx.x;
    uint32_t v[kPer];
#pragma unroll
    for (int j = 0; j < kPer; j++) {
        const uint64_t i = base + (uint64_t)j * 256;
        v[j] = i < n ? idx[i] % n_table : 0u;
    }
    uint32_t r[kPer];
#pragma unroll
    for (int j = 0; j < kPer; j++) r[j] = (uint32_t)table[v[j]];
#pragma unroll
    for (int j = 0; j < kPer; j++) {
        const uint64_t i = base + (uint64_t)j * 256;
        if (i < n) out[i] = r[j];
    }
}

int launch_fill(void *p0, uint64_t bytes0, void *p1, uint64_t bytes1, hipStream_t s) {
    const uint64_t n = (bytes0 > bytes1 ? bytes0 : bytes1) / 4;
    uint32_t grid = (uint32_t)(n / 256 / 4 + 1);
    if (grid > 2048) grid = 2048;
    hipLaunchKernelGGL(k_fill_zero, dim3(grid), dim3(256), 0, s, (uint32_t *)p0, bytes0 / 4,
                       (uint32_t *)p1, bytes1 / 4);
    MC_LAUNCHED("k_fill_zero");
    return MC_OK;
}

// ---------------------------------------------------------------------------
// Single-column step launchers
// ---------------------------------------------------------------------------

template <class T>
int launch_passes(const mc::ColDesc &C, const ColLayout &L, int kind, int passes, hipStream_t s) {
    for (int p = 0; p < passes; p++) {
        hipLaunchKernelGGL(k1_sort_up<T>, dim3(L.sort_tiles), dim3(mc::kBlock), 0, s, C, kind, p);
        MC_LAUNCHED("k1_sort_up");
        hipLaunchKernelGGL(k1_sort_scan<T>,
                           dim3(L.sort_tiles <= mc::kSmallScanTiles ? mc::kSmallScanParts : 256),
                           dim3(mc::kBlock), 0, s, C, kind, p);
        MC_LAUNCHED("k1_sort_scan");
        hipLaunchKernelGGL(k1_sort_down<T>, dim3(L.sort_tiles), dim3(mc::kBlock), 0, s, C, kind, p);
        MC_LAUNCHED("k1_sort_down");
    }
    return MC_OK;
}

template <class T>
int launch_delta_dictionary(const mc::ColDesc &C, const ColLayout &L, uint32_t cus, hipStream_t s,
                            hipEvent_t after_sort) {
    int rc = MC_OK;
    if (C.nd == 0) {
        if (after_sort) MC_HIP(hipEventRecord(after_sort, s));
        return MC_OK;
    }
    if (L.hashed && !L.indexed) {
        hipLaunchKernelGGL(k1_hash_insert<T>, dim3(L.hash_tiles), dim3(mc::kBlock), 0, s, C);
        MC_LAUNCHED("k1_hash_insert");
        hipLaunchKernelGGL(k1_compact<T>, dim3((uint32_t)ceil_div(C.nd, mc::kCompactTile)),
                           dim3(mc::kBlock), 0, s, C);
        MC_LAUNCHED("k1_compact");
    }
    hipLaunchKernelGGL(k1_hist<T>, dim3(L.hist_tiles), dim3(mc::kBlock), 0, s, C);
    MC_LAUNCHED("k1_hist");
    hipLaunchKernelGGL(k1_hist_scan<T>, dim3(1), dim3(mc::kBlock), 0, s, C);
    MC_LAUNCHED("k1_hist_scan");
    // prefix sort: up to three passes (two launches each, or three), then the
    // windows sorted in LDS, folded into the emit (which checks the order)
    if (L.two_launch_pass) {
        for (int slot = 0; slot < mc::kPrefixSlots; slot++) {
            hipLaunchKernelGGL(k1_sort_up2<T>, dim3(L.sort_tiles), dim3(mc::kBlock), 0, s, C, slot);
            MC_LAUNCHED("k1_sort_up2");
            hipLaunchKernelGGL(k1_sort_down2<T>, dim3(L.sort_tiles), dim3(mc::kBlock), 0, s, C, slot);
            MC_LAUNCHED("k1_sort_down2");
        }
    } else {
        rc = launch_passes<T>(C, L, kPassPrefix, mc::kPrefixSlots, s);
        if (rc) return rc;
    }
    if (after_sort) MC_HIP(hipEventRecord(after_sort, s));
    if (L.hashed) {
        hipLaunchKernelGGL(k1_emit_distinct_win<T>, dim3(L.emit_tiles), dim3(mc::kBlock), 0, s, C);
        MC_LAUNCHED("k1_emit_distinct_win");
    } else {
        hipLaunchKernelGGL(k1_emit_count<T>, dim3(L.emit_tiles), dim3(mc::kBlock), 0, s, C);
        MC_LAUNCHED("k1_emit_count");
        hipLaunchKernelGGL(k1_emit_write<T>, dim3(L.emit_tiles), dim3(mc::kBlock), 0, s, C);
        MC_LAUNCHED("k1_emit_write");
    }
    // the full sort and the second emit in one launch, which returns at once
    // unless the order check failed.  At most half the CUs: a CU holds at
    // least 3 of its workgroups (VGPRs), so the launches of up to 6
    // concurrent merges on other streams are resident together.
    {
        const uint32_t grid = std::min<uint32_t>(L.sort_tiles, cus > 1 ? cus / 2 : 1u);
        hipLaunchKernelGGL(k1_full_sort<T>, dim3(grid), dim3(mc::kBlock), 0, s, C);
        MC_LAUNCHED("k1_full_sort");
    }
    if (L.hashed) {
        hipLaunchKernelGGL(k1_rank_rows, dim3(L.hash_tiles), dim3(mc::kBlock), 0, s, C);
        MC_LAUNCHED("k1_rank_rows");
    }
    return MC_OK;
}

template <class T>
int launch_merge(const mc::ColDesc &C, uint64_t merge_tiles, hipStream_t s) {
    const uint64_t grid = merge_tiles ? merge_tiles : 1;
    if (C.mbound) {
        hipLaunchKernelGGL(k1_merge_part<T>, dim3((uint32_t)merge_part_blocks(merge_tiles)),
                           dim3(mc::kBlock), 0, s, C);
        MC_LAUNCHED("k1_merge_part");
    }
    hipLaunchKernelGGL(k1_merge<T>, dim3((uint32_t)grid), dim3(mc::kBlock), 0, s, C);
    MC_LAUNCHED("k1_merge");
    return MC_OK;
}

int launch_repack(const mc::ColDesc &C, uint32_t codes, hipStream_t s,
                  hipEvent_t before_repack = nullptr) {
    if (C.xdev && C.n_um) {
        hipLaunchKernelGGL(k1_xcompact, dim3((uint32_t)ceil_div(C.n_um, mc::kXCompactTile)),
                           dim3(mc::kBlock), 0, s, C);
        MC_LAUNCHED("k1_xcompact");
    }
    if (before_repack) MC_HIP(hipEventRecord(before_repack, s));
    const uint64_t grid = ceil_div(C.n_main + C.nd, codes);
    if (grid == 0) return MC_OK;
    switch (codes) {
        case 1024: hipLaunchKernelGGL(k1_repack<1024>, dim3((uint32_t)grid), dim3(mc::kBlock), 0, s, C); break;
        case 4096: hipLaunchKernelGGL(k1_repack<4096>, dim3((uint32_t)grid), dim3(mc::kBlock), 0, s, C); break;
        default: hipLaunchKernelGGL(k1_repack<2048>, dim3((uint32_t)grid), dim3(mc::kBlock), 0, s, C); break;
    }
    MC_LAUNCHED("k1_repack");
    return MC_OK;
}

// ---------------------------------------------------------------------------
// Argument checks
// ---------------------------------------------------------------------------

// Rows of one column: at 1024 rows per re-encode tile this keeps a launch
// below 2^24 workgroups of 256 threads (2^32 work-items).
constexpr uint64_t kMaxRows = (1ull << 34) - 1024;
// Workgroups of one batched launch (one per tile of every column).
constexpr uint64_t kMaxLaunchTiles = (1ull << 24) - 1;

uint64_t codes_words_bound(uint64_t rows, uint64_t dict_cap) {
    const uint32_t w = mc::code_width(dict_cap);
    return align_up(ceil_div(rows * w, 64), 2);
}

int check_in(const mc_column_in *in) {
    if (!in) return fail(MC_E_ARG, "null input descriptor");
    if (value_len(in->type) == 0) return fail(MC_E_ARG, "unknown value type");
    if (in->bitwidth < 1 || in->bitwidth > 32) return fail(MC_E_ARG, "bitwidth must be 1..32");
    if (in->main_dict_len > (1ull << in->bitwidth))
        return fail(MC_E_ARG, "main dictionary larger than 2^bitwidth");
    if (in->main_dict_len == 0 && in->main_rows > 0)
        return fail(MC_E_ARG, "main rows without a main dictionary");
    if (in->delta_rows >= (1ull << 30)) return fail(MC_E_ARG, "delta_rows must be < 2^30");
    if (in->main_dict_len + in->delta_rows > (1ull << 32))
        return fail(MC_E_ARG, "|U_M| + N_D must be <= 2^32");
    // every per-row launch is a 1-D grid of 256-thread workgroups of at least
    // 1024 rows, and HIP takes fewer than 2^32 work-items per dimension
    if (in->main_rows + in->delta_rows > kMaxRows)
        return fail(MC_E_ARG, "main_rows + delta_rows must be <= 2^34 - 1024");
    if (in->main_dict_len > 0 && !in->main_dict) return fail(MC_E_ARG, "null main_dict");
    if (in->main_rows > 0 && !in->main_codes) return fail(MC_E_ARG, "null main_codes");
    if (in->delta_rows > 0 && !in->delta_values) return fail(MC_E_ARG, "null delta_values");
    if (!aligned16(in->main_dict) || !aligned16(in->main_codes) || !aligned16(in->delta_values))
        return fail(MC_E_ARG, "input buffers must be 16-byte aligned");
    return MC_OK;
}

int check_index(const mc_delta_index *ix) {
    if (!ix) return fail(MC_E_ARG, "null index");
    if (value_len(ix->type) == 0) return fail(MC_E_ARG, "unknown index value type");
    if (ix->capacity >= (1ull << 30)) return fail(MC_E_ARG, "index capacity must be < 2^30");
    if (ix->reserved) return fail(MC_E_ARG, "the index's reserved field must be zero");
    if (!ix->workspace || !aligned16(ix->workspace)) return fail(MC_E_ARG, "bad index workspace");
    if (ix->workspace_bytes < index_layout(ix->type, ix->capacity).size)
        return fail(MC_E_CAP, "index workspace below mc_delta_index_bytes");
    return MC_OK;
}

int check_out(const mc_column_in *in, const mc_column_out *out) {
    if (!out) return fail(MC_E_ARG, "null output descriptor");
    if (!out->result) return fail(MC_E_ARG, "null result pointer");
    if (!aligned16(out->result)) return fail(MC_E_ARG, "result must be 16-byte aligned");
    const uint64_t dict_cap = in->main_dict_len + in->delta_rows;
    const uint64_t rows = in->main_rows + in->delta_rows;
    if (dict_cap > 0 && (!out->new_dict || out->new_dict_cap < dict_cap))
        return fail(MC_E_CAP, "new_dict capacity below |U_M| + N_D");
    if (rows > 0 && (!out->new_codes || out->new_codes_cap_words < codes_words_bound(rows, dict_cap)))
        return fail(MC_E_CAP, "new_codes capacity below the bound");
    if (!aligned16(out->new_dict) || !aligned16(out->new_codes))
        return fail(MC_E_ARG, "output buffers must be 16-byte aligned");
    if (!aligned4(out->x_main) || !aligned4(out->x_delta))
        return fail(MC_E_ARG, "translation tables must be 4-byte aligned");
    return MC_OK;
}

// ---------------------------------------------------------------------------
// Validate mode: U_M order checked on the device before the merge, the error
// word read back after it.
// ---------------------------------------------------------------------------

int launch_check_order(const mc_column_in *in, uint32_t *err, hipStream_t s) {
    if (in->main_dict_len < 2) return MC_OK;
    const uint32_t grid = (uint32_t)std::min<uint64_t>(ceil_div(in->main_dict_len, 256), 2048);
    switch (in->type) {
        case MC_U32:
            hipLaunchKernelGGL(k_check_order<mc::TU32>, dim3(grid), dim3(256), 0, s,
                               in->main_dict, in->main_dict_len, err);
            break;
        case MC_U64:
            hipLaunchKernelGGL(k_check_order<mc::TU64>, dim3(grid), dim3(256), 0, s,
                               in->main_dict, in->main_dict_len, err);
            break;
        default:
            hipLaunchKernelGGL(k_check_order<mc::TS16>, dim3(grid), dim3(256), 0, s,
                               in->main_dict, in->main_dict_len, err);
            break;
    }
    MC_LAUNCHED("k_check_order");
    return MC_OK;
}

// Read the error words of n results after the stream is done; MC_E_DATA
// naming the first column with a data error bit.
int read_errors(const mc_column_out *outs, uint32_t n, hipStream_t s, const char *when) {
    MC_HIP(hipStreamSynchronize(s));
    for (uint32_t j = 0; j < n; j++) {
        uint32_t e = 0;
        MC_HIP(hipMemcpy(&e, &outs[j].result->error, sizeof(e), hipMemcpyDeviceToHost));
        const uint32_t data = e & (MC_DEVERR_CODE_RANGE | MC_DEVERR_DELTA_RANGE | MC_DEVERR_ORDER);
        if (data)
            return fail(MC_E_DATA, std::string(when) + ": column " + std::to_string(j) + ": " +
                                       (data & MC_DEVERR_ORDER ? "main dictionary not strictly "
                                                                 "increasing"
                                        : data & MC_DEVERR_CODE_RANGE
                                            ? "a main code >= |U_M|"
                                            : "a delta index out of range") +
                                       " (error word " + std::to_string(e) + ")");
    }
    return MC_OK;
}

// Step 1 of validate mode for n columns: zero each result, check each U_M's
// order into its error word, wait, report.
int validate_dicts(const mc_column_in *ins, const mc_column_out *outs, uint32_t n,
                   hipStream_t s) {
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    MC_HIP(hipStreamIsCapturing(s, &cap));
    if (cap != hipStreamCaptureStatusNone)
        return fail(MC_E_ARG, "validate mode cannot run on a stream under graph capture");
    for (uint32_t j = 0; j < n; j++) {
        int rc = launch_fill(outs[j].result, sizeof(mc_result), nullptr, 0, s);
        if (rc) return rc;
        rc = launch_check_order(&ins[j], &outs[j].result->error, s);
        if (rc) return rc;
    }
    return read_errors(outs, n, s, "validate");
}

template <class T>
int launch_naive(const mc::ColDesc &C, hipStream_t s) {
    const uint64_t grid = ceil_div(C.n_main + C.nd, mc::kRepackCodes);
    if (grid == 0) return MC_OK;
    hipLaunchKernelGGL(k1_naive<T>, dim3((uint32_t)grid), dim3(mc::kBlock), 0, s, C);
    MC_LAUNCHED("k1_naive");
    return MC_OK;
}

template <class T>
int merge_column_t(mc_ctx *ctx, const mc_column_in *in, const mc_column_out *out, char *ws,
                   const ColLayout &L, hipStream_t s, bool naive = false,
                   const mc_delta_index *ix = nullptr, bool timed = true) {
    mc::ColDesc C = make_desc(in, out, ws, ws + L.z_size, L);
    if (ix) set_index_fields(C, ix);
    hipEvent_t *ev = nullptr;
    if (ctx->timing && timed) {
        if (ctx->used == ctx->ev.size()) {
            std::array<hipEvent_t, 6> set{};
            for (auto &e : set) MC_HIP(hipEventCreate(&e));
            ctx->ev.push_back(set);
        }
        ev = ctx->ev[ctx->used].data();
        MC_HIP(hipEventRecord(ev[0], s));
    }
    int rc = launch_fill(ws, L.z_size, out->result, sizeof(mc_result), s);
    if (rc) return rc;
    if (ix) {
        const IndexLayout X = index_layout(ix->type, ix->capacity);
        hipLaunchKernelGGL(k_or_word, dim3(1), dim3(64), 0, s, C.err,
                           reinterpret_cast<const uint32_t *>(
                               static_cast<char *>(ix->workspace) + X.scal + 80));
        MC_LAUNCHED("k_or_word");
    }
    rc = launch_delta_dictionary<T>(C, L, ctx->cus, s, ev ? ev[1] : nullptr);
    if (rc) return rc;
    if (ev) MC_HIP(hipEventRecord(ev[2], s));
    rc = launch_merge<T>(C, L.merge_tiles, s);
    if (rc) return rc;
    if (ev) MC_HIP(hipEventRecord(ev[3], s));
    if (naive) {
        if (ev) MC_HIP(hipEventRecord(ev[4], s));
        rc = launch_naive<T>(C, s);
    } else {
        rc = launch_repack(C, L.repack_codes, s, ev ? ev[4] : nullptr);
    }
    if (rc) return rc;
    if (ev) {
        MC_HIP(hipEventRecord(ev[5], s));
        ctx->used++;
    }
    return MC_OK;
}

int merge_column_impl(mc_ctx *ctx, const mc_column_in *in, const mc_column_out *out,
                      void *scratch, uint64_t scratch_bytes, hipStream_t s, bool naive = false) {
    if (!ctx) return fail(MC_E_ARG, "null context");
    int rc = check_in(in);
    if (rc) return rc;
    rc = check_out(in, out);
    if (rc) return rc;
    const ColLayout L =
        col_layout(in->type, in->main_dict_len, in->delta_rows, in->main_rows, true, ctx->tune);
    if (!scratch || scratch_bytes < single_scratch(L))
        return fail(MC_E_CAP, "scratch below mc_merge_bounds");
    if (!aligned16(scratch)) return fail(MC_E_ARG, "scratch must be 16-byte aligned");
    if (ctx->validate) {
        rc = validate_dicts(in, out, 1, s);
        if (rc) return rc;
    }
    char *ws = static_cast<char *>(scratch);
    switch (in->type) {
        case MC_U32: rc = merge_column_t<mc::TU32>(ctx, in, out, ws, L, s, naive); break;
        case MC_U64: rc = merge_column_t<mc::TU64>(ctx, in, out, ws, L, s, naive); break;
        default: rc = merge_column_t<mc::TS16>(ctx, in, out, ws, L, s, naive); break;
    }
    if (rc == MC_OK && ctx->validate) rc = read_errors(out, 1, s, "merge");
    return rc;
}

// ---------------------------------------------------------------------------
// Batched plan: every column's workspace, the device descriptor array and
// the per-phase tile maps, all inside the caller's scratch.
// ---------------------------------------------------------------------------

constexpr int kMaxPasses = 16;
// map slots: 0 hist, 1 hist_scan, 2 sort tiles (prefix pass up/down,
// the persistent launch's windows), 3 prefix pass scan, 4 emit, 5..7 merge of the u32 / u64 / str16
// columns, 8 repack, 9 X_M compaction, 10 merge tile boundaries, 11 hash
// insert, 12 compaction of the distinct values, 13 row ranks, 14..29
// fallback pass p up/down (tiles) and 30..45 fallback pass p scan (digits or
// parts), columns with at least p + 1 digit positions, 46 fallback emit: the
// per-column counts of every column with a delta, from which kn_full_sort builds
// the device maps of the columns that need the full sort (device slot p: pass
// p, kMaxPasses + p: scan p, 2 kMaxPasses: emit)
// kMapRepack + 0, 1, 2: the re-encode tiles of the columns whose tile is
// 1024, 2048 or 4096 codes (one launch each; per-class shapes may mix them)
constexpr int kMapHist = 0, kMapHistScan = 1, kMapPass = 2, kMapScan = 3, kMapEmit = 4,
              kMapMerge = 5, kMapRepack = 8, kMapXc = 11, kMapMergePart = 12, kMapHash = 13,
              kMapCompact = 14, kMapRank = 15, kMapFbPass = 16,
              kMapFbScan = kMapFbPass + kMaxPasses, kMapFbEmit = kMapFbScan + kMaxPasses,
              kNumMaps = kMapFbEmit + 1;
int repack_slot(uint32_t codes) { return codes == 1024u ? 0 : codes == 4096u ? 2 : 1; }
constexpr int kNumDevMaps = 2 * kMaxPasses + 1;

// The fallback's maps, one workgroup per device slot s: column j keeps its
// count of the host slot when the prefix sort left it unsorted, else 0;
// exclusive prefix over the columns, the total in entry ncols.  part: 256
// words of LDS.
__device__ void fb_plan_slot(const Batch &B, const uint32_t *hmaps, uint32_t *dmaps,
                             uint32_t npass, uint32_t s, uint32_t *part) {
    const uint32_t hs = s < npass ? kMapFbPass + s
                                  : (s < 2 * npass ? kMapFbScan + (s - npass) : kMapFbEmit);
    const uint32_t ds = s < npass ? s : (s < 2 * npass ? kMaxPasses + (s - npass) : 2 * kMaxPasses);
    const uint32_t n = B.ncols;
    const uint32_t *src = hmaps + (size_t)hs * (n + 1);
    uint32_t *dst = dmaps + (size_t)ds * (n + 1);
    const uint32_t per = (n + 255) / 256;
    const uint32_t j0 = min(n, threadIdx.x * per), j1 = min(n, j0 + per);
    auto count = [&](uint32_t j) -> uint32_t {
        const uint32_t c = src[j + 1] - src[j];
        return c && B.cols[j].sflags[mc::kSfUnsorted] ? c : 0u;
    };
    uint32_t sum = 0;
    for (uint32_t j = j0; j < j1; j++) sum += count(j);
    part[threadIdx.x] = sum;
    __syncthreads();
    for (uint32_t off = 1; off < 256; off <<= 1) {  // inclusive scan of the parts
        const uint32_t v = threadIdx.x >= off ? part[threadIdx.x - off] : 0u;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    uint32_t acc = part[threadIdx.x] - sum;
    for (uint32_t j = j0; j < j1; j++) {
        dst[j] = acc;
        acc += count(j);
    }
    if (threadIdx.x == 255) dst[n] = part[255];
}

// The batched fallback in one launch (as k1_full_sort for one column): it
// returns at once when every column's order check passed, where the launch
// per phase it replaces cost 3 launches per digit position (48 for 16-byte
// values) plus the plan and the second emit, about 160 us per batch of
// launches that returned at once.  Otherwise its workgroups (at most one
// per two compute units, so all are resident; see k1_full_sort) build the
// device maps of the unsorted columns, run every pass's phases striding over
// them, and the second emit, with a grid-wide barrier between phases.  A
// barrier that overruns its bounded wait marks every unsorted column's
// error word.
constexpr size_t kSmemFull = std::max(std::max(kSmemDown, sizeof(mc::EmitSmem<mc::TS16>)),
                                      (size_t)256 * 4);
__device__ void fb_spin_error(const Batch &B) {
    for (uint32_t j = threadIdx.x; j < B.ncols; j += blockDim.x)
        if (B.cols[j].sflags[mc::kSfUnsorted]) mc::flag_error(B.cols[j].err, MC_DEVERR_SPIN);
}
__global__ __launch_bounds__(256) void kn_full_sort(Batch B, const uint32_t *hmaps, uint32_t *dmaps,
                                                    uint32_t npass, uint32_t *bar) {
    __shared__ __attribute__((aligned(16))) char smem[kSmemFull];
    __shared__ uint32_t s_first, s_ok;
    const uint32_t n = B.ncols;
    if (threadIdx.x == 0) s_first = n;
    __syncthreads();
    for (uint32_t j = threadIdx.x; j < n; j += blockDim.x)
        if (B.cols[j].sflags[mc::kSfUnsorted]) atomicMin(&s_first, j);
    __syncthreads();
    if (s_first == n) return;
    uint32_t *err = B.cols[s_first].err;  // the first unsorted column's
    const uint32_t G = gridDim.x;
    uint32_t target = 0;
    auto barrier = [&]() -> bool {
        target += G;
        if (mc::grid_barrier(bar, target, err, &s_ok)) return true;
        fb_spin_error(B);
        return false;
    };
    for (uint32_t sl = blockIdx.x; sl < 2 * npass + 1; sl += G) {
        fb_plan_slot(B, hmaps, dmaps, npass, sl, reinterpret_cast<uint32_t *>(smem));
        __syncthreads();
    }
    if (!barrier()) return;
    auto dmap = [&](uint32_t ds) {
        Batch D = B;
        D.map = dmaps + (size_t)ds * (n + 1);
        return D;
    };
    for (uint32_t p = 0; p < npass; p++) {
        sort_up_units(dmap(p), kPassFull, (int)p, blockIdx.x, G, smem);
        if (!barrier()) return;
        sort_scan_units(dmap(kMaxPasses + p), kPassFull, (int)p, blockIdx.x, G, smem);
        if (!barrier()) return;
        sort_down_units(dmap(p), kPassFull, (int)p, blockIdx.x, G, smem);
        if (!barrier()) return;
    }
    emit_units(dmap(2 * kMaxPasses), true, blockIdx.x, G, smem);
}

struct BatchPlan {
    uint64_t z_total = 0, b_total = 0, desc_off = 0, map_off = 0, dmap_off = 0, total = 0;
    std::vector<uint64_t> z_off, b_off;
    std::vector<ColLayout> L;
    std::vector<uint32_t> maps;  // kNumMaps x (ncols + 1)
    uint32_t max_passes = 0;
    uint32_t repack_codes = mc::kRepackCodes;
    // the persistent launch: its queue plan, the tables' offsets in the
    // copied block (after the maps), the queue counters' offset in the
    // zeroed part, and the item sizes
    bool persistent = false;
    mcq::Plan q;
    uint64_t q_off = 0, qbase_off = 0, qpmap_off = 0, qcum_off = 0, qgcum_off = 0;
    uint64_t fb_bar_off = 0;  // the one-launch fallback's barrier counter (zeroed part)
    uint32_t repack_per = kPersistRepack, merge_per = kPersistMerge, workers = 0;
};

// Item counts of the persistent launch: per column and phase (ncols x
// kNumPhases), and of the global fallback phases.
void persist_counts(const mc_column_in *ins, uint32_t ncols, const BatchPlan &P,
                    std::vector<uint32_t> &counts, std::vector<uint32_t> &gcount) {
    counts.assign((size_t)ncols * mcq::kNumPhases, 0u);
    gcount.assign(mcq::kNumPhases, 0u);
    for (uint32_t j = 0; j < ncols; j++) {
        const ColLayout &L = P.L[j];
        const bool d = ins[j].delta_rows > 0;
        uint32_t *c = &counts[(size_t)j * mcq::kNumPhases];
        const uint32_t scan = L.sort_tiles <= mc::kSmallScanTiles ? mc::kSmallScanParts : 256u;
        c[mcq::kHash] = L.hashed ? L.hash_tiles : 0;
        c[mcq::kCompact] = L.hashed ? (uint32_t)ceil_div(ins[j].delta_rows, mc::kCompactTile) : 0;
        c[mcq::kHist] = L.hist_tiles;
        c[mcq::kHScan] = d ? 1 : 0;
        for (uint32_t sl = 0; sl < (uint32_t)mc::kPrefixSlots; sl++) {
            c[mcq::kPre0Up + 3 * sl] = d ? L.sort_tiles : 0;
            c[mcq::kPre0Up + 3 * sl + 1] = d ? scan : 0;
            c[mcq::kPre0Up + 3 * sl + 2] = d ? L.sort_tiles : 0;
        }
        c[mcq::kWin0] = c[mcq::kWin1] = d ? L.sort_tiles : 0;
        c[mcq::kEmit] = L.emit_tiles;
        c[mcq::kRank] = L.hashed ? L.hash_tiles : 0;
        c[mcq::kMPart] = L.partitioned ? (uint32_t)merge_part_blocks(L.merge_tiles) : 0;
        c[mcq::kMerge] = (uint32_t)ceil_div(L.merge_tiles ? L.merge_tiles : 1, P.merge_per);
        c[mcq::kXc] = (uint32_t)L.xc_tiles;
        c[mcq::kRepack] = (uint32_t)ceil_div(L.repack_tiles, P.repack_per);
    }
    if (P.max_passes) {
        gcount[mcq::kFbPlan] = 2 * P.max_passes + 1;  // one map slot each
        for (uint32_t p = 0; p < P.max_passes; p++)
            for (uint32_t k = 0; k < 3; k++) gcount[mcq::kFbPass0 + 3 * p + k] = kPersistFbItems;
        gcount[mcq::kFbEmit] = kPersistFbItems;
    }
}

int batched_run(mc_ctx *ctx, const mc_column_in *ins, const mc_column_out *outs, uint32_t ncols,
                void *scratch, uint64_t scratch_bytes, hipStream_t stream, const mc_tuning &tune,
                mc_graph **graph, bool use_classes = true);

// Tuning class of a column: value type, input code width class (1-8, 9-16,
// 17-24, 25-32) and size class (main + delta rows below 2^21, below 2^24,
// or more).
uint32_t tune_class_of(const mc_column_in &in) {
    const uint32_t w = in.bitwidth;
    const uint64_t n = in.main_rows + in.delta_rows;
    const uint32_t wc = w <= 8 ? 0u : w <= 16 ? 1u : w <= 24 ? 2u : 3u;
    const uint32_t sc = n < (1ull << 21) ? 0u : n < (1ull << 24) ? 1u : 2u;
    return ((uint32_t)in.type * 4u + wc) * 3u + sc;
}

// classes: the context whose per-class shapes apply, or null (every column
// takes `tune`; also the persistent launch, which has one tile size).
int plan_batch(const mc_column_in *ins, uint32_t ncols, BatchPlan &P,
               const mc_tuning &tune = kDefaultTuning, const mc_ctx *classes = nullptr) {
    P.repack_codes = tune.repack_codes;
    if (tune.batched_launch == MC_BATCHED_PERSISTENT) classes = nullptr;
    P.z_off.resize(ncols);
    P.b_off.resize(ncols);
    P.L.resize(ncols);
    P.maps.assign((size_t)kNumMaps * (ncols + 1), 0u);
    uint64_t z = 0, b = 0;
    for (uint32_t i = 0; i < ncols; i++) {
        int rc = check_in(&ins[i]);
        if (rc) return rc;
        // each column takes the Step 1(a) route it would take alone, with
        // its class's shapes if the context has them
        mc_tuning ti = tune;
        if (classes) {
            const uint32_t c = tune_class_of(ins[i]);
            if (classes->class_set[c]) {
                ti.repack_codes = classes->class_tune[c].repack_codes;
                ti.prefix_run = classes->class_tune[c].prefix_run;
            }
        }
        P.L[i] = col_layout(ins[i].type, ins[i].main_dict_len, ins[i].delta_rows,
                            ins[i].main_rows, /*allow_hash=*/true, ti, /*indexed=*/false,
                            /*batched=*/true);
        P.z_off[i] = z;
        z += P.L[i].z_size;
        P.b_off[i] = b;
        b += P.L[i].b_size;
        if (ins[i].delta_rows > 0 && P.L[i].passes > P.max_passes) P.max_passes = P.L[i].passes;
    }
    P.persistent = tune.batched_launch == MC_BATCHED_PERSISTENT;
    P.repack_per = tune.persist_repack ? tune.persist_repack : kPersistRepack;
    P.merge_per = tune.persist_merge ? tune.persist_merge : kPersistMerge;
    P.workers = tune.persist_workers;
    if (P.max_passes && !P.persistent) {  // the fallback's barrier counter
        z = align_up(z, 256);
        P.fb_bar_off = z;
        z += 4;
    }
    if (P.persistent) {  // queue counters after the columns' zeroed parts
        z = align_up(z, 256);
        P.q_off = z;
        z += (uint64_t)(kQColDone + ncols) * 4;
    }
    P.z_total = align_up(z, 256);
    P.b_total = align_up(b, 256);
    P.desc_off = P.z_total + P.b_total;
    P.map_off = P.desc_off + align_up((uint64_t)ncols * sizeof(mc::ColDesc), 256);
    uint64_t after_maps = P.map_off + align_up((uint64_t)P.maps.size() * 4, 256);
    if (P.persistent) {  // the queue tables travel with the maps
        const uint64_t NP = mcq::kNumPhases;
        P.qbase_off = after_maps;
        P.qgcum_off = P.qbase_off + align_up((NP + 1) * 4, 256);
        P.qpmap_off = P.qgcum_off + align_up(NP * 4, 256);
        P.qcum_off = P.qpmap_off + align_up(NP * (ncols + 1) * 4, 256);
        after_maps = P.qcum_off + align_up((uint64_t)ncols * NP * 4, 256);
    }
    P.dmap_off = after_maps;
    P.total = P.dmap_off + align_up((uint64_t)kNumDevMaps * (ncols + 1) * 4, 256);
    // tile-count prefixes per phase
    auto at = [&](int m, uint32_t j) -> uint32_t & { return P.maps[(size_t)m * (ncols + 1) + j]; };
    for (int m = 0; m < kNumMaps; m++) {
        uint64_t acc = 0;
        for (uint32_t j = 0; j < ncols; j++) {
            const ColLayout &L = P.L[j];
            const bool has_delta = ins[j].delta_rows > 0;
            uint64_t n = 0;
            if (m == kMapHist) n = L.hist_tiles;
            else if (m == kMapHistScan) n = has_delta ? 1 : 0;
            else if (m == kMapPass) n = has_delta ? L.sort_tiles : 0;
            else if (m == kMapScan)  // the prefix passes of three launches only
                n = has_delta && !L.two_launch_pass
                        ? (L.sort_tiles <= mc::kSmallScanTiles ? mc::kSmallScanParts : 256)
                        : 0;
            else if (m >= kMapFbPass && m < kMapFbPass + kMaxPasses)
                n = (has_delta && (uint32_t)(m - kMapFbPass) < L.passes)
                        ? L.sort_tiles
                        : 0;
            else if (m >= kMapFbScan && m < kMapFbScan + kMaxPasses)
                n = (has_delta && (uint32_t)(m - kMapFbScan) < L.passes)
                        ? (L.sort_tiles <= mc::kSmallScanTiles ? mc::kSmallScanParts
                                                               : 256u)
                        : 0;
            else if (m == kMapEmit) n = L.emit_tiles;
            else if (m == kMapFbEmit) n = has_delta ? L.emit_tiles : 0;
            else if (m >= kMapMerge && m < kMapMerge + 3)
                n = (int)ins[j].type == m - kMapMerge ? (L.merge_tiles ? L.merge_tiles : 1) : 0;
            else if (m >= kMapRepack && m < kMapRepack + 3)
                n = repack_slot(L.repack_codes) == m - kMapRepack ? L.repack_tiles : 0;
            else if (m == kMapXc) n = L.xc_tiles;
            else if (m == kMapMergePart) n = L.partitioned ? merge_part_blocks(L.merge_tiles) : 0;
            else if (m == kMapHash || m == kMapRank) n = L.hashed ? L.hash_tiles : 0;
            else if (m == kMapCompact)
                n = L.hashed ? ceil_div(ins[j].delta_rows, mc::kCompactTile) : 0;
            at(m, j) = (uint32_t)acc;
            acc += n;
            if (acc > kMaxLaunchTiles)
                return fail(MC_E_ARG, "batch has too many tiles for one launch (2^24 - 1)");
        }
        at(m, ncols) = (uint32_t)acc;
    }
    if (P.persistent) {
        std::vector<uint32_t> counts, gcount;
        persist_counts(ins, ncols, P, counts, gcount);
        if (!mcq::build_plan(ncols, counts, gcount, P.q))
            return fail(MC_E_ARG, "batch has too many work items for one persistent launch");
    }
    return MC_OK;
}

// Enqueue the batched launch sequence (descriptors and maps already on the device).
int enqueue_batch(const BatchPlan &P, uint32_t ncols, char *ws, uint32_t cus, hipStream_t s) {
    const mc::ColDesc *d_cols = reinterpret_cast<const mc::ColDesc *>(ws + P.desc_off);
    const uint32_t *d_maps = reinterpret_cast<const uint32_t *>(ws + P.map_off);
    uint32_t *d_dmaps = reinterpret_cast<uint32_t *>(ws + P.dmap_off);
    auto batch = [&](int m) {
        Batch B;
        B.cols = d_cols;
        B.map = d_maps + (size_t)m * (ncols + 1);
        B.ncols = ncols;
        return B;
    };
    auto tiles = [&](int m) { return P.maps[(size_t)m * (ncols + 1) + ncols]; };
    int rc = launch_fill(ws, P.z_total, nullptr, 0, s);
    if (rc) return rc;
    hipLaunchKernelGGL(kn_zero_results, dim3((ncols + 255) / 256), dim3(256), 0, s, batch(0));
    MC_LAUNCHED("kn_zero_results");
    if (tiles(kMapHash)) {
        // hashing route: distinct values first, then the sort phases see only them
        hipLaunchKernelGGL(kn_hash_insert, dim3(tiles(kMapHash)), dim3(mc::kBlock), 0, s,
                           batch(kMapHash));
        MC_LAUNCHED("kn_hash_insert");
        hipLaunchKernelGGL(kn_compact, dim3(tiles(kMapCompact)), dim3(mc::kBlock), 0, s,
                           batch(kMapCompact));
        MC_LAUNCHED("kn_compact");
    }
    if (tiles(kMapHist)) {
        hipLaunchKernelGGL(kn_hist, dim3(tiles(kMapHist)), dim3(mc::kBlock), 0, s, batch(kMapHist));
        MC_LAUNCHED("kn_hist");
        hipLaunchKernelGGL(kn_hist_scan, dim3(tiles(kMapHistScan)), dim3(mc::kBlock), 0, s,
                           batch(kMapHistScan));
        MC_LAUNCHED("kn_hist_scan");
    }
    if (P.max_passes) {
        // the prefix passes: one workgroup per tile of every column with a
        // delta; the scan launch only for columns whose passes take three
        for (int p = 0; p < mc::kPrefixSlots; p++) {
            const uint32_t tp = tiles(kMapPass), ts = tiles(kMapScan);
            hipLaunchKernelGGL(kn_sort_up, dim3(tp), dim3(mc::kBlock), 0, s, batch(kMapPass),
                               kPassPrefix, p);
            MC_LAUNCHED("kn_sort_up");
            if (ts) {
                hipLaunchKernelGGL(kn_sort_scan, dim3(ts), dim3(mc::kBlock), 0, s,
                                   batch(kMapScan), kPassPrefix, p);
                MC_LAUNCHED("kn_sort_scan");
            }
            hipLaunchKernelGGL(kn_sort_down, dim3(tp), dim3(mc::kBlock), 0, s, batch(kMapPass),
                               kPassPrefix, p);
            MC_LAUNCHED("kn_sort_down");
        }
    }
    if (tiles(kMapEmit)) {
        // the emit with the windows folded in, then the numbering of the heads
        hipLaunchKernelGGL(kn_emit_count, dim3(tiles(kMapEmit)), dim3(mc::kBlock), 0, s,
                           batch(kMapEmit));
        MC_LAUNCHED("kn_emit_count");
        hipLaunchKernelGGL(kn_emit_write, dim3(tiles(kMapEmit)), dim3(mc::kBlock), 0, s,
                           batch(kMapEmit));
        MC_LAUNCHED("kn_emit_write");
        if (P.max_passes) {  // the full sort of the columns found unsorted, and their emit
            const uint32_t grid =
                std::max(1u, std::min(tiles(kMapFbPass), cus > 1 ? cus / 2 : 1u));
            hipLaunchKernelGGL(kn_full_sort, dim3(grid), dim3(mc::kBlock), 0, s, batch(0), d_maps,
                               d_dmaps, P.max_passes,
                               reinterpret_cast<uint32_t *>(ws + P.fb_bar_off));
            MC_LAUNCHED("kn_full_sort");
        }
    }
    if (tiles(kMapRank)) {
        hipLaunchKernelGGL(kn_rank_rows, dim3(tiles(kMapRank)), dim3(mc::kBlock), 0, s,
                           batch(kMapRank));
        MC_LAUNCHED("kn_rank_rows");
    }
    if (tiles(kMapMergePart)) {
        hipLaunchKernelGGL(kn_merge_part, dim3(tiles(kMapMergePart)), dim3(mc::kBlock), 0, s,
                           batch(kMapMergePart));
        MC_LAUNCHED("kn_merge_part");
    }
    if (tiles(kMapMerge + MC_U32)) {
        hipLaunchKernelGGL(kn_merge<mc::TU32>, dim3(tiles(kMapMerge + MC_U32)), dim3(mc::kBlock),
                           0, s, batch(kMapMerge + MC_U32));
        MC_LAUNCHED("kn_merge<u32>");
    }
    if (tiles(kMapMerge + MC_U64)) {
        hipLaunchKernelGGL(kn_merge<mc::TU64>, dim3(tiles(kMapMerge + MC_U64)), dim3(mc::kBlock),
                           0, s, batch(kMapMerge + MC_U64));
        MC_LAUNCHED("kn_merge<u64>");
    }
    if (tiles(kMapMerge + MC_STR16)) {
        hipLaunchKernelGGL(kn_merge<mc::TS16>, dim3(tiles(kMapMerge + MC_STR16)),
                           dim3(mc::kBlock), 0, s, batch(kMapMerge + MC_STR16));
        MC_LAUNCHED("kn_merge<str16>");
    }
    if (tiles(kMapXc)) {
        hipLaunchKernelGGL(kn_xcompact, dim3(tiles(kMapXc)), dim3(mc::kBlock), 0, s, batch(kMapXc));
        MC_LAUNCHED("kn_xcompact");
    }
    const dim3 rb(mc::kBlock);
    if (tiles(kMapRepack + 1)) {
        hipLaunchKernelGGL(kn_repack<2048>, dim3(tiles(kMapRepack + 1)), rb, 0, s, batch(kMapRepack + 1));
        MC_LAUNCHED("kn_repack<2048>");
    }
    if (tiles(kMapRepack)) {
        hipLaunchKernelGGL(kn_repack<1024>, dim3(tiles(kMapRepack)), rb, 0, s, batch(kMapRepack));
        MC_LAUNCHED("kn_repack<1024>");
    }
    if (tiles(kMapRepack + 2)) {
        hipLaunchKernelGGL(kn_repack<4096>, dim3(tiles(kMapRepack + 2)), rb, 0, s, batch(kMapRepack + 2));
        MC_LAUNCHED("kn_repack<4096>");
    }
    return MC_OK;
}

// ---------------------------------------------------------------------------
// The batched merge as one persistent launch (queue.hpp): a prologue kernel
// clears the workspace's zeroed part, the queue counters and the results;
// then every worker of kn_persist takes tickets from one counter, decodes the
// item (phase, column, index), waits for the item's dependencies (bounded),
// runs the same tile function as the per-phase launches, and counts the item
// done.  Items of the re-encode and the dictionary merge are several tiles
// each (repack_per / merge_per), to spread the per-item cost of the ticket,
// the decode and the wait.
// ---------------------------------------------------------------------------

struct PersistArgs {
    const mc::ColDesc *cols;
    uint32_t ncols;
    uint32_t total;           // tickets
    const uint32_t *base;     // kNumPhases + 1 first tickets
    const uint32_t *pmap;     // kNumPhases x (ncols + 1) column prefixes
    const uint32_t *cum;      // ncols x kNumPhases: column counter targets
    const uint32_t *gcum;     // kNumPhases: fallback counter targets
    uint32_t emit_total;      // emit items of all columns
    uint32_t fb_total;        // items of the global fallback phases
    uint32_t *q;              // queue counters (kQ*), then one done counter per column
    const uint32_t *hmaps;    // per-phase host maps of the batch (fallback slots used)
    uint32_t *dmaps;          // device-built maps of the columns that need the fallback
    uint32_t npass;           // fallback passes (largest value length of the batch)
    uint32_t fb_items;        // items of each global fallback pass phase
    uint32_t merge_per;       // merge tiles per item
    uint32_t repack_per;      // re-encode tiles per item
};

struct PersistSmem {
    uint32_t base[mcq::kNumPhases + 1];
    uint32_t ticket, ph, col, idx, abort;
};

__device__ __forceinline__ uint32_t ld_u32(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Thread 0 waits until *ctr >= target; then every thread of the workgroup
// acquires (the XCDs' L2 caches are not coherent with each other).  Many
// workgroups can wait on one counter at once (every item of a column's next
// phase, every item of the fallback chain), and device-scope loads of one
// word are served one after another, so the polls back off exponentially
// (about 128 to 8,000 clocks apart) to leave room for the increments they
// wait for.  The wait is bounded by time (2 s of the constant 100 MHz
// clock): on overrun the error bit goes to the item's error word and to the
// launch's abort word; then every worker skips the rest of its items (see
// kn_persist), so the launch ends soon after one overrun, with every
// column's error word flagged.  Returns whether the launch is aborting
// (the same value for every thread of the workgroup).
constexpr uint64_t kQueueWaitTicks = 200000000ull;  // 2 s at 100 MHz
__device__ __forceinline__ bool queue_wait(const uint32_t *ctr, uint32_t target, uint32_t *err,
                                           uint32_t *abort_word, uint32_t *s_abort) {
    if (threadIdx.x == 0) {
        uint32_t ab = ld_u32(abort_word) & MC_DEVERR_SPIN;
        if (!ab && ld_u32(ctr) < target) {
            const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
            uint32_t nap = 1;  // s_sleep(2) rounds (about 128 clocks each) between polls
            while (true) {
                for (uint32_t q = 0; q < nap; q++) __builtin_amdgcn_s_sleep(2);
                if (ld_u32(ctr) >= target) break;
                ab = ld_u32(abort_word) & MC_DEVERR_SPIN;
                if (ab) break;
                if (__builtin_amdgcn_s_memrealtime() - t0 > kQueueWaitTicks) {
                    mc::flag_error(abort_word, MC_DEVERR_SPIN);
                    ab = MC_DEVERR_SPIN;
                    break;
                }
                if (nap < 64) nap <<= 1;
            }
        }
        if (ab) mc::flag_error(err, MC_DEVERR_SPIN);
        *s_abort = ab;
    }
    __syncthreads();
    __threadfence();
    return *s_abort != 0;
}

// Decode ticket k with wave 0 (64-lane searches: the phase over the staged
// bases, then the column over the phase's prefix map); the result lands in S.
__device__ inline void queue_decode(const PersistArgs &A, PersistSmem &S, uint32_t k) {
    if (mc::wave_id() != 0) return;
    const int lane = mc::lane_id();
    constexpr uint32_t NP = mcq::kNumPhases;
    // phase = number of x in [1, NP) with base[x] <= k (bases never decrease)
    uint32_t ph = 0;
#pragma unroll
    for (uint32_t r = 0; r < 2; r++) {
        const uint32_t x = r * 64 + (uint32_t)lane;
        ph += (uint32_t)__popcll(__ballot(x >= 1 && x < NP && S.base[x] <= k));
    }
    const uint32_t off = k - S.base[ph];
    uint32_t col = 0, idx = off;
    if (!mcq::is_global(ph)) {
        const uint32_t *m = A.pmap + (size_t)ph * (A.ncols + 1);
        // the last column j in [lo, hi) with m[j] <= off (m[0] = 0 <= off)
        uint32_t lo = 0, hi = A.ncols;
        while (hi - lo > 1) {
            const uint32_t step = (hi - lo + 63) / 64;
            const uint32_t x = lo + (uint32_t)lane * step;
            const bool pred = lane >= 1 && x < hi && m[x] <= off;
            const uint32_t cnt = (uint32_t)__popcll(__ballot(pred));
            lo += cnt * step;
            hi = min(hi, lo + step);
        }
        col = lo;
        idx = off - m[lo];
    }
    if (lane == 0) {
        S.ph = ph;
        S.col = col;
        S.idx = idx;
    }
}

template <class T>
__device__ __forceinline__ uint32_t merge_tiles_of(const mc::ColDesc &C) {
    const uint64_t t = (C.n_um + C.nd_max + mc::merge_tile<T>() - 1) / mc::merge_tile<T>();
    return t ? (uint32_t)t : 1u;
}

// One item of a per-column phase.
template <int CODES>
__device__ void run_column_item(const PersistArgs &A, uint32_t ph, uint32_t j, uint32_t idx,
                                char *smem) {
    const mc::ColDesc &C = A.cols[j];
    if (ph == mcq::kHash) {
        MC_DISPATCH(C, mc::hash_insert_tile, C, idx, smem);
    } else if (ph == mcq::kCompact) {
        MC_DISPATCH(C, mc::compact_tile, C, idx, smem);
    } else if (ph == mcq::kHist) {
        MC_DISPATCH(C, mc::hist_tile, C, idx, smem);
    } else if (ph == mcq::kHScan) {
        MC_DISPATCH(C, mc::hist_scan_col, C, smem);
    } else if (ph >= mcq::kPre0Up && ph < mcq::kWin0) {
        const int slot = (int)(ph - mcq::kPre0Up) / 3, kind = (int)(ph - mcq::kPre0Up) % 3;
        const mc::PassIO io = mc::prefix_io(C, slot);
        if (kind == 0) {
            MC_DISPATCH(C, mc::sort_up_tile, C, io, idx, smem);
        } else if (kind == 1) {
            if (C.sort_tiles <= mc::kSmallScanTiles) {
                MC_DISPATCH(C, mc::sort_scan_small, C, io, idx);
            } else {
                MC_DISPATCH(C, mc::sort_scan_digit, C, io, idx, smem);
            }
        } else {
            MC_DISPATCH(C, mc::sort_down_tile, C, io, idx, smem);
        }
    } else if (ph == mcq::kWin0) {
        MC_DISPATCH(C, mc::window_sort_tile, C, idx, smem);
    } else if (ph == mcq::kWin1) {
        MC_DISPATCH(C, mc::window_seam_tile, C, idx, smem);
    } else if (ph == mcq::kEmit) {
        if (C.drankd) {
            MC_DISPATCH(C, mc::emit_distinct_tile, C, idx, false);
        } else {
            MC_DISPATCH(C, mc::emit_tile, C, smem, false);
        }
    } else if (ph == mcq::kRank) {
        mc::rank_rows_tile(C, idx);
    } else if (ph == mcq::kMPart) {
        MC_DISPATCH(C, mc::merge_partition, C, idx);
    } else if (ph == mcq::kMerge) {
        // tiles [idx * merge_per, ...) of the column, each from its own ticket
        uint32_t n = 0;
        MC_DISPATCH_R(C, n, merge_tiles_of);
        const uint32_t t0 = idx * A.merge_per, t1 = min(n, t0 + A.merge_per);
        for (uint32_t t = t0; t < t1; t++) {
            if (t != t0) __syncthreads();
            MC_DISPATCH(C, mc::merge_tile, C, smem);
        }
    } else if (ph == mcq::kXc) {
        mc::xcompact_tile(C, idx, smem);
    } else if (ph == mcq::kRepack) {
        const uint64_t n = (C.n_main + C.nd + CODES - 1) / CODES;
        const uint64_t t0 = (uint64_t)idx * A.repack_per;
        const uint64_t t1 = min<uint64_t>(n, t0 + A.repack_per);
        for (uint64_t t = t0; t < t1; t++) {
            if (t != t0) __syncthreads();
            mc::repack_tile<CODES>(C, t, smem);
        }
    }
}

// One item of a global fallback phase: item i strides over the device-built
// map of the phase (only the columns the prefix sort left unsorted).
__device__ void run_fallback_item(const PersistArgs &A, PersistSmem &S, uint32_t ph, uint32_t i,
                                  char *smem) {
    if (ph == mcq::kFbPlan) {
        Batch B{A.cols, nullptr, A.ncols};
        fb_plan_slot(B, A.hmaps, A.dmaps, A.npass, i, reinterpret_cast<uint32_t *>(smem));
        return;
    }
    const bool emit = ph == mcq::kFbEmit;
    const uint32_t p = emit ? 0u : (ph - mcq::kFbPass0) / 3, kind = emit ? 0u : (ph - mcq::kFbPass0) % 3;
    const int ds = emit ? 2 * kMaxPasses : (kind == 1 ? kMaxPasses + (int)p : (int)p);
    Batch B{A.cols, A.dmaps + (size_t)ds * (A.ncols + 1), A.ncols};
    const uint32_t total = map_total(B);
    for (uint32_t b = i; b < total; b += A.fb_items) {
        if (b != i) __syncthreads();
        const uint32_t j = find_col(B, b);
        const mc::ColDesc &C = A.cols[j];
        const uint32_t t = b - B.map[j];
        if (emit) {
            if (C.drankd) {
                MC_DISPATCH(C, mc::emit_distinct_tile, C, t, true);
            } else {
                MC_DISPATCH(C, mc::emit_tile, C, smem, true);
            }
            continue;
        }
        mc::PassIO io;
        if (!pass_io(C, kPassFull, (int)p, &io)) continue;
        if (kind == 0) {
            MC_DISPATCH(C, mc::sort_up_tile, C, io, t, smem);
        } else if (kind == 1) {
            if (C.sort_tiles <= mc::kSmallScanTiles) {
                MC_DISPATCH(C, mc::sort_scan_small, C, io, t);
            } else {
                MC_DISPATCH(C, mc::sort_scan_digit, C, io, t, smem);
            }
        } else {
            MC_DISPATCH(C, mc::sort_down_tile, C, io, t, smem);
        }
    }
}

__global__ __launch_bounds__(256) void kn_prologue(Batch B, uint32_t *z, uint64_t nz) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nz; i += stride)
        z[i] = 0u;
    for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < B.ncols; j += stride) {
        mc_result *r = B.cols[j].result;
        r->new_dict_len = 0;
        r->new_codes_words = 0;
        r->delta_dict_len = 0;
        r->new_bitwidth = 0;
        r->error = 0;
    }
}

// At most 168 VGPRs (three waves per SIMD): the hot steps fit; the widest
// (the multi-type sort and fallback paths) spill a little.  Its LDS (the
// largest tile, 52 KB) also leaves room for three workgroups per CU.
template <int CODES>
__global__ __launch_bounds__(256, 3) void kn_persist(PersistArgs A) {
    extern __shared__ __attribute__((aligned(16))) char smem[];
    __shared__ PersistSmem S;
    for (uint32_t x = threadIdx.x; x <= mcq::kNumPhases; x += blockDim.x) S.base[x] = A.base[x];
    __syncthreads();
    uint32_t *const ticket = A.q + kQTicket;
    uint32_t *const colq = A.q + kQColDone;
    while (true) {
        if (threadIdx.x == 0) S.ticket = atomicAdd(ticket, 1u);
        __syncthreads();
        const uint32_t k = S.ticket;
        if (k >= A.total) break;
        queue_decode(A, S, k);
        __syncthreads();
        const uint32_t ph = S.ph, j = S.col, idx = S.idx;
        if (mcq::is_global(ph)) {
            const bool ab = ph == mcq::kFbPlan
                                ? queue_wait(A.q + kQEmitDone, A.emit_total, A.q + kQErr,
                                             A.q + kQErr, &S.abort)
                                : queue_wait(A.q + kQFbDone, A.gcum[ph], A.q + kQErr, A.q + kQErr,
                                             &S.abort);
            if (!ab) run_fallback_item(A, S, ph, idx, smem);
        } else {
            const mc::ColDesc &C = A.cols[j];
            bool ab = queue_wait(colq + j, A.cum[(size_t)j * mcq::kNumPhases + ph], C.err,
                                 A.q + kQErr, &S.abort);
            if (!ab && mcq::after_fallback(ph)) {
                // a column the prefix sort left unsorted waits for the fallback
                // chain (the flag is final once the column's Step 1(a) items
                // are done; thread 0 reads it so that the whole workgroup
                // takes the same branch)
                if (threadIdx.x == 0) S.idx = C.sflags[mc::kSfUnsorted];
                __syncthreads();
                if (S.idx)
                    ab = queue_wait(A.q + kQFbDone, A.fb_total, A.q + kQErr, A.q + kQErr, &S.abort);
            }
            // an aborted launch skips its items: none runs on inputs that were
            // not finished
            if (!ab) run_column_item<CODES>(A, ph, j, idx, smem);
        }
        // the item's writes, then its count (release at device scope)
        __threadfence();
        __syncthreads();
        if (threadIdx.x == 0) {
            if (mcq::is_global(ph)) {
                atomicAdd(A.q + kQFbDone, 1u);
            } else {
                atomicAdd(colq + j, 1u);
                if (ph == mcq::kEmit) atomicAdd(A.q + kQEmitDone, 1u);
            }
        }
    }
}

// Dynamic LDS of kn_persist: the largest tile function it runs.
template <int CODES>
constexpr size_t persist_lds() {
    constexpr size_t a = max3(kSmemHist, kSmemHistScan, kSmemDown);
    constexpr size_t b = max3(sizeof(mc::EmitSmem<mc::TS16>), kSmemHash, sizeof(mc::CompactSmem));
    constexpr size_t c = max3(sizeof(mc::MergeSmem<mc::TU32>), sizeof(mc::MergeSmem<mc::TU64>),
                              sizeof(mc::MergeSmem<mc::TS16>));
    constexpr size_t d = max3(sizeof(mc::XCompactSmem), sizeof(mc::RepackOutSmem<CODES>), kSmemSmall);
    return max3(max3(a, b, c), d, (size_t)64);
}

template <int CODES>
int launch_persist(const BatchPlan &P, uint32_t ncols, char *ws, uint32_t cus, hipStream_t s) {
    PersistArgs A;
    A.cols = reinterpret_cast<const mc::ColDesc *>(ws + P.desc_off);
    A.ncols = ncols;
    A.total = P.q.total();
    A.base = reinterpret_cast<const uint32_t *>(ws + P.qbase_off);
    A.pmap = reinterpret_cast<const uint32_t *>(ws + P.qpmap_off);
    A.cum = reinterpret_cast<const uint32_t *>(ws + P.qcum_off);
    A.gcum = reinterpret_cast<const uint32_t *>(ws + P.qgcum_off);
    A.emit_total = P.q.emit_total;
    A.fb_total = P.q.fb_total;
    A.q = reinterpret_cast<uint32_t *>(ws + P.q_off);
    A.hmaps = reinterpret_cast<const uint32_t *>(ws + P.map_off);
    A.dmaps = reinterpret_cast<uint32_t *>(ws + P.dmap_off);
    A.npass = P.max_passes;
    A.fb_items = kPersistFbItems;
    A.merge_per = P.merge_per;
    A.repack_per = P.repack_per;
    constexpr size_t lds = persist_lds<CODES>();
    uint32_t workers = P.workers;
    if (!workers) {  // as many as the GPU holds at once
        int per_cu = 0;
        MC_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kn_persist<CODES>, mc::kBlock,
                                                            lds));
        workers = (uint32_t)std::max(1, per_cu) * std::max(1u, cus);
    }
    workers = std::max(1u, std::min(workers, A.total));
    if (A.total == 0) return MC_OK;
    hipLaunchKernelGGL(kn_persist<CODES>, dim3(workers), dim3(mc::kBlock), lds, s, A);
    MC_LAUNCHED("kn_persist");
    return MC_OK;
}

// The persistent form of the batched merge: the prologue (zeroed part with
// the queue counters, result scalars), then one persistent launch.
int enqueue_persist(const BatchPlan &P, uint32_t ncols, char *ws, uint32_t cus, hipStream_t s) {
    Batch B;
    B.cols = reinterpret_cast<const mc::ColDesc *>(ws + P.desc_off);
    B.map = nullptr;
    B.ncols = ncols;
    const uint64_t nz = P.z_total / 4;
    const uint32_t grid = (uint32_t)std::min<uint64_t>(
        std::max<uint64_t>(ceil_div(std::max<uint64_t>(nz, ncols), 256 * 4), 1), 2048);
    hipLaunchKernelGGL(kn_prologue, dim3(grid), dim3(256), 0, s, B, reinterpret_cast<uint32_t *>(ws),
                       nz);
    MC_LAUNCHED("kn_prologue");
    switch (P.repack_codes) {
        case 1024: return launch_persist<1024>(P, ncols, ws, cus, s);
        case 4096: return launch_persist<4096>(P, ncols, ws, cus, s);
        default: return launch_persist<2048>(P, ncols, ws, cus, s);
    }
}

}  // namespace

// ===========================================================================
// extern "C" entry points
// ===========================================================================

extern "C" {

const char *mc_last_error(void) { return g_err.c_str(); }

int mc_ctx_create(int device, mc_ctx **out) {
    if (!out) return fail(MC_E_ARG, "null out pointer");
    int n = 0;
    MC_HIP(hipGetDeviceCount(&n));
    if (device < 0 || device >= n) return fail(MC_E_ARG, "no such device");
    mc_ctx *c = new (std::nothrow) mc_ctx();
    if (!c) return fail(MC_E_NOMEM, "context allocation failed");
    c->device = device;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess ||
        cus <= 0) {
        delete c;
        return fail(MC_E_HIP, "cannot read the device's compute unit count");
    }
    c->cus = (uint32_t)cus;
    // the allocation-free workspace of this device: its device address,
    // looked up once per device with that device current
    if (device >= kMaxDevices) {
        delete c;
        return fail(MC_E_ARG, "device index above the library's limit of 64");
    }
    {
        std::lock_guard<std::mutex> lock(g_noalloc_mu);
        if (!g_noalloc_ptr[device]) {
            int prev = 0;
            hipError_t e = hipGetDevice(&prev);
            if (e == hipSuccess && prev != device) e = hipSetDevice(device);
            void *ptr = nullptr;
            if (e == hipSuccess) e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(noalloc_scratch));
            if (prev != device) (void)hipSetDevice(prev);
            if (e != hipSuccess || !ptr) {
                delete c;
                return e != hipSuccess ? hip_fail(e, "hipGetSymbolAddress(noalloc_scratch)")
                                       : fail(MC_E_HIP, "no device address for noalloc_scratch");
            }
            g_noalloc_ptr[device] = ptr;
        }
        c->noalloc_scratch = g_noalloc_ptr[device];
    }
    *out = c;
    return MC_OK;
}

void mc_ctx_destroy(mc_ctx *ctx) {
    if (!ctx) return;
    if (ctx->meta_event) {
        (void)hipEventSynchronize(ctx->meta_event);
        (void)hipEventDestroy(ctx->meta_event);
    }
    if (ctx->meta_host) (void)hipHostFree(ctx->meta_host);
    for (auto &set : ctx->ev)
        for (auto &e : set)
            if (e) (void)hipEventDestroy(e);
    delete ctx;
}

int mc_merge_bounds_ctx(const mc_ctx *ctx, const mc_column_in *in, uint64_t *dict_cap,
                        uint64_t *codes_words, uint64_t *scratch_bytes) {
    int rc = check_in(in);
    if (rc) return rc;
    const uint64_t dc = in->main_dict_len + in->delta_rows;
    const uint64_t rows = in->main_rows + in->delta_rows;
    if (dict_cap) *dict_cap = dc;
    if (codes_words) *codes_words = codes_words_bound(rows, dc);
    if (scratch_bytes)
        *scratch_bytes = single_scratch(col_layout(in->type, in->main_dict_len, in->delta_rows,
                                                   in->main_rows, true,
                                                   ctx ? ctx->tune : kDefaultTuning));
    return MC_OK;
}

int mc_merge_bounds(const mc_column_in *in, uint64_t *dict_cap, uint64_t *codes_words,
                    uint64_t *scratch_bytes) {
    return mc_merge_bounds_ctx(nullptr, in, dict_cap, codes_words, scratch_bytes);
}

int mc_merge_column(mc_ctx *ctx, const mc_column_in *in, const mc_column_out *out, void *scratch,
                    uint64_t scratch_bytes, hipStream_t stream) {
    return merge_column_impl(ctx, in, out, scratch, scratch_bytes, stream);
}

int mc_merge_column_noalloc(mc_ctx *ctx, const mc_column_in *in, const mc_column_out *out,
                            hipStream_t stream) {
    if (!ctx) return fail(MC_E_ARG, "null context");
    int rc = check_in(in);
    if (rc) return rc;
    rc = check_out(in, out);
    if (rc) return rc;
    if (!ctx->noalloc_scratch) return fail(MC_E_ARG, "context has no allocation-free workspace");
    const ColLayout L =
        col_layout(in->type, in->main_dict_len, in->delta_rows, in->main_rows, true, ctx->tune);
    if (single_scratch(L) > MC_NOALLOC_SCRATCH_BYTES)
        return fail(MC_E_CAP, "column needs " + std::to_string(single_scratch(L)) +
                                  " bytes of workspace, above MC_NOALLOC_SCRATCH_BYTES (" +
                                  std::to_string(MC_NOALLOC_SCRATCH_BYTES) + ")");
    // the device address looked up in mc_ctx_create, never the array's name
    char *ws = static_cast<char *>(ctx->noalloc_scratch);
    switch (in->type) {
        case MC_U32: return merge_column_t<mc::TU32>(ctx, in, out, ws, L, stream, false, nullptr, false);
        case MC_U64: return merge_column_t<mc::TU64>(ctx, in, out, ws, L, stream, false, nullptr, false);
        default: return merge_column_t<mc::TS16>(ctx, in, out, ws, L, stream, false, nullptr, false);
    }
}

int mc_merge_column_naive(mc_ctx *ctx, const mc_column_in *in, const mc_column_out *out,
                          void *scratch, uint64_t scratch_bytes, hipStream_t stream) {
    return merge_column_impl(ctx, in, out, scratch, scratch_bytes, stream, true);
}

int mc_delta_dictionary_scratch(int32_t type, uint64_t delta_rows, uint64_t *scratch_bytes) {
    if (value_len(type) == 0) return fail(MC_E_ARG, "unknown value type");
    if (delta_rows >= (1ull << 30)) return fail(MC_E_ARG, "delta_rows must be < 2^30");
    // enough for either route of Step 1(a), whatever a context's tuning picks
    mc_tuning always_hash = kDefaultTuning;
    always_hash.hash_min_rows = 1;
    const uint64_t a = single_scratch(col_layout(type, 0, delta_rows, 0, false));
    const uint64_t b = single_scratch(col_layout(type, 0, delta_rows, 0, true, always_hash));
    if (scratch_bytes) *scratch_bytes = std::max(a, b);
    return MC_OK;
}

int mc_delta_dictionary(mc_ctx *ctx, int32_t type, const void *delta_values, uint64_t delta_rows,
                        void *u_d, uint32_t *drank, uint64_t *d_count, void *scratch,
                        uint64_t scratch_bytes, hipStream_t s) {
    if (!ctx) return fail(MC_E_ARG, "null context");
    if (value_len(type) == 0) return fail(MC_E_ARG, "unknown value type");
    if (delta_rows >= (1ull << 30)) return fail(MC_E_ARG, "delta_rows must be < 2^30");
    if (!d_count) return fail(MC_E_ARG, "null d_count");
    if (delta_rows > 0 && (!delta_values || !u_d || !drank)) return fail(MC_E_ARG, "null buffer");
    if (!aligned16(delta_values) || !aligned16(u_d) || !aligned4(drank) ||
        (reinterpret_cast<uintptr_t>(d_count) & 7u))
        return fail(MC_E_ARG, "misaligned buffer");
    const ColLayout L = col_layout(type, 0, delta_rows, 0, true, ctx->tune);
    if (!scratch || scratch_bytes < single_scratch(L)) return fail(MC_E_CAP, "scratch too small");
    if (!aligned16(scratch)) return fail(MC_E_ARG, "scratch must be 16-byte aligned");
    char *za = static_cast<char *>(scratch), *zb = za + L.z_size;
    mc::ColDesc C;
    memset(&C, 0, sizeof(C));
    C.type = type;
    C.delta = delta_values;
    C.nd = (uint32_t)delta_rows;
    C.sort_tiles = L.sort_tiles;
    C.err = reinterpret_cast<uint32_t *>(za + L.err);
    C.keys0 = zb + L.keys0;
    C.keys1 = zb + L.keys1;
    C.vals0 = reinterpret_cast<uint32_t *>(zb + L.vals0);
    C.vals1 = reinterpret_cast<uint32_t *>(zb + L.vals1);
    C.gh = reinterpret_cast<uint32_t *>(za + L.gh);
    C.base = reinterpret_cast<uint32_t *>(zb + L.base);
    C.trivial = reinterpret_cast<uint32_t *>(za + L.trivial);
    C.tcount = reinterpret_cast<uint32_t *>(zb + L.tcount);
    C.pgsum = L.two_launch_pass ? reinterpret_cast<uint32_t *>(za + L.pgsum) : nullptr;
    C.egsum = reinterpret_cast<uint32_t *>(za + L.egsum);
    C.ecnt = reinterpret_cast<uint32_t *>(zb + L.ecnt);
    C.counters = reinterpret_cast<uint32_t *>(za + L.counters);
    C.sflags = reinterpret_cast<uint32_t *>(za + L.sflags);
    C.emit_status = reinterpret_cast<uint64_t *>(za + L.emit_status);
    C.emit_status2 = reinterpret_cast<uint64_t *>(za + L.emit_status2);
    C.n_ud = d_count;
    C.nd_max = delta_rows;
    C.prefix_run = L.prefix_run;
    C.u_d = u_d;
    C.drank = drank;
    set_hash_fields(C, za, zb, L);
    int rc = launch_fill(za, L.z_size, d_count, 8, s);
    if (rc) return rc;
    switch (type) {
        case MC_U32: return launch_delta_dictionary<mc::TU32>(C, L, ctx->cus, s, nullptr);
        case MC_U64: return launch_delta_dictionary<mc::TU64>(C, L, ctx->cus, s, nullptr);
        default: return launch_delta_dictionary<mc::TS16>(C, L, ctx->cus, s, nullptr);
    }
}

int mc_merge_dictionaries_scratch(uint64_t n_um, uint64_t n_ud_max, uint64_t *scratch_bytes) {
    // the largest over the value types (their merge tiles differ)
    uint64_t z = 0;
    for (int32_t t : {MC_U32, MC_U64, MC_STR16})
        z = std::max<uint64_t>(z, merge_only_layout(t, n_um, n_ud_max).z_size);
    if (scratch_bytes) *scratch_bytes = z;
    return MC_OK;
}

int mc_merge_dictionaries(mc_ctx *ctx, int32_t type, const void *u_m, uint64_t n_um,
                          const void *u_d, const uint64_t *d_n_ud, uint64_t n_ud_max, void *u_new,
                          uint32_t *x_m, uint32_t *x_d, uint64_t rows_total, mc_result *result,
                          void *scratch, uint64_t scratch_bytes, hipStream_t s) {
    if (!ctx) return fail(MC_E_ARG, "null context");
    if (value_len(type) == 0) return fail(MC_E_ARG, "unknown value type");
    if (!d_n_ud || !result) return fail(MC_E_ARG, "null scalar pointer");
    if (n_um + n_ud_max > (1ull << 32)) return fail(MC_E_ARG, "|U_M| + |U_D| must be <= 2^32");
    if ((n_um > 0 && (!u_m || !x_m)) || (n_ud_max > 0 && (!u_d || !x_d)) ||
        (n_um + n_ud_max > 0 && !u_new))
        return fail(MC_E_ARG, "null buffer");
    if (!aligned16(u_m) || !aligned16(u_d) || !aligned16(u_new) || !aligned16(result))
        return fail(MC_E_ARG, "misaligned buffer");
    const ColLayout L = merge_only_layout(type, n_um, n_ud_max);
    if (!scratch || scratch_bytes < L.z_size) return fail(MC_E_CAP, "scratch too small");
    if (!aligned16(scratch)) return fail(MC_E_ARG, "scratch must be 16-byte aligned");
    char *za = static_cast<char *>(scratch);
    mc::ColDesc C;
    memset(&C, 0, sizeof(C));
    C.type = type;
    C.u_m = u_m;
    C.n_um = n_um;
    C.u_d = const_cast<void *>(u_d);
    C.n_ud_in = d_n_ud;
    C.nd_max = n_ud_max;
    C.u_new = u_new;
    C.u_new_cap = n_um + n_ud_max;
    C.x_m = x_m;
    C.x_d = x_d;
    C.result = result;
    C.err = &result->error;
    C.rows_total = rows_total;
    C.counters = reinterpret_cast<uint32_t *>(za + L.counters);
    C.merge_status = reinterpret_cast<uint64_t *>(za + L.merge_status);
    C.mbound = L.partitioned ? reinterpret_cast<uint64_t *>(za + L.mbound) : nullptr;
    int rc = launch_fill(za, L.z_size, result, sizeof(mc_result), s);
    if (rc) return rc;
    switch (type) {
        case MC_U32: return launch_merge<mc::TU32>(C, L.merge_tiles, s);
        case MC_U64: return launch_merge<mc::TU64>(C, L.merge_tiles, s);
        default: return launch_merge<mc::TS16>(C, L.merge_tiles, s);
    }
}

int mc_reencode(mc_ctx *ctx, const uint64_t *main_codes, uint64_t n_main, uint32_t w,
                const uint32_t *x_m, uint64_t n_um, const uint32_t *drank, uint64_t n_delta,
                const uint32_t *x_d, mc_result *result, uint64_t *out, uint64_t out_cap_words,
                hipStream_t s) {
    if (!ctx) return fail(MC_E_ARG, "null context");
    if (w < 1 || w > 32) return fail(MC_E_ARG, "w must be 1..32");
    if (!result) return fail(MC_E_ARG, "null result");
    if ((n_main > 0 && (!main_codes || !x_m)) || (n_delta > 0 && (!drank || !x_d)))
        return fail(MC_E_ARG, "null buffer");
    if (n_main + n_delta > 0 && !out) return fail(MC_E_ARG, "null output");
    if (!aligned16(main_codes) || !aligned16(out) || !aligned16(result))
        return fail(MC_E_ARG, "misaligned buffer");
    if (n_delta >= (1ull << 30)) return fail(MC_E_ARG, "n_delta must be < 2^30");
    if (n_um + n_delta > (1ull << 32)) return fail(MC_E_ARG, "dictionary too large");
    if (n_main > 0 && n_um > (1ull << w)) return fail(MC_E_ARG, "n_um larger than 2^w");
    if (out_cap_words < codes_words_bound(n_main + n_delta, n_um + n_delta))
        return fail(MC_E_CAP, "output capacity below the bound");
    mc::ColDesc C;
    memset(&C, 0, sizeof(C));
    C.w = w;
    C.main_codes = main_codes;
    C.n_main = n_main;
    C.x_m = const_cast<uint32_t *>(x_m);
    C.n_um = n_um;
    C.drank = const_cast<uint32_t *>(drank);
    C.nd = (uint32_t)n_delta;
    C.x_d = const_cast<uint32_t *>(x_d);
    C.result = result;
    C.err = &result->error;
    C.out = out;
    C.out_cap = out_cap_words;
    return launch_repack(C, ctx->tune.repack_codes, s);
}

int mc_ctx_set_timing(mc_ctx *ctx, int enable) {
    if (!ctx) return fail(MC_E_ARG, "null context");
    ctx->timing = enable ? 1 : 0;
    ctx->used = 0;
    return MC_OK;
}

int mc_ctx_step_times(mc_ctx *ctx, float *ms, uint32_t n) {
    if (!ctx || (!ms && n)) return fail(MC_E_ARG, "null argument");
    if (n > MC_STEP_TIMES) return fail(MC_E_ARG, "at most MC_STEP_TIMES step times");
    if (ctx->used == 0) return fail(MC_E_ARG, "no timed merge recorded");
    MC_HIP(hipEventSynchronize(ctx->ev[ctx->used - 1][5]));
    double acc[MC_STEP_TIMES] = {0, 0, 0, 0, 0, 0};
    // event k: 0 start, 1 after the delta sort, 2 after the emit, 3 after the
    // dictionary merge, 4 before the re-encode kernel, 5 end
    const int from[MC_STEP_TIMES] = {0, 1, 2, 3, 0, 4}, to[MC_STEP_TIMES] = {1, 2, 3, 5, 5, 5};
    for (size_t i = 0; i < ctx->used; i++) {
        const auto &e = ctx->ev[i];
        for (uint32_t k = 0; k < n; k++) {
            float x = 0.f;
            MC_HIP(hipEventElapsedTime(&x, e[from[k]], e[to[k]]));
            acc[k] += x;
        }
    }
    for (uint32_t k = 0; k < n; k++) ms[k] = (float)(acc[k] / (double)ctx->used);
    return MC_OK;
}

int mc_copy_bytes(mc_ctx *ctx, const void *src, void *dst, uint64_t bytes, hipStream_t s) {
    if (!ctx) return fail(MC_E_ARG, "null context");
    if ((bytes & 15u) || !aligned16(src) || !aligned16(dst))
        return fail(MC_E_ARG, "copy needs 16-byte aligned buffers and a multiple of 16 bytes");
    if (bytes && (!src || !dst)) return fail(MC_E_ARG, "null buffer");
    if (bytes == 0) return MC_OK;
    // one thread per 16 bytes, within a launch's 2^32 work-items
    const uint64_t grid = std::min<uint64_t>(ceil_div(bytes / 16, 256), (1ull << 24) - 1);
    hipLaunchKernelGGL(k_copy16, dim3((uint32_t)grid), dim3(256), 0, s,
                       static_cast<const v4u32 *>(src), static_cast<v4u32 *>(dst), bytes / 16);
    MC_LAUNCHED("k_copy16");
    return MC_OK;
}

int mc_gather_ref(mc_ctx *ctx, const uint32_t *idx, uint64_t n, const void *table,
                  uint32_t entry_bytes, uint32_t n_table, uint32_t *out, hipStream_t s) {
    if (!ctx) return fail(MC_E_ARG, "null context");
    if (entry_bytes != 2 && entry_bytes != 4) return fail(MC_E_ARG, "entry_bytes must be 2 or 4");
    if (n == 0) return MC_OK;
    if (!idx || !table || !out || n_table == 0) return fail(MC_E_ARG, "null buffer or empty table");
    const uint64_t grid = ceil_div(n, 256 * 8);
    if (grid >= (1ull << 31)) return fail(MC_E_ARG, "too many indices");
    if (entry_bytes == 4)
        hipLaunchKernelGGL(k_gather_ref<uint32_t>, dim3((uint32_t)grid), dim3(256), 0, s, idx, n,
                           static_cast<const uint32_t *>(table), n_table, out);
    else
        hipLaunchKernelGGL(k_gather_ref<uint16_t>, dim3((uint32_t)grid), dim3(256), 0, s, idx, n,
                           static_cast<const uint16_t *>(table), n_table, out);
    MC_LAUNCHED("k_gather_ref");
    return MC_OK;
}

// ---- batched ---------------------------------------------------------------

int mc_delta_index_bytes(int32_t type, uint64_t capacity, uint64_t *bytes) {
    if (value_len(type) == 0) return fail(MC_E_ARG, "unknown value type");
    if (capacity >= (1ull << 30)) return fail(MC_E_ARG, "capacity must be < 2^30");
    if (bytes) *bytes = index_layout(type, capacity).size;
    return MC_OK;
}

int mc_delta_index_reset(mc_ctx *ctx, const mc_delta_index *ix, hipStream_t s) {
    if (!ctx) return fail(MC_E_ARG, "null context");
    int rc = check_index(ix);
    if (rc) return rc;
    const IndexLayout X = index_layout(ix->type, ix->capacity);
    // counters, scalars and the table; the rest is written before it is read
    return launch_fill(ix->workspace, X.rep, nullptr, 0, s);
}

int mc_delta_index_append(mc_ctx *ctx, const mc_delta_index *ix, const void *delta_values,
                          uint64_t row0, uint64_t rows, hipStream_t s) {
    if (!ctx) return fail(MC_E_ARG, "null context");
    int rc = check_index(ix);
    if (rc) return rc;
    if (row0 > ix->capacity || rows > ix->capacity - row0)
        return fail(MC_E_CAP, "rows past the index capacity");
    if (rows == 0) return MC_OK;
    if (!delta_values || !aligned16(delta_values)) return fail(MC_E_ARG, "bad delta buffer");
    const IndexLayout X = index_layout(ix->type, ix->capacity);
    char *w = static_cast<char *>(ix->workspace);
    mc::ColDesc C;
    memset(&C, 0, sizeof(C));
    C.type = ix->type;
    C.delta = delta_values;
    C.nd = (uint32_t)(row0 + rows);
    C.nd_max = ix->capacity;
    C.hrow0 = row0;
    set_index_fields(C, ix);
    C.err = reinterpret_cast<uint32_t *>(w + X.scal + 80);
    const uint64_t ntiles = ceil_div(rows, mc::kCompactTile);
    const dim3 gh((uint32_t)ceil_div(rows, mc::kHashTile)), gc((uint32_t)ntiles), b(mc::kBlock);
    switch (ix->type) {
        case MC_U32:
            hipLaunchKernelGGL(k1_hash_insert<mc::TU32>, gh, b, 0, s, C);
            hipLaunchKernelGGL(k1_compact<mc::TU32>, gc, b, 0, s, C);
            break;
        case MC_U64:
            hipLaunchKernelGGL(k1_hash_insert<mc::TU64>, gh, b, 0, s, C);
            hipLaunchKernelGGL(k1_compact<mc::TU64>, gc, b, 0, s, C);
            break;
        default:
            hipLaunchKernelGGL(k1_hash_insert<mc::TS16>, gh, b, 0, s, C);
            hipLaunchKernelGGL(k1_compact<mc::TS16>, gc, b, 0, s, C);
            break;
    }
    MC_LAUNCHED("k1_hash_insert / k1_compact (index)");
    return MC_OK;
}

int mc_merge_indexed_bounds(const mc_column_in *in, uint64_t *scratch_bytes) {
    int rc = check_in(in);
    if (rc) return rc;
    if (scratch_bytes)
        *scratch_bytes = single_scratch(col_layout(in->type, in->main_dict_len, in->delta_rows,
                                                   in->main_rows, true, kDefaultTuning, true));
    return MC_OK;
}

int mc_merge_column_indexed(mc_ctx *ctx, const mc_column_in *in, const mc_delta_index *ix,
                            const mc_column_out *out, void *scratch, uint64_t scratch_bytes,
                            hipStream_t s) {
    if (!ctx) return fail(MC_E_ARG, "null context");
    int rc = check_in(in);
    if (rc) return rc;
    rc = check_out(in, out);
    if (rc) return rc;
    rc = check_index(ix);
    if (rc) return rc;
    if (ix->type != in->type) return fail(MC_E_ARG, "index and column value types differ");
    if (in->delta_rows > ix->capacity) return fail(MC_E_ARG, "delta_rows past the index capacity");
    const ColLayout L = col_layout(in->type, in->main_dict_len, in->delta_rows, in->main_rows,
                                   true, ctx->tune, true);
    if (!scratch || scratch_bytes < single_scratch(L))
        return fail(MC_E_CAP, "scratch below mc_merge_indexed_bounds");
    if (!aligned16(scratch)) return fail(MC_E_ARG, "scratch must be 16-byte aligned");
    if (ctx->validate) {
        rc = validate_dicts(in, out, 1, s);
        if (rc) return rc;
    }
    char *ws = static_cast<char *>(scratch);
    switch (in->type) {
        case MC_U32: rc = merge_column_t<mc::TU32>(ctx, in, out, ws, L, s, false, ix); break;
        case MC_U64: rc = merge_column_t<mc::TU64>(ctx, in, out, ws, L, s, false, ix); break;
        default: rc = merge_column_t<mc::TS16>(ctx, in, out, ws, L, s, false, ix); break;
    }
    if (rc == MC_OK && ctx->validate) rc = read_errors(out, 1, s, "merge");
    return rc;
}

int mc_merge_batched_bounds_ctx(const mc_ctx *ctx, const mc_column_in *ins, uint32_t ncols,
                                uint64_t *scratch_bytes) {
    if (!ins && ncols) return fail(MC_E_ARG, "null descriptors");
    BatchPlan P;
    int rc = plan_batch(ins, ncols, P, ctx ? ctx->tune : kDefaultTuning);
    if (rc) return rc;
    if (scratch_bytes) *scratch_bytes = P.total;
    return MC_OK;
}

int mc_merge_batched_bounds(const mc_column_in *ins, uint32_t ncols, uint64_t *scratch_bytes) {
    return mc_merge_batched_bounds_ctx(nullptr, ins, ncols, scratch_bytes);
}

int mc_merge_columns_batched(mc_ctx *ctx, const mc_column_in *ins, const mc_column_out *outs,
                             uint32_t ncols, void *scratch, uint64_t scratch_bytes,
                             hipStream_t stream, mc_graph **graph) {
    if (!ctx) return fail(MC_E_ARG, "null context");
    if (!ctx->validate)
        return batched_run(ctx, ins, outs, ncols, scratch, scratch_bytes, stream, ctx->tune,
                           graph);
    if (ncols && (!ins || !outs)) return fail(MC_E_ARG, "null descriptors");
    for (uint32_t j = 0; j < ncols; j++) {  // the checks batched_run makes, before any launch
        int rc = check_in(&ins[j]);
        if (rc == MC_OK) rc = check_out(&ins[j], &outs[j]);
        if (rc) return rc;
    }
    int rc = validate_dicts(ins, outs, ncols, stream);
    if (rc) return rc;
    rc = batched_run(ctx, ins, outs, ncols, scratch, scratch_bytes, stream, ctx->tune, graph);
    if (rc) return rc;
    return read_errors(outs, ncols, stream, "batched merge");
}

int mc_ctx_set_validate(mc_ctx *ctx, int enable) {
    if (!ctx) return fail(MC_E_ARG, "null context");
    ctx->validate = enable ? 1 : 0;
    return MC_OK;
}

int mc_ctx_set_tuning(mc_ctx *ctx, const mc_tuning *t) {
    if (!ctx || !t) return fail(MC_E_ARG, "null argument");
    if (t->repack_codes != 1024 && t->repack_codes != 2048 && t->repack_codes != 4096)
        return fail(MC_E_ARG, "repack_codes must be 1024, 2048 or 4096");
    if (t->prefix_run < 4 || t->prefix_run > 1024)
        return fail(MC_E_ARG, "prefix_run must be in [4, 1024]");
    if (t->batched_launch != MC_BATCHED_PHASES && t->batched_launch != MC_BATCHED_PERSISTENT)
        return fail(MC_E_ARG, "batched_launch must be MC_BATCHED_PHASES or MC_BATCHED_PERSISTENT");
    if (t->batched_launch == MC_BATCHED_PERSISTENT)
        return fail(MC_E_ARG,
                    "MC_BATCHED_PERSISTENT is disabled: its launch stalled on the GPU (also with "
                    "one workgroup) and the cause is not found; use MC_BATCHED_PHASES");
    if (t->persist_repack > 1024 || t->persist_merge > 1024)
        return fail(MC_E_ARG, "persist_repack and persist_merge must be at most 1024");
    ctx->tune = *t;
    return MC_OK;
}

int mc_ctx_get_tuning(const mc_ctx *ctx, mc_tuning *t) {
    if (!ctx || !t) return fail(MC_E_ARG, "null argument");
    *t = ctx->tune;
    return MC_OK;
}

int mc_autotune_batched(mc_ctx *ctx, const mc_column_in *ins, const mc_column_out *outs,
                        uint32_t ncols, void *scratch, uint64_t scratch_bytes, hipStream_t stream,
                        mc_tuning *chosen, float *times_ms) {
    if (!ctx || !chosen) return fail(MC_E_ARG, "null argument");
    hipEvent_t e0 = nullptr, e1 = nullptr;
    MC_HIP(hipEventCreate(&e0));
    hipError_t he = hipEventCreate(&e1);
    if (he != hipSuccess) {
        (void)hipEventDestroy(e0);
        return hip_fail(he, "hipEventCreate");
    }
    // one warm-up run, then the best of two timed runs
    auto time_one = [&](const mc_tuning &t, float *ms) -> int {
        int rc = batched_run(ctx, ins, outs, ncols, scratch, scratch_bytes, stream, t, nullptr,
                             false);
        if (rc) return rc;
        float best = 0.0f;
        for (int r = 0; r < 2; r++) {
            MC_HIP(hipEventRecord(e0, stream));
            rc = batched_run(ctx, ins, outs, ncols, scratch, scratch_bytes, stream, t, nullptr,
                             false);
            if (rc) return rc;
            MC_HIP(hipEventRecord(e1, stream));
            MC_HIP(hipEventSynchronize(e1));
            float x = 0.0f;
            MC_HIP(hipEventElapsedTime(&x, e0, e1));
            best = r == 0 ? x : std::min(best, x);
        }
        *ms = best;
        return MC_OK;
    };
    int rc = MC_OK;
    float times[6] = {0};
    mc_tuning best = kDefaultTuning;
    float best_ms = 0.0f;
    const uint32_t codes[3] = {1024u, 2048u, 4096u}, runs[3] = {16u, 32u, 64u};
    for (int i = 0; i < 3 && rc == MC_OK; i++) {
        mc_tuning t = kDefaultTuning;
        t.repack_codes = codes[i];
        rc = time_one(t, &times[i]);
        if (rc == MC_OK && (i == 0 || times[i] < best_ms)) {
            best = t;
            best_ms = times[i];
        }
    }
    const mc_tuning by_codes = best;
    for (int i = 0; i < 3 && rc == MC_OK; i++) {
        mc_tuning t = by_codes;
        t.prefix_run = runs[i];
        rc = time_one(t, &times[3 + i]);
        if (rc == MC_OK && times[3 + i] < best_ms) {
            best = t;
            best_ms = times[3 + i];
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    ctx->tune = best;
    *chosen = best;
    if (times_ms) memcpy(times_ms, times, sizeof(times));
    return MC_OK;
}

int mc_tune_class(const mc_column_in *in, uint32_t *cls) {
    if (!in || !cls) return fail(MC_E_ARG, "null argument");
    int rc = check_in(in);
    if (rc) return rc;
    *cls = tune_class_of(*in);
    return MC_OK;
}

int mc_ctx_set_class_tuning(mc_ctx *ctx, uint32_t cls, const mc_tuning *t) {
    if (!ctx) return fail(MC_E_ARG, "null context");
    if (cls >= MC_TUNE_CLASSES) return fail(MC_E_ARG, "class out of range");
    if (!t) {
        ctx->class_set[cls] = 0;
        return MC_OK;
    }
    if (t->repack_codes != 1024 && t->repack_codes != 2048 && t->repack_codes != 4096)
        return fail(MC_E_ARG, "repack_codes must be 1024, 2048 or 4096");
    if (t->prefix_run < 4 || t->prefix_run > 1024)
        return fail(MC_E_ARG, "prefix_run must be in [4, 1024]");
    ctx->class_tune[cls] = ctx->tune;
    ctx->class_tune[cls].repack_codes = t->repack_codes;
    ctx->class_tune[cls].prefix_run = t->prefix_run;
    ctx->class_set[cls] = 1;
    return MC_OK;
}

int mc_ctx_get_class_tuning(const mc_ctx *ctx, uint32_t cls, mc_tuning *t, int *is_set) {
    if (!ctx || !t) return fail(MC_E_ARG, "null argument");
    if (cls >= MC_TUNE_CLASSES) return fail(MC_E_ARG, "class out of range");
    *t = ctx->tune;
    if (ctx->class_set[cls]) {
        t->repack_codes = ctx->class_tune[cls].repack_codes;
        t->prefix_run = ctx->class_tune[cls].prefix_run;
    }
    if (is_set) *is_set = ctx->class_set[cls];
    return MC_OK;
}

int mc_autotune_batched_classes(mc_ctx *ctx, const mc_column_in *ins, const mc_column_out *outs,
                                uint32_t ncols, void *scratch, uint64_t scratch_bytes,
                                hipStream_t stream, uint32_t *classes) {
    if (!ctx) return fail(MC_E_ARG, "null context");
    if (ncols && (!ins || !outs)) return fail(MC_E_ARG, "null descriptors");
    std::vector<std::vector<uint32_t>> members(MC_TUNE_CLASSES);
    for (uint32_t j = 0; j < ncols; j++) {
        int rc = check_in(&ins[j]);
        if (rc) return rc;
        members[tune_class_of(ins[j])].push_back(j);
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    MC_HIP(hipEventCreate(&e0));
    hipError_t he = hipEventCreate(&e1);
    if (he != hipSuccess) {
        (void)hipEventDestroy(e0);
        return hip_fail(he, "hipEventCreate");
    }
    std::vector<mc_column_in> sub_in;
    std::vector<mc_column_out> sub_out;
    // one warm-up run, then the best of three timed runs of the class's columns
    auto time_one = [&](const mc_tuning &t, float *ms) -> int {
        const uint32_t n = (uint32_t)sub_in.size();
        int rc = batched_run(ctx, sub_in.data(), sub_out.data(), n, scratch, scratch_bytes, stream,
                             t, nullptr, false);
        if (rc) return rc;
        float best = 0.0f;
        for (int r = 0; r < 3; r++) {
            MC_HIP(hipEventRecord(e0, stream));
            rc = batched_run(ctx, sub_in.data(), sub_out.data(), n, scratch, scratch_bytes, stream,
                             t, nullptr, false);
            if (rc) return rc;
            MC_HIP(hipEventRecord(e1, stream));
            MC_HIP(hipEventSynchronize(e1));
            float x = 0.0f;
            MC_HIP(hipEventElapsedTime(&x, e0, e1));
            best = r == 0 ? x : std::min(best, x);
        }
        *ms = best;
        return MC_OK;
    };
    int rc = MC_OK;
    uint32_t tuned = 0;
    const uint32_t codes[3] = {1024u, 2048u, 4096u}, runs[3] = {16u, 32u, 64u};
    for (uint32_t c = 0; c < MC_TUNE_CLASSES && rc == MC_OK; c++) {
        if (members[c].empty()) continue;
        sub_in.clear();
        sub_out.clear();
        for (uint32_t j : members[c]) {
            sub_in.push_back(ins[j]);
            sub_out.push_back(outs[j]);
        }
        mc_tuning best = ctx->tune;
        float best_ms = 0.0f, x = 0.0f;
        for (int i = 0; i < 3 && rc == MC_OK; i++) {
            mc_tuning t = ctx->tune;
            t.repack_codes = codes[i];
            rc = time_one(t, &x);
            if (rc == MC_OK && (i == 0 || x < best_ms)) {
                best = t;
                best_ms = x;
            }
        }
        const mc_tuning by_codes = best;
        for (int i = 0; i < 3 && rc == MC_OK; i++) {
            mc_tuning t = by_codes;
            t.prefix_run = runs[i];
            if (t.prefix_run == by_codes.prefix_run) continue;  // timed above
            rc = time_one(t, &x);
            if (rc == MC_OK && x < best_ms) {
                best = t;
                best_ms = x;
            }
        }
        if (rc == MC_OK) {
            ctx->class_tune[c] = best;
            ctx->class_set[c] = 1;
            tuned++;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    if (classes) *classes = tuned;
    return MC_OK;
}

}  // extern "C"

namespace {

int batched_run(mc_ctx *ctx, const mc_column_in *ins, const mc_column_out *outs, uint32_t ncols,
                void *scratch, uint64_t scratch_bytes, hipStream_t stream, const mc_tuning &tune,
                mc_graph **graph, bool use_classes) {
    if (ncols == 0) return MC_OK;
    if (!ins || !outs) return fail(MC_E_ARG, "null descriptors");
    BatchPlan P;
    int rc = plan_batch(ins, ncols, P, tune, use_classes ? ctx : nullptr);
    if (rc) return rc;
    for (uint32_t i = 0; i < ncols; i++) {
        rc = check_out(&ins[i], &outs[i]);
        if (rc) return rc;
    }
    if (!scratch || scratch_bytes < P.total) return fail(MC_E_CAP, "scratch below the batched bound");
    if (!aligned16(scratch)) return fail(MC_E_ARG, "scratch must be 16-byte aligned");
    char *ws = static_cast<char *>(scratch);

    // descriptors + maps, staged in the context's pinned buffer and copied on
    // the stream (the previous batch's copy must have left the buffer)
    const uint64_t meta = P.dmap_off - P.desc_off;  // the device-built maps stay out
    if (ctx->meta_event) MC_HIP(hipEventSynchronize(ctx->meta_event));
    if (ctx->meta_cap < meta) {
        if (ctx->meta_host) (void)hipHostFree(ctx->meta_host);
        ctx->meta_host = nullptr;
        ctx->meta_cap = 0;
        MC_HIP(hipHostMalloc(&ctx->meta_host, meta, hipHostMallocDefault));
        ctx->meta_cap = meta;
    }
    if (!ctx->meta_event) MC_HIP(hipEventCreateWithFlags(&ctx->meta_event, hipEventDisableTiming));
    char *h = static_cast<char *>(ctx->meta_host);
    memset(h, 0, meta);
    mc::ColDesc *hd = reinterpret_cast<mc::ColDesc *>(h);
    for (uint32_t i = 0; i < ncols; i++)
        hd[i] = make_desc(&ins[i], &outs[i], ws + P.z_off[i], ws + P.z_total + P.b_off[i], P.L[i]);
    memcpy(h + (P.map_off - P.desc_off), P.maps.data(), P.maps.size() * 4);
    if (P.persistent) {
        memcpy(h + (P.qbase_off - P.desc_off), P.q.base.data(), P.q.base.size() * 4);
        memcpy(h + (P.qgcum_off - P.desc_off), P.q.gcum.data(), P.q.gcum.size() * 4);
        memcpy(h + (P.qpmap_off - P.desc_off), P.q.pmap.data(), P.q.pmap.size() * 4);
        memcpy(h + (P.qcum_off - P.desc_off), P.q.cum.data(), P.q.cum.size() * 4);
    }
    MC_HIP(hipMemcpyAsync(ws + P.desc_off, h, meta, hipMemcpyHostToDevice, stream));
    MC_HIP(hipEventRecord(ctx->meta_event, stream));

    auto enqueue = [&](hipStream_t st) {
        return P.persistent ? enqueue_persist(P, ncols, ws, ctx->cus, st)
                            : enqueue_batch(P, ncols, ws, ctx->cus, st);
    };
    if (!graph) return enqueue(stream);

    mc_graph *g = new (std::nothrow) mc_graph();
    if (!g) return fail(MC_E_NOMEM, "graph allocation failed");
    hipStream_t cs = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e != hipSuccess) {
        delete g;
        return hip_fail(e, "hipStreamCreateWithFlags");
    }
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        rc = enqueue(cs);
        hipGraph_t gr = nullptr;
        hipError_t e2 = hipStreamEndCapture(cs, &gr);
        if (rc == MC_OK && e2 != hipSuccess) rc = hip_fail(e2, "hipStreamEndCapture");
        g->graph = gr;
    } else {
        rc = hip_fail(e, "hipStreamBeginCapture");
    }
    (void)hipStreamDestroy(cs);
    if (rc == MC_OK) {
        e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
        if (e != hipSuccess) rc = hip_fail(e, "hipGraphInstantiate");
    }
    if (rc == MC_OK) {
        e = hipGraphLaunch(g->exec, stream);
        if (e != hipSuccess) rc = hip_fail(e, "hipGraphLaunch");
    }
    if (rc != MC_OK) {
        mc_graph_destroy(g);
        return rc;
    }
    *graph = g;
    return MC_OK;
}

}  // namespace

extern "C" {

int mc_graph_launch(mc_graph *graph, hipStream_t stream) {
    if (!graph || !graph->exec) return fail(MC_E_ARG, "null graph");
    MC_HIP(hipGraphLaunch(graph->exec, stream));
    return MC_OK;
}

void mc_graph_destroy(mc_graph *graph) {
    if (!graph) return;
    if (graph->exec) (void)hipGraphExecDestroy(graph->exec);
    if (graph->graph) (void)hipGraphDestroy(graph->graph);
    delete graph;
}

}  // extern "C"
