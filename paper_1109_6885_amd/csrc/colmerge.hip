// colmerge.hip -- host side of the column-merge library: argument checks,
// workspace layout, kernel launches and the extern "C" entry points that
// include/colmerge.h declares.  Kernels live in sort.hpp (Step 1(a)),
// merge.hpp (Steps 1(b), 2(a)) and repack.hpp (Step 2(b)).
#include <hip/hip_runtime.h>

#include <stdint.h>
#include <string.h>

#include <array>
#include <new>
#include <string>
#include <vector>

#include "colmerge.h"
#include "common.hpp"
#include "merge.hpp"
#include "repack.hpp"
#include "sort.hpp"

struct mc_ctx {
    int device = 0;
    int timing = 0;
    // one set of five events per timed merge since timing was enabled
    std::vector<std::array<hipEvent_t, 5>> ev;
    size_t used = 0;
    hipEvent_t *cur = nullptr;  // events of the merge being enqueued
};

struct mc_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

thread_local std::string g_err;

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
// Workspace layout.  The first region is cleared by one fill kernel at the
// start of every call (tile counters, histograms, prefix words, the sort's
// "same digit" flags); the rest is written before it is read.
// ---------------------------------------------------------------------------

struct Layout {
    uint64_t total = 0;
    uint64_t zero_bytes = 0;  // zeroed region starts at offset 0
    // zeroed
    uint64_t counters = 0;    // u32[16]: [0] emit tiles, [1] merge tiles, [2] error word
    uint64_t n_ud = 0;        // u64
    uint64_t gh = 0;          // u32[passes*256]
    uint64_t trivial = 0;     // u32[16]
    uint64_t emit_status = 0; // u64[emit tiles]
    uint64_t merge_status = 0;// u64[merge tiles]
    // written before read
    uint64_t base = 0;        // u32[passes*256]
    uint64_t tcount = 0;      // u32[256*sort tiles]
    uint64_t keys0 = 0, keys1 = 0, vals0 = 0, vals1 = 0;
    uint64_t u_d = 0, drank = 0, x_d = 0, x_m = 0;
    uint32_t sort_tiles = 0, emit_tiles = 0;
    uint64_t merge_tiles = 0;
};

struct Carver {
    uint64_t off = 0;
    uint64_t take(uint64_t bytes) {
        off = align_up(off, 256);
        uint64_t at = off;
        off += bytes;
        return at;
    }
};

Layout make_layout(int32_t type, uint64_t n_um, uint64_t nd, bool need_dict_scratch) {
    Layout L;
    const uint32_t E = value_len(type);
    const uint32_t P = E;  // one 8-bit digit per value byte
    L.sort_tiles = (uint32_t)ceil_div(nd, sort_tile_of(type));
    L.emit_tiles = (uint32_t)ceil_div(nd, mc::kEmitTile);
    L.merge_tiles = ceil_div(n_um + nd, mc::kMergeTile);
    Carver c;
    L.counters = c.take(16 * 4);
    L.n_ud = c.take(8);
    L.gh = c.take((uint64_t)P * 256 * 4);
    L.trivial = c.take(16 * 4);
    L.emit_status = c.take((uint64_t)L.emit_tiles * 8);
    L.merge_status = c.take(L.merge_tiles * 8);
    L.zero_bytes = align_up(c.off, 256);
    c.off = L.zero_bytes;
    L.base = c.take((uint64_t)P * 256 * 4);
    L.tcount = c.take((uint64_t)256 * L.sort_tiles * 4);
    L.keys0 = c.take(nd * E);
    L.keys1 = c.take(nd * E);
    L.vals0 = c.take(nd * 4);
    L.vals1 = c.take(nd * 4);
    if (need_dict_scratch) L.u_d = c.take(nd * E);
    L.drank = c.take(nd * 4);
    L.x_d = c.take(nd * 4);
    L.x_m = c.take(n_um * 4);
    L.total = align_up(c.off, 256);
    return L;
}

// ---------------------------------------------------------------------------
// Kernels that do not depend on the value type.
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_fill_zero(uint32_t *p0, uint64_t n0, uint32_t *p1,
                                                   uint64_t n1) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n0; i += stride)
        p0[i] = 0u;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n1; i += stride)
        p1[i] = 0u;
}

// Plain 128-bit copy: the achievable streaming bandwidth on this GPU, and
// the kernel of known traffic that calibrates hardware byte counters.
__global__ __launch_bounds__(256) void k_copy16(const uint4 *__restrict__ src,
                                                uint4 *__restrict__ dst, uint64_t n16) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride)
        dst[i] = src[i];
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
// Step launchers
// ---------------------------------------------------------------------------

// Step 1(a): sort the delta and emit U_D / drank.  Scratch regions come from
// the layout; the zeroed region must already be clear.
template <class T>
int launch_delta_dictionary(const void *delta, uint64_t nd, void *u_d, uint32_t *drank,
                            uint64_t *n_ud, char *ws, const Layout &L, uint32_t *err,
                            hipStream_t s, mc_ctx *ctx) {
    if (nd == 0) return MC_OK;
    mc::SortJob J;
    J.src = delta;
    J.keys[0] = ws + L.keys0;
    J.keys[1] = ws + L.keys1;
    J.vals[0] = reinterpret_cast<uint32_t *>(ws + L.vals0);
    J.vals[1] = reinterpret_cast<uint32_t *>(ws + L.vals1);
    J.n = (uint32_t)nd;
    J.ntiles = L.sort_tiles;
    J.gh = reinterpret_cast<uint32_t *>(ws + L.gh);
    J.base = reinterpret_cast<uint32_t *>(ws + L.base);
    J.trivial = reinterpret_cast<uint32_t *>(ws + L.trivial);
    J.tcount = reinterpret_cast<uint32_t *>(ws + L.tcount);
    J.err = err;
    constexpr int P = T::kBytes;
    uint32_t hgrid = (uint32_t)ceil_div(nd, 256 * 16);
    if (hgrid > 1024) hgrid = 1024;
    hipLaunchKernelGGL(mc::k_hist_all<T>, dim3(hgrid), dim3(mc::kBlock), 0, s, J);
    MC_LAUNCHED("k_hist_all");
    hipLaunchKernelGGL(mc::k_hist_scan<T>, dim3(1), dim3(mc::kBlock), 0, s, J);
    MC_LAUNCHED("k_hist_scan");
    for (int p = 0; p < P; p++) {
        hipLaunchKernelGGL(mc::k_sort_up<T>, dim3(J.ntiles), dim3(mc::kBlock), 0, s, J, p);
        MC_LAUNCHED("k_sort_up");
        hipLaunchKernelGGL(mc::k_sort_scan<T>, dim3(256), dim3(mc::kBlock), 0, s, J, p);
        MC_LAUNCHED("k_sort_scan");
        hipLaunchKernelGGL(mc::k_sort_down<T>, dim3(J.ntiles), dim3(mc::kBlock), 0, s, J, p);
        MC_LAUNCHED("k_sort_down");
    }
    if (ctx && ctx->cur) MC_HIP(hipEventRecord(ctx->cur[1], s));
    mc::EmitJob E;
    E.keys = J.keys[(P - 1) & 1];
    E.rows = J.vals[(P - 1) & 1];
    E.n = (uint32_t)nd;
    E.u_d = u_d;
    E.drank = drank;
    E.n_ud = n_ud;
    E.status = reinterpret_cast<uint64_t *>(ws + L.emit_status);
    E.counter = reinterpret_cast<uint32_t *>(ws + L.counters) + 0;
    E.err = err;
    hipLaunchKernelGGL(mc::k_emit<T>, dim3(L.emit_tiles), dim3(mc::kBlock), 0, s, E);
    MC_LAUNCHED("k_emit");
    return MC_OK;
}

template <class T>
int launch_merge(const void *u_m, uint64_t n_um, const void *u_d, const uint64_t *d_n_ud,
                 uint64_t nd_max, void *u_new, uint32_t *x_m, uint32_t *x_d,
                 uint64_t rows_total, mc_result *result, char *ws, const Layout &L,
                 hipStream_t s) {
    mc::MergeJob M;
    M.u_m = u_m;
    M.n_um = n_um;
    M.u_d = u_d;
    M.d_n_ud = d_n_ud;
    M.n_ud_max = nd_max;
    M.u_new = u_new;
    M.x_m = x_m;
    M.x_d = x_d;
    M.rows_total = rows_total;
    M.result = result;
    M.status = reinterpret_cast<uint64_t *>(ws + L.merge_status);
    M.counter = reinterpret_cast<uint32_t *>(ws + L.counters) + 1;
    M.err = &result->error;
    uint64_t grid = ceil_div(n_um + nd_max, mc::kMergeTile);
    if (grid == 0) grid = 1;
    hipLaunchKernelGGL(mc::k_merge<T>, dim3((uint32_t)grid), dim3(mc::kBlock), 0, s, M);
    MC_LAUNCHED("k_merge");
    return MC_OK;
}

int launch_repack(const uint64_t *main_codes, uint64_t n_main, uint32_t w, const uint32_t *x_m,
                  uint64_t n_um, const uint32_t *drank, uint64_t nd, const uint32_t *x_d,
                  mc_result *result, uint64_t *out, uint64_t cap, hipStream_t s) {
    mc::RepackJob R;
    R.main_codes = main_codes;
    R.n_main = n_main;
    R.w = w;
    R.x_m = x_m;
    R.n_um = n_um;
    R.drank = drank;
    R.n_delta = nd;
    R.x_d = x_d;
    R.result = result;
    R.out = out;
    R.out_cap_words = cap;
    R.err = &result->error;
    uint64_t grid = ceil_div(n_main + nd, mc::kRepackCodes);
    if (grid == 0) return MC_OK;
    hipLaunchKernelGGL(mc::k_repack, dim3((uint32_t)grid), dim3(mc::kBlock), 0, s, R);
    MC_LAUNCHED("k_repack");
    return MC_OK;
}

// ---------------------------------------------------------------------------
// Argument checks
// ---------------------------------------------------------------------------

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
    if (in->main_dict_len > 0 && !in->main_dict) return fail(MC_E_ARG, "null main_dict");
    if (in->main_rows > 0 && !in->main_codes) return fail(MC_E_ARG, "null main_codes");
    if (in->delta_rows > 0 && !in->delta_values) return fail(MC_E_ARG, "null delta_values");
    if (!aligned16(in->main_dict) || !aligned16(in->main_codes) || !aligned16(in->delta_values))
        return fail(MC_E_ARG, "input buffers must be 16-byte aligned");
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

template <class T>
int merge_column_t(mc_ctx *ctx, const mc_column_in *in, const mc_column_out *out, char *ws,
                   const Layout &L, hipStream_t s) {
    uint32_t *err = &out->result->error;
    const uint64_t nd = in->delta_rows;
    uint32_t *x_m = out->x_main ? out->x_main : reinterpret_cast<uint32_t *>(ws + L.x_m);
    uint32_t *x_d = out->x_delta ? out->x_delta : reinterpret_cast<uint32_t *>(ws + L.x_d);
    uint32_t *drank = reinterpret_cast<uint32_t *>(ws + L.drank);
    uint64_t *n_ud = reinterpret_cast<uint64_t *>(ws + L.n_ud);
    void *u_d = ws + L.u_d;
    ctx->cur = nullptr;
    if (ctx->timing) {
        if (ctx->used == ctx->ev.size()) {
            std::array<hipEvent_t, 5> set{};
            for (auto &e : set) MC_HIP(hipEventCreate(&e));
            ctx->ev.push_back(set);
        }
        ctx->cur = ctx->ev[ctx->used].data();
        MC_HIP(hipEventRecord(ctx->cur[0], s));
    }
    int rc = launch_fill(ws, L.zero_bytes, out->result, sizeof(mc_result), s);
    if (rc) return rc;
    rc = launch_delta_dictionary<T>(in->delta_values, nd, u_d, drank, n_ud, ws, L, err, s, ctx);
    if (rc) return rc;
    if (ctx->cur) {
        if (nd == 0) MC_HIP(hipEventRecord(ctx->cur[1], s));
        MC_HIP(hipEventRecord(ctx->cur[2], s));
    }
    rc = launch_merge<T>(in->main_dict, in->main_dict_len, u_d, n_ud, nd, out->new_dict, x_m, x_d,
                         in->main_rows + nd, out->result, ws, L, s);
    if (rc) return rc;
    if (ctx->cur) MC_HIP(hipEventRecord(ctx->cur[3], s));
    rc = launch_repack(in->main_codes, in->main_rows, in->bitwidth, x_m, in->main_dict_len, drank,
                       nd, x_d, out->result, out->new_codes, out->new_codes_cap_words, s);
    if (rc) return rc;
    if (ctx->cur) {
        MC_HIP(hipEventRecord(ctx->cur[4], s));
        ctx->used++;
        ctx->cur = nullptr;
    }
    return MC_OK;
}

int merge_column_impl(mc_ctx *ctx, const mc_column_in *in, const mc_column_out *out,
                      void *scratch, uint64_t scratch_bytes, hipStream_t s) {
    if (!ctx) return fail(MC_E_ARG, "null context");
    int rc = check_in(in);
    if (rc) return rc;
    rc = check_out(in, out);
    if (rc) return rc;
    const Layout L = make_layout(in->type, in->main_dict_len, in->delta_rows, true);
    if (!scratch || scratch_bytes < L.total) return fail(MC_E_CAP, "scratch below mc_merge_bounds");
    if (!aligned16(scratch)) return fail(MC_E_ARG, "scratch must be 16-byte aligned");
    char *ws = static_cast<char *>(scratch);
    switch (in->type) {
        case MC_U32: return merge_column_t<mc::TU32>(ctx, in, out, ws, L, s);
        case MC_U64: return merge_column_t<mc::TU64>(ctx, in, out, ws, L, s);
        default: return merge_column_t<mc::TS16>(ctx, in, out, ws, L, s);
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
    *out = c;
    return MC_OK;
}

void mc_ctx_destroy(mc_ctx *ctx) {
    if (!ctx) return;
    for (auto &set : ctx->ev)
        for (auto &e : set)
            if (e) (void)hipEventDestroy(e);
    delete ctx;
}

int mc_merge_bounds(const mc_column_in *in, uint64_t *dict_cap, uint64_t *codes_words,
                    uint64_t *scratch_bytes) {
    int rc = check_in(in);
    if (rc) return rc;
    const uint64_t dc = in->main_dict_len + in->delta_rows;
    const uint64_t rows = in->main_rows + in->delta_rows;
    if (dict_cap) *dict_cap = dc;
    if (codes_words) *codes_words = codes_words_bound(rows, dc);
    if (scratch_bytes)
        *scratch_bytes = make_layout(in->type, in->main_dict_len, in->delta_rows, true).total;
    return MC_OK;
}

int mc_merge_column(mc_ctx *ctx, const mc_column_in *in, const mc_column_out *out, void *scratch,
                    uint64_t scratch_bytes, hipStream_t stream) {
    return merge_column_impl(ctx, in, out, scratch, scratch_bytes, stream);
}

int mc_delta_dictionary_scratch(int32_t type, uint64_t delta_rows, uint64_t *scratch_bytes) {
    if (value_len(type) == 0) return fail(MC_E_ARG, "unknown value type");
    if (delta_rows >= (1ull << 30)) return fail(MC_E_ARG, "delta_rows must be < 2^30");
    if (scratch_bytes) *scratch_bytes = make_layout(type, 0, delta_rows, false).total;
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
    const Layout L = make_layout(type, 0, delta_rows, false);
    if (!scratch || scratch_bytes < L.total) return fail(MC_E_CAP, "scratch too small");
    if (!aligned16(scratch)) return fail(MC_E_ARG, "scratch must be 16-byte aligned");
    char *ws = static_cast<char *>(scratch);
    int rc = launch_fill(ws, L.zero_bytes, d_count, 8, s);
    if (rc) return rc;
    uint32_t *err = reinterpret_cast<uint32_t *>(ws + L.counters) + 2;
    switch (type) {
        case MC_U32:
            return launch_delta_dictionary<mc::TU32>(delta_values, delta_rows, u_d, drank, d_count,
                                                     ws, L, err, s, nullptr);
        case MC_U64:
            return launch_delta_dictionary<mc::TU64>(delta_values, delta_rows, u_d, drank, d_count,
                                                     ws, L, err, s, nullptr);
        default:
            return launch_delta_dictionary<mc::TS16>(delta_values, delta_rows, u_d, drank, d_count,
                                                     ws, L, err, s, nullptr);
    }
}

int mc_merge_dictionaries_scratch(uint64_t n_um, uint64_t n_ud_max, uint64_t *scratch_bytes) {
    // only the counters and the merge prefix words are used
    Carver c;
    c.take(16 * 4);
    c.take(ceil_div(n_um + n_ud_max, mc::kMergeTile) * 8);
    if (scratch_bytes) *scratch_bytes = align_up(c.off, 256);
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
    uint64_t need = 0;
    mc_merge_dictionaries_scratch(n_um, n_ud_max, &need);
    if (!scratch || scratch_bytes < need) return fail(MC_E_CAP, "scratch too small");
    // the merge needs only the counters and its prefix words
    Layout L;
    Carver c;
    L.counters = c.take(16 * 4);
    L.merge_status = c.take(ceil_div(n_um + n_ud_max, mc::kMergeTile) * 8);
    L.zero_bytes = align_up(c.off, 256);
    char *ws = static_cast<char *>(scratch);
    int rc = launch_fill(ws, L.zero_bytes, result, sizeof(mc_result), s);
    if (rc) return rc;
    switch (type) {
        case MC_U32:
            return launch_merge<mc::TU32>(u_m, n_um, u_d, d_n_ud, n_ud_max, u_new, x_m, x_d,
                                          rows_total, result, ws, L, s);
        case MC_U64:
            return launch_merge<mc::TU64>(u_m, n_um, u_d, d_n_ud, n_ud_max, u_new, x_m, x_d,
                                          rows_total, result, ws, L, s);
        default:
            return launch_merge<mc::TS16>(u_m, n_um, u_d, d_n_ud, n_ud_max, u_new, x_m, x_d,
                                          rows_total, result, ws, L, s);
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
    if (!aligned16(main_codes) || !aligned16(out)) return fail(MC_E_ARG, "misaligned buffer");
    if (n_um + n_delta > (1ull << 32)) return fail(MC_E_ARG, "dictionary too large");
    if (out_cap_words < codes_words_bound(n_main + n_delta, n_um + n_delta))
        return fail(MC_E_CAP, "output capacity below the bound");
    return launch_repack(main_codes, n_main, w, x_m, n_um, drank, n_delta, x_d, result, out,
                         out_cap_words, s);
}

int mc_ctx_set_timing(mc_ctx *ctx, int enable) {
    if (!ctx) return fail(MC_E_ARG, "null context");
    ctx->timing = enable ? 1 : 0;
    ctx->used = 0;
    return MC_OK;
}

int mc_ctx_step_times(mc_ctx *ctx, float *ms5) {
    if (!ctx || !ms5) return fail(MC_E_ARG, "null argument");
    if (ctx->used == 0) return fail(MC_E_ARG, "no timed merge recorded");
    MC_HIP(hipEventSynchronize(ctx->ev[ctx->used - 1][4]));
    double acc[5] = {0, 0, 0, 0, 0};
    for (size_t i = 0; i < ctx->used; i++) {
        const auto &e = ctx->ev[i];
        const int from[5] = {0, 1, 2, 3, 0}, to[5] = {1, 2, 3, 4, 4};
        for (int k = 0; k < 5; k++) {
            float ms = 0.f;
            MC_HIP(hipEventElapsedTime(&ms, e[from[k]], e[to[k]]));
            acc[k] += ms;
        }
    }
    for (int k = 0; k < 5; k++) ms5[k] = (float)(acc[k] / (double)ctx->used);
    return MC_OK;
}

int mc_copy_bytes(mc_ctx *ctx, const void *src, void *dst, uint64_t bytes, hipStream_t s) {
    if (!ctx) return fail(MC_E_ARG, "null context");
    if ((bytes & 15u) || !aligned16(src) || !aligned16(dst))
        return fail(MC_E_ARG, "copy needs 16-byte aligned buffers and a multiple of 16 bytes");
    if (bytes && (!src || !dst)) return fail(MC_E_ARG, "null buffer");
    if (bytes == 0) return MC_OK;
    int dev = 0, cus = 256;
    MC_HIP(hipGetDevice(&dev));
    MC_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    uint64_t grid = ceil_div(bytes / 16, 256);
    if (grid > (uint64_t)cus * 16) grid = (uint64_t)cus * 16;
    hipLaunchKernelGGL(k_copy16, dim3((uint32_t)grid), dim3(256), 0, s,
                       static_cast<const uint4 *>(src), static_cast<uint4 *>(dst), bytes / 16);
    MC_LAUNCHED("k_copy16");
    return MC_OK;
}

// ---- batched ---------------------------------------------------------------

int mc_merge_batched_bounds(const mc_column_in *ins, uint32_t ncols, uint64_t *scratch_bytes) {
    if (!ins && ncols) return fail(MC_E_ARG, "null descriptors");
    uint64_t total = 0;
    for (uint32_t i = 0; i < ncols; i++) {
        uint64_t sb = 0;
        int rc = mc_merge_bounds(&ins[i], nullptr, nullptr, &sb);
        if (rc) return rc;
        total += align_up(sb, 256);
    }
    if (scratch_bytes) *scratch_bytes = total;
    return MC_OK;
}

static int enqueue_batched(mc_ctx *ctx, const mc_column_in *ins, const mc_column_out *outs,
                           uint32_t ncols, char *ws, hipStream_t s) {
    uint64_t off = 0;
    const int timing = ctx->timing;  // per-column events are not recorded here
    ctx->timing = 0;
    for (uint32_t i = 0; i < ncols; i++) {
        uint64_t sb = 0;
        int rc = mc_merge_bounds(&ins[i], nullptr, nullptr, &sb);
        if (rc == MC_OK) rc = merge_column_impl(ctx, &ins[i], &outs[i], ws + off, sb, s);
        if (rc) {
            ctx->timing = timing;
            return rc;
        }
        off += align_up(sb, 256);
    }
    ctx->timing = timing;
    return MC_OK;
}

int mc_merge_columns_batched(mc_ctx *ctx, const mc_column_in *ins, const mc_column_out *outs,
                             uint32_t ncols, void *scratch, uint64_t scratch_bytes,
                             hipStream_t stream, mc_graph **graph) {
    if (!ctx) return fail(MC_E_ARG, "null context");
    if (ncols && (!ins || !outs)) return fail(MC_E_ARG, "null descriptors");
    uint64_t need = 0;
    int rc = mc_merge_batched_bounds(ins, ncols, &need);
    if (rc) return rc;
    for (uint32_t i = 0; i < ncols; i++) {
        rc = check_out(&ins[i], &outs[i]);
        if (rc) return rc;
    }
    if (!scratch || scratch_bytes < need) return fail(MC_E_CAP, "scratch below the batched bound");
    if (!aligned16(scratch)) return fail(MC_E_ARG, "scratch must be 16-byte aligned");
    char *ws = static_cast<char *>(scratch);
    if (!graph) return enqueue_batched(ctx, ins, outs, ncols, ws, stream);

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
        rc = enqueue_batched(ctx, ins, outs, ncols, ws, cs);
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
