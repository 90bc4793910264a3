// Host side of libswmi: argument checks, workspace planning, launches, C ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>

#include "swmi.h"
#include "swmi_internal.h"
#include "swmi_host.h"

using namespace swmi;

// ------------------------------------------------------------------------ errors

static thread_local std::string g_err;

sw_status swmi::fail(sw_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

#define HIP_TRY(expr)                                                                       \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess) return fail(SW_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

extern "C" const char* sw_last_error(void) { return g_err.c_str(); }
extern "C" const char* sw_version(void) { return "swmi 0.1 (gfx950)"; }

// ------------------------------------------------------------------------ context

extern "C" sw_status sw_context_create(int device, void* hip_stream, sw_context** out) {
    if (!out) return fail(SW_EINVAL, "sw_context_create: out is NULL");
    *out = nullptr;
    int n = 0;
    HIP_TRY(hipGetDeviceCount(&n));
    if (device < 0 || device >= n) return fail(SW_EINVAL, "sw_context_create: device %d of %d", device, n);
    HIP_TRY(hipSetDevice(device));
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, device));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(SW_EUNSUPPORTED, "sw_context_create: device is %s, kernels are built for gfx950", prop.gcnArchName);
    sw_context* c = new (std::nothrow) sw_context();
    if (!c) return fail(SW_ENOMEM, "sw_context_create: out of host memory");
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    c->num_cu = prop.multiProcessorCount;
    hipError_t e = hipHostMalloc((void**)&c->host_misc, 4096, hipHostMallocDefault);
    if (e != hipSuccess) {
        delete c;
        return fail(SW_ENOMEM, "sw_context_create: hipHostMalloc: %s", hipGetErrorString(e));
    }
    *out = c;
    return SW_OK;
}

extern "C" sw_status sw_context_destroy(sw_context* ctx) {
    if (!ctx) return SW_OK;
    (void)hipSetDevice(ctx->device);
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    else (void)hipDeviceSynchronize();
    for (auto& b : ctx->bufs) (void)hipFree(b.ptr);
    if (ctx->host_misc) (void)hipHostFree(ctx->host_misc);
    delete ctx;
    return SW_OK;
}

sw_status swmi::ctx_buffer(sw_context* ctx, int slot, size_t bytes, void** out) {
    DevBuf& b = ctx->bufs[slot];
    if (b.bytes < bytes) {
        if (b.ptr) {
            (void)hipStreamSynchronize(ctx->stream);
            (void)hipFree(b.ptr);
            b.ptr = nullptr;
            b.bytes = 0;
        }
        const size_t want = std::max(bytes, (size_t)1 << 20);
        hipError_t e = hipMalloc(&b.ptr, want);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(SW_ENOMEM, "device allocation of %zu bytes failed: %s", want, hipGetErrorString(e));
        }
        b.bytes = want;
    }
    *out = b.ptr;
    return SW_OK;
}

// ------------------------------------------------------------------------ checks

sw_status swmi::check_scoring(const sw_scoring* s) {
    if (!s) return fail(SW_EINVAL, "scoring is NULL");
    if (s->match <= 0 || s->match > 127) return fail(SW_EINVAL, "match must be in 1..127 (got %d)", s->match);
    if (s->mismatch < 0 || s->mismatch > 127)
        return fail(SW_EINVAL, "mismatch must be in 0..127 (got %d)", s->mismatch);
    if (s->gap_extend <= 0 || s->gap_open < s->gap_extend || s->gap_open > (1 << 20))
        return fail(SW_EINVAL, "need 0 < gap_extend <= gap_open <= 2^20 (got %d, %d)", s->gap_open, s->gap_extend);
    return SW_OK;
}

sw_status swmi::check_lengths(int64_t la, int64_t lb, const sw_scoring* s) {
    if (la < 0 || lb < 0) return fail(SW_EINVAL, "negative length (%lld, %lld)", (long long)la, (long long)lb);
    const int64_t lim = ((int64_t)1 << 31) - 4096;
    if (la > lim || lb > lim) return fail(SW_EUNSUPPORTED, "sequence longer than %lld", (long long)lim);
    if ((int64_t)s->match * std::min(la, lb) >= ((int64_t)1 << 30))
        return fail(SW_EUNSUPPORTED, "match * min(len) reaches 2^30 (int32 headroom)");
    return SW_OK;
}

sw_status swmi::check_options(const sw_options* o) {
    if (!o) return SW_OK;
    if (o->prune_mode < SW_PRUNE_NONE || o->prune_mode > SW_PRUNE_LEARNED)
        return fail(SW_EINVAL, "unknown prune_mode %d", o->prune_mode);
    if (o->rows_per_lane != 0 && o->rows_per_lane != 4 && o->rows_per_lane != 8)
        return fail(SW_EINVAL, "rows_per_lane must be 0, 4 or 8 (got %d)", o->rows_per_lane);
    if (o->waves_per_cu < 0 || o->waves_per_cu > 16)
        return fail(SW_EINVAL, "waves_per_cu must be 0..16 (got %d)", o->waves_per_cu);
    if (o->threshold < 0) return fail(SW_EINVAL, "threshold must be >= 0");
    if (o->band_width < 0 || o->band_width % kTick)
        return fail(SW_EINVAL, "band_width must be 0 or a positive multiple of 64 (got %d)", o->band_width);
    return SW_OK;
}

// ------------------------------------------------------------------------ plan

static size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

ScorePlan swmi::plan_score(const sw_context* ctx, int64_t M, int64_t N, const sw_options* o) {
    ScorePlan p{};
    p.R = (o && o->rows_per_lane) ? o->rows_per_lane : 8;
    const int wpc = (o && o->waves_per_cu) ? o->waves_per_cu : 8;
    p.M = M;
    p.N = N;
    p.Q = (M + kWave * p.R - 1) / (kWave * p.R);
    // Band width: keep the stripe slots within a fixed budget.
    const int64_t max_grid = (int64_t)ctx->num_cu * wpc;
    const size_t slot_budget = (size_t)8 << 30;
    int64_t grid_est = std::max<int64_t>(1, std::min<int64_t>(max_grid, p.Q * ((N + 63) / 64)));
    int64_t nslot = grid_est + 1;
    int64_t W = (int64_t)(slot_budget / ((size_t)nslot * sizeof(int2))) - (kSlotPad + 2 * kTick);
    W = std::max<int64_t>(kTick, W / kTick * kTick);
    if (o && o->band_width) W = o->band_width;
    const int64_t N64 = (N + kTick - 1) / kTick * kTick;
    p.W = std::min(W, std::max<int64_t>(kTick, N64));
    p.n_bands = (N + p.W - 1) / p.W;
    const int64_t n_tasks = p.Q * p.n_bands;
    p.grid = (int)std::min<int64_t>(max_grid, n_tasks);
    p.nslot = std::max<int64_t>(2, (int64_t)p.grid + 1);
    p.slot_stride = (int64_t)align_up((size_t)(kSlotPad + p.W + 2 * kTick), 64);

    size_t off = 0;
    p.off_a = off;
    off = align_up(off + (size_t)M + 64, 256);
    p.off_b = off;
    off = align_up(off + (size_t)(kBPad + N + kBPadTail), 256);
    p.off_slots = off;
    off = align_up(off + (size_t)p.nslot * p.slot_stride * sizeof(int2), 256);
    p.off_lbuf = off;
    off = align_up(off + (p.n_bands > 1 ? (size_t)M * sizeof(int2) : 0), 256);
    p.off_recs = off;
    off = align_up(off + (size_t)n_tasks * sizeof(TaskRec), 256);
    p.off_zero = off;  // progress + misc: cleared on every call
    p.off_prog = off;
    off = align_up(off + (size_t)n_tasks * sizeof(int32_t), 256);
    p.off_misc = off;
    off = align_up(off + 256, 256);
    p.zero_bytes = off - p.off_zero;
    p.total = off;
    return p;
}

// misc block layout (bytes)
enum { MISC_TICKET = 0, MISC_GBEST = 4, MISC_PRUNED = 8, MISC_BAD_A = 16, MISC_BAD_B = 24, MISC_OUT = 64 };
static const unsigned long long kBadBase = 1ull << 62;

sw_status swmi::run_score(sw_context* ctx, const uint8_t* d_a, int64_t M, const uint8_t* d_b, int64_t N,
                          const sw_scoring* sc, const sw_options* o, void* ws, size_t ws_bytes,
                          sw_score_result* out) {
    const ScorePlan p = plan_score(ctx, M, N, o);
    if (ws_bytes < p.total) return fail(SW_ENOMEM, "workspace of %zu bytes, need %zu", ws_bytes, p.total);
    uint8_t* base = (uint8_t*)ws;
    uint8_t* misc = base + p.off_misc;
    hipStream_t st = ctx->stream;
    HIP_TRY(launch_zero(base + p.off_zero, p.zero_bytes, st));
    HIP_TRY(launch_encode(d_a, M, base + p.off_a, 0, 64, (unsigned long long*)(misc + MISC_BAD_A), st));
    HIP_TRY(launch_encode(d_b, N, base + p.off_b, kBPad, kBPadTail, (unsigned long long*)(misc + MISC_BAD_B), st));

    const int prune = (o && o->prune_mode != SW_PRUNE_NONE) ? 1 : 0;
    const int32_t thr = (o && o->prune_mode == SW_PRUNE_LEARNED) ? o->threshold : 0;
    FwdArgs a{};
    a.a = base + p.off_a;
    a.b = base + p.off_b + kBPad;
    a.M = M;
    a.N = N;
    a.match = sc->match;
    a.mismatch = sc->mismatch;
    a.open = sc->gap_open;
    a.ext = sc->gap_extend;
    a.Q = p.Q;
    a.W = p.W;
    a.n_bands = p.n_bands;
    a.slots = (int2*)(base + p.off_slots);
    a.slot_stride = p.slot_stride;
    a.nslot = p.nslot;
    a.progress = (int32_t*)(base + p.off_prog);
    a.ticket = (uint32_t*)(misc + MISC_TICKET);
    a.gbest = (int32_t*)(misc + MISC_GBEST);
    a.lbuf = (int2*)(base + p.off_lbuf);
    a.recs = (TaskRec*)(base + p.off_recs);
    a.pruned_cells = (unsigned long long*)(misc + MISC_PRUNED);
    a.prune = prune;
    a.threshold = thr;
    HIP_TRY(launch_fwd(a, p.R, p.grid, st));
    HIP_TRY(launch_reduce(a.recs, p.Q * p.n_bands, N, (ScoreOut*)(misc + MISC_OUT), st));
    HIP_TRY(hipMemcpyAsync(ctx->host_misc, misc, 128, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));

    const uint8_t* hm = (const uint8_t*)ctx->host_misc;
    unsigned long long bad_a, bad_b, pruned;
    std::memcpy(&bad_a, hm + MISC_BAD_A, 8);
    std::memcpy(&bad_b, hm + MISC_BAD_B, 8);
    std::memcpy(&pruned, hm + MISC_PRUNED, 8);
    if (bad_a) return fail(SW_EINVAL, "sequence a: byte at offset %llu is not one of ACGTacgt", kBadBase - bad_a);
    if (bad_b) return fail(SW_EINVAL, "sequence b: byte at offset %llu is not one of ACGTacgt", kBadBase - bad_b);
    ScoreOut so;
    std::memcpy(&so, hm + MISC_OUT, sizeof so);
    if (so.status) return fail(SW_EINTERNAL, "score pass: endpoint of the best score was not tracked");
    std::memset(out, 0, sizeof *out);
    out->score = so.score;
    out->end_a = so.end_a;
    out->end_b = so.end_b;
    out->threshold = thr;
    const unsigned long long total = (unsigned long long)M * (unsigned long long)N;
    out->cells_computed = (int64_t)(pruned >= total ? 0 : total - pruned);
    return SW_OK;
}

// ------------------------------------------------------------------------ C ABI: score

extern "C" size_t sw_score_workspace_size(sw_context* ctx, int64_t len_a, int64_t len_b, const sw_options* o) {
    if (!ctx || len_a < 0 || len_b < 0) return 0;
    return plan_score(ctx, len_a, len_b, o).total;
}

extern "C" sw_status sw_score_dev(sw_context* ctx, const uint8_t* d_a, int64_t len_a, const uint8_t* d_b,
                                  int64_t len_b, const sw_scoring* scoring, const sw_options* options,
                                  void* d_workspace, size_t workspace_bytes, sw_score_result* out) {
    if (!ctx || !out) return fail(SW_EINVAL, "sw_score_dev: NULL context or result");
    sw_status st;
    if ((st = check_scoring(scoring)) != SW_OK) return st;
    if ((st = check_lengths(len_a, len_b, scoring)) != SW_OK) return st;
    if ((st = check_options(options)) != SW_OK) return st;
    if ((len_a && !d_a) || (len_b && !d_b)) return fail(SW_EINVAL, "sw_score_dev: NULL sequence pointer");
    if (len_a == 0 || len_b == 0) {
        std::memset(out, 0, sizeof *out);
        out->end_a = out->end_b = -1;
        return SW_OK;
    }
    if (!d_workspace) return fail(SW_EINVAL, "sw_score_dev: NULL workspace");
    HIP_TRY(hipSetDevice(ctx->device));
    return run_score(ctx, d_a, len_a, d_b, len_b, scoring, options, d_workspace, workspace_bytes, out);
}

// Validates host letters on the host (so the offset of a bad letter is exact) and uploads them.
sw_status swmi::upload_pair(sw_context* ctx, const char* a, int64_t la, const char* b, int64_t lb,
                            uint8_t** d_a, uint8_t** d_b) {
    void* buf;
    sw_status st = ctx_buffer(ctx, BUF_INPUT, (size_t)la + (size_t)lb + 512, &buf);
    if (st != SW_OK) return st;
    *d_a = (uint8_t*)buf;
    *d_b = (uint8_t*)buf + align_up((size_t)la + 1, 256);
    HIP_TRY(hipMemcpyAsync(*d_a, a, (size_t)la, hipMemcpyHostToDevice, ctx->stream));
    HIP_TRY(hipMemcpyAsync(*d_b, b, (size_t)lb, hipMemcpyHostToDevice, ctx->stream));
    return SW_OK;
}

extern "C" sw_status sw_score(sw_context* ctx, const char* a, int64_t len_a, const char* b, int64_t len_b,
                              const sw_scoring* scoring, const sw_options* options, sw_score_result* out) {
    if (!ctx || !out) return fail(SW_EINVAL, "sw_score: NULL context or result");
    sw_status st;
    if ((st = check_scoring(scoring)) != SW_OK) return st;
    if ((st = check_lengths(len_a, len_b, scoring)) != SW_OK) return st;
    if ((st = check_options(options)) != SW_OK) return st;
    if ((len_a && !a) || (len_b && !b)) return fail(SW_EINVAL, "sw_score: NULL sequence pointer");
    if (len_a == 0 || len_b == 0) {
        std::memset(out, 0, sizeof *out);
        out->end_a = out->end_b = -1;
        return SW_OK;
    }
    HIP_TRY(hipSetDevice(ctx->device));
    uint8_t *d_a, *d_b;
    if ((st = upload_pair(ctx, a, len_a, b, len_b, &d_a, &d_b)) != SW_OK) return st;
    const size_t need = plan_score(ctx, len_a, len_b, options).total;
    void* ws;
    if ((st = ctx_buffer(ctx, BUF_WORK, need, &ws)) != SW_OK) return st;
    return run_score(ctx, d_a, len_a, d_b, len_b, scoring, options, ws, need, out);
}
