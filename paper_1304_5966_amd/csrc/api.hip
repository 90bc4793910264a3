// Host side of libswmi: errors, context, argument checks, engine planning and
// launch, and the score entry points of the C ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <numeric>
#include <string>

#include "swmi.h"
#include "swmi_host.h"
#include "swmi_internal.h"

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

#define HIP_TRY(expr)                                                                           \
    do {                                                                                        \
        hipError_t e_ = (expr);                                                                 \
        if (e_ != hipSuccess) return fail(SW_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

extern "C" const char* sw_last_error(void) { return g_err.c_str(); }
extern "C" const char* sw_version(void) { return "swmi 0.2 (gfx950)"; }

size_t swmi::align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

const char* swmi::engine_status_text(int32_t status) {
    return status == 2 ? "a stripe hand-off wait timed out (launch abandoned)"
                       : "the endpoint of the best score was not tracked";
}

// ------------------------------------------------------------------------ fixed scratch

// Workspace of sw_score_dev_noalloc: one fixed device array per GPU, held until
// the process ends.  In host code `scratch` names a host-side stand-in, not the
// device memory; the device address comes from hipGetSymbolAddress, once per
// device (scratch_address), and only that address is ever passed to kernels or
// copies.
static __device__ __align__(256) uint8_t scratch[SW_NOALLOC_SCRATCH_BYTES];

static std::mutex g_scratch_mu;
static void* g_scratch_ptr[64];  // device address of `scratch` per device ordinal

// Device address of the scratch array on `device`, which must be current.
static sw_status scratch_address(int device, void** out) {
    if (device < 0 || device >= 64) return fail(SW_EUNSUPPORTED, "device ordinal %d above 63", device);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void* ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(SW_EDEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", device, hipGetErrorString(e));
        g_scratch_ptr[device] = ptr;
    }
    *out = g_scratch_ptr[device];
    return SW_OK;
}

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
        return fail(SW_EUNSUPPORTED, "sw_context_create: device is %s, kernels are built for gfx950",
                    prop.gcnArchName);
    sw_context* c = new (std::nothrow) sw_context();
    if (!c) return fail(SW_ENOMEM, "sw_context_create: out of host memory");
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    c->num_cu = prop.multiProcessorCount;
    sw_status sst = scratch_address(device, &c->scratch);
    if (sst != SW_OK) {
        delete c;
        return sst;
    }
    c->host_misc_bytes = (size_t)64 << 10;
    hipError_t e = hipHostMalloc((void**)&c->host_misc, c->host_misc_bytes, hipHostMallocDefault);
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
    swmi::free_batch_graph(ctx->batch_graph);
    delete ctx;
    return SW_OK;
}

extern "C" sw_status sw_context_set_tuning(sw_context* ctx, int32_t cls, int32_t R, int32_t wpc) {
    if (!ctx) return fail(SW_EINVAL, "null context");
    if (cls < SW_TUNE_PAIR_SMALL || cls > SW_TUNE_BATCH) return fail(SW_EINVAL, "unknown tune class %d", cls);
    if (R != 0 && R != 4 && R != 6 && R != 8) return fail(SW_EINVAL, "rows_per_lane must be 0, 4, 6 or 8 (got %d)", R);
    if (wpc < 0 || wpc > 16) return fail(SW_EINVAL, "waves_per_cu must be 0..16 (got %d)", wpc);
    ctx->tuned_R[cls] = R;
    ctx->tuned_wpc[cls] = wpc;
    return SW_OK;
}

extern "C" sw_status sw_context_set_max_workspace(sw_context* ctx, size_t bytes) {
    if (!ctx) return fail(SW_EINVAL, "null context");
    ctx->max_workspace_bytes = bytes;
    size_t held = 0;
    for (const auto& b : ctx->bufs) held += b.bytes;
    if (bytes && held > bytes) {  // release what the new limit no longer covers
        (void)hipSetDevice(ctx->device);
        if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
        else (void)hipDeviceSynchronize();
        for (auto& b : ctx->bufs) {
            (void)hipFree(b.ptr);
            b.ptr = nullptr;
            b.bytes = 0;
        }
    }
    return SW_OK;
}

extern "C" sw_status sw_context_set_band_width(sw_context* ctx, int32_t cls, int32_t band_width) {
    if (!ctx) return fail(SW_EINVAL, "null context");
    if (cls < SW_TUNE_PAIR_SMALL || cls > SW_TUNE_BATCH) return fail(SW_EINVAL, "unknown tune class %d", cls);
    if (band_width < 0 || band_width % kTick)
        return fail(SW_EINVAL, "band_width must be 0 or a positive multiple of 64 (got %d)", band_width);
    ctx->tuned_bw[cls] = band_width;
    return SW_OK;
}

extern "C" sw_status sw_context_get_band_width(const sw_context* ctx, int32_t cls, int32_t* band_width) {
    if (!ctx || !band_width) return fail(SW_EINVAL, "null argument");
    if (cls < SW_TUNE_PAIR_SMALL || cls > SW_TUNE_BATCH) return fail(SW_EINVAL, "unknown tune class %d", cls);
    *band_width = ctx->tuned_bw[cls];
    return SW_OK;
}

extern "C" sw_status sw_context_get_tuning(const sw_context* ctx, int32_t cls, int32_t* R, int32_t* wpc) {
    if (!ctx || !R || !wpc) return fail(SW_EINVAL, "null argument");
    if (cls < SW_TUNE_PAIR_SMALL || cls > SW_TUNE_BATCH) return fail(SW_EINVAL, "unknown tune class %d", cls);
    *R = ctx->tuned_R[cls];
    *wpc = ctx->tuned_wpc[cls];
    return SW_OK;
}

sw_status swmi::ctx_buffer(sw_context* ctx, int slot, size_t bytes, void** out) {
    DevBuf& b = ctx->bufs[slot];
    if (b.bytes < bytes && ctx->max_workspace_bytes) {
        size_t held = 0;
        for (int i = 0; i < BUF_COUNT; ++i)
            if (i != slot) held += ctx->bufs[i].bytes;
        if (held + bytes > ctx->max_workspace_bytes)
            return fail(SW_ENOMEM, "the call needs %zu more bytes of device workspace; the context holds %zu and "
                        "its limit is %zu (sw_context_set_max_workspace)", bytes, held, ctx->max_workspace_bytes);
    }
    if (b.bytes < bytes) {
        if (b.ptr) {
            (void)hipStreamSynchronize(ctx->stream);
            (void)hipFree(b.ptr);
            b.ptr = nullptr;
            b.bytes = 0;
        }
        size_t want = std::max(bytes, (size_t)1 << 20);
        if (ctx->max_workspace_bytes) want = bytes;  // under a limit, no rounding up
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

sw_status swmi::read_back(sw_context* ctx, const void* dev, size_t bytes, void** host) {
    if (bytes > ctx->host_misc_bytes) return fail(SW_EINTERNAL, "read_back of %zu bytes", bytes);
    HIP_TRY(hipMemcpyAsync(ctx->host_misc, dev, bytes, hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    *host = ctx->host_misc;
    return SW_OK;
}

// ------------------------------------------------------------------------ checks

sw_status swmi::check_scoring(const sw_scoring* s, sw_scoring* norm) {
    if (!s) return fail(SW_EINVAL, "scoring is NULL");
    if (s->gap_extend <= 0 || s->gap_open < s->gap_extend || s->gap_open > (1 << 20))
        return fail(SW_EINVAL, "need 0 < gap_extend <= gap_open <= 2^20 (got %d, %d)", s->gap_open,
                    s->gap_extend);
    *norm = *s;
    if (!s->matrix) {
        if (s->match <= 0 || s->match > 127) return fail(SW_EINVAL, "match must be in 1..127 (got %d)", s->match);
        if (s->mismatch < 0 || s->mismatch > 127)
            return fail(SW_EINVAL, "mismatch must be in 0..127 (got %d)", s->mismatch);
        return SW_OK;
    }
    const sw_matrix* m = s->matrix;
    if (m->size < 1 || m->size > kMaxClasses - 1)
        return fail(SW_EINVAL, "matrix size must be in 1..%d (got %d)", kMaxClasses - 1, m->size);
    if (!m->alphabet || !m->scores) return fail(SW_EINVAL, "matrix alphabet or scores is NULL");
    bool seen[256] = {};
    for (int i = 0; i < m->size; ++i) {
        const uint8_t c = (uint8_t)m->alphabet[i];
        const uint8_t u = (c >= 'a' && c <= 'z') ? (uint8_t)(c - 32) : c;
        if (c < 33 || c > 126) return fail(SW_EINVAL, "matrix letter %d is not a printable byte (%d)", i, c);
        if (seen[u]) return fail(SW_EINVAL, "matrix letter '%c' occurs twice (letters are case-insensitive)", c);
        seen[u] = true;
    }
    int lo = 127, hi = -128;
    for (int i = 0; i < m->size * m->size; ++i) {
        const int v = m->scores[i];
        if (v < -127) return fail(SW_EINVAL, "matrix score %d at %d is below -127", v, i);
        lo = std::min(lo, v);
        hi = std::max(hi, v);
    }
    norm->match = std::max(1, hi);
    norm->mismatch = std::max(0, -lo);
    return SW_OK;
}

sw_status swmi::check_matrix_options(const sw_scoring* sc, const sw_options* o) {
    if (!sc->matrix || !o) return SW_OK;
    if (o->prune_mode == SW_PRUNE_LEARNED && o->threshold == 0 && !o->pair_thresholds)
        return fail(SW_EUNSUPPORTED, "a threshold model needs DNA scoring (its features are DNA k-mers); "
                    "give the threshold instead");
    if (o->flags & SW_FLAG_BOTH_STRANDS)
        return fail(SW_EUNSUPPORTED, "SW_FLAG_BOTH_STRANDS needs DNA scoring (a reverse complement)");
    return SW_OK;
}

static uint8_t upper(uint8_t c) { return (c >= 'a' && c <= 'z') ? (uint8_t)(c - 32) : c; }

EncTable swmi::enc_table(const sw_scoring* sc) {
    EncTable t;
    std::memset(t.cls, -1, sizeof t.cls);
    if (!sc->matrix) {
        t.dna = 1;
        t.pad_code = kPadCode;
        return t;
    }
    const sw_matrix* m = sc->matrix;
    t.dna = 0;
    t.pad_code = m->size;  // the padding class follows the letters
    for (int i = 0; i < m->size; ++i) {
        const uint8_t u = upper((uint8_t)m->alphabet[i]);
        t.cls[u] = (int8_t)i;
        if (u >= 'A' && u <= 'Z') t.cls[u + 32] = (int8_t)i;
    }
    return t;
}

void swmi::subst_table(const sw_scoring* sc, Subst& out) {
    std::memset(&out, 0, sizeof out);
    if (!sc->matrix) return;
    const sw_matrix* m = sc->matrix;
    out.n_class = m->size + 1;
    std::memset(out.s, -128, sizeof out.s);
    for (int i = 0; i < m->size; ++i)
        for (int j = 0; j < m->size; ++j) out.s[i][j] = m->scores[i * m->size + j];
}

int32_t swmi::subst_score(const sw_scoring* sc, uint8_t x, uint8_t y) {
    if (!sc->matrix) {
        if (x > 3 || y > 3) return -128;
        return x == y ? sc->match : -sc->mismatch;
    }
    const int k = sc->matrix->size;
    if (x >= k || y >= k) return -128;
    return sc->matrix->scores[x * k + y];
}

const char* swmi::letters_text(const sw_scoring* sc) {
    return sc->matrix ? "a letter of the matrix alphabet" : "one of ACGTacgt";
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
    if (o->rows_per_lane != 0 && o->rows_per_lane != 4 && o->rows_per_lane != 6 && o->rows_per_lane != 8)
        return fail(SW_EINVAL, "rows_per_lane must be 0, 4, 6 or 8 (got %d)", o->rows_per_lane);
    if (o->waves_per_cu < 0 || o->waves_per_cu > 16)
        return fail(SW_EINVAL, "waves_per_cu must be 0..16 (got %d)", o->waves_per_cu);
    if (o->threshold < 0) return fail(SW_EINVAL, "threshold must be >= 0");
    if (o->flags & ~(SW_FLAG_GRAPH | SW_FLAG_HALVES | SW_FLAG_BOTH_STRANDS))
        return fail(SW_EINVAL, "unknown flags 0x%x", o->flags);
    if ((o->flags & SW_FLAG_HALVES) &&
        (o->prune_mode == SW_PRUNE_LEARNED || o->slab_rows > 0 || (o->flags & SW_FLAG_BOTH_STRANDS)))
        return fail(SW_EUNSUPPORTED, "SW_FLAG_HALVES does not combine with SW_PRUNE_LEARNED, row slabs or both strands");
    if ((o->flags & SW_FLAG_BOTH_STRANDS) && o->prune_mode == SW_PRUNE_LEARNED)
        return fail(SW_EUNSUPPORTED, "SW_FLAG_BOTH_STRANDS does not combine with SW_PRUNE_LEARNED");
    if (o->band_width < 0 || o->band_width % kTick)
        return fail(SW_EINVAL, "band_width must be 0 or a positive multiple of 64 (got %d)", o->band_width);
    if (o->slab_rows < 0) return fail(SW_EINVAL, "slab_rows must be >= 0 (got %d)", o->slab_rows);
    return SW_OK;
}

// ------------------------------------------------------------------------ engine plan

// Waves per workgroup of the global passes' chain launches: SWMI_CHAIN_WAVES
// (1 = off, 4 or 8), 4 if unset (on the 5 Mbp x 4 Mbp alignment: start pass 0.77 s
// and reconstruction 0.52 s, against 0.83 / 1.03 s at 8 and 0.85 / 0.91 s at 1).
static int chain_waves() {
    const char* v = std::getenv("SWMI_CHAIN_WAVES");
    const int w = (v && *v) ? std::atoi(v) : 4;
    return (w == 4 || w == 8) ? w : 1;
}

// Slot memory a launch may take beyond its minimal ring: SWMI_SLOT_ROOM_BYTES
// (bytes; 0 keeps the minimal ring), 8 GiB if unset.
static size_t slot_room_bytes() {
    const char* v = std::getenv("SWMI_SLOT_ROOM_BYTES");
    if (!v || !*v) return (size_t)8 << 30;
    return (size_t)std::strtoull(v, nullptr, 10);
}

EnginePlan swmi::plan_engine(const sw_context* ctx, const std::vector<ProbSpec>& specs, bool local,
                             int rows_per_lane, int waves_per_cu, int band_width) {
    EnginePlan p;
    p.local = local;
    double cells = 0;
    for (const auto& s : specs) cells += (double)s.M * (double)s.N;
    const double per = specs.empty() ? 0.0 : cells / (double)specs.size();
    const int cls = per >= 1e12                      ? SW_TUNE_PAIR_HUGE
                    : per >= 1e10                    ? SW_TUNE_PAIR_LARGE
                    : specs.size() > 1               ? SW_TUNE_BATCH
                                                     : SW_TUNE_PAIR_SMALL;
    const int tR = ctx->tuned_R[cls], tW = ctx->tuned_wpc[cls];
    p.R = rows_per_lane ? rows_per_lane : tR ? tR : 8;
    const int wpc = waves_per_cu ? waves_per_cu : tW ? tW : 8;
    p.wpc = wpc;
    const int64_t rows_per_stripe = (int64_t)kWave * p.R;
    // Largest-first order keeps the long problems from trailing the launch.
    std::vector<std::pair<double, size_t>> keyed(specs.size());  // (-cells, index): ties keep input order
    for (size_t i = 0; i < specs.size(); ++i) keyed[i] = {-(double)specs[i].M * (double)specs[i].N, i};
    std::sort(keyed.begin(), keyed.end());
    std::vector<size_t> order(specs.size());
    for (size_t i = 0; i < specs.size(); ++i) order[i] = keyed[i].second;
    const int64_t max_grid = (int64_t)ctx->num_cu * wpc;
    int64_t stripes = 0, maxN = 64;
    for (const auto& s : specs) {
        stripes += (s.M + rows_per_stripe - 1) / rows_per_stripe;
        maxN = std::max(maxN, s.N);
    }
    // Band width: keep the slot ring (sized as below) within a fixed budget.
    // Wide bands keep the stripe pipeline full: consecutive stripes run about
    // three ticks apart, so a band of T ticks keeps all waves busy only while
    // grid * 3 <= T.  32 GiB (of 288 GB HBM) gives 2 Mi columns at 2048 waves;
    // on the 5 Mbp x 4 Mbp pair that budget (two bands) measured faster than
    // 16, 24 or 64 GiB.
    const int64_t grid_est = std::max<int64_t>(1, std::min<int64_t>(max_grid, stripes * ((maxN + 63) / 64)));
    const int64_t G_est = std::max<int64_t>(1, std::min<int64_t>((int64_t)specs.size(), grid_est));
    const int64_t nslot_est = grid_est + 1 + (G_est > 1 ? 2 * G_est : 0);
    const size_t slot_budget = (size_t)32 << 30;
    int64_t Wg = (int64_t)(slot_budget / ((size_t)nslot_est * sizeof(int2))) - (kSlotPad + 2 * kTick);
    Wg = std::max<int64_t>(kTick, Wg / kTick * kTick);
    // The global recurrence in a diagonal band: a stripe writes only the columns of
    // the ticks that hold band cells, and its slot holds only those (slot_cols).
    // Where such slots fit the budget, each problem is one column band: no stripe
    // then waits for the stripe to its left to finish.
    auto slot_cols = [&](const ProbSpec& s, int64_t W) -> int64_t {
        const int64_t whole = W + 2 * kTick;
        if (local || (s.d_lo <= -kNoBand && s.d_hi >= kNoBand)) return whole;
        return std::min<int64_t>(whole, s.d_hi - s.d_lo + (int64_t)kWave * p.R + 4 * kTick);
    };
    if (!local && !band_width) {
        int64_t cols = kTick;
        for (const auto& s : specs) cols = std::max(cols, slot_cols(s, (s.N + kTick - 1) / kTick * kTick));
        if ((size_t)nslot_est * (size_t)(kSlotPad + cols + 2 * kTick) * sizeof(int2) <= slot_budget)
            Wg = (maxN + kTick - 1) / kTick * kTick;
    }
    if (band_width) Wg = band_width;
    else if (local && ctx->tuned_bw[cls]) Wg = ctx->tuned_bw[cls];  // a tuned width (local passes only)

    int64_t task = 0, lrow = 0, Wmax = kTick, Cmax = kTick;
    p.probs.reserve(specs.size());
    p.order.assign(order.begin(), order.end());
    for (size_t oi : order) {
        const ProbSpec& s = specs[oi];
        Prob pr{};
        pr.a_off = s.a_off;
        pr.b_off = s.b_off;
        pr.M = s.M;
        pr.N = s.N;
        const int64_t N64 = (s.N + kTick - 1) / kTick * kTick;
        pr.W = std::min(Wg, std::max<int64_t>(kTick, N64));
        pr.n_bands = (s.N + pr.W - 1) / pr.W;
        pr.Q = (s.M + rows_per_stripe - 1) / rows_per_stripe;
        pr.task0 = task;
        pr.lbuf_off = lrow;
        pr.out_off = s.out_off;
        pr.d_lo = s.d_lo;
        pr.d_hi = s.d_hi;
        pr.top_kind = s.top_kind;
        pr.left_kind = s.left_kind;
        pr.top_open = s.top_open;
        pr.left_open = s.left_open;
        pr.target = s.target;
        pr.prune = s.prune;
        pr.track = s.track;
        pr.top_off = s.top_off;
        pr.rows_after = s.rows_after;
        task += pr.Q * pr.n_bands;
        if (pr.n_bands > 1) lrow += pr.Q * rows_per_stripe;
        Wmax = std::max(Wmax, pr.W);
        Cmax = std::max(Cmax, slot_cols(s, pr.W));
        p.probs.push_back(pr);
    }
    p.n_probs = (int64_t)p.probs.size();
    p.n_tasks = task;
    p.lbuf_rows = lrow;
    // Tasks holding a cell of their problem's kept band (all of them when unbanded).
    std::vector<uint8_t> active((size_t)p.n_tasks, 1);
    int64_t n_active = p.n_tasks;
    bool banded = false;
    for (const Prob& pr : p.probs) {
        if (pr.d_lo <= -kNoBand && pr.d_hi >= kNoBand) continue;
        banded = true;
        for (int64_t l = 0; l < pr.Q * pr.n_bands; ++l)
            if (!task_in_band(pr, l / pr.Q, l % pr.Q, p.R)) {
                active[(size_t)(pr.task0 + l)] = 0;
                --n_active;
            }
    }
    p.n_tickets = n_active;
    p.grid = (int)std::max<int64_t>(1, std::min<int64_t>(max_grid, n_active));
    // The banded global passes at 4 rows per lane run in chain workgroups (consecutive
    // stripes linked through LDS; with matrix scoring, or scores too large for the
    // shifted domain, the launch runs one wave per workgroup on the same table).
    p.chain = (!local && p.R == 4) ? chain_waves() : 1;

    // Ticket order.  Problems (largest first) go in groups of G; inside a group
    // the tasks go round-robin over the problems (task s of every problem that
    // has one, then task s + 1, ...), so consecutive stripes of a problem are up
    // to G tickets apart and a stripe rarely waits for the one above.  G = one
    // generation of waves (the grid): a same-box sweep on 20 000 pairs gave
    // 3.70 TCUPS at grid/2, 3.82 at grid and 3.83 at twice the grid.
    // Slots: ticket k writes slot k mod nslot, which its previous owner's reader
    // (at most G tickets after that owner) must have finished with.  With one
    // slot per wave plus 2G, that reader is more than a whole generation of
    // waves older than k, so the wait is rare; and since nslot > G every ticket
    // waits only on older tickets.
    // Chain launches take each problem's tasks in runs of `chain` (their waves link
    // through LDS): a consumer is then at most G * chain tickets after its producer.
    const int64_t G = std::max<int64_t>(1, std::min<int64_t>(p.n_probs, (int64_t)p.grid));
    const int64_t run = p.chain;
    p.nslot = std::max<int64_t>(2, (int64_t)p.grid + 1 + (G > 1 ? 2 * G * run : 0));
    p.slot_stride = (int64_t)align_up((size_t)(kSlotPad + (local ? Wmax + 2 * kTick : Cmax) + 2 * kTick), 64);
    // Where slots are small (many short problems), up to 8 GiB of them: tasks of
    // different sizes finish out of ticket order, and a slot whose last reader is
    // a long stripe would otherwise hold up the ticket that reuses it.
    const int64_t roomy = (int64_t)(slot_room_bytes() / ((size_t)p.slot_stride * sizeof(int2)));
    p.nslot = std::max(p.nslot, std::min<int64_t>(p.n_tickets, roomy));
    p.tickets.assign((size_t)p.n_tickets, Ticket{});
    std::vector<int32_t> tick_of((size_t)p.n_tasks, -1);  // task id (task0 + local) -> ticket, -1: none
    std::vector<int32_t> ntask((size_t)p.n_probs);         // tasks per problem (compact copy for the loops)
    for (int64_t pi = 0; pi < p.n_probs; ++pi) ntask[(size_t)pi] = (int32_t)(p.probs[pi].Q * p.probs[pi].n_bands);
    int64_t k = 0;
    std::vector<int32_t> live;  // problems of the group with a task s, in table order
    std::vector<int32_t> cursor;  // chain order: each live problem's next task
    for (int64_t g0 = 0; g0 < p.n_probs; g0 += G) {
        const int64_t g1 = std::min(p.n_probs, g0 + G);
        live.clear();
        for (int64_t pi = g0; pi < g1; ++pi)
            if (ntask[(size_t)pi] > 0) live.push_back((int32_t)pi);
        if (run == 1) {
            for (int32_t s = 0; !live.empty(); ++s) {
                size_t keep = 0;
                for (const int32_t pi : live) {
                    const int64_t id = p.probs[pi].task0 + s;
                    if (!banded || active[(size_t)id]) {
                        Ticket& tk = p.tickets[(size_t)k];
                        tk.pi = pi;
                        tk.local = s;
                        tick_of[(size_t)id] = (int32_t)k;
                        ++k;
                    }
                    if (s + 1 < ntask[(size_t)pi]) live[keep++] = pi;
                }
                live.resize(keep);
            }
        } else {
            // runs of `run` tickets (tasks with a cell in the band) per problem in turn
            cursor.assign((size_t)(g1 - g0), 0);
            while (!live.empty()) {
                size_t keep = 0;
                for (const int32_t pi : live) {
                    int32_t& s = cursor[(size_t)(pi - g0)];
                    for (int64_t taken = 0; taken < run && s < ntask[(size_t)pi]; ++s) {
                        const int64_t id = p.probs[pi].task0 + s;
                        if (banded && !active[(size_t)id]) continue;
                        Ticket& tk = p.tickets[(size_t)k];
                        tk.pi = pi;
                        tk.local = s;
                        tick_of[(size_t)id] = (int32_t)k;
                        ++k;
                        ++taken;
                    }
                    if (s < ntask[(size_t)pi]) live[keep++] = pi;
                }
                live.resize(keep);
            }
        }
    }
    // Links, in ticket order (the tickets are written sequentially; the problems and
    // tick_of are read near the round-robin position).  The reader of a ticket's slot
    // is its consumer, the stripe below.
    for (int64_t j = 0; j < p.n_tickets; ++j) {
        Ticket& tk = p.tickets[(size_t)j];
        const Prob& pr = p.probs[tk.pi];
        const int32_t* tof = tick_of.data() + pr.task0;
        const int64_t l = tk.local, band = l / pr.Q, q = l - band * pr.Q;
        tk.prod = q > 0 ? tof[l - 1] : -1;
        tk.left = band > 0 ? tof[l - pr.Q] : -1;
        tk.corner = (q > 0 && band > 0 && tk.prod < 0) ? tof[l - pr.Q - 1] : -1;
        tk.cons = q + 1 < pr.Q ? tof[l + 1] : -1;
        tk.reuse_reader = j >= p.nslot ? p.tickets[(size_t)(j - p.nslot)].cons : -1;
    }

    size_t off = 0;
    p.off_tickets = off;
    off = align_up(off + (size_t)p.n_tickets * sizeof(Ticket), 256);
    p.off_probs = off;
    off = align_up(off + (size_t)p.n_probs * sizeof(Prob), 256);
    p.off_slots = off;
    off = align_up(off + (size_t)p.nslot * p.slot_stride * sizeof(int2), 256);
    p.off_lbuf = off;
    off = align_up(off + (size_t)p.lbuf_rows * sizeof(int2), 256);
    p.off_recs = off;
    off = align_up(off + (size_t)p.n_tasks * sizeof(TaskRec), 256);
    p.off_outs = off;
    off = align_up(off + (size_t)p.n_probs * sizeof(ScoreOut), 256);
    p.off_zero = off;  // cleared on every launch
    p.off_prog = off;
    off = align_up(off + (size_t)p.n_tickets * sizeof(int32_t), 256);
    p.off_gbest = off;
    off = align_up(off + (size_t)p.n_probs * sizeof(int32_t), 256);
    p.off_pruned = off;
    off = align_up(off + (size_t)p.n_probs * sizeof(unsigned long long), 256);
    p.off_misc = off;
    off = align_up(off + MISC_BYTES, 256);
    p.zero_bytes = off - p.off_zero;
    p.total = off;
    return p;
}

sw_status swmi::upload_engine_table(sw_context* ctx, const EnginePlan& plan, void* ws) {
    HIP_TRY(hipMemcpyAsync((uint8_t*)ws + plan.off_probs, plan.probs.data(), (size_t)plan.n_probs * sizeof(Prob),
                           hipMemcpyHostToDevice, ctx->stream));
    HIP_TRY(hipMemcpyAsync((uint8_t*)ws + plan.off_tickets, plan.tickets.data(),
                           (size_t)plan.n_tickets * sizeof(Ticket), hipMemcpyHostToDevice, ctx->stream));
    return SW_OK;
}

// Schedule-perturbation seed of the engine (a test mode): SWMI_SCHEDULE_JITTER,
// a nonzero integer, makes waves pause at pseudo-random points; results must not
// change.  Read at every launch.
static uint32_t schedule_jitter() {
    const char* v = std::getenv("SWMI_SCHEDULE_JITTER");
    return (v && *v) ? (uint32_t)std::strtoul(v, nullptr, 10) : 0u;
}

// Longest wait of a launch before it gives up (ticks of the device's 100 MHz
// real-time counter): SWMI_WAIT_LIMIT_US microseconds, 120 s if unset.  A tiny
// limit is a test mode that drives the abort path without a hang.
static uint64_t wait_limit_ticks() {
    const char* v = std::getenv("SWMI_WAIT_LIMIT_US");
    const unsigned long long us = (v && *v) ? std::strtoull(v, nullptr, 10) : 120000000ull;
    return (uint64_t)std::max(1ull, std::min(us, 3600000000ull)) * 100ull;
}

// Kernel launches only (capturable in a HIP graph: no copies, no memsets).
sw_status swmi::launch_engine_kernels(sw_context* ctx, const EnginePlan& plan, const uint8_t* a_codes,
                                      const uint8_t* b_codes, const sw_scoring* sc, void* ws, int32_t* out_h,
                                      int32_t* out_f, const int32_t* top_h, const int32_t* top_f) {
    uint8_t* base = (uint8_t*)ws;
    hipStream_t st = ctx->stream;
    HIP_TRY(launch_zero(base + plan.off_zero, plan.zero_bytes, st));
    // Every ticket may wait only on older tickets (the pipeline's deadlock freedom).
    for (int64_t k = 0; k < plan.n_tickets; ++k) {
        const Ticket& t = plan.tickets[(size_t)k];
        if (t.prod >= k || t.left >= k || t.reuse_reader >= k || t.corner >= k)
            return fail(SW_EINTERNAL, "engine plan: ticket %lld waits on a younger ticket", (long long)k);
        if (t.cons >= plan.n_tickets || (t.cons >= 0 && t.cons <= k))
            return fail(SW_EINTERNAL, "engine plan: ticket %lld names consumer %d", (long long)k, t.cons);
        if (!plan.local && t.cons >= 0) {
            // the columns this task writes for its consumer fit its slot
            const Prob& pr = plan.probs[(size_t)t.pi];
            const int64_t band = t.local / pr.Q, q = t.local - band * pr.Q;
            const int W = (int)std::min(pr.W, pr.N - band * pr.W);
            const int n_ticks = (W + 2 * kTick - 2) / kTick;
            int lo, hi, first, last;
            band_ticks(pr, q * (int64_t)kWave * plan.R, band * pr.W, plan.R, n_ticks, lo, hi);
            if (lo > hi) {
                lo = 0;
                hi = n_ticks - 1;
            }
            slot_columns(lo, hi, first, last);
            if (last - first + 1 > plan.slot_stride - kSlotPad)
                return fail(SW_EINTERNAL, "engine plan: ticket %lld writes %d columns to a slot of %lld", (long long)k,
                            last - first + 1, (long long)(plan.slot_stride - kSlotPad));
        }
    }
    EngineArgs a{};
    a.tickets = (const Ticket*)(base + plan.off_tickets);
    a.probs = (const Prob*)(base + plan.off_probs);
    a.n_probs = plan.n_probs;
    a.n_tickets = plan.n_tickets;
    a.a_codes = a_codes;
    a.b_codes = b_codes;
    a.match = sc->match;
    a.mismatch = sc->mismatch;
    a.open = sc->gap_open;
    a.ext = sc->gap_extend;
    a.slots = (int2*)(base + plan.off_slots);
    a.slot_stride = plan.slot_stride;
    a.nslot = plan.nslot;
    a.progress = (int32_t*)(base + plan.off_prog);
    a.ticket = (uint32_t*)(base + plan.off_misc + MISC_TICKET);
    a.gbest = (int32_t*)(base + plan.off_gbest);
    a.lbuf = (int2*)(base + plan.off_lbuf);
    a.recs = (TaskRec*)(base + plan.off_recs);
    a.pruned = (unsigned long long*)(base + plan.off_pruned);
    a.out_h = out_h;
    a.out_f = out_f;
    a.top_h = top_h;
    a.top_f = top_f;
    a.jitter = schedule_jitter();
    a.abort_flag = (int32_t*)(base + plan.off_misc + MISC_ABORT);
    a.wait_limit = wait_limit_ticks();
    subst_table(sc, a.sub);
    for (const Prob& pr : plan.probs)
        if (pr.top_kind == BORDER_BUF && (!top_h || !top_f || pr.top_off < 0))
            return fail(SW_EINTERNAL, "engine plan: a buffer top border without its row");
    const bool cd = sc->match + cd_bias_ext(plan.R) * sc->gap_extend <= 127;
    HIP_TRY(launch_engine(a, plan.R, plan.wpc, plan.local, cd, plan.grid, plan.chain, st));
    HIP_TRY(launch_reduce(a.recs, a.probs, plan.n_probs, plan.R, (ScoreOut*)(base + plan.off_outs), a.gbest,
                          a.pruned, a.abort_flag, st));
    return SW_OK;
}

sw_status swmi::run_engine(sw_context* ctx, const EnginePlan& plan, const uint8_t* a_codes, const uint8_t* b_codes,
                           const sw_scoring* sc, void* ws, int32_t* out_h, int32_t* out_f, const int32_t* top_h,
                           const int32_t* top_f) {
    sw_status st = upload_engine_table(ctx, plan, ws);
    if (st != SW_OK) return st;
    return launch_engine_kernels(ctx, plan, a_codes, b_codes, sc, ws, out_h, out_f, top_h, top_f);
}

// ------------------------------------------------------------------------ score pass

// Strands of a score pass: 1 (A against B) or, with SW_FLAG_BOTH_STRANDS, 2 (also
// A against the reverse complement of B).
static int strands_of(const sw_options* o) { return (o && (o->flags & SW_FLAG_BOTH_STRANDS)) ? 2 : 1; }

// Score workspace: [a codes][b codes, one padded copy per strand][encode flags][slab rows][engine region]
static size_t a_code_bytes(int64_t M) { return align_up((size_t)M + 64, 256); }
static size_t b_code_bytes(int64_t N) { return align_up((size_t)(kBPad + N + kBPadTail), 256); }
static size_t codes_bytes(int64_t M, int64_t N, int S) {
    return a_code_bytes(M) + (size_t)S * b_code_bytes(N) + 256;
}

// One problem per strand over `rows` rows of A (from a_off) and all of B.
static std::vector<ProbSpec> score_specs(int64_t a_off, int64_t rows, int64_t N, const sw_options* o, int S) {
    std::vector<ProbSpec> v((size_t)S);
    for (int s = 0; s < S; ++s) {
        ProbSpec& p = v[(size_t)s];
        p.a_off = a_off;
        p.b_off = (int64_t)((size_t)s * b_code_bytes(N)) + kBPad;
        p.M = rows;
        p.N = N;
        p.prune = (o && o->prune_mode != SW_PRUNE_NONE) ? 1 : 0;
        p.target = (o && o->prune_mode == SW_PRUNE_LEARNED) ? o->threshold : 0;
        p.track = 1;
    }
    return v;
}

// Row slabs: above this many cells per strand the score pass runs as several
// launches of consecutive rows (about 30 s each at the measured rate), so that no
// single launch keeps the device busy for minutes.
static const double kSlabCells = 1.0e14;

// Rows of A per score-pass launch; 0 = the whole matrix in one launch.
static int64_t slab_rows_for(int64_t M, int64_t N, const sw_options* o) {
    if (o && o->slab_rows > 0) return o->slab_rows >= M ? 0 : o->slab_rows;
    const double cells = (double)M * (double)N * strands_of(o);
    if (cells <= kSlabCells) return 0;
    const int64_t n = (int64_t)std::ceil(cells / kSlabCells);
    return (M + n - 1) / n;
}

// One slab-boundary row: {H or F} x (N + 1) columns x strands; four of them
// (H and F, double-buffered).
static size_t slab_row_bytes(int64_t N, int S) { return align_up((size_t)S * (size_t)(N + 1) * sizeof(int32_t), 256); }

static bool uses_model(const sw_options* o) {
    return o && o->prune_mode == SW_PRUNE_LEARNED && o->threshold == 0;
}

// Engine bytes of a score pass in slabs of h rows (0: one launch): the larger of
// the plans of a full slab and of the last one.
static size_t score_engine_bytes(const sw_context* ctx, int64_t M, int64_t N, const sw_options* o, int64_t h, int S) {
    auto plan_bytes = [&](int64_t rows) {
        return plan_engine(ctx, score_specs(0, rows, N, o, S), true, o ? o->rows_per_lane : 0,
                           o ? o->waves_per_cu : 0, o ? o->band_width : 0)
            .total;
    };
    if (!h) return plan_bytes(M);
    const int64_t last = M - (M - 1) / h * h;
    return std::max(plan_bytes(h), plan_bytes(last));
}

size_t swmi::score_workspace_size(const sw_context* ctx, int64_t M, int64_t N, const sw_options* o) {
    if (o && (o->flags & SW_FLAG_HALVES)) return halves_workspace_size(ctx, M, N, o);
    const int S = strands_of(o);
    const int64_t h = slab_rows_for(M, N, o);
    size_t total = codes_bytes(M, N, S) + (h ? 4 * slab_row_bytes(N, S) : 0) + score_engine_bytes(ctx, M, N, o, h, S);
    if (uses_model(o)) total = std::max(total, predict_workspace_size(M, N, 1));
    return total;
}

static void report_progress(const sw_options* o, int64_t done, int64_t total) {
    if (o && o->progress) o->progress(o->progress_user, done, total);
}

// Bad-letter flags of the encode kernels, copied to the host.
static sw_status check_encoded(const uint8_t* flags_host, const sw_scoring* sc) {
    unsigned long long bad_a, bad_b;
    std::memcpy(&bad_a, flags_host, 8);
    std::memcpy(&bad_b, flags_host + 8, 8);
    if (bad_a) return fail(SW_EINVAL, "sequence a: byte at offset %llu is not %s", kBadBase - bad_a, letters_text(sc));
    if (bad_b) return fail(SW_EINVAL, "sequence b: byte at offset %llu is not %s", kBadBase - bad_b, letters_text(sc));
    return SW_OK;
}

// The score pass as consecutive row slabs (paper Section 2, linear memory): slab
// k covers rows [r0, r1) of A against all of B (each strand one problem of the
// launch) and its row 0 is the previous slab's last row (H and F per column, kept
// in the workspace).  The pruning bound of a tile counts the rows of later slabs,
// so it stays a bound of every path through the tile.  Per strand, the best cell
// so far becomes the next slab's target: only cells that reach it are tracked,
// and a tie goes to the earlier slab, whose rows come first -- the
// lexicographically first endpoint.  res[s]: strand s's result.
static sw_status run_score_slabs(sw_context* ctx, const uint8_t* a_codes, int64_t M, const uint8_t* b_codes,
                                 int64_t N, const sw_scoring* sc, const sw_options* o, int64_t h, int S, uint8_t* rows,
                                 uint8_t* eng, size_t eng_bytes, ScoreOut* res) {
    const size_t rb = slab_row_bytes(N, S);
    int32_t* rowH[2] = {(int32_t*)rows, (int32_t*)(rows + rb)};
    int32_t* rowF[2] = {(int32_t*)(rows + 2 * rb), (int32_t*)(rows + 3 * rb)};
    const int32_t t_user = (o && o->prune_mode == SW_PRUNE_LEARNED) ? o->threshold : 0;
    int32_t best[2] = {0, 0}, seen[2] = {0, 0};
    int64_t bi[2] = {-1, -1}, bj[2] = {-1, -1};
    unsigned long long pruned[2] = {0, 0};
    int k = 0;
    for (int64_t r0 = 0; r0 < M; r0 += h, ++k) {
        const Phase ph("swmi score slab");
        const int64_t r1 = std::min(M, r0 + h);
        std::vector<ProbSpec> specs = score_specs(r0, r1 - r0, N, o, S);
        for (int s = 0; s < S; ++s) {
            ProbSpec& ps = specs[(size_t)s];
            ps.top_kind = r0 == 0 ? BORDER_ZERO : BORDER_BUF;
            ps.top_off = r0 == 0 ? -1 : (int64_t)s * (N + 1);
            ps.out_off = r1 < M ? (int64_t)s * (N + 1) : -1;
            ps.rows_after = M - r1;
            ps.target = std::max(t_user, best[s]);
        }
        const EnginePlan p = plan_engine(ctx, specs, true, o ? o->rows_per_lane : 0, o ? o->waves_per_cu : 0,
                                         o ? o->band_width : 0);
        if (p.total > eng_bytes) return fail(SW_EINTERNAL, "row slab plan exceeds its workspace");
        sw_status st = run_engine(ctx, p, a_codes, b_codes, sc, eng, rowH[k & 1], rowF[k & 1],
                                  r0 == 0 ? nullptr : rowH[(k + 1) & 1], r0 == 0 ? nullptr : rowF[(k + 1) & 1]);
        if (st != SW_OK) return st;
        ScoreOut* so;
        if ((st = read_back(ctx, eng + p.off_outs, (size_t)S * sizeof(ScoreOut), (void**)&so)) != SW_OK) return st;
        for (int i = 0; i < S; ++i) {
            const int s = (int)p.order[(size_t)i];  // probs[i] is strand order[i]
            const ScoreOut& r = so[i];
            if (r.status) return fail(SW_EINTERNAL, "row slab %d: %s", k, engine_status_text(r.status));
            pruned[s] += r.pruned_cells;
            if (r.end_a >= 0 && r.score > best[s]) {
                best[s] = r.score;
                bi[s] = r0 + r.end_a;
                bj[s] = r.end_b;
            } else if (r.end_a < 0) {
                seen[s] = std::max(seen[s], r.score);  // largest H of an untracked slab (below its target)
            }
        }
        report_progress(o, r1, M);
    }
    for (int s = 0; s < S; ++s) {
        ScoreOut& r = res[s];
        r.status = 0;
        r.pruned_cells = pruned[s];
        if (best[s] >= seen[s]) {
            r.score = best[s];
            r.end_a = bi[s];
            r.end_b = bj[s];
        } else {  // a learned target missed: the largest H computed, without an endpoint
            r.score = seen[s];
            r.end_a = -1;
            r.end_b = -1;
        }
    }
    return SW_OK;
}

static sw_status run_score_once(sw_context* ctx, const uint8_t* d_a, int64_t M, const uint8_t* d_b, int64_t N,
                                const sw_scoring* sc, const sw_options* o, void* ws, size_t ws_bytes,
                                sw_score_result* out) {
    const Phase ph("swmi score pass");
    const int S = strands_of(o);
    const int64_t h = slab_rows_for(M, N, o);
    const size_t rows_bytes = h ? 4 * slab_row_bytes(N, S) : 0;
    const size_t cb = codes_bytes(M, N, S);
    const size_t need = cb + rows_bytes + score_engine_bytes(ctx, M, N, o, h, S);
    if (ws_bytes < need) return fail(SW_ENOMEM, "workspace of %zu bytes, need %zu", ws_bytes, need);
    uint8_t* a_codes = (uint8_t*)ws;
    uint8_t* b_codes = a_codes + a_code_bytes(M);
    uint8_t* flags = (uint8_t*)ws + cb - 256;
    uint8_t* rows = (uint8_t*)ws + cb;
    uint8_t* eng = rows + rows_bytes;
    hipStream_t st = ctx->stream;
    const EncTable et = enc_table(sc);
    HIP_TRY(launch_zero(flags, 256, st));
    HIP_TRY(launch_encode(d_a, M, a_codes, 0, 64, 0, et, (unsigned long long*)flags, st));
    for (int s = 0; s < S; ++s)  // strand 1: the reverse complement of B
        HIP_TRY(launch_encode(d_b, N, b_codes + (size_t)s * b_code_bytes(N), kBPad, kBPadTail,
                              s ? (ENC_REVERSE | ENC_COMPLEMENT) : 0, et, (unsigned long long*)(flags + 8), st));
    uint8_t* hm = (uint8_t*)ctx->host_misc;
    ScoreOut so[2];
    sw_status s;
    if (h) {
        // letters first: a bad letter must not run a whole slab sequence
        HIP_TRY(hipMemcpyAsync(hm, flags, 16, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        if ((s = check_encoded(hm, sc)) != SW_OK) return s;
        if ((s = run_score_slabs(ctx, a_codes, M, b_codes, N, sc, o, h, S, rows, eng,
                                 ws_bytes - (size_t)(eng - (uint8_t*)ws), so)) != SW_OK)
            return s;
    } else {
        const EnginePlan p = plan_engine(ctx, score_specs(0, M, N, o, S), true, o ? o->rows_per_lane : 0,
                                         o ? o->waves_per_cu : 0, o ? o->band_width : 0);
        if ((s = run_engine(ctx, p, a_codes, b_codes, sc, eng, nullptr, nullptr)) != SW_OK) return s;
        HIP_TRY(hipMemcpyAsync(hm, flags, 16, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipMemcpyAsync(hm + 64, eng + p.off_outs, (size_t)S * sizeof(ScoreOut), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        if ((s = check_encoded(hm, sc)) != SW_OK) return s;
        for (int i = 0; i < S; ++i) std::memcpy(&so[p.order[(size_t)i]], hm + 64 + i * sizeof(ScoreOut), sizeof(ScoreOut));
        for (int i = 0; i < S; ++i)
            if (so[i].status) return fail(SW_EINTERNAL, "score pass: %s", engine_status_text(so[i].status));
        report_progress(o, M, M);
    }
    // the better strand; the forward one on a tie
    const int w = (S == 2 && so[1].score > so[0].score) ? 1 : 0;
    std::memset(out, 0, sizeof *out);
    out->score = so[w].score;
    out->end_a = so[w].end_a;
    out->end_b = so[w].end_b;
    out->strand = w;
    out->threshold = (o && o->prune_mode == SW_PRUNE_LEARNED) ? o->threshold : 0;
    const unsigned long long total = (unsigned long long)M * (unsigned long long)N * (unsigned long long)S;
    unsigned long long pruned = 0;
    for (int i = 0; i < S; ++i) pruned += so[i].pruned_cells;
    out->cells_computed = (int64_t)(pruned >= total ? 0 : total - pruned);
    return SW_OK;
}

// LEARNED mode: T from the model (or the caller), one pass that skips tiles below
// max(running best, T); if the best found is below T the result is not known to
// be optimal and the pass reruns.  The missed pass still reports the largest H it
// computed, a lower bound S' <= S (pruned borders are lower bounds and the
// recurrence is monotone), so the rerun takes S' as its threshold: exact, and it
// cannot miss.  With S' = 0 the rerun uses the running best alone.
sw_status swmi::run_score(sw_context* ctx, const uint8_t* d_a, int64_t M, const uint8_t* d_b, int64_t N,
                          const sw_scoring* sc, const sw_options* o, void* ws, size_t ws_bytes,
                          sw_score_result* out) {
    if (o && (o->flags & SW_FLAG_HALVES)) return run_score_halves(ctx, d_a, M, d_b, N, sc, o, ws, ws_bytes, out);
    if (!o || o->prune_mode != SW_PRUNE_LEARNED) return run_score_once(ctx, d_a, M, d_b, N, sc, o, ws, ws_bytes, out);
    sw_options ol = *o;
    if (ol.threshold == 0) {
        if (!ol.model) return fail(SW_EINVAL, "SW_PRUNE_LEARNED needs a model or a threshold");
        const int64_t oa[2] = {0, M}, ob[2] = {0, N};
        std::vector<int32_t> T;
        sw_status st = predict_thresholds(ctx, ol.model, d_a, oa, d_b, ob, 1, ws, ws_bytes, T);
        if (st != SW_OK) return st;
        ol.threshold = T[0];
    }
    sw_status st = run_score_once(ctx, d_a, M, d_b, N, sc, &ol, ws, ws_bytes, out);
    if (st != SW_OK) return st;
    out->threshold = ol.threshold;
    if (out->score < ol.threshold) {
        const int64_t first = out->cells_computed;
        const int32_t seen = out->score;
        sw_options ob = ol;
        ob.model = nullptr;
        ob.prune_mode = seen > 0 ? SW_PRUNE_LEARNED : SW_PRUNE_BEST;
        ob.threshold = seen > 0 ? seen : 0;
        if ((st = run_score_once(ctx, d_a, M, d_b, N, sc, &ob, ws, ws_bytes, out)) != SW_OK) return st;
        if (out->score < ob.threshold)
            return fail(SW_EINTERNAL, "learned fallback: rerun below the seen lower bound %d", seen);
        out->threshold = ol.threshold;
        out->fallback = 1;
        out->cells_computed += first;
    }
    return SW_OK;
}

// ------------------------------------------------------------------------ C ABI: score

extern "C" size_t sw_score_workspace_size(sw_context* ctx, int64_t len_a, int64_t len_b, const sw_options* o) {
    if (!ctx || len_a < 0 || len_b < 0) return 0;
    return score_workspace_size(ctx, len_a, len_b, o);
}

extern "C" sw_status sw_score_dev(sw_context* ctx, const uint8_t* d_a, int64_t len_a, const uint8_t* d_b,
                                  int64_t len_b, const sw_scoring* scoring, const sw_options* options,
                                  void* d_workspace, size_t workspace_bytes, sw_score_result* out) {
    if (!ctx || !out) return fail(SW_EINVAL, "sw_score_dev: NULL context or result");
    sw_status st;
    sw_scoring sc;
    if ((st = check_scoring(scoring, &sc)) != SW_OK) return st;
    if ((st = check_lengths(len_a, len_b, &sc)) != SW_OK) return st;
    if ((st = check_options(options)) != SW_OK) return st;
    if ((st = check_matrix_options(&sc, options)) != SW_OK) return st;
    if ((len_a && !d_a) || (len_b && !d_b)) return fail(SW_EINVAL, "sw_score_dev: NULL sequence pointer");
    if (len_a == 0 || len_b == 0) {
        std::memset(out, 0, sizeof *out);
        out->end_a = out->end_b = -1;
        return SW_OK;
    }
    if (!d_workspace) return fail(SW_EINVAL, "sw_score_dev: NULL workspace");
    HIP_TRY(hipSetDevice(ctx->device));
    return run_score(ctx, d_a, len_a, d_b, len_b, &sc, options, d_workspace, workspace_bytes, out);
}

extern "C" sw_status sw_score_dev_noalloc(sw_context* ctx, const uint8_t* d_a, int64_t len_a, const uint8_t* d_b,
                                          int64_t len_b, const sw_scoring* scoring, const sw_options* options,
                                          sw_score_result* out) {
    if (!ctx || !out) return fail(SW_EINVAL, "sw_score_dev_noalloc: NULL context or result");
    sw_status st;
    sw_scoring sc;
    if ((st = check_scoring(scoring, &sc)) != SW_OK) return st;
    if ((st = check_lengths(len_a, len_b, &sc)) != SW_OK) return st;
    if ((st = check_options(options)) != SW_OK) return st;
    if ((st = check_matrix_options(&sc, options)) != SW_OK) return st;
    if ((len_a && !d_a) || (len_b && !d_b)) return fail(SW_EINVAL, "sw_score_dev_noalloc: NULL sequence pointer");
    if (len_a == 0 || len_b == 0) {
        std::memset(out, 0, sizeof *out);
        out->end_a = out->end_b = -1;
        return SW_OK;
    }
    const size_t need = score_workspace_size(ctx, len_a, len_b, options);
    if (need > (size_t)SW_NOALLOC_SCRATCH_BYTES)
        return fail(SW_ENOMEM, "sw_score_dev_noalloc: the pair needs %zu bytes of workspace, the fixed scratch "
                    "holds %zu (use sw_score_dev with a caller workspace)", need, (size_t)SW_NOALLOC_SCRATCH_BYTES);
    HIP_TRY(hipSetDevice(ctx->device));
    // Every intermediate the pass reads before writing (encode flags, counters,
    // running bests, records) is cleared by kernels inside run_score.
    return run_score(ctx, d_a, len_a, d_b, len_b, &sc, options, ctx->scratch, SW_NOALLOC_SCRATCH_BYTES, out);
}

// Uploads host letters into the context's input buffer (checked on the device).
sw_status swmi::upload_pair(sw_context* ctx, const char* a, int64_t la, const char* b, int64_t lb,
                            uint8_t** d_a, uint8_t** d_b) {
    void* buf;
    sw_status st = ctx_buffer(ctx, BUF_INPUT, align_up((size_t)la + 1, 256) + (size_t)lb + 256, &buf);
    if (st != SW_OK) return st;
    *d_a = (uint8_t*)buf;
    *d_b = (uint8_t*)buf + align_up((size_t)la + 1, 256);
    if (la) HIP_TRY(hipMemcpyAsync(*d_a, a, (size_t)la, hipMemcpyHostToDevice, ctx->stream));
    if (lb) HIP_TRY(hipMemcpyAsync(*d_b, b, (size_t)lb, hipMemcpyHostToDevice, ctx->stream));
    return SW_OK;
}

extern "C" sw_status sw_score(sw_context* ctx, const char* a, int64_t len_a, const char* b, int64_t len_b,
                              const sw_scoring* scoring, const sw_options* options, sw_score_result* out) {
    if (!ctx || !out) return fail(SW_EINVAL, "sw_score: NULL context or result");
    sw_status st;
    sw_scoring sc;
    if ((st = check_scoring(scoring, &sc)) != SW_OK) return st;
    if ((st = check_lengths(len_a, len_b, &sc)) != SW_OK) return st;
    if ((st = check_options(options)) != SW_OK) return st;
    if ((st = check_matrix_options(&sc, options)) != SW_OK) return st;
    if ((len_a && !a) || (len_b && !b)) return fail(SW_EINVAL, "sw_score: NULL sequence pointer");
    if (len_a == 0 || len_b == 0) {
        std::memset(out, 0, sizeof *out);
        out->end_a = out->end_b = -1;
        return SW_OK;
    }
    HIP_TRY(hipSetDevice(ctx->device));
    uint8_t *d_a, *d_b;
    if ((st = upload_pair(ctx, a, len_a, b, len_b, &d_a, &d_b)) != SW_OK) return st;
    const size_t need = score_workspace_size(ctx, len_a, len_b, options);
    void* ws;
    if ((st = ctx_buffer(ctx, BUF_WORK, need, &ws)) != SW_OK) return st;
    return run_score(ctx, d_a, len_a, d_b, len_b, &sc, options, ws, need, out);
}
