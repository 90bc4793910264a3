// Many independent pairs in one persistent launch of the wavefront engine.
//
// Every pair is a local problem of the engine's table; problems are ordered
// largest first and share the launch's resident waves through the ticket
// counter (a small pair is one or a few stripe tasks, a large one many), so
// uneven lengths balance without per-pair launches.  Results come back per
// pair: score and endpoint under the same tie rule as sw_score.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <memory>
#include <new>
#include <vector>

#include "swmi.h"
#include "swmi_host.h"
#include "swmi_internal.h"

using namespace swmi;

#define HIP_TRY(expr)                                                                           \
    do {                                                                                        \
        hipError_t e_ = (expr);                                                                 \
        if (e_ != hipSuccess) return fail(SW_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

namespace {

struct BatchLayout {
    std::vector<ProbSpec> specs;
    std::vector<int32_t> pair_of_spec;       // spec index -> pair index
    std::vector<int64_t> a_src, a_dst, a_len;  // encode tables
    std::vector<int64_t> b_src, b_dst, b_len;
    int64_t a_bytes = 0, b_bytes = 0;
    size_t off_a = 0, off_b = 0, off_tab = 0, off_flags = 0, off_eng = 0, total = 0;
    EnginePlan plan;
};

// Pairs given as (start, length) into the packed device letters; T: per-pair
// thresholds (LEARNED mode) or null.
sw_status make_layout(sw_context* ctx, const std::vector<int64_t>& as, const std::vector<int64_t>& al,
                      const std::vector<int64_t>& bs, const std::vector<int64_t>& bl, const sw_scoring* sc,
                      const sw_options* o, const std::vector<int32_t>* T, BatchLayout& L) {
    const int32_t n = (int32_t)as.size();
    int64_t apos = 0, bpos = 0;
    for (int32_t p = 0; p < n; ++p) {
        const int64_t la = al[(size_t)p], lb = bl[(size_t)p];
        if (la < 0 || lb < 0) return fail(SW_EINVAL, "sw_batch: offsets of pair %d decrease", p);
        sw_status st = check_lengths(la, lb, sc);
        if (st != SW_OK) return st;
        L.a_src.push_back(as[(size_t)p]);
        L.a_dst.push_back(apos);
        L.a_len.push_back(la);
        L.b_src.push_back(bs[(size_t)p]);
        L.b_dst.push_back(bpos + kBPad);
        L.b_len.push_back(lb);
        if (la > 0 && lb > 0) {
            ProbSpec s;
            s.a_off = apos;
            s.b_off = bpos + kBPad;
            s.M = la;
            s.N = lb;
            s.prune = (o && o->prune_mode != SW_PRUNE_NONE) ? 1 : 0;
            s.target = T ? (*T)[(size_t)p] : ((o && o->prune_mode == SW_PRUNE_LEARNED) ? o->threshold : 0);
            s.track = 1;
            L.specs.push_back(s);
            L.pair_of_spec.push_back(p);
        }
        apos += la;
        bpos += kBPad + lb + kBPadTail;
    }
    L.a_bytes = apos;
    L.b_bytes = bpos;
    L.plan = plan_engine(ctx, L.specs, true, o ? o->rows_per_lane : 0, o ? o->waves_per_cu : 0,
                         o ? o->band_width : 0);
    size_t off = 0;
    L.off_a = off;
    off = align_up(off + (size_t)L.a_bytes + 64, 256);
    L.off_b = off;
    off = align_up(off + (size_t)L.b_bytes + 128, 256);
    L.off_tab = off;
    off = align_up(off + (size_t)n * 6 * sizeof(int64_t), 256);
    L.off_flags = off;
    off = align_up(off + 256, 256);
    L.off_eng = off;
    off += L.plan.total;
    L.total = off;
    return SW_OK;
}

uint64_t mix(uint64_t h, uint64_t v) {
    h ^= v + 0x9e3779b97f4a7c15ull + (h << 6) + (h >> 2);
    return h;
}

// Device work of one batch (capturable): pads, encodes, engine, reduction.
sw_status batch_device_work(sw_context* ctx, const uint8_t* d_a, const uint8_t* d_b, int32_t n, const sw_scoring* sc,
                            BatchLayout& L, uint8_t* base) {
    hipStream_t s = ctx->stream;
    int64_t* tab = (int64_t*)(base + L.off_tab);
    unsigned long long* bad = (unsigned long long*)(base + L.off_flags);
    const EncTable et = enc_table(sc);
    const int32_t pad4 = (int32_t)(0x01010101u * (uint32_t)et.pad_code);  // padding code in every byte
    HIP_TRY(launch_zero(base + L.off_flags, 256, s));
    HIP_TRY(launch_fill_i32((int32_t*)(base + L.off_b), pad4, (size_t)(L.b_bytes + 64 + 3) / 4, s));
    HIP_TRY(launch_encode_many(d_a, tab, tab + n, tab + 2 * (size_t)n, n, base + L.off_a, et, bad, s));
    HIP_TRY(launch_encode_many(d_b, tab + 3 * (size_t)n, tab + 4 * (size_t)n, tab + 5 * (size_t)n, n,
                               base + L.off_b, et, bad + 1, s));
    return launch_engine_kernels(ctx, L.plan, base + L.off_a, base + L.off_b, sc, base + L.off_eng, nullptr, nullptr);
}

// Host copy of the encode table: source offset, destination, length per pair, for a then b.
void fill_tab(const BatchLayout& L, int32_t n, int64_t* h) {
    std::copy(L.a_src.begin(), L.a_src.end(), h);
    std::copy(L.a_dst.begin(), L.a_dst.end(), h + n);
    std::copy(L.a_len.begin(), L.a_len.end(), h + 2 * (size_t)n);
    std::copy(L.b_src.begin(), L.b_src.end(), h + 3 * (size_t)n);
    std::copy(L.b_dst.begin(), L.b_dst.end(), h + 4 * (size_t)n);
    std::copy(L.b_len.begin(), L.b_len.end(), h + 5 * (size_t)n);
}

void clear_out(sw_score_result* out, int32_t n) {
    for (int32_t p = 0; p < n; ++p) {
        std::memset(&out[p], 0, sizeof out[p]);
        out[p].end_a = out[p].end_b = -1;
    }
}

// Per-pair results from the launch's bad-letter flags and per-problem outputs.
sw_status collect(const BatchLayout& L, const unsigned long long* flags, const ScoreOut* so, const sw_scoring* sc,
                  sw_score_result* out) {
    if (flags[0]) return fail(SW_EINVAL, "seqs_a: byte at offset %llu is not %s", kBadBase - flags[0], letters_text(sc));
    if (flags[1]) return fail(SW_EINVAL, "seqs_b: byte at offset %llu is not %s", kBadBase - flags[1], letters_text(sc));
    for (size_t k = 0; k < (size_t)L.plan.n_probs; ++k) {
        const size_t spec = (size_t)L.plan.order[k];
        const int32_t p = L.pair_of_spec[spec];
        if (so[k].status) return fail(SW_EINTERNAL, "batch, pair %d: %s", p, engine_status_text(so[k].status));
        sw_score_result& r = out[p];
        r.score = so[k].score;
        r.end_a = so[k].end_a;
        r.end_b = so[k].end_b;
        const unsigned long long cells = (unsigned long long)L.specs[spec].M * (unsigned long long)L.specs[spec].N;
        r.cells_computed = (int64_t)(so[k].pruned_cells >= cells ? 0 : cells - so[k].pruned_cells);
        r.threshold = L.specs[spec].target;
    }
    return SW_OK;
}

sw_status run_batch(sw_context* ctx, const uint8_t* d_a, const uint8_t* d_b, int32_t n, const sw_scoring* sc,
                    BatchLayout& L, void* ws, size_t ws_bytes, sw_score_result* out) {
    const Phase ph("swmi batch launch");
    if (ws_bytes < L.total) return fail(SW_ENOMEM, "workspace of %zu bytes, need %zu", ws_bytes, L.total);
    clear_out(out, n);
    if (L.specs.empty()) return SW_OK;
    uint8_t* base = (uint8_t*)ws;
    hipStream_t s = ctx->stream;
    std::vector<int64_t> h_tab((size_t)n * 6);
    fill_tab(L, n, h_tab.data());
    HIP_TRY(hipMemcpyAsync(base + L.off_tab, h_tab.data(), h_tab.size() * sizeof(int64_t), hipMemcpyHostToDevice, s));
    sw_status st = upload_engine_table(ctx, L.plan, base + L.off_eng);
    if (st != SW_OK) return st;
    if ((st = batch_device_work(ctx, d_a, d_b, n, sc, L, base)) != SW_OK) return st;
    std::vector<ScoreOut> so((size_t)L.plan.n_probs);
    unsigned long long flags[2];
    HIP_TRY(hipMemcpyAsync(flags, base + L.off_flags, sizeof flags, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(so.data(), base + L.off_eng + L.plan.off_outs, so.size() * sizeof(ScoreOut),
                           hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return collect(L, flags, so.data(), sc, out);
}

// A captured batch: the graph copies the tables from pinned host memory owned
// here, then runs the device work.  A later call whose inputs hash to the same
// key replays it without planning.
struct BatchGraph {
    uint64_t key = 0;
    hipGraphExec_t exec = nullptr;
    BatchLayout L;
    void* pinned = nullptr;  // tables | results (flags, per-problem outputs)
    size_t off_probs = 0, off_tickets = 0, off_flags = 0, off_outs = 0;
};

void destroy(BatchGraph* g) {
    if (!g) return;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->pinned) (void)hipHostFree(g->pinned);
    delete g;
}

// Everything a batch launch depends on: pointers, workspace, pairs, options,
// scoring, the context's tuning and the per-pair thresholds.
uint64_t inputs_key(const sw_context* ctx, const uint8_t* d_a, const uint8_t* d_b, void* ws, size_t ws_bytes,
                    const std::vector<int64_t>& as, const std::vector<int64_t>& al, const std::vector<int64_t>& bs,
                    const std::vector<int64_t>& bl, const sw_scoring* sc, const sw_options* o,
                    const std::vector<int32_t>& T) {
    uint64_t key = 0x51ed270b7f4a7c15ull;
    for (uint64_t v : {(uint64_t)(uintptr_t)d_a, (uint64_t)(uintptr_t)d_b, (uint64_t)(uintptr_t)ws, (uint64_t)ws_bytes,
                       (uint64_t)as.size(), (uint64_t)sc->match, (uint64_t)sc->mismatch, (uint64_t)sc->gap_open,
                       (uint64_t)sc->gap_extend, (uint64_t)o->prune_mode, (uint64_t)(uint32_t)o->threshold,
                       (uint64_t)(uintptr_t)o->model, (uint64_t)o->rows_per_lane, (uint64_t)o->waves_per_cu,
                       (uint64_t)o->band_width, (uint64_t)o->flags})
        key = mix(key, v);
    for (int c = 0; c < 4; ++c)
        key = mix(mix(mix(key, (uint64_t)ctx->tuned_R[c]), (uint64_t)ctx->tuned_wpc[c]), (uint64_t)ctx->tuned_bw[c]);
    if (sc->matrix) {  // the matrix content (a replay bakes its table into the launch)
        const sw_matrix* m = sc->matrix;
        key = mix(key, (uint64_t)m->size);
        for (int i = 0; i < m->size; ++i) key = mix(key, (uint64_t)(uint8_t)m->alphabet[i]);
        for (int i = 0; i < m->size * m->size; ++i) key = mix(key, (uint64_t)(uint8_t)m->scores[i]);
    }
    for (size_t i = 0; i < as.size(); ++i)
        key = mix(mix(mix(mix(key, (uint64_t)as[i]), (uint64_t)al[i]), (uint64_t)bs[i]), (uint64_t)bl[i]);
    for (int32_t t : T) key = mix(key, (uint64_t)(uint32_t)t);
    return key;
}

sw_status run_batch_graph(sw_context* ctx, const uint8_t* d_a, const uint8_t* d_b, const std::vector<int64_t>& as,
                          const std::vector<int64_t>& al, const std::vector<int64_t>& bs,
                          const std::vector<int64_t>& bl, const sw_scoring* sc, const sw_options* o,
                          const std::vector<int32_t>& T, void* ws, size_t ws_bytes, sw_score_result* out) {
    hipStream_t s = ctx->stream;
    if (!s) return fail(SW_EINVAL, "SW_FLAG_GRAPH needs a context bound to a non-null stream");
    const int32_t n = (int32_t)as.size();
    const uint64_t key = inputs_key(ctx, d_a, d_b, ws, ws_bytes, as, al, bs, bl, sc, o, T);
    BatchGraph* g = (BatchGraph*)ctx->batch_graph;
    if (!g || g->key != key) {
        destroy(g);
        ctx->batch_graph = nullptr;
        g = new (std::nothrow) BatchGraph();
        if (!g) return fail(SW_ENOMEM, "batch graph: out of host memory");
        std::unique_ptr<BatchGraph, void (*)(BatchGraph*)> hold(g, destroy);
        sw_status st = make_layout(ctx, as, al, bs, bl, sc, o, T.empty() ? nullptr : &T, g->L);
        if (st != SW_OK) return st;
        const BatchLayout& L = g->L;
        if (ws_bytes < L.total) return fail(SW_ENOMEM, "workspace of %zu bytes, need %zu", ws_bytes, L.total);
        const size_t tab_bytes = align_up((size_t)n * 6 * sizeof(int64_t), 256);
        g->off_probs = tab_bytes;
        g->off_tickets = g->off_probs + align_up((size_t)L.plan.n_probs * sizeof(Prob), 256);
        g->off_flags = g->off_tickets + align_up((size_t)L.plan.n_tickets * sizeof(Ticket), 256);
        g->off_outs = g->off_flags + 256;
        const size_t bytes = g->off_outs + (size_t)L.plan.n_probs * sizeof(ScoreOut) + 256;
        HIP_TRY(hipHostMalloc(&g->pinned, bytes, hipHostMallocDefault));
        uint8_t* hp = (uint8_t*)g->pinned;
        fill_tab(L, n, (int64_t*)hp);
        std::memcpy(hp + g->off_probs, L.plan.probs.data(), (size_t)L.plan.n_probs * sizeof(Prob));
        std::memcpy(hp + g->off_tickets, L.plan.tickets.data(), (size_t)L.plan.n_tickets * sizeof(Ticket));
        if (!L.specs.empty()) {
            uint8_t* base = (uint8_t*)ws;
            uint8_t* eng = base + L.off_eng;
            hipGraph_t graph = nullptr;
            HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
            hipError_t e = hipMemcpyAsync(base + L.off_tab, hp, (size_t)n * 6 * sizeof(int64_t),
                                          hipMemcpyHostToDevice, s);
            if (e == hipSuccess)
                e = hipMemcpyAsync(eng + L.plan.off_probs, hp + g->off_probs, (size_t)L.plan.n_probs * sizeof(Prob),
                                   hipMemcpyHostToDevice, s);
            if (e == hipSuccess)
                e = hipMemcpyAsync(eng + L.plan.off_tickets, hp + g->off_tickets,
                                   (size_t)L.plan.n_tickets * sizeof(Ticket), hipMemcpyHostToDevice, s);
            st = e == hipSuccess ? batch_device_work(ctx, d_a, d_b, n, sc, g->L, base)
                                 : fail(SW_EDEVICE, "batch graph: table copy: %s", hipGetErrorString(e));
            e = hipStreamEndCapture(s, &graph);
            if (st != SW_OK) {
                if (graph) (void)hipGraphDestroy(graph);
                return st;
            }
            if (e != hipSuccess) return fail(SW_EDEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e));
            e = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (e != hipSuccess) {
                g->exec = nullptr;
                return fail(SW_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
            }
        }
        g->key = key;
        ctx->batch_graph = hold.release();
    }
    const BatchLayout& L = g->L;
    clear_out(out, n);
    if (L.specs.empty()) return SW_OK;
    uint8_t* base = (uint8_t*)ws;
    uint8_t* hp = (uint8_t*)g->pinned;
    HIP_TRY(hipGraphLaunch(g->exec, s));
    HIP_TRY(hipMemcpyAsync(hp + g->off_flags, base + L.off_flags, 16, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(hp + g->off_outs, base + L.off_eng + L.plan.off_outs,
                           (size_t)L.plan.n_probs * sizeof(ScoreOut), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return collect(L, (const unsigned long long*)(hp + g->off_flags), (const ScoreOut*)(hp + g->off_outs), sc, out);
}

}  // namespace

void swmi::free_batch_graph(void* g) { destroy((BatchGraph*)g); }

static sw_status pairs_of(const int64_t* offs_a, const int64_t* offs_b, int32_t n, std::vector<int64_t>& as,
                          std::vector<int64_t>& al, std::vector<int64_t>& bs, std::vector<int64_t>& bl) {
    if (n < 0) return fail(SW_EINVAL, "sw_batch: n_pairs < 0");
    if (n > 0 && (!offs_a || !offs_b)) return fail(SW_EINVAL, "sw_batch: NULL offsets");
    for (int32_t p = 0; p < n; ++p) {
        as.push_back(offs_a[p]);
        al.push_back(offs_a[p + 1] - offs_a[p]);
        bs.push_back(offs_b[p]);
        bl.push_back(offs_b[p + 1] - offs_b[p]);
    }
    return SW_OK;
}

static bool batch_uses_model(const sw_options* o) {
    return o && o->prune_mode == SW_PRUNE_LEARNED && o->threshold == 0 && !o->pair_thresholds;
}

extern "C" size_t sw_batch_workspace_size(sw_context* ctx, const int64_t* offs_a, const int64_t* offs_b,
                                          int32_t n_pairs, const sw_scoring* scoring, const sw_options* options) {
    if (!ctx || !scoring) return 0;
    sw_scoring sc;
    if (check_scoring(scoring, &sc) != SW_OK) return 0;
    std::vector<int64_t> as, al, bs, bl;
    if (pairs_of(offs_a, offs_b, n_pairs, as, al, bs, bl) != SW_OK) return 0;
    BatchLayout L;
    if (make_layout(ctx, as, al, bs, bl, &sc, options, nullptr, L) != SW_OK) return 0;
    size_t total = L.total;
    if (batch_uses_model(options)) {
        int64_t mM = 0, mN = 0;
        for (size_t k = 0; k < al.size(); ++k) {
            mM = std::max(mM, al[k]);
            mN = std::max(mN, bl[k]);
        }
        total = std::max(total, predict_workspace_size(mM, mN, n_pairs));
    }
    return total;
}

// Batched pass; in LEARNED mode with a model: thresholds first, then one pass,
// then the pairs whose best fell below their threshold again, each with the
// largest H its missed pass computed as threshold (a lower bound of its optimum:
// exact, cannot miss), flagged as fallbacks.
static sw_status batch_all(sw_context* ctx, const uint8_t* d_a, const uint8_t* d_b, const std::vector<int64_t>& as,
                           const std::vector<int64_t>& al, const std::vector<int64_t>& bs,
                           const std::vector<int64_t>& bl, const sw_scoring* sc, const sw_options* o, void* ws,
                           size_t ws_bytes, sw_score_result* out) {
    const int32_t n = (int32_t)as.size();
    std::vector<int32_t> T;
    if (o && o->prune_mode == SW_PRUNE_LEARNED && o->pair_thresholds) {
        T.assign(o->pair_thresholds, o->pair_thresholds + n);
        for (int32_t p = 0; p < n; ++p)
            if (T[(size_t)p] < 0) return fail(SW_EINVAL, "pair_thresholds[%d] is negative", p);
    } else if (batch_uses_model(o)) {
        if (!o->model) return fail(SW_EINVAL, "SW_PRUNE_LEARNED needs a model or a threshold");
        std::vector<int64_t> oa((size_t)n + 1), ob((size_t)n + 1);
        // predict_thresholds takes offsets of consecutive pairs: pass per-pair starts via
        // a one-pair call each when pairs are not contiguous
        bool contiguous = true;
        for (int32_t p = 0; p + 1 < n; ++p)
            if (as[(size_t)p] + al[(size_t)p] != as[(size_t)p + 1] || bs[(size_t)p] + bl[(size_t)p] != bs[(size_t)p + 1])
                contiguous = false;
        if (contiguous && n > 0) {
            for (int32_t p = 0; p < n; ++p) {
                oa[(size_t)p] = as[(size_t)p];
                ob[(size_t)p] = bs[(size_t)p];
            }
            oa[(size_t)n] = as[(size_t)n - 1] + al[(size_t)n - 1];
            ob[(size_t)n] = bs[(size_t)n - 1] + bl[(size_t)n - 1];
            sw_status st = predict_thresholds(ctx, o->model, d_a, oa.data(), d_b, ob.data(), n, ws, ws_bytes, T);
            if (st != SW_OK) return st;
        } else {
            T.assign((size_t)n, 0);
            for (int32_t p = 0; p < n; ++p) {
                const int64_t a2[2] = {as[(size_t)p], as[(size_t)p] + al[(size_t)p]};
                const int64_t b2[2] = {bs[(size_t)p], bs[(size_t)p] + bl[(size_t)p]};
                std::vector<int32_t> t1;
                sw_status st = predict_thresholds(ctx, o->model, d_a, a2, d_b, b2, 1, ws, ws_bytes, t1);
                if (st != SW_OK) return st;
                T[(size_t)p] = t1[0];
            }
        }
    }
    sw_status st;
    if (o && (o->flags & SW_FLAG_GRAPH)) {
        if ((st = run_batch_graph(ctx, d_a, d_b, as, al, bs, bl, sc, o, T, ws, ws_bytes, out)) != SW_OK) return st;
    } else {
        BatchLayout L;
        if ((st = make_layout(ctx, as, al, bs, bl, sc, o, T.empty() ? nullptr : &T, L)) != SW_OK) return st;
        if ((st = run_batch(ctx, d_a, d_b, n, sc, L, ws, ws_bytes, out)) != SW_OK) return st;
    }
    if (!o || o->prune_mode != SW_PRUNE_LEARNED) return SW_OK;
    std::vector<int64_t> as2, al2, bs2, bl2;
    std::vector<int32_t> idx, T2;
    for (int32_t p = 0; p < n; ++p) {
        const int32_t t = T.empty() ? o->threshold : T[(size_t)p];
        out[p].threshold = t;
        if (out[p].score < t && al[(size_t)p] > 0 && bl[(size_t)p] > 0) {
            idx.push_back(p);
            as2.push_back(as[(size_t)p]);
            al2.push_back(al[(size_t)p]);
            bs2.push_back(bs[(size_t)p]);
            bl2.push_back(bl[(size_t)p]);
            T2.push_back(out[p].score);  // largest H seen by the missed pass
        }
    }
    if (idx.empty()) return SW_OK;
    sw_options ob2 = *o;
    ob2.model = nullptr;
    ob2.prune_mode = SW_PRUNE_LEARNED;
    ob2.threshold = 0;
    BatchLayout L2;
    if ((st = make_layout(ctx, as2, al2, bs2, bl2, sc, &ob2, &T2, L2)) != SW_OK) return st;
    if (L2.total > ws_bytes) return fail(SW_ENOMEM, "batch fallback: workspace too small");
    std::vector<sw_score_result> r2(idx.size());
    if ((st = run_batch(ctx, d_a, d_b, (int32_t)idx.size(), sc, L2, ws, ws_bytes, r2.data())) != SW_OK)
        return st;
    for (size_t k = 0; k < idx.size(); ++k) {
        if (r2[k].score < T2[k])
            return fail(SW_EINTERNAL, "learned fallback: pair %d below the seen lower bound", idx[k]);
        sw_score_result& r = out[idx[k]];
        const int64_t first = r.cells_computed;
        const int32_t t = r.threshold;
        r = r2[k];
        r.cells_computed += first;
        r.threshold = t;
        r.fallback = 1;
    }
    return SW_OK;
}

extern "C" sw_status sw_batch_dev(sw_context* ctx, const uint8_t* d_seqs_a, const int64_t* offs_a,
                                  const uint8_t* d_seqs_b, const int64_t* offs_b, int32_t n_pairs,
                                  const sw_scoring* scoring, const sw_options* options, void* d_workspace,
                                  size_t workspace_bytes, sw_score_result* out) {
    if (!ctx || (n_pairs > 0 && !out)) return fail(SW_EINVAL, "sw_batch_dev: NULL context or results");
    sw_status st;
    sw_scoring sc;
    if ((st = check_scoring(scoring, &sc)) != SW_OK) return st;
    if ((st = check_options(options)) != SW_OK) return st;
    if ((st = check_matrix_options(&sc, options)) != SW_OK) return st;
    if (options && (options->flags & (SW_FLAG_HALVES | SW_FLAG_BOTH_STRANDS)))
        return fail(SW_EUNSUPPORTED, "sw_batch: SW_FLAG_HALVES and SW_FLAG_BOTH_STRANDS are single-pair options");
    std::vector<int64_t> as, al, bs, bl;
    if ((st = pairs_of(offs_a, offs_b, n_pairs, as, al, bs, bl)) != SW_OK) return st;
    if (n_pairs > 0 && (!d_seqs_a || !d_seqs_b)) return fail(SW_EINVAL, "sw_batch_dev: NULL sequences");
    if (n_pairs > 0 && !d_workspace) return fail(SW_EINVAL, "sw_batch_dev: NULL workspace");
    HIP_TRY(hipSetDevice(ctx->device));
    return batch_all(ctx, d_seqs_a, d_seqs_b, as, al, bs, bl, &sc, options, d_workspace, workspace_bytes, out);
}

extern "C" sw_status sw_batch(sw_context* ctx, const char* seqs_a, const int64_t* offs_a, const char* seqs_b,
                              const int64_t* offs_b, int32_t n_pairs, const sw_scoring* scoring,
                              const sw_options* options, sw_score_result* out) {
    if (!ctx || (n_pairs > 0 && !out)) return fail(SW_EINVAL, "sw_batch: NULL context or results");
    sw_status st;
    sw_scoring sc;
    if ((st = check_scoring(scoring, &sc)) != SW_OK) return st;
    if ((st = check_options(options)) != SW_OK) return st;
    if ((st = check_matrix_options(&sc, options)) != SW_OK) return st;
    if (options && (options->flags & (SW_FLAG_HALVES | SW_FLAG_BOTH_STRANDS)))
        return fail(SW_EUNSUPPORTED, "sw_batch: SW_FLAG_HALVES and SW_FLAG_BOTH_STRANDS are single-pair options");
    std::vector<int64_t> as, al, bs, bl;
    if ((st = pairs_of(offs_a, offs_b, n_pairs, as, al, bs, bl)) != SW_OK) return st;
    if (n_pairs == 0) return SW_OK;
    const int64_t na = offs_a[n_pairs] - offs_a[0], nb = offs_b[n_pairs] - offs_b[0];
    if ((na && !seqs_a) || (nb && !seqs_b)) return fail(SW_EINVAL, "sw_batch: NULL sequences");
    if (na < 0 || nb < 0) return fail(SW_EINVAL, "sw_batch: offsets decrease");
    HIP_TRY(hipSetDevice(ctx->device));
    void* in;
    if ((st = ctx_buffer(ctx, BUF_INPUT, align_up((size_t)na + 1, 256) + (size_t)nb + 256, &in)) != SW_OK)
        return st;
    uint8_t* d_a = (uint8_t*)in;
    uint8_t* d_b = d_a + align_up((size_t)na + 1, 256);
    if (na) HIP_TRY(hipMemcpyAsync(d_a, seqs_a + offs_a[0], (size_t)na, hipMemcpyHostToDevice, ctx->stream));
    if (nb) HIP_TRY(hipMemcpyAsync(d_b, seqs_b + offs_b[0], (size_t)nb, hipMemcpyHostToDevice, ctx->stream));
    for (auto& v : as) v -= offs_a[0];
    for (auto& v : bs) v -= offs_b[0];
    const size_t need = sw_batch_workspace_size(ctx, offs_a, offs_b, n_pairs, scoring, options);
    if (!need) return fail(SW_EINTERNAL, "sw_batch: workspace size");
    void* ws;
    if ((st = ctx_buffer(ctx, BUF_WORK, need, &ws)) != SW_OK) return st;
    return batch_all(ctx, d_a, d_b, as, al, bs, bl, &sc, options, ws, need, out);
}
