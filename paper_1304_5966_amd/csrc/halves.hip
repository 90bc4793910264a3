// The two-halves score pass of SW# (paper Section 2, last paragraphs, and
// Figure 1): the split the paper uses to run the first phase on two GPUs, here
// as two problems of one launch on one GPU.
//
//   upper half: rows [0, mid) of A forward, local recurrence; its best score
//               S_up with the first cell holding it, and its last row (H and the
//               deletion-ending F at every vertex of row mid);
//   lower half: rows [mid, M) of A and all of B, both reversed; its best score
//               S_low (where the best local alignment of the lower half starts),
//               and its last row, i.e. the best score of a path that starts at
//               each vertex of row mid and runs down into the lower half.
//
// The midpoint score is Myers and Miller's combination of the two rows: the
// best over columns of a plain crossing (H up + H down) and of a deletion run
// through the midline (F up + F down + open - extend, one opening counted twice).
// The best score is S = max(S_up, S_low, midpoint), and the paper's three
// cases are: (b) the maximum lies in the upper half, (a) in the lower half,
// (c) at the midpoint.
//
// Endpoint (the lexicographically first cell holding S): in case (b) it is the
// upper half's own first cell, since every upper row precedes every lower row.
// Otherwise the alignment ends below the midline; the lower half runs forward
// once more, its row 0 the upper half's last row, with threshold S: only tiles
// that can still reach S are computed (exact, as S is the optimum), and the
// first cell holding S is the endpoint.
//
// Pruning inside the halves is exact as well: a tile's bound counts the rows of
// the other half (a path through it may continue there), so every tile on an
// optimal path -- crossing or not -- is computed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
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

struct HalvesLayout {
    size_t la, lb;    // code bytes of A and of padded B (forward and reversed copies of each)
    size_t codes;     // [fa | fb | rva | rvb]
    size_t flags;     // encode flags (256 bytes)
    size_t rows;      // out_h and out_f: [upper row (N + 1) | lower row (N + 1)] each
    size_t row_bytes;
    size_t task, res; // MidTask, MidResult
    size_t eng, total;
};

ProbSpec upper_spec(int64_t M, int64_t N, int64_t mid, int prune) {
    ProbSpec u;
    u.a_off = 0;
    u.b_off = kBPad;
    u.M = mid;
    u.N = N;
    u.out_off = 0;
    u.rows_after = M - mid;
    u.prune = prune;
    u.track = 1;
    return u;
}

ProbSpec lower_rev_spec(int64_t M, int64_t N, int64_t mid, int prune, const HalvesLayout& L) {
    ProbSpec r;
    r.a_off = (int64_t)(L.la + L.lb);          // reversed A: its first M - mid codes are A[mid..M) reversed
    r.b_off = (int64_t)(L.la + L.lb) + kBPad;  // reversed B
    r.M = M - mid;
    r.N = N;
    r.out_off = N + 1;
    r.rows_after = mid;
    r.prune = prune;
    r.track = 1;
    return r;
}

ProbSpec lower_fwd_spec(int64_t M, int64_t N, int64_t mid, int32_t score) {
    ProbSpec f;
    f.a_off = mid;
    f.b_off = kBPad;
    f.M = M - mid;
    f.N = N;
    f.top_kind = BORDER_BUF;
    f.top_off = 0;
    f.target = score;
    f.prune = 1;
    f.track = 1;
    return f;
}

HalvesLayout layout(const sw_context* ctx, int64_t M, int64_t N, const sw_options* o) {
    HalvesLayout L{};
    L.la = align_up((size_t)M + 64, 256);
    L.lb = align_up((size_t)(kBPad + N + kBPadTail), 256);
    L.codes = 0;
    L.flags = 2 * (L.la + L.lb);
    L.rows = L.flags + 256;
    L.row_bytes = align_up((size_t)(2 * (N + 1)) * sizeof(int32_t), 256);
    L.task = L.rows + 2 * L.row_bytes;
    L.res = L.task + 256;
    L.eng = L.res + 256;
    const int prune = (o && o->prune_mode != SW_PRUNE_NONE) ? 1 : 0;
    const int64_t mid = M / 2;
    const int R = o ? o->rows_per_lane : 0, wpc = o ? o->waves_per_cu : 0, bw = o ? o->band_width : 0;
    const size_t b1 =
        plan_engine(ctx, {upper_spec(M, N, mid, prune), lower_rev_spec(M, N, mid, prune, L)}, true, R, wpc, bw).total;
    const size_t b2 = plan_engine(ctx, {lower_fwd_spec(M, N, mid, 1)}, true, R, wpc, bw).total;
    L.total = L.eng + std::max(b1, b2);
    return L;
}

}  // namespace

size_t swmi::halves_workspace_size(const sw_context* ctx, int64_t M, int64_t N, const sw_options* o) {
    return layout(ctx, M, N, o).total;
}

sw_status swmi::run_score_halves(sw_context* ctx, const uint8_t* d_a, int64_t M, const uint8_t* d_b, int64_t N,
                                 const sw_scoring* sc, const sw_options* o, void* ws, size_t ws_bytes,
                                 sw_score_result* out) {
    if (M < 2) return fail(SW_EUNSUPPORTED, "two-halves score pass: needs at least two rows");
    const Phase ph("swmi two-halves score pass");
    const HalvesLayout L = layout(ctx, M, N, o);
    if (ws_bytes < L.total) return fail(SW_ENOMEM, "workspace of %zu bytes, need %zu", ws_bytes, L.total);
    const int64_t mid = M / 2;
    const int prune = (o && o->prune_mode != SW_PRUNE_NONE) ? 1 : 0;
    const int R = o ? o->rows_per_lane : 0, wpc = o ? o->waves_per_cu : 0, bw = o ? o->band_width : 0;
    uint8_t* base = (uint8_t*)ws;
    uint8_t* fa = base + L.codes;
    uint8_t* fb = fa + L.la;
    uint8_t* rva = fb + L.lb;
    uint8_t* rvb = rva + L.la;
    uint8_t* flags = base + L.flags;
    int32_t* oh = (int32_t*)(base + L.rows);
    int32_t* of = (int32_t*)(base + L.rows + L.row_bytes);
    MidTask* d_task = (MidTask*)(base + L.task);
    MidResult* d_res = (MidResult*)(base + L.res);
    uint8_t* eng = base + L.eng;
    hipStream_t s = ctx->stream;
    const EncTable et = enc_table(sc);
    HIP_TRY(launch_zero(flags, 256, s));
    HIP_TRY(launch_encode(d_a, M, fa, 0, 64, 0, et, (unsigned long long*)flags, s));
    HIP_TRY(launch_encode(d_b, N, fb, kBPad, kBPadTail, 0, et, (unsigned long long*)(flags + 8), s));
    HIP_TRY(launch_encode(d_a, M, rva, 0, 64, ENC_REVERSE, et, (unsigned long long*)flags, s));
    HIP_TRY(launch_encode(d_b, N, rvb, kBPad, kBPadTail, ENC_REVERSE, et, (unsigned long long*)(flags + 8), s));
    HIP_TRY(launch_fill_i32(oh, kNeg, (size_t)(2 * (N + 1)), s));
    HIP_TRY(launch_fill_i32(of, kNeg, (size_t)(2 * (N + 1)), s));

    // Both halves in one launch, then the midline of their last rows.
    const EnginePlan p1 =
        plan_engine(ctx, {upper_spec(M, N, mid, prune), lower_rev_spec(M, N, mid, prune, L)}, true, R, wpc, bw);
    sw_status st = run_engine(ctx, p1, fa, fb, sc, eng, oh, of);
    if (st != SW_OK) return st;
    uint8_t* hm = (uint8_t*)ctx->host_misc;
    const MidTask task{0, N + 1, N};
    std::memcpy(hm + 1024, &task, sizeof task);
    HIP_TRY(hipMemcpyAsync(d_task, hm + 1024, sizeof task, hipMemcpyHostToDevice, s));
    HIP_TRY(launch_midline(d_task, 1, oh, of, sc->gap_open - sc->gap_extend, d_res, s));
    HIP_TRY(hipMemcpyAsync(hm, flags, 16, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(hm + 64, eng + p1.off_outs, 2 * sizeof(ScoreOut), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(hm + 256, d_res, sizeof(MidResult), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    unsigned long long bad_a, bad_b;
    std::memcpy(&bad_a, hm, 8);
    std::memcpy(&bad_b, hm + 8, 8);
    if (bad_a) return fail(SW_EINVAL, "sequence a: byte at offset %llu is not %s", kBadBase - bad_a, letters_text(sc));
    if (bad_b) return fail(SW_EINVAL, "sequence b: byte at offset %llu is not %s", kBadBase - bad_b, letters_text(sc));
    ScoreOut so[2];
    std::memcpy(so, hm + 64, sizeof so);
    MidResult mr;
    std::memcpy(&mr, hm + 256, sizeof mr);
    // plan_engine orders problems by size: probs[k] is spec order[k] (0 upper, 1 lower)
    const ScoreOut& up = so[p1.order[0] == 0 ? 0 : 1];
    const ScoreOut& lo = so[p1.order[0] == 0 ? 1 : 0];
    if (up.status || lo.status)
        return fail(SW_EINTERNAL, "two-halves pass: %s", engine_status_text(up.status ? up.status : lo.status));
    const int64_t S = std::max<int64_t>({(int64_t)up.score, (int64_t)lo.score, mr.value, 0});
    unsigned long long pruned = up.pruned_cells + lo.pruned_cells;
    unsigned long long cells = (unsigned long long)M * (unsigned long long)N;

    std::memset(out, 0, sizeof *out);
    out->end_a = out->end_b = -1;
    if (S == 0) {
        out->split_case = SW_SPLIT_NONE;
    } else if (up.score == S) {
        out->split_case = SW_SPLIT_UPPER;
        out->score = (int32_t)S;
        out->end_a = up.end_a;
        out->end_b = up.end_b;
    } else {
        out->split_case = mr.value == S ? SW_SPLIT_MIDDLE : SW_SPLIT_LOWER;
        // the endpoint lies below the midline: the lower half forward from the upper half's
        // last row, computing only tiles that can still reach S
        const EnginePlan p2 = plan_engine(ctx, {lower_fwd_spec(M, N, mid, (int32_t)S)}, true, R, wpc, bw);
        if ((st = run_engine(ctx, p2, fa, fb, sc, eng, nullptr, nullptr, oh, of)) != SW_OK) return st;
        ScoreOut* e;
        if ((st = read_back(ctx, eng + p2.off_outs, sizeof(ScoreOut), (void**)&e)) != SW_OK) return st;
        if (e->status || e->score != S || e->end_a < 0)
            return fail(SW_EINTERNAL, "two-halves pass: the lower half reaches %d, the halves gave %lld", e->score,
                        (long long)S);
        out->score = (int32_t)S;
        out->end_a = mid + e->end_a;
        out->end_b = e->end_b;
        const unsigned long long lower = (unsigned long long)(M - mid) * (unsigned long long)N;
        cells += lower;
        pruned += e->pruned_cells;
    }
    out->cells_computed = (int64_t)(pruned >= cells ? 0 : cells - pruned);
    return SW_OK;
}
