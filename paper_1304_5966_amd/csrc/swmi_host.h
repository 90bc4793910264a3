// Host-side declarations shared by the C-ABI translation units of libswmi.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <rocprofiler-sdk-roctx/roctx.h>

#include <vector>

#include "swmi.h"
#include "swmi_internal.h"

namespace swmi {

// A named range around a phase of the path (score pass, row slab, start pass,
// reconstruction level, batch), for tracers that record roctx ranges (rocprofv3
// --marker-trace); without a tracer the calls cost next to nothing.
struct Phase {
    explicit Phase(const char* name) { roctxRangePushA(name); }
    ~Phase() { roctxRangePop(); }
    Phase(const Phase&) = delete;
    Phase& operator=(const Phase&) = delete;
};

struct DevBuf {
    void* ptr = nullptr;
    size_t bytes = 0;
};

enum { BUF_INPUT = 0, BUF_WORK = 1, BUF_CODES = 2, BUF_OUT = 3, BUF_META = 4, BUF_COUNT = 5 };

// Learned thresholds (mlp.hip): workspace for n pairs of at most (M, N) letters, and
// T = floor(0.9 * predicted score) per pair from device letters.
size_t predict_workspace_size(int64_t max_M, int64_t max_N, int32_t n);
sw_status predict_thresholds(sw_context* ctx, const sw_model* m, const uint8_t* d_a, const int64_t* offs_a,
                             const uint8_t* d_b, const int64_t* offs_b, int32_t n, void* ws, size_t ws_bytes,
                             std::vector<int32_t>& T);

// Releases a context's captured batch launch (sw_context::batch_graph).
void free_batch_graph(void* g);

}  // namespace swmi

struct sw_context {
    int device = 0;
    hipStream_t stream = nullptr;
    int num_cu = 0;
    // captured batch launch (SW_FLAG_GRAPH) with its layout and pinned tables
    // (batch.hip), replayed while the call's inputs match its key
    void* batch_graph = nullptr;
    // autotuned shapes per workload class (0 = not tuned): rows per lane, waves per CU
    int tuned_R[4] = {0, 0, 0, 0};
    int tuned_wpc[4] = {0, 0, 0, 0};
    int tuned_bw[4] = {0, 0, 0, 0};      // column band width of local passes per class (0: automatic)
    void* scratch = nullptr;             // device address of the library's fixed scratch on `device`
    void* host_misc = nullptr;           // pinned 64 KiB for small host<->device copies
    size_t host_misc_bytes = 0;
    swmi::DevBuf bufs[swmi::BUF_COUNT];  // grow-only device buffers of the host-pointer API
    size_t max_workspace_bytes = 0;      // cap on the sum of bufs (0: none; sw_context_set_max_workspace)
};

namespace swmi {

// Host description of one DP problem (see Prob).
struct ProbSpec {
    int64_t a_off = 0, b_off = 0;  // into the launch's code buffers
    int64_t M = 0, N = 0;
    int32_t top_kind = BORDER_ZERO, left_kind = BORDER_ZERO;
    int32_t top_open = 0, left_open = 0;
    int32_t target = 0, prune = 0, track = 1;
    int64_t d_lo = -kNoBand, d_hi = kNoBand;
    int64_t out_off = -1;
    int64_t top_off = -1;    // BORDER_BUF top: index of row 0's column 0 in the launch's top_h/top_f
    int64_t rows_after = 0;  // rows of the whole matrix below this problem (row slabs)
};

// Decomposition and workspace layout of one engine launch.
struct EnginePlan {
    int R = 8;
    int wpc = 8;  // resident stripe waves per CU the launch is sized for
    int grid = 1;   // waves
    int chain = 1;  // waves per workgroup of a chain launch (1: none); the ticket order keeps runs of `chain`
    bool local = true;
    int64_t n_probs = 0, n_tasks = 0, n_tickets = 0, nslot = 2, slot_stride = 0, lbuf_rows = 0;
    std::vector<Prob> probs;
    std::vector<Ticket> tickets;
    std::vector<int64_t> order;  // order[k] = index in the spec list of probs[k]
    size_t off_tickets = 0, off_probs = 0, off_slots = 0, off_lbuf = 0, off_recs = 0, off_outs = 0;
    size_t off_zero = 0, off_prog = 0, off_gbest = 0, off_pruned = 0, off_misc = 0;
    size_t zero_bytes = 0, total = 0;
};

// misc block (bytes from off_misc)
enum { MISC_TICKET = 0, MISC_BAD_A = 16, MISC_BAD_B = 24, MISC_ABORT = 32, MISC_BYTES = 64 };
constexpr unsigned long long kBadBase = 1ull << 62;

size_t align_up(size_t v, size_t a);
// ScoreOut::status as text.
const char* engine_status_text(int32_t status);
sw_status fail(sw_status st, const char* fmt, ...);
sw_status ctx_buffer(sw_context* ctx, int slot, size_t bytes, void** out);
// Checks a caller's scoring and writes the copy the library works with: with a
// substitution matrix, match = max(1, largest entry) and mismatch = max(0,
// -smallest entry), so that every bound written with match holds.
sw_status check_scoring(const sw_scoring* s, sw_scoring* norm);
// Combinations the matrix scoring does not run (a threshold model, both strands).
sw_status check_matrix_options(const sw_scoring* norm, const sw_options* o);
// Encode table and substitution table of a checked scoring (n_class 0 for DNA).
EncTable enc_table(const sw_scoring* sc);
void subst_table(const sw_scoring* sc, Subst& out);
// s(x, y) of two codes (DNA codes or matrix classes); -128 for the padding code.
int32_t subst_score(const sw_scoring* sc, uint8_t x, uint8_t y);
// The accepted letters, for error messages.
const char* letters_text(const sw_scoring* sc);
sw_status check_lengths(int64_t la, int64_t lb, const sw_scoring* s);
sw_status check_options(const sw_options* o);

// Plans a launch over `specs` (problems are reordered by decreasing cell count).
// rows_per_lane / waves_per_cu / band_width: 0 = automatic.
EnginePlan plan_engine(const sw_context* ctx, const std::vector<ProbSpec>& specs, bool local,
                       int rows_per_lane, int waves_per_cu, int band_width);
// Runs a planned launch inside workspace `ws` (plan.total bytes): clears the
// counters, copies the table, launches the engine and the per-problem reduction
// into the ScoreOut array at ws + plan.off_outs (ordered like plan.probs).
// top_h/top_f: row 0 of BORDER_BUF problems (H and F per column, as out_h/out_f hold them).
sw_status run_engine(sw_context* ctx, const EnginePlan& plan, const uint8_t* a_codes, const uint8_t* b_codes,
                     const sw_scoring* sc, void* ws, int32_t* out_h, int32_t* out_f,
                     const int32_t* top_h = nullptr, const int32_t* top_f = nullptr);
sw_status upload_engine_table(sw_context* ctx, const EnginePlan& plan, void* ws);
sw_status launch_engine_kernels(sw_context* ctx, const EnginePlan& plan, const uint8_t* a_codes,
                                const uint8_t* b_codes, const sw_scoring* sc, void* ws, int32_t* out_h,
                                int32_t* out_f, const int32_t* top_h = nullptr, const int32_t* top_f = nullptr);
// Copies `bytes` from device to the context's pinned buffer and waits for the stream.
sw_status read_back(sw_context* ctx, const void* dev, size_t bytes, void** host);

sw_status upload_pair(sw_context* ctx, const char* a, int64_t la, const char* b, int64_t lb, uint8_t** d_a,
                      uint8_t** d_b);

// Score pass of one pair on device letters (workspace-driven; allocates nothing).
size_t score_workspace_size(const sw_context* ctx, int64_t M, int64_t N, const sw_options* o);
sw_status run_score(sw_context* ctx, const uint8_t* d_a, int64_t M, const uint8_t* d_b, int64_t N,
                    const sw_scoring* sc, const sw_options* o, void* ws, size_t ws_bytes, sw_score_result* out);

// Learned thresholds (mlp.hip): workspace for n pairs of at most (M, N) letters, and
// T = floor(0.9 * predicted score) per pair from device letters.
size_t predict_workspace_size(int64_t max_M, int64_t max_N, int32_t n);
sw_status predict_thresholds(sw_context* ctx, const sw_model* m, const uint8_t* d_a, const int64_t* offs_a,
                             const uint8_t* d_b, const int64_t* offs_b, int32_t n, void* ws, size_t ws_bytes,
                             std::vector<int32_t>& T);

// Two-halves score pass (halves.hip; SW_FLAG_HALVES).
size_t halves_workspace_size(const sw_context* ctx, int64_t M, int64_t N, const sw_options* o);
sw_status run_score_halves(sw_context* ctx, const uint8_t* d_a, int64_t M, const uint8_t* d_b, int64_t N,
                           const sw_scoring* sc, const sw_options* o, void* ws, size_t ws_bytes, sw_score_result* out);

}  // namespace swmi
