// Start-point pass and Myers-Miller reconstruction (SW# paper, Section 2).
#include <hip/hip_runtime.h>

#include <cstdlib>
#include <cstring>

#include "swmi.h"
#include "swmi_host.h"
#include "swmi_internal.h"

using namespace swmi;

extern "C" sw_status sw_start(sw_context* ctx, const char* a, int64_t len_a, const char* b, int64_t len_b,
                              const sw_scoring* scoring, int32_t score, int64_t end_a, int64_t end_b,
                              int64_t* start_a, int64_t* start_b) {
    (void)ctx; (void)a; (void)len_a; (void)b; (void)len_b; (void)scoring; (void)score; (void)end_a;
    (void)end_b; (void)start_a; (void)start_b;
    return fail(SW_EUNSUPPORTED, "sw_start: not built yet");
}

extern "C" sw_status sw_align(sw_context* ctx, const char* a, int64_t len_a, const char* b, int64_t len_b,
                              const sw_scoring* scoring, const sw_options* options, sw_align_result* out) {
    (void)ctx; (void)a; (void)len_a; (void)b; (void)len_b; (void)scoring; (void)options;
    if (out) std::memset(out, 0, sizeof *out);
    return fail(SW_EUNSUPPORTED, "sw_align: not built yet");
}

extern "C" void sw_align_result_free(sw_align_result* r) {
    if (!r) return;
    std::free(r->cigar);
    r->cigar = nullptr;
    r->cigar_len = 0;
}

extern "C" sw_status sw_batch(sw_context* ctx, const char* seqs_a, const int64_t* offs_a, const char* seqs_b,
                              const int64_t* offs_b, int32_t n_pairs, const sw_scoring* scoring,
                              const sw_options* options, sw_score_result* out) {
    (void)ctx; (void)seqs_a; (void)offs_a; (void)seqs_b; (void)offs_b; (void)n_pairs; (void)scoring;
    (void)options; (void)out;
    return fail(SW_EUNSUPPORTED, "sw_batch: not built yet");
}
