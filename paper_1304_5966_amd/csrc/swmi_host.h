// Host-side declarations shared by the C-ABI translation units of libswmi.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "swmi.h"

namespace swmi {

struct DevBuf {
    void* ptr = nullptr;
    size_t bytes = 0;
};

enum { BUF_INPUT = 0, BUF_WORK = 1, BUF_AUX = 2, BUF_AUX2 = 3, BUF_COUNT = 4 };

}  // namespace swmi

struct sw_context {
    int device = 0;
    hipStream_t stream = nullptr;
    int num_cu = 0;
    void* host_misc = nullptr;           // pinned 4 KiB for small device-to-host reads
    swmi::DevBuf bufs[swmi::BUF_COUNT];  // grow-only device buffers of the host-pointer API
};

namespace swmi {

// Work decomposition and workspace layout of one score pass.
struct ScorePlan {
    int R;               // rows per lane
    int grid;            // resident stripe waves (one wave per workgroup)
    int64_t M, N, Q, W, n_bands, nslot, slot_stride;
    size_t off_a, off_b, off_slots, off_lbuf, off_recs, off_zero, off_prog, off_misc;
    size_t zero_bytes, total;
};

sw_status fail(sw_status st, const char* fmt, ...);
sw_status ctx_buffer(sw_context* ctx, int slot, size_t bytes, void** out);
sw_status check_scoring(const sw_scoring* s);
sw_status check_lengths(int64_t la, int64_t lb, const sw_scoring* s);
sw_status check_options(const sw_options* o);
ScorePlan plan_score(const sw_context* ctx, int64_t M, int64_t N, const sw_options* o);
sw_status run_score(sw_context* ctx, const uint8_t* d_a, int64_t M, const uint8_t* d_b, int64_t N,
                    const sw_scoring* sc, const sw_options* o, void* ws, size_t ws_bytes, sw_score_result* out);
sw_status upload_pair(sw_context* ctx, const char* a, int64_t la, const char* b, int64_t lb, uint8_t** d_a,
                      uint8_t** d_b);

}  // namespace swmi
