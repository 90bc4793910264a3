// Internal declarations shared by the HIP translation units of libswmi.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace swmi {

constexpr int kWave = 64;          // wavefront width on gfx950
constexpr int kTick = 64;          // steps a wave runs between boundary exchanges
constexpr int kBPad = 128;         // code bytes before column 0 of the column sequence
constexpr int kBPadTail = 256;     // code bytes after its last column
constexpr int kSlotPad = 64;       // slot index of a band's first column
constexpr uint8_t kPadCode = 4;    // column code that scores -128 against every row
constexpr int32_t kDone = 0x7fffffff;
constexpr uint32_t kPadTable = 0x80808080u;

// One (band, stripe) task's best cell: value, then the smallest row holding it
// in the stripe, then the first column of that row reaching it (-1 if not tracked).
struct TaskRec {
    int32_t score;
    int32_t pad;
    int64_t row;
    int64_t col;
};

// Everything the forward local pass needs; device pointers.
struct FwdArgs {
    const uint8_t* a;        // row codes 0..3, length M
    const uint8_t* b;        // column codes; b[-kBPad .. N + kBPadTail) readable, pads = kPadCode
    int64_t M, N;
    int32_t match, mismatch, open, ext;
    int64_t Q;               // stripes (64 * R rows each)
    int64_t W;               // band width in columns (multiple of 64)
    int64_t n_bands;
    int2* slots;             // nslot rows of slot_stride {H, g} pairs
    int64_t slot_stride;
    int64_t nslot;
    int32_t* progress;       // [n_bands * Q] columns published per task (kDone when finished)
    uint32_t* ticket;        // task counter
    int32_t* gbest;          // running lower bound on the best score
    int2* lbuf;              // [M padded] {H, E} at the last column of the previous band
    TaskRec* recs;           // [n_bands * Q]
    unsigned long long* pruned_cells;  // cells skipped by pruning
    int32_t prune;           // 0: none, 1: skip tiles that cannot reach max(gbest, threshold)
    int32_t threshold;       // external lower bound T (0 = none)
};

struct ScoreOut {
    int32_t score;
    int32_t status;          // 0 ok, else internal error code
    int64_t end_a, end_b;
    unsigned long long pruned_cells;
};

hipError_t launch_encode(const uint8_t* src, int64_t n, uint8_t* dst, int64_t pad_before,
                         int64_t pad_after, unsigned long long* bad, hipStream_t st);
hipError_t launch_fwd(const FwdArgs& args, int rows_per_lane, int grid, hipStream_t st);
hipError_t launch_reduce(const TaskRec* recs, int64_t n, int64_t N, ScoreOut* out, hipStream_t st);
hipError_t launch_zero(void* p, size_t bytes, hipStream_t st);

}  // namespace swmi
