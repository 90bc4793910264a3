// Internal declarations shared by the HIP translation units of libswmi.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace swmi {

constexpr int kWave = 64;          // wavefront width on gfx950
constexpr int kTick = 64;          // steps a wave runs between boundary exchanges
constexpr int kBPad = 128;         // code bytes before column 0 of every column sequence
constexpr int kBPadTail = 256;     // code bytes after its last column
constexpr int kSlotPad = 64;       // slot index of a band's first column
constexpr uint8_t kPadCode = 4;    // column code that scores -128 against every row
constexpr int32_t kDone = 0x7fffffff;
constexpr uint32_t kPadTable = 0x80808080u;
constexpr int32_t kNeg = -(1 << 30);  // minus infinity of the global recurrence
constexpr int64_t kNoBand = (int64_t)1 << 62;

// Shifted ticks of R = 4 and 8 rows per lane shift every cell by its stripe row as
// well as its tick column (times gap_extend), so their score bytes hold s + 2 ext;
// R = 6 shifts by the column only (s + ext).  The bytes must stay within int8.
constexpr bool cd_row_shift(int rows_per_lane) { return rows_per_lane == 4 || rows_per_lane == 8; }
constexpr int cd_bias_ext(int rows_per_lane) { return cd_row_shift(rows_per_lane) ? 2 : 1; }

// Substitution-matrix scoring (protein alignment).  Letters are encoded as their
// index in the matrix alphabet; the class after the last letter is the padding
// class, whose row and column score -128 like kPadCode's.
constexpr int kMaxClasses = 32;  // letters + the padding class
struct Subst {
    int8_t s[kMaxClasses][kMaxClasses];  // s[class of the A letter][class of the B letter]
    int32_t n_class;                     // letters + 1 (0: match / mismatch scoring over ACGT)
    int32_t pad_;
};

// Letter -> code table of the encode kernels (by value in the kernel arguments).
struct EncTable {
    int8_t cls[256];   // class of each byte, -1: not a letter (unused when dna)
    int32_t dna;       // 1: ACGTacgt -> 0..3, padding kPadCode, complement = code ^ 3
    int32_t pad_code;  // code written around column sequences and for rejected letters
};


// Border of a problem's DP matrix (row 0 or column 0).
enum BorderKind : int32_t {
    BORDER_ZERO = 0,  // local alignment: H = 0
    BORDER_NEG = 1,   // anchored: H = -inf (the corner H(0,0) stays 0)
    BORDER_GAP = 2,   // a gap run from the corner: H = -(open_cost + ext * k)
    BORDER_BUF = 3    // top border only: row 0 is a row of a larger matrix, given as H and F
                      // (the vertical-gap state) per column 0..N in EngineArgs::top_h/top_f
};

// One DP problem of a launch.  Rows are the `a` codes, columns the `b` codes;
// DP coordinates are 1-based (row 0 and column 0 are the borders).
struct Prob {
    int64_t a_off;       // first row code in the a-code buffer
    int64_t b_off;       // column 0's code in the b-code buffer (padding around it)
    int64_t M, N;
    int64_t W, n_bands, Q;
    int64_t task0;       // first ticket of this problem (problems are ticket-contiguous)
    int64_t lbuf_off;    // first row of this problem in the band-boundary buffer
    int64_t out_off;     // last-row outputs at out_h/out_f[out_off + j], j = 0..N; -1: none
    int64_t d_lo, d_hi;  // diagonal band j - i kept by the global recurrence (kNoBand: all)
    int64_t top_off;     // BORDER_BUF: row 0's column 0 at top_h/top_f[top_off]
    int64_t rows_after;  // rows of the whole matrix below this problem's last row (row slabs):
                         // a path through a tile may continue there, so its bound counts them
    int32_t top_kind, left_kind;
    int32_t top_open, left_open;  // gap-open cost of BORDER_GAP borders
    int32_t target;      // tiles whose upper bound is below max(running best, target) are skipped
    int32_t prune;       // 1 = skip tiles by that bound (exact; paper Section 2, pruning)
    int32_t track;       // 1 = find the first cell of the best score (endpoint / start point)
    int32_t pad_;
};

// One (band, stripe) task's best cell: value, then the smallest row holding it
// in the stripe, then the first column of that row reaching it (-1 if not tracked).
struct TaskRec {
    int32_t score;
    int32_t pad;
    int64_t row;
    int64_t col;
};

// Ticket k of a launch (tickets are taken in order by the resident waves).
// Only tasks holding a cell of their problem's kept diagonal band get a
// ticket; a task without one has no work, and its neighbours read -inf where
// they would have read its values.  Tasks of different problems are
// interleaved so that a stripe's producer is usually far ahead when the
// stripe starts.  All referenced tickets are older.
struct Ticket {
    int32_t pi;            // problem (index into the table)
    int32_t local;         // task index inside the problem: band * Q + stripe
    int32_t prod;          // ticket of the stripe above in the same band (-1: first stripe, or no task)
    int32_t left;          // ticket of the same stripe in the previous band (-1: band 0, or no task)
    int32_t reuse_reader;  // reader of the slot this ticket reuses (ticket - nslot's consumer), -1 if none
    int32_t corner;        // without a producer task: ticket of the stripe above in the previous
                           // band, whose boundary capture holds this task's corner value; else -1
    int32_t cons;          // ticket of the stripe below in the same band (-1: none); read only as
                           // a scheduling hint, never waited on
    int32_t pad;
};

// Does task (band, stripe q) of problem `pr` hold any cell of the kept
// diagonal band, with stripes of 64 R rows?
__host__ __device__ inline bool task_in_band(const Prob& pr, int64_t band, int64_t q, int R) {
    if (pr.d_lo <= -kNoBand && pr.d_hi >= kNoBand) return true;
    const int64_t R0 = q * (int64_t)(kWave * R);
    const int64_t R1 = R0 + (int64_t)(kWave * R) < pr.M ? R0 + (int64_t)(kWave * R) : pr.M;
    const int64_t c0 = band * pr.W;
    const int64_t W = pr.W < pr.N - c0 ? pr.W : pr.N - c0;
    const int64_t dmin = c0 + 1 - R1, dmax = c0 + W - R0 - 1;
    return !(dmax < pr.d_lo || dmin > pr.d_hi);
}

// Ticks [lo, hi] of a task (stripe rows from R0, band columns from c0, n_ticks
// ticks) that hold a cell of the kept diagonal band: tick tau covers diagonals
// from c0 + 64 tau - R0 - 64 R - 62 to c0 + 64 tau + 63 - R0 (the range the tick
// loop's band test checks).  Unbanded: every tick.  lo > hi: none.
__host__ __device__ inline void band_ticks(const Prob& pr, int64_t R0, int64_t c0, int R, int n_ticks, int& lo,
                                           int& hi) {
    const int64_t a = pr.d_lo - (kTick - 1) + R0 - c0;                       // 64 tau >= a
    const int64_t b = pr.d_hi + R0 + (int64_t)kWave * R + (kTick - 2) - c0;  // 64 tau <= b
    const int64_t l = a <= 0 ? 0 : (a + kTick - 1) / kTick;
    const int64_t h = b < 0 ? -1 : b / kTick;
    lo = (int)(l < n_ticks ? l : n_ticks);
    hi = (int)(h < n_ticks - 1 ? h : n_ticks - 1);
}

// Columns a task of the global recurrence writes to its slot (for its consumer):
// from its first tick's first output column to its last tick's last; slots are
// indexed from the first.
__host__ __device__ inline void slot_columns(int lo, int hi, int& first, int& last) {
    first = kTick * lo - (kTick - 1);
    if (first < 0) first = 0;
    last = kTick * hi;
}

struct EngineArgs {
    const Ticket* tickets;
    const Prob* probs;
    int64_t n_probs;
    int64_t n_tickets;
    const uint8_t* a_codes;
    const uint8_t* b_codes;
    int32_t match, mismatch, open, ext;
    int2* slots;             // nslot rows of slot_stride {H, gap} pairs
    int64_t slot_stride;
    int64_t nslot;
    int32_t* progress;       // [n_tickets] columns published (kDone when finished)
    uint32_t* ticket;
    int32_t* gbest;          // [n_probs] running best of each problem
    int2* lbuf;              // {H, E} at the last column of the previous band, per row
    TaskRec* recs;           // [tasks], at task0 + local; written by ticketed tasks only
    unsigned long long* pruned;  // [n_probs] cells skipped
    int32_t* out_h;          // last-row H of problems with out_off >= 0
    int32_t* out_f;          // last-row F (deletion-ending) of the same
    const int32_t* top_h;    // row 0 of BORDER_BUF problems: H
    const int32_t* top_f;    // and F (deletion-ending), as out_h/out_f write them
    uint32_t jitter;         // schedule-perturbation seed (tests; 0 = off)
    int32_t* abort_flag;     // set when a wait timed out (cleared per launch)
    uint64_t wait_limit;     // a wait longer than this (ticks of the 100 MHz counter) aborts the launch
    Subst sub;               // matrix scoring (n_class > 0): codes are letter classes
};

struct ScoreOut {
    int32_t score;
    int32_t status;          // 0 ok; 1 endpoint not tracked; 2 a wait of the launch timed out
    int64_t end_a, end_b;
    unsigned long long pruned_cells;
};

// Midline of a split (Myers-Miller; the paper's two-halves score pass): the
// forward half's last row (CC = H, DD = deletion-ending F) at out offset fwd_out
// + j and the reversed half's (RR, SS) at rev_out + (N - j), j = 0..N.
struct MidTask {
    int64_t fwd_out, rev_out;  // out_h/out_f offsets of the forward and reversed halves
    int64_t N;                 // columns
};

struct MidResult {
    int64_t value;           // max over j of CC + RR (plain crossing) and DD + SS + g (a deletion run through it)
    int64_t j;               // the first column reaching it (a plain crossing first at equal columns)
    int32_t type;            // 1: plain crossing, 2: deletion run through the midline
    int32_t pad;
    int64_t cc, dd, rr, ss;  // the four last-row values at that column
};

hipError_t launch_midline(const MidTask* tasks, int64_t n, const int32_t* oh, const int32_t* of, int32_t g,
                          MidResult* out, hipStream_t st);

// mode: ENC_REVERSE and/or ENC_COMPLEMENT (0: the letters as they are; the
// complement exists for DNA only).
enum { ENC_REVERSE = 1, ENC_COMPLEMENT = 2 };
hipError_t launch_encode(const uint8_t* src, int64_t n, uint8_t* dst, int64_t pad_before, int64_t pad_after,
                         int mode, const EncTable& tab, unsigned long long* bad, hipStream_t st);
hipError_t launch_encode_many(const uint8_t* src, const int64_t* src_off, const int64_t* dst_off,
                              const int64_t* len, int64_t n, uint8_t* dst, const EncTable& tab,
                              unsigned long long* bad, hipStream_t st);
// cd: run the fast ticks in the shifted domain (requires every substitution
// score plus cd_bias_ext(rows_per_lane) * gap_extend within -127..127).
// waves_per_cu picks the register budget: rows_per_lane 8 and 6 run 2 waves per
// SIMD (256 VGPRs) up to 8 waves per CU and 3 (168 VGPRs) above; rows_per_lane 4 runs 4.
// Matrix scoring (args.sub.n_class > 0) runs the same shapes; its launches take
// n_class * 64 * (4 or 8) bytes of dynamic LDS for the stripe's query profile.
// grid: waves.  chain (4 or 8; 1: off): where chain_variant() holds, the launch runs
// workgroups of `chain` waves that take `chain` consecutive tickets at a time and
// link consecutive stripes through LDS (the ticket table must then keep each
// problem's stripes in runs of `chain` tickets to profit; any valid table is correct).
bool chain_variant(int rows_per_lane, bool local, bool cd, int n_class, int chain);
hipError_t launch_engine(const EngineArgs& args, int rows_per_lane, int waves_per_cu, bool local, bool cd, int grid,
                         int chain, hipStream_t st);
// rows_per_lane: the launch's R (records of tasks outside a kept band are skipped).
hipError_t launch_reduce(const TaskRec* recs, const Prob* probs, int64_t n_probs, int rows_per_lane, ScoreOut* out,
                         const int32_t* gbest, const unsigned long long* pruned, const int32_t* abort_flag,
                         hipStream_t st);
hipError_t launch_zero(void* p, size_t bytes, hipStream_t st);
hipError_t launch_fill_i32(int32_t* p, int32_t v, size_t n, hipStream_t st);

}  // namespace swmi
