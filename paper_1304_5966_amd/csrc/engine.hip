// Wavefront engine for the affine-gap dynamic programs of SW# (paper Section 2)
// on gfx950: the first-phase local pass, the anchored reverse pass and the
// global (Needleman-Wunsch) halves of the Myers-Miller reconstruction.
//
// One launch solves a table of independent problems.  Rows are codes of A,
// columns codes of B; DP coordinates are 1-based with borders at row/column 0.
//
//   local  (first phase; E/F clamped at 0, exact for H since a non-positive gap
//           value never beats the zero floor):
//     E = max(E' - ext, H' - open, 0)   F = max(F' - ext, H' - open)
//     H = max(Hdiag + s, E, F)          (>= 0 through E)
//   global (reverse pass, reconstruction): the same without the zero;
//           "minus infinity" is kNeg = -2^30.
//
// Work decomposition (the paper's wavefront of cell blocks, mapped to wave64):
//  * A stripe is 64*R consecutive rows; lane l owns rows l*R .. l*R+R-1 of it
//    and at step t works on column t-l (anti-diagonal skew of one column per
//    lane).  H, E and H-open live in int32 VGPRs.
//  * Each step the lane below receives the lane above's last-row H and its
//    F-candidate max(F - ext, H - open) through DPP wave_shr:1; lane 0
//    receives the row above the stripe through the DPP "old" operand, read
//    from an LDS staging ring.
//  * Substitution scores: per row a 4-byte table s(a_row, c), c = 0..3; one
//    v_perm_b32 with four column codes as selector yields four score bytes,
//    consumed by sign-extended byte-select adds.  With a substitution matrix
//    (protein) the stripe keeps a query profile in LDS instead: for every
//    letter class c, the lane's R row scores s(a_row, c) as bytes; one LDS read
//    per step at the column's class yields the step's R score bytes.
//  * Columns are cut into bands of W; a task is (problem, band, stripe), taken
//    from an in-order ticket counter through a host-built table (problems in
//    decreasing size; the tasks of a group of problems interleaved, each
//    problem's in band, then stripe order).  A task only waits on older
//    tickets: the stripe above in the
//    same band (its bottom row streamed through a global slot with a published
//    column count), the same stripe in the previous band (its right boundary
//    H,E per row) and the two tasks that last wrote and read the slot being
//    reused.  The oldest unfinished task never waits: no deadlock, no
//    residency assumption.
//  * Every 64 steps (a tick) the wave exchanges 64 boundary columns: the next
//    tick's inputs are prefetched, lane 63's outputs go to the task's slot and
//    the column count is published after the outputs are stored.
//  * Tile skipping (paper Section 2, pruning and banding): before a tick,
//    UB = max(every H on the tick's input borders [, 0]) + match * min(rows
//    left, columns left); the tick is skipped if UB is strictly below
//    max(running best, target), or if it lies outside the kept diagonal band.
//    A skipped tick outputs lower bounds (0 / -inf).  Exact by induction along
//    an optimal path.  Tasks entirely outside the band get no ticket.
//  * Fast ticks run in a shifted domain, for both recurrences, whenever the
//    scores fit it: every value carries (stripe row + tick column) * ext for
//    R = 4 and 8 rows per lane (run_tick_rs), (tick column) * ext for R = 6
//    (run_tick_cd).
//  * First cell of the best score: a tick whose cells can reach max(running
//    best, target) (by the border bound above, over the tick's 127 columns)
//    keeps its lanes' maximum; if a lane reaches it, the tick is replayed from
//    a snapshot in the plain domain to find each row's maximum and the first
//    column holding it.  Other ticks keep no maximum.
#include "swmi_internal.h"

namespace swmi {

// ------------------------------------------------------------------------ helpers

__device__ __forceinline__ int dpp_shr1(int old, int src) {
    // wave_shr:1, bound_ctrl off: lane l <- src of lane l-1; lane 0 keeps `old`
    return __builtin_amdgcn_update_dpp(old, src, 0x138, 0xf, 0xf, false);
}

__device__ __forceinline__ int sext_byte(uint32_t w, int i) { return ((int)(w << (24 - 8 * i))) >> 24; }

__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = max(v, __shfl_xor(v, off));
    return v;
}

// Stripe-to-stripe hand-off.  Producer and consumer usually sit on different
// XCDs, each with its own L2.  Release/acquire at agent scope would write back
// and invalidate a whole L2 on every tick (measured: less than half the
// throughput), so boundary values and column counts are system-scope relaxed
// atomics, which write through and read past the per-XCD caches.  Ordering:
// the producer waits for its boundary stores to complete (vmcnt 0) before
// storing the count; the consumer reads boundary values only after reading a
// sufficient count.
__device__ __forceinline__ int2 ld_shared_i2(const int2* p) {
    const unsigned long long v =
        __hip_atomic_load(reinterpret_cast<const unsigned long long*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    return make_int2((int)(uint32_t)v, (int)(uint32_t)(v >> 32));
}

__device__ __forceinline__ void st_shared_i2(int2* p, int2 v) {
    const unsigned long long w = (unsigned long long)(uint32_t)v.x | ((unsigned long long)(uint32_t)v.y << 32);
    __hip_atomic_store(reinterpret_cast<unsigned long long*>(p), w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

__device__ __forceinline__ int load_count(const int32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

__device__ __forceinline__ void publish_count(int32_t* p, int32_t v) {
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Bounded waits.  A wait that has not ended after `limit` ticks of the 100 MHz
// real-time counter (EngineArgs::wait_limit, 120 s unless the host sets another)
// raises the launch's abort flag; from then on every wait of the launch ends at
// once, the kernel runs to completion on meaningless values (every address comes
// from the ticket table, none from values) and the host reports an internal
// error instead of hanging.

// True: give up waiting (the launch's abort flag is set, or this wait, begun at
// t0, has run out; then it sets the flag).
__device__ __forceinline__ bool wait_expired(int32_t* abort_flag, uint64_t limit, uint64_t t0) {
    if (load_count(abort_flag)) return true;
    if (__builtin_amdgcn_s_memrealtime() - t0 > limit) {
        __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        return true;
    }
    return false;
}

// Called on every unsuccessful poll; true: give up waiting.
__device__ __forceinline__ bool wait_abandoned(int32_t* abort_flag, uint64_t limit, uint64_t& t0, uint32_t& polls) {
    if (polls++ == 0) t0 = __builtin_amdgcn_s_memrealtime();
    if ((polls & 15) != 0) return false;  // every 16th poll (each poll is a memory round trip)
    return wait_expired(abort_flag, limit, t0);
}

// Waits until *flag >= need; `seen` caches the last value read.
__device__ __forceinline__ void wait_at_least(const int32_t* flag, int32_t need, int32_t& seen,
                                              int32_t* abort_flag, uint64_t limit) {
    uint64_t t0 = 0;
    uint32_t polls = 0;
    while (seen < need) {
        seen = load_count(flag);
        if (seen < need) {
            if (wait_abandoned(abort_flag, limit, t0, polls)) {
                seen = need;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
    }
    asm volatile("" ::: "memory");
}

// Chain workgroups (the banded global passes): K waves of one workgroup take K
// consecutive tickets, which for a banded problem are consecutive stripes of one
// band, and each hands its bottom row to the next wave through LDS instead of a
// global slot.  LDS instructions of one wave are executed in order, so a value
// written before a count is there for a wave that has read that count; the
// accesses are relaxed atomics (no reordering by the compiler, no cache
// maintenance).  The last wave of a group hands off through its global slot as
// every other task does.
constexpr int kRing = 4 * kTick;  // columns of a link ring (producer at most 4 ticks ahead)

__device__ __forceinline__ int lds_load(const int* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ void lds_store(int* p, int v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Waits until the LDS word *flag >= need.  An LDS poll is cheap, so the launch's
// abort flag (a memory round trip) is read only every 256th poll.
__device__ __forceinline__ void lds_wait_at_least(const int* flag, int need, int& seen, int32_t* abort_flag,
                                                  uint64_t limit) {
    uint64_t t0 = 0;
    uint32_t polls = 0;
    while (seen < need) {
        seen = lds_load(flag);
        if (seen < need) {
            if (polls++ == 0) t0 = __builtin_amdgcn_s_memrealtime();
            if ((polls & 255) == 0 && wait_expired(abort_flag, limit, t0)) {
                seen = need;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
    }
    asm volatile("" ::: "memory");
}

// Orders the LDS accesses of one wave around a hand-off point (one wave per
// workgroup: the workgroup barrier; chain workgroups: the wave alone).
template <int K>
__device__ __forceinline__ void wave_sync() {
    if constexpr (K == 1) {
        __syncthreads();
    } else {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

// Schedule perturbation (a test mode; off when seed == 0): a wave-uniform
// pseudo-random pause, so that tests see the hand-off protocol under other
// interleavings of producers, consumers and slot reuse.  About one call in
// eight pauses, for up to 15 x 127 x 64 cycles.
__device__ __forceinline__ void jitter_pause(uint32_t seed, int64_t task, int32_t step) {
    if (!seed) return;
    uint32_t h = seed ^ (uint32_t)task * 0x9E3779B1u ^ (uint32_t)step * 0x85EBCA77u;
    h ^= h >> 15;
    h *= 0x2C1B3C6Du;
    h ^= h >> 12;
    h = __builtin_amdgcn_readfirstlane(h);
    if ((h & 7) != 0) return;
    for (uint32_t i = 0; i < ((h >> 3) & 15); ++i) __builtin_amdgcn_s_sleep(127);
}

// Four score bytes s(a, c) + bias for c = 0..3 (pad row: all -128).
__device__ __forceinline__ uint32_t row_table(int code, int match, int mismatch, int bias) {
    if (code > 3) return kPadTable;
    const uint32_t mm = (uint32_t)(uint8_t)(int8_t)(bias - mismatch) * 0x01010101u;
    const int sh = 8 * code;
    return (mm & ~(0xffu << sh)) | ((uint32_t)(uint8_t)(int8_t)(match + bias) << sh);
}

// H on row 0 (top) or column 0 (left) at distance k >= 1 from the corner; a
// BORDER_GAP border is a gap run from the corner whose first position costs
// open_cost and every further one ext.
__device__ __forceinline__ int border_h(int kind, int open_cost, int ext, int64_t k) {
    if (kind == BORDER_ZERO) return 0;
    if (kind == BORDER_NEG) return kNeg;
    return (int)(-((int64_t)open_cost + (int64_t)ext * (k - 1)));
}

template <int R>
struct WaveState {
    int H[R];      // H of the lane's rows at the last column processed
    int E[R];      // E (clamped at 0 in the local recurrence)
    int HA[R];     // H - open
    uint32_t T[R]; // substitution table of each row
    int hup;       // H received from the row above at the previous step (next diagonal of the first row)
    int hl, gl;    // this lane's last-row H and F-candidate of the previous step (DPP sources)
};

// Per-row running maxima; kept in LDS between the ticks that need them.
template <int R>
struct RowBest {
    int best[R];   // running maximum of each row
    int pos[R];    // first column holding best[] (-1 when not tracked)
};

struct TickCtx {
    const int2* in;       // LDS: 64 lane-0 inputs {H, F-candidate} of this tick
    const int2* in_cd;    // the same inputs plus m * ext at step m (H one ext less under the row shift)
    int2* out;            // LDS: 64 lane-63 outputs
    const uint32_t* bring;  // LDS: the tick's column codes, dwords from bbase on (shifted ticks)
    const uint32_t* prof;   // LDS: this lane's query-profile entry of class 0 (matrix scoring)
    uintptr_t bbase;        // address of the first staged dword
    int2* lbuf;           // right-boundary store for the next band (capture)
    int32_t* out_h;       // last-row outputs (reconstruction halves)
    int32_t* out_f;
    int64_t row0;         // lbuf index of this lane's first row
    int64_t col0;         // problem column of step 0 for lane 0
    int64_t out_base;     // out index of band column 0's DP column (c0 + 1)
    int lane;
    int rel0;             // band-relative column of step 0 for lane 0
    int W;                // band width
    int M_rows;           // rows of this lane inside the matrix (0..R)
    int open, ext;
    int out_lane, out_k;  // lane and sub-row holding the last row (-1 if not in this stripe)
    bool capture;         // store H,E at the band's last column into lbuf
};

// Substitution scores of one group of 4 steps for the lane's R rows.
//  DNA:    per row one v_perm_b32 of the row's 4-entry table by the four column
//          codes (pad code 4 selects a byte of kPadTable).
//  matrix: per step one LDS read of the query profile at the step's column
//          class: entry (class, lane) holds the R row scores as bytes, so the
//          read is 4 or 8 bytes at (class * 64 + lane) * (4 or 8) -- bank-conflict
//          free within each half wave.
template <int R, bool PROT>
struct ScoreGroup {
    uint32_t sc[R];
    __device__ __forceinline__ void load(const uint32_t (&T)[R], uint32_t cw, const TickCtx&) {
#pragma unroll
        for (int k = 0; k < R; ++k) sc[k] = __builtin_amdgcn_perm(kPadTable, T[k], cw);
    }
    __device__ __forceinline__ int get(int i, int k) const { return sext_byte(sc[k], i); }
};

template <int R>
struct ScoreGroup<R, true> {
    static constexpr int kW = R > 4 ? 2 : 1;  // dwords per profile entry
    uint32_t w[4][kW];
    __device__ __forceinline__ void load(const uint32_t (&)[R], uint32_t cw, const TickCtx& c) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const uint32_t cls = __builtin_amdgcn_ubfe(cw, 8 * i, 8);
            const uint32_t* e = c.prof + cls * (uint32_t)(kWave * kW);
            if (kW == 2) {
                const uint2 v = *reinterpret_cast<const uint2*>(e);
                w[i][0] = v.x;
                w[i][kW - 1] = v.y;
            } else {
                w[i][0] = *e;
            }
        }
    }
    __device__ __forceinline__ int get(int i, int k) const { return sext_byte(w[i][k >> 2], k & 3); }
};

// Tick modes.
//  kRun:   compute; per-row running maxima.
//  kTrack: replay -- no outputs, no maxima; records the first column where a
//          wanted row reaches its (already known) maximum.
//  kExact: replay -- no outputs; per-row maxima and their first columns.
constexpr int kRun = 0, kTrack = 1, kExact = 2;

// One tick: 64 steps of the skewed stripe in the plain domain.
//  SLOW: per-step predicates -- lanes left of the band's first column hold
//        their state (tick 0); H,E at the band's last column go to lbuf; the
//        last matrix row's H and F go to out_h/out_f.
//  CD:   the row tables hold the shifted-domain scores (s + ext, or s + 2 ext
//        where the row shift is on); subtract the bias.
template <int R, bool LOCAL, int MODE, bool SLOW, bool CD, bool PROT>
__device__ __forceinline__ void run_tick(WaveState<R>& s, RowBest<R>& rb, const uint8_t* first,
                                         const TickCtx& c, const bool (&want)[R]) {
    constexpr bool REPLAY = MODE != kRun;
    const uint32_t* src = reinterpret_cast<const uint32_t*>((uintptr_t)first & ~(uintptr_t)3);
    const uint32_t sh = (uint32_t)((uintptr_t)first & 3);
    uint32_t lo = src[0], hi = src[1];
    // Matrix scoring: the profile reads of a group are issued one group ahead, and
    // the column-code dwords that address them one group before that (LDS reads
    // complete in order, so a code dword read just before its use would also wait
    // for the profile reads in flight).
    uint32_t hi2 = PROT ? src[2] : 0;
    ScoreGroup<R, PROT> sg_next;
    if (PROT) sg_next.load(s.T, __builtin_amdgcn_alignbyte(hi, lo, sh), c);
    // lane 0's inputs are read one 4-step group ahead (the ring holds 64 + 4 entries)
    const int4* in4 = reinterpret_cast<const int4*>(c.in);
    int4 nx0 = in4[0], nx1 = in4[1];
    const int bias = CD ? cd_bias_ext(R) * c.ext : 0;
    constexpr int kUnroll = (SLOW || REPLAY) ? 1 : 2;  // the hot path renames its carried registers
#pragma unroll kUnroll
    for (int g = 0; g < kTick / 4; ++g) {
        const uint32_t cw = __builtin_amdgcn_alignbyte(hi, lo, sh);
        lo = hi;
        if (PROT) {
            hi = hi2;
            hi2 = src[g + 3];
        } else {
            hi = src[g + 2];
        }
        const int2 ins[4] = {make_int2(nx0.x, nx0.y), make_int2(nx0.z, nx0.w), make_int2(nx1.x, nx1.y),
                             make_int2(nx1.z, nx1.w)};
        nx0 = in4[2 * g + 2];
        nx1 = in4[2 * g + 3];
        ScoreGroup<R, PROT> sg;
        if (PROT) {
            sg = sg_next;
            sg_next.load(s.T, __builtin_amdgcn_alignbyte(hi, lo, sh), c);
        } else {
            sg.load(s.T, cw, c);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int m = 4 * g + i;
            const int2 in = ins[i];
            const int upH = dpp_shr1(in.x, s.hl);
            const int upG = dpp_shr1(in.y, s.gl);
            int diag = s.hup;
            s.hup = upH;
            int F = upG;
            const int rel = c.rel0 + m - c.lane;
            const bool act = SLOW ? (rel >= 0) : true;
#pragma unroll
            for (int k = 0; k < R; ++k) {
                const int Hd = diag + sg.get(i, k) - bias;
                const int En = LOCAL ? max(max(s.E[k] - c.ext, s.HA[k]), 0) : max(s.E[k] - c.ext, s.HA[k]);
                const int Hn = max(max(Hd, En), F);
                const int HAn = Hn - c.open;
                if (SLOW) {
                    if (!REPLAY && c.out_k == k && c.lane == c.out_lane && act && rel < c.W) {
                        c.out_h[c.out_base + rel] = Hn;
                        c.out_f[c.out_base + rel] = F;
                    }
                }
                F = max(F - c.ext, HAn);
                diag = s.H[k];
                if (SLOW) {
                    if (act) {
                        s.H[k] = Hn;
                        s.E[k] = En;
                        s.HA[k] = HAn;
                    }
                    if (!REPLAY && c.capture && rel == c.W - 1 && k < c.M_rows)
                        st_shared_i2(c.lbuf + c.row0 + k, make_int2(Hn, En));
                } else {
                    s.H[k] = Hn;
                    s.E[k] = En;
                    s.HA[k] = HAn;
                }
                if (MODE == kTrack) {
                    if (act && want[k] && rb.pos[k] < 0 && Hn == rb.best[k]) rb.pos[k] = (int)(c.col0 + m - c.lane);
                } else if (MODE == kExact) {
                    if (act && Hn > rb.best[k]) {
                        rb.best[k] = Hn;
                        rb.pos[k] = (int)(c.col0 + m - c.lane);
                    }
                } else if (SLOW) {
                    if (act) rb.best[k] = max(rb.best[k], Hn);
                } else {
                    rb.best[k] = max(rb.best[k], Hn);
                }
            }
            s.hl = s.H[R - 1];
            s.gl = F;
            if (!REPLAY && c.lane == kWave - 1) c.out[m] = make_int2(s.hl, s.gl);
        }
    }
}

// One fast tick in the column-shifted domain: at step m every value of lane l
// is stored plus z = (m - l) * ext, i.e. plus ext per DP column.  With
// g = open - ext the local recurrence becomes
//     E~ = max(E~', H~' - g, z)    H~ = max(H~diag + (s + ext), E~, F~)
//     F~(next row) = max(F~, H~ - g) - ext
// (the row tables already hold s + ext): E's extension cost and the zero floor
// cost nothing extra, and a value handed to the next lane keeps its offset
// because that lane works on the same column one step later.  The global
// recurrence (LOCAL = false) is the same without the z term.  Lane 63's
// outputs stay shifted (out[m] carries z = (m - 63) * ext).  Instead of per-row
// maxima the tick returns the lane's exact maximum H (plain domain).
//
// TRACKMAX = false: no running maximum (returns kNeg), for ticks whose cells
// provably stay below the value that would need it.
template <int R, bool TRACKMAX, bool LOCAL, bool PROT>
__device__ __forceinline__ int run_tick_cd(WaveState<R>& s, const uint8_t* first, const TickCtx& c) {
    const int ext = c.ext, g = c.open - c.ext;
    const int off = -(c.lane + 1) * ext;  // the carried state belongs to step -1
    int HA[R];
#pragma unroll
    for (int k = 0; k < R; ++k) {
        s.H[k] += off;
        s.E[k] += off;
        HA[k] = s.H[k] - g;
    }
    s.hup += off;
    s.hl += off;
    s.gl += off;
    int z = -c.lane * ext;
    int acc = kNeg;        // max over the steps so far of (H - z_step), plus the current z
    int ohl = 0, ogl = 0;  // lane 63's output of the even step, stored with the odd one
    // column codes from the LDS copy staged a tick ahead (no memory latency in the loop)
    const uint32_t* src = c.bring + ((((uintptr_t)first & ~(uintptr_t)3) - c.bbase) >> 2);
    const uint32_t sh = (uint32_t)((uintptr_t)first & 3);
    uint32_t lo = src[0], hi = src[1];
    const int4* in4 = reinterpret_cast<const int4*>(c.in_cd);
    int4 nx0 = in4[0], nx1 = in4[1];
    // matrix scoring: profile reads one group ahead, their code dwords two (see run_tick)
    uint32_t hi2 = PROT ? src[2] : 0;
    ScoreGroup<R, PROT> sg_next;
    if (PROT) sg_next.load(s.T, __builtin_amdgcn_alignbyte(hi, lo, sh), c);
#pragma unroll 2
    for (int gi = 0; gi < kTick / 4; ++gi) {
        const uint32_t cw = __builtin_amdgcn_alignbyte(hi, lo, sh);
        lo = hi;
        if (PROT) {
            hi = hi2;
            hi2 = src[gi + 3];
        } else {
            hi = src[gi + 2];
        }
        const int2 ins[4] = {make_int2(nx0.x, nx0.y), make_int2(nx0.z, nx0.w), make_int2(nx1.x, nx1.y),
                             make_int2(nx1.z, nx1.w)};
        nx0 = in4[2 * gi + 2];
        nx1 = in4[2 * gi + 3];
        ScoreGroup<R, PROT> sg;
        if (PROT) {
            sg = sg_next;
            sg_next.load(s.T, __builtin_amdgcn_alignbyte(hi, lo, sh), c);
        } else {
            sg.load(s.T, cw, c);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int m = 4 * gi + i;
            const int upH = dpp_shr1(ins[i].x, s.hl);
            const int upG = dpp_shr1(ins[i].y, s.gl);
            int diag = s.hup;
            s.hup = upH;
            int F = upG;
            if (TRACKMAX) acc += ext;
#pragma unroll
            for (int k = 0; k < R; ++k) {
                const int Hd = diag + sg.get(i, k);
                const int En = LOCAL ? max(max(s.E[k], HA[k]), z) : max(s.E[k], HA[k]);
                const int Hn = max(max(Hd, En), F);
                const int HAn = Hn - g;
                F = max(F, HAn) - ext;
                diag = s.H[k];
                s.H[k] = Hn;
                s.E[k] = En;
                HA[k] = HAn;
                if (TRACKMAX) acc = max(acc, Hn);
            }
            s.hl = s.H[R - 1];
            s.gl = F;
            if (i & 1) {  // lane 63's outputs of two steps in one store
                if (c.lane == kWave - 1)
                    *reinterpret_cast<int4*>(c.out + m - 1) = make_int4(ohl, ogl, s.hl, s.gl);
            } else {
                ohl = s.hl;
                ogl = s.gl;
            }
            z += ext;
        }
    }
    const int back = (kTick - 1 - c.lane) * ext;  // offset of step 63
#pragma unroll
    for (int k = 0; k < R; ++k) {
        s.H[k] -= back;
        s.E[k] -= back;
        s.HA[k] = s.H[k] - c.open;
    }
    s.hup -= back;
    s.hl -= back;
    s.gl -= back;
    return TRACKMAX ? acc - back : kNeg;
}

// Shifted tick in the row-and-column-shifted domain (R = 4 or 8 rows per lane).
// Cell (stripe row r, tick column t) carries (r + t) * ext on top of its value, so
// the extension of E along a row and of F down a column are both absorbed:
// E' = max(E', H' - g) and F' = max(F', H' - g) with g = open - ext, one maximum
// each and the same H' - g for both.  The diagonal step moves one row and one
// column, so the score bytes hold s + 2 ext.  Lane l's rows are stripe rows lR..
// lR + R - 1, so the values passed between lanes need no adjustment; lane 0's H
// from the row above enters with -ext (stripe row -1), and lane 63's outputs carry
// rows 64R - 1 (H) and 64R (F), which the caller removes.  The local zero of row k
// at step m is the row-0 zero of step m + k: the R zeros in use sit in a window of
// registers, and each step advances the one it has finished with by R steps.  The
// window's index is a compile-time constant because R divides the 8 steps of the
// unrolled body.  The running maximum uses the same fact: every cell of one
// anti-diagonal carries the same shift, so each cell is folded into the maximum of
// its anti-diagonal, kept in a second window of R registers that advances with the
// first; the shifts are taken off once, after the tick.
template <int R, bool TRACKMAX, bool LOCAL, bool PROT>
__device__ __forceinline__ int run_tick_rs(WaveState<R>& s, const uint8_t* first, const TickCtx& c) {
    static_assert(8 % R == 0, "the zero window needs R to divide the 8 steps of the unrolled body");
    const int ext = c.ext, g = c.open - c.ext;
    const int rbase = c.lane * R;                // stripe row of the lane's first row
    const int off = (rbase - c.lane - 1) * ext;  // the carried state belongs to step -1
    int HA[R];
#pragma unroll
    for (int k = 0; k < R; ++k) {
        s.H[k] += off + k * ext;
        s.E[k] += off + k * ext;
        HA[k] = s.H[k] - g;
    }
    s.hup += off - ext;            // stripe row rbase - 1
    s.hl += off + (R - 1) * ext;   // stripe row rbase + R - 1
    s.gl += off + R * ext;         // F entering stripe row rbase + R
    int zw[R];                     // zw[j]: zero of row 0 at the window's step congruent to j mod R
#pragma unroll
    for (int j = 0; j < R; ++j) zw[j] = (rbase - c.lane + j) * ext;
    const int zstep = R * ext;
    int aw[R];             // aw[j]: largest shifted H on the window's anti-diagonal congruent to j mod R
#pragma unroll
    for (int j = 0; j < R; ++j) aw[j] = kNeg;
    int ohl = 0, ogl = 0;  // lane 63's output of the even step, stored with the odd one
    const uint32_t* src = c.bring + ((((uintptr_t)first & ~(uintptr_t)3) - c.bbase) >> 2);
    const uint32_t sh = (uint32_t)((uintptr_t)first & 3);
    uint32_t lo = src[0], hi = src[1];
    const int4* in4 = reinterpret_cast<const int4*>(c.in_cd);
    int4 nx0 = in4[0], nx1 = in4[1];
    uint32_t hi2 = PROT ? src[2] : 0;
    ScoreGroup<R, PROT> sg_next;
    if (PROT) sg_next.load(s.T, __builtin_amdgcn_alignbyte(hi, lo, sh), c);
    for (int g2 = 0; g2 < kTick / 8; ++g2) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int gi = 2 * g2 + h;
            const uint32_t cw = __builtin_amdgcn_alignbyte(hi, lo, sh);
            lo = hi;
            if (PROT) {
                hi = hi2;
                hi2 = src[gi + 3];
            } else {
                hi = src[gi + 2];
            }
            const int2 ins[4] = {make_int2(nx0.x, nx0.y), make_int2(nx0.z, nx0.w), make_int2(nx1.x, nx1.y),
                                 make_int2(nx1.z, nx1.w)};
            nx0 = in4[2 * gi + 2];
            nx1 = in4[2 * gi + 3];
            ScoreGroup<R, PROT> sg;
            if (PROT) {
                sg = sg_next;
                sg_next.load(s.T, __builtin_amdgcn_alignbyte(hi, lo, sh), c);
            } else {
                sg.load(s.T, cw, c);
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int m = 4 * gi + i;
                const int j0 = (4 * h + i) % R;  // m mod R
                const int upH = dpp_shr1(ins[i].x, s.hl);
                const int upG = dpp_shr1(ins[i].y, s.gl);
                int diag = s.hup;
                s.hup = upH;
                int F = upG;
#pragma unroll
                for (int k = 0; k < R; ++k) {
                    const int Hd = diag + sg.get(i, k);
                    const int En = LOCAL ? max(max(s.E[k], HA[k]), zw[(j0 + k) % R]) : max(s.E[k], HA[k]);
                    const int Hn = max(max(Hd, En), F);
                    const int HAn = Hn - g;
                    F = max(F, HAn);
                    diag = s.H[k];
                    s.H[k] = Hn;
                    s.E[k] = En;
                    HA[k] = HAn;
                    if (TRACKMAX) aw[(j0 + k) % R] = max(aw[(j0 + k) % R], Hn);
                }
                // anti-diagonal m is complete: its slot moves on to anti-diagonal m + R
                if (LOCAL) zw[j0] += zstep;
                if (TRACKMAX) aw[j0] += zstep;
                s.hl = s.H[R - 1];
                s.gl = F;
                if (i & 1) {
                    if (c.lane == kWave - 1)
                        *reinterpret_cast<int4*>(c.out + m - 1) = make_int4(ohl, ogl, s.hl, s.gl);
                } else {
                    ohl = s.hl;
                    ogl = s.gl;
                }
            }
        }
    }
    const int back = (kTick - 1 - c.lane) * ext;  // column shift of step 63
#pragma unroll
    for (int k = 0; k < R; ++k) {
        s.H[k] -= back + (rbase + k) * ext;
        s.E[k] -= back + (rbase + k) * ext;
        s.HA[k] = s.H[k] - c.open;
    }
    s.hup -= back + (rbase - 1) * ext;
    s.hl -= back + (rbase + R - 1) * ext;
    s.gl -= back + (rbase + R) * ext;
    if (!TRACKMAX) return kNeg;
    // after step 63 slot j holds anti-diagonal 64 + j (R divides 64), whose cells
    // carry (rbase - lane + 64 + j) * ext
    int tmax = kNeg;
#pragma unroll
    for (int j = 0; j < R; ++j) tmax = max(tmax, aw[j] - (rbase - c.lane + kTick + j) * ext);
    return tmax;
}

// CD: fast ticks run in a shifted domain (run_tick_rs for R = 4 and 8,
// run_tick_cd for R = 6); needs match + 2 ext (R = 4, 8) or match + ext (R = 6)
// <= 127 so that the shifted scores fit the score bytes.
// OCC: resident waves per SIMD the register allocation is sized for
// (512 / OCC VGPRs per lane).
// PROT: matrix scoring; the query profile takes p.sub.n_class * 64 * (4 or 8)
// bytes of dynamic LDS.
// K: waves per workgroup.  K = 1: every wave takes its own tickets.  K > 1 (a
// chain workgroup, global recurrence only): the workgroup takes K consecutive
// tickets at a time, wave w the w-th, and waves whose producer is the previous
// wave read their top border from that wave's LDS ring.
template <int R, bool LOCAL, bool CD, int OCC, bool PROT, int K>
__device__ __forceinline__ void engine_body(const EngineArgs& p) {
    static_assert(K == 1 || (!LOCAL && !PROT), "chain workgroups run the global recurrence with DNA scores");
    __shared__ __attribute__((aligned(16))) int2 in_ring_w[K][2][kTick + 4];
    __shared__ __attribute__((aligned(16))) int2 in_ring_cd_w[K][CD ? 2 : 1][kTick + 4];
    // Column codes of a tick: lane l reads from column col0 - l on, 18 dwords (19
    // with matrix scoring, at most index 34); the union over lanes is kBring dwords
    // from the dword holding column col0 - 63.
    constexpr int kBring = 36;
    __shared__ uint32_t b_ring_w[K][CD ? 2 : 1][kBring];
    // Row maxima and the pre-tick snapshot live in LDS (one column per lane) so
    // that the hot loop's registers hold only the recurrence.
    // Matrix scoring at 2 waves per SIMD keeps them in registers instead (16 of the
    // 256 VGPRs at R = 8): the LDS that frees lets the query profile fit 8 waves per CU.
    constexpr bool kRbRegs = PROT && OCC <= 2;
    __shared__ int lds_best_w[K][kRbRegs ? 1 : R][kWave], lds_pos_w[K][kRbRegs ? 1 : R][kWave];
    __shared__ int lds_snap_w[K][2 * R + 3][kWave];
    __shared__ __attribute__((aligned(16))) int2 out_buf_w[K][kTick];
    // Chain links: wave w's bottom row for wave w + 1 (column c at c mod kRing), the
    // columns published, the columns the reader is done with, H at the band's left
    // column; and the group's first ticket.
    constexpr int KL = K > 1 ? K : 1;
    __shared__ __attribute__((aligned(16))) int2 link_ring[KL][K > 1 ? kRing : 1];
    __shared__ int link_cnt[KL], link_used[KL], link_diag[KL];
    __shared__ uint32_t grp_first;
    // Query profile (matrix scoring): entry (class c, lane l) at dword (c * 64 + l) * kPW
    // holds s(row, c) + bias for the R rows of lane l, one byte per row (-128 for
    // rows past the matrix and for the padding class).
    extern __shared__ __attribute__((aligned(16))) uint32_t prof_lds[];
    constexpr int kPW = R > 4 ? 2 : 1;
    constexpr int NEGV = LOCAL ? 0 : kNeg;  // value of an unreachable cell in the recurrence in use
    constexpr int kRs = (CD && cd_row_shift(R)) ? 1 : 0;  // shifted ticks also shift by the stripe row
    const int lane = K > 1 ? (int)(threadIdx.x & (kWave - 1)) : (int)threadIdx.x;
    const int wv = K > 1 ? (int)__builtin_amdgcn_readfirstlane(threadIdx.x / kWave) : 0;
    auto& in_ring = in_ring_w[wv];
    auto& in_ring_cd = in_ring_cd_w[wv];
    auto& b_ring = b_ring_w[wv];
    auto& lds_best = lds_best_w[wv];
    auto& lds_pos = lds_pos_w[wv];
    auto& lds_snap = lds_snap_w[wv];
    auto& out_buf = out_buf_w[wv];

    for (;;) {
        int64_t task;
        if constexpr (K == 1) {
            uint32_t tk = 0;
            if (lane == 0) tk = atomicAdd(p.ticket, 1u);
            task = (int64_t)__builtin_amdgcn_readfirstlane(tk);  // the ticket
            if (task >= p.n_tickets) break;
        } else {
            // Group start: the first ticket, and links reset (the previous group's
            // waves all passed the closing barrier below).
            if (threadIdx.x == 0) grp_first = atomicAdd(p.ticket, (uint32_t)K);
            if (lane == 0) {
                link_cnt[wv] = 0;
                link_used[wv] = 0;
            }
            __syncthreads();
            const int64_t first = (int64_t)grp_first;
            if (first >= p.n_tickets) break;  // the same for every wave of the group
            task = first + wv;
        }
        if (K == 1 || task < p.n_tickets) {
        jitter_pause(p.jitter, task, -1);
        const Ticket tkt = p.tickets[task];
        const int64_t pi = tkt.pi;
        const Prob pr = p.probs[pi];
        const int64_t t = tkt.local;
        const int64_t band = t / pr.Q;
        const int64_t q = t - band * pr.Q;
        const int64_t c0 = band * pr.W;
        const int W = (int)min(pr.W, pr.N - c0);
        const int n_ticks = (W + 2 * kTick - 2) / kTick;  // ceil((W + 63) / 64)
        const int64_t R0 = q * (int64_t)(kWave * R);
        const int64_t R1 = min(R0 + (int64_t)(kWave * R), pr.M);
        const int64_t row0 = R0 + (int64_t)lane * R;
        const bool capture = band + 1 < pr.n_bands;
        const uint8_t* acodes = p.a_codes + pr.a_off;
        const uint8_t* bcodes = p.b_codes + pr.b_off;
        int2* lbuf = p.lbuf + pr.lbuf_off;
        // Neighbour tasks without a ticket hold no cell of the kept band: their
        // values are -inf (the ticket table says which exist).
        const bool prod_active = tkt.prod >= 0;
        const bool left_active = tkt.left >= 0;
        int2* my_slot = p.slots + (task % p.nslot) * p.slot_stride;
        const int2* prod_slot = prod_active ? p.slots + ((int64_t)tkt.prod % p.nslot) * p.slot_stride : nullptr;
        const int32_t* prod_prog = p.progress + (prod_active ? tkt.prod : 0);
        int32_t prod_seen = 0;
        int32_t* gbest = p.gbest + pi;
        // Chain links (wave-uniform): the producer is the previous wave of the group
        // (read its LDS ring), the consumer is the next one (write this wave's ring).
        const bool link_in = K > 1 && prod_active && wv > 0 && (int64_t)tkt.prod == task - 1;
        const bool link_out = K > 1 && wv + 1 < K && tkt.cons >= 0 && (int64_t)tkt.cons == task + 1;
        int link_room = 0;  // the reader's done count, last read (link_out)
        // Global recurrence: the task runs only its ticks [tau_lo, tau_hi] that hold a
        // cell of the kept band (the others would be skipped: their cells are -inf;
        // last-row outputs outside them keep the -inf the caller filled in).  The
        // producer's ticks bound what it writes: its columns outside
        // [prod_first, prod_lim] read -inf (and are not waited for).
        const bool has_out = pr.out_off >= 0 && q == pr.Q - 1;
        // Slots of the global recurrence hold a task's written columns only, from its
        // first (slot_first here, prod_first in the producer's slot).
        int tau_lo = 0, tau_hi = n_ticks - 1;
        int prod_first = 0, prod_lim = INT32_MAX - 1, slot_first = 0;
        if constexpr (!LOCAL) {
            band_ticks(pr, R0, c0, R, n_ticks, tau_lo, tau_hi);
            if (tau_lo > tau_hi) {  // no tick holds a band cell (cannot happen for a ticket)
                tau_lo = 0;
                tau_hi = n_ticks - 1;
            }
            int last;
            slot_columns(tau_lo, tau_hi, slot_first, last);
            if (prod_active) {
                int plo, phi;
                band_ticks(pr, R0 - (int64_t)kWave * R, c0, R, n_ticks, plo, phi);
                if (plo <= phi) slot_columns(plo, phi, prod_first, prod_lim);
            }
        }

        // Older tickets this one depends on.  Slot reuse: the previous owner of the
        // slot must have finished writing it, and that owner's reader (if the
        // owner is not the last stripe of its band) finished reading it.  The
        // owner itself is not implied by its reader's completion: the reader can
        // finish only after the owner's last column, but a last stripe has no
        // reader at all.
        if (task >= p.nslot) {
            int32_t seen = 0;
            wait_at_least(p.progress + task - p.nslot, kDone, seen, p.abort_flag, p.wait_limit);
            if (tkt.reuse_reader >= 0) {
                seen = 0;
                wait_at_least(p.progress + tkt.reuse_reader, kDone, seen, p.abort_flag, p.wait_limit);
            }
        }
        if (left_active) {
            int32_t seen = 0;
            wait_at_least(p.progress + tkt.left, kDone, seen, p.abort_flag, p.wait_limit);
        }

        WaveState<R> s;
        RowBest<R> rb_regs;  // kRbRegs: the row maxima between ticks
        const int M_rows = (int)max((int64_t)0, min((int64_t)R, pr.M - row0));
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const int64_t row = row0 + k;
            int code = PROT ? 0xff : kPadCode;  // rows past the matrix score -128
            int h = NEGV, e = NEGV;
            if (row < pr.M) {
                code = acodes[row];
                if (tau_lo > 0) {  // the ticks left of the band are not run: their cells are -inf
                    h = kNeg;
                    e = kNeg;
                } else if (band == 0) {
                    h = border_h(pr.left_kind, pr.left_open, p.ext, row + 1);
                } else if (left_active) {
                    const int2 lb = ld_shared_i2(lbuf + row);
                    h = lb.x;
                    e = lb.y;
                } else {
                    h = kNeg;
                    e = kNeg;
                }
            }
            s.T[k] = PROT ? (uint32_t)code : row_table(code, p.match, p.mismatch, CD ? cd_bias_ext(R) * p.ext : 0);
            s.H[k] = h;
            s.E[k] = e;
            s.HA[k] = h - p.open;
            if constexpr (kRbRegs) {
                rb_regs.best[k] = LOCAL ? 0 : kNeg;
                rb_regs.pos[k] = -1;
            } else {
                lds_best[k][lane] = LOCAL ? 0 : kNeg;
                lds_pos[k][lane] = -1;
            }
        }
        if (PROT) {
            // This task's query profile.  Each lane writes and later reads only its
            // own entries, so no barrier is needed; the row codes were parked in T.
            const int nc = p.sub.n_class;
            const int bias = CD ? cd_bias_ext(R) * p.ext : 0;
            for (int cl = 0; cl < nc; ++cl) {
                uint32_t w[kPW];
#pragma unroll
                for (int d = 0; d < kPW; ++d) w[d] = 0;
#pragma unroll
                for (int k = 0; k < R; ++k) {
                    const uint32_t rc = s.T[k];
                    const int sv = p.sub.s[min(rc, (uint32_t)(kMaxClasses - 1))][cl];
                    const int v = (rc >= (uint32_t)(nc - 1) || cl == nc - 1) ? -128 : sv + bias;
                    w[k >> 2] |= (uint32_t)(uint8_t)(int8_t)v << (8 * (k & 3));
                }
                uint32_t* e = prof_lds + ((uint32_t)cl * kWave + (uint32_t)lane) * kPW;
                if (kPW == 2) *reinterpret_cast<uint2*>(e) = make_uint2(w[0], w[kPW - 1]);
                else e[0] = w[0];
            }
        }
        s.hup = 0;
        s.hl = s.H[R - 1];
        s.gl = NEGV;
        // H(last row of this stripe, band's left column) for the stripe below.
        if (link_out) {
            if (lane == kWave - 1) lds_store(&link_diag[wv], s.H[R - 1]);
            // The reader needs no column left of its first tick (less one): until it
            // has read, the ring may hold this wave's columns up to that one + kRing - 1.
            int clo, chi;
            band_ticks(pr, R0 + (int64_t)kWave * R, c0, R, n_ticks, clo, chi);
            if (lane == 0) lds_store(&link_used[wv], clo > chi ? 0 : max(0, kTick * clo - 1));
            // The corner is written, and columns left of this wave's first tick are
            // settled (-inf: the reader does not read them).
            asm volatile("" ::: "memory");
            if (lane == 0) lds_store(&link_cnt[wv], max(1, kTick * tau_lo - (kTick - 1)));
        } else if (lane == kWave - 1) {
            st_shared_i2(my_slot + kSlotPad - 1, make_int2(s.H[R - 1], 0));
        }

        // Last-row outputs (reconstruction halves): lane and sub-row of row M-1.
        if (has_out && band == 0 && lane == 0) {
            const int h = border_h(pr.left_kind, pr.left_open, p.ext, pr.M);
            p.out_h[pr.out_off] = h;
            p.out_f[pr.out_off] = h;
        }

        // Inputs of a tick: the row above the stripe at band columns [base, base + 64).
        auto fetch = [&](int base, int need) -> int2 {
            const int rel = base + lane;
            if (rel >= W) return make_int2(NEGV, NEGV);
            if (q == 0) {
                if (pr.top_kind == BORDER_BUF) {
                    // a row of a larger matrix: H and F there give the next row's F-candidate
                    const int h = p.top_h[pr.top_off + c0 + rel + 1];
                    const int f = p.top_f[pr.top_off + c0 + rel + 1];
                    return make_int2(h, max(f - p.ext, h - p.open));
                }
                const int h = border_h(pr.top_kind, pr.top_open, p.ext, c0 + rel + 1);
                if (pr.top_kind == BORDER_GAP) return make_int2(h, h - p.open);
                return make_int2(h, LOCAL ? 0 : kNeg);
            }
            if (!prod_active) return make_int2(kNeg, kNeg);
            if constexpr (!LOCAL) {
                const bool written = rel >= prod_first && rel <= prod_lim;  // else outside the producer's ticks
                need = min(need, prod_lim + 1);
                if (link_in) {
                    int2 v = make_int2(kNeg, kNeg);
                    if (written) {
                        lds_wait_at_least(&link_cnt[wv - 1], need, prod_seen, p.abort_flag, p.wait_limit);
                        v = link_ring[wv - 1][rel & (kRing - 1)];  // rel >= 0
                    }
                    asm volatile("" ::: "memory");
                    // columns below base + 64 are read (LDS executes this wave's accesses
                    // in order); lane 0 holds the smallest column and is active here
                    if (lane == 0) lds_store(&link_used[wv - 1], min(base + kTick, W));
                    return v;
                }
                if (!written) return make_int2(kNeg, kNeg);
            }
            wait_at_least(prod_prog, need, prod_seen, p.abort_flag, p.wait_limit);
            return ld_shared_i2(prod_slot + kSlotPad + (rel - prod_first));
        };
        // H of the row above the stripe at band column rel (0 <= rel < W).
        auto above_h = [&](int rel) -> int {
            if (q == 0) {
                if (pr.top_kind == BORDER_BUF) return p.top_h[pr.top_off + c0 + rel + 1];
                return border_h(pr.top_kind, pr.top_open, p.ext, c0 + rel + 1);
            }
            if (!prod_active || rel < prod_first || rel > prod_lim) return kNeg;
            if (link_in) {
                lds_wait_at_least(&link_cnt[wv - 1], rel + 1, prod_seen, p.abort_flag, p.wait_limit);
                return link_ring[wv - 1][rel & (kRing - 1)].x;
            }
            wait_at_least(prod_prog, rel + 1, prod_seen, p.abort_flag, p.wait_limit);
            return ld_shared_i2(prod_slot + kSlotPad + (rel - prod_first)).x;
        };
        {
            int h_diag = 0;
            if (tau_lo > 0) {
                // lane 0's first diagonal: the row above at the column left of the first tick
                const int rd = kTick * tau_lo - 1;
                h_diag = rd < W ? above_h(rd) : NEGV;
            } else if (q == 0) {
                if (pr.top_kind == BORDER_BUF) h_diag = p.top_h[pr.top_off + c0];
                else h_diag = c0 == 0 ? 0 : border_h(pr.top_kind, pr.top_open, p.ext, c0);
            } else if (link_in) {
                lds_wait_at_least(&link_cnt[wv - 1], 1, prod_seen, p.abort_flag, p.wait_limit);
                h_diag = lds_load(&link_diag[wv - 1]);
            } else if (prod_active) {
                wait_at_least(prod_prog, 1, prod_seen, p.abort_flag, p.wait_limit);
                h_diag = ld_shared_i2(prod_slot + kSlotPad - 1).x;
            } else if (band == 0) {
                h_diag = border_h(pr.left_kind, pr.left_open, p.ext, R0);
            } else if (tkt.corner >= 0) {
                // H(R0 - 1, c0 - 1): the last column of the previous band, captured by
                // the task above-left (no task of that stripe after it writes the row)
                int32_t seen = 0;
                wait_at_least(p.progress + tkt.corner, kDone, seen, p.abort_flag, p.wait_limit);
                h_diag = ld_shared_i2(lbuf + R0 - 1).x;
            } else {
                h_diag = kNeg;
            }
            const int2 v = fetch(kTick * tau_lo, min(kTick * (tau_lo + 1), W));
            in_ring[0][lane] = v;
            if (CD) in_ring_cd[0][lane] = make_int2(v.x + (lane - kRs) * p.ext, v.y + lane * p.ext);
            if (CD && lane < kBring)
                b_ring[0][lane] = reinterpret_cast<const uint32_t*>(
                    ((uintptr_t)(bcodes + c0 + (int64_t)kTick * tau_lo - (kTick - 1)) & ~(uintptr_t)3))[lane];
            if (lane == 0) s.hup = h_diag;
        }
        wave_sync<K>();

        TickCtx c;
        c.prof = prof_lds + (uint32_t)lane * kPW;
        c.out = out_buf;
        c.lbuf = lbuf;
        c.out_h = p.out_h;
        c.out_f = p.out_f;
        c.row0 = row0;
        c.out_base = pr.out_off + c0 + 1;
        c.lane = lane;
        c.W = W;
        c.M_rows = M_rows;
        c.open = p.open;
        c.ext = p.ext;
        c.capture = capture;
        c.out_lane = -1;
        c.out_k = -1;
        if (has_out) {
            c.out_lane = (int)((pr.M - 1 - R0) / R);
            c.out_k = (int)((pr.M - 1 - R0) % R);
        }
        unsigned long long pruned = 0;
        // The producer's column count and the running best are read one tick
        // ahead and consumed a tick later, so no tick starts with a round trip
        // to memory.  Both only grow: a value one tick old is a valid lower bound.
        const bool polls = q > 0 && prod_active;
        int32_t prod_pf = 0;
        // Issue priority on the SIMD (local recurrence only): a stripe whose
        // consumer is within a few ticks of its output, and so likely waiting
        // for it, runs at a raised priority.  The chain's slowest link is then
        // less often the younger wave of a shared SIMD.  A hint only: the
        // consumer's count is never waited on.  The banded global passes keep
        // plain arbitration (there the raised priority measured slower).
        const bool has_cons = LOCAL && tkt.cons >= 0;
        const int32_t* cons_prog = p.progress + (has_cons ? tkt.cons : 0);
        int32_t cons_pf = 0;
        // The stripe's best recorded value and the first stripe row holding it
        // (wave-uniform; from exact row maxima only).
        int sb = LOCAL ? 0 : kNeg;
        int sb_row = 0;
        int gb_pf = __hip_atomic_load(gbest, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);

        const int tau_end = tau_hi + 1;
        for (int tau = tau_lo; tau < tau_end; ++tau) {
            const int cur = (tau - tau_lo) & 1;
            prod_seen = max(prod_seen, prod_pf);
            if (link_in) prod_seen = max(prod_seen, lds_load(&link_cnt[wv - 1]));  // an LDS read: no prefetch
            if (!LOCAL) prod_seen = __builtin_amdgcn_readfirstlane(prod_seen);
            // The next tick's inputs are loaded now, their latency hidden behind this
            // tick.  The banded global passes run as a chain of stripes each right
            // behind its producer: there, if the producer is not far enough yet,
            // they are loaded after this tick instead, so a stripe trails its
            // producer by two ticks, not three (the local passes keep the early
            // load: a late one would expose its latency).
            int2 nxt = make_int2(NEGV, NEGV);
            const int need_nxt = min(kTick * (tau + 2), W);
            const bool nxt_now = tau + 1 < tau_end && (LOCAL || !polls || prod_seen >= need_nxt);
            if (nxt_now) nxt = fetch(kTick * (tau + 1), need_nxt);
            uint32_t b_next = 0;  // next tick's column codes (staged at the end of this tick)
            if (CD && tau + 1 < tau_end && lane < kBring)
                b_next = reinterpret_cast<const uint32_t*>(
                    ((uintptr_t)(bcodes + c0 + (int64_t)kTick * (tau + 1) - (kTick - 1)) & ~(uintptr_t)3))[lane];
            if (polls && !link_in && tau + 2 < tau_end) prod_pf = load_count(prod_prog);
            if (has_cons) cons_pf = load_count(cons_prog);
            const uint8_t* cols = bcodes + c0 + (int64_t)kTick * tau - lane;

            const int gb = gb_pf;
            gb_pf = __hip_atomic_load(gbest, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const int L = max(gb, pr.target);
            const bool slow = (tau == 0) || has_out ||
                              (capture && kTick * tau - (kTick - 1) <= W - 1 && W - 1 <= kTick * tau + (kTick - 1));
            c.in = in_ring[cur];
            c.in_cd = in_ring_cd[CD ? cur : 0];
            c.bring = b_ring[CD ? cur : 0];
            c.bbase = (uintptr_t)(bcodes + c0 + (int64_t)kTick * tau - (kTick - 1)) & ~(uintptr_t)3;
            c.col0 = c0 + (int64_t)kTick * tau;
            c.rel0 = kTick * tau;

            bool skip = false;
            // Can a cell of this tick reach L?  Its H is at most the largest H on the
            // tick's borders (or 0, where a local path starts) plus match per aligned
            // pair, and the tick spans 127 columns.  If not, the shifted tick runs
            // without its running maximum.
            bool track_max = true;
            if (!slow) {
                // diagonal band (global recurrence)
                const int64_t dmax = c.col0 + (kTick - 1) - R0;
                const int64_t dmin = c.col0 - R0 - (int64_t)kWave * R - (kTick - 2);
                if (dmax < pr.d_lo || dmin > pr.d_hi) skip = true;
                if (!skip && (pr.prune || CD)) {
                    int hm = max(s.hup, in_ring[cur][lane].x);
#pragma unroll
                    for (int k = 0; k < R; ++k) hm = max(hm, s.H[k]);
                    hm = wave_max(hm);
                    if (LOCAL) hm = max(hm, 0);
                    if (pr.prune) {
                        const int64_t rows_left = pr.M + pr.rows_after - R0;
                        const int64_t cols_left = pr.N - (c.col0 - (kTick - 1));
                        const int64_t ub = (int64_t)hm + (int64_t)p.match * min(rows_left, cols_left);
                        skip = ub < (int64_t)L;
                    }
                    track_max = (int64_t)hm + (int64_t)p.match * (2 * kTick - 1) >= (int64_t)L;
                }
            }

            auto load_rb = [&](RowBest<R>& rb) {
                if constexpr (kRbRegs) {
                    rb = rb_regs;
                } else {
#pragma unroll
                    for (int k = 0; k < R; ++k) {
                        rb.best[k] = lds_best[k][lane];
                        rb.pos[k] = lds_pos[k][lane];
                    }
                }
            };
            auto store_rb = [&](const RowBest<R>& rb) {
                if constexpr (kRbRegs) {
                    rb_regs = rb;
                } else {
#pragma unroll
                    for (int k = 0; k < R; ++k) {
                        lds_best[k][lane] = rb.best[k];
                        lds_pos[k][lane] = rb.pos[k];
                    }
                }
            };
            auto snapshot = [&]() {
#pragma unroll
                for (int k = 0; k < R; ++k) {
                    lds_snap[k][lane] = s.H[k];
                    lds_snap[R + k][lane] = s.E[k];
                }
                lds_snap[2 * R][lane] = s.hup;
                lds_snap[2 * R + 1][lane] = s.hl;
                lds_snap[2 * R + 2][lane] = s.gl;
            };
            auto restore = [&]() {
#pragma unroll
                for (int k = 0; k < R; ++k) {
                    s.H[k] = lds_snap[k][lane];
                    s.E[k] = lds_snap[R + k][lane];
                    s.HA[k] = s.H[k] - p.open;
                }
                s.hup = lds_snap[2 * R][lane];
                s.hl = lds_snap[2 * R + 1][lane];
                s.gl = lds_snap[2 * R + 2][lane];
            };
            // Best of the rows that may hold the answer, into the problem's running best.
            auto publish_best = [&](const RowBest<R>& rb, const bool (&want)[R]) {
                int mx = kNeg;
#pragma unroll
                for (int k = 0; k < R; ++k)
                    if (want[k] && k < M_rows) mx = max(mx, rb.best[k]);
                mx = wave_max(mx);
                if (lane == 0 && mx > gb) atomicMax(gbest, mx);
            };

            // After row maxima changed: the stripe's best and its first row.
            auto refresh_sb = [&](const RowBest<R>& rb) {
                int v = kNeg, r = INT32_MAX;
#pragma unroll
                for (int k = 0; k < R; ++k)
                    if (k < M_rows && rb.best[k] > v) {
                        v = rb.best[k];
                        r = lane * R + k;
                    }
                const int vm = wave_max(v);
                const unsigned long long bal = __ballot(v == vm);
                sb = vm;
                sb_row = __shfl(r, __ffsll((long long)bal) - 1);
            };

            // Untracked problems (halves of the reconstruction) need no maxima at all.
            if (!pr.track) track_max = false;
            const bool cd_tick = CD && !skip && !slow;
            if (skip) {
                pruned += (unsigned long long)kTick * kWave * R;
#pragma unroll
                for (int k = 0; k < R; ++k) {
                    s.H[k] = NEGV;
                    s.E[k] = NEGV;
                    s.HA[k] = NEGV - p.open;
                }
                // lane 0's next diagonal is the row above at this tick's last column,
                // which lies outside the skipped tile
                s.hup = lane == 0 ? in_ring[cur][kTick - 1].x : NEGV;
                s.hl = NEGV;
                s.gl = NEGV;
                out_buf[lane] = make_int2(NEGV, NEGV);
            } else if (cd_tick) {
                if (track_max) snapshot();  // without the running maximum there is no replay
                int tmax;
                if constexpr (kRs) {
                    tmax = track_max ? run_tick_rs<R, true, LOCAL, PROT>(s, cols, c)
                                     : run_tick_rs<R, false, LOCAL, PROT>(s, cols, c);
                } else {
                    tmax = track_max ? run_tick_cd<R, true, LOCAL, PROT>(s, cols, c)
                                     : run_tick_cd<R, false, LOCAL, PROT>(s, cols, c);
                }
                if (pr.target > 0 && track_max) {
                    // Under an external target, ticks below it are not replayed; keep the
                    // largest H seen in the running best (a valid lower bound of the optimum)
                    // so that a missed target still reports it.
                    const int wm = wave_max(tmax);
                    if (lane == 0 && wm > gb) atomicMax(gbest, wm);
                }
                // The tick is replayed to find row maxima and their first columns when a
                // lane's maximum reached max(running best, target) and either beats the
                // stripe's best or ties it in a row before the one holding it.  Any cell
                // that can be the lexicographically first of the optimum passes both
                // tests; ties in later rows cannot win and are not replayed.
                const bool need = tmax >= L && (tmax > sb || (tmax == sb && lane * R < sb_row));
                if (__any(need)) {
                    restore();
                    bool want[R];
#pragma unroll
                    for (int k = 0; k < R; ++k) want[k] = true;
                    RowBest<R> rb;
                    load_rb(rb);
                    run_tick<R, LOCAL, kExact, false, CD, PROT>(s, rb, cols, c, want);
                    store_rb(rb);
                    publish_best(rb, want);
                    refresh_sb(rb);
                }
            } else {
                RowBest<R> rb;
                load_rb(rb);
                int bstart[R];
#pragma unroll
                for (int k = 0; k < R; ++k) bstart[k] = rb.best[k];
                if (pr.track) snapshot();
                bool want[R];
#pragma unroll
                for (int k = 0; k < R; ++k) want[k] = false;
                // Shifted-domain builds take this path only for slow ticks (and, in
                // principle, untracked problems): the predicated form serves both
                // and keeps the fast plain loop out of those builds.
                if (slow || CD) run_tick<R, LOCAL, kRun, true, CD, PROT>(s, rb, cols, c, want);
                else run_tick<R, LOCAL, kRun, false, CD, PROT>(s, rb, cols, c, want);

                if (pr.track) {
                    bool any = false;
#pragma unroll
                    for (int k = 0; k < R; ++k) {
                        const bool inc = rb.best[k] > bstart[k];
                        want[k] = inc && rb.best[k] >= L;
                        if (inc) rb.pos[k] = -1;
                        any = any || want[k];
                    }
                    if (__any(any)) {
                        // Replay from the snapshot; the replay ends in the same state.
                        restore();
                        if (slow || CD) run_tick<R, LOCAL, kTrack, true, CD, PROT>(s, rb, cols, c, want);
                        else run_tick<R, LOCAL, kTrack, false, CD, PROT>(s, rb, cols, c, want);
                        publish_best(rb, want);
                    }
                }
                store_rb(rb);
                if (CD) refresh_sb(rb);
            }

            // Hand the 64 bottom-row columns of this tick to the stripe below.
            wave_sync<K>();
            if (link_out) {
                // the ring slots of these columns must be read: the reader is done
                // with every column below kTick * tau - kRing + 1
                lds_wait_at_least(&link_used[wv], kTick * tau - kRing + 1, link_room, p.abort_flag, p.wait_limit);
                const int rel = kTick * tau - (kTick - 1) + lane;
                int2 o = out_buf[lane];
                if (cd_tick) {  // lane 63's step `lane` carried (lane - 63) * ext, plus its row shift
                    o.x -= (lane - (kTick - 1) + kRs * (kWave * R - 1)) * p.ext;
                    o.y -= (lane - (kTick - 1) + kRs * kWave * R) * p.ext;
                }
                if (rel >= 0) link_ring[wv][rel & (kRing - 1)] = o;
                jitter_pause(p.jitter, task, tau);
                asm volatile("" ::: "memory");
                if (lane == 0) lds_store(&link_cnt[wv], min(kTick * tau + 1, W));
            } else {
                {
                    const int rel = kTick * tau - (kTick - 1) + lane;
                    int2 o = out_buf[lane];
                    if (cd_tick) {  // lane 63's step `lane` carried (lane - 63) * ext, plus its row shift
                        o.x -= (lane - (kTick - 1) + kRs * (kWave * R - 1)) * p.ext;
                        o.y -= (lane - (kTick - 1) + kRs * kWave * R) * p.ext;
                    }
                    // (global recurrence: only a task with a consumer, only its columns)
                    if (rel >= 0 && (LOCAL || tkt.cons >= 0)) st_shared_i2(my_slot + kSlotPad + (rel - slot_first), o);
                }
                jitter_pause(p.jitter, task, tau);
                publish_count(p.progress + task, min(kTick * tau + 1, W));
            }
            if (has_cons) {
                const int32_t cs = __builtin_amdgcn_readfirstlane(cons_pf);
                if (cs > 0 && min(kTick * tau + 1, W) - cs <= 4 * kTick) __builtin_amdgcn_s_setprio(2);
                else __builtin_amdgcn_s_setprio(0);
            }
            if (!LOCAL && tau + 1 < tau_end && !nxt_now) {
                prod_seen = max(prod_seen, prod_pf);
                nxt = fetch(kTick * (tau + 1), need_nxt);
            }
            in_ring[cur ^ 1][lane] = nxt;
            if (CD) in_ring_cd[cur ^ 1][lane] = make_int2(nxt.x + (lane - kRs) * p.ext, nxt.y + lane * p.ext);
            if (CD && lane < kBring) b_ring[cur ^ 1][lane] = b_next;
            wave_sync<K>();
        }
        if constexpr (!LOCAL) {
            // The ticks not run count as skipped; a lane whose capture column lies in one
            // of them hands -inf to the next band.
            pruned += (unsigned long long)(n_ticks - (tau_end - tau_lo)) * kTick * kWave * R;
            const int tc = (W - 1 + lane) / kTick;
            if (capture && (tc < tau_lo || tc >= tau_end)) {
#pragma unroll
                for (int k = 0; k < R; ++k)
                    if (k < M_rows) st_shared_i2(lbuf + row0 + k, make_int2(kNeg, kNeg));
            }
        }

        // Task record: the stripe's best value, its smallest row, that row's first column.
        {
            int bv = kNeg, bk = 0, bp = -1;
#pragma unroll
            for (int k = 0; k < R; ++k) {
                if constexpr (kRbRegs) {
                    const int b = rb_regs.best[k];
                    if (k < M_rows && b > bv) {
                        bv = b;
                        bk = k;
                        bp = rb_regs.pos[k];
                    }
                } else {
                    const int b = lds_best[k][lane];
                    if (k < M_rows && b > bv) {
                        bv = b;
                        bk = k;
                        bp = lds_pos[k][lane];
                    }
                }
            }
            const int vmax = wave_max(bv);
            const unsigned long long bal = __ballot(bv == vmax);
            const int src = __ffsll((long long)bal) - 1;
            const int rk = __shfl(bk, src);
            const int rp = __shfl(bp, src);
            if (lane == 0) {
                TaskRec r;
                r.score = vmax;
                r.pad = 0;
                r.row = R0 + (int64_t)src * R + rk;
                r.col = rp;
                p.recs[pr.task0 + t] = r;
                if (pruned) atomicAdd(p.pruned + pi, pruned);
            }
        }
        publish_count(p.progress + task, kDone);
        __builtin_amdgcn_s_setprio(0);
        }
        if constexpr (K > 1) __syncthreads();  // group end: every wave is done with the links
    }
}

template <int R, bool LOCAL, bool CD, int OCC, bool PROT>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(OCC))) void engine_kernel(EngineArgs p) {
    engine_body<R, LOCAL, CD, OCC, PROT, 1>(p);
}

// The banded global passes (reverse pass, reconstruction halves) with K waves per
// workgroup linked through LDS; DNA scores in the shifted domain.
template <int R, int K, int OCC>
__global__ __launch_bounds__(64 * K) __attribute__((amdgpu_waves_per_eu(OCC))) void chain_kernel(EngineArgs p) {
    engine_body<R, false, true, OCC, false, K>(p);
}

// ------------------------------------------------------------------------ small kernels

// DNA: A C G T (either case) -> 0..3.  Matrix scoring: the letter's class.
// Anything else is rejected and written as the padding code.
__device__ __forceinline__ uint8_t encode_letter(uint8_t ch, const EncTable& tab, bool& ok) {
    if (!tab.dna) {
        const int c = tab.cls[ch];
        ok = c >= 0;
        return ok ? (uint8_t)c : (uint8_t)tab.pad_code;
    }
    ch &= 0xDF;  // upper case
    const uint8_t code = ch == 'A' ? 0 : ch == 'C' ? 1 : ch == 'G' ? 2 : ch == 'T' ? 3 : 0xff;
    ok = code != 0xff;
    return ok ? code : kPadCode;
}

// mode: bit 0 reverses the sequence, bit 1 complements it (DNA: A<->T, C<->G: code ^ 3).
__global__ void encode_kernel(const uint8_t* __restrict__ src, int64_t n, uint8_t* __restrict__ dst,
                              int64_t pad_before, int64_t pad_after, int mode, EncTable tab,
                              unsigned long long* bad) {
    const int64_t total = pad_before + n + pad_after;
    const uint8_t flip = (mode & 2) ? 3 : 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = i - pad_before;
        uint8_t code = (uint8_t)tab.pad_code;
        if (j >= 0 && j < n) {
            const int64_t sj = (mode & 1) ? n - 1 - j : j;
            bool ok;
            code = encode_letter(src[sj], tab, ok);
            if (!ok) atomicMax(bad, (1ull << 62) - (unsigned long long)sj);  // largest value = first offset
            else code ^= flip;
        }
        dst[i] = code;
    }
}

// Many sequences: sequence k is src[src_off[k] .. +len[k]) -> dst[dst_off[k] .. +len[k]).
// Padding around the destinations is written by the caller (zero kernel + pad fill).
__global__ void encode_many_kernel(const uint8_t* __restrict__ src, const int64_t* __restrict__ src_off,
                                   const int64_t* __restrict__ dst_off, const int64_t* __restrict__ len,
                                   int64_t n, uint8_t* __restrict__ dst, EncTable tab, unsigned long long* bad) {
    for (int64_t k = blockIdx.x; k < n; k += gridDim.x) {
        const int64_t so = src_off[k], d = dst_off[k], L = len[k];
        for (int64_t i = threadIdx.x; i < L; i += blockDim.x) {
            bool ok;
            const uint8_t code = encode_letter(src[so + i], tab, ok);
            if (!ok) atomicMax(bad, (1ull << 62) - (unsigned long long)(so + i));
            dst[d + i] = code;
        }
    }
}

__global__ void fill_u32_kernel(uint32_t* p, uint32_t v, size_t words) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < words; i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// Per problem: best task record (highest score, then smallest row, then smallest column).
__global__ __launch_bounds__(256) void reduce_kernel(const TaskRec* __restrict__ recs, const Prob* __restrict__ probs,
                                                     int64_t n_probs, int R, ScoreOut* out,
                                                     const unsigned long long* __restrict__ pruned,
                                                     const int32_t* __restrict__ gbest,
                                                     const int32_t* __restrict__ abort_flag) {
    __shared__ int32_t s_v[256];
    __shared__ int64_t s_r[256];
    __shared__ int64_t s_c[256];
    const int t = threadIdx.x;
    for (int64_t pi = blockIdx.x; pi < n_probs; pi += gridDim.x) {
        const Prob pr = probs[pi];
        const int64_t n = pr.Q * pr.n_bands;
        int32_t bv = INT32_MIN;
        int64_t br = INT64_MAX, bc = INT64_MAX;
        for (int64_t i = t; i < n; i += blockDim.x) {
            if (!task_in_band(pr, i / pr.Q, i % pr.Q, R)) continue;  // no ticket, no record
            const TaskRec r = recs[pr.task0 + i];
            const int64_t col = r.col < 0 ? INT64_MAX : r.col;
            if (r.score > bv || (r.score == bv && (r.row < br || (r.row == br && col < bc)))) {
                bv = r.score;
                br = r.row;
                bc = col;
            }
        }
        s_v[t] = bv;
        s_r[t] = br;
        s_c[t] = bc;
        __syncthreads();
        for (int off = blockDim.x / 2; off > 0; off >>= 1) {
            if (t < off) {
                const int32_t v2 = s_v[t + off];
                const int64_t r2 = s_r[t + off], c2 = s_c[t + off];
                if (v2 > s_v[t] || (v2 == s_v[t] && (r2 < s_r[t] || (r2 == s_r[t] && c2 < s_c[t])))) {
                    s_v[t] = v2;
                    s_r[t] = r2;
                    s_c[t] = c2;
                }
            }
            __syncthreads();
        }
        if (t == 0) {
            ScoreOut o;
            o.pruned_cells = pruned ? pruned[pi] : 0;
            o.status = 0;
            const bool local = pr.left_kind == BORDER_ZERO;  // the local recurrence has zero borders
            if (local && s_v[0] < pr.target) {
                // Below the target nothing was tracked: report the largest H seen
                // (a lower bound of the optimum), without an endpoint.
                o.score = max(max(s_v[0], gbest[pi]), 0);
                o.end_a = -1;
                o.end_b = -1;
            } else if (local && s_v[0] <= 0) {
                o.score = 0;
                o.end_a = -1;
                o.end_b = -1;
            } else {
                o.score = s_v[0];
                o.end_a = s_r[0];
                o.end_b = s_c[0];
                // cells are tracked from max(running best, target) up: below the target
                // (a learned threshold above the best) the endpoint is unknown by design
                if (pr.track && s_v[0] >= pr.target && (s_c[0] == INT64_MAX || s_c[0] >= pr.N || s_r[0] >= pr.M))
                    o.status = 1;
            }
            if (abort_flag && *abort_flag) o.status = 2;
            out[pi] = o;
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------------ launchers

hipError_t launch_encode(const uint8_t* src, int64_t n, uint8_t* dst, int64_t pad_before, int64_t pad_after,
                         int mode, const EncTable& tab, unsigned long long* bad, hipStream_t st) {
    if ((mode & ENC_COMPLEMENT) && !tab.dna) return hipErrorInvalidValue;
    const int64_t total = pad_before + n + pad_after;
    const int blocks = (int)min((int64_t)4096, (total + 255) / 256);
    hipLaunchKernelGGL(encode_kernel, dim3(max(blocks, 1)), dim3(256), 0, st, src, n, dst, pad_before, pad_after,
                       mode, tab, bad);
    return hipGetLastError();
}

hipError_t launch_encode_many(const uint8_t* src, const int64_t* src_off, const int64_t* dst_off,
                              const int64_t* len, int64_t n, uint8_t* dst, const EncTable& tab,
                              unsigned long long* bad, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const int blocks = (int)min((int64_t)8192, n);
    hipLaunchKernelGGL(encode_many_kernel, dim3(blocks), dim3(256), 0, st, src, src_off, dst_off, len, n, dst, tab,
                       bad);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t* p, int32_t v, size_t n, hipStream_t st) {
    if (!n) return hipSuccess;
    const int blocks = (int)std::min((size_t)4096, (n + 255) / 256);
    hipLaunchKernelGGL(fill_u32_kernel, dim3(blocks), dim3(256), 0, st, (uint32_t*)p, (uint32_t)v, n);
    return hipGetLastError();
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t st) {
    return launch_fill_i32((int32_t*)p, 0, (bytes + 3) / 4, st);
}

template <bool LOCAL, bool CD>
static void launch_variant(const EngineArgs& args, int R, int occ, dim3 g, hipStream_t st) {
    const dim3 b(kWave);
    if (args.sub.n_class > 0) {  // matrix scoring: the query profile in dynamic LDS
        const size_t lds = (size_t)args.sub.n_class * kWave * (R == 4 ? 4 : 8);
        if (R == 6 && occ <= 2) hipLaunchKernelGGL((engine_kernel<6, LOCAL, CD, 2, true>), g, b, lds, st, args);
        else if (R == 6) hipLaunchKernelGGL((engine_kernel<6, LOCAL, CD, 3, true>), g, b, lds, st, args);
        else if (R == 4) hipLaunchKernelGGL((engine_kernel<4, LOCAL, CD, 4, true>), g, b, lds, st, args);
        else if (occ <= 2) hipLaunchKernelGGL((engine_kernel<8, LOCAL, CD, 2, true>), g, b, lds, st, args);
        else hipLaunchKernelGGL((engine_kernel<8, LOCAL, CD, 3, true>), g, b, lds, st, args);
        return;
    }
    if (R == 6 && occ <= 2) hipLaunchKernelGGL((engine_kernel<6, LOCAL, CD, 2, false>), g, b, 0, st, args);
    else if (R == 6) hipLaunchKernelGGL((engine_kernel<6, LOCAL, CD, 3, false>), g, b, 0, st, args);
    else if (R == 4 && !LOCAL && occ <= 2) hipLaunchKernelGGL((engine_kernel<4, false, CD, 2, false>), g, b, 0, st, args);
    else if (R == 4) hipLaunchKernelGGL((engine_kernel<4, LOCAL, CD, 4, false>), g, b, 0, st, args);
    else if (occ <= 2) hipLaunchKernelGGL((engine_kernel<8, LOCAL, CD, 2, false>), g, b, 0, st, args);
    else hipLaunchKernelGGL((engine_kernel<8, LOCAL, CD, 3, false>), g, b, 0, st, args);
}

bool chain_variant(int rows_per_lane, bool local, bool cd, int n_class, int chain) {
    return !local && cd && n_class == 0 && rows_per_lane == 4 && (chain == 4 || chain == 8);
}

hipError_t launch_engine(const EngineArgs& args, int rows_per_lane, int waves_per_cu, bool local, bool cd, int grid,
                         int chain, hipStream_t st) {
    if (rows_per_lane != 4 && rows_per_lane != 6 && rows_per_lane != 8) return hipErrorInvalidValue;
    if (args.sub.n_class < 0 || args.sub.n_class > kMaxClasses) return hipErrorInvalidValue;
    if (grid < 1) return hipErrorInvalidValue;
    if (chain_variant(rows_per_lane, local, cd, args.sub.n_class, chain)) {
        // groups of `chain` waves; each group takes `chain` tickets at a time
        const dim3 g((unsigned)((grid + chain - 1) / chain)), b((unsigned)(kWave * chain));
        if (chain == 8) hipLaunchKernelGGL((chain_kernel<4, 8, 2>), g, b, 0, st, args);
        else hipLaunchKernelGGL((chain_kernel<4, 4, 2>), g, b, 0, st, args);
        return hipGetLastError();
    }
    const int occ = (waves_per_cu + 3) / 4;  // waves per SIMD (4 SIMDs per CU)
    const dim3 g(grid);
    if (local && cd) launch_variant<true, true>(args, rows_per_lane, occ, g, st);
    else if (local) launch_variant<true, false>(args, rows_per_lane, occ, g, st);
    else if (cd) launch_variant<false, true>(args, rows_per_lane, occ, g, st);
    else launch_variant<false, false>(args, rows_per_lane, occ, g, st);
    return hipGetLastError();
}

hipError_t launch_reduce(const TaskRec* recs, const Prob* probs, int64_t n_probs, int rows_per_lane, ScoreOut* out,
                         const int32_t* gbest, const unsigned long long* pruned, const int32_t* abort_flag,
                         hipStream_t st) {
    const int blocks = (int)min((int64_t)4096, max((int64_t)1, n_probs));
    hipLaunchKernelGGL(reduce_kernel, dim3(blocks), dim3(256), 0, st, recs, probs, n_probs, rows_per_lane, out,
                       pruned, gbest, abort_flag);
    return hipGetLastError();
}

}  // namespace swmi
