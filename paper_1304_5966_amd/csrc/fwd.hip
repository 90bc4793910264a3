// Forward local-alignment pass (SW# paper, Section 2, first phase) on gfx950.
//
// Matrix: rows = A (length M), columns = B (length N).  Recurrences (affine
// gaps, abstract of the paper), with E/F clamped at 0 -- exact for H because a
// non-positive gap value can never beat the zero floor:
//   E(i,j) = max(E(i,j-1) - ext, H(i,j-1) - open, 0)
//   F(i,j) = max(F(i-1,j) - ext, H(i-1,j) - open)
//   H(i,j) = max(H(i-1,j-1) + s(A_i,B_j), E(i,j), F(i,j))        (>= 0 through E)
//
// Work decomposition (the paper's wavefront of cell blocks, mapped to wave64):
//  * A stripe is 64*R consecutive rows; lane l owns rows l*R .. l*R+R-1 of it
//    and at step t works on column t-l (anti-diagonal skew of one column per
//    lane).  H, E and the open-gap value H-open live in int32 VGPRs.
//  * Each step the lane below receives the lane above's last-row H and its
//    F-candidate through DPP wave_shr:1; lane 0 receives the row above the
//    stripe through the DPP "old" operand, read from an LDS staging ring.
//  * Substitution scores: per row a 4-byte table s(a_row, c), c = 0..3; a
//    v_perm_b32 with four column codes as selector yields four score bytes,
//    consumed by sign-extended byte-select adds.
//  * Columns are cut into bands of W; a task is (band, stripe).  Tasks are
//    taken from an in-order ticket counter, so a task only ever waits on older
//    tasks: the stripe above in the same band (bottom row, streamed through a
//    global slot with a published column count), the same stripe in the
//    previous band (its right boundary H,E per row), and the task that last
//    read the slot being reused.  The oldest unfinished task never waits,
//    hence no deadlock and no assumption about residency.
//  * Every 64 steps (a tick) the wave exchanges 64 boundary columns: inputs
//    for the next tick are prefetched from the producer slot, outputs of lane
//    63 are written to this task's slot, and the column count is published
//    with release semantics.
//  * Block pruning (paper Section 2): before a tick, UB = max(0, every H on the
//    tick's input borders) + match * min(rows left, columns left); if UB is
//    strictly below max(running best, external T) the tick is skipped and its
//    outputs are the lower bounds H = 0, gap = 0.  Exact by induction along an
//    optimal path.
//  * Endpoint: each lane keeps the running maximum of each of its rows.  When a
//    tick raised a row maximum to at least the running global best, the tick
//    is replayed from a register snapshot to find the first column holding it.
#include "swmi_internal.h"

namespace swmi {

// ------------------------------------------------------------------------ helpers

__device__ __forceinline__ int dpp_shr1(int old, int src) {
    // wave_shr:1 with bound_ctrl off: lane l <- src of lane l-1, lane 0 keeps `old`
    return __builtin_amdgcn_update_dpp(old, src, 0x138, 0xf, 0xf, false);
}

__device__ __forceinline__ int sext_byte(uint32_t w, int i) {
    return ((int)(w << (24 - 8 * i))) >> 24;
}

__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = max(v, __shfl_xor(v, off));
    return v;
}

__device__ __forceinline__ int load_acquire(const int32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void store_release(int32_t* p, int32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// Waits until *flag >= need.  `seen` caches the last value observed with acquire
// semantics, so a satisfied wait costs no memory traffic.
__device__ __forceinline__ void wait_at_least(const int32_t* flag, int32_t need, int32_t& seen) {
    while (seen < need) {
        seen = load_acquire(flag);
        if (seen < need) __builtin_amdgcn_s_sleep(1);
    }
}

__device__ __forceinline__ uint32_t row_table(int code, int match, int mismatch) {
    if (code > 3) return kPadTable;
    const uint32_t mm = (uint32_t)(uint8_t)(int8_t)(-mismatch) * 0x01010101u;
    const int sh = 8 * code;
    return (mm & ~(0xffu << sh)) | ((uint32_t)(uint8_t)match << sh);
}

template <int R>
struct WaveState {
    int H[R];      // H of the lane's rows at the last column processed
    int E[R];      // E, clamped at 0
    int HA[R];     // H - open (shared by E of the next column and F of the next row)
    int best[R];   // running maximum of each row
    int pos[R];    // first column holding best[] (-1 when not tracked)
    uint32_t T[R]; // substitution table of each row
    int hup;       // H received from the row above at the previous step (next diagonal of the first row)
    int hl, gl;    // this lane's last-row H and F-candidate of the previous step (DPP sources)
};

struct TickCtx {
    const int2* in;   // LDS, 64 lane-0 inputs {H, gap} for this tick
    int2* out;        // LDS, 64 lane-63 outputs
    int2* lbuf;       // right-boundary store for the next band (capture ticks)
    int64_t row0;     // first row of this lane
    int64_t col0;     // absolute column of step 0 for lane 0
    int lane;
    int rel0;         // band-relative column of step 0 for lane 0
    int W;            // band width
    int M_rows;       // rows of this lane inside the matrix (0..R)
    int open, ext;
};

// One tick: 64 steps of the skewed stripe.
//  TRACK: replay mode -- no outputs, no maxima; records the first column where
//         a wanted row reaches its maximum.
//  EDGE:  lanes left of the band's first column hold their state (tick 0), and
//         the H,E state at the band's last column is stored for the next band.
//  Column codes: byte m of the lane's window is the code of the column it works
//  on at step m; `first` is the byte address of step 0's column.  One aligned
//  dword is loaded per 4-step group (one group ahead) and byte-aligned.
template <int R, bool TRACK, bool EDGE>
__device__ __forceinline__ void run_tick(WaveState<R>& s, const uint8_t* first, const TickCtx& c,
                                         const bool (&want)[R], bool capture) {
    const uint32_t* src = reinterpret_cast<const uint32_t*>((uintptr_t)first & ~(uintptr_t)3);
    const uint32_t sh = (uint32_t)((uintptr_t)first & 3);
    uint32_t lo = src[0], hi = src[1];
#pragma unroll 1
    for (int g = 0; g < kTick / 4; ++g) {
        const uint32_t cw = __builtin_amdgcn_alignbyte(hi, lo, sh);
        lo = hi;
        hi = src[g + 2];
        uint32_t sc[R];
#pragma unroll
        for (int k = 0; k < R; ++k) sc[k] = __builtin_amdgcn_perm(kPadTable, s.T[k], cw);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int m = 4 * g + i;
            const int2 in = c.in[m];
            const int upH = dpp_shr1(in.x, s.hl);
            const int upG = dpp_shr1(in.y, s.gl);
            int diag = s.hup;
            s.hup = upH;
            int F = upG;
            const int rel = c.rel0 + m - c.lane;
            const bool act = EDGE ? (rel >= 0) : true;
#pragma unroll
            for (int k = 0; k < R; ++k) {
                const int Hd = diag + sext_byte(sc[k], i);
                const int En = max(max(s.E[k] - c.ext, s.HA[k]), 0);
                const int Hn = max(max(Hd, En), F);
                const int HAn = Hn - c.open;
                F = max(F - c.ext, HAn);
                diag = s.H[k];
                if (EDGE) {
                    if (act) {
                        s.H[k] = Hn;
                        s.E[k] = En;
                        s.HA[k] = HAn;
                    }
                    if (!TRACK && capture && rel == c.W - 1 && k < c.M_rows)
                        c.lbuf[c.row0 + k] = make_int2(Hn, En);
                } else {
                    s.H[k] = Hn;
                    s.E[k] = En;
                    s.HA[k] = HAn;
                }
                if (TRACK) {
                    if (act && want[k] && s.pos[k] < 0 && Hn == s.best[k]) s.pos[k] = (int)(c.col0 + m - c.lane);
                } else if (EDGE) {
                    if (act) s.best[k] = max(s.best[k], Hn);
                } else {
                    s.best[k] = max(s.best[k], Hn);
                }
            }
            s.hl = s.H[R - 1];
            s.gl = F;
            if (!TRACK && c.lane == 63) c.out[m] = make_int2(s.hl, s.gl);
        }
    }
}

template <int R>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(R <= 4 ? 4 : 2))) void fwd_kernel(FwdArgs p) {
    __shared__ int2 in_ring[2][kTick];
    __shared__ int2 out_buf[kTick];
    const int lane = threadIdx.x;
    const int64_t n_tasks = p.n_bands * p.Q;
    unsigned long long pruned = 0;

    for (;;) {
        uint32_t tk = 0;
        if (lane == 0) tk = atomicAdd(p.ticket, 1u);
        const int64_t task = (int64_t)__builtin_amdgcn_readfirstlane(tk);
        if (task >= n_tasks) break;
        const int64_t band = task / p.Q;
        const int64_t q = task - band * p.Q;
        const int64_t c0 = band * p.W;
        const int W = (int)min(p.W, p.N - c0);
        const int n_ticks = (W + 2 * kTick - 2) / kTick;  // ceil((W + 63) / 64)
        const int64_t R0 = q * (int64_t)(kWave * R);
        const int64_t row0 = R0 + (int64_t)lane * R;
        const bool capture = band + 1 < p.n_bands;
        int2* my_slot = p.slots + (task % p.nslot) * p.slot_stride;
        const int2* prod_slot = q > 0 ? p.slots + ((task - 1) % p.nslot) * p.slot_stride : nullptr;
        const int32_t* prod_prog = p.progress + (task - 1);
        int32_t prod_seen = 0;

        // Older tasks this one depends on (see the header comment).
        if (band > 0) {
            int32_t seen = 0;
            wait_at_least(p.progress + task - p.Q, kDone, seen);
        }
        if (task >= p.nslot) {
            int32_t seen = 0;
            wait_at_least(p.progress + task - p.nslot + 1, kDone, seen);
        }

        WaveState<R> s;
        int M_rows = (int)max((int64_t)0, min((int64_t)R, p.M - row0));
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const int64_t row = row0 + k;
            int code = kPadCode;
            int h = 0, e = 0;
            if (row < p.M) {
                code = p.a[row];
                if (band > 0) {
                    const int2 lb = p.lbuf[row];
                    h = lb.x;
                    e = lb.y;
                }
            }
            s.T[k] = row_table(code, p.match, p.mismatch);
            s.H[k] = h;
            s.E[k] = e;
            s.HA[k] = h - p.open;
            s.best[k] = 0;
            s.pos[k] = -1;
        }
        s.hup = 0;
        s.hl = s.H[R - 1];
        s.gl = 0;
        // H of the stripe's last row at the column left of the band, for the stripe below.
        if (lane == kWave - 1) my_slot[kSlotPad - 1] = make_int2(s.H[R - 1], 0);

        // Inputs of tick 0 and the diagonal of the first cell.
        {
            int2 v = make_int2(0, 0);
            int h_diag = 0;
            if (q > 0) {
                wait_at_least(prod_prog, min(kTick, W), prod_seen);
                if (lane < W) v = prod_slot[kSlotPad + lane];
                h_diag = prod_slot[kSlotPad - 1].x;
            }
            in_ring[0][lane] = v;
            if (lane == 0) s.hup = h_diag;
        }
        __syncthreads();

        for (int tau = 0; tau < n_ticks; ++tau) {
            const int cur = tau & 1;
            // Prefetch the next tick's inputs (consumed at the end of this tick).
            int2 nxt = make_int2(0, 0);
            if (q > 0 && tau + 1 < n_ticks) {
                const int rel = kTick * (tau + 1) + lane;
                wait_at_least(prod_prog, min(kTick * (tau + 2), W), prod_seen);
                if (rel < W) nxt = prod_slot[kSlotPad + rel];
            }
            const uint8_t* cols = p.b + c0 + (int64_t)kTick * tau - lane;

            const int L = __hip_atomic_load(p.gbest, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const bool edge = (tau == 0) ||
                              (capture && kTick * tau - (kTick - 1) <= W - 1 && W - 1 <= kTick * tau + (kTick - 1));
            TickCtx c;
            c.in = in_ring[cur];
            c.out = out_buf;
            c.lbuf = p.lbuf;
            c.row0 = row0;
            c.col0 = c0 + (int64_t)kTick * tau;
            c.lane = lane;
            c.rel0 = kTick * tau;
            c.W = W;
            c.M_rows = M_rows;
            c.open = p.open;
            c.ext = p.ext;

            bool skip = false;
            if (p.prune && !edge) {
                int hm = max(s.hup, in_ring[cur][lane].x);
#pragma unroll
                for (int k = 0; k < R; ++k) hm = max(hm, s.H[k]);
                hm = max(wave_max(hm), 0);
                const int64_t rows_left = p.M - R0;
                const int64_t cols_left = p.N - (c.col0 - (kTick - 1));
                const int64_t ub = (int64_t)hm + (int64_t)p.match * min(rows_left, cols_left);
                const int64_t thr = max((int64_t)L, (int64_t)p.threshold);
                skip = ub < thr;
            }

            if (skip) {
                pruned += (unsigned long long)kTick * kWave * R;
#pragma unroll
                for (int k = 0; k < R; ++k) {
                    s.H[k] = 0;
                    s.E[k] = 0;
                    s.HA[k] = -p.open;
                }
                s.hup = 0;
                s.hl = 0;
                s.gl = 0;
                if (lane == kWave - 1) {
                    for (int m = 0; m < kTick; ++m) out_buf[m] = make_int2(0, 0);
                }
            } else {
                int H0[R], E0[R], bstart[R];
#pragma unroll
                for (int k = 0; k < R; ++k) {
                    H0[k] = s.H[k];
                    E0[k] = s.E[k];
                    bstart[k] = s.best[k];
                }
                const int hup0 = s.hup, hl0 = s.hl, gl0 = s.gl;
                bool want[R];
#pragma unroll
                for (int k = 0; k < R; ++k) want[k] = false;
                if (edge)
                    run_tick<R, false, true>(s, cols, c, want, capture);
                else
                    run_tick<R, false, false>(s, cols, c, want, capture);

                bool any = false;
#pragma unroll
                for (int k = 0; k < R; ++k) {
                    const bool inc = s.best[k] > bstart[k];
                    want[k] = inc && s.best[k] >= L;
                    if (inc) s.pos[k] = -1;
                    any = any || want[k];
                }
                if (__any(any)) {
                    // Replay from the snapshot; the replay ends in the same state.
#pragma unroll
                    for (int k = 0; k < R; ++k) {
                        s.H[k] = H0[k];
                        s.E[k] = E0[k];
                        s.HA[k] = H0[k] - p.open;
                    }
                    s.hup = hup0;
                    s.hl = hl0;
                    s.gl = gl0;
                    if (edge)
                        run_tick<R, true, true>(s, cols, c, want, capture);
                    else
                        run_tick<R, true, false>(s, cols, c, want, capture);
                    int mx = 0;
#pragma unroll
                    for (int k = 0; k < R; ++k)
                        if (want[k]) mx = max(mx, s.best[k]);
                    mx = wave_max(mx);
                    if (lane == 0 && mx > L) atomicMax(p.gbest, mx);
                }
            }

            // Hand the 64 bottom-row columns of this tick to the stripe below.
            __syncthreads();
            {
                const int rel = kTick * tau - (kTick - 1) + lane;
                if (rel >= 0) my_slot[kSlotPad + rel] = out_buf[lane];
            }
            store_release(p.progress + task, min(kTick * tau + 1, W));
            in_ring[cur ^ 1][lane] = nxt;
            __syncthreads();
        }

        // Task record: the stripe's best value, its smallest row, that row's first column.
        {
            int bv = -1, bk = 0, bp = -1;
#pragma unroll
            for (int k = 0; k < R; ++k) {
                if (s.best[k] > bv) {
                    bv = s.best[k];
                    bk = k;
                    bp = s.pos[k];
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
                p.recs[task] = r;
            }
        }
        store_release(p.progress + task, kDone);
    }
    if (pruned && lane == 0) atomicAdd(p.pruned_cells, pruned);
}

// ------------------------------------------------------------------------ small kernels

__global__ void encode_kernel(const uint8_t* __restrict__ src, int64_t n, uint8_t* __restrict__ dst,
                              int64_t pad_before, int64_t pad_after, unsigned long long* bad) {
    const int64_t total = pad_before + n + pad_after;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = i - pad_before;
        uint8_t code = kPadCode;
        if (j >= 0 && j < n) {
            const uint8_t ch = src[j] & 0xDF;
            code = ch == 'A' ? 0 : ch == 'C' ? 1 : ch == 'G' ? 2 : ch == 'T' ? 3 : 0xff;
            if (code == 0xff) {
                atomicMax(bad, (1ull << 62) - (unsigned long long)j);  // largest value = first offset
                code = kPadCode;
            }
        }
        dst[i] = code;
    }
}

__global__ void zero_kernel(uint32_t* p, size_t words) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < words; i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

// Best task record: highest score, then smallest row, then smallest column.
__global__ __launch_bounds__(1024) void reduce_kernel(const TaskRec* __restrict__ recs, int64_t n, int64_t N,
                                                      ScoreOut* out) {
    __shared__ int32_t s_v[1024];
    __shared__ int64_t s_r[1024];
    __shared__ int64_t s_c[1024];
    const int t = threadIdx.x;
    int32_t bv = -1;
    int64_t br = INT64_MAX, bc = INT64_MAX;
    for (int64_t i = t; i < n; i += blockDim.x) {
        const TaskRec r = recs[i];
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
        o.pruned_cells = 0;
        o.status = 0;
        if (s_v[0] <= 0) {
            o.score = 0;
            o.end_a = -1;
            o.end_b = -1;
        } else {
            o.score = s_v[0];
            o.end_a = s_r[0];
            o.end_b = s_c[0];
            if (s_c[0] == INT64_MAX || s_c[0] >= N) o.status = 1;
        }
        out->score = o.score;
        out->status = o.status;
        out->end_a = o.end_a;
        out->end_b = o.end_b;
    }
}

// ------------------------------------------------------------------------ launchers

hipError_t launch_encode(const uint8_t* src, int64_t n, uint8_t* dst, int64_t pad_before, int64_t pad_after,
                         unsigned long long* bad, hipStream_t st) {
    const int64_t total = pad_before + n + pad_after;
    const int blocks = (int)min((int64_t)4096, (total + 255) / 256);
    hipLaunchKernelGGL(encode_kernel, dim3(max(blocks, 1)), dim3(256), 0, st, src, n, dst, pad_before, pad_after, bad);
    return hipGetLastError();
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t st) {
    const size_t words = (bytes + 3) / 4;
    if (!words) return hipSuccess;
    const int blocks = (int)std::min((size_t)4096, (words + 255) / 256);
    hipLaunchKernelGGL(zero_kernel, dim3(blocks), dim3(256), 0, st, (uint32_t*)p, words);
    return hipGetLastError();
}

hipError_t launch_fwd(const FwdArgs& args, int rows_per_lane, int grid, hipStream_t st) {
    switch (rows_per_lane) {
        case 4:
            hipLaunchKernelGGL(fwd_kernel<4>, dim3(grid), dim3(kWave), 0, st, args);
            break;
        case 8:
            hipLaunchKernelGGL(fwd_kernel<8>, dim3(grid), dim3(kWave), 0, st, args);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_reduce(const TaskRec* recs, int64_t n, int64_t N, ScoreOut* out, hipStream_t st) {
    hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(1024), 0, st, recs, n, N, out);
    return hipGetLastError();
}

}  // namespace swmi
