// Second phase (start point) and reconstruction (Myers-Miller) of SW#
// (paper Section 2), plus sw_batch.
//
// Start point: the global recurrence (no zero floor) on the reversed prefixes
// that end at the endpoint, anchored at the endpoint (every border -inf except
// the corner).  The start is the first reversed cell, in row-major order, whose
// value equals the best score.  Only the diagonals a path of that score can
// reach are kept: with x aligned pairs its total gap length is at most
// (match*x - S) / extend, and x <= the shorter prefix.
//
// Reconstruction: Myers-Miller on the start..end rectangle with gap cost
// g + h*k (g = open - extend, h = extend), ends opening at tb = te = g.
// Each level, every sub-problem with enough rows runs on the GPU as two global
// problems -- the top half forward and the bottom half reversed -- whose last
// rows (H and the deletion-ending F) feed a midline kernel: the first strict
// maximum over columns of CC+RR (plain crossing) and DD+SS+g (a deletion run
// through the midline), a plain crossing ranked first at equal columns.
// Smaller sub-problems continue the same recursion on host threads, so the
// alignment does not depend on where the GPU hands over.  Every sub-problem
// knows its optimal score, which bounds its diagonals as above.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <cstdlib>
#include <deque>
#include <mutex>
#include <cstring>
#include <string>
#include <thread>
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

namespace swmi {

// ------------------------------------------------------------------------ midline kernel

__device__ __forceinline__ bool mid_better(int64_t v, int64_t j, int t, int64_t v2, int64_t j2, int t2) {
    return v > v2 || (v == v2 && (j < j2 || (j == j2 && t < t2)));
}

__global__ __launch_bounds__(256) void midline_kernel(const MidTask* __restrict__ tasks, int64_t n,
                                                      const int32_t* __restrict__ oh, const int32_t* __restrict__ of,
                                                      int32_t g, MidResult* out) {
    __shared__ int64_t sv[256], sj[256];
    __shared__ int32_t st[256];
    const int t = threadIdx.x;
    for (int64_t k = blockIdx.x; k < n; k += gridDim.x) {
        const MidTask mt = tasks[k];
        int64_t bv = INT64_MIN, bj = INT64_MAX;
        int32_t bt = 3;
        for (int64_t j = t; j <= mt.N; j += blockDim.x) {
            const int64_t cc = oh[mt.fwd_out + j], dd = of[mt.fwd_out + j];
            const int64_t rr = oh[mt.rev_out + (mt.N - j)], ss = of[mt.rev_out + (mt.N - j)];
            const int64_t v1 = cc + rr, v2 = dd + ss + g;
            if (mid_better(v1, j, 1, bv, bj, bt)) {
                bv = v1;
                bj = j;
                bt = 1;
            }
            if (mid_better(v2, j, 2, bv, bj, bt)) {
                bv = v2;
                bj = j;
                bt = 2;
            }
        }
        sv[t] = bv;
        sj[t] = bj;
        st[t] = bt;
        __syncthreads();
        for (int off = blockDim.x / 2; off > 0; off >>= 1) {
            if (t < off && mid_better(sv[t + off], sj[t + off], st[t + off], sv[t], sj[t], st[t])) {
                sv[t] = sv[t + off];
                sj[t] = sj[t + off];
                st[t] = st[t + off];
            }
            __syncthreads();
        }
        if (t == 0) {
            MidResult r;
            r.value = sv[0];
            r.j = sj[0];
            r.type = st[0];
            r.pad = 0;
            r.cc = oh[mt.fwd_out + r.j];
            r.dd = of[mt.fwd_out + r.j];
            r.rr = oh[mt.rev_out + (mt.N - r.j)];
            r.ss = of[mt.rev_out + (mt.N - r.j)];
            out[k] = r;
        }
        __syncthreads();
    }
}

hipError_t launch_midline(const MidTask* tasks, int64_t n, const int32_t* oh, const int32_t* of, int32_t g,
                          MidResult* out, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(midline_kernel, dim3((unsigned)std::min<int64_t>(n, 4096)), dim3(256), 0, st, tasks, n, oh, of,
                       g, out);
    return hipGetLastError();
}

}  // namespace swmi

namespace {

// ------------------------------------------------------------------------ CIGAR pieces

struct Cigar {
    std::vector<char> op;
    std::vector<int64_t> len;
    void push(char o, int64_t k) {
        if (k <= 0) return;
        if (!op.empty() && op.back() == o) {
            len.back() += k;
            return;
        }
        op.push_back(o);
        len.push_back(k);
    }
    void append(const Cigar& c) {
        for (size_t i = 0; i < c.op.size(); ++i) push(c.op[i], c.len[i]);
    }
};

// A sub-problem of the reconstruction, in rectangle coordinates.
struct Sub {
    int64_t r0, M;   // rows [r0, r0 + M) of A'
    int64_t c0, N;   // columns [c0, c0 + N) of B'
    int64_t tb, te;  // gap-open cost of a deletion run touching the start / end corner
    int64_t score;   // optimal score of the sub-problem
    bool known;      // score is known (bounds the diagonals)
};

struct Piece {
    bool is_sub;
    Sub sub;
    Cigar ops;
    Cigar* host = nullptr;  // handed to the host threads: their result (HostTail)
};

// Diagonal band [lo, hi] (j - i) holding every path of score >= S, or the full range.
void sub_band(const Sub& s, int match, int h, int64_t& lo, int64_t& hi) {
    lo = -kNoBand;
    hi = kNoBand;
    if (!s.known) return;
    const int64_t G = ((int64_t)match * std::min(s.M, s.N) - s.score) / h;
    if (G < 0) return;
    const int64_t D = s.N - s.M;
    if (G < (D < 0 ? -D : D)) return;  // no such path: keep everything
    // a path has (G + D)/2 insertions and (G - D)/2 deletions at most
    lo = -((G - D) / 2);
    hi = (G + D) / 2;
}

// ------------------------------------------------------------------------ host Myers-Miller

struct HostMM {
    const uint8_t* A;  // codes of A' (DNA 0..3, or matrix classes)
    const uint8_t* B;  // codes of B'
    int64_t g, h;
    int match;         // largest substitution score (band bounds)
    int32_t w_tab[kMaxClasses][kMaxClasses];  // s(x, y) by codes
    std::vector<int64_t> CC, DD, RR, SS;
    std::vector<uint8_t> ra, rb;

    void set_scoring(const sw_scoring* sc) {
        match = sc->match;
        for (int x = 0; x < kMaxClasses; ++x)
            for (int y = 0; y < kMaxClasses; ++y) w_tab[x][y] = subst_score(sc, (uint8_t)x, (uint8_t)y);
    }
    int64_t w(uint8_t x, uint8_t y) const { return w_tab[x][y]; }
    int64_t gap(int64_t k) const { return k > 0 ? g + h * k : 0; }

    // Forward over A[0..M) x B[0..N), columns outside [i + lo, i + hi] unreachable.
    void forward(const uint8_t* a, int64_t M, const uint8_t* b, int64_t N, int64_t tb, int64_t lo, int64_t hi,
                 std::vector<int64_t>& C, std::vector<int64_t>& D) {
        const int64_t NEG = -((int64_t)1 << 50);
        C.assign((size_t)N + 1, NEG);
        D.assign((size_t)N + 1, NEG);
        C[0] = 0;
        for (int64_t j = 1; j <= N && j <= hi; ++j) C[j] = -gap(j);
        for (int64_t i = 1; i <= M; ++i) {
            const int64_t jl = std::max<int64_t>(0, i + lo), jh = std::min<int64_t>(N, i + hi);
            int64_t diag = jl >= 1 ? C[jl - 1] : C[0];
            if (jl == 0) {
                diag = C[0];
                C[0] = -(tb + h * i);
                D[0] = C[0];
            } else {
                C[jl - 1] = NEG;  // left of the band in this row
                D[jl - 1] = NEG;
            }
            int64_t ins = NEG;
            for (int64_t j = std::max<int64_t>(1, jl); j <= jh; ++j) {
                ins = std::max(ins - h, C[j - 1] - g - h);
                D[j] = std::max(D[j] - h, C[j] - g - h);
                const int64_t c = std::max(diag + w(a[i - 1], b[j - 1]), std::max(D[j], ins));
                diag = C[j];
                C[j] = c;
            }
            if (jh + 1 <= N) {  // right of the band in this row
                C[jh + 1] = NEG;
                D[jh + 1] = NEG;
            }
        }
    }

    void solve(const uint8_t* a, int64_t M, const uint8_t* b, int64_t N, int64_t tb, int64_t te, int64_t score,
               bool known, Cigar& out) {
        if (N == 0) {
            out.push('D', M);
            return;
        }
        if (M == 0) {
            out.push('I', N);
            return;
        }
        if (M == 1) {
            const int64_t v_del = -(std::min(tb, te) + h) - gap(N);
            int64_t v_al = INT64_MIN, k_al = -1;
            for (int64_t k = 1; k <= N; ++k) {
                const int64_t v = -gap(k - 1) + w(a[0], b[k - 1]) - gap(N - k);
                if (v > v_al) {
                    v_al = v;
                    k_al = k;
                }
            }
            if (v_al >= v_del) {
                out.push('I', k_al - 1);
                out.push(a[0] == b[k_al - 1] ? '=' : 'X', 1);
                out.push('I', N - k_al);
            } else if (te < tb) {
                out.push('I', N);
                out.push('D', 1);
            } else {
                out.push('D', 1);
                out.push('I', N);
            }
            return;
        }
        Sub s{0, M, 0, N, tb, te, score, known};
        int64_t lo, hi;
        sub_band(s, match, (int)h, lo, hi);
        const int64_t mid = M / 2;
        forward(a, mid, b, N, tb, lo, hi, CC, DD);
        ra.assign(a + mid, a + M);
        std::reverse(ra.begin(), ra.end());
        rb.assign(b, b + N);
        std::reverse(rb.begin(), rb.end());
        const int64_t D = N - M;
        forward(ra.data(), M - mid, rb.data(), N, te, lo == -kNoBand ? lo : D - hi, hi == kNoBand ? hi : D - lo, RR,
                SS);
        int64_t best = INT64_MIN, bj = 0;
        int type = 1;
        for (int64_t j = 0; j <= N; ++j) {
            const int64_t v1 = CC[j] + RR[N - j];
            if (v1 > best) {
                best = v1;
                bj = j;
                type = 1;
            }
            const int64_t v2 = DD[j] + SS[N - j] + g;
            if (v2 > best) {
                best = v2;
                bj = j;
                type = 2;
            }
        }
        const int64_t cc = CC[bj], dd = DD[bj], rr = RR[N - bj], ss = SS[N - bj];
        if (type == 1) {
            solve(a, mid, b, bj, tb, g, cc, known, out);
            solve(a + mid, M - mid, b + bj, N - bj, g, te, rr, known, out);
        } else {
            solve(a, mid - 1, b, bj, tb, 0, dd + g + h, known, out);
            out.push('D', 2);
            solve(a + mid + 1, M - mid - 1, b + bj, N - bj, 0, te, ss + g + h, known, out);
        }
    }
};

// The reconstruction's host part (paper Section 2: the CPU and the GPU work on the
// reconstruction in parallel).  Sub-problems too small for a GPU level go to host
// threads as soon as a level produces them, while the GPU runs the next levels.
class HostTail {
   public:
    HostTail(const uint8_t* A, const uint8_t* B, int64_t g, int64_t h, const sw_scoring* sc, unsigned threads) {
        for (unsigned t = 0; t < threads; ++t)
            th_.emplace_back([=]() {
                HostMM mm;
                mm.A = A;
                mm.B = B;
                mm.g = g;
                mm.h = h;
                mm.set_scoring(sc);
                for (;;) {
                    std::pair<Sub, Cigar*> job;
                    {
                        std::unique_lock<std::mutex> lk(mu_);
                        cv_.wait(lk, [&] { return closed_ || !q_.empty(); });
                        if (q_.empty()) return;
                        job = q_.front();
                        q_.pop_front();
                    }
                    const Sub& sb = job.first;
                    mm.solve(A + sb.r0, sb.M, B + sb.c0, sb.N, sb.tb, sb.te, sb.score, sb.known, *job.second);
                }
            });
    }
    ~HostTail() { finish(); }
    // Queues a sub-problem; its alignment will be in the returned Cigar once finish() returned.
    Cigar* submit(const Sub& s) {
        std::lock_guard<std::mutex> lk(mu_);
        res_.emplace_back();
        Cigar* c = &res_.back();  // deque elements keep their address
        q_.emplace_back(s, c);
        cv_.notify_one();
        return c;
    }
    void finish() {
        {
            std::lock_guard<std::mutex> lk(mu_);
            closed_ = true;
        }
        cv_.notify_all();
        for (auto& t : th_) t.join();
        th_.clear();
    }

   private:
    std::mutex mu_;
    std::condition_variable cv_;
    std::deque<std::pair<Sub, Cigar*>> q_;
    std::deque<Cigar> res_;
    bool closed_ = false;
    std::vector<std::thread> th_;
};

// Children of a sub-problem split at (j, type), with their exact scores.
void split_sub(const Sub& s, const MidResult& r, int64_t g, int64_t h, std::vector<Piece>& out) {
    const int64_t mid = s.M / 2;
    Piece top{}, bot{};
    top.is_sub = bot.is_sub = true;
    if (r.type == 1) {
        top.sub = Sub{s.r0, mid, s.c0, r.j, s.tb, g, r.cc, true};
        bot.sub = Sub{s.r0 + mid, s.M - mid, s.c0 + r.j, s.N - r.j, g, s.te, r.rr, true};
        out.push_back(top);
        out.push_back(bot);
    } else {
        top.sub = Sub{s.r0, mid - 1, s.c0, r.j, s.tb, 0, r.dd + g + h, true};
        bot.sub = Sub{s.r0 + mid + 1, s.M - mid - 1, s.c0 + r.j, s.N - r.j, 0, s.te, r.ss + g + h, true};
        Piece dd{};
        dd.is_sub = false;
        dd.ops.push('D', 2);
        out.push_back(top);
        out.push_back(dd);
        out.push_back(bot);
    }
}

}  // namespace

// ------------------------------------------------------------------------ start point

// Rows per lane for banded global passes.  A stripe of 64 R rows starts 64 R
// columns right of the one above, so across a band W diagonals wide only about
// W / (64 R) stripes run at once; R = 4 doubles that where 512-row stripes
// would leave SIMDs without a wave (fewer than 1.5 per SIMD).
static int banded_rows(const sw_context* ctx, int64_t band_width_sum) {
    return band_width_sum >= (int64_t)kWave * 8 * 6 * ctx->num_cu ? 8 : 4;
}

static sw_status start_pass(sw_context* ctx, const uint8_t* d_a, const uint8_t* d_b, const sw_scoring* sc,
                            int32_t score, int64_t end_a, int64_t end_b, const sw_options* o, int64_t* start_a,
                            int64_t* start_b) {
    const Phase ph("swmi start pass");
    const int64_t M = end_a + 1, N = end_b + 1;
    ProbSpec ps;
    ps.a_off = 0;
    ps.b_off = kBPad;
    ps.M = M;
    ps.N = N;
    ps.top_kind = BORDER_NEG;
    ps.left_kind = BORDER_NEG;
    ps.target = score;
    ps.prune = 1;
    ps.track = 1;
    const int64_t G = ((int64_t)sc->match * std::min(M, N) - score) / sc->gap_extend;
    ps.d_lo = -G;
    ps.d_hi = G;
    const int R = o && o->rows_per_lane ? o->rows_per_lane : banded_rows(ctx, 2 * G + 1);
    const EnginePlan p = plan_engine(ctx, {ps}, false, R, o ? o->waves_per_cu : 0, o ? o->band_width : 0);
    const size_t cb = align_up((size_t)M + 64, 256) + align_up((size_t)(kBPad + N + kBPadTail), 256);
    void* ws;
    sw_status st = ctx_buffer(ctx, BUF_WORK, cb + 256 + p.total, &ws);
    if (st != SW_OK) return st;
    uint8_t* a_codes = (uint8_t*)ws;
    uint8_t* b_codes = a_codes + align_up((size_t)M + 64, 256);
    uint8_t* flags = (uint8_t*)ws + cb;
    uint8_t* eng = flags + 256;
    hipStream_t s = ctx->stream;
    const EncTable et = enc_table(sc);
    HIP_TRY(launch_zero(flags, 256, s));
    HIP_TRY(launch_encode(d_a, M, a_codes, 0, 64, ENC_REVERSE, et, (unsigned long long*)flags, s));
    HIP_TRY(launch_encode(d_b, N, b_codes, kBPad, kBPadTail, ENC_REVERSE, et, (unsigned long long*)(flags + 8), s));
    if ((st = run_engine(ctx, p, a_codes, b_codes, sc, eng, nullptr, nullptr)) != SW_OK) return st;
    uint8_t* hm = (uint8_t*)ctx->host_misc;
    HIP_TRY(hipMemcpyAsync(hm, flags, 16, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(hm + 64, eng + p.off_outs, sizeof(ScoreOut), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    unsigned long long bad_a, bad_b;
    std::memcpy(&bad_a, hm, 8);
    std::memcpy(&bad_b, hm + 8, 8);
    if (bad_a) return fail(SW_EINVAL, "sequence a: byte at offset %llu is not %s", kBadBase - bad_a, letters_text(sc));
    if (bad_b) return fail(SW_EINVAL, "sequence b: byte at offset %llu is not %s", kBadBase - bad_b, letters_text(sc));
    ScoreOut so;
    std::memcpy(&so, hm + 64, sizeof so);
    if (so.status) return fail(SW_EINTERNAL, "reverse pass: %s", engine_status_text(so.status));
    if (so.score != score)
        return fail(SW_EINVAL, "no alignment of score %d ends at (%lld, %lld) (reverse pass reached %d)", score,
                    (long long)end_a, (long long)end_b, so.score);
    *start_a = end_a - so.end_a;
    *start_b = end_b - so.end_b;
    return SW_OK;
}

extern "C" sw_status sw_start(sw_context* ctx, const char* a, int64_t len_a, const char* b, int64_t len_b,
                              const sw_scoring* scoring, int32_t score, int64_t end_a, int64_t end_b,
                              int64_t* start_a, int64_t* start_b) {
    if (!ctx || !start_a || !start_b) return fail(SW_EINVAL, "sw_start: NULL argument");
    sw_status st;
    sw_scoring sc;
    if ((st = check_scoring(scoring, &sc)) != SW_OK) return st;
    if ((st = check_lengths(len_a, len_b, &sc)) != SW_OK) return st;
    if ((len_a && !a) || (len_b && !b)) return fail(SW_EINVAL, "sw_start: NULL sequence pointer");
    if (score <= 0) {
        *start_a = *start_b = -1;
        return SW_OK;
    }
    if (end_a < 0 || end_a >= len_a || end_b < 0 || end_b >= len_b)
        return fail(SW_EINVAL, "sw_start: endpoint (%lld, %lld) outside the sequences", (long long)end_a,
                    (long long)end_b);
    if ((int64_t)scoring->gap_open * (end_a + end_b + 2) >= ((int64_t)1 << 29))
        return fail(SW_EUNSUPPORTED, "gap_open * (end_a + end_b) reaches 2^29 (int32 headroom)");
    HIP_TRY(hipSetDevice(ctx->device));
    uint8_t *d_a, *d_b;
    if ((st = upload_pair(ctx, a, end_a + 1, b, end_b + 1, &d_a, &d_b)) != SW_OK) return st;
    return start_pass(ctx, d_a, d_b, &sc, score, end_a, end_b, nullptr, start_a, start_b);
}

// ------------------------------------------------------------------------ reconstruction

// Rows of a sub-problem from which a level runs it on the GPU.
static const int64_t kGpuRows = 2048;

static sw_status reconstruct(sw_context* ctx, const uint8_t* d_a, const uint8_t* d_b, int64_t M, int64_t N,
                             const sw_scoring* sc, int64_t total_score, const sw_options* o, Cigar& cigar) {
    const Phase ph("swmi reconstruction");
    const int64_t g = sc->gap_open - sc->gap_extend, h = sc->gap_extend;
    hipStream_t s = ctx->stream;
    // Codes: forward a | forward b (padded) | reversed a | reversed b (padded); plus host copies.
    const size_t la = align_up((size_t)M + 64, 256), lb = align_up((size_t)(kBPad + N + kBPadTail), 256);
    void* cbuf;
    sw_status st = ctx_buffer(ctx, BUF_CODES, 2 * (la + lb) + 256, &cbuf);
    if (st != SW_OK) return st;
    uint8_t* fa = (uint8_t*)cbuf;
    uint8_t* fb = fa + la;
    uint8_t* rva = fb + lb;
    uint8_t* rvb = rva + la;
    uint8_t* flags = rvb + lb;
    const EncTable et = enc_table(sc);
    HIP_TRY(launch_zero(flags, 256, s));
    HIP_TRY(launch_encode(d_a, M, fa, 0, 64, 0, et, (unsigned long long*)flags, s));
    HIP_TRY(launch_encode(d_b, N, fb, kBPad, kBPadTail, 0, et, (unsigned long long*)flags, s));
    HIP_TRY(launch_encode(d_a, M, rva, 0, 64, ENC_REVERSE, et, (unsigned long long*)flags, s));
    HIP_TRY(launch_encode(d_b, N, rvb, kBPad, kBPadTail, ENC_REVERSE, et, (unsigned long long*)flags, s));
    std::vector<uint8_t> hA((size_t)M), hB((size_t)N);
    HIP_TRY(hipMemcpyAsync(hA.data(), fa, (size_t)M, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(hB.data(), fb + kBPad, (size_t)N, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));

    std::vector<Piece> pieces(1);
    pieces[0].is_sub = true;
    pieces[0].sub = Sub{0, M, 0, N, g, g, total_score, true};
    // Host threads take the sub-problems below the GPU size as they appear.
    const unsigned nthreads = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    HostTail tail(hA.data(), hB.data(), g, h, sc, nthreads);
    auto hand_small_to_host = [&]() {
        for (auto& pc : pieces)
            if (pc.is_sub && !(pc.sub.M >= kGpuRows && pc.sub.N > 0)) {
                pc.host = tail.submit(pc.sub);
                pc.is_sub = false;
            }
    };
    hand_small_to_host();
    for (;;) {
        // GPU level over every sub-problem with enough rows.
        std::vector<size_t> big;
        for (size_t i = 0; i < pieces.size(); ++i)
            if (pieces[i].is_sub && pieces[i].sub.M >= kGpuRows && pieces[i].sub.N > 0) big.push_back(i);
        if (big.empty()) break;
        const Phase level("swmi reconstruction level");
        std::vector<ProbSpec> specs;
        std::vector<MidTask> mids;
        int64_t out_len = 0, width_sum = 0;
        for (size_t bi : big) {
            const Sub& sb = pieces[bi].sub;
            int64_t lo, hi;
            sub_band(sb, sc->match, (int)h, lo, hi);
            width_sum += 2 * (lo > -kNoBand ? hi - lo + 1 : sb.N);  // both halves
        }
        const int R = o && o->rows_per_lane ? o->rows_per_lane : banded_rows(ctx, width_sum);
        for (size_t bi : big) {
            const Sub& sb = pieces[bi].sub;
            int64_t lo, hi;
            sub_band(sb, sc->match, (int)h, lo, hi);
            const int64_t mid = sb.M / 2;
            ProbSpec f;
            f.a_off = (int64_t)(0) + sb.r0;
            f.b_off = kBPad + sb.c0;
            f.M = mid;
            f.N = sb.N;
            f.top_kind = BORDER_GAP;
            f.top_open = sc->gap_open;
            f.left_kind = BORDER_GAP;
            f.left_open = (int32_t)(sb.tb + h);
            f.track = 0;
            f.d_lo = lo;
            f.d_hi = hi;
            f.out_off = out_len;
            out_len += sb.N + 1;
            ProbSpec r = f;
            // reversed bottom half: rows [mid, M) and all columns, both reversed; the
            // code buffer is [fa | fb | rva | rvb], bases fa (rows) and fb (columns)
            r.a_off = (int64_t)(la + lb) + (M - (sb.r0 + sb.M));
            r.b_off = (int64_t)(la + lb) + kBPad + (N - (sb.c0 + sb.N));
            r.M = sb.M - mid;
            r.left_open = (int32_t)(sb.te + h);
            if (lo > -kNoBand) {
                r.d_lo = (sb.N - sb.M) - hi;
                r.d_hi = (sb.N - sb.M) - lo;
            }
            r.out_off = out_len;
            out_len += sb.N + 1;
            specs.push_back(f);
            specs.push_back(r);
            mids.push_back(MidTask{f.out_off, r.out_off, sb.N});
        }
        const EnginePlan p = plan_engine(ctx, specs, false, R, o ? o->waves_per_cu : 0, o ? o->band_width : 0);
        void* wbuf;
        const size_t out_bytes = align_up((size_t)out_len * sizeof(int32_t), 256);
        const size_t mid_bytes = align_up(mids.size() * sizeof(MidTask), 256);
        const size_t res_bytes = align_up(mids.size() * sizeof(MidResult), 256);
        if ((st = ctx_buffer(ctx, BUF_WORK, p.total + 2 * out_bytes + mid_bytes + res_bytes, &wbuf)) != SW_OK)
            return st;
        uint8_t* eng = (uint8_t*)wbuf;
        int32_t* oh = (int32_t*)(eng + p.total);
        int32_t* of = (int32_t*)((uint8_t*)oh + out_bytes);
        MidTask* d_mid = (MidTask*)((uint8_t*)of + out_bytes);
        MidResult* d_res = (MidResult*)((uint8_t*)d_mid + mid_bytes);
        HIP_TRY(launch_fill_i32(oh, kNeg, (size_t)out_len, s));
        HIP_TRY(launch_fill_i32(of, kNeg, (size_t)out_len, s));
        if ((st = run_engine(ctx, p, fa, fb, sc, eng, oh, of)) != SW_OK) return st;
        HIP_TRY(hipMemcpyAsync(d_mid, mids.data(), mids.size() * sizeof(MidTask), hipMemcpyHostToDevice, s));
        HIP_TRY(launch_midline(d_mid, (int64_t)mids.size(), oh, of, (int32_t)g, d_res, s));
        std::vector<MidResult> res(mids.size());
        int32_t aborted = 0;
        HIP_TRY(hipMemcpyAsync(res.data(), d_res, mids.size() * sizeof(MidResult), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipMemcpyAsync(&aborted, eng + p.off_misc + MISC_ABORT, sizeof aborted, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (aborted) return fail(SW_EINTERNAL, "reconstruction: %s", engine_status_text(2));
        std::vector<Piece> next;
        next.reserve(pieces.size() + 2 * big.size());
        size_t k = 0;
        for (size_t i = 0; i < pieces.size(); ++i) {
            if (k < big.size() && big[k] == i) {
                const Sub& sb = pieces[i].sub;
                if (res[k].value != sb.score)
                    return fail(SW_EINTERNAL, "reconstruction: midline value %lld != sub-problem score %lld",
                                (long long)res[k].value, (long long)sb.score);
                split_sub(sb, res[k], g, h, next);
                ++k;
            } else {
                next.push_back(std::move(pieces[i]));
            }
        }
        pieces.swap(next);
        hand_small_to_host();
    }

    // Every sub-problem is with the host threads now; the pieces in order make the CIGAR.
    tail.finish();
    for (auto& pc : pieces) cigar.append(pc.host ? *pc.host : pc.ops);
    return SW_OK;
}

// Score of a CIGAR placed at (0, 0) of A' x B' (codes: DNA 0..3 or matrix classes), or a
// consistency failure.
static bool rescore(const Cigar& c, const std::vector<uint8_t>& A, const std::vector<uint8_t>& B,
                    const sw_scoring* sc, int64_t& score, int64_t& ea, int64_t& eb) {
    int64_t i = 0, j = 0, s = 0;
    for (size_t k = 0; k < c.op.size(); ++k) {
        const char o = c.op[k];
        const int64_t n = c.len[k];
        if (o == '=' || o == 'X') {
            for (int64_t t = 0; t < n; ++t, ++i, ++j) {
                if (i >= (int64_t)A.size() || j >= (int64_t)B.size()) return false;
                const uint8_t x = A[(size_t)i], y = B[(size_t)j];  // codes: equal iff the letters are
                const bool eq = x == y;
                if (eq != (o == '=')) return false;
                s += subst_score(sc, x, y);
            }
        } else {
            s -= sc->gap_open + (int64_t)sc->gap_extend * (n - 1);
            if (o == 'I') j += n;
            else i += n;
        }
    }
    score = s;
    ea = i - 1;
    eb = j - 1;
    return true;
}

extern "C" sw_status sw_align(sw_context* ctx, const char* a, int64_t len_a, const char* b, int64_t len_b,
                              const sw_scoring* scoring, const sw_options* options, sw_align_result* out) {
    if (!out) return fail(SW_EINVAL, "sw_align: NULL result");
    std::memset(out, 0, sizeof *out);
    out->start_a = out->start_b = out->end_a = out->end_b = -1;
    if (!ctx) return fail(SW_EINVAL, "sw_align: NULL context");
    sw_status st;
    sw_scoring nsc;
    if ((st = check_scoring(scoring, &nsc)) != SW_OK) return st;
    if ((st = check_lengths(len_a, len_b, &nsc)) != SW_OK) return st;
    if ((st = check_options(options)) != SW_OK) return st;
    if ((st = check_matrix_options(&nsc, options)) != SW_OK) return st;
    if ((len_a && !a) || (len_b && !b)) return fail(SW_EINVAL, "sw_align: NULL sequence pointer");
    if ((int64_t)scoring->gap_open * (len_a + len_b + 2) >= ((int64_t)1 << 29))
        return fail(SW_EUNSUPPORTED, "gap_open * (len_a + len_b) reaches 2^29 (int32 headroom)");
    char* empty = (char*)std::malloc(1);
    if (!empty) return fail(SW_ENOMEM, "sw_align: out of host memory");
    empty[0] = 0;
    out->cigar = empty;
    if (len_a == 0 || len_b == 0) return SW_OK;
    HIP_TRY(hipSetDevice(ctx->device));
    sw_score_result sr;
    if ((st = sw_score(ctx, a, len_a, b, len_b, scoring, options, &sr)) != SW_OK) return st;
    out->score = sr.score;
    out->strand = sr.strand;
    if (sr.score <= 0) return SW_OK;
    // The reverse strand won: the later phases run on the reverse complement of B.
    std::string rc;
    if (sr.strand == 1) {
        rc.resize((size_t)len_b);
        for (int64_t j = 0; j < len_b; ++j) {
            const char ch = (char)(b[len_b - 1 - j] & 0xDF);
            rc[(size_t)j] = ch == 'A' ? 'T' : ch == 'C' ? 'G' : ch == 'G' ? 'C' : 'A';  // letters checked by sw_score
        }
        b = rc.data();
    }
    uint8_t *d_a, *d_b;
    if ((st = upload_pair(ctx, a, len_a, b, len_b, &d_a, &d_b)) != SW_OK) return st;
    int64_t sa, sb;
    if ((st = start_pass(ctx, d_a, d_b, &nsc, sr.score, sr.end_a, sr.end_b, options, &sa, &sb)) != SW_OK)
        return st;
    Cigar cig;
    const int64_t M = sr.end_a - sa + 1, N = sr.end_b - sb + 1;
    if ((st = reconstruct(ctx, d_a + sa, d_b + sb, M, N, &nsc, sr.score, options, cig)) != SW_OK) return st;
    // consistency: the alignment must rescore to the best score and span the rectangle
    {
        // codes of the letters (checked by the score pass): DNA 0..3, or matrix classes
        const EncTable et = enc_table(&nsc);
        auto code_of = [&](char ch) -> uint8_t {
            if (!et.dna) return (uint8_t)et.cls[(uint8_t)ch];
            const uint8_t u = (uint8_t)(ch & 0xDF);
            return u == 'A' ? 0 : u == 'C' ? 1 : u == 'G' ? 2 : 3;
        };
        std::vector<uint8_t> A((size_t)M), B((size_t)N);
        for (int64_t i = 0; i < M; ++i) A[(size_t)i] = code_of(a[sa + i]);
        for (int64_t j = 0; j < N; ++j) B[(size_t)j] = code_of(b[sb + j]);
        int64_t s2, ea, eb;
        if (!rescore(cig, A, B, &nsc, s2, ea, eb) || s2 != sr.score || ea != M - 1 || eb != N - 1)
            return fail(SW_EINTERNAL, "reconstruction does not rescore to the best score");
    }
    std::string text;
    for (size_t k = 0; k < cig.op.size(); ++k) {
        text += std::to_string(cig.len[k]);
        text += cig.op[k];
    }
    char* c = (char*)std::malloc(text.size() + 1);
    if (!c) return fail(SW_ENOMEM, "sw_align: out of host memory");
    std::memcpy(c, text.c_str(), text.size() + 1);
    std::free(out->cigar);
    out->cigar = c;
    out->cigar_len = (int64_t)text.size();
    out->start_a = sa;
    out->start_b = sb;
    out->end_a = sr.end_a;
    out->end_b = sr.end_b;
    return SW_OK;
}

extern "C" sw_status sw_mm_host(const char* a, int64_t len_a, const char* b, int64_t len_b,
                                const sw_scoring* scoring, int32_t tb, int32_t te, int32_t score_known,
                                int64_t score, char* cigar, int64_t cap, int64_t* cigar_len) {
    sw_status st;
    sw_scoring sc;
    if ((st = check_scoring(scoring, &sc)) != SW_OK) return st;
    if (len_a < 0 || len_b < 0 || (len_a && !a) || (len_b && !b) || !cigar || cap <= 0 || !cigar_len)
        return fail(SW_EINVAL, "sw_mm_host: bad arguments");
    const EncTable et = enc_table(&sc);
    auto code_of = [&](char ch) -> int {
        if (!et.dna) return et.cls[(uint8_t)ch];
        const uint8_t u = (uint8_t)(ch & 0xDF);
        return u == 'A' ? 0 : u == 'C' ? 1 : u == 'G' ? 2 : u == 'T' ? 3 : -1;
    };
    std::vector<uint8_t> A((size_t)len_a), B((size_t)len_b);
    for (int64_t i = 0; i < len_a; ++i) {
        const int c = code_of(a[i]);
        if (c < 0) return fail(SW_EINVAL, "sequence a: byte at offset %lld is not %s", (long long)i, letters_text(&sc));
        A[(size_t)i] = (uint8_t)c;
    }
    for (int64_t j = 0; j < len_b; ++j) {
        const int c = code_of(b[j]);
        if (c < 0) return fail(SW_EINVAL, "sequence b: byte at offset %lld is not %s", (long long)j, letters_text(&sc));
        B[(size_t)j] = (uint8_t)c;
    }
    const int64_t g = sc.gap_open - sc.gap_extend;
    HostMM mm;
    mm.g = g;
    mm.h = sc.gap_extend;
    mm.set_scoring(&sc);
    mm.A = A.data();
    mm.B = B.data();
    Cigar c;
    mm.solve(A.data(), len_a, B.data(), len_b, tb < 0 ? g : tb, te < 0 ? g : te, score, score_known != 0, c);
    std::string text;
    for (size_t k = 0; k < c.op.size(); ++k) {
        text += std::to_string(c.len[k]);
        text += c.op[k];
    }
    if ((int64_t)text.size() + 1 > cap) return fail(SW_ENOMEM, "sw_mm_host: CIGAR needs %zu bytes", text.size() + 1);
    std::memcpy(cigar, text.c_str(), text.size() + 1);
    *cigar_len = (int64_t)text.size();
    return SW_OK;
}

extern "C" void sw_align_result_free(sw_align_result* r) {
    if (!r) return;
    std::free(r->cigar);
    r->cigar = nullptr;
    r->cigar_len = 0;
}
