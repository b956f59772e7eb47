// Host runtime of the sparse FFT library: parameter validation and defaults,
// the flat-window tables (Section 7 construction, built in FP64 on the host),
// FFT twiddles, device workspaces, the plain (one signal, host round loop)
// and batched (hipGraph-replayed) execution paths, and the C ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <utility>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "sfft_internal.hpp"

using namespace sfft;

namespace {

thread_local std::string g_last_error;

sfft_status_t fail(sfft_status_t s, const std::string& msg) {
    g_last_error = msg;
    return s;
}

#define HIP_TRY(expr)                                                                         \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return fail(SFFT_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));       \
    } while (0)

bool is_pow2(uint64_t v) { return v >= 1 && (v & (v - 1)) == 0; }

uint32_t log2u(uint64_t v) {
    uint32_t l = 0;
    while ((1ull << l) < v) ++l;
    return l;
}

// ------------------------------------------------------------ window ------
// Gaussian width and boxcar half-width of the Section 7 construction:
// C = (1 - alpha/2)/(2B) and sigma_g = (4B/alpha) sqrt(2 ln(3/delta)).  The
// paper's ln(n/delta) comes from replacing delta by delta/n to absorb the
// sqrt(n) its normalisation puts into G; G here carries no sqrt(n), and the
// CDF-tail requirement of the lemma (beyond sqrt(2 ln(3/delta))) is met
// directly, which keeps ||Ghat - G'||_inf < delta with a shorter window.
WindowShape window_shape(uint64_t n, uint64_t B, double alpha, double delta) {
    (void)n;
    WindowShape ws{};   // ftab = nullptr: the closed-form G' of the Gaussian window
    ws.sigma_g = (4.0 * (double)B / alpha) * std::sqrt(2.0 * std::log(3.0 / delta));
    ws.C = (1.0 - alpha / 2.0) / (2.0 * (double)B);
    ws.alpha = alpha;
    // Over the transition band s < 1/(2B) the leading erfc is smallest at the
    // band's edge and the trailing one largest at its start.
    const double r2 = std::sqrt(2.0);
    const double lead_min = std::erfc(ws.sigma_g * (0.5 / (double)B - ws.C) / r2);
    const double tail_max = std::erfc(ws.sigma_g * ((1.0 - alpha) * 0.5 / (double)B + ws.C) / r2);
    ws.two_term = !(tail_max < std::ldexp(lead_min, -60));
    return ws;
}

// G*(t) = exp(-2 pi^2 t^2 / sigma_g^2) * sin(2 pi C t) / (pi t), G*(0) = 2C.
double g_star(double t, const WindowShape& ws) {
    const double pi = 3.14159265358979323846;
    const double gauss = std::exp(-2.0 * pi * pi * t * t / (ws.sigma_g * ws.sigma_g));
    const double box = t == 0.0 ? 2.0 * ws.C : std::sin(2.0 * pi * ws.C * t) / (pi * t);
    return gauss * box;
}

double tail_mass(uint64_t T, const WindowShape& ws) {
    const uint64_t span = (uint64_t)(12.0 * ws.sigma_g) + 2;
    double total = 0.0;
    for (uint64_t t = T; t < T + span; ++t) total += std::fabs(g_star((double)t, ws));
    return 2.0 * total;
}

uint64_t default_w(uint64_t n, uint64_t B, double alpha, double delta) {
    const WindowShape ws = window_shape(n, B, alpha, delta);
    uint64_t lo = 1, hi = n / B;
    if (tail_mass(hi * B / 2, ws) > delta) return n;
    while (lo < hi) {
        const uint64_t mid = (lo + hi) / 2;
        if (tail_mass(mid * B / 2, ws) <= delta) hi = mid; else lo = mid + 1;
    }
    return lo * B;
}

// Kaiser-Bessel flat window (plan field window = 1): the ideal low-pass
// sin(2 pi C t)/(pi t) (the Gaussian construction's C) tapered by
// I0(beta sqrt(1 - (2t/w)^2)) / I0(beta), with Kaiser's empirical rules for
// a ripple of delta/2 over the transition band alpha/(2B) cycles per sample:
// A = -20 log10(delta/2), beta = 0.1102 (A - 8.7) for A > 50, length
// (A - 7.95) / (14.36 alpha / (2B)) + 1 rounded up to a multiple of B.
double kaiser_beta(double delta) {
    const double A = -20.0 * std::log10(delta / 2.0);
    if (A > 50.0) return 0.1102 * (A - 8.7);
    if (A >= 21.0) return 0.5842 * std::pow(A - 21.0, 0.4) + 0.07886 * (A - 21.0);
    return 0.0;
}

uint64_t kaiser_w(uint64_t n, uint64_t B, double alpha, double delta) {
    const double A = -20.0 * std::log10(delta / 2.0);
    const double N = (A - 7.95) / (14.36 * alpha / (2.0 * (double)B)) + 1.0;
    const uint64_t m = (uint64_t)std::ceil(N / (double)B);
    return std::min<uint64_t>(n, m * B);
}

// I0 by its power series sum (x/2)^2k / (k!)^2.
double bessel_i0(double x) {
    const double q = 0.25 * x * x;
    double term = 1.0, total = 1.0;
    for (int k = 1; k < 200; ++k) {
        term *= q / ((double)k * (double)k);
        total += term;
        if (term <= 1e-17 * total) break;
    }
    return total;
}

// G_t of the Kaiser window of length w (t in [-w/2, w/2)).
double kaiser_g(double t, uint64_t w, double C, double beta, double i0_beta) {
    const double pi = 3.14159265358979323846;
    const double box = t == 0.0 ? 2.0 * C : std::sin(2.0 * pi * C * t) / (pi * t);
    const double r = 2.0 * t / (double)w;
    return box * bessel_i0(beta * std::sqrt(std::max(1.0 - r * r, 0.0))) / i0_beta;
}

uint32_t exact_round_bins(const sfft_plan_desc_t& d, uint32_t r) {
    const uint32_t floor_b = d.b_min ? d.b_min : std::max<uint32_t>(2u, d.B >> 4);
    const uint32_t f = std::min(floor_b, d.B);
    const uint32_t shifted = r >= 31 ? 0u : (d.B >> r);
    return std::max(shifted, f);
}

uint32_t zhat_capacity(const sfft_plan_desc_t& d) {
    uint64_t c = 4ull * std::max<uint32_t>(d.k, 16u);
    return (uint32_t)std::min<uint64_t>(c, kMaxZ);
}

}  // namespace

// ------------------------------------------------------------------ plan ---
constexpr uint32_t kMaxChunks = 8;

// Captured graphs of one batch shape: per chunk c, exec_h[c] = state reset +
// HashToBins of the chunk (launch stream), exec_d[c] = decode + output of the
// chunk (auxiliary stream), keyed by every argument pointer and the count;
// or (whole) exec_h[0] = the whole step of a one-chunk batch.
struct GraphCache {
    hipGraphExec_t exec_h[kMaxChunks] = {};
    hipGraphExec_t exec_d[kMaxChunks] = {};
    uint32_t chunks = 0;
    const void* x = nullptr;
    const void* seeds = nullptr;
    const void* o1 = nullptr;
    const void* o2 = nullptr;
    const void* o3 = nullptr;
    const void* o4 = nullptr;
    uint32_t count = 0;
    bool whole = false;   // exec_h[0] holds the whole step (one chunk, no phase events)
    // recorded after every replay: the graphs are destroyed (new arguments,
    // plan destroyed) only once their last replay has finished, so a replay
    // still queued on some stream never depends on how the runtime defers
    // the destruction of an executable graph in flight
    hipEvent_t launched = nullptr;
};

struct sfft_plan_s {
    sfft_plan_desc_t d;
    int device = 0;
    uint32_t R = 0;            // rounds with geometry
    size_t device_bytes = 0;   // device memory held by the plan
    bool dry = false;          // size the plan without touching a device
    // exact batched mode: ends of the round groups.  Group 0 is hashed for
    // every signal; each later group only for signals still decoding.
    std::vector<uint32_t> group_end;
    // exact batched mode: rounds hashed in stream mode (hash_mode) and the
    // workgroups per (signal, round) of those launches
    std::vector<uint8_t> stream_round;
    uint32_t stream_parts = 0;
    uint32_t Bmax = 0;
    uint32_t logBmax = 0;
    uint32_t capz = 0;
    uint32_t cap = 0;
    uint32_t mcap = 0;         // largest modulation table of the pair kernel
    uint32_t nhash = 2;        // raw-bin slots per round: the pair, plus the refinement hashing
    std::vector<RoundDev> geom;
    RoundDev* d_geom = nullptr;
    // general mode
    std::vector<GenRoundDev> groundv;
    std::vector<GenJob> jobs_loc, jobs_est;
    std::vector<uint32_t> loc_first, loc_count, est_first, est_count;
    GenRoundDev* d_groundv = nullptr;
    GenJob* d_jobs_loc = nullptr;
    GenJob* d_jobs_est = nullptr;
    uint32_t nslots = 0;
    double* cand_e = nullptr;
    uint32_t* cand_n = nullptr;
    double* d_g64 = nullptr;
    double* d_ftab = nullptr;  // Kaiser window: G' tables
    float* d_g32 = nullptr;
    double* d_tw64 = nullptr;  // Bmax complex
    float* d_tw32 = nullptr;
    // batched workspace (max_batch signals)
    double* raw = nullptr;
    double* work = nullptr;
    uint64_t* cand_i = nullptr;
    double* cand_v = nullptr;
    uint64_t* zidx = nullptr;
    double* zval = nullptr;
    double* est = nullptr;
    double* fin = nullptr;
    double* gtmp = nullptr;
    uint32_t* gfirst = nullptr;
    uint32_t* gent = nullptr;
    uint64_t* cand_raw = nullptr;
    uint32_t* cand_cnt = nullptr;
    uint8_t* eflag = nullptr;
    uint32_t* egrp = nullptr;
    uint16_t* eord = nullptr;
    double* ecoef = nullptr;
    double* gterm = nullptr;
    uint32_t* ecount = nullptr;
    uint32_t* state = nullptr;
    // plain-path workspace (one signal)
    double* p_raw = nullptr;
    double* p_partial = nullptr;
    double* split_partial = nullptr;   // batched split hashing: [count * group rounds][parts][4 Bmax]
    uint32_t p_parts_max = 0;
    uint64_t* p_idx = nullptr;
    double* p_val = nullptr;
    uint32_t* p_count = nullptr;
    uint32_t* p_info = nullptr;
    hipStream_t capture_stream = nullptr;
    hipStream_t aux_stream = nullptr;          // decode of chunk c overlaps HashToBins of chunk c+1
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    hipEvent_t ev_ready[kMaxChunks] = {};
    hipEvent_t ev_h0[kMaxChunks] = {}, ev_h1[kMaxChunks] = {}, ev_d0[kMaxChunks] = {}, ev_d1[kMaxChunks] = {};
    hipEvent_t ev_t0 = nullptr, ev_t1 = nullptr;
    uint32_t timed_chunks = 0;
    bool timed_once = false;
    GraphCache graph;
    std::mutex mu;
    std::vector<void*> allocations;
};

namespace {

template <class T>
sfft_status_t dev_alloc(sfft_plan_s* p, T** ptr, size_t count) {
    void* q = nullptr;
    const size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
    if (p->dry) {
        p->device_bytes += bytes;
        *ptr = nullptr;
        return SFFT_OK;
    }
    hipError_t e = hipMalloc(&q, bytes);
    if (e != hipSuccess) return fail(SFFT_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
    p->allocations.push_back(q);
    p->device_bytes += bytes;
    *ptr = reinterpret_cast<T*>(q);
    return SFFT_OK;
}

#define ST_TRY(expr)                      \
    do {                                  \
        sfft_status_t s_ = (expr);        \
        if (s_ != SFFT_OK) return s_;     \
    } while (0)

// Default SparseFFT rounds: k_r = k/4^r reaches 1 after ceil(log4 k) rounds;
// two more rounds at k_r = 1 pick up coefficients missed earlier (at
// n = 2^26, k = 1024 with 1% noise: 5 rounds recover 11 of 16 supports
// exactly, 7 rounds all 16), and never fewer than 7: a coefficient is missed
// only when its offset falls near a bin edge (G' too small to locate it) in
// every round, and rounds at k_r = 1 gather a few thousand samples each
// (5% noise, k = 20: 2.1e-4 of the coefficients missed with 5 rounds,
// 4e-5 with 7).
uint32_t general_default_rounds(uint32_t k) {
    uint32_t l4 = 0;
    while ((1ull << (2 * l4)) < k) ++l4;
    return std::max<uint32_t>(7u, l4 + 2);
}

sfft_status_t resolve_and_validate(sfft_plan_desc_t& d) {
    sfft_status_t s = sfft_validate_params(&d);
    if (s != SFFT_OK) return s;
    if (d.w == 0) d.w = d.window == 1 ? kaiser_w(d.n, d.B, d.alpha, d.delta) : default_w(d.n, d.B, d.alpha, d.delta);
    if (d.cap == 0) d.cap = d.k;
    if (d.rounds == 0) d.rounds = d.mode == SFFT_MODE_GENERAL ? general_default_rounds(d.k) : 16;
    if (d.hash_threads == 0) d.hash_threads = 256;
    if (d.refine_shift && d.refine_window == 0) d.refine_window = 16;
    return SFFT_OK;
}

uint32_t pow2_ceil(uint64_t v) {
    uint32_t f = 1;
    while (f < v) f <<= 1;
    return f;
}

bool general_mode(const sfft_plan_s* p) { return p->d.mode == SFFT_MODE_GENERAL; }

// Round r of SparseFFT (Algorithm 2), practical schedule: k_r = k >> 2r,
// B_r = max(B >> r, 4 k_r rounded up to a power of two, b_min), capped at B
// (b_min = B keeps B and w fixed in every round).
void general_round_shape(const sfft_plan_desc_t& d, uint32_t r, uint32_t* k_r, uint32_t* B_r) {
    const uint32_t kr = std::max<uint32_t>(1u, r >= 16 ? 0u : (d.k >> (2 * r)));
    const uint32_t floor_b = std::max<uint32_t>(pow2_ceil(4ull * kr), d.b_min);
    const uint32_t shifted = r >= 31 ? 0u : (d.B >> r);
    *k_r = kr;
    *B_r = std::min<uint32_t>(d.B, std::max(shifted, floor_b));
}

// LocateInner levels of a round with B_r bins: widths W (fixed point) while
// W > 1, shrinking by t/4; beta in [ceil(s n t / (4W)), floor(s n t / (2W))].
void general_levels(const sfft_plan_desc_t& d, uint32_t B_r, GenRoundDev& gr) {
    const uint64_t scale = 1ull << kFracBits;
    uint64_t W = (d.n / B_r) * scale;
    gr.nlev = 0;
    while (W > scale && gr.nlev < kMaxLevels) {
        const double Wr = (double)W / (double)scale;
        const double snt = d.s * (double)d.n * (double)d.t;
        uint64_t lo = (uint64_t)std::ceil(snt / (4.0 * Wr));
        uint64_t hi = (uint64_t)std::floor(snt / (2.0 * Wr));
        lo = std::max<uint64_t>(lo, 1);
        hi = std::max(hi, lo);
        gr.Wfp[gr.nlev] = W;
        gr.blo[gr.nlev] = lo;
        gr.bhi[gr.nlev] = hi;
        ++gr.nlev;
        W = W * 4 / d.t;
    }
}

sfft_status_t build_plan(sfft_plan_s* p) {
    const sfft_plan_desc_t& d = p->d;
    if (!p->dry) HIP_TRY(hipGetDevice(&p->device));
    // round geometry (exact mode schedule)
    p->R = d.rounds;
    p->Bmax = d.B;
    p->logBmax = log2u(d.B);
    p->capz = zhat_capacity(d);
    p->cap = d.cap;
    std::vector<double> g64;
    std::vector<std::pair<uint32_t, double>> seenB;   // (B_r, alpha_r) of each window table
    std::vector<uint64_t> seenOfs;
    // Kaiser window: each window table's G' table (|f| <= n / (2 B_r)) at
    // an offset of the G' tables, and the round's offset
    std::vector<uint64_t> seenF, round_f;
    uint64_t nftab = 0;
    const bool kaiser = d.window == 1;
    const double kbeta = kaiser_beta(d.delta), ki0 = bessel_i0(kbeta);
    p->mcap = 4;
    // exact mode with alpha_decay: alpha shrinks with B up to the first
    // round at the smallest bin count
    const bool decay = !general_mode(p) && d.alpha_decay > 0.0 && d.alpha_decay < 1.0;
    uint32_t r_floor = 0;
    if (decay)
        while (r_floor + 1 < p->R && exact_round_bins(d, r_floor + 1) != exact_round_bins(d, r_floor)) ++r_floor;
    for (uint32_t r = 0; r < p->R; ++r) {
        RoundDev g;
        if (general_mode(p)) {
            GenRoundDev gr;
            std::memset(&gr, 0, sizeof(gr));
            general_round_shape(d, r, &gr.k_r, &g.B);
            general_levels(d, g.B, gr);
            gr.nloc = gr.nlev * d.R_loc;
            gr.slot0 = p->nslots;
            p->loc_first.push_back((uint32_t)p->jobs_loc.size());
            p->est_first.push_back((uint32_t)p->jobs_est.size());
            for (uint32_t q = 0; q < gr.nloc; ++q) p->jobs_loc.push_back(GenJob{r, q, gr.slot0 + q, 0});
            for (uint32_t e = 0; e < d.R_est; ++e) p->jobs_est.push_back(GenJob{r, gr.nloc + e, gr.slot0 + gr.nloc + e, 0});
            p->loc_count.push_back(gr.nloc);
            p->est_count.push_back(d.R_est);
            p->nslots += gr.nloc + d.R_est;
            p->groundv.push_back(gr);
        } else {
            g.B = exact_round_bins(d, r);
        }
        g.logB = log2u(g.B);
        double alpha_r = d.alpha;
        g.w = d.w / d.B * g.B;
        if (decay) {
            const double f = std::pow(d.alpha_decay, (double)std::min(r, r_floor));
            alpha_r = d.alpha * f;
            // sigma_g scales as B / alpha: the same tail mass needs w scaled alike
            g.w = (uint64_t)std::ceil((double)(d.w / d.B) / f - 1e-9) * g.B;
            if (g.w > d.n) return fail(SFFT_EINVAL, "alpha_decay makes a round's window longer than n");
        }
        g.t0 = -(int64_t)(g.w / 2);
        g.ws = window_shape(d.n, g.B, alpha_r, d.delta);
        auto it = std::find(seenB.begin(), seenB.end(), std::make_pair(g.B, alpha_r));
        if (it == seenB.end()) {
            g.gofs = g64.size();
            for (uint64_t u = 0; u < g.w; ++u) {
                const double t = (double)(g.t0 + (int64_t)u);
                g64.push_back(kaiser ? kaiser_g(t, g.w, g.ws.C, kbeta, ki0) : g_star(t, g.ws));
            }
            seenB.emplace_back(g.B, alpha_r);
            seenOfs.push_back(g.gofs);
            seenF.push_back(nftab);
            if (kaiser) nftab += d.n / (2 * g.B) + 1;
            round_f.push_back(seenF.back());
        } else {
            g.gofs = seenOfs[it - seenB.begin()];
            round_f.push_back(seenF[it - seenB.begin()]);
        }
        // modulation table length: the exact pair (a = 0, beta = 1); general
        // pairs need at most 2 w_r / B_r + 4 (beta below w) or w_r / B_r + 2
        // per segment (beta at least w)
        const int64_t iB = g.B;
        const int64_t Llo = floordiv(g.t0 - 1 - (iB - 1), iB);
        const int64_t Lhi = floordiv(g.t0 + (int64_t)g.w - 1, iB);
        p->mcap = std::max<uint32_t>(p->mcap, (uint32_t)(Lhi - Llo + 1));
        if (!general_mode(p) && d.refine_shift) {
            // the pair with the refinement hashing: one window [t0 - A, t0 + w)
            // for A < w + 1, else [t0 - A, t0 - A + w) beside the pair's
            const int64_t iA = (int64_t)d.refine_shift, iw = (int64_t)g.w;
            const int64_t lo0 = g.t0 - iA, hi0 = iA < iw + 1 ? g.t0 + iw : lo0 + iw;
            const int64_t L0 = floordiv(lo0 - (iB - 1), iB), L1 = floordiv(hi0 - 1, iB);
            p->mcap = std::max<uint32_t>(p->mcap, (uint32_t)(L1 - L0 + 1));
        }
        if (general_mode(p)) p->mcap = std::max<uint32_t>(p->mcap, (uint32_t)(2 * (g.w / g.B) + 4));
        p->geom.push_back(g);
    }
    // Round groups of the batched exact path: a signal stops at the earliest
    // `patience` rounds after the first round at the smallest bin count, so
    // group 0 runs to there unless the plan sets `group0`; later groups take
    // 2, 2, 4, 8, ... rounds, or group_step, 2 group_step, 4 group_step, ...
    // (few signals need the long tail, and every group costs two launches).
    if (!general_mode(p)) {
        uint32_t first_floor = p->R;
        for (uint32_t r = 0; r < p->R; ++r)
            if (r + 1 == p->R || p->geom[r + 1].B == p->geom[r].B) {
                first_floor = r;
                break;
            }
        uint32_t e = std::min<uint32_t>(p->R, d.group0 ? d.group0 : first_floor + d.patience + 1);
        p->group_end.push_back(e);
        for (uint32_t g = 1; e < p->R; ++g) {
            const uint32_t len = d.group_step ? d.group_step << (g - 1 < 16 ? g - 1 : 16)
                                              : (g <= 2 ? 2u : 1u << (g - 1));
            e = std::min<uint32_t>(p->R, e + len);
            p->group_end.push_back(e);
        }
    }
    // stream mode: a round whose window covers at least an eighth of the
    // signal reads the signal contiguously (n samples in full lines) instead
    // of gathering w_r + 1 samples at a line each
    p->stream_round.assign(p->R, 0);
    if (!general_mode(p) && d.hash_mode != 0) {
        uint32_t maxB = 0;
        for (uint32_t r = 0; r < p->R; ++r)
            if (d.hash_mode == 2 || 8 * p->geom[r].w >= d.n) {
                p->stream_round[r] = 1;
                maxB = std::max(maxB, p->geom[r].B);
            }
        // about 32 samples per thread and part, parts dividing n / B_r
        uint64_t parts = std::max<uint64_t>(1, std::min<uint64_t>(32, d.n / 8192));
        while (maxB && parts > 1 && parts > d.n / maxB) parts >>= 1;
        p->stream_parts = (uint32_t)parts;
    }
    std::vector<float> g32(g64.begin(), g64.end());
    // twiddles exp(-2 pi i m / Bmax), m < Bmax
    std::vector<double> tw64(2 * (size_t)p->Bmax);
    std::vector<float> tw32(2 * (size_t)p->Bmax);
    const double two_pi = 6.283185307179586476925286766559;
    for (uint32_t m = 0; m < p->Bmax; ++m) {
        const double ang = two_pi * (double)m / (double)p->Bmax;
        tw64[2 * m] = std::cos(ang);
        tw64[2 * m + 1] = -std::sin(ang);
        tw32[2 * m] = (float)tw64[2 * m];
        tw32[2 * m + 1] = (float)tw64[2 * m + 1];
    }
    if (kaiser) {
        ST_TRY(dev_alloc(p, &p->d_ftab, nftab));
        for (uint32_t r = 0; r < p->R; ++r) p->geom[r].ws.ftab = p->d_ftab + round_f[r];
    }
    ST_TRY(dev_alloc(p, &p->d_geom, p->geom.size()));
    ST_TRY(dev_alloc(p, &p->d_g64, g64.size()));
    ST_TRY(dev_alloc(p, &p->d_g32, g32.size()));
    ST_TRY(dev_alloc(p, &p->d_tw64, tw64.size()));
    ST_TRY(dev_alloc(p, &p->d_tw32, tw32.size()));
    if (!p->dry) {
        HIP_TRY(hipMemcpy(p->d_geom, p->geom.data(), p->geom.size() * sizeof(RoundDev), hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(p->d_g64, g64.data(), g64.size() * sizeof(double), hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(p->d_g32, g32.data(), g32.size() * sizeof(float), hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(p->d_tw64, tw64.data(), tw64.size() * sizeof(double), hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(p->d_tw32, tw32.data(), tw32.size() * sizeof(float), hipMemcpyHostToDevice));
        // G' of each Kaiser window table, from its G (the window's response)
        for (size_t q = 0; kaiser && q < seenB.size(); ++q) {
            const uint32_t Bq = seenB[q].first;
            uint64_t wq = 0;
            for (const RoundDev& g : p->geom)
                if (g.gofs == seenOfs[q]) wq = g.w;
            HIP_TRY(launch_window_response(p->d_g64 + seenOfs[q], wq, -(int64_t)(wq / 2), d.n, Bq, seenB[q].second,
                                           p->d_ftab + seenF[q], d.n / (2 * Bq) + 1, nullptr));
        }
        if (kaiser) HIP_TRY(hipStreamSynchronize(nullptr));
    }
    if (general_mode(p)) {
        ST_TRY(dev_alloc(p, &p->d_groundv, p->groundv.size()));
        ST_TRY(dev_alloc(p, &p->d_jobs_loc, p->jobs_loc.size()));
        ST_TRY(dev_alloc(p, &p->d_jobs_est, p->jobs_est.size()));
        if (!p->dry) {
            HIP_TRY(hipMemcpy(p->d_groundv, p->groundv.data(), p->groundv.size() * sizeof(GenRoundDev),
                              hipMemcpyHostToDevice));
            HIP_TRY(hipMemcpy(p->d_jobs_loc, p->jobs_loc.data(), p->jobs_loc.size() * sizeof(GenJob),
                              hipMemcpyHostToDevice));
            HIP_TRY(hipMemcpy(p->d_jobs_est, p->jobs_est.data(), p->jobs_est.size() * sizeof(GenJob),
                              hipMemcpyHostToDevice));
        }
    }
    p->nhash = !general_mode(p) && d.refine_shift ? 3 : 2;
    if (p->nhash == 3 && h2b_pair_lds_bytes(p->Bmax, p->mcap, d.loc_prec == SFFT_F64, d.hash_threads, true) > 160 * 1024)
        return fail(SFFT_EUNSUPPORTED, "refinement hashing: the pair kernel's LDS would exceed 160 KiB (smaller B or FP32 bins)");
    // batched workspace
    const size_t S = d.max_batch;
    const size_t Bm = p->Bmax, R = p->R, Z = p->capz;
    const size_t raw_slots = general_mode(p) ? p->nslots : p->R;
    const size_t meas = general_mode(p) ? (size_t)p->R * d.R_est : p->R;
    const size_t per_slot = 2 * (size_t)p->nhash * Bm;   // doubles of one round's raw bins
    ST_TRY(dev_alloc(p, &p->raw, S * raw_slots * per_slot));
    if (general_mode(p)) {
        ST_TRY(dev_alloc(p, &p->cand_e, S * d.R_est * 2 * Bm));
        ST_TRY(dev_alloc(p, &p->cand_n, S * Bm));
        ST_TRY(dev_alloc(p, &p->gfirst, S * (Bm + 1)));
        ST_TRY(dev_alloc(p, &p->gent, S * Z));
        ST_TRY(dev_alloc(p, &p->cand_raw, S * Bm));
        ST_TRY(dev_alloc(p, &p->cand_cnt, S));
        ST_TRY(dev_alloc(p, &p->gterm, S * std::max<size_t>(R, d.R_est) * Z * 4));
    }
    ST_TRY(dev_alloc(p, &p->work, S * 4 * Bm));
    ST_TRY(dev_alloc(p, &p->cand_i, S * Bm));
    ST_TRY(dev_alloc(p, &p->cand_v, S * 2 * Bm));
    ST_TRY(dev_alloc(p, &p->zidx, S * 2 * Z));
    ST_TRY(dev_alloc(p, &p->zval, S * 4 * Z));
    ST_TRY(dev_alloc(p, &p->est, S * Z * meas * 2));
    ST_TRY(dev_alloc(p, &p->eflag, S * Z * meas));
    ST_TRY(dev_alloc(p, &p->egrp, S * Z * meas));
    ST_TRY(dev_alloc(p, &p->eord, S * Z * meas));
    ST_TRY(dev_alloc(p, &p->ecoef, S * Z * meas * 2));
    ST_TRY(dev_alloc(p, &p->fin, S * Z * 2));
    ST_TRY(dev_alloc(p, &p->gtmp, S * Z * 4));
    ST_TRY(dev_alloc(p, &p->ecount, S * Z));
    ST_TRY(dev_alloc(p, &p->state, S * kStateWords));
    if (!general_mode(p) && (d.hash_split > 1 || p->stream_parts > 0)) {
        // partial folds of the split and stream launches of one round group
        size_t longest = 0, longest_stream = 0;
        for (size_t g = 0, r0 = 0; g < p->group_end.size(); r0 = p->group_end[g], ++g) {
            longest = std::max<size_t>(longest, p->group_end[g] - r0);
            size_t ns = 0;
            for (size_t r = r0; r < p->group_end[g]; ++r) ns += p->stream_round[r];
            longest_stream = std::max(longest_stream, ns);
        }
        const size_t parts = std::max<size_t>(d.hash_split > 1 ? longest * d.hash_split : 0,
                                              longest_stream * p->stream_parts);
        ST_TRY(dev_alloc(p, &p->split_partial, S * parts * 4 * Bm));
    }
    // plain path (one signal): raw bins of every round, split partials
    p->p_parts_max = 64;
    ST_TRY(dev_alloc(p, &p->p_raw, raw_slots * per_slot));
    ST_TRY(dev_alloc(p, &p->p_partial, (size_t)p->p_parts_max * 4 * Bm));
    ST_TRY(dev_alloc(p, &p->p_idx, p->cap));
    ST_TRY(dev_alloc(p, &p->p_val, 2 * (size_t)p->cap));
    ST_TRY(dev_alloc(p, &p->p_count, 1));
    ST_TRY(dev_alloc(p, &p->p_info, 4));
    if (p->dry) return SFFT_OK;
    HIP_TRY(hipStreamCreateWithFlags(&p->capture_stream, hipStreamNonBlocking));
    HIP_TRY(hipStreamCreateWithFlags(&p->aux_stream, hipStreamNonBlocking));
    HIP_TRY(hipEventCreateWithFlags(&p->ev_fork, hipEventDisableTiming));
    HIP_TRY(hipEventCreateWithFlags(&p->ev_join, hipEventDisableTiming));
    for (auto& e : p->ev_ready) HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    if (d.flags & SFFT_FLAG_TIMING) {
        for (uint32_t c = 0; c < kMaxChunks; ++c) {
            HIP_TRY(hipEventCreate(&p->ev_h0[c]));
            HIP_TRY(hipEventCreate(&p->ev_h1[c]));
            HIP_TRY(hipEventCreate(&p->ev_d0[c]));
            HIP_TRY(hipEventCreate(&p->ev_d1[c]));
        }
        HIP_TRY(hipEventCreate(&p->ev_t0));
        HIP_TRY(hipEventCreate(&p->ev_t1));
    }
    return SFFT_OK;
}

bool loc_f64(const sfft_plan_s* p) { return p->d.loc_prec == SFFT_F64; }
bool in_c128(const sfft_plan_s* p) { return p->d.in_dtype == SFFT_C128; }

H2BArgs base_h2b(const sfft_plan_s* p, const void* x) {
    H2BArgs a;
    std::memset(&a, 0, sizeof(a));
    a.x = x;
    a.n = p->d.n;
    a.sig_stride = p->d.n;
    a.plan_seed = p->d.seed;
    a.Bmax = p->Bmax;
    a.logBmax = p->logBmax;
    a.geom = p->d_geom;
    a.gtab = loc_f64(p) ? (const void*)p->d_g64 : (const void*)p->d_g32;
    a.tw = loc_f64(p) ? (const void*)p->d_tw64 : (const void*)p->d_tw32;
    a.sqrt_n = std::sqrt((double)p->d.n);
    a.mcap = p->mcap;
    a.threads = p->d.hash_threads;
    a.order = p->d.hash_order;
    a.nhash = p->nhash;
    a.gamma = general_mode(p) ? 0 : p->d.refine_shift;
    return a;
}

DecodeArgs base_decode(const sfft_plan_s* p, uint32_t count, const uint64_t* seeds, const double* raw,
                       uint64_t* oidx, double* oval, uint32_t* ocount, uint32_t* oinfo) {
    DecodeArgs D;
    std::memset(&D, 0, sizeof(D));
    D.n = p->d.n;
    D.count = count;
    D.rounds = p->R;
    D.r_begin = 0;
    D.r_end = p->R;
    D.patience = p->d.patience;
    D.stop_count = p->d.mode == SFFT_MODE_EXACT ? p->d.stop_count : 0;
    D.stop_patience = p->d.stop_patience;
    D.ratio_tol = p->d.ratio_tol;
    D.nhash = p->nhash;
    D.refine_shift = p->d.refine_shift;
    D.refine_window = p->d.refine_window;
    D.Bmax = p->Bmax;
    D.capz = p->capz;
    D.cap = p->cap;
    D.geom = p->d_geom;
    D.seeds = seeds;
    D.plan_seed = p->d.seed;
    D.raw = raw;
    D.work = p->work;
    D.cand_i = p->cand_i;
    D.cand_v = p->cand_v;
    D.zidx = p->zidx;
    D.zval = p->zval;
    D.est = p->est;
    D.fin = p->fin;
    D.gtmp = p->gtmp;
    D.ecount = p->ecount;
    D.eflag = p->eflag;
    D.egrp = p->egrp;
    D.eord = p->eord;
    D.ecoef = p->ecoef;
    D.state = p->state;
    D.theta = p->d.theta;
    D.g_min = p->d.g_min;
    D.out_scale = (p->d.flags & SFFT_FLAG_NUMPY_NORM) ? std::sqrt((double)p->d.n) : 1.0;
    D.out_idx = oidx;
    D.out_val = oval;
    D.out_count = ocount;
    D.out_info = oinfo;
    return D;
}

GeneralArgs base_general(const sfft_plan_s* p, uint32_t count, const uint64_t* seeds, const double* raw,
                         uint64_t* oidx, double* oval, uint32_t* ocount, uint32_t* oinfo) {
    GeneralArgs G;
    std::memset(&G, 0, sizeof(G));
    G.n = p->d.n;
    G.count = count;
    G.R = p->R;
    G.nslots = p->nslots;
    G.Bmax = p->Bmax;
    G.capz = p->capz;
    G.cap = p->cap;
    G.t = p->d.t;
    G.R_loc = p->d.R_loc;
    G.R_est = p->d.R_est;
    G.s = p->d.s;
    G.g_min = p->d.g_min;
    G.out_scale = (p->d.flags & SFFT_FLAG_NUMPY_NORM) ? std::sqrt((double)p->d.n) : 1.0;
    G.geom = p->d_geom;
    G.groundv = p->d_groundv;
    G.seeds = seeds;
    G.plan_seed = p->d.seed;
    G.raw = raw;
    G.cand_i = p->cand_i;
    G.cand_v = p->cand_v;
    G.cand_e = p->cand_e;
    G.cand_n = p->cand_n;
    G.zidx = p->zidx;
    G.zval = p->zval;
    G.est = p->est;
    G.fin = p->fin;
    G.gtmp = p->gtmp;
    G.ecount = p->ecount;
    G.gfirst = p->gfirst;
    G.gent = p->gent;
    G.cand_raw = p->cand_raw;
    G.cand_cnt = p->cand_cnt;
    G.eflag = p->eflag;
    G.egrp = p->egrp;
    G.eord = p->eord;
    G.ecoef = p->ecoef;
    G.gterm = p->gterm;
    G.nterm = std::max<uint32_t>(p->R, p->d.R_est);
    G.state = p->state;
    G.out_idx = oidx;
    G.out_val = oval;
    G.out_count = ocount;
    G.out_info = oinfo;
    return G;
}

// General-mode HashToBins for rounds [r0, r1): every LocateInner pair in
// loc_prec arithmetic, every EstimateValues hashing in est_prec.
sfft_status_t enqueue_general_hash(sfft_plan_s* p, const void* x, uint32_t count, const uint64_t* seeds, double* raw,
                                   uint32_t r0, uint32_t r1, hipStream_t s, const void* const* xptrs = nullptr) {
    for (int kind = 0; kind < 2; ++kind) {
        const std::vector<uint32_t>& first = kind == 0 ? p->loc_first : p->est_first;
        const std::vector<uint32_t>& cnt = kind == 0 ? p->loc_count : p->est_count;
        const uint32_t j0 = first[r0];
        uint32_t nj = 0;
        for (uint32_t r = r0; r < r1; ++r) nj += cnt[r];
        if (nj == 0) continue;
        const bool f64 = (kind == 0 ? p->d.loc_prec : p->d.est_prec) == SFFT_F64;
        H2BArgs a = base_h2b(p, x);
        a.xptrs = xptrs;
        a.gtab = f64 ? (const void*)p->d_g64 : (const void*)p->d_g32;
        a.tw = f64 ? (const void*)p->d_tw64 : (const void*)p->d_tw32;
        a.seeds = seeds;
        a.count = count;
        a.jobs = (kind == 0 ? p->d_jobs_loc : p->d_jobs_est) + j0;
        a.njobs = nj;
        a.groundv = p->d_groundv;
        a.R_loc = p->d.R_loc;
        a.raw = raw;
        a.raw_rounds = p->nslots;
        HIP_TRY(launch_h2b_pair(a, in_c128(p), f64, s));
    }
    return SFFT_OK;
}

// Per-signal workspace and output pointers advanced to signal `off`.
void offset_decode(const sfft_plan_s* p, DecodeArgs& D, uint32_t off) {
    const uint64_t Bm = p->Bmax, Z = p->capz, o = off;
    D.raw += o * p->R * 2 * p->nhash * Bm;
    D.work += o * 4 * Bm;
    D.cand_i += o * Bm;
    D.cand_v += o * 2 * Bm;
    D.zidx += o * 2 * Z;
    D.zval += o * 4 * Z;
    D.est += o * Z * p->R * 2;
    D.fin += o * 2 * Z;
    D.gtmp += o * Z * 4;
    D.ecount += o * Z;
    D.eflag += o * Z * p->R;
    D.egrp += o * Z * p->R;
    D.eord += o * Z * p->R;
    D.ecoef += o * Z * p->R * 2;
    D.state += o * kStateWords;
    if (D.seeds) D.seeds += o;
    D.out_idx += o * p->cap;
    D.out_val += o * 2 * p->cap;
    D.out_count += o;
    if (D.out_info) D.out_info += o * 4;
}

void offset_general(const sfft_plan_s* p, GeneralArgs& G, uint32_t off) {
    const uint64_t Bm = p->Bmax, Z = p->capz, o = off;
    const uint64_t meas = (uint64_t)p->R * p->d.R_est;
    G.raw += o * p->nslots * 4 * Bm;
    G.cand_i += o * Bm;
    G.cand_v += o * 2 * Bm;
    G.cand_e += o * p->d.R_est * 2 * Bm;
    G.cand_n += o * Bm;
    G.zidx += o * 2 * Z;
    G.zval += o * 4 * Z;
    G.est += o * Z * meas * 2;
    G.fin += o * 2 * Z;
    G.gtmp += o * Z * 4;
    G.ecount += o * Z;
    G.gfirst += o * (Bm + 1);
    G.gent += o * Z;
    G.cand_raw += o * Bm;
    G.cand_cnt += o;
    G.eflag += o * Z * meas;
    G.egrp += o * Z * meas;
    G.eord += o * Z * meas;
    G.ecoef += o * Z * meas * 2;
    G.gterm += o * std::max<uint64_t>(p->R, p->d.R_est) * Z * 4;
    G.state += o * kStateWords;
    if (G.seeds) G.seeds += o;
    G.out_idx += o * p->cap;
    G.out_val += o * 2 * p->cap;
    G.out_count += o;
    if (G.out_info) G.out_info += o * 4;
}

// Workgroup size of an exact-mode pair launch over rounds [r0, r1): the
// plan's hash_threads, halved (not below 256) while it exceeds the largest
// B_r of those rounds - more threads than bins only split each residue's
// sum into more parts.
uint32_t pair_threads(const sfft_plan_s* p, uint32_t r0, uint32_t r1) {
    uint32_t maxB = 0;
    for (uint32_t r = r0; r < r1; ++r) maxB = std::max(maxB, p->geom[r].B);
    uint32_t t = p->d.hash_threads;
    while (t > 256 && t > maxB) t >>= 1;
    return t;
}

// Part 0 of a chunk [off, off + cnt): state reset + HashToBins of every
// round; part 1: decode loop + re-estimation and output.
sfft_status_t enqueue_chunk(sfft_plan_s* p, int part, uint32_t off, uint32_t cnt, const void* x,
                            const uint64_t* seeds, uint64_t* idx, double* val, uint32_t* ocnt, uint32_t* info,
                            hipStream_t s, const void* const* xptrs = nullptr) {
    const size_t elem = in_c128(p) ? 16 : 8;
    const void* xc = xptrs ? nullptr : static_cast<const char*>(x) + (size_t)off * p->d.n * elem;
    const void* const* xpc = xptrs ? xptrs + off : nullptr;
    const uint64_t* sc = seeds ? seeds + off : nullptr;
    DecodeArgs D = base_decode(p, cnt, seeds, p->raw, idx, val, ocnt, info);
    offset_decode(p, D, off);
    if (general_mode(p)) {
        GeneralArgs G = base_general(p, cnt, seeds, p->raw, idx, val, ocnt, info);
        offset_general(p, G, off);
        if (part == 0) {
            HIP_TRY(launch_exact_init(D, s));
            double* rawc = p->raw + (uint64_t)off * p->nslots * 4 * p->Bmax;
            ST_TRY(enqueue_general_hash(p, xc, cnt, sc, rawc, 0, p->R, s, xpc));
        } else {
            HIP_TRY(launch_general_decode(G, 0, p->R, s));
            HIP_TRY(launch_general_finish(G, s));
        }
        return SFFT_OK;
    }
    // the pairs of rounds [a.round_lo, + a.nrounds): the leading stream-mode
    // rounds (windows shrink with the round, so they come first) in one
    // stream launch, the others in one pair launch or its split form
    auto hash = [&](H2BArgs& a) -> sfft_status_t {
        uint32_t ns = 0;
        while (ns < a.nrounds && p->stream_round[a.round_lo + ns]) ++ns;
        if (ns > 0) {
            H2BArgs b = a;
            b.nrounds = ns;
            b.parts = p->stream_parts;
            b.partial = p->split_partial;
            HIP_TRY(launch_h2b_pair_stream(b, in_c128(p), loc_f64(p), s));
        }
        if (ns == a.nrounds) return SFFT_OK;
        H2BArgs g = a;
        g.round_lo = a.round_lo + ns;
        g.nrounds = a.nrounds - ns;
        g.threads = pair_threads(p, g.round_lo, g.round_lo + g.nrounds);
        if (p->d.hash_split > 1) {
            g.parts = p->d.hash_split;
            g.partial = p->split_partial;
            HIP_TRY(launch_h2b_pair_split(g, in_c128(p), loc_f64(p), s));
        } else {
            HIP_TRY(launch_h2b_pair(g, in_c128(p), loc_f64(p), s));
        }
        return SFFT_OK;
    };
    H2BArgs a = base_h2b(p, xc);
    a.xptrs = xpc;
    a.seeds = sc;
    a.count = cnt;
    a.raw = p->raw + (uint64_t)off * p->R * 2 * p->nhash * p->Bmax;
    a.raw_rounds = p->R;
    if (part == 0) {
        HIP_TRY(launch_exact_init(D, s));
        a.round_lo = 0;
        a.nrounds = p->group_end[0];
        a.threads = pair_threads(p, 0, p->group_end[0]);
        ST_TRY(hash(a));
        return SFFT_OK;
    }
    a.state = D.state;
    uint32_t r0 = 0;
    for (size_t g = 0; g < p->group_end.size(); ++g) {
        const uint32_t r1 = p->group_end[g];
        if (g > 0) {
            a.round_lo = r0;
            a.nrounds = r1 - r0;
            a.threads = pair_threads(p, r0, r1);
            ST_TRY(hash(a));
        }
        D.r_begin = r0;
        D.r_end = r1;
        HIP_TRY(launch_exact_decode(D, s));
        r0 = r1;
    }
    HIP_TRY(launch_exact_finish(D, s));
    return SFFT_OK;
}

// Chunks of a batch (default one).  Several chunks let the decode of chunk c
// run beside the HashToBins of chunk c+1, but the decode is latency bound
// and slows sharply next to a kernel that saturates HBM: measured at
// 512 x 2^22, k = 256, one chunk 3.69 ms, two 4.17 ms, four 5.50 ms.
// The plan's `chunks` sets the count; 0 takes SFFT_BATCH_CHUNKS, else one.
uint32_t batch_chunks(const sfft_plan_s* p, uint32_t count) {
    uint32_t c = p->d.chunks;
    if (c == 0) {
        const char* e = std::getenv("SFFT_BATCH_CHUNKS");
        c = e ? (uint32_t)std::atoi(e) : 1u;
    }
    return std::max(1u, std::min({c, kMaxChunks, count}));
}

// part 0 (state reset + first HashToBins launch), 1 (the rest) or 2 (both,
// one graph).
sfft_status_t capture_part(sfft_plan_s* p, int part, uint32_t off, uint32_t cnt, const void* x,
                           const uint64_t* seeds, uint64_t* idx, double* val, uint32_t* ocnt, uint32_t* info,
                           hipGraphExec_t* out) {
    hipGraph_t graph = nullptr;
    HIP_TRY(hipStreamBeginCapture(p->capture_stream, hipStreamCaptureModeThreadLocal));
    sfft_status_t st = enqueue_chunk(p, part == 1 ? 1 : 0, off, cnt, x, seeds, idx, val, ocnt, info,
                                     p->capture_stream);
    if (st == SFFT_OK && part == 2)
        st = enqueue_chunk(p, 1, off, cnt, x, seeds, idx, val, ocnt, info, p->capture_stream);
    hipError_t ee = hipStreamEndCapture(p->capture_stream, &graph);
    if (st != SFFT_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return st;
    }
    if (ee != hipSuccess) return fail(SFFT_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(ee));
    hipError_t ie = hipGraphInstantiate(out, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ie != hipSuccess) {
        *out = nullptr;
        return fail(SFFT_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(ie));
    }
    return SFFT_OK;
}

}  // namespace

// ================================================================== C ABI ==
extern "C" {

const char* sfft_status_string(sfft_status_t s) {
    switch (s) {
        case SFFT_OK: return "SFFT_OK";
        case SFFT_EINVAL: return "SFFT_EINVAL";
        case SFFT_ENOTPOW2: return "SFFT_ENOTPOW2";
        case SFFT_ENOMEM: return "SFFT_ENOMEM";
        case SFFT_EBUDGET: return "SFFT_EBUDGET";
        case SFFT_EHIP: return "SFFT_EHIP";
        case SFFT_ETRUNC: return "SFFT_ETRUNC";
        case SFFT_EUNSUPPORTED: return "SFFT_EUNSUPPORTED";
        case SFFT_EAGAIN: return "SFFT_EAGAIN";
        case SFFT_ECANCELED: return "SFFT_ECANCELED";
    }
    return "SFFT_UNKNOWN";
}

const char* sfft_last_error(void) { return g_last_error.c_str(); }

uint64_t sfft_splitmix64(uint64_t seed, uint64_t c) { return splitmix64(seed, c); }

uint64_t sfft_window_w(uint64_t n, uint32_t B, double alpha, double delta, uint32_t window) {
    if (window == 0) return sfft_default_w(n, B, alpha, delta);
    if (window != 1 || !is_pow2(n) || !is_pow2(B) || B > n || !(alpha > 0.0 && alpha < 1.0) ||
        !(delta > 0.0 && delta < 1.0))
        return 0;
    return kaiser_w(n, B, alpha, delta);
}

uint64_t sfft_default_w(uint64_t n, uint32_t B, double alpha, double delta) {
    if (!is_pow2(n) || !is_pow2(B) || B > n || !(alpha > 0 && alpha < 1) || !(delta > 0 && delta < 1)) return 0;
    return default_w(n, B, alpha, delta);
}

sfft_status_t sfft_desc_init(sfft_plan_desc_t* d, uint64_t n, uint32_t k, uint32_t B, uint64_t w, uint64_t seed) {
    if (!d) return fail(SFFT_EINVAL, "desc is NULL");
    std::memset(d, 0, sizeof(*d));
    d->n = n;
    d->k = k;
    d->B = B;
    d->w = w;
    d->seed = seed;
    d->mode = SFFT_MODE_EXACT;
    d->in_dtype = SFFT_C64;
    d->loc_prec = n >= (1ull << 20) ? SFFT_F64 : SFFT_F32;
    d->est_prec = SFFT_F32;
    d->alpha = 0.5;
    d->delta = 1e-9;
    d->theta = 0.25;
    d->g_min = 0.4;
    d->s = 0.125;
    d->rounds = 0;
    d->b_min = 0;
    d->patience = 3;
    d->t = 16;
    d->R_loc = 3;
    d->R_est = 7;
    d->cap = 0;
    d->flags = 0;
    d->max_batch = 1;
    d->hash_threads = 256;
    d->chunks = 0;
    d->stop_count = 0;
    d->stop_patience = 2;
    d->group0 = 0;
    d->ratio_tol = 0.0;
    d->group_step = 0;
    d->hash_order = 0;
    d->alpha_decay = 0.0;
    d->hash_split = 0;
    d->hash_mode = 0;
    d->refine_shift = 0;
    d->refine_window = 0;
    d->window = 0;
    return SFFT_OK;
}

sfft_status_t sfft_validate_params(const sfft_plan_desc_t* d) {
    if (!d) return fail(SFFT_EINVAL, "desc is NULL");
    if (!is_pow2(d->n) || d->n < 4) return fail(SFFT_ENOTPOW2, "n must be a power of two >= 4");
    if (d->n > (1ull << 40)) return fail(SFFT_EINVAL, "n must be at most 2^40");
    if (d->k < 1 || d->k >= d->n) return fail(SFFT_EINVAL, "k must satisfy 1 <= k < n");
    if (!is_pow2(d->B) || d->B < 2) return fail(SFFT_ENOTPOW2, "B must be a power of two >= 2");
    if (d->B > d->n) return fail(SFFT_EINVAL, "B must be at most n");
    if (d->w != 0 && (d->w % d->B != 0 || d->w < d->B || d->w > d->n))
        return fail(SFFT_EINVAL, "w must be a multiple of B with B <= w <= n (or 0)");
    if (d->mode != SFFT_MODE_EXACT && d->mode != SFFT_MODE_GENERAL) return fail(SFFT_EINVAL, "bad mode");
    if (d->in_dtype != SFFT_C64 && d->in_dtype != SFFT_C128) return fail(SFFT_EINVAL, "bad in_dtype");
    if ((d->loc_prec != SFFT_F32 && d->loc_prec != SFFT_F64) || (d->est_prec != SFFT_F32 && d->est_prec != SFFT_F64))
        return fail(SFFT_EINVAL, "bad precision");
    if (!(d->alpha > 0.0 && d->alpha < 1.0)) return fail(SFFT_EINVAL, "alpha must be in (0, 1)");
    if (!(d->delta > 0.0 && d->delta < 1.0)) return fail(SFFT_EINVAL, "delta must be in (0, 1)");
    if (!(d->theta > 0.0)) return fail(SFFT_EINVAL, "theta must be positive");
    if (!(d->g_min > 0.0 && d->g_min <= 1.0)) return fail(SFFT_EINVAL, "g_min must be in (0, 1]");
    if (d->rounds > kMaxRounds) return fail(SFFT_EINVAL, "rounds must be in [1, 32] (0 = mode default)");
    if (d->patience < 1) return fail(SFFT_EINVAL, "patience must be >= 1");
    if (d->b_min != 0 && (!is_pow2(d->b_min) || d->b_min < 2)) return fail(SFFT_EINVAL, "b_min must be 0 or a power of two >= 2");
    if (d->max_batch < 1 || d->max_batch > (1u << 20)) return fail(SFFT_EINVAL, "max_batch must be in [1, 2^20]");
    if (d->hash_threads != 0 && !h2b_threads_ok(d->hash_threads))
        return fail(SFFT_EINVAL, "hash_threads must be 256, 512 or 1024 (or 0)");
    if (d->chunks > kMaxChunks) return fail(SFFT_EINVAL, "chunks must be in [0, 8]");
    if (d->stop_patience < 1) return fail(SFFT_EINVAL, "stop_patience must be >= 1");
    if (d->group0 > kMaxRounds) return fail(SFFT_EINVAL, "group0 must be in [0, 32]");
    if (!(d->ratio_tol >= 0.0 && d->ratio_tol < 1.0)) return fail(SFFT_EINVAL, "ratio_tol must be in [0, 1)");
    if (d->group_step > kMaxRounds) return fail(SFFT_EINVAL, "group_step must be in [0, 32]");
    if (d->hash_order > 2) return fail(SFFT_EINVAL, "hash_order must be 0, 1 or 2");
    if (!(d->alpha_decay >= 0.0 && d->alpha_decay <= 1.0)) return fail(SFFT_EINVAL, "alpha_decay must be in [0, 1]");
    if (d->mode == SFFT_MODE_GENERAL && d->alpha_decay != 0.0 && d->alpha_decay != 1.0)
        return fail(SFFT_EINVAL, "alpha_decay applies to exact mode only");
    if (d->hash_mode > 2) return fail(SFFT_EINVAL, "hash_mode must be 0, 1 or 2");
    if (d->hash_mode != 0 && (d->mode == SFFT_MODE_GENERAL || d->chunks > 1))
        return fail(SFFT_EINVAL, "hash_mode applies to exact mode with at most one chunk");
    if (d->refine_window > 1024) return fail(SFFT_EINVAL, "refine_window must be in [0, 1024]");
    if (d->window > 1) return fail(SFFT_EINVAL, "window must be 0 (Gaussian) or 1 (Kaiser-Bessel)");
    if (d->refine_shift != 0) {
        const uint64_t E = d->refine_window ? d->refine_window : 16;
        if (d->mode == SFFT_MODE_GENERAL) return fail(SFFT_EINVAL, "refine_shift applies to exact mode only");
        if (d->refine_shift < 2 || d->refine_shift >= d->n || d->refine_shift * (2 * E + 1) >= d->n)
            return fail(SFFT_EINVAL, "refine_shift A needs 2 <= A and A (2 refine_window + 1) < n");
        if (d->hash_split > 1 || d->hash_mode != 0)
            return fail(SFFT_EINVAL, "refine_shift needs hash_split <= 1 and hash_mode 0");
    }
    if (d->hash_split > 64) return fail(SFFT_EINVAL, "hash_split must be in [0, 64]");
    if (d->hash_split > 1 && (d->mode == SFFT_MODE_GENERAL || d->chunks > 1))
        return fail(SFFT_EINVAL, "hash_split applies to exact mode with at most one chunk");
    const uint32_t cap = d->cap ? d->cap : d->k;
    if (cap > kMaxZ) return fail(SFFT_EINVAL, "cap must be at most 8192");
    if (d->mode == SFFT_MODE_GENERAL) {
        if (d->t < 4 || d->t > kMaxT || !is_pow2(d->t) || d->R_loc < 1 || d->R_loc > kMaxRLoc || d->R_est < 1 ||
            d->R_est > kMaxREst || !(d->s > 0 && d->s < 1))
            return fail(SFFT_EINVAL, "bad LocateInner/EstimateValues parameters (t a power of two in [4, 64], R_loc in [1, 8], R_est in [1, 32])");
        const uint32_t R = d->rounds ? d->rounds : general_default_rounds(d->k);
        if ((uint64_t)R * d->R_est > 64) return fail(SFFT_EINVAL, "rounds * R_est must be at most 64");
        if (4ull * std::max<uint32_t>(d->k, 16u) > kMaxZ) return fail(SFFT_EUNSUPPORTED, "general mode needs k <= 1024");
        if ((d->n / d->B) > (1ull << 40)) return fail(SFFT_EINVAL, "n / B too large");
    }
    if (d->B > kMaxZ) return fail(SFFT_EUNSUPPORTED, "B exceeds 4096, the LDS limit of the pair and decode kernels");
    return SFFT_OK;
}

sfft_status_t sfft_plan_ex(const sfft_plan_desc_t* desc, sfft_plan_t* out) {
    if (!desc || !out) return fail(SFFT_EINVAL, "NULL argument");
    sfft_plan_desc_t d = *desc;
    ST_TRY(resolve_and_validate(d));
    if (d.w < d.B || d.w % d.B) return fail(SFFT_EINVAL, "resolved window is not a multiple of B");
    sfft_plan_s* p = new (std::nothrow) sfft_plan_s();
    if (!p) return fail(SFFT_ENOMEM, "host allocation failed");
    p->d = d;
    sfft_status_t s = build_plan(p);
    if (s != SFFT_OK) {
        sfft_destroy(p);
        return s;
    }
    *out = p;
    return SFFT_OK;
}

uint64_t sfft_plan_device_bytes(const sfft_plan_desc_t* desc) {
    if (!desc) return 0;
    sfft_plan_desc_t d = *desc;
    if (resolve_and_validate(d) != SFFT_OK || d.w < d.B || d.w % d.B) return 0;
    sfft_plan_s p;
    p.d = d;
    p.dry = true;
    if (build_plan(&p) != SFFT_OK) return 0;
    return p.device_bytes;
}

// Gathered samples of exact round r's pair launch: w_r + 1, plus A (or w_r
// for A > w_r) with the refinement hashing.
uint64_t refined_samples(const sfft_plan_s* p, uint32_t r) {
    const uint64_t w = p->geom[r].w, A = p->d.refine_shift;
    if (general_mode(p) || A == 0) return w + 1;
    return A < w + 1 ? w + A : 2 * w + 1;
}

uint64_t sfft_plan_samples(const sfft_plan_desc_t* desc) {
    if (!desc) return 0;
    sfft_plan_desc_t d = *desc;
    if (resolve_and_validate(d) != SFFT_OK || d.w < d.B || d.w % d.B) return 0;
    sfft_plan_s p;
    p.d = d;
    p.dry = true;
    if (build_plan(&p) != SFFT_OK) return 0;
    uint64_t samples = 0;
    if (general_mode(&p)) {
        // every round: nlev * R_loc location pairs and R_est estimation hashings
        for (uint32_t r = 0; r < p.R; ++r)
            samples += (2ull * p.groundv[r].nloc + d.R_est) * p.geom[r].w;
    } else {
        // the pair of each round of group 0 (the rounds before the earliest
        // stop): w_r + 1 gathered samples, or the whole signal in stream mode
        for (uint32_t r = 0; r < p.group_end[0]; ++r) samples += p.stream_round[r] ? d.n : refined_samples(&p, r);
    }
    return samples;
}

uint32_t sfft_plan_stream_rounds(const sfft_plan_desc_t* desc) {
    if (!desc) return 0;
    sfft_plan_desc_t d = *desc;
    if (resolve_and_validate(d) != SFFT_OK || d.w < d.B || d.w % d.B) return 0;
    sfft_plan_s p;
    p.d = d;
    p.dry = true;
    if (build_plan(&p) != SFFT_OK || general_mode(&p)) return 0;
    uint32_t c = 0;
    for (uint32_t r = 0; r < p.group_end[0]; ++r) c += p.stream_round[r];
    return c;
}

sfft_status_t sfft_plan(uint64_t n, uint32_t k, uint32_t B, uint64_t w, uint64_t seed, sfft_plan_t* out) {
    sfft_plan_desc_t d;
    sfft_desc_init(&d, n, k, B, w, seed);
    return sfft_plan_ex(&d, out);
}

sfft_status_t sfft_plan_get_desc(sfft_plan_t p, sfft_plan_desc_t* out) {
    if (!p || !out) return fail(SFFT_EINVAL, "NULL argument");
    *out = p->d;
    return SFFT_OK;
}

sfft_status_t sfft_destroy(sfft_plan_t p) {
    if (!p) return SFFT_OK;
    if (p->graph.launched) {
        (void)hipEventSynchronize(p->graph.launched);
        (void)hipEventDestroy(p->graph.launched);
    }
    for (uint32_t c = 0; c < kMaxChunks; ++c) {
        if (p->graph.exec_h[c]) (void)hipGraphExecDestroy(p->graph.exec_h[c]);
        if (p->graph.exec_d[c]) (void)hipGraphExecDestroy(p->graph.exec_d[c]);
    }
    if (p->capture_stream) (void)hipStreamDestroy(p->capture_stream);
    if (p->aux_stream) (void)hipStreamDestroy(p->aux_stream);
    hipEvent_t* evs[] = {&p->ev_fork, &p->ev_join, &p->ev_t0, &p->ev_t1};
    for (hipEvent_t* e : evs)
        if (*e) (void)hipEventDestroy(*e);
    for (uint32_t c = 0; c < kMaxChunks; ++c)
        for (hipEvent_t e : {p->ev_ready[c], p->ev_h0[c], p->ev_h1[c], p->ev_d0[c], p->ev_d1[c]})
            if (e) (void)hipEventDestroy(e);
    for (void* q : p->allocations) (void)hipFree(q);
    delete p;
    return SFFT_OK;
}

sfft_status_t sfft_plan_timings(sfft_plan_t p, double* ms_host, uint32_t n_out) {
    if (!p || !ms_host || n_out < 4) return fail(SFFT_EINVAL, "bad argument");
    if (!(p->d.flags & SFFT_FLAG_TIMING) || !p->timed_once) return fail(SFFT_EINVAL, "timing not enabled or nothing ran");
    double h = 0.0, d = 0.0;
    for (uint32_t c = 0; c < p->timed_chunks; ++c) {
        float a = 0.f, b = 0.f;
        HIP_TRY(hipEventElapsedTime(&a, p->ev_h0[c], p->ev_h1[c]));
        HIP_TRY(hipEventElapsedTime(&b, p->ev_d0[c], p->ev_d1[c]));
        h += a;
        d += b;
    }
    float tail = 0.f, tot = 0.f;
    HIP_TRY(hipEventElapsedTime(&tail, p->ev_h1[p->timed_chunks - 1], p->ev_t1));
    HIP_TRY(hipEventElapsedTime(&tot, p->ev_t0, p->ev_t1));
    ms_host[0] = h;
    ms_host[1] = d;
    ms_host[2] = tail;
    ms_host[3] = tot;
    if (n_out > 4) ms_host[4] = (double)p->timed_chunks;
    return SFFT_OK;
}

sfft_status_t sfft_plan_raw_slot(sfft_plan_t p, uint32_t sig, uint32_t slot, double* out_dev, uint32_t* B_r_out,
                                 void* stream) {
    if (!p || !out_dev || !B_r_out) return fail(SFFT_EINVAL, "NULL argument");
    const uint32_t nslots = general_mode(p) ? p->nslots : p->R;
    if (sig >= p->d.max_batch || slot >= nslots) return fail(SFFT_EINVAL, "signal or slot out of range");
    uint32_t round = slot;
    if (general_mode(p)) {
        round = 0;
        for (uint32_t r = 0; r < p->R; ++r)
            if (p->groundv[r].slot0 <= slot) round = r;
    }
    const uint32_t B = p->geom[round].B;
    const double* src = p->raw + ((uint64_t)sig * nslots + slot) * 2 * p->nhash * (uint64_t)p->Bmax;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    HIP_TRY(hipMemcpyAsync(out_dev, src, 2 * sizeof(double) * B, hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipMemcpyAsync(out_dev + 2 * (size_t)B, src + 2 * (size_t)p->Bmax, 2 * sizeof(double) * B,
                           hipMemcpyDeviceToDevice, s));
    *B_r_out = B;
    return SFFT_OK;
}

sfft_status_t sfft_plan_raw_refine(sfft_plan_t p, uint32_t sig, uint32_t round, double* out_dev, uint32_t* B_r_out,
                                   void* stream) {
    if (!p || !out_dev || !B_r_out) return fail(SFFT_EINVAL, "NULL argument");
    if (p->nhash != 3) return fail(SFFT_EINVAL, "the plan has no refinement hashing");
    if (sig >= p->d.max_batch || round >= p->R) return fail(SFFT_EINVAL, "signal or round out of range");
    const uint32_t B = p->geom[round].B;
    const double* src = p->raw + (((uint64_t)sig * p->R + round) * 3 + 2) * 2 * (uint64_t)p->Bmax;
    HIP_TRY(hipMemcpyAsync(out_dev, src, 2 * sizeof(double) * B, hipMemcpyDeviceToDevice,
                           reinterpret_cast<hipStream_t>(stream)));
    *B_r_out = B;
    return SFFT_OK;
}

uint32_t sfft_plan_desc_bytes(void) { return (uint32_t)sizeof(sfft_plan_desc_t); }

uint64_t sfft_plan_h2b_bytes(sfft_plan_t p, uint32_t count) {
    if (!p) return 0;
    const uint64_t s_in = p->d.in_dtype == SFFT_C128 ? 16 : 8;
    // exact mode: the first launch covers round group 0; general mode: every round
    const uint32_t R = p->group_end.empty() ? p->R : p->group_end[0];
    uint64_t per = 0;
    for (uint32_t r = 0; r < R; ++r) per += refined_samples(p, r) * s_in + (uint64_t)p->nhash * p->geom[r].B * 16ull;
    return per * count;
}

sfft_status_t sfft_plan_round_groups(sfft_plan_t p, uint32_t* ends_host, uint32_t max, uint32_t* n_groups) {
    if (!p || !n_groups) return fail(SFFT_EINVAL, "NULL argument");
    std::vector<uint32_t> ends = p->group_end;
    if (ends.empty()) ends.push_back(p->R);
    for (uint32_t g = 0; g < ends.size() && g < max; ++g)
        if (ends_host) ends_host[g] = ends[g];
    *n_groups = (uint32_t)ends.size();
    return SFFT_OK;
}

sfft_status_t sfft_hash_pair_raw(sfft_plan_t p, const void* x_dev, uint64_t sigma, uint64_t a, uint64_t beta,
                                 uint64_t b, uint32_t B_r, int32_t prec, double* out0_dev, double* out1_dev,
                                 void* stream) {
    if (!p || !x_dev || !out0_dev || !out1_dev) return fail(SFFT_EINVAL, "NULL argument");
    const uint64_t n = p->d.n;
    if ((sigma & 1) == 0 || sigma >= n || a >= n || b >= n || beta >= n)
        return fail(SFFT_EINVAL, "sigma must be odd and sigma, a, b, beta < n");
    if (prec != SFFT_F32 && prec != SFFT_F64) return fail(SFFT_EINVAL, "bad precision");
    uint32_t round = p->R;
    for (uint32_t r = 0; r < p->R; ++r)
        if (p->geom[r].B == B_r) {
            round = r;
            break;
        }
    if (round == p->R) return fail(SFFT_EINVAL, "B_r is not a bin count of the plan's schedule");
    const RoundDev& g = p->geom[round];
    std::lock_guard<std::mutex> lock(p->mu);
    H2BArgs A = base_h2b(p, x_dev);
    A.gtab = prec == SFFT_F64 ? (const void*)p->d_g64 : (const void*)p->d_g32;
    A.tw = prec == SFFT_F64 ? (const void*)p->d_tw64 : (const void*)p->d_tw32;
    A.explicit_job = 1;
    A.sigma = sigma;
    A.a = a;
    A.beta = beta;
    A.b = b;
    A.count = 1;
    A.round_lo = round;
    A.nrounds = 1;
    A.raw = p->p_raw;
    A.raw_rounds = 1;
    A.gamma = 0;
    const int64_t iB = g.B, iw = (int64_t)g.w, ib = (int64_t)beta;
    uint64_t mc;
    if (beta < g.w) {
        mc = (uint64_t)(floordiv(g.t0 + iw - 1, iB) - floordiv(g.t0 - ib - (iB - 1), iB) + 1);
    } else {   // two disjoint segments, each with its own table
        const int64_t s0 = floordiv(g.t0 - ib + iw - 1, iB) - floordiv(g.t0 - ib - (iB - 1), iB) + 1;
        const int64_t s1 = floordiv(g.t0 + iw - 1, iB) - floordiv(g.t0 - (iB - 1), iB) + 1;
        mc = (uint64_t)std::max(s0, s1);
    }
    A.mcap = (uint32_t)mc;
    if (h2b_pair_lds_bytes(p->Bmax, A.mcap, prec == SFFT_F64, A.threads) > 160 * 1024)
        return fail(SFFT_EUNSUPPORTED, "pair does not fit in LDS");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    HIP_TRY(launch_h2b_pair(A, in_c128(p), prec == SFFT_F64, s));
    HIP_TRY(hipMemcpyAsync(out0_dev, p->p_raw, 2 * sizeof(double) * g.B, hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipMemcpyAsync(out1_dev, p->p_raw + 2 * (size_t)p->Bmax, 2 * sizeof(double) * g.B,
                           hipMemcpyDeviceToDevice, s));
    return SFFT_OK;
}

sfft_status_t sfft_execute(sfft_plan_t p, const void* x_dev, uint64_t* idx_host, double* val_host, uint32_t cap,
                           uint32_t* count_host, uint32_t* info_host, void* stream) {
    if (!p || !x_dev || !idx_host || !val_host || !count_host || cap < 1) return fail(SFFT_EINVAL, "bad argument");
    if (p->d.refine_shift) return fail(SFFT_EUNSUPPORTED, "refine_shift needs the batched path (sfft_execute_batch)");
    std::lock_guard<std::mutex> lock(p->mu);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const uint64_t n = p->d.n;
    DecodeArgs D = base_decode(p, 1, nullptr, p->p_raw, p->p_idx, p->p_val, p->p_count, p->p_info);
    HIP_TRY(launch_exact_init(D, s));
    uint32_t st[kStateWords];
    if (general_mode(p)) {
        // one request: each round's hashings in one launch pair, then its decode
        GeneralArgs G = base_general(p, 1, nullptr, p->p_raw, p->p_idx, p->p_val, p->p_count, p->p_info);
        for (uint32_t r = 0; r < p->R; ++r) {
            ST_TRY(enqueue_general_hash(p, x_dev, 1, nullptr, p->p_raw, r, r + 1, s));
            HIP_TRY(launch_general_decode(G, r, r + 1, s));
        }
        HIP_TRY(launch_general_finish(G, s));
    }
    for (uint32_t r = 0; r < p->R && !general_mode(p); ++r) {
        const RoundDev& g = p->geom[r];
        H2BArgs a = base_h2b(p, x_dev);
        a.sigma = draw_sigma(p->d.seed, n, r);
        a.b = draw_b(p->d.seed, n, r);
        a.a = 0;
        a.beta = 1;
        a.raw = p->p_raw;
        a.raw_rounds = p->R;
        a.partial = p->p_partial;
        const int64_t iB = g.B;
        const int64_t Lmin = floordiv(g.t0 - 1 - (iB - 1), iB);
        const int64_t Lmax = floordiv(g.t0 + (int64_t)g.w - 1, iB);
        const uint64_t nL = (uint64_t)(Lmax - Lmin + 1);
        a.lchunk = (uint32_t)((nL + p->p_parts_max - 1) / p->p_parts_max);
        a.parts = (uint32_t)((nL + a.lchunk - 1) / a.lchunk);
        a.mcap = a.lchunk + 2;
        HIP_TRY(launch_h2b_split(a, r, in_c128(p), loc_f64(p), s));
        HIP_TRY(launch_h2b_reduce(a, r, loc_f64(p), s));
        D.r_begin = r;
        D.r_end = r + 1;
        HIP_TRY(launch_exact_decode(D, s));
        HIP_TRY(hipMemcpyAsync(st, p->state, sizeof(st), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (st[ST_DONE]) break;
    }
    if (!general_mode(p)) HIP_TRY(launch_exact_finish(D, s));
    uint32_t cnt = 0, info[4];
    HIP_TRY(hipMemcpyAsync(&cnt, p->p_count, sizeof(cnt), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(info, p->p_info, sizeof(info), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    const uint32_t take = std::min(cnt, cap);
    std::vector<uint64_t> hidx(p->cap);
    std::vector<double> hval(2 * (size_t)p->cap);
    HIP_TRY(hipMemcpy(hidx.data(), p->p_idx, sizeof(uint64_t) * p->cap, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(hval.data(), p->p_val, sizeof(double) * 2 * p->cap, hipMemcpyDeviceToHost));
    std::copy(hidx.begin(), hidx.begin() + take, idx_host);
    std::copy(hval.begin(), hval.begin() + 2 * take, val_host);
    *count_host = take;
    if (info_host) std::copy(info, info + 4, info_host);
    if ((info[SFFT_INFO_FLAGS] & 1u) || cnt > cap) return fail(SFFT_ETRUNC, "more coefficients than cap");
    return SFFT_OK;
}

sfft_status_t sfft_execute_batch(sfft_plan_t p, const void* x_dev, uint32_t count, const uint64_t* seeds_dev,
                                 uint64_t* idx_dev, double* val_dev, uint32_t* count_dev, uint32_t* info_dev,
                                 void* stream) {
    if (!p || !x_dev || !idx_dev || !val_dev || !count_dev) return fail(SFFT_EINVAL, "NULL argument");
    if (count < 1 || count > p->d.max_batch) return fail(SFFT_EINVAL, "count must be in [1, max_batch]");
    std::lock_guard<std::mutex> lock(p->mu);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const bool timing = (p->d.flags & SFFT_FLAG_TIMING) != 0;
    const char* nog = std::getenv("SFFT_NO_GRAPH");
    const bool use_graph = !(nog && nog[0] == '1');
    const uint32_t C = batch_chunks(p, count);
    const uint32_t per = (count + C - 1) / C;
    // one chunk without phase events: the whole step is one graph, with no
    // launch boundary between the first HashToBins launch and the decode
    const bool whole = use_graph && C == 1 && !timing;
    GraphCache& gc = p->graph;
    if (use_graph) {
        const bool hit = gc.exec_h[0] && gc.chunks == C && gc.whole == whole && gc.x == x_dev && gc.count == count &&
                         gc.seeds == seeds_dev && gc.o1 == idx_dev && gc.o2 == val_dev && gc.o3 == count_dev &&
                         gc.o4 == info_dev;
        if (!hit) {
            if (gc.launched) HIP_TRY(hipEventSynchronize(gc.launched));
            for (uint32_t c = 0; c < kMaxChunks; ++c) {
                if (gc.exec_h[c]) HIP_TRY(hipGraphExecDestroy(gc.exec_h[c]));
                if (gc.exec_d[c]) HIP_TRY(hipGraphExecDestroy(gc.exec_d[c]));
                gc.exec_h[c] = gc.exec_d[c] = nullptr;
            }
            gc.exec_h[0] = nullptr;
            if (whole) {
                ST_TRY(capture_part(p, 2, 0, count, x_dev, seeds_dev, idx_dev, val_dev, count_dev, info_dev,
                                    &gc.exec_h[0]));
            } else {
                for (uint32_t c = 0; c < C; ++c) {
                    const uint32_t off = c * per, cnt = std::min(per, count - off);
                    ST_TRY(capture_part(p, 0, off, cnt, x_dev, seeds_dev, idx_dev, val_dev, count_dev, info_dev,
                                        &gc.exec_h[c]));
                    ST_TRY(capture_part(p, 1, off, cnt, x_dev, seeds_dev, idx_dev, val_dev, count_dev, info_dev,
                                        &gc.exec_d[c]));
                }
            }
            gc.whole = whole;
            gc.chunks = C;
            gc.x = x_dev;
            gc.count = count;
            gc.seeds = seeds_dev;
            gc.o1 = idx_dev;
            gc.o2 = val_dev;
            gc.o3 = count_dev;
            gc.o4 = info_dev;
        }
    }
    // fork: the auxiliary stream follows everything already queued on s.  A
    // single chunk has nothing to overlap: its decode follows on s itself
    // (a cross-stream wait costs tens of microseconds per step)
    hipStream_t ds = C > 1 ? p->aux_stream : s;
    if (use_graph && !gc.launched) HIP_TRY(hipEventCreateWithFlags(&gc.launched, hipEventDisableTiming));
    if (whole) {
        HIP_TRY(hipGraphLaunch(gc.exec_h[0], s));
        HIP_TRY(hipEventRecord(gc.launched, s));
        return SFFT_OK;
    }
    if (timing) HIP_TRY(hipEventRecord(p->ev_t0, s));
    if (C > 1) {
        HIP_TRY(hipEventRecord(p->ev_fork, s));
        HIP_TRY(hipStreamWaitEvent(p->aux_stream, p->ev_fork, 0));
    }
    for (uint32_t c = 0; c < C; ++c) {
        const uint32_t off = c * per, cnt = std::min(per, count - off);
        if (timing) HIP_TRY(hipEventRecord(p->ev_h0[c], s));
        if (use_graph) {
            HIP_TRY(hipGraphLaunch(gc.exec_h[c], s));
        } else {
            ST_TRY(enqueue_chunk(p, 0, off, cnt, x_dev, seeds_dev, idx_dev, val_dev, count_dev, info_dev, s));
        }
        if (timing) HIP_TRY(hipEventRecord(p->ev_h1[c], s));
        if (C > 1) {
            HIP_TRY(hipEventRecord(p->ev_ready[c], s));
            HIP_TRY(hipStreamWaitEvent(p->aux_stream, p->ev_ready[c], 0));
        }
        if (timing) HIP_TRY(hipEventRecord(p->ev_d0[c], ds));
        if (use_graph) {
            HIP_TRY(hipGraphLaunch(gc.exec_d[c], ds));
        } else {
            ST_TRY(enqueue_chunk(p, 1, off, cnt, x_dev, seeds_dev, idx_dev, val_dev, count_dev, info_dev, ds));
        }
        if (timing) HIP_TRY(hipEventRecord(p->ev_d1[c], ds));
    }
    // join: s waits for the last decode
    if (C > 1) {
        HIP_TRY(hipEventRecord(p->ev_join, p->aux_stream));
        HIP_TRY(hipStreamWaitEvent(s, p->ev_join, 0));
    }
    if (timing) {
        HIP_TRY(hipEventRecord(p->ev_t1, s));
        p->timed_chunks = C;
        p->timed_once = true;
    }
    if (use_graph) HIP_TRY(hipEventRecord(gc.launched, s));
    return SFFT_OK;
}

}  // extern "C"

namespace sfft {

sfft_status_t set_last_error(sfft_status_t s, const std::string& msg) { return fail(s, msg); }

size_t plan_device_bytes(const sfft_plan_s* p) { return p ? p->device_bytes : 0; }

sfft_status_t plan_enqueue_ptrs(sfft_plan_s* p, const void* const* xptrs_dev, uint32_t count,
                                const uint64_t* seeds_dev, uint64_t* idx_dev, double* val_dev, uint32_t* count_dev,
                                uint32_t* info_dev, hipStream_t s) {
    if (!p || !xptrs_dev || !idx_dev || !val_dev || !count_dev) return fail(SFFT_EINVAL, "NULL argument");
    if (count < 1 || count > p->d.max_batch) return fail(SFFT_EINVAL, "count must be in [1, max_batch]");
    std::lock_guard<std::mutex> lock(p->mu);
    ST_TRY(enqueue_chunk(p, 0, 0, count, nullptr, seeds_dev, idx_dev, val_dev, count_dev, info_dev, s, xptrs_dev));
    ST_TRY(enqueue_chunk(p, 1, 0, count, nullptr, seeds_dev, idx_dev, val_dev, count_dev, info_dev, s, xptrs_dev));
    return SFFT_OK;
}

}  // namespace sfft
