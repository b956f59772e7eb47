// Internal declarations shared by the host runtime and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/sfft.h"
#include "sfft_common.hpp"

namespace sfft {

constexpr uint32_t kThreads = 256;        // workgroup size of every kernel
constexpr uint32_t kMaxRounds = 32;
constexpr uint32_t kMaxZ = 4096;          // zhat capacity and bin-count limit (LDS sort space)
constexpr uint32_t kStateWords = 8;       // per-signal decode state words

// Per-signal decode state (uint32 words in device memory).
enum : uint32_t {
    ST_ZCOUNT = 0,    // entries of zhat
    ST_ZBUF = 1,      // which of the two zhat buffers is current
    ST_EMPTY = 2,     // consecutive rounds with J empty
    ST_ROUNDS = 3,    // rounds decoded
    ST_DONE = 4,      // 1 once the stopping rule fired
    ST_FLAGS = 5,     // bit 0 truncated output, bit 1 zhat overflow
    ST_LASTJ = 6,     // |J| of the last decoded round
    ST_ACCEPT = 7     // accepted candidates of the last decoded round
};

// Geometry of one hashing round (device copy).
struct RoundDev {
    uint32_t B;
    uint32_t logB;
    uint64_t w;
    int64_t t0;          // window support t in [t0, t0 + w), t0 = -w/2
    uint64_t gofs;       // offset of this round's window in the window tables
    WindowShape ws;
};

// ------------------------------------------------------------------ general
constexpr uint32_t kMaxLevels = 24;
constexpr uint32_t kFracBits = 8;          // fixed-point bits of region coordinates
constexpr uint32_t kMaxT = 64;             // LocateInner regions per level
constexpr uint32_t kMaxREst = 32;          // EstimateValues hashings per round
constexpr uint32_t kMaxRLoc = 8;           // LocateInner measurements per level

// One SparseFFT round (Algorithm 2) of the general mode.
struct GenRoundDev {
    uint32_t k_r;
    uint32_t nlev;               // LocateInner levels
    uint32_t slot0;              // first raw-bin slot of this round
    uint32_t nloc;               // nlev * R_loc location pairs, then R_est estimation slots
    uint64_t Wfp[kMaxLevels];    // region width of each level (fixed point)
    uint64_t blo[kMaxLevels];    // beta range of each level
    uint64_t bhi[kMaxLevels];
};

// One hashing job of the general mode: round, index within the round, slot.
struct GenJob {
    uint32_t round;
    uint32_t index;              // < nloc: location pair (level, rep); else estimation
    uint32_t slot;
    uint32_t pad;
};

// Arguments of the HashToBins pair kernels.
struct H2BArgs {
    const void* x;
    const void* const* xptrs;  // [count] per-signal inputs (batched mode) or nullptr: x + sig * sig_stride
    uint64_t n;
    uint64_t sig_stride;       // elements between signals
    const uint64_t* seeds;     // [count] or nullptr
    uint64_t plan_seed;
    uint32_t count;            // signals
    uint32_t round_lo;         // rounds [round_lo, round_lo + nrounds)
    uint32_t nrounds;
    uint32_t Bmax;
    uint32_t logBmax;
    uint32_t explicit_job;     // 1: use sigma/a/beta/b below for every block
    uint64_t sigma, a, beta, b;
    const RoundDev* geom;      // indexed by round
    const void* gtab;          // window tables (double or float)
    const void* tw;            // twiddles e^{-2 pi i m / Bmax}, m < Bmax/2 (double2/float2)
    double* raw;               // [sig][round][2][Bmax] complex128 out
    uint32_t raw_rounds;       // rounds dimension of raw
    double sqrt_n;
    // split (plain path): partial sums [part][2][B] complex128
    double* partial;
    uint32_t parts;
    uint32_t lchunk;
    uint32_t mcap;             // entries of the LDS modulation table
    // general mode: block b = job * count + sig; jobs[job] names round/index/slot
    const GenJob* jobs;
    const GenRoundDev* groundv;
    uint32_t R_loc;
    uint32_t njobs;
    // exact batched mode: when set, blocks of signals whose decode has
    // stopped (state word ST_DONE) return before gathering
    const uint32_t* state;     // [sig][kStateWords] or nullptr
    uint32_t threads;          // workgroup size of the pair launch: 256, 512, 1024 (0 = 256)
    uint32_t order;            // exact batched: workgroup order (plan hash_order)
    uint32_t nhash;            // raw-bin slots per round: 2, or 3 with the refinement hashing
    uint64_t gamma;            // exact batched: shift of the refinement hashing (0: none)
};

struct DecodeArgs {
    uint64_t n;
    uint32_t count;
    uint32_t rounds;           // rounds with raw bins available (raw dimension)
    uint32_t r_begin, r_end;   // rounds decoded by this launch
    uint32_t patience;
    uint32_t stop_count;       // stop after stop_patience empty rounds once this many |zhat| > theta/2 (0: off)
    uint32_t stop_patience;
    uint32_t Bmax;
    uint32_t capz;             // capacity of each zhat buffer
    uint32_t cap;              // output capacity
    const RoundDev* geom;
    const uint64_t* seeds;
    uint64_t plan_seed;
    const double* raw;         // [sig][rounds][nhash][Bmax]
    double* work;              // [sig][2][Bmax] working bins
    uint64_t* cand_i;          // [sig][Bmax]
    double* cand_v;            // [sig][Bmax][2]
    uint64_t* zidx;            // [sig][2][capz]
    double* zval;              // [sig][2][capz][2]
    double* est;               // re-estimation samples: [sig][rounds][capz][2]
    double* fin;               // [sig][capz][2] re-estimated values
    double* gtmp;              // [sig][capz][4] per-entry terms when LDS cannot hold them
    uint32_t* ecount;          // [sig][capz] samples per entry
    uint8_t* eflag;            // [sig][rounds][capz] sample kind: 0 none, 1 isolated, 2 crowded
    uint32_t* egrp;            // [sig][rounds][capz] bin of a shared entry: first grouped position << 16 | members
    uint16_t* eord;            // [sig][rounds][capz] entries grouped by bin
    double* ecoef;             // [sig][rounds][capz][2] term coefficient G' of a shared entry
    uint32_t* state;           // [sig][kStateWords]
    uint32_t nhash;            // raw-bin slots per round: 2, or 3 with the refinement hashing
    uint32_t refine_window;    // half-width of the refinement's candidate window
    uint64_t refine_shift;     // shift A of the refinement hashing (0: off)
    double theta, g_min;
    double ratio_tol;          // decode a bin only if its two squared magnitudes agree within this (0: off)
    double out_scale;
    uint64_t* out_idx;         // [sig][cap]
    double* out_val;           // [sig][cap][2]
    uint32_t* out_count;       // [sig]
    uint32_t* out_info;        // [sig][4] or nullptr
};

struct GeneralArgs {
    uint64_t n;
    uint32_t count;
    uint32_t R;                  // rounds
    uint32_t nslots;             // raw-bin slots per signal
    uint32_t Bmax;
    uint32_t capz;
    uint32_t cap;
    uint32_t t;
    uint32_t R_loc;
    uint32_t R_est;
    double s;
    double g_min;
    double out_scale;
    const RoundDev* geom;        // per round
    const GenRoundDev* groundv;  // per round
    const uint64_t* seeds;
    uint64_t plan_seed;
    const double* raw;           // [sig][nslots][2][Bmax]
    uint64_t* cand_i;            // [sig][Bmax] located candidates
    double* cand_v;              // [sig][Bmax][2] estimates
    double* cand_e;              // [sig][Bmax][R_est][2] per-measurement estimates
    uint32_t* cand_n;            // [sig][Bmax] valid measurements per candidate
    uint64_t* zidx;              // [sig][2][capz]
    double* zval;                // [sig][2][capz][2]
    double* est;                 // [sig][capz][R * R_est][2]
    double* fin;                 // [sig][capz][2]
    double* gtmp;                // [sig][capz][4] per-entry terms of the LocateSignal hashing
    uint32_t* ecount;            // [sig][capz]
    uint32_t* state;             // [sig][kStateWords]
    uint32_t* gfirst;            // [sig][Bmax + 1] LocateSignal grouping: first entry of each bin
    uint32_t* gent;              // [sig][capz] entries grouped by bin (ascending within a bin)
    uint64_t* cand_raw;          // [sig][Bmax] located candidates in arrival order
    uint32_t* cand_cnt;          // [sig] located candidates, then distinct candidates
    uint8_t* eflag;              // [sig][capz][R * R_est] re-estimation sample: 0 none, 1 isolated, 2 crowded
    uint32_t* egrp;              // [sig][capz][R * R_est] bin of a shared entry: first grouped position << 16 | members
    uint16_t* eord;              // [sig][R * R_est][capz] entries grouped by bin
    double* ecoef;               // [sig][capz][R * R_est][2] term coefficient G' omega^{a sigma i} of a shared entry
    double* gterm;               // [sig][nterm][capz][4] term spill of the per-hashing workgroups
    uint32_t nterm;              // max(R, R_est)
    uint64_t* out_idx;
    double* out_val;
    uint32_t* out_count;
    uint32_t* out_info;
};

// kernel launchers (sfft_kernels.hip); return hipError_t of the launch
hipError_t launch_h2b_pair(const H2BArgs& a, bool in_c128, bool acc_f64, hipStream_t s);
hipError_t launch_h2b_split(const H2BArgs& a, uint32_t round, bool in_c128, bool acc_f64, hipStream_t s);
hipError_t launch_h2b_reduce(const H2BArgs& a, uint32_t round, bool acc_f64, hipStream_t s);
// exact batched pair launch split over a.parts workgroups per (signal,
// round): partials in a.partial ([count * nrounds][parts][4 Bmax] doubles)
hipError_t launch_h2b_pair_split(const H2BArgs& a, bool in_c128, bool acc_f64, hipStream_t s);
// the same pair in stream mode: a.parts workgroups per (signal, round) read
// contiguous shares of the signal (a.parts divides n / B_r); partials as above
hipError_t launch_h2b_pair_stream(const H2BArgs& a, bool in_c128, bool acc_f64, hipStream_t s);
size_t h2b_stream_lds_bytes(uint32_t Bmax, uint64_t max_mcount, bool acc_f64);
hipError_t launch_exact_init(const DecodeArgs& a, hipStream_t s);
hipError_t launch_exact_decode(const DecodeArgs& a, hipStream_t s);
hipError_t launch_exact_finish(const DecodeArgs& a, hipStream_t s);

// general mode: every round [r_begin, r_end) as stage, locate, select,
// estimate and merge launches; the finish as re-estimation and output
hipError_t launch_general_decode(const GeneralArgs& a, uint32_t r_begin, uint32_t r_end, hipStream_t s);
hipError_t launch_general_finish(const GeneralArgs& a, hipStream_t s);

// G'_f, f < count, of a window G (w samples from t0): 1 in the pass band,
// 0 from n / (2B) on, its real response sum_t G_t cos(2 pi f t / n) clamped
// to [0, 1] in between.
hipError_t launch_window_response(const double* G, uint64_t w, int64_t t0, uint64_t n, uint32_t B, double alpha,
                                  double* out, uint64_t count, hipStream_t s);
size_t h2b_pair_lds_bytes(uint32_t Bmax, uint64_t max_mcount, bool acc_f64, uint32_t threads, bool tri = false);
bool h2b_threads_ok(uint32_t threads);
size_t decode_lds_bytes(uint32_t capz, uint32_t Bmax);

// dense path (sfft_dense.hip): top `cap` bins by magnitude of `count`
// spectra [count][n] complex64 (n a power of two >= 2^10), ascending index,
// values * scale in complex128; with keep_above >= 0 only magnitudes
// (times scale) above it are kept.  scratch: dense_topk_scratch_bytes(count)
// of device memory, overwritten.
size_t dense_topk_scratch_bytes(uint32_t count);
// the static scratch of the no-allocation top-k: its capacity in spectra and
// the current device's address of it (looked up once per device)
uint32_t dense_topk_noalloc_max_count();
hipError_t dense_topk_noalloc_scratch(uint32_t** out);
hipError_t launch_dense_topk(const float2* spec, uint64_t n, uint32_t count, uint32_t cap, double scale,
                             double keep_above, uint64_t* out_idx, double* out_val, uint32_t* out_count,
                             uint32_t* scratch, hipStream_t s);

}  // namespace sfft

// Host runtime entry points used by the server (sfft_host.cpp).
struct sfft_plan_s;
namespace sfft {
// Both parts of the batched path for `count` signals given by device
// pointers, on stream s, without graphs or timing events.
sfft_status_t plan_enqueue_ptrs(sfft_plan_s* p, const void* const* xptrs_dev, uint32_t count,
                                const uint64_t* seeds_dev, uint64_t* idx_dev, double* val_dev, uint32_t* count_dev,
                                uint32_t* info_dev, hipStream_t s);
size_t plan_device_bytes(const sfft_plan_s* p);
sfft_status_t set_last_error(sfft_status_t s, const std::string& msg);
}  // namespace sfft
