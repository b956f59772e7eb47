// Serving runtime: continuous batching of sparse FFT requests of mixed n, k
// and mode on one GPU.
//
//  * Shapes.  A request (n, k, mode) maps to a plan shape: k rounded up to a
//    power of two (at least 8), B from that k, the default window for the
//    mode's delta.  Where that window would cover the whole signal (w >= n)
//    the request takes the dense path (full-length FFT + top-k), as it does
//    where a request served alone is predicted to finish sooner on it.
//  * Instances.  Each shape gets up to `instances` resident plan instances
//    (window tables, workspace for `slots` signals, a stream and pinned
//    staging), created on demand and kept; idle instances are evicted in
//    least-recently-used order when a new one would exceed the device-memory
//    budget.  Sizes come from sfft_plan_device_bytes before anything is
//    allocated, so the budget is never exceeded.  An instance is built on a
//    thread of its own (building a dense-path instance warms its FFT plans
//    and takes up to tens of milliseconds): only its shape's requests wait.
//  * Scheduling.  One host thread takes, for every shape with waiting
//    requests (oldest first), an idle instance and up to `slots` of its
//    requests, and enqueues that batch on the instance's stream: batches of
//    different shapes run concurrently and requests that arrive meanwhile are
//    admitted as instances come free.  The batched path reads each signal in
//    place through a pointer array.  Completion is recorded by a host
//    callback on the stream after the results' device-to-host copy.
//  * Results depend only on (signal, seed, shape): a request gives the same
//    answer alone and in any mix.
#include <dlfcn.h>
#include <hip/hip_runtime.h>
#include <hipfft/hipfft.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "sfft_internal.hpp"

using sfft::set_last_error;
using Clock = std::chrono::steady_clock;

struct sfft_server_s;

namespace {

double ms_between(Clock::time_point a, Clock::time_point b) {
    return std::chrono::duration<double, std::milli>(b - a).count();
}

uint32_t pow2_at_least_u32(uint32_t v) {
    uint32_t p = 1;
    while (p < v) p <<= 1;
    return p;
}

bool pow2(uint64_t v) { return v && !(v & (v - 1)); }

// ------------------------------------------------------------------ shapes --
sfft_status_t shape_for(uint64_t n, uint32_t k, int32_t mode, const sfft_server_desc_t& sd, sfft_plan_desc_t* d,
                        int32_t* dense) {
    if (!pow2(n) || n < (1ull << 10) || n > (1ull << 30)) return set_last_error(SFFT_ENOTPOW2, "n must be 2^10..2^30");
    if (k < 1 || k > 1024) return set_last_error(SFFT_EINVAL, "k must be in [1, 1024]");
    if (mode != SFFT_MODE_EXACT && mode != SFFT_MODE_GENERAL) return set_last_error(SFFT_EINVAL, "bad mode");
    const uint32_t kb = pow2_at_least_u32(std::max<uint32_t>(k, 8));
    uint64_t B = mode == SFFT_MODE_EXACT ? 4ull * kb : 16ull * kb;
    B = std::max<uint64_t>(B, mode == SFFT_MODE_EXACT ? 64 : 256);
    B = std::min<uint64_t>({B, 4096, n / 16});
    sfft_desc_init(d, n, kb, (uint32_t)B, 0, 0);
    d->mode = mode;
    d->delta = mode == SFFT_MODE_EXACT ? sd.delta_exact : sd.delta_general;
    d->theta = sd.theta;
    if (mode == SFFT_MODE_EXACT) {
        // A coefficient is invisible in a round when its offset falls where G'
        // is near 0 (about 22% of offsets at alpha = 1/2); five empty rounds
        // before stopping make losing one to that negligible (on the oracle
        // at n = 2^20, k = 600: 797/800 supports exact with 3, 800/800 with 5).
        // at least 32 bins in the late rounds: with 8 (B = 256) a few wrong
        // early locations can no longer be untangled (seen at n = 2^16, k = 59)
        d->b_min = std::max<uint32_t>(32, (uint32_t)B / 32);
        if (d->b_min > B) d->b_min = (uint32_t)B;
        d->rounds = 24;
        d->patience = 5;
        // served batches are small: without a split each (signal, round) is
        // one workgroup walking a window of about 96 B samples on one CU.
        // One part per 256 bins (fixed per shape, so results do not depend
        // on the batch); at n = 2^24, k = 1024 this takes a request alone
        // from 1.06 to 0.67 ms.
        d->hash_split = std::min<uint32_t>(16, std::max<uint32_t>(1, (uint32_t)B / 256));
        // rounds whose window covers an eighth of the signal or more read it
        // contiguously (stream mode) instead of gathering
        d->hash_mode = 1;
    }
    d->cap = kb;
    d->max_batch = sd.slots;
    // the Kaiser-Bessel flat window: the same flatness with about half the
    // Gaussian construction's samples
    d->window = 1;
    d->w = sfft_window_w(n, (uint32_t)B, d->alpha, d->delta, 1);
    *dense = d->w >= n || sfft_validate_params(d) != SFFT_OK;
    if (!*dense && !(sd.flags & SFFT_SERVER_SPARSE_ONLY)) {
        // the path a request served alone finishes sooner on: the sparse
        // path pays a launch chain (its floor) plus a cost per gathered or
        // streamed sample, the dense FFT a floor plus a cost per sample of
        // the signal (constants fitted to solo service times on MI355X)
        const uint64_t samples = sfft_plan_samples(d);
        const uint64_t streamed = (uint64_t)sfft_plan_stream_rounds(d) * n;
        const double sparse_ms =
            mode == SFFT_MODE_EXACT
                ? SFFT_SERVER_EXACT_MS + 1e-6 * (SFFT_SERVER_GATHER_NS * (double)(samples - streamed) +
                                                 SFFT_SERVER_STREAM_NS * (double)streamed)
                : SFFT_SERVER_GENERAL_MS + 1e-6 * SFFT_SERVER_GENERAL_NS * (double)samples;
        const double dense_ms = SFFT_SERVER_DENSE_MS + 1e-6 * SFFT_SERVER_DENSE_NS * (double)n;
        *dense = samples == 0 || sparse_ms > dense_ms;
    }
    if (sd.flags & SFFT_SERVER_DENSE_ONLY) *dense = 1;
    if (*dense) d->w = n;
    return SFFT_OK;
}

// A shape is named by (log2 n, log2 of the rounded k, mode); the rest of it
// is a function of these and the server description.
uint64_t shape_key(uint64_t n, uint32_t k, int32_t mode) {
    const uint32_t kb = pow2_at_least_u32(std::max<uint32_t>(k, 8));
    uint32_t ln = 0;
    while ((1ull << ln) < n) ++ln;
    uint32_t lk = 0;
    while ((1u << lk) < kb) ++lk;
    return ((uint64_t)ln << 16) | ((uint64_t)lk << 8) | (uint64_t)(mode & 0xFF);
}

struct ShapeInfo {
    sfft_plan_desc_t desc;
    int32_t dense;
    size_t bytes;   // device bytes of one instance
};

// ------------------------------------------------------------- hipFFT -----
// The dense path's FFT library is opened on first use, so processes that
// never take the dense path never load it.
struct FftLib {
    bool tried = false;
    void* lib = nullptr;
    hipfftResult (*plan1d)(hipfftHandle*, int, hipfftType, int) = nullptr;
    hipfftResult (*set_stream)(hipfftHandle, hipStream_t) = nullptr;
    hipfftResult (*exec_c2c)(hipfftHandle, hipfftComplex*, hipfftComplex*, int) = nullptr;
    hipfftResult (*destroy)(hipfftHandle) = nullptr;
    bool ok() const { return plan1d && set_stream && exec_c2c && destroy; }
};

FftLib& fftlib() {
    static FftLib f;
    static std::mutex mu;
    std::lock_guard<std::mutex> lock(mu);
    if (!f.tried) {
        f.tried = true;
        f.lib = dlopen("libhipfft.so.0", RTLD_NOW | RTLD_GLOBAL);
        if (!f.lib) f.lib = dlopen("libhipfft.so", RTLD_NOW | RTLD_GLOBAL);
        if (f.lib) {
            f.plan1d = reinterpret_cast<decltype(f.plan1d)>(dlsym(f.lib, "hipfftPlan1d"));
            f.set_stream = reinterpret_cast<decltype(f.set_stream)>(dlsym(f.lib, "hipfftSetStream"));
            f.exec_c2c = reinterpret_cast<decltype(f.exec_c2c)>(dlsym(f.lib, "hipfftExecC2C"));
            f.destroy = reinterpret_cast<decltype(f.destroy)>(dlsym(f.lib, "hipfftDestroy"));
        }
    }
    return f;
}

// --------------------------------------------------------------- objects --
struct ShapeInfo;

struct Request {
    uint64_t ticket = 0;
    sfft_request_t r{};
    uint64_t key = 0;
    const ShapeInfo* shape = nullptr;
    Clock::time_point t_submit, t_launch, t_done;
    int32_t status = SFFT_EAGAIN;
    uint32_t count = 0, flags = 0, rounds = 0;
    int32_t path = 0;
    bool launched = false;
    bool done = false;
    std::string message;   // why it failed (empty on success)
};

struct Instance {
    sfft_server_s* srv = nullptr;
    uint64_t key = 0;
    sfft_plan_desc_t desc{};
    int32_t dense = 0;
    uint32_t slots = 0, cap = 0;
    sfft_plan_t plan = nullptr;
    // dense path: FFT plans for batches of 1, 2, 4, ... slots; a batch of m
    // signals runs as the plans of m's binary digits
    static constexpr uint32_t kFftPlans = 11;
    hipfftHandle fft[kFftPlans] = {};
    float2* d_dense = nullptr;      // [slots][n] staging + spectra (dense path)
    uint32_t* d_topk = nullptr;     // dense path: top-k selection scratch
    hipStream_t stream = nullptr;
    const void** d_xptrs = nullptr;
    uint64_t* d_seeds = nullptr;
    uint64_t* d_idx = nullptr;
    double* d_val = nullptr;
    uint32_t* d_cnt = nullptr;
    uint32_t* d_info = nullptr;
    const void** h_xptrs = nullptr;  // pinned staging and results
    uint64_t* h_seeds = nullptr;
    uint64_t* h_idx = nullptr;
    double* h_val = nullptr;
    uint32_t* h_cnt = nullptr;
    uint32_t* h_info = nullptr;
    size_t bytes = 0;
    bool fake = false;
    bool busy = false;
    bool building = false;                  // its build thread has not finished
    sfft_status_t build_status = SFFT_OK;   // what the build returned
    std::string build_message;              // and its message, when it failed
    std::vector<Request*> batch;
    Clock::time_point last_used;
};

}  // namespace

struct sfft_server_s {
    sfft_server_desc_t d{};
    // shapes seen so far (computing one sizes a window, which takes
    // milliseconds of host time): guarded by shape_mu, never erased
    std::mutex shape_mu;
    std::map<uint64_t, ShapeInfo> shapes;
    std::mutex mu;
    std::condition_variable cv_sched, cv_done;
    uint64_t events = 0;   // bumped with every cv_sched notification, so that none is missed
    std::map<uint64_t, std::deque<Request*>> queues;
    std::unordered_map<uint64_t, std::unique_ptr<Request>> reqs;
    std::vector<std::unique_ptr<Instance>> inst;
    size_t bytes_in_use = 0, peak_bytes = 0;
    uint64_t next_ticket = 1;
    uint32_t pending = 0, inflight = 0;
    uint32_t builders = 0;   // instance builds in progress
    std::condition_variable cv_build;
    bool stop = false;
    std::thread th;
    // fake device: batches finish at their due time on this thread
    std::thread fake_th;
    std::condition_variable cv_fake;
    std::multimap<Clock::time_point, Instance*> fake_due;
    // statistics since the last reset
    std::vector<double> lat_ms, queue_ms, service_ms;
    uint64_t completed = 0, dense = 0, failed = 0, batches = 0, batched = 0, evictions = 0;
    Clock::time_point t_first, t_last;
    bool have_first = false;
};

namespace {

#define SRV_TRY_SHAPE(expr)           \
    do {                              \
        sfft_status_t s_ = (expr);    \
        if (s_ != SFFT_OK) return s_; \
    } while (0)

size_t instance_buffer_bytes(uint32_t slots, uint32_t cap) {
    return (size_t)slots * (8 + 8 + (size_t)cap * 8 + (size_t)cap * 16 + 4 + 16);
}

size_t instance_bytes(const sfft_plan_desc_t& d, int32_t dense) {
    const size_t bufs = instance_buffer_bytes(d.max_batch, d.cap);
    if (dense) return bufs + (size_t)d.max_batch * d.n * sizeof(float2) + sfft::dense_topk_scratch_bytes(d.max_batch);
    return bufs + sfft_plan_device_bytes(&d);
}

// The cached shape of a request, computed on first use.
sfft_status_t server_shape(sfft_server_s* s, uint64_t n, uint32_t k, int32_t mode, const ShapeInfo** out,
                           uint64_t* key) {
    if (!pow2(n) || n < (1ull << 10) || n > (1ull << 30)) return set_last_error(SFFT_ENOTPOW2, "n must be 2^10..2^30");
    if (k < 1 || k > 1024) return set_last_error(SFFT_EINVAL, "k must be in [1, 1024]");
    if (mode != SFFT_MODE_EXACT && mode != SFFT_MODE_GENERAL) return set_last_error(SFFT_EINVAL, "bad mode");
    *key = shape_key(n, k, mode);
    std::lock_guard<std::mutex> lock(s->shape_mu);
    auto it = s->shapes.find(*key);
    if (it == s->shapes.end()) {
        ShapeInfo info;
        SRV_TRY_SHAPE(shape_for(n, k, mode, s->d, &info.desc, &info.dense));
        info.bytes = instance_bytes(info.desc, info.dense);
        it = s->shapes.emplace(*key, info).first;
    }
    *out = &it->second;
    return SFFT_OK;
}

void destroy_instance(Instance* in) {
    if (in->fake) return;
    if (in->stream) (void)hipStreamSynchronize(in->stream);
    if (in->plan) sfft_destroy(in->plan);
    for (hipfftHandle h : in->fft)
        if (h) fftlib().destroy(h);
    for (void* q : {(void*)in->d_dense, (void*)in->d_topk, (void*)in->d_xptrs, (void*)in->d_seeds, (void*)in->d_idx, (void*)in->d_val,
                    (void*)in->d_cnt, (void*)in->d_info})
        if (q) (void)hipFree(q);
    for (void* q : {(void*)in->h_xptrs, (void*)in->h_seeds, (void*)in->h_idx, (void*)in->h_val, (void*)in->h_cnt,
                    (void*)in->h_info})
        if (q) (void)hipHostFree(q);
    if (in->stream) (void)hipStreamDestroy(in->stream);
}

#define SRV_HIP(expr)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess) return set_last_error(SFFT_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

template <class T>
sfft_status_t dmalloc(T** p, size_t count) {
    SRV_HIP(hipMalloc(reinterpret_cast<void**>(p), std::max<size_t>(count, 1) * sizeof(T)));
    return SFFT_OK;
}
template <class T>
sfft_status_t hmalloc(T** p, size_t count) {
    SRV_HIP(hipHostMalloc(reinterpret_cast<void**>(p), std::max<size_t>(count, 1) * sizeof(T), hipHostMallocDefault));
    return SFFT_OK;
}

#define SRV_TRY(expr)                 \
    do {                              \
        sfft_status_t s_ = (expr);    \
        if (s_ != SFFT_OK) return s_; \
    } while (0)

sfft_status_t build_instance(Instance* in) {
    if (in->fake) return SFFT_OK;
    const uint32_t S = in->slots, cap = in->cap;
    SRV_HIP(hipStreamCreateWithFlags(&in->stream, hipStreamNonBlocking));
    SRV_TRY(dmalloc(&in->d_xptrs, S));
    SRV_TRY(dmalloc(&in->d_seeds, S));
    SRV_TRY(dmalloc(&in->d_idx, (size_t)S * cap));
    SRV_TRY(dmalloc(&in->d_val, (size_t)S * cap * 2));
    SRV_TRY(dmalloc(&in->d_cnt, S));
    SRV_TRY(dmalloc(&in->d_info, (size_t)S * 4));
    SRV_TRY(hmalloc(&in->h_xptrs, S));
    SRV_TRY(hmalloc(&in->h_seeds, S));
    SRV_TRY(hmalloc(&in->h_idx, (size_t)S * cap));
    SRV_TRY(hmalloc(&in->h_val, (size_t)S * cap * 2));
    SRV_TRY(hmalloc(&in->h_cnt, S));
    SRV_TRY(hmalloc(&in->h_info, (size_t)S * 4));
    if (in->dense) {
        FftLib& f = fftlib();
        if (!f.ok()) return set_last_error(SFFT_EUNSUPPORTED, "dense path needs libhipfft, which could not be loaded");
        SRV_TRY(dmalloc(&in->d_dense, (size_t)S * in->desc.n));
        SRV_TRY(dmalloc(&in->d_topk, sfft::dense_topk_scratch_bytes(S) / sizeof(uint32_t)));
        for (uint32_t b = 0; b < Instance::kFftPlans && (1u << b) <= S; ++b) {
            if (f.plan1d(&in->fft[b], (int)in->desc.n, HIPFFT_C2C, (int)(1u << b)) != HIPFFT_SUCCESS)
                return set_last_error(SFFT_EHIP, "hipfftPlan1d failed");
            if (f.set_stream(in->fft[b], in->stream) != HIPFFT_SUCCESS)
                return set_last_error(SFFT_EHIP, "hipfftSetStream failed");
        }
        // A plan's first execution loads its kernels and sets up its work
        // space; run each once now so that no request's service time (and no
        // other shape's launch, the scheduler being one thread) pays for it.
        SRV_HIP(hipMemsetAsync(in->d_dense, 0, (size_t)S * in->desc.n * sizeof(float2), in->stream));
        for (uint32_t b = 0; b < Instance::kFftPlans && in->fft[b]; ++b) {
            auto* buf = reinterpret_cast<hipfftComplex*>(in->d_dense);
            if (f.exec_c2c(in->fft[b], buf, buf, HIPFFT_FORWARD) != HIPFFT_SUCCESS)
                return set_last_error(SFFT_EHIP, "hipfftExecC2C failed");
        }
        SRV_HIP(hipStreamSynchronize(in->stream));
    } else {
        SRV_TRY(sfft_plan_ex(&in->desc, &in->plan));
    }
    return SFFT_OK;
}

// Results of a finished batch into each request's host buffers (the
// request's own k: the largest |v| first, ties to the smaller index, then
// ascending index), statistics, and the instance back to idle.
void complete_batch(Instance* in) {
    sfft_server_s* s = in->srv;
    std::lock_guard<std::mutex> lock(s->mu);
    const Clock::time_point now = Clock::now();
    for (size_t q = 0; q < in->batch.size(); ++q) {
        Request* rq = in->batch[q];
        const uint64_t* idx = in->fake ? nullptr : in->h_idx + q * in->cap;
        const double* val = in->fake ? nullptr : in->h_val + q * in->cap * 2;
        uint32_t c = in->fake ? 0u : std::min(in->h_cnt[q], in->cap);
        std::vector<uint32_t> order(c);
        for (uint32_t e = 0; e < c; ++e) order[e] = e;
        if (c > rq->r.k) {
            std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) {
                const double ma = std::hypot(val[2 * a], val[2 * a + 1]), mb = std::hypot(val[2 * b], val[2 * b + 1]);
                return ma > mb;
            });
            order.resize(rq->r.k);
            std::sort(order.begin(), order.end());
            c = rq->r.k;
        }
        for (uint32_t e = 0; e < c; ++e) {
            if (rq->r.idx_host) rq->r.idx_host[e] = idx[order[e]];
            if (rq->r.val_host) {
                rq->r.val_host[2 * e] = val[2 * order[e]];
                rq->r.val_host[2 * e + 1] = val[2 * order[e] + 1];
            }
        }
        rq->count = c;
        rq->flags = (in->dense || in->fake) ? 0 : in->h_info[q * 4 + SFFT_INFO_FLAGS];
        rq->rounds = (in->dense || in->fake) ? 0 : in->h_info[q * 4 + SFFT_INFO_ROUNDS];
        rq->path = in->dense;
        rq->status = SFFT_OK;
        rq->t_done = now;
        rq->done = true;
        s->lat_ms.push_back(ms_between(rq->t_submit, now));
        s->queue_ms.push_back(ms_between(rq->t_submit, rq->t_launch));
        s->service_ms.push_back(ms_between(rq->t_launch, now));
        ++s->completed;
        if (in->dense) ++s->dense;
    }
    s->t_last = now;
    s->inflight -= (uint32_t)in->batch.size();
    in->batch.clear();
    in->busy = false;
    in->last_used = now;
    ++s->events;
    s->cv_sched.notify_all();
    s->cv_done.notify_all();
}

void on_batch_done(void* arg) { complete_batch(static_cast<Instance*>(arg)); }

// Enqueue one batch on the instance's stream (no server lock held).
sfft_status_t launch_batch(Instance* in) {
    if (in->fake) {
        sfft_server_s* s = in->srv;
        std::lock_guard<std::mutex> lock(s->mu);
        s->fake_due.emplace(Clock::now() + std::chrono::duration_cast<Clock::duration>(
                                                std::chrono::duration<double, std::milli>(s->d.fake_service_ms)),
                            in);
        s->cv_fake.notify_all();
        return SFFT_OK;
    }
    const uint32_t m = (uint32_t)in->batch.size();
    const uint64_t n = in->desc.n;
    for (uint32_t q = 0; q < m; ++q) {
        in->h_xptrs[q] = in->batch[q]->r.x_dev;
        in->h_seeds[q] = in->batch[q]->r.seed;
    }
    hipStream_t st = in->stream;
    if (in->dense) {
        for (uint32_t q = 0; q < m; ++q)
            SRV_HIP(hipMemcpyAsync(in->d_dense + (size_t)q * n, in->h_xptrs[q], n * sizeof(float2),
                                   hipMemcpyDeviceToDevice, st));
        // only the m signals of the batch are transformed
        uint32_t done = 0;
        for (int b = (int)Instance::kFftPlans - 1; b >= 0; --b) {
            if (!(m & (1u << b))) continue;
            auto* buf = reinterpret_cast<hipfftComplex*>(in->d_dense + (size_t)done * n);
            if (!in->fft[b] || fftlib().exec_c2c(in->fft[b], buf, buf, HIPFFT_FORWARD) != HIPFFT_SUCCESS)
                return set_last_error(SFFT_EHIP, "hipfftExecC2C failed");
            done += 1u << b;
        }
        const double keep = in->desc.mode == SFFT_MODE_EXACT ? 0.5 * in->desc.theta : -1.0;
        SRV_HIP(sfft::launch_dense_topk(in->d_dense, n, m, in->cap, 1.0 / std::sqrt((double)n), keep, in->d_idx,
                                        in->d_val, in->d_cnt, in->d_topk, st));
    } else {
        SRV_HIP(hipMemcpyAsync(in->d_xptrs, in->h_xptrs, m * sizeof(void*), hipMemcpyHostToDevice, st));
        SRV_HIP(hipMemcpyAsync(in->d_seeds, in->h_seeds, m * sizeof(uint64_t), hipMemcpyHostToDevice, st));
        SRV_TRY(sfft::plan_enqueue_ptrs(in->plan, in->d_xptrs, m, in->d_seeds, in->d_idx, in->d_val, in->d_cnt,
                                        in->d_info, st));
        SRV_HIP(hipMemcpyAsync(in->h_info, in->d_info, (size_t)m * 4 * sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    }
    SRV_HIP(hipMemcpyAsync(in->h_idx, in->d_idx, (size_t)m * in->cap * sizeof(uint64_t), hipMemcpyDeviceToHost, st));
    SRV_HIP(hipMemcpyAsync(in->h_val, in->d_val, (size_t)m * in->cap * 2 * sizeof(double), hipMemcpyDeviceToHost, st));
    SRV_HIP(hipMemcpyAsync(in->h_cnt, in->d_cnt, (size_t)m * sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    SRV_HIP(hipLaunchHostFunc(st, on_batch_done, in));
    return SFFT_OK;
}

void fail_requests(sfft_server_s* s, std::vector<Request*>& rs, sfft_status_t st, const std::string& msg) {
    const Clock::time_point now = Clock::now();
    for (Request* r : rs) {
        r->status = st;
        r->message = msg;
        r->done = true;
        r->t_done = now;
        ++s->failed;
    }
    s->inflight -= (uint32_t)rs.size();
    rs.clear();
    s->cv_done.notify_all();
}

// An idle instance for `key`, creating one (and evicting idle instances of
// other shapes, least recently used first) when the budget allows.  Called
// with the lock held; returns nullptr when the shape has to wait.
// Builds one instance on its own thread, then makes it idle (or records the
// failure, its resources already released) and wakes the scheduler.
void build_worker(sfft_server_s* s, Instance* in) {
    if (!in->fake) (void)hipSetDevice(s->d.device);
    const sfft_status_t st = build_instance(in);
    // the message of a failure is thread-local: take it on this thread
    const std::string msg = st != SFFT_OK ? std::string(sfft_last_error()) : std::string();
    if (st != SFFT_OK) destroy_instance(in);
    std::lock_guard<std::mutex> lock(s->mu);
    in->building = false;
    in->build_status = st;
    in->build_message = msg;
    if (st == SFFT_OK) {
        in->busy = false;
        in->last_used = Clock::now();
    }
    --s->builders;
    ++s->events;
    s->cv_sched.notify_all();
    s->cv_build.notify_all();
}

Instance* instance_for(sfft_server_s* s, uint64_t key, const Request* head, std::unique_lock<std::mutex>& lk,
                       sfft_status_t* hard_fail, std::string* why) {
    uint32_t have = 0;
    for (auto it = s->inst.begin(); it != s->inst.end(); ++it) {
        Instance* in = it->get();
        if (in->key != key) continue;
        if (!in->building && in->build_status != SFFT_OK) {
            // a failed build (already released): the shape cannot run
            *hard_fail = in->build_status;
            *why = "instance build failed: " + in->build_message;
            s->bytes_in_use -= in->bytes;
            s->inst.erase(it);
            return nullptr;
        }
        ++have;
        if (!in->busy) return in;
    }
    if (have >= s->d.instances) return nullptr;
    const ShapeInfo* shape = head->shape;
    const sfft_plan_desc_t& d = shape->desc;
    const int32_t dense = shape->dense;
    const size_t need = shape->bytes;
    if (need > s->d.budget_bytes) {
        *hard_fail = SFFT_EBUDGET;
        *why = "one instance of this shape exceeds the server's budget";
        return nullptr;
    }
    // Dense-path instances stay resident unless SFFT_SERVER_EVICT_DENSE: their
    // bytes are held for good, and a shape that cannot fit beside them never
    // will.
    const bool evict_dense = (s->d.flags & SFFT_SERVER_EVICT_DENSE) != 0;
    if (!evict_dense) {
        size_t pinned = 0;
        for (auto& up : s->inst)
            if (up->dense) pinned += up->bytes;
        if (pinned + need > s->d.budget_bytes) {
            if (have == 0) {   // else the shape's own instances serve it
                *hard_fail = SFFT_EBUDGET;
                *why = "the budget is held by resident dense-path instances, which are not evicted";
            }
            return nullptr;
        }
    }
    // Evict idle instances, least recently used first.  Their memory is
    // released with the lock dropped: freeing device memory synchronises the
    // device, and the completion callbacks of running batches take the lock.
    // No eviction runs while an instance is being built, so that the frees
    // never overlap a build's allocations, FFT plan set-up and warm-up.
    std::vector<std::unique_ptr<Instance>> evicted;
    while (s->bytes_in_use + need > s->d.budget_bytes && s->builders == 0) {
        // idle instances whose shape has no waiting request (an instance just
        // built for waiting requests is about to be used)
        auto victim = s->inst.end();
        for (auto it = s->inst.begin(); it != s->inst.end(); ++it) {
            if ((*it)->busy || ((*it)->dense && !evict_dense)) continue;
            const auto q = s->queues.find((*it)->key);
            if (q != s->queues.end() && !q->second.empty()) continue;
            if (victim == s->inst.end() || (*it)->last_used < (*victim)->last_used) victim = it;
        }
        if (victim == s->inst.end()) break;
        s->bytes_in_use -= (*victim)->bytes;
        ++s->evictions;
        evicted.push_back(std::move(*victim));
        s->inst.erase(victim);
    }
    if (!evicted.empty()) {
        lk.unlock();
        for (auto& e : evicted) destroy_instance(e.get());
        evicted.clear();
        lk.lock();
    }
    if (s->bytes_in_use + need > s->d.budget_bytes) return nullptr;   // wait for a busy instance to finish
    auto in = std::make_unique<Instance>();
    in->srv = s;
    in->key = key;
    in->desc = d;
    in->dense = dense;
    in->slots = s->d.slots;
    in->cap = d.cap;
    in->bytes = need;
    in->fake = (s->d.flags & SFFT_SERVER_FAKE_DEVICE) != 0;
    in->busy = true;   // reserved while it is built
    in->building = true;
    Instance* raw = in.get();
    s->inst.push_back(std::move(in));
    s->bytes_in_use += need;
    s->peak_bytes = std::max(s->peak_bytes, s->bytes_in_use);
    ++s->builders;
    try {
        std::thread(build_worker, s, raw).detach();
    } catch (...) {
        --s->builders;
        s->bytes_in_use -= need;
        s->inst.pop_back();
        *hard_fail = SFFT_ENOMEM;
        *why = "could not start a build thread";
    }
    return nullptr;   // the shape's requests wait for the build
}

// Fake device: completes each batch when its time has come.
void fake_device(sfft_server_s* s) {
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        if (s->fake_due.empty()) {
            if (s->stop && s->inflight == 0) break;
            s->cv_fake.wait_for(lk, std::chrono::milliseconds(50));
            continue;
        }
        const auto due = s->fake_due.begin()->first;
        if (Clock::now() < due) {
            s->cv_fake.wait_until(lk, due);
            continue;
        }
        Instance* in = s->fake_due.begin()->second;
        s->fake_due.erase(s->fake_due.begin());
        lk.unlock();
        complete_batch(in);
        lk.lock();
    }
}

void scheduler(sfft_server_s* s) {
    if (!(s->d.flags & SFFT_SERVER_FAKE_DEVICE)) (void)hipSetDevice(s->d.device);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        if (s->stop && s->pending == 0 && s->inflight == 0) break;
        const uint64_t seen = s->events;   // events from here on end the wait below
        std::vector<std::pair<Clock::time_point, uint64_t>> order;
        for (auto& kv : s->queues)
            if (!kv.second.empty()) order.emplace_back(kv.second.front()->t_submit, kv.first);
        std::sort(order.begin(), order.end());
        bool launched = false;
        for (auto& o : order) {
            auto& q = s->queues[o.second];
            if (q.empty()) continue;
            sfft_status_t hard = SFFT_OK;
            std::string why;
            Instance* in = instance_for(s, o.second, q.front(), lk, &hard, &why);
            if (!in) {
                if (hard != SFFT_OK) {   // the shape can never run: fail its waiting requests
                    std::vector<Request*> rs(q.begin(), q.end());
                    s->pending -= (uint32_t)rs.size();
                    s->inflight += (uint32_t)rs.size();
                    q.clear();
                    fail_requests(s, rs, hard, why);
                }
                continue;
            }
            const Clock::time_point now = Clock::now();
            while (!q.empty() && in->batch.size() < in->slots) {
                Request* r = q.front();
                q.pop_front();
                r->t_launch = now;
                r->launched = true;
                in->batch.push_back(r);
            }
            s->pending -= (uint32_t)in->batch.size();
            s->inflight += (uint32_t)in->batch.size();
            in->busy = true;
            ++s->batches;
            s->batched += in->batch.size();
            lk.unlock();
            const sfft_status_t st = launch_batch(in);
            // launch_batch's message is this thread's: take it before the lock
            const std::string msg = st != SFFT_OK ? "launch failed: " + std::string(sfft_last_error()) : std::string();
            lk.lock();
            if (st != SFFT_OK) {
                fail_requests(s, in->batch, st, msg);
                in->busy = false;
            }
            launched = true;
        }
        if (!launched) s->cv_sched.wait(lk, [&] { return s->events != seen; });
    }
}

double percentile(std::vector<double> v, double q) {
    if (v.empty()) return 0.0;
    std::sort(v.begin(), v.end());
    const double pos = q / 100.0 * (double)(v.size() - 1);
    const size_t lo = (size_t)std::floor(pos), hi = std::min(lo + 1, v.size() - 1);
    return v[lo] + (v[hi] - v[lo]) * (pos - (double)lo);
}

}  // namespace

extern "C" {

sfft_status_t sfft_server_desc_init(sfft_server_desc_t* d) {
    if (!d) return set_last_error(SFFT_EINVAL, "NULL argument");
    std::memset(d, 0, sizeof(*d));
    d->budget_bytes = 16ull << 30;
    d->slots = 32;
    d->instances = 2;
    d->device = 0;
    d->delta_exact = 1e-9;
    d->delta_general = 1e-6;
    d->theta = 0.25;
    d->fake_service_ms = 1.0;
    return SFFT_OK;
}

uint64_t sfft_dense_topk_scratch_bytes(uint32_t count) { return sfft::dense_topk_scratch_bytes(count); }

sfft_status_t sfft_dense_topk(const void* spec_dev, uint64_t n, uint32_t count, uint32_t cap, double scale,
                              double keep_above, uint64_t* idx_dev, double* val_dev, uint32_t* count_dev,
                              void* scratch_dev, void* stream) {
    if (!spec_dev || !idx_dev || !val_dev || !count_dev || !scratch_dev || count == 0 || cap == 0 || cap > 8192 ||
        !(scale > 0))
        return set_last_error(SFFT_EINVAL, "bad dense top-k arguments");
    if (!pow2(n) || n < (1ull << 10) || n > (1ull << 30)) return set_last_error(SFFT_ENOTPOW2, "n must be 2^10..2^30");
    const hipError_t e = sfft::launch_dense_topk(static_cast<const float2*>(spec_dev), n, count, cap, scale, keep_above,
                                                 idx_dev, val_dev, count_dev, static_cast<uint32_t*>(scratch_dev),
                                                 static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return set_last_error(SFFT_EHIP, std::string("dense top-k: ") + hipGetErrorString(e));
    return SFFT_OK;
}

uint32_t sfft_dense_topk_noalloc_max_count(void) { return sfft::dense_topk_noalloc_max_count(); }

sfft_status_t sfft_dense_topk_noalloc(const void* spec_dev, uint64_t n, uint32_t count, uint32_t cap, double scale,
                                      double keep_above, uint64_t* idx_dev, double* val_dev, uint32_t* count_dev,
                                      void* stream) {
    if (!spec_dev || !idx_dev || !val_dev || !count_dev || count == 0 || cap == 0 || cap > 8192 || !(scale > 0))
        return set_last_error(SFFT_EINVAL, "bad dense top-k arguments");
    if (count > sfft::dense_topk_noalloc_max_count())
        return set_last_error(SFFT_EINVAL, "count " + std::to_string(count) + " exceeds the static scratch (" +
                                               std::to_string(sfft::dense_topk_noalloc_max_count()) + " spectra)");
    if (!pow2(n) || n < (1ull << 10) || n > (1ull << 30)) return set_last_error(SFFT_ENOTPOW2, "n must be 2^10..2^30");
    uint32_t* scratch = nullptr;
    hipError_t e = sfft::dense_topk_noalloc_scratch(&scratch);
    if (e != hipSuccess)
        return set_last_error(SFFT_EHIP, std::string("static top-k scratch: ") + hipGetErrorString(e));
    e = sfft::launch_dense_topk(static_cast<const float2*>(spec_dev), n, count, cap, scale, keep_above, idx_dev,
                               val_dev, count_dev, scratch, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return set_last_error(SFFT_EHIP, std::string("dense top-k: ") + hipGetErrorString(e));
    return SFFT_OK;
}

sfft_status_t sfft_server_shape(const sfft_server_desc_t* sd, uint64_t n, uint32_t k, int32_t mode,
                                sfft_plan_desc_t* plan_out, int32_t* dense_out, uint64_t* bytes_out) {
    if (!sd || !plan_out || !dense_out) return set_last_error(SFFT_EINVAL, "NULL argument");
    SRV_TRY(shape_for(n, k, mode, *sd, plan_out, dense_out));
    if (bytes_out) *bytes_out = instance_bytes(*plan_out, *dense_out);
    return SFFT_OK;
}

sfft_status_t sfft_server_create(const sfft_server_desc_t* d, sfft_server_t* out) {
    if (!d || !out) return set_last_error(SFFT_EINVAL, "NULL argument");
    if (d->slots < 1 || d->slots > 1024 || d->instances < 1 || d->instances > 16 || d->budget_bytes == 0 ||
        !(d->theta > 0) || !(d->delta_exact > 0 && d->delta_exact < 1) ||
        !(d->delta_general > 0 && d->delta_general < 1) ||
        (d->flags & ~(SFFT_SERVER_FAKE_DEVICE | SFFT_SERVER_DENSE_ONLY | SFFT_SERVER_SPARSE_ONLY |
                      SFFT_SERVER_EVICT_DENSE)) ||
        ((d->flags & SFFT_SERVER_DENSE_ONLY) && (d->flags & SFFT_SERVER_SPARSE_ONLY)) ||
        !(d->fake_service_ms >= 0))
        return set_last_error(SFFT_EINVAL, "bad server description");
    auto* s = new (std::nothrow) sfft_server_s();
    if (!s) return set_last_error(SFFT_ENOMEM, "host allocation failed");
    s->d = *d;
    s->th = std::thread(scheduler, s);
    if (d->flags & SFFT_SERVER_FAKE_DEVICE) s->fake_th = std::thread(fake_device, s);
    *out = s;
    return SFFT_OK;
}

sfft_status_t sfft_server_submit(sfft_server_t srv, const sfft_request_t* req, uint64_t* ticket) {
    if (!srv || !req || !ticket || !req->x_dev) return set_last_error(SFFT_EINVAL, "NULL argument");
    const ShapeInfo* shape = nullptr;
    uint64_t key = 0;
    SRV_TRY(server_shape(srv, req->n, req->k, req->mode, &shape, &key));
    if (shape->bytes > srv->d.budget_bytes)
        return set_last_error(SFFT_EBUDGET, "one instance of this shape exceeds the server's budget");
    auto r = std::make_unique<Request>();
    r->r = *req;
    r->key = key;
    r->shape = shape;
    r->t_submit = Clock::now();
    std::lock_guard<std::mutex> lock(srv->mu);
    if (srv->stop) return set_last_error(SFFT_EINVAL, "server is shutting down");
    r->ticket = srv->next_ticket++;
    *ticket = r->ticket;
    if (!srv->have_first) {
        srv->have_first = true;
        srv->t_first = r->t_submit;
    }
    srv->queues[r->key].push_back(r.get());
    srv->reqs[r->ticket] = std::move(r);
    ++srv->pending;
    ++srv->events;
    srv->cv_sched.notify_all();
    return SFFT_OK;
}

static sfft_status_t take_result(sfft_server_s* s, std::unordered_map<uint64_t, std::unique_ptr<Request>>::iterator it,
                                 sfft_request_result_t* res) {
    Request* r = it->second.get();
    if (res) {
        res->status = r->status;
        res->count = r->count;
        res->flags = r->flags;
        res->rounds = r->rounds;
        res->path = r->path;
        res->queue_ms = r->t_launch.time_since_epoch().count() ? ms_between(r->t_submit, r->t_launch) : 0.0;
        res->service_ms = r->t_launch.time_since_epoch().count() ? ms_between(r->t_launch, r->t_done) : 0.0;
        res->latency_ms = ms_between(r->t_submit, r->t_done);
        std::memset(res->message, 0, sizeof(res->message));
        std::strncpy(res->message, r->message.c_str(), sizeof(res->message) - 1);
    }
    const sfft_status_t st = (sfft_status_t)r->status;
    s->reqs.erase(it);
    return st;
}

sfft_status_t sfft_server_cancel(sfft_server_t srv, uint64_t ticket) {
    if (!srv) return set_last_error(SFFT_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lock(srv->mu);
    auto it = srv->reqs.find(ticket);
    if (it == srv->reqs.end()) return set_last_error(SFFT_EINVAL, "unknown ticket");
    Request* r = it->second.get();
    if (r->launched || r->done) return SFFT_EAGAIN;
    auto& q = srv->queues[r->key];
    q.erase(std::find(q.begin(), q.end(), r));
    --srv->pending;
    r->status = SFFT_ECANCELED;
    r->message = "canceled";
    r->t_done = Clock::now();
    r->done = true;
    srv->cv_done.notify_all();
    ++srv->events;
    srv->cv_sched.notify_all();
    return SFFT_OK;
}

sfft_status_t sfft_server_poll(sfft_server_t srv, uint64_t ticket, sfft_request_result_t* res) {
    if (!srv) return set_last_error(SFFT_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lock(srv->mu);
    auto it = srv->reqs.find(ticket);
    if (it == srv->reqs.end()) return set_last_error(SFFT_EINVAL, "unknown ticket");
    if (!it->second->done) return SFFT_EAGAIN;
    return take_result(srv, it, res);
}

sfft_status_t sfft_server_wait(sfft_server_t srv, uint64_t ticket, double timeout_ms, sfft_request_result_t* res) {
    if (!srv) return set_last_error(SFFT_EINVAL, "NULL argument");
    std::unique_lock<std::mutex> lk(srv->mu);
    auto it = srv->reqs.find(ticket);
    if (it == srv->reqs.end()) return set_last_error(SFFT_EINVAL, "unknown ticket");
    Request* r = it->second.get();
    const auto pred = [&] { return r->done; };
    if (timeout_ms < 0) {
        srv->cv_done.wait(lk, pred);
    } else if (!srv->cv_done.wait_for(lk, std::chrono::duration<double, std::milli>(timeout_ms), pred)) {
        return SFFT_EAGAIN;
    }
    return take_result(srv, srv->reqs.find(ticket), res);
}

sfft_status_t sfft_server_stats(sfft_server_t srv, sfft_server_stats_t* st) {
    if (!srv || !st) return set_last_error(SFFT_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lock(srv->mu);
    std::memset(st, 0, sizeof(*st));
    st->completed = srv->completed;
    st->dense = srv->dense;
    st->failed = srv->failed;
    st->batches = srv->batches;
    st->evictions = srv->evictions;
    st->pending = srv->pending;
    st->inflight = srv->inflight;
    st->instances = (uint32_t)srv->inst.size();
    st->bytes_in_use = srv->bytes_in_use;
    st->peak_bytes = srv->peak_bytes;
    st->mean_batch = srv->batches ? (double)srv->batched / (double)srv->batches : 0.0;
    st->p50_ms = percentile(srv->lat_ms, 50);
    st->p99_ms = percentile(srv->lat_ms, 99);
    st->queue_p50_ms = percentile(srv->queue_ms, 50);
    st->service_p50_ms = percentile(srv->service_ms, 50);
    const double span = srv->have_first ? ms_between(srv->t_first, srv->t_last) : 0.0;
    st->rate = span > 0 ? (double)srv->completed / (span * 1e-3) : 0.0;
    return SFFT_OK;
}

sfft_status_t sfft_server_reset_stats(sfft_server_t srv) {
    if (!srv) return set_last_error(SFFT_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lock(srv->mu);
    srv->lat_ms.clear();
    srv->queue_ms.clear();
    srv->service_ms.clear();
    srv->completed = srv->dense = srv->failed = srv->batches = srv->batched = srv->evictions = 0;
    srv->have_first = false;
    srv->peak_bytes = srv->bytes_in_use;
    return SFFT_OK;
}

sfft_status_t sfft_server_destroy(sfft_server_t srv) {
    if (!srv) return SFFT_OK;
    {
        std::lock_guard<std::mutex> lock(srv->mu);
        srv->stop = true;
        ++srv->events;
        srv->cv_sched.notify_all();
    }
    if (srv->th.joinable()) srv->th.join();
    {
        std::unique_lock<std::mutex> lk(srv->mu);
        srv->cv_fake.notify_all();
        srv->cv_build.wait(lk, [&] { return srv->builders == 0; });   // builds of canceled requests
    }
    if (srv->fake_th.joinable()) srv->fake_th.join();
    for (auto& up : srv->inst)
        if (up->build_status == SFFT_OK) destroy_instance(up.get());   // failed builds are already released
    delete srv;
    return SFFT_OK;
}

}  // extern "C"
