// Host runtime and C ABI of the CasHash matcher (see include/cashash.h).
//
// Device-memory mode runs every step on caller buffers already in HBM.
// Host-memory mode streams images to the device under a byte budget: blocks
// of images are resident at a time and block pairs are visited in the load
// order of the paper's matching scheduler ("Data Scheduling Strategy for
// Image Matching"), with the next block prefetched on a copy stream.
#include <algorithm>
#include <cstdarg>
#include <cstdlib>
#include <map>
#include <memory>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include <fcntl.h>
#include <sys/stat.h>
#include <unistd.h>

#include <future>
#include <mutex>
#include <thread>

#include "cashash.h"
#include "cashash_internal.h"
#include "cashash_launch.h"
#include "cashash_pool.h"
#include "cashash_sched.h"

using namespace cashash;

// ------------------------------------------------------------------ errors
static thread_local std::string g_err;

static int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
static int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIPCHK(x)                                                                                   \
    do {                                                                                            \
        hipError_t e_ = (x);                                                                        \
        if (e_ != hipSuccess)                                                                       \
            return fail(e_ == hipErrorOutOfMemory ? CASHASH_E_NOMEM : CASHASH_E_DEVICE, "%s: %s (%s:%d)", \
                        #x, hipGetErrorString(e_), __FILE__, __LINE__);                           \
    } while (0)

#define RETCHK(x)            \
    do {                     \
        int r_ = (x);        \
        if (r_ != CASHASH_OK) return r_; \
    } while (0)

// ------------------------------------------------------------------ buffers
// Waits for the work queued on the context's own streams (defined below).
static void quiesce(const cashash_ctx* c);

struct DevBuf {
    void* p = nullptr;
    size_t cap = 0;
    const cashash_ctx* owner = nullptr;  // whose streams may still use the block
    int ensure(size_t n) {
        if (n <= cap && p) return CASHASH_OK;
        if (p) {
            quiesce(owner);  // the context's kernels in flight may still read the old block
            hipFree(p);
        }
        p = nullptr;
        cap = 0;
        size_t want = std::max<size_t>(n, 256);
        if (hipMalloc(&p, want) != hipSuccess) {
            p = nullptr;
            return fail(CASHASH_E_NOMEM, "device allocation of %zu bytes failed", want);
        }
        cap = want;
        return CASHASH_OK;
    }
    template <class T> T* as() const { return reinterpret_cast<T*>(p); }
    void release() {
        if (p) hipFree(p);
        p = nullptr;
        cap = 0;
    }
};

struct HostPinned {
    void* p = nullptr;
    size_t cap = 0;
    const cashash_ctx* owner = nullptr;  // whose copies may still use the block
    int ensure(size_t n) {
        if (n <= cap && p) return CASHASH_OK;
        if (p) {
            quiesce(owner);  // a copy of an earlier, failed call may still be in flight
            hipHostFree(p);
        }
        p = nullptr;
        cap = 0;
        size_t want = std::max<size_t>(n, 4096);
        if (hipHostMalloc(&p, want, hipHostMallocDefault) != hipSuccess) {
            p = nullptr;
            return fail(CASHASH_E_NOMEM, "pinned host allocation of %zu bytes failed", want);
        }
        cap = want;
        return CASHASH_OK;
    }
    void release() {
        if (p) hipHostFree(p);
        p = nullptr;
        cap = 0;
    }
};

// Small host vectors are staged into one pinned block and uploaded with a
// single copy; each piece is 256-byte aligned on the device.
struct Uploader {
    std::vector<uint8_t> host;
    std::vector<size_t> offs;
    template <class T> size_t add(const std::vector<T>& v) {
        size_t off = (host.size() + 255) & ~size_t(255);
        host.resize(off + v.size() * sizeof(T));
        if (!v.empty()) std::memcpy(host.data() + off, v.data(), v.size() * sizeof(T));
        offs.push_back(off);
        return off;
    }
};

// Matcher launch shape: queries per work item and persistent blocks per CU.
struct Shape {
    int qt;
    int bpc;
};

struct cashash_ctx {
    int device = 0;
    cashash_config cfg{};
    hipStream_t stream = nullptr;
    bool own_stream = false;
    hipStream_t copy_stream = nullptr;
    // host-memory mode: output downloads, apart from the uploads on
    // copy_stream, so that both directions of the link are busy at once and
    // a part's download overlaps the next part's kernels
    hipStream_t d2h_stream = nullptr;
    int n_cu = 256;
    std::vector<double> R64;  // [176][128]
    DevBuf dR64, dR32, dFrag, dBias, dS, dCount;
    // uploaded tables (images, pairs, tiles ...): one double-buffered area for
    // the code builder and one for the matcher, so that the matcher's table
    // addresses (baked into captured launches) do not move between calls
    DevBuf meta[3][2];
    HostPinned meta_host[3][2];
    hipEvent_t meta_ev[3][2] = {{nullptr, nullptr}, {nullptr, nullptr}, {nullptr, nullptr}};
    int meta_turn[3] = {0, 0, 0};
    std::vector<uint8_t> meta_last[3][2];  // bytes each meta buffer holds (empty: unknown)
    const void* meta_last_at[3][2] = {};   // ... at this device address
    DevBuf near, tables;      // near-margin masks; bucket tables
    // device-resident row chunks of the last image-size list seen by the
    // device-memory code builder (column sums: 2048 rows, projection: 16
    // rows), reused while the sizes repeat
    std::vector<int32_t> chunk_key;
    DevBuf chunk_dev;
    int chunk_ncol = 0, chunk_ntile = 0;
    DevBuf stage, outbuf[2];  // host-memory mode: resident image slots; part outputs (two parts in flight)
    HostPinned pin[2];        // host-memory mode upload staging
    hipEvent_t pin_ev[2] = {nullptr, nullptr};
    int pin_turn = 0;
    HostPinned pin_out[2], pin_small;
    hipEvent_t slot_load_ev[3] = {nullptr, nullptr, nullptr};
    hipEvent_t slot_free_ev[3] = {nullptr, nullptr, nullptr};
    hipEvent_t ev0 = nullptr, ev1 = nullptr;  // autotuner timing
    // per match job in flight (host-memory mode keeps two): kernel start and
    // end, and the end of its output download
    hipEvent_t job_ev[2][3] = {{nullptr, nullptr, nullptr}, {nullptr, nullptr, nullptr}};
    hipEvent_t part_ev[2] = {nullptr, nullptr};  // host-memory mode: a part's kernels are done
    int job_turn = 0;
    std::unique_ptr<WorkPool> pool;  // host threads of the bulk host copies
    double last_ms = 0.0;
    int64_t last_launches = 0;
    DevBuf items;             // matcher work items of the current job
    // captured persistent-matcher launches, keyed by their launch arguments
    struct GraphEntry {
        std::string key;
        hipGraphExec_t exec;
        uint64_t used;
    };
    std::vector<GraphEntry> graphs;
    uint64_t graph_clock = 0;
    bool use_graphs = true;
    int64_t graph_replays = 0;
    bool last_replayed = false;
    DevBuf counters;          // per-segment work counters of the persistent matcher
    std::map<std::string, Shape> tuned;
    bool tune_loaded = false;
    int last_shape_qt = 0, last_shape_bpc = 0;
    // geometry-aware first stage: subset images, stage-1 outputs, per-pair
    // results and error flags; stage boundary events of the two-stage call
    DevBuf geo_sub, geo_m1, geo_pair, geo_err;
    hipEvent_t geo_ev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    double geo_ms[4] = {0, 0, 0, 0};
    // recorded on the caller's legacy default stream at each entry point when
    // the context runs on a stream of its own (cfg.stream == NULL)
    hipEvent_t caller_ev = nullptr;
    // device address of this device's allocation-free scratch array (null if
    // it could not be looked up; scratch_err says why)
    uint8_t* scratch = nullptr;
    std::string scratch_err;
};

static void quiesce(const cashash_ctx* c) {
    if (!c) return;
    if (c->stream) hipStreamSynchronize(c->stream);
    if (c->copy_stream) hipStreamSynchronize(c->copy_stream);
    if (c->d2h_stream) hipStreamSynchronize(c->d2h_stream);
}

static std::vector<DevBuf*> dev_bufs(cashash_ctx* c) {
    return {&c->dR64, &c->dR32, &c->dFrag, &c->dBias, &c->dS, &c->dCount, &c->meta[0][0], &c->meta[0][1],
            &c->meta[1][0], &c->meta[1][1], &c->meta[2][0], &c->meta[2][1], &c->near, &c->tables, &c->stage,
            &c->outbuf[0], &c->outbuf[1], &c->items, &c->counters, &c->geo_sub, &c->geo_m1, &c->geo_pair, &c->geo_err, &c->chunk_dev};
}

static int validate_config(const cashash_config* c) {
    if (c->k < 1 || c->k > CASHASH_MAX_K) return fail(CASHASH_E_LIMIT, "k=%d outside 1..%d", c->k, CASHASH_MAX_K);
    if (c->ratio_num <= 0 || c->ratio_den <= 0 || c->ratio_num > 65535 || c->ratio_den > 65535)
        return fail(CASHASH_E_INVAL, "ratio %d/%d: both must be in 1..65535", c->ratio_num, c->ratio_den);
    if (c->max_hamming < 0 || c->max_hamming > 128)
        return fail(CASHASH_E_LIMIT, "max_hamming=%d outside 0..128", c->max_hamming);
    if (!(c->margin_coef > 0.0) || !std::isfinite(c->margin_coef) || c->margin_coef > 1e3)
        return fail(CASHASH_E_INVAL, "margin_coef must be positive and finite");
    if (c->mode != CASHASH_MODE_BATCHED_BF16X2 && c->mode != CASHASH_MODE_PLAIN_FP32_PER_PAIR)
        return fail(CASHASH_E_INVAL, "unknown mode %d", c->mode);
    if (c->mem != CASHASH_MEM_HOST && c->mem != CASHASH_MEM_DEVICE)
        return fail(CASHASH_E_INVAL, "unknown mem %d", c->mem);
    if (c->device_budget_bytes < 0) return fail(CASHASH_E_INVAL, "negative device budget");
    return CASHASH_OK;
}

// The fast projection's rounding error is below 4.6e-5 |r| |x| (bf16 hi+lo
// representation 2^-16 |r||x| plus fp32 accumulation of 256 exact products
// even with round-toward-zero, 2^-23 * 256 |r||x|), so it is trusted outside
// margin_coef |x| only when 5e-5 |r| < margin_coef.
static int check_rows(const std::vector<double>& R, double coef) {
    for (int j = 0; j < kRows; ++j) {
        double s = 0.0;
        for (int i = 0; i < kDim; ++i) {
            const double v = R[j * kDim + i];
            if (!std::isfinite(v)) return fail(CASHASH_E_UNSAFE_MATRIX, "row %d has a non-finite entry", j);
            s += v * v;
        }
        if (!(5e-5 * std::sqrt(s) < coef))
            return fail(CASHASH_E_UNSAFE_MATRIX, "row %d has norm %.4g: 5e-5*norm must be < margin_coef=%.4g", j,
                        std::sqrt(s), coef);
    }
    return CASHASH_OK;
}

static uint16_t bf16_round(float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    const uint32_t lsb = (u >> 16) & 1u;
    u += 0x7FFFu + lsb;  // round to nearest even (values are finite)
    return (uint16_t)(u >> 16);
}
static double bf16_value(uint16_t h) {
    uint32_t u = (uint32_t)h << 16;
    float f;
    std::memcpy(&f, &u, 4);
    return (double)f;
}

// hi = bf16(r) and lo = bf16(r - hi) (r - hi is exact in binary64), laid out
// as the MFMA A-operand fragments lane l loads for (part, row tile, k step).
static std::vector<uint16_t> make_frag(const std::vector<double>& R) {
    std::vector<uint16_t> f((size_t)kFragBytes / 2);
    for (int rt = 0; rt < kRowTiles; ++rt)
        for (int ks = 0; ks < 4; ++ks)
            for (int l = 0; l < 64; ++l)
                for (int i = 0; i < 8; ++i) {
                    const double r = R[(16 * rt + l % 16) * kDim + 32 * ks + 8 * (l / 16) + i];
                    // round binary64 -> bf16 through fp32: exact for the hi part's
                    // purpose since any rounding error is absorbed by lo
                    const uint16_t hi = bf16_round((float)r);
                    const uint16_t lo = bf16_round((float)(r - bf16_value(hi)));
                    f[((((size_t)0 * kRowTiles + rt) * 4 + ks) * 64 + l) * 8 + i] = hi;
                    f[((((size_t)1 * kRowTiles + rt) * 4 + ks) * 64 + l) * 8 + i] = lo;
                }
    return f;
}

extern "C" void cashash_default_config(cashash_config* c) {
    if (!c) return;
    c->k = 10;
    c->ratio_num = 4;
    c->ratio_den = 5;
    c->max_hamming = 128;
    c->margin_coef = 1e-3;
    c->mode = CASHASH_MODE_BATCHED_BF16X2;
    c->mem = CASHASH_MEM_DEVICE;
    c->device_budget_bytes = 0;
    c->stream = nullptr;
}

extern "C" const char* cashash_last_error(void) { return g_err.c_str(); }

static void destroy_ctx(cashash_ctx* c) {
    if (!c) return;
    if (c->stream) hipStreamSynchronize(c->stream);
    for (hipStream_t* st : {&c->copy_stream, &c->d2h_stream})
        if (*st) {
            hipStreamSynchronize(*st);
            hipStreamDestroy(*st);
        }
    for (DevBuf* b : dev_bufs(c)) b->release();
    for (HostPinned* h : {&c->meta_host[0][0], &c->meta_host[0][1], &c->meta_host[1][0], &c->meta_host[1][1],
                          &c->meta_host[2][0], &c->meta_host[2][1], &c->pin[0], &c->pin[1], &c->pin_out[0], &c->pin_out[1],
                          &c->pin_small})
        h->release();
    for (hipEvent_t e : {c->ev0, c->ev1, c->meta_ev[0][0], c->meta_ev[0][1], c->meta_ev[1][0], c->meta_ev[1][1],
                         c->meta_ev[2][0], c->meta_ev[2][1], c->geo_ev[0], c->geo_ev[1], c->geo_ev[2], c->geo_ev[3],
                         c->geo_ev[4], c->pin_ev[0], c->pin_ev[1],
                         c->slot_load_ev[0], c->slot_load_ev[1], c->slot_load_ev[2], c->slot_free_ev[0],
                         c->slot_free_ev[1], c->slot_free_ev[2], c->caller_ev, c->job_ev[0][0], c->job_ev[0][1],
                         c->job_ev[0][2], c->job_ev[1][0], c->job_ev[1][1], c->job_ev[1][2], c->part_ev[0],
                         c->part_ev[1]})
        if (e) hipEventDestroy(e);
    for (auto& g : c->graphs) hipGraphExecDestroy(g.exec);
    if (c->own_stream && c->stream) hipStreamDestroy(c->stream);
    delete c;
}

extern "C" void cashash_destroy(cashash_ctx* c) { destroy_ctx(c); }

extern "C" int cashash_set_config(cashash_ctx* c, const cashash_config* cfg) {
    if (!c) return fail(CASHASH_E_INVAL, "null context");
    cashash_config n;
    if (cfg)
        n = *cfg;
    else
        cashash_default_config(&n);
    RETCHK(validate_config(&n));
    RETCHK(check_rows(c->R64, n.margin_coef));
    if (n.stream != c->cfg.stream || !c->stream) {
        if (c->stream) hipStreamSynchronize(c->stream);
        if (c->own_stream && c->stream) hipStreamDestroy(c->stream);
        c->stream = nullptr;
        c->own_stream = false;
        if (n.stream) {
            c->stream = (hipStream_t)n.stream;
        } else {
            HIPCHK(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
            c->own_stream = true;
        }
    }
    c->cfg = n;
    return CASHASH_OK;
}

// ------------------------------------------------------------------ allocation-free scratch
// The one device region of cashash_match_pairs_noalloc.  Every GPU the
// library runs on holds its own copy at its own address until the process
// ends.  In host code `scratch` only names the symbol: its device address is
// looked up once per device (hipGetSymbolAddress, with that device current,
// at the first context created on it) and only that address is ever passed
// to kernels or copies.
static __device__ __align__(256) uint8_t scratch[CASHASH_NOALLOC_SCRATCH_BYTES];
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static uint8_t* g_scratch_addr[kMaxDevices];
static hipError_t g_scratch_rc[kMaxDevices];
static bool g_scratch_done[kMaxDevices];

// Device address of `scratch` on `dev` (which must be the current device).
static uint8_t* scratch_address(int dev, std::string& err) {
    if (dev < 0 || dev >= kMaxDevices) {
        err = "device index beyond the scratch table";
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_done[dev]) {
        void* p = nullptr;
        g_scratch_rc[dev] = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        g_scratch_addr[dev] = g_scratch_rc[dev] == hipSuccess ? static_cast<uint8_t*>(p) : nullptr;
        g_scratch_done[dev] = true;
    }
    if (!g_scratch_addr[dev]) {
        err = std::string("hipGetSymbolAddress of the scratch array failed: ") + hipGetErrorString(g_scratch_rc[dev]);
        hipGetLastError();  // do not leave the failure for the next call to report
    }
    return g_scratch_addr[dev];
}

extern "C" int cashash_create(cashash_ctx** out, const double* r_code, const double* r_bucket,
                              const cashash_config* cfg) {
    if (!out || !r_code || !r_bucket) return fail(CASHASH_E_INVAL, "null argument to cashash_create");
    *out = nullptr;
    cashash_config n;
    if (cfg)
        n = *cfg;
    else
        cashash_default_config(&n);
    RETCHK(validate_config(&n));
    std::vector<double> R((size_t)kRows * kDim);
    std::memcpy(R.data(), r_code, sizeof(double) * kCodeBits * kDim);
    std::memcpy(R.data() + (size_t)kCodeBits * kDim, r_bucket, sizeof(double) * kTables * kKeyBits * kDim);
    RETCHK(check_rows(R, n.margin_coef));
    cashash_ctx* c = new cashash_ctx();
    c->R64 = std::move(R);
    for (DevBuf* b : dev_bufs(c)) b->owner = c;
    for (HostPinned* h : {&c->meta_host[0][0], &c->meta_host[0][1], &c->meta_host[1][0], &c->meta_host[1][1],
                          &c->meta_host[2][0], &c->meta_host[2][1], &c->pin[0], &c->pin[1], &c->pin_out[0],
                          &c->pin_out[1], &c->pin_small})
        h->owner = c;
    auto bail = [&](int code) {
        std::string keep = g_err;
        destroy_ctx(c);
        g_err = keep;
        return code;
    };
    if (hipGetDevice(&c->device) != hipSuccess) return bail(fail(CASHASH_E_DEVICE, "no HIP device"));
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, c->device) != hipSuccess)
        return bail(fail(CASHASH_E_DEVICE, "hipGetDeviceProperties failed"));
    c->n_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
    c->scratch = scratch_address(c->device, c->scratch_err);
    {
        const char* g = std::getenv("CASHASH_GRAPHS");
        c->use_graphs = !(g && g[0] == '0');
    }
    int r = cashash_set_config(c, &n);
    if (r) return bail(r);
    if (hipStreamCreateWithFlags(&c->copy_stream, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&c->d2h_stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreate(&c->ev0) != hipSuccess || hipEventCreate(&c->ev1) != hipSuccess)
        return bail(fail(CASHASH_E_DEVICE, "stream/event creation failed"));
    for (int i = 0; i < 5; ++i)
        if (hipEventCreate(&c->geo_ev[i]) != hipSuccess) return bail(fail(CASHASH_E_DEVICE, "event creation failed"));
    for (int j = 0; j < 2; ++j)
        if (hipEventCreate(&c->job_ev[j][0]) != hipSuccess || hipEventCreate(&c->job_ev[j][1]) != hipSuccess ||
            hipEventCreateWithFlags(&c->job_ev[j][2], hipEventDisableTiming) != hipSuccess)
            return bail(fail(CASHASH_E_DEVICE, "event creation failed"));
    {
        // host copy threads: CASHASH_HOST_THREADS, else up to 16 of the host's
        int nt = (int)std::min(16u, std::max(1u, std::thread::hardware_concurrency()));
        if (const char* e = std::getenv("CASHASH_HOST_THREADS")) nt = std::max(1, std::min(64, std::atoi(e)));
        c->pool.reset(new WorkPool(nt));
    }
    for (hipEvent_t* e : {&c->meta_ev[0][0], &c->meta_ev[0][1], &c->meta_ev[1][0], &c->meta_ev[1][1],
                          &c->meta_ev[2][0], &c->meta_ev[2][1], &c->pin_ev[0], &c->pin_ev[1], &c->slot_load_ev[0],
                          &c->slot_load_ev[1], &c->slot_load_ev[2], &c->slot_free_ev[0], &c->slot_free_ev[1],
                          &c->slot_free_ev[2], &c->caller_ev, &c->part_ev[0], &c->part_ev[1]})
        if (hipEventCreateWithFlags(e, hipEventDisableTiming) != hipSuccess)
            return bail(fail(CASHASH_E_DEVICE, "event creation failed"));
    if ((r = c->pin_small.ensure(4096))) return bail(r);
    std::vector<float> R32(c->R64.size());
    for (size_t i = 0; i < R32.size(); ++i) R32[i] = (float)c->R64[i];
    std::vector<uint16_t> frag = make_frag(c->R64);
    if ((r = c->dR64.ensure(c->R64.size() * 8)) || (r = c->dR32.ensure(R32.size() * 4)) ||
        (r = c->dFrag.ensure(frag.size() * 2)) || (r = c->dBias.ensure(kRows * 4)) || (r = c->dS.ensure(kDim * 8)) ||
        (r = c->dCount.ensure(64 * 8)) || (r = c->counters.ensure(kSegments * kCounterStride * 4)))
        return bail(r);
    if (hipMemcpy(c->dR64.p, c->R64.data(), c->R64.size() * 8, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(c->dR32.p, R32.data(), R32.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(c->dFrag.p, frag.data(), frag.size() * 2, hipMemcpyHostToDevice) != hipSuccess)
        return bail(fail(CASHASH_E_DEVICE, "upload of projection matrices failed"));
    *out = c;
    return CASHASH_OK;
}

extern "C" int cashash_last_kernel_ms(cashash_ctx* c, double* ms, int64_t* launches) {
    if (!c || !ms || !launches) return fail(CASHASH_E_INVAL, "null argument");
    *ms = c->last_ms;
    *launches = c->last_launches;
    return CASHASH_OK;
}

// ------------------------------------------------------------------ helpers
static double now_ms() {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// A caller that passes no stream works on the legacy default stream, where
// it may still have work queued that writes this call's inputs or reads its
// output buffers (a caching allocator hands out blocks as soon as their last
// use is queued).  The context's own stream is non-blocking, so it is made
// to wait for everything queued there so far.  A caller stream given in
// cfg.stream is the context's stream itself and is ordered already.
static int follow_caller(cashash_ctx* c) {
    if (!c->own_stream) return CASHASH_OK;
    // nothing the caller queued is still pending: no ordering needed (saves
    // the event record and the stream wait, tens of microseconds per call)
    const hipError_t q = hipStreamQuery(nullptr);
    if (q == hipSuccess) return CASHASH_OK;
    if (q != hipErrorNotReady) HIPCHK(q);
    HIPCHK(hipEventRecord(c->caller_ev, nullptr));
    HIPCHK(hipStreamWaitEvent(c->stream, c->caller_ev, 0));
    return CASHASH_OK;
}

// Uploads small tables on the compute stream (so they follow the kernels that
// read the previous contents).  Two buffers alternate; a buffer's pinned
// source is rewritten only after its previous copy has completed.
enum { kMetaCodes = 0, kMetaMatch = 1, kMetaGeo = 2 };

static int upload_meta(cashash_ctx* c, Uploader& up, std::vector<const void*>& dptr, int area) {
    const int b = c->meta_turn[area];
    c->meta_turn[area] ^= 1;
    DevBuf& dev = c->meta[area][b];
    const size_t need = up.host.size();
    std::vector<uint8_t>& last = c->meta_last[area][b];
    if (!(need <= dev.cap && c->meta_last_at[area][b] == dev.p && last.size() == need &&
          std::memcmp(last.data(), up.host.data(), need) == 0)) {
        // the buffer does not hold these bytes already (a call on the same
        // inputs two calls ago left them there: no copy then)
        HIPCHK(hipEventSynchronize(c->meta_ev[area][b]));
        HostPinned& host = c->meta_host[area][b];
        if (need > dev.cap) RETCHK(dev.ensure(std::max<size_t>({need, 2 * dev.cap, (size_t)1 << 20})));
        if (need > host.cap) RETCHK(host.ensure(std::max<size_t>({need, 2 * host.cap, (size_t)1 << 20})));
        std::memcpy(host.p, up.host.data(), need);
        last.clear();  // unknown until the copy is queued
        HIPCHK(hipMemcpyAsync(dev.p, host.p, need, hipMemcpyHostToDevice, c->stream));
        HIPCHK(hipEventRecord(c->meta_ev[area][b], c->stream));
        last.assign(up.host.begin(), up.host.end());
        c->meta_last_at[area][b] = dev.p;
    }
    dptr.clear();
    for (size_t o : up.offs) dptr.push_back(dev.as<uint8_t>() + o);
    return CASHASH_OK;
}

static int check_images(const cashash_images* im) {
    if (!im || im->n_images < 0 || (im->n_images > 0 && (!im->desc || !im->n_feat)))
        return fail(CASHASH_E_INVAL, "invalid image set");
    for (int m = 0; m < im->n_images; ++m) {
        const int n = im->n_feat[m];
        if (n < 0) return fail(CASHASH_E_INVAL, "image %d: negative n_feat", m);
        if (n > CASHASH_MAX_FEAT) return fail(CASHASH_E_LIMIT, "image %d: n_feat=%d > %d", m, n, CASHASH_MAX_FEAT);
    }
    return CASHASH_OK;
}

static bool misaligned(const void* p, uintptr_t a) { return ((uintptr_t)p & (a - 1)) != 0; }
static size_t al256(size_t n) { return (n + 255) & ~size_t(255); }

// ------------------------------------------------------------------ codes (device-resident core)
struct CodeJob {
    std::vector<ImgDev> imgs;
    std::vector<CodeOut> outs;
};

// Column sums over `imgs`, accumulated into c->dS (not cleared here).
static void row_chunks(const std::vector<ImgDev>& imgs, int rows, std::vector<RowChunk>& v) {
    for (int m = 0; m < (int)imgs.size(); ++m)
        for (int r0 = 0; r0 < imgs[m].n; r0 += rows) v.push_back({m, r0, std::min(rows, imgs[m].n - r0), 0});
}

// The column-sum and projection chunks of imgs on the device, rebuilt (with a
// synchronous upload) only when the image sizes differ from the last call's.
static int cached_chunks(cashash_ctx* c, const std::vector<ImgDev>& imgs) {
    bool same = c->chunk_key.size() == imgs.size();
    for (size_t m = 0; same && m < imgs.size(); ++m) same = c->chunk_key[m] == imgs[m].n;
    if (same) return CASHASH_OK;
    std::vector<RowChunk> v;
    row_chunks(imgs, 2048, v);
    const int ncol = (int)v.size();
    row_chunks(imgs, 16, v);
    c->chunk_key.clear();
    RETCHK(c->chunk_dev.ensure(std::max<size_t>(1, v.size()) * sizeof(RowChunk)));
    HIPCHK(hipStreamSynchronize(c->stream));  // earlier kernels may still read the old chunks
    if (!v.empty()) HIPCHK(hipMemcpy(c->chunk_dev.p, v.data(), v.size() * sizeof(RowChunk), hipMemcpyHostToDevice));
    c->chunk_ncol = ncol;
    c->chunk_ntile = (int)v.size() - ncol;
    for (const ImgDev& im : imgs) c->chunk_key.push_back(im.n);
    return CASHASH_OK;
}

// Column sums of imgs into c->dS; dchunks: device chunks (cached_chunks), or
// nullptr to build and upload them with the image table.
// dI: the image table already on the device (with dchunks), or nullptr.
static int run_colsum(cashash_ctx* c, const std::vector<ImgDev>& imgs, const RowChunk* dchunks = nullptr,
                      int n_chunks = 0, const ImgDev* dI = nullptr) {
    std::vector<RowChunk> chunks;
    if (!dchunks) {
        row_chunks(imgs, 2048, chunks);
        n_chunks = (int)chunks.size();
    }
    if (n_chunks == 0) return CASHASH_OK;
    if (!dI || !dchunks) {
        Uploader up;
        up.add(imgs);
        if (!dchunks) up.add(chunks);
        std::vector<const void*> d;
        RETCHK(upload_meta(c, up, d, kMetaCodes));
        dI = (const ImgDev*)d[0];
        if (!dchunks) dchunks = (const RowChunk*)d[1];
    }
    HIPCHK(launch_colsum(c->stream, dI, dchunks, n_chunks, c->dS.as<unsigned long long>()));
    return CASHASH_OK;
}

// Projection + binary64 fix-up of `imgs` into `outs`, given c->dBias and c->dS.
// dI, dO: the image and output tables already on the device (with dtiles), or nullptr.
static int run_project(cashash_ctx* c, const std::vector<ImgDev>& imgs, std::vector<CodeOut> outs, double n_tot,
                       const RowChunk* dtiles = nullptr, int n_tiles = 0, const ImgDev* dIp = nullptr,
                       const CodeOut* dOp = nullptr) {
    std::vector<RowChunk> tiles;
    if (!dtiles) {
        row_chunks(imgs, 16, tiles);
        n_tiles = (int)tiles.size();
    }
    if (n_tiles == 0) return CASHASH_OK;
    const int nt = n_tiles;
    const bool mfma = c->cfg.mode == CASHASH_MODE_BATCHED_BF16X2;
    // near list: one segment per projection wavefront, each large enough for
    // every descriptor that wavefront handles; per-segment counts in front
    // (MFMA form: a wavefront takes groups of kProjTB tiles, kProjTB * 16 descriptors)
    const int groups = (nt + kProjTB - 1) / kProjTB;
    const int grid = mfma ? std::max(1, std::min((groups + 3) / 4, c->n_cu * 8)) : (int)(((int64_t)nt * 16 + 255) / 256);
    const uint32_t n_seg = (uint32_t)grid * 4;
    const uint32_t seg_cap = mfma ? (uint32_t)((groups + n_seg - 1) / n_seg) * kProjTB * 16 : 64;
    const uint64_t n_cap = (uint64_t)n_seg * seg_cap;
    if (n_cap >= ((uint64_t)1 << 32)) return fail(CASHASH_E_LIMIT, "more than 2^32 near-list places");
    // segment counts, near list, recompute work area
    const size_t count_bytes = al256((size_t)n_seg * 4);
    const size_t list_bytes = al256((size_t)n_cap * sizeof(NearEntry));
    RETCHK(c->near.ensure(count_bytes + list_bytes + near_work_bytes(n_cap)));
    uint32_t* seg_count = c->near.as<uint32_t>();
    NearEntry* near = reinterpret_cast<NearEntry*>(c->near.as<uint8_t>() + count_bytes);
    void* work = c->near.as<uint8_t>() + count_bytes + list_bytes;
    const ImgDev* dI = dIp;
    const CodeOut* dO = dOp;
    const RowChunk* dT = dtiles;
    if (!dI || !dO || !dtiles) {
        Uploader up;
        up.add(imgs);
        up.add(outs);
        if (!dtiles) up.add(tiles);
        std::vector<const void*> d;
        RETCHK(upload_meta(c, up, d, kMetaCodes));
        dI = (const ImgDev*)d[0];
        dO = (const CodeOut*)d[1];
        if (!dtiles) dT = (const RowChunk*)d[2];
    }
    const float coef = (float)c->cfg.margin_coef;
    if (mfma) {
        HIPCHK(launch_proj_mfma(c->stream, grid, dI, dO, dT, nt, c->dFrag.as<uint4>(), c->dBias.as<float>(), coef,
                                near, seg_count, seg_cap, work));
    } else {
        HIPCHK(launch_proj_fp32(c->stream, dI, dO, dT, nt, c->dR32.as<float>(), c->dBias.as<float>(), coef, near,
                                seg_count, work));
    }
    // the recompute: as many wavefronts as the near list has segments, at
    // most 16 per compute unit
    const int fix_grid = (int)std::max<int64_t>(1, std::min<int64_t>((n_seg + 3) / 4, (int64_t)c->n_cu * 4));
    HIPCHK(launch_near_recompute(c->stream, fix_grid, dI, dO, near, seg_count, seg_cap, n_seg, c->dR64.as<double>(),
                        c->dS.as<unsigned long long>(), n_tot, work, c->dCount.as<unsigned long long>()));
    return CASHASH_OK;
}

static int build_codes_device(cashash_ctx* c, const cashash_images* im, uint64_t* const* codes_out,
                              uint8_t* const* keys_out, int64_t* near_count) {
    std::vector<ImgDev> imgs(im->n_images);
    std::vector<CodeOut> outs(im->n_images);
    double n_tot = 0;
    for (int m = 0; m < im->n_images; ++m) {
        const int n = im->n_feat[m];
        if (n > 0 && (!im->desc[m] || !codes_out[m] || !keys_out[m]))
            return fail(CASHASH_E_INVAL, "image %d: null descriptor or output pointer", m);
        if (n > 0 && (misaligned(im->desc[m], 16) || misaligned(codes_out[m], 8) || misaligned(keys_out[m], 2)))
            return fail(CASHASH_E_INVAL, "image %d: descriptors need 16-byte, codes 8-byte, keys 2-byte alignment", m);
        imgs[m] = ImgDev{im->desc[m], nullptr, nullptr, nullptr, nullptr, nullptr, n, 0};
        outs[m] = CodeOut{codes_out[m], keys_out[m], 0};  // pad
        n_tot += n;
    }
    if (n_tot == 0) {
        *near_count = 0;
        return CASHASH_OK;
    }
    RETCHK(cached_chunks(c, imgs));
    const RowChunk* dch = c->chunk_dev.as<RowChunk>();
    // one upload of the image and output tables serves the sums and the projection
    Uploader up;
    up.add(imgs);
    up.add(outs);
    std::vector<const void*> d;
    RETCHK(upload_meta(c, up, d, kMetaCodes));
    HIPCHK(launch_fill_u64(c->stream, c->dS.as<unsigned long long>(), kDim, 0ull));
    HIPCHK(launch_fill_u64(c->stream, c->dCount.as<unsigned long long>(), 8, 0ull));
    RETCHK(run_colsum(c, imgs, dch, c->chunk_ncol, (const ImgDev*)d[0]));
    HIPCHK(launch_bias(c->stream, c->dR64.as<double>(), c->dS.as<unsigned long long>(), n_tot, c->dBias.as<float>()));
    RETCHK(run_project(c, imgs, outs, n_tot, dch + c->chunk_ncol, c->chunk_ntile, (const ImgDev*)d[0],
                       (const CodeOut*)d[1]));
    // the recompute count through pinned memory (offset 128 of pin_small)
    unsigned long long* pc = reinterpret_cast<unsigned long long*>(static_cast<uint8_t*>(c->pin_small.p) + 128);
    HIPCHK(hipMemcpyAsync(pc, c->dCount.p, 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    *near_count = (int64_t)*pc;
    return CASHASH_OK;
}

// ------------------------------------------------------------------ matching (device-resident core)
struct MatchJob {
    bool epi = false;
    double max_px = 0.0;
    std::vector<ImgDev> imgs;      // all images (train ones get tables)
    std::vector<int32_t> pair_q, pair_t;
    std::vector<int64_t> pair_out; // first output slot of each pair
    const double* F = nullptr;     // host [n_pairs][9]
    int32_t* o_idx = nullptr;      // device outputs
    int32_t* o_d1 = nullptr;
    int32_t* o_d2 = nullptr;
    int64_t bucket_entries = 0, union_size = 0, ranked = 0;
    int turn = 0;                  // which of the two in-flight job slots (events, statistics) it uses
};

// ------------------------------------------------------------------ launch shape and autotuning
// A launch shape is the number of queries per work item (one wavefront takes
// one item at a time) and, for the persistent batched launch, the number of
// resident blocks per compute unit.  A tile's kept candidates must fit the
// per-wave tile list: qt * k <= kSelCap (kSelCapEpi for the band kernel, which
// also tries 7 blocks per compute unit, the occupancy it is compiled for).

static int sel_cap(bool epi) { return epi ? kSelCapEpi : kSelCap; }

static std::vector<Shape> shape_candidates(int k, bool batched, bool epi) {
    std::vector<Shape> v;
    const int qmax = std::min(kMaxTile, sel_cap(epi) / k);
    if (batched) {
        // persistent blocks per CU: around the occupancy each kernel is
        // compiled for (7 blocks for the band kernel, 6 or 5 for the others)
        static const int kBpcPlain[3] = {4, 6, 8}, kBpcEpi[3] = {6, 7, 8};
        const int* bpcs = epi ? kBpcEpi : kBpcPlain;
        for (int qt : {8, 16, 32})
            for (int i = 0; i < 3; ++i)
                if (qt <= qmax || qt == 16) v.push_back(Shape{std::min(qt, qmax), bpcs[i]});
    } else {
        for (int qt : {1, 2, 4, 8, 16, 32})
            if (qt <= qmax) v.push_back(Shape{qt, 0});
    }
    // drop duplicates from clamping
    std::vector<Shape> u;
    for (const Shape& s : v) {
        bool dup = false;
        for (const Shape& t : u) dup |= (t.qt == s.qt && t.bpc == s.bpc);
        if (!dup) u.push_back(s);
    }
    return u;
}

static Shape default_shape(int k, bool batched, bool epi) {
    return batched ? Shape{std::min(kMaxTile, sel_cap(epi) / k), epi ? 7 : 6} : Shape{std::min(4, sel_cap(epi) / k), 0};
}

static bool autotune_enabled() {
    const char* e = std::getenv("CASHASH_AUTOTUNE");
    return !(e && e[0] == '0');
}

// Shapes are cached per (form, epipolar, k, train size class, query size
// class), in memory and, if CASHASH_AUTOTUNE_CACHE names a file, as JSON lines.
static std::string tune_key(bool batched, bool epi, int k, double mean_nt, double mean_nq) {
    char b[128];
    snprintf(b, sizeof b, "gfx950/%s/%s/k%d/nt%d/nq%d", batched ? "batched" : "plain", epi ? "epi" : "plain", k,
             (int)std::lround(std::log2(std::max(1.0, mean_nt))), (int)std::lround(std::log2(std::max(1.0, mean_nq))));
    return b;
}

static void tune_cache_load(cashash_ctx* c);
static void tune_cache_store(cashash_ctx* c, const std::string& key, Shape sh);

// Per-pair item tables for one query-tile size, in processing order.
static std::vector<PairTiles> pair_tiles(const MatchJob& J, const std::vector<int64_t>& order, int qt,
                                         std::vector<int64_t>* first_of) {
    std::vector<PairTiles> pt;
    int64_t items = 0;
    if (first_of) first_of->assign(order.size() + 1, 0);
    for (size_t oi = 0; oi < order.size(); ++oi) {
        const int64_t p = order[oi];
        const int nq = J.imgs[J.pair_q[p]].n;
        if (first_of) (*first_of)[oi] = items;
        if (nq == 0) continue;
        pt.push_back(PairTiles{(int32_t)p, (int32_t)items});
        items += (nq + qt - 1) / qt;
    }
    if (first_of) (*first_of)[order.size()] = items;
    return pt;
}

struct MatchPlan {
    const ImgDev* dI = nullptr;
    const PairDev* dP = nullptr;
    MatchParams prm{};
    std::vector<int64_t> order;
    Item* items = nullptr;          // work items (items_cap of them)
    int64_t items_cap = 0;
    uint32_t* counter = nullptr;    // per-segment work counters of the persistent launch
};

// Segment boundaries (in items) that split the estimated cost (queries x
// train size) of the first n_run items, taken in pair order, into kSegments
// nearly equal parts.  Costs are summed per pair; inside a pair every tile
// but the last has qt queries.
static void segment_bounds(const MatchJob& J, const std::vector<int64_t>& order, const std::vector<int64_t>& first_of,
                           int qt, int64_t oi_lo, int64_t oi_hi, int64_t item_lo, int64_t item_hi, int32_t* seg) {
    // items are relative to item_lo in the result
    const int64_t n_run = item_hi - item_lo;
    std::vector<double> cum((size_t)(oi_hi - oi_lo) + 1, 0.0);
    for (int64_t oi = oi_lo; oi < oi_hi; ++oi) {
        const int64_t p = order[oi];
        const int64_t lo = first_of[oi], hi = std::min(first_of[oi + 1], item_hi);
        const double nq_run = hi > lo ? std::min<double>(J.imgs[J.pair_q[p]].n, (double)(hi - lo) * qt) : 0.0;
        cum[oi - oi_lo + 1] = cum[oi - oi_lo] + nq_run * std::max(1, J.imgs[J.pair_t[p]].n);
    }
    const double total = cum.back();
    for (int x = 0; x <= kSegments; ++x) {
        const double target = total * x / kSegments;
        const size_t k = (size_t)(std::lower_bound(cum.begin(), cum.end(), target) - cum.begin());
        int64_t item = 0;
        if (k > 0) {
            // inside pair k-1 of the range: place the boundary proportionally to its cost
            const int64_t oi = oi_lo + (int64_t)k - 1;
            const double c0 = cum[k - 1], c1 = cum[k];
            const int64_t lo = first_of[oi] - item_lo, hi = std::min(first_of[oi + 1], item_hi) - item_lo;
            const double f = c1 > c0 ? (target - c0) / (c1 - c0) : 1.0;
            item = lo + (int64_t)std::llround(f * (double)(hi - lo));
        }
        seg[x] = (int32_t)std::min<int64_t>(std::max<int64_t>(item, 0), n_run);
    }
    seg[0] = 0;
    seg[kSegments] = (int32_t)n_run;
    for (int x = 1; x <= kSegments; ++x) seg[x] = std::max(seg[x], seg[x - 1]);
}

// Register slots of the matcher instantiation a pair runs in.
static int slots_for(const MatchJob& J, int64_t p) {
    const int n = J.imgs[J.pair_t[p]].n;
    return J.epi || n <= kLargeTrain ? 4 : n <= kHugeTrain ? 6 : 8;
}

// Generate the work items of shape qt on the device (into P.items, which
// holds P.items_cap of them).
static int make_items(cashash_ctx* c, const MatchPlan& P, int qt, const PairTiles* dPT, int32_t n_pt,
                      int64_t n_items) {
    if (n_items > (int64_t)INT32_MAX) return fail(CASHASH_E_LIMIT, "too many query tiles in one call");
    if (n_items > P.items_cap) return fail(CASHASH_E_INVAL, "work item buffer too small");
    HIPCHK(launch_make_items(c->stream, dPT, n_pt, P.dP, P.dI, qt, P.items, (int32_t)n_items));
    return CASHASH_OK;
}

// The matcher over items [0, n_items) (batched: one persistent launch) or,
// in the plain form, one launch per pair over its own items.
static int enqueue_matcher(cashash_ctx* c, const MatchPlan& P, MatchJob& J, Shape sh, bool batched,
                           const std::vector<int64_t>& first_of, int64_t n_pairs_run, int64_t n_items,
                           unsigned long long* stats, int64_t* launches, bool use_graph) {
    uint32_t* counter = P.counter;
    const Item* items = P.items;
    if (batched) {
        // one persistent launch per register-slot group (pairs are ordered
        // small-train group first), each over its own item range
        struct Launch {
            int ns, grid;
            int64_t item_lo, n;
            MatchParams prm;
        };
        std::vector<Launch> ls;
        int64_t oi = 0;
        while (oi < n_pairs_run) {
            const int ns = slots_for(J, P.order[oi]);
            int64_t oe = oi;
            while (oe < n_pairs_run && slots_for(J, P.order[oe]) == ns) ++oe;
            const int64_t ilo = first_of[oi], ihi = std::min(first_of[oe], n_items);
            if (ihi > ilo) {
                Launch L;
                L.ns = ns;
                L.item_lo = ilo;
                L.n = ihi - ilo;
                const int blocks_needed = (int)((L.n + kWavesPerBlock - 1) / kWavesPerBlock);
                L.grid = std::max(1, std::min(blocks_needed, c->n_cu * sh.bpc));
                L.prm = P.prm;
                // segments of about equal estimated cost (queries x train size), one per XCD
                segment_bounds(J, P.order, first_of, sh.qt, oi, oe, ilo, ihi, L.prm.seg);
                const int64_t waves = (int64_t)L.grid * kWavesPerBlock;
                L.prm.grab = (int32_t)std::max<int64_t>(1, std::min<int64_t>(8, L.n / std::max<int64_t>(1, waves * 64)));
                ls.push_back(L);
            }
            oi = oe;
        }
        auto issue = [&]() -> hipError_t {
            for (const Launch& L : ls) {
                hipError_t e = launch_fill_u32(c->stream, counter, kSegments * kCounterStride, 0u);
                if (e == hipSuccess)
                    e = launch_match(c->stream, J.epi, L.ns, L.grid, P.dI, P.dP, items + L.item_lo, (int32_t)L.n,
                                     counter, L.prm, J.o_idx, J.o_d1, J.o_d2, stats);
                if (e != hipSuccess) return e;
            }
            return hipSuccess;
        };
        c->last_replayed = false;
        if (use_graph && c->use_graphs && !ls.empty()) {
            // counter resets + persistent launches as one captured graph,
            // replayed while the launch arguments are unchanged
            std::string key;
            auto put = [&key](const void* v, size_t n) { key.append(static_cast<const char*>(v), n); };
            const int epi = J.epi ? 1 : 0;
            const void* ptrs[] = {P.dI, P.dP, items, counter, J.o_idx, J.o_d1, J.o_d2, stats};
            put(&epi, sizeof epi);
            put(ptrs, sizeof ptrs);
            for (const Launch& L : ls) {
                put(&L.ns, sizeof L.ns);
                put(&L.grid, sizeof L.grid);
                put(&L.item_lo, sizeof L.item_lo);
                put(&L.n, sizeof L.n);
                put(&L.prm, sizeof L.prm);
            }
            hipGraphExec_t exec = nullptr;
            for (auto& g : c->graphs)
                if (g.key == key) {
                    exec = g.exec;
                    g.used = ++c->graph_clock;
                    c->graph_replays++;
                    c->last_replayed = true;
                }
            if (!exec) {
                hipGraph_t graph = nullptr;
                HIPCHK(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
                const hipError_t e1 = issue();
                const hipError_t e2 = hipStreamEndCapture(c->stream, &graph);
                HIPCHK(e1);
                HIPCHK(e2);
                const hipError_t e3 = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
                hipGraphDestroy(graph);
                HIPCHK(e3);
                if (c->graphs.size() >= 4) {
                    auto old = std::min_element(c->graphs.begin(), c->graphs.end(),
                                                [](const auto& a, const auto& b) { return a.used < b.used; });
                    hipGraphExecDestroy(old->exec);
                    c->graphs.erase(old);
                }
                c->graphs.push_back({key, exec, ++c->graph_clock});
            }
            HIPCHK(hipGraphLaunch(exec, c->stream));
        } else {
            HIPCHK(issue());
        }
        *launches += (int64_t)ls.size();
    } else {
        for (int64_t oi = 0; oi < n_pairs_run; ++oi) {
            const int64_t nit = first_of[oi + 1] - first_of[oi];
            if (nit == 0) continue;
            HIPCHK(launch_match(c->stream, J.epi, slots_for(J, P.order[oi]),
                                (int)((nit + kWavesPerBlock - 1) / kWavesPerBlock), P.dI, P.dP, items + first_of[oi],
                                (int32_t)nit, nullptr, P.prm, J.o_idx, J.o_d1, J.o_d2, stats));
            *launches += 1;
        }
    }
    return CASHASH_OK;
}

// Pinned slot of job slot `turn`'s statistics (bucket entries, union,
// ranked), after the first 256 bytes of pin_small.
static unsigned long long* job_stats_host(cashash_ctx* c, int turn) {
    return reinterpret_cast<unsigned long long*>(static_cast<uint8_t*>(c->pin_small.p) + 256 + 64 * turn);
}

// One caller-fixed device region that a match job carves its scratch out of
// (bucket tables, uploaded tables, work items, counters, statistics) instead
// of the context's growable buffers: the allocation-free entry point.
struct ScratchArea {
    uint8_t* base = nullptr;
    size_t cap = 0, used = 0;
    // the host copies of the uploaded tables, kept until the call ends (the
    // uploads read pageable memory)
    std::vector<std::vector<uint8_t>> host;
    uint8_t* take(size_t n) {
        const size_t o = (used + 255) & ~size_t(255);
        if (o > cap || n > cap - o) return nullptr;
        used = o + n;
        return base + o;
    }
};

// Uploads the Uploader's tables into the scratch area on c->stream.
static int upload_scratch(cashash_ctx* c, ScratchArea& sa, Uploader& up, std::vector<const void*>& dptr) {
    uint8_t* dst = sa.take(std::max<size_t>(up.host.size(), 1));
    if (!dst) return fail(CASHASH_E_LIMIT, "the call needs more than the %zu-byte scratch", sa.cap);
    sa.host.push_back(std::move(up.host));
    const std::vector<uint8_t>& h = sa.host.back();
    if (!h.empty()) HIPCHK(hipMemcpyAsync(dst, h.data(), h.size(), hipMemcpyHostToDevice, c->stream));
    dptr.clear();
    for (size_t o : up.offs) dptr.push_back(dst + o);
    return CASHASH_OK;
}

// Enqueues bucket tables and matcher launches for J on c->stream, plus the
// read-back of the statistics into pinned memory; finish_match_job waits.
// With a scratch area (sa) every device buffer of the job is taken from it,
// the launch shape is the cached or default one (no tuning) and no graph is
// captured, so nothing is allocated.
static int launch_match_job(cashash_ctx* c, MatchJob& J, ScratchArea* sa = nullptr) {
    const int n_img = (int)J.imgs.size();
    const int64_t n_pairs = (int64_t)J.pair_q.size();
    // bucket tables for every train image
    std::vector<int32_t> train_list;
    std::vector<char> is_train(n_img, 0);
    for (int64_t p = 0; p < n_pairs; ++p)
        if (!is_train[J.pair_t[p]]) {
            is_train[J.pair_t[p]] = 1;
            train_list.push_back(J.pair_t[p]);
        }
    size_t tbytes = 0;
    std::vector<size_t> toff(n_img, 0), eoff(n_img, 0);
    for (int m : train_list) {
        toff[m] = tbytes;
        tbytes += (size_t)kTables * kOffStride * 4;
        tbytes = (tbytes + 255) & ~size_t(255);
        eoff[m] = tbytes;
        tbytes += ent_bytes(J.imgs[m].n, J.epi);
        tbytes = (tbytes + 255) & ~size_t(255);
    }
    // the band kernel reads whole 64-entry chunks of keypoints from a run's
    // start (lanes past the run are masked): up to 64 entries past the last
    // table's end
    if (J.epi) tbytes += 512;
    // the pair plan (host work): visiting order, launch shapes, per-shape tile
    // tables and the pair table.  Batched: items ordered by train image, so
    // the waves running together share one train image's tables in L2.
    MatchPlan P;
    P.order.resize(n_pairs);
    const bool batched = c->cfg.mode == CASHASH_MODE_BATCHED_BF16X2;
    std::string key;
    std::vector<Shape> cands;
    bool tune = false;
    std::vector<int> qts;
    std::vector<std::vector<PairTiles>> pts;
    std::vector<std::vector<int64_t>> firsts;
    int64_t max_items = 1;
    Uploader up2;  // pairs, then the per-shape tile tables
    auto plan = [&]() {
        double sum_nt = 0, sum_nq = 0;
        for (int64_t p = 0; p < n_pairs; ++p) {
            sum_nt += J.imgs[J.pair_t[p]].n;
            sum_nq += J.imgs[J.pair_q[p]].n;
        }
        if (batched) {
            // stable counting sort by (register-slot group, train image)
            std::vector<int64_t> start((size_t)3 * n_img + 1, 0);
            auto bucket = [&](int64_t p) { return (slots_for(J, p) / 2 - 2) * n_img + J.pair_t[p]; };
            for (int64_t p = 0; p < n_pairs; ++p) start[(size_t)bucket(p) + 1]++;
            for (size_t i = 1; i < start.size(); ++i) start[i] += start[i - 1];
            for (int64_t p = 0; p < n_pairs; ++p) P.order[(size_t)start[(size_t)bucket(p)]++] = p;
        } else {
            std::iota(P.order.begin(), P.order.end(), 0);
        }
        // launch shapes: cached, tuned now, or the default
        tune_cache_load(c);
        key = tune_key(batched, J.epi, c->cfg.k, n_pairs ? sum_nt / n_pairs : 0.0, n_pairs ? sum_nq / n_pairs : 0.0);
        auto hit = c->tuned.find(key);
        tune = !sa && hit == c->tuned.end() && autotune_enabled() && n_pairs > 0;
        if (hit != c->tuned.end())
            cands.push_back(
                Shape{std::max(1, std::min({hit->second.qt, kMaxTile, sel_cap(J.epi) / c->cfg.k})), hit->second.bpc});
        else if (tune)
            cands = shape_candidates(c->cfg.k, batched, J.epi);
        else
            cands.push_back(default_shape(c->cfg.k, batched, J.epi));
        for (const Shape& sh : cands)
            if (std::find(qts.begin(), qts.end(), sh.qt) == qts.end()) qts.push_back(sh.qt);
        firsts.resize(qts.size());
        for (size_t i = 0; i < qts.size(); ++i) pts.push_back(pair_tiles(J, P.order, qts[i], &firsts[i]));
        for (auto& f : firsts) max_items = std::max(max_items, f[n_pairs]);
        P.items_cap = max_items;
        std::vector<PairDev> pd(n_pairs);
        for (int64_t p = 0; p < n_pairs; ++p) {
            pd[p].qi = J.pair_q[p];
            pd[p].ti = J.pair_t[p];
            pd[p].out = J.pair_out[p];
            for (int i = 0; i < 9; ++i) pd[p].F[i] = J.epi ? J.F[9 * p + i] : 0.0;
        }
        up2.add(pd);
        for (auto& t : pts) up2.add(t);
    };
    auto upload = [&](Uploader& up, std::vector<const void*>& d) {
        return sa ? upload_scratch(c, *sa, up, d) : upload_meta(c, up, d, kMetaMatch);
    };
    // the bucket tables (device work): placed, their image and table views
    // uploaded, the bucket kernel launched
    std::vector<const void*> d;
    auto tables = [&]() -> int {
        uint8_t* tbase = nullptr;
        if (sa) {
            tbase = sa->take(std::max<size_t>(tbytes, 1));
        } else {
            RETCHK(c->tables.ensure(tbytes));
            tbase = c->tables.as<uint8_t>();
        }
        std::vector<TableOut> touts(n_img, TableOut{nullptr, nullptr});
        for (int m : train_list) {
            touts[m] = TableOut{reinterpret_cast<uint32_t*>(tbase + toff[m]), tbase + eoff[m]};
            J.imgs[m].off = touts[m].off;
            J.imgs[m].ent = touts[m].ent;
        }
        Uploader up1;  // image views, table outputs, train list
        up1.add(J.imgs);
        up1.add(touts);
        up1.add(train_list);
        RETCHK(upload(up1, d));
        P.dI = (const ImgDev*)d[0];
        HIPCHK(launch_bucket(c->stream, J.epi, P.dI, (const TableOut*)d[1], (const int32_t*)d[2],
                             (int)train_list.size()));
        return CASHASH_OK;
    };
    if (sa) {
        // the whole call must fit the scratch before any device work starts
        plan();
        const size_t up1_bytes = ((((size_t)n_img * sizeof(ImgDev) + 255) & ~size_t(255)) +
                                  (((size_t)n_img * sizeof(TableOut) + 255) & ~size_t(255)) +
                                  train_list.size() * sizeof(int32_t));
        ScratchArea probe;
        probe.base = sa->base;
        probe.cap = sa->cap;
        probe.used = sa->used;
        const size_t pieces[] = {std::max<size_t>(tbytes, 1), std::max<size_t>(up1_bytes, 1),
                                 std::max<size_t>(up2.host.size(), 1), (size_t)max_items * sizeof(Item),
                                 (size_t)kSegments * kCounterStride * 4, 64};
        size_t need = 0;
        for (size_t n : pieces) need = ((need + 255) & ~size_t(255)) + n;
        for (size_t n : pieces)
            if (!probe.take(n))
                return fail(CASHASH_E_LIMIT, "the call needs %zu bytes of scratch, more than its %zu bytes", need,
                            sa->cap);
        RETCHK(tables());
    } else {
        // the bucket tables are built while the host plans the pairs
        RETCHK(tables());
        plan();
    }
    RETCHK(upload(up2, d));
    P.dP = (const PairDev*)d[0];
    P.prm.k = c->cfg.k;
    P.prm.tau = c->cfg.max_hamming;
    P.prm.num2 = (int64_t)c->cfg.ratio_num * c->cfg.ratio_num;
    P.prm.den2 = (int64_t)c->cfg.ratio_den * c->cfg.ratio_den;
    P.prm.max_px = J.max_px;
    // work items (the most any candidate shape needs), counters, statistics
    unsigned long long* stats = nullptr;
    if (sa) {
        P.items = reinterpret_cast<Item*>(sa->take((size_t)max_items * sizeof(Item)));
        P.counter = reinterpret_cast<uint32_t*>(sa->take((size_t)kSegments * kCounterStride * 4));
        stats = reinterpret_cast<unsigned long long*>(sa->take(64));
    } else {
        RETCHK(c->items.ensure((size_t)max_items * sizeof(Item)));
        P.items = c->items.as<Item>();
        P.counter = c->counters.as<uint32_t>();
        stats = c->dCount.as<unsigned long long>() + 8;
    }

    Shape best = cands[0];
    if (tune && cands.size() > 1) {
        // time every candidate shape on a prefix of the pairs (outputs are
        // identical for every shape; the full run rewrites them)
        const int64_t sample_pairs = batched ? std::max<int64_t>(1, std::min<int64_t>(n_pairs, n_pairs / 4 + 8))
                                             : std::min<int64_t>(n_pairs, 12);
        // the first round warms up; each shape keeps its fastest later time
        std::vector<float> shape_ms(cands.size(), 1e30f);
        for (int rep = 0; rep < 3; ++rep)
            for (size_t ci = 0; ci < cands.size(); ++ci) {
                const Shape& sh = cands[ci];
                const size_t qi = (size_t)(std::find(qts.begin(), qts.end(), sh.qt) - qts.begin());
                const int64_t n_it = firsts[qi][sample_pairs];
                RETCHK(make_items(c, P, sh.qt, (const PairTiles*)d[1 + qi], (int32_t)pts[qi].size(),
                                  firsts[qi][n_pairs]));
                int64_t dummy_launches = 0;
                HIPCHK(hipEventRecord(c->ev0, c->stream));
                RETCHK(enqueue_matcher(c, P, J, sh, batched, firsts[qi], sample_pairs, n_it, stats, &dummy_launches,
                                       false));
                HIPCHK(hipEventRecord(c->ev1, c->stream));
                HIPCHK(hipEventSynchronize(c->ev1));
                float ms = 0.f;
                HIPCHK(hipEventElapsedTime(&ms, c->ev0, c->ev1));
                if (rep > 0) shape_ms[ci] = std::min(shape_ms[ci], ms);
            }
        best = cands[(size_t)(std::min_element(shape_ms.begin(), shape_ms.end()) - shape_ms.begin())];
        c->tuned[key] = best;
        tune_cache_store(c, key, best);
    } else if (tune) {
        c->tuned[key] = best;
    }
    const size_t qi = (size_t)(std::find(qts.begin(), qts.end(), best.qt) - qts.begin());
    const int64_t n_items = firsts[qi][n_pairs];
    RETCHK(make_items(c, P, best.qt, (const PairTiles*)d[1 + qi], (int32_t)pts[qi].size(), n_items));
    HIPCHK(launch_fill_u64(c->stream, stats, 3, 0ull));
    J.turn = c->job_turn;
    c->job_turn ^= 1;
    HIPCHK(hipEventRecord(c->job_ev[J.turn][0], c->stream));
    RETCHK(enqueue_matcher(c, P, J, best, batched, firsts[qi], n_pairs, n_items, stats, &c->last_launches,
                           sa == nullptr));
    HIPCHK(hipEventRecord(c->job_ev[J.turn][1], c->stream));
    c->last_shape_qt = best.qt;
    c->last_shape_bpc = best.bpc;
    HIPCHK(hipMemcpyAsync(job_stats_host(c, J.turn), stats, 24, hipMemcpyDeviceToHost, c->stream));
    return CASHASH_OK;
}

static void tune_cache_load(cashash_ctx* c) {
    if (c->tune_loaded) return;
    c->tune_loaded = true;
    const char* path = std::getenv("CASHASH_AUTOTUNE_CACHE");
    if (!path || !path[0]) return;
    FILE* f = std::fopen(path, "r");
    if (!f) return;
    char line[512];
    while (std::fgets(line, sizeof line, f)) {
        char key[256];
        int qt = 0, bpc = 0;
        if (std::sscanf(line, " {\"key\": \"%255[^\"]\", \"qt\": %d, \"bpc\": %d}", key, &qt, &bpc) == 3 && qt > 0)
            c->tuned[key] = Shape{qt, bpc};
    }
    std::fclose(f);
}

static void tune_cache_store(cashash_ctx* c, const std::string& key, Shape sh) {
    (void)c;
    const char* path = std::getenv("CASHASH_AUTOTUNE_CACHE");
    if (!path || !path[0]) return;
    FILE* f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "{\"key\": \"%s\", \"qt\": %d, \"bpc\": %d}\n", key.c_str(), sh.qt, sh.bpc);
    std::fclose(f);
}

// Waits for job J (the whole stream, or only up to the job's done event,
// recorded by the host-memory path after its output download) and takes its
// statistics and kernel time.
static int finish_match_job(cashash_ctx* c, MatchJob& J, bool whole_stream = true) {
    if (whole_stream)
        HIPCHK(hipStreamSynchronize(c->stream));
    else
        HIPCHK(hipEventSynchronize(c->job_ev[J.turn][2]));
    const unsigned long long* st = job_stats_host(c, J.turn);
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, c->job_ev[J.turn][0], c->job_ev[J.turn][1]));
    c->last_ms += ms;
    J.bucket_entries += (int64_t)st[0];
    J.union_size += (int64_t)st[1];
    J.ranked += (int64_t)st[2];
    return CASHASH_OK;
}

// ------------------------------------------------------------------ host-memory mode

// Chunked upload of caller host memory through two pinned buffers on the copy
// stream: the CPU fills one buffer while the other is in flight.
// One array of a block upload: `bytes` from host `src` to offset `off` of the
// block's device range.
struct UpPiece {
    size_t off;
    const void* src;
    size_t bytes;
};

// Uploads a block's arrays (pieces in ascending, non-overlapping offsets) into
// the device range at dst.  The span from the first piece to the end of the
// last is staged through the two pinned buffers in windows of 16 MiB: the host
// threads pack a window from the pieces it overlaps, one copy on the copy
// stream sends it, and the next window is packed into the other buffer while
// it travels.  Bytes of the span between pieces (alignment padding, or areas
// that kernels write later) carry whatever the buffer held.  A block of many
// small images so costs a few large copies, not one copy and one wait per
// array.
static int h2d_block(cashash_ctx* c, uint8_t* dst, const std::vector<UpPiece>& pieces, int64_t* h2d) {
    if (pieces.empty()) return CASHASH_OK;
    const size_t chunk = (size_t)16 << 20, grain = (size_t)1 << 20;
    RETCHK(c->pin[0].ensure(chunk));
    RETCHK(c->pin[1].ensure(chunk));
    const size_t lo = pieces.front().off, hi = pieces.back().off + pieces.back().bytes;
    struct Seg {
        size_t at;
        const uint8_t* src;
        size_t n;
    };
    std::vector<Seg> segs;
    size_t pi = 0;
    for (size_t w0 = lo; w0 < hi; w0 += chunk) {
        const size_t w1 = std::min(hi, w0 + chunk);
        const int b = c->pin_turn;
        c->pin_turn ^= 1;
        HIPCHK(hipEventSynchronize(c->pin_ev[b]));
        segs.clear();
        while (pi < pieces.size() && pieces[pi].off + pieces[pi].bytes <= w0) ++pi;
        for (size_t k = pi; k < pieces.size() && pieces[k].off < w1; ++k) {
            const size_t a = std::max(pieces[k].off, w0), e = std::min(pieces[k].off + pieces[k].bytes, w1);
            for (size_t g = a; g < e; g += grain)
                segs.push_back(Seg{g - w0, static_cast<const uint8_t*>(pieces[k].src) + (g - pieces[k].off),
                                   std::min(grain, e - g)});
        }
        uint8_t* pb = static_cast<uint8_t*>(c->pin[b].p);
        c->pool->run((int64_t)segs.size(), [&](int64_t i) { std::memcpy(pb + segs[i].at, segs[i].src, segs[i].n); });
        HIPCHK(hipMemcpyAsync(dst + w0, pb, w1 - w0, hipMemcpyHostToDevice, c->copy_stream));
        HIPCHK(hipEventRecord(c->pin_ev[b], c->copy_stream));
    }
    for (const UpPiece& p : pieces) *h2d += (int64_t)p.bytes;
    return CASHASH_OK;
}

static int64_t default_budget(cashash_ctx* c) {
    if (c->cfg.device_budget_bytes > 0) return c->cfg.device_budget_bytes;
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) return (int64_t)1 << 30;
    return (int64_t)(fr / 4);
}

// Resident layout of one image inside a slot.
struct SlotImage {
    size_t desc, codes, keys, kp, end;
};
static SlotImage slot_layout(int n, bool with_codes, bool with_kp) {
    SlotImage L;
    L.desc = 0;
    L.codes = al256((size_t)n * kDim);
    L.keys = L.codes + (with_codes ? al256((size_t)n * 16) : 0);
    L.kp = L.keys + (with_codes ? al256((size_t)n * 6) : 0);
    L.end = L.kp + (with_kp ? al256((size_t)n * 8) : 0);
    return L;
}

// Codes: pass 1 streams every block for the column sums, pass 2 streams the
// blocks again (last block first, so the one still resident is reused) to
// project them.  Two slots: one in use, one being filled.
// Passes of the host-mode code builder.  Both (the default) clears the sums,
// sums every block, sets the bias and projects.  kPassSums alone adds these
// images' column sums to c->dS; kPassCodes alone projects them with the bias
// already set for a whole set of n_tot_set descriptors (the disk level runs
// the two over groups of a larger set).
enum { kPassSums = 1, kPassCodes = 2 };

static int build_codes_host(cashash_ctx* c, const cashash_images* im, uint64_t* const* codes_out,
                            uint8_t* const* keys_out, int64_t* near_count, cashash_stats* stats,
                            int passes = kPassSums | kPassCodes, double n_tot_set = 0.0) {
    const bool both = passes == (kPassSums | kPassCodes);
    const int M = im->n_images;
    double n_tot = 0;
    std::vector<int64_t> bytes(M);
    for (int m = 0; m < M; ++m) {
        const int n = im->n_feat[m];
        if (n > 0 && (!im->desc[m] || ((passes & kPassCodes) && (!codes_out[m] || !keys_out[m]))))
            return fail(CASHASH_E_INVAL, "image %d: null descriptor or output pointer", m);
        bytes[m] = (int64_t)al256((size_t)n * kDim);  // descriptors only: codes go to an output area
        n_tot += n;
    }
    *near_count = 0;
    if (n_tot == 0) return CASHASH_OK;
    const int64_t budget = default_budget(c);
    const int64_t slot = budget / 2;
    // blocks of consecutive images
    std::vector<int> first{0};
    int64_t fill = 0;
    for (int m = 0; m < M; ++m) {
        if (bytes[m] > slot)
            return fail(CASHASH_E_NOMEM, "image %d needs %lld device bytes; budget %lld allows %lld per block", m,
                        (long long)bytes[m], (long long)budget, (long long)slot);
        if (fill + bytes[m] > slot && fill > 0) {
            first.push_back(m);
            fill = 0;
        }
        fill += bytes[m];
    }
    first.push_back(M);
    const int nb = (int)first.size() - 1;
    RETCHK(c->stage.ensure((size_t)slot * 2));
    int64_t h2d = 0, d2h = 0, loads = 0;
    int resident[2] = {-1, -1};
    std::vector<size_t> place(M, 0);
    auto load = [&](int b, int s) -> int {
        if (resident[s] == b) return CASHASH_OK;
        HIPCHK(hipStreamWaitEvent(c->copy_stream, c->slot_free_ev[s], 0));
        std::vector<UpPiece> pieces;
        size_t off = 0;
        for (int m = first[b]; m < first[b + 1]; ++m) {
            place[m] = (size_t)s * slot + off;
            if (im->n_feat[m] > 0) pieces.push_back(UpPiece{off, im->desc[m], (size_t)im->n_feat[m] * kDim});
            off += (size_t)bytes[m];
            loads++;
        }
        RETCHK(h2d_block(c, c->stage.as<uint8_t>() + (size_t)s * slot, pieces, &h2d));
        HIPCHK(hipEventRecord(c->slot_load_ev[s], c->copy_stream));
        resident[s] = b;
        return CASHASH_OK;
    };
    // image views of block b; with out, the codes and keys of its images go to
    // one device output area (image i's codes at pos[i], its keys right after)
    // that comes back with a single copy
    std::vector<size_t> pos;
    auto views = [&](int b, std::vector<ImgDev>& iv, std::vector<CodeOut>* ov, uint8_t* out) {
        iv.clear();
        if (ov) ov->clear();
        pos.assign(1, 0);
        for (int m = first[b]; m < first[b + 1]; ++m) {
            const int n = im->n_feat[m];
            iv.push_back(ImgDev{c->stage.as<uint8_t>() + place[m], nullptr, nullptr, nullptr, nullptr, nullptr, n, 0});
            const size_t at = pos.back();
            if (ov) ov->push_back(CodeOut{reinterpret_cast<uint64_t*>(out + at), out + at + (size_t)n * 16, 0});
            pos.push_back(at + (((size_t)n * 22 + 15) & ~size_t(15)));  // codes stay 16-byte aligned
        }
    };
    std::vector<ImgDev> iv;
    std::vector<CodeOut> ov;
    if (both) {
        HIPCHK(launch_fill_u64(c->stream, c->dS.as<unsigned long long>(), kDim, 0ull));
        HIPCHK(launch_fill_u64(c->stream, c->dCount.as<unsigned long long>(), 8, 0ull));
    }
    if (passes & kPassSums) {
        for (int b = 0; b < nb; ++b) {
            const int s = b & 1;
            RETCHK(load(b, s));
            HIPCHK(hipStreamWaitEvent(c->stream, c->slot_load_ev[s], 0));
            views(b, iv, nullptr, nullptr);
            RETCHK(run_colsum(c, iv));
            HIPCHK(hipEventRecord(c->slot_free_ev[s], c->stream));
            if (b + 1 < nb) RETCHK(load(b + 1, (b + 1) & 1));  // prefetch while the sums run
        }
    }
    if (both)
        HIPCHK(launch_bias(c->stream, c->dR64.as<double>(), c->dS.as<unsigned long long>(), n_tot,
                           c->dBias.as<float>()));
    for (int b = nb - 1; (passes & kPassCodes) && b >= 0; --b) {
        int s = resident[0] == b ? 0 : resident[1] == b ? 1 : (b & 1);
        RETCHK(load(b, s));
        HIPCHK(hipStreamWaitEvent(c->stream, c->slot_load_ev[s], 0));
        size_t out_bytes = 0;
        for (int m = first[b]; m < first[b + 1]; ++m) out_bytes += (((size_t)im->n_feat[m] * 22 + 15) & ~size_t(15));
        RETCHK(c->outbuf[0].ensure(std::max<size_t>(out_bytes, 16)));
        RETCHK(c->pin_out[0].ensure(std::max<size_t>(out_bytes, 16)));
        views(b, iv, &ov, c->outbuf[0].as<uint8_t>());
        RETCHK(run_project(c, iv, ov, both ? n_tot : n_tot_set));
        HIPCHK(hipEventRecord(c->slot_free_ev[s], c->stream));
        HIPCHK(hipMemcpyAsync(c->pin_out[0].p, c->outbuf[0].p, out_bytes, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        const uint8_t* ho = static_cast<const uint8_t*>(c->pin_out[0].p);
        c->pool->run(first[b + 1] - first[b], [&](int64_t i) {
            const int m = first[b] + (int)i;
            const size_t n = (size_t)im->n_feat[m];
            if (!n) return;
            std::memcpy(codes_out[m], ho + pos[i], n * 16);
            std::memcpy(keys_out[m], ho + pos[i] + n * 16, n * 6);
        });
        for (int m = first[b]; m < first[b + 1]; ++m) d2h += (int64_t)im->n_feat[m] * 22;
    }
    unsigned long long cnt = 0;
    HIPCHK(hipStreamSynchronize(c->stream));
    HIPCHK(hipMemcpy(&cnt, c->dCount.p, 8, hipMemcpyDeviceToHost));
    *near_count = (int64_t)cnt;
    if (stats) {
        stats->h2d_bytes += h2d;
        stats->d2h_bytes += d2h;
        stats->image_loads += loads;
    }
    return CASHASH_OK;
}

// Matching: the block scheduler's steps run one after another; each step's
// missing blocks are loaded into free slots of three, the next step's new
// block is prefetched while the current step computes, and each step's
// outputs come back through pinned memory.
// Host-memory matching runs a scheduler step's pairs in parts (12 output
// bytes per query), so that a part's download and copy-out overlap the next
// part's kernels.  A part costs a launch and the bucket tables of its train
// images, so steps before the last use parts of up to 2^25 queries: their
// tails overlap the next step's parts.  The last step's tail is exposed, so
// it uses parts of a fifth of its queries, between 2^23 and 2^24.
constexpr int64_t kPartQueries = (int64_t)1 << 25;
constexpr int64_t kLastPartMin = (int64_t)1 << 23, kLastPartMax = (int64_t)1 << 24;

// CASHASH_PART_QUERIES, if set (1 .. 2^27), fixes the part size of every
// step (small inputs then run as many parts, as tests do); 0 otherwise.
static int64_t part_queries_env() {
    const char* e = std::getenv("CASHASH_PART_QUERIES");
    if (e && e[0]) {
        const long long v = std::atoll(e);
        if (v >= 1 && v <= ((int64_t)1 << 27)) return (int64_t)v;
    }
    return 0;
}

static int match_host(cashash_ctx* c, const cashash_images* im, const uint64_t* const* codes,
                      const uint8_t* const* keys, const float* const* kp, MatchJob& J, int32_t* o_idx,
                      int32_t* o_d1, int32_t* o_d2, cashash_stats* stats) {
    const int M = im->n_images;
    const int64_t n_pairs = (int64_t)J.pair_q.size();
    std::vector<int64_t> bytes(M), data_bytes(M);
    for (int m = 0; m < M; ++m) {
        const int n = im->n_feat[m];
        data_bytes[m] = (int64_t)slot_layout(n, true, J.epi).end;
        bytes[m] = data_bytes[m] + (int64_t)(al256((size_t)kTables * kOffStride * 4) +
                                             al256(ent_bytes(n, J.epi)));
    }
    // three image slots plus bucket tables for up to two blocks
    const int64_t budget = default_budget(c);
    const int64_t slot = budget / 5;
    std::vector<int32_t> pv((size_t)2 * n_pairs);
    for (int64_t p = 0; p < n_pairs; ++p) {
        pv[2 * p] = J.pair_q[p];
        pv[2 * p + 1] = J.pair_t[p];
    }
    Schedule S;
    const int pr = plan_schedule(M, bytes.data(), n_pairs, pv.data(), slot, S);
    if (pr == -1)
        return fail(CASHASH_E_NOMEM, "an image does not fit the device budget (%lld bytes per block of %lld)",
                    (long long)slot, (long long)budget);
    if (pr) return fail(CASHASH_E_INVAL, "scheduler rejected the pair list");
    RETCHK(c->stage.ensure((size_t)slot * 3));
    int slot_block[3] = {-1, -1, -1};
    int64_t slot_used_at[3] = {-1, -1, -1};
    std::vector<size_t> place(M, 0);
    int64_t h2d = 0, d2h = 0, loads = 0;
    auto load_block = [&](int b, int s) -> int {
        HIPCHK(hipStreamWaitEvent(c->copy_stream, c->slot_free_ev[s], 0));
        std::vector<UpPiece> pieces;
        size_t off = 0;
        for (int i = S.block_first[b]; i < S.block_first[b + 1]; ++i) {
            const int m = S.block_images[i];
            const size_t n = (size_t)im->n_feat[m];
            const SlotImage L = slot_layout((int)n, true, J.epi);
            place[m] = (size_t)s * slot + off;
            if (n) {
                pieces.push_back(UpPiece{off + L.desc, im->desc[m], n * kDim});
                pieces.push_back(UpPiece{off + L.codes, codes[m], n * 16});
                pieces.push_back(UpPiece{off + L.keys, keys[m], n * 6});
                if (J.epi) pieces.push_back(UpPiece{off + L.kp, kp[m], n * 8});
            }
            off += (size_t)data_bytes[m];
            loads++;
        }
        RETCHK(h2d_block(c, c->stage.as<uint8_t>() + (size_t)s * slot, pieces, &h2d));
        HIPCHK(hipEventRecord(c->slot_load_ev[s], c->copy_stream));
        slot_block[s] = b;
        return CASHASH_OK;
    };
    // a slot for block b that holds neither of the protected blocks, least recently used first
    auto pick_slot = [&](int p0, int p1) {
        int best = -1;
        for (int s = 0; s < 3; ++s) {
            if (slot_block[s] == p0 || slot_block[s] == p1) continue;
            if (best < 0 || slot_used_at[s] < slot_used_at[best]) best = s;
        }
        return best;
    };
    auto slot_of = [&](int b) {
        for (int s = 0; s < 3; ++s)
            if (slot_block[s] == b) return s;
        return -1;
    };
    c->last_ms = 0.0;
    const int64_t part_env = part_queries_env();
    // a step whose kernels and download are queued; its outputs are copied
    // into the caller's arrays (over the host threads) once the next step is
    // queued behind it
    struct Pending {
        bool valid = false;
        MatchJob job;
        std::vector<int64_t> pairs;  // its pairs (indices into the call's pair list)
        int64_t nq = 0;
    } pending;
    auto drain = [&](Pending& pd) -> int {
        pd.valid = false;
        MatchJob& Jp = pd.job;
        RETCHK(finish_match_job(c, Jp, false));
        const int32_t* ho = reinterpret_cast<const int32_t*>(c->pin_out[Jp.turn].p);
        const int64_t nqp = pd.nq;
        c->pool->run((int64_t)Jp.pair_q.size(), [&](int64_t i) {
            const int64_t p = pd.pairs[i];
            const int64_t n = im->n_feat[J.pair_q[p]];
            if (!n) return;
            std::memcpy(o_idx + J.pair_out[p], ho + Jp.pair_out[i], (size_t)n * 4);
            std::memcpy(o_d1 + J.pair_out[p], ho + nqp + Jp.pair_out[i], (size_t)n * 4);
            std::memcpy(o_d2 + J.pair_out[p], ho + 2 * nqp + Jp.pair_out[i], (size_t)n * 4);
        });
        d2h += nqp * 12;
        J.bucket_entries += Jp.bucket_entries;
        J.union_size += Jp.union_size;
        J.ranked += Jp.ranked;
        return CASHASH_OK;
    };
    for (size_t st = 0; st < S.steps.size(); ++st) {
        const SchedStep& step = S.steps[st];
        for (int b : {step.bi, step.bk}) {
            if (slot_of(b) >= 0) continue;
            const int s = pick_slot(step.bi, step.bk);
            RETCHK(load_block(b, s));
        }
        const int si = slot_of(step.bi), sk = slot_of(step.bk);
        HIPCHK(hipStreamWaitEvent(c->stream, c->slot_load_ev[si], 0));
        HIPCHK(hipStreamWaitEvent(c->stream, c->slot_load_ev[sk], 0));
        slot_used_at[si] = slot_used_at[sk] = (int64_t)st;
        std::vector<ImgDev> views(M, ImgDev{nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, 0, 0});
        for (int b : {step.bi, step.bk})
            for (int i = S.block_first[b]; i < S.block_first[b + 1]; ++i) {
                const int m = S.block_images[i];
                const int n = im->n_feat[m];
                const SlotImage L = slot_layout(n, true, J.epi);
                uint8_t* base = c->stage.as<uint8_t>() + place[m];
                views[m] = ImgDev{base + L.desc, reinterpret_cast<const uint64_t*>(base + L.codes), base + L.keys,
                                  J.epi ? reinterpret_cast<const float*>(base + L.kp) : nullptr, nullptr, nullptr, n,
                                  0};
            }
        // the step's pairs, grouped by register-slot group (a part of one
        // group is one persistent launch, not up to three) and then by train
        // image (each part builds the bucket tables of its own train images),
        // in parts (sized as above), so that a part's download and copy-out
        // overlap the next part's kernels
        std::vector<int64_t> ord(S.order.begin() + step.pair_begin, S.order.begin() + step.pair_end);
        auto group = [&](int64_t p) {
            const int n = im->n_feat[J.pair_t[p]];
            return J.epi || n <= kLargeTrain ? 0 : n <= kHugeTrain ? 1 : 2;
        };
        std::stable_sort(ord.begin(), ord.end(), [&](int64_t x, int64_t y) {
            const int gx = group(x), gy = group(y);
            return gx != gy ? gx < gy : J.pair_t[x] < J.pair_t[y];
        });
        int64_t part_max = part_env;
        if (!part_max) {
            int64_t step_q = 0;
            for (int64_t p : ord) step_q += im->n_feat[J.pair_q[p]];
            part_max = st + 1 < S.steps.size() ? kPartQueries
                                                : std::min(kLastPartMax, std::max(kLastPartMin, step_q / 5));
        }
        for (size_t pb = 0; pb < ord.size();) {
            size_t pe = pb;
            int64_t nq = 0;
            while (pe < ord.size() && (pe == pb || nq + im->n_feat[J.pair_q[ord[pe]]] <= part_max))
                nq += im->n_feat[J.pair_q[ord[pe++]]];
            MatchJob Js;
            Js.epi = J.epi;
            Js.max_px = J.max_px;
            Js.imgs = views;
            std::vector<double> Fs;
            int64_t q_at = 0;
            for (size_t i = pb; i < pe; ++i) {
                const int64_t p = ord[i];
                Js.pair_q.push_back(J.pair_q[p]);
                Js.pair_t.push_back(J.pair_t[p]);
                Js.pair_out.push_back(q_at);
                q_at += im->n_feat[J.pair_q[p]];
                if (J.epi) Fs.insert(Fs.end(), J.F + 9 * p, J.F + 9 * p + 9);
            }
            Js.F = J.epi ? Fs.data() : nullptr;
            const int turn = c->job_turn;  // the slot launch_match_job takes
            RETCHK(c->outbuf[turn].ensure((size_t)std::max<int64_t>(nq, 1) * 12));
            Js.o_idx = c->outbuf[turn].as<int32_t>();
            Js.o_d1 = Js.o_idx + nq;
            Js.o_d2 = Js.o_d1 + nq;
            RETCHK(c->pin_out[turn].ensure((size_t)std::max<int64_t>(nq, 1) * 12));
            RETCHK(launch_match_job(c, Js));
            HIPCHK(hipEventRecord(c->slot_free_ev[si], c->stream));
            HIPCHK(hipEventRecord(c->slot_free_ev[sk], c->stream));
            // the download runs on its own stream once the part's kernels
            // (and its statistics copy) are done, while the next part's
            // kernels run.  Both buffers of this turn are free: the host
            // drained the part that last used them before this part was
            // queued (drain waits for that part's download)
            HIPCHK(hipEventRecord(c->part_ev[Js.turn], c->stream));
            HIPCHK(hipStreamWaitEvent(c->d2h_stream, c->part_ev[Js.turn], 0));
            if (nq)
                HIPCHK(hipMemcpyAsync(c->pin_out[Js.turn].p, c->outbuf[Js.turn].p, (size_t)nq * 12,
                                      hipMemcpyDeviceToHost, c->d2h_stream));
            HIPCHK(hipEventRecord(c->job_ev[Js.turn][2], c->d2h_stream));
            // prefetch the next step's new block while this one computes
            if (pb == 0 && st + 1 < S.steps.size()) {
                const SchedStep& nx = S.steps[st + 1];
                for (int b : {nx.bi, nx.bk}) {
                    if (slot_of(b) >= 0) continue;
                    const int s = pick_slot(step.bi, step.bk);
                    if (s < 0) break;
                    RETCHK(load_block(b, s));
                    break;  // one block ahead
                }
            }
            // the previous part's results go to the caller while this one computes
            if (pending.valid) RETCHK(drain(pending));
            pending.valid = true;
            pending.job = std::move(Js);
            pending.job.F = nullptr;  // Fs ends with this part; the job's pair table holds F already
            pending.pairs.assign(ord.begin() + pb, ord.begin() + pe);
            pending.nq = nq;
            pb = pe;
        }
    }
    if (pending.valid) RETCHK(drain(pending));
    if (stats) {
        stats->h2d_bytes = h2d;
        stats->d2h_bytes = d2h;
        stats->image_loads = loads;
    }
    return CASHASH_OK;
}

// Exposed for tests of the host logic: plan the block schedule and report its
// shape.  steps_out (may be NULL) receives up to max_steps rows of
// (bi, bk, first pair position, end pair position); order_out (may be NULL)
// receives the n_pairs pair indices in visiting order.
extern "C" int cashash_plan_schedule(int32_t n_images, const int64_t* img_bytes, int64_t n_pairs,
                                     const int32_t* pairs, int64_t slot_bytes, int64_t* n_steps, int64_t* n_blocks,
                                     int64_t* block_loads, int64_t* image_loads, int64_t* steps_out,
                                     int64_t max_steps, int64_t* order_out) {
    if (!img_bytes || (n_pairs > 0 && !pairs) || !n_steps || !n_blocks || !block_loads || !image_loads)
        return fail(CASHASH_E_INVAL, "null argument");
    Schedule S;
    const int r = plan_schedule(n_images, img_bytes, n_pairs, pairs, slot_bytes, S);
    if (r == -1) return fail(CASHASH_E_NOMEM, "an image exceeds the slot size");
    if (r) return fail(CASHASH_E_INVAL, "bad schedule input");
    *n_steps = (int64_t)S.steps.size();
    *n_blocks = (int64_t)S.block_first.size() - 1;
    *block_loads = S.block_loads;
    *image_loads = S.image_loads;
    if (steps_out)
        for (int64_t i = 0; i < std::min<int64_t>(max_steps, (int64_t)S.steps.size()); ++i) {
            steps_out[4 * i] = S.steps[i].bi;
            steps_out[4 * i + 1] = S.steps[i].bk;
            steps_out[4 * i + 2] = S.steps[i].pair_begin;
            steps_out[4 * i + 3] = S.steps[i].pair_end;
        }
    if (order_out) std::copy(S.order.begin(), S.order.end(), order_out);
    return CASHASH_OK;
}

// ------------------------------------------------------------------ public entry points
static void zero_stats(cashash_stats* s) {
    if (s) std::memset(s, 0, sizeof *s);
}

extern "C" int cashash_build_codes(cashash_ctx* c, const cashash_images* im, uint64_t* const* codes_out,
                                   uint8_t* const* keys_out, cashash_stats* stats) {
    if (!c) return fail(CASHASH_E_INVAL, "null context");
    RETCHK(check_images(im));
    if (im->n_images > 0 && (!codes_out || !keys_out)) return fail(CASHASH_E_INVAL, "null output arrays");
    zero_stats(stats);
    RETCHK(follow_caller(c));
    const double t0 = now_ms();
    int64_t near_count = 0;
    if (c->cfg.mem == CASHASH_MEM_DEVICE) {
        RETCHK(build_codes_device(c, im, codes_out, keys_out, &near_count));
    } else {
        RETCHK(build_codes_host(c, im, codes_out, keys_out, &near_count, stats));
    }
    if (stats) {
        stats->near_margin_recomputes = near_count;
        stats->ms_codes = now_ms() - t0;
    }
    return CASHASH_OK;
}

// out_offsets (device mode only): first output slot of each pair; null =
// pairs packed one after another in list order.
static int match_common(cashash_ctx* c, const cashash_images* im, const uint64_t* const* codes,
                        const uint8_t* const* keys, const float* const* kp, int64_t n_pairs, const int32_t* pairs,
                        const double* F, double max_px, bool epi, int32_t* o_idx, int32_t* o_d1, int32_t* o_d2,
                        cashash_stats* stats, const int64_t* out_offsets = nullptr,
                        ScratchArea* sa = nullptr) {
    if (!c) return fail(CASHASH_E_INVAL, "null context");
    RETCHK(check_images(im));
    if (n_pairs < 0) return fail(CASHASH_E_INVAL, "negative n_pairs");
    zero_stats(stats);
    if (n_pairs == 0) return CASHASH_OK;
    if (!pairs || !codes || !keys) return fail(CASHASH_E_INVAL, "null pairs, codes or keys");
    if (epi) {
        if (!kp || !F) return fail(CASHASH_E_INVAL, "null keypoints or F");
        if (!(max_px >= 0.0) || !std::isfinite(max_px)) return fail(CASHASH_E_INVAL, "max_px must be finite and >= 0");
        for (int64_t i = 0; i < 9 * n_pairs; ++i)
            if (!std::isfinite(F[i])) return fail(CASHASH_E_INVAL, "F of pair %lld is not finite", (long long)(i / 9));
    }
    RETCHK(follow_caller(c));
    const double t0 = now_ms();
    MatchJob J;
    J.epi = epi;
    J.max_px = max_px;
    J.F = F;
    J.pair_q.resize(n_pairs);
    J.pair_t.resize(n_pairs);
    J.pair_out.resize(n_pairs);
    int64_t total_q = 0;
    std::vector<char> used(im->n_images, 0);
    for (int64_t p = 0; p < n_pairs; ++p) {
        const int32_t q = pairs[2 * p], t = pairs[2 * p + 1];
        if (q < 0 || t < 0 || q >= im->n_images || t >= im->n_images)
            return fail(CASHASH_E_INVAL, "pair %lld = (%d, %d) out of range", (long long)p, q, t);
        J.pair_q[p] = q;
        J.pair_t[p] = t;
        J.pair_out[p] = out_offsets ? out_offsets[p] : total_q;
        total_q += im->n_feat[q];
        used[q] = used[t] = 1;
    }
    for (int m = 0; m < im->n_images; ++m) {
        if (!used[m] || im->n_feat[m] == 0) continue;
        if (!im->desc[m] || !codes[m] || !keys[m] || (epi && !kp[m]))
            return fail(CASHASH_E_INVAL, "image %d: null descriptor, code, key or keypoint pointer", m);
        if (misaligned(im->desc[m], 16) || misaligned(codes[m], 8) || misaligned(keys[m], 2) ||
            (epi && misaligned(kp[m], 4)))
            return fail(CASHASH_E_INVAL, "image %d: misaligned buffer", m);
    }
    if (total_q > 0 && (!o_idx || !o_d1 || !o_d2)) return fail(CASHASH_E_INVAL, "null output arrays");
    c->last_launches = 0;
    c->last_replayed = false;
    if (out_offsets && c->cfg.mem != CASHASH_MEM_DEVICE)
        return fail(CASHASH_E_INVAL, "explicit output offsets need device memory");
    if (c->cfg.mem == CASHASH_MEM_DEVICE) {
        if (misaligned(o_idx, 4) || misaligned(o_d1, 4) || misaligned(o_d2, 4))
            return fail(CASHASH_E_INVAL, "misaligned output arrays");
        J.imgs.resize(im->n_images);
        for (int m = 0; m < im->n_images; ++m)
            J.imgs[m] = ImgDev{im->desc[m], codes[m], keys[m], epi ? kp[m] : nullptr, nullptr, nullptr,
                               im->n_feat[m], 0};
        J.o_idx = o_idx;
        J.o_d1 = o_d1;
        J.o_d2 = o_d2;
        c->last_ms = 0.0;
        RETCHK(launch_match_job(c, J, sa));
        RETCHK(finish_match_job(c, J));
    } else {
        RETCHK(match_host(c, im, codes, keys, kp, J, o_idx, o_d1, o_d2, stats));
    }
    if (stats) {
        stats->pairs = n_pairs;
        stats->queries = total_q;
        stats->bucket_entries = J.bucket_entries;
        stats->union_size = J.union_size;
        stats->ranked = J.ranked;
        stats->tile_queries = c->last_shape_qt;
        stats->blocks_per_cu = c->last_shape_bpc;
        stats->graph_replayed = c->last_replayed ? 1 : 0;
        stats->ms_match = now_ms() - t0;
    }
    return CASHASH_OK;
}

extern "C" int cashash_match_pairs(cashash_ctx* c, const cashash_images* im, const uint64_t* const* codes,
                                   const uint8_t* const* keys, int64_t n_pairs, const int32_t* pairs,
                                   int32_t* match_idx, int32_t* d1sq, int32_t* d2sq, cashash_stats* stats) {
    return match_common(c, im, codes, keys, nullptr, n_pairs, pairs, nullptr, 0.0, false, match_idx, d1sq, d2sq,
                        stats);
}

extern "C" int cashash_match_pairs_noalloc(cashash_ctx* c, const cashash_images* im, const uint64_t* const* codes,
                                           const uint8_t* const* keys, int64_t n_pairs, const int32_t* pairs,
                                           int32_t* match_idx, int32_t* d1sq, int32_t* d2sq, cashash_stats* stats) {
    if (!c) return fail(CASHASH_E_INVAL, "null context");
    if (c->cfg.mem != CASHASH_MEM_DEVICE)
        return fail(CASHASH_E_INVAL, "cashash_match_pairs_noalloc needs cfg.mem = CASHASH_MEM_DEVICE");
    if (!c->scratch) return fail(CASHASH_E_DEVICE, "no scratch on device %d: %s", c->device, c->scratch_err.c_str());
    ScratchArea sa;
    sa.base = c->scratch;
    sa.cap = (size_t)CASHASH_NOALLOC_SCRATCH_BYTES;
    return match_common(c, im, codes, keys, nullptr, n_pairs, pairs, nullptr, 0.0, false, match_idx, d1sq, d2sq,
                        stats, nullptr, &sa);
}

extern "C" int cashash_match_pairs_epipolar(cashash_ctx* c, const cashash_images* im, const uint64_t* const* codes,
                                            const uint8_t* const* keys, const float* const* kp_xy, int64_t n_pairs,
                                            const int32_t* pairs, const double* F, double max_px, int32_t* match_idx,
                                            int32_t* d1sq, int32_t* d2sq, cashash_stats* stats) {
    return match_common(c, im, codes, keys, kp_xy, n_pairs, pairs, F, max_px, true, match_idx, d1sq, d2sq, stats);
}

// ------------------------------------------------------------------ geometry-aware first stage (Sec. 3.1)
extern "C" int64_t cashash_subset_size(int32_t n, int32_t frac_num, int32_t frac_den) {
    if (n < 0 || frac_num <= 0 || frac_den <= 0 || frac_num > frac_den) return -1;
    return ((int64_t)n * frac_num + frac_den - 1) / frac_den;
}

extern "C" void cashash_default_geometric_config(cashash_geometric_config* g) {
    if (!g) return;
    g->frac_num = 1;
    g->frac_den = 5;
    g->min_matches = 16;
    g->n_hyp = 256;
    g->ransac_px = 2.0;
    g->band_px = 4.0;
    g->rand8 = nullptr;
}

static int need_device(cashash_ctx* c, const char* what) {
    if (c->cfg.mem != CASHASH_MEM_DEVICE)
        return fail(CASHASH_E_INVAL, "%s needs device-resident inputs (cfg.mem = CASHASH_MEM_DEVICE)", what);
    return CASHASH_OK;
}

static int check_counts(int32_t n_images, const int32_t* n_feat) {
    if (n_images < 0 || (n_images > 0 && !n_feat)) return fail(CASHASH_E_INVAL, "invalid image counts");
    for (int m = 0; m < n_images; ++m) {
        if (n_feat[m] < 0) return fail(CASHASH_E_INVAL, "image %d: negative n_feat", m);
        if (n_feat[m] > CASHASH_MAX_FEAT) return fail(CASHASH_E_LIMIT, "image %d: n_feat > %d", m, CASHASH_MAX_FEAT);
    }
    return CASHASH_OK;
}

// Top-scale rows of every image into rows_out[m] (device).
static int run_select(cashash_ctx* c, int32_t n_images, const float* const* scales, const int32_t* n_feat,
                      int32_t num, int32_t den, int32_t* const* rows_out) {
    std::vector<SelectImg> v(n_images);
    for (int m = 0; m < n_images; ++m) {
        const int64_t mm = cashash_subset_size(n_feat[m], num, den);
        if (mm > 0 && (!scales[m] || !rows_out[m]))
            return fail(CASHASH_E_INVAL, "image %d: null scale or row pointer", m);
        if (misaligned(scales[m], 4) || misaligned(rows_out[m], 4))
            return fail(CASHASH_E_INVAL, "image %d: misaligned scale or row buffer", m);
        v[m] = SelectImg{scales[m], rows_out[m], n_feat[m], (int32_t)mm};
    }
    if (n_images == 0) return CASHASH_OK;
    Uploader up;
    up.add(v);
    std::vector<const void*> d;
    RETCHK(upload_meta(c, up, d, kMetaGeo));
    HIPCHK(launch_top_scale(c->stream, (const SelectImg*)d[0], n_images));
    return CASHASH_OK;
}

extern "C" int cashash_select_top_scale(cashash_ctx* c, int32_t n_images, const float* const* scales,
                                        const int32_t* n_feat, int32_t frac_num, int32_t frac_den,
                                        int32_t* const* rows_out) {
    if (!c) return fail(CASHASH_E_INVAL, "null context");
    RETCHK(need_device(c, "cashash_select_top_scale"));
    RETCHK(check_counts(n_images, n_feat));
    if (cashash_subset_size(0, frac_num, frac_den) < 0) return fail(CASHASH_E_INVAL, "need 0 < frac_num <= frac_den");
    if (n_images > 0 && (!scales || !rows_out)) return fail(CASHASH_E_INVAL, "null scale or row arrays");
    RETCHK(follow_caller(c));
    RETCHK(run_select(c, n_images, scales, n_feat, frac_num, frac_den, rows_out));
    HIPCHK(hipStreamSynchronize(c->stream));
    return CASHASH_OK;
}

// Gather of rows; row errors are OR-ed into c->geo_err (not cleared here).
static int run_gather(cashash_ctx* c, const std::vector<GatherImg>& g) {
    std::vector<RowChunk> chunks;
    for (int m = 0; m < (int)g.size(); ++m)
        for (int r0 = 0; r0 < g[m].m; r0 += 32) chunks.push_back({m, r0, std::min(32, g[m].m - r0), 0});
    if (chunks.empty()) return CASHASH_OK;
    Uploader up;
    up.add(g);
    up.add(chunks);
    std::vector<const void*> d;
    RETCHK(upload_meta(c, up, d, kMetaGeo));
    HIPCHK(launch_gather_rows(c->stream, (const GatherImg*)d[0], (const RowChunk*)d[1], (int)chunks.size(),
                              c->geo_err.as<unsigned>()));
    return CASHASH_OK;
}

static int read_geo_err(cashash_ctx* c) {
    unsigned e = 0;
    HIPCHK(hipMemcpyAsync(c->pin_small.p, c->geo_err.p, 4, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    std::memcpy(&e, c->pin_small.p, 4);
    if (e & 1u) return fail(CASHASH_E_INVAL, "a row index is outside its image");
    if (e & 2u) return fail(CASHASH_E_INVAL, "a match index is outside its train image");
    if (e & 4u) return fail(CASHASH_E_LIMIT, "a pair has more matches than the LDS list holds");
    return CASHASH_OK;
}

static int clear_geo_err(cashash_ctx* c) {
    RETCHK(c->geo_err.ensure(256));
    HIPCHK(launch_fill_u32(c->stream, c->geo_err.as<uint32_t>(), 1, 0u));
    return CASHASH_OK;
}

extern "C" int cashash_gather_rows(cashash_ctx* c, int32_t n_images, const int32_t* n_feat, const int32_t* n_rows,
                                   const int32_t* const* rows, const uint8_t* const* desc,
                                   const uint64_t* const* codes, const uint8_t* const* keys, const float* const* kp,
                                   uint8_t* const* desc_out, uint64_t* const* codes_out, uint8_t* const* keys_out,
                                   float* const* kp_out) {
    if (!c) return fail(CASHASH_E_INVAL, "null context");
    RETCHK(need_device(c, "cashash_gather_rows"));
    RETCHK(check_counts(n_images, n_feat));
    if (n_images > 0 && (!n_rows || !rows)) return fail(CASHASH_E_INVAL, "null row arrays");
    if (!desc != !desc_out || !codes != !codes_out || !keys != !keys_out || !kp != !kp_out)
        return fail(CASHASH_E_INVAL, "each field needs both its input and its output array, or neither");
    std::vector<GatherImg> g(n_images);
    for (int m = 0; m < n_images; ++m) {
        if (n_rows[m] < 0 || n_rows[m] > CASHASH_MAX_FEAT) return fail(CASHASH_E_INVAL, "image %d: bad n_rows", m);
        GatherImg& x = g[m];
        x = GatherImg{desc ? desc[m] : nullptr, codes ? codes[m] : nullptr, keys ? keys[m] : nullptr,
                      kp ? kp[m] : nullptr, rows[m], desc_out ? desc_out[m] : nullptr,
                      codes_out ? codes_out[m] : nullptr, keys_out ? keys_out[m] : nullptr,
                      kp_out ? kp_out[m] : nullptr, n_feat[m], n_rows[m]};
        if (x.m == 0) continue;
        if (!x.rows || (desc && (!x.desc || !x.o_desc)) || (codes && (!x.codes || !x.o_codes)) ||
            (keys && (!x.keys || !x.o_keys)) || (kp && (!x.kp || !x.o_kp)))
            return fail(CASHASH_E_INVAL, "image %d: null buffer", m);
        if (misaligned(x.rows, 4) || misaligned(x.desc, 16) || misaligned(x.o_desc, 16) || misaligned(x.codes, 8) ||
            misaligned(x.o_codes, 8) || misaligned(x.keys, 2) || misaligned(x.o_keys, 2) || misaligned(x.kp, 4) ||
            misaligned(x.o_kp, 4))
            return fail(CASHASH_E_INVAL, "image %d: misaligned buffer", m);
    }
    RETCHK(follow_caller(c));
    RETCHK(clear_geo_err(c));
    RETCHK(run_gather(c, g));
    return read_geo_err(c);
}

// Fundamental matrices of `pairs` from the stage-1 outputs `match_idx` (flat,
// pair p at out[p]) over images of n_feat points with keypoints kp.  Per-pair
// results go to c->geo_pair: F [P][9] doubles, then n_matches, n_inliers,
// best_h, status (int32 [P] each).
static int run_fundamental(cashash_ctx* c, int32_t n_images, const int32_t* n_feat, const float* const* kp,
                           int64_t n_pairs, const int32_t* pairs, const std::vector<int64_t>& out,
                           const int32_t* match_idx, const uint32_t* rand8, int32_t n_hyp, double thr,
                           int32_t min_matches) {
    std::vector<GeoImg> gi(n_images);
    for (int m = 0; m < n_images; ++m) gi[m] = GeoImg{kp ? kp[m] : nullptr, n_feat[m], 0};
    std::vector<GeoPair> gp(n_pairs);
    int cap = 8;
    std::vector<char> used(n_images, 0);
    for (int64_t p = 0; p < n_pairs; ++p) {
        const int32_t q = pairs[2 * p], t = pairs[2 * p + 1];
        gp[p] = GeoPair{q, t, out[p]};
        cap = std::max(cap, n_feat[q]);
        used[q] = used[t] = 1;
    }
    for (int m = 0; m < n_images; ++m)
        if (used[m] && n_feat[m] > 0 && (!gi[m].kp || misaligned(gi[m].kp, 4)))
            return fail(CASHASH_E_INVAL, "image %d: null or misaligned keypoints", m);
    if (cap > kGeoMaxMatches)
        return fail(CASHASH_E_LIMIT, "a query image has %d points; at most %d per image here", cap, kGeoMaxMatches);
    const size_t P = (size_t)n_pairs;
    RETCHK(c->geo_pair.ensure(P * 9 * 8 + 4 * P * 4 + 256));
    GeoOut go;
    go.F = c->geo_pair.as<double>();
    go.n_matches = reinterpret_cast<int32_t*>(go.F + 9 * P);
    go.n_inliers = go.n_matches + P;
    go.best_h = go.n_inliers + P;
    go.status = go.best_h + P;
    std::vector<uint32_t> rv(rand8, rand8 + 8 * (size_t)n_hyp);
    Uploader up;
    up.add(gi);
    up.add(gp);
    up.add(rv);
    std::vector<const void*> d;
    RETCHK(upload_meta(c, up, d, kMetaGeo));
    GeoParams prm{n_hyp, min_matches, thr, cap, 0};
    HIPCHK(launch_fundamental(c->stream, (const GeoImg*)d[0], (const GeoPair*)d[1], n_pairs, match_idx,
                              (const uint32_t*)d[2], prm, go, c->geo_err.as<unsigned>()));
    return CASHASH_OK;
}

static int check_geo_args(int32_t n_hyp, const uint32_t* rand8, double thr, int32_t min_matches) {
    if (n_hyp < 1 || n_hyp > (1 << 20)) return fail(CASHASH_E_INVAL, "n_hyp must be in 1..2^20");
    if (!rand8) return fail(CASHASH_E_INVAL, "null random draws");
    if (!(thr >= 0.0) || !std::isfinite(thr)) return fail(CASHASH_E_INVAL, "inlier threshold must be finite and >= 0");
    if (min_matches < 0) return fail(CASHASH_E_INVAL, "min_matches must be >= 0");
    return CASHASH_OK;
}

static int copy_pair_results(cashash_ctx* c, int64_t n_pairs, double* F_out, int32_t* n_matches, int32_t* n_inliers,
                             int32_t* best_hyp, int32_t* status) {
    const size_t P = (size_t)n_pairs;
    const double* F = c->geo_pair.as<double>();
    const int32_t* nm = reinterpret_cast<const int32_t*>(F + 9 * P);
    struct Piece {
        void* dst;
        const void* src;
        size_t bytes;
    };
    for (const Piece& pc : {Piece{F_out, F, P * 72}, Piece{n_matches, nm, P * 4}, Piece{n_inliers, nm + P, P * 4},
                            Piece{best_hyp, nm + 2 * P, P * 4}, Piece{status, nm + 3 * P, P * 4}})
        if (pc.dst) HIPCHK(hipMemcpyAsync(pc.dst, pc.src, pc.bytes, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return CASHASH_OK;
}

static int check_pairs(int32_t n_images, int64_t n_pairs, const int32_t* pairs) {
    if (n_pairs < 0) return fail(CASHASH_E_INVAL, "negative n_pairs");
    if (n_pairs > 0 && !pairs) return fail(CASHASH_E_INVAL, "null pairs");
    if (n_pairs > INT32_MAX) return fail(CASHASH_E_LIMIT, "too many pairs");
    for (int64_t p = 0; p < n_pairs; ++p) {
        const int32_t q = pairs[2 * p], t = pairs[2 * p + 1];
        if (q < 0 || t < 0 || q >= n_images || t >= n_images)
            return fail(CASHASH_E_INVAL, "pair %lld = (%d, %d) out of range", (long long)p, q, t);
    }
    return CASHASH_OK;
}

extern "C" int cashash_estimate_fundamental(cashash_ctx* c, int32_t n_images, const int32_t* n_feat,
                                            const float* const* kp_xy, int64_t n_pairs, const int32_t* pairs,
                                            const int32_t* match_idx, const uint32_t* rand8, int32_t n_hyp,
                                            double thr_px, int32_t min_matches, double* F_out, int32_t* n_matches,
                                            int32_t* n_inliers, int32_t* best_hyp, int32_t* status) {
    if (!c) return fail(CASHASH_E_INVAL, "null context");
    RETCHK(need_device(c, "cashash_estimate_fundamental"));
    RETCHK(check_counts(n_images, n_feat));
    RETCHK(check_pairs(n_images, n_pairs, pairs));
    RETCHK(check_geo_args(n_hyp, rand8, thr_px, min_matches));
    if (n_pairs == 0) return CASHASH_OK;
    if (!kp_xy || !F_out || !n_matches || !n_inliers || !status) return fail(CASHASH_E_INVAL, "null argument");
    std::vector<int64_t> out(n_pairs);
    int64_t total = 0;
    for (int64_t p = 0; p < n_pairs; ++p) {
        out[p] = total;
        total += n_feat[pairs[2 * p]];
    }
    if (total > 0 && (!match_idx || misaligned(match_idx, 4)))
        return fail(CASHASH_E_INVAL, "null or misaligned match_idx");
    RETCHK(follow_caller(c));
    RETCHK(clear_geo_err(c));
    RETCHK(run_fundamental(c, n_images, n_feat, kp_xy, n_pairs, pairs, out, match_idx, rand8, n_hyp, thr_px,
                           min_matches));
    RETCHK(read_geo_err(c));
    return copy_pair_results(c, n_pairs, F_out, n_matches, n_inliers, best_hyp, status);
}

extern "C" int cashash_match_pairs_geometric(cashash_ctx* c, const cashash_images* im, const uint64_t* const* codes,
                                             const uint8_t* const* keys, const float* const* kp_xy,
                                             const float* const* scales, int64_t n_pairs, const int32_t* pairs,
                                             const cashash_geometric_config* g, double* F_out, int32_t* n_matches,
                                             int32_t* n_inliers, int32_t* status, int32_t* match_idx, int32_t* d1sq,
                                             int32_t* d2sq, cashash_stats* stats) {
    if (!c) return fail(CASHASH_E_INVAL, "null context");
    RETCHK(need_device(c, "cashash_match_pairs_geometric"));
    RETCHK(check_images(im));
    zero_stats(stats);
    if (!g) return fail(CASHASH_E_INVAL, "null geometric config");
    if (cashash_subset_size(0, g->frac_num, g->frac_den) < 0)
        return fail(CASHASH_E_INVAL, "need 0 < frac_num <= frac_den");
    RETCHK(check_geo_args(g->n_hyp, g->rand8, g->ransac_px, g->min_matches));
    if (!(g->band_px >= 0.0) || !std::isfinite(g->band_px)) return fail(CASHASH_E_INVAL, "band_px must be finite and >= 0");
    RETCHK(check_pairs(im->n_images, n_pairs, pairs));
    if (n_pairs == 0) return CASHASH_OK;
    if (!codes || !keys || !kp_xy || !scales || !F_out || !n_matches || !n_inliers || !status)
        return fail(CASHASH_E_INVAL, "null argument");
    RETCHK(follow_caller(c));
    const double t0 = now_ms();
    const int n_img = im->n_images;
    std::vector<char> used(n_img, 0);
    for (int64_t p = 0; p < n_pairs; ++p) used[pairs[2 * p]] = used[pairs[2 * p + 1]] = 1;
    // subset sizes and one device block for the subset images
    std::vector<int32_t> ms(n_img, 0);
    std::vector<size_t> o_rows(n_img), o_desc(n_img), o_codes(n_img), o_keys(n_img), o_kp(n_img);
    size_t bytes = 0;
    auto take = [&](size_t n) {
        const size_t o = bytes;
        bytes += al256(n);
        return o;
    };
    for (int m = 0; m < n_img; ++m) {
        if (!used[m] || im->n_feat[m] == 0) continue;
        if (!scales[m] || !kp_xy[m] || !codes[m] || !keys[m] || !im->desc[m])
            return fail(CASHASH_E_INVAL, "image %d: null input buffer", m);
        ms[m] = (int32_t)cashash_subset_size(im->n_feat[m], g->frac_num, g->frac_den);
        o_rows[m] = take((size_t)ms[m] * 4);
        o_desc[m] = take((size_t)ms[m] * kDim);
        o_codes[m] = take((size_t)ms[m] * 16);
        o_keys[m] = take((size_t)ms[m] * kTables);
        o_kp[m] = take((size_t)ms[m] * 8);
    }
    RETCHK(c->geo_sub.ensure(bytes));
    uint8_t* base = c->geo_sub.as<uint8_t>();
    std::vector<int32_t*> rows(n_img, nullptr);
    std::vector<uint8_t*> sdesc(n_img, nullptr), skeys(n_img, nullptr);
    std::vector<uint64_t*> scodes(n_img, nullptr);
    std::vector<float*> skp(n_img, nullptr);
    std::vector<GatherImg> gat(n_img);
    for (int m = 0; m < n_img; ++m) {
        if (ms[m] > 0) {
            rows[m] = reinterpret_cast<int32_t*>(base + o_rows[m]);
            sdesc[m] = base + o_desc[m];
            scodes[m] = reinterpret_cast<uint64_t*>(base + o_codes[m]);
            skeys[m] = base + o_keys[m];
            skp[m] = reinterpret_cast<float*>(base + o_kp[m]);
        }
        gat[m] = GatherImg{im->desc[m], codes[m], keys[m], kp_xy[m], rows[m], sdesc[m], scodes[m], skeys[m], skp[m],
                           im->n_feat[m], ms[m]};
    }
    std::vector<int64_t> out1(n_pairs), out2(n_pairs);
    int64_t total1 = 0, total2 = 0;
    for (int64_t p = 0; p < n_pairs; ++p) {
        out1[p] = total1;
        out2[p] = total2;
        total1 += ms[pairs[2 * p]];
        total2 += im->n_feat[pairs[2 * p]];
    }
    if (total2 > 0 && (!match_idx || !d1sq || !d2sq)) return fail(CASHASH_E_INVAL, "null output arrays");
    RETCHK(c->geo_m1.ensure((size_t)std::max<int64_t>(total1, 1) * 12));
    int32_t* m1 = c->geo_m1.as<int32_t>();
    const size_t T1 = (size_t)std::max<int64_t>(total1, 1);

    // subset selection and gather
    HIPCHK(hipEventRecord(c->geo_ev[0], c->stream));
    RETCHK(clear_geo_err(c));
    std::vector<int32_t> n_sel(n_img);
    for (int m = 0; m < n_img; ++m) n_sel[m] = ms[m] > 0 ? im->n_feat[m] : 0;
    RETCHK(run_select(c, n_img, scales, n_sel.data(), g->frac_num, g->frac_den, rows.data()));
    RETCHK(run_gather(c, gat));
    HIPCHK(hipEventRecord(c->geo_ev[1], c->stream));
    // stage 1: CasHash matching of the subsets
    cashash_images sub{n_img, const_cast<const uint8_t* const*>(sdesc.data()), ms.data()};
    cashash_stats st1;
    RETCHK(match_common(c, &sub, const_cast<const uint64_t* const*>(scodes.data()),
                        const_cast<const uint8_t* const*>(skeys.data()), nullptr, n_pairs, pairs, nullptr, 0.0, false,
                        m1, m1 + T1, m1 + 2 * T1, &st1));
    HIPCHK(hipEventRecord(c->geo_ev[2], c->stream));
    // fundamental matrices from the stage-1 matches
    RETCHK(run_fundamental(c, n_img, ms.data(), const_cast<const float* const*>(skp.data()), n_pairs, pairs, out1, m1,
                           g->rand8, g->n_hyp, g->ransac_px, g->min_matches));
    HIPCHK(hipEventRecord(c->geo_ev[3], c->stream));
    RETCHK(read_geo_err(c));
    RETCHK(copy_pair_results(c, n_pairs, F_out, n_matches, n_inliers, nullptr, status));
    // stage 2: guided matching of the accepted pairs; the others get -1
    std::vector<int32_t> acc_pairs;
    std::vector<double> acc_F;
    std::vector<int64_t> acc_out;
    for (int64_t p = 0; p < n_pairs; ++p) {
        if (status[p] != 0) continue;
        acc_pairs.push_back(pairs[2 * p]);
        acc_pairs.push_back(pairs[2 * p + 1]);
        acc_F.insert(acc_F.end(), F_out + 9 * p, F_out + 9 * p + 9);
        acc_out.push_back(out2[p]);
    }
    if (total2 > 0) {
        HIPCHK(launch_fill_u32(c->stream, reinterpret_cast<uint32_t*>(match_idx), total2, 0xFFFFFFFFu));
        HIPCHK(launch_fill_u32(c->stream, reinterpret_cast<uint32_t*>(d1sq), total2, 0xFFFFFFFFu));
        HIPCHK(launch_fill_u32(c->stream, reinterpret_cast<uint32_t*>(d2sq), total2, 0xFFFFFFFFu));
    }
    cashash_stats st2;
    zero_stats(&st2);
    const int64_t n_acc = (int64_t)acc_out.size();
    if (n_acc > 0)
        RETCHK(match_common(c, im, codes, keys, kp_xy, n_acc, acc_pairs.data(), acc_F.data(), g->band_px, true,
                            match_idx, d1sq, d2sq, &st2, acc_out.data()));
    HIPCHK(hipEventRecord(c->geo_ev[4], c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    for (int i = 0; i < 4; ++i) {
        float ms_ = 0.f;
        HIPCHK(hipEventElapsedTime(&ms_, c->geo_ev[i], c->geo_ev[i + 1]));
        c->geo_ms[i] = ms_;
    }
    if (stats) {
        *stats = st2;
        stats->pairs = n_pairs;
        stats->queries = total2;
        stats->ms_match = now_ms() - t0;
    }
    return CASHASH_OK;
}

extern "C" int cashash_last_geometric_ms(cashash_ctx* c, double* ms4) {
    if (!c || !ms4) return fail(CASHASH_E_INVAL, "null argument");
    for (int i = 0; i < 4; ++i) ms4[i] = c->geo_ms[i];
    return CASHASH_OK;
}

// ------------------------------------------------------------------ disk level ("Three-Level Data Scheduling Strategy")
// The whole set lives on disk; groups of images are read into host memory by
// a second thread while the current group (pair) is processed, and each
// group (pair) is handed to the host-memory path, which streams blocks to
// the device.  File layouts (little-endian, headers padded to 64 bytes):
//   set    "CASHSET1", n_images, flags (bit 0: keypoints), feature prefix
//          sums [n_images + 1], then at a 64-byte boundary the descriptors
//          uint8 [N][128] and, if flagged, keypoints float32 [N][2]
//   codes  "CASHCOD1", n_images, N; at 64: codes uint64 [N][2], keys uint8 [N][6]
//   output "CASHOUT1", n_pairs, total queries T; at 64: match_idx, d1sq, d2sq int32 [T] each
//   progress "CASHPRG1", plan hash, n_steps; at 64: one byte per group pair (1 = written)
namespace {

const char kSetMagic[8] = {'C', 'A', 'S', 'H', 'S', 'E', 'T', '1'};
const char kCodMagic[8] = {'C', 'A', 'S', 'H', 'C', 'O', 'D', '1'};
const char kOutMagic[8] = {'C', 'A', 'S', 'H', 'O', 'U', 'T', '1'};
const char kPrgMagic[8] = {'C', 'A', 'S', 'H', 'P', 'R', 'G', '1'};
constexpr int64_t kFileHeader = 64;

struct Fd {
    int fd = -1;
    Fd() = default;
    Fd(const Fd&) = delete;
    Fd& operator=(const Fd&) = delete;
    ~Fd() {
        if (fd >= 0) ::close(fd);
    }
};

bool read_at(int fd, void* buf, size_t n, int64_t off) {
    uint8_t* p = static_cast<uint8_t*>(buf);
    while (n > 0) {
        const ssize_t r = ::pread(fd, p, n, (off_t)off);
        if (r <= 0) return false;
        p += r;
        n -= (size_t)r;
        off += r;
    }
    return true;
}

bool write_at(int fd, const void* buf, size_t n, int64_t off) {
    const uint8_t* p = static_cast<const uint8_t*>(buf);
    while (n > 0) {
        const ssize_t r = ::pwrite(fd, p, n, (off_t)off);
        if (r <= 0) return false;
        p += r;
        n -= (size_t)r;
        off += r;
    }
    return true;
}

int64_t al64(int64_t n) { return (n + 63) & ~int64_t(63); }

struct SetFile {
    Fd f;
    int32_t n_images = 0;
    int64_t flags = 0;
    std::vector<int64_t> offs;  // feature prefix sums
    int64_t desc_off = 0;
    std::vector<int32_t> n_feat;
};

int open_set(const char* path, SetFile& s) {
    if (!path) return fail(CASHASH_E_INVAL, "null set path");
    s.f.fd = ::open(path, O_RDONLY);
    if (s.f.fd < 0) return fail(CASHASH_E_IO, "cannot open set file %s", path);
    char magic[8];
    int64_t hdr[2];
    if (!read_at(s.f.fd, magic, 8, 0) || std::memcmp(magic, kSetMagic, 8) != 0 || !read_at(s.f.fd, hdr, 16, 8))
        return fail(CASHASH_E_IO, "%s is not a set file", path);
    if (hdr[0] < 0 || hdr[0] > INT32_MAX) return fail(CASHASH_E_IO, "%s: bad image count", path);
    s.n_images = (int32_t)hdr[0];
    s.flags = hdr[1];
    s.offs.resize((size_t)s.n_images + 1);
    if (!read_at(s.f.fd, s.offs.data(), s.offs.size() * 8, 24)) return fail(CASHASH_E_IO, "%s: short header", path);
    s.n_feat.resize(s.n_images);
    if (s.offs[0] != 0) return fail(CASHASH_E_IO, "%s: bad offsets", path);
    for (int m = 0; m < s.n_images; ++m) {
        const int64_t n = s.offs[m + 1] - s.offs[m];
        if (n < 0 || n > CASHASH_MAX_FEAT) return fail(CASHASH_E_IO, "%s: image %d has a bad feature count", path, m);
        s.n_feat[m] = (int32_t)n;
    }
    s.desc_off = al64(24 + 8 * ((int64_t)s.n_images + 1));
    struct stat st;
    if (::fstat(s.f.fd, &st) != 0 || st.st_size < s.desc_off + s.offs.back() * kDim)
        return fail(CASHASH_E_IO, "%s is shorter than its header says", path);
    return CASHASH_OK;
}

uint64_t fnv1a(uint64_t h, const void* p, size_t n) {
    const uint8_t* b = static_cast<const uint8_t*>(p);
    for (size_t i = 0; i < n; ++i) {
        h ^= b[i];
        h *= 1099511628211ull;
    }
    return h;
}

}  // namespace

extern "C" int cashash_set_write(const char* path, const cashash_images* im, const float* const* kp_xy) {
    RETCHK(check_images(im));
    if (!path) return fail(CASHASH_E_INVAL, "null path");
    const int M = im->n_images;
    std::vector<int64_t> offs((size_t)M + 1, 0);
    for (int m = 0; m < M; ++m) {
        if (im->n_feat[m] > 0 && (!im->desc[m] || (kp_xy && !kp_xy[m])))
            return fail(CASHASH_E_INVAL, "image %d: null buffer", m);
        offs[m + 1] = offs[m] + im->n_feat[m];
    }
    Fd f;
    f.fd = ::open(path, O_WRONLY | O_CREAT | O_TRUNC, 0644);
    if (f.fd < 0) return fail(CASHASH_E_IO, "cannot create %s", path);
    const int64_t hdr[2] = {(int64_t)M, kp_xy ? 1 : 0};
    const int64_t desc_off = al64(24 + 8 * ((int64_t)M + 1));
    bool ok = write_at(f.fd, kSetMagic, 8, 0) && write_at(f.fd, hdr, 16, 8) &&
              write_at(f.fd, offs.data(), offs.size() * 8, 24);
    const int64_t N = offs.back();
    for (int m = 0; ok && m < M; ++m)
        if (im->n_feat[m] > 0)
            ok = write_at(f.fd, im->desc[m], (size_t)im->n_feat[m] * kDim, desc_off + offs[m] * kDim);
    for (int m = 0; ok && kp_xy && m < M; ++m)
        if (im->n_feat[m] > 0)
            ok = write_at(f.fd, kp_xy[m], (size_t)im->n_feat[m] * 8, desc_off + N * kDim + offs[m] * 8);
    if (ok && N == 0) ok = ::ftruncate(f.fd, (off_t)desc_off) == 0;
    if (!ok) return fail(CASHASH_E_IO, "write to %s failed", path);
    return CASHASH_OK;
}

extern "C" int cashash_build_codes_disk(cashash_ctx* c, const char* set_path, const char* codes_path,
                                        int64_t host_budget_bytes, cashash_stats* stats) {
    if (!c) return fail(CASHASH_E_INVAL, "null context");
    if (c->cfg.mem != CASHASH_MEM_HOST) return fail(CASHASH_E_INVAL, "the disk level needs cfg.mem = CASHASH_MEM_HOST");
    if (!codes_path) return fail(CASHASH_E_INVAL, "null codes path");
    if (host_budget_bytes <= 0) return fail(CASHASH_E_INVAL, "host_budget_bytes must be > 0");
    zero_stats(stats);
    const double t0 = now_ms();
    SetFile S;
    RETCHK(open_set(set_path, S));
    const int M = S.n_images;
    const int64_t N = S.offs.back();
    // groups: consecutive images, two resident (current + prefetched)
    const int64_t slot = host_budget_bytes / 2;
    std::vector<int> first{0};
    int64_t fill = 0;
    for (int m = 0; m < M; ++m) {
        const int64_t b = (int64_t)S.n_feat[m] * kDim;
        if (b > slot) return fail(CASHASH_E_NOMEM, "image %d does not fit a host group of %lld bytes", m, (long long)slot);
        if (fill + b > slot && fill > 0) {
            first.push_back(m);
            fill = 0;
        }
        fill += b;
    }
    first.push_back(M);
    const int ng = (int)first.size() - 1;
    std::vector<uint8_t> buf[2];
    buf[0].resize((size_t)std::max<int64_t>(slot, 1));
    buf[1].resize((size_t)std::max<int64_t>(slot, 1));
    int64_t disk = 0, group_loads = 0;
    auto read_group = [&](int g, int s) -> bool {
        const int64_t r0 = S.offs[first[g]], r1 = S.offs[first[g + 1]];
        return read_at(S.f.fd, buf[s].data(), (size_t)(r1 - r0) * kDim, S.desc_off + r0 * kDim);
    };
    auto view = [&](int g, int s, std::vector<const uint8_t*>& dp, std::vector<int32_t>& nf) {
        dp.clear();
        nf.clear();
        const int64_t r0 = S.offs[first[g]];
        for (int m = first[g]; m < first[g + 1]; ++m) {
            dp.push_back(buf[s].data() + (S.offs[m] - r0) * kDim);
            nf.push_back(S.n_feat[m]);
        }
    };
    Fd out;
    out.fd = ::open(codes_path, O_RDWR | O_CREAT | O_TRUNC, 0644);
    if (out.fd < 0) return fail(CASHASH_E_IO, "cannot create %s", codes_path);
    const int64_t hdr[2] = {(int64_t)M, N};
    if (!write_at(out.fd, kCodMagic, 8, 0) || !write_at(out.fd, hdr, 16, 8) ||
        ::ftruncate(out.fd, (off_t)(kFileHeader + N * 22)) != 0)
        return fail(CASHASH_E_IO, "write to %s failed", codes_path);
    HIPCHK(launch_fill_u64(c->stream, c->dS.as<unsigned long long>(), kDim, 0ull));
    HIPCHK(launch_fill_u64(c->stream, c->dCount.as<unsigned long long>(), 8, 0ull));
    int64_t near = 0;
    for (int pass = 0; pass < 2; ++pass) {
        // first line: the group in progress; second line: the next group read ahead
        if (ng > 0 && !read_group(0, 0)) return fail(CASHASH_E_IO, "read of %s failed", set_path);
        group_loads += ng > 0;
        for (int g = 0; g < ng; ++g) {
            const int s = g & 1;
            std::future<bool> ahead;
            if (g + 1 < ng) ahead = std::async(std::launch::async, read_group, g + 1, s ^ 1);
            std::vector<const uint8_t*> dp;
            std::vector<int32_t> nf;
            view(g, s, dp, nf);
            cashash_images gi{(int32_t)nf.size(), dp.data(), nf.data()};
            int rc;
            if (pass == 0) {
                rc = build_codes_host(c, &gi, nullptr, nullptr, &near, stats, kPassSums);
            } else {
                const int64_t r0 = S.offs[first[g]], r1 = S.offs[first[g + 1]];
                std::vector<uint8_t> cb((size_t)(r1 - r0) * 22);
                std::vector<uint64_t*> co;
                std::vector<uint8_t*> ko;
                for (int m = first[g]; m < first[g + 1]; ++m) {
                    co.push_back(reinterpret_cast<uint64_t*>(cb.data() + (S.offs[m] - r0) * 16));
                    ko.push_back(cb.data() + (r1 - r0) * 16 + (S.offs[m] - r0) * 6);
                }
                rc = build_codes_host(c, &gi, co.data(), ko.data(), &near, stats, kPassCodes, (double)N);
                if (rc == CASHASH_OK &&
                    (!write_at(out.fd, cb.data(), (size_t)(r1 - r0) * 16, kFileHeader + r0 * 16) ||
                     !write_at(out.fd, cb.data() + (r1 - r0) * 16, (size_t)(r1 - r0) * 6, kFileHeader + N * 16 + r0 * 6)))
                    rc = fail(CASHASH_E_IO, "write to %s failed", codes_path);
            }
            const bool read_ok = !ahead.valid() || ahead.get();
            if (rc != CASHASH_OK) return rc;
            if (!read_ok) return fail(CASHASH_E_IO, "read of %s failed", set_path);
            disk += (S.offs[first[g + 1]] - S.offs[first[g]]) * kDim;
            group_loads += g + 1 < ng;
        }
        if (pass == 0 && N > 0)
            HIPCHK(launch_bias(c->stream, c->dR64.as<double>(), c->dS.as<unsigned long long>(), (double)N,
                               c->dBias.as<float>()));
    }
    if (::fdatasync(out.fd) != 0) return fail(CASHASH_E_IO, "sync of %s failed", codes_path);
    if (stats) {
        stats->near_margin_recomputes = near;
        stats->disk_bytes = disk;
        stats->group_loads = group_loads;
        stats->ms_codes = now_ms() - t0;
    }
    return CASHASH_OK;
}

extern "C" int cashash_match_pairs_disk(cashash_ctx* c, const char* set_path, const char* codes_path,
                                        int64_t n_pairs, const int32_t* pairs, const char* out_path,
                                        const char* progress_path, int64_t host_budget_bytes, int64_t max_steps,
                                        int64_t* steps_left, cashash_stats* stats) {
    if (!c) return fail(CASHASH_E_INVAL, "null context");
    if (c->cfg.mem != CASHASH_MEM_HOST) return fail(CASHASH_E_INVAL, "the disk level needs cfg.mem = CASHASH_MEM_HOST");
    if (!codes_path || !out_path) return fail(CASHASH_E_INVAL, "null path");
    if (host_budget_bytes <= 0) return fail(CASHASH_E_INVAL, "host_budget_bytes must be > 0");
    if (max_steps < 0) return fail(CASHASH_E_INVAL, "max_steps must be >= 0");
    zero_stats(stats);
    const double t0 = now_ms();
    SetFile S;
    RETCHK(open_set(set_path, S));
    const int M = S.n_images;
    const int64_t N = S.offs.back();
    RETCHK(check_pairs(M, n_pairs, pairs));
    Fd cf;
    cf.fd = ::open(codes_path, O_RDONLY);
    if (cf.fd < 0) return fail(CASHASH_E_IO, "cannot open codes file %s", codes_path);
    {
        char magic[8];
        int64_t hdr[2];
        if (!read_at(cf.fd, magic, 8, 0) || std::memcmp(magic, kCodMagic, 8) != 0 || !read_at(cf.fd, hdr, 16, 8) ||
            hdr[0] != M || hdr[1] != N)
            return fail(CASHASH_E_IO, "%s is not the codes file of %s", codes_path, set_path);
    }
    // group pairs: the block-pair scheduler over images with host slots of a
    // third of the budget (two groups in progress, one read ahead)
    const int64_t slot = host_budget_bytes / 3;
    std::vector<int64_t> img_bytes(M);
    for (int m = 0; m < M; ++m) img_bytes[m] = (int64_t)S.n_feat[m] * (kDim + 22);
    Schedule G;
    const int pr = plan_schedule(M, img_bytes.data(), n_pairs, pairs, slot, G);
    if (pr == -1) return fail(CASHASH_E_NOMEM, "an image does not fit a host group of %lld bytes", (long long)slot);
    if (pr) return fail(CASHASH_E_INVAL, "scheduler rejected the pair list");
    const int64_t n_steps = (int64_t)G.steps.size();
    std::vector<int64_t> out_off(n_pairs);
    int64_t T = 0;
    for (int64_t p = 0; p < n_pairs; ++p) {
        out_off[p] = T;
        T += S.n_feat[pairs[2 * p]];
    }
    // output file (kept if it already has the right header: a resumed run)
    Fd of;
    of.fd = ::open(out_path, O_RDWR | O_CREAT, 0644);
    if (of.fd < 0) return fail(CASHASH_E_IO, "cannot open %s", out_path);
    {
        const int64_t hdr[2] = {n_pairs, T};
        char magic[8];
        int64_t old[2] = {-1, -1};
        struct stat st;
        const bool same = ::fstat(of.fd, &st) == 0 && st.st_size == (off_t)(kFileHeader + 12 * T) &&
                          read_at(of.fd, magic, 8, 0) && std::memcmp(magic, kOutMagic, 8) == 0 &&
                          read_at(of.fd, old, 16, 8) && old[0] == n_pairs && old[1] == T;
        if (!same && (::ftruncate(of.fd, 0) != 0 || ::ftruncate(of.fd, (off_t)(kFileHeader + 12 * T)) != 0 ||
                      !write_at(of.fd, kOutMagic, 8, 0) || !write_at(of.fd, hdr, 16, 8)))
            return fail(CASHASH_E_IO, "write to %s failed", out_path);
    }
    // progress: one byte per group pair, valid only for the same plan
    uint64_t hash = 1469598103934665603ull;
    hash = fnv1a(hash, S.offs.data(), S.offs.size() * 8);
    hash = fnv1a(hash, pairs, (size_t)n_pairs * 8);
    hash = fnv1a(hash, &slot, 8);
    hash = fnv1a(hash, &n_steps, 8);
    // the matching configuration (it decides every output) ...
    {
        const int32_t cfgv[5] = {c->cfg.k, c->cfg.ratio_num, c->cfg.ratio_den, c->cfg.max_hamming, c->cfg.mode};
        hash = fnv1a(hash, cfgv, sizeof cfgv);
    }
    // ... and the identity of the set and codes files: size and modification
    // time, so that a regenerated file invalidates the progress
    for (int fd : {S.f.fd, cf.fd}) {
        struct stat st;
        if (::fstat(fd, &st) != 0) return fail(CASHASH_E_IO, "cannot stat an input file");
        const int64_t id[4] = {(int64_t)st.st_size, (int64_t)st.st_mtim.tv_sec, (int64_t)st.st_mtim.tv_nsec,
                               (int64_t)st.st_ino};
        hash = fnv1a(hash, id, sizeof id);
    }
    std::vector<uint8_t> done((size_t)n_steps, 0);
    Fd pf;
    if (progress_path) {
        pf.fd = ::open(progress_path, O_RDWR | O_CREAT, 0644);
        if (pf.fd < 0) return fail(CASHASH_E_IO, "cannot open %s", progress_path);
        char magic[8];
        uint64_t h = 0;
        int64_t ns = -1;
        const bool same = read_at(pf.fd, magic, 8, 0) && std::memcmp(magic, kPrgMagic, 8) == 0 &&
                          read_at(pf.fd, &h, 8, 8) && read_at(pf.fd, &ns, 8, 16) && h == hash && ns == n_steps &&
                          (n_steps == 0 || read_at(pf.fd, done.data(), (size_t)n_steps, kFileHeader));
        if (!same) {
            std::fill(done.begin(), done.end(), 0);
            const int64_t zero = 0;
            if (::ftruncate(pf.fd, 0) != 0 || !write_at(pf.fd, kPrgMagic, 8, 0) || !write_at(pf.fd, &hash, 8, 8) ||
                !write_at(pf.fd, &n_steps, 8, 16) || !write_at(pf.fd, &zero, 8, 24) ||
                (n_steps > 0 && !write_at(pf.fd, done.data(), (size_t)n_steps, kFileHeader)) || ::fdatasync(pf.fd) != 0)
                return fail(CASHASH_E_IO, "write to %s failed", progress_path);
        }
    }
    // three host slots of groups: descriptors, codes and keys of each image
    std::vector<uint8_t> hbuf[3];
    int slot_group[3] = {-1, -1, -1};
    int64_t slot_used[3] = {-1, -1, -1};
    std::vector<int64_t> place(M, -1);  // image -> offset in its slot
    std::vector<int> slot_of_img(M, -1);
    int64_t disk = 0, group_loads = 0;
    auto read_group = [&](int g, int s) -> bool {
        // called on the read-ahead thread for a slot nobody else touches
        std::vector<uint8_t>& b = hbuf[s];
        int64_t need = 0;
        for (int i = G.block_first[g]; i < G.block_first[g + 1]; ++i) need += img_bytes[G.block_images[i]];
        if ((int64_t)b.size() < need) b.resize((size_t)need);
        int64_t off = 0;
        for (int i = G.block_first[g]; i < G.block_first[g + 1]; ++i) {
            const int m = G.block_images[i];
            const int64_t n = S.n_feat[m], r0 = S.offs[m];
            if (n > 0 && (!read_at(S.f.fd, b.data() + off, (size_t)n * kDim, S.desc_off + r0 * kDim) ||
                          !read_at(cf.fd, b.data() + off + n * kDim, (size_t)n * 16, kFileHeader + r0 * 16) ||
                          !read_at(cf.fd, b.data() + off + n * (kDim + 16), (size_t)n * 6, kFileHeader + N * 16 + r0 * 6)))
                return false;
            off += img_bytes[m];
        }
        return true;
    };
    auto bind_group = [&](int g, int s) {
        int64_t off = 0;
        for (int i = G.block_first[g]; i < G.block_first[g + 1]; ++i) {
            const int m = G.block_images[i];
            place[m] = off;
            slot_of_img[m] = s;
            off += img_bytes[m];
        }
        slot_group[s] = g;
        disk += off;
        group_loads++;
    };
    auto slot_holding = [&](int g) {
        for (int s = 0; s < 3; ++s)
            if (slot_group[s] == g) return s;
        return -1;
    };
    auto free_slot = [&](int keep0, int keep1, int busy) {
        int best = -1;
        for (int s = 0; s < 3; ++s) {
            if (s == busy || (slot_group[s] >= 0 && (slot_group[s] == keep0 || slot_group[s] == keep1))) continue;
            if (best < 0 || slot_used[s] < slot_used[best]) best = s;
        }
        return best;
    };
    std::future<bool> ahead;
    int ahead_group = -1, ahead_slot = -1;
    auto finish_ahead = [&]() -> bool {
        if (!ahead.valid()) return true;
        const bool ok = ahead.get();
        if (ok) bind_group(ahead_group, ahead_slot);
        ahead_group = ahead_slot = -1;
        return ok;
    };
    int64_t ran = 0;
    cashash_stats st_step;
    // outputs are written (and synced, then the progress byte) by a writer
    // thread while the next group pair computes; two buffers alternate
    std::vector<int32_t> o_bufs[2];
    int cur = 0;
    std::future<bool> writer;
    int64_t writing = -1;  // group pair whose outputs the writer holds
    auto finish_write = [&]() -> bool {
        if (!writer.valid()) return true;
        const bool ok = writer.get();
        if (ok) done[writing] = 1;
        writing = -1;
        return ok;
    };
    for (int64_t st = 0; st < n_steps; ++st) {
        if (done[st]) continue;
        if (max_steps > 0 && ran >= max_steps) break;
        const SchedStep& step = G.steps[st];
        for (int g : {step.bi, step.bk}) {
            if (slot_holding(g) >= 0) continue;
            if (ahead_group == g) {
                if (!finish_ahead()) return fail(CASHASH_E_IO, "read of %s or %s failed", set_path, codes_path);
                continue;
            }
            if (!finish_ahead()) return fail(CASHASH_E_IO, "read of %s or %s failed", set_path, codes_path);
            const int s = free_slot(step.bi, step.bk, -1);
            slot_group[s] = -1;
            if (!read_group(g, s)) return fail(CASHASH_E_IO, "read of %s or %s failed", set_path, codes_path);
            bind_group(g, s);
        }
        const int si = slot_holding(step.bi), sk = slot_holding(step.bk);
        slot_used[si] = slot_used[sk] = st;
        // read ahead the next pending step's missing group
        if (!ahead.valid())
            for (int64_t nx = st + 1; nx < n_steps; ++nx) {
                if (done[nx]) continue;
                for (int g : {G.steps[nx].bi, G.steps[nx].bk}) {
                    if (slot_holding(g) >= 0) continue;
                    const int s = free_slot(step.bi, step.bk, -1);
                    if (s < 0) break;
                    slot_group[s] = -1;
                    ahead_group = g;
                    ahead_slot = s;
                    ahead = std::async(std::launch::async, read_group, g, s);
                    break;
                }
                break;
            }
        // host-memory matching of this group pair's pairs
        std::vector<const uint8_t*> dp(M, nullptr), kp8(M, nullptr);
        std::vector<const uint64_t*> cp(M, nullptr);
        for (int g : {step.bi, step.bk})
            for (int i = G.block_first[g]; i < G.block_first[g + 1]; ++i) {
                const int m = G.block_images[i];
                const uint8_t* base = hbuf[slot_of_img[m]].data() + place[m];
                const int64_t n = S.n_feat[m];
                dp[m] = base;
                cp[m] = reinterpret_cast<const uint64_t*>(base + n * kDim);
                kp8[m] = base + n * (kDim + 16);
            }
        cashash_images view{M, dp.data(), S.n_feat.data()};
        MatchJob J;
        int64_t nq = 0;
        for (int64_t i = step.pair_begin; i < step.pair_end; ++i) {
            const int64_t p = G.order[i];
            J.pair_q.push_back(pairs[2 * p]);
            J.pair_t.push_back(pairs[2 * p + 1]);
            J.pair_out.push_back(nq);
            nq += S.n_feat[pairs[2 * p]];
        }
        std::vector<int32_t>& o_buf = o_bufs[cur];
        o_buf.assign((size_t)std::max<int64_t>(nq, 1) * 3, 0);
        zero_stats(&st_step);
        const int rc = match_host(c, &view, cp.data(), kp8.data(), nullptr, J, o_buf.data(), o_buf.data() + nq,
                                  o_buf.data() + 2 * nq, &st_step);
        if (rc != CASHASH_OK) {
            finish_ahead();
            finish_write();
            return rc;
        }
        if (!finish_write()) {
            finish_ahead();
            return fail(CASHASH_E_IO, "write to %s or %s failed", out_path, progress_path ? progress_path : "");
        }
        writing = st;
        writer = std::async(std::launch::async, [&, st, nq, b = cur, pb = step.pair_begin, pe = step.pair_end,
                                                 po = std::move(J.pair_out)]() {
            const std::vector<int32_t>& ob = o_bufs[b];
            for (int64_t i = pb; i < pe; ++i) {
                const int64_t p = G.order[i];
                const int64_t n = S.n_feat[pairs[2 * p]];
                for (int a = 0; n > 0 && a < 3; ++a)
                    if (!write_at(of.fd, ob.data() + a * nq + po[i - pb], (size_t)n * 4,
                                  kFileHeader + 4 * (a * T + out_off[p])))
                        return false;
            }
            if (pf.fd >= 0) {
                // durable outputs before the progress byte that vouches for them
                const uint8_t one = 1;
                if (::fdatasync(of.fd) != 0 || !write_at(pf.fd, &one, 1, kFileHeader + st) || ::fdatasync(pf.fd) != 0)
                    return false;
            }
            return true;
        });
        cur ^= 1;
        ++ran;
        if (stats) {
            stats->pairs += (int64_t)J.pair_q.size();
            stats->queries += nq;
            stats->bucket_entries += J.bucket_entries;
            stats->union_size += J.union_size;
            stats->ranked += J.ranked;
            stats->h2d_bytes += st_step.h2d_bytes;
            stats->d2h_bytes += st_step.d2h_bytes;
            stats->image_loads += st_step.image_loads;
        }
    }
    if (!finish_write()) {
        finish_ahead();
        return fail(CASHASH_E_IO, "write to %s or %s failed", out_path, progress_path ? progress_path : "");
    }
    if (!finish_ahead()) return fail(CASHASH_E_IO, "read of %s or %s failed", set_path, codes_path);
    int64_t left = 0;
    for (int64_t st = 0; st < n_steps; ++st) left += done[st] ? 0 : 1;
    if (steps_left) *steps_left = left;
    if (stats) {
        stats->disk_bytes = disk;
        stats->group_loads = group_loads;
        stats->ms_match = now_ms() - t0;
    }
    return CASHASH_OK;
}
