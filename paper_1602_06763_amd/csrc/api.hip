// C ABI of the library (declared in include/relapack.h) and the per-thread /
// per-device state behind it: stream, status block, workspace, plan
// recording and the per-kernel-family timers.
#include "common.hpp"

#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>

namespace rl {

namespace {

constexpr int kMaxDev = 16;
constexpr int kScratchSlots = 12;   // 0-6 mixed solver, 7 LU row tracker, 8 correction-solve block inverses,
                                    // 9 launch order of a batch, 10 GMRES basis, 11 copy of a
                                    // triangular product's right-hand block

struct DevState {
    bool init = false;
    DevStatus *dstat = nullptr;
    DevStatus *hstat = nullptr;
    unsigned long long *panel_rec = nullptr;
    unsigned int panel_epoch = 0;   // next free epoch of the panel records
    int *rowsrc = nullptr;
    size_t rowsrc_elems = 0;
    void *slot[kScratchSlots] = {};
    size_t slot_bytes[kScratchSlots] = {};
    int num_cu = 256;
    // single-launch triangular solve
    unsigned long long *trsv_x = nullptr;   // epoch-tagged solution words
    size_t trsv_x_words = 0;
    unsigned long long *trsv_ticket = nullptr;
    unsigned long long trsv_tickets = 0;
    unsigned int trsv_epoch = 0;
    // LU look-ahead: CU-masked stream pair (created on first use)
    bool la_tried = false;
    LaStreams la;
};

DevState g_dev[kMaxDev];
std::mutex g_mu;
// One library call at a time per device: the status block, the panel's
// exchange records, the solve's tickets and the workspace are per device.
std::recursive_mutex g_call_mu[kMaxDev];

struct TraceRec {
    int kind;
    double flops, bytes;
    hipEvent_t e0, e1;
};

thread_local Ctx t_ctx;
thread_local int t_err = 0;
thread_local int t_locked = -1;   // device whose call lock this thread holds
thread_local std::vector<TraceRec> t_trace;
thread_local std::vector<hipEvent_t> t_evpool;
thread_local size_t t_evused = 0;

__global__ void fill_int_k(int *p, long long n, int v) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void fill_u64_k(unsigned long long *p, long long n, unsigned long long v) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void zero_u64_one_k(unsigned long long *p) {
    if (threadIdx.x == 0) *p = 0ull;
}

__global__ void reset_status_k(DevStatus *s) {
    if (threadIdx.x == 0) { s->info = 0; s->error = 0; s->barrier = 0u; s->ovf = 0; }
}

}  // namespace

Ctx &ctx() { return t_ctx; }

int launch_error(hipError_t e) {
    if (!t_err) t_err = (int)e;
    return (int)e;
}

void ensure_device(Ctx &c) {
    int dev = 0;
    RL_CHECK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDev) { launch_error(hipErrorInvalidDevice); return; }
    std::lock_guard<std::mutex> lk(g_mu);
    DevState &d = g_dev[dev];
    if (!d.init) {
        hipDeviceProp_t p;
        if (hipGetDeviceProperties(&p, dev) == hipSuccess) d.num_cu = p.multiProcessorCount;
        RL_CHECK(hipMalloc(&d.dstat, sizeof(DevStatus)));
        RL_CHECK(hipHostMalloc(&d.hstat, sizeof(DevStatus), hipHostMallocDefault));
        d.init = true;
    }
    c.device = dev;
    c.dstat = d.dstat;
    c.hstat = d.hstat;
    c.rowsrc = d.rowsrc;
    c.rowsrc_elems = d.rowsrc_elems;
    c.num_cu = d.num_cu;
}

static void ensure_rowsrc(Ctx &c, size_t m) {
    std::lock_guard<std::mutex> lk(g_mu);
    DevState &d = g_dev[c.device];
    if (d.rowsrc_elems < m) {
        if (d.rowsrc) { RL_CHECK(hipStreamSynchronize(c.stream)); RL_CHECK(hipFree(d.rowsrc)); }
        d.rowsrc = nullptr;
        RL_CHECK(hipMalloc(&d.rowsrc, m * sizeof(int)));
        d.rowsrc_elems = m;
    }
    c.rowsrc = d.rowsrc;
    c.rowsrc_elems = d.rowsrc_elems;
}

void *workspace(Ctx &c, int slot, size_t bytes) {
    if (c.fixed) {
        // a caller-free call holds only the LU row tracker
        if (slot == 7 && bytes <= c.fixed->tracker_bytes) return c.fixed->tracker;
        launch_error(hipErrorOutOfMemory);
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    DevState &d = g_dev[c.device];
    if (d.slot_bytes[slot] < bytes) {
        if (d.slot[slot]) { RL_CHECK(hipStreamSynchronize(c.stream)); RL_CHECK(hipFree(d.slot[slot])); }
        d.slot[slot] = nullptr;
        if (hipMalloc(&d.slot[slot], bytes) != hipSuccess) {
            d.slot_bytes[slot] = 0;
            launch_error(hipErrorOutOfMemory);
            return nullptr;
        }
        d.slot_bytes[slot] = bytes;
    }
    return d.slot[slot];
}

unsigned long long *panel_records(Ctx &c, unsigned int *epoch) {
    const long long words = (long long)kLuLeaf * kRecSlots * kRecWords;
    if (c.fixed) {
        unsigned int &e = *c.fixed->epoch;
        if (e < 2u * kLuLeaf || e > 0xFFFFFFFFu - 2u * kLuLeaf) {
            hipLaunchKernelGGL(fill_u64_k, dim3((unsigned)((words + 255) / 256)), dim3(256), 0, c.stream,
                               c.fixed->rec, words, 0ull);
            RL_CHECK(hipGetLastError());
            e = 2u * kLuLeaf;
        }
        *epoch = e;
        e += kLuLeaf;
        return c.fixed->rec;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    DevState &d = g_dev[c.device];
    if (!d.panel_rec) {
        if (hipMalloc(&d.panel_rec, (size_t)words * sizeof(unsigned long long)) != hipSuccess) {
            d.panel_rec = nullptr;
            launch_error(hipErrorOutOfMemory);
            return nullptr;
        }
        d.panel_epoch = 0;
    }
    // epochs below 2·kLuLeaf are never handed out, so zeroed words never match;
    // on wrap-around the records are cleared again (stream-ordered before the panel)
    if (d.panel_epoch < 2u * kLuLeaf || d.panel_epoch > 0xFFFFFFFFu - 2u * kLuLeaf) {
        hipLaunchKernelGGL(fill_u64_k, dim3((unsigned)((words + 255) / 256)), dim3(256), 0, c.stream, d.panel_rec,
                           words, 0ull);
        RL_CHECK(hipGetLastError());
        d.panel_epoch = 2u * kLuLeaf;
    }
    *epoch = d.panel_epoch;
    d.panel_epoch += kLuLeaf;
    return d.panel_rec;
}

namespace {
// off by default: on MI355X it measured slower (dgetrf n = 16384: 142.0 ms
// off, 153.3 ms on; n = 32768: 602.4 against 626.9 ms), see relapack.h
bool g_la_on = false;
}

bool lookahead_enabled() { return g_la_on; }
void lookahead_enable(bool on) { g_la_on = on; }

// The update of the rest of the right half runs on a stream restricted to
// all but 64 CUs (logical CU i sits on XCD i mod 8, so the first 64 are 8 per
// XCD); the block factored ahead runs on an unrestricted stream, so its
// cooperative panels (up to 64 resident workgroups, one per CU, at
// m <= 32768) always find the 64 CUs the update leaves free, and its other
// kernels take the whole chip once the update is done.
bool lookahead_streams(Ctx &c, LaStreams *out) {
    std::lock_guard<std::mutex> lk(g_mu);
    DevState &d = g_dev[c.device];
    if (!d.la_tried) {
        d.la_tried = true;
        const int ncu = d.num_cu, small = 64;
        if (ncu >= 2 * small && ncu <= 1024) {
            const int words = (ncu + 31) / 32;
            std::vector<uint32_t> mb(words, 0u);
            for (int i = small; i < ncu; ++i) mb[i / 32] |= 1u << (i % 32);
            hipStream_t a = nullptr, b = nullptr;
            bool ok = hipStreamCreateWithFlags(&a, hipStreamNonBlocking) == hipSuccess &&
                      hipExtStreamCreateWithCUMask(&b, (uint32_t)words, mb.data()) == hipSuccess;
            for (int e = 0; ok && e < 3; ++e)
                ok = hipEventCreateWithFlags(&d.la.ev[e], hipEventDisableTiming) == hipSuccess;
            if (ok) {
                d.la.small = a;
                d.la.big = b;
                d.la.small_cu = ncu;
                d.la.big_cu = ncu - small;
            } else {
                if (a) (void)hipStreamDestroy(a);
                if (b) (void)hipStreamDestroy(b);
                for (auto &e : d.la.ev) {
                    if (e) (void)hipEventDestroy(e);
                    e = nullptr;
                }
                (void)hipGetLastError();
            }
        }
    }
    *out = d.la;
    return d.la.small != nullptr;
}

TrsvWork trsv_work(Ctx &c, long long m, int nb, int launches, long long row_words, int tickets_per_block) {
    TrsvWork w;
    if (c.fixed) {   // never reached: caller-free calls take the recursive solves
        launch_error(hipErrorOutOfMemory);
        return w;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    DevState &d = g_dev[c.device];
    const long long words = m * row_words;
    if (d.trsv_x_words < (size_t)words) {
        if (d.trsv_x) { RL_CHECK(hipStreamSynchronize(c.stream)); RL_CHECK(hipFree(d.trsv_x)); }
        d.trsv_x = nullptr;
        if (hipMalloc(&d.trsv_x, (size_t)words * sizeof(unsigned long long)) != hipSuccess) {
            d.trsv_x_words = 0;
            launch_error(hipErrorOutOfMemory);
            return w;
        }
        // epochs start at 1, so zeroed words never match
        hipLaunchKernelGGL(fill_u64_k, dim3((unsigned)((words + 255) / 256)), dim3(256), 0, c.stream, d.trsv_x,
                           words, 0ull);
        d.trsv_x_words = (size_t)words;
    }
    if (!d.trsv_ticket) {
        RL_CHECK(hipMalloc(&d.trsv_ticket, sizeof(unsigned long long)));
        hipLaunchKernelGGL(zero_u64_one_k, dim3(1), dim3(64), 0, c.stream, d.trsv_ticket);
        d.trsv_tickets = 0;
    }
    w.xw = d.trsv_x;
    w.ticket = d.trsv_ticket;
    w.ticket_base = d.trsv_tickets;
    w.epoch = d.trsv_epoch + 1;
    d.trsv_tickets += (unsigned long long)nb * (unsigned long long)launches * (unsigned long long)tickets_per_block;
    d.trsv_epoch += (unsigned)launches;
    return w;
}

void trace_begin(Ctx &c, int kind) {
    (void)kind;
    if (!c.trace || c.plan) return;
    if (t_evused + 2 > t_evpool.size()) {
        for (int i = 0; i < 64; ++i) {
            hipEvent_t e;
            RL_CHECK(hipEventCreate(&e));
            t_evpool.push_back(e);
        }
    }
    RL_CHECK(hipEventRecord(t_evpool[t_evused], c.stream));
}

void trace_end(Ctx &c, int kind, double flops, double bytes) {
    if (!c.trace || c.plan) return;
    hipEvent_t e0 = t_evpool[t_evused], e1 = t_evpool[t_evused + 1];
    RL_CHECK(hipEventRecord(e1, c.stream));
    t_evused += 2;
    t_trace.push_back(TraceRec{kind, flops, bytes, e0, e1});
}

void trace_kernel_begin(Ctx &c) {
    c.tev_armed = false;
    c.tev_used = false;
    if (!c.trace || c.plan) return;
    if (t_evused + 2 > t_evpool.size()) {
        for (int i = 0; i < 64; ++i) {
            hipEvent_t e;
            RL_CHECK(hipEventCreate(&e));
            t_evpool.push_back(e);
        }
    }
    c.tev0 = t_evpool[t_evused];
    c.tev1 = t_evpool[t_evused + 1];
    c.tev_armed = true;
}

void trace_kernel_end(Ctx &c, int kind, double flops, double bytes) {
    c.tev_armed = false;
    if (!c.trace || c.plan || !c.tev_used) return;
    c.tev_used = false;
    t_trace.push_back(TraceRec{kind, flops, bytes, t_evpool[t_evused], t_evpool[t_evused + 1]});
    t_evused += 2;
}

// Begin / end of one library call.
static bool call_begin(Ctx &c, bool abort_on_info) {
    t_err = 0;
    ensure_device(c);
    if (t_err) return false;
    if (t_locked < 0) {
        g_call_mu[c.device].lock();
        t_locked = c.device;
    }
    c.abort_on_info = abort_on_info;
    c.level = 0;
    hipLaunchKernelGGL(reset_status_k, dim3(1), dim3(64), 0, c.stream, c.dstat);
    RL_CHECK(hipGetLastError());
    return t_err == 0;
}

static int call_end(Ctx &c) {
    if (!t_err) {
        RL_CHECK(hipMemcpyAsync(c.hstat, c.dstat, sizeof(DevStatus), hipMemcpyDeviceToHost, c.stream));
        RL_CHECK(hipStreamSynchronize(c.stream));
    } else if (t_locked >= 0) {
        (void)hipStreamSynchronize(c.stream);   // nothing of this call may still run once the lock is released
    }
    const int r = t_err ? -1000 - t_err : (c.hstat->error ? -2000 - c.hstat->error : c.hstat->info);
    if (t_locked >= 0) {
        g_call_mu[t_locked].unlock();
        t_locked = -1;
    }
    return r;
}

static inline bool is(char a, char b) { return a == b || a == (char)(b + ('a' - 'A')); }

}  // namespace rl

using namespace rl;

namespace rl {

template <typename T>
static int potrf_batched_call(char uplo, int count, const int *n, T *const *A, const int *lda, int *info) {
    if (!is(uplo, 'L') && !is(uplo, 'U')) return -1;
    if (count < 0) return -2;
    if (count == 0) return 0;
    if (!n || !A || !lda || !info) return -3;
    Ctx &c = ctx();
    if (!call_begin(c, false)) return call_end(c);
    potrf_batched<T>(c, is(uplo, 'U'), count, n, A, lda, info);
    const int r = call_end(c);
    return r < 0 ? r : 0;
}

template <typename T>
static int getrf_batched_call(int count, const int *n, T *const *A, const int *lda, int *const *ipiv, int *info) {
    if (count < 0) return -1;
    if (count == 0) return 0;
    if (!n || !A || !lda || !ipiv || !info) return -2;
    Ctx &c = ctx();
    if (!call_begin(c, false)) return call_end(c);
    getrf_batched<T>(c, count, n, A, lda, ipiv, info);
    const int r = call_end(c);
    return r < 0 ? r : 0;
}

// ---- allocation-free LU: fixed device workspace ------------------------------
// relapack_dgetrf_noalloc runs on this array instead of the grow-only
// workspace: status block, the source row of every position after a panel,
// the row tracker (two buffers, the inverse slots, the batch source map) and
// the panel exchange records, for at most kNaMaxM rows. Every GPU the library
// runs on holds one copy (about 8.6 MB) until the process ends; host code
// reaches it only through the address hipGetSymbolAddress returns per device.
constexpr long long kNaMaxM = kLaswpBatchRows;
constexpr size_t kNaStatusOff = 0;
constexpr size_t kNaRowsrcOff = 256;
constexpr size_t kNaTrackerOff = kNaRowsrcOff + (size_t)kNaMaxM * sizeof(int);
constexpr size_t kNaTrackerBytes = (size_t)(4 + 2 * kLaswpDepth) * (size_t)kNaMaxM * sizeof(int);
constexpr size_t kNaRecOff = kNaTrackerOff + kNaTrackerBytes;
constexpr size_t kNaRecBytes = (size_t)kLuLeaf * kRecSlots * kRecWords * sizeof(unsigned long long);
constexpr size_t kNaBytes = kNaRecOff + kNaRecBytes;
static_assert(kNaRecOff % 256 == 0, "records start on a 256-byte boundary");

}  // namespace rl

static __device__ __align__(256) unsigned char scratch[rl::kNaBytes];

namespace rl {
namespace {

struct NaDev {
    unsigned char *ptr = nullptr;   // this device's copy of `scratch`
    int num_cu = 256;
    unsigned int epoch = 0;         // next free epoch of its panel records
    FixedWs ws;
};
NaDev g_na[kMaxDev];
thread_local DevStatus t_na_status;   // host copy of the status block (pageable)

// Device address of `scratch` on the current device, looked up once per
// device; the call lock of that device is taken as for every other call.
bool na_call_begin(Ctx &c) {
    t_err = 0;
    int dev = 0;
    RL_CHECK(hipGetDevice(&dev));
    if (t_err) return false;
    if (dev < 0 || dev >= kMaxDev) { launch_error(hipErrorInvalidDevice); return false; }
    NaDev &d = g_na[dev];
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (!d.ptr) {
            void *p = nullptr;
            const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !p) {
                launch_error(e != hipSuccess ? e : hipErrorInvalidSymbol);
                return false;
            }
            int cu = 0;
            if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cu > 0)
                d.num_cu = cu;
            unsigned char *b = (unsigned char *)p;
            d.ws.tracker = (int *)(b + kNaTrackerOff);
            d.ws.tracker_bytes = kNaTrackerBytes;
            d.ws.rec = (unsigned long long *)(b + kNaRecOff);
            d.ws.epoch = &d.epoch;
            d.epoch = 0;   // the first panel clears the records
            d.ptr = b;
        }
    }
    if (t_locked < 0) {
        g_call_mu[dev].lock();
        t_locked = dev;
    }
    c.device = dev;
    c.dstat = (DevStatus *)(d.ptr + kNaStatusOff);
    c.hstat = &t_na_status;
    c.rowsrc = (int *)(d.ptr + kNaRowsrcOff);
    c.rowsrc_elems = (size_t)kNaMaxM;
    c.num_cu = d.num_cu;
    c.fixed = &d.ws;
    c.abort_on_info = false;
    c.level = 0;
    hipLaunchKernelGGL(reset_status_k, dim3(1), dim3(64), 0, c.stream, c.dstat);
    RL_CHECK(hipGetLastError());
    return t_err == 0;
}

int na_call_end(Ctx &c) {
    const int r = call_end(c);
    c.fixed = nullptr;
    c.dstat = nullptr;
    c.hstat = nullptr;
    c.rowsrc = nullptr;
    c.rowsrc_elems = 0;
    c.lu_tracked = false;
    return r;
}

}  // namespace

template <typename R>
static void zpotrf_call(char uplo, int n, void *A, int lda, int *info) {
    if (!info) return;
    if (!is(uplo, 'L') && !is(uplo, 'U')) { *info = -1; return; }
    if (n < 0) { *info = -2; return; }
    if (lda < (n > 1 ? n : 1)) { *info = -4; return; }
    *info = 0;
    if (n == 0) return;
    Ctx &c = ctx();
    if (!call_begin(c, true)) { *info = call_end(c); return; }
    zpotrf_top<R>(c, is(uplo, 'L') ? 'L' : 'U', n, A, lda);
    *info = call_end(c);
}

template <typename R>
static void zgetrf_call(int m, int n, void *A, int lda, int *ipiv, int *info) {
    if (!info) return;
    if (m < 0) { *info = -1; return; }
    if (n < 0) { *info = -2; return; }
    if (lda < (m > 1 ? m : 1)) { *info = -4; return; }
    *info = 0;
    if (m == 0 || n == 0) return;
    Ctx &c = ctx();
    if (!call_begin(c, false)) { *info = call_end(c); return; }
    ensure_rowsrc(c, (size_t)m);
    zgetrf_top<R>(c, m, n, A, lda, ipiv);
    *info = call_end(c);
}

}  // namespace rl

extern "C" {

int relapack_version(void) { return 1; }

int relapack_batched_tune(int routine, int bucket, int leaf, int tile) {
    if (routine < 0 || routine > 3) return -1;
    if (bucket < 0 || bucket > 3) return -2;
    return batched_tune_set(routine, bucket, leaf, tile) ? 0 : -3;
}

int relapack_batched_tune_get(int routine, int bucket, int *leaf, int *tile) {
    if (routine < 0 || routine > 3) return -1;
    if (bucket < 0 || bucket > 3) return -2;
    return batched_tune_get(routine, bucket, leaf, tile) ? 0 : -2;
}

void relapack_batched_graphs(int on) { batched_graphs(on != 0); }

void relapack_lookahead(int on) { lookahead_enable(on != 0); }

int relapack_set_stream(void *stream) {
    ctx().stream = (hipStream_t)stream;
    return 0;
}

void *relapack_get_stream(void) { return (void *)ctx().stream; }

void relapack_finalize(void) {
    batched_release();
    for (int i = 0; i < kMaxDev; ++i) {
        // the same lock order as a call: the device's call lock, then the state lock
        std::lock_guard<std::recursive_mutex> call_lk(g_call_mu[i]);
        std::lock_guard<std::mutex> lk(g_mu);
        DevState &d = g_dev[i];
        if (!d.init) continue;
        int cur = 0;
        (void)hipGetDevice(&cur);
        (void)hipSetDevice(i);
        (void)hipDeviceSynchronize();
        (void)hipFree(d.dstat);
        (void)hipHostFree(d.hstat);
        if (d.panel_rec) (void)hipFree(d.panel_rec);
        if (d.rowsrc) (void)hipFree(d.rowsrc);
        if (d.trsv_x) (void)hipFree(d.trsv_x);
        if (d.trsv_ticket) (void)hipFree(d.trsv_ticket);
        if (d.la.small) (void)hipStreamDestroy(d.la.small);
        if (d.la.big) (void)hipStreamDestroy(d.la.big);
        for (auto &e : d.la.ev)
            if (e) (void)hipEventDestroy(e);
        for (int s = 0; s < kScratchSlots; ++s)
            if (d.slot[s]) (void)hipFree(d.slot[s]);
        d = DevState();
        (void)hipSetDevice(cur);
    }
}

void relapack_dpotrf(char uplo, int n, double *A, int lda, int *info) {
    if (!info) return;
    if (!is(uplo, 'L') && !is(uplo, 'U')) { *info = -1; return; }
    if (n < 0) { *info = -2; return; }
    if (lda < (n > 1 ? n : 1)) { *info = -4; return; }
    *info = 0;
    if (n == 0) return;
    Ctx &c = ctx();
    if (!call_begin(c, true)) { *info = call_end(c); return; }
    potrf_rec<double>(c, Mfma::F64, is(uplo, 'L') ? 'L' : 'U', n, A, lda, 0);
    *info = call_end(c);
}

void relapack_dgetrf(int m, int n, double *A, int lda, int *ipiv, int *info) {
    if (!info) return;
    if (m < 0) { *info = -1; return; }
    if (n < 0) { *info = -2; return; }
    if (lda < (m > 1 ? m : 1)) { *info = -4; return; }
    *info = 0;
    if (m == 0 || n == 0) return;
    Ctx &c = ctx();
    if (!call_begin(c, false)) { *info = call_end(c); return; }
    ensure_rowsrc(c, (size_t)m);
    getrf_top<double>(c, Mfma::F64, m, n, A, lda, ipiv);
    *info = call_end(c);
}

void relapack_zpotrf(char uplo, int n, void *A, int lda, int *info) { zpotrf_call<double>(uplo, n, A, lda, info); }
void relapack_cpotrf(char uplo, int n, void *A, int lda, int *info) { zpotrf_call<float>(uplo, n, A, lda, info); }
void relapack_zgetrf(int m, int n, void *A, int lda, int *ipiv, int *info) {
    zgetrf_call<double>(m, n, A, lda, ipiv, info);
}
void relapack_cgetrf(int m, int n, void *A, int lda, int *ipiv, int *info) {
    zgetrf_call<float>(m, n, A, lda, ipiv, info);
}

void relapack_zgemm(char ta, char tb, int m, int n, int k, double alpha, const void *A, int lda, const void *B,
                    int ldb, double beta, void *C, int ldc, int *info) {
    if (!info) return;
    auto op = [](char t) { return is(t, 'N') ? 0 : is(t, 'T') ? 1 : is(t, 'C') ? 2 : -1; };
    const int oa = op(ta), ob = op(tb);
    if (oa < 0) { *info = -1; return; }
    if (ob < 0) { *info = -2; return; }
    if (m < 0) { *info = -3; return; }
    if (n < 0) { *info = -4; return; }
    if (k < 0) { *info = -5; return; }
    const int nrowa = oa ? k : m, nrowb = ob ? n : k;
    if (lda < (nrowa > 1 ? nrowa : 1)) { *info = -8; return; }
    if (ldb < (nrowb > 1 ? nrowb : 1)) { *info = -10; return; }
    if (ldc < (m > 1 ? m : 1)) { *info = -13; return; }
    *info = 0;
    if (m == 0 || n == 0) return;
    Ctx &c = ctx();
    if (!call_begin(c, false)) { *info = call_end(c); return; }
    zgemm_top<double>(c, oa, ob, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc);
    *info = call_end(c);
}

void relapack_dgetrf_noalloc(int m, int n, double *A, int lda, int *ipiv, int *info) {
    if (!info) return;
    if (m < 0 || m > kNaMaxM) { *info = -1; return; }
    if (n < 0) { *info = -2; return; }
    if (lda < (m > 1 ? m : 1)) { *info = -4; return; }
    *info = 0;
    if (m == 0 || n == 0) return;
    Ctx &c = ctx();
    if (!na_call_begin(c)) { *info = na_call_end(c); return; }
    getrf_top<double>(c, Mfma::F64, m, n, A, lda, ipiv);
    *info = na_call_end(c);
}

void relapack_dpotrs(char uplo, int n, int nrhs, const double *A, int lda, double *B, int ldb,
                     int *info) {
    if (!info) return;
    if (!is(uplo, 'L') && !is(uplo, 'U')) { *info = -1; return; }
    if (n < 0) { *info = -2; return; }
    if (nrhs < 0) { *info = -3; return; }
    if (lda < (n > 1 ? n : 1)) { *info = -5; return; }
    if (ldb < (n > 1 ? n : 1)) { *info = -7; return; }
    *info = 0;
    if (n == 0 || nrhs == 0) return;
    Ctx &c = ctx();
    if (!call_begin(c, false)) { *info = call_end(c); return; }
    if (is(uplo, 'L')) {
        trsm<double, double>(c, Mfma::F64, 'L', 'L', 'N', 'N', n, nrhs, A, lda, B, ldb);
        trsm<double, double>(c, Mfma::F64, 'L', 'L', 'T', 'N', n, nrhs, A, lda, B, ldb);
    } else {
        trsm<double, double>(c, Mfma::F64, 'L', 'U', 'T', 'N', n, nrhs, A, lda, B, ldb);
        trsm<double, double>(c, Mfma::F64, 'L', 'U', 'N', 'N', n, nrhs, A, lda, B, ldb);
    }
    *info = call_end(c);
}

void relapack_dgetrs(char trans, int n, int nrhs, const double *A, int lda, const int *ipiv, double *B,
                     int ldb, int *info) {
    if (!info) return;
    if (!is(trans, 'N') && !is(trans, 'T') && !is(trans, 'C')) { *info = -1; return; }
    if (n < 0) { *info = -2; return; }
    if (nrhs < 0) { *info = -3; return; }
    if (lda < (n > 1 ? n : 1)) { *info = -5; return; }
    if (ldb < (n > 1 ? n : 1)) { *info = -8; return; }
    *info = 0;
    if (n == 0 || nrhs == 0) return;
    Ctx &c = ctx();
    if (!call_begin(c, false)) { *info = call_end(c); return; }
    if (is(trans, 'N')) {
        laswp_rows<double>(c, nrhs, B, ldb, ipiv, 0, n, false);
        trsm<double, double>(c, Mfma::F64, 'L', 'L', 'N', 'U', n, nrhs, A, lda, B, ldb);
        trsm<double, double>(c, Mfma::F64, 'L', 'U', 'N', 'N', n, nrhs, A, lda, B, ldb);
    } else {
        trsm<double, double>(c, Mfma::F64, 'L', 'U', 'T', 'N', n, nrhs, A, lda, B, ldb);
        trsm<double, double>(c, Mfma::F64, 'L', 'L', 'T', 'U', n, nrhs, A, lda, B, ldb);
        laswp_rows<double>(c, nrhs, B, ldb, ipiv, 0, n, true);
    }
    *info = call_end(c);
}

void relapack_dgemm(char ta, char tb, int m, int n, int k, double alpha, const double *A, int lda,
                    const double *B, int ldb, double beta, double *C, int ldc, int *info) {
    if (!info) return;
    const bool tra = is(ta, 'T') || is(ta, 'C'), trb = is(tb, 'T') || is(tb, 'C');
    if (!tra && !is(ta, 'N')) { *info = -1; return; }
    if (!trb && !is(tb, 'N')) { *info = -2; return; }
    if (m < 0) { *info = -3; return; }
    if (n < 0) { *info = -4; return; }
    if (k < 0) { *info = -5; return; }
    const int nrowa = tra ? k : m, nrowb = trb ? n : k;
    if (lda < (nrowa > 1 ? nrowa : 1)) { *info = -8; return; }
    if (ldb < (nrowb > 1 ? nrowb : 1)) { *info = -10; return; }
    if (ldc < (m > 1 ? m : 1)) { *info = -13; return; }
    *info = 0;
    if (m == 0 || n == 0) return;
    Ctx &c = ctx();
    if (!call_begin(c, false)) { *info = call_end(c); return; }
    gemm<double, double, double>(c, Mfma::F64, tra ? 'T' : 'N', trb ? 'T' : 'N', 0, m, n, k, alpha, A,
                                 lda, B, ldb, beta, C, ldc);
    *info = call_end(c);
}

void relapack_dsyrk(char uplo, char trans, int n, int k, double alpha, const double *A, int lda,
                    double beta, double *C, int ldc, int *info) {
    if (!info) return;
    if (!is(uplo, 'L') && !is(uplo, 'U')) { *info = -1; return; }
    const bool tr = is(trans, 'T') || is(trans, 'C');
    if (!tr && !is(trans, 'N')) { *info = -2; return; }
    if (n < 0) { *info = -3; return; }
    if (k < 0) { *info = -4; return; }
    const int nrowa = tr ? k : n;
    if (lda < (nrowa > 1 ? nrowa : 1)) { *info = -7; return; }
    if (ldc < (n > 1 ? n : 1)) { *info = -10; return; }
    *info = 0;
    if (n == 0) return;
    Ctx &c = ctx();
    if (!call_begin(c, false)) { *info = call_end(c); return; }
    const char tri = is(uplo, 'L') ? 'L' : 'U';
    // C = beta*C + alpha*op(A)*op(A)ᵀ; the kernel covers lower tiles with N·T
    // and upper tiles with T·N, so map the four cases onto those two.
    if (tri == 'L' && !tr)
        gemm<double, double, double>(c, Mfma::F64, 'N', 'T', 'L', n, n, k, alpha, A, lda, A, lda, beta, C, ldc);
    else if (tri == 'U' && tr)
        gemm<double, double, double>(c, Mfma::F64, 'T', 'N', 'U', n, n, k, alpha, A, lda, A, lda, beta, C, ldc);
    else if (tri == 'L' && tr)
        gemm<double, double, double>(c, Mfma::F64, 'T', 'N', 'L', n, n, k, alpha, A, lda, A, lda, beta, C, ldc);
    else
        gemm<double, double, double>(c, Mfma::F64, 'N', 'T', 'U', n, n, k, alpha, A, lda, A, lda, beta, C, ldc);
    *info = call_end(c);
}

void relapack_dtrsm(char side, char uplo, char transa, char diag, int m, int n, const double *A,
                    int lda, double *B, int ldb, int *info) {
    if (!info) return;
    if (!is(side, 'L') && !is(side, 'R')) { *info = -1; return; }
    if (!is(uplo, 'L') && !is(uplo, 'U')) { *info = -2; return; }
    if (!is(transa, 'N') && !is(transa, 'T') && !is(transa, 'C')) { *info = -3; return; }
    if (!is(diag, 'N') && !is(diag, 'U')) { *info = -4; return; }
    if (m < 0) { *info = -5; return; }
    if (n < 0) { *info = -6; return; }
    const int nt = is(side, 'L') ? m : n;
    if (lda < (nt > 1 ? nt : 1)) { *info = -8; return; }
    if (ldb < (m > 1 ? m : 1)) { *info = -10; return; }
    *info = 0;
    if (m == 0 || n == 0) return;
    Ctx &c = ctx();
    if (!call_begin(c, false)) { *info = call_end(c); return; }
    trsm<double, double>(c, Mfma::F64, is(side, 'L') ? 'L' : 'R', is(uplo, 'L') ? 'L' : 'U',
                         is(transa, 'N') ? 'N' : 'T', is(diag, 'U') ? 'U' : 'N', m, n, A, lda, B, ldb);
    *info = call_end(c);
}

// ---- mixed precision ------------------------------------------------------------

static bool prec_ok(int prec) { return prec == 32 || prec == 16 || prec == 'b' || prec == 'B'; }
static Mfma prec_to_mode(int prec) {
    return prec == 16 ? Mfma::F16 : (prec == 32 ? Mfma::F32 : Mfma::BF16);
}

void relapack_dposv_mixed(char uplo, int n, int nrhs, const double *A, int lda, const double *B, int ldb,
                          double *X, int ldx, int prec, int *iter, double *berr, int *info) {
    if (!info) return;
    if (!is(uplo, 'L') && !is(uplo, 'U')) { *info = -1; return; }
    if (n < 0) { *info = -2; return; }
    if (nrhs < 0) { *info = -3; return; }
    if (lda < (n > 1 ? n : 1)) { *info = -5; return; }
    if (ldb < (n > 1 ? n : 1)) { *info = -7; return; }
    if (ldx < (n > 1 ? n : 1)) { *info = -9; return; }
    if (!prec_ok(prec)) { *info = -10; return; }
    *info = 0;
    if (iter) *iter = 0;
    if (berr) *berr = 0.0;
    if (n == 0 || nrhs == 0) return;
    Ctx &c = ctx();
    if (!call_begin(c, false)) { *info = call_end(c); return; }
    int it = 0;
    double be = 0.0;
    const int r = mixed_solve(c, true, is(uplo, 'L') ? 'L' : 'U', n, nrhs, A, lda, nullptr, B, ldb, X, ldx,
                              prec, &it, &be);
    const int e = call_end(c);
    *info = e < 0 ? e : r;
    if (iter) *iter = it;
    if (berr) *berr = be;
}

void relapack_mixed_last(int *sweeps, int *gmres_from, int *gmres_sweeps, int *gmres_steps) {
    const MixedStats st = mixed_last_stats();
    if (sweeps) *sweeps = st.sweeps;
    if (gmres_from) *gmres_from = st.switched_at;
    if (gmres_sweeps) *gmres_sweeps = st.gmres_sweeps;
    if (gmres_steps) *gmres_steps = st.gmres_steps;
}

void relapack_dgesv_mixed(int n, int nrhs, const double *A, int lda, int *ipiv, const double *B, int ldb,
                          double *X, int ldx, int prec, int *iter, double *berr, int *info) {
    if (!info) return;
    if (n < 0) { *info = -1; return; }
    if (nrhs < 0) { *info = -2; return; }
    if (lda < (n > 1 ? n : 1)) { *info = -4; return; }
    if (ldb < (n > 1 ? n : 1)) { *info = -7; return; }
    if (ldx < (n > 1 ? n : 1)) { *info = -9; return; }
    if (!prec_ok(prec)) { *info = -10; return; }
    *info = 0;
    if (iter) *iter = 0;
    if (berr) *berr = 0.0;
    if (n == 0 || nrhs == 0) return;
    Ctx &c = ctx();
    if (!call_begin(c, false)) { *info = call_end(c); return; }
    ensure_rowsrc(c, (size_t)n);
    int it = 0;
    double be = 0.0;
    const int r = mixed_solve(c, false, 'N', n, nrhs, A, lda, ipiv, B, ldb, X, ldx, prec, &it, &be);
    const int e = call_end(c);
    *info = e < 0 ? e : r;
    if (iter) *iter = it;
    if (berr) *berr = be;
}

void relapack_scale_spd_f32(char uplo, int n, const double *A, int lda, double *d, float *S, int lds,
                            int *info) {
    if (!info) return;
    if (!is(uplo, 'L') && !is(uplo, 'U')) { *info = -1; return; }
    if (n < 0) { *info = -2; return; }
    if (lda < (n > 1 ? n : 1)) { *info = -4; return; }
    if (lds < (n > 1 ? n : 1)) { *info = -7; return; }
    *info = 0;
    if (n == 0) return;
    Ctx &c = ctx();
    if (!call_begin(c, false)) { *info = call_end(c); return; }
    scale_spd_f32(c, is(uplo, 'L') ? 'L' : 'U', n, A, lda, d, S, lds);
    *info = call_end(c);
}

void relapack_scale_ge_f32(int n, const double *A, int lda, double *r, double *cs, float *S, int lds,
                           int *info) {
    if (!info) return;
    if (n < 0) { *info = -1; return; }
    if (lda < (n > 1 ? n : 1)) { *info = -3; return; }
    if (lds < (n > 1 ? n : 1)) { *info = -7; return; }
    *info = 0;
    if (n == 0) return;
    Ctx &c = ctx();
    if (!call_begin(c, false)) { *info = call_end(c); return; }
    scale_ge_f32(c, n, A, lda, r, cs, S, lds);
    *info = call_end(c);
}

void relapack_spotrf_lp(char uplo, int n, float *A, int lda, int prec, int *info) {
    if (!info) return;
    if (!is(uplo, 'L') && !is(uplo, 'U')) { *info = -1; return; }
    if (n < 0) { *info = -2; return; }
    if (lda < (n > 1 ? n : 1)) { *info = -4; return; }
    if (!prec_ok(prec)) { *info = -5; return; }
    *info = 0;
    if (n == 0) return;
    Ctx &c = ctx();
    if (!call_begin(c, true)) { *info = call_end(c); return; }
    potrf_rec<float>(c, prec_to_mode(prec), is(uplo, 'L') ? 'L' : 'U', n, A, lda, 0);
    *info = call_end(c);
}

void relapack_sgetrf_lp(int m, int n, float *A, int lda, int *ipiv, int prec, int *info) {
    if (!info) return;
    if (m < 0) { *info = -1; return; }
    if (n < 0) { *info = -2; return; }
    if (lda < (m > 1 ? m : 1)) { *info = -4; return; }
    if (!prec_ok(prec)) { *info = -6; return; }
    *info = 0;
    if (m == 0 || n == 0) return;
    Ctx &c = ctx();
    if (!call_begin(c, false)) { *info = call_end(c); return; }
    ensure_rowsrc(c, (size_t)m);
    getrf_top<float>(c, prec_to_mode(prec), m, n, A, lda, ipiv);
    *info = call_end(c);
}

// ---- FP32 factorizations (FP32 storage, FP32 matrix-core updates) ---------

void relapack_spotrf(char uplo, int n, float *A, int lda, int *info) {
    if (!info) return;
    relapack_spotrf_lp(uplo, n, A, lda, 32, info);
}

void relapack_sgetrf(int m, int n, float *A, int lda, int *ipiv, int *info) {
    if (!info) return;
    relapack_sgetrf_lp(m, n, A, lda, ipiv, 32, info);
}

// ---- batched factorizations ------------------------------------------------

int relapack_dpotrf_batched(char uplo, int count, const int *n, double *const *A, const int *lda, int *info) {
    return rl::potrf_batched_call<double>(uplo, count, n, A, lda, info);
}
int relapack_spotrf_batched(char uplo, int count, const int *n, float *const *A, const int *lda, int *info) {
    return rl::potrf_batched_call<float>(uplo, count, n, A, lda, info);
}
int relapack_dgetrf_batched(int count, const int *n, double *const *A, const int *lda, int *const *ipiv,
                            int *info) {
    return rl::getrf_batched_call<double>(count, n, A, lda, ipiv, info);
}
int relapack_sgetrf_batched(int count, const int *n, float *const *A, const int *lda, int *const *ipiv,
                            int *info) {
    return rl::getrf_batched_call<float>(count, n, A, lda, ipiv, info);
}

// ---- triangular product, inverse, SPD inverse ------------------------------

void relapack_dtrmm(char side, char uplo, char transa, char diag, int m, int n, double alpha,
                    const double *A, int lda, double *B, int ldb, int *info) {
    if (!info) return;
    if (!is(side, 'L') && !is(side, 'R')) { *info = -1; return; }
    if (!is(uplo, 'L') && !is(uplo, 'U')) { *info = -2; return; }
    if (!is(transa, 'N') && !is(transa, 'T') && !is(transa, 'C')) { *info = -3; return; }
    if (!is(diag, 'N') && !is(diag, 'U')) { *info = -4; return; }
    if (m < 0) { *info = -5; return; }
    if (n < 0) { *info = -6; return; }
    const int nrowa = is(side, 'L') ? m : n;
    if (lda < (nrowa > 1 ? nrowa : 1)) { *info = -9; return; }
    if (ldb < (m > 1 ? m : 1)) { *info = -11; return; }
    *info = 0;
    if (m == 0 || n == 0) return;
    Ctx &c = ctx();
    if (!call_begin(c, false)) { *info = call_end(c); return; }
    trmm(c, side, uplo, transa, diag, m, n, alpha, A, lda, B, ldb);
    *info = call_end(c);
}

void relapack_dtrtri(char uplo, char diag, int n, double *A, int lda, int *info) {
    if (!info) return;
    if (!is(uplo, 'L') && !is(uplo, 'U')) { *info = -1; return; }
    if (!is(diag, 'N') && !is(diag, 'U')) { *info = -2; return; }
    if (n < 0) { *info = -3; return; }
    if (lda < (n > 1 ? n : 1)) { *info = -5; return; }
    *info = 0;
    if (n == 0) return;
    Ctx &c = ctx();
    if (!call_begin(c, true)) { *info = call_end(c); return; }
    if (is(diag, 'N')) diag_zero(c, n, A, lda);
    trtri_rec(c, is(uplo, 'L') ? 'L' : 'U', is(diag, 'U') ? 'U' : 'N', n, A, lda);
    *info = call_end(c);
}

void relapack_dlauum(char uplo, int n, double *A, int lda, int *info) {
    if (!info) return;
    if (!is(uplo, 'L') && !is(uplo, 'U')) { *info = -1; return; }
    if (n < 0) { *info = -2; return; }
    if (lda < (n > 1 ? n : 1)) { *info = -4; return; }
    *info = 0;
    if (n == 0) return;
    Ctx &c = ctx();
    if (!call_begin(c, false)) { *info = call_end(c); return; }
    lauum_rec(c, is(uplo, 'L') ? 'L' : 'U', n, A, lda);
    *info = call_end(c);
}

void relapack_dpotri(char uplo, int n, double *A, int lda, int *info) {
    if (!info) return;
    if (!is(uplo, 'L') && !is(uplo, 'U')) { *info = -1; return; }
    if (n < 0) { *info = -2; return; }
    if (lda < (n > 1 ? n : 1)) { *info = -4; return; }
    *info = 0;
    if (n == 0) return;
    Ctx &c = ctx();
    if (!call_begin(c, true)) { *info = call_end(c); return; }
    const char u = is(uplo, 'L') ? 'L' : 'U';
    diag_zero(c, n, A, lda);
    trtri_rec(c, u, 'N', n, A, lda);
    lauum_rec(c, u, n, A, lda);
    *info = call_end(c);
}

// ---- tracing ----------------------------------------------------------------

void relapack_trace_enable(int on) {
    Ctx &c = ctx();
    c.trace = on != 0;
    t_trace.clear();
    t_evused = 0;
}

// Per kernel family k in [0, cap): out[4k..4k+3] = {launches, total ms, flops, bytes}.
// Synchronizes the library stream. Returns the number of families written.
int relapack_trace_collect(double *out, int cap) {
    Ctx &c = ctx();
    if (hipStreamSynchronize(c.stream) != hipSuccess) return -1;
    for (int i = 0; i < 4 * cap; ++i) out[i] = 0.0;
    for (auto &r : t_trace) {
        if (r.kind < 0 || r.kind >= cap) continue;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, r.e0, r.e1) != hipSuccess) ms = 0.f;
        out[4 * r.kind + 0] += 1.0;
        out[4 * r.kind + 1] += ms;
        out[4 * r.kind + 2] += r.flops;
        out[4 * r.kind + 3] += r.bytes;
    }
    t_trace.clear();
    t_evused = 0;
    return cap;
}

// ---- plan mode: the call sequence of one factorization, without launching ---

// routine: "potrf_L", "potrf_U", "getrf", "trtri_L", "trtri_U", "lauum_L" or
// "lauum_U". Writes up to cap records of
// {kind, level, m, n, k} (5 int64 each) into rec; returns the total count.
long long relapack_plan(const char *routine, long long m, long long n, int leaf, long long *rec,
                        long long cap) {
    Ctx &c = ctx();
    std::vector<PlanRec> out;
    Ctx saved = c;
    c.plan = true;
    c.plan_out = &out;
    c.plan_leaf = leaf;
    c.level = 0;
    c.abort_on_info = false;
    std::string r = routine ? routine : "";
    if (r == "potrf_L") potrf_rec<double>(c, Mfma::F64, 'L', n, nullptr, n, 0);
    else if (r == "potrf_U") potrf_rec<double>(c, Mfma::F64, 'U', n, nullptr, n, 0);
    else if (r == "getrf") getrf_top<double>(c, Mfma::F64, m, n, nullptr, m, nullptr);
    else if (r == "trtri_L" || r == "trtri_U") trtri_rec(c, r[6], 'N', n, nullptr, n);
    else if (r == "lauum_L" || r == "lauum_U") lauum_rec(c, r[6], n, nullptr, n);
    else { c = saved; return -1; }
    c = saved;
    for (long long i = 0; i < (long long)out.size() && i < cap; ++i) {
        rec[5 * i + 0] = out[i].kind;
        rec[5 * i + 1] = out[i].level;
        rec[5 * i + 2] = out[i].m;
        rec[5 * i + 3] = out[i].n;
        rec[5 * i + 4] = out[i].k;
    }
    return (long long)out.size();
}

long long relapack_split(long long n) { return split_size(n); }

}  // extern "C"
