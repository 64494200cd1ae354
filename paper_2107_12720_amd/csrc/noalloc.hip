// noalloc.hip -- trim_csr_noalloc: AC-6 trimming of an explicit graph whose
// working memory is a fixed device array of this library, for callers that
// cannot allocate (code under HIP graph capture, tight serving loops, hosts
// that forbid hipMalloc).  The kernels are those of trim_csr with AC-6.
//
// The array, `scratch`, is a file-scope __device__ variable: every GPU the
// library runs on holds its own copy, at its own address, until the process
// ends.  Host code never uses the name `scratch` as an address (in host code
// it is only a stand-in); on the first call on a device, with that device
// current, hipGetSymbolAddress gives that device's copy, which is kept per
// device and passed to the kernels.  Layout (256-byte aligned pieces), for
// n <= TRIM_NOALLOC_MAX_N and at most TRIM_NOALLOC_WORKERS workers:
//   list heads   2n int32        records   n uint64
//   sinks bitmap n/32 + 2 words  queue     6n + 64 * 4 * workers uint32
//   forest links n int32         forest lists 2n uint32
//   split S_more heads 3n int32
//   control      kCtrInts int32  partials  kPartSlots * kPartStride uint64
// about 69 MB in all.  Every call overwrites what it reads before reading it,
// except the queue, whose free slots must hold kNone: the first call on a
// device fills it with a kernel, and every later call leaves it that way
// (consumers restore each slot they take; a call abandoned by the watchdog
// restores the whole queue in its output kernel).  Calls that overlap on one
// GPU share the array and race.
#include <mutex>

#include "trim_internal.h"
#include "trim_device.h"

namespace trim {
namespace {

constexpr long long kWords256 = 32;   // uint64 words per 256 bytes
constexpr long long round256(long long words) {
    return (words + kWords256 - 1) / kWords256 * kWords256;
}
constexpr long long kMaxN = TRIM_NOALLOC_MAX_N;
static_assert(kMaxN <= kSplitMaxN, "the fixed array holds the split S_more heads");
constexpr long long kQueueWordsU32 =
    kQueuePerVertexSplit * kMaxN + 64LL * 4 * TRIM_NOALLOC_WORKERS;
// offsets in uint64 words
constexpr long long kOffHead = 0;
constexpr long long kOffRec = kOffHead + round256(kMaxN);             // 2n int32
constexpr long long kOffSinks = kOffRec + round256(kMaxN);            // n uint64
constexpr long long kOffQueue = kOffSinks + round256(kMaxN / 64 + 2); // n/32 + 2 (+1) uint32
constexpr long long kOffJp = kOffQueue + round256((kQueueWordsU32 + 1) / 2);   // n int32
constexpr long long kOffLists = kOffJp + round256(kMaxN / 2);                     // 2n uint32
constexpr long long kOffExt = kOffLists + round256(kMaxN);   // (kMoreLists - 1) n int32
constexpr long long kOffCtr = kOffExt + round256(((kMoreLists - 1) * kMaxN + 1) / 2);
constexpr long long kOffPart = kOffCtr + round256(kCtrInts / 2);
constexpr long long kScratchWords = kOffPart + round256((long long)kPartSlots * kPartStride);

static __device__ __align__(256) uint64_t scratch[kScratchWords];

// Host-side state per device: the device's address of `scratch`, its CU
// count, and whether its queue has been filled.
constexpr int kMaxDevices = 64;
struct DeviceState {
    uint64_t* base = nullptr;
    int cus = 0;
    bool queue_ready = false;
};
std::mutex g_mu;
DeviceState g_dev[kMaxDevices];

__global__ void fill_none(uint32_t* q, long long words) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < words;
         i += (long long)gridDim.x * blockDim.x)
        q[i] = kNone;
}

int herr(hipError_t e, const char* what) {
    char buf[256];
    snprintf(buf, sizeof buf, "%s: %s", what, hipGetErrorString(e));
    return report_error(TRIM_E_HIP, buf);
}

// Set-up on the current device `dev`: the address of its copy of the array
// (once), and the queue fill (once, enqueued on `s` before the call's own
// kernels).
int setup(int dev, hipStream_t s, DeviceState** out) {
    std::lock_guard<std::mutex> lock(g_mu);
    DeviceState& d = g_dev[dev];
    if (!d.base) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return herr(e, "hipGetSymbolAddress(scratch)");
        int cus = 0;
        if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) !=
            hipSuccess)
            return herr(e, "hipDeviceGetAttribute");
        if (ac6_max_workers_per_cu(256) * cus < TRIM_NOALLOC_WORKERS)
            return report_error(TRIM_E_UNSUPPORTED,
                                "trim_csr_noalloc: this device cannot hold its workers at once");
        d.base = static_cast<uint64_t*>(p);
        d.cus = cus;
    }
    if (!d.queue_ready) {
        hipLaunchKernelGGL(fill_none, dim3(1024), dim3(256), 0, s,
                           reinterpret_cast<uint32_t*>(d.base + kOffQueue), kQueueWordsU32);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return herr(e, "queue fill");
        d.queue_ready = true;
    }
    *out = &d;
    return TRIM_OK;
}

}  // namespace
}  // namespace trim

extern "C" int trim_csr_noalloc(const trim_csr_t* g, const trim_opts_t* o,
                                uint32_t* live_bitmap, uint64_t* worker_edges,
                                trim_stats_t* stats, void* stream) {
    using namespace trim;
    if (!g) return report_error(TRIM_E_INVAL, "trim_csr_noalloc: NULL graph");
    if (g->n < 0 || g->n > TRIM_NOALLOC_MAX_N) {
        char buf[160];
        snprintf(buf, sizeof buf, "trim_csr_noalloc: n = %d outside [0, %d] (its fixed array)",
                 g->n, TRIM_NOALLOC_MAX_N);
        return report_error(TRIM_E_INVAL, buf);
    }
    if (g->m < 0 || g->m >= (int64_t)1 << 31)
        return report_error(TRIM_E_INVAL, "trim_csr_noalloc: m out of range [0, 2^31)");
    if (!g->row_off) return report_error(TRIM_E_INVAL, "row_off is NULL");
    if (g->m > 0 && !g->col) return report_error(TRIM_E_INVAL, "col is NULL");
    if (g->n > 0 && !live_bitmap) return report_error(TRIM_E_INVAL, "live_bitmap is NULL");
    if (!worker_edges) return report_error(TRIM_E_INVAL, "worker_edges is NULL");
    int rc = check_options(o);
    if (!rc && o && o->rounds > 1)
        rc = report_error(TRIM_E_INVAL, "trim_csr_noalloc: opts.rounds must be 0 or 1");
    if (rc) return rc;
    if (o && o->graph) return report_error(TRIM_E_INVAL, "trim_csr_noalloc: opts.graph is 0");
    if (o && o->workers > TRIM_NOALLOC_WORKERS)
        return report_error(TRIM_E_INVAL, "trim_csr_noalloc: opts.workers > TRIM_NOALLOC_WORKERS");
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return herr(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return report_error(TRIM_E_UNSUPPORTED, "device id");
    hipStream_t s = (hipStream_t)stream;
    DeviceState* d = nullptr;
    if ((rc = setup(dev, s, &d))) return rc;
    Work w;
    w.a = reinterpret_cast<int*>(d->base + kOffHead);
    w.b = d->base + kOffRec;
    w.c = reinterpret_cast<int*>(d->base + kOffSinks);
    w.q = reinterpret_cast<uint32_t*>(d->base + kOffQueue);
    w.jp = reinterpret_cast<int*>(d->base + kOffJp);
    w.e = reinterpret_cast<uint32_t*>(d->base + kOffLists);
    w.ext = reinterpret_cast<int*>(d->base + kOffExt);
    w.qwords = kQueueWordsU32;
    w.cap = kMaxN;
    w.ctr = reinterpret_cast<int*>(d->base + kOffCtr);
    w.part = d->base + kOffPart;
    LaunchCfg lc;
    lc.block = (o && o->block) ? o->block : 256;
    lc.chunk = o ? o->chunk : 0;
    lc.schedule = o ? o->schedule : 0;
    lc.workers = (o && o->workers > 0) ? o->workers : TRIM_NOALLOC_WORKERS;
    lc.budget = (o && o->budget > 0) ? o->budget : TRIM_DEFAULT_BUDGET;
    lc.forest = !(o && (o->flags & TRIM_FLAG_STEPWISE));
    lc.cus = d->cus;
    lc.stream = s;
    if (o && o->validate) {
        int bad = 0;
        if ((e = validate_csr(*g, w, s)) != hipSuccess ||
            (e = hipMemcpyAsync(&bad, w.ctr + kBad, sizeof(int), hipMemcpyDeviceToHost, s)) !=
                hipSuccess ||
            (e = hipStreamSynchronize(s)) != hipSuccess)
            return herr(e, "validate");
        if (bad) return report_error(TRIM_E_BADGRAPH, "graph validation found problems");
    }
    e = ac6_csr(*g, w, lc, live_bitmap, worker_edges, stats);
    if (e != hipSuccess) return herr(e, "kernel launch");
    return TRIM_OK;
}
