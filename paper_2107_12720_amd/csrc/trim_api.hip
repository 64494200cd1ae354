// trim_api.hip -- the C ABI of libtrim (include/trim.h): contexts, argument
// checks, working memory and launch sequencing.  All compute is in the kernel
// files; this layer never touches graph data on the host.
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <unordered_map>

#include "trim_internal.h"
#include "scc_internal.h"

static_assert(sizeof(trim_stats_t) == 18 * sizeof(uint64_t), "trim_stats_t layout");
static_assert(sizeof(trim_opts_t) == 9 * sizeof(int32_t), "trim_opts_t layout");

struct trim_ctx {
    int device = 0;
    int cus = 0;
    // device memory held by the context, against its cap (0 = none)
    uint64_t mem_budget = 0;
    uint64_t mem_used = 0;
    std::unordered_map<void*, size_t> sizes;
    size_t cap_n = 0;
    trim::Work w;
    // two-sided AC-6 extras, sized for cap_n2 vertices
    size_t cap_n2 = 0;
    trim::Work2 w2;
    // SCC decomposition arrays, sized for cap_scc vertices
    size_t cap_scc = 0;
    trim::SccWork sw;
    int occ6 = 0, occ4 = 0, occ3 = 0;   // resident workgroups per CU (occ6: both AC-6 forms)
    // captured launch sequence of trim_batch and the arguments it was made for
    hipGraphExec_t gexec = nullptr;
    uint64_t gkey[25] = {};
    trim::Timer timer;
    // tile tables of the preprocessing and reordering kernels
    int* tiles = nullptr;
    long long cap_tiles = 0;
    // per-XCD in-degree copies of trim_mlp_prepare
    int* copies = nullptr;
    long long cap_copies = 0;
    // per-vertex features of trim_mlp_score (float2 per vertex)
    float* vf = nullptr;
    long long cap_vf = 0;
};

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int hip_fail(hipError_t e, const char* what) {
    return fail(TRIM_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

// Every device allocation of a context goes through these two, so the context
// knows what it holds and can refuse what would exceed its cap.
hipError_t dmalloc(trim_ctx* c, void** p, size_t bytes) {
    *p = nullptr;
    if (c->mem_budget && c->mem_used + bytes > c->mem_budget) return hipErrorOutOfMemory;
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        return e;
    }
    c->sizes[*p] = bytes;
    c->mem_used += bytes;
    return hipSuccess;
}
template <class T>
hipError_t dmalloc(trim_ctx* c, T** p, size_t bytes) {
    return dmalloc(c, reinterpret_cast<void**>(p), bytes);
}
void dfree(trim_ctx* c, void* p) {
    if (!p) return;
    auto it = c->sizes.find(p);
    if (it != c->sizes.end()) {
        c->mem_used -= it->second;
        c->sizes.erase(it);
    }
    (void)hipFree(p);
}

void free_work(trim_ctx* c) {
    dfree(c, c->w.a);
    dfree(c, c->w.b);
    dfree(c, c->w.c);
    dfree(c, c->w.d);
    dfree(c, c->w.q);
    dfree(c, c->w.e);
    dfree(c, c->w.ext);
    dfree(c, c->w.hl);
    c->w.hl = nullptr;
    c->w.hcap = 0;
    c->w.q = nullptr;
    c->w.e = nullptr;
    c->w.ext = nullptr;
    c->w.jp = nullptr;
    c->w.a = nullptr;
    c->w.b = nullptr;
    c->w.c = nullptr;
    c->w.d = nullptr;
    c->cap_n = 0;
}

int ensure(trim_ctx* c, int64_t n) {
    size_t need = (size_t)(n > 0 ? n : 1);
    if (need <= c->cap_n) return TRIM_OK;
    free_work(c);
    size_t cap = need + need / 8 + 64;
    // the split S_more lists (and the queue room they need) for graphs that
    // use them
    const bool split = (long long)need <= trim::kSplitMaxN;
    const size_t qslots =
        cap * (split ? trim::kQueuePerVertexSplit : 3) + (size_t)trim::kQueueSlots;
    if (dmalloc(c, &c->w.a, cap * 8) != hipSuccess ||
        dmalloc(c, &c->w.b, cap * 8) != hipSuccess ||
        dmalloc(c, &c->w.c, cap * 4) != hipSuccess ||
        dmalloc(c, &c->w.d, cap * 4) != hipSuccess ||
        dmalloc(c, &c->w.e, cap * 12) != hipSuccess ||
        (split && dmalloc(c, &c->w.ext, cap * 4 * (trim::kMoreLists - 1)) != hipSuccess) ||
        dmalloc(c, &c->w.q, qslots * 4) != hipSuccess ||
        // free queue slots hold kNone (all ones); consumers restore it
        hipMemset(c->w.q, 0xFF, qslots * 4) != hipSuccess) {
        (void)hipGetLastError();
        free_work(c);
        return fail(TRIM_E_NOMEM, "cannot allocate working memory for %lld vertices",
                    (long long)n);
    }
    c->cap_n = cap;
    c->w.cap = (long long)cap;
    c->w.jp = reinterpret_cast<int*>(c->w.e + 2 * cap);   // after the two lists
    c->w.qwords = (long long)qslots;
    return TRIM_OK;
}

// The round list of late support registration (2 ints per vertex) and its
// three round filters, allocated on first use.
int ensure_rounds(trim_ctx* c, int64_t n) {
    const long long need = n > 0 ? n : 1;
    if (need <= c->w.hcap) return TRIM_OK;
    dfree(c, c->w.hl);
    c->w.hl = nullptr;
    c->w.hcap = 0;
    const long long cap = need + need / 8 + 64;
    const size_t filters = 3 * ((size_t)1 << (trim::kRoundFilterMaxLog2 - 5));
    if (dmalloc(c, &c->w.hl, ((size_t)cap * 2 + filters) * sizeof(int)) != hipSuccess) {
        (void)hipGetLastError();
        c->w.hl = nullptr;
        return fail(TRIM_E_NOMEM, "cannot allocate the round lists for %lld vertices",
                    (long long)n);
    }
    c->w.hcap = cap;
    return TRIM_OK;
}

void free_work2(trim_ctx* c) {
    dfree(c, c->w2.hin);
    dfree(c, c->w2.rec_in);
    dfree(c, c->w2.q);
    c->w2 = trim::Work2{};
    c->cap_n2 = 0;
}

// Two-sided AC-6 queue: kQueuePerVertexTwo slots per vertex, or
// kQueuePerVertexTwoSplit where the out-side S_more lists are split (graphs
// up to kSplitMaxN vertices).
int ensure2(trim_ctx* c, int64_t n) {
    size_t need = (size_t)(n > 0 ? n : 1);
    if (need <= c->cap_n2) return TRIM_OK;
    free_work2(c);
    size_t cap = need + need / 8 + 64;
    const size_t per = (long long)need <= trim::kSplitMaxN ? trim::kQueuePerVertexTwoSplit
                                                            : trim::kQueuePerVertexTwo;
    const size_t qbytes = (cap * per + (size_t)trim::kQueueSlots) * 4;
    if (dmalloc(c, &c->w2.hin, cap * 8) != hipSuccess ||
        dmalloc(c, &c->w2.rec_in, cap * 8) != hipSuccess ||
        dmalloc(c, &c->w2.q, qbytes) != hipSuccess ||
        hipMemset(c->w2.q, 0xFF, qbytes) != hipSuccess) {
        (void)hipGetLastError();
        free_work2(c);
        return fail(TRIM_E_NOMEM, "cannot allocate two-sided working memory for %lld vertices",
                    (long long)n);
    }
    c->cap_n2 = cap;
    c->w2.qwords = (long long)(cap * per) + trim::kQueueSlots;
    return TRIM_OK;
}

void free_scc(trim_ctx* c) {
    dfree(c, c->sw.assigned);
    dfree(c, c->sw.live);
    dfree(c, c->sw.flags);
    dfree(c, c->sw.color);
    dfree(c, c->sw.misc);
    dfree(c, c->sw.front[0]);
    dfree(c, c->sw.front[1]);
    dfree(c, c->sw.pre);
    dfree(c, c->sw.bsum);
    c->sw = trim::SccWork{};
    c->cap_scc = 0;
}

int ensure_scc(trim_ctx* c, int64_t n) {
    size_t need = (size_t)(n > 0 ? n : 1);
    if (need <= c->cap_scc) return TRIM_OK;
    free_scc(c);
    size_t cap = need + need / 8 + 64;
    const size_t words = cap / 32 + 64;
    if (dmalloc(c, &c->sw.assigned, words * 4) != hipSuccess ||
        dmalloc(c, &c->sw.live, words * 4) != hipSuccess ||
        dmalloc(c, &c->sw.flags, cap * 4) != hipSuccess ||
        dmalloc(c, &c->sw.color, cap * 4) != hipSuccess ||
        dmalloc(c, &c->sw.misc, trim::kSccMisc * 8) != hipSuccess ||
        dmalloc(c, &c->sw.front[0], (2 * cap + 64) * 4) != hipSuccess ||
        dmalloc(c, &c->sw.front[1], (2 * cap + 64) * 4) != hipSuccess ||
        dmalloc(c, &c->sw.pre, (2 * cap + 64) * 4) != hipSuccess ||
        dmalloc(c, &c->sw.bsum, ((2 * cap + 64) / trim::kScanChunk + 64) * 4) !=
            hipSuccess) {
        (void)hipGetLastError();
        free_scc(c);
        return fail(TRIM_E_NOMEM, "cannot allocate SCC working memory for %lld vertices",
                    (long long)n);
    }
    c->cap_scc = cap;
    return TRIM_OK;
}

int ensure_tiles(trim_ctx* c, long long m) {
    const long long need = trim::tile_scratch_ints(m > 0 ? m : 1);
    if (need <= c->cap_tiles) return TRIM_OK;
    dfree(c, c->tiles);
    c->tiles = nullptr;
    c->cap_tiles = 0;
    const long long cap = need + need / 8 + 64;
    if (dmalloc(c, &c->tiles, (size_t)cap * 4) != hipSuccess) {
        (void)hipGetLastError();
        c->tiles = nullptr;
        return fail(TRIM_E_NOMEM, "cannot allocate tile tables for %lld edges", m);
    }
    c->cap_tiles = cap;
    return TRIM_OK;
}

// AC-3's single cooperative launch is limited to two workgroups per CU.  With
// eight per CU (the occupancy maximum, 2,048 workgroups) the rounds kernel
// stopped making progress; the round barrier needs every workgroup resident,
// and the launch at the occupancy maximum evidently did not give that (the
// barrier protocol itself is checked on the host with the full workgroup
// count).  That configuration stays off: opts.workers above the cap is an
// argument error.  More workgroups only lengthen the barrier anyway: a round
// costs least at one per CU, the default.
constexpr int kAc3MaxPerCu = 2;

int max_workers(const trim_ctx* c, int algo) {
    int per_cu = algo == TRIM_AC6 ? c->occ6 : algo == TRIM_AC4 ? c->occ4 : c->occ3;
    if (algo == TRIM_AC3 && per_cu > kAc3MaxPerCu) per_cu = kAc3MaxPerCu;
    int max_p = per_cu * c->cus;
    if (max_p > trim::kMaxWorkers) max_p = trim::kMaxWorkers;
    return max_p < 1 ? 1 : max_p;
}

int workers_for(trim_ctx* c, int algo, const trim_opts_t* o) {
    int per_cu = algo == TRIM_AC6 ? c->occ6 : algo == TRIM_AC4 ? c->occ4 : c->occ3;
    int def = (algo == TRIM_AC3 ? 1 : (per_cu < 2 ? per_cu : 2)) * c->cus;
    int p = (o && o->workers > 0) ? o->workers : def;
    const int max_p = max_workers(c, algo);
    if (p > max_p) p = max_p;   // only the default can exceed it; check_workers refuses more
    if (p < 1) p = 1;
    return p;
}

int check_workers(trim_ctx* c, int algo, const trim_opts_t* o) {
    if (o && o->workers > max_workers(c, algo))
        return fail(TRIM_E_INVAL, "opts.workers = %d exceeds the limit %d for AC-%d", o->workers,
                    max_workers(c, algo), algo);
    return TRIM_OK;
}

int check_opts(const trim_opts_t* o) {
    if (!o) return TRIM_OK;
    if (o->block != 0 && (o->block < 64 || o->block > 1024 || o->block % 64 != 0))
        return fail(TRIM_E_INVAL, "opts.block must be 0 or a multiple of 64 in [64, 1024]");
    if (o->workers < 0) return fail(TRIM_E_INVAL, "opts.workers must be >= 0");
    if (o->chunk < 0 || o->chunk > (1 << 24))
        return fail(TRIM_E_INVAL, "opts.chunk must be in [0, 2^24]");
    if (o->graph != 0 && o->graph != 1) return fail(TRIM_E_INVAL, "opts.graph must be 0 or 1");
    if (o->schedule & ~(TRIM_SCHED_REVERSE | TRIM_SCHED_JITTER))
        return fail(TRIM_E_INVAL, "opts.schedule has unknown bits");
    if (o->budget < 0) return fail(TRIM_E_INVAL, "opts.budget must be >= 0");
    if (o->flags & ~(TRIM_FLAG_STEPWISE | TRIM_FLAG_BATCH_UNION | TRIM_FLAG_FOREST))
        return fail(TRIM_E_INVAL, "opts.flags has unknown bits");
    if (o->rounds < 0 || o->rounds > TRIM_MAX_ROUNDS)
        return fail(TRIM_E_INVAL, "opts.rounds must be in [0, %d]", TRIM_MAX_ROUNDS);
    return TRIM_OK;
}

// opts.rounds >= 2 (late support registration) is for one-sided AC-6 on one
// graph only.
int check_rounds(const trim_opts_t* o, int algo, bool allowed, const char* call) {
    if (o && o->rounds > 1 && (!allowed || algo != TRIM_AC6))
        return fail(TRIM_E_INVAL, "%s: opts.rounds = %d needs AC-6 on trim_csr or trim_implicit "
                    "(0 or 1 here)", call, o->rounds);
    return TRIM_OK;
}

trim::LaunchCfg launch_cfg(trim_ctx* c, int algo, const trim_opts_t* o, void* stream) {
    trim::LaunchCfg lc;
    lc.block = (o && o->block) ? o->block : 256;
    lc.chunk = o ? o->chunk : 0;
    lc.schedule = o ? o->schedule : 0;
    lc.workers = workers_for(c, algo, o);
    lc.budget = (o && o->budget > 0) ? o->budget : TRIM_DEFAULT_BUDGET;
    lc.forest = !(o && (o->flags & TRIM_FLAG_STEPWISE));
    lc.rounds = o ? o->rounds : 0;
    lc.cus = c->cus;
    lc.stream = (hipStream_t)stream;
    if (c->timer.keep > 0) lc.timer = c->timer.next();
    return lc;
}

__global__ void validate_kernel(const int* row_off, const int* col, int n, long long m,
                                int* bad) {
    int errs = 0;
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    const int stride = gridDim.x * blockDim.x;
    if (tid == 0 && (row_off[0] != 0 || (long long)row_off[n] != m)) errs++;
    for (int v = tid; v < n; v += stride)
        if (row_off[v] > row_off[v + 1]) errs++;
    for (long long e = tid; e < m; e += stride) {
        const int w = col[e];
        if (w < 0 || w >= n) errs++;
    }
    if (errs) atomicAdd(bad, errs);
}

}  // namespace

namespace trim {
// Error reporting and option checks for the entry points in other files.
int report_error(int code, const char* msg) { return fail(code, "%s", msg); }
int check_options(const trim_opts_t* o) { return check_opts(o); }

hipError_t validate_csr(const trim_csr_t& g, const Work& w, hipStream_t s) {
    hipError_t e = hipMemsetAsync(w.ctr + kBad, 0, sizeof(int), s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(validate_kernel, dim3(1024), dim3(256), 0, s, g.row_off, g.col, g.n,
                       (long long)g.m, w.ctr + kBad);
    if (g.rrow_off && g.rcol)
        hipLaunchKernelGGL(validate_kernel, dim3(1024), dim3(256), 0, s, g.rrow_off, g.rcol, g.n,
                           (long long)g.m, w.ctr + kBad);
    return hipGetLastError();
}
}  // namespace trim

namespace {
// opts.validate: the device check of offsets and targets (of G^T too when
// given), read back synchronously.
int validate_graph(trim_ctx* c, const trim_csr_t& g, hipStream_t s) {
    int bad = 0;
    hipError_t e = trim::validate_csr(g, c->w, s);
    if (e != hipSuccess) return hip_fail(e, "validate");
    if ((e = hipMemcpyAsync(&bad, c->w.ctr + trim::kBad, sizeof(int), hipMemcpyDeviceToHost, s)) !=
            hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
        return hip_fail(e, "validate readback");
    if (bad) return fail(TRIM_E_BADGRAPH, "graph validation found %d problems", bad);
    return TRIM_OK;
}
}  // namespace

extern "C" {

int trim_version(void) { return TRIM_ABI_VERSION; }

const char* trim_last_error(void) { return g_err.c_str(); }

int trim_ctx_create(trim_ctx** out, int device, uint64_t mem_budget) {
    if (!out) return fail(TRIM_E_INVAL, "trim_ctx_create: out is NULL");
    *out = nullptr;
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
    if (device < 0 || device >= ndev)
        return fail(TRIM_E_INVAL, "device %d out of range (%d devices)", device, ndev);
    if ((e = hipSetDevice(device)) != hipSuccess) return hip_fail(e, "hipSetDevice");
    hipDeviceProp_t prop;
    if ((e = hipGetDeviceProperties(&prop, device)) != hipSuccess)
        return hip_fail(e, "hipGetDeviceProperties");
    trim_ctx* c = new trim_ctx;
    c->device = device;
    c->mem_budget = mem_budget;
    c->cus = prop.multiProcessorCount;
    c->occ6 = trim::ac6_max_workers_per_cu(256);
    {
        const int occ6t = trim::ac6_two_max_workers_per_cu(256);
        if (occ6t < c->occ6) c->occ6 = occ6t;
    }
    c->occ4 = trim::ac4_max_workers_per_cu(256);
    c->occ3 = trim::ac3_max_workers_per_cu(256);
    if ((e = dmalloc(c, &c->w.ctr, trim::kCtrInts * sizeof(int))) != hipSuccess ||
        (e = dmalloc(c, &c->w.wedges, trim::kMaxWorkers * sizeof(uint64_t))) !=
            hipSuccess ||
        (e = dmalloc(c, &c->w.part,
                       (size_t)trim::kPartSlots * trim::kPartStride * sizeof(uint64_t))) !=
            hipSuccess) {
        dfree(c, c->w.ctr);
        dfree(c, c->w.wedges);
        delete c;
        return fail(TRIM_E_NOMEM, "cannot allocate control block (%llu bytes cap): %s",
                    (unsigned long long)mem_budget, hipGetErrorString(e));
    }
    *out = c;
    return TRIM_OK;
}

int trim_ctx_destroy(trim_ctx* c) {
    if (!c) return TRIM_OK;
    (void)hipSetDevice(c->device);
    free_work(c);
    free_work2(c);
    free_scc(c);
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    for (auto& sl : c->timer.slot)
        for (auto& ev : sl.ev)
            if (ev) (void)hipEventDestroy(ev);
    dfree(c, c->w.ctr);
    dfree(c, c->w.wedges);
    dfree(c, c->w.part);
    dfree(c, c->tiles);
    dfree(c, c->copies);
    dfree(c, c->vf);
    delete c;
    return TRIM_OK;
}

int trim_num_workers(trim_ctx* c, int algo, const trim_opts_t* o, int32_t* P) {
    if (!c || !P) return fail(TRIM_E_INVAL, "trim_num_workers: NULL argument");
    if (algo != TRIM_AC3 && algo != TRIM_AC4 && algo != TRIM_AC6)
        return fail(TRIM_E_INVAL, "unknown algorithm %d", algo);
    int rc = check_opts(o);
    if (rc || (rc = check_workers(c, algo, o))) return rc;
    *P = workers_for(c, algo, o);
    return TRIM_OK;
}

int trim_max_workers(trim_ctx* c, int algo, int32_t* P) {
    if (!c || !P) return fail(TRIM_E_INVAL, "trim_max_workers: NULL argument");
    if (algo != TRIM_AC3 && algo != TRIM_AC4 && algo != TRIM_AC6)
        return fail(TRIM_E_INVAL, "unknown algorithm %d", algo);
    *P = max_workers(c, algo);
    return TRIM_OK;
}

int trim_ctx_mem_used(trim_ctx* c, uint64_t* bytes) {
    if (!c || !bytes) return fail(TRIM_E_INVAL, "trim_ctx_mem_used: NULL argument");
    *bytes = c->mem_used;
    return TRIM_OK;
}

int trim_ctx_status(trim_ctx* c, void* stream) {
    if (!c) return fail(TRIM_E_INVAL, "trim_ctx_status: NULL context");
    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    int stalled = 0;
    hipStream_t s = (hipStream_t)stream;
    if ((e = hipMemcpyAsync(&stalled, c->w.ctr + trim::kStall, sizeof(int),
                            hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
        return hip_fail(e, "trim_ctx_status");
    if (stalled)
        return fail(TRIM_E_STALLED, "the last call exceeded its step budget and was abandoned");
    return TRIM_OK;
}

int trim_csr(trim_ctx* c, int algo, const trim_csr_t* g, const trim_opts_t* o,
             uint32_t* live_bitmap, uint64_t* worker_edges, trim_stats_t* stats, void* stream) {
    if (!c || !g) return fail(TRIM_E_INVAL, "trim_csr: NULL context or graph");
    if (algo != TRIM_AC3 && algo != TRIM_AC4 && algo != TRIM_AC6)
        return fail(TRIM_E_INVAL, "unknown algorithm %d", algo);
    if (g->n < 0 || g->n > (1 << 29)) return fail(TRIM_E_INVAL, "n = %d out of range", g->n);
    if (g->m < 0 || g->m >= (int64_t)1 << 31)
        return fail(TRIM_E_INVAL, "m = %lld out of range [0, 2^31)", (long long)g->m);
    if (!g->row_off) return fail(TRIM_E_INVAL, "row_off is NULL");
    if (g->m > 0 && !g->col) return fail(TRIM_E_INVAL, "col is NULL");
    if (g->n > 0 && !live_bitmap) return fail(TRIM_E_INVAL, "live_bitmap is NULL");
    if (!worker_edges) return fail(TRIM_E_INVAL, "worker_edges is NULL");
    if (algo == TRIM_AC4 && (!g->rrow_off || (g->m > 0 && !g->rcol)))
        return fail(TRIM_E_INVAL, "AC-4 needs the transposed graph (rrow_off, rcol)");
    int rc = check_opts(o);
    if (!rc) rc = check_rounds(o, algo, true, "trim_csr");
    if (rc || (rc = check_workers(c, algo, o))) return rc;
    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    if ((rc = ensure(c, g->n))) return rc;
    if (algo == TRIM_AC6 && o && o->rounds > 1 && (rc = ensure_rounds(c, g->n))) return rc;
    trim::LaunchCfg lc = launch_cfg(c, algo, o, stream);
    if (o && o->validate && (rc = validate_graph(c, *g, lc.stream))) return rc;
    switch (algo) {
        case TRIM_AC6: e = trim::ac6_csr(*g, c->w, lc, live_bitmap, worker_edges, stats); break;
        case TRIM_AC4: e = trim::ac4_csr(*g, c->w, lc, live_bitmap, worker_edges, stats); break;
        default: e = trim::ac3_csr(*g, c->w, lc, live_bitmap, worker_edges, stats); break;
    }
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    return TRIM_OK;
}

int trim_csr_preset(trim_ctx* c, int algo, const trim_csr_t* g, const uint32_t* preset_dead,
                    const trim_opts_t* o, uint32_t* live_bitmap, uint64_t* worker_edges,
                    trim_stats_t* stats, void* stream) {
    if (!c || !g) return fail(TRIM_E_INVAL, "trim_csr_preset: NULL context or graph");
    if (g && g->n > 0 && !preset_dead) return fail(TRIM_E_INVAL, "preset_dead is NULL");
    if (g->n == 0) preset_dead = nullptr;
    if (algo != TRIM_AC3 && algo != TRIM_AC4 && algo != TRIM_AC6)
        return fail(TRIM_E_INVAL, "unknown algorithm %d", algo);
    if (g->n < 0 || g->n > (1 << 29)) return fail(TRIM_E_INVAL, "n = %d out of range", g->n);
    if (g->m < 0 || g->m >= (int64_t)1 << 31)
        return fail(TRIM_E_INVAL, "m = %lld out of range [0, 2^31)", (long long)g->m);
    if (!g->row_off) return fail(TRIM_E_INVAL, "row_off is NULL");
    if (g->m > 0 && !g->col) return fail(TRIM_E_INVAL, "col is NULL");
    if (g->n > 0 && !live_bitmap) return fail(TRIM_E_INVAL, "live_bitmap is NULL");
    if (!worker_edges) return fail(TRIM_E_INVAL, "worker_edges is NULL");
    if (algo == TRIM_AC4 && (!g->rrow_off || (g->m > 0 && !g->rcol)))
        return fail(TRIM_E_INVAL, "AC-4 needs the transposed graph (rrow_off, rcol)");
    int rc = check_opts(o);
    if (!rc) rc = check_rounds(o, algo, false, "trim_csr_preset");
    if (rc || (rc = check_workers(c, algo, o))) return rc;
    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    if ((rc = ensure(c, g->n))) return rc;
    trim::LaunchCfg lc = launch_cfg(c, algo, o, stream);
    if (o && o->validate && (rc = validate_graph(c, *g, lc.stream))) return rc;
    switch (algo) {
        case TRIM_AC6:
            e = trim::ac6_csr(*g, c->w, lc, live_bitmap, worker_edges, stats, preset_dead);
            break;
        case TRIM_AC4:
            e = trim::ac4_csr(*g, c->w, lc, live_bitmap, worker_edges, stats, preset_dead);
            break;
        default:
            e = trim::ac3_csr(*g, c->w, lc, live_bitmap, worker_edges, stats, preset_dead);
            break;
    }
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    return TRIM_OK;
}

int trim_scc(trim_ctx* c, const trim_csr_t* g, const trim_opts_t* o, int32_t* label,
             trim_scc_stats_t* stats, void* stream) {
    if (!c || !g) return fail(TRIM_E_INVAL, "trim_scc: NULL context or graph");
    if (g->n < 0 || g->n > (1 << 29)) return fail(TRIM_E_INVAL, "n = %d out of range", g->n);
    if (g->m < 0 || g->m >= (int64_t)1 << 31)
        return fail(TRIM_E_INVAL, "m = %lld out of range [0, 2^31)", (long long)g->m);
    if (!g->row_off || !g->rrow_off) return fail(TRIM_E_INVAL, "row_off or rrow_off is NULL");
    if (g->m > 0 && (!g->col || !g->rcol)) return fail(TRIM_E_INVAL, "col or rcol is NULL");
    if (g->n > 0 && !label) return fail(TRIM_E_INVAL, "label is NULL");
    int rc = check_opts(o);
    if (!rc) rc = check_rounds(o, TRIM_AC6, false, "trim_scc");
    if (rc || (rc = check_workers(c, TRIM_AC6, o))) return rc;
    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    if ((rc = ensure(c, g->n)) || (rc = ensure2(c, g->n)) || (rc = ensure_scc(c, g->n))) return rc;
    trim::LaunchCfg lc = launch_cfg(c, TRIM_AC6, o, stream);
    lc.timer = nullptr;   // many launches; timed as a whole by the caller
    if (o && o->validate && (rc = validate_graph(c, *g, lc.stream))) return rc;
    trim::SccCounts k;
    e = trim::scc_run(*g, c->w, c->w2, c->sw, lc, label, &k);
    if (e != hipSuccess) return hip_fail(e, "SCC decomposition");
    if (k.stalled) return fail(TRIM_E_STALLED, "SCC decomposition made no progress");
    if (stats) {
        stats->n_scc = k.n_scc;
        stats->trimmed = k.trimmed;
        stats->giant = k.giant;
        stats->trims = k.trims;
        stats->color_rounds = k.color_rounds;
        stats->color_sweeps = k.color_sweeps;
        stats->search_levels = k.search_levels;
        stats->search_edges = k.search_edges;
        stats->search_ors = k.search_ors;
        stats->trim_ms = k.trim_ms;
        stats->search_ms = k.search_ms;
        stats->color_ms = k.color_ms;
        stats->paired = k.paired;
        stats->size2_ms = k.size2_ms;
    }
    return TRIM_OK;
}

int trim_size2(trim_ctx* c, const trim_csr_t* g, const uint32_t* preset_dead, int32_t* partner,
               int64_t* n_paired, void* stream) {
    if (!c || !g) return fail(TRIM_E_INVAL, "trim_size2: NULL context or graph");
    if (g->n < 0 || g->n > (1 << 29)) return fail(TRIM_E_INVAL, "n = %d out of range", g->n);
    if (g->m < 0 || g->m >= (int64_t)1 << 31)
        return fail(TRIM_E_INVAL, "m = %lld out of range [0, 2^31)", (long long)g->m);
    if (!g->row_off || !g->rrow_off) return fail(TRIM_E_INVAL, "row_off or rrow_off is NULL");
    if (g->m > 0 && (!g->col || !g->rcol)) return fail(TRIM_E_INVAL, "col or rcol is NULL");
    if (g->n > 0 && !partner) return fail(TRIM_E_INVAL, "partner is NULL");
    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    int rc;
    if ((rc = ensure_scc(c, g->n))) return rc;
    long long np = 0;
    e = trim::size2_run(*g, c->sw, preset_dead, partner, n_paired ? &np : nullptr,
                        (hipStream_t)stream, c->cus);
    if (e != hipSuccess) return hip_fail(e, "size-2 check");
    if (n_paired) *n_paired = np;
    return TRIM_OK;
}

int trim_csr_two_sided(trim_ctx* c, int algo, const trim_csr_t* g, const trim_opts_t* o,
                       uint32_t* live_bitmap, uint64_t* worker_edges, trim_stats_t* stats,
                       void* stream) {
    if (!c || !g) return fail(TRIM_E_INVAL, "trim_csr_two_sided: NULL context or graph");
    if (algo != TRIM_AC3 && algo != TRIM_AC4 && algo != TRIM_AC6)
        return fail(TRIM_E_INVAL, "unknown algorithm %d", algo);
    if (g->n < 0 || g->n > (1 << 29)) return fail(TRIM_E_INVAL, "n = %d out of range", g->n);
    if (g->m < 0 || g->m >= (int64_t)1 << 31)
        return fail(TRIM_E_INVAL, "m = %lld out of range [0, 2^31)", (long long)g->m);
    if (!g->row_off || !g->rrow_off) return fail(TRIM_E_INVAL, "row_off or rrow_off is NULL");
    if (g->m > 0 && (!g->col || !g->rcol)) return fail(TRIM_E_INVAL, "col or rcol is NULL");
    if (g->n > 0 && !live_bitmap) return fail(TRIM_E_INVAL, "live_bitmap is NULL");
    if (!worker_edges) return fail(TRIM_E_INVAL, "worker_edges is NULL");
    int rc = check_opts(o);
    if (!rc) rc = check_rounds(o, algo, false, "trim_csr_two_sided");
    if (rc || (rc = check_workers(c, algo, o))) return rc;
    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    if ((rc = ensure(c, g->n))) return rc;
    if (algo != TRIM_AC4 && (rc = ensure2(c, g->n))) return rc;
    trim::LaunchCfg lc = launch_cfg(c, algo, o, stream);
    if (o && o->validate && (rc = validate_graph(c, *g, lc.stream))) return rc;
    e = algo == TRIM_AC6   ? trim::ac6_two_csr(*g, c->w, c->w2, lc, live_bitmap, worker_edges, stats)
        : algo == TRIM_AC4 ? trim::ac4_two_csr(*g, c->w, lc, live_bitmap, worker_edges, stats)
                           : trim::ac3_two_csr(*g, c->w, c->w2, lc, live_bitmap, worker_edges, stats);
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    return TRIM_OK;
}

int trim_implicit(trim_ctx* c, int algo, const trim_implicit_t* g, const trim_opts_t* o,
                  uint32_t* live_bitmap, uint64_t* worker_edges, trim_stats_t* stats,
                  void* stream) {
    if (!c || !g) return fail(TRIM_E_INVAL, "trim_implicit: NULL context or graph");
    if (algo == TRIM_AC4)
        return fail(TRIM_E_UNSUPPORTED,
                    "AC-4 needs the transposed graph and cannot run on an implicit graph");
    if (algo != TRIM_AC3 && algo != TRIM_AC6)
        return fail(TRIM_E_INVAL, "unknown algorithm %d", algo);
    if (g->log2n < 1 || g->log2n > 29)
        return fail(TRIM_E_INVAL, "log2n = %d out of range [1, 29]", g->log2n);
    if (!g->deg_table) return fail(TRIM_E_INVAL, "deg_table is NULL");
    if (!live_bitmap || !worker_edges) return fail(TRIM_E_INVAL, "NULL output");
    int rc = check_opts(o);
    if (!rc) rc = check_rounds(o, algo, true, "trim_implicit");
    if (rc || (rc = check_workers(c, algo, o))) return rc;
    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    if ((rc = ensure(c, (int64_t)1 << g->log2n))) return rc;
    if (algo == TRIM_AC6 && o && o->rounds > 1 &&
        (rc = ensure_rounds(c, (int64_t)1 << g->log2n)))
        return rc;
    trim::LaunchCfg lc = launch_cfg(c, algo, o, stream);
    // implicit graphs: the forest collapse only on request (see the header)
    lc.forest = o && (o->flags & TRIM_FLAG_FOREST) && !(o->flags & TRIM_FLAG_STEPWISE);
    e = algo == TRIM_AC6 ? trim::ac6_implicit(*g, c->w, lc, live_bitmap, worker_edges, stats)
                         : trim::ac3_implicit(*g, c->w, lc, live_bitmap, worker_edges, stats);
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    return TRIM_OK;
}

int trim_batch(trim_ctx* c, int32_t G, const int64_t* vbase, const int32_t* row_off,
               const int32_t* col, int64_t total_n, int64_t total_m, const int64_t* bitmap_base,
               const trim_opts_t* o, uint32_t* live_bitmaps, uint64_t* graph_edges,
               trim_stats_t* stats, void* stream) {
    if (!c) return fail(TRIM_E_INVAL, "trim_batch: NULL context");
    if (G < 1) return fail(TRIM_E_INVAL, "G = %d must be >= 1", G);
    if (!vbase || !row_off || !bitmap_base || !live_bitmaps || !graph_edges)
        return fail(TRIM_E_INVAL, "trim_batch: NULL array");
    if (total_n < 0 || total_n > (1 << 29) || total_m < 0 || total_m >= (int64_t)1 << 31)
        return fail(TRIM_E_INVAL, "batch sizes out of range");
    if (total_m > 0 && !col) return fail(TRIM_E_INVAL, "col is NULL");
    int rc = check_opts(o);
    if (!rc) rc = check_rounds(o, TRIM_AC6, false, "trim_batch");
    if (rc || (rc = check_workers(c, TRIM_AC6, o))) return rc;
    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    if ((rc = ensure(c, total_n > G ? total_n : G))) return rc;
    trim::LaunchCfg lc = launch_cfg(c, TRIM_AC6, o, stream);
    if (o && o->graph) lc.timer = nullptr;   // no event records inside a captured graph
    const bool uni = o && (o->flags & TRIM_FLAG_BATCH_UNION);
    // the owned path sizes its grid from its own occupancy unless workers are given
    trim::LaunchCfg lco = lc;
    lco.workers = (o && o->workers > 0) ? o->workers : 0;
    auto run = [&]() {
        return uni ? trim::ac6_batch(G, vbase, row_off, col, total_n, bitmap_base, c->w, lc,
                                     live_bitmaps, graph_edges, stats)
                   : trim::ac6_batch_owned(G, vbase, row_off, col, total_n, bitmap_base, c->w,
                                           lco, live_bitmaps, graph_edges, stats);
    };
    if (!(o && o->graph)) {
        e = run();
        if (e != hipSuccess) return hip_fail(e, "kernel launch");
        return TRIM_OK;
    }
    if (!stream) return fail(TRIM_E_INVAL, "opts.graph needs a non-NULL stream");
    const uint64_t key[25] = {(uint64_t)G, (uint64_t)vbase, (uint64_t)row_off, (uint64_t)col,
                              (uint64_t)total_n, (uint64_t)total_m, (uint64_t)bitmap_base,
                              (uint64_t)live_bitmaps, (uint64_t)graph_edges, (uint64_t)stats,
                              (uint64_t)stream, (uint64_t)lc.block,
                              (uint64_t)lc.chunk | ((uint64_t)lc.schedule << 32),
                              (uint64_t)lc.workers, (uint64_t)c->w.a, (uint64_t)c->w.b,
                              (uint64_t)c->w.c, (uint64_t)c->w.d, (uint64_t)c->w.q,
                              (uint64_t)c->w.part, (uint64_t)c->w.ctr, (uint64_t)c->w.wedges,
                              (uint64_t)c->w.e, (uint64_t)lc.forest | ((uint64_t)lc.budget << 1),
                              1u | ((uint64_t)uni << 1)};
    if (!c->gexec || memcmp(key, c->gkey, sizeof key) != 0) {
        if (c->gexec) {
            (void)hipGraphExecDestroy(c->gexec);
            c->gexec = nullptr;
        }
        hipGraph_t graph = nullptr;
        if ((e = hipStreamBeginCapture(lc.stream, hipStreamCaptureModeThreadLocal)) != hipSuccess)
            return hip_fail(e, "hipStreamBeginCapture");
        hipError_t le = run();
        e = hipStreamEndCapture(lc.stream, &graph);
        if (le != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            return hip_fail(le, "kernel launch during capture");
        }
        if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
        e = hipGraphInstantiate(&c->gexec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) {
            c->gexec = nullptr;
            return hip_fail(e, "hipGraphInstantiate");
        }
        memcpy(c->gkey, key, sizeof key);
    }
    if ((e = hipGraphLaunch(c->gexec, lc.stream)) != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    return TRIM_OK;
}

namespace {
int check_graph(trim_ctx* c, const trim_csr_t* g, const char* who) {
    if (!c || !g) return fail(TRIM_E_INVAL, "%s: NULL context or graph", who);
    if (g->n < 0 || g->n > (1 << 29)) return fail(TRIM_E_INVAL, "%s: n out of range", who);
    if (g->m < 0 || g->m >= (int64_t)1 << 31) return fail(TRIM_E_INVAL, "%s: m out of range", who);
    if (!g->row_off || (g->m > 0 && !g->col)) return fail(TRIM_E_INVAL, "%s: NULL CSR", who);
    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    return TRIM_OK;
}
int launched(hipError_t e) { return e == hipSuccess ? TRIM_OK : hip_fail(e, "kernel launch"); }
}  // namespace

int trim_mlp_prepare(trim_ctx* c, const trim_csr_t* g, int32_t* indeg, int32_t* src,
                     void* stream) {
    int rc = check_graph(c, g, "trim_mlp_prepare");
    if (rc) return rc;
    if (!indeg || (g->m > 0 && !src)) return fail(TRIM_E_INVAL, "trim_mlp_prepare: NULL output");
    if ((rc = ensure_tiles(c, g->m))) return rc;
    int* copies = nullptr;
    if (g->n <= trim::kXcdCopiesMaxN) {
        const long long need = (long long)trim::kXcdCopies * (g->n > 0 ? g->n : 1);
        if (need > c->cap_copies) {
            dfree(c, c->copies);
            c->copies = nullptr;
            c->cap_copies = 0;
            if (dmalloc(c, &c->copies, (size_t)need * 4) != hipSuccess) {
                (void)hipGetLastError();
                c->copies = nullptr;
                return fail(TRIM_E_NOMEM, "cannot allocate in-degree copies for %d vertices",
                            g->n);
            }
            c->cap_copies = need;
        }
        copies = c->copies;
    }
    return launched(trim::mlp_prepare(g->row_off, g->col, g->n, g->m, indeg, src, c->tiles,
                                      copies, (hipStream_t)stream));
}

int trim_mlp_grad(trim_ctx* c, const trim_csr_t* g, const int32_t* indeg, const int32_t* src,
                  const uint32_t* live_bitmap, const uint16_t* params_bf16,
                  const int64_t* edge_ids, int64_t count, uint64_t seed, int32_t step,
                  float* grad, void* stream) {
    int rc = check_graph(c, g, "trim_mlp_grad");
    if (rc) return rc;
    if (!indeg || !src || !live_bitmap || !params_bf16 || !grad)
        return fail(TRIM_E_INVAL, "trim_mlp_grad: NULL argument");
    if (count < 1 || g->m < 1) return fail(TRIM_E_INVAL, "trim_mlp_grad: no edges to sample");
    return launched(trim::mlp_grad_launch(g->row_off, g->col, indeg, src, g->m, live_bitmap,
                                          (const short*)params_bf16, (const long long*)edge_ids,
                                          count, seed, step, grad, c->cus, (hipStream_t)stream));
}

int trim_mlp_adam(trim_ctx* c, float* params, uint16_t* params_bf16, float* adam_m,
                  float* adam_v, float* grad, float lr, float beta1, float beta2, float eps,
                  int32_t step, void* stream) {
    if (!c || !params || !params_bf16 || !adam_m || !adam_v || !grad)
        return fail(TRIM_E_INVAL, "trim_mlp_adam: NULL argument");
    if (step < 1 || !(lr > 0.f) || !(beta1 >= 0.f && beta1 < 1.f) ||
        !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
        return fail(TRIM_E_INVAL, "trim_mlp_adam: bad hyper-parameters");
    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    return launched(trim::mlp_adam_launch(params, (short*)params_bf16, adam_m, adam_v, grad, lr,
                                          beta1, beta2, eps, step, (hipStream_t)stream));
}

int trim_mlp_score(trim_ctx* c, const trim_csr_t* g, const int32_t* indeg, const int32_t* src,
                   const uint16_t* params_bf16, float* scores, void* stream) {
    int rc = check_graph(c, g, "trim_mlp_score");
    if (rc) return rc;
    if (!indeg || (g->m > 0 && (!src || !scores)) || !params_bf16)
        return fail(TRIM_E_INVAL, "trim_mlp_score: NULL argument");
    const long long need = 2LL * (g->n > 0 ? g->n : 1);   // float2 per vertex
    if (need > c->cap_vf) {
        dfree(c, c->vf);
        c->vf = nullptr;
        c->cap_vf = 0;
        if (dmalloc(c, &c->vf, (size_t)need * 4) != hipSuccess) {
            (void)hipGetLastError();
            c->vf = nullptr;
            return fail(TRIM_E_NOMEM, "cannot allocate vertex features for %d vertices", g->n);
        }
        c->cap_vf = need;
    }
    return launched(trim::mlp_score_launch(g->row_off, g->col, indeg, src, g->n, g->m,
                                           (const short*)params_bf16, scores,
                                           reinterpret_cast<float2*>(c->vf), c->cus,
                                           (hipStream_t)stream));
}

int trim_edge_keys(trim_ctx* c, const trim_csr_t* g, int32_t kind, uint64_t seed, float* keys,
                   void* stream) {
    int rc = check_graph(c, g, "trim_edge_keys");
    if (rc) return rc;
    if (kind != 0 && kind != 1) return fail(TRIM_E_INVAL, "trim_edge_keys: kind must be 0 or 1");
    if (g->m > 0 && !keys) return fail(TRIM_E_INVAL, "trim_edge_keys: NULL keys");
    return launched(
        trim::edge_keys_launch(g->row_off, g->col, g->m, kind, seed, keys, (hipStream_t)stream));
}

int trim_order_by_key(trim_ctx* c, const trim_csr_t* g, const float* keys, float lo, float hi,
                      int32_t* col_out, void* stream) {
    int rc = check_graph(c, g, "trim_order_by_key");
    if (rc) return rc;
    if (g->m > 0 && (!keys || !col_out)) return fail(TRIM_E_INVAL, "trim_order_by_key: NULL");
    if (col_out == g->col) return fail(TRIM_E_INVAL, "trim_order_by_key: col_out aliases col");
    if ((rc = ensure_tiles(c, g->m))) return rc;
    const long long T = (g->m + trim::kTileE - 1) / trim::kTileE;
    return launched(trim::order_launch(g->row_off, g->col, g->n, g->m, keys, lo, hi, col_out,
                                       c->tiles, c->tiles + 3 * T, (hipStream_t)stream));
}

int trim_ctx_set_timing(trim_ctx* c, int enable) {
    if (!c) return fail(TRIM_E_INVAL, "trim_ctx_set_timing: NULL context");
    if (enable < 0 || enable > trim::Timer::kCalls)
        return fail(TRIM_E_INVAL, "trim_ctx_set_timing: enable outside [0, 64]");
    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    for (; c->timer.created < enable; ++c->timer.created)
        for (auto& ev : c->timer.slot[c->timer.created].ev)
            if ((e = hipEventCreate(&ev)) != hipSuccess) return hip_fail(e, "hipEventCreate");
    c->timer.keep = enable;
    c->timer.calls = 0;
    return TRIM_OK;
}

int trim_ctx_kernel_times(trim_ctx* c, int max, const char** names, float* ms) {
    if (!c || (max > 0 && (!names || !ms)))
        return fail(TRIM_E_INVAL, "trim_ctx_kernel_times: NULL argument");
    trim::Timer& t = c->timer;
    if (t.keep == 0 || t.calls == 0) return 0;
    const long long first = t.calls > t.keep ? t.calls - t.keep : 0;
    const trim::Timer::Slot& last = t.slot[(t.calls - 1) % t.keep];
    if (last.count > 0) {
        hipError_t e = hipEventSynchronize(last.ev[2 * last.count - 1]);
        if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
    }
    int k = 0;
    for (long long call = first; call < t.calls; ++call) {
        const trim::Timer::Slot& sl = t.slot[call % t.keep];
        for (int i = 0; i < sl.count && k < max; ++i, ++k) {
            names[k] = sl.names[i];
            float v = 0.f;
            hipError_t e = hipEventElapsedTime(&v, sl.ev[2 * i], sl.ev[2 * i + 1]);
            if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
            ms[k] = v;
        }
    }
    return k;
}

}  // extern "C"
