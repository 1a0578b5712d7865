// C ABI (include/perc.h) and the host runtime behind it: lattice handles with
// per-device tables, stream-ordered work memory, the job batches of the three
// execution forms, the tuning cache and the test hook. Every step of the inspection
// runs in the HIP kernels of kernels.hip.
#include "perc.h"

#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <chrono>
#include <deque>
#include <thread>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "perc_internal.hpp"

using namespace perc;

struct perc_lattice {
    LatticeDesc d;
};

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

int hip_fail(hipError_t e, const char* what) {
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return PERC_EHIP;
}

#define HIP_TRY(expr)                                     \
    do {                                                  \
        hipError_t e_ = (expr);                           \
        if (e_ != hipSuccess) return hip_fail(e_, #expr); \
    } while (0)

#define PERC_TRY(expr)                  \
    do {                                \
        int rc_ = (expr);               \
        if (rc_ != PERC_OK) return rc_; \
    } while (0)

constexpr size_t kMaxLds = 160 * 1024;
// The span form advances every configuration by two one-step launches between plans.
constexpr bool kSpanPairs = true;

// Workgroups per span step launch (16 per CU, a multiple of the 8 XCDs): enough that the
// tiles of several cell ranges run side by side on every XCD (measured at W=32 L=1024:
// 1024 -> 178.5 us, 2048 -> 158.8, 4096 -> 153.9, 8192 -> 154.1 per step).
constexpr int32_t kSpanGrid = 4096;

// ---------------------------------------------------------------------------------
// Per-device lattice tables and one-time kernel preparation.
// ---------------------------------------------------------------------------------
std::mutex g_prep_mu;
std::vector<int> g_prepared;

int prepare(int dev) {
    std::lock_guard<std::mutex> g(g_prep_mu);
    if (std::find(g_prepared.begin(), g_prepared.end(), dev) != g_prepared.end()) return PERC_OK;
    HIP_TRY(prepare_kernels(dev));
    g_prepared.push_back(dev);
    return PERC_OK;
}

template <typename T>
int upload(T** dst, const std::vector<T>& src) {
    HIP_TRY(hipMalloc(reinterpret_cast<void**>(dst), sizeof(T) * std::max<size_t>(src.size(), 1)));
    if (!src.empty()) HIP_TRY(hipMemcpy(*dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice));
    return PERC_OK;
}

// Device tables of each column set, per device: uploaded on first use and kept for the
// process (one set per fiber width in use; every fiber length shares them).
std::mutex g_coldev_mu;
std::map<std::pair<int, int32_t>, ColumnDevice> g_coldev;

int column_device(const ColumnSet& cs, int dev, ColumnDevice& out) {
    std::lock_guard<std::mutex> g(g_coldev_mu);
    auto it = g_coldev.find({dev, cs.W});
    if (it != g_coldev.end()) {
        out = it->second;
        return PERC_OK;
    }
    ColumnDevice n;
    PERC_TRY(upload(&n.nboff, cs.contact));
    PERC_TRY(upload(&n.lanes, cs.lanes));
    PERC_TRY(upload(&n.tile, cs.tile));
    PERC_TRY(upload(&n.rank, cs.rank));
    PERC_TRY(upload(&n.sig, cs.sig));
    if (!cs.contact2.empty()) {
        PERC_TRY(upload(&n.nboff2, cs.contact2));
        PERC_TRY(upload(&n.tile2, cs.tile2));
    }
    if (!cs.contact_whole.empty()) {
        PERC_TRY(upload(&n.nboff_whole, cs.contact_whole16));
        PERC_TRY(upload(&n.lanes_whole, cs.lanes_whole));
        PERC_TRY(upload(&n.nboff2_whole, cs.contact_whole));
        PERC_TRY(upload(&n.tile_whole, std::vector<int32_t>{0, cs.C, 0, cs.C, 0, cs.C}));
    }
    g_coldev.emplace(std::make_pair(dev, cs.W), n);
    out = n;
    return PERC_OK;
}

// The kernels' view of a shape; with `whole`, the one-tile tiling of the whole
// cross-section (fibers of at most kWholeCols columns), whose tile is also its own
// outer range for the two-step walk.
int shape_of(const LatticeDesc& d, DevShape& sh, bool whole = false) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    PERC_TRY(prepare(dev));
    ColumnDevice cd;
    PERC_TRY(column_device(*d.cs, dev, cd));
    if (whole && !cd.nboff_whole) return fail(PERC_EINVAL, "the fiber has more columns than one tile holds");
    sh.nboff = whole ? cd.nboff_whole : cd.nboff;
    sh.lanes = whole ? cd.lanes_whole : cd.lanes;
    sh.lane_stride = whole ? d.cs->lane_stride_whole : d.cs->lane_stride;
    sh.tile = whole ? cd.tile_whole : cd.tile;
    sh.rank = cd.rank;
    sh.sig = cd.sig;
    sh.nboff2 = whole ? cd.nboff2_whole : cd.nboff2;
    sh.tile2 = whole ? cd.tile_whole + 4 : cd.tile2;
    sh.C = d.C; sh.CP = d.CP; sh.U = d.U; sh.L = d.L;
    sh.ntile = whole ? 1 : d.ntile;
    sh.span_max = whole ? d.C : d.span_max;
    sh.tile_max = whole ? d.C : d.tile_max;
    sh.W = d.W;
    sh.ends = d.ends;
    sh.span2_max = whole ? d.C : d.cs->span2_max;
    sh.N = d.N; sh.words = d.words;
    return PERC_OK;
}

int shape_for(const perc_lattice* lat, DevShape& sh) { return shape_of(lat->d, sh); }

// ---------------------------------------------------------------------------------
// Work memory kept between calls: one grow-only device buffer per device, lent to one
// call at a time. A fresh stream-ordered allocation of tens of GiB costs the driver's
// page mapping and clearing on every call (measured: 0.5 to 1.3 s for one 40 GiB
// allocation and 0.8 s for its release, against 0.42 s of kernels), so large work
// memory is reused instead. The call that next borrows the buffer waits (on its own
// stream) for the event the previous borrower recorded when it returned it; a call that
// finds the buffer lent to another host thread allocates its own, stream-ordered.
// ---------------------------------------------------------------------------------
constexpr int64_t kWaveBudget = 128ll << 30;  // span-form work memory per wave, at most
constexpr size_t kCacheMin = 64ull << 20;  // smaller pieces come from the stream pool
constexpr size_t kCacheGrain = 1ull << 30;
constexpr int kCacheDevices = 64;

struct WorkCache {
    std::mutex mu;
    char* base = nullptr;
    size_t size = 0;
    bool busy = false;
    hipEvent_t done = nullptr;  // recorded on the last borrower's stream when returned
    bool pending = false;
};
// Per device: the buffer of the callers' streams, and one for the library's side stream
// (below), whose work runs beside a caller's.
WorkCache g_cache[kCacheDevices][2];

// A second stream per device for the persistent part of a mixed batch (created on first
// use, default priority, kept for the process).
std::mutex g_side_mu;
hipStream_t g_side[kCacheDevices] = {};
int side_stream(hipStream_t* out) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kCacheDevices) return fail(PERC_EINVAL, "device index beyond the library's table");
    std::lock_guard<std::mutex> g(g_side_mu);
    if (!g_side[dev]) HIP_TRY(hipStreamCreateWithFlags(&g_side[dev], hipStreamNonBlocking));
    *out = g_side[dev];
    return PERC_OK;
}

bool is_side_stream(int dev, hipStream_t s) {
    std::lock_guard<std::mutex> g(g_side_mu);
    return s && s == g_side[dev];
}

// The bytes of the cached buffers a new call could borrow (counted as free memory by
// the budgets, since hipMemGetInfo reports them as used).
size_t cache_idle_bytes() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kCacheDevices) return 0;
    size_t idle = 0;
    for (WorkCache& c : g_cache[dev]) {
        std::lock_guard<std::mutex> g(c.mu);
        idle += c.busy ? 0 : c.size;
    }
    return idle;
}

// Borrow at least `bytes` of the device's buffer for work on stream s (the side stream's
// own buffer for work on it); nullptr when it is lent out, the device is out of range or
// it cannot grow (the caller then allocates).
char* cache_borrow(size_t bytes, hipStream_t s, WorkCache** owner) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kCacheDevices) return nullptr;
    WorkCache& c = g_cache[dev][is_side_stream(dev, s) ? 1 : 0];
    std::lock_guard<std::mutex> g(c.mu);
    if (c.busy) return nullptr;
    if (!c.done && hipEventCreateWithFlags(&c.done, hipEventDisableTiming) != hipSuccess) {
        c.done = nullptr;
        return nullptr;
    }
    if (c.size < bytes) {
        if (c.base) {
            // the previous borrower's work must end before its memory is released
            if (c.pending && hipEventSynchronize(c.done) != hipSuccess) return nullptr;
            (void)hipFree(c.base);
            c.base = nullptr;
            c.size = 0;
            c.pending = false;
        }
        const size_t want = (bytes + kCacheGrain - 1) / kCacheGrain * kCacheGrain;
        if (hipMalloc(reinterpret_cast<void**>(&c.base), want) != hipSuccess) {
            (void)hipGetLastError();
            c.base = nullptr;
            return nullptr;
        }
        c.size = want;
    }
    if (c.pending && hipStreamWaitEvent(s, c.done, 0) != hipSuccess) return nullptr;
    c.busy = true;
    *owner = &c;
    return c.base;
}

void cache_return(WorkCache* c, hipStream_t s) {
    std::lock_guard<std::mutex> g(c->mu);
    c->pending = hipEventRecord(c->done, s) == hipSuccess;
    if (!c->pending) (void)hipStreamSynchronize(s);  // no event: wait here instead
    c->busy = false;
}

int cache_trim() {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kCacheDevices) return PERC_OK;
    bool busy = false;  // the idle buffers are released even when another is lent out
    for (WorkCache& c : g_cache[dev]) {
        std::lock_guard<std::mutex> g(c.mu);
        if (c.busy) {
            busy = true;
            continue;
        }
        if (c.pending) HIP_TRY(hipEventSynchronize(c.done));
        c.pending = false;
        if (c.base) HIP_TRY(hipFree(c.base));
        c.base = nullptr;
        c.size = 0;
    }
    return busy ? fail(PERC_EBUSY, "a work buffer is in use by a call") : PERC_OK;
}

// A device allocation that, when the device is short of memory, releases the idle work
// buffer (above) and tries once more.
int device_alloc(void** p, size_t bytes) {
    hipError_t e = hipMalloc(p, bytes);
    if (e == hipErrorOutOfMemory) {
        (void)hipGetLastError();
        if (cache_trim() != PERC_EHIP) e = hipMalloc(p, bytes);  // whatever it could release
    }
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return fail(e == hipErrorOutOfMemory ? PERC_ENOMEM : PERC_EHIP,
                    std::string("device allocation of ") + std::to_string(bytes) + " bytes: " + hipGetErrorString(e));
    }
    return PERC_OK;
}

// ---------------------------------------------------------------------------------
// Work memory of one call: one allocation (the cached buffer when large) carved into
// aligned pieces.
// ---------------------------------------------------------------------------------
struct Arena {
    hipStream_t s = nullptr;
    char* base = nullptr;
    size_t size = 0, used = 0;
    WorkCache* cached = nullptr;
    ~Arena() {
        if (cached) cache_return(cached, s);
        else if (base) (void)hipFreeAsync(base, s);
    }
    static size_t align(size_t v) { return (v + 255) & ~(size_t)255; }
    // bytes take<T>(count) uses (a piece is never empty)
    template <typename T>
    static size_t need(size_t count) {
        return align(sizeof(T) * std::max<size_t>(count, 1));
    }
    int reserve(size_t bytes, hipStream_t stream) {
        s = stream;
        size = std::max<size_t>(bytes, 256);
        if (size >= kCacheMin && (base = cache_borrow(size, s, &cached))) return PERC_OK;
        hipError_t e = hipMallocAsync(reinterpret_cast<void**>(&base), size, s);
        if (e == hipErrorOutOfMemory) {
            (void)hipGetLastError();
            if (cache_trim() != PERC_EHIP) e = hipMallocAsync(reinterpret_cast<void**>(&base), size, s);
        }
        if (e != hipSuccess) {
            base = nullptr;
            return fail(PERC_ENOMEM, std::string("work memory of ") + std::to_string(size) + " bytes: " +
                                         hipGetErrorString(e));
        }
        return PERC_OK;
    }
    template <typename T>
    T* take(size_t count) {
        T* p = reinterpret_cast<T*>(base + used);
        used += align(sizeof(T) * std::max<size_t>(count, 1));
        return p;
    }
    // every piece taken lies inside the reservation (checked before any launch)
    int check() const {
        return used <= size ? PERC_OK : fail(PERC_EINVAL, "internal: work memory carved beyond its reservation");
    }
};

// Pinned words the host polls between steps. Kept until the process ends: the HIP
// runtime may already be gone when thread-local destructors run at exit.
struct PinnedHdr {
    int32_t* h = nullptr;
    PinnedHdr() {
        if (hipHostMalloc(reinterpret_cast<void**>(&h), 64, hipHostMallocDefault) != hipSuccess) h = nullptr;
    }
};
thread_local PinnedHdr g_pinned;

// ---------------------------------------------------------------------------------
// Optional profiling of the span/plain step kernel: HIP events on the launching
// stream around every step launch (graphs are not used while it is on: HIP reports no
// elapsed time for events recorded as graph nodes) and the tube slots the steps
// processed (counted by the planner).
// ---------------------------------------------------------------------------------
struct Profiler {
    std::mutex mu;
    bool on = false;
    int64_t launches = 0;
    double ms = 0.0;
    int64_t tube_steps = 0;
    int64_t p_launches = 0;  // the persistent launches' part
    double p_ms = 0.0;
    int64_t p_tube_steps = 0;
};
Profiler g_prof;

bool profiling() {
    std::lock_guard<std::mutex> g(g_prof.mu);
    return g_prof.on;
}

SpanArgs second_of(const SpanArgs& a);  // the second launch of a pair

// The plan launch's arguments; the last plan of a run of steps lists the slots for the
// extension launch that starts the next run.
SpanArgs last_plan(const SpanArgs& a, bool last) {
    SpanArgs b = a;
    b.list_ext = last ? 1 : 0;
    return b;
}

class StepTimer {
  public:
    explicit StepTimer(bool on) : on_(on) {}
    ~StepTimer() {
        for (auto& p : pending_) { free_.push_back(p.first); free_.push_back(p.second); }
        for (hipEvent_t e : free_) (void)hipEventDestroy(e);
    }
    // one step launch, or with a.pair the pair of launches (back to back, one event pair
    // around both: the average per launch is half the pair's time)
    hipError_t step(const SpanArgs& a, hipStream_t s) {
        if (!on_) {
            hipError_t e = launch_span_step(a, s);
            if (e == hipSuccess && a.pair) e = launch_span_step(second_of(a), s);
            return e;
        }
        std::pair<hipEvent_t, hipEvent_t> ev;
        hipError_t e = take(&ev.first);
        if (e == hipSuccess) e = take(&ev.second);
        if (e != hipSuccess) return e;
        pending_.push_back(ev);
        launches_ += a.pair ? 2 : 1;
        e = hipEventRecord(ev.first, s);
        if (e == hipSuccess) e = launch_span_step(a, s);
        if (e == hipSuccess && a.pair) e = launch_span_step(second_of(a), s);
        if (e == hipSuccess) e = hipEventRecord(ev.second, s);
        return e;
    }
    // after the stream has been synchronised: add the durations since the last call
    hipError_t collect() {
        if (!on_) return hipSuccess;
        double ms = 0.0;
        for (auto& p : pending_) {
            float t = 0.0f;
            hipError_t e = hipEventElapsedTime(&t, p.first, p.second);
            if (e != hipSuccess) return e;
            ms += t;
            free_.push_back(p.first);
            free_.push_back(p.second);
        }
        std::lock_guard<std::mutex> g(g_prof.mu);
        g_prof.launches += launches_;
        g_prof.ms += ms;
        pending_.clear();
        launches_ = 0;
        return hipSuccess;
    }
    bool on() const { return on_; }

  private:
    hipError_t take(hipEvent_t* e) {
        if (!free_.empty()) { *e = free_.back(); free_.pop_back(); return hipSuccess; }
        return hipEventCreate(e);
    }
    bool on_;
    int64_t launches_ = 0;  // step launches timed by the pending event pairs
    std::vector<hipEvent_t> free_;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pending_;
};

// ---------------------------------------------------------------------------------
// Tuning: explicit options, else the autotune cache, else shape rules.
// ---------------------------------------------------------------------------------
struct TuneKey {
    int32_t W, L, bucket;
    bool operator<(const TuneKey& o) const { return std::tie(W, L, bucket) < std::tie(o.W, o.L, o.bucket); }
};
std::mutex g_tune_mu;
std::map<TuneKey, Tuning> g_tune;

int32_t size_bucket(int64_t n) {
    int32_t b = 0;
    while (n > 1 && b < 40) { n >>= 1; ++b; }
    return b;
}

struct ShapeNeed {
    int32_t span_max = 0, tile_max = 0, C = 0;
    int64_t items = 0;   // column tiles x cells of the largest shape
    int32_t span2_max = 0;
    bool two_step = true;  // every shape has the two-step contact table
    int32_t CP = 0;
};

// Threads per workgroup for these shapes: one per column of the widest tile, and the
// staged halo range must fit two columns per thread.
int32_t block_for(const ShapeNeed& nd) {
    const int32_t b = std::max<int32_t>(64, ((nd.tile_max + 63) / 64) * 64);
    return std::max<int32_t>(b, ((nd.span_max + 2 * 64 - 1) / (2 * 64)) * 64);
}

// Default cells walked per work item (a multiple of 8): long walks amortise the
// staged groups of the prologue; a single configuration needs short ones to give
// every CU work.
int32_t cells_for(const ShapeNeed& nd, int32_t form) {
    if (form == FORM_PLAIN) return (int32_t)(std::max<int64_t>(1, std::min<int64_t>(4, nd.items / 8192)) * 8);
    // a persistent workgroup walks its configuration alone: long walks (batched W=16
    // L=256 sweep: 32 cells 443 ms, 64 cells 418 ms, 128 cells 408 ms of kernel time)
    if (form == FORM_PERSIST || form == FORM_PERSIST2) return 128;
    // span: fewer boundary groups per cell than 64-cell items, still fine-grained enough
    // for the end of a launch (W=32 L=1024 x 768: 48 cells 3.85 TB/s, 64 3.92, 80 3.95,
    // 96 3.93 of step kernel)
    return 80;
}

int check_walk(const ShapeNeed& nd, int32_t block) {
    if (block < nd.tile_max)
        return fail(PERC_EINVAL, "block must be at least the widest column tile (" + std::to_string(nd.tile_max) + ")");
    if (nd.span_max > 2 * block || lds_total(nd.span_max) > kMaxLds)
        return fail(PERC_EINVAL, "the fiber cross-section is too wide for one workgroup tile (halo range " +
                                     std::to_string(nd.span_max) + " columns)");
    return PERC_OK;
}

// The two-step form also stages the outer range (two columns per thread at most) and
// holds two rings in LDS.
bool two_step_fits(const ShapeNeed& nd, int32_t block) {
    return nd.two_step && block >= nd.tile_max && nd.span_max <= 2 * block && nd.span2_max <= 2 * block &&
           lds_total2(nd.span_max, nd.span2_max) <= kMaxLds;
}

int check_walk2(const ShapeNeed& nd, int32_t block) {
    PERC_TRY(check_walk(nd, block));
    if (!two_step_fits(nd, block))
        return fail(PERC_EINVAL, "the two-step form needs the outer range (" + std::to_string(nd.span2_max) +
                                     " columns) within two columns per thread and both rings in LDS");
    return PERC_OK;
}

int resolve(const ShapeNeed& nd, int64_t state_words, int64_t n_jobs, const perc_options* opt, Tuning& tu,
            const TuneKey* key) {
    tu = Tuning{};
    if (opt) {
        tu.form = opt->form;
        tu.depth = opt->depth;
        tu.block = opt->block;
        tu.grid = opt->grid;
        tu.graph_steps = opt->graph_steps;
    }
    if (tu.form < FORM_AUTO || tu.form > FORM_PERSIST2) return fail(PERC_EINVAL, "unknown execution form");
    if (tu.form == FORM_AUTO && key) {
        std::lock_guard<std::mutex> g(g_tune_mu);
        auto it = g_tune.find(*key);
        if (it != g_tune.end()) {
            const Tuning c = it->second;
            tu.form = c.form;
            if (!tu.depth) tu.depth = c.depth;
            if (!tu.block) tu.block = c.block;
            if (!tu.grid) tu.grid = c.grid;
        }
    }
    if (tu.form == FORM_AUTO) {
        // many configurations of modest size: one workgroup each; else spread
        tu.form = (n_jobs >= 2048 && state_words * 9 <= (64ll << 20)) ? FORM_PERSIST : FORM_SPAN;
    }
    if (tu.depth == 0) tu.depth = cells_for(nd, tu.form);
    if (tu.depth < 1 || tu.depth > (1 << 20)) return fail(PERC_EINVAL, "depth (cells per work item) must be 1..2^20");
    tu.depth = (tu.depth + 7) & ~7;  // items are whole pairs of cell groups
    if (tu.form == FORM_PERSIST2) {
        // one thread per column of the whole cross-section
        if (nd.C > kWholeCols)
            return fail(PERC_EINVAL, "the two-step persistent form needs fibers of at most " +
                                         std::to_string(kWholeCols) + " columns (W <= 17)");
        const int32_t bw = std::max<int32_t>(64, ((nd.C + 63) / 64) * 64);
        if (tu.block == 0) tu.block = bw;
        if (tu.block < bw) return fail(PERC_EINVAL, "block must hold one thread per column (" + std::to_string(bw) + ")");
    }
    if (tu.block == 0) tu.block = block_for(nd);
    if (tu.block < 64 || tu.block > 1024 || tu.block % 64)
        return fail(PERC_EINVAL, "block must be 64..1024, a multiple of 64");
    if (tu.form != FORM_PERSIST2) PERC_TRY(tu.form == FORM_SPAN2 ? check_walk2(nd, tu.block) : check_walk(nd, tu.block));
    if (tu.graph_steps == 0) tu.graph_steps = 8;
    if (tu.graph_steps < 1 || tu.graph_steps > 256) return fail(PERC_EINVAL, "graph_steps must be 1..256");
    if (tu.grid < 0) return fail(PERC_EINVAL, "grid must be >= 0");
    return PERC_OK;
}

// ---------------------------------------------------------------------------------
// Jobs: one configuration each (a lattice shape, and caller bits or a Philox draw).
// ---------------------------------------------------------------------------------
struct HostJob {
    const perc_lattice* lat;
    const uint32_t* bits;
    uint64_t seed, cfg, thr;
    int32_t group;
};

uint64_t threshold_of(double p) {
    if (p >= 1.0) return (uint64_t)1 << 32;
    return (uint64_t)std::floor(p * 4294967296.0);
}

struct Shapes {
    std::vector<const perc_lattice*> lats;
    std::vector<DevShape> dev;
    std::vector<int32_t> of_job;
    ShapeNeed need;
    int64_t max_state = 0, max_words = 0;
};

void collect_shapes(const std::vector<HostJob>& jobs, Shapes& S) {
    std::map<const perc_lattice*, int32_t> idx;
    S.of_job.resize(jobs.size());
    for (size_t j = 0; j < jobs.size(); ++j) {
        auto it = idx.find(jobs[j].lat);
        if (it == idx.end()) {
            it = idx.emplace(jobs[j].lat, (int32_t)S.lats.size()).first;
            S.lats.push_back(jobs[j].lat);
        }
        S.of_job[j] = it->second;
    }
    for (const perc_lattice* l : S.lats) {
        const LatticeDesc& d = l->d;
        S.need.span_max = std::max(S.need.span_max, d.span_max);
        S.need.tile_max = std::max(S.need.tile_max, d.tile_max);
        S.need.C = std::max(S.need.C, d.C);
        S.need.items = std::max<int64_t>(S.need.items, (int64_t)d.U * d.ntile);
        S.need.span2_max = std::max(S.need.span2_max, d.cs->span2_max);
        S.need.two_step = S.need.two_step && !d.cs->contact2.empty();
        S.need.CP = std::max(S.need.CP, d.CP);
        S.max_state = std::max<int64_t>(S.max_state, state_words(d));
        S.max_words = std::max<int64_t>(S.max_words, d.words);
    }
}

int device_shapes(Shapes& S, bool whole = false) {
    S.dev.resize(S.lats.size());
    for (size_t i = 0; i < S.lats.size(); ++i) PERC_TRY(shape_of(S.lats[i]->d, S.dev[i], whole));
    return PERC_OK;
}

bool stream_capturing(hipStream_t s) {
    if (!s) return false;
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &st) != hipSuccess) return false;
    return st != hipStreamCaptureStatusNone;
}

int64_t slot_words(const LatticeDesc& d) { return (state_words(d) + 63) & ~(int64_t)63; }
int64_t bits_words(const LatticeDesc& d) { return (d.words + 63) & ~(int64_t)63; }

// Span and plain forms: waves of slots sized to the memory budget.
// The second launch of a pair: the same work list, reading the first launch's output.
SpanArgs second_of(const SpanArgs& a) {
    SpanArgs b = a;
    b.sub = 1;
    return b;
}

int run_span(const std::vector<HostJob>& jobs, const Shapes& S, BatchOut out, const Tuning& tu, hipStream_t s) {
    const int64_t n = (int64_t)jobs.size();
    if (n == 0) return PERC_OK;
    if (stream_capturing(s)) return fail(PERC_EINVAL, "the span and plain forms synchronise; not capturable");
    const bool plain = tu.form == FORM_PLAIN;
    const bool fused = tu.form == FORM_SPAN2;
    size_t free_b = 0, total_b = 0;
    HIP_TRY(hipMemGetInfo(&free_b, &total_b));
    // one wave holds as many jobs as half the free memory allows, at most 128 GiB: a batch
    // that fits runs as one work list, without a tail per wave (the 35-shape aspect-ratio
    // sweep, ~120 GiB of state: 344 -> 336 ms of step kernel at 96 GiB, two waves)
    const int64_t budget = std::min<int64_t>((int64_t)((free_b + cache_idle_bytes()) / 2), kWaveBudget);
    if (!g_pinned.h) return fail(PERC_ENOMEM, "pinned host buffer");
    int32_t* h = g_pinned.h;
    const int lds = (int)(fused ? lds_total2(S.need.span_max, S.need.span2_max) : lds_total(S.need.span_max));
    Arena shape_ar;
    PERC_TRY(shape_ar.reserve(sizeof(DevShape) * S.dev.size(), s));
    DevShape* d_shapes = shape_ar.take<DevShape>(S.dev.size());
    HIP_TRY(hipMemcpyAsync(d_shapes, S.dev.data(), sizeof(DevShape) * S.dev.size(), hipMemcpyHostToDevice, s));
    StepTimer timer(profiling());
    const bool use_graph = !plain && s != nullptr && !timer.on();
    int64_t w0 = 0;
    while (w0 < n) {
        // slots of this wave: as many jobs as the budget holds (one for the plain form)
        int64_t w1 = w0, words = 0, bitw = 0;
        while (w1 < n) {
            const LatticeDesc& d = jobs[w1].lat->d;
            const int64_t sw = slot_words(d);
            const int64_t bw = jobs[w1].bits ? 0 : bits_words(d);
            const int64_t bytes = (words + sw) * 9 + (bitw + bw) * 4 + (w1 - w0 + 1) * (96 + 4 * S.need.CP);
            if (w1 > w0 && (bytes > budget || plain || w1 - w0 >= (1 << 20))) break;
            words += sw;
            bitw += bw;
            ++w1;
        }
        const int32_t nb = (int32_t)(w1 - w0);
        std::vector<int32_t> h_shape(nb), h_group(nb);
        std::vector<int64_t> h_off(nb), h_boff(nb, -1);
        std::vector<Job> h_jobs(nb);
        int64_t off = 0, boff = 0;
        for (int32_t b = 0; b < nb; ++b) {
            const HostJob& hj = jobs[w0 + b];
            const LatticeDesc& d = hj.lat->d;
            h_shape[b] = S.of_job[w0 + b];
            h_off[b] = off;
            off += slot_words(d);
            if (!hj.bits) {
                h_boff[b] = boff;
                boff += bits_words(d);
            }
            h_jobs[b] = Job{hj.bits, hj.seed, hj.cfg, hj.thr, h_shape[b], hj.group};
            h_group[b] = hj.group;
        }
        Arena ar;
        // every piece as take<>() carves it below (an empty piece still takes 256 bytes)
        const size_t bytes = Arena::need<float>(off) * 2 + Arena::need<uint8_t>(off) + Arena::need<uint32_t>(boff) +
                             Arena::need<CfgState>(nb) + Arena::need<int32_t>(nb) * 4 + Arena::need<int64_t>(nb + 1) * 2 +
                             Arena::need<void*>(nb) + Arena::need<Job>(nb) + Arena::need<int32_t>(16) +
                             Arena::need<int32_t>(nb) + Arena::need<int64_t>(nb + 1) +
                             (fused ? Arena::need<float>((size_t)nb * S.need.CP) : 0);
        PERC_TRY(ar.reserve(bytes, s));
        SpanArgs a{};
        a.shapes = d_shapes;
        a.ya = ar.take<float>(off);
        a.yb = ar.take<float>(off);
        a.code = ar.take<uint8_t>(off);
        uint32_t* scratch_bits = ar.take<uint32_t>(boff);
        a.st = ar.take<CfgState>(nb);
        a.active = ar.take<int32_t>(nb);
        a.active2 = ar.take<int32_t>(nb);
        int32_t* d_shape = ar.take<int32_t>(nb);
        int32_t* d_group = ar.take<int32_t>(nb);
        a.chunk_off = ar.take<int64_t>(nb + 1);
        int64_t* d_off = ar.take<int64_t>(nb + 1);
        uint32_t** d_bits = ar.take<uint32_t*>(nb);
        Job* d_jobs = ar.take<Job>(nb);
        a.hdr = ar.take<int32_t>(16);
        a.ext_ids = ar.take<int32_t>(nb);
        a.ext_off = ar.take<int64_t>(nb + 1);
        // the span form runs two one-step launches between plans (the planner decides
        // both steps), which halves the planner launches
        a.pair = (!fused && !plain && kSpanPairs) ? 1 : 0;
        // lazy initialisation (not for the plain form, which polls after every step): a
        // run of steps between two extension launches is graph_steps plans of two steps
        // each; the margin covers it, the window past the front and a group
        a.lazy = plain ? 0 : 1;
        a.init_margin = 2 * tu.graph_steps + 12;
        if (fused) {
            a.fused = 1;
            a.far1_stride = S.need.CP;
            a.far1 = ar.take<float>((size_t)nb * S.need.CP);
            a.r1_off = (int32_t)lds_ring2_words(S.need.span2_max);
        }
        PERC_TRY(ar.check());
        std::vector<const uint32_t*> h_bits(nb);
        for (int32_t b = 0; b < nb; ++b) h_bits[b] = h_jobs[b].bits ? h_jobs[b].bits : scratch_bits + h_boff[b];
        HIP_TRY(hipMemcpyAsync(d_shape, h_shape.data(), sizeof(int32_t) * nb, hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(d_group, h_group.data(), sizeof(int32_t) * nb, hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(d_off, h_off.data(), sizeof(int64_t) * nb, hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(d_bits, h_bits.data(), sizeof(void*) * nb, hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(d_jobs, h_jobs.data(), sizeof(Job) * nb, hipMemcpyHostToDevice, s));
        a.slot_shape = d_shape;
        a.slot_off = d_off;
        a.slot_bits = d_bits;
        a.work = reinterpret_cast<unsigned long long*>(a.hdr + 8);
        a.out.perc = out.perc + w0;
        a.out.steps = out.steps + w0;
        a.out.hit = out.hit ? out.hit + w0 : nullptr;
        a.out.group_count = out.group_count;
        a.out.group = out.group_count ? d_group : nullptr;
        a.n_slot = nb;
        a.depth = tu.depth;
        a.block = tu.block;
        a.grid = tu.grid ? tu.grid : kSpanGrid;
        a.lds = lds;
        // the planner shortens the items of work lists smaller than the device holds
        a.resident = fused ? 0 : span_step_resident(a.block, a.lds);
        HIP_TRY(launch_fill_u32(reinterpret_cast<uint32_t*>(a.hdr), 16, 0u, s));
        if (boff) HIP_TRY(launch_sample_slots(d_shapes, d_jobs, nb, d_bits, s));
        HIP_TRY(launch_span_init(a, s));
        if (plain) {
            for (;;) {
                HIP_TRY(hipMemcpyAsync(h, a.hdr, 64, hipMemcpyDeviceToHost, s));
                HIP_TRY(hipStreamSynchronize(s));
                HIP_TRY(timer.collect());
                if (h[0] == 0) break;
                HIP_TRY(timer.step(a, s));
                HIP_TRY(launch_span_plan(a, s));
            }
        } else {
            hipGraphExec_t exec = nullptr;
            if (use_graph) {
                hipGraph_t graph = nullptr;
                HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
                hipError_t ce = a.lazy ? launch_span_extend(a, s) : hipSuccess;
                for (int i = 0; i < tu.graph_steps && ce == hipSuccess; ++i) {
                    ce = launch_span_step(a, s);
                    if (ce == hipSuccess && a.pair) ce = launch_span_step(second_of(a), s);
                    if (ce == hipSuccess) ce = launch_span_plan(last_plan(a, i == tu.graph_steps - 1), s);
                }
                hipError_t ee = hipStreamEndCapture(s, &graph);
                if (ce != hipSuccess) {
                    if (graph) (void)hipGraphDestroy(graph);
                    return hip_fail(ce, "capture");
                }
                if (ee != hipSuccess) return hip_fail(ee, "hipStreamEndCapture");
                hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
                (void)hipGraphDestroy(graph);
                if (ie != hipSuccess) return hip_fail(ie, "hipGraphInstantiate");
            }
            int reps = 1;
            int rc = PERC_OK;
            for (;;) {
                for (int r = 0; r < reps && rc == PERC_OK; ++r) {
                    if (exec) {
                        hipError_t e = hipGraphLaunch(exec, s);
                        if (e != hipSuccess) rc = hip_fail(e, "hipGraphLaunch");
                    } else {
                        if (a.lazy) {
                            hipError_t e = launch_span_extend(a, s);
                            if (e != hipSuccess) rc = hip_fail(e, "span extend");
                        }
                        for (int i = 0; i < tu.graph_steps && rc == PERC_OK; ++i) {
                            hipError_t e = timer.step(a, s);
                            if (e == hipSuccess) e = launch_span_plan(last_plan(a, i == tu.graph_steps - 1), s);
                            if (e != hipSuccess) rc = hip_fail(e, "span step");
                        }
                    }
                }
                if (rc != PERC_OK) break;
                hipError_t e = hipMemcpyAsync(h, a.hdr, 64, hipMemcpyDeviceToHost, s);
                if (e == hipSuccess) e = hipStreamSynchronize(s);
                if (e == hipSuccess) e = timer.collect();
                if (e != hipSuccess) {
                    rc = hip_fail(e, "span poll");
                    break;
                }
                if (h[0] == 0) break;
                reps = std::min(reps * 2, 8);
            }
            if (exec) (void)hipGraphExecDestroy(exec);
            if (rc != PERC_OK) return rc;
        }
        if (h[2]) return fail(PERC_ECAP, "a configuration reached the step cap");
        if (timer.on()) {
            unsigned long long tubes = 0;
            std::memcpy(&tubes, h + 8, sizeof(tubes));
            std::lock_guard<std::mutex> g(g_prof.mu);
            g_prof.tube_steps += (int64_t)tubes;
        }
        HIP_TRY(launch_span_finish(a, s));
        w0 = w1;
    }
    return PERC_OK;
}

// Persistent form: every job in one launch; scratch per resident workgroup.
// Persistent form: the jobs in chunks whose drawn occupancy fits kPersistBitsBudget; per
// chunk one sampling launch for the Philox jobs, then one persistent launch over all the
// chunk's jobs with scratch per resident workgroup.
constexpr int64_t kPersistBitsBudget = 8ll << 30;

int run_persist_chunk(const std::vector<HostJob>& jobs, int64_t j0, int64_t j1, const Shapes& S, BatchOut out,
                      const Tuning& tu, int grid, int lds, hipStream_t s) {
    const int64_t n = j1 - j0;
    const bool two = tu.form == FORM_PERSIST2;
    grid = (int)std::min<int64_t>(grid, n);
    const int64_t sw = (S.max_state + 63) & ~(int64_t)63;
    std::vector<Job> h_jobs(n);
    std::vector<int64_t> h_idx;
    int64_t bits_total = 0;
    for (int64_t j = 0; j < n; ++j) {
        const HostJob& hj = jobs[j0 + j];
        h_jobs[j] = Job{hj.bits, hj.seed, hj.cfg, hj.thr, S.of_job[j0 + j], hj.group};
        if (!hj.bits) {
            h_idx.push_back(j);
            bits_total += bits_words(hj.lat->d);
        }
    }
    const int64_t n_draw = (int64_t)h_idx.size();
    // queue order: longest expected inspections first, so that the launch does not end
    // with every workgroup on a long one: larger fibers first, then higher p (the
    // expected step count grows with p up to the threshold and stays high above it);
    // caller-given occupancy (p unknown) last, in job order
    std::vector<int64_t> h_order(n);
    for (int64_t j = 0; j < n; ++j) h_order[j] = j;
    std::stable_sort(h_order.begin(), h_order.end(), [&](int64_t x, int64_t y) {
        const HostJob& a = jobs[j0 + x];
        const HostJob& b = jobs[j0 + y];
        if (a.lat->d.N != b.lat->d.N) return a.lat->d.N > b.lat->d.N;
        if ((a.bits == nullptr) != (b.bits == nullptr)) return a.bits == nullptr;
        return a.thr > b.thr;
    });
    Arena ar;
    const size_t bytes = Arena::need<float>((size_t)grid * sw) * 2 + Arena::need<uint8_t>((size_t)grid * sw) +
                         Arena::need<uint32_t>(bits_total) + Arena::need<int64_t>(n_draw) + Arena::need<Job>(n) +
                         Arena::need<int64_t>(n) +
                         Arena::need<DevShape>(S.dev.size()) + Arena::need<unsigned long long>(3) +
                         (two ? Arena::need<float>((size_t)grid * S.need.CP) : 0);
    PERC_TRY(ar.reserve(bytes, s));
    PersistArgs a{};
    a.ya = ar.take<float>(grid * sw);
    a.yb = ar.take<float>(grid * sw);
    a.code = ar.take<uint8_t>(grid * sw);
    a.state_stride = sw;
    uint32_t* drawn = ar.take<uint32_t>(bits_total);
    int64_t* d_idx = ar.take<int64_t>(n_draw);
    Job* d_jobs = ar.take<Job>(n);
    int64_t* d_order = ar.take<int64_t>(n);
    DevShape* d_shapes = ar.take<DevShape>(S.dev.size());
    int64_t boff = 0;
    for (int64_t k = 0; k < n_draw; ++k) {
        Job& jb = h_jobs[h_idx[k]];
        jb.bits = drawn + boff;
        boff += bits_words(jobs[j0 + h_idx[k]].lat->d);
    }
    if (two) {
        a.two = 1;
        a.far1_stride = S.need.CP;
        a.far1 = ar.take<float>((size_t)grid * S.need.CP);
        a.r1_off = (int32_t)lds_ring2_words(S.need.C);
    }
    a.queue = ar.take<unsigned long long>(3);
    PERC_TRY(ar.check());
    // the cap flag goes to the caller's word when it has one (a synchronous call reads it)
    a.err = out.cap ? out.cap : reinterpret_cast<uint32_t*>(a.queue + 1);
    const bool prof = profiling();
    if (prof) a.work = a.queue + 2;
    HIP_TRY(hipMemcpyAsync(d_jobs, h_jobs.data(), sizeof(Job) * n, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(d_shapes, S.dev.data(), sizeof(DevShape) * S.dev.size(), hipMemcpyHostToDevice, s));
    if (n_draw) HIP_TRY(hipMemcpyAsync(d_idx, h_idx.data(), sizeof(int64_t) * n_draw, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(d_order, h_order.data(), sizeof(int64_t) * n, hipMemcpyHostToDevice, s));
    a.shapes = d_shapes;
    a.jobs = d_jobs;
    a.order = d_order;
    a.n_jobs = n;
    a.out = out;
    a.out.perc = out.perc + j0;
    a.out.steps = out.steps + j0;
    a.out.hit = out.hit ? out.hit + j0 : nullptr;
    a.depth = tu.depth;
    a.block = tu.block;
    a.grid = grid;
    a.lds = lds;
    HIP_TRY(launch_fill_u32(reinterpret_cast<uint32_t*>(a.queue), 6, 0u, s));
    HIP_TRY(launch_sample_jobs(d_shapes, d_jobs, d_idx, n_draw, s));
    if (!prof) {
        HIP_TRY(launch_persist(a, s));
        return PERC_OK;
    }
    // profiled: the persistent launch between HIP events on its stream, and the tube
    // slots its steps advanced (synchronous)
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    hipError_t e = hipEventRecord(e0, s);
    if (e == hipSuccess) e = launch_persist(a, s);
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    unsigned long long tubes = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&tubes, a.work, sizeof(tubes), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    HIP_TRY(e);
    std::lock_guard<std::mutex> g(g_prof.mu);
    g_prof.launches += 1;
    g_prof.ms += ms;
    g_prof.tube_steps += (int64_t)tubes;
    g_prof.p_launches += 1;
    g_prof.p_ms += ms;
    g_prof.p_tube_steps += (int64_t)tubes;
    return PERC_OK;
}

int run_persist(const std::vector<HostJob>& jobs, const Shapes& S, BatchOut out, const Tuning& tu, hipStream_t s) {
    const int64_t n = (int64_t)jobs.size();
    if (n == 0) return PERC_OK;
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    int cus = 0;
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const bool two = tu.form == FORM_PERSIST2;
    // two steps per pass: the whole cross-section is the tile and its own outer range
    const int lds = (int)(two ? lds_total2(S.need.C, S.need.C) : lds_total(S.need.span_max));
    int grid = tu.grid;
    if (grid == 0)
        grid = cus * std::max(1, two ? persist2_resident_per_cu(tu.block, lds) : persist_resident_per_cu(tu.block, lds));
    for (int64_t j0 = 0; j0 < n;) {
        int64_t j1 = j0, words = 0;
        while (j1 < n) {
            const int64_t w = jobs[j1].bits ? 0 : bits_words(jobs[j1].lat->d);
            if (j1 > j0 && (words + w) * 4 > kPersistBitsBudget) break;
            words += w;
            ++j1;
        }
        PERC_TRY(run_persist_chunk(jobs, j0, j1, S, out, tu, grid, lds, s));
        j0 = j1;
    }
    return PERC_OK;
}

int validate_lat(const perc_lattice* lat) {
    if (!lat) return fail(PERC_EINVAL, "lattice is NULL");
    return PERC_OK;
}

// Run a list of jobs with outputs indexed by job (device pointers; steps required).
int run_jobs(const std::vector<HostJob>& jobs, BatchOut out, const perc_options* opt, hipStream_t s);

// Fibers the mixed form runs in the span form: those of several column tiles whose step
// over every tile and cell, which a persistent workgroup walks alone, is long (tiles x
// unit cells above kMixedWork). On the aspect-ratio sweep (W = 8..32, L = W..64 W) limits
// of 600 to 3,600 gave the same time within 2 %, 4-6 % below the span form alone; the
// near-cubic ablation fibers (at most 112) stay persistent, 27 % faster than split by
// width; so do fibers of one tile, however long (W = 3, L up to 3,072: 20 % faster than
// with their long ones in the span form, whose items of a 37-column tile are too small).
bool wide_fiber(const LatticeDesc& d) { return d.ntile > 1 && (int64_t)d.ntile * d.U > kMixedWork; }

// The mixed form: the jobs on short-walk fibers (wide_fiber false) in the persistent form,
// the others in the span form (opt's depth, block, grid and graph steps apply to the span
// part). The persistent part is one launch on a second stream, which runs beside the
// span part's steps on the caller's stream (the span form's short walks leave the device
// room); each part writes its outputs to a buffer of its own, scattered to the jobs'
// places on the caller's stream once both are done; group counts and the step-cap flag
// accumulate in the batch's own. A persistent workgroup walks its configuration's tiles
// and cells one after another, so it suits short walks; the span form spreads the tiles
// and cell ranges of long ones over workgroups.
int run_mixed(const std::vector<HostJob>& jobs, BatchOut out, const perc_options* opt, hipStream_t s) {
    std::vector<HostJob> part[2];
    std::vector<int64_t> idx;
    idx.reserve(jobs.size());
    for (int k = 0; k < 2; ++k)
        for (int64_t i = 0; i < (int64_t)jobs.size(); ++i)
            if (wide_fiber(jobs[i].lat->d) == (k == 1)) {
                part[k].push_back(jobs[i]);
                idx.push_back(i);
            }
    perc_options o[2] = {perc_options{FORM_PERSIST, 0, 0, 0, 0}, opt ? *opt : perc_options{}};
    o[1].form = FORM_SPAN;
    if (part[0].empty() || part[1].empty()) return run_jobs(jobs, out, &o[part[0].empty() ? 1 : 0], s);
    // the span part synchronises; checked before the side stream is tied to s
    if (stream_capturing(s)) return fail(PERC_EINVAL, "the mixed form synchronises; not capturable");
    const int64_t n = (int64_t)jobs.size();
    Arena ar;
    PERC_TRY(ar.reserve(Arena::need<int64_t>(n) + Arena::need<uint8_t>(n) + Arena::need<int32_t>(n) +
                            (out.hit ? Arena::need<float>(n) : 0), s));
    int64_t* d_idx = ar.take<int64_t>(n);
    uint8_t* t_perc = ar.take<uint8_t>(n);
    int32_t* t_steps = ar.take<int32_t>(n);
    float* t_hit = out.hit ? ar.take<float>(n) : nullptr;
    PERC_TRY(ar.check());
    HIP_TRY(hipMemcpyAsync(d_idx, idx.data(), sizeof(int64_t) * n, hipMemcpyHostToDevice, s));
    hipStream_t side = nullptr;
    PERC_TRY(side_stream(&side));
    hipEvent_t ev[2] = {nullptr, nullptr};
    for (hipEvent_t& e : ev) HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    BatchOut po[2] = {out, out};
    po[0].perc = t_perc;
    po[0].steps = t_steps;
    po[0].hit = t_hit;
    const int64_t n0 = (int64_t)part[0].size();
    po[1].perc = t_perc + n0;
    po[1].steps = t_steps + n0;
    po[1].hit = t_hit ? t_hit + n0 : nullptr;
    int rc[2] = {PERC_OK, PERC_OK};
    // the persistent part on the side stream, after everything enqueued so far on s
    hipError_t e = hipEventRecord(ev[0], s);
    if (e == hipSuccess) e = hipStreamWaitEvent(side, ev[0], 0);
    if (e == hipSuccess) {
        rc[0] = run_jobs(part[0], po[0], &o[0], side);
        e = hipEventRecord(ev[1], side);
        // the span part on s meanwhile; s then waits for the side stream
        if (e == hipSuccess && (rc[0] == PERC_OK || rc[0] == PERC_ECAP)) rc[1] = run_jobs(part[1], po[1], &o[1], s);
        if (e == hipSuccess) e = hipStreamWaitEvent(s, ev[1], 0);
        if (e != hipSuccess) (void)hipStreamSynchronize(side);  // no event: wait here instead
    }
    for (hipEvent_t ee : ev) (void)hipEventDestroy(ee);
    HIP_TRY(e);
    for (int k = 0; k < 2; ++k)
        if (rc[k] != PERC_OK && rc[k] != PERC_ECAP) return rc[k];
    HIP_TRY(launch_scatter_out(n, d_idx, t_perc, t_steps, t_hit, out.perc, out.steps, out.hit, s));
    return rc[0] != PERC_OK ? rc[0] : rc[1];
}

// Jobs on short-walk fibers, and the others.
void count_kinds(const std::vector<HostJob>& jobs, int64_t& n_narrow, int64_t& n_wide) {
    n_narrow = n_wide = 0;
    for (const HostJob& j : jobs) (wide_fiber(j.lat->d) ? n_wide : n_narrow) += 1;
}

int run_jobs(const std::vector<HostJob>& jobs, BatchOut out, const perc_options* opt, hipStream_t s) {
    if (opt && opt->form == FORM_MIXED) return run_mixed(jobs, out, opt, s);
    if (!opt || opt->form == FORM_AUTO) {
        // a batch of both kinds with many narrow fibers: each kind in its own form
        int64_t n_narrow, n_wide;
        count_kinds(jobs, n_narrow, n_wide);
        if (n_narrow >= 2048 && n_wide > 0) {
            perc_options o = opt ? *opt : perc_options{};
            o.form = FORM_MIXED;
            return run_mixed(jobs, out, &o, s);
        }
    }
    Shapes S;
    collect_shapes(jobs, S);
    TuneKey key{0, 0, 0};
    const bool one = S.lats.size() == 1;
    if (one) key = TuneKey{S.lats[0]->d.W, S.lats[0]->d.L, size_bucket((int64_t)jobs.size())};
    Tuning tu;
    PERC_TRY(resolve(S.need, S.max_state, (int64_t)jobs.size(), opt, tu, one ? &key : nullptr));
    PERC_TRY(device_shapes(S, tu.form == FORM_PERSIST2));
    if (tu.form == FORM_PERSIST || tu.form == FORM_PERSIST2) return run_persist(jobs, S, out, tu, s);
    return run_span(jobs, S, out, tu, s);
}

int inspect_impl(const perc_lattice* lat, const uint32_t* occ_bits, int64_t n_cfg, uint8_t* perc, int32_t* steps,
                 float* hit, const perc_options* opt, void* stream) {
    PERC_TRY(validate_lat(lat));
    if (n_cfg < 0) return fail(PERC_EINVAL, "n_cfg < 0");
    if (n_cfg == 0) return PERC_OK;
    if (!occ_bits || !perc) return fail(PERC_EINVAL, "occ_bits and perc must be device pointers");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    Arena ar;
    if (!steps) {
        PERC_TRY(ar.reserve(sizeof(int32_t) * n_cfg, s));
        steps = ar.take<int32_t>(n_cfg);
    }
    std::vector<HostJob> jobs(n_cfg);
    for (int64_t i = 0; i < n_cfg; ++i) jobs[i] = HostJob{lat, occ_bits + i * lat->d.words, 0, 0, 0, -1};
    BatchOut out;
    out.perc = perc;
    out.steps = steps;
    out.hit = hit;
    return run_jobs(jobs, out, opt, s);
}

int pi_impl(const perc_lattice* lat, double p, int64_t n_cfg, uint64_t seed, perc_pi_out* out,
            const perc_options* opt, void* stream) {
    PERC_TRY(validate_lat(lat));
    if (!out) return fail(PERC_EINVAL, "out is NULL");
    if (!(p >= 0.0 && p <= 1.0)) return fail(PERC_EINVAL, "p must be in [0, 1]");
    if (n_cfg < 0) return fail(PERC_EINVAL, "n_cfg < 0");
    out->n_perc = 0;
    out->pi = 0.0;
    if (n_cfg == 0) return PERC_OK;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const uint64_t thr = threshold_of(p);
    Arena ar;
    const size_t bytes = (out->bits ? 0 : Arena::align((size_t)n_cfg)) +
                         (out->steps ? 0 : Arena::align(sizeof(int32_t) * n_cfg)) + Arena::align(64);
    PERC_TRY(ar.reserve(bytes, s));
    BatchOut bo;
    bo.perc = out->bits ? out->bits : ar.take<uint8_t>(n_cfg);
    bo.steps = out->steps ? out->steps : ar.take<int32_t>(n_cfg);
    bo.hit = out->hit;
    // [0]: percolating count, [1]: step-cap flag of the persistent form
    unsigned long long* count = ar.take<unsigned long long>(2);
    PERC_TRY(ar.check());
    bo.cap = reinterpret_cast<uint32_t*>(count + 1);
    HIP_TRY(launch_fill_u32(reinterpret_cast<uint32_t*>(count), 4, 0u, s));
    std::vector<HostJob> jobs(n_cfg);
    for (int64_t i = 0; i < n_cfg; ++i) jobs[i] = HostJob{lat, nullptr, seed, (uint64_t)i, thr, -1};
    PERC_TRY(run_jobs(jobs, bo, opt, s));
    HIP_TRY(launch_count(bo.perc, n_cfg, count, s));
    unsigned long long host_count[2] = {0, 0};
    HIP_TRY(hipMemcpyAsync(host_count, count, sizeof(host_count), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (host_count[1]) return fail(PERC_ECAP, "a configuration reached the step cap");
    out->n_perc = (int64_t)host_count[0];
    out->pi = (double)host_count[0] / (double)n_cfg;
    return PERC_OK;
}

// Jobs of the C ABI to host jobs (validated).
int convert_jobs(const perc_job* jobs, int64_t n_jobs, int32_t n_groups, std::vector<HostJob>& hj) {
    hj.resize(n_jobs);
    for (int64_t j = 0; j < n_jobs; ++j) {
        const perc_job& x = jobs[j];
        PERC_TRY(validate_lat(x.lat));
        if (!x.occ_bits && !(x.p >= 0.0 && x.p <= 1.0)) return fail(PERC_EINVAL, "job p must be in [0, 1]");
        if (x.cfg < 0) return fail(PERC_EINVAL, "job cfg must be >= 0");
        if (x.group >= n_groups) return fail(PERC_EINVAL, "job group out of range");
        hj[j] = HostJob{x.lat, x.occ_bits, x.seed, (uint64_t)x.cfg, x.occ_bits ? 0 : threshold_of(x.p),
                        x.group < 0 ? -1 : x.group};
    }
    return PERC_OK;
}

// ---------------------------------------------------------------------------------
// Autotuning: time candidate execution settings on a sample batch.
// ---------------------------------------------------------------------------------
int autotune(const std::vector<HostJob>& hj, int64_t n_target, perc_options* best, double* best_ms, hipStream_t s) {
    Shapes S;
    collect_shapes(hj, S);
    const int32_t b0 = block_for(S.need);
    std::vector<perc_options> cands;
    for (int32_t depth : {32, 64, 80, 128}) {
        cands.push_back(perc_options{FORM_SPAN, depth, b0, 0, 16});
        if (b0 + 64 <= 1024) cands.push_back(perc_options{FORM_SPAN, depth, b0 + 64, 0, 16});
    }
    for (int32_t depth : {64, 128, 256}) cands.push_back(perc_options{FORM_PERSIST, depth, b0, 0, 0});
    if (S.need.C <= kWholeCols)
        for (int32_t depth : {64, 128}) cands.push_back(perc_options{FORM_PERSIST2, depth, 0, 0, 0});
    if (two_step_fits(S.need, b0))
        for (int32_t depth : {64, 128}) cands.push_back(perc_options{FORM_SPAN2, depth, b0, 0, 16});
    int64_t n_narrow, n_wide;
    count_kinds(hj, n_narrow, n_wide);
    if (n_narrow > 0 && n_wide > 0)
        for (int32_t depth : {64, 80}) cands.push_back(perc_options{FORM_MIXED, depth, 0, 0, 16});
    const int64_t n = (int64_t)hj.size();
    Arena ar;
    PERC_TRY(ar.reserve(Arena::align((size_t)n) + Arena::align(4 * (size_t)n), s));
    BatchOut out;
    out.perc = ar.take<uint8_t>(n);
    out.steps = ar.take<int32_t>(n);
    PERC_TRY(ar.check());
    double best_t = -1.0;
    perc_options best_o{};
    bool warm = false;
    for (const perc_options& o : cands) {
        double t_min = -1.0;
        for (int rep = 0; rep < (warm ? 2 : 3); ++rep) {
            HIP_TRY(hipStreamSynchronize(s));
            const auto t0 = std::chrono::steady_clock::now();
            const int rc = run_jobs(hj, out, &o, s);
            if (rc == PERC_EINVAL) break;  // a candidate these shapes cannot take (e.g. LDS)
            PERC_TRY(rc);
            HIP_TRY(hipStreamSynchronize(s));
            const double t = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
            if (!warm) {  // the first run of all pays one-time preparation
                warm = true;
                continue;
            }
            if (t_min < 0.0 || t < t_min) t_min = t;
        }
        if (t_min >= 0.0 && (best_t < 0.0 || t_min < best_t)) {
            best_t = t_min;
            best_o = o;
        }
    }
    if (best_t < 0.0) return fail(PERC_EINVAL, "no candidate setting runs these jobs");
    if (S.lats.size() == 1) {
        const LatticeDesc& d = S.lats[0]->d;
        Tuning t;
        t.form = best_o.form;
        t.depth = best_o.depth;
        t.block = best_o.block;
        t.graph_steps = best_o.graph_steps;
        t.grid = 0;
        std::lock_guard<std::mutex> g(g_tune_mu);
        g_tune[TuneKey{d.W, d.L, size_bucket(n_target > 0 ? n_target : n)}] = t;
    }
    if (best) *best = best_o;
    if (best_ms) *best_ms = best_t;
    return PERC_OK;
}

// ---------------------------------------------------------------------------------
// Serving: continuous batching of single inspections (see perc.h).
// ---------------------------------------------------------------------------------

// First-fit allocator of [0, capacity) in whole units, free blocks coalesced.
class RangeAlloc {
public:
    void reset(int64_t capacity) {
        free_.clear();
        if (capacity > 0) free_[0] = capacity;
        used_ = 0;
    }
    int64_t alloc(int64_t n) {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < n) continue;
            const int64_t off = it->first, rest = it->second - n;
            free_.erase(it);
            if (rest > 0) free_[off + n] = rest;
            used_ += n;
            return off;
        }
        return -1;
    }
    void release(int64_t off, int64_t n) {
        used_ -= n;
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    int64_t used() const { return used_; }

private:
    std::map<int64_t, int64_t> free_;
    int64_t used_ = 0;
};

// occupancy words of one request in the server pool (16-word granules)
int64_t server_bits_words(const LatticeDesc& d) { return (d.words + 15) & ~(int64_t)15; }

int64_t steady_ns() {
    return std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

struct ServerSlot {
    bool busy = false;
    perc_result res{};
    int64_t state_off = 0, state_words = 0, bits_off = 0, bits_n = 0;
    int32_t shape = -1;
    int64_t seq = 0;      // admission order
    bool cancel = false;  // cancelled while in flight: retired at the next tick
};

}  // namespace

struct perc_server {
    perc_server_config cfg{};
    hipStream_t s = nullptr;
    bool host_only = false;
    // device pools: state words (two FP32 buffers and the codes share offsets), occupancy
    char* mem = nullptr;
    float* ya = nullptr;
    float* yb = nullptr;
    uint8_t* code = nullptr;
    uint32_t* bits = nullptr;
    int64_t state_cap = 0, bits_cap = 0, pool_bytes = 0;
    RangeAlloc state_alloc, bits_alloc;
    // per-slot device arrays and the planner's work list
    SpanArgs a{};
    DevShape* d_shapes = nullptr;
    int32_t* d_slot_shape = nullptr;
    int64_t* d_slot_off = nullptr;
    const uint32_t** d_slot_bits = nullptr;
    Job* d_new_jobs = nullptr;
    uint32_t** d_new_bits = nullptr;
    int32_t* d_ids = nullptr;
    // pinned host staging: hdr (16), fin (max_slots), perc, steps, hit, upload of ids
    char* pin = nullptr;
    int32_t* h_hdr = nullptr;
    int32_t* h_fin = nullptr;
    uint8_t* h_perc = nullptr;
    int32_t* h_steps = nullptr;
    float* h_hit = nullptr;
    int32_t* h_ids = nullptr;
    Job* h_new_jobs = nullptr;
    uint32_t** h_new_bits = nullptr;
    CfgState* h_st = nullptr;
    // host mirrors
    std::vector<DevShape> shapes;
    std::vector<int32_t> shape_ref;
    std::map<std::pair<int32_t, int32_t>, int32_t> shape_of_wl;
    std::vector<int32_t> free_shapes;
    std::vector<int32_t> h_slot_shape;
    std::vector<int64_t> h_slot_off;
    std::vector<const uint32_t*> h_slot_bits;
    std::vector<ServerSlot> slots;
    std::vector<int32_t> free_slots;
    std::deque<perc_result> queue;
    std::deque<perc_result> done;
    int32_t n_act = 0;
    int64_t ticks = 0, completed = 0, admitted = 0, rejected = 0, cancelled = 0;
    hipGraphExec_t exec = nullptr;
};

namespace {

constexpr int32_t kServerMaxW = 128;

void server_release(perc_server* v) {
    if (!v) return;
    if (v->exec) (void)hipGraphExecDestroy(v->exec);
    if (v->mem) (void)hipFree(v->mem);
    if (v->pin) (void)hipHostFree(v->pin);
    delete v;
}

template <typename T>
T* carve(char*& p, int64_t n) {
    T* r = reinterpret_cast<T*>(p);
    p += ((int64_t)sizeof(T) * std::max<int64_t>(n, 1) + 255) & ~(int64_t)255;
    return r;
}

int server_init(perc_server* v, const perc_server_config* cfg, hipStream_t s) {
    v->cfg = cfg ? *cfg : perc_server_config{};
    perc_server_config& c = v->cfg;
    if (c.max_slots <= 0) c.max_slots = 1024;
    if (c.tick_steps <= 0) c.tick_steps = 16;
    if (c.max_w <= 0) c.max_w = 64;
    if (c.max_queue <= 0) c.max_queue = 1 << 20;
    if (c.lookahead < 0) return fail(PERC_EINVAL, "lookahead must be >= 0");
    if (c.max_slots > (1 << 20)) return fail(PERC_EINVAL, "max_slots must be <= 2^20");
    if (c.tick_steps > 4096) return fail(PERC_EINVAL, "tick_steps must be <= 4096");
    if (c.max_w > kServerMaxW) return fail(PERC_EINVAL, "max_w must be <= 128");
    v->s = s;
    v->host_only = c.host_only != 0;
    const int32_t M = c.max_slots;
    if (c.hbm_bytes <= 0) {
        if (v->host_only) return fail(PERC_EINVAL, "host_only needs an explicit hbm_bytes");
        size_t free_b = 0, total_b = 0;
        HIP_TRY(hipMemGetInfo(&free_b, &total_b));
        c.hbm_bytes = std::min<int64_t>((int64_t)((free_b + cache_idle_bytes()) / 2), 64ll << 30);
    }
    // pool: per state word 9 bytes (two FP32 buffers, and one byte of code region, of
    // which the four-bit codes use half), occupancy words an eighth of the state words (a
    // tube needs 1/32 of a word, rounded per request)
    const int64_t unit = 9 * 16 + 2 * 4;
    const int64_t blocks = c.hbm_bytes / unit;
    v->state_cap = blocks * 16;
    v->bits_cap = blocks * 2;
    v->pool_bytes = v->state_cap * 9 + v->bits_cap * 4;
    if (v->state_cap < 64) return fail(PERC_EINVAL, "hbm_bytes too small");
    v->state_alloc.reset(v->state_cap);
    v->bits_alloc.reset(v->bits_cap);
    v->slots.assign(M, ServerSlot{});
    for (int32_t b = M - 1; b >= 0; --b) v->free_slots.push_back(b);
    v->h_slot_shape.assign(M, 0);
    v->h_slot_off.assign(M, 0);
    v->h_slot_bits.assign(M, nullptr);
    if (v->host_only) return PERC_OK;

    // launch shape: one thread per column of the widest tile of any accepted width
    ShapeNeed nd;
    for (int32_t w = 0; w <= c.max_w; ++w) {
        std::string err;
        auto cs = column_set(w, err);
        if (!cs) return fail(PERC_EINVAL, err);
        nd.span_max = std::max(nd.span_max, cs->span_max);
        nd.tile_max = std::max(nd.tile_max, cs->tile_max);
        nd.C = std::max(nd.C, cs->C);
    }
    Tuning tu;
    perc_options o = c.opt;
    o.form = FORM_SPAN;
    PERC_TRY(resolve(nd, 0, 1, &o, tu, nullptr));
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    PERC_TRY(prepare(dev));
    // one device allocation for the pools and every per-slot array (carved below; each
    // piece rounded to 256 bytes)
    auto al = [](int64_t b) { return (std::max<int64_t>(b, 1) + 255) & ~(int64_t)255; };
    const int64_t bytes = al(4 * v->state_cap) * 2 + al(v->state_cap) + al(4 * v->bits_cap) +
                          al((int64_t)sizeof(DevShape) * M) + al(4ll * M) + al(8ll * M) + al(8ll * M) +
                          al((int64_t)sizeof(Job) * M) + al(8ll * M) + al(4ll * M) + al((int64_t)sizeof(CfgState) * M) +
                          al(4ll * M) * 2 + al(8ll * (M + 1)) + al(64) + al(4ll * M) + al(M) + al(4ll * M) * 2;
    PERC_TRY(device_alloc(reinterpret_cast<void**>(&v->mem), (size_t)bytes));
    char* p = v->mem;
    v->ya = carve<float>(p, v->state_cap);
    v->yb = carve<float>(p, v->state_cap);
    v->code = carve<uint8_t>(p, v->state_cap);
    v->bits = carve<uint32_t>(p, v->bits_cap);
    v->d_shapes = carve<DevShape>(p, M);
    v->d_slot_shape = carve<int32_t>(p, M);
    v->d_slot_off = carve<int64_t>(p, M);
    v->d_slot_bits = carve<const uint32_t*>(p, M);
    v->d_new_jobs = carve<Job>(p, M);
    v->d_new_bits = carve<uint32_t*>(p, M);
    v->d_ids = carve<int32_t>(p, M);
    SpanArgs& a = v->a;
    a = SpanArgs{};
    a.st = carve<CfgState>(p, M);
    a.active = carve<int32_t>(p, M);
    a.active2 = carve<int32_t>(p, M);
    a.chunk_off = carve<int64_t>(p, M + 1);
    a.hdr = carve<int32_t>(p, 16);
    a.fin = carve<int32_t>(p, M);
    a.out.perc = carve<uint8_t>(p, M);
    a.out.steps = carve<int32_t>(p, M);
    a.out.hit = carve<float>(p, M);
    a.shapes = v->d_shapes;
    a.slot_shape = v->d_slot_shape;
    a.slot_off = v->d_slot_off;
    a.slot_bits = v->d_slot_bits;
    a.ya = v->ya;
    a.yb = v->yb;
    a.code = v->code;
    a.work = nullptr;
    a.n_slot = M;
    a.depth = tu.depth;
    a.block = tu.block;
    a.grid = tu.grid ? tu.grid : kSpanGrid;
    a.lds = (int)lds_total(nd.span_max);
    a.resident = span_step_resident(a.block, a.lds);
    // an even tick runs pairs of step launches between plans
    a.pair = (kSpanPairs && v->cfg.tick_steps % 2 == 0) ? 1 : 0;
    HIP_TRY(launch_fill_u32(reinterpret_cast<uint32_t*>(a.hdr), 16, 0u, s));
    HIP_TRY(launch_fill_u32(reinterpret_cast<uint32_t*>(a.st), (int64_t)M * (int64_t)(sizeof(CfgState) / 4), 0u, s));
    const size_t pin_bytes =
        64 + (size_t)M * (4 + 1 + 4 + 4 + 4) + (size_t)M * (sizeof(Job) + sizeof(void*) + sizeof(CfgState)) + 1024;
    HIP_TRY(hipHostMalloc(reinterpret_cast<void**>(&v->pin), pin_bytes, hipHostMallocDefault));
    char* q = v->pin;
    v->h_hdr = reinterpret_cast<int32_t*>(q); q += 64;
    v->h_fin = reinterpret_cast<int32_t*>(q); q += (size_t)M * 4;
    v->h_steps = reinterpret_cast<int32_t*>(q); q += (size_t)M * 4;
    v->h_hit = reinterpret_cast<float*>(q); q += (size_t)M * 4;
    v->h_ids = reinterpret_cast<int32_t*>(q); q += (size_t)M * 4;
    q = reinterpret_cast<char*>(((uintptr_t)q + 15) & ~(uintptr_t)15);
    v->h_new_jobs = reinterpret_cast<Job*>(q); q += (size_t)M * sizeof(Job);
    v->h_new_bits = reinterpret_cast<uint32_t**>(q); q += (size_t)M * sizeof(void*);
    v->h_st = reinterpret_cast<CfgState*>(q); q += (size_t)M * sizeof(CfgState);
    v->h_perc = reinterpret_cast<uint8_t*>(q);
    HIP_TRY(hipStreamSynchronize(s));
    return PERC_OK;
}

int server_shape(perc_server* v, const LatticeDesc& d, int32_t& idx) {
    auto key = std::make_pair(d.W, d.L);
    auto it = v->shape_of_wl.find(key);
    if (it != v->shape_of_wl.end()) {
        idx = it->second;
        v->shape_ref[idx] += 1;
        return PERC_OK;
    }
    DevShape sh{};
    if (!v->host_only) PERC_TRY(shape_of(d, sh));
    if (!v->free_shapes.empty()) {
        idx = v->free_shapes.back();
        v->free_shapes.pop_back();
        v->shapes[idx] = sh;
        v->shape_ref[idx] = 1;
    } else {
        idx = (int32_t)v->shapes.size();
        v->shapes.push_back(sh);
        v->shape_ref.push_back(1);
    }
    v->shape_of_wl[key] = idx;
    return PERC_OK;
}

void server_unshape(perc_server* v, int32_t idx, int32_t W, int32_t L) {
    if (--v->shape_ref[idx] == 0) {
        v->shape_of_wl.erase(std::make_pair(W, L));
        v->free_shapes.push_back(idx);
    }
}

void server_retire(perc_server* v, int32_t b, int64_t now) {
    ServerSlot& sl = v->slots[b];
    sl.res.t_done_ns = now;
    if (sl.cancel) {
        sl.res.status = PERC_ECANCELED;
        sl.res.perc = 0;
        sl.res.steps = 0;
        sl.res.hit = 0.0f;
        v->cancelled += 1;
    } else {
        v->completed += 1;
    }
    v->done.push_back(sl.res);
    v->state_alloc.release(sl.state_off, sl.state_words);
    v->bits_alloc.release(sl.bits_off, sl.bits_n);
    server_unshape(v, sl.shape, sl.res.W, sl.res.L);
    sl.busy = false;
    sl.cancel = false;
    v->free_slots.push_back(b);
}

// Admit queued requests in queue order while a slot and pool room are free; a request
// that does not fit is passed over only while at most `lookahead` have been (0: strict
// FIFO, the first one that does not fit stops admission).
int server_admit(perc_server* v, std::vector<int32_t>& new_ids) {
    const int64_t now = steady_ns();
    int64_t passed = 0;
    auto it = v->queue.begin();
    while (it != v->queue.end() && !v->free_slots.empty()) {
        const perc_result& r = *it;
        LatticeDesc d;
        std::string err;
        if (!build_lattice(r.W, r.L, d, err)) return fail(PERC_EINVAL, err);
        const int64_t sw = slot_words(d), bw = server_bits_words(d);
        const int64_t so = v->state_alloc.alloc(sw);
        const int64_t bo = so < 0 ? -1 : v->bits_alloc.alloc(bw);
        if (so >= 0 && bo < 0) v->state_alloc.release(so, sw);
        if (bo < 0) {
            if (++passed > v->cfg.lookahead) break;
            ++it;
            continue;
        }
        int32_t idx = -1;
        PERC_TRY(server_shape(v, d, idx));
        const int32_t b = v->free_slots.back();
        v->free_slots.pop_back();
        ServerSlot& sl = v->slots[b];
        sl.busy = true;
        sl.res = r;
        sl.res.t_admit_ns = now;
        sl.state_off = so;
        sl.state_words = sw;
        sl.bits_off = bo;
        sl.bits_n = bw;
        sl.shape = idx;
        sl.seq = v->admitted++;
        sl.cancel = false;
        it = v->queue.erase(it);
        v->h_slot_shape[b] = idx;
        v->h_slot_off[b] = so;
        v->h_slot_bits[b] = v->bits ? v->bits + bo : nullptr;
        new_ids.push_back(b);
    }
    return PERC_OK;
}

int server_tick(perc_server* v) {
    std::vector<int32_t> new_ids;
    PERC_TRY(server_admit(v, new_ids));
    v->ticks += 1;
    if (v->host_only) {
        // fake executor: every request admitted before this tick completes now, in
        // admission order
        std::vector<std::pair<int64_t, int32_t>> fin;
        for (int32_t b = 0; b < (int32_t)v->slots.size(); ++b) {
            const ServerSlot& sl = v->slots[b];
            if (sl.busy && (sl.cancel || std::find(new_ids.begin(), new_ids.end(), b) == new_ids.end()))
                fin.emplace_back(sl.seq, b);
        }
        std::sort(fin.begin(), fin.end());
        const int64_t now = steady_ns();
        for (const auto& f : fin) {
            v->slots[f.second].res.status = PERC_OK;
            server_retire(v, f.second, now);
        }
        return (int)fin.size();
    }
    hipStream_t s = v->s;
    SpanArgs& a = v->a;
    // with the step profiler on, the tick launches its steps directly between HIP events
    // and the planner counts the tube slots it schedules (device word hdr[8..9])
    const bool prof = profiling();
    a.work = prof ? reinterpret_cast<unsigned long long*>(a.hdr + 8) : nullptr;
    StepTimer timer(prof);
    const int32_t k = (int32_t)new_ids.size();
    if (k > 0) {
        for (int32_t i = 0; i < k; ++i) {
            const int32_t b = new_ids[i];
            const perc_result& r = v->slots[b].res;
            v->h_ids[i] = b;
            v->h_new_jobs[i] = Job{nullptr, r.seed, r.cfg, threshold_of(r.p), v->h_slot_shape[b], -1};
            v->h_new_bits[i] = const_cast<uint32_t*>(v->h_slot_bits[b]);
        }
        HIP_TRY(hipMemcpyAsync(v->d_shapes, v->shapes.data(), sizeof(DevShape) * v->shapes.size(),
                               hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(v->d_slot_shape, v->h_slot_shape.data(), sizeof(int32_t) * v->slots.size(),
                               hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(v->d_slot_off, v->h_slot_off.data(), sizeof(int64_t) * v->slots.size(),
                               hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(v->d_slot_bits, v->h_slot_bits.data(), sizeof(void*) * v->slots.size(),
                               hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(v->d_ids, v->h_ids, sizeof(int32_t) * k, hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(v->d_new_jobs, v->h_new_jobs, sizeof(Job) * k, hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(v->d_new_bits, v->h_new_bits, sizeof(void*) * k, hipMemcpyHostToDevice, s));
        HIP_TRY(launch_sample_slots(v->d_shapes, v->d_new_jobs, k, v->d_new_bits, s));
        SpanArgs ai = a;
        ai.ids = v->d_ids;
        ai.n_ids = k;
        HIP_TRY(launch_span_init_only(ai, s));
        // the new slots join the active list; the planner gives them their initial
        // decision and lays out the next step for every active slot
        HIP_TRY(hipMemcpyAsync(a.active + v->n_act, v->h_ids, sizeof(int32_t) * k, hipMemcpyHostToDevice, s));
        v->h_hdr[0] = v->n_act + k;
        HIP_TRY(hipMemcpyAsync(a.hdr, v->h_hdr, sizeof(int32_t), hipMemcpyHostToDevice, s));
        HIP_TRY(launch_span_plan(a, s));
        v->n_act += k;
    }
    if (prof && (v->n_act > 0 || k > 0)) {
        for (int i = 0; i < v->cfg.tick_steps; i += a.pair ? 2 : 1) {
            HIP_TRY(timer.step(a, s));
            HIP_TRY(launch_span_plan(a, s));
        }
        HIP_TRY(launch_span_finish(a, s));
    } else if (v->n_act > 0 || k > 0) {
        if (!v->exec && s) {
            hipGraph_t graph = nullptr;
            HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
            hipError_t ce = hipSuccess;
            for (int i = 0; i < v->cfg.tick_steps && ce == hipSuccess; i += a.pair ? 2 : 1) {
                ce = launch_span_step(a, s);
                if (ce == hipSuccess && a.pair) ce = launch_span_step(second_of(a), s);
                if (ce == hipSuccess) ce = launch_span_plan(a, s);
            }
            hipError_t ee = hipStreamEndCapture(s, &graph);
            if (ce != hipSuccess) {
                if (graph) (void)hipGraphDestroy(graph);
                return hip_fail(ce, "capture");
            }
            if (ee != hipSuccess) return hip_fail(ee, "hipStreamEndCapture");
            hipError_t ie = hipGraphInstantiate(&v->exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (ie != hipSuccess) return hip_fail(ie, "hipGraphInstantiate");
        }
        if (v->exec) {
            HIP_TRY(hipGraphLaunch(v->exec, s));
        } else {
            for (int i = 0; i < v->cfg.tick_steps; i += a.pair ? 2 : 1) {
                HIP_TRY(launch_span_step(a, s));
                if (a.pair) HIP_TRY(launch_span_step(second_of(a), s));
                HIP_TRY(launch_span_plan(a, s));
            }
        }
        HIP_TRY(launch_span_finish(a, s));
    }
    const int32_t M = (int32_t)v->slots.size();
    HIP_TRY(hipMemcpyAsync(v->h_hdr, a.hdr, 64, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(v->h_fin, a.fin, sizeof(int32_t) * M, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(v->h_perc, a.out.perc, M, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(v->h_steps, a.out.steps, sizeof(int32_t) * M, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(v->h_hit, a.out.hit, sizeof(float) * M, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(v->h_st, a.st, sizeof(CfgState) * M, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    const int64_t now = steady_ns();
    const int32_t nfin = v->h_hdr[3];
    const bool cap = v->h_hdr[2] != 0;
    if (prof) {
        HIP_TRY(timer.collect());
        unsigned long long tubes = 0;
        std::memcpy(&tubes, v->h_hdr + 8, sizeof(tubes));
        if (tubes) {
            {
                std::lock_guard<std::mutex> g(g_prof.mu);
                g_prof.tube_steps += (int64_t)tubes;
            }
            static const unsigned long long kZero = 0;
            HIP_TRY(hipMemcpyAsync(a.hdr + 8, &kZero, sizeof(kZero), hipMemcpyHostToDevice, s));
            HIP_TRY(hipStreamSynchronize(s));
        }
    }
    for (int32_t i = 0; i < nfin; ++i) {
        const int32_t b = v->h_fin[i];
        ServerSlot& sl = v->slots[b];
        sl.res.perc = v->h_perc[b];
        sl.res.steps = v->h_steps[b];
        sl.res.hit = v->h_hit[b];
        sl.res.status = v->h_st[b].done == 2 ? PERC_ECAP : PERC_OK;
        server_retire(v, b, now);
    }
    // slots cancelled in flight: the planner of this tick dropped them from the work list
    int32_t ncan = 0;
    for (int32_t b = 0; b < M; ++b)
        if (v->slots[b].busy && v->slots[b].cancel) {
            server_retire(v, b, now);
            ++ncan;
        }
    v->n_act = v->h_hdr[0];
    if (nfin > 0 || cap) {
        v->h_hdr[2] = 0;
        v->h_hdr[3] = 0;
        HIP_TRY(hipMemcpyAsync(a.hdr + 2, v->h_hdr + 2, 2 * sizeof(int32_t), hipMemcpyHostToDevice, s));
        HIP_TRY(hipStreamSynchronize(s));
    }
    return nfin + ncan;
}

int server_submit(perc_server* v, int32_t W, int32_t L, double p, uint64_t seed, uint64_t cfg, uint64_t tag,
                  int64_t t_arrive) {
    if (W < 0 || W > v->cfg.max_w) return fail(PERC_EINVAL, "W outside [0, max_w]");
    if (!(p >= 0.0 && p <= 1.0)) return fail(PERC_EINVAL, "p must be in [0, 1]");
    LatticeDesc d;
    std::string err;
    if (!build_lattice(W, L, d, err)) return fail(PERC_EINVAL, err);
    if (slot_words(d) > v->state_cap || server_bits_words(d) > v->bits_cap) {
        v->rejected += 1;
        return fail(PERC_EBUSY, "the request's resident state exceeds the server pool");
    }
    if ((int64_t)v->queue.size() >= v->cfg.max_queue) {
        v->rejected += 1;
        return fail(PERC_EBUSY, "the request queue is full");
    }
    perc_result r{};
    r.tag = tag;
    r.W = W;
    r.L = L;
    r.p = p;
    r.seed = seed;
    r.cfg = cfg;
    r.t_arrive_ns = t_arrive >= 0 ? t_arrive : steady_ns();
    v->queue.push_back(r);
    return PERC_OK;
}

int server_cancel(perc_server* v, uint64_t tag) {
    int n = 0;
    const int64_t now = steady_ns();
    for (auto it = v->queue.begin(); it != v->queue.end();) {
        if (it->tag != tag) {
            ++it;
            continue;
        }
        perc_result r = *it;
        r.status = PERC_ECANCELED;
        r.t_admit_ns = now;
        r.t_done_ns = now;
        v->done.push_back(r);
        v->cancelled += 1;
        it = v->queue.erase(it);
        ++n;
    }
    for (int32_t b = 0; b < (int32_t)v->slots.size(); ++b) {
        ServerSlot& sl = v->slots[b];
        if (!sl.busy || sl.cancel || sl.res.tag != tag) continue;
        sl.cancel = true;
        ++n;
        if (v->host_only) continue;
        // between ticks no device work is in flight and the slot is undecided; marking it
        // done makes the next planner drop it from the work list without a decision
        static const int32_t kCancelled = 5;
        HIP_TRY(hipMemcpyAsync(&v->a.st[b].done, &kCancelled, sizeof(int32_t), hipMemcpyHostToDevice, v->s));
    }
    if (n && !v->host_only) HIP_TRY(hipStreamSynchronize(v->s));
    return n;
}

// Work buffers of the single-configuration entry points: the codes of occ_bits and its
// forward initial state in ya, yb and the detector words zero, in the plain layout.
struct OneRun {
    Arena ar;
    DevShape sh;
    float* ya = nullptr;
    float* yb = nullptr;
    uint8_t* code = nullptr;
    float* det = nullptr;
    uint32_t* det_r = nullptr;
    int32_t depth = 0, block = 0;
    int64_t stride = 0, n = 1;  // state words per configuration, configurations
};

int one_setup(const perc_lattice* lat, const uint32_t* occ_bits, hipStream_t s, OneRun& r, int64_t n = 1) {
    const LatticeDesc& d = lat->d;
    ShapeNeed nd;
    nd.span_max = d.span_max;
    nd.tile_max = d.tile_max;
    nd.C = d.C;
    nd.items = (int64_t)d.U * d.ntile;
    r.block = block_for(nd);
    PERC_TRY(check_walk(nd, r.block));
    r.depth = cells_for(nd, n > 1 ? FORM_SPAN : FORM_PLAIN);
    PERC_TRY(shape_for(lat, r.sh));
    const int64_t cw = slot_words(d);
    r.stride = cw;
    r.n = n;
    PERC_TRY(r.ar.reserve(Arena::align(sizeof(float) * cw * n) * 2 + Arena::align((size_t)(cw * n)) +
                              Arena::align(sizeof(CfgState) * n) + Arena::align(sizeof(DevShape)) +
                              Arena::align(sizeof(int64_t) * (n + 1)) * 2 + Arena::align(sizeof(int32_t) * n) +
                              Arena::align(sizeof(void*) * n) + Arena::align(64) * 4,
                          s));
    Arena& ar = r.ar;
    r.ya = ar.take<float>(cw * n);
    r.yb = ar.take<float>(cw * n);
    r.code = ar.take<uint8_t>(cw * n);
    CfgState* st = ar.take<CfgState>(n);
    DevShape* d_shape = ar.take<DevShape>(1);
    r.det = ar.take<float>(2);
    r.det_r = reinterpret_cast<uint32_t*>(r.det + 1);
    int32_t* hdr = ar.take<int32_t>(16);
    int32_t* slot_shape = ar.take<int32_t>(n);
    int64_t* slot_off = ar.take<int64_t>(n + 1);
    const uint32_t** slot_bits = ar.take<const uint32_t*>(n);
    int64_t* chunk_off = ar.take<int64_t>(n + 1);
    PERC_TRY(ar.check());
    std::vector<int64_t> h_off(n);
    std::vector<const uint32_t*> h_bits(n);
    for (int64_t i = 0; i < n; ++i) {
        h_off[i] = i * cw;
        h_bits[i] = occ_bits + i * d.words;
    }
    HIP_TRY(hipMemcpyAsync(d_shape, &r.sh, sizeof(DevShape), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(slot_bits, h_bits.data(), sizeof(void*) * n, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(slot_off, h_off.data(), sizeof(int64_t) * n, hipMemcpyHostToDevice, s));
    HIP_TRY(launch_fill_u32(reinterpret_cast<uint32_t*>(r.ya), cw * n, 0u, s));
    HIP_TRY(launch_fill_u32(reinterpret_cast<uint32_t*>(r.yb), cw * n, 0u, s));
    HIP_TRY(launch_fill_u32(reinterpret_cast<uint32_t*>(r.det), 2, 0u, s));
    HIP_TRY(launch_fill_u32(reinterpret_cast<uint32_t*>(hdr), 16, 0u, s));
    HIP_TRY(launch_fill_u32(reinterpret_cast<uint32_t*>(slot_shape), n, 0u, s));
    // the host vectors must outlive the copies above
    HIP_TRY(hipStreamSynchronize(s));
    SpanArgs a{};
    a.shapes = d_shape;
    a.slot_shape = slot_shape;
    a.slot_off = slot_off;
    a.slot_bits = slot_bits;
    a.ya = r.ya;
    a.yb = r.yb;
    a.code = r.code;
    a.st = st;
    a.chunk_off = chunk_off;
    a.hdr = hdr;
    a.n_slot = (int32_t)n;
    a.depth = r.depth;
    a.block = r.block;
    a.grid = (int)std::min<int64_t>(((d.U + r.depth - 1) / r.depth) * (int64_t)d.ntile * n, 4096);
    a.lds = (int)lds_total(d.span_max);
    HIP_TRY(launch_span_init_only(a, s));
    return PERC_OK;
}

// ---------------------------------------------------------------------------------
// The inspection in the span form with every work buffer carved from the library's
// fixed per-device array (perc_inspect_noalloc): no device, pinned or pool allocation,
// no graph; the host polls the planner's header with plain copies.
// ---------------------------------------------------------------------------------
struct Carver {
    char* base;
    size_t size, used = 0;
    template <typename T>
    T* take(size_t count) {
        T* p = reinterpret_cast<T*>(base + used);
        used += Arena::align(sizeof(T) * std::max<size_t>(count, 1));
        return p;
    }
    bool fits() const { return used <= size; }
};

int noalloc_impl(const perc_lattice* lat, const uint32_t* occ_bits, int64_t n_cfg, uint8_t* perc, int32_t* steps,
                 float* hit, hipStream_t s) {
    PERC_TRY(validate_lat(lat));
    if (n_cfg < 0) return fail(PERC_EINVAL, "n_cfg < 0");
    if (n_cfg == 0) return PERC_OK;
    if (!occ_bits || !perc) return fail(PERC_EINVAL, "occ_bits and perc must be device pointers");
    if (stream_capturing(s)) return fail(PERC_EINVAL, "the inspection synchronises; not capturable");
    const LatticeDesc& d = lat->d;
    const ColumnSet& cs = *d.cs;
    ShapeNeed nd;
    nd.span_max = d.span_max;
    nd.tile_max = d.tile_max;
    nd.C = d.C;
    nd.items = (int64_t)d.U * d.ntile;
    const int32_t block = block_for(nd);
    PERC_TRY(check_walk(nd, block));
    void* region = nullptr;
    size_t region_bytes = 0;
    HIP_TRY(scratch_region(&region, &region_bytes));
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    PERC_TRY(prepare(dev));
    // tables of the shape, then the slots of one wave
    Carver cv{reinterpret_cast<char*>(region), region_bytes};
    DevShape* d_shape = cv.take<DevShape>(1);
    uint32_t* d_nboff = cv.take<uint32_t>(cs.contact.size());
    uint16_t* d_lanes = cv.take<uint16_t>(cs.lanes.size());
    int32_t* d_tile = cv.take<int32_t>(cs.tile.size());
    int32_t* d_rank = cv.take<int32_t>(cs.rank.size());
    int32_t* d_sig = cv.take<int32_t>(cs.sig.size());
    int32_t* d_hdr = cv.take<int32_t>(16);
    const size_t fixed = cv.used;
    const int64_t sw = slot_words(d);
    // bytes of one wave of nb slots, in the order the wave carves them below
    auto wave_bytes = [&](int64_t nb) {
        auto al = [](size_t b) { return Arena::align(std::max<size_t>(b, 1)); };
        const size_t n = (size_t)nb;
        return al(sizeof(float) * sw * n) * 2 + al((size_t)sw * n) + al(sizeof(CfgState) * n) +
               al(sizeof(int32_t) * n) * 3 + al(sizeof(int64_t) * (n + 1)) * 2 + al(sizeof(void*) * n) +
               (steps ? 0 : al(sizeof(int32_t) * n));
    };
    if (fixed + wave_bytes(1) > region_bytes)
        return fail(PERC_EINVAL, "one configuration of this fiber needs " + std::to_string(fixed + wave_bytes(1)) +
                                     " bytes of work memory, more than the fixed " + std::to_string(region_bytes));
    // configurations per wave: as many as the array holds (bisection on the exact carve)
    int64_t lo = 1, hi = std::min<int64_t>(n_cfg, 1 << 16);
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) / 2;
        if (fixed + wave_bytes(mid) <= region_bytes) lo = mid; else hi = mid - 1;
    }
    const int64_t per_wave = lo;
    DevShape sh;
    sh.nboff = d_nboff;
    sh.lanes = d_lanes;
    sh.lane_stride = cs.lane_stride;
    sh.tile = d_tile;
    sh.rank = d_rank;
    sh.sig = d_sig;
    sh.nboff2 = nullptr;
    sh.tile2 = nullptr;
    sh.C = d.C; sh.CP = d.CP; sh.U = d.U; sh.L = d.L;
    sh.ntile = d.ntile; sh.span_max = d.span_max; sh.tile_max = d.tile_max; sh.W = d.W;
    sh.ends = d.ends;
    sh.span2_max = 0;
    sh.N = d.N; sh.words = d.words;
    HIP_TRY(hipMemcpyAsync(d_shape, &sh, sizeof(DevShape), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(d_nboff, cs.contact.data(), sizeof(uint32_t) * cs.contact.size(), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(d_lanes, cs.lanes.data(), sizeof(uint16_t) * cs.lanes.size(), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(d_tile, cs.tile.data(), sizeof(int32_t) * cs.tile.size(), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(d_rank, cs.rank.data(), sizeof(int32_t) * cs.rank.size(), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(d_sig, cs.sig.data(), sizeof(int32_t) * cs.sig.size(), hipMemcpyHostToDevice, s));
    const int lds = (int)lds_total(d.span_max);
    const int32_t resident = span_step_resident(block, lds);
    for (int64_t w0 = 0; w0 < n_cfg; w0 += per_wave) {
        const int32_t nb = (int32_t)std::min<int64_t>(per_wave, n_cfg - w0);
        Carver wv{reinterpret_cast<char*>(region) + fixed, region_bytes - fixed};
        SpanArgs a{};
        a.shapes = d_shape;
        a.ya = wv.take<float>(sw * nb);
        a.yb = wv.take<float>(sw * nb);
        a.code = wv.take<uint8_t>(sw * nb);
        a.st = wv.take<CfgState>(nb);
        a.active = wv.take<int32_t>(nb);
        a.active2 = wv.take<int32_t>(nb);
        int32_t* slot_shape = wv.take<int32_t>(nb);
        a.chunk_off = wv.take<int64_t>(nb + 1);
        int64_t* slot_off = wv.take<int64_t>(nb + 1);
        const uint32_t** slot_bits = wv.take<const uint32_t*>(nb);
        int32_t* own_steps = steps ? nullptr : wv.take<int32_t>(nb);
        if (!wv.fits()) return fail(PERC_EINVAL, "work memory carve exceeds the fixed array");
        a.slot_shape = slot_shape;
        a.slot_off = slot_off;
        a.slot_bits = slot_bits;
        a.hdr = d_hdr;
        a.work = reinterpret_cast<unsigned long long*>(d_hdr + 8);
        a.out.perc = perc + w0;
        a.out.steps = steps ? steps + w0 : own_steps;
        a.out.hit = hit ? hit + w0 : nullptr;
        a.n_slot = nb;
        a.depth = 64;
        a.block = block;
        a.grid = kSpanGrid;
        a.lds = lds;
        a.pair = kSpanPairs ? 1 : 0;
        a.resident = resident;
        HIP_TRY(launch_slot_table(slot_shape, slot_off, slot_bits, nb, sw, occ_bits + w0 * d.words, d.words, s));
        HIP_TRY(launch_fill_u32(reinterpret_cast<uint32_t*>(d_hdr), 16, 0u, s));
        HIP_TRY(launch_span_init(a, s));
        int32_t h[16];
        int reps = 1;
        for (;;) {
            HIP_TRY(hipMemcpyAsync(h, d_hdr, sizeof(h), hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
            if (h[0] == 0) break;
            for (int i = 0; i < 8 * reps; ++i) {
                HIP_TRY(launch_span_step(a, s));
                if (a.pair) HIP_TRY(launch_span_step(second_of(a), s));
                HIP_TRY(launch_span_plan(a, s));
            }
            reps = std::min(reps * 2, 8);
        }
        if (h[2]) return fail(PERC_ECAP, "a configuration reached the step cap");
        HIP_TRY(launch_span_finish(a, s));
    }
    // the next call may overwrite the array: the work of this one ends first
    HIP_TRY(hipStreamSynchronize(s));
    return PERC_OK;
}

}  // namespace

// =================================================================================
// extern "C" entry points
// =================================================================================

extern "C" {

perc_lattice* perc_lattice_create_ex(int32_t W, int32_t L, int32_t flags) {
    if (flags & ~PERC_LATTICE_NO_END_CONTACTS) {
        g_err = "unknown lattice flags";
        return nullptr;
    }
    perc_lattice* lat = new (std::nothrow) perc_lattice();
    if (!lat) {
        g_err = "out of host memory";
        return nullptr;
    }
    std::string err;
    if (!build_lattice(W, L, lat->d, err)) {
        g_err = err;
        delete lat;
        return nullptr;
    }
    lat->d.ends = (flags & PERC_LATTICE_NO_END_CONTACTS) ? 0 : 1;
    return lat;
}

perc_lattice* perc_lattice_create(int32_t W, int32_t L) { return perc_lattice_create_ex(W, L, 0); }

void perc_lattice_destroy(perc_lattice* lat) { delete lat; }

int64_t perc_lattice_sites(const perc_lattice* lat) { return lat ? lat->d.N : -1; }
int64_t perc_lattice_words(const perc_lattice* lat) { return lat ? lat->d.words : -1; }
int32_t perc_lattice_columns(const perc_lattice* lat) { return lat ? lat->d.C : -1; }
int64_t perc_lattice_state_bytes(const perc_lattice* lat) { return lat ? slot_words(lat->d) * 9 : -1; }

int perc_site_coord(const perc_lattice* lat, int64_t s, int32_t* q, int32_t* r, int32_t* k) {
    PERC_TRY(validate_lat(lat));
    const LatticeDesc& d = lat->d;
    if (s < 0 || s >= d.N) return fail(PERC_EINVAL, "site index out of range");
    const ColumnSet& cs = *d.cs;
    const int64_t u = s / d.C;
    const int32_t c = cs.by_rank[s - u * d.C];
    if (q) *q = cs.q[c];
    if (r) *r = cs.r[c];
    if (k) *k = (int32_t)(3 * u + cs.sig[c]);
    return PERC_OK;
}

int perc_site_neighbors(const perc_lattice* lat, int64_t s, int64_t* nbr, int32_t* count) {
    PERC_TRY(validate_lat(lat));
    const LatticeDesc& d = lat->d;
    if (s < 0 || s >= d.N || !nbr || !count) return fail(PERC_EINVAL, "bad site or NULL output");
    const ColumnSet& cs = *d.cs;
    const int64_t u = s / d.C;
    const int32_t c = cs.by_rank[s - u * d.C];
    std::vector<int64_t> out;
    auto add = [&](int64_t uu, int32_t cc) {
        if (uu < 0 || uu >= d.U || cc >= d.C) return;
        const int64_t t = uu * d.C + cs.rank[cc];
        if (t < d.N) out.push_back(t);
    };
    for (int i = 0; i < kSide; ++i) {
        const int32_t v = cs.nb[(size_t)i * d.C + c];
        add(u + ((v & 3) - 1), v >> 2);
    }
    if (d.ends) {
        add(u - 1, c);
        add(u + 1, c);
    }
    std::sort(out.begin(), out.end());
    *count = (int32_t)out.size();
    for (size_t i = 0; i < out.size(); ++i) nbr[i] = out[i];
    return PERC_OK;
}

const char* perc_last_error(void) { return g_err.c_str(); }

int perc_profile_enable(int32_t on) {
    std::lock_guard<std::mutex> g(g_prof.mu);
    g_prof.on = on != 0;
    g_prof.launches = 0;
    g_prof.ms = 0.0;
    g_prof.tube_steps = 0;
    g_prof.p_launches = 0;
    g_prof.p_ms = 0.0;
    g_prof.p_tube_steps = 0;
    return PERC_OK;
}

int perc_profile_read(perc_profile* out) {
    if (!out) return fail(PERC_EINVAL, "out is NULL");
    std::lock_guard<std::mutex> g(g_prof.mu);
    out->step_launches = g_prof.launches;
    out->step_ms = g_prof.ms;
    out->tube_steps = g_prof.tube_steps;
    out->persist_launches = g_prof.p_launches;
    out->persist_ms = g_prof.p_ms;
    out->persist_tube_steps = g_prof.p_tube_steps;
    return PERC_OK;
}

int perc_sample(const perc_lattice* lat, double p, uint64_t seed, int64_t cfg0, int64_t n_cfg, uint32_t* occ_bits,
                void* stream) {
    PERC_TRY(validate_lat(lat));
    if (!(p >= 0.0 && p <= 1.0)) return fail(PERC_EINVAL, "p must be in [0, 1]");
    if (n_cfg < 0 || cfg0 < 0) return fail(PERC_EINVAL, "n_cfg and cfg0 must be >= 0");
    if (n_cfg == 0) return PERC_OK;
    if (!occ_bits) return fail(PERC_EINVAL, "occ_bits is NULL");
    DevShape sh;
    PERC_TRY(shape_for(lat, sh));
    HIP_TRY(launch_sample(sh, occ_bits, n_cfg, (uint64_t)cfg0, threshold_of(p), seed,
                          reinterpret_cast<hipStream_t>(stream)));
    return PERC_OK;
}

int perc_sample_fixed(const perc_lattice* lat, double p, uint64_t seed, int64_t cfg0, int64_t n_cfg,
                      uint32_t* occ_bits, void* stream) {
    PERC_TRY(validate_lat(lat));
    if (!(p >= 0.0 && p <= 1.0)) return fail(PERC_EINVAL, "p must be in [0, 1]");
    if (n_cfg < 0 || cfg0 < 0) return fail(PERC_EINVAL, "n_cfg and cfg0 must be >= 0");
    if (n_cfg == 0) return PERC_OK;
    if (!occ_bits) return fail(PERC_EINVAL, "occ_bits is NULL");
    DevShape sh;
    PERC_TRY(shape_for(lat, sh));
    const int64_t K = (int64_t)std::floor((double)lat->d.N * p + 0.5);
    HIP_TRY(launch_sample_fixed(sh, occ_bits, n_cfg, (uint64_t)cfg0, K, seed, reinterpret_cast<hipStream_t>(stream)));
    return PERC_OK;
}

int perc_inspect(const perc_lattice* lat, const uint32_t* occ_bits, int64_t n_cfg, uint8_t* perc, int32_t* steps,
                 void* stream) {
    return inspect_impl(lat, occ_bits, n_cfg, perc, steps, nullptr, nullptr, stream);
}

int perc_inspect_ex(const perc_lattice* lat, const uint32_t* occ_bits, int64_t n_cfg, uint8_t* perc, int32_t* steps,
                    float* hit, const perc_options* opt, void* stream) {
    return inspect_impl(lat, occ_bits, n_cfg, perc, steps, hit, opt, stream);
}

int perc_inspect_noalloc(const perc_lattice* lat, const uint32_t* occ_bits, int64_t n_cfg, uint8_t* perc,
                         int32_t* steps, float* hit, void* stream) {
    return noalloc_impl(lat, occ_bits, n_cfg, perc, steps, hit, reinterpret_cast<hipStream_t>(stream));
}

int perc_pi(const perc_lattice* lat, double p, int64_t n_cfg, uint64_t seed, perc_pi_out* out, void* stream) {
    return pi_impl(lat, p, n_cfg, seed, out, nullptr, stream);
}

int perc_pi_ex(const perc_lattice* lat, double p, int64_t n_cfg, uint64_t seed, perc_pi_out* out,
               const perc_options* opt, void* stream) {
    return pi_impl(lat, p, n_cfg, seed, out, opt, stream);
}

int perc_batch(const perc_job* jobs, int64_t n_jobs, uint8_t* perc, int32_t* steps, float* hit, int64_t* group_count,
               int32_t n_groups, const perc_options* opt, void* stream) {
    if (n_jobs < 0 || n_groups < 0) return fail(PERC_EINVAL, "n_jobs and n_groups must be >= 0");
    if (n_groups > 0 && !group_count) return fail(PERC_EINVAL, "group_count is NULL");
    if (n_jobs == 0) {
        for (int32_t g = 0; g < n_groups; ++g) group_count[g] = 0;
        return PERC_OK;
    }
    if (!jobs || !perc) return fail(PERC_EINVAL, "jobs and perc must not be NULL");
    std::vector<HostJob> hj;
    PERC_TRY(convert_jobs(jobs, n_jobs, n_groups, hj));
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    Arena ar;
    PERC_TRY(ar.reserve(Arena::align(sizeof(int32_t) * n_jobs) + Arena::align(8 * (size_t)(n_groups + 1)), s));
    BatchOut out;
    out.perc = perc;
    int32_t* own_steps = ar.take<int32_t>(n_jobs);
    out.steps = steps ? steps : own_steps;
    out.hit = hit;
    // the group counts, then the step-cap flag of the persistent form (read when the call
    // is synchronous)
    unsigned long long* d_groups = ar.take<unsigned long long>(n_groups + 1);
    PERC_TRY(ar.check());
    if (n_groups > 0) {
        HIP_TRY(launch_fill_u32(reinterpret_cast<uint32_t*>(d_groups), 2 * (int64_t)(n_groups + 1), 0u, s));
        out.group_count = d_groups;
        out.cap = reinterpret_cast<uint32_t*>(d_groups + n_groups);
    }
    PERC_TRY(run_jobs(hj, out, opt, s));
    if (n_groups > 0) {
        std::vector<unsigned long long> h(n_groups + 1);
        HIP_TRY(hipMemcpyAsync(h.data(), d_groups, 8 * (size_t)(n_groups + 1), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (h[n_groups]) return fail(PERC_ECAP, "a configuration reached the step cap");
        for (int32_t g = 0; g < n_groups; ++g) group_count[g] = (int64_t)h[g];
    }
    return PERC_OK;
}

int perc_state_after(const perc_lattice* lat, const uint32_t* occ_bits, int32_t K, float* x_out, uint8_t* reach_out,
                     void* stream) {
    PERC_TRY(validate_lat(lat));
    if (K < 0) return fail(PERC_EINVAL, "K < 0");
    if (!occ_bits || !x_out || !reach_out) return fail(PERC_EINVAL, "NULL device pointer");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    OneRun r;
    PERC_TRY(one_setup(lat, occ_bits, s, r));
    float* cur = r.ya;
    float* nxt = r.yb;
    for (int32_t m = 0; m < K; ++m) {
        HIP_TRY(launch_far_sum(r.sh, cur, r.det, r.det_r, s));
        HIP_TRY(launch_chunk_step(r.sh, cur, nxt, r.code, r.depth, r.block, s));
        std::swap(cur, nxt);
    }
    HIP_TRY(launch_export(r.sh, cur, r.code, r.det, r.det_r, x_out, reach_out, s));
    return PERC_OK;
}

int perc_first_passage(const perc_lattice* lat, const uint32_t* occ_bits, int32_t M, float* f_out, void* stream) {
    return perc_first_passage_batch(lat, occ_bits, 1, M, f_out, stream);
}

int perc_first_passage_batch(const perc_lattice* lat, const uint32_t* occ_bits, int64_t n_cfg, int32_t M, float* f_out,
                             void* stream) {
    PERC_TRY(validate_lat(lat));
    if (M < 1) return fail(PERC_EINVAL, "M < 1");
    if (n_cfg < 0 || n_cfg > (1 << 20)) return fail(PERC_EINVAL, "n_cfg must be in [0, 2^20]");
    if (n_cfg == 0) return PERC_OK;
    if (!occ_bits || !f_out) return fail(PERC_EINVAL, "NULL device pointer");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    OneRun r;
    PERC_TRY(one_setup(lat, occ_bits, s, r, n_cfg));
    const int n = (int)n_cfg;
    HIP_TRY(launch_backward_init(r.sh, r.code, r.ya, r.stride, n, s));
    float* cur = r.ya;
    float* nxt = r.yb;
    for (int32_t m = 1; m < M; ++m) {
        HIP_TRY(launch_multi_step(r.sh, cur, nxt, r.code, r.stride, n, r.depth, r.block, s));
        std::swap(cur, nxt);
    }
    HIP_TRY(launch_export_raw(r.sh, cur, f_out, r.stride, n, s));
    return PERC_OK;
}

int perc_steps_hist(const uint8_t* perc, const int32_t* steps, int64_t n, int32_t nbins, uint64_t* hist,
                    void* stream) {
    if (n < 0) return fail(PERC_EINVAL, "n < 0");
    if (nbins < 1) return fail(PERC_EINVAL, "nbins < 1");
    if (!hist || (n > 0 && (!perc || !steps))) return fail(PERC_EINVAL, "NULL device pointer");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    HIP_TRY(launch_steps_hist(perc, steps, n, nbins, reinterpret_cast<unsigned long long*>(hist), s));
    return PERC_OK;
}

perc_server* perc_server_create(const perc_server_config* cfg, void* stream) {
    perc_server* v = new (std::nothrow) perc_server();
    if (!v) {
        g_err = "out of host memory";
        return nullptr;
    }
    if (server_init(v, cfg, reinterpret_cast<hipStream_t>(stream)) != PERC_OK) {
        server_release(v);
        return nullptr;
    }
    return v;
}

void perc_server_destroy(perc_server* srv) {
    if (srv && srv->s && !srv->host_only) (void)hipStreamSynchronize(srv->s);
    server_release(srv);
}

int perc_server_submit(perc_server* srv, int32_t W, int32_t L, double p, uint64_t seed, uint64_t cfg, uint64_t tag,
                       int64_t t_arrive_ns) {
    if (!srv) return fail(PERC_EINVAL, "server is NULL");
    return server_submit(srv, W, L, p, seed, cfg, tag, t_arrive_ns);
}

int perc_server_cancel(perc_server* srv, uint64_t tag) {
    if (!srv) return fail(PERC_EINVAL, "server is NULL");
    return server_cancel(srv, tag);
}

int perc_server_tick(perc_server* srv) {
    if (!srv) return fail(PERC_EINVAL, "server is NULL");
    return server_tick(srv);
}

int perc_server_poll(perc_server* srv, perc_result* out, int32_t max) {
    if (!srv || (!out && max > 0) || max < 0) return fail(PERC_EINVAL, "bad poll arguments");
    int32_t n = 0;
    while (n < max && !srv->done.empty()) {
        out[n++] = srv->done.front();
        srv->done.pop_front();
    }
    return n;
}

int perc_server_stats_read(const perc_server* srv, perc_server_stats* out) {
    if (!srv || !out) return fail(PERC_EINVAL, "NULL argument");
    out->queued = (int64_t)srv->queue.size();
    out->in_flight = (int64_t)(srv->slots.size() - srv->free_slots.size());
    out->completed = srv->completed;
    out->ticks = srv->ticks;
    out->pool_bytes = srv->pool_bytes;
    out->pool_used_bytes = srv->state_alloc.used() * 9 + srv->bits_alloc.used() * 4;
    out->rejected = srv->rejected;
    out->cancelled = srv->cancelled;
    return PERC_OK;
}

int perc_server_run(perc_server* srv, const perc_request* reqs, int64_t n, perc_result* out) {
    if (!srv || n < 0 || (n > 0 && (!reqs || !out))) return fail(PERC_EINVAL, "bad run arguments");
    for (int64_t i = 1; i < n; ++i)
        if (reqs[i].t_arrive_ns < reqs[i - 1].t_arrive_ns) return fail(PERC_EINVAL, "arrivals must be non-decreasing");
    const int64_t t0 = steady_ns();
    int64_t next = 0, got = 0;
    while (got < n) {
        const int64_t now = steady_ns();
        while (next < n && t0 + reqs[next].t_arrive_ns <= now) {
            const perc_request& q = reqs[next];
            const int rc = server_submit(srv, q.W, q.L, q.p, q.seed, q.cfg, q.tag, t0 + q.t_arrive_ns);
            if (rc == PERC_EBUSY) {  // shed: the result says so at once
                perc_result r{};
                r.tag = q.tag;
                r.W = q.W;
                r.L = q.L;
                r.p = q.p;
                r.seed = q.seed;
                r.cfg = q.cfg;
                r.status = PERC_EBUSY;
                r.t_arrive_ns = t0 + q.t_arrive_ns;
                r.t_admit_ns = r.t_done_ns = steady_ns();
                out[got++] = r;
            } else if (rc != PERC_OK) {
                return rc;
            }
            ++next;
        }
        if (got >= n) break;
        while (!srv->done.empty() && got < n) {
            out[got++] = srv->done.front();
            srv->done.pop_front();
        }
        const bool idle = srv->queue.empty() && srv->free_slots.size() == srv->slots.size();
        if (idle) {
            if (next >= n) break;  // every request was refused or retired
            if (next < n) {
                std::this_thread::sleep_until(std::chrono::steady_clock::time_point(
                    std::chrono::nanoseconds(t0 + reqs[next].t_arrive_ns)));
            }
            continue;
        }
        const int rc = server_tick(srv);
        if (rc < 0) return rc;
        while (!srv->done.empty() && got < n) {
            out[got++] = srv->done.front();
            srv->done.pop_front();
        }
    }
    return PERC_OK;
}


int perc_stream_copy(const void* src, void* dst, int64_t bytes, int32_t grid, void* stream) {
    if (bytes < 0 || bytes % 16) return fail(PERC_EINVAL, "bytes must be a non-negative multiple of 16");
    if (bytes > 0 && (!src || !dst)) return fail(PERC_EINVAL, "NULL device pointer");
    if ((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) & 15)
        return fail(PERC_EINVAL, "src and dst must be 16-byte aligned");
    if (grid < 0) return fail(PERC_EINVAL, "grid must be >= 0");
    HIP_TRY(launch_stream_copy(src, dst, bytes / 16, grid ? grid : kSpanGrid, reinterpret_cast<hipStream_t>(stream)));
    return PERC_OK;
}

int perc_trim(void) { return cache_trim(); }

int perc_autotune(const perc_job* jobs, int64_t n_jobs, int64_t n_target, perc_options* best, double* best_ms,
                  void* stream) {
    if (n_jobs <= 0 || !jobs) return fail(PERC_EINVAL, "autotuning needs a non-empty job sample");
    std::vector<HostJob> hj;
    PERC_TRY(convert_jobs(jobs, n_jobs, 0, hj));
    return autotune(hj, n_target, best, best_ms, reinterpret_cast<hipStream_t>(stream));
}

}  // extern "C"
