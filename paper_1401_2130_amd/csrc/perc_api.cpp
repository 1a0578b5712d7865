// C ABI (include/perc.h) and the host runtime behind it: lattice handles with
// per-device tables, stream-ordered work memory, the three execution forms and the
// test hook. Every step of the inspection runs in the HIP kernels of kernels.hip.
#include "perc.h"

#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "perc_internal.hpp"

using namespace perc;

struct perc_lattice {
    LatticeDesc d;
    std::mutex mu;
    std::vector<LatticeDevice> dev;
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

#define HIP_TRY(expr)                                         \
    do {                                                      \
        hipError_t e_ = (expr);                               \
        if (e_ != hipSuccess) return hip_fail(e_, #expr);     \
    } while (0)

#define PERC_TRY(expr)                 \
    do {                               \
        int rc_ = (expr);              \
        if (rc_ != PERC_OK) return rc_; \
    } while (0)

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

int tables_for(const perc_lattice* lat_c, int32_t depth, DevTables& t) {
    perc_lattice* lat = const_cast<perc_lattice*>(lat_c);
    const int di = depth_index(depth);
    if (di < 0) return fail(PERC_EINVAL, "unsupported chunk depth");
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    PERC_TRY(prepare(dev));
    const LatticeDesc& d = lat->d;
    std::lock_guard<std::mutex> g(lat->mu);
    LatticeDevice* ld = nullptr;
    for (auto& x : lat->dev)
        if (x.device == dev) ld = &x;
    if (!ld) {
        LatticeDevice n;
        n.device = dev;
        const size_t tb = sizeof(uint32_t) * (size_t)kSide * std::max(d.C, 1);
        for (int i = 0; i < kNumDepths; ++i) {
            const std::vector<uint32_t> tab = contact_table(d, kDepthList[i]);
            HIP_TRY(hipMalloc(&n.nboff[i], tb));
            HIP_TRY(hipMemcpy(n.nboff[i], tab.data(), sizeof(uint32_t) * tab.size(), hipMemcpyHostToDevice));
        }
        HIP_TRY(hipMalloc(&n.top, sizeof(int32_t) * (size_t)std::max(d.C, 1)));
        HIP_TRY(hipMemcpy(n.top, d.top.data(), sizeof(int32_t) * d.top.size(), hipMemcpyHostToDevice));
        lat->dev.push_back(n);
        ld = &lat->dev.back();
    }
    t.nboff = ld->nboff[di];
    t.top = ld->top;
    t.C = d.C; t.CP = d.CP; t.U = d.U; t.L = d.L;
    t.N = d.N; t.words = d.words;
    return PERC_OK;
}

// ---------------------------------------------------------------------------------
// Stream-ordered work memory: one allocation carved into aligned pieces.
// ---------------------------------------------------------------------------------
struct Arena {
    hipStream_t s = nullptr;
    char* base = nullptr;
    size_t size = 0, used = 0;
    ~Arena() {
        if (base) (void)hipFreeAsync(base, s);
    }
    static size_t align(size_t v) { return (v + 255) & ~(size_t)255; }
    int reserve(size_t bytes, hipStream_t stream) {
        s = stream;
        size = std::max<size_t>(bytes, 256);
        hipError_t e = hipMallocAsync(reinterpret_cast<void**>(&base), size, s);
        if (e != hipSuccess) {
            base = nullptr;
            return fail(PERC_ENOMEM, std::string("work memory of ") + std::to_string(size) +
                                         " bytes: " + hipGetErrorString(e));
        }
        return PERC_OK;
    }
    template <typename T>
    T* take(size_t count) {
        T* p = reinterpret_cast<T*>(base + used);
        used += align(sizeof(T) * std::max<size_t>(count, 1));
        return p;
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
// stream around every step launch (graphs are not used while it is on) and the tube
// slots the steps processed (cells scheduled by the planner times the columns).
// ---------------------------------------------------------------------------------
struct Profiler {
    std::mutex mu;
    bool on = false;
    int64_t launches = 0;
    double ms = 0.0;
    int64_t tube_steps = 0;
};
Profiler g_prof;

bool profiling() {
    std::lock_guard<std::mutex> g(g_prof.mu);
    return g_prof.on;
}

class StepTimer {
  public:
    explicit StepTimer(bool on) : on_(on) {}
    ~StepTimer() {
        for (auto& p : pending_) { free_.push_back(p.first); free_.push_back(p.second); }
        for (hipEvent_t e : free_) (void)hipEventDestroy(e);
    }
    hipError_t step(const SpanArgs& a, hipStream_t s) {
        if (!on_) return launch_span_step(a, s);
        std::pair<hipEvent_t, hipEvent_t> ev;
        hipError_t e = take(&ev.first);
        if (e == hipSuccess) e = take(&ev.second);
        if (e != hipSuccess) return e;
        pending_.push_back(ev);
        e = hipEventRecord(ev.first, s);
        if (e == hipSuccess) e = launch_span_step(a, s);
        if (e == hipSuccess) e = hipEventRecord(ev.second, s);
        return e;
    }
    // After the stream has been synchronised: add the durations of the launches since
    // the last call.
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
        g_prof.launches += (int64_t)pending_.size();
        g_prof.ms += ms;
        pending_.clear();
        return hipSuccess;
    }
    bool on() const { return on_; }

  private:
    hipError_t take(hipEvent_t* e) {
        if (!free_.empty()) { *e = free_.back(); free_.pop_back(); return hipSuccess; }
        return hipEventCreate(e);
    }
    bool on_;
    std::vector<hipEvent_t> free_;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pending_;
};

// ---------------------------------------------------------------------------------
// Tuning: explicit options, else cached autotune results, else shape rules.
// ---------------------------------------------------------------------------------
bool valid_depth(int32_t d) { return depth_index(d) >= 0; }

int32_t depth_within(int32_t C, size_t lds_budget, int32_t cap) {
    int32_t best = 0;
    for (int32_t d : kDepthList)
        if (d <= cap && lds_bytes_for(C, d) <= lds_budget) best = d;
    return best;
}

int64_t state_bytes(const LatticeDesc& d) { return (int64_t)d.U * d.CP * 9; }

int resolve(const LatticeDesc& d, int64_t n_cfg, const perc_options* opt, Tuning& tu) {
    tu = Tuning{};
    if (opt) {
        tu.form = opt->form;
        tu.depth = opt->depth;
        tu.block = opt->block;
        tu.grid = opt->grid;
        tu.graph_steps = opt->graph_steps;
    }
    if (tu.form < FORM_AUTO || tu.form > FORM_PERSIST) return fail(PERC_EINVAL, "unknown execution form");
    if (tu.form == FORM_AUTO) {
        // many configurations of modest size: one workgroup each; otherwise spread
        tu.form = (n_cfg >= 1024 && state_bytes(d) <= (64ll << 20)) ? FORM_PERSIST : FORM_SPAN;
    }
    const size_t kMaxLds = 160 * 1024;
    if (tu.depth == 0) {
        // plain: one configuration, as many workgroups per step as possible; span: the
        // deepest chunk that fits (measured best on W=32); persistent: two per CU
        if (tu.form == FORM_PLAIN) tu.depth = depth_within(d.C, kMaxLds, 1);
        else if (tu.form == FORM_SPAN) tu.depth = depth_within(d.C, kMaxLds, 15);
        else tu.depth = depth_within(d.C, 80 * 1024, 15);
        if (tu.depth == 0) tu.depth = depth_within(d.C, kMaxLds, 15);
    }
    if (!valid_depth(tu.depth)) return fail(PERC_EINVAL, "depth must be one of 1, 3, 5, 7, 9, 15");
    if (lds_bytes_for(d.C, tu.depth) > kMaxLds)
        return fail(PERC_EINVAL, "chunk of " + std::to_string(tu.depth) + " cells of " + std::to_string(d.C) +
                                     " columns exceeds the LDS of one workgroup");
    if (tu.block == 0) {
        const int32_t want = tu.form == FORM_PLAIN ? 512 : 1024;
        tu.block = std::max<int32_t>(64, std::min<int32_t>(want, ((d.C + 63) / 64) * 64));
    }
    if (tu.block < 64 || tu.block > 1024 || tu.block % 64) return fail(PERC_EINVAL, "block must be 64..1024, multiple of 64");
    if (tu.graph_steps == 0) tu.graph_steps = 8;
    if (tu.graph_steps < 1 || tu.graph_steps > 256) return fail(PERC_EINVAL, "graph_steps must be 1..256");
    if (tu.grid < 0) return fail(PERC_EINVAL, "grid must be >= 0");
    return PERC_OK;
}

// ---------------------------------------------------------------------------------
// Span and plain forms.
// ---------------------------------------------------------------------------------
bool stream_capturing(hipStream_t s) {
    if (!s) return false;
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &st) != hipSuccess) return false;
    return st != hipStreamCaptureStatusNone;
}

int run_span(const LatticeDesc& d, const DevTables& t, const uint32_t* bits, int64_t n_cfg, BatchOut out,
             const Tuning& tu, hipStream_t s) {
    if (n_cfg == 0) return PERC_OK;
    if (stream_capturing(s)) return fail(PERC_EINVAL, "the span and plain forms synchronise; not capturable");
    const bool plain = tu.form == FORM_PLAIN;
    const int64_t cell_words = (int64_t)t.U * t.CP;
    const int64_t per_cfg = cell_words * 9 + 64;
    size_t free_b = 0, total_b = 0;
    HIP_TRY(hipMemGetInfo(&free_b, &total_b));
    const int64_t budget = std::max<int64_t>(per_cfg, std::min<int64_t>((int64_t)(free_b / 2), 48ll << 30));
    int64_t n_slot = plain ? 1 : std::min<int64_t>(n_cfg, std::max<int64_t>(1, budget / per_cfg));
    n_slot = std::min<int64_t>(n_slot, 1 << 20);
    Arena ar;
    const size_t bytes = Arena::align(sizeof(float) * n_slot * cell_words) * 2 +
                         Arena::align((size_t)n_slot * cell_words) + Arena::align(sizeof(CfgState) * n_slot) +
                         Arena::align(sizeof(int32_t) * n_slot) * 2 + Arena::align(sizeof(int64_t) * (n_slot + 1)) +
                         Arena::align(64);
    PERC_TRY(ar.reserve(bytes, s));
    SpanArgs a{};
    a.t = t;
    a.ya = ar.take<float>(n_slot * cell_words);
    a.yb = ar.take<float>(n_slot * cell_words);
    a.code = ar.take<uint8_t>(n_slot * cell_words);
    a.st = ar.take<CfgState>(n_slot);
    a.active = ar.take<int32_t>(n_slot);
    a.active2 = ar.take<int32_t>(n_slot);
    a.chunk_off = ar.take<int64_t>(n_slot + 1);
    a.hdr = ar.take<int32_t>(16);
    a.depth = tu.depth;
    a.block = tu.block;
    a.grid = tu.grid ? tu.grid : 2048;
    a.cap = d.N + 1;
    if (!g_pinned.h) return fail(PERC_ENOMEM, "pinned host buffer");
    int32_t* h = g_pinned.h;
    a.work = reinterpret_cast<unsigned long long*>(a.hdr + 8);
    StepTimer timer(profiling());
    // HIP gives no elapsed time for events recorded as graph nodes: while profiling,
    // steps are launched directly with an event pair around each
    const bool use_graph = !plain && s != nullptr && !timer.on();
    for (int64_t w = 0; w < n_cfg; w += n_slot) {
        const int64_t nb = std::min<int64_t>(n_slot, n_cfg - w);
        a.n_slot = (int32_t)nb;
        a.bits = bits + w * t.words;
        a.out.perc = out.perc + w;
        a.out.steps = out.steps + w;
        a.out.hit = out.hit ? out.hit + w : nullptr;
        HIP_TRY(launch_fill_u32(reinterpret_cast<uint32_t*>(a.hdr), 16, 0u, s));
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
                hipError_t ce = hipSuccess;
                for (int i = 0; i < tu.graph_steps && ce == hipSuccess; ++i) {
                    ce = launch_span_step(a, s);
                    if (ce == hipSuccess) ce = launch_span_plan(a, s);
                }
                hipError_t ee = hipStreamEndCapture(s, &graph);
                if (ce != hipSuccess) { if (graph) (void)hipGraphDestroy(graph); return hip_fail(ce, "capture"); }
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
                        for (int i = 0; i < tu.graph_steps && rc == PERC_OK; ++i) {
                            hipError_t e = timer.step(a, s);
                            if (e == hipSuccess) e = launch_span_plan(a, s);
                            if (e != hipSuccess) rc = hip_fail(e, "span step");
                        }
                    }
                }
                if (rc != PERC_OK) break;
                hipError_t e = hipMemcpyAsync(h, a.hdr, 64, hipMemcpyDeviceToHost, s);
                if (e == hipSuccess) e = hipStreamSynchronize(s);
                if (e == hipSuccess) e = timer.collect();
                if (e != hipSuccess) { rc = hip_fail(e, "span poll"); break; }
                if (h[0] == 0) break;
                reps = std::min(reps * 2, 8);
            }
            if (exec) (void)hipGraphExecDestroy(exec);
            if (rc != PERC_OK) return rc;
        }
        if (h[2]) return fail(PERC_ECAP, "a configuration reached the step cap");
        if (timer.on()) {
            unsigned long long cells = 0;
            std::memcpy(&cells, h + 8, sizeof(cells));
            std::lock_guard<std::mutex> g(g_prof.mu);
            g_prof.tube_steps += (int64_t)cells * t.C;
        }
        HIP_TRY(launch_span_finish(a, s));
    }
    return PERC_OK;
}

// ---------------------------------------------------------------------------------
// Persistent form.
// ---------------------------------------------------------------------------------
int run_persist(const LatticeDesc& d, const DevTables& t, const uint32_t* bits, int64_t n_cfg, uint64_t cfg0,
                uint64_t thr, uint64_t seed, BatchOut out, const Tuning& tu, hipStream_t s) {
    if (n_cfg == 0) return PERC_OK;
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    int cus = 0;
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    int grid = tu.grid;
    if (grid == 0) {
        const int per_cu = std::max(1, persist_resident_per_cu(tu.depth, tu.block, t.C));
        grid = cus * per_cu;
    }
    grid = (int)std::min<int64_t>(grid, n_cfg);
    const int64_t cell_words = (int64_t)t.U * t.CP;
    Arena ar;
    const size_t bytes = Arena::align(sizeof(float) * grid * cell_words) * 2 + Arena::align((size_t)grid * cell_words) +
                         (bits ? 0 : Arena::align(sizeof(uint32_t) * grid * t.words)) + Arena::align(64);
    PERC_TRY(ar.reserve(bytes, s));
    PersistArgs a{};
    a.t = t;
    a.bits = bits;
    a.ya = ar.take<float>(grid * cell_words);
    a.yb = ar.take<float>(grid * cell_words);
    a.code = ar.take<uint8_t>(grid * cell_words);
    a.bits_scratch = bits ? nullptr : ar.take<uint32_t>(grid * t.words);
    a.queue = ar.take<unsigned long long>(2);
    a.err = reinterpret_cast<uint32_t*>(a.queue + 1);
    a.n_cfg = n_cfg;
    a.cfg0 = cfg0;
    a.threshold = thr;
    a.seed = seed;
    a.tag = ((uint32_t)d.W << 16) | (uint32_t)d.L;
    a.out = out;
    a.depth = tu.depth;
    a.block = tu.block;
    a.grid = grid;
    a.cap = d.N + 1;
    HIP_TRY(launch_fill_u32(reinterpret_cast<uint32_t*>(a.queue), 4, 0u, s));
    HIP_TRY(launch_persist(a, s));
    return PERC_OK;
}

int validate_lat(const perc_lattice* lat) {
    if (!lat) return fail(PERC_EINVAL, "lattice is NULL");
    return PERC_OK;
}

uint64_t threshold_of(double p) {
    if (p >= 1.0) return (uint64_t)1 << 32;
    return (uint64_t)std::floor(p * 4294967296.0);
}

int inspect_impl(const perc_lattice* lat, const uint32_t* occ_bits, int64_t n_cfg, uint8_t* perc, int32_t* steps,
                 float* hit, const perc_options* opt, void* stream) {
    PERC_TRY(validate_lat(lat));
    if (n_cfg < 0) return fail(PERC_EINVAL, "n_cfg < 0");
    if (n_cfg == 0) return PERC_OK;
    if (!occ_bits || !perc) return fail(PERC_EINVAL, "occ_bits and perc must be device pointers");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    Tuning tu;
    PERC_TRY(resolve(lat->d, n_cfg, opt, tu));
    DevTables t;
    PERC_TRY(tables_for(lat, tu.depth, t));
    Arena ar;
    if (!steps) {
        PERC_TRY(ar.reserve(sizeof(int32_t) * n_cfg, s));
        steps = ar.take<int32_t>(n_cfg);
    }
    BatchOut out{perc, steps, hit};
    if (tu.form == FORM_PERSIST) return run_persist(lat->d, t, occ_bits, n_cfg, 0, 0, 0, out, tu, s);
    return run_span(lat->d, t, occ_bits, n_cfg, out, tu, s);
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
    Tuning tu;
    PERC_TRY(resolve(lat->d, n_cfg, opt, tu));
    DevTables t;
    PERC_TRY(tables_for(lat, tu.depth, t));
    const uint64_t thr = threshold_of(p);
    Arena ar;
    const size_t bytes = (out->bits ? 0 : Arena::align((size_t)n_cfg)) +
                         (out->steps ? 0 : Arena::align(sizeof(int32_t) * n_cfg)) +
                         (tu.form == FORM_PERSIST ? 0 : Arena::align(sizeof(uint32_t) * n_cfg * t.words)) +
                         Arena::align(64);
    PERC_TRY(ar.reserve(bytes, s));
    BatchOut bo;
    bo.perc = out->bits ? out->bits : ar.take<uint8_t>(n_cfg);
    bo.steps = out->steps ? out->steps : ar.take<int32_t>(n_cfg);
    bo.hit = out->hit;
    unsigned long long* count = ar.take<unsigned long long>(1);
    if (tu.form == FORM_PERSIST) {
        PERC_TRY(run_persist(lat->d, t, nullptr, n_cfg, 0, thr, seed, bo, tu, s));
    } else {
        uint32_t* bits = ar.take<uint32_t>(n_cfg * t.words);
        const uint32_t tag = ((uint32_t)lat->d.W << 16) | (uint32_t)lat->d.L;
        HIP_TRY(launch_sample(t, bits, n_cfg, 0, thr, seed, tag, s));
        PERC_TRY(run_span(lat->d, t, bits, n_cfg, bo, tu, s));
    }
    HIP_TRY(launch_fill_u32(reinterpret_cast<uint32_t*>(count), 2, 0u, s));
    HIP_TRY(launch_count(bo.perc, n_cfg, count, s));
    unsigned long long host_count = 0;
    HIP_TRY(hipMemcpyAsync(&host_count, count, sizeof(host_count), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    out->n_perc = (int64_t)host_count;
    out->pi = (double)host_count / (double)n_cfg;
    return PERC_OK;
}

}  // namespace

// =================================================================================
// extern "C" entry points
// =================================================================================
extern "C" {

perc_lattice* perc_lattice_create(int32_t W, int32_t L) {
    perc_lattice* lat = new (std::nothrow) perc_lattice();
    if (!lat) { g_err = "out of host memory"; return nullptr; }
    std::string err;
    if (!build_lattice(W, L, lat->d, err)) {
        g_err = err;
        delete lat;
        return nullptr;
    }
    return lat;
}

void perc_lattice_destroy(perc_lattice* lat) {
    if (!lat) return;
    int cur = 0;
    const bool have = hipGetDevice(&cur) == hipSuccess;
    for (auto& x : lat->dev) {
        if (hipSetDevice(x.device) == hipSuccess) {
            for (uint32_t* p : x.nboff) (void)hipFree(p);
            (void)hipFree(x.top);
        }
    }
    if (have) (void)hipSetDevice(cur);
    delete lat;
}

int64_t perc_lattice_sites(const perc_lattice* lat) { return lat ? lat->d.N : -1; }
int64_t perc_lattice_words(const perc_lattice* lat) { return lat ? lat->d.words : -1; }
int32_t perc_lattice_columns(const perc_lattice* lat) { return lat ? lat->d.C : -1; }
int64_t perc_lattice_state_bytes(const perc_lattice* lat) { return lat ? state_bytes(lat->d) : -1; }

int perc_site_coord(const perc_lattice* lat, int64_t s, int32_t* q, int32_t* r, int32_t* k) {
    PERC_TRY(validate_lat(lat));
    const LatticeDesc& d = lat->d;
    if (s < 0 || s >= d.N) return fail(PERC_EINVAL, "site index out of range");
    const int64_t u = s / d.C, c = s - u * d.C;
    if (q) *q = d.q[c];
    if (r) *r = d.r[c];
    if (k) *k = (int32_t)(3 * u + d.sig[c]);
    return PERC_OK;
}

int perc_site_neighbors(const perc_lattice* lat, int64_t s, int64_t* nbr, int32_t* count) {
    PERC_TRY(validate_lat(lat));
    const LatticeDesc& d = lat->d;
    if (s < 0 || s >= d.N || !nbr || !count) return fail(PERC_EINVAL, "bad site or NULL output");
    const int64_t u = s / d.C, c = s - u * d.C;
    std::vector<int64_t> out;
    auto add = [&](int64_t uu, int64_t cc) {
        if (uu < 0 || uu >= d.U || cc >= d.C) return;
        const int64_t t = uu * d.C + cc;
        if (t < d.N) out.push_back(t);
    };
    for (int i = 0; i < kSide; ++i) {
        const int32_t v = d.nb[(size_t)i * d.C + c];
        add(u + ((v & 3) - 1), v >> 2);
    }
    add(u - 1, c);
    add(u + 1, c);
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
    return PERC_OK;
}

int perc_profile_read(perc_profile* out) {
    if (!out) return fail(PERC_EINVAL, "out is NULL");
    std::lock_guard<std::mutex> g(g_prof.mu);
    out->step_launches = g_prof.launches;
    out->step_ms = g_prof.ms;
    out->tube_steps = g_prof.tube_steps;
    return PERC_OK;
}

int perc_sample(const perc_lattice* lat, double p, uint64_t seed, int64_t cfg0, int64_t n_cfg, uint32_t* occ_bits,
                void* stream) {
    PERC_TRY(validate_lat(lat));
    if (!(p >= 0.0 && p <= 1.0)) return fail(PERC_EINVAL, "p must be in [0, 1]");
    if (n_cfg < 0 || cfg0 < 0) return fail(PERC_EINVAL, "n_cfg and cfg0 must be >= 0");
    if (n_cfg == 0) return PERC_OK;
    if (!occ_bits) return fail(PERC_EINVAL, "occ_bits is NULL");
    DevTables t;
    PERC_TRY(tables_for(lat, 1, t));
    const uint32_t tag = ((uint32_t)lat->d.W << 16) | (uint32_t)lat->d.L;
    HIP_TRY(launch_sample(t, occ_bits, n_cfg, (uint64_t)cfg0, threshold_of(p), seed, tag,
                          reinterpret_cast<hipStream_t>(stream)));
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

int perc_pi(const perc_lattice* lat, double p, int64_t n_cfg, uint64_t seed, perc_pi_out* out, void* stream) {
    return pi_impl(lat, p, n_cfg, seed, out, nullptr, stream);
}

int perc_pi_ex(const perc_lattice* lat, double p, int64_t n_cfg, uint64_t seed, perc_pi_out* out,
               const perc_options* opt, void* stream) {
    return pi_impl(lat, p, n_cfg, seed, out, opt, stream);
}

int perc_state_after(const perc_lattice* lat, const uint32_t* occ_bits, int32_t K, float* x_out, uint8_t* reach_out,
                     void* stream) {
    PERC_TRY(validate_lat(lat));
    if (K < 0) return fail(PERC_EINVAL, "K < 0");
    if (!occ_bits || !x_out || !reach_out) return fail(PERC_EINVAL, "NULL device pointer");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const LatticeDesc& d = lat->d;
    const int32_t depth = depth_within(d.C, 80 * 1024, 3) ? depth_within(d.C, 80 * 1024, 3) : 1;
    DevTables t;
    PERC_TRY(tables_for(lat, depth, t));
    const int64_t cell_words = (int64_t)t.U * t.CP;
    Arena ar;
    PERC_TRY(ar.reserve(Arena::align(sizeof(float) * cell_words) * 2 + Arena::align((size_t)cell_words) +
                            Arena::align(sizeof(CfgState)) + Arena::align(64) * 4, s));
    float* ya = ar.take<float>(cell_words);
    float* yb = ar.take<float>(cell_words);
    uint8_t* code = ar.take<uint8_t>(cell_words);
    CfgState* st = ar.take<CfgState>(1);
    float* det = ar.take<float>(2);
    uint32_t* det_r = reinterpret_cast<uint32_t*>(det + 1);
    int32_t* hdr = ar.take<int32_t>(16);
    HIP_TRY(launch_fill_u32(reinterpret_cast<uint32_t*>(ya), cell_words, 0u, s));
    HIP_TRY(launch_fill_u32(reinterpret_cast<uint32_t*>(yb), cell_words, 0u, s));
    HIP_TRY(launch_fill_u32(reinterpret_cast<uint32_t*>(det), 2, 0u, s));
    HIP_TRY(launch_fill_u32(reinterpret_cast<uint32_t*>(hdr), 16, 0u, s));
    SpanArgs a{};
    a.t = t;
    a.bits = occ_bits;
    a.ya = ya; a.yb = yb; a.code = code; a.st = st;
    a.hdr = hdr;
    a.n_slot = 1;
    a.depth = depth;
    a.block = 256;
    HIP_TRY(launch_span_init_only(a, s));
    float* cur = ya;
    float* nxt = yb;
    for (int32_t m = 0; m < K; ++m) {
        HIP_TRY(launch_far_sum(t, cur, det, det_r, s));
        HIP_TRY(launch_chunk_step(t, cur, nxt, code, t.U, depth, 256, s));
        std::swap(cur, nxt);
    }
    HIP_TRY(launch_export(t, cur, code, det, det_r, x_out, reach_out, s));
    return PERC_OK;
}

}  // extern "C"
