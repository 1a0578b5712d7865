// Internal declarations shared by the host runtime (lattice.cpp, engine.cpp, api.cpp)
// and the device code (kernels.hip). Not part of the public C ABI (include/perc.h).
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

namespace perc {

// ---------------------------------------------------------------------------------
// Lattice descriptor (Sec. II.A, Fig. 1).
//
// Columns (q, r) are the points of the projected triangular net (axial coordinates,
// spacing = one tube spacing) inside the hexagon of hex radius W. Column (q, r) holds
// the tubes of the (111) layers k with k = sigma (mod 3), sigma = (q - r) mod 3 (ABC
// stacking). Columns are numbered c = 0..C-1 in (sigma, q, r) order, so that the
// "unit cell" u (layers 3u, 3u+1, 3u+2) holds every column exactly once, tube (u, c)
// sits on layer k = 3u + sigma(c), and the canonical site index is s = u*C + c. This
// equals lexicographic (k, q, r) order; the last cell holds only the columns with
// 3u + sigma < L, which are a prefix of the column order, so N = sites with s < N.
//
// The 12 side contacts of a tube are the FCC nearest neighbours: 6 in its layer,
// 3 in the layer above and 3 below; the 2 end contacts are the tubes of the same
// column in cells u-1 and u+1. A side contact of column c lies in column nb_col and
// cell u + nb_dcell (dcell in {-1, 0, +1}).
// ---------------------------------------------------------------------------------
constexpr int kSide = 12;

struct LatticeDesc {
    int32_t W = 0, L = 0;
    int32_t C = 0;       // columns
    int32_t U = 0;       // unit cells, ceil(L / 3)
    int32_t CP = 0;      // padded row length of the state arrays: multiple of 32, >= C + 1
    int64_t N = 0;       // sites
    int64_t words = 0;   // ceil(N / 32)
    int32_t nsig[3] = {0, 0, 0};
    std::vector<int32_t> q, r, sig;  // per column
    std::vector<int32_t> top;        // per column: cell of its far-end tube, -1 if empty
    // per side contact i (0..11) and column c: packed (nb_col << 2) | (dcell + 1);
    // a contact outside the hexagon points at column C (a zero pad).
    std::vector<int32_t> nb;         // [kSide][C]
};

bool build_lattice(int32_t W, int32_t L, LatticeDesc& out, std::string& err);

// Chunk depths (unit cells per workgroup chunk) the kernels are built for.
constexpr int kNumDepths = 6;
constexpr int32_t kDepthList[kNumDepths] = {1, 3, 5, 7, 9, 15};
inline int depth_index(int32_t d) {
    for (int i = 0; i < kNumDepths; ++i)
        if (kDepthList[i] == d) return i;
    return -1;
}

// Contact table of one chunk depth D: for side contact i of column c, the LDS byte
// offset ((nb_col * (D + 2) + dcell + 1) * 4) of that contact in a chunk staged
// column-major with D + 2 slots per column; the tube in slot j reads it at that offset
// plus (j - 1) * 4.
std::vector<uint32_t> contact_table(const LatticeDesc& d, int32_t depth);

// Device copies of the per-column tables, one per HIP device that used the lattice.
struct LatticeDevice {
    int device = -1;
    uint32_t* nboff[kNumDepths] = {};  // [kSide][C] per depth
    int32_t* top = nullptr;             // [C]
};

#if defined(__HIPCC__)
#define PERC_HD __host__ __device__
#else
#define PERC_HD
#endif

// Dynamic LDS of a chunk kernel (byte offsets; every kernel of the inspection keeps
// all its LDS here, so the state chunk starts at address 0):
//   [0, state)   state words, column-major, (C + 1) columns x (D + 2) slots
//   code         degree codes of the D computed cells, [c][D] bytes
//   rcp          16 floats, 1/deg per code
//   misc         16 words of flags and counters
//   part         256 floats of partial sums
struct LdsMap {
    uint32_t code, rcp, misc, part, total;
};
PERC_HD inline LdsMap lds_map(int32_t C, int32_t D) {
    LdsMap m;
    const uint32_t state = (uint32_t)(C + 1) * (uint32_t)(D + 2) * 4u;
    m.code = (state + 15u) & ~15u;
    m.rcp = (m.code + (uint32_t)C * (uint32_t)D + 15u) & ~15u;
    m.misc = m.rcp + 64u;
    m.part = m.misc + 64u;
    m.total = m.part + 1024u;
    return m;
}

// ---------------------------------------------------------------------------------
// Execution forms and tuning knobs.
// ---------------------------------------------------------------------------------
enum Form : int32_t {
    FORM_AUTO = 0,
    FORM_PLAIN = 1,    // one configuration at a time, host checks flags every step
    FORM_SPAN = 2,     // many configurations, each spread over many workgroups, one
                       // launch per step over a device-built work list, graph-replayed
    FORM_PERSIST = 3,  // one workgroup per configuration, whole inspection in one launch
};

struct Tuning {
    int32_t form = FORM_AUTO;
    int32_t depth = 0;      // cells per chunk (odd: 1, 3, 5, 7, 9, ...); 0 = choose
    int32_t block = 0;      // threads per workgroup (64..1024); 0 = choose
    int32_t graph_steps = 0;  // steps per graph replay (span form); 0 = choose
    int32_t grid = 0;       // workgroups per launch (span step / persistent); 0 = choose
};

// Per-configuration device state of the span and plain forms.
struct CfgState {
    int32_t front;   // largest cell holding a reached tube
    int32_t m;       // steps done
    int32_t done;    // 0 = active, 1 = decided, 2 = cap reached (error)
    uint32_t flags;  // OR of the flags of the last launch; cleared by the planner
};

constexpr uint32_t F_GREW = 1u;      // some tube joined the reached set
constexpr uint32_t F_FRONT = 2u;     // the reached set entered cell front+1
constexpr uint32_t F_FAR = 4u;       // a far-end tube is reached: detector next step
constexpr uint32_t F_NONEMPTY = 8u;  // (initialisation) some start tube is metallic

// Outputs of a batch, device pointers (any may be null except perc/steps).
struct BatchOut {
    uint8_t* perc = nullptr;
    int32_t* steps = nullptr;
    float* hit = nullptr;  // first-passage probability of the detector at the stop
};

// ---------------------------------------------------------------------------------
// Kernel launchers (kernels.hip).
// ---------------------------------------------------------------------------------
struct DevTables {
    const uint32_t* nboff;  // contact table of the chunk depth in use
    const int32_t* top;
    int32_t C, CP, U, L;
    int64_t N, words;
};

// Philox4x32-10 occupancy for configurations cfg0..cfg0+n_cfg-1 (canonical bits).
hipError_t launch_sample(const DevTables& t, uint32_t* bits, int64_t n_cfg, uint64_t cfg0,
                         uint64_t threshold, uint64_t seed, uint32_t tag, hipStream_t s);

// Span/plain forms: state arrays are [n_slot][U][CP]; slot b inspects bits + b*words.
struct SpanArgs {
    DevTables t;
    const uint32_t* bits;      // [n_slot][words]
    float* ya;                 // [n_slot][U][CP]
    float* yb;
    uint8_t* code;             // [n_slot][U][CP]
    CfgState* st;              // [n_slot]
    int32_t* active;           // [n_slot] active slot list (first entry count in hdr)
    int32_t* active2;          // scratch for compaction
    int64_t* chunk_off;        // [n_slot + 1] prefix sums of chunks per active slot
    int32_t* hdr;              // [4]: n_active, total chunks, error flag, spare
    unsigned long long* work;  // cells scheduled over all steps (planner adds), or null
    BatchOut out;
    int32_t n_slot;
    int32_t depth;             // cells per chunk
    int32_t block;
    int32_t grid;
    int64_t cap;               // step cap (never reached for a correct lattice)
};

hipError_t launch_span_init(const SpanArgs& a, hipStream_t s);     // codes, y0, first plan
hipError_t launch_span_init_only(const SpanArgs& a, hipStream_t s);  // codes and y0 only
hipError_t launch_span_step(const SpanArgs& a, hipStream_t s);     // one step over work list
hipError_t launch_span_plan(const SpanArgs& a, hipStream_t s);     // decide, compact, plan
hipError_t launch_span_finish(const SpanArgs& a, hipStream_t s);   // first-hit probabilities

// Persistent form: one workgroup per configuration, scratch per resident workgroup.
struct PersistArgs {
    DevTables t;
    const uint32_t* bits;      // caller's bits [n_cfg][words], or null to sample
    uint32_t* bits_scratch;    // [grid][words] when sampling
    float* ya;                 // [grid][U][CP]
    float* yb;
    uint8_t* code;             // [grid][U][CP]
    unsigned long long* queue; // next configuration to take
    uint32_t* err;             // set when a configuration reached the step cap
    int64_t n_cfg;
    uint64_t cfg0;
    uint64_t threshold;
    uint64_t seed;
    uint32_t tag;
    BatchOut out;
    int32_t depth;
    int32_t block;
    int32_t grid;
    int64_t cap;
};
hipError_t launch_persist(const PersistArgs& a, hipStream_t s);

// Test hook: export x = |y| deg (canonical order) and the reach bits, detector last.
hipError_t launch_export(const DevTables& t, const float* y, const uint8_t* code, const float* det_mass,
                         const uint32_t* det_reached, float* x_out, uint8_t* reach_out, hipStream_t s);
hipError_t launch_chunk_step(const DevTables& t, const float* yin, float* yout, const uint8_t* code, int front,
                             int depth, int block, hipStream_t s);
hipError_t launch_far_sum(const DevTables& t, const float* y, float* det_mass, uint32_t* det_reached,
                          hipStream_t s);

// Count of percolating configurations (integer, deterministic).
hipError_t launch_count(const uint8_t* perc, int64_t n, unsigned long long* count, hipStream_t s);

size_t lds_bytes_for(int32_t C, int32_t depth);
hipError_t launch_fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t s);
int persist_resident_per_cu(int depth, int block, int C);
hipError_t prepare_kernels(int device);
int32_t max_depth_for(int32_t C);

}  // namespace perc
