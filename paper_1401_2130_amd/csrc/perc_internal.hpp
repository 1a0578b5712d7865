// Internal declarations shared by the host runtime (lattice.cpp, perc_api.cpp) and
// the device code (kernels.hip). Not part of the public C ABI (include/perc.h).
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstdint>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#if defined(__HIPCC__)
#define PERC_HD __host__ __device__
#define PERC_HD_INLINE __host__ __device__ __forceinline__
#else
#define PERC_HD
#define PERC_HD_INLINE inline
#endif

namespace perc {

// ---------------------------------------------------------------------------------
// Lattice descriptor (Sec. II.A, Fig. 1).
//
// Columns (q, r) are the points of the projected triangular net (axial coordinates,
// spacing = one tube spacing) inside the hexagon of hex radius W. Column (q, r) holds
// the tubes of the (111) layers k with k = sigma (mod 3), sigma = (q - r) mod 3 (ABC
// stacking). The "unit cell" u (layers 3u, 3u+1, 3u+2) holds every column exactly once:
// tube (u, c) sits on layer k = 3u + sigma(c), and all 14 contacts of a tube lie in
// cells u-1, u, u+1.
//
// Internally columns are numbered c = 0..C-1 in (q, r) order, so that the contacts of
// a column lie within two q-rows of it and a tile of consecutive columns needs only a
// narrow halo. The canonical site order of the ABI is lexicographic (k, q, r): tube
// (u, c) has canonical index u*C + rank[c], with rank the (sigma, q, r) order; the tubes
// of the last, partial cell are a prefix of that order, so a tube exists iff its
// canonical index is below N.
//
// The 12 side contacts of a tube are the FCC nearest neighbours: 6 in its layer,
// 3 in the layer above and 3 below; the 2 end contacts are the tubes of the same
// column in cells u-1 and u+1.
// ---------------------------------------------------------------------------------
constexpr int kSide = 12;
constexpr int kTileCols = 512;  // target columns per tile

// Everything that depends on the cross-section only (hex radius W): built once per W
// and shared by every fiber length (see column_set).
struct ColumnSet {
    int32_t W = 0;
    int32_t C = 0;       // columns
    int32_t CP = 0;      // row length of the state arrays: multiple of 32, >= C
    int32_t nsig[3] = {0, 0, 0};
    std::vector<int32_t> q, r, sig;  // per internal column
    std::vector<int32_t> rank;       // canonical rank of internal column c
    std::vector<int32_t> by_rank;    // internal column of canonical rank k
    // per side contact i (0..11) and column c: packed (nb_col << 2) | (dcell + 1);
    // a contact outside the hexagon has nb_col = C
    std::vector<int32_t> nb;         // [kSide][C]
    int32_t ntile = 1;
    std::vector<int32_t> tile;       // [ntile][4]: first col, end col, halo first, halo end
    int32_t span_max = 0;            // widest halo range
    int32_t tile_max = 0;            // widest tile
    // Lanes of the tile walks (layout below): lane l of the walk of tile k computes column
    // tile[4k] + lanes[k * lane_stride + l]; lane_stride = the tile width rounded up to 64.
    int32_t lane_stride = 64;
    std::vector<uint16_t> lanes;     // [ntile][lane_stride]
    std::vector<uint32_t> contact;   // contact table (layout below), two contacts per word, by lane
    // Two steps per pass: the first step is computed on the whole halo range [hs, he) of
    // a tile, which reads the outer range [hs2, he2) (the halo of the halo range).
    std::vector<int32_t> tile2;      // [ntile][2]: outer first, outer end
    int32_t span2_max = 0;           // widest outer range
    // [ntile][kSide][span_max]: LDS word (ring of the outer range) of side contact i of
    // halo-range column lc of tile k, as in `contact`; empty when span_max or span2_max
    // exceeds kMaxSpan2 (the two-step form is not offered for such widths)
    std::vector<uint32_t> contact2;
    // One tile holding the whole cross-section (no halo), for fibers of at most
    // kWholeCols columns (one thread per column): the contact table of that tile,
    // [kSide][C], LDS words relative to column 0. It also serves as the two-step table
    // (outer range = halo range = all columns). Empty for wider fibers.
    std::vector<uint32_t> contact_whole;
    // the one-step walks' view of that tile: its lanes and, by lane, two contacts per word
    int32_t lane_stride_whole = 64;
    std::vector<uint16_t> lanes_whole;      // [lane_stride_whole]
    std::vector<uint32_t> contact_whole16;  // [kSide / 2][lane_stride_whole]
};
constexpr int32_t kMaxSpan2 = 2048;
constexpr int32_t kWholeCols = 1024;

// The column set of hex radius W, built on first use and kept for the process (one per
// distinct W; thread safe). Null with a message for a bad W.
std::shared_ptr<const ColumnSet> column_set(int32_t W, std::string& err);

// A fiber: the column set of its W and the quantities that depend on L.
struct LatticeDesc {
    std::shared_ptr<const ColumnSet> cs;
    int32_t W = 0, L = 0;
    int32_t C = 0, CP = 0;
    int32_t U = 0;       // unit cells, ceil(L / 3)
    int64_t N = 0;       // sites
    int64_t words = 0;   // ceil(N / 32)
    int32_t ntile = 1, span_max = 0, tile_max = 0;
    int32_t ends = 1;    // 1: the two end contacts per tube; 0: regular FCC
    // cell of the far-end tube of column c (the highest layer k < L with k = sigma), or
    // -1 if the column holds no tube
    int32_t top(int32_t c) const {
        const int32_t sg = cs->sig[c];
        return sg < L ? (L - 1 - sg) / 3 : -1;
    }
};

bool build_lattice(int32_t W, int32_t L, LatticeDesc& out, std::string& err);

// Words of one configuration's state (and bytes of its degree codes): the cells in
// groups of four, each group a [CP] row of 4-word quads (word k of quad (g, c) is cell
// 4g+k of column c).
inline int64_t state_words(const LatticeDesc& d) { return (int64_t)((d.U + 3) / 4) * 4 * d.CP; }

// The LDS ring of the walking kernels holds, per staged column, ten words: cell u in
// row (u mod 8) + 1, with row 0 mirroring the slot-7 cell and row 9 the slot-0 cell,
// so that the cells u-1, u, u+1 sit in consecutive rows for every u. Columns are
// grouped in blocks of 64; a block stores its ten rows of 64 words one after another,
// so word (row, lcol) is at (lcol / 64) * 640 + row * 64 + lcol % 64. Lanes reading
// consecutive columns then hit consecutive banks whatever the row, and a row offset
// is a compile-time multiple of 64 words. Block 0 is the zero pad: its words are zero
// whenever a walk reads the ring, and a missing contact reads one of them.
constexpr int kRows = 10;
constexpr int kRingCells = 8;
constexpr int kBlkCols = 64;
constexpr int kBlkWords = kRows * kBlkCols;
constexpr int kPadCols = kBlkCols;  // LDS column of the first staged column
PERC_HD_INLINE int32_t ring_word(int32_t row, int32_t lcol) {
    return (lcol / kBlkCols) * kBlkWords + row * kBlkCols + lcol % kBlkCols;
}

// Contact table: for side contact i of column c (in tile k), the LDS word
// ring_word(1 + dcell, lcol) of that contact for a tube in ring slot 0, lcol being
// kPadCols + its column within the tile's staged range [halo first, halo end). A tube in
// slot s reads it s rows (64 s words) further. A missing contact reads a word of the
// zero pad block, ring_word(1, b).
//
// LDS serves the 32-bit reads of a wave in two halves of 32 lanes, over 32 banks (bank =
// word mod 32; the ring's row offsets are multiples of 64 words, so a contact's bank is
// the same in every row). The lanes of a tile walk are laid out so that no half-wave
// reads two different words of one bank for one contact direction: columns go to lanes
// in order, and where the next column's contacts would share a bank with a different
// word its half-wave already reads (the q-row boundaries of the hexagon shift the
// contact columns by one or two), the previous column is repeated on an idle lane first
// (ColumnSet::lanes; the repeat computes and stores exactly what the first does). A
// missing contact takes the pad word of a bank no other contact of its direction in its
// half-wave reads. The one-step table is stored by lane:
// word [j][k * lane_stride + l] holds contacts 2j (low 16 bits) and 2j + 1 of lane l of
// tile k.


// One lattice shape as the kernels see it (device pointers to the tables of its
// column set; the far cell of a column follows from sigma and L).
struct DevShape {
    const uint32_t* nboff;  // [kSide / 2][ntile * lane_stride] contact table by lane
    const uint16_t* lanes;  // [ntile][lane_stride] column (within its tile) of each lane
    const int32_t* tile;    // [ntile][4]
    const int32_t* rank;    // [C]
    const int32_t* sig;     // [C]
    const uint32_t* nboff2; // [ntile][kSide][span_max] two-step contact table (null: none)
    const int32_t* tile2;   // [ntile][2] outer ranges (null: none)
    int32_t C, CP, U, L;
    int32_t ntile, span_max, tile_max, W;
    int32_t ends;           // 1 with end contacts (modified lattice), 0 regular FCC
    int32_t span2_max;      // widest outer range (two-step form)
    int32_t lane_stride;    // lanes per tile in `lanes` (a multiple of 64)
    int64_t N, words;
};

// Device copies of the tables of one column set on one HIP device (kept for the process).
struct ColumnDevice {
    uint32_t* nboff = nullptr;
    uint16_t* lanes = nullptr;
    int32_t* tile = nullptr;
    int32_t* rank = nullptr;
    int32_t* sig = nullptr;
    uint32_t* nboff2 = nullptr;
    int32_t* tile2 = nullptr;
    uint32_t* nboff_whole = nullptr;  // the whole-cross-section tile, two contacts per word (null: none)
    uint16_t* lanes_whole = nullptr;  // its lanes
    uint32_t* nboff2_whole = nullptr; // the same, one contact per word (its two-step table)
    int32_t* tile_whole = nullptr;    // {0, C, 0, C, 0, C}: tile, then its outer range
};

// Dynamic LDS of the walking kernels: the ring from address 0, kPadCols + span columns
// (zero pad block, staged range) in whole blocks, then a fixed tail (the last kLdsTail bytes of
// the launch's allocation): the code table (1/deg per degree code: 16 words in a
// 256-byte slot), misc (16 words), part (256 floats).
constexpr uint32_t kLdsTail = 256u + 64u + 1024u;
PERC_HD inline uint32_t lds_total(int32_t span) {
    const uint32_t blocks = (uint32_t)(span + kPadCols + kBlkCols - 1) / kBlkCols;
    return blocks * kBlkWords * 4u + kLdsTail;
}
// Two steps per pass: the outer ring (outer range) from address 0, the inner ring (halo
// range) from word lds_ring2_words(span2), then the tail.
PERC_HD inline uint32_t lds_ring2_words(int32_t span2) {
    return (uint32_t)((span2 + kPadCols + kBlkCols - 1) / kBlkCols) * kBlkWords;
}
PERC_HD inline uint32_t lds_total2(int32_t span, int32_t span2) {
    return lds_ring2_words(span2) * 4u + lds_total(span);
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
    FORM_SPAN2 = 4,    // the span form with two steps per launch (one pass over HBM)
    FORM_PERSIST2 = 5, // the persistent form with two steps per pass over the whole
                       // cross-section (fibers of at most kWholeCols columns)
    FORM_MIXED = 6,    // per fiber: the persistent form for short walks (column tiles x
                       // unit cells at most kMixedWork), the span form beside it for the rest
};
constexpr int64_t kMixedWork = 600;

struct Tuning {
    int32_t form = FORM_AUTO;
    int32_t depth = 0;        // cells per work item (a tile walks them in one pass); 0 = choose
    int32_t block = 0;        // threads per workgroup (64..1024); 0 = choose
    int32_t graph_steps = 0;  // steps per graph replay (span form); 0 = choose
    int32_t grid = 0;         // workgroups per launch (span step / persistent); 0 = choose
};

// Per-configuration device state of the span and plain forms.
struct CfgState {
    int32_t front;    // largest cell holding a reached tube
    int32_t m;        // steps done
    int32_t done;     // 0 = active, 1 = decided, 2 = cap reached (error), 3 = decided with a
                      // detector hit after the first step of a two-step launch (the far-end
                      // words of that step are in SpanArgs::far1), 4 = the same after the
                      // first launch of a pair (that state is in the buffer not named by par),
                      // 5 = cancelled by the host (the planner drops it undecided)
    uint32_t flags;   // OR of the flags of the last launch (its first step); cleared by the planner
    uint32_t flags2;  // second-step flags of a two-step launch; cleared by the planner
    int32_t par;      // state buffer holding the newest state: 0 = ya, 1 = yb
    int32_t hz;       // degree codes are computed for cells [0, hz)
    int32_t hz_from;  // >= 0: cells [hz_from, hz) await the next extension launch
    int32_t ext_gen;  // extension launches done when hz_from was set
};

constexpr uint32_t F_GREW = 1u;      // some tube joined the reached set
constexpr uint32_t F_FRONT = 2u;     // the reached set entered cell front+1
constexpr uint32_t F_FAR = 4u;       // a far-end tube is reached: detector next step
constexpr uint32_t F_NONEMPTY = 8u;  // (initialisation) some start tube is metallic
constexpr uint32_t F_STEPPED = 16u;  // the last step launch advanced the configuration
constexpr uint32_t F_FUSED = 32u;    // ... by two steps (flags2 holds the second step's flags)
constexpr uint32_t F_FRONT2 = 64u;   // (second step) the reached set entered cell front+2

// Outputs, device pointers indexed by slot (span) or job (persistent).
struct BatchOut {
    uint8_t* perc = nullptr;
    int32_t* steps = nullptr;
    float* hit = nullptr;                       // first-passage probability at the stop
    unsigned long long* group_count = nullptr;  // percolating count per job group
    const int32_t* group = nullptr;             // group of each slot (span form), or null
    uint32_t* cap = nullptr;                    // persistent form: set to 1 when a configuration
                                                // reached the step cap (nullable)
};

// A configuration to inspect: its shape, and either caller bits or a Philox draw.
struct Job {
    const uint32_t* bits;  // canonical occupancy (device), or null: sample from Philox
    uint64_t seed;         // Philox key
    uint64_t cfg;          // Philox configuration index
    uint64_t thr;          // floor(p * 2^32)
    int32_t shape;         // index into the shape array
    int32_t group;         // output group (Pi count), or -1
};

// ---------------------------------------------------------------------------------
// Kernel launchers (kernels.hip).
// ---------------------------------------------------------------------------------

// Philox4x32-10 occupancy for configurations cfg0..cfg0+n_cfg-1 (canonical bits).
hipError_t launch_sample(const DevShape& sh, uint32_t* bits, int64_t n_cfg, uint64_t cfg0, uint64_t threshold,
                         uint64_t seed, hipStream_t s);

// Fixed-count occupancy: the K tubes with the smallest 64-bit Philox keys per configuration.
hipError_t launch_sample_fixed(const DevShape& sh, uint32_t* bits, int64_t n_cfg, uint64_t cfg0, int64_t K,
                               uint64_t seed, hipStream_t s);

// Philox occupancy of jobs idx[0..n): each into the buffer its bits pointer names.
hipError_t launch_sample_jobs(const DevShape* shapes, const Job* jobs, const int64_t* idx, int64_t n, hipStream_t s);

// Philox occupancy of the slots whose job has no caller bits (jobs indexed by slot).
hipError_t launch_sample_slots(const DevShape* shapes, const Job* jobs, int32_t n_slot, uint32_t* const* slot_bits,
                               hipStream_t s);

// Span/plain forms. Slot b holds one configuration: shape slot_shape[b], state words at
// slot_off[b] in ya/yb/code, occupancy bits slot_bits[b] (device pointer).
struct SpanArgs {
    const DevShape* shapes;
    const int32_t* slot_shape;
    const int64_t* slot_off;
    const uint32_t* const* slot_bits;
    float* ya;
    float* yb;
    uint8_t* code;
    CfgState* st;              // [n_slot]
    int32_t* active;           // [n_slot] active slots
    int32_t* active2;          // scratch for compaction
    int64_t* chunk_off;        // [n_slot + 1] prefix sums of items per active slot
    int32_t* hdr;              // [16]: n_active, total items, error flag, finished count, -,
                               // cells per item of the planned step (the planner's choice),
                               // slots listed for an extension, extension launches done
    unsigned long long* work;  // tube slots scheduled over all steps (planner adds)
    BatchOut out;
    const int32_t* ids;        // slots to initialise (null: all n_slot)
    int32_t n_ids;
    int32_t* fin;              // slots decided by the planner are appended here (nullable)
    int32_t n_slot;
    int32_t depth;             // cells per work item
    int32_t block;
    int32_t grid;
    int32_t lds;               // dynamic LDS bytes of the walking kernels
    int32_t fused;             // 1: each step launch does two steps (k_span_step2)
    int32_t pair;              // 1: two one-step launches between plans (sub 0, then sub 1)
    int32_t sub;               // this launch's place in a pair
    int32_t r1_off;            // two-step form: LDS word offset of the inner ring
    float* far1;               // two-step form: [n_slot][far1_stride] first-step far-end words
    int32_t far1_stride;
    int32_t resident;          // step-kernel workgroups the device holds at once (0: items
                               // always `depth` cells; else the planner shortens the items of
                               // short work lists so that they spread over the device)
    // Lazy initialisation (1): a slot starts with the codes of its first cells only; a plan
    // that finds its front within init_margin cells of hz lists it (ext_ids, items prefix
    // ext_off) and moves hz on; the extension launch at the start of the next run of steps
    // computes the listed ranges. 0: every cell is initialised at once (hz = U).
    int32_t lazy;
    int32_t init_margin;       // > the steps a launch sequence runs between extensions + 3
    int32_t* ext_ids;          // [n_slot]
    int64_t* ext_off;          // [n_slot + 1]
    int32_t list_ext;          // 1: this plan (the last before an extension launch) lists
};

// Workgroups of k_span_step with this block size and dynamic LDS that the current device
// runs at once (0 if the runtime cannot tell).
int32_t span_step_resident(int32_t block, int32_t lds);

hipError_t launch_span_init(const SpanArgs& a, hipStream_t s);       // codes, y0, first plan
hipError_t launch_span_init_only(const SpanArgs& a, hipStream_t s);  // codes and y0 only
hipError_t launch_span_step(const SpanArgs& a, hipStream_t s);       // one step (two if a.fused) over the work list
hipError_t launch_span_step2(const SpanArgs& a, hipStream_t s);      // two steps over the work list
hipError_t launch_span_plan(const SpanArgs& a, hipStream_t s);       // decide, compact, plan
hipError_t launch_span_extend(const SpanArgs& a, hipStream_t s);     // codes of the listed ranges
hipError_t launch_span_finish(const SpanArgs& a, hipStream_t s);     // first-hit probabilities, counts

// Persistent form: one workgroup per job, scratch per resident workgroup.
struct PersistArgs {
    const DevShape* shapes;
    const Job* jobs;           // [n_jobs], every one with its occupancy bits
    int64_t n_jobs;
    float* ya;                 // [grid][state_stride]
    float* yb;
    uint8_t* code;
    int64_t state_stride;
    unsigned long long* queue;  // next position of `order` to take
    const int64_t* order;       // [n_jobs] the job at each queue position (longest expected first)
    uint32_t* err;              // set when a configuration reached the step cap
    unsigned long long* work;   // tube slots the steps advanced (nullable)
    BatchOut out;
    int32_t depth;
    int32_t block;
    int32_t grid;
    int32_t lds;
    // two steps per pass (every shape the whole-cross-section tile): first-step far-end
    // words per workgroup, and the LDS word offset of the inner ring
    int32_t two;
    int32_t r1_off;
    float* far1;               // [grid][far1_stride]
    int64_t far1_stride;
};
hipError_t launch_persist(const PersistArgs& a, hipStream_t s);
int persist2_resident_per_cu(int block, int lds_bytes);

// Test hook: one step of one configuration over all cells; detector accumulation;
// export of x = |y| deg (canonical order) and the reach bits, detector last.
hipError_t launch_chunk_step(const DevShape& sh, const float* yin, float* yout, const uint8_t* code, int depth,
                             int block, hipStream_t s);
hipError_t launch_far_sum(const DevShape& sh, const float* y, float* det_mass, uint32_t* det_reached,
                          hipStream_t s);
hipError_t launch_backward_init(const DevShape& sh, const uint8_t* code, float* y, int64_t stride, int n_cfg,
                                hipStream_t s);
hipError_t launch_export_raw(const DevShape& sh, const float* y, float* f_out, int64_t stride, int n_cfg,
                             hipStream_t s);
hipError_t launch_multi_step(const DevShape& sh, const float* yin, float* yout, const uint8_t* code, int64_t stride,
                             int n_cfg, int depth, int block, hipStream_t s);
hipError_t launch_steps_hist(const uint8_t* perc, const int32_t* steps, int64_t n, int32_t nbins,
                             unsigned long long* hist, hipStream_t s);
hipError_t launch_export(const DevShape& sh, const float* y, const uint8_t* code, const float* det_mass,
                         const uint32_t* det_reached, float* x_out, uint8_t* reach_out, hipStream_t s);

// Count of percolating configurations (integer, deterministic).
hipError_t launch_count(const uint8_t* perc, int64_t n, unsigned long long* count, hipStream_t s);
hipError_t launch_fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t s);
// Outputs of job i of a part (perc, steps and, if non-null, hit) to the places of job
// idx[i] of the batch.
hipError_t launch_scatter_out(int64_t n, const int64_t* idx, const uint8_t* perc, const int32_t* steps,
                              const float* hit, uint8_t* perc_out, int32_t* steps_out, float* hit_out,
                              hipStream_t s);

int persist_resident_per_cu(int block, int lds_bytes);

// Streaming copy of n16 16-byte words (perc_stream_copy).
hipError_t launch_stream_copy(const void* src, void* dst, int64_t n16, int grid, hipStream_t s);

// The fixed work array of perc_inspect_noalloc on the current device: its device address
// (taken with hipGetSymbolAddress on the first call per device) and size.
constexpr size_t kScratchBytes = (size_t)256 << 20;
hipError_t scratch_region(void** ptr, size_t* bytes);
// slot_shape[b] = 0, slot_off[b] = b * stride, slot_bits[b] = bits + b * words, b < n.
hipError_t launch_slot_table(int32_t* slot_shape, int64_t* slot_off, const uint32_t** slot_bits, int32_t n,
                             int64_t stride, const uint32_t* bits, int64_t words, hipStream_t s);
hipError_t prepare_kernels(int device);

}  // namespace perc
