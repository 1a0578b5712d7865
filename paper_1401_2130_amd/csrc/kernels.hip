// HIP kernels (gfx950, wave64) of the percolation inspection.
//
// The method (Sec. II.B, Eq. 1-4): a random walker on the metallic tubes moves to
// each metallic contact with probability 1/deg; a detector site joined to every
// metallic far-end tube absorbs it. Mass injected uniformly on the metallic start
// tubes is pushed forward one step at a time (x <- x P, Jacobi). The configuration
// percolates iff the detector ever receives non-zero probability; the iteration
// stops at the first such step or when the set of tubes with non-zero probability in
// exact arithmetic (the reached set) stops growing.
//
// Representation (one FP32 word per tube, per state buffer): y = x / deg, the mass the
// tube sends along each of its deg contacts, so a receiver sums its neighbours' words
// and scales by its own 1/deg only. The word of a tube is non-zero exactly when the
// tube is in the reached set: a reached tube whose FP32 mass underflows keeps the
// smallest positive (denormal) value instead of zero (denormals are preserved in these
// kernels), so the sum over a tube's contacts is non-zero iff one of them is reached.
// The decision never looks at a mass beyond that test; the floor moves a mass by at
// most 2^-149 per step.
// Per tube a byte `code` holds deg (0..14) of a metallic tube, 15 for an insulating or
// absent one. A metallic tube of degree 0 keeps its mass (self-loop, Sec. II.B).
//
// Cell u of column c holds layer 3u + sigma(c) (see perc_internal.hpp); the state of a
// configuration is stored in groups of four cells (layout below). Work is cut into
// items: one tile of consecutive columns x a range of cells. A workgroup walks its
// item along the fiber axis, one thread per column of the tile: the tile's halo range
// of columns is staged in an LDS ring of eight cell slots (plus two mirrored rows, so
// that any three consecutive cells sit in consecutive rows), four-cell groups are
// fetched two groups ahead, with two barriers per group. The 14 contacts of a tube
// are LDS reads at per-column word offsets held in registers for the whole walk plus a
// compile-time row offset. All LDS of these kernels is dynamic, so the ring sits at
// address 0.
#include <hip/hip_runtime.h>

#include <mutex>

#include "perc_internal.hpp"

namespace perc {

namespace {

constexpr int kMaxBlock = 1024;
constexpr int kXcds = 8;         // MI355X: workgroups are dealt round-robin over 8 XCDs
constexpr int kLoadCols = 2;     // staged columns per thread: span <= 2 * blockDim

extern __shared__ __align__(16) unsigned char lds[];

__device__ __forceinline__ void lds_put_u32(uint32_t off, uint32_t v) { *reinterpret_cast<uint32_t*>(lds + off) = v; }

// Fixed tail of the dynamic LDS of a launch of `total` bytes.
struct Tail {
    float* ct;  // the code table
    uint32_t* misc;
    float* part;
};
__device__ __forceinline__ Tail lds_tail(int total) {
    const uint32_t t = (uint32_t)total - kLdsTail;  // a multiple of 16
    return Tail{reinterpret_cast<float*>(lds + t), reinterpret_cast<uint32_t*>(lds + t + 256),
                reinterpret_cast<float*>(lds + t + 320)};
}

// ------------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11): ten rounds; each round takes
// the 32x32 -> 64-bit products of counter words 0 and 2 with the two multipliers and
// mixes the high halves with counter words 1, 3 and the round key; the key advances
// by the two Weyl increments between rounds.
// ------------------------------------------------------------------------------
struct Ctr4 { uint32_t v0, v1, v2, v3; };

__device__ __forceinline__ Ctr4 philox4x32_10(Ctr4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint32_t a = c.v0, b = c.v2;
        const uint32_t lo0 = a * 0xD2511F53u, hi0 = __umulhi(a, 0xD2511F53u);
        const uint32_t lo1 = b * 0xCD9E8D57u, hi1 = __umulhi(b, 0xCD9E8D57u);
        c = Ctr4{hi1 ^ c.v1 ^ k0, lo1, hi0 ^ c.v3 ^ k1, lo0};
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// Occupancy word w (sites 32w .. 32w+31) of global configuration gcfg: site s uses
// output word s mod 4 of counter (s / 4, gcfg lo, gcfg hi, tag) under key = seed; it is
// metallic iff that 32-bit draw is below the threshold floor(p * 2^32).
__device__ __forceinline__ uint32_t sample_word(int64_t w, int64_t N, uint64_t gcfg, uint64_t thr,
                                                uint32_t k0, uint32_t k1, uint32_t tag) {
    uint32_t out = 0;
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        const int64_t s0 = w * 32 + b * 4;
        if (s0 >= N) break;
        const Ctr4 r = philox4x32_10(Ctr4{(uint32_t)(s0 >> 2), (uint32_t)gcfg, (uint32_t)(gcfg >> 32), tag},
                                     k0, k1);
        const uint32_t v[4] = {r.v0, r.v1, r.v2, r.v3};
#pragma unroll
        for (int e = 0; e < 4; ++e)
            if (s0 + e < N && (uint64_t)v[e] < thr) out |= 1u << (b * 4 + e);
    }
    return out;
}

__device__ __forceinline__ uint32_t shape_tag(const DevShape& sh) { return ((uint32_t)sh.W << 16) | (uint32_t)sh.L; }

// Per degree code d, one word (consecutive words: the lanes of a half-wave reading
// different codes hit different LDS banks): the correctly rounded FP32 reciprocal 1/d
// for d = 1..14; 1 for d = 0 (a metallic tube without metallic contact keeps its mass);
// 0 for 15 (insulating). A tube's self weight and reach floor follow from its code.
__device__ __forceinline__ void fill_codes(float* ct) {
    if (threadIdx.x < 16) {
        const int d = threadIdx.x;
        ct[d] = d == 0 ? 1.0f : (d == 15 ? 0.0f : 1.0f / (float)d);
    }
}

__device__ __forceinline__ float mag(uint32_t w) { return __uint_as_float(w & 0x7fffffffu); }

// A new state quad to HBM as a streaming (non-temporal) store: it is read again only by
// the next step, so it should not take L2 lines from the input state, whose halo
// columns neighbouring tiles of the same cells read again.
__device__ __forceinline__ void store_quad_nt(float* y, uint32_t q, uint32_t a, uint32_t b, uint32_t c, uint32_t d) {
    typedef uint32_t v4u __attribute__((ext_vector_type(4)));
    const v4u v = {a, b, c, d};
    __builtin_nontemporal_store(v, reinterpret_cast<v4u*>(y) + q);
}

// Cell of the far-end tube of column c: the highest layer k < L with k = sigma (mod 3),
// or -1 if the column holds no tube.
__device__ __forceinline__ int top_of(const DevShape& sh, int c) {
    const int sg = sh.sig[c];
    return sg < sh.L ? (sh.L - 1 - sg) / 3 : -1;
}


struct TileV {
    int ts, te, hs, he;
    int lm;  // first lane of the tile in the lane tables
};
// A value every lane of the workgroup reads from the same address, moved into scalar
// registers (the compiler cannot prove such loads uniform when the kernel also
// writes global memory).
__device__ __forceinline__ int32_t uniform_i32(const int32_t* p) { return __builtin_amdgcn_readfirstlane(*p); }
__device__ __forceinline__ int64_t uniform_i64(const int64_t* p) {
    const uint32_t* w = reinterpret_cast<const uint32_t*>(p);
    const uint32_t lo = __builtin_amdgcn_readfirstlane(w[0]), hi = __builtin_amdgcn_readfirstlane(w[1]);
    return (int64_t)(((uint64_t)hi << 32) | lo);
}
template <typename T>
__device__ __forceinline__ T uniform_load(const T* p) {
    static_assert(sizeof(T) % 4 == 0, "whole words");
    T v;
    const uint32_t* src = reinterpret_cast<const uint32_t*>(p);
    uint32_t* dst = reinterpret_cast<uint32_t*>(&v);
#pragma unroll
    for (int i = 0; i < (int)(sizeof(T) / 4); ++i) dst[i] = __builtin_amdgcn_readfirstlane(src[i]);
    return v;
}

__device__ __forceinline__ TileV load_tile(const DevShape& sh, int k) {
    const int32_t* p = sh.tile + 4 * k;
    return TileV{uniform_i32(p), uniform_i32(p + 1), uniform_i32(p + 2), uniform_i32(p + 3), k * sh.lane_stride};
}

// ------------------------------------------------------------------------------
// State layout in HBM: the cells of a configuration are taken in groups of four
// (cells 4g .. 4g+3); word k of the 16-byte quad (g, c) holds cell 4g+k of column c,
// quads in [group][CP] order, so one 16-byte load or store moves four cells of a
// column and a wave's 64 columns are 1 KiB contiguous.
// ------------------------------------------------------------------------------
__device__ __forceinline__ uint32_t quad_of(const DevShape& sh, int g, int c) { return (uint32_t)g * sh.CP + c; }
__device__ __forceinline__ uint32_t word_of(const DevShape& sh, int u, int c) {
    return quad_of(sh, u >> 2, c) * 4u + (uint32_t)(u & 3);
}
// Degree codes: four bits per tube (0..14 the degree of a metallic tube, 15 insulating
// or absent), eight cells 8o..8o+7 of column c in one 32-bit word, cell u in bits
// 4 (u mod 8) .. +3, words in [octet][CP] order. The word holding group g:
__device__ __forceinline__ uint32_t code_word_g(const DevShape& sh, int g, int c) {
    return (uint32_t)(g >> 1) * sh.CP + c;
}
__device__ __forceinline__ uint32_t code_of(const uint32_t* __restrict__ code8, const DevShape& sh, int u, int c) {
    return (code8[(uint32_t)(u >> 3) * sh.CP + c] >> (4 * (u & 7))) & 0xfu;
}

// ------------------------------------------------------------------------------
// The ring (ring_word in perc_internal.hpp): per staged column, cell u in row
// (u mod 8) + 1, the slot-7 cell also in row 0 and the slot-0 cell also in row 9, so
// the cells u-1, u, u+1 sit in consecutive rows for every u; rows are 64 words apart
// within a block of 64 columns. Block 0 (LDS columns 0..63) is the zero pad: a missing
// contact reads one of its words, in a bank that no other lane of the wave reads for
// that contact, and staged column lc is LDS column lc + kPadCols.
//
// A walk covers whole groups from an 8-aligned cell, one cell per phase, eight phases
// unrolled so that every ring slot is a compile-time constant. At the second cell of
// group g the next group g+1 goes from registers into the ring (its slots held group
// g-1, whose last cell only the first cell of g reads) and group g+2 is fetched: four
// cells of work between the issue of a load and its use. Two barriers per group
// suffice: one before that write (after the first cell's reads) and one before the
// last cell, the first to read group g+1. Global
// loads are never predicated: the group index is clamped into the configuration and
// the words are masked when written to the ring.
// ------------------------------------------------------------------------------
// NJ: staged column slots per thread (span <= NJ * blockDim).
template <int NJ>
struct StageN {
    int col[NJ];         // global column of each staged column of this thread (clamped)
    uint32_t* slot[NJ];  // its LDS column (row 0)
    bool ok[NJ];         // inside the halo range
    int nj;              // staged column slots the workgroup needs (uniform)
};
using Stage = StageN<kLoadCols>;

__device__ __forceinline__ Stage stage_columns(const TileV& tv) {
    Stage st;
    const int span = tv.he - tv.hs;
    st.nj = (span + (int)blockDim.x - 1) / (int)blockDim.x;
    uint32_t* base = reinterpret_cast<uint32_t*>(lds);
#pragma unroll
    for (int j = 0; j < kLoadCols; ++j) {
        const int lc = (int)threadIdx.x + j * (int)blockDim.x;
        st.ok[j] = lc < span;
        st.col[j] = st.ok[j] ? tv.hs + lc : tv.hs;
        st.slot[j] = base + ring_word(0, st.ok[j] ? lc + kPadCols : 0);
    }
    return st;
}

// The pad block (block 0: every row of LDS columns 0..63) of the ring at r holds zeros.
// (One word per store: with 16-byte stores the step walk needs more VGPRs than six
// waves per SIMD allow.)
__device__ __forceinline__ void zero_pad(uint32_t* r) {
    for (int i = (int)threadIdx.x; i < kBlkWords; i += (int)blockDim.x) r[i] = 0u;
}
__device__ __forceinline__ void zero_pad() { zero_pad(reinterpret_cast<uint32_t*>(lds)); }

// Four ring words v[0..3] of group g into ring slots S0 .. S0+3 (S0 = 0 or 4) of staged
// column j, with the mirror of the slot-0 or slot-7 cell. Cells outside [0, vmax] hold
// no mass (their words are not meaningful) and are written as zero.
template <int S0>
__device__ __forceinline__ void put_quad(uint32_t* slot, int g, int vmax, uint4 q) {
    const int u = 4 * g;
    const uint32_t a = (u >= 0 && u <= vmax) ? q.x : 0u;
    const uint32_t b = (u + 1 >= 0 && u + 1 <= vmax) ? q.y : 0u;
    const uint32_t c = (u + 2 >= 0 && u + 2 <= vmax) ? q.z : 0u;
    const uint32_t d = (u + 3 >= 0 && u + 3 <= vmax) ? q.w : 0u;
    slot[(S0 + 1) * kBlkCols] = a;
    slot[(S0 + 2) * kBlkCols] = b;
    slot[(S0 + 3) * kBlkCols] = c;
    slot[(S0 + 4) * kBlkCols] = d;
    if (S0 == 0) slot[(kRingCells + 1) * kBlkCols] = a;
    if (S0 == 4) slot[0] = d;
}

// Raw state quads of group g (clamped into [0, vmax / 4]) for the staged columns.
template <int NJ>
__device__ __forceinline__ void load_quads(const DevShape& sh, const StageN<NJ>& st, const float* __restrict__ y, int g,
                                           int vmax, uint4 (&out)[NJ]) {
    const uint4* q = reinterpret_cast<const uint4*>(y) + (uint32_t)min(max(g, 0), vmax >> 2) * sh.CP;
#pragma unroll
    for (int j = 0; j < NJ; ++j) out[j] = j < st.nj ? q[st.col[j]] : make_uint4(0u, 0u, 0u, 0u);
}

template <int S0, int NJ>
__device__ __forceinline__ void put_quads(const StageN<NJ>& st, int g, int vmax, const uint4 (&q)[NJ]) {
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        if (j >= st.nj) break;
        if (st.ok[j]) put_quad<S0>(st.slot[j], g, vmax, q[j]);
    }
}

// Per-thread view of its own column: the 12 contacts and its own ring words. The lane
// tables give each thread its column; an idle lane repeats a column of the tile (so does
// every thread beyond the tables): it computes (and stores) exactly what that column's
// lane does, so no compute or store needs a lane predicate.
struct Own {
    const uint32_t* nb[kSide];
    const uint32_t* me;
    int c, top;
};

__device__ __forceinline__ Own own_column_in(const DevShape& sh, const TileV& tv, const uint32_t* base) {
    Own w;
    const int l = tv.lm + min((int)threadIdx.x, sh.lane_stride - 1);
    const int nl = sh.ntile * sh.lane_stride;
#pragma unroll
    for (int j = 0; j < kSide / 2; ++j) {
        const uint32_t v = sh.nboff[j * nl + l];  // contacts 2j and 2j + 1
        w.nb[2 * j] = base + (v & 0xffffu);
        w.nb[2 * j + 1] = base + (v >> 16);
    }
    w.c = tv.ts + (int)sh.lanes[l];
    w.me = base + ring_word(0, w.c - tv.hs + kPadCols);
    w.top = top_of(sh, w.c);
    return w;
}
__device__ __forceinline__ Own own_column(const DevShape& sh, const TileV& tv) {
    return own_column_in(sh, tv, reinterpret_cast<const uint32_t*>(lds));
}

// The update of one tube (Eq. 3 on the stored words y = x / deg): the 12 side contacts
// and the two end contacts summed in one fixed pairwise order (in-layer pairs, up/down
// layer pairs, then the end contacts), then the table entry of the tube's degree code.
// Every walk calls this, so a tube gets the same bits whichever kernel computes it.
__device__ __forceinline__ uint32_t tube_update(const uint32_t (&n)[kSide], uint32_t dn, uint32_t up, uint32_t own,
                                                int32_t ends, const float* ct, uint32_t cd) {
    const float s01 = mag(n[0]) + mag(n[1]);
    const float s23 = mag(n[2]) + mag(n[3]);
    const float s45 = mag(n[4]) + mag(n[5]);
    const float s67 = mag(n[6]) + mag(n[7]);
    const float s89 = mag(n[8]) + mag(n[9]);
    const float sab = mag(n[10]) + mag(n[11]);
    const float sud = ends ? mag(dn) + mag(up) : 0.0f;
    const float sum = ((s01 + s23) + (s45 + s67)) + ((s89 + sab) + sud);
    // the table entry's 1/deg from LDS; its self weight (1 for degree 0) and reach floor
    // (2^-149, bits 1, for a metallic tube) follow from the code itself
    const float rcp = ct[cd];
    const float self = cd == 0u ? 1.0f : 0.0f;
    const uint32_t floor_bits = cd < 15u ? 1u : 0u;
    // a metallic tube of degree 0 has no metallic contact (sum == 0): it keeps its own
    // mass (self weight 1); for every other code the own word enters with weight 0
    const float x = fmaf(__uint_as_float(own), self, sum);
    // reached: metallic (the floor is 0 otherwise), and reached before or next to a
    // reached tube. The new word is non-zero exactly for reached tubes: cells beyond
    // the cut have no reached input, cells beyond U are coded insulating.
    // All words are non-negative floats (never -0), ordered like their bit patterns, so
    // max(x / deg, floor if x != 0 or own != 0) is an unsigned maximum, and the floor's
    // bits (0 or 1) against the bits of x | own (0 exactly when neither is reached) an
    // unsigned minimum.
    const uint32_t floor_w = min(floor_bits, __float_as_uint(x) | own);
    return max(__float_as_uint(x * rcp), floor_w);
}

struct StepState {
    uint4 next[kLoadCols];  // staged quads of the group after the current one
    uint32_t cq[2];         // code words of the current and the next eight cells
    uint32_t res[4];        // new words of the current group
    uint32_t grew = 0;      // OR of the new words of tubes that were not reached before
    uint32_t far = 0, entered = 0, entered2 = 0;
};

// Cell u = u8 + K (ring slot K) of a step walk.
template <int K>
__device__ __forceinline__ void step_cell(const DevShape& sh, const Stage& st, const Own& w, const float* ct,
                                          const float* __restrict__ yin, float* __restrict__ yout,
                                          const uint32_t* __restrict__ code4, int u8, int ue, int front, int vmax,
                                          int top_min, StepState& ss) {
    constexpr int k = K & 3, par = K >> 2;
    const int u = u8 + K, g = u >> 2;
    if (k & 1) __syncthreads();
    if (k == 1) {
        put_quads<(par ^ 1) * 4>(st, g + 1, vmax, ss.next);
        // group g + 2 only if a cell the walk computes reads it: the cells of the last
        // group the walk enters, (ue - 1) / 4, read one group further (a uniform branch;
        // a skipped load leaves words that no computed cell reads)
        if (g + 2 <= ((ue - 1) >> 2) + 1) load_quads(sh, st, yin, g + 2, vmax, ss.next);
        // the code word of the next eight cells, once per eight cells, if the walk gets there
        if (K == 1 && u8 + 8 < ue) ss.cq[1] = code4[(uint32_t)min((u8 >> 3) + 1, (sh.U - 1) >> 3) * sh.CP + w.c];
    }
    const uint32_t cd = (ss.cq[0] >> (4 * K)) & 0xfu;
    if (K == 7) ss.cq[0] = ss.cq[1];
    const uint32_t own = w.me[(K + 1) * kBlkCols];
    const uint32_t dn = w.me[K * kBlkCols];
    const uint32_t up = w.me[(K + 2) * kBlkCols];
    uint32_t n[kSide];
#pragma unroll
    for (int i = 0; i < kSide; ++i) n[i] = w.nb[i][K * kBlkCols];
    ss.res[k] = tube_update(n, dn, up, own, sh.ends, ct, cd);
    ss.grew |= own == 0u ? ss.res[k] : 0u;
    if (k == 3) {
        const int u4 = u - 3;
        store_quad_nt(yout, quad_of(sh, g, w.c), ss.res[0], ss.res[1], ss.res[2], ss.res[3]);
        // far-end tubes lie in the last cells of the fiber; the front cell in one group
        if (u4 + 3 >= top_min) {
            const int kt = w.top - u4;
            ss.far |= kt == 0 ? ss.res[0] : kt == 1 ? ss.res[1] : kt == 2 ? ss.res[2] : kt == 3 ? ss.res[3] : 0u;
        }
        const int kf = front + 1 - u4, kf2 = front + 2 - u4;
        if (kf >= 0 && kf < 4)
            ss.entered |= kf == 0 ? ss.res[0] : kf == 1 ? ss.res[1] : kf == 2 ? ss.res[2] : ss.res[3];
        if (kf2 >= 0 && kf2 < 4)
            ss.entered2 |= kf2 == 0 ? ss.res[0] : kf2 == 1 ? ss.res[1] : kf2 == 2 ? ss.res[2] : ss.res[3];
    }
}

// One Jacobi step of the tile's tubes in cells [ub, ue) (cut at min(U, front+2); ub a
// multiple of 8), reading yin, whose reached tubes lie in cells <= front, and writing
// yout. Returns this thread's step flags; the front flags tell whether the new state
// reaches cell front_chk+1 (F_FRONT) and front_chk+2 (F_FRONT2). The
// 14 contributions are summed in one fixed pairwise order, so a tube gets the same
// FP32 result in every execution form, item layout and batch composition. The words
// written for cells of the last group at or beyond the cut are zero (their inputs are
// beyond the front) or lie in the padding beyond U: no other item writes them and no
// reader uses them.
// LEAD: the three leading groups are loaded together (one memory latency before the
// first cell instead of two; the persistent form's walks, one per tile and step, gain
// from it, the span form's do not).
template <bool LEAD = false>
__device__ __forceinline__ uint32_t walk_step(const DevShape& sh, const TileV& tv, const float* ct,
                                              const float* __restrict__ yin, float* __restrict__ yout,
                                              const uint8_t* __restrict__ code, int ub, int ue, int front,
                                              int front_chk) {
    ue = min(ue, min(sh.U, front + 2));
    if (ub >= ue) return 0u;
    const int vmax = min(front, sh.U - 1);
    const int top_min = (sh.L - 3) / 3;  // no far-end tube lies in an earlier cell
    const uint32_t* code4 = reinterpret_cast<const uint32_t*>(code);
    const Stage st = stage_columns(tv);
    const Own w = own_column(sh, tv);
    const int g0 = ub >> 2;
    __syncthreads();  // the ring may still be read by a previous item
    zero_pad();
    StepState ss;
    uint4 q[kLoadCols];
    // group g0 - 1 lies below the fiber when the walk starts at its base: its words are
    // written as zero and nothing is loaded (a uniform branch)
#pragma unroll
    for (int j = 0; j < kLoadCols; ++j) q[j] = make_uint4(0u, 0u, 0u, 0u);
    if (LEAD) {
        uint4 q0[kLoadCols];
        if (g0 > 0) load_quads(sh, st, yin, g0 - 1, vmax, q);
        load_quads(sh, st, yin, g0, vmax, q0);
        load_quads(sh, st, yin, g0 + 1, vmax, ss.next);
        put_quads<4>(st, g0 - 1, vmax, q);
        put_quads<0>(st, g0, vmax, q0);
    } else {
        if (g0 > 0) load_quads(sh, st, yin, g0 - 1, vmax, q);
        put_quads<4>(st, g0 - 1, vmax, q);
        load_quads(sh, st, yin, g0, vmax, q);
        put_quads<0>(st, g0, vmax, q);
        load_quads(sh, st, yin, g0 + 1, vmax, ss.next);
    }
    ss.cq[0] = code4[code_word_g(sh, g0, w.c)];
    ss.cq[1] = 0xffffffffu;  // (g0 is even: the first word covers g0 and g0 + 1)
    __syncthreads();
    for (int u8 = ub; u8 < ue; u8 += kRingCells) {
        step_cell<0>(sh, st, w, ct, yin, yout, code4, u8, ue, front_chk, vmax, top_min, ss);
        step_cell<1>(sh, st, w, ct, yin, yout, code4, u8, ue, front_chk, vmax, top_min, ss);
        step_cell<2>(sh, st, w, ct, yin, yout, code4, u8, ue, front_chk, vmax, top_min, ss);
        step_cell<3>(sh, st, w, ct, yin, yout, code4, u8, ue, front_chk, vmax, top_min, ss);
        if (u8 + 4 >= ue) break;
        step_cell<4>(sh, st, w, ct, yin, yout, code4, u8, ue, front_chk, vmax, top_min, ss);
        step_cell<5>(sh, st, w, ct, yin, yout, code4, u8, ue, front_chk, vmax, top_min, ss);
        step_cell<6>(sh, st, w, ct, yin, yout, code4, u8, ue, front_chk, vmax, top_min, ss);
        step_cell<7>(sh, st, w, ct, yin, yout, code4, u8, ue, front_chk, vmax, top_min, ss);
    }
    return (ss.grew ? F_GREW : 0u) | (ss.far ? F_FAR : 0u) | (ss.entered ? F_FRONT : 0u) |
           (ss.entered2 ? F_FRONT2 : 0u);
}

// ------------------------------------------------------------------------------
// Two steps per pass. An item is a tile and a cell range, as for one step. The outer
// ring R0 holds the input state of the tile's outer range [os, oe) (the halo of its halo
// range); the first step is computed for every column of the halo range [hs, he) into
// the inner ring R1, which has the layout of the one-step ring (so the one-step contact
// table addresses it); the second step is computed for the tile's columns from R1 and
// written to HBM. The first step runs one group of four cells ahead of the second, and
// the cell ranges of neighbouring items overlap by one group of first-step work on each
// side. Every tube is computed by tube_update, so the two steps give the bits of two
// single steps; first-step words of a tube computed by several items are identical.
// ------------------------------------------------------------------------------

// Halo-range columns of this thread that compute the first step (up to NJ).
template <int NJ>
struct Prod {
    const uint32_t* nb[NJ][kSide];  // R0 word of each side contact (slot 0)
    const uint32_t* me[NJ];         // own column in R0 (row 0)
    uint32_t* out[NJ];              // own column in R1 (row 0)
    int c[NJ];
    int top[NJ];
    bool ok[NJ];  // a halo-range column (else a copy of the first one, not stored)
    int n;        // column slots in use (uniform)
};

template <int NJ>
__device__ __forceinline__ StageN<NJ> stage_range(int hs, int he, uint32_t* base) {
    StageN<NJ> st;
    const int span = he - hs;
    st.nj = (span + (int)blockDim.x - 1) / (int)blockDim.x;
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        const int lc = (int)threadIdx.x + j * (int)blockDim.x;
        st.ok[j] = lc < span;
        st.col[j] = st.ok[j] ? hs + lc : hs;
        st.slot[j] = base + ring_word(0, st.ok[j] ? lc + kPadCols : 0);
    }
    return st;
}

template <int NJ>
__device__ __forceinline__ Prod<NJ> prod_columns(const DevShape& sh, int k, const TileV& tv, int os,
                                                 const uint32_t* r0, uint32_t* r1) {
    Prod<NJ> p;
    const int span = tv.he - tv.hs;
    p.n = (span + (int)blockDim.x - 1) / (int)blockDim.x;
    const uint32_t* tab = sh.nboff2 + (size_t)k * kSide * sh.span_max;
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        const int lc = (int)threadIdx.x + j * (int)blockDim.x;
        p.ok[j] = lc < span;
        const int l = p.ok[j] ? lc : 0;
        p.c[j] = tv.hs + l;
#pragma unroll
        for (int i = 0; i < kSide; ++i) p.nb[j][i] = r0 + tab[i * sh.span_max + l];
        p.me[j] = r0 + ring_word(0, p.c[j] - os + kPadCols);
        p.out[j] = r1 + ring_word(0, l + kPadCols);
        p.top[j] = top_of(sh, p.c[j]);
    }
    return p;
}

template <int NJ>
struct Step2State {
    uint4 next[NJ];        // staged outer quads of the group after the current one
    uint32_t cq1[2][NJ];   // halo-range code words, by group parity
    uint32_t cq2[2];       // tile code words, by group parity
    uint32_t r2[4];        // second-step words of the group before
    uint32_t first0[NJ];   // first-step words of the group's first cell (stored late)
    uint32_t grew1 = 0, far1 = 0, ent1 = 0;
    uint32_t grew2 = 0, far2 = 0, ent2a = 0, ent2b = 0;
};

// First step of cell u (ring slot K) for every halo-range column of this thread, written
// to the same slot of R1 (with the mirror row of slots 0 and 7). Words outside [0, vmax1]
// are set to zero: those cells hold no mass after the first step.
template <int K, int NJ>
__device__ __forceinline__ void first_cell(const DevShape& sh, const Prod<NJ>& p, const float* ct, int u, int vmax1,
                                           int front, float* __restrict__ far1, Step2State<NJ>& ss) {
    constexpr int k = K & 3, par = K >> 2;
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        if (j >= p.n) break;
        const uint32_t cd = (ss.cq1[par][j] >> (4 * K)) & 0xfu;
        const uint32_t own = p.me[j][(K + 1) * kBlkCols];
        const uint32_t dn = p.me[j][K * kBlkCols];
        const uint32_t up = p.me[j][(K + 2) * kBlkCols];
        uint32_t n[kSide];
#pragma unroll
        for (int i = 0; i < kSide; ++i) n[i] = p.nb[j][i][K * kBlkCols];
        uint32_t v = tube_update(n, dn, up, own, sh.ends, ct, cd);
        v = (u >= 0 && u <= vmax1) ? v : 0u;
        if ((K & 3) == 0) {
            ss.first0[j] = v;  // its R1 row may still be read before the next barrier
        } else if (p.ok[j]) {
            p.out[j][(K + 1) * kBlkCols] = v;
            if (K == kRingCells - 1) p.out[j][0] = v;
        }
        ss.grew1 |= own == 0u ? v : 0u;
        ss.ent1 |= u == front + 1 ? v : 0u;
        if (u == p.top[j]) {
            ss.far1 |= v;
            if (far1 && p.ok[j]) far1[p.c[j]] = __uint_as_float(v);
        }
    }
}

// The first-step words of the first cell of a group (ring slot K), with the mirror row.
template <int K, int NJ>
__device__ __forceinline__ void store_first0(const Prod<NJ>& p, const Step2State<NJ>& ss) {
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        if (j >= p.n) break;
        if (!p.ok[j]) continue;
        p.out[j][(K + 1) * kBlkCols] = ss.first0[j];
        if (K == 0) p.out[j][(kRingCells + 1) * kBlkCols] = ss.first0[j];
    }
}

// Second step of cell u (ring slot K of R1) for this thread's tile column; at the last
// cell of the group its quad goes to HBM.
template <int K, int NJ>
__device__ __forceinline__ void second_cell(const DevShape& sh, const Own& w, const float* ct, int u, int front,
                                            int top_min, float* __restrict__ yout, Step2State<NJ>& ss) {
    constexpr int k = K & 3, par = K >> 2;
    const uint32_t cd = (ss.cq2[par] >> (4 * K)) & 0xfu;
    const uint32_t own = w.me[(K + 1) * kBlkCols];
    const uint32_t dn = w.me[K * kBlkCols];
    const uint32_t up = w.me[(K + 2) * kBlkCols];
    uint32_t n[kSide];
#pragma unroll
    for (int i = 0; i < kSide; ++i) n[i] = w.nb[i][K * kBlkCols];
    ss.r2[k] = tube_update(n, dn, up, own, sh.ends, ct, cd);
    ss.grew2 |= own == 0u ? ss.r2[k] : 0u;
    if (k == 3) {
        const int u4 = u - 3;
        store_quad_nt(yout, quad_of(sh, u4 >> 2, w.c), ss.r2[0], ss.r2[1], ss.r2[2], ss.r2[3]);
        if (u4 + 3 >= top_min) {
            const int kt = w.top - u4;
            ss.far2 |= kt == 0 ? ss.r2[0] : kt == 1 ? ss.r2[1] : kt == 2 ? ss.r2[2] : kt == 3 ? ss.r2[3] : 0u;
        }
        const int ka = front + 1 - u4, kb = front + 2 - u4;
        if (ka >= 0 && ka < 4) ss.ent2a |= ka == 0 ? ss.r2[0] : ka == 1 ? ss.r2[1] : ka == 2 ? ss.r2[2] : ss.r2[3];
        if (kb >= 0 && kb < 4) ss.ent2b |= kb == 0 ? ss.r2[0] : kb == 1 ? ss.r2[1] : kb == 2 ? ss.r2[2] : ss.r2[3];
    }
}

template <int NJ>
struct Walk2 {
    const StageN<NJ>* st;
    const Prod<NJ>* p;
    const Own* w;
    const float* ct;
    const float* yin;
    float* yout;
    const uint32_t* code4;
    float* far1;
    int front, vmax0, vmax1, top_min, last_q;
};

__device__ __forceinline__ int clamp_q(int g, int last_q) { return min(max(g, 0), last_q); }

// Group G of the first step (R0 slots 4P..4P+3, written to the same slots of R1) and,
// if `second`, group G-1 of the second step (R1 slots of the other parity). Three
// barriers: before the outer group G+1 replaces G-1 in R0 and before any first-step word
// of G replaces G-2 in R1 (second-step cells of G-2 may still read it until then: the
// words of the first cell are held back to after it); before the last first-step cell,
// which reads G+1 in R0 and replaces the last cell of G-2 in R1 (or its mirror), the
// only R1 word of G-2 the first second-step cell reads; before the second-step cells
// that read group G. The first three first-step cells write rows that no second-step
// cell between the first two barriers reads.
template <int P, int NJ>
__device__ __forceinline__ void half2(const DevShape& sh, const Walk2<NJ>& k2, int G, bool second, Step2State<NJ>& ss) {
    constexpr int K0 = 4 * P, Q0 = 4 * (P ^ 1);
    const int u = 4 * G;
    first_cell<K0>(sh, *k2.p, k2.ct, u, k2.vmax1, k2.front, k2.far1, ss);
    __syncthreads();
    store_first0<K0>(*k2.p, ss);
    put_quads<Q0>(*k2.st, G + 1, k2.vmax0, ss.next);
    load_quads(sh, *k2.st, k2.yin, G + 2, k2.vmax0, ss.next);
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        if (j >= k2.p->n) break;
        ss.cq1[P ^ 1][j] = k2.code4[code_word_g(sh, clamp_q(G + 1, k2.last_q), k2.p->c[j])];
    }
    ss.cq2[P] = k2.code4[code_word_g(sh, clamp_q(G, k2.last_q), k2.w->c)];
    first_cell<K0 + 1>(sh, *k2.p, k2.ct, u + 1, k2.vmax1, k2.front, k2.far1, ss);
    first_cell<K0 + 2>(sh, *k2.p, k2.ct, u + 2, k2.vmax1, k2.front, k2.far1, ss);
    if (second) second_cell<Q0>(sh, *k2.w, k2.ct, u - 4, k2.front, k2.top_min, k2.yout, ss);
    __syncthreads();
    first_cell<K0 + 3>(sh, *k2.p, k2.ct, u + 3, k2.vmax1, k2.front, k2.far1, ss);
    __syncthreads();
    if (second) {
        second_cell<Q0 + 1>(sh, *k2.w, k2.ct, u - 3, k2.front, k2.top_min, k2.yout, ss);
        second_cell<Q0 + 2>(sh, *k2.w, k2.ct, u - 2, k2.front, k2.top_min, k2.yout, ss);
        second_cell<Q0 + 3>(sh, *k2.w, k2.ct, u - 1, k2.front, k2.top_min, k2.yout, ss);
    }
}

// Two steps of the tile's tubes in cells [ub, ue) (cut at min(U, front+3); ub a multiple
// of 8): reads yin, writes the second step's words to yout and the first step's words of
// the far-end tubes to far1 (indexed by column; nullable). Returns the first step's flags
// and stores the second step's in *fl2. NJ: column slots per thread of the halo and
// outer ranges (1 when the workgroup has a thread per column of the whole tile).
template <int NJ>
__device__ __forceinline__ uint32_t walk_step2(const DevShape& sh, int k, const TileV& tv, const float* ct,
                                               const float* __restrict__ yin, float* __restrict__ yout,
                                               const uint8_t* __restrict__ code, float* __restrict__ far1, int ub,
                                               int ue, int front, int r1_off, uint32_t* fl2) {
    ue = min(ue, min(sh.U, front + 3));
    *fl2 = 0u;
    if (ub >= ue) return 0u;
    uint32_t* r0 = reinterpret_cast<uint32_t*>(lds);
    uint32_t* r1 = r0 + r1_off;
    const int os = uniform_i32(sh.tile2 + 2 * k), oe = uniform_i32(sh.tile2 + 2 * k + 1);
    const StageN<NJ> st = stage_range<NJ>(os, oe, r0);
    const Prod<NJ> p = prod_columns<NJ>(sh, k, tv, os, r0, r1);
    const Own w = own_column_in(sh, tv, r1);
    Walk2<NJ> k2;
    k2.st = &st;
    k2.p = &p;
    k2.w = &w;
    k2.ct = ct;
    k2.yin = yin;
    k2.yout = yout;
    k2.code4 = reinterpret_cast<const uint32_t*>(code);
    k2.far1 = far1;
    k2.front = front;
    k2.vmax0 = min(front, sh.U - 1);
    k2.vmax1 = min(front + 1, sh.U - 1);
    k2.top_min = (sh.L - 3) / 3;
    k2.last_q = (sh.U + 3) / 4 - 1;
    const int g0 = ub >> 2, gl = (ue - 1) >> 2;
    __syncthreads();  // the rings may still be read by a previous item
    zero_pad(r0);
    zero_pad(r1);
    Step2State<NJ> ss;
    uint4 q[NJ];
    load_quads(sh, st, yin, g0 - 2, k2.vmax0, q);
    put_quads<0>(st, g0 - 2, k2.vmax0, q);
    load_quads(sh, st, yin, g0 - 1, k2.vmax0, q);
    put_quads<4>(st, g0 - 1, k2.vmax0, q);
    load_quads(sh, st, yin, g0, k2.vmax0, ss.next);
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        if (j >= p.n) break;
        ss.cq1[1][j] = k2.code4[code_word_g(sh, clamp_q(g0 - 1, k2.last_q), p.c[j])];
    }
    __syncthreads();
    half2<1>(sh, k2, g0 - 1, false, ss);
    half2<0>(sh, k2, g0, false, ss);
    for (int G = g0 + 1; G <= gl + 1; G += 2) {
        half2<1>(sh, k2, G, true, ss);
        if (G + 1 > gl + 1) break;
        half2<0>(sh, k2, G + 1, true, ss);
    }
    *fl2 = (ss.grew2 ? F_GREW : 0u) | (ss.far2 ? F_FAR : 0u) | (ss.ent2a ? F_FRONT : 0u) | (ss.ent2b ? F_FRONT2 : 0u);
    return (ss.grew1 ? F_GREW : 0u) | (ss.far1 ? F_FAR : 0u) | (ss.ent1 ? F_FRONT : 0u);
}

// ------------------------------------------------------------------------------
// Initialisation walk: the ring holds the occupancy (0/1) of the staged tubes; each
// tube's degree code is its number of metallic contacts (detector edge included), 15
// if it is insulating or absent.
// ------------------------------------------------------------------------------

// Raw occupancy words holding the bits of the four cells of group g (clamped into the
// configuration; put_occ_quad masks what lies outside).
__device__ __forceinline__ void load_occ_quad(const DevShape& sh, const Stage& st, const int (&rk)[kLoadCols],
                                              const uint32_t* __restrict__ bits, int g, uint32_t (&out)[4][kLoadCols]) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int64_t vc = (int64_t)min(max(4 * g + k, 0), sh.U - 1) * sh.C;
#pragma unroll
        for (int j = 0; j < kLoadCols; ++j) {
            const int64_t s = vc + rk[j];
            out[k][j] = j < st.nj ? bits[(s < sh.N ? s : sh.N - 1) >> 5] : 0u;
        }
    }
}

template <int S0>
__device__ __forceinline__ void put_occ_quad(const DevShape& sh, const Stage& st, const int (&rk)[kLoadCols], int g,
                                             const uint32_t (&raw)[4][kLoadCols]) {
#pragma unroll
    for (int j = 0; j < kLoadCols; ++j) {
        if (j >= st.nj) break;
        if (!st.ok[j]) continue;
        uint32_t b[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int v = 4 * g + k;
            const int64_t s = (int64_t)v * sh.C + rk[j];
            b[k] = (v >= 0 && v < sh.U && s < sh.N) ? (raw[k][j] >> (uint32_t)(s & 31)) & 1u : 0u;
        }
        st.slot[j][(S0 + 1) * kBlkCols] = b[0];
        st.slot[j][(S0 + 2) * kBlkCols] = b[1];
        st.slot[j][(S0 + 3) * kBlkCols] = b[2];
        st.slot[j][(S0 + 4) * kBlkCols] = b[3];
        if (S0 == 0) st.slot[j][(kRingCells + 1) * kBlkCols] = b[0];
        if (S0 == 4) st.slot[j][0] = b[3];
    }
}

struct InitState {
    uint32_t next[4][kLoadCols];  // raw occupancy words of the group after the current one
    uint32_t cq = 0;              // codes of the current eight cells
    float y0 = 0.0f;
    uint32_t fl = 0;
};

template <int K>
__device__ __forceinline__ void init_cell(const DevShape& sh, const Stage& st, const Own& w,
                                          const int (&rk)[kLoadCols], const float* ct,
                                          const uint32_t* __restrict__ bits, uint32_t* __restrict__ code4,
                                          float* __restrict__ y0, int u8, int ue, float x0, InitState& is) {
    constexpr int k = K & 3, par = K >> 2;
    const int u = u8 + K, g = u >> 2;
    if (k & 1) __syncthreads();
    if (k == 1) {
        put_occ_quad<(par ^ 1) * 4>(sh, st, rk, g + 1, is.next);
        load_occ_quad(sh, st, rk, bits, g + 2, is.next);
    }
    const uint32_t me = w.me[(K + 1) * kBlkCols];
    // end contacts (same column, the cells below and above) unless the lattice is regular FCC
    uint32_t deg = (sh.ends ? w.me[K * kBlkCols] + w.me[(K + 2) * kBlkCols] : 0u) + (u == w.top ? 1u : 0u);
#pragma unroll
    for (int i = 0; i < kSide; ++i) deg += w.nb[i][K * kBlkCols];
    const uint32_t cd = me ? deg : 15u;
    is.cq |= cd << (4 * K);
    if (u == 0 && me) {
        is.y0 = x0 * ct[cd];
        is.fl |= F_NONEMPTY;
        if (u == w.top) is.fl |= F_FAR;
    }
    // one code word per eight cells; a walk ending after four cells ends the fiber, whose
    // cells beyond it are coded absent
    if (K == 7 || (K == 3 && u8 + 4 >= ue)) {
        code4[code_word_g(sh, g, w.c)] = K == 7 ? is.cq : (is.cq | 0xffff0000u);
        is.cq = 0;
    }
    if (k == 3) {
        if (g == 0)
            reinterpret_cast<uint4*>(y0)[quad_of(sh, 0, w.c)] = make_uint4(__float_as_uint(is.y0), 0u, 0u, 0u);
    }
}

// Degree codes of the tile's tubes in cells [ub, ue) (whole groups; ub a multiple of
// 8) from the occupancy, and the start state (group 0): x0 = 1/|S0| on every metallic
// start tube, reached. Returns the initialisation flags (start set non-empty, a start
// tube on the far surface).
// LEAD: the three leading groups of occupancy are loaded together (the span form's
// initialisation launch gains from it; the persistent form keeps its registers).
template <bool LEAD = false>
__device__ __forceinline__ uint32_t walk_init(const DevShape& sh, const TileV& tv, const float* ct,
                                              const uint32_t* __restrict__ bits, uint8_t* __restrict__ code,
                                              float* __restrict__ y0, int ub, int ue, float x0) {
    ue = min(ue, sh.U);
    if (ub >= ue) return 0u;
    uint32_t* code4 = reinterpret_cast<uint32_t*>(code);
    const Stage st = stage_columns(tv);
    int rk[kLoadCols];
#pragma unroll
    for (int j = 0; j < kLoadCols; ++j) rk[j] = sh.rank[st.col[j]];
    const Own w = own_column(sh, tv);
    const int g0 = ub >> 2;
    __syncthreads();
    zero_pad();
    InitState is;
    // (group g0 - 1 below the fiber: masked to zero, not loaded)
    uint32_t raw[4][kLoadCols] = {};
    if (LEAD) {
        uint32_t raw0[4][kLoadCols];
        if (g0 > 0) load_occ_quad(sh, st, rk, bits, g0 - 1, raw);
        load_occ_quad(sh, st, rk, bits, g0, raw0);
        load_occ_quad(sh, st, rk, bits, g0 + 1, is.next);
        put_occ_quad<4>(sh, st, rk, g0 - 1, raw);
        put_occ_quad<0>(sh, st, rk, g0, raw0);
    } else {
        if (g0 > 0) load_occ_quad(sh, st, rk, bits, g0 - 1, raw);
        put_occ_quad<4>(sh, st, rk, g0 - 1, raw);
        load_occ_quad(sh, st, rk, bits, g0, raw);
        put_occ_quad<0>(sh, st, rk, g0, raw);
        load_occ_quad(sh, st, rk, bits, g0 + 1, is.next);
    }
    __syncthreads();
    for (int u8 = ub; u8 < ue; u8 += kRingCells) {
        init_cell<0>(sh, st, w, rk, ct, bits, code4, y0, u8, ue, x0, is);
        init_cell<1>(sh, st, w, rk, ct, bits, code4, y0, u8, ue, x0, is);
        init_cell<2>(sh, st, w, rk, ct, bits, code4, y0, u8, ue, x0, is);
        init_cell<3>(sh, st, w, rk, ct, bits, code4, y0, u8, ue, x0, is);
        if (u8 + 4 >= ue) break;
        init_cell<4>(sh, st, w, rk, ct, bits, code4, y0, u8, ue, x0, is);
        init_cell<5>(sh, st, w, rk, ct, bits, code4, y0, u8, ue, x0, is);
        init_cell<6>(sh, st, w, rk, ct, bits, code4, y0, u8, ue, x0, is);
        init_cell<7>(sh, st, w, rk, ct, bits, code4, y0, u8, ue, x0, is);
    }
    return is.fl;
}

// Number of metallic start tubes (every tube of cell 0) of one configuration.
__device__ __forceinline__ int count_start(const DevShape& sh, const uint32_t* __restrict__ bits, uint32_t* red) {
    const int64_t n0 = min((int64_t)sh.C, sh.N);
    int cnt = 0;
    for (int64_t w = threadIdx.x; w * 32 < n0; w += blockDim.x) {
        uint32_t b = bits[w];
        const int64_t rem = n0 - w * 32;
        if (rem < 32) b &= (1u << rem) - 1u;
        cnt += __popc(b);
    }
    __syncthreads();
    if (threadIdx.x == 0) *red = 0;
    __syncthreads();
    if (cnt) atomicAdd(red, (uint32_t)cnt);
    __syncthreads();
    const int total = (int)*red;
    __syncthreads();
    return total;
}

// Sum over the far-end tubes of |y| (the mass the detector receives next step) and
// whether any of them is reached. Cells beyond `front` hold no mass and are not read
// (their words may be stale). Fixed order independent of blockDim: 256 virtual lanes
// each add their columns in increasing order, then a fixed pairwise tree.
__device__ __forceinline__ void far_sum(const DevShape& sh, const float* __restrict__ y, int front, float* part,
                                        uint32_t* reached, float* result) {
    __syncthreads();
    if (threadIdx.x == 0) *reached = 0;
    __syncthreads();
    for (int v = threadIdx.x; v < 256; v += blockDim.x) {
        float s = 0.0f;
        uint32_t r = 0;
        for (int c = v; c < sh.C; c += 256) {
            const int u = top_of(sh, c);
            if (u < 0 || u > front) continue;
            const uint32_t w = __float_as_uint(y[word_of(sh, u, c)]);
            s += mag(w);
            r |= w != 0u ? 1u : 0u;
        }
        part[v] = s;
        if (r) atomicOr(reached, 1u);
    }
    __syncthreads();
    for (int width = 128; width >= 1; width >>= 1) {
        for (int v = threadIdx.x; v < width; v += blockDim.x) part[v] = part[v] + part[v + width];
        __syncthreads();
    }
    if (threadIdx.x == 0) *result = part[0];
    __syncthreads();
}

// far_sum over words given per column (the far-end word of column c at w[c]), in the same
// order as far_sum, so the result has the same bits as far_sum over a state holding them.
__device__ __forceinline__ void far_sum_cols(const DevShape& sh, const float* __restrict__ wc, int front, float* part,
                                             uint32_t* reached, float* result) {
    __syncthreads();
    if (threadIdx.x == 0) *reached = 0;
    __syncthreads();
    for (int v = threadIdx.x; v < 256; v += blockDim.x) {
        float s = 0.0f;
        uint32_t r = 0;
        for (int c = v; c < sh.C; c += 256) {
            const int u = top_of(sh, c);
            if (u < 0 || u > front) continue;
            const uint32_t w = __float_as_uint(wc[c]);
            s += mag(w);
            r |= w != 0u ? 1u : 0u;
        }
        part[v] = s;
        if (r) atomicOr(reached, 1u);
    }
    __syncthreads();
    for (int width = 128; width >= 1; width >>= 1) {
        for (int v = threadIdx.x; v < width; v += blockDim.x) part[v] = part[v] + part[v + width];
        __syncthreads();
    }
    if (threadIdx.x == 0) *result = part[0];
    __syncthreads();
}

// Items [0, total) of a launch (tile index fastest): the workgroups of one XCD share one
// contiguous range and deal it round-robin, so the workgroups that run side by side on
// an XCD walk the neighbouring tiles of one cell range at the same time and read each
// other's halo columns from that XCD's L2.
struct ItemRange {
    int64_t begin, end, stride;
};
__device__ __forceinline__ ItemRange my_items(int64_t total) {
    const int G = gridDim.x;
    if (G % kXcds != 0) {
        const int64_t b = total * blockIdx.x / G, e = total * (blockIdx.x + 1) / G;
        return ItemRange{b, e, 1};
    }
    const int x = blockIdx.x % kXcds, lb = blockIdx.x / kXcds, per = G / kXcds;
    const int64_t xb = total * x / kXcds, xe = total * (x + 1) / kXcds;
    return ItemRange{xb + lb, xe, per};
}

__device__ __forceinline__ int items_of(const DevShape& sh, int ncells, int E) {
    return ((ncells + E - 1) / E) * sh.ntile;
}

__device__ __forceinline__ int find_entry(const int64_t* off, int n, int64_t g) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (uniform_i64(off + mid) <= g) lo = mid; else hi = mid - 1;
    }
    return __builtin_amdgcn_readfirstlane(lo);
}

// The entry i >= lo with off[i] <= g < off[i + 1] (off non-decreasing, off[n] > g): 64
// boundaries per probe, one load per lane and a ballot, so jumping over many short
// entries costs one or two loads instead of one dependent load per entry. Every wave
// computes the same (uniform) result.
__device__ __forceinline__ int advance_entry(const int64_t* off, int n, int lo, int64_t g) {
    const int lane = threadIdx.x & 63;
    for (;;) {
        const int idx = min(lo + 1 + lane, n);
        const unsigned long long m = __ballot(off[idx] <= g);
        const int c = __popcll(m);
        lo += c;
        if (c < 64) return __builtin_amdgcn_readfirstlane(lo);
    }
}

// OR of a flag word over the workgroup, added to *dst: one atomic per wave that has a
// flag (no barrier).
__device__ __forceinline__ void flags_to(uint32_t* dst, uint32_t fl) {
    uint32_t w = 0;
    if (__ballot(fl & F_GREW)) w |= F_GREW;
    if (__ballot(fl & F_FRONT)) w |= F_FRONT;
    if (__ballot(fl & F_FAR)) w |= F_FAR;
    if (__ballot(fl & F_NONEMPTY)) w |= F_NONEMPTY;
    if (__ballot(fl & F_STEPPED)) w |= F_STEPPED;
    if (__ballot(fl & F_FUSED)) w |= F_FUSED;
    if (__ballot(fl & F_FRONT2)) w |= F_FRONT2;
    if (w && (threadIdx.x & 63) == 0) atomicOr(dst, w);
}

// ------------------------------------------------------------------------------
// Kernels
// ------------------------------------------------------------------------------

__global__ void __launch_bounds__(256) k_sample(uint32_t* __restrict__ bits, int64_t words, int64_t N,
                                                int64_t n_cfg, uint64_t cfg0, uint64_t thr, uint32_t k0,
                                                uint32_t k1, uint32_t tag) {
    const int64_t total = n_cfg * words;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t cfg = i / words, w = i - cfg * words;
        bits[i] = sample_word(w, N, cfg0 + (uint64_t)cfg, thr, k0, k1, tag);
    }
}

// Fixed-count ensemble (Sec. II.A: Np of the N tubes metallic, chosen uniformly): the K
// tubes with the smallest 64-bit keys, ties by tube index. Tube s takes words 2(s&1)
// (high) and 2(s&1)+1 (low) of the Philox block with counter (s >> 1, cfg lo, cfg hi,
// tag | 2^31), a counter space apart from the Bernoulli draws. One workgroup per
// configuration: a most-significant-digit radix select (six digits of 11 bits, LDS
// histograms, keys regenerated every pass) finds the key T of rank K-1 and how many keys
// equal to T are taken; a last pass writes the bits, taking equal keys in tube order.
__device__ __forceinline__ uint64_t fixed_key(int64_t s, uint64_t cfg, uint32_t k0, uint32_t k1, uint32_t tag) {
    const Ctr4 r = philox4x32_10(Ctr4{(uint32_t)(s >> 1), (uint32_t)cfg, (uint32_t)(cfg >> 32), tag | 0x80000000u},
                                 k0, k1);
    return (s & 1) ? (((uint64_t)r.v2 << 32) | r.v3) : (((uint64_t)r.v0 << 32) | r.v1);
}

constexpr int kSelBits = 11;
constexpr int kSelBins = 1 << kSelBits;

__global__ void __launch_bounds__(1024) k_sample_fixed(uint32_t* __restrict__ bits, int64_t words, int64_t N,
                                                       int64_t K, int64_t n_cfg, uint64_t cfg0, uint32_t k0,
                                                       uint32_t k1, uint32_t tag) {
    __shared__ uint32_t hist[kSelBins];
    __shared__ uint32_t scan[1024];
    __shared__ uint64_t sel_prefix;
    __shared__ int64_t sel_rank;
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int64_t c = blockIdx.x; c < n_cfg; c += gridDim.x) {
        const uint64_t cfg = cfg0 + (uint64_t)c;
        uint32_t* out = bits + c * words;
        if (K <= 0 || K >= N) {  // none or every tube
            for (int64_t w = tid; w < words; w += nt) {
                const int64_t rem = N - w * 32;
                out[w] = K <= 0 ? 0u : (rem >= 32 ? 0xffffffffu : ((1u << rem) - 1u));
            }
            continue;
        }
        uint64_t prefix = 0, mask = 0;
        int64_t rank = K - 1;  // rank of the target among the keys that match the prefix
        for (int shift = 64 - kSelBits; shift > -kSelBits; shift -= kSelBits) {
            const int sh = shift < 0 ? 0 : shift;
            const int width = shift < 0 ? kSelBits + shift : kSelBits;
            const uint64_t dmask = ((uint64_t)1 << width) - 1;
            for (int b = tid; b < kSelBins; b += nt) hist[b] = 0;
            __syncthreads();
            for (int64_t s = tid; s < N; s += nt) {
                const uint64_t key = fixed_key(s, cfg, k0, k1, tag);
                if ((key & mask) == prefix) atomicAdd(&hist[(key >> sh) & dmask], 1u);
            }
            __syncthreads();
            // find the digit whose cumulative count passes rank (thread 0; 2048 bins)
            if (tid == 0) {
                int64_t below = 0;
                uint32_t b = 0;
                for (; b < (uint32_t)(1u << width); ++b) {
                    if (below + hist[b] > rank) break;
                    below += hist[b];
                }
                sel_prefix = prefix | ((uint64_t)b << sh);
                sel_rank = rank - below;
            }
            __syncthreads();
            prefix = sel_prefix;
            rank = sel_rank;
            mask |= dmask << sh;
            __syncthreads();
        }
        // prefix = T, the key of rank K-1; rank + 1 keys equal to T are taken (by index)
        const uint64_t T = prefix;
        const int64_t need_eq = rank + 1;
        const int64_t wpt = (words + nt - 1) / nt;  // contiguous words per thread
        const int64_t w0 = min((int64_t)tid * wpt, words), w1 = min(w0 + wpt, words);
        uint32_t eq = 0;
        for (int64_t w = w0; w < w1; ++w)
            for (int i = 0; i < 32; ++i) {
                const int64_t s = w * 32 + i;
                if (s < N && fixed_key(s, cfg, k0, k1, tag) == T) ++eq;
            }
        scan[tid] = eq;
        __syncthreads();
        for (int off = 1; off < nt; off <<= 1) {
            const uint32_t v = tid >= off ? scan[tid - off] : 0u;
            __syncthreads();
            scan[tid] += v;
            __syncthreads();
        }
        int64_t eq_before = (int64_t)scan[tid] - eq;
        for (int64_t w = w0; w < w1; ++w) {
            uint32_t word = 0;
            for (int i = 0; i < 32; ++i) {
                const int64_t s = w * 32 + i;
                if (s >= N) break;
                const uint64_t key = fixed_key(s, cfg, k0, k1, tag);
                if (key < T || (key == T && eq_before++ < need_eq)) word |= 1u << i;
            }
            out[w] = word;
        }
        __syncthreads();
    }
}

// Occupancy of the slots whose job samples from Philox, one workgroup per slot, into
// the slot's bits buffer.
__global__ void __launch_bounds__(256) k_sample_slots(const DevShape* shapes, const Job* jobs, int32_t n_slot,
                                                      uint32_t* const* slot_bits) {
    for (int b = blockIdx.x; b < n_slot; b += gridDim.x) {
        const Job job = jobs[b];
        if (job.bits) continue;
        const DevShape sh = shapes[job.shape];
        uint32_t* dst = slot_bits[b];
        const uint32_t k0 = (uint32_t)job.seed, k1 = (uint32_t)(job.seed >> 32);
        for (int64_t w = threadIdx.x; w < sh.words; w += blockDim.x)
            dst[w] = sample_word(w, sh.N, job.cfg, job.thr, k0, k1, shape_tag(sh));
    }
}

// Occupancy of the listed jobs, one workgroup per job, into the buffer each job's bits
// pointer names (the persistent form draws every configuration before it starts).
__global__ void __launch_bounds__(256) k_sample_jobs(const DevShape* shapes, const Job* jobs, const int64_t* idx,
                                                     int64_t n) {
    for (int64_t i = blockIdx.x; i < n; i += gridDim.x) {
        const Job job = jobs[idx[i]];
        const DevShape sh = shapes[job.shape];
        uint32_t* dst = const_cast<uint32_t*>(job.bits);
        const uint32_t k0 = (uint32_t)job.seed, k1 = (uint32_t)(job.seed >> 32);
        for (int64_t w = threadIdx.x; w < sh.words; w += blockDim.x)
            dst[w] = sample_word(w, sh.N, job.cfg, job.thr, k0, k1, shape_tag(sh));
    }
}

// Item layout of the initialisation (all cells of every slot) and the slot states.
// Slots to initialise: the listed ones (a.ids), else all.
__device__ __forceinline__ int init_count(const SpanArgs& a) { return a.ids ? a.n_ids : a.n_slot; }
// Lazy initialisation: the cells an extension adds (whole items, more than the margin),
// and the cells initialised at first (all of them without lazy initialisation).
__device__ __forceinline__ int ext_cells(const SpanArgs& a) {
    return ((a.init_margin + a.depth) / a.depth) * a.depth;
}
__device__ __forceinline__ int init_horizon(const SpanArgs& a, int U) { return a.lazy ? min(U, ext_cells(a)) : U; }
__device__ __forceinline__ int init_slot(const SpanArgs& a, int i) { return a.ids ? a.ids[i] : i; }

__global__ void __launch_bounds__(kMaxBlock) k_span_layout(SpanArgs a) {
    __shared__ int64_t sums[kMaxBlock];
    const int tid = threadIdx.x, nt = blockDim.x;
    const int n = init_count(a);
    const int per = (n + nt - 1) / nt;
    const int i0 = min(n, tid * per), i1 = min(n, i0 + per);
    int64_t mine = 0;
    for (int i = i0; i < i1; ++i) {
        const int b = init_slot(a, i);
        const DevShape& sh = a.shapes[a.slot_shape[b]];
        const int hz = init_horizon(a, sh.U);
        mine += items_of(sh, hz, a.depth);
        a.st[b] = CfgState{0, -1, 0, 0u, 0u, 0, hz, -1, 0};  // m = -1: initialised, not yet decided
    }
    sums[tid] = mine;
    __syncthreads();
    for (int off = 1; off < nt; off <<= 1) {
        const int64_t v = tid >= off ? sums[tid - off] : 0;
        __syncthreads();
        sums[tid] += v;
        __syncthreads();
    }
    int64_t pos = sums[tid] - mine;
    for (int i = i0; i < i1; ++i) {
        a.chunk_off[i] = pos;
        const DevShape& sh = a.shapes[a.slot_shape[init_slot(a, i)]];
        pos += items_of(sh, init_horizon(a, sh.U), a.depth);
    }
    if (tid == nt - 1) a.chunk_off[n] = sums[nt - 1];
}

// Initialisation of every slot: items (slot, cell range, tile) over all cells.
__global__ void __launch_bounds__(kMaxBlock) k_span_init(SpanArgs a) {
    const Tail tl = lds_tail(a.lds);
    fill_codes(tl.ct);
    const int E = a.depth;
    const int n = init_count(a);
    const ItemRange it = my_items(uniform_i64(a.chunk_off + n));
    int i = it.begin < it.end ? find_entry(a.chunk_off, n, it.begin) : 0;
    for (int64_t g = it.begin; g < it.end; g += it.stride) {
        i = advance_entry(a.chunk_off, n, i, g);
        const int b = a.ids ? uniform_i32(a.ids + i) : i;
        const DevShape sh = uniform_load(a.shapes + uniform_i32(a.slot_shape + b));
        const int local = (int)(g - uniform_i64(a.chunk_off + i));
        const int r = local / sh.ntile, k = local - r * sh.ntile;
        const int ub = r * E;
        const uint32_t* bits = reinterpret_cast<const uint32_t*>(uniform_i64(reinterpret_cast<const int64_t*>(a.slot_bits + b)));
        float x0 = 0.0f;
        if (ub == 0) {
            const int n0 = count_start(sh, bits, tl.misc + 1);
            x0 = n0 > 0 ? 1.0f / (float)n0 : 0.0f;
        }
        const int64_t off = uniform_i64(a.slot_off + b);
        const uint32_t fl = walk_init<true>(sh, load_tile(sh, k), tl.ct, bits, a.code + off, a.ya + off, ub, ub + E, x0);
        if (ub == 0) flags_to(&a.st[b].flags, fl);
    }
}

// Lazy initialisation: the degree codes of the ranges [hz_from, hz) of the slots the last
// plan listed (items: listed slot, cell range, tile). Counts its launches in hdr[7], which
// tells the planner that the ranges listed before it are done.
__global__ void __launch_bounds__(kMaxBlock) k_span_extend(SpanArgs a) {
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(a.hdr + 7, 1);
    const int n = uniform_i32(a.hdr + 6);
    if (n == 0) return;
    const Tail tl = lds_tail(a.lds);
    fill_codes(tl.ct);
    const int E = a.depth;
    const ItemRange it = my_items(uniform_i64(a.ext_off + n));
    int i = it.begin < it.end ? find_entry(a.ext_off, n, it.begin) : 0;
    for (int64_t g = it.begin; g < it.end; g += it.stride) {
        i = advance_entry(a.ext_off, n, i, g);
        const int b = uniform_i32(a.ext_ids + i);
        const DevShape sh = uniform_load(a.shapes + uniform_i32(a.slot_shape + b));
        const int base = uniform_i32(&a.st[b].hz_from);
        const int local = (int)(g - uniform_i64(a.ext_off + i));
        const int r = local / sh.ntile, k = local - r * sh.ntile;
        const int ub = base + r * E;  // > 0: the start state is not touched
        const uint32_t* bits = reinterpret_cast<const uint32_t*>(uniform_i64(reinterpret_cast<const int64_t*>(a.slot_bits + b)));
        const int64_t off = uniform_i64(a.slot_off + b);
        (void)walk_init<true>(sh, load_tile(sh, k), tl.ct, bits, a.code + off, a.ya + off, ub, ub + E, 0.0f);
    }
}

// Inclusive scan of one value per thread over the workgroup (blockDim a multiple of 64):
// shuffles inside each wave, then the wave totals through `tot` (one slot per wave, LDS);
// *all receives the sum over the workgroup. One barrier; `tot` may be reused only after
// another barrier.
template <typename T>
__device__ __forceinline__ T block_scan(T v, T* tot, T* all) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const T t = __shfl_up(v, off, 64);
        if (lane >= off) v += t;
    }
    if (lane == 63) tot[wid] = v;
    __syncthreads();
    T base = 0, sum = 0;
    for (int w = 0; w < nw; ++w) {
        const T x = tot[w];
        base += w < wid ? x : (T)0;
        sum += x;
    }
    *all = sum;
    return v + base;
}

// Decide every listed configuration (all slots if first, else the active list) from
// its flags, write the outputs of those that stopped (and list them in a.fin), and lay
// out the items of the next step for the rest. A slot just initialised (m = -1) gets
// the initial decision; a slot the last step launch touched (F_STEPPED) the step
// decision; any other keeps its state (it is only laid out again). One workgroup of
// kMaxBlock threads.
__global__ void __launch_bounds__(kMaxBlock) k_span_plan(SpanArgs a, int first) {
    __shared__ int32_t keep_s[kMaxBlock / 64];
    __shared__ int64_t chunk_s[kMaxBlock / 64];
    __shared__ int64_t chunk2_s[kMaxBlock / 64];
    __shared__ int32_t ext_s[kMaxBlock / 64];
    __shared__ int64_t exti_s[kMaxBlock / 64];
    const int tid = threadIdx.x, nt = blockDim.x;
    const int gen = a.lazy ? a.hdr[7] : 0;  // extension launches done so far
    const int n_act = first ? a.n_slot : a.hdr[0];
    const int per = (n_act + nt - 1) / nt;
    const int i0 = min(n_act, tid * per), i1 = min(n_act, i0 + per);
    const int E = a.depth;
    int32_t keep = 0, ext = 0;
    int64_t chunks = 0, ext_items = 0;
    for (int i = i0; i < i1; ++i) {
        const int b = first ? i : a.active[i];
        const DevShape& sh = a.shapes[a.slot_shape[b]];
        CfgState s = a.st[b];
        const uint32_t f = s.flags, f2 = s.flags2;
        s.flags = 0;
        s.flags2 = 0;
        if (s.done) {  // cancelled by the host: leaves the work list without a decision
            a.st[b] = s;
            continue;
        }
        int dec = -1;  // -1 continue, 0 no, 1 yes
        int32_t steps = 0;
        if (s.m < 0) {
            s.m = 0;
            if (!(f & F_NONEMPTY)) { dec = 0; steps = 0; }
            else if (f & F_FAR) { dec = 1; steps = 1; }
        } else if (f & F_STEPPED) {
            // a step launch writes the other buffer; a pair of launches writes both, the
            // newest state back in the buffer the pair started from
            if (!a.pair) s.par ^= 1;
            s.m += 1;
            if (f & F_FRONT) s.front += 1;
            if (f & F_FAR) { dec = 1; steps = s.m + 1; if (f & F_FUSED) s.done = a.pair ? 4 : 3; }
            else if (!(f & F_GREW)) { dec = 0; steps = s.m; }
            else if (f & F_FUSED) {
                // the second step of a two-step launch, decided as a step of its own; its
                // front flags are relative to the front before the first step
                s.m += 1;
                if ((f & F_FRONT) ? (f2 & F_FRONT2) : (f2 & F_FRONT)) s.front += 1;
                if (f2 & F_FAR) { dec = 1; steps = s.m + 1; }
                else if (!(f2 & F_GREW)) { dec = 0; steps = s.m; }
                else if (s.m > sh.N) { dec = 0; steps = s.m; s.done = 2; a.hdr[2] = 1; }
            }
            else if (s.m > sh.N) { dec = 0; steps = s.m; s.done = 2; a.hdr[2] = 1; }
        }
        if (dec >= 0) {
            if (s.done == 0) s.done = 1;
            a.out.perc[b] = (uint8_t)dec;
            a.out.steps[b] = steps;
            if (a.fin) a.fin[atomicAdd(a.hdr + 3, 1)] = b;
        } else {
            keep += 1;
            chunks += items_of(sh, min(sh.U, s.front + (a.fused || a.pair ? 3 : 2)), E);
            if (a.lazy) {
                if (s.hz_from >= 0 && gen > s.ext_gen) s.hz_from = -1;  // its range is computed
                if (s.hz_from < 0 && s.hz < sh.U && s.front + a.init_margin >= s.hz) {
                    s.hz_from = s.hz;
                    s.hz = min(sh.U, s.hz + ext_cells(a));
                    s.ext_gen = gen;
                }
                if (s.hz_from >= 0) {
                    ext += 1;
                    ext_items += items_of(sh, s.hz - s.hz_from, E);
                }
            }
        }
        a.st[b] = s;
    }
    int32_t n_keep;
    int64_t n_chunks;
    int32_t kpos = block_scan(keep, keep_s, &n_keep) - keep;
    int64_t cpos = block_scan(chunks, chunk_s, &n_chunks) - chunks;
    int32_t n_ext = 0;
    int64_t n_ext_items = 0;
    int32_t epos = 0;
    int64_t eoff = 0;
    const bool lst = a.lazy && a.list_ext;  // only the plan before an extension launch lists
    if (lst) {
        epos = block_scan(ext, ext_s, &n_ext) - ext;
        eoff = block_scan(ext_items, exti_s, &n_ext_items) - ext_items;
    }
    // A work list shorter than what the device runs at once (the last, slowest
    // configurations of a batch): items of a half, a quarter or an eighth of the depth
    // (whole octets of cells), as long as the list stays within that size, so that the
    // walks spread over more workgroups. Results do not depend on the item depth.
    int Eu = E;
    if (!a.fused && a.resident > 0 && n_chunks > 0) {
        int f = 1;
        while (f < 8 && E / (2 * f) >= 8 && n_chunks * (2 * f) <= (int64_t)a.resident) f *= 2;
        if (f > 1) {
            Eu = (E / f) & ~7;
            chunks = 0;
            for (int i = i0; i < i1; ++i) {
                const int b = first ? i : a.active[i];
                const CfgState s = a.st[b];
                if (s.done) continue;
                const DevShape& sh = a.shapes[a.slot_shape[b]];
                chunks += items_of(sh, min(sh.U, s.front + (a.pair ? 3 : 2)), Eu);
            }
            cpos = block_scan(chunks, chunk2_s, &n_chunks) - chunks;
        }
    }
    unsigned long long tubes = 0;
    for (int i = i0; i < i1; ++i) {
        const int b = first ? i : a.active[i];
        const CfgState s = a.st[b];
        if (s.done) continue;
        const DevShape& sh = a.shapes[a.slot_shape[b]];
        a.active2[kpos] = b;
        a.chunk_off[kpos] = cpos;
        kpos += 1;
        cpos += items_of(sh, min(sh.U, s.front + (a.fused || a.pair ? 3 : 2)), Eu);
        // tube slots advanced by one step each; two steps per plan count the window twice
        tubes += (unsigned long long)min(sh.U, s.front + 2) * (unsigned long long)sh.C * (a.fused || a.pair ? 2ull : 1ull);
        if (lst && s.hz_from >= 0) {  // listed for the next extension launch
            a.ext_ids[epos] = b;
            a.ext_off[epos] = eoff;
            epos += 1;
            eoff += items_of(sh, s.hz - s.hz_from, E);
        }
    }
    if (a.work && tubes) atomicAdd(a.work, tubes);
    __syncthreads();
    for (int i = tid; i < n_keep; i += nt) a.active[i] = a.active2[i];
    if (tid == 0) {
        a.chunk_off[n_keep] = n_chunks;
        a.hdr[0] = n_keep;
        a.hdr[1] = (int32_t)min(n_chunks, (int64_t)INT32_MAX);
        a.hdr[5] = Eu;
        if (lst) {
            a.hdr[6] = n_ext;
            a.ext_off[n_ext] = n_ext_items;
        }
    }
}

// One step over the work list: items (active slot, cell range, tile).
__global__ void __launch_bounds__(kMaxBlock) k_span_step(SpanArgs a) {
    const Tail tl = lds_tail(a.lds);
    fill_codes(tl.ct);
    const int n_act = uniform_i32(a.hdr);
    const int E = uniform_i32(a.hdr + 5);  // the planned cells per item
    const ItemRange it = my_items(uniform_i32(a.hdr + 1));
    if (it.begin >= it.end) return;
    int lo = find_entry(a.chunk_off, n_act, it.begin);
    int64_t lo_begin = uniform_i64(a.chunk_off + lo);
    int64_t lo_end = uniform_i64(a.chunk_off + lo + 1);
    for (int64_t g = it.begin; g < it.end; g += it.stride) {
        if (g >= lo_end) {  // a later active slot
            lo = advance_entry(a.chunk_off, n_act, lo, g);
            lo_begin = uniform_i64(a.chunk_off + lo);
            lo_end = uniform_i64(a.chunk_off + lo + 1);
        }
        const int b = uniform_i32(a.active + lo);
        const DevShape sh = uniform_load(a.shapes + uniform_i32(a.slot_shape + b));
        const int local = (int)(g - lo_begin);
        const int r = local / sh.ntile, k = local - r * sh.ntile;
        const CfgState s = uniform_load(a.st + b);
        const int64_t off = uniform_i64(a.slot_off + b);
        // the second launch of a pair reads the first one's output and writes the buffer
        // the pair started from; its input reaches one cell further
        const int par = s.par ^ a.sub;
        const float* yin = (par ? a.yb : a.ya) + off;
        float* yout = (par ? a.ya : a.yb) + off;
        const uint32_t fl = walk_step(sh, load_tile(sh, k), tl.ct, yin, yout, a.code + off, r * E, r * E + E,
                                      s.front + a.sub, s.front);
        if (a.sub) {
            flags_to(&a.st[b].flags, threadIdx.x < 64 ? F_FUSED : 0u);
            flags_to(&a.st[b].flags2, fl);
        } else {
            flags_to(&a.st[b].flags, (fl & ~F_FRONT2) | (threadIdx.x < 64 ? F_STEPPED : 0u));
        }
    }
}

// Two steps over the work list (two-step form): items (active slot, cell range, tile).
__global__ void __launch_bounds__(kMaxBlock) k_span_step2(SpanArgs a) {
    const Tail tl = lds_tail(a.lds);
    fill_codes(tl.ct);
    const int n_act = uniform_i32(a.hdr);
    const int E = a.depth;
    const ItemRange it = my_items(uniform_i32(a.hdr + 1));
    if (it.begin >= it.end) return;
    int lo = find_entry(a.chunk_off, n_act, it.begin);
    int64_t lo_begin = uniform_i64(a.chunk_off + lo);
    int64_t lo_end = uniform_i64(a.chunk_off + lo + 1);
    for (int64_t g = it.begin; g < it.end; g += it.stride) {
        if (g >= lo_end) {
            lo = advance_entry(a.chunk_off, n_act, lo, g);
            lo_begin = uniform_i64(a.chunk_off + lo);
            lo_end = uniform_i64(a.chunk_off + lo + 1);
        }
        const int b = uniform_i32(a.active + lo);
        const DevShape sh = uniform_load(a.shapes + uniform_i32(a.slot_shape + b));
        const int local = (int)(g - lo_begin);
        const int r = local / sh.ntile, k = local - r * sh.ntile;
        const CfgState s = uniform_load(a.st + b);
        const int64_t off = uniform_i64(a.slot_off + b);
        const float* yin = (s.par ? a.yb : a.ya) + off;
        float* yout = (s.par ? a.ya : a.yb) + off;
        uint32_t fl2 = 0;
        const uint32_t fl = walk_step2<kLoadCols>(sh, k, load_tile(sh, k), tl.ct, yin, yout, a.code + off,
                                       a.far1 + (int64_t)b * a.far1_stride, r * E, r * E + E, s.front, a.r1_off, &fl2);
        flags_to(&a.st[b].flags, fl | (threadIdx.x < 64 ? (F_STEPPED | F_FUSED) : 0u));
        flags_to(&a.st[b].flags2, fl2);
    }
}

// One step of n_cfg configurations of one shape over all cells (state, codes of
// configuration i at i * stride words / bytes): items (configuration, cell range, tile),
// dealt as in the span form, each walked with the same device code as the batches;
// every cell is processed (the state buffers are zero where nothing was written).
__global__ void __launch_bounds__(kMaxBlock) k_chunk_step(DevShape sh, const float* yin, float* yout,
                                                          const uint8_t* code, int64_t stride, int n_cfg, int E,
                                                          int lds_bytes) {
    const Tail tl = lds_tail(lds_bytes);
    fill_codes(tl.ct);
    const int per_cfg = ((sh.U + E - 1) / E) * sh.ntile;
    const ItemRange it = my_items((int64_t)per_cfg * n_cfg);
    for (int64_t g = it.begin; g < it.end; g += it.stride) {
        const int i = (int)(g / per_cfg), local = (int)(g - (int64_t)i * per_cfg);
        const int r = local / sh.ntile, k = local - r * sh.ntile;
        const int64_t off = (int64_t)i * stride;
        (void)walk_step(sh, load_tile(sh, k), tl.ct, yin + off, yout + off, code + off, r * E, r * E + E, sh.U,
                        sh.U);
    }
}

// Per slot: first-hit probability of a percolating configuration (the detector mass at
// the stop is the far-end sum of the state after steps-1 steps) and the group counts.
__global__ void __launch_bounds__(256) k_span_finish(SpanArgs a) {
    __shared__ float part[256];
    __shared__ uint32_t reached;
    __shared__ float result;
    const int n = a.fin ? a.hdr[3] : a.n_slot;
    for (int i = blockIdx.x; i < n; i += gridDim.x) {
        const int b = a.fin ? a.fin[i] : i;
        const int pc = a.out.perc[b];
        if (threadIdx.x == 0 && a.out.group_count && a.out.group && pc) {
            const int grp = a.out.group[b];
            if (grp >= 0) atomicAdd(&a.out.group_count[grp], 1ull);
        }
        if (!a.out.hit) continue;
        if (!pc) {
            if (threadIdx.x == 0) a.out.hit[b] = 0.0f;
            continue;
        }
        const DevShape sh = a.shapes[a.slot_shape[b]];
        const CfgState st = a.st[b];
        if (st.done == 3)  // after the first step of a two-step launch: its far-end words
            far_sum_cols(sh, a.far1 + (int64_t)b * a.far1_stride, st.front, part, &reached, &result);
        else if (st.done == 4)  // after the first launch of a pair: the other buffer
            far_sum(sh, (st.par ? a.ya : a.yb) + a.slot_off[b], st.front, part, &reached, &result);
        else  // the state after steps - 1 steps, the newest one
            far_sum(sh, (st.par ? a.yb : a.ya) + a.slot_off[b], st.front, part, &reached, &result);
        if (threadIdx.x == 0) a.out.hit[b] = result;
        __syncthreads();
    }
}

// The persistent form: each workgroup pulls configurations from a device queue and runs
// the whole inspection of each (codes and start state, every step, the outputs) on its
// own state buffers; Philox occupancy is drawn for all configurations beforehand
// (k_sample_jobs, at the full occupancy of a sampling kernel). TWO: two steps per pass of the whole-cross-section tile (the
// first step kept in LDS, walk_step2); the decisions are those of single steps.
template <bool TWO>
__device__ __forceinline__ void persist_body(const PersistArgs& a) {
    const Tail tl = lds_tail(a.lds);
    fill_codes(tl.ct);
    const int E = a.depth;
    float* ya = a.ya + blockIdx.x * a.state_stride;
    float* yb = a.yb + blockIdx.x * a.state_stride;
    uint8_t* code = a.code + blockIdx.x * a.state_stride;
    float* far1 = TWO ? a.far1 + blockIdx.x * a.far1_stride : nullptr;
    unsigned long long work = 0;  // tube slots advanced by this workgroup's steps
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) {
            const unsigned long long c = atomicAdd(a.queue, 1ull);
            tl.misc[2] = (uint32_t)c;
            tl.misc[3] = (uint32_t)(c >> 32);
        }
        __syncthreads();
        const int64_t q = (int64_t)(((uint64_t)tl.misc[3] << 32) | tl.misc[2]);
        if (q >= a.n_jobs) {
            if (threadIdx.x == 0 && a.work && work) atomicAdd(a.work, work);
            break;
        }
        const int64_t j = uniform_i64(a.order + q);  // outputs stay indexed by job
        const Job job = uniform_load(a.jobs + j);
        const DevShape sh = uniform_load(a.shapes + job.shape);
        const uint32_t* bits = job.bits;  // the caller's, or drawn by k_sample_jobs beforehand
        // initialisation: codes of every cell, start state in ya
        const int n0 = count_start(sh, bits, tl.misc + 1);
        const float x0 = n0 > 0 ? 1.0f / (float)n0 : 0.0f;
        uint32_t f = 0;
        for (int ub = 0; ub < sh.U; ub += E)
            for (int k = 0; k < sh.ntile; ++k) f |= walk_init(sh, load_tile(sh, k), tl.ct, bits, code, ya, ub, ub + E, x0);
        __syncthreads();
        if (threadIdx.x == 0) tl.misc[0] = 0;
        __syncthreads();
        if (f) atomicOr(&tl.misc[0], f);
        __syncthreads();
        f = tl.misc[0];
        int32_t perc = -1, steps = 0, mm = 0, front = 0, par = 0;
        bool hit_first = false;  // decided on the first step of a two-step pass
        if (!(f & F_NONEMPTY)) { perc = 0; steps = 0; }
        else if (f & F_FAR) { perc = 1; steps = 1; }
        while (perc < 0) {
            const float* yin = par ? yb : ya;
            float* yout = par ? ya : yb;
            par ^= 1;
            if (!TWO) {
                const int ulim = min(sh.U, front + 2);
                work += (unsigned long long)ulim * (unsigned long long)sh.C;
                uint32_t fl = 0;
                for (int ub = 0; ub < ulim; ub += E)
                    for (int k = 0; k < sh.ntile; ++k)
                        fl |= walk_step<true>(sh, load_tile(sh, k), tl.ct, yin, yout, code, ub, ub + E, front, front);
                __syncthreads();
                if (threadIdx.x == 0) tl.misc[0] = 0;
                __syncthreads();
                if (fl) atomicOr(&tl.misc[0], fl);
                __syncthreads();
                f = tl.misc[0];
                mm += 1;
                if (f & F_FRONT) front += 1;
                if (f & F_FAR) { perc = 1; steps = mm + 1; }
                else if (!(f & F_GREW)) { perc = 0; steps = mm; }
                else if (mm > sh.N) { perc = 0; steps = mm; if (threadIdx.x == 0) atomicOr(a.err, 1u); }
            } else {
                const int ulim = min(sh.U, front + 3);
                uint32_t fl = 0, fl2 = 0;
                for (int ub = 0; ub < ulim; ub += E)
                    for (int k = 0; k < sh.ntile; ++k) {
                        uint32_t g2 = 0;
                        fl |= walk_step2<1>(sh, k, load_tile(sh, k), tl.ct, yin, yout, code, far1, ub, ub + E, front,
                                         a.r1_off, &g2);
                        fl2 |= g2;
                    }
                __syncthreads();
                if (threadIdx.x == 0) { tl.misc[0] = 0; tl.misc[6] = 0; }
                __syncthreads();
                if (fl) atomicOr(&tl.misc[0], fl);
                if (fl2) atomicOr(&tl.misc[6], fl2);
                __syncthreads();
                f = tl.misc[0];
                const uint32_t f2 = tl.misc[6];
                // the first step
                mm += 1;
                work += (unsigned long long)min(sh.U, front + 2) * (unsigned long long)sh.C;
                if (f & F_FRONT) front += 1;
                if (f & F_FAR) { perc = 1; steps = mm + 1; hit_first = true; }
                else if (!(f & F_GREW)) { perc = 0; steps = mm; }
                else if (mm > sh.N) { perc = 0; steps = mm; if (threadIdx.x == 0) atomicOr(a.err, 1u); }
                else {
                    // the second step; its front flags are relative to the front before the first
                    mm += 1;
                    work += (unsigned long long)min(sh.U, front + 2) * (unsigned long long)sh.C;
                    if ((f & F_FRONT) ? (f2 & F_FRONT2) : (f2 & F_FRONT)) front += 1;
                    if (f2 & F_FAR) { perc = 1; steps = mm + 1; }
                    else if (!(f2 & F_GREW)) { perc = 0; steps = mm; }
                    else if (mm > sh.N) { perc = 0; steps = mm; if (threadIdx.x == 0) atomicOr(a.err, 1u); }
                }
            }
        }
        if (threadIdx.x == 0) {
            a.out.perc[j] = (uint8_t)perc;
            a.out.steps[j] = steps;
            if (a.out.group_count && job.group >= 0 && perc == 1) atomicAdd(&a.out.group_count[job.group], 1ull);
        }
        if (a.out.hit) {
            float h = 0.0f;
            if (perc == 1) {
                // the detector mass at the stop: the far-end sum of the state after steps-1
                // steps (the newest one, or the first step of the last pass)
                if (TWO && hit_first)
                    far_sum_cols(sh, far1, front, tl.part, tl.misc + 4, reinterpret_cast<float*>(tl.misc + 5));
                else
                    far_sum(sh, par ? yb : ya, front, tl.part, tl.misc + 4, reinterpret_cast<float*>(tl.misc + 5));
                h = __uint_as_float(tl.misc[5]);
            }
            if (threadIdx.x == 0) a.out.hit[j] = h;
        }
    }
}

// Register budget: six waves per SIMD (80 VGPRs). The initialisation phase alone would
// take 96 VGPRs (two workgroups per CU at the usual 448 threads); capped, a few words of
// its set-up spill (outside the step walk) and a third workgroup fits on every CU.
__global__ void __launch_bounds__(kMaxBlock) __attribute__((amdgpu_waves_per_eu(6))) k_persist(PersistArgs a) {
    persist_body<false>(a);
}

__global__ void __launch_bounds__(kMaxBlock) k_persist2(PersistArgs a) { persist_body<true>(a); }

// Test hook support: far-end sum added to the detector mass, reach of the detector.
__global__ void __launch_bounds__(256) k_far_acc(DevShape sh, const float* y, float* det_mass,
                                                 uint32_t* det_reached) {
    __shared__ float part[256];
    __shared__ uint32_t reached;
    __shared__ float result;
    far_sum(sh, y, sh.U, part, &reached, &result);
    if (threadIdx.x == 0) {
        *det_mass = *det_mass + result;
        if (reached) *det_reached = 1u;
    }
}

// x = |y| deg and the reach bit of every tube, scattered to canonical order.
__global__ void __launch_bounds__(256) k_export(DevShape sh, const float* __restrict__ y,
                                                const uint8_t* __restrict__ code, const float* det_mass,
                                                const uint32_t* det_reached, float* __restrict__ x_out,
                                                uint8_t* __restrict__ reach_out) {
    const int64_t total = (int64_t)sh.U * sh.C;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= total;
         i += (int64_t)gridDim.x * blockDim.x) {
        if (i == total) {
            x_out[sh.N] = *det_mass;
            reach_out[sh.N] = (uint8_t)(*det_reached ? 1 : 0);
            continue;
        }
        const int64_t u = i / sh.C, c = i - u * sh.C;
        const int64_t s = u * sh.C + sh.rank[c];
        if (s >= sh.N) continue;
        const uint32_t g = word_of(sh, (int)u, (int)c);
        const uint32_t w = __float_as_uint(y[g]);
        const uint32_t cd = code_of(reinterpret_cast<const uint32_t*>(code), sh, (int)u, (int)c);
        float x = 0.0f;
        if (cd < 15u) x = mag(w) * (cd == 0u ? 1.0f : (float)cd);
        x_out[s] = x;
        reach_out[s] = (uint8_t)(w != 0u ? 1 : 0);
    }
}

// Backward form of Eq. 3 over all sources: f^(1) of every tube, the probability that a
// walker on it enters the detector at its next move (1/deg on metallic far-end tubes, 0
// elsewhere), written over every word of the state, padding included. Later terms use
// the forward step's map unchanged: f^(m)_i = (1/deg_i) sum over metallic contacts k of
// f^(m-1)_k, the detector column excluded.
__global__ void __launch_bounds__(256) k_backward_init(DevShape sh, const uint8_t* __restrict__ code0,
                                                       float* __restrict__ y0, int64_t stride, int n_cfg) {
    const int64_t total = (int64_t)((sh.U + 3) / 4) * sh.CP * 4;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total * n_cfg;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t cfg = t / total, i = t - cfg * total;
        const uint8_t* code = code0 + cfg * stride;
        float* y = y0 + cfg * stride;
        const int64_t q = i >> 2;
        const int grp = (int)(q / sh.CP), c = (int)(q - (int64_t)grp * sh.CP);
        const int u = grp * 4 + (int)(i & 3);
        float v = 0.0f;
        if (c < sh.C && u < sh.U && u == top_of(sh, c)) {
            const uint32_t cd = code_of(reinterpret_cast<const uint32_t*>(code), sh, u, c);
            if (cd > 0u && cd < 15u) v = 1.0f / (float)cd;
        }
        y[i] = v;
    }
}

// The state words themselves (no degree factor), scattered to canonical order.
__global__ void __launch_bounds__(256) k_export_raw(DevShape sh, const float* __restrict__ y0,
                                                    float* __restrict__ f_out, int64_t stride, int n_cfg) {
    const int64_t total = (int64_t)sh.U * sh.C;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total * n_cfg;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t cfg = t / total, i = t - cfg * total;
        const int64_t u = i / sh.C, c = i - u * sh.C;
        const int64_t s = u * sh.C + sh.rank[c];
        if (s < sh.N) f_out[cfg * sh.N + s] = mag(__float_as_uint(y0[cfg * stride + word_of(sh, (int)u, (int)c)]));
    }
}

// Histogram of the stop step m* over the percolating configurations (the shortest
// spanning path has m* tubes): bin min(m*, nbins - 1).
__global__ void __launch_bounds__(256) k_steps_hist(const uint8_t* __restrict__ perc,
                                                    const int32_t* __restrict__ steps, int64_t n, int32_t nbins,
                                                    unsigned long long* __restrict__ hist) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        if (!perc[i]) continue;
        const int32_t m = steps[i];
        const int32_t b = m < 0 ? 0 : (m >= nbins ? nbins - 1 : m);
        atomicAdd(&hist[b], 1ull);
    }
}

__global__ void __launch_bounds__(256) k_fill_u32(uint32_t* __restrict__ p, int64_t n, uint32_t v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void __launch_bounds__(256) k_scatter_out(int64_t n, const int64_t* __restrict__ idx,
                                                     const uint8_t* __restrict__ perc, const int32_t* __restrict__ steps,
                                                     const float* __restrict__ hit, uint8_t* __restrict__ perc_out,
                                                     int32_t* __restrict__ steps_out, float* __restrict__ hit_out) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = idx[i];
        perc_out[j] = perc[i];
        steps_out[j] = steps[i];
        if (hit) hit_out[j] = hit[i];
    }
}

__global__ void __launch_bounds__(256) k_count(const uint8_t* __restrict__ perc, int64_t n,
                                               unsigned long long* count) {
    __shared__ unsigned long long red;
    if (threadIdx.x == 0) red = 0;
    __syncthreads();
    unsigned long long c = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        c += perc[i] ? 1ull : 0ull;
    if (c) atomicAdd(&red, c);
    __syncthreads();
    if (threadIdx.x == 0 && red) atomicAdd(count, red);
}

// Slot tables of a batch of n configurations of one shape whose occupancy words lie back
// to back from `bits` and whose state slots lie `stride` words apart.
__global__ void __launch_bounds__(256) k_slot_table(int32_t* __restrict__ slot_shape, int64_t* __restrict__ slot_off,
                                                    const uint32_t** __restrict__ slot_bits, int32_t n, int64_t stride,
                                                    const uint32_t* bits, int64_t words) {
    for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < n; b += gridDim.x * blockDim.x) {
        slot_shape[b] = 0;
        slot_off[b] = (int64_t)b * stride;
        slot_bits[b] = bits + (int64_t)b * words;
    }
}

// Streaming copy, the HBM ceiling the step kernels are compared with: each workgroup
// copies one contiguous chunk with 16-byte loads and non-temporal 16-byte stores (the
// step kernel's access pattern without the stencil).
__global__ void __launch_bounds__(512) k_stream_copy(const uint4* __restrict__ src, uint4* __restrict__ dst, int64_t n,
                                                     int64_t per) {
    typedef uint32_t v4u __attribute__((ext_vector_type(4)));
    const int64_t b = (int64_t)blockIdx.x * per, e = min(b + per, n);
    for (int64_t i = b + threadIdx.x; i < e; i += blockDim.x) {
        const uint4 v = src[i];
        const v4u w = {v.x, v.y, v.z, v.w};
        __builtin_nontemporal_store(w, reinterpret_cast<v4u*>(dst) + i);
    }
}

// Work memory of the entry point that allocates nothing (perc_inspect_noalloc): one
// array per device, part of the code object, kept until the process ends. Host code
// never passes the array's name to a kernel: it takes the device address once per
// device (scratch_region) and carves that.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr size_t kDynLds = 160 * 1024;  // dynamic LDS limit set once per device

template <typename K>
hipError_t allow_lds(K kernel) {
    return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)kDynLds);
}

}  // namespace

hipError_t prepare_kernels(int device) {
    int cur = 0;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device) return hipErrorInvalidDevice;
    e = allow_lds(k_span_init);
    if (e == hipSuccess) e = allow_lds(k_span_extend);
    if (e == hipSuccess) e = allow_lds(k_span_step);
    if (e == hipSuccess) e = allow_lds(k_span_step2);
    if (e == hipSuccess) e = allow_lds(k_chunk_step);
    if (e == hipSuccess) e = allow_lds(k_persist);
    if (e == hipSuccess) e = allow_lds(k_persist2);
    return e;
}

hipError_t scratch_region(void** ptr, size_t* bytes) {
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static void* addr[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> g(mu);
    if (!addr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        addr[dev] = p;
    }
    *ptr = addr[dev];
    *bytes = kScratchBytes;
    return hipSuccess;
}

hipError_t launch_stream_copy(const void* src, void* dst, int64_t n16, int grid, hipStream_t s) {
    if (n16 <= 0) return hipSuccess;
    const int64_t per = (n16 + grid - 1) / grid;
    hipLaunchKernelGGL(k_stream_copy, dim3(grid), dim3(512), 0, s, reinterpret_cast<const uint4*>(src),
                       reinterpret_cast<uint4*>(dst), n16, per);
    return hipGetLastError();
}

hipError_t launch_slot_table(int32_t* slot_shape, int64_t* slot_off, const uint32_t** slot_bits, int32_t n,
                             int64_t stride, const uint32_t* bits, int64_t words, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_slot_table, dim3((n + 255) / 256), dim3(256), 0, s, slot_shape, slot_off, slot_bits, n, stride,
                       bits, words);
    return hipGetLastError();
}

int32_t span_step_resident(int32_t block, int32_t lds) {
    int n = 0, dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_span_step, block, lds) != hipSuccess) return 0;
    return n * cus;
}

int persist_resident_per_cu(int block, int lds_bytes) {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_persist, block, lds_bytes) != hipSuccess) return 1;
    return n;
}

int persist2_resident_per_cu(int block, int lds_bytes) {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_persist2, block, lds_bytes) != hipSuccess) return 1;
    return n;
}

hipError_t launch_fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int grid = (int)std::min<int64_t>((n + 255) / 256, 16384);
    hipLaunchKernelGGL(k_fill_u32, dim3(grid), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_scatter_out(int64_t n, const int64_t* idx, const uint8_t* perc, const int32_t* steps,
                              const float* hit, uint8_t* perc_out, int32_t* steps_out, float* hit_out,
                              hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int grid = (int)std::min<int64_t>((n + 255) / 256, 16384);
    hipLaunchKernelGGL(k_scatter_out, dim3(grid), dim3(256), 0, s, n, idx, perc, steps, hit, perc_out, steps_out,
                       hit_out);
    return hipGetLastError();
}

hipError_t launch_sample(const DevShape& sh, uint32_t* bits, int64_t n_cfg, uint64_t cfg0, uint64_t threshold,
                         uint64_t seed, hipStream_t s) {
    const int64_t total = n_cfg * sh.words;
    if (total <= 0) return hipSuccess;
    const int grid = (int)std::min<int64_t>((total + 255) / 256, 65536);
    const uint32_t tag = ((uint32_t)sh.W << 16) | (uint32_t)sh.L;
    hipLaunchKernelGGL(k_sample, dim3(grid), dim3(256), 0, s, bits, sh.words, sh.N, n_cfg, cfg0, threshold,
                       (uint32_t)seed, (uint32_t)(seed >> 32), tag);
    return hipGetLastError();
}

hipError_t launch_sample_fixed(const DevShape& sh, uint32_t* bits, int64_t n_cfg, uint64_t cfg0, int64_t K,
                               uint64_t seed, hipStream_t s) {
    if (n_cfg <= 0) return hipSuccess;
    const int grid = (int)std::min<int64_t>(n_cfg, 65536);
    const uint32_t tag = ((uint32_t)sh.W << 16) | (uint32_t)sh.L;
    hipLaunchKernelGGL(k_sample_fixed, dim3(grid), dim3(1024), 0, s, bits, sh.words, sh.N, K, n_cfg, cfg0,
                       (uint32_t)seed, (uint32_t)(seed >> 32), tag);
    return hipGetLastError();
}

hipError_t launch_sample_slots(const DevShape* shapes, const Job* jobs, int32_t n_slot, uint32_t* const* slot_bits,
                               hipStream_t s) {
    if (n_slot <= 0) return hipSuccess;
    const int grid = std::min(n_slot, 65536);
    hipLaunchKernelGGL(k_sample_slots, dim3(grid), dim3(256), 0, s, shapes, jobs, n_slot, slot_bits);
    return hipGetLastError();
}

hipError_t launch_sample_jobs(const DevShape* shapes, const Job* jobs, const int64_t* idx, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int grid = (int)std::min<int64_t>(n, 65536);
    hipLaunchKernelGGL(k_sample_jobs, dim3(grid), dim3(256), 0, s, shapes, jobs, idx, n);
    return hipGetLastError();
}

hipError_t launch_span_init_only(const SpanArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_span_layout, dim3(1), dim3(kMaxBlock), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_span_init, dim3(a.grid), dim3(a.block), a.lds, s, a);
    return hipGetLastError();
}

hipError_t launch_span_init(const SpanArgs& a, hipStream_t s) {
    hipError_t e = launch_span_init_only(a, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_span_plan, dim3(1), dim3(kMaxBlock), 0, s, a, 1);
    return hipGetLastError();
}

hipError_t launch_span_step(const SpanArgs& a, hipStream_t s) {
    if (a.fused) return launch_span_step2(a, s);
    hipLaunchKernelGGL(k_span_step, dim3(a.grid), dim3(a.block), a.lds, s, a);
    return hipGetLastError();
}

hipError_t launch_span_extend(const SpanArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_span_extend, dim3(a.grid), dim3(a.block), a.lds, s, a);
    return hipGetLastError();
}

hipError_t launch_span_plan(const SpanArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_span_plan, dim3(1), dim3(kMaxBlock), 0, s, a, 0);
    return hipGetLastError();
}

hipError_t launch_span_finish(const SpanArgs& a, hipStream_t s) {
    if (!a.out.hit && !a.out.group_count) return hipSuccess;
    const int grid = std::min(a.fin ? std::max(a.n_slot, 1) : a.n_slot, 4096);
    if (grid <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_span_finish, dim3(grid), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_span_step2(const SpanArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_span_step2, dim3(a.grid), dim3(a.block), a.lds, s, a);
    return hipGetLastError();
}

hipError_t launch_chunk_step(const DevShape& sh, const float* yin, float* yout, const uint8_t* code, int depth,
                             int block, hipStream_t s) {
    return launch_multi_step(sh, yin, yout, code, 0, 1, depth, block, s);
}

hipError_t launch_multi_step(const DevShape& sh, const float* yin, float* yout, const uint8_t* code, int64_t stride,
                             int n_cfg, int depth, int block, hipStream_t s) {
    const int lds = (int)lds_total(sh.span_max);
    const int64_t items = (int64_t)((sh.U + depth - 1) / depth) * sh.ntile * n_cfg;
    // several items per workgroup when there are many (whole multiples of the XCD count)
    const int grid = items <= 4096 ? (int)items : 4096;
    hipLaunchKernelGGL(k_chunk_step, dim3(grid), dim3(block), lds, s, sh, yin, yout, code, stride, n_cfg, depth, lds);
    return hipGetLastError();
}

hipError_t launch_persist(const PersistArgs& a, hipStream_t s) {
    if (a.two)
        hipLaunchKernelGGL(k_persist2, dim3(a.grid), dim3(a.block), a.lds, s, a);
    else
        hipLaunchKernelGGL(k_persist, dim3(a.grid), dim3(a.block), a.lds, s, a);
    return hipGetLastError();
}

hipError_t launch_far_sum(const DevShape& sh, const float* y, float* det_mass, uint32_t* det_reached,
                          hipStream_t s) {
    hipLaunchKernelGGL(k_far_acc, dim3(1), dim3(256), 0, s, sh, y, det_mass, det_reached);
    return hipGetLastError();
}

hipError_t launch_export(const DevShape& sh, const float* y, const uint8_t* code, const float* det_mass,
                         const uint32_t* det_reached, float* x_out, uint8_t* reach_out, hipStream_t s) {
    const int grid = (int)std::min<int64_t>(((int64_t)sh.U * sh.C + 1 + 255) / 256, 65536);
    hipLaunchKernelGGL(k_export, dim3(grid), dim3(256), 0, s, sh, y, code, det_mass, det_reached, x_out, reach_out);
    return hipGetLastError();
}

hipError_t launch_backward_init(const DevShape& sh, const uint8_t* code, float* y, int64_t stride, int n_cfg,
                                hipStream_t s) {
    const int64_t total = (int64_t)((sh.U + 3) / 4) * sh.CP * 4 * n_cfg;
    const int grid = (int)std::min<int64_t>((total + 255) / 256, 65536);
    hipLaunchKernelGGL(k_backward_init, dim3(grid), dim3(256), 0, s, sh, code, y, stride, n_cfg);
    return hipGetLastError();
}

hipError_t launch_export_raw(const DevShape& sh, const float* y, float* f_out, int64_t stride, int n_cfg,
                             hipStream_t s) {
    const int grid = (int)std::min<int64_t>(((int64_t)sh.U * sh.C * n_cfg + 255) / 256, 65536);
    hipLaunchKernelGGL(k_export_raw, dim3(grid), dim3(256), 0, s, sh, y, f_out, stride, n_cfg);
    return hipGetLastError();
}

hipError_t launch_steps_hist(const uint8_t* perc, const int32_t* steps, int64_t n, int32_t nbins,
                             unsigned long long* hist, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int grid = (int)std::min<int64_t>((n + 255) / 256, 1024);
    hipLaunchKernelGGL(k_steps_hist, dim3(grid), dim3(256), 0, s, perc, steps, n, nbins, hist);
    return hipGetLastError();
}

hipError_t launch_count(const uint8_t* perc, int64_t n, unsigned long long* count, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int grid = (int)std::min<int64_t>((n + 255) / 256, 1024);
    hipLaunchKernelGGL(k_count, dim3(grid), dim3(256), 0, s, perc, n, count);
    return hipGetLastError();
}

}  // namespace perc
