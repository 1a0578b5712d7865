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
// Representation (one 32-bit word per tube, per state buffer):
//   value  = y = x / deg, the mass the tube sends along each of its deg contacts, so a
//            receiver sums its neighbours' words and scales by its own 1/deg only;
//   sign   = reached bit. Probabilities are non-negative, so the sign bit is free; it
//            carries the exact reached set even where the FP32 value has underflowed
//            to zero (the decision never looks at the FP32 value).
// Per tube a byte `code` holds deg (0..14) of a metallic tube, 15 for an insulating or
// absent one. A metallic tube of degree 0 keeps its mass (self-loop, Sec. II.B).
//
// The state of one configuration is [U cells][CP] words, cell u holding layer 3u + sigma
// of every column (see perc_internal.hpp). A chunk of D consecutive cells is staged in
// LDS column-major with one halo cell on each side: word (column c, slot j) at byte
// (c*(D+2) + j)*4, so the 14 contacts of tube (j, c) are LDS reads at per-column byte
// offsets plus the compile-time immediate -- no address arithmetic per tube. All LDS of
// these kernels is dynamic (layout: lds_map), so the chunk sits at LDS address 0.
#include <hip/hip_runtime.h>

#include "perc_internal.hpp"

namespace perc {

namespace {

constexpr int kMaxBlock = 1024;
constexpr int kXcds = 8;  // MI355X: workgroups are dealt round-robin over 8 XCDs

extern __shared__ __align__(16) unsigned char lds[];

__device__ __forceinline__ uint32_t lds_u32(uint32_t off) { return *reinterpret_cast<const uint32_t*>(lds + off); }
__device__ __forceinline__ float lds_f32(uint32_t off) { return *reinterpret_cast<const float*>(lds + off); }
__device__ __forceinline__ uint32_t lds_u8(uint32_t off) { return lds[off]; }
__device__ __forceinline__ void lds_put_u32(uint32_t off, uint32_t v) { *reinterpret_cast<uint32_t*>(lds + off) = v; }

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

// 1/deg per code: code 0 keeps its mass (factor 1), 1..14 the correctly rounded
// FP32 reciprocal, 15 (insulating) sends nothing.
__device__ __forceinline__ void fill_rcp(float* rcp) {
    if (threadIdx.x < 16) {
        const int d = threadIdx.x;
        rcp[d] = d == 0 ? 1.0f : (d == 15 ? 0.0f : 1.0f / (float)d);
    }
}

__device__ __forceinline__ float mag(uint32_t w) { return __uint_as_float(w & 0x7fffffffu); }

// Stage cells u0-1 .. u0+D of a state buffer (column-major) and the degree codes of
// cells u0 .. u0+D-1 into LDS. Cells beyond the reached front or outside the fiber and
// the pad column C read as zero; codes outside the fiber as 15.
template <int D>
__device__ __forceinline__ void stage_chunk(const DevTables& t, const LdsMap& m, const float* __restrict__ y,
                                            const uint8_t* __restrict__ code, int u0, int front) {
    constexpr int SJ = D + 2;
    const int C = t.C;
    for (int c = threadIdx.x; c <= C; c += blockDim.x) {
        float v[SJ];
#pragma unroll
        for (int j = 0; j < SJ; ++j) {
            const int u = u0 - 1 + j;
            v[j] = (c < C && u >= 0 && u <= front && u < t.U) ? y[(uint32_t)(u * t.CP + c)] : 0.0f;
        }
        uint32_t cd[D];
#pragma unroll
        for (int j = 1; j <= D; ++j) {
            const int u = u0 - 1 + j;
            cd[j - 1] = (c < C && u < t.U) ? code[(uint32_t)(u * t.CP + c)] : 15u;
        }
#pragma unroll
        for (int j = 0; j < SJ; ++j) lds_put_u32((uint32_t)(c * SJ + j) * 4u, __float_as_uint(v[j]));
        if (c < C) {
#pragma unroll
            for (int j = 0; j < D; ++j) lds[m.code + (uint32_t)(c * D + j)] = (unsigned char)cd[j];
        }
    }
}

// One Jacobi step for cells u0 .. u0+D-1 (those below min(U, front+2)), reading the
// staged input and writing y' to `yout`. Returns the OR of the step flags seen by
// this thread. The 14 contributions are summed in one fixed pairwise order, so a tube
// gets the same FP32 result in every execution form and batch composition.
template <int D>
__device__ __forceinline__ uint32_t step_chunk(const DevTables& t, const LdsMap& m, float* __restrict__ yout,
                                               int u0, int front) {
    constexpr int SJ = D + 2;
    const int C = t.C;
    const int ulim = min(t.U, front + 2);
    uint32_t grew = 0, far = 0, entered = 0;
    // the contact table entries of the next column are loaded while this one computes
    uint32_t o_next[kSide];
    int top_next = -1;
    if ((int)threadIdx.x < C) {
#pragma unroll
        for (int i = 0; i < kSide; ++i) o_next[i] = t.nboff[i * C + threadIdx.x];
        top_next = t.top[threadIdx.x];
    }
    for (int c = threadIdx.x; c < C; c += blockDim.x) {
        uint32_t o[kSide];
#pragma unroll
        for (int i = 0; i < kSide; ++i) o[i] = o_next[i];
        const int top = top_next;
        const int cn = c + (int)blockDim.x;
        if (cn < C) {
#pragma unroll
            for (int i = 0; i < kSide; ++i) o_next[i] = t.nboff[i * C + cn];
            top_next = t.top[cn];
        }
        const uint32_t oc = (uint32_t)(c * SJ) * 4u;
        const uint32_t ocd = m.code + (uint32_t)(c * D);
#pragma unroll
        for (int j = 1; j <= D; ++j) {
            const int u = u0 - 1 + j;
            if (u >= ulim) break;
            const uint32_t own = lds_u32(oc + j * 4);
            const uint32_t dn = lds_u32(oc + (j - 1) * 4);
            const uint32_t up = lds_u32(oc + (j + 1) * 4);
            uint32_t n[kSide];
#pragma unroll
            for (int i = 0; i < kSide; ++i) n[i] = lds_u32(o[i] + (j - 1) * 4);
            const uint32_t cd = lds_u8(ocd + (j - 1));
            uint32_t any = own | dn | up;
#pragma unroll
            for (int i = 0; i < kSide; ++i) any |= n[i];
            // fixed order: in-layer pairs, up/down-layer pairs, then the end contacts
            const float s01 = mag(n[0]) + mag(n[1]);
            const float s23 = mag(n[2]) + mag(n[3]);
            const float s45 = mag(n[4]) + mag(n[5]);
            const float s67 = mag(n[6]) + mag(n[7]);
            const float s89 = mag(n[8]) + mag(n[9]);
            const float sab = mag(n[10]) + mag(n[11]);
            const float sud = mag(dn) + mag(up);
            const float sum = ((s01 + s23) + (s45 + s67)) + ((s89 + sab) + sud);
            // a metallic tube of degree 0 has no metallic contact (sum == 0): it keeps
            // its own mass
            const float x = sum + (cd == 0u ? mag(own) : 0.0f);
            const uint32_t newr = (any >> 31) & (cd < 15u ? 1u : 0u);
            const float yn = x * lds_f32(m.rcp + cd * 4u);
            yout[(uint32_t)(u * t.CP + c)] = __uint_as_float(__float_as_uint(yn) | (newr << 31));
            grew |= newr & ~(own >> 31);
            far |= newr & (u == top ? 1u : 0u);
            if (u == front + 1) entered |= newr;
        }
    }
    return (grew ? F_GREW : 0u) | (far ? F_FAR : 0u) | (entered ? F_FRONT : 0u);
}

// Number of metallic start tubes (every tube of cell 0) of one configuration.
__device__ __forceinline__ int count_start(const DevTables& t, const uint32_t* __restrict__ bits, int* red) {
    const int64_t n0 = min((int64_t)t.C, t.N);
    int cnt = 0;
    for (int64_t w = threadIdx.x; w * 32 < n0; w += blockDim.x) {
        uint32_t b = bits[w];
        const int64_t rem = n0 - w * 32;
        if (rem < 32) b &= (1u << rem) - 1u;
        cnt += __popc(b);
    }
    if (threadIdx.x == 0) *red = 0;
    __syncthreads();
    if (cnt) atomicAdd(red, cnt);
    __syncthreads();
    const int total = *red;
    __syncthreads();
    return total;
}

// Degree codes of cells u0 .. u0+D-1 from the occupancy (staged as 0/1 words in the
// state area of the LDS), and the initial state of the start tubes (cell 0):
// x0 = 1/|S0| on every metallic start tube, reached.
template <int D>
__device__ __forceinline__ uint32_t init_chunk(const DevTables& t, const LdsMap& m, const uint32_t* __restrict__ bits,
                                               uint8_t* __restrict__ code, float* __restrict__ y0, int u0, float x0) {
    constexpr int SJ = D + 2;
    const int C = t.C;
    for (int c = threadIdx.x; c <= C; c += blockDim.x) {
#pragma unroll
        for (int j = 0; j < SJ; ++j) {
            const int u = u0 - 1 + j;
            const int64_t s = (int64_t)u * C + c;
            uint32_t o = 0;
            if (c < C && u >= 0 && u < t.U && s < t.N) o = (bits[s >> 5] >> (s & 31)) & 1u;
            lds_put_u32((uint32_t)(c * SJ + j) * 4u, o);
        }
    }
    __syncthreads();
    uint32_t fl = 0;
    for (int c = threadIdx.x; c < C; c += blockDim.x) {
        uint32_t o[kSide];
#pragma unroll
        for (int i = 0; i < kSide; ++i) o[i] = t.nboff[i * C + c];
        const int top = t.top[c];
        const uint32_t oc = (uint32_t)(c * SJ) * 4u;
#pragma unroll
        for (int j = 1; j <= D; ++j) {
            const int u = u0 - 1 + j;
            if (u >= t.U) break;
            const uint32_t me = lds_u32(oc + j * 4);
            uint32_t deg = lds_u32(oc + (j - 1) * 4) + lds_u32(oc + (j + 1) * 4) + (u == top ? 1u : 0u);
#pragma unroll
            for (int i = 0; i < kSide; ++i) deg += lds_u32(o[i] + (j - 1) * 4);
            const uint32_t cd = me ? deg : 15u;
            code[(uint32_t)(u * t.CP + c)] = (uint8_t)cd;
            if (u == 0) {
                float yv = 0.0f;
                if (me) {
                    yv = __uint_as_float(__float_as_uint(x0 * lds_f32(m.rcp + cd * 4u)) | 0x80000000u);
                    fl |= F_NONEMPTY;
                    if (u == top) fl |= F_FAR;
                }
                y0[c] = yv;
            }
        }
    }
    __syncthreads();
    return fl;
}

// Sum over the far-end tubes of |y| (the mass the detector receives next step) and
// whether any of them is reached. Cells beyond `front` hold no mass and are not read
// (their words may be stale). Fixed order independent of blockDim: 256 virtual lanes
// each add their columns in increasing order, then a fixed pairwise tree.
__device__ __forceinline__ void far_sum(const DevTables& t, const float* __restrict__ y, int front, float* part,
                                        uint32_t* reached, float* result) {
    if (threadIdx.x == 0) *reached = 0;
    __syncthreads();
    for (int v = threadIdx.x; v < 256; v += blockDim.x) {
        float s = 0.0f;
        uint32_t r = 0;
        for (int c = v; c < t.C; c += 256) {
            const int u = t.top[c];
            if (u < 0 || u > front) continue;
            const uint32_t w = __float_as_uint(y[(uint32_t)(u * t.CP + c)]);
            s += mag(w);
            r |= w >> 31;
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

// Items [0, total) of a launch, dealt so that the workgroups of one XCD take one
// contiguous range (neighbouring chunks of a configuration then share that XCD's L2).
struct ItemRange {
    int64_t begin, end, stride;
};
__device__ __forceinline__ ItemRange xcd_items(int64_t total) {
    const int G = gridDim.x;
    if (G % kXcds != 0 || total < G) return ItemRange{(int64_t)blockIdx.x, total, (int64_t)G};
    const int x = blockIdx.x % kXcds, lb = blockIdx.x / kXcds, per = G / kXcds;
    const int64_t b = total * x / kXcds, e = total * (x + 1) / kXcds;
    return ItemRange{b + lb, e, (int64_t)per};
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

template <int D>
__global__ void __launch_bounds__(kMaxBlock) k_span_init(SpanArgs a) {
    const DevTables& t = a.t;
    const LdsMap m = lds_map(t.C, D);
    float* rcp = reinterpret_cast<float*>(lds + m.rcp);
    uint32_t* misc = reinterpret_cast<uint32_t*>(lds + m.misc);
    fill_rcp(rcp);
    const int64_t stride = (int64_t)t.U * t.CP;
    const int nchunk = (t.U + D - 1) / D;
    const int64_t total = (int64_t)a.n_slot * nchunk;
    __syncthreads();
    for (int64_t g = blockIdx.x; g < total; g += gridDim.x) {
        const int b = (int)(g / nchunk);
        const int u0 = (int)(g - (int64_t)b * nchunk) * D;
        const uint32_t* bits = a.bits + (int64_t)b * t.words;
        float x0 = 0.0f;
        if (u0 == 0) {
            const int n0 = count_start(t, bits, reinterpret_cast<int*>(misc + 1));
            x0 = n0 > 0 ? 1.0f / (float)n0 : 0.0f;
        }
        const uint32_t fl = init_chunk<D>(t, m, bits, a.code + b * stride, a.ya + b * stride, u0, x0);
        if (u0 == 0) {
            if (threadIdx.x == 0) misc[0] = 0;
            __syncthreads();
            if (fl) atomicOr(&misc[0], fl);
            __syncthreads();
            if (threadIdx.x == 0) a.st[b] = CfgState{0, 0, 0, misc[0]};
            __syncthreads();
        }
    }
}

// Decide every active configuration from the flags of the last launch, write the
// outputs of those that stopped, and lay out the chunks of the next step for the rest.
// did_step = 0 right after initialisation. One workgroup of kMaxBlock threads.
__global__ void __launch_bounds__(kMaxBlock) k_span_plan(SpanArgs a, int did_step, int first) {
    __shared__ int32_t keep_s[kMaxBlock];
    __shared__ int64_t chunk_s[kMaxBlock];
    const int tid = threadIdx.x, nt = blockDim.x;
    const int n_act = first ? a.n_slot : a.hdr[0];
    const int per = (n_act + nt - 1) / nt;
    const int i0 = min(n_act, tid * per), i1 = min(n_act, i0 + per);
    const int D = a.depth, U = a.t.U;
    int32_t keep = 0;
    int64_t chunks = 0;
    for (int i = i0; i < i1; ++i) {
        const int b = first ? i : a.active[i];
        CfgState s = a.st[b];
        const uint32_t f = s.flags;
        s.flags = 0;
        int dec = -1;  // -1 continue, 0 no, 1 yes
        int32_t steps = 0;
        if (!did_step) {
            if (!(f & F_NONEMPTY)) { dec = 0; steps = 0; }
            else if (f & F_FAR) { dec = 1; steps = 1; }
        } else {
            s.m += 1;
            if (f & F_FRONT) s.front += 1;
            if (f & F_FAR) { dec = 1; steps = s.m + 1; }
            else if (!(f & F_GREW)) { dec = 0; steps = s.m; }
            else if (s.m >= a.cap) { dec = 0; steps = s.m; s.done = 2; a.hdr[2] = 1; }
        }
        if (dec >= 0) {
            if (s.done == 0) s.done = 1;
            a.out.perc[b] = (uint8_t)dec;
            a.out.steps[b] = steps;
        } else {
            keep += 1;
            chunks += (min(U, s.front + 2) + D - 1) / D;
        }
        a.st[b] = s;
    }
    keep_s[tid] = keep;
    chunk_s[tid] = chunks;
    __syncthreads();
    // inclusive scans over the threads (Hillis-Steele)
    for (int off = 1; off < nt; off <<= 1) {
        const int32_t kv = tid >= off ? keep_s[tid - off] : 0;
        const int64_t cv = tid >= off ? chunk_s[tid - off] : 0;
        __syncthreads();
        keep_s[tid] += kv;
        chunk_s[tid] += cv;
        __syncthreads();
    }
    int32_t kpos = keep_s[tid] - keep;
    int64_t cpos = chunk_s[tid] - chunks;
    const int32_t n_keep = keep_s[nt - 1];
    const int64_t n_chunks = chunk_s[nt - 1];
    unsigned long long cells = 0;
    for (int i = i0; i < i1; ++i) {
        const int b = first ? i : a.active[i];
        const CfgState s = a.st[b];
        if (s.done) continue;
        a.active2[kpos] = b;
        a.chunk_off[kpos] = cpos;
        kpos += 1;
        cpos += (min(U, s.front + 2) + D - 1) / D;
        cells += (unsigned long long)min(U, s.front + 2);
    }
    if (a.work && cells) atomicAdd(a.work, cells);
    __syncthreads();
    for (int i = tid; i < n_keep; i += nt) a.active[i] = a.active2[i];
    if (tid == 0) {
        a.chunk_off[n_keep] = n_chunks;
        a.hdr[0] = n_keep;
        a.hdr[1] = (int32_t)min(n_chunks, (int64_t)INT32_MAX);
    }
}

template <int D>
__global__ void __launch_bounds__(kMaxBlock) k_span_step(SpanArgs a) {
    const DevTables& t = a.t;
    const LdsMap m = lds_map(t.C, D);
    uint32_t* misc = reinterpret_cast<uint32_t*>(lds + m.misc);
    fill_rcp(reinterpret_cast<float*>(lds + m.rcp));
    const int n_act = a.hdr[0];
    const int64_t total = a.hdr[1];
    const int64_t stride = (int64_t)t.U * t.CP;
    const ItemRange it = xcd_items(total);
    for (int64_t g = it.begin; g < it.end; g += it.stride) {
        // active entry i with chunk_off[i] <= g < chunk_off[i+1]
        int lo = 0, hi = n_act - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (a.chunk_off[mid] <= g) lo = mid; else hi = mid - 1;
        }
        const int b = a.active[lo];
        const int u0 = (int)(g - a.chunk_off[lo]) * D;
        const CfgState s = a.st[b];
        const float* yin = ((s.m & 1) ? a.yb : a.ya) + b * stride;
        float* yout = ((s.m & 1) ? a.ya : a.yb) + b * stride;
        __syncthreads();  // previous item finished with the LDS
        if (threadIdx.x == 0) misc[0] = 0;
        stage_chunk<D>(t, m, yin, a.code + b * stride, u0, s.front);
        __syncthreads();
        const uint32_t fl = step_chunk<D>(t, m, yout, u0, s.front);
        if (fl) atomicOr(&misc[0], fl);
        __syncthreads();
        if (threadIdx.x == 0 && misc[0]) atomicOr(&a.st[b].flags, misc[0]);
    }
}

// One step of one configuration over cells [0, U) with an explicit front (test hook):
// workgroup b handles cells b*D .. b*D+D-1 with the same device code as the batches.
template <int D>
__global__ void __launch_bounds__(kMaxBlock) k_chunk_step(DevTables t, const float* yin, float* yout,
                                                          const uint8_t* code, int front) {
    const LdsMap m = lds_map(t.C, D);
    fill_rcp(reinterpret_cast<float*>(lds + m.rcp));
    const int u0 = blockIdx.x * D;
    stage_chunk<D>(t, m, yin, code, u0, front);
    __syncthreads();
    (void)step_chunk<D>(t, m, yout, u0, front);
}

// First-hit probability of every configuration that percolated: the detector mass
// at the stop equals the far-end sum of the state after steps-1 steps.
__global__ void __launch_bounds__(256) k_span_finish(SpanArgs a) {
    __shared__ float part[256];
    __shared__ uint32_t reached;
    __shared__ float result;
    const DevTables& t = a.t;
    const int64_t stride = (int64_t)t.U * t.CP;
    for (int b = blockIdx.x; b < a.n_slot; b += gridDim.x) {
        if (!a.out.perc[b]) {
            if (threadIdx.x == 0) a.out.hit[b] = 0.0f;
            continue;
        }
        const int m = a.out.steps[b] - 1;  // state after m steps sits in ya if m even
        const float* y = ((m & 1) ? a.yb : a.ya) + b * stride;
        far_sum(t, y, a.st[b].front, part, &reached, &result);
        if (threadIdx.x == 0) a.out.hit[b] = result;
        __syncthreads();
    }
}

template <int D>
__global__ void __launch_bounds__(kMaxBlock) k_persist(PersistArgs a) {
    const DevTables& t = a.t;
    const LdsMap m = lds_map(t.C, D);
    uint32_t* misc = reinterpret_cast<uint32_t*>(lds + m.misc);
    float* part = reinterpret_cast<float*>(lds + m.part);
    fill_rcp(reinterpret_cast<float*>(lds + m.rcp));
    const int64_t stride = (int64_t)t.U * t.CP;
    float* ya = a.ya + blockIdx.x * stride;
    float* yb = a.yb + blockIdx.x * stride;
    uint8_t* code = a.code + blockIdx.x * stride;
    const uint32_t k0 = (uint32_t)a.seed, k1 = (uint32_t)(a.seed >> 32);
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) {
            const unsigned long long c = atomicAdd(a.queue, 1ull);
            misc[2] = (uint32_t)c;
            misc[3] = (uint32_t)(c >> 32);
        }
        __syncthreads();
        const int64_t cfg = (int64_t)(((uint64_t)misc[3] << 32) | misc[2]);
        if (cfg >= a.n_cfg) break;
        const uint32_t* bits;
        if (a.bits) {
            bits = a.bits + cfg * t.words;
        } else {
            uint32_t* sb = a.bits_scratch + blockIdx.x * t.words;
            for (int64_t w = threadIdx.x; w < t.words; w += blockDim.x)
                sb[w] = sample_word(w, t.N, a.cfg0 + (uint64_t)cfg, a.threshold, k0, k1, a.tag);
            __syncthreads();
            bits = sb;
        }
        // initialisation: codes of every cell, start state in ya
        const int n0 = count_start(t, bits, reinterpret_cast<int*>(misc + 1));
        const float x0 = n0 > 0 ? 1.0f / (float)n0 : 0.0f;
        if (threadIdx.x == 0) misc[0] = 0;
        __syncthreads();
        for (int u0 = 0; u0 < t.U; u0 += D) {
            const uint32_t fl = init_chunk<D>(t, m, bits, code, ya, u0, x0);
            if (fl) atomicOr(&misc[0], fl);
        }
        __syncthreads();
        uint32_t f = misc[0];
        int32_t perc = -1, steps = 0, mm = 0, front = 0;
        if (!(f & F_NONEMPTY)) { perc = 0; steps = 0; }
        else if (f & F_FAR) { perc = 1; steps = 1; }
        while (perc < 0) {
            const float* yin = (mm & 1) ? yb : ya;
            float* yout = (mm & 1) ? ya : yb;
            __syncthreads();
            if (threadIdx.x == 0) misc[0] = 0;
            const int ulim = min(t.U, front + 2);
            for (int u0 = 0; u0 < ulim; u0 += D) {
                __syncthreads();
                stage_chunk<D>(t, m, yin, code, u0, front);
                __syncthreads();
                const uint32_t fl = step_chunk<D>(t, m, yout, u0, front);
                if (fl) atomicOr(&misc[0], fl);
            }
            __syncthreads();
            f = misc[0];
            mm += 1;
            if (f & F_FRONT) front += 1;
            if (f & F_FAR) { perc = 1; steps = mm + 1; }
            else if (!(f & F_GREW)) { perc = 0; steps = mm; }
            else if (mm >= a.cap) { perc = 0; steps = mm; if (threadIdx.x == 0) atomicOr(a.err, 1u); }
        }
        if (threadIdx.x == 0) {
            a.out.perc[cfg] = (uint8_t)perc;
            a.out.steps[cfg] = steps;
        }
        if (a.out.hit) {
            float h = 0.0f;
            if (perc == 1) {
                __syncthreads();
                far_sum(t, ((steps - 1) & 1) ? yb : ya, front, part, misc + 4, reinterpret_cast<float*>(misc + 5));
                h = __uint_as_float(misc[5]);
            }
            if (threadIdx.x == 0) a.out.hit[cfg] = h;
        }
    }
}

// Test hook support: far-end sum added to the detector mass, reach of the detector.
__global__ void __launch_bounds__(256) k_far_acc(DevTables t, const float* y, float* det_mass,
                                                 uint32_t* det_reached) {
    __shared__ float part[256];
    __shared__ uint32_t reached;
    __shared__ float result;
    far_sum(t, y, t.U, part, &reached, &result);
    if (threadIdx.x == 0) {
        *det_mass = *det_mass + result;
        if (reached) *det_reached = 1u;
    }
}

__global__ void __launch_bounds__(256) k_export(DevTables t, const float* __restrict__ y,
                                                const uint8_t* __restrict__ code, const float* det_mass,
                                                const uint32_t* det_reached, float* __restrict__ x_out,
                                                uint8_t* __restrict__ reach_out) {
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s <= t.N;
         s += (int64_t)gridDim.x * blockDim.x) {
        if (s == t.N) {
            x_out[s] = *det_mass;
            reach_out[s] = (uint8_t)(*det_reached ? 1 : 0);
            continue;
        }
        const int64_t u = s / t.C, c = s - u * t.C;
        const int64_t g = u * t.CP + c;
        const uint32_t w = __float_as_uint(y[g]);
        const uint32_t cd = code[g];
        float x = 0.0f;
        if (cd < 15u) x = mag(w) * (cd == 0u ? 1.0f : (float)cd);
        x_out[s] = x;
        reach_out[s] = (uint8_t)(w >> 31);
    }
}

__global__ void __launch_bounds__(256) k_fill_u32(uint32_t* __restrict__ p, int64_t n, uint32_t v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
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

// ------------------------------------------------------------------------------
// Depth dispatch
// ------------------------------------------------------------------------------
template <template <int> class F, typename... Args>
hipError_t dispatch_depth(int depth, Args&&... args) {
    switch (depth) {
        case 1: return F<1>::run(args...);
        case 3: return F<3>::run(args...);
        case 5: return F<5>::run(args...);
        case 7: return F<7>::run(args...);
        case 9: return F<9>::run(args...);
        case 15: return F<15>::run(args...);
        default: return hipErrorInvalidValue;
    }
}

constexpr size_t kDynLds = 160 * 1024;  // dynamic LDS limit set once per device

template <typename K>
hipError_t allow_lds(K kernel) {
    return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)kDynLds);
}

template <int D>
struct PrepDepth {
    static hipError_t run() {
        hipError_t e = allow_lds(k_span_init<D>);
        if (e == hipSuccess) e = allow_lds(k_span_step<D>);
        if (e == hipSuccess) e = allow_lds(k_chunk_step<D>);
        if (e == hipSuccess) e = allow_lds(k_persist<D>);
        return e;
    }
};

template <int D>
struct ResidentPersist {
    static hipError_t run(int block, int C, int* out) {
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(out, k_persist<D>, block, lds_map(C, D).total);
    }
};

template <int D>
struct RunSpanInit {
    static hipError_t run(const SpanArgs& a, hipStream_t s) {
        const size_t lds = lds_map(a.t.C, D).total;
        const int64_t nchunk = (a.t.U + D - 1) / D;
        const int64_t items = (int64_t)a.n_slot * nchunk;
        const int grid = (int)std::min<int64_t>(items, 65536);
        if (grid <= 0) return hipSuccess;
        hipLaunchKernelGGL(k_span_init<D>, dim3(grid), dim3(a.block), lds, s, a);
        return hipGetLastError();
    }
};

template <int D>
struct RunSpanStep {
    static hipError_t run(const SpanArgs& a, hipStream_t s) {
        const size_t lds = lds_map(a.t.C, D).total;
        hipLaunchKernelGGL(k_span_step<D>, dim3(a.grid), dim3(a.block), lds, s, a);
        return hipGetLastError();
    }
};

template <int D>
struct RunChunkStep {
    static hipError_t run(const DevTables& t, const float* yin, float* yout, const uint8_t* code, int front,
                          int block, hipStream_t s) {
        const size_t lds = lds_map(t.C, D).total;
        const int grid = (t.U + D - 1) / D;
        hipLaunchKernelGGL(k_chunk_step<D>, dim3(grid), dim3(block), lds, s, t, yin, yout, code, front);
        return hipGetLastError();
    }
};

template <int D>
struct RunPersist {
    static hipError_t run(const PersistArgs& a, hipStream_t s) {
        const size_t lds = lds_map(a.t.C, D).total;
        hipLaunchKernelGGL(k_persist<D>, dim3(a.grid), dim3(a.block), lds, s, a);
        return hipGetLastError();
    }
};

}  // namespace

size_t lds_bytes_for(int32_t C, int32_t depth) { return lds_map(C, depth).total; }

int32_t max_depth_for(int32_t C) {
    int32_t best = 0;
    for (int32_t d : kDepthList)
        if (lds_bytes_for(C, d) <= kDynLds) best = d;
    return best;
}

hipError_t prepare_kernels(int device) {
    int cur = 0;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device) return hipErrorInvalidDevice;
    for (int d : kDepthList) {
        e = dispatch_depth<PrepDepth>(d);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

int persist_resident_per_cu(int depth, int block, int C) {
    int n = 0;
    if (dispatch_depth<ResidentPersist>(depth, block, C, &n) != hipSuccess) return 1;
    return n;
}

hipError_t launch_fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int grid = (int)std::min<int64_t>((n + 255) / 256, 16384);
    hipLaunchKernelGGL(k_fill_u32, dim3(grid), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_sample(const DevTables& t, uint32_t* bits, int64_t n_cfg, uint64_t cfg0, uint64_t threshold,
                         uint64_t seed, uint32_t tag, hipStream_t s) {
    const int64_t total = n_cfg * t.words;
    if (total <= 0) return hipSuccess;
    const int grid = (int)std::min<int64_t>((total + 255) / 256, 65536);
    hipLaunchKernelGGL(k_sample, dim3(grid), dim3(256), 0, s, bits, t.words, t.N, n_cfg, cfg0, threshold,
                       (uint32_t)seed, (uint32_t)(seed >> 32), tag);
    return hipGetLastError();
}

hipError_t launch_span_init_only(const SpanArgs& a, hipStream_t s) {
    return dispatch_depth<RunSpanInit>(a.depth, a, s);
}

hipError_t launch_span_init(const SpanArgs& a, hipStream_t s) {
    hipError_t e = dispatch_depth<RunSpanInit>(a.depth, a, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_span_plan, dim3(1), dim3(kMaxBlock), 0, s, a, 0, 1);
    return hipGetLastError();
}

hipError_t launch_span_step(const SpanArgs& a, hipStream_t s) { return dispatch_depth<RunSpanStep>(a.depth, a, s); }

hipError_t launch_span_plan(const SpanArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_span_plan, dim3(1), dim3(kMaxBlock), 0, s, a, 1, 0);
    return hipGetLastError();
}

hipError_t launch_span_finish(const SpanArgs& a, hipStream_t s) {
    if (!a.out.hit) return hipSuccess;
    const int grid = std::min(a.n_slot, 4096);
    if (grid <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_span_finish, dim3(grid), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_chunk_step(const DevTables& t, const float* yin, float* yout, const uint8_t* code, int front,
                             int depth, int block, hipStream_t s) {
    return dispatch_depth<RunChunkStep>(depth, t, yin, yout, code, front, block, s);
}

hipError_t launch_persist(const PersistArgs& a, hipStream_t s) { return dispatch_depth<RunPersist>(a.depth, a, s); }

hipError_t launch_far_sum(const DevTables& t, const float* y, float* det_mass, uint32_t* det_reached,
                          hipStream_t s) {
    hipLaunchKernelGGL(k_far_acc, dim3(1), dim3(256), 0, s, t, y, det_mass, det_reached);
    return hipGetLastError();
}

hipError_t launch_export(const DevTables& t, const float* y, const uint8_t* code, const float* det_mass,
                         const uint32_t* det_reached, float* x_out, uint8_t* reach_out, hipStream_t s) {
    const int grid = (int)std::min<int64_t>((t.N + 1 + 255) / 256, 65536);
    hipLaunchKernelGGL(k_export, dim3(grid), dim3(256), 0, s, t, y, code, det_mass, det_reached, x_out, reach_out);
    return hipGetLastError();
}

hipError_t launch_count(const uint8_t* perc, int64_t n, unsigned long long* count, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int grid = (int)std::min<int64_t>((n + 255) / 256, 1024);
    hipLaunchKernelGGL(k_count, dim3(grid), dim3(256), 0, s, perc, n, count);
    return hipGetLastError();
}

}  // namespace perc
