// Lattice descriptor of the modified FCC fiber (Sec. II.A, Fig. 1): hexagonal
// cross-section of hex radius W (unit = distance between neighbouring tube axes),
// L (111) layers stacked ABC along the fiber axis, 12 side contacts (FCC nearest
// neighbours) and 2 end contacts (the next tube of the same column) per tube.
#include <algorithm>
#include <cstdlib>
#include <map>

#include "perc_internal.hpp"

namespace perc {

namespace {

int hexdist(int q, int r) { return std::max({std::abs(q), std::abs(r), std::abs(q + r)}); }
int mod3(int v) { return ((v % 3) + 3) % 3; }

// Side contacts as (dq, dr, dk): the 6 in-layer neighbours at distance sqrt(3) tube
// spacings, then the 3 of the layer above and the 3 of the layer below, whose axes are
// one tube spacing away in projection (one layer = sqrt(2) spacings along the axis).
constexpr int kSideOff[kSide][3] = {
    {1, 1, 0}, {2, -1, 0}, {1, -2, 0}, {-1, -1, 0}, {-2, 1, 0}, {-1, 2, 0},
    {1, 0, 1}, {-1, 1, 1}, {0, -1, 1},
    {0, 1, -1}, {-1, 0, -1}, {1, -1, -1},
};

// Missing contacts read a word of the ring's zero pad block (block 0). t[0 .. n) are
// the table words of one contact direction for the lanes of one workgroup in order
// (lane l reads t[l]; lanes n and beyond, up to the next multiple of 64, read t[0]), with
// kMissing where the contact is missing. The ring's row offsets are multiples of 64
// words, so a word's bank is its index mod 64 (mod 32 where LDS serves a wave in two
// halves) in every row. Each missing contact gets the pad word of row 1 in a bank that no
// real contact of the lanes of its wave (64 lanes) and half-wave (32 lanes) reads, where
// one is free in both, else one free in the half-wave; the missing contacts of one
// half-wave share that word (one address: a broadcast).
constexpr uint32_t kMissing = 0xffffffffu;
void place_pads(uint32_t* t, int n) {
    for (int w0 = 0; w0 < n; w0 += 64) {
        const int w1 = std::min(n, w0 + 64);
        const bool dup = w1 - w0 < 64 && w0 > 0;  // lanes n.. of this wave read t[0]
        uint64_t used64 = 0;
        for (int l = w0; l < w1; ++l)
            if (t[l] != kMissing) used64 |= 1ull << (t[l] % 64);
        if (dup && t[0] != kMissing) used64 |= 1ull << (t[0] % 64);
        for (int h0 = w0; h0 < w0 + 64 && h0 < n; h0 += 32) {
            const int h1 = std::min(n, h0 + 32);
            uint32_t used32 = 0;
            bool pads = false;
            for (int l = h0; l < h1; ++l) {
                if (t[l] != kMissing) used32 |= 1u << (t[l] % 32);
                else pads = true;
            }
            if (h1 - h0 < 32 && dup && t[0] != kMissing) used32 |= 1u << (t[0] % 32);
            if (!pads) continue;
            int b = -1;
            for (int c = 0; c < 64 && b < 0; ++c)
                if (!((used64 >> c) & 1u) && !((used32 >> (c % 32)) & 1u)) b = c;
            for (int c = 0; c < 32 && b < 0; ++c)
                if (!((used32 >> c) & 1u)) b = c;
            if (b < 0) b = 0;
            for (int l = h0; l < h1; ++l)
                if (t[l] == kMissing) t[l] = (uint32_t)ring_word(1, b);
        }
    }
}

std::shared_ptr<ColumnSet> build_columns(int32_t W) {
    auto cs = std::make_shared<ColumnSet>();
    ColumnSet& d = *cs;
    d.W = W;
    // internal column order: (q, r) lexicographic, so that every contact of a column
    // lies within two q-rows of it
    for (int q = -W; q <= W; ++q)
        for (int r = -W; r <= W; ++r)
            if (hexdist(q, r) <= W) { d.q.push_back(q); d.r.push_back(r); d.sig.push_back(mod3(q - r)); }
    const int C = (int)d.q.size();
    d.C = C;
    d.CP = std::max(32, ((C + 31) / 32) * 32);
    // canonical rank: (sigma, q, r) order inside a cell = lexicographic (k, q, r) overall
    std::vector<int32_t> by_canon(C);
    for (int c = 0; c < C; ++c) by_canon[c] = c;
    std::stable_sort(by_canon.begin(), by_canon.end(), [&](int a, int b) {
        if (d.sig[a] != d.sig[b]) return d.sig[a] < d.sig[b];
        if (d.q[a] != d.q[b]) return d.q[a] < d.q[b];
        return d.r[a] < d.r[b];
    });
    d.rank.assign(C, 0);
    d.by_rank = by_canon;
    for (int k = 0; k < C; ++k) d.rank[by_canon[k]] = k;
    for (int c = 0; c < C; ++c) d.nsig[d.sig[c]]++;
    const int S = 2 * W + 1;
    std::vector<int32_t> index((size_t)S * S, -1);
    for (int c = 0; c < C; ++c) index[(size_t)(d.q[c] + W) * S + (d.r[c] + W)] = c;
    d.nb.assign((size_t)kSide * C, 0);
    for (int c = 0; c < C; ++c) {
        for (int i = 0; i < kSide; ++i) {
            const int q2 = d.q[c] + kSideOff[i][0], r2 = d.r[c] + kSideOff[i][1];
            const int s2 = d.sig[c] + kSideOff[i][2];  // in -1..3
            const int dcell = s2 < 0 ? -1 : (s2 > 2 ? 1 : 0);
            int col = C, dc = 0;  // outside the hexagon: no tube
            if (hexdist(q2, r2) <= W) {
                col = index[(size_t)(q2 + W) * S + (r2 + W)];
                dc = dcell;
            }
            d.nb[(size_t)i * C + c] = (col << 2) | (dc + 1);
        }
    }
    // column tiles of about kTileCols columns, each with the range of columns its
    // contacts reach (the halo)
    const int nt = std::max(1, (C + kTileCols - 1) / kTileCols);
    d.ntile = nt;
    d.tile.assign((size_t)nt * 4, 0);
    d.span_max = 0;
    d.tile_max = 0;
    for (int k = 0; k < nt; ++k) {
        const int ts = (int)((int64_t)C * k / nt), te = (int)((int64_t)C * (k + 1) / nt);
        int hs = ts, he = te;
        for (int c = ts; c < te; ++c)
            for (int i = 0; i < kSide; ++i) {
                const int col = d.nb[(size_t)i * C + c] >> 2;
                if (col < C) { hs = std::min(hs, col); he = std::max(he, col + 1); }
            }
        d.tile[(size_t)k * 4 + 0] = ts; d.tile[(size_t)k * 4 + 1] = te;
        d.tile[(size_t)k * 4 + 2] = hs; d.tile[(size_t)k * 4 + 3] = he;
        d.span_max = std::max(d.span_max, he - hs);
        d.tile_max = std::max(d.tile_max, te - ts);
    }
    // contact table: LDS word of each side contact within its tile's staged range
    d.contact.assign((size_t)kSide * C, 0u);
    for (int k = 0; k < nt; ++k) {
        const int ts = d.tile[k * 4 + 0], te = d.tile[k * 4 + 1];
        const int hs = d.tile[k * 4 + 2];
        for (int c = ts; c < te; ++c)
            for (int i = 0; i < kSide; ++i) {
                const int32_t v = d.nb[(size_t)i * C + c];
                const int32_t col = v >> 2, dcp1 = v & 3;  // dcell + 1
                // LDS word of the contact: column kPadCols + its place in the staged range
                d.contact[(size_t)i * C + c] = col < C ? (uint32_t)ring_word(dcp1, col - hs + kPadCols) : kMissing;
            }
        for (int i = 0; i < kSide; ++i) place_pads(&d.contact[(size_t)i * C + ts], te - ts);
    }
    // The one-step walks read the table as two 16-bit LDS word offsets per word (contacts
    // 2j and 2j + 1 of a column in word j): half the loads per work item. Every fiber the
    // walks accept has a halo range of at most 2,048 columns (two per thread of a
    // 1,024-thread workgroup), whose offsets stay below 21,200 words; wider cross-sections
    // are refused before any launch, so their (truncated) packed words are never read.
    auto pack16 = [C](const std::vector<uint32_t>& t) {
        std::vector<uint32_t> p((size_t)(kSide / 2) * C);
        for (int j = 0; j < kSide / 2; ++j)
            for (int c = 0; c < C; ++c)
                p[(size_t)j * C + c] =
                    (t[(size_t)(2 * j) * C + c] & 0xffffu) | ((t[(size_t)(2 * j + 1) * C + c] & 0xffffu) << 16);
        return p;
    };
    d.contact = pack16(d.contact);
    // outer ranges: every column a halo-range column contacts
    d.tile2.assign((size_t)nt * 2, 0);
    d.span2_max = 0;
    for (int k = 0; k < nt; ++k) {
        const int hs = d.tile[k * 4 + 2], he = d.tile[k * 4 + 3];
        int os = hs, oe = he;
        for (int c = hs; c < he; ++c)
            for (int i = 0; i < kSide; ++i) {
                const int col = d.nb[(size_t)i * C + c] >> 2;
                if (col < C) { os = std::min(os, col); oe = std::max(oe, col + 1); }
            }
        d.tile2[(size_t)k * 2 + 0] = os;
        d.tile2[(size_t)k * 2 + 1] = oe;
        d.span2_max = std::max(d.span2_max, oe - os);
    }
    if (C <= kWholeCols) {
        d.contact_whole.assign((size_t)kSide * C, 0u);
        for (int c = 0; c < C; ++c)
            for (int i = 0; i < kSide; ++i) {
                const int32_t v = d.nb[(size_t)i * C + c];
                const int32_t col = v >> 2, dcp1 = v & 3;
                d.contact_whole[(size_t)i * C + c] = col < C ? (uint32_t)ring_word(dcp1, col + kPadCols) : kMissing;
            }
        for (int i = 0; i < kSide; ++i) place_pads(&d.contact_whole[(size_t)i * C], C);
        d.contact_whole16 = pack16(d.contact_whole);
    }
    if (d.span_max <= kMaxSpan2 && d.span2_max <= kMaxSpan2) {
        const size_t sm = (size_t)d.span_max;
        d.contact2.assign((size_t)nt * kSide * sm, 0u);
        for (int k = 0; k < nt; ++k) {
            const int hs = d.tile[k * 4 + 2], he = d.tile[k * 4 + 3], os = d.tile2[k * 2];
            for (int c = hs; c < he; ++c)
                for (int i = 0; i < kSide; ++i) {
                    const int32_t v = d.nb[(size_t)i * C + c];
                    const int32_t col = v >> 2, dcp1 = v & 3;
                    d.contact2[((size_t)k * kSide + i) * sm + (size_t)(c - hs)] =
                        col < C ? (uint32_t)ring_word(dcp1, col - os + kPadCols) : kMissing;
                }
            for (int i = 0; i < kSide; ++i) place_pads(&d.contact2[((size_t)k * kSide + i) * sm], he - hs);
        }
    }
    return cs;
}

std::mutex g_cols_mu;
std::map<int32_t, std::shared_ptr<const ColumnSet>> g_cols;

}  // namespace

std::shared_ptr<const ColumnSet> column_set(int32_t W, std::string& err) {
    if (W < 0 || W > 1024) { err = "W must be in [0, 1024]"; return nullptr; }
    std::lock_guard<std::mutex> g(g_cols_mu);
    auto it = g_cols.find(W);
    if (it != g_cols.end()) return it->second;
    std::shared_ptr<const ColumnSet> cs = build_columns(W);
    g_cols.emplace(W, cs);
    return cs;
}

bool build_lattice(int32_t W, int32_t L, LatticeDesc& d, std::string& err) {
    if (W < 0 || W > 1024) { err = "W must be in [0, 1024]"; return false; }
    // L < 2^16 keeps the sampler's stream tag (W << 16) | L distinct for every shape
    if (L < 1 || L > 65535) { err = "L must be in [1, 65535]"; return false; }
    d = LatticeDesc{};
    d.cs = column_set(W, err);
    if (!d.cs) return false;
    const ColumnSet& cs = *d.cs;
    d.W = W; d.L = L;
    d.C = cs.C; d.CP = cs.CP;
    d.ntile = cs.ntile; d.span_max = cs.span_max; d.tile_max = cs.tile_max;
    d.U = (L + 2) / 3;
    // sites: every column of every full cell, then the columns of the last cell whose
    // layer exists (a prefix in canonical rank: sigma < L - 3 (U - 1))
    const int k_last = 3 * (d.U - 1);
    int64_t n = (int64_t)(d.U - 1) * d.C;
    for (int sg = 0; sg < 3; ++sg)
        if (k_last + sg < L) n += cs.nsig[sg];
    d.N = n;
    d.words = (n + 31) / 32;
    if (n > (int64_t)INT32_MAX) { err = "lattice exceeds 2^31 - 1 sites"; return false; }
    // state arrays are indexed with 32-bit offsets inside one configuration
    if (state_words(d) > (int64_t)INT32_MAX) { err = "lattice state exceeds 2^31 - 1 words"; return false; }
    return true;
}

}  // namespace perc
