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
                // LDS word of the contact: column 1 + its place in the staged range; a
                // missing contact reads row 0 of the zero pad column 0 (one address for
                // all of them, so such reads broadcast)
                d.contact[(size_t)i * C + c] = col < C ? (uint32_t)ring_word(dcp1, col - hs + 1) : 0u;
            }
    }
    // The one-step walks read the table as two 16-bit LDS word offsets per word (contacts
    // 2j and 2j + 1 of a column in word j): half the loads per work item. Every fiber the
    // walks accept has a halo range of at most 2,048 columns (two per thread of a
    // 1,024-thread workgroup), whose offsets stay below 21,000 words; wider cross-sections
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
                d.contact_whole[(size_t)i * C + c] = col < C ? (uint32_t)ring_word(dcp1, col + 1) : 0u;
            }
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
                        col < C ? (uint32_t)ring_word(dcp1, col - os + 1) : 0u;
                }
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
