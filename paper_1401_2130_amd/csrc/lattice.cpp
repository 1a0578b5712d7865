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

// Contact tables are built column by column with kMissing for a missing contact, then
// laid out for the lanes that read them (the LDS bank rules are with ring_word).
constexpr uint32_t kMissing = 0xffffffffu;
constexpr int kHalf = 32;  // lanes of a half-wave = LDS banks

// Lanes of the walk of the tile [ts, te) over at most B lanes: column ts + lanes[l] on
// lane l. tab[i * C + c] is the LDS word of contact i of column c (kMissing: none).
// Columns go to lanes in order; a column whose real contacts would add a second word to
// a bank of its half-wave (for the same direction) waits behind an idle lane that
// repeats the previous column (the repeat reads the same words), while the budget leaves
// room for the remaining columns. Lanes after the last column repeat it.
std::vector<uint16_t> lane_map(const std::vector<uint32_t>& tab, int C, int ts, int te, int B) {
    std::vector<uint16_t> lanes;
    lanes.reserve((size_t)B);
    uint32_t word[kSide][kHalf];
    for (int c = ts; c < te;) {
        const int l = (int)lanes.size();
        if (l % kHalf == 0)
            for (auto& row : word)
                for (uint32_t& w : row) w = kMissing;
        bool fits = true;
        for (int i = 0; i < kSide && fits; ++i) {
            const uint32_t a = tab[(size_t)i * C + c];
            if (a != kMissing && word[i][a % kHalf] != kMissing && word[i][a % kHalf] != a) fits = false;
        }
        if (fits || l % kHalf == 0 || l + 1 + (te - c) > B) {
            for (int i = 0; i < kSide; ++i) {
                const uint32_t a = tab[(size_t)i * C + c];
                if (a != kMissing) word[i][a % kHalf] = a;
            }
            lanes.push_back((uint16_t)(c - ts));
            ++c;
        } else {
            lanes.push_back(lanes.back());
        }
    }
    while ((int)lanes.size() < B) lanes.push_back(lanes.back());
    return lanes;
}

// Missing contacts of direction i (t: that direction's words by column, from column
// `base`; lane l reads column base + lanes[l]) get the pad word of row 1 in a bank that no
// real contact of their half-wave reads; the missing contacts of one half-wave share it
// (one address: a broadcast).
void place_pads(uint32_t* t, int base, const std::vector<uint16_t>& lanes) {
    const int n = (int)lanes.size();
    for (int h0 = 0; h0 < n; h0 += kHalf) {
        const int h1 = std::min(n, h0 + kHalf);
        uint32_t used = 0;
        bool pads = false;
        for (int l = h0; l < h1; ++l) {
            const uint32_t a = t[base + lanes[(size_t)l]];
            if (a != kMissing) used |= 1u << (a % kHalf);
            else pads = true;
        }
        if (!pads) continue;
        int b = 0;
        while (b < kHalf - 1 && ((used >> b) & 1u)) ++b;
        for (int l = h0; l < h1; ++l) {
            uint32_t& a = t[base + lanes[(size_t)l]];
            if (a == kMissing) a = (uint32_t)ring_word(1, b);
        }
    }
}

// Lanes 0 .. n-1 on columns 0 .. n-1 and the rest of the last wave on column 0 (the walks
// that stage a range give every surplus lane its first column).
std::vector<uint16_t> identity_lanes(int n) {
    std::vector<uint16_t> lanes((size_t)((n + 63) / 64) * 64, 0);
    for (int l = 0; l < n; ++l) lanes[(size_t)l] = (uint16_t)l;
    return lanes;
}

// The one-step walks read a table as two 16-bit LDS word offsets per word, by lane:
// word [j][k * B + l] holds contacts 2j (low 16 bits) and 2j + 1 of lane l of tile k (half
// the loads of one word per contact). Every fiber the walks accept has a halo range of at
// most 2,048 columns (two per thread of a 1,024-thread workgroup), whose offsets stay
// below 21,200 words; wider cross-sections are refused before any launch, so their
// (truncated) packed words are never read.
void pack_lanes(const std::vector<uint32_t>& tab, int C, int ts, const std::vector<uint16_t>& lanes, int k,
                int nt, std::vector<uint32_t>& out) {
    const size_t B = lanes.size(), stride = (size_t)nt * B;
    for (int j = 0; j < kSide / 2; ++j)
        for (size_t l = 0; l < B; ++l) {
            const int c = ts + lanes[l];
            out[(size_t)j * stride + (size_t)k * B + l] =
                (tab[(size_t)(2 * j) * C + c] & 0xffffu) | ((tab[(size_t)(2 * j + 1) * C + c] & 0xffffu) << 16);
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
    // (kPadCols + its place in the range), then the lanes of each tile and, by lane, the
    // packed table
    std::vector<uint32_t> tab((size_t)kSide * C, kMissing);
    d.lane_stride = ((d.tile_max + 63) / 64) * 64;
    d.lanes.assign((size_t)nt * d.lane_stride, 0);
    d.contact.assign((size_t)(kSide / 2) * nt * d.lane_stride, 0u);
    for (int k = 0; k < nt; ++k) {
        const int ts = d.tile[k * 4 + 0], te = d.tile[k * 4 + 1];
        const int hs = d.tile[k * 4 + 2];
        for (int c = ts; c < te; ++c)
            for (int i = 0; i < kSide; ++i) {
                const int32_t v = d.nb[(size_t)i * C + c];
                const int32_t col = v >> 2, dcp1 = v & 3;  // dcell + 1
                if (col < C) tab[(size_t)i * C + c] = (uint32_t)ring_word(dcp1, col - hs + kPadCols);
            }
        const std::vector<uint16_t> lanes = lane_map(tab, C, ts, te, d.lane_stride);
        for (int i = 0; i < kSide; ++i) place_pads(&tab[(size_t)i * C], ts, lanes);
        std::copy(lanes.begin(), lanes.end(), d.lanes.begin() + (size_t)k * d.lane_stride);
        pack_lanes(tab, C, ts, lanes, k, nt, d.contact);
    }
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
        std::vector<uint32_t> tw((size_t)kSide * C, kMissing);
        for (int c = 0; c < C; ++c)
            for (int i = 0; i < kSide; ++i) {
                const int32_t v = d.nb[(size_t)i * C + c];
                const int32_t col = v >> 2, dcp1 = v & 3;
                if (col < C) tw[(size_t)i * C + c] = (uint32_t)ring_word(dcp1, col + kPadCols);
            }
        // the two-step walks' first step reads it by column, one column per lane in order
        d.contact_whole = tw;
        const std::vector<uint16_t> ident = identity_lanes(C);
        for (int i = 0; i < kSide; ++i) place_pads(&d.contact_whole[(size_t)i * C], 0, ident);
        // the one-step walks (and the second step) by lane
        d.lane_stride_whole = ((C + 63) / 64) * 64;
        d.lanes_whole = lane_map(tw, C, 0, C, d.lane_stride_whole);
        for (int i = 0; i < kSide; ++i) place_pads(&tw[(size_t)i * C], 0, d.lanes_whole);
        d.contact_whole16.assign((size_t)(kSide / 2) * d.lane_stride_whole, 0u);
        pack_lanes(tw, C, 0, d.lanes_whole, 0, 1, d.contact_whole16);
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
            const std::vector<uint16_t> ident = identity_lanes(he - hs);
            for (int i = 0; i < kSide; ++i) place_pads(&d.contact2[((size_t)k * kSide + i) * sm], 0, ident);
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
