// Lattice descriptor of the modified FCC fiber (Sec. II.A, Fig. 1): hexagonal
// cross-section of hex radius W (unit = distance between neighbouring tube axes),
// L (111) layers stacked ABC along the fiber axis, 12 side contacts (FCC nearest
// neighbours) and 2 end contacts (the next tube of the same column) per tube.
#include <algorithm>
#include <cstdlib>

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

}  // namespace

bool build_lattice(int32_t W, int32_t L, LatticeDesc& d, std::string& err) {
    if (W < 0 || W > 1024) { err = "W must be in [0, 1024]"; return false; }
    if (L < 1 || L > (1 << 22)) { err = "L must be in [1, 4194304]"; return false; }
    d = LatticeDesc{};
    d.W = W; d.L = L;
    struct Col { int sig, q, r; };
    std::vector<Col> cols;
    for (int q = -W; q <= W; ++q)
        for (int r = -W; r <= W; ++r)
            if (hexdist(q, r) <= W) cols.push_back({mod3(q - r), q, r});
    std::sort(cols.begin(), cols.end(), [](const Col& a, const Col& b) {
        if (a.sig != b.sig) return a.sig < b.sig;
        if (a.q != b.q) return a.q < b.q;
        return a.r < b.r;
    });
    const int C = (int)cols.size();
    d.C = C;
    d.U = (L + 2) / 3;
    d.CP = ((C + 1 + 31) / 32) * 32;
    d.q.resize(C); d.r.resize(C); d.sig.resize(C); d.top.resize(C);
    const int S = 2 * W + 1;
    std::vector<int32_t> index((size_t)S * S, -1);
    for (int c = 0; c < C; ++c) {
        d.q[c] = cols[c].q; d.r[c] = cols[c].r; d.sig[c] = cols[c].sig;
        d.nsig[cols[c].sig]++;
        index[(size_t)(cols[c].q + W) * S + (cols[c].r + W)] = c;
        // far-end tube: the highest layer k < L with k = sig (mod 3)
        d.top[c] = cols[c].sig < L ? (L - 1 - cols[c].sig) / 3 : -1;
    }
    // sites: every column of every full cell, then the prefix of the last cell
    int64_t n = (int64_t)(d.U - 1) * C;
    const int k_last = 3 * (d.U - 1);
    for (int c = 0; c < C; ++c)
        if (k_last + d.sig[c] < L) ++n;
    d.N = n;
    d.words = (n + 31) / 32;
    if (n > (int64_t)INT32_MAX) { err = "lattice exceeds 2^31 - 1 sites"; return false; }
    d.nb.assign((size_t)kSide * C, 0);
    for (int c = 0; c < C; ++c) {
        for (int i = 0; i < kSide; ++i) {
            const int q2 = d.q[c] + kSideOff[i][0], r2 = d.r[c] + kSideOff[i][1];
            const int s2 = d.sig[c] + kSideOff[i][2];  // in -1..3
            const int dcell = s2 < 0 ? -1 : (s2 > 2 ? 1 : 0);
            int col = C, dc = 0;  // outside the hexagon: the zero pad column
            if (hexdist(q2, r2) <= W) {
                col = index[(size_t)(q2 + W) * S + (r2 + W)];
                dc = dcell;
            }
            d.nb[(size_t)i * C + c] = (col << 2) | (dc + 1);
        }
    }
    return true;
}

std::vector<uint32_t> contact_table(const LatticeDesc& d, int32_t depth) {
    const uint32_t SJ = (uint32_t)depth + 2u;
    std::vector<uint32_t> t((size_t)kSide * d.C);
    for (size_t e = 0; e < t.size(); ++e) {
        const int32_t v = d.nb[e];
        const uint32_t col = (uint32_t)(v >> 2), dcp1 = (uint32_t)(v & 3);  // dcell + 1
        t[e] = (col * SJ + dcp1) * 4u;
    }
    return t;
}

}  // namespace perc
