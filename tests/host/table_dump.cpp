// Prints the host-built tables of the tile walks of hex radius W (argv[1]) for the
// table tests: C ntile lane_stride, then per tile "ts te hs he", the lane map, the packed
// one-step contact table by lane, the side-contact list (column << 2 | dcell + 1, column
// C for a missing contact), then the whole-cross-section lane map and table (or 0).
#include <cstdio>
#include <cstdlib>

#include "perc_internal.hpp"

int main(int argc, char** argv) {
    if (argc < 2) return 2;
    std::string err;
    auto cs = perc::column_set(std::atoi(argv[1]), err);
    if (!cs) { std::fprintf(stderr, "%s\n", err.c_str()); return 1; }
    std::printf("%d %d %d\n", cs->C, cs->ntile, cs->lane_stride);
    for (int k = 0; k < cs->ntile; ++k)
        std::printf("%d %d %d %d\n", cs->tile[k * 4], cs->tile[k * 4 + 1], cs->tile[k * 4 + 2], cs->tile[k * 4 + 3]);
    for (uint16_t v : cs->lanes) std::printf("%u\n", (unsigned)v);
    for (uint32_t v : cs->contact) std::printf("%u\n", v);
    for (int32_t v : cs->nb) std::printf("%d\n", v);
    std::printf("%d\n", cs->contact_whole16.empty() ? 0 : cs->lane_stride_whole);
    for (uint16_t v : cs->lanes_whole) std::printf("%u\n", (unsigned)v);
    for (uint32_t v : cs->contact_whole16) std::printf("%u\n", v);
    return 0;
}
