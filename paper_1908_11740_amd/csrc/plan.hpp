// Host-side planning of the join's work lists: the capacity bounds the
// workspace is sized from, the check of a finished classification (debug
// mode) and the autotuner cache's line format.  Plain C++ without HIP, so
// that the CPU tests compile it with the address and undefined-behaviour
// sanitizers and check the bounds against an independent walk of the
// classification's cutting rule.
#pragma once

#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <utility>
#include <vector>

namespace sj {
namespace plan {

// The cutting rule of the small tiles' span units (see k_classify): runs of
// consecutive tiles in blocked order whose entry counts are at most
// small_cap, cut where the run's running entry count crosses a multiple of
// unit_cap, at every multiple of unit_tiles within a classification chunk of
// chunk_tiles tiles, at chunk starts and at every tile of more than
// small_cap entries.
struct SpanRules {
    int small_cap;
    int unit_cap;
    int unit_tiles;
    int64_t chunk_tiles;
};

// Upper bound on the span units of C tiles holding m entries (both sides).
// Per chunk: one run start at the chunk's first tile, one per multiple of
// unit_tiles, one per crossing of a multiple of unit_cap (at most
// weight / unit_cap), one after every cutting tile (at most
// m / (small_cap + 1) of them overall).
inline int64_t span_units_bound(int64_t C, int64_t m, const SpanRules& r) {
    const int64_t chunks = (C + r.chunk_tiles - 1) / r.chunk_tiles;
    return m / r.unit_cap + m / (r.small_cap + 1) + chunks * (r.chunk_tiles / r.unit_tiles + 2) + 1;
}

// Largest number of entries a span unit can hold: a run that stays below
// the next multiple of unit_cap, plus its last tile.
inline int64_t span_unit_max_entries(const SpanRules& r) {
    return (int64_t)r.unit_cap - 1 + r.small_cap;
}

// A span unit as k_classify writes it: (R start, NR, S start, NS) and
// (first blocked tile, tile count).
struct Unit {
    uint32_t r0, nr, s0, ns;
    uint32_t t0, tiles;
};

// Check span units against the partition's tile offsets (C + 1 per side):
// every unit lies inside the grid, its spans are exactly the offsets of its
// first and end tile, it holds at most max_entries entries and max_tiles
// tiles, none of its tiles has more than small_cap entries, it holds a
// tile with both lists non-empty, and no two units share a tile.  Returns
// -1 if all pass, else the index of a failing unit, with *why set.
inline int64_t check_units(const uint32_t* offR, const uint32_t* offS, int64_t C, const Unit* u,
                           int64_t n, int64_t max_entries, int max_tiles, int small_cap,
                           const char** why) {
    for (int64_t i = 0; i < n; ++i) {
        const Unit& x = u[i];
        const int64_t t0 = x.t0, te = (int64_t)x.t0 + x.tiles;
        if (x.tiles < 1 || te > C) { *why = "tile range outside the grid"; return i; }
        if ((int64_t)x.tiles > max_tiles) { *why = "too many tiles"; return i; }
        if (x.r0 != offR[t0] || x.nr != offR[te] - offR[t0] || x.s0 != offS[t0] ||
            x.ns != offS[te] - offS[t0]) {
            *why = "spans differ from the tile offsets";
            return i;
        }
        if ((int64_t)x.nr + x.ns > max_entries) { *why = "too many entries"; return i; }
        bool joinable = false;
        for (int64_t t = t0; t < te; ++t) {
            const uint32_t nr = offR[t + 1] - offR[t], ns = offS[t + 1] - offS[t];
            if ((int64_t)nr + ns > small_cap) { *why = "a tile above small_cap"; return i; }
            joinable = joinable || (nr && ns);
        }
        if (!joinable) { *why = "no joinable tile"; return i; }
    }
    // workgroups reserve their chunk's units in any order: sort by first tile
    std::vector<std::pair<uint32_t, int64_t>> by_tile((size_t)n);
    for (int64_t i = 0; i < n; ++i) by_tile[(size_t)i] = {u[i].t0, i};
    std::sort(by_tile.begin(), by_tile.end());
    for (size_t j = 1; j < by_tile.size(); ++j) {
        const Unit& a = u[by_tile[j - 1].second];
        if ((int64_t)a.t0 + a.tiles > (int64_t)by_tile[j].first) {
            *why = "units share a tile";
            return by_tile[j].second;
        }
    }
    return -1;
}

// One line of the autotuner cache file:
//   arch k log2_mR log2_mS mode block small_cap med_cap split_tau ms
struct TuneLine {
    char arch[64];
    int k, lr, ls, mode, block, small_cap, med_cap, split_tau;
    double ms;
};

inline void format_tune_line(const TuneLine& t, char* out, size_t cap) {
    std::snprintf(out, cap, "%s %d %d %d %d %d %d %d %d %.6f\n", t.arch, t.k, t.lr, t.ls, t.mode,
                  t.block, t.small_cap, t.med_cap, t.split_tau, t.ms);
}

// 1: a valid entry in *t; 0: a comment or blank line; -1: malformed.
inline int parse_tune_line(const char* line, int k_max, TuneLine* t) {
    while (*line == ' ' || *line == '\t') ++line;
    if (*line == '#' || *line == '\n' || *line == '\r' || *line == '\0') return 0;
    TuneLine x{};
    char tail[2];
    const int got = std::sscanf(line, "%63s %d %d %d %d %d %d %d %d %lf %1s", x.arch, &x.k, &x.lr,
                                &x.ls, &x.mode, &x.block, &x.small_cap, &x.med_cap, &x.split_tau,
                                &x.ms, tail);
    if (got != 10) return -1;
    if (x.block != 64 && x.block != 128 && x.block != 256 && x.block != 512) return -1;
    if (x.small_cap < 2 || x.med_cap < 2 || x.split_tau < 0 || x.k < 1 || x.k > k_max) return -1;
    if (x.lr < 0 || x.lr > 62 || x.ls < 0 || x.ls > 62 || x.mode < 0 || x.mode > 15) return -1;
    *t = x;
    return 1;
}

}  // namespace plan
}  // namespace sj
