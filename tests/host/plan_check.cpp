// CPU check of the library's host-side planning (paper_1908_11740_amd/csrc/
// plan.hpp), built with the address and undefined-behaviour sanitizers by
// tests/test_host_sanitizers.py.
//
// An independent sequential walk of the span-unit cutting rule (the rule
// k_classify applies in parallel) builds the units of random tile layouts;
// the walk's unit count must stay within span_units_bound (the capacity the
// library allocates), every unit must pass check_units, and planted faults
// in the units must be caught.  The autotuner cache lines must round-trip
// and malformed lines must be rejected.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <string>
#include <vector>

#include "../../paper_1908_11740_amd/csrc/plan.hpp"

using namespace sj::plan;

static int failures = 0;
#define CHECK(c)                                                           \
    do {                                                                   \
        if (!(c)) {                                                        \
            std::fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #c); \
            ++failures;                                                    \
        }                                                                  \
    } while (0)

// The cutting rule, tile by tile: a tile of more than small_cap entries
// belongs to no unit and ends the current one; a new unit begins at the
// first tile of a chunk, after a cutting tile, at every multiple of
// unit_tiles within the chunk, and where the chunk's running entry count of
// run tiles reaches a new multiple of unit_cap.  Units without a tile whose
// two lists are both non-empty are dropped.
static std::vector<Unit> walk_units(const std::vector<uint32_t>& offR, const std::vector<uint32_t>& offS,
                                    int64_t C, const SpanRules& r) {
    std::vector<Unit> units;
    for (int64_t c0 = 0; c0 < C; c0 += r.chunk_tiles) {
        const int64_t c1 = std::min<int64_t>(C, c0 + r.chunk_tiles);
        int64_t run_weight = 0;     // entries of run tiles before t in this chunk
        int64_t start = -1;         // first tile of the open unit
        bool joinable = false;
        auto close = [&](int64_t end) {
            if (start >= 0 && joinable)
                units.push_back(Unit{offR[start], offR[end] - offR[start], offS[start],
                                     offS[end] - offS[start], (uint32_t)start,
                                     (uint32_t)(end - start)});
            start = -1;
            joinable = false;
        };
        bool prev_cut = true;
        int64_t prev_weight_before = 0;
        for (int64_t t = c0; t < c1; ++t) {
            const uint32_t nr = offR[t + 1] - offR[t], ns = offS[t + 1] - offS[t];
            const bool cut = (int64_t)nr + ns > r.small_cap;
            if (cut) {
                close(t);
                prev_cut = true;
                continue;
            }
            const int64_t tl = t - c0;
            const bool begins = tl == 0 || prev_cut || tl % r.unit_tiles == 0 ||
                                run_weight / r.unit_cap != prev_weight_before / r.unit_cap;
            if (begins) {
                close(t);
                start = t;
            }
            joinable = joinable || (nr && ns);
            prev_cut = false;
            prev_weight_before = run_weight;
            run_weight += nr + ns;
        }
        close(c1);
    }
    return units;
}

// Offsets of C tiles whose counts come from gen(rng).
template <class G>
static void layout(int64_t C, std::mt19937_64& rng, G gen, std::vector<uint32_t>& offR,
                   std::vector<uint32_t>& offS) {
    offR.assign((size_t)C + 1, 0);
    offS.assign((size_t)C + 1, 0);
    for (int64_t t = 0; t < C; ++t) {
        uint32_t nr, ns;
        gen(rng, nr, ns);
        offR[t + 1] = offR[t] + nr;
        offS[t + 1] = offS[t] + ns;
    }
}

static void check_layout(const char* name, int64_t C, const std::vector<uint32_t>& offR,
                         const std::vector<uint32_t>& offS, const SpanRules& r) {
    const std::vector<Unit> u = walk_units(offR, offS, C, r);
    const int64_t m = (int64_t)offR[C] + offS[C];
    const int64_t bound = span_units_bound(C, m, r);
    const char* why = "";
    const int64_t bad = check_units(offR.data(), offS.data(), C, u.data(), (int64_t)u.size(),
                                    span_unit_max_entries(r), r.unit_tiles, r.small_cap, &why);
    std::printf("%-28s C=%-8lld m=%-9lld units=%-7zu bound=%lld\n", name, (long long)C,
                (long long)m, u.size(), (long long)bound);
    CHECK((int64_t)u.size() <= bound);
    if (bad >= 0) std::fprintf(stderr, "%s: unit %lld: %s\n", name, (long long)bad, why);
    CHECK(bad < 0);
    if (u.size() < 2) return;
    // planted faults are caught
    std::vector<Unit> v = u;
    v[v.size() / 2].nr += 1;
    CHECK(check_units(offR.data(), offS.data(), C, v.data(), (int64_t)v.size(),
                      span_unit_max_entries(r), r.unit_tiles, r.small_cap, &why) >= 0);
    v = u;
    v[1].t0 = v[0].t0;  // two units on the same tiles
    v[1].tiles = v[0].tiles;
    v[1].r0 = v[0].r0, v[1].nr = v[0].nr, v[1].s0 = v[0].s0, v[1].ns = v[0].ns;
    CHECK(check_units(offR.data(), offS.data(), C, v.data(), (int64_t)v.size(),
                      span_unit_max_entries(r), r.unit_tiles, r.small_cap, &why) >= 0);
    v = u;
    v.back().tiles = (uint32_t)(C - v.back().t0 + 1);  // past the grid
    CHECK(check_units(offR.data(), offS.data(), C, v.data(), (int64_t)v.size(),
                      span_unit_max_entries(r), r.unit_tiles, r.small_cap, &why) >= 0);
}

static void tune_lines() {
    TuneLine t{};
    std::snprintf(t.arch, sizeof(t.arch), "gfx950");
    t.k = 1411, t.lr = 24, t.ls = 23, t.mode = 1, t.block = 256, t.small_cap = 256;
    t.med_cap = 2048, t.split_tau = 637, t.ms = 0.9209;
    char line[256];
    format_tune_line(t, line, sizeof(line));
    TuneLine u{};
    CHECK(parse_tune_line(line, 8192, &u) == 1);
    CHECK(std::strcmp(u.arch, "gfx950") == 0 && u.k == 1411 && u.lr == 24 && u.ls == 23 &&
          u.mode == 1 && u.block == 256 && u.small_cap == 256 && u.med_cap == 2048 &&
          u.split_tau == 637 && u.ms > 0.92 && u.ms < 0.9210);
    CHECK(parse_tune_line("# comment\n", 8192, &u) == 0);
    CHECK(parse_tune_line("   \n", 8192, &u) == 0);
    const char* bad[] = {"gfx950 12 x\n", "gfx950 1 2 3 0 100 256 1024 0 1.0\n",
                         "gfx950 9000 2 3 0 256 256 1024 0 1.0\n",
                         "gfx950 64 2 3 0 256 1 1024 0 1.0\n",
                         "gfx950 64 2 3 0 256 256 1024 0 1.0 extra\n",
                         "gfx950 64 2 3 16 256 256 1024 0 1.0\n"};
    for (const char* b : bad) CHECK(parse_tune_line(b, 8192, &u) == -1);
    // an over-long architecture name is cut at 63 characters, not overflowed
    std::string longname(200, 'g');
    CHECK(parse_tune_line((longname + " 64 2 3 0 256 256 1024 0 1.0\n").c_str(), 8192, &u) == -1);
}

int main() {
    std::mt19937_64 rng(2024);
    const SpanRules rules[] = {{256, 768, 255, 4096}, {128, 896, 63, 4096}, {512, 1536, 511, 4096},
                               {256, 256, 127, 4096}};
    for (const SpanRules& r : rules) {
        std::vector<uint32_t> offR, offS;
        // sparse: mostly empty and one-sided tiles
        layout(50000, rng, [](std::mt19937_64& g, uint32_t& a, uint32_t& b) {
            std::poisson_distribution<int> p(0.7);
            a = p(g), b = p(g);
        }, offR, offS);
        check_layout("sparse", 50000, offR, offS, r);
        // clustered: heavy-tailed counts with tiles above small_cap
        layout(30001, rng, [&r](std::mt19937_64& g, uint32_t& a, uint32_t& b) {
            std::lognormal_distribution<double> ln(2.0, 1.4);
            a = (uint32_t)std::min(ln(g), 3.0 * r.small_cap);
            b = (uint32_t)std::min(ln(g), 3.0 * r.small_cap);
        }, offR, offS);
        check_layout("heavy-tailed", 30001, offR, offS, r);
        // every tile just below small_cap: one tile per unit at most a few
        layout(9000, rng, [&r](std::mt19937_64& g, uint32_t& a, uint32_t& b) {
            a = (uint32_t)(r.small_cap / 2), b = (uint32_t)(r.small_cap - r.small_cap / 2 - (g() & 1));
        }, offR, offS);
        check_layout("full tiles", 9000, offR, offS, r);
        // one-sided only: no units at all
        layout(5000, rng, [](std::mt19937_64& g, uint32_t& a, uint32_t& b) {
            a = (uint32_t)(g() % 5), b = 0;
        }, offR, offS);
        check_layout("one-sided", 5000, offR, offS, r);
        // a partial last chunk and a one-tile grid
        layout(4097, rng, [](std::mt19937_64& g, uint32_t& a, uint32_t& b) {
            a = 1 + (uint32_t)(g() % 3), b = 1 + (uint32_t)(g() % 3);
        }, offR, offS);
        check_layout("partial chunk", 4097, offR, offS, r);
        layout(1, rng, [](std::mt19937_64&, uint32_t& a, uint32_t& b) { a = 3, b = 4; }, offR, offS);
        check_layout("one tile", 1, offR, offS, r);
    }
    tune_lines();
    if (failures) {
        std::fprintf(stderr, "%d check(s) failed\n", failures);
        return 1;
    }
    std::printf("plan checks passed\n");
    return 0;
}
