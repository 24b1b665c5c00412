// CPU check of the row-sweep strip table (lb_strip_table.h), built with g++.
// Reads geometries from stdin ("count mode", then "nx ny x_in tube_len tube_h
// y0 active" per line; mode 0 checks one table of all of them, mode 1 a table
// of each one alone) and prints one line per property checked, "name value".
#include <algorithm>
#include <cstdio>
#include <map>
#include <tuple>
#include <vector>

#include "lb_strip_table.h"

using lbk::StripDev;

static bool solid(const lb_geometry& g, int x, int y) {
    return g.tube_len > 0 && x >= g.x_in && x < g.x_in + g.tube_len && (y < g.y0 || y >= g.y0 + g.tube_h);
}

struct Counts {
    long long bad_bounds = 0, bad_align32 = 0, twice = 0, missed = 0, inactive = 0, bad_parity = 0, bad_xcd = 0;
    long long over_capacity = 0, max_extra = 0;
};

static void check(const std::vector<lb_geometry>& G, const std::vector<int>& active, Counts& r) {
    const int n = (int)G.size();
    long long &bad_bounds = r.bad_bounds, &bad_align32 = r.bad_align32, &twice = r.twice, &missed = r.missed;
    long long &inactive = r.inactive, &bad_parity = r.bad_parity, &bad_xcd = r.bad_xcd;
    long long &over_capacity = r.over_capacity, &max_extra = r.max_extra;
    for (int width : {62, 192}) {
        // the capacity the library allocates (every capillary active)
        const int cap_count = lbk::strip_capacity(G, width);
        for (int chunk : {0, 4, 5, 6, 8, 11, 12, 16, 24, 32, 4096}) {
            std::vector<StripDev> S;
            int count = -1, xcd[9];
            lbk::build_strips(G, active, chunk, width, 2, &S, &count, xcd);
            if (count != (int)S.size() || xcd[0] != 0 || xcd[8] != count) ++bad_xcd;
            for (int x = 0; x < 8; ++x) bad_xcd += xcd[x] > xcd[x + 1];
            over_capacity += count > cap_count;
            std::vector<std::vector<unsigned char>> cov(n);
            for (int k = 0; k < n; ++k) cov[k].assign((size_t)G[k].nx * G[k].ny, 0);
            // strips of one column (cap, xs, xe), for the row parity of the chunk starts
            std::map<std::tuple<int, int, int>, std::vector<std::pair<int, int>>> cols;
            for (const StripDev& s : S) {
                if (s.cap < 0 || s.cap >= n) { ++bad_bounds; continue; }
                const lb_geometry& g = G[s.cap];
                if (!active[s.cap]) ++inactive;
                if (s.xs < 0 || s.xe > g.nx || s.xe <= s.xs || s.xe - s.xs > width || s.ya < 0 || s.yb > g.ny ||
                    s.yb <= s.ya) {
                    ++bad_bounds;
                    continue;
                }
                if (width == 192 && s.xs % 32 != 0) ++bad_align32;
                cols[{s.cap, s.xs, s.xe}].push_back({s.ya, s.yb});
                for (int y = s.ya; y < s.yb; ++y)
                    for (int x = s.xs; x < s.xe; ++x) ++cov[s.cap][(size_t)y * g.nx + x];
            }
            // chunks of a column start an even number of rows after the column's first row
            for (auto& kv : cols) {
                auto& v = kv.second;
                std::sort(v.begin(), v.end());
                int start = v[0].first, prev_end = v[0].first;
                for (auto& r : v) {
                    if (r.first != prev_end) start = r.first;   // a new column of this (cap, xs, xe)
                    if ((r.first - start) % 2 != 0) ++bad_parity;
                    prev_end = r.second;
                }
            }
            for (int k = 0; k < n; ++k) {
                if (!active[k]) continue;
                const lb_geometry& g = G[k];
                long long extra = 0;
                for (int y = 0; y < g.ny; ++y)
                    for (int x = 0; x < g.nx; ++x) {
                        const int c = cov[k][(size_t)y * g.nx + x];
                        twice += c > 1;
                        if (solid(g, x, y)) extra += c;
                        else missed += c != 1;
                    }
                // solid nodes swept, at each end of the tube (one longer than a strip):
                // one wall row over the strip's width (odd tube heights), and up to 31
                // tube columns of every wall row (the cut is rounded to 32 columns)
                const long long walls = g.tube_len > 0 ? g.ny - g.tube_h : 0;
                max_extra = std::max(max_extra, extra - 2LL * (width + 31LL * walls));
            }
        }
    }
}

int main() {
    int n = 0, mode = 0;
    if (std::scanf("%d %d", &n, &mode) != 2 || n <= 0) return 2;
    std::vector<lb_geometry> G(n);
    std::vector<int> active(n);
    for (int k = 0; k < n; ++k) {
        lb_geometry g{};
        if (std::scanf("%d %d %d %d %d %d %d", &g.nx, &g.ny, &g.x_in, &g.tube_len, &g.tube_h, &g.y0, &active[k]) != 7)
            return 2;
        G[k] = g;
    }
    Counts r;
    if (mode == 0) {
        check(G, active, r);
    } else {
        for (int k = 0; k < n; ++k) check({G[k]}, {active[k]}, r);
    }
    std::printf("bad_bounds %lld\nbad_align32 %lld\ntwice %lld\nmissed %lld\ninactive %lld\n", r.bad_bounds,
                r.bad_align32, r.twice, r.missed, r.inactive);
    std::printf("bad_parity %lld\nbad_xcd %lld\nover_capacity %lld\nmax_extra_solid %lld\n", r.bad_parity,
                r.bad_xcd, r.over_capacity, r.max_extra);
    return 0;
}
