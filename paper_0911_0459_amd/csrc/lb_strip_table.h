// Strip table of the row-sweep kernels: the columns and rows that each
// workgroup sweeps.  Host code only, so that it also builds without HIP.
#pragma once
#include <algorithm>
#include <cstddef>
#include <vector>

#include "lbcap.h"

namespace lbk {

struct StripDev {
    int cap;
    int xs, xe;                   // output columns [xs, xe): at most 62, or 192 in a wide strip
    int ya, yb;                   // output rows [ya, yb), ya >= 0, yb <= ny
};

// Strips of `width` output columns (62 for one wavefront, 192 for a wide
// strip); a strip lying entirely in the tube section only covers the channel
// rows, and one that the tube enters or leaves covers the channel rows, with
// its wall rows in strips of their own over the reservoir columns.  chunk = 0
// keeps whole strips.
constexpr int LB_MIN_CHUNK = 4;   // smallest rows per strip chunk
constexpr size_t LB_STRIP_GROUP = 16;  // neighbouring strip columns listed chunk by chunk
constexpr int LB_TAIL_MIN_CHUNK = 12;  // chunks from this height on end each XCD run with short chunks
constexpr size_t LB_TAIL_COLS = 64;    // columns per XCD run whose last rows go to short chunks

// Strip table of the row-sweep kernels.  Every strip column (width output
// columns of one capillary, over the rows that hold fluid) is cut into
// ceil(rows / chunk) chunks of balanced height (no short remainder chunk, whose
// prologue would cost as much as a full chunk's).  The columns are dealt to the
// 8 XCDs in contiguous runs of about equal row count.  For chunks of
// LB_TAIL_MIN_CHUNK rows or more, the last 2 * small rows of the last
// LB_TAIL_COLS columns of each run are cut into chunks of small =
// max(4, chunk / 4) rows and listed at the end of the run, so that a step ends
// on short strips (a small tail) while most rows go through long strips (few
// prologues, little re-read at chunk edges).
// Within a run, groups of LB_STRIP_GROUP neighbouring columns are listed chunk
// by chunk across the group, so that strips sharing halo columns run at the
// same time, and the chunks of one column share an L2.
// The kernels' row loops are unrolled by align = 2 so that request buffers swap
// roles without copies, and the copies of a row's arithmetic may round
// differently: every chunk starts a multiple of align rows after the column's
// first row, so that each row is computed by the same copy whatever the
// chunking, and the results do not depend on it.
// xcd_start[x] .. xcd_start[x + 1] is XCD x's run.
inline void build_strips(const std::vector<lb_geometry>& G, const std::vector<int>& active, int chunk, int width,
                         int align, std::vector<StripDev>* out, int* count, int* xcd_start = nullptr) {
    struct Col { int cap, xs, xe, ya, yb; };
    std::vector<Col> cols;
    long long rows = 0;
    auto add = [&](int k, int xs, int xe, int ya, int yb) {
        cols.push_back(Col{k, xs, xe, ya, yb});
        rows += yb - ya;
    };
    for (size_t k = 0; k < G.size(); ++k) {
        if (!active[k]) continue;
        const lb_geometry& g = G[k];
        const bool tube = g.tube_len > 0;
        const int te = g.x_in + g.tube_len;
        for (int xs = 0; xs < g.nx; xs += width) {
            const int xe = std::min(xs + width, g.nx);
            if (tube && xs >= g.x_in && xe <= te) {
                add((int)k, xs, xe, g.y0, g.y0 + g.tube_h);
                continue;
            }
            // The tube enters (or leaves) the column: its wall rows hold fluid only in
            // the reservoir columns [rs, re), cut at a multiple of 32 columns so that
            // every strip's stores still cover whole 128-byte lines.
            int rs = xs, re = xs;
            if (tube && xs < g.x_in && g.x_in < xe && xe <= te) re = std::min(xe, (g.x_in + 31) / 32 * 32);
            if (tube && g.x_in <= xs && xs < te && te < xe) rs = std::max(xs, te / 32 * 32), re = xe;
            if (re - rs <= 0 || re - rs >= xe - xs) {
                add((int)k, xs, xe, 0, g.ny);
                continue;
            }
            // channel rows over the whole width; with an odd tube height one wall row
            // more, so that the wall strip above starts on the channel's row parity
            const int yc = std::min(g.ny, g.y0 + g.tube_h + (g.tube_h & 1));
            add((int)k, xs, xe, g.y0, yc);
            if (g.y0 > 0) add((int)k, rs, re, 0, g.y0);
            if (yc < g.ny) add((int)k, rs, re, yc, g.ny);
        }
    }
    auto down = [&](int v) { return v - v % align; };
    const int small = down(std::max(LB_MIN_CHUNK, chunk / 4) + align - 1);   // rounded up to align
    int n = 0;
    if (out) out->clear();
    std::vector<StripDev> tails;
    size_t ci = 0;
    long long done = 0;
    for (int x = 0; x < 8; ++x) {
        if (xcd_start) xcd_start[x] = n;
        const long long goal = rows * (x + 1) / 8;
        tails.clear();
        const size_t c0 = ci;
        for (; ci < cols.size() && (done < goal || x == 7); ++ci) done += cols[ci].yb - cols[ci].ya;
        // (shorter chunks end a step without a tail: at 8 rows, tails measured slower)
        const size_t tail_from =
            chunk < LB_TAIL_MIN_CHUNK ? ci : (ci - c0 > LB_TAIL_COLS ? ci - LB_TAIL_COLS : c0);
        // rows of column j before its tail (a multiple of align when a tail follows)
        auto body_of = [&](size_t j) {
            const int r = cols[j].yb - cols[j].ya;
            return j >= tail_from ? down(r - std::min(r, 2 * small)) : r;
        };
        auto chunks_of = [&](size_t j) { return (body_of(j) + chunk - 1) / chunk; };
        // start of chunk k of column j, relative to its first row (k = chunks_of: the end)
        auto start_of = [&](size_t j, int k) {
            const int nb = chunks_of(j), body = body_of(j);
            return k >= nb ? body : down((int)((long long)k * body / nb));
        };
        for (size_t g0 = c0; g0 < ci; g0 += LB_STRIP_GROUP) {
            const size_t g1 = std::min(ci, g0 + LB_STRIP_GROUP);
            if (chunk <= 0) {
                for (size_t j = g0; j < g1; ++j) {
                    if (out) out->push_back(StripDev{cols[j].cap, cols[j].xs, cols[j].xe, cols[j].ya, cols[j].yb});
                    ++n;
                }
                continue;
            }
            for (int k = 0;; ++k) {
                bool any = false;
                for (size_t j = g0; j < g1; ++j) {
                    if (k >= chunks_of(j)) continue;
                    any = true;
                    const int y0 = cols[j].ya + start_of(j, k), y1 = cols[j].ya + start_of(j, k + 1);
                    if (y0 == y1) continue;   // (rounding to align emptied it)
                    if (out) out->push_back(StripDev{cols[j].cap, cols[j].xs, cols[j].xe, y0, y1});
                    ++n;
                }
                if (!any) break;
            }
        }
        for (size_t j = tail_from; j < ci; ++j) {
            const Col& c = cols[j];
            for (int y = c.ya + body_of(j); y < c.yb; y += small) {
                tails.push_back(StripDev{c.cap, c.xs, c.xe, y, std::min(y + small, c.yb)});
                ++n;
            }
        }
        if (out) out->insert(out->end(), tails.begin(), tails.end());
    }
    if (xcd_start) xcd_start[8] = n;
    if (count) *count = n;
}

// Strips that a table of this width may need, at any chunking the library
// accepts (0, or 4 rows and more) and for any set of active capillaries: a
// column of r rows has at most ceil(r / 4) chunks, and one more where a tail
// cuts its last rows into chunks of their own (the body and the tail each
// rounded up: ceil(a / 4) + ceil(b / 4) <= ceil((a + b) / 4) + 1).
inline int strip_capacity(const std::vector<lb_geometry>& G, int width) {
    const std::vector<int> all(G.size(), 1);
    int fine = 0, columns = 0;
    build_strips(G, all, LB_MIN_CHUNK, width, 1, nullptr, &fine);
    build_strips(G, all, 0, width, 1, nullptr, &columns);
    return fine + columns;
}

}  // namespace lbk
