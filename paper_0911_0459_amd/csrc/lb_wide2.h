// Two time steps per sweep ("fused" wide strips) of lbcap, van der Waals model.
//
// A single-step sweep reads the nine populations of every node and writes
// them back once per time step.  This sweep reads f*(t-1) once, runs the
// step to f*(t) in the workgroup's LDS and the next step to f*(t+1), and
// writes only that: per two time steps one read (plus the halo) and one
// write instead of two of each.  The arithmetic per node and step is that of
// lb_wide_vdw (vdw_node_collide, the same stencils and pulls); the
// intermediate f*(t) stays FP32 exactly as it would be stored.
//
// Reach of the two steps around an output node (x, y): step 2 pulls f*(t)
// from (x, y) and its 8 neighbours, and its stencils need rho(t+1) of the 8
// neighbours, hence f*(t) two nodes out; step 1 at those nodes needs rho(t)
// one node further out, pulled from f*(t-1) one more node out.  A workgroup
// therefore owns the output columns [xs, xe) (at most WIDE_OUT = 192,
// pitch-aligned stores as in lb_wide_vdw) of a chunk of rows [ya, yb):
//   stage A  pulls f*(t-1), forms the moments of f(t) and rho(t)   columns xs-3 .. xe+2, rows ya-3 .. yb+2
//   stage B  step 1 (stencils of rho(t), collision) -> f*(t)       columns xs-2 .. xe+1, rows ya-2 .. yb+1
//   stage C  pulls f*(t) in LDS, moments of f(t+1), rho(t+1)       columns xs-1 .. xe,   rows ya-1 .. yb
//   stage D  step 2 -> f*(t+1), stored                             columns xs   .. xe-1, rows ya   .. yb-1
// Three main wavefronts own the output columns, one per lane; lanes 0..5 of a
// fourth (halo) wavefront take the columns xs-1, xs+192, xs-2, xs+193, xs-3,
// xs+194 (stages C, B and A need the first two, four and six of them).
//
// The stages of one sweep row are skewed so that each reads only LDS rows
// written before the previous barrier; iteration k runs
//   X phase: A on row k+4, C on row k+1      | barrier
//   Y phase: B on row k+3, D on row k        | barrier
// with rho(t), f*(t) and rho(t+1) in three rings of three rows each.  All
// wavefronts are in the same phase at any time, and every ring slot written in
// a phase holds a row that no stage reads in that phase or needs later:
//   rho(t)   written in X(k) (row k+4), read in Y phases (rows k+2..k+4 in Y(k));
//   f*(t)    written in Y(k) (row k+3), read in X phases (rows k..k+2 in X(k));
//   rho(t+1) written in X(k) (row k+1), read in Y phases (rows k-1..k+1 in Y(k)).
// The pulls of stage A are requested one iteration ahead and stay in flight
// across the barriers (LDS-only barriers); the loop is unrolled by two so the
// two request buffers swap roles without copies, and the rows of every stage
// keep their position in the unrolled pair whatever the chunking (chunks
// start an even number of rows apart), so the results do not depend on it.
#pragma once
#include "lb_wide.h"

namespace lbk {

constexpr int W2A = WIDE_OUT + 6;   // rho(t) ring row: columns xs-3 .. xs+194
constexpr int W2F = WIDE_OUT + 4;   // f*(t) ring row: columns xs-2 .. xs+193
constexpr int W2B = WIDE_OUT + 2;   // rho(t+1) ring row: columns xs-1 .. xs+192

// Role of a thread of a fused wide strip.
struct Wide2Lane {
    int dx;     // its column minus xs
    bool main;  // step 2 at an output column (stage D)
    bool q2;    // stage C: moments of f(t+1) at its column
    bool s1;    // stage B: step 1 at its column
    bool q1;    // stage A: moments of f(t) at its column
};

__device__ __forceinline__ Wide2Lane wide2_lane() {
    const int w = threadIdx.x >> 6, k = threadIdx.x & (SW - 1);
    Wide2Lane r;
    if (w < NWM) {
        r.dx = SW * w + k;
        r.main = r.q2 = r.s1 = r.q1 = true;
    } else {
        // lanes 0..5: xs-1, xs+192, xs-2, xs+193, xs-3, xs+194; the others
        // repeat lane 0's loads and write nothing
        const int depth = k >> 1;
        r.dx = k >= 6 ? -1 : ((k & 1) ? WIDE_OUT + depth : -1 - depth);
        r.main = false;
        r.q2 = k < 2;
        r.s1 = k < 4;
        r.q1 = k < 6;
    }
    return r;
}

// Reads f*(t-1) of one wide strip chunk and its halo, writes f*(t+1).
template <typename CT, bool FORCE = true>
__global__ void __launch_bounds__(WIDE_THREADS) lb_wide2_vdw(StripArgs a) {
    const int si = strip_index(a);
    if (si < 0) return;
    const StripDev s = a.strips[si];
    const CapDev c = a.caps[s.cap];
    const Geo g = geo_of(c);
    const int P = (int)c.plane;
    const int sb = a.cur ^ c.par;
    const Planes fs = planes_of((sb ? a.arena1 : a.arena0) + c.off_f, 9, P, c.pitch);
    const Planes fd = planes_of((sb ? a.arena0 : a.arena1) + c.off_f, 9, P, c.pitch);

    __shared__ float QA[3][W2A];        // drho(t)
    __shared__ float FR[3][9][W2F];     // shifted f*(t), FP32 as a single step stores it
    __shared__ float QB[3][W2B];        // drho(t+1)

    const Wide2Lane W = wide2_lane();
    // lanes past column xe+2 (the last one the sweep reads) repeat that column:
    // their loads share its addresses
    const int xl = min(s.xs + W.dx, s.xe + 2);
    const LaneCols L = lane_cols(g, xl);
    const bool out_col = W.main && xl < s.xe;
    // ring indices of the lane's column; lanes that do not take part in a
    // stage get an index whose neighbours are in range
    const int ja_w = W.dx + 3;
    const int ja = W.s1 ? W.dx + 3 : 1;
    const int jf = (W.s1 || W.q2) ? W.dx + 2 : 1;
    const int jb = W.q2 ? W.dx + 1 : 1;
    const float G2 = 2.f * c.G;
    const Mom<float> zero{0.f, 0.f, 0.f, 0.f, 0.f};

    int b = 0;   // (k - ya + 7) mod 3 in iteration k: row k + d is in slot (b + d + 2) mod 3
    auto slot = [&](int d) {
        int v = b + d + 2;
        v -= v >= 3 ? 3 : 0;
        v -= v >= 3 ? 3 : 0;
        v -= v >= 3 ? 3 : 0;
        return v;
    };
    auto row_flags = [&](int y, unsigned& sm, bool& fl) {
        const RowInfo r = row_info(g, y);
        sm = solid_bits(L, r);
        fl = !(L.t0 && r.w0);
        return r;
    };
    // pull of f(t+1) from the f*(t) ring (bounce-back from solid sources), row slots
    // of the row below (sm1), at (s0) and above (sp1)
    auto pull_ring = [&](int sm1, int s0, int sp1, unsigned sm, float (&f)[9]) {
        f[0] = FR[s0][0][jf];
#pragma unroll
        for (int i = 1; i < 9; ++i) {
            const bool bb = (sm >> opp_(i)) & 1u;
            const int sy = ey_(i) > 0 ? sm1 : (ey_(i) < 0 ? sp1 : s0);
            const float* p = bb ? &FR[s0][opp_(i)][jf] : &FR[sy][i][jf - ex_(i)];
            f[i] = *p;
        }
    };

    // requests of stage A, one iteration ahead: row ya-3 for the first one
    float fa[9], fb[9];
    {
        unsigned sm0;
        bool fl0;
        const RowInfo r0 = row_flags(s.ya - 3, sm0, fl0);
        pull_lane(fs, L, r0, sm0, fb);
    }
    Mom<float> mA_cur = zero, mB_cur = zero;   // moments of f(t) of row k+3, of f(t+1) of row k

    // iteration k: fn holds the pulls of row k+4, fp receives those of row k+5
    auto iter = [&](int k, const float (&fn)[9], float (&fp)[9]) {
        {
            unsigned smq;
            bool flq;
            const RowInfo rq = row_flags(min(k + 5, s.yb + 2), smq, flq);
            pull_lane(fs, L, rq, smq, fp);
        }
        __builtin_amdgcn_sched_barrier(0);
        // ---- X phase: A on row k+4, C on row k+1
        Mom<float> mA_n = zero, mB_n = zero;
        if (k + 4 <= s.yb + 2) {
            unsigned sma;
            bool fla;
            row_flags(k + 4, sma, fla);
            if (fla) mA_n = moments_of(fn, sma != 0u);
            if (W.q1) QA[slot(4)][ja_w] = mA_n.drho;
        }
        if (k >= s.ya - 2) {
            unsigned smc;
            bool flc;
            row_flags(k + 1, smc, flc);
            if (W.q2) {
                if (flc) {
                    float f[9];
                    pull_ring(slot(0), slot(1), slot(2), smc, f);
                    mB_n = moments_of(f, smc != 0u);
                }
                QB[slot(1)][jb] = mB_n.drho;
            }
        }
        lds_barrier();
        // ---- Y phase: B (step 1) on row k+3, D (step 2) on row k
        if (k >= s.ya - 5 && k <= s.yb - 2) {
            unsigned smb;
            bool flb;
            row_flags(k + 3, smb, flb);
            if (W.s1 && flb) {
                float dxf, dyf, lapf;
                stencil3(QA[slot(2)], QA[slot(3)], QA[slot(4)], ja, smb, G2, dxf, dyf, lapf);
                CT o[9];
                vdw_node_collide<CT, FORCE>(c, mA_cur, smb, dxf, dyf, lapf, o);
                const int sf = slot(3);
#pragma unroll
                for (int i = 0; i < 9; ++i) FR[sf][i][jf] = (float)o[i];
            }
        }
        __builtin_amdgcn_sched_barrier(0);
        if (k >= s.ya) {
            unsigned smd;
            bool fld;
            const RowInfo rd = row_flags(k, smd, fld);
            if (out_col && fld) {
                float dxf, dyf, lapf;
                stencil3(QB[slot(-1)], QB[slot(0)], QB[slot(1)], jb, smd, G2, dxf, dyf, lapf);
                CT o[9];
                vdw_node_collide<CT, FORCE>(c, mB_cur, smd, dxf, dyf, lapf, o);
                const int srow = rd.y0 * fd.rb;
#pragma unroll
                for (int i = 0; i < 9; ++i) st(fd, (float)o[i], L.b0, i * fd.pb + srow);
            }
        }
        lds_barrier();
        mA_cur = mA_n;
        mB_cur = mB_n;
        b = b == 2 ? 0 : b + 1;
    };
    for (int k = s.ya - 7; k < s.yb; k += 2) {
        iter(k, fb, fa);
        if (k + 1 >= s.yb) break;
        iter(k + 1, fa, fb);
    }
}

}  // namespace lbk
