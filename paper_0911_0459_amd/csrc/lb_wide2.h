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

// ---- binary model --------------------------------------------------------------
// Two time steps per sweep of the binary model (population storage, phi in
// fixed point as in every binary sweep): reads f*(t-1) and phi(t), writes
// f*(t+1) and phi(t+2).  The arithmetic per node and step is that of
// lb_wide_bin (bin_node_state, phi_delta, the same stencils and pulls; every
// collision takes the velocity its pulls formed), and the intermediate f*(t)
// stays FP32 as a single step would store it, phi(t+1) in fixed point.
//
// Reach: the step at a node needs u and A = Gamma mu - phi |u|^2 / 2 of its
// neighbours (the phi update) and phi of its neighbours (the stencils), hence
// the pulls of the neighbours and phi two nodes out.  Two steps reach four.
// Stages of a row r, with the columns they cover:
//   load  phi(t) of row r into a ring                                 xs-4 .. xe+3
//   A     pulls of f*(t-1), moments of f(t), u(t); stencils of phi(t),
//         A(t)                                                        xs-3 .. xe+2
//   B     step 1: collision -> f*(t) into rings; phi(t+1) into a ring xs-2 .. xe+1
//   C     pulls of f*(t) from the rings, moments of f(t+1), u(t+1);
//         stencils of phi(t+1), A(t+1)                                xs-1 .. xe
//   D     step 2: collision -> f*(t+1) stored; phi(t+2) stored        xs   .. xe-1
// Three main wavefronts own the output columns, one per lane; lanes 0..7 of
// the halo wavefront take xs-1, xs+192, xs-2, xs+193, xs-3, xs+194, xs-4,
// xs+195 (stage C needs the first two, B four, A six, the load eight).
//
// Iteration k runs
//   X phase: A on row k+4, C on row k+1                            | barrier
//   Y phase: B on row k+3, D on row k; phi(t) of row k+6 loaded    | barrier
// Rings (every ring slot written in a phase holds a row that no stage reads in
// that phase or later):
//   phi(t)    6 rows: written in Y(k) (row k+6), read by A (rows k+3..k+5 in
//             X(k)) and B (rows k+2..k+4 in Y(k));
//   u, A (t)  3 rows: written in X(k) (row k+4), read by B (k+2..k+4 in Y(k));
//   f*(t)     written in Y(k) (row k+3), pulled by C in X(k) (row k+1): f3, f5,
//             f7 from rows k and k+1 (3 rows), f4, f6, f8 from k+1 and k+2 and
//             f1, f2 from k+1 (2 rows each); f0 stays in its lane's register;
//   phi(t+1)  6 rows: written in Y(k) (row k+3), read by C (k..k+2 in X(k))
//             and D (k-1..k+1 in Y(k));
//   u, A (t+1) 3 rows: written in X(k) (row k+1), read by D (k-1..k+1 in Y(k)).
// 39,200 bytes of LDS: four workgroups per CU.  The pulls of stage A are
// requested an iteration ahead and stay in flight across the LDS-only
// barriers; the loop is unrolled by two (chunks start an even number of rows
// apart), so every row of every stage is computed by the same copy of the loop
// body whatever the chunking.
constexpr int W2R = WIDE_OUT + 8;   // ring row: columns xs-4 .. xs+195

// Role of a thread of a binary fused wide strip.
struct Wide2BinLane {
    int dx;     // its column minus xs
    bool main;  // stage D at an output column
    bool c;     // stage C at its column
    bool b;     // stage B
    bool a;     // stage A
    bool ld;    // loads phi(t) of its column
};

__device__ __forceinline__ Wide2BinLane wide2bin_lane() {
    const int w = threadIdx.x >> 6, k = threadIdx.x & (SW - 1);
    Wide2BinLane r;
    if (w < NWM) {
        r.dx = SW * w + k;
        r.main = r.c = r.b = r.a = r.ld = true;
    } else {
        // lanes 0..7 as above; the others repeat lane 0's loads and write nothing
        const int depth = k >> 1;
        r.dx = k >= 8 ? -1 : ((k & 1) ? WIDE_OUT + depth : -1 - depth);
        r.main = false;
        r.c = k < 2;
        r.b = k < 4;
        r.a = k < 6;
        r.ld = k < 8;
    }
    return r;
}

// Reads f*(t-1) and phi(t) of one wide strip chunk and its halo, writes
// f*(t+1) and phi(t+2).
template <typename MT, typename CT, typename ST = CT, bool FORCE = true>
__global__ void __launch_bounds__(WIDE_THREADS, 4) lb_wide2_bin(StripArgs a) {
    const int si = strip_index(a);
    if (si < 0) return;
    const StripDev s = a.strips[si];
    const CapDev c = a.caps[s.cap];
    const Geo g = geo_of(c);
    const int P = (int)c.plane;
    const int sb = a.cur ^ c.par;
    const Planes fs = planes_of((sb ? a.arena1 : a.arena0) + c.off_f, 9, P, c.pitch);
    const Planes ps = planes_of((sb ? a.arena1 : a.arena0) + c.off_phi, 1, P, c.pitch);
    const Planes fd = planes_of((sb ? a.arena0 : a.arena1) + c.off_f, 9, P, c.pitch);
    const Planes pd = planes_of((sb ? a.arena0 : a.arena1) + c.off_phi, 1, P, c.pitch);

    __shared__ float P1[6][W2R];       // phi(t)
    __shared__ float U1[3][3][W2R];    // ux, uy, A of f(t)
    __shared__ float FU[3][3][W2R];    // f*(t): f3, f5, f7
    __shared__ float FD[2][3][W2R];    // f*(t): f4, f6, f8
    __shared__ float FH[2][2][W2R];    // f*(t): f1, f2
    __shared__ float P2[6][W2R];       // phi(t+1)
    __shared__ float U2[3][3][W2R];    // ux, uy, A of f(t+1)

    const Wide2BinLane W = wide2bin_lane();
    // lanes past column xe+3 (the last one the sweep reads) repeat that column:
    // their loads share its addresses
    const int xl = min(s.xs + W.dx, s.xe + 3);
    const LaneCols L = lane_cols(g, xl);
    const bool out_col = W.main && xl < s.xe;
    const int j = W.dx + 4;   // the lane's index in a ring row
    const float G2 = 2.f * c.G;
    const float kap = c.kappa, Gam = c.Gamma;

    // row k + d of iteration k is in slot (t6 + d) mod 6 of a ring of 6 rows,
    // its index modulo 3 or 2 in the smaller rings
    int t6 = 0;
    auto m6 = [&](int d) {   // -1 <= d <= 6
        int v = t6 + d;
        v += v < 0 ? 6 : 0;
        v -= v >= 6 ? 6 : 0;
        v -= v >= 6 ? 6 : 0;
        return v;
    };
    auto m3 = [&](int d) {
        const int v = m6(d);
        return v >= 3 ? v - 3 : v;
    };
    auto m2 = [&](int d) { return m6(d) & 1; };
    // the sweep reaches four rows beyond its chunk: rows wrapped periodically in
    // full (row_info wraps once), for lattices of fewer than four rows too
    auto row_at = [&](int y) {
        while (y < 0) y += g.ny;
        while (y >= g.ny) y -= g.ny;
        return row_info(g, y);
    };
    auto row_flags = [&](int y, unsigned& sm, bool& fl) {
        const RowInfo r = row_at(y);
        sm = solid_bits(L, r);
        fl = !(L.t0 && r.w0);
        return r;
    };
    auto phi_entry = [&](int y, float m) {   // m: fixed point
        const RowInfo r = row_at(y);
        return (L.t0 && r.w0) ? 0.f : phi_of_fixed(m);
    };

    struct Req {
        float f[9];   // pulls of f*(t-1), row k+5 (requested in iteration k)
        float pm;     // phi(t) of row k+7, fixed point
    };
    // pulls and stencils of a row, kept for its collision in the next phase Y;
    // two of them swap roles every iteration (a lane that does not pull a row
    // leaves the older contents, which no collision reads)
    struct Pulled {
        Mom<float> mom;
        float dx, dy, lap;
    };
    const int k0 = s.ya - 7;
    // prologue: phi(t) of rows k0+3 .. k0+5 into the ring, their fixed-point
    // values for the phi updates of step 1
    int q0a, q0b, q0c;   // phi(t) of this lane's column, rows k+3, k+4, k+5 in iteration k
    {
        const float m3v = ld(ps, L.b0, row_at(k0 + 3).y0 * ps.rb);
        const float m4v = ld(ps, L.b0, row_at(k0 + 4).y0 * ps.rb);
        const float m5v = ld(ps, L.b0, row_at(k0 + 5).y0 * ps.rb);
        if (W.ld) {
            P1[3][j] = phi_entry(k0 + 3, m3v);
            P1[4][j] = phi_entry(k0 + 4, m4v);
            P1[5][j] = phi_entry(k0 + 5, m5v);
        }
        q0a = __builtin_bit_cast(int, m3v);
        q0b = __builtin_bit_cast(int, m4v);
        q0c = __builtin_bit_cast(int, m5v);
    }
    Req RA, RB;
    {
        unsigned sm0;
        bool fl0;
        const RowInfo r0 = row_flags(k0 + 4, sm0, fl0);
        pull_lane(fs, L, r0, sm0, RA.f);
        RA.pm = ld(ps, L.b0, row_at(k0 + 6).y0 * ps.rb);
    }
    Pulled SA0{{0.f, 0.f, 0.f, 0.f, 0.f}, 0.f, 0.f, 0.f}, SA1 = SA0, SC0 = SA0, SC1 = SA0;
    float f0a = 0.f, f0b = 0.f;   // f0 of f*(t) at this lane's column, rows of each parity
    int q1a = 0, q1b = 0, q1c = 0;   // phi(t+1), fixed point, rows k, k+1, k+2 in iteration k
    t6 = 0;
    lds_barrier();

    // iteration k: n holds the requests for row k+4 (pulls) and k+6 (phi),
    // p receives those for rows k+5 and k+7
    auto iter = [&](int k, const Req& n, Req& p, const Pulled& a_cur, Pulled& a_nxt, const Pulled& c_cur,
                    Pulled& c_nxt, float& f0) {
        {
            unsigned smq;
            bool flq;
            const RowInfo rq = row_flags(min(k + 5, s.yb + 2), smq, flq);
            pull_lane(fs, L, rq, smq, p.f);
            p.pm = ld(ps, L.b0, row_at(min(k + 7, s.yb + 3)).y0 * ps.rb);
        }
        __builtin_amdgcn_sched_barrier(0);
        // ---- X phase: A on row k+4, C on row k+1
        if (k + 4 <= s.yb + 2 && W.a) {
            unsigned sma;
            bool fla;
            row_flags(k + 4, sma, fla);
            float ux = 0.f, uy = 0.f, am = 0.f;
            if (fla) {
                const bool bnd = sma != 0u;
                a_nxt.mom = moments_of(n.f, bnd);
                const float F = bnd ? 0.f : c.Fx;
                const float inv_rho = recip(c.rho_ref + a_nxt.mom.drho);
                ux = (a_nxt.mom.jx + 0.5f * F) * inv_rho;
                uy = a_nxt.mom.jy * inv_rho;
                stencil3(P1[m6(3)], P1[m6(4)], P1[m6(5)], j, sma, G2, a_nxt.dx, a_nxt.dy, a_nxt.lap);
                const float ph = P1[m6(4)][j];
                const float gmu = Gam * (mu_bulk(c, ph) - kap * a_nxt.lap);
                am = gmu - 0.5f * ph * (ux * ux + uy * uy);
            }
            const int u4 = m3(4);
            U1[u4][0][j] = ux;
            U1[u4][1][j] = uy;
            U1[u4][2][j] = am;
        }
        if (k >= s.ya - 2 && W.c) {
            unsigned smc;
            bool flc;
            row_flags(k + 1, smc, flc);
            float ux = 0.f, uy = 0.f, am = 0.f;
            if (flc) {
                const int u0 = m3(0), u1 = m3(1), h1 = m2(1), h2 = m2(2);
                // streaming source of direction i: row k+1-ey_i, column offset -ex_i
                auto src = [&](int i) -> const float* {
                    switch (i) {
                        case 1: return &FH[h1][0][j - 1];
                        case 2: return &FH[h1][1][j + 1];
                        case 3: return &FU[u0][0][j];
                        case 4: return &FD[h2][0][j];
                        case 5: return &FU[u0][1][j - 1];
                        case 6: return &FD[h2][1][j + 1];
                        case 7: return &FU[u0][2][j + 1];
                        default: return &FD[h2][2][j - 1];
                    }
                };
                // the node's own population i (row k+1), taken by bounce-back
                auto own = [&](int i) -> const float* {
                    switch (i) {
                        case 1: return &FH[h1][0][j];
                        case 2: return &FH[h1][1][j];
                        case 3: return &FU[u1][0][j];
                        case 4: return &FD[h1][0][j];
                        case 5: return &FU[u1][1][j];
                        case 6: return &FD[h1][1][j];
                        case 7: return &FU[u1][2][j];
                        default: return &FD[h1][2][j];
                    }
                };
                float f[9];
                f[0] = f0;
#pragma unroll
                for (int i = 1; i < 9; ++i) {
                    const bool bb = (smc >> opp_(i)) & 1u;
                    f[i] = *(bb ? own(opp_(i)) : src(i));
                }
                const bool bnd = smc != 0u;
                c_nxt.mom = moments_of(f, bnd);
                const float F = bnd ? 0.f : c.Fx;
                const float inv_rho = recip(c.rho_ref + c_nxt.mom.drho);
                ux = (c_nxt.mom.jx + 0.5f * F) * inv_rho;
                uy = c_nxt.mom.jy * inv_rho;
                stencil3(P2[m6(0)], P2[m6(1)], P2[m6(2)], j, smc, G2, c_nxt.dx, c_nxt.dy, c_nxt.lap);
                const float ph = P2[m6(1)][j];
                const float gmu = Gam * (mu_bulk(c, ph) - kap * c_nxt.lap);
                am = gmu - 0.5f * ph * (ux * ux + uy * uy);
            }
            const int u1 = m3(1);
            U2[u1][0][j] = ux;
            U2[u1][1][j] = uy;
            U2[u1][2][j] = am;
        }
        lds_barrier();
        // ---- Y phase: B (step 1) on row k+3, D (step 2) on row k; phi(t) of row k+6
        int q1_new = 0;
        if (k >= s.ya - 5 && k + 3 <= s.yb + 1 && W.b) {
            unsigned smb;
            bool flb;
            row_flags(k + 3, smb, flb);
            float p1 = 0.f;
            if (flb) {
                const int u3 = m3(3);
                const float phi = P1[m6(3)][j];
                const float uxf = U1[u3][0][j], uyf = U1[u3][1][j];
                CT o[9];
                pops_of_state(
                    bin_node_state<CT, ST, FORCE>(c, a_cur.mom, smb, phi, a_cur.dx, a_cur.dy, a_cur.lap, uxf, uyf), o);
                const int h3 = m2(3);
                FU[u3][0][j] = (float)o[3];
                FU[u3][1][j] = (float)o[5];
                FU[u3][2][j] = (float)o[7];
                FD[h3][0][j] = (float)o[4];
                FD[h3][1][j] = (float)o[6];
                FD[h3][2][j] = (float)o[8];
                FH[h3][0][j] = (float)o[1];
                FH[h3][1][j] = (float)o[2];
                f0 = (float)o[0];
                // the phi update below is not to be interleaved with the collision
                // (its LDS reads would be hoisted into the collision's register peak)
                __builtin_amdgcn_sched_barrier(0);
                const float dphi = phi_delta(smb, phi, uxf, uyf, U1[u3][2][j],
                                             [&](int i, float& am, float& pp, float& x, float& yy) {
                                                 const int un = m3(3 - ey_(i)), kn = j - ex_(i);
                                                 am = U1[un][2][kn];
                                                 pp = P1[m6(3 - ey_(i))][kn];
                                                 x = U1[un][0][kn];
                                                 yy = U1[un][1][kn];
                                             });
                q1_new = q0a + fixed_of_phi(dphi);
                p1 = phi_of_fixed(phi_bits(q1_new));
            }
            P2[m6(3)][j] = p1;
        }
        __builtin_amdgcn_sched_barrier(0);
        if (k >= s.ya && out_col) {
            unsigned smd;
            bool fld;
            const RowInfo rd = row_flags(k, smd, fld);
            if (fld) {
                const int u0 = m3(0);
                const float phi = P2[m6(0)][j];
                const float uxf = U2[u0][0][j], uyf = U2[u0][1][j];
                CT o[9];
                pops_of_state(
                    bin_node_state<CT, ST, FORCE>(c, c_cur.mom, smd, phi, c_cur.dx, c_cur.dy, c_cur.lap, uxf, uyf), o);
                const int srow = rd.y0 * fd.rb;
#pragma unroll
                for (int i = 0; i < 9; ++i) st(fd, (float)o[i], L.b0, i * fd.pb + srow);
                __builtin_amdgcn_sched_barrier(0);
                const float dphi = phi_delta(smd, phi, uxf, uyf, U2[u0][2][j],
                                             [&](int i, float& am, float& pp, float& x, float& yy) {
                                                 const int un = m3(-ey_(i)), kn = j - ex_(i);
                                                 am = U2[un][2][kn];
                                                 pp = P2[m6(-ey_(i))][kn];
                                                 x = U2[un][0][kn];
                                                 yy = U2[un][1][kn];
                                             });
                st(pd, phi_bits(q1a + fixed_of_phi(dphi)), L.b0, rd.y0 * pd.rb);
            }
        }
        if (W.ld) P1[m6(6)][j] = phi_entry(k + 6, n.pm);
        lds_barrier();
        // ---- rotate the fixed-point pipelines
        q0a = q0b;
        q0b = q0c;
        q0c = __builtin_bit_cast(int, n.pm);
        q1a = q1b;
        q1b = q1c;
        q1c = q1_new;
        t6 = t6 == 5 ? 0 : t6 + 1;
    };
    for (int k = k0; k < s.yb; k += 2) {
        iter(k, RA, RB, SA0, SA1, SC0, SC1, f0a);
        if (k + 1 >= s.yb) break;
        iter(k + 1, RB, RA, SA1, SA0, SC1, SC0, f0b);
    }
}

}  // namespace lbk
