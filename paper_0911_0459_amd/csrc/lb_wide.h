// Cooperative row-sweep ("wide strip") kernels of lbcap: the time step of
// lb_strip_bin / lb_strip_vdw with every wavefront's output columns aligned to
// whole 128-byte lines.
//
// A workgroup owns the output columns xs .. xe-1 (at most WIDE_OUT = 192) of a
// chunk of rows (xs a multiple of 32; rows are pitched to 64 floats, so each
// wavefront stores whole cache lines and no line is shared with another
// workgroup) and marches along y as the single-wave strips do.  Its NWM = 3
// main wavefronts produce the outputs, one column per lane.  The step at a
// column needs the velocity and the chemical potential one column to either
// side and the order field two columns to either side: a fourth (halo)
// wavefront computes the velocity and the chemical potential of the columns
// xs-1 and xs+192 (lanes 0 and 1) and loads the order field of xs-2 and xs+193
// (lanes 2 and 3); its other lanes repeat lane 0's loads and store nothing.  In
// a strip narrower than 192 columns, the main lanes at xe and xe+1 supply those
// neighbours.  Four wavefronts per workgroup spread evenly over the four SIMDs
// of a CU.
//
// Rows of phi, u and mu live in LDS rings shared by the four wavefronts.  The
// wavefronts meet at LDS-only barriers (two per row for the binary model, one
// for van der Waals); the rings hold one row more than a row's stencils read,
// so a wavefront that has passed a row's last barrier can already fill the
// next row's slots while the others still read the current ones.  The
// population loads requested one row ahead stay in flight across the barriers.
#pragma once
#include "lb_strip.h"

namespace lbk {

constexpr int WIDE_OUT = 192;                  // output columns per wide strip
constexpr int NWM = WIDE_OUT / SW;             // main wavefronts
constexpr int WIDE_THREADS = (NWM + 1) * SW;   // main wavefronts and the halo wavefront
constexpr int WU = WIDE_OUT + 2;               // u / mu row: columns xs-1 .. xs+WIDE_OUT
constexpr int WP = WIDE_OUT + 4;               // phi row: columns xs-2 .. xs+WIDE_OUT+1

// Workgroup barrier that orders LDS accesses only.  __syncthreads() would also
// wait for every outstanding global load, including the row requested ahead.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Role of a thread of a wide strip.
struct WideLane {
    int dx;     // its column minus xs (wrapped periodically by lane_cols)
    int uj;     // index of its column in a row of columns xs-1.. (0 for lanes that compute no u)
    int pj;     // index of its column in a row of columns xs-2..
    int qj;     // pj for lanes that compute u, else 2 (a safe index for their unused stencils)
    bool main;  // a main wavefront lane: one output column
    bool um;    // computes u and mu (main lanes; halo lanes 0 and 1)
    bool ph;    // stores phi (main lanes; halo lanes 0..3)
};

__device__ __forceinline__ WideLane wide_lane() {
    const int w = threadIdx.x >> 6, k = threadIdx.x & (SW - 1);
    WideLane r;
    if (w < NWM) {
        r.dx = SW * w + k;
        r.main = r.um = r.ph = true;
    } else {
        r.dx = k == 1 ? WIDE_OUT : (k == 2 ? -2 : (k == 3 ? WIDE_OUT + 1 : -1));
        r.main = false;
        r.um = k < 2;
        r.ph = k < 4;
    }
    r.uj = r.um ? r.dx + 1 : 0;
    r.pj = r.dx + 2;
    r.qj = r.um ? r.pj : 2;
    return r;
}

// ---- binary model --------------------------------------------------------------
// Reads f*(t-1) and phi(t) of one wide strip chunk, writes f*(t) and phi(t+1).
// (at most 80 vector registers and 19 KB of LDS: six wavefronts per SIMD, six
// workgroups per CU; seven fit, but evict more of the halo lines that
// neighbouring strips share and measured slower)
template <typename MT, typename CT, typename ST = CT, bool FORCE = true>
__global__ void __launch_bounds__(WIDE_THREADS, 6) lb_wide_bin(StripArgs a) {
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

    // One LDS ring of RING rows, each slot holding the row's phi, ux, uy and
    // A = Gamma mu - phi |u|^2 / 2 (the part of g^eq that does not depend on the
    // direction) over the columns xs-2 .. xs+WIDE_OUT+1: one address register
    // serves all four, at immediate offsets.  Row y+d of the row being finished,
    // y, is in slot sl(d).  No barrier ends a row: a wavefront that has passed
    // row y's second barrier and starts row y+1 writes phi row y+3 and u row y+2
    // (slots 4 and 3 rows on from y-1 in a ring of 6), while a slower one may
    // still be in row y's last phase reading rows y-1..y+1; and it waits at row
    // y+1's first barrier before it writes A of row y+2.
    enum { R_PH = 0, R_UX = 1, R_UY = 2, R_AM = 3, RING = 6 };
    __shared__ float RG[RING][4][WP];

    const WideLane W = wide_lane();
    // lanes past column xe+1 (the last one that an output column reads) repeat
    // that column: their loads share its addresses
    const int xl = min(s.xs + W.dx, s.xe + 1);
    const LaneCols L = lane_cols(g, xl);
    const bool out_col = W.main && xl < s.xe;
    const int pj = W.pj, qj = W.qj;
    const float G2 = 2.f * c.G;
    const float kap = c.kappa, Gam = c.Gamma;
    int ry = 2;   // slot of the row being finished (the chunk's first row to begin with)
    auto sl = [&](int d) {   // slot of that row + d, -2 <= d <= 3
        int v = ry + d;
        v += v < 0 ? RING : 0;
        v -= v >= RING ? RING : 0;
        return v;
    };

    // phi is loaded unconditionally (solid nodes have valid addresses) and
    // masked when stored, so that no instruction waits on it early
    auto phi_load = [&](const RowInfo& r) { return ld(ps, L.b0, r.y0 * ps.rb); };
    auto phi_store = [&](int slot, const RowInfo& r, float m) {   // m: fixed point
        if (W.ph) RG[slot][R_PH][pj] = (L.t0 && r.w0) ? 0.f : phi_of_fixed(m);
    };
    // moments of a pulled row (FP32, kept by the caller) and its velocity into LDS
    auto u_row = [&](int slot, const float (&f)[9], bool fluid, unsigned sm, Mom<float>& m) {
        float ux = 0.f, uy = 0.f;
        if (fluid) {
            const bool bnd = sm != 0u;
            m = moments_of(f, bnd);
            const float F = bnd ? 0.f : c.Fx;
            const float inv_rho = recip(c.rho_ref + m.drho);
            ux = (m.jx + 0.5f * F) * inv_rho;
            uy = m.jy * inv_rho;
        } else {
            m = Mom<float>{0.f, 0.f, 0.f, 0.f, 0.f};
        }
        if (W.um) {
            RG[slot][R_UX][qj] = ux;
            RG[slot][R_UY][qj] = uy;
        }
    };
    // stencils of phi (row slots below, at, above), Gamma mu and A of the row at slot `at`
    auto mu_row = [&](int below, int at, int above, bool fluid, unsigned sm, float& dx, float& dy, float& lap) {
        float v = 0.f;
        dx = dy = lap = 0.f;
        if (fluid) {
            stencil3(RG[below][R_PH], RG[at][R_PH], RG[above][R_PH], qj, sm, G2, dx, dy, lap);
            const float ph = RG[at][R_PH][qj];
            const float gmu = Gam * (mu_bulk(c, ph) - kap * lap);
            const float ux = RG[at][R_UX][qj], uy = RG[at][R_UY][qj];
            v = gmu - 0.5f * ph * (ux * ux + uy * uy);
        }
        if (W.um) RG[at][R_AM][qj] = v;
    };

    // ---- prologue: phi rows ya-2..ya+1; u, mu of rows ya-1, ya
    int q_cur = 0, q_next = 0;   // fixed-point phi of this lane's column, rows y and y+1
    for (int d = -2; d <= 1; ++d) {
        const RowInfo rr = row_info(g, s.ya + d);
        const float m = phi_load(rr);
        if (d == 0) q_cur = __builtin_bit_cast(int, m);
        if (d == 1) q_next = __builtin_bit_cast(int, m);
        phi_store(sl(d), rr, m);
    }
    float f[9];
    Mom<float> mom_cur;
    RowInfo ri = row_info(g, s.ya - 1);
    unsigned sm = solid_bits(L, ri);
    bool fl = !(L.t0 && ri.w0);
    pull_lane(fs, L, ri, sm, f);
    u_row(sl(-1), f, fl, sm, mom_cur);
    ri = row_info(g, s.ya);
    unsigned sm_cur = solid_bits(L, ri);
    bool fl_cur = !(L.t0 && ri.w0);
    pull_lane(fs, L, ri, sm_cur, f);
    u_row(sl(0), f, fl_cur, sm_cur, mom_cur);
    lds_barrier();
    float dx_cur, dy_cur, lap_cur, t0, t1, t2;
    mu_row(sl(-2), sl(-1), sl(0), fl, sm, t0, t1, t2);
    mu_row(sl(-1), sl(0), sl(1), fl_cur, sm_cur, dx_cur, dy_cur, lap_cur);
    // Requests run one row ahead of the arithmetic; the two request buffers swap
    // roles every row (the loop is unrolled by two), so a finished request is
    // never copied: a copy would wait for every load in flight.
    struct Ahead {
        float f[9];       // pulled populations of row y+1
        float pm;         // phi of row y+2
        RowInfo rph;      // row y+2
        unsigned sm;
        bool fl;
    };
    Ahead A, B;
    {
        const RowInfo rn = row_info(g, s.ya + 1);
        A.sm = solid_bits(L, rn);
        A.fl = !(L.t0 && rn.w0);
        pull_lane(fs, L, rn, A.sm, A.f);
        A.rph = row_info(g, s.ya + 2);
        A.pm = phi_load(A.rph);
    }

    // one row y: n holds the requests for row y+1, p receives those for row y+2
    auto iter = [&](int y, Ahead& n, Ahead& p) {
        // (a) requests for the next row: row y+2 pulled, phi row y+3 (in the last
        // row of the chunk a repeat of the previous requests: cache hits, unused)
        const int ya2 = y + 1 < s.yb ? y + 2 : y + 1;
        const RowInfo ri_p = row_info(g, ya2);
        p.sm = solid_bits(L, ri_p);
        p.fl = !(L.t0 && ri_p.w0);
        p.rph = row_info(g, ya2 + 1);
        pull_lane(fs, L, ri_p, p.sm, p.f);
        p.pm = phi_load(p.rph);
        __builtin_amdgcn_sched_barrier(0);
        // (b) phi row y+2; u and moments of row y+1
        const int q_new = __builtin_bit_cast(int, n.pm);
        phi_store(sl(2), n.rph, n.pm);
        Mom<float> mom_n;
        u_row(sl(1), n.f, n.fl, n.sm, mom_n);
        lds_barrier();
        // (c) stencils and mu of row y+1
        float dx_n, dy_n, lap_n;
        mu_row(sl(0), sl(1), sl(2), n.fl, n.sm, dx_n, dy_n, lap_n);
        lds_barrier();
        // (d) collision and phi update of row y (main lanes)
        if (out_col && fl_cur) {
            const int s0 = sl(0);
            const float phi = RG[s0][R_PH][pj];
            const float uxf = RG[s0][R_UX][pj], uyf = RG[s0][R_UY][pj];
            CT o[9];
            pops_of_state(bin_node_state<CT, ST, FORCE>(c, mom_cur, sm_cur, phi, dx_cur, dy_cur, lap_cur, uxf, uyf),
                          o);
            const int srow = row_info(g, y).y0 * fd.rb;
#pragma unroll
            for (int i = 0; i < 9; ++i) st(fd, (float)o[i], L.b0, i * fd.pb + srow);
            // the phi update below is not to be interleaved with the collision
            // (its LDS reads would be hoisted into the collision's register peak)
            __builtin_amdgcn_sched_barrier(0);
            // phi(t+1) (phi_delta, as in lb_strip_bin)
            const float dphi = phi_delta(sm_cur, phi, uxf, uyf, RG[s0][R_AM][pj],
                                         [&](int i, float& a, float& p, float& x, float& y) {
                                             const int sn = sl(-ey_(i)), kn = pj - ex_(i);
                                             a = RG[sn][R_AM][kn];
                                             p = RG[sn][R_PH][kn];
                                             x = RG[sn][R_UX][kn];
                                             y = RG[sn][R_UY][kn];
                                         });
            st(pd, phi_bits(q_cur + fixed_of_phi(dphi)), L.b0, srow);
        }
        // (e) rotate the row state
        mom_cur = mom_n;
        sm_cur = n.sm;
        fl_cur = n.fl;
        dx_cur = dx_n;
        dy_cur = dy_n;
        lap_cur = lap_n;
        q_cur = q_next;
        q_next = q_new;
        ry = ry == RING - 1 ? 0 : ry + 1;
    };
    for (int y = s.ya; y < s.yb; y += 2) {
        iter(y, A, B);
        if (y + 1 >= s.yb) break;
        iter(y + 1, B, A);
    }
}

// ---- van der Waals model ---------------------------------------------------------
// (the node's collision is vdw_node_collide, shared with lb_strip_vdw)
template <typename CT, bool FORCE = true>
__global__ void __launch_bounds__(WIDE_THREADS) lb_wide_vdw(StripArgs a) {
    const int si = strip_index(a);
    if (si < 0) return;
    const StripDev s = a.strips[si];
    const CapDev c = a.caps[s.cap];
    const Geo g = geo_of(c);
    const int P = (int)c.plane;
    const int sb = a.cur ^ c.par;
    const Planes fs = planes_of((sb ? a.arena1 : a.arena0) + c.off_f, 9, P, c.pitch);
    const Planes fd = planes_of((sb ? a.arena0 : a.arena1) + c.off_f, 9, P, c.pitch);

    // drho rows, row y in slot y mod 4: a wavefront that has passed row y's
    // barrier writes row y+2 (slot y-2 mod 4) while a slower one still reads rows
    // y-1..y+1, then waits at row y+1's barrier
    __shared__ float Q[4][WU];
    const WideLane W = wide_lane();
    // lanes past column xe+1 (the last one that an output column reads) repeat
    // that column: their loads share its addresses
    const int xl = min(s.xs + W.dx, s.xe + 1);
    const LaneCols L = lane_cols(g, xl);
    const bool out_col = W.main && xl < s.xe;
    const int uj = W.uj;
    const float G2 = 2.f * c.G;
    const int yo = 4;   // rows are addressed in the ring as y + 4 (y >= ya - 1 >= -1)
    auto s4 = [](int y) { return y & 3; };
    auto q_store = [&](int slot, float drho) {
        if (W.um) Q[slot][uj] = drho;
    };

    // FP32 moments of a pulled row (zero at solid nodes): formed when the row
    // arrives, they give the row's entry in Q (drho) and, a row later, the
    // collision's input, so only the request buffers hold populations
    auto moments_row = [&](const float (&f)[9], bool fluid, unsigned sm) {
        return fluid ? moments_of(f, sm != 0u) : Mom<float>{0.f, 0.f, 0.f, 0.f, 0.f};
    };
    // Requests run one row ahead of the arithmetic; the two request buffers swap
    // roles every row (the loop is unrolled by two), so a finished request is
    // never copied: a copy would wait for every load in flight.
    float fa[9], fb[9];
    RowInfo ri = row_info(g, s.ya - 1);
    bool fl = !(L.t0 && ri.w0);
    unsigned sm = solid_bits(L, ri);
    pull_lane(fs, L, ri, sm, fa);
    q_store(s4(s.ya - 1 + yo), moments_row(fa, fl, sm).drho);
    ri = row_info(g, s.ya);
    unsigned sm_cur = solid_bits(L, ri);
    bool fl_cur = !(L.t0 && ri.w0);
    pull_lane(fs, L, ri, sm_cur, fa);
    Mom<float> mom_cur = moments_row(fa, fl_cur, sm_cur);
    q_store(s4(s.ya + yo), mom_cur.drho);
    RowInfo ri_n = row_info(g, s.ya + 1);
    unsigned sm_n = solid_bits(L, ri_n);
    bool fl_n = !(L.t0 && ri_n.w0);
    pull_lane(fs, L, ri_n, sm_n, fb);

    // one row y: fn holds the request for row y+1, fp receives the one for row y+2
    auto iter = [&](int y, const float (&fn)[9], float (&fp)[9]) {
        const int yr = y + yo;
        // request for row y+2 (in the last row of the chunk a repeat of the
        // previous one: cache hits, unused)
        const RowInfo ri_p = row_info(g, y + 1 < s.yb ? y + 2 : y + 1);
        const unsigned sm_p = solid_bits(L, ri_p);
        const bool fl_p = !(L.t0 && ri_p.w0);
        pull_lane(fs, L, ri_p, sm_p, fp);
        __builtin_amdgcn_sched_barrier(0);
        const Mom<float> mom_n = moments_row(fn, fl_n, sm_n);
        q_store(s4(yr + 1), mom_n.drho);
        lds_barrier();
        if (out_col && fl_cur) {
            float dxf, dyf, lapf;
            stencil3(Q[s4(yr - 1)], Q[s4(yr)], Q[s4(yr + 1)], uj, sm_cur, G2, dxf, dyf, lapf);
            CT o[9];
            vdw_node_collide<CT, FORCE>(c, mom_cur, sm_cur, dxf, dyf, lapf, o);
            const int srow = row_info(g, y).y0 * fd.rb;
#pragma unroll
            for (int i = 0; i < 9; ++i) st(fd, (float)o[i], L.b0, i * fd.pb + srow);
        }
        mom_cur = mom_n;
        sm_cur = sm_n;
        fl_cur = fl_n;
        sm_n = sm_p;
        fl_n = fl_p;
    };
    for (int y = s.ya; y < s.yb; y += 2) {
        iter(y, fb, fa);
        if (y + 1 >= s.yb) break;
        iter(y + 1, fa, fb);
    }
}

}  // namespace lbk
