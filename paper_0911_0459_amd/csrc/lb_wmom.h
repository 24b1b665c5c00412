// Wide row sweep of the binary model over a post-collision state stored as
// seven moment planes ("moment storage", schedule 6).
//
// With the rates of Appendix A the moments e, eps, qx and qy relax fully to
// their equilibria, so the nine post-collision populations of a node follow
// from seven numbers (PostState: rho - rho_ref, j*, the axis and diagonal
// common parts b and d, pxx*, pxy*).  This sweep stores those seven (j* as
// j*/3), FP32, and phi: 32 bytes per node and step instead of 40 of the
// population storage.  phi is in fixed point, as in every binary sweep
// (phi_of_fixed).
//
// Streaming needs the populations of the neighbours, so each lane loads the
// state of its own column only (aligned 256-byte row segments), rebuilds the
// nine populations (FP32, from j/3: see pops_of_stored) and puts them into
// LDS, where the pulls read them.  The halo wavefront's lanes 0..3 (columns
// xs-1, xs+192, xs-2, xs+193) load and rebuild the columns the main lanes'
// pulls and stencils reach, as they load phi in lb_wide_bin.
//
// Per sweep row y, three phases:
//   1. requests for row y+3 (state and phi); row y+2 rebuilt from the state
//      requested a row earlier, its phi into the phi ring;
//   -- barrier --
//   2. pulls of row y+1 (moments, u), the stencils of phi and Gamma mu of row
//      y+1 (its part A of g^eq);
//   -- barrier --
//   3. collision and phi update of row y, state and phi stored.
// A row's populations are kept in LDS only as long as some pull reads them:
// f4, f6, f8 (streamed downwards) until the pull of the row itself (its
// bounce-back), f1, f2 likewise, f3, f5, f7 (streamed upwards) until the pull
// of the row above; f0 never leaves the lane (it stays in a register for one
// row).  So the rings hold 2, 2 and 3 rows.  Phase 1 of row y+1 overwrites only
// entries that phase 2 of row y or earlier was the last to read: every
// wavefront has passed row y's second barrier before it starts row y+1.  phi
// is read by the stencils (phase 2) and phi updates (phase 3) of rows up to
// two apart, and a wavefront may be in phase 1 of row y+1 while another is in
// phase 3 of row y: a ring of six rows.  u and A of a row are written in phase
// 2 and read by the phi updates of the three rows around it: a ring of three.
// The LDS total (26 KB) admits six workgroups per CU.
// The loop starts four rows before the chunk with the later phases switched off
// until their rows begin, so that every row of every phase is computed by the
// same copy of the loop body (unrolled by two) whatever the chunking.
#pragma once
#include "lb_wide.h"

namespace lbk {

constexpr int NMOM = 7;   // planes of the stored post-collision state

// The stored planes: rho - rho_ref, jx*/3, jy*/3, b, d, pxx*, pxy*.  The
// momentum is stored divided by 3 because the populations take j/3 and
// j/12 = (j/3)/4: rebuilt from j itself in FP32, the rounded constants 1/3 and
// 1/12 (both 3e-8 too large) would amplify the streamed momentum by that much
// every step, a bias that moves an interface measurably over 10^4 steps.  From
// j/3 the rebuild uses exact scalings by powers of two and rounded sums only.
__device__ __forceinline__ void pops_of_stored(const float (&m)[NMOM], float (&f)[9]) {
    const float a7 = 0.25f * m[5], a8 = 0.25f * m[6];
    const float jx3 = m[1], jy3 = m[2];
    const float jpp = 0.25f * (jx3 + jy3), jpm = 0.25f * (jx3 - jy3);
    const float cx = m[3] + a7, cy = m[3] - a7, cp = m[4] + a8, cm = m[4] - a8;
    f[1] = cx + jx3;
    f[2] = cx - jx3;
    f[3] = cy + jy3;
    f[4] = cy - jy3;
    f[5] = cp + jpp;
    f[6] = cp - jpp;
    f[7] = cm - jpm;
    f[8] = cm + jpm;
    f[0] = m[0] - 4.f * (m[3] + m[4]);
}

// Reads the state of step t-1 (seven planes) and phi(t) of one wide strip
// chunk, writes the state of step t and phi(t+1).
template <typename MT, typename CT, typename ST = CT, bool FORCE = true>
__global__ void __launch_bounds__(WIDE_THREADS, 6) lb_wmom_bin(StripArgs a) {
    const int si = strip_index(a);
    if (si < 0) return;
    const StripDev s = a.strips[si];
    const CapDev c = a.caps[s.cap];
    const Geo g = geo_of(c);
    const int P = (int)c.plane;
    const int sb = a.cur ^ c.par;
    const Planes ms = planes_of((sb ? a.arena1 : a.arena0) + c.off_f, NMOM, P, c.pitch);
    const Planes ps = planes_of((sb ? a.arena1 : a.arena0) + c.off_phi, 1, P, c.pitch);
    const Planes md = planes_of((sb ? a.arena0 : a.arena1) + c.off_f, NMOM, P, c.pitch);
    const Planes pd = planes_of((sb ? a.arena0 : a.arena1) + c.off_phi, 1, P, c.pitch);

    // columns xs-2 .. xs+193 throughout
    __shared__ float PH[6][WP];      // phi
    __shared__ float UA[3][3][WP];   // ux, uy, A
    __shared__ float FU[3][3][WP];   // f3, f5, f7
    __shared__ float FD[2][3][WP];   // f4, f6, f8
    __shared__ float FH[2][2][WP];   // f1, f2

    const WideLane W = wide_lane();
    // lanes past column xe+1 (the last one that an output column reads) repeat
    // that column: their loads share its addresses
    const int xl = min(s.xs + W.dx, s.xe + 1);
    const LaneCols L = lane_cols(g, xl);
    const bool out_col = W.main && xl < s.xe;
    const int pj = W.pj, qj = W.qj;
    const float G2 = 2.f * c.G;
    const float kap = c.kappa, Gam = c.Gamma;
    // row y (the row finished in phase 3) has index t6 modulo 6; the slot of row
    // y + d in a ring of 6, 3 or 2 rows is its index modulo the ring size
    int t6 = 0;
    auto m6 = [&](int d) {   // -2 <= d <= 3
        int v = t6 + d;
        v += v < 0 ? 6 : 0;
        v -= v >= 6 ? 6 : 0;
        return v;
    };
    auto m3 = [&](int d) {
        const int v = m6(d);
        return v >= 3 ? v - 3 : v;
    };
    auto m2 = [&](int d) { return m6(d) & 1; };

    struct Ahead {
        float m[NMOM];   // state of the requested row
        float pm;        // its phi
        RowInfo r;
    };
    auto request = [&](int y, Ahead& q) {
        q.r = row_info(g, y);
        const int srow = q.r.y0 * ms.rb;
#pragma unroll
        for (int k = 0; k < NMOM; ++k) q.m[k] = ld(ms, L.b0, k * ms.pb + srow);
        q.pm = ld(ps, L.b0, q.r.y0 * ps.rb);
    };

    // what phase 2 leaves for the collision of its row in phase 3.  Two of them
    // swap roles every row (the loop is unrolled by two); a lane that does not
    // pull a row (a halo lane, a solid node) leaves the older contents, which
    // no collision reads
    struct Pulled {
        Mom<float> mom;
        float dx, dy, lap;   // stencils of phi
    };
    Ahead A, B;
    request(s.ya - 2, A);
    Pulled PA{{0.f, 0.f, 0.f, 0.f, 0.f}, 0.f, 0.f, 0.f}, PB = PA;
    unsigned sm_cur = 0u;
    bool fl_cur = false;
    float f0_cur = 0.f;   // f0 of row y+1 (this lane's column)
    // phi of this lane's column in fixed point, rows y+1 and y (the update adds to it)
    int q_next = 0, q_cur = 0;

    // iteration y: n holds the requests for row y+2, p receives those for row y+3;
    // cur holds row y's pulls, nxt receives row y+1's
    auto iter = [&](int y, const Ahead& n, Ahead& p, const Pulled& cur, Pulled& nxt) {
        // ---- phase 1: requests for row y+3 (past the chunk's last rebuilt row,
        // yb+1, a repeat of it: cache hits, unused); row y+2 rebuilt, its phi
        request(y + 3 <= s.yb + 1 ? y + 3 : s.yb + 1, p);
        __builtin_amdgcn_sched_barrier(0);
        float f0_next = 0.f;
        const int q_new = __builtin_bit_cast(int, n.pm);   // row y+2
        if (W.ph) {
            float f[9];
            pops_of_stored(n.m, f);
            const int u = m3(2), h = m2(2);
            FU[u][0][pj] = f[3];
            FU[u][1][pj] = f[5];
            FU[u][2][pj] = f[7];
            FD[h][0][pj] = f[4];
            FD[h][1][pj] = f[6];
            FD[h][2][pj] = f[8];
            FH[h][0][pj] = f[1];
            FH[h][1][pj] = f[2];
            f0_next = f[0];
            PH[m6(2)][pj] = (L.t0 && n.r.w0) ? 0.f : phi_of_fixed(n.pm);
        }
        lds_barrier();
        // ---- phase 2: pulls, moments and u of row y+1; stencils and A of row y+1
        const RowInfo rn = row_info(g, y + 1);
        const unsigned sm_n = solid_bits(L, rn);
        const bool fl_n = !(L.t0 && rn.w0);
        if (y >= s.ya - 2 && W.um) {
            float ux = 0.f, uy = 0.f, am = 0.f;
            if (fl_n) {
                const int u0 = m3(0), u1 = m3(1), h1 = m2(1), h2 = m2(2);
                // streaming source of direction i: row y+1-ey_i, column offset -ex_i
                auto src = [&](int i) -> const float* {
                    switch (i) {
                        case 1: return &FH[h1][0][pj - 1];
                        case 2: return &FH[h1][1][pj + 1];
                        case 3: return &FU[u0][0][pj];
                        case 4: return &FD[h2][0][pj];
                        case 5: return &FU[u0][1][pj - 1];
                        case 6: return &FD[h2][1][pj + 1];
                        case 7: return &FU[u0][2][pj + 1];
                        default: return &FD[h2][2][pj - 1];
                    }
                };
                // the node's own population i (row y+1), taken by bounce-back
                auto own = [&](int i) -> const float* {
                    switch (i) {
                        case 1: return &FH[h1][0][pj];
                        case 2: return &FH[h1][1][pj];
                        case 3: return &FU[u1][0][pj];
                        case 4: return &FD[h1][0][pj];
                        case 5: return &FU[u1][1][pj];
                        case 6: return &FD[h1][1][pj];
                        case 7: return &FU[u1][2][pj];
                        default: return &FD[h1][2][pj];
                    }
                };
                float f[9];
                f[0] = f0_cur;
#pragma unroll
                for (int i = 1; i < 9; ++i) {
                    const bool bb = (sm_n >> opp_(i)) & 1u;
                    f[i] = *(bb ? own(opp_(i)) : src(i));
                }
                const bool bnd = sm_n != 0u;
                nxt.mom = moments_of(f, bnd);
                const float F = bnd ? 0.f : c.Fx;
                const float inv_rho = recip(c.rho_ref + nxt.mom.drho);
                ux = (nxt.mom.jx + 0.5f * F) * inv_rho;
                uy = nxt.mom.jy * inv_rho;
                stencil3(PH[m6(0)], PH[m6(1)], PH[m6(2)], qj, sm_n, G2, nxt.dx, nxt.dy, nxt.lap);
                const float ph = PH[m6(1)][qj];
                const float gmu = Gam * (mu_bulk(c, ph) - kap * nxt.lap);
                am = gmu - 0.5f * ph * (ux * ux + uy * uy);
            }
            const int u1 = m3(1);
            UA[u1][0][qj] = ux;
            UA[u1][1][qj] = uy;
            UA[u1][2][qj] = am;
        }
        lds_barrier();
        // ---- phase 3: collision and phi update of row y (main lanes)
        if (y >= s.ya && out_col && fl_cur) {
            const float phi = PH[m6(0)][pj];
            const int u0 = m3(0);
            const float uxf = UA[u0][0][pj], uyf = UA[u0][1][pj];
            const PostState<CT> st8 =
                bin_node_state<CT, ST, FORCE>(c, cur.mom, sm_cur, phi, cur.dx, cur.dy, cur.lap, uxf, uyf);
            const int srow = row_info(g, y).y0 * md.rb;
            st(md, (float)st8.drho, L.b0, 0 * md.pb + srow);
            st(md, (float)third(st8.jx), L.b0, 1 * md.pb + srow);
            st(md, (float)third(st8.jy), L.b0, 2 * md.pb + srow);
            st(md, (float)st8.b, L.b0, 3 * md.pb + srow);
            st(md, (float)st8.d, L.b0, 4 * md.pb + srow);
            st(md, (float)st8.pxx, L.b0, 5 * md.pb + srow);
            st(md, (float)st8.pxy, L.b0, 6 * md.pb + srow);
            // the phi update below is not to be interleaved with the collision
            // (its LDS reads would be hoisted into the collision's register peak)
            __builtin_amdgcn_sched_barrier(0);
            const float dphi = phi_delta(sm_cur, phi, uxf, uyf, UA[u0][2][pj],
                                         [&](int i, float& am, float& pp, float& x, float& yy) {
                                             const int un = m3(-ey_(i)), kn = pj - ex_(i);
                                             am = UA[un][2][kn];
                                             pp = PH[m6(-ey_(i))][kn];
                                             x = UA[un][0][kn];
                                             yy = UA[un][1][kn];
                                         });
            st(pd, phi_bits(q_cur + fixed_of_phi(dphi)), L.b0, srow);
        }
        // ---- rotate the row state
        sm_cur = sm_n;
        fl_cur = fl_n;
        f0_cur = f0_next;
        q_cur = q_next;
        q_next = q_new;
        t6 = t6 == 5 ? 0 : t6 + 1;
    };
    for (int y = s.ya - 4; y < s.yb; y += 2) {
        iter(y, A, B, PA, PB);
        if (y + 1 >= s.yb) break;
        iter(y + 1, B, A, PB, PA);
    }
}

// In-place conversion of one arena's f regions (every capillary: blockIdx.y
// strides over them)
// between the nine populations and the seven-plane post-collision state: the
// library switches the storage when a launch configuration of the other
// storage is set.  From populations (which a step leaves in the seven-
// dimensional post-collision space): drho = sum f, j/3 with j = sum e f, b and
// d the means of the axis and of the diagonal populations,
// pxx* = (f1+f2)-(f3+f4), pxy* = (f5+f6)-(f7+f8); back by the inverse map.
// FP64 arithmetic, one rounding per stored value.  (phi is in fixed point in
// either storage.)
template <bool TO_STATE>
__global__ void __launch_bounds__(256) lb_convert_kernel(const CapDev* caps, int ncaps, float* arena) {
    for (int cap = blockIdx.y; cap < ncaps; cap += gridDim.y) {
        const CapDev c = caps[cap];
        float* base = arena + c.off_f;
        for (long long k = blockIdx.x * 256LL + threadIdx.x; k < c.plane; k += 256LL * gridDim.x) {
            float* p = base + k;
            if (TO_STATE) {
                double f[9];
#pragma unroll
                for (int i = 0; i < 9; ++i) f[i] = p[i * c.plane];
                const double ax = (f[1] + f[2]), ay = (f[3] + f[4]), dp = (f[5] + f[6]), dm = (f[7] + f[8]);
                const float m[NMOM] = {(float)(f[0] + ((ax + ay) + (dp + dm))),
                                       (float)((((f[1] - f[2]) + (f[5] - f[6])) + (f[8] - f[7])) / 3.0),
                                       (float)((((f[3] - f[4]) + (f[5] - f[6])) + (f[7] - f[8])) / 3.0),
                                       (float)(0.25 * (ax + ay)),
                                       (float)(0.25 * (dp + dm)),
                                       (float)(ax - ay),
                                       (float)(dp - dm)};
#pragma unroll
                for (int i = 0; i < NMOM; ++i) p[i * c.plane] = m[i];
            } else {
                double m[NMOM], o[9];
#pragma unroll
                for (int i = 0; i < NMOM; ++i) m[i] = p[i * c.plane];
                pops_of_state(PostState<double>{m[0], 3.0 * m[1], 3.0 * m[2], m[3], m[4], m[5], m[6]}, o);
#pragma unroll
                for (int i = 0; i < 9; ++i) p[i * c.plane] = (float)o[i];
            }
        }
    }
}

}  // namespace lbk
