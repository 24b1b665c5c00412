// Wide row sweep of the binary model over a post-collision state stored as
// seven moment planes ("moment storage", schedule 6).
//
// With the rates of Appendix A the moments e, eps, qx and qy relax fully to
// their equilibria, so the nine post-collision populations of a node follow
// from seven numbers (PostState: rho - rho_ref, j*, the axis and diagonal
// common parts b and d, pxx*, pxy*).  This sweep stores those seven, FP32, and
// phi: 32 bytes per node and step instead of 40 of the population storage.
//
// Streaming needs the populations of the neighbours, so each lane loads the
// state of its own column only (aligned 256-byte row segments), rebuilds the
// nine populations in arithmetic type CT exactly as a population step forms
// them before its store, and puts them, FP32, into an LDS ring of three rows;
// the pulls of a row then read the ring.  The halo wavefront's lanes 0..3
// (columns xs-1, xs+192, xs-2, xs+193) load and rebuild the columns the main
// lanes' pulls and stencils reach, as they load phi in lb_wide_bin.
//
// Per sweep row y, three phases:
//   1. requests for row y+3 (state and phi); the ring row y+2 rebuilt from the
//      state requested a row earlier, phi row y+2 into the phi ring;
//   -- barrier --
//   2. pulls of row y+1 from the ring rows y..y+2 (moments, u), the stencils
//      of phi and Gamma mu of row y+1 (its part A of g^eq);
//   -- barrier --
//   3. collision and phi update of row y, state and phi stored.
// Phase 1 of row y+1 writes the population ring slot of row y-1+3 = y+2's
// predecessor... precisely: the slot of row y, which phase 2 of row y was the
// last to read (every wavefront passed row y's second barrier before it), and
// phi row y+3, which no stencil of rows y-1..y+1 reads (a ring of six rows).
// The loop starts four rows before the chunk with the later phases switched off
// until their rows begin, so that every row of every phase is computed by the
// same copy of the loop body (unrolled by two) whatever the chunking.
#pragma once
#include "lb_wide.h"

namespace lbk {

constexpr int NMOM = 7;   // planes of the stored post-collision state

// The populations of a stored state (FP32 planes as loaded), formed in
// arithmetic type CT like the population storage's and rounded to FP32 as it
// would store them.
template <typename CT>
__device__ __forceinline__ void pops_of_stored(const float (&m)[NMOM], float (&f)[9]) {
    const PostState<CT> s{(CT)m[0], (CT)m[1], (CT)m[2], (CT)m[3], (CT)m[4], (CT)m[5], (CT)m[6]};
    CT o[9];
    pops_of_state(s, o);
#pragma unroll
    for (int i = 0; i < 9; ++i) f[i] = (float)o[i];
}

// Reads the state of step t-1 (seven planes) and phi(t) of one wide strip
// chunk, writes the state of step t and phi(t+1).
// (LDS: the phi/u/A ring of lb_wide_bin and the population ring, 40 KB: four
// workgroups per CU)
template <typename MT, typename CT, typename ST = CT, bool FORCE = true>
__global__ void __launch_bounds__(WIDE_THREADS, 4) lb_wmom_bin(StripArgs a) {
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

    enum { R_PH = 0, R_UX = 1, R_UY = 2, R_AM = 3, RING = 6 };
    __shared__ float RG[RING][4][WP];   // phi, ux, uy, A of six rows (as lb_wide_bin)
    __shared__ float FR[3][9][WP];      // rebuilt populations of three rows, columns xs-2 .. xs+193

    const WideLane W = wide_lane();
    // lanes past column xe+1 (the last one that an output column reads) repeat
    // that column: their loads share its addresses
    const int xl = min(s.xs + W.dx, s.xe + 1);
    const LaneCols L = lane_cols(g, xl);
    const bool out_col = W.main && xl < s.xe;
    const int pj = W.pj, qj = W.qj;
    const float G2 = 2.f * c.G;
    const float kap = c.kappa, Gam = c.Gamma;
    // row y (the row finished in phase 3) is in phi/u/A slot ry; row y+2 is in
    // population slot fw
    int ry = 0, fw = 0;
    auto sl = [&](int d) {   // phi/u/A slot of row y + d, -2 <= d <= 3
        int v = ry + d;
        v += v < 0 ? RING : 0;
        v -= v >= RING ? RING : 0;
        return v;
    };
    auto fs3 = [&](int d) {   // population slot of row y + d, 0 <= d <= 2
        int v = fw + d + 1;   // row y + 2 is in slot fw
        v -= v >= 3 ? 3 : 0;
        v -= v >= 3 ? 3 : 0;
        return v;
    };

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

    Ahead A, B;
    request(s.ya - 2, A);
    Mom<float> mom_cur{0.f, 0.f, 0.f, 0.f, 0.f};
    unsigned sm_cur = 0u;
    bool fl_cur = false;
    float dx_cur = 0.f, dy_cur = 0.f, lap_cur = 0.f;

    // iteration y: n holds the requests for row y+2, p receives those for row y+3
    auto iter = [&](int y, const Ahead& n, Ahead& p) {
        // ---- phase 1: requests for row y+3 (past the chunk's last ring row,
        // yb+1, a repeat of it: cache hits, unused); ring row y+2 and phi row y+2
        request(y + 3 <= s.yb + 1 ? y + 3 : s.yb + 1, p);
        __builtin_amdgcn_sched_barrier(0);
        if (W.ph) {
            float f[9];
            pops_of_stored<CT>(n.m, f);
            const int sf = fw;
#pragma unroll
            for (int i = 0; i < 9; ++i) FR[sf][i][pj] = f[i];
            RG[sl(2)][R_PH][pj] = (L.t0 && n.r.w0) ? 0.f : n.pm;
        }
        lds_barrier();
        // ---- phase 2: pulls, moments and u of row y+1; stencils and A of row y+1
        Mom<float> mom_n{0.f, 0.f, 0.f, 0.f, 0.f};
        const RowInfo rn = row_info(g, y + 1);
        const unsigned sm_n = solid_bits(L, rn);
        const bool fl_n = !(L.t0 && rn.w0);
        float dx_n = 0.f, dy_n = 0.f, lap_n = 0.f;
        if (y >= s.ya - 2 && W.um) {
            float ux = 0.f, uy = 0.f, am = 0.f;
            if (fl_n) {
                const int sm1 = fs3(0), s0 = fs3(1), sp1 = fs3(2);
                float f[9];
                f[0] = FR[s0][0][pj];
#pragma unroll
                for (int i = 1; i < 9; ++i) {
                    const bool bb = (sm_n >> opp_(i)) & 1u;
                    const int sy = ey_(i) > 0 ? sm1 : (ey_(i) < 0 ? sp1 : s0);
                    const float* q = bb ? &FR[s0][opp_(i)][pj] : &FR[sy][i][pj - ex_(i)];
                    f[i] = *q;
                }
                const bool bnd = sm_n != 0u;
                mom_n = moments_of(f, bnd);
                const float F = bnd ? 0.f : c.Fx;
                const float inv_rho = 1.f / (c.rho_ref + mom_n.drho);
                ux = (mom_n.jx + 0.5f * F) * inv_rho;
                uy = mom_n.jy * inv_rho;
                stencil3(RG[sl(0)][R_PH], RG[sl(1)][R_PH], RG[sl(2)][R_PH], qj, sm_n, G2, dx_n, dy_n, lap_n);
                const float ph = RG[sl(1)][R_PH][qj];
                const float gmu = Gam * (mu_bulk(c, ph) - kap * lap_n);
                am = gmu - 0.5f * ph * (ux * ux + uy * uy);
            }
            RG[sl(1)][R_UX][qj] = ux;
            RG[sl(1)][R_UY][qj] = uy;
            RG[sl(1)][R_AM][qj] = am;
        }
        lds_barrier();
        // ---- phase 3: collision and phi update of row y (main lanes)
        if (y >= s.ya && out_col && fl_cur) {
            const int s0 = sl(0);
            const float phi = RG[s0][R_PH][pj];
            const PostState<CT> st8 = bin_node_state<CT, ST, FORCE>(c, mom_cur, sm_cur, phi, dx_cur, dy_cur, lap_cur);
            const int srow = row_info(g, y).y0 * md.rb;
            st(md, (float)st8.drho, L.b0, 0 * md.pb + srow);
            st(md, (float)st8.jx, L.b0, 1 * md.pb + srow);
            st(md, (float)st8.jy, L.b0, 2 * md.pb + srow);
            st(md, (float)st8.b, L.b0, 3 * md.pb + srow);
            st(md, (float)st8.d, L.b0, 4 * md.pb + srow);
            st(md, (float)st8.pxx, L.b0, 5 * md.pb + srow);
            st(md, (float)st8.pxy, L.b0, 6 * md.pb + srow);
            // the phi update below is not to be interleaved with the collision
            // (its LDS reads would be hoisted into the collision's register peak)
            __builtin_amdgcn_sched_barrier(0);
            const float uxf = RG[s0][R_UX][pj], uyf = RG[s0][R_UY][pj];
            const float dphi = phi_delta(sm_cur, phi, uxf, uyf, RG[s0][R_AM][pj],
                                         [&](int i, float& am, float& p, float& x, float& yy) {
                                             const int sn = sl(-ey_(i)), kn = pj - ex_(i);
                                             am = RG[sn][R_AM][kn];
                                             p = RG[sn][R_PH][kn];
                                             x = RG[sn][R_UX][kn];
                                             yy = RG[sn][R_UY][kn];
                                         });
            st(pd, phi + dphi, L.b0, srow);
        }
        // ---- rotate the row state
        mom_cur = mom_n;
        sm_cur = sm_n;
        fl_cur = fl_n;
        dx_cur = dx_n;
        dy_cur = dy_n;
        lap_cur = lap_n;
        ry = ry == RING - 1 ? 0 : ry + 1;
        fw = fw == 2 ? 0 : fw + 1;
    };
    for (int y = s.ya - 4; y < s.yb; y += 2) {
        iter(y, A, B);
        if (y + 1 >= s.yb) break;
        iter(y + 1, B, A);
    }
}

// In-place conversion of one arena's f regions (every capillary, blockIdx.y)
// between the nine populations and the seven-plane post-collision state: the
// library switches the storage when a launch configuration of the other
// storage is set.  From populations (which a step leaves in the seven-
// dimensional post-collision space): drho = sum f, j = sum e f, b and d the
// means of the axis and of the diagonal populations, pxx* = (f1+f2)-(f3+f4),
// pxy* = (f5+f6)-(f7+f8); back by pops_of_stored.  FP64 arithmetic.
template <bool TO_STATE>
__global__ void __launch_bounds__(256) lb_convert_kernel(const CapDev* caps, float* arena) {
    const CapDev c = caps[blockIdx.y];
    float* base = arena + c.off_f;
    for (long long k = blockIdx.x * 256LL + threadIdx.x; k < c.plane; k += 256LL * gridDim.x) {
        float* p = base + k;
        if (TO_STATE) {
            double f[9];
#pragma unroll
            for (int i = 0; i < 9; ++i) f[i] = p[i * c.plane];
            const double ax = (f[1] + f[2]), ay = (f[3] + f[4]), dp = (f[5] + f[6]), dm = (f[7] + f[8]);
            const float m[NMOM] = {(float)(f[0] + ((ax + ay) + (dp + dm))),
                                   (float)(((f[1] - f[2]) + (f[5] - f[6])) + (f[8] - f[7])),
                                   (float)(((f[3] - f[4]) + (f[5] - f[6])) + (f[7] - f[8])),
                                   (float)(0.25 * (ax + ay)),
                                   (float)(0.25 * (dp + dm)),
                                   (float)(ax - ay),
                                   (float)(dp - dm)};
#pragma unroll
            for (int i = 0; i < NMOM; ++i) p[i * c.plane] = m[i];
        } else {
            float m[NMOM], f[9];
#pragma unroll
            for (int i = 0; i < NMOM; ++i) m[i] = p[i * c.plane];
            pops_of_stored<double>(m, f);
#pragma unroll
            for (int i = 0; i < 9; ++i) p[i * c.plane] = f[i];
        }
    }
}

}  // namespace lbk
