// Row-sweep ("strip") kernels of lbcap: the same time step as lb_step_kernel,
// organised for HBM traffic instead of for tiles.
//
// One wavefront owns a strip of 64 lattice columns, xs-1 .. xs+62, and marches
// along y through a chunk of rows.  Lanes 1..62 produce the outputs of columns
// xs .. xs+61; lanes 0 and 63 are the one-column halo and only supply
// velocities and chemical potentials to their neighbours.  Rows of the order
// field, of u and of mu live in small LDS ring buffers, so along y every
// population plane row is read from memory exactly once per step and no row
// is recomputed; along x the halo costs 2 of 64 lanes.  The populations of the
// row two ahead are requested before the current row is finished (software
// pipelining), which keeps enough loads in flight per wave to cover HBM
// latency without a large occupancy.
//
// The collision (moments, velocity, relaxation, reconstruction) is evaluated in
// the arithmetic type CT (double by default): the shifted FP32 populations are
// stored as before, but in FP32 arithmetic the rounding of the reconstructed
// populations of a steady flow repeats every step at every node and acts like
// a small spurious body force, which shifts a moving meniscus by ~1e-4 lattice
// units per 1e4 steps.  The order-parameter path (mu, g^eq, phi update) is
// FP32: its rounding does not accumulate that way.
#pragma once
#include "lb_kernels.h"

namespace lbk {

constexpr int STRIP_OUT = 62;     // output columns per strip
constexpr int SW = 64;            // lanes per strip = one wavefront
constexpr int PHW = SW + 2;       // phi row in LDS: columns xs-2 .. xs+63

struct StripDev {
    int cap, xs, ya, yb;          // output columns [xs, xs+62), output rows [ya, yb)
};

struct StripArgs {
    const CapDev* caps;
    const StripDev* strips;
    int nstrips;
    int xcd_group;                // 1: each XCD takes a contiguous run of strips
    float* arena0;
    float* arena1;
    int cur;
};

__device__ __forceinline__ int wrap_small(int v, int n) {
    // |v - [0, n)| is at most a few rows/columns here
    while (v < 0) v += n;
    while (v >= n) v -= n;
    return v;
}

// Pulled populations of node (x, y) (wrapped coordinates), or zeros for a solid node.
struct Pulled {
    float f[9];
    unsigned solid;   // neighbour solid bits
    bool fluid;
};

__device__ __forceinline__ void pull_node(const float* __restrict__ fs, long long P, const Geo& g, int x, int y,
                                          Pulled& p) {
    p.fluid = !g.solid(x, y);
    const Hood h = hood_of(g, x, y);
    p.solid = h.solid;
    if (p.fluid) {
        pull9(fs, P, g, h, x, y, p.f);
    } else {
#pragma unroll
        for (int i = 0; i < 9; ++i) p.f[i] = 0.f;
    }
}

// Moments in CT, velocity u = (j + F/2)/rho after the rest rule.
template <typename CT>
__device__ __forceinline__ Mom<CT> moments_ct(const CapDev& c, const Pulled& p, CT& ux, CT& uy, CT& F) {
    CT f[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) f[i] = (CT)p.f[i];
    const bool bnd = p.solid != 0u;
    Mom<CT> m = moments_of(f, bnd);
    F = bnd ? CT(0) : (CT)c.Fx;
    const CT inv_rho = CT(1) / ((CT)c.rho_ref + m.drho);
    ux = (m.jx + CT(0.5) * F) * inv_rho;
    uy = m.jy * inv_rho;
    return m;
}

// Stencils of Eq. (best) on three LDS rows (below, centre, above) at index j,
// wall ghosts as in `stencil`.
__device__ __forceinline__ void stencil3(const float* __restrict__ rm, const float* __restrict__ r0,
                                         const float* __restrict__ rp, int j, unsigned sm, float G2, float& dxq,
                                         float& dyq, float& lapq) {
    auto Q = [&](int dx, int dy) -> float { return (dy < 0 ? rm : (dy > 0 ? rp : r0))[j + dx]; };
    const float qc = r0[j];
    float v1 = Q(1, 0) - qc, v2 = Q(-1, 0) - qc, v3 = Q(0, 1) - qc, v4 = Q(0, -1) - qc;
    float v5 = Q(1, 1) - qc, v6 = Q(-1, -1) - qc, v7 = Q(-1, 1) - qc, v8 = Q(1, -1) - qc;
    if (sm) {
        if (sm & (1u << 1)) v1 = (Q(-1, 0) - qc) - G2;
        if (sm & (1u << 2)) v2 = (Q(1, 0) - qc) - G2;
        if (sm & (1u << 3)) v3 = (Q(0, -1) - qc) - G2;
        if (sm & (1u << 4)) v4 = (Q(0, 1) - qc) - G2;
        auto diag = [&](int dx, int dy, int dxi, int dyi) -> float {
            if (sm & (1u << dxi)) return (Q(-dx, dy) - qc) - G2;
            if (sm & (1u << dyi)) return (Q(dx, -dy) - qc) - G2;
            return (Q(-dx, -dy) - qc) - G2;
        };
        if (sm & (1u << 5)) v5 = diag(1, 1, 1, 3);
        if (sm & (1u << 6)) v6 = diag(-1, -1, 2, 4);
        if (sm & (1u << 7)) v7 = diag(-1, 1, 2, 3);
        if (sm & (1u << 8)) v8 = diag(1, -1, 1, 4);
    }
    dxq = ((v5 + v8) - (v7 + v6) + 4.f * (v1 - v2)) * (1.f / 12.f);
    dyq = ((v5 + v7) - (v8 + v6) + 4.f * (v3 - v4)) * (1.f / 12.f);
    lapq = (((v5 + v6) + (v7 + v8)) + 4.f * ((v1 + v2) + (v3 + v4))) * (1.f / 6.f);
}

__device__ __forceinline__ int strip_index(const StripArgs& a) {
    if (!a.xcd_group) return blockIdx.x;
    const int per = (a.nstrips + 7) >> 3;
    return (blockIdx.x & 7) * per + (blockIdx.x >> 3);
}

// ---- binary model --------------------------------------------------------------
template <bool INIT, typename CT>
__global__ void __launch_bounds__(SW) lb_strip_bin(StripArgs a) {
    const int si = strip_index(a);
    if (si >= a.nstrips) return;
    const StripDev s = a.strips[si];
    const CapDev& c = a.caps[s.cap];
    const Geo g = geo_of(c);
    const long long P = c.plane;
    const int sb = a.cur ^ c.par;
    const float* __restrict__ src = sb ? a.arena1 : a.arena0;
    float* __restrict__ dst = sb ? a.arena0 : a.arena1;
    const float* __restrict__ fs = src + c.off_f;
    const float* __restrict__ ps = src + c.off_phi;
    float* __restrict__ fd = dst + c.off_f;
    float* __restrict__ pd = dst + c.off_phi;

    __shared__ float PH[5][PHW];      // phi rows, column xs-2+j at index j
    __shared__ float UX[3][SW], UY[3][SW], MU[3][SW];   // column xs-1+k at lane k

    const int k = threadIdx.x;
    const int xl = s.xs + k - 1;                 // lane column (unwrapped)
    const int col = wrap_small(xl, g.nx);
    const bool out_col = k >= 1 && k <= STRIP_OUT && xl < g.nx;
    const float G2 = 2.f * c.G;
    const float kap = c.kappa, Gam = c.Gamma;
    auto slot5 = [&](int y) { return (y - s.ya + 10) % 5; };
    auto slot3 = [&](int y) { return (y - s.ya + 9) % 3; };

    auto load_phi_row = [&](int y, float& main, float& extra) {
        const int yw = wrap_small(y, g.ny);
        main = g.solid(col, yw) ? 0.f : ps[(long long)yw * g.pitch + col];
        extra = 0.f;
        if (k < 2) {
            const int xe = wrap_small(k == 0 ? s.xs - 2 : s.xs + SW - 1, g.nx);
            extra = g.solid(xe, yw) ? 0.f : ps[(long long)yw * g.pitch + xe];
        }
    };
    auto store_phi_row = [&](int y, float main, float extra) {
        float* r = PH[slot5(y)];
        r[k + 1] = main;
        if (k == 0) r[0] = extra;
        if (k == 1) r[PHW - 1] = extra;
    };
    auto pull_row = [&](int y, Pulled& p) {
        if (INIT) {
            const int yw = wrap_small(y, g.ny);
            p.fluid = !g.solid(col, yw);
            p.solid = hood_of(g, col, yw).solid;
#pragma unroll
            for (int i = 0; i < 9; ++i) p.f[i] = 0.f;   // f = f^eq at u = 0, rho = 1
        } else {
            pull_node(fs, P, g, col, wrap_small(y, g.ny), p);
        }
    };
    // u of a pulled row into the ring (float), moments kept by the caller
    auto put_u = [&](int y, const Pulled& p, Mom<CT>& m, CT& ux, CT& uy, CT& F) {
        if (p.fluid) {
            m = moments_ct<CT>(c, p, ux, uy, F);
        } else {
            m = Mom<CT>{CT(0), CT(0), CT(0), CT(0), CT(0)};
            ux = uy = F = CT(0);
        }
        UX[slot3(y)][k] = (float)ux;
        UY[slot3(y)][k] = (float)uy;
    };
    auto put_mu = [&](int y) {
        const int yw = wrap_small(y, g.ny);
        float v = 0.f;
        if (!g.solid(col, yw)) {
            float dx, dy, lap;
            stencil3(PH[slot5(y - 1)], PH[slot5(y)], PH[slot5(y + 1)], k + 1, hood_of(g, col, yw).solid, G2, dx,
                     dy, lap);
            v = Gam * (mu_bulk(c, PH[slot5(y)][k + 1]) - kap * lap);
        }
        MU[slot3(y)][k] = v;
    };

    // ---- prologue: rows ya-2 .. ya+1 of phi, u and mu of rows ya-1 and ya
    {
        float m0, e0;
        for (int y = s.ya - 2; y <= s.ya + 1; ++y) {
            load_phi_row(y, m0, e0);
            store_phi_row(y, m0, e0);
        }
    }
    Pulled pa;
    Mom<CT> mom_cur, mom_tmp;
    CT ux_cur, uy_cur, F_cur, tx, ty, tf;
    pull_row(s.ya - 1, pa);
    put_u(s.ya - 1, pa, mom_tmp, tx, ty, tf);
    pull_row(s.ya, pa);
    put_u(s.ya, pa, mom_cur, ux_cur, uy_cur, F_cur);
    unsigned solid_cur = pa.solid;
    bool fluid_cur = pa.fluid;
    __syncthreads();
    put_mu(s.ya - 1);
    put_mu(s.ya);
    // loads for the first iteration: pulled row ya+1, phi row ya+2
    Pulled pnext;
    float phn_m, phn_e;
    pull_row(s.ya + 1, pnext);
    load_phi_row(s.ya + 2, phn_m, phn_e);

    for (int y = s.ya; y < s.yb; ++y) {
        // (a) request the next iteration's data
        Pulled ppre;
        float php_m = 0.f, php_e = 0.f;
        const bool more = y + 1 < s.yb;
        if (more) {
            pull_row(y + 2, ppre);
            load_phi_row(y + 3, php_m, php_e);
        }
        // (b) row y+1: u, moments; phi row y+2
        store_phi_row(y + 2, phn_m, phn_e);
        Mom<CT> mom_next;
        CT ux_n, uy_n, F_n;
        put_u(y + 1, pnext, mom_next, ux_n, uy_n, F_n);
        const unsigned solid_next = pnext.solid;
        const bool fluid_next = pnext.fluid;
        __syncthreads();
        // (c) mu of row y+1
        put_mu(y + 1);
        __syncthreads();
        // (d) row y: collision and phi update
        const int yw = wrap_small(y, g.ny);
        if (out_col && fluid_cur) {
            const float* rm = PH[slot5(y - 1)];
            const float* r0 = PH[slot5(y)];
            const float* rp = PH[slot5(y + 1)];
            float dxf, dyf, lapf;
            stencil3(rm, r0, rp, k + 1, solid_cur, G2, dxf, dyf, lapf);
            const float phi = r0[k + 1];
            Mom<CT> m = mom_cur;
            if (INIT) {
                m.pxx = (CT)kap * ((CT)dxf * (CT)dxf - (CT)dyf * (CT)dyf);
                m.pxy = (CT)kap * (CT)dxf * (CT)dyf;
            }
            const CT ph = (CT)phi, phib = (CT)c.phib;
            const CT dX = m.drho * (CT(1) / CT(3)) +
                          CT(0.25) * (CT)c.B * ((ph - phib) * (ph + phib)) * (CT(3) * ph * ph + phib * phib) -
                          (CT)kap * ph * (CT)lapf;
            const CT pc = ph < CT(-1) ? CT(-1) : (ph > CT(1) ? CT(1) : ph);
            const CT nu = (CT)c.nu_g + CT(0.5) * (pc + CT(1)) * ((CT)c.nu_l - (CT)c.nu_g);
            const CT omega = CT(2) / (CT(6) * nu + CT(1));
            CT o[9];
            collide(c, m, (CT)c.rho_ref + m.drho, ux_cur, uy_cur, dX, CT(0), omega, (CT)dxf, (CT)dyf, F_cur, o);
            const long long idx = (long long)yw * g.pitch + col;
#pragma unroll
            for (int i = 0; i < 9; ++i) fd[(long long)i * P + idx] = (float)o[i];
            // phi(t+1) = phi(t) + sum_i [g^eq_i(source) - g^eq_i(r)]
            const float uxf = (float)ux_cur, uyf = (float)uy_cur;
            const float gmu = MU[slot3(y)][k];
            float go[9];
#pragma unroll
            for (int i = 1; i < 9; ++i) go[i] = geq_i(i, phi, uxf, uyf, gmu);
            float delta = 0.f;
#pragma unroll
            for (int i = 1; i < 9; ++i) {
                float gin;
                if ((solid_cur >> opp_(i)) & 1u) {
                    gin = go[opp_(i)];
                } else {
                    const int sy = y - ey_(i), sk = k - ex_(i);
                    gin = geq_i(i, PH[slot5(sy)][sk + 1], UX[slot3(sy)][sk], UY[slot3(sy)][sk], MU[slot3(sy)][sk]);
                }
                delta += gin - go[i];
            }
            pd[idx] = phi + delta;
        }
        // (e) rotate
        mom_cur = mom_next;
        ux_cur = ux_n;
        uy_cur = uy_n;
        F_cur = F_n;
        solid_cur = solid_next;
        fluid_cur = fluid_next;
        if (more) {
            pnext = ppre;
            phn_m = php_m;
            phn_e = php_e;
        }
        __syncthreads();
    }
}

// ---- van der Waals model ---------------------------------------------------------
template <bool INIT, typename CT>
__global__ void __launch_bounds__(SW) lb_strip_vdw(StripArgs a) {
    const int si = strip_index(a);
    if (si >= a.nstrips) return;
    const StripDev s = a.strips[si];
    const CapDev& c = a.caps[s.cap];
    const Geo g = geo_of(c);
    const long long P = c.plane;
    const int sb = a.cur ^ c.par;
    const float* __restrict__ src = sb ? a.arena1 : a.arena0;
    float* __restrict__ dst = sb ? a.arena0 : a.arena1;
    const float* __restrict__ fs = src + c.off_f;
    float* __restrict__ fd = dst + c.off_f;

    __shared__ float Q[3][SW];         // drho rows, column xs-1+k at lane k
    const int k = threadIdx.x;
    const int xl = s.xs + k - 1;
    const int col = wrap_small(xl, g.nx);
    const bool out_col = k >= 1 && k <= STRIP_OUT && xl < g.nx;
    const float G2 = 2.f * c.G;
    auto slot3 = [&](int y) { return (y - s.ya + 9) % 3; };
    // request a row: pulled populations (or, at initialisation, the initial field in f[0])
    auto request = [&](int y, Pulled& p) {
        const int yw = wrap_small(y, g.ny);
        if (INIT) {
            p.fluid = !g.solid(col, yw);
            p.solid = hood_of(g, col, yw).solid;
#pragma unroll
            for (int i = 1; i < 9; ++i) p.f[i] = 0.f;
            p.f[0] = p.fluid ? fs[(long long)yw * g.pitch + col] - c.rho_ref : 0.f;
        } else {
            pull_node(fs, P, g, col, yw, p);
        }
    };
    // drho of a requested row (for INIT, f[0] holds it)
    auto drho_of = [&](const Pulled& p) -> float { return p.fluid ? sum9(p.f) : 0.f; };

    Pulled pc0, pn;
    {
        Pulled t;
        request(s.ya - 1, t);
        Q[slot3(s.ya - 1)][k] = drho_of(t);
    }
    request(s.ya, pc0);
    Q[slot3(s.ya)][k] = drho_of(pc0);
    request(s.ya + 1, pn);
    for (int y = s.ya; y < s.yb; ++y) {
        Pulled pp;
        const bool more = y + 1 < s.yb;
        if (more) request(y + 2, pp);
        Q[slot3(y + 1)][k] = drho_of(pn);
        __syncthreads();
        const int yw = wrap_small(y, g.ny);
        if (out_col && pc0.fluid) {
            const float* rm = Q[slot3(y - 1)];
            const float* r0 = Q[slot3(y)];
            const float* rp = Q[slot3(y + 1)];
            float dxf, dyf, lapf;
            stencil3(rm, r0, rp, k, pc0.solid, G2, dxf, dyf, lapf);
            const bool bnd = pc0.solid != 0u;
            const CT F = bnd ? CT(0) : (CT)c.Fx;
            Mom<CT> m;
            if (INIT) {
                m.drho = (CT)r0[k];
                m.jx = m.jy = CT(0);
                m.pxx = (CT)c.kappa * ((CT)dxf * (CT)dxf - (CT)dyf * (CT)dyf);
                m.pxy = (CT)c.kappa * (CT)dxf * (CT)dyf;
            } else {
                CT f[9];
#pragma unroll
                for (int i = 0; i < 9; ++i) f[i] = (CT)pc0.f[i];
                m = moments_of(f, bnd);
            }
            const CT rho_ref = (CT)c.rho_ref;
            const CT rho = rho_ref + m.drho;
            const CT inv_rho = CT(1) / rho;
            const CT ux = (m.jx + CT(0.5) * F) * inv_rho;
            const CT uy = m.jy * inv_rho;
            const CT T = (CT)c.T, av = (CT)c.a;
            const CT ib = CT(1) / (CT(1) - (CT)c.b * rho);
            const CT dX = m.drho * (T * ib * (CT)c.ibr - av * (rho + rho_ref)) - (CT)c.kappa * rho * (CT)lapf;
            const CT omega = (CT)c.omega_l;
            CT lam = CT(0);
            if (c.lam_on != 0.f) {
                const CT dp0 = T * ib * ib - CT(2) * av * rho;
                lam = (CT(1) / omega - CT(0.5)) * (CT(1) / CT(3) - dp0);
            }
            CT o[9];
            collide(c, m, rho, ux, uy, dX, lam, omega, (CT)dxf, (CT)dyf, F, o);
            const long long idx = (long long)yw * g.pitch + col;
#pragma unroll
            for (int i = 0; i < 9; ++i) fd[(long long)i * P + idx] = (float)o[i];
        }
        pc0 = pn;
        if (more) pn = pp;
        __syncthreads();
    }
}

}  // namespace lbk
