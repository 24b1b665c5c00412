// HIP kernels of lbcap for gfx950 (CDNA4).
//
// One fused kernel performs a whole time step of the free-energy MRT scheme
// (Eq. latbolt, Eq. latbolt2, Appendix A) for one 64 x TY tile of nodes:
//
//   pull streaming of f*(t-1) (and g*) with bounce-back from solid sources
//   -> rest of boundary nodes (Sec. 2.2)
//   -> moments rho, j, pxx, pxy (and phi)
//   -> q = rho or phi into an LDS tile with a one-node halo; the halo values
//      are recomputed from their own pulled populations
//   -> stencils of Eq. (best), wall ghosts for solid neighbours (wetting)
//   -> bulk pressure, chemical potential, phi-dependent omega (Eq. nu)
//   -> equilibrium moments in closed form -> MRT relaxation in moment space
//   -> f*(t) = M^-1 m* written once per population (and g*(t) = g^eq).
//
// The 9x9 change of basis is done in registers: with the rates of Appendix A
// only rho, j, pxx and pxy of the pre-collision state survive the collision
// (e, eps, qx, qy relax fully to their equilibria), so M^-1 m* reduces to a
// handful of FMAs per population.  Setting boundary nodes to rest only changes
// j (and qx, qy, which the collision discards), so it is applied in moment
// space as j = 0.
//
// Populations are SoA FP32 planes [9][ny][pitch], x fastest, pitch a multiple
// of 64 floats; one wavefront covers one 64-wide row segment, so every load and
// store of a population is a contiguous 256-byte access.
#pragma once
#include "lb_internal.h"

namespace lbk {

__host__ __device__ constexpr int ex_(int i) {
    return (i == 1 || i == 5 || i == 8) ? 1 : ((i == 2 || i == 6 || i == 7) ? -1 : 0);
}
__host__ __device__ constexpr int ey_(int i) {
    return (i == 3 || i == 5 || i == 7) ? 1 : ((i == 4 || i == 6 || i == 8) ? -1 : 0);
}
__host__ __device__ constexpr int opp_(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }

constexpr int W2 = TILE_W + 2;  // LDS row length (tile plus halo)

struct Geo {
    int nx, ny, pitch, x_in, x_end, y0, y1;
    __device__ __forceinline__ bool tube_col(int x) const { return x >= x_in && x < x_end; }
    __device__ __forceinline__ bool wall_row(int y) const { return y < y0 || y >= y1; }
    __device__ __forceinline__ bool solid(int x, int y) const { return tube_col(x) && wall_row(y); }
};

__device__ __forceinline__ Geo geo_of(const CapDev& c) {
    Geo g;
    g.nx = c.nx;
    g.ny = c.ny;
    g.pitch = c.pitch;
    g.x_in = c.x_in;
    g.x_end = c.x_end;
    g.y0 = c.y0;
    g.y1 = c.y1;
    return g;
}

__device__ __forceinline__ int wrap_mod(int v, int n) {
    v %= n;
    return v < 0 ? v + n : v;
}

// 3x3 neighbourhood of a fluid node: wrapped coordinates and solid flags,
// indexed by D2Q9 direction d (neighbour r + e_d).
struct Hood {
    int xm, xp, ym, yp;
    unsigned solid;  // bit d set when neighbour r + e_d is solid (d = 1..8)
};

__device__ __forceinline__ Hood hood_of(const Geo& g, int x, int y) {
    Hood h;
    h.xm = x == 0 ? g.nx - 1 : x - 1;
    h.xp = x == g.nx - 1 ? 0 : x + 1;
    h.ym = y == 0 ? g.ny - 1 : y - 1;
    h.yp = y == g.ny - 1 ? 0 : y + 1;
    const bool cm = g.tube_col(h.xm), c0 = g.tube_col(x), cp = g.tube_col(h.xp);
    const bool rm = g.wall_row(h.ym), r0 = g.wall_row(y), rp = g.wall_row(h.yp);
    unsigned s = 0;
    s |= (cp && r0) << 1;  // (1,0)
    s |= (cm && r0) << 2;  // (-1,0)
    s |= (c0 && rp) << 3;  // (0,1)
    s |= (c0 && rm) << 4;  // (0,-1)
    s |= (cp && rp) << 5;  // (1,1)
    s |= (cm && rm) << 6;  // (-1,-1)
    s |= (cm && rp) << 7;  // (-1,1)
    s |= (cp && rm) << 8;  // (1,-1)
    h.solid = s;
    return h;
}

// Pull streaming of one population set at fluid node (x, y): direction i comes
// from r - e_i, which is the neighbour in direction opp(i); a solid source is
// replaced by the node's own opposite population (bounce-back).
__device__ __forceinline__ void pull9(const float* __restrict__ base, long long plane, const Geo& g,
                                      const Hood& h, int x, int y, float (&f)[9]) {
    const long long own = (long long)y * g.pitch + x;
    const int xs[3] = {h.xm, x, h.xp};
    const int ys[3] = {h.ym, y, h.yp};
    f[0] = base[own];
#pragma unroll
    for (int i = 1; i < 9; ++i) {
        const int sx = xs[1 - ex_(i)], sy = ys[1 - ey_(i)];
        const bool bb = (h.solid >> opp_(i)) & 1u;
        const long long idx = bb ? (long long)opp_(i) * plane + own
                                 : (long long)i * plane + (long long)sy * g.pitch + sx;
        f[i] = base[idx];
    }
}

__device__ __forceinline__ float sum9(const float (&f)[9]) {
    // pairwise order, identical for every node
    return ((f[0] + (f[1] + f[2])) + (f[3] + f[4])) + ((f[5] + f[6]) + (f[7] + f[8]));
}

// q of one LDS slot: sum of the pulled populations of the q-carrying set.
__device__ __forceinline__ float slot_q(const float* __restrict__ qbase, long long plane, const Geo& g,
                                        int x, int y) {
    Hood h = hood_of(g, x, y);
    float f[9];
    pull9(qbase, plane, g, h, x, y, f);
    return sum9(f);
}

template <int MODEL, int TY, bool INIT>
__device__ __forceinline__ void step_tile(const StepArgs& a, int tile, float* qs) {
    const TileDev t = a.tiles[tile];
    const CapDev& c = a.caps[t.cap];
    const Geo g = geo_of(c);
    const long long P = c.plane;
    const float* __restrict__ fsrc = a.src + c.off_f;
    const float* __restrict__ gsrc = a.src + c.off_g;
    const float* __restrict__ qsrc = MODEL == 0 ? fsrc : gsrc;
    const int lx = threadIdx.x, ly = threadIdx.y;
    const int tid = lx + TILE_W * ly;
    const int x = t.x0 + lx, y = t.y0 + ly;
    const bool own = (x < g.nx) && (y < g.ny) && c.active;
    const int xw = x < g.nx ? x : wrap_mod(x, g.nx);
    const int yw = y < g.ny ? y : wrap_mod(y, g.ny);
    const bool fluid = !g.solid(xw, yw);

    // ---- phase 1: own populations and q of every LDS slot -----------------
    float f[9];
    float qv = 0.f;
    Hood h = hood_of(g, xw, yw);
    if (fluid) {
        if (INIT) {
            qv = a.init_q[c.off_f + (long long)yw * g.nx + xw];
        } else if (own) {
            pull9(fsrc, P, g, h, xw, yw, f);
            if (MODEL == 0) {
                qv = sum9(f);
            } else {
                float gg[9];
                pull9(gsrc, P, g, h, xw, yw, gg);
                qv = sum9(gg);
            }
        } else {
            qv = slot_q(qsrc, P, g, xw, yw);
        }
    }
    qs[(ly + 1) * W2 + lx + 1] = qv;
    constexpr int NH = 2 * W2 + 2 * TY;
    for (int k = tid; k < NH; k += TILE_W * TY) {
        int sx, sy;
        if (k < W2) {
            sx = k;
            sy = 0;
        } else if (k < 2 * W2) {
            sx = k - W2;
            sy = TY + 1;
        } else {
            const int m = k - 2 * W2;
            sx = (m & 1) ? W2 - 1 : 0;
            sy = 1 + (m >> 1);
        }
        const int gx = wrap_mod(t.x0 + sx - 1, g.nx);
        const int gy = wrap_mod(t.y0 + sy - 1, g.ny);
        float v = 0.f;
        if (!g.solid(gx, gy)) {
            if (INIT)
                v = a.init_q[c.off_f + (long long)gy * g.nx + gx];
            else
                v = slot_q(qsrc, P, g, gx, gy);
        }
        qs[sy * W2 + sx] = v;
    }
    __syncthreads();
    if (!(own && fluid)) return;

    // ---- phase 2: collision of the own node -------------------------------
    const unsigned sm = h.solid;
    const bool bnd = sm != 0u;
    float rho, jx, jy, pxx = 0.f, pxy = 0.f;
    if (INIT) {
        rho = MODEL == 0 ? qv : 1.f;
        jx = jy = 0.f;
    } else {
        rho = MODEL == 0 ? qv : sum9(f);
        jx = ((f[1] - f[2]) + (f[5] - f[6])) + (f[8] - f[7]);
        jy = ((f[3] - f[4]) + (f[5] - f[6])) + (f[7] - f[8]);
        pxx = (f[1] + f[2]) - (f[3] + f[4]);
        pxy = (f[5] + f[6]) - (f[7] + f[8]);
        if (bnd) jx = jy = 0.f;  // boundary node set to rest
    }
    const float F = bnd ? 0.f : c.Fx;

    // stencils of Eq. (best) with wall ghosts (rule W)
    const int cidx = (ly + 1) * W2 + lx + 1;
    const float qc = qs[cidx];
    float v1 = qs[cidx + 1], v2 = qs[cidx - 1], v3 = qs[cidx + W2], v4 = qs[cidx - W2];
    float v5 = qs[cidx + W2 + 1], v6 = qs[cidx - W2 - 1], v7 = qs[cidx + W2 - 1], v8 = qs[cidx - W2 + 1];
    if (bnd) {
        const float G2 = 2.f * c.G;
        // axis neighbours: mirror through the node
        if (sm & (1u << 1)) v1 = qs[cidx - 1] - G2;
        if (sm & (1u << 2)) v2 = qs[cidx + 1] - G2;
        if (sm & (1u << 3)) v3 = qs[cidx - W2] - G2;
        if (sm & (1u << 4)) v4 = qs[cidx + W2] - G2;
        // diagonals: mirror across the wall that blocks them, else through the node
        // (dx, dy): the diagonal; dxi / dyi: direction indices of (dx,0) and (0,dy)
        auto diag = [&](int dx, int dy, int dxi, int dyi) -> float {
            if (sm & (1u << dxi)) return qs[cidx + dy * W2 - dx] - G2;
            if (sm & (1u << dyi)) return qs[cidx - dy * W2 + dx] - G2;
            return qs[cidx - dy * W2 - dx] - G2;
        };
        if (sm & (1u << 5)) v5 = diag(1, 1, 1, 3);
        if (sm & (1u << 6)) v6 = diag(-1, -1, 2, 4);
        if (sm & (1u << 7)) v7 = diag(-1, 1, 2, 3);
        if (sm & (1u << 8)) v8 = diag(1, -1, 1, 4);
    }
    const float dxq = ((v5 + v8) - (v7 + v6) + 4.f * (v1 - v2)) * (1.f / 12.f);
    const float dyq = ((v5 + v7) - (v8 + v6) + 4.f * (v3 - v4)) * (1.f / 12.f);
    const float lapq = (((v5 + v6) + (v7 + v8)) + 4.f * ((v1 + v2) + (v3 + v4)) - 20.f * qc) * (1.f / 6.f);

    if (INIT) {
        // moments of f^eq at u = 0: P_xx - P_yy and P_xy of Eq. (pt)
        pxx = c.kappa * (dxq * dxq - dyq * dyq);
        pxy = c.kappa * dxq * dyq;
    }

    const float inv_rho = 1.f / rho;
    const float ux = (jx + 0.5f * F) * inv_rho;
    const float uy = jy * inv_rho;

    // thermodynamics: X = p0 - kappa q lap q; lambda; omega
    float X, lam = 0.f, omega, mu = 0.f, phi = 0.f;
    if (MODEL == 0) {
        const float ib = 1.f / (1.f - c.b * rho);
        const float p0 = rho * c.T * ib - c.a * rho * rho;
        X = p0 - c.kappa * rho * lapq;
        omega = c.omega_l;
        if (c.lam_on != 0.f) {
            const float dp0 = c.T * ib * ib - 2.f * c.a * rho;
            lam = (1.f / omega - 0.5f) * (1.f / 3.f - dp0);
        }
    } else {
        phi = qc;
        const float p2 = phi * phi;
        const float p0 = rho * (1.f / 3.f) - 0.5f * c.A * p2 + 0.75f * c.B * p2 * p2;
        X = p0 - c.kappa * phi * lapq;
        mu = -c.A * phi + c.B * p2 * phi - c.kappa * lapq;
        const float pc = fminf(fmaxf(phi, -1.f), 1.f);
        const float nu = c.nu_g + 0.5f * (pc + 1.f) * (c.nu_l - c.nu_g);
        omega = 2.f / (6.f * nu + 1.f);
    }

    // equilibrium moments in closed form (M f^eq with the Eq. equilibrium weights)
    const float udq = ux * dxq + uy * dyq;
    const float trQ = rho * (ux * ux + uy * uy) + 4.f * lam * udq;
    const float dQ = rho * (ux * ux - uy * uy) + 2.f * lam * (ux * dxq - uy * dyq);
    const float Qxy = rho * ux * uy + lam * (ux * dyq + uy * dxq);
    const float grad2 = dxq * dxq + dyq * dyq;
    const float pxx_eq = c.kappa * (dxq * dxq - dyq * dyq) + dQ;
    const float pxy_eq = c.kappa * dxq * dyq + Qxy;

    // relaxed moments (e, eps, qx, qy at equilibrium; shear modes at rate omega)
    // plus the Guo source (I - S/2) M F in moment space
    const float uF = ux * F;
    float b = X * (1.f / 3.f) + trQ * (1.f / 12.f) + c.kappa * grad2 * (1.f / 12.f) + uF * (1.f / 12.f);
    float d = X * (1.f / 12.f) + trQ * (1.f / 12.f) - c.kappa * grad2 * (1.f / 24.f) + uF * (1.f / 12.f);
    const float hw = 1.f - 0.5f * omega;
    const float pxs = pxx - omega * (pxx - pxx_eq) + hw * 2.f * uF;
    const float pys = pxy - omega * (pxy - pxy_eq) + hw * (uy * F);
    const float jxs = jx + F, jys = jy;
    const float a7 = 0.25f * pxs, a8 = 0.25f * pys;
    const float jx3 = jxs * (1.f / 3.f), jy3 = jys * (1.f / 3.f);
    const float jpp = (jxs + jys) * (1.f / 12.f), jpm = (jxs - jys) * (1.f / 12.f);

    float o[9];
    o[1] = b + jx3 + a7;
    o[2] = b - jx3 + a7;
    o[3] = b + jy3 - a7;
    o[4] = b - jy3 - a7;
    o[5] = d + jpp + a8;
    o[6] = d - jpp + a8;
    o[7] = d - jpm - a8;
    o[8] = d + jpm - a8;
    o[0] = rho - 4.f * (b + d);

    float* __restrict__ fdst = a.dst + c.off_f;
    const long long own_idx = (long long)yw * g.pitch + xw;
#pragma unroll
    for (int i = 0; i < 9; ++i) fdst[(long long)i * P + own_idx] = o[i];

    if (MODEL == 1) {
        // g* = g^eq (all g rates are 1), Appendix A
        const float Gm = c.Gamma * mu;
        const float u2 = ux * ux + uy * uy;
        const float base_ax = (1.f / 3.f) * (Gm - 0.5f * phi * u2);
        const float base_dg = (1.f / 12.f) * (Gm - 0.5f * phi * u2);
        float gq[9];
        // axis: w = 1/3, e.u = +-ux / +-uy, 1.5 phi (e.u)^2 term
        gq[1] = base_ax + (1.f / 3.f) * phi * (ux + 1.5f * ux * ux);
        gq[2] = base_ax + (1.f / 3.f) * phi * (-ux + 1.5f * ux * ux);
        gq[3] = base_ax + (1.f / 3.f) * phi * (uy + 1.5f * uy * uy);
        gq[4] = base_ax + (1.f / 3.f) * phi * (-uy + 1.5f * uy * uy);
        const float upp = ux + uy, upm = ux - uy;
        gq[5] = base_dg + (1.f / 12.f) * phi * (upp + 1.5f * upp * upp);
        gq[6] = base_dg + (1.f / 12.f) * phi * (-upp + 1.5f * upp * upp);
        gq[7] = base_dg + (1.f / 12.f) * phi * (-upm + 1.5f * upm * upm);
        gq[8] = base_dg + (1.f / 12.f) * phi * (upm + 1.5f * upm * upm);
        gq[0] = phi - (5.f / 3.f) * Gm - (2.f / 3.f) * phi * u2;
        float* __restrict__ gdst = a.dst + c.off_g;
#pragma unroll
        for (int i = 0; i < 9; ++i) gdst[(long long)i * P + own_idx] = gq[i];
    }
}

template <int MODEL, int TY, bool INIT>
__global__ void __launch_bounds__(TILE_W* TY) lb_step_kernel(StepArgs a) {
    __shared__ float qs[(TY + 2) * W2];
    if (a.schedule == 2) {
        for (int tile = blockIdx.x; tile < a.ntiles; tile += gridDim.x) {
            step_tile<MODEL, TY, INIT>(a, tile, qs);
            __syncthreads();
        }
    } else {
        int tile = blockIdx.x;
        if (a.schedule == 1) {
            const int per = (a.ntiles + 7) >> 3;
            tile = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
        }
        if (tile < a.ntiles) step_tile<MODEL, TY, INIT>(a, tile, qs);
    }
}

// ---- macroscopic fields of one capillary -----------------------------------
// rho = sum f*, u = (j* - F/2)/rho (the collision added F to j), phi = sum g*.
template <int MODEL>
__global__ void lb_moments_kernel(const CapDev* caps, int cap, const float* __restrict__ st,
                                  float* rho_o, float* ux_o, float* uy_o, float* phi_o) {
    const CapDev& c = caps[cap];
    const Geo g = geo_of(c);
    const long long n = (long long)g.nx * g.ny;
    for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < n;
         k += (long long)gridDim.x * blockDim.x) {
        const int y = (int)(k / g.nx), x = (int)(k % g.nx);
        float r = 0.f, u = 0.f, v = 0.f, p = 0.f;
        if (!g.solid(x, y)) {
            const Hood h = hood_of(g, x, y);
            const long long own = (long long)y * g.pitch + x;
            float f[9];
#pragma unroll
            for (int i = 0; i < 9; ++i) f[i] = st[c.off_f + i * c.plane + own];
            r = sum9(f);
            const float jx = ((f[1] - f[2]) + (f[5] - f[6])) + (f[8] - f[7]);
            const float jy = ((f[3] - f[4]) + (f[5] - f[6])) + (f[7] - f[8]);
            const float F = h.solid ? 0.f : c.Fx;
            u = (jx - 0.5f * F) / r;
            v = jy / r;
            if (MODEL == 1) {
#pragma unroll
                for (int i = 0; i < 9; ++i) f[i] = st[c.off_g + i * c.plane + own];
                p = sum9(f);
            }
        }
        if (rho_o) rho_o[k] = r;
        if (ux_o) ux_o[k] = u;
        if (uy_o) uy_o[k] = v;
        if (phi_o) phi_o[k] = p;
    }
}

// ---- filled length of every capillary (one workgroup per capillary) --------
__device__ __forceinline__ float centre_q(const CapDev& c, const float* __restrict__ st, int MODEL,
                                          int x, int ya, int yb) {
    const long long base = MODEL == 0 ? c.off_f : c.off_g;
    float fa[9], fb[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        fa[i] = st[base + i * c.plane + (long long)ya * c.pitch + x];
        fb[i] = st[base + i * c.plane + (long long)yb * c.pitch + x];
    }
    return 0.5f * (sum9(fa) + sum9(fb));
}

__global__ void __launch_bounds__(256)
lb_interface_kernel(const CapDev* caps, int ncap, int model, const float* __restrict__ st,
                    float* l_now, float* hist, long long* hist_t, int* hist_n, int hist_cap,
                    long long t_now, int record) {
    const int cap = blockIdx.x;
    if (cap >= ncap) return;
    const CapDev& c = caps[cap];
    __shared__ int kmin_s;
    if (threadIdx.x == 0) kmin_s = 0x7fffffff;
    __syncthreads();
    const int H = c.y1 - c.y0;
    const int L = c.x_end - c.x_in;
    const int ya = (H % 2 == 0) ? c.y0 + H / 2 - 1 : c.y0 + (H - 1) / 2;
    const int yb = (H % 2 == 0) ? c.y0 + H / 2 : ya;
    int kmin = 0x7fffffff;
    for (int k = threadIdx.x; k < L; k += blockDim.x) {
        const float q = centre_q(c, st, model, c.x_in + k, ya, yb);
        if (q < c.q_mid) {
            kmin = k;
            break;  // later k of this thread are larger
        }
    }
    atomicMin(&kmin_s, kmin);
    __syncthreads();
    if (threadIdx.x == 0) {
        const int k = kmin_s;
        float l;
        if (k == 0x7fffffff)
            l = (float)L;
        else if (k == 0)
            l = 0.f;
        else {
            const float qp = centre_q(c, st, model, c.x_in + k - 1, ya, yb);
            const float qk = centre_q(c, st, model, c.x_in + k, ya, yb);
            l = (float)(k - 1) + (qp - c.q_mid) / (qp - qk);
        }
        l_now[cap] = l;
        if (record && c.active) {
            const int n = hist_n[cap];
            if (n < hist_cap) {
                hist[(long long)c.hist_off + n] = l + 0.5f * (float)H;
                hist_t[(long long)c.hist_off + n] = t_now;
            }
            hist_n[cap] = n + 1;
        }
    }
}

// ---- health scan: non-finite population or rho <= 0 -> flag per capillary ---
template <int MODEL>
__global__ void lb_health_kernel(const CapDev* caps, const TileDev* tiles, int ntiles,
                                 const float* __restrict__ st, int* flags) {
    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const TileDev t = tiles[tile];
        const CapDev& c = caps[t.cap];
        const Geo g = geo_of(c);
        for (int r = threadIdx.x / TILE_W; r < 8; r += blockDim.x / TILE_W) {
            const int x = t.x0 + (threadIdx.x % TILE_W), y = t.y0 + r;
            if (x >= g.nx || y >= g.ny || r >= t.rows || g.solid(x, y)) continue;
            const long long own = (long long)y * g.pitch + x;
            float s = 0.f;
            bool bad = false;
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                const float v = st[c.off_f + i * c.plane + own];
                bad |= !isfinite(v);
                s += v;
            }
            if (MODEL == 1) {
#pragma unroll
                for (int i = 0; i < 9; ++i) bad |= !isfinite(st[c.off_g + i * c.plane + own]);
            }
            if (bad || !(s > 0.f)) atomicOr(&flags[t.cap], 1);
        }
    }
}

}  // namespace lbk
