// HIP kernels of lbcap for gfx950 (CDNA4).
//
// One fused kernel performs a whole time step of the free-energy MRT scheme
// (Eq. latbolt, Eq. latbolt2, Appendix A) for one 64 x TY tile of nodes:
//
//   pull streaming of f*(t-1) with bounce-back from solid sources
//   -> rest of boundary nodes (Sec. 2.2)
//   -> moments rho, j, pxx, pxy
//   -> the order field q (rho, or phi) in an LDS tile with a halo
//   -> stencils of Eq. (best), wall ghosts for solid neighbours (wetting)
//   -> bulk pressure, chemical potential, phi-dependent omega (Eq. nu)
//   -> equilibrium moments in closed form -> MRT relaxation in moment space
//   -> f*(t) = M^-1 m* written once per population.
//
// The 9x9 change of basis is done in registers: with the rates of Appendix A
// only rho, j, pxx and pxy of the pre-collision state survive the collision
// (e, eps, qx, qy relax fully to their equilibria), so M^-1 m* reduces to a
// handful of FMAs per population.  Setting boundary nodes to rest only changes
// j (and qx, qy, which the collision discards), so it is applied in moment
// space as j = 0.
//
// Binary model: every relaxation rate of g is 1 (Appendix A), so g after
// collision is g^eq(phi, u, mu) of the node and is never stored.  Streaming
// then gives phi(r, t+1) = sum_i g^eq_i(r - e_i, t) (g^eq_opp(i)(r, t) for a solid
// source), which the kernel evaluates from phi, u and mu of the node and its
// eight neighbours: phi is read with a two-node halo (the neighbours' mu needs
// their Laplacian) and u of the one-node halo comes from the neighbours' own
// pulled populations.  The update is formed as the sum of the small
// differences g^eq_i(r - e_i) - g^eq_i(r) and added to the stored phi(t), a
// fixed-point number (phi_of_fixed), as a whole number of grid steps.
//
// Populations are SoA FP32 planes [9][ny][pitch], x fastest, pitch a multiple
// of 64 floats; one wavefront covers one 64-wide row segment, so every load and
// store of a population is a contiguous 256-byte access.
//
// FP32 storage keeps the accuracy of FP64 runs by storing f shifted by a
// constant rest state: s_i = f_i - r_i, where r is the equilibrium of density
// rho_ref at rest without gradients.  The reference carries density but no
// momentum and no stress, so j, pxx and pxy are sums of the small s_i, and the
// collision output is formed from differences to the reference (X - X_ref,
// rho - rho_ref) without cancelling large numbers.
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

constexpr int W2 = TILE_W + 2;  // LDS row: tile plus one-node halo
constexpr int W4 = TILE_W + 4;  // LDS row: tile plus two-node halo

template <int MODEL, int TY>
struct Lds {
    // vdW: q with a one-node halo.  Binary: phi with a two-node halo, then
    // ux, uy and mu with a one-node halo.
    static constexpr int PH = MODEL == 0 ? (TY + 2) * W2 : (TY + 4) * W4;
    static constexpr int R1 = (TY + 2) * W2;
    static constexpr int SIZE = MODEL == 0 ? PH : PH + 3 * R1;
};

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

// 3x3 neighbourhood of a node (wrapped coordinates): neighbour coordinates and
// solid flags, bit d set when neighbour r + e_d is solid (d = 1..8).
struct Hood {
    int xm, xp, ym, yp;
    unsigned solid;
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
    s |= (unsigned)(cp && r0) << 1;  // (1,0)
    s |= (unsigned)(cm && r0) << 2;  // (-1,0)
    s |= (unsigned)(c0 && rp) << 3;  // (0,1)
    s |= (unsigned)(c0 && rm) << 4;  // (0,-1)
    s |= (unsigned)(cp && rp) << 5;  // (1,1)
    s |= (unsigned)(cm && rm) << 6;  // (-1,-1)
    s |= (unsigned)(cm && rp) << 7;  // (-1,1)
    s |= (unsigned)(cp && rm) << 8;  // (1,-1)
    h.solid = s;
    return h;
}

// Pull streaming of the f set at fluid node (x, y): direction i comes from
// r - e_i, the neighbour in direction opp(i); a solid source is replaced by the
// node's own opposite population (bounce-back).  Loads FP32, returns type R.
template <typename R>
__device__ __forceinline__ void pull9(const float* __restrict__ base, long long plane, const Geo& g,
                                      const Hood& h, int x, int y, R (&f)[9]) {
    const long long own = (long long)y * g.pitch + x;
    f[0] = (R)base[own];
#pragma unroll
    for (int i = 1; i < 9; ++i) {
        const int sx = ex_(i) > 0 ? h.xm : (ex_(i) < 0 ? h.xp : x);
        const int sy = ey_(i) > 0 ? h.ym : (ey_(i) < 0 ? h.yp : y);
        const bool bb = (h.solid >> opp_(i)) & 1u;
        const long long idx = bb ? (long long)opp_(i) * plane + own
                                 : (long long)i * plane + (long long)sy * g.pitch + sx;
        f[i] = (R)base[idx];
    }
}

// Zeroth moment: the eight moving populations first (small), the rest
// population last, so the result is rounded once at its own magnitude.
template <typename R>
__device__ __forceinline__ R sum9(const R (&f)[9]) {
    return f[0] + (((f[1] + f[2]) + (f[3] + f[4])) + ((f[5] + f[6]) + (f[7] + f[8])));
}

// The stored phi (binary model) is a 32-bit fixed-point number with 29
// fraction bits, kept in the bits of its FP32 plane: a grid of 1.9e-9 instead
// of FP32's 6e-8 at |phi| ~ 1.  Each step adds its update as a whole number of
// grid steps, so that the small updates in the tails of an interface are kept
// instead of rounded away (FP32 storage loses phi systematically there, 2e-4
// of the total over 2e5 steps; the fixed point keeps it to 1e-8).  Range +-4.
constexpr float PHI_FIX_SCALE = 536870912.f;              // 2^29
constexpr float PHI_FIX_STEP = 1.f / 536870912.f;         // 2^-29 (exact)

template <typename R = float>
__device__ __forceinline__ R phi_of_fixed(float bits) {
    return (R)__builtin_bit_cast(int, bits) * (R)PHI_FIX_STEP;
}
// the nearest grid point of an update (saturating)
__device__ __forceinline__ int fixed_of_phi(float phi) { return (int)__builtin_rintf(phi * PHI_FIX_SCALE); }
__device__ __forceinline__ int fixed_of_phi(double phi) { return (int)__builtin_rint(phi * (double)PHI_FIX_SCALE); }
__device__ __forceinline__ float phi_bits(int q) { return __builtin_bit_cast(float, q); }

// Pre-collision moments of a pulled (shifted) population set; rest of boundary
// nodes applied as j = 0.
template <typename R>
struct Mom {
    R drho, jx, jy, pxx, pxy;
};

template <typename R>
__device__ __forceinline__ Mom<R> moments_of(const R (&f)[9], bool bnd) {
    Mom<R> m;
    m.drho = sum9(f);
    m.jx = ((f[1] - f[2]) + (f[5] - f[6])) + (f[8] - f[7]);
    m.jy = ((f[3] - f[4]) + (f[5] - f[6])) + (f[7] - f[8]);
    m.pxx = (f[1] + f[2]) - (f[3] + f[4]);
    m.pxy = (f[5] + f[6]) - (f[7] + f[8]);
    if (bnd) m.jx = m.jy = R(0);
    return m;
}

// Stencils of Eq. (best) around LDS index ci (row stride RS) with the wall
// ghost rule for solid neighbours: an axis neighbour is mirrored through the
// node; a diagonal one is mirrored across the wall that blocks it (the x wall
// first), or through the node at a convex corner; every ghost is lowered by
// 2G so that the normal derivative at a flat wall is G.
// The stencils are evaluated on the differences to the centre value, which are
// small and exact for close neighbours, so no sum of large values cancels.
template <int RS, typename R>
__device__ __forceinline__ void stencil(const R* __restrict__ q, int ci, unsigned sm, R G2, R& dxq, R& dyq,
                                        R& lapq) {
    const R qc = q[ci];
    R v1 = q[ci + 1] - qc, v2 = q[ci - 1] - qc, v3 = q[ci + RS] - qc, v4 = q[ci - RS] - qc;
    R v5 = q[ci + RS + 1] - qc, v6 = q[ci - RS - 1] - qc, v7 = q[ci + RS - 1] - qc, v8 = q[ci - RS + 1] - qc;
    if (sm) {
        if (sm & (1u << 1)) v1 = (q[ci - 1] - qc) - G2;
        if (sm & (1u << 2)) v2 = (q[ci + 1] - qc) - G2;
        if (sm & (1u << 3)) v3 = (q[ci - RS] - qc) - G2;
        if (sm & (1u << 4)) v4 = (q[ci + RS] - qc) - G2;
        // (dx, dy): the diagonal; dxi / dyi: direction indices of (dx,0) and (0,dy)
        auto diag = [&](int dx, int dy, int dxi, int dyi) -> R {
            if (sm & (1u << dxi)) return (q[ci + dy * RS - dx] - qc) - G2;
            if (sm & (1u << dyi)) return (q[ci - dy * RS + dx] - qc) - G2;
            return (q[ci - dy * RS - dx] - qc) - G2;
        };
        if (sm & (1u << 5)) v5 = diag(1, 1, 1, 3);
        if (sm & (1u << 6)) v6 = diag(-1, -1, 2, 4);
        if (sm & (1u << 7)) v7 = diag(-1, 1, 2, 3);
        if (sm & (1u << 8)) v8 = diag(1, -1, 1, 4);
    }
    dxq = ((v5 + v8) - (v7 + v6) + R(4) * (v1 - v2)) * (R(1) / R(12));
    dyq = ((v5 + v7) - (v8 + v6) + R(4) * (v3 - v4)) * (R(1) / R(12));
    lapq = (((v5 + v6) + (v7 + v8)) + R(4) * ((v1 + v2) + (v3 + v4))) * (R(1) / R(6));
}

// Bulk part of the binary chemical potential, -A phi + B phi^3 = B phi (phi - phib)(phi + phib),
// in the factored form that does not cancel near the bulk values.
template <typename R>
__device__ __forceinline__ R mu_bulk(const CapDev& c, R phi) {
    return (R)c.B * phi * ((phi - (R)c.phib) * (phi + (R)c.phib));
}

// Coefficients of the Galilean term of the van der Waals equilibrium.  The
// non-ideal p0 leaves the first-order momentum flux with
// -(tau - 1/2)(1/3 - dp0/drho)[u_a d_b rho + u_b d_a rho + delta_ab u.grad rho]
// (Chapman-Enskog), tau the relaxation time of the moments that carry it: the
// traceless stresses relax at omega, the trace (the energy moment e) at 1
// (Appendix A rates).  Each part of the bracket gets its own coefficient,
//   lam = (1/omega - 1/2)(1/3 - dp0/drho),  lam_b = (1/2)(1/3 - dp0/drho),
// which coincide with the single lambda of Eq. (equilibrium) at omega = 1.
// inv_omega_mh: 1/omega - 1/2; dp0: dp0/drho at the node.
template <typename R>
__device__ __forceinline__ void vdw_lambdas(R inv_omega_mh, R dp0, R& lam, R& lam_b) {
    const R base = R(1) / R(3) - dp0;
    lam = inv_omega_mh * base;
    lam_b = R(0.5) * base;
}

// The post-collision state of a node.  With the rates of Appendix A the
// moments e, eps, qx and qy relax fully to their equilibria (qx* = -jx*,
// qy* = -jy*), so f* = M^-1 m* depends on seven numbers only: the density
// (minus rho_ref), the momentum j* (with the forcing), the common parts b and d
// of the axis and diagonal populations (e* and eps*, minus their reference
// values X_ref/3 and X_ref/12) and the relaxed stresses pxx*, pxy*.
template <typename R>
struct PostState {
    R drho, jx, jy, b, d, pxx, pxy;
};

// The shifted post-collision populations f* = M^-1 m* of a post-collision
// state.  The even (common) part of each opposite pair is formed first and the
// small momentum term added last, so both members of a pair round at the same
// magnitude and their difference keeps the momentum.
//
// x/3 in the arithmetic type.  In FP32 the product with 1/3 rounded to FP32
// (3e-8 too large) would scale every streamed momentum by the same 1 + 3e-8:
// an amplification of j by that much per step, which moves an interface
// measurably over 10^4 steps.  There the quotient is corrected with the exact
// remainder x - 3q (one FMA), which leaves an unbiased rounding error.
template <typename R>
__device__ __forceinline__ R third(R x) {
    if constexpr (sizeof(R) == 4) {
        const float q = x * (1.f / 3.f);
        return __builtin_fmaf(__builtin_fmaf(-3.f, q, x), 1.f / 3.f, q);
    } else {
        return x * (R(1) / R(3));
    }
}

template <typename R>
__device__ __forceinline__ void pops_of_state(const PostState<R>& s, R (&o)[9]) {
    const R a7 = R(0.25) * s.pxx, a8 = R(0.25) * s.pxy;
    const R jx3 = third(s.jx), jy3 = third(s.jy);
    // j/12 as (j/3)/4 in FP32 (see third); FP64 keeps the direct product
    const R jpp = sizeof(R) == 4 ? R(0.25) * (jx3 + jy3) : (s.jx + s.jy) * (R(1) / R(12));
    const R jpm = sizeof(R) == 4 ? R(0.25) * (jx3 - jy3) : (s.jx - s.jy) * (R(1) / R(12));
    const R cx = s.b + a7, cy = s.b - a7, cp = s.d + a8, cm = s.d - a8;
    o[1] = cx + jx3;
    o[2] = cx - jx3;
    o[3] = cy + jy3;
    o[4] = cy - jy3;
    o[5] = cp + jpp;
    o[6] = cp - jpp;
    o[7] = cm - jpm;
    o[8] = cm + jpm;
    o[0] = s.drho - R(4) * (s.b + s.d);   // rest population minus rho_ref - 5/3 X_ref
}

// MRT collision of one node in moment space (Appendix A rates, Guo source
// (I - S/2) M F), returning the post-collision state.
//   m:   pre-collision moments (rho - rho_ref, j after rest, pxx, pxy)
//   dX:  X - X_ref, X = p0 - kappa q lap(q) the isotropic part of Eq. (equilibrium)
//   lam, lam_b: coefficients of the traceless part and of the isotropic part of
//        the Galilean term lambda [u_a d_b q + u_b d_a q + delta_ab u.grad q] of
//        Eq. (equilibrium) (equal in the printed form; see vdw_lambdas)
//   dq: gradient of q; F: body force on this node
// LAM = false drops the Galilean terms at compile time (lam must then be 0, as
// in the binary model) and FORCE = false the forcing terms (F must then be 0);
// the results are the same, with fewer instructions.
template <typename R, typename S = R, bool LAM = true, bool FORCE = true>
__device__ __forceinline__ PostState<R> collide_state(const CapDev& c, const Mom<R>& m, R rho, R ux, R uy, R dX,
                                                      R lam, R lam_b, R omega, R dxq, R dyq, R F) {
    const R kappa = (R)c.kappa;
    const R u2 = rho * (ux * ux + uy * uy);
    const R trQ = LAM ? u2 + R(4) * lam_b * (ux * dxq + uy * dyq) : u2;
    const R grad2 = dxq * dxq + dyq * dyq;
    // traceless stresses of the equilibrium and their relaxation in S
    const S sux = (S)ux, suy = (S)uy, sdx = (S)dxq, sdy = (S)dyq, srho = (S)rho, slam = (S)lam;
    const S dQ0 = srho * (sux * sux - suy * suy), Qxy0 = srho * sux * suy;
    const S dQ = LAM ? dQ0 + S(2) * slam * (sux * sdx - suy * sdy) : dQ0;
    const S Qxy = LAM ? Qxy0 + slam * (sux * sdy + suy * sdx) : Qxy0;
    const S pxx_eq = (S)c.kappa * (sdx * sdx - sdy * sdy) + dQ;
    const S pxy_eq = (S)c.kappa * sdx * sdy + Qxy;
    const R uF = ux * F;
    // common parts of the axis (b) and diagonal (d) populations minus their
    // reference values X_ref/3 and X_ref/12 (e, eps at equilibrium plus source)
    const R b = FORCE ? dX * (R(1) / R(3)) + (trQ + kappa * grad2 + uF) * (R(1) / R(12))
                      : dX * (R(1) / R(3)) + (trQ + kappa * grad2) * (R(1) / R(12));
    const R d = FORCE ? dX * (R(1) / R(12)) + (trQ - R(0.5) * kappa * grad2 + uF) * (R(1) / R(12))
                      : dX * (R(1) / R(12)) + (trQ - R(0.5) * kappa * grad2) * (R(1) / R(12));
    const R hw = R(1) - R(0.5) * omega;
    const R pxr = (R)((S)m.pxx - (S)omega * ((S)m.pxx - pxx_eq));
    const R pyr = (R)((S)m.pxy - (S)omega * ((S)m.pxy - pxy_eq));
    const R pxs = FORCE ? pxr + hw * R(2) * uF : pxr;
    const R pys = FORCE ? pyr + hw * (uy * F) : pyr;
    const R jxs = FORCE ? m.jx + F : m.jx, jys = m.jy;   // qx*, qy* = -jx*, -jy*
    return PostState<R>{m.drho, jxs, jys, b, d, pxs, pys};
}

// The collision returning the shifted post-collision populations.
template <typename R, typename S = R, bool LAM = true, bool FORCE = true>
__device__ __forceinline__ void collide(const CapDev& c, const Mom<R>& m, R rho, R ux, R uy, R dX, R lam, R lam_b,
                                        R omega, R dxq, R dyq, R F, R (&o)[9]) {
    pops_of_state(collide_state<R, S, LAM, FORCE>(c, m, rho, ux, uy, dX, lam, lam_b, omega, dxq, dyq, F), o);
}

// g^eq_i (i >= 1) of Appendix A from phi, u and Gamma mu.
template <typename R>
__device__ __forceinline__ R geq_i(int i, R phi, R ux, R uy, R gmu) {
    const R eu = (R)ex_(i) * ux + (R)ey_(i) * uy;
    const R w = i <= 4 ? R(1) / R(3) : R(1) / R(12);
    return w * (gmu + phi * (eu + R(1.5) * eu * eu - R(0.5) * (ux * ux + uy * uy)));
}

// LDS slot (sx, sy) of the one-node ring around a 64 x TY tile, k < 2 W2 + 2 TY.
template <int TY>
__device__ __forceinline__ void ring_slot(int k, int& sx, int& sy) {
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
}

struct TileCtx {
    TileDev t;
    const CapDev* c;
    Geo g;
    const float* src;
    float* dst;
};

__device__ __forceinline__ TileCtx tile_ctx(const StepArgs& a, int tile) {
    TileCtx k;
    k.t = a.tiles[tile];
    k.c = &a.caps[k.t.cap];
    k.g = geo_of(*k.c);
    const int sb = a.cur ^ k.c->par;
    k.src = sb ? a.arena1 : a.arena0;
    k.dst = sb ? a.arena0 : a.arena1;
    return k;
}

// ---- van der Waals liquid-gas model -----------------------------------------
template <int TY, bool INIT, typename R>
__device__ __forceinline__ void step_tile_vdw(const StepArgs& a, int tile, R* qs) {
    const TileCtx k = tile_ctx(a, tile);
    const CapDev& c = *k.c;
    const Geo& g = k.g;
    const long long P = c.plane;
    const float* __restrict__ fsrc = k.src + c.off_f;
    const int lx = threadIdx.x, ly = threadIdx.y;
    const int tid = lx + TILE_W * ly;
    const int x = k.t.x0 + lx, y = k.t.y0 + ly;
    const bool own = (x < g.nx) && (y < g.ny) && c.active;
    const int xw = x < g.nx ? x : wrap_mod(x, g.nx);
    const int yw = y < g.ny ? y : wrap_mod(y, g.ny);
    const bool fluid = !g.solid(xw, yw);
    const R rho_ref = (R)c.rho_ref;

    // phase 1: drho of every LDS slot; own populations kept in registers
    R f[9];
    R qv = R(0);
    const Hood h = hood_of(g, xw, yw);
    if (fluid) {
        if (INIT) {
            qv = (R)fsrc[(long long)yw * g.pitch + xw] - rho_ref;
        } else {
            pull9(fsrc, P, g, h, xw, yw, f);
            qv = sum9(f);
        }
    }
    qs[(ly + 1) * W2 + lx + 1] = qv;
    for (int r = tid; r < 2 * W2 + 2 * TY; r += TILE_W * TY) {
        int sx, sy;
        ring_slot<TY>(r, sx, sy);
        const int gx = wrap_mod(k.t.x0 + sx - 1, g.nx);
        const int gy = wrap_mod(k.t.y0 + sy - 1, g.ny);
        R v = R(0);
        if (!g.solid(gx, gy)) {
            if (INIT) {
                v = (R)fsrc[(long long)gy * g.pitch + gx] - rho_ref;
            } else {
                R ff[9];
                pull9(fsrc, P, g, hood_of(g, gx, gy), gx, gy, ff);
                v = sum9(ff);
            }
        }
        qs[sy * W2 + sx] = v;
    }
    __syncthreads();
    if (!(own && fluid)) return;

    // phase 2: collision of the own node
    const bool bnd = h.solid != 0u;
    Mom<R> m;
    if (INIT) {
        m.drho = qv;
        m.jx = m.jy = R(0);
    } else {
        m = moments_of(f, bnd);
    }
    const R F = bnd ? R(0) : (R)c.Fx;
    const R kappa = (R)c.kappa;
    R dxq, dyq, lapq;
    stencil<W2>(qs, (ly + 1) * W2 + lx + 1, h.solid, R(2) * (R)c.G, dxq, dyq, lapq);
    if (INIT) {
        // f = f^eq at u = 0: its stress moments are those of Eq. (pt)
        m.pxx = kappa * (dxq * dxq - dyq * dyq);
        m.pxy = kappa * dxq * dyq;
    }
    const R rho = rho_ref + m.drho;
    const R inv_rho = R(1) / rho;
    const R ux = (m.jx + R(0.5) * F) * inv_rho;
    const R uy = m.jy * inv_rho;
    const R T = (R)c.T, av = (R)c.a;
    const R ib = R(1) / (R(1) - (R)c.b * rho);
    // p0(rho) - p0(rho_ref) = drho [T / ((1 - b rho)(1 - b rho_ref)) - a (rho + rho_ref)]
    const R dX = m.drho * (T * ib * (R)c.ibr - av * (rho + rho_ref)) - kappa * rho * lapq;
    const R omega = (R)c.omega_l;
    R lam = R(0), lam_b = R(0);
    if (c.lam_on != 0.f) vdw_lambdas(R(1) / omega - R(0.5), T * ib * ib - R(2) * av * rho, lam, lam_b);
    R o[9];
    collide(c, m, rho, ux, uy, dX, lam, lam_b, omega, dxq, dyq, F, o);
    float* __restrict__ fdst = k.dst + c.off_f;
    const long long own_idx = (long long)yw * g.pitch + xw;
#pragma unroll
    for (int i = 0; i < 9; ++i) fdst[(long long)i * P + own_idx] = (float)o[i];
}

// ---- binary model, g eliminated ----------------------------------------------
// Velocity of a fluid node from its pulled populations (rest and force rules).
template <typename R>
__device__ __forceinline__ void node_u(const CapDev& c, const float* __restrict__ fsrc, const Geo& g, int x, int y,
                                       bool init, R& ux, R& uy) {
    const Hood h = hood_of(g, x, y);
    const bool bnd = h.solid != 0u;
    const R F = bnd ? R(0) : (R)c.Fx;
    if (init) {
        ux = R(0.5) * F / (R)c.rho_ref;
        uy = R(0);
        return;
    }
    R f[9];
    pull9(fsrc, c.plane, g, h, x, y, f);
    const Mom<R> m = moments_of(f, bnd);
    const R inv_rho = R(1) / ((R)c.rho_ref + m.drho);
    ux = (m.jx + R(0.5) * F) * inv_rho;
    uy = m.jy * inv_rho;
}

template <int TY, bool INIT, typename R>
__device__ __forceinline__ void step_tile_bin(const StepArgs& a, int tile, R* lds) {
    R* PH = lds;                                  // phi, two-node halo, row W4
    R* UX = lds + Lds<1, TY>::PH;                 // one-node halo, row W2
    R* UY = UX + Lds<1, TY>::R1;
    R* MU = UY + Lds<1, TY>::R1;
    const TileCtx k = tile_ctx(a, tile);
    const CapDev& c = *k.c;
    const Geo& g = k.g;
    const long long P = c.plane;
    const float* __restrict__ fsrc = k.src + c.off_f;
    const float* __restrict__ psrc = k.src + c.off_phi;
    const int lx = threadIdx.x, ly = threadIdx.y;
    const int tid = lx + TILE_W * ly;
    constexpr int NT = TILE_W * TY;
    const int x = k.t.x0 + lx, y = k.t.y0 + ly;
    const bool own = (x < g.nx) && (y < g.ny) && c.active;
    const int xw = x < g.nx ? x : wrap_mod(x, g.nx);
    const int yw = y < g.ny ? y : wrap_mod(y, g.ny);
    const bool fluid = !g.solid(xw, yw);
    const Hood h = hood_of(g, xw, yw);
    const bool bnd = h.solid != 0u;
    const R G2 = R(2) * (R)c.G;
    const R kappa = (R)c.kappa, Gam = (R)c.Gamma;

    // phase 1a: phi(t) on the tile and a two-node halo
    for (int r = tid; r < (TY + 4) * W4; r += NT) {
        const int sx = r % W4, sy = r / W4;
        const int gx = wrap_mod(k.t.x0 + sx - 2, g.nx);
        const int gy = wrap_mod(k.t.y0 + sy - 2, g.ny);
        PH[r] = g.solid(gx, gy) ? R(0) : phi_of_fixed<R>(psrc[(long long)gy * g.pitch + gx]);
    }
    // phase 1b: own moments and u; u of the one-node ring
    R f[9];
    Mom<R> m{R(0), R(0), R(0), R(0), R(0)};
    R ux = R(0), uy = R(0);
    const R F = bnd ? R(0) : (R)c.Fx;
    if (fluid) {
        if (INIT) {
            m.drho = R(1) - (R)c.rho_ref;
        } else {
            pull9(fsrc, P, g, h, xw, yw, f);
            m = moments_of(f, bnd);
        }
        const R inv_rho = R(1) / ((R)c.rho_ref + m.drho);
        ux = (m.jx + R(0.5) * F) * inv_rho;
        uy = m.jy * inv_rho;
    }
    const int o1 = (ly + 1) * W2 + lx + 1;
    UX[o1] = ux;
    UY[o1] = uy;
    for (int r = tid; r < 2 * W2 + 2 * TY; r += NT) {
        int sx, sy;
        ring_slot<TY>(r, sx, sy);
        const int gx = wrap_mod(k.t.x0 + sx - 1, g.nx);
        const int gy = wrap_mod(k.t.y0 + sy - 1, g.ny);
        R vx = R(0), vy = R(0);
        if (!g.solid(gx, gy)) node_u(c, fsrc, g, gx, gy, INIT, vx, vy);
        UX[sy * W2 + sx] = vx;
        UY[sy * W2 + sx] = vy;
    }
    __syncthreads();

    // phase 2a: Gamma mu on the tile and its one-node ring (stencils of phi)
    R dxq = R(0), dyq = R(0), lapq = R(0), phi = R(0);
    const int o2 = (ly + 2) * W4 + lx + 2;
    if (fluid) {
        phi = PH[o2];
        stencil<W4>(PH, o2, h.solid, G2, dxq, dyq, lapq);
        MU[o1] = Gam * (mu_bulk(c, phi) - kappa * lapq);
    } else {
        MU[o1] = R(0);
    }
    for (int r = tid; r < 2 * W2 + 2 * TY; r += NT) {
        int sx, sy;
        ring_slot<TY>(r, sx, sy);
        const int gx = wrap_mod(k.t.x0 + sx - 1, g.nx);
        const int gy = wrap_mod(k.t.y0 + sy - 1, g.ny);
        R v = R(0);
        if (!g.solid(gx, gy)) {
            const int pi = (sy + 1) * W4 + sx + 1;
            R ddx, ddy, dl;
            stencil<W4>(PH, pi, hood_of(g, gx, gy).solid, G2, ddx, ddy, dl);
            v = Gam * (mu_bulk(c, PH[pi]) - kappa * dl);
        }
        MU[sy * W2 + sx] = v;
    }
    __syncthreads();
    if (!(own && fluid)) return;

    // phase 2b: collision of f
    if (INIT) {
        m.pxx = kappa * (dxq * dxq - dyq * dyq);
        m.pxy = kappa * dxq * dyq;
    }
    const R rho = (R)c.rho_ref + m.drho;
    const R p2 = phi * phi;
    const R phib = (R)c.phib;
    // p0 - X_ref = drho/3 + (B/4)(phi^2 - phib^2)(3 phi^2 + phib^2), X_ref = rho_ref/3 + A^2/(4B)
    const R dX = m.drho * (R(1) / R(3)) + R(0.25) * (R)c.B * ((phi - phib) * (phi + phib)) * (R(3) * p2 + phib * phib) -
                 kappa * phi * lapq;
    const R pc = phi < R(-1) ? R(-1) : (phi > R(1) ? R(1) : phi);
    const R nu_l = (R)c.nu_l, nu_g = (R)c.nu_g;
    const R nu = nu_g + R(0.5) * (pc + R(1)) * (nu_l - nu_g);
    const R omega = R(2) / (R(6) * nu + R(1));
    R o[9];
    collide<R, R, false>(c, m, rho, ux, uy, dX, R(0), R(0), omega, dxq, dyq, F, o);
    float* __restrict__ fdst = k.dst + c.off_f;
    const long long own_idx = (long long)yw * g.pitch + xw;
#pragma unroll
    for (int i = 0; i < 9; ++i) fdst[(long long)i * P + own_idx] = (float)o[i];

    // phase 2c: phi(t+1) = phi(t) + sum_i [g^eq_i(source of i) - g^eq_i(r)]
    const R gmu = MU[o1];
    R go[9];
#pragma unroll
    for (int i = 1; i < 9; ++i) go[i] = geq_i(i, phi, ux, uy, gmu);
    R delta = R(0);
#pragma unroll
    for (int i = 1; i < 9; ++i) {
        R gin;
        if ((h.solid >> opp_(i)) & 1u) {
            gin = go[opp_(i)];   // bounce-back of g*_opp(i)(r)
        } else {
            const int s1 = o1 - ey_(i) * W2 - ex_(i);
            const int s2 = o2 - ey_(i) * W4 - ex_(i);
            gin = geq_i(i, PH[s2], UX[s1], UY[s1], MU[s1]);
        }
        delta += gin - go[i];
    }
    k.dst[c.off_phi + own_idx] = phi_bits(__builtin_bit_cast(int, psrc[own_idx]) + fixed_of_phi(delta));
}

// R: arithmetic type of the step (float, or double with FP32 storage).
template <int MODEL, int TY, bool INIT, typename R>
__global__ void __launch_bounds__(TILE_W* TY) lb_step_kernel(StepArgs a) {
    __shared__ R lds[Lds<MODEL, TY>::SIZE];
    auto one = [&](int tile) {
        if (MODEL == 0)
            step_tile_vdw<TY, INIT, R>(a, tile, lds);
        else
            step_tile_bin<TY, INIT, R>(a, tile, lds);
    };
    if (a.schedule == 2) {
        for (int tile = blockIdx.x; tile < a.ntiles; tile += gridDim.x) {
            one(tile);
            __syncthreads();
        }
    } else {
        int tile = blockIdx.x;
        if (a.schedule == 1) {
            const int per = (a.ntiles + 7) >> 3;
            tile = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
        }
        if (tile < a.ntiles) one(tile);
    }
}

// ---- macroscopic fields of one capillary -----------------------------------
// rho = rho_ref + sum s*, u = (j* - F/2)/rho (the collision added F to j), phi(t)
// from the phi plane of the other arena.
template <int MODEL>
__global__ void lb_moments_kernel(const CapDev* caps, int cap, const float* __restrict__ st,
                                  const float* __restrict__ prev, float* rho_o, float* ux_o, float* uy_o,
                                  float* phi_o) {
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
            float jx, jy;
            if (c.mstore) {   // planes drho, jx*/3, jy*/3, ...
                r = c.rho_ref + st[c.off_f + own];
                jx = 3.f * st[c.off_f + c.plane + own];
                jy = 3.f * st[c.off_f + 2 * c.plane + own];
            } else {
                float f[9];
#pragma unroll
                for (int i = 0; i < 9; ++i) f[i] = st[c.off_f + i * c.plane + own];
                r = c.rho_ref + sum9(f);
                jx = ((f[1] - f[2]) + (f[5] - f[6])) + (f[8] - f[7]);
                jy = ((f[3] - f[4]) + (f[5] - f[6])) + (f[7] - f[8]);
            }
            const float F = h.solid ? 0.f : c.Fx;
            u = (jx - 0.5f * F) / r;
            v = jy / r;
            if (MODEL == 1) p = phi_of_fixed(prev[c.off_phi + own]);
        }
        if (rho_o) rho_o[k] = r;
        if (ux_o) ux_o[k] = u;
        if (uy_o) uy_o[k] = v;
        if (phi_o) phi_o[k] = p;
    }
}

// ---- filled length of every capillary (one workgroup per capillary) --------
template <int MODEL>
__device__ __forceinline__ float centre_q(const CapDev& c, const float* __restrict__ st,
                                          const float* __restrict__ prev, int x, int ya, int yb) {
    if (MODEL == 1) {
        const float a = prev[c.off_phi + (long long)ya * c.pitch + x], b = prev[c.off_phi + (long long)yb * c.pitch + x];
        return 0.5f * (phi_of_fixed(a) + phi_of_fixed(b));
    }
    if (c.mstore)
        return 0.5f * ((c.rho_ref + st[c.off_f + (long long)ya * c.pitch + x]) +
                       (c.rho_ref + st[c.off_f + (long long)yb * c.pitch + x]));
    float fa[9], fb[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        fa[i] = st[c.off_f + i * c.plane + (long long)ya * c.pitch + x];
        fb[i] = st[c.off_f + i * c.plane + (long long)yb * c.pitch + x];
    }
    return 0.5f * ((c.rho_ref + sum9(fa)) + (c.rho_ref + sum9(fb)));
}

template <int MODEL>
__global__ void __launch_bounds__(256)
lb_interface_kernel(const CapDev* caps, int ncap, float* arena0, float* arena1, int cur, float* l_now,
                    float* hist, long long* hist_t, int* hist_n, int hist_cap, long long t_now, int record) {
    const int cap = blockIdx.x;
    if (cap >= ncap) return;
    const CapDev& c = caps[cap];
    if (!c.active) return;
    const int sb = cur ^ c.par;
    const float* st = sb ? arena1 : arena0;
    const float* prev = sb ? arena0 : arena1;
    __shared__ int kmin_s;
    if (threadIdx.x == 0) kmin_s = 0x7fffffff;
    __syncthreads();
    const int H = c.y1 - c.y0;
    const int L = c.x_end - c.x_in;
    const int ya = (H % 2 == 0) ? c.y0 + H / 2 - 1 : c.y0 + (H - 1) / 2;
    const int yb = (H % 2 == 0) ? c.y0 + H / 2 : ya;
    int kmin = 0x7fffffff;
    for (int k = threadIdx.x; k < L; k += blockDim.x) {
        if (centre_q<MODEL>(c, st, prev, c.x_in + k, ya, yb) < c.q_mid) {
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
            const float qp = centre_q<MODEL>(c, st, prev, c.x_in + k - 1, ya, yb);
            const float qk = centre_q<MODEL>(c, st, prev, c.x_in + k, ya, yb);
            l = (float)(k - 1) + (qp - c.q_mid) / (qp - qk);
        }
        l_now[cap] = l;
        if (record) {
            const int n = hist_n[cap];
            if (n < hist_cap) {
                hist[(long long)c.hist_off + n] = l + 0.5f * (float)H;
                hist_t[(long long)c.hist_off + n] = t_now;
            }
            hist_n[cap] = n + 1;
        }
    }
}

// ---- health scan: non-finite value or rho <= 0 -> flag per capillary --------
template <int MODEL>
__global__ void lb_health_kernel(const CapDev* caps, const TileDev* tiles, int ntiles, float* arena0,
                                 float* arena1, int cur, int* flags) {
    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const TileDev t = tiles[tile];
        const CapDev& c = caps[t.cap];
        const Geo g = geo_of(c);
        const float* st = (cur ^ c.par) ? arena1 : arena0;
        for (int r = threadIdx.x / TILE_W; r < 8; r += blockDim.x / TILE_W) {
            const int x = t.x0 + (threadIdx.x % TILE_W), y = t.y0 + r;
            if (x >= g.nx || y >= g.ny || r >= t.rows || g.solid(x, y)) continue;
            const long long own = (long long)y * g.pitch + x;
            float s = c.rho_ref;
            bool bad = false;
            if (c.mstore) {   // the state's planes; the first one is drho
#pragma unroll
                for (int i = 0; i < 7; ++i) bad |= !isfinite(st[c.off_f + i * c.plane + own]);
                s += st[c.off_f + own];
            } else {
#pragma unroll
                for (int i = 0; i < 9; ++i) {
                    const float v = st[c.off_f + i * c.plane + own];
                    bad |= !isfinite(v);
                    s += v;
                }
            }
            if (bad || !(s > 0.f)) atomicOr(&flags[t.cap], 1);
        }
    }
}

}  // namespace lbk
