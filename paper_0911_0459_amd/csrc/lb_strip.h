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
// The collision (velocity, equilibrium, relaxation, reconstruction) is
// evaluated in the arithmetic type CT (double by default) from the FP32 moments
// of the pulled populations: the shifted FP32 populations are stored as
// before, but in FP32 arithmetic the rounding of the reconstructed populations
// of a steady flow repeats every step at every node and acts like a small
// spurious body force, which shifts a moving meniscus by ~1e-4 lattice units
// per 1e4 steps.  The order-parameter path (mu, g^eq, phi update) is FP32: its
// rounding does not accumulate that way.
#pragma once
#include "lb_kernels.h"
#include "lb_strip_table.h"

namespace lbk {

constexpr int STRIP_OUT = 62;     // output columns per strip
constexpr int SW = 64;            // lanes per strip = one wavefront
constexpr int PHW = SW + 2;       // phi row in LDS: columns xs-2 .. xs+63

struct StripArgs {
    const CapDev* caps;
    const StripDev* strips;
    int nstrips;
    int xcd_start[9];             // XCD x works through strips xcd_start[x] .. xcd_start[x + 1] - 1
    float* arena0;
    float* arena1;
    int cur;
};

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

// Ordering of the LDS ring buffers between the lanes of the single wavefront
// of a strip.  LDS instructions of one wavefront execute in program order, so
// only the compiler must not move LDS accesses across this point; a workgroup
// barrier would in addition wait for every outstanding global load, including
// the row requested ahead of time.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Workgroups are dealt to the 8 XCDs round-robin: workgroup b runs on XCD b % 8
// as that XCD's (b / 8)-th; -1 past the end of the XCD's run.
__device__ __forceinline__ int strip_index(const StripArgs& a) {
    const int x = blockIdx.x & 7;
    const int i = a.xcd_start[x] + (int)(blockIdx.x >> 3);
    return i < a.xcd_start[x + 1] ? i : -1;
}

// Column data of one lane, fixed for the whole strip: the lane's column and its
// two neighbours (periodic), and whether each lies in the tube section.
struct LaneCols {
    int c0, cm, cp;
    int b0, bm, bp;       // the same columns as byte offsets within a row
    bool t0, tm, tp;
};

__device__ __forceinline__ LaneCols lane_cols(const Geo& g, int xl) {
    LaneCols L;
    L.c0 = wrap_mod(xl, g.nx);
    L.cm = L.c0 == 0 ? g.nx - 1 : L.c0 - 1;
    L.cp = L.c0 == g.nx - 1 ? 0 : L.c0 + 1;
    L.b0 = 4 * L.c0;
    L.bm = 4 * L.cm;
    L.bp = 4 * L.cp;
    L.t0 = g.tube_col(L.c0);
    L.tm = g.tube_col(L.cm);
    L.tp = g.tube_col(L.cp);
    return L;
}

// Row data: wrapped row and neighbours, their offsets, whether they are wall rows.
struct RowInfo {
    int y0, ym, yp;
    bool w0, wm, wp;
    bool any;   // some wall row among ym, y0, yp (same for every lane)
};

__device__ __forceinline__ RowInfo row_info(const Geo& g, int y) {
    RowInfo r;
    r.y0 = y < 0 ? y + g.ny : (y >= g.ny ? y - g.ny : y);
    r.ym = r.y0 == 0 ? g.ny - 1 : r.y0 - 1;
    r.yp = r.y0 == g.ny - 1 ? 0 : r.y0 + 1;
    r.w0 = g.wall_row(r.y0);
    r.wm = g.wall_row(r.ym);
    r.wp = g.wall_row(r.yp);
    r.any = r.w0 || r.wm || r.wp;
    return r;
}

// Solid-neighbour bits of the lane's node on this row (bit d: r + e_d solid).
__device__ __forceinline__ unsigned solid_bits(const LaneCols& L, const RowInfo& r) {
    return ((unsigned)(L.tp && r.w0) << 1) | ((unsigned)(L.tm && r.w0) << 2) | ((unsigned)(L.t0 && r.wp) << 3) |
           ((unsigned)(L.t0 && r.wm) << 4) | ((unsigned)(L.tp && r.wp) << 5) | ((unsigned)(L.tm && r.wm) << 6) |
           ((unsigned)(L.tm && r.wp) << 7) | ((unsigned)(L.tp && r.wm) << 8);
}

// One capillary's planes of an arena seen through a buffer resource.  Accesses
// take a 32-bit per-lane byte offset (the column) and a scalar byte offset (the
// plane and the row), so no per-lane 64-bit address arithmetic is spent on
// them; the hardware checks every access against the region's size.
constexpr int RAW_BUFFER_WORD3 = 0x00020000;   // descriptor dword 3: raw 32-bit data, no swizzle

struct Planes {
    __amdgpu_buffer_rsrc_t rs;
    int pb;                       // bytes per plane
    int rb;                       // bytes per row
};

__device__ __forceinline__ Planes planes_of(const float* base, int nplanes, int P, int pitch) {
    Planes q;
    q.rs = __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(base), (short)0, nplanes * P * 4, RAW_BUFFER_WORD3);
    q.pb = 4 * P;
    q.rb = 4 * pitch;
    return q;
}

// (the b32 builtins move raw 32-bit words: the float is reinterpreted, not converted).
// The scalar offset is the same in every lane; readfirstlane states so, because
// a value the compiler keeps in a vector register would turn each access into
// a loop over the distinct values of the lanes.
__device__ __forceinline__ float ld(const Planes& q, int voff, int soff) {
    return __builtin_bit_cast(
        float, __builtin_amdgcn_raw_buffer_load_b32(q.rs, voff, __builtin_amdgcn_readfirstlane(soff), 0));
}

__device__ __forceinline__ void st(const Planes& q, float v, int voff, int soff) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), q.rs, voff,
                                          __builtin_amdgcn_readfirstlane(soff), 0);
}

// 1/x for a positive normal x in the collision's arithmetic type: the
// hardware FP32 reciprocal (1 ulp) refined by one Newton step, with far fewer
// instructions and registers than the correctly rounded division.  In FP64 the
// step squares the relative error of the FP32 estimate (below 2^-22 after the
// rounding of x to FP32), leaving it below 1e-13, far below the FP32 rounding
// of the stored state.  In FP32 the step's own FMA rounds the result to
// within about half an ulp (the Newton step from either side lands below 1/x
// by the square of the estimate's error, 1e-14 relative, so the rounding
// carries no bias that a conserved quantity could accumulate).
__device__ __forceinline__ double recip(double x) {
    const double r = (double)__builtin_amdgcn_rcpf((float)x);
    return __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
}

__device__ __forceinline__ float recip(float x) {
    const float r = __builtin_amdgcn_rcpf(x);
    return __builtin_fmaf(r, __builtin_fmaf(-x, r, 1.f), r);
}

// Makes a uniform FP32 value opaque to loop-invariant code motion (an empty asm
// statement that claims to modify it in its scalar register).  Material
// constants converted to FP64 inside the sweep would otherwise be converted
// once, before the loop, and held in a pair of vector registers for the whole
// sweep; vector registers bound the occupancy of these kernels, the
// conversions are cheap.
__device__ __forceinline__ void uniform_opaque(float& v) { asm volatile("" : "+s"(v)); }

// Pull of the lane's node on a row (bounce-back for solid sources).  Straight-line
// code, the source chosen by selects: a branch around the loads (even a uniform
// one) makes the compiler's wait counting assume the path without them, so
// that every later use of an older load would wait for these ones as well.
// For each direction the scalar offset is the smaller of the two candidate
// sources (streaming: plane i, the source row; bounce-back: plane opp(i), the
// node's own row), so the per-lane offset of either choice is non-negative.
__device__ __forceinline__ void pull_lane(const Planes& q, const LaneCols& L, const RowInfo& r, unsigned sm,
                                          float (&f)[9]) {
    const int s0 = r.y0 * q.rb, sm_ = r.ym * q.rb, sp = r.yp * q.rb;
    auto get = [&](int i, int col, int srow) -> float {
        const bool bb = (sm >> opp_(i)) & 1u;
        if (i & 1) {   // opp(i) = i + 1: the streaming source has the smaller offset
            return ld(q, bb ? L.b0 + q.pb + (s0 - srow) : col, i * q.pb + srow);
        } else {       // opp(i) = i - 1: the bounce-back source has the smaller offset
            return ld(q, bb ? L.b0 : col + q.pb + (srow - s0), (i - 1) * q.pb + s0);
        }
    };
    f[0] = ld(q, L.b0, s0);
    f[1] = get(1, L.bm, s0);
    f[2] = get(2, L.bp, s0);
    f[3] = get(3, L.b0, sm_);
    f[4] = get(4, L.b0, sp);
    f[5] = get(5, L.bm, sm_);
    f[6] = get(6, L.bp, sp);
    f[7] = get(7, L.bp, sm_);
    f[8] = get(8, L.bm, sp);
}

// phi(t+1) - phi(t) at a node (binary model), shared by the row-sweep kernels so
// that both compile the same arithmetic.  phi, ux, uy, am: the node's order
// parameter, velocity and direction-free part A = Gamma mu - phi |u|^2 / 2;
// src(i, a, p, x, y) fetches A, phi, ux, uy of the source node r - e_i.
//   phi(t+1) = phi(t) + sum_i g^eq_i(source of i) - sum_i g^eq_i(r), i >= 1.
// With g^eq_i = w_i (A + phi e_i.u (1 + 3/2 e_i.u)), sum_i w_i = 5/3 and
// sum_i w_i (e_i.u)^2 = |u|^2 (Appendix A moments), this is
//   sum_i w_i [(A_src - A) + phi_src e_i.u_src (1 + 3/2 e_i.u_src)] - 3/2 phi |u|^2.
// Writing the A part as differences makes the update of a uniform region
// exactly zero; a closed-form sum_i w_i A would not round like the eight
// incoming terms, and the same small excess at every bulk node would drift the
// total phi steadily.  A solid source contributes the bounce-back of
// g*_opp(i)(r) (no A difference); its source entries are fetched but unused.
template <typename Src>
__device__ __forceinline__ float phi_delta(unsigned sm, float phi, float ux, float uy, float am, Src src) {
    auto adv = [](int i, float pp, float ax, float ay) {
        // e_i.u with the unit components folded at compile time (0 * ay cannot
        // be dropped by the compiler: it is not 0 for an infinite ay)
        const int ex = ex_(i), ey = ey_(i);
        const float t = ey == 0 ? ax : (ex == 0 ? ay : (ex == ey ? ax + ay : ax - ay));
        const float eu = (ex < 0 || (ex == 0 && ey < 0)) ? -t : t;
        return pp * eu * (1.f + 1.5f * eu);
    };
    auto incoming = [&](int i) {
        float a, p, x, y;
        src(i, a, p, x, y);
        return (a - am) + adv(i, p, x, y);
    };
    float sa = 0.f, sd = 0.f;   // axis and diagonal sums
    if (sm == 0u) {   // no solid neighbour: every source streams
#pragma unroll
        for (int i = 1; i < 9; ++i) {
            if (i <= 4) sa += incoming(i);
            else sd += incoming(i);
        }
    } else {
#pragma unroll
        for (int i = 1; i < 9; ++i) {
            const float t = ((sm >> opp_(i)) & 1u) ? adv(opp_(i), phi, ux, uy) : incoming(i);
            if (i <= 4) sa += t;
            else sd += t;
        }
    }
    return (sa * (1.f / 3.f) + sd * (1.f / 12.f)) - 1.5f * phi * (ux * ux + uy * uy);
}

// ---- binary model --------------------------------------------------------------
// Reads f*(t-1) and phi(t) of one strip chunk, writes f*(t) and phi(t+1).
template <typename MT, typename CT, typename ST = CT, bool FORCE = true>
__global__ void __launch_bounds__(SW) lb_strip_bin(StripArgs a) {
    const int si = strip_index(a);
    if (si < 0) return;
    const StripDev s = a.strips[si];
    // by value: one scalar load at entry, kept in registers (a reference would be
    // re-read from memory after every global store of the loop)
    const CapDev c = a.caps[s.cap];
    const Geo g = geo_of(c);
    const int P = (int)c.plane;
    const int sb = a.cur ^ c.par;
    const Planes fs = planes_of((sb ? a.arena1 : a.arena0) + c.off_f, 9, P, c.pitch);
    const Planes ps = planes_of((sb ? a.arena1 : a.arena0) + c.off_phi, 1, P, c.pitch);
    const Planes fd = planes_of((sb ? a.arena0 : a.arena1) + c.off_f, 9, P, c.pitch);
    const Planes pd = planes_of((sb ? a.arena0 : a.arena1) + c.off_phi, 1, P, c.pitch);

    __shared__ float PH[5][PHW];                         // phi rows, column xs-2+j at index j
    // column xs-1+k at lane k: velocity and Gamma mu - phi |u|^2 / 2, the part of g^eq
    // that does not depend on the direction
    __shared__ float UX[3][SW], UY[3][SW], AM[3][SW];

    const int k = threadIdx.x;
    // lanes past column xe+1 (the last one that an output column reads) repeat
    // that column: their loads share its addresses
    const int xl = min(s.xs + k - 1, s.xe + 1);
    const LaneCols L = lane_cols(g, xl);
    const bool out_col = k >= 1 && k <= STRIP_OUT && xl < s.xe;
    // the two extra phi columns, xs-2 (lane 0) and xs+63 (lane 1)
    const int ce = wrap_mod(k == 0 ? s.xs - 2 : s.xs + SW - 1, g.nx);
    const bool te = g.tube_col(ce);
    const float G2 = 2.f * c.G;
    const float kap = c.kappa, Gam = c.Gamma;

    // phi loads are issued unconditionally (solid nodes have valid addresses) and
    // masked when stored, so that no instruction waits on them early
    const int bx = 4 * (k < 2 ? ce : L.c0);
    auto phi_load = [&](const RowInfo& r, float& m, float& e) {
        m = ld(ps, L.b0, r.y0 * ps.rb);
        e = ld(ps, bx, r.y0 * ps.rb);
    };
    auto phi_store = [&](int sl, const RowInfo& r, float m, float e) {   // m, e: fixed point
        PH[sl][k + 1] = (L.t0 && r.w0) ? 0.f : phi_of_fixed(m);
        if (k == 0) PH[sl][0] = (te && r.w0) ? 0.f : phi_of_fixed(e);
        if (k == 1) PH[sl][PHW - 1] = (te && r.w0) ? 0.f : phi_of_fixed(e);
    };
    // moments of a pulled row (FP32, kept by the caller) and its velocity into LDS
    auto u_row = [&](int sl, const float (&f)[9], bool fluid, unsigned sm, Mom<float>& m) {
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
        UX[sl][k] = ux;
        UY[sl][k] = uy;
    };
    // stencils of phi (rows s5m, s50, s5p), Gamma mu and the direction-free part of g^eq
    auto mu_row = [&](int sl, int s5m, int s50, int s5p, bool fluid, unsigned sm, float& dx, float& dy,
                      float& lap, float& gmu) {
        float v = 0.f;
        dx = dy = lap = gmu = 0.f;
        if (fluid) {
            stencil3(PH[s5m], PH[s50], PH[s5p], k + 1, sm, G2, dx, dy, lap);
            const float ph = PH[s50][k + 1];
            gmu = Gam * (mu_bulk(c, ph) - kap * lap);
            const float ux = UX[sl][k], uy = UY[sl][k];
            v = gmu - 0.5f * ph * (ux * ux + uy * uy);
        }
        AM[sl][k] = v;
    };

    // ring slots: row y+d of the phi ring is (p5 + 2 + d) mod 5, of the u/mu ring (p3 + 1 + d) mod 3
    int p5 = 0, p3 = 0;   // slots of rows ya-2 and ya-1
    auto r5 = [&](int d) { int v = p5 + 2 + d; v -= v >= 5 ? 5 : 0; v -= v >= 5 ? 5 : 0; return v; };
    auto r3 = [&](int d) { int v = p3 + 1 + d; v -= v >= 3 ? 3 : 0; v -= v >= 3 ? 3 : 0; return v; };

    // ---- prologue: phi rows ya-2..ya+1; u, mu of rows ya-1, ya
    int q_cur = 0, q_next = 0;   // fixed-point phi of this lane's column, rows y and y+1
    for (int d = -2; d <= 1; ++d) {
        float m, e;
        const RowInfo rr = row_info(g, s.ya + d);
        phi_load(rr, m, e);
        if (d == 0) q_cur = __builtin_bit_cast(int, m);
        if (d == 1) q_next = __builtin_bit_cast(int, m);
        phi_store(r5(d), rr, m, e);
    }
    float f[9];
    Mom<float> mom_cur;
    RowInfo ri = row_info(g, s.ya - 1);
    unsigned sm = solid_bits(L, ri);
    bool fl = !(L.t0 && ri.w0);
    pull_lane(fs, L, ri, sm, f);
    u_row(r3(-1), f, fl, sm, mom_cur);
    ri = row_info(g, s.ya);
    unsigned sm_cur = solid_bits(L, ri);
    bool fl_cur = !(L.t0 && ri.w0);
    pull_lane(fs, L, ri, sm_cur, f);
    u_row(r3(0), f, fl_cur, sm_cur, mom_cur);
    wave_sync();
    float dx_cur, dy_cur, lap_cur, gmu_cur, t0, t1, t2, t3;
    mu_row(r3(-1), r5(-2), r5(-1), r5(0), fl, sm, t0, t1, t2, t3);
    mu_row(r3(0), r5(-1), r5(0), r5(1), fl_cur, sm_cur, dx_cur, dy_cur, lap_cur, gmu_cur);
    // Requests run one row ahead of the arithmetic.  The two request buffers swap
    // roles every row (the loop is unrolled by two), so a finished request is
    // never copied: a copy would wait for every load in flight.
    struct Ahead {
        float f[9];       // pulled populations of row y+1
        float pm, pe;     // phi of row y+2 (own column, extra column)
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
        phi_load(A.rph, A.pm, A.pe);
    }

    // one row y: n holds the requests for row y+1, p receives those for row y+2
    auto iter = [&](int y, Ahead& n, Ahead& p) {
        // (a) requests for the next row: row y+2 pulled, phi row y+3.  In the last
        // row of the chunk they repeat the previous requests (cache hits, unused):
        // loads under a branch would make every later wait a wait for all loads.
        const int ya2 = y + 1 < s.yb ? y + 2 : y + 1;
        const RowInfo ri_p = row_info(g, ya2);
        p.sm = solid_bits(L, ri_p);
        p.fl = !(L.t0 && ri_p.w0);
        p.rph = row_info(g, ya2 + 1);
        pull_lane(fs, L, ri_p, p.sm, p.f);
        phi_load(p.rph, p.pm, p.pe);
        // keep the uses of the previous requests below the new ones
        __builtin_amdgcn_sched_barrier(0);
        // (b) phi row y+2; u and moments of row y+1
        const int q_new = __builtin_bit_cast(int, n.pm);
        phi_store(r5(2), n.rph, n.pm, n.pe);
        Mom<float> mom_n;
        u_row(r3(1), n.f, n.fl, n.sm, mom_n);
        wave_sync();
        // (c) stencils and mu of row y+1
        float dx_n, dy_n, lap_n, gmu_n;
        mu_row(r3(1), r5(0), r5(1), r5(2), n.fl, n.sm, dx_n, dy_n, lap_n, gmu_n);
        wave_sync();
        // (d) collision and phi update of row y
        if (out_col && fl_cur) {
            const float phi = PH[r5(0)][k + 1];
            const Mom<CT> mc{(CT)mom_cur.drho, (CT)mom_cur.jx, (CT)mom_cur.jy, (CT)mom_cur.pxx, (CT)mom_cur.pxy};
            const CT F_cur = (FORCE && !sm_cur) ? (CT)c.Fx : CT(0);
            const CT rho_c = (CT)c.rho_ref + mc.drho;
            const CT inv_rho = recip(rho_c);
            const CT ux_cur = (FORCE ? mc.jx + CT(0.5) * F_cur : mc.jx) * inv_rho, uy_cur = mc.jy * inv_rho;
            const CT ph = (CT)phi, phib = (CT)c.phib;
            const CT dX = mc.drho * (CT(1) / CT(3)) +
                          CT(0.25) * (CT)c.B * ((ph - phib) * (ph + phib)) * (CT(3) * ph * ph + phib * phib) -
                          (CT)kap * ph * (CT)lap_cur;
            // the relaxation rate only scales the shear stresses (FP32) and the
            // forcing term, so it is formed in FP32 with the hardware reciprocal
            // (1 ulp)
            const float pc = phi < -1.f ? -1.f : (phi > 1.f ? 1.f : phi);
            const float nu = c.nu_g + 0.5f * (pc + 1.f) * (c.nu_l - c.nu_g);
            const CT omega = (CT)(2.f * __builtin_amdgcn_rcpf(6.f * nu + 1.f));
            CT o[9];
            collide<CT, ST, false, FORCE>(c, mc, rho_c, ux_cur, uy_cur, dX, CT(0), CT(0), omega, (CT)dx_cur, (CT)dy_cur, F_cur, o);
            const int srow = row_info(g, y).y0 * fd.rb;
#pragma unroll
            for (int i = 0; i < 9; ++i) st(fd, (float)o[i], L.b0, i * fd.pb + srow);
            // the phi update below is not to be interleaved with the collision
            // (its LDS reads would be hoisted into the collision's register peak)
            __builtin_amdgcn_sched_barrier(0);
            const float uxf = UX[r3(0)][k], uyf = UY[r3(0)][k];
            const float dphi = phi_delta(sm_cur, phi, uxf, uyf, AM[r3(0)][k],
                                         [&](int i, float& a, float& p, float& x, float& y) {
                                             const int s3 = r3(-ey_(i)), sk = k - ex_(i);
                                             a = AM[s3][sk];
                                             p = PH[r5(-ey_(i))][sk + 1];
                                             x = UX[s3][sk];
                                             y = UY[s3][sk];
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
        gmu_cur = gmu_n;
        q_cur = q_next;
        q_next = q_new;
        p5 = p5 == 4 ? 0 : p5 + 1;
        p3 = p3 == 2 ? 0 : p3 + 1;
        wave_sync();
    };
    for (int y = s.ya; y < s.yb; y += 2) {
        iter(y, A, B);
        if (y + 1 >= s.yb) break;
        iter(y + 1, B, A);
    }
}

// ---- van der Waals model ---------------------------------------------------------
// Collision of one fluid node of the van der Waals model from the FP32 moments
// of its pulled populations and the stencils of rho (every vdW row sweep calls
// it, so they compile the same arithmetic): thermodynamics of Sec. 2, the
// Galilean coefficients of vdw_lambdas, MRT relaxation with the non-shear part
// in arithmetic type CT and the shear relaxation in FP32 (as for the binary
// model).  sm: the node's solid-neighbour bits (boundary nodes take no body
// force).
template <typename CT, bool FORCE>
__device__ __forceinline__ void vdw_node_collide(const CapDev& c, const Mom<float>& mom, unsigned sm, float dxf,
                                                 float dyf, float lapf, CT (&o)[9]) {
    // constants of the FP64 part, converted where used (see uniform_opaque)
    CapDev cd = c;
    uniform_opaque(cd.Fx);
    uniform_opaque(cd.rho_ref);
    uniform_opaque(cd.T);
    uniform_opaque(cd.a);
    uniform_opaque(cd.b);
    uniform_opaque(cd.ibr);
    uniform_opaque(cd.kappa);
    uniform_opaque(cd.omega_l);
    const bool bnd = sm != 0u;
    const CT F = (FORCE && !bnd) ? (CT)cd.Fx : CT(0);
    const Mom<CT> m{(CT)mom.drho, (CT)mom.jx, (CT)mom.jy, (CT)mom.pxx, (CT)mom.pxy};
    const CT rho_ref = (CT)cd.rho_ref;
    const CT rho = rho_ref + m.drho;
    const CT inv_rho = recip(rho);
    const CT ux = (FORCE ? m.jx + CT(0.5) * F : m.jx) * inv_rho;
    const CT uy = m.jy * inv_rho;
    const CT T = (CT)cd.T, av = (CT)cd.a;
    const CT ib = recip(CT(1) - (CT)cd.b * rho);
    const CT dX = m.drho * (T * ib * (CT)cd.ibr - av * (rho + rho_ref)) - (CT)cd.kappa * rho * (CT)lapf;
    const CT omega = (CT)cd.omega_l;
    CT lam = CT(0), lam_b = CT(0);
    if (cd.lam_on != 0.f) vdw_lambdas(recip(omega) - CT(0.5), T * ib * ib - CT(2) * av * rho, lam, lam_b);
    collide<CT, float, true, FORCE>(cd, m, rho, ux, uy, dX, lam, lam_b, omega, (CT)dxf, (CT)dyf, F, o);
}

// Post-collision state of one fluid node of the binary model (the wide row
// sweeps share it): from the FP32 moments of its pulled populations, its
// order parameter and the stencils of phi, the bulk pressure and interface
// terms of X (Sec. 3.1), the phi-dependent relaxation rate of Eq. (nu) and the
// MRT relaxation with the non-shear part in type CT, the shear part in ST.
// uxf, uyf: the node's velocity as the sweep formed it from the same moments in
// FP32 ((j + F/2) recip(rho)); the FP32 collision takes it as it is, the FP64
// one forms its own.
template <typename CT, typename ST, bool FORCE>
__device__ __forceinline__ PostState<CT> bin_node_state(const CapDev& c, const Mom<float>& mom, unsigned sm,
                                                        float phi, float dxf, float dyf, float lapf, float uxf,
                                                        float uyf) {
    // constants of the FP64 part, converted where used (see uniform_opaque)
    CapDev cd = c;
    uniform_opaque(cd.kappa);
    uniform_opaque(cd.Fx);
    uniform_opaque(cd.rho_ref);
    uniform_opaque(cd.phib);
    uniform_opaque(cd.B);
    const Mom<CT> mc{(CT)mom.drho, (CT)mom.jx, (CT)mom.jy, (CT)mom.pxx, (CT)mom.pxy};
    const CT F = (FORCE && !sm) ? (CT)cd.Fx : CT(0);
    const CT rho = (CT)cd.rho_ref + mc.drho;
    CT ux, uy;
    if constexpr (sizeof(CT) == 4) {
        ux = uxf;
        uy = uyf;
    } else {
        const CT inv_rho = recip(rho);
        ux = (FORCE ? mc.jx + CT(0.5) * F : mc.jx) * inv_rho;
        uy = mc.jy * inv_rho;
    }
    const CT ph = (CT)phi, phib = (CT)cd.phib;
    const CT dX = mc.drho * (CT(1) / CT(3)) +
                  CT(0.25) * (CT)cd.B * ((ph - phib) * (ph + phib)) * (CT(3) * ph * ph + phib * phib) -
                  (CT)cd.kappa * ph * (CT)lapf;
    // the relaxation rate only scales the shear stresses (FP32) and the
    // forcing term: FP32 with the hardware reciprocal (1 ulp)
    const float pc = phi < -1.f ? -1.f : (phi > 1.f ? 1.f : phi);
    const float nu = cd.nu_g + 0.5f * (pc + 1.f) * (cd.nu_l - cd.nu_g);
    const CT omega = (CT)(2.f * __builtin_amdgcn_rcpf(6.f * nu + 1.f));
    return collide_state<CT, ST, false, FORCE>(cd, mc, rho, ux, uy, dX, CT(0), CT(0), omega, (CT)dxf, (CT)dyf, F);
}

template <typename CT, bool FORCE = true>
__global__ void __launch_bounds__(SW) lb_strip_vdw(StripArgs a) {
    const int si = strip_index(a);
    if (si < 0) return;
    const StripDev s = a.strips[si];
    // by value: one scalar load at entry, kept in registers (a reference would be
    // re-read from memory after every global store of the loop)
    const CapDev c = a.caps[s.cap];
    const Geo g = geo_of(c);
    const int P = (int)c.plane;
    const int sb = a.cur ^ c.par;
    const Planes fs = planes_of((sb ? a.arena1 : a.arena0) + c.off_f, 9, P, c.pitch);
    const Planes fd = planes_of((sb ? a.arena0 : a.arena1) + c.off_f, 9, P, c.pitch);

    __shared__ float Q[3][SW];         // drho rows, column xs-1+k at lane k
    const int k = threadIdx.x;
    // lanes past column xe+1 (the last one that an output column reads) repeat
    // that column: their loads share its addresses
    const int xl = min(s.xs + k - 1, s.xe + 1);
    const LaneCols L = lane_cols(g, xl);
    const bool out_col = k >= 1 && k <= STRIP_OUT && xl < s.xe;
    const float G2 = 2.f * c.G;
    int p3 = 0;   // slot of row ya-1
    auto r3 = [&](int d) { int v = p3 + 1 + d; v -= v >= 3 ? 3 : 0; v -= v >= 3 ? 3 : 0; return v; };

    // FP32 moments of a pulled row (zero at solid nodes): formed when the row
    // arrives, they give the row's entry in Q (drho) and, a row later, the
    // collision's input, so only the request buffers hold populations
    auto moments_row = [&](const float (&f)[9], bool fluid, unsigned sm) {
        return fluid ? moments_of(f, sm != 0u) : Mom<float>{0.f, 0.f, 0.f, 0.f, 0.f};
    };
    // Requests run one row ahead of the arithmetic; the two request buffers swap
    // roles every row (the loop is unrolled by two), so a finished request is
    // never copied (a copy waits for every load in flight).
    float fa[9], fb[9];
    RowInfo ri = row_info(g, s.ya - 1);
    bool fl = !(L.t0 && ri.w0);
    unsigned sm = solid_bits(L, ri);
    pull_lane(fs, L, ri, sm, fa);
    Q[r3(-1)][k] = moments_row(fa, fl, sm).drho;
    ri = row_info(g, s.ya);
    unsigned sm_cur = solid_bits(L, ri);
    bool fl_cur = !(L.t0 && ri.w0);
    pull_lane(fs, L, ri, sm_cur, fa);
    Mom<float> mom_cur = moments_row(fa, fl_cur, sm_cur);
    Q[r3(0)][k] = mom_cur.drho;
    RowInfo ri_n = row_info(g, s.ya + 1);
    unsigned sm_n = solid_bits(L, ri_n);
    bool fl_n = !(L.t0 && ri_n.w0);
    pull_lane(fs, L, ri_n, sm_n, fb);

    // one row y: fn holds the request for row y+1, fp receives the one for row y+2
    auto iter = [&](int y, const float (&fn)[9], float (&fp)[9]) {
        // request for row y+2; in the last row of the chunk it repeats the previous
        // one (cache hits, unused): a load under a branch would make every later
        // wait a wait for all loads
        const RowInfo ri_p = row_info(g, y + 1 < s.yb ? y + 2 : y + 1);
        const unsigned sm_p = solid_bits(L, ri_p);
        const bool fl_p = !(L.t0 && ri_p.w0);
        pull_lane(fs, L, ri_p, sm_p, fp);
        // keep the uses of the previous requests below the new ones
        __builtin_amdgcn_sched_barrier(0);
        const Mom<float> mom_n = moments_row(fn, fl_n, sm_n);
        Q[r3(1)][k] = mom_n.drho;
        wave_sync();
        if (out_col && fl_cur) {
            float dxf, dyf, lapf;
            stencil3(Q[r3(-1)], Q[r3(0)], Q[r3(1)], k, sm_cur, G2, dxf, dyf, lapf);
            CT o[9];
            vdw_node_collide<CT, FORCE>(c, mom_cur, sm_cur, dxf, dyf, lapf, o);
            const int srow = row_info(g, y).y0 * fd.rb;
#pragma unroll
            for (int i = 0; i < 9; ++i) st(fd, (float)o[i], L.b0, i * fd.pb + srow);
        }
        sm_cur = sm_n;
        fl_cur = fl_n;
        sm_n = sm_p;
        fl_n = fl_p;
        mom_cur = mom_n;
        p3 = p3 == 2 ? 0 : p3 + 1;
        wave_sync();
    };
    for (int y = s.ya; y < s.yb; y += 2) {
        iter(y, fb, fa);
        if (y + 1 >= s.yb) break;
        iter(y + 1, fa, fb);
    }
}

}  // namespace lbk
