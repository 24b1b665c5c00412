// Host runtime and C ABI of lbcap (see include/lbcap.h).
//
// A context holds one or more capillaries ("a batch") of the same model in a
// single device allocation:
//   [CapDev table][tile table][l_now][l history][history steps][history count]
//   [health flags][population arena A][population arena B]
// Every capillary owns a region of each arena: 9 FP32 planes of shifted f and,
// for the binary model, one plane of phi, each plane ny x pitch with pitch = nx
// rounded up to 64 floats.  Capillary k reads arena (cur ^ par_k): it holds
// f*(t) (and phi(t+1)); the other arena's phi plane holds phi(t).  A step
// writes the other arena and flips cur.  Retiring a capillary drops its tiles
// and freezes both arenas' regions; reviving it sets par_k so that it reads
// the arena it was frozen in, with no copies.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "lbcap.h"
#include "lb_internal.h"
#include "lb_kernels.h"
#include "lb_strip.h"
#include "lb_strip_table.h"
#include "lb_wide.h"
#include "lb_wide2.h"
#include "lb_wmom.h"
#include "lb_thermo.h"

using namespace lbk;

namespace {

thread_local std::string g_err;

lb_status fail(lb_status s, const std::string& m) {
    g_err = m;
    return s;
}

#define HIP_TRY(call)                                                                         \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return fail(LB_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_));     \
    } while (0)

constexpr size_t ALIGN = 256;
size_t align_up(size_t v, size_t a = ALIGN) { return (v + a - 1) / a * a; }

bool solid_at(const lb_geometry& g, int x, int y) {
    x %= g.nx;
    if (x < 0) x += g.nx;
    y %= g.ny;
    if (y < 0) y += g.ny;
    if (g.tube_len <= 0) return false;
    if (x < g.x_in || x >= g.x_in + g.tube_len) return false;
    return y < g.y0 || y >= g.y0 + g.tube_h;
}

// Every ghost source of the wall rule must be a fluid node.
bool ghost_sources_fluid(const lb_geometry& g) {
    if (g.tube_len <= 0) return true;
    static const int ex[9] = {0, 1, -1, 0, 0, 1, -1, -1, 1};
    static const int ey[9] = {0, 0, 0, 1, -1, 1, -1, 1, -1};
    auto check_node = [&](int x, int y) -> bool {
        if (solid_at(g, x, y)) return true;
        for (int d = 1; d < 9; ++d) {
            if (!solid_at(g, x + ex[d], y + ey[d])) continue;
            int sx, sy;
            if (ex[d] == 0 || ey[d] == 0) {
                sx = x - ex[d];
                sy = y - ey[d];
            } else if (solid_at(g, x + ex[d], y)) {
                sx = x - ex[d];
                sy = y + ey[d];
            } else if (solid_at(g, x, y + ey[d])) {
                sx = x + ex[d];
                sy = y - ey[d];
            } else {
                sx = x - ex[d];
                sy = y - ey[d];
            }
            if (solid_at(g, sx, sy)) return false;
        }
        return true;
    };
    // fluid nodes with a solid neighbour lie on the channel's first and last
    // rows or on the reservoir columns facing the tube's end faces
    const int rows[2] = {g.y0, g.y0 + g.tube_h - 1};
    for (int r : rows)
        for (int x = 0; x < g.nx; ++x)
            if (!check_node(x, r)) return false;
    const int cols[2] = {g.x_in - 1, g.x_in + g.tube_len};
    for (int cx : cols)
        for (int y = 0; y < g.ny; ++y)
            if (!check_node(cx, y)) return false;
    return true;
}

lb_status validate(const lb_params& p, const lb_geometry& g) {
    if (p.model != LB_VDW && p.model != LB_BINARY) return fail(LB_EINVAL, "unknown model");
    if (g.nx < 3 || g.ny < 3) return fail(LB_EINVAL, "lattice must be at least 3x3");
    if ((long long)g.nx * g.ny > (1LL << 31)) return fail(LB_EINVAL, "lattice too large");
    if (g.tube_len < 0) return fail(LB_EINVAL, "negative tube length");
    if (g.tube_len > 0) {
        if (g.x_in < 0 || g.x_in + g.tube_len > g.nx)
            return fail(LB_EINVAL, "tube does not fit in the lattice along x");
        if (g.tube_h < 3 || g.y0 < 1 || g.y0 + g.tube_h > g.ny - 1)
            return fail(LB_EINVAL, "tube rows must satisfy H >= 3, y0 >= 1, y0 + H <= ny - 1");
        if (!ghost_sources_fluid(g)) return fail(LB_EINVAL, "wall ghost source is solid (geometry too thin)");
    }
    if (!(p.nu_l > 0.0) || !std::isfinite(p.nu_l)) return fail(LB_EINVAL, "nu_l must be positive");
    if (p.model == LB_BINARY && (!(p.nu_g > 0.0) || !std::isfinite(p.nu_g)))
        return fail(LB_EINVAL, "nu_g must be positive");
    if (!(p.kappa >= 0.0) || !std::isfinite(p.kappa)) return fail(LB_EINVAL, "kappa must be >= 0");
    if (!std::isfinite(p.force_x)) return fail(LB_EINVAL, "force must be finite");
    if (std::isnan(p.theta_deg) && !std::isfinite(p.wall_grad)) return fail(LB_EINVAL, "wall gradient must be finite");
    if (!std::isnan(p.theta_deg) && !(p.theta_deg > 0.0 && p.theta_deg < 180.0))
        return fail(LB_EINVAL, "contact angle must be in (0, 180)");
    if (p.model == LB_VDW && !(p.b > 0.0 && p.T > 0.0 && std::isfinite(p.a)))
        return fail(LB_EINVAL, "vdW needs b > 0, T > 0");
    if (p.model == LB_BINARY && (!(p.Gamma >= 0.0) || !std::isfinite(p.Gamma) || !std::isfinite(p.A) || !std::isfinite(p.B)))
        return fail(LB_EINVAL, "binary needs finite A, B and Gamma >= 0");
    return LB_OK;
}

struct Layout {
    std::vector<CapDev> caps;
    long long arena_floats = 0;
    long long fluid = 0;
    int max_tiles = 0;
    int max_strips = 0;
    size_t off_strips = 0;
    size_t off_caps, off_tiles, off_lnow, off_hist, off_hist_t, off_hist_n, off_flags, off_arena0, off_arena1,
        total;
};

int count_tiles(const lb_geometry& g, int rows) {
    int n = 0;
    for (int y0 = 0; y0 < g.ny; y0 += rows)
        for (int x0 = 0; x0 < g.nx; x0 += TILE_W) {
            bool any = false;
            for (int y = y0; y < std::min(y0 + rows, g.ny) && !any; ++y) {
                const bool wall_row = g.tube_len > 0 && (y < g.y0 || y >= g.y0 + g.tube_h);
                if (!wall_row) {
                    any = true;
                    break;
                }
                const int xe = std::min(x0 + TILE_W, g.nx);
                if (x0 < g.x_in || xe > g.x_in + g.tube_len) any = true;
            }
            n += any;
        }
    return n;
}

void build_tiles(const std::vector<lb_geometry>& G, const std::vector<int>& active, int rows,
                 std::vector<TileDev>& out) {
    out.clear();
    for (size_t k = 0; k < G.size(); ++k) {
        if (!active[k]) continue;
        const lb_geometry& g = G[k];
        for (int y0 = 0; y0 < g.ny; y0 += rows)
            for (int x0 = 0; x0 < g.nx; x0 += TILE_W) {
                bool any = false;
                for (int y = y0; y < std::min(y0 + rows, g.ny) && !any; ++y) {
                    const bool wall_row = g.tube_len > 0 && (y < g.y0 || y >= g.y0 + g.tube_h);
                    if (!wall_row) any = true;
                    const int xe = std::min(x0 + TILE_W, g.nx);
                    if (x0 < g.x_in || xe > g.x_in + g.tube_len) any = true;
                }
                if (any) out.push_back(TileDev{(int)k, x0, y0, std::min(rows, g.ny - y0)});
            }
    }
}

lb_status make_layout(int n, const lb_params* P, const lb_geometry* G, Layout& L) {
    L.caps.resize(n);
    long long off = 0;
    L.fluid = 0;
    L.max_tiles = 0;
    for (int k = 0; k < n; ++k) {
        const lb_params& p = P[k];
        const lb_geometry& g = G[k];
        lb_status s = validate(p, g);
        if (s) return s;
        if (p.model != P[0].model) return fail(LB_EINVAL, "all capillaries of a batch must use one model");
        CapDev c;
        std::memset(&c, 0, sizeof c);
        c.nx = g.nx;
        c.ny = g.ny;
        c.pitch = (int)align_up((size_t)g.nx, TILE_W);
        c.x_in = g.tube_len > 0 ? g.x_in : 0;
        c.x_end = g.tube_len > 0 ? g.x_in + g.tube_len : 0;
        c.y0 = g.tube_len > 0 ? g.y0 : 0;
        c.y1 = g.tube_len > 0 ? g.y0 + g.tube_h : 0;
        c.active = 1;
        c.par = 0;
        c.plane = (long long)g.ny * c.pitch;
        // the kernels address one capillary's planes with 32-bit byte offsets
        if (10 * 4 * c.plane > 0x7fffffffLL) return fail(LB_EINVAL, "lattice too large: one capillary's state must stay below 2 GiB");
        c.off_f = off;
        c.off_phi = off + 9 * c.plane;
        off += (p.model == LB_BINARY ? 10 : 9) * c.plane;
        c.kappa = (float)p.kappa;
        c.a = (float)p.a;
        c.b = (float)p.b;
        c.T = (float)p.T;
        c.A = (float)p.A;
        c.B = (float)p.B;
        c.Gamma = (float)p.Gamma;
        c.nu_l = (float)p.nu_l;
        c.nu_g = (float)(p.model == LB_BINARY ? p.nu_g : p.nu_l);
        c.omega_l = (float)(2.0 / (6.0 * p.nu_l + 1.0));
        double G = p.wall_grad;
        if (!std::isnan(p.theta_deg)) {
            lb_status s2 = lb_wall_gradient_for_angle(&p, p.theta_deg, &G);
            if (s2) return s2;
        }
        c.G = (float)G;
        c.Fx = (float)p.force_x;
        c.lam_on = (p.model == LB_VDW && p.lambda_mode == 0) ? 1.f : 0.f;
        // vdW mid density: mean of the coexisting densities (critical density above Tc)
        double mid = 0.0;
        if (p.model == LB_VDW) {
            double rl, rg;
            mid = lbt::vdw_coexistence(p.a, p.b, p.T, &rl, &rg) ? 0.5 * (rl + rg) : 1.0 / (3.0 * p.b);
        }
        const double qm = std::isnan(p.q_mid) ? mid : p.q_mid;
        c.q_mid = (float)qm;
        // reference rest state of the shifted f storage
        if (p.model == LB_VDW) {
            const double rr = mid;
            c.rho_ref = (float)rr;
            c.X_ref = (float)(rr * p.T / (1.0 - p.b * rr) - p.a * rr * rr);
            c.ibr = (float)(1.0 / (1.0 - p.b * (double)c.rho_ref));
            c.phib2 = 0.f;
        } else {
            c.rho_ref = 1.f;
            c.X_ref = (float)(1.0 / 3.0 + p.A * p.A / (4.0 * p.B));
            c.ibr = 0.f;
            c.phib2 = (float)(p.A / p.B);
            c.phib = (float)std::sqrt(p.A / p.B);
        }
        c.hist_off = k * LB_HISTORY_CAP;
        L.caps[k] = c;
        long long solid = g.tube_len > 0 ? (long long)g.tube_len * (g.ny - g.tube_h) : 0;
        L.fluid += (long long)g.nx * g.ny - solid;
        L.max_tiles += count_tiles(g, 1);
    }
    L.arena_floats = off;
    {
        // room for the strip table of either width at any chunking
        const std::vector<lb_geometry> gv(G, G + n);
        L.max_strips = std::max(strip_capacity(gv, STRIP_OUT), strip_capacity(gv, WIDE_OUT));
    }
    size_t o = 0;
    L.off_caps = o;
    o = align_up(o + sizeof(CapDev) * n);
    L.off_tiles = o;
    o = align_up(o + sizeof(TileDev) * (size_t)L.max_tiles);
    L.off_strips = o;
    o = align_up(o + sizeof(StripDev) * (size_t)L.max_strips);
    L.off_lnow = o;
    o = align_up(o + sizeof(float) * n);
    L.off_hist = o;
    o = align_up(o + sizeof(float) * (size_t)n * LB_HISTORY_CAP);
    L.off_hist_t = o;
    o = align_up(o + sizeof(long long) * (size_t)n * LB_HISTORY_CAP);
    L.off_hist_n = o;
    o = align_up(o + sizeof(int) * n);
    L.off_flags = o;
    o = align_up(o + sizeof(int) * n);
    L.off_arena0 = o;
    o = align_up(o + sizeof(float) * (size_t)L.arena_floats);
    L.off_arena1 = o;
    o = align_up(o + sizeof(float) * (size_t)L.arena_floats);
    L.total = o;
    return LB_OK;
}

uint64_t fnv1a(const void* p, size_t n, uint64_t h = 1469598103934665603ULL) {
    const unsigned char* c = (const unsigned char*)p;
    for (size_t i = 0; i < n; ++i) {
        h ^= c[i];
        h *= 1099511628211ULL;
    }
    return h;
}

// Launch shapes found by lb_autotune, per (model, size class); a context uses
// one only when its caller asks (lb_use_tuned_launch_config), so that a run's
// launch shape never depends on what else the process tuned before it.
std::mutex g_tune_mu;
std::map<std::pair<int, int>, lb_launch_config> g_tune_cache;

// floor(log2(fluid nodes)): the size class of the tuning cache
int size_class(long long fluid) {
    int c = 0;
    while (fluid > 1) {
        fluid >>= 1;
        ++c;
    }
    return c;
}

}  // namespace

struct lb_ctx {
    int model = 0;
    int n = 0;
    std::vector<lb_params> P;
    std::vector<lb_geometry> G;
    Layout L;
    std::vector<int> active;
    std::vector<int> frozen_buf;  // read-arena of a retired capillary
    char* mem = nullptr;
    bool own_mem = false;
    CapDev* d_caps = nullptr;
    TileDev* d_tiles = nullptr;
    int ntiles = 0;
    StripDev* d_strips = nullptr;
    int nstrips = 0;
    int xcd_start[9] = {};    // strip runs of the 8 XCDs
    float* d_lnow = nullptr;
    float* d_hist = nullptr;
    long long* d_hist_t = nullptr;
    int* d_hist_n = nullptr;
    int* d_flags = nullptr;
    float* arena[2] = {nullptr, nullptr};
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int cur = 0;
    long t = 0;
    lb_launch_config cfg{4, 4, 4, 64, 0, 8};
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    hipGraph_t graph[2] = {nullptr, nullptr};
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    long timed_steps = 0;
    int unstable = 0;
    bool any_force = false;   // some capillary has a body force (row sweeps keep the forcing terms)
    int mstore = 0;           // 1: the arenas hold the seven-plane post-collision state (schedule 6)
};

namespace {

void drop_graphs(lb_ctx* c) {
    for (int p = 0; p < 2; ++p) {
        if (c->gexec[p]) (void)hipGraphExecDestroy(c->gexec[p]);
        if (c->graph[p]) (void)hipGraphDestroy(c->graph[p]);
        c->gexec[p] = nullptr;
        c->graph[p] = nullptr;
    }
}

// Converts the f regions of arena b of every capillary to the storage
// `to_state` (1: seven-plane post-collision state, 0: nine populations).
lb_status convert_arena(lb_ctx* c, int b, int to_state) {
    long long most = 0;
    for (const CapDev& d : c->L.caps) most = std::max(most, d.plane);
    const int gx = (int)std::min<long long>((most + 255) / 256, 1024);
    const int gy = std::min(c->n, 65535);   // the kernel strides over further capillaries
    if (to_state)
        hipLaunchKernelGGL(lb_convert_kernel<true>, dim3(gx, gy), dim3(256), 0, c->stream, c->d_caps, c->n,
                           c->arena[b]);
    else
        hipLaunchKernelGGL(lb_convert_kernel<false>, dim3(gx, gy), dim3(256), 0, c->stream, c->d_caps, c->n,
                           c->arena[b]);
    HIP_TRY(hipGetLastError());
    return LB_OK;
}

// Records the storage the arenas hold (without converting them).
lb_status mark_storage(lb_ctx* c, int m) {
    c->mstore = m;
    for (CapDev& d : c->L.caps) d.mstore = m;
    HIP_TRY(hipMemcpyAsync(c->d_caps, c->L.caps.data(), sizeof(CapDev) * c->n, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return LB_OK;
}

// Switches both arenas (all capillaries, retired ones too) to storage m.
lb_status set_storage(lb_ctx* c, int m) {
    if (m == c->mstore) return LB_OK;
    for (int b = 0; b < 2; ++b)
        if (lb_status s = convert_arena(c, b, m)) return s;
    return mark_storage(c, m);
}

// output columns per strip of the row-sweep schedules (3: one wavefront, 4: a workgroup)
int strip_width(const lb_launch_config& cfg) { return cfg.schedule >= 4 ? WIDE_OUT : STRIP_OUT; }

// time steps one launch of the step kernel advances (schedule 5: two per sweep)
int steps_per_launch(const lb_launch_config& cfg) { return cfg.schedule == 5 ? 2 : 1; }

lb_status upload_tiles(lb_ctx* c) {
    std::vector<TileDev> tiles;
    build_tiles(c->G, c->active, c->cfg.tile_rows, tiles);
    if ((int)tiles.size() > c->L.max_tiles) return fail(LB_EINVAL, "tile table overflow");
    c->ntiles = (int)tiles.size();
    if (!tiles.empty())
        HIP_TRY(hipMemcpyAsync(c->d_tiles, tiles.data(), sizeof(TileDev) * tiles.size(), hipMemcpyHostToDevice,
                               c->stream));
    std::vector<StripDev> strips;
    build_strips(c->G, c->active, c->cfg.chunk_rows, strip_width(c->cfg), 2, &strips, nullptr, c->xcd_start);
    if ((int)strips.size() > c->L.max_strips) return fail(LB_EINVAL, "strip table overflow");
    c->nstrips = (int)strips.size();
    if (!strips.empty())
        HIP_TRY(hipMemcpyAsync(c->d_strips, strips.data(), sizeof(StripDev) * strips.size(), hipMemcpyHostToDevice,
                               c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    drop_graphs(c);
    return LB_OK;
}

template <int MODEL, int TY, bool INIT, typename R>
void launch_step_t(lb_ctx* c, const StepArgs& a, int grid) {
    hipLaunchKernelGGL((lb_step_kernel<MODEL, TY, INIT, R>), dim3(grid), dim3(TILE_W, TY), 0, c->stream, a);
}

template <int MODEL, bool INIT, typename R>
void launch_step_r(lb_ctx* c, const StepArgs& a, int grid) {
    switch (c->cfg.tile_rows) {
        case 1: launch_step_t<MODEL, 1, INIT, R>(c, a, grid); break;
        case 2: launch_step_t<MODEL, 2, INIT, R>(c, a, grid); break;
        case 8: launch_step_t<MODEL, 8, INIT, R>(c, a, grid); break;
        default: launch_step_t<MODEL, 4, INIT, R>(c, a, grid); break;
    }
}

template <int MODEL, bool INIT>
void launch_step_m(lb_ctx* c, const StepArgs& a, int grid) {
    if (c->cfg.fp64_arith)
        launch_step_r<MODEL, INIT, double>(c, a, grid);
    else
        launch_step_r<MODEL, INIT, float>(c, a, grid);
}

int grid_of(const lb_ctx* c) {
    const int n = c->ntiles;
    if (c->cfg.schedule == 1) return 8 * ((n + 7) / 8);
    if (c->cfg.schedule == 2) return std::max(1, std::min(n, c->cfg.persist_blocks_per_cu * 256));
    return n;
}

// Extra (unused) LDS per one-wavefront binary strip: with it at most 16 strips
// share a CU (4 wavefronts per SIMD), which measured faster than the 5 that
// its registers would allow.
constexpr size_t STRIP_BIN_LDS_PAD = 6 * 1024;

template <int MODEL, typename MT, typename CT, typename ST, bool FORCE>
void launch_strip_f(lb_ctx* c, const StripArgs& a, int grid, bool fused) {
    const bool wide = c->cfg.schedule >= 4;
    if constexpr (MODEL == 0) {
        if (fused)
            hipLaunchKernelGGL((lb_wide2_vdw<CT, FORCE>), dim3(grid), dim3(WIDE_THREADS), 0, c->stream, a);
        else if (wide)
            hipLaunchKernelGGL((lb_wide_vdw<CT, FORCE>), dim3(grid), dim3(WIDE_THREADS), 0, c->stream, a);
        else
            hipLaunchKernelGGL((lb_strip_vdw<CT, FORCE>), dim3(grid), dim3(SW), 0, c->stream, a);
    } else {
        if (fused)
            hipLaunchKernelGGL((lb_wide2_bin<MT, CT, ST, FORCE>), dim3(grid), dim3(WIDE_THREADS), 0, c->stream, a);
        else if (c->cfg.schedule == 6)
            hipLaunchKernelGGL((lb_wmom_bin<MT, CT, ST, FORCE>), dim3(grid), dim3(WIDE_THREADS), 0, c->stream, a);
        else if (wide)
            hipLaunchKernelGGL((lb_wide_bin<MT, CT, ST, FORCE>), dim3(grid), dim3(WIDE_THREADS), 0, c->stream, a);
        else
            hipLaunchKernelGGL((lb_strip_bin<MT, CT, ST, FORCE>), dim3(grid), dim3(SW), STRIP_BIN_LDS_PAD,
                               c->stream, a);
    }
}

// without a body force anywhere in the batch the forcing terms are compiled out
template <int MODEL, typename MT, typename CT, typename ST = CT>
void launch_strip_t(lb_ctx* c, const StripArgs& a, int grid, bool fused) {
    if (c->any_force)
        launch_strip_f<MODEL, MT, CT, ST, true>(c, a, grid, fused);
    else
        launch_strip_f<MODEL, MT, CT, ST, false>(c, a, grid, fused);
}

// Enqueue one step (or the initialisation when init is true) from arena cur;
// fused: two steps in one sweep (schedule 5), else a single step (schedule 5
// then takes the single-step wide strips, for odd step counts).
void enqueue_step(lb_ctx* c, bool init, bool fused = false) {
    if (c->ntiles == 0) return;
    if (!init && c->cfg.schedule >= 3) {
        if (c->nstrips == 0) return;
        StripArgs a;
        a.caps = c->d_caps;
        a.strips = c->d_strips;
        a.nstrips = c->nstrips;
        int longest = 0;
        for (int x = 0; x < 8; ++x) {
            a.xcd_start[x] = c->xcd_start[x];
            longest = std::max(longest, c->xcd_start[x + 1] - c->xcd_start[x]);
        }
        a.xcd_start[8] = c->xcd_start[8];
        a.arena0 = c->arena[0];
        a.arena1 = c->arena[1];
        a.cur = c->cur;
        const int grid = 8 * longest;
        if (c->model == LB_VDW) {
            if (c->cfg.fp64_arith)
                launch_strip_t<0, double, double>(c, a, grid, fused);
            else
                launch_strip_t<0, float, float>(c, a, grid, fused);
        } else {
            // the collision's non-shear part in FP64 (the shear relaxation is exact enough in FP32)
            if (c->cfg.fp64_arith)
                launch_strip_t<1, float, double, float>(c, a, grid, fused);
            else
                launch_strip_t<1, float, float, float>(c, a, grid, fused);
        }
        return;
    }
    StepArgs a;
    a.caps = c->d_caps;
    a.tiles = c->d_tiles;
    a.ntiles = c->ntiles;
    a.schedule = init ? 0 : c->cfg.schedule;
    a.arena0 = c->arena[0];
    a.arena1 = c->arena[1];
    // the initialisation reads the field uploaded into arena 1, writes arena 0
    a.cur = init ? 1 : c->cur;
    a.init = init ? 1 : 0;
    const int grid = init ? c->ntiles : grid_of(c);
    if (c->model == LB_VDW) {
        if (init)
            launch_step_m<0, true>(c, a, grid);
        else
            launch_step_m<0, false>(c, a, grid);
    } else {
        if (init)
            launch_step_m<1, true>(c, a, grid);
        else
            launch_step_m<1, false>(c, a, grid);
    }
}

// Every launch reads arena cur and writes the other one, so each flips cur,
// whether it advances one time step or two.  A run of graph_steps steps is
// one graph per starting arena (capture does not execute).
lb_status capture_graph(lb_ctx* c, int p) {
    const int spl = steps_per_launch(c->cfg);
    const int launches = c->cfg.graph_steps / spl;
    const int keep = c->cur;
    c->cur = p;
    HIP_TRY(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    for (int s = 0; s < launches; ++s) {
        enqueue_step(c, false, spl == 2);
        c->cur ^= 1;
    }
    c->cur = keep;
    hipGraph_t gr = nullptr;
    HIP_TRY(hipStreamEndCapture(c->stream, &gr));
    c->graph[p] = gr;
    HIP_TRY(hipGraphInstantiate(&c->gexec[p], gr, nullptr, nullptr, 0));
    return LB_OK;
}

bool graphs_used(const lb_ctx* c, long n) {
    const int K = c->cfg.graph_steps;
    return K >= 2 && (K % 2) == 0 && n >= K && c->ntiles > 0;
}

// The graphs a run of n steps will replay, captured beforehand (so that the
// capture is not inside a caller's timed region).
lb_status prepare_graphs(lb_ctx* c, long n) {
    if (!graphs_used(c, n)) return LB_OK;
    const int launches = c->cfg.graph_steps / steps_per_launch(c->cfg);
    const int parities = (launches & 1) && n >= 2L * c->cfg.graph_steps ? 2 : 1;
    for (int q = 0; q < parities; ++q) {
        const int p = c->cur ^ q;
        if (!c->gexec[p])
            if (lb_status s = capture_graph(c, p)) return s;
    }
    return LB_OK;
}

// readable: leave the state as the read-outs expect it.  They take phi (binary
// model) from the buffer that the last step read: after a single step that is
// phi of the state's own time, after a two-step launch the phi of the step
// before (the one in between stays in LDS).  With two steps per launch the
// binary model's last step is therefore a single step.
lb_status run_steps(lb_ctx* c, long n, bool readable = true) {
    const int K = c->cfg.graph_steps;
    const int spl = steps_per_launch(c->cfg);
    const bool tail = readable && spl == 2 && c->model == LB_BINARY && n > 0;
    if (tail) --n;
    if (graphs_used(c, n)) {
        const int launches = K / spl;   // K is even
        while (n >= K) {
            if (!c->gexec[c->cur])
                if (lb_status s = capture_graph(c, c->cur)) return s;
            HIP_TRY(hipGraphLaunch(c->gexec[c->cur], c->stream));
            c->cur ^= launches & 1;
            c->t += K;
            n -= K;
        }
    }
    for (; n >= spl; n -= spl) {
        enqueue_step(c, false, spl == 2);
        c->cur ^= 1;
        c->t += spl;
    }
    if (n > 0) {   // an odd step of a two-step schedule
        enqueue_step(c, false, false);
        c->cur ^= 1;
        c->t += 1;
    }
    if (tail) {
        enqueue_step(c, false, false);
        c->cur ^= 1;
        c->t += 1;
    }
    HIP_TRY(hipGetLastError());
    return LB_OK;
}

lb_status check_ctx(const lb_ctx* c) {
    if (!c) return fail(LB_EINVAL, "null context");
    return LB_OK;
}

lb_status create(lb_ctx** out, int n, const lb_params* P, const lb_geometry* G, const double* const* init_q,
                 void* d_state, size_t bytes, void* stream) {
    if (!out) return fail(LB_EINVAL, "null output pointer");
    *out = nullptr;
    if (n < 1 || !P || !G || !init_q) return fail(LB_EINVAL, "need at least one capillary with parameters, geometry and initial field");
    lb_ctx* c = new lb_ctx();
    c->n = n;
    c->model = P[0].model;
    c->P.assign(P, P + n);
    c->G.assign(G, G + n);
    lb_status s = make_layout(n, P, G, c->L);
    if (s) {
        delete c;
        return s;
    }
    for (const CapDev& d : c->L.caps) c->any_force = c->any_force || d.Fx != 0.f;
    // initial fields: finite, and inside the van der Waals range
    for (int k = 0; k < n; ++k) {
        if (!init_q[k]) {
            delete c;
            return fail(LB_EINVAL, "null initial field");
        }
        const lb_geometry& g = G[k];
        for (int y = 0; y < g.ny; ++y)
            for (int x = 0; x < g.nx; ++x) {
                if (solid_at(g, x, y)) continue;
                const double v = init_q[k][(size_t)y * g.nx + x];
                if (!std::isfinite(v)) {
                    delete c;
                    return fail(LB_EINVAL, "non-finite initial field");
                }
                if (c->model == LB_VDW && !(v > 0.0 && P[k].b * v < 1.0)) {
                    delete c;
                    return fail(LB_EINVAL, "vdW initial density must satisfy 0 < rho < 1/b");
                }
                if (c->model == LB_BINARY && !(std::fabs(v) < 3.5)) {
                    delete c;
                    return fail(LB_EINVAL, "binary initial phi must satisfy |phi| < 3.5 (fixed-point range 4)");
                }
            }
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
        delete c;
        return fail(LB_EDEVICE, "no HIP device");
    }
    if (d_state) {
        if (bytes < c->L.total || ((uintptr_t)d_state % ALIGN) != 0) {
            delete c;
            return fail(LB_EINVAL, "d_state too small or not 256-byte aligned");
        }
        c->mem = (char*)d_state;
    } else {
        if (hipMalloc(&c->mem, c->L.total) != hipSuccess) {
            delete c;
            return fail(LB_ENOMEM, "device allocation of the lattice state failed");
        }
        c->own_mem = true;
    }
    c->d_caps = (CapDev*)(c->mem + c->L.off_caps);
    c->d_tiles = (TileDev*)(c->mem + c->L.off_tiles);
    c->d_strips = (StripDev*)(c->mem + c->L.off_strips);
    c->d_lnow = (float*)(c->mem + c->L.off_lnow);
    c->d_hist = (float*)(c->mem + c->L.off_hist);
    c->d_hist_t = (long long*)(c->mem + c->L.off_hist_t);
    c->d_hist_n = (int*)(c->mem + c->L.off_hist_n);
    c->d_flags = (int*)(c->mem + c->L.off_flags);
    c->arena[0] = (float*)(c->mem + c->L.off_arena0);
    c->arena[1] = (float*)(c->mem + c->L.off_arena1);
    c->active.assign(n, 1);
    c->frozen_buf.assign(n, 0);
    if (stream) {
        c->stream = (hipStream_t)stream;
    } else {
        if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
            lb_free(c);
            return fail(LB_EDEVICE, "stream creation failed");
        }
        c->own_stream = true;
    }
    if (hipEventCreate(&c->ev0) != hipSuccess || hipEventCreate(&c->ev1) != hipSuccess) {
        lb_free(c);
        return fail(LB_EDEVICE, "event creation failed");
    }
    auto bail = [&](lb_status st) {
        std::string m = g_err;
        lb_free(c);
        g_err = m;
        return st;
    };
    if (hipMemcpyAsync(c->d_caps, c->L.caps.data(), sizeof(CapDev) * n, hipMemcpyHostToDevice, c->stream) != hipSuccess ||
        hipMemsetAsync(c->d_hist_n, 0, sizeof(int) * n, c->stream) != hipSuccess ||
        hipMemsetAsync(c->d_flags, 0, sizeof(int) * n, c->stream) != hipSuccess ||
        hipMemsetAsync(c->d_lnow, 0, sizeof(float) * n, c->stream) != hipSuccess)
        return bail(fail(LB_EDEVICE, "upload of descriptors failed"));
    // default launch shape: the moment storage for the binary model (its
    // fastest sweep), the wide population sweep for van der Waals
    if (c->model == LB_BINARY) {
        c->cfg.schedule = 6;
        c->cfg.chunk_rows = 20;
    }
    s = upload_tiles(c);
    if (s) return bail(s);
    // initial fields go to arena 1 as FP32 planes (pitched): the phi plane for
    // the binary model, plane 0 for vdW; that plane of arena 1 then holds
    // phi(0) / is rewritten by the first step
    for (int k = 0; k < n; ++k) {
        const lb_geometry& g = G[k];
        const CapDev& d = c->L.caps[k];
        std::vector<float> h((size_t)g.nx * g.ny);
        for (size_t i = 0; i < h.size(); ++i) {
            if (c->model == LB_BINARY) {   // phi in fixed point (29 fraction bits)
                const int q = (int)std::lrint(init_q[k][i] * 536870912.0);
                std::memcpy(&h[i], &q, sizeof q);
            } else {
                h[i] = (float)init_q[k][i];
            }
        }
        float* dst = c->arena[1] + (c->model == LB_BINARY ? d.off_phi : d.off_f);
        if (hipMemcpy2DAsync(dst, sizeof(float) * d.pitch, h.data(), sizeof(float) * g.nx, sizeof(float) * g.nx,
                             g.ny, hipMemcpyHostToDevice, c->stream) != hipSuccess ||
            hipStreamSynchronize(c->stream) != hipSuccess)
            return bail(fail(LB_EDEVICE, "upload of the initial field failed"));
    }
    // the initialisation always uses one workgroup per tile
    const lb_launch_config keep = c->cfg;
    enqueue_step(c, true);
    c->cfg = keep;
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(c->stream) != hipSuccess)
        return bail(fail(LB_EDEVICE, "initialisation kernel failed"));
    c->cur = 0;
    c->t = 0;
    // the initialisation writes populations; the moment storage converts them
    if (lb_status s2 = set_storage(c, c->cfg.schedule == 6 ? 1 : 0)) return bail(s2);
    *out = c;
    return LB_OK;
}

// Arena capillary k reads (holds f*(t)); the other one holds phi(t).
int buf_of(const lb_ctx* c, int k) { return c->active[k] ? (c->cur ^ c->L.caps[k].par) : c->frozen_buf[k]; }

lb_status moments_into(lb_ctx* c, int k, float* rho, float* ux, float* uy, float* phi) {
    const int b = buf_of(c, k);
    const float* st = c->arena[b];
    const float* prev = c->arena[b ^ 1];
    const long long n = (long long)c->G[k].nx * c->G[k].ny;
    const int grid = (int)std::min<long long>((n + 255) / 256, 4096);
    if (c->model == LB_VDW)
        hipLaunchKernelGGL(lb_moments_kernel<0>, dim3(grid), dim3(256), 0, c->stream, c->d_caps, k, st, prev, rho,
                           ux, uy, phi);
    else
        hipLaunchKernelGGL(lb_moments_kernel<1>, dim3(grid), dim3(256), 0, c->stream, c->d_caps, k, st, prev, rho,
                           ux, uy, phi);
    HIP_TRY(hipGetLastError());
    return LB_OK;
}

lb_status host_moments(lb_ctx* c, int k, double* rho, double* ux, double* uy, double* phi) {
    const long long n = (long long)c->G[k].nx * c->G[k].ny;
    // scratch: planes 0..3 of the capillary's f region in the arena it does
    // not read (rewritten by its next step; that arena's phi plane is untouched)
    float* scratch = c->arena[buf_of(c, k) ^ 1] + c->L.caps[k].off_f;
    float* out[4] = {scratch, scratch + n, scratch + 2 * n, scratch + 3 * n};
    lb_status s = moments_into(c, k, out[0], out[1], out[2], out[3]);
    if (s) return s;
    std::vector<float> h((size_t)(4 * n));
    HIP_TRY(hipMemcpyAsync(h.data(), scratch, sizeof(float) * 4 * n, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    double* dst[4] = {rho, ux, uy, phi};
    bool bad = false;
    for (int q = 0; q < 4; ++q) {
        for (long long i = 0; i < n; ++i) {
            const float v = h[(size_t)(q * n + i)];
            if (!std::isfinite(v)) bad = true;
            if (dst[q]) dst[q][i] = v;
        }
    }
    if (bad) {
        c->unstable = 1;
        return fail(LB_EUNSTABLE, "non-finite field");
    }
    return LB_OK;
}

lb_status launch_interface(lb_ctx* c, int record) {
    if (c->model == LB_VDW)
        hipLaunchKernelGGL(lb_interface_kernel<0>, dim3(c->n), dim3(256), 0, c->stream, c->d_caps, c->n,
                           c->arena[0], c->arena[1], c->cur, c->d_lnow, c->d_hist, c->d_hist_t, c->d_hist_n,
                           LB_HISTORY_CAP, (long long)c->t, record);
    else
        hipLaunchKernelGGL(lb_interface_kernel<1>, dim3(c->n), dim3(256), 0, c->stream, c->d_caps, c->n,
                           c->arena[0], c->arena[1], c->cur, c->d_lnow, c->d_hist, c->d_hist_t, c->d_hist_n,
                           LB_HISTORY_CAP, (long long)c->t, record);
    HIP_TRY(hipGetLastError());
    return LB_OK;
}

lb_status launch_health(lb_ctx* c) {
    if (c->ntiles == 0) return LB_OK;
    const int grid = std::min(c->ntiles, 2048);
    // 512 threads: 8 rows of 64 (tiles have at most 8 rows)
    if (c->model == LB_VDW)
        hipLaunchKernelGGL(lb_health_kernel<0>, dim3(grid), dim3(512), 0, c->stream, c->d_caps, c->d_tiles,
                           c->ntiles, c->arena[0], c->arena[1], c->cur, c->d_flags);
    else
        hipLaunchKernelGGL(lb_health_kernel<1>, dim3(grid), dim3(512), 0, c->stream, c->d_caps, c->d_tiles,
                           c->ntiles, c->arena[0], c->arena[1], c->cur, c->d_flags);
    HIP_TRY(hipGetLastError());
    return LB_OK;
}

lb_status cap_index(const lb_ctx* c, int cap) {
    if (cap < 0 || cap >= c->n) return fail(LB_EINVAL, "capillary index out of range");
    return LB_OK;
}

lb_status set_active(lb_ctx* c, int k, int on) {
    if (c->active[k] == on) return LB_OK;
    if (!on) {
        c->frozen_buf[k] = c->cur ^ c->L.caps[k].par;
    } else {
        c->L.caps[k].par = c->cur ^ c->frozen_buf[k];
    }
    c->active[k] = on;
    c->L.caps[k].active = on;
    HIP_TRY(hipMemcpyAsync(&c->d_caps[k], &c->L.caps[k], sizeof(CapDev), hipMemcpyHostToDevice, c->stream));
    return upload_tiles(c);
}

// Plain copy, one 16-byte element per thread (the fastest of the simple copy
// shapes on this GPU): the achievable-bandwidth reference of the step kernel's
// roofline and the calibration kernel of the HBM byte counters.
__global__ void __launch_bounds__(256) lb_copy_kernel(const float4* __restrict__ src, float4* __restrict__ dst,
                                                      size_t n4) {
    const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (i < n4) dst[i] = src[i];
}

}  // namespace

// error hook of the other translation units of the library
lb_status lbk::set_error(lb_status s, const char* msg) { return fail(s, msg); }

extern "C" {

lb_status lb_stream_copy(void* dst, const void* src, size_t bytes, void* hip_stream) {
    if (!dst || !src || bytes % 16 != 0 || ((uintptr_t)dst % 16) != 0 || ((uintptr_t)src % 16) != 0)
        return fail(LB_EINVAL, "copy needs 16-byte aligned pointers and a multiple of 16 bytes");
    const size_t n4 = bytes / 16;
    if (n4 == 0) return LB_OK;
    if ((n4 + 255) / 256 > 0x7fffffffull) return fail(LB_EINVAL, "copy too large");
    const unsigned grid = (unsigned)((n4 + 255) / 256);
    hipLaunchKernelGGL(lb_copy_kernel, dim3(grid), dim3(256), 0, (hipStream_t)hip_stream, (const float4*)src,
                       (float4*)dst, n4);
    HIP_TRY(hipGetLastError());
    return LB_OK;
}

const char* lb_last_error(void) { return g_err.c_str(); }

size_t lb_state_bytes(const lb_params* p, const lb_geometry* g) {
    if (!p || !g) return 0;
    Layout L;
    if (make_layout(1, p, g, L) != LB_OK) return 0;
    return L.total;
}

lb_status lb_init(lb_ctx** out, const lb_params* p, const lb_geometry* g, const double* init_q, void* d_state,
                  size_t bytes, void* hip_stream) {
    const double* q[1] = {init_q};
    return create(out, 1, p, g, q, d_state, bytes, hip_stream);
}

lb_status lb_batch_init(lb_ctx** out, int n, const lb_params* p, const lb_geometry* g, const double* const* init_q,
                        void* hip_stream) {
    return create(out, n, p, g, init_q, nullptr, 0, hip_stream);
}

lb_status lb_step(lb_ctx* c, long nsteps) { return lb_batch_step(c, nsteps, 0); }

lb_status lb_batch_step(lb_ctx* c, long nsteps, int sample_every) {
    if (lb_status s = check_ctx(c)) return s;
    if (nsteps < 0 || sample_every < 0) return fail(LB_EINVAL, "negative step count");
    // graphs are captured before the timing events, which then bracket the launches only
    if (lb_status s = prepare_graphs(c, sample_every > 0 ? std::min<long>(nsteps, sample_every) : nsteps)) return s;
    HIP_TRY(hipEventRecord(c->ev0, c->stream));
    long left = nsteps;
    while (left > 0) {
        long chunk = left;
        if (sample_every > 0) chunk = std::min(left, sample_every - (c->t % sample_every));
        lb_status s = run_steps(c, chunk);
        if (s) return s;
        left -= chunk;
        if (sample_every > 0 && c->t % sample_every == 0) {
            if ((s = launch_interface(c, 1))) return s;
            if ((s = launch_health(c))) return s;
        }
    }
    HIP_TRY(hipEventRecord(c->ev1, c->stream));
    c->timed_steps = nsteps;
    return LB_OK;
}

lb_status lb_last_step_kernel_us(lb_ctx* c, double* us) {
    if (lb_status s = check_ctx(c)) return s;
    if (!us) return fail(LB_EINVAL, "null output");
    *us = 0.0;
    if (c->timed_steps <= 0) return LB_OK;
    HIP_TRY(hipEventSynchronize(c->ev1));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, c->ev0, c->ev1));
    *us = 1000.0 * ms / (double)c->timed_steps;
    return LB_OK;
}

long lb_time(const lb_ctx* c) { return c ? c->t : -1; }

int lb_batch_size(const lb_ctx* c) { return c ? c->n : 0; }

long long lb_fluid_nodes(const lb_ctx* c) { return c ? c->L.fluid : 0; }

lb_status lb_batch_health(lb_ctx* c, int* flags) {
    if (lb_status s = check_ctx(c)) return s;
    HIP_TRY(hipMemsetAsync(c->d_flags, 0, sizeof(int) * c->n, c->stream));
    if (lb_status s = launch_health(c)) return s;
    std::vector<int> h(c->n);
    HIP_TRY(hipMemcpyAsync(h.data(), c->d_flags, sizeof(int) * c->n, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    bool any = false;
    for (int k = 0; k < c->n; ++k) {
        if (flags) flags[k] = h[k];
        any |= h[k] != 0;
    }
    if (any) {
        c->unstable = 1;
        return fail(LB_EUNSTABLE, "non-finite population or non-positive density");
    }
    return LB_OK;
}

lb_status lb_check(lb_ctx* c) {
    if (lb_status s = check_ctx(c)) return s;
    lb_status s = lb_batch_health(c, nullptr);
    if (s == LB_OK && c->unstable) return fail(LB_EUNSTABLE, "instability latched earlier");
    return s;
}

lb_status lb_moments(lb_ctx* c, double* rho, double* ux, double* uy, double* phi) {
    return lb_batch_moments(c, 0, rho, ux, uy, phi);
}

lb_status lb_batch_moments(lb_ctx* c, int cap, double* rho, double* ux, double* uy, double* phi) {
    if (lb_status s = check_ctx(c)) return s;
    if (lb_status s = cap_index(c, cap)) return s;
    return host_moments(c, cap, rho, ux, uy, phi);
}

lb_status lb_moments_device(lb_ctx* c, float* rho, float* ux, float* uy, float* phi) {
    if (lb_status s = check_ctx(c)) return s;
    return moments_into(c, 0, rho, ux, uy, phi);
}

lb_status lb_interface_length(lb_ctx* c, double* l, double* l_eff) {
    if (lb_status s = check_ctx(c)) return s;
    if (c->G[0].tube_len <= 0) return fail(LB_EINVAL, "no tube in this geometry");
    if (!c->active[0]) return fail(LB_ESTATE, "capillary is retired");
    if (lb_status s = launch_interface(c, 0)) return s;
    float h = 0.f;
    HIP_TRY(hipMemcpyAsync(&h, c->d_lnow, sizeof(float), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    if (!std::isfinite(h)) return fail(LB_EUNSTABLE, "non-finite interface position");
    if (l) *l = h;
    if (l_eff) *l_eff = h + 0.5 * c->G[0].tube_h;
    return LB_OK;
}

lb_status lb_meniscus_angle(lb_ctx* c, int cap, int edge_rows, double* theta_deg, double* radius, double* apex_x) {
    if (lb_status s = check_ctx(c)) return s;
    if (lb_status s = cap_index(c, cap)) return s;
    const lb_geometry& g = c->G[cap];
    if (g.tube_len <= 0) return fail(LB_EINVAL, "no tube in this geometry");
    const size_t n = (size_t)g.nx * g.ny;
    std::vector<double> rho(n), ux(n), uy(n), phi(n);
    if (lb_status s = host_moments(c, cap, rho.data(), ux.data(), uy.data(), phi.data())) return s;
    const double* q = c->model == LB_BINARY ? phi.data() : rho.data();
    return lb_meniscus_angle_field(q, &g, (double)c->L.caps[cap].q_mid, edge_rows, theta_deg, radius, apex_x);
}

lb_status lb_tube_flow(lb_ctx* c, int cap, int margin, double v_meniscus, double* u_centre, lb_tube_flow_stats* out) {
    if (lb_status s = check_ctx(c)) return s;
    if (lb_status s = cap_index(c, cap)) return s;
    const lb_geometry& g = c->G[cap];
    if (g.tube_len <= 0) return fail(LB_EINVAL, "no tube in this geometry");
    const size_t n = (size_t)g.nx * g.ny;
    std::vector<double> rho(n), ux(n), phi(n);
    if (lb_status s = host_moments(c, cap, rho.data(), ux.data(), nullptr, phi.data())) return s;
    const double* q = c->model == LB_BINARY ? phi.data() : rho.data();
    return lb_tube_flow_field(q, rho.data(), ux.data(), &g, (double)c->L.caps[cap].q_mid, margin, v_meniscus,
                              u_centre, out);
}

lb_status lb_batch_l_history(lb_ctx* c, int cap, double* l, long* steps, int max_samples, int* n_samples) {
    if (lb_status s = check_ctx(c)) return s;
    if (lb_status s = cap_index(c, cap)) return s;
    int n = 0;
    HIP_TRY(hipMemcpyAsync(&n, c->d_hist_n + cap, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    const int m = std::min(std::min(n, LB_HISTORY_CAP), std::max(max_samples, 0));
    if (m > 0) {
        std::vector<float> h(m);
        std::vector<long long> ht(m);
        HIP_TRY(hipMemcpyAsync(h.data(), c->d_hist + c->L.caps[cap].hist_off, sizeof(float) * m,
                               hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(hipMemcpyAsync(ht.data(), c->d_hist_t + c->L.caps[cap].hist_off, sizeof(long long) * m,
                               hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(hipStreamSynchronize(c->stream));
        for (int i = 0; i < m; ++i) {
            if (l) l[i] = h[i];
            if (steps) steps[i] = (long)ht[i];
        }
    }
    if (n_samples) *n_samples = n;
    return LB_OK;
}

lb_status lb_batch_retire(lb_ctx* c, int cap) {
    if (lb_status s = check_ctx(c)) return s;
    if (lb_status s = cap_index(c, cap)) return s;
    return set_active(c, cap, 0);
}

lb_status lb_batch_revive(lb_ctx* c, int cap) {
    if (lb_status s = check_ctx(c)) return s;
    if (lb_status s = cap_index(c, cap)) return s;
    return set_active(c, cap, 1);
}

lb_status lb_wall_gradient_for_angle(const lb_params* p, double theta_deg, double* grad) {
    if (!p || !grad) return fail(LB_EINVAL, "null argument");
    bool ok;
    if (p->model == LB_BINARY)
        ok = lbt::binary_wall_gradient(p->kappa, p->A, p->B, theta_deg, grad);
    else
        ok = lbt::vdw_wall_gradient(p->kappa, p->a, p->b, p->T, theta_deg, grad);
    if (!ok) return fail(LB_EINVAL, "no partial-wetting wall gradient for this angle and these constants");
    return LB_OK;
}

lb_status lb_set_wall_gradient(lb_ctx* c, int cap, double grad) {
    if (lb_status s = check_ctx(c)) return s;
    if (lb_status s = cap_index(c, cap)) return s;
    if (!std::isfinite(grad)) return fail(LB_EINVAL, "wall gradient must be finite");
    c->P[cap].wall_grad = grad;
    c->P[cap].theta_deg = std::nan("");
    c->L.caps[cap].G = (float)grad;
    HIP_TRY(hipMemcpyAsync(&c->d_caps[cap], &c->L.caps[cap], sizeof(CapDev), hipMemcpyHostToDevice, c->stream));
    // the host descriptor may change again before the stream reaches the copy
    HIP_TRY(hipStreamSynchronize(c->stream));
    return LB_OK;
}

lb_status lb_vdw_coexistence(const lb_params* p, double* rho_l, double* rho_g) {
    if (!p || !rho_l || !rho_g) return fail(LB_EINVAL, "null argument");
    if (!lbt::vdw_coexistence(p->a, p->b, p->T, rho_l, rho_g)) return fail(LB_EINVAL, "no coexistence (T >= Tc?)");
    return LB_OK;
}

struct CkptHeader {
    uint64_t magic;
    uint64_t hash;
    int64_t t;
    int32_t n, model;
    int64_t floats;
    int32_t mstore, pad;   // storage of the saved f planes
};

constexpr uint64_t CKPT_MAGIC = 0x4C42434150434B34ULL;   // phi in fixed point

static uint64_t setup_hash(const lb_ctx* c) {
    uint64_t h = fnv1a(c->P.data(), sizeof(lb_params) * c->P.size());
    return fnv1a(c->G.data(), sizeof(lb_geometry) * c->G.size(), h);
}

// Floats of capillary k's region in one arena (f planes, and phi).
static long long region_floats(const lb_ctx* c, int k) {
    return (c->model == LB_BINARY ? 10 : 9) * c->L.caps[k].plane;
}

size_t lb_checkpoint_bytes(const lb_ctx* c) {
    if (!c) return 0;
    size_t floats = 0;
    for (int k = 0; k < c->n; ++k)
        floats += (size_t)region_floats(c, k) + (c->model == LB_BINARY ? (size_t)c->L.caps[k].plane : 0);
    return sizeof(CkptHeader) + sizeof(int) * c->n + sizeof(float) * floats;
}

// Image: header, active flags, then per capillary its read-arena region
// (f*(t), phi(t+1)) followed, for the binary model, by phi(t).
lb_status lb_save(lb_ctx* c, void* host_buf, size_t bytes) {
    if (lb_status s = check_ctx(c)) return s;
    if (!host_buf || bytes < lb_checkpoint_bytes(c)) return fail(LB_EINVAL, "checkpoint buffer too small");
    CkptHeader h{CKPT_MAGIC, setup_hash(c), c->t, c->n, c->model, c->L.arena_floats, c->mstore, 0};
    char* p = (char*)host_buf;
    std::memcpy(p, &h, sizeof h);
    std::memcpy(p + sizeof h, c->active.data(), sizeof(int) * c->n);
    float* dst = (float*)(p + sizeof h + sizeof(int) * c->n);
    for (int k = 0; k < c->n; ++k) {
        const CapDev& d = c->L.caps[k];
        const int b = buf_of(c, k);
        const long long nf = region_floats(c, k);
        HIP_TRY(hipMemcpyAsync(dst, c->arena[b] + d.off_f, sizeof(float) * nf, hipMemcpyDeviceToHost, c->stream));
        dst += nf;
        if (c->model == LB_BINARY) {
            HIP_TRY(hipMemcpyAsync(dst, c->arena[b ^ 1] + d.off_phi, sizeof(float) * d.plane, hipMemcpyDeviceToHost,
                                   c->stream));
            dst += d.plane;
        }
    }
    HIP_TRY(hipStreamSynchronize(c->stream));
    return LB_OK;
}

lb_status lb_load(lb_ctx* c, const void* host_buf, size_t bytes) {
    if (lb_status s = check_ctx(c)) return s;
    if (!host_buf || bytes < lb_checkpoint_bytes(c)) return fail(LB_EINVAL, "checkpoint buffer too small");
    CkptHeader h;
    std::memcpy(&h, host_buf, sizeof h);
    if (h.magic != CKPT_MAGIC || h.hash != setup_hash(c) || h.n != c->n || h.floats != c->L.arena_floats ||
        (h.mstore != 0 && h.mstore != 1))
        return fail(LB_EINVAL, "checkpoint belongs to another setup");
    const char* p = (const char*)host_buf;
    std::vector<int> act(c->n);
    std::memcpy(act.data(), p + sizeof h, sizeof(int) * c->n);
    const float* src = (const float*)(p + sizeof h + sizeof(int) * c->n);
    // every capillary reads arena cur after the load
    for (int k = 0; k < c->n; ++k) {
        CapDev& d = c->L.caps[k];
        const long long nf = region_floats(c, k);
        HIP_TRY(hipMemcpyAsync(c->arena[c->cur] + d.off_f, src, sizeof(float) * nf, hipMemcpyHostToDevice,
                               c->stream));
        src += nf;
        if (c->model == LB_BINARY) {
            HIP_TRY(hipMemcpyAsync(c->arena[c->cur ^ 1] + d.off_phi, src, sizeof(float) * d.plane,
                                   hipMemcpyHostToDevice, c->stream));
            src += d.plane;
        }
        c->active[k] = act[k] ? 1 : 0;
        c->frozen_buf[k] = c->cur;
        d.par = 0;
        d.active = c->active[k];
    }
    // an image of the other storage is converted to the context's
    if (h.mstore != c->mstore)
        if (lb_status s = convert_arena(c, c->cur, c->mstore)) return s;
    HIP_TRY(hipStreamSynchronize(c->stream));
    HIP_TRY(hipMemcpyAsync(c->d_caps, c->L.caps.data(), sizeof(CapDev) * c->n, hipMemcpyHostToDevice, c->stream));
    c->t = (long)h.t;
    c->unstable = 0;
    return upload_tiles(c);
}

lb_status lb_get_launch_config(const lb_ctx* c, lb_launch_config* cfg) {
    if (!c || !cfg) return fail(LB_EINVAL, "null argument");
    *cfg = c->cfg;
    return LB_OK;
}

lb_status lb_set_launch_config(lb_ctx* c, const lb_launch_config* cfg) {
    if (!c || !cfg) return fail(LB_EINVAL, "null argument");
    const int r = cfg->tile_rows;
    if (r != 1 && r != 2 && r != 4 && r != 8) return fail(LB_EINVAL, "tile_rows must be 1, 2, 4 or 8");
    if (cfg->schedule < 0 || cfg->schedule > 6) return fail(LB_EINVAL, "schedule must be 0, 1, 2, 3, 4, 5 or 6");
    if (cfg->schedule == 6 && c->model != LB_BINARY)
        return fail(LB_EINVAL, "schedule 6 (moment storage) is built for the binary model only");
    if (cfg->schedule == 2 && (cfg->persist_blocks_per_cu < 1 || cfg->persist_blocks_per_cu > 32))
        return fail(LB_EINVAL, "persistent workgroups per CU must be in 1..32");
    if (cfg->graph_steps != 0 && (cfg->graph_steps < 2 || cfg->graph_steps % 2 != 0 || cfg->graph_steps > 4096))
        return fail(LB_EINVAL, "graph_steps must be 0 or an even number in 2..4096");
    if (cfg->fp64_arith != 0 && cfg->fp64_arith != 1) return fail(LB_EINVAL, "fp64_arith must be 0 or 1");
    const int ch = cfg->chunk_rows;
    if (ch != 0 && (ch < LB_MIN_CHUNK || ch > 4096))
        return fail(LB_EINVAL, "chunk_rows must be 0 or in 4..4096");
    const bool retile = r != c->cfg.tile_rows || cfg->chunk_rows != c->cfg.chunk_rows ||
                        strip_width(*cfg) != strip_width(c->cfg);
    c->cfg = *cfg;
    drop_graphs(c);
    if (lb_status s = set_storage(c, cfg->schedule == 6 ? 1 : 0)) return s;
    if (retile) return upload_tiles(c);
    return LB_OK;
}

lb_status lb_use_tuned_launch_config(lb_ctx* c, int* found) {
    if (lb_status s = check_ctx(c)) return s;
    if (found) *found = 0;
    lb_launch_config cf = c->cfg;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_cache.find({c->model, size_class(c->L.fluid)});
        if (it == g_tune_cache.end()) return LB_OK;
        // the shape only: the arithmetic stays the context's own choice
        cf.tile_rows = it->second.tile_rows;
        cf.schedule = it->second.schedule;
        cf.persist_blocks_per_cu = it->second.persist_blocks_per_cu;
        cf.graph_steps = it->second.graph_steps;
        cf.chunk_rows = it->second.chunk_rows;
    }
    if (lb_status s = lb_set_launch_config(c, &cf)) return s;
    if (found) *found = 1;
    return LB_OK;
}

lb_status lb_autotune(lb_ctx* c, int trial_steps, lb_launch_config* best, double* us_per_step) {
    if (lb_status s = check_ctx(c)) return s;
    if (trial_steps < 2) return fail(LB_EINVAL, "trial_steps must be >= 2");
    // back up both arenas: the trials advance the lattices
    const size_t ab = sizeof(float) * (size_t)c->L.arena_floats;
    float* raw = nullptr;
    if (hipMalloc(&raw, 2 * ab) != hipSuccess) return fail(LB_ENOMEM, "no device memory for the autotune backup");
    struct Backup {
        float* p;
        ~Backup() { (void)hipFree(p); }
    } backup{raw};
    HIP_TRY(hipMemcpyAsync(backup.p, c->arena[0], ab, hipMemcpyDeviceToDevice, c->stream));
    HIP_TRY(hipMemcpyAsync((char*)backup.p + ab, c->arena[1], ab, hipMemcpyDeviceToDevice, c->stream));
    const long t0 = c->t;
    const int cur0 = c->cur;
    const int mstore0 = c->mstore;
    const lb_launch_config orig = c->cfg;
    std::vector<lb_launch_config> cand;
    const int ar = orig.fp64_arith;   // the arithmetic is a choice of the caller, not tuned
    for (int ch : {6, 8, 12, 16, 32}) cand.push_back({orig.tile_rows, 3, 4, 0, ar, ch});
    for (int ch : {8, 12, 16, 32}) cand.push_back({orig.tile_rows, 4, 4, 0, ar, ch});
    for (int ch : {8, 12, 16, 24, 32}) cand.push_back({orig.tile_rows, 5, 4, 0, ar, ch});
    if (c->model == LB_BINARY)
        for (int ch : {16, 20, 24, 32}) cand.push_back({orig.tile_rows, 6, 4, 0, ar, ch});
    for (int r : {4, 8}) {
        cand.push_back({r, 1, 4, 0, ar, orig.chunk_rows});
        cand.push_back({r, 2, 4, 0, ar, orig.chunk_rows});
    }
    double best_us = 1e300;
    lb_launch_config best_cfg = orig;
    lb_status st = LB_OK;
    auto hip_ok = [&](hipError_t e, const char* what) {
        if (e == hipSuccess) return true;
        st = fail(LB_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
        return false;
    };
    for (const auto& cf0 : cand) {
        lb_launch_config cf = cf0;
        if ((st = lb_set_launch_config(c, &cf))) break;
        // (the state is restored afterwards: no read-out needs the last step single)
        if ((st = run_steps(c, 2, false))) break;  // warm-up
        if (!hip_ok(hipEventRecord(c->ev0, c->stream), "hipEventRecord")) break;
        if ((st = run_steps(c, trial_steps, false))) break;
        float ms = 0.f;
        if (!hip_ok(hipEventRecord(c->ev1, c->stream), "hipEventRecord") ||
            !hip_ok(hipEventSynchronize(c->ev1), "hipEventSynchronize") ||
            !hip_ok(hipEventElapsedTime(&ms, c->ev0, c->ev1), "hipEventElapsedTime"))
            break;
        const double us = 1000.0 * ms / trial_steps;
        if (us < best_us) {
            best_us = us;
            best_cfg = cf;
        }
    }
    // graphs reduce launch gaps: keep them for the winner
    best_cfg.graph_steps = 64;
    // restore the state and time, also after a failed trial
    HIP_TRY(hipMemcpyAsync(c->arena[0], backup.p, ab, hipMemcpyDeviceToDevice, c->stream));
    HIP_TRY(hipMemcpyAsync(c->arena[1], (char*)backup.p + ab, ab, hipMemcpyDeviceToDevice, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    c->cur = cur0;
    c->t = t0;
    // the backup holds the storage of the start; the final setting converts it if needed
    if (lb_status s2 = mark_storage(c, mstore0)) return s2;
    if (st) {
        const std::string msg = g_err;
        lb_set_launch_config(c, &orig);
        g_err = msg;
        return st;
    }
    if ((st = lb_set_launch_config(c, &best_cfg))) return st;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune_cache[{c->model, size_class(c->L.fluid)}] = best_cfg;
    }
    if (best) *best = best_cfg;
    if (us_per_step) *us_per_step = best_us;
    c->timed_steps = 0;
    return LB_OK;
}

void lb_free(lb_ctx* c) {
    if (!c) return;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    drop_graphs(c);
    if (c->ev0) (void)hipEventDestroy(c->ev0);
    if (c->ev1) (void)hipEventDestroy(c->ev1);
    if (c->own_mem && c->mem) (void)hipFree(c->mem);
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

}  // extern "C"
