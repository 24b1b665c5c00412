/*
 * Oracle for the free-energy MRT lattice Boltzmann scheme of Pooley,
 * Kusumaatmaja & Yeomans (arXiv:0911.0459), FP64, plain CPU loops.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test suite, the smoke check and the
 * benchmark's CPU-baseline leg; never by the product path.  It shares no code
 * with the GPU library.  Every step is written the slow, literal way:
 * the equilibria are formed population by population, the collision is the
 * 9x9 matrix product M^-1 S M (f - f^eq) of Eq. (latbolt), M^-1 is obtained by
 * Gauss-Jordan elimination of the Appendix A matrix, and streaming, bounce-back
 * and the rest step are separate sweeps over the lattice.
 *
 * Readings of points the paper leaves open (each also used by the GPU library,
 * which implements them independently):
 *  - lattice units dx = dt = c = 1;
 *  - e5 = (1,1), e6 = (-1,-1), e7 = (-1,1), e8 = (1,-1), which makes the jx and jy
 *    rows of the Appendix A matrix the momentum components;
 *  - lambda (Eq. equilibrium, value not given): for vdW the Chapman-Enskog
 *    values that restore Galilean invariance under the Appendix A rates, one
 *    for the traceless part of the bracket, (1/omega - 1/2)(1/3 - dp0/drho),
 *    and one for its isotropic part, (1/2)(1/3 - dp0/drho) (equal to each other
 *    at omega = 1, the printed single-lambda form); binary 0.  lambda_mode = 1
 *    switches it off.  Pinned by the Galilean invariance of a translating
 *    interface (see orc_feq), which only a moving state tests;
 *  - binary f^eq: the Eq. (equilibrium) form with X = p0 - kappa phi lap(phi) and the
 *    kappa terms in the gradients of phi, so that its second moment is the binary
 *    pressure tensor of Sec. 3.1 plus rho u u;
 *  - nu(phi) of Eq. (nu) uses phi clamped to [-1, 1];
 *  - "setting boundary nodes to rest" (Sec. 2.2): after streaming, every fluid node
 *    with a solid node among its 8 neighbours loses its momentum,
 *    f_i <- f_i - w_i e_i.j, which keeps rho and the even moments;
 *  - wetting (Sec. 2.2): the wall gradient enters the stencils through ghost values
 *    for solid neighbours (rule W, see ghost_source below), in the equilibrium only;
 *  - body force: Guo, Zheng & Shi, Phys. Rev. E 65, 046308 (2002), transformed by
 *    M^-1 (I - S/2) M, u = (j + F/2)/rho, applied on non-boundary fluid nodes only.
 */
#include "lb_oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

static __thread char g_err[512];

static void set_err(const char* msg) {
    snprintf(g_err, sizeof g_err, "%s", msg);
}

const char* orc_error(void) { return g_err; }

#ifdef _OPENMP
#include <omp.h>
int orc_threads(void) { return omp_get_max_threads(); }
#else
int orc_threads(void) { return 1; }
#endif

/* ---- D2Q9 velocity set (Sec. 2.1) ------------------------------------------ */
static const int EX[9] = {0, 1, -1, 0, 0, 1, -1, -1, 1};
static const int EY[9] = {0, 0, 0, 1, -1, 1, -1, 1, -1};
static const int OPP[9] = {0, 2, 1, 4, 3, 6, 5, 8, 7};

/* ---- weights of Eq. (equilibrium), Appendix A ------------------------------ */
static const double W[9] = {0.0, 1.0 / 3, 1.0 / 3, 1.0 / 3, 1.0 / 3,
                            1.0 / 12, 1.0 / 12, 1.0 / 12, 1.0 / 12};
static const double WXX[9] = {0.0, 1.0 / 3, 1.0 / 3, -1.0 / 6, -1.0 / 6,
                              -1.0 / 24, -1.0 / 24, -1.0 / 24, -1.0 / 24};
static const double WYY[9] = {0.0, -1.0 / 6, -1.0 / 6, 1.0 / 3, 1.0 / 3,
                              -1.0 / 24, -1.0 / 24, -1.0 / 24, -1.0 / 24};
static const double WXY[9] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.25, 0.25, -0.25, -0.25};

/* Standard D2Q9 lattice weights (c_s^2 = 1/3) used by Guo's forcing term only. */
static const double WGUO[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                               1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};

/* ---- change-of-basis matrix M, Appendix A ---------------------------------- */
static const double MM[9][9] = {
    {1, 1, 1, 1, 1, 1, 1, 1, 1},
    {-4, -1, -1, -1, -1, 2, 2, 2, 2},
    {4, -2, -2, -2, -2, 1, 1, 1, 1},
    {0, 1, -1, 0, 0, 1, -1, -1, 1},
    {0, -2, 2, 0, 0, 1, -1, -1, 1},
    {0, 0, 0, 1, -1, 1, -1, 1, -1},
    {0, 0, 0, -2, 2, 1, -1, 1, -1},
    {0, 1, 1, -1, -1, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 1, 1, -1, -1},
};

static double MINV[9][9];
static int minv_ready = 0;

/* Gauss-Jordan elimination with partial pivoting of the 9x9 matrix M. */
static void build_minv(void) {
    double a[9][18];
    for (int r = 0; r < 9; ++r) {
        for (int c = 0; c < 9; ++c) a[r][c] = MM[r][c];
        for (int c = 0; c < 9; ++c) a[r][9 + c] = (r == c) ? 1.0 : 0.0;
    }
    for (int col = 0; col < 9; ++col) {
        int piv = col;
        for (int r = col + 1; r < 9; ++r)
            if (fabs(a[r][col]) > fabs(a[piv][col])) piv = r;
        if (piv != col)
            for (int c = 0; c < 18; ++c) {
                double t = a[col][c];
                a[col][c] = a[piv][c];
                a[piv][c] = t;
            }
        double d = a[col][col];
        for (int c = 0; c < 18; ++c) a[col][c] /= d;
        for (int r = 0; r < 9; ++r) {
            if (r == col) continue;
            double m = a[r][col];
            if (m == 0.0) continue;
            for (int c = 0; c < 18; ++c) a[r][c] -= m * a[col][c];
        }
    }
    for (int r = 0; r < 9; ++r)
        for (int c = 0; c < 9; ++c) MINV[r][c] = a[r][9 + c];
    minv_ready = 1;
}

static void ensure_minv(void) {
#pragma omp critical(orc_minv)
    {
        if (!minv_ready) build_minv();
    }
}

void orc_matrix_M(double* out) {
    for (int r = 0; r < 9; ++r)
        for (int c = 0; c < 9; ++c) out[9 * r + c] = MM[r][c];
}

void orc_matrix_Minv(double* out) {
    ensure_minv();
    for (int r = 0; r < 9; ++r)
        for (int c = 0; c < 9; ++c) out[9 * r + c] = MINV[r][c];
}

/* ---- geometry (Sec. 2.2, Fig. 1b) -------------------------------------------
 * A tube of tube_h fluid rows [y0, y0+tube_h) between solid blocks occupies the
 * columns [x_in, x_in+tube_len); every other node is fluid (reservoir). */
static int wrapi(int v, int n) {
    v %= n;
    return v < 0 ? v + n : v;
}

static int is_solid_xy(const orc_geom* g, int x, int y) {
    x = wrapi(x, g->nx);
    y = wrapi(y, g->ny);
    if (g->tube_len <= 0) return 0;
    if (x < g->x_in || x >= g->x_in + g->tube_len) return 0;
    return (y < g->y0 || y >= g->y0 + g->tube_h);
}

void orc_solid_mask(const orc_geom* g, unsigned char* mask) {
    for (int y = 0; y < g->ny; ++y)
        for (int x = 0; x < g->nx; ++x) mask[y * g->nx + x] = (unsigned char)is_solid_xy(g, x, y);
}

/* Rule W: value standing in for q at a solid neighbour r+d of fluid node r.
 * Axis d: mirror through r, q(r-d).  Diagonal d: if the x-neighbour r+(dx,0) is
 * solid mirror across that wall, q(r+(-dx,dy)); else if r+(0,dy) is solid mirror
 * across that wall, q(r+(dx,-dy)); else (convex corner) q(r-d).  The ghost is
 * that value minus 2G, so that the paper's gradient stencil at a node next to a
 * flat wall returns exactly G along the inward normal.  Returns the source node
 * (x, y) through sx, sy. */
static void ghost_source(const orc_geom* g, int x, int y, int dx, int dy, int* sx, int* sy) {
    if (dx == 0 || dy == 0) {
        *sx = x - dx;
        *sy = y - dy;
    } else if (is_solid_xy(g, x + dx, y)) {
        *sx = x - dx;
        *sy = y + dy;
    } else if (is_solid_xy(g, x, y + dy)) {
        *sx = x + dx;
        *sy = y - dy;
    } else {
        *sx = x - dx;
        *sy = y - dy;
    }
}

static int check_geometry(const orc_geom* g) {
    if (g->nx < 3 || g->ny < 3) {
        set_err("lattice must be at least 3x3");
        return ORC_EINVAL;
    }
    if (g->tube_len < 0) {
        set_err("negative tube length");
        return ORC_EINVAL;
    }
    if (g->tube_len > 0) {
        if (g->x_in < 0 || g->x_in + g->tube_len > g->nx) {
            set_err("tube does not fit in the lattice along x");
            return ORC_EINVAL;
        }
        if (g->tube_h < 3 || g->y0 < 1 || g->y0 + g->tube_h > g->ny - 1) {
            set_err("tube rows must satisfy H >= 3, y0 >= 1, y0 + H <= ny - 1");
            return ORC_EINVAL;
        }
    }
    /* every ghost source used by rule W must be a fluid node */
    for (int y = 0; y < g->ny; ++y)
        for (int x = 0; x < g->nx; ++x) {
            if (is_solid_xy(g, x, y)) continue;
            for (int i = 1; i < 9; ++i) {
                if (!is_solid_xy(g, x + EX[i], y + EY[i])) continue;
                int sx, sy;
                ghost_source(g, x, y, EX[i], EY[i], &sx, &sy);
                if (is_solid_xy(g, sx, sy)) {
                    set_err("wall ghost source is solid (geometry too thin)");
                    return ORC_EINVAL;
                }
            }
        }
    return ORC_OK;
}

/* ---- finite-difference stencils, Eq. (best) ---------------------------------- */
static double neighbour_value(const orc_geom* g, const double* q, double G, int x, int y, int dx,
                              int dy) {
    int nx = g->nx, ny = g->ny;
    if (!is_solid_xy(g, x + dx, y + dy)) return q[wrapi(y + dy, ny) * nx + wrapi(x + dx, nx)];
    int sx, sy;
    ghost_source(g, x, y, dx, dy, &sx, &sy);
    return q[wrapi(sy, ny) * nx + wrapi(sx, nx)] - 2.0 * G;
}

static void stencils_at(const orc_geom* g, const double* q, double G, int x, int y, double* dxq,
                        double* dyq, double* lapq) {
    double qc = q[y * g->nx + x];
    double e = neighbour_value(g, q, G, x, y, 1, 0);
    double w = neighbour_value(g, q, G, x, y, -1, 0);
    double n = neighbour_value(g, q, G, x, y, 0, 1);
    double s = neighbour_value(g, q, G, x, y, 0, -1);
    double ne = neighbour_value(g, q, G, x, y, 1, 1);
    double nw = neighbour_value(g, q, G, x, y, -1, 1);
    double se = neighbour_value(g, q, G, x, y, 1, -1);
    double sw = neighbour_value(g, q, G, x, y, -1, -1);
    /* d/dx = (1/12) [-1 0 1; -4 0 4; -1 0 1],  d/dy its transpose */
    *dxq = (ne + 4.0 * e + se - nw - 4.0 * w - sw) / 12.0;
    *dyq = (ne + 4.0 * n + nw - se - 4.0 * s - sw) / 12.0;
    /* lap = (1/6) [1 4 1; 4 -20 4; 1 4 1] */
    *lapq = (ne + nw + se + sw + 4.0 * (e + w + n + s) - 20.0 * qc) / 6.0;
}

int orc_gradients(const orc_geom* g, double wall_grad, const double* q, double* dxq,
                  double* dyq, double* lapq) {
    int rc = check_geometry(g);
    if (rc) return rc;
    for (int y = 0; y < g->ny; ++y)
        for (int x = 0; x < g->nx; ++x) {
            int k = y * g->nx + x;
            if (is_solid_xy(g, x, y)) {
                dxq[k] = dyq[k] = lapq[k] = 0.0;
                continue;
            }
            stencils_at(g, q, wall_grad, x, y, &dxq[k], &dyq[k], &lapq[k]);
        }
    return ORC_OK;
}

/* ---- equilibria, Appendix A ------------------------------------------------- */
/* f^eq of Eq. (equilibrium) for i = 1..8 and Eq. (feq0) for i = 0.  X is the
 * isotropic part p0 - kappa q lap q.  The Galilean correction
 * lambda [u_a d_b q + u_b d_a q + delta_ab u.grad q] of Q is split into its
 * traceless part [u_a d_b q + u_b d_a q - delta_ab u.grad q] and its isotropic
 * part 2 delta_ab u.grad q, with coefficients lam_s and lam_b; the paper's form
 * is lam_s = lam_b = lambda. */
static void feq_general(double rho, double ux, double uy, double X, double lam_s, double lam_b,
                        double kappa, double dxq, double dyq, double* feq) {
    double Q[2][2];
    double udq = ux * dxq + uy * dyq;
    double u[2] = {ux, uy}, dq[2] = {dxq, dyq};
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            Q[a][b] = rho * u[a] * u[b] + lam_s * (u[a] * dq[b] + u[b] * dq[a] - (a == b ? udq : 0.0)) +
                      lam_b * (a == b ? 2.0 * udq : 0.0);
    double sum = 0.0;
    for (int i = 1; i < 9; ++i) {
        double e[2] = {(double)EX[i], (double)EY[i]};
        double eu = e[0] * ux + e[1] * uy;
        double quad = 0.0;
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) quad += (e[a] * e[b] - (a == b ? 1.0 / 3.0 : 0.0)) * Q[a][b];
        feq[i] = W[i] * (X + rho * eu + 1.5 * quad) +
                 kappa * (WXX[i] * dxq * dxq + WYY[i] * dyq * dyq + WXY[i] * dxq * dyq);
        sum += feq[i];
    }
    feq[0] = rho - sum;
}

/* lambda of the Galilean term (van der Waals model).  Chapman-Enskog: with a
 * non-ideal p0 the first-order momentum flux keeps the term
 *   -(tau - 1/2)(1/3 - dp0/drho)[u_a d_b rho + u_b d_a rho + delta_ab u.grad rho],
 * tau being the relaxation time of the moments that carry it.  With the rates
 * of Appendix A, S = diag(0,1,1,0,1,0,1,omega,omega), the traceless part of the
 * second moment relaxes at omega (tau = 1/omega) and its trace, the energy
 * moment e, at 1 (tau = 1).  A single lambda can cancel both parts only when
 * omega = 1, so the bracket is split (see feq_general) and each part gets the
 * coefficient of its own moment:
 *   lam_s = (1/omega - 1/2)(1/3 - dp0/drho)   traceless part,
 *   lam_b = (1 - 1/2)(1/3 - dp0/drho)          isotropic part;
 * at omega = 1 this is the single-lambda form written in Eq. (equilibrium).
 * lambda_mode 0 takes these values and 1 sets both to 0 (both modes also in
 * the GPU library).  Two more modes exist only to test the reading on the CPU:
 * 2 flips both signs (a planted mistake) and 3 is the single-lambda form with
 * the stress rate, lam_s = lam_b = (1/omega - 1/2)(1/3 - dp0/drho). */
void orc_feq(const orc_params* p, double rho, double ux, double uy, double omega, double X,
             double dxq, double dyq, double* feq) {
    double lam_s = 0.0, lam_b = 0.0;
    if (p->model == ORC_VDW && p->lambda_mode != 1) {
        double dp0 = p->T / ((1.0 - p->b * rho) * (1.0 - p->b * rho)) - 2.0 * p->a * rho;
        lam_s = (1.0 / omega - 0.5) * (1.0 / 3.0 - dp0);
        lam_b = (1.0 - 0.5) * (1.0 / 3.0 - dp0);
        if (p->lambda_mode == 2) {
            lam_s = -lam_s;
            lam_b = -lam_b;
        }
        if (p->lambda_mode == 3) lam_b = lam_s;
    }
    feq_general(rho, ux, uy, X, lam_s, lam_b, p->kappa, dxq, dyq, feq);
}

/* g^eq of Appendix A with Gamma = 2M/dt. */
void orc_geq(const orc_params* p, double phi, double ux, double uy, double mu, double* geq) {
    double sum = 0.0;
    for (int i = 1; i < 9; ++i) {
        double e[2] = {(double)EX[i], (double)EY[i]};
        double u[2] = {ux, uy};
        double eu = e[0] * ux + e[1] * uy;
        double quad = 0.0;
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b)
                quad += (e[a] * e[b] - (a == b ? 1.0 / 3.0 : 0.0)) * phi * u[a] * u[b];
        geq[i] = W[i] * (p->Gamma * mu + phi * eu + 1.5 * quad);
        sum += geq[i];
    }
    geq[0] = phi - sum;
}

/* ---- collision, Eq. (latbolt) with Appendix A's M and S -------------------- */
void orc_collide(const orc_params* p, const double* f, const double* feq, double omega, double ux,
                 double uy, double Fx, double Fy, double* fstar) {
    (void)p;
    ensure_minv();
    double S[9] = {0, 1, 1, 0, 1, 0, 1, omega, omega};
    double d[9], m[9], back[9];
    for (int i = 0; i < 9; ++i) d[i] = f[i] - feq[i];
    for (int k = 0; k < 9; ++k) {
        m[k] = 0.0;
        for (int i = 0; i < 9; ++i) m[k] += MM[k][i] * d[i];
        m[k] *= S[k];
    }
    for (int i = 0; i < 9; ++i) {
        back[i] = 0.0;
        for (int k = 0; k < 9; ++k) back[i] += MINV[i][k] * m[k];
        fstar[i] = f[i] - back[i];
    }
    if (Fx != 0.0 || Fy != 0.0) {
        /* Guo forcing term F_i = t_i [3 (e_i - u) + 9 (e_i.u) e_i] . F, applied as
         * M^-1 (I - S/2) M F. */
        double Fb[9], mF[9];
        for (int i = 0; i < 9; ++i) {
            double eu = EX[i] * ux + EY[i] * uy;
            Fb[i] = WGUO[i] * ((3.0 * (EX[i] - ux) + 9.0 * eu * EX[i]) * Fx +
                               (3.0 * (EY[i] - uy) + 9.0 * eu * EY[i]) * Fy);
        }
        for (int k = 0; k < 9; ++k) {
            mF[k] = 0.0;
            for (int i = 0; i < 9; ++i) mF[k] += MM[k][i] * Fb[i];
            mF[k] *= (1.0 - 0.5 * S[k]);
        }
        for (int i = 0; i < 9; ++i) {
            double acc = 0.0;
            for (int k = 0; k < 9; ++k) acc += MINV[i][k] * mF[k];
            fstar[i] += acc;
        }
    }
}

/* ---- state ------------------------------------------------------------------ */
struct orc_state {
    orc_params p;
    orc_geom g;
    int n;
    unsigned char* solid;
    unsigned char* boundary;
    double* f[9];
    double* gp[9];
    double* fs[9];
    double* gs[9];
    double *rho, *ux, *uy, *phi, *q, *dxq, *dyq, *lapq;
    long t;
};

static double* dalloc(int n) { return (double*)calloc((size_t)n, sizeof(double)); }

void orc_free(orc_state* s) {
    if (!s) return;
    for (int i = 0; i < 9; ++i) {
        free(s->f[i]);
        free(s->gp[i]);
        free(s->fs[i]);
        free(s->gs[i]);
    }
    free(s->solid);
    free(s->boundary);
    free(s->rho);
    free(s->ux);
    free(s->uy);
    free(s->phi);
    free(s->q);
    free(s->dxq);
    free(s->dyq);
    free(s->lapq);
    free(s);
}

static double viscosity(const orc_params* p, double phi) {
    if (p->model == ORC_VDW) return p->nu_l;
    /* Eq. (nu) with phi clamped to [-1, 1] */
    double c = phi < -1.0 ? -1.0 : (phi > 1.0 ? 1.0 : phi);
    return p->nu_g + 0.5 * (c + 1.0) * (p->nu_l - p->nu_g);
}

static double omega_of_nu(double nu) { return 2.0 / (6.0 * nu + 1.0); }

/* Bulk pressure p0: van der Waals (Sec. 2) or phi^4 (Sec. 3.1). */
static double bulk_pressure(const orc_params* p, double rho, double phi) {
    if (p->model == ORC_VDW) return rho * p->T / (1.0 - p->b * rho) - p->a * rho * rho;
    return rho / 3.0 - 0.5 * p->A * phi * phi + 0.75 * p->B * phi * phi * phi * phi;
}

/* Equilibria of one node from its moments and stencils. */
static void node_equilibria(const orc_state* s, int k, double* feq, double* geq) {
    const orc_params* p = &s->p;
    double rho = s->rho[k], ux = s->ux[k], uy = s->uy[k], phi = s->phi[k];
    double qv = s->q[k];
    double omega = omega_of_nu(viscosity(p, phi));
    double X = bulk_pressure(p, rho, phi) - p->kappa * qv * s->lapq[k];
    orc_feq(p, rho, ux, uy, omega, X, s->dxq[k], s->dyq[k], feq);
    if (p->model == ORC_BINARY) {
        double mu = -p->A * phi + p->B * phi * phi * phi - p->kappa * s->lapq[k];
        orc_geq(p, phi, ux, uy, mu, geq);
    }
}

static int check_params(const orc_params* p) {
    if (p->model != ORC_VDW && p->model != ORC_BINARY) {
        set_err("unknown model");
        return ORC_EINVAL;
    }
    if (!(p->nu_l > 0.0) || (p->model == ORC_BINARY && !(p->nu_g > 0.0))) {
        set_err("viscosities must be positive (0 < omega < 2)");
        return ORC_EINVAL;
    }
    if (!(p->kappa >= 0.0) || !isfinite(p->wall_grad) || !isfinite(p->force_x)) {
        set_err("kappa must be >= 0 and wall gradient / force finite");
        return ORC_EINVAL;
    }
    if (p->model == ORC_BINARY && !(p->Gamma >= 0.0)) {
        set_err("mobility coefficient must be >= 0");
        return ORC_EINVAL;
    }
    if (p->model == ORC_VDW && !(p->b > 0.0 && p->T > 0.0)) {
        set_err("vdW needs b > 0 and T > 0");
        return ORC_EINVAL;
    }
    return ORC_OK;
}

/* S1: moments of the current populations.  u = (j + F/2)/rho on non-boundary
 * nodes (Guo), j/rho on boundary nodes where no force acts. */
static void compute_moments(orc_state* s) {
    int nx = s->g.nx, ny = s->g.ny;
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            int k = y * nx + x;
            if (s->solid[k]) {
                s->rho[k] = s->ux[k] = s->uy[k] = s->phi[k] = s->q[k] = 0.0;
                continue;
            }
            double rho = 0.0, jx = 0.0, jy = 0.0, phi = 0.0;
            for (int i = 0; i < 9; ++i) {
                rho += s->f[i][k];
                jx += EX[i] * s->f[i][k];
                jy += EY[i] * s->f[i][k];
            }
            if (s->p.model == ORC_BINARY)
                for (int i = 0; i < 9; ++i) phi += s->gp[i][k];
            double Fx = s->boundary[k] ? 0.0 : s->p.force_x;
            s->rho[k] = rho;
            s->ux[k] = (jx + 0.5 * Fx) / rho;
            s->uy[k] = jy / rho;
            s->phi[k] = phi;
            s->q[k] = (s->p.model == ORC_VDW) ? rho : phi;
        }
}

/* S2: stencils of q with the wall ghosts. */
static void compute_stencils(orc_state* s) {
    int nx = s->g.nx, ny = s->g.ny;
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            int k = y * nx + x;
            if (s->solid[k]) continue;
            stencils_at(&s->g, s->q, s->p.wall_grad, x, y, &s->dxq[k], &s->dyq[k], &s->lapq[k]);
        }
}

int orc_create(const orc_params* p, const orc_geom* g, const double* init_q, orc_state** out) {
    return orc_create_flow(p, g, init_q, NULL, NULL, out);
}

int orc_create_flow(const orc_params* p, const orc_geom* g, const double* init_q, const double* init_ux,
                    const double* init_uy, orc_state** out) {
    *out = NULL;
    int rc = check_params(p);
    if (rc) return rc;
    rc = check_geometry(g);
    if (rc) return rc;
    int n = g->nx * g->ny;
    for (int y = 0; y < g->ny; ++y)
        for (int x = 0; x < g->nx; ++x) {
            if (is_solid_xy(g, x, y)) continue;
            double v = init_q[y * g->nx + x];
            if (!isfinite(v) || (init_ux && !isfinite(init_ux[y * g->nx + x])) ||
                (init_uy && !isfinite(init_uy[y * g->nx + x]))) {
                set_err("non-finite initial field");
                return ORC_EINVAL;
            }
            if (p->model == ORC_VDW && !(v > 0.0 && p->b * v < 1.0)) {
                set_err("vdW initial density must satisfy 0 < rho < 1/b");
                return ORC_EINVAL;
            }
        }
    ensure_minv();
    orc_state* s = (orc_state*)calloc(1, sizeof(orc_state));
    s->p = *p;
    s->g = *g;
    s->n = n;
    s->solid = (unsigned char*)calloc((size_t)n, 1);
    s->boundary = (unsigned char*)calloc((size_t)n, 1);
    for (int i = 0; i < 9; ++i) {
        s->f[i] = dalloc(n);
        s->gp[i] = dalloc(n);
        s->fs[i] = dalloc(n);
        s->gs[i] = dalloc(n);
    }
    s->rho = dalloc(n);
    s->ux = dalloc(n);
    s->uy = dalloc(n);
    s->phi = dalloc(n);
    s->q = dalloc(n);
    s->dxq = dalloc(n);
    s->dyq = dalloc(n);
    s->lapq = dalloc(n);
    orc_solid_mask(g, s->solid);
    for (int y = 0; y < g->ny; ++y)
        for (int x = 0; x < g->nx; ++x) {
            int k = y * g->nx + x;
            if (s->solid[k]) continue;
            for (int i = 1; i < 9; ++i)
                if (is_solid_xy(g, x + EX[i], y + EY[i])) s->boundary[k] = 1;
        }
    /* Initial state: u = 0, f = f^eq, g = g^eq of the initial field. */
    for (int k = 0; k < n; ++k) {
        if (s->solid[k]) continue;
        if (p->model == ORC_VDW) {
            s->rho[k] = init_q[k];
            s->phi[k] = 0.0;
            s->q[k] = init_q[k];
        } else {
            s->rho[k] = 1.0;
            s->phi[k] = init_q[k];
            s->q[k] = init_q[k];
        }
        s->ux[k] = init_ux ? init_ux[k] : 0.0;
        s->uy[k] = init_uy ? init_uy[k] : 0.0;
    }
    compute_stencils(s);
    for (int k = 0; k < n; ++k) {
        if (s->solid[k]) continue;
        double feq[9], geq[9];
        node_equilibria(s, k, feq, geq);
        for (int i = 0; i < 9; ++i) {
            s->f[i][k] = feq[i];
            s->gp[i][k] = (p->model == ORC_BINARY) ? geq[i] : 0.0;
        }
    }
    s->t = 0;
    *out = s;
    return ORC_OK;
}

long orc_time(const orc_state* s) { return s->t; }

int orc_set_wall_gradient(orc_state* s, double wall_grad) {
    if (!isfinite(wall_grad)) {
        set_err("wall gradient must be finite");
        return ORC_EINVAL;
    }
    s->p.wall_grad = wall_grad;
    return ORC_OK;
}

/* One time step in the order of Eq. (latbolt) / (latbolt2) followed by the
 * wall treatment of Sec. 2.2:
 *   S1 moments, S2 stencils, S3 thermodynamics, S4 equilibria, S5 collision,
 *   S6 streaming with bounce-back, S7 rest at boundary nodes. */
static void one_step(orc_state* s) {
    const orc_params* p = &s->p;
    int nx = s->g.nx, ny = s->g.ny;
    compute_moments(s);   /* S1 */
    compute_stencils(s);  /* S2 */
    /* S3-S5: equilibria and collision; g relaxes fully to g^eq (rates 1). */
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            int k = y * nx + x;
            if (s->solid[k]) continue;
            double feq[9], geq[9], fl[9], fst[9];
            node_equilibria(s, k, feq, geq);
            for (int i = 0; i < 9; ++i) fl[i] = s->f[i][k];
            double omega = omega_of_nu(viscosity(p, s->phi[k]));
            double Fx = s->boundary[k] ? 0.0 : p->force_x;
            orc_collide(p, fl, feq, omega, s->ux[k], s->uy[k], Fx, 0.0, fst);
            for (int i = 0; i < 9; ++i) s->fs[i][k] = fst[i];
            if (p->model == ORC_BINARY)
                for (int i = 0; i < 9; ++i) s->gs[i][k] = geq[i];
        }
    /* S6: pull streaming f_i(r, t+1) = f*_i(r - e_i), bounce-back from solid. */
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            int k = y * nx + x;
            if (s->solid[k]) continue;
            for (int i = 0; i < 9; ++i) {
                int sx = wrapi(x - EX[i], nx), sy = wrapi(y - EY[i], ny);
                int ks = sy * nx + sx;
                if (s->solid[ks]) {
                    s->f[i][k] = s->fs[OPP[i]][k];
                    if (p->model == ORC_BINARY) s->gp[i][k] = s->gs[OPP[i]][k];
                } else {
                    s->f[i][k] = s->fs[i][ks];
                    if (p->model == ORC_BINARY) s->gp[i][k] = s->gs[i][ks];
                }
            }
        }
    /* S7: boundary nodes are set to rest: f_i <- f_i - w_i e_i.j. */
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            int k = y * nx + x;
            if (!s->boundary[k]) continue;
            double jx = 0.0, jy = 0.0;
            for (int i = 0; i < 9; ++i) {
                jx += EX[i] * s->f[i][k];
                jy += EY[i] * s->f[i][k];
            }
            for (int i = 1; i < 9; ++i) s->f[i][k] -= W[i] * (EX[i] * jx + EY[i] * jy);
        }
    s->t += 1;
}

int orc_step(orc_state* s, long nsteps) {
    for (long n = 0; n < nsteps; ++n) one_step(s);
    /* health check: non-finite population or non-positive density */
    int bad = 0;
    for (int k = 0; k < s->n && !bad; ++k) {
        if (s->solid[k]) continue;
        double rho = 0.0;
        for (int i = 0; i < 9; ++i) {
            if (!isfinite(s->f[i][k]) || !isfinite(s->gp[i][k])) bad = 1;
            rho += s->f[i][k];
        }
        if (!(rho > 0.0)) bad = 1;
    }
    if (bad) {
        set_err("non-finite or non-positive density after stepping");
        return ORC_EUNSTABLE;
    }
    return ORC_OK;
}

void orc_moments(const orc_state* s, double* rho, double* ux, double* uy, double* phi) {
    orc_state* m = (orc_state*)s;
    compute_moments(m);
    for (int k = 0; k < s->n; ++k) {
        if (rho) rho[k] = s->rho[k];
        if (ux) ux[k] = s->ux[k];
        if (uy) uy[k] = s->uy[k];
        if (phi) phi[k] = s->phi[k];
    }
}

void orc_get_pop(const orc_state* s, int which, double* out) {
    for (int i = 0; i < 9; ++i) {
        const double* src = which == 0 ? s->f[i] : s->gp[i];
        memcpy(out + (size_t)i * s->n, src, sizeof(double) * (size_t)s->n);
    }
}

/* Filled length l (Fig. 1b): the centreline value q_c(x) (mean of the two
 * middle rows for even H) is scanned from the tube inlet; l is the linearly
 * interpolated position of the first crossing below q_mid, 0 if the inlet node
 * is already below q_mid, tube_len if there is no crossing.  l_eff = l + H/2. */
int orc_interface_length(const orc_state* s, double q_mid, double* l, double* l_eff) {
    const orc_geom* g = &s->g;
    if (g->tube_len <= 0) {
        set_err("no tube in this geometry");
        return ORC_EINVAL;
    }
    orc_state* m = (orc_state*)s;
    compute_moments(m);
    int H = g->tube_h;
    int ya, yb;
    if (H % 2 == 0) {
        ya = g->y0 + H / 2 - 1;
        yb = g->y0 + H / 2;
    } else {
        ya = yb = g->y0 + (H - 1) / 2;
    }
    double prev = 0.0, res = (double)g->tube_len;
    for (int k = 0; k < g->tube_len; ++k) {
        int x = g->x_in + k;
        double qc = 0.5 * (s->q[ya * g->nx + x] + s->q[yb * g->nx + x]);
        if (qc < q_mid) {
            if (k == 0)
                res = 0.0;
            else
                res = (k - 1) + (prev - q_mid) / (prev - qc);
            break;
        }
        prev = qc;
    }
    *l = res;
    *l_eff = res + 0.5 * H;
    return ORC_OK;
}
