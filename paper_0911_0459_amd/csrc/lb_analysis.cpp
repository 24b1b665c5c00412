// Meniscus analysis of lbcap (host code): the dynamic contact angle of the
// meniscus in the tube, from a circle fitted to the interface (the analysis
// behind the paper's dynamic angles, Sec. 3.2 and Fig. 5).
//
// In each tube row away from the walls the interface is located as for the
// filled length: the first position from the inlet where q falls below q_mid,
// linearly interpolated.  A circle whose centre lies on the channel centreline
// (the meniscus of a symmetric channel is symmetric) is fitted to these points
// by linear least squares in the form
//     x' = -A (x'^2 + y'^2) - C,
// with x' the interface position minus its mean and y' the distance from the
// centreline.  A is minus half the signed curvature, so a flat interface
// (A = 0) is no special case.  With the walls half a node outside the boundary
// rows the channel is H wide, and a circle of radius R meets the walls at the
// angle theta with cos(theta) = (H/2) / R, measured through the liquid (the
// liquid fills from the inlet side): positive when the centre lies on the gas
// side (a wetting meniscus), negative otherwise.
#include <algorithm>
#include <cmath>
#include <vector>

#include "lbcap.h"
#include "lb_internal.h"

extern "C" lb_status lb_meniscus_angle_field(const double* q, const lb_geometry* g, double q_mid, int edge_rows,
                                              double* theta_deg, double* radius, double* apex_x) {
    if (!q || !g) return lbk::set_error(LB_EINVAL, "null argument");
    if (g->tube_len <= 0 || g->tube_h <= 0) return lbk::set_error(LB_EINVAL, "the geometry has no tube");
    if (edge_rows < 0 || g->tube_h - 2 * edge_rows < 3)
        return lbk::set_error(LB_EINVAL, "edge_rows leaves fewer than 3 rows to fit");
    if (!std::isfinite(q_mid)) return lbk::set_error(LB_EINVAL, "q_mid must be finite");
    const int nx = g->nx;
    const double yc = g->y0 + 0.5 * (g->tube_h - 1);
    std::vector<double> xs, ys;
    for (int y = g->y0 + edge_rows; y < g->y0 + g->tube_h - edge_rows; ++y) {
        const double* row = q + (size_t)y * nx;
        if (row[g->x_in] < q_mid) continue;   // no liquid at the inlet in this row
        for (int k = 1; k < g->tube_len; ++k) {
            const double a = row[g->x_in + k - 1], b = row[g->x_in + k];
            if (b < q_mid) {
                xs.push_back(g->x_in + (k - 1) + (a - q_mid) / (a - b));
                ys.push_back(y - yc);
                break;
            }
        }
    }
    const size_t n = xs.size();
    if (n < 3) return lbk::set_error(LB_ESTATE, "no meniscus in the tube");
    double xm = 0.0;
    for (double x : xs) xm += x;
    xm /= (double)n;
    // normal equations of x' = -A s - C in the unknowns (A, C)
    double ss = 0.0, s1 = 0.0, sx = 0.0, x1 = 0.0;
    for (size_t i = 0; i < n; ++i) {
        const double xp = xs[i] - xm, s = xp * xp + ys[i] * ys[i];
        ss += s * s;
        s1 += s;
        sx += s * xp;
        x1 += xp;
    }
    const double det = ss * (double)n - s1 * s1;
    if (!(std::fabs(det) > 0.0)) return lbk::set_error(LB_ESTATE, "degenerate interface points");
    // minimise sum (x' + A s + C)^2:  [ss s1; s1 n] [A; C] = -[sx; x1]
    const double A = -(sx * (double)n - s1 * x1) / det;
    const double C = -(ss * x1 - s1 * sx) / det;
    const double half = 0.5 * g->tube_h;
    double cos_t, R, apex;
    if (std::fabs(A) < 1e-14) {
        cos_t = 0.0;
        R = INFINITY;
        apex = xm - C;
    } else {
        const double xcp = -0.5 / A;                       // centre, relative to xm
        R = std::sqrt(std::fmax(xcp * xcp - C / A, 0.0));
        const double sgn = A < 0.0 ? 1.0 : -1.0;           // centre on the gas side: wetting
        cos_t = sgn * std::fmin(1.0, half / R);
        apex = xm + xcp - sgn * R;
    }
    if (theta_deg) *theta_deg = std::acos(cos_t) * (180.0 / M_PI);
    if (radius) *radius = R;
    if (apex_x) *apex_x = apex;
    return LB_OK;
}

// ---- flow along the tube (Sec. 2.2, Fig. 3) ----------------------------------
// The liquid column is the set of channel rows from x_in + margin to the
// meniscus (the filled length) minus margin, the gas ahead of it the rows from
// the meniscus plus margin to the tube's end minus margin.  Over each region
// the mean density and the mass-weighted mean x velocity sum(rho u_x) /
// sum(rho) are formed; with the meniscus speed v the rates at which mass
// crosses the interface, per unit width, are rho (v - u) on either side: the
// rate of condensation when positive.  In a steady moving interface the two
// sides carry the same rate (mass conservation across the interface).
extern "C" lb_status lb_tube_flow_field(const double* q, const double* rho, const double* ux, const lb_geometry* g,
                                         double q_mid, int margin, double v_meniscus, double* u_centre,
                                         lb_tube_flow_stats* out) {
    if (!q || !rho || !ux || !g || !out) return lbk::set_error(LB_EINVAL, "null argument");
    if (g->tube_len <= 0 || g->tube_h <= 0) return lbk::set_error(LB_EINVAL, "the geometry has no tube");
    if (margin < 0 || !std::isfinite(q_mid) || !std::isfinite(v_meniscus))
        return lbk::set_error(LB_EINVAL, "margin must be >= 0, q_mid and v_meniscus finite");
    const int nx = g->nx, H = g->tube_h;
    const int ya = (H % 2 == 0) ? g->y0 + H / 2 - 1 : g->y0 + (H - 1) / 2;
    const int yb = (H % 2 == 0) ? g->y0 + H / 2 : ya;
    auto at = [&](const double* f, int x, int y) { return f[(size_t)y * nx + x]; };
    // filled length from the centreline order field (the definition of lb_interface_length)
    double l = g->tube_len;
    for (int k = 0; k < g->tube_len; ++k) {
        const int x = g->x_in + k;
        const double qc = 0.5 * (at(q, x, ya) + at(q, x, yb));
        if (qc < q_mid) {
            if (k == 0) {
                l = 0.0;
            } else {
                const double qp = 0.5 * (at(q, x - 1, ya) + at(q, x - 1, yb));
                l = (k - 1) + (qp - q_mid) / (qp - qc);
            }
            break;
        }
    }
    if (u_centre)
        for (int k = 0; k < g->tube_len; ++k) {
            const int x = g->x_in + k;
            u_centre[k] = 0.5 * (at(ux, x, ya) + at(ux, x, yb));
        }
    auto region = [&](int x0, int x1, double& rho_m, double& u_m, int& cols) {
        double m = 0.0, p = 0.0;
        long n = 0;
        for (int x = x0; x < x1; ++x)
            for (int y = g->y0; y < g->y0 + H; ++y) {
                m += at(rho, x, y);
                p += at(rho, x, y) * at(ux, x, y);
                ++n;
            }
        cols = std::max(0, x1 - x0);
        rho_m = n > 0 ? m / (double)n : 0.0;
        u_m = m > 0.0 ? p / m : 0.0;
    };
    const int xm = g->x_in + (int)std::floor(l);
    int cl = 0, cg = 0;
    region(g->x_in + margin, std::min(xm - margin, g->x_in + g->tube_len), out->rho_liquid, out->u_liquid, cl);
    region(std::max(xm + 1 + margin, g->x_in), g->x_in + g->tube_len - margin, out->rho_gas, out->u_gas, cg);
    out->l = l;
    out->liquid_cols = cl;
    out->gas_cols = cg;
    out->condensation_liquid_side = cl > 0 ? out->rho_liquid * (v_meniscus - out->u_liquid) : 0.0;
    out->condensation_gas_side = cg > 0 ? out->rho_gas * (v_meniscus - out->u_gas) : 0.0;
    return LB_OK;
}

// ---- Washburn's law with the drag of the gas (Eq. 1 - 3) ---------------------
// The capillary pressure 2 gamma cos(theta) / H drives the liquid column of
// length l and the gas column of length L - l ahead of it, each in Poiseuille
// flow (Eq. 1: dp/dx = -12 eta v / H^2), at the speed v = dl/dt:
//   2 gamma cos(theta) / H = 12 v (eta_l l + eta_g (L - l)) / H^2,
// whose integral from l(0) = l0 is
//   (eta_l - eta_g) (l^2 - l0^2) / 2 + eta_g L (l - l0) = gamma H cos(theta) t / 6.
// eta_g = 0 gives Eq. 3, l^2 = l0^2 + gamma H cos(theta) t / (3 eta_l).
extern "C" lb_status lb_washburn_length(double t, double l0, double H, double L, double gamma, double cos_theta,
                                         double eta_l, double eta_g, double* l) {
    if (!l) return lbk::set_error(LB_EINVAL, "null argument");
    if (!(t >= 0.0) || !(l0 >= 0.0) || !(H > 0.0) || !(L >= l0) || !(eta_l > 0.0) || !(eta_g >= 0.0) ||
        !std::isfinite(gamma) || !std::isfinite(cos_theta) || !std::isfinite(t))
        return lbk::set_error(LB_EINVAL, "need t >= 0, 0 <= l0 <= L, H > 0, eta_l > 0, eta_g >= 0");
    const double a = 0.5 * (eta_l - eta_g), b = eta_g * L;
    const double c = a * l0 * l0 + b * l0 + gamma * H * cos_theta * t / 6.0;   // a l^2 + b l = c
    double x;
    if (a == 0.0) {
        x = c / b;
    } else {
        const double disc = b * b + 4.0 * a * c;
        if (!(disc >= 0.0)) return lbk::set_error(LB_EINVAL, "no real filled length (gas column stalls the flow)");
        // the root continuous with l0, without cancellation
        x = 2.0 * c / (b + std::sqrt(disc));
    }
    *l = x;
    return LB_OK;
}
