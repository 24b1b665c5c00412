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
