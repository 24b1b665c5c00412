// Host-side thermodynamics of lbcap: Maxwell coexistence of the van der Waals
// bulk pressure (Sec. 2) and the wall gradient that gives a chosen equilibrium
// contact angle (Young's law, Eq. Young, with Cahn's construction for a
// surface energy -h q_s and the boundary condition kappa dn q = -h).
#include <cmath>

#include "lb_thermo.h"

namespace lbt {

namespace {

// van der Waals free energy density W with p0 = rho W' - W = rho T/(1-b rho) - a rho^2.
struct Vdw {
    double a, b, T;
    double W(double r) const { return r * T * std::log(r / (1.0 - b * r)) - a * r * r; }
    double mu(double r) const { return T * std::log(r / (1.0 - b * r)) + T / (1.0 - b * r) - 2.0 * a * r; }
    double p0(double r) const { return r * T / (1.0 - b * r) - a * r * r; }
    double dmu(double r) const {
        const double s = 1.0 - b * r;
        return T / (r * s) + T * b / (s * s) - 2.0 * a;
    }
};

// Composite Simpson rule on n (even) panels.
template <class F>
double simpson(F f, double lo, double hi, int n) {
    const double h = (hi - lo) / n;
    double s = f(lo) + f(hi);
    for (int i = 1; i < n; ++i) s += f(lo + i * h) * ((i & 1) ? 4.0 : 2.0);
    return s * h / 3.0;
}

// Root of a monotone-bracketed function by bisection.
template <class F>
double bisect(F f, double lo, double hi, int iters = 200) {
    double flo = f(lo);
    for (int k = 0; k < iters; ++k) {
        const double mid = 0.5 * (lo + hi);
        const double fm = f(mid);
        if ((fm < 0) == (flo < 0)) {
            lo = mid;
            flo = fm;
        } else {
            hi = mid;
        }
    }
    return 0.5 * (lo + hi);
}

}  // namespace

bool vdw_coexistence(double a, double b, double T, double* rl, double* rg) {
    Vdw v{a, b, T};
    // spinodals bound the two branches: dp0/drho = rho dmu/drho = 0
    const double rc = 1.0 / (3.0 * b);
    if (!(T < 8.0 * a / (27.0 * b))) return false;  // above the critical temperature
    // Newton on (p0(l) - p0(g), mu(l) - mu(g)) from a start on each branch
    double l = 1.3 * rc, g = 0.7 * rc;
    l = std::fmin(l, 0.95 / b);
    for (int it = 0; it < 200; ++it) {
        const double f1 = v.p0(l) - v.p0(g);
        const double f2 = v.mu(l) - v.mu(g);
        // d p0/d rho = rho dmu/drho
        const double j11 = l * v.dmu(l), j12 = -g * v.dmu(g);
        const double j21 = v.dmu(l), j22 = -v.dmu(g);
        const double det = j11 * j22 - j12 * j21;
        if (det == 0.0) return false;
        double dl = (f1 * j22 - f2 * j12) / det;
        double dg = (j11 * f2 - j21 * f1) / det;
        // damp steps that would leave the physical range
        double sc = 1.0;
        while ((l - sc * dl) <= rc || (l - sc * dl) >= 1.0 / b || (g - sc * dg) <= 0.0 || (g - sc * dg) >= rc)
            sc *= 0.5;
        l -= sc * dl;
        g -= sc * dg;
        if (std::fabs(dl) + std::fabs(dg) < 1e-15) break;
    }
    *rl = l;
    *rg = g;
    return std::isfinite(l) && std::isfinite(g) && l > g;
}

// cos(theta) of the binary phi^4 model as a function of Omega (closed form of the
// Cahn construction for quartic wells): cos = ((1+O)^1.5 - (1-O)^1.5)/2.
static double binary_cos_of_omega(double O) {
    return 0.5 * (std::pow(1.0 + O, 1.5) - std::pow(1.0 - O, 1.5));
}

bool binary_wall_gradient(double kappa, double A, double B, double theta_deg, double* G) {
    if (!(kappa > 0 && A > 0 && B > 0)) return false;
    const double c = std::cos(theta_deg * M_PI / 180.0);
    if (!(theta_deg > 0.0 && theta_deg < 180.0)) return false;
    // cos is odd and increasing in Omega on [-1, 1] and reaches +-sqrt(2) at the
    // ends, so every angle in (0, 180) has a root with |Omega| < 1
    const double O = bisect([&](double o) { return binary_cos_of_omega(o) - c; }, -1.0, 1.0);
    // Omega = h sqrt(B/A) sqrt(2/(kappa A)) with h = -kappa G
    *G = -O * A / std::sqrt(2.0 * kappa * B);
    return true;
}

bool vdw_wall_gradient(double kappa, double a, double b, double T, double theta_deg, double* G) {
    double rl, rg;
    if (!(kappa > 0) || !vdw_coexistence(a, b, T, &rl, &rg)) return false;
    if (!(theta_deg > 0.0 && theta_deg < 180.0)) return false;
    if (std::fabs(theta_deg - 90.0) < 1e-12) {
        *G = 0.0;
        return true;
    }
    Vdw v{a, b, T};
    const double mub = v.mu(rl), pb = v.p0(rl);
    auto dW = [&](double r) { return std::fmax(v.W(r) - mub * r + pb, 0.0); };
    auto root = [&](double r) { return std::sqrt(2.0 * kappa * dW(r)); };
    const int N = 4000;
    const double gamma_lg = simpson(root, rg, rl, N);
    // barrier top between the phases
    double rh = rg, best = 0.0;
    for (int i = 1; i < N; ++i) {
        const double r = rg + (rl - rg) * i / N;
        if (dW(r) > best) {
            best = dW(r);
            rh = r;
        }
    }
    const double hmax = root(rh);
    auto cos_of_h = [&](double h) -> double {
        double sg, sl;
        if (h > 0) {
            sg = bisect([&](double r) { return root(r) - h; }, rg, rh);
            double hi = rl;
            while (root(hi) < h) hi = rl + 2.0 * (hi - rl) + 1e-3;
            sl = bisect([&](double r) { return root(r) - h; }, rl, hi);
        } else {
            sl = bisect([&](double r) { return h + root(r); }, rh, rl);
            double lo = rg;
            while (root(lo) < -h) lo = rg - 2.0 * (rg - lo) - 1e-3;
            sg = bisect([&](double r) { return h + root(r); }, lo, rg);
        }
        auto span = [&](double p, double q) { return p < q ? simpson(root, p, q, N) : simpson(root, q, p, N); };
        const double gsg = -h * sg + span(sg, rg);
        const double gsl = -h * sl + span(sl, rl);
        return (gsg - gsl) / gamma_lg;
    };
    const double c = std::cos(theta_deg * M_PI / 180.0);
    const double lim = 0.999 * hmax;
    if (c > cos_of_h(lim) || c < cos_of_h(-lim)) return false;
    const double h = bisect([&](double hh) { return cos_of_h(hh) - c; }, -lim, lim, 80);
    *G = -h / kappa;
    return true;
}

}  // namespace lbt
