// Overdamped motion of a Janus cylinder driven by its radiation force and
// torque (arXiv 2509.22308, Sec. IV.C): host-side integration over a design
// map row.  Interpolation: the periodic cubic spline through the map's
// samples in phi0 (C2, exact at the samples); integrator: the classical
// fourth-order Runge-Kutta method with a fixed step.
#include <cmath>
#include <vector>

#include "../../include/jlb.h"
#include "jlb_host_internal.h"

namespace jlb {
namespace {

// Periodic cubic spline on the uniform grid x_k = x0 + k h, k = 0..n-1,
// period n h.  Second derivatives m_k solve the cyclic system
//   m_{k-1} + 4 m_k + m_{k+1} = 6 (y_{k+1} - 2 y_k + y_{k-1}) / h^2,
// done here by the Sherman-Morrison form of the Thomas algorithm.
struct PeriodicSpline {
    int n = 0;
    double x0 = 0.0, h = 1.0;
    std::vector<double> y, m;

    void build(int n_, double x0_, const double *y_)
    {
        n = n_;
        x0 = x0_;
        h = 2.0 * M_PI / n;
        y.assign(y_, y_ + n);
        std::vector<double> r(n);
        for (int k = 0; k < n; ++k)
            r[k] = 6.0 * (y[(k + 1) % n] - 2.0 * y[k] + y[(k + n - 1) % n]) / (h * h);
        // A = tridiag(1, 4, 1) with corners 1: A = B + u v^T, u = (g, 0.., 1), v = (1, 0.., 1/g)
        const double g = -4.0;
        std::vector<double> diag(n, 4.0);
        diag[0] -= g;
        diag[n - 1] -= 1.0 / g;
        auto thomas = [&](std::vector<double> d) {
            std::vector<double> c(n), dd(n);
            c[0] = 1.0 / diag[0];
            dd[0] = d[0] / diag[0];
            for (int k = 1; k < n; ++k) {
                const double den = diag[k] - c[k - 1];
                c[k] = 1.0 / den;
                dd[k] = (d[k] - dd[k - 1]) / den;
            }
            for (int k = n - 2; k >= 0; --k) dd[k] -= c[k] * dd[k + 1];
            return dd;
        };
        std::vector<double> u(n, 0.0);
        u[0] = g;
        u[n - 1] = 1.0;
        const std::vector<double> zr = thomas(r), zu = thomas(u);
        const double fac = (zr[0] + zr[n - 1] / g) / (1.0 + zu[0] + zu[n - 1] / g);
        m.resize(n);
        for (int k = 0; k < n; ++k) m[k] = zr[k] - fac * zu[k];
    }

    double operator()(double x) const
    {
        const double u = (x - x0) / h;
        const double fl = std::floor(u);
        const double t = u - fl;
        long k = (long)fl % n;
        if (k < 0) k += n;
        const long k1 = (k + 1) % n;
        const double s = 1.0 - t;
        return s * y[k] + t * y[k1] + h * h / 6.0 * ((s * s * s - s) * m[k] + (t * t * t - t) * m[k1]);
    }
};

}  // namespace
}  // namespace jlb

using namespace jlb;

extern "C" int jlb_trajectory(int32_t n, double phi_first, const double *fx, const double *fy, const double *tz,
                              double phi_start, double dt, int64_t nsteps, double log_l_over_a,
                              int32_t record_every, double *out)
{
    clear_error();
    if (n < 4) return fail(JLB_E_ARG, "need at least 4 samples per period, got %d", n);
    if (!fx || !fy || !tz || !out) return fail(JLB_E_ARG, "null array");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(JLB_E_ARG, "dt must be > 0");
    if (nsteps < 0 || record_every < 1) return fail(JLB_E_ARG, "nsteps >= 0 and record_every >= 1");
    if (!std::isfinite(phi_first) || !std::isfinite(phi_start) || !std::isfinite(log_l_over_a))
        return fail(JLB_E_ARG, "non-finite argument");
    for (int k = 0; k < n; ++k)
        if (!std::isfinite(fx[k]) || !std::isfinite(fy[k]) || !std::isfinite(tz[k]))
            return fail(JLB_E_ARG, "non-finite map value at sample %d", k);
    PeriodicSpline sx, sy, st;
    sx.build(n, phi_first, fx);
    sy.build(n, phi_first, fy);
    st.build(n, phi_first, tz);
    const double cv = log_l_over_a / (4.0 * M_PI), cw = 1.0 / (2.0 * M_PI);
    // state (x, y, phi); the right-hand side depends on phi only
    auto rhs = [&](double phi, double d[3]) {
        d[0] = cv * sx(phi);
        d[1] = cv * sy(phi);
        d[2] = cw * st(phi);
    };
    double x = 0.0, y = 0.0, phi = phi_start;
    int64_t rec = 0;
    auto record = [&](int64_t step) {
        out[4 * rec + 0] = (double)step * dt;
        out[4 * rec + 1] = x;
        out[4 * rec + 2] = y;
        out[4 * rec + 3] = phi;
        ++rec;
    };
    record(0);
    for (int64_t s = 1; s <= nsteps; ++s) {
        double k1[3], k2[3], k3[3], k4[3];
        rhs(phi, k1);
        rhs(phi + 0.5 * dt * k1[2], k2);
        rhs(phi + 0.5 * dt * k2[2], k3);
        rhs(phi + dt * k3[2], k4);
        x += dt / 6.0 * (k1[0] + 2.0 * k2[0] + 2.0 * k3[0] + k4[0]);
        y += dt / 6.0 * (k1[1] + 2.0 * k2[1] + 2.0 * k3[1] + k4[1]);
        phi += dt / 6.0 * (k1[2] + 2.0 * k2[2] + 2.0 * k3[2] + k4[2]);
        if (s % record_every == 0) record(s);
    }
    return JLB_OK;
}
