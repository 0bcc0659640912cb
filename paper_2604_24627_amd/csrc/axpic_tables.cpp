// axpic_tables.cpp -- host construction of the energy quantile tables.
//
// The thermal channels draw x = E/T by inverting a cumulative distribution:
//   Compton-like : number density x^4/(e^x - 1)/(24 zeta5)  (the number form of the
//                  power kernel E^5/(e^{E/T}-1), Sec. II.G)
//   brems        : Gamma(k, 1) density x^{k-1} e^{-x}/Gamma(k) (Sec. II.H)
// The quantile x(u) is tabulated against z = ln(u/(1-u)).  It obeys the ODE
//   dy/dz = u(1-u) / (x f(x)),  y = ln x,  u(1-u) = 1/(2 + 2 cosh z),
// which is integrated with classical RK4 from a starting point obtained by
// Newton iteration on the small-x expansion of the CDF.
#include <cmath>
#include <vector>

#include "axpic_tables.h"

namespace axpic_host {

static const double kZeta5 = 1.0369277551433699263;

// Bernoulli numbers B_0..B_20 (B_1 = -1/2): t/(e^t - 1) = sum B_n t^n / n!.
static const double kB[21] = {1.0, -0.5, 1.0 / 6, 0.0, -1.0 / 30, 0.0, 1.0 / 42, 0.0, -1.0 / 30,
                              0.0, 5.0 / 66, 0.0, -691.0 / 2730, 0.0, 7.0 / 6, 0.0,
                              -3617.0 / 510, 0.0, 43867.0 / 798, 0.0, -174611.0 / 330};

// x f(x) for the two distributions.
static double xf_compton(double x) { return std::pow(x, 5) / std::expm1(x) / (24.0 * kZeta5); }
static double xf_gamma(double x, double k) {
    return std::exp(k * std::log(x) - x - std::lgamma(k));
}

// Small-x CDFs: Compton: (1/(24 zeta5)) sum_n B_n x^{n+4} / (n! (n+4));
// Gamma: x^k e^{-x} sum_n x^n / Gamma(k+n+1).
static double cdf_small_compton(double x) {
    double s = 0.0, fact = 1.0, xp = std::pow(x, 4);
    for (int n = 0; n <= 20; ++n) {
        if (n > 0) fact *= n;
        s += kB[n] * xp / (fact * (n + 4));
        xp *= x;
    }
    return s / (24.0 * kZeta5);
}
static double cdf_small_gamma(double x, double k) {
    double s = 0.0, term = std::exp(-std::lgamma(k + 1.0));
    for (int n = 0; n < 60; ++n) {
        s += term;
        term *= x / (k + n + 1.0);
    }
    return std::exp(k * std::log(x) - x) * s;
}

template <class CDF, class XF>
static void build(double* tab, CDF cdf_small, XF xf) {
    const int N = kTabN;
    const double h = (kTabZ1 - kTabZ0) / N;
    const double u0 = 1.0 / (1.0 + std::exp(-kTabZ0));
    // starting point: Newton on the small-x CDF, dC/dx = f(x)
    double x = 0.05;
    for (int it = 0; it < 200; ++it) {
        double f = xf(x) / x;
        double dx = (cdf_small(x) - u0) / f;
        double xn = x - dx;
        if (!(xn > 0.0)) xn = 0.5 * x;
        if (std::fabs(xn - x) < 1e-16 * x) { x = xn; break; }
        x = xn;
    }
    auto rhs = [&](double z, double y) {
        double uu = 1.0 / (2.0 + 2.0 * std::cosh(z));
        return uu / xf(std::exp(y));
    };
    double y = std::log(x);
    const int sub = 32;
    const double hs = h / sub;
    for (int j = 0; j <= N; ++j) {
        double z = kTabZ0 + j * h;
        tab[j] = y;
        tab[N + 1 + j] = rhs(z, y);
        if (j == N) break;
        for (int s = 0; s < sub; ++s) {
            double zz = z + s * hs;
            double k1 = rhs(zz, y);
            double k2 = rhs(zz + 0.5 * hs, y + 0.5 * hs * k1);
            double k3 = rhs(zz + 0.5 * hs, y + 0.5 * hs * k2);
            double k4 = rhs(zz + hs, y + hs * k3);
            y += hs / 6.0 * (k1 + 2 * k2 + 2 * k3 + k4);
        }
    }
}

void build_compton_table(double* tab) {
    build(tab, [](double x) { return cdf_small_compton(x); },
          [](double x) { return xf_compton(x); });
}

void build_gamma_table(double* tab, double k) {
    build(tab, [k](double x) { return cdf_small_gamma(x, k); },
          [k](double x) { return xf_gamma(x, k); });
}

}  // namespace axpic_host
