// Host-side float64 background cosmology for libcola: expansion rate, growth factors, COLA
// kick/drift time integrals, Eq. 3 time nodes and the BBKS linear spectrum amplitude.
//
// Paper: flat LCDM of Sec. 2.1; time nodes of Eq. 3 (Sec. 4.2) with n counting both ends
// (Sec. 4.3: a_i equal to the step width gives z_i = 9 for 10 nodes, 39 for 40).
// Growth and time integrals follow from Eq. 2 with p = a^2 dx/dt and H0 = 1:
//   dx/da = p / (a^3 E),  dp/da = (3/2) Omega_m g / (a^2 E),
//   D'' + (2 + dlnE/dlna) D' = (3/2) Omega_m / (a^3 E^2) * {D1 | D2 - D1^2},  ' = d/dlna.

#include "cola_internal.h"

#include <algorithm>
#include <cmath>
#include <vector>

namespace cola {

double hubble_e(double a, double om) { return std::sqrt(om / (a * a * a) + (1.0 - om)); }

namespace {

// 16-point Gauss-Legendre nodes and weights on [-1, 1] (symmetric half).
const double kGLx[8] = {0.0950125098376374, 0.2816035507792589, 0.4580167776572274,
                        0.6178762444026438, 0.7554044083550030, 0.8656312023878318,
                        0.9445750230732326, 0.9894009349916499};
const double kGLw[8] = {0.1894506104550685, 0.1826034150449236, 0.1691565193950025,
                        0.1495959888165767, 0.1246289712555339, 0.0951585116824928,
                        0.0622535239386479, 0.0271524594117541};

template <class F>
double gauss_legendre(F f, double lo, double hi, int panels) {
    double sum = 0.0;
    double w = (hi - lo) / panels;
    for (int p = 0; p < panels; ++p) {
        double c = lo + (p + 0.5) * w, h = 0.5 * w;
        for (int i = 0; i < 8; ++i) sum += h * kGLw[i] * (f(c - h * kGLx[i]) + f(c + h * kGLx[i]));
    }
    return sum;
}

struct GrowthState { double d1, v1, d2, v2; };

GrowthState growth_rhs(double y, const GrowthState& s, double om) {
    double a = std::exp(y);
    double ea3 = om / (a * a * a);
    double e2 = ea3 + (1.0 - om);
    double dlne = -1.5 * ea3 / e2;
    double coef = 1.5 * ea3 / e2;
    return {s.v1, -(2.0 + dlne) * s.v1 + coef * s.d1,
            s.v2, -(2.0 + dlne) * s.v2 + coef * (s.d2 - s.d1 * s.d1)};
}

GrowthState rk4_step(const GrowthState& s, double y, double h, double om) {
    auto axpy = [](const GrowthState& a, double c, const GrowthState& b) {
        return GrowthState{a.d1 + c * b.d1, a.v1 + c * b.v1, a.d2 + c * b.d2, a.v2 + c * b.v2};
    };
    GrowthState k1 = growth_rhs(y, s, om);
    GrowthState k2 = growth_rhs(y + 0.5 * h, axpy(s, 0.5 * h, k1), om);
    GrowthState k3 = growth_rhs(y + 0.5 * h, axpy(s, 0.5 * h, k2), om);
    GrowthState k4 = growth_rhs(y + h, axpy(s, h, k3), om);
    GrowthState r = s;
    r.d1 += h / 6.0 * (k1.d1 + 2 * k2.d1 + 2 * k3.d1 + k4.d1);
    r.v1 += h / 6.0 * (k1.v1 + 2 * k2.v1 + 2 * k3.v1 + k4.v1);
    r.d2 += h / 6.0 * (k1.d2 + 2 * k2.d2 + 2 * k3.d2 + k4.d2);
    r.v2 += h / 6.0 * (k1.v2 + 2 * k2.v2 + 2 * k3.v2 + k4.v2);
    return r;
}

// Classic RK4 in y = ln a from deep matter domination (a = 1e-6: growing modes D1 = a,
// D2 = -3/7 a^2) with steps of 5e-4 in ln a.  The states on that grid are kept per Omega_m (and
// per thread) up to a = 2, so a value at any a costs one table lookup and at most a few steps.
constexpr double kGrowthStart = 1e-6, kGrowthStep = 5e-4;

struct GrowthTable {
    double om = -1.0;
    std::vector<GrowthState> s;  // state at y = ln(1e-6) + i * kGrowthStep
};

const GrowthTable& growth_table(double om) {
    static thread_local GrowthTable t;
    if (t.om != om) {
        const double y0 = std::log(kGrowthStart);
        const int n = static_cast<int>(std::ceil((std::log(2.0) - y0) / kGrowthStep)) + 1;
        t.s.resize(n);
        t.s[0] = GrowthState{kGrowthStart, kGrowthStart, -3.0 / 7.0 * kGrowthStart * kGrowthStart,
                             -6.0 / 7.0 * kGrowthStart * kGrowthStart};
        for (int i = 1; i < n; ++i) t.s[i] = rk4_step(t.s[i - 1], y0 + (i - 1) * kGrowthStep, kGrowthStep, om);
        t.om = om;
    }
    return t;
}

GrowthState integrate_growth(double a_target, double om) {
    const GrowthTable& t = growth_table(om);
    const double y0 = std::log(kGrowthStart), y = std::log(a_target);
    long i = static_cast<long>(std::floor((y - y0) / kGrowthStep));
    i = std::max(0L, std::min(i, static_cast<long>(t.s.size()) - 1));
    GrowthState s = t.s[i];
    double yi = y0 + i * kGrowthStep;
    const int n = std::max(0, static_cast<int>(std::ceil((y - yi) / kGrowthStep - 1e-12)));
    if (n > 0) {
        const double h = (y - yi) / n;
        for (int k = 0; k < n; ++k, yi += h) s = rk4_step(s, yi, h, om);
    }
    return s;
}

}  // namespace

Growth growth(double a, double om) {
    const GrowthState norm = integrate_growth(1.0, om);
    GrowthState s = integrate_growth(a, om);
    double n1 = norm.d1;
    Growth g;
    g.d1 = s.d1 / n1;
    g.d2 = s.d2 / (n1 * n1);
    g.dd1_da = s.v1 / n1 / a;
    g.dd2_da = s.v2 / (n1 * n1) / a;
    return g;
}

double kick_integral(double a0, double a1, double om) {
    if (a1 == a0) return 0.0;
    return gauss_legendre([om](double a) { return 1.0 / (a * a * hubble_e(a, om)); }, a0, a1, 16);
}

double drift_integral(double a0, double a1, double om) {
    if (a1 == a0) return 0.0;
    return gauss_legendre([om](double a) { return 1.0 / (a * a * a * hubble_e(a, om)); }, a0, a1, 16);
}

// Eq. 3: nodes equally spaced in f(a) between a_0 and a_final, f = a, ln a or a^p.
std::vector<double> time_nodes(const cola_problem& p) {
    const double a0 = 1.0 / (1.0 + p.z_init);
    const int n = p.n_steps;
    std::vector<double> a(n);
    if (p.sampling == 1) {
        const double df = (std::log(p.a_final) - std::log(a0)) / (n - 1);
        for (int j = 0; j < n; ++j) a[j] = std::exp(std::log(a0) + j * df);
    } else if (p.sampling == 2) {
        const double q = p.sampling_power;
        const double f0 = std::pow(a0, q);
        const double df = (std::pow(p.a_final, q) - f0) / (n - 1);
        for (int j = 0; j < n; ++j) a[j] = std::pow(f0 + j * df, 1.0 / q);
    } else {
        const double da = (p.a_final - a0) / (n - 1);
        for (int j = 0; j < n; ++j) a[j] = a0 + j * da;
    }
    a[0] = a0;
    a[n - 1] = p.a_final;
    return a;
}

Schedule make_schedule(const cola_problem& p, const cola_cosmology& c) {
    Schedule s;
    s.omega_m = c.omega_m;
    s.a = time_nodes(p);
    int n = p.n_steps;
    s.d1.resize(n);
    s.d2.resize(n);
    for (int j = 0; j < n; ++j) {
        Growth g = growth(s.a[j], c.omega_m);
        s.d1[j] = g.d1;
        s.d2[j] = g.d2;
    }
    s.k_out.resize(n - 1);
    s.k_in.resize(n - 1);
    s.drift.resize(n - 1);
    for (int j = 0; j < n - 1; ++j) {
        double ah = 0.5 * (s.a[j] + s.a[j + 1]);
        s.k_out[j] = kick_integral(s.a[j], ah, c.omega_m);
        s.k_in[j] = kick_integral(ah, s.a[j + 1], c.omega_m);
        s.drift[j] = drift_integral(s.a[j], s.a[j + 1], c.omega_m);
    }
    return s;
}

// ----------------------------------------------------------------------------- BBKS

double bbks_gamma(const cola_cosmology& c) {
    return c.omega_m * c.h * std::exp(-c.omega_b * (1.0 + std::sqrt(2.0 * c.h) / c.omega_m));
}

double bbks_transfer(double k, double gamma) {
    double q = k / gamma;
    if (q <= 0.0) return 1.0;
    double poly = 1.0 + 3.89 * q + std::pow(16.1 * q, 2) + std::pow(5.46 * q, 3) + std::pow(6.71 * q, 4);
    return std::log1p(2.34 * q) / (2.34 * q) * std::pow(poly, -0.25);
}

static double tophat(double x) {
    if (x < 0.1) {
        double x2 = x * x;
        return 1.0 - x2 / 10.0 + x2 * x2 / 280.0 - x2 * x2 * x2 / 15120.0;
    }
    return 3.0 * (std::sin(x) - x * std::cos(x)) / (x * x * x);
}

// A of P(k) = A k^n_s T^2 with sigma(8 h^-1 Mpc) = sigma_8:
// sigma^2 = int dlnk k^3 P W^2(kR) / (2 pi^2), cut into one-oscillation panels of kR.
double linear_amplitude(const cola_cosmology& c) {
    const double r = 8.0, pi = 3.14159265358979323846;
    double gamma = bbks_gamma(c);
    auto integrand = [&](double lnk) {
        double k = std::exp(lnk);
        double t = bbks_transfer(k, gamma);
        double w = tophat(k * r);
        return k * k * k * std::pow(k, c.n_s) * t * t * w * w / (2.0 * pi * pi);
    };
    double sum = gauss_legendre(integrand, std::log(1e-7), std::log(1.0 / r), 48);
    for (double x = 1.0; x < 2000.0; x += pi) {
        double x1 = std::min(x + pi, 2000.0);
        sum += gauss_legendre(integrand, std::log(x / r), std::log(x1 / r), 1);
    }
    return c.sigma_8 * c.sigma_8 / sum;
}

}  // namespace cola
