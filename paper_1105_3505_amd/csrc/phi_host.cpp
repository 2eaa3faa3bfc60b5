// phi, the lattice fundamental solution, on the host.
//
// Route: integrating eq. (1.8) over t1 in closed form (remark closing Section 3) leaves
//   phi(m) = (1/pi) int_0^pi (cos(m2 t) lambda(t)^|m1| - 1) / sqrt(c^2 - 4) dt,
//   c = 4 - 2 cos t,  lambda = (c - sqrt(c^2 - 4)) / 2,  |m1| >= |m2|
// (the t1 integral is the classical int cos(k x)/(c - 2 cos x) dx = 2 pi lambda^k / sqrt(c^2-4)).
// With s = sin(t/2) the pieces have cancellation-free forms:
//   sqrt(c^2 - 4) = 4 s sqrt(1 + s^2),  lambda = exp(-2 asinh s),
//   cos(m2 t) lambda^k - 1 = expm1(-2 k asinh s) - 2 sin^2(m2 t / 2) exp(-2 k asinh s).
// The integrand is analytic on [0, pi] (its limit at 0 is -k/2); it varies on the scale 1/k
// near 0 and oscillates m2/2 times, so panels are geometric near 0 and half a period wide
// after, each with 20-point Gauss-Legendre.  Beyond |m|_inf = 128 the expansion eq. (3.1)
// (true Euler constant) is used; its error there is below 4e-14.
#include "host_math.h"

#include <algorithm>
#include <cmath>
#include <mutex>
#include <thread>

namespace lfmm {
namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr double kEulerGamma = 0.57721566490153286061;

struct GaussRule {
    double x[20], w[20];  // on [-1, 1]
    GaussRule() {
        const int n = 20;
        for (int i = 0; i < n; ++i) {
            // Newton iteration on the Legendre polynomial P_n from a cosine initial guess
            double z = std::cos(kPi * (i + 0.75) / (n + 0.5)), dp = 0;
            for (int it = 0; it < 100; ++it) {
                double p0 = 1.0, p1 = z;
                for (int k = 2; k <= n; ++k) {
                    double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                    p0 = p1;
                    p1 = p2;
                }
                dp = n * (z * p1 - p0) / (z * z - 1.0);
                double dz = p1 / dp;
                z -= dz;
                if (std::fabs(dz) < 1e-17) break;
            }
            x[i] = z;
            w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
        }
    }
};

const GaussRule& gauss() {
    static const GaussRule rule;
    return rule;
}

// integrand of the reduced integral, k = |m1| >= j = |m2|
inline double reduced_integrand(double t, double k, double j) {
    double s = std::sin(0.5 * t);
    if (s == 0.0) return -0.5 * k;
    double q = std::sqrt(1.0 + s * s);
    double e = -2.0 * k * std::asinh(s);
    double sj = std::sin(0.5 * j * t);
    double num = std::expm1(e) - 2.0 * sj * sj * std::exp(e);
    return num / (4.0 * s * q);
}

}  // namespace

double phi_reduced_integral(int64_t m1, int64_t m2) {
    int64_t k = std::llabs(m1), j = std::llabs(m2);
    if (j > k) std::swap(j, k);
    if (k == 0) return 0.0;
    const GaussRule& g = gauss();
    // panel breakpoints: geometric near 0, then half periods of sin^2(j t / 2)
    double width = kPi / double(std::max<int64_t>(j, 2));
    std::vector<double> bp{0.0};
    double h = 1.0 / double(k);
    while (h < width) {
        bp.push_back(h);
        h *= 2.0;
    }
    double t0 = bp.back();
    int nuni = int(std::ceil((kPi - t0) / width));
    for (int i = 1; i <= nuni; ++i) bp.push_back(t0 + (kPi - t0) * double(i) / nuni);
    double sum = 0.0, comp = 0.0;
    for (size_t p = 0; p + 1 < bp.size(); ++p) {
        double a = bp[p], b = bp[p + 1], c = 0.5 * (a + b), r = 0.5 * (b - a);
        double part = 0.0;
        for (int i = 0; i < 20; ++i) part += g.w[i] * reduced_integrand(c + r * g.x[i], double(k), double(j));
        part *= r;
        double t = sum + part;  // Neumaier
        comp += (std::fabs(sum) >= std::fabs(part)) ? (sum - t) + part : (part - t) + sum;
        sum = t;
    }
    return (sum + comp) / kPi;
}

double phi_expansion(double a, double b) {
    double r2 = a * a + b * b;
    double c = a * a / r2, s = b * b / r2;
    double lead = -(0.5 * std::log(r2) + kEulerGamma + 0.5 * std::log(8.0)) / (2.0 * kPi);
    double t4 = (c * c - 6.0 * c * s + s * s) / (24.0 * kPi * r2);
    double c2 = c * c, s2 = s * s;
    double t8 = (43.0 * c2 * c2 - 772.0 * c2 * c * s + 1570.0 * c2 * s2 - 772.0 * c * s2 * s + 43.0 * s2 * s2)
                / (480.0 * kPi * r2 * r2);
    return lead + t4 + t8;
}

std::vector<double> build_phi_table(int radius) {
    std::vector<double> tab(size_t(octant_size(radius)), 0.0);
    unsigned nthreads = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    std::vector<std::thread> pool;
    for (unsigned t = 0; t < nthreads; ++t) {
        pool.emplace_back([&, t]() {
            // rows a interleaved over threads (cost grows with a)
            for (int a = int(t); a <= radius; a += int(nthreads))
                for (int b = 0; b <= a; ++b) tab[size_t(octant_index(a, b))] = phi_reduced_integral(a, b);
        });
    }
    for (auto& th : pool) th.join();
    return tab;
}

const std::vector<double>& phi_table() {
    static std::once_flag once;
    static std::vector<double> tab;
    std::call_once(once, [] { tab = build_phi_table(kPhiTableRadius); });
    return tab;
}

double phi(int64_t m1, int64_t m2) {
    int64_t a = std::llabs(m1), b = std::llabs(m2);
    if (b > a) std::swap(a, b);
    if (a <= kPhiTableRadius) return phi_table()[size_t(octant_index(a, b))];
    return phi_expansion(double(a), double(b));
}

}  // namespace lfmm
