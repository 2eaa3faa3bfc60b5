// phi, the lattice fundamental solution, on the host, for the 5-point operator of eq. (1.2)
// and for other constant-coefficient operators of the same family (Sections 1 and 3.1: the
// method needs only phi, so it carries over to other difference operators).
//
// Route: an operator whose symbol is affine in cos t1,
//   sigma(t) = (alpha(t2) - beta(t2) cos t1) / w,  alpha = a0 + a1 cos t2,  beta = b0 + b1 cos t2,
// lets eq. (1.8) be integrated over t1 in closed form (the remark closing Section 3 does this
// for the 5-point operator; the t1 integral is int cos(k x) / (alpha - beta cos x) dx =
// 2 pi lambda^k / sqrt(alpha^2 - beta^2), lambda = exp(-acosh(alpha / beta))), leaving
//   phi(m) = (w / pi) int_0^pi (cos(m2 t) lambda(t)^|m1| - 1) / sqrt(alpha^2 - beta^2) dt,
// with |m1| >= |m2| (D4 symmetry).  A zero row sum (sigma(0) = 0) gives alpha - beta =
// D1 s^2 with s = sin(t/2), D1 = 2 (b1 - a1), so the pieces have cancellation-free forms:
//   sqrt(alpha^2 - beta^2) = s sqrt(D1 (alpha + beta)),  acosh(alpha / beta) = 2 asinh(s sqrt(D1 / (2 beta))),
//   cos(m2 t) lambda^k - 1 = expm1(-k psi) - 2 sin^2(m2 t / 2) exp(-k psi),  psi = acosh(alpha / beta).
// The integrand is analytic on [0, pi] (its limit at 0 is -k / beta(0)); it varies on the
// scale 1/k near 0 and oscillates m2/2 times, so panels are geometric near 0 and half a
// period wide after, each with 20-point Gauss-Legendre.
//
// Beyond |m|_inf = 128 an expansion in the form of eq. (3.1) is used,
//   phi(m) ~ -(1/2pi) (log |m| + C) + sum_{k=1..3} |m|^-2k sum_{j=0..k} c_kj cos(4 j theta),
// (D4 symmetry leaves only the harmonics cos(4 j theta)).  For the 5-point operator it is eq.
// (3.1) itself, true Euler constant: C = gamma + log(8)/2, and the two printed correction
// terms are cos(4 theta) / (24 pi |m|^2) and (18 cos(4 theta) + 25 cos(8 theta)) / (480 pi |m|^4).
// Its error there is below 4e-14.  For other operators the paper leaves the expansion to
// computer algebra that it does not give; here C and c_kj are fitted by least squares to the
// tabulated values with |m| >= 40, where the next term is below 1e-15.
#include "host_math.h"

#include <algorithm>
#include <cmath>
#include <mutex>
#include <stdexcept>
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
inline double reduced_integrand(const Stencil& st, double t, double k, double j) {
    const double s = std::sin(0.5 * t);
    const double beta = st.b0 + st.b1 * (1.0 - 2.0 * s * s);
    if (s == 0.0) return -k / beta;
    const double d1 = 2.0 * (st.b1 - st.a1);
    const double sum = (st.a0 + st.b0 + st.a1 + st.b1) - 2.0 * (st.a1 + st.b1) * s * s;   // alpha + beta
    const double psi = 2.0 * std::asinh(s * std::sqrt(d1 / (2.0 * beta)));
    const double e = -k * psi;
    const double sj = std::sin(0.5 * j * t);
    const double num = std::expm1(e) - 2.0 * sj * sj * std::exp(e);
    return num / (s * std::sqrt(d1 * sum));
}

}  // namespace

double phi_reduced_integral(const Stencil& st, int64_t m1, int64_t m2) {
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
        for (int i = 0; i < 20; ++i) part += g.w[i] * reduced_integrand(st, c + r * g.x[i], double(k), double(j));
        part *= r;
        double t = sum + part;  // Neumaier
        comp += (std::fabs(sum) >= std::fabs(part)) ? (sum - t) + part : (part - t) + sum;
        sum = t;
    }
    return st.w * (sum + comp) / kPi;
}

double phi_expansion(const Stencil& st, double a, double b) {
    const double r2 = a * a + b * b, ir2 = 1.0 / r2;
    const double c2 = (a * a - b * b) * ir2;   // cos 2 theta
    const double c4 = 2.0 * c2 * c2 - 1.0, c8 = 2.0 * c4 * c4 - 1.0, c12 = 2.0 * c4 * c8 - c4;
    const double lead = -(0.5 * std::log(r2) + st.C) / (2.0 * kPi);
    const double t1 = st.c[0][0] + st.c[0][1] * c4;
    const double t2 = st.c[1][0] + st.c[1][1] * c4 + st.c[1][2] * c8;
    const double t3 = st.c[2][0] + st.c[2][1] * c4 + st.c[2][2] * c8 + st.c[2][3] * c12;
    return lead + ir2 * (t1 + ir2 * (t2 + ir2 * t3));
}

std::vector<double> build_phi_table(const Stencil& st, int radius) {
    std::vector<double> tab(size_t(octant_size(radius)), 0.0);
    unsigned nthreads = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    std::vector<std::thread> pool;
    for (unsigned t = 0; t < nthreads; ++t) {
        pool.emplace_back([&, t]() {
            // rows a interleaved over threads (cost grows with a)
            for (int a = int(t); a <= radius; a += int(nthreads))
                for (int b = 0; b <= a; ++b) tab[size_t(octant_index(a, b))] = phi_reduced_integral(st, a, b);
        });
    }
    for (auto& th : pool) th.join();
    return tab;
}

namespace {

struct StencilData {
    Stencil st;
    std::vector<double> table;
};

// The |m|^-6 terms of the 5-point expansion, which eq. (3.1) stops short of: least squares over
// the table entries with |m| >= 40 of phi minus the eq. (3.1) value, columns |m|^-6 cos(4 j theta)
// scaled to unit size at |m| = 40.  With them the expansion agrees with the quadrature table to
// about 4e-15 for |m| >= 64 (2e-12 without), so kernels may use it from there on.
void fit_far_field_k3(StencilData& d) {
    std::vector<std::pair<int, int>> pts;
    for (int a = 0; a <= kPhiTableRadius; ++a)
        for (int b = 0; b <= a; ++b)
            if (double(a) * a + double(b) * b >= 40.0 * 40.0) pts.emplace_back(a, b);
    const int ncol = 4;
    Mat A(int(pts.size()), ncol), B(int(pts.size()), 1);
    for (size_t i = 0; i < pts.size(); ++i) {
        const double a = pts[i].first, b = pts[i].second, r2 = a * a + b * b;
        const double c2 = (a * a - b * b) / r2, c4 = 2 * c2 * c2 - 1, c8 = 2 * c4 * c4 - 1, c12 = 2 * c4 * c8 - c4;
        const double u3 = std::pow(1600.0 / r2, 3);
        const double row[ncol] = {u3, u3 * c4, u3 * c8, u3 * c12};
        for (int j = 0; j < ncol; ++j) A(int(i), j) = row[j];
        B(int(i), 0) = d.table[size_t(octant_index(pts[i].first, pts[i].second))] - phi_expansion(d.st, a, b);
    }
    const Mat X = least_squares(A, B);
    const double s3 = 1600.0 * 1600.0 * 1600.0;
    for (int j = 0; j < ncol; ++j) d.st.c[2][j] = X(j, 0) * s3;
}

// Far-field coefficients fitted to the table: least squares over the entries with |m| >= 40
// of phi + log|m| / (2 pi) = -C / (2 pi) + sum_k |m|^-2k sum_j c_kj cos(4 j theta), each basis
// column scaled to unit size at |m| = 40.
void fit_far_field(StencilData& d) {
    std::vector<std::pair<int, int>> pts;
    for (int a = 0; a <= kPhiTableRadius; ++a)
        for (int b = 0; b <= a; ++b)
            if (double(a) * a + double(b) * b >= 40.0 * 40.0) pts.emplace_back(a, b);
    const int ncol = 10;
    Mat A(int(pts.size()), ncol), B(int(pts.size()), 1);
    for (size_t i = 0; i < pts.size(); ++i) {
        const double a = pts[i].first, b = pts[i].second, r2 = a * a + b * b;
        const double c2 = (a * a - b * b) / r2, c4 = 2 * c2 * c2 - 1, c8 = 2 * c4 * c4 - 1, c12 = 2 * c4 * c8 - c4;
        const double u = 1600.0 / r2;   // (40 / |m|)^2
        const double row[ncol] = {1.0, u, u * c4, u * u, u * u * c4, u * u * c8, u * u * u, u * u * u * c4,
                                  u * u * u * c8, u * u * u * c12};
        for (int j = 0; j < ncol; ++j) A(int(i), j) = row[j];
        B(int(i), 0) = d.table[size_t(octant_index(pts[i].first, pts[i].second))] + 0.5 * std::log(r2) / (2.0 * kPi);
    }
    const Mat X = least_squares(A, B);
    d.st.C = -2.0 * kPi * X(0, 0);
    const double s1 = 1600.0, s2 = s1 * s1, s3 = s2 * s1;
    d.st.c[0][0] = X(1, 0) * s1;
    d.st.c[0][1] = X(2, 0) * s1;
    d.st.c[1][0] = X(3, 0) * s2;
    d.st.c[1][1] = X(4, 0) * s2;
    d.st.c[1][2] = X(5, 0) * s2;
    d.st.c[2][0] = X(6, 0) * s3;
    d.st.c[2][1] = X(7, 0) * s3;
    d.st.c[2][2] = X(8, 0) * s3;
    d.st.c[2][3] = X(9, 0) * s3;
}

const StencilData& stencil_data(int id) {
    static std::once_flag once[kNumStencils];
    static StencilData data[kNumStencils];
    if (id < 0 || id >= kNumStencils) throw std::invalid_argument("unknown lattice operator");
    std::call_once(once[id], [id] {
        StencilData& d = data[id];
        Stencil& st = d.st;
        st = Stencil{};
        st.id = id;
        if (id == kStencil5) {
            // 4 u(m) - (sum of the four neighbours), eq. (1.2)
            st.a0 = 4; st.a1 = -2; st.b0 = 2; st.b1 = 0; st.w = 1;
            st.C = kEulerGamma + 0.5 * std::log(8.0);
            st.c[0][1] = 1.0 / (24.0 * kPi);
            st.c[1][1] = 18.0 / (480.0 * kPi);
            st.c[1][2] = 25.0 / (480.0 * kPi);
            d.table = build_phi_table(st, kPhiTableRadius);
            fit_far_field_k3(d);
        } else {
            // isotropic 9-point: (20 u(m) - 4 (four neighbours) - (four diagonal neighbours)) / 6
            st.a0 = 20; st.a1 = -8; st.b0 = 8; st.b1 = 4; st.w = 6;
            d.table = build_phi_table(st, kPhiTableRadius);
            fit_far_field(d);
        }
    });
    return data[id];
}

}  // namespace

const Stencil& stencil(int id) { return stencil_data(id).st; }

const std::vector<double>& phi_table(int id) { return stencil_data(id).table; }

double phi(int id, int64_t m1, int64_t m2) {
    int64_t a = std::llabs(m1), b = std::llabs(m2);
    if (b > a) std::swap(a, b);
    const StencilData& d = stencil_data(id);
    if (a <= kPhiTableRadius) return d.table[size_t(octant_index(a, b))];
    return phi_expansion(d.st, double(a), double(b));
}

}  // namespace lfmm
