/*
 * ORACLE (test infrastructure only) -- direct evaluation of the lattice convolution.
 *
 * Only the tests, the smoke check and the CPU-baseline leg of the benchmark may load this
 * code.  It shares nothing with the GPU library.
 *
 * Computes, for every target t,   u(t) = sum over sources s of phi(t - s) f(s),
 * the finite form of eq. (1.7) (Section 1), term by term in source order, with
 * Neumaier-compensated summation.  phi comes from a caller-supplied octant table
 * (phi(a,b), 0 <= b <= a <= radius, built by the quadrature of Section 3.2) and, for
 * offsets with |m|_inf > radius, from the truncated asymptotic expansion eq. (3.1) with the
 * true Euler constant -- the 5-point operator's expansion, used only when the caller says so
 * (expansion != 0); otherwise such an offset gives NaN (the tables of other operators have
 * no expansion here).  phi(0) = 0, so a target on a source gets no self term (eq. 2.2).
 *
 * Build: gcc -O2 -fopenmp -shared -fPIC direct.c -o _direct.so -lm   (no fast-math)
 */
#include <math.h>
#include <stdint.h>
#include <omp.h>

static const double kPi = 3.14159265358979323846;
static const double kEulerGamma = 0.57721566490153286061;

/* eq. (3.1) truncated after the |m|^-8 term; (a, b) != (0, 0). */
static double phi_expansion(double a, double b)
{
    double r2 = a * a + b * b;
    double c = a * a / r2, s = b * b / r2;
    double lead = -(0.5 * log(r2) + kEulerGamma + 0.5 * log(8.0)) / (2.0 * kPi);
    double t4 = (c * c - 6.0 * c * s + s * s) / (24.0 * kPi * r2);
    double t8 = (43.0 * c * c * c * c - 772.0 * c * c * c * s + 1570.0 * c * c * s * s
                 - 772.0 * c * s * s * s + 43.0 * s * s * s * s) / (480.0 * kPi * r2 * r2);
    return lead + t4 + t8;
}

static double phi_at(int64_t dx, int64_t dy, const double *table, int64_t radius, int64_t expansion)
{
    int64_t a = dx < 0 ? -dx : dx;
    int64_t b = dy < 0 ? -dy : dy;
    if (b > a) { int64_t t = a; a = b; b = t; }
    if (a <= radius) return table[a * (a + 1) / 2 + b];
    return expansion ? phi_expansion((double)a, (double)b) : NAN;
}

int oracle_threads(void) { return omp_get_max_threads(); }

void oracle_phi(int64_t n, const int32_t *mxy, const double *table, int64_t radius, int64_t expansion,
                double *out)
{
    for (int64_t i = 0; i < n; ++i) out[i] = phi_at(mxy[2 * i], mxy[2 * i + 1], table, radius, expansion);
}

void oracle_direct_sum(int64_t nt, const int32_t *txy, int64_t ns, const int32_t *sxy,
                       const double *f, const double *table, int64_t radius, int64_t expansion, double *u)
{
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t i = 0; i < nt; ++i) {
        const int64_t tx = txy[2 * i], ty = txy[2 * i + 1];
        double sum = 0.0, comp = 0.0;
        for (int64_t j = 0; j < ns; ++j) {
            double term = phi_at(tx - (int64_t)sxy[2 * j], ty - (int64_t)sxy[2 * j + 1], table, radius, expansion) * f[j];
            double t = sum + term;
            if (fabs(sum) >= fabs(term)) comp += (sum - t) + term;
            else comp += (term - t) + sum;
            sum = t;
        }
        u[i] = sum + comp;
    }
}
