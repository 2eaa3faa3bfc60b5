// Dense FP64 factorizations for the operator precompute: Householder QR with column
// pivoting (Businger-Golub) for the interpolative decomposition that picks skeletons
// (Section 5: rank-revealing QR of A^{F,Y}), and Householder least squares for the
// outgoing-from-sources operator (eq. 5.1).  Sizes are a few hundred, so clarity wins
// over blocking.
#include "host_math.h"

#include <algorithm>
#include <cmath>
#include <stdexcept>

namespace lfmm {
namespace {

// Householder vector for x (length n): returns beta and overwrites x with v (v[0] = 1
// implied by storing it), so that (I - beta v v^T) x = alpha e1.  Returns alpha.
double householder(double* x, int n, double& beta) {
    double sigma = 0.0;
    for (int i = 1; i < n; ++i) sigma += x[i] * x[i];
    double x0 = x[0];
    if (sigma == 0.0) {
        beta = 0.0;
        return x0;
    }
    double mu = std::sqrt(x0 * x0 + sigma);
    double v0 = (x0 <= 0.0) ? (x0 - mu) : (-sigma / (x0 + mu));
    beta = 2.0 * v0 * v0 / (sigma + v0 * v0);
    for (int i = 1; i < n; ++i) x[i] /= v0;
    x[0] = 1.0;
    return mu;
}

void apply_householder(const double* v, int n, double beta, double* y) {
    if (beta == 0.0) return;
    double d = 0.0;
    for (int i = 0; i < n; ++i) d += v[i] * y[i];
    d *= beta;
    for (int i = 0; i < n; ++i) y[i] -= d * v[i];
}

// Solve R x = b in place for the leading k x k upper triangle of a column-major m-row R.
void back_substitute(const Mat& R, int k, double* b) {
    for (int i = k - 1; i >= 0; --i) {
        double s = b[i];
        for (int j = i + 1; j < k; ++j) s -= R(i, j) * b[j];
        b[i] = s / R(i, i);
    }
}

}  // namespace

IDResult interpolative_decomposition(const Mat& A0, double tol, int max_rank) {
    Mat A = A0;
    const int m = A.rows, n = A.cols;
    std::vector<int> perm(static_cast<size_t>(n));
    for (int j = 0; j < n; ++j) perm[size_t(j)] = j;
    std::vector<double> betas;
    const int kmax = std::min({m, n, max_rank});
    double first = -1.0;
    int k = 0;
    for (; k < kmax; ++k) {
        // exact remaining column norms (no downdating; sizes are small)
        int best = -1;
        double bestn = -1.0;
        for (int j = k; j < n; ++j) {
            double s = 0.0;
            for (int i = k; i < m; ++i) s += A(i, j) * A(i, j);
            if (s > bestn) {
                bestn = s;
                best = j;
            }
        }
        double nrm = std::sqrt(bestn);
        if (first < 0.0) first = nrm;
        if (nrm <= tol * first || nrm == 0.0) break;
        if (best != k) {
            for (int i = 0; i < m; ++i) std::swap(A(i, k), A(i, best));
            std::swap(perm[size_t(k)], perm[size_t(best)]);
        }
        double beta;
        double alpha = householder(&A(k, k), m - k, beta);
        std::vector<double> v(&A(k, k), &A(k, k) + (m - k));
        for (int j = k + 1; j < n; ++j) apply_householder(v.data(), m - k, beta, &A(k, j));
        A(k, k) = alpha;
        for (int i = k + 1; i < m; ++i) A(i, k) = 0.0;
        betas.push_back(beta);
    }
    IDResult r;
    r.skel.assign(perm.begin(), perm.begin() + k);
    r.S = Mat(k, n);
    // S(:, perm[j]) = e_j for j < k;  S(:, perm[j]) = R11^{-1} R12(:, j-k) otherwise
    for (int j = 0; j < n; ++j) {
        std::vector<double> col(size_t(k), 0.0);
        if (j < k) {
            col[size_t(j)] = 1.0;
        } else {
            for (int i = 0; i < k; ++i) col[size_t(i)] = A(i, j);
            back_substitute(A, k, col.data());
        }
        for (int i = 0; i < k; ++i) r.S(i, perm[size_t(j)]) = col[size_t(i)];
    }
    return r;
}

Mat least_squares(const Mat& A0, const Mat& B0) {
    Mat A = A0, B = B0;
    const int m = A.rows, n = A.cols;
    if (m < n || B.rows != m) throw std::runtime_error("least_squares: bad shapes");
    for (int k = 0; k < n; ++k) {
        double beta;
        double alpha = householder(&A(k, k), m - k, beta);
        std::vector<double> v(&A(k, k), &A(k, k) + (m - k));
        for (int j = k + 1; j < n; ++j) apply_householder(v.data(), m - k, beta, &A(k, j));
        for (int j = 0; j < B.cols; ++j) apply_householder(v.data(), m - k, beta, &B(k, j));
        A(k, k) = alpha;
        if (alpha == 0.0) throw std::runtime_error("least_squares: rank deficient");
    }
    Mat X(n, B.cols);
    std::vector<double> col(static_cast<size_t>(n));
    for (int j = 0; j < B.cols; ++j) {
        for (int i = 0; i < n; ++i) col[size_t(i)] = B(i, j);
        back_substitute(A, n, col.data());
        for (int i = 0; i < n; ++i) X(i, j) = col[size_t(i)];
    }
    return X;
}

}  // namespace lfmm
