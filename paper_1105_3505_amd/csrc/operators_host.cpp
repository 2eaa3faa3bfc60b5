// Skeletons and translation operators of the model boxes (Sections 5, 7 and 8.1).
//
// The kernel is translation invariant, so every box of one level shares the operators of
// a model box with its lower-left corner at the origin (Section 8.1).  For a box of side s:
//
// * Proxy ring F: lattice points on the boundary of the concentric box of side 3s, i.e. of
//   [-s, 2s-1]^2.  A potential that is discrete-harmonic outside that square and decays is
//   bounded there by its values on F (discrete maximum principle), so matching on F matches
//   every well-separated target (Section 4.2 definition, Section 5).
// * Leaf: the candidate set Y is the box boundary.  For the 5-point operator every exterior
//   field of sources in the box is reproduced exactly by charges on the boundary nodes
//   (harmonic extension inside the box), so Y loses nothing and only the ID truncates.
//   A rank-revealing QR of A^{F,Y} picks the skeleton Yhat (Section 5).
// * T_ofs solves min || A^{F,box} - A^{F,Yhat} T || (eq. 5.1).  Small leaves store it for the
//   densely loaded model box and select columns per source (Remark 8.2); large leaves keep
//   the pseudo-inverse of A^{F,Yhat} and apply it to A^{F,tau} q on the fly.
// * Level above: candidates are the four shifted child skeletons; the ID gives the parent
//   skeleton and the interpolation matrix S, whose column blocks are T_ofo (Section 7).
// * Every ID and least-squares system carries one extra row of ones: the total charge.  It
//   keeps the equivalent charges' sum equal to the true sum, so the log|x| far field that a
//   non-zero box charge produces is represented exactly as well.
#include "host_math.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <stdexcept>

namespace lfmm {

std::vector<int64_t> box_boundary(int64_t s) {
    std::vector<int64_t> pts;
    for (int64_t y = 0; y < s; ++y)
        for (int64_t x = 0; x < s; ++x)
            if (x == 0 || y == 0 || x == s - 1 || y == s - 1) {
                pts.push_back(x);
                pts.push_back(y);
            }
    return pts;
}

std::vector<int64_t> proxy_ring(int64_t s, int per_edge) {
    const int64_t lo = -s, hi = 2 * s - 1, len = hi - lo;  // each edge: len points from a corner
    std::vector<int64_t> pts;
    int64_t n_edge = (4 * len <= 4 * int64_t(per_edge)) ? len : int64_t(per_edge);
    for (int e = 0; e < 4; ++e) {
        for (int64_t i = 0; i < n_edge; ++i) {
            int64_t t = (n_edge == len) ? i : int64_t(std::llround(double(i) * double(len) / double(n_edge)));
            int64_t x, y;
            switch (e) {
                case 0: x = lo + t; y = lo; break;   // bottom, left to right
                case 1: x = hi; y = lo + t; break;   // right, bottom to top
                case 2: x = hi - t; y = hi; break;   // top, right to left
                default: x = lo; y = hi - t; break;  // left, top to bottom
            }
            pts.push_back(x);
            pts.push_back(y);
        }
    }
    return pts;
}

namespace {

// [phi(F_i - Y_j)] with a trailing row of ones (the charge sum)
Mat kernel_matrix_with_charge(int stencil_id, const std::vector<int64_t>& F, const std::vector<int64_t>& Y) {
    const int nf = int(F.size() / 2), ny = int(Y.size() / 2);
    Mat A(nf + 1, ny);
    for (int j = 0; j < ny; ++j) {
        for (int i = 0; i < nf; ++i) A(i, j) = phi(stencil_id, F[2 * i] - Y[2 * j], F[2 * i + 1] - Y[2 * j + 1]);
        A(nf, j) = 1.0;
    }
    return A;
}

Mat columns(const Mat& A, const std::vector<int>& idx) {
    Mat B(A.rows, int(idx.size()));
    for (size_t j = 0; j < idx.size(); ++j)
        for (int i = 0; i < A.rows; ++i) B(i, int(j)) = A(i, idx[j]);
    return B;
}

}  // namespace

OperatorSet build_operators_uncached(int64_t leaf_side, int nlevels, const OperatorParams& p) {
    auto t0 = std::chrono::steady_clock::now();
    if (leaf_side < 1 || nlevels < 1) throw std::runtime_error("build_operators: bad sizes");
    OperatorSet ops;
    ops.eps = p.eps;
    ops.leaf_side = leaf_side;
    ops.nlevels = nlevels;
    ops.level.resize(size_t(nlevels));

    // ---- leaf level ------------------------------------------------------------------
    {
        const int64_t s = leaf_side;
        std::vector<int64_t> Y = box_boundary(s);
        std::vector<int64_t> F = proxy_ring(s, p.proxy_per_edge);
        Mat A = kernel_matrix_with_charge(p.stencil, F, Y);
        IDResult id = interpolative_decomposition(A, p.eps, p.max_rank);
        LevelOps& L0 = ops.level[0];
        L0.side = s;
        L0.rank = int(id.skel.size());
        for (int j : id.skel) {
            L0.skel.push_back(Y[2 * size_t(j)]);
            L0.skel.push_back(Y[2 * size_t(j) + 1]);
        }
        Mat Ask = columns(A, id.skel);
        LeafOps& lf = ops.leaf;
        lf.side = s;
        lf.proxy = F;
        if (s <= p.dense_leaf_max) {
            lf.dense = true;
            std::vector<int64_t> cells;
            for (int64_t y = 0; y < s; ++y)
                for (int64_t x = 0; x < s; ++x) {
                    cells.push_back(x);
                    cells.push_back(y);
                }
            Mat B = kernel_matrix_with_charge(p.stencil, F, cells);
            lf.T = least_squares(Ask, B);
        } else {
            lf.dense = false;
            Mat I(Ask.rows, Ask.rows);
            for (int i = 0; i < Ask.rows; ++i) I(i, i) = 1.0;
            lf.Pi = least_squares(Ask, I);
        }
    }

    // ---- coarser levels ----------------------------------------------------------------
    for (int h = 1; h < nlevels; ++h) {
        const LevelOps& ch = ops.level[size_t(h - 1)];
        LevelOps& L = ops.level[size_t(h)];
        L.side = ch.side * 2;
        const int64_t half = ch.side;
        std::vector<int64_t> Y;
        for (int c = 0; c < 4; ++c) {
            int64_t ox = (c & 1) ? half : 0, oy = (c & 2) ? half : 0;
            for (int q = 0; q < ch.rank; ++q) {
                Y.push_back(ch.skel[2 * size_t(q)] + ox);
                Y.push_back(ch.skel[2 * size_t(q) + 1] + oy);
            }
        }
        std::vector<int64_t> F = proxy_ring(L.side, p.proxy_per_edge);
        Mat A = kernel_matrix_with_charge(p.stencil, F, Y);
        IDResult id = interpolative_decomposition(A, p.eps, p.max_rank);
        L.rank = int(id.skel.size());
        for (int j : id.skel) {
            L.skel.push_back(Y[2 * size_t(j)]);
            L.skel.push_back(Y[2 * size_t(j) + 1]);
        }
        for (int c = 0; c < 4; ++c) {
            L.ofo[c] = Mat(L.rank, ch.rank);
            for (int q = 0; q < ch.rank; ++q)
                for (int r = 0; r < L.rank; ++r) L.ofo[c](r, q) = id.S(r, c * ch.rank + q);
        }
    }
    ops.max_rank = 0;
    for (auto& L : ops.level) ops.max_rank = std::max(ops.max_rank, L.rank);
    ops.build_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return ops;
}

}  // namespace lfmm
