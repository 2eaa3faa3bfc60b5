// Host-side numerics of the lattice FMM library: the lattice fundamental solution phi,
// dense FP64 linear algebra (pivoted QR, interpolative decomposition, least squares) and
// the per-level translation operators of the model boxes.  None of this runs on the GPU;
// it is the one-time precompute whose results the kernels read.
#pragma once

#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

namespace lfmm {

// ---------------------------------------------------------------------------------------
// phi: fundamental solution of a lattice operator, A phi = delta: the 5-point operator of
// eq. (1.2), or the isotropic 9-point operator (the method carries over to other
// constant-coefficient difference operators, Sections 1 and 3.1).
// ---------------------------------------------------------------------------------------

// Radius (infinity norm) of the tabulated octant; beyond it the far-field expansion holds
// to about 4e-15 (the terms of eq. (3.1) and fitted |m|^-6 terms).
constexpr int kPhiTableRadius = 128;

enum { kStencil5 = 0, kStencil9 = 1, kNumStencils = 2 };

// A D4-symmetric operator with zero row sum whose symbol is affine in cos t1:
// sigma(t) = (alpha(t2) - beta(t2) cos t1) / w, alpha = a0 + a1 cos t2, beta = b0 + b1 cos t2;
// and its far-field expansion phi ~ -(1/2pi)(log|m| + C) + sum_k |m|^-2k sum_j c[k-1][j] cos(4 j theta).
struct Stencil {
    int id = 0;
    double a0 = 0, a1 = 0, b0 = 0, b1 = 0, w = 1;
    double C = 0;
    double c[3][4] = {};
};

// The operator's data, its table built (and, for operators other than the 5-point one, its
// far-field coefficients fitted) on first use.
const Stencil& stencil(int id);

// bfloat16 (8 significant bits, FP32's exponent range): the bits of the value nearest to x,
// rounded to FP32 first and then to nearest-even (the two roundings can differ from one
// direct rounding by one unit in the last bit; the splits that use it take the remainder
// exactly, so that only changes how the value is shared between the parts), and the
// value of such bits.
inline uint16_t bf16_rne(double x) {
    const float f = float(x);
    uint32_t u;
    std::memcpy(&u, &f, 4);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return uint16_t(u >> 16);
}
inline double bf16_value(uint16_t b) {
    const uint32_t u = uint32_t(b) << 16;
    float f;
    std::memcpy(&f, &u, 4);
    return double(f);
}

inline int64_t octant_index(int64_t a, int64_t b) { return a * (a + 1) / 2 + b; }
inline int64_t octant_size(int64_t r) { return (r + 1) * (r + 2) / 2; }

// phi(m) by the one-dimensional integral obtained by integrating eq. (1.8) over t1
// analytically (remark closing Section 3), with 20-point Gauss-Legendre panels.
double phi_reduced_integral(const Stencil& st, int64_t m1, int64_t m2);

// The far-field expansion (for the 5-point operator eq. (3.1) with the true Euler constant and
// fitted |m|^-6 terms); (a, b) != 0.
double phi_expansion(const Stencil& st, double a, double b);

// Octant table phi(a, b), 0 <= b <= a <= radius, in octant_index order (multithreaded).
std::vector<double> build_phi_table(const Stencil& st, int radius);

// Process-wide table of radius kPhiTableRadius of operator id, built on first use.
const std::vector<double>& phi_table(int id);

// phi of operator id at an integer offset: table inside the radius, expansion outside.
double phi(int id, int64_t m1, int64_t m2);

// ---------------------------------------------------------------------------------------
// Dense column-major matrices and the factorizations the precompute needs.
// ---------------------------------------------------------------------------------------
struct Mat {
    int rows = 0, cols = 0;
    std::vector<double> a;  // column-major
    Mat() = default;
    Mat(int r, int c) : rows(r), cols(c), a(size_t(r) * size_t(c), 0.0) {}
    double& operator()(int i, int j) { return a[size_t(j) * rows + i]; }
    double operator()(int i, int j) const { return a[size_t(j) * rows + i]; }
};

// Interpolative decomposition by Householder QR with column pivoting: A ~ A(:, skel) * S,
// rank chosen as the number of pivots whose remaining column norm exceeds tol * (first
// pivot's norm), capped at max_rank.  S is rank x cols with the identity on the skeleton.
struct IDResult {
    std::vector<int> skel;  // indices of the skeleton columns, in pivot order
    Mat S;                  // interpolation matrix
};
IDResult interpolative_decomposition(const Mat& A, double tol, int max_rank);

// Least-squares solution X of min ||A X - B|| for a full-column-rank A (Householder QR).
Mat least_squares(const Mat& A, const Mat& B);

// ---------------------------------------------------------------------------------------
// Translation operators for the model box of every level (Sections 5, 7 and 8.1).
// ---------------------------------------------------------------------------------------
struct LevelOps {
    int64_t side = 0;            // box side in lattice units
    int rank = 0;                // number of skeleton points P
    std::vector<int64_t> skel;   // 2*rank lattice offsets from the box's lower-left corner
    // Children of the model box at this level, in child order c = (x bit) + 2 (y bit):
    // T_ofo^(c), rank x rank_child, column-major.  Empty at the leaf level.
    Mat ofo[4];
};

struct LeafOps {
    int64_t side = 0;
    bool dense = false;          // dense-model outgoing operator (small leaves)
    Mat T;                       // dense: rank x side^2, column j = local cell j = x + side*y
    Mat Pi;                      // proxy form: rank x (nproxy + 1); last column is the charge sum
    std::vector<int64_t> proxy;  // 2*nproxy lattice offsets of the proxy ring from the corner
};

struct OperatorSet {
    double eps = 0;
    int64_t leaf_side = 0;
    int nlevels = 0;             // heights h = 0 (leaf) .. nlevels-1
    int max_rank = 0;
    std::vector<LevelOps> level; // indexed by height above the leaf
    LeafOps leaf;
    double build_seconds = 0;
};

struct OperatorParams {
    int stencil = 0;             // lattice operator whose phi the operators sample
    double eps = 1e-12;          // ID tolerance, relative to the first pivot
    int proxy_per_edge = 64;     // proxy points per ring edge once the full ring is larger
    int max_rank = 64;           // skeleton cap (kernels store P_pad = 64 coefficients)
    int64_t dense_leaf_max = 32; // largest leaf side with a dense-model operator
};

// Builds leaf and level operators for leaves of side leaf_side and nlevels heights; with
// LFMM_CACHE_DIR set in the environment, through the on-disk cache of opcache_host.cpp.
OperatorSet build_operators(int64_t leaf_side, int nlevels, const OperatorParams& p);
OperatorSet build_operators_uncached(int64_t leaf_side, int nlevels, const OperatorParams& p);

// Proxy ring of a box of side s with lower-left corner at the origin: the lattice points
// on the boundary of the concentric box of side 3s, all of them when there are at most
// 4*per_edge, else per_edge evenly spaced points on each edge.
std::vector<int64_t> proxy_ring(int64_t s, int per_edge);

// Lattice points on the boundary of the box [0, s)^2 (all points when s <= 2).
std::vector<int64_t> box_boundary(int64_t s);

}  // namespace lfmm
