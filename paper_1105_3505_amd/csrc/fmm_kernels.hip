// Evaluation passes of the lattice FMM on gfx950 (Section 8.2).
//
// Expansions are stored box-major: box g owns kRankPad consecutive FP64 coefficients in Q
// (outgoing, q-hat) and U (incoming, u-hat).  Boxes of every level are numbered
// consecutively level by level, each level in Morton order; leaves are the last level.
//
//   P2M   q^tau   = T_ofs^tau q(J^tau)             one wave per leaf, lanes = skeleton index
//   M2M   q^tau   = sum_c T_ofo^(c) q^child_c      one wave per parent
//   M2L   u^tau   = sum_{sigma in L_int} T_ifo^d q^sigma   FP64 MFMA, 16 boxes per wave
//   L2L   u^child += T_ofo^(c)T u^tau              one wave per child
//   L2P + near field + un-permutation              one wave per leaf, lanes = targets
#include "kernels.h"

#include <hip/hip_runtime.h>

namespace lfmm {

namespace {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;
constexpr int kOctRadius = 128;
constexpr double kPi = 3.14159265358979323846;
constexpr double kEulerGamma = 0.57721566490153286061;

typedef double double4_t __attribute__((ext_vector_type(4)));

// Interaction-list slot k of a box in child position c lies at offset slot c_dslot[c][k]
// of the 7 x 7 offset grid; the order matches the list builder (dy outer, dx inner).
struct DSlots { int8_t s[4][kNumInteractions]; };
__constant__ DSlots c_dslot;

__device__ inline uint32_t compact_bits(uint64_t x) {
    x &= 0x5555555555555555ull;
    x = (x | (x >> 1)) & 0x3333333333333333ull;
    x = (x | (x >> 2)) & 0x0F0F0F0F0F0F0F0Full;
    x = (x | (x >> 4)) & 0x00FF00FF00FF00FFull;
    x = (x | (x >> 8)) & 0x0000FFFF0000FFFFull;
    x = (x | (x >> 16)) & 0x00000000FFFFFFFFull;
    return uint32_t(x);
}

// eq. (3.1), truncated after the |m|^-8 term, true Euler constant; (a, b) != 0
__device__ inline double phi_expansion_dev(double a, double b) {
    double r2 = a * a + b * b;
    double ir2 = 1.0 / r2;
    double c = a * a * ir2, s = b * b * ir2;
    double lead = -(0.5 * log(r2) + (kEulerGamma + 0.5 * 2.0794415416798357)) * (1.0 / (2.0 * kPi));
    double t4 = (c * c - 6.0 * c * s + s * s) * ir2 * (1.0 / (24.0 * kPi));
    double c2 = c * c, s2 = s * s;
    double t8 = (43.0 * c2 * c2 - 772.0 * c2 * c * s + 1570.0 * c2 * s2 - 772.0 * c * s2 * s + 43.0 * s2 * s2)
                * ir2 * ir2 * (1.0 / (480.0 * kPi));
    return lead + t4 + t8;
}

// phi at offset (a, b), a, b >= 0: octant table inside radius 128, expansion outside
__device__ inline double phi_oct(int a, int b, const double* oct) {
    int hi = max(a, b), lo = min(a, b);
    if (hi <= kOctRadius) return oct[hi * (hi + 1) / 2 + lo];
    return phi_expansion_dev(double(hi), double(lo));
}

__global__ void k_gather_f(const double* f, const int32_t* perm, int64_t n, double* fs) {
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) fs[i] = f[perm[i]];
}

template <int P>
__global__ __launch_bounds__(kBlock) void k_p2m_dense(int64_t nleaves, int32_t leaf_off, const int32_t* box_pt0,
                                                       const int32_t* box_pt1, const uint64_t* box_key, int64_t side,
                                                       const int2* pts, const double* fs, const double* leafT,
                                                       double* Q) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    int64_t leaf = int64_t(blockIdx.x) * kWaves + wave;
    if (leaf >= nleaves) return;
    const int32_t g = leaf_off + int32_t(leaf);
    const int32_t p0 = box_pt0[g], p1 = box_pt1[g];
    const uint64_t key = box_key[g];
    const int32_t cx = int32_t(compact_bits(key) * side), cy = int32_t(compact_bits(key >> 1) * side);
    double acc = 0.0;
    const int l = lane < P ? lane : 0;
    for (int32_t j = p0; j < p1; ++j) {
        int2 p = pts[j];
        int64_t loc = int64_t(p.x - cx) + side * int64_t(p.y - cy);
        acc += leafT[loc * P + l] * fs[j];
    }
    if (lane < P) Q[size_t(g) * P + lane] = acc;
}

template <int P>
__global__ __launch_bounds__(kBlock) void k_m2m(int32_t begin, int32_t end, int height, const int32_t* box_child,
                                                 const double* ofo_cm, double* Q) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int32_t g = begin + int32_t(blockIdx.x) * kWaves + wave;
    if (g >= end) return;
    const int l = lane < P ? lane : 0;
    double acc = 0.0;
    for (int c = 0; c < 4; ++c) {
        const int32_t ch = box_child[size_t(g) * 4 + c];
        if (ch < 0) continue;
        const double* T = ofo_cm + (size_t(height) * 4 + c) * P * P;   // [q][r]
        const double* qc = Q + size_t(ch) * P;
        #pragma unroll 8
        for (int q = 0; q < P; ++q) acc += T[q * P + l] * qc[q];
    }
    if (lane < P) Q[size_t(g) * P + lane] = acc;
}

template <int P>
__global__ __launch_bounds__(kBlock) void k_l2l(int32_t begin, int32_t end, int height_parent,
                                                 const int32_t* box_parent, const uint64_t* box_key,
                                                 const double* ofo_rm, double* U) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int32_t g = begin + int32_t(blockIdx.x) * kWaves + wave;
    if (g >= end) return;
    const int l = lane < P ? lane : 0;
    const int32_t par = box_parent[g];
    const int c = int(box_key[g] & 3ull);
    const double* T = ofo_rm + (size_t(height_parent) * 4 + c) * P * P;   // [r][q]
    const double* up = U + size_t(par) * P;
    double acc = U[size_t(g) * P + l];
    #pragma unroll 8
    for (int r = 0; r < P; ++r) acc += T[r * P + l] * up[r];
    if (lane < P) U[size_t(g) * P + lane] = acc;
}

// M2L on the FP64 matrix cores.  A wave owns a tile of up to 16 target boxes sharing a
// level and a child position, so all 16 share the 27 operators T_ifo^d.  For each list
// slot k: C[p][box] += sum_q T^d[p][q] Q[src_k(box)][q], as 16x16x4 MFMA steps.  In step kk
// lane group g (= lane / 16) contributes column q = g * P/4 + kk, so each lane's operands
// for one slot are P/4 consecutive doubles of a row of T^d and of the source's Q.
// Accumulator element i of lane (g, n) is row 4 g + i, column n of the 16 x 16 block.
template <int P>
__global__ __launch_bounds__(kBlock) void k_m2l(const M2LTile* tiles, const int32_t* ntiles_p,
                                                 const int32_t* cls_box, const int32_t* ilist, int32_t ilist_off,
                                                 const double* Q, double* U, const double* ifo) {
    constexpr int MT = P / 16, KQ = P / 4;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int n = lane & 15, g = lane >> 4;
    const int32_t ntiles = *ntiles_p;
    for (int32_t t = int32_t(blockIdx.x) * kWaves + wave; t < ntiles; t += int32_t(gridDim.x) * kWaves) {
        const M2LTile tl = tiles[t];
        const int32_t box = (n < tl.count) ? cls_box[tl.start + n] : -1;
        const int32_t* il = ilist + size_t(box >= 0 ? box - ilist_off : 0) * kNumInteractions;
        double4_t acc[MT];
        #pragma unroll
        for (int m = 0; m < MT; ++m) acc[m] = double4_t{0.0, 0.0, 0.0, 0.0};
        for (int k = 0; k < kNumInteractions; ++k) {
            const int d = c_dslot.s[tl.cls][k];
            const int32_t src = (box >= 0) ? il[k] : -1;
            double b[KQ];
            if (src >= 0) {
                const double* qs = Q + size_t(src) * P + g * KQ;
                #pragma unroll
                for (int kk = 0; kk < KQ; ++kk) b[kk] = qs[kk];
            } else {
                #pragma unroll
                for (int kk = 0; kk < KQ; ++kk) b[kk] = 0.0;
            }
            const double* T = ifo + (size_t(tl.height) * kNumIfoSlots + d) * P * P;
            #pragma unroll
            for (int m = 0; m < MT; ++m) {
                const double* a = T + size_t(16 * m + n) * P + g * KQ;
                #pragma unroll
                for (int kk = 0; kk < KQ; ++kk)
                    acc[m] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[kk], b[kk], acc[m], 0, 0, 0);
            }
        }
        if (box >= 0) {
            double* ub = U + size_t(box) * P;
            #pragma unroll
            for (int m = 0; m < MT; ++m) {
                #pragma unroll
                for (int i = 0; i < 4; ++i) ub[16 * m + 4 * g + i] = acc[m][i];
            }
        }
    }
}

// Mixed-precision M2L: the same products on the FP32 matrix cores.  T_ifo and q-hat are split
// into FP32 hi + lo parts; each 16x16x4 step forms T_hi q_hi in one FP32 accumulator and
// T_hi q_lo + T_lo q_hi in another (the cross terms are ~2^-24 of the first and would be
// rounded away if added to it), and both are flushed into FP64 accumulators after every
// step, so FP32 rounding acts on four-term partial sums only.  u-hat is stored in FP64.
typedef float float4_t __attribute__((ext_vector_type(4)));

template <int P>
__global__ __launch_bounds__(kBlock) void k_m2l_mixed(const M2LTile* tiles, const int32_t* ntiles_p,
                                                       const int32_t* cls_box, const int32_t* ilist,
                                                       int32_t ilist_off, const double* Q, double* U,
                                                       const float* ifo_hi, const float* ifo_lo) {
    constexpr int MT = P / 16, KQ = P / 4;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int n = lane & 15, g = lane >> 4;
    const int32_t ntiles = *ntiles_p;
    const float4_t zero = {0.f, 0.f, 0.f, 0.f};
    for (int32_t t = int32_t(blockIdx.x) * kWaves + wave; t < ntiles; t += int32_t(gridDim.x) * kWaves) {
        const M2LTile tl = tiles[t];
        const int32_t box = (n < tl.count) ? cls_box[tl.start + n] : -1;
        const int32_t* il = ilist + size_t(box >= 0 ? box - ilist_off : 0) * kNumInteractions;
        double4_t acc[MT];
        #pragma unroll
        for (int m = 0; m < MT; ++m) acc[m] = double4_t{0.0, 0.0, 0.0, 0.0};
        for (int k = 0; k < kNumInteractions; ++k) {
            const int d = c_dslot.s[tl.cls][k];
            const int32_t src = (box >= 0) ? il[k] : -1;
            float bh[KQ], bl[KQ];
            #pragma unroll
            for (int kk = 0; kk < KQ; ++kk) {
                const double q = (src >= 0) ? Q[size_t(src) * P + g * KQ + kk] : 0.0;
                bh[kk] = float(q);
                bl[kk] = float(q - double(bh[kk]));
            }
            const size_t base = (size_t(tl.height) * kNumIfoSlots + d) * P * P;
            #pragma unroll
            for (int m = 0; m < MT; ++m) {
                const float* ah = ifo_hi + base + size_t(16 * m + n) * P + g * KQ;
                const float* al = ifo_lo + base + size_t(16 * m + n) * P + g * KQ;
                #pragma unroll
                for (int kk = 0; kk < KQ; ++kk) {
                    float4_t main = __builtin_amdgcn_mfma_f32_16x16x4f32(ah[kk], bh[kk], zero, 0, 0, 0);
                    float4_t cross = __builtin_amdgcn_mfma_f32_16x16x4f32(ah[kk], bl[kk], zero, 0, 0, 0);
                    cross = __builtin_amdgcn_mfma_f32_16x16x4f32(al[kk], bh[kk], cross, 0, 0, 0);
                    #pragma unroll
                    for (int i = 0; i < 4; ++i) acc[m][i] += double(main[i]) + double(cross[i]);
                }
            }
        }
        if (box >= 0) {
            double* ub = U + size_t(box) * P;
            #pragma unroll
            for (int m = 0; m < MT; ++m) {
                #pragma unroll
                for (int i = 0; i < 4; ++i) ub[16 * m + 4 * g + i] = acc[m][i];
            }
        }
    }
}

// Leaf pass: for every point of a leaf (lanes = targets), the far field T_tfi u-hat with
// T_tfi = T_ofs^T (Section 7, symmetric kernel and targets = sources), plus the direct sum
// over the points of the leaf and its neighbors (Section 8.2 step 5), written back in the
// caller's point order.  QUAD: every near offset lies in a W x W quadrant table in LDS;
// otherwise the octant table of radius 128 sits in LDS and larger offsets use eq. (3.1).
template <int P, bool QUAD>
__global__ __launch_bounds__(kBlock) void k_leaf_eval(int64_t nleaves, int32_t leaf_off, const int32_t* box_pt0,
                                                       const int32_t* box_pt1, const uint64_t* box_key,
                                                       const int32_t* nlist, int64_t side, int W, const int2* pts,
                                                       const double* fs, const int32_t* perm, const double* U,
                                                       const double* leafT, int far, const double* phi_oct_tab,
                                                       double* u) {
    extern __shared__ double tab[];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    if (QUAD) {
        for (int i = tid; i < W * W; i += kBlock) {
            int dy = i / W, dx = i - dy * W;
            int hi = max(dx, dy), lo = min(dx, dy);
            tab[i] = phi_oct_tab[hi * (hi + 1) / 2 + lo];
        }
        __syncthreads();
    }
    for (int64_t leaf = int64_t(blockIdx.x) * kWaves + wave; leaf < nleaves; leaf += int64_t(gridDim.x) * kWaves) {
        const int32_t g = leaf_off + int32_t(leaf);
        const int32_t p0 = box_pt0[g], p1 = box_pt1[g];
        const uint64_t key = box_key[g];
        const int32_t cx = int32_t(compact_bits(key) * side), cy = int32_t(compact_bits(key >> 1) * side);
        const int32_t* nl = nlist + size_t(leaf) * 9;
        for (int32_t i0 = p0; i0 < p1; i0 += 64) {
            const int32_t i = i0 + lane;
            const bool valid = i < p1;
            const int2 pi = pts[valid ? i : p0];
            double acc = 0.0;
            for (int q = 0; q < 9; ++q) {
                const int32_t nb = nl[q];
                if (nb < 0) continue;
                const int32_t s0 = box_pt0[nb], s1 = box_pt1[nb];
                for (int32_t j = s0; j < s1; ++j) {
                    const int2 pj = pts[j];
                    const int dx = abs(pi.x - pj.x), dy = abs(pi.y - pj.y);
                    double ph;
                    if (QUAD) {
                        ph = tab[dy * W + dx];
                    } else {
                        ph = phi_oct(dx, dy, phi_oct_tab);
                    }
                    acc += ph * fs[j];
                }
            }
            if (far) {
                const int64_t loc = int64_t(pi.x - cx) + side * int64_t(pi.y - cy);
                const double* tl = leafT + loc * P;
                const double* uh = U + size_t(g) * P;
                #pragma unroll 8
                for (int p = 0; p < P; ++p) acc += tl[p] * uh[p];
            }
            if (valid) u[perm[i]] = acc;
        }
    }
}

// Brute-force sum over all sources for blocks of 256 targets; sources staged through LDS.
__global__ __launch_bounds__(kBlock) void k_direct(int64_t nt, const int2* txy, int64_t ns, const int2* sxy,
                                                    const double* f, const double* phi_oct, double* u) {
    __shared__ int2 sp[kBlock];
    __shared__ double sf[kBlock];
    const int64_t t = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    const bool valid = t < nt;
    const int2 pt = valid ? txy[t] : make_int2(0, 0);
    double acc = 0.0;
    for (int64_t j0 = 0; j0 < ns; j0 += kBlock) {
        const int64_t j = j0 + threadIdx.x;
        if (j < ns) {
            sp[threadIdx.x] = sxy[j];
            sf[threadIdx.x] = f[j];
        }
        __syncthreads();
        const int cnt = int(min<int64_t>(kBlock, ns - j0));
        for (int k = 0; k < cnt; ++k) {
            int64_t dx = int64_t(pt.x) - sp[k].x, dy = int64_t(pt.y) - sp[k].y;
            dx = dx < 0 ? -dx : dx;
            dy = dy < 0 ? -dy : dy;
            const int64_t hi = dx > dy ? dx : dy, lo = dx > dy ? dy : dx;
            double ph;
            if (hi <= kOctRadius) ph = phi_oct[hi * (hi + 1) / 2 + lo];
            else ph = phi_expansion_dev(double(hi), double(lo));
            acc += ph * sf[k];
        }
        __syncthreads();
    }
    if (valid) u[t] = acc;
}

inline unsigned grid_for(int64_t n, int per_block = kBlock) {
    int64_t g = (n + per_block - 1) / per_block;
    return unsigned(g < 1 ? 1 : g);
}

}  // namespace

hipError_t upload_dslots() {
    DSlots ds{};
    for (int c = 0; c < 4; ++c) {
        int cx = c & 1, cy = c >> 1, k = 0;
        for (int dy = -2 - cy; dy <= 3 - cy; ++dy)
            for (int dx = -2 - cx; dx <= 3 - cx; ++dx) {
                if (dx >= -1 && dx <= 1 && dy >= -1 && dy <= 1) continue;
                ds.s[c][k++] = int8_t((dy + 3) * 7 + (dx + 3));
            }
    }
    // synchronous copy, then read back: the table steers every M2L product
    hipError_t e = hipMemcpyToSymbol(HIP_SYMBOL(c_dslot), &ds, sizeof(ds), 0, hipMemcpyHostToDevice);
    if (e != hipSuccess) return e;
    DSlots back{};
    e = hipMemcpyFromSymbol(&back, HIP_SYMBOL(c_dslot), sizeof(back), 0, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return e;
    for (int c = 0; c < 4; ++c)
        for (int k = 0; k < kNumInteractions; ++k)
            if (back.s[c][k] != ds.s[c][k]) return hipErrorInvalidValue;
    return hipSuccess;
}

void launch_gather_f(const double* f, const int32_t* perm, int64_t n, double* fs, hipStream_t st) {
    hipLaunchKernelGGL(k_gather_f, dim3(grid_for(n)), dim3(kBlock), 0, st, f, perm, n, fs);
}

void launch_p2m_dense(int64_t nleaves, int32_t leaf_off, const int32_t* box_pt0, const int32_t* box_pt1,
                      const uint64_t* box_key, int L, int64_t side, const int32_t* pts, const double* fs,
                      const double* leafT, double* Q, hipStream_t st) {
    (void)L;
    if (nleaves <= 0) return;
    hipLaunchKernelGGL(k_p2m_dense<kRankPad>, dim3(grid_for(nleaves, kWaves)), dim3(kBlock), 0, st, nleaves,
                       leaf_off, box_pt0, box_pt1, box_key, side, reinterpret_cast<const int2*>(pts), fs, leafT, Q);
}

void launch_m2m(int32_t box_begin, int32_t box_end, int height, const int32_t* box_child, const double* ofo_cm,
                const double* Q_in, double* Q_out, hipStream_t st) {
    (void)Q_in;
    if (box_end <= box_begin) return;
    hipLaunchKernelGGL(k_m2m<kRankPad>, dim3(grid_for(box_end - box_begin, kWaves)), dim3(kBlock), 0, st, box_begin,
                       box_end, height, box_child, ofo_cm, Q_out);
}

void launch_l2l(int32_t box_begin, int32_t box_end, int height_parent, const int32_t* box_parent,
                const uint64_t* box_key, const double* ofo_rm, double* U, hipStream_t st) {
    if (box_end <= box_begin) return;
    hipLaunchKernelGGL(k_l2l<kRankPad>, dim3(grid_for(box_end - box_begin, kWaves)), dim3(kBlock), 0, st, box_begin,
                       box_end, height_parent, box_parent, box_key, ofo_rm, U);
}

void launch_m2l(const M2LTile* tiles, const int32_t* ntiles, int32_t max_tiles, const int32_t* cls_box,
                const int32_t* ilist, int32_t ilist_off, const double* Q, double* U, const double* ifo,
                hipStream_t st) {
    if (max_tiles <= 0) return;
    unsigned g = grid_for(max_tiles, kWaves);
    if (g > 2048) g = 2048;
    hipLaunchKernelGGL(k_m2l<kRankPad>, dim3(g), dim3(kBlock), 0, st, tiles, ntiles, cls_box, ilist, ilist_off, Q, U,
                       ifo);
}

void launch_m2l_mixed(const M2LTile* tiles, const int32_t* ntiles, int32_t max_tiles, const int32_t* cls_box,
                      const int32_t* ilist, int32_t ilist_off, const double* Q, double* U, const float* ifo_hi,
                      const float* ifo_lo, hipStream_t st) {
    if (max_tiles <= 0) return;
    unsigned g = grid_for(max_tiles, kWaves);
    if (g > 2048) g = 2048;
    hipLaunchKernelGGL(k_m2l_mixed<kRankPad>, dim3(g), dim3(kBlock), 0, st, tiles, ntiles, cls_box, ilist, ilist_off,
                       Q, U, ifo_hi, ifo_lo);
}

void launch_leaf_eval(int64_t nleaves, int32_t leaf_off, const int32_t* box_pt0, const int32_t* box_pt1,
                      const uint64_t* box_key, const int32_t* nlist, int L, int64_t side, const int32_t* pts,
                      const double* fs, const int32_t* perm, const double* U, const double* leafT, bool far,
                      const double* phi_oct, double* u, hipStream_t st) {
    (void)L;
    if (nleaves <= 0) return;
    unsigned g = grid_for(nleaves, kWaves);
    if (g > 4096) g = 4096;
    const int W = int(2 * side);
    if (2 * side <= 64) {
        size_t lds = size_t(W) * W * sizeof(double);
        hipLaunchKernelGGL((k_leaf_eval<kRankPad, true>), dim3(g), dim3(kBlock), lds, st, nleaves, leaf_off, box_pt0,
                           box_pt1, box_key, nlist, side, W, reinterpret_cast<const int2*>(pts), fs, perm, U, leafT,
                           far ? 1 : 0, phi_oct, u);
    } else {
        hipLaunchKernelGGL((k_leaf_eval<kRankPad, false>), dim3(g), dim3(kBlock), 0, st, nleaves, leaf_off,
                           box_pt0, box_pt1, box_key, nlist, side, W, reinterpret_cast<const int2*>(pts), fs, perm, U,
                           leafT, far ? 1 : 0, phi_oct, u);
    }
}

void launch_direct(int64_t nt, const int32_t* txy, int64_t ns, const int32_t* sxy, const double* f,
                   const double* phi_oct, double* u, hipStream_t st) {
    if (nt <= 0) return;
    hipLaunchKernelGGL(k_direct, dim3(grid_for(nt)), dim3(kBlock), 0, st, nt, reinterpret_cast<const int2*>(txy), ns,
                       reinterpret_cast<const int2*>(sxy), f, phi_oct, u);
}

}  // namespace lfmm
