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

#include <algorithm>

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
// The FP64 16x16x4 instruction returns element i of lane (g, n) as row g + 4 i, column n
// of the 16 x 16 block (the FP32 16x16x4 one returns row 4 g + i).
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
                for (int i = 0; i < 4; ++i) ub[16 * m + g + 4 * i] = acc[m][i];
            }
        }
    }
}

// XCD-aware tile order: blocks are dispatched round-robin over the 8 XCDs (block b runs on
// XCD b % 8), so block b walks the b % 8-th contiguous eighth of the tile list; spatially
// close tiles, which share source expansions, then meet in the same L2.
__device__ inline int32_t xcd_tile(int32_t b, int32_t G, int32_t step, int32_t ntiles) {
    const int32_t x = b & 7, local = b >> 3, per = (G + 7 - x) >> 3;   // blocks on XCD x
    const int32_t chunk = (ntiles + 7) >> 3;
    const int32_t t = x * chunk + local + step * per;
    return (t < min(ntiles, (x + 1) * chunk)) ? t : -1;
}

// M2L with the 27 list slots of a 16-box tile split over the four waves of a block (slots
// k = wave, wave + 4, ...), partial products reduced through LDS in a fixed order, so the
// result is deterministic and a level with few boxes still gives every SIMD several waves.
template <int P>
__global__ __launch_bounds__(kBlock) void k_m2l_split(const M2LTile* tiles, const int32_t* ntiles_p,
                                                       const int32_t* cls_box, const int32_t* ilist,
                                                       int32_t ilist_off, const double* Q, double* U,
                                                       const double* ifo) {
    constexpr int MT = P / 16, KQ = P / 4;
    __shared__ double red[kWaves - 1][P][16];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int n = lane & 15, g = lane >> 4;
    const int32_t ntiles = *ntiles_p;
    const int32_t G = int32_t(gridDim.x);
    for (int32_t step = 0;; ++step) {
        const int32_t t = xcd_tile(int32_t(blockIdx.x), G, step, ntiles);
        if (t < 0) break;                                   // uniform over the block
        const M2LTile tl = tiles[t];
        const int32_t box = (n < tl.count) ? cls_box[tl.start + n] : -1;
        const int32_t* il = ilist + size_t(box >= 0 ? box - ilist_off : 0) * kNumInteractions;
        double4_t acc[MT];
        #pragma unroll
        for (int m = 0; m < MT; ++m) acc[m] = double4_t{0.0, 0.0, 0.0, 0.0};
        for (int k = wave; k < kNumInteractions; k += kWaves) {
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
        if (wave > 0) {
            #pragma unroll
            for (int m = 0; m < MT; ++m) {
                #pragma unroll
                for (int i = 0; i < 4; ++i) red[wave - 1][16 * m + g + 4 * i][n] = acc[m][i];
            }
        }
        __syncthreads();
        if (wave == 0 && box >= 0) {
            double* ub = U + size_t(box) * P;
            #pragma unroll
            for (int m = 0; m < MT; ++m) {
                #pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int r = 16 * m + g + 4 * i;   // FP64 output layout
                    double v = acc[m][i];
                    #pragma unroll
                    for (int w = 0; w < kWaves - 1; ++w) v += red[w][r][n];
                    ub[r] = v;
                }
            }
        }
        __syncthreads();
    }
}

// Mixed-precision M2L on the FP32 matrix cores.  Each operator is written T^d = c_d 1 1^T + R^d
// with c_d its mean entry: the constant part, which carries the large log|d| level of the
// kernel, is applied in FP64 as c_d times the source's charge sum; only the remainder R^d,
// several times smaller, goes through FP32.  R^d and q-hat are split into FP32 hi + lo parts;
// each 16x16x4 step forms R_hi q_hi in one FP32 accumulator and R_hi q_lo + R_lo q_hi in
// another (the cross terms are ~2^-24 of the first and would be rounded away if added to
// it), and both are flushed into FP64 accumulators after every step, so FP32 rounding acts on
// four-term partial sums only.  u-hat is stored in FP64.
typedef float float4_t __attribute__((ext_vector_type(4)));

template <int P>
__global__ __launch_bounds__(kBlock) void k_m2l_mixed(const M2LTile* tiles, const int32_t* ntiles_p,
                                                       const int32_t* cls_box, const int32_t* ilist,
                                                       int32_t ilist_off, const double* Q, double* U,
                                                       const float* ifo_hi, const float* ifo_lo,
                                                       const double* mono, const int32_t* rank) {
    constexpr int MT = P / 16, KQ = P / 4;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int n = lane & 15, g = lane >> 4;
    const int32_t ntiles = *ntiles_p;
    const float4_t zero = {0.f, 0.f, 0.f, 0.f};
    for (int32_t t = int32_t(blockIdx.x) * kWaves + wave; t < ntiles; t += int32_t(gridDim.x) * kWaves) {
        const M2LTile tl = tiles[t];
        const int32_t box = (n < tl.count) ? cls_box[tl.start + n] : -1;
        const int32_t* il = ilist + size_t(box >= 0 ? box - ilist_off : 0) * kNumInteractions;
        const int rk = rank[tl.height];
        double4_t acc[MT];
        #pragma unroll
        for (int m = 0; m < MT; ++m) acc[m] = double4_t{0.0, 0.0, 0.0, 0.0};
        for (int k = 0; k < kNumInteractions; ++k) {
            const int d = c_dslot.s[tl.cls][k];
            const int32_t src = (box >= 0) ? il[k] : -1;
            float bh[KQ], bl[KQ];
            double qsum = 0.0;
            #pragma unroll
            for (int kk = 0; kk < KQ; ++kk) {
                const double q = (src >= 0) ? Q[size_t(src) * P + g * KQ + kk] : 0.0;
                qsum += q;
                bh[kk] = float(q);
                bl[kk] = float(q - double(bh[kk]));
            }
            // charge sum of source column n: the four lane groups hold a quarter each
            qsum += __shfl_xor(qsum, 16, 64);
            qsum += __shfl_xor(qsum, 32, 64);
            const double cq = mono[size_t(tl.height) * kNumIfoSlots + d] * qsum;
            #pragma unroll
            for (int m = 0; m < MT; ++m) {
                #pragma unroll
                for (int i = 0; i < 4; ++i)
                    if (16 * m + 4 * g + i < rk) acc[m][i] += cq;   // padded rows stay zero
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

// Near field + L2P, second form, for leaves of side <= 32.  A wave takes one leaf at a time:
// the points of the 9 leaves around it are staged once into the wave's part of LDS, and the
// wave's 64 lanes are split into S slices of T lanes (T = targets per pass, a power of two),
// slice s summing sources s, s + S, ...; slices are reduced with xor shuffles.  For leaves of
// side s <= 16 phi sits in a window table over all offsets in [-(2s-1), 2s-1]^2 and each
// point carries the key K = 8 (y W + x) mod 2^32 (W = 4s - 1), so the byte offset of phi(x_i
// - x_j) in the table is K_i - K_j plus a constant: one integer subtraction per pair.  For
// side 32 a quadrant table over |dx|, |dy| < 64 is used.
constexpr int kStage = 384;   // staged sources per wave and pass

struct SrcRec {
    uint32_t a, b;   // window mode: a = key; quadrant mode: a = x, b = y
    double f;
};

__device__ inline void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int P, bool WINDOW>
__global__ __launch_bounds__(kBlock) void k_leaf_near(int64_t nleaves, int32_t leaf_off, const int32_t* box_pt0,
                                                       const int32_t* box_pt1, const uint64_t* box_key,
                                                       const int32_t* nlist, int64_t side, int W, const int2* pts,
                                                       const uint32_t* pkey, const double* fs, const int32_t* perm,
                                                       const double* U, const double* leafT, int far,
                                                       const double* phi_oct_tab, double* u) {
    extern __shared__ double smem[];
    double* tab = smem;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    SrcRec* stage = reinterpret_cast<SrcRec*>(smem + ((W * W + 1) & ~1)) + wave * kStage;   // 16-B aligned
    const int c = WINDOW ? int(2 * side - 1) : 0;
    for (int i = tid; i < W * W; i += kBlock) {
        int dy = i / W - c, dx = i - (i / W) * W - c;
        dx = dx < 0 ? -dx : dx;
        dy = dy < 0 ? -dy : dy;
        int hi = max(dx, dy), lo = min(dx, dy);
        tab[i] = phi_oct_tab[hi * (hi + 1) / 2 + lo];
    }
    __syncthreads();
    const char* tb = reinterpret_cast<const char*>(tab) + size_t(8) * size_t(c * W + c);
    for (int64_t leaf = int64_t(blockIdx.x) * kWaves + wave; leaf < nleaves; leaf += int64_t(gridDim.x) * kWaves) {
        const int32_t g = leaf_off + int32_t(leaf);
        const int32_t p0 = box_pt0[g], p1 = box_pt1[g];
        const int32_t nt = p1 - p0;
        int T = 1;
        while (T < nt && T < 64) T <<= 1;
        const int S = 64 / T, t = lane & (T - 1), sl = lane / T;
        // the 9 neighbour ranges (uniform)
        int32_t b0[9], cnt[9], total = 0;
        const int32_t* nl = nlist + size_t(leaf) * 9;
        #pragma unroll
        for (int q = 0; q < 9; ++q) {
            const int32_t nb = nl[q];
            b0[q] = nb >= 0 ? box_pt0[nb] : 0;
            cnt[q] = nb >= 0 ? box_pt1[nb] - b0[q] : 0;
            total += cnt[q];
        }
        const uint64_t key = box_key[g];
        const int32_t cx = int32_t(compact_bits(key) * side), cy = int32_t(compact_bits(key >> 1) * side);
        for (int32_t i0 = p0; i0 < p1; i0 += T) {
            const int32_t i = i0 + t;
            const bool valid = i < p1;
            const int32_t ii = valid ? i : p0;
            const int2 pi = pts[ii];
            const uint32_t ki = WINDOW ? pkey[ii] : 0u;
            double acc = 0.0;
            for (int32_t c0 = 0; c0 < total; c0 += kStage) {
                const int32_t cn = min(kStage, total - c0);
                for (int32_t pos = lane; pos < cn; pos += 64) {
                    int32_t r = c0 + pos, j = -1;
                    #pragma unroll
                    for (int q = 0; q < 9; ++q) {   // static indices: the ranges stay in registers
                        if (j < 0) {
                            if (r < cnt[q]) j = b0[q] + r;
                            else r -= cnt[q];
                        }
                    }
                    SrcRec rec;
                    if (WINDOW) {
                        rec.a = pkey[j];
                        rec.b = 0u;
                    } else {
                        const int2 pj = pts[j];
                        rec.a = uint32_t(pj.x);
                        rec.b = uint32_t(pj.y);
                    }
                    rec.f = fs[j];
                    stage[pos] = rec;
                }
                wave_sync_lds();
                for (int32_t jj = sl; jj < cn; jj += S) {
                    const SrcRec rec = stage[jj];
                    double ph;
                    if (WINDOW) {
                        ph = *reinterpret_cast<const double*>(tb + int32_t(ki - rec.a));
                    } else {
                        const int dx = abs(pi.x - int32_t(rec.a)), dy = abs(pi.y - int32_t(rec.b));
                        ph = tab[dy * W + dx];
                    }
                    acc += ph * rec.f;
                }
                wave_sync_lds();
            }
            if (far) {
                const int64_t loc = int64_t(pi.x - cx) + side * int64_t(pi.y - cy);
                const double* tl = leafT + loc * P;
                const double* uh = U + size_t(g) * P;
                for (int p = sl; p < P; p += S) acc += tl[p] * uh[p];
            }
            for (int o = T; o < 64; o <<= 1) acc += __shfl_xor(acc, o, 64);
            if (sl == 0 && valid) u[perm[i]] = acc;
        }
    }
}

__global__ void k_point_keys(const int2* pts, int64_t n, uint32_t W, uint32_t* key) {
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) {
        const int2 p = pts[i];
        key[i] = 8u * (uint32_t(p.y) * W + uint32_t(p.x));   // modulo 2^32 on purpose
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
                bool simple, hipStream_t st) {
    if (max_tiles <= 0) return;
    if (simple) {
        unsigned g = grid_for(max_tiles, kWaves);
        if (g > 2048) g = 2048;
        hipLaunchKernelGGL(k_m2l<kRankPad>, dim3(g), dim3(kBlock), 0, st, tiles, ntiles, cls_box, ilist, ilist_off,
                           Q, U, ifo);
        return;
    }
    // one tile per block and step; a multiple of 8 blocks keeps the XCD chunks balanced
    int64_t g = std::min<int64_t>(max_tiles, 8192);
    g = std::max<int64_t>(8, (g + 7) / 8 * 8);
    hipLaunchKernelGGL(k_m2l_split<kRankPad>, dim3(unsigned(g)), dim3(kBlock), 0, st, tiles, ntiles, cls_box, ilist,
                       ilist_off, Q, U, ifo);
}

void launch_point_keys(const int32_t* pts, int64_t n, int64_t side, uint32_t* key, hipStream_t st) {
    hipLaunchKernelGGL(k_point_keys, dim3(grid_for(n)), dim3(kBlock), 0, st, reinterpret_cast<const int2*>(pts), n,
                       uint32_t(4 * side - 1), key);
}

void launch_m2l_mixed(const M2LTile* tiles, const int32_t* ntiles, int32_t max_tiles, const int32_t* cls_box,
                      const int32_t* ilist, int32_t ilist_off, const double* Q, double* U, const float* ifo_hi,
                      const float* ifo_lo, const double* mono, const int32_t* rank, hipStream_t st) {
    if (max_tiles <= 0) return;
    unsigned g = grid_for(max_tiles, kWaves);
    if (g > 2048) g = 2048;
    hipLaunchKernelGGL(k_m2l_mixed<kRankPad>, dim3(g), dim3(kBlock), 0, st, tiles, ntiles, cls_box, ilist, ilist_off,
                       Q, U, ifo_hi, ifo_lo, mono, rank);
}

void launch_leaf_eval(int64_t nleaves, int32_t leaf_off, const int32_t* box_pt0, const int32_t* box_pt1,
                      const uint64_t* box_key, const int32_t* nlist, int L, int64_t side, const int32_t* pts,
                      const uint32_t* pkey, const double* fs, const int32_t* perm, const double* U,
                      const double* leafT, bool far, const double* phi_oct, double* u, bool simple, hipStream_t st) {
    (void)L;
    if (nleaves <= 0) return;
    unsigned g = grid_for(nleaves, kWaves);
    if (g > 4096) g = 4096;
    if (!simple && side <= 16 && pkey) {
        const int Ww = int(4 * side - 1);
        size_t lds = size_t((Ww * Ww + 1) & ~1) * sizeof(double) + size_t(kWaves) * kStage * sizeof(SrcRec);
        hipLaunchKernelGGL((k_leaf_near<kRankPad, true>), dim3(g), dim3(kBlock), lds, st, nleaves, leaf_off, box_pt0,
                           box_pt1, box_key, nlist, side, Ww, reinterpret_cast<const int2*>(pts), pkey, fs, perm, U,
                           leafT, far ? 1 : 0, phi_oct, u);
        return;
    }
    if (!simple && side <= 32) {
        const int Wq = int(2 * side);
        size_t lds = size_t((Wq * Wq + 1) & ~1) * sizeof(double) + size_t(kWaves) * kStage * sizeof(SrcRec);
        hipLaunchKernelGGL((k_leaf_near<kRankPad, false>), dim3(g), dim3(kBlock), lds, st, nleaves, leaf_off,
                           box_pt0, box_pt1, box_key, nlist, side, Wq, reinterpret_cast<const int2*>(pts), pkey, fs,
                           perm, U, leafT, far ? 1 : 0, phi_oct, u);
        return;
    }
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
