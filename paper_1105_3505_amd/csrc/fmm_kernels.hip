// Evaluation passes of the lattice FMM on gfx950 (Section 8.2), for a forest of instances.
//
// Expansions are stored box-major: box g owns kRankPad consecutive FP64 coefficients in Q
// (outgoing, q-hat) and U (incoming, u-hat).
//
//   P2M   q^tau   = T_ofs^tau q(J^tau)                 one wave per leaf, lanes = skeleton index
//   M2M   q^tau   = sum_c T_ofo^(c) q^child_c          FP64 MFMA box-matrix kernel
//   M2L   u^tau   = sum_{sigma in L_int} T_ifo^d q^sigma   FP64 MFMA box-matrix kernel
//   L2L   u^child += T_ofo^(c)T u^tau                  FP64 MFMA box-matrix kernel
//   L2P + near field + un-permutation                  one wave per leaf, lanes = targets x slices
#include "kernels.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <stdexcept>

namespace lfmm {

namespace {

constexpr int kBlock = 256;
constexpr int kBf16Block = 512;   // bf16 M2L: eight waves per 128-box tile
constexpr int kWaves = kBlock / 64;
// Levels of at most this many 64-box tiles run M2M and L2L on the fine-grained kernels, which
// spread one tile over twelve blocks (measured: M2M gains up to 64 tiles, L2L up to 256).
constexpr int32_t kFineM2mTiles = 64;
constexpr int32_t kFineL2lTiles = 256;
constexpr double kPi = 3.14159265358979323846;
constexpr double kEulerGamma = 0.57721566490153286061;

typedef double double4_t __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));
typedef double double2_t __attribute__((ext_vector_type(2)));
typedef int int2_t __attribute__((ext_vector_type(2)));
typedef int int4_t __attribute__((ext_vector_type(4)));

// Interaction-list slot k of a box in child position c lies at offset slot c_dslot[c][k]
// of the 7 x 7 offset grid; the order matches the list builder (dy outer, dx inner).
struct DSlots { int s[4][kNumInteractions]; };
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

// Far-field expansion of phi (eq. (3.1) for the 5-point operator, true Euler constant;
// coefficients of the context's operator in *e); (a, b) != 0
__device__ inline double phi_expansion_dev(double a, double b, const PhiFar* e) {
    const double r2 = a * a + b * b;
    const double ir2 = 1.0 / r2;
    const double c2 = (a * a - b * b) * ir2;   // cos 2 theta
    const double c4 = 2.0 * c2 * c2 - 1.0, c8 = 2.0 * c4 * c4 - 1.0, c12 = 2.0 * c4 * c8 - c4;
    const double lead = -(0.5 * log(r2) + e->C) * (1.0 / (2.0 * kPi));
    const double t1 = e->c[0][0] + e->c[0][1] * c4;
    const double t2 = e->c[1][0] + e->c[1][1] * c4 + e->c[1][2] * c8;
    const double t3 = e->c[2][0] + e->c[2][1] * c4 + e->c[2][2] * c8 + e->c[2][3] * c12;
    return lead + ir2 * (t1 + ir2 * (t2 + ir2 * t3));
}

// phi at offset (a, b), a, b >= 0: the device octant table (quadrature values inside radius
// 128, the expansion evaluated once between 128 and kPhiDeviceRadius), the expansion outside
__device__ inline double phi_oct(int a, int b, const double* oct, const PhiFar* far) {
    const int hi = max(a, b), lo = min(a, b);
    if (hi <= kPhiDeviceRadius) return oct[hi * (hi + 1) / 2 + lo];
    return phi_expansion_dev(double(hi), double(lo), far);
}

// Octant entries with r0 < hi <= r1 (index hi (hi + 1) / 2 + lo) set to the expansion, so
// that lookups replace the logarithm and division of the expansion for offsets up to r1.
__global__ void k_phi_extend(double* oct, int r0, int r1, const PhiFar* far) {
    const int64_t i0 = int64_t(r0 + 1) * (r0 + 2) / 2, i1 = int64_t(r1 + 1) * (r1 + 2) / 2;
    const int64_t i = i0 + int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= i1) return;
    int64_t hi = int64_t((sqrt(8.0 * double(i) + 1.0) - 1.0) * 0.5);
    while (hi * (hi + 1) / 2 > i) --hi;
    while ((hi + 1) * (hi + 2) / 2 <= i) ++hi;
    const int64_t lo = i - hi * (hi + 1) / 2;
    oct[i] = phi_expansion_dev(double(hi), double(lo), far);
}

inline unsigned grid_for(int64_t n, int per_block = kBlock) {
    const int64_t g = (n + per_block - 1) / per_block;
    return unsigned(g < 1 ? 1 : g);
}

// Load of sorted point s: in the caller's order, the instance-local index perm_local[s] of
// instance pinst[s]; with sorted loads, index s itself (coalesced); zero for a point that is a
// target only.  Also stored at fs[s] for the near field: P2M visits every point once.
__device__ inline double gather_f(const ExecPtrs* tab, const ExecPtrs& single, const int32_t* perm_local,
                                  const int32_t* pinst, int64_t s, double* fs) {
    const ExecPtrs e = tab ? tab[pinst[s]] : single;
    const double* f = e.f;
    const int32_t nsrc = e.nsrc;
    const bool sorted = e.sorted != 0;
    const int32_t j = perm_local[s];
    const double v = j < nsrc ? f[sorted ? s : int64_t(j)] : 0.0;
    fs[s] = v;
    return v;
}

// P2M with the dense-model operator (Remark 8.2): q-hat[p] = sum_j T[loc(j)][p] f_j; one
// wave per leaf, lane p < P accumulating entry p.  The leaf's points are loaded once, one
// per lane (coalesced), and handed to all lanes by shuffles, so the only memory reads in the
// loop are the operator rows, whose addresses are known in advance and can be in flight
// together.  Each entry is one sum over the leaf's points in order, as in k_p2m_lds: which of
// the two kernels a launch takes depends on the plan (the mean points per leaf), so a leaf must
// get the same bits from both for an instance alone and in a forest to agree.
template <int P>
__global__ __launch_bounds__(kBlock) void k_p2m(int32_t leaf0, int32_t leaf1, const int32_t* box_pt0,
                                                 const int32_t* box_pt1, const uint64_t* box_key, int64_t side,
                                                 const int2* pts, const ExecPtrs* tab, ExecPtrs single,
                                                 const int32_t* perm_local, const int32_t* pinst,
                                                 double* fs, const double* leafT, double* Q) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int32_t g = leaf0 + int32_t(blockIdx.x) * kWaves + wave;
    if (g >= leaf1) return;
    const int32_t p0 = box_pt0[g], p1 = box_pt1[g];
    const uint64_t key = box_key[g];
    const int32_t cx = int32_t(compact_bits(key) * side), cy = int32_t(compact_bits(key >> 1) * side);
    const int l = lane < P ? lane : 0;
    double a = 0.0;
    for (int32_t c0 = p0; c0 < p1; c0 += 64) {
        const int32_t j = c0 + lane;
        int32_t loc = 0;   // lanes past the leaf's points carry a zero load at cell 0
        double f = 0.0;
        if (j < p1) {
            const int2 q = pts[j];
            loc = int32_t(int64_t(q.x - cx) + side * int64_t(q.y - cy));
            f = gather_f(tab, single, perm_local, pinst, j, fs);
        }
        const int cnt = min(64, p1 - c0);
        for (int k = 0; k < cnt; k += 4) {   // k + 3 < 64: the tail reads the zero-load lanes
            const int32_t l0 = __shfl(loc, k, 64), l1 = __shfl(loc, k + 1, 64);
            const int32_t l2 = __shfl(loc, k + 2, 64), l3 = __shfl(loc, k + 3, 64);
            const double f0 = __shfl(f, k, 64), f1 = __shfl(f, k + 1, 64);
            const double f2 = __shfl(f, k + 2, 64), f3 = __shfl(f, k + 3, 64);
            // the four rows are loaded together; the sum takes them in point order
            const double t0 = leafT[int64_t(l0) * P + l], t1 = leafT[int64_t(l1) * P + l];
            const double t2 = leafT[int64_t(l2) * P + l], t3 = leafT[int64_t(l3) * P + l];
            a += t0 * f0;
            a += t1 * f1;
            a += t2 * f2;
            a += t3 * f3;
        }
    }
    if (lane < P) Q[size_t(g) * P + lane] = a;
}

// P2M with the leaf operator staged in LDS (leaf sides whose T_ofs fits: side^2 P doubles):
// persistent blocks of kP2mThreads copy T_ofs once, then each wave takes 8 leaves at a time,
// one per 8-lane group; lane l of a group accumulates rows l, l + 8, ..., l + 40 of Q-hat over
// the leaf's points, which the group loads 8 at a time and broadcasts by shuffles.  A group
// past the others' point counts adds zero loads at cell 0.  The next leaves' box data are
// loaded while the current ones are summed.
constexpr int kP2mThreads = 1024;
constexpr int kP2mGroup = 8;                   // lanes per leaf
constexpr int kP2mLeaves = 64 / kP2mGroup;     // leaves per wave and step
// leaves with T_ofs too large for LDS take the grouped kernel (global T_ofs) when they hold
// at most this many points on average, else one wave each
constexpr int kP2mSparsePoints = 16;

// STAGED false: the same grouping for leaves whose T_ofs is too large for LDS but that hold few
// points each (the sparse leaves of clustered inputs): the operator rows come from global memory
// (L2-resident), eight lanes reading one 384-byte row together.
template <int P, bool STAGED = true>
__global__ __launch_bounds__(kP2mThreads) void k_p2m_lds(int32_t leaf0, int32_t leaf1, const int32_t* box_pt0,
                                                        const int32_t* box_pt1, const uint64_t* box_key, int64_t side,
                                                        const int2* pts, const ExecPtrs* tab, ExecPtrs single,
                                                        const int32_t* perm_local,
                                                        const int32_t* pinst, double* fs, const double* leafT,
                                                        double* Q) {
    constexpr int R = P / kP2mGroup;   // rows per lane
    static_assert(P % kP2mGroup == 0, "rows split evenly over a group");
    extern __shared__ double sT_lds[];
    const int ncell = int(side * side);
    if (STAGED) {
        const double2* src = reinterpret_cast<const double2*>(leafT);
        double2* dst = reinterpret_cast<double2*>(sT_lds);
        for (int i = int(threadIdx.x); i < ncell * P / 2; i += kP2mThreads) dst[i] = src[i];
    }
    const double* sT = STAGED ? sT_lds : leafT;
    const int wave = int(threadIdx.x) >> 6, lane = int(threadIdx.x) & 63, l = lane % kP2mGroup;
    const int grp = lane / kP2mGroup;
    const int32_t nleaf = leaf1 - leaf0;
    const int32_t stride = int32_t(gridDim.x) * (kP2mThreads / 64) * kP2mLeaves;
    int32_t q = (int32_t(blockIdx.x) * (kP2mThreads / 64) + wave) * kP2mLeaves;
    // box data of this lane's leaf at step q
    auto box = [&](int32_t qq, int32_t& p0, int32_t& npt, int32_t& cx, int32_t& cy) {
        p0 = 0;
        npt = 0;
        cx = cy = 0;
        if (qq + grp < nleaf) {
            const int32_t g = leaf0 + qq + grp;
            p0 = box_pt0[g];
            npt = box_pt1[g] - p0;
            const uint64_t key = box_key[g];
            cx = int32_t(compact_bits(key) * side);
            cy = int32_t(compact_bits(key >> 1) * side);
        }
    };
    int32_t p0, npt, cx, cy;
    box(q, p0, npt, cx, cy);
    __syncthreads();
    for (; q < nleaf; q += stride) {
        int32_t np0, nnpt, ncx, ncy;
        box(q + stride, np0, nnpt, ncx, ncy);
        int32_t nmax = npt;
        #pragma unroll
        for (int o = kP2mGroup; o < 64; o <<= 1) nmax = max(nmax, __shfl_xor(nmax, o, 64));
        double a[R];
        #pragma unroll
        for (int r = 0; r < R; ++r) a[r] = 0.0;
        for (int32_t c0 = 0; c0 < nmax; c0 += kP2mGroup) {
            int32_t loc = 0;
            double f = 0.0;
            if (c0 + l < npt) {
                const int2 pt = pts[p0 + c0 + l];
                loc = int32_t(int64_t(pt.x - cx) + side * int64_t(pt.y - cy));
                f = gather_f(tab, single, perm_local, pinst, p0 + c0 + l, fs);
            }
            #pragma unroll
            for (int k = 0; k < kP2mGroup; ++k) {
                const int src = (lane & ~(kP2mGroup - 1)) | k;
                const int32_t lk = __shfl(loc, src, 64);
                const double fk = __shfl(f, src, 64);
                const double* row = sT + lk * P + l;
                #pragma unroll
                for (int r = 0; r < R; ++r) a[r] += row[kP2mGroup * r] * fk;
            }
        }
        if (q + grp < nleaf) {
            double* out = Q + size_t(leaf0 + q + grp) * P + l;
            #pragma unroll
            for (int r = 0; r < R; ++r) out[kP2mGroup * r] = a[r];
        }
        p0 = np0;
        npt = nnpt;
        cx = ncx;
        cy = ncy;
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

// Box-matrix passes on the FP64 matrix cores: for a tile of up to 64 target boxes that share
// their operators, out[box] (+)= sum over slots k of A_k in[src_k(box)] with 48 x 48 A_k:
//   M2M (step 2): 4 children, A_k = T_ofo^(k) at the tile's height, in = out = Q;
//   L2L (step 4): the parent, A = T_ofo^(c)T at the parent's height, in = out = U, added.
// Wave w of the block owns boxes 16 w .. 16 w + 15 (the 16 columns of its products) and runs
// every slot, so no partial sums cross waves.  Operators are stored in fragment order (lane
// l's operands of one instruction next to lane l+1's), staged once per block in LDS with
// coalesced loads, double-buffered, and read by all four waves; the next slot's operator and
// source expansion are loaded into registers while the current slot's instructions run, and
// the list entry behind the expansion read one slot before that.  One barrier per slot: the
// buffer a slot writes was last read two slots earlier, before the previous slot's barrier.
// Absent sources (empty list slots, lanes past the tile) read the all-zero row `zrow`.
//
// FP64: 16x16x4 instruction, step kk of row block m takes column g * 12 + kk in lane group
// g = lane / 16; element i of lane (g, n) is row 16 m + g + 4 i, column n.
__device__ inline int32_t uniform(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }

// Pointers into global memory by address space, so that loads through them are global (not
// flat) loads: flat loads also count as LDS operations, and waiting for the LDS reads of a
// slot would then wait for the next slot's prefetch too.
template <class T>
using gptr = const __attribute__((address_space(1))) T*;
template <class T>
__device__ inline gptr<T> global(const T* p) {
    return (gptr<T>)(p);   // generic to global address space
}

template <int MODE>
__device__ inline void boxmat_tiles(const BoxTile* tiles, int32_t ntiles, const int32_t* box_list,
                                    const int32_t* src_tab, const OpsPtrs* ops, const double* in, int32_t zrow,
                                    double* out, const int8_t* role = nullptr) {
    constexpr int P = kRankPad, MT = P / 16, KQ = P / 4, NJ = KQ / 2;
    static_assert(MODE == kModeM2M || MODE == kModeL2L, "M2L has a kernel of its own");
    constexpr int NS = (MODE == kModeM2M) ? 4 : 1;
    constexpr int SW = NS;   // source table width
    constexpr int A2 = P * P / 2;                      // double2_t per operator: 4.5 per thread
    static_assert(A2 == 4 * kBlock + kBlock / 2, "staging below assumes P = 48");
    static_assert(MT == 3, "three row blocks");
    __shared__ double2_t sA[2][A2];
    __shared__ int s_dsl[4];   // operator of each slot of the tile
    const int tid = int(threadIdx.x), wave = tid >> 6, lane = tid & 63;
    const int n = lane & 15, g = lane >> 4;
    const int32_t G = int32_t(gridDim.x);
    const double2_t z2 = {0.0, 0.0};
    for (int32_t step = 0;; ++step) {
        const int32_t t = uniform(xcd_tile(int32_t(blockIdx.x), G, step, ntiles));
        if (t < 0) break;                                  // uniform over the block
        const int32_t count = uniform(tiles[t].count);
        if (count == 0) continue;
        const int32_t start = uniform(tiles[t].start), height = uniform(tiles[t].height);
        const int32_t cls = uniform(tiles[t].cls), opi = uniform(tiles[t].ops);
        const int col = 16 * wave + n;
        const int32_t box = (col < count) ? (box_list ? box_list[start + col] : start + col) : -1;
        const gptr<int32_t> srcs = global(src_tab + size_t(box >= 0 ? box : 0) * SW);
        const double* base = (MODE == kModeM2M) ? ops[opi].ofo_rm : ops[opi].ofo_cm;
        const gptr<double2_t> Ah = global(reinterpret_cast<const double2_t*>(base));
        const gptr<double> Xg = global(in) + g * KQ;
        if (tid < NS) s_dsl[tid] = (MODE == kModeM2M) ? height * 4 + tid : (height + 1) * 4 + cls;
        __syncthreads();
        const int* dsl = s_dsl;
        // slot 0 operands
        int32_t src = (box >= 0) ? srcs[0] : -1;
        src = src < 0 ? zrow : src;
        const gptr<double2_t> qs = reinterpret_cast<gptr<double2_t>>(Xg + size_t(src) * P);
        double2_t rb0 = qs[0], rb1 = qs[1], rb2 = qs[2], rb3 = qs[3], rb4 = qs[4], rb5 = qs[5];
        int32_t src_next = (box >= 0 && NS > 1) ? srcs[1] : -1;
        const gptr<double2_t> Ak = Ah + size_t(dsl[0]) * A2;
        int32_t dsl_next = NS > 1 ? dsl[1] : 0;   // operator of the next slot, read a slot ahead
        double2_t ra0 = Ak[tid], ra1 = Ak[tid + kBlock], ra2 = Ak[tid + 2 * kBlock], ra3 = Ak[tid + 3 * kBlock];
        double2_t ra4 = (tid < kBlock / 2) ? Ak[tid + 4 * kBlock] : z2;
        double4_t acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = acc0, acc2 = acc0;
        // M2M and L2L sum their contraction as four partial products added in order, the same
        // arithmetic as the fine-grained kernels below, so that a box's result does not depend
        // on which kernel its level runs on.
        double4_t run0 = acc0, run1 = acc0, run2 = acc0;
        auto fold = [&](bool first) {
            const double4_t z4 = {0.0, 0.0, 0.0, 0.0};
            if (first) {
                run0 = acc0;
                run1 = acc1;
                run2 = acc2;
            } else {
                run0 += acc0;
                run1 += acc1;
                run2 += acc2;
            }
            acc0 = z4;
            acc1 = z4;
            acc2 = z4;
        };
        for (int k = 0; k < NS; ++k) {
            double2_t* buf = sA[k & 1];
            buf[tid] = ra0;
            buf[tid + kBlock] = ra1;
            buf[tid + 2 * kBlock] = ra2;
            buf[tid + 3 * kBlock] = ra3;
            if (tid < kBlock / 2) buf[tid + 4 * kBlock] = ra4;
            const double2_t b[NJ] = {rb0, rb1, rb2, rb3, rb4, rb5};
            __syncthreads();
            if (k + 1 < NS) {
                // expansions first: their address waits only for the list entry read a slot ago
                const int32_t sn = src_next < 0 ? zrow : src_next;
                const gptr<double2_t> qn = reinterpret_cast<gptr<double2_t>>(Xg + size_t(sn) * P);
                rb0 = qn[0];
                rb1 = qn[1];
                rb2 = qn[2];
                rb3 = qn[3];
                rb4 = qn[4];
                rb5 = qn[5];
                src_next = (box >= 0 && k + 2 < NS) ? srcs[k + 2] : -1;
                const gptr<double2_t> An = Ah + size_t(uniform(dsl_next)) * A2;
                ra0 = An[tid];
                ra1 = An[tid + kBlock];
                ra2 = An[tid + 2 * kBlock];
                ra3 = An[tid + 3 * kBlock];
                if (tid < kBlock / 2) ra4 = An[tid + 4 * kBlock];
                dsl_next = (k + 2 < NS) ? dsl[k + 2] : 0;
            }
            // every wave runs the products (a wave past the tile's boxes multiplies the zero
            // row): no branch around them, so the accumulators stay in place between slots
            {
                #pragma unroll
                for (int j = 0; j < NJ; ++j) {
                    const double2_t a0 = buf[(0 * NJ + j) * 64 + lane];
                    const double2_t a1 = buf[(1 * NJ + j) * 64 + lane];
                    const double2_t a2 = buf[(2 * NJ + j) * 64 + lane];
                    #pragma unroll
                    for (int e = 0; e < 2; ++e) {
                        if (MODE == kModeL2L && (2 * j + e) % 3 == 0 && j + e > 0) {
                            fold(2 * j + e == 3);   // step 3 c starts the c-th partial sum
                        }
                        acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(e ? a0.y : a0.x, e ? b[j].y : b[j].x, acc0, 0, 0, 0);
                        acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(e ? a1.y : a1.x, e ? b[j].y : b[j].x, acc1, 0, 0, 0);
                        acc2 = __builtin_amdgcn_mfma_f64_16x16x4f64(e ? a2.y : a2.x, e ? b[j].y : b[j].x, acc2, 0, 0, 0);
                    }
                }
            }
            if (MODE == kModeM2M) fold(k == 0);   // one partial sum per child slot
        }
        if (MODE == kModeL2L) fold(false);
        acc0 = run0;
        acc1 = run1;
        acc2 = run2;
        if (box >= 0) {
            double* ob = out + size_t(box) * P;
            // a pruned box of the adaptive tree has no M2L result: it takes its parent's alone
            const bool add = MODE == kModeL2L && !(role != nullptr && role[box] == kRolePruned);
            #pragma unroll
            for (int i = 0; i < 4; ++i) {
                if (add) {
                    ob[g + 4 * i] += acc0[i];
                    ob[16 + g + 4 * i] += acc1[i];
                    ob[32 + g + 4 * i] += acc2[i];
                } else {
                    ob[g + 4 * i] = acc0[i];
                    ob[16 + g + 4 * i] = acc1[i];
                    ob[32 + g + 4 * i] = acc2[i];
                }
            }
        }
        __syncthreads();   // the next tile's first slot rewrites a buffer read above
    }
}

// M2L (Section 8.2 step 3) on the FP64 matrix cores for tiles of up to 128 target boxes that
// share their 27 operators (same operator set, height and child position).  Wave w owns the two
// 16-box column blocks of boxes 32 w .. 32 w + 31, so each operator staged in LDS (once per slot
// and block, double-buffered, one barrier per slot) feeds 72 matrix instructions per wave: the
// staging and the barrier cost half as much per product as with one column block, and a launch
// of the 1e6-point plan fits the device in one round of blocks.  The tile's interaction lists
// are copied into LDS when the tile starts, so the slot loop issues no dependent global loads:
// within a slot the wave runs its two column blocks one after the other, and the source
// expansion of the next (slot, column block) pair is loaded from global memory while the
// current pair's products run (its list entry read from LDS one pair earlier).  Absent sources
// (empty list slots, boxes past the tile) read the zero row.
// 16x16x4 FP64 instruction: step kk of row block m takes column g * 12 + kk in lane group
// g = lane / 16; element i of lane (g, n) is row 16 m + g + 4 i, column n.
__global__ __launch_bounds__(kBlock, 3) void k_m2l(const BoxTile* tiles, const int32_t* ntiles_dev,
                                                    const int32_t* box_list, const int32_t* il27, const OpsPtrs* ops,
                                                    const double* Q, int32_t zrow, double* U) {
    const int32_t ntiles = uniform(*ntiles_dev);
    constexpr int P = kRankPad, KQ = P / 4, NJ = KQ / 2, NS = kNumInteractions;
    constexpr int A2 = P * P / 2;                      // double2_t per operator: 4.5 per thread
    static_assert(A2 == 4 * kBlock + kBlock / 2, "staging below assumes P = 48");
    static_assert(kM2LTile == 128, "two column blocks per wave");
    __shared__ double2_t sA[2][A2];
    __shared__ int32_t s_src[kM2LTile * NS];     // source box of (tile column, slot), zrow if none
    __shared__ int32_t s_box[kM2LTile];
    __shared__ int s_dsl[NS];
    const int tid = int(threadIdx.x), wave = tid >> 6, lane = tid & 63;
    const int n = lane & 15, g = lane >> 4;
    const int32_t G = int32_t(gridDim.x);
    const double2_t z2 = {0.0, 0.0};
    for (int32_t step = 0;; ++step) {
        const int32_t t = uniform(xcd_tile(int32_t(blockIdx.x), G, step, ntiles));
        if (t < 0) break;                                  // uniform over the block
        const int32_t count = uniform(tiles[t].count);
        if (count == 0) continue;
        const int32_t start = uniform(tiles[t].start), height = uniform(tiles[t].height);
        const int32_t cls = uniform(tiles[t].cls), opi = uniform(tiles[t].ops);
        if (tid < NS) s_dsl[tid] = height * kNumIfoSlots + c_dslot.s[cls][tid];
        if (tid < kM2LTile) s_box[tid] = (tid < count) ? box_list[start + tid] : -1;
        __syncthreads();
        for (int i = tid; i < kM2LTile * NS; i += kBlock) {
            const int b = i / NS;
            const int32_t box = s_box[b];
            const int32_t src = box >= 0 ? il27[size_t(box) * NS + (i - b * NS)] : -1;
            s_src[i] = src < 0 ? zrow : src;
        }
        const gptr<double2_t> Ah = global(reinterpret_cast<const double2_t*>(ops[opi].ifo));
        const gptr<double> Xg = global(Q) + g * KQ;
        const int col0 = 32 * wave + n;
        const int32_t box0 = s_box[col0], box1 = s_box[col0 + 16];
        __syncthreads();
        const int* dsl = s_dsl;
        const int32_t* src0 = s_src + col0 * NS;          // this lane's two columns' lists
        const int32_t* src1 = src0 + 16 * NS;
        auto load_q = [&](int32_t src, double2_t (&r)[NJ]) {
            const gptr<double2_t> q = reinterpret_cast<gptr<double2_t>>(Xg + size_t(src) * P);
            #pragma unroll
            for (int j = 0; j < NJ; ++j) r[j] = q[j];
        };
        double2_t bq[NJ], nq[NJ];
        load_q(src0[0], nq);                               // pair (slot 0, block 0)
        int32_t idx_next = src1[0];                        // pair (slot 0, block 1)
        const gptr<double2_t> A0 = Ah + size_t(dsl[0]) * A2;
        int32_t dsl_next = dsl[1];
        double2_t ra0 = A0[tid], ra1 = A0[tid + kBlock], ra2 = A0[tid + 2 * kBlock], ra3 = A0[tid + 3 * kBlock];
        double2_t ra4 = (tid < kBlock / 2) ? A0[tid + 4 * kBlock] : z2;
        double4_t acc[2][3];
        #pragma unroll
        for (int c = 0; c < 2; ++c)
            #pragma unroll
            for (int m = 0; m < 3; ++m) acc[c][m] = double4_t{0.0, 0.0, 0.0, 0.0};
        for (int k = 0; k < NS; ++k) {
            double2_t* buf = sA[k & 1];
            buf[tid] = ra0;
            buf[tid + kBlock] = ra1;
            buf[tid + 2 * kBlock] = ra2;
            buf[tid + 3 * kBlock] = ra3;
            if (tid < kBlock / 2) buf[tid + 4 * kBlock] = ra4;
            __syncthreads();
            if (k + 1 < NS) {   // the next slot's operator, into registers
                const gptr<double2_t> An = Ah + size_t(uniform(dsl_next)) * A2;
                ra0 = An[tid];
                ra1 = An[tid + kBlock];
                ra2 = An[tid + 2 * kBlock];
                ra3 = An[tid + 3 * kBlock];
                if (tid < kBlock / 2) ra4 = An[tid + 4 * kBlock];
                dsl_next = (k + 2 < NS) ? dsl[k + 2] : 0;
            }
            // the slot's products at raised issue priority, the staging and barrier at the normal
            // one, so that a wave keeps the matrix pipe through its run of products (measured 1-3 %
            // faster here; the same in the bf16 kernel measured 19 % slower)
            __builtin_amdgcn_s_setprio(1);
            #pragma unroll
            for (int c = 0; c < 2; ++c) {
                // each pass reads its operator fragments from LDS anew: holding the first pass's
                // fragments in registers for the second would cost 72 VGPRs (a third of them)
                asm volatile("" ::: "memory");
                #pragma unroll
                for (int j = 0; j < NJ; ++j) bq[j] = nq[j];
                // the next pair: (k, block 1) after block 0, (k + 1, block 0) after block 1
                if (c == 0 || k + 1 < NS) {
                    load_q(idx_next, nq);
                    idx_next = (c == 0) ? (k + 1 < NS ? src0[k + 1] : zrow) : src1[k + 1];
                }
                #pragma unroll
                for (int j = 0; j < NJ; ++j) {
                    const double2_t a0 = buf[(0 * NJ + j) * 64 + lane];
                    const double2_t a1 = buf[(1 * NJ + j) * 64 + lane];
                    const double2_t a2 = buf[(2 * NJ + j) * 64 + lane];
                    acc[c][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0.x, bq[j].x, acc[c][0], 0, 0, 0);
                    acc[c][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1.x, bq[j].x, acc[c][1], 0, 0, 0);
                    acc[c][2] = __builtin_amdgcn_mfma_f64_16x16x4f64(a2.x, bq[j].x, acc[c][2], 0, 0, 0);
                    acc[c][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0.y, bq[j].y, acc[c][0], 0, 0, 0);
                    acc[c][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1.y, bq[j].y, acc[c][1], 0, 0, 0);
                    acc[c][2] = __builtin_amdgcn_mfma_f64_16x16x4f64(a2.y, bq[j].y, acc[c][2], 0, 0, 0);
                }
            }
            __builtin_amdgcn_s_setprio(0);
        }
        #pragma unroll
        for (int c = 0; c < 2; ++c) {
            const int32_t box = c ? box1 : box0;
            if (box >= 0) {
                double* ob = U + size_t(box) * P;
                // plain stores: streaming (non-temporal) ones were measured to leave the time
                // unchanged and to send these 8-byte pieces to memory uncombined (2.4x the
                // written bytes)
                #pragma unroll
                for (int i = 0; i < 4; ++i) {
                    ob[g + 4 * i] = acc[c][0][i];
                    ob[16 + g + 4 * i] = acc[c][1][i];
                    ob[32 + g + 4 * i] = acc[c][2][i];
                }
            }
        }
        __syncthreads();   // the next tile rewrites the staging buffers and lists read above
    }
}

__global__ __launch_bounds__(kBlock) void k_m2m(const BoxTile* tiles, int32_t ntiles, const int32_t* box_child,
                                                 const OpsPtrs* ops, double* Q, int32_t zrow) {
    boxmat_tiles<kModeM2M>(tiles, ntiles, nullptr, box_child, ops, Q, zrow, Q);
}

__global__ __launch_bounds__(kBlock) void k_l2l(const BoxTile* tiles, int32_t ntiles, const int32_t* box_list,
                                                 const int32_t* box_parent, const OpsPtrs* ops, double* U,
                                                 int32_t zrow, const int8_t* role) {
    boxmat_tiles<kModeL2L>(tiles, ntiles, box_list, box_parent, ops, U, zrow, U, role);
}

// Box-matrix passes for levels with few boxes (M2M and L2L).  The kernels above run a 64-box
// tile on one block whose waves each run every slot, so a level of a handful of tiles lasts a
// whole sequence of dependent products on one SIMD.  Here block (t, q, m) computes rows
// 16 m .. 16 m + 15 of boxes 16 q .. 16 q + 15 of tile t, and its four waves split the
// contraction: in M2M wave w applies the operator of child slot w; in L2L wave w takes steps
// 3 w .. 3 w + 2 of the twelve 16x16x4 steps of the parent's operator.  The four partial
// products meet in LDS in a fixed order, and wave w writes element w of every lane's four.
// Operator fragments are read straight from the fragment-ordered table (the rows of one row
// block are contiguous there), without LDS staging.
template <int MODE>
__device__ inline void boxmat_fine(const BoxTile* tiles, const int32_t* box_list, const int32_t* src_tab,
                                   const OpsPtrs* ops, const double* in, int32_t zrow, double* out,
                                   const int8_t* role = nullptr) {
    constexpr int P = kRankPad, KQ = P / 4, NJ = KQ / 2, A2 = P * P / 2;
    static_assert(MODE == kModeM2M || MODE == kModeL2L, "fine mode serves M2M and L2L");
    __shared__ double red[4][4][64];
    const int tid = int(threadIdx.x), wave = tid >> 6, lane = tid & 63;
    const int n = lane & 15, g = lane >> 4;
    const int32_t b = int32_t(blockIdx.x);
    const int m = b % 3, q = (b / 3) & 3;
    const int32_t t = b / 12;
    const int32_t count = uniform(tiles[t].count);
    if (16 * q >= count) return;                       // uniform over the block, before any barrier
    const int32_t start = uniform(tiles[t].start), height = uniform(tiles[t].height);
    const int32_t cls = uniform(tiles[t].cls), opi = uniform(tiles[t].ops);
    const int col = 16 * q + n;
    const int32_t box = (col < count) ? (MODE == kModeL2L ? box_list[start + col] : start + col) : -1;
    int32_t src = -1;
    if (box >= 0) src = (MODE == kModeM2M) ? src_tab[size_t(box) * 4 + wave] : src_tab[box];
    src = src < 0 ? zrow : src;
    const gptr<double> xs = global(in) + size_t(src) * P + g * KQ;
    const bool add = MODE == kModeL2L && box >= 0 && !(role != nullptr && role[box] == kRolePruned);
    const double old = add ? out[size_t(box) * P + 16 * m + g + 4 * wave] : 0.0;
    const double4_t zero4 = {0.0, 0.0, 0.0, 0.0};
    double4_t acc = zero4;
    if (MODE == kModeM2M) {
        const gptr<double2_t> A = global(reinterpret_cast<const double2_t*>(ops[opi].ofo_rm)) +
                                  size_t(height * 4 + wave) * A2 + size_t(m * NJ) * 64 + lane;
        const gptr<double2_t> xb = reinterpret_cast<gptr<double2_t>>(xs);
        double2_t a[NJ], x[NJ];
        #pragma unroll
        for (int j = 0; j < NJ; ++j) {
            x[j] = xb[j];
            a[j] = A[j * 64];
        }
        #pragma unroll
        for (int j = 0; j < NJ; ++j) {
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[j].x, x[j].x, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[j].y, x[j].y, acc, 0, 0, 0);
        }
    } else {
        const gptr<double> A = global(ops[opi].ofo_cm) + size_t((height + 1) * 4 + cls) * (2 * A2) +
                               size_t(m * NJ) * 128 + 2 * lane;
        double a[3], x[3];
        #pragma unroll
        for (int r = 0; r < 3; ++r) {
            const int s = 3 * wave + r, j = s >> 1, e = s & 1;   // step s = 2 j + e
            x[r] = xs[s];
            a[r] = A[j * 128 + e];
        }
        #pragma unroll
        for (int r = 0; r < 3; ++r) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[r], x[r], acc, 0, 0, 0);
    }
    #pragma unroll
    for (int i = 0; i < 4; ++i) red[wave][i][lane] = acc[i];
    __syncthreads();
    const double v = ((red[0][wave][lane] + red[1][wave][lane]) + red[2][wave][lane]) + red[3][wave][lane];
    if (box >= 0) {
        out[size_t(box) * P + 16 * m + g + 4 * wave] = (MODE == kModeL2L) ? old + v : v;
    }
}

__global__ __launch_bounds__(kBlock) void k_m2m_fine(const BoxTile* tiles, const int32_t* box_child,
                                                      const OpsPtrs* ops, double* Q, int32_t zrow) {
    boxmat_fine<kModeM2M>(tiles, nullptr, box_child, ops, Q, zrow, Q);
}

__global__ __launch_bounds__(kBlock) void k_l2l_fine(const BoxTile* tiles, const int32_t* box_list,
                                                      const int32_t* box_parent, const OpsPtrs* ops, double* U,
                                                      int32_t zrow, const int8_t* role) {
    boxmat_fine<kModeL2L>(tiles, box_list, box_parent, ops, U, zrow, U, role);
}

// Mixed-precision operands of the outgoing expansions, once per box: q-hat split into FP32
// hi + lo parts (hi = fl32(q), lo = fl32(q - hi), so that hi + lo equals q to about 2^-48) and
// its charge sum in FP64, for boxes [0, nrows) (the all-zero row included).
__global__ void k_split_q(const double* Q, int32_t nrows, float* Qh, float* Ql, double* qs) {
    constexpr int P = kRankPad;
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t box = t / 64;
    const int lane = int(t & 63);
    if (box >= nrows) return;   // uniform over the wave: a wave is one box
    const double q = lane < P ? Q[box * P + lane] : 0.0;
    const float hi = float(q);
    if (lane < P) {
        Qh[box * P + lane] = hi;
        Ql[box * P + lane] = float(q - double(hi));
    }
    double s = q;
    #pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if (lane == 0) qs[box] = s;
}

// Mixed-precision M2L on the FP32 matrix cores, on the same 128-box tiles as k_m2l (each wave's
// two column blocks in two passes over the 27 slots) with the same staging.  Each
// operator is written T^d = c_d 1 1^T + R^d with c_d its mean entry: the constant part,
// which carries the large log|d| level of the kernel, is applied in FP64 as c_d times the
// source's charge sum; only the remainder R^d, several times smaller, goes through FP32.
// R^d and q-hat are split into FP32 hi + lo parts (q-hat once per box by k_split_q).  Each
// 4-term step of R_hi q_hi is an FP32 product of its own, converted and added to the FP64
// accumulators at once, so FP32 rounding acts on four terms at a time; the cross terms
// R_hi q_lo and R_lo q_hi (about 2^-24 of the main term) accumulate in two FP32 accumulators
// over the slot and are flushed once.  The FP32 instruction returns element i of lane (g, n)
// as row 4 g + i.
__global__ __launch_bounds__(kBlock) void k_m2l_mixed(const BoxTile* tiles, const int32_t* ntiles_p,
                                                       const int32_t* box_list, const int32_t* il27,
                                                       const OpsPtrs* ops, const float* Qh, const float* Ql,
                                                       const double* qs, int32_t zrow, double* U) {
    constexpr int P = kRankPad, MT = P / 16, KQ = P / 4, NJ4 = KQ / 4;
    constexpr int A4 = P * P / 4;                      // float4 per operator part: 2.25 per thread
    static_assert(A4 == 2 * kBlock + kBlock / 4, "staging below assumes P = 48");
    __shared__ float4_t sH[2][A4];
    __shared__ float4_t sL[2][A4];
    __shared__ int s_dsl[kNumInteractions];
    const int tid = int(threadIdx.x), wave = tid >> 6, lane = tid & 63;
    const int n = lane & 15, g = lane >> 4;
    const int32_t ntiles = uniform(*ntiles_p);
    const int32_t G = int32_t(gridDim.x);
    const float4_t zero = {0.f, 0.f, 0.f, 0.f};
    for (int32_t step = 0;; ++step) {
        const int32_t t = uniform(xcd_tile(int32_t(blockIdx.x), G, step, ntiles));
        if (t < 0) break;
        const int32_t count = uniform(tiles[t].count);
        if (count == 0) continue;
        const int32_t start = uniform(tiles[t].start), height = uniform(tiles[t].height);
        const int32_t cls = uniform(tiles[t].cls), opi = uniform(tiles[t].ops);
        const int rk = ops[opi].rank[height];
        const size_t hbase = size_t(height) * kNumIfoSlots * A4;
        const gptr<float4_t> Hh = global(reinterpret_cast<const float4_t*>(ops[opi].ifo_hi)) + hbase;
        const gptr<float4_t> Lh = global(reinterpret_cast<const float4_t*>(ops[opi].ifo_lo)) + hbase;
        const gptr<double> mono = global(ops[opi].mono) + size_t(height) * kNumIfoSlots;
        // lane group g supplies rows 12 g .. 12 g + 11 of its column's q-hat
        const gptr<float4_t> QH = global(reinterpret_cast<const float4_t*>(Qh)) + 3 * g;
        const gptr<float4_t> QL = global(reinterpret_cast<const float4_t*>(Ql)) + 3 * g;
        const gptr<double> QS = global(qs);
        if (tid < kNumInteractions) s_dsl[tid] = c_dslot.s[cls][tid];
        __syncthreads();
        const int* dsl = s_dsl;
        // the wave's two 16-box column blocks (boxes 32 w .. 32 w + 31 of the tile), one pass each
        for (int cb = 0; cb < 2; ++cb) {
        const bool wave_on = 32 * wave + 16 * cb < count;
        const int col = 32 * wave + 16 * cb + n;
        const int32_t box = (col < count) ? box_list[start + col] : -1;
        const gptr<int32_t> il = global(il27 + size_t(box >= 0 ? box : 0) * kNumInteractions);
        int32_t src = (box >= 0) ? il[0] : -1;
        src = src < 0 ? zrow : src;
        float4_t h0 = QH[size_t(src) * 12], h1 = QH[size_t(src) * 12 + 1], h2 = QH[size_t(src) * 12 + 2];
        float4_t l0 = QL[size_t(src) * 12], l1 = QL[size_t(src) * 12 + 1], l2 = QL[size_t(src) * 12 + 2];
        double qsum = QS[src];
        int32_t src_next = (box >= 0) ? il[1] : -1;
        size_t off = size_t(dsl[0]) * A4;
        float4_t rh0 = Hh[off + tid], rh1 = Hh[off + tid + kBlock];
        float4_t rl0 = Lh[off + tid], rl1 = Lh[off + tid + kBlock];
        float4_t rh2 = (tid < kBlock / 4) ? Hh[off + tid + 2 * kBlock] : zero;
        float4_t rl2 = (tid < kBlock / 4) ? Lh[off + tid + 2 * kBlock] : zero;
        double4_t acc[MT];
        #pragma unroll
        for (int m = 0; m < MT; ++m) acc[m] = double4_t{0.0, 0.0, 0.0, 0.0};
        for (int k = 0; k < kNumInteractions; ++k) {
            const int bsel = k & 1;
            sH[bsel][tid] = rh0;
            sH[bsel][tid + kBlock] = rh1;
            sL[bsel][tid] = rl0;
            sL[bsel][tid + kBlock] = rl1;
            if (tid < kBlock / 4) {
                sH[bsel][tid + 2 * kBlock] = rh2;
                sL[bsel][tid + 2 * kBlock] = rl2;
            }
            const float4_t bh[NJ4] = {h0, h1, h2}, bl[NJ4] = {l0, l1, l2};
            const double cq = qsum;
            const int d = dsl[k];
            __syncthreads();
            if (k + 1 < kNumInteractions) {
                const int32_t sn = src_next < 0 ? zrow : src_next;
                h0 = QH[size_t(sn) * 12];
                h1 = QH[size_t(sn) * 12 + 1];
                h2 = QH[size_t(sn) * 12 + 2];
                l0 = QL[size_t(sn) * 12];
                l1 = QL[size_t(sn) * 12 + 1];
                l2 = QL[size_t(sn) * 12 + 2];
                qsum = QS[sn];
                src_next = (box >= 0 && k + 2 < kNumInteractions) ? il[k + 2] : -1;
                off = size_t(dsl[k + 1]) * A4;
                rh0 = Hh[off + tid];
                rh1 = Hh[off + tid + kBlock];
                rl0 = Lh[off + tid];
                rl1 = Lh[off + tid + kBlock];
                if (tid < kBlock / 4) {
                    rh2 = Hh[off + tid + 2 * kBlock];
                    rl2 = Lh[off + tid + 2 * kBlock];
                }
            }
            if (wave_on) {
                const double mq = mono[d] * cq;   // constant part of T^d times the charge sum
                #pragma unroll
                for (int m = 0; m < MT; ++m) {
                    #pragma unroll
                    for (int i = 0; i < 4; ++i)
                        if (16 * m + 4 * g + i < rk) acc[m][i] += mq;   // padded rows stay zero
                }
                #pragma unroll
                for (int m = 0; m < MT; ++m) {
                    float4_t c1 = zero, c2 = zero;
                    #pragma unroll
                    for (int j4 = 0; j4 < NJ4; ++j4) {
                        const float4_t ah = sH[bsel][(m * NJ4 + j4) * 64 + lane];
                        const float4_t al = sL[bsel][(m * NJ4 + j4) * 64 + lane];
                        #pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            const float4_t p = __builtin_amdgcn_mfma_f32_16x16x4f32(ah[e], bh[j4][e], zero, 0, 0, 0);
                            c1 = __builtin_amdgcn_mfma_f32_16x16x4f32(ah[e], bl[j4][e], c1, 0, 0, 0);
                            c2 = __builtin_amdgcn_mfma_f32_16x16x4f32(al[e], bh[j4][e], c2, 0, 0, 0);
                            #pragma unroll
                            for (int i = 0; i < 4; ++i) acc[m][i] += double(p[i]);
                        }
                    }
                    #pragma unroll
                    for (int i = 0; i < 4; ++i) acc[m][i] += double(c1[i]) + double(c2[i]);
                }
            }
        }
        if (box >= 0) {
            double* ub = U + size_t(box) * P;
            #pragma unroll
            for (int m = 0; m < MT; ++m) {
                #pragma unroll
                for (int i = 0; i < 4; ++i) ub[16 * m + 4 * g + i] = acc[m][i];   // FP32 output layout
            }
        }
        __syncthreads();   // the next pass (or tile) rewrites the staging buffers
        }
    }
}

// bf16 mixed precision.  On gfx950 the bf16 matrix instructions run 32 times faster than the
// FP64 ones (16x16x32 in 16 cycles against 16x16x4 in 64), while FP32 runs only twice as fast,
// so that a split FP32 product (three instructions) cannot beat FP64.  Here q-hat and R^d
// (T^d less its constant part, applied in FP64 as for the FP32 form) are each split into three
// bf16 parts, x = x0 + x1 + x2 with x_k the rounded remainder of the parts before (about 24
// significant bits in all), and R q is formed from the six products R_a q_b with a + b <= 2:
// the dropped ones are below 2^-24 of the leading product.  bf16 x bf16 products are exact in
// FP32.  The six 48-term products are 36 (product, group of 8 columns) pieces, laid along the
// contraction of nine K = 32 instructions that sum into one FP32 accumulator, which is added
// to the FP64 accumulator once per interaction.
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));

// bits of the bf16 nearest to x (through FP32, as the operators' host split) and their value
__device__ inline uint32_t bf16_bits(double x) {
    uint32_t u = __float_as_uint(float(x));
    u += 0x7FFFu + ((u >> 16) & 1u);
    return u >> 16;
}
__device__ inline double bf16_val(uint32_t b) { return double(__uint_as_float(b << 16)); }

// q-hat in three bf16 parts (row of a box: part p holds entries p * 48 .. p * 48 + 47) and its
// FP64 charge sum, for boxes [0, nrows) (the all-zero row included); each remainder is exact.
// Eight lanes per box, lane g < 6 taking entries 8 g .. 8 g + 7 (one 64-byte read, one 16-byte
// write per part); the charge sum adds the six lanes' partial sums in a fixed order.
__global__ void k_split_q_bf16(const double* Q, int32_t nrows, uint16_t* Qb, double* qs) {
    constexpr int P = kRankPad;
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t box = t >> 3;
    const int g = int(t & 7);
    if (box >= nrows) return;   // uniform over each 8-lane group
    double part_sum = 0.0;
    if (g < P / 8) {
        const double2* src = reinterpret_cast<const double2*>(Q + box * P + 8 * g);
        double q[8];
        #pragma unroll
        for (int e = 0; e < 4; ++e) {
            const double2 v = src[e];
            q[2 * e] = v.x;
            q[2 * e + 1] = v.y;
        }
        uint32_t bits[3][4];
        #pragma unroll
        for (int e = 0; e < 8; ++e) {
            part_sum += q[e];
            double r = q[e];
            #pragma unroll
            for (int part = 0; part < 3; ++part) {
                const uint32_t b = bf16_bits(r);
                r -= bf16_val(b);
                if (e & 1) bits[part][e >> 1] |= b << 16;
                else bits[part][e >> 1] = b;
            }
        }
        uint4* row = reinterpret_cast<uint4*>(Qb + box * (3 * P));
        #pragma unroll
        for (int part = 0; part < 3; ++part)
            row[part * (P / 8) + g] = make_uint4(bits[part][0], bits[part][1], bits[part][2], bits[part][3]);
    }
    part_sum += __shfl_xor(part_sum, 1, 64);
    part_sum += __shfl_xor(part_sum, 2, 64);
    part_sum += __shfl_xor(part_sum, 4, 64);
    if (g == 0) qs[box] = part_sum;
}

// M2L on the bf16 matrix cores, on the same 128-box tiles as k_m2l: eight waves per tile, wave w
// owning the 16-box column block w, four waves per SIMD.  (Two column blocks per wave would
// read each operator fragment from LDS once for two products, but its registers allow only
// two waves per SIMD, too few to hide the latencies of a slot that lasts a quarter of an FP64
// one; measured slower.)  The operator's three parts (13.5 KB) are staged in LDS once per slot
// and block.
//
// Contraction layout.  16x16x32 bf16 instruction: lane (g, n) supplies row n of the operator
// and column n of q-hat at contraction indices 8 g .. 8 g + 7 (one group of 8 columns of one
// part each); element i of its result is row 4 g + i, column n.  Lane group g owns column
// groups c = 3 (g & 1) + t, t = 0, 1, 2; in instruction j = 3 t + r it takes column group
// 3 (g & 1) + t of the product
//   g = 0, 1:  r = 0: R0 q0,  r = 1: R1 q0,  r = 2: R2 q0
//   g = 2, 3:  r = 0: R0 q1,  r = 1: R1 q1,  r = 2: R0 q2
// so every (product, column group) piece appears once, and a lane reads three groups of q-hat
// (g = 0, 1: q0) or six (g = 2, 3: q1 and q2) per source.
//
// Rounding.  The leading product R0 q0 sits in the instructions r = 0 (a third of it in each);
// each of them starts from zero and is added to the FP64 accumulator at once, so FP32 rounds
// partial sums of a third of the leading product only.  The r = 1, 2 instructions (at most
// 2^-8 of it) share one FP32 sum per interaction.  The constant part c_d times the source's
// charge sum is summed per column in FP64 and added once at the end.
//
// The next slot's q-hat groups are loaded into the registers of group t as soon as the
// current slot's instructions 3 t .. 3 t + 2 have read them.
__global__ __launch_bounds__(kBf16Block, 4) void k_m2l_bf16(const BoxTile* tiles, const int32_t* ntiles_dev,
                                                              const int32_t* box_list, const int32_t* il27,
                                                              const OpsPtrs* ops, const uint16_t* Qb,
                                                              const double* qs, int32_t zrow, double* U) {
    const int32_t ntiles = uniform(*ntiles_dev);
    constexpr int P = kRankPad, NS = kNumInteractions, NF = kBf16OpVecs, NT = kBf16Block;
    static_assert(kM2LTile == 16 * (kBf16Block / 64), "one column block per wave");
    constexpr int NST = (NF + NT - 1) / NT;     // staged groups per thread
    constexpr uint32_t QB = kBf16QVecs * 16;    // bytes of q-hat parts per box
    __shared__ u32x4_t sA[2][NF];
    __shared__ int32_t s_src[kM2LTile * NS];     // source box of (tile column, slot), zrow if none
    __shared__ int32_t s_box[kM2LTile];
    __shared__ int s_dsl[NS];
    __shared__ double s_mono[NS];
    const int tid = int(threadIdx.x), wave = tid >> 6, lane = tid & 63;
    const int n = lane & 15, g = lane >> 4;
    const bool q0_lanes = g < 2;                 // lane groups 0, 1: the three products with q0
    const int c0 = 3 * (g & 1);                  // first column group of the lane group
    const int32_t G = int32_t(gridDim.x);
    const u32x4_t z4 = {0u, 0u, 0u, 0u};
    const float4_t zero = {0.f, 0.f, 0.f, 0.f};
    // operator fragment of instruction j = 3 t + r, row block m: group
    // pa * 288 + 96 m + 16 (c0 + t) + n with pa = r, except pa = 0 for r = 2 on lanes 2, 3
    const int abase = c0 * 16 + n;
    const int abase2 = abase + (q0_lanes ? 2 * 288 : 0);
    // q-hat groups of a source, byte offsets: lanes 0, 1 part 0, groups c0 .. c0 + 2 (twice, so
    // that instruction r = 2 reads the second copy on every lane); lanes 2, 3 part 1, then part 2
    const uint32_t qoff1 = uint32_t((q0_lanes ? 0 : 6) + c0) * 16u;
    const uint32_t qoff2 = uint32_t((q0_lanes ? 0 : 12) + c0) * 16u;
    const int col = 16 * wave + n;               // this lane's column of the tile
    for (int32_t step = 0;; ++step) {
        const int32_t t = uniform(xcd_tile(int32_t(blockIdx.x), G, step, ntiles));
        if (t < 0) break;                                  // uniform over the block
        const int32_t count = uniform(tiles[t].count);
        if (count == 0) continue;
        const int32_t start = uniform(tiles[t].start), height = uniform(tiles[t].height);
        const int32_t cls = uniform(tiles[t].cls), opi = uniform(tiles[t].ops);
        if (tid < NS) {
            const int d = height * kNumIfoSlots + c_dslot.s[cls][tid];
            s_dsl[tid] = d;
            s_mono[tid] = ops[opi].mono[d];
        }
        if (tid < kM2LTile) s_box[tid] = (tid < count) ? box_list[start + tid] : -1;
        __syncthreads();
        for (int i = tid; i < kM2LTile * NS; i += NT) {
            const int b = i / NS;
            const int32_t box = s_box[b];
            const int32_t src = box >= 0 ? il27[size_t(box) * NS + (i - b * NS)] : -1;
            s_src[i] = src < 0 ? zrow : src;
        }
        const int rk = uniform(ops[opi].rank[height]);
        const gptr<u32x4_t> Ah = global(reinterpret_cast<const u32x4_t*>(ops[opi].ifo_b));
        const gptr<double> QS = global(qs);
        const gptr<uint8_t> Xb = global(reinterpret_cast<const uint8_t*>(Qb));
        const int32_t box = s_box[col];
        __syncthreads();
        const int32_t* srcs = s_src + col * NS;
        // q-hat groups of the slot's source: [t] first part, [3 + t] the part that instruction
        // 3 t + 2 reads; sources addressed by 32-bit byte offsets from Qb
        u32x4_t bq[6];
        uint32_t qn = uint32_t(srcs[0]) * QB;
        double nsum = QS[srcs[0]];
        auto load_group = [&](int tt) {
            bq[tt] = *reinterpret_cast<gptr<u32x4_t>>(Xb + (qn + qoff1 + 16u * tt));
            bq[3 + tt] = *reinterpret_cast<gptr<u32x4_t>>(Xb + (qn + qoff2 + 16u * tt));
        };
        #pragma unroll
        for (int tt = 0; tt < 3; ++tt) load_group(tt);
        int32_t dsl_next = s_dsl[1];
        u32x4_t ra[NST];
        {
            const gptr<u32x4_t> A0 = Ah + size_t(s_dsl[0]) * NF;
            #pragma unroll
            for (int e = 0; e < NST; ++e) ra[e] = (e * NT + tid < NF) ? A0[e * NT + tid] : z4;
        }
        double4_t acc[3];
        #pragma unroll
        for (int m = 0; m < 3; ++m) acc[m] = double4_t{0.0, 0.0, 0.0, 0.0};
        double mono_acc = 0.0;
        for (int k = 0; k < NS; ++k) {
            u32x4_t* buf = sA[k & 1];
            #pragma unroll
            for (int e = 0; e < NST; ++e)
                if (e * NT + tid < NF) buf[e * NT + tid] = ra[e];
            mono_acc += s_mono[k] * nsum;   // constant part of T^d times the charge sum
            __syncthreads();
            if (k + 1 < NS) {   // the next slot's operator, into registers; its source
                const gptr<u32x4_t> An = Ah + size_t(uniform(dsl_next)) * NF;
                #pragma unroll
                for (int e = 0; e < NST; ++e)
                    if (e * NT + tid < NF) ra[e] = An[e * NT + tid];
                dsl_next = (k + 2 < NS) ? s_dsl[k + 2] : 0;
                const int32_t sn = srcs[k + 1];
                qn = uint32_t(sn) * QB;
                nsum = QS[sn];
            }
            asm volatile("" ::: "memory");
            float4_t small[3];
            #pragma unroll
            for (int tt = 0; tt < 3; ++tt) {
                #pragma unroll
                for (int r = 0; r < 3; ++r) {
                    const int j = 3 * tt + r;
                    // three operator fragments in flight: more would cost the fourth wave per SIMD
                    asm volatile("" ::: "memory");
                    #pragma unroll
                    for (int m = 0; m < 3; ++m) {
                        const u32x4_t a =
                            (r == 2) ? buf[abase2 + 96 * m + 16 * tt] : buf[abase + r * 288 + 96 * m + 16 * tt];
                        // r = 2: q0 (lanes 0, 1) or q2 (lanes 2, 3); else the lane group's first part
                        const u32x4_t b = (r == 2) ? bq[3 + tt] : bq[tt];
                        const bf16x8_t av = __builtin_bit_cast(bf16x8_t, a), bv = __builtin_bit_cast(bf16x8_t, b);
                        if (r == 0) {
                            const float4_t p = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, zero, 0, 0, 0);
                            #pragma unroll
                            for (int i = 0; i < 4; ++i) acc[m][i] += double(p[i]);
                        } else {
                            small[m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, j == 1 ? zero : small[m], 0,
                                                                               0, 0);
                        }
                    }
                }
                if (k + 1 < NS) load_group(tt);   // group tt of the next slot's source
            }
            #pragma unroll
            for (int m = 0; m < 3; ++m)
                #pragma unroll
                for (int i = 0; i < 4; ++i) acc[m][i] += double(small[m][i]);
        }
        if (box >= 0) {
            double* ob = U + size_t(box) * P;
            #pragma unroll
            for (int m = 0; m < 3; ++m)
                #pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int row = 16 * m + 4 * g + i;
                    ob[row] = acc[m][i] + (row < rk ? mono_acc : 0.0);   // padded rows stay zero
                }
        }
        __syncthreads();   // the next tile rewrites the staging buffers and lists read above
    }
}

// Leaf pass: far field T_tfi u-hat with T_tfi = T_ofs^T (Section 7, symmetric kernel and
// targets = sources) plus the direct sum over the points of the leaf and its neighbours
// (Section 8.2 step 5), written back in the caller's point order.
//
// A wave takes one group: the (up to four) leaves of one parent box, whose targets are one
// contiguous run of Morton-ordered points, one target per lane.  The sources are the points
// of the union of the leaves' neighbourhoods (a 4 x 4 block of leaves at most), listed per
// group at plan time as point ranges with their leaf coordinates.  The wave walks those
// ranges in lockstep: range and source reads are uniform over the wave (scalar loads), and a
// lane adds a range's sources only if that leaf neighbours its own leaf (the group's own leaves
// are one range, near to every lane).
//   WINDOW (side <= 16): phi sits in a window table over all offsets in [-(2s-1), 2s-1]^2 and
//     each point carries the key K = 8 (y W + x) mod 2^32 (W = 4s - 1), so the byte offset of
//     phi(x_i - x_j) is K_i - K_j plus a constant: one subtraction per pair.
//   QUAD (side 32): a table over |dx|, |dy| < 64.
//   GLOBAL (side >= 64): the device octant table (radius kPhiDeviceRadius) in global memory,
//     eq. (3.1) beyond.
enum LeafMode { kWindow = 0, kQuad = 1, kGlobal = 2 };
constexpr int kNearXcdChunk = 512;     // groups per chunk of the near field's XCD-aware walk
constexpr int kNearTabMax = 64 * 64;   // doubles: W^2 for the window (side 16) and quad (side 32) tables
// Block size per mode.  With an LDS phi table, 512-thread blocks share one table among eight
// waves and run persistently (each builds its table once); with the global table, 256-thread
// blocks take one group per wave and the hardware balances uneven groups.
constexpr int near_threads(int mode) { return mode == kGlobal ? 256 : 512; }

// read-only data that every lane of a wave reads at the same address: constant address
// space, so that uniform reads become scalar loads
template <class T>
using cptr = const __attribute__((address_space(4))) T*;
template <class T>
__device__ inline cptr<T> as_const(const T* p) {
    return (cptr<T>)(p);   // generic to constant address space
}

// One group of leaves (see k_near).
//   SLICED = false (groups of more than 32 targets): one target per lane over the whole group,
//     sources read at wave-uniform addresses (scalar loads); a lane adds a range's sources only
//     if that range's leaf neighbours its own leaf.
//   SLICED = true (groups of at most 32 targets): leaf by leaf; the n targets of a leaf take T lanes each
//     (T = the power of two at or above n, at most 64) of S = 64 / T slices, slice s summing
//     every S-th source of each neighbouring range, and the slices are added by xor shuffles.
template <int P, int MODE, bool SLICED>
__device__ inline void near_group(int32_t qq, const NearGroup* groups, const int4* ents, const int32_t* box_pt0,
                                  const int32_t* box_pt1, const uint64_t* box_key, const int32_t* box_inst,
                                  int64_t side, int W, const double* tab, const char* tb, uint32_t kofs,
                                  const int2* pts,
                                  const uint32_t* pkey, const double* fs, const int32_t* perm_local,
                                  const ExecPtrs* tab_ptrs, ExecPtrs single, const double* U,
                                  const double* leafT, const double* leafTt, const uint8_t* far_inst,
                                  const double* phi_oct_tab, const PhiFar* phi_far) {
    const int lane = threadIdx.x & 63;
    const cptr<int4_t> E = as_const(reinterpret_cast<const int4_t*>(ents));
    const cptr<uint32_t> SK = as_const(pkey);
    const cptr<double> SF = as_const(fs);
    const cptr<int2_t> SP = as_const(reinterpret_cast<const int2_t*>(pts));
    const int32_t leaf0 = uniform(groups[qq].leaf0), nleaf = uniform(groups[qq].nleaf);
    const int32_t ne = uniform(groups[qq].ne);
    // first point of each leaf of the group (uniform) and the end of the last
    int32_t bnd[5];
    bnd[0] = uniform(box_pt0[leaf0]);
    bnd[1] = nleaf > 1 ? uniform(box_pt0[leaf0 + 1]) : bnd[0];
    bnd[2] = nleaf > 2 ? uniform(box_pt0[leaf0 + 2]) : bnd[0];
    bnd[3] = nleaf > 3 ? uniform(box_pt0[leaf0 + 3]) : bnd[0];
    const int32_t t_end = uniform(box_pt1[leaf0 + nleaf - 1]);
    bnd[nleaf] = t_end;
    const int32_t k_inst = uniform(box_inst[leaf0]);
    const bool far = far_inst[k_inst] != 0;
    const ExecPtrs eio = tab_ptrs ? tab_ptrs[k_inst] : single;
    double* u = eio.u;
    const bool sorted_out = eio.sorted != 0;   // u indexed by sorted point
    const int32_t tgt0 = eio.tgt0;   // first target index
    // passes: the whole group once (group mode) or each leaf in turn (sliced mode)
    for (int c0 = 0; c0 < (SLICED ? nleaf : 1); ++c0) {
        const int32_t p0 = SLICED ? bnd[c0] : bnd[0];
        const int32_t p1 = SLICED ? bnd[c0 + 1] : t_end;
        int T = 64;
        if (SLICED) {
            T = 1;
            while (T < p1 - p0 && T < 64) T <<= 1;
        }
        const int S = 64 / T, tl = lane & (T - 1), sl = lane / T;
        for (int32_t i0 = p0; i0 < p1; i0 += T) {
            const int32_t i = i0 + tl;
            const bool valid = i < p1;
            const int32_t ii = valid ? i : p0;
            const int c = SLICED ? c0 : (nleaf > 1 && ii >= bnd[1]) + (nleaf > 2 && ii >= bnd[2]) +
                                            (nleaf > 3 && ii >= bnd[3]);
            const int32_t leaf = leaf0 + c;
            const uint64_t key = box_key[leaf];
            const int32_t tx = int32_t(compact_bits(key)), ty = int32_t(compact_bits(key >> 1));
            const int2 pi = pts[ii];
            // the window centre's byte offset is folded into the target's key once, so that a
            // pair costs one subtraction for its table address
            const uint32_t ki = (MODE == kWindow) ? pkey[ii] + kofs : 0u;
            const int32_t pout = perm_local[ii];
            double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
            auto phi_at = [&](uint32_t kj, int2_t pj) -> double {
                if (MODE == kWindow) return *reinterpret_cast<const double*>(tb + int32_t(ki - kj));
                const int dx = abs(pi.x - pj.x), dy = abs(pi.y - pj.y);
                if (MODE == kQuad) return tab[dy * W + dx];
                return phi_oct(dx, dy, phi_oct_tab, phi_far);
            };
            auto src_key = [&](int32_t j) -> uint32_t {
                if (MODE != kWindow) return 0u;
                return SLICED ? pkey[j] : SK[j];
            };
            auto src_pt = [&](int32_t j) -> int2_t {
                if (MODE == kWindow) return int2_t{0, 0};
                if (SLICED) {
                    const int2 p = pts[j];
                    return int2_t{p.x, p.y};
                }
                return SP[j];
            };
            auto src_f = [&](int32_t j) -> double { return SLICED ? fs[j] : SF[j]; };
            for (int e = 0; e < ne; ++e) {
                const int4_t en = E[size_t(qq) * kNearEntries + e];   // (first point, end, leaf x, leaf y)
                const bool near = (en.z == kNearAll || abs(en.z - tx) <= 1) &&
                                  (en.w == kNearAll || abs(en.w - ty) <= 1);   // uniform when sliced
                if (near) {
                    int32_t j = en.x + sl;
                    if (!SLICED)   // sixteen sources per step: few waits for their scalar loads
                        for (; j + 15 < en.y; j += 16) {
                            #pragma unroll
                            for (int r = 0; r < 16; r += 4) {
                                a0 += phi_at(src_key(j + r), src_pt(j + r)) * src_f(j + r);
                                a1 += phi_at(src_key(j + r + 1), src_pt(j + r + 1)) * src_f(j + r + 1);
                                a2 += phi_at(src_key(j + r + 2), src_pt(j + r + 2)) * src_f(j + r + 2);
                                a3 += phi_at(src_key(j + r + 3), src_pt(j + r + 3)) * src_f(j + r + 3);
                            }
                        }
                    if (!SLICED)
                        for (; j + 7 < en.y; j += 8) {
                            a0 += phi_at(src_key(j), src_pt(j)) * src_f(j);
                            a1 += phi_at(src_key(j + 1), src_pt(j + 1)) * src_f(j + 1);
                            a2 += phi_at(src_key(j + 2), src_pt(j + 2)) * src_f(j + 2);
                            a3 += phi_at(src_key(j + 3), src_pt(j + 3)) * src_f(j + 3);
                            a0 += phi_at(src_key(j + 4), src_pt(j + 4)) * src_f(j + 4);
                            a1 += phi_at(src_key(j + 5), src_pt(j + 5)) * src_f(j + 5);
                            a2 += phi_at(src_key(j + 6), src_pt(j + 6)) * src_f(j + 6);
                            a3 += phi_at(src_key(j + 7), src_pt(j + 7)) * src_f(j + 7);
                        }
                    for (; j + 3 * S < en.y; j += 4 * S) {
                        a0 += phi_at(src_key(j), src_pt(j)) * src_f(j);
                        a1 += phi_at(src_key(j + S), src_pt(j + S)) * src_f(j + S);
                        a2 += phi_at(src_key(j + 2 * S), src_pt(j + 2 * S)) * src_f(j + 2 * S);
                        a3 += phi_at(src_key(j + 3 * S), src_pt(j + 3 * S)) * src_f(j + 3 * S);
                    }
                    if (!SLICED) {
                        // the last one to three sources with their loads issued together (one wait)
                        const int32_t rem = en.y - j;
                        if (rem == 3) {
                            a0 += phi_at(src_key(j), src_pt(j)) * src_f(j);
                            a1 += phi_at(src_key(j + 1), src_pt(j + 1)) * src_f(j + 1);
                            a2 += phi_at(src_key(j + 2), src_pt(j + 2)) * src_f(j + 2);
                        } else if (rem == 2) {
                            a0 += phi_at(src_key(j), src_pt(j)) * src_f(j);
                            a1 += phi_at(src_key(j + 1), src_pt(j + 1)) * src_f(j + 1);
                        } else if (rem == 1) {
                            a0 += phi_at(src_key(j), src_pt(j)) * src_f(j);
                        }
                    } else {
                        for (; j < en.y; j += S) a0 += phi_at(src_key(j), src_pt(j)) * src_f(j);
                    }
                }
            }
            if (far) {
                const int64_t loc = int64_t(pi.x - tx * side) + side * int64_t(pi.y - ty * side);
                const double* tlp = leafT + loc * P;
                const double* uh = U + size_t(leaf) * P;
                if (SLICED) {
                    for (int p = sl; p < P; p += S) a1 += tlp[p] * uh[p];
                } else {
                    // coefficient pairs from the coefficient-major table: the wave's lanes read
                    // pair p of their cells from one span of 16 side^2 bytes (about half as many
                    // cache lines per load as whole rows of the cell-major table)
                    const int64_t nc = side * side;
                    const double2_t* tl2 = reinterpret_cast<const double2_t*>(leafTt) + loc;
                    const double2_t* uh2 = reinterpret_cast<const double2_t*>(uh);
                    #pragma unroll
                    for (int p = 0; p < P / 2; p += 2) {
                        const double2_t x0 = tl2[p * nc], y0 = uh2[p], x1 = tl2[(p + 1) * nc], y1 = uh2[p + 1];
                        a0 += x0.x * y0.x;
                        a1 += x0.y * y0.y;
                        a2 += x1.x * y1.x;
                        a3 += x1.y * y1.y;
                    }
                }
            }
            double acc = (a0 + a1) + (a2 + a3);
            if (SLICED)
                for (int o = T; o < 64; o <<= 1) acc += __shfl_xor(acc, o, 64);
            if (valid && sl == 0 && pout >= tgt0) u[sorted_out ? int64_t(ii) : int64_t(pout - tgt0)] = acc;
        }
    }
}

// Window mode is held to six waves per SIMD (80 VGPRs): left free, the compiler keeps all 24
// coefficient-pair loads of the far field in flight (103 VGPRs, four waves per SIMD), which
// measured slower.
template <int P, int MODE>
__global__ __launch_bounds__(near_threads(MODE), MODE == kWindow ? 6 : 1) void k_near(int32_t q0, int32_t q1, const NearGroup* groups,
                                                      const int4* ents, const int32_t* box_pt0,
                                                      const int32_t* box_pt1, const uint64_t* box_key,
                                                      const int32_t* box_inst, int64_t side, int W, const int2* pts,
                                                      const uint32_t* pkey, const double* fs,
                                                      const int32_t* perm_local, const ExecPtrs* tab_ptrs,
                                                      ExecPtrs single, const double* U,
                                                      const double* leafT, const double* leafTt,
                                                      const uint8_t* far_inst, const double* phi_oct_tab,
                                                      const PhiFar* phi_far) {
    constexpr int kNearBlock = near_threads(MODE), kNearWaves = kNearBlock / 64;
    // fixed-size table (largest window: side 32), so that its base is a compile-time constant
    // and folds into the address of every read
    __shared__ double tab[MODE == kGlobal ? 1 : kNearTabMax];
    const int tid = threadIdx.x, wave = tid >> 6;
    if (MODE != kGlobal) {
        const int c = (MODE == kWindow) ? int(2 * side - 1) : 0;
        constexpr int kU = 8;   // loads in flight per thread
        for (int i0 = tid; i0 < W * W; i0 += kNearBlock * kU) {
            double v[kU];
            #pragma unroll
            for (int u = 0; u < kU; ++u) {
                const int i = i0 + u * kNearBlock;
                v[u] = 0.0;
                if (i < W * W) {
                    int dy = i / W - c, dx = i - (i / W) * W - c;
                    dx = dx < 0 ? -dx : dx;
                    dy = dy < 0 ? -dy : dy;
                    const int hi = max(dx, dy), lo = min(dx, dy);
                    v[u] = phi_oct_tab[hi * (hi + 1) / 2 + lo];
                }
            }
            #pragma unroll
            for (int u = 0; u < kU; ++u)
                if (i0 + u * kNearBlock < W * W) tab[i0 + u * kNearBlock] = v[u];
        }
        __syncthreads();
    }
    const int cw = (MODE == kWindow) ? int(2 * side - 1) : 0;
    const char* tb = reinterpret_cast<const char*>(tab);
    const uint32_t kofs = 8u * uint32_t(cw * W + cw);
    // XCD-aware walk of the group list: block b runs on XCD b % 8, and XCD x takes the chunks x,
    // x + 8, x + 16, ... of kNearXcdChunk consecutive (Morton-ordered) groups, so that most sources
    // that neighbouring groups share are read through one L2 (on 1e6 uniform points 5 % faster than
    // the plain walk; one contiguous eighth per XCD was 8 % faster there but leaves an XCD with all
    // of a dense region's work, which the same split made 1.1-1.8x slower in the clustered kernels).
    // With fewer than 8 blocks, the plain walk.
    const int32_t G = int32_t(gridDim.x);
    int32_t x = 0, first = int32_t(blockIdx.x), nb = G, C = q1 - q0 + 1;
    if (G >= 8) {
        x = first & 7;
        first >>= 3;
        nb = (G + 7 - x) >> 3;   // blocks on XCD x
        C = kNearXcdChunk;
    }
    for (int32_t l = first * kNearWaves + wave;; l += nb * kNearWaves) {
        const int32_t q = q0 + (8 * (l / C) + x) * C + l % C;   // increases with l
        if (q >= q1) break;
        const int32_t qq = uniform(q);
        const int32_t leaf0 = uniform(groups[qq].leaf0), nleaf = uniform(groups[qq].nleaf);
        const int32_t nt = uniform(box_pt1[leaf0 + nleaf - 1]) - uniform(box_pt0[leaf0]);
        // group mode when half a wave or more is busy and phi comes from an LDS table; leaf by
        // leaf otherwise (the octant table in global memory is read faster a leaf at a time)
        if (MODE != kGlobal && nt > 32)
            near_group<P, MODE, false>(qq, groups, ents, box_pt0, box_pt1, box_key, box_inst, side, W, tab, tb, kofs, pts,
                                       pkey, fs, perm_local, tab_ptrs, single, U, leafT, leafTt, far_inst,
                                       phi_oct_tab, phi_far);
        else
            near_group<P, MODE, true>(qq, groups, ents, box_pt0, box_pt1, box_key, box_inst, side, W, tab, tb, kofs, pts,
                                      pkey, fs, perm_local, tab_ptrs, single, U, leafT, leafTt, far_inst,
                                      phi_oct_tab, phi_far);
    }
}

// Load statistics for the input checks: per block, the sum, the sum of magnitudes and the
// number of non-finite entries of its slice of f (fixed slices and a fixed tree order, so
// the totals do not depend on timing); then one block adds the partials in block order.
constexpr int kStatBlocks = 256;
__global__ __launch_bounds__(kBlock) void k_load_stats_part(const double* f, int64_t n, double* part) {
    __shared__ double ss[kBlock], sa[kBlock], sn[kBlock];
    const int64_t per = (n + kStatBlocks - 1) / kStatBlocks;
    const int64_t i0 = int64_t(blockIdx.x) * per, i1 = min(n, i0 + per);
    double s = 0.0, a = 0.0, bad = 0.0;
    for (int64_t i = i0 + threadIdx.x; i < i1; i += kBlock) {
        const double v = f[i];
        if (isfinite(v)) {
            s += v;
            a += fabs(v);
        } else {
            bad += 1.0;
        }
    }
    ss[threadIdx.x] = s;
    sa[threadIdx.x] = a;
    sn[threadIdx.x] = bad;
    __syncthreads();
    for (int o = kBlock / 2; o > 0; o >>= 1) {
        if (int(threadIdx.x) < o) {
            ss[threadIdx.x] += ss[threadIdx.x + o];
            sa[threadIdx.x] += sa[threadIdx.x + o];
            sn[threadIdx.x] += sn[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[3 * blockIdx.x] = ss[0];
        part[3 * blockIdx.x + 1] = sa[0];
        part[3 * blockIdx.x + 2] = sn[0];
    }
}

__global__ void k_load_stats_final(const double* part, double* out) {
    if (threadIdx.x != 0) return;
    double s = 0.0, a = 0.0, bad = 0.0;
    for (int b = 0; b < kStatBlocks; ++b) {
        s += part[3 * b];
        a += part[3 * b + 1];
        bad += part[3 * b + 2];
    }
    out[0] = s;
    out[1] = a;
    out[2] = bad;
}

// Leaf pass for leaf sides >= 64 (phi from the device octant table: every offset
// of a near pair, at most 2 side - 1 = 255, is a table entry).  Such leaves are the sparse
// ones of widely spread or clustered inputs: a group (the up to four leaves of one parent) holds
// a few dozen targets and its 4 x 4 block of source leaves a few hundred sources.  A wave takes
// one group.  It first copies the sources of all the group's ranges into LDS (coordinates and
// loads; the ranges' loads are independent, so their latencies overlap), then sums from LDS:
// the group's targets take T lanes each (T the power of two at or above their count, at most
// 64) of S = 64 / T slices, slice s taking every S-th staged source; a pair counts when the
// source's leaf neighbours the target's (leaf coordinates from the point coordinates), and its
// phi is a gather from the table.  The slices' sums meet by xor shuffles.  Groups with more
// than kStageCap sources are summed in chunks of that many.  L2P (T_tfi = T_ofs^T) and the
// caller-order write are as in k_near.
constexpr int kStageCap = 512;
constexpr int kStagedWaves = 4;
constexpr int kStageRound = 8;   // staged elements per lane with their loads in flight together

template <int P>
__global__ __launch_bounds__(64 * kStagedWaves) void k_near_staged(
    int32_t q0, int32_t q1, const NearGroup* groups, const int4* ents, const int32_t* box_pt0, const int32_t* box_pt1,
    const uint64_t* box_key, const int32_t* box_inst, int64_t side, const int2* pts, const double* fs,
    const int32_t* perm_local, const ExecPtrs* tab_ptrs, ExecPtrs single, const double* U,
    const double* leafT, const uint8_t* far_inst, const double* phi_oct_tab) {
    __shared__ int2 s_xy[kStagedWaves][kStageCap];
    __shared__ double s_f[kStagedWaves][kStageCap];
    const int lane = int(threadIdx.x) & 63, wave = int(threadIdx.x) >> 6;
    const int32_t q = q0 + int32_t(blockIdx.x) * kStagedWaves + wave;
    if (q >= q1) return;   // uniform over the wave; no block-wide barrier below
    const int32_t qq = uniform(q);
    int2* sxy = s_xy[wave];
    double* sf = s_f[wave];
    const cptr<int4_t> E = as_const(reinterpret_cast<const int4_t*>(ents)) + size_t(qq) * kNearEntries;
    const int32_t leaf0 = uniform(groups[qq].leaf0), nleaf = uniform(groups[qq].nleaf);
    const int32_t ne = uniform(groups[qq].ne);
    int ls = 0;
    while ((int64_t(1) << ls) < side) ++ls;
    const int32_t t0 = uniform(box_pt0[leaf0]), t_end = uniform(box_pt1[leaf0 + nleaf - 1]);
    const int32_t k_inst = uniform(box_inst[leaf0]);
    const bool far = far_inst[k_inst] != 0;
    const ExecPtrs eio = tab_ptrs ? tab_ptrs[k_inst] : single;
    double* u = eio.u;
    const bool sorted_out = eio.sorted != 0;   // u indexed by sorted point
    const int32_t tgt0 = eio.tgt0;
    // first points of the group's leaves, to find each target's leaf
    int32_t bnd1 = t_end, bnd2 = t_end, bnd3 = t_end;
    if (nleaf > 1) bnd1 = uniform(box_pt0[leaf0 + 1]);
    if (nleaf > 2) bnd2 = uniform(box_pt0[leaf0 + 2]);
    if (nleaf > 3) bnd3 = uniform(box_pt0[leaf0 + 3]);
    // entries: start offset of each range in the concatenated source list
    int32_t e_p0[kNearEntries], e_off[kNearEntries + 1];
    e_off[0] = 0;
    #pragma unroll
    for (int e = 0; e < kNearEntries; ++e) {
        int32_t a = 0, b = 0;
        if (e < ne) {
            const int4_t en = E[e];
            a = en.x;
            b = en.y;
        }
        e_p0[e] = a;
        e_off[e + 1] = e_off[e] + (b - a);
    }
    const int32_t ns = e_off[kNearEntries];
    const int32_t nt = t_end - t0;
    int T = 1;
    while (T < nt && T < 64) T <<= 1;
    const int S = 64 / T, tl = lane & (T - 1), sl = lane / T;
    for (int32_t i0 = t0; i0 < t_end; i0 += T) {
        const int32_t i = i0 + tl;
        const bool valid = i < t_end;
        const int32_t ii = valid ? i : t0;
        const int2 pi = pts[ii];
        const int tlx = pi.x >> ls, tly = pi.y >> ls;
        double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
        for (int32_t c0 = 0; c0 < ns; c0 += kStageCap) {
            const int32_t c1 = min(ns, c0 + kStageCap);
            // stage sources [c0, c1) of the concatenated list (after the wave's reads of the
            // previous chunk: other lanes' reads, so a fence and not only program order)
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            // eight elements per lane and round, every load issued before the stores: element t of
            // the concatenated list is point t + (e_p0[e] - e_off[e]) of the range e holding it
            for (int32_t base = c0; base < c1; base += 64 * kStageRound) {
                int2 v[kStageRound];
                double w[kStageRound];
                #pragma unroll
                for (int r = 0; r < kStageRound; ++r) {
                    const int32_t t = base + r * 64 + lane;
                    int32_t shift = e_p0[0] - e_off[0];
                    #pragma unroll
                    for (int e = 1; e < kNearEntries; ++e)
                        if (t >= e_off[e]) shift = e_p0[e] - e_off[e];
                    const int32_t j = t < c1 ? t + shift : t0;
                    v[r] = pts[j];
                    w[r] = fs[j];
                }
                #pragma unroll
                for (int r = 0; r < kStageRound; ++r) {
                    const int32_t t = base + r * 64 + lane;
                    if (t < c1) {
                        sxy[t - c0] = v[r];
                        sf[t - c0] = w[r];
                    }
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            const int32_t m = c1 - c0;
            auto pair = [&](int32_t j) -> double {
                const int2 pj = sxy[j];
                const int dlx = (pj.x >> ls) - tlx, dly = (pj.y >> ls) - tly;
                const bool nb = dlx >= -1 && dlx <= 1 && dly >= -1 && dly <= 1;
                const int dx = abs(pi.x - pj.x), dy = abs(pi.y - pj.y);
                const int hi = max(dx, dy), lo = min(dx, dy);
                const double ph = nb ? phi_oct_tab[hi * (hi + 1) / 2 + lo] : 0.0;
                return ph * sf[j];
            };
            int32_t j = sl;
            for (; j + 3 * S < m; j += 4 * S) {
                a0 += pair(j);
                a1 += pair(j + S);
                a2 += pair(j + 2 * S);
                a3 += pair(j + 3 * S);
            }
            for (; j < m; j += S) a0 += pair(j);
        }
        if (far) {
            const int c = (ii >= bnd1) + (ii >= bnd2) + (ii >= bnd3);
            const int32_t leaf = leaf0 + c;
            const int64_t loc = int64_t(pi.x - tlx * side) + side * int64_t(pi.y - tly * side);
            const double* tlp = leafT + loc * P;
            const double* uh = U + size_t(leaf) * P;
            for (int p = sl; p < P; p += S) a1 += tlp[p] * uh[p];
        }
        double acc = (a0 + a1) + (a2 + a3);
        for (int o = T; o < 64; o <<= 1) acc += __shfl_xor(acc, o, 64);
        const int32_t pout = perm_local[ii];
        if (valid && sl == 0 && pout >= tgt0) u[sorted_out ? int64_t(ii) : int64_t(pout - tgt0)] = acc;
    }
}

// ---- adaptive tree passes ----------------------------------------------------------------

__device__ inline double readlane_d(double v, int k) {
    const int2_t w = __builtin_bit_cast(int2_t, v);
    return __builtin_bit_cast(double, int2_t{__builtin_amdgcn_readlane(w.x, k), __builtin_amdgcn_readlane(w.y, k)});
}

// Lower-left corner of box g in its instance's root coordinates (root side 2^D).
__device__ inline int2 box_corner(const uint64_t* box_key, const int8_t* box_lev, int32_t g, int D) {
    const uint64_t k = box_key[g];
    const int sh = D - int(box_lev[g]);
    return make_int2(int32_t(compact_bits(k)) << sh, int32_t(compact_bits(k >> 1)) << sh);
}

// P2L (X lists): one wave per box tau, lane p for skeleton point p of tau; the points of each
// leaf of X(tau) are read 64 at a time (one coalesced load per lane) and broadcast lane by
// lane, every skeleton lane adding phi(y_p - x_j) f_j.  The sum joins tau's incoming
// expansion, which M2L wrote before and L2L reads after (the incoming skeleton is the
// outgoing one, T_ifi = T_ofo^T).
__global__ __launch_bounds__(kBlock) void k_p2l(int32_t nx, const int32_t* xitems, AdaptiveLists L,
                                                const int32_t* box_pt0, const int32_t* box_pt1,
                                                const uint64_t* box_key, const int8_t* box_lev,
                                                const int32_t* box_inst, const InstInfo* inst, const OpsPtrs* ops,
                                                const int2* pts, const double* fs, double* U,
                                                const double* phi_oct_tab, const PhiFar* phi_far) {
    constexpr int P = kRankPad;
    const int lane = int(threadIdx.x) & 63, wave = int(threadIdx.x) >> 6;
    const int32_t q = int32_t(blockIdx.x) * kWaves + wave;
    if (q >= nx) return;
    const int32_t tau = uniform(xitems[q]);
    const int32_t k_inst = uniform(box_inst[tau]);
    const int D = uniform(inst[k_inst].D), Lf = uniform(inst[k_inst].L), opi = uniform(inst[k_inst].ops);
    const int h = Lf - int(box_lev[tau]);
    const int rank = uniform(ops[opi].rank[h]);
    const int2 c = box_corner(box_key, box_lev, tau, D);
    const bool on = lane < rank;
    int2 y = c;
    if (on) {
        const int32_t* sk = ops[opi].skel + (size_t(h) * P + lane) * 2;
        y = make_int2(c.x + sk[0], c.y + sk[1]);
    }
    double acc = 0.0;
    const int32_t e0 = uniform(L.off[2][tau]), e1 = uniform(L.off[2][tau + 1]);
    for (int32_t e = e0; e < e1; ++e) {
        const int32_t sg = uniform(L.ent[2][e]);
        const int32_t j0 = uniform(box_pt0[sg]), j1 = uniform(box_pt1[sg]);
        for (int32_t base = j0; base < j1; base += 64) {
            const int32_t j = base + lane;
            const bool ok = j < j1;
            const int2 pj = ok ? pts[j] : make_int2(0, 0);
            const double fj = ok ? fs[j] : 0.0;
            const int m = min(64, j1 - base);
            for (int k = 0; k < m; ++k) {
                const int32_t xk = __builtin_amdgcn_readlane(pj.x, k), yk = __builtin_amdgcn_readlane(pj.y, k);
                const double fk = readlane_d(fj, k);
                acc += phi_oct(abs(y.x - xk), abs(y.y - yk), phi_oct_tab, phi_far) * fk;
            }
        }
    }
    if (on && e1 > e0) U[size_t(tau) * P + lane] += acc;
}

// Near field of the adaptive leaves (Section 8.2 step 5 on the adaptive tree), one wave per
// leaf tau: the sources are the points of the U-list leaves and, for the W-list boxes, their
// skeleton points carrying their outgoing expansions (M2P: phi(x_i - y_p) q_p).  The wave
// first writes a descriptor of each list entry into LDS (up to 64 at a time: kind, start,
// corner, and the prefix sum of the entry lengths), then copies the sources into LDS in
// chunks of kStageCap, each lane finding an element's entry by bisection over the prefix sums
// and keeping kStageRound loads in flight, and sums from LDS as k_near_staged does (T lanes per
// target, S slices).  L2P runs at each point's finest box (its incoming expansion holds those
// of the adaptive leaf relayed by L2L), then the caller-order write.
constexpr int kAdWaves = 4;

struct AdWaveLds {
    int2 xy[kStageCap];
    double f[kStageCap];
    int32_t off[65];   // prefix sums of the entry lengths of the batch
    int32_t a[64];     // U entry: first point; W entry: box
    int32_t h[64];     // W entry: height of the box (its skeleton); U entry: -1
    int2 c[64];        // W entry: corner of the box
};

template <int P>
__global__ __launch_bounds__(64 * kAdWaves) void k_near_adaptive(
    int32_t nitems, const int32_t* items, AdaptiveLists L, const int32_t* box_pt0, const int32_t* box_pt1,
    const uint64_t* box_key, const int8_t* box_lev, const int32_t* box_inst, const InstInfo* inst,
    const OpsPtrs* ops, const int2* pts, const double* fs, const double* Q, const int32_t* pt_box, const double* U,
    const int32_t* perm_local, const ExecPtrs* tab_ptrs, ExecPtrs single,
    const uint8_t* far_inst, const double* phi_oct_tab, const PhiFar* phi_far) {
    __shared__ AdWaveLds s_w[kAdWaves];
    const int lane = int(threadIdx.x) & 63, wave = int(threadIdx.x) >> 6;
    const int32_t q = int32_t(blockIdx.x) * kAdWaves + wave;
    if (q >= nitems) return;   // uniform over the wave; no block-wide barrier below
    AdWaveLds& S = s_w[wave];
    const int32_t tau = uniform(items[q]);
    const int32_t k_inst = uniform(box_inst[tau]);
    const int D = uniform(inst[k_inst].D), Lf = uniform(inst[k_inst].L), opi = uniform(inst[k_inst].ops);
    const OpsPtrs& O = ops[opi];
    const int32_t side0 = int32_t(O.side);
    const double* leafT = O.leafT;
    const int32_t* skel = O.skel;
    const bool far = far_inst[k_inst] != 0;
    const ExecPtrs eio = tab_ptrs ? tab_ptrs[k_inst] : single;
    double* u = eio.u;
    const bool sorted_out = eio.sorted != 0;   // u indexed by sorted point
    const int32_t tgt0 = eio.tgt0;
    const int32_t t0 = uniform(box_pt0[tau]), t_end = uniform(box_pt1[tau]);
    const int32_t u0 = uniform(L.off[0][tau]), nu = uniform(L.off[0][tau + 1]) - u0;
    const int32_t w0 = uniform(L.off[1][tau]), nw = uniform(L.off[1][tau + 1]) - w0;
    const int32_t ne = nu + nw;
    const int32_t nt = t_end - t0;
    int T = 1;
    while (T < nt && T < 64) T <<= 1;
    const int Sl = 64 / T, tl = lane & (T - 1), sl = lane / T;
    auto wave_sync = [] {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    };
    for (int32_t i0 = t0; i0 < t_end; i0 += T) {
        const int32_t i = i0 + tl;
        const bool valid = i < t_end;
        const int32_t ii = valid ? i : t0;
        const int2 pi = pts[ii];
        double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
        for (int32_t eb = 0; eb < ne; eb += 64) {
            // descriptors of entries eb .. eb + 63
            const int32_t e = eb + lane;
            int32_t len = 0, a = 0, hh = -1;
            int2 cc = make_int2(0, 0);
            if (e < nu) {
                const int32_t sg = L.ent[0][u0 + e];
                a = box_pt0[sg];
                len = box_pt1[sg] - a;
            } else if (e < ne) {
                const int32_t d = L.ent[1][w0 + e - nu];
                hh = Lf - int(box_lev[d]);
                len = O.rank[hh];
                a = d;
                cc = box_corner(box_key, box_lev, d, D);
            }
            int32_t incl = len;
            #pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const int32_t v = __shfl_up(incl, o, 64);
                if (lane >= o) incl += v;
            }
            const int32_t total = __builtin_amdgcn_readlane(incl, 63);
            wave_sync();   // the previous batch's reads of the descriptors are done
            S.off[lane] = incl - len;
            if (lane == 63) S.off[64] = total;
            S.a[lane] = a;
            S.h[lane] = hh;
            S.c[lane] = cc;
            for (int32_t c0 = 0; c0 < total; c0 += kStageCap) {
                const int32_t c1 = min(total, c0 + kStageCap);
                wave_sync();   // descriptors written; the previous chunk's sums are done
                for (int32_t base = c0; base < c1; base += 64 * kStageRound) {
                    int2 v[kStageRound];
                    double w[kStageRound];
                    #pragma unroll
                    for (int r = 0; r < kStageRound; ++r) {
                        const int32_t t = base + r * 64 + lane;
                        v[r] = make_int2(0, 0);
                        w[r] = 0.0;
                        if (t < c1) {
                            int lo = 0, hi = 63;   // last entry starting at or before t
                            while (lo < hi) {
                                const int mid = (lo + hi + 1) >> 1;
                                if (S.off[mid] <= t) lo = mid;
                                else hi = mid - 1;
                            }
                            const int32_t k = t - S.off[lo];
                            const int32_t hk = S.h[lo];
                            if (hk < 0) {
                                v[r] = pts[S.a[lo] + k];
                                w[r] = fs[S.a[lo] + k];
                            } else {
                                const int32_t* sk = skel + (size_t(hk) * P + k) * 2;
                                const int2 c = S.c[lo];
                                v[r] = make_int2(c.x + sk[0], c.y + sk[1]);
                                w[r] = Q[size_t(S.a[lo]) * P + k];
                            }
                        }
                    }
                    #pragma unroll
                    for (int r = 0; r < kStageRound; ++r) {
                        const int32_t t = base + r * 64 + lane;
                        if (t < c1) {
                            S.xy[t - c0] = v[r];
                            S.f[t - c0] = w[r];
                        }
                    }
                }
                wave_sync();
                const int32_t m = c1 - c0;
                auto pair = [&](int32_t j) -> double {
                    const int2 pj = S.xy[j];
                    return phi_oct(abs(pi.x - pj.x), abs(pi.y - pj.y), phi_oct_tab, phi_far) * S.f[j];
                };
                int32_t j = sl;
                for (; j + 3 * Sl < m; j += 4 * Sl) {
                    a0 += pair(j);
                    a1 += pair(j + Sl);
                    a2 += pair(j + 2 * Sl);
                    a3 += pair(j + 3 * Sl);
                }
                for (; j < m; j += Sl) a0 += pair(j);
            }
        }
        if (far) {
            const int32_t b = pt_box[ii];
            const int64_t loc = int64_t(pi.x & (side0 - 1)) + int64_t(side0) * int64_t(pi.y & (side0 - 1));
            const double* tlp = leafT + loc * P;
            const double* uh = U + size_t(b) * P;
            for (int p = sl; p < P; p += Sl) a1 += tlp[p] * uh[p];
        }
        double acc = (a0 + a1) + (a2 + a3);
        for (int o = T; o < 64; o <<= 1) acc += __shfl_xor(acc, o, 64);
        const int32_t pout = perm_local[ii];
        if (valid && sl == 0 && pout >= tgt0) u[sorted_out ? int64_t(ii) : int64_t(pout - tgt0)] = acc;
    }
}

// Brute-force sum over all sources for blocks of 256 targets; sources staged through LDS.
__global__ __launch_bounds__(kBlock) void k_direct(int64_t nt, const int2* txy, int64_t ns, const int2* sxy,
                                                    const double* f, const double* phi_oct, const PhiFar* far,
                                                    double* u) {
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
            if (hi <= kPhiDeviceRadius) ph = phi_oct[hi * (hi + 1) / 2 + lo];
            else ph = phi_expansion_dev(double(hi), double(lo), far);
            acc += ph * sf[k];
        }
        __syncthreads();
    }
    if (valid) u[t] = acc;
}

}  // namespace

hipError_t upload_dslots() {
    DSlots ds{};
    for (int c = 0; c < 4; ++c) {
        const int cx = c & 1, cy = c >> 1;
        int k = 0;
        for (int dy = -2 - cy; dy <= 3 - cy; ++dy)
            for (int dx = -2 - cx; dx <= 3 - cx; ++dx) {
                if (dx >= -1 && dx <= 1 && dy >= -1 && dy <= 1) continue;
                ds.s[c][k++] = (dy + 3) * 7 + (dx + 3);
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

// Per device: compute units and the LDS a block may use (the staged P2M is set up to use it).
struct P2mDevice {
    int cus = 0, lds = 0;
};

P2mDevice p2m_device() {
    static P2mDevice dev[64];
    static std::once_flag once[64];
    int d = 0;
    if (hipGetDevice(&d) != hipSuccess || d < 0 || d >= 64) return P2mDevice{};
    std::call_once(once[d], [&] {
        int cus = 0, lds = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, d) != hipSuccess ||
            hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, d) != hipSuccess ||
            hipFuncSetAttribute(reinterpret_cast<const void*>(&k_p2m_lds<kRankPad>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, lds) != hipSuccess) {
            (void)hipGetLastError();
            return;   // the unstaged kernel serves every side
        }
        dev[d] = P2mDevice{cus, lds};
    });
    return dev[d];
}

void launch_p2m(int32_t leaf0, int32_t leaf1, const int32_t* box_pt0, const int32_t* box_pt1, const uint64_t* box_key,
                int64_t side, const int32_t* pts, const ExecPtrs* tab, const ExecPtrs& single,
                const int32_t* perm_local, const int32_t* pinst, double* fs, const double* leafT, double* Q,
                double avg_pts, hipStream_t st) {
    if (leaf1 <= leaf0) return;
    const size_t lds = size_t(side * side) * kRankPad * sizeof(double);
    const P2mDevice dv = p2m_device();
    if (dv.cus > 0 && lds <= size_t(dv.lds)) {
        const int per_cu = std::max(1, std::min(2, int(size_t(dv.lds) / lds)));
        const int64_t per_block = (kP2mThreads / 64) * kP2mLeaves;
        const int64_t want = (int64_t(leaf1 - leaf0) + per_block - 1) / per_block;
        const int64_t grid = std::max<int64_t>(1, std::min<int64_t>(want, int64_t(dv.cus) * per_cu));
        hipLaunchKernelGGL(k_p2m_lds<kRankPad>, dim3(unsigned(grid)), dim3(kP2mThreads), lds, st, leaf0, leaf1,
                           box_pt0, box_pt1, box_key, side, reinterpret_cast<const int2*>(pts), tab, single,
                           perm_local, pinst, fs, leafT, Q);
        return;
    }
    if (avg_pts <= double(kP2mSparsePoints)) {
        // few points per leaf: eight leaves per wave, T_ofs rows from global memory
        const int64_t per_block = (kP2mThreads / 64) * kP2mLeaves;
        const int64_t grid = std::max<int64_t>(1, (int64_t(leaf1 - leaf0) + per_block - 1) / per_block);
        hipLaunchKernelGGL((k_p2m_lds<kRankPad, false>), dim3(unsigned(grid)), dim3(kP2mThreads), 0, st, leaf0, leaf1,
                           box_pt0, box_pt1, box_key, side, reinterpret_cast<const int2*>(pts), tab, single,
                           perm_local, pinst, fs, leafT, Q);
        return;
    }
    hipLaunchKernelGGL(k_p2m<kRankPad>, dim3(grid_for(leaf1 - leaf0, kWaves)), dim3(kBlock), 0, st, leaf0, leaf1,
                       box_pt0, box_pt1, box_key, side, reinterpret_cast<const int2*>(pts), tab, single,
                       perm_local, pinst, fs, leafT, Q);
}

void launch_m2m(const BoxTile* tiles, int32_t ntiles, const int32_t* box_child, const OpsPtrs* ops, double* Q,
                int32_t zrow, hipStream_t st) {
    if (ntiles <= 0) return;
    if (ntiles <= kFineM2mTiles) {
        hipLaunchKernelGGL(k_m2m_fine, dim3(unsigned(ntiles) * 12u), dim3(kBlock), 0, st, tiles, box_child, ops, Q,
                           zrow);
        return;
    }
    int64_t g = std::min<int64_t>(ntiles, 8192);
    g = std::max<int64_t>(8, (g + 7) / 8 * 8);
    hipLaunchKernelGGL(k_m2m, dim3(static_cast<unsigned>(g)), dim3(kBlock), 0, st, tiles, ntiles, box_child, ops, Q,
                       zrow);
}

void launch_l2l(const BoxTile* tiles, int32_t ntiles, const int32_t* box_list, const int32_t* box_parent,
                const OpsPtrs* ops, double* U, int32_t zrow, const int8_t* role, hipStream_t st) {
    if (ntiles <= 0) return;
    if (ntiles <= kFineL2lTiles) {
        hipLaunchKernelGGL(k_l2l_fine, dim3(unsigned(ntiles) * 12u), dim3(kBlock), 0, st, tiles, box_list, box_parent,
                           ops, U, zrow, role);
        return;
    }
    int64_t g = std::min<int64_t>(ntiles, 8192);
    g = std::max<int64_t>(8, (g + 7) / 8 * 8);
    hipLaunchKernelGGL(k_l2l, dim3(static_cast<unsigned>(g)), dim3(kBlock), 0, st, tiles, ntiles, box_list,
                       box_parent, ops, U, zrow, role);
}

void launch_m2l(const BoxTile* tiles, const int32_t* ntiles_dev, int32_t max_tiles, const int32_t* box_list,
                const int32_t* il27, const OpsPtrs* ops, const double* Q, int32_t zrow, double* U, hipStream_t st) {
    if (max_tiles <= 0) return;
    int64_t g = std::min<int64_t>(max_tiles, 8192);
    g = std::max<int64_t>(8, (g + 7) / 8 * 8);
    hipLaunchKernelGGL(k_m2l, dim3(static_cast<unsigned>(g)), dim3(kBlock), 0, st, tiles, ntiles_dev, box_list, il27,
                       ops, Q, zrow, U);
}

void launch_split_q(const double* Q, int32_t nrows, float* Qh, float* Ql, double* qs, hipStream_t st) {
    if (nrows <= 0) return;
    hipLaunchKernelGGL(k_split_q, dim3(grid_for(int64_t(nrows) * 64)), dim3(kBlock), 0, st, Q, nrows, Qh, Ql, qs);
}

void launch_m2l_mixed(const BoxTile* tiles, const int32_t* ntiles_dev, int32_t max_tiles, const int32_t* box_list,
                      const int32_t* il27, const OpsPtrs* ops, const float* Qh, const float* Ql, const double* qs,
                      int32_t zrow, double* U, hipStream_t st) {
    if (max_tiles <= 0) return;
    int64_t g = std::min<int64_t>(max_tiles, 8192);
    g = std::max<int64_t>(8, (g + 7) / 8 * 8);
    hipLaunchKernelGGL(k_m2l_mixed, dim3(static_cast<unsigned>(g)), dim3(kBlock), 0, st, tiles, ntiles_dev, box_list,
                       il27, ops, Qh, Ql, qs, zrow, U);
}

void launch_split_q_bf16(const double* Q, int32_t nrows, uint16_t* Qb, double* qs, hipStream_t st) {
    if (nrows <= 0) return;
    hipLaunchKernelGGL(k_split_q_bf16, dim3(grid_for(int64_t(nrows) * 8)), dim3(kBlock), 0, st, Q, nrows, Qb, qs);
}

void launch_m2l_bf16(const BoxTile* tiles, const int32_t* ntiles_dev, int32_t max_tiles, const int32_t* box_list,
                     const int32_t* il27, const OpsPtrs* ops, const uint16_t* Qb, const double* qs, int32_t zrow,
                     double* U, hipStream_t st) {
    if (max_tiles <= 0) return;
    int64_t g = std::min<int64_t>(max_tiles, 8192);
    g = std::max<int64_t>(8, (g + 7) / 8 * 8);
    hipLaunchKernelGGL(k_m2l_bf16, dim3(static_cast<unsigned>(g)), dim3(kBf16Block), 0, st, tiles, ntiles_dev,
                       box_list, il27, ops, Qb, qs, zrow, U);
}

void launch_near(int32_t q0, int32_t q1, const NearGroup* groups, const int4* ents, const int32_t* box_pt0,
                 const int32_t* box_pt1, const uint64_t* box_key, const int32_t* box_inst, int64_t side,
                 const int32_t* pts, const uint32_t* pkey, const double* fs, const int32_t* perm_local,
                 const ExecPtrs* tab, const ExecPtrs& single, const double* U, const double* leafT,
                 const double* leafTt, const uint8_t* far_inst, const double* phi_oct, const PhiFar* phi_far,
                 hipStream_t st) {
    if (q1 <= q0) return;
    if (side <= 32 && leafTt == nullptr) throw std::logic_error("near field without its coefficient-major T_ofs");
    // with an LDS table: persistent blocks, as many as fit on the device at once, so that
    // each builds its table once and then walks many groups; else one group per wave
    auto grid = [&](const void* fn, int threads, size_t lds, bool persistent) {
        unsigned g = std::min<unsigned>(grid_for(q1 - q0, threads / 64), 8192u);
        const int cus = p2m_device().cus;
        int per = 0;
        if (!persistent) return g;
        if (cus > 0 && hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, threads, lds) == hipSuccess && per > 0)
            g = std::min<unsigned>(g, unsigned(cus) * unsigned(per));
        else
            (void)hipGetLastError();
        return std::max(g, 1u);
    };
    const int2* p2 = reinterpret_cast<const int2*>(pts);
    if (side <= 16) {
        const int W = int(4 * side - 1);
        const size_t lds = 0;   // the table is a fixed-size shared array
        if (W * W > kNearTabMax) throw std::logic_error("near-field window table larger than its array");
        constexpr int nt = near_threads(kWindow);
        const unsigned g = grid(reinterpret_cast<const void*>(&k_near<kRankPad, kWindow>), nt, lds, true);
        hipLaunchKernelGGL((k_near<kRankPad, kWindow>), dim3(g), dim3(nt), lds, st, q0, q1, groups, ents,
                           box_pt0, box_pt1, box_key, box_inst, side, W, p2, pkey, fs, perm_local, tab, single, U,
                           leafT, leafTt, far_inst, phi_oct, phi_far);
    } else if (side <= 32) {
        const int W = int(2 * side);
        const size_t lds = 0;
        if (W * W > kNearTabMax) throw std::logic_error("near-field quadrant table larger than its array");
        constexpr int nt = near_threads(kQuad);
        const unsigned g = grid(reinterpret_cast<const void*>(&k_near<kRankPad, kQuad>), nt, lds, true);
        hipLaunchKernelGGL((k_near<kRankPad, kQuad>), dim3(g), dim3(nt), lds, st, q0, q1, groups, ents,
                           box_pt0, box_pt1, box_key, box_inst, side, W, p2, pkey, fs, perm_local, tab, single, U,
                           leafT, leafTt, far_inst, phi_oct, phi_far);
    } else {
        // every near offset (at most 2 side - 1 <= 255) lies inside the device octant table
        if (2 * side - 1 > kPhiDeviceRadius) throw std::logic_error("leaf wider than the near-field table allows");
        const unsigned g = unsigned((q1 - q0 + kStagedWaves - 1) / kStagedWaves);
        hipLaunchKernelGGL(k_near_staged<kRankPad>, dim3(g), dim3(64 * kStagedWaves), 0, st, q0, q1, groups, ents,
                           box_pt0, box_pt1, box_key, box_inst, side, p2, fs, perm_local, tab, single,
                           U, leafT, far_inst, phi_oct);
    }
}

size_t load_stats_scratch_bytes() { return size_t(kStatBlocks) * 3 * sizeof(double); }

void launch_load_stats(const double* f, int64_t n, double* scratch, double* out3, hipStream_t st) {
    hipLaunchKernelGGL(k_load_stats_part, dim3(kStatBlocks), dim3(kBlock), 0, st, f, n, scratch);
    hipLaunchKernelGGL(k_load_stats_final, dim3(1), dim3(64), 0, st, scratch, out3);
}

void launch_phi_extend(double* oct, int r0, int r1, const PhiFar* far, hipStream_t st) {
    if (r1 <= r0) return;
    const int64_t n = int64_t(r1 + 1) * (r1 + 2) / 2 - int64_t(r0 + 1) * (r0 + 2) / 2;
    hipLaunchKernelGGL(k_phi_extend, dim3(grid_for(n)), dim3(kBlock), 0, st, oct, r0, r1, far);
}

void launch_p2l(int32_t nx, const int32_t* xitems, const AdaptiveLists& lists, const int32_t* box_pt0,
                const int32_t* box_pt1, const uint64_t* box_key, const int8_t* box_lev, const int32_t* box_inst,
                const InstInfo* inst, const OpsPtrs* ops, const int32_t* pts, const double* fs, double* U,
                const double* phi_oct, const PhiFar* phi_far, hipStream_t st) {
    if (nx <= 0) return;
    const unsigned g = unsigned((nx + kWaves - 1) / kWaves);
    hipLaunchKernelGGL(k_p2l, dim3(g), dim3(kBlock), 0, st, nx, xitems, lists, box_pt0, box_pt1, box_key, box_lev,
                       box_inst, inst, ops, reinterpret_cast<const int2*>(pts), fs, U, phi_oct, phi_far);
}

void launch_near_adaptive(int32_t nitems, const int32_t* items, const AdaptiveLists& lists, const int32_t* box_pt0,
                          const int32_t* box_pt1, const uint64_t* box_key, const int8_t* box_lev,
                          const int32_t* box_inst, const InstInfo* inst, const OpsPtrs* ops, const int32_t* pts,
                          const double* fs, const double* Q, const int32_t* pt_box, const double* U,
                          const int32_t* perm_local, const ExecPtrs* tab, const ExecPtrs& single,
                          const uint8_t* far_inst, const double* phi_oct, const PhiFar* phi_far, hipStream_t st) {
    if (nitems <= 0) return;
    const unsigned g = unsigned((nitems + kAdWaves - 1) / kAdWaves);
    hipLaunchKernelGGL(k_near_adaptive<kRankPad>, dim3(g), dim3(64 * kAdWaves), 0, st, nitems, items, lists, box_pt0,
                       box_pt1, box_key, box_lev, box_inst, inst, ops, reinterpret_cast<const int2*>(pts), fs, Q,
                       pt_box, U, perm_local, tab, single, far_inst, phi_oct, phi_far);
}

void launch_direct(int64_t nt, const int32_t* txy, int64_t ns, const int32_t* sxy, const double* f,
                   const double* phi_oct, const PhiFar* far, double* u, hipStream_t st) {
    if (nt <= 0) return;
    hipLaunchKernelGGL(k_direct, dim3(grid_for(nt)), dim3(kBlock), 0, st, nt, reinterpret_cast<const int2*>(txy), ns,
                       reinterpret_cast<const int2*>(sxy), f, phi_oct, far, u);
}

}  // namespace lfmm
