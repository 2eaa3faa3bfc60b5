// Quadtree construction on the GPU for a forest of instances (Section 6, Definition 6.1).
//
// Points of every instance are shifted to the origin of their root box [0, 2^D)^2 and given
// keys (instance << 2 Dmax) | Morton(x, y) (first coordinate in the even bits), so one sort
// orders all instances at once and every box of every level is a contiguous run of points.
// The leaf level L of an instance is the smallest level whose boxes hold at most N_leaf of
// its points (Section 6).  The common-prefix length of consecutive keys tells, per point, at
// which levels a new box starts; one pass over the sorted keys yields L and the box count of
// every level; scans over the leaves then place every box.  Neighbour and interaction lists
// are built top-down: the boxes around a box are children of the boxes around its parent.
#include "kernels.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <utility>

namespace lfmm {

namespace {

constexpr int kBlock = 256;

__device__ inline uint64_t spread_bits(uint32_t v) {
    uint64_t x = v;
    x = (x | (x << 16)) & 0x0000FFFF0000FFFFull;
    x = (x | (x << 8)) & 0x00FF00FF00FF00FFull;
    x = (x | (x << 4)) & 0x0F0F0F0F0F0F0F0Full;
    x = (x | (x << 2)) & 0x3333333333333333ull;
    x = (x | (x << 1)) & 0x5555555555555555ull;
    return x;
}

__device__ inline uint32_t compact_bits(uint64_t x) {
    x &= 0x5555555555555555ull;
    x = (x | (x >> 1)) & 0x3333333333333333ull;
    x = (x | (x >> 2)) & 0x0F0F0F0F0F0F0F0Full;
    x = (x | (x >> 4)) & 0x00FF00FF00FF00FFull;
    x = (x | (x >> 8)) & 0x0000FFFF0000FFFFull;
    x = (x | (x >> 16)) & 0x00000000FFFFFFFFull;
    return uint32_t(x);
}

__device__ inline uint64_t morton_mask(int Dmax) {
    return (Dmax >= 32) ? ~0ull : ((1ull << (2 * Dmax)) - 1ull);
}

// levels (of a root of side 2^Dmax) at which the boxes of Morton parts a and b coincide
__device__ inline int common_levels(uint64_t a, uint64_t b, int Dmax) {
    const uint64_t x = (a ^ b) & morton_mask(Dmax);
    if (x == 0) return Dmax;
    return (__clzll(x) - (64 - 2 * Dmax)) >> 1;
}

// instance owning position i: the largest k with off[k] <= i (off has K + 1 entries)
__device__ inline int32_t find_inst(const int32_t* off, int32_t K, int64_t i) {
    int32_t lo = 0, hi = K - 1;
    while (lo < hi) {
        int32_t mid = (lo + hi + 1) >> 1;
        if (off[mid] <= i) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

inline unsigned grid_for(int64_t n, int per_block = kBlock) {
    int64_t g = (n + per_block - 1) / per_block;
    return unsigned(g < 1 ? 1 : g);
}

__global__ void k_concat(int32_t K, const int2* const* xy_tab, const int32_t* pt_off, int64_t n, int2* xyc) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t k = find_inst(pt_off, K, i);
    xyc[i] = xy_tab[k][i - pt_off[k]];
}

// {min x, min y, max x, max y} of n points into box (device), by atomics; box is set to the
// empty box first by k_extent_init on the same stream.
__global__ void k_extent_init(int32_t* box, int32_t nbox) {
    const int32_t i = int32_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < nbox) {
        box[4 * i] = INT_MAX;
        box[4 * i + 1] = INT_MAX;
        box[4 * i + 2] = INT_MIN;
        box[4 * i + 3] = INT_MIN;
    }
}

__global__ void k_extent(const int2* xy, int64_t n, int32_t* box) {
    int v[4] = {INT_MAX, INT_MAX, INT_MIN, INT_MIN};
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
        const int2 p = xy[i];
        v[0] = min(v[0], p.x); v[1] = min(v[1], p.y);
        v[2] = max(v[2], p.x); v[3] = max(v[3], p.y);
    }
    #pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        v[0] = min(v[0], __shfl_xor(v[0], o, 64));
        v[1] = min(v[1], __shfl_xor(v[1], o, 64));
        v[2] = max(v[2], __shfl_xor(v[2], o, 64));
        v[3] = max(v[3], __shfl_xor(v[3], o, 64));
    }
    if ((threadIdx.x & 63) == 0) {
        atomicMin(&box[0], v[0]);
        atomicMin(&box[1], v[1]);
        atomicMax(&box[2], v[2]);
        atomicMax(&box[3], v[3]);
    }
}

// v = {min x, min y, max x, max y} over the block: wave shuffles, then the four waves
// through LDS; thread 0 gets the result in v and true
__device__ inline bool block_minmax4(int v[4]) {
    #pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        v[0] = min(v[0], __shfl_xor(v[0], o, 64));
        v[1] = min(v[1], __shfl_xor(v[1], o, 64));
        v[2] = max(v[2], __shfl_xor(v[2], o, 64));
        v[3] = max(v[3], __shfl_xor(v[3], o, 64));
    }
    __shared__ int s[kBlock / 64][4];
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0)
        for (int q = 0; q < 4; ++q) s[wave][q] = v[q];
    __syncthreads();
    if (threadIdx.x != 0) return false;
    for (int q = 0; q < 4; ++q) v[q] = s[0][q];
    for (int w = 1; w < kBlock / 64; ++w) {
        v[0] = min(v[0], s[w][0]); v[1] = min(v[1], s[w][1]);
        v[2] = max(v[2], s[w][2]); v[3] = max(v[3], s[w][3]);
    }
    return true;
}

__global__ void k_bbox_chunks(const int2* xy, const Chunk* chunks, int32_t* part, int32_t* dmax) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *dmax = 0;   // the deepest root box, raised by k_bbox_final
    const Chunk c = chunks[blockIdx.x];
    int v[4] = {INT_MAX, INT_MAX, INT_MIN, INT_MIN};
    // all of the thread's points loaded before any is used (one wait, not one per point)
    constexpr int kIt = kChunk / kBlock;
    int2 q[kIt];
    #pragma unroll
    for (int it = 0; it < kIt; ++it) {
        const int32_t i = c.begin + it * kBlock + int32_t(threadIdx.x);
        q[it] = i < c.end ? xy[i] : xy[c.begin];   // a chunk's first point stands in past its end
    }
    #pragma unroll
    for (int it = 0; it < kIt; ++it) {
        v[0] = min(v[0], q[it].x); v[1] = min(v[1], q[it].y);
        v[2] = max(v[2], q[it].x); v[3] = max(v[3], q[it].y);
    }
    if (block_minmax4(v))
        for (int q = 0; q < 4; ++q) part[size_t(blockIdx.x) * 4 + q] = v[q];
}

// One block per instance: its chunks' partial boxes reduced by the block, written to bbox
// (host memory) and as the instance's root box, depth D (the smallest with 2^D >= extent),
// point range and N_leaf (max_leaf, or 0 when the host sets it later) into inst, for the
// kernels up to the level statistics; the deepest D goes to dmax.
__global__ void k_bbox_final(const int32_t* part, const int32_t* chunk_first, const int32_t* pt_off,
                             int32_t max_leaf, int32_t* bbox, InstInfo* inst, int32_t* dmax) {
    const int32_t k = int32_t(blockIdx.x);
    int v[4] = {INT_MAX, INT_MAX, INT_MIN, INT_MIN};
    for (int32_t c = chunk_first[k] + int32_t(threadIdx.x); c < chunk_first[k + 1]; c += kBlock) {
        v[0] = min(v[0], part[4 * c]); v[1] = min(v[1], part[4 * c + 1]);
        v[2] = max(v[2], part[4 * c + 2]); v[3] = max(v[3], part[4 * c + 3]);
    }
    if (!block_minmax4(v)) return;
    for (int q = 0; q < 4; ++q) bbox[size_t(k) * 4 + q] = v[q];
    const int64_t extent = max(int64_t(v[2]) - v[0], int64_t(v[3]) - v[1]) + 1;
    int D = 0;
    while (D < 32 && (int64_t(1) << D) < extent) ++D;
    InstInfo& I = inst[k];
    I.pt0 = pt_off[k];
    I.pt1 = pt_off[k + 1];
    I.ox = v[0];
    I.oy = v[1];
    I.D = D;
    I.max_leaf = max(max_leaf, 0);
    atomicMax(dmax, D);
}

// ---- radix sort pieces shared with the key kernel: 8-bit digits, tiles of kRsTile keys ----
// (striped: item i of thread t of a tile is key tile * kRsTile + i * kBlock + t)
constexpr int kRsItems = 16;
constexpr int kRsTile = kBlock * kRsItems;

// Index of the count of digit d in tile t: digit-major (d * ntiles + t, so that one flat
// exclusive scan gives every tile's output offsets) or tile-major (t * 256 + d).
__device__ inline size_t rs_index(int d, int64_t t, int64_t ntiles, bool digit_major) {
    return digit_major ? size_t(d) * size_t(ntiles) + size_t(t) : size_t(t) * 256 + size_t(d);
}

// Digit counts of this block's tile (digits of invalid items are 256) into C.
__device__ inline void rs_count_tile(const uint32_t (&dg)[kRsItems], uint32_t* C, int64_t ntiles, bool digit_major) {
    __shared__ uint32_t cnt[256];
    cnt[threadIdx.x] = 0;
    __syncthreads();
    #pragma unroll
    for (int i = 0; i < kRsItems; ++i)
        if (dg[i] < 256u) atomicAdd(&cnt[dg[i]], 1u);
    __syncthreads();
    C[rs_index(int(threadIdx.x), blockIdx.x, ntiles, digit_major)] = cnt[threadIdx.x];
}

// Morton key (instance above it) and index of every point, one tile of kRsTile points per
// block, with the tile's counts of the lowest digit when C is given; also zeroes the nzero
// counters that the level statistics accumulate into.
__global__ void k_keys(const int2* xy, const int32_t* pt_off, int32_t K, const InstInfo* inst, const int32_t* dmax,
                       int64_t n, uint64_t* keys, uint32_t* vals, int32_t* zero, int32_t nzero, uint32_t* C,
                       int64_t ntiles, bool digit_major) {
    const int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int Dmax = (K > 1) ? *dmax : 0;   // instance bits sit above the deepest Morton code
    for (int64_t z = g; z < nzero; z += int64_t(gridDim.x) * blockDim.x) zero[z] = 0;
    // all loads of the tile first (few waves per SIMD: the latency is hidden by loads in flight)
    int2 pt[kRsItems];
    #pragma unroll
    for (int it = 0; it < kRsItems; ++it) {
        const int64_t i = int64_t(blockIdx.x) * kRsTile + int64_t(it) * kBlock + threadIdx.x;
        pt[it] = i < n ? xy[i] : make_int2(0, 0);
    }
    uint32_t dg[kRsItems];
    #pragma unroll
    for (int it = 0; it < kRsItems; ++it) {
        const int64_t i = int64_t(blockIdx.x) * kRsTile + int64_t(it) * kBlock + threadIdx.x;
        dg[it] = 256u;
        if (i >= n) continue;
        const int32_t k = (K > 1) ? find_inst(pt_off, K, i) : 0;
        const int2 p = pt[it];
        const uint32_t x = uint32_t(int64_t(p.x) - inst[k].ox), y = uint32_t(int64_t(p.y) - inst[k].oy);
        const uint64_t m = spread_bits(x) | (spread_bits(y) << 1);
        const uint64_t key = (K > 1) ? ((uint64_t(k) << (2 * Dmax)) | m) : m;
        keys[i] = key;
        vals[i] = uint32_t(i);
        dg[it] = uint32_t(key & 255u);
    }
    if (C) rs_count_tile(dg, C, ntiles, digit_major);
}

// One block per chunk of one instance.  Per sorted point: its coordinates in the instance's
// root box decoded from the Morton key (no gather of the input), its instance-local index
// and instance; the number of levels its box shares with the previous point's (-1 at the
// instance's first point), a histogram of those counts (equal values of a wave are counted
// with ballots, one LDS add per distinct value), and the levels shared with the point N_leaf
// positions ahead (a box of that level would hold more than N_leaf points).  The block adds
// its non-zero counts and its maximum to the instance's totals with device-scope atomics
// (hist: [K][kMaxLevels + 2], then maxc: [K]; zero before the launch), and the last block
// to finish (counter *done, zero before the launch) copies the totals to host memory.  Each
// thread waits for its own atomics (vector memory count zero) before the barrier that
// precedes the counter, and the totals are read back with atomics, so no device-wide fence
// is needed.
__global__ void k_level_stats(const uint64_t* keys, const uint32_t* vals, const Chunk* chunks,
                              const InstInfo* inst, int Dmax, int32_t K, int2* pts, int32_t* perm_local,
                              int32_t* pinst, int8_t* cl, int32_t* hist, int32_t R, int32_t* done,
                              int32_t* host_out) {
    constexpr int NH = kMaxLevels + 2;
    __shared__ int32_t h[NH];
    __shared__ int32_t wmax[kBlock / 64];
    __shared__ int is_last;
    const Chunk c = chunks[blockIdx.x];
    const InstInfo& I = inst[c.inst];
    const int shift = Dmax - I.D;
    const int nleaf = I.max_leaf;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (threadIdx.x < NH) h[threadIdx.x] = 0;
    __syncthreads();
    int mc = -1;
    // every key the chunk needs is loaded first (its own, the previous and the one N_leaf on)
    constexpr int kIt = kChunk / kBlock;
    uint64_t kk[kIt], kp[kIt], ka[kIt];
    uint32_t ix[kIt];
    #pragma unroll
    for (int it = 0; it < kIt; ++it) {
        const int32_t s = c.begin + it * kBlock + int32_t(threadIdx.x);
        const bool valid = s < c.end;
        kk[it] = valid ? keys[s] : 0ull;
        ix[it] = valid ? vals[s] : 0u;
        kp[it] = (valid && s != I.pt0) ? keys[s - 1] : 0ull;
        ka[it] = (valid && s + nleaf < I.pt1) ? keys[s + nleaf] : 0ull;
    }
    #pragma unroll
    for (int it = 0; it < kIt; ++it) {
        const int32_t s = c.begin + it * kBlock + int32_t(threadIdx.x);
        const bool valid = s < c.end;
        int v = -1;
        if (valid) {
            const uint64_t m = kk[it] & morton_mask(Dmax);
            pts[s] = make_int2(int32_t(compact_bits(m)), int32_t(compact_bits(m >> 1)));
            perm_local[s] = int32_t(ix[it]) - I.pt0;
            pinst[s] = c.inst;
            v = (s == I.pt0) ? -1 : common_levels(kk[it], kp[it], Dmax) - shift;
            cl[s] = int8_t(v);
            if (s + nleaf < I.pt1) mc = max(mc, common_levels(kk[it], ka[it], Dmax) - shift);
        }
        // LDS atomics straight from every lane: the few distinct levels of a wave's neighbouring
        // keys make short queues, cheaper than a chain of leader elections
        if (valid) atomicAdd(&h[v + 1], 1);
    }
    #pragma unroll
    for (int o = 32; o > 0; o >>= 1) mc = max(mc, __shfl_xor(mc, o, 64));
    if (lane == 0) wmax[wave] = mc;
    __syncthreads();
    // the block's counts go to copy blockIdx % R of the counters: with one instance split over
    // hundreds of chunks, the blocks' atomics then queue on R lines instead of one
    const size_t per = size_t(K) * (NH + 1);
    int32_t* hc = hist + size_t(blockIdx.x % unsigned(R)) * per;
    int32_t* maxc = hc + size_t(K) * NH;
    if (threadIdx.x == 0) {
        int bm = wmax[0];
        for (int w = 1; w < kBlock / 64; ++w) bm = max(bm, wmax[w]);
        if (bm >= 0) atomicMax(&maxc[c.inst], bm);
    }
    if (threadIdx.x < NH && h[threadIdx.x] != 0) atomicAdd(&hc[size_t(c.inst) * NH + threadIdx.x], h[threadIdx.x]);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) is_last = atomicAdd(done, 1) == int(gridDim.x) - 1;
    __syncthreads();
    if (is_last)
        for (size_t i = threadIdx.x; i < per; i += blockDim.x) {
            const bool is_max = i >= size_t(K) * NH;
            int32_t v = 0;
            // device-scope loads (past this compute unit's caches), all in flight together
            #pragma unroll
            for (int32_t r = 0; r < kLevelStatsCopies; ++r) {
                if (r >= R) break;
                const int32_t x = __hip_atomic_load(&hist[size_t(r) * per + i], __ATOMIC_RELAXED,
                                                    __HIP_MEMORY_SCOPE_AGENT);
                v = is_max ? max(v, x) : v + x;
            }
            host_out[i] = v;
        }
}

// One thread per (leaf, level): the leaf that starts a box of that level writes the box and
// its parent link.
__global__ void k_build_boxes(const int32_t* lscan, const int8_t* leaf_cl, const int32_t* leaf_pt0,
                              const uint64_t* leaf_key, const int32_t* leaf_inst, const InstInfo* inst, int64_t nleaf,
                              uint64_t* box_key, int32_t* box_pt0, int32_t* box_parent, int32_t* box_child,
                              int32_t* box_inst, int8_t* box_lev) {
    const int64_t b = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int lev = blockIdx.y;
    if (b >= nleaf) return;
    const int32_t k = leaf_inst[b];
    const InstInfo& I = inst[k];
    if (lev > I.L) return;
    const int c = leaf_cl[b];
    if (lev != I.L && c >= lev) return;
    const int32_t local = (lev == I.L) ? int32_t(b) - I.leaf_rank0
                                        : lscan[size_t(lev) * nleaf + b] - lscan[size_t(lev) * nleaf + I.leaf_rank0];
    const int32_t g = I.lev_base[lev] + local;
    box_key[g] = leaf_key[b] >> (2 * (I.L - lev));
    box_pt0[g] = leaf_pt0[b];
    box_inst[g] = k;
    box_lev[g] = int8_t(lev);
    for (int q = 0; q < 4; ++q) box_child[size_t(g) * 4 + q] = -1;
    if (lev == 0) {
        box_parent[g] = -1;
        return;
    }
    int32_t pl = 0;
    if (lev - 1 > 0) {
        const size_t row = size_t(lev - 1) * nleaf;
        pl = lscan[row + b] + ((c < lev - 1) ? 1 : 0) - 1 - lscan[row + I.leaf_rank0];
    }
    box_parent[g] = I.lev_base[lev - 1] + pl;
}

__global__ void k_link_boxes(const uint64_t* box_key, const int32_t* box_parent, const int32_t* box_inst,
                             const int8_t* box_lev, const InstInfo* inst, int64_t nbox, const int32_t* box_pt0,
                             int32_t* box_child, int32_t* box_pt1, double* zq, double* zu) {
    const int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (g < kRankPad) {   // the all-zero rows of Q-hat and U-hat
        zq[g] = 0.0;
        zu[g] = 0.0;
    }
    if (g >= nbox) return;
    const int32_t p = box_parent[g];
    if (p >= 0) box_child[size_t(p) * 4 + int(box_key[g] & 3ull)] = int32_t(g);
    const InstInfo& I = inst[box_inst[g]];
    const int lev = box_lev[g];
    const int32_t local = int32_t(g) - I.lev_base[lev];
    box_pt1[g] = (local + 1 < I.lev_count[lev]) ? box_pt0[g + 1] : I.pt1;
}

// index of the box with Morton key `key` among the boxes [lo, hi) of one level of one
// instance (sorted by key), or -1
__device__ inline int32_t find_box(const uint64_t* box_key, int32_t lo, int32_t hi, uint64_t key) {
    const int32_t end = hi;
    while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        if (box_key[mid] < key) lo = mid + 1;
        else hi = mid;
    }
    return (lo < end && box_key[lo] == key) ? lo : -1;
}

__device__ inline uint64_t morton2(uint32_t x, uint32_t y) { return spread_bits(x) | (spread_bits(y) << 1); }

// 3 x 3 neighbourhood of every box (slot (dy + 1) * 3 + dx + 1), one thread per (box, slot):
// the box of that cell found by search among the boxes of its level, or directly when the
// level holds every cell (its boxes are then the cells in Morton order).  No dependence
// between levels, so one launch covers all of them.
__global__ void k_neighbours(const uint64_t* box_key, const int32_t* box_inst, const int8_t* box_lev,
                             const InstInfo* inst, int64_t nbox, int32_t* nb9) {
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= nbox * 9) return;
    const int64_t g = t / 9;
    const int q = int(t - g * 9);
    int32_t r = int32_t(g);
    if (q != 4) {
        const int lev = box_lev[g];
        const InstInfo& I = inst[box_inst[g]];
        const int32_t lo = I.lev_base[lev], cnt = I.lev_count[lev];
        const uint64_t key = box_key[g];
        const int64_t x = int64_t(compact_bits(key)) + q % 3 - 1, y = int64_t(compact_bits(key >> 1)) + q / 3 - 1;
        const int64_t side = int64_t(1) << lev;
        r = -1;
        if (x >= 0 && y >= 0 && x < side && y < side) {
            const uint64_t m = morton2(uint32_t(x), uint32_t(y));
            r = (int64_t(cnt) == side * side) ? lo + int32_t(m) : find_box(box_key, lo, lo + cnt, m);
        }
    }
    nb9[t] = r;
}

// interaction list of every box of level >= 2 (Definition 6.1), one thread per (box, slot):
// the children of its parent's neighbours that are not its own neighbours, slot k being the
// k-th such cell in row-major order of the 6 x 6 block they cover (which depends on the box's
// position in its parent)
__global__ void k_interactions(const uint64_t* box_key, const int32_t* box_parent, const int32_t* box_child,
                               const int8_t* box_lev, int64_t nbox, const int32_t* nb9, int32_t* il27) {
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= nbox * kNumInteractions) return;
    const int64_t g = t / kNumInteractions;
    const int k = int(t - g * kNumInteractions);
    int32_t r = -1;
    if (box_lev[g] >= 2) {
        const uint64_t key = box_key[g];
        const int32_t bx = int32_t(compact_bits(key)), by = int32_t(compact_bits(key >> 1));
        const int cx = bx & 1, cy = by & 1;
        // the 6 x 6 block starts 2 + c cells before the box; its own neighbourhood fills rows and
        // columns 1 + c .. 3 + c of it: 6 cells in each row above, 3 in each row beside, 6 below
        const int r0 = 1 + cy, c0 = 1 + cx;
        int row, col;
        if (k < 6 * r0) {
            row = k / 6;
            col = k % 6;
        } else if (k < 6 * r0 + 9) {
            const int j = k - 6 * r0, i = j % 3;
            row = r0 + j / 3;
            col = i < c0 ? i : i + 3;
        } else {
            const int j = k - 6 * r0 - 9;
            row = r0 + 3 + j / 6;
            col = j % 6;
        }
        const int32_t x = bx + col - 2 - cx, y = by + row - 2 - cy;
        if (x >= 0 && y >= 0) {
            const int32_t ox = (x >> 1) - (bx >> 1), oy = (y >> 1) - (by >> 1);
            const int32_t q = nb9[size_t(box_parent[g]) * 9 + size_t((oy + 1) * 3 + ox + 1)];
            if (q >= 0) r = box_child[size_t(q) * 4 + size_t((x & 1) + 2 * (y & 1))];
        }
    }
    il27[t] = r;
}

__device__ inline int32_t scan_at(const int32_t* cscan, const int32_t* ctotal, int64_t nbox, int c, int64_t g) {
    return (g < nbox) ? cscan[size_t(c) * nbox + g] : ctotal[c];
}

// with role: whether box g takes part in M2L (pruned boxes of level >= 3 do not; those of
// level 2 keep their tile so that M2L writes their zero expansion)
__device__ inline bool m2l_box(const int8_t* box_lev, const int8_t* role, int64_t g) {
    return role == nullptr || role[g] != kRolePruned || box_lev[g] < 3;
}

// box -> position in the class list of every group containing it
__global__ void k_class_boxes(const BoxGroup* groups, int32_t ngroups, const int32_t* cscan, const int32_t* ctotal,
                              const uint64_t* box_key, const int8_t* box_lev, const int8_t* role, int64_t nbox,
                              int32_t* cls_box) {
    const int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (g >= nbox || !m2l_box(box_lev, role, g)) return;
    const int c = int(box_key[g] & 3ull);
    for (int32_t q = 0; q < ngroups; ++q) {   // groups are few (heights x leaf sides x 2)
        const BoxGroup G = groups[q];
        if (g < G.g0 || g >= G.g1) continue;
        const int32_t pos = cscan[size_t(c) * nbox + g] - scan_at(cscan, ctotal, nbox, c, G.g0);
        cls_box[G.cls_base + c * (G.g1 - G.g0) + pos] = int32_t(g);
    }
}

// slots of the interleaved tile order before round i: sum over classes of min(nt[c], i)
__device__ inline int32_t rounds_before(const int32_t* nt, int32_t i) {
    return min(nt[0], i) + min(nt[1], i) + min(nt[2], i) + min(nt[3], i);
}

// one thread per tile slot of the groups (group q owns slots [tile_base, tile_base + tile_cap),
// groups in slot order).  Tiles of the four classes are interleaved (round r holds the r-th
// tile of class 0, 1, 2, 3 in turn, classes with fewer tiles dropping out), so that tiles
// next to each other in the list cover the same region of the level and share their
// source expansions in cache; empty tiles fill the rest of the group.
__global__ void k_class_tiles(const BoxGroup* groups, int32_t ngroups, int32_t slot0, int32_t nslots,
                              const int32_t* cscan, const int32_t* ctotal, int64_t nbox, BoxTile* tiles) {
    const int32_t t = slot0 + int32_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= slot0 + nslots) return;
    int32_t lo = 0, hi = ngroups - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (groups[mid].tile_base <= t) lo = mid;
        else hi = mid - 1;
    }
    const BoxGroup G = groups[lo];
    const int32_t r = t - G.tile_base;
    int32_t cnt[4], nt[4];
    for (int c = 0; c < 4; ++c) {
        cnt[c] = scan_at(cscan, ctotal, nbox, c, G.g1) - scan_at(cscan, ctotal, nbox, c, G.g0);
        nt[c] = (cnt[c] + G.tile_boxes - 1) / G.tile_boxes;
    }
    BoxTile tl;
    tl.ops = G.ops;
    tl.height = G.height;
    tl.cls = 0;
    tl.start = 0;
    tl.count = 0;   // an empty tile unless a round below holds slot r
    tl.pad0 = tl.pad1 = tl.pad2 = 0;
    // round i holds the i-th tile of every class with more than i tiles; before(i) slots
    // precede round i.  Find the round of slot r by bisection, then its class.
    const int32_t rounds = max(max(nt[0], nt[1]), max(nt[2], nt[3]));
    if (r < rounds_before(nt, rounds)) {
        int32_t lo_i = 0, hi_i = rounds - 1;   // largest i with before(i) <= r
        while (lo_i < hi_i) {
            const int32_t mid = (lo_i + hi_i + 1) >> 1;
            if (rounds_before(nt, mid) <= r) lo_i = mid;
            else hi_i = mid - 1;
        }
        int32_t rem = r - rounds_before(nt, lo_i);
        for (int c = 0; c < 4; ++c) {
            if (nt[c] <= lo_i) continue;
            if (rem == 0) {
                tl.cls = c;
                tl.start = G.cls_base + c * (G.g1 - G.g0) + lo_i * G.tile_boxes;
                tl.count = min(G.tile_boxes, cnt[c] - lo_i * G.tile_boxes);
                break;
            }
            --rem;
        }
    }
    tiles[t] = tl;
}

// ---- adaptive tree ------------------------------------------------------------------------
// Role of every box: a box belongs to the adaptive tree when its parent holds more than N_leaf
// points (the root always); it is a leaf of it when it holds at most N_leaf points or lies on
// the finest level.  Counts are monotone along parent links, so no pass over ancestors.
__global__ void k_roles(const int32_t* box_pt0, const int32_t* box_pt1, const int32_t* box_parent,
                        const int8_t* box_lev, const int32_t* box_inst, const InstInfo* inst, int64_t nbox,
                        int8_t* role) {
    const int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (g >= nbox) return;
    const InstInfo& I = inst[box_inst[g]];
    const int lev = box_lev[g];
    const int32_t p = box_parent[g];
    const bool member = lev == 0 || p < 0 || box_pt1[p] - box_pt0[p] > I.max_leaf;
    const bool leaf = box_pt1[g] - box_pt0[g] <= I.max_leaf || lev >= I.L;
    role[g] = member ? (leaf ? kRoleLeaf : kRoleInner) : kRolePruned;
}

__global__ void k_filter_interactions(const int8_t* role, int64_t nbox, int32_t* il27) {
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= nbox * kNumInteractions) return;
    const int64_t g = t / kNumInteractions;
    const int32_t r = il27[t];
    if (r >= 0 && (role[g] == kRolePruned || role[r] == kRolePruned)) il27[t] = -1;
}

// Box (level, x, y), x and y in units of its level.
struct BoxAt {
    int lev;
    int32_t x, y;
};

__device__ inline BoxAt box_at(const uint64_t* box_key, const int8_t* box_lev, int32_t g) {
    const uint64_t k = box_key[g];
    return BoxAt{int(box_lev[g]), int32_t(compact_bits(k)), int32_t(compact_bits(k >> 1))};
}

// whether the closed squares of two disjoint boxes of one instance meet (share an edge or a
// corner)
__device__ inline bool touches(BoxAt a, BoxAt b) {
    if (a.lev < b.lev) {
        const BoxAt t = a;
        a = b;
        b = t;
    }
    const int d = a.lev - b.lev;   // b covers [x << d, (x + 1) << d) in units of a's level
    const int64_t x0 = int64_t(b.x) << d, x1 = (int64_t(b.x) + 1) << d;
    const int64_t y0 = int64_t(b.y) << d, y1 = (int64_t(b.y) + 1) << d;
    return int64_t(a.x) + 1 >= x0 && int64_t(a.x) <= x1 && int64_t(a.y) + 1 >= y0 && int64_t(a.y) <= y1;
}

struct ListOut {
    bool fill;
    int32_t* cnt;            // [3][nbox + 1] counts (count pass; the last of each row zero)
    const int32_t* off[3];   // row starts (fill pass)
    int32_t* ent[3];
    int64_t nbox;
    __device__ void put(int r, int32_t g, int32_t& n, int32_t v) const {
        if (fill) ent[r][off[r][g] + n] = v;
        ++n;
    }
};

// Depth of the stack of the W/U descent below a colleague: each level leaves at most three
// siblings waiting, over at most kMaxLevels levels.
constexpr int kListStack = 3 * kMaxLevels + 4;

// X entries of box a (level >= 2): the leaves coarser than a that touch a's parent but not a,
// among the neighbours of a's ancestors; out(list, entry) takes each.
template <class Out>
__device__ inline void x_entries(int32_t a, const uint64_t* box_key, const int32_t* box_parent, const int8_t* box_lev,
                                 const int8_t* role, const int32_t* nb9, Out out) {
    const BoxAt ab = box_at(box_key, box_lev, a);
    const int32_t p = box_parent[a];
    const BoxAt par = box_at(box_key, box_lev, p);
    for (int32_t b = p; b >= 0 && box_lev[b] >= 1; b = box_parent[b])
        for (int q = 0; q < 9; ++q) {
            if (q == 4) continue;
            const int32_t c = nb9[size_t(b) * 9 + q];
            if (c < 0 || role[c] != kRoleLeaf) continue;
            const BoxAt cb = box_at(box_key, box_lev, c);
            if (touches(par, cb) && !touches(ab, cb)) out(c);
        }
}

// U and W of every adaptive leaf and X of every box of the adaptive tree, one thread per box.
//   U(tau): tau; the colleagues that are leaves; below the other colleagues (inner boxes), the
//     descendants that touch tau and are leaves (a descent through those that touch tau);
//     and the coarser leaves that touch tau, found among the neighbours of its ancestors
//     (a leaf touching tau touches the ancestor of tau on its own level).
//   W(tau): in that descent, the children that do not touch tau.
//   X(tau): the leaves coarser than tau that touch its parent but not tau, among the
//     neighbours of its ancestors.
// Expansions pay only for boxes with more points than skeleton points: a W box holding at most
// kDirectMax points joins U instead (its points summed directly: fewer terms than its
// skeleton), and a box holding at most kDirectMax points keeps no X list: the leaves below it
// take its X entries into their U lists.  Every (target, source) pair stays counted once.
__global__ void k_adaptive_lists(const uint64_t* box_key, const int32_t* box_parent, const int32_t* box_child,
                                 const int8_t* box_lev, const int8_t* role, const int32_t* nb9,
                                 const int32_t* box_pt0, const int32_t* box_pt1, int64_t nbox, ListOut o) {
    const int64_t gg = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (gg > nbox) return;
    const int32_t g = int32_t(gg);
    const size_t stride = size_t(nbox) + 1;
    if (gg == nbox || role[g] == kRolePruned) {
        if (!o.fill)
            for (int r = 0; r < 3; ++r) o.cnt[size_t(r) * stride + g] = 0;
        return;
    }
    const int8_t rg = role[g];
    const BoxAt tau = box_at(box_key, box_lev, g);
    int32_t nu = 0, nw = 0, nx = 0;
    if (rg == kRoleLeaf) {
        o.put(0, g, nu, g);
        int32_t stack[kListStack];
        int sp = 0;
        for (int q = 0; q < 9; ++q) {
            if (q == 4) continue;
            const int32_t c = nb9[size_t(g) * 9 + q];
            if (c < 0 || role[c] == kRolePruned) continue;
            if (role[c] == kRoleLeaf) {
                o.put(0, g, nu, c);
                continue;
            }
            stack[sp++] = c;
            while (sp > 0) {
                const int32_t b = stack[--sp];
                for (int k = 3; k >= 0; --k) {   // pushed in reverse: children visited in order
                    const int32_t d = box_child[size_t(b) * 4 + k];
                    if (d < 0) continue;
                    if (!touches(tau, box_at(box_key, box_lev, d))) {
                        if (box_pt1[d] - box_pt0[d] <= kDirectMax) o.put(0, g, nu, d);
                        else o.put(1, g, nw, d);
                    } else if (role[d] == kRoleLeaf) o.put(0, g, nu, d);
                    else if (sp < kListStack) stack[sp++] = d;
                }
            }
        }
        for (int32_t a = box_parent[g]; a >= 0 && box_lev[a] >= 1; a = box_parent[a])
            for (int q = 0; q < 9; ++q) {
                if (q == 4) continue;
                const int32_t c = nb9[size_t(a) * 9 + q];
                if (c >= 0 && role[c] == kRoleLeaf && touches(tau, box_at(box_key, box_lev, c))) o.put(0, g, nu, c);
            }
        // X entries of tau and of its ancestors small enough to keep none (counts grow upwards)
        for (int32_t a = g; a >= 0 && box_lev[a] >= 2 && box_pt1[a] - box_pt0[a] <= kDirectMax; a = box_parent[a])
            x_entries(a, box_key, box_parent, box_lev, role, nb9, [&](int32_t c) { o.put(0, g, nu, c); });
    }
    if (tau.lev >= 2 && box_pt1[g] - box_pt0[g] > kDirectMax)
        x_entries(g, box_key, box_parent, box_lev, role, nb9, [&](int32_t c) { o.put(2, g, nx, c); });
    if (!o.fill) {
        o.cnt[g] = nu;
        o.cnt[stride + g] = nw;
        o.cnt[2 * stride + g] = nx;
    }
}

__global__ void k_compact_positive(const int32_t* cnt, const int32_t* pos, int64_t nbox, int32_t* items) {
    const int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (g < nbox && cnt[g] > 0) items[pos[g]] = int32_t(g);
}

// finest box of every point: a thread per finest box (their blocks follow the instance order
// of the height blocks, not the point order) writes its index over its points
__global__ void k_point_boxes(const int32_t* box_pt0, const int32_t* box_pt1, int32_t nleaf, int32_t* pt_box) {
    const int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (g >= nleaf) return;
    for (int32_t i = box_pt0[g]; i < box_pt1[g]; ++i) pt_box[i] = int32_t(g);
}

// Near-field groups, 16 lanes per group: the group's leaves (the children of a height-1 box,
// or a root that is a leaf) and the union of their neighbour lists, as point ranges in box
// order (Morton order, so ranges of adjacent leaves follow each other).  Lane j stands for
// cell (j mod 4, j / 4) of the 4 x 4 block of leaf cells around the parent, whose children sit
// at cells 1..2; it reads the box at its cell from the neighbour list of the first child of
// the group next to that cell, and its entry goes to the rank of its box among the group's.
// The children themselves make one entry (their points are one run) marked near to all, and
// so do the two cells above them and the two below (near by y alone).
__global__ void k_near_groups(int32_t q0, int32_t h1_start, int32_t h1_count, const int32_t* roots, int32_t nroots,
                              const int32_t* box_child, const int32_t* nb9, const int32_t* box_pt0,
                              const int32_t* box_pt1, const uint64_t* box_key, NearGroup* groups, int4* ents) {
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int32_t q = int32_t(t >> 4);
    const int j = int(threadIdx.x & 15), lane = int(threadIdx.x & 63);
    const bool active = q < h1_count + nroots;   // the same for all 16 lanes of a group
    int32_t b = -1, leaf0 = -1, nleaf = 0;
    if (active) {
        if (q < h1_count) {
            const int32_t P = h1_start + q;
            const int ox = j & 3, oy = j >> 2;
            bool done = false;
            for (int c = 0; c < 4; ++c) {
                const int32_t ch = box_child[size_t(P) * 4 + c];
                if (ch < 0) continue;
                if (leaf0 < 0) leaf0 = ch;
                ++nleaf;
                const int dx = ox - 1 - (c & 1), dy = oy - 1 - (c >> 1);
                if (done || dx < -1 || dx > 1 || dy < -1 || dy > 1) continue;
                b = nb9[size_t(ch) * 9 + (dy + 1) * 3 + dx + 1];
                done = true;
            }
        } else {
            leaf0 = roots[q - h1_count];
            nleaf = 1;
            if (j < 9) b = nb9[size_t(leaf0) * 9 + j];
        }
    }
    // the group's own leaves (cells 1..2 x 1..2: consecutive boxes, so one run of points, and
    // neighbours of every target of the group) become one entry, held by the first of them
    const bool own = active && q < h1_count && (j & 3) >= 1 && (j & 3) <= 2 && (j >> 2) >= 1 && (j >> 2) <= 2;
    if (own && b != leaf0) b = -1;
    // likewise the two cells above (and the two below) the children: two children of one parent,
    // so consecutive boxes, and neighbours in x of every target; one entry, near by y alone
    const bool rowpair = active && q < h1_count && (j & 3) >= 1 && (j & 3) <= 2 && ((j >> 2) == 0 || (j >> 2) == 3);
    const int32_t bp = __shfl(b, (lane & ~3) | (3 - (j & 3)), 64);   // the other cell of the pair
    int32_t b_end = b;                                                // last box of the entry
    if (rowpair && b >= 0 && bp >= 0) {
        if (b < bp) b_end = bp;
        else b = -1;
    }
    int rank = 0, cnt = 0;
    #pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int32_t bi = __shfl(b, (lane & 48) | i, 64);
        cnt += bi >= 0 ? 1 : 0;
        rank += (bi >= 0 && bi < b) ? 1 : 0;
    }
    if (!active) return;
    if (b >= 0 && own) {
        ents[size_t(q0 + q) * kNearEntries + rank] = make_int4(box_pt0[b], box_pt1[b + nleaf - 1], kNearAll, kNearAll);
    } else if (b >= 0 && rowpair) {
        ents[size_t(q0 + q) * kNearEntries + rank] =
            make_int4(box_pt0[b], box_pt1[b_end], kNearAll, int32_t(compact_bits(box_key[b] >> 1)));
    } else if (b >= 0) {
        const uint64_t key = box_key[b];
        ents[size_t(q0 + q) * kNearEntries + rank] =
            make_int4(box_pt0[b], box_pt1[b], int32_t(compact_bits(key)), int32_t(compact_bits(key >> 1)));
    }
    if (j == 0) {
        NearGroup G;
        G.leaf0 = leaf0;
        G.nleaf = nleaf;
        G.ne = cnt;
        G.pad = 0;
        groups[q0 + q] = G;
    }
}

// ---- exclusive scan over rows of int32 -------------------------------------------------
constexpr int kScanItems = 8;
constexpr int kScanTile = kBlock * kScanItems;

// exclusive scan over the NT threads of a block (thread order); *total = the sum
template <int NT = kBlock>
__device__ inline int32_t block_exclusive_scan(int32_t v, int32_t* total) {
    __shared__ int32_t wsum[NT / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int32_t x = v;
    #pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) wsum[wave] = x;
    __syncthreads();
    int32_t pre = 0, tot = 0;
    for (int w = 0; w < NT / 64; ++w) {
        if (w < wave) pre += wsum[w];
        tot += wsum[w];
    }
    __syncthreads();
    *total = tot;
    return pre + x - v;
}

// ---- radix sort passes -----------------------------------------------------------------------
// Digit counts of every tile for the digit at `shift`.
__global__ void k_rs_count(const uint64_t* keys, int64_t n, int shift, uint32_t* C, int64_t ntiles, bool digit_major) {
    uint32_t dg[kRsItems];
    #pragma unroll
    for (int it = 0; it < kRsItems; ++it) {
        const int64_t i = int64_t(blockIdx.x) * kRsTile + int64_t(it) * kBlock + threadIdx.x;
        dg[it] = i < n ? uint32_t((keys[i] >> shift) & 255u) : 256u;
    }
    rs_count_tile(dg, C, ntiles, digit_major);
}

// Stable scatter of one tile by the digit at `shift`, kRsScatterThreads threads per tile.
// The tile's output start for digit d is offs[d][tile] when offs is given (a flat exclusive
// scan of the digit-major counts), else computed here from the tile-major counts C: the
// totals of every digit scanned over the digits, plus the counts of d in the tiles before
// this one.  Wave w ranks the tile's keys w * 512 .. w * 512 + 511 in rounds of 64 (eight
// ballots find the lanes with equal digits; a per-wave running count per digit in LDS orders
// the rounds), the waves are ordered by per-digit prefixes, and the keys are staged in LDS
// in output order and written as runs of consecutive addresses.
constexpr int kRsScatterThreads = 512;
constexpr int kRsWaves = kRsScatterThreads / 64;
constexpr int kRsRounds = kRsTile / kRsScatterThreads;

__global__ __launch_bounds__(kRsScatterThreads) void k_rs_scatter(const uint64_t* kin, const uint32_t* vin,
                                                                  uint64_t* kout, uint32_t* vout, int64_t n, int shift,
                                                                  const uint32_t* C, const int32_t* offs,
                                                                  int64_t ntiles) {
    __shared__ uint32_t s_start[256];
    __shared__ uint32_t s_pref[256];
    __shared__ uint32_t cnt[kRsWaves][256];   // per wave: running digit counts, then prefixes over the waves
    __shared__ union {
        uint32_t red[2][kRsWaves][256];       // partial sums of the counts of earlier tiles
        struct {
            uint64_t k[kRsTile];
            uint32_t v[kRsTile];
        } st;
    } sm;
    const int tid = int(threadIdx.x), wave = tid >> 6, lane = tid & 63;
    const int64_t tile = blockIdx.x, base = tile * kRsTile;
    // output start of each digit's run of this tile (thread d < 256 for digit d)
    uint32_t start = 0;
    if (offs) {
        if (tid < 256) start = uint32_t(offs[size_t(tid) * size_t(ntiles) + size_t(tile)]);
    } else {
        // lane l of wave w sums digits 4l .. 4l + 3 over the rows w, w + kRsWaves, ..., 16 rows
        // of 1 KB in flight per wave
        const uint4* C4 = reinterpret_cast<const uint4*>(C);
        uint32_t tot[4] = {0u, 0u, 0u, 0u}, bef[4] = {0u, 0u, 0u, 0u};
        for (int64_t j0 = wave; j0 < ntiles; j0 += kRsWaves * 16) {
            uint4 v[16];
            #pragma unroll
            for (int u = 0; u < 16; ++u) {
                const int64_t j = j0 + kRsWaves * u;
                v[u] = j < ntiles ? C4[size_t(j) * 64 + size_t(lane)] : make_uint4(0u, 0u, 0u, 0u);
            }
            #pragma unroll
            for (int u = 0; u < 16; ++u) {
                const uint32_t m = (j0 + kRsWaves * u < tile) ? ~0u : 0u;
                tot[0] += v[u].x; tot[1] += v[u].y; tot[2] += v[u].z; tot[3] += v[u].w;
                bef[0] += v[u].x & m; bef[1] += v[u].y & m; bef[2] += v[u].z & m; bef[3] += v[u].w & m;
            }
        }
        #pragma unroll
        for (int q = 0; q < 4; ++q) {
            sm.red[0][wave][4 * lane + q] = tot[q];
            sm.red[1][wave][4 * lane + q] = bef[q];
        }
        __syncthreads();
        uint32_t total = 0, before = 0;
        if (tid < 256)
            #pragma unroll
            for (int w = 0; w < kRsWaves; ++w) {
                total += sm.red[0][w][tid];
                before += sm.red[1][w][tid];
            }
        int32_t all;
        start = uint32_t(block_exclusive_scan<kRsScatterThreads>(int32_t(total), &all)) + before;
    }
    for (int q = tid; q < kRsWaves * 256; q += kRsScatterThreads) (&cnt[0][0])[q] = 0u;
    uint64_t key[kRsRounds];
    uint32_t val[kRsRounds];
    const int64_t wbase = base + int64_t(wave) * (kRsRounds * 64) + lane;
    #pragma unroll
    for (int r = 0; r < kRsRounds; ++r) {
        const int64_t i = wbase + int64_t(r) * 64;
        key[r] = i < n ? kin[i] : 0ull;
        val[r] = i < n ? vin[i] : 0u;
    }
    __syncthreads();
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    uint32_t pw[kRsRounds];   // position among this wave's keys of the same digit
    #pragma unroll
    for (int r = 0; r < kRsRounds; ++r) {
        const bool valid = wbase + int64_t(r) * 64 < n;
        const uint32_t d = uint32_t((key[r] >> shift) & 255u);
        uint64_t mask = __ballot(valid);
        #pragma unroll
        for (int b = 0; b < 8; ++b) {
            const uint64_t bb = __ballot(valid && ((d >> b) & 1u));
            mask &= ((d >> b) & 1u) ? bb : ~bb;
        }
        const uint32_t rk = uint32_t(__popcll(mask & lt_mask));
        const uint32_t off = valid ? cnt[wave][d] : 0u;
        pw[r] = off + rk;
        if (valid && rk == 0) cnt[wave][d] = off + uint32_t(__popcll(mask));
    }
    __syncthreads();
    uint32_t run = 0;
    if (tid < 256)
        #pragma unroll
        for (int w = 0; w < kRsWaves; ++w) {
            const uint32_t c = cnt[w][tid];
            cnt[w][tid] = run;
            run += c;
        }
    int32_t tcount;
    const uint32_t pref = uint32_t(block_exclusive_scan<kRsScatterThreads>(int32_t(run), &tcount));
    if (tid < 256) {
        s_pref[tid] = pref;
        s_start[tid] = start - pref;   // output position of local position p of digit d: s_start[d] + p
    }
    __syncthreads();
    #pragma unroll
    for (int r = 0; r < kRsRounds; ++r)
        if (wbase + int64_t(r) * 64 < n) {
            const uint32_t d = uint32_t((key[r] >> shift) & 255u);
            const uint32_t pos = s_pref[d] + cnt[wave][d] + pw[r];
            sm.st.k[pos] = key[r];
            sm.st.v[pos] = val[r];
        }
    __syncthreads();
    for (int p = tid; p < tcount; p += kRsScatterThreads) {
        const uint64_t k = sm.st.k[p];
        const uint32_t o = s_start[(k >> shift) & 255u] + uint32_t(p);
        kout[o] = k;
        vout[o] = sm.st.v[p];
    }
}

// Two-launch exclusive scan of `rows` rows of n values each (row r, item i = src(r, i)): the
// first launch sums each tile of kScanTile items, the second adds the sums of the tiles
// before its own (a block-wide reduction over at most a few thousand values) and scans
// its tile.  Sources compute flags on the fly, so no flag array is stored.
struct RowsArray {   // values from an array, row stride n
    const int32_t* in;
    int64_t n;
    __device__ int32_t operator()(int r, int64_t i) const { return in[size_t(r) * n + i]; }
};
struct LeafStart {   // 1 where a leaf of its instance starts at Morton-ordered point i
    const int8_t* cl;
    const int32_t* pinst;
    const InstInfo* inst;
    __device__ int32_t operator()(int, int64_t i) const { return cl[i] < inst[pinst[i]].L ? 1 : 0; }
};
struct LevelStart {   // row lev: 1 where leaf b starts a box of level lev < L of its instance
    const int8_t* leaf_cl;
    const int32_t* leaf_inst;
    const InstInfo* inst;
    __device__ int32_t operator()(int lev, int64_t b) const {
        return (lev < inst[leaf_inst[b]].L && leaf_cl[b] < lev) ? 1 : 0;
    }
};
struct ChildClass {   // row c: 1 where box g sits in child position c of its parent
    const uint64_t* box_key;
    __device__ int32_t operator()(int c, int64_t g) const { return int(box_key[g] & 3ull) == c ? 1 : 0; }
};
struct ChildClassM2L {   // the same over the boxes that take part in M2L
    const uint64_t* box_key;
    const int8_t* box_lev;
    const int8_t* role;
    __device__ int32_t operator()(int c, int64_t g) const {
        return (int(box_key[g] & 3ull) == c && m2l_box(box_lev, role, g)) ? 1 : 0;
    }
};
struct TileNonEmpty {   // 1 where tile i holds boxes
    const BoxTile* tiles;
    __device__ int32_t operator()(int, int64_t i) const { return tiles[i].count > 0 ? 1 : 0; }
};
struct TileScatter {    // non-empty tile i to its rank among them
    const BoxTile* in;
    BoxTile* out;
    __device__ void operator()(int, int64_t i, int32_t x, int32_t v) const {
        if (v) out[x] = in[i];
    }
};
struct RowsPositive {   // 1 where the value is positive, row stride n
    const int32_t* in;
    int64_t n;
    __device__ int32_t operator()(int r, int64_t i) const { return in[size_t(r) * n + i] > 0 ? 1 : 0; }
};

__device__ inline int32_t block_sum(int32_t v) {
    __shared__ int32_t ws[kBlock / 64];
    #pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = v;
    __syncthreads();
    int32_t t = 0;
    for (int w = 0; w < kBlock / 64; ++w) t += ws[w];
    __syncthreads();
    return t;
}

template <class Src>
__global__ void k_scan_sums(Src src, int64_t n, int32_t* bsum, int nblk) {
    const int row = blockIdx.y;
    const int64_t base = int64_t(blockIdx.x) * kScanTile + int64_t(threadIdx.x) * kScanItems;
    int32_t sum = 0;
    #pragma unroll
    for (int k = 0; k < kScanItems; ++k)
        if (base + k < n) sum += src(row, base + k);
    sum = block_sum(sum);
    if (threadIdx.x == 0) bsum[size_t(row) * nblk + blockIdx.x] = sum;
}

// Where the prefixes go: by default into the output rows.
struct StoreSink {
    int32_t* out;
    int64_t n;
    __device__ void operator()(int row, int64_t i, int32_t x, int32_t) const { out[size_t(row) * n + i] = x; }
};
// Leaf starts: the point that starts leaf x writes that leaf's first point, key, level count
// and instance; every point of a leaf side of at most 16 also gets its window key
// K = 8 (y W + x) mod 2^32 (W = 4 side - 1) for the near field.
struct LeafSink {
    const uint64_t* keys;
    const int8_t* cl;
    const int32_t* pinst;
    const InstInfo* inst;
    int Dmax;
    const int2* pts;
    uint32_t* pkey;
    int32_t* leaf_pt0;
    uint64_t* leaf_key;
    int8_t* leaf_cl;
    int32_t* leaf_inst;
    __device__ void operator()(int, int64_t s, int32_t r, int32_t flag) const {
        const int32_t k = pinst[s];
        const InstInfo& I = inst[k];
        if (flag) {
            leaf_pt0[r] = int32_t(s);
            leaf_key[r] = (keys[s] & morton_mask(Dmax)) >> (2 * (I.D - I.L));
            leaf_cl[r] = cl[s];
            leaf_inst[r] = k;
        }
        const int64_t side = int64_t(1) << (I.D - I.L);
        if (side <= 16) {
            const int2 p = pts[s];
            const uint32_t W = uint32_t(4 * side - 1);
            pkey[s] = 8u * (uint32_t(p.y) * W + uint32_t(p.x));   // modulo 2^32 on purpose
        }
    }
};

template <class Src, class Sink>
__global__ void k_scan_apply(Src src, Sink sink, int64_t n, const int32_t* bsum, int nblk, int32_t* totals) {
    const int row = blockIdx.y;
    const int32_t* bs = bsum + size_t(row) * nblk;
    int32_t pre = 0;
    for (int t = threadIdx.x; t < int(blockIdx.x); t += kBlock) pre += bs[t];
    pre = block_sum(pre);
    const int64_t base = int64_t(blockIdx.x) * kScanTile + int64_t(threadIdx.x) * kScanItems;
    int32_t v[kScanItems];
    int32_t s = 0;
    #pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = (base + k < n) ? src(row, base + k) : 0;
        s += v[k];
    }
    int32_t tot;
    int32_t x = pre + block_exclusive_scan(s, &tot);
    #pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        if (base + k < n) sink(row, base + k, x, v[k]);
        x += v[k];
    }
    if (totals && blockIdx.x == unsigned(nblk - 1) && threadIdx.x == 0) totals[row] = pre + tot;
}

template <class Src, class Sink>
void scan_sink(Src src, Sink sink, int64_t n, int rows, int32_t* totals, void* scratch, hipStream_t st) {
    if (n <= 0 || rows <= 0) return;
    const int64_t nb = (n + kScanTile - 1) / kScanTile;
    int32_t* bsum = static_cast<int32_t*>(scratch);
    hipLaunchKernelGGL(k_scan_sums<Src>, dim3(unsigned(nb), unsigned(rows)), dim3(kBlock), 0, st, src, n, bsum,
                       int(nb));
    hipLaunchKernelGGL((k_scan_apply<Src, Sink>), dim3(unsigned(nb), unsigned(rows)), dim3(kBlock), 0, st, src, sink,
                       n, bsum, int(nb), totals);
}

template <class Src>
void scan_source(Src src, int32_t* out, int64_t n, int rows, int32_t* totals, void* scratch, hipStream_t st) {
    scan_sink(src, StoreSink{out, n}, n, rows, totals, scratch, st);
}

}  // namespace

size_t scan_scratch_bytes(int64_t n, int rows) {
    const int64_t nb = (n + kScanTile - 1) / kScanTile;
    return size_t(nb) * size_t(rows) * sizeof(int32_t) + 256;
}

void scan_rows(const int32_t* in, int32_t* out, int64_t n, int rows, int32_t* totals, void* scratch, hipStream_t st) {
    scan_source(RowsArray{in, n}, out, n, rows, totals, scratch, st);
}

void scan_leaf_starts(const int8_t* cl, const int32_t* pinst, const InstInfo* inst, int64_t n, const uint64_t* keys,
                      int Dmax, const int32_t* pts, uint32_t* pkey, int32_t* leaf_pt0, uint64_t* leaf_key,
                      int8_t* leaf_cl, int32_t* leaf_inst, void* scratch, hipStream_t st) {
    scan_sink(LeafStart{cl, pinst, inst},
              LeafSink{keys, cl, pinst, inst, Dmax, reinterpret_cast<const int2*>(pts), pkey, leaf_pt0, leaf_key,
                       leaf_cl, leaf_inst},
              n, 1, nullptr, scratch, st);
}

void scan_level_starts(const int8_t* leaf_cl, const int32_t* leaf_inst, const InstInfo* inst, int64_t nleaf,
                       int Lmax, int32_t* out, void* scratch, hipStream_t st) {
    scan_source(LevelStart{leaf_cl, leaf_inst, inst}, out, nleaf, Lmax, nullptr, scratch, st);
}

void scan_child_classes(const uint64_t* box_key, int64_t nbox, int32_t* out, int32_t* totals, void* scratch,
                        hipStream_t st) {
    scan_source(ChildClass{box_key}, out, nbox, 4, totals, scratch, st);
}

void scan_child_classes_active(const uint64_t* box_key, const int8_t* box_lev, const int8_t* role, int64_t nbox,
                               int32_t* out, int32_t* totals, void* scratch, hipStream_t st) {
    scan_source(ChildClassM2L{box_key, box_lev, role}, out, nbox, 4, totals, scratch, st);
}

void scan_positive(const int32_t* cnt, int64_t n, int rows, int32_t* out, int32_t* totals, void* scratch,
                   hipStream_t st) {
    scan_source(RowsPositive{cnt, n}, out, n, rows, totals, scratch, st);
}

void compact_tiles(const BoxTile* in, int32_t n, BoxTile* out, int32_t* count, void* scratch, hipStream_t st) {
    if (n <= 0) return;
    scan_sink(TileNonEmpty{in}, TileScatter{in, out}, n, 1, count, scratch, st);
}

// Tiles whose counts a scatter block sums itself (tile-major counts, no scan launches); above
// this, one flat exclusive scan of the digit-major counts gives the offsets.
constexpr int64_t kRsSelfScanTiles = 512;

int64_t radix_tiles(int64_t n) { return (n + kRsTile - 1) / kRsTile; }

bool radix_digit_major(int64_t n) { return radix_tiles(n) > kRsSelfScanTiles; }

size_t radix_scratch_bytes(int64_t n) {
    const size_t counts = size_t(256) * size_t(radix_tiles(n)) * sizeof(int32_t);
    return ((2 * counts + 255) & ~size_t(255)) + scan_scratch_bytes(256 * radix_tiles(n), 1) + 256;
}

uint32_t* radix_counts(void* scratch) { return static_cast<uint32_t*>(scratch); }

int radix_sort_passes(uint64_t* keys, uint32_t* vals, uint64_t* keys_tmp, uint32_t* vals_tmp, int64_t n, int p0,
                      int p1, bool counted0, void* scratch, hipStream_t st) {
    if (n <= 1 || p1 <= 0) return 0;
    const int64_t nt = radix_tiles(n);
    const bool dm = radix_digit_major(n);
    const size_t counts = size_t(256) * size_t(nt);
    uint32_t* C = radix_counts(scratch);
    int32_t* offs = reinterpret_cast<int32_t*>(C + counts);
    void* sscr = static_cast<char*>(scratch) + ((2 * counts * sizeof(int32_t) + 255) & ~size_t(255));
    for (int p = p0; p < p1; ++p) {
        uint64_t* ka = (p & 1) ? keys_tmp : keys;
        uint64_t* kb = (p & 1) ? keys : keys_tmp;
        uint32_t* va = (p & 1) ? vals_tmp : vals;
        uint32_t* vb = (p & 1) ? vals : vals_tmp;
        const int shift = 8 * p;
        if (p > 0 || !counted0)
            hipLaunchKernelGGL(k_rs_count, dim3(unsigned(nt)), dim3(kBlock), 0, st, ka, n, shift, C, nt, dm);
        if (dm) scan_rows(reinterpret_cast<const int32_t*>(C), offs, int64_t(counts), 1, nullptr, sscr, st);
        hipLaunchKernelGGL(k_rs_scatter, dim3(unsigned(nt)), dim3(kRsScatterThreads), 0, st, ka, va, kb, vb, n,
                           shift, C, dm ? offs : nullptr, nt);
    }
    return p1 & 1;
}

int radix_sort_pairs(uint64_t* keys, uint32_t* vals, uint64_t* keys_tmp, uint32_t* vals_tmp, int64_t n, int nbits,
                     bool counted0, void* scratch, hipStream_t st) {
    if (nbits <= 0) return 0;
    return radix_sort_passes(keys, vals, keys_tmp, vals_tmp, n, 0, (nbits + 7) / 8, counted0, scratch, st);
}

// Small host-to-device copy run as a kernel: the source is pinned host memory, read with
// system-scope loads (coherent with the host's writes), so the copy is ordered on the stream
// like the kernels around it.  dst and src are 8-byte aligned; the last word is written byte
// by byte when len is not a multiple of 8 (src may be read up to the next multiple of 8).
__global__ void k_upload(const uint64_t* src, uint64_t* dst, int64_t len) {
    const int64_t nw = len >> 3;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < nw; i += int64_t(gridDim.x) * blockDim.x)
        dst[i] = __hip_atomic_load(src + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    const int rem = int(len & 7);
    if (rem != 0 && blockIdx.x == 0 && threadIdx.x == 0) {
        const uint64_t w = __hip_atomic_load(src + nw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        unsigned char* d = reinterpret_cast<unsigned char*>(dst + nw);
        for (int b = 0; b < rem; ++b) d[b] = static_cast<unsigned char>(w >> (8 * b));
    }
}

void launch_upload(void* dst, const void* pinned_src, size_t len, hipStream_t st) {
    if (len == 0) return;
    const int64_t nw = int64_t(len >> 3) + 1;
    const unsigned g = unsigned(std::min<int64_t>((nw + kBlock - 1) / kBlock, 64));
    hipLaunchKernelGGL(k_upload, dim3(g), dim3(kBlock), 0, st, static_cast<const uint64_t*>(pinned_src),
                       static_cast<uint64_t*>(dst), int64_t(len));
}

void launch_extents(int32_t K, const int64_t* n, const int32_t* const* xy, int32_t* box, hipStream_t st) {
    hipLaunchKernelGGL(k_extent_init, dim3(grid_for(K)), dim3(kBlock), 0, st, box, K);
    for (int32_t k = 0; k < K; ++k) {
        const unsigned g = std::min<unsigned>(grid_for(n[k]), 1024u);
        hipLaunchKernelGGL(k_extent, dim3(g), dim3(kBlock), 0, st, reinterpret_cast<const int2*>(xy[k]), n[k],
                           box + 4 * size_t(k));
    }
}

void launch_concat(int32_t K, const int32_t* const* xy_tab, const int32_t* pt_off, int64_t n, int32_t* xyc,
                   hipStream_t st) {
    hipLaunchKernelGGL(k_concat, dim3(grid_for(n)), dim3(kBlock), 0, st, K,
                       reinterpret_cast<const int2* const*>(xy_tab), pt_off, n, reinterpret_cast<int2*>(xyc));
}

void launch_bbox_chunks(const int32_t* xy, const Chunk* chunks, int32_t nchunks, int32_t* part, int32_t* dmax,
                        hipStream_t st) {
    hipLaunchKernelGGL(k_bbox_chunks, dim3(unsigned(nchunks)), dim3(kBlock), 0, st, reinterpret_cast<const int2*>(xy),
                       chunks, part, dmax);
}

void launch_bbox_final(const int32_t* part, const int32_t* chunk_first, const int32_t* pt_off, int32_t K,
                       int32_t max_leaf, int32_t* bbox, InstInfo* inst, int32_t* dmax, hipStream_t st) {
    hipLaunchKernelGGL(k_bbox_final, dim3(static_cast<unsigned>(K)), dim3(kBlock), 0, st, part, chunk_first, pt_off,
                       max_leaf, bbox, inst, dmax);
}

void launch_keys(const int32_t* xy, const int32_t* pt_off, int32_t K, const InstInfo* inst, const int32_t* dmax,
                 int64_t n, uint64_t* keys, uint32_t* vals, int32_t* zero, int32_t nzero, void* radix_scratch,
                 hipStream_t st) {
    const int64_t nt = radix_tiles(n);
    hipLaunchKernelGGL(k_keys, dim3(unsigned(nt)), dim3(kBlock), 0, st, reinterpret_cast<const int2*>(xy), pt_off, K,
                       inst, dmax, n, keys, vals, zero, nzero,
                       radix_scratch ? radix_counts(radix_scratch) : static_cast<uint32_t*>(nullptr), nt,
                       radix_digit_major(n));
}

void launch_level_stats(const uint64_t* keys, const uint32_t* vals, const Chunk* chunks, int32_t nchunks,
                        const InstInfo* inst, int Dmax, int32_t K, int32_t* pts, int32_t* perm_local, int32_t* pinst,
                        int8_t* cl, int32_t* hist, int32_t copies, int32_t* done, int32_t* host_out,
                        hipStream_t st) {
    hipLaunchKernelGGL(k_level_stats, dim3(unsigned(nchunks)), dim3(kBlock), 0, st, keys, vals, chunks, inst, Dmax, K,
                       reinterpret_cast<int2*>(pts), perm_local, pinst, cl, hist, std::max(copies, 1), done,
                       host_out);
}

void launch_build_boxes(const int32_t* lscan, const int8_t* leaf_cl, const int32_t* leaf_pt0, const uint64_t* leaf_key,
                        const int32_t* leaf_inst, const InstInfo* inst, int64_t nleaf, int Lmax, uint64_t* box_key,
                        int32_t* box_pt0, int32_t* box_parent, int32_t* box_child, int32_t* box_inst,
                        int8_t* box_lev, hipStream_t st) {
    hipLaunchKernelGGL(k_build_boxes, dim3(grid_for(nleaf), unsigned(Lmax + 1)), dim3(kBlock), 0, st, lscan, leaf_cl,
                       leaf_pt0, leaf_key, leaf_inst, inst, nleaf, box_key, box_pt0, box_parent, box_child, box_inst,
                       box_lev);
}

void launch_link_boxes(const uint64_t* box_key, const int32_t* box_parent, const int32_t* box_inst,
                       const int8_t* box_lev, const InstInfo* inst, int64_t nbox, const int32_t* box_pt0,
                       int32_t* box_child, int32_t* box_pt1, double* zq, double* zu, hipStream_t st) {
    hipLaunchKernelGGL(k_link_boxes, dim3(grid_for(std::max<int64_t>(nbox, kRankPad))), dim3(kBlock), 0, st, box_key,
                       box_parent, box_inst, box_lev, inst, nbox, box_pt0, box_child, box_pt1, zq, zu);
}

void launch_lists(const uint64_t* box_key, const int32_t* box_parent, const int32_t* box_child,
                  const int32_t* box_inst, const int8_t* box_lev, const InstInfo* inst, int64_t nbox, int32_t* nb9,
                  int32_t* il27, hipStream_t st) {
    if (nbox <= 0) return;
    hipLaunchKernelGGL(k_neighbours, dim3(grid_for(nbox * 9)), dim3(kBlock), 0, st, box_key, box_inst, box_lev, inst,
                       nbox, nb9);
    hipLaunchKernelGGL(k_interactions, dim3(grid_for(nbox * kNumInteractions)), dim3(kBlock), 0, st, box_key,
                       box_parent, box_child, box_lev, nbox, nb9, il27);
}

void launch_class_lists(const BoxGroup* groups, int32_t ngroups, int32_t slot0, int32_t nslots,
                        const int32_t* cscan, const int32_t* ctotal, const uint64_t* box_key,
                        const int8_t* box_lev, const int8_t* role, int64_t nbox, int32_t* cls_box,
                        BoxTile* tiles, hipStream_t st) {
    if (ngroups <= 0) return;
    hipLaunchKernelGGL(k_class_boxes, dim3(grid_for(nbox)), dim3(kBlock), 0, st, groups, ngroups, cscan, ctotal,
                       box_key, box_lev, role, nbox, cls_box);
    if (nslots > 0)
        hipLaunchKernelGGL(k_class_tiles, dim3(grid_for(nslots)), dim3(kBlock), 0, st, groups, ngroups, slot0, nslots,
                           cscan, ctotal, nbox, tiles);
}

void launch_roles(const int32_t* box_pt0, const int32_t* box_pt1, const int32_t* box_parent, const int8_t* box_lev,
                  const int32_t* box_inst, const InstInfo* inst, int64_t nbox, int8_t* role, hipStream_t st) {
    if (nbox <= 0) return;
    hipLaunchKernelGGL(k_roles, dim3(grid_for(nbox)), dim3(kBlock), 0, st, box_pt0, box_pt1, box_parent, box_lev,
                       box_inst, inst, nbox, role);
}

void launch_filter_interactions(const int8_t* role, int64_t nbox, int32_t* il27, hipStream_t st) {
    if (nbox <= 0) return;
    hipLaunchKernelGGL(k_filter_interactions, dim3(grid_for(nbox * kNumInteractions)), dim3(kBlock), 0, st, role,
                       nbox, il27);
}

void launch_adaptive_lists(bool fill, const uint64_t* box_key, const int32_t* box_parent, const int32_t* box_child,
                           const int8_t* box_lev, const int8_t* role, const int32_t* nb9, const int32_t* box_pt0,
                           const int32_t* box_pt1, int64_t nbox, int32_t* cnt, const int32_t* off,
                           int32_t* const* ent, hipStream_t st) {
    if (nbox <= 0) return;
    ListOut o{};
    o.fill = fill;
    o.cnt = cnt;
    o.nbox = nbox;
    for (int r = 0; r < 3; ++r) {
        o.off[r] = off ? off + size_t(r) * size_t(nbox + 1) : nullptr;
        o.ent[r] = ent ? ent[r] : nullptr;
    }
    hipLaunchKernelGGL(k_adaptive_lists, dim3(grid_for(nbox + 1)), dim3(kBlock), 0, st, box_key, box_parent,
                       box_child, box_lev, role, nb9, box_pt0, box_pt1, nbox, o);
}

void launch_compact_positive(const int32_t* cnt, const int32_t* pos, int64_t nbox, int32_t* items, hipStream_t st) {
    if (nbox <= 0) return;
    hipLaunchKernelGGL(k_compact_positive, dim3(grid_for(nbox)), dim3(kBlock), 0, st, cnt, pos, nbox, items);
}

void launch_point_boxes(const int32_t* box_pt0, const int32_t* box_pt1, int32_t nleaf, int32_t* pt_box,
                        hipStream_t st) {
    if (nleaf <= 0) return;
    hipLaunchKernelGGL(k_point_boxes, dim3(grid_for(nleaf)), dim3(kBlock), 0, st, box_pt0, box_pt1, nleaf, pt_box);
}

void launch_near_groups(int32_t q0, int32_t h1_start, int32_t h1_count, const int32_t* roots, int32_t nroots,
                        const int32_t* box_child, const int32_t* nb9, const int32_t* box_pt0,
                        const int32_t* box_pt1, const uint64_t* box_key, NearGroup* groups, int4* ents,
                        hipStream_t st) {
    const int32_t n = h1_count + nroots;
    if (n <= 0) return;
    hipLaunchKernelGGL(k_near_groups, dim3(grid_for(int64_t(n) * 16)), dim3(kBlock), 0, st, q0, h1_start, h1_count,
                       roots, nroots,
                       box_child, nb9, box_pt0, box_pt1, box_key, groups, ents);
}

}  // namespace lfmm
