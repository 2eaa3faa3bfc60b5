// Quadtree construction on the GPU (Section 6, Definition 6.1).
//
// Points are shifted to the origin of the root box [0, 2^D)^2 and given Morton keys (the
// first coordinate in the even bits), so that every box of every level is a contiguous run
// of the key-sorted points and the boxes of a level are sorted by key.  A leaf level L is
// the smallest level whose boxes hold at most N_leaf points (Section 6).  The common-prefix
// length of consecutive keys tells, per point, at which levels a new box starts; one pass
// over the sorted keys therefore yields L and the box count of every level.
#include "kernels.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstdio>
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

// number of levels at which the boxes of keys a and b coincide (keys hold 2D bits)
__device__ inline int common_levels(uint64_t a, uint64_t b, int D) {
    if (a == b) return D;
    int lz = __clzll(a ^ b) - (64 - 2 * D);
    return lz >> 1;
}

inline unsigned grid_for(int64_t n, int per_block = kBlock) {
    int64_t g = (n + per_block - 1) / per_block;
    if (g < 1) g = 1;
    return unsigned(g);
}

__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_bbox(const int2* xy, int64_t n, int32_t* out4) {
    int mnx = INT_MAX, mny = INT_MAX, mxx = INT_MIN, mxy = INT_MIN;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
        int2 p = xy[i];
        mnx = min(mnx, p.x); mny = min(mny, p.y);
        mxx = max(mxx, p.x); mxy = max(mxy, p.y);
    }
    __shared__ int s[4][kBlock];
    s[0][threadIdx.x] = mnx; s[1][threadIdx.x] = mny; s[2][threadIdx.x] = mxx; s[3][threadIdx.x] = mxy;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (int(threadIdx.x) < w) {
            s[0][threadIdx.x] = min(s[0][threadIdx.x], s[0][threadIdx.x + w]);
            s[1][threadIdx.x] = min(s[1][threadIdx.x], s[1][threadIdx.x + w]);
            s[2][threadIdx.x] = max(s[2][threadIdx.x], s[2][threadIdx.x + w]);
            s[3][threadIdx.x] = max(s[3][threadIdx.x], s[3][threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        atomicMin(&out4[0], s[0][0]); atomicMin(&out4[1], s[1][0]);
        atomicMax(&out4[2], s[2][0]); atomicMax(&out4[3], s[3][0]);
    }
}

__global__ void k_morton(const int2* xy, int64_t n, int32_t ox, int32_t oy, uint64_t* keys, uint32_t* vals) {
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int2 p = xy[i];
    uint32_t x = uint32_t(int64_t(p.x) - ox), y = uint32_t(int64_t(p.y) - oy);
    keys[i] = spread_bits(x) | (spread_bits(y) << 1);
    vals[i] = uint32_t(i);
}

// ---- radix sort: 8-bit digits, tiles of 4096 keys per block ----------------------------
constexpr int kRsItems = 16;
constexpr int kRsTile = kBlock * kRsItems;

__global__ void k_rs_hist(const uint64_t* keys, int64_t n, int shift, uint32_t* hist, int nblk) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    int64_t base = int64_t(blockIdx.x) * kRsTile;
    for (int i = threadIdx.x; i < kRsTile; i += kBlock) {
        int64_t idx = base + i;
        if (idx < n) atomicAdd(&h[(keys[idx] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[size_t(threadIdx.x) * nblk + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter: within a round of 256 keys, lanes of a wave find equal digits by eight
// ballots; waves are ordered through LDS counts; rounds and blocks are ordered by offsets.
__global__ void k_rs_scatter(const uint64_t* kin, const uint32_t* vin, uint64_t* kout, uint32_t* vout,
                             int64_t n, int shift, const int32_t* offs, int nblk) {
    __shared__ uint32_t running[256];
    __shared__ uint32_t wcnt[kBlock / 64][256];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    running[tid] = uint32_t(offs[size_t(tid) * nblk + blockIdx.x]);
    const int64_t base = int64_t(blockIdx.x) * kRsTile;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int r = 0; r < kRsItems; ++r) {
        for (int w = 0; w < kBlock / 64; ++w) wcnt[w][tid] = 0;
        __syncthreads();
        int64_t idx = base + int64_t(r) * kBlock + tid;
        bool valid = idx < n;
        uint64_t key = valid ? kin[idx] : 0ull;
        uint32_t d = uint32_t((key >> shift) & 255u);
        uint64_t mask = __ballot(valid);
        #pragma unroll
        for (int b = 0; b < 8; ++b) {
            uint64_t bb = __ballot(valid && ((d >> b) & 1u));
            mask &= ((d >> b) & 1u) ? bb : ~bb;
        }
        uint32_t rank = uint32_t(__popcll(mask & lt_mask));
        if (valid && rank == 0) wcnt[wave][d] = uint32_t(__popcll(mask));
        __syncthreads();
        if (valid) {
            uint32_t pre = 0;
            for (int w = 0; w < wave; ++w) pre += wcnt[w][d];
            uint32_t pos = running[d] + pre + rank;
            kout[pos] = key;
            vout[pos] = vin[idx];
        }
        __syncthreads();
        uint32_t add = 0;
        for (int w = 0; w < kBlock / 64; ++w) add += wcnt[w][tid];
        running[tid] += add;
        __syncthreads();
    }
}

// ---- exclusive scan over rows of int32 -------------------------------------------------
constexpr int kScanItems = 8;
constexpr int kScanTile = kBlock * kScanItems;

__device__ inline int32_t block_exclusive_scan(int32_t v, int32_t* total) {
    __shared__ int32_t wsum[kBlock / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int32_t x = v;
    #pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) wsum[wave] = x;
    __syncthreads();
    int32_t pre = 0, tot = 0;
    for (int w = 0; w < kBlock / 64; ++w) {
        if (w < wave) pre += wsum[w];
        tot += wsum[w];
    }
    __syncthreads();
    *total = tot;
    return pre + x - v;
}

__global__ void k_scan_tiles(const int32_t* in, int32_t* out, int64_t n, int32_t* bsum, int nblk) {
    const int row = blockIdx.y;
    const int32_t* rin = in + size_t(row) * n;
    int32_t* rout = out + size_t(row) * n;
    int64_t base = int64_t(blockIdx.x) * kScanTile + int64_t(threadIdx.x) * kScanItems;
    int32_t v[kScanItems];
    int32_t s = 0;
    #pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = (base + k < n) ? rin[base + k] : 0;
        s += v[k];
    }
    int32_t tot;
    int32_t pre = block_exclusive_scan(s, &tot);
    #pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        if (base + k < n) rout[base + k] = pre;
        pre += v[k];
    }
    if (threadIdx.x == 0) bsum[size_t(row) * nblk + blockIdx.x] = tot;
}

__global__ void k_scan_add(int32_t* out, int64_t n, const int32_t* bscan, int nblk) {
    const int row = blockIdx.y;
    int32_t add = bscan[size_t(row) * nblk + blockIdx.x];
    int64_t base = int64_t(blockIdx.x) * kScanTile;
    for (int k = threadIdx.x; k < kScanTile; k += kBlock)
        if (base + k < n) out[size_t(row) * n + base + k] += add;
}

__global__ void k_scan_totals(const int32_t* in, const int32_t* out, int64_t n, int rows, int32_t* totals) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < rows) totals[r] = (n > 0) ? out[size_t(r) * n + n - 1] + in[size_t(r) * n + n - 1] : 0;
}

// ---- levels -------------------------------------------------------------------------------
__global__ void k_gather_points(const int2* xy, const uint32_t* perm, int64_t n, int32_t ox, int32_t oy,
                                int2* pts, int32_t* perm_out) {
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t j = perm[i];
    int2 p = xy[j];
    pts[i] = make_int2(int32_t(int64_t(p.x) - ox), int32_t(int64_t(p.y) - oy));
    perm_out[i] = int32_t(j);
}

__global__ void k_level_stats(const uint64_t* keys, int64_t n, int D, int nleaf, int8_t* cl,
                              int32_t* hist, int32_t* maxc) {
    __shared__ int32_t h[66];
    if (threadIdx.x < 66) h[threadIdx.x] = 0;
    __syncthreads();
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    int mc = -1;
    if (i < n) {
        uint64_t k = keys[i];
        int c = (i == 0) ? -1 : common_levels(k, keys[i - 1], D);
        cl[i] = int8_t(c);
        atomicAdd(&h[c + 1], 1);
        if (i + nleaf < n) mc = common_levels(k, keys[i + nleaf], D);
    }
    // wave max, then one atomic per wave
    for (int o = 32; o > 0; o >>= 1) mc = max(mc, __shfl_xor(mc, o, 64));
    if ((threadIdx.x & 63) == 0 && mc >= 0) atomicMax(maxc, mc);
    __syncthreads();
    if (threadIdx.x < D + 2 && h[threadIdx.x] != 0) atomicAdd(&hist[threadIdx.x], h[threadIdx.x]);
}

__global__ void k_leaf_flags(const int8_t* cl, int64_t n, int L, int32_t* flags) {
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) flags[i] = (cl[i] < L) ? 1 : 0;
}

__global__ void k_leaf_scatter(const int32_t* flags, const int32_t* scan, const uint64_t* keys, const int8_t* cl,
                               int64_t n, int D, int L, int32_t* leaf_pt0, uint64_t* leaf_key, int8_t* leaf_cl) {
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n || !flags[i]) return;
    int32_t j = scan[i];
    leaf_pt0[j] = int32_t(i);
    leaf_key[j] = keys[i] >> (2 * (D - L));
    leaf_cl[j] = cl[i];
}

__global__ void k_level_flags(const int8_t* leaf_cl, int64_t nleaf, int32_t* flags) {
    int64_t b = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    int lev = blockIdx.y;   // rows 0 .. L-1
    if (b < nleaf) flags[size_t(lev) * nleaf + b] = (leaf_cl[b] < lev) ? 1 : 0;
}

struct LevelOffsets { int32_t off[34]; };

// One thread per (level, leaf): the leaf that starts a level-lev box writes that box, links
// it to its parent and records itself as the parent's child.
__global__ void k_build_boxes(const int32_t* lvl_scan, const int8_t* leaf_cl, const int32_t* leaf_pt0,
                              const uint64_t* leaf_key, int64_t nleaf, int L, LevelOffsets lo,
                              uint64_t* box_key, int32_t* box_pt0, int32_t* box_parent, int32_t* box_child) {
    int64_t b = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    int lev = blockIdx.y;   // 0 .. L
    if (b >= nleaf) return;
    int c = leaf_cl[b];
    bool starts = (lev == L) || (c < lev);
    if (!starts) return;
    int32_t j = (lev == L) ? int32_t(b) : lvl_scan[size_t(lev) * nleaf + b];
    int32_t g = lo.off[lev] + j;
    uint64_t key = leaf_key[b] >> (2 * (L - lev));
    box_key[g] = key;
    box_pt0[g] = leaf_pt0[b];
    for (int q = 0; q < 4; ++q) box_child[size_t(g) * 4 + q] = -1;
    if (lev == 0) {
        box_parent[g] = -1;
        return;
    }
    // ancestor at level lev-1 of leaf b: inclusive count of starting leaves minus one
    int32_t p;
    if (lev - 1 == 0) p = 0;
    else p = lvl_scan[size_t(lev - 1) * nleaf + b] + ((c < lev - 1) ? 1 : 0) - 1;
    int32_t pg = lo.off[lev - 1] + p;
    box_parent[g] = pg;
}

__global__ void k_link_children(const uint64_t* box_key, const int32_t* box_parent, int32_t first, int32_t end,
                                int32_t* box_child) {
    int32_t g = first + int32_t(blockIdx.x * blockDim.x + threadIdx.x);
    if (g >= end) return;
    int32_t p = box_parent[g];
    if (p >= 0) box_child[size_t(p) * 4 + int(box_key[g] & 3ull)] = g;
}

__global__ void k_box_ends(const int32_t* box_pt0, int32_t first, int32_t end, int32_t npts, int32_t* box_pt1) {
    int32_t g = first + int32_t(blockIdx.x * blockDim.x + threadIdx.x);
    if (g >= end) return;
    box_pt1[g] = (g + 1 < end) ? box_pt0[g + 1] : npts;
}

__device__ inline int32_t find_box(const uint64_t* keys, int32_t first, int32_t end, uint64_t key) {
    // boxes of one level sorted by key in [first, end)
    int32_t lo = first, hi = end;
    while (lo < hi) {
        int32_t mid = (lo + hi) >> 1;
        if (keys[mid] < key) lo = mid + 1;
        else hi = mid;
    }
    return (lo < end && keys[lo] == key) ? lo : -1;
}

// Interaction lists (27 fixed slots per box of level >= 2, in the order of the offset table)
// and neighbor lists (9 slots per leaf, the leaf itself in the middle), -1 for absent boxes.
__global__ void k_lists(const uint64_t* box_key, LevelOffsets lo, int L, int32_t* ilist, int32_t* nlist,
                        int32_t* cls_cnt, int32_t* cls_box) {
    int lev = blockIdx.y + 2;   // levels 2..L
    int32_t first = lo.off[lev], end = lo.off[lev + 1];
    int32_t g = first + int32_t(blockIdx.x * blockDim.x + threadIdx.x);
    if (g >= end) return;
    uint64_t key = box_key[g];
    int32_t bx = int32_t(compact_bits(key)), by = int32_t(compact_bits(key >> 1));
    int32_t side = 1 << lev;
    int cx = bx & 1, cy = by & 1, cls = cx + 2 * cy;
    int32_t* il = ilist + size_t(g - lo.off[2]) * kNumInteractions;
    int k = 0;
    for (int dy = -2 - cy; dy <= 3 - cy; ++dy) {
        for (int dx = -2 - cx; dx <= 3 - cx; ++dx) {
            if (dx >= -1 && dx <= 1 && dy >= -1 && dy <= 1) continue;
            int32_t x = bx + dx, y = by + dy, idx = -1;
            if (x >= 0 && y >= 0 && x < side && y < side)
                idx = find_box(box_key, first, end, spread_bits(uint32_t(x)) | (spread_bits(uint32_t(y)) << 1));
            il[k++] = idx;
        }
    }
    int32_t slot = atomicAdd(&cls_cnt[(lev - 2) * 4 + cls], 1);
    cls_box[size_t(4) * (first - lo.off[2]) + size_t(cls) * (end - first) + slot] = g;
    if (lev == L) {
        int32_t* nl = nlist + size_t(g - first) * 9;
        int q = 0;
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                int32_t x = bx + dx, y = by + dy, idx = -1;
                if (x >= 0 && y >= 0 && x < side && y < side)
                    idx = find_box(box_key, first, end, spread_bits(uint32_t(x)) | (spread_bits(uint32_t(y)) << 1));
                nl[q++] = idx;
            }
    }
}

// Neighbor lists when the leaf level is 0 or 1 (no interaction lists): every leaf is a
// neighbor of every other.
__global__ void k_lists_shallow(LevelOffsets lo, int L, int32_t* nlist) {
    int32_t first = lo.off[L], end = lo.off[L + 1];
    int32_t g = first + int32_t(threadIdx.x);
    if (g >= end) return;
    for (int q = 0; q < 9; ++q) {
        int32_t other = first + q;
        nlist[size_t(g - first) * 9 + q] = (q < end - first) ? other : -1;
    }
}

__global__ void k_m2l_tiles(const int32_t* cls_cnt, LevelOffsets lo, int L, M2LTile* tiles, int32_t* ntiles) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int32_t t = 0;
    for (int lev = 2; lev <= L; ++lev) {
        int32_t first = lo.off[lev], end = lo.off[lev + 1];
        for (int c = 0; c < 4; ++c) {
            int32_t cnt = cls_cnt[(lev - 2) * 4 + c];
            int32_t start = 4 * (first - lo.off[2]) + c * (end - first);
            for (int32_t s = 0; s < cnt; s += 16) {
                M2LTile tl;
                tl.height = L - lev;
                tl.cls = c;
                tl.start = start + s;
                tl.count = min(16, cnt - s);
                tiles[t++] = tl;
            }
        }
    }
    *ntiles = t;
}

LevelOffsets make_offsets(const int32_t* off, int L) {
    LevelOffsets lo{};
    for (int i = 0; i <= L + 1 && i < 34; ++i) lo.off[i] = off[i];
    return lo;
}

}  // namespace

void launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(n)), dim3(kBlock), 0, st, p, n, v);
}

void launch_bbox(const int32_t* xy, int64_t n, int32_t* out4, hipStream_t st) {
    unsigned g = grid_for(n);
    if (g > 1024) g = 1024;
    hipLaunchKernelGGL(k_bbox, dim3(g), dim3(kBlock), 0, st, reinterpret_cast<const int2*>(xy), n, out4);
}

void launch_morton(const int32_t* xy, int64_t n, int32_t ox, int32_t oy, uint64_t* keys, uint32_t* vals,
                   hipStream_t st) {
    hipLaunchKernelGGL(k_morton, dim3(grid_for(n)), dim3(kBlock), 0, st, reinterpret_cast<const int2*>(xy), n,
                       ox, oy, keys, vals);
}

size_t scan_scratch_bytes(int64_t n, int rows) {
    // block sums of every recursion level, for all rows
    size_t total = 0;
    int64_t m = n;
    while (m > 0) {
        int64_t nb = (m + kScanTile - 1) / kScanTile;
        total += size_t(nb) * rows * 2 * sizeof(int32_t);
        if (nb <= 1) break;
        m = nb;
    }
    return total + 256;
}

void scan_rows(const int32_t* in, int32_t* out, int64_t n, int rows, int32_t* totals, void* scratch,
               hipStream_t st) {
    if (n <= 0 || rows <= 0) return;
    int64_t nb = (n + kScanTile - 1) / kScanTile;
    int32_t* bsum = static_cast<int32_t*>(scratch);
    int32_t* bscan = bsum + size_t(nb) * rows;
    hipLaunchKernelGGL(k_scan_tiles, dim3(unsigned(nb), unsigned(rows)), dim3(kBlock), 0, st, in, out, n, bsum,
                       int(nb));
    if (nb > 1) {
        scan_rows(bsum, bscan, nb, rows, nullptr, bscan + size_t(nb) * rows, st);
        hipLaunchKernelGGL(k_scan_add, dim3(unsigned(nb), unsigned(rows)), dim3(kBlock), 0, st, out, n, bscan,
                           int(nb));
    }
    if (totals)
        hipLaunchKernelGGL(k_scan_totals, dim3(grid_for(rows)), dim3(kBlock), 0, st, in, out, n, rows, totals);
}

size_t radix_scratch_bytes(int64_t n) {
    int64_t nblk = (n + kRsTile - 1) / kRsTile;
    size_t hist = size_t(256) * size_t(nblk) * sizeof(int32_t);
    return 2 * hist + scan_scratch_bytes(256 * nblk, 1) + 256;
}

void radix_sort_pairs(uint64_t* keys, uint32_t* vals, uint64_t* keys_tmp, uint32_t* vals_tmp, int64_t n,
                      int nbits, void* scratch, hipStream_t st) {
    if (n <= 1 || nbits <= 0) return;
    int nblk = int((n + kRsTile - 1) / kRsTile);
    int32_t* hist = static_cast<int32_t*>(scratch);
    int32_t* offs = hist + size_t(256) * nblk;
    void* sscr = offs + size_t(256) * nblk;
    uint64_t *ka = keys, *kb = keys_tmp;
    uint32_t *va = vals, *vb = vals_tmp;
    int passes = (nbits + 7) / 8;
    for (int p = 0; p < passes; ++p) {
        int shift = 8 * p;
        hipLaunchKernelGGL(k_rs_hist, dim3(nblk), dim3(kBlock), 0, st, ka, n, shift,
                           reinterpret_cast<uint32_t*>(hist), nblk);
        scan_rows(hist, offs, int64_t(256) * nblk, 1, nullptr, sscr, st);
        hipLaunchKernelGGL(k_rs_scatter, dim3(nblk), dim3(kBlock), 0, st, ka, va, kb, vb, n, shift, offs, nblk);
        std::swap(ka, kb);
        std::swap(va, vb);
    }
    if (ka != keys) {
        (void)hipMemcpyAsync(keys, ka, size_t(n) * sizeof(uint64_t), hipMemcpyDeviceToDevice, st);
        (void)hipMemcpyAsync(vals, va, size_t(n) * sizeof(uint32_t), hipMemcpyDeviceToDevice, st);
    }
}

void launch_gather_points(const int32_t* xy, const uint32_t* perm, int64_t n, int32_t ox, int32_t oy, int32_t* pts,
                          int32_t* perm_out, hipStream_t st) {
    hipLaunchKernelGGL(k_gather_points, dim3(grid_for(n)), dim3(kBlock), 0, st, reinterpret_cast<const int2*>(xy),
                       perm, n, ox, oy, reinterpret_cast<int2*>(pts), perm_out);
}

void launch_level_stats(const uint64_t* keys, int64_t n, int D, int nleaf, int8_t* cl, int32_t* hist, int32_t* maxc,
                        hipStream_t st) {
    hipLaunchKernelGGL(k_level_stats, dim3(grid_for(n)), dim3(kBlock), 0, st, keys, n, D, nleaf, cl, hist, maxc);
}

void launch_leaf_flags(const int8_t* cl, int64_t n, int L, int32_t* flags, hipStream_t st) {
    hipLaunchKernelGGL(k_leaf_flags, dim3(grid_for(n)), dim3(kBlock), 0, st, cl, n, L, flags);
}

void launch_leaf_scatter(const int32_t* flags, const int32_t* scan, const uint64_t* keys, const int8_t* cl, int64_t n,
                         int D, int L, int32_t* leaf_pt0, uint64_t* leaf_key, int8_t* leaf_cl, hipStream_t st) {
    hipLaunchKernelGGL(k_leaf_scatter, dim3(grid_for(n)), dim3(kBlock), 0, st, flags, scan, keys, cl, n, D, L,
                       leaf_pt0, leaf_key, leaf_cl);
}

void launch_level_flags(const int8_t* leaf_cl, int64_t nleaf, int L, int32_t* flags, hipStream_t st) {
    if (L <= 0) return;
    hipLaunchKernelGGL(k_level_flags, dim3(grid_for(nleaf), unsigned(L)), dim3(kBlock), 0, st, leaf_cl, nleaf,
                       flags);
}

void launch_build_boxes(const int32_t* lvl_scan, const int8_t* leaf_cl, const int32_t* leaf_pt0,
                        const uint64_t* leaf_key, int64_t nleaf, int L, const int32_t* level_off, int64_t npts,
                        uint64_t* box_key, int32_t* box_pt0, int32_t* box_pt1, int32_t* box_parent,
                        int32_t* box_child, hipStream_t st) {
    LevelOffsets lo = make_offsets(level_off, L);
    hipLaunchKernelGGL(k_build_boxes, dim3(grid_for(nleaf), unsigned(L + 1)), dim3(kBlock), 0, st, lvl_scan,
                       leaf_cl, leaf_pt0, leaf_key, nleaf, L, lo, box_key, box_pt0, box_parent, box_child);
    for (int lev = 1; lev <= L; ++lev) {
        int32_t first = level_off[lev], end = level_off[lev + 1];
        hipLaunchKernelGGL(k_link_children, dim3(grid_for(end - first)), dim3(kBlock), 0, st, box_key, box_parent,
                           first, end, box_child);
    }
    for (int lev = 0; lev <= L; ++lev) {
        int32_t first = level_off[lev], end = level_off[lev + 1];
        hipLaunchKernelGGL(k_box_ends, dim3(grid_for(end - first)), dim3(kBlock), 0, st, box_pt0, first, end,
                           int32_t(npts), box_pt1);
    }
}

void launch_lists(const uint64_t* box_key, const int32_t* level_off, int L, int32_t* ilist, int32_t* nlist,
                  int32_t* cls_cnt, int32_t* cls_box, hipStream_t st) {
    LevelOffsets lo = make_offsets(level_off, L);
    if (L >= 2) {
        int32_t maxb = 0;
        for (int lev = 2; lev <= L; ++lev) maxb = std::max(maxb, level_off[lev + 1] - level_off[lev]);
        hipLaunchKernelGGL(k_lists, dim3(grid_for(maxb), unsigned(L - 1)), dim3(kBlock), 0, st, box_key, lo, L,
                           ilist, nlist, cls_cnt, cls_box);
    } else {
        hipLaunchKernelGGL(k_lists_shallow, dim3(1), dim3(64), 0, st, lo, L, nlist);
    }
}

void launch_m2l_tiles(const int32_t* cls_cnt, const int32_t* level_off, int L, M2LTile* tiles, int32_t* ntiles,
                      hipStream_t st) {
    LevelOffsets lo = make_offsets(level_off, L);
    hipLaunchKernelGGL(k_m2l_tiles, dim3(1), dim3(64), 0, st, cls_cnt, lo, L, tiles, ntiles);
}

}  // namespace lfmm
