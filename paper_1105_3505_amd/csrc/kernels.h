// Device-side data layouts and kernel launchers of the lattice FMM (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace lfmm {

// Skeleton size the kernels are compiled for: every expansion vector holds kRankPad FP64
// coefficients (the ID rank is capped there; unused slots stay zero).  Three 16-row tiles
// of the 16x16x4 FP64 matrix instruction.
constexpr int kRankPad = 48;

// Interaction offsets: the 27 boxes of a box's interaction list (Definition 6.1) lie at
// offsets (dx, dy) in [-3, 3]^2 minus [-1, 1]^2 that depend only on the box's position c in
// its parent (c = x bit + 2 y bit).  Offsets index a 7 x 7 grid, d = (dy + 3) * 7 + dx + 3.
constexpr int kNumIfoSlots = 49;
constexpr int kNumInteractions = 27;

struct M2LTile {        // up to 16 boxes of one level and one child position
    int32_t height;     // height above the leaf level (selects the operators)
    int32_t cls;        // child position c of every box in the tile
    int32_t start;      // first entry in the class-sorted box array
    int32_t count;      // 1..16
};

// Per leaf side: operators in device memory (uploaded once, shared by every plan).
struct DevOps {
    int64_t leaf_side = 0;
    int nlev = 0;                  // heights 0 .. nlev-1
    double* leafT = nullptr;       // [side^2][kRankPad]: T_ofs column of each cell, cell-major
    double* ofo_cm = nullptr;      // [nlev][4][q child][r parent]  (M2M reads columns)
    double* ofo_rm = nullptr;      // [nlev][4][r parent][q child]  (L2L reads rows)
    double* ifo = nullptr;         // [nlev][49][p][q] row-major T_ifo per offset slot
    // mixed precision: T_ifo^d = c_d 1 1^T + R^d with c_d the mean entry; R^d in FP32 hi + lo
    float* ifo_hi = nullptr;
    float* ifo_lo = nullptr;
    double* mono = nullptr;        // [nlev][49] c_d
    int32_t* rank = nullptr;       // [nlev] skeleton size of each height
};

// ---- launchers (all enqueue on `st`) ----------------------------------------------------
void launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t st);
void launch_bbox(const int32_t* xy, int64_t n, int32_t* out4, hipStream_t st);
void launch_morton(const int32_t* xy, int64_t n, int32_t ox, int32_t oy, uint64_t* keys,
                   uint32_t* vals, hipStream_t st);
// LSD radix sort of (keys, vals) on bits [0, nbits); tmp buffers of the same sizes.  The
// sorted result ends in (keys, vals).  scratch: radix_scratch_bytes(n) bytes.
size_t radix_scratch_bytes(int64_t n);
void radix_sort_pairs(uint64_t* keys, uint32_t* vals, uint64_t* keys_tmp, uint32_t* vals_tmp,
                      int64_t n, int nbits, void* scratch, hipStream_t st);
// exclusive scan of `rows` rows of n int32 each (row stride n); totals[rows] if non-null.
size_t scan_scratch_bytes(int64_t n, int rows);
void scan_rows(const int32_t* in, int32_t* out, int64_t n, int rows, int32_t* totals,
               void* scratch, hipStream_t st);
void launch_gather_points(const int32_t* xy, const uint32_t* perm, int64_t n, int32_t ox,
                          int32_t oy, int32_t* pts, int32_t* perm_out, hipStream_t st);
void launch_level_stats(const uint64_t* keys, int64_t n, int D, int nleaf, int8_t* cl,
                        int32_t* hist /*[D+2]*/, int32_t* maxc, hipStream_t st);
void launch_leaf_flags(const int8_t* cl, int64_t n, int L, int32_t* flags, hipStream_t st);
void launch_leaf_scatter(const int32_t* flags, const int32_t* scan, const uint64_t* keys,
                         const int8_t* cl, int64_t n, int D, int L, int32_t* leaf_pt0,
                         uint64_t* leaf_key, int8_t* leaf_cl, hipStream_t st);
void launch_level_flags(const int8_t* leaf_cl, int64_t nleaf, int L, int32_t* flags,
                        hipStream_t st);
void launch_build_boxes(const int32_t* lvl_scan, const int8_t* leaf_cl, const int32_t* leaf_pt0,
                        const uint64_t* leaf_key, int64_t nleaf, int L, const int32_t* level_off,
                        int64_t npts, uint64_t* box_key, int32_t* box_pt0, int32_t* box_pt1,
                        int32_t* box_parent, int32_t* box_child, hipStream_t st);
void launch_box_ends(const int32_t* level_off_host, int L, int64_t npts, const int32_t* box_pt0,
                     int32_t* box_pt1, hipStream_t st);
void launch_lists(const uint64_t* box_key, const int32_t* level_off_host, int L,
                  int32_t* ilist, int32_t* nlist, int32_t* cls_cnt, int32_t* cls_box,
                  hipStream_t st);
void launch_m2l_tiles(const int32_t* cls_cnt, const int32_t* level_off_host, int L,
                      M2LTile* tiles, int32_t* ntiles, hipStream_t st);

// ---- evaluation passes --------------------------------------------------------------------
void launch_gather_f(const double* f, const int32_t* perm, int64_t n, double* fs, hipStream_t st);
void launch_p2m_dense(int64_t nleaves, int32_t leaf_off, const int32_t* box_pt0,
                      const int32_t* box_pt1, const uint64_t* box_key, int L, int64_t side,
                      const int32_t* pts, const double* fs, const double* leafT, double* Q,
                      hipStream_t st);
void launch_m2m(int32_t box_begin, int32_t box_end, int height, const int32_t* box_child,
                const double* ofo_cm, const double* Q_in, double* Q_out, hipStream_t st);
void launch_l2l(int32_t box_begin, int32_t box_end, int height_parent, const int32_t* box_parent,
                const uint64_t* box_key, const double* ofo_rm, double* U, hipStream_t st);
void launch_m2l(const M2LTile* tiles, const int32_t* ntiles, int32_t max_tiles,
                const int32_t* cls_box, const int32_t* ilist, int32_t ilist_off, const double* Q,
                double* U, const double* ifo, bool simple, hipStream_t st);
// window keys 8 (y (4 side - 1) + x) mod 2^32 of the Morton-ordered points
void launch_point_keys(const int32_t* pts, int64_t n, int64_t side, uint32_t* key, hipStream_t st);
void launch_m2l_mixed(const M2LTile* tiles, const int32_t* ntiles, int32_t max_tiles, const int32_t* cls_box,
                      const int32_t* ilist, int32_t ilist_off, const double* Q, double* U, const float* ifo_hi,
                      const float* ifo_lo, const double* mono, const int32_t* rank, hipStream_t st);
void launch_leaf_eval(int64_t nleaves, int32_t leaf_off, const int32_t* box_pt0,
                      const int32_t* box_pt1, const uint64_t* box_key, const int32_t* nlist,
                      int L, int64_t side, const int32_t* pts, const uint32_t* pkey, const double* fs,
                      const int32_t* perm, const double* U, const double* leafT, bool far,
                      const double* phi_oct, double* u, bool simple, hipStream_t st);
void launch_direct(int64_t nt, const int32_t* txy, int64_t ns, const int32_t* sxy,
                   const double* f, const double* phi_oct, double* u, hipStream_t st);

}  // namespace lfmm
