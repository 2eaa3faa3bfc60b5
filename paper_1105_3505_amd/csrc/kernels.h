// Device-side data layouts and kernel launchers of the lattice FMM (gfx950).
//
// A plan is a forest: K independent point sets (instances) whose trees live in shared
// arrays, so that every pass is one launch over all instances.  Points are concatenated in
// instance order and Morton-sorted inside each instance.  Boxes are numbered by height
// above their instance's leaf level first (all leaves of all instances form the first
// block, height 0), then by instance, then by Morton key; so the boxes one launch of M2M or
// L2L needs (one height, all instances) are one contiguous range.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace lfmm {

// Skeleton size the kernels are compiled for: every expansion vector holds kRankPad FP64
// coefficients (the ID rank is capped there; unused slots stay zero).  Three 16-row tiles
// of the 16x16x4 matrix instruction.
constexpr int kRankPad = 48;

// Interaction offsets: the 27 boxes of a box's interaction list (Definition 6.1) lie at
// offsets (dx, dy) in [-3, 3]^2 minus [-1, 1]^2 that depend only on the box's position c in
// its parent (c = x bit + 2 y bit).  Offsets index a 7 x 7 grid, d = (dy + 3) * 7 + dx + 3.
constexpr int kNumIfoSlots = 49;
constexpr int kNumInteractions = 27;
constexpr int kMaxLevels = 32;

struct InstInfo {                   // one instance of a forest
    int32_t pt0, pt1;               // its Morton-ordered points
    int32_t ox, oy;                 // lower-left corner of its root box
    int32_t D, L;                   // root box side 2^D, leaf level L
    int32_t ops;                    // operator set (leaf side)
    int32_t leaf_rank0;             // leaves of the instances before it (point order)
    int32_t max_leaf;               // N_leaf of Section 6 for this instance
    int32_t lev_base[kMaxLevels];   // first box of level l
    int32_t lev_count[kMaxLevels];  // boxes of level l
};

// Tile of up to 16 target boxes that share their operators (same operator set, height and,
// for M2L and L2L, child position).  Boxes are box_list[start .. start + count) or, when
// box_list is null, the consecutive boxes start .. start + count - 1.
struct BoxTile {
    int32_t ops, height, cls, start, count, pad0, pad1, pad2;
};

// Group of target boxes for the tiled passes: contiguous box range [g0, g1) of one height
// and one operator set; class lists for it start at cls_base (4 regions of g1 - g0 slots).
struct BoxGroup {
    int32_t ops, height, g0, g1, cls_base, tile_base, tile_cap, tile_boxes;
};

// Boxes per tile: the M2L kernels give 32 boxes (two 16-column blocks) to each of their 4
// waves, the M2M / L2L box-matrix kernels 16.
constexpr int kM2LTile = 128;
// bf16 mixed precision: 16-byte groups of 8 bf16 per operator (3 parts x 3 row blocks x 6
// column groups x 16 rows) and per outgoing expansion (3 parts x 6 groups)
constexpr int kBf16OpVecs = 3 * 3 * 6 * 16;
constexpr int kBf16QVecs = 3 * 6;
constexpr int kBoxMatTile = 64;

// Per leaf side: operators in device memory (uploaded once, shared by every plan).
struct DevOps {
    int64_t leaf_side = 0;
    int nlev = 0;                  // heights 0 .. nlev-1
    double* leafT = nullptr;       // [side^2][kRankPad]: T_ofs column of each cell, cell-major
    // sides up to 32 (the near-field kernel with an LDS phi table): the same entries
    // coefficient-major in pairs, [kRankPad / 2][side^2][2], so that lanes evaluating the far
    // field at different cells read one pair each from a span of 16 side^2 bytes
    double* leafTt = nullptr;
    // [nlev][4] operators in the fragment order of ifo below: T_ofo (M2M, rows = parent
    // skeleton) and T_ofo^T (L2L, rows = child skeleton)
    double* ofo_rm = nullptr;
    double* ofo_cm = nullptr;
    // T_ifo per height and offset slot, [nlev][49][48 x 48] in fragment order: element
    // ((m * 6 + j) * 64 + l) * 2 + e is row 16 m + (l % 16), column (l / 16) * 12 + 2 j + e
    double* ifo = nullptr;
    // mixed precision: T_ifo^d = c_d 1 1^T + R^d with c_d the mean entry; R^d in FP32 hi + lo,
    // element ((m * 3 + j) * 64 + l) * 4 + e is row 16 m + (l % 16), column (l / 16) * 12 + 4 j + e
    float* ifo_hi = nullptr;
    float* ifo_lo = nullptr;
    // bf16 mixed precision: R^d = R0 + R1 + R2 (three bf16 parts, each the rounded remainder
    // of the ones before), [nlev][49][kBf16OpVecs] groups of 8 bf16 in fragment order: group
    // ((p * 3 + m) * 6 + s) * 16 + n holds R_p[16 m + n][8 s .. 8 s + 7]
    uint16_t* ifo_b = nullptr;
    double* mono = nullptr;        // [nlev][49] c_d
    int32_t* rank = nullptr;       // [nlev] skeleton size of each height
    int32_t* skel = nullptr;       // [nlev][kRankPad][2] skeleton points, offsets from the box corner
};

// Device copy of the operator pointers of every operator set a plan uses.
struct OpsPtrs {
    const double* leafT;
    const double* ofo_rm;
    const double* ofo_cm;
    const double* ifo;
    const float* ifo_hi;
    const float* ifo_lo;
    const uint16_t* ifo_b;
    const double* mono;
    const int32_t* rank;
    const int32_t* skel;
    int64_t side;
    int32_t nlev, pad;
};

// Far-field expansion of phi in the form of eq. (3.1) (device copy, per context):
// phi ~ -(1/2pi)(log|m| + C) + sum_k |m|^-2k sum_j c[k-1][j] cos(4 j theta)
struct PhiFar {
    double C;
    double c[3][4];
};

// Near-field group: the leaves leaf0 .. leaf0 + nleaf - 1 (the children of one parent box,
// or a root that is a leaf), whose sources are the ne point ranges listed for the group.
struct NearGroup {
    int32_t leaf0, nleaf, ne, pad;
};
// At most 16 source leaves per group (the 4 x 4 block around a parent's children); entry
// (first point, end point, leaf x, leaf y) in leaf coordinates of the group's level.
constexpr int kNearEntries = 16;
// leaf coordinate of a near-field entry that matches every target of its group: both for the
// group's own leaves (one run of points), x alone for the two cells above or below them
constexpr int32_t kNearAll = -(1 << 30);

// Per-execute load/potential pointers of each instance, with the roles of its points: an
// instance's points are its sources followed by its targets (the same points when targets =
// sources).  Point of local index j carries the load f[j] if j < nsrc (else zero), and its
// potential goes to u[j - tgt0] if j >= tgt0 (else nowhere).
// Loads and potentials of one instance for an execute: in the caller's order (f[j] for the
// instance's source j, u[j - tgt0] for its target j), or, with sorted set, indexed by the
// plan's global Morton-ordered point index (f, u then span every point of the plan).
struct ExecPtrs {
    const double* f;
    double* u;
    int32_t nsrc, tgt0;
    int32_t sorted, pad;
};

enum BoxMatMode { kModeM2M = 1, kModeL2L = 2 };

// Adaptive tree (Section 6: a box is refined while it holds more than N_leaf points), kept on
// top of the uniform-depth tree: every box of the uniform tree takes a role.  Boxes below an
// adaptive leaf only relay expansions (their outgoing ones up to the leaf, its incoming one
// down to the finest level, where P2M and L2P run): composing T_ofo with T_ofs, and T_ofs^T
// with T_ofo^T, is the leaf's own operator at its height.
enum BoxRole : int8_t { kRolePruned = 0, kRoleInner = 1, kRoleLeaf = 2 };
// Lists of the adaptive tree (Carrier, Greengard and Rokhlin): for a leaf tau, U = the leaves
// touching it (tau included), W = the boxes whose parents touch tau but which do not touch it,
// inside the colleagues of tau; for any box, X = the leaves coarser than it that touch its
// parent but not it (the dual of W).  V is the interaction list of Definition 6.1 with pruned
// boxes taken out.  CSR rows of the three lists, indexed by box.
// Boxes with at most this many points take no expansion route in the adaptive lists (their
// points are fewer than the skeleton points an expansion would cost): W entries and X lists
// of such boxes turn into direct (U) entries.
constexpr int32_t kDirectMax = kRankPad;
struct AdaptiveLists {
    const int32_t* off[3];     // [nbox + 1] each: U, W, X
    const int32_t* ent[3];
};

// ---- construction (forest_kernels.hip) ---------------------------------------------------
size_t radix_scratch_bytes(int64_t n);
// LSD radix sort of (keys, vals) on bits [0, nbits), 8-bit digits; returns which pair of
// buffers holds the result: 0 = (keys, vals), 1 = (keys_tmp, vals_tmp).  counted0: the tile
// counts of the lowest digit are in the scratch already (launch_keys given the scratch).
int radix_sort_pairs(uint64_t* keys, uint32_t* vals, uint64_t* keys_tmp, uint32_t* vals_tmp,
                     int64_t n, int nbits, bool counted0, void* scratch, hipStream_t st);
// Passes p0 .. p1 - 1 of that sort (pass p: bits [8 p, 8 p + 8), reading the pair pass p - 1
// wrote; pass 0 reads (keys, vals)), so that a sort can start before its bit count is known:
// passes over digits that are zero in every key leave the order unchanged.  Returns the pair
// that holds the data after pass p1 - 1.
int radix_sort_passes(uint64_t* keys, uint32_t* vals, uint64_t* keys_tmp, uint32_t* vals_tmp,
                      int64_t n, int p0, int p1, bool counted0, void* scratch, hipStream_t st);
// Copies len bytes from pinned host memory to device memory with a kernel (ordered on the
// stream like a kernel; no copy engine).  Both 8-byte aligned; the source block must extend to
// the next multiple of 8 bytes.
void launch_upload(void* dst, const void* pinned_src, size_t len, hipStream_t st);
// exclusive scan of `rows` rows of n int32 each (row stride n); totals[rows] if non-null.
// Two launches; scratch holds one sum per 2048 items and row.
size_t scan_scratch_bytes(int64_t n, int rows);
void scan_rows(const int32_t* in, int32_t* out, int64_t n, int rows, int32_t* totals,
               void* scratch, hipStream_t st);

struct Chunk { int32_t inst, begin, end, pad; };   // <= kChunk points of one instance
constexpr int32_t kChunk = 2048;

// {min x, min y, max x, max y} of each of K point sets (n[k] points at xy[k], device; n and xy
// host arrays) into box[4 K] (device)
void launch_extents(int32_t K, const int64_t* n, const int32_t* const* xy, int32_t* box, hipStream_t st);
void launch_concat(int32_t K, const int32_t* const* xy_tab, const int32_t* pt_off, int64_t n,
                   int32_t* xyc, hipStream_t st);
// partial root boxes per chunk; also zeroes *dmax
void launch_bbox_chunks(const int32_t* xy, const Chunk* chunks, int32_t nchunks, int32_t* part,
                        int32_t* dmax, hipStream_t st);
// one block per instance: root boxes to bbox, and the instances' root boxes, depths, point
// ranges and N_leaf (max_leaf, 0 if not positive) into inst; the deepest depth into *dmax
void launch_bbox_final(const int32_t* part, const int32_t* chunk_first, const int32_t* pt_off, int32_t K,
                       int32_t max_leaf, int32_t* bbox, InstInfo* inst, int32_t* dmax, hipStream_t st);
// keys and indices of the points (root boxes from inst, the deepest depth from *dmax);
// zeroes zero[0, nzero); with radix_scratch (of radix_scratch_bytes(n)) also the sort's tile
// counts of the lowest digit
void launch_keys(const int32_t* xy, const int32_t* pt_off, int32_t K, const InstInfo* inst,
                 const int32_t* dmax, int64_t n, uint64_t* keys, uint32_t* vals, int32_t* zero,
                 int32_t nzero, void* radix_scratch, hipStream_t st);
// sorted points (coordinates in the root box, decoded from the keys), instance-local indices
// and instances; per-level box counts and look-ahead maxima of every instance into hist
// ([K][kMaxLevels + 2] counts, then [K] maxima; zero before the launch), copied to host_out
// (host memory) by the last block; *done counts finished blocks (zero before the launch)
// hist: `copies` zeroed copies of [K][kMaxLevels + 2] histograms and K maxima, added up into
// host_out by the last block
constexpr int kLevelStatsCopies = 16;
void launch_level_stats(const uint64_t* keys, const uint32_t* vals, const Chunk* chunks, int32_t nchunks,
                        const InstInfo* inst, int Dmax, int32_t K, int32_t* pts, int32_t* perm_local, int32_t* pinst,
                        int8_t* cl, int32_t* hist, int32_t copies, int32_t* done, int32_t* host_out,
                        hipStream_t st);
// exclusive scans of the flags "a leaf starts here" (per point), "leaf b starts a box of
// level lev" (row lev, per leaf) and "box g is child c of its parent" (row c, per box)
void scan_leaf_starts(const int8_t* cl, const int32_t* pinst, const InstInfo* inst, int64_t n,
                      const uint64_t* keys, int Dmax, const int32_t* pts, uint32_t* pkey, int32_t* leaf_pt0,
                      uint64_t* leaf_key, int8_t* leaf_cl, int32_t* leaf_inst, void* scratch, hipStream_t st);
void scan_level_starts(const int8_t* leaf_cl, const int32_t* leaf_inst, const InstInfo* inst, int64_t nleaf,
                       int Lmax, int32_t* out, void* scratch, hipStream_t st);
void scan_child_classes(const uint64_t* box_key, int64_t nbox, int32_t* out, int32_t* totals, void* scratch,
                        hipStream_t st);
void launch_build_boxes(const int32_t* lscan, const int8_t* leaf_cl, const int32_t* leaf_pt0,
                        const uint64_t* leaf_key, const int32_t* leaf_inst, const InstInfo* inst,
                        int64_t nleaf, int Lmax, uint64_t* box_key, int32_t* box_pt0,
                        int32_t* box_parent, int32_t* box_child, int32_t* box_inst,
                        int8_t* box_lev, hipStream_t st);
void launch_link_boxes(const uint64_t* box_key, const int32_t* box_parent, const int32_t* box_inst,
                       const int8_t* box_lev, const InstInfo* inst, int64_t nbox,
                       const int32_t* box_pt0, int32_t* box_child, int32_t* box_pt1, double* zq,
                       double* zu, hipStream_t st);   // also zeroes the rows zq, zu (kRankPad each)
// neighbour (9 slots, every box) and interaction (27 slots, boxes of level >= 2) lists of
// every box: neighbours by search among the boxes of the same level, then interaction
// lists from the parents' neighbours
void launch_lists(const uint64_t* box_key, const int32_t* box_parent, const int32_t* box_child,
                  const int32_t* box_inst, const int8_t* box_lev, const InstInfo* inst, int64_t nbox, int32_t* nb9,
                  int32_t* il27, hipStream_t st);
// class lists (boxes of each group sorted by child position) and the tiles over them;
// the groups own tile slots [slot0, slot0 + nslots); with role non-null, boxes of role
// kRolePruned below level 3 are left out (cscan / ctotal must count the same boxes)
void launch_class_lists(const BoxGroup* groups, int32_t ngroups, int32_t slot0, int32_t nslots,
                        const int32_t* cscan, const int32_t* ctotal, const uint64_t* box_key,
                        const int8_t* box_lev, const int8_t* role, int64_t nbox, int32_t* cls_box,
                        BoxTile* tiles, hipStream_t st);
// scan_child_classes restricted to the boxes that launch_class_lists keeps for role
void scan_child_classes_active(const uint64_t* box_key, const int8_t* box_lev, const int8_t* role, int64_t nbox,
                               int32_t* out, int32_t* totals, void* scratch, hipStream_t st);
// roles of the boxes of the adaptive tree (N_leaf and leaf level from each box's instance)
void launch_roles(const int32_t* box_pt0, const int32_t* box_pt1, const int32_t* box_parent, const int8_t* box_lev,
                  const int32_t* box_inst, const InstInfo* inst, int64_t nbox, int8_t* role, hipStream_t st);
// interaction-list slots naming a pruned box, or of a pruned box, set to -1 (V lists)
void launch_filter_interactions(const int8_t* role, int64_t nbox, int32_t* il27, hipStream_t st);
// U, W and X lists: fill = false counts them into cnt[3][nbox + 1] (the last of each row
// zero); fill = true writes entries at the row starts off[3][nbox + 1] into ent[3]
void launch_adaptive_lists(bool fill, const uint64_t* box_key, const int32_t* box_parent, const int32_t* box_child,
                           const int8_t* box_lev, const int8_t* role, const int32_t* nb9, const int32_t* box_pt0,
                           const int32_t* box_pt1, int64_t nbox, int32_t* cnt, const int32_t* off,
                           int32_t* const* ent, hipStream_t st);
// the non-empty tiles of in[0, n) to the front of out, in order; their number to *count (device)
void compact_tiles(const BoxTile* in, int32_t n, BoxTile* out, int32_t* count, void* scratch, hipStream_t st);
// items[pos[g]] = g for the boxes with cnt[g] > 0 (pos = exclusive scan of those flags)
void launch_compact_positive(const int32_t* cnt, const int32_t* pos, int64_t nbox, int32_t* items, hipStream_t st);
void scan_positive(const int32_t* cnt, int64_t n, int rows, int32_t* out, int32_t* totals, void* scratch,
                   hipStream_t st);
// finest (height-0) box of every point: the box g of [0, nleaf) with box_pt0[g] <= i < box_pt1[g]
void launch_point_boxes(const int32_t* box_pt0, const int32_t* box_pt1, int32_t nleaf, int32_t* pt_box,
                        hipStream_t st);
// near-field groups [q0, q0 + h1_count + nroots): the children of the height-1 boxes
// h1_start .. h1_start + h1_count - 1, then the root leaves roots[0 .. nroots)
void launch_near_groups(int32_t q0, int32_t h1_start, int32_t h1_count, const int32_t* roots, int32_t nroots,
                        const int32_t* box_child, const int32_t* nb9, const int32_t* box_pt0,
                        const int32_t* box_pt1, const uint64_t* box_key, NearGroup* groups, int4* ents,
                        hipStream_t st);

// ---- evaluation passes (fmm_kernels.hip) ---------------------------------------------------
// P2M of the leaves [leaf0, leaf1); reads the loads (tab per instance, or single for a
// single-instance plan when tab is null) in the caller's order through perm_local / pinst, or
// in Morton order when the entry is sorted, and stores them in Morton order at fs; avg_pts,
// the average number of points per leaf, picks the kernel for leaves too wide for LDS
void launch_p2m(int32_t leaf0, int32_t leaf1, const int32_t* box_pt0, const int32_t* box_pt1,
                const uint64_t* box_key, int64_t side, const int32_t* pts, const ExecPtrs* tab,
                const ExecPtrs& single, const int32_t* perm_local, const int32_t* pinst,
                double* fs, const double* leafT, double* Q, double avg_pts, hipStream_t st);
// M2M over the consecutive-box tiles of one height (Q row zrow is all zeros)
void launch_m2m(const BoxTile* tiles, int32_t ntiles, const int32_t* box_child, const OpsPtrs* ops, double* Q,
                int32_t zrow, hipStream_t st);
// L2L over the class-sorted tiles of one height (U row zrow is all zeros); boxes of role
// kRolePruned (role non-null) take the parent's expansion alone (no M2L wrote theirs)
void launch_l2l(const BoxTile* tiles, int32_t ntiles, const int32_t* box_list, const int32_t* box_parent,
                const OpsPtrs* ops, double* U, int32_t zrow, const int8_t* role, hipStream_t st);
// M2L over the class-sorted tiles, *ntiles_dev of them (max_tiles at most); Q row zrow is all
// zeros (read for absent sources)
void launch_m2l(const BoxTile* tiles, const int32_t* ntiles_dev, int32_t max_tiles, const int32_t* box_list,
                const int32_t* il27, const OpsPtrs* ops, const double* Q, int32_t zrow, double* U, hipStream_t st);
// mixed-precision operands of Q rows [0, nrows): FP32 hi and lo parts and FP64 charge sums
void launch_split_q(const double* Q, int32_t nrows, float* Qh, float* Ql, double* qs, hipStream_t st);
void launch_split_q_bf16(const double* Q, int32_t nrows, uint16_t* Qb, double* qs, hipStream_t st);
void launch_m2l_bf16(const BoxTile* tiles, const int32_t* ntiles_dev, int32_t max_tiles, const int32_t* box_list,
                     const int32_t* il27, const OpsPtrs* ops, const uint16_t* Qb, const double* qs, int32_t zrow,
                     double* U, hipStream_t st);
void launch_m2l_mixed(const BoxTile* tiles, const int32_t* ntiles_dev, int32_t max_tiles,
                      const int32_t* box_list, const int32_t* il27, const OpsPtrs* ops,
                      const float* Qh, const float* Ql, const double* qs, int32_t zrow, double* U,
                      hipStream_t st);
// L2P + near field + un-permutation for the groups [q0, q1) of one leaf side
void launch_near(int32_t q0, int32_t q1, const NearGroup* groups, const int4* ents, const int32_t* box_pt0,
                 const int32_t* box_pt1, const uint64_t* box_key, const int32_t* box_inst, int64_t side,
                 const int32_t* pts, const uint32_t* pkey, const double* fs, const int32_t* perm_local,
                 const ExecPtrs* tab, const ExecPtrs& single, const double* U, const double* leafT,
                 const double* leafTt, const uint8_t* far_inst, const double* phi_oct, const PhiFar* phi_far,
                 hipStream_t st);
// Adaptive tree passes.  P2L (X lists): u-hat of box tau += phi(skeleton of tau - x_j) f_j over
// the points of its X leaves, for the nx boxes xitems.  Near field of the adaptive leaves
// (items): U-list sources, W-list skeletons with their q-hat (M2P), L2P at each point's finest
// box, un-permutation.
void launch_p2l(int32_t nx, const int32_t* xitems, const AdaptiveLists& lists, const int32_t* box_pt0,
                const int32_t* box_pt1, const uint64_t* box_key, const int8_t* box_lev, const int32_t* box_inst,
                const InstInfo* inst, const OpsPtrs* ops, const int32_t* pts, const double* fs, double* U,
                const double* phi_oct, const PhiFar* phi_far, hipStream_t st);
void launch_near_adaptive(int32_t nitems, const int32_t* items, const AdaptiveLists& lists, const int32_t* box_pt0,
                          const int32_t* box_pt1, const uint64_t* box_key, const int8_t* box_lev,
                          const int32_t* box_inst, const InstInfo* inst, const OpsPtrs* ops, const int32_t* pts,
                          const double* fs, const double* Q, const int32_t* pt_box, const double* U,
                          const int32_t* perm_local, const ExecPtrs* tab, const ExecPtrs& single,
                          const uint8_t* far_inst, const double* phi_oct, const PhiFar* phi_far, hipStream_t st);
// Radius of the device phi table: the host's quadrature table (radius 128) followed by the
// far-field expansion for the octant entries up to this radius, filled by
// launch_phi_extend(oct, 128, radius).  4.2 MB: near-field offsets between the wide leaves of
// adaptive trees stay table lookups (a gather) instead of logarithms.
constexpr int kPhiDeviceRadius = 1024;
constexpr size_t kPhiDeviceEntries = size_t(kPhiDeviceRadius + 1) * (kPhiDeviceRadius + 2) / 2;
void launch_phi_extend(double* oct, int r0, int r1, const PhiFar* far, hipStream_t st);
// Sum, sum of magnitudes and count of non-finite entries of f[0, n) into out3 (device);
// scratch holds load_stats_scratch_bytes().
size_t load_stats_scratch_bytes();
void launch_load_stats(const double* f, int64_t n, double* scratch, double* out3, hipStream_t st);
void launch_direct(int64_t nt, const int32_t* txy, int64_t ns, const int32_t* sxy,
                   const double* f, const double* phi_oct, const PhiFar* far, double* u, hipStream_t st);
hipError_t upload_dslots();

}  // namespace lfmm
