// Device part of the C ABI: contexts (phi table and cached operators on the GPU), plans
// (the quadtree of one point set, built on the GPU) and evaluation (Section 8.2 passes).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "api_common.h"
#include "host_math.h"
#include "kernels.h"
#include "lfmm.h"

namespace lfmm {
hipError_t upload_dslots();
}

using namespace lfmm;

namespace {

#define LFMM_HIP(call)                                                                              \
    do {                                                                                            \
        hipError_t e_ = (call);                                                                     \
        if (e_ != hipSuccess) throw HipFailure(std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

struct HipFailure {
    std::string msg;
    explicit HipFailure(std::string m) : msg(std::move(m)) {}
};

struct NoMemory {
    std::string msg;
};

// Device blocks cached by power-of-two size class, so that building and dropping plans
// does not call hipMalloc/hipFree (each costs far more than a small solve).  A block is
// returned only after the work that used it is ordered before any later user (same
// stream, or a synchronisation before the release).
class DevicePool {
  public:
    static size_t size_class(size_t bytes) {
        size_t c = size_t(1) << 16;
        while (c < bytes) c <<= 1;
        return c;
    }
    void* acquire(size_t bytes, size_t* got) {
        size_t cls = size_class(bytes);
        {
            std::lock_guard<std::mutex> lock(mu_);
            auto it = free_.find(cls);
            if (it != free_.end()) {
                void* p = it->second;
                free_.erase(it);
                cached_ -= cls;
                *got = cls;
                return p;
            }
        }
        void* p = nullptr;
        hipError_t e = hipMalloc(&p, cls);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            trim();   // give cached blocks back and try once more
            e = hipMalloc(&p, cls);
            if (e != hipSuccess) {
                (void)hipGetLastError();
                throw NoMemory{"device allocation of " + std::to_string(cls) + " bytes failed"};
            }
        }
        *got = cls;
        return p;
    }
    void release(void* p, size_t cls) {
        std::lock_guard<std::mutex> lock(mu_);
        free_.emplace(cls, p);
        cached_ += cls;
    }
    void trim() {
        std::lock_guard<std::mutex> lock(mu_);
        for (auto& kv : free_) (void)hipFree(kv.second);
        free_.clear();
        cached_ = 0;
    }
    size_t cached_bytes() const { return cached_; }
    ~DevicePool() { trim(); }

  private:
    std::multimap<size_t, void*> free_;
    size_t cached_ = 0;
    std::mutex mu_;
};

// One device allocation carved into aligned pieces (from a pool when one is given).
class Arena {
  public:
    explicit Arena(DevicePool* pool = nullptr) : pool_(pool) {}
    void reserve(size_t bytes) { total_ += align(bytes); }
    void allocate() {
        if (total_ == 0) return;
        if (pool_) {
            base_ = pool_->acquire(total_, &cap_);
            return;
        }
        hipError_t e = hipMalloc(&base_, total_);
        if (e != hipSuccess) {
            base_ = nullptr;
            (void)hipGetLastError();
            throw NoMemory{"device allocation of " + std::to_string(total_) + " bytes failed"};
        }
        cap_ = total_;
    }
    template <class T>
    T* take(size_t count) {
        size_t b = align(count * sizeof(T));
        if (used_ + b > total_) throw HipFailure("arena overflow");
        T* p = reinterpret_cast<T*>(static_cast<char*>(base_) + used_);
        used_ += b;
        return p;
    }
    void release() {
        if (base_) {
            if (pool_) pool_->release(base_, cap_);
            else (void)hipFree(base_);
        }
        base_ = nullptr;
        total_ = used_ = cap_ = 0;
    }
    size_t bytes() const { return cap_; }
    void set_pool(DevicePool* p) { pool_ = p; }
    ~Arena() { release(); }

  private:
    static size_t align(size_t b) { return (b + 255) & ~size_t(255); }
    DevicePool* pool_ = nullptr;
    void* base_ = nullptr;
    size_t total_ = 0, used_ = 0, cap_ = 0;
};

struct CachedOps {
    OperatorSet host;
    DevOps dev;
    Arena mem;
};

}  // namespace

struct lfmm_ctx {
    int device = 0;
    lfmm_options opt{};
    DevicePool pool;             // plan storage and temporaries (declared first: freed last)
    Arena table_mem;
    double* phi_oct = nullptr;   // octant table, radius 128
    std::map<int64_t, CachedOps*> ops;                // deepest operator set per leaf side
    std::vector<std::unique_ptr<CachedOps>> all_ops;  // every set built; plans may hold any
    std::mutex mu;
};

struct lfmm_plan {
    lfmm_ctx* ctx = nullptr;
    CachedOps* ops = nullptr;
    int64_t n = 0;
    int D = 0, L = 0;
    int64_t side = 1;
    std::vector<int32_t> off;    // level offsets, L + 2 entries
    int32_t nboxes = 0, nleaves = 0, leaf_off = 0, ilist_off = 0, max_tiles = 0;
    Arena mem;
    int32_t *pts = nullptr, *perm = nullptr, *box_pt0 = nullptr, *box_pt1 = nullptr, *box_parent = nullptr,
            *box_child = nullptr, *ilist = nullptr, *nlist = nullptr, *cls_cnt = nullptr, *cls_box = nullptr,
            *ntiles = nullptr;
    uint64_t* box_key = nullptr;
    M2LTile* tiles = nullptr;
    double *Q = nullptr, *U = nullptr, *fs = nullptr;
    uint32_t* pkey = nullptr;    // window keys of the points (leaves of side <= 16)
    bool failed = false;
    bool timing = false;
    bool timed_once = false;
    hipEvent_t ev[LFMM_NUM_PHASES + 1] = {};
    ~lfmm_plan() {
        for (auto& e : ev)
            if (e) (void)hipEventDestroy(e);
    }
};

namespace {

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

int bits_for_extent(int64_t extent) {
    // smallest D with extent < 2^D (extent = max coordinate difference + 1 cells)
    int D = 0;
    while ((int64_t(1) << D) < extent) ++D;
    return D;
}

// Uploads (or extends) the operators for leaves of `side` with at least `nlev` heights.
CachedOps* get_ops(lfmm_ctx* ctx, int64_t side, int nlev, hipStream_t st) {
    std::lock_guard<std::mutex> lock(ctx->mu);
    auto it = ctx->ops.find(side);
    if (it != ctx->ops.end() && it->second->host.nlevels >= nlev) return it->second;
    auto co = std::make_unique<CachedOps>();
    nlev = std::max(nlev, 1);
    co->host = build_operators(side, nlev, operator_params(ctx->opt));
    const int P = kRankPad;
    for (auto& lv : co->host.level)
        if (lv.rank > P) throw HipFailure("skeleton rank above the compiled pad");
    const OperatorSet& H = co->host;
    const int64_t s2 = side * side;
    std::vector<double> leafT(size_t(s2) * P, 0.0);
    for (int64_t c = 0; c < s2; ++c)
        for (int p = 0; p < H.level[0].rank; ++p) leafT[size_t(c) * P + p] = H.leaf.T(p, int(c));
    std::vector<double> ofo_cm(size_t(nlev) * 4 * P * P, 0.0), ofo_rm(size_t(nlev) * 4 * P * P, 0.0);
    for (int h = 1; h < nlev; ++h)
        for (int c = 0; c < 4; ++c) {
            const Mat& T = H.level[size_t(h)].ofo[c];
            for (int r = 0; r < T.rows; ++r)
                for (int q = 0; q < T.cols; ++q) {
                    ofo_cm[((size_t(h) * 4 + c) * P + q) * P + r] = T(r, q);
                    ofo_rm[((size_t(h) * 4 + c) * P + r) * P + q] = T(r, q);
                }
        }
    // T_ifo^d[p][q] = phi(yhat_p - yhat_q - d * side_h): incoming skeleton of the target box
    // against the outgoing skeleton of the source box at box offset d (Section 7, 8.1)
    std::vector<double> ifo(size_t(nlev) * kNumIfoSlots * P * P, 0.0);
    for (int h = 0; h < nlev; ++h) {
        const LevelOps& lv = H.level[size_t(h)];
        for (int dy = -3; dy <= 3; ++dy)
            for (int dx = -3; dx <= 3; ++dx) {
                if (std::abs(dx) <= 1 && std::abs(dy) <= 1) continue;
                int slot = (dy + 3) * 7 + (dx + 3);
                double* T = ifo.data() + (size_t(h) * kNumIfoSlots + slot) * P * P;
                for (int p = 0; p < lv.rank; ++p)
                    for (int q = 0; q < lv.rank; ++q)
                        T[size_t(p) * P + q] = phi(lv.skel[2 * p] - lv.skel[2 * q] - dx * lv.side,
                                                   lv.skel[2 * p + 1] - lv.skel[2 * q + 1] - dy * lv.side);
            }
    }
    co->mem.reserve(leafT.size() * sizeof(double));
    co->mem.reserve(ofo_cm.size() * sizeof(double));
    co->mem.reserve(ofo_rm.size() * sizeof(double));
    co->mem.reserve(ifo.size() * sizeof(double));
    // mixed precision: T^d = c_d 1 1^T + R^d (c_d = mean entry over the true rank), R^d split
    // into FP32 hi + lo; padded rows and columns stay zero
    std::vector<float> ifo_hi(ifo.size(), 0.f), ifo_lo(ifo.size(), 0.f);
    std::vector<double> mono(size_t(nlev) * kNumIfoSlots, 0.0);
    std::vector<int32_t> ranks(static_cast<size_t>(nlev), 0);
    for (int h = 0; h < nlev; ++h) {
        const int r = H.level[size_t(h)].rank;
        ranks[size_t(h)] = r;
        for (int slot = 0; slot < kNumIfoSlots; ++slot) {
            const size_t base = (size_t(h) * kNumIfoSlots + slot) * P * P;
            double mean = 0.0;
            for (int p = 0; p < r; ++p)
                for (int q = 0; q < r; ++q) mean += ifo[base + size_t(p) * P + q];
            mean /= double(r) * double(r);
            mono[size_t(h) * kNumIfoSlots + slot] = mean;
            for (int p = 0; p < r; ++p)
                for (int q = 0; q < r; ++q) {
                    const double rem = ifo[base + size_t(p) * P + q] - mean;
                    const float hi = float(rem);
                    ifo_hi[base + size_t(p) * P + q] = hi;
                    ifo_lo[base + size_t(p) * P + q] = float(rem - double(hi));
                }
        }
    }
    co->mem.reserve(ifo.size() * sizeof(float));
    co->mem.reserve(ifo.size() * sizeof(float));
    co->mem.reserve(mono.size() * sizeof(double));
    co->mem.reserve(ranks.size() * sizeof(int32_t));
    co->mem.allocate();
    co->dev.leaf_side = side;
    co->dev.nlev = nlev;
    co->dev.leafT = co->mem.take<double>(leafT.size());
    co->dev.ofo_cm = co->mem.take<double>(ofo_cm.size());
    co->dev.ofo_rm = co->mem.take<double>(ofo_rm.size());
    co->dev.ifo = co->mem.take<double>(ifo.size());
    co->dev.ifo_hi = co->mem.take<float>(ifo.size());
    co->dev.ifo_lo = co->mem.take<float>(ifo.size());
    co->dev.mono = co->mem.take<double>(mono.size());
    co->dev.rank = co->mem.take<int32_t>(ranks.size());
    LFMM_HIP(hipMemcpyAsync(co->dev.leafT, leafT.data(), leafT.size() * 8, hipMemcpyHostToDevice, st));
    LFMM_HIP(hipMemcpyAsync(co->dev.ofo_cm, ofo_cm.data(), ofo_cm.size() * 8, hipMemcpyHostToDevice, st));
    LFMM_HIP(hipMemcpyAsync(co->dev.ofo_rm, ofo_rm.data(), ofo_rm.size() * 8, hipMemcpyHostToDevice, st));
    LFMM_HIP(hipMemcpyAsync(co->dev.ifo, ifo.data(), ifo.size() * 8, hipMemcpyHostToDevice, st));
    LFMM_HIP(hipMemcpyAsync(co->dev.ifo_hi, ifo_hi.data(), ifo.size() * 4, hipMemcpyHostToDevice, st));
    LFMM_HIP(hipMemcpyAsync(co->dev.ifo_lo, ifo_lo.data(), ifo.size() * 4, hipMemcpyHostToDevice, st));
    LFMM_HIP(hipMemcpyAsync(co->dev.mono, mono.data(), mono.size() * 8, hipMemcpyHostToDevice, st));
    LFMM_HIP(hipMemcpyAsync(co->dev.rank, ranks.data(), ranks.size() * 4, hipMemcpyHostToDevice, st));
    LFMM_HIP(hipStreamSynchronize(st));
    CachedOps* raw = co.get();
    ctx->ops[side] = raw;             // a shallower set stays alive for the plans using it
    ctx->all_ops.push_back(std::move(co));
    return raw;
}

void build_plan(lfmm_plan* pl, const int32_t* xy, hipStream_t st) {
    lfmm_ctx* ctx = pl->ctx;
    const int64_t n = pl->n;
    const int nleaf_max = ctx->opt.max_leaf;

    // ---- temporaries sized by n ----------------------------------------------------------
    Arena tmp(&ctx->pool);
    // one reserve per take below (each piece is 256-byte aligned)
    tmp.reserve(4 * 4);                             // bbox
    tmp.reserve(64 * 4);                            // level histogram + max
    tmp.reserve(size_t(n) * 8);                     // keys
    tmp.reserve(size_t(n) * 8);                     // keys_tmp
    tmp.reserve(size_t(n) * 4);                     // vals
    tmp.reserve(size_t(n) * 4);                     // vals_tmp
    tmp.reserve(size_t(n));                         // cl
    tmp.reserve(size_t(n) * 4);                     // flags
    tmp.reserve(size_t(n) * 4);                     // scan
    tmp.reserve(radix_scratch_bytes(n));
    tmp.reserve(scan_scratch_bytes(n, 1));
    tmp.allocate();
    int32_t* bbox = tmp.take<int32_t>(4);
    int32_t* stats = tmp.take<int32_t>(64);
    uint64_t* keys = tmp.take<uint64_t>(n);
    uint64_t* keys_tmp = tmp.take<uint64_t>(n);
    uint32_t* vals = tmp.take<uint32_t>(n);
    uint32_t* vals_tmp = tmp.take<uint32_t>(n);
    int8_t* cl = tmp.take<int8_t>(n);
    int32_t* flags = tmp.take<int32_t>(n);
    int32_t* scan = tmp.take<int32_t>(n);
    void* rscr = tmp.take<char>(radix_scratch_bytes(n));
    void* sscr = tmp.take<char>(scan_scratch_bytes(n, 1));

    // ---- root box --------------------------------------------------------------------------
    int32_t init[4] = {INT32_MAX, INT32_MAX, INT32_MIN, INT32_MIN};
    LFMM_HIP(hipMemcpyAsync(bbox, init, sizeof(init), hipMemcpyHostToDevice, st));
    launch_bbox(xy, n, bbox, st);
    int32_t bb[4];
    LFMM_HIP(hipMemcpyAsync(bb, bbox, sizeof(bb), hipMemcpyDeviceToHost, st));
    LFMM_HIP(hipStreamSynchronize(st));
    const int64_t extent = std::max(int64_t(bb[2]) - bb[0], int64_t(bb[3]) - bb[1]) + 1;
    if (extent > (int64_t(1) << 31)) throw std::out_of_range("coordinate extent of 2^31 or more");
    const int D = bits_for_extent(extent);
    pl->D = D;

    // ---- Morton order ----------------------------------------------------------------------
    launch_morton(xy, n, bb[0], bb[1], keys, vals, st);
    radix_sort_pairs(keys, vals, keys_tmp, vals_tmp, n, 2 * D, rscr, st);

    // ---- leaf level and box counts ----------------------------------------------------------
    LFMM_HIP(hipMemsetAsync(stats, 0, 64 * 4, st));
    launch_level_stats(keys, n, D, nleaf_max, cl, stats, stats + 40, st);
    int32_t hs[64];
    LFMM_HIP(hipMemcpyAsync(hs, stats, sizeof(hs), hipMemcpyDeviceToHost, st));
    LFMM_HIP(hipStreamSynchronize(st));
    int L = (n > nleaf_max) ? std::min(D, hs[40] + 1) : 0;
    // leaves no wider than the dense-model limit (Remark 8.2)
    int min_L = 0;
    while ((int64_t(1) << (D - min_L)) > kDenseLeafMax) ++min_L;
    L = std::max(L, min_L);
    pl->L = L;
    pl->side = int64_t(1) << (D - L);
    pl->off.assign(size_t(L) + 2, 0);
    for (int lev = 0; lev <= L; ++lev) {
        int32_t b = 0;
        for (int c = -1; c < lev; ++c) b += hs[c + 1];
        pl->off[size_t(lev) + 1] = pl->off[size_t(lev)] + b;
    }
    pl->nboxes = pl->off[size_t(L) + 1];
    pl->nleaves = pl->off[size_t(L) + 1] - pl->off[size_t(L)];
    pl->leaf_off = pl->off[size_t(L)];
    pl->ilist_off = (L >= 2) ? pl->off[2] : pl->nboxes;
    const int32_t n_m2l = pl->nboxes - pl->ilist_off;
    int32_t max_tiles = 0;
    for (int lev = 2; lev <= L; ++lev) max_tiles += (pl->off[size_t(lev) + 1] - pl->off[size_t(lev)] + 15) / 16 + 4;
    pl->max_tiles = max_tiles;

    // ---- plan storage ------------------------------------------------------------------------
    const int P = kRankPad;
    const int64_t nb = pl->nboxes, nl = pl->nleaves;
    Arena& m = pl->mem;
    m.set_pool(&ctx->pool);
    // one reserve per take below (each piece is 256-byte aligned)
    m.reserve(size_t(n) * 8);                   // pts
    m.reserve(size_t(n) * 4);                   // perm
    m.reserve(size_t(n) * 8);                   // fs
    m.reserve(size_t(nb) * 8);                  // box_key
    m.reserve(size_t(nb) * 4);                  // pt0
    m.reserve(size_t(nb) * 4);                  // pt1
    m.reserve(size_t(nb) * 4);                  // parent
    m.reserve(size_t(nb) * 16);                 // child
    m.reserve(size_t(std::max(n_m2l, 1)) * 4 * kNumInteractions);
    m.reserve(size_t(nl) * 4 * 9);
    m.reserve(4 * 4 * 34);                      // class counters
    m.reserve(size_t(std::max(n_m2l, 1)) * 4 * 4);   // class-sorted boxes (4 regions per level)
    m.reserve(4 * 4);                           // tile count
    m.reserve(size_t(max_tiles + 1) * sizeof(M2LTile));
    m.reserve(size_t(nb) * P * 8);              // Q
    m.reserve(size_t(nb) * P * 8);              // U
    m.reserve(size_t(n) * 4);                   // point keys
    m.allocate();
    pl->pts = m.take<int32_t>(size_t(n) * 2);
    pl->perm = m.take<int32_t>(n);
    pl->fs = m.take<double>(n);
    pl->box_key = m.take<uint64_t>(nb);
    pl->box_pt0 = m.take<int32_t>(nb);
    pl->box_pt1 = m.take<int32_t>(nb);
    pl->box_parent = m.take<int32_t>(nb);
    pl->box_child = m.take<int32_t>(size_t(nb) * 4);
    pl->ilist = m.take<int32_t>(size_t(std::max(n_m2l, 1)) * kNumInteractions);
    pl->nlist = m.take<int32_t>(size_t(nl) * 9);
    pl->cls_cnt = m.take<int32_t>(4 * 34);
    pl->cls_box = m.take<int32_t>(size_t(std::max(n_m2l, 1)) * 4);
    pl->ntiles = m.take<int32_t>(4);
    pl->tiles = m.take<M2LTile>(size_t(max_tiles + 1));
    pl->Q = m.take<double>(size_t(nb) * P);
    pl->U = m.take<double>(size_t(nb) * P);
    pl->pkey = m.take<uint32_t>(n);

    launch_gather_points(xy, vals, n, bb[0], bb[1], pl->pts, pl->perm, st);
    if (pl->side <= 16) launch_point_keys(pl->pts, n, pl->side, pl->pkey, st);

    // ---- leaves ------------------------------------------------------------------------------
    // level-scan temporaries reuse the sort buffers: leaf arrays need <= n entries each
    int32_t* leaf_pt0 = reinterpret_cast<int32_t*>(keys_tmp);
    Arena tmp2(&ctx->pool);
    tmp2.reserve(size_t(nl) * 8);                              // leaf keys
    tmp2.reserve(size_t(nl));                                  // leaf cl
    tmp2.reserve(size_t(std::max(L, 1)) * nl * 4);             // level flags
    tmp2.reserve(size_t(std::max(L, 1)) * nl * 4);             // level scans
    tmp2.reserve(scan_scratch_bytes(nl, std::max(L, 1)));
    tmp2.allocate();
    uint64_t* lkey = tmp2.take<uint64_t>(nl);
    int8_t* lcl = tmp2.take<int8_t>(nl);
    int32_t* lflags = tmp2.take<int32_t>(size_t(std::max(L, 1)) * nl);
    int32_t* lscan = tmp2.take<int32_t>(size_t(std::max(L, 1)) * nl);
    void* lscr = tmp2.take<char>(scan_scratch_bytes(nl, std::max(L, 1)));

    launch_leaf_flags(cl, n, L, flags, st);
    scan_rows(flags, scan, n, 1, nullptr, sscr, st);
    launch_leaf_scatter(flags, scan, keys, cl, n, D, L, leaf_pt0, lkey, lcl, st);
    if (L > 0) {
        launch_level_flags(lcl, nl, L, lflags, st);
        scan_rows(lflags, lscan, nl, L, nullptr, lscr, st);
    }
    launch_build_boxes(lscan, lcl, leaf_pt0, lkey, nl, L, pl->off.data(), n, pl->box_key, pl->box_pt0,
                       pl->box_pt1, pl->box_parent, pl->box_child, st);
    LFMM_HIP(hipMemsetAsync(pl->cls_cnt, 0, 4 * 4 * 34, st));
    launch_lists(pl->box_key, pl->off.data(), L, pl->ilist, pl->nlist, pl->cls_cnt, pl->cls_box, st);
    if (L >= 2) {
        launch_m2l_tiles(pl->cls_cnt, pl->off.data(), L, pl->tiles, pl->ntiles, st);
    } else {
        LFMM_HIP(hipMemsetAsync(pl->ntiles, 0, 4, st));
    }
    LFMM_HIP(hipGetLastError());
    pl->ops = get_ops(ctx, pl->side, std::max(L - 1, 1), st);
    LFMM_HIP(hipStreamSynchronize(st));
    tmp.release();
    tmp2.release();
}

void run_plan(lfmm_plan* pl, const double* f, double* u, hipStream_t st) {
    const DevOps& op = pl->ops->dev;
    const int L = pl->L;
    const bool simple = (pl->ctx->opt.flags & LFMM_FLAG_SIMPLE_KERNELS) != 0;
    auto mark = [&](int k) {
        if (pl->timing) LFMM_HIP(hipEventRecord(pl->ev[k], st));
    };
    mark(0);
    launch_gather_f(f, pl->perm, pl->n, pl->fs, st);
    mark(1);
    const bool far = L >= 2;
    if (far) {
        launch_p2m_dense(pl->nleaves, pl->leaf_off, pl->box_pt0, pl->box_pt1, pl->box_key, L, pl->side, pl->pts,
                         pl->fs, op.leafT, pl->Q, st);
    }
    mark(2);
    if (far) {
        for (int lev = L - 1; lev >= 2; --lev)
            launch_m2m(pl->off[size_t(lev)], pl->off[size_t(lev) + 1], L - lev, pl->box_child, op.ofo_cm, pl->Q,
                       pl->Q, st);
    }
    mark(3);
    if (far) {
        if (pl->ctx->opt.precision == LFMM_MIXED)
            launch_m2l_mixed(pl->tiles, pl->ntiles, pl->max_tiles, pl->cls_box, pl->ilist, pl->ilist_off, pl->Q,
                             pl->U, op.ifo_hi, op.ifo_lo, op.mono, op.rank, st);
        else
            launch_m2l(pl->tiles, pl->ntiles, pl->max_tiles, pl->cls_box, pl->ilist, pl->ilist_off, pl->Q, pl->U,
                       op.ifo, simple, st);
    }
    mark(4);
    if (far) {
        for (int lev = 2; lev <= L - 1; ++lev)
            launch_l2l(pl->off[size_t(lev) + 1], pl->off[size_t(lev) + 2], L - lev, pl->box_parent, pl->box_key,
                       op.ofo_rm, pl->U, st);
    }
    mark(5);
    launch_leaf_eval(pl->nleaves, pl->leaf_off, pl->box_pt0, pl->box_pt1, pl->box_key, pl->nlist, L, pl->side,
                     pl->pts, pl->side <= 16 ? pl->pkey : nullptr, pl->fs, pl->perm, pl->U, op.leafT, far,
                     pl->ctx->phi_oct, u, simple, st);
    mark(6);
    if (pl->timing) pl->timed_once = true;
}

template <class F>
lfmm_status guarded(F&& f) {
    // the per-thread "last error" may hold an error from another library's HIP call (the
    // caller's framework shares this thread): clear it so that only our launches are checked
    (void)hipGetLastError();
    try {
        return f();
    } catch (const HipFailure& e) {
        return fail(LFMM_E_HIP, e.msg);
    } catch (const NoMemory& e) {
        return fail(LFMM_E_NOMEM, e.msg);
    } catch (const std::bad_alloc&) {
        return fail(LFMM_E_NOMEM, "host allocation failed");
    } catch (const std::out_of_range& e) {
        return fail(LFMM_E_RANGE, e.what());
    } catch (const std::exception& e) {
        return fail(LFMM_E_INVAL, e.what());
    }
}

}  // namespace

extern "C" {

lfmm_status lfmm_ctx_create(int32_t device, const lfmm_options* opt, lfmm_ctx** out) {
    if (!out) return fail(LFMM_E_INVAL, "null output");
    *out = nullptr;
    lfmm_options o;
    lfmm_options_init(&o);
    if (opt) o = *opt;
    lfmm_status st = validate_options(&o);
    if (st != LFMM_OK) return st;
    if (o.max_rank > kRankPad) return fail(LFMM_E_UNSUPPORTED, "max_rank above the compiled pad of 48");
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) {
        (void)hipGetLastError();
        return fail(LFMM_E_NODEVICE, "no HIP device " + std::to_string(device));
    }
    return guarded([&]() -> lfmm_status {
        LFMM_HIP(hipSetDevice(device));
        auto ctx = std::make_unique<lfmm_ctx>();
        ctx->device = device;
        ctx->opt = o;
        const std::vector<double>& tab = phi_table();
        ctx->table_mem.reserve(tab.size() * sizeof(double));
        ctx->table_mem.allocate();
        ctx->phi_oct = ctx->table_mem.take<double>(tab.size());
        LFMM_HIP(hipMemcpy(ctx->phi_oct, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice));
        LFMM_HIP(upload_dslots());
        LFMM_HIP(hipDeviceSynchronize());
        *out = ctx.release();
        return LFMM_OK;
    });
}

lfmm_status lfmm_ctx_destroy(lfmm_ctx* ctx) {
    if (!ctx) return LFMM_OK;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    delete ctx;
    return LFMM_OK;
}

lfmm_status lfmm_plan_create(lfmm_ctx* ctx, int64_t n, const int32_t* xy, void* stream, lfmm_plan** out) {
    if (!ctx || !out || !xy) return fail(LFMM_E_INVAL, "null argument");
    *out = nullptr;
    if (n < 1 || n > (int64_t(1) << 30)) return fail(LFMM_E_INVAL, "n must lie in [1, 2^30]");
    return guarded([&]() -> lfmm_status {
        LFMM_HIP(hipSetDevice(ctx->device));
        auto pl = std::make_unique<lfmm_plan>();
        pl->ctx = ctx;
        pl->n = n;
        build_plan(pl.get(), xy, as_stream(stream));
        *out = pl.release();
        return LFMM_OK;
    });
}

lfmm_status lfmm_execute(lfmm_plan* pl, const double* f, double* u, void* stream) {
    if (!pl || !f || !u) return fail(LFMM_E_INVAL, "null argument");
    if (pl->failed) return fail(LFMM_E_HIP, "plan is in a failed state");
    return guarded([&]() -> lfmm_status {
        LFMM_HIP(hipSetDevice(pl->ctx->device));
        run_plan(pl, f, u, as_stream(stream));
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) {
            pl->failed = true;
            throw HipFailure(std::string("kernel launch: ") + hipGetErrorString(e));
        }
        return LFMM_OK;
    });
}

lfmm_status lfmm_execute_batch(lfmm_ctx* ctx, int32_t n_plans, lfmm_plan* const* plans, const double* const* f,
                               double* const* u, void* stream) {
    if (!ctx || n_plans < 0 || (n_plans > 0 && (!plans || !f || !u))) return fail(LFMM_E_INVAL, "null argument");
    for (int32_t k = 0; k < n_plans; ++k) {
        if (!plans[k] || plans[k]->ctx != ctx) return fail(LFMM_E_INVAL, "plan of another context");
        lfmm_status s = lfmm_execute(plans[k], f[k], u[k], stream);
        if (s != LFMM_OK) return s;
    }
    return LFMM_OK;
}

lfmm_status lfmm_plan_get_info(lfmm_plan* pl, lfmm_plan_info* out) {
    if (!pl || !out) return fail(LFMM_E_INVAL, "null argument");
    return guarded([&]() -> lfmm_status {
        LFMM_HIP(hipSetDevice(pl->ctx->device));
        std::memset(out, 0, sizeof(*out));
        out->n_points = pl->n;
        out->root_bits = pl->D;
        out->leaf_level = pl->L;
        out->leaf_side = pl->side;
        out->rank = kRankPad;
        out->leaf_kind = 0;
        out->n_boxes = pl->nboxes;
        out->n_leaves = pl->nleaves;
        // pair counts from the lists (host side, for reporting)
        std::vector<int32_t> pt0(size_t(pl->nboxes)), pt1(size_t(pl->nboxes)), nl(size_t(pl->nleaves) * 9);
        LFMM_HIP(hipMemcpy(pt0.data(), pl->box_pt0, pt0.size() * 4, hipMemcpyDeviceToHost));
        LFMM_HIP(hipMemcpy(pt1.data(), pl->box_pt1, pt1.size() * 4, hipMemcpyDeviceToHost));
        LFMM_HIP(hipMemcpy(nl.data(), pl->nlist, nl.size() * 4, hipMemcpyDeviceToHost));
        int64_t near = 0;
        for (int32_t b = 0; b < pl->nleaves; ++b) {
            int32_t g = pl->leaf_off + b;
            int64_t nt = pt1[size_t(g)] - pt0[size_t(g)], ns = 0;
            for (int q = 0; q < 9; ++q) {
                int32_t s = nl[size_t(b) * 9 + q];
                if (s >= 0) ns += pt1[size_t(s)] - pt0[size_t(s)];
            }
            near += nt * ns;
        }
        out->near_pairs = near;
        int64_t m2l = 0;
        if (pl->L >= 2) {
            std::vector<int32_t> il(size_t(pl->nboxes - pl->ilist_off) * kNumInteractions);
            LFMM_HIP(hipMemcpy(il.data(), pl->ilist, il.size() * 4, hipMemcpyDeviceToHost));
            for (int32_t v : il) m2l += (v >= 0);
        }
        out->m2l_pairs = m2l;
        return LFMM_OK;
    });
}

lfmm_status lfmm_plan_export(lfmm_plan* pl, int32_t item, void* out, size_t* bytes) {
    if (!pl || !bytes) return fail(LFMM_E_INVAL, "null argument");
    const void* src = nullptr;
    size_t size = 0;
    const size_t nb = size_t(pl->nboxes), n = size_t(pl->n), P = kRankPad;
    switch (item) {
        case LFMM_EXPORT_POINTS: src = pl->pts; size = n * 8; break;
        case LFMM_EXPORT_PERM: src = pl->perm; size = n * 4; break;
        case LFMM_EXPORT_LEVEL_OFFSETS: src = pl->off.data(); size = pl->off.size() * 4; break;
        case LFMM_EXPORT_BOX_KEY: src = pl->box_key; size = nb * 8; break;
        case LFMM_EXPORT_BOX_BEGIN: src = pl->box_pt0; size = nb * 4; break;
        case LFMM_EXPORT_BOX_END: src = pl->box_pt1; size = nb * 4; break;
        case LFMM_EXPORT_BOX_PARENT: src = pl->box_parent; size = nb * 4; break;
        case LFMM_EXPORT_BOX_CHILD: src = pl->box_child; size = nb * 16; break;
        case LFMM_EXPORT_INTERACTION:
            src = pl->ilist;
            size = size_t(pl->nboxes - pl->ilist_off) * kNumInteractions * 4;
            break;
        case LFMM_EXPORT_NEIGHBOR: src = pl->nlist; size = size_t(pl->nleaves) * 9 * 4; break;
        case LFMM_EXPORT_QHAT: src = pl->Q; size = nb * P * 8; break;
        case LFMM_EXPORT_UHAT: src = pl->U; size = nb * P * 8; break;
        case LFMM_EXPORT_LOADS: src = pl->fs; size = n * 8; break;
        default: return fail(LFMM_E_INVAL, "unknown export item");
    }
    if (!out) {
        *bytes = size;
        return LFMM_OK;
    }
    if (*bytes < size) return fail(LFMM_E_INVAL, "output buffer too small");
    *bytes = size;
    return guarded([&]() -> lfmm_status {
        LFMM_HIP(hipSetDevice(pl->ctx->device));
        LFMM_HIP(hipDeviceSynchronize());
        if (item == LFMM_EXPORT_LEVEL_OFFSETS) std::memcpy(out, src, size);
        else if (size) LFMM_HIP(hipMemcpy(out, src, size, hipMemcpyDeviceToHost));
        return LFMM_OK;
    });
}

lfmm_status lfmm_plan_set_timing(lfmm_plan* pl, int32_t enable) {
    if (!pl) return fail(LFMM_E_INVAL, "null plan");
    return guarded([&]() -> lfmm_status {
        LFMM_HIP(hipSetDevice(pl->ctx->device));
        if (enable && !pl->ev[0])
            for (auto& e : pl->ev) LFMM_HIP(hipEventCreate(&e));
        pl->timing = enable != 0;
        return LFMM_OK;
    });
}

lfmm_status lfmm_plan_phase_times(lfmm_plan* pl, double* ms) {
    if (!pl || !ms) return fail(LFMM_E_INVAL, "null argument");
    if (!pl->timed_once) return fail(LFMM_E_INVAL, "no timed execute yet");
    return guarded([&]() -> lfmm_status {
        LFMM_HIP(hipSetDevice(pl->ctx->device));
        LFMM_HIP(hipEventSynchronize(pl->ev[LFMM_NUM_PHASES]));
        for (int k = 0; k < LFMM_NUM_PHASES; ++k) {
            float t = 0.f;
            LFMM_HIP(hipEventElapsedTime(&t, pl->ev[k], pl->ev[k + 1]));
            ms[k] = double(t);
        }
        return LFMM_OK;
    });
}

lfmm_status lfmm_plan_footprint_bytes(const lfmm_ctx* ctx, int64_t n, size_t* out) {
    if (!ctx || !out || n < 0) return fail(LFMM_E_INVAL, "bad argument");
    // boxes <= 4/3 * n / (leaf occupancy >= 1) bounded by 2 n; per box: Q, U, keys and lists
    const size_t nb = size_t(2 * n + 64);
    size_t per_box = size_t(kRankPad) * 16 + 8 + 4 * 7 + 4 * kNumInteractions + 4 * 4 + 4 * 9;
    size_t per_point = 8 + 4 + 8;
    size_t tmp = size_t(n) * (16 + 8 + 1 + 8) + radix_scratch_bytes(n) + scan_scratch_bytes(n, 1);
    *out = nb * per_box + size_t(n) * per_point + tmp + (1u << 20);
    return LFMM_OK;
}

lfmm_status lfmm_plan_destroy(lfmm_plan* pl) {
    if (!pl) return LFMM_OK;
    (void)hipSetDevice(pl->ctx->device);
    // kernels of this plan may still run on any stream: finish them before the blocks go
    // back to the context's pool for reuse
    (void)hipDeviceSynchronize();
    delete pl;
    return LFMM_OK;
}

lfmm_status lfmm_solve(lfmm_ctx* ctx, int64_t n, const int32_t* xy, const double* f, double* u, void* stream) {
    lfmm_plan* pl = nullptr;
    lfmm_status s = lfmm_plan_create(ctx, n, xy, stream, &pl);
    if (s != LFMM_OK) return s;
    s = lfmm_execute(pl, f, u, stream);
    if (s == LFMM_OK) {
        hipError_t e = hipStreamSynchronize(as_stream(stream));
        if (e != hipSuccess) s = fail(LFMM_E_HIP, hipGetErrorString(e));
    }
    lfmm_plan_destroy(pl);
    return s;
}

lfmm_status lfmm_direct(lfmm_ctx* ctx, int64_t nt, const int32_t* txy, int64_t ns, const int32_t* sxy,
                        const double* f, double* u, void* stream) {
    if (!ctx || nt < 0 || ns < 0 || (nt > 0 && (!txy || !u)) || (ns > 0 && (!sxy || !f)))
        return fail(LFMM_E_INVAL, "bad argument");
    return guarded([&]() -> lfmm_status {
        LFMM_HIP(hipSetDevice(ctx->device));
        launch_direct(nt, txy, ns, sxy, f, ctx->phi_oct, u, as_stream(stream));
        LFMM_HIP(hipGetLastError());
        return LFMM_OK;
    });
}

}  // extern "C"
