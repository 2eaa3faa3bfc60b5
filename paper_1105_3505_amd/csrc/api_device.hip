// Device part of the C ABI: contexts (phi table and cached operators on the GPU), plans
// (the quadtrees of one or more point sets, built on the GPU) and evaluation (Section 8.2).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <exception>
#include <limits>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <set>
#include <string>
#include <vector>

#include "api_common.h"
#include "host_math.h"
#include "kernels.h"
#include "lfmm.h"

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

struct Unsupported {
    std::string msg;
};

// Bump allocation from a fixed device region (the static workspace of the allocation-free
// solve): nothing is freed, the whole region is reused by the next call.
struct StaticRegion {
    char* base = nullptr;
    size_t cap = 0, used = 0;
    void* take(size_t bytes) {
        bytes = (bytes + 255) & ~size_t(255);
        if (used + bytes > cap)
            throw std::out_of_range("the point set needs more than the " + std::to_string(cap >> 20) +
                                    " MiB static workspace");
        void* p = base + used;
        used += bytes;
        return p;
    }
};

// An event recorded after the last work that uses some blocks; blocks released "after" it
// become reusable once the device has passed it.
struct Fence {
    hipEvent_t ev = nullptr;
    Fence(hipStream_t st) {
        LFMM_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        LFMM_HIP(hipEventRecord(ev, st));
    }
    Fence(const Fence&) = delete;
    Fence& operator=(const Fence&) = delete;
    bool passed() const { return hipEventQuery(ev) == hipSuccess; }
    ~Fence() {
        if (ev) (void)hipEventDestroy(ev);
    }
};
using FencePtr = std::shared_ptr<Fence>;

// Blocks released after a fence, handed back to their free list once it has passed.
struct Deferred {
    struct Item {
        size_t cls;
        void* p;
        FencePtr fence;
    };
    std::vector<Item> items;
    template <class F>
    void reap(F&& give_back, bool wait) {
        size_t k = 0;
        for (Item& it : items) {
            if (wait) (void)hipEventSynchronize(it.fence->ev);
            if (wait || it.fence->passed()) give_back(it.cls, it.p);
            else items[k++] = std::move(it);
        }
        items.resize(k);
    }
};

// Device blocks cached by power-of-two size class, so that building and dropping plans
// does not call hipMalloc/hipFree (each costs far more than a small solve).  A block is
// returned only after the work that used it is ordered before any later user: a release
// follows a synchronisation, or names the fence after which the block is free.
// Failure injection for tests of the out-of-memory paths: while LFMM_TEST_FAIL_ALLOC=k is set in
// the environment, the k-th device block requested after it was set (or changed) fails as if
// hipMalloc had, and the requests after it proceed.  Unset, one environment read per request.
bool injected_alloc_failure() {
    static std::mutex mu;
    static std::string last;
    static long count = 0;
    const char* e = std::getenv("LFMM_TEST_FAIL_ALLOC");
    const std::string v = e ? e : "";
    std::lock_guard<std::mutex> lock(mu);
    if (v != last) {
        last = v;
        count = 0;
    }
    if (v.empty()) return false;
    const long k = std::atol(v.c_str());
    return k > 0 && ++count == k;
}

class DevicePool {
  public:
    static size_t size_class(size_t bytes) {
        size_t c = size_t(1) << 16;
        while (c < bytes) c <<= 1;
        return c;
    }
    void* acquire(size_t bytes, size_t* got) {
        size_t cls = size_class(bytes);
        if (injected_alloc_failure()) throw NoMemory{"injected device allocation failure (LFMM_TEST_FAIL_ALLOC)"};
        {
            std::lock_guard<std::mutex> lock(mu_);
            if (!pending_.items.empty()) pending_.reap([&](size_t c, void* q) { give_back(c, q); }, false);
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
        give_back(cls, p);
    }
    void release_after(void* p, size_t cls, const FencePtr& fence) {
        std::lock_guard<std::mutex> lock(mu_);
        pending_.items.push_back(Deferred::Item{cls, p, fence});
    }
    void trim() {
        std::lock_guard<std::mutex> lock(mu_);
        pending_.reap([&](size_t c, void* q) { give_back(c, q); }, true);
        for (auto& kv : free_) (void)hipFree(kv.second);
        free_.clear();
        cached_ = 0;
    }
    size_t cached_bytes() const { return cached_; }
    ~DevicePool() { trim(); }

  private:
    void give_back(size_t cls, void* p) {
        free_.emplace(cls, p);
        cached_ += cls;
    }
    std::multimap<size_t, void*> free_;
    Deferred pending_;
    size_t cached_ = 0;
    std::mutex mu_;
};

// One device allocation carved into aligned pieces (from a pool when one is given).
class Arena {
  public:
    explicit Arena(DevicePool* pool = nullptr, StaticRegion* region = nullptr) : pool_(pool), region_(region) {}
    void reserve(size_t bytes) { total_ += align(bytes); }
    void allocate() {
        if (total_ == 0) return;
        if (region_) {
            base_ = region_->take(total_);
            cap_ = total_;
            return;
        }
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
        if (base_ && !region_) {
            if (pool_) pool_->release(base_, cap_);
            else (void)hipFree(base_);
        }
        base_ = nullptr;
        total_ = used_ = cap_ = 0;
    }
    // back to the pool once the device has passed `fence` (pool arenas only)
    void release_after(const FencePtr& fence) {
        if (base_ && pool_ && !region_) {
            pool_->release_after(base_, cap_, fence);
            base_ = nullptr;
            total_ = used_ = cap_ = 0;
        }
        release();
    }
    size_t bytes() const { return cap_; }
    void set_pool(DevicePool* p, StaticRegion* region = nullptr) {
        pool_ = p;
        region_ = region;
    }
    ~Arena() { release(); }

  private:
    static size_t align(size_t b) { return (b + 255) & ~size_t(255); }
    DevicePool* pool_ = nullptr;
    StaticRegion* region_ = nullptr;
    void* base_ = nullptr;
    size_t total_ = 0, used_ = 0, cap_ = 0;
};

struct CachedOps {
    OperatorSet host;
    DevOps dev;
    Arena mem;
};

}  // namespace
// Pinned host blocks for the per-execute pointer tables of batched plans, cached by size
// class: allocating or freeing pinned memory may synchronise the device.
class PinnedPool {
  public:
    void* acquire(size_t bytes, size_t* got) {
        size_t cls = 4096;
        while (cls < bytes) cls <<= 1;
        *got = cls;
        {
            std::lock_guard<std::mutex> lock(mu_);
            if (!pending_.items.empty())
                pending_.reap([&](size_t c, void* q) { free_.emplace(c, q); }, false);
            auto it = free_.find(cls);
            if (it != free_.end()) {
                void* p = it->second;
                free_.erase(it);
                return p;
            }
        }
        void* p = nullptr;
        LFMM_HIP(hipHostMalloc(&p, cls));
        // kernels read these blocks through the host pointer (the upload copies)
        void* dp = nullptr;
        if (hipHostGetDevicePointer(&dp, p, 0) != hipSuccess || dp != p) {
            (void)hipHostFree(p);
            throw std::runtime_error("pinned host memory is not addressable from the device at its host address");
        }
        return p;
    }
    void release(void* p, size_t cls) {
        std::lock_guard<std::mutex> lock(mu_);
        free_.emplace(cls, p);
    }
    void release_after(void* p, size_t cls, const FencePtr& fence) {
        std::lock_guard<std::mutex> lock(mu_);
        pending_.items.push_back(Deferred::Item{cls, p, fence});
    }
    ~PinnedPool() {
        pending_.reap([&](size_t c, void* q) { free_.emplace(c, q); }, true);
        for (auto& kv : free_) (void)hipHostFree(kv.second);
    }

  private:
    std::multimap<size_t, void*> free_;
    Deferred pending_;
    std::mutex mu_;
};

// Workspace of lfmm_solve_static: one file-scope device array per GPU, held until the process
// ends.  Host code never passes the array's name to a kernel (on the host it is a stand-in, not
// a device address): each context looks up the address on its device at creation.
namespace {
constexpr size_t kStaticScratchBytes = size_t(64) << 20;
constexpr int64_t kStaticMaxPoints = int64_t(1) << 16;
std::mutex g_static_mu[64];   // calls on one device take turns (they share its array)
}  // namespace
static __device__ __align__(256) char scratch[kStaticScratchBytes];

struct lfmm_ctx {
    int device = 0;
    void* static_scratch = nullptr;   // device address of `scratch` on this context's device
    lfmm_options opt{};
    PinnedPool pinned;
    DevicePool pool;             // plan storage and temporaries (declared first: freed last)
    Arena table_mem;
    double* phi_oct = nullptr;   // octant table, radius kPhiDeviceRadius
    PhiFar* phi_far = nullptr;   // far-field expansion coefficients of the context's operator
    std::map<int64_t, CachedOps*> ops;                // deepest operator set per leaf side
    std::vector<std::unique_ptr<CachedOps>> all_ops;  // every set built; plans may hold any
    std::map<std::pair<int, int>, int32_t> tuned;     // (size class, density class) -> N_leaf
    hipStream_t capture = nullptr;                    // stream that graph captures record on
    std::mutex mu;
    // live plans and servers, destroyed with the context if the caller has not done so
    std::set<lfmm_plan*> plans;
    std::set<lfmm_server*> servers;
    std::mutex reg_mu;
    ~lfmm_ctx() {
        if (capture) (void)hipStreamDestroy(capture);
    }
};

namespace {

// size and density classes of a point set for the tuning table: rounded log2 of n and of
// n / (root box area)
std::pair<int, int> tune_key(int64_t n, int D) {
    const double ln = std::log2(double(std::max<int64_t>(n, 1)));
    return {int(std::lround(ln)), int(std::lround(ln - 2.0 * D))};
}

constexpr int32_t kDefaultMaxLeaf = 64;

}  // namespace

struct TileRange {
    int32_t t0 = 0, n = 0;
};

struct lfmm_plan {
    lfmm_ctx* ctx = nullptr;
    int32_t K = 0;                          // instances
    int64_t n = 0;                          // points of all instances
    std::vector<int32_t> pt_off;            // K + 1
    std::vector<int32_t> nsrc, tgt0, nout;  // per instance: sources, first target, targets
    std::vector<InstInfo> inst;             // host copy of the instance table
    std::vector<CachedOps*> ops;            // operator sets used, by index
    int Dmax = 0, Lmax = 0, Hmax = 0;
    int32_t nbox = 0, nleaf = 0;
    std::vector<int32_t> hbase;             // first box of each height, Hmax + 2 entries
    std::vector<TileRange> leaf_of_ops;     // leaves of each operator set
    std::vector<TileRange> near_of_ops;     // near-field groups of each operator set
    int32_t nq = 0;
    TileRange m2l;                          // M2L tiles (class-sorted, some empty)
    std::vector<TileRange> m2m, l2l;        // tiles per height
    int64_t m2l_pairs = 0;
    Arena mem_small, mem_pts, mem_box, mem_ad;
    InstInfo* d_inst = nullptr;
    OpsPtrs* d_ops = nullptr;
    uint8_t* d_far = nullptr;
    ExecPtrs* d_exec = nullptr;
    BoxTile* m2m_tiles = nullptr;           // M2M tiles (pl->m2m ranges index them)
    int32_t* d_m2l_ntiles = nullptr;
    int32_t *pts = nullptr, *perm = nullptr, *pinst = nullptr;
    uint32_t* pkey = nullptr;
    double* fs = nullptr;
    uint64_t* box_key = nullptr;
    int32_t *box_pt0 = nullptr, *box_pt1 = nullptr, *box_parent = nullptr, *box_child = nullptr,
            *box_inst = nullptr, *nb9 = nullptr, *il27 = nullptr, *cls_box = nullptr;
    int8_t* box_lev = nullptr;
    BoxTile* tiles = nullptr;
    NearGroup* groups = nullptr;
    int4* ents = nullptr;
    double *Q = nullptr, *U = nullptr;
    float *Qh = nullptr, *Ql = nullptr;     // mixed precision: FP32 parts of Q (with its zero row)
    double* qsum = nullptr;                 // and the charge sum of each row
    uint16_t* Qb = nullptr;                 // bf16 mixed precision: the three bf16 parts of Q
    // adaptive tree (LFMM_FLAG_ADAPTIVE)
    bool adaptive = false;
    int8_t* role = nullptr;                 // BoxRole of every box
    int32_t* list_off = nullptr;            // [3][nbox + 1] row starts of the U, W, X lists
    int32_t* list_ent[3] = {};              // their entries
    int64_t list_len[3] = {};
    int32_t* ad_leaves = nullptr;           // adaptive leaves (near-field items)
    int32_t* ad_xboxes = nullptr;           // boxes with a non-empty X list (P2L items)
    int32_t n_ad_leaves = 0, n_ad_xboxes = 0;
    int32_t* pt_box = nullptr;              // finest box of every point
    BoxTile* m2l_tiles = nullptr;           // the non-empty M2L tiles, compacted
    // pinned staging of the per-execute pointer table: kExecRing slots of K entries, each
    // rewritten only after the upload that read it (its event); the host copy of the table
    // last uploaded to d_exec lets an execute with the same pointers skip the upload
    static constexpr int kExecRing = 4;
    ExecPtrs* h_exec = nullptr;
    size_t h_exec_cls = 0;
    hipEvent_t exec_copied[kExecRing] = {};
    int exec_slot = 0;
    std::vector<ExecPtrs> exec_last;
    bool failed = false;
    uint32_t timing_mask = 0;   // phases whose bounding events later executes record
    uint32_t timed_mask = 0;    // phases timed by the most recent timed execute
    bool use_graph = false;                 // execute replays a captured HIP graph
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    hipEvent_t ev[LFMM_NUM_PHASES + 1] = {};
    FencePtr built;                         // end of the build, on build_stream
    StaticRegion* sreg = nullptr;           // allocation-free solve: every device block from here
    hipStream_t build_stream = nullptr;
    bool one_stream = true;                 // every execute so far ran on build_stream
    ~lfmm_plan() {
        {
            std::lock_guard<std::mutex> lock(ctx->reg_mu);
            ctx->plans.erase(this);
        }
        if (gexec) (void)hipGraphExecDestroy(gexec);
        if (graph) (void)hipGraphDestroy(graph);
        for (auto& e : ev)
            if (e) (void)hipEventDestroy(e);
        for (hipEvent_t e : exec_copied)
            if (e) (void)hipEventDestroy(e);
        if (h_exec) ctx->pinned.release(h_exec, h_exec_cls);
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

// Uploads (or extends) the operators for leaves of `side` with at least `nlev` heights.  With
// lookup_only (allocation-free solves) a missing set is an Unsupported request instead.
CachedOps* get_ops(lfmm_ctx* ctx, int64_t side, int nlev, hipStream_t st, bool lookup_only = false) {
    std::lock_guard<std::mutex> lock(ctx->mu);
    auto it = ctx->ops.find(side);
    if (it != ctx->ops.end() && it->second->host.nlevels >= nlev) return it->second;
    if (lookup_only)
        throw Unsupported{"the context holds no operators for leaf side " + std::to_string(side) + " with " +
                          std::to_string(nlev) + " heights (a plan of such a point set builds them)"};
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
    std::vector<double> leafTt(side <= 32 ? leafT.size() : 0);
    for (int64_t c = 0; c < s2 && !leafTt.empty(); ++c)
        for (int p = 0; p < P; ++p) leafTt[(size_t(p / 2) * size_t(s2) + size_t(c)) * 2 + (p & 1)] = leafT[size_t(c) * P + p];
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
                        T[size_t(p) * P + q] = phi(ctx->opt.stencil, lv.skel[2 * p] - lv.skel[2 * q] - dx * lv.side,
                                                   lv.skel[2 * p + 1] - lv.skel[2 * q + 1] - dy * lv.side);
            }
    }
    co->mem.reserve(leafT.size() * sizeof(double));
    if (!leafTt.empty()) co->mem.reserve(leafTt.size() * sizeof(double));
    co->mem.reserve(ofo_cm.size() * sizeof(double));
    co->mem.reserve(ofo_rm.size() * sizeof(double));
    co->mem.reserve(ifo.size() * sizeof(double));
    // mixed precision: T^d = c_d 1 1^T + R^d (c_d = mean entry over the true rank), R^d split
    // into FP32 hi + lo; padded rows and columns stay zero
    std::vector<float> ifo_hi(ifo.size(), 0.f), ifo_lo(ifo.size(), 0.f);
    std::vector<double> mono(size_t(nlev) * kNumIfoSlots, 0.0);
    std::vector<int32_t> ranks(static_cast<size_t>(nlev), 0);
    std::vector<int32_t> skel(size_t(nlev) * P * 2, 0);   // skeleton points of each height
    for (int h = 0; h < nlev; ++h) {
        const LevelOps& lv = H.level[size_t(h)];
        for (int p = 0; p < lv.rank; ++p) {
            skel[(size_t(h) * P + p) * 2] = int32_t(lv.skel[2 * p]);
            skel[(size_t(h) * P + p) * 2 + 1] = int32_t(lv.skel[2 * p + 1]);
        }
    }
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
    // bf16 mixed precision: R^d = T^d - c_d 1 1^T (the FP64 remainder, not the FP32 parts)
    // split into three bf16 parts R_p, each the round-to-nearest of what the earlier parts
    // leave, laid out in the kernel's fragment order (group of 8 bf16 per lane and part)
    std::vector<uint16_t> ifo_b(size_t(nlev) * kNumIfoSlots * kBf16OpVecs * 8, 0);
    for (int h = 0; h < nlev; ++h) {
        const int r = H.level[size_t(h)].rank;
        for (int slot = 0; slot < kNumIfoSlots; ++slot) {
            const size_t base = (size_t(h) * kNumIfoSlots + slot) * P * P;
            const double mean = mono[size_t(h) * kNumIfoSlots + slot];
            uint16_t* ob = ifo_b.data() + (size_t(h) * kNumIfoSlots + slot) * kBf16OpVecs * 8;
            for (int row = 0; row < r; ++row)
                for (int col = 0; col < r; ++col) {
                    double rem = ifo[base + size_t(row) * P + col] - mean;
                    const int m = row / 16, n = row % 16, sg = col / 8, e = col % 8;
                    for (int part = 0; part < 3; ++part) {
                        const uint16_t b = bf16_rne(rem);
                        ob[(size_t((part * 3 + m) * 6 + sg) * 16 + n) * 8 + e] = b;
                        rem -= bf16_value(b);   // exact: b is within 2^-8 of rem
                    }
                }
        }
    }
    // fragment order for the M2L kernels: lane l's operands of one matrix instruction sit
    // next to lane l+1's, so a wave reads 1 KB contiguous per load (P = 48: 3 row blocks,
    // lane group g = l / 16 covers columns 12 g .. 12 g + 11)
    {
        // FP64 order: element ((m * 6 + j) * 64 + l) * 2 + e is row 16 m + l % 16, column
        // 12 (l / 16) + 2 j + e; FP32 order: ((m * 3 + j) * 64 + l) * 4 + e, column 12 (l / 16) + 4 j + e
        auto frag64 = [&](std::vector<double>& a) {
            std::vector<double> out(a.size());
            for (size_t base = 0; base < a.size(); base += size_t(P) * P)
                for (int m = 0; m < P / 16; ++m)
                    for (int l = 0; l < 64; ++l) {
                        const int row = 16 * m + (l & 15), c0 = (l >> 4) * (P / 4);
                        for (int k = 0; k < P / 4; ++k)
                            out[base + ((size_t(m) * (P / 8) + k / 2) * 64 + l) * 2 + (k & 1)] =
                                a[base + size_t(row) * P + c0 + k];
                    }
            a.swap(out);
        };
        auto frag32 = [&](std::vector<float>& a) {
            std::vector<float> out(a.size());
            for (size_t base = 0; base < a.size(); base += size_t(P) * P)
                for (int m = 0; m < P / 16; ++m)
                    for (int l = 0; l < 64; ++l) {
                        const int row = 16 * m + (l & 15), c0 = (l >> 4) * (P / 4);
                        for (int k = 0; k < P / 4; ++k)
                            out[base + ((size_t(m) * (P / 16) + k / 4) * 64 + l) * 4 + (k & 3)] =
                                a[base + size_t(row) * P + c0 + k];
                    }
            a.swap(out);
        };
        frag64(ifo);
        frag64(ofo_rm);
        frag64(ofo_cm);
        frag32(ifo_hi);
        frag32(ifo_lo);
    }
    co->mem.reserve(ifo.size() * sizeof(float));
    co->mem.reserve(ifo.size() * sizeof(float));
    co->mem.reserve(ifo_b.size() * sizeof(uint16_t));
    co->mem.reserve(mono.size() * sizeof(double));
    co->mem.reserve(ranks.size() * sizeof(int32_t));
    co->mem.reserve(skel.size() * sizeof(int32_t));
    co->mem.allocate();
    co->dev.leaf_side = side;
    co->dev.nlev = nlev;
    co->dev.leafT = co->mem.take<double>(leafT.size());
    co->dev.leafTt = leafTt.empty() ? nullptr : co->mem.take<double>(leafTt.size());
    co->dev.ofo_cm = co->mem.take<double>(ofo_cm.size());
    co->dev.ofo_rm = co->mem.take<double>(ofo_rm.size());
    co->dev.ifo = co->mem.take<double>(ifo.size());
    co->dev.ifo_hi = co->mem.take<float>(ifo.size());
    co->dev.ifo_lo = co->mem.take<float>(ifo.size());
    co->dev.ifo_b = co->mem.take<uint16_t>(ifo_b.size());
    co->dev.mono = co->mem.take<double>(mono.size());
    co->dev.rank = co->mem.take<int32_t>(ranks.size());
    co->dev.skel = co->mem.take<int32_t>(skel.size());
    LFMM_HIP(hipMemcpyAsync(co->dev.leafT, leafT.data(), leafT.size() * 8, hipMemcpyHostToDevice, st));
    if (co->dev.leafTt)
        LFMM_HIP(hipMemcpyAsync(co->dev.leafTt, leafTt.data(), leafTt.size() * 8, hipMemcpyHostToDevice, st));
    LFMM_HIP(hipMemcpyAsync(co->dev.ofo_cm, ofo_cm.data(), ofo_cm.size() * 8, hipMemcpyHostToDevice, st));
    LFMM_HIP(hipMemcpyAsync(co->dev.ofo_rm, ofo_rm.data(), ofo_rm.size() * 8, hipMemcpyHostToDevice, st));
    LFMM_HIP(hipMemcpyAsync(co->dev.ifo, ifo.data(), ifo.size() * 8, hipMemcpyHostToDevice, st));
    LFMM_HIP(hipMemcpyAsync(co->dev.ifo_hi, ifo_hi.data(), ifo.size() * 4, hipMemcpyHostToDevice, st));
    LFMM_HIP(hipMemcpyAsync(co->dev.ifo_lo, ifo_lo.data(), ifo.size() * 4, hipMemcpyHostToDevice, st));
    LFMM_HIP(hipMemcpyAsync(co->dev.ifo_b, ifo_b.data(), ifo_b.size() * 2, hipMemcpyHostToDevice, st));
    LFMM_HIP(hipMemcpyAsync(co->dev.mono, mono.data(), mono.size() * 8, hipMemcpyHostToDevice, st));
    LFMM_HIP(hipMemcpyAsync(co->dev.rank, ranks.data(), ranks.size() * 4, hipMemcpyHostToDevice, st));
    LFMM_HIP(hipMemcpyAsync(co->dev.skel, skel.data(), skel.size() * 4, hipMemcpyHostToDevice, st));
    LFMM_HIP(hipStreamSynchronize(st));
    CachedOps* raw = co.get();
    ctx->ops[side] = raw;             // a shallower set stays alive for the plans using it
    ctx->all_ops.push_back(std::move(co));
    return raw;
}

OpsPtrs ops_ptrs(const CachedOps* co) {
    OpsPtrs p{};
    p.leafT = co->dev.leafT;
    p.ofo_rm = co->dev.ofo_rm;
    p.ofo_cm = co->dev.ofo_cm;
    p.ifo = co->dev.ifo;
    p.ifo_hi = co->dev.ifo_hi;
    p.ifo_lo = co->dev.ifo_lo;
    p.ifo_b = co->dev.ifo_b;
    p.mono = co->dev.mono;
    p.rank = co->dev.rank;
    p.skel = co->dev.skel;
    p.side = co->dev.leaf_side;
    p.nlev = co->dev.nlev;
    return p;
}

// Host-to-device copies of small tables, gathered so that tables that lie next to each other
// in device memory (less than one 256-byte alignment step apart, so that nothing else lies
// between them) go in one copy from pinned memory.  The copies are kernels that read the
// pinned block directly: a copy-engine transfer costs tens of microseconds of hand-over
// between the copy and compute queues on the stream.  The pinned blocks are held until the
// Stager is destroyed, which must come after the stream has passed the copies.
class Stager {
  public:
    // direct: plain copies from pageable host memory (no pinned blocks), kept alive until the
    // Stager is destroyed, which must come after the stream has passed them
    explicit Stager(lfmm_ctx* ctx, bool direct = false) : ctx_(ctx), direct_(direct) {}
    Stager(const Stager&) = delete;
    Stager& operator=(const Stager&) = delete;
    template <class T>
    void add(T* dst, const std::vector<T>& v) {
        if (v.empty()) return;
        const char* b = reinterpret_cast<const char*>(v.data());
        pieces_.push_back(Piece{reinterpret_cast<char*>(dst), std::vector<char>(b, b + v.size() * sizeof(T))});
    }
    void flush(hipStream_t st) {
        std::sort(pieces_.begin(), pieces_.end(), [](const Piece& a, const Piece& b) { return a.dst < b.dst; });
        size_t i = 0;
        while (i < pieces_.size()) {
            size_t j = i + 1;
            char* end = pieces_[i].dst + pieces_[i].data.size();
            while (j < pieces_.size() && pieces_[j].dst >= end && pieces_[j].dst - end < 256) {
                end = pieces_[j].dst + pieces_[j].data.size();
                ++j;
            }
            const size_t len = size_t(end - pieces_[i].dst);
            if (direct_) {
                kept_.emplace_back(len);
                for (size_t k = i; k < j; ++k)
                    std::memcpy(kept_.back().data() + (pieces_[k].dst - pieces_[i].dst), pieces_[k].data.data(),
                                pieces_[k].data.size());
                LFMM_HIP(hipMemcpyAsync(pieces_[i].dst, kept_.back().data(), len, hipMemcpyHostToDevice, st));
                i = j;
                continue;
            }
            size_t cls = 0;
            char* h = static_cast<char*>(ctx_->pinned.acquire(len, &cls));
            held_.push_back({h, cls});
            for (size_t k = i; k < j; ++k)
                std::memcpy(h + (pieces_[k].dst - pieces_[i].dst), pieces_[k].data.data(), pieces_[k].data.size());
            launch_upload(pieces_[i].dst, h, len, st);
            i = j;
        }
        pieces_.clear();
    }
    // the pinned blocks go back once the device has passed `fence` (after the copies)
    void retire(const FencePtr& fence) {
        for (auto& b : held_) ctx_->pinned.release_after(b.first, b.second, fence);
        held_.clear();
    }
    ~Stager() {
        for (auto& b : held_) ctx_->pinned.release(b.first, b.second);
    }

  private:
    struct Piece {
        char* dst;
        std::vector<char> data;
    };
    lfmm_ctx* ctx_;
    bool direct_ = false;
    std::vector<Piece> pieces_;
    std::vector<std::pair<void*, size_t>> held_;
    std::vector<std::vector<char>> kept_;
};

// On the way out of a failed build: finish the device work before the blocks it uses go
// back to their pools.
struct SyncOnUnwind {
    int pending = std::uncaught_exceptions();
    ~SyncOnUnwind() {
        if (std::uncaught_exceptions() > pending) (void)hipDeviceSynchronize();
    }
};

}  // namespace

// One point set of a forest: its sources and, when tgt is not null, targets of its own.
struct InstanceInput {
    int64_t n_src = 0;
    const int32_t* src = nullptr;
    int64_t n_tgt = 0;
    const int32_t* tgt = nullptr;   // null: the targets are the sources
};

namespace {

// Builds the forest of K point sets: Section 6 tree of every instance, lists of Definition 6.1,
// operator sets for every leaf side used, and the tiles of the matrix passes.  An instance with
// targets of its own gets one tree over the union of its sources and targets (its points are
// the sources, then the targets): a target-only point carries a zero load, so the far and
// near fields of the union are those of the sources, and the incoming expansion of any box
// holding targets is evaluated at them by T_tfi = T_ofs^T of the dense model box, which
// covers every cell of the box (Section 4.3, incoming skeleton; Remark 8.2).
void acquire_exec_staging(lfmm_plan* pl) {
    pl->h_exec = static_cast<ExecPtrs*>(pl->ctx->pinned.acquire(
        size_t(lfmm_plan::kExecRing) * size_t(pl->K) * sizeof(ExecPtrs), &pl->h_exec_cls));
    for (hipEvent_t& e : pl->exec_copied) LFMM_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
}

void build_forest(lfmm_plan* pl, int32_t K, const InstanceInput* in, int32_t max_leaf, hipStream_t st) {
    lfmm_ctx* ctx = pl->ctx;
    pl->K = K;
    pl->pt_off.assign(size_t(K) + 1, 0);
    pl->nsrc.assign(size_t(K), 0);
    pl->tgt0.assign(size_t(K), 0);
    pl->nout.assign(size_t(K), 0);
    // coordinate segments in point order: the sources of an instance, then its own targets
    std::vector<const int32_t*> seg_ptr;
    std::vector<int32_t> seg_off{0};
    for (int32_t k = 0; k < K; ++k) {
        const InstanceInput& I = in[k];
        const int64_t nk = I.n_src + (I.tgt ? I.n_tgt : 0);
        pl->pt_off[size_t(k) + 1] = pl->pt_off[size_t(k)] + int32_t(nk);
        pl->nsrc[size_t(k)] = int32_t(I.n_src);
        pl->tgt0[size_t(k)] = I.tgt ? int32_t(I.n_src) : 0;
        pl->nout[size_t(k)] = I.tgt ? int32_t(I.n_tgt) : int32_t(I.n_src);
        if (I.n_src > 0) {
            seg_ptr.push_back(I.src);
            seg_off.push_back(seg_off.back() + int32_t(I.n_src));
        }
        if (I.tgt && I.n_tgt > 0) {
            seg_ptr.push_back(I.tgt);
            seg_off.push_back(seg_off.back() + int32_t(I.n_tgt));
        }
    }
    const int32_t nseg = int32_t(seg_ptr.size());
    const int64_t n = pl->pt_off[size_t(K)];
    pl->n = n;

    // chunks of <= kChunk points, each inside one instance
    std::vector<Chunk> chunks;
    std::vector<int32_t> chunk_first(static_cast<size_t>(K) + 1, 0);
    for (int32_t k = 0; k < K; ++k) {
        chunk_first[size_t(k)] = int32_t(chunks.size());
        for (int32_t b = pl->pt_off[size_t(k)]; b < pl->pt_off[size_t(k) + 1]; b += kChunk)
            chunks.push_back(Chunk{k, b, std::min(b + kChunk, pl->pt_off[size_t(k) + 1]), 0});
    }
    chunk_first[size_t(K)] = int32_t(chunks.size());
    const int32_t nch = int32_t(chunks.size());

    // ---- temporaries sized by n (one reserve per take) ------------------------------------
    StaticRegion* const sreg = pl->sreg;
    Arena tmp(&ctx->pool, sreg);
    tmp.reserve(size_t(nseg) * sizeof(void*));  // coordinate segments
    tmp.reserve(size_t(nseg + 1) * 4);          // segment offsets
    tmp.reserve(size_t(K + 1) * 4);             // pt_off
    tmp.reserve(size_t(nch) * sizeof(Chunk));
    tmp.reserve(size_t(K + 1) * 4);             // chunk_first
    tmp.reserve(size_t(nch) * 16);              // bbox partials
    tmp.reserve(size_t(K) * sizeof(InstInfo));  // instances up to the level statistics
    // copies of the level statistics: enough that no copy takes the atomics of more than about
    // 32 chunks of one instance
    int32_t max_chunks = 0;
    for (int32_t k = 0; k < K; ++k)
        max_chunks = std::max(max_chunks, chunk_first[size_t(k) + 1] - chunk_first[size_t(k)]);
    const int32_t stat_copies = std::min(kLevelStatsCopies, std::max(1, max_chunks / 32));
    tmp.reserve(size_t(stat_copies) * K * (kMaxLevels + 3) * 4 + 4);   // level histograms, look-ahead maxima, counter
    tmp.reserve(4);                             // deepest root box
    tmp.reserve(nseg > 1 ? size_t(n) * 8 : 0);  // concatenated points
    tmp.reserve(size_t(n) * 8);                 // keys
    tmp.reserve(size_t(n) * 8);                 // keys_tmp
    tmp.reserve(size_t(n) * 4);                 // vals
    tmp.reserve(size_t(n) * 4);                 // vals_tmp
    tmp.reserve(size_t(n));                     // cl
    tmp.reserve(radix_scratch_bytes(n));
    tmp.reserve(scan_scratch_bytes(n, 1));
    tmp.allocate();
    SyncOnUnwind unwind_tmp;
    const int32_t** d_xytab = tmp.take<const int32_t*>(nseg);
    int32_t* d_segoff = tmp.take<int32_t>(nseg + 1);
    int32_t* d_ptoff = tmp.take<int32_t>(K + 1);
    Chunk* d_chunks = tmp.take<Chunk>(nch);
    int32_t* d_chfirst = tmp.take<int32_t>(K + 1);
    int32_t* d_part = tmp.take<int32_t>(size_t(nch) * 4);
    InstInfo* d_inst0 = tmp.take<InstInfo>(K);
    const int32_t nstats = stat_copies * K * (kMaxLevels + 3);
    int32_t* d_stats = tmp.take<int32_t>(size_t(nstats) + 1);   // zeroed by the key kernel
    int32_t* d_dmax = tmp.take<int32_t>(1);
    // results of the two read-backs: pinned host memory that the kernels write (the root boxes
    // by the kernel itself, the level statistics by one copy); in the static workspace, device
    // memory copied back into rb_host
    const size_t rb_words = size_t(K) * (kMaxLevels + 7);
    size_t rb_cls = 0;
    int32_t* rb = sreg ? static_cast<int32_t*>(sreg->take(rb_words * 4))
                       : static_cast<int32_t*>(ctx->pinned.acquire(rb_words * 4, &rb_cls));
    struct Release {
        lfmm_ctx* c;
        void* p;
        size_t cls;
        ~Release() {
            if (p) c->pinned.release(p, cls);
        }
    } rb_guard{ctx, sreg ? nullptr : rb, rb_cls};
    std::vector<int32_t> rb_host(sreg ? rb_words : 0);
    int32_t* bb = rb;                      // [K][4] root boxes
    int32_t* stats = rb + size_t(K) * 4;   // [K][34] histograms, then [K] maxima
    int32_t* d_xyc = (nseg > 1) ? tmp.take<int32_t>(size_t(n) * 2) : nullptr;
    uint64_t* keys = tmp.take<uint64_t>(n);
    uint64_t* keys_tmp = tmp.take<uint64_t>(n);
    uint32_t* vals = tmp.take<uint32_t>(n);
    uint32_t* vals_tmp = tmp.take<uint32_t>(n);
    int8_t* cl = tmp.take<int8_t>(n);
    void* rscr = tmp.take<char>(radix_scratch_bytes(n));
    void* sscr = tmp.take<char>(scan_scratch_bytes(n, 1));

    Stager stage_a(ctx, sreg != nullptr);
    stage_a.add(d_xytab, seg_ptr);
    stage_a.add(d_segoff, seg_off);
    stage_a.add(d_ptoff, pl->pt_off);
    stage_a.add(d_chunks, chunks);
    stage_a.add(d_chfirst, chunk_first);
    stage_a.flush(st);
    const int32_t* xy = seg_ptr[0];
    if (nseg > 1) {
        launch_concat(nseg, d_xytab, d_segoff, n, d_xyc, st);
        xy = d_xyc;
    }

    // N_leaf of every instance: the caller's, else the options', else the tuned value for
    // the instance's size and density (known after the root boxes), else the default
    int32_t ml_all = max_leaf > 0 ? max_leaf : ctx->opt.max_leaf;
    if (ml_all <= 0) {
        std::lock_guard<std::mutex> lock(ctx->mu);
        if (ctx->tuned.empty()) ml_all = kDefaultMaxLeaf;
    }

    // ---- root boxes ----------------------------------------------------------------------
    launch_bbox_chunks(xy, d_chunks, nch, d_part, d_dmax, st);
    // root boxes straight to pinned host memory, and the instance table of the next kernels
    // (N_leaf too when there is one for all) straight to the device
    launch_bbox_final(d_part, d_chfirst, d_ptoff, K, std::max(ml_all, 0), bb, d_inst0, d_dmax, st);
    std::unique_ptr<Fence> bb_ready;
    if (!sreg) bb_ready = std::make_unique<Fence>(st);
    // Morton keys and, for large inputs, the first two passes of their sort go out before the
    // host reads the root boxes: the keys need only the device's instance table, and distinct
    // points need at least 16 key bits once there are 2^16 of them (a pass over digits that
    // are zero everywhere would change nothing either).
    launch_keys(xy, d_ptoff, K, d_inst0, d_dmax, n, keys, vals, d_stats, nstats + 1, n > 1 ? rscr : nullptr, st);
    const int early_passes = (n >= (int64_t(1) << 16)) ? 2 : 0;
    int which = radix_sort_passes(keys, vals, keys_tmp, vals_tmp, n, 0, early_passes, true, rscr, st);
    // point storage, taken while the device works
    Arena& mp = pl->mem_pts;
    mp.set_pool(&ctx->pool, sreg);
    mp.reserve(size_t(n) * 8);                  // pts
    mp.reserve(size_t(n) * 4);                  // perm
    mp.reserve(size_t(n) * 4);                  // pinst
    mp.reserve(size_t(n) * 4);                  // pkey
    mp.reserve(size_t(n) * 8);                  // fs
    mp.allocate();
    pl->pts = mp.take<int32_t>(size_t(n) * 2);
    pl->perm = mp.take<int32_t>(n);
    pl->pinst = mp.take<int32_t>(n);
    pl->pkey = mp.take<uint32_t>(n);
    pl->fs = mp.take<double>(n);
    if (sreg) {
        LFMM_HIP(hipMemcpyAsync(rb_host.data(), bb, size_t(K) * 16, hipMemcpyDeviceToHost, st));
        LFMM_HIP(hipStreamSynchronize(st));
        bb = rb_host.data();
    } else {
        LFMM_HIP(hipEventSynchronize(bb_ready->ev));
    }
    pl->inst.assign(size_t(K), InstInfo{});
    int Dmax = 0;
    for (int32_t k = 0; k < K; ++k) {
        InstInfo& I = pl->inst[size_t(k)];
        const int32_t* b = &bb[size_t(k) * 4];
        const int64_t extent = std::max(int64_t(b[2]) - b[0], int64_t(b[3]) - b[1]) + 1;
        if (extent > (int64_t(1) << 31)) throw std::out_of_range("coordinate extent of 2^31 or more");
        I.pt0 = pl->pt_off[size_t(k)];
        I.pt1 = pl->pt_off[size_t(k) + 1];
        I.ox = b[0];
        I.oy = b[1];
        I.D = bits_for_extent(extent);
        Dmax = std::max(Dmax, I.D);
        int32_t ml = ml_all;
        if (ml <= 0) {
            std::lock_guard<std::mutex> lock(ctx->mu);
            auto it = ctx->tuned.find(tune_key(I.pt1 - I.pt0, I.D));
            ml = it != ctx->tuned.end() ? it->second : kDefaultMaxLeaf;
        }
        I.max_leaf = ml;
    }
    int ibits = 0;
    while ((int64_t(1) << ibits) < K) ++ibits;
    if (2 * Dmax + ibits > 64) throw std::out_of_range("too many instances for the coordinate extent");
    pl->Dmax = Dmax;

    Stager stage_b(ctx, sreg != nullptr);
    if (ml_all <= 0) {   // per-instance N_leaf: the host writes the instance table
        stage_b.add(d_inst0, pl->inst);
        stage_b.flush(st);
    }

    // ---- Morton order: the rest of the sort ------------------------------------------------
    const int kbits = 2 * Dmax + ibits;
    which = radix_sort_passes(keys, vals, keys_tmp, vals_tmp, n, early_passes,
                              std::max(early_passes, (kbits + 7) / 8), true, rscr, st);
    uint64_t* skeys = which ? keys_tmp : keys;
    uint32_t* svals = which ? vals_tmp : vals;

    // ---- leaf levels and box counts ---------------------------------------------------------
    launch_level_stats(skeys, svals, d_chunks, nch, d_inst0, Dmax, K, pl->pts, pl->perm, pl->pinst, cl, d_stats,
                       stat_copies, d_stats + nstats, stats, st);
    if (sreg) {
        LFMM_HIP(hipMemcpyAsync(rb_host.data() + size_t(K) * 4, stats, (rb_words - size_t(K) * 4) * 4,
                                hipMemcpyDeviceToHost, st));
        stats = rb_host.data() + size_t(K) * 4;
    }
    LFMM_HIP(hipStreamSynchronize(st));
    const int32_t* hist = stats;
    const int32_t* maxc = stats + size_t(K) * (kMaxLevels + 2);

    std::map<int64_t, int> side_index;
    std::vector<int> nlev_of_side;
    std::vector<int64_t> side_of;
    int Lmax = 0;
    std::vector<std::vector<int32_t>> cnt(static_cast<size_t>(K));
    for (int32_t k = 0; k < K; ++k) {
        InstInfo& I = pl->inst[size_t(k)];
        const int64_t nk = I.pt1 - I.pt0;
        int L = (nk > I.max_leaf) ? std::min(I.D, maxc[size_t(k)] + 1) : 0;
        int min_L = 0;   // leaves no wider than the dense-model limit (Remark 8.2)
        while ((int64_t(1) << (I.D - min_L)) > kDenseLeafMax) ++min_L;
        L = std::max(L, min_L);
        I.L = L;
        Lmax = std::max(Lmax, L);
        const int64_t side = int64_t(1) << (I.D - L);
        auto it = side_index.find(side);
        if (it == side_index.end()) {
            it = side_index.emplace(side, int(side_of.size())).first;
            side_of.push_back(side);
            nlev_of_side.push_back(1);
        }
        I.ops = it->second;
        nlev_of_side[size_t(I.ops)] = std::max(nlev_of_side[size_t(I.ops)], std::max(L - 1, 1));
        cnt[size_t(k)].assign(size_t(L) + 1, 0);
        for (int lev = 0; lev <= L; ++lev) {
            int32_t b = 0;
            for (int c = -1; c < lev; ++c) b += hist[size_t(k) * (kMaxLevels + 2) + size_t(c + 1)];
            cnt[size_t(k)][size_t(lev)] = b;
            I.lev_count[lev] = b;
        }
    }
    pl->Lmax = Lmax;
    pl->Hmax = Lmax;
    if (side_of.size() > 64) throw std::out_of_range("more than 64 distinct leaf sides in one plan");
    pl->ops.resize(side_of.size());
    for (size_t o = 0; o < side_of.size(); ++o)
        pl->ops[o] = get_ops(ctx, side_of[o], nlev_of_side[o], st, sreg != nullptr);

    // instance order inside every height block: by operator set, then deepest first, so that
    // the boxes of one operator set with level >= 2 (or >= 3) form one contiguous range
    std::vector<int32_t> order(static_cast<size_t>(K));
    for (int32_t k = 0; k < K; ++k) order[size_t(k)] = k;
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
        const InstInfo &A = pl->inst[size_t(a)], &B = pl->inst[size_t(b)];
        if (A.ops != B.ops) return A.ops < B.ops;
        return A.L > B.L;
    });
    const int H = pl->Hmax;
    pl->hbase.assign(size_t(H) + 2, 0);
    int32_t cur = 0;
    for (int h = 0; h <= H; ++h) {
        pl->hbase[size_t(h)] = cur;
        for (int32_t k : order) {
            InstInfo& I = pl->inst[size_t(k)];
            if (I.L < h) continue;
            const int lev = I.L - h;
            I.lev_base[lev] = cur;
            cur += cnt[size_t(k)][size_t(lev)];
        }
    }
    pl->hbase[size_t(H) + 1] = cur;
    pl->nbox = cur;
    pl->nleaf = pl->hbase[1];
    {
        int32_t r = 0;
        for (int32_t k = 0; k < K; ++k) {
            pl->inst[size_t(k)].leaf_rank0 = r;
            r += cnt[size_t(k)][size_t(pl->inst[size_t(k)].L)];
        }
    }
    // range of boxes of height h, operator set o and level >= minlev
    auto range_of = [&](int h, int o, int minlev, int32_t& g0, int32_t& g1) {
        g0 = g1 = -1;
        for (int32_t k : order) {
            const InstInfo& I = pl->inst[size_t(k)];
            if (I.ops != o || I.L < h || I.L - h < minlev) continue;
            const int lev = I.L - h;
            if (g0 < 0) g0 = I.lev_base[lev];
            g1 = I.lev_base[lev] + cnt[size_t(k)][size_t(lev)];
        }
    };
    pl->leaf_of_ops.assign(side_of.size(), TileRange{});
    for (size_t o = 0; o < side_of.size(); ++o) {
        int32_t g0, g1;
        range_of(0, int(o), 0, g0, g1);
        if (g0 >= 0) pl->leaf_of_ops[o] = TileRange{g0, g1 - g0};
    }
    // near-field groups per operator set: the children of its height-1 boxes, then its roots
    // that are leaves (instances of one leaf)
    pl->near_of_ops.assign(side_of.size(), TileRange{});
    std::vector<int32_t> h1_start(side_of.size(), 0), h1_count(side_of.size(), 0);
    std::vector<std::vector<int32_t>> roots(side_of.size());
    for (int32_t k : order) {
        const InstInfo& I = pl->inst[size_t(k)];
        if (I.L == 0) roots[size_t(I.ops)].push_back(I.lev_base[0]);
    }
    std::vector<int32_t> root_list;
    std::vector<int32_t> root_off(side_of.size(), 0);
    for (size_t o = 0; o < side_of.size(); ++o) {
        int32_t g0, g1;
        range_of(1, int(o), 0, g0, g1);
        if (g0 >= 0) {
            h1_start[o] = g0;
            h1_count[o] = g1 - g0;
        }
        root_off[o] = int32_t(root_list.size());
        root_list.insert(root_list.end(), roots[o].begin(), roots[o].end());
        pl->near_of_ops[o] = TileRange{pl->nq, h1_count[o] + int32_t(roots[o].size())};
        pl->nq += pl->near_of_ops[o].n;
    }
    // groups for the class-sorted passes and the M2M tiles
    std::vector<BoxGroup> m2l_groups, l2l_groups;
    std::vector<BoxTile> m2m_tiles;
    pl->m2m.assign(size_t(H) + 1, TileRange{});
    pl->l2l.assign(size_t(H) + 1, TileRange{});
    int32_t cls_slots = 0, tile_slots = 0;
    for (int h = 0; h <= H; ++h)
        for (size_t o = 0; o < side_of.size(); ++o) {
            int32_t g0, g1;
            range_of(h, int(o), 2, g0, g1);
            if (g0 < 0 || g1 <= g0) continue;
            const int32_t cap = (g1 - g0 + kM2LTile - 1) / kM2LTile + 3;
            m2l_groups.push_back(BoxGroup{int32_t(o), h, g0, g1, cls_slots, tile_slots, cap, kM2LTile});
            cls_slots += 4 * (g1 - g0);
            tile_slots += cap;
        }
    pl->m2l = TileRange{0, tile_slots};
    for (int h = 0; h <= H; ++h) {
        pl->l2l[size_t(h)].t0 = tile_slots;
        for (size_t o = 0; o < side_of.size(); ++o) {
            int32_t g0, g1;
            range_of(h, int(o), 3, g0, g1);
            if (g0 < 0 || g1 <= g0) continue;
            const int32_t cap = (g1 - g0 + kBoxMatTile - 1) / kBoxMatTile + 3;
            l2l_groups.push_back(BoxGroup{int32_t(o), h, g0, g1, cls_slots, tile_slots, cap, kBoxMatTile});
            cls_slots += 4 * (g1 - g0);
            tile_slots += cap;
        }
        pl->l2l[size_t(h)].n = tile_slots - pl->l2l[size_t(h)].t0;
    }
    // M2M tiles: runs of consecutive boxes, built here (their own table)
    for (int h = 1; h <= H; ++h) {
        pl->m2m[size_t(h)].t0 = int32_t(m2m_tiles.size());
        for (size_t o = 0; o < side_of.size(); ++o) {
            int32_t g0, g1;
            range_of(h, int(o), 2, g0, g1);
            for (int32_t s = g0; g0 >= 0 && s < g1; s += kBoxMatTile)
                m2m_tiles.push_back(BoxTile{int32_t(o), h, 0, s, std::min(kBoxMatTile, g1 - s), 0, 0, 0});
        }
        pl->m2m[size_t(h)].n = int32_t(m2m_tiles.size()) - pl->m2m[size_t(h)].t0;
    }
    std::vector<BoxGroup> groups = m2l_groups;
    groups.insert(groups.end(), l2l_groups.begin(), l2l_groups.end());

    // small tables, uploaded in one copy (ExecPtrs last: written at execute time)
    Arena& ms = pl->mem_small;
    ms.set_pool(&ctx->pool, sreg);
    ms.reserve(size_t(K) * sizeof(InstInfo));
    ms.reserve(size_t(64) * sizeof(OpsPtrs));
    ms.reserve(size_t(K));                      // far flags
    ms.reserve(16);                             // M2L tile count
    ms.reserve(std::max<size_t>(groups.size(), 1) * sizeof(BoxGroup));
    ms.reserve(std::max<size_t>(m2m_tiles.size(), 1) * sizeof(BoxTile));
    ms.reserve(std::max<size_t>(root_list.size(), 1) * sizeof(int32_t));
    ms.reserve(size_t(K) * sizeof(ExecPtrs));
    ms.allocate();
    pl->d_inst = ms.take<InstInfo>(K);
    pl->d_ops = ms.take<OpsPtrs>(64);
    pl->d_far = ms.take<uint8_t>(K);
    pl->d_m2l_ntiles = ms.take<int32_t>(4);
    BoxGroup* d_groups = ms.take<BoxGroup>(std::max<size_t>(groups.size(), 1));
    pl->m2m_tiles = ms.take<BoxTile>(std::max<size_t>(m2m_tiles.size(), 1));
    int32_t* d_roots = ms.take<int32_t>(std::max<size_t>(root_list.size(), 1));
    pl->d_exec = ms.take<ExecPtrs>(K);

    // ---- plan storage sized by the boxes --------------------------------------------------------
    const int64_t nb = pl->nbox, nl = pl->nleaf;
    const int P = kRankPad;
    Arena& mb = pl->mem_box;
    mb.set_pool(&ctx->pool, sreg);
    mb.reserve(size_t(nb) * 8);                          // key
    for (int q = 0; q < 5; ++q) mb.reserve(size_t(nb) * 4);   // pt0, pt1, parent, inst, (pad)
    mb.reserve(size_t(nb));                              // level
    mb.reserve(size_t(nb) * 16);                         // child
    mb.reserve(size_t(nb) * 36);                         // neighbour lists
    mb.reserve(size_t(nb) * 4 * kNumInteractions);       // interaction lists
    mb.reserve(size_t(std::max(cls_slots, 1)) * 4);
    mb.reserve(size_t(std::max(tile_slots, 1)) * sizeof(BoxTile));
    mb.reserve(size_t(nb + 1) * P * 8);                  // Q and its zero row
    mb.reserve(size_t(std::max(pl->nq, 1)) * sizeof(NearGroup));
    mb.reserve(size_t(std::max(pl->nq, 1)) * kNearEntries * sizeof(int4));
    mb.reserve(size_t(nb + 1) * P * 8);                  // U and its zero row
    const bool mixed = ctx->opt.precision == LFMM_MIXED;
    const bool mixed_bf16 = ctx->opt.precision == LFMM_MIXED_BF16;
    if (mixed) {
        mb.reserve(size_t(nb + 1) * P * 4);              // Q hi
        mb.reserve(size_t(nb + 1) * P * 4);              // Q lo
        mb.reserve(size_t(nb + 1) * 8);                  // charge sums
    }
    if (mixed_bf16) {
        // the bf16 M2L kernel addresses Q's parts by 32-bit byte offsets
        if ((uint64_t(nb) + 1) * uint64_t(kBf16QVecs) * 16u > uint64_t(UINT32_MAX))
            throw std::out_of_range("LFMM_MIXED_BF16 plans hold at most " +
                                    std::to_string(uint64_t(UINT32_MAX) / (kBf16QVecs * 16u) - 1) + " boxes");
        mb.reserve(size_t(nb + 1) * P * 6);              // Q in three bf16 parts
        mb.reserve(size_t(nb + 1) * 8);                  // charge sums
    }
    const bool adaptive = (ctx->opt.flags & LFMM_FLAG_ADAPTIVE) != 0;
    pl->adaptive = adaptive;
    if (adaptive) {
        mb.reserve(size_t(nb));                          // roles
        mb.reserve(size_t(3) * size_t(nb + 1) * 4);      // list row starts
        mb.reserve(size_t(n) * 4);                       // finest box of each point
        mb.reserve(size_t(std::max(pl->m2l.n, 1)) * sizeof(BoxTile));   // compacted M2L tiles
    }
    mb.allocate();
    pl->box_key = mb.take<uint64_t>(nb);
    pl->box_pt0 = mb.take<int32_t>(nb);
    pl->box_pt1 = mb.take<int32_t>(nb);
    pl->box_parent = mb.take<int32_t>(nb);
    pl->box_inst = mb.take<int32_t>(nb);
    (void)mb.take<int32_t>(nb);
    pl->box_lev = mb.take<int8_t>(nb);
    pl->box_child = mb.take<int32_t>(size_t(nb) * 4);
    pl->nb9 = mb.take<int32_t>(size_t(nb) * 9);
    pl->il27 = mb.take<int32_t>(size_t(nb) * kNumInteractions);
    pl->cls_box = mb.take<int32_t>(std::max(cls_slots, 1));
    pl->tiles = mb.take<BoxTile>(std::max(tile_slots, 1));
    pl->Q = mb.take<double>(size_t(nb + 1) * P);
    pl->U = mb.take<double>(size_t(nb + 1) * P);
    pl->groups = mb.take<NearGroup>(size_t(std::max(pl->nq, 1)));
    pl->ents = mb.take<int4>(size_t(std::max(pl->nq, 1)) * kNearEntries);
    if (mixed) {
        pl->Qh = mb.take<float>(size_t(nb + 1) * P);
        pl->Ql = mb.take<float>(size_t(nb + 1) * P);
        pl->qsum = mb.take<double>(size_t(nb + 1));
    }
    if (mixed_bf16) {
        pl->Qb = mb.take<uint16_t>(size_t(nb + 1) * P * 3);
        pl->qsum = mb.take<double>(size_t(nb + 1));
    }
    if (adaptive) {
        pl->role = mb.take<int8_t>(nb);
        pl->list_off = mb.take<int32_t>(size_t(3) * size_t(nb + 1));
        pl->pt_box = mb.take<int32_t>(n);
        pl->m2l_tiles = mb.take<BoxTile>(size_t(std::max(pl->m2l.n, 1)));
    }

    // ---- tables ---------------------------------------------------------------------------------
    Stager stage_c(ctx, sreg != nullptr);
    stage_c.add(d_roots, root_list);
    stage_c.add(pl->d_inst, pl->inst);
    std::vector<OpsPtrs> optab(64);   // the whole table, so that the upload stays one copy
    for (size_t o = 0; o < pl->ops.size(); ++o) optab[o] = ops_ptrs(pl->ops[o]);
    stage_c.add(pl->d_ops, optab);
    std::vector<uint8_t> far(static_cast<size_t>(K));
    for (int32_t k = 0; k < K; ++k) far[size_t(k)] = pl->inst[size_t(k)].L >= 2 ? 1 : 0;
    stage_c.add(pl->d_far, far);
    stage_c.add(d_groups, groups);
    stage_c.add(pl->m2m_tiles, m2m_tiles);
    std::vector<int32_t> m2l_n{pl->m2l.n};
    stage_c.add(pl->d_m2l_ntiles, m2l_n);
    stage_c.flush(st);

    // ---- leaves ---------------------------------------------------------------------------------
    Arena tmp2(&ctx->pool, sreg);
    const int rows = std::max(Lmax, 1);
    tmp2.reserve(size_t(nl) * 4);                        // leaf first point
    tmp2.reserve(size_t(nl) * 8);                        // leaf keys
    tmp2.reserve(size_t(nl));                            // leaf cl
    tmp2.reserve(size_t(nl) * 4);                        // leaf instance
    tmp2.reserve(size_t(rows) * nl * 4);                 // level scans
    tmp2.reserve(scan_scratch_bytes(nl, rows));
    tmp2.reserve(size_t(nb) * 4 * 4);                    // class scans
    tmp2.reserve(64);                                    // class totals
    tmp2.reserve(scan_scratch_bytes(nb, 4));
    if (adaptive) {
        tmp2.reserve(size_t(nb) * 4 * 4);                // class scans over the M2L boxes
        tmp2.reserve(64);                                // their totals
        tmp2.reserve(size_t(3) * size_t(nb + 1) * 4);    // list lengths
        tmp2.reserve(size_t(3) * size_t(nb + 1) * 4);    // item positions
        tmp2.reserve(64);                                // totals of both
        tmp2.reserve(scan_scratch_bytes(nb + 1, 3));
    }
    tmp2.allocate();
    SyncOnUnwind unwind_tmp2;
    int32_t* leaf_pt0 = tmp2.take<int32_t>(nl);
    uint64_t* leaf_key = tmp2.take<uint64_t>(nl);
    int8_t* leaf_cl = tmp2.take<int8_t>(nl);
    int32_t* leaf_inst = tmp2.take<int32_t>(nl);
    int32_t* lscan = tmp2.take<int32_t>(size_t(rows) * nl);
    void* lscr = tmp2.take<char>(scan_scratch_bytes(nl, rows));
    int32_t* cscan = tmp2.take<int32_t>(size_t(nb) * 4);
    int32_t* ctotal = tmp2.take<int32_t>(16);
    void* cscr = tmp2.take<char>(scan_scratch_bytes(nb, 4));
    int32_t *cscan_v = nullptr, *ctotal_v = nullptr, *lcnt = nullptr, *lpos = nullptr, *ltot = nullptr;
    void* lscr2 = nullptr;
    if (adaptive) {
        cscan_v = tmp2.take<int32_t>(size_t(nb) * 4);
        ctotal_v = tmp2.take<int32_t>(16);
        lcnt = tmp2.take<int32_t>(size_t(3) * size_t(nb + 1));
        lpos = tmp2.take<int32_t>(size_t(3) * size_t(nb + 1));
        ltot = tmp2.take<int32_t>(16);
        lscr2 = tmp2.take<char>(scan_scratch_bytes(nb + 1, 3));
    }

    // leaves (and the window keys of the points) straight from the scan of the leaf starts
    scan_leaf_starts(cl, pl->pinst, pl->d_inst, n, skeys, Dmax, pl->pts, pl->pkey, leaf_pt0, leaf_key, leaf_cl,
                     leaf_inst, sscr, st);
    if (Lmax > 0) scan_level_starts(leaf_cl, leaf_inst, pl->d_inst, nl, Lmax, lscan, lscr, st);
    launch_build_boxes(lscan, leaf_cl, leaf_pt0, leaf_key, leaf_inst, pl->d_inst, nl, Lmax, pl->box_key, pl->box_pt0,
                       pl->box_parent, pl->box_child, pl->box_inst, pl->box_lev, st);
    // also zeroes row nb of Q-hat and U-hat, which the box-matrix kernels read for absent sources
    launch_link_boxes(pl->box_key, pl->box_parent, pl->box_inst, pl->box_lev, pl->d_inst, nb, pl->box_pt0,
                      pl->box_child, pl->box_pt1, pl->Q + size_t(nb) * P, pl->U + size_t(nb) * P, st);
    launch_lists(pl->box_key, pl->box_parent, pl->box_child, pl->box_inst, pl->box_lev, pl->d_inst, nb, pl->nb9,
                 pl->il27, st);
    const int32_t m2l_slots = pl->m2l.n;
    const int32_t n_m2l_groups = int32_t(m2l_groups.size());
    if (!adaptive) {
        for (size_t o = 0; o < side_of.size(); ++o)   // groups need the leaves' neighbour lists
            launch_near_groups(pl->near_of_ops[o].t0, h1_start[o], h1_count[o], d_roots + root_off[o],
                               int32_t(roots[o].size()), pl->box_child, pl->nb9, pl->box_pt0, pl->box_pt1,
                               pl->box_key, pl->groups, pl->ents, st);
        scan_child_classes(pl->box_key, nb, cscan, ctotal, cscr, st);
        launch_class_lists(d_groups, int32_t(groups.size()), 0, tile_slots, cscan, ctotal, pl->box_key, pl->box_lev,
                           nullptr, nb, pl->cls_box, pl->tiles, st);
    } else {
        // roles, V lists (interaction lists without pruned boxes) and the M2L tiles over the
        // boxes that take part; L2L keeps every box (pruned ones relay expansions)
        launch_roles(pl->box_pt0, pl->box_pt1, pl->box_parent, pl->box_lev, pl->box_inst, pl->d_inst, nb, pl->role,
                     st);
        launch_filter_interactions(pl->role, nb, pl->il27, st);
        scan_child_classes_active(pl->box_key, pl->box_lev, pl->role, nb, cscan_v, ctotal_v, cscr, st);
        launch_class_lists(d_groups, n_m2l_groups, 0, m2l_slots, cscan_v, ctotal_v, pl->box_key, pl->box_lev,
                           pl->role, nb, pl->cls_box, pl->tiles, st);
        // most slots stay empty (pruned boxes): M2L walks the non-empty tiles only, so that its
        // XCD-contiguous split of the tile list stays balanced
        compact_tiles(pl->tiles, m2l_slots, pl->m2l_tiles, pl->d_m2l_ntiles, cscr, st);
        scan_child_classes(pl->box_key, nb, cscan, ctotal, cscr, st);
        launch_class_lists(d_groups + n_m2l_groups, int32_t(groups.size()) - n_m2l_groups, m2l_slots,
                           tile_slots - m2l_slots, cscan, ctotal, pl->box_key, pl->box_lev, nullptr, nb,
                           pl->cls_box, pl->tiles, st);
        // U, W, X lists: lengths, row starts, item positions, one read-back of the totals
        const int64_t nb1 = nb + 1;
        launch_adaptive_lists(false, pl->box_key, pl->box_parent, pl->box_child, pl->box_lev, pl->role, pl->nb9,
                              pl->box_pt0, pl->box_pt1, nb, lcnt, nullptr, nullptr, st);
        scan_rows(lcnt, pl->list_off, nb1, 3, ltot, lscr2, st);
        scan_positive(lcnt, nb1, 3, lpos, ltot + 4, lscr2, st);
        launch_point_boxes(pl->box_pt0, pl->box_pt1, pl->nleaf, pl->pt_box, st);
        int32_t tot[8] = {};
        LFMM_HIP(hipMemcpyAsync(tot, ltot, sizeof(tot), hipMemcpyDeviceToHost, st));
        LFMM_HIP(hipStreamSynchronize(st));
        Arena& ma = pl->mem_ad;
        ma.set_pool(&ctx->pool, sreg);
        for (int r = 0; r < 3; ++r) {
            pl->list_len[r] = tot[r];
            ma.reserve(size_t(std::max(tot[r], 1)) * 4);
        }
        pl->n_ad_leaves = tot[4];
        pl->n_ad_xboxes = tot[6];
        ma.reserve(size_t(std::max(tot[4], 1)) * 4);
        ma.reserve(size_t(std::max(tot[6], 1)) * 4);
        ma.allocate();
        for (int r = 0; r < 3; ++r) pl->list_ent[r] = ma.take<int32_t>(size_t(std::max(tot[r], 1)));
        pl->ad_leaves = ma.take<int32_t>(size_t(std::max(tot[4], 1)));
        pl->ad_xboxes = ma.take<int32_t>(size_t(std::max(tot[6], 1)));
        launch_adaptive_lists(true, pl->box_key, pl->box_parent, pl->box_child, pl->box_lev, pl->role, pl->nb9,
                              pl->box_pt0, pl->box_pt1, nb, nullptr, pl->list_off, pl->list_ent, st);
        launch_compact_positive(lcnt, lpos, nb, pl->ad_leaves, st);
        launch_compact_positive(lcnt + 2 * nb1, lpos + 2 * nb1, nb, pl->ad_xboxes, st);
    }
    LFMM_HIP(hipGetLastError());
    // staging for the per-execute pointer table of batched plans (and of graph replays,
    // whose kernels always read the table)
    pl->use_graph = (ctx->opt.flags & LFMM_FLAG_GRAPH) != 0 && !sreg;
    if (K > 1 || pl->use_graph) {
        acquire_exec_staging(pl);
    }
    pl->build_stream = st;
    if (sreg) {   // the staged host copies must have been read before they go
        LFMM_HIP(hipStreamSynchronize(st));
        return;
    }
    // no synchronisation: the temporaries and staging blocks go back to their pools once the
    // device has passed the end of the build, and executes on other streams wait for it
    pl->built = std::make_shared<Fence>(st);
    pl->build_stream = st;
    tmp.release_after(pl->built);
    tmp2.release_after(pl->built);
    stage_c.retire(pl->built);
}

// Enqueues the evaluation passes (Section 8.2) on st.  tab = per-instance load/potential
// pointers on the device, or null with f1/u1 those of the single instance (in the plan's
// Morton order when sorted).
void enqueue_passes(lfmm_plan* pl, const ExecPtrs* tab, const double* f1, double* u1, uint32_t marks, hipStream_t st,
                    bool sorted = false) {
    const ExecPtrs single{f1, u1, pl->nsrc[0], pl->tgt0[0], sorted ? 1 : 0, 0};
    const bool mixed = pl->ctx->opt.precision == LFMM_MIXED;
    const bool mixed_bf16 = pl->ctx->opt.precision == LFMM_MIXED_BF16;
    auto mark = [&](int k) {
        // event k opens phase k and closes phase k - 1
        if ((marks >> k & 1u) || (k > 0 && (marks >> (k - 1) & 1u))) LFMM_HIP(hipEventRecord(pl->ev[k], st));
    };
    mark(0);
    mark(1);   // the loads are gathered into Morton order by P2M itself
    for (size_t o = 0; o < pl->ops.size(); ++o) {
        const TileRange& r = pl->leaf_of_ops[o];
        launch_p2m(r.t0, r.t0 + r.n, pl->box_pt0, pl->box_pt1, pl->box_key, pl->ops[o]->dev.leaf_side, pl->pts, tab,
                   single, pl->perm, pl->pinst, pl->fs, pl->ops[o]->dev.leafT, pl->Q,
                   double(pl->n) / double(std::max<int32_t>(pl->nleaf, 1)), st);
    }
    mark(2);
    for (int h = 1; h <= pl->Hmax; ++h) {
        const TileRange& r = pl->m2m[size_t(h)];
        if (r.n > 0) launch_m2m(pl->m2m_tiles + r.t0, r.n, pl->box_child, pl->d_ops, pl->Q, pl->nbox, st);
    }
    mark(3);
    if (pl->m2l.n > 0) {
        const BoxTile* mt = pl->m2l_tiles ? pl->m2l_tiles : pl->tiles + pl->m2l.t0;
        if (mixed_bf16) {
            launch_split_q_bf16(pl->Q, pl->nbox + 1, pl->Qb, pl->qsum, st);
            launch_m2l_bf16(mt, pl->d_m2l_ntiles, pl->m2l.n, pl->cls_box, pl->il27, pl->d_ops, pl->Qb, pl->qsum,
                            pl->nbox, pl->U, st);
        } else if (mixed) {
            launch_split_q(pl->Q, pl->nbox + 1, pl->Qh, pl->Ql, pl->qsum, st);
            launch_m2l_mixed(mt, pl->d_m2l_ntiles, pl->m2l.n, pl->cls_box, pl->il27, pl->d_ops, pl->Qh, pl->Ql,
                             pl->qsum, pl->nbox, pl->U, st);
        }
        else
            launch_m2l(mt, pl->d_m2l_ntiles, pl->m2l.n, pl->cls_box, pl->il27, pl->d_ops, pl->Q, pl->nbox, pl->U, st);
    }
    mark(4);
    AdaptiveLists lists{};
    if (pl->adaptive) {
        for (int r = 0; r < 3; ++r) {
            lists.off[r] = pl->list_off + size_t(r) * size_t(pl->nbox + 1);
            lists.ent[r] = pl->list_ent[r];
        }
        // P2L of the X lists (after M2L wrote the incoming expansions, before L2L reads
        // them), timed with the downward pass
        launch_p2l(pl->n_ad_xboxes, pl->ad_xboxes, lists, pl->box_pt0, pl->box_pt1, pl->box_key, pl->box_lev,
                   pl->box_inst, pl->d_inst, pl->d_ops, pl->pts, pl->fs, pl->U, pl->ctx->phi_oct, pl->ctx->phi_far,
                   st);
    }
    for (int h = pl->Hmax; h >= 0; --h) {
        const TileRange& r = pl->l2l[size_t(h)];
        if (r.n > 0)
            launch_l2l(pl->tiles + r.t0, r.n, pl->cls_box, pl->box_parent, pl->d_ops, pl->U, pl->nbox, pl->role, st);
    }
    mark(5);
    if (pl->adaptive) {
        launch_near_adaptive(pl->n_ad_leaves, pl->ad_leaves, lists, pl->box_pt0, pl->box_pt1, pl->box_key,
                             pl->box_lev, pl->box_inst, pl->d_inst, pl->d_ops, pl->pts, pl->fs, pl->Q, pl->pt_box,
                             pl->U, pl->perm, tab, single, pl->d_far, pl->ctx->phi_oct, pl->ctx->phi_far,
                             st);
        mark(6);
        return;
    }
    for (size_t o = 0; o < pl->ops.size(); ++o) {
        const TileRange& r = pl->near_of_ops[o];
        launch_near(r.t0, r.t0 + r.n, pl->groups, pl->ents, pl->box_pt0, pl->box_pt1, pl->box_key, pl->box_inst,
                    pl->ops[o]->dev.leaf_side, pl->pts, pl->pkey, pl->fs, pl->perm, tab, single, pl->U,
                    pl->ops[o]->dev.leafT, pl->ops[o]->dev.leafTt, pl->d_far, pl->ctx->phi_oct, pl->ctx->phi_far,
                    st);
    }
    mark(6);
}


// sorted: f[0] and u[0] span every point of the plan in its Morton order (lfmm_execute_sorted)
void run_forest(lfmm_plan* pl, const double* const* f, double* const* u, hipStream_t st, bool sorted = false) {
    if (st != pl->build_stream) {
        pl->one_stream = false;
        if (pl->built) LFMM_HIP(hipStreamWaitEvent(st, pl->built->ev, 0));
    }
    if (pl->K == 1 && !pl->use_graph) {
        enqueue_passes(pl, nullptr, f[0], u[0], pl->timing_mask, st, sorted);
        if (pl->timing_mask) pl->timed_mask = pl->timing_mask;
        return;
    }
    std::vector<ExecPtrs> table(static_cast<size_t>(pl->K));
    for (int32_t k = 0; k < pl->K; ++k)
        table[size_t(k)] = ExecPtrs{sorted ? f[0] : f[k], sorted ? u[0] : u[k], pl->nsrc[size_t(k)],
                                    pl->tgt0[size_t(k)], sorted ? 1 : 0, 0};
    const bool same = pl->exec_last.size() == table.size() &&
                      std::memcmp(pl->exec_last.data(), table.data(), table.size() * sizeof(ExecPtrs)) == 0;
    if (!same) {
        // the upload is stream-ordered after every earlier execute on st (which read d_exec);
        // the staging slot is rewritten only after the upload that last read it
        const int slot = pl->exec_slot;
        pl->exec_slot = (slot + 1) % lfmm_plan::kExecRing;
        ExecPtrs* h = pl->h_exec + size_t(slot) * size_t(pl->K);
        LFMM_HIP(hipEventSynchronize(pl->exec_copied[slot]));
        std::memcpy(h, table.data(), table.size() * sizeof(ExecPtrs));
        launch_upload(pl->d_exec, h, size_t(pl->K) * sizeof(ExecPtrs), st);
        LFMM_HIP(hipEventRecord(pl->exec_copied[slot], st));
        pl->exec_last.swap(table);
    }
    if (!pl->use_graph) {
        enqueue_passes(pl, pl->d_exec, nullptr, nullptr, pl->timing_mask, st);
        if (pl->timing_mask) pl->timed_mask = pl->timing_mask;
        return;
    }
    if (!pl->gexec) {
        // record the passes once, on the context's capture stream (a capture cannot run on
        // the legacy default stream), and replay them on st from then on
        lfmm_ctx* ctx = pl->ctx;
        if (!ctx->capture) LFMM_HIP(hipStreamCreateWithFlags(&ctx->capture, hipStreamNonBlocking));
        LFMM_HIP(hipStreamBeginCapture(ctx->capture, hipStreamCaptureModeThreadLocal));
        try {
            enqueue_passes(pl, pl->d_exec, nullptr, nullptr, false, ctx->capture);
        } catch (...) {
            hipGraph_t g = nullptr;
            (void)hipStreamEndCapture(ctx->capture, &g);
            if (g) (void)hipGraphDestroy(g);
            throw;
        }
        LFMM_HIP(hipStreamEndCapture(ctx->capture, &pl->graph));
        LFMM_HIP(hipGraphInstantiate(&pl->gexec, pl->graph, nullptr, nullptr, 0));
    }
    LFMM_HIP(hipGraphLaunch(pl->gexec, st));
}

}  // namespace

void lfmm::plan_destroy_completed(lfmm_plan* pl) { delete pl; }


int lfmm::ctx_device(const lfmm_ctx* ctx) { return ctx->device; }

int32_t lfmm::ctx_flags(const lfmm_ctx* ctx) { return ctx->opt.flags; }

void lfmm::ctx_add_server(lfmm_ctx* ctx, lfmm_server* srv) {
    std::lock_guard<std::mutex> lock(ctx->reg_mu);
    ctx->servers.insert(srv);
}

void lfmm::ctx_remove_server(lfmm_ctx* ctx, lfmm_server* srv) {
    std::lock_guard<std::mutex> lock(ctx->reg_mu);
    ctx->servers.erase(srv);
}

namespace {

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
    } catch (const Unsupported& e) {
        return fail(LFMM_E_UNSUPPORTED, e.msg);
    } catch (const std::bad_alloc&) {
        return fail(LFMM_E_NOMEM, "host allocation failed");
    } catch (const std::out_of_range& e) {
        return fail(LFMM_E_RANGE, e.what());
    } catch (const std::exception& e) {
        return fail(LFMM_E_INVAL, e.what());
    }
}

lfmm_status create_forest(lfmm_ctx* ctx, int32_t K, const InstanceInput* in, int32_t max_leaf, void* stream,
                          lfmm_plan** out) {
    if (!ctx || !out || !in || K < 1) return fail(LFMM_E_INVAL, "null argument or no instance");
    *out = nullptr;
    int64_t total = 0;
    for (int32_t k = 0; k < K; ++k) {
        if (in[k].n_src < 1 || in[k].n_src > (int64_t(1) << 30) || !in[k].src)
            return fail(LFMM_E_INVAL, "every instance needs 1 <= n_src <= 2^30 and source coordinates");
        if (in[k].tgt && (in[k].n_tgt < 1 || in[k].n_tgt > (int64_t(1) << 30)))
            return fail(LFMM_E_INVAL, "an instance with target coordinates needs 1 <= n_tgt <= 2^30");
        if (!in[k].tgt && in[k].n_tgt != 0 && in[k].n_tgt != in[k].n_src)
            return fail(LFMM_E_INVAL, "without target coordinates n_tgt must be 0 or n_src (targets = sources)");
        total += in[k].n_src + (in[k].tgt ? in[k].n_tgt : 0);
    }
    if (total > (int64_t(1) << 30)) return fail(LFMM_E_INVAL, "more than 2^30 points in one plan");
    return guarded([&]() -> lfmm_status {
        LFMM_HIP(hipSetDevice(ctx->device));
        auto pl = std::make_unique<lfmm_plan>();
        pl->ctx = ctx;
        build_forest(pl.get(), K, in, max_leaf, as_stream(stream));
        {
            std::lock_guard<std::mutex> lock(ctx->reg_mu);
            ctx->plans.insert(pl.get());
        }
        *out = pl.release();
        return LFMM_OK;
    });
}

// Checks of the loads of K instances (f[k] holds nsrc[k] values) before any pass: a NaN or
// infinite load is an invalid input (LFMM_E_INVAL); a total load that is not zero (|sum f| >
// 1e-12 sum |f|, the well-posedness condition of Section 1) is reported as LFMM_W_NONZERO_SUM,
// and the finite sum is still computed.  Synchronises the stream (the statistics are read
// back).  Runs inside guarded().
lfmm_status check_loads(lfmm_ctx* ctx, int32_t K, const double* const* f, const int32_t* nsrc, hipStream_t st,
                        StaticRegion* sreg = nullptr) {
    Arena a(&ctx->pool, sreg);
    a.reserve(load_stats_scratch_bytes());
    a.reserve(size_t(K) * 3 * sizeof(double));
    a.allocate();
    double* scr = a.take<double>(load_stats_scratch_bytes() / sizeof(double));
    double* out = a.take<double>(size_t(K) * 3);
    for (int32_t k = 0; k < K; ++k) launch_load_stats(f[k], nsrc[k], scr, out + 3 * size_t(k), st);
    LFMM_HIP(hipGetLastError());
    std::vector<double> h(size_t(K) * 3);
    LFMM_HIP(hipMemcpyAsync(h.data(), out, h.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    LFMM_HIP(hipStreamSynchronize(st));
    a.release();
    lfmm_status res = LFMM_OK;
    for (int32_t k = 0; k < K; ++k) {
        const double sum = h[3 * size_t(k)], mag = h[3 * size_t(k) + 1], bad = h[3 * size_t(k) + 2];
        if (bad > 0.0)
            return fail(LFMM_E_INVAL, "loads of instance " + std::to_string(k) + " hold " +
                                          std::to_string(int64_t(bad)) + " non-finite values");
        if (res == LFMM_OK && std::fabs(sum) > 1e-12 * mag)
            res = fail(LFMM_W_NONZERO_SUM, "total load of instance " + std::to_string(k) + " is " +
                                               std::to_string(sum) + ", not zero");
    }
    return res;
}

lfmm_status execute_forest(lfmm_plan* pl, const double* const* f, double* const* u, void* stream, bool check,
                           bool sorted = false) {
    if (pl->failed) return fail(LFMM_E_HIP, "plan is in a failed state");
    return guarded([&]() -> lfmm_status {
        LFMM_HIP(hipSetDevice(pl->ctx->device));
        lfmm_status res = LFMM_OK;
        if (check || (pl->ctx->opt.flags & LFMM_FLAG_CHECK_LOADS)) {
            // sorted loads: one vector over every point of the plan
            const int32_t n_all = int32_t(pl->n);
            res = sorted ? check_loads(pl->ctx, 1, f, &n_all, as_stream(stream), pl->sreg)
                         : check_loads(pl->ctx, pl->K, f, pl->nsrc.data(), as_stream(stream), pl->sreg);
            if (res < 0) return res;
        }
        run_forest(pl, f, u, as_stream(stream), sorted);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) {
            pl->failed = true;
            throw HipFailure(std::string("kernel launch: ") + hipGetErrorString(e));
        }
        return res;
    });
}

}  // namespace

lfmm_status lfmm::root_bits_of(lfmm_ctx* ctx, int32_t K, const int64_t* n, const int32_t* const* xy, void* stream,
                               int32_t* bits) {
    if (!ctx || K < 1 || !n || !xy || !bits) return fail(LFMM_E_INVAL, "null argument");
    return guarded([&]() -> lfmm_status {
        LFMM_HIP(hipSetDevice(ctx->device));
        hipStream_t st = as_stream(stream);
        Arena a(&ctx->pool);
        a.reserve(size_t(K) * 16);
        a.allocate();
        int32_t* box = a.take<int32_t>(size_t(K) * 4);
        launch_extents(K, n, xy, box, st);
        LFMM_HIP(hipGetLastError());
        std::vector<int32_t> h(size_t(K) * 4);
        LFMM_HIP(hipMemcpyAsync(h.data(), box, h.size() * 4, hipMemcpyDeviceToHost, st));
        LFMM_HIP(hipStreamSynchronize(st));
        a.release();
        for (int32_t k = 0; k < K; ++k) {
            const int64_t ext = std::max(int64_t(h[4 * size_t(k) + 2]) - h[4 * size_t(k)],
                                         int64_t(h[4 * size_t(k) + 3]) - h[4 * size_t(k) + 1]) + 1;
            bits[k] = ext > (int64_t(1) << 31) ? 32 : bits_for_extent(ext);
        }
        return LFMM_OK;
    });
}

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
        // the allocation-free solve's workspace on this device
        void* sp = nullptr;
        LFMM_HIP(hipGetSymbolAddress(&sp, HIP_SYMBOL(scratch)));
        ctx->static_scratch = sp;
        // phi: the quadrature table (radius 128), then eq. 3.1 precomputed out to the device
        // table's radius (neighbour offsets of leaves up to side 128 stay inside it)
        const std::vector<double>& tab = phi_table(o.stencil);
        if (tab.size() != size_t(129) * 130 / 2) throw HipFailure("phi table of unexpected size");
        const Stencil& sten = stencil(o.stencil);
        PhiFar far{};
        far.C = sten.C;
        for (int k = 0; k < 3; ++k)
            for (int j = 0; j < 4; ++j) far.c[k][j] = sten.c[k][j];
        ctx->table_mem.reserve(kPhiDeviceEntries * sizeof(double));
        ctx->table_mem.reserve(sizeof(PhiFar));
        ctx->table_mem.allocate();
        ctx->phi_oct = ctx->table_mem.take<double>(kPhiDeviceEntries);
        ctx->phi_far = ctx->table_mem.take<PhiFar>(1);
        LFMM_HIP(hipMemcpy(ctx->phi_oct, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice));
        LFMM_HIP(hipMemcpy(ctx->phi_far, &far, sizeof(PhiFar), hipMemcpyHostToDevice));
        launch_phi_extend(ctx->phi_oct, 128, kPhiDeviceRadius, ctx->phi_far, nullptr);
        LFMM_HIP(hipGetLastError());
        LFMM_HIP(upload_dslots());
        LFMM_HIP(hipDeviceSynchronize());
        *out = ctx.release();
        return LFMM_OK;
    });
}

lfmm_status lfmm_ctx_destroy(lfmm_ctx* ctx) {
    if (!ctx) return LFMM_OK;
    (void)hipSetDevice(ctx->device);
    // servers first (their workers build and drop plans), then the plans still alive
    std::vector<lfmm_server*> servers;
    {
        std::lock_guard<std::mutex> lock(ctx->reg_mu);
        servers.assign(ctx->servers.begin(), ctx->servers.end());
    }
    for (lfmm_server* s : servers) lfmm_server_destroy(s);
    (void)hipDeviceSynchronize();
    std::vector<lfmm_plan*> plans;
    {
        std::lock_guard<std::mutex> lock(ctx->reg_mu);
        plans.assign(ctx->plans.begin(), ctx->plans.end());
    }
    for (lfmm_plan* p : plans) delete p;
    delete ctx;
    return LFMM_OK;
}

lfmm_status lfmm_plan_create(lfmm_ctx* ctx, int64_t n_src, const int32_t* src_xy, int64_t n_tgt,
                             const int32_t* tgt_xy, void* stream, lfmm_plan** out) {
    if (!ctx || !out || !src_xy) return fail(LFMM_E_INVAL, "null argument");
    InstanceInput in;
    in.n_src = n_src;
    in.src = src_xy;
    in.n_tgt = n_tgt;
    in.tgt = tgt_xy;
    return create_forest(ctx, 1, &in, 0, stream, out);
}

lfmm_status lfmm_plan_create_batch(lfmm_ctx* ctx, int32_t n_inst, const int64_t* n_src_host,
                                   const int32_t* const* src_xy_dev, const int64_t* n_tgt_host,
                                   const int32_t* const* tgt_xy_dev, void* stream, lfmm_plan** out) {
    if (!ctx || !out || !n_src_host || !src_xy_dev || n_inst < 1)
        return fail(LFMM_E_INVAL, "null argument or no instance");
    if (tgt_xy_dev && !n_tgt_host) return fail(LFMM_E_INVAL, "target coordinates without target counts");
    std::vector<InstanceInput> in(static_cast<size_t>(n_inst));
    for (int32_t k = 0; k < n_inst; ++k) {
        in[size_t(k)].n_src = n_src_host[k];
        in[size_t(k)].src = src_xy_dev[k];
        in[size_t(k)].n_tgt = n_tgt_host ? n_tgt_host[k] : 0;
        in[size_t(k)].tgt = tgt_xy_dev ? tgt_xy_dev[k] : nullptr;
    }
    return create_forest(ctx, n_inst, in.data(), 0, stream, out);
}

// Times every candidate N_leaf on the K point sets in[] (one plan holding all of them, every
// instance with that N_leaf) and records the fastest for the size and density class of each.
static lfmm_status autotune_forest(lfmm_ctx* ctx, int32_t K, const InstanceInput* in, int32_t n_cand, const int32_t* cand,
                                   int32_t objective, int32_t reps, void* stream, int32_t* best, double* ms) {
    return guarded([&]() -> lfmm_status {
        LFMM_HIP(hipSetDevice(ctx->device));
        hipStream_t st = as_stream(stream);
        int64_t n = 0;
        for (int32_t k = 0; k < K; ++k) n += in[k].n_src;
        Arena io(&ctx->pool);
        io.reserve(size_t(n) * sizeof(double));
        io.reserve(size_t(n) * sizeof(double));
        io.allocate();
        double* f = io.take<double>(size_t(n));
        double* u = io.take<double>(size_t(n));
        LFMM_HIP(hipMemsetAsync(f, 0, size_t(n) * sizeof(double), st));
        std::vector<const double*> fa(static_cast<size_t>(K));
        std::vector<double*> ua(static_cast<size_t>(K));
        for (int32_t k = 0, off = 0; k < K; off += int32_t(in[k].n_src), ++k) {
            fa[size_t(k)] = f + off;
            ua[size_t(k)] = u + off;
        }
        hipEvent_t e0 = nullptr, e1 = nullptr;
        LFMM_HIP(hipEventCreate(&e0));
        LFMM_HIP(hipEventCreate(&e1));
        struct Ev {
            hipEvent_t a, b;
            ~Ev() {
                (void)hipEventDestroy(a);
                (void)hipEventDestroy(b);
            }
        } guard{e0, e1};
        double best_ms = 0.0;
        std::vector<std::pair<int, int>> keys;
        for (int32_t c = 0; c < n_cand; ++c) {
            double total = 0.0;
            for (int r = 0; r < reps + 1; ++r) {   // the first round warms the operator cache
                LFMM_HIP(hipStreamSynchronize(st));
                const auto t0 = std::chrono::steady_clock::now();
                auto pl = std::make_unique<lfmm_plan>();
                pl->ctx = ctx;
                build_forest(pl.get(), K, in, cand[c], st);
                const double build_ms =
                    std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
                if (keys.empty())
                    for (int32_t k = 0; k < K; ++k)
                        keys.push_back(tune_key(pl->inst[size_t(k)].pt1 - pl->inst[size_t(k)].pt0,
                                                pl->inst[size_t(k)].D));
                LFMM_HIP(hipEventRecord(e0, st));
                run_forest(pl.get(), fa.data(), ua.data(), st);
                LFMM_HIP(hipEventRecord(e1, st));
                LFMM_HIP(hipEventSynchronize(e1));
                float exec_ms = 0.f;
                LFMM_HIP(hipEventElapsedTime(&exec_ms, e0, e1));
                if (r > 0) total += (objective == 0 ? build_ms : 0.0) + double(exec_ms);
            }
            const double t = total / reps;
            if (ms) ms[c] = t;
            if (c == 0 || t < best_ms) {
                best_ms = t;
                *best = cand[c];
            }
        }
        {
            std::lock_guard<std::mutex> lock(ctx->mu);
            for (const auto& key : keys) ctx->tuned[key] = *best;
        }
        LFMM_HIP(hipStreamSynchronize(st));
        return LFMM_OK;
    });
}

static lfmm_status check_tune_args(int32_t n_cand, const int32_t* cand, int32_t objective, int32_t reps) {
    if (!cand || n_cand < 1 || reps < 1 || (objective != 0 && objective != 1)) return fail(LFMM_E_INVAL, "bad argument");
    for (int32_t c = 0; c < n_cand; ++c)
        if (cand[c] < 1 || cand[c] > 4096) return fail(LFMM_E_INVAL, "candidates must lie in [1, 4096]");
    return LFMM_OK;
}

lfmm_status lfmm_autotune(lfmm_ctx* ctx, int64_t n, const int32_t* xy, int32_t n_cand, const int32_t* cand,
                          int32_t objective, int32_t reps, void* stream, int32_t* best, double* ms) {
    if (!ctx || !xy || !best) return fail(LFMM_E_INVAL, "bad argument");
    const lfmm_status s = check_tune_args(n_cand, cand, objective, reps);
    if (s != LFMM_OK) return s;
    if (n < 1 || n > (int64_t(1) << 30)) return fail(LFMM_E_INVAL, "n must lie in [1, 2^30]");
    InstanceInput one;
    one.n_src = n;
    one.src = xy;
    return autotune_forest(ctx, 1, &one, n_cand, cand, objective, reps, stream, best, ms);
}

lfmm_status lfmm_autotune_batch(lfmm_ctx* ctx, int32_t n_inst, const int64_t* n_host, const int32_t* const* xy_dev,
                                int32_t n_cand, const int32_t* cand, int32_t objective, int32_t reps, void* stream,
                                int32_t* best, double* ms) {
    if (!ctx || !n_host || !xy_dev || !best || n_inst < 1) return fail(LFMM_E_INVAL, "bad argument");
    const lfmm_status s = check_tune_args(n_cand, cand, objective, reps);
    if (s != LFMM_OK) return s;
    std::vector<InstanceInput> in(static_cast<size_t>(n_inst));
    int64_t total = 0;
    for (int32_t k = 0; k < n_inst; ++k) {
        if (!xy_dev[k] || n_host[k] < 1) return fail(LFMM_E_INVAL, "every instance needs points");
        in[size_t(k)].n_src = n_host[k];
        in[size_t(k)].src = xy_dev[k];
        total += n_host[k];
    }
    if (total > (int64_t(1) << 30)) return fail(LFMM_E_INVAL, "at most 2^30 points in all");
    return autotune_forest(ctx, n_inst, in.data(), n_cand, cand, objective, reps, stream, best, ms);
}

lfmm_status lfmm_execute(lfmm_plan* pl, const double* f, double* u, void* stream) {
    if (!pl || !f || !u) return fail(LFMM_E_INVAL, "null argument");
    if (pl->K != 1) return fail(LFMM_E_INVAL, "plan holds several instances: use lfmm_execute_instances");
    const double* fa[1] = {f};
    double* ua[1] = {u};
    return execute_forest(pl, fa, ua, stream, false);
}

lfmm_status lfmm_execute_sorted(lfmm_plan* pl, const double* f_sorted, double* u_sorted, void* stream) {
    if (!pl || !f_sorted || !u_sorted) return fail(LFMM_E_INVAL, "null argument");
    const double* fa[1] = {f_sorted};
    double* ua[1] = {u_sorted};
    return execute_forest(pl, fa, ua, stream, false, true);
}

lfmm_status lfmm_execute_instances(lfmm_plan* pl, const double* const* f, double* const* u, void* stream) {
    if (!pl || !f || !u) return fail(LFMM_E_INVAL, "null argument");
    for (int32_t k = 0; k < pl->K; ++k)
        if (!f[k] || !u[k]) return fail(LFMM_E_INVAL, "null load or potential pointer");
    return execute_forest(pl, f, u, stream, false);
}

lfmm_status lfmm_execute_batch(lfmm_ctx* ctx, int32_t n_plans, lfmm_plan* const* plans, const double* const* f,
                               double* const* u, void* stream) {
    if (!ctx || n_plans < 0 || (n_plans > 0 && (!plans || !f || !u))) return fail(LFMM_E_INVAL, "null argument");
    lfmm_status res = LFMM_OK;
    for (int32_t k = 0; k < n_plans; ++k) {
        if (!plans[k] || plans[k]->ctx != ctx) return fail(LFMM_E_INVAL, "plan of another context");
        lfmm_status s = lfmm_execute(plans[k], f[k], u[k], stream);
        if (s < 0) return s;
        if (s != LFMM_OK) res = s;
    }
    return res;
}

lfmm_status lfmm_plan_get_info(lfmm_plan* pl, lfmm_plan_info* out) {
    if (!pl || !out) return fail(LFMM_E_INVAL, "null argument");
    return guarded([&]() -> lfmm_status {
        LFMM_HIP(hipSetDevice(pl->ctx->device));
        std::memset(out, 0, sizeof(*out));
        const InstInfo& I0 = pl->inst[0];
        out->n_points = pl->n;
        out->n_instances = pl->K;
        out->root_bits = I0.D;
        out->leaf_level = I0.L;
        out->leaf_side = int64_t(1) << (I0.D - I0.L);
        out->rank = kRankPad;
        out->leaf_kind = 0;
        out->n_boxes = pl->nbox;
        out->n_leaves = pl->nleaf;
        // pair counts from the lists (host side, for reporting)
        const size_t nb = size_t(pl->nbox);
        std::vector<int32_t> pt0(nb), pt1(nb), nb9(nb * 9), il(nb * kNumInteractions);
        std::vector<int8_t> lev(nb);
        LFMM_HIP(hipMemcpy(pt0.data(), pl->box_pt0, nb * 4, hipMemcpyDeviceToHost));
        LFMM_HIP(hipMemcpy(pt1.data(), pl->box_pt1, nb * 4, hipMemcpyDeviceToHost));
        LFMM_HIP(hipMemcpy(nb9.data(), pl->nb9, nb * 36, hipMemcpyDeviceToHost));
        LFMM_HIP(hipMemcpy(il.data(), pl->il27, nb * 4 * kNumInteractions, hipMemcpyDeviceToHost));
        LFMM_HIP(hipMemcpy(lev.data(), pl->box_lev, nb, hipMemcpyDeviceToHost));
        int64_t near = 0, m2l = 0;
        for (int32_t g = 0; g < pl->nleaf && !pl->adaptive; ++g) {
            int64_t ns = 0;
            for (int q = 0; q < 9; ++q) {
                const int32_t s = nb9[size_t(g) * 9 + q];
                if (s >= 0) ns += pt1[size_t(s)] - pt0[size_t(s)];
            }
            near += int64_t(pt1[size_t(g)] - pt0[size_t(g)]) * ns;
        }
        for (size_t g = 0; g < nb; ++g)
            if (lev[g] >= 2)
                for (int k = 0; k < kNumInteractions; ++k) m2l += (il[g * kNumInteractions + k] >= 0);
        if (pl->adaptive) {
            // U, W, X lists: near pairs, multipole evaluations and P2L terms
            const size_t nb1 = nb + 1;
            std::vector<int32_t> off(3 * nb1), rank;
            std::vector<int32_t> ent[3];
            LFMM_HIP(hipMemcpy(off.data(), pl->list_off, off.size() * 4, hipMemcpyDeviceToHost));
            for (int r = 0; r < 3; ++r) {
                ent[r].resize(size_t(pl->list_len[r]));
                if (!ent[r].empty())
                    LFMM_HIP(hipMemcpy(ent[r].data(), pl->list_ent[r], ent[r].size() * 4, hipMemcpyDeviceToHost));
            }
            std::vector<int32_t> binst(nb);
            LFMM_HIP(hipMemcpy(binst.data(), pl->box_inst, nb * 4, hipMemcpyDeviceToHost));
            auto rank_of = [&](size_t g) {
                const InstInfo& I = pl->inst[size_t(binst[g])];
                return pl->ops[size_t(I.ops)]->host.level[size_t(I.L - lev[g])].rank;
            };
            int64_t m2p = 0, p2l = 0;
            for (size_t g = 0; g < nb; ++g) {
                const int64_t ng = pt1[g] - pt0[g];
                for (int32_t e = off[g]; e < off[g + 1]; ++e) near += ng * (pt1[size_t(ent[0][size_t(e)])] - pt0[size_t(ent[0][size_t(e)])]);
                for (int32_t e = off[nb1 + g]; e < off[nb1 + g + 1]; ++e) m2p += ng * rank_of(size_t(ent[1][size_t(e)]));
                for (int32_t e = off[2 * nb1 + g]; e < off[2 * nb1 + g + 1]; ++e)
                    p2l += int64_t(rank_of(g)) * (pt1[size_t(ent[2][size_t(e)])] - pt0[size_t(ent[2][size_t(e)])]);
            }
            out->adaptive = 1;
            out->n_leaves = pl->n_ad_leaves;
            out->m2p_terms = m2p;
            out->p2l_terms = p2l;
        }
        out->near_pairs = near;
        out->m2l_pairs = m2l;
        out->device_bytes =
            int64_t(pl->mem_small.bytes() + pl->mem_pts.bytes() + pl->mem_box.bytes() + pl->mem_ad.bytes());
        int64_t nt = 0;
        for (int32_t k = 0; k < pl->K; ++k) nt += pl->nout[size_t(k)];
        out->n_targets = nt;
        return LFMM_OK;
    });
}

lfmm_status lfmm_plan_export(lfmm_plan* pl, int32_t item, void* out, size_t* bytes) {
    if (!pl || !bytes) return fail(LFMM_E_INVAL, "null argument");
    const void* src = nullptr;
    size_t size = 0;
    const size_t nb = size_t(pl->nbox), n = size_t(pl->n), P = kRankPad;
    std::vector<int32_t> levels;
    std::vector<int8_t> roles;
    bool host = false;
    switch (item) {
        case LFMM_EXPORT_POINTS: src = pl->pts; size = n * 8; break;
        case LFMM_EXPORT_PERM: src = pl->perm; size = n * 4; break;
        case LFMM_EXPORT_LEVEL_BASE:
        case LFMM_EXPORT_LEVEL_COUNT: {
            const InstInfo& I0 = pl->inst[0];
            for (int lev = 0; lev <= I0.L; ++lev)
                levels.push_back(item == LFMM_EXPORT_LEVEL_BASE ? I0.lev_base[lev] : I0.lev_count[lev]);
            src = levels.data();
            size = levels.size() * 4;
            host = true;
            break;
        }
        case LFMM_EXPORT_BOX_KEY: src = pl->box_key; size = nb * 8; break;
        case LFMM_EXPORT_BOX_BEGIN: src = pl->box_pt0; size = nb * 4; break;
        case LFMM_EXPORT_BOX_END: src = pl->box_pt1; size = nb * 4; break;
        case LFMM_EXPORT_BOX_PARENT: src = pl->box_parent; size = nb * 4; break;
        case LFMM_EXPORT_BOX_CHILD: src = pl->box_child; size = nb * 16; break;
        case LFMM_EXPORT_INTERACTION: src = pl->il27; size = nb * kNumInteractions * 4; break;
        case LFMM_EXPORT_NEIGHBOR: src = pl->nb9; size = nb * 9 * 4; break;
        case LFMM_EXPORT_QHAT: src = pl->Q; size = nb * P * 8; break;
        case LFMM_EXPORT_UHAT: src = pl->U; size = nb * P * 8; break;
        case LFMM_EXPORT_LOADS: src = pl->fs; size = n * 8; break;
        case LFMM_EXPORT_BOX_LEVEL: src = pl->box_lev; size = nb; break;
        case LFMM_EXPORT_BOX_INSTANCE: src = pl->box_inst; size = nb * 4; break;
        case LFMM_EXPORT_BOX_ROLE:
        case LFMM_EXPORT_LIST_U:
        case LFMM_EXPORT_LIST_W:
        case LFMM_EXPORT_LIST_X: {
            if (item == LFMM_EXPORT_BOX_ROLE) {
                size = nb;
                if (pl->adaptive) {
                    src = pl->role;
                    break;
                }
                // uniform tree: the leaves (the height-0 block) and inner boxes
                roles.assign(nb, int8_t(kRoleInner));
                std::fill(roles.begin(), roles.begin() + pl->nleaf, int8_t(kRoleLeaf));
                src = roles.data();
                host = true;
                break;
            }
            if (!pl->adaptive) return fail(LFMM_E_INVAL, "list items of a plan without LFMM_FLAG_ADAPTIVE");
            const int r = item - LFMM_EXPORT_LIST_U;
            size = (nb + 1 + size_t(pl->list_len[r])) * 4;
            if (!out) break;
            if (*bytes < size) return fail(LFMM_E_INVAL, "output buffer too small");
            return guarded([&]() -> lfmm_status {
                LFMM_HIP(hipSetDevice(pl->ctx->device));
                LFMM_HIP(hipDeviceSynchronize());
                int32_t* o32 = static_cast<int32_t*>(out);
                LFMM_HIP(hipMemcpy(o32, pl->list_off + size_t(r) * (nb + 1), (nb + 1) * 4, hipMemcpyDeviceToHost));
                if (pl->list_len[r] > 0)
                    LFMM_HIP(hipMemcpy(o32 + nb + 1, pl->list_ent[r], size_t(pl->list_len[r]) * 4,
                                       hipMemcpyDeviceToHost));
                *bytes = size;
                return LFMM_OK;
            });
        }
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
        if (host) std::memcpy(out, src, size);
        else if (size) LFMM_HIP(hipMemcpy(out, src, size, hipMemcpyDeviceToHost));
        return LFMM_OK;
    });
}

lfmm_status lfmm_plan_set_timing_phases(lfmm_plan* pl, uint32_t phase_mask) {
    if (!pl) return fail(LFMM_E_INVAL, "null plan");
    if (phase_mask >> LFMM_NUM_PHASES) return fail(LFMM_E_INVAL, "phase mask names no phase");
    return guarded([&]() -> lfmm_status {
        LFMM_HIP(hipSetDevice(pl->ctx->device));
        if (phase_mask && !pl->ev[0])
            for (auto& e : pl->ev) LFMM_HIP(hipEventCreate(&e));
        pl->timing_mask = phase_mask;
        return LFMM_OK;
    });
}

lfmm_status lfmm_plan_set_timing(lfmm_plan* pl, int32_t enable) {
    return lfmm_plan_set_timing_phases(pl, enable ? (1u << LFMM_NUM_PHASES) - 1u : 0u);
}

lfmm_status lfmm_plan_phase_times(lfmm_plan* pl, double* ms) {
    if (!pl || !ms) return fail(LFMM_E_INVAL, "null argument");
    if (!pl->timed_mask) return fail(LFMM_E_INVAL, "no timed execute yet");
    return guarded([&]() -> lfmm_status {
        LFMM_HIP(hipSetDevice(pl->ctx->device));
        const uint32_t m = pl->timed_mask;
        int last = 0;   // the last event recorded closes the last timed phase
        for (int k = 0; k < LFMM_NUM_PHASES; ++k)
            if (m >> k & 1u) last = k + 1;
        LFMM_HIP(hipEventSynchronize(pl->ev[last]));
        for (int k = 0; k < LFMM_NUM_PHASES; ++k) {
            ms[k] = std::numeric_limits<double>::quiet_NaN();
            if (!(m >> k & 1u)) continue;
            float t = 0.f;
            LFMM_HIP(hipEventElapsedTime(&t, pl->ev[k], pl->ev[k + 1]));
            ms[k] = double(t);
        }
        return LFMM_OK;
    });
}

lfmm_status lfmm_plan_footprint_bytes(const lfmm_ctx* ctx, int64_t n_src, int64_t n_tgt, int32_t root_bits,
                                      size_t* out) {
    if (!ctx || !out || n_src < 0 || n_tgt < 0 || root_bits < -1 || root_bits > 31)
        return fail(LFMM_E_INVAL, "bad argument");
    if (ctx->opt.flags & LFMM_FLAG_ADAPTIVE)
        return fail(LFMM_E_UNSUPPORTED, "footprint bound of uniform trees only (context has LFMM_FLAG_ADAPTIVE)");
    // Bound on the device memory one single-instance plan holds, construction temporaries
    // included, each arena counted at the pool block that serves it (a power of two of at
    // least 64 KiB, so at most twice its size plus 64 KiB).  Level l of the tree holds at most
    // min(4^l, n) boxes and the leaves lie at a level <= D, the root box's bits.
    const int D = root_bits < 0 ? 31 : root_bits;
    const int64_t n = n_src + n_tgt;
    size_t nb = 0;
    for (int l = 0; l <= D; ++l) nb += size_t(std::min<int64_t>(l < 31 ? int64_t(1) << (2 * l) : n, n));
    const size_t nl = size_t(std::min<int64_t>(n, int64_t(nb)));
    const size_t P = kRankPad, al = 256;
    auto block = [](size_t b) { return 2 * b + (size_t(1) << 16); };
    // points: coordinates, permutation, instance, window key, loads
    const size_t pts = size_t(n) * 28 + 5 * al;
    // boxes: key, four int32 fields and a pad, level, children, neighbour and interaction lists,
    // class lists (M2L and L2L groups, four slots per box each), tiles, Q and U with their zero
    // rows, near-field groups and their 16 entries
    const size_t tiles = nb / 32 + 8 * size_t(D + 2);
    const size_t mixed = ctx->opt.precision == LFMM_MIXED        ? (nb + 1) * (P * 8 + 8) + 3 * al
                         : ctx->opt.precision == LFMM_MIXED_BF16 ? (nb + 1) * (P * 6 + 8) + 2 * al
                                                                 : 0;
    const size_t box = nb * (8 + 20 + 1 + 16 + 36 + 4 * kNumInteractions + 32) + tiles * sizeof(BoxTile) +
                       2 * (nb + 1) * P * 8 + nl * (sizeof(NearGroup) + kNearEntries * 16) + 14 * al + mixed;
    const size_t small = sizeof(InstInfo) + 64 * sizeof(OpsPtrs) + 16 + 4 * size_t(D + 2) * sizeof(BoxGroup) +
                         (nb / 64 + size_t(D + 2)) * sizeof(BoxTile) + sizeof(ExecPtrs) + 16 * al;
    // construction temporaries: concatenated points, keys and indices (two copies), common
    // levels, sort and scan scratch; then per leaf: first point, key, level, instance and one
    // scan row per level; per box: class scans
    const size_t chunks = size_t(n) / kChunk + 1;   // each: its range and box partials
    const size_t tmp = size_t(n) * (8 + 16 + 8 + 1) + radix_scratch_bytes(n) + scan_scratch_bytes(n, 1) +
                       chunks * 2 * 16 + (kMaxLevels + 10) * 4 * 4 * kLevelStatsCopies + 24 * al;
    const size_t rows = size_t(std::max(D, 1));
    const size_t tmp2 = nl * (4 + 8 + 1 + 4 + 4 * rows) + scan_scratch_bytes(int64_t(nl), int(rows)) + nb * 16 + 64 +
                        scan_scratch_bytes(int64_t(nb), 4) + 10 * al;
    *out = block(pts) + block(box) + block(small) + block(tmp) + block(tmp2);
    return LFMM_OK;
}

lfmm_status lfmm_plan_destroy(lfmm_plan* pl) {
    if (!pl) return LFMM_OK;
    (void)hipSetDevice(pl->ctx->device);
    if (pl->one_stream && !pl->use_graph) {
        // all of the plan's work was issued on its build stream: its blocks go back to the
        // context's pools once that stream passes this point, without waiting here
        try {
            const FencePtr done = std::make_shared<Fence>(pl->build_stream);
            pl->mem_small.release_after(done);
            pl->mem_pts.release_after(done);
            pl->mem_box.release_after(done);
            if (pl->h_exec) {
                pl->ctx->pinned.release_after(pl->h_exec, pl->h_exec_cls, done);
                pl->h_exec = nullptr;
            }
            delete pl;
            return LFMM_OK;
        } catch (...) {
            (void)hipGetLastError();   // no fence: wait for the device as below
        }
    }
    // kernels of this plan may still run on any stream: finish them before the blocks go
    // back to the context's pool for reuse
    (void)hipDeviceSynchronize();
    delete pl;
    return LFMM_OK;
}

lfmm_status lfmm_solve(lfmm_ctx* ctx, int64_t n, const int32_t* xy, const double* f, double* u, void* stream) {
    if (!ctx || !xy || !f || !u) return fail(LFMM_E_INVAL, "null argument");
    lfmm_plan* pl = nullptr;
    lfmm_status s = lfmm_plan_create(ctx, n, xy, 0, nullptr, stream, &pl);
    if (s != LFMM_OK) return s;
    const double* fa[1] = {f};
    double* ua[1] = {u};
    s = execute_forest(pl, fa, ua, stream, true);
    if (s >= 0) {
        const std::string warn = g_last_error;
        hipError_t e = hipStreamSynchronize(as_stream(stream));
        if (e != hipSuccess) s = fail(LFMM_E_HIP, hipGetErrorString(e));
        else if (s != LFMM_OK) g_last_error = warn;
    }
    lfmm_plan_destroy(pl);
    return s;
}

lfmm_status lfmm_solve_static(lfmm_ctx* ctx, int64_t n, const int32_t* xy, const double* f, double* u,
                              void* stream) {
    if (!ctx || !xy || !f || !u) return fail(LFMM_E_INVAL, "null argument");
    if (n < 1) return fail(LFMM_E_INVAL, "n must be at least 1");
    if (n > kStaticMaxPoints)
        return fail(LFMM_E_RANGE, "lfmm_solve_static takes at most " + std::to_string(kStaticMaxPoints) + " points");
    if (!ctx->static_scratch) return fail(LFMM_E_HIP, "no static workspace on this device");
    if (ctx->opt.flags & LFMM_FLAG_ADAPTIVE)
        return fail(LFMM_E_UNSUPPORTED, "lfmm_solve_static builds uniform trees only (context has LFMM_FLAG_ADAPTIVE)");
    std::lock_guard<std::mutex> lock(g_static_mu[ctx->device & 63]);
    return guarded([&]() -> lfmm_status {
        LFMM_HIP(hipSetDevice(ctx->device));
        hipStream_t st = as_stream(stream);
        StaticRegion reg;
        reg.base = static_cast<char*>(ctx->static_scratch);
        reg.cap = kStaticScratchBytes;
        lfmm_plan pl;
        pl.ctx = ctx;
        pl.sreg = &reg;
        InstanceInput in;
        in.n_src = n;
        in.src = xy;
        build_forest(&pl, 1, &in, 0, st);
        const double* fa[1] = {f};
        double* ua[1] = {u};
        const lfmm_status res = check_loads(ctx, 1, fa, pl.nsrc.data(), st, &reg);
        if (res < 0) return res;
        const std::string warn = g_last_error;
        run_forest(&pl, fa, ua, st);
        LFMM_HIP(hipGetLastError());
        LFMM_HIP(hipStreamSynchronize(st));
        if (res != LFMM_OK) g_last_error = warn;
        return res;
    });
}

lfmm_status lfmm_direct(lfmm_ctx* ctx, int64_t nt, const int32_t* txy, int64_t ns, const int32_t* sxy,
                        const double* f, double* u, void* stream) {
    if (!ctx || nt < 0 || ns < 0 || (nt > 0 && (!txy || !u)) || (ns > 0 && (!sxy || !f)))
        return fail(LFMM_E_INVAL, "bad argument");
    return guarded([&]() -> lfmm_status {
        LFMM_HIP(hipSetDevice(ctx->device));
        launch_direct(nt, txy, ns, sxy, f, ctx->phi_oct, ctx->phi_far, u, as_stream(stream));
        LFMM_HIP(hipGetLastError());
        return LFMM_OK;
    });
}

}  // extern "C"
