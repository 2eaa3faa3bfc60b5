// On-disk cache of the per-leaf-side operator sets (Section 8.1 precompute).  Building the
// skeletons and translation operators of one leaf side takes up to a second on the host; with
// LFMM_CACHE_DIR set, a set is stored there the first time it is built and read back by later
// processes.  A file holds a text key line (format version, lattice operator, every parameter
// of the build) and the set's numbers in native binary; any mismatch, short read or
// inconsistent size makes the cache miss and the set is rebuilt (and the file rewritten).
// Files are written to a temporary name and renamed, so readers never see a partial file.
#include "host_math.h"

#include <cstdio>
#include <cstdlib>
#include <sstream>
#include <string>
#include <unistd.h>

namespace lfmm {

namespace {

uint64_t fnv1a(const void* data, size_t n, uint64_t h = 1469598103934665603ull) {
    const unsigned char* c = static_cast<const unsigned char*>(data);
    for (size_t i = 0; i < n; ++i) h = (h ^ c[i]) * 1099511628211ull;
    return h;
}

uint64_t fnv1a(const std::string& s) { return fnv1a(s.data(), s.size()); }

// The key names every input of the build, the phi table included (by a hash of its bytes), so
// that a library whose phi differs never reads another's operators.
std::string cache_key(int64_t leaf_side, int nlevels, const OperatorParams& p) {
    const std::vector<double>& tab = phi_table(p.stencil);
    std::ostringstream k;
    k.precision(17);
    k << "lfmm-opset-v1 stencil " << p.stencil << " phi " << std::hex << fnv1a(tab.data(), tab.size() * 8)
      << std::dec << " eps " << p.eps << " proxy " << p.proxy_per_edge << " maxrank " << p.max_rank << " dense "
      << p.dense_leaf_max << " side " << leaf_side << " levels " << nlevels;
    return k.str();
}

struct Writer {
    FILE* f;
    bool ok = true;
    template <class T>
    void put(const T& v) { ok = ok && std::fwrite(&v, sizeof(T), 1, f) == 1; }
    template <class T>
    void vec(const std::vector<T>& v) {
        put(uint64_t(v.size()));
        ok = ok && (v.empty() || std::fwrite(v.data(), sizeof(T), v.size(), f) == v.size());
    }
    void mat(const Mat& m) {
        put(int32_t(m.rows));
        put(int32_t(m.cols));
        vec(m.a);
    }
};

struct Reader {
    FILE* f;
    bool ok = true;
    template <class T>
    void get(T& v) { ok = ok && std::fread(&v, sizeof(T), 1, f) == 1; }
    template <class T>
    void vec(std::vector<T>& v, uint64_t max_items) {
        uint64_t n = 0;
        get(n);
        ok = ok && n <= max_items;
        if (!ok) return;
        v.resize(size_t(n));
        ok = n == 0 || std::fread(v.data(), sizeof(T), size_t(n), f) == n;
    }
    void mat(Mat& m) {
        int32_t r = 0, c = 0;
        get(r);
        get(c);
        ok = ok && r >= 0 && c >= 0 && int64_t(r) * c <= (int64_t(1) << 28);
        if (!ok) return;
        m.rows = r;
        m.cols = c;
        vec(m.a, uint64_t(r) * uint64_t(c));
        ok = ok && m.a.size() == size_t(r) * size_t(c);
    }
};

void write_set(FILE* f, const std::string& key, const OperatorSet& s, bool& ok) {
    Writer w{f};
    w.ok = std::fprintf(f, "%s\n", key.c_str()) > 0;
    w.put(s.eps);
    w.put(s.leaf_side);
    w.put(int32_t(s.nlevels));
    w.put(int32_t(s.max_rank));
    for (const LevelOps& lv : s.level) {
        w.put(lv.side);
        w.put(int32_t(lv.rank));
        w.vec(lv.skel);
        for (const Mat& m : lv.ofo) w.mat(m);
    }
    w.put(s.leaf.side);
    w.put(int32_t(s.leaf.dense ? 1 : 0));
    w.mat(s.leaf.T);
    w.mat(s.leaf.Pi);
    w.vec(s.leaf.proxy);
    ok = w.ok;
}

bool read_set(FILE* f, const std::string& key, int64_t leaf_side, int nlevels, OperatorSet& s) {
    std::string line;
    for (int c = std::fgetc(f); c != EOF && c != '\n' && line.size() < 4096; c = std::fgetc(f)) line.push_back(char(c));
    if (line != key) return false;
    Reader r{f};
    int32_t nl = 0, mr = 0;
    r.get(s.eps);
    r.get(s.leaf_side);
    r.get(nl);
    r.get(mr);
    if (!r.ok || s.leaf_side != leaf_side || nl != nlevels) return false;
    s.nlevels = nl;
    s.max_rank = mr;
    s.level.assign(size_t(nl), LevelOps{});
    for (LevelOps& lv : s.level) {
        int32_t rank = 0;
        r.get(lv.side);
        r.get(rank);
        lv.rank = rank;
        r.vec(lv.skel, 2 * 4096);
        for (Mat& m : lv.ofo) r.mat(m);
        if (!r.ok || rank < 0 || lv.skel.size() != size_t(2 * rank)) return false;
    }
    int32_t dense = 0;
    r.get(s.leaf.side);
    r.get(dense);
    s.leaf.dense = dense != 0;
    r.mat(s.leaf.T);
    r.mat(s.leaf.Pi);
    r.vec(s.leaf.proxy, 1 << 20);
    return r.ok && std::fgetc(f) == EOF;
}

}  // namespace

OperatorSet build_operators(int64_t leaf_side, int nlevels, const OperatorParams& p) {
    const char* dir = std::getenv("LFMM_CACHE_DIR");
    if (!dir || !*dir) return build_operators_uncached(leaf_side, nlevels, p);
    const std::string key = cache_key(leaf_side, nlevels, p);
    char name[64];
    std::snprintf(name, sizeof(name), "/opset_%016llx.bin", static_cast<unsigned long long>(fnv1a(key)));
    const std::string path = std::string(dir) + name;
    if (FILE* f = std::fopen(path.c_str(), "rb")) {
        OperatorSet s;
        const bool hit = read_set(f, key, leaf_side, nlevels, s);
        std::fclose(f);
        if (hit) return s;
    }
    OperatorSet s = build_operators_uncached(leaf_side, nlevels, p);
    const std::string tmp = path + ".tmp." + std::to_string(long(getpid()));
    if (FILE* f = std::fopen(tmp.c_str(), "wb")) {
        bool ok = false;
        write_set(f, key, s, ok);
        ok = (std::fclose(f) == 0) && ok;
        if (!ok || std::rename(tmp.c_str(), path.c_str()) != 0) std::remove(tmp.c_str());
    }
    return s;
}

}  // namespace lfmm
