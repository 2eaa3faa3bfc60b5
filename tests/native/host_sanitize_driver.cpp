// Driver of the host-only C ABI (options, phi, operator sets, the on-disk operator cache) for
// a build of the host sources under AddressSanitizer and UndefinedBehaviorSanitizer
// (tests/test_host_sanitizers.py).  Exits non-zero on a wrong result; the sanitizers abort on
// a memory or undefined-behaviour error.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "lfmm.h"

static int check(bool ok, const char* what) {
    if (!ok) std::fprintf(stderr, "failed: %s\n", what);
    return ok ? 0 : 1;
}

int main() {
    int bad = 0;
    lfmm_options o;
    bad += check(lfmm_options_init(&o) == LFMM_OK, "options_init");
    // phi of both operators at a spread of offsets, inside and outside the tabulated octant
    std::vector<int32_t> m;
    for (int a = -300; a <= 300; a += 37)
        for (int b = -260; b <= 260; b += 29) {
            m.push_back(a);
            m.push_back(b);
        }
    const int64_t n = int64_t(m.size() / 2);
    std::vector<double> v5(static_cast<size_t>(n)), v9(static_cast<size_t>(n));
    bad += check(lfmm_host_phi(LFMM_STENCIL_5, n, m.data(), v5.data()) == LFMM_OK, "phi 5");
    bad += check(lfmm_host_phi(LFMM_STENCIL_9, n, m.data(), v9.data()) == LFMM_OK, "phi 9");
    for (int64_t i = 0; i < n; ++i) bad += check(std::isfinite(v5[size_t(i)]) && std::isfinite(v9[size_t(i)]), "finite");
    const int32_t e1[2] = {1, 0};
    double p1 = 0.0;
    bad += check(lfmm_host_phi(LFMM_STENCIL_5, 1, e1, &p1) == LFMM_OK && std::fabs(p1 + 0.25) < 1e-15, "phi(e1)");
    bad += check(lfmm_host_phi(7, 1, e1, &p1) == LFMM_E_INVAL, "bad stencil rejected");
    // operator sets of two leaf sides, every accessor, twice (the second time through the cache
    // when LFMM_CACHE_DIR is set)
    for (int rep = 0; rep < 2; ++rep)
        for (int64_t side : {8, 64}) {
            lfmm_opset* h = nullptr;
            bad += check(lfmm_host_opset_create(side, 3, &o, &h) == LFMM_OK, "opset_create");
            if (!h) return 1;
            for (int lev = 0; lev < 3; ++lev) {
                int64_t s = 0;
                int32_t r = 0;
                bad += check(lfmm_host_opset_level(h, lev, &s, &r) == LFMM_OK && r > 0, "opset_level");
                std::vector<int64_t> sk(size_t(2 * r));
                bad += check(lfmm_host_opset_skeleton(h, lev, sk.data()) == LFMM_OK, "opset_skeleton");
                if (lev > 0) {
                    int64_t s0 = 0;
                    int32_t r0 = 0;
                    lfmm_host_opset_level(h, lev - 1, &s0, &r0);
                    std::vector<double> t(size_t(r) * size_t(r0));
                    for (int c = 0; c < 4; ++c) bad += check(lfmm_host_opset_ofo(h, lev, c, t.data()) == LFMM_OK, "ofo");
                }
            }
            int64_t s = 0;
            int32_t r = 0;
            lfmm_host_opset_level(h, 0, &s, &r);
            std::vector<double> leaf(size_t(r) * size_t(side * side));
            bad += check(lfmm_host_opset_leaf(h, leaf.data()) == LFMM_OK, "opset_leaf");
            bad += check(lfmm_host_opset_level(h, 9, &s, &r) == LFMM_E_INVAL, "bad level rejected");
            bad += check(lfmm_host_opset_destroy(h) == LFMM_OK, "opset_destroy");
        }
    o.max_rank = 40;
    lfmm_opset* h = nullptr;
    bad += check(lfmm_host_opset_create(16, 2, &o, &h) == LFMM_E_INVAL && h == nullptr, "bad options rejected");
    std::printf("host driver: %s\n", bad ? "FAILED" : "ok");
    return bad ? 1 : 0;
}
