// The two applications of the lattice convolution in Section 10, on top of resident plans:
//
//  * a lattice with inclusions (Section 10.1): (A + B) u = 0, u -> v = c1 m1 + c2 m2 at
//    infinity, reduced to mu + B S mu = -B S B v on the nodes the modified bars touch
//    (eq. 10.4), then u = v - S (B v + mu);
//  * a Dirichlet problem on a finite lattice (Section 10.2): u = D q with the double-layer-like
//    operator D of eq. 10.6 (a dipole across each boundary node along its outward normal), q
//    from D q = g on the boundary (eq. 10.7).
//
// S and D are applied by lattice FMM plans (the sources of D are the dipole ends); the dense
// equations are solved by restarted GMRES whose vector operations (classical Gram-Schmidt run
// twice, updates, norms) are kernels on the device.  The small Hessenberg least-squares
// problem (Givens rotations) is solved on the host from one read-back per iteration.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <limits>
#include <memory>
#include <string>
#include <unordered_map>
#include <vector>

#include "api_common.h"
#include "lfmm.h"

using namespace lfmm;

namespace {

constexpr int kThreads = 256;
constexpr int kDotBlocks = 256;

inline unsigned blocks_for(int64_t n) { return unsigned(std::max<int64_t>(1, (n + kThreads - 1) / kThreads)); }

// ---- vector kernels -------------------------------------------------------------------------

// Partial dot products of w with the k vectors V[j] (stride ldv) over fixed slices of [0, n),
// one slice per block, reduced in a fixed order: part[j * kDotBlocks + block].
__global__ __launch_bounds__(kThreads) void k_dots_part(const double* V, int64_t ldv, int k, const double* w,
                                                        int64_t n, double* part) {
    __shared__ double red[kThreads];
    const int64_t per = (n + kDotBlocks - 1) / kDotBlocks;
    const int64_t i0 = int64_t(blockIdx.x) * per, i1 = min(n, i0 + per);
    for (int j = 0; j < k; ++j) {
        const double* v = V + size_t(j) * size_t(ldv);
        double s = 0.0;
        for (int64_t i = i0 + threadIdx.x; i < i1; i += kThreads) s += v[i] * w[i];
        red[threadIdx.x] = s;
        __syncthreads();
        for (int o = kThreads / 2; o > 0; o >>= 1) {
            if (int(threadIdx.x) < o) red[threadIdx.x] += red[threadIdx.x + o];
            __syncthreads();
        }
        if (threadIdx.x == 0) part[size_t(j) * kDotBlocks + blockIdx.x] = red[0];
        __syncthreads();
    }
}

__global__ void k_dots_final(const double* part, int k, double* out) {
    const int j = int(blockIdx.x) * blockDim.x + int(threadIdx.x);
    if (j >= k) return;
    double s = 0.0;
    for (int b = 0; b < kDotBlocks; ++b) s += part[size_t(j) * kDotBlocks + b];
    out[j] = s;
}

// w += sign * sum_j h[j] V[j]
__global__ void k_combine(const double* V, int64_t ldv, int k, const double* h, double sign, double* w, int64_t n) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int j = 0; j < k; ++j) s += h[j] * V[size_t(j) * size_t(ldv) + size_t(i)];
    w[i] += sign * s;
}

__global__ void k_fill(double* out, double v, int64_t n) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) out[i] = v;
}

__global__ void k_scale_copy(const double* a, double s, double* out, int64_t n) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) out[i] = s * a[i];
}

// out = a - b
__global__ void k_sub(const double* a, const double* b, double* out, int64_t n) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) out[i] = a[i] - b[i];
}

// ---- operators of Section 10 ------------------------------------------------------------------

// out[i] = cb * base[i] + cs * sum over the bars at node i of delta (s[i] - s[other end])
// (B applied to s, Section 10.1: each bar adds delta (e_a - e_b)(e_a - e_b)^T); base may be null
__global__ void k_bars(const int32_t* rowptr, const int32_t* col, const double* dlt, const double* s,
                       const double* base, double cb, double cs, double* out, int64_t n) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double si = s[i];
    double acc = 0.0;
    for (int32_t e = rowptr[i]; e < rowptr[i + 1]; ++e) acc += dlt[e] * (si - s[col[e]]);
    out[i] = (base ? cb * base[i] : 0.0) + cs * acc;
}

// v(m) = c1 m1 + c2 m2 at the points xy (the far-field condition of eq. 10.2)
__global__ void k_linear(const int2* xy, double c1, double c2, double* out, int64_t n) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) out[i] = c1 * double(xy[i].x) + c2 * double(xy[i].y);
}

// u[i] = c1 x_i + c2 y_i - u[i]  (u = v - S(...) in place)
__global__ void k_linear_minus(const int2* xy, double c1, double c2, double* u, int64_t n) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) u[i] = c1 * double(xy[i].x) + c2 * double(xy[i].y) - u[i];
}

// loads of the dipoles of D: +q at n + nu(n) (first half), -q at n (second half)
__global__ void k_dipole_loads(const double* q, double* f2, int64_t n) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) {
        f2[i] = q[i];
        f2[n + i] = -q[i];
    }
}

// ---- device buffers ---------------------------------------------------------------------------

struct HipError {
    std::string msg;
};

#define SOLVER_HIP(call)                                                                         \
    do {                                                                                         \
        hipError_t e_ = (call);                                                                  \
        if (e_ != hipSuccess) throw HipError{std::string(#call) + ": " + hipGetErrorString(e_)}; \
    } while (0)

template <class T>
struct DevBuf {
    T* p = nullptr;
    size_t n = 0;
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    void alloc(size_t count) {
        free();
        if (count == 0) count = 1;
        SOLVER_HIP(hipMalloc(reinterpret_cast<void**>(&p), count * sizeof(T)));
        n = count;
    }
    void free() {
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
    }
    ~DevBuf() { free(); }
};

struct Status {
    lfmm_status s;
    std::string msg;
};

// ---- restarted GMRES ----------------------------------------------------------------------------

// Solves A x = b (device vectors of n) by GMRES(m) with x0 = 0; apply(in, out) enqueues A in
// on the stream.  Stops when the relative residual |b - A x| / |b| estimated by the Givens
// recurrence is <= tol, or after max_iter iterations; then reports the true relative residual.
struct Gmres {
    int64_t n = 0;
    int m = 0;
    DevBuf<double> V, w, part, h, r;

    void setup(int64_t n_, int m_) {
        n = n_;
        m = m_;
        V.alloc(size_t(m + 1) * size_t(n));
        w.alloc(size_t(n));
        r.alloc(size_t(n));
        part.alloc(size_t(m + 2) * kDotBlocks);
        h.alloc(size_t(2 * (m + 2)));
    }

    // out[0..k) = V[0..k)^T x
    void dots(const double* Vb, int k, const double* x, double* out, hipStream_t st) {
        hipLaunchKernelGGL(k_dots_part, dim3(kDotBlocks), dim3(kThreads), 0, st, Vb, n, k, x, n, part.p);
        hipLaunchKernelGGL(k_dots_final, dim3(1), dim3(64), 0, st, part.p, k, out);
    }

    double norm(const double* x, hipStream_t st) {
        dots(x, 1, x, h.p, st);
        double v = 0.0;
        SOLVER_HIP(hipMemcpyAsync(&v, h.p, sizeof(double), hipMemcpyDeviceToHost, st));
        SOLVER_HIP(hipStreamSynchronize(st));
        return std::sqrt(std::max(v, 0.0));
    }

    lfmm_solver_stats run(const std::function<void(const double*, double*)>& apply, const double* b, double* x,
                          double tol, int max_iter, hipStream_t st) {
        lfmm_solver_stats out{};
        hipLaunchKernelGGL(k_fill, dim3(blocks_for(n)), dim3(kThreads), 0, st, x, 0.0, n);
        const double bn = norm(b, st);
        if (bn == 0.0) {
            out.converged = 1;
            return out;
        }
        std::vector<double> H(size_t(m + 1) * m), cs(m), sn(m), g(m + 1), hv(size_t(2 * (m + 2)));
        auto Hat = [&](int i, int j) -> double& { return H[size_t(i) * m + size_t(j)]; };
        SOLVER_HIP(hipMemcpyAsync(r.p, b, size_t(n) * sizeof(double), hipMemcpyDeviceToDevice, st));
        double beta = bn;
        int iters = 0;
        bool done = false;
        while (!done) {
            hipLaunchKernelGGL(k_scale_copy, dim3(blocks_for(n)), dim3(kThreads), 0, st, r.p, 1.0 / beta, V.p, n);
            std::fill(g.begin(), g.end(), 0.0);
            g[0] = beta;
            int j = 0;
            for (; j < m; ++j) {
                double* vj = V.p + size_t(j) * size_t(n);
                apply(vj, w.p);
                // classical Gram-Schmidt, twice: h = V^T w; w -= V h (both passes summed); the
                // two coefficient sets and |w|^2 come back in one read
                double* h1 = h.p;
                double* h2 = h.p + (m + 2);
                dots(V.p, j + 1, w.p, h1, st);
                hipLaunchKernelGGL(k_combine, dim3(blocks_for(n)), dim3(kThreads), 0, st, V.p, n, j + 1, h1, -1.0,
                                   w.p, n);
                dots(V.p, j + 1, w.p, h2, st);
                hipLaunchKernelGGL(k_combine, dim3(blocks_for(n)), dim3(kThreads), 0, st, V.p, n, j + 1, h2, -1.0,
                                   w.p, n);
                dots(w.p, 1, w.p, h.p + (2 * m + 3), st);
                SOLVER_HIP(hipMemcpyAsync(hv.data(), h.p, hv.size() * sizeof(double), hipMemcpyDeviceToHost, st));
                SOLVER_HIP(hipStreamSynchronize(st));
                SOLVER_HIP(hipGetLastError());
                const double wn = std::sqrt(std::max(hv[size_t(2 * m + 3)], 0.0));
                for (int i = 0; i <= j; ++i) Hat(i, j) = hv[size_t(i)] + hv[size_t(m + 2 + i)];
                Hat(j + 1, j) = wn;
                if (wn > 0.0)
                    hipLaunchKernelGGL(k_scale_copy, dim3(blocks_for(n)), dim3(kThreads), 0, st, w.p, 1.0 / wn,
                                       V.p + size_t(j + 1) * size_t(n), n);
                // previous rotations, then a new one that zeroes H(j+1, j)
                for (int i = 0; i < j; ++i) {
                    const double a = Hat(i, j), c = Hat(i + 1, j);
                    Hat(i, j) = cs[size_t(i)] * a + sn[size_t(i)] * c;
                    Hat(i + 1, j) = -sn[size_t(i)] * a + cs[size_t(i)] * c;
                }
                const double a = Hat(j, j), c = Hat(j + 1, j);
                const double rho = std::hypot(a, c);
                cs[size_t(j)] = rho > 0.0 ? a / rho : 1.0;
                sn[size_t(j)] = rho > 0.0 ? c / rho : 0.0;
                Hat(j, j) = rho;
                Hat(j + 1, j) = 0.0;
                g[size_t(j) + 1] = -sn[size_t(j)] * g[size_t(j)];
                g[size_t(j)] = cs[size_t(j)] * g[size_t(j)];
                ++iters;
                if (std::fabs(g[size_t(j) + 1]) <= tol * bn || iters >= max_iter || wn == 0.0) {
                    ++j;
                    done = true;
                    break;
                }
            }
            if (!done) j = m;
            // y = H(0..j, 0..j)^-1 g; x += V y
            std::vector<double> y(size_t(j), 0.0);
            for (int i = j - 1; i >= 0; --i) {
                double s = g[size_t(i)];
                for (int k = i + 1; k < j; ++k) s -= Hat(i, k) * y[size_t(k)];
                y[size_t(i)] = Hat(i, i) != 0.0 ? s / Hat(i, i) : 0.0;
            }
            SOLVER_HIP(hipMemcpyAsync(h.p, y.data(), size_t(j) * sizeof(double), hipMemcpyHostToDevice, st));
            hipLaunchKernelGGL(k_combine, dim3(blocks_for(n)), dim3(kThreads), 0, st, V.p, n, j, h.p, 1.0, x, n);
            // true residual r = b - A x (also the next cycle's start)
            apply(x, w.p);
            hipLaunchKernelGGL(k_sub, dim3(blocks_for(n)), dim3(kThreads), 0, st, b, w.p, r.p, n);
            beta = norm(r.p, st);
            if (beta <= tol * bn) done = true;
            if (iters >= max_iter) done = true;
        }
        out.iterations = iters;
        out.rel_residual = beta / bn;
        out.converged = out.rel_residual <= tol ? 1 : 0;
        return out;
    }
};

lfmm_status check_solver_options(const lfmm_solver_options* o, double* tol, int* max_iter, int* restart) {
    *tol = 1e-12;
    *max_iter = 500;
    *restart = 50;
    if (!o) return LFMM_OK;
    if (o->tol > 0.0) *tol = o->tol;
    if (o->max_iter > 0) *max_iter = o->max_iter;
    if (o->restart > 0) *restart = o->restart;
    if (!(*tol < 1.0) || *restart > 512 || *max_iter > 1000000)
        return fail(LFMM_E_INVAL, "solver options: tol in (0, 1), restart <= 512, max_iter <= 1e6");
    return LFMM_OK;
}

template <class F>
lfmm_status run_guarded(F&& f) {
    (void)hipGetLastError();
    try {
        return f();
    } catch (const HipError& e) {
        return fail(LFMM_E_HIP, e.msg);
    } catch (const Status& e) {
        return fail(e.s, e.msg);
    } catch (const std::bad_alloc&) {
        return fail(LFMM_E_NOMEM, "host allocation failed");
    }
}

void check(lfmm_status s) {
    if (s < 0) throw Status{s, lfmm_last_error()};
}

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

}  // namespace

// ---- lattice with inclusions ----------------------------------------------------------------------

struct lfmm_inclusions {
    lfmm_ctx* ctx = nullptr;
    int device = 0;
    int64_t nn = 0;                       // nodes touched by the bars (Omega_inc)
    std::vector<int32_t> nodes;           // host copy, [nn][2]
    DevBuf<int32_t> xy, rowptr, col;
    DevBuf<double> dlt, v, s, t;
    lfmm_plan* plan = nullptr;            // the nodes, targets = sources: S on Omega_inc
    ~lfmm_inclusions() {
        if (plan) lfmm_plan_destroy(plan);
    }
};

struct lfmm_dirichlet {
    lfmm_ctx* ctx = nullptr;
    int device = 0;
    int64_t n = 0;                        // boundary nodes
    DevBuf<int32_t> src;                  // [2n][2]: n + nu(n) first, then n
    DevBuf<int32_t> gam;                  // [n][2]
    DevBuf<double> f2;                    // dipole loads
    lfmm_plan* plan = nullptr;            // sources: the dipole ends; targets: the boundary
    ~lfmm_dirichlet() {
        if (plan) lfmm_plan_destroy(plan);
    }
};

extern "C" {

lfmm_status lfmm_inclusions_create(lfmm_ctx* ctx, int64_t n_bars, const int32_t* bars, const double* delta,
                                   void* stream, lfmm_inclusions** out) {
    if (!ctx || !bars || !delta || !out || n_bars < 1) return fail(LFMM_E_INVAL, "null argument or no bar");
    if (n_bars > (int64_t(1) << 28)) return fail(LFMM_E_INVAL, "too many bars");
    *out = nullptr;
    for (int64_t k = 0; k < n_bars; ++k) {
        if (!std::isfinite(delta[k])) return fail(LFMM_E_INVAL, "non-finite conductance change");
        if (bars[4 * k] == bars[4 * k + 2] && bars[4 * k + 1] == bars[4 * k + 3])
            return fail(LFMM_E_INVAL, "a bar joins a node to itself");
    }
    return run_guarded([&]() -> lfmm_status {
        auto inc = std::make_unique<lfmm_inclusions>();
        inc->ctx = ctx;
        inc->device = ctx_device(ctx);
        SOLVER_HIP(hipSetDevice(inc->device));
        // nodes in first-appearance order; per node its bars as (other end, delta)
        std::unordered_map<uint64_t, int32_t> index;
        index.reserve(size_t(2 * n_bars));
        std::vector<int32_t> ends(size_t(2 * n_bars));
        for (int64_t k = 0; k < 2 * n_bars; ++k) {
            const uint64_t key = (uint64_t(uint32_t(bars[2 * k])) << 32) | uint32_t(bars[2 * k + 1]);
            auto it = index.find(key);
            if (it == index.end()) {
                it = index.emplace(key, int32_t(inc->nodes.size() / 2)).first;
                inc->nodes.push_back(bars[2 * k]);
                inc->nodes.push_back(bars[2 * k + 1]);
            }
            ends[size_t(k)] = it->second;
        }
        const int64_t nn = int64_t(inc->nodes.size() / 2);
        inc->nn = nn;
        std::vector<int32_t> rp(size_t(nn) + 1, 0), cl(size_t(2 * n_bars));
        std::vector<double> dl(size_t(2 * n_bars));
        for (int64_t k = 0; k < n_bars; ++k) {
            ++rp[size_t(ends[size_t(2 * k)]) + 1];
            ++rp[size_t(ends[size_t(2 * k + 1)]) + 1];
        }
        for (int64_t i = 0; i < nn; ++i) rp[size_t(i) + 1] += rp[size_t(i)];
        std::vector<int32_t> fill(rp.begin(), rp.end() - 1);
        for (int64_t k = 0; k < n_bars; ++k) {
            const int32_t a = ends[size_t(2 * k)], b = ends[size_t(2 * k + 1)];
            cl[size_t(fill[size_t(a)])] = b;
            dl[size_t(fill[size_t(a)]++)] = delta[k];
            cl[size_t(fill[size_t(b)])] = a;
            dl[size_t(fill[size_t(b)]++)] = delta[k];
        }
        inc->xy.alloc(size_t(2 * nn));
        inc->rowptr.alloc(size_t(nn) + 1);
        inc->col.alloc(cl.size());
        inc->dlt.alloc(dl.size());
        inc->v.alloc(size_t(nn));
        inc->s.alloc(size_t(nn));
        inc->t.alloc(size_t(nn));
        SOLVER_HIP(hipMemcpy(inc->xy.p, inc->nodes.data(), size_t(2 * nn) * 4, hipMemcpyHostToDevice));
        SOLVER_HIP(hipMemcpy(inc->rowptr.p, rp.data(), rp.size() * 4, hipMemcpyHostToDevice));
        SOLVER_HIP(hipMemcpy(inc->col.p, cl.data(), cl.size() * 4, hipMemcpyHostToDevice));
        SOLVER_HIP(hipMemcpy(inc->dlt.p, dl.data(), dl.size() * 8, hipMemcpyHostToDevice));
        check(lfmm_plan_create(ctx, nn, inc->xy.p, 0, nullptr, stream, &inc->plan));
        *out = inc.release();
        return LFMM_OK;
    });
}

lfmm_status lfmm_inclusions_nodes(const lfmm_inclusions* inc, int64_t* n_nodes, int32_t* nodes_xy_host) {
    if (!inc || !n_nodes) return fail(LFMM_E_INVAL, "null argument");
    *n_nodes = inc->nn;
    if (nodes_xy_host) std::memcpy(nodes_xy_host, inc->nodes.data(), inc->nodes.size() * sizeof(int32_t));
    return LFMM_OK;
}

lfmm_status lfmm_inclusions_solve(lfmm_inclusions* inc, double c1, double c2, const lfmm_solver_options* opt,
                                  double* mu_dev, lfmm_solver_stats* stats, void* stream) {
    if (!inc || !mu_dev) return fail(LFMM_E_INVAL, "null argument");
    if (!std::isfinite(c1) || !std::isfinite(c2)) return fail(LFMM_E_INVAL, "non-finite field");
    double tol = 0.0;
    int max_iter = 0, restart = 0;
    lfmm_status s = check_solver_options(opt, &tol, &max_iter, &restart);
    if (s != LFMM_OK) return s;
    return run_guarded([&]() -> lfmm_status {
        SOLVER_HIP(hipSetDevice(inc->device));
        hipStream_t st = as_stream(stream);
        const int64_t nn = inc->nn;
        const unsigned gb = blocks_for(nn);
        const int2* xy = reinterpret_cast<const int2*>(inc->xy.p);
        // right-hand side of eq. 10.4: -B S B v
        DevBuf<double> rhs;
        rhs.alloc(size_t(nn));
        hipLaunchKernelGGL(k_linear, dim3(gb), dim3(kThreads), 0, st, xy, c1, c2, inc->v.p, nn);
        hipLaunchKernelGGL(k_bars, dim3(gb), dim3(kThreads), 0, st, inc->rowptr.p, inc->col.p, inc->dlt.p, inc->v.p,
                           nullptr, 0.0, 1.0, inc->t.p, nn);
        check(lfmm_execute(inc->plan, inc->t.p, inc->s.p, stream));
        hipLaunchKernelGGL(k_bars, dim3(gb), dim3(kThreads), 0, st, inc->rowptr.p, inc->col.p, inc->dlt.p, inc->s.p,
                           nullptr, 0.0, -1.0, rhs.p, nn);
        // operator: mu -> mu + B S mu
        auto apply = [&](const double* in, double* o) {
            check(lfmm_execute(inc->plan, in, inc->s.p, stream));
            hipLaunchKernelGGL(k_bars, dim3(gb), dim3(kThreads), 0, st, inc->rowptr.p, inc->col.p, inc->dlt.p,
                               inc->s.p, in, 1.0, 1.0, o, nn);
        };
        Gmres gm;
        gm.setup(nn, std::min<int>(restart, int(std::max<int64_t>(nn, 1))));
        const lfmm_solver_stats r = gm.run(apply, rhs.p, mu_dev, tol, max_iter, st);
        SOLVER_HIP(hipStreamSynchronize(st));
        if (stats) *stats = r;
        return LFMM_OK;
    });
}

lfmm_status lfmm_inclusions_potential(lfmm_inclusions* inc, double c1, double c2, const double* mu_dev,
                                      int64_t n_tgt, const int32_t* tgt_xy_dev, double* u_dev, void* stream) {
    if (!inc || !mu_dev || !tgt_xy_dev || !u_dev || n_tgt < 1) return fail(LFMM_E_INVAL, "null argument or no target");
    return run_guarded([&]() -> lfmm_status {
        SOLVER_HIP(hipSetDevice(inc->device));
        hipStream_t st = as_stream(stream);
        const int64_t nn = inc->nn;
        const unsigned gb = blocks_for(nn);
        // loads B v + mu on the nodes, their field at the targets, u = v - that field
        hipLaunchKernelGGL(k_linear, dim3(gb), dim3(kThreads), 0, st, reinterpret_cast<const int2*>(inc->xy.p), c1, c2,
                           inc->v.p, nn);
        hipLaunchKernelGGL(k_bars, dim3(gb), dim3(kThreads), 0, st, inc->rowptr.p, inc->col.p, inc->dlt.p, inc->v.p,
                           mu_dev, 1.0, 1.0, inc->t.p, nn);
        lfmm_plan* pt = nullptr;
        check(lfmm_plan_create(inc->ctx, nn, inc->xy.p, n_tgt, tgt_xy_dev, stream, &pt));
        lfmm_status s = lfmm_execute(pt, inc->t.p, u_dev, stream);
        lfmm_plan_destroy(pt);
        check(s);
        hipLaunchKernelGGL(k_linear_minus, dim3(blocks_for(n_tgt)), dim3(kThreads), 0, st,
                           reinterpret_cast<const int2*>(tgt_xy_dev), c1, c2, u_dev, n_tgt);
        SOLVER_HIP(hipGetLastError());
        return LFMM_OK;
    });
}

lfmm_status lfmm_inclusions_destroy(lfmm_inclusions* inc) {
    if (!inc) return LFMM_OK;
    (void)hipSetDevice(inc->device);
    (void)hipDeviceSynchronize();
    delete inc;
    return LFMM_OK;
}

// ---- Dirichlet problem ------------------------------------------------------------------------------

lfmm_status lfmm_dirichlet_create(lfmm_ctx* ctx, int64_t n, const int32_t* gamma_xy, const int8_t* normal,
                                  void* stream, lfmm_dirichlet** out) {
    if (!ctx || !gamma_xy || !normal || !out || n < 1) return fail(LFMM_E_INVAL, "null argument or no boundary node");
    if (n > (int64_t(1) << 28)) return fail(LFMM_E_INVAL, "too many boundary nodes");
    *out = nullptr;
    static const int32_t step[4][2] = {{1, 0}, {-1, 0}, {0, 1}, {0, -1}};
    std::vector<int32_t> src(size_t(4 * n));
    for (int64_t i = 0; i < n; ++i) {
        const int c = normal[i];
        if (c < 0 || c > 3) return fail(LFMM_E_INVAL, "normal codes are 0..3 (+x, -x, +y, -y)");
        const int64_t x = int64_t(gamma_xy[2 * i]) + step[c][0], y = int64_t(gamma_xy[2 * i + 1]) + step[c][1];
        if (x < INT32_MIN || x > INT32_MAX || y < INT32_MIN || y > INT32_MAX)
            return fail(LFMM_E_RANGE, "a normal step leaves the int32 lattice");
        src[size_t(2 * i)] = int32_t(x);
        src[size_t(2 * i + 1)] = int32_t(y);
        src[size_t(2 * (n + i))] = gamma_xy[2 * i];
        src[size_t(2 * (n + i) + 1)] = gamma_xy[2 * i + 1];
    }
    return run_guarded([&]() -> lfmm_status {
        auto dir = std::make_unique<lfmm_dirichlet>();
        dir->ctx = ctx;
        dir->device = ctx_device(ctx);
        dir->n = n;
        SOLVER_HIP(hipSetDevice(dir->device));
        dir->src.alloc(size_t(4 * n));
        dir->gam.alloc(size_t(2 * n));
        dir->f2.alloc(size_t(2 * n));
        SOLVER_HIP(hipMemcpy(dir->src.p, src.data(), src.size() * 4, hipMemcpyHostToDevice));
        SOLVER_HIP(hipMemcpy(dir->gam.p, gamma_xy, size_t(2 * n) * 4, hipMemcpyHostToDevice));
        check(lfmm_plan_create(ctx, 2 * n, dir->src.p, n, dir->gam.p, stream, &dir->plan));
        *out = dir.release();
        return LFMM_OK;
    });
}

lfmm_status lfmm_dirichlet_apply(lfmm_dirichlet* dir, const double* q_dev, double* out_dev, void* stream) {
    if (!dir || !q_dev || !out_dev) return fail(LFMM_E_INVAL, "null argument");
    return run_guarded([&]() -> lfmm_status {
        SOLVER_HIP(hipSetDevice(dir->device));
        hipLaunchKernelGGL(k_dipole_loads, dim3(blocks_for(dir->n)), dim3(kThreads), 0, as_stream(stream), q_dev,
                           dir->f2.p, dir->n);
        check(lfmm_execute(dir->plan, dir->f2.p, out_dev, stream));
        SOLVER_HIP(hipGetLastError());
        return LFMM_OK;
    });
}

lfmm_status lfmm_dirichlet_solve(lfmm_dirichlet* dir, const double* g_dev, const lfmm_solver_options* opt,
                                 double* q_dev, lfmm_solver_stats* stats, void* stream) {
    if (!dir || !g_dev || !q_dev) return fail(LFMM_E_INVAL, "null argument");
    double tol = 0.0;
    int max_iter = 0, restart = 0;
    lfmm_status s = check_solver_options(opt, &tol, &max_iter, &restart);
    if (s != LFMM_OK) return s;
    return run_guarded([&]() -> lfmm_status {
        SOLVER_HIP(hipSetDevice(dir->device));
        hipStream_t st = as_stream(stream);
        auto apply = [&](const double* in, double* o) {
            hipLaunchKernelGGL(k_dipole_loads, dim3(blocks_for(dir->n)), dim3(kThreads), 0, st, in, dir->f2.p, dir->n);
            check(lfmm_execute(dir->plan, dir->f2.p, o, stream));
        };
        Gmres gm;
        gm.setup(dir->n, std::min<int>(restart, int(std::max<int64_t>(dir->n, 1))));
        const lfmm_solver_stats r = gm.run(apply, g_dev, q_dev, tol, max_iter, st);
        SOLVER_HIP(hipStreamSynchronize(st));
        if (stats) *stats = r;
        return LFMM_OK;
    });
}

lfmm_status lfmm_dirichlet_potential(lfmm_dirichlet* dir, const double* q_dev, int64_t n_tgt,
                                     const int32_t* tgt_xy_dev, double* u_dev, void* stream) {
    if (!dir || !q_dev || !tgt_xy_dev || !u_dev || n_tgt < 1) return fail(LFMM_E_INVAL, "null argument or no target");
    return run_guarded([&]() -> lfmm_status {
        SOLVER_HIP(hipSetDevice(dir->device));
        hipLaunchKernelGGL(k_dipole_loads, dim3(blocks_for(dir->n)), dim3(kThreads), 0, as_stream(stream), q_dev,
                           dir->f2.p, dir->n);
        lfmm_plan* pt = nullptr;
        check(lfmm_plan_create(dir->ctx, 2 * dir->n, dir->src.p, n_tgt, tgt_xy_dev, stream, &pt));
        lfmm_status s = lfmm_execute(pt, dir->f2.p, u_dev, stream);
        lfmm_plan_destroy(pt);
        check(s);
        SOLVER_HIP(hipGetLastError());
        return LFMM_OK;
    });
}

lfmm_status lfmm_dirichlet_destroy(lfmm_dirichlet* dir) {
    if (!dir) return LFMM_OK;
    (void)hipSetDevice(dir->device);
    (void)hipDeviceSynchronize();
    delete dir;
    return LFMM_OK;
}

}  // extern "C"
