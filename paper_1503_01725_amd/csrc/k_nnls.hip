// Commissioning solve (Sec. 2.2.3 Eq. 8, Sec. 2.2.4): min_{x>=0} ||A x - b||^2
// by gradient projection x+ = max(0, x - s g) with Armijo's rule along the
// projection arc.  The trial step is the Barzilai-Borwein step of the previous
// iteration (the first one 1/||A||_F^2).  All vector work is FP64 on the GPU;
// the host only takes the scalar accept / stop decisions.  Every reduction has
// a fixed order, so a solve is reproducible bit for bit.
#include <cmath>
#include <cstring>
#include <vector>

#include "common.hpp"

namespace psl {
namespace {

constexpr int kB = 256;
constexpr int kColChunk = 32;   // columns per block of the A x product

// part[c][i] = sum over columns j in chunk c of A[i, j] x[j]   (A column-major)
__global__ void __launch_bounds__(kB) k_ax_partial(const double* A, const double* x, int64_t m,
                                                   int64_t n, double* part) {
    const int64_t i = blockIdx.x * int64_t(kB) + threadIdx.x;
    const int64_t j0 = int64_t(blockIdx.y) * kColChunk;
    const int64_t j1 = j0 + kColChunk < n ? j0 + kColChunk : n;
    if (i >= m) return;
    double acc = 0.0;
    for (int64_t j = j0; j < j1; ++j) acc = fma(A[j * m + i], x[j], acc);
    part[int64_t(blockIdx.y) * m + i] = acc;
}

// r = sum_c part[c] - b
__global__ void __launch_bounds__(kB) k_residual(const double* part, int chunks, const double* b,
                                                 int64_t m, double* r) {
    const int64_t i = blockIdx.x * int64_t(kB) + threadIdx.x;
    if (i >= m) return;
    double acc = 0.0;
    for (int c = 0; c < chunks; ++c) acc += part[int64_t(c) * m + i];
    r[i] = acc - b[i];
}

// g[j] = 2 A[:, j] . r   (one wave per column)
__global__ void __launch_bounds__(kB) k_atr(const double* A, const double* r, int64_t m, int64_t n,
                                            double* g) {
    const int64_t j = blockIdx.x * int64_t(kB / 64) + threadIdx.x / 64;
    const int lane = threadIdx.x & 63;
    if (j >= n) return;
    const double* col = A + j * m;
    double acc = 0.0;
    for (int64_t i = lane; i < m; i += 64) acc = fma(col[i], r[i], acc);
    for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if (lane == 0) g[j] = 2.0 * acc;
}

// xn = max(0, x - s g)
__global__ void __launch_bounds__(kB) k_project(const double* x, const double* g, double s,
                                                int64_t n, double* xn) {
    const int64_t j = blockIdx.x * int64_t(kB) + threadIdx.x;
    if (j < n) xn[j] = fmax(x[j] - s * g[j], 0.0);
}

// Single-block fixed-order sums: out[k] = sum_i f_k(i) for the requested kind.
enum { kSumSq = 0, kDecrease = 1, kStats = 2 };
__global__ void __launch_bounds__(1024) k_sums(int kind, const double* a, const double* b2,
                                               const double* c, const double* d, int64_t n,
                                               double* out) {
    __shared__ double sh[3][1024 / 64];
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 1024) {
        if (kind == kSumSq) {
            s0 = fma(a[i], a[i], s0);                       // a = r
        } else if (kind == kDecrease) {
            s0 = fma(b2[i], a[i] - c[i], s0);               // g . (xn - x)
        } else {
            const double dx = a[i] - c[i];                  // xn - x
            const double dg = d[i] - b2[i];                 // gn - g
            s0 = fma(dx, dx, s0);
            s1 = fma(dx, dg, s1);
            const double pg = a[i] > 0.0 ? d[i] : fmin(d[i], 0.0);
            s2 = fma(pg, pg, s2);
        }
    }
    for (int off = 32; off >= 1; off >>= 1) {
        s0 += __shfl_xor(s0, off, 64);
        s1 += __shfl_xor(s1, off, 64);
        s2 += __shfl_xor(s2, off, 64);
    }
    const int w = threadIdx.x / 64;
    if ((threadIdx.x & 63) == 0) {
        sh[0][w] = s0;
        sh[1][w] = s1;
        sh[2][w] = s2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double t0 = 0.0, t1 = 0.0, t2 = 0.0;
        for (int k = 0; k < 1024 / 64; ++k) {
            t0 += sh[0][k];
            t1 += sh[1][k];
            t2 += sh[2][k];
        }
        out[0] = t0;
        out[1] = t1;
        out[2] = t2;
    }
}

struct Solver {
    int64_t m, n;
    int chunks;
    DevBuf A, b, x, xn, g, gn, r, part, sums;
    hipStream_t s = nullptr;

    double host3[3];
    void sync_sums() {
        PSL_HIP(hipMemcpyAsync(host3, sums.p, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
        PSL_HIP(hipStreamSynchronize(s));
    }
    // r = A v - b ; returns ||r||^2
    double objective(const double* v) {
        dim3 grid(unsigned((m + kB - 1) / kB), unsigned(chunks));
        hipLaunchKernelGGL(k_ax_partial, grid, dim3(kB), 0, s, A.as<double>(), v, m, n,
                           part.as<double>());
        hipLaunchKernelGGL(k_residual, dim3(unsigned((m + kB - 1) / kB)), dim3(kB), 0, s,
                           part.as<double>(), chunks, b.as<double>(), m, r.as<double>());
        hipLaunchKernelGGL(k_sums, dim3(1), dim3(1024), 0, s, int(kSumSq), r.as<double>(),
                           nullptr, nullptr, nullptr, m, sums.as<double>());
        PSL_HIP(hipGetLastError());
        sync_sums();
        return host3[0];
    }
    void gradient(double* out) {
        hipLaunchKernelGGL(k_atr, dim3(unsigned((n + kB / 64 - 1) / (kB / 64))), dim3(kB), 0, s,
                           A.as<double>(), r.as<double>(), m, n, out);
        PSL_HIP(hipGetLastError());
    }
};

}  // namespace
}  // namespace psl

using namespace psl;

extern "C" int commission_nnls(const double* A, int64_t m, int64_t n, const double* b, double* x,
                               const psl_nnls_opts* opts, psl_nnls_report* report) {
    int status = PSL_OK;
    const int rc = guarded([&] {
        PSL_CHECK(A && b && x && opts, "commission_nnls: null argument");
        PSL_CHECK(m >= 1 && n >= 1, "m and n must be >= 1");
        PSL_CHECK(opts->armijo_sigma > 0 && opts->armijo_sigma < 1 && opts->armijo_beta > 0 &&
                      opts->armijo_beta < 1 && opts->max_iter >= 0,
                  "bad Armijo parameters");
        Solver S;
        S.m = m;
        S.n = n;
        S.chunks = int((n + kColChunk - 1) / kColChunk);
        PSL_HIP(hipStreamCreateWithFlags(&S.s, hipStreamNonBlocking));
        struct StreamGuard {
            hipStream_t s;
            ~StreamGuard() { (void)hipStreamDestroy(s); }
        } guard{S.s};
        S.A.alloc(size_t(m) * n * 8);
        S.b.alloc(size_t(m) * 8);
        S.x.alloc(size_t(n) * 8);
        S.xn.alloc(size_t(n) * 8);
        S.g.alloc(size_t(n) * 8);
        S.gn.alloc(size_t(n) * 8);
        S.r.alloc(size_t(m) * 8);
        S.part.alloc(size_t(m) * S.chunks * 8);
        S.sums.alloc(3 * 8);
        std::vector<double> x0(x, x + n);
        for (double& v : x0) v = v > 0.0 ? v : 0.0;
        double fro = 0.0;
        for (int64_t i = 0; i < m * n; ++i) fro += A[i] * A[i];
        PSL_HIP(hipMemcpy(S.A.p, A, size_t(m) * n * 8, hipMemcpyHostToDevice));
        PSL_HIP(hipMemcpy(S.b.p, b, size_t(m) * 8, hipMemcpyHostToDevice));
        PSL_HIP(hipMemcpy(S.x.p, x0.data(), size_t(n) * 8, hipMemcpyHostToDevice));

        double* dx = S.x.as<double>();
        double* dxn = S.xn.as<double>();
        double* dg = S.g.as<double>();
        double* dgn = S.gn.as<double>();
        const unsigned gb = unsigned((n + kB - 1) / kB);

        double f = S.objective(dx);
        S.gradient(dg);
        // |g0| and the projected gradient at x0
        hipLaunchKernelGGL(k_sums, dim3(1), dim3(1024), 0, S.s, int(kStats), dx, dg, dx, dg, n,
                           S.sums.as<double>());
        S.sync_sums();
        hipLaunchKernelGGL(k_sums, dim3(1), dim3(1024), 0, S.s, int(kSumSq), dg, nullptr, nullptr,
                           nullptr, n, S.sums.as<double>() );
        const double pg0 = std::sqrt(S.host3[2]);
        S.sync_sums();
        const double g0 = std::sqrt(S.host3[0]);
        double step = fro > 0.0 ? 1.0 / fro : 1.0;
        double pg = pg0;
        int64_t it = 0;
        bool converged = pg <= opts->pg_tol * g0;
        while (!converged && it < opts->max_iter) {
            ++it;
            double s = step, fn = f;
            bool accepted = false;
            for (int ls = 0; ls < 200; ++ls) {
                hipLaunchKernelGGL(k_project, dim3(gb), dim3(kB), 0, S.s, dx, dg, s, n, dxn);
                hipLaunchKernelGGL(k_sums, dim3(1), dim3(1024), 0, S.s, int(kDecrease), dxn, dg, dx,
                                   nullptr, n, S.sums.as<double>());
                S.sync_sums();
                const double dec = S.host3[0];
                fn = S.objective(dxn);
                if (fn <= f + opts->armijo_sigma * dec) {
                    accepted = true;
                    break;
                }
                s *= opts->armijo_beta;
            }
            if (!accepted) break;
            S.gradient(dgn);
            hipLaunchKernelGGL(k_sums, dim3(1), dim3(1024), 0, S.s, int(kStats), dxn, dg, dx, dgn, n,
                               S.sums.as<double>());
            S.sync_sums();
            const double sxx = S.host3[0], sxg = S.host3[1];
            pg = std::sqrt(S.host3[2]);
            step = sxg > 0.0 ? sxx / sxg : 2.0 * s;
            const double rel = (f - fn) / (f > 0.0 ? f : 1.0);
            std::swap(dx, dxn);
            std::swap(dg, dgn);
            f = fn;
            if ((rel < opts->delta && pg <= opts->pg_tol * g0) || f == 0.0) converged = true;
        }
        PSL_HIP(hipMemcpy(x, dx, size_t(n) * 8, hipMemcpyDeviceToHost));
        if (report) {
            report->iters = it;
            report->f = f;
            report->pg_norm = pg;
        }
        if (!converged) {
            status = PSL_ENOTCONV;
            set_last_error("commission_nnls: iteration limit reached before convergence");
        }
    });
    return rc != PSL_OK ? rc : status;
}
