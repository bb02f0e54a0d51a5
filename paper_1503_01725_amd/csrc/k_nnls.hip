// Commissioning solve (Sec. 2.2.3 Eq. 8, Sec. 2.2.4): min_{x>=0} ||A x - b||^2
// by gradient projection x+ = max(0, x - s g) with Armijo's rule along the
// projection arc.  The trial step is the Barzilai-Borwein step of the previous
// iteration (the first one 1/||A||_F^2).  All vector work and every accept /
// stop decision run in FP64 on the GPU: an iteration is five kernels that
// read and update a small device state (the two decisions are single-block
// kernels, so no grid-wide fence is needed), a batch of iterations is one
// graph replay, and the host reads the state once per replay.  Each iteration tests
// kTrials Armijo steps s, s beta, s beta^2, ... from one pass over A and takes
// the first that passes, which is the step the sequential rule would take.
// Every reduction has a fixed order, so a solve is reproducible bit for bit.
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

// Single-block fixed-order sums used before the first iteration:
// kSumSq: out[0] = sum a^2; kStats (with a = x, d = g): out[2] = |projected g|^2.
enum { kSumSq = 0, kStats = 2 };
__global__ void __launch_bounds__(1024) k_sums(int kind, const double* a, const double* d, int64_t n,
                                               double* out) {
    __shared__ double sh[1024 / 64];
    double s0 = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 1024) {
        if (kind == kSumSq) {
            s0 = fma(a[i], a[i], s0);
        } else {
            const double pg = a[i] > 0.0 ? d[i] : fmin(d[i], 0.0);
            s0 = fma(pg, pg, s0);
        }
    }
    for (int off = 32; off >= 1; off >>= 1) s0 += __shfl_xor(s0, off, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x / 64] = s0;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int k = 0; k < 1024 / 64; ++k) t += sh[k];
        out[kind] = t;
    }
}

constexpr int kTrials = 8;        // Armijo trial steps evaluated per pass over A
constexpr int kMaxTrials = 200;   // trials per iteration before the search gives up
constexpr int kStepsPerGraph = 32;
static_assert(kTrials * kColChunk == kB, "one thread per (trial, column) of a chunk");
static_assert(kMaxTrials % kTrials == 0, "the trial limit falls on a batch boundary");

// Solver state shared by the iteration kernels (device memory, 8-byte fields
// first).  One graph step either rejects kTrials more steps of the current
// iteration or completes it.
struct NnlsState {
    double f;        // F at the current x
    double s;        // first trial step of the next batch
    double fn;       // F at the accepted trial point
    double s_acc;    // step of the accepted trial
    double pg;       // projected-gradient norm at the current x
    int64_t it;      // iterations started
    int32_t ls;      // trials already rejected in the current iteration
    int32_t acc;     // trial accepted by the last batch, -1 = none
    int32_t done;    // converged, iteration limit, or line search exhausted
    int32_t converged;
};

// Sums K per-thread values over the block in a fixed order; out (shared, K
// entries) is valid for every thread on return.
template <int K>
__device__ void block_sums(double (&v)[K], double* out) {
    __shared__ double sh[K][kB / 64];
    for (int k = 0; k < K; ++k)
        for (int off = 32; off >= 1; off >>= 1) v[k] += __shfl_xor(v[k], off, 64);
    if ((threadIdx.x & 63) == 0)
        for (int k = 0; k < K; ++k) sh[k][threadIdx.x / 64] = v[k];
    __syncthreads();
    if (threadIdx.x < K) {
        double t = 0.0;
        for (int w = 0; w < kB / 64; ++w) t += sh[threadIdx.x][w];
        out[threadIdx.x] = t;
    }
    __syncthreads();
}

// Trial points xn_t = max(0, x - s beta^t g) of one column chunk and their
// partial products part[t][chunk][i] = sum_{j in chunk} A[i, j] xn_t[j].
// Grid (row blocks, column chunks); row block 0 also stores xn_t.
__global__ void __launch_bounds__(kB) k_trial_ax(const double* A, const double* x, const double* g,
                                                 int64_t m, int64_t n, int chunks, double beta,
                                                 const NnlsState* st, double* xn, double* part) {
    if (st->done) return;
    __shared__ double xs[kTrials][kColChunk];
    const int64_t j0 = int64_t(blockIdx.y) * kColChunk;
    const int ncol = int(n - j0 < kColChunk ? n - j0 : kColChunk);
    {
        const int t = threadIdx.x / kColChunk, jj = threadIdx.x % kColChunk;
        double s = st->s;
        for (int k = 0; k < t; ++k) s *= beta;
        if (jj < ncol) {
            const double v = fmax(x[j0 + jj] - s * g[j0 + jj], 0.0);
            xs[t][jj] = v;
            if (blockIdx.x == 0) xn[int64_t(t) * n + j0 + jj] = v;
        }
    }
    __syncthreads();
    const int64_t i = blockIdx.x * int64_t(kB) + threadIdx.x;
    if (i >= m) return;
    double acc[kTrials];
    for (int t = 0; t < kTrials; ++t) acc[t] = 0.0;
    if (ncol == kColChunk) {
        // all loads of the chunk in flight together
        double a[kColChunk];
#pragma unroll
        for (int jj = 0; jj < kColChunk; ++jj) a[jj] = A[(j0 + jj) * m + i];
#pragma unroll
        for (int jj = 0; jj < kColChunk; ++jj)
            for (int t = 0; t < kTrials; ++t) acc[t] = fma(a[jj], xs[t][jj], acc[t]);
    } else {
        for (int jj = 0; jj < ncol; ++jj) {
            const double a = A[(j0 + jj) * m + i];
            for (int t = 0; t < kTrials; ++t) acc[t] = fma(a, xs[t][jj], acc[t]);
        }
    }
    for (int t = 0; t < kTrials; ++t) part[(int64_t(t) * chunks + blockIdx.y) * m + i] = acc[t];
}

// Residuals r_t = A xn_t - b and per-block partials of |r_t|^2 in
// rpart[t][row block]; grid (row blocks, trials).
__global__ void __launch_bounds__(kB) k_trial_residual(const double* part, int chunks,
                                                       const double* b, int64_t m,
                                                       const NnlsState* st, double* r,
                                                       double* rpart) {
    if (st->done) return;
    const int64_t i = blockIdx.x * int64_t(kB) + threadIdx.x;
    const int trial = blockIdx.y;
    double v = 0.0;
    if (i < m) {
        const double* p = part + int64_t(trial) * chunks * m + i;
        // groups of 8 guarded loads in flight; the sum keeps chunk order
        for (int c = 0; c < chunks; c += 8) {
            double q[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) q[k] = c + k < chunks ? p[int64_t(c + k) * m] : 0.0;
#pragma unroll
            for (int k = 0; k < 8; ++k)
                if (c + k < chunks) v += q[k];
        }
        v -= b[i];
        r[int64_t(trial) * m + i] = v;
    }
    double sq[1] = {v * v};
    __shared__ double red[1];
    block_sums<1>(sq, red);
    if (threadIdx.x == 0) rpart[trial * gridDim.x + blockIdx.x] = red[0];
}

// One block: F(xn_t) from the partials in block order, the decrease
// g.(xn_t - x), and Armijo's test applied to the trials in order.
__global__ void __launch_bounds__(kB) k_trial_select(const double* rpart, int row_blocks,
                                                     const double* x, const double* g,
                                                     const double* xn, int64_t n, double sigma,
                                                     double beta, NnlsState* st) {
    if (st->done) return;
    __shared__ double fn[kTrials];
    if (threadIdx.x < kTrials) {
        const double* p = rpart + threadIdx.x * row_blocks;
        double t = 0.0;
        for (int k = 0; k < row_blocks; k += 8) {
            double q[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) q[u] = k + u < row_blocks ? p[k + u] : 0.0;
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (k + u < row_blocks) t += q[u];
        }
        fn[threadIdx.x] = t;
    }
    double d[kTrials];
    for (int t = 0; t < kTrials; ++t) d[t] = 0.0;
#pragma unroll 4
    for (int64_t j = threadIdx.x; j < n; j += kB) {
        const double gj = g[j], xj = x[j];
        for (int t = 0; t < kTrials; ++t) d[t] = fma(gj, xn[int64_t(t) * n + j] - xj, d[t]);
    }
    __shared__ double dec[kTrials];
    block_sums<kTrials>(d, dec);
    if (threadIdx.x == 0) {
        const double f = st->f;
        const int ls = st->ls;
        double s = st->s;
        if (ls == 0) st->it = st->it + 1;
        int acc = -1;
        for (int t = 0; t < kTrials; ++t) {
            if (fn[t] <= f + sigma * dec[t]) {
                acc = t;
                break;
            }
            s *= beta;
        }
        if (acc >= 0) {
            st->fn = fn[acc];
            st->s_acc = s;
            st->ls = 0;
        } else {
            st->s = s;
            st->ls = ls + kTrials;
            if (ls + kTrials >= kMaxTrials) st->done = 1;
        }
        st->acc = acc;
    }
}

// Gradient at the accepted trial point, gn[j] = 2 A[:, j] . r_acc, one wave
// per column.
__global__ void __launch_bounds__(kB) k_trial_grad(const double* A, const double* r, int64_t m,
                                                   int64_t n, const NnlsState* st, double* gn) {
    if (st->done || st->acc < 0) return;
    const double* ra = r + int64_t(st->acc) * m;
    const int64_t j = blockIdx.x * int64_t(kB / 64) + threadIdx.x / 64;
    const int lane = threadIdx.x & 63;
    if (j >= n) return;
    const double* col = A + j * m;
    double v = 0.0;
    for (int64_t i = lane; i < m; i += 8 * 64) {
        double a[8], q[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const bool in = i + k * 64 < m;
            a[k] = in ? col[i + k * 64] : 0.0;
            q[k] = in ? ra[i + k * 64] : 0.0;
        }
#pragma unroll
        for (int k = 0; k < 8; ++k)
            if (i + k * 64 < m) v = fma(a[k], q[k], v);
    }
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    if (lane == 0) gn[j] = 2.0 * v;
}

// One block: Barzilai-Borwein step, projected gradient and stop test at the
// accepted trial point, which becomes the current x (and gn the current g).
__global__ void __launch_bounds__(kB) k_accept(const double* xn, const double* gn, int64_t n,
                                               double delta, double pg_stop, int64_t max_iter,
                                               double* x, double* g, NnlsState* st) {
    if (st->done || st->acc < 0) return;
    const double* xa = xn + int64_t(st->acc) * n;
    double v[3] = {0.0, 0.0, 0.0};
#pragma unroll 4
    for (int64_t k = threadIdx.x; k < n; k += kB) {
        const double dx = xa[k] - x[k];
        const double dg = gn[k] - g[k];
        v[0] = fma(dx, dx, v[0]);
        v[1] = fma(dx, dg, v[1]);
        const double p = xa[k] > 0.0 ? gn[k] : fmin(gn[k], 0.0);
        v[2] = fma(p, p, v[2]);
    }
    __shared__ double sums[3];
    block_sums<3>(v, sums);
    for (int64_t k = threadIdx.x; k < n; k += kB) {
        x[k] = xa[k];
        g[k] = gn[k];
    }
    if (threadIdx.x == 0) {
        const double f = st->f, fnew = st->fn;
        const double pg = sqrt(sums[2]);
        st->s = sums[1] > 0.0 ? sums[0] / sums[1] : 2.0 * st->s_acc;
        const double rel = (f - fnew) / (f > 0.0 ? f : 1.0);
        const int conv = (rel < delta && pg <= pg_stop) || fnew == 0.0;
        st->f = fnew;
        st->pg = pg;
        st->converged = conv;
        st->done = conv || st->it >= max_iter;
        st->acc = -1;
    }
}

struct Solver {
    int64_t m, n;
    int chunks;
    DevBuf A, b, x, xn, g, gn, r, part, rpart, sums, state;
    hipStream_t s = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    ~Solver() {
        // work still in flight (an error path) finishes before its graph and
        // buffers go
        if (s) (void)hipStreamSynchronize(s);
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (s) (void)hipStreamDestroy(s);
    }

    double host_sums[3];
    void sync_sums() {
        PSL_HIP(hipMemcpyAsync(host_sums, sums.p, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
        PSL_HIP(hipStreamSynchronize(s));
    }
    unsigned row_blocks() const { return unsigned((m + kB - 1) / kB); }
    // r = A x - b (first m entries of r); returns ||r||^2
    double objective() {
        hipLaunchKernelGGL(k_ax_partial, dim3(row_blocks(), unsigned(chunks)), dim3(kB), 0, s,
                           A.as<double>(), x.as<double>(), m, n, part.as<double>());
        hipLaunchKernelGGL(k_residual, dim3(row_blocks()), dim3(kB), 0, s, part.as<double>(),
                           chunks, b.as<double>(), m, r.as<double>());
        hipLaunchKernelGGL(k_sums, dim3(1), dim3(1024), 0, s, int(kSumSq), r.as<double>(), nullptr,
                           m, sums.as<double>());
        PSL_HIP(hipGetLastError());
        sync_sums();
        return host_sums[kSumSq];
    }
    // One iteration step: kTrials Armijo trials, then (when one passed) the
    // gradient and the state update.
    void enqueue_step(const psl_nnls_opts* o) {
        NnlsState* st = state.as<NnlsState>();
        hipLaunchKernelGGL(k_trial_ax, dim3(row_blocks(), unsigned(chunks)), dim3(kB), 0, s,
                           A.as<double>(), x.as<double>(), g.as<double>(), m, n, chunks,
                           o->armijo_beta, st, xn.as<double>(), part.as<double>());
        hipLaunchKernelGGL(k_trial_residual, dim3(row_blocks(), unsigned(kTrials)), dim3(kB), 0, s,
                           part.as<double>(), chunks, b.as<double>(), m, st, r.as<double>(),
                           rpart.as<double>());
        hipLaunchKernelGGL(k_trial_select, dim3(1), dim3(kB), 0, s, rpart.as<double>(),
                           int(row_blocks()), x.as<double>(), g.as<double>(), xn.as<double>(), n,
                           o->armijo_sigma, o->armijo_beta, st);
        hipLaunchKernelGGL(k_trial_grad, dim3(unsigned((n + kB / 64 - 1) / (kB / 64))), dim3(kB),
                           0, s, A.as<double>(), r.as<double>(), m, n, st, gn.as<double>());
        hipLaunchKernelGGL(k_accept, dim3(1), dim3(kB), 0, s, xn.as<double>(), gn.as<double>(), n,
                           o->delta, pg_stop, o->max_iter, x.as<double>(), g.as<double>(), st);
        PSL_HIP(hipGetLastError());
    }
    double pg_stop = 0.0;
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
        PSL_CHECK(m <= (int64_t(1) << 40) / n && n <= int64_t(65535) * kColChunk,
                  "commission_nnls: matrix too large");
        PSL_CHECK(opts->armijo_sigma > 0 && opts->armijo_sigma < 1 && opts->armijo_beta > 0 &&
                      opts->armijo_beta < 1 && opts->max_iter >= 0,
                  "bad Armijo parameters");
        Solver S;
        S.m = m;
        S.n = n;
        S.chunks = int((n + kColChunk - 1) / kColChunk);
        PSL_HIP(hipStreamCreateWithFlags(&S.s, hipStreamNonBlocking));
        S.A.alloc(size_t(m) * n * 8);
        S.b.alloc(size_t(m) * 8);
        S.x.alloc(size_t(n) * 8);
        S.xn.alloc(size_t(n) * kTrials * 8);
        S.g.alloc(size_t(n) * 8);
        S.gn.alloc(size_t(n) * 8);
        S.r.alloc(size_t(m) * kTrials * 8);
        S.part.alloc(size_t(m) * S.chunks * kTrials * 8);
        S.rpart.alloc(size_t(S.row_blocks()) * kTrials * 8);
        S.sums.alloc(3 * 8);
        S.state.alloc(sizeof(NnlsState));
        std::vector<double> x0(x, x + n);
        for (double& v : x0) v = v > 0.0 ? v : 0.0;
        double fro = 0.0;
        for (int64_t i = 0; i < m * n; ++i) fro += A[i] * A[i];
        PSL_HIP(hipMemcpy(S.A.p, A, size_t(m) * n * 8, hipMemcpyHostToDevice));
        PSL_HIP(hipMemcpy(S.b.p, b, size_t(m) * 8, hipMemcpyHostToDevice));
        PSL_HIP(hipMemcpy(S.x.p, x0.data(), size_t(n) * 8, hipMemcpyHostToDevice));

        // F, grad F, |grad F| and the projected gradient at the start point
        NnlsState h{};
        h.f = S.objective();
        hipLaunchKernelGGL(k_atr, dim3(unsigned((n + kB / 64 - 1) / (kB / 64))), dim3(kB), 0, S.s,
                           S.A.as<double>(), S.r.as<double>(), m, n, S.g.as<double>());
        hipLaunchKernelGGL(k_sums, dim3(1), dim3(1024), 0, S.s, int(kSumSq), S.g.as<double>(),
                           nullptr, n, S.sums.as<double>());
        hipLaunchKernelGGL(k_sums, dim3(1), dim3(1024), 0, S.s, int(kStats), S.x.as<double>(),
                           S.g.as<double>(), n, S.sums.as<double>());
        PSL_HIP(hipGetLastError());
        S.sync_sums();
        const double g0 = std::sqrt(S.host_sums[kSumSq]);
        S.pg_stop = opts->pg_tol * g0;
        h.pg = std::sqrt(S.host_sums[kStats]);
        h.s = fro > 0.0 ? 1.0 / fro : 1.0;
        h.acc = -1;
        h.converged = h.pg <= S.pg_stop;
        h.done = h.converged || opts->max_iter == 0;
        PSL_HIP(hipMemcpy(S.state.p, &h, sizeof h, hipMemcpyHostToDevice));

        if (!h.done) {
            PSL_HIP(hipStreamBeginCapture(S.s, hipStreamCaptureModeThreadLocal));
            try {
                for (int k = 0; k < kStepsPerGraph; ++k) S.enqueue_step(opts);
            } catch (...) {
                hipGraph_t g = nullptr;
                (void)hipStreamEndCapture(S.s, &g);
                if (g) (void)hipGraphDestroy(g);
                throw;
            }
            PSL_HIP(hipStreamEndCapture(S.s, &S.graph));
            PSL_HIP(hipGraphInstantiate(&S.exec, S.graph, nullptr, nullptr, 0));
            // Every step either rejects kTrials trials of the current iteration
            // or completes it, and the state turns done at max_iter iterations or
            // kMaxTrials rejected trials, so this loop ends.
            const int64_t max_replays =
                opts->max_iter / kStepsPerGraph * (kMaxTrials / kTrials) + kMaxTrials;
            for (int64_t rep = 0; !h.done; ++rep) {
                PSL_CHECK(rep < max_replays, "commission_nnls: solver state did not advance");
                PSL_HIP(hipGraphLaunch(S.exec, S.s));
                PSL_HIP(hipMemcpyAsync(&h, S.state.p, sizeof h, hipMemcpyDeviceToHost, S.s));
                PSL_HIP(hipStreamSynchronize(S.s));
            }
        }
        PSL_HIP(hipMemcpy(x, S.x.p, size_t(n) * 8, hipMemcpyDeviceToHost));
        if (report) {
            report->iters = h.it;
            report->f = h.f;
            report->pg_norm = h.pg;
        }
        if (!h.converged) {
            status = PSL_ENOTCONV;
            set_last_error("commission_nnls: iteration limit reached before convergence");
        }
    });
    return rc != PSL_OK ? rc : status;
}
