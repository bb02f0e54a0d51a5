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
#include <mutex>
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

// Buffers of one solve: device pointers into either the solver's own
// allocations (commission_nnls) or the library's static scratch array
// (commission_nnls_noalloc).
struct Solver {
    int64_t m = 0, n = 0;
    int chunks = 0;
    const double *A = nullptr, *b = nullptr;
    double *x = nullptr, *xn = nullptr, *g = nullptr, *gn = nullptr, *r = nullptr,
           *part = nullptr, *rpart = nullptr, *sums = nullptr;
    NnlsState* state = nullptr;
    hipStream_t s = nullptr;
    double pg_stop = 0.0;
    double host_sums[3];

    unsigned row_blocks() const { return unsigned((m + kB - 1) / kB); }
    unsigned col_blocks() const { return unsigned((n + kB / 64 - 1) / (kB / 64)); }
    void sync_sums() {
        PSL_HIP(hipMemcpyAsync(host_sums, sums, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
        PSL_HIP(hipStreamSynchronize(s));
    }
    // r = A x - b (first m entries of r); returns ||r||^2
    double objective() {
        hipLaunchKernelGGL(k_ax_partial, dim3(row_blocks(), unsigned(chunks)), dim3(kB), 0, s, A,
                           x, m, n, part);
        hipLaunchKernelGGL(k_residual, dim3(row_blocks()), dim3(kB), 0, s, part, chunks, b, m, r);
        hipLaunchKernelGGL(k_sums, dim3(1), dim3(1024), 0, s, int(kSumSq), r, nullptr, m, sums);
        PSL_HIP(hipGetLastError());
        sync_sums();
        return host_sums[kSumSq];
    }
    // One iteration step: kTrials Armijo trials, then (when one passed) the
    // gradient and the state update.
    void enqueue_step(const psl_nnls_opts* o) {
        hipLaunchKernelGGL(k_trial_ax, dim3(row_blocks(), unsigned(chunks)), dim3(kB), 0, s, A, x,
                           g, m, n, chunks, o->armijo_beta, state, xn, part);
        hipLaunchKernelGGL(k_trial_residual, dim3(row_blocks(), unsigned(kTrials)), dim3(kB), 0, s,
                           part, chunks, b, m, state, r, rpart);
        hipLaunchKernelGGL(k_trial_select, dim3(1), dim3(kB), 0, s, rpart, int(row_blocks()), x, g,
                           xn, n, o->armijo_sigma, o->armijo_beta, state);
        hipLaunchKernelGGL(k_trial_grad, dim3(col_blocks()), dim3(kB), 0, s, A, r, m, n, state, gn);
        hipLaunchKernelGGL(k_accept, dim3(1), dim3(kB), 0, s, xn, gn, n, o->delta, pg_stop,
                           o->max_iter, x, g, state);
        PSL_HIP(hipGetLastError());
    }

    // F, grad F and the projected gradient at the start point x (already
    // clamped to x >= 0); fro = ||A||_F^2.  Returns the initial state, which is
    // also written to the device.
    NnlsState start(const psl_nnls_opts* opts, double fro) {
        NnlsState h{};
        h.f = objective();
        hipLaunchKernelGGL(k_atr, dim3(col_blocks()), dim3(kB), 0, s, A, r, m, n, g);
        hipLaunchKernelGGL(k_sums, dim3(1), dim3(1024), 0, s, int(kSumSq), g, nullptr, n, sums);
        hipLaunchKernelGGL(k_sums, dim3(1), dim3(1024), 0, s, int(kStats), x, g, n, sums);
        PSL_HIP(hipGetLastError());
        sync_sums();
        const double g0 = std::sqrt(host_sums[kSumSq]);
        pg_stop = opts->pg_tol * g0;
        h.pg = std::sqrt(host_sums[kStats]);
        h.s = fro > 0.0 ? 1.0 / fro : 1.0;
        h.acc = -1;
        h.converged = h.pg <= pg_stop;
        h.done = h.converged || opts->max_iter == 0;
        PSL_HIP(hipMemcpyAsync(state, &h, sizeof h, hipMemcpyHostToDevice, s));
        PSL_HIP(hipStreamSynchronize(s));
        return h;
    }

    // Runs iteration steps until the state says done, kStepsPerGraph steps
    // between reads of the state: replayed from a captured graph, or (graph =
    // false) launched directly.  Every step either rejects kTrials trials of
    // the current iteration or completes it, and the state turns done at
    // max_iter iterations or kMaxTrials rejected trials, so the loop ends.
    void iterate(const psl_nnls_opts* opts, NnlsState& h, bool graph) {
        if (h.done) return;
        hipGraph_t gr = nullptr;
        hipGraphExec_t exec = nullptr;
        struct Release {
            hipStream_t s;
            hipGraph_t& g;
            hipGraphExec_t& e;
            ~Release() {
                // work still in flight (an error path) finishes before its graph goes
                (void)hipStreamSynchronize(s);
                if (e) (void)hipGraphExecDestroy(e);
                if (g) (void)hipGraphDestroy(g);
            }
        } rel{s, gr, exec};
        if (graph) {
            PSL_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
            try {
                for (int k = 0; k < kStepsPerGraph; ++k) enqueue_step(opts);
            } catch (...) {
                hipGraph_t g = nullptr;
                (void)hipStreamEndCapture(s, &g);
                if (g) (void)hipGraphDestroy(g);
                throw;
            }
            PSL_HIP(hipStreamEndCapture(s, &gr));
            PSL_HIP(hipGraphInstantiate(&exec, gr, nullptr, nullptr, 0));
        }
        const int64_t max_replays =
            opts->max_iter / kStepsPerGraph * (kMaxTrials / kTrials) + kMaxTrials;
        for (int64_t rep = 0; !h.done; ++rep) {
            PSL_CHECK(rep < max_replays, "commission_nnls: solver state did not advance");
            if (graph) {
                PSL_HIP(hipGraphLaunch(exec, s));
            } else {
                for (int k = 0; k < kStepsPerGraph; ++k) enqueue_step(opts);
            }
            PSL_HIP(hipMemcpyAsync(&h, state, sizeof h, hipMemcpyDeviceToHost, s));
            PSL_HIP(hipStreamSynchronize(s));
        }
    }
};

void check_nnls_args(int64_t m, int64_t n, const psl_nnls_opts* opts) {
    PSL_CHECK(m >= 1 && n >= 1, "m and n must be >= 1");
    PSL_CHECK(m <= (int64_t(1) << 40) / n && n <= int64_t(65535) * kColChunk,
              "commission_nnls: matrix too large");
    PSL_CHECK(opts->armijo_sigma > 0 && opts->armijo_sigma < 1 && opts->armijo_beta > 0 &&
                  opts->armijo_beta < 1 && opts->max_iter >= 0,
              "bad Armijo parameters");
}

void fill_report(const NnlsState& h, psl_nnls_report* report, int& status) {
    if (report) {
        report->iters = h.it;
        report->f = h.f;
        report->pg_norm = h.pg;
    }
    if (!h.converged) {
        status = PSL_ENOTCONV;
        set_last_error("commission_nnls: iteration limit reached before convergence");
    }
}

}  // namespace
}  // namespace psl

using namespace psl;

extern "C" int commission_nnls(const double* A, int64_t m, int64_t n, const double* b, double* x,
                               const psl_nnls_opts* opts, psl_nnls_report* report) {
    int status = PSL_OK;
    const int rc = guarded([&] {
        PSL_CHECK(A && b && x && opts, "commission_nnls: null argument");
        check_nnls_args(m, n, opts);
        Solver S;
        S.m = m;
        S.n = n;
        S.chunks = int((n + kColChunk - 1) / kColChunk);
        DevBuf dA, db, dx, dxn, dg, dgn, dr, dpart, drpart, dsums, dstate;
        struct StreamGuard {
            hipStream_t s = nullptr;
            ~StreamGuard() {
                if (s) {
                    (void)hipStreamSynchronize(s);
                    (void)hipStreamDestroy(s);
                }
            }
        } sg;
        PSL_HIP(hipStreamCreateWithFlags(&sg.s, hipStreamNonBlocking));
        S.s = sg.s;
        dA.alloc(size_t(m) * n * 8);
        db.alloc(size_t(m) * 8);
        dx.alloc(size_t(n) * 8);
        dxn.alloc(size_t(n) * kTrials * 8);
        dg.alloc(size_t(n) * 8);
        dgn.alloc(size_t(n) * 8);
        dr.alloc(size_t(m) * kTrials * 8);
        dpart.alloc(size_t(m) * S.chunks * kTrials * 8);
        drpart.alloc(size_t(S.row_blocks()) * kTrials * 8);
        dsums.alloc(3 * 8);
        dstate.alloc(sizeof(NnlsState));
        S.A = dA.as<double>();
        S.b = db.as<double>();
        S.x = dx.as<double>();
        S.xn = dxn.as<double>();
        S.g = dg.as<double>();
        S.gn = dgn.as<double>();
        S.r = dr.as<double>();
        S.part = dpart.as<double>();
        S.rpart = drpart.as<double>();
        S.sums = dsums.as<double>();
        S.state = dstate.as<NnlsState>();
        std::vector<double> x0(x, x + n);
        for (double& v : x0) v = v > 0.0 ? v : 0.0;
        double fro = 0.0;
        for (int64_t i = 0; i < m * n; ++i) fro += A[i] * A[i];
        PSL_HIP(hipMemcpy(dA.p, A, size_t(m) * n * 8, hipMemcpyHostToDevice));
        PSL_HIP(hipMemcpy(db.p, b, size_t(m) * 8, hipMemcpyHostToDevice));
        PSL_HIP(hipMemcpy(dx.p, x0.data(), size_t(n) * 8, hipMemcpyHostToDevice));
        NnlsState h = S.start(opts, fro);
        S.iterate(opts, h, true);
        PSL_HIP(hipMemcpy(x, dx.p, size_t(n) * 8, hipMemcpyDeviceToHost));
        fill_report(h, report, status);
    });
    return rc != PSL_OK ? rc : status;
}

// ---------------------------------------------------------------------------
// Allocation-free variant: the solver's vectors live in a fixed device array.
// ---------------------------------------------------------------------------
// One copy per device, held until the process ends.  Host code never uses
// this name as an address: it reads the device address of the current
// device's copy with hipGetSymbolAddress once and passes that pointer.
static __device__ __align__(256) double scratch[PSL_NNLS_SCRATCH_BYTES / sizeof(double)];

namespace psl {
namespace {

constexpr size_t kScratchBytes = PSL_NNLS_SCRATCH_BYTES;

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

void* scratch_address() {
    int dev = 0;
    PSL_HIP(hipGetDevice(&dev));
    PSL_CHECK(dev >= 0 && dev < kMaxDevices, "commission_nnls_noalloc: device index %d", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        PSL_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        PSL_CHECK(p != nullptr, "commission_nnls_noalloc: no address for the scratch array");
        g_scratch_ptr[dev] = p;
    }
    return g_scratch_ptr[dev];
}

// Bytes of scratch a solve of an m x n system uses (each piece 256-byte aligned).
size_t scratch_bytes(int64_t m, int64_t n) {
    const int64_t chunks = (n + kColChunk - 1) / kColChunk;
    const int64_t rb = (m + kB - 1) / kB;
    auto up = [](int64_t doubles) { return (size_t(doubles) * 8 + 255) / 256 * 256; };
    return up(n * kTrials) + 2 * up(n) + up(m * kTrials) + up(m * chunks * kTrials) +
           up(rb * kTrials) + up(3) + (sizeof(NnlsState) + 255) / 256 * 256;
}

__global__ void __launch_bounds__(kB) k_clamp_nonneg(double* x, int64_t n) {
    const int64_t i = blockIdx.x * int64_t(kB) + threadIdx.x;
    if (i < n) x[i] = x[i] > 0.0 ? x[i] : 0.0;
}

}  // namespace
}  // namespace psl

extern "C" int commission_nnls_noalloc(const double* A_dev, int64_t m, int64_t n,
                                       const double* b_dev, double* x_dev,
                                       const psl_nnls_opts* opts, psl_nnls_report* report,
                                       void* stream) {
    int status = PSL_OK;
    const int rc = guarded([&] {
        PSL_CHECK(A_dev && b_dev && x_dev && opts, "commission_nnls_noalloc: null argument");
        check_nnls_args(m, n, opts);
        const size_t need = scratch_bytes(m, n);
        PSL_CHECK(need <= kScratchBytes,
                  "commission_nnls_noalloc: a %lld x %lld system needs %zu bytes of scratch, "
                  "more than the %zu available",
                  (long long)m, (long long)n, need, kScratchBytes);
        char* base = static_cast<char*>(scratch_address());
        auto take = [&base](size_t bytes) {
            char* p = base;
            base += (bytes + 255) / 256 * 256;
            return p;
        };
        Solver S;
        S.m = m;
        S.n = n;
        S.chunks = int((n + kColChunk - 1) / kColChunk);
        S.s = static_cast<hipStream_t>(stream);
        S.A = A_dev;
        S.b = b_dev;
        S.x = x_dev;
        S.xn = reinterpret_cast<double*>(take(size_t(n) * kTrials * 8));
        S.g = reinterpret_cast<double*>(take(size_t(n) * 8));
        S.gn = reinterpret_cast<double*>(take(size_t(n) * 8));
        S.r = reinterpret_cast<double*>(take(size_t(m) * kTrials * 8));
        S.part = reinterpret_cast<double*>(take(size_t(m) * S.chunks * kTrials * 8));
        S.rpart = reinterpret_cast<double*>(take(size_t(S.row_blocks()) * kTrials * 8));
        S.sums = reinterpret_cast<double*>(take(3 * 8));
        S.state = reinterpret_cast<NnlsState*>(take(sizeof(NnlsState)));
        hipLaunchKernelGGL(k_clamp_nonneg, dim3(unsigned((n + kB - 1) / kB)), dim3(kB), 0, S.s,
                           x_dev, n);
        // ||A||_F^2 on the device (one block, fixed order), into sums[0]
        hipLaunchKernelGGL(k_sums, dim3(1), dim3(1024), 0, S.s, int(kSumSq), A_dev, nullptr, m * n,
                           S.sums);
        PSL_HIP(hipGetLastError());
        S.sync_sums();
        const double fro = S.host_sums[kSumSq];
        NnlsState h = S.start(opts, fro);
        S.iterate(opts, h, false);
        fill_report(h, report, status);
    });
    return rc != PSL_OK ? rc : status;
}
