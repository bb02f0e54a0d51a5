// Batched runtime: runs every batch of every replica of a plan (Sec. 2.1.3:
// sampling and transport kernels iterated, one particle type per batch) as one
// stream of launches, optionally captured once into a hipGraph and replayed,
// with the particle stacks owned by the tally's workspace.  Also the autotuner
// that picks the batch size and the energy-band width from measured times.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <memory>
#include <vector>

#include "common.hpp"
#include "schedule.hpp"

namespace psl {
namespace {

__global__ void k_set_u32(uint32_t* p, uint32_t v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

__global__ void k_inc_u32(uint32_t* p) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p += 1u;
}

enum Phase { kSample = 0, kPhoton, kSort, kElectron, kFold, kPhases };

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// One structure-of-arrays stack carved out of a single allocation.
void carve(DevBuf& mem, uint32_t cap, psl_particles& p) {
    const size_t f = align256(size_t(cap) * 4), h = align256(size_t(cap) * 8);
    mem.alloc(7 * f + h + f + 256);
    char* b = mem.as<char>();
    float** fl[7] = {&p.x, &p.y, &p.z, &p.u, &p.v, &p.w, &p.e};
    for (int i = 0; i < 7; ++i) *fl[i] = reinterpret_cast<float*>(b + i * f);
    p.hid = reinterpret_cast<uint64_t*>(b + 7 * f);
    p.tag = reinterpret_cast<uint32_t*>(b + 7 * f + h);
    p.count = reinterpret_cast<uint32_t*>(b + 7 * f + h + f);
    p.capacity = cap;
    p.ptype = 0;
}

struct GraphKey {
    const psl_plan* plan = nullptr;
    const psl_phantom* phantom = nullptr;
    uint32_t max_batch = 0;
    int32_t band_width = 0, sort = 0, timing = 0, lane_load = 0, pipes = 0;
    uint32_t rep0 = 0, n_rep = 0;
    uint64_t seed = 0, n_hist = 0;
    float cut_e = 0, cut_g = 0, frac = 0;
    int32_t ms = 0;
    uint32_t ph_cap = 0, el_cap = 0;
    uint64_t n_batches = 0;
    uint64_t tab_gen = 0;   // physics-table generation of the phantom
    int32_t dens = 0;
    uint32_t physics = 0;        // optional photon processes
    const void* rec = nullptr;   // deposit recording buffer (kernels differ)
    bool operator==(const GraphKey& o) const { return std::memcmp(this, &o, sizeof o) == 0; }
};

}  // namespace

// One batch pipeline: particle stacks, transport scratch and a stream.
// Batches of a replica alternate between the pipelines, so that one
// pipeline's photon transport can overlap the other's electron transport
// (and the tail of each persistent kernel is filled by the other's work).
struct Pipe {
    uint32_t ph_cap = 0, el_cap = 0;
    DevBuf ph_mem, el_mem, ws_mem;
    psl_particles phs{}, els{};
    TransportWs ws{};
    hipStream_t st = nullptr;
    hipEvent_t join = nullptr;
    Pipe() = default;
    Pipe(const Pipe&) = delete;
    Pipe& operator=(const Pipe&) = delete;
    ~Pipe() {
        if (join) (void)hipEventDestroy(join);
        if (st) (void)hipStreamDestroy(st);
    }
};

constexpr int kMaxPipes = 2;

struct Runner {
    std::array<Pipe, kMaxPipes> pipes;
    DevBuf rep;
    hipStream_t cs = nullptr;
    hipEvent_t start = nullptr, done = nullptr, fork = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    GraphKey key{};
    bool have_graph = false;
    // timing: (phase, start, end) for every timed launch of the last run
    std::vector<hipEvent_t> pool;
    std::vector<std::array<int, 3>> timed;
    size_t pool_used = 0;

    ~Runner() {
        drop_graph();
        for (hipEvent_t e : pool) (void)hipEventDestroy(e);
        if (start) (void)hipEventDestroy(start);
        if (done) (void)hipEventDestroy(done);
        if (fork) (void)hipEventDestroy(fork);
        if (cs) (void)hipStreamDestroy(cs);
    }
    void drop_graph() {
        // a launch of the old graph may still run (psl_run returns at once)
        if (exec && cs) (void)hipStreamSynchronize(cs);
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
        have_graph = false;
    }
    void init() {
        if (!cs) {
            PSL_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
            PSL_HIP(hipEventCreateWithFlags(&start, hipEventDisableTiming));
            PSL_HIP(hipEventCreateWithFlags(&done, hipEventDisableTiming));
            PSL_HIP(hipEventCreateWithFlags(&fork, hipEventDisableTiming));
            for (Pipe& p : pipes) {
                PSL_HIP(hipStreamCreateWithFlags(&p.st, hipStreamNonBlocking));
                PSL_HIP(hipEventCreateWithFlags(&p.join, hipEventDisableTiming));
            }
            rep.alloc(256);
        }
    }
    void ensure_stacks(int n_pipes, uint32_t ph, uint32_t el, uint32_t physics) {
        const bool pair = (physics & kPhysPair) != 0u;
        const bool hard = (physics & (kPhysDelta | kPhysBrem)) != 0u;
        for (int i = 0; i < n_pipes; ++i) {
            Pipe& p = pipes[i];
            if (ph > p.ph_cap) {
                drop_graph();
                carve(p.ph_mem, ph, p.phs);
                p.ph_cap = ph;
            }
            if (el > p.el_cap) {
                drop_graph();
                carve(p.el_mem, el, p.els);
                p.el_cap = el;
            }
            const uint32_t need = std::max(p.ph_cap, p.el_cap);
            uint32_t ann = pair ? 2u * p.ph_cap : 0u;
            // bremsstrahlung photons of an electron pass: at most one stack
            // entry per electron the pass may hold
            if (physics & kPhysBrem) ann = std::max(ann, need);
            const uint32_t del = hard ? need : 0u;
            if (p.ws.perm_cap < need || p.ws.ann_cap < ann || p.ws.del_cap < del) {
                drop_graph();
                p.ws = alloc_transport_ws(p.ws_mem, std::max(need, p.ws.perm_cap),
                                          std::max(ann, p.ws.ann_cap), std::max(del, p.ws.del_cap));
            }
        }
    }
    hipEvent_t event() {
        if (pool_used == pool.size()) {
            hipEvent_t e;
            PSL_HIP(hipEventCreate(&e));
            pool.push_back(e);
        }
        return pool[pool_used++];
    }
    int timed_pair(int phase) {
        const int a = int(pool_used);
        event();
        event();
        timed.push_back({phase, a, a + 1});
        return int(timed.size()) - 1;
    }
};

namespace {

// Pipelines in use: as many as asked, but never more than the batches of a
// replica, so that no pipeline's stream joins a capture without work.
int n_pipes_of(const psl_run_opts& o, const psl_plan* plan) {
    const int want = o.pipelines >= 2 ? o.pipelines : 1;
    return int(std::max<size_t>(1, std::min<size_t>(size_t(want), plan->batches.size())));
}

// Enqueues all launches of replicas [rep0, rep0 + n_rep) on stream s; with
// several pipelines the batches of each replica fork onto the pipelines' streams
// and join back on s before the replica's fold.
void enqueue(Runner& R, psl_plan* plan, const psl_phantom* ph, psl_tally* tally,
             const psl_transport_params* prm, const psl_run_opts& o, uint32_t rep0, uint32_t n_rep,
             hipStream_t s) {
    uint32_t* rep = R.rep.as<uint32_t>();
    const int np = n_pipes_of(o, plan);
    hipLaunchKernelGGL(k_set_u32, dim3(1), dim3(64), 0, s, rep, rep0);
    const size_t nb = plan->batches.size();
    // The schedule (pipelines of the batches, fork / join / fold order) is
    // built and checked as host data first, then executed.  Batches go
    // largest first onto the least loaded pipeline (cost ~ histories), so
    // that the pipelines finish a replica together; n_pipes_of never gives a
    // pipeline without a batch.
    std::vector<uint32_t> sizes(nb);
    for (size_t i = 0; i < nb; ++i) sizes[i] = plan->batches[i].n;
    const std::vector<SchedOp> ops = build_schedule(sizes.data(), nb, np, n_rep);
    const std::string bad = check_schedule(ops, nb, np, n_rep);
    PSL_CHECK(bad.empty(), "launch schedule: %s", bad.c_str());
    for (const SchedOp& op : ops) {
        if (op.kind == SchedOp::kFork) {
            PSL_HIP(hipEventRecord(R.fork, s));
            for (int p = 0; p < np; ++p) PSL_HIP(hipStreamWaitEvent(R.pipes[p].st, R.fork, 0));
        } else if (op.kind == SchedOp::kJoin) {
            for (int p = 0; p < np; ++p) {
                PSL_HIP(hipEventRecord(R.pipes[p].join, R.pipes[p].st));
                PSL_HIP(hipStreamWaitEvent(s, R.pipes[p].join, 0));
            }
        } else if (op.kind == SchedOp::kFold) {
            int tf = -1;
            if (o.timing) {
                tf = R.timed_pair(kFold);
                PSL_HIP(hipEventRecord(R.pool[R.timed[tf][1]], s));
            }
            launch_fold(tally, s);
            if (o.timing) PSL_HIP(hipEventRecord(R.pool[R.timed[tf][2]], s));
        } else if (op.kind == SchedOp::kNextRep) {
            hipLaunchKernelGGL(k_inc_u32, dim3(1), dim3(64), 0, s, rep);
        } else {
            const size_t i = size_t(op.batch);
            const psl_batch& b = plan->batches[i];
            Pipe& P = R.pipes[size_t(op.pipe)];
            hipStream_t q = np > 1 ? P.st : s;
            P.phs.ptype = b.stype == 2 ? 1 : 0;
            int ts = -1;
            if (o.timing) {
                ts = R.timed_pair(kSample);
                PSL_HIP(hipEventRecord(R.pool[R.timed[ts][1]], q));
            }
            // dense output, tags only for rejected histories: no stack atomics
            launch_sample(plan, ph, 0, rep, b.h0, b.n, plan->batch_jlo[i], plan->batch_jhi[i],
                          b.stype, o.seed, &P.phs, 2, tally, q);
            if (o.timing) PSL_HIP(hipEventRecord(R.pool[R.timed[ts][2]], q));
            PhaseEvents ev{};
            if (o.timing) {
                const int tp = b.stype == 2 ? -1 : R.timed_pair(kPhoton);
                const int tso = R.timed_pair(kSort);
                const int tel = R.timed_pair(kElectron);
                if (tp >= 0) {
                    ev.photon0 = R.pool[R.timed[tp][1]];
                    ev.photon1 = R.pool[R.timed[tp][2]];
                }
                ev.sort0 = R.pool[R.timed[tso][1]];
                ev.sort1 = R.pool[R.timed[tso][2]];
                ev.electron0 = R.pool[R.timed[tel][1]];
                ev.electron1 = R.pool[R.timed[tel][2]];
            }
            launch_transport(ph, &P.phs, &P.els, tally, P.ws, prm, o.seed, q,
                             o.sort_electrons != 0, o.lane_load > 0 ? o.lane_load : 4,
                             o.timing ? &ev : nullptr, o.max_batch);
        }
    }
    PSL_HIP(hipGetLastError());
}

void run_impl(psl_plan* plan, const psl_phantom* ph, psl_tally* tally,
              const psl_transport_params* prm, const psl_run_opts& o, uint32_t rep0,
              uint32_t n_rep, hipStream_t user) {
    PSL_CHECK(o.max_batch >= 64, "max_batch must be >= 64");
    PSL_CHECK(o.band_width >= 1, "band_width must be >= 1");
    PSL_CHECK(o.lane_load >= 0 && o.lane_load <= 4096, "lane_load must be in [0, 4096]");
    PSL_CHECK(o.pipelines >= 0 && o.pipelines <= kMaxPipes, "pipelines must be 0, 1 or 2");
    PSL_CHECK(tally->phantom == ph, "tally belongs to another phantom");
    PSL_CHECK(prm->e_cut_photon > 0.f && prm->e_cut_electron > 0.f && prm->step_frac > 0.f &&
                  prm->step_frac < 1.f,
              "bad transport parameters");
    PSL_CHECK(tally->imap || plan->n_cols == 1 ||
                  std::all_of(plan->col_weight.begin(), plan->col_weight.end(),
                              [&](double c) { return c == plan->col_weight[0]; }),
              "a voxel tally needs an Eq. (3) plan");
    PSL_CHECK(!tally->imap || plan->n_cols <= tally->n_cols, "plan has more columns than the tally");
    if (!tally->runner) tally->runner = new Runner();
    Runner& R = *tally->runner;
    R.init();
    if (plan->cur_max_batch != o.max_batch || plan->cur_band_width != o.band_width) {
        int64_t nb = 0;
        const int rc = psl_plan_set_batching(plan, o.max_batch, o.band_width, &nb);
        if (rc != PSL_OK) fail(rc, "%s", psl_last_error());
    }
    // every push costs the photon at least the electron cut-off; one more
    // entry per photon covers the unused ends of the waves' reserved chunks
    const double emax = plan->model->e_max;
    const uint32_t per = uint32_t(std::max(1.0, std::floor(emax / prm->e_cut_electron))) + 1;
    const uint64_t el_need = uint64_t(o.max_batch) * per;
    PSL_CHECK(el_need < (uint64_t(1) << 32), "electron stack would exceed 2^32 entries");
    // annihilation photons take ids g | (2 sub + k) << 48
    PSL_CHECK(!(prm->physics & kPhysPair) ||
                  double(plan->n_hist) * double(plan->n_replica) < double(uint64_t(1) << 48),
              "pair production needs history ids below 2^48");
    PSL_CHECK(o.max_batch <= (1u << 30), "max_batch too large");
    R.ensure_stacks(n_pipes_of(o, plan), o.max_batch, uint32_t(el_need), prm->physics);
    ensure_physics(const_cast<psl_phantom*>(ph), prm);
    ensure_device(plan);

    R.timed.clear();
    R.pool_used = 0;
    // HIP events recorded inside a captured graph carry no timestamps, so a
    // timed run always launches eagerly, with an event pair around each kernel
    if (!o.use_graph || o.timing) {
        enqueue(R, plan, ph, tally, prm, o, rep0, n_rep, user);
        PSL_HIP(hipEventRecord(R.done, user));
        return;
    }
    GraphKey k;
    std::memset(&k, 0, sizeof k);   // padding takes part in the comparison
    k.plan = plan;
    k.phantom = ph;
    k.max_batch = o.max_batch;
    k.band_width = o.band_width;
    k.sort = o.sort_electrons;
    k.lane_load = o.lane_load;
    k.timing = o.timing;
    k.rep0 = rep0;
    k.n_rep = n_rep;
    k.seed = o.seed;
    k.n_hist = plan->n_hist;
    k.cut_e = prm->e_cut_electron;
    k.cut_g = prm->e_cut_photon;
    k.frac = prm->step_frac;
    k.ms = prm->ms_enable;
    k.dens = prm->density_effect;
    k.physics = prm->physics;
    k.tab_gen = ph->tab_gen;
    k.rec = tally->rec;
    k.pipes = n_pipes_of(o, plan);
    k.ph_cap = R.pipes[0].ph_cap;
    k.el_cap = R.pipes[0].el_cap;
    k.n_batches = plan->batches.size();
    if (!(R.have_graph && R.key == k)) {
        R.drop_graph();
        PSL_HIP(hipStreamBeginCapture(R.cs, hipStreamCaptureModeThreadLocal));
        try {
            enqueue(R, plan, ph, tally, prm, o, rep0, n_rep, R.cs);
        } catch (...) {
            hipGraph_t g = nullptr;
            (void)hipStreamEndCapture(R.cs, &g);
            if (g) (void)hipGraphDestroy(g);
            throw;
        }
        PSL_HIP(hipStreamEndCapture(R.cs, &R.graph));
        PSL_HIP(hipGraphInstantiate(&R.exec, R.graph, nullptr, nullptr, 0));
        std::memcpy(&R.key, &k, sizeof k);
        R.have_graph = true;
    }
    PSL_HIP(hipEventRecord(R.start, user));
    PSL_HIP(hipStreamWaitEvent(R.cs, R.start, 0));
    PSL_HIP(hipGraphLaunch(R.exec, R.cs));
    PSL_HIP(hipEventRecord(R.done, R.cs));
    PSL_HIP(hipStreamWaitEvent(user, R.done, 0));
}

}  // namespace
}  // namespace psl

using namespace psl;

psl_tally::~psl_tally() { delete runner; }

extern "C" int psl_run(psl_plan* plan, const psl_phantom* phantom, psl_tally* tally,
                       const psl_transport_params* params, const psl_run_opts* opts, void* stream) {
    return guarded([&] {
        PSL_CHECK(plan && phantom && tally && params && opts, "psl_run: null argument");
        run_impl(plan, phantom, tally, params, *opts, 0, plan->n_replica,
                 static_cast<hipStream_t>(stream));
    });
}

extern "C" int psl_run_get_timing(psl_tally* tally, psl_run_timing* out) {
    return guarded([&] {
        PSL_CHECK(tally && out, "null argument");
        std::memset(out, 0, sizeof *out);
        if (!tally->runner) return;
        Runner& R = *tally->runner;
        PSL_HIP(hipEventSynchronize(R.done));
        PSL_HIP(hipDeviceSynchronize());
        for (const auto& t : R.timed) {
            float ms = 0.f;
            PSL_HIP(hipEventElapsedTime(&ms, R.pool[t[1]], R.pool[t[2]]));
            out->ms[t[0]] += ms;
            out->launches[t[0]] += 1;
        }
    });
}

extern "C" int psl_autotune(psl_plan* plan, const psl_phantom* phantom, psl_tally* tally,
                            const psl_transport_params* params, uint64_t seed,
                            const uint32_t* max_batch, int32_t n_m, const int32_t* band_width,
                            int32_t n_w, const int32_t* lane_load, int32_t n_l, uint32_t replica,
                            psl_run_opts* best, double* ms_out) {
    return guarded([&] {
        PSL_CHECK(plan && phantom && tally && params && max_batch && band_width && lane_load &&
                      best,
                  "psl_autotune: null argument");
        PSL_CHECK(n_m >= 1 && n_w >= 1 && n_l >= 1, "empty candidate set");
        PSL_CHECK(replica < plan->n_replica, "replica out of range");
        hipEvent_t e0, e1;
        PSL_HIP(hipEventCreate(&e0));
        PSL_HIP(hipEventCreate(&e1));
        std::vector<psl_run_opts> cand;
        std::vector<double> times;
        for (int i = 0; i < n_m; ++i)
            for (int j = 0; j < n_w; ++j)
              for (int l = 0; l < n_l; ++l)
                for (int srt = 0; srt < 2; ++srt)
                  for (int pp = 1; pp <= kMaxPipes; ++pp) {
                    psl_run_opts o{};
                    o.max_batch = max_batch[i];
                    o.band_width = band_width[j];
                    o.lane_load = lane_load[l];
                    o.pipelines = pp;
                    o.use_graph = 1;
                    o.sort_electrons = srt;
                    o.timing = 0;
                    o.seed = seed;
                    // first launch captures and warms up, the second is timed
                    run_impl(plan, phantom, tally, params, o, replica, 1, nullptr);
                    PSL_HIP(hipEventRecord(e0, nullptr));
                    run_impl(plan, phantom, tally, params, o, replica, 1, nullptr);
                    PSL_HIP(hipEventRecord(e1, nullptr));
                    PSL_HIP(hipEventSynchronize(e1));
                    float ms = 0.f;
                    PSL_HIP(hipEventElapsedTime(&ms, e0, e1));
                    if (ms_out) ms_out[(((i * n_w + j) * n_l + l) * 2 + srt) * kMaxPipes + (pp - 1)] = ms;
                    cand.push_back(o);
                    times.push_back(ms);
                }
        // Second round: the candidates within 5 % of the fastest are timed
        // again over three back-to-back replays (a single replay leaves a few
        // percent of noise and misses the sustained rate); the pick is the
        // first of them in the order of the arrays (sort off and one pipeline
        // first) within 1 % of the fastest, so that near-ties resolve the same
        // way from run to run.
        const double best_ms = *std::min_element(times.begin(), times.end());
        std::vector<size_t> fin;
        for (size_t c = 0; c < cand.size(); ++c)
            if (times[c] <= 1.05 * best_ms) fin.push_back(c);
        std::vector<double> t2(fin.size());
        for (size_t k = 0; k < fin.size(); ++k) {
            const psl_run_opts& o = cand[fin[k]];
            run_impl(plan, phantom, tally, params, o, replica, 1, nullptr);
            PSL_HIP(hipEventRecord(e0, nullptr));
            for (int rep = 0; rep < 3; ++rep) run_impl(plan, phantom, tally, params, o, replica, 1, nullptr);
            PSL_HIP(hipEventRecord(e1, nullptr));
            PSL_HIP(hipEventSynchronize(e1));
            float ms = 0.f;
            PSL_HIP(hipEventElapsedTime(&ms, e0, e1));
            t2[k] = ms / 3.0;
        }
        const double best2 = *std::min_element(t2.begin(), t2.end());
        for (size_t k = 0; k < fin.size(); ++k)
            if (t2[k] <= 1.01 * best2) {
                *best = cand[fin[k]];
                break;
            }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        const int rc = tally_dose(tally, PSL_TALLY_RESET, nullptr, nullptr, nullptr, nullptr);
        if (rc != PSL_OK) fail(rc, "%s", psl_last_error());
        PSL_HIP(hipDeviceSynchronize());
        if (tally->runner) tally->runner->drop_graph();
    });
}
