// Transport and tally kernels.
//
// Photons: Woodcock (delta) tracking with the majorant mu_max(E) = rho_max n_e
// sigma_KN(E); a tentative collision is real with probability rho_v / rho_max;
// Compton scattering angle by Kahn's rejection method for the Klein-Nishina
// distribution; Compton electrons at or above the electron cut-off are pushed
// onto an electron stack, below it deposited on the spot.
// Electrons: continuous slowing down along straight steps that end at the
// exit face of the current voxel or after losing a fraction of the energy
// (T' = R^-1(R(T) - rho s)); Highland Gaussian multiple-scattering deflection
// after each step.  Deposits accumulate per lane while the electron stays in
// one voxel and are flushed with one FP32 atomic when it leaves.
// Between the two, electrons are grouped by energy band (counting sort) so
// that the waves of the electron kernel hold particles of similar range.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>

#include "device.hpp"

namespace psl {
namespace {

constexpr float kMe = 0.51099895f;
constexpr float kX0Water = 36.08f;      // g/cm^2
constexpr int kMaxElectronSteps = 100000;
constexpr int kMaxPhotonSteps = 1000000;   // safety bounds: never reached by valid input
constexpr int kMaxKahnTrials = 1000;
constexpr int kBands = kSortBands;
constexpr int kBlock = 256;
// LDS uniform buffers per lane (ring slots) of the photon and electron kernels
constexpr int kPhotonPool = 16;
constexpr int kElectronPool = 8;
// idle lanes of an electron-kernel wavefront that trigger a refill
constexpr int kRefillLanes = 8;

struct Stack {
    float *x, *y, *z, *u, *v, *w, *e;
    uint64_t* hid;
    uint32_t* tag;
    uint32_t* count;
    uint32_t capacity;
};

Stack to_stack(const psl_particles* p) {
    return Stack{p->x, p->y, p->z, p->u, p->v, p->w, p->e, p->hid, p->tag, p->count, p->capacity};
}

struct TransportArgs {
    Stack in;
    Stack el;                  // electron stack (photon kernel output / electron kernel input)
    const uint32_t* perm;      // electron order (nullable: identity)
    uint32_t* queue;           // [0] photon, [1] electron work-queue heads (zeroed per launch)
    PhantomDev ph;
    PhysicsDev phys;
    TallyDev tally;
    float e_cut_e, e_cut_g, step_frac;
    int ms;
    uint32_t seed_lo, seed_hi;
    uint32_t push_chunk;       // electron-stack entries a wave reserves per atomic
    Stack ann;                 // photons out of the electron kernel: annihilation and
                               // bremsstrahlung (count null: none expected)
    uint32_t secondary;        // photon kernel: the input holds secondary photons
    // electron hard events (kPhysDelta | kPhysBrem bits; 0: none): delta
    // electrons go to el_next; the pass's generation decides whether its
    // secondaries are followed (gen + 1 <= kGenMax) or deposited
    uint32_t hard;
    uint32_t gen;
    Stack el_next;
};

// ---- hardware transcendentals ---------------------------------------------
// Sine and cosine of a whole turn times r (v_sin_f32 / v_cos_f32 take their
// argument in revolutions, |r| <= 256); reciprocal, natural logarithm and
// square root from v_rcp_f32, v_log_f32 and v_sqrt_f32 without the range
// scaling the library wraps around them for denormal arguments, which the
// transport never produces (energies >= the cut-offs, lengths and 1 - u >=
// 2^-24, or guarded zeros).  About 1 ulp, far below the statistical noise.
__device__ __forceinline__ void sincos_turn(float r, float& s, float& c) {
    s = __builtin_amdgcn_sinf(r);
    c = __builtin_amdgcn_cosf(r);
}
__device__ __forceinline__ float hw_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float hw_log(float x) {
    return __builtin_amdgcn_logf(x) * 0.693147180559945309f;
}
__device__ __forceinline__ float hw_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }

// ---- table lookups (linear interpolation) ---------------------------------
__device__ __forceinline__ float lerp_tab(const float* tab, int n, float x) {
    x = fminf(fmaxf(x, 0.f), float(n - 1) - 1e-3f);
    const int i = int(x);
    const float f = x - float(i);
    return fmaf(f, tab[i + 1] - tab[i], tab[i]);
}

__device__ __forceinline__ float kn_mu(const PhysicsDev& P, const float* tab, float e) {
    return lerp_tab(tab, KN_TAB_N, (hw_log(e) - P.kn_lne0) * P.kn_inv_dlne);
}

__device__ __forceinline__ float csda_range(const PhysicsDev& P, const float* tab, float t) {
    if (!(t > P.t_cut)) return 0.f;
    return lerp_tab(tab, RNG_TAB_N, (hw_log(t) - P.rng_lnt0) * P.rng_inv_dlnt);
}

__device__ __forceinline__ float csda_energy(const PhysicsDev& P, const float* tab, float r) {
    if (!(r > 0.f)) return P.t_cut;
    return lerp_tab(tab, INV_TAB_N, (hw_log(r + P.r_off) - P.inv_u0) * P.inv_inv_du);
}

// Cumulative attenuations per unit density at photon energy e (x Compton,
// y + photoelectric, z + Rayleigh, w the total), linear in ln E.
__device__ __forceinline__ float4 xs_at(const PhysicsDev& P, const float4* tab, float e) {
    float x = (hw_log(e) - P.kn_lne0) * P.kn_inv_dlne;
    x = fminf(fmaxf(x, 0.f), float(KN_TAB_N - 1) - 1e-3f);
    const int i = int(x);
    const float f = x - float(i);
    const float4 lo = tab[i], hi = tab[i + 1];
    return make_float4(fmaf(f, hi.x - lo.x, lo.x), fmaf(f, hi.y - lo.y, lo.y),
                       fmaf(f, hi.z - lo.z, lo.z), fmaf(f, hi.w - lo.w, lo.w));
}

// Rayleigh: cumulative A(t) of the squared form factor (linear in t between
// the table's nodes: 0, then log-spaced from node 1).
__device__ __forceinline__ float ray_cumulative(const PhysicsDev& P, float t) {
    const float t1 = P.ray_t[1];
    if (t <= t1) return P.ray_a[1] * (t / t1);
    float x = (hw_log(t) - P.ray_lt1) * P.ray_inv_dlt + 1.f;
    x = fminf(x, float(RAY_TAB_N - 1) - 1e-3f);
    const int i = max(int(x), 1);
    const float ta = P.ray_t[i], tb = P.ray_t[i + 1];
    const float f = fminf(fmaxf((t - ta) / (tb - ta), 0.f), 1.f);
    return fmaf(f, P.ray_a[i + 1] - P.ray_a[i], P.ray_a[i]);
}

// Rayleigh: the t at which A(t) reaches `target` (binary search over the
// table, linear in t between nodes).
__device__ __forceinline__ float ray_t_at(const PhysicsDev& P, float target) {
    int lo = 0, hi = RAY_TAB_N - 1;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (P.ray_a[mid] <= target) lo = mid;
        else hi = mid;
    }
    const float a0 = P.ray_a[lo], a1 = P.ray_a[hi];
    const float f = a1 > a0 ? fminf(fmaxf((target - a0) / (a1 - a0), 0.f), 1.f) : 0.f;
    return fmaf(f, P.ray_t[hi] - P.ray_t[lo], P.ray_t[lo]);
}

// ---- geometry -------------------------------------------------------------
__device__ __forceinline__ void rotate(float& u, float& v, float& w, float cos_t, float cphi,
                                       float sphi) {
    const float sin_t = hw_sqrt(fmaxf(0.f, 1.f - cos_t * cos_t));
    float nu, nv, nw;
    // transverse length from u and v (exact next to the axis, unlike 1 - w^2)
    const float t = hw_sqrt(u * u + v * v);
    if (t > 1e-30f) {
        const float it = hw_rcp(t);
        nu = u * cos_t + sin_t * (u * w * cphi - v * sphi) * it;
        nv = v * cos_t + sin_t * (v * w * cphi + u * sphi) * it;
        nw = w * cos_t - sin_t * cphi * t;
    } else {
        nu = sin_t * cphi;
        nv = sin_t * sphi;
        nw = (w > 0.f ? 1.f : -1.f) * cos_t;
    }
    const float inv = rsqrtf(nu * nu + nv * nv + nw * nw);
    u = nu * inv;
    v = nv * inv;
    w = nw * inv;
}

// Tally cell of voxel v for a particle of column `tag` (index-map mode: the
// voxel's row and the column), or -1 when the voxel is not tallied or the
// column is beyond the tally (counted as an overflow).
__device__ __forceinline__ int tally_cell(const TallyDev& T, int v, uint32_t tag) {
    if (!T.imap) return v;
    const int row = T.imap[v];
    if (row <= 0) return -1;
    const int col = int(tag & kColumnMask);
    if (col >= T.n_cols) {
        // particle tag from a plan with more columns than this tally
        atomicAdd(T.counters + C_OVERFLOW, 1ull);
        return -1;
    }
    return (row - 1) * T.n_cols + col;
}

// Appends cell c to the deposit recording (kRec builds only).
__device__ __forceinline__ void record_cell(const TallyDev& T, int c) {
    const uint32_t slot = atomicAdd(T.rec_count, 1u);
    if (slot < T.rec_cap) T.rec[slot] = uint32_t(c);
}

template <bool kRec>
__device__ __forceinline__ void deposit(const TallyDev& T, int v, uint32_t tag, float e,
                                        uint32_t& n_atomic) {
    if (e == 0.f) return;
    const int c = tally_cell(T, v, tag);
    if (c < 0) return;
    if constexpr (kRec) record_cell(T, c);
    atomicAdd(T.grid + c, e);
    ++n_atomic;
}

// Three deposits (v < 0: none; the first two of particle tag01, the third of
// tag2) whose index-map lookups are all issued before any atomic, so that no
// lookup waits behind an atomic.
template <bool kRec>
__device__ __forceinline__ void deposit3(const TallyDev& T, int v0, float e0, int v1, float e1,
                                         uint32_t tag01, int v2, float e2, uint32_t tag2,
                                         uint32_t& n_atomic) {
    const int c0 = v0 >= 0 && e0 != 0.f ? tally_cell(T, v0, tag01) : -1;
    const int c1 = v1 >= 0 && e1 != 0.f ? tally_cell(T, v1, tag01) : -1;
    const int c2 = v2 >= 0 && e2 != 0.f ? tally_cell(T, v2, tag2) : -1;
    if (c0 >= 0) {
        if constexpr (kRec) record_cell(T, c0);
        atomicAdd(T.grid + c0, e0);
        ++n_atomic;
    }
    if (c1 >= 0) {
        if constexpr (kRec) record_cell(T, c1);
        atomicAdd(T.grid + c1, e1);
        ++n_atomic;
    }
    if (c2 >= 0) {
        if constexpr (kRec) record_cell(T, c2);
        atomicAdd(T.grid + c2, e2);
        ++n_atomic;
    }
}

// Waits until every vector memory operation of the wave has completed
// (s_waitcnt vmcnt(0), expcnt and lgkmcnt left free).  Loads, stores and
// atomics share one in-order counter, so a load that is used after a later
// store or atomic can only be waited on together with it; the kernels below
// end the loads of an iteration with this wait before issuing its deposits
// and stores, so that the next iteration uses its loaded values without
// waiting for writes it has just made.
__device__ __forceinline__ void wait_loads() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// ---- work queue -------------------------------------------------------------
// Entries [0, n) of a stack are split in two.  Three quarters go out
// statically, an equal share to each wave of the grid, with no atomics.  The
// rest is handed out dynamically, kChunk entries per returning atomic on one
// global counter, which evens out the waves' differing amounts of work; each
// such atomic stalls its wave for a device-wide round trip, so they are kept
// to the tail.  A wave hands its entries to its idle lanes over the
// following iterations.
constexpr uint32_t kChunk = 128;
constexpr uint32_t kNone = 0xFFFFFFFFu;

struct WaveQueue {
    uint32_t base, left, dyn0;   // dyn0: first entry of the dynamic part
    uint32_t wave, waves, share, slot;
    bool drained;
    __device__ explicit WaveQueue(uint32_t n) {
        const uint32_t per_block = blockDim.x >> 6;
        waves = gridDim.x * per_block;
        wave = blockIdx.x * per_block + (threadIdx.x >> 6);
        share = uint32_t(uint64_t(n) * 3u / 4u / waves);
        base = wave * share;
        left = share;
        dyn0 = waves * share;
        drained = false;
        // the wave's place in the interleave: workgroups go to the eight
        // XCDs in turn, so the waves of one XCD take neighbouring positions
        // and share cache lines in that XCD's L2 (a bijection of the waves
        // whatever the placement)
        slot = wave;
        if ((gridDim.x & 7u) == 0u) {
            const uint32_t xcd = blockIdx.x & 7u, per_xcd = (gridDim.x >> 3) * per_block;
            slot = xcd * per_xcd + (blockIdx.x >> 3) * per_block + (threadIdx.x >> 6);
        }
    }
    // Stack position of queue entry q for a stack ordered roughly longest
    // work first: the static shares interleave (the wave's t-th entry is
    // position t * waves + slot), so that every wave gets the same mix and
    // starts with its longest histories; the dynamic part keeps its order.
    __device__ __forceinline__ uint32_t strided(uint32_t q) const {
        return q < dyn0 ? (q - wave * share) * waves + slot : q;
    }
};

__device__ __forceinline__ uint32_t take_work(bool need, WaveQueue& q, uint32_t* head, uint32_t n) {
    const unsigned long long m = __ballot(need);
    if (m == 0ull) return kNone;
    const int lane = threadIdx.x & 63;
    if (q.left == 0 && !q.drained) {
        uint32_t b = 0;
        if (lane == 0) b = atomicAdd(head, kChunk);
        b = q.dyn0 + __shfl(b, 0, 64);
        if (b >= n) {
            q.drained = true;
        } else {
            q.base = b;
            q.left = min(kChunk, n - b);
        }
    }
    const uint32_t give = min(uint32_t(__popcll(m)), q.left);
    const uint32_t rank = uint32_t(__popcll(m & ((1ull << lane) - 1ull)));
    const uint32_t idx = (need && rank < give) ? q.base + rank : kNone;
    q.base += give;
    q.left -= give;
    return idx;
}

// ---- photon kernel --------------------------------------------------------
// One lane follows one photon at a time through Woodcock flights and Compton
// collisions.  A lane's photon is a small state machine (flight, Kahn trials,
// scattering) that advances as far as the uniforms topped up at the start of
// the iteration allow and resumes in the next iteration, so every Philox block
// of the wavefront is generated at the one top-up point.
// With the optional processes (kFull) a real collision picks its process
// with one more uniform; Rayleigh trials (two uniforms each) and the
// deflection, and the pair's energy-sharing trials (two uniforms each) and the
// positron's push, are further phases of the same machine.
enum PhotonPhase : uint32_t {
    kFlight = 0, kKahn = 1, kScatter = 2, kRayleigh = 3, kRayTurn = 4, kPair = 5, kPairPositron = 6
};

template <bool kRec, bool kFull>
__global__ void __launch_bounds__(kBlock) k_photon(TransportArgs a) {
    __shared__ float s_kn[kFull ? 1 : KN_TAB_N];
    __shared__ float4 s_xs[kFull ? KN_TAB_N : 1];
    __shared__ float s_pool[kPhotonPool * kBlock];
    if constexpr (kFull) {
        for (int i = threadIdx.x; i < KN_TAB_N; i += blockDim.x) s_xs[i] = a.phys.xs[i];
    } else {
        for (int i = threadIdx.x; i < KN_TAB_N; i += blockDim.x) s_kn[i] = a.phys.kn[i];
    }
    __syncthreads();

    const PhantomDev& G = a.ph;
    const uint32_t n = min(*a.in.count, a.in.capacity);
    dev::LocalStats ls;
    double& esc_g = ls.l[L_ESC_G];
    double& dep = ls.l[L_DEP];
    uint32_t &c_wc = ls.c[C_WC_STEPS], &c_real = ls.c[C_REAL], &c_push = ls.c[C_E_PUSHED],
             &c_local = ls.c[C_E_LOCAL], &c_atom = ls.c[C_DEPOSITS],
             &c_unc = ls.c[C_ESC_UNCOLLIDED], &c_kahn = ls.c[C_KAHN_TRIALS],
             &c_over = ls.c[C_OVERFLOW], &c_photo = ls.c[C_PHOTO], &c_ray = ls.c[C_RAYLEIGH],
             &c_pair = ls.c[C_PAIR];
    // electron-stack slots reserved by this wave and not used yet
    uint32_t el_base = 0, el_left = 0;
    // per-lane photon state
    float px = 0.f, py = 0.f, pz = 0.f, du = 0.f, dv = 0.f, dw = 0.f, e = 0.f;
    // Kahn variable E/E' of the current collision; with kFull also the bound
    // of the Rayleigh trials' cumulative, then the accepted cos theta, or the
    // pair positron's kinetic energy
    float kx = 1.f;
    uint64_t g = 0;
    uint32_t tag = 0, n_push = 0, phase = kFlight, trials = 0;
    int steps = 0, cv = 0;   // cv: voxel of the current collision
    bool collided = false, alive = false;
    WaveQueue wq(n);
    dev::PoolStream<kPhotonPool, kBlock> st(s_pool, a.seed_lo, a.seed_hi);
    // Order of an iteration: the physics step (no global writes), then the
    // refill of idle lanes (their loads are waited on), then this step's
    // global writes.  A load issued after a store or atomic can only be
    // waited on together with it (one in-order counter), so the refill's
    // wait covers the writes of the previous iteration, issued a whole step
    // earlier, rather than those just made.
    for (;;) {
        if (__ballot(alive) == 0ull && wq.drained && wq.left == 0) break;
        // a flight and its collision test (2), three Kahn trials (9) and the
        // azimuth (1) fit in one iteration
        st.topup(alive, kFull ? 13 : 12, 13);
        // this step's writes, deferred: one deposit, one electron
        int w_v = -1;
        float w_e = 0.f;
        uint32_t w_tag = tag;
        bool push = false;
        float qx = 0.f, qy = 0.f, qz = 0.f, te = 0.f, ex = 0.f, ey = 0.f, ez = 0.f;
        uint64_t w_g = g;
        uint32_t w_ptag = 0;
        if (alive && phase == kFlight) {
            if (!(e >= a.e_cut_g) || steps >= kMaxPhotonSteps) {
                // below the cut-off on entry, or the safety bound: absorb here
                const int vx = min(max(int(floorf((px - G.origin[0]) * G.inv_vox[0])), 0), G.nx - 1);
                const int vy = min(max(int(floorf((py - G.origin[1]) * G.inv_vox[1])), 0), G.ny - 1);
                const int vz = min(max(int(floorf((pz - G.origin[2]) * G.inv_vox[2])), 0), G.nz - 1);
                const float ee = isfinite(e) ? e : 0.f;
                w_v = (vz * G.ny + vy) * G.nx + vx;
                w_e = ee;
                dep += ee;
                c_over += steps >= kMaxPhotonSteps ? 1u : 0u;
                alive = false;
            } else {
                ++steps;
                // one Woodcock flight
                float4 xs4;
                float mu;
                if constexpr (kFull) {
                    xs4 = xs_at(a.phys, s_xs, e);
                    mu = xs4.w * G.rho_max;
                } else {
                    mu = kn_mu(a.phys, s_kn, e) * G.rho_max;
                }
                const float s = -hw_log(1.f - st.pop()) * hw_rcp(mu);
                px = fmaf(s, du, px);
                py = fmaf(s, dv, py);
                pz = fmaf(s, dw, pz);
                const float fx = floorf((px - G.origin[0]) * G.inv_vox[0]);
                const float fy = floorf((py - G.origin[1]) * G.inv_vox[1]);
                const float fz = floorf((pz - G.origin[2]) * G.inv_vox[2]);
                if (!(fx >= 0.f && fx < float(G.nx) && fy >= 0.f && fy < float(G.ny) &&
                      fz >= 0.f && fz < float(G.nz))) {
                    esc_g += e;
                    c_unc += collided ? 0u : 1u;
                    alive = false;
                } else {
                    cv = (int(fz) * G.ny + int(fy)) * G.nx + int(fx);
                    ++c_wc;
                    // real collision if u < rho_v / rho_max; below the
                    // phantom's smallest ratio that holds in every voxel and
                    // the density is not read
                    const float u = st.pop();
                    if (u < G.real_min || u < G.dens[cv] * G.inv_rho_max) {
                        collided = true;
                        ++c_real;
                        phase = kKahn;
                        trials = 0;
                        if constexpr (kFull) {
                            // the process, in proportion to the attenuations
                            const float up = st.pop() * xs4.w;
                            if (up >= xs4.x) {
                                if (up < xs4.y) {
                                    // photoelectric absorption: the photoelectron
                                    // along the photon, the binding energy here
                                    ++c_photo;
                                    const float b = a.phys.photo_bind;
                                    const float tpe = e - b;
                                    if (tpe >= a.e_cut_e) {
                                        qx = du; qy = dv; qz = dw;
                                        te = tpe;
                                        ++n_push;
                                        ++c_push;
                                        push = true;
                                        ex = px; ey = py; ez = pz;
                                        w_ptag = tag | (n_push << 16);
                                        w_v = cv;
                                        w_e = b;
                                        dep += b;
                                    } else {
                                        w_v = cv;
                                        w_e = e;
                                        dep += e;
                                        ++c_local;
                                    }
                                    alive = false;
                                } else if (up < xs4.z) {
                                    ++c_ray;
                                    phase = kRayleigh;
                                    const float x0 = e * a.phys.ka0_per_mev;
                                    kx = ray_cumulative(a.phys, 4.f * x0 * x0);
                                } else {
                                    ++c_pair;
                                    phase = kPair;
                                }
                            }
                        }
                    }
                }
            }
        }
        if (alive && phase == kKahn) {
            // Kahn's method for x = E/E' in [1, 1 + 2k], three uniforms a
            // trial, at most three trials per iteration (a photon that needs
            // more goes on in the next one, so that the wavefront does not
            // loop for its few unlucky lanes).  Both proposals come from one
            // reciprocal and the lane selects, so the two branches of the
            // method do not diverge across the wavefront.
            const float k = e * (1.f / kMe);
            const float k2 = 2.f * k;
            const float ik = kMe * hw_rcp(e);
            const float p_a = (1.f + k2) * hw_rcp(9.f + k2);
            const float i1k2 = hw_rcp(1.f + k2);
            for (int tr = 0; tr < 3 && st.cnt >= 3u; ++tr) {
                const float r1 = st.pop(), r2 = st.pop(), r3 = st.pop();
                ++c_kahn;
                ++trials;
                const float xa = fmaf(k2, r2, 1.f);          // proposal of the first branch
                const float ia = hw_rcp(xa);
                const float xb = (1.f + k2) * ia;            // proposal of the second branch
                const float cb = 1.f - (xb - 1.f) * ik;
                const bool first = r1 <= p_a;
                const bool acc = first ? r3 <= 4.f * (ia - ia * ia)
                                       : r3 <= 0.5f * fmaf(cb, cb, xa * i1k2);
                kx = first ? xa : xb;
                if (acc || trials >= uint32_t(kMaxKahnTrials)) {
                    phase = kScatter;
                    break;
                }
            }
        }
        if (alive && phase == kScatter && st.cnt >= 1u) {
            const float cos_t = 1.f - (kx - 1.f) * kMe * hw_rcp(e);
            float sphi, cphi;
            sincos_turn(st.pop(), sphi, cphi);
            const float e1 = e * hw_rcp(kx);
            te = e - e1;
            float nu = du, nv = dv, nw = dw;
            rotate(nu, nv, nw, cos_t, cphi, sphi);
            if (te >= a.e_cut_e) {
                // electron direction from momentum conservation: p_e = E d - E' d'
                qx = e * du - e1 * nu;
                qy = e * dv - e1 * nv;
                qz = e * dw - e1 * nw;
                const float inv = rsqrtf(qx * qx + qy * qy + qz * qz);
                qx *= inv;
                qy *= inv;
                qz *= inv;
                ++n_push;
                ++c_push;
                push = true;
                ex = px; ey = py; ez = pz;
                w_ptag = tag | (n_push << 16);
            } else {
                w_v = cv;
                w_e = te;
                dep += te;
                ++c_local;
            }
            e = e1;
            du = nu; dv = nv; dw = nw;
            phase = kFlight;
            if (e < a.e_cut_g) {
                // absorbed where it scattered (same voxel as a local electron)
                w_v = cv;
                w_e += e;
                dep += e;
                alive = false;
            }
        }
        if constexpr (kFull) {
            if (alive && phase == kRayleigh) {
                // t = (q a0)^2 from the squared form factor below its bound
                // (kx), accepted with (1 + cos^2 theta) / 2
                const float x0 = e * a.phys.ka0_per_mev;
                const float inv2x2 = 0.5f * hw_rcp(x0 * x0);
                while (st.cnt >= 2u) {
                    const float u1 = st.pop(), u2 = st.pop();
                    const float t = ray_t_at(a.phys, u1 * kx);
                    const float c = fmaxf(1.f - t * inv2x2, -1.f);
                    if (u2 <= 0.5f * (1.f + c * c)) {
                        kx = c;
                        phase = kRayTurn;
                        break;
                    }
                }
            }
            if (alive && phase == kRayTurn && st.cnt >= 1u) {
                float sphi, cphi;
                sincos_turn(st.pop(), sphi, cphi);
                rotate(du, dv, dw, kx, cphi, sphi);
                phase = kFlight;
            }
            if (alive && phase == kPair) {
                // the electron's share eps of E - 2 mc^2, density 1 - 4/3 eps (1 - eps)
                while (st.cnt >= 2u) {
                    const float u1 = st.pop(), u2 = st.pop();
                    if (u2 <= 1.f - (4.f / 3.f) * u1 * (1.f - u1)) {
                        const float kin = e - 2.f * kMe;
                        const float tm = u1 * kin;
                        kx = kin - tm;
                        if (tm >= a.e_cut_e) {
                            qx = du; qy = dv; qz = dw;
                            te = tm;
                            ++n_push;
                            ++c_push;
                            push = true;
                            ex = px; ey = py; ez = pz;
                            w_ptag = tag | (n_push << 16);
                        } else {
                            w_v = cv;
                            w_e = tm;
                            dep += tm;
                            ++c_local;
                        }
                        phase = kPairPositron;
                        break;
                    }
                }
            } else if (alive && phase == kPairPositron) {
                // the positron, pushed whatever its energy: it annihilates
                // where it stops
                qx = du; qy = dv; qz = dw;
                te = kx;
                ++n_push;
                ++c_push;
                push = true;
                ex = px; ey = py; ez = pz;
                w_ptag = tag | kPositronBit | (n_push << 16);
                alive = false;
            }
        }
        // refill idle lanes from the wave's chunk of the photon stack: the
        // entry's tag and data are loaded together (one memory latency), the
        // data kept only if the tag marks a live entry
        {
            const uint32_t i = take_work(!alive, wq, a.queue, n);
            if (i != kNone) {
                const uint32_t tg = a.in.tag[i];
                const float nx = a.in.x[i], ny = a.in.y[i], nz = a.in.z[i];
                const float nu = a.in.u[i], nv = a.in.v[i], nw = a.in.w[i];
                const float ne = a.in.e[i];
                const uint64_t ng = a.in.hid[i];
                // the empty asm takes every loaded value, so that the
                // compiler keeps the data loads ahead of the tag test
                // instead of moving them into it (one wait for all)
                asm volatile("" ::"v"(tg), "v"(nx), "v"(ny), "v"(nz), "v"(nu), "v"(nv), "v"(nw),
                             "v"(ne), "v"(ng));
                const bool take = (tg >> 24) == 0u;   // skip entries marked rejected / empty
                px = take ? nx : px; py = take ? ny : py; pz = take ? nz : pz;
                du = take ? nu : du; dv = take ? nv : dv; dw = take ? nw : dw;
                e = take ? ne : e;
                g = take ? ng : g;
                if (take) {
                    tag = tg & 0xFFFFu;
                    st.init(g, dev::kTagTransport, 0);
                    n_push = 0;
                    steps = 0;
                    phase = kFlight;
                    // uncollided escapes are counted for source photons only
                    collided = a.secondary != 0u;
                    alive = true;
                }
            }
        }
        wait_loads();
        // this step's writes: the electron first (its chunk reservation
        // returns a value, which must not wait behind the deposit's atomic)
        // wave-convergent push: slots from the wave's reserved chunk of the
        // electron stack, a new chunk of push_chunk when it runs out
        const unsigned long long m = __ballot(push);
        if (m != 0ull) {
            const int lane = threadIdx.x & 63;
            const uint32_t k_push = uint32_t(__popcll(m));
            const uint32_t rank = uint32_t(__popcll(m & ((1ull << lane) - 1ull)));
            uint32_t fresh = 0;
            if (k_push > el_left) {
                if (lane == 0) fresh = atomicAdd(a.el.count, a.push_chunk);
                fresh = __shfl(fresh, 0, 64);
            }
            const uint32_t slot = rank < el_left ? el_base + rank : fresh + (rank - el_left);
            if (k_push > el_left) {
                el_base = fresh + (k_push - el_left);
                el_left = a.push_chunk - (k_push - el_left);
            } else {
                el_base += k_push;
                el_left -= k_push;
            }
            if (push) {
                if (slot < a.el.capacity) {
                    a.el.x[slot] = ex; a.el.y[slot] = ey; a.el.z[slot] = ez;
                    a.el.u[slot] = qx; a.el.v[slot] = qy; a.el.w[slot] = qz;
                    a.el.e[slot] = te;
                    a.el.hid[slot] = w_g;
                    a.el.tag[slot] = w_ptag;
                } else {
                    ++c_over;
                }
            }
        }
        if (w_v >= 0) deposit<kRec>(a.tally, w_v, w_tag, w_e, c_atom);
    }
    // the unused rest of the wave's last chunk stays in the stack as empty entries
    if (el_left > 0) {
        const int lane = threadIdx.x & 63;
        for (uint32_t j = uint32_t(lane); j < el_left; j += 64) {
            const uint32_t slot = el_base + j;
            if (slot < a.el.capacity) a.el.tag[slot] = 1u << 24;
        }
    }
    dev::flush_stats(a.tally.stats, ls);
}

// ---- electron energy bands (counting sort) --------------------------------
// Block b of a fixed grid of kSortBlocks owns the chunk [b c, (b+1) c) of the
// stack.  Pass 1 writes per-block band counts, pass 2 turns them into offsets
// (band-major, highest band first, so long-range electrons start first),
// pass 3 scatters the indices; only LDS atomics are used.

// log-spaced bands between the electron cut-off and the table top
__device__ __forceinline__ int band_of(float t, float lt0, float inv_w) {
    const int b = int((__logf(t) - lt0) * inv_w);
    return min(max(b, 0), kBands - 1);
}

// Lanes of a wave with the same band share one LDS atomic; returns the lane's
// slot relative to the LDS counter of its band.
__device__ __forceinline__ uint32_t wave_band_rank(bool valid, int b, uint32_t* s_cnt) {
    const int lane = threadIdx.x & 63;
    const unsigned long long below = (1ull << lane) - 1ull;
    bool pending = valid;
    uint32_t slot = 0;
    for (;;) {
        const unsigned long long act = __ballot(pending);
        if (act == 0ull) break;
        const int leader = __ffsll((long long)act) - 1;
        const int lb = __shfl(b, leader, 64);
        const unsigned long long mine = __ballot(pending && b == lb);
        uint32_t base = 0;
        if (lane == leader) base = atomicAdd(s_cnt + lb, uint32_t(__popcll(mine)));
        base = __shfl(base, leader, 64);
        if (pending && b == lb) {
            slot = base + uint32_t(__popcll(mine & below));
            pending = false;
        }
    }
    return slot;
}

__global__ void __launch_bounds__(kBlock) k_band_count(const float* e, const uint32_t* tag,
                                                      const uint32_t* count, uint32_t cap,
                                                      uint32_t* hist, float lt0, float inv_w) {
    __shared__ uint32_t s_cnt[kBands];
    if (threadIdx.x < kBands) s_cnt[threadIdx.x] = 0;
    __syncthreads();
    const uint32_t n = min(*count, cap);
    const uint32_t chunk = (n + kSortBlocks - 1) / kSortBlocks;
    const uint32_t i0 = blockIdx.x * chunk, i1 = min(i0 + chunk, n);
    for (uint32_t base = i0; base < i1; base += blockDim.x) {
        const uint32_t i = base + threadIdx.x;
        const bool valid = i < i1;
        // entries marked rejected / empty go to band 0, where the kernel skips them
        const int b = valid && (tag[i] >> 24) == 0u ? band_of(e[i], lt0, inv_w) : 0;
        wave_band_rank(valid, b, s_cnt);
    }
    __syncthreads();
    if (threadIdx.x < kBands) hist[threadIdx.x * kSortBlocks + blockIdx.x] = s_cnt[threadIdx.x];
}

// exclusive scan over (band descending, block ascending)
__global__ void __launch_bounds__(1024) k_band_scan(const uint32_t* hist, uint32_t* offs) {
    constexpr int kPer = kBands * kSortBlocks / 1024;
    __shared__ uint32_t s_sum[1024];
    uint32_t vals[kPer];
    uint32_t tot = 0;
    for (int k = 0; k < kPer; ++k) {
        const int pos = threadIdx.x * kPer + k;               // position in scan order
        const int band = kBands - 1 - pos / kSortBlocks, blk = pos % kSortBlocks;
        vals[k] = hist[band * kSortBlocks + blk];
        tot += vals[k];
    }
    s_sum[threadIdx.x] = tot;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const uint32_t v = threadIdx.x >= off ? s_sum[threadIdx.x - off] : 0u;
        __syncthreads();
        s_sum[threadIdx.x] += v;
        __syncthreads();
    }
    uint32_t run = s_sum[threadIdx.x] - tot;
    for (int k = 0; k < kPer; ++k) {
        const int pos = threadIdx.x * kPer + k;
        const int band = kBands - 1 - pos / kSortBlocks, blk = pos % kSortBlocks;
        offs[band * kSortBlocks + blk] = run;
        run += vals[k];
    }
}

__global__ void __launch_bounds__(kBlock) k_band_scatter(const float* e, const uint32_t* tag,
                                                        const uint32_t* count, uint32_t cap,
                                                        const uint32_t* offs, uint32_t* perm,
                                                        float lt0, float inv_w) {
    __shared__ uint32_t s_cnt[kBands];
    __shared__ uint32_t s_off[kBands];
    if (threadIdx.x < kBands) {
        s_cnt[threadIdx.x] = 0;
        s_off[threadIdx.x] = offs[threadIdx.x * kSortBlocks + blockIdx.x];
    }
    __syncthreads();
    const uint32_t n = min(*count, cap);
    const uint32_t chunk = (n + kSortBlocks - 1) / kSortBlocks;
    const uint32_t i0 = blockIdx.x * chunk, i1 = min(i0 + chunk, n);
    for (uint32_t base = i0; base < i1; base += blockDim.x) {
        const uint32_t i = base + threadIdx.x;
        const bool valid = i < i1;
        // entries marked rejected / empty go to band 0, where the kernel skips them
        const int b = valid && (tag[i] >> 24) == 0u ? band_of(e[i], lt0, inv_w) : 0;
        const uint32_t r = wave_band_rank(valid, b, s_cnt);
        if (valid) perm[s_off[b] + r] = i;
    }
}

// ---- electron kernel ------------------------------------------------------
// Distance along (dx, dy, dz) from p to the exit face of voxel i on one axis.
__device__ __forceinline__ void face_distance(float p, float d, int i, float o, float vx, int ax,
                                              float& sb, int& axis) {
    if (d != 0.f) {
        const float face = o + float(i + (d > 0.f ? 1 : 0)) * vx;
        const float t = (face - p) * hw_rcp(d);
        if (t < sb) {
            sb = t;
            axis = ax;
        }
    }
}

// Writes the two photons of a positron's annihilation at rest at (x, y, z):
// mc^2 each, back to back along an isotropic direction (cos theta = 2u - 1,
// azimuth u' in turns), ids g | (2 sub + k) << 48, the positron's column.
// ---- electron hard events ----------------------------------------------------
// Random stream of a secondary from a hard event (kind 1 delta electron, 2
// bremsstrahlung photon) or an annihilation photon of a secondary family
// (kind 3): the splitmix64 finaliser (Steele, Lea and Flood, OOPSLA 2014) of
// the parent's stream (g, sub), its event index j and the kind; the child
// keeps the history id (low 48 bits), takes 0x8000 | 15 hashed bits as the
// high 16 bits and 8 hashed bits as its sub (electrons).
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
__device__ __forceinline__ void child_id(uint64_t g, uint32_t sub, uint32_t j, uint32_t kind,
                                         uint64_t& g_out, uint32_t& sub_out) {
    const uint64_t h =
        mix64(mix64(g) ^ ((uint64_t(sub) << 32) | (uint64_t(j) << 8) | uint64_t(kind)));
    g_out = (g & 0xFFFFFFFFFFFFull) | (uint64_t(0x8000u | uint32_t(h & 0x7FFFu)) << 48);
    sub_out = uint32_t(h >> 16) & 0xFFu;
}

// Hard-event cross-sections per unit density (cm^2/g) at kinetic energy t:
// x Moller (transfers above the electron cut-off), y = x + bremsstrahlung
// (photons above the photon cut-off); linear in ln T between the range
// table's nodes.
__device__ __forceinline__ float2 hard_xs(const PhysicsDev& P, float t) {
    float x = (hw_log(t) - P.rng_lnt0) * P.rng_inv_dlnt;
    x = fminf(fmaxf(x, 0.f), float(RNG_TAB_N - 1) - 1e-3f);
    const int i = int(x);
    const float f = x - float(i);
    const float2 a = P.hard[i], b = P.hard[i + 1];
    return make_float2(fmaf(f, b.x - a.x, a.x), fmaf(f, b.y - a.y, a.y));
}

// Moller energy transfer eps = w / t in [tc / t, 1/2]: 1/eps^2 by inversion,
// kept with probability h(eps) / 2.25 (h = eps^2 times the cross-section's
// bracket, at most 2.25 on [0, 1/2]); two uniforms a trial.
template <class St>
__device__ float moller_eps(St& st, float t, float tc) {
    const float tau = t * (1.f / kMe), gam = tau + 1.f, a = tau / gam;
    const float c2 = (2.f * tau + 1.f) / (gam * gam), ec = tc / t;
    float eps = ec;
    for (int trial = 0; trial < 1000; ++trial) {
        const float u1 = st.next(), u2 = st.next();
        eps = ec / (1.f - u1 * (1.f - 2.f * ec));
        const float r = eps / (1.f - eps);
        const float h = 1.f + r * r + a * a * eps * eps - c2 * r;
        if (u2 * 2.25f <= h) break;
    }
    return eps;
}

// Bremsstrahlung photon spectrum k dsigma/dk up to a constant (Bethe-Heitler,
// Born, unscreened: formula 3BN of Koch and Motz), FP64: its terms cancel
// strongly for soft photons.  0 at and beyond the tip.
__device__ double brem_shape(double t, double km) {
    constexpr double me = 0.51099895000;
    const double e0 = 1.0 + t / me, k = km / me, e = e0 - k;
    if (!(k > 0.0) || !(e > 1.0)) return 0.0;
    const double p0 = sqrt(e0 * e0 - 1.0), p = sqrt(e * e - 1.0);
    const double L = 2.0 * log((e0 * e + p0 * p - 1.0) / k);
    const double l0 = log((e0 + p0) / (e0 - p0)), l = log((e + p) / (e - p));
    const double p02 = p0 * p0, p2 = p * p, p03 = p02 * p0, p3 = p2 * p;
    const double br = 4.0 / 3.0 - 2.0 * e0 * e * (p2 + p02) / (p2 * p02) + l0 * e / p03 +
                      l * e0 / p3 - l * l0 / (p0 * p) +
                      L * (8.0 * e0 * e / (3.0 * p0 * p) + k * k * (e0 * e0 * e * e + p02 * p2) / (p03 * p3) +
                           k / (2.0 * p0 * p) *
                               (l0 * (e0 * e + p02) / p03 - l * (e0 * e + p2) / p3 +
                                2.0 * k * e0 * e / (p2 * p02)));
    const double v = (p / p0) * br;
    return v > 0.0 ? v : 0.0;
}

// Photon energy of a hard bremsstrahlung event (kc < t): k = kc (t/kc)^u,
// kept with probability shape(k) / shape(kc) (the spectrum k dsigma/dk falls
// with k); two uniforms a trial.
template <class St>
__device__ float brem_k(St& st, float t, float kc) {
    const double top = brem_shape(t, kc), lr = log(double(t) / double(kc));
    double k = kc;
    for (int trial = 0; trial < 1000; ++trial) {
        const float u1 = st.next(), u2 = st.next();
        k = double(kc) * exp(double(u1) * lr);
        if (double(u2) * top <= brem_shape(t, k)) break;
    }
    return float(k);
}

__device__ __forceinline__ void annihilate(const Stack& ann, float x, float y, float z, float u1,
                                          float u2, uint64_t g, uint32_t sub, uint32_t col,
                                          uint32_t& c_over) {
    const float c = 2.f * u1 - 1.f;
    float sphi, cphi;
    sincos_turn(u2, sphi, cphi);
    const float sn = hw_sqrt(fmaxf(0.f, 1.f - c * c));
    const float ux = sn * cphi, uy = sn * sphi;
    const uint32_t slot = atomicAdd(ann.count, 2u);
#pragma unroll
    for (uint32_t k = 0; k < 2u; ++k) {
        const uint32_t i = slot + k;
        if (i >= ann.capacity) {
            ++c_over;
            continue;
        }
        const float sg = k ? -1.f : 1.f;
        ann.x[i] = x; ann.y[i] = y; ann.z[i] = z;
        ann.u[i] = sg * ux; ann.v[i] = sg * uy; ann.w[i] = sg * c;
        ann.e[i] = kMe;
        uint64_t gk = g | (uint64_t(2u * sub + k) << 48);
        if (g >> 48) {
            uint32_t unused;
            child_id(g, sub, k, 3u, gk, unused);
        }
        ann.hid[i] = gk;
        ann.tag[i] = col;
    }
}

template <bool kRec, bool kFull>
__global__ void __launch_bounds__(kBlock) k_electron(TransportArgs a, Stack s) {
    __shared__ float s_rng[RNG_TAB_N];
    __shared__ float s_inv[INV_TAB_N];
    __shared__ float s_pool[kElectronPool * kBlock];
    for (int i = threadIdx.x; i < RNG_TAB_N; i += blockDim.x) s_rng[i] = a.phys.rng[i];
    for (int i = threadIdx.x; i < INV_TAB_N; i += blockDim.x) s_inv[i] = a.phys.inv[i];
    __syncthreads();

    const PhantomDev& G = a.ph;
    const PhysicsDev& P = a.phys;
    const float tcut = a.e_cut_e;
    const uint32_t n = min(*s.count, s.capacity);
    dev::LocalStats ls;
    double &esc_e = ls.l[L_ESC_E], &dep = ls.l[L_DEP], &path = ls.l[L_EPATH];
    uint32_t &c_steps = ls.c[C_E_STEPS], &c_atom = ls.c[C_DEPOSITS], &c_bnd = ls.c[C_E_BOUNDARY],
             &c_guard = ls.c[C_GUARD], &c_local = ls.c[C_E_LOCAL], &c_ann = ls.c[C_ANNIHIL],
             &c_over = ls.c[C_OVERFLOW], &c_moller = ls.c[C_MOLLER], &c_brem = ls.c[C_BREM],
             &c_capped = ls.c[C_CAPPED];
    (void)c_ann;
    (void)c_over;
    (void)c_moller;
    (void)c_brem;
    (void)c_capped;
    // positrons annihilate where they stop (kFull builds with an annihilation
    // stack; otherwise the flag is not read)
    bool positron = false;
    // per-lane electron state
    float px = 0.f, py = 0.f, pz = 0.f, dx = 0.f, dy = 0.f, dz = 0.f, t = 0.f, pend_e = 0.f;
    float rho = 0.f;   // density of the current voxel
    int ix = 0, iy = 0, iz = 0, cur_v = 0, pend_v = 0, steps = 0;
    uint32_t tag = 0;
    bool alive = false;
    // hard events (kFull with a.hard): mean free paths left to the next one,
    // and the electron's event index (its secondaries' streams)
    float lam = 0.f;
    uint32_t n_hard = 0;
    WaveQueue wq(n);
    dev::PoolStream<kElectronPool, kBlock> st(s_pool, a.seed_lo, a.seed_hi);
    // Order of an iteration as in k_photon: the CSDA step (deposits
    // deferred), the refill of idle lanes, then this step's deposits.
    for (;;) {
        if (__ballot(alive) == 0ull && wq.drained && wq.left == 0) break;
        // one multiple-scattering deflection (two uniforms) per step, at most
        // one step per iteration
        st.topup(alive && (a.ms || (kFull && positron)), 2, 5);
        // the next step's density, loaded into its own register (written
        // by nothing else before the end of the iteration, so that the load
        // is not waited on early) and taken over after the iteration's wait
        float rho_nx;
        asm volatile("v_mov_b32 %0, 0" : "=v"(rho_nx));   // not sunk into the other paths
        bool new_rho = false;
        // this step's deposits, deferred: the voxel left and the last voxel,
        // and a refilled electron that is below the cut-off on entry
        int w_v0 = -1, w_v1 = -1, w_v2 = -1;
        float w_e0 = 0.f, w_e1 = 0.f, w_e2 = 0.f;
        const uint32_t w_tag = tag;
        uint32_t w_tag2 = 0;
        if (alive) {
            bool done = false, escaped = false;
            if (kFull && !(t >= tcut)) {
                // a positron below the cut-off on entry: its energy went into
                // the voxel at the refill; it annihilates now
                done = true;
            } else if (steps >= kMaxElectronSteps) {
                pend_e += t;
                dep += t;
                ++c_guard;
                done = true;
            } else {
                ++steps;
                const float rho_s = rho;   // medium of this step
                float sb = INFINITY;
                int axis = 0;
                face_distance(px, dx, ix, G.origin[0], G.vox[0], 0, sb, axis);
                face_distance(py, dy, iy, G.origin[1], G.vox[1], 1, sb, axis);
                face_distance(pz, dz, iz, G.origin[2], G.vox[2], 2, sb, axis);
                sb = fmaxf(sb, 0.f);
                // energy-loss limited step
                const float r0 = csda_range(P, s_rng, t);
                const float ef = t * (1.f - a.step_frac);
                const bool fin = !(ef > tcut);
                float sf = INFINITY;
                if (rho_s > 0.f) sf = (fin ? r0 : r0 - csda_range(P, s_rng, ef)) * hw_rcp(rho_s);
                ++c_steps;
                // hard events: the distance to the next one at the rate of the
                // step's initial energy; a step ends there if it comes first
                float sig_h = 0.f, sh = INFINITY;
                if constexpr (kFull) {
                    if (a.hard && rho_s > 0.f) {
                        sig_h = hard_xs(P, t).y;
                        if (sig_h > 0.f) sh = lam * hw_rcp(rho_s * sig_h);
                    }
                }
                const bool event = sh < sf && sh < sb;
                const bool boundary = !event && !(sf <= sb);
                const float sl = event ? sh : (boundary ? sb : sf);
                if constexpr (kFull) {
                    if (!event) lam -= rho_s * sig_h * sl;
                }
                if (!event && !boundary && fin) {
                    // the residual range ends inside this voxel
                    path += sl;
                    pend_e += t;
                    dep += t;
                    done = true;
                } else {
                    const float tn = csda_energy(P, s_inv, r0 - rho_s * sl);
                    const float de = fmaxf(t - tn, 0.f);
                    pend_e += de;
                    dep += de;
                    px = fmaf(sl, dx, px);
                    py = fmaf(sl, dy, py);
                    pz = fmaf(sl, dz, pz);
                    path += sl;
                    const float t_old = t;
                    t -= de;
                    bool out = false;
                    if (boundary) {
                        ++c_bnd;
                        if (axis == 0) {
                            ix += dx > 0.f ? 1 : -1;
                            out = ix < 0 || ix >= G.nx;
                        } else if (axis == 1) {
                            iy += dy > 0.f ? 1 : -1;
                            out = iy < 0 || iy >= G.ny;
                        } else {
                            iz += dz > 0.f ? 1 : -1;
                            out = iz < 0 || iz >= G.nz;
                        }
                        if (out) {
                            // an escaping positron takes its rest energy along
                            esc_e += t + (kFull && positron ? 2.f * kMe : 0.f);
                            done = true;
                            escaped = true;
                        } else {
                            cur_v = (iz * G.ny + iy) * G.nx + ix;
                            // the next step's density, loaded while the rest
                            // of this iteration runs
                            rho_nx = G.dens[cur_v];
                            new_rho = true;
                            w_v0 = pend_v;
                            w_e0 = pend_e;
                            pend_v = cur_v;
                            pend_e = 0.f;
                        }
                    }
                    if (!out) {
                        if (t < tcut) {
                            pend_e += t;
                            dep += t;
                            done = true;
                        } else if (a.ms) {
                            // Highland width (PDG) for the step, beta*c*p at the mid-step energy
                            const float tx = rho_s * sl * (1.f / kX0Water);
                            const float tm = 0.5f * (t_old + t);
                            const float bcp = tm * (tm + 2.f * kMe) * hw_rcp(tm + kMe);
                            float th0 = 0.f;
                            if (tx > 0.f)
                                th0 = fmaxf(13.6f * hw_rcp(bcp) * hw_sqrt(tx) *
                                                fmaf(0.038f, hw_log(tx), 1.f),
                                            0.f);
                            const float u1 = st.pop(), u2 = st.pop();
                            const float th =
                                fminf(th0 * hw_sqrt(-2.f * hw_log(1.f - u1)), 3.14159265358979f);
                            float sphi, cphi;
                            sincos_turn(u2, sphi, cphi);
                            rotate(dx, dy, dz, __builtin_amdgcn_cosf(th * 0.15915494309189535f),
                                   cphi, sphi);
                        }
                        if constexpr (kFull) {
                            if (event && !done) {
                                // the hard event, after the step's continuous loss and
                                // deflection: the process in proportion to the
                                // cross-sections at this energy (one uniform)
                                // (the table's interpolation is not trusted below the
                                // thresholds: Moller needs t > 2 tc, a photon of at
                                // least kc needs t > kc)
                                const float2 hx = hard_xs(P, t);
                                const float sm = t > 2.f * tcut ? hx.x : 0.f;
                                const float stot = sm + (t > a.e_cut_g ? hx.y - hx.x : 0.f);
                                const float u = st.next();
                                const uint32_t j = n_hard++;
                                if (stot > 0.f) {
                                    const uint64_t gpar = (uint64_t(st.g1) << 32) | st.g0;
                                    const uint32_t spar = st.tagsub & 0xFFFFu;
                                    const uint32_t col = tag & kColumnMask;
                                    const bool follow = a.gen + 1u <= kGenMax;
                                    uint64_t gc = 0;
                                    uint32_t sc = 0;
                                    if (u * stot < sm) {
                                        // Moller: the delta electron takes w, both
                                        // directions from two-body kinematics
                                        const float tt = t;
                                        const float eps = moller_eps(st, tt, tcut);
                                        const float w = eps * tt, t1 = tt - w;
                                        const float up = st.next();
                                        float sphi, cphi;
                                        sincos_turn(up, sphi, cphi);
                                        const float cd = hw_sqrt(w * (tt + 2.f * kMe) /
                                                                 (tt * (w + 2.f * kMe)));
                                        const float cp = hw_sqrt(t1 * (tt + 2.f * kMe) /
                                                                 (tt * (t1 + 2.f * kMe)));
                                        float ddx = dx, ddy = dy, ddz = dz;
                                        rotate(ddx, ddy, ddz, cd, cphi, sphi);
                                        rotate(dx, dy, dz, cp, -cphi, -sphi);
                                        t = t1;
                                        ++c_moller;
                                        bool pushed = false;
                                        if (follow) {
                                            child_id(gpar, spar, j, 1u, gc, sc);
                                            const uint32_t slot = atomicAdd(a.el_next.count, 1u);
                                            if (slot < a.el_next.capacity) {
                                                a.el_next.x[slot] = px; a.el_next.y[slot] = py;
                                                a.el_next.z[slot] = pz;
                                                a.el_next.u[slot] = ddx; a.el_next.v[slot] = ddy;
                                                a.el_next.w[slot] = ddz;
                                                a.el_next.e[slot] = w;
                                                a.el_next.hid[slot] = gc;
                                                a.el_next.tag[slot] = col | (sc << 16);
                                                pushed = true;
                                            }
                                        }
                                        if (!pushed) {
                                            // past the generation cap, or no room
                                            pend_e += w;
                                            dep += w;
                                            if (follow) ++c_over; else ++c_capped;
                                        }
                                    } else {
                                        // bremsstrahlung: the photon along the electron
                                        const float k = brem_k(st, t, a.e_cut_g);
                                        t -= k;
                                        ++c_brem;
                                        bool pushed = false;
                                        if (follow && a.ann.count) {
                                            child_id(gpar, spar, j, 2u, gc, sc);
                                            const uint32_t slot = atomicAdd(a.ann.count, 1u);
                                            if (slot < a.ann.capacity) {
                                                a.ann.x[slot] = px; a.ann.y[slot] = py;
                                                a.ann.z[slot] = pz;
                                                a.ann.u[slot] = dx; a.ann.v[slot] = dy;
                                                a.ann.w[slot] = dz;
                                                a.ann.e[slot] = k;
                                                a.ann.hid[slot] = gc;
                                                a.ann.tag[slot] = col;
                                                pushed = true;
                                            }
                                        }
                                        if (!pushed) {
                                            pend_e += k;
                                            dep += k;
                                            if (follow && a.ann.count) ++c_over; else ++c_capped;
                                        }
                                    }
                                }
                                if (t < tcut) {
                                    pend_e += t;
                                    dep += t;
                                    done = true;
                                } else {
                                    lam = -hw_log(1.f - st.next());
                                }
                            }
                        }
                    }
                }
            }
            if (done) {
                alive = false;
                if constexpr (kFull) {
                    if (positron && !escaped) {
                        // (next(), not pop(): a hard event may have used the
                        // uniforms the top-up provided)
                        const float u1 = st.next(), u2 = st.next();
                        ++c_ann;
                        if (a.gen + 1u <= kGenMax) {
                            annihilate(a.ann, px, py, pz, u1, u2,
                                       (uint64_t(st.g1) << 32) | st.g0, st.tagsub & 0xFFFFu,
                                       tag & kColumnMask, c_over);
                        } else {
                            // above the generation cap: 2 mc^2 where it stops
                            pend_e += 2.f * kMe;
                            dep += 2.f * kMe;
                            ++c_capped;
                        }
                    }
                }
                w_v1 = pend_v;
                w_e1 = pend_e;
            }
        }
        // refill idle lanes from the wave's chunk of the (band-ordered) stack;
        // tag and data loaded together as in k_photon
        {
            // Idle lanes refill together, once at least kRefillLanes of them
            // wait (or none is alive): a refill with only the few lanes whose
            // electron ended this step would run the whole load sequence for
            // them, almost every iteration.
            const unsigned long long idle = __ballot(!alive);
            const bool refill = __popcll(idle) >= kRefillLanes || idle == ~0ull;
            const uint32_t q = refill ? take_work(!alive, wq, a.queue + 1, n) : kNone;
            const uint32_t i = q != kNone ? (a.perm ? a.perm[wq.strided(q)] : wq.strided(q)) : 0u;
            uint32_t tg = 1u << 24;
            float nx = 0.f, ny = 0.f, nz = 0.f, nu = 0.f, nv = 0.f, nw = 0.f, ne = 0.f;
            uint64_t g = 0;
            if (q != kNone) {
                tg = s.tag[i];
                nx = s.x[i]; ny = s.y[i]; nz = s.z[i];
                nu = s.u[i]; nv = s.v[i]; nw = s.w[i];
                ne = s.e[i];
                g = s.hid[i];
                asm volatile("" ::"v"(tg), "v"(nx), "v"(ny), "v"(nz), "v"(nu), "v"(nv), "v"(nw),
                             "v"(ne), "v"(g));
            }
            const bool take = (tg >> 24) == 0u;   // skip entries marked rejected / empty
            px = take ? nx : px; py = take ? ny : py; pz = take ? nz : pz;
            dx = take ? nu : dx; dy = take ? nv : dy; dz = take ? nw : dz;
            t = take ? ne : t;
            if (take) {
                tag = tg & 0xFFFFu;
                if constexpr (kFull) positron = (tg & kPositronBit) != 0u && a.ann.count != nullptr;
                ix = min(max(int(floorf((px - G.origin[0]) * G.inv_vox[0])), 0), G.nx - 1);
                iy = min(max(int(floorf((py - G.origin[1]) * G.inv_vox[1])), 0), G.ny - 1);
                iz = min(max(int(floorf((pz - G.origin[2]) * G.inv_vox[2])), 0), G.nz - 1);
                cur_v = (iz * G.ny + iy) * G.nx + ix;
                if (t < tcut) {
                    // below the cut-off on entry: local deposit, deferred
                    // with this iteration's others (its own tag)
                    w_v2 = cur_v;
                    w_e2 = t;
                    w_tag2 = tag;
                    dep += t;
                    ++c_local;
                    if constexpr (kFull) {
                        if (positron) {
                            // kept alive one more iteration to annihilate
                            // with uniforms of its own stream
                            st.init(g, dev::kTagTransport, (tg >> 16) & 0xFFu);
                            pend_v = cur_v;
                            pend_e = 0.f;
                            t = 0.f;
                            steps = 0;
                            alive = true;
                        }
                    }
                } else {
                    st.init(g, dev::kTagTransport, (tg >> 16) & 0xFFu);
                    pend_v = cur_v;
                    pend_e = 0.f;
                    rho_nx = G.dens[cur_v];
                    new_rho = true;
                    steps = 0;
                    alive = true;
                    if constexpr (kFull) {
                        if (a.hard) {
                            // mean free paths to the first hard event
                            lam = -hw_log(1.f - st.next());
                            n_hard = 0;
                        }
                    }
                }
            }
        }
        wait_loads();
        if (new_rho) rho = rho_nx;
        // this step's deposits
        deposit3<kRec>(a.tally, w_v0, w_e0, w_v1, w_e1, w_tag, w_v2, w_e2, w_tag2, c_atom);
    }
    dev::flush_stats(a.tally.stats, ls);
}

// ---- small utility kernels (no hipMemsetAsync, so graphs replay cleanly) --
__global__ void k_reset_queues(uint32_t* el_count, uint32_t* queue, uint32_t* ann_count,
                               uint32_t* del_count) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        if (el_count) *el_count = 0u;
        if (ann_count) *ann_count = 0u;
        if (del_count) *del_count = 0u;
        queue[0] = 0u;
        queue[1] = 0u;
    }
}

__global__ void k_zero_u32(uint32_t* p, int n) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0u;
}

template <class T>
__global__ void k_zero(T* p, int64_t n) {
    for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * blockDim.x)
        p[i] = T(0);
}

__global__ void k_fold(float* grid, double* sum, double* sum2, int64_t n,
                       unsigned long long* counters) {
    for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * blockDim.x) {
        const double e = grid[i];
        sum[i] += e;
        sum2[i] += e * e;
        grid[i] = 0.f;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(counters + C_FOLDS, 1ull);
}

// dose = k * mean, sigma = k * sqrt(var / R), with k per cell
__global__ void k_finalize(const double* sum, const double* sum2, int64_t n, int n_cols,
                           const float* rho_cell, int rho_per_row, const double* col_w,
                           double scale, const unsigned long long* counters, double* dose,
                           double* sigma) {
    const double R = double(counters[C_FOLDS]);
    for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * blockDim.x) {
        const int64_t row = rho_per_row ? i / n_cols : i;
        const int col = rho_per_row ? int(i % n_cols) : 0;
        const double rho = rho_cell[row];
        const double k = rho > 0.0 ? scale * col_w[col] / rho : 0.0;
        double mean = 0.0, var = 0.0;
        if (R > 0) {
            mean = sum[i] / R;
            if (R > 1) var = fmax((sum2[i] / R - mean * mean) * R / (R - 1.0), 0.0);
        }
        dose[i] = k * mean;
        sigma[i] = R > 0 ? k * sqrt(var / R) : 0.0;
    }
}

// Largest and smallest density (the smallest as the complement of its bit
// pattern, so that both reduce with atomicMax from zero) and a flag for
// negative or non-finite values.
__global__ void k_density_scan(const float* dens, int64_t n, unsigned int* max_bits,
                               unsigned int* bad, unsigned int* min_bits_c) {
    unsigned int m = 0, mc = 0, b = 0;
    for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * blockDim.x) {
        const float r = dens[i];
        if (!(r >= 0.f) || !isfinite(r)) {
            b = 1;
        } else {
            m = max(m, __float_as_uint(r));
            mc = max(mc, ~__float_as_uint(r));
        }
    }
    // non-negative floats order like their bit patterns
    for (int off = 32; off >= 1; off >>= 1) {
        m = max(m, (unsigned int)__shfl_xor(int(m), off, 64));
        mc = max(mc, (unsigned int)__shfl_xor(int(mc), off, 64));
        b |= (unsigned int)__shfl_xor(int(b), off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        atomicMax(max_bits, m);
        atomicMax(min_bits_c, mc);
        if (b) atomicOr(bad, 1u);
    }
}

__global__ void k_row_density(const int32_t* imap, const float* dens, int64_t n, float* row_rho,
                              int n_rows, unsigned int* bad) {
    for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * blockDim.x) {
        const int r = imap[i];
        if (r > 0) {
            if (r > n_rows) atomicOr(bad, 1u);
            else row_rho[r - 1] = dens[i];
        } else if (r < 0) {
            atomicOr(bad, 1u);
        }
    }
}

int grid_for(int64_t n, int cap = 4096) {
    return int(std::max<int64_t>(1, std::min<int64_t>((n + kBlock - 1) / kBlock, cap)));
}

}  // namespace

// Launch helpers used by the runtime as well.
void launch_zero_u32(uint32_t* p, int n, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, s, p, n);
}

TransportWs alloc_transport_ws(DevBuf& buf, uint32_t perm_cap, uint32_t ann_cap,
                               uint32_t del_cap) {
    const size_t q = 256, b = size_t(2) * kBands * kSortBlocks * 4, pm = size_t(perm_cap) * 4;
    // a particle stack: seven FP32 arrays, the ids, the tags and a count
    auto stack_bytes = [](uint32_t cap) {
        return cap ? size_t(cap) * (7 * 4 + 8 + 4) + 256 + 8 * 16 : size_t(0);
    };
    buf.alloc(q + b + pm + stack_bytes(ann_cap) + 2 * stack_bytes(del_cap));
    TransportWs ws;
    char* base = buf.as<char>();
    ws.queues = reinterpret_cast<uint32_t*>(base);
    ws.bands = reinterpret_cast<uint32_t*>(base + q);
    ws.perm = reinterpret_cast<uint32_t*>(base + q + b);
    ws.perm_cap = perm_cap;
    size_t off = (q + b + pm + 255) / 256 * 256;
    auto take = [&](size_t bytes) {
        void* r = base + off;
        off += (bytes + 15) / 16 * 16;
        return r;
    };
    auto carve_stack = [&](psl_particles& p, uint32_t cap, int32_t ptype) {
        float** f[7] = {&p.x, &p.y, &p.z, &p.u, &p.v, &p.w, &p.e};
        for (float** fp : f) *fp = static_cast<float*>(take(size_t(cap) * 4));
        p.hid = static_cast<uint64_t*>(take(size_t(cap) * 8));
        p.tag = static_cast<uint32_t*>(take(size_t(cap) * 4));
        p.count = static_cast<uint32_t*>(take(16));
        p.capacity = cap;
        p.ptype = ptype;
    };
    if (ann_cap) {
        carve_stack(ws.ann, ann_cap, 0);
        ws.ann_cap = ann_cap;
    }
    if (del_cap) {
        carve_stack(ws.del[0], del_cap, 1);
        carve_stack(ws.del[1], del_cap, 1);
        ws.del_cap = del_cap;
    }
    return ws;
}

namespace {

// Grid of a persistent transport launch over a stack of `capacity` entries.
int transport_grid(uint32_t capacity, int lane_load) {
    const int64_t per_block = int64_t(kBlock) * std::max(1, lane_load);
    return int(std::max<int64_t>(1, std::min<int64_t>((int64_t(capacity) + per_block - 1) / per_block, 2048)));
}

template <bool kRec, bool kFull>
void launch_photon(const TransportArgs& a, int grid, hipStream_t stream) {
    hipLaunchKernelGGL((k_photon<kRec, kFull>), dim3(grid), dim3(kBlock), 0, stream, a);
}

template <bool kRec, bool kFull>
void launch_electron(const TransportArgs& a, const Stack& s, int grid, hipStream_t stream) {
    hipLaunchKernelGGL((k_electron<kRec, kFull>), dim3(grid), dim3(kBlock), 0, stream, a, s);
}

void photon_kernel(const TransportArgs& a, bool full, int grid, hipStream_t stream) {
    if (a.tally.rec) {
        if (full) launch_photon<true, true>(a, grid, stream);
        else launch_photon<true, false>(a, grid, stream);
    } else {
        if (full) launch_photon<false, true>(a, grid, stream);
        else launch_photon<false, false>(a, grid, stream);
    }
    PSL_HIP(hipGetLastError());
}

void electron_kernel(const TransportArgs& a, const Stack& s, bool full, int grid,
                     hipStream_t stream) {
    if (a.tally.rec) {
        if (full) launch_electron<true, true>(a, s, grid, stream);
        else launch_electron<true, false>(a, s, grid, stream);
    } else {
        if (full) launch_electron<false, true>(a, s, grid, stream);
        else launch_electron<false, false>(a, s, grid, stream);
    }
    PSL_HIP(hipGetLastError());
}

// Electron energy-band order of `estack` into ws.perm (counting sort).
void sort_bands(const psl_phantom* ph, const TransportWs& ws, const Stack& estack,
                hipStream_t stream) {
    uint32_t* hist = ws.bands;
    uint32_t* offs = hist + kBands * kSortBlocks;
    PSL_CHECK(ws.perm_cap >= estack.capacity, "electron order buffer too small");
    const float lt0 = std::log(ph->phys.t_cut);
    const float inv_w = float(kBands) / (std::log(ph->phys.t_max) - lt0);
    hipLaunchKernelGGL(k_band_count, dim3(kSortBlocks), dim3(kBlock), 0, stream, estack.e,
                       estack.tag, estack.count, estack.capacity, hist, lt0, inv_w);
    hipLaunchKernelGGL(k_band_scan, dim3(1), dim3(1024), 0, stream, hist, offs);
    hipLaunchKernelGGL(k_band_scatter, dim3(kSortBlocks), dim3(kBlock), 0, stream, estack.e,
                       estack.tag, estack.count, estack.capacity, offs, ws.perm, lt0, inv_w);
}

}  // namespace

void launch_transport(const psl_phantom* phc, const psl_particles* in, psl_particles* el,
                      psl_tally* tally, const TransportWs& ws, const psl_transport_params* prm,
                      uint64_t seed, hipStream_t stream, bool sort_electrons, int lane_load,
                      const PhaseEvents* ev, uint32_t grid_items) {
    psl_phantom* ph = const_cast<psl_phantom*>(phc);
    const bool full = prm->physics != 0u;
    // positrons (pair production) need a stack for their annihilation photons
    const bool pair = (prm->physics & kPhysPair) != 0u && in->ptype == 0;
    PSL_CHECK(!pair || ws.ann_cap >= 2u * in->capacity,
              "annihilation photon stack too small (%u for %u photons)", ws.ann_cap,
              in->capacity);
    // electron hard events: delta electrons into ws.del, bremsstrahlung
    // photons (with the annihilation photons) into ws.ann
    const uint32_t hard = prm->physics & (kPhysDelta | kPhysBrem);
    const bool use_ann = pair || (hard & kPhysBrem) != 0u;
    const uint32_t e_cap = in->ptype == 0 ? el->capacity : in->capacity;
    PSL_CHECK(!hard || ws.del_cap >= e_cap, "delta-electron stacks too small (%u for %u)",
              ws.del_cap, e_cap);
    PSL_CHECK(!(hard & kPhysBrem) || ws.ann_cap >= e_cap,
              "secondary photon stack too small (%u for %u)", ws.ann_cap, e_cap);
    TransportArgs a{};
    a.in = to_stack(in);
    a.el = to_stack(el);
    a.perm = nullptr;
    a.ph = ph->g;
    a.phys = ph->phys;
    a.tally = tally->dev();
    a.e_cut_e = prm->e_cut_electron;
    a.e_cut_g = prm->e_cut_photon;
    a.step_frac = prm->step_frac;
    a.ms = prm->ms_enable;
    a.seed_lo = uint32_t(seed);
    a.seed_hi = uint32_t(seed >> 32);
    a.queue = ws.queues;
    if (use_ann) a.ann = to_stack(&ws.ann);
    a.hard = hard;
    a.gen = 0u;
    if (hard) a.el_next = to_stack(&ws.del[0]);
    Stack estack = a.el;
    // The transport kernels are persistent: every lane takes histories from a
    // queue until it is drained.  The grid is sized to the batch (about
    // lane_load histories per lane), not to the stacks, so that a lane works
    // through several histories and a wave is not held up by the one long
    // history among 64 short ones.  The batched runtime sizes it by its batch
    // size, which its stacks (grown, never shrunk) may exceed.
    const uint32_t items = grid_items ? std::min(grid_items, in->capacity) : in->capacity;
    const int tg = transport_grid(items, lane_load);
    // A wave reserves electron-stack entries push_chunk at a time (one
    // returning atomic each); the unused ends of the waves' last chunks
    // (fewer than push_chunk per wave) must fit in the one spare entry per
    // photon that the stack's capacity provides: 256 where the grid allows,
    // else 64 as the capacity rule states.
    const int64_t waves = int64_t(tg) * (kBlock / 64);
    a.push_chunk = waves * 255 <= int64_t(in->capacity) ? 256u : 64u;
    hipLaunchKernelGGL(k_reset_queues, dim3(1), dim3(64), 0, stream,
                       in->ptype == 0 ? el->count : nullptr, a.queue,
                       use_ann ? ws.ann.count : nullptr, hard ? ws.del[0].count : nullptr);
    if (in->ptype == 0) {
        if (ev) PSL_HIP(hipEventRecord(ev->photon0, stream));
        photon_kernel(a, full, tg, stream);
        if (ev) PSL_HIP(hipEventRecord(ev->photon1, stream));
    } else {
        estack = a.in;
    }
    if (ev) PSL_HIP(hipEventRecord(ev->sort0, stream));
    if (sort_electrons) {
        sort_bands(ph, ws, estack, stream);
        a.perm = ws.perm;
    }
    if (ev) PSL_HIP(hipEventRecord(ev->sort1, stream));
    if (ev) PSL_HIP(hipEventRecord(ev->electron0, stream));
    electron_kernel(a, estack, full, tg, stream);
    if (ev) PSL_HIP(hipEventRecord(ev->electron1, stream));
    if (hard) {
        // Generations 1 .. kGenMax: the photons the previous electron pass
        // made (bremsstrahlung, annihilation), whose electrons join that
        // pass's delta electrons, then those electrons, whose own delta
        // electrons go to the other stack.  Secondaries of the last
        // generation are deposited where they are made (in the kernels).
        Stack cur = to_stack(&ws.del[0]);
        Stack other = in->ptype == 0 ? a.el : to_stack(&ws.del[1]);
        const int tg2 = transport_grid(std::min(ws.del_cap, 2u * items), lane_load);
        const int64_t waves2 = int64_t(tg2) * (kBlock / 64);
        for (uint32_t gen = 1; gen <= kGenMax; ++gen) {
            TransportArgs b = a;
            b.gen = gen;
            b.in = to_stack(&ws.ann);
            b.secondary = 1u;
            b.perm = nullptr;
            b.el = cur;
            b.el_next = other;
            b.push_chunk = waves2 * 255 <= int64_t(cur.capacity) ? 256u : 64u;
            if (use_ann) {
                // (without bremsstrahlung or pairs no electron makes photons)
                hipLaunchKernelGGL(k_reset_queues, dim3(1), dim3(64), 0, stream, nullptr, b.queue,
                                   nullptr, nullptr);
                photon_kernel(b, true, tg2, stream);
            }
            // the photons are consumed: the stack takes this pass's new ones
            hipLaunchKernelGGL(k_reset_queues, dim3(1), dim3(64), 0, stream, other.count, b.queue,
                               use_ann ? ws.ann.count : nullptr, nullptr);
            if (sort_electrons) {
                sort_bands(ph, ws, cur, stream);
                b.perm = ws.perm;
            }
            electron_kernel(b, cur, true, tg2, stream);
            std::swap(cur, other);
        }
    } else if (pair) {
        // The photons of the positrons' annihilations, as photon histories of
        // their own (mc^2 each: they cannot make pairs, so no further pass),
        // then the electrons they set in motion.
        TransportArgs b = a;
        b.gen = 1u;
        b.in = to_stack(&ws.ann);
        b.ann = Stack{};
        b.secondary = 1u;
        b.perm = nullptr;
        const int tg2 = transport_grid(std::min(ws.ann_cap, 2u * items), lane_load);
        const int64_t waves2 = int64_t(tg2) * (kBlock / 64);
        b.push_chunk = waves2 * 255 <= int64_t(ws.ann_cap) ? 256u : 64u;
        hipLaunchKernelGGL(k_reset_queues, dim3(1), dim3(64), 0, stream, el->count, b.queue,
                           nullptr, nullptr);
        photon_kernel(b, true, tg2, stream);
        if (sort_electrons) {
            sort_bands(ph, ws, estack, stream);
            b.perm = ws.perm;
        }
        electron_kernel(b, estack, true, tg2, stream);
    }
}

void launch_fold(psl_tally* t, hipStream_t s) {
    hipLaunchKernelGGL(k_fold, dim3(grid_for(t->cells)), dim3(kBlock), 0, s, t->grid.as<float>(),
                       t->sum.as<double>(), t->sum2.as<double>(), t->cells, t->dev().counters);
    PSL_HIP(hipGetLastError());
}


}  // namespace psl

using namespace psl;

extern "C" int psl_phantom_create(const float* density_dev, int32_t nx, int32_t ny, int32_t nz,
                                  const double vox[3], const double origin[3], psl_phantom** out) {
    return guarded([&] {
        PSL_CHECK(density_dev && vox && origin && out, "psl_phantom_create: null argument");
        PSL_CHECK(nx >= 1 && ny >= 1 && nz >= 1, "phantom dimensions must be >= 1");
        PSL_CHECK(int64_t(nx) * ny * nz < (int64_t(1) << 31), "phantom has too many voxels");
        for (int k = 0; k < 3; ++k) PSL_CHECK(vox[k] > 0 && std::isfinite(origin[k]), "bad voxel size / origin");
        auto ph = std::make_unique<psl_phantom>();
        PSL_HIP(hipGetDevice(&ph->device));
        PhantomDev& g = ph->g;
        g.dens = density_dev;
        g.nx = nx;
        g.ny = ny;
        g.nz = nz;
        const int n[3] = {nx, ny, nz};
        for (int k = 0; k < 3; ++k) {
            g.vox[k] = float(vox[k]);
            g.inv_vox[k] = float(1.0 / vox[k]);
            g.origin[k] = float(origin[k]);
            g.hi[k] = float(origin[k] + n[k] * vox[k]);
        }
        DevBuf scratch;
        scratch.alloc(12);
        unsigned int* w = scratch.as<unsigned int>();
        const int64_t nv = int64_t(nx) * ny * nz;
        hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, nullptr, w, 3);
        hipLaunchKernelGGL(k_density_scan, dim3(grid_for(nv, 1024)), dim3(kBlock), 0, nullptr,
                           density_dev, nv, w, w + 1, w + 2);
        PSL_HIP(hipGetLastError());
        unsigned int hw[3];
        PSL_HIP(hipMemcpy(hw, w, 12, hipMemcpyDeviceToHost));
        PSL_CHECK(hw[1] == 0, "densities must be finite and >= 0");
        float rmax, rmin;
        std::memcpy(&rmax, &hw[0], 4);
        const unsigned int min_bits = ~hw[2];
        std::memcpy(&rmin, &min_bits, 4);
        PSL_CHECK(rmax > 0.f, "phantom has no matter (max density 0)");
        g.rho_max = rmax;
        g.inv_rho_max = 1.f / rmax;
        // the same FP32 product as the kernel's collision test, so that
        // rho * inv_rho_max >= real_min holds in floating point for every voxel
        g.real_min = rmin * g.inv_rho_max;
        *out = ph.release();
    });
}

extern "C" void psl_phantom_free(psl_phantom* p) { delete p; }

extern "C" int psl_tally_create(const psl_phantom* ph, const int32_t* imap, int32_t n_rows,
                                int32_t n_cols, psl_tally** out) {
    return guarded([&] {
        PSL_CHECK(ph && out, "psl_tally_create: null argument");
        auto t = std::make_unique<psl_tally>();
        t->phantom = ph;
        const int64_t nv = int64_t(ph->g.nx) * ph->g.ny * ph->g.nz;
        if (imap) {
            PSL_CHECK(n_rows >= 1 && n_cols >= 1 && n_cols <= 32768, "bad n_rows / n_cols");
            t->imap = imap;
            t->n_rows = n_rows;
            t->n_cols = n_cols;
            t->cells = int64_t(n_rows) * n_cols;
        } else {
            t->n_rows = 0;
            t->n_cols = 1;
            t->cells = nv;
        }
        t->grid.alloc(size_t(t->cells) * 4);
        t->sum.alloc(size_t(t->cells) * 8);
        t->sum2.alloc(size_t(t->cells) * 8);
        t->stats.alloc(size_t(dev::kStripes) * dev::kStatWords * 8);
        t->ws = alloc_transport_ws(t->ws_mem, 0);
        t->col_w.alloc(size_t(t->n_cols) * 8);
        if (imap) {
            t->row_rho.alloc(size_t(n_rows) * 4);
            DevBuf flag;
            flag.alloc(4);
            hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, nullptr, flag.as<uint32_t>(), 1);
            hipLaunchKernelGGL(k_zero<float>, dim3(grid_for(n_rows)), dim3(kBlock), 0, nullptr,
                               t->row_rho.as<float>(), int64_t(n_rows));
            hipLaunchKernelGGL(k_row_density, dim3(grid_for(nv, 1024)), dim3(kBlock), 0, nullptr,
                               imap, ph->g.dens, nv, t->row_rho.as<float>(), n_rows,
                               flag.as<unsigned int>());
            unsigned int bad = 0;
            PSL_HIP(hipMemcpy(&bad, flag.p, 4, hipMemcpyDeviceToHost));
            PSL_CHECK(bad == 0, "index map entries must be in [0, n_rows]");
        }
        psl_tally* raw = t.release();
        const int rc = tally_dose(raw, PSL_TALLY_RESET, nullptr, nullptr, nullptr, nullptr);
        PSL_HIP(hipDeviceSynchronize());
        if (rc != PSL_OK) {
            delete raw;
            fail(rc, "tally reset failed");
        }
        *out = raw;
    });
}

extern "C" void psl_tally_free(psl_tally* t) { delete t; }

extern "C" int transport_batch(const psl_phantom* phantom, const psl_particles* in,
                               psl_particles* electrons, psl_tally* tally,
                               const psl_transport_params* params, uint64_t seed, void* stream) {
    return guarded([&] {
        PSL_CHECK(phantom && in && tally && params, "transport_batch: null argument");
        PSL_CHECK(tally->phantom == phantom, "tally belongs to another phantom");
        PSL_CHECK(in->ptype == 0 || in->ptype == 1, "in->ptype must be 0 (photon) or 1 (electron)");
        PSL_CHECK(in->count && in->x && in->e && in->hid && in->tag, "particle stack has null arrays");
        PSL_CHECK(params->e_cut_photon > 0.f && params->e_cut_electron > 0.f &&
                      params->step_frac > 0.f && params->step_frac < 1.f,
                  "bad transport parameters");
        if (in->ptype == 0) {
            PSL_CHECK(electrons && electrons->count && electrons->x && electrons->e,
                      "photon transport needs an electron stack");
        }
        const psl_particles* es = in->ptype == 0 ? electrons : in;
        ensure_physics(const_cast<psl_phantom*>(phantom), params);
        const bool hard = (params->physics & (kPhysDelta | kPhysBrem)) != 0u;
        uint32_t ann_need =
            (params->physics & kPhysPair) && in->ptype == 0 ? 2u * in->capacity : 0u;
        if (params->physics & kPhysBrem) ann_need = std::max(ann_need, es->capacity);
        const uint32_t del_need = hard ? es->capacity : 0u;
        PSL_CHECK(ann_need == 0 || in->capacity <= (1u << 30), "photon stack too large");
        if (tally->ws.perm_cap < es->capacity || tally->ws.ann_cap < ann_need ||
            tally->ws.del_cap < del_need)
            tally->ws = alloc_transport_ws(tally->ws_mem, std::max(es->capacity, tally->ws.perm_cap),
                                           std::max(ann_need, tally->ws.ann_cap),
                                           std::max(del_need, tally->ws.del_cap));
        psl_particles dummy = *in;
        launch_transport(phantom, in, in->ptype == 0 ? electrons : &dummy, tally, tally->ws,
                         params, seed, static_cast<hipStream_t>(stream), true, 4);
    });
}

extern "C" int tally_dose(psl_tally* t, int32_t ops, const psl_plan* plan, double* dose,
                          double* sigma, void* stream) {
    return guarded([&] {
        PSL_CHECK(t, "tally_dose: null tally");
        hipStream_t s = static_cast<hipStream_t>(stream);
        if (ops & PSL_TALLY_RESET) {
            hipLaunchKernelGGL(k_zero<float>, dim3(grid_for(t->cells)), dim3(kBlock), 0, s,
                               t->grid.as<float>(), t->cells);
            hipLaunchKernelGGL(k_zero<double>, dim3(grid_for(t->cells)), dim3(kBlock), 0, s,
                               t->sum.as<double>(), t->cells);
            hipLaunchKernelGGL(k_zero<double>, dim3(grid_for(t->cells)), dim3(kBlock), 0, s,
                               t->sum2.as<double>(), t->cells);
            hipLaunchKernelGGL(k_zero<double>, dim3(4), dim3(kBlock), 0, s, t->stats.as<double>(),
                               int64_t(dev::kStripes) * dev::kStatWords);
            PSL_HIP(hipGetLastError());
        }
        if (ops & PSL_TALLY_FOLD) launch_fold(t, s);
        if (ops & PSL_TALLY_FINALIZE) {
            PSL_CHECK(plan && dose && sigma, "FINALIZE needs a plan and output arrays");
            PSL_CHECK(plan->n_cols == t->n_cols || (!t->imap && t->n_cols == 1),
                      "plan has %d tally columns, tally %d", plan->n_cols, t->n_cols);
            std::vector<double> cw(size_t(t->n_cols));
            if (t->imap) {
                cw = plan->col_weight;
            } else {
                // a voxel tally holds all columns together: one weight per history
                cw[0] = plan->col_weight[0];
                for (double c : plan->col_weight)
                    PSL_CHECK(c == cw[0], "a voxel tally needs an Eq. (3) plan (equal column weights)");
            }
            PSL_HIP(hipMemcpyAsync(t->col_w.p, cw.data(), cw.size() * 8, hipMemcpyHostToDevice, s));
            const PhantomDev& g = t->phantom->g;
            const double vol = double(g.vox[0]) * g.vox[1] * g.vox[2];
            const double scale = 1.602176634e-10 / vol;
            const float* rho = t->imap ? t->row_rho.as<float>() : g.dens;
            hipLaunchKernelGGL(k_finalize, dim3(grid_for(t->cells)), dim3(kBlock), 0, s,
                               t->sum.as<double>(), t->sum2.as<double>(), t->cells, t->n_cols, rho,
                               t->imap ? 1 : 0, t->col_w.as<double>(), scale, t->dev().counters,
                               dose, sigma);
            PSL_HIP(hipGetLastError());
            PSL_HIP(hipStreamSynchronize(s));   // cw lives on this stack frame
        }
    });
}

extern "C" int psl_tally_record(psl_tally* t, uint32_t* cells_dev, uint32_t capacity,
                                uint32_t* count_dev) {
    return guarded([&] {
        PSL_CHECK(t, "psl_tally_record: null tally");
        if (!cells_dev) {
            t->rec = nullptr;
            t->rec_count = nullptr;
            t->rec_cap = 0;
            return;
        }
        PSL_CHECK(count_dev && capacity > 0, "psl_tally_record: count and capacity required");
        t->rec = cells_dev;
        t->rec_count = count_dev;
        t->rec_cap = capacity;
    });
}

extern "C" int psl_tally_stats(psl_tally* t, double* ledger, uint64_t* counters) {
    int status = PSL_OK;
    int rc = guarded([&] {
        PSL_CHECK(t, "psl_tally_stats: null tally");
        PSL_HIP(hipDeviceSynchronize());
        std::vector<double> buf(size_t(dev::kStripes) * dev::kStatWords);
        PSL_HIP(hipMemcpy(buf.data(), t->stats.p, buf.size() * 8, hipMemcpyDeviceToHost));
        double led[L_N] = {0};
        uint64_t c[C_N] = {0};
        for (int k = 0; k < dev::kStripes; ++k) {
            const double* row = buf.data() + size_t(k) * dev::kStatWords;
            for (int i = 0; i < L_N; ++i) led[i] += row[i];
            const uint64_t* cr = reinterpret_cast<const uint64_t*>(row + L_N);
            for (int i = 0; i < C_N; ++i) c[i] += cr[i];
        }
        if (ledger) std::memcpy(ledger, led, L_N * 8);
        if (counters) std::memcpy(counters, c, C_N * 8);
        if (c[C_OVERFLOW]) {
            status = PSL_EOVERFLOW;
            set_last_error("a particle stack overflowed; results are invalid");
        }
    });
    return rc != PSL_OK ? rc : status;
}
