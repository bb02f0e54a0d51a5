// Internal definitions shared by the host and device translation units of
// libpsl.so: handle structs, device data layouts and launcher declarations.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <stdexcept>
#include <string>
#include <vector>

#include "psl.h"

namespace psl {

// ---------------------------------------------------------------------------
// Errors: internal code throws psl::Error; every exported function converts it
// into a status code and a thread-local message.
// ---------------------------------------------------------------------------
struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

[[noreturn]] void fail(int code, const char* fmt, ...);
void set_last_error(const char* msg);
void clear_last_error();

#define PSL_CHECK(cond, ...)                                   \
    do {                                                       \
        if (!(cond)) ::psl::fail(PSL_EINVAL, __VA_ARGS__);     \
    } while (0)

#define PSL_HIP(call)                                                                   \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess)                                                           \
            ::psl::fail(e_ == hipErrorOutOfMemory ? PSL_ENOMEM : PSL_EDEVICE, "%s: %s", \
                        #call, hipGetErrorString(e_));                                  \
    } while (0)

// Runs `body`, converting exceptions into status codes.
template <class F>
int guarded(F&& body) {
    try {
        clear_last_error();
        body();
        return PSL_OK;
    } catch (const Error& e) {
        set_last_error(e.what());
        return e.code;
    } catch (const std::bad_alloc&) {
        set_last_error("host allocation failed");
        return PSL_ENOMEM;
    } catch (const std::exception& e) {
        set_last_error(e.what());
        return PSL_EDEVICE;
    }
}

// Owning device buffer.
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf() { release(); }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    void alloc(size_t n) {
        release();
        if (n == 0) n = 1;
        PSL_HIP(hipMalloc(&p, n));
        bytes = n;
    }
    template <class T>
    T* as() const { return static_cast<T*>(p); }
    template <class T>
    void upload(const std::vector<T>& v) {
        alloc(v.size() * sizeof(T));
        if (!v.empty()) PSL_HIP(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    }
};

// Scratch of one transport pipeline: the two work-queue heads, the band
// counters / offsets of the electron energy sort and the electron order.
constexpr int kSortBands = 8;       // electron energy bands of the counting sort
constexpr int kSortBlocks = 1024;   // fixed grid of the counting sort
// Histories per entry of a plan's chunk index (the sampling kernel's search
// starts from it).
constexpr int kChunkShift = 10;

struct TransportWs {
    uint32_t* queues = nullptr;     // [64]
    uint32_t* bands = nullptr;      // [2 * kSortBands * kSortBlocks]
    uint32_t* perm = nullptr;       // [perm_cap]
    uint32_t perm_cap = 0;
    // photons from positron annihilation (pair production on): a photon
    // stack of ann_cap entries (x, y, z, u, v, w, E, id, tag, count)
    psl_particles ann{};
    uint32_t ann_cap = 0;
    // delta electrons (electron hard events on): two electron stacks of
    // del_cap entries, written by one electron pass and read by the next
    psl_particles del[2]{};
    uint32_t del_cap = 0;
};

// ---------------------------------------------------------------------------
// Device layouts
// ---------------------------------------------------------------------------

// One in-area PSL of a plan's history list.
struct PslEntry {
    uint8_t ix, iy, stype, ebin;
    uint16_t beam, tag;
};
static_assert(sizeof(PslEntry) == 8, "PslEntry must pack into 8 bytes");

// Per-beam constants for the sampling kernel.
struct BeamDev {
    float R[9];          // beam -> patient rotation, row-major
    float iso[3];
    float jx1, jx2;      // X jaw edges at the height of their upper surface
    float jy1, jy2;      // Y jaw edges at the height of their upper surface
    float pad[2];
};

// Scatter direction component (Eq. 6): cumulative probability, alpha mean,
// alpha width, beta width.
struct ScatterComp {
    float cdf, mu, sa, sb;
};

// Tabulated physics for the transport kernels.
constexpr int KN_TAB_N = 1024;      // sigma_KN(E) n_e on a log-E grid
constexpr int RNG_TAB_N = 1024;     // CSDA range R(T) on a log-T grid
constexpr int INV_TAB_N = 2048;     // T(R) on a uniform R grid
constexpr int RAY_TAB_N = 1024;     // Rayleigh: cumulative of F^2 over t = (q a0)^2

// Optional photon processes (psl_transport_params.physics bits).
constexpr uint32_t kPhysPhoto = 1u, kPhysRayleigh = 2u, kPhysPair = 4u, kPhysDelta = 8u,
                   kPhysBrem = 16u;
// Generations of secondaries that are transported (delta electrons,
// bremsstrahlung and annihilation photons are one above their parent); above
// it a secondary's energy is deposited where it is made.
constexpr uint32_t kGenMax = 3u;
// Particle tag bit 15 marks a positron (tally columns use bits 0-14).
constexpr uint32_t kPositronBit = 0x8000u;
constexpr uint32_t kColumnMask = 0x7FFFu;

struct PhysicsDev {
    float kn_lne0, kn_inv_dlne;     // ln E of node 0, 1 / node spacing in ln E
    float rng_lnt0, rng_inv_dlnt;   // same for the range table (ln T)
    float inv_u0, inv_inv_du;       // inverse table: u = ln(R + r_off), node 0 and 1/spacing
    float r_off, r_tab_max;         // offset of u, largest tabulated range (g/cm^2)
    float t_cut, t_max;
    const float* kn;                // [KN_TAB_N] n_e sigma_KN (1/cm at unit density)
    const float* rng;               // [RNG_TAB_N] R(T) g/cm^2
    const float* inv;               // [INV_TAB_N] T(R) MeV
    // optional photon processes (null / zero when none is enabled)
    uint32_t physics;               // kPhys* bits the tables were built for
    const float4* xs;               // [KN_TAB_N] cumulative attenuations at unit density
                                    // (1/cm) on the kn grid: x Compton, y + photoelectric,
                                    // z + Rayleigh, w + pair (the total)
    const float* ray_t;             // [RAY_TAB_N] t nodes: 0, then log-spaced
    const float* ray_a;             // [RAY_TAB_N] integral of F^2 from 0 to t
    float ray_lt1, ray_inv_dlt;     // ln t of node 1, 1 / spacing in ln t
    float ka0_per_mev;              // k a0 per MeV of photon energy
    float photo_bind;               // K binding energy of oxygen (MeV)
    // optional electron hard events: per unit density (cm^2/g) on the range
    // table's grid, x = Moller collisions above the electron cut-off, y = x +
    // bremsstrahlung above the photon cut-off (null when neither is enabled)
    const float2* hard;
};

// Energy ledger and counter slots (match psl_tally_stats).
enum { L_SRC = 0, L_JAW, L_MISSED, L_INVALID, L_ESC_G, L_ESC_E, L_DEP, L_EPATH, L_N };
enum {
    C_HIST = 0, C_ENTERED, C_WC_STEPS, C_REAL, C_E_PUSHED, C_E_LOCAL, C_E_STEPS, C_DEPOSITS,
    C_ESC_UNCOLLIDED, C_KAHN_TRIALS, C_E_BOUNDARY, C_GUARD, C_OVERFLOW, C_FOLDS,
    C_PHOTO, C_RAYLEIGH, C_PAIR, C_ANNIHIL, C_MOLLER, C_BREM, C_CAPPED, C_N = 24
};

// Device-side tally state.  `stats` holds kStripes copies of the ledger
// (L_N doubles) followed by the counters (C_N uint64), summed by the host.
struct TallyDev {
    float* grid;            // FP32 replica cells
    double* stats;          // [kStripes][L_N + C_N]
    unsigned long long* counters;   // counters of copy 0
    const int32_t* imap;    // nullable voxel -> row+1
    int32_t n_cols;
    // nullable: while set, the cell of every deposit atomic is appended here
    // in the order the transport kernels issue them (measurement only)
    uint32_t* rec;
    uint32_t* rec_count;
    uint32_t rec_cap;
};

// Geometry of a phantom as seen by the kernels.
struct PhantomDev {
    const float* dens;
    int nx, ny, nz;
    float vox[3], inv_vox[3], origin[3], hi[3];
    float rho_max, inv_rho_max;
    float real_min;    // smallest rho / rho_max over the voxels (FP32 product)
};

struct Runner;   // batched-runtime workspace (runtime.hip)
struct UNet;     // denoiser (k_denoise.hip)

}  // namespace psl

// ---------------------------------------------------------------------------
// Handles
// ---------------------------------------------------------------------------
struct psl_model {
    psl_psr_desc d{};                  // scalars; pointer fields unused after build
    std::vector<double> w_psr, sc_c, sc_mu, sc_sa, sc_sb;
    std::vector<double> w_psl;         // [3][n_ebin][n_psl][n_psl]
    std::vector<double> cdf;           // [n_ebin][n_ring][K]
    double e_max = 0.0;
    std::vector<psl::ScatterComp> scatter_host;
    mutable psl::DevBuf scatter;       // ScatterComp [n_ebin][n_ring][K], uploaded on first use
};

struct psl_plan {
    const psl_model* model = nullptr;
    std::vector<psl_beam> beams;
    std::vector<int32_t> boxes;        // [n_beams][3][4]
    std::vector<int32_t> beam, stype, ebin, ix, iy, tag;
    std::vector<double> w;
    std::vector<uint64_t> cum;
    std::vector<double> col_weight;    // per tally column
    uint64_t n_hist = 0;
    uint32_t n_replica = 1;
    int32_t n_cols = 1;
    double s_area = 0.0;
    std::vector<psl_batch> batches;
    std::vector<int64_t> batch_jlo, batch_jhi;   // list range of each batch
    uint32_t cur_max_batch = 0;        // batching the lists above were built for
    int32_t cur_band_width = 0;
    std::vector<psl::PslEntry> list_host;
    std::vector<psl::BeamDev> beams_host;
    // device copies, uploaded on first use (set-up itself needs no GPU)
    mutable psl::DevBuf d_list;        // PslEntry [n_list]
    mutable psl::DevBuf d_cum;         // uint64 [n_list]
    // uint32 [(n_hist >> kChunkShift) + 2]: entry c = first list index whose
    // inclusive count prefix exceeds c << kChunkShift (n_list past the end)
    mutable psl::DevBuf d_chunk;
    mutable psl::DevBuf d_beams;       // BeamDev [n_beams]
};

struct psl_phantom {
    psl::PhantomDev g{};
    int device = 0;
    // physics tables per transport-parameter set; tab_gen counts rebuilds, so
    // that a captured graph holding the old table address is never replayed
    float t_cut_tab = -1.f;
    int32_t dens_tab = -1;
    int32_t phys_tab = -1;
    float kc_tab = -1.f;   // photon cut-off of the bremsstrahlung tables
    uint64_t tab_gen = 0;
    psl::DevBuf tabs;
    psl::PhysicsDev phys{};
};

struct psl_tally {
    const psl_phantom* phantom = nullptr;
    int32_t n_rows = 0, n_cols = 1;
    int64_t cells = 0;
    const int32_t* imap = nullptr;
    psl::DevBuf grid;      // float [cells]
    psl::DevBuf sum;       // double [cells]
    psl::DevBuf sum2;      // double [cells]
    psl::DevBuf stats;     // double ledger [L_N] + u64 counters [C_N]
    psl::DevBuf row_rho;   // float [n_rows] density of each row's voxel (index-map mode)
    psl::DevBuf col_w;     // double [n_cols] column weights (finalize scratch)
    psl::DevBuf ws_mem;    // transport scratch of transport_batch (queues, bands, order)
    psl::TransportWs ws{};
    uint32_t folds = 0;
    psl::Runner* runner = nullptr;     // batched-runtime workspace (runtime.hip)
    uint32_t* rec = nullptr;           // deposit-cell recording (psl_tally_record)
    uint32_t* rec_count = nullptr;
    uint32_t rec_cap = 0;
    ~psl_tally();
    psl::TallyDev dev() const {
        psl::TallyDev t;
        t.grid = grid.as<float>();
        t.stats = stats.as<double>();
        t.counters = reinterpret_cast<unsigned long long*>(stats.as<double>() + psl::L_N);
        t.imap = imap;
        t.n_cols = n_cols;
        t.rec = rec;
        t.rec_count = rec_count;
        t.rec_cap = rec_cap;
        return t;
    }
};

namespace psl {
// Physics tables (host FP64 -> device FP32); defined in physics.cpp.
void ensure_physics(psl_phantom* ph, const psl_transport_params* p);
// Device copies of a model's / plan's sampling tables; defined in host_model.cpp.
void ensure_device(const psl_model* m);
void ensure_device(const psl_plan* p);

// Allocates the scratch for an electron stack of up to perm_cap entries in
// buf, and a stack of ann_cap annihilation photons (0: none).
TransportWs alloc_transport_ws(DevBuf& buf, uint32_t perm_cap, uint32_t ann_cap = 0,
                               uint32_t del_cap = 0);


// Optional HIP events recorded around the transport launches (may be null).
struct PhaseEvents {
    hipEvent_t photon0, photon1, sort0, sort1, electron0, electron1;
};

// Kernel launchers shared by the public calls and the batched runtime.
void launch_sample(const psl_plan* plan, const psl_phantom* ph, uint32_t replica,
                   const uint32_t* rep_dev, uint64_t h0, uint32_t n, int64_t jlo, int64_t jhi,
                   int stype, uint64_t seed, const psl_particles* out, int dense, psl_tally* tally,
                   hipStream_t stream);
void launch_transport(const psl_phantom* ph, const psl_particles* in, psl_particles* el,
                      psl_tally* tally, const TransportWs& ws, const psl_transport_params* prm,
                      uint64_t seed, hipStream_t stream, bool sort_electrons, int lane_load,
                      const PhaseEvents* ev = nullptr, uint32_t grid_items = 0);
void launch_zero_u32(uint32_t* p, int n, hipStream_t s);
void launch_fold(psl_tally* t, hipStream_t s);
}  // namespace psl
