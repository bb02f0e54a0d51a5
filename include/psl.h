/*
 * psl.h -- C ABI of the MI355X (gfx950) Monte Carlo dose engine built around
 * the analytic phase-space-ring (PSR) linac source model of Tian et al.,
 * "An analytic linear accelerator source model for Monte Carlo dose
 * calculations. II" (arXiv:1503.01725).
 *
 * Conventions
 *   - Every call returns a psl_status; on failure psl_last_error() (thread
 *     local) holds a message.  No C++ exception crosses this boundary.
 *   - Units: cm, MeV, g/cm^3.  Doses are Gy per model particle.
 *   - Handles (psl_model, psl_plan, psl_phantom, psl_tally) are owned by the
 *     library and released with the matching *_free call.  A plan keeps a
 *     pointer to its model, a tally to its phantom: free dependants first.
 *   - Pointers documented as "device" are HIP device pointers owned by the
 *     caller (for example torch tensors); the library never frees them.
 *     Pointers documented as "host" are read (or written) before the call
 *     returns.
 *   - Calls taking a `stream` (a hipStream_t, NULL = default stream) are
 *     asynchronous: they validate arguments on the host, enqueue work and
 *     return.  Conditions detected on the device (a particle stack too small,
 *     a particle column beyond the tally, the step guard of a transport loop)
 *     are counted in the tally's event counters, which psl_tally_stats
 *     reads (it returns PSL_EOVERFLOW after an overflow).
 *   - Distinct handles may be used from different host threads; one handle
 *     must not be used by two threads at once.
 */
#ifndef PSL_H
#define PSL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PSL_OK = 0,
    PSL_EINVAL = -1,     /* bad argument (reported before any device work)    */
    PSL_ENOMEM = -2,     /* device or host allocation failed                  */
    PSL_EDEVICE = -3,    /* HIP runtime error                                 */
    PSL_EOVERFLOW = -4,  /* a particle stack was too small; results invalid   */
    PSL_ENOTCONV = -5    /* iterative solve hit its iteration limit           */
} psl_status;

/* Message of the last failing call on this thread ("" if none). */
const char* psl_last_error(void);

/* Opaque, library-owned handles. */
typedef struct psl_model psl_model;
typedef struct psl_plan psl_plan;
typedef struct psl_phantom psl_phantom;
typedef struct psl_tally psl_tally;

/* ------------------------------------------------------------------------
 * Source model (Sec. 2.1.1; Eqs. 4-7 for the direction models)
 * ------------------------------------------------------------------------ */

/* A PSR model: 3 sub-sources (0 primary photon, 1 scatter photon,
 * 2 electron) x n_ebin energy bins x n_ring rings on the plane z = z_plane.
 * Energy bin b covers [e_lo + b e_width, e_lo + (b+1) e_width); ring j covers
 * [j ring_dr, (j+1) ring_dr).  The PSL grid is n_psl x n_psl squares of side
 * psl_dx with edges at psl_x0 + k psl_dx in x and y.  Heights (beam frame,
 * particles travel towards +z): focal spot z_target, scatter source
 * z_scatter, upper surfaces of the Y and X jaws z_jaw_y and z_jaw_x; the plane
 * is the isocentre plane.  All arrays are host memory, copied by psl_build. */
typedef struct {
    int32_t n_ebin, n_ring, n_comp, n_psl;
    double e_lo, e_width, ring_dr, psl_x0, psl_dx;
    double z_target, z_plane, z_scatter, z_jaw_y, z_jaw_x;
    double sigma_spot;          /* focal-spot Gaussian width, Eq. (4)        */
    double sig_ea, sig_eb;      /* electron angular widths, Eq. (7)          */
    const double* w_psr;        /* [3][n_ebin][n_ring] PSR weights           */
    const double* sc_c;         /* [n_ebin][n_ring][n_comp] mixture weights, Eq. (6) */
    const double* sc_mu;        /* [n_ebin][n_ring][n_comp] alpha means (rad)     */
    const double* sc_sa;        /* [n_ebin][n_ring][n_comp] alpha widths (rad)    */
    const double* sc_sb;        /* [n_ebin][n_ring][n_comp] beta widths (rad)     */
} psl_psr_desc;

/* Converts the PSR model to its PSL representation once (Sec. 2.1.1, Eq. 2:
 * interpolated ring weight / (2 pi r) at each PSL centre, normalised over all
 * sub-sources, energies and locations), builds the scatter component table
 * P_{i,k} (step S4) and uploads the sampling tables to the current device.
 * Limits: n_psl <= 255, n_ebin <= 255, 1 <= n_comp <= 8.  Synchronous. */
int psl_build(const psl_psr_desc* desc, psl_model** out);

/* Copies the FP64 PSL weights [3][n_ebin][n_psl][n_psl] to host memory. */
int psl_model_weights(const psl_model* model, double* w_psl_host);
void psl_model_free(psl_model* model);

/* ------------------------------------------------------------------------
 * Plan: sampling areas (Sec. 2.1.2, Fig. 3, step S1) and particles per PSL
 * (step S2, Eq. 3), with the history order of Sec. 2.1.3.
 * ------------------------------------------------------------------------ */

/* One beam: jaw edges projected to the isocentre plane (x1 < x2, y1 < y2),
 * gantry angle (rotation about patient +y) and couch angle (about +z), and
 * the isocentre in patient coordinates. */
typedef struct {
    double x1, x2, y1, y2;
    double gantry_deg, couch_deg;
    double iso[3];
} psl_beam;

/* Builds the list of in-area PSLs of all beams in the order beam, sub-source,
 * energy bin, y, x (location innermost, energy outer; Sec. 2.1.3) and their
 * particle counts.
 *   basis_of_psr: NULL, or host [3][n_ebin][n_ring] basis id of each PSR (the
 *     PSL takes the id of the ring its centre lies in).  A particle then
 *     carries the tally column beam * n_basis + basis (Sec. 2.2.2), where
 *     n_basis = 1 + the largest id; n_beams * n_basis must not exceed 32768
 *     (the column travels in 15 bits of the particle tag).
 *   hist_per_basis: 0 -> Eq. (3): n_hist histories spread over the whole list
 *     in proportion to the PSL weights.  > 0 (needs basis_of_psr) ->
 *     commissioning: each (beam, basis) receives hist_per_basis histories
 *     spread over its own PSLs; the list order is then beam, basis, sub-source,
 *     energy, y, x, and n_hist is ignored.
 *   Counts are rounded systematically on a 2^-40 fixed-point prefix so that
 *   they add up to the requested totals exactly.
 * The plan refers to `model`, which must outlive it.  Synchronous. */
int psl_plan_create(const psl_model* model, const psl_beam* beams, int32_t n_beams,
                    uint64_t n_hist, uint32_t n_replica, const uint16_t* basis_of_psr,
                    uint64_t hist_per_basis, psl_plan** out);

typedef struct {
    uint64_t n_hist;        /* histories per replica (N)                        */
    uint32_t n_replica;
    int32_t n_beams;
    int64_t n_list;         /* in-area PSLs with positive weight                */
    int32_t n_cols;         /* tally columns (1 without a basis map)            */
    double s_area;          /* sum of in-area PSL weights (Eq. 3 denominator)   */
    double e_max;           /* highest source energy of the model               */
} psl_plan_info;
int psl_plan_get_info(const psl_plan* plan, psl_plan_info* info);

/* Host copies of the plan: the sampling box [ix0, ix1, iy0, iy1] of every
 * (beam, sub-source) (int32 [n_beams][3][4]); and the list (any pointer may
 * be NULL): int32 beam, stype, ebin, ix, iy, tag and uint64 inclusive prefix
 * of counts, n_list entries each. */
int psl_plan_boxes(const psl_plan* plan, int32_t* boxes);
int psl_plan_list(const psl_plan* plan, int32_t* beam, int32_t* stype, int32_t* ebin,
                  int32_t* ix, int32_t* iy, int32_t* tag, double* w, uint64_t* cum);

/* Per-column particle weight (model particles per history): S_A/N for Eq. (3)
 * plans, S_{beam,basis}/n_{beam,basis} for commissioning plans.  n_cols
 * doubles, host memory. */
int psl_plan_col_weight(const psl_plan* plan, double* w_host);

/* Batches (Sec. 2.1.3): maximal runs of consecutive histories inside one
 * (beam, sub-source, energy band) with at most max_batch histories, where
 * band = energy bin / band_width.  psl_plan_set_batching fixes the split and
 * returns the number of batches; psl_plan_get_batch reads one. */
typedef struct {
    uint64_t h0;            /* first history (within a replica)               */
    uint32_t n;             /* histories in the batch                          */
    int32_t stype;          /* sub-source: 0 primary, 1 scatter, 2 electron   */
    int32_t beam;
    int32_t band;
} psl_batch;
int psl_plan_set_batching(psl_plan* plan, uint32_t max_batch, int32_t band_width,
                          int64_t* n_batches);
int psl_plan_get_batch(const psl_plan* plan, int64_t index, psl_batch* batch);
void psl_plan_free(psl_plan* plan);

/* ------------------------------------------------------------------------
 * Phantom
 * ------------------------------------------------------------------------ */
/* The voxel phantom the dose is computed in (Sec. 2.3 and Sec. 3.1: a water
 * phantom, and patient CT volumes as densities of a water-like medium).
 * density_dev: device float32 [nz][ny][nx] mass densities (water-like medium
 * scaled by density), x fastest; must stay valid while the phantom is used.
 * vox: voxel size (cm); origin: patient coordinates of the outer corner of
 * voxel (0,0,0).  The maximum density is found on the device.  Synchronous. */
int psl_phantom_create(const float* density_dev, int32_t nx, int32_t ny, int32_t nz,
                       const double vox[3], const double origin[3], psl_phantom** out);
void psl_phantom_free(psl_phantom* phantom);

/* ------------------------------------------------------------------------
 * Particles (steps S3-S5)
 * ------------------------------------------------------------------------ */

/* Structure-of-arrays particle stack, all arrays device memory of `capacity`
 * entries, caller-allocated.  tag bits 0-15: tally column; bits 16-23: random
 * sub-stream id; bits 24-31: status (0 ok, 1 jaw-rejected, 2 missed the
 * phantom, 3 invalid direction; dense sampling output only).  `count` is a
 * device uint32.  `ptype` (host field) is 0 for photons, 1 for electrons and
 * is set by sample_batch. */
typedef struct {
    float *x, *y, *z, *u, *v, *w, *e;
    uint64_t* hid;
    uint32_t* tag;
    uint32_t* count;
    uint32_t capacity;
    int32_t ptype;
} psl_particles;

enum {
    PSL_SAMPLE_DENSE = 1,   /* write history h0+i at slot i with its status
                               (every history, also rejected ones, whose slot
                               holds the beam-frame plane position and
                               direction) and set *count = n, instead of
                               compacting accepted particles                */
    PSL_SAMPLE_PLANE = 2    /* dense phase-space-plane records: every history
                               at slot i with its beam-frame position
                               (x, y, z = 0) and direction at the plane, its
                               energy and id, tag = column | beam << 16 |
                               status << 24 (status 0, or 3 for an invalid
                               direction); no jaw test and no transform (the
                               records of a particle-file source; the plan may
                               hold at most 255 beams)                       */
};

/* Samples histories [h0, h0+n) of replica `replica` (global id
 * g = replica * N + h) from one sub-source (the range must not cross a
 * sub-source change; batches from psl_plan_get_batch never do):
 *   - PSL by binary search of h in the count prefix; position and energy
 *     uniform in the PSL and its bin;
 *   - direction from Eq. (5) (primary: Gaussian focal spot, Eq. 4), Eq. (6)
 *     (scatter: K-component Gaussian mixture in alpha, beta) or Eq. (7)
 *     (electron), rotated by theta = atan2(y, x);
 *   - jaw rejection at the upper jaw surfaces; beam -> patient transform;
 *     start at the entry of the particle's line into the phantom box.
 * Random numbers: Philox4x32-10 keyed by `seed`, counter (block, 1<<16,
 * g_lo, g_hi).  Without PSL_SAMPLE_DENSE accepted particles are appended at
 * *out->count (which the caller zeroes) and rejected ones only enter the
 * tally's energy ledger.  Needs out->capacity >= n (dense) or room for n more.
 * The tally receives the source-side energy ledger. */
int sample_batch(const psl_plan* plan, const psl_phantom* phantom, uint32_t replica,
                 uint64_t h0, uint32_t n, uint64_t seed, psl_particles* out,
                 uint32_t flags, psl_tally* tally, void* stream);

/* The second half of sample_batch for phase-space-plane records (a source
 * read from particle files, as the paper's earlier PSL-file source model
 * does: particles at the plane translated and rotated on the GPU,
 * Sec. 3.1, Table 1): for the first n records of `plane` (written with
 * PSL_SAMPLE_PLANE for the same plan, possibly stored and read back), jaw
 * rejection, beam -> patient transform and phantom entry, with the same
 * arithmetic as sample_batch, so that the output is bit for bit what
 * sample_batch with PSL_SAMPLE_DENSE writes for those histories.  Dense
 * output in `out` (capacity >= n, *out->count = n, out->ptype = plane->ptype);
 * the tally receives the jaw and phantom-miss part of the ledger (the plane
 * sampling entered the rest).  A record whose beam index is not in the plan
 * is rejected as invalid.  Asynchronous on `stream`. */
int psl_transform_batch(const psl_plan* plan, const psl_phantom* phantom,
                        const psl_particles* plane, uint32_t n, psl_particles* out,
                        psl_tally* tally, void* stream);

/* ------------------------------------------------------------------------
 * Transport and tally
 * ------------------------------------------------------------------------ */

/* Physics switches.  Photons: free-electron Klein-Nishina Compton scattering
 * with Woodcock tracking; absorbed locally below e_cut_photon.  Electrons:
 * continuous slowing down with the Bethe collision stopping power of water
 * (optionally less the density-effect correction) scaled by density, steps
 * ending at voxel faces or after losing step_frac of
 * their energy, Highland Gaussian multiple scattering (ms_enable); absorbed
 * locally below e_cut_electron (Sec. 2.3 names the cut-offs). */
typedef struct {
    float e_cut_electron;   /* MeV, e.g. 0.2; at least 30/255 MeV, so that a
                               photon of up to 30 MeV (the top of the physics
                               tables) sets at most 255 electrons in motion,
                               the range of their 8-bit sub-stream ids      */
    float e_cut_photon;     /* MeV, e.g. 0.01  */
    float step_frac;        /* e.g. 0.1        */
    int32_t ms_enable;      /* 1 = on          */
    int32_t density_effect; /* 1 = collision stopping power less Sternheimer's
                               density-effect correction delta(T) of water;
                               0 = Bethe without it; other values: error */
    uint32_t physics;       /* optional photon processes and electron hard
                               events, PSL_PHYS_* bits (0 = Compton only and
                               continuous electron loss, the plain method)   */
} psl_transport_params;

/* Optional photon processes of psl_transport_params.physics (Sec. 2.3: the
 * paper's engine models them, naming only the cut-offs), all for water with
 * density scaling:
 *   PHOTO     photoelectric absorption on oxygen's two K electrons (Stobbe's
 *             hydrogenic cross-section, Slater-screened charge 7.7); the
 *             photoelectron (E less the K binding energy, along the photon)
 *             is transported or deposited like a Compton electron, the
 *             binding energy is deposited on the spot;
 *   RAYLEIGH  coherent scattering: the Thomson cross-section times the
 *             squared form factor of the molecule as independent hydrogenic
 *             atoms (oxygen 1s^2 2s^2 2p^4 with Slater-screened charges);
 *   PAIR      pair production in the nuclear field (unscreened Bethe-Heitler
 *             in Maximon's expansions, Z^2 summed over the molecule); the
 *             kinetic energy is shared with density 1 - 4/3 eps (1 - eps),
 *             both particles move along the photon; the positron is
 *             transported like an electron and annihilates at rest into two
 *             mc^2 photons, back to back and isotropic, each followed as a
 *             photon history of its own (id g | (2 sub + k) << 48, history ids
 *             below 2^48), which needs e_cut_electron <= mc^2. */
/* Optional electron hard events (each switchable; the paper's engine has
 * them, Sec. 2.3), water with density scaling:
 *   DELTA  Moller collisions transferring at least e_cut_electron (up to half
 *          the energy) are sampled as events, the delta electron transported
 *          on its own; below the cut-off the loss is continuous with the
 *          collision stopping power restricted to smaller transfers (ICRU 37,
 *          Rohrlich-Carlson F-);
 *   BREM   bremsstrahlung photons of at least e_cut_photon (Bethe-Heitler Born
 *          spectrum without screening, formula 3BN of Koch and Motz, with
 *          Z(Z+1) for the atomic electrons) are sampled as events, the photon
 *          along the electron and transported; below the cut-off the radiated
 *          energy is a continuous loss.
 * Events come at the rate of a step's initial energy: the number of mean free
 * paths to the next one is drawn at the start and after each event.  Delta
 * electrons and photons from electrons (bremsstrahlung, annihilation) are one
 * generation above their parent; generations up to 3 are transported, later
 * ones deposited where made (counted).  A secondary's random stream is the
 * splitmix64 hash of its parent's stream, event index and kind (the history
 * id kept in the low 48 bits, 0x8000 | 15 hashed bits above). */
enum { PSL_PHYS_PHOTO = 1, PSL_PHYS_RAYLEIGH = 2, PSL_PHYS_PAIR = 4, PSL_PHYS_DELTA = 8,
       PSL_PHYS_BREM = 16 };

/* A dose tally on `phantom`.  index_map_dev == NULL: one cell per voxel.
 * Otherwise (Sec. 2.2.2) index_map_dev is a device int32 [nz][ny][nx] map,
 * 0 = voxel not tallied, k > 0 = row k-1, and the tally is a 2D array
 * [n_rows][n_cols] addressed by (row, particle tag), n_cols <= 32768.  Holds an FP32 replica
 * array, FP64 sum and sum-of-squares arrays, the energy ledger and event
 * counters.  Synchronous. */
int psl_tally_create(const psl_phantom* phantom, const int32_t* index_map_dev, int32_t n_rows,
                     int32_t n_cols, psl_tally** out);
void psl_tally_free(psl_tally* tally);

/* Transports every particle of `in` (photons or electrons, per in->ptype) to
 * completion and adds the deposits of this replica to the tally's FP32 array.
 * Entries whose status bits are non-zero (dense sampling output of rejected
 * histories) are skipped.  Electrons set in motion by photons go through
 * `electrons`, a caller stack whose capacity must cover
 * in->capacity * (floor(e_max / e_cut_electron) + 1): each push costs the
 * photon at least e_cut_electron, and the stack is filled in chunks of 256
 * per wavefront (64 where the grid's wavefronts times 255 exceed
 * in->capacity) whose unused ends stay in it as empty (skipped) entries.  The
 * electron stack is grouped into energy bands before electron transport.  The
 * persistent transport grids hold ceil(in->capacity / 1024) workgroups of 256
 * (at most 2048), about four histories per lane.  Random numbers: Philox4x32-10 keyed
 * by `seed`, counter (block, 2<<16 | sub, g_lo, g_hi), sub 0 for the source
 * particle and 1+n for the electron of its n-th push. */
int transport_batch(const psl_phantom* phantom, const psl_particles* in,
                    psl_particles* electrons, psl_tally* tally,
                    const psl_transport_params* params, uint64_t seed, void* stream);

enum {
    PSL_TALLY_RESET = 1,     /* zero every array, ledger and counter          */
    PSL_TALLY_FOLD = 2,      /* sum += E_r, sum2 += E_r^2, E_r = 0 (FP64)     */
    PSL_TALLY_FINALIZE = 4   /* dose and its standard error from the folds    */
};

/* Tally operations, applied in the order RESET, FOLD, FINALIZE when several
 * bits are set.  FINALIZE writes dose_dev and sigma_dev (device FP64, one per
 * cell) in Gy per model particle, an absolute dose as the commissioning of
 * Sec. 2.2.2 needs it: mean over folded replicas of
 * 1.602176634e-10 * E / (rho V) * (column weight of `plan`: the Eq. (3)
 * normaliser over the histories of the column), and the standard error of
 * that mean.  plan, dose_dev and sigma_dev may be NULL without
 * FINALIZE. */
int tally_dose(psl_tally* tally, int32_t ops, const psl_plan* plan, double* dose_dev,
               double* sigma_dev, void* stream);

/* Synchronises with the device and reads the energy ledger (MeV, host double
 * [8]: source, jaw-rejected, missed phantom, invalid, escaped photons, escaped
 * electrons (an escaping positron adds its rest energy 2 mc^2), deposited,
 * electron path length in cm), the event counters (host uint64 [24]:
 * histories, entered, Woodcock steps, real interactions, particles pushed by
 * photons, local electron deposits, electron steps, atomic deposits,
 * uncollided escapes of source photons, Kahn trials, electron face crossings,
 * step-guard hits, overflows (a particle stack too small, or a particle column
 * beyond the tally), replicas folded, photoelectric absorptions, Rayleigh
 * scatterings, pair productions, positron annihilations, hard Moller
 * collisions, hard bremsstrahlung events, secondaries past the generation cap
 * (deposited where made); the rest are zero).
 * Returns PSL_EOVERFLOW if an overflow was counted since the last RESET.
 * Either output may be NULL. */
int psl_tally_stats(psl_tally* tally, double* ledger, uint64_t* counters);

/* Deposit recording, for measuring the atomic ceiling of the dose tally on
 * the address stream the transport really produces (Sec. 2.2.2: every
 * deposit of a run goes into the one shared dose array).  While cells_dev
 * (device uint32 [capacity]) is set, every FP32 deposit atomic that the
 * transport kernels issue into this tally also appends its cell index, in the
 * order the kernels issue them (the lanes of one wave's atomic in ascending
 * lane order, consecutive in the buffer).  *count_dev (device uint32, zeroed
 * by the caller) counts every recorded deposit; entries past `capacity` are
 * counted but not stored.  The recording kernels are separate builds, so
 * runs without a recording are unaffected.  cells_dev NULL stops the
 * recording.  The caller owns both buffers and keeps them alive while set. */
int psl_tally_record(psl_tally* tally, uint32_t* cells_dev, uint32_t capacity,
                     uint32_t* count_dev);

/* ------------------------------------------------------------------------
 * Batched runtime (Sec. 2.1.3: the sampling and transport kernels are iterated
 * over batches of one particle type; Sec. 2.2.2: all fields and basis doses in
 * one run)
 * ------------------------------------------------------------------------ */
typedef struct {
    uint32_t max_batch;      /* histories per batch (M), >= 64, e.g. 131072        */
    int32_t band_width;      /* energy bins per band, >= 1                          */
    int32_t use_graph;       /* 1: capture every launch of every replica once in a
                                hipGraph and replay it (cached while the plan,
                                phantom, options and parameters stay the same)     */
    int32_t sort_electrons;  /* 1: group electrons by energy band before transport */
    int32_t timing;          /* 1: launch eagerly (no graph) with a HIP event pair
                                around every kernel, read by psl_run_get_timing     */
    uint64_t seed;           /* Philox key                                          */
    int32_t lane_load;       /* histories per lane of the persistent transport
                                grids: they launch ceil(max_batch / (256 *
                                lane_load)) workgroups of 256, at most 2048
                                (0 = 4)                                            */
    int32_t pipelines;       /* 1 or 2 batch pipelines (own stacks and stream each);
                                with 2 the batches of a replica alternate between
                                them and run concurrently, joined before the
                                replica's fold; a replica of one batch uses one
                                (0 = 1)                                             */
} psl_run_opts;

/* Runs every batch of every replica of `plan` -- sample_batch, transport_batch
 * and one tally FOLD per replica, with replica r using history ids
 * g = r * N + h -- on `stream` (and, with two pipelines, on two streams of
 * the runtime forked from and joined back to `stream`).  Particle stacks live in the tally's workspace
 * (allocated on first use; the electron stack holds max_batch *
 * floor(e_max / e_cut_electron) entries, so it cannot overflow).  The tally is
 * not reset.  Asynchronous. */
int psl_run(psl_plan* plan, const psl_phantom* phantom, psl_tally* tally,
            const psl_transport_params* params, const psl_run_opts* opts, void* stream);

/* Kernel time of the last psl_run with timing = 1, summed per phase
 * (0 sampling, 1 photon transport, 2 electron energy sort, 3 electron
 * transport, 4 fold), and the number of launches of each.  Synchronises. */
typedef struct {
    double ms[5];
    uint64_t launches[5];
} psl_run_timing;
int psl_run_get_timing(psl_tally* tally, psl_run_timing* out);

/* Autotuner: times one replica (`replica`) of the plan for every candidate
 * (max_batch[i], band_width[j], lane_load[l], sort_electrons s in {0, 1},
 * pipelines p in {1, 2}) with graph replay, writes the measured milliseconds
 * to ms_out[(((i * n_w + j) * n_l + l) * 2 + s) * 2 + p - 1] (nullable).  The
 * candidates within 5 % of the fastest are timed again over three
 * back-to-back replays; *best is the first of them in that order within 1 %
 * of the fastest of that round (use_graph = 1, seed as given), so that
 * near-ties resolve alike from run to run.  Resets the tally afterwards.
 * Synchronous. */
int psl_autotune(psl_plan* plan, const psl_phantom* phantom, psl_tally* tally,
                 const psl_transport_params* params, uint64_t seed, const uint32_t* max_batch,
                 int32_t n_m, const int32_t* band_width, int32_t n_w, const int32_t* lane_load,
                 int32_t n_l, uint32_t replica, psl_run_opts* best, double* ms_out);

/* ------------------------------------------------------------------------
 * Ceiling probes (measurement helpers for the dose path's roofline)
 * ------------------------------------------------------------------------ */

/* FP32 atomic adds of 1.0 (result unused) into grid_dev[addr_dev[i]] for
 * i < n, the instruction the dose tally uses (every deposit of the transport
 * kernels goes into the shared FP32 replica grid; the paper does not
 * describe its tally); addresses outside [0, cells) are skipped.  Runs one
 * warm-up and `repeats` timed launches on a private stream and writes the
 * average milliseconds per launch to *ms_out.  grid_dev (device FP32
 * [cells]) accumulates every launch.  Synchronous. */
int psl_probe_atomics(float* grid_dev, int64_t cells, const int32_t* addr_dev, int64_t n,
                      int32_t repeats, double* ms_out);

/* Streaming device-to-device copy of `bytes` (a multiple of 16, both
 * buffers 16-byte aligned) with 16-byte loads and stores; average
 * milliseconds per launch over `repeats` timed launches after one warm-up.
 * Synchronous. */
int psl_probe_copy(void* dst_dev, const void* src_dev, int64_t bytes, int32_t repeats,
                   double* ms_out);

/* ------------------------------------------------------------------------
 * Commissioning (Sec. 2.2.3, Eq. 8; Sec. 2.2.4)
 * ------------------------------------------------------------------------ */
typedef struct {
    double delta;           /* stop when the relative decrease of F < delta ... */
    double pg_tol;          /* ... and |projected gradient| <= pg_tol |grad F(x0)| */
    double armijo_sigma;    /* sufficient-decrease constant, e.g. 1e-4         */
    double armijo_beta;     /* step reduction factor, e.g. 0.5                 */
    int64_t max_iter;
} psl_nnls_opts;

typedef struct {
    int64_t iters;
    double f;               /* ||A x - b||^2 at the returned x */
    double pg_norm;
} psl_nnls_report;

/* Solves min_{x >= 0} ||A x - b||^2 by gradient projection
 * x+ = max(0, x - s grad F(x)) with Armijo's rule; the trial step is the
 * Barzilai-Borwein step of the previous iteration.  A: host FP64 m x n,
 * column-major; b: host m; x: host n, in = start (e.g. all ones, the original
 * PSR weights), out = solution.  All vector work and the accept / stop
 * decisions run as FP64 kernels on the current device, on a stream of the
 * solver's own; each iteration tests up to 8 Armijo steps per pass over A and
 * takes the first that passes, i.e. the step of the sequential rule, and at
 * most 200 trials per iteration.  Sums have a fixed order, so a solve is
 * reproducible bit for bit.  Device memory: A plus 8 m ceil(n/32) + 9 m + 11 n
 * doubles, freed on return.  Synchronous.  Returns PSL_ENOTCONV (with x and
 * report filled) when max_iter is reached or the line search fails. */
int commission_nnls(const double* A, int64_t m, int64_t n, const double* b, double* x,
                    const psl_nnls_opts* opts, psl_nnls_report* report);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * solve as commission_nnls with every operand already on the device and the
 * solver's vectors in a fixed scratch array of PSL_NNLS_SCRATCH_BYTES that
 * the library holds on each device until the process ends.  It calls no
 * device or host allocator and creates no stream or graph.
 *   A_dev: device FP64 m x n, column-major; b_dev: device m; x_dev: device
 *   n, in = start (negative entries are clamped to 0 first), out = solution.
 *   The scratch holds 8 n + 2 n + 8 m + 8 m ceil(n / 32) + 8 ceil(m / 256)
 *   doubles plus a small state, each piece rounded up to 256 bytes; a system
 *   that needs more returns PSL_EINVAL before any device work (the
 *   1656 x 720 commissioning system needs 2.6 MB).
 *   stream: hipStream_t the kernels run on (NULL = default stream); the
 *   call synchronises with it once per 32 iteration steps and returns when
 *   the solve is done.
 * Same iterations, stop test and report as commission_nnls; ||A||_F^2 for the
 * first trial step is summed on the device, so the two calls can differ by
 * rounding.  Every call on one device shares that device's scratch array:
 * calls that overlap on one device (from two host threads or two streams)
 * race and give wrong results.  Returns PSL_ENOTCONV (x and report filled)
 * when max_iter is reached or the line search fails. */
#define PSL_NNLS_SCRATCH_BYTES (4u << 20)
int commission_nnls_noalloc(const double* A_dev, int64_t m, int64_t n, const double* b_dev,
                            double* x_dev, const psl_nnls_opts* opts, psl_nnls_report* report,
                            void* stream);

/* ------------------------------------------------------------------------
 * Learned 3D dose denoiser (not part of the paper's method): a 4-level U-Net
 * with c, 2c, 4c, 8c channels (two 3x3x3 conv + ReLU per level, 2x2x2 max
 * pooling down, 2x2x2 stride-2 transposed conv up, skip concatenation, 1x1x1
 * head plus the input dose), BF16 activations and weights on MFMA with FP32
 * accumulation, FP32 master weights, Adam on the mean squared error.
 * ------------------------------------------------------------------------ */
typedef struct psl_unet psl_unet;

/* Network for volumes of d x h x w voxels (multiples of 8) and base width
 * c in {8, 16, 32}; allocates all activation buffers.  Synchronous. */
int psl_unet_create(int32_t base_width, int32_t d, int32_t h, int32_t w, psl_unet** out);
void psl_unet_free(psl_unet* net);

/* Number of FP32 parameters.  Flat layout (host arrays), in this order: per
 * encoder level k = 0..3 conv a, conv b; per decoder level k = 2, 1, 0 the
 * transposed conv, conv a, conv b; the head.  Each conv: weights
 * [c_out][c_in][3][3][3] then bias [c_out]; each transposed conv: weights
 * [c_in][c_out][2][2][2] then bias [c_out]; head: weights [c] then bias [1].
 * The decoder's conv a reads [skip channels | upsampled channels]. */
int psl_unet_param_count(const psl_unet* net, int64_t* n);
/* Copies FP32 parameters in (resets the Adam state) / out. Synchronous. */
int psl_unet_set_params(psl_unet* net, const float* host);
int psl_unet_get_params(const psl_unet* net, float* host);

/* input_dev: device FP32 [2][d][h][w] (dose scaled by its maximum, density);
 * pred_dev: device FP32 [d][h][w] (scaled dose), written directly, must not
 * overlap input_dev.  Inference only: the last layer's activations, which
 * only the backward pass reads, are not kept.  Asynchronous. */
int psl_unet_forward(psl_unet* net, const float* input_dev, float* pred_dev, void* stream);

/* Forward + backward + one Adam step (beta 0.9 / 0.999, eps 1e-8) at learning
 * rate lr.  target_dev: device FP32 [d][h][w].  If loss_dev (device FP64
 * [64]) is given it receives partial sums whose total is the MSE before the
 * step.  Asynchronous. */
int psl_unet_train_step(psl_unet* net, const float* input_dev, const float* target_dev, float lr,
                        double* loss_dev, void* stream);

/* Loss and FP32 gradients (host, flat layout above) without an update; for
 * checking the backward kernels.  Synchronous. */
int psl_unet_gradients(psl_unet* net, const float* input_dev, const float* target_dev,
                       float* grads_host, double* loss);

/* Error gate of the denoiser, with the plain engine as the judge: compares a
 * candidate dose (cand_dev, device FP32 [nz][ny][nx], the network's
 * prediction on the dose scale) with an independent plain-engine dose and its
 * standard error (plain_dev, plain_sigma_dev, device FP64, same layout; the
 * plain run must use other random numbers than the run the candidate was made
 * from).  With M the largest mean of the candidate over blocks of block^3
 * voxels (edge in [1, 64]; a hot voxel does not set it), the voxels compared
 * are those where the candidate exceeds cutoff (in [0, 1)) times M (a choice
 * independent of the plain dose's noise).  With t = (cand - plain)^2 - sigma^2
 * per voxel and T_b, n_b its sum and voxel count over each block, writes host
 * double out[10]: voxels compared, M, the sum of (cand - plain)^2, the sum of
 * sigma^2, the sums over blocks of T_b^2, T_b n_b and n_b^2, the voxel count
 * and the plain dose summed over the candidate's top region (the blocks whose
 * candidate mean is at least 95 % of M), and the number of blocks with
 * compared voxels.  Since the plain dose is the true dose plus
 * independent noise of variance sigma^2, the mean of t estimates the
 * candidate's mean squared error against the true dose over those voxels;
 * the block sums give its standard error allowing for noise correlated
 * within a block; out[8] / out[7] reads the true dose of the candidate's top
 * region (a scale that a spurious hot spot of the candidate does not
 * inflate).  Sums are taken in a fixed order.  Synchronous on `stream`. */
int psl_dose_gate(const float* cand_dev, const double* plain_dev, const double* plain_sigma_dev,
                  int32_t nx, int32_t ny, int32_t nz, int32_t block, double cutoff, double* out,
                  void* stream);

#ifdef __cplusplus
}
#endif

#endif /* PSL_H */
