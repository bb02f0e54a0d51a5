/*
 * oracle.c -- plain, slow, FP64 CPU reference of the analytic phase-space-ring
 * (PSR) source model dose path of Tian et al., "An analytic linear accelerator
 * source model for Monte Carlo dose calculations. II" (arXiv:1503.01725).
 *
 * THIS IS TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load it.  It shares no code, header, table
 * or constant generator with the GPU engine; both sides receive the same
 * seeded inputs and each implements the counter-based Philox4x32-10 generator
 * from its published definition (Salmon et al., SC'11).
 *
 * Everything is written in the order the paper (or, where the paper is silent,
 * the documented reading) states it, with no blocking or fusion:
 *   - PSR -> PSL conversion ............ Sec. 2.1.1, Eqs. (1)-(2), steps 1-4
 *   - sampling areas ................... Sec. 2.1.2, Fig. 3, step S1
 *   - particles per PSL ................ step S2, Eq. (3)
 *   - history order .................... Sec. 2.1.3 (locations inner, energy outer)
 *   - primary / scatter / electron ..... steps S3-S5, Eqs. (4)-(7)
 *   - jaw rejection .................... Sec. 2.1.2 (upper jaw surfaces)
 *   - transport physics ................ paper silent (Sec. 2.3 only names the
 *                                        cut-offs); Klein-Nishina Compton with
 *                                        Woodcock tracking, Bethe CSDA electrons
 *                                        with Highland Gaussian multiple scattering
 *   - PSR-indexed tally ................ Sec. 2.2.2 (index map + 2D array)
 *   - commissioning .................... Sec. 2.2.3 Eq. (8), Sec. 2.2.4
 *
 * Parity pins live in tests/test_oracle_*.py.  Functions without an external
 * pin say so in their comment ("parity unpinned").
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_PI 3.14159265358979323846
#define OR_INF (1.0 / 0.0)

/* Physical constants (CODATA 2018). */
#define OR_ME 0.51099895000            /* electron rest energy, MeV */
#define OR_RE 2.8179403262e-13         /* classical electron radius, cm */
#define OR_NA 6.02214076e23            /* Avogadro, 1/mol */
#define OR_ZA_WATER (10.0 / 18.0153)   /* Z/A of water, mol/g */
#define OR_I_WATER 75.0e-6             /* mean excitation energy of water, MeV */
#define OR_X0_WATER 36.08              /* radiation length of water, g/cm^2 */
#define OR_MEV_PER_G_TO_GY 1.602176634e-10

enum { OR_TAG_SRC = 1, OR_TAG_TR = 2 };
enum { OR_ST_OK = 0, OR_ST_JAW = 1, OR_ST_MISSED = 2, OR_ST_INVALID = 3 };
enum { OR_SUB_PRIMARY = 0, OR_SUB_SCATTER = 1, OR_SUB_ELECTRON = 2 };

/* ledger[] slots */
enum { L_SRC = 0, L_JAW, L_MISSED, L_INVALID, L_ESC_G, L_ESC_E, L_DEP, L_EPATH, L_N };
/* counters[] slots */
enum { C_HIST = 0, C_ENTERED, C_WC_STEPS, C_REAL, C_E_PUSHED, C_E_LOCAL, C_E_STEPS,
       C_DEPOSITS, C_ESC_UNCOLLIDED, C_KAHN_TRIALS, C_E_BOUNDARY, C_GUARD, C_OVERFLOW,
       C_FOLDS, C_PHOTO = 14, C_RAYLEIGH, C_PAIR, C_ANNIHIL, C_MOLLER, C_BREM, C_CAPPED,
       C_N = 24 };

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as    */
/* easy as 1, 2, 3", SC'11): 10 rounds of the 4x32 Philox S-box with the     */
/* Weyl key schedule.                                                         */
/* ------------------------------------------------------------------------ */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* A stream of uniforms for one particle: key = seed, counter =
 * (block, tag<<16 | sub, g_lo, g_hi).  Uniforms are consumed in order, four
 * per Philox block; u = (x >> 8) * 2^-24, so u is in [0, 1) and exact in FP32. */
typedef struct {
    uint32_t key[2];
    uint32_t ctr[4];
    uint32_t buf[4];
    int left;
} or_stream;

static void stream_init(or_stream* s, uint64_t seed, uint64_t g, uint32_t tag, uint32_t sub)
{
    s->key[0] = (uint32_t)seed;
    s->key[1] = (uint32_t)(seed >> 32);
    s->ctr[0] = 0;
    s->ctr[1] = (tag << 16) | (sub & 0xFFFFu);
    s->ctr[2] = (uint32_t)g;
    s->ctr[3] = (uint32_t)(g >> 32);
    s->left = 0;
}

static double stream_u01(or_stream* s)
{
    if (s->left == 0) {
        or_philox4x32_10(s->ctr, s->key, s->buf);
        s->ctr[0] += 1;
        s->left = 4;
    }
    uint32_t x = s->buf[4 - s->left];
    s->left -= 1;
    return (double)(x >> 8) * (1.0 / 16777216.0);
}

/* test hook: n consecutive uniforms of stream (seed, g, tag, sub) */
void or_stream_uniforms(uint64_t seed, uint64_t g, uint32_t tag, uint32_t sub, int n, double* out)
{
    or_stream s;
    stream_init(&s, seed, g, tag, sub);
    for (int i = 0; i < n; ++i) out[i] = stream_u01(&s);
}

/* ------------------------------------------------------------------------ */
/* Inputs                                                                     */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t n_ebin, n_ring, n_comp, n_psl;
    double e_lo, e_width, ring_dr, psl_x0, psl_dx;
    double z_target, z_plane, z_scatter, z_jaw_y, z_jaw_x;
    double sigma_spot, sig_ea, sig_eb;
    const double* w_psr;   /* [3][n_ebin][n_ring] */
    const double* sc_c;    /* [n_ebin][n_ring][K] */
    const double* sc_mu;
    const double* sc_sa;
    const double* sc_sb;
} or_model;

typedef struct {
    double x1, x2, y1, y2;   /* jaw edges projected to the isocentre plane */
    double gantry_deg, couch_deg;
    double iso[3];
} or_beam;

typedef struct {
    int32_t nx, ny, nz, pad;
    double vox[3];
    double origin[3];
    const float* density;    /* [nz][ny][nx] */
} or_phantom;

typedef struct {
    double e_cut_e, e_cut_g, step_frac;
    int32_t ms_enable;
    int32_t density_effect;  /* 1 = collision stopping power with delta(T) */
    int32_t physics;         /* OR_PHYS_* bits: photoelectric, Rayleigh, pair */
} or_params;

typedef struct {
    int64_t n_list;
    const int32_t* beam;
    const int32_t* stype;
    const int32_t* ebin;
    const int32_t* ix;
    const int32_t* iy;
    const int32_t* tag;      /* tally column (basis) carried by the particle */
    const uint64_t* cum;     /* inclusive prefix of per-PSL counts */
    uint64_t n_hist;         /* N = cum[n_list-1] */
} or_plan;

/* ------------------------------------------------------------------------ */
/* Sec. 2.1.1: PSR -> PSL conversion.                                         */
/* ------------------------------------------------------------------------ */

/* Step 2 of Sec. 2.1.1: ring weight at radius r by linear interpolation between
 * ring centres; inside the first centre the first ring's weight, between the
 * last centre and the model's outer radius the last ring's weight, 0 beyond. */
static double ring_weight_at(const double* w_ring, int n_ring, double dr, double r)
{
    double r_outer = (double)n_ring * dr;
    if (r > r_outer) return 0.0;
    double t = r / dr - 0.5;
    if (t <= 0.0) return w_ring[0];
    if (t >= (double)(n_ring - 1)) return w_ring[n_ring - 1];
    int j = (int)floor(t);
    double f = t - (double)j;
    return (1.0 - f) * w_ring[j] + f * w_ring[j + 1];
}

/* Eq. (2) in discrete form (Sec. 2.1.1 steps 1-4): PSL weight = interpolated
 * ring weight / (2 pi r) at the PSL centre, normalised so that the sum over all
 * sub-sources, energies and locations is 1.  The normalising sum runs in the
 * order (s, b, iy, ix).  Output w_psl[3][n_ebin][n_psl][n_psl]; returns the sum. */
double or_psl_build(const or_model* m, double* w_psl)
{
    const int n = m->n_psl;
    for (int s = 0; s < 3; ++s)
        for (int b = 0; b < m->n_ebin; ++b) {
            const double* wr = m->w_psr + ((size_t)s * m->n_ebin + b) * m->n_ring;
            for (int iy = 0; iy < n; ++iy)
                for (int ix = 0; ix < n; ++ix) {
                    double xc = m->psl_x0 + ((double)ix + 0.5) * m->psl_dx;
                    double yc = m->psl_x0 + ((double)iy + 0.5) * m->psl_dx;
                    double r = sqrt(xc * xc + yc * yc);
                    double w = ring_weight_at(wr, m->n_ring, m->ring_dr, r);
                    w_psl[(((size_t)s * m->n_ebin + b) * n + iy) * n + ix] = w / ((2.0 * OR_PI) * r);
                }
        }
    size_t total = (size_t)3 * m->n_ebin * n * n;
    double sum = 0.0;
    for (size_t i = 0; i < total; ++i) sum += w_psl[i];
    for (size_t i = 0; i < total; ++i) w_psl[i] = w_psl[i] / sum;
    return sum;
}

/* Step S4: cumulative component table P_{i,k} = sum_{j<=k} c_{i,j} / sum_j c_{i,j}
 * for k = 0..K-2 (the last entry is 1 by definition).  Output [n_ebin][n_ring][K]. */
void or_scatter_cdf(const or_model* m, double* P)
{
    const int K = m->n_comp;
    for (int i = 0; i < m->n_ebin * m->n_ring; ++i) {
        const double* c = m->sc_c + (size_t)i * K;
        double tot = 0.0;
        for (int k = 0; k < K; ++k) tot += c[k];
        double acc = 0.0;
        for (int k = 0; k < K; ++k) {
            acc += c[k];
            P[(size_t)i * K + k] = (k == K - 1) ? 1.0 : acc / tot;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Sec. 2.1.2 / Fig. 3 / step S1: sampling areas.                             */
/* ------------------------------------------------------------------------ */
#define OR_AREA_NSIGMA 4.0

/* Largest angular width of a sub-source's direction model (rad). */
static double sub_source_sigma_max(const or_model* m, int stype)
{
    if (stype == OR_SUB_ELECTRON) return fmax(m->sig_ea, m->sig_eb);
    double smax = 0.0;
    size_t n = (size_t)m->n_ebin * m->n_ring * m->n_comp;
    for (size_t i = 0; i < n; ++i) {
        smax = fmax(smax, m->sc_sa[i]);
        smax = fmax(smax, m->sc_sb[i]);
    }
    return smax;
}

/* One axis of the sampling strip at the plane for jaw edges e1 < e2 given at
 * the isocentre plane, jaw upper surface at height zj. */
static void sampling_strip(const or_model* m, int stype, double e1, double e2, double zj,
                           double* lo, double* hi)
{
    const double zt = m->z_target, zp = m->z_plane;
    /* jaw edges at the height of the upper surface (faces focus on the target) */
    double j1 = e1 * (zj - zt) / (zp - zt);
    double j2 = e2 * (zj - zt) / (zp - zt);
    if (stype == OR_SUB_PRIMARY) {
        /* jaw opening seen from the focal spot, widened by the shadow of an
         * n-sigma focal spot through the jaw edge */
        double margin = OR_AREA_NSIGMA * m->sigma_spot * (zp - zj) / (zj - zt);
        *lo = e1 - margin;
        *hi = e2 + margin;
        return;
    }
    /* The mean ray of a plane point comes from a source point on the axis at
     * height zs (scatter source; electrons: zs -> -inf, vertical mean ray).
     * The ray through the jaw edge lands at c = j (zp - zs)/(zj - zs); a
     * deviation d from the mean direction moves the crossing point at the jaw
     * by (zp - zj) tan(d), i.e. the plane point by that times (zp - zs)/(zj - zs). */
    double c1, c2, magnify;
    if (stype == OR_SUB_SCATTER) {
        double zs = m->z_scatter;
        magnify = (zp - zs) / (zj - zs);
    } else {
        magnify = 1.0;
    }
    c1 = j1 * magnify;
    c2 = j2 * magnify;
    double margin = (zp - zj) * tan(OR_AREA_NSIGMA * sub_source_sigma_max(m, stype)) * magnify;
    *lo = c1 - margin;
    *hi = c2 + margin;
}

/* PSL index box [ix0, ix1] x [iy0, iy1] (inclusive) of the PSLs whose squares
 * overlap the sampling rectangle with positive area; the rectangle is the
 * intersection of the x strip (X jaws) and the y strip (Y jaws). */
void or_sampling_box(const or_model* m, const or_beam* bm, int stype, int32_t box[4])
{
    double xlo, xhi, ylo, yhi;
    sampling_strip(m, stype, bm->x1, bm->x2, m->z_jaw_x, &xlo, &xhi);
    sampling_strip(m, stype, bm->y1, bm->y2, m->z_jaw_y, &ylo, &yhi);
    const double x0 = m->psl_x0, dx = m->psl_dx;
    int ix0 = (int)floor((xlo - x0) / dx), ix1 = (int)ceil((xhi - x0) / dx) - 1;
    int iy0 = (int)floor((ylo - x0) / dx), iy1 = (int)ceil((yhi - x0) / dx) - 1;
    if (ix0 < 0) ix0 = 0;
    if (iy0 < 0) iy0 = 0;
    if (ix1 > m->n_psl - 1) ix1 = m->n_psl - 1;
    if (iy1 > m->n_psl - 1) iy1 = m->n_psl - 1;
    box[0] = ix0; box[1] = ix1; box[2] = iy0; box[3] = iy1;
}

/* ------------------------------------------------------------------------ */
/* Step S2 / Eq. (3): particles per PSL, and the history order of Sec. 2.1.3. */
/* ------------------------------------------------------------------------ */
static int psl_ring_of_centre(const or_model* m, int ix, int iy)
{
    double xc = m->psl_x0 + ((double)ix + 0.5) * m->psl_dx;
    double yc = m->psl_x0 + ((double)iy + 0.5) * m->psl_dx;
    int ring = (int)floor(sqrt(xc * xc + yc * yc) / m->ring_dr);
    return ring < m->n_ring - 1 ? ring : m->n_ring - 1;
}

/* Systematic rounding of N * q_i / sum(q) inside one group of list entries
 * [a, b): n_i = round(N*Q_i/S) - round(N*Q_{i-1}/S), Q the running prefix of q.
 * The totals add to N exactly and each n_i is the floor or ceiling of its
 * fractional share.  128-bit integer arithmetic. */
static void systematic_counts(const uint64_t* q, int64_t a, int64_t b, uint64_t n_group,
                              uint64_t* n_out)
{
    unsigned __int128 S = 0;
    for (int64_t i = a; i < b; ++i) S += q[i];
    if (S == 0) {
        for (int64_t i = a; i < b; ++i) n_out[i] = 0;
        return;
    }
    unsigned __int128 acc = 0, prev = 0;
    for (int64_t i = a; i < b; ++i) {
        acc += q[i];
        unsigned __int128 cum = ((unsigned __int128)n_group * acc + S / 2) / S;
        n_out[i] = (uint64_t)(cum - prev);
        prev = cum;
    }
}

/* Builds the list of in-area PSLs and their particle counts.
 *
 * Order (Sec. 2.1.3; S1 repeats S2-S5 per beam, S3->S5 are the sub-sources):
 * beam, sub-source, energy bin, iy, ix -- location is the inner loop, energy
 * the outer one.  With hist_per_basis > 0 (commissioning, Sec. 2.2.2) each
 * (beam, basis) group receives hist_per_basis histories spread over its own
 * PSLs and the order is beam, basis, sub-source, energy, iy, ix.  Otherwise
 * Eq. (3) allocates n_hist over the whole list (the denominator sums the
 * sampling areas of all beams).
 *
 * The tally tag of an entry is beam * n_basis + basis when a basis map is given,
 * else 0.  Weights are quantised to q = llround(w * 2^40) before rounding.
 *
 * Outputs (caller-allocated, max_list entries): beam, stype, ebin, ix, iy, tag,
 * w (FP64 weight), cum (inclusive prefix of counts); group_w / group_n are the
 * per-(beam, basis) weight sum and history count (index beam * n_basis + basis,
 * or [0] for the whole list).  Returns the list length or -1 if max_list is too
 * small. */
int64_t or_plan_build(const or_model* m, const double* w_psl, const or_beam* beams, int n_beams,
                      uint64_t n_hist, const uint16_t* basis_map, int32_t n_basis,
                      uint64_t hist_per_basis, int64_t max_list,
                      int32_t* beam_o, int32_t* stype_o, int32_t* ebin_o, int32_t* ix_o,
                      int32_t* iy_o, int32_t* tag_o, double* w_o, uint64_t* cum_o,
                      double* group_w, uint64_t* group_n)
{
    const int n = m->n_psl;
    int64_t len = 0;
    int stratified = (hist_per_basis > 0 && basis_map != NULL);
    int nb = basis_map ? n_basis : 1;
    int* ring_of = (int*)malloc(sizeof(int) * (size_t)n * n);
    for (int iy = 0; iy < n; ++iy)
        for (int ix = 0; ix < n; ++ix) ring_of[iy * n + ix] = psl_ring_of_centre(m, ix, iy);
    for (int beam = 0; beam < n_beams; ++beam) {
        int32_t boxes[3][4];
        for (int s = 0; s < 3; ++s) or_sampling_box(m, &beams[beam], s, boxes[s]);
        int k_lo = 0, k_hi = stratified ? nb : 1;
        for (int k = k_lo; k < k_hi; ++k)
            for (int s = 0; s < 3; ++s)
                for (int b = 0; b < m->n_ebin; ++b)
                    for (int iy = boxes[s][2]; iy <= boxes[s][3]; ++iy)
                        for (int ix = boxes[s][0]; ix <= boxes[s][1]; ++ix) {
                            double w = w_psl[(((size_t)s * m->n_ebin + b) * n + iy) * n + ix];
                            if (!(w > 0.0)) continue;
                            int basis = 0;
                            if (basis_map) {
                                int ring = ring_of[iy * n + ix];
                                basis = basis_map[((size_t)s * m->n_ebin + b) * m->n_ring + ring];
                                if (stratified && basis != k) continue;
                            }
                            if (len >= max_list) { free(ring_of); return -1; }
                            beam_o[len] = beam; stype_o[len] = s; ebin_o[len] = b;
                            ix_o[len] = ix; iy_o[len] = iy;
                            tag_o[len] = basis_map ? beam * nb + basis : 0;
                            w_o[len] = w;
                            len++;
                        }
    }
    free(ring_of);
    uint64_t* q = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(len > 0 ? len : 1));
    uint64_t* cnt = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(len > 0 ? len : 1));
    for (int64_t i = 0; i < len; ++i) q[i] = (uint64_t)llround(w_o[i] * 1099511627776.0);
    if (stratified) {
        for (int g = 0; g < n_beams * nb; ++g) { group_w[g] = 0.0; group_n[g] = 0; }
        int64_t a = 0;
        while (a < len) {
            int64_t b = a;
            while (b < len && tag_o[b] == tag_o[a]) ++b;
            systematic_counts(q, a, b, hist_per_basis, cnt);
            double wsum = 0.0;
            for (int64_t i = a; i < b; ++i) wsum += w_o[i];
            group_w[tag_o[a]] = wsum;
            group_n[tag_o[a]] = hist_per_basis;
            a = b;
        }
    } else {
        systematic_counts(q, 0, len, n_hist, cnt);
        double wsum = 0.0;
        for (int64_t i = 0; i < len; ++i) wsum += w_o[i];
        group_w[0] = wsum;
        group_n[0] = n_hist;
    }
    uint64_t acc = 0;
    for (int64_t i = 0; i < len; ++i) { acc += cnt[i]; cum_o[i] = acc; }
    free(q);
    free(cnt);
    return len;
}

/* ------------------------------------------------------------------------ */
/* Geometry helpers                                                           */
/* ------------------------------------------------------------------------ */

/* Beam frame -> patient frame rotation R = Rz(couch) * Ry(gantry). */
static void beam_rotation(const or_beam* bm, double R[9])
{
    double g = bm->gantry_deg * OR_PI / 180.0, c = bm->couch_deg * OR_PI / 180.0;
    double cg = cos(g), sg = sin(g), cc = cos(c), sc = sin(c);
    /* Ry(g) = [[cg,0,sg],[0,1,0],[-sg,0,cg]];  Rz(c) = [[cc,-sc,0],[sc,cc,0],[0,0,1]] */
    double Ry[9] = {cg, 0.0, sg, 0.0, 1.0, 0.0, -sg, 0.0, cg};
    double Rz[9] = {cc, -sc, 0.0, sc, cc, 0.0, 0.0, 0.0, 1.0};
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double a = 0.0;
            for (int k = 0; k < 3; ++k) a += Rz[i * 3 + k] * Ry[k * 3 + j];
            R[i * 3 + j] = a;
        }
}

/* Entry of the infinite line p + t d into the phantom box (slab method).
 * *t_entry / *t_exit receive the parameters where the line enters and leaves;
 * returns 1 if t_exit > t_entry (the line crosses the box), else 0. */
static int ray_box_entry(const or_phantom* ph, const double p[3], const double d[3],
                         double* t_entry, double* t_exit)
{
    double tmin = -OR_INF, tmax = OR_INF;
    const int n[3] = {ph->nx, ph->ny, ph->nz};
    for (int a = 0; a < 3; ++a) {
        double lo = ph->origin[a], hi = ph->origin[a] + (double)n[a] * ph->vox[a];
        if (d[a] != 0.0) {
            double t1 = (lo - p[a]) / d[a], t2 = (hi - p[a]) / d[a];
            double tn = fmin(t1, t2), tf = fmax(t1, t2);
            if (tn > tmin) tmin = tn;
            if (tf < tmax) tmax = tf;
        } else if (p[a] < lo || p[a] > hi) {
            tmax = -OR_INF;
        }
    }
    *t_entry = tmin;
    *t_exit = tmax;
    return tmax > tmin;
}

/* Voxel index of a point, or -1 outside the phantom. */
static int64_t voxel_of(const or_phantom* ph, const double p[3], int idx[3])
{
    const int n[3] = {ph->nx, ph->ny, ph->nz};
    for (int a = 0; a < 3; ++a) {
        double f = floor((p[a] - ph->origin[a]) / ph->vox[a]);
        if (!(f >= 0.0 && f < (double)n[a])) return -1;
        idx[a] = (int)f;
    }
    return ((int64_t)idx[2] * ph->ny + idx[1]) * ph->nx + idx[0];
}

/* Voxel index of a point on or inside the box, clamped onto the grid. */
static void voxel_clamped(const or_phantom* ph, const double p[3], int idx[3])
{
    const int n[3] = {ph->nx, ph->ny, ph->nz};
    for (int a = 0; a < 3; ++a) {
        double f = floor((p[a] - ph->origin[a]) / ph->vox[a]);
        if (f < 0.0) f = 0.0;
        if (f > (double)(n[a] - 1)) f = (double)(n[a] - 1);
        idx[a] = (int)f;
    }
}

/* Turns direction d by polar angle theta (given by cos) and azimuth phi about
 * the old direction: the new direction makes angle theta with d, and phi is
 * measured from the plane of d and the z axis (from the x axis when d lies on
 * the z axis).  The transverse length t = sqrt(u^2 + v^2) is taken from u and
 * v, not from 1 - w^2, so that the rotation stays exact next to the axis. */
static void rotate_direction(double d[3], double cos_t, double phi)
{
    double sin_t = sqrt(fmax(0.0, 1.0 - cos_t * cos_t));
    double cp = cos(phi), sp = sin(phi);
    double u = d[0], v = d[1], w = d[2];
    double nu, nv, nw;
    double t = sqrt(u * u + v * v);
    if (t > 1e-30) {
        nu = u * cos_t + sin_t * (u * w * cp - v * sp) / t;
        nv = v * cos_t + sin_t * (v * w * cp + u * sp) / t;
        nw = w * cos_t - sin_t * cp * t;
    } else {
        nu = sin_t * cp;
        nv = sin_t * sp;
        nw = (w > 0.0 ? 1.0 : -1.0) * cos_t;
    }
    double norm = sqrt(nu * nu + nv * nv + nw * nw);
    d[0] = nu / norm; d[1] = nv / norm; d[2] = nw / norm;
}

/* test hook: rotate_direction applied to a copy of d */
void or_rotate_direction(const double d[3], double cos_t, double phi, double out[3])
{
    out[0] = d[0]; out[1] = d[1]; out[2] = d[2];
    rotate_direction(out, cos_t, phi);
}

/* ------------------------------------------------------------------------ */
/* Steps S3-S5: sampling one history.                                         */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t j, k, status, stype, beam, ebin, ix, iy, tag, pad;
    double xb, yb;            /* position on the plane, beam frame */
    double ub, vb, wb;        /* direction, beam frame (after the rotation by theta) */
    double e;
    double xs, ys;            /* focal-spot point (primary) */
    double alpha, beta;       /* local direction angles (scatter, electron) */
    double jaw_margin;        /* distance of the back-traced point to the nearest jaw edge */
    double box_margin;        /* chord length of the line through the phantom box */
    double ring_margin;       /* distance of r to the nearest ring edge (scatter) */
    double x, y, z, u, v, w;  /* patient frame, at the phantom entry */
} or_sample_rec;

/* First index j with cum[j] > h (upper bound). */
static int64_t upper_bound_u64(const uint64_t* cum, int64_t n, uint64_t h)
{
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (cum[mid] > h) hi = mid; else lo = mid + 1;
    }
    return lo;
}

typedef struct {
    const or_model* m;
    const double* cdf;      /* [n_ebin][n_ring][K] */
    const or_plan* plan;
    const or_beam* beams;
    double (*R)[9];         /* per-beam rotations */
    const or_phantom* ph;
} or_sampler;

static void sample_history(const or_sampler* S, uint64_t seed, uint64_t g, or_sample_rec* rec)
{
    const or_model* m = S->m;
    const or_plan* P = S->plan;
    uint64_t h = g % P->n_hist;
    int64_t j = upper_bound_u64(P->cum, P->n_list, h);
    memset(rec, 0, sizeof(*rec));
    rec->j = (int32_t)j;
    rec->k = -1;
    rec->stype = P->stype[j];
    rec->beam = P->beam[j];
    rec->ebin = P->ebin[j];
    rec->ix = P->ix[j];
    rec->iy = P->iy[j];
    rec->tag = P->tag[j];
    const or_beam* bm = &S->beams[rec->beam];

    or_stream st;
    stream_init(&st, seed, g, OR_TAG_SRC, 0);
    double u0 = stream_u01(&st), u1 = stream_u01(&st), u2 = stream_u01(&st), u3 = stream_u01(&st);
    double u4 = stream_u01(&st), u5 = stream_u01(&st);

    /* uniform position inside the PSL and uniform energy inside the bin */
    double x = (m->psl_x0 + (double)rec->ix * m->psl_dx) + m->psl_dx * u0;
    double y = (m->psl_x0 + (double)rec->iy * m->psl_dx) + m->psl_dx * u1;
    double e = (m->e_lo + (double)rec->ebin * m->e_width) + m->e_width * u2;
    double r = sqrt(x * x + y * y);
    double ct = 1.0, stt = 0.0;
    if (r > 0.0) { ct = x / r; stt = y / r; }

    /* Box-Muller pair */
    double rad = sqrt(-2.0 * log(1.0 - u4));
    double g1 = rad * cos(2.0 * OR_PI * u5), g2 = rad * sin(2.0 * OR_PI * u5);

    double ul, vl, wl;
    int invalid = 0;
    if (rec->stype == OR_SUB_PRIMARY) {
        /* Eq. (4): focal-spot point from a 2D Gaussian; Eq. (5): direction */
        double zph = m->z_plane - m->z_target;
        double xs = m->sigma_spot * g1, ys = m->sigma_spot * g2;
        double dxr = r - xs;
        double D = sqrt(dxr * dxr + ys * ys + zph * zph);
        ul = dxr / D; vl = -ys / D; wl = zph / D;
        rec->xs = xs; rec->ys = ys;
    } else {
        double alpha, beta;
        if (rec->stype == OR_SUB_SCATTER) {
            /* Eq. (6): PSR index from the sampled radius, component from the
             * cumulative table (decision taken in FP32), then one Gaussian */
            int ring = (int)floor(r / m->ring_dr);
            rec->ring_margin = fmin(r - ring * m->ring_dr, (ring + 1) * m->ring_dr - r);
            if (ring > m->n_ring - 1) ring = m->n_ring - 1;
            size_t base = ((size_t)rec->ebin * m->n_ring + ring) * m->n_comp;
            int k = 0;
            while (k < m->n_comp - 1 && !((float)u3 < (float)S->cdf[base + k])) ++k;
            rec->k = k;
            alpha = m->sc_mu[base + k] + m->sc_sa[base + k] * g1;
            beta = m->sc_sb[base + k] * g2;
        } else {
            /* Eq. (7): zero-mean Gaussian angles */
            alpha = m->sig_ea * g1;
            beta = m->sig_eb * g2;
        }
        rec->alpha = alpha; rec->beta = beta;
        if (fabs(alpha) >= 0.5 * OR_PI || fabs(beta) >= 0.5 * OR_PI) invalid = 1;
        /* alpha = atan(u/w), beta = atan(v/w) */
        double ta = tan(alpha), tb = tan(beta);
        double nrm = sqrt(ta * ta + tb * tb + 1.0);
        ul = ta / nrm; vl = tb / nrm; wl = 1.0 / nrm;
    }
    /* rotation of the local (radial, tangential) frame by theta = atan2(y, x) */
    double u = ct * ul - stt * vl;
    double v = stt * ul + ct * vl;
    double w = wl;
    rec->xb = x; rec->yb = y; rec->ub = u; rec->vb = v; rec->wb = w; rec->e = e;

    if (invalid) { rec->status = OR_ST_INVALID; return; }

    /* jaw rejection at the upper jaw surfaces (closed intervals) */
    const double zt = m->z_target, zp = m->z_plane;
    double yj = y + (v / w) * (m->z_jaw_y - zp);
    double xj = x + (u / w) * (m->z_jaw_x - zp);
    double ky = (m->z_jaw_y - zt) / (zp - zt), kx = (m->z_jaw_x - zt) / (zp - zt);
    double y1 = bm->y1 * ky, y2 = bm->y2 * ky, x1 = bm->x1 * kx, x2 = bm->x2 * kx;
    rec->jaw_margin = fmin(fmin(fabs(yj - y1), fabs(yj - y2)), fmin(fabs(xj - x1), fabs(xj - x2)));
    if (!(yj >= y1 && yj <= y2 && xj >= x1 && xj <= x2)) { rec->status = OR_ST_JAW; return; }

    /* beam frame -> patient frame; the plane is the isocentre plane */
    const double* R = S->R[rec->beam];
    double pb[3] = {x, y, 0.0}, db[3] = {u, v, w}, p[3], d[3];
    for (int i = 0; i < 3; ++i) {
        p[i] = bm->iso[i] + R[i * 3 + 0] * pb[0] + R[i * 3 + 1] * pb[1] + R[i * 3 + 2] * pb[2];
        d[i] = R[i * 3 + 0] * db[0] + R[i * 3 + 1] * db[1] + R[i * 3 + 2] * db[2];
    }
    double t, t_exit;
    int hit = ray_box_entry(S->ph, p, d, &t, &t_exit);
    /* chord length through the box (negative: distance by which it misses) */
    rec->box_margin = t_exit - t;
    if (!hit) { rec->status = OR_ST_MISSED; return; }
    rec->x = p[0] + t * d[0]; rec->y = p[1] + t * d[1]; rec->z = p[2] + t * d[2];
    rec->u = d[0]; rec->v = d[1]; rec->w = d[2];
    rec->status = OR_ST_OK;
}

/* ------------------------------------------------------------------------ */
/* Photon physics: free-electron Klein-Nishina Compton scattering.            */
/* ------------------------------------------------------------------------ */

/* Total Klein-Nishina cross-section per electron (cm^2), textbook form. */
double or_kn_sigma(double e)
{
    double k = e / OR_ME;
    double a = 1.0 + 2.0 * k;
    double l = log(a);
    return 2.0 * OR_PI * OR_RE * OR_RE *
           ((1.0 + k) / (k * k) * (2.0 * (1.0 + k) / a - l / k) + l / (2.0 * k) -
            (1.0 + 3.0 * k) / (a * a));
}

/* Electron density of water at unit mass density (electrons / cm^3). */
static double ne_water(void) { return OR_NA * OR_ZA_WATER; }

/* Kahn's rejection method for the Klein-Nishina distribution of
 * x = E/E' in [1, 1+2k]: with probability (1+2k)/(9+2k) propose x uniform and
 * accept with 4(x-1)/x^2, otherwise propose x with density ~1/x^2 and accept
 * with (cos^2 + 1/x)/2.  Three uniforms per trial. Returns x. */
static double kahn_sample(or_stream* st, double k, uint64_t* trials)
{
    for (;;) {
        double r1 = stream_u01(st), r2 = stream_u01(st), r3 = stream_u01(st);
        if (trials) (*trials)++;
        if (r1 <= (1.0 + 2.0 * k) / (9.0 + 2.0 * k)) {
            double x = 1.0 + 2.0 * k * r2;
            if (r3 <= 4.0 * (1.0 / x - 1.0 / (x * x))) return x;
        } else {
            double x = (1.0 + 2.0 * k) / (1.0 + 2.0 * k * r2);
            double c = 1.0 - (x - 1.0) / k;
            if (r3 <= 0.5 * (c * c + 1.0 / x)) return x;
        }
    }
}

/* Compton scattering of a photon of energy e moving along d on a free
 * electron at rest, for x = E/E' (cos theta = 1 - (x - 1)/k, k = E/mc^2) and
 * azimuth phi: scattered energy E' = E/x and direction d1 (d turned by theta,
 * phi); the electron takes T = E - E' and the momentum E d - E' d1 (units of
 * MeV/c), whose direction is returned in de. */
static void compton_kinematics(double e, const double d[3], double x, double phi, double* e1,
                               double d1[3], double* te, double de[3])
{
    double k = e / OR_ME;
    double cos_t = 1.0 - (x - 1.0) / k;
    *e1 = e / x;
    *te = e - *e1;
    d1[0] = d[0]; d1[1] = d[1]; d1[2] = d[2];
    rotate_direction(d1, cos_t, phi);
    double nrm = 0.0;
    for (int a = 0; a < 3; ++a) { de[a] = e * d[a] - (*e1) * d1[a]; nrm += de[a] * de[a]; }
    nrm = sqrt(nrm);
    for (int a = 0; a < 3; ++a) de[a] /= nrm;
}

/* test hook: compton_kinematics; out = {E', T, d1[3], de[3]} */
void or_compton(double e, const double d[3], double x, double phi, double out[8])
{
    compton_kinematics(e, d, x, phi, &out[0], &out[2], &out[1], &out[5]);
}

/* test hook: n Klein-Nishina scattering cosines at energy e (stream g = i) */
void or_kn_sample_cos(double e, uint64_t seed, int n, double* cos_out)
{
    double k = e / OR_ME;
    for (int i = 0; i < n; ++i) {
        or_stream st;
        stream_init(&st, seed, (uint64_t)i, OR_TAG_TR, 0);
        double x = kahn_sample(&st, k, NULL);
        cos_out[i] = 1.0 - (x - 1.0) / k;
    }
}

/* Gauss-Legendre nodes/weights on [-1, 1] from Newton iteration on P_n. */
#define OR_GL_N 8
static double gl_x[OR_GL_N], gl_w[OR_GL_N];
static void gl_init(void)
{
    const int n = OR_GL_N;
    for (int i = 0; i < n; ++i) {
        double z = cos(OR_PI * ((double)i + 0.75) / ((double)n + 0.5)), pp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p1 = 1.0, p2 = 0.0;
            for (int j = 1; j <= n; ++j) {
                double p3 = p2;
                p2 = p1;
                p1 = ((2.0 * j - 1.0) * z * p2 - (j - 1.0) * p3) / j;
            }
            pp = n * (z * p1 - p2) / (z * z - 1.0);
            double z1 = z;
            z = z1 - p1 / pp;
            if (fabs(z - z1) < 1e-16) break;
        }
        gl_x[i] = z;
        gl_w[i] = 2.0 / ((1.0 - z * z) * pp * pp);
    }
}

/* ------------------------------------------------------------------------ */
/* Fuller photon physics, each switchable: photoelectric absorption, Rayleigh */
/* (coherent) scattering and pair production in water.  The paper's engine    */
/* models them (Sec. 2.3 names only its cut-offs) without giving forms; the   */
/* forms below are published analytic ones.                                   */
/* ------------------------------------------------------------------------ */
#define OR_ALPHA 7.2973525693e-3          /* fine-structure constant */
#define OR_A0 0.529177210903e-8           /* Bohr radius, cm */
#define OR_RY 13.605693122994e-6          /* Rydberg energy, MeV */
#define OR_HBARC 1.973269804e-11          /* hbar c, MeV cm */
#define OR_ZETA3 1.2020569031595942       /* Riemann zeta(3) */
#define OR_MOL_PER_G (OR_NA / 18.0153)    /* water molecules per gram */
/* Slater-screened nuclear charges seen by oxygen's 1s and n = 2 electrons
 * (Slater's rules: 8 - 0.30 and 8 - 2 x 0.85 - 5 x 0.35). */
#define OR_Z_O_1S 7.70
#define OR_Z_O_2 4.55
enum { OR_PHYS_PHOTO = 1, OR_PHYS_RAYLEIGH = 2, OR_PHYS_PAIR = 4, OR_PHYS_DELTA = 8,
       OR_PHYS_BREM = 16 };

/* Photoeffect cross-section (cm^2) of one electron of a hydrogenic K shell of
 * nuclear charge z, in Stobbe's exact non-relativistic form:
 *   sigma = (2^9 pi^2 / 3) alpha (a0/z)^2 (I/E)^4 exp(-4 nu arccot nu)
 *           / (1 - exp(-2 pi nu)),   I = z^2 Ry,  nu = sqrt(I / (E - I)),
 * zero below the edge E = I. */
double or_sigma_k_electron(double e, double z)
{
    double i_k = z * z * OR_RY;
    if (!(e > i_k)) return 0.0;
    double nu = sqrt(i_k / (e - i_k));
    double r = i_k / e;
    double a = OR_A0 / z;
    return 512.0 * OR_PI * OR_PI / 3.0 * OR_ALPHA * a * a * r * r * r * r *
           exp(-4.0 * nu * atan(1.0 / nu)) / (-expm1(-2.0 * OR_PI * nu));
}

/* Binding energy of oxygen's K shell in the same hydrogenic model (MeV). */
double or_photo_binding(void) { return OR_Z_O_1S * OR_Z_O_1S * OR_RY; }

/* Photoelectric attenuation of water per unit density (cm^2/g): the two K
 * electrons of oxygen (hydrogen's and oxygen's outer shells neglected). */
double or_mu_photo(double e)
{
    return OR_MOL_PER_G * 2.0 * or_sigma_k_electron(e, OR_Z_O_1S);
}

/* Form factors of one hydrogenic electron, from the Fourier transform of its
 * charge density, in s = q a0 / z (q the momentum transfer in 1/cm):
 *   1s: 1 / (1 + s^2/4)^2,  2s: (1 - 3 s^2 + 2 s^4) / (1 + s^2)^4,
 *   2p (orientation averaged): (1 - s^2) / (1 + s^2)^4. */
static double ff_1s(double s) { double a = 1.0 + 0.25 * s * s; return 1.0 / (a * a); }
static double ff_2s(double s)
{
    double s2 = s * s, d = 1.0 + s2, d2 = d * d;
    return (1.0 - 3.0 * s2 + 2.0 * s2 * s2) / (d2 * d2);
}
static double ff_2p(double s)
{
    double s2 = s * s, d = 1.0 + s2, d2 = d * d;
    return (1.0 - s2) / (d2 * d2);
}

/* Squared form factor of a water molecule as independent atoms (interference
 * between the atoms neglected) at t = (q a0)^2: two hydrogen 1s electrons
 * (z = 1) and oxygen 1s^2 2s^2 2p^4 with the screened charges above.
 * F^2(0) = 1 + 1 + 8^2 = 66. */
double or_ff2_water(double t)
{
    double q = sqrt(t);
    double fh = ff_1s(q);
    double fo = 2.0 * ff_1s(q / OR_Z_O_1S) + 2.0 * ff_2s(q / OR_Z_O_2) + 4.0 * ff_2p(q / OR_Z_O_2);
    return 2.0 * fh * fh + fo * fo;
}

/* Cumulative A(t) = integral_0^t F^2(t') dt' on panels whose ends are spaced
 * logarithmically (8-point Gauss-Legendre per panel); A(t) between the ends
 * by the same rule over the partial panel. */
#define OR_FF_N 4000
#define OR_FF_TLO 1e-6
#define OR_FF_THI 1e10
static double ff_t[OR_FF_N + 1], ff_a[OR_FF_N + 1];
static int ff_ready = 0;

static double gl_ff2(double a, double b)
{
    double m = 0.5 * (a + b), h = 0.5 * (b - a), s = 0.0;
    for (int i = 0; i < 8; ++i) s += gl_w[i] * or_ff2_water(m + h * gl_x[i]);
    return h * s;
}

static void ff_init(void)
{
    if (ff_ready) return;
    gl_init();
    ff_t[0] = 0.0;
    ff_a[0] = 0.0;
    double r = pow(OR_FF_THI / OR_FF_TLO, 1.0 / (OR_FF_N - 1));
    for (int i = 1; i <= OR_FF_N; ++i) {
        ff_t[i] = OR_FF_TLO * pow(r, i - 1);
        ff_a[i] = ff_a[i - 1] + gl_ff2(ff_t[i - 1], ff_t[i]);
    }
    ff_ready = 1;
}

/* index i of the panel [t_i, t_i+1] holding t (t < t_N) */
static int ff_panel(double t)
{
    int lo = 0, hi = OR_FF_N;
    while (hi - lo > 1) {
        int mid = (lo + hi) / 2;
        if (ff_t[mid] <= t) lo = mid; else hi = mid;
    }
    return lo;
}

double or_ff2_cumulative(double t)
{
    ff_init();
    if (t >= ff_t[OR_FF_N]) t = ff_t[OR_FF_N];
    int i = ff_panel(t);
    return ff_a[i] + gl_ff2(ff_t[i], t);
}

/* The t with A(t) = a, for 0 <= a <= A(t_N): the panel by bisection on the
 * cumulative, then bisection on t inside it. */
static double ff_invert(double a)
{
    int lo = 0, hi = OR_FF_N;
    while (hi - lo > 1) {
        int mid = (lo + hi) / 2;
        if (ff_a[mid] <= a) lo = mid; else hi = mid;
    }
    double tl = ff_t[lo], th = ff_t[hi];
    for (int it = 0; it < 200 && th - tl > 1e-15 * th; ++it) {
        double tm = 0.5 * (tl + th);
        if (ff_a[lo] + gl_ff2(ff_t[lo], tm) <= a) tl = tm; else th = tm;
    }
    return 0.5 * (tl + th);
}

/* k a0 for a photon of energy e (MeV): (q a0)^2 ranges over [0, 4 (k a0)^2]. */
static double ka0_of(double e) { return e * OR_A0 / OR_HBARC; }

/* Rayleigh cross-section of a water molecule (cm^2): the Thomson differential
 * cross-section (r_e^2/2)(1 + cos^2 theta) times F^2, with
 * cos theta = 1 - t / (2 x^2), x = k a0, integrated over the sphere:
 *   sigma = pi r_e^2 / (2 x^2) * integral_0^{4x^2} (1 + cos^2 theta) F^2(t) dt. */
double or_sigma_rayleigh(double e)
{
    ff_init();
    double x = ka0_of(e), x2 = x * x, tm = 4.0 * x2;
    double sum = 0.0;
    for (int i = 0; i < OR_FF_N && ff_t[i] < tm; ++i) {
        double a = ff_t[i], b = ff_t[i + 1] < tm ? ff_t[i + 1] : tm;
        double m = 0.5 * (a + b), h = 0.5 * (b - a), s = 0.0;
        for (int j = 0; j < 8; ++j) {
            double t = m + h * gl_x[j], c = 1.0 - t / (2.0 * x2);
            s += gl_w[j] * (1.0 + c * c) * or_ff2_water(t);
        }
        sum += h * s;
    }
    return OR_PI * OR_RE * OR_RE / (2.0 * x2) * sum;
}

double or_mu_rayleigh(double e) { return OR_MOL_PER_G * or_sigma_rayleigh(e); }

/* Rayleigh polar angle: t drawn from F^2 on [0, 4x^2] by inverting the
 * cumulative (one uniform), accepted with (1 + cos^2 theta)/2 (one uniform),
 * repeated until accepted.  Returns cos theta. */
static double rayleigh_sample(or_stream* st, double e)
{
    ff_init();
    double x = ka0_of(e), x2 = x * x;
    double amax = or_ff2_cumulative(4.0 * x2);
    for (;;) {
        double u1 = stream_u01(st), u2 = stream_u01(st);
        double t = ff_invert(u1 * amax);
        double c = 1.0 - t / (2.0 * x2);
        if (c < -1.0) c = -1.0;
        if (u2 <= 0.5 * (1.0 + c * c)) return c;
    }
}

/* test hook: n Rayleigh scattering cosines at energy e (stream g = i) */
void or_rayleigh_sample_cos(double e, uint64_t seed, int n, double* cos_out)
{
    for (int i = 0; i < n; ++i) {
        or_stream st;
        stream_init(&st, seed, (uint64_t)i, OR_TAG_TR, 0);
        cos_out[i] = rayleigh_sample(&st, e);
    }
}

/* Pair production in the field of a nucleus, unscreened Bethe-Heitler, per
 * unit Z^2 (cm^2), in Maximon's expansions (k = E / mc^2):
 *   2 < k < 4:  (2 pi/3) alpha r_e^2 ((k-2)/k)^3 (1 + e/2 + 23e^2/40 + 11e^3/60
 *               + 29e^4/960),  e = (2k - 4)/(2 + k + 2 sqrt(2k));
 *   k >= 4:     alpha r_e^2 [28/9 L - 218/27 + (2/k)^2 (6L - 7/2 + 2/3 L^3 - L^2
 *               - pi^2/3 L + 2 zeta(3) + pi^2/6) - (2/k)^4 (3/16 L + 1/8)
 *               - (2/k)^6 (29/(9*256) L - 77/(27*512))],  L = ln 2k. */
double or_sigma_pair_z2(double e)
{
    double k = e / OR_ME;
    if (!(k > 2.0)) return 0.0;
    double ar2 = OR_ALPHA * OR_RE * OR_RE;
    if (k < 4.0) {
        double ep = (2.0 * k - 4.0) / (2.0 + k + 2.0 * sqrt(2.0 * k));
        double r = (k - 2.0) / k;
        return 2.0 * OR_PI / 3.0 * ar2 * r * r * r *
               (1.0 + ep / 2.0 + 23.0 * ep * ep / 40.0 + 11.0 * ep * ep * ep / 60.0 +
                29.0 * ep * ep * ep * ep / 960.0);
    }
    double l = log(2.0 * k), q2 = (2.0 / k) * (2.0 / k);
    return ar2 * (28.0 / 9.0 * l - 218.0 / 27.0 +
                  q2 * (6.0 * l - 3.5 + 2.0 / 3.0 * l * l * l - l * l - OR_PI * OR_PI / 3.0 * l +
                        2.0 * OR_ZETA3 + OR_PI * OR_PI / 6.0) -
                  q2 * q2 * (3.0 / 16.0 * l + 0.125) -
                  q2 * q2 * q2 * (29.0 / (9.0 * 256.0) * l - 77.0 / (27.0 * 512.0)));
}

/* Pair attenuation of water per unit density (cm^2/g): sum of Z^2 over the
 * molecule's nuclei, 1 + 1 + 64 = 66 (production on the electrons neglected). */
double or_mu_pair(double e) { return OR_MOL_PER_G * 66.0 * or_sigma_pair_z2(e); }

/* Fraction eps of the pair's kinetic energy E - 2mc^2 that the electron takes:
 * density proportional to eps^2 + (1-eps)^2 + (2/3) eps (1-eps) = 1 - (4/3)
 * eps (1-eps) on [0, 1] (the Bethe-Heitler sharing without its logarithmic
 * factor), by rejection from the uniform (two uniforms a trial). */
static double pair_share_sample(or_stream* st)
{
    for (;;) {
        double u1 = stream_u01(st), u2 = stream_u01(st);
        if (u2 <= 1.0 - 4.0 / 3.0 * u1 * (1.0 - u1)) return u1;
    }
}

/* test hook: n pair energy shares (stream g = i) */
void or_pair_share_sample(uint64_t seed, int n, double* out)
{
    for (int i = 0; i < n; ++i) {
        or_stream st;
        stream_init(&st, seed, (uint64_t)i, OR_TAG_TR, 0);
        out[i] = pair_share_sample(&st);
    }
}

/* Attenuation of water per unit density (cm^2/g) of the enabled processes;
 * parts[4] (nullable) receives Compton, photoelectric, Rayleigh, pair. */
double or_mu_total(double e, int32_t physics, double parts[4])
{
    double mc = ne_water() * or_kn_sigma(e);
    double mp = (physics & OR_PHYS_PHOTO) ? or_mu_photo(e) : 0.0;
    double mr = (physics & OR_PHYS_RAYLEIGH) ? or_mu_rayleigh(e) : 0.0;
    double mx = (physics & OR_PHYS_PAIR) ? or_mu_pair(e) : 0.0;
    if (parts) { parts[0] = mc; parts[1] = mp; parts[2] = mr; parts[3] = mx; }
    return mc + mp + mr + mx;
}

/* ------------------------------------------------------------------------ */
/* Electron physics: Bethe collision stopping power (ICRU 37 form, optionally */
/* with the density-effect correction), CSDA range and its inverse, Highland  */
/* multiple-scattering width.                                                 */
/* ------------------------------------------------------------------------ */

/* Density-effect correction delta(T) of liquid water in Sternheimer's
 * parametrisation (Sternheimer, Berger and Seltzer 1984, I = 75 eV), with
 * x = log10(beta gamma) = log10(p / m c):
 *   0                                   for x < x0 (an insulator: delta0 = 0),
 *   2 ln(10) x - Cbar + a (x1 - x)^m     for x0 <= x < x1,
 *   2 ln(10) x - Cbar                   for x >= x1.
 * Cbar = 2 ln(I / hbar omega_p) + 1 with the plasma energy of water. */
#define OR_DE_CBAR 3.5017
#define OR_DE_X0 0.2400
#define OR_DE_X1 2.8004
#define OR_DE_A 0.09116
#define OR_DE_M 3.4773
double or_density_delta(double t)
{
    double tau = t / OR_ME;
    double x = log10(sqrt(tau * (tau + 2.0)));
    if (x < OR_DE_X0) return 0.0;
    double d = 2.0 * log(10.0) * x - OR_DE_CBAR;
    if (x < OR_DE_X1) d += OR_DE_A * pow(OR_DE_X1 - x, OR_DE_M);
    return d;
}

/* Mass collision stopping power of water for electrons, MeV cm^2 / g; the
 * Bethe bracket less delta(T) when dens is set. */
double or_s_col_d(double t, int dens)
{
    double tau = t / OR_ME;
    double gam = tau + 1.0;
    double beta2 = 1.0 - 1.0 / (gam * gam);
    double i_rel = OR_I_WATER / OR_ME;
    double f_minus = 1.0 - beta2 + (tau * tau / 8.0 - (2.0 * tau + 1.0) * log(2.0)) / (gam * gam);
    double bracket = log(tau * tau * (tau + 2.0) / (2.0 * i_rel * i_rel)) + f_minus;
    if (dens) bracket -= or_density_delta(t);
    return 2.0 * OR_PI * OR_RE * OR_RE * OR_ME * OR_NA * OR_ZA_WATER / beta2 * bracket;
}
double or_s_col(double t) { return or_s_col_d(t, 0); }

/* Range nodes: T_k log-spaced from t_cut upwards, C_k = int_{t_cut}^{T_k} dT/S. */
#define OR_RNG_N 4000
#define OR_RNG_TMAX 30.0
/* The continuous stopping power S of the range tables: the collision stopping
 * power (restricted to transfers below the electron cut-off tc when delta
 * rays are on) plus, with bremsstrahlung on, the radiative loss to photons
 * below the photon cut-off kc (`soft`, at the nodes; linear in ln T between
 * them: it is below 1e-3 of S at these cut-offs). */
typedef struct {
    double t_cut, ratio, kc;
    int dens, phys;
    double t[OR_RNG_N], c[OR_RNG_N], soft[OR_RNG_N];
} or_range_table;

double or_s_col_restricted(double t, double tc, int dens);
double or_brem_soft(double t, double kc);

static double rt_soft(const or_range_table* rt, double t)
{
    double x = log(t / rt->t_cut) / log(rt->ratio);
    if (x <= 0.0) return rt->soft[0];
    if (x >= OR_RNG_N - 1) return rt->soft[OR_RNG_N - 1];
    int k = (int)x;
    double f = x - k;
    return (1.0 - f) * rt->soft[k] + f * rt->soft[k + 1];
}

static double rt_stop(const or_range_table* rt, double t)
{
    double s = (rt->phys & 8) ? or_s_col_restricted(t, rt->t_cut, rt->dens)
                              : or_s_col_d(t, rt->dens);
    if (rt->phys & 16) s += rt_soft(rt, t);
    return s;
}

static double gl_panel_inv_s(const or_range_table* rt, double a, double b)
{
    double c = 0.5 * (a + b), h = 0.5 * (b - a), s = 0.0;
    for (int i = 0; i < OR_GL_N; ++i) s += gl_w[i] / rt_stop(rt, c + h * gl_x[i]);
    return s * h;
}

/* Kinetic energy at which log10(beta gamma) = x. */
static double t_of_x(double x)
{
    double bg = pow(10.0, x);
    return OR_ME * (sqrt(1.0 + bg * bg) - 1.0);
}

/* int_a^b dT / S(T); with the density effect the integrand has kinks where
 * delta(T) changes branch (x0, x1), so panels are split there. */
static double gl_integral_inv_s(const or_range_table* rt, double a, double b)
{
    if (rt->dens) {
        const double knots[2] = {t_of_x(OR_DE_X0), t_of_x(OR_DE_X1)};
        for (int k = 0; k < 2; ++k)
            if (a < knots[k] && knots[k] < b)
                return gl_integral_inv_s(rt, a, knots[k]) + gl_integral_inv_s(rt, knots[k], b);
    }
    return gl_panel_inv_s(rt, a, b);
}

/* phys: the OR_PHYS_* bits (only delta rays and bremsstrahlung matter here);
 * kc: the photon cut-off. */
static void range_table_init(or_range_table* rt, double t_cut, int dens, int phys, double kc)
{
    gl_init();
    rt->t_cut = t_cut;
    rt->dens = dens;
    rt->phys = phys & (8 | 16);
    rt->kc = kc;
    rt->ratio = pow(OR_RNG_TMAX / t_cut, 1.0 / (OR_RNG_N - 1));
    for (int k = 0; k < OR_RNG_N; ++k) {
        rt->t[k] = t_cut * pow(rt->ratio, (double)k);
        rt->soft[k] = (rt->phys & 16) ? or_brem_soft(rt->t[k], kc) : 0.0;
    }
    rt->c[0] = 0.0;
    for (int k = 1; k < OR_RNG_N; ++k)
        rt->c[k] = rt->c[k - 1] + gl_integral_inv_s(rt, rt->t[k - 1], rt->t[k]);
}

/* CSDA range above the cut-off: R(T) = int_{t_cut}^{T} dT'/S(T') (g/cm^2). */
static double range_of(const or_range_table* rt, double t)
{
    if (t <= rt->t_cut) return 0.0;
    int k = (int)floor(log(t / rt->t_cut) / log(rt->ratio));
    if (k < 0) k = 0;
    if (k > OR_RNG_N - 1) k = OR_RNG_N - 1;
    while (k > 0 && rt->t[k] > t) --k;
    while (k < OR_RNG_N - 1 && rt->t[k + 1] <= t) ++k;
    return rt->c[k] + gl_integral_inv_s(rt, rt->t[k], t);
}

/* Inverse of range_of by bracketing on the nodes, then safeguarded Newton. */
static double range_inverse(const or_range_table* rt, double rr)
{
    if (rr <= 0.0) return rt->t_cut;
    int lo = 0, hi = OR_RNG_N - 1;
    if (rr >= rt->c[hi]) return rt->t[hi];
    while (hi - lo > 1) {
        int mid = (lo + hi) / 2;
        if (rt->c[mid] <= rr) lo = mid; else hi = mid;
    }
    double a = rt->t[lo], b = rt->t[hi];
    double t = a + (b - a) * (rr - rt->c[lo]) / (rt->c[hi] - rt->c[lo]);
    for (int it = 0; it < 60; ++it) {
        double f = rt->c[lo] + gl_integral_inv_s(rt, rt->t[lo], t) - rr;
        if (f > 0.0) b = t; else a = t;
        double tn = t - f * rt_stop(rt, t);
        if (!(tn > a && tn < b)) tn = 0.5 * (a + b);
        if (fabs(tn - t) <= 1e-15 * t) { t = tn; break; }
        t = tn;
    }
    return t;
}

/* test hooks */
static or_range_table g_test_rt;
static double g_test_rt_cut = -1.0, g_test_rt_kc = -1.0;
static int g_test_rt_dens = -1, g_test_rt_phys = -1;
static void ensure_test_rt(double t_cut, int dens, int phys, double kc)
{
    phys &= 8 | 16;
    if (g_test_rt_cut != t_cut || g_test_rt_dens != dens || g_test_rt_phys != phys ||
        g_test_rt_kc != kc) {
        range_table_init(&g_test_rt, t_cut, dens, phys, kc);
        g_test_rt_cut = t_cut;
        g_test_rt_dens = dens;
        g_test_rt_phys = phys;
        g_test_rt_kc = kc;
    }
}
double or_range_p(double t, double t_cut, int dens, int phys, double kc)
{
    ensure_test_rt(t_cut, dens, phys, kc);
    return range_of(&g_test_rt, t);
}
double or_range_inv_p(double rr, double t_cut, int dens, int phys, double kc)
{
    ensure_test_rt(t_cut, dens, phys, kc);
    return range_inverse(&g_test_rt, rr);
}
/* the continuous stopping power the range tables integrate (MeV cm^2/g) */
double or_s_cont(double t, double t_cut, int dens, int phys, double kc)
{
    ensure_test_rt(t_cut, dens, phys, kc);
    return rt_stop(&g_test_rt, t);
}
double or_range_d(double t, double t_cut, int dens) { return or_range_p(t, t_cut, dens, 0, 0.0); }
double or_range_inv_d(double rr, double t_cut, int dens)
{
    return or_range_inv_p(rr, t_cut, dens, 0, 0.0);
}
double or_range(double t, double t_cut) { return or_range_d(t, t_cut, 0); }
double or_range_inv(double rr, double t_cut) { return or_range_inv_d(rr, t_cut, 0); }

/* Highland width (PDG) of the projected multiple-scattering angle for an
 * electron of kinetic energy t over t_x radiation lengths; 0 where the
 * logarithmic correction turns it negative. */
double or_highland(double t, double t_x)
{
    if (!(t_x > 0.0)) return 0.0;
    double betacp = t * (t + 2.0 * OR_ME) / (t + OR_ME);
    double th = 13.6 / betacp * sqrt(t_x) * (1.0 + 0.038 * log(t_x));
    return th > 0.0 ? th : 0.0;
}

/* Multiple-scattering width of one electron step: the Highland width at the
 * step's mean kinetic energy t_mid for a path of s cm in water-like medium of
 * density rho (thickness rho s / X0 radiation lengths). */
double or_ms_width(double t_mid, double rho, double s)
{
    return or_highland(t_mid, rho * s / OR_X0_WATER);
}

/* Polar deflection for projected-angle width theta0: |theta| of a 2D Gaussian,
 * theta = theta0 sqrt(-2 ln(1-u)), capped at pi. */
static double ms_polar(double theta0, double u)
{
    double th = theta0 * sqrt(-2.0 * log(1.0 - u));
    return th < OR_PI ? th : OR_PI;
}

/* test hook: n polar deflections for width theta0 (stream g = i) */
void or_ms_sample(double theta0, uint64_t seed, int n, double* theta_out)
{
    for (int i = 0; i < n; ++i) {
        or_stream st;
        stream_init(&st, seed, (uint64_t)i, OR_TAG_TR, 0);
        double u = stream_u01(&st);
        theta_out[i] = ms_polar(theta0, u);
    }
}

/* ------------------------------------------------------------------------ */
/* Electron hard events, each switchable: Moller delta rays (energy transfers */
/* at or above the electron cut-off tc) and bremsstrahlung photons (at or     */
/* above the photon cut-off kc).  Below the cut-offs the losses stay           */
/* continuous: the collision stopping power restricted to transfers below tc  */
/* and the radiative loss to photons below kc.  The paper's engine has both   */
/* processes (Sec. 2.3 names its cut-offs only); the forms below are the      */
/* Moller cross-section and the Bethe-Heitler (Born, unscreened) photon       */
/* spectrum, formula 3BN of Koch and Motz (1959), with Z(Z+1) for the atomic  */
/* electrons' share.                                                          */
/* ------------------------------------------------------------------------ */
#define OR_ZZ1_WATER 76.0            /* sum of Z (Z + 1) over the atoms of H2O */
#define OR_MOL_G (1.0 / 18.0153)     /* mol of H2O per gram */

/* Electron density of water per gram (electrons / g). */
static double ne_per_gram(void) { return OR_NA * OR_ZA_WATER; }

/* Moller differential cross-section per target electron for an electron of
 * kinetic energy t transferring w (cm^2 / MeV), eps = w / t:
 *   2 pi re^2 mc^2 / (beta^2 t^2) [1/eps^2 + 1/(1-eps)^2 + (tau/(tau+1))^2
 *                                 - (2 tau + 1) / (tau+1)^2 / (eps (1-eps))]. */
double or_moller_dsig(double t, double w)
{
    double tau = t / OR_ME, gam = tau + 1.0, beta2 = 1.0 - 1.0 / (gam * gam);
    double eps = w / t;
    double a = tau / gam;
    double br = 1.0 / (eps * eps) + 1.0 / ((1.0 - eps) * (1.0 - eps)) + a * a -
                (2.0 * tau + 1.0) / (gam * gam) / (eps * (1.0 - eps));
    return 2.0 * OR_PI * OR_RE * OR_RE * OR_ME / (beta2 * t * t) * br;
}

/* Its integral over w in [tc, t/2] (the two electrons are identical: the
 * more energetic one is the primary), per gram of water (cm^2/g); 0 where
 * t <= 2 tc.  With ec = tc / t, the closed form of the bracket's integral
 * over eps in [ec, 1/2] is
 *   1/ec - 1/(1-ec) + (tau/(tau+1))^2 (1/2 - ec) - (2 tau+1)/(tau+1)^2 ln((1-ec)/ec). */
double or_moller_sigma(double t, double tc)
{
    if (!(t > 2.0 * tc)) return 0.0;
    double tau = t / OR_ME, gam = tau + 1.0, beta2 = 1.0 - 1.0 / (gam * gam);
    double ec = tc / t, a = tau / gam;
    double br = 1.0 / ec - 1.0 / (1.0 - ec) + a * a * (0.5 - ec) -
                (2.0 * tau + 1.0) / (gam * gam) * log((1.0 - ec) / ec);
    return ne_per_gram() * 2.0 * OR_PI * OR_RE * OR_RE * OR_ME / (beta2 * t) * br;
}

/* Collision stopping power of water restricted to energy transfers below tc
 * (ICRU 37, the Rohrlich-Carlson F-(tau, Delta) with Delta = tc / mc^2, at
 * most tau / 2 where it is the unrestricted one), MeV cm^2/g, less the
 * density-effect delta(T) when dens is set. */
double or_s_col_restricted(double t, double tc, int dens)
{
    double tau = t / OR_ME, gam = tau + 1.0, beta2 = 1.0 - 1.0 / (gam * gam);
    double dl = tc / OR_ME;
    if (dl > 0.5 * tau) dl = 0.5 * tau;
    double i_rel = OR_I_WATER / OR_ME;
    double f_minus = -1.0 - beta2 + log((tau - dl) * dl) + tau / (tau - dl) +
                     (0.5 * dl * dl + (2.0 * tau + 1.0) * log(1.0 - dl / tau)) / (gam * gam);
    double bracket = log(2.0 * (tau + 2.0) / (i_rel * i_rel)) + f_minus;
    if (dens) bracket -= or_density_delta(t);
    return 2.0 * OR_PI * OR_RE * OR_RE * OR_ME * OR_NA * OR_ZA_WATER / beta2 * bracket;
}

/* Bremsstrahlung: k dsigma/dk of an electron of kinetic energy t emitting a
 * photon of energy k in water, per gram (cm^2/g), from formula 3BN (energies
 * in units of mc^2: E0 = 1 + t, E = E0 - k, p the momenta):
 *   Z^2 alpha re^2 (p/p0) { 4/3 - 2 E0 E (p^2 + p0^2)/(p^2 p0^2) + e0 E/p0^3
 *     + e E0/p^3 - e e0/(p0 p) + L [8 E0 E/(3 p0 p) + k^2 (E0^2 E^2 + p0^2 p^2)/(p0^3 p^3)
 *     + k/(2 p0 p) (e0 (E0 E + p0^2)/p0^3 - e (E0 E + p^2)/p^3 + 2 k E0 E/(p^2 p0^2))] }
 * with L = 2 ln((E0 E + p0 p - 1)/k), e0 = ln((E0+p0)/(E0-p0)), e = ln((E+p)/(E-p)),
 * and Z^2 -> sum of Z(Z+1) over the molecule.  0 at and beyond the tip. */
double or_brem_kdsig(double t, double k_mev)
{
    double e0t = 1.0 + t / OR_ME, k = k_mev / OR_ME, et = e0t - k;
    if (!(k > 0.0) || !(et > 1.0)) return 0.0;
    double p0 = sqrt(e0t * e0t - 1.0), p = sqrt(et * et - 1.0);
    double L = 2.0 * log((e0t * et + p0 * p - 1.0) / k);
    double eps0 = log((e0t + p0) / (e0t - p0)), eps = log((et + p) / (et - p));
    double p02 = p0 * p0, p2 = p * p, p03 = p02 * p0, p3 = p2 * p;
    double br = 4.0 / 3.0 - 2.0 * e0t * et * (p2 + p02) / (p2 * p02) + eps0 * et / p03 +
                eps * e0t / p3 - eps * eps0 / (p0 * p) +
                L * (8.0 * e0t * et / (3.0 * p0 * p) +
                     k * k * (e0t * e0t * et * et + p02 * p2) / (p03 * p3) +
                     k / (2.0 * p0 * p) *
                         (eps0 * (e0t * et + p02) / p03 - eps * (e0t * et + p2) / p3 +
                          2.0 * k * e0t * et / (p2 * p02)));
    double v = (p / p0) * br;
    if (v < 0.0) v = 0.0;
    return OR_ZZ1_WATER * OR_ALPHA * OR_RE * OR_RE * OR_NA * OR_MOL_G * v;
}

/* Integrals over ln k by 8-point Gauss-Legendre on n equal panels of [a, b]
 * (ln k); `weight_k` multiplies the integrand by k (energy moment). */
static double brem_int_lnk(double t, double lna, double lnb, int n, int weight_k)
{
    gl_init();
    double h = (lnb - lna) / n, s = 0.0;
    for (int i = 0; i < n; ++i) {
        double c = lna + (i + 0.5) * h;
        for (int j = 0; j < OR_GL_N; ++j) {
            double k = exp(c + 0.5 * h * gl_x[j]);
            s += gl_w[j] * or_brem_kdsig(t, k) * (weight_k ? k : 1.0);
        }
    }
    return 0.5 * h * s;
}

/* Photons of kc <= k < t, per gram (cm^2/g): the integral of k dsigma/dk
 * over ln k. */
double or_brem_sigma(double t, double kc)
{
    if (!(t > kc)) return 0.0;
    return brem_int_lnk(t, log(kc), log(t), 64, 0);
}

/* Energy radiated in photons below min(kc, t), per gram (MeV cm^2/g): the
 * integral of k dsigma/dk over k, on ln k from 1e-12 kc (the rest is below
 * 1e-10 of it). */
double or_brem_soft(double t, double kc)
{
    double top = kc < t ? kc : t;
    if (!(top > 0.0)) return 0.0;
    return brem_int_lnk(t, log(top * 1e-12), log(top), 96, 1);
}

/* Energy transfer of a hard Moller collision (t > 2 tc): eps = w / t from
 * 1/eps^2 on [ec, 1/2] by inversion, eps = ec / (1 - u (1 - 2 ec)), kept with
 * probability h(eps) / 2.25 where the differential cross-section is
 * h(eps) / eps^2 up to a constant,
 *   h = 1 + (eps/(1-eps))^2 + (tau/(tau+1))^2 eps^2 - (2 tau+1)/(tau+1)^2 eps/(1-eps),
 * and h <= 2.25 on [0, 1/2].  Two uniforms a trial, at most 1000 trials. */
static double moller_sample(or_stream* st, double t, double tc)
{
    double tau = t / OR_ME, gam = tau + 1.0, a = tau / gam;
    double c2 = (2.0 * tau + 1.0) / (gam * gam);
    double ec = tc / t, eps = ec;
    for (int trial = 0; trial < 1000; ++trial) {
        double u1 = stream_u01(st), u2 = stream_u01(st);
        eps = ec / (1.0 - u1 * (1.0 - 2.0 * ec));
        double r = eps / (1.0 - eps);
        double h = 1.0 + r * r + a * a * eps * eps - c2 * r;
        if (u2 * 2.25 <= h) break;
    }
    return eps;
}

/* Photon energy of a hard bremsstrahlung event (kc < t): k = kc (t/kc)^u
 * (density 1/k), kept with probability k dsigma/dk (t, k) / k dsigma/dk (t,
 * kc); k dsigma/dk decreases with k on (0, t) (checked in the tests), so the
 * bound holds.  Two uniforms a trial, at most 1000 trials. */
static double brem_sample(or_stream* st, double t, double kc)
{
    double top = or_brem_kdsig(t, kc), lr = log(t / kc), k = kc;
    for (int trial = 0; trial < 1000; ++trial) {
        double u1 = stream_u01(st), u2 = stream_u01(st);
        k = kc * exp(u1 * lr);
        if (u2 * top <= or_brem_kdsig(t, k)) break;
    }
    return k;
}

/* test hooks: samples on streams g = i */
void or_moller_sample(double t, double tc, uint64_t seed, int n, double* eps_out)
{
    for (int i = 0; i < n; ++i) {
        or_stream st;
        stream_init(&st, seed, (uint64_t)i, OR_TAG_TR, 0);
        eps_out[i] = moller_sample(&st, t, tc);
    }
}
void or_brem_sample(double t, double kc, uint64_t seed, int n, double* k_out)
{
    for (int i = 0; i < n; ++i) {
        or_stream st;
        stream_init(&st, seed, (uint64_t)i, OR_TAG_TR, 0);
        k_out[i] = brem_sample(&st, t, kc);
    }
}

/* Random-number stream of a secondary made in a hard event or by a positron
 * of a secondary family: the splitmix64 finaliser (Steele, Lea and Flood,
 * OOPSLA 2014) of the parent's stream (g, sub), the parent's event index j
 * and the kind (1 delta electron, 2 bremsstrahlung photon, 3 annihilation
 * photon); the child keeps the history id (low 48 bits of g), takes
 * 0x8000 | 15 hashed bits as the high 16 bits (disjoint from the annihilation
 * photons' 2 sub + k of a source photon's family) and 8 hashed bits as its
 * sub (electrons; photons take sub 0). */
static uint64_t mix64(uint64_t z)
{
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
void or_child_id(uint64_t g, uint32_t sub, uint32_t j, uint32_t kind, uint64_t* g_out,
                 uint32_t* sub_out)
{
    uint64_t h = mix64(mix64(g) ^ (((uint64_t)sub << 32) | ((uint64_t)j << 8) | (uint64_t)kind));
    *g_out = (g & 0xFFFFFFFFFFFFull) | ((uint64_t)(0x8000u | (uint32_t)(h & 0x7FFFu)) << 48);
    *sub_out = (uint32_t)(h >> 16) & 0xFFu;
}

/* Generations: source photons and source electrons are generation 0; the
 * electrons a photon sets in motion share its generation; delta electrons,
 * bremsstrahlung photons and annihilation photons are one above their
 * parent's.  A particle above OR_GEN_MAX is not followed: its energy (for
 * annihilation photons the 2 mc^2) is deposited where it was made (counted
 * as capped). */
#define OR_GEN_MAX 3

/* ------------------------------------------------------------------------ */
/* Transport and tally                                                        */
/* ------------------------------------------------------------------------ */
typedef struct {
    const or_phantom* ph;
    const or_params* tp;
    const or_range_table* rt;
    double rho_max;
    const int32_t* imap;       /* optional voxel -> row+1 */
    int64_t n_cols;            /* tally columns in index-map mode */
    double* grid;              /* this thread's energy array */
    double ledger[L_N];
    uint64_t cnt[C_N];
} or_tracker;

static void deposit(or_tracker* T, int64_t v, double e, int32_t tag)
{
    if (e == 0.0) return;
    T->ledger[L_DEP] += e;
    T->cnt[C_DEPOSITS]++;
    if (T->imap) {
        int32_t row = T->imap[v];
        if (row > 0) T->grid[(int64_t)(row - 1) * T->n_cols + tag] += e;
    } else {
        T->grid[v] += e;
    }
}

#define OR_MAX_E_STEPS 100000

/* Condensed-history electron (CSDA + Highland Gaussian deflections).
 * Steps end at voxel faces or after a fractional energy loss step_frac;
 * the voxel index is carried explicitly and changes by one at each face. */
static void transport_photon(or_tracker* T, double p[3], double d[3], double e,
                             uint64_t seed, uint64_t g, int32_t tag, int secondary, int gen);

/* A positron (generation gen) that has come to rest at p annihilates into
 * two photons of mc^2 each, back to back, the first along an isotropic
 * direction (cos theta = 2u - 1, phi = 2 pi u', two uniforms of the
 * positron's stream).  Each photon is followed as a photon history of its
 * own (generation gen + 1), id g | (2 sub + k) << 48 in a source photon's
 * family (the history ids of a plan stay below 2^48), else the child stream
 * of kind 3 with event index k.  Above the generation cap the 2 mc^2 are
 * deposited at p. */
static void annihilate(or_tracker* T, or_stream* st, const double p[3], uint64_t seed,
                       uint64_t g, uint32_t sub, int32_t tag, int gen, int64_t v)
{
    double c = 2.0 * stream_u01(st) - 1.0, phi = 2.0 * OR_PI * stream_u01(st);
    double sn = sqrt(1.0 - c * c);
    double da[3] = {sn * cos(phi), sn * sin(phi), c};
    T->cnt[C_ANNIHIL]++;
    if (gen + 1 > OR_GEN_MAX) {
        deposit(T, v, 2.0 * OR_ME, tag);
        T->cnt[C_CAPPED]++;
        return;
    }
    for (int k = 0; k < 2; ++k) {
        double pp[3] = {p[0], p[1], p[2]};
        double dd[3] = {k ? -da[0] : da[0], k ? -da[1] : da[1], k ? -da[2] : da[2]};
        uint64_t gk = g | ((uint64_t)(2u * sub + (uint32_t)k) << 48);
        if (g >> 48) {
            uint32_t unused;
            or_child_id(g, sub, (uint32_t)k, 3u, &gk, &unused);
        }
        transport_photon(T, pp, dd, OR_ME, seed, gk, tag, 1, gen + 1);
    }
}

/* A hard event of an electron (or positron) of kinetic energy *e at p,
 * direction d, in voxel v, stream st of (g, sub), generation gen, event index
 * j: the process in proportion to the Moller and bremsstrahlung
 * cross-sections at *e (one uniform; neither possible: no event).  Moller:
 * the delta electron takes w = eps *e, the directions from two-body
 * kinematics, cos = sqrt(w (t + 2 mc^2) / (t (w + 2 mc^2))) for the delta and
 * the same with t - w for the primary, azimuths phi and phi + pi (one more
 * uniform).  Bremsstrahlung: the photon takes k along d, the electron keeps
 * its direction.  The secondary (generation gen + 1) is followed at once, or
 * deposited at p above the generation cap. */
static void transport_electron(or_tracker* T, double p[3], double d[3], double e,
                               uint64_t seed, uint64_t g, uint32_t sub, int32_t tag, int positron,
                               int gen);
static void hard_event(or_tracker* T, or_stream* st, const double p[3], double d[3], double* e,
                       int64_t v, uint64_t seed, uint64_t g, uint32_t sub, int32_t tag, int gen,
                       uint32_t j)
{
    const int32_t phys = T->tp->physics;
    const double tc = T->tp->e_cut_e, kc = T->tp->e_cut_g;
    double sm = (phys & OR_PHYS_DELTA) ? or_moller_sigma(*e, tc) : 0.0;
    double sb = (phys & OR_PHYS_BREM) ? or_brem_sigma(*e, kc) : 0.0;
    double u = stream_u01(st);
    if (!(sm + sb > 0.0)) return;
    uint64_t gc;
    uint32_t subc;
    double pp[3] = {p[0], p[1], p[2]};
    if (u * (sm + sb) < sm) {
        double t = *e, eps = moller_sample(st, t, tc);
        double w = eps * t, t1 = t - w;
        double phi = 2.0 * OR_PI * stream_u01(st);
        double cd = sqrt(w * (t + 2.0 * OR_ME) / (t * (w + 2.0 * OR_ME)));
        double cp = sqrt(t1 * (t + 2.0 * OR_ME) / (t * (t1 + 2.0 * OR_ME)));
        double dd[3] = {d[0], d[1], d[2]};
        rotate_direction(dd, cd, phi);
        rotate_direction(d, cp, phi + OR_PI);
        *e = t1;
        T->cnt[C_MOLLER]++;
        if (gen + 1 > OR_GEN_MAX) {
            deposit(T, v, w, tag);
            T->cnt[C_CAPPED]++;
            return;
        }
        or_child_id(g, sub, j, 1u, &gc, &subc);
        transport_electron(T, pp, dd, w, seed, gc, subc, tag, 0, gen + 1);
    } else {
        double k = brem_sample(st, *e, kc);
        *e -= k;
        T->cnt[C_BREM]++;
        if (gen + 1 > OR_GEN_MAX) {
            deposit(T, v, k, tag);
            T->cnt[C_CAPPED]++;
            return;
        }
        or_child_id(g, sub, j, 2u, &gc, &subc);
        double dd[3] = {d[0], d[1], d[2]};
        transport_photon(T, pp, dd, k, seed, gc, tag, 1, gen + 1);
    }
}

/* With delta rays or bremsstrahlung on, the continuous loss is the
 * restricted one (range tables) and hard events come at a rate sigma_h =
 * sigma_Moller + sigma_brem per gram taken at the step's initial energy: the
 * number of mean free paths to the next one, -ln(1 - u), is drawn at the
 * start and after each event (one uniform), a step ends at the event if it
 * comes before the face and the energy-loss limit, and the event happens
 * after that step's continuous loss and deflection (hard_event). */
static void transport_electron(or_tracker* T, double p[3], double d[3], double e,
                               uint64_t seed, uint64_t g, uint32_t sub, int32_t tag, int positron,
                               int gen)
{
    const or_phantom* ph = T->ph;
    const double tcut = T->tp->e_cut_e, f = T->tp->step_frac;
    const int32_t phys = T->tp->physics;
    const int hard = (phys & (OR_PHYS_DELTA | OR_PHYS_BREM)) != 0;
    const int n[3] = {ph->nx, ph->ny, ph->nz};
    int idx[3];
    voxel_clamped(ph, p, idx);
    or_stream st;
    stream_init(&st, seed, g, OR_TAG_TR, sub);
    if (e < tcut) {
        int64_t v0 = ((int64_t)idx[2] * ph->ny + idx[1]) * ph->nx + idx[0];
        deposit(T, v0, e, tag);
        T->cnt[C_E_LOCAL]++;
        if (positron) annihilate(T, &st, p, seed, g, sub, tag, gen, v0);
        return;
    }
    double lam = hard ? -log(1.0 - stream_u01(&st)) : 0.0;
    uint32_t n_hard = 0;
    for (int step = 0;; ++step) {
        int64_t v = ((int64_t)idx[2] * ph->ny + idx[1]) * ph->nx + idx[0];
        if (step >= OR_MAX_E_STEPS) {
            deposit(T, v, e, tag);
            T->cnt[C_GUARD]++;
            if (positron) annihilate(T, &st, p, seed, g, sub, tag, gen, v);
            return;
        }
        double rho = (double)ph->density[v];
        /* distance to the exit face of the current voxel */
        double sb = OR_INF;
        int axis = -1;
        for (int a = 0; a < 3; ++a) {
            double face;
            if (d[a] > 0.0) face = ph->origin[a] + (double)(idx[a] + 1) * ph->vox[a];
            else if (d[a] < 0.0) face = ph->origin[a] + (double)idx[a] * ph->vox[a];
            else continue;
            double t = (face - p[a]) / d[a];
            if (t < sb) { sb = t; axis = a; }
        }
        if (sb < 0.0) sb = 0.0;
        /* energy-loss limited step */
        double r0 = range_of(T->rt, e);
        double e_f = e * (1.0 - f);
        int final = !(e_f > tcut);
        double sf;
        if (rho > 0.0) sf = (final ? r0 : r0 - range_of(T->rt, e_f)) / rho;
        else sf = OR_INF;
        T->cnt[C_E_STEPS]++;
        double sig_h = 0.0, sh = OR_INF;
        if (hard && rho > 0.0) {
            sig_h = ((phys & OR_PHYS_DELTA) ? or_moller_sigma(e, tcut) : 0.0) +
                    ((phys & OR_PHYS_BREM) ? or_brem_sigma(e, T->tp->e_cut_g) : 0.0);
            if (sig_h > 0.0) sh = lam / (rho * sig_h);
        }
        if (sh < sf && sh < sb) {
            /* a hard event ends this step */
            double e_new = range_inverse(T->rt, r0 - rho * sh);
            deposit(T, v, e - e_new, tag);
            for (int a = 0; a < 3; ++a) p[a] += sh * d[a];
            T->ledger[L_EPATH] += sh;
            double e_old = e;
            e = e_new;
            if (e < tcut) {
                deposit(T, v, e, tag);
                if (positron) annihilate(T, &st, p, seed, g, sub, tag, gen, v);
                return;
            }
            if (T->tp->ms_enable) {
                double th0 = or_ms_width(0.5 * (e_old + e), rho, sh);
                double u1 = stream_u01(&st), u2 = stream_u01(&st);
                rotate_direction(d, cos(ms_polar(th0, u1)), 2.0 * OR_PI * u2);
            }
            hard_event(T, &st, p, d, &e, v, seed, g, sub, tag, gen, n_hard++);
            if (e < tcut) {
                deposit(T, v, e, tag);
                if (positron) annihilate(T, &st, p, seed, g, sub, tag, gen, v);
                return;
            }
            lam = -log(1.0 - stream_u01(&st));
            continue;
        }
        lam -= rho * sig_h * (sf <= sb ? sf : sb);
        if (sf <= sb) {
            if (final) {
                /* the residual range ends inside this voxel */
                T->ledger[L_EPATH] += sf;
                deposit(T, v, e, tag);
                if (positron) annihilate(T, &st, p, seed, g, sub, tag, gen, v);
                return;
            }
            double e_new = range_inverse(T->rt, r0 - rho * sf);
            deposit(T, v, e - e_new, tag);
            for (int a = 0; a < 3; ++a) p[a] += sf * d[a];
            T->ledger[L_EPATH] += sf;
            double e_old = e;
            e = e_new;
            if (e < tcut) {
                deposit(T, v, e, tag);
                if (positron) annihilate(T, &st, p, seed, g, sub, tag, gen, v);
                return;
            }
            if (T->tp->ms_enable) {
                double th0 = or_ms_width(0.5 * (e_old + e), rho, sf);
                double u1 = stream_u01(&st), u2 = stream_u01(&st);
                rotate_direction(d, cos(ms_polar(th0, u1)), 2.0 * OR_PI * u2);
            }
        } else {
            double e_new = range_inverse(T->rt, r0 - rho * sb);
            deposit(T, v, e - e_new, tag);
            for (int a = 0; a < 3; ++a) p[a] += sb * d[a];
            T->ledger[L_EPATH] += sb;
            T->cnt[C_E_BOUNDARY]++;
            double e_old = e;
            e = e_new;
            idx[axis] += d[axis] > 0.0 ? 1 : -1;
            if (idx[axis] < 0 || idx[axis] >= n[axis]) {
                /* an escaping positron takes its rest energy (2 mc^2, the
                 * annihilation photons') out of the phantom as well */
                T->ledger[L_ESC_E] += e + (positron ? 2.0 * OR_ME : 0.0);
                return;
            }
            if (e < tcut) {
                int64_t v2 = ((int64_t)idx[2] * ph->ny + idx[1]) * ph->nx + idx[0];
                deposit(T, v2, e, tag);
                if (positron) annihilate(T, &st, p, seed, g, sub, tag, gen, v2);
                return;
            }
            if (T->tp->ms_enable) {
                double th0 = or_ms_width(0.5 * (e_old + e), rho, sb);
                double u1 = stream_u01(&st), u2 = stream_u01(&st);
                rotate_direction(d, cos(ms_polar(th0, u1)), 2.0 * OR_PI * u2);
            }
        }
    }
}

typedef struct { double p[3], d[3], e; uint32_t sub; int positron; } or_electron;

/* Woodcock (delta) tracking with the majorant mu_max(E) = rho_max mu(E), mu
 * the attenuation per unit density of the enabled processes; a tentative
 * collision is real with probability rho_voxel / rho_max.  Without the
 * optional processes mu = n_e sigma_KN.  With them a real collision picks its
 * process with one more uniform, in proportion to the processes' attenuations:
 *   Compton: Klein-Nishina (Kahn), the electron pushed at or above the
 *            electron cut-off, deposited on the spot below it;
 *   photoelectric: the photon is absorbed; the photoelectron (E minus the K
 *            binding energy, along the photon's direction) is pushed or
 *            deposited like a Compton electron, the binding energy is
 *            deposited on the spot;
 *   Rayleigh: the photon is deflected without losing energy;
 *   pair: the photon is absorbed; the electron takes eps (E - 2 mc^2) and the
 *            positron the rest, both along the photon's direction; the
 *            electron is pushed or deposited like a Compton electron, the
 *            positron is always pushed (it annihilates where it stops).
 * Pushed particles take sub-ids 1, 2, ... in the order they are created.  The
 * photon is absorbed locally below its cut-off.  Escapes without a real
 * collision are counted for source photons only (not `secondary` ones, the
 * annihilation photons). */
static void transport_photon(or_tracker* T, double p[3], double d[3], double e,
                             uint64_t seed, uint64_t g, int32_t tag, int secondary, int gen)
{
    const or_phantom* ph = T->ph;
    const int32_t phys = T->tp->physics;
    const double ecut = T->tp->e_cut_e;
    or_stream st;
    stream_init(&st, seed, g, OR_TAG_TR, 0);
    or_electron stack[256];
    int n_e = 0;
    uint32_t n_push = 0;
    int collided = secondary;
    const double ne = ne_water();
    for (;;) {
        double parts[4];
        double mu_max = phys ? T->rho_max * or_mu_total(e, phys, parts)
                             : ne * T->rho_max * or_kn_sigma(e);
        double s = -log(1.0 - stream_u01(&st)) / mu_max;
        for (int a = 0; a < 3; ++a) p[a] += s * d[a];
        int idx[3];
        int64_t v = voxel_of(ph, p, idx);
        if (v < 0) {
            T->ledger[L_ESC_G] += e;
            if (!collided) T->cnt[C_ESC_UNCOLLIDED]++;
            break;
        }
        T->cnt[C_WC_STEPS]++;
        double ur = stream_u01(&st);
        if (!(ur < (double)ph->density[v] / T->rho_max)) continue;
        collided = 1;
        T->cnt[C_REAL]++;
        int process = 0;   /* 0 Compton, 1 photoelectric, 2 Rayleigh, 3 pair */
        if (phys) {
            double up = stream_u01(&st) * (parts[0] + parts[1] + parts[2] + parts[3]);
            double acc = parts[0];
            if (up >= acc) { process = 1; acc += parts[1]; }
            if (process == 1 && up >= acc) { process = 2; acc += parts[2]; }
            if (process == 2 && up >= acc) process = 3;
        }
        if (process == 1) {
            /* photoelectric absorption */
            double b = or_photo_binding();
            double te = e - b;
            T->cnt[C_PHOTO]++;
            if (te >= ecut) {
                or_electron* el = &stack[n_e++];
                for (int a = 0; a < 3; ++a) { el->p[a] = p[a]; el->d[a] = d[a]; }
                el->e = te;
                el->sub = 1 + n_push++;
                el->positron = 0;
                T->cnt[C_E_PUSHED]++;
                deposit(T, v, b, tag);
            } else {
                deposit(T, v, e, tag);
                T->cnt[C_E_LOCAL]++;
            }
            break;
        }
        if (process == 2) {
            /* Rayleigh: deflection only */
            double c = rayleigh_sample(&st, e);
            double phi = 2.0 * OR_PI * stream_u01(&st);
            rotate_direction(d, c, phi);
            T->cnt[C_RAYLEIGH]++;
            continue;
        }
        if (process == 3) {
            /* pair production */
            double eps = pair_share_sample(&st);
            double kin = e - 2.0 * OR_ME;
            double tm = eps * kin, tp = kin - tm;
            T->cnt[C_PAIR]++;
            if (tm >= ecut) {
                or_electron* el = &stack[n_e++];
                for (int a = 0; a < 3; ++a) { el->p[a] = p[a]; el->d[a] = d[a]; }
                el->e = tm;
                el->sub = 1 + n_push++;
                el->positron = 0;
                T->cnt[C_E_PUSHED]++;
            } else {
                deposit(T, v, tm, tag);
                T->cnt[C_E_LOCAL]++;
            }
            or_electron* po = &stack[n_e++];
            for (int a = 0; a < 3; ++a) { po->p[a] = p[a]; po->d[a] = d[a]; }
            po->e = tp;
            po->sub = 1 + n_push++;
            po->positron = 1;
            T->cnt[C_E_PUSHED]++;
            break;
        }
        double k = e / OR_ME;
        double x = kahn_sample(&st, k, &T->cnt[C_KAHN_TRIALS]);
        double phi = 2.0 * OR_PI * stream_u01(&st);
        double e1, te, d1[3], de[3];
        compton_kinematics(e, d, x, phi, &e1, d1, &te, de);
        if (te >= ecut) {
            or_electron* el = &stack[n_e++];
            for (int a = 0; a < 3; ++a) { el->p[a] = p[a]; el->d[a] = de[a]; }
            el->e = te;
            el->sub = 1 + n_push++;
            el->positron = 0;
            T->cnt[C_E_PUSHED]++;
        } else {
            deposit(T, v, te, tag);
            T->cnt[C_E_LOCAL]++;
        }
        e = e1;
        for (int a = 0; a < 3; ++a) d[a] = d1[a];
        if (e < T->tp->e_cut_g) { deposit(T, v, e, tag); break; }
        if (n_e >= 254) break;   /* cannot happen: at most E/e_cut_e + 1 pushes, < 256 */
    }
    for (int i = 0; i < n_e; ++i)
        transport_electron(T, stack[i].p, stack[i].d, stack[i].e, seed, g, stack[i].sub, tag,
                           stack[i].positron, gen);
}

static double phantom_rho_max(const or_phantom* ph)
{
    size_t n = (size_t)ph->nx * ph->ny * ph->nz;
    double m = 0.0;
    for (size_t i = 0; i < n; ++i) if (ph->density[i] > m) m = ph->density[i];
    return m;
}

static void tracker_init(or_tracker* T, const or_phantom* ph, const or_params* tp,
                         const or_range_table* rt, double rho_max, const int32_t* imap,
                         int64_t n_cols, double* grid)
{
    memset(T, 0, sizeof(*T));
    T->ph = ph; T->tp = tp; T->rt = rt; T->rho_max = rho_max;
    T->imap = imap; T->n_cols = n_cols; T->grid = grid;
}

#define OR_MAX_THREADS 64
static int n_threads_of(int req)
{
#ifdef _OPENMP
    int nt = req > 0 ? req : omp_get_max_threads();
    return nt < OR_MAX_THREADS ? nt : OR_MAX_THREADS;
#else
    (void)req;
    return 1;
#endif
}

/* Samples histories g = r*N + h for r in [rep0, rep0+n_rep), h = h0, h0 + stride,
 * ... < h1, and transports them.  Energy per replica is accumulated in FP64; sum/sum2 receive
 * the sum over replicas of E_r and E_r^2 per tally cell (V voxels, or
 * n_rows * n_cols cells in index-map mode).  ledger[8], counters[16]. */
int or_run(const or_model* m, const or_plan* plan, const or_beam* beams, int n_beams,
           const or_phantom* ph, const or_params* tp, uint64_t seed, uint32_t rep0,
           uint32_t n_rep, uint64_t h0, uint64_t h1, uint64_t stride, const int32_t* imap,
           int64_t n_rows,
           int64_t n_cols, double* sum, double* sum2, double* ledger, uint64_t* counters,
           int n_threads)
{
    if (!plan->n_list || h1 > plan->n_hist || h0 > h1 || stride == 0) return -1;
    const int64_t n_sel = (int64_t)((h1 - h0 + stride - 1) / stride);
    gl_init();
    double* cdf = (double*)malloc(sizeof(double) * (size_t)m->n_ebin * m->n_ring * m->n_comp);
    or_scatter_cdf(m, cdf);
    double (*R)[9] = malloc(sizeof(double[9]) * (size_t)n_beams);
    for (int b = 0; b < n_beams; ++b) beam_rotation(&beams[b], R[b]);
    or_sampler S = {m, cdf, plan, beams, R, ph};
    or_range_table* rt = (or_range_table*)malloc(sizeof(or_range_table));
    range_table_init(rt, tp->e_cut_e, tp->density_effect, tp->physics, tp->e_cut_g);
    double rho_max = phantom_rho_max(ph);
    int64_t cells = imap ? n_rows * n_cols : (int64_t)ph->nx * ph->ny * ph->nz;
    int nt = n_threads_of(n_threads);
    double* grids = (double*)malloc(sizeof(double) * (size_t)cells * nt);
    double* er = (double*)malloc(sizeof(double) * (size_t)cells);
    double led[L_N] = {0};
    uint64_t cnt[C_N] = {0};
    for (int64_t c = 0; c < cells; ++c) { sum[c] = 0.0; sum2[c] = 0.0; }
    for (uint32_t r = rep0; r < rep0 + n_rep; ++r) {
        memset(grids, 0, sizeof(double) * (size_t)cells * nt);
        or_tracker trk[OR_MAX_THREADS];
#pragma omp parallel num_threads(nt)
        {
#ifdef _OPENMP
            int tid = omp_get_thread_num();
#else
            int tid = 0;
#endif
            or_tracker* T = &trk[tid];
            tracker_init(T, ph, tp, rt, rho_max, imap, n_cols, grids + (size_t)cells * tid);
#pragma omp for schedule(static)
            for (int64_t k = 0; k < n_sel; ++k) {
                uint64_t h = h0 + (uint64_t)k * stride;
                uint64_t g = (uint64_t)r * plan->n_hist + h;
                or_sample_rec rec;
                sample_history(&S, seed, g, &rec);
                T->cnt[C_HIST]++;
                T->ledger[L_SRC] += rec.e;
                if (rec.status == OR_ST_JAW) { T->ledger[L_JAW] += rec.e; continue; }
                if (rec.status == OR_ST_INVALID) { T->ledger[L_INVALID] += rec.e; continue; }
                if (rec.status == OR_ST_MISSED) { T->ledger[L_MISSED] += rec.e; continue; }
                T->cnt[C_ENTERED]++;
                double p[3] = {rec.x, rec.y, rec.z}, d[3] = {rec.u, rec.v, rec.w};
                if (rec.stype == OR_SUB_ELECTRON)
                    transport_electron(T, p, d, rec.e, seed, g, 0, rec.tag, 0, 0);
                else
                    transport_photon(T, p, d, rec.e, seed, g, rec.tag, 0, 0);
            }
        }
        for (int64_t c = 0; c < cells; ++c) {
            double a = 0.0;
            for (int t = 0; t < nt; ++t) a += grids[(size_t)cells * t + c];
            er[c] = a;
        }
        for (int64_t c = 0; c < cells; ++c) { sum[c] += er[c]; sum2[c] += er[c] * er[c]; }
        for (int t = 0; t < nt; ++t) {
            for (int i = 0; i < L_N; ++i) led[i] += trk[t].ledger[i];
            for (int i = 0; i < C_N; ++i) cnt[i] += trk[t].cnt[i];
        }
    }
    for (int i = 0; i < L_N; ++i) ledger[i] = led[i];
    for (int i = 0; i < C_N; ++i) counters[i] = cnt[i];
    free(cdf); free(R); free(rt); free(grids); free(er);
    return 0;
}

/* Per-history sampling records for g in [g0, g0+n) (test hook). */
int or_sample(const or_model* m, const or_plan* plan, const or_beam* beams, int n_beams,
              const or_phantom* ph, uint64_t seed, uint64_t g0, int64_t n, or_sample_rec* out)
{
    double* cdf = (double*)malloc(sizeof(double) * (size_t)m->n_ebin * m->n_ring * m->n_comp);
    or_scatter_cdf(m, cdf);
    double (*R)[9] = malloc(sizeof(double[9]) * (size_t)n_beams);
    for (int b = 0; b < n_beams; ++b) beam_rotation(&beams[b], R[b]);
    or_sampler S = {m, cdf, plan, beams, R, ph};
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) sample_history(&S, seed, g0 + (uint64_t)i, &out[i]);
    free(cdf); free(R);
    return 0;
}

/* Transports given particles (ptype 0 photon, 1 electron) that start on or in
 * the phantom; energy per cell summed into edep.  Particle i uses history id
 * hid[i] for its random streams. */
int or_transport(const or_phantom* ph, const or_params* tp, uint64_t seed, int64_t n,
                 const int32_t* ptype, const double* pos, const double* dir, const double* e,
                 const uint64_t* hid, const int32_t* tag, const int32_t* imap, int64_t n_rows,
                 int64_t n_cols, double* edep, double* ledger, uint64_t* counters, int n_threads)
{
    gl_init();
    or_range_table* rt = (or_range_table*)malloc(sizeof(or_range_table));
    range_table_init(rt, tp->e_cut_e, tp->density_effect, tp->physics, tp->e_cut_g);
    double rho_max = phantom_rho_max(ph);
    int64_t cells = imap ? n_rows * n_cols : (int64_t)ph->nx * ph->ny * ph->nz;
    int nt = n_threads_of(n_threads);
    double* grids = (double*)calloc((size_t)cells * nt, sizeof(double));
    or_tracker trk[OR_MAX_THREADS];
#pragma omp parallel num_threads(nt)
    {
#ifdef _OPENMP
        int tid = omp_get_thread_num();
#else
        int tid = 0;
#endif
        or_tracker* T = &trk[tid];
        tracker_init(T, ph, tp, rt, rho_max, imap, n_cols, grids + (size_t)cells * tid);
#pragma omp for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            double p[3] = {pos[3 * i], pos[3 * i + 1], pos[3 * i + 2]};
            double d[3] = {dir[3 * i], dir[3 * i + 1], dir[3 * i + 2]};
            T->cnt[C_HIST]++;
            T->ledger[L_SRC] += e[i];
            if (ptype[i] == 1)
                transport_electron(T, p, d, e[i], seed, hid[i], 0, tag ? tag[i] : 0, 0, 0);
            else
                transport_photon(T, p, d, e[i], seed, hid[i], tag ? tag[i] : 0, 0, 0);
        }
    }
    for (int64_t c = 0; c < cells; ++c) {
        double a = 0.0;
        for (int t = 0; t < nt; ++t) a += grids[(size_t)cells * t + c];
        edep[c] = a;
    }
    for (int i = 0; i < L_N; ++i) ledger[i] = 0.0;
    for (int i = 0; i < C_N; ++i) counters[i] = 0;
    for (int t = 0; t < nt; ++t) {
        for (int i = 0; i < L_N; ++i) ledger[i] += trk[t].ledger[i];
        for (int i = 0; i < C_N; ++i) counters[i] += trk[t].cnt[i];
    }
    free(rt); free(grids);
    return 0;
}

/* Dose in Gy per model particle from summed replica energies (MeV):
 * D = 1.602176634e-10 * mean_r(E) / (rho V) * weight_per_history, and the
 * standard error of the replica mean. */
void or_finalize(const or_phantom* ph, const double* sum, const double* sum2, uint32_t n_rep,
                 double weight_per_history, double* dose, double* sigma)
{
    int64_t V = (int64_t)ph->nx * ph->ny * ph->nz;
    double vol = ph->vox[0] * ph->vox[1] * ph->vox[2];
    for (int64_t v = 0; v < V; ++v) {
        double rho = (double)ph->density[v];
        double k = rho > 0.0 ? OR_MEV_PER_G_TO_GY * weight_per_history / (rho * vol) : 0.0;
        double mean = sum[v] / n_rep;
        double var = n_rep > 1 ? (sum2[v] / n_rep - mean * mean) * n_rep / (n_rep - 1) : 0.0;
        if (var < 0.0) var = 0.0;
        dose[v] = k * mean;
        sigma[v] = k * sqrt(var / n_rep);
    }
}

/* ------------------------------------------------------------------------ */
/* Sec. 2.2.3-2.2.4: commissioning, min_{x>=0} ||Ax - b||^2 (Eq. 8) by        */
/* gradient projection x+ = max(0, x - s grad F) with Armijo's rule.          */
/* The trial step is the Barzilai-Borwein step of the previous iteration (the */
/* first one 1/||A||_F^2); it is halved until F(x+) <= F(x) + sigma g.(x+ - x).*/
/* Stops when the relative decrease of F is below delta and the projected     */
/* gradient is below pg_tol * |g0|, or after max_iter iterations.             */
/* A is m x n column-major.                                                   */
/* ------------------------------------------------------------------------ */
static double nnls_objective(const double* A, int64_t m, int64_t n, const double* b,
                             const double* x, double* r)
{
    for (int64_t i = 0; i < m; ++i) r[i] = -b[i];
    for (int64_t j = 0; j < n; ++j) {
        double xj = x[j];
        if (xj == 0.0) continue;
        const double* col = A + j * m;
        for (int64_t i = 0; i < m; ++i) r[i] += col[i] * xj;
    }
    double f = 0.0;
    for (int64_t i = 0; i < m; ++i) f += r[i] * r[i];
    return f;
}

static void nnls_gradient(const double* A, int64_t m, int64_t n, const double* r, double* g)
{
    for (int64_t j = 0; j < n; ++j) {
        const double* col = A + j * m;
        double s = 0.0;
        for (int64_t i = 0; i < m; ++i) s += col[i] * r[i];
        g[j] = 2.0 * s;
    }
}

static double projected_gradient_norm(const double* x, const double* g, int64_t n)
{
    double s = 0.0;
    for (int64_t j = 0; j < n; ++j) {
        double pg = x[j] > 0.0 ? g[j] : (g[j] < 0.0 ? g[j] : 0.0);
        s += pg * pg;
    }
    return sqrt(s);
}

/* report[0] = iterations, [1] = F, [2] = projected-gradient norm, [3] = converged */
int or_nnls_gp(const double* A, int64_t m, int64_t n, const double* b, double* x,
               double delta, double pg_tol, double armijo_sigma, double armijo_beta,
               int64_t max_iter, double* report)
{
    double* r = (double*)malloc(sizeof(double) * (size_t)m);
    double* g = (double*)malloc(sizeof(double) * (size_t)n);
    double* xn = (double*)malloc(sizeof(double) * (size_t)n);
    double* gn = (double*)malloc(sizeof(double) * (size_t)n);
    for (int64_t j = 0; j < n; ++j) if (!(x[j] > 0.0)) x[j] = 0.0;
    double f = nnls_objective(A, m, n, b, x, r);
    nnls_gradient(A, m, n, r, g);
    double g0 = 0.0;
    for (int64_t j = 0; j < n; ++j) g0 += g[j] * g[j];
    g0 = sqrt(g0);
    double fro = 0.0;
    for (int64_t i = 0; i < m * n; ++i) fro += A[i] * A[i];
    double step = fro > 0.0 ? 1.0 / fro : 1.0;
    int64_t it = 0;
    int converged = 0;
    double pg = projected_gradient_norm(x, g, n);
    if (pg <= pg_tol * g0) converged = 1;
    while (!converged && it < max_iter) {
        ++it;
        double s = step, fn = f;
        int accepted = 0;
        for (int ls = 0; ls < 200; ++ls) {
            double dec = 0.0;
            for (int64_t j = 0; j < n; ++j) {
                double y = x[j] - s * g[j];
                xn[j] = y > 0.0 ? y : 0.0;
                dec += g[j] * (xn[j] - x[j]);
            }
            fn = nnls_objective(A, m, n, b, xn, r);
            if (fn <= f + armijo_sigma * dec) { accepted = 1; break; }
            s *= armijo_beta;
        }
        if (!accepted) break;
        nnls_gradient(A, m, n, r, gn);
        /* Barzilai-Borwein trial step for the next iteration */
        double sxx = 0.0, sxg = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            double dx = xn[j] - x[j], dg = gn[j] - g[j];
            sxx += dx * dx;
            sxg += dx * dg;
        }
        step = (sxg > 0.0) ? sxx / sxg : 2.0 * s;
        double rel = (f - fn) / (f > 0.0 ? f : 1.0);
        memcpy(x, xn, sizeof(double) * (size_t)n);
        memcpy(g, gn, sizeof(double) * (size_t)n);
        f = fn;
        pg = projected_gradient_norm(x, g, n);
        if (rel < delta && pg <= pg_tol * g0) converged = 1;
        if (f == 0.0) converged = 1;
    }
    report[0] = (double)it;
    report[1] = f;
    report[2] = pg;
    report[3] = (double)converged;
    free(r); free(g); free(xn); free(gn);
    return converged ? 0 : 1;
}
