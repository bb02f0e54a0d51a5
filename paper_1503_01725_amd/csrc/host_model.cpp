// Host side of the source model: PSR -> PSL conversion (Sec. 2.1.1), sampling
// areas (Sec. 2.1.2), particles per PSL (step S2, Eq. 3), the history order of
// Sec. 2.1.3 and batching.  All of it is integer or FP64 work done once per
// model / plan; compiled without floating-point contraction so that the
// weights and counts are reproducible bit for bit.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstring>
#include <memory>

#include "common.hpp"

namespace psl {

static thread_local std::string g_last_error;

void set_last_error(const char* msg) { g_last_error = msg ? msg : ""; }
void clear_last_error() { g_last_error.clear(); }

void fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    throw Error(code, buf);
}

namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr double kAreaSigmas = 4.0;   // buffer of a sampling area, in widths
constexpr double kQuantum = 1099511627776.0;   // 2^40

// PSL weight of a location of one (sub-source, bin): Sec. 2.1.1 steps 1-3.
double psl_weight(const double* ring_w, int n_ring, double dr, double xc, double yc) {
    const double r = std::sqrt(xc * xc + yc * yc);
    double wr;
    if (r > double(n_ring) * dr) {
        wr = 0.0;                                     // outside the model
    } else {
        const double t = r / dr - 0.5;                // position in ring-centre units
        if (t <= 0.0) {
            wr = ring_w[0];
        } else if (t >= double(n_ring - 1)) {
            wr = ring_w[n_ring - 1];
        } else {
            const int j = int(std::floor(t));
            const double f = t - double(j);
            wr = (1.0 - f) * ring_w[j] + f * ring_w[j + 1];
        }
    }
    return wr / ((2.0 * kPi) * r);
}

double widest_angle(const psl_model& m, int stype) {
    if (stype == 2) return std::max(m.d.sig_ea, m.d.sig_eb);
    double s = 0.0;
    for (size_t i = 0; i < m.sc_sa.size(); ++i) s = std::max(s, std::max(m.sc_sa[i], m.sc_sb[i]));
    return s;
}

// Sampling strip along one axis at the plane (Fig. 3).  e1, e2: jaw edges at
// the isocentre plane; zj: height of the jaw pair's upper surface.
void strip(const psl_model& m, int stype, double e1, double e2, double zj, double& lo,
           double& hi) {
    const double zt = m.d.z_target, zp = m.d.z_plane;
    const double j1 = e1 * (zj - zt) / (zp - zt);
    const double j2 = e2 * (zj - zt) / (zp - zt);
    if (stype == 0) {
        // primary: the opening itself plus the shadow a focal spot of
        // kAreaSigmas widths casts through the jaw edge onto the plane
        const double margin = kAreaSigmas * m.d.sigma_spot * (zp - zj) / (zj - zt);
        lo = e1 - margin;
        hi = e2 + margin;
        return;
    }
    // scatter: mean rays come from the scatter source on the axis, so plane
    // distances are jaw-height distances magnified by (zp - zs)/(zj - zs);
    // electrons: vertical mean ray, no magnification
    const double mag = (stype == 1) ? (zp - m.d.z_scatter) / (zj - m.d.z_scatter) : 1.0;
    const double margin = (zp - zj) * std::tan(kAreaSigmas * widest_angle(m, stype)) * mag;
    lo = j1 * mag - margin;
    hi = j2 * mag + margin;
}

// PSLs overlapping [lo, hi] with positive length along one axis.
void index_range(const psl_model& m, double lo, double hi, int& i0, int& i1) {
    i0 = int(std::floor((lo - m.d.psl_x0) / m.d.psl_dx));
    i1 = int(std::ceil((hi - m.d.psl_x0) / m.d.psl_dx)) - 1;
    i0 = std::max(i0, 0);
    i1 = std::min(i1, m.d.n_psl - 1);
}

void beam_matrix(const psl_beam& b, double R[9]) {
    const double g = b.gantry_deg * kPi / 180.0, c = b.couch_deg * kPi / 180.0;
    const double cg = std::cos(g), sg = std::sin(g), cc = std::cos(c), sc = std::sin(c);
    // Rz(couch) * Ry(gantry)
    const double ry[3][3] = {{cg, 0.0, sg}, {0.0, 1.0, 0.0}, {-sg, 0.0, cg}};
    const double rz[3][3] = {{cc, -sc, 0.0}, {sc, cc, 0.0}, {0.0, 0.0, 1.0}};
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double a = 0.0;
            for (int k = 0; k < 3; ++k) a += rz[i][k] * ry[k][j];
            R[i * 3 + j] = a;
        }
}

// Systematic rounding inside one group: entry i gets
// round(total * Q_i / S) - round(total * Q_{i-1} / S), Q the running sum.
void allocate_group(const std::vector<uint64_t>& q, size_t a, size_t b, uint64_t total,
                    std::vector<uint64_t>& n) {
    unsigned __int128 S = 0;
    for (size_t i = a; i < b; ++i) S += q[i];
    if (S == 0) {
        for (size_t i = a; i < b; ++i) n[i] = 0;
        return;
    }
    unsigned __int128 run = 0, done = 0;
    for (size_t i = a; i < b; ++i) {
        run += q[i];
        const unsigned __int128 upto = (static_cast<unsigned __int128>(total) * run + S / 2) / S;
        n[i] = static_cast<uint64_t>(upto - done);
        done = upto;
    }
}

}  // namespace

void ensure_device(const psl_model* m) {
    if (!m->scatter.p) m->scatter.upload(m->scatter_host);
}

void ensure_device(const psl_plan* p) {
    ensure_device(p->model);
    if (!p->d_list.p) p->d_list.upload(p->list_host);
    if (!p->d_cum.p) p->d_cum.upload(p->cum);
    if (!p->d_chunk.p) {
        // one merge pass over the prefix: entry c is the first j with
        // cum[j] > c * 2^kChunkShift
        const uint64_t n_chunk = (p->n_hist >> kChunkShift) + 2;
        PSL_CHECK(p->cum.size() < (size_t(1) << 32), "plan list too long for the chunk index");
        std::vector<uint32_t> chunk(n_chunk);
        size_t j = 0;
        for (uint64_t c = 0; c < n_chunk; ++c) {
            const uint64_t h = c << kChunkShift;
            while (j < p->cum.size() && !(p->cum[j] > h)) ++j;
            chunk[c] = uint32_t(j);
        }
        p->d_chunk.upload(chunk);
    }
    if (!p->d_beams.p) p->d_beams.upload(p->beams_host);
}

}  // namespace psl

using namespace psl;

extern "C" const char* psl_last_error(void) { return g_last_error.c_str(); }

extern "C" int psl_build(const psl_psr_desc* desc, psl_model** out) {
    return guarded([&] {
        PSL_CHECK(desc && out, "psl_build: null argument");
        const psl_psr_desc& d = *desc;
        PSL_CHECK(d.n_ebin >= 1 && d.n_ebin <= 255, "n_ebin must be in [1, 255]");
        PSL_CHECK(d.n_ring >= 1 && d.n_psl >= 1 && d.n_psl <= 255, "bad n_ring / n_psl");
        PSL_CHECK(d.n_comp >= 1 && d.n_comp <= 8, "n_comp must be in [1, 8]");
        PSL_CHECK(d.w_psr && d.sc_c && d.sc_mu && d.sc_sa && d.sc_sb, "null model array");
        PSL_CHECK(d.e_width > 0 && d.ring_dr > 0 && d.psl_dx > 0 && d.e_lo >= 0, "bad grid");
        PSL_CHECK(d.z_target < d.z_jaw_y && d.z_target < d.z_jaw_x && d.z_jaw_y < d.z_plane &&
                      d.z_jaw_x < d.z_plane && d.z_scatter < d.z_jaw_y &&
                      d.z_scatter < d.z_jaw_x && d.z_target < d.z_scatter,
                  "heights must satisfy target < scatter < jaws < plane");
        auto m = std::make_unique<psl_model>();
        m->d = d;
        const size_t n_w = size_t(3) * d.n_ebin * d.n_ring;
        const size_t n_s = size_t(d.n_ebin) * d.n_ring * d.n_comp;
        m->w_psr.assign(d.w_psr, d.w_psr + n_w);
        m->sc_c.assign(d.sc_c, d.sc_c + n_s);
        m->sc_mu.assign(d.sc_mu, d.sc_mu + n_s);
        m->sc_sa.assign(d.sc_sa, d.sc_sa + n_s);
        m->sc_sb.assign(d.sc_sb, d.sc_sb + n_s);
        for (double v : m->w_psr) PSL_CHECK(std::isfinite(v) && v >= 0, "PSR weights must be >= 0");
        for (size_t i = 0; i < n_s; ++i)
            PSL_CHECK(m->sc_c[i] >= 0 && m->sc_sa[i] >= 0 && m->sc_sb[i] >= 0,
                      "scatter parameters must be >= 0");
        m->d.w_psr = m->d.sc_c = m->d.sc_mu = m->d.sc_sa = m->d.sc_sb = nullptr;
        m->e_max = d.e_lo + d.n_ebin * d.e_width;

        // Sec. 2.1.1: weight of every PSL, then one normalisation over all
        // sub-sources, energies and locations (sum in (s, b, y, x) order)
        const int n = d.n_psl;
        m->w_psl.resize(size_t(3) * d.n_ebin * n * n);
        size_t k = 0;
        for (int s = 0; s < 3; ++s)
            for (int b = 0; b < d.n_ebin; ++b) {
                const double* ring_w = &m->w_psr[(size_t(s) * d.n_ebin + b) * d.n_ring];
                for (int iy = 0; iy < n; ++iy) {
                    const double yc = d.psl_x0 + (double(iy) + 0.5) * d.psl_dx;
                    for (int ix = 0; ix < n; ++ix) {
                        const double xc = d.psl_x0 + (double(ix) + 0.5) * d.psl_dx;
                        m->w_psl[k++] = psl_weight(ring_w, d.n_ring, d.ring_dr, xc, yc);
                    }
                }
            }
        double total = 0.0;
        for (double v : m->w_psl) total += v;
        PSL_CHECK(total > 0.0 && std::isfinite(total), "model has no positive PSL weight");
        for (double& v : m->w_psl) v = v / total;

        // step S4: cumulative component probabilities, and the device table
        const int K = d.n_comp;
        m->cdf.resize(n_s);
        std::vector<ScatterComp> tab(n_s);
        for (size_t i = 0; i < size_t(d.n_ebin) * d.n_ring; ++i) {
            double tot = 0.0;
            for (int c = 0; c < K; ++c) tot += m->sc_c[i * K + c];
            PSL_CHECK(tot > 0.0, "scatter mixture weights of a PSR add up to 0");
            double run = 0.0;
            for (int c = 0; c < K; ++c) {
                run += m->sc_c[i * K + c];
                m->cdf[i * K + c] = (c == K - 1) ? 1.0 : run / tot;
                tab[i * K + c] = ScatterComp{float(m->cdf[i * K + c]), float(m->sc_mu[i * K + c]),
                                             float(m->sc_sa[i * K + c]), float(m->sc_sb[i * K + c])};
            }
        }
        m->scatter_host = std::move(tab);
        *out = m.release();
    });
}

extern "C" int psl_model_weights(const psl_model* model, double* w) {
    return guarded([&] {
        PSL_CHECK(model && w, "null argument");
        std::memcpy(w, model->w_psl.data(), model->w_psl.size() * sizeof(double));
    });
}

extern "C" void psl_model_free(psl_model* model) { delete model; }

extern "C" int psl_plan_create(const psl_model* model, const psl_beam* beams, int32_t n_beams,
                               uint64_t n_hist, uint32_t n_replica, const uint16_t* basis_of_psr,
                               uint64_t hist_per_basis, psl_plan** out) {
    return guarded([&] {
        PSL_CHECK(model && beams && out, "psl_plan_create: null argument");
        PSL_CHECK(n_beams >= 1 && n_beams <= 65535, "n_beams must be in [1, 65535]");
        PSL_CHECK(n_replica >= 1, "n_replica must be >= 1");
        const bool stratified = hist_per_basis > 0;
        PSL_CHECK(!stratified || basis_of_psr, "hist_per_basis needs a basis map");
        PSL_CHECK(stratified || n_hist >= 1, "n_hist must be >= 1");
        const psl_model& m = *model;
        const int n = m.d.n_psl, nb = m.d.n_ebin, nr = m.d.n_ring;
        for (int i = 0; i < n_beams; ++i)
            PSL_CHECK(beams[i].x1 < beams[i].x2 && beams[i].y1 < beams[i].y2,
                      "beam %d: jaw edges must satisfy x1 < x2, y1 < y2", i);

        auto p = std::make_unique<psl_plan>();
        p->model = model;
        p->beams.assign(beams, beams + n_beams);
        p->n_replica = n_replica;
        int n_basis = 1;
        if (basis_of_psr) {
            int mx = 0;
            for (size_t i = 0; i < size_t(3) * nb * nr; ++i) mx = std::max(mx, int(basis_of_psr[i]));
            n_basis = mx + 1;
            // tally columns travel in bits 0-14 of a particle's tag (bit 15
            // marks a positron)
            PSL_CHECK(int64_t(n_basis) * n_beams <= 32768, "n_beams * n_basis must be <= 32768");
        }
        p->n_cols = basis_of_psr ? n_basis * n_beams : 1;

        // basis id of every PSL location (ring of its centre), per (s, b)
        std::vector<int> ring_of(size_t(n) * n);
        for (int iy = 0; iy < n; ++iy)
            for (int ix = 0; ix < n; ++ix) {
                const double xc = m.d.psl_x0 + (double(ix) + 0.5) * m.d.psl_dx;
                const double yc = m.d.psl_x0 + (double(iy) + 0.5) * m.d.psl_dx;
                ring_of[size_t(iy) * n + ix] =
                    std::min(int(std::floor(std::sqrt(xc * xc + yc * yc) / m.d.ring_dr)), nr - 1);
            }

        p->boxes.resize(size_t(n_beams) * 12);
        for (int bi = 0; bi < n_beams; ++bi) {
            const psl_beam& bm = beams[bi];
            for (int s = 0; s < 3; ++s) {
                double xlo, xhi, ylo, yhi;
                strip(m, s, bm.x1, bm.x2, m.d.z_jaw_x, xlo, xhi);
                strip(m, s, bm.y1, bm.y2, m.d.z_jaw_y, ylo, yhi);
                int* box = &p->boxes[size_t(bi) * 12 + s * 4];
                index_range(m, xlo, xhi, box[0], box[1]);
                index_range(m, ylo, yhi, box[2], box[3]);
            }
        }

        // the list: beam, [basis,] sub-source, bin, y, x (Sec. 2.1.3)
        auto append = [&](int bi, int s, int b, int iy, int ix, int basis) {
            const double w = m.w_psl[((size_t(s) * nb + b) * n + iy) * n + ix];
            p->beam.push_back(bi);
            p->stype.push_back(s);
            p->ebin.push_back(b);
            p->ix.push_back(ix);
            p->iy.push_back(iy);
            p->tag.push_back(basis_of_psr ? bi * n_basis + basis : 0);
            p->w.push_back(w);
        };
        for (int bi = 0; bi < n_beams; ++bi) {
            const int* bx = &p->boxes[size_t(bi) * 12];
            for (int k = 0; k < (stratified ? n_basis : 1); ++k)
                for (int s = 0; s < 3; ++s)
                    for (int b = 0; b < nb; ++b)
                        for (int iy = bx[s * 4 + 2]; iy <= bx[s * 4 + 3]; ++iy)
                            for (int ix = bx[s * 4 + 0]; ix <= bx[s * 4 + 1]; ++ix) {
                                if (!(m.w_psl[((size_t(s) * nb + b) * n + iy) * n + ix] > 0.0))
                                    continue;
                                int basis = 0;
                                if (basis_of_psr) {
                                    basis = basis_of_psr[(size_t(s) * nb + b) * nr +
                                                         ring_of[size_t(iy) * n + ix]];
                                    if (stratified && basis != k) continue;
                                }
                                append(bi, s, b, iy, ix, basis);
                            }
        }
        const size_t L = p->w.size();
        PSL_CHECK(L > 0, "no PSL with positive weight inside the sampling areas");

        // step S2, Eq. (3): counts by systematic rounding of quantised weights
        std::vector<uint64_t> q(L), cnt(L);
        for (size_t i = 0; i < L; ++i) q[i] = uint64_t(std::llround(p->w[i] * kQuantum));
        p->col_weight.assign(p->n_cols, 0.0);
        if (stratified) {
            size_t a = 0;
            while (a < L) {
                size_t b = a;
                while (b < L && p->tag[b] == p->tag[a]) ++b;
                allocate_group(q, a, b, hist_per_basis, cnt);
                double ws = 0.0;
                for (size_t i = a; i < b; ++i) ws += p->w[i];
                p->col_weight[p->tag[a]] = ws / double(hist_per_basis);
                a = b;
            }
        } else {
            allocate_group(q, 0, L, n_hist, cnt);
        }
        double s_area = 0.0;
        for (size_t i = 0; i < L; ++i) s_area += p->w[i];
        p->s_area = s_area;
        p->cum.resize(L);
        uint64_t run = 0;
        for (size_t i = 0; i < L; ++i) p->cum[i] = (run += cnt[i]);
        p->n_hist = run;
        PSL_CHECK(p->n_hist > 0, "plan has no histories");
        if (!stratified)
            for (auto& cw : p->col_weight) cw = s_area / double(n_hist);

        // device copies
        std::vector<PslEntry> ent(L);
        for (size_t i = 0; i < L; ++i)
            ent[i] = PslEntry{uint8_t(p->ix[i]), uint8_t(p->iy[i]), uint8_t(p->stype[i]),
                              uint8_t(p->ebin[i]), uint16_t(p->beam[i]), uint16_t(p->tag[i])};
        p->list_host = std::move(ent);
        std::vector<BeamDev> bd(n_beams);
        const double zt = m.d.z_target, zp = m.d.z_plane;
        for (int bi = 0; bi < n_beams; ++bi) {
            double R[9];
            beam_matrix(beams[bi], R);
            BeamDev& o = bd[bi];
            for (int i = 0; i < 9; ++i) o.R[i] = float(R[i]);
            for (int i = 0; i < 3; ++i) o.iso[i] = float(beams[bi].iso[i]);
            const double kx = (m.d.z_jaw_x - zt) / (zp - zt), ky = (m.d.z_jaw_y - zt) / (zp - zt);
            o.jx1 = float(beams[bi].x1 * kx);
            o.jx2 = float(beams[bi].x2 * kx);
            o.jy1 = float(beams[bi].y1 * ky);
            o.jy2 = float(beams[bi].y2 * ky);
            o.pad[0] = o.pad[1] = 0.f;
        }
        p->beams_host = std::move(bd);
        *out = p.release();
        int64_t nbatch = 0;
        int rc = psl_plan_set_batching(*out, 131072, 1, &nbatch);
        if (rc != PSL_OK) fail(rc, "%s", psl_last_error());
    });
}

extern "C" int psl_plan_get_info(const psl_plan* p, psl_plan_info* info) {
    return guarded([&] {
        PSL_CHECK(p && info, "null argument");
        info->n_hist = p->n_hist;
        info->n_replica = p->n_replica;
        info->n_beams = int32_t(p->beams.size());
        info->n_list = int64_t(p->w.size());
        info->n_cols = p->n_cols;
        info->s_area = p->s_area;
        info->e_max = p->model->e_max;
    });
}

extern "C" int psl_plan_boxes(const psl_plan* p, int32_t* boxes) {
    return guarded([&] {
        PSL_CHECK(p && boxes, "null argument");
        std::memcpy(boxes, p->boxes.data(), p->boxes.size() * sizeof(int32_t));
    });
}

extern "C" int psl_plan_list(const psl_plan* p, int32_t* beam, int32_t* stype, int32_t* ebin,
                             int32_t* ix, int32_t* iy, int32_t* tag, double* w, uint64_t* cum) {
    return guarded([&] {
        PSL_CHECK(p, "null plan");
        const size_t L = p->w.size();
        auto cp = [L](auto* dst, const auto& src) {
            if (dst) std::memcpy(dst, src.data(), L * sizeof(src[0]));
        };
        cp(beam, p->beam);
        cp(stype, p->stype);
        cp(ebin, p->ebin);
        cp(ix, p->ix);
        cp(iy, p->iy);
        cp(tag, p->tag);
        cp(w, p->w);
        cp(cum, p->cum);
    });
}

extern "C" int psl_plan_col_weight(const psl_plan* p, double* w) {
    return guarded([&] {
        PSL_CHECK(p && w, "null argument");
        std::memcpy(w, p->col_weight.data(), p->col_weight.size() * sizeof(double));
    });
}

extern "C" int psl_plan_set_batching(psl_plan* p, uint32_t max_batch, int32_t band_width,
                                     int64_t* n_batches) {
    return guarded([&] {
        PSL_CHECK(p, "null plan");
        PSL_CHECK(max_batch >= 1, "max_batch must be >= 1");
        PSL_CHECK(band_width >= 1, "band_width must be >= 1");
        p->batches.clear();
        p->batch_jlo.clear();
        p->batch_jhi.clear();
        uint64_t prev = 0;
        bool open = false;
        psl_batch cur{};
        for (size_t j = 0; j < p->cum.size(); ++j) {
            uint64_t left = p->cum[j] - prev;
            uint64_t h = prev;
            prev = p->cum[j];
            const int band = p->ebin[j] / band_width;
            while (left > 0) {
                if (open && (cur.beam != p->beam[j] || cur.stype != p->stype[j] ||
                             cur.band != band || cur.n == max_batch)) {
                    p->batches.push_back(cur);
                    open = false;
                }
                if (!open) {
                    cur = psl_batch{h, 0, p->stype[j], p->beam[j], band};
                    open = true;
                }
                const uint64_t take = std::min<uint64_t>(left, max_batch - cur.n);
                cur.n += uint32_t(take);
                left -= take;
                h += take;
            }
        }
        if (open) p->batches.push_back(cur);
        p->batch_jlo.resize(p->batches.size());
        p->batch_jhi.resize(p->batches.size());
        // tighten the list ranges: [first entry with cum > h0, first with cum >= h0+n] + 1
        for (size_t i = 0; i < p->batches.size(); ++i) {
            const uint64_t h0 = p->batches[i].h0, h1 = h0 + p->batches[i].n;
            const auto b0 = std::upper_bound(p->cum.begin(), p->cum.end(), h0);
            const auto b1 = std::upper_bound(p->cum.begin(), p->cum.end(), h1 - 1);
            p->batch_jlo[i] = b0 - p->cum.begin();
            p->batch_jhi[i] = (b1 - p->cum.begin()) + 1;
        }
        p->cur_max_batch = max_batch;
        p->cur_band_width = band_width;
        if (n_batches) *n_batches = int64_t(p->batches.size());
    });
}

extern "C" int psl_plan_get_batch(const psl_plan* p, int64_t i, psl_batch* b) {
    return guarded([&] {
        PSL_CHECK(p && b, "null argument");
        PSL_CHECK(i >= 0 && i < int64_t(p->batches.size()), "batch index out of range");
        *b = p->batches[size_t(i)];
    });
}

extern "C" void psl_plan_free(psl_plan* p) { delete p; }
