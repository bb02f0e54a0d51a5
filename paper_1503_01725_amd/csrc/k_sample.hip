// Source sampling kernel (steps S3-S5): one thread per history.  A batch holds
// one sub-source, so the kernel is specialised per sub-source and its waves
// never diverge on the direction model (Sec. 2.1.3).
#include "device.hpp"

namespace psl {
namespace {

struct SampleArgs {
    const PslEntry* list;
    const uint64_t* cum;
    const uint32_t* chunk;       // chunk index of the count prefix (see psl_plan)
    int64_t jlo, jhi;            // list range holding the batch's histories
    uint64_t h0, n_hist;
    uint32_t n, rep;
    const uint32_t* rep_dev;     // replica index in device memory (graph replays), or null
    uint32_t seed_lo, seed_hi;
    const ScatterComp* sc;       // [n_ebin][n_ring][K]
    int n_ring, n_comp;
    float inv_ring_dr;
    float psl_x0, psl_dx, e_lo, e_width;
    float sigma_spot, z_phsp, sig_ea, sig_eb;
    float zjy, zjx;              // jaw surfaces relative to the plane (negative)
    const BeamDev* beams;
    float box_lo[3], box_hi[3];
    float *x, *y, *z, *u, *v, *w, *e;
    uint64_t* hid;
    uint32_t* tag;
    uint32_t* count;
    uint32_t capacity;
    int dense;                   // 0 compact, 1 dense (full records), 2 dense (tags only if
                                 // rejected), 3 phase-space-plane records (no jaws, no transform)
    double* stats;
    unsigned long long* counters;
};

enum : uint32_t { kOk = 0, kJaw = 1, kMissed = 2, kInvalid = 3 };

// First j in [lo, hi) with cum[j] > h.
__device__ __forceinline__ int64_t upper_bound(const uint64_t* cum, int64_t lo, int64_t hi,
                                               uint64_t h) {
    while (lo < hi) {
        const int64_t mid = lo + ((hi - lo) >> 1);
        if (cum[mid] > h) hi = mid; else lo = mid + 1;
    }
    return lo;
}

// Second half of a history's source step: jaw rejection at the upper jaw
// surfaces (closed intervals), beam frame -> patient frame (the plane is the
// isocentre plane), then the entry of the particle's line into the phantom
// box (slab method).  Shared by the fused sampler and the transform of
// phase-space-plane records, so both give the same bits.  Returns kOk, kJaw
// or kMissed; p* and d* are set for kOk.
__device__ __forceinline__ uint32_t to_patient(const BeamDev& B, float zjy, float zjx,
                                               const float* box_lo, const float* box_hi, float x,
                                               float y, float ub, float vb, float wb, float& px,
                                               float& py, float& pz, float& du, float& dv,
                                               float& dw) {
    const float yj = fmaf(vb / wb, zjy, y);
    const float xj = fmaf(ub / wb, zjx, x);
    if (!(yj >= B.jy1 && yj <= B.jy2 && xj >= B.jx1 && xj <= B.jx2)) return kJaw;
    const float p0 = B.iso[0] + B.R[0] * x + B.R[1] * y;
    const float p1 = B.iso[1] + B.R[3] * x + B.R[4] * y;
    const float p2 = B.iso[2] + B.R[6] * x + B.R[7] * y;
    du = B.R[0] * ub + B.R[1] * vb + B.R[2] * wb;
    dv = B.R[3] * ub + B.R[4] * vb + B.R[5] * wb;
    dw = B.R[6] * ub + B.R[7] * vb + B.R[8] * wb;
    const float pp[3] = {p0, p1, p2}, dd[3] = {du, dv, dw};
    float tmin = -INFINITY, tmax = INFINITY;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        if (dd[ax] != 0.f) {
            const float inv = 1.f / dd[ax];
            const float t1 = (box_lo[ax] - pp[ax]) * inv;
            const float t2 = (box_hi[ax] - pp[ax]) * inv;
            tmin = fmaxf(tmin, fminf(t1, t2));
            tmax = fminf(tmax, fmaxf(t1, t2));
        } else if (pp[ax] < box_lo[ax] || pp[ax] > box_hi[ax]) {
            tmax = -INFINITY;
        }
    }
    if (!(tmax > tmin)) return kMissed;
    px = fmaf(tmin, du, p0);
    py = fmaf(tmin, dv, p1);
    pz = fmaf(tmin, dw, p2);
    return kOk;
}

template <int STYPE>
__global__ void __launch_bounds__(256) k_sample(SampleArgs a) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = i < a.n;
    // The block's histories are consecutive, so their PSLs lie between the
    // PSLs of its first and last history: two threads locate those, then every
    // thread searches only that short range (cached) instead of the whole list.
    // The two searches start from the chunk index, which brackets the answer
    // for any h by the entries of h's chunk and of the next one.
    __shared__ int64_t s_range[2];
    {
        const uint32_t first = blockIdx.x * blockDim.x;
        const uint32_t last = min(first + blockDim.x, a.n) - 1u;
        const uint64_t hf = a.h0 + first, hl = a.h0 + last;
        const int64_t lo = max(a.jlo, int64_t(a.chunk[hf >> kChunkShift]));
        const int64_t hi = min(a.jhi, int64_t(a.chunk[(hl >> kChunkShift) + 1]) + 1);
        if (threadIdx.x == 0) s_range[0] = upper_bound(a.cum, lo, hi, hf);
        if (threadIdx.x == 64 || (blockDim.x <= 64 && threadIdx.x == 0))
            s_range[1] = upper_bound(a.cum, lo, hi, hl) + 1;
    }
    __syncthreads();
    const int64_t jb0 = s_range[0], jb1 = s_range[1];
    dev::LocalStats ls;
    bool accept = false;
    float px = 0.f, py = 0.f, pz = 0.f, du = 0.f, dv = 0.f, dw = 0.f, en = 0.f;
    uint64_t g = 0;
    uint32_t tag = 0, status = kOk;
    if (live) {
        const uint64_t h = a.h0 + i;
        const uint32_t rep = a.rep_dev ? *a.rep_dev : a.rep;
        g = uint64_t(rep) * a.n_hist + h;
        const int64_t j = upper_bound(a.cum, jb0, jb1, h);
        const PslEntry ent = a.list[j];
        tag = ent.tag;

        dev::Stream st;
        st.init(a.seed_lo, a.seed_hi, g, dev::kTagSource, 0);
        const float u0 = st.next(), u1 = st.next(), u2 = st.next(), u3 = st.next();
        const float u4 = st.next(), u5 = st.next();

        // position uniform in the PSL square, energy uniform in the bin
        const float x = fmaf(a.psl_dx, u0, fmaf(float(ent.ix), a.psl_dx, a.psl_x0));
        const float y = fmaf(a.psl_dx, u1, fmaf(float(ent.iy), a.psl_dx, a.psl_x0));
        en = fmaf(a.e_width, u2, fmaf(float(ent.ebin), a.e_width, a.e_lo));
        const float r = sqrtf(x * x + y * y);
        float ct = 1.f, sn = 0.f;
        if (r > 0.f) {
            ct = x / r;
            sn = y / r;
        }
        // Box-Muller pair
        const float rad = sqrtf(-2.f * logf(1.f - u4));
        float sphi, cphi;
        sincospif(2.f * u5, &sphi, &cphi);
        const float g1 = rad * cphi, g2 = rad * sphi;

        float ul, vl, wl;
        bool invalid = false;
        if (STYPE == 0) {
            // Eq. (4)-(5): focal-spot point, then the ray from it
            const float xs = a.sigma_spot * g1, ys = a.sigma_spot * g2;
            const float dx = r - xs;
            const float D = sqrtf(dx * dx + ys * ys + a.z_phsp * a.z_phsp);
            ul = dx / D;
            vl = -ys / D;
            wl = a.z_phsp / D;
        } else {
            float al, be;
            if (STYPE == 1) {
                // Eq. (6): PSR of the sampled radius, component by the cumulative
                // table, then that component's Gaussian in (alpha, beta)
                int ring = int(floorf(r * a.inv_ring_dr));
                ring = min(ring, a.n_ring - 1);
                const ScatterComp* c = a.sc + (size_t(ent.ebin) * a.n_ring + ring) * a.n_comp;
                int k = 0;
                while (k < a.n_comp - 1 && !(u3 < c[k].cdf)) ++k;
                const ScatterComp cc = c[k];
                al = fmaf(cc.sa, g1, cc.mu);
                be = cc.sb * g2;
            } else {
                // Eq. (7): zero-mean Gaussian angles
                al = a.sig_ea * g1;
                be = a.sig_eb * g2;
            }
            invalid = !(fabsf(al) < 1.57079632679f && fabsf(be) < 1.57079632679f);
            const float ta = tanf(al), tb = tanf(be);
            const float nrm = sqrtf(ta * ta + tb * tb + 1.f);
            ul = ta / nrm;
            vl = tb / nrm;
            wl = 1.f / nrm;
        }
        // rotate the local (radial, tangential) frame by theta = atan2(y, x)
        const float ub = ct * ul - sn * vl;
        const float vb = sn * ul + ct * vl;
        const float wb = wl;

        ls.l[L_SRC] = en;
        ls.c[C_HIST] = 1;
        if (invalid) {
            status = kInvalid;
            ls.l[L_INVALID] = en;
        } else if (a.dense == 3) {
            // phase-space-plane record: the beam travels in the tag
            tag |= uint32_t(ent.beam) << 16;
        } else {
            status = to_patient(a.beams[ent.beam], a.zjy, a.zjx, a.box_lo, a.box_hi, x, y, ub, vb,
                                wb, px, py, pz, du, dv, dw);
            if (status == kOk) {
                accept = true;
                ls.c[C_ENTERED] = 1;
            } else if (status == kJaw) {
                ls.l[L_JAW] = en;
            } else {
                ls.l[L_MISSED] = en;
            }
        }
        if (!accept) {
            // rejected particles (and plane records) keep their beam-frame
            // state for dense output
            px = x;
            py = y;
            pz = 0.f;
            du = ub;
            dv = vb;
            dw = wb;
        }
    }

    if (a.dense) {
        if (blockIdx.x == 0 && threadIdx.x == 0) *a.count = a.n;
        if (live) {
            if (accept || a.dense == 1 || a.dense == 3) {
                a.x[i] = px; a.y[i] = py; a.z[i] = pz;
                a.u[i] = du; a.v[i] = dv; a.w[i] = dw;
                a.e[i] = en;
                a.hid[i] = g;
            }
            a.tag[i] = tag | (status << 24);
        }
    } else {
        const uint32_t slot = dev::wave_reserve(accept, a.count);
        if (accept) {
            if (slot < a.capacity) {
                a.x[slot] = px; a.y[slot] = py; a.z[slot] = pz;
                a.u[slot] = du; a.v[slot] = dv; a.w[slot] = dw;
                a.e[slot] = en;
                a.hid[slot] = g;
                a.tag[slot] = tag;
            } else {
                ls.c[C_OVERFLOW] += 1;
            }
        }
    }
    dev::flush_stats(a.stats, ls);
}

// Phase-space-plane records -> transport stack: the second half of k_sample
// for a source that comes from particle files (the paper's PSL-file source
// model, which reads particles at the plane and translates / rotates them on
// the GPU; Sec. 3.1, Table 1).  One thread per record; dense output in the
// layout of PSL_SAMPLE_DENSE.
struct TransformArgs {
    const float *x, *y, *u, *v, *w, *e;
    const uint64_t* hid;
    const uint32_t* tag;
    uint32_t n;
    float zjy, zjx;
    const BeamDev* beams;
    int n_beams;
    float box_lo[3], box_hi[3];
    float *ox, *oy, *oz, *ou, *ov, *ow, *oe;
    uint64_t* ohid;
    uint32_t* otag;
    uint32_t* ocount;
    double* stats;
};

__global__ void __launch_bounds__(256) k_transform(TransformArgs a) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    dev::LocalStats ls;
    if (i < a.n) {
        const uint32_t tg = a.tag[i];
        uint32_t status = tg >> 24;
        const float x = a.x[i], y = a.y[i], ub = a.u[i], vb = a.v[i], wb = a.w[i], en = a.e[i];
        float px = x, py = y, pz = 0.f, du = ub, dv = vb, dw = wb;
        if (status == kOk) {
            const int beam = int((tg >> 16) & 0xFFu);
            if (beam >= a.n_beams) {
                // not a record of this plan: rejected as invalid
                status = kInvalid;
                ls.l[L_INVALID] = en;
            } else {
                float qx, qy, qz, qu, qv, qw;
                status = to_patient(a.beams[beam], a.zjy, a.zjx, a.box_lo, a.box_hi, x, y, ub, vb,
                                    wb, qx, qy, qz, qu, qv, qw);
                if (status == kOk) {
                    px = qx; py = qy; pz = qz;
                    du = qu; dv = qv; dw = qw;
                    ls.c[C_ENTERED] = 1;
                } else if (status == kJaw) {
                    ls.l[L_JAW] = en;
                } else {
                    ls.l[L_MISSED] = en;
                }
            }
        }
        a.ox[i] = px; a.oy[i] = py; a.oz[i] = pz;
        a.ou[i] = du; a.ov[i] = dv; a.ow[i] = dw;
        a.oe[i] = en;
        a.ohid[i] = a.hid[i];
        a.otag[i] = (tg & 0xFFFFu) | (status << 24);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) *a.ocount = a.n;
    dev::flush_stats(a.stats, ls);
}

}  // namespace

// Host launcher shared by sample_batch and the batched runtime.
void launch_sample(const psl_plan* plan, const psl_phantom* ph, uint32_t replica,
                   const uint32_t* rep_dev, uint64_t h0, uint32_t n, int64_t jlo, int64_t jhi,
                   int stype, uint64_t seed, const psl_particles* out, int dense, psl_tally* tally,
                   hipStream_t stream) {
    ensure_device(plan);
    const psl_model& m = *plan->model;
    SampleArgs a{};
    a.list = plan->d_list.as<PslEntry>();
    a.cum = plan->d_cum.as<uint64_t>();
    a.chunk = plan->d_chunk.as<uint32_t>();
    a.jlo = jlo;
    a.jhi = jhi;
    a.h0 = h0;
    a.n_hist = plan->n_hist;
    a.n = n;
    a.rep = replica;
    a.rep_dev = rep_dev;
    a.seed_lo = uint32_t(seed);
    a.seed_hi = uint32_t(seed >> 32);
    a.sc = m.scatter.as<ScatterComp>();
    a.n_ring = m.d.n_ring;
    a.n_comp = m.d.n_comp;
    a.inv_ring_dr = float(1.0 / m.d.ring_dr);
    a.psl_x0 = float(m.d.psl_x0);
    a.psl_dx = float(m.d.psl_dx);
    a.e_lo = float(m.d.e_lo);
    a.e_width = float(m.d.e_width);
    a.sigma_spot = float(m.d.sigma_spot);
    a.z_phsp = float(m.d.z_plane - m.d.z_target);
    a.sig_ea = float(m.d.sig_ea);
    a.sig_eb = float(m.d.sig_eb);
    a.zjy = float(m.d.z_jaw_y - m.d.z_plane);
    a.zjx = float(m.d.z_jaw_x - m.d.z_plane);
    a.beams = plan->d_beams.as<BeamDev>();
    for (int k = 0; k < 3; ++k) {
        a.box_lo[k] = ph->g.origin[k];
        a.box_hi[k] = ph->g.hi[k];
    }
    a.x = out->x; a.y = out->y; a.z = out->z;
    a.u = out->u; a.v = out->v; a.w = out->w;
    a.e = out->e;
    a.hid = out->hid;
    a.tag = out->tag;
    a.count = out->count;
    a.capacity = out->capacity;
    a.dense = dense;
    TallyDev t = tally->dev();
    a.stats = t.stats;
    a.counters = t.counters;
    const dim3 block(256), grid((n + 255) / 256);
    if (stype == 0) hipLaunchKernelGGL(k_sample<0>, grid, block, 0, stream, a);
    else if (stype == 1) hipLaunchKernelGGL(k_sample<1>, grid, block, 0, stream, a);
    else hipLaunchKernelGGL(k_sample<2>, grid, block, 0, stream, a);
    PSL_HIP(hipGetLastError());
}

// Plane records carry the beam index in tag bits 16-23.
bool plane_beams_fit(const psl_plan* plan) { return plan->beams.size() <= 255; }

}  // namespace psl

using namespace psl;

extern "C" int sample_batch(const psl_plan* plan, const psl_phantom* phantom, uint32_t replica,
                            uint64_t h0, uint32_t n, uint64_t seed, psl_particles* out,
                            uint32_t flags, psl_tally* tally, void* stream) {
    return guarded([&] {
        PSL_CHECK(plan && phantom && out && tally, "sample_batch: null argument");
        PSL_CHECK(n >= 1, "n must be >= 1");
        PSL_CHECK(h0 + n <= plan->n_hist, "history range [%llu, %llu) beyond the plan's %llu",
                  (unsigned long long)h0, (unsigned long long)(h0 + n),
                  (unsigned long long)plan->n_hist);
        PSL_CHECK(replica < plan->n_replica, "replica %u >= n_replica %u", replica,
                  plan->n_replica);
        PSL_CHECK(out->x && out->y && out->z && out->u && out->v && out->w && out->e &&
                      out->hid && out->tag && out->count,
                  "particle stack has a null array");
        const bool plane = (flags & PSL_SAMPLE_PLANE) != 0;
        const bool dense = plane || (flags & PSL_SAMPLE_DENSE) != 0;
        PSL_CHECK(!dense || out->capacity >= n, "dense output needs capacity >= n");
        PSL_CHECK(dense || out->capacity >= n, "stack capacity must be >= n");
        PSL_CHECK(!plane || plane_beams_fit(plan), "plane records carry the beam in 8 bits: at most 255 beams");
        const auto b0 = std::upper_bound(plan->cum.begin(), plan->cum.end(), h0);
        const auto b1 = std::upper_bound(plan->cum.begin(), plan->cum.end(), h0 + n - 1);
        const int64_t jlo = b0 - plan->cum.begin(), jhi = (b1 - plan->cum.begin()) + 1;
        const int stype = plan->stype[size_t(jlo)];
        PSL_CHECK(plan->stype[size_t(jhi - 1)] == stype,
                  "histories [h0, h0+n) span more than one sub-source");
        for (int64_t j = jlo; j < jhi; ++j)
            PSL_CHECK(plan->stype[size_t(j)] == stype,
                      "histories [h0, h0+n) span more than one sub-source");
        out->ptype = stype == 2 ? 1 : 0;
        launch_sample(plan, phantom, replica, nullptr, h0, n, jlo, jhi, stype, seed, out,
                      plane ? 3 : dense ? 1 : 0, tally, static_cast<hipStream_t>(stream));
    });
}

extern "C" int psl_transform_batch(const psl_plan* plan, const psl_phantom* phantom,
                                   const psl_particles* plane, uint32_t n, psl_particles* out,
                                   psl_tally* tally, void* stream) {
    return guarded([&] {
        PSL_CHECK(plan && phantom && plane && out && tally, "psl_transform_batch: null argument");
        PSL_CHECK(n >= 1, "n must be >= 1");
        PSL_CHECK(plane->capacity >= n && out->capacity >= n, "stack capacities must be >= n");
        PSL_CHECK(plane->x && plane->y && plane->u && plane->v && plane->w && plane->e &&
                      plane->hid && plane->tag,
                  "plane stack has a null array");
        PSL_CHECK(out->x && out->y && out->z && out->u && out->v && out->w && out->e && out->hid &&
                      out->tag && out->count,
                  "particle stack has a null array");
        PSL_CHECK(plane->x != out->x && plane->tag != out->tag, "in-place transform not supported");
        PSL_CHECK(tally->phantom == phantom, "tally belongs to another phantom");
        ensure_device(plan);
        const psl_model& m = *plan->model;
        TransformArgs a{};
        a.x = plane->x; a.y = plane->y; a.u = plane->u; a.v = plane->v; a.w = plane->w;
        a.e = plane->e;
        a.hid = plane->hid;
        a.tag = plane->tag;
        a.n = n;
        a.zjy = float(m.d.z_jaw_y - m.d.z_plane);
        a.zjx = float(m.d.z_jaw_x - m.d.z_plane);
        a.beams = plan->d_beams.as<BeamDev>();
        a.n_beams = int(plan->beams.size());
        for (int k = 0; k < 3; ++k) {
            a.box_lo[k] = phantom->g.origin[k];
            a.box_hi[k] = phantom->g.hi[k];
        }
        a.ox = out->x; a.oy = out->y; a.oz = out->z;
        a.ou = out->u; a.ov = out->v; a.ow = out->w;
        a.oe = out->e;
        a.ohid = out->hid;
        a.otag = out->tag;
        a.ocount = out->count;
        a.stats = tally->dev().stats;
        out->ptype = plane->ptype;
        hipLaunchKernelGGL(k_transform, dim3((n + 255) / 256), dim3(256), 0,
                           static_cast<hipStream_t>(stream), a);
        PSL_HIP(hipGetLastError());
    });
}
