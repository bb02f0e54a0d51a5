"""ctypes front-end of the FP64 CPU oracle (oracle.c).

TEST INFRASTRUCTURE: only tests, the smoke check and the benchmark's CPU
baseline import this module.  It never imports the GPU package; inputs come
from the seeded generators in ``paper_1503_01725_amd.workloads`` (passed in by
the caller as plain numpy arrays / dataclasses).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

GCC_FLAGS = ["-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
             "-std=gnu11", "-Wall"]


def build(force: bool = False) -> str:
    """Compiles oracle.c into liboracle.so (FP64, no contraction, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", *GCC_FLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        _declare(_lib)
    return _lib


P = C.POINTER
dp = P(C.c_double)
fp = P(C.c_float)
i32p = P(C.c_int32)
u64p = P(C.c_uint64)
u32p = P(C.c_uint32)
u16p = P(C.c_uint16)


class OrModel(C.Structure):
    _fields_ = [("n_ebin", C.c_int32), ("n_ring", C.c_int32), ("n_comp", C.c_int32),
                ("n_psl", C.c_int32), ("e_lo", C.c_double), ("e_width", C.c_double),
                ("ring_dr", C.c_double), ("psl_x0", C.c_double), ("psl_dx", C.c_double),
                ("z_target", C.c_double), ("z_plane", C.c_double), ("z_scatter", C.c_double),
                ("z_jaw_y", C.c_double), ("z_jaw_x", C.c_double), ("sigma_spot", C.c_double),
                ("sig_ea", C.c_double), ("sig_eb", C.c_double), ("w_psr", dp), ("sc_c", dp),
                ("sc_mu", dp), ("sc_sa", dp), ("sc_sb", dp)]


class OrBeam(C.Structure):
    _fields_ = [("x1", C.c_double), ("x2", C.c_double), ("y1", C.c_double), ("y2", C.c_double),
                ("gantry_deg", C.c_double), ("couch_deg", C.c_double), ("iso", C.c_double * 3)]


class OrPhantom(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("pad", C.c_int32),
                ("vox", C.c_double * 3), ("origin", C.c_double * 3), ("density", fp)]


class OrParams(C.Structure):
    _fields_ = [("e_cut_e", C.c_double), ("e_cut_g", C.c_double), ("step_frac", C.c_double),
                ("ms_enable", C.c_int32), ("density_effect", C.c_int32), ("physics", C.c_int32)]


class OrPlan(C.Structure):
    _fields_ = [("n_list", C.c_int64), ("beam", i32p), ("stype", i32p), ("ebin", i32p),
                ("ix", i32p), ("iy", i32p), ("tag", i32p), ("cum", u64p), ("n_hist", C.c_uint64)]


SAMPLE_REC = np.dtype([("j", "i4"), ("k", "i4"), ("status", "i4"), ("stype", "i4"),
                       ("beam", "i4"), ("ebin", "i4"), ("ix", "i4"), ("iy", "i4"),
                       ("tag", "i4"), ("pad", "i4"), ("xb", "f8"), ("yb", "f8"),
                       ("ub", "f8"), ("vb", "f8"), ("wb", "f8"), ("e", "f8"),
                       ("xs", "f8"), ("ys", "f8"), ("alpha", "f8"), ("beta", "f8"),
                       ("jaw_margin", "f8"), ("box_margin", "f8"), ("ring_margin", "f8"), ("x", "f8"), ("y", "f8"),
                       ("z", "f8"), ("u", "f8"), ("v", "f8"), ("w", "f8")])

LEDGER = ("src", "jaw", "missed", "invalid", "esc_g", "esc_e", "dep", "e_path")
COUNTERS = ("hist", "entered", "wc_steps", "real", "e_pushed", "e_local", "e_steps",
            "deposits", "esc_uncollided", "kahn_trials", "e_boundary", "guard", "overflow",
            "folds", "photo", "rayleigh", "pair", "annihil", "moller", "brem", "capped")
N_COUNTERS = 24
# optional photon processes (bits of params(physics=...))
PHYS_PHOTO, PHYS_RAYLEIGH, PHYS_PAIR = 1, 2, 4
# optional electron hard events: Moller delta rays, bremsstrahlung photons
PHYS_DELTA, PHYS_BREM = 8, 16
GEN_MAX = 3
ST_OK, ST_JAW, ST_MISSED, ST_INVALID = 0, 1, 2, 3


def _declare(L):
    L.or_philox4x32_10.argtypes = [u32p, u32p, u32p]
    L.or_stream_uniforms.argtypes = [C.c_uint64, C.c_uint64, C.c_uint32, C.c_uint32, C.c_int, dp]
    L.or_psl_build.argtypes = [P(OrModel), dp]
    L.or_psl_build.restype = C.c_double
    L.or_scatter_cdf.argtypes = [P(OrModel), dp]
    L.or_sampling_box.argtypes = [P(OrModel), P(OrBeam), C.c_int, i32p]
    L.or_plan_build.argtypes = [P(OrModel), dp, P(OrBeam), C.c_int, C.c_uint64, u16p, C.c_int32,
                                C.c_uint64, C.c_int64, i32p, i32p, i32p, i32p, i32p, i32p, dp,
                                u64p, dp, u64p]
    L.or_plan_build.restype = C.c_int64
    L.or_kn_sigma.argtypes = [C.c_double]
    L.or_kn_sigma.restype = C.c_double
    L.or_kn_sample_cos.argtypes = [C.c_double, C.c_uint64, C.c_int, dp]
    for name in ("or_sigma_pair_z2", "or_mu_pair", "or_mu_photo", "or_mu_rayleigh",
                 "or_sigma_rayleigh", "or_ff2_water", "or_ff2_cumulative"):
        getattr(L, name).argtypes = [C.c_double]
        getattr(L, name).restype = C.c_double
    L.or_sigma_k_electron.argtypes = [C.c_double, C.c_double]
    L.or_sigma_k_electron.restype = C.c_double
    L.or_photo_binding.argtypes = []
    L.or_photo_binding.restype = C.c_double
    L.or_mu_total.argtypes = [C.c_double, C.c_int32, dp]
    L.or_mu_total.restype = C.c_double
    L.or_rayleigh_sample_cos.argtypes = [C.c_double, C.c_uint64, C.c_int, dp]
    L.or_pair_share_sample.argtypes = [C.c_uint64, C.c_int, dp]
    L.or_moller_dsig.argtypes = [C.c_double, C.c_double]
    L.or_moller_dsig.restype = C.c_double
    L.or_moller_sigma.argtypes = [C.c_double, C.c_double]
    L.or_moller_sigma.restype = C.c_double
    L.or_s_col_restricted.argtypes = [C.c_double, C.c_double, C.c_int]
    L.or_s_col_restricted.restype = C.c_double
    L.or_brem_kdsig.argtypes = [C.c_double, C.c_double]
    L.or_brem_kdsig.restype = C.c_double
    L.or_brem_sigma.argtypes = [C.c_double, C.c_double]
    L.or_brem_sigma.restype = C.c_double
    L.or_brem_soft.argtypes = [C.c_double, C.c_double]
    L.or_brem_soft.restype = C.c_double
    L.or_moller_sample.argtypes = [C.c_double, C.c_double, C.c_uint64, C.c_int, dp]
    L.or_moller_sample.restype = None
    L.or_brem_sample.argtypes = [C.c_double, C.c_double, C.c_uint64, C.c_int, dp]
    L.or_brem_sample.restype = None
    L.or_child_id.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32,
                              P(C.c_uint64), P(C.c_uint32)]
    L.or_child_id.restype = None
    L.or_range_p.argtypes = [C.c_double, C.c_double, C.c_int, C.c_int, C.c_double]
    L.or_range_p.restype = C.c_double
    L.or_range_inv_p.argtypes = [C.c_double, C.c_double, C.c_int, C.c_int, C.c_double]
    L.or_range_inv_p.restype = C.c_double
    L.or_s_cont.argtypes = [C.c_double, C.c_double, C.c_int, C.c_int, C.c_double]
    L.or_s_cont.restype = C.c_double
    L.or_s_col.argtypes = [C.c_double]
    L.or_s_col.restype = C.c_double
    L.or_s_col_d.argtypes = [C.c_double, C.c_int]
    L.or_s_col_d.restype = C.c_double
    L.or_density_delta.argtypes = [C.c_double]
    L.or_density_delta.restype = C.c_double
    L.or_range_d.argtypes = [C.c_double, C.c_double, C.c_int]
    L.or_range_d.restype = C.c_double
    L.or_range_inv_d.argtypes = [C.c_double, C.c_double, C.c_int]
    L.or_range_inv_d.restype = C.c_double
    L.or_range.argtypes = [C.c_double, C.c_double]
    L.or_range.restype = C.c_double
    L.or_range_inv.argtypes = [C.c_double, C.c_double]
    L.or_range_inv.restype = C.c_double
    L.or_highland.argtypes = [C.c_double, C.c_double]
    L.or_highland.restype = C.c_double
    L.or_ms_sample.argtypes = [C.c_double, C.c_uint64, C.c_int, dp]
    L.or_ms_width.argtypes = [C.c_double, C.c_double, C.c_double]
    L.or_ms_width.restype = C.c_double
    L.or_rotate_direction.argtypes = [dp, C.c_double, C.c_double, dp]
    L.or_compton.argtypes = [C.c_double, dp, C.c_double, C.c_double, dp]
    L.or_run.argtypes = [P(OrModel), P(OrPlan), P(OrBeam), C.c_int, P(OrPhantom), P(OrParams),
                         C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint64, C.c_uint64, C.c_uint64,
                         i32p, C.c_int64, C.c_int64, dp, dp, dp, u64p, C.c_int]
    L.or_sample.argtypes = [P(OrModel), P(OrPlan), P(OrBeam), C.c_int, P(OrPhantom), C.c_uint64,
                            C.c_uint64, C.c_int64, C.c_void_p]
    L.or_transport.argtypes = [P(OrPhantom), P(OrParams), C.c_uint64, C.c_int64, i32p, dp, dp, dp,
                               u64p, i32p, i32p, C.c_int64, C.c_int64, dp, dp, u64p, C.c_int]
    L.or_finalize.argtypes = [P(OrPhantom), dp, dp, C.c_uint32, C.c_double, dp, dp]
    L.or_nnls_gp.argtypes = [dp, C.c_int64, C.c_int64, dp, dp, C.c_double, C.c_double, C.c_double,
                             C.c_double, C.c_int64, dp]
    L.or_nnls_gp.restype = C.c_int


def _ptr(a, t):
    return a.ctypes.data_as(t)


# --------------------------------------------------------------------------
# Wrapping of the seeded inputs (duck-typed: any object with the fields of
# workloads.PsrModel / Beam / Phantom works).
# --------------------------------------------------------------------------
class Model:
    """Keeps the numpy buffers alive together with the C struct."""

    def __init__(self, m):
        self.src = m
        self._keep = [np.ascontiguousarray(a, dtype=np.float64)
                      for a in (m.w_psr, m.sc_c, m.sc_mu, m.sc_sa, m.sc_sb)]
        w, c, mu, sa, sb = self._keep
        self.c = OrModel(m.n_ebin, m.n_ring, m.n_comp, m.n_psl, m.e_lo, m.e_width, m.ring_dr,
                         m.psl_x0, m.psl_dx, m.z_target, m.z_plane, m.z_scatter, m.z_jaw_y,
                         m.z_jaw_x, m.sigma_spot, m.sig_ea, m.sig_eb, _ptr(w, dp), _ptr(c, dp),
                         _ptr(mu, dp), _ptr(sa, dp), _ptr(sb, dp))


def beams_array(beams):
    arr = (OrBeam * len(beams))()
    for i, b in enumerate(beams):
        arr[i] = OrBeam(b.x1, b.x2, b.y1, b.y2, b.gantry_deg, b.couch_deg,
                        (C.c_double * 3)(*b.iso))
    return arr


class Phantom:
    def __init__(self, ph):
        self.src = ph
        self.dens = np.ascontiguousarray(ph.density, dtype=np.float32)
        nz, ny, nx = self.dens.shape
        self.c = OrPhantom(nx, ny, nz, 0, (C.c_double * 3)(*ph.vox),
                           (C.c_double * 3)(*ph.origin), _ptr(self.dens, fp))
        self.n_vox = nx * ny * nz


def params(e_cut_e=0.2, e_cut_g=0.01, step_frac=0.1, ms=True, density_effect=False, physics=0):
    return OrParams(e_cut_e, e_cut_g, step_frac, 1 if ms else 0, 1 if density_effect else 0,
                    int(physics))


def philox(ctr, key):
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().or_philox4x32_10(_ptr(c, u32p), _ptr(k, u32p), _ptr(out, u32p))
    return out


def stream_uniforms(seed, g, tag, sub, n):
    out = np.zeros(n)
    lib().or_stream_uniforms(seed, g, tag, sub, n, _ptr(out, dp))
    return out


def psl_build(model):
    M = Model(model)
    w = np.zeros((3, model.n_ebin, model.n_psl, model.n_psl))
    total = lib().or_psl_build(C.byref(M.c), _ptr(w, dp))
    return w, total


def scatter_cdf(model):
    M = Model(model)
    P_ = np.zeros((model.n_ebin, model.n_ring, model.n_comp))
    lib().or_scatter_cdf(C.byref(M.c), _ptr(P_, dp))
    return P_


def sampling_box(model, beam, stype):
    M = Model(model)
    b = beams_array([beam])
    box = np.zeros(4, dtype=np.int32)
    lib().or_sampling_box(C.byref(M.c), b, stype, _ptr(box, i32p))
    return tuple(int(v) for v in box)


@dataclass
class Plan:
    beam: np.ndarray
    stype: np.ndarray
    ebin: np.ndarray
    ix: np.ndarray
    iy: np.ndarray
    tag: np.ndarray
    w: np.ndarray
    cum: np.ndarray
    group_w: np.ndarray
    group_n: np.ndarray
    n_hist: int

    @property
    def counts(self):
        return np.diff(np.concatenate([[0], self.cum])).astype(np.uint64)

    def c_struct(self):
        return OrPlan(len(self.cum), _ptr(self.beam, i32p), _ptr(self.stype, i32p),
                      _ptr(self.ebin, i32p), _ptr(self.ix, i32p), _ptr(self.iy, i32p),
                      _ptr(self.tag, i32p), _ptr(self.cum, u64p), self.n_hist)


def plan_build(model, w_psl, beams, n_hist, basis_map=None, hist_per_basis=0):
    M = Model(model)
    b = beams_array(beams)
    max_list = len(beams) * 3 * model.n_ebin * model.n_psl * model.n_psl
    arrs = [np.zeros(max_list, dtype=np.int32) for _ in range(6)]
    w = np.zeros(max_list)
    cum = np.zeros(max_list, dtype=np.uint64)
    n_basis = int(basis_map.max()) + 1 if basis_map is not None else 1
    groups = len(beams) * n_basis
    gw = np.zeros(groups)
    gn = np.zeros(groups, dtype=np.uint64)
    bm = None if basis_map is None else np.ascontiguousarray(basis_map, dtype=np.uint16)
    w_psl = np.ascontiguousarray(w_psl, dtype=np.float64)
    n = lib().or_plan_build(C.byref(M.c), _ptr(w_psl, dp), b, len(beams), n_hist,
                            None if bm is None else _ptr(bm, u16p), n_basis, hist_per_basis,
                            max_list, *[_ptr(a, i32p) for a in arrs], _ptr(w, dp),
                            _ptr(cum, u64p), _ptr(gw, dp), _ptr(gn, u64p))
    if n < 0:
        raise RuntimeError("plan list overflow")
    n = int(n)
    total = int(cum[n - 1]) if n else 0
    return Plan(*[a[:n].copy() for a in arrs], w[:n].copy(), cum[:n].copy(), gw, gn, total)


def sample(model, plan, beams, phantom, seed, g0, n):
    M = Model(model)
    b = beams_array(beams)
    ph = Phantom(phantom)
    pc = plan.c_struct()
    out = np.zeros(n, dtype=SAMPLE_REC)
    lib().or_sample(C.byref(M.c), C.byref(pc), b, len(beams), C.byref(ph.c), seed, g0, n,
                    out.ctypes.data_as(C.c_void_p))
    return out


def run(model, plan, beams, phantom, seed, n_rep, h0=0, h1=None, rep0=0, tparams=None,
        index_map=None, n_rows=0, n_cols=0, n_threads=0, stride=1):
    """Samples and transports histories; returns (sum, sum2, ledger, counters)."""
    M = Model(model)
    b = beams_array(beams)
    ph = Phantom(phantom)
    pc = plan.c_struct()
    tp = tparams or params()
    h1 = plan.n_hist if h1 is None else h1
    if index_map is not None:
        imap = np.ascontiguousarray(index_map, dtype=np.int32)
        cells = n_rows * n_cols
    else:
        imap = None
        cells = ph.n_vox
    s = np.zeros(cells)
    s2 = np.zeros(cells)
    led = np.zeros(8)
    cnt = np.zeros(N_COUNTERS, dtype=np.uint64)
    rc = lib().or_run(C.byref(M.c), C.byref(pc), b, len(beams), C.byref(ph.c), C.byref(tp),
                      seed, rep0, n_rep, h0, h1, stride, None if imap is None else _ptr(imap, i32p),
                      n_rows, n_cols, _ptr(s, dp), _ptr(s2, dp), _ptr(led, dp),
                      _ptr(cnt, u64p), n_threads)
    if rc != 0:
        raise RuntimeError("or_run failed")
    return s, s2, dict(zip(LEDGER, led)), dict(zip(COUNTERS, cnt[:len(COUNTERS)].tolist()))


def transport(phantom, seed, ptype, pos, dirs, e, hid, tag=None, tparams=None,
              index_map=None, n_rows=0, n_cols=0, n_threads=0):
    ph = Phantom(phantom)
    tp = tparams or params()
    n = len(e)
    ptype = np.ascontiguousarray(ptype, dtype=np.int32)
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    dirs = np.ascontiguousarray(dirs, dtype=np.float64)
    e = np.ascontiguousarray(e, dtype=np.float64)
    hid = np.ascontiguousarray(hid, dtype=np.uint64)
    tg = None if tag is None else np.ascontiguousarray(tag, dtype=np.int32)
    if index_map is not None:
        imap = np.ascontiguousarray(index_map, dtype=np.int32)
        cells = n_rows * n_cols
    else:
        imap = None
        cells = ph.n_vox
    edep = np.zeros(cells)
    led = np.zeros(8)
    cnt = np.zeros(N_COUNTERS, dtype=np.uint64)
    lib().or_transport(C.byref(ph.c), C.byref(tp), seed, n, _ptr(ptype, i32p), _ptr(pos, dp),
                       _ptr(dirs, dp), _ptr(e, dp), _ptr(hid, u64p),
                       None if tg is None else _ptr(tg, i32p),
                       None if imap is None else _ptr(imap, i32p), n_rows, n_cols,
                       _ptr(edep, dp), _ptr(led, dp), _ptr(cnt, u64p), n_threads)
    return edep, dict(zip(LEDGER, led)), dict(zip(COUNTERS, cnt[:len(COUNTERS)].tolist()))


def finalize(phantom, s, s2, n_rep, weight_per_history):
    ph = Phantom(phantom)
    dose = np.zeros(ph.n_vox)
    sig = np.zeros(ph.n_vox)
    lib().or_finalize(C.byref(ph.c), _ptr(np.ascontiguousarray(s), dp),
                      _ptr(np.ascontiguousarray(s2), dp), n_rep, weight_per_history,
                      _ptr(dose, dp), _ptr(sig, dp))
    return dose, sig


def kn_sigma(e):
    return lib().or_kn_sigma(e)


def kn_sample_cos(e, seed, n):
    out = np.zeros(n)
    lib().or_kn_sample_cos(e, seed, n, _ptr(out, dp))
    return out


def s_col(t, density_effect=False):
    """Mass collision stopping power of water, MeV cm^2/g (Bethe, ICRU 37 form;
    less the density-effect term when density_effect is set)."""
    return lib().or_s_col_d(t, 1 if density_effect else 0)


def density_delta(t):
    """Sternheimer density-effect correction delta(T) of liquid water."""
    return lib().or_density_delta(t)


def csda_range(t, t_cut=0.2, density_effect=False):
    return lib().or_range_d(t, t_cut, 1 if density_effect else 0)


def csda_range_inv(r, t_cut=0.2, density_effect=False):
    return lib().or_range_inv_d(r, t_cut, 1 if density_effect else 0)


def highland(t, t_x):
    return lib().or_highland(t, t_x)


def ms_width(t_mid, rho, s):
    """Highland width of one electron step (s cm at density rho, mean energy t_mid)."""
    return lib().or_ms_width(t_mid, rho, s)


def rotate_direction(d, cos_t, phi):
    """The transport's direction rotation applied to a copy of d."""
    d = np.ascontiguousarray(d, dtype=np.float64)
    out = np.zeros(3)
    lib().or_rotate_direction(_ptr(d, dp), cos_t, phi, _ptr(out, dp))
    return out


def compton(e, d, x, phi):
    """Compton kinematics for x = E/E' and azimuth phi: (E', T, photon dir, electron dir)."""
    d = np.ascontiguousarray(d, dtype=np.float64)
    out = np.zeros(8)
    lib().or_compton(e, _ptr(d, dp), x, phi, _ptr(out, dp))
    return out[0], out[1], out[2:5].copy(), out[5:8].copy()


def ms_sample(theta0, seed, n):
    out = np.zeros(n)
    lib().or_ms_sample(theta0, seed, n, _ptr(out, dp))
    return out


def nnls_gp(A, b, x0=None, delta=1e-10, pg_tol=1e-8, sigma=1e-4, beta=0.5, max_iter=100000):
    A = np.asfortranarray(A, dtype=np.float64)
    m, n = A.shape
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.ones(n) if x0 is None else np.array(x0, dtype=np.float64)
    rep = np.zeros(4)
    Aflat = np.ascontiguousarray(A.T).ravel()   # column-major storage
    lib().or_nnls_gp(_ptr(Aflat, dp), m, n, _ptr(b, dp), _ptr(x, dp), delta, pg_tol, sigma, beta,
                     max_iter, _ptr(rep, dp))
    return x, dict(iters=int(rep[0]), f=rep[1], pg=rep[2], converged=bool(rep[3]))


# --------------------------------------------------------------------------
# Optional photon processes (test hooks)
# --------------------------------------------------------------------------
def sigma_k_electron(e, z):
    """Stobbe photoeffect cross-section of one hydrogenic K electron (cm^2)."""
    return lib().or_sigma_k_electron(e, z)


def photo_binding():
    return lib().or_photo_binding()


def mu_photo(e):
    return lib().or_mu_photo(e)


def ff2_water(t):
    return lib().or_ff2_water(t)


def ff2_cumulative(t):
    return lib().or_ff2_cumulative(t)


def sigma_rayleigh(e):
    return lib().or_sigma_rayleigh(e)


def mu_rayleigh(e):
    return lib().or_mu_rayleigh(e)


def sigma_pair_z2(e):
    return lib().or_sigma_pair_z2(e)


def mu_pair(e):
    return lib().or_mu_pair(e)


def mu_total(e, physics):
    """Attenuation per unit density (cm^2/g) and its parts (Compton,
    photoelectric, Rayleigh, pair)."""
    parts = np.zeros(4)
    tot = lib().or_mu_total(e, physics, _ptr(parts, dp))
    return tot, parts


def moller_dsig(t, w):
    """Moller d sigma / dW per target electron (cm^2/MeV)."""
    return lib().or_moller_dsig(t, w)


def moller_sigma(t, tc):
    """Hard Moller collisions (W >= tc) per gram of water (cm^2/g)."""
    return lib().or_moller_sigma(t, tc)


def s_col_restricted(t, tc, density_effect=False):
    return lib().or_s_col_restricted(t, tc, 1 if density_effect else 0)


def brem_kdsig(t, k):
    """k d sigma / dk of bremsstrahlung in water (cm^2/g), formula 3BN."""
    return lib().or_brem_kdsig(t, k)


def brem_sigma(t, kc):
    return lib().or_brem_sigma(t, kc)


def brem_soft(t, kc):
    return lib().or_brem_soft(t, kc)


def moller_sample(t, tc, seed, n):
    out = np.zeros(n)
    lib().or_moller_sample(t, tc, seed, n, _ptr(out, dp))
    return out


def brem_sample(t, kc, seed, n):
    out = np.zeros(n)
    lib().or_brem_sample(t, kc, seed, n, _ptr(out, dp))
    return out


def child_id(g, sub, j, kind):
    go, so = C.c_uint64(), C.c_uint32()
    lib().or_child_id(g, sub, j, kind, C.byref(go), C.byref(so))
    return go.value, so.value


def range_p(t, t_cut, physics, kc, density_effect=False):
    return lib().or_range_p(t, t_cut, 1 if density_effect else 0, int(physics), kc)


def range_inv_p(rr, t_cut, physics, kc, density_effect=False):
    return lib().or_range_inv_p(rr, t_cut, 1 if density_effect else 0, int(physics), kc)


def s_cont(t, t_cut, physics, kc, density_effect=False):
    """The continuous stopping power the range tables integrate (MeV cm^2/g)."""
    return lib().or_s_cont(t, t_cut, 1 if density_effect else 0, int(physics), kc)


def rayleigh_sample_cos(e, seed, n):
    out = np.zeros(n)
    lib().or_rayleigh_sample_cos(e, seed, n, _ptr(out, dp))
    return out


def pair_share_sample(seed, n):
    out = np.zeros(n)
    lib().or_pair_share_sample(seed, n, _ptr(out, dp))
    return out
