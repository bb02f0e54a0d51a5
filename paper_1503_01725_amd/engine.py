"""Python objects over the C ABI.  PyTorch provides device memory and streams;
every step of the dose path runs in libpsl's kernels."""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np
import torch

from . import _native as N


def _release(obj, free_fn):
    """Frees a library handle once; a no-op during interpreter shutdown, when
    the binding module may already be gone."""
    h = getattr(obj, "h", None)
    if h and N is not None and getattr(N, "lib", None) is not None:
        getattr(N.lib(), free_fn)(h)
    obj.h = None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _stream_ptr(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


class Model:
    """psl_build over a PSR model (any object with the fields of workloads.PsrModel)."""

    def __init__(self, m):
        self.src = m
        self._keep = [_f64(a) for a in (m.w_psr, m.sc_c, m.sc_mu, m.sc_sa, m.sc_sb)]
        w, c, mu, sa, sb = (a.ctypes.data_as(N.dp) for a in self._keep)
        self.desc = N.psl_psr_desc(m.n_ebin, m.n_ring, m.n_comp, m.n_psl, m.e_lo, m.e_width,
                                   m.ring_dr, m.psl_x0, m.psl_dx, m.z_target, m.z_plane,
                                   m.z_scatter, m.z_jaw_y, m.z_jaw_x, m.sigma_spot, m.sig_ea,
                                   m.sig_eb, w, c, mu, sa, sb)
        self.h = N.psl_build(self.desc)

    def weights(self) -> np.ndarray:
        m = self.src
        out = np.zeros((3, m.n_ebin, m.n_psl, m.n_psl))
        N.check(N.lib().psl_model_weights(self.h, out.ctypes.data_as(N.dp)))
        return out

    def __del__(self):
        try:
            _release(self, "psl_model_free")
        except TypeError:      # interpreter shutdown: module globals already cleared
            pass


def _beams(beams):
    arr = (N.psl_beam * len(beams))()
    for i, b in enumerate(beams):
        arr[i] = N.psl_beam(b.x1, b.x2, b.y1, b.y2, b.gantry_deg, b.couch_deg,
                            (C.c_double * 3)(*b.iso))
    return arr


@dataclass
class PlanList:
    beam: np.ndarray
    stype: np.ndarray
    ebin: np.ndarray
    ix: np.ndarray
    iy: np.ndarray
    tag: np.ndarray
    w: np.ndarray
    cum: np.ndarray

    @property
    def counts(self):
        return np.diff(np.concatenate([[0], self.cum])).astype(np.uint64)


class Plan:
    def __init__(self, model: Model, beams, n_hist, n_replica=1, basis_map=None,
                 hist_per_basis=0):
        self.model = model
        self.beams = list(beams)
        self._bm = None
        bptr = None
        if basis_map is not None:
            self._bm = np.ascontiguousarray(basis_map, dtype=np.uint16)
            bptr = self._bm.ctypes.data_as(N.u16p)
        self.h = N.psl_plan_create(model.h, _beams(self.beams), int(n_hist), int(n_replica),
                                   bptr, int(hist_per_basis))
        self.info = N.psl_plan_info()
        N.check(N.lib().psl_plan_get_info(self.h, C.byref(self.info)))

    @property
    def n_hist(self):
        return int(self.info.n_hist)

    @property
    def n_replica(self):
        return int(self.info.n_replica)

    @property
    def n_cols(self):
        return int(self.info.n_cols)

    def boxes(self) -> np.ndarray:
        out = np.zeros((len(self.beams), 3, 4), dtype=np.int32)
        N.check(N.lib().psl_plan_boxes(self.h, out.ctypes.data_as(N.i32p)))
        return out

    def list(self) -> PlanList:
        n = int(self.info.n_list)
        ints = [np.zeros(n, dtype=np.int32) for _ in range(6)]
        w = np.zeros(n)
        cum = np.zeros(n, dtype=np.uint64)
        N.check(N.lib().psl_plan_list(self.h, *[a.ctypes.data_as(N.i32p) for a in ints],
                                      w.ctypes.data_as(N.dp), cum.ctypes.data_as(N.u64p)))
        return PlanList(*ints, w, cum)

    def col_weight(self) -> np.ndarray:
        out = np.zeros(self.n_cols)
        N.check(N.lib().psl_plan_col_weight(self.h, out.ctypes.data_as(N.dp)))
        return out

    def set_batching(self, max_batch=131072, band_width=1) -> int:
        n = C.c_int64()
        N.check(N.lib().psl_plan_set_batching(self.h, max_batch, band_width, C.byref(n)))
        return n.value

    def batch(self, i) -> N.psl_batch:
        b = N.psl_batch()
        N.check(N.lib().psl_plan_get_batch(self.h, i, C.byref(b)))
        return b

    def __del__(self):
        try:
            _release(self, "psl_plan_free")
        except TypeError:      # interpreter shutdown: module globals already cleared
            pass


class Phantom:
    def __init__(self, ph, device="cuda"):
        self.src = ph
        self.density = torch.as_tensor(np.ascontiguousarray(ph.density, dtype=np.float32),
                                       device=device)
        nz, ny, nx = self.density.shape
        self.shape = (nz, ny, nx)
        self.h = N.psl_phantom_create(self.density.data_ptr(), nx, ny, nz, ph.vox, ph.origin)

    def __del__(self):
        try:
            _release(self, "psl_phantom_free")
        except TypeError:      # interpreter shutdown: module globals already cleared
            pass


class Tally:
    def __init__(self, phantom: Phantom, index_map=None, n_rows=0, n_cols=1):
        self.phantom = phantom
        self.imap = None
        if index_map is not None:
            self.imap = torch.as_tensor(np.ascontiguousarray(index_map, dtype=np.int32),
                                        device=phantom.density.device)
            self.cells = n_rows * n_cols
            self.shape = (n_rows, n_cols)
        else:
            self.cells = int(np.prod(phantom.shape))
            self.shape = phantom.shape
        self.h = N.psl_tally_create(phantom.h, self.imap.data_ptr() if self.imap is not None else 0,
                                    n_rows, n_cols)

    def op(self, ops, plan=None, stream=None):
        N.tally_dose(self.h, ops, plan.h if plan else None, 0, 0, _stream_ptr(stream))

    def finalize(self, plan, stream=None):
        dev = self.phantom.density.device
        dose = torch.zeros(self.cells, dtype=torch.float64, device=dev)
        sig = torch.zeros(self.cells, dtype=torch.float64, device=dev)
        N.tally_dose(self.h, N.PSL_TALLY_FINALIZE, plan.h, dose.data_ptr(), sig.data_ptr(),
                     _stream_ptr(stream))
        return dose.view(self.shape), sig.view(self.shape)

    def stats(self):
        led = np.zeros(8)
        cnt = np.zeros(N.N_COUNTERS, dtype=np.uint64)
        rc = N.lib().psl_tally_stats(self.h, led.ctypes.data_as(N.dp), cnt.ctypes.data_as(N.u64p))
        names_l = ("src", "jaw", "missed", "invalid", "esc_g", "esc_e", "dep", "e_path")
        names_c = ("hist", "entered", "wc_steps", "real", "e_pushed", "e_local", "e_steps",
                   "deposits", "esc_uncollided", "kahn_trials", "e_boundary", "guard", "overflow",
                   "folds", "photo", "rayleigh", "pair", "annihil", "moller", "brem", "capped")
        out = dict(zip(names_l, led.tolist())), dict(zip(names_c, cnt[:len(names_c)].tolist()))
        if rc != N.PSL_OK:
            raise N.PslError(rc, N.lib().psl_last_error().decode())
        return out

    def __del__(self):
        try:
            _release(self, "psl_tally_free")
        except TypeError:      # interpreter shutdown: module globals already cleared
            pass


class Particles:
    """A structure-of-arrays particle stack in device memory."""

    FIELDS = ("x", "y", "z", "u", "v", "w", "e")

    def __init__(self, capacity, device="cuda"):
        self.capacity = int(capacity)
        self.t = {f: torch.empty(self.capacity, dtype=torch.float32, device=device)
                  for f in self.FIELDS}
        self.t["hid"] = torch.empty(self.capacity, dtype=torch.int64, device=device)
        self.t["tag"] = torch.empty(self.capacity, dtype=torch.int32, device=device)
        self.t["count"] = torch.zeros(1, dtype=torch.int32, device=device)
        self.c = N.psl_particles(*[self.t[f].data_ptr() for f in self.FIELDS],
                                 self.t["hid"].data_ptr(), self.t["tag"].data_ptr(),
                                 self.t["count"].data_ptr(), self.capacity, 0)

    def zero_count(self):
        self.t["count"].zero_()

    def count(self) -> int:
        return int(self.t["count"].item())

    def host(self, n=None):
        n = self.count() if n is None else n
        out = {f: self.t[f][:n].cpu().numpy() for f in self.FIELDS}
        out["hid"] = self.t["hid"][:n].cpu().numpy().view(np.uint64)
        tag = self.t["tag"][:n].cpu().numpy().view(np.uint32)
        out["tag"] = tag & 0xFFFF
        out["sub"] = (tag >> 16) & 0xFF
        out["status"] = tag >> 24
        return out


def transport_params(e_cut_electron=0.2, e_cut_photon=0.01, step_frac=0.1, ms=True,
                     density_effect=False, physics=0):
    """psl_transport_params; physics: PSL_PHYS_* bits of the optional photon
    processes (photoelectric 1, Rayleigh 2, pair 4) and electron hard events
    (Moller delta rays 8, bremsstrahlung 16); 0 = the plain method."""
    return N.psl_transport_params(e_cut_electron, e_cut_photon, step_frac, 1 if ms else 0,
                                  1 if density_effect else 0, int(physics))


def electron_capacity(photon_capacity, e_max, e_cut_electron):
    """Electron stack size that can never overflow: a photon pays at least the
    electron cut-off for every electron it sets in motion, and one more entry
    per photon covers the unused ends of the per-wave chunks."""
    return int(photon_capacity * (max(1, int(np.floor(e_max / e_cut_electron))) + 1))


def run_plan_eager(plan: Plan, phantom: Phantom, tally: Tally, params, seed, max_batch=131072,
                   band_width=1, stream=None, replicas=None, reset=True):
    """Reference batch loop through the public calls (sample_batch ->
    transport_batch per batch, one FOLD per replica)."""
    nb = plan.set_batching(max_batch, band_width)
    e_cap = electron_capacity(max_batch, plan.info.e_max, params.e_cut_electron)
    ph_stack = Particles(max_batch)
    el_stack = Particles(e_cap)
    s = _stream_ptr(stream)
    if reset:
        tally.op(N.PSL_TALLY_RESET, stream=stream)
    reps = range(plan.n_replica) if replicas is None else replicas
    for r in reps:
        for i in range(nb):
            b = plan.batch(i)
            ph_stack.zero_count()
            N.sample_batch(plan.h, phantom.h, r, b.h0, b.n, seed, ph_stack.c, 0, tally.h, s)
            N.transport_batch(phantom.h, ph_stack.c, el_stack.c, tally.h, params, seed, s)
        tally.op(N.PSL_TALLY_FOLD, stream=stream)


def run_opts(max_batch=131072, band_width=1, use_graph=True, sort_electrons=True, timing=False,
             seed=0, lane_load=0, pipelines=0):
    """Options of psl_run; lane_load 0 = four histories per lane of the
    persistent transport grids; pipelines 0 = one batch pipeline."""
    return N.psl_run_opts(int(max_batch), int(band_width), 1 if use_graph else 0,
                          1 if sort_electrons else 0, 1 if timing else 0, int(seed),
                          int(lane_load), int(pipelines))


def run_plan(plan: Plan, phantom: Phantom, tally: Tally, params, opts, stream=None):
    """All batches of all replicas through the native runtime (psl_run)."""
    N.psl_run(plan.h, phantom.h, tally.h, params, opts, _stream_ptr(stream))


def autotune(plan: Plan, phantom: Phantom, tally: Tally, params, seed,
             max_batches=(65536, 131072, 262144, 524288), band_widths=(1, 2, 4), lane_loads=(4,)):
    """Fastest (max_batch, band_width, lane_load, sort, pipelines) by timing one
    replica; returns the options and the times [n_m, n_w, n_l, 2, 2] in ms."""
    return N.psl_autotune(plan.h, phantom.h, tally.h, params, seed, max_batches, band_widths,
                          lane_loads)


def commission_nnls(A, b, x0=None, delta=1e-10, pg_tol=1e-8, sigma=1e-4, beta=0.5,
                    max_iter=100000):
    """Eq. (8) by gradient projection + Armijo on the GPU (FP64)."""
    A = np.asfortranarray(A, dtype=np.float64)
    m, n = A.shape
    a_flat = np.ascontiguousarray(A.T).ravel()        # column-major storage
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.ones(n) if x0 is None else np.array(x0, dtype=np.float64)
    opts = N.psl_nnls_opts(delta, pg_tol, sigma, beta, max_iter)
    rep = N.psl_nnls_report()
    rc = N.commission_nnls(a_flat.ctypes.data_as(N.dp), m, n, b.ctypes.data_as(N.dp),
                           x.ctypes.data_as(N.dp), opts, rep)
    return x, dict(iters=int(rep.iters), f=rep.f, pg=rep.pg_norm, converged=rc == N.PSL_OK)


class UNet:
    """The 3D U-Net denoiser (psl_unet_*): c base channels, d x h x w volumes."""

    def __init__(self, c, d, h, w):
        self.c, self.shape = c, (d, h, w)
        out = C.c_void_p()
        N.check(N.lib().psl_unet_create(c, d, h, w, C.byref(out)))
        self.h = out
        n = C.c_int64()
        N.check(N.lib().psl_unet_param_count(self.h, C.byref(n)))
        self.n_params = n.value
        self.loss_parts = torch.zeros(64, dtype=torch.float64, device="cuda")

    def set_params(self, flat):
        flat = np.ascontiguousarray(flat, dtype=np.float32)
        assert flat.size == self.n_params
        N.check(N.lib().psl_unet_set_params(self.h, flat.ctypes.data_as(N.fp)))

    def get_params(self):
        out = np.zeros(self.n_params, dtype=np.float32)
        N.check(N.lib().psl_unet_get_params(self.h, out.ctypes.data_as(N.fp)))
        return out

    def forward(self, inp, stream=None):
        pred = torch.empty(self.shape, dtype=torch.float32, device="cuda")
        N.check(N.lib().psl_unet_forward(self.h, inp.data_ptr(), pred.data_ptr(),
                                         _stream_ptr(stream)))
        return pred

    def train_step(self, inp, tgt, lr, stream=None):
        N.check(N.lib().psl_unet_train_step(self.h, inp.data_ptr(), tgt.data_ptr(), lr,
                                            self.loss_parts.data_ptr(), _stream_ptr(stream)))
        return self.loss_parts

    def gradients(self, inp, tgt):
        g = np.zeros(self.n_params, dtype=np.float32)
        loss = C.c_double()
        N.check(N.lib().psl_unet_gradients(self.h, inp.data_ptr(), tgt.data_ptr(),
                                           g.ctypes.data_as(N.fp), C.byref(loss)))
        return g, loss.value

    def __del__(self):
        try:
            _release(self, "psl_unet_free")
        except TypeError:      # interpreter shutdown: module globals already cleared
            pass
