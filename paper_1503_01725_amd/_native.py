"""ctypes binding of libpsl.so (include/psl.h): argument marshalling only.

Every function here has the name of the C entry point it calls and raises
``PslError`` on a non-zero status.  There is no fallback: if the library is
missing the import fails loudly.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpsl.so")

PSL_OK, PSL_EINVAL, PSL_ENOMEM, PSL_EDEVICE, PSL_EOVERFLOW, PSL_ENOTCONV = 0, -1, -2, -3, -4, -5
PSL_SAMPLE_DENSE = 1
PSL_SAMPLE_PLANE = 2
PSL_TALLY_RESET, PSL_TALLY_FOLD, PSL_TALLY_FINALIZE = 1, 2, 4

P = C.POINTER
dp, fp = P(C.c_double), P(C.c_float)
i32p, u16p, u32p, u64p = P(C.c_int32), P(C.c_uint16), P(C.c_uint32), P(C.c_uint64)
vp = C.c_void_p


class PslError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"[{code}] {msg}")
        self.code = code


class psl_psr_desc(C.Structure):
    _fields_ = [("n_ebin", C.c_int32), ("n_ring", C.c_int32), ("n_comp", C.c_int32),
                ("n_psl", C.c_int32), ("e_lo", C.c_double), ("e_width", C.c_double),
                ("ring_dr", C.c_double), ("psl_x0", C.c_double), ("psl_dx", C.c_double),
                ("z_target", C.c_double), ("z_plane", C.c_double), ("z_scatter", C.c_double),
                ("z_jaw_y", C.c_double), ("z_jaw_x", C.c_double), ("sigma_spot", C.c_double),
                ("sig_ea", C.c_double), ("sig_eb", C.c_double), ("w_psr", dp), ("sc_c", dp),
                ("sc_mu", dp), ("sc_sa", dp), ("sc_sb", dp)]


class psl_beam(C.Structure):
    _fields_ = [("x1", C.c_double), ("x2", C.c_double), ("y1", C.c_double), ("y2", C.c_double),
                ("gantry_deg", C.c_double), ("couch_deg", C.c_double), ("iso", C.c_double * 3)]


class psl_plan_info(C.Structure):
    _fields_ = [("n_hist", C.c_uint64), ("n_replica", C.c_uint32), ("n_beams", C.c_int32),
                ("n_list", C.c_int64), ("n_cols", C.c_int32), ("s_area", C.c_double),
                ("e_max", C.c_double)]


class psl_batch(C.Structure):
    _fields_ = [("h0", C.c_uint64), ("n", C.c_uint32), ("stype", C.c_int32),
                ("beam", C.c_int32), ("band", C.c_int32)]


class psl_particles(C.Structure):
    _fields_ = [("x", vp), ("y", vp), ("z", vp), ("u", vp), ("v", vp), ("w", vp), ("e", vp),
                ("hid", vp), ("tag", vp), ("count", vp), ("capacity", C.c_uint32),
                ("ptype", C.c_int32)]


class psl_transport_params(C.Structure):
    _fields_ = [("e_cut_electron", C.c_float), ("e_cut_photon", C.c_float),
                ("step_frac", C.c_float), ("ms_enable", C.c_int32),
                ("density_effect", C.c_int32), ("physics", C.c_uint32)]


# optional photon processes (psl_transport_params.physics)
PSL_PHYS_PHOTO, PSL_PHYS_RAYLEIGH, PSL_PHYS_PAIR = 1, 2, 4
PSL_PHYS_DELTA, PSL_PHYS_BREM = 8, 16
N_COUNTERS = 24


class psl_run_opts(C.Structure):
    _fields_ = [("max_batch", C.c_uint32), ("band_width", C.c_int32), ("use_graph", C.c_int32),
                ("sort_electrons", C.c_int32), ("timing", C.c_int32), ("seed", C.c_uint64),
                ("lane_load", C.c_int32), ("pipelines", C.c_int32)]


class psl_run_timing(C.Structure):
    _fields_ = [("ms", C.c_double * 5), ("launches", C.c_uint64 * 5)]


PHASES = ("sample", "photon", "sort", "electron", "fold")


class psl_nnls_opts(C.Structure):
    _fields_ = [("delta", C.c_double), ("pg_tol", C.c_double), ("armijo_sigma", C.c_double),
                ("armijo_beta", C.c_double), ("max_iter", C.c_int64)]


class psl_nnls_report(C.Structure):
    _fields_ = [("iters", C.c_int64), ("f", C.c_double), ("pg_norm", C.c_double)]


# name -> argtypes (restype int unless listed in _RESTYPE)
_SIGS = {
    "psl_last_error": [],
    "psl_build": [P(psl_psr_desc), P(vp)],
    "psl_model_weights": [vp, dp],
    "psl_model_free": [vp],
    "psl_plan_create": [vp, P(psl_beam), C.c_int32, C.c_uint64, C.c_uint32, u16p, C.c_uint64,
                        P(vp)],
    "psl_plan_get_info": [vp, P(psl_plan_info)],
    "psl_plan_boxes": [vp, i32p],
    "psl_plan_list": [vp, i32p, i32p, i32p, i32p, i32p, i32p, dp, u64p],
    "psl_plan_col_weight": [vp, dp],
    "psl_plan_set_batching": [vp, C.c_uint32, C.c_int32, P(C.c_int64)],
    "psl_plan_get_batch": [vp, C.c_int64, P(psl_batch)],
    "psl_plan_free": [vp],
    "psl_phantom_create": [vp, C.c_int32, C.c_int32, C.c_int32, dp, dp, P(vp)],
    "psl_phantom_free": [vp],
    "sample_batch": [vp, vp, C.c_uint32, C.c_uint64, C.c_uint32, C.c_uint64, P(psl_particles),
                     C.c_uint32, vp, vp],
    "psl_transform_batch": [vp, vp, P(psl_particles), C.c_uint32, P(psl_particles), vp, vp],
    "psl_tally_create": [vp, vp, C.c_int32, C.c_int32, P(vp)],
    "psl_tally_free": [vp],
    "transport_batch": [vp, P(psl_particles), P(psl_particles), vp, P(psl_transport_params),
                        C.c_uint64, vp],
    "tally_dose": [vp, C.c_int32, vp, vp, vp, vp],
    "psl_tally_stats": [vp, dp, u64p],
    "psl_tally_record": [vp, vp, C.c_uint32, vp],
}
_RESTYPE = {"psl_last_error": C.c_char_p, "psl_model_free": None, "psl_plan_free": None,
            "psl_phantom_free": None, "psl_tally_free": None}
_SIGS.update({
    "commission_nnls": [dp, C.c_int64, C.c_int64, dp, dp, P(psl_nnls_opts), P(psl_nnls_report)],
    "commission_nnls_noalloc": [vp, C.c_int64, C.c_int64, vp, vp, P(psl_nnls_opts),
                                P(psl_nnls_report), vp],
    "psl_run": [vp, vp, vp, P(psl_transport_params), P(psl_run_opts), vp],
    "psl_run_get_timing": [vp, P(psl_run_timing)],
    "psl_autotune": [vp, vp, vp, P(psl_transport_params), C.c_uint64, u32p, C.c_int32, i32p,
                     C.c_int32, i32p, C.c_int32, C.c_uint32, P(psl_run_opts), dp],
})
_SIGS.update({
    "psl_probe_atomics": [vp, C.c_int64, vp, C.c_int64, C.c_int32, dp],
    "psl_probe_copy": [vp, vp, C.c_int64, C.c_int32, dp],
})
_SIGS.update({
    "psl_unet_create": [C.c_int32, C.c_int32, C.c_int32, C.c_int32, P(vp)],
    "psl_unet_free": [vp],
    "psl_unet_param_count": [vp, P(C.c_int64)],
    "psl_unet_set_params": [vp, fp],
    "psl_unet_get_params": [vp, fp],
    "psl_unet_forward": [vp, vp, vp, vp],
    "psl_unet_train_step": [vp, vp, vp, C.c_float, vp, vp],
    "psl_unet_gradients": [vp, vp, vp, fp, dp],
    "psl_dose_gate": [vp, vp, vp, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_double, dp,
                      vp],
})
_RESTYPE["psl_unet_free"] = None
_OPTIONAL = {}

_lib = None


def lib() -> C.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_1503_01725_amd.build` (no CPU fallback exists)")
        # PyTorch ships its own HIP runtime under the same soname as the
        # system one libpsl.so links; loading torch first makes the library
        # bind to that already-loaded runtime, so that one runtime serves the
        # tensors the caller allocates and the library's own calls.
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        for name, args in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = _RESTYPE.get(name, C.c_int)
        for name, args in _OPTIONAL.items():
            if args is not None and hasattr(L, name):
                f = getattr(L, name)
                f.argtypes = args
                f.restype = C.c_int
        _lib = L
    return _lib


def check(rc: int) -> int:
    if rc != PSL_OK:
        raise PslError(rc, lib().psl_last_error().decode())
    return rc


def exported_symbols():
    """Names of every function declared in include/psl.h."""
    import re
    hdr = os.path.join(os.path.dirname(_HERE), "include", "psl.h")
    text = open(hdr).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(?:int|void|const char\*)\s+(\w+)\s*\(", text)))


def _call(name, *args):
    return check(getattr(lib(), name)(*args))


# Same-named thin wrappers --------------------------------------------------
def psl_build(desc):
    out = vp()
    _call("psl_build", C.byref(desc), C.byref(out))
    return out


def psl_plan_create(model, beams, n_hist, n_replica, basis_map_ptr, hist_per_basis):
    out = vp()
    _call("psl_plan_create", model, beams, len(beams), n_hist, n_replica, basis_map_ptr,
          hist_per_basis, C.byref(out))
    return out


def psl_phantom_create(density_ptr, nx, ny, nz, vox, origin):
    out = vp()
    _call("psl_phantom_create", vp(density_ptr), nx, ny, nz, (C.c_double * 3)(*vox),
          (C.c_double * 3)(*origin), C.byref(out))
    return out


def psl_tally_create(phantom, index_map_ptr, n_rows, n_cols):
    out = vp()
    _call("psl_tally_create", phantom, vp(index_map_ptr) if index_map_ptr else None, n_rows,
          n_cols, C.byref(out))
    return out


def sample_batch(plan, phantom, replica, h0, n, seed, particles, flags, tally, stream):
    return _call("sample_batch", plan, phantom, replica, h0, n, seed, C.byref(particles), flags,
                 tally, vp(stream))


def psl_transform_batch(plan, phantom, plane, n, out, tally, stream):
    return _call("psl_transform_batch", plan, phantom, C.byref(plane), n, C.byref(out), tally,
                 vp(stream))


def transport_batch(phantom, particles, electrons, tally, params, seed, stream):
    return _call("transport_batch", phantom, C.byref(particles), C.byref(electrons), tally,
                 C.byref(params), seed, vp(stream))


def tally_dose(tally, ops, plan, dose_ptr, sigma_ptr, stream):
    return _call("tally_dose", tally, ops, plan, vp(dose_ptr) if dose_ptr else None,
                 vp(sigma_ptr) if sigma_ptr else None, vp(stream))


def psl_run(plan, phantom, tally, params, opts, stream):
    return _call("psl_run", plan, phantom, tally, C.byref(params), C.byref(opts), vp(stream))


def psl_run_get_timing(tally):
    t = psl_run_timing()
    _call("psl_run_get_timing", tally, C.byref(t))
    return {p: (t.ms[i], int(t.launches[i])) for i, p in enumerate(PHASES)}


def psl_autotune(plan, phantom, tally, params, seed, max_batches, band_widths, lane_loads=(4,),
                 replica=0):
    import numpy as np
    mb = np.ascontiguousarray(max_batches, dtype=np.uint32)
    bw = np.ascontiguousarray(band_widths, dtype=np.int32)
    ll = np.ascontiguousarray(lane_loads, dtype=np.int32)
    ms = np.zeros(len(mb) * len(bw) * len(ll) * 2 * 2)
    best = psl_run_opts()
    _call("psl_autotune", plan, phantom, tally, C.byref(params), seed, mb.ctypes.data_as(u32p),
          len(mb), bw.ctypes.data_as(i32p), len(bw), ll.ctypes.data_as(i32p), len(ll), replica,
          C.byref(best), ms.ctypes.data_as(dp))
    return best, ms.reshape(len(mb), len(bw), len(ll), 2, 2)


def psl_probe_atomics(grid_ptr, cells, addr_ptr, n, repeats=5):
    ms = C.c_double()
    _call("psl_probe_atomics", grid_ptr, cells, addr_ptr, n, repeats, C.byref(ms))
    return ms.value


def psl_probe_copy(dst_ptr, src_ptr, nbytes, repeats=5):
    ms = C.c_double()
    _call("psl_probe_copy", dst_ptr, src_ptr, nbytes, repeats, C.byref(ms))
    return ms.value


def commission_nnls(a_ptr, m, n, b_ptr, x_ptr, opts, report):
    rc = lib().commission_nnls(a_ptr, m, n, b_ptr, x_ptr, C.byref(opts), C.byref(report))
    if rc not in (PSL_OK, PSL_ENOTCONV):
        check(rc)
    return rc


def commission_nnls_noalloc(a_dev, m, n, b_dev, x_dev, opts, report, stream):
    rc = lib().commission_nnls_noalloc(a_dev, m, n, b_dev, x_dev, C.byref(opts),
                                       C.byref(report), stream)
    if rc not in (PSL_OK, PSL_ENOTCONV):
        check(rc)
    return rc
