"""A particle-file source beside on-the-fly sampling: the comparison the paper
makes between its analytic source and its earlier PSL-file source model
(Sec. 3.1, Table 1).

The file source stores phase-space-plane records (beam-frame position and
direction at the plane, energy, history id, tag with the beam index), one
file per batch of a plan, written from this framework's own model with
sample_batch(PSL_SAMPLE_PLANE).  A dose calculation from files then reads
each batch's file from disk (T_par_rd), copies it to the GPU (T_par_cp),
applies jaws, beam -> patient transform and phantom entry on the GPU with
psl_transform_batch (T_par_tr) and transports it (T_sim); the on-the-fly path
samples and transforms in one kernel (T_par_gen_tr) before the same
transport.  Both paths transport the same particles bit for bit, so their
doses agree to FP32 atomic-add rounding and their event counters exactly.

File layout (little endian): 8-byte magic ``PSLREC01``, uint64 record count
n, int32 particle type (0 photon, 1 electron), uint32 zero; then n float32
each of x, y, u, v, w, e, n uint64 history ids and n uint32 tags.

Usage: python -m paper_1503_01725_amd.pslfile [--histories 2e7] [--dir D]
Prints one JSON line with the Table 1 breakdown for both paths.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import tempfile
import time

import numpy as np

MAGIC = b"PSLREC01"
HEADER_BYTES = 24
FLOAT_FIELDS = ("x", "y", "u", "v", "w", "e")
RECORD_BYTES = 4 * len(FLOAT_FIELDS) + 8 + 4


def offsets(n: int) -> dict:
    """Byte offset of each array in a file of n records."""
    off, o = {}, HEADER_BYTES
    for f in FLOAT_FIELDS:
        off[f] = o
        o += 4 * n
    off["hid"] = o
    o += 8 * n
    off["tag"] = o
    off["end"] = o + 4 * n
    return off


def write_records(path: str, rec: dict, ptype: int) -> int:
    """Writes the records (arrays of equal length) and returns the file size;
    the file is flushed to disk and dropped from the page cache, so that a
    later read comes from the disk as the paper's reads did."""
    n = len(rec["e"])
    head = MAGIC + np.array([n], dtype="<u8").tobytes() + np.array([ptype, 0], dtype="<i4").tobytes()
    with open(path, "wb") as fh:
        fh.write(head)
        for f in FLOAT_FIELDS:
            fh.write(np.ascontiguousarray(rec[f], dtype="<f4").tobytes())
        fh.write(np.ascontiguousarray(rec["hid"], dtype="<u8").tobytes())
        fh.write(np.ascontiguousarray(rec["tag"], dtype="<u4").tobytes())
        fh.flush()
        os.fsync(fh.fileno())
        drop_cache(fh.fileno())
    return offsets(n)["end"]


def drop_cache(fd: int) -> None:
    if hasattr(os, "posix_fadvise"):
        os.posix_fadvise(fd, 0, 0, os.POSIX_FADV_DONTNEED)


def read_header(path: str):
    with open(path, "rb") as fh:
        head = fh.read(HEADER_BYTES)
    if len(head) != HEADER_BYTES or head[:8] != MAGIC:
        raise ValueError(f"{path}: not a particle record file")
    n = int(np.frombuffer(head[8:16], dtype="<u8")[0])
    ptype = int(np.frombuffer(head[16:20], dtype="<i4")[0])
    if os.path.getsize(path) != offsets(n)["end"]:
        raise ValueError(f"{path}: size does not match {n} records")
    return n, ptype


def read_records(path: str):
    """The records as numpy arrays (host-side checks)."""
    n, ptype = read_header(path)
    raw = np.fromfile(path, dtype=np.uint8)
    off = offsets(n)
    rec = {f: raw[off[f]:off[f] + 4 * n].view("<f4") for f in FLOAT_FIELDS}
    rec["hid"] = raw[off["hid"]:off["hid"] + 8 * n].view("<u8")
    rec["tag"] = raw[off["tag"]:off["tag"] + 4 * n].view("<u4")
    return rec, ptype


class FileSource:
    """Reads record files into one pinned host buffer and one device buffer
    (both sized for the largest file) and describes the device copy as a
    plane-record stack for psl_transform_batch."""

    def __init__(self, max_bytes: int):
        import torch
        self.host = torch.empty(max_bytes, dtype=torch.uint8, pin_memory=True)
        self.dev = torch.empty(max_bytes, dtype=torch.uint8, device="cuda")
        self.view = memoryview(self.host.numpy())

    def read(self, path: str):
        """Disk -> pinned host buffer; returns (n, ptype, bytes)."""
        n, ptype = read_header(path)
        size = offsets(n)["end"]
        with open(path, "rb", buffering=0) as fh:
            got = fh.readinto(self.view[:size])
        if got != size:
            raise IOError(f"{path}: short read ({got} of {size} bytes)")
        return n, ptype, size

    def copy(self, size: int, stream=None):
        """Pinned host -> device (asynchronous on the stream)."""
        import torch
        s = stream if stream is not None else torch.cuda.current_stream()
        with torch.cuda.stream(s):
            self.dev[:size].copy_(self.host[:size], non_blocking=True)

    def plane_stack(self, n: int, ptype: int):
        from . import _native as N
        base = self.dev.data_ptr()
        off = offsets(n)
        return N.psl_particles(base + off["x"], base + off["y"], None, base + off["u"],
                               base + off["v"], base + off["w"], base + off["e"],
                               base + off["hid"], base + off["tag"], None, n, ptype)


def generate(plan, phantom, tally, seed, directory, max_batch, band_width, replica=0, log=print):
    """One record file per batch of the plan (PSL_SAMPLE_PLANE); returns the
    paths and the total bytes.  The tally receives the plane part of the
    source ledger (reset it before a dose calculation)."""
    import torch
    from . import engine as eng
    N = eng.N
    nb = plan.set_batching(max_batch, band_width)
    st = eng.Particles(max_batch)
    paths, total = [], 0
    for i in range(nb):
        b = plan.batch(i)
        N.sample_batch(plan.h, phantom.h, replica, b.h0, b.n, seed, st.c, N.PSL_SAMPLE_PLANE,
                       tally.h, eng._stream_ptr())
        torch.cuda.synchronize()
        h = st.host(b.n)
        tag = (h["tag"].astype(np.uint32) | (h["sub"].astype(np.uint32) << 16)
               | (h["status"].astype(np.uint32) << 24))
        rec = {f: h[f] for f in FLOAT_FIELDS}
        rec["hid"] = h["hid"]
        rec["tag"] = tag
        path = os.path.join(directory, f"batch{i:05d}.psl")
        total += write_records(path, rec, 1 if b.stype == 2 else 0)
        paths.append(path)
    log(f"[pslfile] wrote {nb} files, {total / 1e9:.3f} GB")
    return paths, total


def run_from_files(paths, plan, phantom, tally, params, seed, max_batch, src: FileSource):
    """Dose calculation of replica 0 from record files through the public
    calls (read -> copy -> psl_transform_batch -> transport_batch per batch,
    one FOLD); returns the time breakdown in seconds."""
    import torch
    from . import engine as eng
    N = eng.N
    e_cap = eng.electron_capacity(max_batch, plan.info.e_max, params.e_cut_electron)
    ph_stack = eng.Particles(max_batch)
    el_stack = eng.Particles(e_cap)
    s = torch.cuda.current_stream()
    sp = eng._stream_ptr(s)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    t = dict(rd=0.0, cp=0.0, tr=0.0, sim=0.0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for path in paths:
        r0 = time.perf_counter()
        n, ptype, size = src.read(path)
        t["rd"] += time.perf_counter() - r0
        ev[0].record(s)
        src.copy(size, s)
        ev[1].record(s)
        plane = src.plane_stack(n, ptype)
        N.psl_transform_batch(plan.h, phantom.h, plane, n, ph_stack.c, tally.h, sp)
        ev[2].record(s)
        N.transport_batch(phantom.h, ph_stack.c, el_stack.c, tally.h, params, seed, sp)
        ev[3].record(s)
        ev[3].synchronize()
        t["cp"] += ev[0].elapsed_time(ev[1]) / 1e3
        t["tr"] += ev[1].elapsed_time(ev[2]) / 1e3
        t["sim"] += ev[2].elapsed_time(ev[3]) / 1e3
    tally.op(N.PSL_TALLY_FOLD)
    torch.cuda.synchronize()
    t["total"] = time.perf_counter() - t0
    return t


def run_on_the_fly(plan, phantom, tally, params, seed, max_batch, band_width):
    """The same loop with the source sampled on the GPU (dense output, so the
    transport sees the same stacks as from the files)."""
    import torch
    from . import engine as eng
    N = eng.N
    nb = plan.set_batching(max_batch, band_width)
    e_cap = eng.electron_capacity(max_batch, plan.info.e_max, params.e_cut_electron)
    ph_stack = eng.Particles(max_batch)
    el_stack = eng.Particles(e_cap)
    s = torch.cuda.current_stream()
    sp = eng._stream_ptr(s)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    t = dict(gen_tr=0.0, sim=0.0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(nb):
        b = plan.batch(i)
        ev[0].record(s)
        N.sample_batch(plan.h, phantom.h, 0, b.h0, b.n, seed, ph_stack.c, N.PSL_SAMPLE_DENSE,
                       tally.h, sp)
        ev[1].record(s)
        N.transport_batch(phantom.h, ph_stack.c, el_stack.c, tally.h, params, seed, sp)
        ev[2].record(s)
        ev[2].synchronize()
        t["gen_tr"] += ev[0].elapsed_time(ev[1]) / 1e3
        t["sim"] += ev[1].elapsed_time(ev[2]) / 1e3
    tally.op(N.PSL_TALLY_FOLD)
    torch.cuda.synchronize()
    t["total"] = time.perf_counter() - t0
    return t


def main():
    import torch
    from . import engine as eng
    from . import workloads as wl
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--workload", default="water128_10")
    ap.add_argument("--histories", type=float, default=2e7)
    ap.add_argument("--max-batch", type=int, default=1 << 22)
    ap.add_argument("--band-width", type=int, default=24)
    ap.add_argument("--dir", default="")
    args = ap.parse_args()

    def log(m):
        print(m, file=sys.stderr, flush=True)

    W = wl.workload(args.workload)
    n_hist = int(args.histories)
    model = eng.Model(W.model)
    t0 = time.perf_counter()
    plan = eng.Plan(model, W.beams, n_hist, n_replica=1)
    t_init = time.perf_counter() - t0
    ph = eng.Phantom(W.phantom)
    prm = eng.transport_params()
    seed = W.seed
    tdir = args.dir or tempfile.mkdtemp(prefix="pslrec_", dir=os.environ.get("TMPDIR", "/tmp"))
    gen_tally = eng.Tally(ph)     # receives the plane part of the ledger
    tally_f = eng.Tally(ph)
    tally_o = eng.Tally(ph)
    try:
        paths, total_bytes = generate(plan, ph, gen_tally, seed, tdir, args.max_batch,
                                      args.band_width, log=log)
        src = FileSource(max(os.path.getsize(p) for p in paths))
        # a warm-up run loads every transport kernel, then the timed runs
        run_on_the_fly(plan, ph, tally_o, prm, seed, args.max_batch, args.band_width)
        tally_o.op(eng.N.PSL_TALLY_RESET)
        t_otf = run_on_the_fly(plan, ph, tally_o, prm, seed, args.max_batch, args.band_width)
        log(f"[pslfile] on the fly: {t_otf}")
        t_file = run_from_files(paths, plan, ph, tally_f, prm, seed, args.max_batch, src)
        log(f"[pslfile] from files: {t_file}")
        dose_o, _ = tally_o.finalize(plan)
        dose_f, _ = tally_f.finalize(plan)
        do, df = dose_o.cpu().numpy(), dose_f.cpu().numpy()
        _, cnt_o = tally_o.stats()
        _, cnt_f = tally_f.stats()
    finally:
        for f in os.listdir(tdir):
            if f.endswith(".psl"):
                os.remove(os.path.join(tdir, f))
        if not args.dir:
            os.rmdir(tdir)
    keys = ("entered", "wc_steps", "real", "e_pushed", "e_steps", "deposits")
    ref = np.abs(do).max()
    out = {
        "workload": args.workload, "histories": n_hist, "batches": len(paths),
        "file_bytes": int(total_bytes), "t_src_init_s": t_init,
        "file_source": {"T_total_s": t_file["total"], "T_sim_s": t_file["sim"],
                        "T_par_rd_s": t_file["rd"], "T_par_cp_s": t_file["cp"],
                        "T_par_tr_s": t_file["tr"],
                        "read_GBps": total_bytes / max(t_file["rd"], 1e-12) / 1e9},
        "on_the_fly": {"T_total_s": t_otf["total"], "T_sim_s": t_otf["sim"],
                       "T_par_gen_tr_s": t_otf["gen_tr"]},
        "gain": t_file["total"] / t_otf["total"],
        "dose_max_abs_diff_rel_dmax": float(np.abs(do - df).max() / ref),
        "counters_equal": all(int(cnt_o[k]) == int(cnt_f[k]) for k in keys),
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
