"""ctypes binding of ``liblbsq.so`` (the C ABI in ``include/lbsq.h``).

Argument marshalling only: every step of the lattice Boltzmann squirmer path
runs in the library's gfx950 kernels.  PyTorch, when present, supplies the
device memory (through the allocator callbacks of ``lb_params``) and the HIP
stream; nothing here computes.

The library must be built (``python -m paper_1903_04799_amd.build``); there
is no fallback: loading fails loudly when it is missing.
"""
from __future__ import annotations

import ctypes as C
import os
from pathlib import Path

import numpy as np

LIB_PATH = Path(__file__).resolve().parent / "liblbsq.so"

LB_OK, LB_EINVAL, LB_ENOMEM, LB_EDEVICE, LB_EGEOM, LB_ESTATE, LB_ENAN, LB_EBUDGET = 0, -1, -2, -3, -4, -5, -6, -7
LB_ECANCELED = -8
STORAGE = {"f32": 0, "f16": 1, "bf16": 2}
LAYOUT = {"auto": 0, "inplace": 1, "ab": 2}
MODES = {"free": 0, "fixed": 1, "prescribed": 2}
Q = 19

EXPORTED = [
    "lb_create", "lb_set_static_mask", "lb_add_squirmer", "lb_step", "lb_step_batch", "lb_sync",
    "lb_read_fields", "lb_force_torque", "lb_force_parts", "lb_body_state", "lb_links",
    "lb_read_populations", "lb_write_populations", "lb_audit", "lb_info", "lb_state_size",
    "lb_save_state", "lb_load_state", "lb_kernel_timing", "lb_kernel_time", "lb_destroy",
    "lb_strerror", "lb_server_create", "lb_server_submit", "lb_server_progress", "lb_server_results",
    "lb_server_stats_get", "lb_server_clock", "lb_server_destroy", "lb_server_cancel",
    "lb_read_fields_noalloc",
]
LB_REQ_MAXBODY = 8
LB_SERVER_MAXACTIVE = 64

ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class LbParams(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
                ("nu", C.c_double), ("magic", C.c_double), ("rho0", C.c_double),
                ("storage", C.c_int), ("scale_log2", C.c_int),
                ("wca_sigma", C.c_double), ("wca_eps", C.c_double),
                ("g", C.c_double * 3), ("audit_every", C.c_int),
                ("stream", C.c_void_p), ("alloc", ALLOC_FN), ("free", FREE_FN),
                ("alloc_ctx", C.c_void_p), ("layout", C.c_int)]


class LbSquirmer(C.Structure):
    _fields_ = [("pos", C.c_double * 3), ("e", C.c_double * 3), ("R", C.c_double),
                ("B1", C.c_double), ("beta", C.c_double), ("mode", C.c_int),
                ("v", C.c_double * 3), ("w", C.c_double * 3), ("rho_p", C.c_double)]


class LbServerParams(C.Structure):
    _fields_ = [("budget_bytes", C.c_size_t), ("max_active", C.c_int), ("chunk_steps", C.c_int),
                ("use_graph", C.c_int), ("storage", C.c_int), ("scale_log2", C.c_int),
                ("wca_sigma", C.c_double), ("wca_eps", C.c_double), ("stream", C.c_void_p),
                ("layout", C.c_int)]


class LbRequest(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int), ("nu", C.c_double),
                ("nbody", C.c_int), ("body", LbSquirmer * LB_REQ_MAXBODY), ("nsteps", C.c_int64),
                ("tag", C.c_uint64)]


_V3 = (C.c_double * 3) * LB_REQ_MAXBODY


class LbResult(C.Structure):
    _fields_ = [("ticket", C.c_uint64), ("tag", C.c_uint64), ("status", C.c_int), ("nbody", C.c_int),
                ("steps", C.c_int64), ("fluid_cells", C.c_uint64),
                ("pos", _V3), ("e", _V3), ("v", _V3), ("w", _V3), ("F", _V3), ("T", _V3),
                ("mass", C.c_double), ("t_submit", C.c_double), ("t_admit", C.c_double),
                ("t_done", C.c_double)]


class LbServerStats(C.Structure):
    _fields_ = [("cell_updates", C.c_uint64), ("chunks", C.c_uint64), ("graphs", C.c_uint64),
                ("completed", C.c_uint64), ("arena_in_use", C.c_size_t)]


class LBError(RuntimeError):
    def __init__(self, code, what=""):
        self.code = code
        super().__init__("%s: %s (%d)" % (what, strerror(code), code))


_lib = None


def load():
    """Load the built library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not LIB_PATH.exists():
        raise ImportError("liblbsq.so not built: run `python -m paper_1903_04799_amd.build` "
                          "(expected at %s)" % LIB_PATH)
    # torch ships its own copy of the HIP runtime under the same soname as the
    # system one.  Loading torch first makes the library bind to that copy, so
    # the process holds one HIP runtime and torch-allocated memory is valid here.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = C.CDLL(str(LIB_PATH))
    vp, dp, ip = C.c_void_p, C.POINTER(C.c_double), C.c_int
    sig = {
        "lb_create": [C.POINTER(LbParams), C.POINTER(vp)],
        "lb_set_static_mask": [vp, vp, C.c_size_t],
        "lb_add_squirmer": [vp, C.POINTER(LbSquirmer), C.POINTER(ip)],
        "lb_step": [vp, ip],
        "lb_step_batch": [C.POINTER(vp), ip, ip],
        "lb_sync": [vp],
        "lb_read_fields": [vp, dp, dp, vp],
        "lb_read_fields_noalloc": [vp, dp, dp, vp],
        "lb_force_torque": [vp, ip, dp, dp],
        "lb_force_parts": [vp, ip, dp, dp, dp, dp],
        "lb_body_state": [vp, ip, dp, dp, dp, dp, dp],
        "lb_links": [vp, vp, vp, vp, C.c_size_t, C.POINTER(C.c_size_t)],
        "lb_read_populations": [vp, dp],
        "lb_write_populations": [vp, dp],
        "lb_audit": [vp, dp, dp],
        "lb_info": [vp, C.POINTER(C.c_uint64), C.POINTER(C.c_int64)],
        "lb_state_size": [vp, C.POINTER(C.c_size_t)],
        "lb_save_state": [vp, vp, C.c_size_t],
        "lb_load_state": [vp, vp, C.c_size_t],
        "lb_kernel_timing": [vp, ip],
        "lb_kernel_time": [vp, dp, C.POINTER(C.c_int64)],
        "lb_destroy": [vp],
        "lb_server_create": [C.POINTER(LbServerParams), C.POINTER(vp)],
        "lb_server_submit": [vp, C.POINTER(LbRequest), C.POINTER(C.c_uint64)],
        "lb_server_progress": [vp, ip, C.POINTER(ip), C.POINTER(ip)],
        "lb_server_results": [vp, C.POINTER(LbResult), ip, C.POINTER(ip)],
        "lb_server_stats_get": [vp, C.POINTER(LbServerStats)],
        "lb_server_clock": [vp, dp],
        "lb_server_destroy": [vp],
        "lb_server_cancel": [vp, C.c_uint64],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = C.c_int
    L.lb_strerror.argtypes = [C.c_int]
    L.lb_strerror.restype = C.c_char_p
    _lib = L
    return L


def strerror(code):
    return load().lb_strerror(int(code)).decode()


def _check(rc, what):
    if rc != LB_OK:
        raise LBError(rc, what)


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


class _TorchMemory:
    """Device allocator callbacks backed by torch's caching allocator."""

    def __init__(self, device):
        import torch
        self.torch = torch
        self.device = device
        self.blocks = {}
        self.nalloc = 0  # allocator calls made by the library so far
        self.alloc_cb = ALLOC_FN(self._alloc)
        self.free_cb = FREE_FN(self._free)

    def _alloc(self, nbytes, ctx):
        self.nalloc += 1
        try:
            t = self.torch.empty(int(nbytes), dtype=self.torch.uint8, device=self.device)
        except Exception:
            return None
        self.blocks[t.data_ptr()] = t
        return t.data_ptr()

    def _free(self, ptr, ctx):
        self.blocks.pop(ptr, None)


def _torch_cuda():
    try:
        import torch
        return torch if torch.cuda.is_available() else None
    except Exception:
        return None


def _squirmer(pos, e=(1.0, 0.0, 0.0), R=4.0, B1=0.0, beta=0.0, mode="free", v=(0.0, 0.0, 0.0),
              w=(0.0, 0.0, 0.0), rho_p=0.0, out=None):
    q = out if out is not None else LbSquirmer()
    q.pos = (C.c_double * 3)(*map(float, pos))
    q.e = (C.c_double * 3)(*map(float, e))
    q.R, q.B1, q.beta = float(R), float(B1), float(beta)
    q.mode = MODES[mode] if isinstance(mode, str) else int(mode)
    q.v = (C.c_double * 3)(*map(float, v))
    q.w = (C.c_double * 3)(*map(float, w))
    q.rho_p = float(rho_p)
    return q


class Sim:
    """One periodic D3Q19 box with squirmers, resident on the GPU."""

    def __init__(self, shape, nu=1.0 / 6.0, magic=3.0 / 16.0, rho0=1.0, storage="f32",
                 scale_log2=None, wca_sigma=1.0, wca_eps=0.01, g=(0.0, 0.0, 0.0), audit_every=100,
                 stream=None, torch_memory=True, layout="auto"):
        L = load()
        nx, ny, nz = (int(v) for v in shape)
        self.shape = (nx, ny, nz)
        self.n = nx * ny * nz
        p = LbParams()
        p.nx, p.ny, p.nz = nx, ny, nz
        p.nu, p.magic, p.rho0 = float(nu), float(magic), float(rho0)
        p.storage = STORAGE[storage]
        if scale_log2 is None:
            scale_log2 = 14 if storage == "f16" else 0
        p.scale_log2 = int(scale_log2)
        p.wca_sigma, p.wca_eps = float(wca_sigma), float(wca_eps)
        p.g = (C.c_double * 3)(*[float(x) for x in g])
        p.audit_every = int(audit_every)
        p.layout = LAYOUT[layout]
        self._mem = None
        torch = _torch_cuda()
        if stream is None and torch is not None:
            stream = torch.cuda.current_stream().cuda_stream
        p.stream = stream
        if torch_memory and torch is not None:
            self._mem = _TorchMemory(torch.device("cuda", torch.cuda.current_device()))
            p.alloc, p.free = self._mem.alloc_cb, self._mem.free_cb
        self.params = p
        self.storage = storage
        h = C.c_void_p()
        _check(L.lb_create(C.byref(p), C.byref(h)), "lb_create")
        self.h = h
        self.nbody = 0

    # -- life cycle --------------------------------------------------------
    def close(self):
        if getattr(self, "h", None):
            load().lb_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- set-up ------------------------------------------------------------
    def set_static_mask(self, solid):
        m = np.ascontiguousarray(np.asarray(solid).reshape(-1) != 0, dtype=np.uint8)
        _check(load().lb_set_static_mask(self.h, m.ctypes.data, m.size), "lb_set_static_mask")

    def add_squirmer(self, pos, e=(1.0, 0.0, 0.0), R=4.0, B1=0.0, beta=0.0, mode="free",
                     v=(0.0, 0.0, 0.0), w=(0.0, 0.0, 0.0), rho_p=0.0):
        q = _squirmer(pos, e, R, B1, beta, mode, v, w, rho_p)
        i = C.c_int(-1)
        _check(load().lb_add_squirmer(self.h, C.byref(q), C.byref(i)), "lb_add_squirmer")
        self.nbody += 1
        return i.value

    # -- stepping ----------------------------------------------------------
    def step(self, n=1):
        _check(load().lb_step(self.h, int(n)), "lb_step")

    def sync(self):
        _check(load().lb_sync(self.h), "lb_sync")

    # -- readout -----------------------------------------------------------
    def fields(self):
        nx, ny, nz = self.shape
        rho = np.empty(self.n)
        u = np.empty(3 * self.n)
        own = np.empty(self.n, dtype=np.uint8)
        _check(load().lb_read_fields(self.h, _dptr(rho), _dptr(u), own.ctypes.data), "lb_read_fields")
        return rho.reshape(nz, ny, nx), u.reshape(3, nz, ny, nx), own.reshape(nz, ny, nx)

    def fields_noalloc(self):
        """The same as ``fields()`` through lb_read_fields_noalloc, which
        allocates no device memory."""
        nx, ny, nz = self.shape
        rho = np.empty(self.n)
        u = np.empty(3 * self.n)
        own = np.empty(self.n, dtype=np.uint8)
        _check(load().lb_read_fields_noalloc(self.h, _dptr(rho), _dptr(u), own.ctypes.data),
               "lb_read_fields_noalloc")
        return rho.reshape(nz, ny, nx), u.reshape(3, nz, ny, nx), own.reshape(nz, ny, nx)

    def force_torque(self, i=0):
        F, T = np.empty(3), np.empty(3)
        _check(load().lb_force_torque(self.h, int(i), _dptr(F), _dptr(T)), "lb_force_torque")
        return F, T

    def force_parts(self, i=0):
        a = [np.empty(3) for _ in range(4)]
        _check(load().lb_force_parts(self.h, int(i), *[_dptr(x) for x in a]), "lb_force_parts")
        return dict(zip(("Fbb", "Tbb", "Fc", "Tc"), a))

    def body(self, i=0):
        a = [np.empty(3) for _ in range(5)]
        _check(load().lb_body_state(self.h, int(i), *[_dptr(x) for x in a]), "lb_body_state")
        return dict(zip(("pos", "e", "v", "w", "Fwca"), a))

    def links(self):
        L = load()
        n = C.c_size_t(0)
        rc = L.lb_links(self.h, None, None, None, 0, C.byref(n))
        if rc not in (LB_OK, LB_EINVAL):
            _check(rc, "lb_links")
        cnt = n.value
        cell = np.empty(cnt, dtype=np.uint32)
        d = np.empty(cnt, dtype=np.uint8)
        o = np.empty(cnt, dtype=np.uint8)
        _check(L.lb_links(self.h, cell.ctypes.data, d.ctypes.data, o.ctypes.data, cnt, C.byref(n)),
               "lb_links")
        return cell, d, o

    def populations(self):
        nx, ny, nz = self.shape
        f = np.empty(Q * self.n)
        _check(load().lb_read_populations(self.h, _dptr(f)), "lb_read_populations")
        return f.reshape(Q, nz, ny, nx)

    def set_populations(self, f):
        f = np.ascontiguousarray(f, dtype=np.float64).reshape(-1)
        if f.size != Q * self.n:
            raise ValueError("populations must have 19*N entries")
        _check(load().lb_write_populations(self.h, _dptr(f)), "lb_write_populations")

    def audit(self):
        m = C.c_double()
        P = np.empty(3)
        _check(load().lb_audit(self.h, C.byref(m), _dptr(P)), "lb_audit")
        return m.value, P

    def info(self):
        nf, st = C.c_uint64(), C.c_int64()
        _check(load().lb_info(self.h, C.byref(nf), C.byref(st)), "lb_info")
        return {"n_fluid": nf.value, "steps": st.value}

    # -- checkpoint --------------------------------------------------------
    def save_state(self):
        n = C.c_size_t()
        _check(load().lb_state_size(self.h, C.byref(n)), "lb_state_size")
        buf = C.create_string_buffer(n.value)
        _check(load().lb_save_state(self.h, buf, n.value), "lb_save_state")
        return buf.raw

    def load_state(self, blob):
        buf = C.create_string_buffer(blob, len(blob))
        _check(load().lb_load_state(self.h, buf, len(blob)), "lb_load_state")

    # -- measurement ---------------------------------------------------------
    def kernel_timing(self, enable=True):
        _check(load().lb_kernel_timing(self.h, 1 if enable else 0), "lb_kernel_timing")

    def kernel_time(self):
        ms, n = C.c_double(), C.c_int64()
        _check(load().lb_kernel_time(self.h, C.byref(ms), C.byref(n)), "lb_kernel_time")
        return ms.value, n.value


def step_batch(sims, nsteps):
    arr = (C.c_void_p * len(sims))(*[s.h for s in sims])
    _check(load().lb_step_batch(arr, len(sims), int(nsteps)), "lb_step_batch")


class Server:
    """Continuous-batching server of independent squirmer simulations
    (``lb_server_*``): requests are queued, admitted by device-memory budget,
    advanced together in batched chunks and retired with their results."""

    def __init__(self, budget_bytes, max_active=16, chunk_steps=100, use_graph=True, storage="f32",
                 scale_log2=None, wca_sigma=1.0, wca_eps=0.01, stream=None, layout="auto"):
        L = load()
        p = LbServerParams()
        p.budget_bytes = int(budget_bytes)
        p.max_active = int(max_active)
        p.chunk_steps = int(chunk_steps)
        p.use_graph = 1 if use_graph else 0
        p.storage = STORAGE[storage]
        p.scale_log2 = int(14 if (scale_log2 is None and storage == "f16") else (scale_log2 or 0))
        p.wca_sigma, p.wca_eps = float(wca_sigma), float(wca_eps)
        p.stream = stream
        p.layout = LAYOUT[layout]
        h = C.c_void_p()
        _check(L.lb_server_create(C.byref(p), C.byref(h)), "lb_server_create")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            load().lb_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def submit(self, shape, bodies, nsteps, nu=1.0 / 6.0, tag=0):
        """Queue one request; bodies is a list of keyword dicts of
        ``Sim.add_squirmer``.  Returns the ticket."""
        if len(bodies) > LB_REQ_MAXBODY:
            raise ValueError("at most %d bodies per request" % LB_REQ_MAXBODY)
        rq = LbRequest()
        rq.nx, rq.ny, rq.nz = (int(v) for v in shape)
        rq.nu = float(nu)
        rq.nbody = len(bodies)
        for i, b in enumerate(bodies):
            _squirmer(out=rq.body[i], **b)
        rq.nsteps = int(nsteps)
        rq.tag = int(tag)
        t = C.c_uint64()
        _check(load().lb_server_submit(self.h, C.byref(rq), C.byref(t)), "lb_server_submit")
        return t.value

    def cancel(self, ticket):
        """Cancel a queued or resident request (``lb_server_cancel``).
        Returns True if it was cancelled, False if it had already ended or is
        in its final chunk."""
        rc = load().lb_server_cancel(self.h, C.c_uint64(int(ticket)))
        if rc == LB_ESTATE:
            return False
        _check(rc, "lb_server_cancel")
        return True

    def progress(self, wait=False):
        a, q = C.c_int(), C.c_int()
        _check(load().lb_server_progress(self.h, 1 if wait else 0, C.byref(a), C.byref(q)),
               "lb_server_progress")
        return a.value, q.value

    def results(self, cap=256):
        buf = (LbResult * cap)()
        n = C.c_int()
        _check(load().lb_server_results(self.h, buf, cap, C.byref(n)), "lb_server_results")
        out = []
        for r in buf[:n.value]:
            nb = r.nbody
            d = {k: getattr(r, k) for k in ("ticket", "tag", "status", "nbody", "steps", "fluid_cells",
                                             "mass", "t_submit", "t_admit", "t_done")}
            for k in ("pos", "e", "v", "w", "F", "T"):
                d[k] = np.array([list(getattr(r, k)[i]) for i in range(nb)]).reshape(nb, 3)
            out.append(d)
        return out

    def stats(self):
        st = LbServerStats()
        _check(load().lb_server_stats_get(self.h, C.byref(st)), "lb_server_stats_get")
        return {k: getattr(st, k) for k, _ in LbServerStats._fields_}

    def clock(self):
        t = C.c_double()
        _check(load().lb_server_clock(self.h, C.byref(t)), "lb_server_clock")
        return t.value
