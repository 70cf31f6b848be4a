"""Python handle on the FP64 CPU oracle (``lbsq_oracle.c``).

TEST INFRASTRUCTURE ONLY: the plain, slow reference implementation of the
lattice Boltzmann squirmer method of arXiv:1903.04799 that the GPU library is
checked against.  Only the tests, the smoke check and the CPU-baseline leg of
the benchmark may import this module.  It shares no code with the GPU path.

The C source follows the paper section by section (see its header for the
readings taken where the printed equations are garbled or silent).  This
module only marshals arguments.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from pathlib import Path

import numpy as np

HERE = Path(__file__).resolve().parent
SRC = HERE / "lbsq_oracle.c"
LIB = HERE / "liboracle.so"

FREE, FIXED, PRESCRIBED = 0, 1, 2
Q = 19


def build(force: bool = False) -> Path:
    """Compile the oracle with gcc (OpenMP on the stream/collide loop)."""
    if force or not LIB.exists() or LIB.stat().st_mtime < SRC.stat().st_mtime:
        tmp = LIB.with_suffix(".so.tmp%d" % os.getpid())
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fopenmp", "-fPIC", "-shared",
             "-o", str(tmp), str(SRC), "-lm"])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(str(LIB))
        dp = C.POINTER(C.c_double)
        L.or_create.restype = C.c_void_p
        L.or_create.argtypes = [C.c_int, C.c_int, C.c_int, C.c_double, C.c_double, C.c_double,
                                dp, C.c_double, C.c_double]
        L.or_destroy.argtypes = [C.c_void_p]
        L.or_set_static_mask.argtypes = [C.c_void_p, C.c_void_p, dp]
        L.or_add_body.argtypes = [C.c_void_p, dp, dp, C.c_double, C.c_double, C.c_double, C.c_int,
                                  dp, dp, C.c_double]
        L.or_step.argtypes = [C.c_void_p, C.c_int]
        L.or_convert_only.argtypes = [C.c_void_p]
        L.or_get_fields.argtypes = [C.c_void_p, dp, dp, C.c_void_p]
        L.or_get_populations.argtypes = [C.c_void_p, dp]
        L.or_set_populations.argtypes = [C.c_void_p, dp]
        L.or_body_state.argtypes = [C.c_void_p, C.c_int, dp]
        L.or_set_body_state.argtypes = [C.c_void_p, C.c_int, dp, dp, dp, dp]
        L.or_links.restype = C.c_size_t
        L.or_links.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t]
        L.or_conversions.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(C.c_size_t),
                                     C.c_void_p, C.c_void_p, C.POINTER(C.c_size_t), C.c_size_t]
        L.or_step_stats.argtypes = [C.c_void_p, dp]
        L.or_audit.argtypes = [C.c_void_p, dp, dp]
        L.or_get_step.restype = C.c_long
        L.or_get_step.argtypes = [C.c_void_p]
        L.or_relaxation_rates.argtypes = [C.c_void_p, dp, dp]
        L.or_threads.restype = C.c_int
        L.or_threads.argtypes = []
        L.or_set_threads.argtypes = [C.c_int]
        L.or_lattice.argtypes = [C.POINTER(C.c_int), dp]
        L.or_feq.argtypes = [C.c_double, dp, dp]
        L.or_slip.argtypes = [dp, dp, C.c_double, C.c_double, dp]
        L.or_wca.restype = C.c_double
        L.or_wca.argtypes = [C.c_double, C.c_double, C.c_double]
        L.or_rotate.argtypes = [dp, dp]
        L.or_integrate.argtypes = [dp, dp, dp, dp, dp, dp, C.c_double, C.c_double, C.c_int,
                                   C.POINTER(C.c_int)]
        L.or_inside.restype = C.c_int
        L.or_inside.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, dp, C.c_double]
        _lib = L
    return _lib


def _d(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(C.POINTER(C.c_double))


def threads():
    """OpenMP threads the oracle's stream/collide loop uses."""
    return int(lib().or_threads())


def set_threads(n):
    lib().or_set_threads(int(n))


def lattice():
    c = (C.c_int * 57)()
    w = (C.c_double * 19)()
    lib().or_lattice(c, w)
    return np.array(c[:], dtype=np.int64).reshape(19, 3), np.array(w[:])


def feq(rho, u):
    out = np.zeros(19)
    _, up = _d(u)
    lib().or_feq(float(rho), up, out.ctypes.data_as(C.POINTER(C.c_double)))
    return out


def slip(d, e, B1, beta):
    out = np.zeros(3)
    _, dp_ = _d(d)
    _, ep = _d(e)
    lib().or_slip(dp_, ep, float(B1), float(beta), out.ctypes.data_as(C.POINTER(C.c_double)))
    return out


def wca(r, sigma, eps):
    return lib().or_wca(float(r), float(sigma), float(eps))


def rotate(e, w):
    e = np.array(e, dtype=np.float64)
    _, wp = _d(w)
    lib().or_rotate(e.ctypes.data_as(C.POINTER(C.c_double)), wp)
    return e


def integrate(pos, e, v, w, F, T, m, I, mode, box):
    """One symplectic-Euler step of a rigid body; returns new (pos, e, v, w)."""
    arrs = [np.array(a, dtype=np.float64) for a in (pos, e, v, w)]
    _, Fp = _d(F)
    _, Tp = _d(T)
    b = (C.c_int * 3)(*[int(x) for x in box])
    ptrs = [a.ctypes.data_as(C.POINTER(C.c_double)) for a in arrs]
    lib().or_integrate(*ptrs, Fp, Tp, float(m), float(I), int(mode), b)
    return tuple(arrs)


def inside(n, cell, pos, R):
    _, pp = _d(pos)
    return bool(lib().or_inside(int(n[0]), int(n[1]), int(n[2]), int(cell[0]), int(cell[1]),
                                int(cell[2]), pp, float(R)))


class OracleSim:
    """One periodic box simulated by the FP64 oracle."""

    def __init__(self, nx, ny, nz, nu=1.0 / 6.0, magic=3.0 / 16.0, rho0=1.0, g=(0.0, 0.0, 0.0),
                 wca_sigma=1.0, wca_eps=0.01):
        self.shape = (int(nx), int(ny), int(nz))
        self.n = int(nx) * int(ny) * int(nz)
        self._g, gp = _d(g)
        h = lib().or_create(int(nx), int(ny), int(nz), float(nu), float(magic), float(rho0), gp,
                            float(wca_sigma), float(wca_eps))
        if not h:
            raise ValueError("oracle: invalid parameters")
        self.h = C.c_void_p(h)
        self.nbody = 0

    def close(self):
        if self.h:
            lib().or_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def rates(self):
        a, b = C.c_double(), C.c_double()
        lib().or_relaxation_rates(self.h, C.byref(a), C.byref(b))
        return a.value, b.value

    def set_static_mask(self, solid, wall_u=None):
        solid = np.ascontiguousarray(solid, dtype=np.uint8).reshape(-1)
        assert solid.size == self.n
        wu = None
        if wall_u is not None:
            self._wall_u, wu = _d(np.asarray(wall_u, dtype=np.float64).reshape(3, self.n))
        rc = lib().or_set_static_mask(self.h, solid.ctypes.data, wu)
        if rc:
            raise RuntimeError("oracle: static mask rejected (%d)" % rc)

    def add_body(self, pos, e, R, B1=0.0, beta=0.0, mode=FREE, v=(0, 0, 0), w=(0, 0, 0), rho_p=1.0):
        _, pp = _d(pos)
        _, ep = _d(e)
        _, vp = _d(v)
        _, wp = _d(w)
        rc = lib().or_add_body(self.h, pp, ep, float(R), float(B1), float(beta), int(mode), vp, wp,
                               float(rho_p))
        if rc < 0:
            raise ValueError("oracle: add_body failed (%d)" % rc)
        self.nbody += 1
        return rc

    def step(self, n=1):
        rc = lib().or_step(self.h, int(n))
        if rc:
            raise RuntimeError("oracle: geometry error (%d)" % rc)

    def convert_only(self):
        """Test-only: convert the cells the bodies covered or uncovered since
        the owners were last computed (after ``set_body``), eq. (consforce),
        with nothing else of a step."""
        rc = lib().or_convert_only(self.h)
        if rc:
            raise RuntimeError("oracle: geometry error (%d)" % rc)

    @property
    def t(self):
        return lib().or_get_step(self.h)

    def fields(self):
        nx, ny, nz = self.shape
        rho = np.zeros(self.n)
        u = np.zeros(3 * self.n)
        own = np.zeros(self.n, dtype=np.uint8)
        lib().or_get_fields(self.h, rho.ctypes.data_as(C.POINTER(C.c_double)),
                            u.ctypes.data_as(C.POINTER(C.c_double)), own.ctypes.data)
        return (rho.reshape(nz, ny, nx), u.reshape(3, nz, ny, nx), own.reshape(nz, ny, nx))

    def populations(self):
        f = np.zeros(19 * self.n)
        lib().or_get_populations(self.h, f.ctypes.data_as(C.POINTER(C.c_double)))
        nx, ny, nz = self.shape
        return f.reshape(19, nz, ny, nx)

    def set_populations(self, f):
        f, fp = _d(np.asarray(f).reshape(-1))
        assert f.size == 19 * self.n
        lib().or_set_populations(self.h, fp)

    def body(self, i):
        out = np.zeros(41)
        if lib().or_body_state(self.h, int(i), out.ctypes.data_as(C.POINTER(C.c_double))):
            raise IndexError(i)
        names = ["pos", "e", "v", "w", "F", "T", "Fbb", "Tbb", "Fc", "Tc", "Fwca", "Fc_next", "Tc_next"]
        d = {k: out[3 * a:3 * a + 3].copy() for a, k in enumerate(names)}
        d["m"], d["I"] = out[39], out[40]
        return d

    def set_body(self, i, pos, e, v, w):
        ps = [_d(a) for a in (pos, e, v, w)]
        if lib().or_set_body_state(self.h, int(i), *[p[1] for p in ps]):
            raise IndexError(i)

    def links(self):
        cap = 19 * self.n
        cell = np.zeros(cap, dtype=np.uint32)
        d = np.zeros(cap, dtype=np.uint8)
        b = np.zeros(cap, dtype=np.uint8)
        cnt = lib().or_links(self.h, cell.ctypes.data, d.ctypes.data, b.ctypes.data, cap)
        return cell[:cnt].copy(), d[:cnt].copy(), b[:cnt].copy()

    def conversions(self):
        cap = self.n
        cov = np.zeros(cap, dtype=np.uint32)
        covb = np.zeros(cap, dtype=np.uint8)
        unc = np.zeros(cap, dtype=np.uint32)
        uncb = np.zeros(cap, dtype=np.uint8)
        nc, nu = C.c_size_t(), C.c_size_t()
        lib().or_conversions(self.h, cov.ctypes.data, covb.ctypes.data, C.byref(nc),
                             unc.ctypes.data, uncb.ctypes.data, C.byref(nu), cap)
        return (cov[:nc.value].copy(), covb[:nc.value].copy(), unc[:nu.value].copy(),
                uncb[:nu.value].copy())

    def step_stats(self):
        out = np.zeros(5)
        lib().or_step_stats(self.h, out.ctypes.data_as(C.POINTER(C.c_double)))
        return {"link_mass": out[0], "covered_mass": out[1], "uncovered_mass": out[2],
                "ncovered": int(out[3]), "nuncovered": int(out[4])}

    def audit(self):
        m = C.c_double()
        P = np.zeros(3)
        lib().or_audit(self.h, C.byref(m), P.ctypes.data_as(C.POINTER(C.c_double)))
        return m.value, P
