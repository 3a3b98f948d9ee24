"""Python front-end of the FP64 reference renderer (``splotch_oracle.c``).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the
benchmark's CPU-baseline leg are the only callers.  The product path never
imports this module.

``build()`` compiles ``liboracle.so`` with gcc (-O2, OpenMP, no fast-math);
``render()`` runs the plain per-particle definition in double precision and
returns the optical-depth plane L, the image I = 1 - exp(-L), the exact
number of (particle, pixel) samples and the active-particle count.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from pathlib import Path

import numpy as np

HERE = Path(__file__).resolve().parent
SRC = HERE / "splotch_oracle.c"
LIB = HERE / "liboracle.so"


class _Camera(C.Structure):
    _fields_ = [("eye", C.c_double * 3), ("target", C.c_double * 3),
                ("up", C.c_double * 3), ("fov_deg", C.c_double),
                ("z_near", C.c_double), ("width", C.c_int32), ("height", C.c_int32)]


class _Params(C.Structure):
    _fields_ = [("chi", C.c_double), ("brightness", C.c_double * 4),
                ("fixed_sigma_frac", C.c_double * 4), ("scalar_min", C.c_double),
                ("scalar_max", C.c_double), ("scalar_log10", C.c_int32),
                ("col_norm", C.c_int32), ("colour_mode", C.c_int32),
                ("absorption", C.c_double * 4), ("prefilter", C.c_double)]


class _Stats(C.Structure):
    _fields_ = [("samples", C.c_int64), ("active", C.c_int64),
                ("threads_used", C.c_int32)]


def build(force: bool = True) -> Path:
    """Compile the oracle shared library (gcc, -O2 -fopenmp)."""
    if force or not LIB.exists() or LIB.stat().st_mtime < SRC.stat().st_mtime:
        tmp = LIB.with_suffix(".so.tmp")
        subprocess.run(["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fPIC", "-shared",
                        "-fopenmp", "-ffp-contract=off", "-o", str(tmp), str(SRC), "-lm"],
                       check=True)
        os.replace(tmp, LIB)
    return LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not LIB.exists():
            build()
        lib = C.CDLL(str(LIB))
        lib.oracle_render.restype = C.c_int
        lib.oracle_render_ordered.restype = C.c_int
        lib.oracle_project.restype = C.c_int
        lib.oracle_max_threads.restype = C.c_int
        _lib = lib
    return _lib


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _ptr(a, ty=C.c_float):
    return a.ctypes.data_as(C.POINTER(ty)) if a is not None else None


def _camera(cam) -> _Camera:
    c = _Camera()
    # the float32 values the GPU path receives, widened to double
    for k in range(3):
        c.eye[k] = float(np.float32(cam.eye[k]))
        c.target[k] = float(np.float32(cam.target[k]))
        c.up[k] = float(np.float32(cam.up[k]))
    c.fov_deg = float(np.float32(cam.fov_deg))
    c.z_near = float(np.float32(cam.z_near))
    c.width, c.height = int(cam.width), int(cam.height)
    return c


def _params(prm) -> _Params:
    p = _Params()
    p.chi = float(np.float32(prm.chi))
    for k in range(4):
        p.brightness[k] = float(np.float32(prm.brightness[k]))
        p.fixed_sigma_frac[k] = float(np.float32(prm.fixed_sigma_frac[k]))
    p.scalar_min = float(np.float32(prm.scalar_min))
    p.scalar_max = float(np.float32(prm.scalar_max))
    p.scalar_log10 = int(prm.scalar_log10)
    p.col_norm = int(prm.col_norm)
    p.colour_mode = int(getattr(prm, "colour_mode", 0))
    for k in range(4):
        p.absorption[k] = float(np.float32(getattr(prm, "absorption", (0.0,) * 4)[k]))
    p.prefilter = float(np.float32(getattr(prm, "prefilter", 0.0)))
    return p


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def render(ps, cam, cmap, prm, threads: int = 0, want_count: bool = False,
           want_image: bool = True, window=None) -> dict:
    """FP64 render of particle set ``ps`` (float32 SoA) with camera ``cam``,
    palette ``cmap`` (M x 3 float32; None in the vector colour mode) and
    parameters ``prm``.  ``window`` = (x0, y0, w, h) renders only that block
    of pixels (the same values the full image holds there)."""
    lib = _load()
    n = ps.n
    arrs = [None if a is None else _f32(a)
            for a in (ps.x, ps.y, ps.z, ps.h, ps.intensity, ps.scalar,
                      getattr(ps, "vx", None), getattr(ps, "vy", None), getattr(ps, "vz", None))]
    sp = None if ps.species is None else np.ascontiguousarray(ps.species, dtype=np.uint8)
    cm = np.zeros((0, 3), np.float32) if cmap is None else _f32(cmap).reshape(-1, 3)
    W, H = int(cam.width), int(cam.height)
    win = None
    if window is not None:
        win = np.array(window, np.int32)
        W, H = int(win[2]), int(win[3])
    L = np.empty((H, W, 3), np.float64)
    I = np.empty((H, W, 3), np.float64) if want_image else None
    cnt = np.empty((H, W), np.int32) if want_count else None
    st = _Stats()
    c, p = _camera(cam), _params(prm)
    if int(getattr(prm, "transfer", 0)) == 1:
        # E != A: ordered compositing along each ray (L = absorption depth)
        I = np.empty((H, W, 3), np.float64)
        rc = lib.oracle_render_ordered(
            C.c_int64(n), *[_ptr(a) for a in arrs],
            _ptr(sp, C.c_uint8) if sp is not None else None,
            C.byref(c), C.c_int32(cm.shape[0]), _ptr(cm) if cm.shape[0] else None, C.byref(p),
            _ptr(win, C.c_int32) if win is not None else None, C.c_int32(threads),
            _ptr(L, C.c_double), _ptr(I, C.c_double), C.byref(st))
        if rc != 0:
            raise RuntimeError(f"oracle_render_ordered failed with code {rc}")
        return dict(L=L, I=I, count=None, samples=int(st.samples), active=int(st.active),
                    threads=int(st.threads_used))
    rc = lib.oracle_render(
        C.c_int64(n), *[_ptr(a) for a in arrs],
        _ptr(sp, C.c_uint8) if sp is not None else None,
        C.byref(c), C.c_int32(cm.shape[0]), _ptr(cm) if cm.shape[0] else None, C.byref(p),
        _ptr(win, C.c_int32) if win is not None else None, C.c_int32(threads),
        _ptr(L, C.c_double), _ptr(I, C.c_double) if I is not None else None,
        _ptr(cnt, C.c_int32) if cnt is not None else None, C.byref(st))
    if rc != 0:
        raise RuntimeError(f"oracle_render failed with code {rc}")
    return dict(L=L, I=I, count=cnt, samples=int(st.samples), active=int(st.active),
                threads=int(st.threads_used))


def project(ps, cam, prm) -> dict:
    """Screen position, screen sigma and depth of every particle (O1-O5)."""
    lib = _load()
    n = ps.n
    arrs = [_f32(a) for a in (ps.x, ps.y, ps.z, ps.h)]
    sp = None if ps.species is None else np.ascontiguousarray(ps.species, dtype=np.uint8)
    X, Y, S, D = (np.empty(n, np.float64) for _ in range(4))
    c, p = _camera(cam), _params(prm)
    rc = lib.oracle_project(C.c_int64(n), *[_ptr(a) for a in arrs],
                            _ptr(sp, C.c_uint8) if sp is not None else None,
                            C.byref(c), C.byref(p), _ptr(X, C.c_double),
                            _ptr(Y, C.c_double), _ptr(S, C.c_double), _ptr(D, C.c_double))
    if rc != 0:
        raise RuntimeError("oracle_project: degenerate camera")
    return dict(X=X, Y=Y, sigma=S, depth=D)
