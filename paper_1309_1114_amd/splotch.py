"""Python binding of ``libsplotch.so`` (the C ABI in include/splotch.h).

Argument marshalling only: every step of the render runs in the library's
HIP kernels.  PyTorch supplies device memory and the stream.  If the built
library is missing this module raises instead of falling back to anything.
"""
from __future__ import annotations

import ctypes as C
from pathlib import Path

import numpy as np

PKG = Path(__file__).resolve().parent
LIB_PATH = PKG / "libsplotch.so"

MAX_SPECIES = 4
OK = 0
ERR_INVALID_ARG = -1
ERR_WORKSPACE = -2
ERR_HIP = -3
ERR_OVERFLOW = -4
ERR_UNSUPPORTED = -5
ACCUM_FP32 = 0
ACCUM_INT64 = 1
STAGES = ("clear", "count", "scan", "scatter", "items", "large", "splat", "resolve")
NUM_STAGES = len(STAGES)


class Particles(C.Structure):
    _fields_ = [("n", C.c_int64), ("x", C.c_void_p), ("y", C.c_void_p), ("z", C.c_void_p),
                ("h", C.c_void_p), ("intensity", C.c_void_p), ("scalar", C.c_void_p),
                ("species", C.c_void_p), ("vx", C.c_void_p), ("vy", C.c_void_p),
                ("vz", C.c_void_p)]


class CameraS(C.Structure):
    _fields_ = [("eye", C.c_float * 3), ("target", C.c_float * 3), ("up", C.c_float * 3),
                ("fov_deg", C.c_float), ("z_near", C.c_float), ("width", C.c_int32),
                ("height", C.c_int32)]


class Colormap(C.Structure):
    _fields_ = [("n", C.c_int32), ("rgb", C.c_void_p)]


class ParamsS(C.Structure):
    _fields_ = [("chi", C.c_float), ("brightness", C.c_float * MAX_SPECIES),
                ("fixed_sigma_frac", C.c_float * MAX_SPECIES), ("scalar_min", C.c_float),
                ("scalar_max", C.c_float), ("scalar_log10", C.c_int32), ("col_norm", C.c_int32),
                ("accum", C.c_int32), ("frac_bits", C.c_int32), ("tile", C.c_int32),
                ("halo", C.c_int32), ("max_clip_tiles", C.c_int32), ("chunk", C.c_int32),
                ("colour_mode", C.c_int32), ("transfer", C.c_int32),
                ("absorption", C.c_float * MAX_SPECIES), ("prefilter", C.c_float)]


class Image(C.Structure):
    _fields_ = [("rgb", C.c_void_p), ("log_accum", C.c_void_p), ("center_count", C.c_void_p),
                ("region_mask", C.c_void_p), ("region_size", C.c_int32)]


class Job(C.Structure):
    _fields_ = [("particles", Particles), ("camera", CameraS), ("colormap", Colormap),
                ("params", ParamsS), ("image", Image)]


class Stats(C.Structure):
    _fields_ = [("n_input", C.c_int64), ("n_active", C.c_int64), ("n_entries", C.c_int64),
                ("n_large", C.c_int64), ("n_items", C.c_int64), ("overflow", C.c_int32),
                ("passes", C.c_int32), ("tile", C.c_int32), ("halo", C.c_int32),
                ("max_clip_tiles", C.c_int32), ("chunk", C.c_int32),
                ("radius_hist", C.c_int64 * 5), ("radius_mean", C.c_double),
                ("n_samples", C.c_int64)]


_lib = None


class SplotchError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} ({status})")
        self.status = status


def load():
    """Load the built library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not LIB_PATH.exists():
            raise RuntimeError(f"{LIB_PATH} is not built: run __graft_entry__.build() first")
        lib = C.CDLL(str(LIB_PATH))
        lib.splotch_status_string.restype = C.c_char_p
        lib.splotch_last_error.restype = C.c_char_p
        lib.splotch_last_error.argtypes = [C.c_void_p]
        lib.splotch_abi_version.restype = C.c_int32
        for name in ("splotch_default_params", "splotch_ctx_create", "splotch_ctx_destroy",
                     "splotch_render_workspace_size", "splotch_render", "splotch_get_stats",
                     "splotch_set_timing", "splotch_get_stage_times",
                     "splotch_batch_workspace_size", "splotch_render_batched",
                     "splotch_autotune", "splotch_tune_save", "splotch_tune_load"):
            getattr(lib, name).restype = C.c_int32
        lib.splotch_ctx_create.argtypes = [C.POINTER(C.c_void_p), C.c_int32]
        lib.splotch_ctx_destroy.argtypes = [C.c_void_p]
        lib.splotch_render_workspace_size.argtypes = [C.c_void_p, C.POINTER(Particles),
                                                      C.POINTER(CameraS), C.POINTER(ParamsS),
                                                      C.POINTER(C.c_size_t)]
        lib.splotch_render.argtypes = [C.c_void_p, C.POINTER(Particles), C.POINTER(CameraS),
                                       C.POINTER(Colormap), C.POINTER(ParamsS), C.POINTER(Image),
                                       C.c_void_p, C.c_size_t, C.c_void_p]
        lib.splotch_render_noalloc.restype = C.c_int32
        lib.splotch_render_noalloc.argtypes = [C.c_void_p, C.POINTER(Particles),
                                               C.POINTER(CameraS), C.POINTER(Colormap),
                                               C.POINTER(ParamsS), C.POINTER(Image), C.c_void_p]
        lib.splotch_get_stats.argtypes = [C.c_void_p, C.c_void_p, C.POINTER(Stats)]
        lib.splotch_set_timing.argtypes = [C.c_void_p, C.c_int32]
        lib.splotch_batch_workspace_size.argtypes = [C.c_void_p, C.POINTER(Job), C.c_int32,
                                                     C.POINTER(C.c_size_t)]
        lib.splotch_render_batched.argtypes = [C.c_void_p, C.POINTER(Job), C.c_int32, C.c_void_p,
                                               C.c_size_t, C.c_void_p]
        for name in ("splotch_set_radius_stats", "splotch_set_sample_count"):
            getattr(lib, name).restype = C.c_int32
            getattr(lib, name).argtypes = [C.c_void_p, C.c_int32]
        for name in ("splotch_render_stream_workspace_size", "splotch_render_streamed"):
            getattr(lib, name).restype = C.c_int32
        lib.splotch_render_stream_workspace_size.argtypes = [
            C.c_void_p, C.POINTER(Particles), C.POINTER(CameraS), C.POINTER(ParamsS), C.c_int64,
            C.POINTER(C.c_size_t)]
        lib.splotch_render_streamed.argtypes = [
            C.c_void_p, C.POINTER(Particles), C.POINTER(CameraS), C.POINTER(Colormap),
            C.POINTER(ParamsS), C.POINTER(Image), C.c_int64, C.c_void_p, C.c_size_t, C.c_void_p]
        lib.splotch_autotune.argtypes = [C.c_void_p, C.POINTER(Job), C.c_void_p, C.c_size_t,
                                         C.c_void_p, C.POINTER(ParamsS), C.POINTER(C.c_float)]
        lib.splotch_tune_save.argtypes = [C.c_void_p, C.c_char_p]
        lib.splotch_tune_load.argtypes = [C.c_void_p, C.c_char_p]
        lib.splotch_get_stage_times.argtypes = [C.c_void_p, C.c_void_p, C.POINTER(C.c_float),
                                                C.POINTER(C.c_int32)]
        _lib = lib
    return _lib


def camera_struct(cam) -> CameraS:
    c = CameraS()
    for k in range(3):
        c.eye[k], c.target[k], c.up[k] = cam.eye[k], cam.target[k], cam.up[k]
    c.fov_deg, c.z_near = cam.fov_deg, cam.z_near
    c.width, c.height = int(cam.width), int(cam.height)
    return c


def params_struct(prm) -> ParamsS:
    p = ParamsS()
    p.chi = prm.chi
    for k in range(MAX_SPECIES):
        p.brightness[k] = prm.brightness[k]
        p.fixed_sigma_frac[k] = prm.fixed_sigma_frac[k]
    p.scalar_min, p.scalar_max = prm.scalar_min, prm.scalar_max
    p.scalar_log10, p.col_norm = int(prm.scalar_log10), int(prm.col_norm)
    p.accum, p.frac_bits = int(prm.accum), int(prm.frac_bits)
    p.tile, p.halo = int(prm.tile), int(prm.halo)
    p.max_clip_tiles, p.chunk = int(prm.max_clip_tiles), int(prm.chunk)
    p.colour_mode = int(getattr(prm, "colour_mode", 0))
    p.transfer = int(getattr(prm, "transfer", 0))
    for k in range(MAX_SPECIES):
        p.absorption[k] = getattr(prm, "absorption", (0.0,) * MAX_SPECIES)[k]
    p.prefilter = float(getattr(prm, "prefilter", 0.0))
    return p


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _check_dev(t, dtype, name):
    import torch
    if t is None:
        return
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous {dtype} tensor")


_REQUIRED = ("x", "y", "z", "h", "intensity")
_OPTIONAL = ("scalar", "vx", "vy", "vz")   # the colour mode says which are read


def _struct_of(parts: dict, check) -> Particles:
    n = int(parts["x"].numel())
    for k in _REQUIRED + _OPTIONAL + ("species",):
        t = parts.get(k)
        if t is None:
            if k in _REQUIRED:
                raise ValueError(f"particle array {k} missing")
            continue
        check(t, k)
        if t.numel() != n:
            raise ValueError(f"particle array {k} has the wrong length")
    if len({parts.get(k) is None for k in ("vx", "vy", "vz")}) != 1:
        raise ValueError("vx, vy and vz go together")
    return Particles(n, *(_ptr(parts.get(k)) for k in _REQUIRED + ("scalar", "species", "vx",
                                                                     "vy", "vz")))


def particles_struct(parts: dict) -> Particles:
    """``parts``: dict of device tensors x, y, z, h, intensity (float32,
    contiguous, same length), the colour input (scalar for the palette
    mode, vx, vy, vz for the vector mode) and optional species (uint8)."""
    import torch

    def check(t, k):
        _check_dev(t, torch.uint8 if k == "species" else torch.float32, k)
    return _struct_of(parts, check)


def host_particles_struct(parts: dict) -> Particles:
    """``parts``: the arrays of ``particles_struct`` as CPU torch tensors
    (page-locked for overlapped copies)."""
    import torch

    def check(t, k):
        want = torch.uint8 if k == "species" else torch.float32
        if t.is_cuda or t.dtype != want or not t.is_contiguous():
            raise ValueError(f"{k} must be a contiguous host {want} tensor")
    return _struct_of(parts, check)


def _colormap(cmap) -> Colormap:
    """Palette struct; None (allowed in the vector colour mode) is empty."""
    import torch
    if cmap is None:
        return Colormap(0, None)
    _check_dev(cmap, torch.float32, "colormap")
    return Colormap(int(cmap.numel() // 3), _ptr(cmap))


def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


class Renderer:
    """One library context on one device."""

    def __init__(self, device: int = 0):
        self.lib = load()
        self.device = device
        h = C.c_void_p()
        st = self.lib.splotch_ctx_create(C.byref(h), int(device))
        if st != OK:
            raise SplotchError(st, "splotch_ctx_create failed")
        self.ctx = h
        self._ws = None

    def close(self):
        if self.ctx:
            self.lib.splotch_ctx_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _err(self, st, what):
        msg = self.lib.splotch_last_error(self.ctx).decode()
        raise SplotchError(st, f"{what}: {msg}")

    def workspace_size(self, parts_s: Particles, cam, prm) -> int:
        out = C.c_size_t()
        st = self.lib.splotch_render_workspace_size(self.ctx, C.byref(parts_s),
                                                    C.byref(camera_struct(cam)),
                                                    C.byref(params_struct(prm)), C.byref(out))
        if st != OK:
            self._err(st, "splotch_render_workspace_size")
        return int(out.value)

    def workspace(self, nbytes: int):
        """A cached device workspace of at least nbytes (torch allocation)."""
        import torch
        if self._ws is None or self._ws.numel() < nbytes:
            self._ws = torch.empty(max(nbytes, 256), dtype=torch.uint8,
                                   device=f"cuda:{self.device}")
        return self._ws

    def render(self, parts: dict, cam, cmap, prm, rgb=None, log_accum=None, center_count=None,
               workspace=None, workspace_bytes=None, stream=None, region_mask=None,
               region_size=64):
        """Render into ``rgb`` (H x W x 3 float32 device tensor; allocated if
        None).  Returns rgb.  Asynchronous on ``stream``.  region_mask: uint8
        device tensor with one byte per region of region_size pixels (only
        the marked regions are drawn and written)."""
        import torch
        W, H = int(cam.width), int(cam.height)
        if rgb is None:
            rgb = torch.empty((H, W, 3), dtype=torch.float32, device=f"cuda:{self.device}")
        _check_dev(rgb, torch.float32, "rgb")
        _check_dev(log_accum, torch.float32, "log_accum")
        _check_dev(center_count, torch.int32, "center_count")
        for t, shape in ((rgb, (H, W, 3)), (log_accum, (H, W, 3)), (center_count, (H, W))):
            if t is not None and tuple(t.shape) != shape:
                raise ValueError(f"output shape {tuple(t.shape)} != {shape}")
        ps = particles_struct(parts)
        cs, pr = camera_struct(cam), params_struct(prm)
        if workspace is None:
            need = self.workspace_size(ps, cam, prm)
            workspace = self.workspace(need)
            workspace_bytes = need
        elif workspace_bytes is None:
            workspace_bytes = workspace.numel() * workspace.element_size()
        cm = _colormap(cmap)
        if region_mask is not None:
            _check_dev(region_mask, torch.uint8, "region_mask")
            nrx, nry = -(-W // int(region_size)), -(-H // int(region_size))
            if region_mask.numel() != nrx * nry:
                raise ValueError(f"region_mask needs {nry} x {nrx} entries")
        img = Image(_ptr(rgb), _ptr(log_accum), _ptr(center_count), _ptr(region_mask),
                    int(region_size) if region_mask is not None else 0)
        st = self.lib.splotch_render(self.ctx, C.byref(ps), C.byref(cs), C.byref(cm), C.byref(pr),
                                     C.byref(img), _ptr(workspace), C.c_size_t(workspace_bytes),
                                     _stream_ptr(stream))
        if st != OK:
            self._err(st, "splotch_render")
        return rgb

    def render_noalloc(self, parts: dict, cam, cmap, prm, rgb, log_accum=None,
                       center_count=None, stream=None):
        """The allocation-free render (splotch_render_noalloc): the library's
        fixed per-device scratch is the workspace; every output tensor is
        given by the caller.  Returns rgb.  Asynchronous on ``stream``."""
        import torch
        W, H = int(cam.width), int(cam.height)
        _check_dev(rgb, torch.float32, "rgb")
        _check_dev(log_accum, torch.float32, "log_accum")
        _check_dev(center_count, torch.int32, "center_count")
        for t, shape in ((rgb, (H, W, 3)), (log_accum, (H, W, 3)), (center_count, (H, W))):
            if t is not None and tuple(t.shape) != shape:
                raise ValueError(f"output shape {tuple(t.shape)} != {shape}")
        ps = particles_struct(parts)
        img = Image(_ptr(rgb), _ptr(log_accum), _ptr(center_count))
        st = self.lib.splotch_render_noalloc(self.ctx, C.byref(ps), C.byref(camera_struct(cam)),
                                             C.byref(_colormap(cmap)),
                                             C.byref(params_struct(prm)), C.byref(img),
                                             _stream_ptr(stream))
        if st != OK:
            self._err(st, "splotch_render_noalloc")
        return rgb

    def stream_workspace_size(self, host_parts: dict, cam, prm, chunk: int) -> int:
        out = C.c_size_t()
        st = self.lib.splotch_render_stream_workspace_size(
            self.ctx, C.byref(host_particles_struct(host_parts)), C.byref(camera_struct(cam)),
            C.byref(params_struct(prm)), C.c_int64(int(chunk)), C.byref(out))
        if st != OK:
            self._err(st, "splotch_render_stream_workspace_size")
        return int(out.value)

    def render_streamed(self, host_parts: dict, cam, cmap, prm, chunk: int, rgb=None,
                        log_accum=None, center_count=None, workspace=None, stream=None):
        """Render particles held in host memory (see splotch_render_streamed).
        The host tensors must stay alive until the stream has finished."""
        import torch
        W, H = int(cam.width), int(cam.height)
        if rgb is None:
            rgb = torch.empty((H, W, 3), dtype=torch.float32, device=f"cuda:{self.device}")
        _check_dev(rgb, torch.float32, "rgb")
        _check_dev(log_accum, torch.float32, "log_accum")
        _check_dev(center_count, torch.int32, "center_count")
        ps = host_particles_struct(host_parts)
        need = self.stream_workspace_size(host_parts, cam, prm, chunk)
        if workspace is None:
            workspace = self.workspace(need)
        nbytes = workspace.numel() * workspace.element_size()
        cm = _colormap(cmap)
        img = Image(_ptr(rgb), _ptr(log_accum), _ptr(center_count))
        st = self.lib.splotch_render_streamed(self.ctx, C.byref(ps), C.byref(camera_struct(cam)),
                                              C.byref(cm), C.byref(params_struct(prm)),
                                              C.byref(img), C.c_int64(int(chunk)),
                                              _ptr(workspace), C.c_size_t(nbytes),
                                              _stream_ptr(stream))
        if st != OK:
            self._err(st, "splotch_render_streamed")
        return rgb

    def _job(self, parts, cam, cmap, prm, rgb, log_accum=None, center_count=None) -> Job:
        import torch
        W, H = int(cam.width), int(cam.height)
        _check_dev(rgb, torch.float32, "rgb")
        _check_dev(log_accum, torch.float32, "log_accum")
        _check_dev(center_count, torch.int32, "center_count")
        for t, shape in ((rgb, (H, W, 3)), (log_accum, (H, W, 3)), (center_count, (H, W))):
            if t is not None and tuple(t.shape) != shape:
                raise ValueError(f"output shape {tuple(t.shape)} != {shape}")
        return Job(particles_struct(parts), camera_struct(cam),
                   _colormap(cmap), params_struct(prm),
                   Image(_ptr(rgb), _ptr(log_accum), _ptr(center_count)))

    def make_jobs(self, specs):
        """specs: list of dicts with parts, cam, cmap, prm, rgb (and optional
        log_accum, center_count).  Returns a ctypes array of splotch_job."""
        arr = (Job * len(specs))()
        for i, sp in enumerate(specs):
            arr[i] = self._job(sp["parts"], sp["cam"], sp["cmap"], sp["prm"], sp["rgb"],
                               sp.get("log_accum"), sp.get("center_count"))
        return arr

    def batch_workspace_size(self, jobs) -> int:
        out = C.c_size_t()
        st = self.lib.splotch_batch_workspace_size(self.ctx, jobs, len(jobs), C.byref(out))
        if st != OK:
            self._err(st, "splotch_batch_workspace_size")
        return int(out.value)

    def render_batched(self, jobs, workspace=None, workspace_bytes=None, stream=None):
        """Render a ctypes job array (see make_jobs) in one batched launch."""
        if workspace is None:
            need = self.batch_workspace_size(jobs)
            workspace = self.workspace(need)
            workspace_bytes = need
        elif workspace_bytes is None:
            workspace_bytes = workspace.numel() * workspace.element_size()
        st = self.lib.splotch_render_batched(self.ctx, jobs, len(jobs), _ptr(workspace),
                                             C.c_size_t(workspace_bytes), _stream_ptr(stream))
        if st != OK:
            self._err(st, "splotch_render_batched")

    def autotune(self, parts, cam, cmap, prm, rgb, workspace=None, workspace_bytes=None,
                 stream=None):
        """Tune the schedule for this job's size bucket; returns (Params, ms)."""
        from dataclasses import replace
        job = self._job(parts, cam, cmap, prm, rgb)
        if workspace is None:
            need = self.workspace_size(job.particles, cam, prm)
            workspace = self.workspace(need)
            workspace_bytes = need
        elif workspace_bytes is None:
            workspace_bytes = workspace.numel() * workspace.element_size()
        best = ParamsS()
        ms = C.c_float()
        st = self.lib.splotch_autotune(self.ctx, C.byref(job), _ptr(workspace),
                                       C.c_size_t(workspace_bytes), _stream_ptr(stream),
                                       C.byref(best), C.byref(ms))
        if st != OK:
            self._err(st, "splotch_autotune")
        return replace(prm, tile=best.tile, halo=best.halo, max_clip_tiles=best.max_clip_tiles,
                       chunk=best.chunk), float(ms.value)

    def tune_save(self, path):
        st = self.lib.splotch_tune_save(self.ctx, str(path).encode())
        if st != OK:
            self._err(st, "splotch_tune_save")

    def tune_load(self, path):
        st = self.lib.splotch_tune_load(self.ctx, str(path).encode())
        if st != OK:
            self._err(st, "splotch_tune_load")

    def set_radius_stats(self, on: bool):
        """Collect the radius histogram and mean radius in later renders."""
        st = self.lib.splotch_set_radius_stats(self.ctx, int(bool(on)))
        if st != OK:
            self._err(st, "splotch_set_radius_stats")

    def set_sample_count(self, on: bool):
        """Count the samples drawn (stats()["n_samples"]) in later renders."""
        st = self.lib.splotch_set_sample_count(self.ctx, int(bool(on)))
        if st != OK:
            self._err(st, "splotch_set_sample_count")

    def set_timing(self, on: bool):
        st = self.lib.splotch_set_timing(self.ctx, 1 if on else 0)
        if st != OK:
            self._err(st, "splotch_set_timing")

    def stage_times(self, stream=None):
        """(per-stage milliseconds summed over the timed renders, count)."""
        ms = (C.c_float * NUM_STAGES)()
        n = C.c_int32()
        st = self.lib.splotch_get_stage_times(self.ctx, _stream_ptr(stream), ms, C.byref(n))
        if st != OK:
            self._err(st, "splotch_get_stage_times")
        return dict(zip(STAGES, list(ms))), int(n.value)

    def stats(self, stream=None, check=True) -> dict:
        s = Stats()
        st = self.lib.splotch_get_stats(self.ctx, _stream_ptr(stream), C.byref(s))
        if st not in (OK, ERR_OVERFLOW) or (check and st != OK):
            self._err(st, "splotch_get_stats")
        out = {k: getattr(s, k) for k, _ in Stats._fields_}
        out["radius_hist"] = list(out["radius_hist"])
        return out


def to_host(ps, pinned=True) -> dict:
    """Host torch tensors of a ParticleSet (page-locked if pinned)."""
    import torch
    out = {}
    for k, v in ps.arrays().items():
        if v is None:
            continue
        t = torch.from_numpy(np.ascontiguousarray(v))
        out[k] = t.pin_memory() if pinned else t
    return out


def to_device(ps, device="cuda:0") -> dict:
    """Copy a host ParticleSet (synth.ParticleSet) to device tensors."""
    import torch
    out = {}
    for k, v in ps.arrays().items():
        if v is None:
            out[k] = None
            continue
        out[k] = torch.from_numpy(np.ascontiguousarray(v)).to(device)
    return out
