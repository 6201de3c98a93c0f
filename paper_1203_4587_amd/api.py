"""Python binding of libcsmri: argument marshalling only.

Every array is a torch CUDA tensor (complex64 / uint8, C-contiguous) whose
device pointer is handed to the C ABI together with torch's current stream;
the plan's own device memory comes from torch's caching allocator through
the ABI's allocator callback.  No reconstruction arithmetic happens here.

Layouts (see include/csmri.h): image (nt, nv, nh), k-space (nt, nc, nv, nh),
coil maps (nc, nv, nh), mask (nt, nv) uint8.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import torch

from . import _lib
from ._lib import CsAllocator, CsPlanDesc, CsState, check

PRIORS = {"tv": _lib.CS_PRIOR_TEMPORAL_TV, "dft": _lib.CS_PRIOR_TEMPORAL_DFT,
          "frame": _lib.CS_PRIOR_TEMPORAL_FRAME}


def _ptr(t: torch.Tensor) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream=None) -> ctypes.c_void_p:
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _need(t: torch.Tensor, name: str, dtype: torch.dtype, shape) -> None:
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be on a CUDA/HIP device")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")


class _TorchAllocator:
    """cs_allocator backed by torch's caching allocator on one device."""

    def __init__(self, device: int):
        self.device = device
        self.live = {}

        def alloc(nbytes, ctx):
            try:
                ptr = torch.cuda.caching_allocator_alloc(int(nbytes), self.device)
            except RuntimeError:
                return None
            self.live[ptr] = nbytes
            return ptr

        def free(ptr, ctx):
            if ptr in self.live:
                del self.live[ptr]
                torch.cuda.caching_allocator_delete(ptr)

        self._alloc = _lib.ALLOC_FN(alloc)
        self._free = _lib.FREE_FN(free)
        self.struct = CsAllocator(self._alloc, self._free, None)


@dataclass
class State:
    """Solver state in image layout (see cs_state in include/csmri.h).

    TV   : s0 = m, s1 = d1 (nt-1 frames), s2 = x, s3 = d2
    DFT  : s0 = w, s1 = v, s2 = d, s3 unused
    frame: s0 = w, s1 = v, s2 = d (2 nt coefficient frames each), s3 unused
    """
    s0: torch.Tensor
    s1: torch.Tensor
    s2: torch.Tensor
    s3: torch.Tensor | None
    iter: int = 0

    @classmethod
    def empty(cls, prior: str, nt: int, nv: int, nh: int, device) -> "State":
        def img(frames):
            return torch.zeros((frames, nv, nh), dtype=torch.complex64, device=device)
        if prior == "tv":
            return cls(img(nt), img(nt - 1), img(nt), img(nt), 0)
        if prior == "frame":
            return cls(img(2 * nt), img(2 * nt), img(2 * nt), None, 0)
        return cls(img(nt), img(nt), img(nt), None, 0)


class Plan:
    """A reconstruction plan for one dynamic slice (cs_plan_create)."""

    def __init__(self, coil: torch.Tensor, mask: torch.Tensor, mu: float, prior: str = "tv",
                 mu_ratio: float = 0.5, flags: int = 0, use_torch_allocator: bool = True, stream=None):
        lib = _lib.load()
        if prior not in PRIORS:
            raise ValueError(f"prior must be one of {sorted(PRIORS)}")
        if coil.dim() != 3 or mask.dim() != 2:
            raise ValueError("coil must be (nc, nv, nh) and mask (nt, nv)")
        nc, nv, nh = coil.shape
        nt = mask.shape[0]
        _need(coil, "coil", torch.complex64, (nc, nv, nh))
        _need(mask, "mask", torch.uint8, (nt, nv))
        self.nv, self.nh, self.nt, self.nc = int(nv), int(nh), int(nt), int(nc)
        self.prior = prior
        self.device = coil.device
        self.desc = CsPlanDesc(self.nv, self.nh, self.nt, self.nc, PRIORS[prior], float(mu_ratio), int(flags))
        self._alloc = _TorchAllocator(coil.device.index or 0) if use_torch_allocator else None
        handle = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            st = lib.cs_plan_create(ctypes.byref(self.desc), _ptr(coil), _ptr(mask), float(mu),
                                    ctypes.byref(self._alloc.struct) if self._alloc else None,
                                    _stream(stream), ctypes.byref(handle))
        check(st, "cs_plan_create")
        self._h = handle
        self.mu = float(mu)

    # -- lifetime
    def close(self) -> None:
        if getattr(self, "_h", None) and self._h.value:
            _lib.load().cs_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def handle(self) -> ctypes.c_void_p:
        if not self._h or not self._h.value:
            raise RuntimeError("plan is closed")
        return self._h

    @property
    def nbytes(self) -> int:
        n = ctypes.c_size_t()
        check(_lib.load().cs_plan_bytes(self.handle, ctypes.byref(n)), "cs_plan_bytes")
        return n.value

    # -- shapes
    @property
    def image_shape(self):
        return (self.nt, self.nv, self.nh)

    @property
    def kspace_shape(self):
        return (self.nt, self.nc, self.nv, self.nh)

    # -- operators
    def apply_A(self, x: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        _need(x, "x", torch.complex64, self.image_shape)
        y = out if out is not None else torch.empty(self.kspace_shape, dtype=torch.complex64, device=x.device)
        _need(y, "out", torch.complex64, self.kspace_shape)
        check(_lib.load().cs_apply_A(self.handle, _ptr(x), _ptr(y), _stream(stream)), "cs_apply_A")
        return y

    def apply_AH(self, y: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        _need(y, "y", torch.complex64, self.kspace_shape)
        x = out if out is not None else torch.empty(self.image_shape, dtype=torch.complex64, device=y.device)
        _need(x, "out", torch.complex64, self.image_shape)
        check(_lib.load().cs_apply_AH(self.handle, _ptr(y), _ptr(x), _stream(stream)), "cs_apply_AH")
        return x

    def block_inverse(self, b: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        _need(b, "b", torch.complex64, self.image_shape)
        x = out if out is not None else torch.empty(self.image_shape, dtype=torch.complex64, device=b.device)
        _need(x, "out", torch.complex64, self.image_shape)
        check(_lib.load().cs_apply_block_inverse(self.handle, _ptr(b), _ptr(x), _stream(stream)),
              "cs_apply_block_inverse")
        return x

    def kernel_timing(self, enable: bool = True) -> None:
        """Start (or stop) HIP-event timing of every per-iteration kernel launch."""
        check(_lib.load().cs_kernel_timing(self.handle, int(enable)), "cs_kernel_timing")

    def kernel_times(self) -> dict:
        """{kind: (launches, total_ms)} accumulated since timing was enabled."""
        recs = (_lib.CsKernelTime * 8)()
        n = ctypes.c_int()
        check(_lib.load().cs_kernel_times(self.handle, recs, 8, ctypes.byref(n)), "cs_kernel_times")
        return {recs[i].name.decode(): (int(recs[i].launches), float(recs[i].ms)) for i in range(min(n.value, 8))}

    @property
    def flags(self) -> int:
        f = ctypes.c_uint32()
        check(_lib.load().cs_plan_flags(self.handle, ctypes.byref(f)), "cs_plan_flags")
        return f.value

    @flags.setter
    def flags(self, value: int) -> None:
        check(_lib.load().cs_plan_set_flags(self.handle, int(value)), "cs_plan_set_flags")

    @property
    def fft_tiles(self):
        """(columns per workgroup of the vertical FFT passes, sampled rows per
        workgroup of the horizontal ones) in use."""
        c, r = ctypes.c_int32(), ctypes.c_int32()
        check(_lib.load().cs_plan_fft_tiles(self.handle, ctypes.byref(c), ctypes.byref(r)), "cs_plan_fft_tiles")
        return int(c.value), int(r.value)

    @fft_tiles.setter
    def fft_tiles(self, value) -> None:
        check(_lib.load().cs_plan_set_fft_tiles(self.handle, int(value[0]), int(value[1])), "cs_plan_set_fft_tiles")

    def tune(self, y: torch.Tensor, lam: float, iters: int = 10, cache: str | None = None,
             stream=None) -> dict:
        """cs_plan_tune: time every execution form on y, keep the fastest.

        With `cache` (a JSON file path), a previous result for the same device
        and slice shape is reused instead of timing again, and new results are
        stored there.  Returns {"flags": chosen, "candidates": [(flags, ms/iter)]}.
        """
        _need(y, "y", torch.complex64, self.kspace_shape)
        key = "|".join(map(str, (torch.cuda.get_device_name(self.device), self.nv, self.nh, self.nt, self.nc,
                                 self.prior)))
        if cache is not None:
            entry = _tune_cache_read(cache).get(key)
            if entry is not None:
                keep = self.flags & _lib.CS_FLAG_NO_REFACTOR
                self.flags = keep | (int(entry["flags"]) & ~_lib.CS_FLAG_NO_REFACTOR)
                if "fft_tiles" in entry:
                    self.fft_tiles = entry["fft_tiles"]
                return {"flags": self.flags, "candidates": [tuple(c) for c in entry["candidates"]],
                        "fft_tiles": self.fft_tiles, "cached": True}
        recs = (_lib.CsTuneEntry * 8)()
        n = ctypes.c_int32()
        check(_lib.load().cs_plan_tune(self.handle, _ptr(y), float(lam), int(iters), recs, 8, ctypes.byref(n),
                                       _stream(stream)), "cs_plan_tune")
        cands = [(int(recs[i].flags), float(recs[i].ms_per_iter)) for i in range(min(n.value, 8))]
        result = {"flags": self.flags, "candidates": cands, "fft_tiles": self.fft_tiles, "cached": False}
        if cache is not None:
            _tune_cache_write(cache, key, {"flags": result["flags"], "candidates": cands,
                                           "fft_tiles": list(result["fft_tiles"])})
        return result

    def solve_until(self, y: torch.Tensor, lam: float, max_iters: int, tol: float = 1e-3,
                    check_every: int = 5, mu: float | None = None, state: State | None = None,
                    out: torch.Tensor | None = None, stream=None):
        """cs_admm_solve_until: iterate until Delta(k) < tol (checked every
        `check_every` iterations) or max_iters.  Returns (x, iterations, Delta)."""
        _need(y, "y", torch.complex64, self.kspace_shape)
        x = out if out is not None else torch.empty(self.image_shape, dtype=torch.complex64, device=y.device)
        _need(x, "out", torch.complex64, self.image_shape)
        cstate = _state_struct(self, state)
        done = ctypes.c_int32()
        delta = ctypes.c_float()
        st = _lib.load().cs_admm_solve_until(self.handle, _ptr(y), float(lam), float(self.mu if mu is None else mu),
                                             int(max_iters), float(tol), int(check_every), _ptr(x),
                                             ctypes.byref(cstate) if cstate else None, ctypes.byref(done),
                                             ctypes.byref(delta), _stream(stream))
        check(st, "cs_admm_solve_until")
        if mu is not None:
            self.mu = float(mu)
        if cstate is not None:
            state.iter = int(cstate.iter)
        return x, int(done.value), float(delta.value)

    def new_state(self) -> State:
        return State.empty(self.prior, self.nt, self.nv, self.nh, self.device)

    def solve(self, y: torch.Tensor, lam: float, iters: int, mu: float | None = None,
              state: State | None = None, trace: bool = False, out: torch.Tensor | None = None,
              stream=None):
        """cs_admm_solve.  Returns x, or (x, J) with J the per-iteration objective
        (a float32 tensor of length iters) when trace=True."""
        _need(y, "y", torch.complex64, self.kspace_shape)
        x = out if out is not None else torch.empty(self.image_shape, dtype=torch.complex64, device=y.device)
        _need(x, "out", torch.complex64, self.image_shape)
        cstate = _state_struct(self, state)
        J = torch.empty(max(iters, 1), dtype=torch.float32, device=y.device) if trace else None
        st = _lib.load().cs_admm_solve(self.handle, _ptr(y), float(lam), float(self.mu if mu is None else mu),
                                       int(iters), _ptr(x), ctypes.byref(cstate) if cstate else None,
                                       _ptr(J) if J is not None else None, _stream(stream))
        check(st, "cs_admm_solve")
        if mu is not None:
            self.mu = float(mu)
        if cstate is not None:
            state.iter = int(cstate.iter)
        return (x, J[:iters]) if trace else x


def _state_struct(plan: "Plan", state: "State | None"):
    if state is None:
        return None
    nt = plan.nt
    fr = {"tv": (nt, nt - 1, nt, nt), "dft": (nt, nt, nt, None), "frame": (2 * nt, 2 * nt, 2 * nt, None)}[plan.prior]
    for name, frames in zip(("s0", "s1", "s2", "s3"), fr):
        if frames is not None:
            _need(getattr(state, name), f"state.{name}", torch.complex64, (frames, plan.nv, plan.nh))
    return CsState(state.s0.data_ptr(), state.s1.data_ptr(), state.s2.data_ptr(),
                   state.s3.data_ptr() if state.s3 is not None else None, int(state.iter))


def _tune_cache_read(path: str) -> dict:
    import json
    import os
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        return json.load(f)


def _tune_cache_write(path: str, key: str, entry: dict) -> None:
    import json
    import os
    data = _tune_cache_read(path)
    data[key] = entry
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


@dataclass
class Slice:
    """One slice of a batch: coil maps (nc, nv, nh), mask (nt, nv), prior, mu."""
    coil: torch.Tensor
    mask: torch.Tensor
    prior: str = "tv"
    mu: float = 0.1
    mu_ratio: float = 0.5
    flags: int = 0


class _BorrowedPlan(Plan):
    """A plan owned by a batch (cs_batch_plan): usable, never destroyed here."""

    def __init__(self, handle: ctypes.c_void_p, sl: Slice, batch: "Batch"):
        self._h = handle
        self._batch = batch  # keeps the batch alive
        nc, nv, nh = sl.coil.shape
        self.nv, self.nh, self.nt, self.nc = int(nv), int(nh), int(sl.mask.shape[0]), int(nc)
        self.prior = sl.prior
        self.device = sl.coil.device
        self.mu = float(sl.mu)

    def close(self) -> None:
        self._h = ctypes.c_void_p()


class Batch:
    """Many independent slices solved by one graph launch (cs_batch_create / cs_batch_solve)."""

    def __init__(self, slices, use_torch_allocator: bool = True, stream=None):
        lib = _lib.load()
        slices = list(slices)
        if not slices:
            raise ValueError("a batch needs at least one slice")
        descs = (_lib.CsSliceDesc * len(slices))()
        for i, sl in enumerate(slices):
            if sl.prior not in PRIORS:
                raise ValueError(f"slice {i}: prior must be one of {sorted(PRIORS)}")
            if sl.coil.dim() != 3 or sl.mask.dim() != 2:
                raise ValueError(f"slice {i}: coil must be (nc, nv, nh) and mask (nt, nv)")
            nc, nv, nh = sl.coil.shape
            nt = sl.mask.shape[0]
            _need(sl.coil, f"slices[{i}].coil", torch.complex64, (nc, nv, nh))
            _need(sl.mask, f"slices[{i}].mask", torch.uint8, (nt, nv))
            descs[i] = _lib.CsSliceDesc(CsPlanDesc(int(nv), int(nh), int(nt), int(nc), PRIORS[sl.prior],
                                                   float(sl.mu_ratio), int(sl.flags)),
                                        sl.coil.data_ptr(), sl.mask.data_ptr(), float(sl.mu))
        self.slices = slices
        self.device = slices[0].coil.device
        self._alloc = _TorchAllocator(self.device.index or 0) if use_torch_allocator else None
        handle = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            st = lib.cs_batch_create(descs, len(slices), ctypes.byref(self._alloc.struct) if self._alloc else None,
                                     _stream(stream), ctypes.byref(handle))
        check(st, "cs_batch_create")
        self._h = handle

    def close(self) -> None:
        if getattr(self, "_h", None) and self._h.value:
            _lib.load().cs_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __len__(self) -> int:
        return len(self.slices)

    @property
    def handle(self) -> ctypes.c_void_p:
        if not self._h or not self._h.value:
            raise RuntimeError("batch is closed")
        return self._h

    def plan(self, i: int) -> Plan:
        h = ctypes.c_void_p()
        check(_lib.load().cs_batch_plan(self.handle, int(i), ctypes.byref(h)), "cs_batch_plan")
        return _BorrowedPlan(h, self.slices[i], self)

    def image_shape(self, i: int):
        sl = self.slices[i]
        return (int(sl.mask.shape[0]), int(sl.coil.shape[1]), int(sl.coil.shape[2]))

    def kspace_shape(self, i: int):
        sl = self.slices[i]
        return (int(sl.mask.shape[0]), int(sl.coil.shape[0]), int(sl.coil.shape[1]), int(sl.coil.shape[2]))

    def solve(self, ys, lams, iters: int, outs=None, stream=None):
        """cs_batch_solve: ys[i] is slice i's k-space, lams[i] its lambda; returns the images."""
        n = len(self.slices)
        ys = list(ys)
        if len(ys) != n:
            raise ValueError(f"need {n} k-space arrays, got {len(ys)}")
        if isinstance(lams, (int, float)):
            lams = [float(lams)] * n
        lams = [float(v) for v in lams]
        if len(lams) != n:
            raise ValueError(f"need {n} lambdas, got {len(lams)}")
        if outs is None:
            outs = [torch.empty(self.image_shape(i), dtype=torch.complex64, device=self.device) for i in range(n)]
        outs = list(outs)
        for i in range(n):
            _need(ys[i], f"ys[{i}]", torch.complex64, self.kspace_shape(i))
            _need(outs[i], f"outs[{i}]", torch.complex64, self.image_shape(i))
        yp = (ctypes.c_void_p * n)(*[t.data_ptr() for t in ys])
        xp = (ctypes.c_void_p * n)(*[t.data_ptr() for t in outs])
        lp = (ctypes.c_float * n)(*lams)
        check(_lib.load().cs_batch_solve(self.handle, yp, lp, int(iters), xp, _stream(stream)), "cs_batch_solve")
        return outs


def read_stream(buf: torch.Tensor, sink: torch.Tensor, blocks: int = 0, stream=None) -> None:
    """Launch cs_read_stream over the bytes of the contiguous device tensor
    `buf` (a measurement aid: a pure HBM read stream, nothing written in
    practice; `sink` is a device float32 tensor of at least one element)."""
    if not buf.is_cuda or not buf.is_contiguous():
        raise ValueError("buf must be a contiguous device tensor")
    if not sink.is_cuda or sink.dtype != torch.float32 or sink.numel() < 1:
        raise ValueError("sink must be a device float32 tensor with at least one element")
    nbytes = buf.numel() * buf.element_size()
    check(_lib.load().cs_read_stream(_ptr(buf), nbytes, int(blocks), _ptr(sink), _stream(stream)), "cs_read_stream")


def to_device(a, device="cuda", dtype=None) -> torch.Tensor:
    """numpy -> contiguous torch tensor on the GPU (complex128 -> complex64)."""
    import numpy as np
    arr = np.asarray(a)
    if dtype is None:
        dtype = torch.uint8 if arr.dtype == np.uint8 else torch.complex64
    if dtype == torch.complex64:
        arr = arr.astype(np.complex64)
    return torch.from_numpy(np.ascontiguousarray(arr)).to(device=device, dtype=dtype)
