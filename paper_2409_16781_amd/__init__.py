"""MI355X D3Q19 lattice Boltzmann library: Python binding of the C ABI in include/lb.h.

The binding only marshals arguments: every step of the update runs in the
HIP kernels of ``liblbm355.so``.  PyTorch provides device memory and the
stream; there is no CPU fallback, and importing ``Lattice`` without the built
library raises.

Array conventions (torch tensors on the GPU, C-contiguous):
  rho  (nz, ny, nx)      float64 in, float32 out
  u    (3, nz, ny, nx)   float64 in, float32 out (u_x, u_y, u_z)
  f    (19, nz, ny, nx)  raw storage: float32 (LB_F32) or 16-bit words
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "liblbm355.so")

LB_OK, LB_EINVAL, LB_ENOMEM, LB_EHIP, LB_EUNSTABLE, LB_ESTATE = 0, -1, -2, -3, -4, -5
LB_F32, LB_F16S, LB_BF16S, LB_S16 = 0, 1, 2, 3
LB_HOST, LB_DEVICE = 0, 1
LB_INPLACE = 0x100
CODECS = {"f32": LB_F32, "f16": LB_F16S, "bf16": LB_BF16S, "s16": LB_S16}

# Every function the C ABI exports, with its ctypes signature.
_P = ctypes.c_void_p
_SIGNATURES = {
    "lb_create": (_P, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double, _P]),
    "lb_create_ex": (_P, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double, _P, ctypes.c_int, _P]),
    "lb_destroy": (None, [_P]),
    "lb_set_force": (ctypes.c_int, [_P, ctypes.c_double, ctypes.c_double, ctypes.c_double]),
    "lb_init_eq": (ctypes.c_int, [_P, _P, _P]),
    "lb_step": (ctypes.c_int, [_P, ctypes.c_int]),
    "lb_step_noalloc": (ctypes.c_int, [_P, ctypes.c_int]),
    "lb_step_macros": (ctypes.c_int, [_P, ctypes.c_int, _P, _P]),
    "lb_macros": (ctypes.c_int, [_P, _P, _P]),
    "lb_sums": (ctypes.c_int, [_P, _P, ctypes.c_int]),
    "lb_get_f": (ctypes.c_int, [_P, _P, ctypes.c_size_t, ctypes.c_int]),
    "lb_set_f": (ctypes.c_int, [_P, _P, ctypes.c_size_t, ctypes.c_int]),
    "lb_sync": (ctypes.c_int, [_P]),
    "lb_get_scales": (ctypes.c_int, [_P, _P]),
    "lb_set_scales": (ctypes.c_int, [_P, _P]),
    "lb_last_error": (ctypes.c_char_p, []),
    "lb_steps_done": (ctypes.c_longlong, [_P]),
    "lb_query": (ctypes.c_longlong, [_P, ctypes.c_int]),
    "lb_time_steps": (ctypes.c_int, [_P, ctypes.c_int, _P]),
    "lb_time_step_kernel": (ctypes.c_int, [_P, ctypes.c_int, _P]),
    "lb_tune": (ctypes.c_int, [_P, ctypes.c_int]),
    "lb_copy_probe": (ctypes.c_int, [_P, ctypes.c_int, _P]),
    "lb_set_force_field": (ctypes.c_int, [_P, _P]),
    "lb_grad_force_x": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int, _P, _P]),
    "lb_outlet_flux": (ctypes.c_int, [_P, _P]),
    "lb_grad_outlet_flux_x": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int, _P, _P]),
    "lb2d_create": (_P, [ctypes.c_int, ctypes.c_int, ctypes.c_double, _P, ctypes.c_double, ctypes.c_double, _P]),
    "lb2d_destroy": (None, [_P]),
    "lb2d_init_eq": (ctypes.c_int, [_P, _P, _P]),
    "lb2d_step": (ctypes.c_int, [_P, ctypes.c_int]),
    "lb2d_macros": (ctypes.c_int, [_P, _P, _P]),
    "lb2d_sums": (ctypes.c_int, [_P, _P, ctypes.c_int]),
    "lb2d_get_f": (ctypes.c_int, [_P, _P, ctypes.c_size_t, ctypes.c_int]),
    "lb2d_set_f": (ctypes.c_int, [_P, _P, ctypes.c_size_t, ctypes.c_int]),
    "lb2d_sync": (ctypes.c_int, [_P]),
    "lb2d_steps_done": (ctypes.c_longlong, [_P]),
    "lb2d_time_steps": (ctypes.c_int, [_P, ctypes.c_int, _P]),
    "lb_batch_create": (_P, [ctypes.c_int, _P, _P, _P, ctypes.c_int, _P, ctypes.c_int]),
    "lb_batch_destroy": (None, [_P]),
    "lb_batch_set_force": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double]),
    "lb_batch_init_eq": (ctypes.c_int, [_P, ctypes.c_int, _P, _P]),
    "lb_batch_step": (ctypes.c_int, [_P, ctypes.c_int]),
    "lb_batch_macros": (ctypes.c_int, [_P, ctypes.c_int, _P, _P]),
    "lb_batch_sums": (ctypes.c_int, [_P, ctypes.c_int, _P, ctypes.c_int]),
    "lb_batch_get_f": (ctypes.c_int, [_P, ctypes.c_int, _P, ctypes.c_size_t, ctypes.c_int]),
    "lb_batch_set_f": (ctypes.c_int, [_P, ctypes.c_int, _P, ctypes.c_size_t, ctypes.c_int]),
    "lb_batch_sync": (ctypes.c_int, [_P]),
    "lb_batch_steps_done": (ctypes.c_longlong, [_P]),
    "lb_batch_query": (ctypes.c_longlong, [_P, ctypes.c_int]),
    "lb_batch_time_steps": (ctypes.c_int, [_P, ctypes.c_int, _P]),
    "lb_batch_time_step_kernel": (ctypes.c_int, [_P, ctypes.c_int, _P]),
}

_lib = None


class LBError(RuntimeError):
    def __init__(self, code: int, where: str, msg: str):
        super().__init__(f"{where} failed ({code}): {msg}")
        self.code = code


def lib() -> ctypes.CDLL:
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2409_16781_amd._build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def last_error() -> str:
    return lib().lb_last_error().decode()


def _check(rc: int, where: str):
    if rc != LB_OK:
        raise LBError(rc, where, last_error())
    return rc


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


class Lattice:
    """A D3Q19 lattice on the GPU (owns the library handle).

    ``stream``: a torch.cuda.Stream, or None for torch's current stream.
    """

    def __init__(self, nx: int, ny: int, nz: int, tau: float, flags=None, codec: str = "f32", stream=None,
                 inplace: bool = False):
        import torch

        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self.n = self.nx * self.ny * self.nz
        self.codec = codec
        if codec not in CODECS:
            raise ValueError(f"codec must be one of {sorted(CODECS)}")
        self._stream = stream if stream is not None else torch.cuda.current_stream()
        fl = None
        if flags is not None:
            fl = np.ascontiguousarray(flags, dtype=np.uint8)
            if fl.shape != (self.nz, self.ny, self.nx):
                raise ValueError("flags must have shape (nz, ny, nx)")
        self._flags = fl
        h = lib().lb_create_ex(self.nx, self.ny, self.nz, float(tau),
                               None if fl is None else fl.ctypes.data_as(ctypes.c_void_p),
                               CODECS[codec] | (LB_INPLACE if inplace else 0),
                               ctypes.c_void_p(self._stream.cuda_stream))
        if not h:
            raise LBError(LB_EINVAL, "lb_create_ex", last_error())
        self._h = ctypes.c_void_p(h)

    # -- lifetime -----------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None):
            lib().lb_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    # -- ABI calls ----------------------------------------------------------
    def set_force(self, fx: float, fy: float = 0.0, fz: float = 0.0):
        _check(lib().lb_set_force(self._h, float(fx), float(fy), float(fz)), "lb_set_force")

    def init_eq(self, rho=None, u=None):
        """rho (nz,ny,nx), u (3,nz,ny,nx): float64 CUDA tensors (or None)."""
        import torch

        for t, shape in ((rho, (self.nz, self.ny, self.nx)), (u, (3, self.nz, self.ny, self.nx))):
            if t is not None:
                if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous() or tuple(t.shape) != shape:
                    raise ValueError(f"expected a contiguous float64 CUDA tensor of shape {shape}")
        _check(lib().lb_init_eq(self._h, _ptr(rho), _ptr(u)), "lb_init_eq")

    def step(self, n: int = 1):
        _check(lib().lb_step(self._h, int(n)), "lb_step")

    def step_noalloc(self, n: int = 1):
        """As step(), with no device allocation in the call (the totals'
        scratch is the library's static per-device array)."""
        _check(lib().lb_step_noalloc(self._h, int(n)), "lb_step_noalloc")

    def step_macros(self, n: int = 1):
        """n steps; the last one also returns its (rho, u) as float32 tensors."""
        import torch

        rho = torch.empty((self.nz, self.ny, self.nx), dtype=torch.float32, device="cuda")
        u = torch.empty((3, self.nz, self.ny, self.nx), dtype=torch.float32, device="cuda")
        _check(lib().lb_step_macros(self._h, int(n), _ptr(rho), _ptr(u)), "lb_step_macros")
        return rho, u

    def macros(self):
        import torch

        rho = torch.empty((self.nz, self.ny, self.nx), dtype=torch.float32, device="cuda")
        u = torch.empty((3, self.nz, self.ny, self.nx), dtype=torch.float32, device="cuda")
        _check(lib().lb_macros(self._h, _ptr(rho), _ptr(u)), "lb_macros")
        return rho, u

    def sums(self, k: int = 1) -> np.ndarray:
        out = np.zeros((k, 4), dtype=np.float64)
        rc = lib().lb_sums(self._h, out.ctypes.data_as(ctypes.c_void_p), int(k))
        if rc == LB_EUNSTABLE:
            raise LBError(rc, "lb_sums", last_error())
        _check(rc, "lb_sums")
        return out

    def _raw_dtype(self):
        return np.float32 if self.codec == "f32" else np.uint16

    def get_scales(self) -> np.ndarray:
        """Exponents of scaled 16-bit storage (codec "s16") for the rest, axis
        and diagonal populations: g_i = code * 2^-e."""
        out = np.zeros(3, dtype=np.int32)
        _check(lib().lb_get_scales(self._h, out.ctypes.data_as(ctypes.c_void_p)), "lb_get_scales")
        return out

    def set_scales(self, exps):
        e = np.ascontiguousarray(exps, dtype=np.int32)
        if e.shape != (3,):
            raise ValueError("3 exponents expected (rest, axis, diagonal)")
        _check(lib().lb_set_scales(self._h, e.ctypes.data_as(ctypes.c_void_p)), "lb_set_scales")

    def get_f(self) -> np.ndarray:
        """Raw stored state on the host: (19, nz, ny, nx) float32 or uint16 words."""
        out = np.empty((19, self.nz, self.ny, self.nx), dtype=self._raw_dtype())
        _check(lib().lb_get_f(self._h, out.ctypes.data_as(ctypes.c_void_p), out.nbytes, LB_HOST), "lb_get_f")
        return out

    def set_f(self, f: np.ndarray):
        f = np.ascontiguousarray(f, dtype=self._raw_dtype())
        if f.shape != (19, self.nz, self.ny, self.nx):
            raise ValueError("state must have shape (19, nz, ny, nx)")
        _check(lib().lb_set_f(self._h, f.ctypes.data_as(ctypes.c_void_p), f.nbytes, LB_HOST), "lb_set_f")

    def get_f_device(self, out):
        """Raw state into a contiguous CUDA tensor of 19 * N storage elements."""
        if not (out.is_cuda and out.is_contiguous()):
            raise ValueError("expected a contiguous CUDA tensor")
        _check(lib().lb_get_f(self._h, _ptr(out), out.numel() * out.element_size(), LB_DEVICE), "lb_get_f")

    def set_f_device(self, f):
        """Raw state from a contiguous CUDA tensor of 19 * N storage elements."""
        if not (f.is_cuda and f.is_contiguous()):
            raise ValueError("expected a contiguous CUDA tensor")
        _check(lib().lb_set_f(self._h, _ptr(f), f.numel() * f.element_size(), LB_DEVICE), "lb_set_f")

    def sync(self):
        _check(lib().lb_sync(self._h), "lb_sync")

    def set_force_field(self, fx=None):
        """Per-site x-force (float32 CUDA tensor (nz, ny, nx)) added to the
        uniform one; None removes it.  FP32 storage."""
        import torch

        if fx is not None:
            if fx.dtype != torch.float32 or not fx.is_cuda or not fx.is_contiguous() or \
                    tuple(fx.shape) != (self.nz, self.ny, self.nx):
                raise ValueError("expected a contiguous float32 CUDA tensor of shape (nz, ny, nx)")
        self._fx_field = fx
        _check(lib().lb_set_force_field(self._h, _ptr(fx)), "lb_set_force_field")

    def grad_force_x(self, nsteps: int, every: int, seed):
        """Advance nsteps steps and return dJ/dF_x (float32 (nz, ny, nx)) for
        an objective with dJ/dS_N = seed (float32 CUDA tensor (19, nz, ny, nx))."""
        import torch

        if seed.dtype != torch.float32 or not seed.is_cuda or not seed.is_contiguous() or \
                tuple(seed.shape) != (19, self.nz, self.ny, self.nx):
            raise ValueError("seed must be a contiguous float32 CUDA tensor of shape (19, nz, ny, nx)")
        grad = torch.empty((self.nz, self.ny, self.nx), dtype=torch.float32, device="cuda")
        _check(lib().lb_grad_force_x(self._h, int(nsteps), int(every), _ptr(seed), _ptr(grad)), "lb_grad_force_x")
        return grad

    def outlet_flux(self) -> float:
        """J = sum of rho u_x over the fluid sites of the plane x = nx - 1 of
        the current state (lb_outlet_flux; synchronises)."""
        J = ctypes.c_double(0.0)
        _check(lib().lb_outlet_flux(self._h, ctypes.byref(J)), "lb_outlet_flux")
        return J.value

    def grad_outlet_flux_x(self, nsteps: int, every: int):
        """Advance nsteps steps; return (J, dJ/dF_x) of the outlet flux of the
        final state (float, float32 CUDA tensor (nz, ny, nx))."""
        import torch

        grad = torch.empty((self.nz, self.ny, self.nx), dtype=torch.float32, device="cuda")
        J = ctypes.c_double(0.0)
        _check(lib().lb_grad_outlet_flux_x(self._h, int(nsteps), int(every), _ptr(grad), ctypes.byref(J)),
               "lb_grad_outlet_flux_x")
        return J.value, grad

    @property
    def steps_done(self) -> int:
        return int(lib().lb_steps_done(self._h))

    def query(self, key: int) -> int:
        return int(lib().lb_query(self._h, int(key)))

    @property
    def info(self) -> dict:
        keys = ["variant", "sites_per_thread", "solids", "bytes_per_population", "grid", "block_rows", "n_fluid",
                "array_bytes", "inplace", "codec", "rescales", "tile_order", "pull_nt"]
        return {k: self.query(i) for i, k in enumerate(keys)}

    def time_steps(self, n: int) -> float:
        ms = ctypes.c_double(0.0)
        _check(lib().lb_time_steps(self._h, int(n), ctypes.byref(ms)), "lb_time_steps")
        return ms.value

    def tune(self, reps: int = 10) -> dict:
        """Time the step kernel's launch shapes on this lattice and keep the
        fastest (state unchanged); returns the lattice info."""
        _check(lib().lb_tune(self._h, int(reps)), "lb_tune")
        return self.info

    def time_step_kernel(self, n: int) -> float:
        """Mean duration (ms) of the step kernel alone over n eager steps."""
        ms = ctypes.c_double(0.0)
        _check(lib().lb_time_step_kernel(self._h, int(n), ctypes.byref(ms)), "lb_time_step_kernel")
        return ms.value

    def copy_probe(self, reps: int = 10) -> float:
        ms = ctypes.c_double(0.0)
        _check(lib().lb_copy_probe(self._h, int(reps), ctypes.byref(ms)), "lb_copy_probe")
        return ms.value


class Lattice2D:
    """A two-dimensional D2Q9 lattice (the paper's own model); flags (ny, nx)
    with 0 fluid, 1 wall, 2 lid moving with velocity ``lid``."""

    def __init__(self, nx: int, ny: int, tau: float, flags=None, lid=(0.0, 0.0), stream=None):
        import torch

        self.nx, self.ny = int(nx), int(ny)
        self.n = self.nx * self.ny
        fl = None
        if flags is not None:
            fl = np.ascontiguousarray(flags, dtype=np.uint8)
            if fl.shape != (self.ny, self.nx):
                raise ValueError("flags must have shape (ny, nx)")
        self._flags = fl
        self._stream = stream if stream is not None else torch.cuda.current_stream()
        h = lib().lb2d_create(self.nx, self.ny, float(tau), None if fl is None else fl.ctypes.data_as(ctypes.c_void_p),
                              float(lid[0]), float(lid[1]), ctypes.c_void_p(self._stream.cuda_stream))
        if not h:
            raise LBError(LB_EINVAL, "lb2d_create", last_error())
        self._h = ctypes.c_void_p(h)

    def close(self):
        if getattr(self, "_h", None):
            lib().lb2d_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init_eq(self, rho=None, u=None):
        """rho (ny, nx), u (2, ny, nx): float64 CUDA tensors (or None)."""
        import torch

        for t, shape in ((rho, (self.ny, self.nx)), (u, (2, self.ny, self.nx))):
            if t is not None and (tuple(t.shape) != shape or t.dtype != torch.float64 or not t.is_cuda
                                  or not t.is_contiguous()):
                raise ValueError(f"expected a contiguous float64 CUDA tensor of shape {shape}")
        _check(lib().lb2d_init_eq(self._h, _ptr(rho), _ptr(u)), "lb2d_init_eq")

    def step(self, n: int = 1):
        _check(lib().lb2d_step(self._h, int(n)), "lb2d_step")

    def macros(self):
        import torch

        rho = torch.empty((self.ny, self.nx), dtype=torch.float32, device="cuda")
        u = torch.empty((2, self.ny, self.nx), dtype=torch.float32, device="cuda")
        _check(lib().lb2d_macros(self._h, _ptr(rho), _ptr(u)), "lb2d_macros")
        return rho, u

    def sums(self, k: int = 1) -> np.ndarray:
        out = np.zeros((k, 3), dtype=np.float64)
        rc = lib().lb2d_sums(self._h, out.ctypes.data_as(ctypes.c_void_p), int(k))
        if rc == LB_EUNSTABLE:
            raise LBError(rc, "lb2d_sums", last_error())
        _check(rc, "lb2d_sums")
        return out

    def get_f(self, device: bool = False):
        """Raw state g = f - w as (9, ny, nx) float32: numpy, or a CUDA tensor with device=True."""
        if device:
            import torch

            out = torch.empty((9, self.ny, self.nx), dtype=torch.float32, device="cuda")
            _check(lib().lb2d_get_f(self._h, _ptr(out), out.numel() * 4, LB_DEVICE), "lb2d_get_f")
            return out
        out = np.empty((9, self.ny, self.nx), dtype=np.float32)
        _check(lib().lb2d_get_f(self._h, out.ctypes.data_as(ctypes.c_void_p), out.nbytes, LB_HOST), "lb2d_get_f")
        return out

    def set_f(self, f):
        """Set the raw state from a (9, ny, nx) float32 numpy array or CUDA tensor."""
        if hasattr(f, "is_cuda") and f.is_cuda:
            if tuple(f.shape) != (9, self.ny, self.nx) or str(f.dtype) != "torch.float32" or not f.is_contiguous():
                raise ValueError("state must be a contiguous float32 tensor of shape (9, ny, nx)")
            _check(lib().lb2d_set_f(self._h, _ptr(f), f.numel() * 4, LB_DEVICE), "lb2d_set_f")
            return
        f = np.ascontiguousarray(f, dtype=np.float32)
        if f.shape != (9, self.ny, self.nx):
            raise ValueError("state must have shape (9, ny, nx)")
        _check(lib().lb2d_set_f(self._h, f.ctypes.data_as(ctypes.c_void_p), f.nbytes, LB_HOST), "lb2d_set_f")

    def sync(self):
        _check(lib().lb2d_sync(self._h), "lb2d_sync")

    @property
    def steps_done(self) -> int:
        return int(lib().lb2d_steps_done(self._h))

    def time_steps(self, n: int) -> float:
        ms = ctypes.c_double(0.0)
        _check(lib().lb2d_time_steps(self._h, int(n), ctypes.byref(ms)), "lb2d_time_steps")
        return ms.value


def outlet_flux(lat: "Lattice") -> float:
    """J = sum of rho u_x over the fluid sites of the plane x = nx - 1 of the
    lattice's current state (computed by the library)."""
    return lat.outlet_flux()


def _outlet_flux_function():
    import torch

    class OutletFlux(torch.autograd.Function):
        """J(fx) = outlet flux after ``nsteps`` steps from the lattice's
        current state with per-site x-force field fx.  The backward pass
        restores the saved initial state and runs lb_grad_force_x
        (checkpointed recomputation every ``every`` steps, adjoint kernels);
        the lattice is left at step nsteps after either pass."""

        @staticmethod
        def forward(ctx, fx, lat, nsteps, every):
            state0 = torch.empty((19, lat.nz, lat.ny, lat.nx), dtype=torch.float32, device="cuda")
            lat.get_f_device(state0)
            lat.set_force_field(fx.detach().contiguous())
            lat.step(nsteps)
            J = torch.tensor(lat.outlet_flux(), dtype=torch.float64, device="cuda")
            ctx.lat, ctx.nsteps, ctx.every = lat, nsteps, every
            ctx.save_for_backward(fx.detach(), state0)
            return J

        @staticmethod
        def backward(ctx, gJ):
            fx, state0 = ctx.saved_tensors
            lat = ctx.lat
            lat.set_f_device(state0)
            lat.set_force_field(fx.contiguous())
            _, g = lat.grad_outlet_flux_x(ctx.nsteps, ctx.every)
            return (gJ * g.double()).to(fx.dtype), None, None, None

    return OutletFlux


def outlet_flux_autograd(fx, lat: "Lattice", nsteps: int, every: int):
    """Differentiable outlet flux: torch.autograd sees J as a function of the
    per-site x-force fx (float32 CUDA tensor (nz, ny, nx))."""
    return _outlet_flux_function().apply(fx, lat, int(nsteps), int(every))


class Batch:
    """Many independent D3Q19 lattices advanced by one kernel launch per step.

    ``dims``: list of (nx, ny, nz); ``taus``: one relaxation time per domain;
    ``flags``: None or a list with one (nz, ny, nx) uint8 array (or None) per
    domain; ``autotune``: time the candidate launch shapes once and keep the
    fastest.  Per-domain arrays follow the ``Lattice`` conventions.
    """

    def __init__(self, dims, taus, flags=None, codec: str = "f32", stream=None, autotune: bool = False):
        import torch

        if codec not in CODECS:
            raise ValueError(f"codec must be one of {sorted(CODECS)}")
        self.codec = codec
        self.dims = [tuple(int(v) for v in d) for d in dims]
        self.count = len(self.dims)
        if len(taus) != self.count:
            raise ValueError("one tau per domain")
        dims_arr = np.ascontiguousarray(np.array(self.dims, dtype=np.int32).reshape(-1))
        tau_arr = np.ascontiguousarray(np.array(taus, dtype=np.float64))
        self._keep = [dims_arr, tau_arr]
        fl_ptrs = None
        if flags is not None:
            if len(flags) != self.count:
                raise ValueError("one flag array (or None) per domain")
            arrs = []
            ptrs = (ctypes.c_void_p * self.count)()
            for k, (f, (nx, ny, nz)) in enumerate(zip(flags, self.dims)):
                if f is None:
                    ptrs[k] = None
                    continue
                a = np.ascontiguousarray(f, dtype=np.uint8)
                if a.shape != (nz, ny, nx):
                    raise ValueError(f"flags of domain {k} must have shape {(nz, ny, nx)}")
                arrs.append(a)
                ptrs[k] = a.ctypes.data_as(ctypes.c_void_p)
            self._keep += [arrs, ptrs]
            fl_ptrs = ctypes.cast(ptrs, ctypes.c_void_p)
        self._stream = stream if stream is not None else torch.cuda.current_stream()
        h = lib().lb_batch_create(self.count, dims_arr.ctypes.data_as(ctypes.c_void_p),
                                  tau_arr.ctypes.data_as(ctypes.c_void_p), fl_ptrs, CODECS[codec],
                                  ctypes.c_void_p(self._stream.cuda_stream), 1 if autotune else 0)
        if not h:
            raise LBError(LB_EINVAL, "lb_batch_create", last_error())
        self._h = ctypes.c_void_p(h)

    def close(self):
        if getattr(self, "_h", None):
            lib().lb_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _shape(self, d):
        nx, ny, nz = self.dims[d]
        return nz, ny, nx

    def set_force(self, fx: float, fy: float = 0.0, fz: float = 0.0, domain: int = -1):
        _check(lib().lb_batch_set_force(self._h, int(domain), float(fx), float(fy), float(fz)), "lb_batch_set_force")

    def init_eq(self, d: int, rho=None, u=None):
        import torch

        shp = self._shape(d)
        for t, shape in ((rho, shp), (u, (3,) + shp)):
            if t is not None:
                if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous() or tuple(t.shape) != shape:
                    raise ValueError(f"expected a contiguous float64 CUDA tensor of shape {shape}")
        _check(lib().lb_batch_init_eq(self._h, int(d), _ptr(rho), _ptr(u)), "lb_batch_init_eq")

    def step(self, n: int = 1):
        _check(lib().lb_batch_step(self._h, int(n)), "lb_batch_step")

    def macros(self, d: int):
        import torch

        shp = self._shape(d)
        rho = torch.empty(shp, dtype=torch.float32, device="cuda")
        u = torch.empty((3,) + shp, dtype=torch.float32, device="cuda")
        _check(lib().lb_batch_macros(self._h, int(d), _ptr(rho), _ptr(u)), "lb_batch_macros")
        return rho, u

    def sums(self, d: int, k: int = 1) -> np.ndarray:
        out = np.zeros((k, 4), dtype=np.float64)
        rc = lib().lb_batch_sums(self._h, int(d), out.ctypes.data_as(ctypes.c_void_p), int(k))
        if rc == LB_EUNSTABLE:
            raise LBError(rc, "lb_batch_sums", last_error())
        _check(rc, "lb_batch_sums")
        return out

    def _raw_dtype(self):
        return np.float32 if self.codec == "f32" else np.uint16

    def get_f(self, d: int) -> np.ndarray:
        out = np.empty((19,) + self._shape(d), dtype=self._raw_dtype())
        _check(lib().lb_batch_get_f(self._h, int(d), out.ctypes.data_as(ctypes.c_void_p), out.nbytes, LB_HOST),
               "lb_batch_get_f")
        return out

    def set_f(self, d: int, f: np.ndarray):
        f = np.ascontiguousarray(f, dtype=self._raw_dtype())
        if f.shape != (19,) + self._shape(d):
            raise ValueError("state must have shape (19, nz, ny, nx)")
        _check(lib().lb_batch_set_f(self._h, int(d), f.ctypes.data_as(ctypes.c_void_p), f.nbytes, LB_HOST),
               "lb_batch_set_f")

    def sync(self):
        _check(lib().lb_batch_sync(self._h), "lb_batch_sync")

    @property
    def steps_done(self) -> int:
        return int(lib().lb_batch_steps_done(self._h))

    def query(self, key: int) -> int:
        return int(lib().lb_batch_query(self._h, int(key)))

    @property
    def info(self) -> dict:
        keys = ["variant", "sites_per_lane", "grid", "tiles", "tile_order", "domains", "sites", "fluid_sites",
                "array_bytes", "seg_bytes", "grid_mult", "autotuned", "wg_cap"]
        return {k: self.query(i) for i, k in enumerate(keys)}

    def time_steps(self, n: int) -> float:
        ms = ctypes.c_double(0.0)
        _check(lib().lb_batch_time_steps(self._h, int(n), ctypes.byref(ms)), "lb_batch_time_steps")
        return ms.value

    def time_step_kernel(self, n: int) -> float:
        ms = ctypes.c_double(0.0)
        _check(lib().lb_batch_time_step_kernel(self._h, int(n), ctypes.byref(ms)), "lb_batch_time_step_kernel")
        return ms.value


def decode_state(raw: np.ndarray, codec: str, scales=None) -> np.ndarray:
    """Raw stored words -> float64 shifted populations g = f - w (host-side
    view).  Scaled 16-bit codes ("s16") need the lattice's 3 exponents
    (Lattice.get_scales(): rest, axis, diagonal)."""
    if codec == "f32":
        return raw.astype(np.float64)
    if codec == "f16":
        return raw.view(np.float16).astype(np.float64)
    if codec == "s16":
        if scales is None:
            raise ValueError("s16 codes need their exponents")
        e = np.asarray(scales, dtype=np.float64)[[0] + [1] * 6 + [2] * 12]
        return raw.view(np.int16).astype(np.float64) * np.exp2(-e).reshape((19,) + (1,) * (raw.ndim - 1))
    return (raw.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


WEIGHTS = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)
