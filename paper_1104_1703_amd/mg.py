"""Python binding of ``libmg.so`` (the gfx950 masked multigrid library).

Argument marshalling only: every step of the solver runs in the library's
HIP kernels.  Device memory comes from torch tensors; the library's own level
buffers can come from torch's caching allocator through the allocator
callback of ``mg_options``.  The library must be built (``build.py``); if it is
missing or cannot be loaded, importing the solver raises.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libmg.so")

MG_OK, MG_NOT_CONVERGED, MG_ERR_ARG, MG_ERR_NO_ACTIVE, MG_ERR_HIP, MG_ERR_DIVERGED, MG_ERR_ALLOC = 0, 1, -1, -2, -3, -4, -5
MG_FP64, MG_MIXED = 0, 1
MG_BC_AUTO, MG_BC_FIRST, MG_BC_SECOND = 0, 1, 2

_ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
_FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class Allocator(C.Structure):
    _fields_ = [("alloc", _ALLOC_FN), ("free", _FREE_FN), ("ctx", C.c_void_p)]


class Options(C.Structure):
    _fields_ = [("n_pre", C.c_int32), ("n_post", C.c_int32), ("n_cycles", C.c_int32), ("n_coarse_sweeps", C.c_int32),
                ("min_coarse_dim", C.c_int32), ("max_cycles", C.c_int32), ("precision", C.c_int32),
                ("bc_order", C.c_int32), ("eta", C.c_double), ("first_order_hold", C.c_int32),
                ("use_graph", C.c_int32), ("fuse_passes", C.c_int32), ("tune", C.c_int32),
                ("item_depth_fine", C.c_int32), ("item_depth_l1", C.c_int32), ("item_depth_coarse", C.c_int32),
                ("fuse_restrict", C.c_int32), ("allocator", Allocator)]


class SolveInfo(C.Structure):
    _fields_ = [("cycles", C.c_int32), ("order_used", C.c_int32), ("switched_at_cycle", C.c_int32),
                ("status", C.c_int32), ("r_ref", C.c_double), ("r0", C.c_double), ("r_final", C.c_double),
                ("ms", C.c_double), ("history", C.c_double * 257)]

    def as_dict(self):
        n = min(self.cycles, 256)
        return {"status": self.status, "cycles": self.cycles, "order_used": self.order_used,
                "switched_at": self.switched_at_cycle, "r_ref": self.r_ref, "r0": self.r0,
                "r_final": self.r_final, "ms": self.ms, "history": [self.history[i] for i in range(n + 1)]}


# every symbol the C header declares: (name, restype, argtypes)
_P = C.c_void_p
_I = C.c_int32
_D = C.c_double
SYMBOLS = [
    ("mg_default_options", None, [C.POINTER(Options)]),
    ("mg_create_hierarchy", C.c_int, [_P, _I, _I, _I, _D, C.POINTER(Options), _P, C.POINTER(_P)]),
    ("mg_destroy_hierarchy", None, [_P]),
    ("mg_solve", C.c_int, [_P, _P, _P, _P, _D, C.POINTER(SolveInfo)]),
    ("mg_residual_norm", C.c_int, [_P, _P, _P, _P, C.POINTER(_D)]),
    ("mg_residual_norm_noalloc", C.c_int, [_P, _P, _P, _P, _P]),
    ("mg_status_string", C.c_char_p, [C.c_int]),
    ("mg_last_error", C.c_char_p, []),
    ("mg_num_levels", _I, [_P, _I]),
    ("mg_level_dims", C.c_int, [_P, _I, C.POINTER(_I)]),
    ("mg_level_active", C.c_int64, [_P, _I, _I]),
    ("mg_level_item_depth", C.c_int32, [_P, _I, _I]),
    ("mg_level_counts", C.c_int, [_P, _I, _P]),
    ("mg_level_diag", C.c_int, [_P, _I, _I, _P]),
    ("mg_fold", C.c_int, [_P, _P, _P, _P]),
    ("mg_smooth", C.c_int, [_P, _I, _I, _P, _P, _I]),
    ("mg_residual", C.c_int, [_P, _I, _I, _P, _P, _P]),
    ("mg_restrict_residual", C.c_int, [_P, _I, _I, _P, _P, _P]),
    ("mg_prolong", C.c_int, [_P, _I, _I, _P, _P]),
    ("mg_vcycle", C.c_int, [_P, _I, _P, _P]),
    ("mg_time_smoother", C.c_int, [_P, _I, _I]),
    ("mg_kernel_timing", C.c_int, [_P, _I]),
    ("mg_kernel_timing_read", C.c_int, [_P, C.POINTER(_D), C.POINTER(_I)]),
    ("mg_stream", _P, [_P]),
    ("mg_create_batch", C.c_int, [_I, _P, _P, _P, C.POINTER(Options), _P, C.POINTER(_P)]),
    ("mg_solve_batch", C.c_int, [_P, _P, _P, _P, _D, _P, C.POINTER(_D)]),
    ("mg_destroy_batch", None, [_P]),
    ("mg_batch_size", _I, [_P]),
    ("mg_batch_grid", _I, [_P]),
    ("mg_batch_phases", _I, [_P, _I]),
    ("mg_batch_validate", _I, [_P, C.c_char_p, _I]),
    ("mg_batch_set_engine", C.c_int, [_P, _I]),
    ("mg_amr_dirichlet", C.c_int, [_P, _I, _I, _I, _D, _P, _I, _I, _I, _D, _P, _P, _P]),
    ("mg_amr_grad5", C.c_int, [_P, _P, _I, _I, _I, _D, _P, _P, _I, _I, _I, _D, _P, _P, _P, _P]),
    # learned first guess
    ("mg_unet_create", C.c_int, [C.c_uint64, _P, _P, C.POINTER(_P)]),
    ("mg_unet_destroy", None, [_P]),
    ("mg_unet_num_params", C.c_int64, [_P]),
    ("mg_unet_stream", _P, [_P]),
    ("mg_unet_step", _I, [_P]),
    ("mg_unet_set_params", C.c_int, [_P, _P, C.c_int64]),
    ("mg_unet_get_params", C.c_int, [_P, _P, C.c_int64]),
    ("mg_unet_get_grads", C.c_int, [_P, _P, C.c_int64]),
    ("mg_unet_tensor", C.c_int, [_P, _I, _I, _P, C.c_int64]),
    ("mg_unet_save", C.c_int, [_P, C.c_char_p]),
    ("mg_unet_load", C.c_int, [_P, C.c_char_p]),
    ("mg_unet_loss_grad", C.c_int, [_P, _I, _P, _P, _P, _P, _I, _I, _I, C.POINTER(_D)]),
    ("mg_unet_train_step", C.c_int, [_P, _I, _P, _P, _P, _P, _I, _I, _I, C.c_float, C.c_float, C.POINTER(_D)]),
    ("mg_unet_infer", C.c_int, [_P, _P, _P, _P, _I, _I, _I, _I, _P]),
    ("mg_coarsen_problem", C.c_int, [_P, _P, _P, _I, _I, _I, _I, _P, _P, _P, _P]),
    ("mg_upsample_guess", C.c_int, [_P, _I, _I, _I, _P, _P, _P]),
    ("mg_nn_conv3d_fwd", C.c_int, [_P, _I, _I, _P, _I, _P, _P, _P, _I, _I, _I, _I, _I, _I, _P]),
    ("mg_nn_conv3d_bwd_weight", C.c_int, [_P, _I, _P, _I, _I, _P, _I, _P, _P, _I, _I, _I, _I, _P]),
    ("mg_nn_weight_flip", C.c_int, [_P, _I, _I, _P, _P]),
    ("mg_nn_relu_bwd", C.c_int, [_P, _P, C.c_int64, _P]),
    ("mg_nn_pool2", C.c_int, [_P, _P, _I, _I, _I, _I, _I, _P]),
    ("mg_nn_pool2_bwd", C.c_int, [_P, _P, _I, _I, _I, _I, _I, _P]),
    ("mg_nn_split_grad", C.c_int, [_P, _I, _I, _P, _P, _I, _I, _I, _I, _P]),
    ("mg_nn_adamw", C.c_int, [_P, _P, _P, _P, _P, C.c_int64, C.c_float, C.c_float, C.c_float, C.c_float,
                              C.c_float, _I, _P]),
    ("mg_nn_mfma_selftest", C.c_int, [_P, _P]),
]

_lib = None


def load_library(path: str = LIB_PATH):
    """Load libmg.so and declare every exported symbol.  Raises if absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise RuntimeError(f"libmg.so not built ({path}); run `python -m paper_1104_1703_amd.build`")
        lib = C.CDLL(path)
        for name, res, args in SYMBOLS:
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


class MGError(RuntimeError):
    def __init__(self, status, where):
        lib = load_library()
        msg = lib.mg_status_string(status).decode()
        detail = lib.mg_last_error().decode()
        super().__init__(f"{where}: {msg} ({status}){': ' + detail if detail else ''}")
        self.status = status


def _check(status, where, ok=(MG_OK,)):
    if status not in ok:
        raise MGError(status, where)
    return status


def default_options(**kw) -> Options:
    o = Options()
    load_library().mg_default_options(C.byref(o))
    for k, v in kw.items():
        if k == "bc_order" and isinstance(v, str):
            v = {"auto": MG_BC_AUTO, "first": MG_BC_FIRST, "second": MG_BC_SECOND}[v]
        if k == "precision" and isinstance(v, str):
            v = {"fp64": MG_FP64, "mixed": MG_MIXED}[v]
        if k == "allocator":
            continue
        setattr(o, k, v)
    return o


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("tensor must live on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return C.c_void_p(t.data_ptr())


class _TorchAllocator:
    """Routes the library's level buffers through torch's caching allocator."""

    def __init__(self, device, stream):
        self.device = device
        self.stream = stream

        def _alloc(nbytes, ctx):
            try:
                return int(torch.cuda.caching_allocator_alloc(int(nbytes), self.device, self.stream))
            except Exception:  # out of memory: the library reports MG_ERR_ALLOC
                return None

        def _free(ptr, ctx):
            torch.cuda.caching_allocator_delete(int(ptr))

        self.alloc_fn = _ALLOC_FN(_alloc)
        self.free_fn = _FREE_FN(_free)

    def fill(self, opts: Options):
        opts.allocator.alloc = self.alloc_fn
        opts.allocator.free = self.free_fn
        opts.allocator.ctx = None


class Hierarchy:
    """Multigrid hierarchy of a mask on the current CUDA (HIP) device.

    ``mask``: int8 tensor (nz, ny, nx) with +1 active / -1 inactive cells
    and an inactive outermost layer.  Options are ``mg_options`` fields
    (n_pre, n_post, n_cycles, n_coarse_sweeps, min_coarse_dim, max_cycles,
    precision 'fp64'|'mixed', bc_order 'auto'|'first'|'second', eta,
    first_order_hold, use_graph, fuse_passes, fuse_restrict, tune,
    item_depth_fine, item_depth_l1, item_depth_coarse); ``torch_allocator``
    routes buffers through torch's caching allocator.
    """

    def __init__(self, mask: torch.Tensor, h: float, stream=None, torch_allocator: bool = True, **options):
        lib = load_library()
        if mask.dtype != torch.int8:
            raise ValueError("mask must be int8")
        self.device = mask.device
        # a dedicated stream per hierarchy (graphs cannot be captured on the
        # legacy default stream); calls order it against the caller's stream
        self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
        self.shape = tuple(mask.shape)
        self.h = float(h)
        self.opts = default_options(**options)
        self._alloc = None
        if torch_allocator:
            self._alloc = _TorchAllocator(self.device, self.stream)
            self._alloc.fill(self.opts)
        nz, ny, nx = self.shape
        out = C.c_void_p()
        mask = mask.contiguous()
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        with torch.cuda.device(self.device):
            st = lib.mg_create_hierarchy(_ptr(mask), nx, ny, nz, self.h, C.byref(self.opts),
                                         C.c_void_p(self.stream.cuda_stream), C.byref(out))
        _check(st, "mg_create_hierarchy")
        self._h = out

    def _enter(self):
        self.stream.wait_stream(torch.cuda.current_stream(self.device))

    def _leave(self):
        torch.cuda.current_stream(self.device).wait_stream(self.stream)

    def _call(self, fn, *args):
        self._enter()
        with torch.cuda.device(self.device):
            st = fn(*args)
        self._leave()
        return st

    def close(self):
        if getattr(self, "_h", None):
            with torch.cuda.device(self.device):
                load_library().mg_destroy_hierarchy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # ---- introspection ----
    def nlevels(self, order: int = 0) -> int:
        return int(load_library().mg_num_levels(self._h, order))

    def dims(self, level: int):
        d = (C.c_int32 * 3)()
        _check(load_library().mg_level_dims(self._h, level, d), "mg_level_dims")
        return int(d[2]), int(d[1]), int(d[0])

    def n_active(self, level: int = 0, order: int = 2) -> int:
        return int(load_library().mg_level_active(self._h, level, order))

    def item_depth(self, level: int = 0, order: int = 2) -> int:
        """Planes per smoother work item of a level (default, given or tuned)."""
        return int(load_library().mg_level_item_depth(self._h, level, order))

    def item_depths(self):
        """{order: [depth of each level]} for both boundary orders."""
        return {o: [self.item_depth(l, o) for l in range(self.nlevels(o))] for o in (1, 2)}

    def counts(self, level: int) -> torch.Tensor:
        out = torch.empty(self.dims(level), dtype=torch.int32, device=self.device)
        _check(self._call(load_library().mg_level_counts, self._h, level, _ptr(out)), "mg_level_counts")
        return out

    def diag(self, level: int, order: int = 2) -> torch.Tensor:
        out = torch.empty(self.dims(level), dtype=torch.float64, device=self.device)
        _check(self._call(load_library().mg_level_diag, self._h, level, order, _ptr(out)), "mg_level_diag")
        return out

    # ---- solve ----
    def solve(self, rho, phi=None, dirichlet=None, tol: float = 1e-10, check: bool = True):
        """Solve in place into ``phi`` (zeros if None); returns (phi, info dict)."""
        if phi is None:
            phi = torch.zeros(self.shape, dtype=torch.float64, device=self.device)
        info = SolveInfo()
        st = self._call(load_library().mg_solve, self._h, _ptr(rho), _ptr(phi), _ptr(dirichlet), float(tol),
                        C.byref(info))
        if check:
            _check(st, "mg_solve", ok=(MG_OK, MG_NOT_CONVERGED))
        return phi, info.as_dict()

    def residual_norm(self, rho, phi, dirichlet=None) -> float:
        out = C.c_double()
        st = self._call(load_library().mg_residual_norm, self._h, _ptr(rho), _ptr(phi), _ptr(dirichlet),
                        C.byref(out))
        _check(st, "mg_residual_norm")
        return float(out.value)

    def residual_norm_noalloc(self, rho, phi, dirichlet=None, out=None):
        """The residual norm written to a one-element float64 device tensor,
        with no allocation or synchronisation inside the library."""
        if out is None:
            out = torch.empty(1, dtype=torch.float64, device=self.device)
        _check(self._call(load_library().mg_residual_norm_noalloc, self._h, _ptr(rho), _ptr(phi), _ptr(dirichlet),
                          _ptr(out)), "mg_residual_norm_noalloc")
        return out

    # ---- single steps ----
    def fold(self, rho, dirichlet=None):
        f = torch.empty(self.shape, dtype=torch.float64, device=self.device)
        _check(self._call(load_library().mg_fold, self._h, _ptr(rho), _ptr(dirichlet), _ptr(f)), "mg_fold")
        return f

    def smooth(self, level, x, f, passes=1, order=2):
        x = x.clone().contiguous()
        _check(self._call(load_library().mg_smooth, self._h, level, order, _ptr(x), _ptr(f), passes), "mg_smooth")
        return x

    def residual(self, level, x, f, order=2):
        r = torch.empty_like(x)
        _check(self._call(load_library().mg_residual, self._h, level, order, _ptr(x), _ptr(f), _ptr(r)), "mg_residual")
        return r

    def restrict_residual(self, level, x, f, order=2):
        fc = torch.empty(self.dims(level + 1), dtype=torch.float64, device=self.device)
        _check(self._call(load_library().mg_restrict_residual, self._h, level, order, _ptr(x), _ptr(f), _ptr(fc)),
               "mg_restrict_residual")
        return fc

    def prolong(self, level, xc, x, order=2):
        x = x.clone().contiguous()
        _check(self._call(load_library().mg_prolong, self._h, level, order, _ptr(xc), _ptr(x)), "mg_prolong")
        return x

    def vcycle(self, x, f, order=2):
        x = x.clone().contiguous()
        _check(self._call(load_library().mg_vcycle, self._h, order, _ptr(x), _ptr(f)), "mg_vcycle")
        return x

    def time_smoother(self, launches: int, order: int = 2):
        _check(self._call(load_library().mg_time_smoother, self._h, order, launches), "mg_time_smoother")

    TIMING_KINDS = {"plain": 1, "residual": 2, "prolong": 3, "norm": 4}

    def kernel_timing(self, enable, kind: str = "plain"):
        """Start (clearing the record) or stop HIP-event timing of one kind of
        finest-level red-black launch inside later solves: "plain", "residual"
        (the pass that also restricts the residual), "prolong" (the pass that
        applies the prolongation) or "norm" (the pass forming the input norm)."""
        code = self.TIMING_KINDS[kind] if enable else 0
        _check(self._call(load_library().mg_kernel_timing, self._h, code), "mg_kernel_timing")

    def kernel_timing_read(self):
        """(summed milliseconds, launches) of the recorded launches."""
        ms, n = C.c_double(0.0), C.c_int32(0)
        _check(self._call(load_library().mg_kernel_timing_read, self._h, C.byref(ms), C.byref(n)),
               "mg_kernel_timing_read")
        return ms.value, n.value


class Batch:
    """Many independent masked grids solved together: each multigrid cycle
    of all patches runs as one program of phase launches (the per-patch
    lockstep engine where the programs do not cover the options).

    ``masks``: list of int8 tensors (each (nz, ny, nx), inactive outer layer);
    ``hs``: cell widths.  Options as for :class:`Hierarchy` (FP64 only).
    """

    def __init__(self, masks, hs, stream=None, torch_allocator: bool = True, **options):
        lib = load_library()
        self.n = len(masks)
        self.device = masks[0].device
        self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
        self.shapes = [tuple(m.shape) for m in masks]
        self.opts = default_options(**options)
        self._alloc = None
        if torch_allocator:
            self._alloc = _TorchAllocator(self.device, self.stream)
            self._alloc.fill(self.opts)
        self._masks = [m.contiguous() for m in masks]
        ptrs = (C.c_void_p * self.n)(*[m.data_ptr() for m in self._masks])
        dims = (C.c_int32 * (3 * self.n))()
        for i, (nz, ny, nx) in enumerate(self.shapes):
            dims[3 * i], dims[3 * i + 1], dims[3 * i + 2] = nx, ny, nz
        hv = (C.c_double * self.n)(*[float(h) for h in hs])
        out = C.c_void_p()
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        with torch.cuda.device(self.device):
            st = lib.mg_create_batch(self.n, ptrs, dims, hv, C.byref(self.opts), C.c_void_p(self.stream.cuda_stream),
                                     C.byref(out))
        self._masks = None
        _check(st, "mg_create_batch")
        self._b = out

    @property
    def grid(self) -> int:
        return int(load_library().mg_batch_grid(self._b))

    def phases(self, order: int = 2) -> int:
        return int(load_library().mg_batch_phases(self._b, order))

    def validate(self):
        """(violations, description) of the host-side check of the phase tables."""
        buf = C.create_string_buffer(1024)
        n = int(load_library().mg_batch_validate(self._b, buf, len(buf)))
        return n, buf.value.decode()

    def set_engine(self, phased):
        """Phase programs (True or "phased"), the same programs as one
        cooperative launch per V-cycle ("persistent"), or per-patch lockstep
        cycles (False or "lockstep")."""
        v = {"lockstep": 0, "phased": 1, "persistent": 2}[phased] if isinstance(phased, str) else (1 if phased else 0)
        _check(load_library().mg_batch_set_engine(self._b, v), "mg_batch_set_engine")

    def solve(self, rhos, phis=None, dirichlets=None, tol: float = 1e-10, check: bool = True):
        """Solve every patch in place; returns (phis, list of info dicts, ms)."""
        lib = load_library()
        if phis is None:
            phis = [torch.zeros(sh, dtype=torch.float64, device=self.device) for sh in self.shapes]
        for t in list(rhos) + list(phis) + [d for d in (dirichlets or []) if d is not None]:
            _ptr(t)  # device, contiguous
        rp = (C.c_void_p * self.n)(*[t.data_ptr() for t in rhos])
        pp = (C.c_void_p * self.n)(*[t.data_ptr() for t in phis])
        dp = None
        if dirichlets is not None:
            dp = (C.c_void_p * self.n)(*[(d.data_ptr() if d is not None else None) for d in dirichlets])
        infos = (SolveInfo * self.n)()
        ms = C.c_double()
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        with torch.cuda.device(self.device):
            st = lib.mg_solve_batch(self._b, rp, pp, dp, float(tol), infos, C.byref(ms))
        torch.cuda.current_stream(self.device).wait_stream(self.stream)
        if check:
            _check(st, "mg_solve_batch", ok=(MG_OK, MG_NOT_CONVERGED))
        return phis, [infos[i].as_dict() for i in range(self.n)], float(ms.value)

    def close(self):
        if getattr(self, "_b", None):
            with torch.cuda.device(self.device):
                load_library().mg_destroy_batch(self._b)
            self._b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------- learned guess
class UNet:
    """The learned first-guess network (a 3D U-Net run by the library's BF16
    matrix-core kernels).  Parameters live on the device; ``params`` /
    ``set_params`` copy them as float32 host arrays."""

    def __init__(self, seed: int = 0, device=None, stream=None, torch_allocator: bool = True):
        lib = load_library()
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
        self._alloc = None
        ap = None
        if torch_allocator:
            self._alloc = _TorchAllocator(self.device, self.stream)
            self._astruct = Allocator(self._alloc.alloc_fn, self._alloc.free_fn, None)
            ap = C.byref(self._astruct)
        out = C.c_void_p()
        with torch.cuda.device(self.device):
            st = lib.mg_unet_create(int(seed), ap, C.c_void_p(self.stream.cuda_stream), C.byref(out))
        _check(st, "mg_unet_create")
        self._u = out
        self.num_params = int(lib.mg_unet_num_params(self._u))

    def _call(self, fn, *args):
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        with torch.cuda.device(self.device):
            st = fn(*args)
        torch.cuda.current_stream(self.device).wait_stream(self.stream)
        return st

    @property
    def step(self) -> int:
        return int(load_library().mg_unet_step(self._u))

    def params(self):
        import numpy as np
        out = np.empty(self.num_params, np.float32)
        _check(self._call(load_library().mg_unet_get_params, self._u, out.ctypes.data_as(C.c_void_p),
                          self.num_params), "mg_unet_get_params")
        return out

    def grads(self):
        import numpy as np
        out = np.empty(self.num_params, np.float32)
        _check(self._call(load_library().mg_unet_get_grads, self._u, out.ctypes.data_as(C.c_void_p),
                          self.num_params), "mg_unet_get_grads")
        return out

    TENSOR_KINDS = {"act": 0, "act_grad": 1, "pool": 2, "pool_grad": 3, "input": 4, "cat_grad": 5}

    def tensor(self, kind: str, index: int, shape):
        """Copy of a tensor the network keeps between layers (BF16,
        channels-last ``shape`` of the last batch); kinds as in mg.h."""
        out = torch.empty(tuple(shape), dtype=torch.bfloat16, device=self.device)
        _check(self._call(load_library().mg_unet_tensor, self._u, self.TENSOR_KINDS[kind], int(index), _ptr(out),
                          out.numel()), "mg_unet_tensor")
        return out

    def set_params(self, p):
        import numpy as np
        p = np.ascontiguousarray(p, dtype=np.float32)
        _check(self._call(load_library().mg_unet_set_params, self._u, p.ctypes.data_as(C.c_void_p), p.size),
               "mg_unet_set_params")

    def save(self, path: str):
        _check(self._call(load_library().mg_unet_save, self._u, os.fsencode(path)), "mg_unet_save")

    def load(self, path: str):
        _check(self._call(load_library().mg_unet_load, self._u, os.fsencode(path)), "mg_unet_load")

    @staticmethod
    def _batch(rho, mask, dirichlet, target):
        if rho.dim() == 3:
            rho, mask, target = rho[None], mask[None], target[None]
            dirichlet = None if dirichlet is None else dirichlet[None]
        n, nz, ny, nx = rho.shape
        return n, nz, ny, nx, rho, mask, dirichlet, target

    def loss_grad(self, rho, mask, target, dirichlet=None) -> float:
        """Loss and gradients (kept on the device) for a batch (n, nz, ny, nx)."""
        n, nz, ny, nx, rho, mask, dirichlet, target = self._batch(rho, mask, dirichlet, target)
        loss = C.c_double()
        _check(self._call(load_library().mg_unet_loss_grad, self._u, n, _ptr(rho), _ptr(mask), _ptr(dirichlet),
                          _ptr(target), nx, ny, nz, C.byref(loss)), "mg_unet_loss_grad")
        return float(loss.value)

    def train_step(self, rho, mask, target, dirichlet=None, lr: float = 1e-3, weight_decay: float = 0.0,
                   sync: bool = True):
        """One AdamW step on a batch; returns the loss (None if not sync)."""
        n, nz, ny, nx, rho, mask, dirichlet, target = self._batch(rho, mask, dirichlet, target)
        loss = C.c_double()
        _check(self._call(load_library().mg_unet_train_step, self._u, n, _ptr(rho), _ptr(mask), _ptr(dirichlet),
                          _ptr(target), nx, ny, nz, float(lr), float(weight_decay),
                          C.byref(loss) if sync else None), "mg_unet_train_step")
        return float(loss.value) if sync else None

    def infer(self, rho, mask, dirichlet=None, stride: int = 1, out=None):
        """First guess phi0 (float64, shape of rho) from the network at 1/stride resolution."""
        nz, ny, nx = rho.shape
        if out is None:
            out = torch.empty(rho.shape, dtype=torch.float64, device=self.device)
        _check(self._call(load_library().mg_unet_infer, self._u, _ptr(rho), _ptr(mask), _ptr(dirichlet), nx, ny, nz,
                          int(stride), _ptr(out)), "mg_unet_infer")
        return out

    def close(self):
        if getattr(self, "_u", None):
            with torch.cuda.device(self.device):
                load_library().mg_unet_destroy(self._u)
            self._u = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def coarsen_problem(rho, mask, dirichlet=None, stride: int = 2):
    """Coarse copy (rho_c, mask_c, dirichlet_c) of a problem on the 1/stride grid."""
    nz, ny, nx = rho.shape
    shp = (nz // stride, ny // stride, nx // stride)
    rho_c = torch.empty(shp, dtype=torch.float64, device=rho.device)
    mask_c = torch.empty(shp, dtype=torch.int8, device=rho.device)
    b_c = None if dirichlet is None else torch.empty(shp, dtype=torch.float64, device=rho.device)
    st = load_library().mg_coarsen_problem(_ptr(rho), _ptr(mask), _ptr(dirichlet), nx, ny, nz, int(stride),
                                           _ptr(rho_c), _ptr(mask_c), _ptr(b_c),
                                           C.c_void_p(torch.cuda.current_stream(rho.device).cuda_stream))
    _check(st, "mg_coarsen_problem")
    return rho_c, mask_c, b_c


def upsample_guess(phi_c, mask, out=None):
    """Linear up-sampling by 2 of phi_c onto the active cells of ``mask``."""
    nzc, nyc, nxc = phi_c.shape
    if out is None:
        out = torch.empty(mask.shape, dtype=torch.float64, device=phi_c.device)
    st = load_library().mg_upsample_guess(_ptr(phi_c), nxc, nyc, nzc, _ptr(mask), _ptr(out),
                                          C.c_void_p(torch.cuda.current_stream(phi_c.device).cuda_stream))
    _check(st, "mg_upsample_guess")
    return out


def _origin(o):
    return (C.c_double * 3)(*[float(v) for v in o])


def amr_dirichlet(phi_c, hc: float, origin_c, shape, hf: float, origin_f, out=None):
    """Dirichlet field of a refined patch (shape, hf, corner origin_f) from
    the coarser potential phi_c (cell width hc, corner origin_c): the
    one-way interface values of mg_amr_dirichlet."""
    cnz, cny, cnx = phi_c.shape
    nz, ny, nx = shape
    if out is None:
        out = torch.empty(shape, dtype=torch.float64, device=phi_c.device)
    st = load_library().mg_amr_dirichlet(_ptr(phi_c), cnx, cny, cnz, float(hc), _origin(origin_c), nx, ny, nz,
                                         float(hf), _origin(origin_f), _ptr(out),
                                         C.c_void_p(torch.cuda.current_stream(phi_c.device).cuda_stream))
    _check(st, "mg_amr_dirichlet")
    return out


def amr_grad5(phi, mask, h: float, origin, coarse=None, bnd=None, out=None):
    """5-point gradient (3, nz, ny, nx) of phi on the active cells of mask;
    coarse = (phi_c, hc, origin_c) supplies values beyond the level, else
    bnd (the level's Dirichlet field) inside the array."""
    nz, ny, nx = phi.shape
    if out is None:
        out = torch.empty((3,) + tuple(phi.shape), dtype=torch.float64, device=phi.device)
    pc, hc, oc = coarse if coarse is not None else (None, 1.0, (0.0, 0.0, 0.0))
    cnz, cny, cnx = pc.shape if pc is not None else (0, 0, 0)
    st = load_library().mg_amr_grad5(_ptr(phi), _ptr(mask), nx, ny, nz, float(h), _origin(origin), _ptr(pc), cnx,
                                     cny, cnz, float(hc), _origin(oc), _ptr(bnd), _ptr(out),
                                     C.c_void_p(torch.cuda.current_stream(phi.device).cuda_stream))
    _check(st, "mg_amr_grad5")
    return out


class nn:
    """Thin wrappers of the exported network kernels (BF16 channels-last
    tensors; every call enqueues on torch's current stream)."""

    @staticmethod
    def _s(t):
        return C.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)

    @staticmethod
    def conv3d(a, w, bias=None, b=None, up_a=False, relu=True):
        """Output (n, d, h, wd, cout) at the resolution of ``b`` (if given) or of ``a``."""
        if up_a and b is None:
            raise ValueError("an up-sampled input needs the full-resolution input for its shape")
        n, d, h, wd = (b if b is not None else a).shape[:4]
        cb = 0 if b is None else b.shape[-1]
        cout = w.shape[1]
        out = torch.empty((n, d, h, wd, cout), dtype=torch.bfloat16, device=a.device)
        st = load_library().mg_nn_conv3d_fwd(_ptr(a), a.shape[-1], int(up_a), _ptr(b), cb, _ptr(w), _ptr(bias),
                                             _ptr(out), cout, int(relu), n, d, h, wd, nn._s(a))
        _check(st, "mg_nn_conv3d_fwd")
        return out

    @staticmethod
    def conv3d_bwd_weight(dout, a, b=None, up_a=False, dw=None, dbias=None):
        n, d, h, wd, cout = dout.shape
        cin = a.shape[-1] + (0 if b is None else b.shape[-1])
        if dw is None:
            dw = torch.zeros((27, cout, cin), dtype=torch.float32, device=dout.device)
        if dbias is None:
            dbias = torch.zeros(cout, dtype=torch.float32, device=dout.device)
        st = load_library().mg_nn_conv3d_bwd_weight(_ptr(dout), cout, _ptr(a), a.shape[-1], int(up_a), _ptr(b),
                                                    0 if b is None else b.shape[-1], _ptr(dw), _ptr(dbias), n, d, h,
                                                    wd, nn._s(dout))
        _check(st, "mg_nn_conv3d_bwd_weight")
        return dw, dbias

    @staticmethod
    def weight_flip(w):
        _, cout, cin = w.shape
        wt = torch.empty((27, cin, cout), dtype=w.dtype, device=w.device)
        _check(load_library().mg_nn_weight_flip(_ptr(w), cout, cin, _ptr(wt), nn._s(w)), "mg_nn_weight_flip")
        return wt

    @staticmethod
    def relu_bwd(dy, y):
        dy = dy.clone()
        _check(load_library().mg_nn_relu_bwd(_ptr(dy), _ptr(y), dy.numel(), nn._s(dy)), "mg_nn_relu_bwd")
        return dy

    @staticmethod
    def pool2(x):
        n, d, h, wd, c = x.shape
        out = torch.empty((n, d // 2, h // 2, wd // 2, c), dtype=x.dtype, device=x.device)
        _check(load_library().mg_nn_pool2(_ptr(x), _ptr(out), c, n, d, h, wd, nn._s(x)), "mg_nn_pool2")
        return out

    @staticmethod
    def pool2_bwd(dout, din):
        n, d, h, wd, c = din.shape
        din = din.clone()
        _check(load_library().mg_nn_pool2_bwd(_ptr(dout), _ptr(din), c, n, d, h, wd, nn._s(din)), "mg_nn_pool2_bwd")
        return din

    @staticmethod
    def split_grad(dx, ca):
        n, d, h, wd, cin = dx.shape
        cb = cin - ca
        dup = torch.empty((n, d // 2, h // 2, wd // 2, ca), dtype=dx.dtype, device=dx.device)
        dskip = torch.empty((n, d, h, wd, cb), dtype=dx.dtype, device=dx.device) if cb else None
        _check(load_library().mg_nn_split_grad(_ptr(dx), ca, cb, _ptr(dup), _ptr(dskip), n, d, h, wd, nn._s(dx)),
               "mg_nn_split_grad")
        return dup, dskip

    @staticmethod
    def adamw(p, g, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8, weight_decay=0.0, p_bf16=None):
        _check(load_library().mg_nn_adamw(_ptr(p), _ptr(p_bf16), _ptr(g), _ptr(m), _ptr(v), p.numel(), float(lr),
                                          float(beta1), float(beta2), float(eps), float(weight_decay), int(step),
                                          nn._s(p)), "mg_nn_adamw")

    @staticmethod
    def mfma_selftest(device="cuda"):
        out = torch.zeros((16, 16), dtype=torch.float32, device=device)
        _check(load_library().mg_nn_mfma_selftest(_ptr(out), nn._s(out)), "mg_nn_mfma_selftest")
        return out
