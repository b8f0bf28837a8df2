"""Python binding of the C ABI in ``include/vanse.h`` (ctypes, argument
marshalling only).

Every step of the VANSE lattice Boltzmann path runs in the HIP kernels of
``libvanse.so``; this module only passes pointers of torch tensors and the
current torch stream.  If the library is missing the import of the binding
fails loudly: there is no CPU fallback.

Low-level names mirror the C ABI (``vanse_create``, ``vanse_set_porosity``,
``vanse_step``, ``vanse_moments`` ...).  :class:`Solver` wraps one handle.
"""
from __future__ import annotations

import collections
import ctypes
import os
import threading

import torch  # loads the HIP runtime the library binds to (same soname)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvanse.so")

D2Q9, D3Q19, D3Q27 = 0, 1, 2
QUAD_NONE = 8
FP64, FP32_SHIFTED, FP16_SHIFTED, FX16_SHIFTED = 0, 1, 2, 3
OK, EINVAL, ENOMEM, EDEVICE, ESTATE, EUNSTABLE = 0, -1, -2, -3, -4, -5
DTYPES = {"fp64": FP64, "fp32_shifted": FP32_SHIFTED, "fp16_shifted": FP16_SHIFTED,
          "fx16_shifted": FX16_SHIFTED}
LATTICES = {"D2Q9": D2Q9, "D3Q19": D3Q19, "D3Q27": D3Q27}

_STATUS = {EINVAL: "EINVAL", ENOMEM: "ENOMEM", EDEVICE: "EDEVICE", ESTATE: "ESTATE",
           EUNSTABLE: "EUNSTABLE"}

EXPORTS = [
    "vanse_create", "vanse_destroy", "vanse_set_stream", "vanse_set_porosity",
    "vanse_set_force", "vanse_init", "vanse_step", "vanse_moments", "vanse_diagnostics",
    "vanse_populations", "vanse_time", "vanse_device_bytes", "vanse_last_error",
    "vanse_lattice_info", "vanse_copy_probe", "vanse_set_tuning", "vanse_set_tile",
    "vanse_autotune", "vanse_set_force_field", "vanse_set_fused",
    "vanse_batch_create", "vanse_batch_destroy", "vanse_batch_set_stream",
    "vanse_batch_set_tuning", "vanse_batch_step", "vanse_batch_autotune",
    "vanse_batch_last_error", "vanse_batch_update", "vanse_batch_two_step_layout",
    "vanse_diagnostics_noalloc", "vanse_batch_two_step_tiles",
]
TUNE_NONTEMPORAL, TUNE_XCD_REMAP, TUNE_FLAT, TUNE_NT_STORES, TUNE_TWO_STEP = 1, 2, 4, 8, 16


class Launch(collections.namedtuple(
        "Launch", "tile_x tile_y flags fused_rows fused_planes steps_run")):
    """Launch shape chosen by Solver.autotune (fused_rows = 0: single steps)."""


class VanseError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%s): %s" % (_STATUS.get(code, code), code, msg))
        self.code = code


_lock = threading.Lock()
_lib = None


def load_library(path: str = LIB_PATH):
    """Load ``libvanse.so`` and declare the C signatures.  Raises if the
    library has not been built."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(path):
            raise ImportError(
                "libvanse.so not found at %s: build it with "
                "`python -m paper_2208_09267_amd.build` (there is no CPU fallback)" % path)
        lib = ctypes.CDLL(path)
        P, i, d, i64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_int64
        I64P = ctypes.POINTER(ctypes.c_int64)
        sig = {
            "vanse_create": (i, [i, I64P, d, i, ctypes.POINTER(P)]),
            "vanse_destroy": (i, [P]),
            "vanse_set_stream": (i, [P, P]),
            "vanse_set_porosity": (i, [P, d, P, d, i]),
            "vanse_set_force": (i, [P, P]),
            "vanse_init": (i, [P, P, P]),
            "vanse_step": (i, [P, i64]),
            "vanse_moments": (i, [P, P, P, P]),
            "vanse_diagnostics": (i, [P, P]),
            "vanse_populations": (i, [P, P]),
            "vanse_time": (i, [P, I64P]),
            "vanse_device_bytes": (i, [P, I64P]),
            "vanse_last_error": (ctypes.c_char_p, [P]),
            "vanse_lattice_info": (i, [i, P, P, P, P]),
            "vanse_copy_probe": (i, [P, P, i64, P]),
            "vanse_set_tuning": (i, [P, i, i]),
            "vanse_set_tile": (i, [P, i, i]),
            "vanse_set_force_field": (i, [P, P]),
            "vanse_set_fused": (i, [P, i, i]),
            "vanse_autotune": (i, [P, i, ctypes.POINTER(i), ctypes.POINTER(i),
                                   ctypes.POINTER(i), ctypes.POINTER(i), ctypes.POINTER(i),
                                   I64P]),
            "vanse_batch_create": (i, [ctypes.POINTER(P), i, ctypes.POINTER(P)]),
            "vanse_batch_destroy": (i, [P]),
            "vanse_batch_set_stream": (i, [P, P]),
            "vanse_batch_set_tuning": (i, [P, i, i, i]),
            "vanse_batch_step": (i, [P, i64]),
            "vanse_batch_autotune": (i, [P, i, ctypes.POINTER(i), ctypes.POINTER(i), I64P]),
            "vanse_batch_last_error": (ctypes.c_char_p, [P]),
            "vanse_batch_two_step_layout": (i, [P, i, ctypes.POINTER(i), ctypes.POINTER(i)]),
            "vanse_batch_update": (i, [P, ctypes.POINTER(P), i]),
            "vanse_diagnostics_noalloc": (i, [i, I64P, P, P, i, P, P, P, P]),
            "vanse_batch_two_step_tiles": (i, [P, i, ctypes.POINTER(i), ctypes.POINTER(i),
                                               ctypes.POINTER(i)]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
        return lib


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda or not t.is_contiguous() or t.dtype != torch.float64:
        raise ValueError("expected a contiguous float64 CUDA tensor")
    return ctypes.c_void_p(t.data_ptr())


def _stream_handle():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def lattice_info(lattice: int):
    """(d, xi[Q][3], w[Q]) of the library's direction order."""
    lib = load_library()
    d, q = ctypes.c_int(), ctypes.c_int()
    xi = (ctypes.c_int * 81)()
    w = (ctypes.c_double * 27)()
    rc = lib.vanse_lattice_info(lattice, ctypes.byref(d), ctypes.byref(q), xi, w)
    if rc:
        raise VanseError(rc, lib.vanse_last_error(None).decode())
    Q = q.value
    return d.value, [[xi[3 * k + a] for a in range(3)] for k in range(Q)], [w[k] for k in range(Q)]


def copy_probe(dst: torch.Tensor, src: torch.Tensor):
    lib = load_library()
    n = min(dst.numel() * dst.element_size(), src.numel() * src.element_size())
    n -= n % 16
    rc = lib.vanse_copy_probe(ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src.data_ptr()),
                              n, _stream_handle())
    if rc:
        raise VanseError(rc, lib.vanse_last_error(None).decode())


def diagnostics_noalloc(lattice, dims, f, phi, quad_axes=0, F=None, force=None, out=None):
    """vanse_diagnostics_noalloc: the sums of Solver.diagnostics from
    caller-owned FP64 CUDA tensors (f [Q, ncells] natural order, phi
    [ncells], force [d, ncells] or None) into `out` (a float64 CUDA tensor
    of 7, allocated here when None), asynchronously on the current stream;
    the library allocates nothing.  Returns out."""
    lib = load_library()
    if isinstance(lattice, str):
        lattice = LATTICES[lattice]
    dims = list(dims) + [1] * (3 - len(dims))
    arr = (ctypes.c_int64 * 3)(*[int(v) for v in dims])
    if out is None:
        out = torch.empty(7, dtype=torch.float64, device=f.device)
    # the library takes plain device pointers and cannot see their sizes:
    # check them here (an unknown lattice or bad dims is the library's EINVAL)
    q = {D2Q9: 9, D3Q19: 19, D3Q27: 27}.get(lattice)
    if q is not None and all(int(v) >= 1 for v in dims):
        n = int(dims[0]) * int(dims[1]) * int(dims[2])
        d = 2 if lattice == D2Q9 else 3
        for name, t, want in (("f", f, q * n), ("phi", phi, n), ("force", force, d * n)):
            if t is not None and t.numel() != want:
                raise ValueError("%s must have %d values, not %d" % (name, want, t.numel()))
    if out.numel() < 7:
        raise ValueError("out must hold 7 values")
    Fh = None if F is None else (ctypes.c_double * 3)(*[float(v) for v in list(F) + [0.0] * (3 - len(F))])
    rc = lib.vanse_diagnostics_noalloc(lattice, arr, _ptr(f), _ptr(phi), int(quad_axes), Fh,
                                       _ptr(force), _ptr(out), _stream_handle())
    if rc:
        raise VanseError(rc, lib.vanse_last_error(None).decode())
    return out


class Solver:
    """One periodic VANSE lattice Boltzmann solve on the current GPU.

    ``Solver(lattice, dims, tau, dtype)`` -> ``set_porosity`` -> (``set_force``)
    -> ``init`` -> ``step(n)`` -> ``moments()`` / ``diagnostics()``.
    All launches go to the torch current stream at the time of the call.
    """

    def __init__(self, lattice, dims, tau, dtype=FP64):
        self.lib = load_library()
        if isinstance(lattice, str):
            lattice = LATTICES[lattice]
        if isinstance(dtype, str):
            dtype = DTYPES[dtype]
        dims = list(dims) + [1] * (3 - len(dims))
        self.lattice, self.dtype, self.tau = lattice, dtype, float(tau)
        self.dims = tuple(int(v) for v in dims)
        self.d = 2 if lattice == D2Q9 else 3
        self.q = {D2Q9: 9, D3Q19: 19, D3Q27: 27}[lattice]
        self.ncells = self.dims[0] * self.dims[1] * self.dims[2]
        self.device = torch.device("cuda", torch.cuda.current_device())
        h = ctypes.c_void_p()
        arr = (ctypes.c_int64 * 3)(*self.dims)
        rc = self.lib.vanse_create(lattice, arr, self.tau, dtype, ctypes.byref(h))
        if rc:
            raise VanseError(rc, self.lib.vanse_last_error(None).decode())
        self.h = h

    # -- plumbing ------------------------------------------------------
    def _check(self, rc):
        if rc:
            raise VanseError(rc, self.lib.vanse_last_error(self.h).decode())

    def _bind_stream(self):
        self._check(self.lib.vanse_set_stream(self.h, _stream_handle()))

    def close(self):
        if getattr(self, "h", None):
            self.lib.vanse_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- the C ABI -------------------------------------------------------
    def set_porosity(self, eps_mean, eps_pert=None, period=0.0, quad_axes=0):
        self._bind_stream()
        if eps_pert is not None:
            eps_pert = eps_pert.to(self.device, torch.float64).contiguous().view(-1)
            if eps_pert.numel() != self.ncells:
                raise ValueError("eps_pert must have %d cells" % self.ncells)
        self._check(self.lib.vanse_set_porosity(self.h, float(eps_mean), _ptr(eps_pert),
                                                float(period), int(quad_axes)))

    def set_tuning(self, block=256, flags=0):
        """Threads per block (64 .. 1024) and TUNE_* flags of the step kernel;
        results are bitwise identical for every setting."""
        self._check(self.lib.vanse_set_tuning(self.h, int(block), int(flags)))

    def set_tile(self, tile_x=256, tile_y=1):
        """Tile of the step kernel (see vanse_set_tile); bitwise-neutral."""
        self._check(self.lib.vanse_set_tile(self.h, int(tile_x), int(tile_y)))

    def set_fused(self, rows=2, planes=32):
        """Two-step launch with tiles of `rows` full x-rows and `planes`
        z-planes (see vanse_set_fused; rows=0 switches it off); results are
        bitwise identical to single steps."""
        self._bind_stream()
        self._check(self.lib.vanse_set_fused(self.h, int(rows), int(planes)))

    def autotune(self, steps_per_trial=4):
        """Pick the fastest launch shape on real steps (see vanse_autotune).
        Returns a Launch(tile_x, tile_y, flags, fused_rows, fused_planes,
        steps_run)."""
        self._bind_stream()
        v = [ctypes.c_int() for _ in range(5)]
        n = ctypes.c_int64()
        self._check(self.lib.vanse_autotune(self.h, int(steps_per_trial),
                                            *[ctypes.byref(x) for x in v], ctypes.byref(n)))
        return Launch(*[x.value for x in v], n.value)

    def set_force_field(self, F=None):
        """Per-cell force density, FP64 [d, ncells] (None switches it off)."""
        self._bind_stream()
        if F is not None:
            F = F.to(self.device, torch.float64).contiguous().view(self.d, self.ncells)
            self._keep_force = F  # alive until the copy has run
        self._check(self.lib.vanse_set_force_field(self.h, _ptr(F)))

    def set_force(self, F):
        F = list(F) + [0.0] * (3 - len(F))
        arr = (ctypes.c_double * 3)(*[float(v) for v in F])
        self._check(self.lib.vanse_set_force(self.h, arr))

    def init(self, rho0=None, u0=None):
        self._bind_stream()
        if rho0 is not None:
            rho0 = rho0.to(self.device, torch.float64).contiguous().view(-1)
        if u0 is not None:
            u0 = u0.to(self.device, torch.float64).contiguous().view(self.d, self.ncells)
        self._keep = (rho0, u0)  # alive until the init kernel has run
        self._check(self.lib.vanse_init(self.h, _ptr(rho0), _ptr(u0)))

    def step(self, n=1):
        self._bind_stream()
        self._check(self.lib.vanse_step(self.h, int(n)))

    def moments(self):
        """(rho[ncells], p[ncells], u[d, ncells]) as FP64 tensors at t_n."""
        self._bind_stream()
        rho = torch.empty(self.ncells, dtype=torch.float64, device=self.device)
        p = torch.empty_like(rho)
        u = torch.empty(self.d, self.ncells, dtype=torch.float64, device=self.device)
        self._check(self.lib.vanse_moments(self.h, _ptr(rho), _ptr(p), _ptr(u)))
        return rho, p, u

    def populations(self):
        """f_i(x, t_n) as an FP64 tensor [Q, ncells] in the library's order."""
        self._bind_stream()
        f = torch.empty(self.q, self.ncells, dtype=torch.float64, device=self.device)
        self._check(self.lib.vanse_populations(self.h, _ptr(f)))
        return f

    def diagnostics(self):
        """(mass, momentum[3], force_sum[3]); synchronises."""
        self._bind_stream()
        out = (ctypes.c_double * 7)()
        self._check(self.lib.vanse_diagnostics(self.h, out))
        return out[0], [out[1], out[2], out[3]], [out[4], out[5], out[6]]

    @property
    def time(self):
        t = ctypes.c_int64()
        self._check(self.lib.vanse_time(self.h, ctypes.byref(t)))
        return t.value

    @property
    def device_bytes(self):
        b = ctypes.c_int64()
        self._check(self.lib.vanse_device_bytes(self.h, ctypes.byref(b)))
        return b.value


class Batch:
    """Many independent solves advanced together: one batched kernel launch
    per time step (hipGraph-captured in chunks).  The solvers stay owned by
    the caller and must outlive the batch."""

    def __init__(self, solvers):
        self.lib = load_library()
        self.solvers = list(solvers)
        arr = (ctypes.c_void_p * len(self.solvers))(*[s.h.value for s in self.solvers])
        h = ctypes.c_void_p()
        rc = self.lib.vanse_batch_create(arr, len(self.solvers), ctypes.byref(h))
        if rc:
            raise VanseError(rc, self.lib.vanse_batch_last_error(None).decode())
        self.h = h

    def _check(self, rc):
        if rc:
            raise VanseError(rc, self.lib.vanse_batch_last_error(self.h).decode())

    def _bind_stream(self):
        self._check(self.lib.vanse_batch_set_stream(self.h, _stream_handle()))

    def set_tuning(self, block=256, flags=0, chunk=16):
        self._check(self.lib.vanse_batch_set_tuning(self.h, int(block), int(flags), int(chunk)))

    def update(self, solvers):
        """Replace the members (same lattice and dtype), reusing the tables."""
        solvers = list(solvers)
        arr = (ctypes.c_void_p * len(solvers))(*[s.h.value for s in solvers])
        self._check(self.lib.vanse_batch_update(self.h, arr, len(solvers)))
        self.solvers = solvers

    def step(self, n=1):
        self._bind_stream()
        self._check(self.lib.vanse_batch_step(self.h, int(n)))

    def autotune(self, steps_per_trial=10):
        """Returns (block, flags, steps_run); the trial steps are real steps."""
        self._bind_stream()
        b, f, n = ctypes.c_int(), ctypes.c_int(), ctypes.c_int64()
        self._check(self.lib.vanse_batch_autotune(self.h, int(steps_per_trial), ctypes.byref(b),
                                                  ctypes.byref(f), ctypes.byref(n)))
        return b.value, f.value, n.value

    def two_step_layout(self):
        """[(rows, planes)] per member of the two-step layout in effect."""
        n = len(self.solvers)
        rows, planes = (ctypes.c_int * n)(), (ctypes.c_int * n)()
        self._check(self.lib.vanse_batch_two_step_layout(self.h, n, rows, planes))
        return list(zip(rows, planes))

    def two_step_tiles(self):
        """[(cols, rows, planes)] per member of the two-step layout in effect
        (cols = nx for tiles of full x-rows)."""
        n = len(self.solvers)
        cols, rows, planes = (ctypes.c_int * n)(), (ctypes.c_int * n)(), (ctypes.c_int * n)()
        self._check(self.lib.vanse_batch_two_step_tiles(self.h, n, cols, rows, planes))
        return list(zip(cols, rows, planes))

    def close(self):
        if getattr(self, "h", None):
            self.lib.vanse_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
