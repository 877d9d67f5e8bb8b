"""Python binding of libsapdd (the C ABI in include/sapdd.h): argument marshalling only.

Every operation runs in the HIP library; this module converts numpy arrays (host
pointers) or torch CUDA tensors (device pointers) into the C calls and raises
SapddError on a negative status. There is no CPU fallback: if libsapdd.so is missing or
cannot be loaded, `load_library` raises.

Arrays use the canonical layouts of the header: complex128 links [t,z,y,x,4,3,3],
spinors [rhs,t,z,y,x,4,3] (or [t,z,y,x,4,3] for one right-hand side) and clover
[t,z,y,x,12,12].
"""
from __future__ import annotations

import ctypes as C
import os
import weakref
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# SAPDD_LIB points the binding at another build of the library (for comparing builds)
LIB_PATH = os.environ.get("SAPDD_LIB") or os.path.join(HERE, "libsapdd.so")

OK, EINVAL, ENOMEM, EDEVICE, ENOCONV, ESINGULAR, ENAN, EFULL = 0, -1, -2, -3, -4, -5, -6, -7
F64, F32, F16, F16_LINKS = 0, 1, 2, 3
DEVICE_PTRS, USE_X0, NO_GRAPH, LINKS12, ELASTIC = 1, 2, 4, 8, 16
# "f16l": FP16 links and clover with FP32 Schwarz spinors (Schwarz precision only)
PRECS = {"f64": F64, "f32": F32, "f16": F16, "f16l": F16_LINKS}

# Entry points declared in include/sapdd.h (the CPU tests check the library exports them).
EXPORTS = (
    "sapdd_create", "sapdd_destroy", "sapdd_last_error", "sapdd_load_gauge",
    "sapdd_compute_clover", "sapdd_load_clover", "sapdd_free_field", "sapdd_apply_D",
    "sapdd_apply_block_D", "sapdd_sap", "sapdd_sap_noalloc", "sapdd_solve", "sapdd_solve_footprint", "sapdd_copy",
    "sapdd_profile", "sapdd_batch_create", "sapdd_batch_destroy", "sapdd_batch_add",
    "sapdd_batch_step", "sapdd_batch_poll", "sapdd_batch_memory", "sapdd_batch_trim", "sapdd_batch_take", "sapdd_mg_setup", "sapdd_mg_destroy",
    "sapdd_mg_prolongator", "sapdd_mg_coarse_operator", "sapdd_mg_coarse_solve", "sapdd_mg_precond",
    "sapdd_mg_solve", "sapdd_batch_set_mg",
)
KERNELS = ("sap_half", "dslash", "gram_schmidt", "block_dslash", "update", "copy", "mg_fine", "mg_coarse")


class SapddError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"sapdd error {code}: {msg}")
        self.code = code


class Params(C.Structure):
    _fields_ = [("block", C.c_int * 4), ("nmr", C.c_int), ("ncy", C.c_int), ("restart", C.c_int),
                ("max_iter", C.c_int), ("tol", C.c_double), ("sap_prec", C.c_int), ("flags", C.c_int),
                ("deflate", C.c_int), ("gap", C.c_double)]


class MgParams(C.Structure):
    _fields_ = [("nvec", C.c_int), ("setup_iters", C.c_int), ("coarse_iters", C.c_int),
                ("coarse_cycles", C.c_int), ("coarse_form", C.c_int)]


class KernelProfile(C.Structure):
    _fields_ = [("launches", C.c_longlong * 8), ("seconds", C.c_double * 8)]

    def as_dict(self):
        return {k: dict(launches=int(self.launches[i]), seconds=float(self.seconds[i]))
                for i, k in enumerate(KERNELS)}


class Stats(C.Structure):
    _fields_ = [("iters", C.c_int), ("restarts", C.c_int), ("converged", C.c_int),
                ("true_relres", C.c_double), ("implicit_relres", C.c_double),
                ("t_total", C.c_double), ("t_sap", C.c_double), ("t_dslash", C.c_double),
                ("t_gs", C.c_double), ("t_host", C.c_double), ("gap_restarts", C.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libsapdd.so and declare its signatures. Raises if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_1502_04025_amd.build`")
    try:  # torch carries its own HIP runtime: load it first so the library binds to that one
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = C.CDLL(path)
    P, I, D, VP = C.POINTER, C.c_int, C.c_double, C.c_void_p
    lib.sapdd_create.argtypes = [I, VP, P(VP)]
    lib.sapdd_destroy.argtypes = [VP]
    lib.sapdd_destroy.restype = None
    lib.sapdd_last_error.argtypes = [VP]
    lib.sapdd_last_error.restype = C.c_char_p
    lib.sapdd_load_gauge.argtypes = [VP, P(I), P(I), VP, I, I, P(VP)]
    lib.sapdd_compute_clover.argtypes = [VP, VP, D]
    lib.sapdd_load_clover.argtypes = [VP, VP, VP, I]
    lib.sapdd_free_field.argtypes = [VP, VP]
    lib.sapdd_apply_D.argtypes = [VP, VP, D, I, I, VP, VP, I]
    lib.sapdd_apply_block_D.argtypes = [VP, VP, D, I, I, VP, VP, I]
    lib.sapdd_sap.argtypes = [VP, VP, P(D), P(Params), I, VP, VP]
    lib.sapdd_sap_noalloc.argtypes = [VP, VP, P(D), P(Params), I, VP, VP]
    lib.sapdd_solve.argtypes = [VP, VP, P(D), P(Params), I, VP, VP, P(Stats)]
    lib.sapdd_solve_footprint.argtypes = [VP, P(Params), I]
    lib.sapdd_solve_footprint.restype = C.c_longlong
    lib.sapdd_copy.argtypes = [VP, VP, VP, C.c_longlong]
    lib.sapdd_profile.argtypes = [VP, I, P(KernelProfile)]
    lib.sapdd_batch_create.argtypes = [VP, VP, P(Params), I, P(VP)]
    lib.sapdd_batch_destroy.argtypes = [VP]
    lib.sapdd_batch_add.argtypes = [VP, D, VP, VP, I, P(I)]
    lib.sapdd_batch_step.argtypes = [VP, P(I)]
    lib.sapdd_batch_poll.argtypes = [VP, I, P(Stats)]
    lib.sapdd_batch_memory.argtypes = [VP, P(C.c_longlong)]
    lib.sapdd_batch_memory.restype = C.c_longlong
    lib.sapdd_batch_trim.argtypes = [VP, I]
    lib.sapdd_batch_trim.restype = C.c_longlong
    lib.sapdd_batch_take.argtypes = [VP, I, VP, I, P(Stats)]
    lib.sapdd_mg_setup.argtypes = [VP, VP, D, P(Params), P(MgParams), VP, I, P(VP)]
    lib.sapdd_mg_destroy.argtypes = [VP]
    lib.sapdd_mg_prolongator.argtypes = [VP, VP, I]
    lib.sapdd_mg_coarse_operator.argtypes = [VP, VP, I]
    lib.sapdd_mg_coarse_solve.argtypes = [VP, I, VP, VP, I]
    lib.sapdd_mg_precond.argtypes = [VP, I, VP, VP, I]
    lib.sapdd_mg_solve.argtypes = [VP, P(Params), I, VP, VP, P(Stats)]
    lib.sapdd_batch_set_mg.argtypes = [VP, VP]
    for name in EXPORTS:
        if name not in ("sapdd_destroy", "sapdd_last_error", "sapdd_solve_footprint", "sapdd_batch_memory",
                        "sapdd_batch_trim"):
            getattr(lib, name).restype = I
    _lib = lib
    return lib


def _is_torch(a) -> bool:
    return type(a).__module__.startswith("torch")


def _ptr(a, writable=False):
    """(pointer, is_device) of a C-contiguous complex128 numpy array or torch tensor."""
    if _is_torch(a):
        if not a.is_contiguous():
            raise ValueError("tensor must be contiguous")
        import torch
        if a.dtype != torch.complex128:
            raise ValueError("tensor must be complex128")
        return C.c_void_p(a.data_ptr()), a.is_cuda
    if not isinstance(a, np.ndarray) or a.dtype != np.complex128 or not a.flags.c_contiguous:
        raise ValueError("array must be a C-contiguous complex128 numpy array")
    if writable and not a.flags.writeable:
        raise ValueError("output array is read-only")
    return C.c_void_p(a.ctypes.data), False


def _empty_like(a):
    if _is_torch(a):
        import torch
        return torch.empty_like(a)
    return np.empty_like(a)


@dataclass
class SolveResult:
    x: object
    stats: list
    status: int


class Context:
    """One device + stream + workspaces. stream: a torch.cuda.Stream, a raw hipStream_t
    integer, or None for the null stream."""

    def __init__(self, device: int = 0, stream=None):
        self.lib = load_library()
        if stream is not None and not isinstance(stream, int):
            stream = stream.cuda_stream
        h = C.c_void_p()
        rc = self.lib.sapdd_create(int(device), C.c_void_p(stream or 0), C.byref(h))
        if rc != OK:
            raise SapddError(rc, "sapdd_create failed")
        self.h = h
        self.device = device

    def _check(self, rc):
        if rc != OK:
            raise SapddError(rc, self.lib.sapdd_last_error(self.h).decode())
        return rc

    def close(self):
        if getattr(self, "h", None):
            self.lib.sapdd_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def load_gauge(self, links, block, antiperiodic: bool = True) -> "Field":
        lt, lz, ly, lx = links.shape[:4]
        if tuple(links.shape[4:]) != (4, 3, 3):
            raise ValueError("links must have shape [t,z,y,x,4,3,3]")
        dims = (C.c_int * 4)(lx, ly, lz, lt)
        blk = (C.c_int * 4)(*[int(b) for b in block])
        p, dev = _ptr(links)
        h = C.c_void_p()
        self._check(self.lib.sapdd_load_gauge(self.h, dims, blk, p, int(bool(antiperiodic)),
                                              DEVICE_PTRS if dev else 0, C.byref(h)))
        return Field(self, h, (lx, ly, lz, lt), tuple(int(b) for b in block))

    def profile(self, enable, families=None):
        """Return the per-kernel profile accumulated so far, reset it and switch
        profiling on or off; `families` (names from KERNELS) limits the recording."""
        kp = KernelProfile()
        code = int(bool(enable))
        if enable and families:
            code = sum(1 << KERNELS.index(f) for f in families) << 1
        self._check(self.lib.sapdd_profile(self.h, code, C.byref(kp)))
        return kp.as_dict()

    def copy(self, src, dst, nbytes: int):
        self._check(self.lib.sapdd_copy(self.h, C.c_void_p(src), C.c_void_p(dst), int(nbytes)))


class Field:
    """A resident gauge field (links + clover term) with a fixed Schwarz blocking."""

    def __init__(self, ctx: Context, h, dims, block):
        self.ctx, self.h, self.dims, self.block = ctx, h, dims, block
        self._deps = weakref.WeakSet()  # batches and multigrid objects built on this field

    def free(self):
        """Free the field; batches and multigrid objects built on it are closed first (the
        library requires that order)."""
        if self.h:
            for d in list(self._deps):
                d.close()
            self.ctx.lib.sapdd_free_field(self.ctx.h, self.h)
            self.h = None

    def __del__(self):
        try:
            if self.h and self.ctx.h:
                self.free()
        except Exception:
            pass

    def compute_clover(self, csw: float):
        self.ctx._check(self.ctx.lib.sapdd_compute_clover(self.ctx.h, self.h, float(csw)))

    def load_clover(self, clover):
        p, dev = _ptr(clover)
        self.ctx._check(self.ctx.lib.sapdd_load_clover(self.ctx.h, self.h, p, DEVICE_PTRS if dev else 0))

    @staticmethod
    def _nrhs(psi):
        return 1 if psi.ndim == 6 else int(psi.shape[0])

    def _apply(self, fn, kappa, psi, prec, out, flags=0):
        out = _empty_like(psi) if out is None else out
        pi, dev = _ptr(psi)
        po, dev2 = _ptr(out, writable=True)
        if dev != dev2:
            raise ValueError("input and output must both be host or both be device arrays")
        self.ctx._check(fn(self.ctx.h, self.h, float(kappa), PRECS[prec] if isinstance(prec, str) else int(prec),
                           self._nrhs(psi), pi, po, (DEVICE_PTRS if dev else 0) | flags))
        return out

    def apply_D(self, kappa, psi, prec="f64", out=None):
        return self._apply(self.ctx.lib.sapdd_apply_D, kappa, psi, prec, out)

    def apply_block_D(self, kappa, psi, prec="f64", out=None, links12=False):
        """M_B psi; links12: links read as their first two rows (FP32/FP16 storage)."""
        return self._apply(self.ctx.lib.sapdd_apply_block_D, kappa, psi, prec, out, LINKS12 if links12 else 0)

    def params(self, nmr=4, ncy=5, restart=16, max_iter=1000, tol=1e-10, prec="f64", flags=0,
               deflate=0, gap=0.0) -> Params:
        p = Params()
        for i in range(4):
            p.block[i] = self.block[i]
        p.nmr, p.ncy, p.restart, p.max_iter, p.tol = nmr, ncy, restart, max_iter, tol
        p.sap_prec = PRECS[prec] if isinstance(prec, str) else int(prec)
        p.flags = flags
        p.deflate = deflate
        p.gap = float(gap)
        return p

    def sap(self, kappa, psi, out=None, **kw):
        """SAP(psi); kappa is a float or one value per right-hand side."""
        prm = self.params(**kw)
        nrhs = self._nrhs(psi)
        kap = np.broadcast_to(np.asarray(kappa, dtype=np.float64), (nrhs,)).copy()
        out = _empty_like(psi) if out is None else out
        pi, dev = _ptr(psi)
        po, _ = _ptr(out, writable=True)
        if dev:
            prm.flags |= DEVICE_PTRS
        self.ctx._check(self.ctx.lib.sapdd_sap(self.ctx.h, self.h, kap.ctypes.data_as(C.POINTER(C.c_double)),
                                               C.byref(prm), nrhs, pi, po))
        return out

    def sap_noalloc(self, kappa, psi, out, **kw):
        """SAP(psi) through the allocation-free entry point (psi and out must be device tensors)."""
        prm = self.params(**kw)
        nrhs = self._nrhs(psi)
        kap = np.broadcast_to(np.asarray(kappa, dtype=np.float64), (nrhs,)).copy()
        pi, dev = _ptr(psi)
        po, dev2 = _ptr(out, writable=True)
        if dev and dev2:
            prm.flags |= DEVICE_PTRS  # the library rejects host arrays itself
        self.ctx._check(self.ctx.lib.sapdd_sap_noalloc(self.ctx.h, self.h, kap.ctypes.data_as(C.POINTER(C.c_double)),
                                                       C.byref(prm), nrhs, pi, po))
        return out

    def footprint(self, nrhs=1, **kw) -> int:
        prm = self.params(**kw)
        return int(self.ctx.lib.sapdd_solve_footprint(self.h, C.byref(prm), int(nrhs)))

    def solve(self, kappa, b, x=None, x0=None, raise_on_noconv=True, **kw) -> SolveResult:
        """Solve M x = b; kappa is a float or one value per right-hand side."""
        nrhs = self._nrhs(b)
        prm = self.params(**kw)
        kap = np.broadcast_to(np.asarray(kappa, dtype=np.float64), (nrhs,)).copy()
        if x is None:
            x = _empty_like(b)
        if x0 is not None:
            x[...] = x0
            prm.flags |= USE_X0
        pb, dev = _ptr(b)
        px, _ = _ptr(x, writable=True)
        if dev:
            prm.flags |= DEVICE_PTRS
        stats = (Stats * nrhs)()
        rc = self.ctx.lib.sapdd_solve(self.ctx.h, self.h, kap.ctypes.data_as(C.POINTER(C.c_double)),
                                      C.byref(prm), nrhs, pb, px, stats)
        if rc != OK and not (rc == ENOCONV and not raise_on_noconv):
            self.ctx._check(rc)
        return SolveResult(x, [s.as_dict() for s in stats], rc)


class Batch:
    """Continuous-batching solver on one field (sapdd_batch_*): slots join with add(),
    every step() runs one FGMRES restart cycle for all unfinished slots, finished slots
    leave with take()."""

    def __init__(self, field: "Field", capacity: int, elastic: bool = False, **kw):
        """elastic: commit a slot's device memory only while it is in use."""
        self.field = field
        self.ctx = field.ctx
        prm = field.params(**kw)
        if elastic:
            prm.flags |= ELASTIC
        self.prm = prm
        h = C.c_void_p()
        self.ctx._check(self.ctx.lib.sapdd_batch_create(self.ctx.h, field.h, C.byref(prm), int(capacity),
                                                        C.byref(h)))
        self.h = h
        self.capacity = int(capacity)
        field._deps.add(self)

    def close(self):
        if getattr(self, "h", None):
            self.ctx.lib.sapdd_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            if self.ctx.h:
                self.close()
        except Exception:
            pass

    def add(self, kappa: float, b, x0=None) -> int:
        """Admit one right-hand side (canonical spinor [t,z,y,x,4,3]); returns its slot.
        Raises SapddError with code EFULL when every slot is taken."""
        pb, dev = _ptr(b)
        px = C.c_void_p(0)
        if x0 is not None:
            px, _ = _ptr(x0)
        slot = C.c_int()
        self.ctx._check(self.ctx.lib.sapdd_batch_add(self.h, float(kappa), pb, px, DEVICE_PTRS if dev else 0,
                                                     C.byref(slot)))
        return slot.value

    def memory(self):
        """(bytes the batch holds now, most bytes one more slot can commit)."""
        slot = C.c_longlong()
        held = self.ctx.lib.sapdd_batch_memory(self.h, C.byref(slot))
        return int(held), int(slot.value)

    def trim(self, keep: int = 0) -> int:
        """Elastic batch: release the memory of free slots kept from earlier use, keeping at
        most `keep` of them; returns the bytes released."""
        n = self.ctx.lib.sapdd_batch_trim(self.h, int(keep))
        if n < 0:
            self.ctx._check(int(n))
        return int(n)

    def step(self) -> int:
        """One restart cycle for every unfinished slot; returns how many are unfinished."""
        n = C.c_int()
        self.ctx._check(self.ctx.lib.sapdd_batch_step(self.h, C.byref(n)))
        return n.value

    def poll(self, slot: int):
        st = Stats()
        rc = self.ctx.lib.sapdd_batch_poll(self.h, int(slot), C.byref(st))
        if rc < 0:
            raise SapddError(rc, "bad slot")
        return bool(rc), st.as_dict()

    def set_mg(self, mg: "Multigrid"):
        """Precondition with the two-level multigrid instead of SAP (no slot in use; every
        right-hand side added later must use the multigrid's kappa)."""
        self.ctx._check(self.ctx.lib.sapdd_batch_set_mg(self.h, mg.h))
        self.mg = mg  # keeps the multigrid alive as long as the batch
        mg._users.add(self)

    def take(self, slot: int, out):
        """Copy the solution of a slot into `out` (host array or device tensor), free it."""
        po, dev = _ptr(out, writable=True)
        st = Stats()
        self.ctx._check(self.ctx.lib.sapdd_batch_take(self.h, int(slot), po, DEVICE_PTRS if dev else 0,
                                                      C.byref(st)))
        return st.as_dict()


class Multigrid:
    """Two-level multigrid preconditioner with SAP as smoother (sapdd_mg_*), for one field
    and kappa. vecs: the nvec test vectors (canonical spinors [nvec,t,z,y,x,4,3]);
    coarse_form: 0 = two launches per coarse Arnoldi step (batches), 1 = one (a single
    system); smoother keywords (nmr, ncy, prec) as Field.params."""

    def __init__(self, field: "Field", kappa: float, vecs, setup_iters=0, coarse_iters=16, coarse_cycles=1,
                 coarse_form=0, **smoother):
        self.field, self.ctx, self.kappa = field, field.ctx, float(kappa)
        self.nvec = int(vecs.shape[0])
        self.K = 2 * self.nvec
        self.grid = tuple(field.dims[mu] // field.block[mu] for mu in range(4))  # x, y, z, t
        prm = field.params(**smoother)
        mp = MgParams(self.nvec, int(setup_iters), int(coarse_iters), int(coarse_cycles), int(coarse_form))
        pv, dev = _ptr(vecs)
        h = C.c_void_p()
        self.ctx._check(self.ctx.lib.sapdd_mg_setup(self.ctx.h, field.h, self.kappa, C.byref(prm), C.byref(mp), pv,
                                                    DEVICE_PTRS if dev else 0, C.byref(h)))
        self.h = h
        self._users = weakref.WeakSet()  # batches that precondition with this multigrid
        field._deps.add(self)

    def close(self):
        """Destroy the multigrid; batches that precondition with it are closed first."""
        if getattr(self, "h", None):
            for b in list(self._users):
                b.close()
            self.ctx.lib.sapdd_mg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            if self.ctx.h:
                self.close()
        except Exception:
            pass

    def _coarse_shape(self):
        gx, gy, gz, gt = self.grid
        return (gt, gz, gy, gx)

    def prolongator(self):
        """The nvec interpolation fields as canonical spinors (host array)."""
        lx, ly, lz, lt = self.field.dims
        out = np.empty((self.nvec, lt, lz, ly, lx, 4, 3), dtype=np.complex128)
        po, _ = _ptr(out, writable=True)
        self.ctx._check(self.ctx.lib.sapdd_mg_prolongator(self.h, po, 0))
        return out

    def coarse_operator(self):
        """D_c as [Gt,Gz,Gy,Gx,9,K,K] (block d: 0 itself, 1 + 2 mu forward, 2 + 2 mu
        backward neighbour; row, column)."""
        out = np.empty(self._coarse_shape() + (9, self.K, self.K), dtype=np.complex128)
        po, _ = _ptr(out, writable=True)
        self.ctx._check(self.ctx.lib.sapdd_mg_coarse_operator(self.h, po, 0))
        return out

    def coarse_solve(self, rhs):
        """The coarse solve of D_c e = rhs (restarted GMRES from zero), rhs [n,Gt,Gz,Gy,Gx,K]."""
        rhs = np.ascontiguousarray(rhs, dtype=np.complex128)
        out = np.empty_like(rhs)
        pi, _ = _ptr(rhs)
        po, _ = _ptr(out, writable=True)
        self.ctx._check(self.ctx.lib.sapdd_mg_coarse_solve(self.h, int(rhs.shape[0]), pi, po, 0))
        return out

    def precond(self, psi, out=None):
        """B(psi) for canonical spinors [nrhs,t,z,y,x,4,3]."""
        out = _empty_like(psi) if out is None else out
        pi, dev = _ptr(psi)
        po, _ = _ptr(out, writable=True)
        self.ctx._check(self.ctx.lib.sapdd_mg_precond(self.h, Field._nrhs(psi), pi, po, DEVICE_PTRS if dev else 0))
        return out

    def solve(self, b, x=None, x0=None, raise_on_noconv=True, **kw) -> SolveResult:
        """Solve M x = b with FGMRES preconditioned by the multigrid cycle; solver and
        smoother keywords as Field.params."""
        nrhs = Field._nrhs(b)
        prm = self.field.params(**kw)
        if x is None:
            x = _empty_like(b)
        if x0 is not None:
            x[...] = x0
            prm.flags |= USE_X0
        pb, dev = _ptr(b)
        px, _ = _ptr(x, writable=True)
        if dev:
            prm.flags |= DEVICE_PTRS
        stats = (Stats * nrhs)()
        rc = self.ctx.lib.sapdd_mg_solve(self.h, C.byref(prm), nrhs, pb, px, stats)
        if rc != OK and not (rc == ENOCONV and not raise_on_noconv):
            self.ctx._check(rc)
        return SolveResult(x, [s.as_dict() for s in stats], rc)
