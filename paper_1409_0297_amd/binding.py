"""ctypes binding of include/spp.h: the same entry points, argument marshalling only.

Device arrays are PyTorch CUDA tensors (ROCm); their data pointers and the
current stream are handed to the C ABI unchanged.  Every computation happens
in libspp.so.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))

SPP_OK, SPP_EINVAL, SPP_ESINGULAR_SHIFT, SPP_EBREAKDOWN = 0, -1, -2, -3
SPP_NOT_CONVERGED, SPP_ENOMEM, SPP_EHIP, SPP_ENOTIMPL = -4, -5, -6, -7
SPP_HELMHOLTZ, SPP_SCHRODINGER, SPP_MAXWELL = 0, 1, 2
SPP_C128, SPP_C64_FRONTS = 0, 1
SPP_ORDER_OCTREE, SPP_ORDER_BISECT = 0, 1
SPP_F_UNPRECONDITIONED = 1
SPP_F_TIMING = 2
SPP_F_PARTIAL_PIVOTING = 4
SPP_F_GRAPHS = 8
SPP_F_PERSISTENT = 16
SPP_F_AUTOTUNE = 32
SPP_F_NO_SIDE = 64
SPP_F_STREAMED = 128
SPP_K_FFT, SPP_K_GEMV, SPP_K_TRI, SPP_K_GEMM, SPP_K_PANEL, SPP_K_QAPPLY = 0, 1, 2, 3, 4, 5
SPP_K_INV, SPP_K_SOLVE_BLK = 6, 7
KERNEL_CLASSES = {"fft": 0, "gemv": 1, "tri": 2, "gemm": 3, "panel": 4, "qapply": 5, "inv": 6, "solve_blk": 7}

ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class spp_problem(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("n", ctypes.c_int32), ("b", ctypes.c_int32),
                ("kind", ctypes.c_int32), ("omega", ctypes.c_double), ("ell", ctypes.c_double),
                ("energy", ctypes.c_double), ("coeff", ctypes.c_void_p)]


class spp_options(ctypes.Structure):
    _fields_ = [("prec", ctypes.c_int32), ("order", ctypes.c_int32), ("tol", ctypes.c_double),
                ("max_iter", ctypes.c_int32), ("flags", ctypes.c_int32), ("restart", ctypes.c_int32),
                ("pattern", ctypes.c_int32), ("alloc", ALLOC_FN), ("free", FREE_FN),
                ("alloc_ctx", ctypes.c_void_p)]


class spp_stats_t(ctypes.Structure):
    _fields_ = [("s", ctypes.c_double), ("shift_moves", ctypes.c_int32),
                ("n_fronts", ctypes.c_int32), ("n_levels", ctypes.c_int32),
                ("max_front", ctypes.c_int32), ("factor_entries", ctypes.c_int64),
                ("factor_bytes", ctypes.c_int64), ("factor_flops", ctypes.c_double),
                ("t_setup_ms", ctypes.c_double), ("t_factor_ms", ctypes.c_double),
                ("t_solve_ms", ctypes.c_double), ("last_iters", ctypes.c_int32),
                ("breakdown_front", ctypes.c_int32), ("last_cycles", ctypes.c_int32),
                ("storage", ctypes.c_int32), ("pivot_growth", ctypes.c_double),
                ("min_pivot", ctypes.c_double), ("device_bytes", ctypes.c_int64),
                ("small_pivots", ctypes.c_int32), ("reserved_stats", ctypes.c_int32)]


_LIB = None


def library_path() -> str:
    return os.path.join(HERE, "libspp.so")


def library():
    """Loads libspp.so once; raises if it has not been built."""
    global _LIB
    if _LIB is not None:
        return _LIB
    path = library_path()
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library {path} is missing: run __graft_entry__.build() first")
    lib = ctypes.CDLL(path)
    P, I, D, V = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double, None
    sig = {
        "spp_setup": (I, [ctypes.POINTER(spp_problem), ctypes.POINTER(spp_options), P, ctypes.POINTER(P)]),
        "spp_setup_batch": (I, [ctypes.POINTER(spp_problem), I, ctypes.POINTER(spp_options), P, ctypes.POINTER(P)]),
        "spp_get_shift": (I, [P, I, ctypes.POINTER(D), ctypes.POINTER(I)]),
        "spp_solve": (I, [P, P, I, P, ctypes.POINTER(I), ctypes.POINTER(D), P]),
        "spp_solve_batch": (I, [P, ctypes.POINTER(P), ctypes.POINTER(I), ctypes.POINTER(P), ctypes.POINTER(I),
                                ctypes.POINTER(D), P]),
        "spp_apply_operator": (I, [P, P, P, I, P]),
        "spp_apply_operator_noalloc": (I, [P, P, P, I, P]),
        "spp_apply_green": (I, [P, P, P, I, P]),
        "spp_apply_q": (I, [P, P, P, I, P]),
        "spp_apply_precond": (I, [P, P, P, I, P]),
        "spp_get_coefficients": (I, [P, ctypes.POINTER(D), P]),
        "spp_get_stencil": (I, [P, I, ctypes.POINTER(I), ctypes.POINTER(I), P, P, P]),
        "spp_stats": (I, [P, ctypes.POINTER(spp_stats_t)]),
        "spp_kernel_timing": (I, [P, I, ctypes.POINTER(D), ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(D),
                                  ctypes.POINTER(D)]),
        "spp_kernel_timing_reset": (I, [P]),
        "spp_destroy": (V, [P]),
        "spp_error_string": (ctypes.c_char_p, [I]),
        "spp_cnn_create": (I, [I, I, ctypes.POINTER(I), I, I, ctypes.POINTER(P)]),
        "spp_cnn_weights": (I, [P, P, P, ctypes.POINTER(ctypes.c_int64)]),
        "spp_cnn_forward": (I, [P, P, I, P, P]),
        "spp_cnn_loss_grad": (I, [P, P, P, I, ctypes.POINTER(D), P, P]),
        "spp_cnn_adam_step": (I, [P, ctypes.c_float, P]),
        "spp_cnn_destroy": (V, [P]),
        "spp_cnn_last_error": (ctypes.c_char_p, []),
        "spp_attach_cnn": (I, [P, P, D]),
        "spp_learned_stats": (I, [P, ctypes.POINTER(I), ctypes.POINTER(I)]),
        "spp_get_krylov": (I, [P, I, P, P]),
        "spp_autotune": (I, [P, I, P]),
        "spp_tune_set": (I, [ctypes.c_char_p, I]),
        "spp_tune_get": (I, [ctypes.c_char_p, ctypes.POINTER(I)]),
        "spp_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _LIB = lib
    return lib


class SppError(RuntimeError):
    def __init__(self, code: int, where: str):
        lib = library()
        msg = f"{where}: {lib.spp_error_string(code).decode()} ({lib.spp_last_error().decode()})"
        super().__init__(msg)
        self.code = code


def _check(code: int, where: str, allow=(SPP_OK,)):
    if code not in allow:
        raise SppError(code, where)
    return code


# ----------------------------------------------------------------- raw entry points
def spp_setup(problem: spp_problem, options: spp_options, stream: int) -> int:
    h = ctypes.c_void_p()
    code = library().spp_setup(ctypes.byref(problem), ctypes.byref(options), ctypes.c_void_p(stream),
                               ctypes.byref(h))
    if code != SPP_OK and h.value:
        library().spp_destroy(h)
    _check(code, "spp_setup")
    return h.value


def spp_setup_batch(problems, options: spp_options, stream: int) -> int:
    arr = (spp_problem * len(problems))(*problems)
    h = ctypes.c_void_p()
    code = library().spp_setup_batch(arr, len(problems), ctypes.byref(options), ctypes.c_void_p(stream),
                                     ctypes.byref(h))
    if code != SPP_OK and h.value:
        library().spp_destroy(h)
    _check(code, "spp_setup_batch")
    return h.value


def spp_get_shift(handle, problem: int):
    s = ctypes.c_double()
    moves = ctypes.c_int32()
    _check(library().spp_get_shift(handle, problem, ctypes.byref(s), ctypes.byref(moves)), "spp_get_shift")
    return s.value, moves.value


def spp_solve(handle, f_ptr, nrhs, u_ptr, stream, nproblems: int = 1):
    """iters / relres are returned per (problem, right-hand side), problem-major."""
    iters = (ctypes.c_int32 * (nrhs * nproblems))()
    relres = (ctypes.c_double * (nrhs * nproblems))()
    code = library().spp_solve(handle, f_ptr, nrhs, u_ptr, iters, relres, ctypes.c_void_p(stream))
    _check(code, "spp_solve", allow=(SPP_OK, SPP_NOT_CONVERGED))
    return code, list(iters), list(relres)


def spp_solve_batch(handle, f_ptrs, nrhs, u_ptrs, stream):
    """Per-problem right-hand sides: f_ptrs / u_ptrs / nrhs one entry per
    problem; iters / relres are returned problem by problem."""
    n = len(nrhs)
    tot = sum(nrhs)
    fa = (ctypes.c_void_p * n)(*f_ptrs)
    ua = (ctypes.c_void_p * n)(*u_ptrs)
    na = (ctypes.c_int32 * n)(*nrhs)
    iters = (ctypes.c_int32 * max(tot, 1))()
    relres = (ctypes.c_double * max(tot, 1))()
    code = library().spp_solve_batch(handle, fa, na, ua, iters, relres, ctypes.c_void_p(stream))
    _check(code, "spp_solve_batch", allow=(SPP_OK, SPP_NOT_CONVERGED))
    return code, list(iters)[:tot], list(relres)[:tot]


class TorchAllocator:
    """spp_options allocator hook backed by PyTorch's caching allocator on the
    current device and stream (argument marshalling only: torch hands out the
    memory, the library uses it).  Counts the blocks it served."""

    def __init__(self):
        import torch
        self.torch = torch
        self.served = 0
        self.freed = 0
        self.bytes = 0

        def _alloc(nbytes, ctx):
            try:
                ptr = torch.cuda.caching_allocator_alloc(int(nbytes), torch.cuda.current_device(),
                                                         torch.cuda.current_stream())
            except RuntimeError:
                return None
            self.served += 1
            self.bytes += int(nbytes)
            return ptr

        def _free(ptr, ctx):
            self.freed += 1
            torch.cuda.caching_allocator_delete(ptr)

        self.alloc = ALLOC_FN(_alloc)
        self.free = FREE_FN(_free)

    def install(self, options: spp_options) -> spp_options:
        options.alloc = self.alloc
        options.free = self.free
        return options


def _apply(name, handle, a_ptr, b_ptr, nrhs, stream):
    _check(getattr(library(), name)(handle, a_ptr, b_ptr, nrhs, ctypes.c_void_p(stream)), name)


def spp_apply_operator(handle, z_ptr, w_ptr, nrhs, stream):
    _apply("spp_apply_operator", handle, z_ptr, w_ptr, nrhs, stream)


def spp_apply_operator_noalloc(handle, z_ptr, w_ptr, nrhs, stream):
    _apply("spp_apply_operator_noalloc", handle, z_ptr, w_ptr, nrhs, stream)


def spp_apply_green(handle, f_ptr, g_ptr, nrhs, stream):
    _apply("spp_apply_green", handle, f_ptr, g_ptr, nrhs, stream)


def spp_apply_q(handle, r_ptr, y_ptr, nrhs, stream):
    _apply("spp_apply_q", handle, r_ptr, y_ptr, nrhs, stream)


def spp_apply_precond(handle, r_ptr, z_ptr, nrhs, stream):
    _apply("spp_apply_precond", handle, r_ptr, z_ptr, nrhs, stream)


def spp_get_coefficients(handle, q_ptr):
    s = ctypes.c_double()
    _check(library().spp_get_coefficients(handle, ctypes.byref(s), q_ptr), "spp_get_coefficients")
    return s.value


def spp_get_stencil(handle, set_type, offsets=None, T=None, C=None):
    nS, nB = ctypes.c_int32(), ctypes.c_int32()
    _check(library().spp_get_stencil(handle, set_type, ctypes.byref(nS), ctypes.byref(nB),
                                     offsets, T, C), "spp_get_stencil")
    return nS.value, nB.value


def spp_stats(handle) -> dict:
    st = spp_stats_t()
    _check(library().spp_stats(handle, ctypes.byref(st)), "spp_stats")
    return {name: getattr(st, name) for name, _ in spp_stats_t._fields_}


def spp_kernel_timing(handle, kclass: int) -> dict:
    ms, n, by, fl = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double(), ctypes.c_double()
    _check(library().spp_kernel_timing(handle, kclass, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(by),
                                       ctypes.byref(fl)), "spp_kernel_timing")
    return {"ms": ms.value, "launches": n.value, "bytes": by.value, "flops": fl.value}


def spp_kernel_timing_reset(handle):
    _check(library().spp_kernel_timing_reset(handle), "spp_kernel_timing_reset")


def spp_destroy(handle):
    if handle:
        library().spp_destroy(handle)


def spp_error_string(code: int) -> str:
    return library().spp_error_string(code).decode()


def spp_last_error() -> str:
    return library().spp_last_error().decode()


# ----------------------------------------------------------------- convenience wrapper
class Solver:
    """One factorised problem: setup(grid, omega or E, c or V) -> factor; solve(f) -> u.

    ``coeff``: c(x_j) (Helmholtz), V(ell x_j) (Schroedinger) or eps(x_j)
    (Maxwell) as a float64 tensor of shape (n,)*d on the GPU (numpy arrays are
    copied there).  Maxwell fields have d components: vectors are
    (nrhs, d n^d), component-major.
    """

    def __init__(self, kind: str, n: int, d: int, b: int, coeff, omega: float = 0.0,
                 ell: float = 1.0, energy: float = 0.0, prec: str = "c128", order: str = "octree",
                 tol: float = 1e-10, max_iter: int = 200, unpreconditioned: bool = False,
                 timing: bool = False, partial_pivoting: bool = False, graphs: bool = False,
                 persistent: bool = False, autotune: bool = False, side_products: bool = True,
                 restart: int = 0, allocator: "TorchAllocator" = None, streamed: bool = False,
                 pattern: str = "sets"):
        import torch
        self.torch = torch
        self.n, self.d, self.b = n, d, b
        self.nc = d if kind == "maxwell" else 1      # unknowns per grid point
        self.npts = n ** d
        self.N = self.nc * self.npts
        dev = torch.device("cuda")
        c = torch.as_tensor(coeff, dtype=torch.float64, device=dev).contiguous()
        self._coeff = c
        kinds = {"helmholtz": SPP_HELMHOLTZ, "schrodinger": SPP_SCHRODINGER, "maxwell": SPP_MAXWELL}
        pb = spp_problem(dim=d, n=n, b=b, kind=kinds[kind],
                         omega=omega, ell=ell, energy=energy, coeff=c.data_ptr())
        op = spp_options(prec=SPP_C128 if prec == "c128" else SPP_C64_FRONTS,
                         order=SPP_ORDER_OCTREE if order == "octree" else SPP_ORDER_BISECT,
                         tol=tol, max_iter=max_iter,
                         flags=(SPP_F_UNPRECONDITIONED if unpreconditioned else 0)
                         | (SPP_F_TIMING if timing else 0)
                         | (SPP_F_PARTIAL_PIVOTING if partial_pivoting else 0)
                         | (SPP_F_GRAPHS if graphs else 0)
                         | (SPP_F_PERSISTENT if persistent else 0)
                         | (SPP_F_AUTOTUNE if autotune else 0)
                         | (0 if side_products else SPP_F_NO_SIDE)
                         | (SPP_F_STREAMED if streamed else 0), restart=restart,
                         pattern=0 if pattern == "sets" else 1)
        self._allocator = allocator
        if allocator is not None:
            allocator.install(op)
        self.handle = spp_setup(pb, op, self._stream())

    def _stream(self) -> int:
        return self.torch.cuda.current_stream().cuda_stream

    def _vec(self, x):
        t = self.torch.as_tensor(x, dtype=self.torch.complex128, device="cuda").contiguous()
        return t.reshape(-1, self.N) if t.numel() % self.N == 0 else t

    def _out(self, like):
        return self.torch.empty_like(like)

    def solve(self, f):
        fv = self._vec(f)
        u = self._out(fv)
        code, iters, relres = spp_solve(self.handle, fv.data_ptr(), fv.shape[0], u.data_ptr(), self._stream())
        return u, iters, relres, code

    def apply_operator(self, z):
        zv = self._vec(z)
        w = self._out(zv)
        spp_apply_operator(self.handle, zv.data_ptr(), w.data_ptr(), zv.shape[0], self._stream())
        return w

    def apply_green(self, f):
        fv = self._vec(f)
        g = self._out(fv)
        spp_apply_green(self.handle, fv.data_ptr(), g.data_ptr(), fv.shape[0], self._stream())
        return g

    def apply_q(self, r):
        rv = self._vec(r)
        y = self._out(rv)
        spp_apply_q(self.handle, rv.data_ptr(), y.data_ptr(), rv.shape[0], self._stream())
        return y

    def apply_precond(self, r):
        rv = self._vec(r)
        z = self._out(rv)
        spp_apply_precond(self.handle, rv.data_ptr(), z.data_ptr(), rv.shape[0], self._stream())
        return z

    def coefficients(self):
        q = self.torch.empty(self.npts, dtype=self.torch.float64, device="cuda")
        s = spp_get_coefficients(self.handle, q.data_ptr())
        self.torch.cuda.synchronize()
        return s, q

    def stencil(self, set_type: int):
        import numpy as np
        nS, nB = spp_get_stencil(self.handle, set_type)
        off = np.zeros(((nS + nB) // self.nc, self.d), dtype=np.int32)
        T = np.zeros((nS, nB), dtype=np.complex128)
        C = np.zeros((nS, nS + nB), dtype=np.complex128)
        spp_get_stencil(self.handle, set_type, off.ctypes.data, T.ctypes.data, C.ctypes.data)
        return off, T, C

    def stats(self) -> dict:
        return spp_stats(self.handle)

    def attach_cnn(self, cnn, rho: float = 0.9):
        """Use a trained CNN as the first preconditioner stage (None detaches)."""
        self._cnn = cnn
        spp_attach_cnn(self.handle, cnn.handle if cnn is not None else None, rho)

    def learned_stats(self):
        return spp_learned_stats(self.handle)

    def krylov(self, j: int, nrhs: int = 1):
        """(v_j, z_j) of the last solve as (nrhs, N) complex tensors."""
        v = self.torch.empty((nrhs, self.N), dtype=self.torch.complex128, device="cuda")
        z = self.torch.empty_like(v)
        spp_get_krylov(self.handle, j, v.data_ptr(), z.data_ptr())
        return v, z

    def close(self):
        if getattr(self, "handle", None):
            spp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BatchSolver:
    """Several independent problems factorised and solved together.

    ``problems``: list of dicts with keys kind ("helmholtz" / "schrodinger"),
    n, d, b, coeff and omega or ell / energy.  Every problem must have the
    same d.  ``solve(fs)`` takes one (nrhs, n_i^d) right-hand-side array per
    problem (the same nrhs for all) and returns per-problem solutions,
    iteration counts and true relative residuals.
    """

    def __init__(self, problems, prec: str = "c128", order: str = "octree", tol: float = 1e-10,
                 max_iter: int = 200, timing: bool = False, graphs: bool = False, persistent: bool = False,
                 restart: int = 0):
        import torch
        self.torch = torch
        self.sizes = [p["n"] ** p["d"] for p in problems]
        self.offsets = [0]
        for N in self.sizes:
            self.offsets.append(self.offsets[-1] + N)
        self._coeffs = []
        pbs = []
        for p in problems:
            c = torch.as_tensor(p["coeff"], dtype=torch.float64, device="cuda").contiguous().reshape(-1)
            self._coeffs.append(c)
            kinds = {"helmholtz": SPP_HELMHOLTZ, "schrodinger": SPP_SCHRODINGER, "maxwell": SPP_MAXWELL}
            pbs.append(spp_problem(dim=p["d"], n=p["n"], b=p["b"], kind=kinds[p["kind"]],
                                   omega=p.get("omega", 0.0), ell=p.get("ell", 1.0), energy=p.get("energy", 0.0),
                                   coeff=c.data_ptr()))
        op = spp_options(prec=SPP_C128 if prec == "c128" else SPP_C64_FRONTS,
                         order=SPP_ORDER_OCTREE if order == "octree" else SPP_ORDER_BISECT,
                         tol=tol, max_iter=max_iter,
                         flags=(SPP_F_TIMING if timing else 0) | (SPP_F_GRAPHS if graphs else 0)
                         | (SPP_F_PERSISTENT if persistent else 0), restart=restart)
        self.handle = spp_setup_batch(pbs, op, torch.cuda.current_stream().cuda_stream)

    def _stream(self) -> int:
        return self.torch.cuda.current_stream().cuda_stream

    def pack(self, xs):
        """Per-problem (nrhs, N_i) arrays -> one batch vector [problem][nrhs][N_i]."""
        parts = [self.torch.as_tensor(x, dtype=self.torch.complex128, device="cuda").reshape(-1, N)
                 for x, N in zip(xs, self.sizes)]
        nrhs = parts[0].shape[0]
        return self.torch.cat([p.reshape(-1) for p in parts]).contiguous(), nrhs

    def unpack(self, v, nrhs):
        return [v[nrhs * o0:nrhs * o1].reshape(nrhs, o1 - o0)
                for o0, o1 in zip(self.offsets[:-1], self.offsets[1:])]

    def solve(self, fs):
        fv, nrhs = self.pack(fs)
        u = self.torch.empty_like(fv)
        code, iters, relres = spp_solve(self.handle, fv.data_ptr(), nrhs, u.data_ptr(), self._stream(),
                                        nproblems=len(self.sizes))
        per = lambda a: [a[i * nrhs:(i + 1) * nrhs] for i in range(len(self.sizes))]
        return self.unpack(u, nrhs), per(iters), per(relres), code

    def solve_each(self, fs):
        """spp_solve_batch: fs[i] is an (nrhs_i, N_i) array for problem i, nrhs_i may differ
        (0 allowed, then None); returns per-problem solutions, iterations and residuals."""
        parts, ptrs, outs, optrs, counts = [], [], [], [], []
        for x, N in zip(fs, self.sizes):
            if x is None:
                parts.append(None); outs.append(None); ptrs.append(None); optrs.append(None); counts.append(0)
                continue
            t = self.torch.as_tensor(x, dtype=self.torch.complex128, device="cuda").reshape(-1, N).contiguous()
            o = self.torch.empty_like(t)
            parts.append(t); outs.append(o); ptrs.append(t.data_ptr()); optrs.append(o.data_ptr())
            counts.append(t.shape[0])
        code, iters, relres = spp_solve_batch(self.handle, ptrs, counts, optrs, self._stream())
        it, rr, o = [], [], 0
        for c in counts:
            it.append(iters[o:o + c]); rr.append(relres[o:o + c]); o += c
        return outs, it, rr, code

    def apply(self, name, xs):
        xv, nrhs = self.pack(xs)
        y = self.torch.empty_like(xv)
        {"operator": spp_apply_operator, "green": spp_apply_green, "q": spp_apply_q,
         "precond": spp_apply_precond}[name](self.handle, xv.data_ptr(), y.data_ptr(), nrhs, self._stream())
        return self.unpack(y, nrhs)

    def shift(self, i: int):
        return spp_get_shift(self.handle, i)

    def stats(self) -> dict:
        return spp_stats(self.handle)

    def close(self):
        if getattr(self, "handle", None):
            spp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ----------------------------------------------------------------- learned stage
SPP_CNN_BF16 = 0
SPP_CNN_F32 = 1


class CnnError(RuntimeError):
    def __init__(self, code: int, where: str):
        lib = library()
        super().__init__(f"{where}: {lib.spp_error_string(code).decode()} ({lib.spp_cnn_last_error().decode()})")
        self.code = code


def _cnn_check(code: int, where: str):
    if code != SPP_OK:
        raise CnnError(code, where)


class CNN:
    """The learned preconditioner network on the GPU (weights in (Cout, Cin, 3, 3) per layer)."""

    def __init__(self, n: int, channels=(2, 32, 32, 32, 32, 32, 2), dtype: str = "bf16", max_batch: int = 32):
        import numpy as np
        import torch
        self.torch, self.np = torch, np
        self.n, self.channels, self.max_batch = n, tuple(channels), max_batch
        ch = (ctypes.c_int32 * len(channels))(*channels)
        h = ctypes.c_void_p()
        _cnn_check(library().spp_cnn_create(n, len(channels) - 1, ch, SPP_CNN_BF16 if dtype == "bf16" else SPP_CNN_F32,
                                            max_batch, ctypes.byref(h)), "spp_cnn_create")
        self.handle = h.value
        cnt = ctypes.c_int64()
        _cnn_check(library().spp_cnn_weights(self.handle, None, None, ctypes.byref(cnt)), "spp_cnn_weights")
        self.count = cnt.value
        self.shapes = [(co, ci, 3, 3) for ci, co in zip(channels[:-1], channels[1:])]

    def _stream(self) -> int:
        return self.torch.cuda.current_stream().cuda_stream

    def set_weights(self, ws):
        flat = self.np.concatenate([self.np.asarray(w, dtype=self.np.float32).reshape(-1) for w in ws])
        assert flat.size == self.count
        flat = self.np.ascontiguousarray(flat)
        _cnn_check(library().spp_cnn_weights(self.handle, flat.ctypes.data, None, None), "spp_cnn_weights")

    def _split(self, flat):
        out, o = [], 0
        for s in self.shapes:
            k = int(self.np.prod(s))
            out.append(flat[o:o + k].reshape(s))
            o += k
        return out

    def get_weights(self):
        flat = self.np.zeros(self.count, dtype=self.np.float32)
        _cnn_check(library().spp_cnn_weights(self.handle, None, flat.ctypes.data, None), "spp_cnn_weights")
        return self._split(flat)

    def _dev(self, x):
        t = self.torch.as_tensor(x, dtype=self.torch.complex128, device="cuda").contiguous()
        return t.reshape(-1, self.n * self.n)

    def forward(self, x):
        xv = self._dev(x)
        y = self.torch.empty_like(xv)
        _cnn_check(library().spp_cnn_forward(self.handle, xv.data_ptr(), xv.shape[0], y.data_ptr(),
                                             ctypes.c_void_p(self._stream())), "spp_cnn_forward")
        return y

    def loss_grad(self, x, t, want_grads: bool = False):
        xv, tv = self._dev(x), self._dev(t)
        loss = ctypes.c_double()
        g = self.np.zeros(self.count, dtype=self.np.float32) if want_grads else None
        _cnn_check(library().spp_cnn_loss_grad(self.handle, xv.data_ptr(), tv.data_ptr(), xv.shape[0],
                                               ctypes.byref(loss), g.ctypes.data if want_grads else None,
                                               ctypes.c_void_p(self._stream())), "spp_cnn_loss_grad")
        return (loss.value, self._split(g)) if want_grads else loss.value

    def adam_step(self, lr: float = 1e-3):
        _cnn_check(library().spp_cnn_adam_step(self.handle, ctypes.c_float(lr), ctypes.c_void_p(self._stream())),
                   "spp_cnn_adam_step")

    def close(self):
        if getattr(self, "handle", None):
            library().spp_cnn_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def spp_attach_cnn(handle, cnn_handle, rho: float = 0.9):
    _check(library().spp_attach_cnn(handle, cnn_handle, ctypes.c_double(rho)), "spp_attach_cnn")


def spp_learned_stats(handle):
    a, r = ctypes.c_int32(), ctypes.c_int32()
    _check(library().spp_learned_stats(handle, ctypes.byref(a), ctypes.byref(r)), "spp_learned_stats")
    return a.value, r.value


def spp_get_krylov(handle, j: int, v_ptr, z_ptr):
    _check(library().spp_get_krylov(handle, j, v_ptr, z_ptr), "spp_get_krylov")


def spp_autotune(handle, nrhs: int, stream: int):
    _check(library().spp_autotune(handle, nrhs, ctypes.c_void_p(stream)), "spp_autotune")


def spp_tune_set(key: str, value: int):
    """Set (value >= 0) or remove (value < 0) one entry of the tuning table."""
    _check(library().spp_tune_set(key.encode(), int(value)), "spp_tune_set")


def spp_tune_get(key: str):
    """The tuning table's entry for key, or None if it has none."""
    v = ctypes.c_int32(0)
    code = library().spp_tune_get(key.encode(), ctypes.byref(v))
    return v.value if code == SPP_OK else None
