"""Python binding of libmbl: argument marshalling only.

Every numerical step runs in the HIP kernels of libmbl.so; this module turns
torch tensors into device pointers and streams and checks status codes.
Blocks are row-major (n, b) tensors on a HIP device; FP64 or FP32.
"""

import atexit
import ctypes as C
import os
import weakref

import numpy as np
import torch

from . import _lib
from ._lib import MBL_F32, MBL_F64, MBL_MIXED, MBL_PCG32, MblError  # noqa: F401

PRECISIONS = {"f64": MBL_F64, "mixed": MBL_MIXED, "pcg32": MBL_PCG32}


# -- device memory -------------------------------------------------------------
# The library's device work space is taken from torch's caching allocator
# through mbl_set_allocator, so one pool owns all device memory: what a solve
# frees goes back to torch and is reused by tensors and by later solves.  The
# callbacks receive the library's stream; torch keeps the block stream-ordered
# on it.  MBL_TORCH_ALLOCATOR=0 leaves the library on its own stream-ordered
# pool.
def _torch_alloc(nbytes, stream, ctx):
    try:
        torch.cuda._lazy_init()
        return torch._C._cuda_cudaCachingAllocator_raw_alloc(int(nbytes), int(stream or 0))
    except Exception:
        return None  # the library reports MBL_ENOMEM


def _torch_free(ptr, stream, ctx):
    torch._C._cuda_cudaCachingAllocator_raw_delete(int(ptr))


_allocator = None  # (alloc, free) ctypes callbacks in use
# Every pair ever installed stays alive: buffers are freed by the callback that
# allocated them, which may be long after another pair was installed.
_installed = []
_handles = weakref.WeakSet()  # open Hamiltonians and servers


def use_allocator(alloc=None, free=None):
    """Install device allocation callbacks: alloc(nbytes, stream) -> int
    pointer (0 on failure) and free(ptr, stream); (None, None) restores the
    library's own pool.  Buffers are always released by the allocator that
    made them."""
    global _allocator
    lib = _lib.load()
    if alloc is None:
        _lib.check(lib.mbl_set_allocator(_lib.AllocFn(), _lib.FreeFn(), None))
        _allocator = None
        return
    cb = (_lib.AllocFn(lambda n, s, c: alloc(n, s)), _lib.FreeFn(lambda p, s, c: free(p, s)))
    _installed.append(cb)
    _lib.check(lib.mbl_set_allocator(cb[0], cb[1], None))
    _allocator = cb


def use_torch_allocator():
    """Route the library's device memory through torch's caching allocator."""
    use_allocator(lambda n, s: _torch_alloc(n, s, None), lambda p, s: _torch_free(p, s, None))


def _install_default_allocator():
    if os.environ.get("MBL_TORCH_ALLOCATOR", "1") == "0":
        return
    try:
        use_torch_allocator()
    except ImportError:
        pass  # library not built: the first solver call raises


@atexit.register
def _release_at_exit():
    # close what is still open while the callbacks can still run
    for obj in list(_handles):
        try:
            obj.close()
        except Exception:
            pass
    if _allocator is not None:
        try:
            use_allocator(None)
        except Exception:
            pass


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def _prec(t):
    if t.dtype == torch.float64:
        return MBL_F64
    if t.dtype == torch.float32:
        return MBL_F32
    raise TypeError(f"blocks must be float64 or float32, got {t.dtype}")


def _block(t, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if t.dim() != 2 or t.stride(1) != 1:
        raise ValueError(f"{name} must be a row-major 2-D tensor (unit column stride)")
    return C.c_void_p(t.data_ptr()), t.stride(0)


class Hamiltonian:
    """One S^z sector of the random-field spin chain (paper eq. (1)/(2))."""

    def __init__(self, L, h, Sz=0.0, J=1.0, Delta=1.0, stream=None):
        lib = _lib.load()
        h = np.ascontiguousarray(np.asarray(h, dtype=np.float64))
        if h.shape != (L,):
            raise ValueError("h must have length L")
        self.L, self.Sz, self.J, self.Delta = int(L), float(Sz), float(J), float(Delta)
        self.h = h.copy()
        handle = C.c_void_p()
        _lib.check(lib.mbl_hamiltonian_create(
            self.L, self.Sz, self.J, self.Delta, h.ctypes.data_as(_lib.dptr), _stream(stream),
            C.byref(handle)))
        self._h = handle
        n = C.c_int64()
        _lib.check(lib.mbl_hamiltonian_dim(self._h, C.byref(n)))
        self.n = n.value
        _handles.add(self)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.load().mbl_hamiltonian_destroy(self._h)
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

    # -- sector --------------------------------------------------------------
    def states(self):
        out = np.empty(self.n, dtype=np.uint64)
        _lib.check(_lib.load().mbl_sector_states(self._h, out.ctypes.data_as(_lib.u64p)))
        return out

    def rank(self, states):
        q = np.ascontiguousarray(np.asarray(states, dtype=np.uint64))
        out = np.empty(q.shape, dtype=np.int64)
        _lib.check(_lib.load().mbl_rank(self._h, q.ctypes.data_as(_lib.u64p), q.size,
                                        out.ctypes.data_as(_lib.i64p)))
        return out

    def diagonal(self, sigma=0.0, device="cuda", stream=None):
        d = torch.empty(self.n, dtype=torch.float64, device=device)
        j = torch.empty(self.n, dtype=torch.float64, device=device)
        _lib.check(_lib.load().mbl_diagonal(self._h, float(sigma), C.c_void_p(d.data_ptr()),
                                            C.c_void_p(j.data_ptr()), _stream(stream)))
        return d, j

    # -- operators -----------------------------------------------------------
    def apply(self, X, sigma=0.0, out=None, stream=None):
        """(H - sigma I) X."""
        px, ldx = _block(X, "X")
        Y = torch.empty_like(X, memory_format=torch.contiguous_format) if out is None else out
        py, ldy = _block(Y, "Y")
        _lib.check(_lib.load().mbl_apply_block(self._h, float(sigma), _prec(X), px, ldx, py, ldy,
                                               X.shape[1], _stream(stream)))
        return Y

    def fold_apply(self, X, sigma=0.0, stream=None):
        """(H - sigma I)^2 X (returns Y, and the intermediate (H - sigma I) X)."""
        px, ldx = _block(X, "X")
        T = torch.empty_like(X, memory_format=torch.contiguous_format)
        Y = torch.empty_like(X, memory_format=torch.contiguous_format)
        pt, ldt = _block(T, "T")
        py, ldy = _block(Y, "Y")
        _lib.check(_lib.load().mbl_fold_apply(self._h, float(sigma), _prec(X), px, ldx, pt, ldt,
                                              py, ldy, X.shape[1], _stream(stream)))
        return Y, T

    def pcg(self, R, sigma, m, stream=None):
        """m Jacobi-PCG steps on (H - sigma)^2 W = R, per column, from W = 0."""
        pr, ldr = _block(R, "R")
        W = torch.empty_like(R, memory_format=torch.contiguous_format)
        pw, ldw = _block(W, "W")
        _lib.check(_lib.load().mbl_pcg(self._h, float(sigma), _prec(R), pr, ldr, pw, ldw,
                                       R.shape[1], int(m), _stream(stream)))
        return W

    def spectrum_bounds(self, tol=1e-12, stream=None):
        lo, hi = C.c_double(), C.c_double()
        _lib.check(_lib.load().mbl_spectrum_bounds(self._h, float(tol), C.byref(lo), C.byref(hi),
                                                   _stream(stream)))
        return lo.value, hi.value

    def entanglement_entropy(self, V, cut=None, stream=None):
        """Entanglement entropy of each column of V (n x nev FP64) across the
        cut after `cut` sites (default: half chain)."""
        cut = self.L // 2 if cut is None else int(cut)
        pv, ldv = _block(V, "V")
        if V.dtype != torch.float64:
            raise TypeError("V must be float64")
        S = np.zeros(V.shape[1])
        _lib.check(_lib.load().mbl_entanglement_entropy(self._h, pv, ldv, V.shape[1], cut,
                                                        S.ctypes.data_as(_lib.dptr),
                                                        _stream(stream)))
        return S

    def solve_slices(self, sigmas, nev, block, tol=1e-10, precision="f64", concurrency=4,
                     max_iter=400, pcg_iters=0, seed=0x5EED, lock=False):
        """Eigenvalue chunks: the nev pairs nearest each shift (values and residuals)."""
        lib = _lib.load()
        sig = np.ascontiguousarray(np.asarray(sigmas, dtype=np.float64))
        opts = _lib.SolveOpts()
        _lib.check(lib.mbl_solve_opts_default(C.byref(opts)))
        opts.max_iter, opts.pcg_iters, opts.seed = int(max_iter), int(pcg_iters), int(seed)
        opts.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        opts.lock = int(bool(lock))
        ev = np.zeros((len(sig), nev))
        rs = np.zeros((len(sig), nev))
        _lib.check(lib.mbl_slices_solve(self._h, len(sig), sig.ctypes.data_as(_lib.dptr), int(nev),
                                        int(block), float(tol), C.byref(opts),
                                        ev.ctypes.data_as(_lib.dptr),
                                        rs.ctypes.data_as(_lib.dptr), int(concurrency)))
        return ev, rs

    def solve(self, sigma, nev, block, tol=1e-10, precision="f64", max_iter=400, pcg_iters=0,
              seed=0x5EED, verbose=False, want_vectors=True, device="cuda", stream=None,
              raise_on_noconv=True, timing=False, lock=False, max_seconds=0.0, cancel=None,
              guard_cg=0.0):
        """nev eigenpairs nearest sigma by LOBPCG on the spectral fold.

        lock=True turns on soft locking of converged wanted pairs (the inner
        CG then runs on fewer columns; see mbl_solve_opts.lock).  max_seconds
        > 0 limits the wall time and `cancel` (a ctypes.c_int another thread
        may set nonzero) stops the solve; both return the best pairs so far
        with status MBL_ECANCELLED (raised unless raise_on_noconv is False).
        guard_cg in (0, 1] gives the block columns beyond nev that share of the
        CG steps (0: the library's default by sector size and nev; see
        mbl_solve_opts.guard_cg).  timing=True fills the info dict with event
        times of the CG kernels and of the apply, Gram and small dense phases.

        Returns (evals [nev] numpy, evecs (n, nev) float64 tensor or None,
        resid [nev] numpy, info dict).
        """
        lib = _lib.load()
        opts = _lib.SolveOpts()
        _lib.check(lib.mbl_solve_opts_default(C.byref(opts)))
        opts.max_iter = int(max_iter)
        opts.pcg_iters = int(pcg_iters)
        opts.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        opts.verbose = int(verbose)
        opts.timing = int(bool(timing))
        opts.seed = int(seed)
        opts.lock = int(bool(lock))
        opts.max_seconds = float(max_seconds)
        opts.guard_cg = float(guard_cg)
        if cancel is not None:
            opts.cancel = C.pointer(cancel)
        ev = np.zeros(nev)
        rs = np.zeros(nev)
        info = _lib.SolveInfo()
        V = torch.empty((self.n, nev), dtype=torch.float64, device=device) if want_vectors else None
        st = lib.mbl_lobpcg_solve(
            self._h, float(sigma), int(nev), int(block), float(tol), C.byref(opts),
            ev.ctypes.data_as(_lib.dptr), C.c_void_p(V.data_ptr()) if V is not None else None,
            nev, rs.ctypes.data_as(_lib.dptr), C.byref(info), _stream(stream))
        _lib.check(st, allow=() if raise_on_noconv else (_lib.MBL_ENOCONV, _lib.MBL_ECANCELLED))
        d = {}
        for f, _ in _lib.SolveInfo._fields_:
            v = getattr(info, f)
            d[f] = list(v) if hasattr(v, "__len__") else v
        d["status"] = _lib.STATUS_NAMES.get(st, st)
        return ev, V, rs, d


def gram(A, B, stream=None):
    """A^T B in FP64 (matrix-core kernel, fixed-order reduction)."""
    pa, lda = _block(A, "A")
    pb, ldb = _block(B, "B")
    if A.dtype != B.dtype or A.shape[0] != B.shape[0]:
        raise ValueError("A and B must share dtype and row count")
    Cm = torch.empty((A.shape[1], B.shape[1]), dtype=torch.float64, device=A.device)
    _lib.check(_lib.load().mbl_gram(_prec(A), A.shape[0], pa, lda, A.shape[1], pb, ldb,
                                    B.shape[1], C.c_void_p(Cm.data_ptr()), B.shape[1],
                                    _stream(stream)))
    return Cm


def gram_noalloc(A, B, out, stream=None):
    """A^T B into the caller's FP64 (p, q) device matrix `out`, with no device
    allocation: the library's fixed per-GPU scratch holds the partial sums
    (same kernels and bits as gram()).  Calls that overlap on one GPU race."""
    pa, lda = _block(A, "A")
    pb, ldb = _block(B, "B")
    if A.dtype != B.dtype or A.shape[0] != B.shape[0]:
        raise ValueError("A and B must share dtype and row count")
    if (out.dtype != torch.float64 or out.device != A.device or out.dim() != 2
            or tuple(out.shape) != (A.shape[1], B.shape[1]) or out.stride(1) != 1):
        raise ValueError("out must be an FP64 (p, q) row-major device matrix beside A")
    _lib.check(_lib.load().mbl_gram_noalloc(_prec(A), A.shape[0], pa, lda, A.shape[1], pb, ldb,
                                            B.shape[1], C.c_void_p(out.data_ptr()),
                                            out.stride(0), _stream(stream)))
    return out


def block_combine(A, Cm, stream=None):
    """A @ Cm with Cm an FP64 (p, q) device matrix; result in A's dtype."""
    pa, lda = _block(A, "A")
    Cm = Cm.contiguous()
    if Cm.dtype != torch.float64 or Cm.shape[0] != A.shape[1]:
        raise ValueError("C must be float64 with p rows")
    Y = torch.empty((A.shape[0], Cm.shape[1]), dtype=A.dtype, device=A.device)
    py, ldy = _block(Y, "Y")
    _lib.check(_lib.load().mbl_block_combine(_prec(A), A.shape[0], pa, lda, A.shape[1],
                                             C.c_void_p(Cm.data_ptr()), Cm.shape[1], py, ldy,
                                             Cm.shape[1], _stream(stream)))
    return Y


def small_eigh(A, stream=None):
    """Symmetric eigendecomposition of a small FP64 device matrix (Jacobi)."""
    A = A.contiguous()
    m = A.shape[0]
    w = torch.empty(m, dtype=torch.float64, device=A.device)
    V = torch.empty((m, m), dtype=torch.float64, device=A.device)
    _lib.check(_lib.load().mbl_small_eigh(m, C.c_void_p(A.data_ptr()), m, C.c_void_p(w.data_ptr()),
                                          C.c_void_p(V.data_ptr()), m, _stream(stream)))
    return w, V


# -- many independent solves -------------------------------------------------

def _problem(d):
    """ctypes Problem from a dict (keeps the h array alive in the dict)."""
    h = np.ascontiguousarray(np.asarray(d["h"], dtype=np.float64))
    d["_h_keep"] = h
    prec = d.get("precision", "f64")
    pr = _lib.Problem()
    pr.L = int(d["L"])
    pr.Sz = float(d.get("Sz", 0.0))
    pr.J = float(d.get("J", 1.0))
    pr.Delta = float(d.get("Delta", 1.0))
    pr.h_host = h.ctypes.data_as(_lib.dptr)
    pr.sigma = float(d.get("sigma", 0.0))
    pr.eps = float(d.get("eps", -1.0))
    pr.nev = int(d["nev"])
    pr.block = int(d["block"])
    pr.tol = float(d.get("tol", 1e-10))
    pr.precision = PRECISIONS[prec] if isinstance(prec, str) else int(prec)
    pr.max_iter = int(d.get("max_iter", 400))
    pr.pcg_iters = int(d.get("pcg_iters", 0))
    pr.seed = int(d.get("seed", 0x5EED))
    pr.want_vectors = int(bool(d.get("want_vectors", False)))
    return pr


def _result_dict(r, ev, rs):
    return {"status": _lib.STATUS_NAMES.get(r.status, r.status), "sigma": r.sigma,
            "nconv": r.nconv, "iters": r.iters, "applies": r.applies,
            "max_resid": r.max_resid, "seconds": r.seconds, "latency": r.latency,
            "evals": ev, "resid": rs}


def gap_ratio(evals):
    """Mean adjacent gap ratio of a set of eigenvalues (library host routine)."""
    e = np.ascontiguousarray(np.asarray(evals, dtype=np.float64))
    out = C.c_double()
    _lib.check(_lib.load().mbl_gap_ratio(e.ctypes.data_as(_lib.dptr), len(e), C.byref(out)))
    return out.value


def footprint_bytes(L, block, precision="f64", Sz=0.0):
    """Device bytes one solve holds at its peak (the server's admission model)."""
    out = C.c_size_t()
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    _lib.check(_lib.load().mbl_footprint_bytes(int(L), float(Sz), int(block), prec, C.byref(out)))
    return out.value


def batch_solve(problems, concurrency=4, vectors=False, device="cuda"):
    """Solve a list of problem dicts (keys: L, h, nev, block, and optionally
    Sz, J, Delta, sigma or eps, tol, precision, max_iter, pcg_iters, seed),
    `concurrency` at a time.  Returns a list of result dicts (with 'evecs'
    tensors when vectors=True)."""
    lib = _lib.load()
    k = len(problems)
    P = (_lib.Problem * k)(*[_problem(d) for d in problems])
    R = (_lib.Result * k)()
    keep = []
    for i, d in enumerate(problems):
        ev = np.zeros(int(d["nev"]))
        rs = np.zeros(int(d["nev"]))
        keep.append((ev, rs))
        R[i].evals_host = ev.ctypes.data_as(_lib.dptr)
        R[i].resid_host = rs.ctypes.data_as(_lib.dptr)
        if vectors:
            from math import comb
            n = comb(int(d["L"]), int(round(float(d.get("Sz", 0.0)) + d["L"] / 2)))
            V = torch.empty((n, int(d["nev"])), dtype=torch.float64, device=device)
            keep[-1] = (ev, rs, V)
            R[i].evecs_dev = C.c_void_p(V.data_ptr())
            R[i].ldv = int(d["nev"])
    lib.mbl_batch_solve(k, P, R, int(concurrency))
    out = []
    for i in range(k):
        dd = _result_dict(R[i], keep[i][0], keep[i][1])
        if vectors:
            dd["evecs"] = keep[i][2]
        out.append(dd)
    return out


class Server:
    """Serving loop with continuous batching and HBM-footprint admission."""

    def __init__(self, max_slots=4, hbm_budget=0, device=None):
        self._lib = _lib.load()
        dev = torch.cuda.current_device() if device is None else int(device)
        h = C.c_void_p()
        _lib.check(self._lib.mbl_server_create(dev, int(hbm_budget), int(max_slots), C.byref(h)))
        self._s = h
        self._keep = {}
        _handles.add(self)

    def submit(self, problem):
        pr = _problem(dict(problem))
        t = C.c_uint64()
        _lib.check(self._lib.mbl_server_submit(self._s, C.byref(pr), C.byref(t)))
        self._keep[t.value] = problem
        return t.value

    def wait(self, ticket, timeout=-1.0, vectors_out=None):
        d = self._keep[ticket]
        ev = np.zeros(int(d["nev"]))
        rs = np.zeros(int(d["nev"]))
        r = _lib.Result()
        r.evals_host = ev.ctypes.data_as(_lib.dptr)
        r.resid_host = rs.ctypes.data_as(_lib.dptr)
        if vectors_out is not None:
            r.evecs_dev = C.c_void_p(vectors_out.data_ptr())
            r.ldv = vectors_out.stride(0)
        st = self._lib.mbl_server_wait(self._s, int(ticket), float(timeout), C.byref(r))
        if st == _lib.MBL_ETIMEOUT:
            return None
        _lib.check(st)
        del self._keep[ticket]
        return _result_dict(r, ev, rs)

    def cancel(self, ticket):
        """Cancel a request that has not finished (its result, still to be
        waited for, then has status MBL_ECANCELLED)."""
        _lib.check(self._lib.mbl_server_cancel(self._s, int(ticket)))

    def stats(self):
        st = _lib.ServerStats()
        _lib.check(self._lib.mbl_server_stats_get(self._s, C.byref(st)))
        return {f: getattr(st, f) for f, _ in _lib.ServerStats._fields_}

    def close(self):
        if getattr(self, "_s", None) is not None and self._s.value:
            self._lib.mbl_server_destroy(self._s)
            self._s = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_install_default_allocator()
