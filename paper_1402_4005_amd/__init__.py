"""Python binding of the BAMG HIP library (``libbamg.so``, C ABI in
``include/bamg.h``): bootstrap-AMG preconditioned GMRES for the stationary
vector of an irreducible Markov chain on an MI355X.

This module only marshals arguments: torch tensors provide device memory and
the HIP stream; every step of the method runs in the library's kernels. It
fails loudly when the library is not built or no GPU is present; there is no
CPU fallback.
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import weakref

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbamg.so")

OK = 0
NOT_CONVERGED = 1
COARSEN_GEOMETRIC, COARSEN_MIS, COARSEN_CR = 0, 1, 2
SMOOTH_JACOBI, SMOOTH_KACZMARZ = 0, 1
PRECISION_FP64, PRECISION_MIXED = 0, 1
DTYPE_F64, DTYPE_F32 = 0, 1
GEOM_NONE, GEOM_LINE, GEOM_GRID2D = 0, 1, 2
LEARNED_OFF, LEARNED_USE, LEARNED_RECORD = 0, 1, 2
CYCLE_V, CYCLE_W, CYCLE_F, CYCLE_NONE = 0, 1, 2, 3
MLP_IN, MLP_HIDDEN, MLP_OUT, MLP_NPARAMS = 96, 64, 8, 10888
WHAT = {"B": 0, "Bt": 1, "M": 2, "N": 3, "P": 4, "Q": 5, "Qt": 6}


class BamgError(RuntimeError):
    def __init__(self, code, msg=""):
        super().__init__(f"bamg status {code}: {status_string(code)} {msg}".strip())
        self.code = code


class Csr(C.Structure):
    _fields_ = [("n", C.c_int64), ("nnz", C.c_int64), ("row_ptr", C.c_void_p),
                ("col_idx", C.c_void_p), ("val", C.c_void_p), ("on_device", C.c_int32)]


class Geometry(C.Structure):
    _fields_ = [("kind", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32)]


class HostCsr(C.Structure):
    _fields_ = [("nrows", C.c_int64), ("ncols", C.c_int64), ("nnz", C.c_int64),
                ("row_ptr", C.c_void_p), ("col_idx", C.c_void_p), ("val", C.c_void_p)]


class LevelOps(C.Structure):
    _fields_ = [("B", HostCsr), ("P", HostCsr), ("Q", HostCsr)]


class Options(C.Structure):
    _fields_ = [("r", C.c_int32), ("setup_cycles", C.c_int32), ("nu_pre", C.c_int32),
                ("nu_post", C.c_int32), ("nu_setup", C.c_int32), ("omega", C.c_double),
                ("max_interp", C.c_int32), ("max_levels", C.c_int32), ("coarse_max", C.c_int32),
                ("coarsening", C.c_int32), ("seed", C.c_uint64), ("smoother", C.c_int32),
                ("precision", C.c_int32), ("interp_rule", C.c_int32), ("validate", C.c_int32),
                ("use_graph", C.c_int32), ("learned", C.c_int32), ("mlp", C.c_void_p),
                ("autotune", C.c_int32), ("fuse_last_level", C.c_int32),
                ("cycle", C.c_int32), ("mu", C.c_int32), ("restriction", C.c_int32),
                ("profile_setup", C.c_int32), ("learned_max_iters", C.c_int32),
                ("cr_theta", C.c_double), ("cr_beta", C.c_double), ("cr_sweeps", C.c_int32),
                ("cr_rounds", C.c_int32), ("flexible", C.c_int32)]


class SolveInfo(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("restarts", C.c_int32), ("converged", C.c_int32),
                ("breakdowns", C.c_int32), ("rel_residual", C.c_double), ("x_min", C.c_double),
                ("t_solve_ms", C.c_double), ("setup_cycles", C.c_int32),
                ("mlp_fallback", C.c_int32), ("t_setup_ms", C.c_double),
                ("mlp_rows", C.c_int64), ("ls_fallbacks", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib():
    """Load libbamg.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        # torch's HIP runtime must be the one the library binds to (same
        # SONAME): load it first so there is a single runtime in the process
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run paper_1402_4005_amd/build.py "
                               "(or __graft_entry__.build()) first")
        L = C.CDLL(LIB_PATH)
        P, V = C.POINTER, C.c_void_p
        L.bamg_default_options.argtypes = [P(Options)]
        L.bamg_setup.argtypes = [P(Csr), P(Geometry), P(Options), V, V, P(V)]
        L.bamg_vcycle.argtypes = [V, V, V, C.c_int32, V]
        L.bamg_setup_from_levels.argtypes = [C.c_int32, V, V, V, P(Options), V, V, P(V)]
        L.bamg_gmres_solve.argtypes = [V, V, C.c_int32, C.c_double, C.c_int32, C.c_int32,
                                       P(SolveInfo), V]
        L.bamg_hierarchy_info.argtypes = [V, V, V, V, V, V]
        L.bamg_set_cycle.argtypes = [V, C.c_int32]
        L.bamg_level_nnz.argtypes = [V, C.c_int32, C.c_int32, V, V]
        L.bamg_level_csr.argtypes = [V, C.c_int32, C.c_int32, V, V, V]
        L.bamg_level_cf.argtypes = [V, C.c_int32, V, V]
        L.bamg_level_vectors.argtypes = [V, C.c_int32, V, V]
        L.bamg_sigma.argtypes = [V, V]
        L.bamg_x0.argtypes = [V, V, V]
        L.bamg_coarse_pinv.argtypes = [V, V]
        L.bamg_vcycle_bytes.argtypes = [V, V]
        L.bamg_level_lanes.argtypes = [V, C.c_int32, P(C.c_int32)]
        L.bamg_level_set_lanes.argtypes = [V, C.c_int32, C.c_int32]
        L.bamg_level_threads.argtypes = [V, C.c_int32, P(C.c_int32)]
        L.bamg_level_set_threads.argtypes = [V, C.c_int32, C.c_int32]
        L.bamg_kernel_profile_begin.argtypes = [V, C.c_int32]
        L.bamg_kernel_profile_end.argtypes = [V, V, V, V]
        L.bamg_destroy.argtypes = [V]
        L.bamg_destroy.restype = None
        L.bamg_status_string.argtypes = [C.c_int32]
        L.bamg_status_string.restype = C.c_char_p
        L.bamg_last_error.argtypes = []
        L.bamg_last_error.restype = C.c_char_p
        L.bamg_mlp_create.argtypes = [V, P(V)]
        L.bamg_mlp_get_params.argtypes = [V, V]
        L.bamg_mlp_destroy.argtypes = [V]
        L.bamg_mlp_destroy.restype = None
        L.bamg_mlp_forward.argtypes = [V, V, C.c_int64, V, C.c_int32, V]
        L.bamg_mlp_loss_grad.argtypes = [V, V, V, V, C.c_int64, P(C.c_double), V, V]
        L.bamg_mlp_train.argtypes = [V, V, V, V, C.c_int64, C.c_int32, C.c_int32, C.c_float,
                                     V, V]
        L.bamg_harvest.argtypes = [V, C.c_int32, V, V, V, P(C.c_int64), V]
        L.bamg_setup_batched.argtypes = [C.c_int32, V, V, V, V, C.c_int32, V, P(V)]
        L.bamg_batch_status.argtypes = [V, C.c_int32, P(C.c_int32), P(V)]
        L.bamg_gmres_solve_batched.argtypes = [V, V, C.c_int32, C.c_double, C.c_int32, V, V, V]
        L.bamg_batch_set_solver.argtypes = [V, C.c_int32]
        L.bamg_batch_destroy.argtypes = [V]
        L.bamg_batch_destroy.restype = None
        L.bamg_learned_stats.argtypes = [V, P(C.c_int64), P(C.c_int64)]
        _lib = L
    return _lib


def status_string(code) -> str:
    try:
        return lib().bamg_status_string(code).decode()
    except Exception:
        return "?"


def _check(code):
    if code < 0:
        raise BamgError(code, lib().bamg_last_error().decode())
    return code


def default_options(**kw) -> Options:
    o = Options()
    _check(lib().bamg_default_options(C.byref(o)))
    names = {
        "coarsening": {"geom": COARSEN_GEOMETRIC, "geometric": COARSEN_GEOMETRIC, "mis": COARSEN_MIS,
                       "cr": COARSEN_CR},
        "smoother": {"jacobi": SMOOTH_JACOBI, "kaczmarz": SMOOTH_KACZMARZ},
        "precision": {"fp64": PRECISION_FP64, "mixed": PRECISION_MIXED},
        "learned": {"off": LEARNED_OFF, "use": LEARNED_USE, "record": LEARNED_RECORD},
        "cycle": {"V": CYCLE_V, "W": CYCLE_W, "F": CYCLE_F, "none": CYCLE_NONE},
        "restriction": {"ls": 0, "average": 1},
    }
    for k, v in kw.items():
        if k in names and isinstance(v, str):
            v = names[k][v]
        if k == "mlp" and isinstance(v, MLP):
            v = v.h.value
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("no GPU visible: the BAMG library runs only on the device")
    return torch


def _stream(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


_ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p)
_FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)


class Allocator(C.Structure):
    _fields_ = [("ctx", C.c_void_p), ("alloc", _ALLOC_FN), ("free", _FREE_FN)]


def _torch_alloc(ctx, nbytes, stream):
    try:
        return _torch()._C._cuda_cudaCachingAllocator_raw_alloc(nbytes, stream or 0)
    except RuntimeError:
        return None  # the library reports BAMG_E_NOMEM


def _torch_free(ctx, ptr, stream):
    _torch()._C._cuda_cudaCachingAllocator_raw_delete(ptr)


_TORCH_ALLOCATOR = Allocator(None, _ALLOC_FN(_torch_alloc), _FREE_FN(_torch_free))
_LIVE = weakref.WeakSet()  # hierarchies whose memory may come from torch


@atexit.register
def _close_live():
    # before torch's own teardown: a handle freed later would call into it
    for h in list(_LIVE):
        h.close()


def _allocator(kind):
    """bamg_allocator for `kind`: "torch" = torch's caching allocator (blocks
    are stream-ordered on the handle's stream and reused by later handles
    without a device synchronisation), "hip" = the library's own
    hipMalloc / hipFree."""
    if kind == "torch":
        return C.byref(_TORCH_ALLOCATOR)
    if kind == "hip":
        return None
    raise ValueError(f"allocator {kind!r}: 'torch' or 'hip'")


class Hierarchy:
    """A BAMG hierarchy set up on the GPU (wraps ``bamg_handle``).

    ``A`` is the column-stochastic transition matrix in CSR by destination
    state: ``indptr``/``indices``/``data`` as numpy arrays (host) or torch
    CUDA tensors (device; int32, int32, float64).
    """

    def __init__(self, indptr, indices, data, geom=(0, 0, 0), opts: Options | None = None,
                 stream=None, allocator="torch"):
        torch = _torch()
        self.opts = opts if opts is not None else default_options()
        on_dev = isinstance(indptr, torch.Tensor)
        if on_dev:
            self._keep = (indptr.contiguous().to(torch.int32), indices.contiguous().to(torch.int32),
                          data.contiguous().to(torch.float64))
            ptrs = [t.data_ptr() for t in self._keep]
            n = self._keep[0].numel() - 1
            nnz = self._keep[1].numel()
        else:
            self._keep = (np.ascontiguousarray(indptr, np.int32),
                          np.ascontiguousarray(indices, np.int32),
                          np.ascontiguousarray(data, np.float64))
            ptrs = [a.ctypes.data for a in self._keep]
            n = len(self._keep[0]) - 1
            nnz = len(self._keep[1])
        self.n = n
        A = Csr(n, nnz, ptrs[0], ptrs[1], ptrs[2], 1 if on_dev else 0)
        g = Geometry(*geom)
        h = C.c_void_p()
        self._stream = _stream(stream)
        _check(lib().bamg_setup(C.byref(A), C.byref(g), C.byref(self.opts),
                                _allocator(allocator), self._stream, C.byref(h)))
        self.h = h
        _LIVE.add(self)
        self.mixed = self.opts.precision == PRECISION_MIXED

    @classmethod
    def from_chain(cls, chain, opts: Options | None = None, on_device=False, stream=None,
                   allocator="torch"):
        if on_device:
            torch = _torch()
            return cls(torch.from_numpy(chain.indptr).cuda(), torch.from_numpy(chain.indices).cuda(),
                       torch.from_numpy(chain.data).cuda(), chain.geom, opts, stream, allocator)
        return cls(chain.indptr, chain.indices, chain.data, chain.geom, opts, stream, allocator)

    @classmethod
    def from_levels(cls, B, P, Q, coarse_pinv, x0, opts: Options | None = None, stream=None,
                    allocator="torch"):
        """A handle on an explicitly given hierarchy (bamg_setup_from_levels):
        B a list of the level operators B_l, P and Q lists of the transfers
        (one fewer), all scipy sparse (converted to sorted CSR); coarse_pinv
        the dense pseudo-inverse of the last B; x0 the initial iterate."""
        import scipy.sparse as sp
        _torch()
        self = cls.__new__(cls)
        self.opts = opts if opts is not None else default_options()
        nl = len(B)
        if len(P) != nl - 1 or len(Q) != nl - 1:
            raise ValueError("P and Q need one entry per level above the coarsest")
        keep = []

        def host(A):
            A = sp.csr_matrix(A)
            A.sort_indices()
            arrs = (np.ascontiguousarray(A.indptr, np.int32),
                    np.ascontiguousarray(A.indices, np.int32),
                    np.ascontiguousarray(A.data, np.float64))
            keep.extend(arrs)
            return HostCsr(A.shape[0], A.shape[1], A.nnz, *[a.ctypes.data for a in arrs])

        ops = (LevelOps * nl)()
        for l in range(nl):
            ops[l].B = host(B[l])
            if l + 1 < nl:
                ops[l].P = host(P[l])
                ops[l].Q = host(Q[l])
        pinv = np.ascontiguousarray(coarse_pinv, np.float64)
        x0a = np.ascontiguousarray(x0, np.float64)
        self.n = B[0].shape[0]
        self._keep = ()
        h = C.c_void_p()
        self._stream = _stream(stream)
        _check(lib().bamg_setup_from_levels(nl, ops, pinv.ctypes.data, x0a.ctypes.data,
                                            C.byref(self.opts), _allocator(allocator),
                                            self._stream, C.byref(h)))
        self.h = h
        _LIVE.add(self)
        self.mixed = self.opts.precision == PRECISION_MIXED
        return self

    def close(self):
        if getattr(self, "h", None):
            lib().bamg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------------- solve
    def vcycle(self, b, x=None, stream=None):
        """x = C b (one V-cycle from zero); b a CUDA tensor of length n."""
        torch = _torch()
        dt = DTYPE_F32 if b.dtype == torch.float32 else DTYPE_F64
        b = b.contiguous()
        if x is None:
            x = torch.empty_like(b)
        _check(lib().bamg_vcycle(self.h, C.c_void_p(b.data_ptr()), C.c_void_p(x.data_ptr()), dt,
                                 _stream(stream)))
        return x

    def gmres(self, x=None, restart=20, tol=1e-10, maxit=500, stream=None):
        """GMRES(restart) on the preconditioned residual equation; returns
        (x scaled to sum 1, SolveInfo). x: optional CUDA float64 initial iterate."""
        torch = _torch()
        use_x0 = x is not None
        if x is None:
            x = torch.empty(self.n, dtype=torch.float64, device="cuda")
        info = SolveInfo()
        st = lib().bamg_gmres_solve(self.h, C.c_void_p(x.data_ptr()), restart, tol, maxit,
                                    1 if use_x0 else 0, C.byref(info), _stream(stream))
        _check(st)
        return x, info

    # ------------------------------------------------------------ inspection
    def info(self):
        lv = C.c_int32()
        nl = np.zeros(32, np.int64)
        nz = np.zeros(32, np.int64)
        oc, og = C.c_double(), C.c_double()
        _check(lib().bamg_hierarchy_info(self.h, C.byref(lv), nl.ctypes.data, nz.ctypes.data,
                                         C.byref(oc), C.byref(og)))
        L = lv.value
        return {"levels": L, "n": nl[:L].tolist(), "nnz": nz[:L].tolist(), "oc": oc.value,
                "og": og.value}

    @property
    def levels(self):
        return self.info()["levels"]

    def csr(self, l, what):
        code = WHAT[what]
        rows, nnz = C.c_int64(), C.c_int64()
        _check(lib().bamg_level_nnz(self.h, l, code, C.byref(rows), C.byref(nnz)))
        rp = np.zeros(rows.value + 1, np.int32)
        ci = np.zeros(nnz.value, np.int32)
        v = np.zeros(nnz.value, np.float64)
        _check(lib().bamg_level_csr(self.h, l, code, rp.ctypes.data, ci.ctypes.data, v.ctypes.data))
        return rp, ci, v

    def scipy(self, l, what):
        import scipy.sparse as sp
        rp, ci, v = self.csr(l, what)
        info = self.info()
        n = info["n"][l]
        nc = info["n"][l + 1] if l + 1 < info["levels"] else n
        shape = {"P": (n, nc), "Qt": (n, nc), "Q": (nc, n)}.get(what, (n, n))
        return sp.csr_matrix((v, ci, rp), shape=shape)

    def cf(self, l):
        n = self.info()["n"][l]
        cf = np.zeros(n, np.int32)
        cidx = np.zeros(n, np.int32)
        _check(lib().bamg_level_cf(self.h, l, cf.ctypes.data, cidx.ctypes.data))
        return cf, cidx

    def vectors(self, l):
        n = self.info()["n"][l]
        r = self.opts.r
        U = np.zeros((n, r))
        V = np.zeros((n, r))
        _check(lib().bamg_level_vectors(self.h, l, U.ctypes.data, V.ctypes.data))
        return U, V

    def sigma(self):
        s = np.zeros(self.opts.r)
        _check(lib().bamg_sigma(self.h, s.ctypes.data))
        return s

    def x0(self):
        torch = _torch()
        x = torch.empty(self.n, dtype=torch.float64, device="cuda")
        _check(lib().bamg_x0(self.h, C.c_void_p(x.data_ptr()), _stream(None)))
        return x

    def vcycle_bytes(self) -> float:
        b = C.c_double()
        _check(lib().bamg_vcycle_bytes(self.h, C.byref(b)))
        return b.value

    def lanes(self, l):
        """Lanes per CSR row used by level l's sweeps."""
        v = C.c_int32()
        _check(lib().bamg_level_lanes(self.h, l, C.byref(v)))
        return v.value

    def set_cycle(self, cycle):
        """Preconditioner shape: 'V', 'W', 'F' or 'none' (C = I)."""
        code = {"V": CYCLE_V, "W": CYCLE_W, "F": CYCLE_F, "none": CYCLE_NONE}.get(cycle, cycle)
        _check(lib().bamg_set_cycle(self.h, code))

    def set_lanes(self, l, lanes):
        """Pin the lanes per row (1, 2, 4) of level l's sweeps and residual."""
        _check(lib().bamg_level_set_lanes(self.h, l, lanes))

    def threads(self, l):
        """Workgroup size of level l's sweeps and residual."""
        v = C.c_int32()
        _check(lib().bamg_level_threads(self.h, l, C.byref(v)))
        return v.value

    def set_threads(self, l, threads):
        """Pin the workgroup size (64 ... 1024) of level l's sweeps and residual."""
        _check(lib().bamg_level_set_threads(self.h, l, threads))

    def profile_begin(self, kernel=0):
        _check(lib().bamg_kernel_profile_begin(self.h, kernel))

    def profile_end(self):
        n, ms, by = C.c_int64(), C.c_double(), C.c_double()
        _check(lib().bamg_kernel_profile_end(self.h, C.byref(n), C.byref(ms), C.byref(by)))
        return n.value, ms.value, by.value

    def harvest(self, level):
        """Cycle-1 features and final P rows of level `level`'s F points
        (handle set up with learned="record"): CUDA float32 tensors
        X (nF x 96), T (nF x 8), M (nF x 8)."""
        torch = _torch()
        nf = C.c_int64()
        _check(lib().bamg_harvest(self.h, level, None, None, None, C.byref(nf), None))
        n = nf.value
        X = torch.empty((n, MLP_IN), dtype=torch.float32, device="cuda")
        T = torch.empty((n, MLP_OUT), dtype=torch.float32, device="cuda")
        M = torch.empty((n, MLP_OUT), dtype=torch.float32, device="cuda")
        if n:
            _check(lib().bamg_harvest(self.h, level, C.c_void_p(X.data_ptr()),
                                      C.c_void_p(T.data_ptr()), C.c_void_p(M.data_ptr()),
                                      C.byref(nf), _stream(None)))
        return X, T, M

    def learned_stats(self):
        """(rows taken from the MLP, rows that fell back to the exact LS fit)."""
        a, b = C.c_int64(), C.c_int64()
        _check(lib().bamg_learned_stats(self.h, C.byref(a), C.byref(b)))
        return a.value, b.value

    def coarse_pinv(self):
        info = self.info()
        nL = info["n"][-1]
        B = np.zeros((nL, nL))
        _check(lib().bamg_coarse_pinv(self.h, B.ctypes.data))
        return B


class Batch:
    """Many chains set up and solved together (bamg_setup_batched): chains
    is a list of chaingen.Chain, opts a list of Options (one per chain)."""

    @staticmethod
    def upload(chains):
        """Device copies (row_ptr, col_idx, val) of the chains' matrices, to
        pass as `arrays` when the inputs should already sit in device memory."""
        torch = _torch()
        return [tuple(torch.from_numpy(a).cuda() for a in (ch.indptr, ch.indices, ch.data))
                for ch in chains]

    def __init__(self, chains, opts, nstreams=0, stream=None, arrays=None):
        self.n = len(chains)
        self._keep = arrays if arrays is not None else Batch.upload(chains)
        A = (Csr * self.n)()
        G = (Geometry * self.n)()
        O = (Options * self.n)()
        for i, (ch, o) in enumerate(zip(chains, opts)):
            rp, ci, va = self._keep[i]
            A[i] = Csr(ch.n, ch.nnz, rp.data_ptr(), ci.data_ptr(), va.data_ptr(), 1)
            G[i] = Geometry(*ch.geom)
            O[i] = o
        self.sizes = [ch.n for ch in chains]
        self.h = C.c_void_p()
        _check(lib().bamg_setup_batched(self.n, C.byref(A), C.byref(G), C.byref(O), None,
                                        nstreams, _stream(stream), C.byref(self.h)))
        self._keep = None

    def status(self, i):
        st = C.c_int32()
        hh = C.c_void_p()
        _check(lib().bamg_batch_status(self.h, i, C.byref(st), C.byref(hh)))
        return st.value

    SOLVERS = {"auto": 0, "persistent": 1, "streams": 2}

    def set_solver(self, solver):
        """'auto' (default: chains up to 5000 states in one persistent launch,
        a workgroup per chain, the others per chain on the library streams,
        both at once), 'persistent' (every chain the launch can take) or
        'streams' (none)."""
        _check(lib().bamg_batch_set_solver(self.h, Batch.SOLVERS[solver]))

    def gmres(self, restart=20, tol=1e-10, maxit=500, stream=None):
        """Solve every chain; returns (list of x tensors or None, infos, statuses)."""
        torch = _torch()
        xs = [torch.empty(n, dtype=torch.float64, device="cuda") for n in self.sizes]
        ptrs = (C.c_void_p * self.n)(*[x.data_ptr() for x in xs])
        infos = (SolveInfo * self.n)()
        sts = (C.c_int32 * self.n)()
        _check(lib().bamg_gmres_solve_batched(self.h, ptrs, restart, tol, maxit, infos, sts,
                                              _stream(stream)))
        out = [x if sts[i] >= 0 else None for i, x in enumerate(xs)]
        return out, list(infos), list(sts)

    def close(self):
        if getattr(self, "h", None) and self.h.value:
            lib().bamg_batch_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class MLP:
    """Interpolation-weight network on the device (bamg_mlp_*). Parameters
    are FP32 in the order W1, b1, W2, b2, W3, b3 (include/bamg.h)."""

    def __init__(self, params):
        p = np.ascontiguousarray(params, np.float32)
        if p.shape != (MLP_NPARAMS,):
            raise ValueError(f"expected {MLP_NPARAMS} parameters")
        self.h = C.c_void_p()
        _check(lib().bamg_mlp_create(p.ctypes.data_as(C.c_void_p), C.byref(self.h)))

    def close(self):
        if getattr(self, "h", None) and self.h.value:
            lib().bamg_mlp_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def params(self) -> np.ndarray:
        out = np.zeros(MLP_NPARAMS, np.float32)
        _check(lib().bamg_mlp_get_params(self.h, out.ctypes.data_as(C.c_void_p)))
        return out

    def forward(self, X, mode=1, stream=None):
        """Y = MLP(X); X CUDA float32 (n x 96). mode 1 = BF16 MFMA, 0 = FP32."""
        torch = _torch()
        X = X.contiguous()
        Y = torch.empty((X.shape[0], MLP_OUT), dtype=torch.float32, device=X.device)
        _check(lib().bamg_mlp_forward(self.h, C.c_void_p(X.data_ptr()), X.shape[0],
                                      C.c_void_p(Y.data_ptr()), mode, _stream(stream)))
        return Y

    def loss_grad(self, X, T, M, stream=None):
        torch = _torch()
        g = torch.empty(MLP_NPARAMS, dtype=torch.float32, device=X.device)
        loss = C.c_double()
        _check(lib().bamg_mlp_loss_grad(self.h, C.c_void_p(X.data_ptr()),
                                        C.c_void_p(T.data_ptr()), C.c_void_p(M.data_ptr()),
                                        X.shape[0], C.byref(loss), C.c_void_p(g.data_ptr()),
                                        _stream(stream)))
        return loss.value, g

    def train(self, X, T, M, batch=1024, epochs=10, lr=1e-3, stream=None):
        """Adam on the masked squared error; returns the mean loss per epoch."""
        losses = np.zeros(max(epochs, 1), np.float64)
        _check(lib().bamg_mlp_train(self.h, C.c_void_p(X.data_ptr()), C.c_void_p(T.data_ptr()),
                                    C.c_void_p(M.data_ptr()), X.shape[0], batch, epochs, lr,
                                    losses.ctypes.data_as(C.c_void_p), _stream(stream)))
        return losses[:epochs]


def mlp_init_params(seed):
    """He-normal weights and zero biases, seeded (float32, MLP_NPARAMS)."""
    rng = np.random.default_rng(seed)
    parts = []
    for (o, i) in ((MLP_HIDDEN, MLP_IN), (MLP_HIDDEN, MLP_HIDDEN), (MLP_OUT, MLP_HIDDEN)):
        parts.append(rng.standard_normal(o * i) * np.sqrt(2.0 / i))
        parts.append(np.zeros(o))
    return np.concatenate(parts).astype(np.float32)


def options_for(chain, **kw) -> Options:
    """Options with the chain's geometry: geometric coarsening on a grid or a
    line, greedy MIS coarsening otherwise."""
    kind = chain.geom[0]
    base = {"coarsening": COARSEN_GEOMETRIC if kind else COARSEN_MIS}
    base.update(kw)
    return default_options(**base)
