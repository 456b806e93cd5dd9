"""ctypes binding of the plain FP64 CPU oracle (``bamg_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the tests, by ``__graft_entry__.smoke``
and by the CPU-baseline leg of ``bench.py``. The product package never
imports it, and it imports nothing from the product package.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bamg_oracle.c")
_LIB = os.path.join(_HERE, "liborc.so")

ORC_OK = 0
ORC_NOT_CONVERGED = 1
STATUS = {0: "OK", 1: "NOT_CONVERGED", -1: "E_ARG", -2: "E_NOT_STOCHASTIC", -3: "E_REDUCIBLE",
          -4: "E_BAD_DIAG", -5: "E_COARSE", -6: "E_BREAKDOWN", -9: "E_NOMEM"}


class OracleError(RuntimeError):
    def __init__(self, code):
        super().__init__(f"oracle status {code} ({STATUS.get(code, '?')})")
        self.code = code


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math, no FMA contraction;
    OpenMP over independent row loops only, so any thread count gives the
    same bits)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
                               "-fno-fast-math", "-fopenmp", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class Options(C.Structure):
    _fields_ = [("r", C.c_int32), ("setup_cycles", C.c_int32), ("nu_pre", C.c_int32),
                ("nu_post", C.c_int32), ("nu_setup", C.c_int32), ("omega", C.c_double),
                ("max_interp", C.c_int32), ("max_levels", C.c_int32), ("coarse_max", C.c_int32),
                ("coarsening", C.c_int32), ("geom_kind", C.c_int32), ("nx", C.c_int32),
                ("ny", C.c_int32), ("seed", C.c_uint64), ("smoother", C.c_int32),
                ("interp_rule", C.c_int32), ("record_features", C.c_int32),
                ("cycle", C.c_int32), ("mu", C.c_int32), ("restriction", C.c_int32),
                ("cr_theta", C.c_double), ("cr_beta", C.c_double), ("cr_sweeps", C.c_int32),
                ("cr_rounds", C.c_int32)]


class Info(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("restarts", C.c_int32), ("converged", C.c_int32),
                ("rel_residual", C.c_double), ("x_min", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        P = C.POINTER
        _lib.orc_setup.argtypes = [C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, P(Options),
                                   P(C.c_void_p)]
        _lib.orc_destroy.argtypes = [C.c_void_p]
        _lib.orc_num_levels.argtypes = [C.c_void_p]
        _lib.orc_set_threads.argtypes = [C.c_int]
        for name in ("orc_level_dims", "orc_level_cf", "orc_level_vectors"):
            getattr(_lib, name).argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p][: 3 if name == "orc_level_dims" else 4]
        _lib.orc_level_csr.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p]
        for name in ("orc_sigma", "orc_x0", "orc_coarse_pinv"):
            getattr(_lib, name).argtypes = [C.c_void_p, C.c_void_p]
        _lib.orc_complexity.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        _lib.orc_vcycle.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        _lib.orc_cycle.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_int]
        _lib.orc_smooth.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p]
        _lib.orc_gmres.argtypes = [C.c_void_p, C.c_void_p, C.c_int32, C.c_double, C.c_int32,
                                   C.c_int32, C.c_int32, P(Info)]
        _lib.orc_philox4x64.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        _lib.orc_uniform_pm1.argtypes = [C.c_uint64] * 4
        _lib.orc_uniform_pm1.restype = C.c_double
        for name in ("orc_ls_row", "orc_ls_row_sum1"):
            getattr(_lib, name).argtypes = [C.c_int, C.c_int] + [C.c_void_p] * 4
        _lib.orc_fit_point.argtypes = [C.c_int, C.c_int, C.c_int] + [C.c_void_p] * 3 + \
            [C.c_int, C.c_void_p]
        _lib.orc_rayleigh_sigma.argtypes = [C.c_int] + [C.c_void_p] * 12
        _lib.orc_gsvd.argtypes = [C.c_int] + [C.c_void_p] * 6
        _lib.orc_svd_jacobi.argtypes = [C.c_int] + [C.c_void_p] * 4
        _lib.orc_mis.argtypes = [C.c_int, C.c_void_p, C.c_void_p, C.c_uint64, C.c_int, C.c_void_p]
        _lib.orc_cr.argtypes = [C.c_int] + [C.c_void_p] * 5 + [
            C.c_uint64, C.c_int, C.c_double, C.c_double, C.c_int, C.c_int, C.c_double,
            C.c_void_p, C.c_void_p, C.c_void_p]
        _lib.orc_row_colouring.argtypes = [C.c_int] + [C.c_void_p] * 5
        _lib.orc_default_options.argtypes = [P(Options)]
        _lib.orc_harvest.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p,
                                     C.c_void_p]
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


def default_options(**kw) -> Options:
    o = Options()
    lib().orc_default_options(C.byref(o))
    for k, v in kw.items():
        if k == "coarsening" and isinstance(v, str):
            v = {"geom": 0, "mis": 1, "cr": 2}[v]
        if k == "smoother" and isinstance(v, str):
            v = {"jacobi": 0, "kaczmarz": 1}[v]
        if k == "cycle" and isinstance(v, str):
            v = {"V": 0, "W": 1, "F": 2}[v]
        if k == "restriction" and isinstance(v, str):
            v = {"ls": 0, "average": 1}[v]
        setattr(o, k, v)
    return o


def options_for(chain, **kw) -> Options:
    """Options with the chain's geometry filled in (geometric coarsening when
    the chain has a grid, greedy MIS otherwise)."""
    kind, nx, ny = chain.geom
    base = dict(geom_kind=kind, nx=nx, ny=ny, coarsening=0 if kind else 1)
    base.update(kw)
    return default_options(**base)


class Hierarchy:
    """A set-up oracle hierarchy; wraps ``orc_ctx``."""

    def __init__(self, chain, opts: Options):
        self.opts = opts
        self.n = chain.n
        self._keep = (np.ascontiguousarray(chain.indptr, np.int32),
                      np.ascontiguousarray(chain.indices, np.int32),
                      np.ascontiguousarray(chain.data, np.float64))
        h = C.c_void_p()
        st = lib().orc_setup(self.n, _p(self._keep[0]), _p(self._keep[1]), _p(self._keep[2]),
                             C.byref(opts), C.byref(h))
        if st != ORC_OK:
            raise OracleError(st)
        self.h = h

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_destroy(self.h)
            self.h = None

    @property
    def levels(self) -> int:
        return lib().orc_num_levels(self.h)

    def dims(self, l):
        d = np.zeros(6, np.int64)
        st = lib().orc_level_dims(self.h, l, _p(d))
        if st:
            raise OracleError(st)
        return d

    def csr(self, l, what):
        """what: 'B', 'Bt', 'M', 'N', 'P', 'Q', 'Qt' -> (indptr, indices, data)."""
        code = {"B": 0, "Bt": 1, "M": 2, "N": 3, "P": 4, "Q": 5, "Qt": 6}[what]
        d = self.dims(l)
        n, nc = int(d[0]), int(d[1])
        nnz = {0: d[2], 1: d[2], 2: d[3], 3: d[3], 4: d[4], 5: d[4], 6: d[4]}[code]
        nr = nc if code == 5 else n
        rp = np.zeros(nr + 1, np.int32)
        ci = np.zeros(int(nnz), np.int32)
        v = np.zeros(int(nnz), np.float64)
        st = lib().orc_level_csr(self.h, l, code, _p(rp), _p(ci), _p(v))
        if st:
            raise OracleError(st)
        return rp, ci, v

    def scipy(self, l, what):
        import scipy.sparse as sp
        rp, ci, v = self.csr(l, what)
        d = self.dims(l)
        n, nc = int(d[0]), int(d[1])
        shape = {"P": (n, nc), "Qt": (n, nc), "Q": (nc, n)}.get(what, (n, n))
        return sp.csr_matrix((v, ci, rp), shape=shape)

    def cf(self, l):
        n = int(self.dims(l)[0])
        cf = np.zeros(n, np.int32)
        cidx = np.zeros(n, np.int32)
        st = lib().orc_level_cf(self.h, l, _p(cf), _p(cidx))
        if st:
            raise OracleError(st)
        return cf, cidx

    def vectors(self, l):
        n = int(self.dims(l)[0])
        r = self.opts.r
        U = np.zeros((n, r))
        V = np.zeros((n, r))
        lib().orc_level_vectors(self.h, l, _p(U), _p(V))
        return U, V

    def sigma(self):
        s = np.zeros(self.opts.r)
        lib().orc_sigma(self.h, _p(s))
        return s

    def x0(self):
        x = np.zeros(self.n)
        lib().orc_x0(self.h, _p(x))
        return x

    def harvest(self, l):
        """Cycle-1 MLP features of level l's F points (needs
        record_features=1) and the final P rows: X (nF x 96), T, M (nF x 8)."""
        nf = C.c_int64()
        st = lib().orc_harvest(self.h, l, C.byref(nf), None, None, None)
        if st:
            raise OracleError(st)
        X = np.zeros((nf.value, 96))
        T = np.zeros((nf.value, 8))
        M = np.zeros((nf.value, 8))
        lib().orc_harvest(self.h, l, C.byref(nf), _p(X), _p(T), _p(M))
        return X, T, M

    def coarse_pinv(self):
        nL = int(self.dims(self.levels - 1)[0])
        B = np.zeros((nL, nL))
        lib().orc_coarse_pinv(self.h, _p(B))
        return B

    def complexity(self):
        oc, og = C.c_double(), C.c_double()
        lib().orc_complexity(self.h, C.byref(oc), C.byref(og))
        return oc.value, og.value

    def vcycle(self, b):
        b = np.ascontiguousarray(b, np.float64)
        x = np.zeros_like(b)
        lib().orc_vcycle(self.h, _p(b), _p(x))
        return x

    def cycle(self, b, kind="V", x=None):
        """One cycle of type kind ('V', 'W', 'F') for B x = b on level 0, from
        x = 0, or from the given x."""
        b = np.ascontiguousarray(b, np.float64)
        xz = x is None
        x = np.zeros_like(b) if xz else np.array(x, np.float64, copy=True)
        st = lib().orc_cycle(self.h, {"V": 0, "W": 1, "F": 2}[kind], _p(b), _p(x), 1 if xz else 0)
        if st:
            raise OracleError(st)
        return x

    def smooth(self, l, b, x):
        b = np.ascontiguousarray(b, np.float64)
        x = np.array(x, np.float64, copy=True)
        st = lib().orc_smooth(self.h, l, _p(b), _p(x))
        if st:
            raise OracleError(st)
        return x

    def gmres(self, m=20, tol=1e-10, maxit=500, x0=None, precondition=True):
        x = np.zeros(self.n) if x0 is None else np.array(x0, np.float64, copy=True)
        info = Info()
        st = lib().orc_gmres(self.h, _p(x), m, tol, maxit, 0 if x0 is None else 1,
                             1 if precondition else 0, C.byref(info))
        if st < 0:
            raise OracleError(st)
        return x, info


def set_threads(n: int) -> int:
    """Threads of the oracle's OpenMP row loops (same results for any count);
    returns the previous count."""
    return lib().orc_set_threads(n)


def philox4x64(ctr, key):
    c = np.ascontiguousarray(ctr, np.uint64)
    k = np.ascontiguousarray(key, np.uint64)
    out = np.zeros(4, np.uint64)
    lib().orc_philox4x64(_p(c), _p(k), _p(out))
    return out


def uniform_pm1(seed, side, k, i):
    return lib().orc_uniform_pm1(seed, side, k, i)


def ls_row(G, g, w):
    G = np.ascontiguousarray(G, np.float64)
    r, m = G.shape
    p = np.zeros(m)
    st = lib().orc_ls_row(r, m, _p(G), _p(np.ascontiguousarray(g, np.float64)),
                          _p(np.ascontiguousarray(w, np.float64)), _p(p))
    if st:
        raise OracleError(st)
    return p


def ls_row_sum1(G, g, w):
    G = np.ascontiguousarray(G, np.float64)
    r, m = G.shape
    q = np.zeros(m)
    st = lib().orc_ls_row_sum1(r, m, _p(G), _p(np.ascontiguousarray(g, np.float64)),
                               _p(np.ascontiguousarray(w, np.float64)), _p(q))
    if st:
        raise OracleError(st)
    return q


def fit_point(G, g, w, rule=1, sum1=False):
    """One F point's weights as the setup fits them (rule 0 plain LS, rule 1
    with negative weights removed; sum1 for the constrained Q fit)."""
    G = np.ascontiguousarray(G, np.float64)
    r, m = G.shape
    p = np.zeros(m)
    st = lib().orc_fit_point(rule, r, m, _p(G), _p(np.ascontiguousarray(g, np.float64)),
                             _p(np.ascontiguousarray(w, np.float64)), 1 if sum1 else 0, _p(p))
    if st:
        raise OracleError(st)
    return p


def rayleigh_sigma(B, M, N, u, v):
    """eq. singular_value for one pair (u, v); B, M, N scipy sparse."""
    import scipy.sparse as sp
    mats = []
    for X in (B, M, N):
        X = sp.csr_matrix(X)
        X.sort_indices()
        mats += [np.ascontiguousarray(X.indptr, np.int32), np.ascontiguousarray(X.indices, np.int32),
                 np.ascontiguousarray(X.data, np.float64)]
    u = np.ascontiguousarray(u, np.float64)
    v = np.ascontiguousarray(v, np.float64)
    out = np.zeros(1)
    st = lib().orc_rayleigh_sigma(B.shape[0], *[_p(a) for a in mats], _p(u), _p(v), _p(out))
    if st:
        raise OracleError(st)
    return float(out[0])


def gsvd(B, M, N):
    n = B.shape[0]
    s = np.zeros(n)
    U = np.zeros((n, n))
    V = np.zeros((n, n))
    st = lib().orc_gsvd(n, _p(np.ascontiguousarray(B, np.float64)),
                        _p(np.ascontiguousarray(M, np.float64)),
                        _p(np.ascontiguousarray(N, np.float64)), _p(s), _p(U), _p(V))
    if st:
        raise OracleError(st)
    # U, V come back column-major: column t is row t of the arrays
    return s, U.T.copy(), V.T.copy()


def svd_jacobi(B):
    n = B.shape[0]
    s = np.zeros(n)
    U = np.zeros((n, n))
    V = np.zeros((n, n))
    st = lib().orc_svd_jacobi(n, _p(np.ascontiguousarray(B, np.float64)), _p(s), _p(U), _p(V))
    if st:
        raise OracleError(st)
    return s, U.T.copy(), V.T.copy()


def mis(indptr, indices, seed, level):
    n = len(indptr) - 1
    cf = np.zeros(n, np.int32)
    lib().orc_mis(n, _p(np.ascontiguousarray(indptr, np.int32)),
                  _p(np.ascontiguousarray(indices, np.int32)), seed, level, _p(cf))
    return cf


def cr(B, G, seed, level, theta=0.8, beta=0.7, sweeps=5, rounds=10, omega=0.7):
    """Compatible-relaxation C/F split (R-CR) of the scipy CSR operator B on
    the CSR pattern G (symmetrised, no diagonal): (cf, per-round rates)."""
    n = B.shape[0]
    cf = np.zeros(n, np.int32)
    rates = np.zeros(max(rounds, 1), np.float64)
    nr = C.c_int32()
    st = lib().orc_cr(n, _p(np.ascontiguousarray(B.indptr, np.int32)),
                      _p(np.ascontiguousarray(B.indices, np.int32)),
                      _p(np.ascontiguousarray(B.data, np.float64)),
                      _p(np.ascontiguousarray(G.indptr, np.int32)),
                      _p(np.ascontiguousarray(G.indices, np.int32)), seed, level, theta, beta,
                      sweeps, rounds, omega, _p(cf), _p(rates), C.byref(nr))
    if st:
        raise OracleError(st)
    return cf, rates[:nr.value]


def row_colouring(indptr, indices, cindptr, cindices):
    n = len(indptr) - 1
    col = np.zeros(n, np.int32)
    lib().orc_row_colouring(n, _p(np.ascontiguousarray(indptr, np.int32)),
                            _p(np.ascontiguousarray(indices, np.int32)),
                            _p(np.ascontiguousarray(cindptr, np.int32)),
                            _p(np.ascontiguousarray(cindices, np.int32)), _p(col))
    return col
