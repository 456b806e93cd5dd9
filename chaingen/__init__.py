"""Seeded synthetic Markov-chain generators.

This module builds the transition matrices the method is run on. It holds
none of the method's arithmetic: it only writes down transition
probabilities and returns the column-stochastic matrix ``A`` (entry
``a_ij = p_ji``, Section 2 of the paper) in CSR form, rows indexed by the
destination state. Both the HIP path and the CPU oracle consume its output.

Workloads (Section 7 of the paper):

* ``tandem``       -- two-station tandem queueing network on an N x N grid
                      (Table 3); uniformised, blocked moves become self-loops.
* ``birth_death``  -- one-dimensional birth-death chain (Table 1).
* ``grid2d``       -- uniform random walk on an nx x ny grid (Table 2).
* ``delaunay_walk``-- random walk on the Delaunay triangulation of uniform
                      random points in the unit square (Table 4).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

__all__ = [
    "Chain",
    "tandem",
    "tandem_random_rates",
    "birth_death",
    "grid2d",
    "delaunay_walk",
]


class Chain:
    """A chain in CSR form: ``indptr``/``indices``/``data`` of ``A``.

    ``geom`` is ``(kind, nx, ny)`` with kind 0 = none, 1 = 1-D line of nx
    states, 2 = 2-D grid with state index ``iy * nx + ix``.
    """

    def __init__(self, A: sp.csr_matrix, geom=(0, 0, 0), name="chain", extra=None):
        A = sp.csr_matrix(A, dtype=np.float64)
        A.sum_duplicates()
        A.sort_indices()
        self.n = A.shape[0]
        self.indptr = np.ascontiguousarray(A.indptr, dtype=np.int32)
        self.indices = np.ascontiguousarray(A.indices, dtype=np.int32)
        self.data = np.ascontiguousarray(A.data, dtype=np.float64)
        self.geom = tuple(int(g) for g in geom)
        self.name = name
        self.extra = extra or {}

    @property
    def nnz(self) -> int:
        return int(self.indptr[-1])

    def to_scipy(self) -> sp.csr_matrix:
        return sp.csr_matrix((self.data, self.indices, self.indptr), shape=(self.n, self.n))


def _from_moves(n, src, dst, prob, geom, name, extra=None) -> Chain:
    """Assemble ``A`` with ``a[dst, src] += prob`` (column-stochastic)."""
    A = sp.coo_matrix((prob, (dst, src)), shape=(n, n)).tocsr()
    return Chain(A, geom, name, extra)


def tandem(N: int, lam: float, mu1: float, mu2: float, model: str = "diag") -> Chain:
    """Tandem queueing network on the state grid ``(n1, n2) in [0, N-1]^2``.

    Uniformised so that ``lam + mu1 + mu2 = 1``; a move that would leave the
    grid is a self-loop. ``model="diag"`` follows the paper's description of
    its Fig. 4b (arrival = diagonal move (+1,+1), service 1 = (-1,0),
    service 2 = (0,-1)); ``model="serial"`` is the classic serial tandem
    (arrival (+1,0), transfer (-1,+1), departure (0,-1)). State index is
    ``n2 * N + n1`` (ix = n1, iy = n2).
    """
    s = lam + mu1 + mu2
    lam, mu1, mu2 = lam / s, mu1 / s, mu2 / s
    n1, n2 = np.meshgrid(np.arange(N), np.arange(N), indexing="xy")
    n1 = n1.ravel()
    n2 = n2.ravel()
    idx = n2 * N + n1
    if model == "diag":
        moves = [((1, 1), lam), ((-1, 0), mu1), ((0, -1), mu2)]
    elif model == "serial":
        moves = [((1, 0), lam), ((-1, 1), mu1), ((0, -1), mu2)]
    else:
        raise ValueError(model)
    src, dst, prob = [], [], []
    for (d1, d2), p in moves:
        t1, t2 = n1 + d1, n2 + d2
        ok = (t1 >= 0) & (t1 < N) & (t2 >= 0) & (t2 < N)
        tgt = np.where(ok, t2 * N + t1, idx)
        src.append(idx)
        dst.append(tgt)
        prob.append(np.full(idx.shape, p))
    return _from_moves(N * N, np.concatenate(src), np.concatenate(dst), np.concatenate(prob),
                       (2, N, N), f"tandem{N}", {"rates": (lam, mu1, mu2), "model": model})


def tandem_random_rates(seed: int):
    """Rates (lam, mu1, mu2) drawn i.i.d. uniform in [0.2, 0.5], normalised to sum 1."""
    rng = np.random.default_rng(seed)
    r = rng.uniform(0.2, 0.5, size=3)
    r = r / r.sum()
    return float(r[0]), float(r[1]), float(r[2])


def birth_death(n: int, mu: float = 0.96) -> Chain:
    """Birth-death chain on states 0..n-1 (Table 1 workload).

    From state j: move to j-1 with probability mu/(1+mu), to j+1 with
    probability 1/(1+mu); blocked moves are self-loops. Detailed balance
    gives pi_i proportional to mu^(-i).
    """
    j = np.arange(n)
    pl, pr = mu / (1 + mu), 1 / (1 + mu)
    left = np.where(j > 0, j - 1, j)
    right = np.where(j < n - 1, j + 1, j)
    src = np.concatenate([j, j])
    dst = np.concatenate([left, right])
    prob = np.concatenate([np.full(n, pl), np.full(n, pr)])
    return _from_moves(n, src, dst, prob, (1, n, 1), f"birthdeath{n}", {"mu": mu})


def grid2d(nx: int, ny: int) -> Chain:
    """Uniform random walk on the 4-neighbour nx x ny grid (Table 2 workload).

    Transition probabilities are 1/deg; the stationary vector is
    proportional to the degree.
    """
    ix, iy = np.meshgrid(np.arange(nx), np.arange(ny), indexing="xy")
    ix = ix.ravel()
    iy = iy.ravel()
    idx = iy * nx + ix
    src, dst = [], []
    for dx, dy in ((1, 0), (-1, 0), (0, 1), (0, -1)):
        tx, ty = ix + dx, iy + dy
        ok = (tx >= 0) & (tx < nx) & (ty >= 0) & (ty < ny)
        src.append(idx[ok])
        dst.append((ty * nx + tx)[ok])
    src = np.concatenate(src)
    dst = np.concatenate(dst)
    deg = np.bincount(src, minlength=nx * ny).astype(np.float64)
    return _from_moves(nx * ny, src, dst, 1.0 / deg[src], (2, nx, ny), f"grid{nx}x{ny}",
                       {"deg": deg})


def hub_walk(n: int, hubs: int, links: int, seed: int) -> Chain:
    """Random walk on a ring of ``n`` states (each joined to the states one
    and two steps away) plus ``hubs`` extra states, each joined to ``links``
    distinct ring states drawn with numpy's PCG64 seeded by ``seed``.
    ``a_ij = 1/deg(j)`` for every edge, so pi_i is proportional to deg(i).
    The hubs give rows far longer than the rest (a stress case for per-row
    work)."""
    rng = np.random.default_rng(seed)
    i = np.arange(n)
    e = [np.stack([i, (i + 1) % n], 1), np.stack([i, (i + 2) % n], 1)]
    for h in range(hubs):
        tgt = rng.choice(n, size=links, replace=False)
        e.append(np.stack([np.full(links, n + h), tgt], 1))
    e = np.concatenate(e)
    src = np.concatenate([e[:, 0], e[:, 1]])
    dst = np.concatenate([e[:, 1], e[:, 0]])
    N = n + hubs
    deg = np.bincount(src, minlength=N).astype(np.float64)
    return _from_moves(N, src, dst, 1.0 / deg[src], (0, 0, 0), f"hub{n}x{hubs}",
                       {"deg": deg})


def _morton_order(pts: np.ndarray) -> np.ndarray:
    """Permutation that sorts points in [0,1)^2 along a Z-order curve."""
    q = np.minimum((pts * 65536.0).astype(np.uint64), 65535)

    def spread(v):
        v = (v | (v << np.uint64(8))) & np.uint64(0x00FF00FF)
        v = (v | (v << np.uint64(4))) & np.uint64(0x0F0F0F0F)
        v = (v | (v << np.uint64(2))) & np.uint64(0x33333333)
        v = (v | (v << np.uint64(1))) & np.uint64(0x55555555)
        return v

    code = spread(q[:, 0]) | (spread(q[:, 1]) << np.uint64(1))
    return np.argsort(code, kind="stable")


def delaunay_walk(npts: int, seed: int, order: str = "morton") -> Chain:
    """Random walk on the Delaunay triangulation of ``npts`` uniform points.

    Points are uniform in the unit square (numpy PCG64 seeded by ``seed``);
    the triangulation is scipy's Qhull (input generation only). States are
    labelled along a Z-order curve (``order="morton"``) so that graph
    neighbours sit close in memory; ``order="random"`` keeps draw order.
    ``a_ij = 1/deg(j)`` for every edge, so pi_i is proportional to deg(i).
    """
    from scipy.spatial import Delaunay

    rng = np.random.default_rng(seed)
    pts = rng.random((npts, 2))
    if order == "morton":
        pts = pts[_morton_order(pts)]
    tri = Delaunay(pts)
    s = tri.simplices.astype(np.int64)
    e = np.concatenate([s[:, [0, 1]], s[:, [1, 2]], s[:, [2, 0]]])
    e = np.sort(e, axis=1)
    e = np.unique(e[:, 0] * npts + e[:, 1])
    a, b = e // npts, e % npts
    src = np.concatenate([a, b])
    dst = np.concatenate([b, a])
    deg = np.bincount(src, minlength=npts).astype(np.float64)
    return _from_moves(npts, src, dst, 1.0 / deg[src], (0, 0, 0), f"delaunay{npts}",
                       {"deg": deg, "edges": len(e), "hull": len(tri.convex_hull)})
