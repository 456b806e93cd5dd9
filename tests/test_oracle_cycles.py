"""Pins of the oracle's cycle shapes, setup passes and restriction variants
(the cycle shapes named after the two-grid method in Section 3, the inner
loop mu of Algorithm 1, the simple-averaging restriction of Section 5).

* With two levels the coarse problem is solved by the pseudo-inverse, so a
  second coarse correction adds B_c^+ (I - B_c B_c^+) Q r = 0: W-, F- and
  V-cycles coincide. With three levels the F-cycle's coarse correction (an
  F-cycle, then a V-cycle, on a two-level problem) is two V-cycles, which is
  the W-cycle's: F = W there. With four levels all three differ.
* A cycle is an affine stationary iteration x <- E x + C b with E = I - C B,
  so the cycle from a guess x0 equals x0 + C (b - B x0), C the cycle from
  zero: this pins the nonzero-guess path (smoothing from x0, the coarsest
  correction x + B_L^+ (b - B_L x)) against the zero-start one.
* Simple averaging: every entry of column i of Q is 1/|J_i|, so 1^T Q = 1^T
  and 1^T B_c = 0 hold as with the constrained fit.
* mu passes: mu = 1 is the default setup; with mu = 2 the invariants of
  Section 5 (1^T Q = 1^T, 1^T B_l = 0, symmetric M_l and N_l) still hold on
  every level (parity beyond these invariants is unpinned).
"""
import numpy as np
import pytest

import chaingen
import oracle


def rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def hier(levels, **kw):
    ch = chaingen.tandem(33, 11 / 31, 10 / 31, 10 / 31)
    o = oracle.options_for(ch, r=6, max_levels=levels, coarse_max=1, **kw)
    return ch, oracle.Hierarchy(ch, o)


def test_two_levels_all_cycles_equal():
    ch, h = hier(2)
    b = np.random.default_rng(1).standard_normal(ch.n)
    v = h.cycle(b, "V")
    assert rel(h.cycle(b, "W"), v) < 1e-12
    assert rel(h.cycle(b, "F"), v) < 1e-12


def test_three_levels_f_equals_w_and_differs_from_v():
    ch, h = hier(3)
    b = np.random.default_rng(2).standard_normal(ch.n)
    w, f, v = h.cycle(b, "W"), h.cycle(b, "F"), h.cycle(b, "V")
    assert rel(f, w) < 1e-12
    assert rel(w, v) > 1e-6


def test_four_levels_shapes_differ():
    ch = chaingen.tandem(65, 11 / 31, 10 / 31, 10 / 31)
    h = oracle.Hierarchy(ch, oracle.options_for(ch, r=8, max_levels=4, coarse_max=1))
    assert h.levels == 4
    b = np.random.default_rng(3).standard_normal(ch.n)
    w, f, v = h.cycle(b, "W"), h.cycle(b, "F"), h.cycle(b, "V")
    assert rel(w, f) > 1e-8 and rel(f, v) > 1e-8 and rel(w, v) > 1e-8


@pytest.mark.parametrize("kind", ["V", "W", "F"])
def test_cycle_from_a_guess_is_affine(kind):
    ch = chaingen.tandem(65, 11 / 31, 10 / 31, 10 / 31)
    h = oracle.Hierarchy(ch, oracle.options_for(ch, r=8, max_levels=4, coarse_max=1))
    B = h.scipy(0, "B")
    rng = np.random.default_rng(4)
    b, x0 = rng.standard_normal(ch.n), rng.standard_normal(ch.n)
    got = h.cycle(b, kind, x=x0)
    want = x0 + h.cycle(b - B @ x0, kind)
    assert rel(got, want) < 1e-11


def test_options_cycle_used_by_vcycle_and_gmres():
    ch, h = hier(3, cycle="W")
    b = np.random.default_rng(5).standard_normal(ch.n)
    assert np.array_equal(h.vcycle(b), h.cycle(b, "W"))
    x, info = h.gmres(m=20, tol=1e-12, maxit=200)
    assert info.converged
    _, hv = hier(3)
    _, iv = hv.gmres(m=20, tol=1e-12, maxit=200)
    assert info.iterations <= iv.iterations


def test_simple_averaging_restriction():
    ch, h = hier(3, restriction="average")
    for l in range(h.levels - 1):
        # pattern of Q^T is P's (structurally: P may store zero weights)
        rp_p, ci_p, _ = h.csr(l, "P")
        rp_q, ci_q, _ = h.csr(l, "Qt")
        assert np.array_equal(rp_p, rp_q) and np.array_equal(ci_p, ci_q)
        Q = h.scipy(l, "Q").tocsc()
        Q.sort_indices()
        counts = np.diff(Q.indptr)
        for i in range(Q.shape[1]):
            col = Q.data[Q.indptr[i]:Q.indptr[i + 1]]
            assert np.array_equal(col, np.full(counts[i], 1.0 / counts[i]))
        Bc = h.scipy(l + 1, "B")
        assert np.abs(np.asarray(Bc.sum(axis=0))).max() < 1e-13 * np.abs(Bc.data).max()
    _, hl = hier(3)
    assert not np.allclose(h.scipy(0, "Q").toarray(), hl.scipy(0, "Q").toarray())


def test_mu_passes():
    ch, h1 = hier(3)
    _, hm1 = hier(3, mu=1)
    assert np.array_equal(h1.csr(0, "P")[2], hm1.csr(0, "P")[2])
    _, h2 = hier(3, mu=2)
    assert not np.array_equal(h1.csr(0, "P")[2], h2.csr(0, "P")[2])
    for l in range(h2.levels):
        B = h2.scipy(l, "B")
        assert np.abs(np.asarray(B.sum(axis=0))).max() < 1e-13 * np.abs(B.data).max()
        if l > 0:
            M, N = h2.scipy(l, "M"), h2.scipy(l, "N")
            assert abs(M - M.T).max() < 1e-14 * abs(M).max()
            assert abs(N - N.T).max() < 1e-14 * abs(N).max()
        if l < h2.levels - 1:
            Q = h2.scipy(l, "Q")
            assert np.abs(np.asarray(Q.sum(axis=0)) - 1).max() < 1e-13
    x, info = h2.gmres(m=20, tol=1e-12, maxit=300)
    assert info.converged
