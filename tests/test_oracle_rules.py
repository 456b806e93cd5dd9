"""Pins of three oracle rules that the end-to-end checks cannot tell apart
from plausible slips (CPU only):

* the algebraic choice of the interpolation sets J_i (Section 4.1: at most c
  coarse neighbours; R-JI ranks them by common-neighbour count, ties to the
  smaller index), against a dense brute force over the symmetrised pattern;
* the active-set fit R-ACT (a reading added to eq. ls_interpolation: while a
  weight is negative the most negative point leaves J_i and the fit is
  redone), against numpy's least squares on the final support and a
  hand-worked case where the other drop orders give other supports;
* the sigma update of eq. singular_value, which returns the exact singular
  value for exact generalized singular vectors (Section 4.2), against
  numpy's SVD and Cholesky factors.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import chaingen
import oracle


# ----------------------------------------------------------------- J_i
def brute_force_J(B, cf, cidx, c):
    """Dense brute force of R-JI: S = pattern(B + B^T) without the diagonal;
    the score of a coarse neighbour j of F point i is (S @ S)[i, j], the
    number of common neighbours; the c best by (score descending, index
    ascending) are kept and listed by ascending coarse index. C points
    interpolate from themselves."""
    n = B.shape[0]
    S = ((abs(B) + abs(B.T)).toarray() != 0).astype(np.int64)
    np.fill_diagonal(S, 0)
    S2 = S @ S
    rows = []
    for i in range(n):
        if cf[i]:
            rows.append([cidx[i]])
            continue
        cand = [j for j in np.flatnonzero(S[i]) if cf[j]]
        cand.sort(key=lambda j: (-S2[i, j], j))
        rows.append(sorted(cidx[j] for j in cand[:c]))
    return rows


@pytest.mark.parametrize("make,c", [
    (lambda: chaingen.delaunay_walk(600, 21), 3),
    (lambda: chaingen.delaunay_walk(600, 21), 2),
    (lambda: chaingen.hub_walk(600, 3, 80, 5), 3),
], ids=["delaunay600_c3", "delaunay600_c2", "hub600_c3"])
def test_algebraic_J_matches_brute_force(make, c):
    ch = make()
    h = oracle.Hierarchy(ch, oracle.options_for(ch, r=8, max_interp=c, coarse_max=40,
                                                max_levels=4))
    assert h.levels >= 3
    checked = 0
    for l in (0, 1):
        B = h.scipy(l, "B")
        cf, cidx = h.cf(l)
        want = brute_force_J(B, cf, cidx, c)
        rp, ci, _ = h.csr(l, "P")
        got = [list(ci[rp[i]:rp[i + 1]]) for i in range(len(rp) - 1)]
        assert got == want, l
        # the cap binds somewhere, so the ranking is really exercised
        S = ((abs(B) + abs(B.T)).toarray() != 0)
        np.fill_diagonal(S, False)
        ncand = np.array([(S[i] & (cf == 1)).sum() for i in range(len(cf))])
        assert ((cf == 0) & (ncand > c)).any()
        checked += 1
    assert checked == 2


# --------------------------------------------------------------- R-ACT
def wls(G, g, w, cols):
    p = np.zeros(G.shape[1])
    sw = np.sqrt(w)
    p[cols] = np.linalg.lstsq(G[:, cols] * sw[:, None], g * sw, rcond=None)[0]
    return p


def kkt_sum1(G, g, w, cols):
    """min sum_{k>=1} w_k (g_k - G_k q)^2 subject to sum(q) = 1, on cols."""
    Gs, gs, ws = G[1:, cols], g[1:], w[1:]
    m = len(cols)
    K = np.zeros((m + 1, m + 1))
    K[:m, :m] = 2 * Gs.T @ (ws[:, None] * Gs)
    K[:m, m] = 1
    K[m, :m] = 1
    rhs = np.concatenate([2 * Gs.T @ (ws * gs), [1.0]])
    q = np.zeros(G.shape[1])
    q[cols] = np.linalg.solve(K, rhs)[:m]
    return q


def test_active_set_hand_worked_case():
    """r = 4 equations, m = 3 points, unit weights.
      G columns: c0 = (1, 0, -1, -1), c1 = (-1, 1, 0, -1), c2 = (0, -1, 1, 1);
      g = (2, -5, 3, 7) = -2 c0 - 4 c1 + 1 c2 exactly, so plain LS gives
      (-2, -4, 1).
    Most negative first (R-ACT): drop c1. Normal equations on {c0, c2}:
      [[3, -2], [-2, 3]] (a, b) = (c0.g, c2.g) = (-8, 15), det 5,
      a = (3(-8) + 2(15))/5 = 6/5, b = (3(15) + 2(-8))/5 = 29/5: both >= 0.
    First negative first: drop c0; on {c1, c2}: [[3, -2], [-2, 3]] (a, b) =
      (-14, 15) gives a = -12/5 < 0, so c1 goes too and c2 alone gives
      15/3 = 5: the result (0, 0, 5), as also when every negative point is
      dropped at once."""
    G = np.array([[1.0, -1.0, 0.0], [0.0, 1.0, -1.0], [-1.0, 0.0, 1.0], [-1.0, -1.0, 1.0]])
    g = np.array([2.0, -5.0, 3.0, 7.0])
    w = np.ones(4)
    assert np.allclose(oracle.fit_point(G, g, w, rule=0), [-2.0, -4.0, 1.0], atol=1e-14)
    assert np.allclose(oracle.fit_point(G, g, w, rule=1), [6 / 5, 0.0, 29 / 5], atol=1e-14)
    # the two-point case of the same rule: the single survivor may stay negative
    G2 = np.array([[1.0, 1.0], [0.0, 1.0]])
    g2 = np.array([-4.0, -3.0])  # plain LS (-1, -3); c1 leaves; c0 alone: -4
    assert np.allclose(oracle.fit_point(G2, g2, np.ones(2), rule=1), [-4.0, 0.0], atol=1e-14)


def test_active_set_equals_plain_ls_when_nonnegative():
    rng = np.random.default_rng(3)
    hits = 0
    for _ in range(200):
        r, m = rng.integers(4, 9), rng.integers(1, 5)
        G = rng.uniform(0.1, 1.0, (r, m))
        pstar = rng.uniform(0.05, 1.0, m)
        g = G @ pstar + 1e-3 * rng.standard_normal(r)
        w = rng.uniform(0.1, 1.0, r)
        plain = wls(G, g, w, list(range(m)))
        if (plain < 0).any():
            continue
        hits += 1
        got = oracle.fit_point(G, g, w, rule=1)
        assert np.allclose(got, plain, rtol=1e-12, atol=1e-12)
    assert hits > 100


@pytest.mark.parametrize("sum1", [False, True], ids=["P_row", "Q_column"])
def test_active_set_is_ls_on_its_support(sum1):
    """On random rows with negative plain weights, the result is the (KKT)
    least-squares solution on its own support, nonnegative there unless a
    single point is left, and exactly 0 off it."""
    rng = np.random.default_rng(11)
    dropped = 0
    for _ in range(300):
        r, m = int(rng.integers(5, 9)), int(rng.integers(2, 5))
        G = rng.standard_normal((r, m))
        g = rng.standard_normal(r)
        w = rng.uniform(0.2, 1.0, r)
        p = oracle.fit_point(G, g, w, rule=1, sum1=sum1)
        supp = [t for t in range(m) if p[t] != 0.0]
        assert supp, p
        ref = kkt_sum1(G, g, w, supp) if sum1 else wls(G, g, w, supp)
        assert np.allclose(p, ref, rtol=1e-10, atol=1e-11), (p, ref)
        if len(supp) > 1:
            assert (p[supp] >= 0).all()
        if sum1:
            assert abs(p.sum() - 1.0) < 1e-12
        dropped += len(supp) < m
    assert dropped > 50


def test_plain_rule_is_weighted_lstsq():
    rng = np.random.default_rng(2)
    for _ in range(50):
        r, m = 8, int(rng.integers(1, 5))
        G, g, w = rng.standard_normal((r, m)), rng.standard_normal(r), rng.uniform(0.1, 1, r)
        assert np.allclose(oracle.fit_point(G, g, w, rule=0), wls(G, g, w, list(range(m))),
                           rtol=1e-11, atol=1e-12)
        assert np.allclose(oracle.fit_point(G, g, w, rule=0, sum1=True),
                           kkt_sum1(G, g, w, list(range(m))), rtol=1e-10, atol=1e-11)


# --------------------------------------------------------------- sigma
def random_sparse(n, density, rng):
    A = sp.random(n, n, density=density, random_state=rng, data_rvs=rng.standard_normal)
    return (A + sp.identity(n) * 3.0).tocsr()


def random_spd(n, rng):
    A = sp.random(n, n, density=0.1, random_state=rng, data_rvs=rng.standard_normal)
    return (A @ A.T + sp.identity(n) * 2.0).tocsr()


def test_sigma_exact_for_svd_pairs():
    """M = N = I (level 0): eq. singular_value on the exact singular vectors
    of a dense SVD returns each singular value, for any positive scaling of
    u and v."""
    rng = np.random.default_rng(7)
    n = 40
    B = random_sparse(n, 0.15, rng)
    U, s, Vt = np.linalg.svd(B.toarray())
    I = sp.identity(n, format="csr")
    for k in range(n):
        a, b = rng.uniform(0.1, 10, 2)
        sig = oracle.rayleigh_sigma(B, I, I, a * U[:, k], b * Vt[k])
        assert abs(sig - s[k]) <= 1e-13 * s[0], (k, sig, s[k])


def test_sigma_exact_for_generalized_pairs():
    """M, N SPD: the generalized triplets B v = s M u, B^T u = s N v come from
    the SVD of L_M^-1 B L_N^-T (u = L_M^-T u~, v = L_N^-T v~); the quotient
    returns s for each."""
    rng = np.random.default_rng(8)
    n = 36
    B, M, N = random_sparse(n, 0.12, rng), random_spd(n, rng), random_spd(n, rng)
    LM, LN = np.linalg.cholesky(M.toarray()), np.linalg.cholesky(N.toarray())
    Bt = np.linalg.solve(LN, np.linalg.solve(LM, B.toarray()).T).T  # L_M^-1 B L_N^-T
    Ut, s, Vtt = np.linalg.svd(Bt)
    for k in range(n):
        u = np.linalg.solve(LM.T, Ut[:, k])
        v = np.linalg.solve(LN.T, Vtt[k])
        assert np.allclose(B @ v, s[k] * (M @ u), atol=1e-11 * s[0])
        sig = oracle.rayleigh_sigma(B, M, N, 2.5 * u, 0.3 * v)
        assert abs(sig - s[k]) <= 1e-13 * s[0], (k, sig, s[k])


def test_sigma_of_coarsest_triplets_is_their_value():
    """The oracle's coarsest-level triplets (from its generalized SVD) give
    back their own sigma through the quotient (the last setup step before
    interpolation back up)."""
    ch = chaingen.tandem(14, 11 / 31, 10 / 31, 10 / 31)
    h = oracle.Hierarchy(ch, oracle.options_for(ch, r=6, max_levels=2, coarse_max=1,
                                                setup_cycles=1))
    L = h.levels - 1
    # sigma is refreshed by the level-0 post-relaxation; recompute the
    # coarsest triplets from the stored coarse operators instead
    B, M, N = h.scipy(L, "B"), h.scipy(L, "M"), h.scipy(L, "N")
    s, U, V = oracle.gsvd(B.toarray(), M.toarray(), N.toarray())
    for k in range(6):
        sig = oracle.rayleigh_sigma(B, M, N, U[:, k], V[:, k])
        assert abs(abs(sig) - s[k]) <= 1e-12 * max(s.max(), 1.0), (k, sig, s[k])
