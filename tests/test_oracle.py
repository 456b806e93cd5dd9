"""Pins of the FP64 CPU oracle against things other than itself: library
routines (numpy, scipy), closed forms, dense solves on small chains, brute
force and the invariants the paper states. No GPU needed."""
import json
import os

import numpy as np
import pytest
import scipy.linalg as sl
import scipy.sparse as sp

import chaingen
import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def dense_null(ch):
    """Stationary vector by a dense solve: one row of B replaced by 1^T."""
    A = ch.to_scipy().toarray()
    B = np.eye(ch.n) - A
    M = B.copy()
    M[0, :] = 1.0
    rhs = np.zeros(ch.n)
    rhs[0] = 1.0
    x = np.linalg.solve(M, rhs)
    x = x + np.linalg.solve(M, rhs - M @ x)  # one refinement step
    return x / x.sum()


def rel_l1(x, y):
    return np.abs(x - y).sum() / np.abs(y).sum()


# ----------------------------------------------------------- generators
def test_tandem_generator_shape_and_stochastic():
    for N in (5, 14, 33):
        ch = chaingen.tandem(N, 11 / 31, 10 / 31, 10 / 31)
        A = ch.to_scipy()
        assert ch.n == N * N
        assert np.allclose(np.asarray(A.sum(axis=0)).ravel(), 1.0, atol=1e-15)
        assert (A.data >= 0).all()
        B = sp.eye(ch.n) - A
        B = sp.csr_matrix(B)
        B.sum_duplicates()
        # diagonal + three moves: nnz(B) = (2N-1)^2
        pattern = (abs(A) + sp.eye(ch.n)).tocsr()
        assert pattern.nnz == (2 * N - 1) ** 2


def test_delaunay_generator_euler_and_closed_form():
    ch = chaingen.delaunay_walk(2000, 3)
    A = ch.to_scipy()
    assert np.allclose(np.asarray(A.sum(axis=0)).ravel(), 1.0, atol=1e-14)
    E, h = ch.extra["edges"], ch.extra["hull"]
    assert E == 3 * ch.n - 3 - h  # Euler's formula for a triangulation
    deg = ch.extra["deg"]
    pi = deg / deg.sum()
    assert np.abs(A @ pi - pi).max() < 1e-15


def test_birth_death_closed_form():
    ch = chaingen.birth_death(40, 0.96)
    x = dense_null(ch)
    i = np.arange(40)
    pi = 0.96 ** (-i)
    pi /= pi.sum()
    assert rel_l1(x, pi) < 1e-13


# ---------------------------------------------------------------- Philox
def test_philox_matches_numpy():
    rng = np.random.default_rng(1)
    for _ in range(20):
        ctr = rng.integers(0, 2**63, size=4, dtype=np.uint64)
        key = rng.integers(0, 2**63, size=2, dtype=np.uint64)
        bg = np.random.Philox(key=key, counter=ctr)
        ref = bg.random_raw(4)  # numpy steps the counter before its first block
        c1 = ctr.copy()
        c1[0] += np.uint64(1)
        assert (oracle.philox4x64(c1, key) == ref).all()


def test_uniform_pm1_from_top_bits():
    for seed, side, k, i in [(14024001, 0, 3, 17), (5, 1, 0, 1), (2**40 + 7, 1, 7, 262143)]:
        # numpy's Philox-4x64-10 with the counter one step back yields block (i, k, side, 0)
        bg = np.random.Philox(key=np.array([seed, 0], np.uint64),
                              counter=np.array([i - 1, k, side, 0], np.uint64))
        w = int(bg.random_raw(1)[0])
        u = oracle.uniform_pm1(seed, side, k, i)
        assert u == 2.0 * (w >> 11) / 2.0**53 - 1.0
        assert -1.0 <= u < 1.0


# ------------------------------------------------------------ LS fits
def test_ls_row_planted_and_lstsq():
    rng = np.random.default_rng(2)
    for r, m in [(8, 4), (6, 3), (8, 1), (6, 2)]:
        G = rng.standard_normal((r, m))
        p_true = rng.standard_normal(m)
        w = rng.uniform(0.1, 1.0, r)
        p = oracle.ls_row(G, G @ p_true, w)
        assert np.allclose(p, p_true, atol=1e-12)
        g = rng.standard_normal(r)
        ref = np.linalg.lstsq(np.sqrt(w)[:, None] * G, np.sqrt(w) * g, rcond=None)[0]
        assert np.allclose(oracle.ls_row(G, g, w), ref, atol=1e-12)


def test_ls_row_sum1_planted_and_kkt():
    rng = np.random.default_rng(3)
    for r, m in [(8, 4), (6, 3), (8, 2)]:
        G = rng.standard_normal((r, m))
        q_true = rng.standard_normal(m)
        q_true /= q_true.sum()
        w = rng.uniform(0.1, 1.0, r)
        q = oracle.ls_row_sum1(G, G @ q_true, w)
        assert np.allclose(q, q_true, atol=1e-11)
        # KKT of min sum_{k>=1} w_k (g_k - G_k q)^2 s.t. 1^T q = 1
        g = rng.standard_normal(r)
        Gw = np.sqrt(w[1:])[:, None] * G[1:]
        gw = np.sqrt(w[1:]) * g[1:]
        K = np.zeros((m + 1, m + 1))
        K[:m, :m] = Gw.T @ Gw
        K[:m, m] = 1
        K[m, :m] = 1
        rhs = np.concatenate([Gw.T @ gw, [1.0]])
        ref = np.linalg.solve(K, rhs)[:m]
        assert np.allclose(oracle.ls_row_sum1(G, g, w), ref, atol=1e-10)
        assert abs(oracle.ls_row_sum1(G, g, w).sum() - 1) < 1e-14


def test_ls_rank_deficient_drops_column():
    rng = np.random.default_rng(4)
    G = rng.standard_normal((8, 3))
    G[:, 2] = G[:, 0]  # duplicated interpolation point
    g = G[:, 0] * 0.5 + G[:, 1] * 0.25
    p = oracle.ls_row(G, g, np.ones(8))
    assert p[2] == 0.0
    assert np.allclose(G @ p, g, atol=1e-12)


# ------------------------------------------------ dense linear algebra
def test_svd_jacobi_matches_numpy():
    rng = np.random.default_rng(5)
    B = rng.standard_normal((30, 30))
    s, U, V = oracle.svd_jacobi(B)
    assert np.allclose(np.sort(s), np.sort(np.linalg.svd(B, compute_uv=False)), rtol=1e-12)
    assert np.allclose(U @ np.diag(s) @ V.T, B, atol=1e-12)


def test_gsvd_matches_pencil_eigh():
    rng = np.random.default_rng(6)
    n = 25
    B = rng.standard_normal((n, n))
    X = rng.standard_normal((n, n))
    M = X @ X.T + n * np.eye(n)
    Y = rng.standard_normal((n, n))
    N = Y @ Y.T + n * np.eye(n)
    s, U, V = oracle.gsvd(B, M, N)
    # eq. generalized_eigenvalue: eigenvalues of ([[0,B],[B^T,0]], diag(M,N)) are +-sigma
    H = np.block([[np.zeros((n, n)), B], [B.T, np.zeros((n, n))]])
    D = sl.block_diag(M, N)
    ev = sl.eigh(H, D, eigvals_only=True)
    assert np.allclose(np.sort(ev[ev > 0]), s, rtol=1e-10)
    for k in range(n):
        assert np.linalg.norm(B @ V[:, k] - s[k] * M @ U[:, k]) < 1e-10
        assert np.linalg.norm(B.T @ U[:, k] - s[k] * N @ V[:, k]) < 1e-10
        assert abs(U[:, k] @ M @ U[:, k] - 1) < 1e-10
        assert abs(V[:, k] @ N @ V[:, k] - 1) < 1e-10


# ------------------------------------------------------------- MIS
def luby_rounds(indptr, indices, keys):
    """Parallel-rounds MIS: every undecided local maximum of the priority
    joins, its neighbours leave (a different algorithm with the same
    lexicographically-first result)."""
    n = len(indptr) - 1
    state = np.full(n, -1)
    while (state == -1).any():
        und = np.where(state == -1)[0]
        join = []
        for v in und:
            nb = indices[indptr[v]:indptr[v + 1]]
            nb = nb[state[nb] == -1]
            if all((keys[v], v) > (keys[u], u) for u in nb):
                join.append(v)
        for v in join:
            state[v] = 1
        for v in join:
            nb = indices[indptr[v]:indptr[v + 1]]
            state[nb[state[nb] == -1]] = 0
    return state


def test_mis_independent_maximal_and_equals_luby():
    ch = chaingen.delaunay_walk(600, 9)
    G = (ch.to_scipy() + ch.to_scipy().T).tocsr()
    G.setdiag(0)
    G.eliminate_zeros()
    G.sort_indices()
    seed, level = 77, 2
    cf = oracle.mis(G.indptr, G.indices, seed, level)
    for v in range(ch.n):
        nb = G.indices[G.indptr[v]:G.indptr[v + 1]]
        if cf[v] == 1:
            assert (cf[nb] == 0).all()
        else:
            assert (cf[nb] == 1).any()
    keys = np.array([int(oracle.philox4x64([i, level, 2, 0], [seed, 0])[0]) for i in range(ch.n)],
                    dtype=object)
    assert (luby_rounds(G.indptr, G.indices, keys) == cf).all()


def test_row_colouring_valid():
    ch = chaingen.tandem(12, 11 / 31, 10 / 31, 10 / 31)
    B = sp.csr_matrix(sp.eye(ch.n) - ch.to_scipy())
    B.sort_indices()
    Bt = B.T.tocsr()
    Bt.sort_indices()
    col = oracle.row_colouring(B.indptr, B.indices, Bt.indptr, Bt.indices)
    for j in range(ch.n):
        rows = Bt.indices[Bt.indptr[j]:Bt.indptr[j + 1]]
        assert len(set(col[rows])) == len(rows)


# ------------------------------------------------------- hierarchy pins
@pytest.fixture(scope="module")
def tandem14():
    ch = chaingen.tandem(14, 11 / 31, 10 / 31, 10 / 31)
    h = oracle.Hierarchy(ch, oracle.options_for(ch, r=6, coarse_max=20, setup_cycles=2))
    return ch, h


def test_geometric_coarsening_sizes(tandem14):
    ch, h = tandem14
    N = 14
    for l in range(h.levels):
        assert h.dims(l)[0] == N * N
        N = (N + 1) // 2


def test_transfer_structure_and_constraint(tandem14):
    ch, h = tandem14
    for l in range(h.levels - 1):
        cf, cidx = h.cf(l)
        P = h.scipy(l, "P")
        Qt = h.scipy(l, "Qt")
        C = np.where(cf == 1)[0]
        # eq. Pstructure: identity on coarse rows
        assert (P[C].toarray() == np.eye(len(C))[np.arange(len(C))]).all()
        # Section 5: 1^T Q = 1^T
        assert np.abs(np.asarray(Qt.sum(axis=1)).ravel() - 1).max() < 1e-13
        # R-ACT: no negative weights
        assert P.data.min() >= 0 and Qt.data.min() >= 0
        # R-Q: same pattern
        assert (P.indptr == Qt.indptr).all() and (P.indices == Qt.indices).all()


def test_galerkin_equals_dense_product(tandem14):
    ch, h = tandem14
    for l in range(h.levels - 1):
        B = h.scipy(l, "B").toarray()
        M = h.scipy(l, "M").toarray()
        N = h.scipy(l, "N").toarray()
        P = h.scipy(l, "P").toarray()
        Q = h.scipy(l, "Q").toarray()
        assert np.allclose(Q, h.scipy(l, "Qt").toarray().T, atol=0)
        Bc = h.scipy(l + 1, "B").toarray()
        scale = np.abs(B).max()
        assert np.abs(Bc - Q @ B @ P).max() < 1e-13 * scale * max(1, np.abs(P).max()) * 10
        assert np.allclose(h.scipy(l + 1, "M").toarray(), Q @ M @ Q.T, atol=1e-12)
        assert np.allclose(h.scipy(l + 1, "N").toarray(), P.T @ N @ P, atol=1e-12)
        # Section 5: the column sums of the coarse operator stay zero
        assert np.abs(Bc.sum(axis=0)).max() < 1e-13 * np.abs(Bc).max()
        Mc = h.scipy(l + 1, "M").toarray()
        assert np.allclose(Mc, Mc.T) and np.linalg.eigvalsh(Mc).min() > 0


def test_coarse_pinv_matches_numpy(tandem14):
    ch, h = tandem14
    L = h.levels - 1
    BL = h.scipy(L, "B").toarray()
    assert np.allclose(h.coarse_pinv(), np.linalg.pinv(BL, rcond=1e-10), atol=1e-9 * np.abs(np.linalg.pinv(BL)).max())


def test_smoother_fixed_point(tandem14):
    ch, h = tandem14
    rng = np.random.default_rng(7)
    for l in range(h.levels - 1):
        B = h.scipy(l, "B")
        xs = rng.standard_normal(B.shape[0])
        b = B @ xs
        assert np.allclose(h.smooth(l, b, xs), xs, atol=1e-13)
        # one sweep from another point moves toward the fixed point in the B-residual sense
        x1 = h.smooth(l, b, np.zeros_like(xs))
        assert np.allclose(x1, 0.7 * b / B.diagonal(), atol=1e-15)


def test_kaczmarz_sweep_is_a_sequence_of_projections():
    # Section 3 lists Kaczmarz relaxation: each row update is the orthogonal
    # projection onto {x : B_i x = b_i}. On a consistent system this makes
    # ||x - x*|| non-increasing for every solution x*, leaves the rows of the
    # last colour exactly satisfied (later rows of that colour touch other
    # columns only), and repeated sweeps converge to a solution.
    ch = chaingen.tandem(12, 11 / 31, 10 / 31, 10 / 31)
    h = oracle.Hierarchy(ch, oracle.options_for(ch, r=6, max_levels=2, coarse_max=1,
                                                smoother="kaczmarz"))
    B = sp.csr_matrix(sp.eye(ch.n) - ch.to_scipy())
    B.sort_indices()
    Bt = B.T.tocsr()
    Bt.sort_indices()
    col = oracle.row_colouring(B.indptr, B.indices, Bt.indptr, Bt.indices)
    last = col == col.max()
    rng = np.random.default_rng(3)
    xs = rng.standard_normal(ch.n)
    b = B @ xs
    x = rng.standard_normal(ch.n)
    err = [np.linalg.norm(x - xs)]
    for _ in range(400):
        x = h.smooth(0, b, x)
        err.append(np.linalg.norm(x - xs))
        r = b - B @ x
        assert np.abs(r[last]).max() < 1e-12 * max(1.0, np.abs(b).max())
    err = np.array(err)
    assert np.all(np.diff(err) <= 1e-12 * err[0])
    # approaching the solution set {xs + t x_null} (Kaczmarz converges slowly)
    assert np.linalg.norm(b - B @ x) < 1e-3 * np.linalg.norm(b)


def test_two_grid_propagator_formula():
    """V-cycle with two levels and an exact coarse solve: I - C B equals
    S^nu2 (I - P B_c^+ Q B) S^nu1 (eq. error_propagator_twogrid; pre-smoothing
    acts first)."""
    ch = chaingen.tandem(9, 11 / 31, 10 / 31, 10 / 31)
    h = oracle.Hierarchy(ch, oracle.options_for(ch, r=6, max_levels=2, coarse_max=1, nu_pre=2, nu_post=3))
    n = ch.n
    B = h.scipy(0, "B").toarray()
    P = h.scipy(0, "P").toarray()
    Q = h.scipy(0, "Q").toarray()
    Bc = h.scipy(1, "B").toarray()
    S = np.eye(n) - 0.7 * B / np.diag(B)[:, None]
    E = np.linalg.matrix_power(S, 3) @ (np.eye(n) - P @ np.linalg.pinv(Bc, rcond=1e-10) @ Q @ B) @ np.linalg.matrix_power(S, 2)
    C = np.column_stack([h.vcycle(e) for e in np.eye(n)])
    assert np.abs((np.eye(n) - C @ B) - E).max() < 1e-10


def test_singular_vectors_approximate_smallest_triplets():
    ch = chaingen.delaunay_walk(700, 11)
    h = oracle.Hierarchy(ch, oracle.options_for(ch, r=8, max_interp=3, nu_pre=5, nu_post=5, nu_setup=5,
                                                coarse_max=200, setup_cycles=2))
    B = np.eye(ch.n) - ch.to_scipy().toarray()
    true = np.linalg.svd(B, compute_uv=False)[::-1][:8]
    s = np.sort(np.abs(h.sigma()))
    assert abs(s[0]) < 1e-12
    assert np.allclose(s[1:], true[1:], rtol=0.1)
    U, V = h.vectors(0)
    for k in range(1, 8):
        sk = h.sigma()[k]
        assert np.linalg.norm(B @ V[:, k] - sk * U[:, k]) < 0.02
        assert np.linalg.norm(B.T @ U[:, k] - sk * V[:, k]) < 0.02


# ------------------------------------------------------- end-to-end pins
@pytest.mark.parametrize("cycles", [1, 2])
@pytest.mark.parametrize("levels", [2, 3])
def test_tandem_against_dense_null_space(cycles, levels):
    ch = chaingen.tandem(14, 11 / 31, 10 / 31, 10 / 31)  # 196 states
    h = oracle.Hierarchy(ch, oracle.options_for(ch, r=6, max_levels=levels, coarse_max=1, setup_cycles=cycles))
    x, info = h.gmres(m=20, tol=1e-14, maxit=300)
    assert info.converged
    xe = dense_null(ch)
    assert rel_l1(x, xe) < 1e-10
    assert x.min() > 0 and abs(x.sum() - 1) < 1e-14


def test_delaunay_closed_form():
    ch = chaingen.delaunay_walk(3000, 12)
    h = oracle.Hierarchy(ch, oracle.options_for(ch, r=8, max_interp=3, nu_pre=5, nu_post=5, nu_setup=5,
                                                coarse_max=500))
    x, info = h.gmres(m=20, tol=1e-14, maxit=300)
    deg = ch.extra["deg"]
    assert rel_l1(x, deg / deg.sum()) < 1e-10
    assert info.iterations < 40


def test_hub_walk_closed_form():
    """A random walk with a few high-degree hubs (long rows on every level):
    the method still reaches pi proportional to the degree."""
    ch = chaingen.hub_walk(600, 3, 80, 5)
    h = oracle.Hierarchy(ch, oracle.options_for(ch, r=8, max_interp=3, nu_pre=5, nu_post=5,
                                                nu_setup=5, coarse_max=60))
    x, info = h.gmres(m=20, tol=1e-14, maxit=300)
    deg = ch.extra["deg"]
    assert info.converged
    assert rel_l1(x, deg / deg.sum()) < 1e-10


def test_birth_death_closed_form_method():
    n = 257
    ch = chaingen.birth_death(n, 0.96)
    h = oracle.Hierarchy(ch, oracle.options_for(ch, r=8, max_interp=2, coarse_max=29))
    x, info = h.gmres(m=20, tol=1e-14, maxit=300)
    pi = 0.96 ** (-np.arange(n))
    assert rel_l1(x, pi / pi.sum()) < 1e-10


def test_unpreconditioned_gmres_reaches_null_vector():
    """Theorem 1: GMRES on the consistent singular system converges to the
    null-space component of x0; after scaling that is the stationary vector."""
    ch = chaingen.tandem(8, 11 / 31, 10 / 31, 10 / 31)
    h = oracle.Hierarchy(ch, oracle.options_for(ch, r=6, max_levels=2, coarse_max=1))
    x, info = h.gmres(m=50, tol=1e-12, maxit=3000, precondition=False)
    assert info.converged
    assert rel_l1(x, dense_null(ch)) < 1e-9


def test_iteration_counts_near_paper_table3():
    data = json.load(open(os.path.join(GOLDEN, "paper_tables.json")))
    tab = data["table3_tandem"]
    ch = chaingen.tandem(33, 11 / 31, 10 / 31, 10 / 31)
    for cyc, key in ((1, "bamg"), (2, "bamg2")):
        h = oracle.Hierarchy(ch, oracle.options_for(ch, r=8, coarse_max=289, setup_cycles=cyc))
        x, info = h.gmres(m=20, tol=data["tol"], maxit=200)
        # loose: randomness and unstated details (parity of counts is unpinned)
        assert info.iterations <= tab[key][0] + 6


def test_error_paths():
    ch = chaingen.tandem(6, 11 / 31, 10 / 31, 10 / 31)
    bad = chaingen.Chain(ch.to_scipy() * 1.01, ch.geom)
    with pytest.raises(oracle.OracleError) as e:
        oracle.Hierarchy(bad, oracle.options_for(ch, r=6, max_levels=2, coarse_max=1))
    assert e.value.code == -2
    # two disconnected cycles -> reducible
    A = sp.lil_matrix((6, 6))
    for i in range(3):
        A[(i + 1) % 3, i] = 1.0
        A[3 + (i + 1) % 3, 3 + i] = 1.0
    with pytest.raises(oracle.OracleError) as e:
        oracle.Hierarchy(chaingen.Chain(A.tocsr()), oracle.default_options(r=2, coarsening=1, coarse_max=1, max_levels=2))
    assert e.value.code == -3
    h = oracle.Hierarchy(ch, oracle.options_for(ch, r=6, max_levels=2, coarse_max=1))
    x, info = h.gmres(m=5, tol=1e-30, maxit=1)
    assert info.converged == 0 and info.iterations == 1
