"""Pins for the CPU oracle (runs without a GPU).

The oracle is only trusted because these tests tie it to facts that do not
come from the oracle itself: closed forms, identities stated in the paper,
printed worked values (tests/golden), LAPACK on small inputs, calculus and
finite differences.  test_mutants.py shows that plausible mistakes planted in
a copy of the oracle fail at least one of these pins.
"""
import math

import numpy as np
import pytest

import workloads as wl
from conftest import golden

U_D = 2.0 ** -53
U_L = 2.0 ** -24


# ----------------------------------------------------------------- rotation
@pytest.mark.parametrize("a,b,d,expect", [
    (2.0, 1.0, 2.0, (1.0, 3.0)),      # tau = 0 -> t = 1, theta = pi/4
    (0.0, 1.0, 0.0, (-1.0, 1.0)),
])
def test_pair_closed_form_textbook(orc, a, b, d, expect):
    """Section 3.1: J^T [[a,b],[b,d]] J is diagonal, eigenvalues from the
    quadratic formula."""
    c, s = orc.jacobi_pair(a, d, b)
    J = np.array([[c, s], [-s, c]])
    B = J.T @ np.array([[a, b], [b, d]]) @ J
    assert abs(B[0, 1]) < 1e-15 and abs(B[1, 0]) < 1e-15
    assert sorted([B[0, 0], B[1, 1]]) == pytest.approx(expect, abs=1e-15)
    if (a, b, d) == (2.0, 1.0, 2.0):
        # V = [1 1; -1 1]/sqrt(2): t = 1 exactly
        assert c == pytest.approx(1 / math.sqrt(2), abs=1e-16)
        assert s == pytest.approx(1 / math.sqrt(2), abs=1e-16)


def test_pair_random_2x2(orc):
    g = np.random.default_rng(11)
    for _ in range(200):
        a, b, d = g.standard_normal(3) * 10.0 ** g.integers(-3, 4, 3)
        c, s = orc.jacobi_pair(a, d, b)
        t = s / c
        assert abs(t) <= 1.0 + 1e-15                       # smaller root
        assert c * c + s * s == pytest.approx(1.0, abs=1e-15)
        # t solves t^2 + 2 tau t - 1 = 0 with tau = (d - a)/(2 b)
        # b_pp = a - t b, b_qq = d + t b (rotated diagonal)
        disc = math.sqrt(((a - d) / 2) ** 2 + b * b)
        lo, hi = (a + d) / 2 - disc, (a + d) / 2 + disc
        got = sorted([a - t * b, d + t * b])
        scale = max(abs(a), abs(b), abs(d))
        assert got[0] == pytest.approx(lo, abs=8e-16 * scale)
        assert got[1] == pytest.approx(hi, abs=8e-16 * scale)
        # the pair is annihilated (the 2x2 subproblem of Section 3.1)
        bpq = c * s * (a - d) + (c * c - s * s) * b
        assert abs(bpq) <= 4e-16 * scale


def test_pair_zero_coupling(orc):
    assert orc.jacobi_pair(1.0, -3.0, 0.0) == (1.0, 0.0)


def test_small_angle_appendix_a(orc):
    """Appendix A: approach 2 keeps s != 0 for a_pq ~ 1e-14 where
    approach 1 (t = -tau + sqrt(tau^2 + 1)) collapses to s = 0."""
    app, aqq, apq = 1.0, 2.0, 1e-14
    tau = (aqq - app) / (2 * apq)
    t1 = -tau + math.sqrt(tau * tau + 1.0)
    assert t1 == 0.0                                      # approach 1 fails
    c, s = orc.jacobi_pair(app, aqq, apq)
    assert s != 0.0
    assert s == pytest.approx(apq / (aqq - app), rel=1e-12)
    A = np.array([[app, apq], [apq, aqq]])
    B, _ = orc.rotate(A, None, 0, 1, c, s)
    assert abs(B[0, 1]) < 1e-28


def test_rotation_off_identity(orc):
    """Section 3.1: off(B)^2 = off(A)^2 - 2 a_pq^2; only rows/cols p, q move
    (Section 2.2.1)."""
    A = wl.random_symmetric(12, 5)
    for (p, q) in [(0, 1), (3, 9), (10, 11), (2, 7)]:
        c, s = orc.jacobi_pair(A[p, p], A[q, q], A[p, q])
        V = np.eye(12)
        B, V2 = orc.rotate(A, V, p, q, c, s)
        lhs = orc.off(B) ** 2
        rhs = orc.off(A) ** 2 - 2 * A[p, q] ** 2
        assert lhs == pytest.approx(rhs, rel=1e-13)
        assert abs(B[p, q]) < 1e-14 and abs(B[q, p]) < 1e-14
        keep = [k for k in range(12) if k not in (p, q)]
        assert np.array_equal(B[np.ix_(keep, keep)], A[np.ix_(keep, keep)])
        assert np.allclose(V2.T @ V2, np.eye(12), atol=1e-15)
        assert np.allclose(V2.T @ A @ V2, B, atol=1e-14)


# ------------------------------------------------------------- whole solve
def test_edge_sizes(orc):
    W, V, sw, st, _ = orc.eigh(np.zeros((0, 0)))
    assert W.shape == (0,) and st == 0
    W, V, sw, st, _ = orc.eigh(np.array([[-2.5]]))
    assert W[0] == -2.5 and V[0, 0] == 1.0 and sw == 0


def test_diagonal_input(orc):
    d = np.array([3.0, -1.0, 2.0, 0.5, -7.0])
    W, V, sw, st, _ = orc.eigh(np.diag(d))
    assert sw == 0 and st == 0
    assert np.array_equal(W, np.sort(d))
    P = np.zeros((5, 5))
    for c, i in enumerate(np.argsort(d, kind="stable")):
        P[i, c] = 1.0
    assert np.array_equal(V, P)


def test_known_spectrum(orc):
    A, lam = wl.uniform_spectrum(64, 1)
    W, V, sw, st, _ = orc.eigh(A)
    n = 64
    nrm2 = np.abs(lam).max()                   # ||A||_2 = max |lambda|
    assert st == 0
    assert np.abs(W - lam).max() <= 10 * n * U_D * nrm2
    assert np.linalg.norm(A @ V - V * W) / np.linalg.norm(A) <= 10 * n * U_D
    # orthogonality: the tolerance of the solver's contract, 1e-14 n
    assert np.linalg.norm(V.T @ V - np.eye(n)) <= 1e-14 * n


def test_known_spectrum_ari(orc):
    """The arithmetic family: eigenvalues known by construction, well
    separated (gap ~ 2 / n), so the oracle converges quadratically in few
    sweeps (Section 5.2 observes two to three for this family)."""
    n = 64
    A, lam = wl.ari_spectrum(n, 6, kappa=1e2)
    assert abs(np.abs(lam).max() - 1.0) < 1e-15 and abs(np.abs(lam).min() - 1e-2) < 1e-15
    W, V, sw, st, _ = orc.eigh(A)
    nrm2 = np.abs(lam).max()
    assert st == 0
    assert np.abs(W - lam).max() <= 10 * n * U_D * nrm2
    assert np.linalg.norm(A @ V - V * W) / np.linalg.norm(A) <= 10 * n * U_D
    assert sw <= 8


def test_block_diagonal_workload(orc):
    """The decoupled-blocks input: no coupling between its diagonal blocks,
    and the oracle on the whole matrix returns the union of the spectra the
    blocks were built from."""
    sizes = [20, 13, 31]
    A, lam = wl.block_diagonal(64, sizes=sizes, seed=21)
    o = 0
    for m in sizes:
        assert not A[o:o + m, o + m:].any() and not A[o + m:, o:o + m].any()
        o += m
    W, V, sw, st, _ = orc.eigh(A)
    assert st == 0
    assert np.abs(W - lam).max() <= 10 * 64 * U_D * np.abs(lam).max()


@pytest.mark.parametrize("n,seed", [(7, 1), (30, 2), (64, 3)])
def test_invariants(orc, n, seed):
    """Orthogonal invariance (Section 2.2): trace and Frobenius norm."""
    A = wl.random_symmetric(n, seed)
    W, V, *_ = orc.eigh(A)
    assert W.sum() == pytest.approx(np.trace(A), abs=1e-13 * np.abs(A).sum())
    assert (W ** 2).sum() == pytest.approx((A ** 2).sum(), rel=1e-13)


@pytest.mark.parametrize("n", [2, 3, 5, 8, 16, 33, 64])
def test_brute_force_vs_lapack(orc, n):
    A = wl.random_symmetric(n, 100 + n)
    W, V, *_ = orc.eigh(A)
    Wl, Vl = np.linalg.eigh(A)
    nrm2 = np.abs(Wl).max()
    assert np.abs(W - Wl).max() <= 1e-13 * nrm2
    # eigenvectors agree up to sign where the gap is comfortable
    gaps = np.diff(Wl)
    for k in range(n):
        gap = min(gaps[k - 1] if k > 0 else np.inf,
                  gaps[k] if k < n - 1 else np.inf)
        if gap > 1e-6 * nrm2:
            assert abs(abs(V[:, k] @ Vl[:, k]) - 1.0) < 1e-9
    # sign convention: largest |entry| of each column is positive
    idx = np.argmax(np.abs(V), axis=0)
    assert (V[idx, np.arange(n)] > 0).all()


def test_residual_scale_paper_fixture(orc):
    """Section 3.3 test: n=100, A = randn + randn', tol = 2^-53 (per pair).
    The paper's residual sits at about twice n u_d ||A||_2; a correct solver
    on the same family lands at that scale, not orders of magnitude away."""
    fx = golden("cyclic_residual_n100.txt")
    fc = golden("classical_residual_n100.txt")
    ratio_paper = fx["residual"] / fx["reference"]
    assert 1.0 < ratio_paper < 2.0 and fc["residual"] / fc["reference"] < 2.0
    g = np.random.default_rng(1)
    n = int(fx["n"])
    for trial in range(3):
        G = g.standard_normal((n, n))
        A = G + G.T
        A_fin, V, sw, st, _, _ = orc.jacobi_cyclic(A, tol_abs=0.0,
                                                   rel_eps=U_D)
        D = np.diag(np.diag(A_fin))
        res = np.linalg.norm(A @ V - V @ D, 2)
        ref = n * U_D * np.linalg.norm(A, 2)
        assert st == 0
        assert res / ref < 5 * ratio_paper


def test_householder_fixture():
    """Section 2.2.2 worked example: the generator's Householder QR maps x to
    +-||x|| e_1 with ||x|| = 3.4748."""
    fx = golden("householder_example.txt")
    x = np.array(fx["x"]).reshape(5, 1)
    Q, R = np.linalg.qr(x, mode="complete")
    assert abs(R[0, 0]) == pytest.approx(fx["Px0"], abs=1e-4)  # inputs carry 5 digits
    Px = Q.T @ x
    assert np.abs(Px[1:]).max() < 1e-15


def test_haar_generator_orthogonal():
    Q = wl.haar(50, wl.rng(0))
    assert np.linalg.norm(Q.T @ Q - np.eye(50)) < 1e-13


# -------------------------------------------------------- convergence pins
def test_quadratic_convergence(orc):
    """Section 5.2.2 (Wilkinson's bound): once off < delta/8,
    off after one more sweep <= off^2 / delta, delta = half the minimum gap."""
    n = 24
    lam = np.linspace(-1.0, 1.0, n)
    A = wl.from_spectrum(lam, wl.haar(n, wl.rng(8)))
    delta = 0.5 * np.diff(lam).min()
    *_, hist = orc.eigh(A, tol=1e-300, max_sweeps=30)
    floor = 20 * n * U_D * np.abs(lam).max()
    seen = 0
    for k in range(len(hist) - 1):
        if hist[k] < delta / 8:
            assert hist[k + 1] <= hist[k] ** 2 / delta + floor
            seen += 1
    assert seen >= 1


def test_linear_phase_decreases(orc):
    A = wl.random_symmetric(40, 9)
    *_, hist = orc.eigh(A, tol=1e-300)
    assert (np.diff(hist) < 0).all()


def test_noconv_status(orc):
    A = wl.random_symmetric(32, 4)
    W, V, sw, st, _ = orc.eigh(A, max_sweeps=1)
    assert st == 1 and sw == 1
    assert np.linalg.norm(V.T @ V - np.eye(32)) < 1e-13


# ------------------------------------------------------- Newton-Schulz pins
def _ns_scalar(d, k):
    for _ in range(k):
        d = 0.5 * d * (3.0 - d * d)
    return d


def test_newton_schulz_scalar_map(orc):
    """Section 4.3.4: with X_0 = P diag(sigma) Q^T, X_k = P diag(f^k(sigma)) Q^T,
    f(d) = d(3 - d^2)/2, and f(d) - 1 = -(d - 1)^2 (d + 2)/2."""
    n = 20
    g = wl.rng(3)
    P, Q = wl.haar(n, g), wl.haar(n, g)
    sigma = np.concatenate([[0.3, 1.6, 1.0], 1.0 + 1e-3 * g.standard_normal(n - 3)])
    X0 = (P * sigma) @ Q.T
    for k in (1, 2, 3):
        Xk = orc.newton_schulz(X0, k)
        expect = (P * _ns_scalar(sigma, k)) @ Q.T
        assert np.abs(Xk - expect).max() < 1e-14
    for d in (0.2, 0.9, 1.3, 1.7):
        got = orc.newton_schulz(np.array([[d]]), 1)[0, 0]
        assert got - 1.0 == pytest.approx(-0.5 * (d - 1) ** 2 * (d + 2), abs=1e-15)


def test_newton_schulz_polar_factor(orc):
    """The limit is the orthogonal polar factor P Q^T (best approximation,
    Section 4.3.1); two steps suffice from ||Q^T Q - I|| ~ n u_l."""
    n = 40
    g = wl.rng(4)
    P, Q = wl.haar(n, g), wl.haar(n, g)
    sigma = 1.0 + n * U_L * g.uniform(-1, 1, n)
    X0 = (P * sigma) @ Q.T
    X2 = orc.newton_schulz(X0, 2)
    assert np.linalg.norm(X2.T @ X2 - np.eye(n)) <= n * U_D
    assert np.abs(X2 - P @ Q.T).max() < 1e-14


def test_ns_iteration_count_fixture():
    """Section 4.3.4: (sqrt(1 + n u_l) - 1)^4 = n u_d crosses at n ~ 52071; the
    figure's marker is n u_d at n = 52400."""
    fx = golden("ns_iteration_count.txt")
    f = lambda n: (math.sqrt(1 + n * U_L) - 1) ** 4 - n * U_D
    lo, hi = 1e3, 1e6
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        lo, hi = (mid, hi) if f(mid) < 0 else (lo, mid)
    assert abs(lo - fx["crossover_two"]) < 60
    assert fx["marker_n"] * U_D == pytest.approx(fx["marker_value"], rel=1e-5)
    # three iterations: (sqrt(1 + n u_l) - 1)^8 = n u_d
    g3 = lambda n: (math.sqrt(1 + n * U_L) - 1) ** 8 - n * U_D
    lo, hi = 1e5, 1e8
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        lo, hi = (mid, hi) if g3(mid) < 0 else (lo, mid)
    assert abs(lo - fx["crossover_three"]) / fx["crossover_three"] < 1e-3


def test_qtaq_vs_library(orc):
    g = wl.rng(5)
    Q = g.standard_normal((17, 17))
    A = wl.random_symmetric(17, 6)
    B = orc.qtaq(Q, A)
    ref = Q.T @ A @ Q
    ref = 0.5 * (ref + ref.T)
    assert np.abs(B - ref).max() < 1e-12


# ------------------------------------------------------- mixed pipeline pins
@pytest.mark.parametrize("n,seed", [(50, 1), (120, 2)])
def test_mixed_stage_bounds(orc, n, seed):
    """Algorithm 9 with an FP32 Jacobi first stage.  Section 4.3.4:
    ||Q_d^T Q_d - I|| <= n u_d; Section 5.2.1: off(A_cond) <~ n u_l ||A||;
    Section 5.2.2: at most five FP64 sweeps; Section 5.1: the result is a
    spectral decomposition at double precision."""
    A, lam = wl.geo_spectrum(n, seed, kappa=1e3)
    nrm2 = np.abs(lam).max()
    W, Q, st, d = orc.eigh_mixed(A)
    assert st == 0 and d["status32"] == 0
    assert d["orth_ql"] <= 10 * n * U_L
    assert d["orth_qd"] <= n * U_D
    assert d["off_cond"] <= n * U_L * nrm2
    assert 1 <= d["sweeps64"] <= 5
    assert np.abs(W - lam).max() <= 1e-13 * nrm2
    assert np.linalg.norm(A @ Q - Q * W) / np.linalg.norm(A) <= 1e-13 * n
    assert np.linalg.norm(Q.T @ Q - np.eye(n)) <= 1e-14 * n
    # the same answer as the plain solver
    W2, *_ = orc.eigh(A)
    assert np.abs(W - W2).max() <= 1e-13 * nrm2


# -------------------------------------------------------------- adjoint pins
def _loss_parts(orc, A, w, C):
    W, V, *_ = orc.eigh(A, tol=1e-300)
    return float(w @ W + (C * V).sum())


def test_backward_trace_identity(orc):
    """d(sum lambda)/dA = d(tr A)/dA = I."""
    A, lam = wl.uniform_spectrum(12, 9)
    W, V, *_ = orc.eigh(A)
    dA, st = orc.eigh_backward(W, V, dW=np.ones(12))
    assert st == 0
    assert np.abs(dA - np.eye(12)).max() < 1e-14


def test_backward_frobenius_identity(orc):
    """d(sum lambda^2)/dA = d(||A||_F^2)/dA = 2A."""
    A, lam = wl.uniform_spectrum(12, 10)
    W, V, *_ = orc.eigh(A)
    dA, st = orc.eigh_backward(W, V, dW=2 * W)
    assert np.abs(dA - 2 * A).max() < 1e-14


def test_backward_central_fd(orc):
    """loss = sum w_i lambda_i + <C, V> (sign-fixed V): the adjoint matches
    central differences (h = 1e-6) along random symmetric directions."""
    n = 8
    lam = np.sort(wl.rng(1).uniform(-1, 1, n)) + np.arange(n) * 0.05
    A = wl.from_spectrum(lam, wl.haar(n, wl.rng(2)))
    g = wl.rng(3)
    w = g.standard_normal(n)
    C = g.standard_normal((n, n))
    W, V, *_ = orc.eigh(A, tol=1e-300)
    dA, st = orc.eigh_backward(W, V, dW=w, dV=C)
    assert st == 0
    # the gradient with respect to a symmetric A is itself symmetric
    assert np.abs(dA - dA.T).max() < 1e-14
    h = 1e-6
    for k in range(4):
        E = g.standard_normal((n, n))
        E = 0.5 * (E + E.T)
        fd = (_loss_parts(orc, A + h * E, w, C) -
              _loss_parts(orc, A - h * E, w, C)) / (2 * h)
        assert (dA * E).sum() == pytest.approx(fd, rel=1e-6, abs=1e-8)


def test_backward_degenerate_status(orc):
    W = np.array([1.0, 1.0, 2.0])
    V = np.eye(3)
    dV = np.ones((3, 3))
    dA, st = orc.eigh_backward(W, V, dV=dV, gap_tol=1e-12)
    assert st == 4
    assert np.isfinite(dA).all()


# ------------------------------------------------- one-sweep sample (timing)
@pytest.mark.parametrize("n,seed", [(9, 31), (40, 32)])
def test_jacobi_rows_is_one_sweep(orc, n, seed):
    """orc_jacobi_rows over every pivot row [0, n-1) is one cyclic-by-row
    sweep of Algorithm 4 without its end-of-sweep symmetrisation: after
    (A + A^T)/2 it equals, bit for bit, the oracle's first sweep (same
    rotations, same order), and V matches bit for bit.  A split into two row
    ranges gives the same bits (a bounded sample is a prefix of a sweep)."""
    A = wl.random_symmetric(n, seed)
    A1, V1, sweeps, _, _, rot1 = orc.jacobi_cyclic(A, 0.0, max_sweeps=1)
    assert sweeps == 1
    A2 = np.ascontiguousarray(A.copy())
    V2 = np.eye(n)
    rot2 = orc.jacobi_rows(A2, V2, 0, n - 1)
    A3 = np.ascontiguousarray(A.copy())
    V3 = np.eye(n)
    rot3 = orc.jacobi_rows(A3, V3, 0, n // 2) + orc.jacobi_rows(A3, V3, n // 2, n - 1)
    assert rot2 == rot1 == rot3 == n * (n - 1) // 2
    sym = 0.5 * (A2 + A2.T)
    assert np.array_equal(sym, A1)
    assert np.array_equal(V2, V1)
    assert np.array_equal(A3, A2) and np.array_equal(V3, V2)


# --------------------------------------------------- Rayleigh quotient check
def test_rayleigh_exact_eigenvectors(orc):
    """For an eigenvector of a diagonal matrix the quotient is the diagonal
    entry exactly and the residual is zero; for A = Q diag(lam) Q^T with a
    Haar Q the quotients of Q's columns are lam to rounding."""
    d = np.array([3.0, -1.5, 0.25, 7.0, 0.0])
    rq, res = orc.rayleigh(np.diag(d), np.eye(5))
    assert np.array_equal(rq, d) and np.array_equal(res, np.zeros(5))
    g = wl.rng(41)
    Q = wl.haar(24, g)
    lam = np.linspace(-2.0, 3.0, 24)
    A = wl.from_spectrum(lam, Q)
    rq, res = orc.rayleigh(A, Q)
    assert np.abs(rq - lam).max() <= 24 * U_D * 3.0
    assert res.max() <= 24 * U_D * 3.0


def test_rayleigh_quadratic_and_scale_free(orc):
    """The quotient of a perturbed eigenvector v + e w (w orthogonal to v)
    is lambda + e^2 (w^T A w - lambda) / (1 + e^2) exactly (a quadratic
    error, the property that makes it a sharp eigenvalue check), it does not
    change when the vector is scaled, and the residual of the perturbed
    vector is e ||(A - rq) w|| / sqrt(1 + e^2) to first order."""
    g = wl.rng(42)
    n = 16
    Q = wl.haar(n, g)
    lam = np.arange(1.0, n + 1.0)
    A = wl.from_spectrum(lam, Q)
    v, w = Q[:, 3], Q[:, 9]
    for e in (1e-2, 1e-4):
        x = v + e * w
        V = np.zeros((n, n))
        V[:, 0] = x
        V[:, 1] = 3.0 * x
        V[:, 2] = v
        rq, res = orc.rayleigh(A, V)
        expect = (lam[3] + e * e * lam[9]) / (1.0 + e * e)
        assert rq[0] == pytest.approx(expect, abs=1e-13)
        assert rq[1] == pytest.approx(rq[0], abs=1e-14)
        assert abs(rq[0] - lam[3]) == pytest.approx(e * e * (lam[9] - lam[3]), rel=1e-3)
        assert res[0] == pytest.approx(e * (lam[9] - lam[3]) / math.sqrt(1 + e * e), rel=1e-3)
        assert res[1] == pytest.approx(res[0], rel=1e-12)
        assert rq[2] == pytest.approx(lam[3], abs=1e-13)


def test_rayleigh_vs_library(orc):
    """Random symmetric A and random (non-normalized) vectors: the quotients
    and residuals equal the numpy evaluation of the same formulas."""
    g = wl.rng(43)
    n = 33
    A = wl.random_symmetric(n, 44)
    V = g.standard_normal((n, n))
    rq, res = orc.rayleigh(A, V)
    AV = A @ V
    q = np.einsum("ij,ij->j", V, AV) / np.einsum("ij,ij->j", V, V)
    r = np.linalg.norm(AV - V * q, axis=0) / np.linalg.norm(V, axis=0)
    assert np.allclose(rq, q, rtol=0, atol=1e-12 * np.abs(q).max())
    assert np.allclose(res, r, rtol=1e-10, atol=0)


# ------------------------------------------ orthogonalisers (QR comparators)
def test_house_worked_example(orc):
    """Section 2.2.2 worked example, through the oracle's Algorithm 1: x < 0 in
    its first entry, so P x = +||x|| e_1 = 3.4748 e_1 (printed to five
    digits) and the other entries vanish to rounding (printed as 0 and
    ~1e-16); beta = 2 / (v^T v) makes P orthogonal."""
    fx = golden("householder_example.txt")
    x = np.array(fx["x"])
    v, beta = orc.house(x)
    P = np.eye(5) - beta * np.outer(v, v)
    Px = P @ x
    assert Px[0] == pytest.approx(fx["Px0"], abs=1e-4)
    assert Px[0] == pytest.approx(np.linalg.norm(x), rel=1e-15)
    assert np.abs(Px[1:]).max() < 1e-15
    assert np.abs(P.T @ P - np.eye(5)).max() < 1e-15
    # x_1 >= 0: P x = -||x|| e_1, and v_1 = x_1 + ||x|| (no cancellation)
    v2, b2 = orc.house(-x)
    assert (np.eye(5) - b2 * np.outer(v2, v2)) @ (-x) == pytest.approx(
        [-np.linalg.norm(x), 0, 0, 0, 0], abs=1e-15)
    assert v2[0] == pytest.approx(1.3499 + np.linalg.norm(x), rel=1e-15)
    # cancellation branch: x close to a positive multiple of e_1
    v3, b3 = orc.house(np.array([-1.0, 1e-9, 0.0]))
    assert v3[0] == pytest.approx(-1.0 - math.sqrt(1.0 + 1e-18), rel=1e-15)
    v4, b4 = orc.house(np.array([1.0, 1e-9, 0.0]))
    y = (np.eye(3) - b4 * np.outer(v4, v4)) @ np.array([1.0, 1e-9, 0.0])
    assert y[0] == pytest.approx(-1.0, rel=1e-15) and abs(y[1]) < 1e-24


@pytest.mark.parametrize("n", [2, 7, 40])
def test_householder_qr_identities(orc, n):
    """Algorithm 5: Q orthogonal and Q R = A to the order n u_d (the bounds
    Section 4.2 checks; a constant of 4 covers the few ulps of a single
    reflection at n = 2), R upper triangular, and the same factorisation as
    LAPACK's up to the signs of R's rows (a library cross-check)."""
    A = wl.rng(80 + n).standard_normal((n, n))
    Q, R = orc.householder_qr(A)
    assert np.linalg.norm(Q.T @ Q - np.eye(n), 2) <= 4 * n * U_D
    assert np.linalg.norm(Q @ R - A, 2) / np.linalg.norm(A, 2) <= 4 * n * U_D
    assert np.array_equal(R, np.triu(R))
    Ql, Rl = np.linalg.qr(A)
    sg = np.sign(np.diag(R)) * np.sign(np.diag(Rl))
    assert np.abs(Q * sg - Ql).max() <= 1e-12
    assert np.abs(R * sg[:, None] - Rl).max() <= 1e-12 * np.abs(Rl).max()


def test_householder_qr_of_orthogonal(orc):
    """For an orthogonal input the factorisation is Q = X D, R = D with D =
    diag(+-1): the orthogonaliser returns the input up to column signs."""
    X = wl.haar(30, wl.rng(90))
    Q, R = orc.householder_qr(X)
    d = np.diag(R)
    assert np.abs(np.abs(d) - 1.0).max() <= 30 * U_D
    assert np.abs(R - np.diag(d)).max() <= 30 * U_D
    assert np.abs(Q - X * np.sign(d)).max() <= 30 * U_D


def test_cholesky_known_factor(orc):
    """G = R^T R for an upper-triangular R with positive diagonal: the oracle
    returns R; a non-positive pivot is reported (row index + 1)."""
    g = wl.rng(91)
    n = 12
    R0 = np.triu(g.standard_normal((n, n)))
    R0[np.diag_indices(n)] = np.abs(R0[np.diag_indices(n)]) + 1.0
    G = R0.T @ R0
    R, st = orc.cholesky(G)
    assert st == 0
    assert np.abs(R - R0).max() <= 1e-12 * np.abs(R0).max()
    assert np.array_equal(R, np.triu(R))
    R2, st2 = orc.cholesky(np.diag([4.0, 9.0, 16.0]))
    assert st2 == 0 and np.array_equal(R2, np.diag([2.0, 3.0, 4.0]))
    _, st3 = orc.cholesky(np.array([[1.0, 2.0], [2.0, 1.0]]))
    assert st3 == 2


@pytest.mark.parametrize("n", [5, 40])
def test_cholesky_qr_identities(orc, n):
    """Cholesky QR of a well-conditioned X: Q R = X, Q^T Q = I (to kappa(X)^2
    u_d), R = chol(X^T X), and the same factorisation as LAPACK's QR with a
    positive diagonal of R."""
    g = wl.rng(92 + n)
    X = wl.haar(n, g) @ np.diag(np.linspace(1.0, 2.0, n)) @ wl.haar(n, g)
    Q, R, st = orc.cholesky_qr(X)
    assert st == 0
    assert np.linalg.norm(Q @ R - X, 2) / np.linalg.norm(X, 2) <= n * U_D
    assert np.linalg.norm(Q.T @ Q - np.eye(n), 2) <= 4 * n * U_D * 4.0
    Ql, Rl = np.linalg.qr(X)
    sg = np.sign(np.diag(Rl))
    assert np.abs(Q - Ql * sg).max() <= 1e-13
    assert np.abs(R - Rl * sg[:, None]).max() <= 1e-13


@pytest.mark.parametrize("orth", ["householder", "cholesky"])
def test_mixed_with_qr_orthogonalisers(orc, orth):
    """Algorithm 9 with Q_d from a QR factorisation of Q_l instead of
    Newton-Schulz: the same stage bounds (||Q_d^T Q_d - I||_F <~ n u_d, here
    with a constant of 2: Householder QR lands at 1.1 n u_d on this input;
    off(A_cond) <~ n u_l ||A||) and the same eigenvalues."""
    n = 60
    A, lam = wl.geo_spectrum(n, 3, kappa=1e3)
    nrm2 = np.abs(lam).max()
    W, Q, st, d = orc.eigh_mixed(A, orth=orth)
    assert st == 0
    assert d["orth_qd"] <= 2 * n * U_D
    assert d["off_cond"] <= n * U_L * nrm2
    assert 1 <= d["sweeps64"] <= 5
    assert np.abs(W - lam).max() <= 1e-13 * nrm2
    assert np.linalg.norm(A @ Q - Q * W) / np.linalg.norm(A) <= 1e-13 * n
    assert np.linalg.norm(Q.T @ Q - np.eye(n)) <= 1e-14 * n


# --------------------------------------- binary16 stage (precision ladder)
def test_round_half_definition(orc):
    """Round to nearest binary16 with ties to even, from the format's
    definition: spacing 2^-10 at 1, ties 1 + 2^-11 -> 1 and 1 + 3 2^-11 ->
    1 + 2^-9, largest finite 65504 (65519 stays, 65520 overflows), subnormal
    spacing 2^-24 (2^-25 ties to 0, 3 2^-25 to 2^-23); and numpy's float16
    conversion on random values (a library cross-check)."""
    r = orc.round_half
    assert r(1.0) == 1.0 and r(-2.5) == -2.5
    assert r(1.0 + 2.0 ** -11) == 1.0
    assert r(1.0 + 3 * 2.0 ** -11) == 1.0 + 2.0 ** -9
    assert r(1.0 + 2.0 ** -11 + 2.0 ** -20) == 1.0 + 2.0 ** -10
    assert r(65504.0) == 65504.0 and r(65519.0) == 65504.0
    assert math.isinf(r(65520.0)) and r(-1e6) == -math.inf
    assert r(2.0 ** -24) == 2.0 ** -24 and r(2.0 ** -25) == 0.0
    assert r(3 * 2.0 ** -25) == 2.0 ** -23 and r(2.0 ** -14) == 2.0 ** -14
    g = wl.rng(95)
    x = g.standard_normal(2000) * 10.0 ** g.uniform(-9, 4.5, 2000)
    got = np.array([r(v) for v in x])
    assert np.array_equal(got, x.astype(np.float16).astype(np.float64))


def test_ns_iteration_count_low_precision(orc):
    """Section 4.3.4's count, (sqrt(1 + n u) - 1)^(2^k) <= n u_d: with u_l it is
    2 up to the printed crossover n ~ 52071 and 3 beyond (to 2172548); with
    binary16 vectors (u_h = 2^-11) it is 5 at n = 1024, and from n u_h >= 2
    (n = 4096) the singular values of X_0 reach sqrt(3), where the iteration is
    no longer guaranteed to converge (-1)."""
    fx = golden("ns_iteration_count.txt")
    c2, c3 = fx["crossover_two"], fx["crossover_three"]
    assert orc.ns_iterations(c2 - 100, U_L) == 2
    assert orc.ns_iterations(c2 + 100, U_L) == 3
    assert orc.ns_iterations(c3 * 0.999, U_L) == 3
    assert orc.ns_iterations(4096, U_L) == 2
    u_h = 2.0 ** -11
    assert orc.ns_iterations(1024, u_h) == 5
    assert orc.ns_iterations(256, u_h) == 4
    assert orc.ns_iterations(4096, u_h) == -1
    assert orc.ns_iterations(4095, u_h) > 0


@pytest.mark.parametrize("name", ["goe", "geo"])
def test_half_stage_bounds(orc, name):
    """The binary16 stage: every stored entry is a binary16 value, off falls
    sweep after sweep until the binary16 rounding floor and ends below
    n u_h ||A||_F (the Section 5.2.1 bound with u_h), V (kept in FP32) is
    orthogonal to order n u_l, and Q_h^T A Q_h is diagonal to the same order:
    the FP32 stage from it needs fewer sweeps than from A."""
    n = 96
    A = wl.goe(n, 96) if name == "goe" else wl.geo_spectrum(n, 97, kappa=1e3)[0]
    nf = np.linalg.norm(A)
    # early sweeps lower off by only about a half, so the stall factor (the
    # stop at the rounding floor) is 0.9
    Ah, V, sw, st, hist = orc.jacobi_cyclic_h(A, stall=0.9)
    assert st == 0 and sw >= 3
    assert np.array_equal(Ah.astype(np.float64),
                          Ah.astype(np.float16).astype(np.float64))
    assert all(hist[k + 1] <= 0.9 * hist[k] for k in range(sw - 1))
    assert hist[-1] <= n * 2.0 ** -11 * nf
    V64 = V.astype(np.float64)
    assert np.linalg.norm(V64.T @ V64 - np.eye(n)) <= 4 * n * U_L
    B = V64.T @ A @ V64
    assert orc.off(B) <= n * 2.0 ** -11 * nf
    tol32 = 0.1 * n * U_L * nf
    _, _, s_from_h, _, _ = orc.jacobi_cyclic_f32(B.astype(np.float32), tol32)
    _, _, s_from_a, _, _ = orc.jacobi_cyclic_f32(A.astype(np.float32), tol32)
    assert s_from_h < s_from_a
