"""GPU parity: libjacobi (through its C ABI) against the CPU oracle.

Bars (the solver's contract): max |W - W_ref| <= 1e-13 ||A||_2,
||A V - V W||_F / ||A||_F <= 1e-13 n, ||V^T V - I||_F <= 1e-14 n.  Eigenvectors
are unique only up to sign and within clusters, so V is judged by residual and
orthogonality, by its sign convention, and by |v_k . v_k(oracle)| ~ 1 where
the gap around lambda_k exceeds 1e-6 ||A||_2.
"""
import numpy as np
import pytest

import oracle
import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def pj():
    import paper_2509_00495_amd as pj
    print("\n" + pj.device_summary(), flush=True)
    return pj


def gpu(A):
    return torch.tensor(np.ascontiguousarray(A), dtype=torch.float64, device="cuda")


def check(A, W, V, W_ref, V_ref=None, label=""):
    n = A.shape[0]
    if n == 0:
        return
    nrm2 = max(np.abs(W_ref).max(), 1e-300)
    err = np.abs(W - W_ref).max()
    res = np.linalg.norm(A @ V - V * W) / max(np.linalg.norm(A), 1e-300)
    orth = np.linalg.norm(V.T @ V - np.eye(n))
    print(f"  {label} n={n}: |dW|/|A|={err / nrm2:.2e} res={res:.2e} orth={orth:.2e}",
          flush=True)
    assert err <= 1e-13 * nrm2, (label, err)
    assert res <= 1e-13 * n, (label, res)
    assert orth <= 1e-14 * n, (label, orth)
    assert (np.diff(W) >= 0).all()
    idx = np.argmax(np.abs(V), axis=0)
    assert (V[idx, np.arange(n)] > 0).all()
    if V_ref is not None:
        gaps = np.diff(W_ref)
        for k in range(n):
            g = min(gaps[k - 1] if k > 0 else np.inf, gaps[k] if k < n - 1 else np.inf)
            if g > 1e-6 * nrm2:
                assert abs(abs(V[:, k] @ V_ref[:, k]) - 1.0) < 1e-8, (label, k)


def run(pj, fn, A, **kw):
    print(f"  -> {fn} n={A.shape[0]} {kw}", flush=True)
    opts = pj.make_opts(**kw) if kw else None
    W, V, info = getattr(pj, fn)(gpu(A), opts=opts, return_info=True)
    torch.cuda.synchronize()
    print(f"     sweeps={info['sweeps']} sweeps32={info['sweeps32']} "
          f"orth_est={info['orth_est']:.2e} polished={info['polished']}", flush=True)
    return W.cpu().numpy(), V.cpu().numpy(), info


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 7, 16, 31, 64, 100, 128])
def test_small_path_vs_oracle(pj, n):
    A = wl.random_symmetric(n, 1000 + n)
    W, V, info = run(pj, "eigh", A)
    assert info["path"] == 0 and info["status"] == 0
    Wo, Vo, *_ = oracle.eigh(A)
    check(A, W, V, Wo, Vo, "small")


def test_uniform64_known_spectrum(pj):
    """n=64, lam ~ U[-1,1]: plain FP64 Jacobi, tol 1e-15 n ||A||_F."""
    A, lam = wl.uniform_spectrum(64, 1)
    W, V, info = run(pj, "eigh", A)
    Wo, Vo, *_ = oracle.eigh(A)
    check(A, W, V, Wo, Vo, "uniform64")
    assert np.abs(W - lam).max() <= 1e-13 * np.abs(lam).max()
    assert info["tol"] == pytest.approx(1e-15 * 64 * np.linalg.norm(A), rel=1e-12)


@pytest.mark.parametrize("n,block", [(5, 16), (33, 16), (64, 32), (130, 16), (200, 32),
                                     (257, 16), (300, 32)])
def test_block_path_vs_oracle(pj, n, block):
    A = wl.random_symmetric(n, 2000 + n)
    W, V, info = run(pj, "eigh", A, small_max_n=-1, block=block)
    assert info["path"] == 1 and info["status"] == 0
    Wo, Vo, *_ = oracle.eigh(A)
    check(A, W, V, Wo, Vo, f"block b={block}")


@pytest.mark.parametrize("n,block", [(130, 16), (300, 32)])
def test_block_path_circle_schedule(pj, n, block):
    """schedule=1: every pair of each 2b x 2b tile in every round."""
    A = wl.random_symmetric(n, 2500 + n)
    W, V, info = run(pj, "eigh", A, small_max_n=-1, block=block, schedule=1)
    assert info["path"] == 1 and info["status"] == 0
    Wo, Vo, *_ = oracle.eigh(A)
    check(A, W, V, Wo, Vo, f"circle b={block}")


@pytest.mark.parametrize("serial_v", [1, 2])
@pytest.mark.parametrize("fn", ["eigh", "eigh_mixed"])
def test_block_path_serial_v(pj, fn, serial_v):
    """serial_v=1: every eigenvector update on the caller's stream after the
    B update; 2: on the second stream (the default runs it inside the next
    round's pair-solve launch)."""
    A = wl.random_symmetric(260, 2600)
    W, V, info = run(pj, fn, A, small_max_n=-1, block=32, serial_v=serial_v)
    assert info["path"] == 1 and info["status"] == 0
    Wo, Vo, *_ = oracle.eigh(A)
    check(A, W, V, Wo, Vo, f"serial_v={serial_v} {fn}")


@pytest.mark.parametrize("fn", ["eigh", "eigh_mixed"])
def test_shared_launch_bitwise(pj, fn):
    """The V update inside the next round's pair-solve launch (row ranges of
    each pair's columns on the workgroups the solves leave free) does per tile
    exactly the arithmetic of the standalone update kernel: the default and
    serial_v = 1 agree bitwise.  A tile skipped or updated twice would break
    this."""
    A = wl.random_symmetric(520, 5200)
    W0, V0, i0 = run(pj, fn, A, small_max_n=-1, block=32)
    W1, V1, i1 = run(pj, fn, A, small_max_n=-1, block=32, serial_v=1)
    assert i0["sweeps"] == i1["sweeps"]
    assert np.array_equal(W0, W1) and np.array_equal(V0, V1)


@pytest.mark.parametrize("fn", ["eigh", "eigh_mixed"])
def test_shared_launch_bitwise_4096(pj, fn):
    """At n = 4096 the pair-solve workgroups of the FP64 shared launch also take
    the last tiles of their pair's V update (the split the timing model picks
    there is nonzero); the result still equals the standalone update's bitwise."""
    A = torch.tensor(wl.goe(4096, 3), device="cuda")
    print(f"  -> {fn} n=4096 default vs serial_v=1", flush=True)
    W0, V0 = getattr(pj, fn)(A)
    W1, V1 = getattr(pj, fn)(A, opts=pj.make_opts(serial_v=1))
    torch.cuda.synchronize()
    assert torch.equal(W0, W1) and torch.equal(V0, V1)


@pytest.mark.parametrize("n,block,inner", [(128, 16, 2), (192, 32, 3)])
def test_block_path_inner_sweeps(pj, n, block, inner):
    A = wl.random_symmetric(n, 3000 + n)
    W, V, info = run(pj, "eigh", A, small_max_n=-1, block=block, inner_sweeps=inner)
    Wo, Vo, *_ = oracle.eigh(A)
    check(A, W, V, Wo, Vo, f"inner={inner}")


@pytest.mark.parametrize("n", [7, 64, 96, 200, 300])
def test_mixed_vs_oracle(pj, n):
    A, lam = wl.geo_spectrum(n, 4000 + n, kappa=1e4)
    W, V, info = run(pj, "eigh_mixed", A)
    assert info["status"] == 0
    Wo, Vo, *_ = oracle.eigh(A)
    check(A, W, V, Wo, Vo, "mixed")
    assert np.abs(W - lam).max() <= 1e-13 * np.abs(lam).max()
    # stage diagnostics against the paper's bounds (Sections 4.3.4, 5.2.1)
    print(f"  mixed stages: sweeps32={info['sweeps32']} sweeps64={info['sweeps']} "
          f"ns={info['ns_iters']} off_cond/|A|={info['off_cond'] / np.abs(lam).max():.2e} "
          f"orth_ns={info['orth_ns']:.2e}", flush=True)
    assert info["ns_iters"] == 2
    assert info["off_cond"] <= 10 * n * 2.0 ** -24 * np.linalg.norm(A)


@pytest.mark.parametrize("n", [96, 300])
def test_mixed_stages_vs_oracle(pj, n):
    """Each stage of the mixed path beside the oracle's same stage on the
    same matrix (Algorithm 9 with the FP32 Jacobi first stage, both with the
    FP32 stop at 0.1 n u_l ||A||_F): ||Q_l^T Q_l - I||_F (order n u_l, the
    starting point of Section 4.3.4's count), ||Q_d^T Q_d - I||_F (order n u_d
    after two Newton-Schulz steps), off(Q_d^T A Q_d) (Section 5.2.1: order
    n u_l ||A||_F) and the final eigenvalues (1e-13 ||A||_2, element by
    element).  The two use different orderings (block round-robin against
    cyclic-by-row), so the stage values are compared through their bounds
    and their order of magnitude, not digit by digit."""
    U_L, U_D = 2.0 ** -24, 2.0 ** -53
    A, lam = wl.geo_spectrum(n, 8000 + n, kappa=1e4)
    W, V, info = run(pj, "eigh_mixed", A, timing=1)
    Wo, _, st, d = oracle.eigh_mixed(A, c32=0.1)
    assert info["status"] == 0 and st == 0
    nf = np.linalg.norm(A)
    nrm2 = np.abs(lam).max()
    gpu = dict(orth_ql=info["orth_ql"], orth_qd=info["orth_qd"], off_cond=info["off_cond"])
    print(f"  stages n={n}: gpu {gpu}  oracle orth_ql={d['orth_ql']:.2e} "
          f"orth_qd={d['orth_qd']:.2e} off_cond={d['off_cond']:.2e}", flush=True)
    for k in ("orth_ql", "orth_qd", "off_cond"):
        assert gpu[k] > 0.0
        assert 0.02 <= gpu[k] / d[k] <= 50.0, k
    assert gpu["orth_ql"] <= 10 * n * U_L and d["orth_ql"] <= 10 * n * U_L
    npad = -(-n // 16) * 16 if n <= 256 else -(-n // 64) * 64
    assert gpu["orth_qd"] <= 4 * npad * U_D and d["orth_qd"] <= 4 * n * U_D
    assert gpu["off_cond"] <= 10 * n * U_L * nf and d["off_cond"] <= 10 * n * U_L * nf
    assert np.abs(W - Wo).max() <= 1e-13 * nrm2
    assert np.abs(W - lam).max() <= 1e-13 * nrm2


def test_mixed_one_ns_step_polished(pj):
    """One Newton-Schulz step leaves Q_d with an orthogonality error far above
    the bar (about 1e-10 here).  The output stage must detect it (randomized
    estimate) and apply its own Newton-Schulz step, so that V meets the
    orthogonality and residual bars.  The eigenvalues of Q_d^T A Q_d still
    differ from A's by about that error times ||A||, which is why two steps
    are the default; that bound is what is checked for W."""
    A = wl.goe(300, 78)
    W, V, info = run(pj, "eigh_mixed", A, ns_iters=1)
    n = A.shape[0]
    assert info["ns_iters"] == 1
    assert info["polished"] == 1
    Wo, *_ = oracle.eigh(A)
    nrm2 = np.abs(Wo).max()
    res = np.linalg.norm(A @ V - V * W) / np.linalg.norm(A)
    orth = np.linalg.norm(V.T @ V - np.eye(n))
    err = np.abs(W - Wo).max()
    print(f"  ns=1: orth_ns={info['orth_ns']:.2e} |dW|/|A|={err / nrm2:.2e} res={res:.2e} "
          f"orth={orth:.2e}", flush=True)
    assert orth <= 1e-14 * n
    assert res <= 1e-13 * n
    assert err <= 10 * info["orth_ns"] * nrm2


def test_output_columns_normalized(pj):
    """The output stage scales every eigenvector to unit norm: the column norms
    are 1 to a few ulps, on both block paths.  (n = 300: at n = 512 the oracle's
    own eigenvalues, the diagonal after its sweeps, already drift by about
    1.4e-13 ||A||_2 on this input.)"""
    A = wl.goe(300, 79)
    for fn in ("eigh", "eigh_mixed"):
        W, V, info = run(pj, fn, A, small_max_n=-1)
        dev = np.abs(np.linalg.norm(V, axis=0) - 1.0).max()
        print(f"  {fn}: max | ||v_k|| - 1 | = {dev:.2e}", flush=True)
        assert dev <= 64 * 2.0 ** -53
        # the randomized estimate (4 probes) tracks the true orthogonality
        orth = np.linalg.norm(V.T @ V - np.eye(A.shape[0]))
        print(f"  {fn}: orth={orth:.2e} estimate={info['orth_est']:.2e}", flush=True)
        assert orth / 4 <= info["orth_est"] <= 4 * orth
        Wo, Vo, *_ = oracle.eigh(A)
        check(A, W, V, Wo, Vo, fn)


@pytest.mark.parametrize("fn", ["eigh", "eigh_mixed"])
def test_ari_known_spectrum(pj, fn):
    """Arithmetic family (magnitudes linear from 1 to 1/kappa, random signs),
    block path: eigenvalues against the spectrum the matrix was built from."""
    A, lam = wl.ari_spectrum(520, 7, kappa=1e2)
    W, V, info = run(pj, fn, A, small_max_n=-1)
    assert info["status"] == 0
    n = A.shape[0]
    nrm2 = np.abs(lam).max()
    print(f"  ari {fn}: sweeps={info['sweeps']} sweeps32={info['sweeps32']} "
          f"|W-lam|/|A|_2={np.abs(W - lam).max() / nrm2:.2e}", flush=True)
    assert np.abs(W - lam).max() <= 1e-13 * nrm2
    assert np.linalg.norm(A @ V - V * W) / np.linalg.norm(A) <= 1e-13 * n
    assert np.linalg.norm(V.T @ V - np.eye(n)) <= 1e-14 * n


@pytest.mark.parametrize("fn", ["eigh", "eigh_mixed"])
@pytest.mark.parametrize("sizes", [[256] * 4, [300, 200, 524]])
def test_pair_skip_block_diagonal(pj, fn, sizes):
    """Decoupled diagonal blocks: a block pair that joins two of them has no
    coupling, rotates nothing and leaves U = I, so the B tiles of two such
    pairs (and the V columns of such a pair) are left out of the updates.
    Eigenvalues against the spectrum the blocks were built from, residual
    and orthogonality bars; with blocks aligned to the block size, tiles
    must actually have been left out."""
    A, lam = wl.block_diagonal(1024, sizes=sizes, seed=21)
    W, V, info = run(pj, fn, A)
    assert info["status"] == 0
    n = A.shape[0]
    nrm2 = np.abs(lam).max()
    print(f"  blockdiag {sizes} {fn}: sweeps={info['sweeps']} sweeps32={info['sweeps32']} "
          f"skipped_tiles={info['skipped_tiles']} "
          f"|W-lam|/|A|_2={np.abs(W - lam).max() / nrm2:.2e}", flush=True)
    assert np.abs(W - lam).max() <= 1e-13 * nrm2
    assert np.linalg.norm(A @ V - V * W) / np.linalg.norm(A) <= 1e-13 * n
    assert np.linalg.norm(V.T @ V - np.eye(n)) <= 1e-14 * n
    assert info["skipped_tiles"] >= 0
    if all(m % info["block"] == 0 for m in sizes):
        assert info["skipped_tiles"] > 0


@pytest.mark.parametrize("fn", ["eigh", "eigh_mixed"])
@pytest.mark.parametrize("case,serial_v", [("blockdiag", 0), ("goe", 0), ("blockdiag", 1),
                                           ("blockdiag", 2)])
def test_pair_skip_changes_nothing(pj, fn, case, serial_v):
    """A left-out update is one whose rotation is exactly the identity, so
    the outputs with pair skipping equal those without it bit for bit, with
    the V update inside the next pair-solve launch (serial_v = 0), after the
    B update (1) or on the side stream, which reads the flags of the
    double-buffered round (2)."""
    A = (wl.block_diagonal(1024, 4, seed=22)[0] if case == "blockdiag"
         else wl.goe(1024, 23))
    W1, V1, i1 = run(pj, fn, A, serial_v=serial_v)
    W0, V0, i0 = run(pj, fn, A, no_pair_skip=1)
    print(f"  {case} {fn}: skipped_tiles {i1['skipped_tiles']} / {i0['skipped_tiles']}", flush=True)
    assert i0["skipped_tiles"] == 0
    if case == "blockdiag":
        assert i1["skipped_tiles"] > 0
    assert (i1["sweeps"], i1["sweeps32"]) == (i0["sweeps"], i0["sweeps32"])
    assert np.array_equal(W1, W0) and np.array_equal(V1, V0)


@pytest.mark.parametrize("fn", ["eigh", "eigh_mixed"])
def test_geo1024_vs_oracle_fixture(pj, fn):
    """The n = 1024 geometric workload (magnitudes 1 .. 1e-6, random signs) at
    full size: eigenvalues against the spectrum it was built from (the bar),
    and against the oracle's stored run on the same matrix
    (tests/golden/oracle_geo1024.txt, written by make_oracle_fixtures.py)
    within the oracle's own distance from that spectrum (its eigenvalues are
    the diagonal after 15 sweeps of rotations, which drifts by 2.5e-13 ||A||_2
    here), plus the residual and orthogonality bars."""
    import os
    A, lam = wl.geo_spectrum(1024, 2)
    gold = os.path.join(os.path.dirname(__file__), "golden", "oracle_geo1024.txt")
    Wo = np.loadtxt(gold, ndmin=2)[:, 0]
    W, V, info = run(pj, fn, A)
    assert info["status"] == 0
    n = A.shape[0]
    nrm2 = np.abs(lam).max()
    print(f"  geo1024 {fn}: |W-W_oracle|/|A|_2={np.abs(W - Wo).max() / nrm2:.2e} "
          f"|W-lam|/|A|_2={np.abs(W - lam).max() / nrm2:.2e}", flush=True)
    assert np.abs(W - lam).max() <= 1e-13 * nrm2
    assert np.abs(W - Wo).max() <= np.abs(Wo - lam).max() + 1e-13 * nrm2
    assert np.linalg.norm(A @ V - V * W) / np.linalg.norm(A) <= 1e-13 * n
    assert np.linalg.norm(V.T @ V - np.eye(n)) <= 1e-14 * n


def test_mixed_goe(pj):
    A = wl.goe(256, 77)
    W, V, info = run(pj, "eigh_mixed", A)
    Wo, Vo, *_ = oracle.eigh(A)
    check(A, W, V, Wo, Vo, "mixed goe")


def test_diagonal_input(pj):
    d = np.array([3.0, -1.0, 2.0, 0.5, -7.0, 0.0])
    for kw in ({}, dict(small_max_n=-1)):
        W, V, info = run(pj, "eigh", np.diag(d), **kw)
        assert np.array_equal(W, np.sort(d))
        assert info["sweeps"] == 0
        P = np.zeros((6, 6))
        for c, i in enumerate(np.argsort(d, kind="stable")):
            P[i, c] = 1.0
        assert np.array_equal(V, P)


def test_noconv_status(pj):
    A = wl.random_symmetric(64, 5)
    for kw in (dict(max_sweeps=1), dict(max_sweeps=1, small_max_n=-1)):
        W, V, info = pj.eigh(gpu(A), opts=pj.make_opts(**kw), check=False, return_info=True)
        assert info["status"] == pj.NOCONV, kw
        V = V.cpu().numpy()
        assert np.linalg.norm(V.T @ V - np.eye(64)) < 1e-12


def test_nonfinite_and_notsym(pj):
    A = wl.random_symmetric(8, 6)
    A[2, 3] = np.nan
    for kw in (None, pj.make_opts(small_max_n=-1)):
        with pytest.raises(pj.JacobiError) as e:
            pj.eigh(gpu(A), opts=kw)
        assert e.value.status == pj.NONFINITE
    B = wl.random_symmetric(8, 7)
    B[0, 1] += 1e-3
    with pytest.raises(pj.JacobiError) as e:
        pj.eigh(gpu(B), opts=pj.make_opts(check_symmetry=1, small_max_n=-1))
    assert e.value.status == pj.NOTSYM
    W, V = pj.eigh(gpu(B))   # without the check A is symmetrised
    Bs = 0.5 * (B + B.T)
    Wo, *_ = oracle.eigh(Bs)
    assert np.abs(W.cpu().numpy() - Wo).max() < 1e-13 * np.abs(Wo).max()


def test_strided_input(pj):
    """lda > n: a view into a larger matrix."""
    A = wl.random_symmetric(40, 8)
    big = np.zeros((40, 56))
    big[:, :40] = A
    At = torch.tensor(big, device="cuda")[:, :40]
    for kw in (None, pj.make_opts(small_max_n=-1)):
        W, V = pj.eigh(At, opts=kw)
        Wo, Vo, *_ = oracle.eigh(A)
        check(A, W.cpu().numpy(), V.cpu().numpy(), Wo, Vo, "strided")


@pytest.mark.parametrize("fn", ["eigh", "eigh_mixed"])
def test_goe4096_properties(pj, fn):
    """The n = 4096 workload, in the launch configuration the benchmark times.
    The oracle cannot solve it in test time, so the checks are size-independent.
    Eigenvalues: with r_k = A v_k - rho_k v_k and rho_k = v_k^T A v_k, the
    Kato-Temple bound puts an eigenvalue within |r_k|^2 / delta_k of rho_k,
    delta_k being the distance from rho_k to the rest of the spectrum (taken
    from the computed neighbours less the residual norms); w_k must lie within
    1e-13 ||A||_2 of that certified interval wherever delta_k > 1e-6 ||A||_2.
    Plus the residual and orthogonality bars and the trace and Frobenius
    invariants."""
    A = wl.goe(4096, 3)
    n = A.shape[0]
    W, V, info = run(pj, fn, A)
    assert info["status"] == 0 and info["path"] == 1
    nrm2 = np.abs(W).max()
    AV = A @ V
    rho = np.einsum("ij,ij->j", V, AV) / np.einsum("ij,ij->j", V, V)
    rk = np.linalg.norm(AV - V * rho, axis=0)
    R = AV - V * W
    res = np.linalg.norm(R) / np.linalg.norm(A)
    orth = np.linalg.norm(V.T @ V - np.eye(n))
    gap = np.minimum(np.r_[np.inf, np.diff(W)], np.r_[np.diff(W), np.inf])
    delta = gap - 2 * rk.max()
    sep = delta > 1e-6 * nrm2
    kt = np.where(sep, rk ** 2 / np.where(sep, delta, 1.0), np.inf)
    err = np.abs(W - rho) + kt
    print(f"  {fn} n={n}: res={res:.2e} orth={orth:.2e} max|r_k|/|A|_2={rk.max() / nrm2:.2e} "
          f"separated={sep.sum()} max certified |dW|/|A|_2={err[sep].max() / nrm2:.2e}",
          flush=True)
    assert sep.sum() >= 0.99 * n
    assert err[sep].max() <= 1e-13 * nrm2
    assert res <= 1e-13 * n
    assert orth <= 1e-14 * n
    assert abs(W.sum() - np.trace(A)) <= 1e-13 * n * nrm2
    assert abs(np.sqrt((W * W).sum()) - np.linalg.norm(A)) <= 1e-13 * np.linalg.norm(A)
    assert (np.diff(W) >= 0).all()
    idx = np.argmax(np.abs(V), axis=0)
    assert (V[idx, np.arange(n)] > 0).all()
