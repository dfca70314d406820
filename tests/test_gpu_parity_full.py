"""GPU parity at full size, on forced code paths and on edge inputs.

* The n = 4096 workload and the n = 1024 geometric workload against the
  oracle's stored runs (tests/golden/oracle_*.txt, written by
  make_oracle_fixtures.py from the oracle alone).  Each fixture line holds the
  oracle's eigenvalue (its diagonal after the sweeps), the Rayleigh quotient
  rq of the oracle's eigenvector and that vector's residual norm res.  By the
  Kato-Temple bound an eigenvalue lies within res^2 / gap of rq, so the
  oracle's certified eigenvalue interval is [rq - res^2/gap, rq + res^2/gap];
  the library's eigenvalues must lie within 1e-13 ||A||_2 of it.
* Code paths that the default launch configuration only takes near
  n = 4096 (the stream-K split of the symmetric FP64 products and the share
  of the V update taken by the pair-solve workgroups), forced at n = 1024
  through jacobi_opts, against the same fixture.
* Inputs scaled by 2^+-500 (every result scales exactly), repeated
  eigenvalues and a zero diagonal through the block path, and pair skipping
  in an oracle-compared solve.
"""
import os
import sys

import numpy as np
import pytest

import oracle
import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

GOLD = os.path.join(os.path.dirname(__file__), "golden")
sys.path.insert(0, GOLD)
import make_oracle_fixtures as fixtures  # noqa: E402


@pytest.fixture(scope="module")
def pj():
    import paper_2509_00495_amd as pj
    print("\n" + pj.device_summary(), flush=True)
    return pj


def gpu(A):
    return torch.tensor(np.ascontiguousarray(A), dtype=torch.float64, device="cuda")


def solve(pj, fn, A, **kw):
    print(f"  -> {fn} n={A.shape[0]} {kw}", flush=True)
    opts = pj.make_opts(**kw) if kw else None
    W, V, info = getattr(pj, fn)(gpu(A), opts=opts, return_info=True)
    torch.cuda.synchronize()
    print(f"     status={info['status']} sweeps={info['sweeps']} sweeps32={info['sweeps32']} "
          f"skipped_tiles={info['skipped_tiles']}", flush=True)
    return W.cpu().numpy(), V.cpu().numpy(), info


def bars(A, W, V, label):
    n = A.shape[0]
    res = np.linalg.norm(A @ V - V * W) / np.linalg.norm(A)
    orth = np.linalg.norm(V.T @ V - np.eye(n))
    print(f"  {label}: res={res:.2e} orth={orth:.2e}", flush=True)
    assert res <= 1e-13 * n, (label, res)
    assert orth <= 1e-14 * n, (label, orth)
    assert (np.diff(W) >= 0).all()
    idx = np.argmax(np.abs(V), axis=0)
    assert (V[idx, np.arange(n)] > 0).all()


def certified(rq, res):
    """Half-widths of the oracle's Kato-Temple intervals around rq (gap from
    the neighbouring quotients less both residuals); inf where the gap does
    not separate."""
    gap = np.minimum(np.r_[np.inf, np.diff(rq)], np.r_[np.diff(rq), np.inf])
    delta = gap - 2 * res.max()
    return np.where(delta > 0, res ** 2 / np.where(delta > 0, delta, 1.0), np.inf)


def vs_fixture(W, name, nrm2, label):
    """max over k of the distance from W_k to the oracle's certified interval,
    relative to ||A||_2, for every separated eigenvalue; returns it and the
    number of separated ones."""
    wo, rq, res, head = fixtures.load(name)
    kt = certified(rq, res)
    sep = np.isfinite(kt)
    dist = np.maximum(np.abs(W - rq) - kt, 0.0)
    worst = dist[sep].max() / nrm2
    print(f"  {label}: vs oracle {name}: separated {sep.sum()} of {len(rq)}, "
          f"max dist to certified interval {worst:.2e} ||A||_2, oracle diag readout "
          f"|w - rq| {np.abs(wo - rq).max() / nrm2:.2e}, max res {res.max() / nrm2:.2e}",
          flush=True)
    return worst, sep.sum()


# ------------------------------------------------------------ full size
@pytest.mark.parametrize("fn", ["eigh", "eigh_mixed"])
def test_goe4096_vs_oracle_fixture(pj, fn):
    """The n = 4096 workload, in the launch configuration the benchmark times,
    against the oracle's stored run of the same matrix."""
    if not os.path.exists(os.path.join(GOLD, "oracle_goe4096.txt")):
        pytest.skip("oracle fixture for the n = 4096 workload not written")
    A = wl.goe(4096, 3)
    W, V, info = solve(pj, fn, A)
    assert info["status"] == 0 and info["path"] == 1
    wo, rq, res, _ = fixtures.load("goe4096")
    nrm2 = np.abs(rq).max()
    worst, nsep = vs_fixture(W, "goe4096", nrm2, fn)
    assert nsep >= 0.99 * len(rq)
    assert worst <= 1e-13
    bars(A, W, V, fn)


GOE_VARIANTS = [dict(orth=1), dict(orth=2), dict(ladder=1)]


@pytest.mark.parametrize("kw", GOE_VARIANTS, ids=["householder", "cholesky", "ladder"])
def test_goe4096_variants_vs_oracle_fixture(pj, kw):
    """The mixed path's other orthogonalisers (Section 4.4) and the binary16
    first stage at n = 4096, against the same stored oracle run."""
    if not os.path.exists(os.path.join(GOLD, "oracle_goe4096.txt")):
        pytest.skip("oracle fixture for the n = 4096 workload not written")
    A = wl.goe(4096, 3)
    W, V, info = solve(pj, "eigh_mixed", A, **kw)
    assert info["status"] == 0 and info["path"] == 1
    _, rq, _, _ = fixtures.load("goe4096")
    worst, nsep = vs_fixture(W, "goe4096", np.abs(rq).max(), f"eigh_mixed {kw}")
    assert nsep >= 0.99 * len(rq)
    assert worst <= 1e-13
    bars(A, W, V, f"eigh_mixed {kw}")


FORCED = [("eigh", dict(pair_v_split=4)),
          ("eigh_mixed", dict(pair_v_split=4)),
          ("eigh_mixed", dict(gemm_slots=16)),
          ("eigh_mixed", dict(gemm_slots=7, pair_v_split=2))]


@pytest.mark.parametrize("fn,kw", FORCED, ids=[f"{f}-{k}" for f, k in FORCED])
def test_geo1024_forced_paths_vs_oracle(pj, fn, kw):
    """n = 1024 geometric workload with the pair-solve workgroups taking part
    of the V update (pair_v_split) and/or the symmetric FP64 products split
    over fewer resident slots than their tiles (gemm_slots: 36 upper tiles
    over 16 or 7 workgroups, every tile in at most two parts): eigenvalues
    against the known spectrum and the oracle's certified interval, residual
    and orthogonality bars."""
    A, lam = wl.geo_spectrum(1024, 2)
    W, V, info = solve(pj, fn, A, **kw)
    assert info["status"] == 0
    nrm2 = np.abs(lam).max()
    assert np.abs(W - lam).max() <= 1e-13 * nrm2
    worst, nsep = vs_fixture(W, "geo1024", nrm2, f"{fn} {kw}")
    assert nsep >= 0.9 * len(lam)
    assert worst <= 1e-13
    bars(A, W, V, f"{fn} {kw}")


@pytest.mark.parametrize("fn", ["eigh", "eigh_mixed"])
def test_pair_v_split_bitwise(pj, fn):
    """Tiles of the V update taken by the pair-solve workgroups get the same
    per-tile arithmetic as the standalone update: forced splits agree bit for
    bit with serial_v = 1."""
    A = wl.goe(1024, 24)
    W0, V0, i0 = solve(pj, fn, A, pair_v_split=3)
    W1, V1, i1 = solve(pj, fn, A, serial_v=1)
    assert (i0["sweeps"], i0["sweeps32"]) == (i1["sweeps"], i1["sweeps32"])
    assert np.array_equal(W0, W1) and np.array_equal(V0, V1)


def test_stream_k_split_close_to_unsplit(pj):
    """The split symmetric products sum each split tile's two parts in a
    fix-up pass: the mixed solve with the split forced differs from the
    unsplit one only by rounding."""
    A = wl.goe(1024, 25)
    W0, V0, _ = solve(pj, "eigh_mixed", A, gemm_slots=16)
    W1, V1, _ = solve(pj, "eigh_mixed", A)
    assert np.abs(W0 - W1).max() <= 1e-13 * np.abs(W1).max()


# ------------------------------------------------------------ edge inputs
SCALE_CASES = [("eigh", 64, {}), ("eigh", 300, dict(small_max_n=-1)),
               ("eigh_mixed", 300, {})]


@pytest.mark.parametrize("k", [500, -500, 1000, -1000])
@pytest.mark.parametrize("fn,n,kw", SCALE_CASES, ids=[f"{c[0]}-{c[1]}" for c in SCALE_CASES])
def test_scaled_input(pj, fn, n, kw, k):
    """2^k A for |k| up to 1000: the library scales the input by an exact power
    of two on ingest and the eigenvalues back, so the result is 2^k times the
    result for A bit for bit, and within the bars of the oracle's result on A
    (the oracle itself is not run on 2^k A: its sums of squares would leave
    the FP64 range)."""
    A = wl.random_symmetric(n, 5000 + n)
    W0, V0, i0 = solve(pj, fn, A, **kw)
    Ws, Vs, i1 = solve(pj, fn, np.ldexp(A, k), **kw)
    assert i1["status"] == 0
    Wu = np.ldexp(Ws, -k)
    print(f"  2^{k}: bitwise W {np.array_equal(Wu, W0)} V {np.array_equal(Vs, V0)} "
          f"max|dW| {np.abs(Wu - W0).max():.2e}", flush=True)
    assert np.array_equal(Wu, W0) and np.array_equal(Vs, V0)
    assert i1["sweeps"] == i0["sweeps"] and i1["sweeps32"] == i0["sweeps32"]
    Wo, *_ = oracle.eigh(A)
    assert np.abs(Wu - Wo).max() <= 1e-13 * np.abs(Wo).max()
    bars(A, Wu, Vs, f"{fn} 2^{k}")


@pytest.mark.parametrize("fn", ["eigh", "eigh_mixed"])
def test_repeated_eigenvalues_block_path(pj, fn):
    """Q diag(1, ..., 1, 2, ..., 2) Q^T (two eigenvalues of multiplicity 130)
    through the block path: eigenvalues against the spectrum and the oracle,
    and the eigenvectors span the two eigenspaces (residual bar)."""
    n = 260
    lam = np.r_[np.ones(n // 2), 2 * np.ones(n // 2)]
    A = wl.from_spectrum(lam, wl.haar(n, wl.rng(51)))
    W, V, info = solve(pj, fn, A, small_max_n=-1)
    assert info["status"] == 0
    assert np.abs(W - lam).max() <= 1e-13 * 2
    # the oracle's eigenvalues as Rayleigh quotients of its eigenvectors: its
    # diagonal readout after the many sweeps this input takes drifts by about
    # 1.4e-13 ||A||_2 here
    Wo, Vo, *_ = oracle.eigh(A)
    rq, res = oracle.rayleigh(A, Vo)
    print(f"  oracle: |w - lam| {np.abs(Wo - lam).max():.2e} |rq - lam| "
          f"{np.abs(rq - lam).max():.2e}", flush=True)
    assert np.abs(W - rq).max() <= 1e-13 * 2
    bars(A, W, V, f"repeated {fn}")


@pytest.mark.parametrize("fn,n,kw", [("eigh", 40, {}), ("eigh", 200, dict(small_max_n=-1)),
                                     ("eigh_mixed", 200, {})])
def test_zero_diagonal(pj, fn, n, kw):
    """[[0, G], [G^T, 0]]: a zero diagonal (tau = 0 for every first rotation,
    t = 1) with eigenvalues +-sigma(G); against the oracle and the singular
    values."""
    g = wl.rng(52)
    G = g.standard_normal((n // 2, n // 2))
    A = np.zeros((n, n))
    A[: n // 2, n // 2:] = G
    A[n // 2:, : n // 2] = G.T
    W, V, info = solve(pj, fn, A, **kw)
    assert info["status"] == 0
    sv = np.linalg.svd(G, compute_uv=False)
    lam = np.sort(np.r_[sv, -sv])
    Wo, *_ = oracle.eigh(A)
    nrm2 = sv.max()
    assert np.abs(W - Wo).max() <= 1e-13 * nrm2
    assert np.abs(W - lam).max() <= 1e-13 * nrm2
    bars(A, W, V, f"zero diagonal {fn}")


@pytest.mark.parametrize("fn", ["eigh", "eigh_mixed"])
def test_pair_skip_active_vs_oracle(pj, fn):
    """Two decoupled diagonal blocks aligned to the block size: block pairs
    that join them stop rotating, tiles are left out of the FP64 updates, and
    the result still matches the oracle."""
    A, lam = wl.block_diagonal(320, sizes=[160, 160], seed=53)
    W, V, info = solve(pj, fn, A, small_max_n=-1, block=32)
    assert info["status"] == 0
    assert info["skipped_tiles"] > 0
    Wo, *_ = oracle.eigh(A)
    nrm2 = np.abs(lam).max()
    assert np.abs(W - Wo).max() <= 1e-13 * nrm2
    assert np.abs(W - lam).max() <= 1e-13 * nrm2
    bars(A, W, V, f"pair skip {fn}")


def test_nonfinite_mixed_and_batched(pj):
    """A NaN in the input: NONFINITE from the mixed path and per matrix from
    the batched path."""
    A = wl.random_symmetric(300, 54)
    A[7, 9] = np.nan
    with pytest.raises(pj.JacobiError) as e:
        pj.eigh_mixed(gpu(A))
    assert e.value.status == pj.NONFINITE
    B = wl.random_symmetric(9, 55)
    C = B.copy()
    C[1, 2] = np.inf
    packed = torch.tensor(np.r_[B.ravel(), C.ravel()], device="cuda")
    W, V, st = pj.eigh_batched(packed, [9, 9], check=False)
    assert st.cpu().tolist() == [0, pj.NONFINITE]
