"""Batches of one order above 128 through jacobi_eigh_batched: the block path
with one launch per step for the whole batch.  Every matrix's W, V and status
must be bitwise those of jacobi_eigh on it with the same options (the batch
runs each matrix through the launches of a single solve), and the full
differentiation workload (256 matrices of order 256) must meet the bars
against its constructed spectra."""
import time

import numpy as np
import pytest

import oracle
import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def pj():
    import paper_2509_00495_amd as pj
    return pj


def _pack(mats):
    return torch.tensor(np.concatenate([np.asarray(m).ravel() for m in mats]),
                        dtype=torch.float64, device="cuda")


def _single(pj, A, tol, opts):
    """(W, V, status) of jacobi_eigh on one matrix; W, V None when the call
    writes no outputs."""
    try:
        W, V, info = pj.eigh(torch.tensor(A, device="cuda"), tol, opts=opts, check=False,
                             return_info=True)
    except pj.JacobiError as e:
        return None, None, e.status
    torch.cuda.synchronize()
    return W.cpu().numpy(), V.cpu().numpy(), info["status"]


def _mixed_set(n):
    """Matrices whose solves end differently: GOE, a known spectrum, decoupled
    blocks (pair skipping acts), a diagonal matrix (no sweep), the zero
    matrix, a GOE scaled by 2^-600 and by 2^+600 (exact power-of-two scaling on
    ingest), and a matrix holding a NaN (non-finite: no outputs)."""
    mats = [wl.goe(n, 31), wl.uniform_spectrum(n, 32)[0],
            wl.block_diagonal(n, 4, 33)[0], np.diag(np.linspace(-1.0, 1.0, n)),
            np.zeros((n, n)), np.ldexp(wl.goe(n, 34), -600), np.ldexp(wl.goe(n, 35), 600)]
    bad = wl.goe(n, 36)
    bad[3, 5] = bad[5, 3] = np.nan
    mats.append(bad)
    mats.append(wl.goe(n, 37))
    return mats


@pytest.mark.parametrize("n", [150, 256])
def test_block_batch_bitwise_vs_single(pj, n):
    mats = _mixed_set(n)
    ns = [n] * len(mats)
    print(f"  -> block batch n={n} batch={len(mats)}", flush=True)
    W, V, st = pj.eigh_batched(_pack(mats), ns, check=False)
    torch.cuda.synchronize()
    W, V, st = W.cpu().numpy(), V.cpu().numpy(), st.cpu().numpy()
    for k, A in enumerate(mats):
        Ws, Vs, ss = _single(pj, A, None, None)
        assert st[k] == ss, (k, st[k], ss)
        if Ws is None:
            continue
        assert np.array_equal(W[k * n:(k + 1) * n], Ws), k
        assert np.array_equal(V[k * n * n:(k + 1) * n * n].reshape(n, n), Vs), k
    assert list(st[:7]) == [0] * 7 and st[7] == pj.NONFINITE and st[8] == 0
    # the GOE matrix against the oracle
    Wo, *_ = oracle.eigh(mats[0])
    assert np.abs(W[:n] - Wo).max() <= 1e-13 * np.abs(Wo).max()


def test_block_batch_options_bitwise(pj):
    """Explicit tol, max_sweeps (matrices stop with NOCONV at different
    points), the full schedule and no pair skipping: still bitwise the single
    solves with the same options."""
    n = 200
    mats = [wl.goe(n, 41), wl.geo_spectrum(n, 42, kappa=1e4)[0], wl.goe(n, 43)]
    ns = [n] * len(mats)
    for opts, tol in ((pj.make_opts(max_sweeps=3), None),
                      (pj.make_opts(schedule=1, no_pair_skip=1), None),
                      (None, 1e-9)):
        W, V, st = pj.eigh_batched(_pack(mats), ns, tol=tol, opts=opts, check=False)
        torch.cuda.synchronize()
        W, V, st = W.cpu().numpy(), V.cpu().numpy(), st.cpu().numpy()
        for k, A in enumerate(mats):
            Ws, Vs, ss = _single(pj, A, tol, opts)
            assert st[k] == ss, (k, st[k], ss)
            assert np.array_equal(W[k * n:(k + 1) * n], Ws), k
            assert np.array_equal(V[k * n * n:(k + 1) * n * n].reshape(n, n), Vs), k


def test_block_batch_uneven_large_rejected(pj):
    mats = [wl.goe(130, 1), wl.goe(140, 2)]
    with pytest.raises(pj.JacobiError) as e:
        pj.eigh_batched(_pack(mats), [130, 140])
    assert e.value.status == -2


def test_block_batch_full_differentiation_workload(pj):
    """The 256 x (n = 256) gapped batch in one call: every matrix within the
    bars of its constructed spectrum; the call's time against 256 single
    solves (printed)."""
    mats, lams, _, _ = wl.gapped_batch()
    b, n = lams.shape
    A = torch.tensor(mats, device="cuda")
    W, V, st = pj.eigh_batched(A.reshape(-1), [n] * b)  # warm-up
    torch.cuda.synchronize()
    t = time.perf_counter()
    W, V, st = pj.eigh_batched(A.reshape(-1), [n] * b)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    t = time.perf_counter()
    singles = [pj.eigh(A[k]) for k in range(8)]
    torch.cuda.synchronize()
    dt1 = (time.perf_counter() - t) / 8
    print(f"  batched {1e3 * dt:.1f} ms for {b} matrices; single solves {1e3 * dt1:.2f} ms each",
          flush=True)
    assert (st.cpu().numpy() == 0).all()
    W = W.cpu().numpy().reshape(b, n)
    V = V.cpu().numpy().reshape(b, n, n)
    # a batch this large gives each pair-solve workgroup its pair's V columns
    # (no separate V workgroups): still bitwise the single solves
    for k, (Ws, Vs) in enumerate(singles):
        assert np.array_equal(W[k], Ws.cpu().numpy()), k
        assert np.array_equal(V[k], Vs.cpu().numpy()), k
    for k in range(b):
        Ak, Wk, Vk = mats[k], W[k], V[k]
        assert np.abs(Wk - lams[k]).max() <= 1e-13 * np.abs(lams[k]).max(), k
        assert np.linalg.norm(Ak @ Vk - Vk * Wk) / np.linalg.norm(Ak) <= 1e-13 * n, k
        assert np.linalg.norm(Vk.T @ Vk - np.eye(n)) <= 1e-14 * n, k


def test_block_batch_two_host_threads(pj):
    """Two host threads, each on its own stream and workspace, run block-path
    batches at the same time (they share the library's pool streams): every
    result is bitwise that of the same call made alone."""
    import threading
    n = 200
    sets = [[wl.goe(n, 51 + k) for k in range(4)], [wl.goe(n, 61 + k) for k in range(4)]]
    alone = []
    for mats in sets:
        W, V, st = pj.eigh_batched(_pack(mats), [n] * len(mats), ws=pj.Workspace())
        torch.cuda.synchronize()
        alone.append((W.cpu().numpy(), V.cpu().numpy(), st.cpu().numpy()))
    out = [None, None]
    errs = []

    def work(i):
        try:
            stream = torch.cuda.Stream()
            ws = pj.Workspace()
            A = _pack(sets[i])
            torch.cuda.synchronize()
            with torch.cuda.stream(stream):
                for _ in range(3):
                    W, V, st = pj.eigh_batched(A, [n] * len(sets[i]), ws=ws)
                stream.synchronize()
            out[i] = (W.cpu().numpy(), V.cpu().numpy(), st.cpu().numpy())
        except Exception as e:  # reported below
            errs.append(e)

    print("  -> two threads, block-path batches of 4 at n=200", flush=True)
    th = [threading.Thread(target=work, args=(i,)) for i in range(2)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    assert not errs, errs
    for i in range(2):
        for a, b in zip(out[i], alone[i]):
            assert np.array_equal(a, b), i


def test_block_batch_offsets_and_workspace(pj):
    """Matrices at explicit, non-packed offsets (gaps between them, eigenvalues
    scattered), through the C ABI with a caller workspace: one byte short of
    jacobi_workspace_bytes returns JACOBI_WORKSPACE before anything runs, the
    exact size solves; every matrix bitwise its single solve."""
    import ctypes
    n, b = 160, 3
    mats = [wl.goe(n, 71 + k) for k in range(b)]
    a_off = [0, n * n + 37, 2 * n * n + 1000]
    w_off = [500, 3, 250]
    tot = a_off[-1] + n * n
    A = torch.zeros(tot, dtype=torch.float64, device="cuda")
    for k, M in enumerate(mats):
        A[a_off[k]:a_off[k] + n * n] = torch.tensor(M.ravel(), device="cuda")
    W = torch.full((700,), 7.0, dtype=torch.float64, device="cuda")
    V = torch.zeros(tot, dtype=torch.float64, device="cuda")
    st = torch.zeros(b, dtype=torch.int32, device="cuda")
    lib = pj.jacobi._lib()
    need = pj.workspace_bytes(2, n, b)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    i64 = ctypes.c_int64 * b
    args = lambda nbytes: (A.data_ptr(), i64(*[n] * b), i64(*a_off), b, W.data_ptr(),
                           i64(*w_off), V.data_ptr(), 0.0, 0, None, ws.data_ptr(), nbytes,
                           ctypes.c_void_p(torch.cuda.current_stream().cuda_stream),
                           st.data_ptr())
    print(f"  -> block batch n={n} at offsets {a_off}, workspace {need} bytes", flush=True)
    assert lib.jacobi_eigh_batched(*args(need - 1)) == pj.WORKSPACE
    assert lib.jacobi_eigh_batched(*args(need)) == 0
    torch.cuda.synchronize()
    Wh, Vh = W.cpu().numpy(), V.cpu().numpy()
    assert (st.cpu().numpy() == 0).all()
    for k, M in enumerate(mats):
        Ws, Vs, ss = _single(pj, M, None, None)
        assert np.array_equal(Wh[w_off[k]:w_off[k] + n], Ws), k
        assert np.array_equal(Vh[a_off[k]:a_off[k] + n * n].reshape(n, n), Vs), k
    # the gaps are untouched
    assert (Vh[n * n:n * n + 37] == 0).all() and (Wh[163:250] == 7.0).all()
