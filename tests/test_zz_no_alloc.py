"""jacobi_eigh_batched_noalloc (the batched solve with the library's fixed
device scratch, for callers that cannot allocate) against jacobi_eigh_batched
through the C ABI: two calls in a row, the second with a smaller batch, and
one with explicit (non-packed) offsets.  With the same workgroup size both
entry points run the same kernel arithmetic, so the outputs agree bit for
bit; a few matrices are also checked against the oracle."""
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
    return torch.tensor(np.concatenate([m.ravel() for m in mats]), device="cuda")


def _solve_both(pj, mats, ns, threads):
    A = _pack(mats)
    opts = pj.make_opts(threads=threads)
    print(f"  -> batched batch={len(ns)} n_max={max(ns)} threads={threads}", flush=True)
    W0, V0, s0 = pj.eigh_batched(A, ns, opts=opts)
    W1 = torch.full_like(W0, float("nan"))
    V1 = torch.full_like(V0, float("nan"))
    s1 = torch.full_like(s0, -1)
    print(f"  -> batched_noalloc batch={len(ns)}", flush=True)
    st = pj.eigh_batched_noalloc(A, ns, W1, V1, s1, opts=opts)
    torch.cuda.synchronize()
    return (W0, V0, s0), (W1, V1, s1), st


@pytest.mark.parametrize("threads", [256, 1024])
def test_noalloc_matches_batched_two_calls(pj, threads):
    ns1, mats1, lams1 = wl.clustered_batch(batch=300, seed=71)
    ns2, mats2, lams2 = wl.clustered_batch(batch=40, seed=72, n_lo=4, n_hi=40)
    for ns, mats, lams in ((ns1, mats1, lams1), (ns2, mats2, lams2)):
        (W0, V0, s0), (W1, V1, s1), st = _solve_both(pj, mats, ns, threads)
        assert st == 0
        assert torch.equal(s0, s1) and int(s1.max()) == 0
        assert torch.equal(W0, W1) and torch.equal(V0, V1)
        Wn = W1.cpu().numpy()
        o = 0
        for k, (n, A, lam) in enumerate(zip(ns, mats, lams)):
            w = Wn[o:o + n]
            assert np.abs(w - lam).max() <= 1e-13 * np.abs(lam).max()
            if k < 3:
                Wo, *_ = oracle.eigh(A)
                assert np.abs(w - Wo).max() <= 1e-13 * np.abs(Wo).max()
            o += n


def test_noalloc_offsets_and_validation(pj):
    """Matrices at explicit offsets with gaps: the gaps stay untouched."""
    ns, mats, _ = wl.clustered_batch(batch=5, seed=73, n_lo=8, n_hi=30)
    a_off, w_off, ao, wo = [], [], 7, 3
    for n in ns:
        a_off.append(ao)
        w_off.append(wo)
        ao += n * n + 5
        wo += n + 2
    A = torch.zeros(ao, dtype=torch.float64, device="cuda")
    for n, M, o in zip(ns, mats, a_off):
        A[o:o + n * n] = torch.tensor(M.ravel(), device="cuda")
    V = torch.full((ao,), 7.0, dtype=torch.float64, device="cuda")
    W = torch.full((wo,), 7.0, dtype=torch.float64, device="cuda")
    s = torch.full((5,), -1, dtype=torch.int32, device="cuda")
    st = pj.eigh_batched_noalloc(A, ns, W, V, s, a_off=a_off, w_off=w_off)
    torch.cuda.synchronize()
    assert st == 0 and int(s.max()) == 0
    Wn, Vn = W.cpu().numpy(), V.cpu().numpy()
    mask_w = np.ones(wo, bool)
    mask_v = np.ones(ao, bool)
    for n, M, o, q in zip(ns, mats, a_off, w_off):
        Wo, *_ = oracle.eigh(M)
        assert np.abs(Wn[q:q + n] - Wo).max() <= 1e-13 * np.abs(Wo).max()
        Vk = Vn[o:o + n * n].reshape(n, n)
        assert np.linalg.norm(M @ Vk - Vk * Wn[q:q + n]) <= 1e-13 * n * np.linalg.norm(M)
        mask_w[q:q + n] = False
        mask_v[o:o + n * n] = False
    assert (Wn[mask_w] == 7.0).all() and (Vn[mask_v] == 7.0).all()
    # a batch whose scratch (about 60 bytes per matrix) exceeds the fixed
    # 64 MiB array: rejected before any launch or copy.  The buffers are sized
    # for the whole batch all the same, so that the call would be valid if it
    # were accepted.
    nb = 1 << 21
    big = [8] * nb
    Ab = torch.zeros(nb * 64, dtype=torch.float64, device="cuda")
    Vb = torch.zeros(nb * 64, dtype=torch.float64, device="cuda")
    Wb = torch.zeros(nb * 8, dtype=torch.float64, device="cuda")
    sb = torch.full((nb,), -1, dtype=torch.int32, device="cuda")
    st = pj.eigh_batched_noalloc(Ab, big, Wb, Vb, sb)
    torch.cuda.synchronize()
    assert st == pj.WORKSPACE
    assert int(sb.min()) == -1 and int(sb.max()) == -1
