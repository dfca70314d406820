"""GPU parity of the batched solver and of the adjoint, through the C ABI."""
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
    return torch.tensor(np.concatenate([m.ravel() for m in mats]), dtype=torch.float64,
                        device="cuda")


def _unpack(W, V, ns):
    W, V = W.cpu().numpy(), V.cpu().numpy()
    out, wo, vo = [], 0, 0
    for n in ns:
        out.append((W[wo:wo + n], V[vo:vo + n * n].reshape(n, n)))
        wo += n
        vo += n * n
    return out


def _check(A, W, V, Wref, label):
    n = A.shape[0]
    nrm2 = max(np.abs(Wref).max(), 1e-300)
    assert np.abs(W - Wref).max() <= 1e-13 * nrm2, label
    assert np.linalg.norm(A @ V - V * W) / np.linalg.norm(A) <= 1e-13 * n, label
    assert np.linalg.norm(V.T @ V - np.eye(n)) <= 1e-14 * n, label


def test_batched_uneven_vs_oracle(pj):
    g = wl.rng(11)
    ns = [int(x) for x in g.integers(1, 129, 60)] + [1, 2, 3, 128, 127, 64, 65]
    mats = [wl.random_symmetric(n, 500 + k) for k, n in enumerate(ns)]
    print(f"  -> eigh_batched batch={len(ns)} n_max={max(ns)}", flush=True)
    W, V, st = pj.eigh_batched(_pack(mats), ns)
    torch.cuda.synchronize()
    assert (st.cpu().numpy() == 0).all()
    for k, (A, (Wk, Vk)) in enumerate(zip(mats, _unpack(W, V, ns))):
        Wo, *_ = oracle.eigh(A)
        _check(A, Wk, Vk, Wo, f"matrix {k} n={ns[k]}")


def test_batched_clustered_sample(pj):
    """The clustered workload shape (5 clusters of width 1e-8), 200 matrices."""
    ns, mats, lams = wl.clustered_batch(batch=200, seed=4)
    print(f"  -> eigh_batched clustered batch=200", flush=True)
    W, V, st = pj.eigh_batched(_pack(mats), ns)
    torch.cuda.synchronize()
    assert (st.cpu().numpy() == 0).all()
    for k, (A, lam, (Wk, Vk)) in enumerate(zip(mats, lams, _unpack(W, V, ns))):
        _check(A, Wk, Vk, lam, f"clustered {k}")


def test_batched_matches_single(pj):
    """The persistent batched launch and the single-matrix call agree bitwise
    (same kernel, same per-matrix arithmetic)."""
    ns = [17, 64, 100]
    mats = [wl.random_symmetric(n, 900 + n) for n in ns]
    W, V, st = pj.eigh_batched(_pack(mats), ns)
    for A, (Wk, Vk) in zip(mats, _unpack(W, V, ns)):
        W1, V1 = pj.eigh(torch.tensor(A, device="cuda"))
        assert np.array_equal(W1.cpu().numpy(), Wk)
        assert np.array_equal(V1.cpu().numpy(), Vk)


def test_backward_vs_oracle(pj):
    mats, lams, ws, Cs = wl.gapped_batch(batch=3, n=32, seed=5)
    Wt, Vt = [], []
    for A in mats:
        W, V = pj.eigh(torch.tensor(A, device="cuda"))
        Wt.append(W)
        Vt.append(V)
    Wt, Vt = torch.stack(Wt), torch.stack(Vt)
    dW = torch.tensor(ws, device="cuda")
    dV = torch.tensor(Cs, device="cuda")
    print("  -> eigh_backward batch=3 n=32", flush=True)
    dA, st = pj.eigh_backward(Wt, Vt, dW, dV, return_status=True)
    assert st == 0
    dA = dA.cpu().numpy()
    for k in range(3):
        ref, st = oracle.eigh_backward(Wt[k].cpu().numpy(), Vt[k].cpu().numpy(), ws[k], Cs[k])
        assert np.abs(dA[k] - ref).max() <= 1e-12 * max(np.abs(ref).max(), 1.0)
        assert np.abs(dA[k] - dA[k].T).max() == 0.0


def test_backward_closed_forms(pj):
    A, lam = wl.uniform_spectrum(40, 3)
    W, V = pj.eigh(torch.tensor(A, device="cuda"))
    dA = pj.eigh_backward(W, V, dW=torch.ones_like(W)).cpu().numpy()
    assert np.abs(dA - np.eye(40)).max() < 1e-13
    dA = pj.eigh_backward(W, V, dW=2 * W).cpu().numpy()
    assert np.abs(dA - 2 * A).max() < 1e-13


def test_backward_degenerate(pj):
    W = torch.tensor([[1.0, 1.0, 2.0]], device="cuda", dtype=torch.float64)
    V = torch.eye(3, device="cuda", dtype=torch.float64)[None].contiguous()
    dV = torch.ones((1, 3, 3), device="cuda", dtype=torch.float64)
    dA, st = pj.eigh_backward(W, V, dV=dV, gap_tol=1e-12, return_status=True)
    assert st == pj.DEGENERATE
    assert torch.isfinite(dA).all()


def test_autograd_central_fd(pj):
    """loss = sum w_i lam_i + <C, V>: autograd through EighFn vs central
    differences (h = 1e-6) of the GPU forward itself."""
    n = 24
    lam = np.sort(wl.rng(21).uniform(-1, 1, n)) + np.arange(n) * 0.02
    A = wl.from_spectrum(lam, wl.haar(n, wl.rng(22)))
    g = wl.rng(23)
    w = torch.tensor(g.standard_normal(n), device="cuda")
    C = torch.tensor(g.standard_normal((n, n)), device="cuda")
    At = torch.tensor(A, device="cuda", requires_grad=True)
    W, V = pj.eigh_autograd(At)
    loss = (w * W).sum() + (C * V).sum()
    loss.backward()
    G = At.grad.cpu().numpy()

    def f(M):
        W, V = pj.eigh(torch.tensor(M, device="cuda"), tol=1e-300 + 1e-30)
        return float((w * W).sum() + (C * V).sum())

    h = 1e-6
    for k in range(3):
        E = g.standard_normal((n, n))
        E = 0.5 * (E + E.T)
        fd = (f(A + h * E) - f(A - h * E)) / (2 * h)
        assert (G * E).sum() == pytest.approx(fd, rel=1e-5, abs=1e-7)
