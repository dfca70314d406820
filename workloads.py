"""Seeded synthetic inputs for the mixed-precision Jacobi eigensolver.

This module is shared by the tests, the benchmark and the smoke check.  It
holds no part of the eigensolver's arithmetic: it only draws random numbers
and assembles symmetric test matrices with a known (or GOE) spectrum.  Both
the CPU oracle and the GPU library receive its outputs as plain inputs.

Recipes (all use numpy ``Generator(PCG64(seed))``; a batch draws one child
seed per matrix from ``SeedSequence(seed).spawn(k)``):

* Haar-distributed orthogonal ``Q``: Householder QR of an i.i.d. N(0,1)
  matrix, with the columns rescaled by ``sign(diag(R))`` (zero signs count as
  +1) so the factor is uniquely defined.
* ``A = Q diag(lam) Q^T`` is formed in FP64 and then symmetrised as
  ``(A + A^T)/2``, the same clean-up the paper's test-matrix generator applies
  after forming its product (Appendix B, test matrices).

The five workloads:

``uniform``   n=64, lam i.i.d. U[-1, 1]                          (seed 1)
``geo``       n=1024, lam_i = s_i 10^(-6 i/(n-1)), s_i = +-1       (seed 2)
              (geometric singular values with random signs, kappa = 1e6,
              the paper's "geo" test family, Section 2.4)
``goe``       n=4096, A = (G + G^T)/2 with G i.i.d. N(0,1)         (seed 3)
``clustered`` 10000 matrices, n_i uniform in {8..128}; 5 cluster
              centres c_k ~ U[-1,1]; eigenvalue j joins cluster j mod 5
              with an offset U[-5e-9, 5e-9] (cluster width 1e-8)    (seed 4)
``gapped``    256 matrices of n=256, lam sorted in [-1, 1] with minimum
              gap >= 1e-3, built as sort(U[0, 2 - (n-1) 1e-3]) + i 1e-3 - 1
              (a uniform draw from the gapped simplex), plus the loss
              weights w ~ N(0,1)^n and C ~ N(0,1)^{n x n}          (seed 5)
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "rng", "haar", "from_spectrum", "uniform_spectrum", "geo_spectrum",
    "goe", "clustered_batch", "gapped_batch", "random_symmetric",
    "WORKLOADS",
]


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def haar(n: int, g: np.random.Generator) -> np.ndarray:
    """Haar orthogonal matrix from the Householder QR of a Gaussian matrix."""
    if n == 0:
        return np.zeros((0, 0))
    G = g.standard_normal((n, n))
    Q, R = np.linalg.qr(G)
    d = np.sign(np.diag(R))
    d[d == 0] = 1.0
    return Q * d[None, :]


def from_spectrum(lam: np.ndarray, Q: np.ndarray) -> np.ndarray:
    """A = Q diag(lam) Q^T, symmetrised."""
    A = (Q * lam[None, :]) @ Q.T
    return 0.5 * (A + A.T)


def uniform_spectrum(n: int = 64, seed: int = 1):
    """Known spectrum, lam i.i.d. U[-1, 1]. Returns (A, lam_sorted)."""
    g = rng(seed)
    lam = g.uniform(-1.0, 1.0, n)
    Q = haar(n, g)
    return from_spectrum(lam, Q), np.sort(lam)


def geo_spectrum(n: int = 1024, seed: int = 2, kappa: float = 1e6):
    """Geometric magnitudes 1 .. 1/kappa with Rademacher signs."""
    g = rng(seed)
    i = np.arange(n, dtype=np.float64)
    mag = kappa ** (-i / max(n - 1, 1))
    signs = g.choice(np.array([-1.0, 1.0]), n)
    lam = signs * mag
    Q = haar(n, g)
    return from_spectrum(lam, Q), np.sort(lam)


def ari_spectrum(n: int = 1024, seed: int = 6, kappa: float = 1e2):
    """Arithmetic magnitudes: |lambda_i| falls linearly from 1 to 1/kappa
    (the second family of test matrices of Section 2.4), Rademacher signs,
    Haar Q.  Returns (A, lam_sorted)."""
    g = rng(seed)
    i = np.arange(n, dtype=np.float64)
    mag = 1.0 - i / max(n - 1, 1) * (1.0 - 1.0 / kappa)
    signs = g.choice(np.array([-1.0, 1.0]), n)
    lam = signs * mag
    Q = haar(n, g)
    return from_spectrum(lam, Q), np.sort(lam)


def block_diagonal(n: int = 4096, nblocks: int = 8, seed: int = 9, sizes=None):
    """Decoupled subsystems: A = diag(A_1, ..., A_k) with zero coupling between
    the diagonal blocks, A_i = Q_i diag(lam_i) Q_i^T, lam_i uniform on
    [-1, 1], Haar Q_i.  `sizes` gives the block orders (default: nblocks equal
    blocks).  Returns (A, lam_sorted)."""
    g = rng(seed)
    if sizes is None:
        sizes = [n // nblocks] * nblocks
        sizes[-1] += n - sum(sizes)
    assert sum(sizes) == n
    A = np.zeros((n, n))
    lams = []
    o = 0
    for m in sizes:
        lam = g.uniform(-1.0, 1.0, m)
        A[o:o + m, o:o + m] = from_spectrum(lam, haar(m, g))
        lams.append(lam)
        o += m
    return A, np.sort(np.concatenate(lams))

def goe(n: int = 4096, seed: int = 3) -> np.ndarray:
    """A = (G + G^T)/2, G i.i.d. N(0,1); spectrum not known in closed form."""
    g = rng(seed)
    G = g.standard_normal((n, n))
    return 0.5 * (G + G.T)


def random_symmetric(n: int, seed: int) -> np.ndarray:
    """Small generic symmetric matrices for property tests."""
    return goe(n, seed)


def clustered_batch(batch: int = 10000, seed: int = 4, n_lo: int = 8,
                    n_hi: int = 128, n_clusters: int = 5,
                    width: float = 1e-8):
    """Uneven-n batch with tightly clustered spectra.

    Returns (ns, mats, lams): list of sizes, list of A_i, list of sorted lam_i.
    """
    g = rng(seed)
    ns = g.integers(n_lo, n_hi + 1, size=batch)
    children = np.random.SeedSequence(seed).spawn(batch)
    mats, lams = [], []
    for k, n in enumerate(ns):
        gk = np.random.Generator(np.random.PCG64(children[k]))
        centres = gk.uniform(-1.0, 1.0, n_clusters)
        j = np.arange(n)
        lam = centres[j % n_clusters] + gk.uniform(-0.5 * width, 0.5 * width, n)
        Q = haar(int(n), gk)
        mats.append(from_spectrum(lam, Q))
        lams.append(np.sort(lam))
    return [int(n) for n in ns], mats, lams


def gapped_batch(batch: int = 256, n: int = 256, seed: int = 5,
                 min_gap: float = 1e-3):
    """Known, well separated spectra plus the loss weights (w, C).

    Returns (mats, lams, ws, Cs): arrays of shape (batch, n, n), (batch, n),
    (batch, n), (batch, n, n).
    """
    children = np.random.SeedSequence(seed).spawn(batch)
    mats = np.empty((batch, n, n))
    lams = np.empty((batch, n))
    ws = np.empty((batch, n))
    Cs = np.empty((batch, n, n))
    span = 2.0 - (n - 1) * min_gap
    for k in range(batch):
        gk = np.random.Generator(np.random.PCG64(children[k]))
        u = np.sort(gk.uniform(0.0, span, n))
        lam = u + np.arange(n) * min_gap - 1.0
        Q = haar(n, gk)
        mats[k] = from_spectrum(lam, Q)
        lams[k] = lam
        ws[k] = gk.standard_normal(n)
        Cs[k] = gk.standard_normal((n, n))
    return mats, lams, ws, Cs


# name -> (description, builder) for the bench and the tests
WORKLOADS = {
    "uniform64": "n=64, lam ~ U[-1,1], Haar Q, plain FP64 Jacobi, tol 1e-15 n ||A||_F",
    "geo1024": "n=1024, lam_i = +-10^(-6 i/(n-1)), Haar Q, mixed vs plain FP64",
    "goe4096": "n=4096, A=(G+G^T)/2, mixed vs plain FP64",
    "clustered10000": "10000 matrices, n~U{8..128}, 5 clusters of width 1e-8",
    "gapped256x256": "256 matrices n=256, min gap 1e-3, loss sum w.lam + <C, V>",
}
