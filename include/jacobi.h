/*
 * libjacobi: mixed-precision Jacobi eigensolver for dense real symmetric
 * matrices, A = V diag(W) V^T, on AMD Instinct MI355X (gfx950).
 *
 * Method: Z. Zhou, "A Mixed Precision Eigensolver Based on the Jacobi
 * Algorithm" (arXiv 2509.00495).  Algorithm 4 (cyclic Jacobi, Section 3.3)
 * is run as a parallel round-robin block Jacobi; Algorithm 9 (Section 5.1)
 * replaces the single-precision eigensolver by the same Jacobi kernels in
 * FP32, orthogonalises with Newton-Schulz (Algorithm 8, Section 4.3.4) and
 * finishes with FP64 Jacobi sweeps on Q_d^T A Q_d.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Matrices are dense, ROW-MAJOR, FP64.  Row i of A starts at A + i*lda.
 * - All array arguments are DEVICE pointers owned by the caller, unless the
 *   argument says "host".  The library never frees or keeps them.
 * - `stream` is a hipStream_t passed as void* (NULL = the null stream).  Work
 *   is enqueued on it in order; a call returns after its last readback
 *   (convergence flags are read once per sweep), so outputs are ready on
 *   `stream` when the call returns.
 * - `work`/`work_bytes`: device scratch of at least jacobi_workspace_bytes()
 *   bytes, 256-byte aligned.  work == NULL makes the call allocate and free
 *   its own scratch (hipMalloc/hipFree, synchronising).
 * - A is read, never written; it is symmetrised on ingest, B = (A + A^T)/2.
 * - Outputs: W ascending; column k of V is the eigenvector of W[k], scaled by
 *   +-1 so its entry of largest magnitude (lowest row on ties) is positive.
 * - Errors: arguments are validated on the host before anything is launched;
 *   argument i invalid -> return -i (LAPACK convention).  Positive codes are
 *   listed below.
 */
#ifndef LIBJACOBI_H
#define LIBJACOBI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes (return values; negative = invalid argument position). */
#define JACOBI_OK 0
#define JACOBI_NOCONV 1     /* max_sweeps reached; outputs hold the last iterate */
#define JACOBI_NOTSYM 2     /* opts->check_symmetry and A != A^T exactly */
#define JACOBI_NONFINITE 3  /* A holds NaN or Inf (or the iteration produced one) */
#define JACOBI_DEGENERATE 4 /* backward: an eigenvalue gap < gap_tol with nonzero coupling */
#define JACOBI_DEVICE 5     /* a HIP runtime call failed */
#define JACOBI_WORKSPACE 6  /* work_bytes smaller than jacobi_workspace_bytes() */

/* Tuning and stopping options.  Zero-initialise and set what you need; a zero
 * field selects the default.  May be NULL. */
typedef struct jacobi_opts {
    int32_t max_sweeps;     /* per stage; default 30 */
    int32_t block;          /* block size b of the block path: 16 or 32; default
                               16 for n <= 160, else 32 */
    int32_t inner_sweeps;   /* inner sweeps of each 2b x 2b pair solve; default 1 */
    int32_t ns_iters;       /* Newton-Schulz iterations: 0 = the count of
                               Algorithm 8 (2 for n < 52 000, else 3); -1 =
                               adaptive as Algorithm 7 (stop once
                               ||I - X^T X||_F <= n u_d, at most 3); > 0 fixed */
    double c32;             /* FP32 stage stops at off <= c32 n u_l ||A||_F (or when a
                               sweep no longer lowers off); default 0.1 */
    int32_t check_symmetry; /* nonzero: return JACOBI_NOTSYM unless A == A^T exactly */
    int32_t small_max_n;    /* n up to which one workgroup solves the whole matrix;
                               default 128, 0 keeps the default, -1 forces the block path */
    int32_t threads;        /* threads per workgroup of the one-workgroup solver:
                               256, 512 or 1024; default by n (256 up to
                               n = 72, 1024 above) */
    int32_t timing;         /* nonzero: time every pair-solve and apply launch of
                               the block path with HIP events on `stream`
                               (results in jacobi_info.t_*) */
    int32_t schedule;       /* order of the rotations in a block-path sweep:
                               0 (default) = every index pair once per sweep:
                               the first round of a sweep rotates all pairs of
                               its 2b x 2b tiles, the others only pairs that
                               join the two blocks of a tile; 1 = all pairs of
                               every tile in every round */
    int32_t serial_v;       /* where the eigenvector update of a round runs:
                               0 (default) = inside the next round's
                               pair-solve launch, on the compute units the
                               pair solves leave free; 1 = on `stream` after
                               the round's B update; 2 = on a second,
                               library-owned stream beside the next round;
                               other values are rejected */
    int32_t tune;           /* batched path, when `threads` is 0: 0 (default) = the
                               workgroup size (256, 512 or 1024 threads) and the place
                               of V (LDS beside S, or global scratch) are
                               chosen by measurement: the first call for a
                               (device, n_max, batch size class) times every
                               candidate on its own input and keeps the
                               fastest for later calls; 1 = fixed choice by
                               n_max, without measuring */
    int32_t graph;          /* batched path: nonzero = issue the call's launches
                               as a hipGraph, captured on the first call with
                               a given set of arguments, workspace and tuned
                               configuration and replayed by later identical
                               calls (needs a caller workspace; ignored
                               without one; at most 64 graphs are kept per
                               process, later new argument sets launch
                               directly); 0 (default) = direct launches */
    int32_t no_pair_skip;   /* nonzero: the FP64 block sweeps update every B tile
                               and V column, also those of block pairs that
                               applied no rotation in a round (the results are
                               the same; 0, the default, leaves those out) */
    int32_t gemm_slots;     /* symmetric FP64 products of the mixed path (the
                               Newton-Schulz residual I - X^T X and
                               Q_d^T (A Q_d)): the number of resident
                               workgroups a product with more 128 x 128 upper
                               tiles than that is split over (stream-K with a
                               fix-up pass); 0 (default) = two per compute
                               unit.  A small value makes small orders take
                               the split path (used by the tests) */
    int32_t pair_v_split;   /* shared pair-solve + V-update launch of the block
                               path (2b = 64): 16-row tiles of each pair's V
                               update that its pair-solve workgroup takes once
                               its solve is done; 0 (default) = a timing model
                               (nonzero only near n = 4096 in FP64), -1 = none,
                               k > 0 = k tiles (at most what leaves every V
                               workgroup one tile) */
    int32_t orth;           /* mixed path, how Q_l becomes Q_d: 0 (default) =
                               Newton-Schulz (Algorithm 8, Section 4.3.4);
                               1 = Q of the Householder QR of Q_l (Algorithm 5,
                               Section 4.2), blocked; 2 = Q of its Cholesky QR
                               (X^T X = R^T R, Q = X R^-1).  1 and 2 are the
                               comparators of Section 4.4 */
    int32_t ladder;         /* mixed path: 1 = a binary16 stage first (the
                               lower-precision ladder named as further work,
                               Chapter 6): Jacobi sweeps with every stored
                               entry of B rounded to binary16 (FP32 arithmetic,
                               FP64 angles, V in FP32) until a sweep lowers off
                               by less than 10%, then B = Q_h^T A Q_h and the FP32
                               stage from V = Q_h; 0 (default) = none */
} jacobi_opts;

/* Diagnostics filled on return (host struct, may be NULL). */
typedef struct jacobi_info {
    int32_t sweeps;         /* FP64 sweeps (plain), or FP64-stage sweeps (mixed) */
    int32_t sweeps32;       /* FP32-stage sweeps (mixed only) */
    int32_t ns_iters;       /* Newton-Schulz iterations run (mixed only) */
    int32_t path;           /* 0 = one-workgroup solver, 1 = block path */
    int32_t block;          /* block size used by the block path */
    int32_t polished;       /* 1 if the output stage's Newton-Schulz step on V
                               ran (the estimate below exceeded 0.2 of the
                               1e-14 n bar) */
    int32_t skipped_tiles;  /* block path, FP64 sweeps: off-diagonal tile
                               updates of B left out because neither block
                               pair of the tile rotated in that round (U = I
                               there; the results are unchanged), summed over
                               the sweeps (a diagnostic: wraps past 2^31 - 1) */
    int32_t sweeps16;       /* binary16-stage sweeps (mixed path with opts->ladder) */
    double norm_f;          /* ||A||_F of the symmetrised input */
    double tol;             /* absolute threshold on off(B) actually used */
    double off_final;       /* off(B) when the FP64 stage stopped */
    double off32;           /* off(B32) when the FP32 stage stopped (mixed) */
    double off_cond;        /* off(Q_d^T A Q_d) before the FP64 stage (mixed) */
    double orth_ns;         /* ||I - X^T X||_F of the last Newton-Schulz step of
                               the mixed pipeline (the residual it corrected) */
    double orth_est;        /* block path: randomized estimate of ||V^T V - I||_F
                               of the accumulated eigenvectors with unit-norm
                               columns, before any Newton-Schulz step (4
                               Rademacher probes) */
    /* with opts->timing: summed kernel time (ms) and launch counts of the
     * block path, index 0 = FP64 stage, 1 = FP32 stage; "pair" is the launch
     * of a round's pair solves (with serial_v = 0 it also carries the previous
     * round's V update, as in untimed solves), "apply" the update of the
     * off-diagonal tiles of B, "applyv" a V update launched on its own (with
     * serial_v = 0 only the last round of each stage; the other rounds count
     * as zero-length launches) */
    double t_pair_ms[2];
    double t_apply_ms[2];
    double t_applyv_ms[2];
    int32_t n_pair[2];
    int32_t n_apply[2];
    int32_t n_applyv[2];
    int32_t reserved_i2[2];
    double orth_qd;         /* with opts->timing, mixed path: ||Q_d^T Q_d - I||_F of
                               the orthogonaliser's output (0 otherwise) */
    double t_orth_ms;       /* with opts->timing, mixed path: time of the Q_l -> Q_d
                               step (HIP events on `stream`) */
    double off16;           /* off(B) when the binary16 stage stopped (ladder) */
    double orth_ql;         /* mixed path: ||Q_l^T Q_l - I||_F of the FP32 stage's
                               eigenvectors (with Newton-Schulz always; with the
                               QR orthogonalisers only with opts->timing, else 0) */
} jacobi_info;

/* Plain FP64 Jacobi eigendecomposition (Algorithm 4, Section 3.3, run as a
 * round-robin block Jacobi; Alg. 2 angles with approach 2 of Appendix A).
 *   A    [in]  n x n, leading dimension lda >= max(1, n)
 *   n    [in]  order, n >= 0 (n = 0 is a no-op)
 *   W    [out] n eigenvalues, ascending
 *   V    [out] n x n eigenvectors (columns), leading dimension ldv >= max(1, n);
 *              every column is scaled to unit 2-norm and its entry of
 *              largest magnitude is positive
 *   tol  [in]  stop when off(B) <= tol (absolute); tol <= 0 selects
 *              1e-15 * n * ||A||_F.  NaN is an invalid argument.
 * Returns JACOBI_OK, JACOBI_NOCONV (outputs still written), JACOBI_NOTSYM,
 * JACOBI_NONFINITE (outputs not written), JACOBI_DEVICE, JACOBI_WORKSPACE or -i.
 * Argument positions for -i: A 1, n 2, lda 3, W 4, V 5, ldv 6, tol 7, opts 8. */
int jacobi_eigh(const double *A, int64_t n, int64_t lda, double *W, double *V,
                int64_t ldv, double tol, const jacobi_opts *opts, void *work,
                size_t work_bytes, void *stream, jacobi_info *info);

/* Mixed-precision eigendecomposition (Algorithm 9, Section 5.1): FP32 Jacobi
 * on fl32(A) gives Q_l (angles in FP64, updates on FP32 MFMA), Newton-Schulz in
 * FP64 gives Q_d (Section 4.3.4), then FP64 Jacobi on B = Q_d^T A Q_d starting
 * from V = Q_d until off(B) <= tol.  Same arguments and results as jacobi_eigh. */
int jacobi_eigh_mixed(const double *A, int64_t n, int64_t lda, double *W,
                      double *V, int64_t ldv, double tol,
                      const jacobi_opts *opts, void *work, size_t work_bytes,
                      void *stream, jacobi_info *info);

/* Batched eigendecomposition of matrices of uneven order in one persistent
 * launch (each workgroup pops matrices from a device work queue, largest
 * first, and runs Algorithm 4, Section 3.3, on the whole matrix in LDS).
 * A batch whose orders are all equal and above 128 runs on the block path
 * instead (the parallel block Jacobi of jacobi_eigh, Section 3.3): one launch
 * per step serves every matrix still sweeping, ingest and output stay per
 * matrix, and each matrix's W, V and status are bitwise those of jacobi_eigh
 * on it with the same opts (opts.timing, serial_v, graph, tune and threads do
 * not apply there; the workspace holds one single-solve workspace per matrix).
 * That path synchronises with the host between sweeps: on a stream being
 * captured into a HIP graph it returns JACOBI_DEVICE before launching.
 *   A      [in]  matrix i is n_i x n_i row-major (ld = n_i) at offset a_off[i]
 *                doubles
 *   n      [in, HOST] batch orders, 1 <= n_i <= 128, or all equal (any order
 *                up to 2^20)
 *   a_off  [in, HOST] batch offsets of the matrices in A (and of the
 *                eigenvectors in V), in doubles, >= 0; NULL = packed
 *                (sum_{j<i} n_j^2)
 *   batch  [in]  number of matrices, >= 0 (at most 65535 for the block path)
 *   W      [out] n_i eigenvalues of matrix i at offset w_off[i]
 *   w_off  [in, HOST] batch offsets into W, >= 0; NULL = packed (sum_{j<i} n_j)
 *   V      [out] eigenvectors of matrix i, n_i x n_i row-major at a_off[i]
 *   tol    [in]  absolute threshold on off for every matrix; <= 0 selects
 *                1e-15 * n_i * ||A_i||_F per matrix
 *   mixed  [in]  reserved, must be 0 (the batched path is plain FP64)
 *   status [out] batch int32 per-matrix status codes (device), may be NULL
 * Output regions of different matrices must not overlap (nothing checks it).
 * Returns the largest per-matrix status, or -i, JACOBI_DEVICE, JACOBI_WORKSPACE.
 * Argument positions for -i: A 1, n 2, a_off 3, batch 4, W 5, w_off 6, V 7,
 * tol 8, mixed 9, opts 10. */
int jacobi_eigh_batched(const double *A, const int64_t *n, const int64_t *a_off,
                        int64_t batch, double *W, const int64_t *w_off, double *V,
                        double tol, int mixed, const jacobi_opts *opts, void *work,
                        size_t work_bytes, void *stream, int32_t *status);

/* Adjoint of the eigendecomposition for a batch of equal-order matrices
 * (first-order perturbation theory for distinct eigenvalues; the paper does
 * not treat derivatives):
 *   dA = sym(V (diag(dW) + F o (V^T dV)) V^T),  F_ij = 1/(W_j - W_i), F_ii = 0,
 *   sym(G) = (G + G^T)/2.
 *   W  [in]  batch x n eigenvalues as returned by jacobi_eigh (packed)
 *   V  [in]  batch matrices of n x n eigenvectors, row-major with row stride
 *            ld, matrix k at V + k * n * ld
 *   dW [in]  batch x n (packed), or NULL (zero)
 *   dV [in]  laid out like V, or NULL (zero)
 *   n  [in]  order, >= 0;  ld [in] >= max(1, n);  batch [in] >= 0
 *   dA [out] laid out like V, symmetric
 *   gap_tol [in] pairs with |W_j - W_i| < gap_tol get F_ij = 0; if such a
 *           pair has nonzero (V^T dV)_ij the call returns JACOBI_DEGENERATE
 *           (dA is still written).
 * Returns JACOBI_OK, JACOBI_DEGENERATE, JACOBI_DEVICE, JACOBI_WORKSPACE or -i
 * (positions: W 1, V 2, dW 3, dV 4, n 5, ld 6, batch 7, dA 8, gap_tol 9). */
int jacobi_eigh_backward(const double *W, const double *V, const double *dW,
                         const double *dV, int64_t n, int64_t ld, int64_t batch,
                         double *dA, double gap_tol, void *work,
                         size_t work_bytes, void *stream);

/* jacobi_eigh_batched for callers that cannot allocate: code being captured
 * into a HIP graph, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments, results and status codes as jacobi_eigh_batched for orders
 * 1 <= n_i <= 128 (larger orders return -2), without
 * work/work_bytes: the call allocates nothing (no hipMalloc/hipFree, no
 * host heap, no events or streams) and takes its scratch from a fixed
 * 64 MiB device array that each GPU the library runs on holds until the
 * process ends.  The descriptor table is built on the device; the launch
 * configuration is the one the batched autotuner stored for this (device,
 * n_max, batch size class, workgroup size) if any, else the fixed choice by
 * n_max (nothing is measured and no graph is used here).  A batch whose
 * scratch (about 76 bytes per matrix plus the eigenvector scratch of the
 * resident workgroups, about 32 MiB at n_max = 128) exceeds the array
 * returns JACOBI_WORKSPACE before anything is launched.  Every call on one
 * GPU uses that GPU's array and leaves its contents behind (the call clears
 * what must start at zero); calls that overlap on one GPU race. */
int jacobi_eigh_batched_noalloc(const double *A, const int64_t *n,
                                const int64_t *a_off, int64_t batch, double *W,
                                const int64_t *w_off, double *V, double tol,
                                int mixed, const jacobi_opts *opts,
                                void *stream, int32_t *status);

/* Workspace query (LAPACK style).  op: 0 = eigh, 1 = eigh_mixed,
 * 2 = eigh_batched (n_max = largest order, batch = count; above 128 the
 * block path's batch of one order),
 * 3 = eigh_backward (n_max = n).  Returns bytes; 0 for invalid op. */
size_t jacobi_workspace_bytes(int op, int64_t n_max, int64_t batch,
                              const jacobi_opts *opts);

/* Human-readable text for a status code (static storage). */
const char *jacobi_status_string(int status);

/* Library version string (static storage). */
const char *jacobi_version(void);

/* One line describing the current HIP device (name, arch, CU count, LDS per
 * workgroup, clocks) written into buf (host, len bytes).  Returns
 * JACOBI_OK or JACOBI_DEVICE. */
int jacobi_device_summary(char *buf, size_t len);

/* Text of the last HIP runtime error seen by a call of this thread that
 * returned JACOBI_DEVICE (static storage). */
const char *jacobi_last_hip_error(void);

#ifdef __cplusplus
}
#endif

#endif /* LIBJACOBI_H */
