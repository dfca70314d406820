// Internal declarations of libjacobi: kernel descriptors and launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <type_traits>
#include <stddef.h>
#include <stdint.h>

#include <vector>

#include "../../include/jacobi.h"
#include <hip/hip_ext.h>

namespace lj {

// One matrix of the one-workgroup solver.  Offsets are in doubles from the
// base pointers passed to the launch.
struct SmallDesc {
    int64_t a_off, w_off, v_off;
    int32_t n, lda, ldv, orig;
    double *info; // optional device output: sweeps, ||A||_F, tol, off
};

// ---- one-workgroup solver (kernels_small.hip)
size_t small_smem_bytes(int m_max, int pool);
// doubles of the one-workgroup solver's eigenvector store for order n: V is
// kept transposed, m = n rounded up to 4 rows of (n rounded up to 2) entries
__host__ __device__ inline int64_t small_vt_elems(int64_t n)
{
    return ((n + 3) & ~(int64_t)3) * ((n + 1) & ~(int64_t)1);
}
hipError_t launch_small(const double *A, double *W, double *V, const SmallDesc *desc,
                        int count, int *queue, double tol, int max_sweeps,
                        double *vscratch, int64_t vscratch_stride, int pool,
                        int m_max, int nthreads, int grid, int32_t *status,
                        hipStream_t stream);
int small_max_active(int m_max, int pool, int nthreads);

// a launch with nothing to do: its timing events (if any) are recorded back
// to back, so that reading them gives zero instead of an error
inline hipError_t record_pair(hipEvent_t e0, hipEvent_t e1, hipStream_t s)
{
    if (e0) {
        hipError_t e = hipEventRecord(e0, s);
        if (e != hipSuccess)
            return e;
        return hipEventRecord(e1, s);
    }
    return hipSuccess;
}

// Launch on `s`; with e0 and e1 (timing events) the launch records them at the
// kernel's own start and end (hipExtLaunchKernel), so their difference is the
// kernel's duration without the gaps that separate event records add.
template <typename F, typename... Args>
inline void launch_timed(F kernel, dim3 grid, dim3 block, uint32_t shm, hipStream_t s,
                         hipEvent_t e0, hipEvent_t e1, Args... args)
{
    if (e0)
        hipExtLaunchKernelGGL(kernel, grid, block, shm, s, e0, e1, 0, args...);
    else
        hipLaunchKernelGGL(kernel, grid, block, shm, s, args...);
}

// ---- block path (kernels_block.hip); T = double or float
// A batch of equal-order solves in one launch per step (blockIdx.y = matrix):
// every matrix's buffers sit at the same offsets of equally sized workspace
// regions sW bytes apart, so each kernel moves its workspace pointers by
// m sW; the pair tables are shared.  act (device, count ints, or null): a
// matrix whose entry is 0 is left alone (its workgroups return at once);
// thr (device, count doubles, or null): per-matrix absolute rotation
// thresholds replacing the scalar one.
struct Batch {
    int64_t count = 1;
    int64_t sW = 0;
    const int *act = nullptr;
    const double *thr = nullptr;
};
// (byte arithmetic on the pointer itself: an integer round trip would lose
// its global address space and turn every access into a flat one)
template <typename P>
__device__ __forceinline__ P *bat(P *p, int64_t m, int64_t sW)
{
    typedef typename std::conditional<std::is_const<P>::value, const char, char>::type C;
    return p ? reinterpret_cast<P *>(reinterpret_cast<C *>(p) + m * sW) : p;
}
inline bool batched(const Batch &bt)
{
    return bt.count > 1 || bt.sW != 0 || bt.act != nullptr || bt.thr != nullptr;
}

template <typename T>
hipError_t launch_pair_solve(T *B, int64_t ldb, int b, int npairs, const int2 *pairs,
                             const int2 *psmap, T *U, double eps, double thr, int inner, int r16,
                             int cross, double *partial, int *rot_flag, int *prot,
                             hipStream_t s, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr,
                             const Batch &bt = Batch());
// the same pair solves, plus the V update V[:, cols] <- V[:, cols] vU of the
// previous round (pairs vpairs, rotations vU, rotation flags vprot or null)
// on further workgroups of the same launch; vsplit: 16-row V tiles per pair
// its pair-solve workgroup takes after its solve (0 = timing model, -1 = none)
template <typename T>
hipError_t launch_pair_solve_v(T *B, int64_t ldb, int b, int npairs, const int2 *pairs,
                               const int2 *psmap, T *U, double eps, double thr, int inner,
                               int r16, int cross, double *partial, int *rot_flag, int *prot, T *V,
                               int64_t ldv, int64_t nrows, const int2 *vpairs, const T *vU,
                               const int *vprot, hipStream_t s, int vsplit = 0,
                               hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr,
                               const Batch &bt = Batch());
// experiments: V workgroups of the shared launch (0 = default), a minimum
// dynamic LDS per workgroup (larger keeps one workgroup per compute unit) and
// the working wavefronts per V workgroup (0 = all)
void tune_pair_v(int wgs, size_t lds, int waves);
// wavefronts of the pair-solve workgroup for 2b = M (one off^2 partial each)
constexpr int pair_solve_waves(int M) { return M == 64 ? 16 : 4; }
// thread -> block map of the pair solve (b(b+1)/2 entries for M = 2b)
void pair_solve_map(int M, int cross, int2 *out);
// r16 (FP32 data only): every stored entry of B is rounded to binary16 (the
// binary16 stage of the precision ladder).
// B_kl <- U_k^T B_kl U_l (into B's upper blocks) for every two pairs k < l of
// the round; tile t = l (l - 1) / 2 + k; partial[t (2b / 16) + w] gets twice
// the squared sum of wavefront w's part of tile t when want_off.  With the
// round's rotation flags prot (or null) and no want_off, the tiles of two
// unrotated pairs are left out and counted into *skipped (kernels_update.hip)
template <typename T>
hipError_t launch_update_b(T *B, int64_t ldb, int b, int npairs, const int2 *pairs, const T *U,
                           double *partial, int want_off, int r16, const int *prot, int *skipped,
                           hipStream_t s, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr,
                           const Batch &bt = Batch());
template <typename T>
int update_b_blocks_per_cu(int b);
// grid sizing of the V update: total resident wavefronts (0 = from occupancy)
void tune_update_v(int total_waves);

// V[:, cols(pair)] <- V[:, cols(pair)] U_pair for all pairs, leaving out the
// unrotated ones when the round's rotation flags prot are given
// (kernels_update.hip)
template <typename T>
hipError_t launch_update_v(T *V, int64_t ldv, int64_t nrows, int b, int npairs,
                           const int2 *pairs, const T *U, const int *prot, hipStream_t s,
                           hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr,
                           const Batch &bt = Batch());
// out[0] = sum of x[0 .. count) by one workgroup (per matrix of a batch)
hipError_t launch_sum(const double *x, int64_t count, double *out, hipStream_t s,
                      const Batch &bt = Batch());
// p[0 .. count_per) = value in every matrix's region (p moved by m sW)
hipError_t launch_fill_batch_i32(int *p, int64_t count_per, int value, const Batch &bt,
                                 hipStream_t s);
hipError_t launch_max(const double *x, int64_t count, double *out, hipStream_t s);
// x <- 2^k x for count entries (exact), also written to copy when not null
hipError_t launch_scale_pow2(double *x, int64_t count, int k, double *copy, hipStream_t s);
// B = (A + A^T)/2 zero-padded to npad; norm_partial[0, INGEST_BLOCKS) gets the
// partial sums of squares, [INGEST_BLOCKS, 2 INGEST_BLOCKS) the partial
// maxima of |b_ij|; flags[0] non-finite, flags[1] asymmetric
template <typename T>
hipError_t launch_ingest(const double *A, int64_t lda, int64_t n, T *B, int64_t npad,
                         double *norm_partial, int *flags, int check_sym, hipStream_t s);
template <typename T>
hipError_t launch_eye(T *V, int64_t npad, hipStream_t s);
template <typename T>
hipError_t launch_off2_partial(const T *B, int64_t npad, double *partial, hipStream_t s);
hipError_t launch_fill_i32(int *p, int64_t count, int value, hipStream_t s);
hipError_t launch_cast_f32(const double *src, float *dst, int64_t count, hipStream_t s);
hipError_t launch_widen_f64(const float *src, double *dst, int64_t count, hipStream_t s);
hipError_t launch_cast_f32_scaled(const double *src, float *dst, int64_t count, int k, int r16,
                                  hipStream_t s);
hipError_t launch_diag(const double *B, int64_t ldb, int64_t n, double *w, hipStream_t s);
// w_k = inv_k^2 sum_i V[i][k] T[i][k] (Rayleigh quotients of the normalized
// columns when T = A V); part holds 16 n doubles
hipError_t launch_rayleigh(const double *V, int64_t ldv, const double *T, int64_t ldt,
                           int64_t n, const double *inv, double *part, double *w,
                           hipStream_t s);
// per column of V (rows < n): entry of largest magnitude per row chunk (cmax,
// cidx), squared norm per chunk (csq), all 16 n; inv = 1 / column norm (npad
// entries, 1 past n)
hipError_t launch_colstats(const double *V, int64_t ldv, int64_t n, int64_t npad, double *cmax,
                           int *cidx, double *csq, double *inv, hipStream_t s);
// partial[b] (b < nblocks) = block sums of ||D^-1 V^T V D^-1 X - X||^2 over the
// k = 4 columns of X (npad x 4, zero past n), D^-1 = diag(inv); Y (npad x 4)
// and P (16 n x 4) are scratch
hipError_t launch_orth_probe(const double *V, int64_t ldv, int64_t n, int64_t npad, int k,
                             const double *X, const double *inv, double *Y, double *P,
                             double *partial, int nblocks, hipStream_t s);
// ascending order of w, output columns V[:, perm] scaled by sign / norm
hipError_t launch_finalize(const double *w, const double *V, int64_t ldv_in, int64_t n,
                           double *W, double *Vout, int64_t ldv, int *perm, double *sg,
                           const double *cmax, const int *cidx, const double *inv,
                           hipStream_t s);
constexpr int SIGN_CHUNKS_HOST = 16; // row chunks of the column-sign pass
hipError_t launch_rademacher(double *X, int64_t rows, int64_t n, int k, uint64_t seed,
                             hipStream_t s);
constexpr int INGEST_BLOCKS = 1024;
constexpr int OFF_BLOCKS = 1024;

// ---- FP64 GEMM (kernels_gemm.hip)
// C = alpha * op(A) * op(B) + beta * C0 + gamma * I, all row-major FP64,
// batched over `batch` with element strides sA, sB, sC, sC0.
hipError_t launch_gemm64(int transA, int transB, int64_t M, int64_t N, int64_t K,
                         double alpha, const double *A, int64_t lda, int64_t sA,
                         const double *B, int64_t ldb, int64_t sB, double beta,
                         const double *C0, int64_t ldc0, int64_t sC0, double gamma,
                         double *C, int64_t ldc, int64_t sC, int64_t batch,
                         hipStream_t s);
// The same for a square N x N result known to be symmetric (alpha op(A) op(B)
// symmetric and C0 symmetric): upper tiles computed, mirrored below.  With a
// scratch buffer (device, scratch_doubles entries, not aliasing the operands)
// large enough for the split tiles, a product with more tiles than resident
// workgroups splits its (tile, K stage) iterations evenly over them and adds
// the two parts of each split tile in a fix-up pass.  slots > 0 replaces the
// resident workgroup count (two per compute unit) in that decision.
hipError_t launch_gemm64_sym(int transA, int transB, int64_t N, int64_t K, double alpha,
                             const double *A, int64_t lda, const double *B, int64_t ldb,
                             double beta, const double *C0, int64_t ldc0, double gamma, double *C,
                             int64_t ldc, hipStream_t s, double *scratch = nullptr,
                             int64_t scratch_doubles = 0, int slots = 0);
hipError_t launch_sq_partial(const double *X, int64_t count, double *partial,
                             hipStream_t s);
// backward elementwise: M <- diag(dW) + F o M (F from gaps), flags DEGENERATE
hipError_t launch_adjoint_mid(double *M, const double *W, const double *dW, int64_t n,
                              int64_t batch, double gap_tol, int has_dv, int *flag,
                              hipStream_t s);
hipError_t launch_sym_out(const double *G, double *dA, int64_t n, int64_t ld, int64_t batch,
                          hipStream_t s);

// ---- orthogonalisers (orthogonalize.hip): Q from a QR factorisation of X,
// n x n with leading dimension ld, X destroyed
constexpr int ORTH_CB = 64; // diagonal block order of the blocked Cholesky
constexpr int ORTH_HB = 16; // panel width of the blocked Householder QR
// Cholesky QR: G scratch (may alias Q), Rf receives R's upper triangle, Rinv
// ceil(n / 64) 64 x 64 blocks, bad set when a pivot is not positive
hipError_t cholesky_qr(double *X, double *Q, double *G, double *Rf, int64_t n, int64_t ld,
                       double *Rinv, int *bad, hipStream_t s);
// Householder QR: Vs (n x n, ld) keeps the reflectors, Ts ceil(n / 16) 16 x 16
// factors, W and W2 16 x n scratch
hipError_t householder_qr(double *X, double *Q, double *Vs, int64_t n, int64_t ld, double *Ts,
                          double *W, double *W2, hipStream_t s);

} // namespace lj
