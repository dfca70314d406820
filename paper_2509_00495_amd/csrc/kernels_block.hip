// Round-robin block Jacobi for large n (the block path).
//
// B (n_pad x n_pad, symmetric) is split into N = n_pad / b block rows and
// columns, N even.  A sweep is N-1 rounds; in each round the N/2 disjoint
// block pairs (P, Q) of the round-robin schedule are processed:
//   1. pair solve: one workgroup per pair stages the 2b x 2b diagonal tile
//      [B_PP B_PQ; B_QP B_QQ] in LDS, runs `inner` sweeps of the parallel
//      scalar Jacobi on it (FP64 angles), accumulates the orthogonal 2b x 2b
//      rotation U_PQ and writes the rotated tile back;
//   2. apply: every off-diagonal tile pair (k < l) becomes U_k^T B_kl U_l
//      (two MFMA GEMMs, the result and its transpose are written), and every
//      row tile of V becomes V_rows,l U_l (one MFMA GEMM).
// Entries of B coupling a padding index are zero and stay exactly zero, so
// padding never mixes with the matrix.
#include "internal.hpp"
#include "lds_jacobi.hpp"

namespace lj {

__host__ __device__ inline size_t align8(size_t x) { return (x + 7) & ~(size_t)7; }

// ------------------------------------------------------------- pair solve
// Rotated diagonal entry of a pair after its rotation: a_pp - t a_pq for the
// first position of the pair, a_qq + t a_pq for the second (Section 3.1).
template <typename T>
__device__ inline T rotated_diag(T a, double t, T apq, int second)
{
    double v = second ? (double)a + t * (double)apq : (double)a - t * (double)apq;
    return (T)v;
}

// One workgroup per block pair (P, Q) of the round.  S (the 2b x 2b tile) and
// U (its accumulated rotation, rows in logical order, columns in physical
// order) are double-buffered in LDS; each round reads buffer a and writes the
// rotated, permuted result to buffer b.  Each thread owns a fixed 2x2 block
// (k <= l) of S and fixed (row, pair) items of U for the whole kernel.  The
// angles of the next round are produced inside the same phase: every pair of
// the next round joins one position of current pair k with one of current
// pair l != k, so the owner of block (k, l) knows the new coupling (its own
// result) and recomputes the two new diagonal entries from the current ones;
// a round therefore costs one barrier.  Starting slot s holds tile index s.
template <typename T, int M, int NT>
__global__ __launch_bounds__(NT) void pair_solve_kernel(T *__restrict__ B, int64_t ldb,
                                                        const int2 *__restrict__ pairs,
                                                        const int2 *__restrict__ psmap,
                                                        T *__restrict__ U, double eps,
                                                        double thr, int inner,
                                                        double *__restrict__ partial,
                                                        int *rot_flag)
{
    constexpr int b = M / 2, h = M / 2, ld = M + 1;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *S0 = (T *)smem_raw;
    T *S1 = S0 + M * ld;
    T *U0 = S1 + M * ld;
    T *U1 = U0 + M * ld;
    double *csA = (double *)(smem_raw + align8(4 * sizeof(T) * M * ld));
    double *csB = csA + 3 * h;
    double *red = csB + 3 * h;
    int *ired = (int *)(red + 16);
    const int tid = threadIdx.x;
    const int pk = blockIdx.x;
    const int2 pq = pairs[pk];
    for (int idx = tid; idx < M * M; idx += NT) {
        int p = idx / M, q = idx % M;
        int i = ps_slot(p, M), j = ps_slot(q, M);
        int64_t gi = i < b ? (int64_t)pq.x * b + i : (int64_t)pq.y * b + (i - b);
        int64_t gj = j < b ? (int64_t)pq.x * b + j : (int64_t)pq.y * b + (j - b);
        S0[p * ld + q] = B[gi * ldb + gj];
        U0[p * ld + q] = (T)(p == ps_slot(q, M) ? 1 : 0); // U[row i][phys col q]
    }
    // fixed work assignment: block (bk, bl), bk <= bl, from the host-built
    // map whose first h entries are the blocks hosting the next round's pairs
    // (so their angle computations share one wavefront)
    constexpr int NBLK = h * (h + 1) / 2;
    int bk = -1, bl = -1;
    if (tid < NBLK) {
        const int2 e = psmap[tid];
        bk = e.x;
        bl = e.y;
    }
    const int dk0 = bk >= 0 ? ps_sigma(2 * bk, M) : 0, dk1 = bk >= 0 ? ps_sigma(2 * bk + 1, M) : 0;
    const int dl0 = bk >= 0 ? ps_sigma(2 * bl, M) : 0, dl1 = bk >= 0 ? ps_sigma(2 * bl + 1, M) : 0;
    // the next-round pair hosted by this block, if any: entry (ha, hc) =
    // (2bk+ha, 2bl+hc) becomes next pair hk (a block hosts at most one; the
    // host-built map puts the hosting blocks on threads 0 .. h-1).  Scalars,
    // not arrays, so nothing lands in scratch memory.
    int hosted = 0, ha = 0, hc = 0, hk = 0, hfirst = 0;
    if (bk >= 0 && bk != bl) {
        for (int a = 0; a < 2; ++a)
            for (int c = 0; c < 2; ++c) {
                int sp = ps_sigma(2 * bk + a, M), sq = ps_sigma(2 * bl + c, M);
                if ((sp >> 1) == (sq >> 1)) {
                    hosted = 1;
                    ha = a;
                    hc = c;
                    hk = sp >> 1;
                    hfirst = (sp & 1) == 0; // the row position lands first
                }
            }
    }
    constexpr int NU = M * h; // (row, pair) items of U
    __syncthreads();
    int rot = 0;
    // angles of round 0
    if (tid < h) {
        const int p = 2 * tid, q = p + 1;
        double app = (double)S0[p * ld + p], aqq = (double)S0[q * ld + q];
        double apq = (double)S0[p * ld + q];
        double c = 1.0, sn = 0.0, t = 0.0;
        if (jacobi_should_rotate(app, aqq, apq, eps, thr)) {
            jacobi_angle(app, aqq, apq, c, sn, t);
            rot = 1;
        }
        csA[tid] = c;
        csA[h + tid] = sn;
        csA[2 * h + tid] = t;
    }
    __syncthreads();
    T *Sa = S0, *Sb = S1, *Ua = U0, *Ub = U1;
    double *ca = csA, *cb = csB;
    const int rounds = inner * (M - 1);
    for (int r = 0; r < rounds; ++r) {
        if (bk >= 0) {
            const int k = bk, l = bl;
            const int pk0 = 2 * k, pk1 = pk0 + 1, pl0 = 2 * l, pl1 = pl0 + 1;
            if (k == l) {
                const double tk = ca[2 * h + k];
                const T apq = Sa[pk0 * ld + pk1];
                Sb[dk0 * ld + dk0] = rotated_diag<T>(Sa[pk0 * ld + pk0], tk, apq, 0);
                Sb[dk1 * ld + dk1] = rotated_diag<T>(Sa[pk1 * ld + pk1], tk, apq, 1);
                T z = ca[h + k] == 0.0 ? apq : (T)0;
                Sb[dk0 * ld + dk1] = z;
                Sb[dk1 * ld + dk0] = z;
            } else {
                const T ck = (T)ca[k], sk = (T)ca[h + k], cl = (T)ca[l], sl = (T)ca[h + l];
                T x00 = Sa[pk0 * ld + pl0], x01 = Sa[pk0 * ld + pl1];
                T x10 = Sa[pk1 * ld + pl0], x11 = Sa[pk1 * ld + pl1];
                T y00 = ck * x00 - sk * x10, y01 = ck * x01 - sk * x11;
                T y10 = sk * x00 + ck * x10, y11 = sk * x01 + ck * x11;
                T z[2][2];
                z[0][0] = cl * y00 - sl * y01;
                z[0][1] = sl * y00 + cl * y01;
                z[1][0] = cl * y10 - sl * y11;
                z[1][1] = sl * y10 + cl * y11;
                Sb[dk0 * ld + dl0] = z[0][0];
                Sb[dk0 * ld + dl1] = z[0][1];
                Sb[dk1 * ld + dl0] = z[1][0];
                Sb[dk1 * ld + dl1] = z[1][1];
                Sb[dl0 * ld + dk0] = z[0][0];
                Sb[dl1 * ld + dk0] = z[0][1];
                Sb[dl0 * ld + dk1] = z[1][0];
                Sb[dl1 * ld + dk1] = z[1][1];
                // angle of the next round for the hosted pair
                if (hosted) {
                    const int pe = pk0 + ha, qe = pl0 + hc;
                    const T dpe = rotated_diag<T>(Sa[pe * ld + pe], ca[2 * h + k],
                                                  Sa[pk0 * ld + pk1], ha);
                    const T dqe = rotated_diag<T>(Sa[qe * ld + qe], ca[2 * h + l],
                                                  Sa[pl0 * ld + pl1], hc);
                    const double app = (double)(hfirst ? dpe : dqe);
                    const double aqq = (double)(hfirst ? dqe : dpe);
                    const T zz = ha ? (hc ? z[1][1] : z[1][0]) : (hc ? z[0][1] : z[0][0]);
                    const double apq = (double)zz;
                    double cc = 1.0, sn = 0.0, t = 0.0;
                    if (jacobi_should_rotate(app, aqq, apq, eps, thr)) {
                        jacobi_angle(app, aqq, apq, cc, sn, t);
                        if (r + 1 < rounds)
                            rot = 1;
                    }
                    cb[hk] = cc;
                    cb[h + hk] = sn;
                    cb[2 * h + hk] = t;
                }
            }
        }
        // U items go to the wavefronts after the first (which carries the
        // angle computations)
        for (int it = tid - WAVE; it >= 0 && it < NU; it += NT - WAVE) {
            const int i = it / h, k = it % h;
            const int p0 = 2 * k, p1 = p0 + 1;
            const T c = (T)ca[k], sn = (T)ca[h + k];
            T u0 = Ua[i * ld + p0], u1 = Ua[i * ld + p1];
            Ub[i * ld + ps_sigma(p0, M)] = c * u0 - sn * u1;
            Ub[i * ld + ps_sigma(p1, M)] = sn * u0 + c * u1;
        }
        __syncthreads();
        T *tmp = Sa;
        Sa = Sb;
        Sb = tmp;
        tmp = Ua;
        Ua = Ub;
        Ub = tmp;
        double *tc = ca;
        ca = cb;
        cb = tc;
    }
    // back in the starting layout: position p holds tile index ps_slot(p)
    T *Uk = U + (int64_t)pk * M * M;
    for (int idx = tid; idx < M * M; idx += NT) {
        int p = idx / M, q = idx % M;
        int i = ps_slot(p, M), j = ps_slot(q, M);
        int64_t gi = i < b ? (int64_t)pq.x * b + i : (int64_t)pq.y * b + (i - b);
        int64_t gj = j < b ? (int64_t)pq.x * b + j : (int64_t)pq.y * b + (j - b);
        B[gi * ldb + gj] = Sa[p * ld + q];
        Uk[p * M + j] = Ua[p * ld + q]; // U[row p][logical column j]
    }
    double off2 = lds_off2<T, NT>(Sa, ld, M, red);
    int any = block_or<NT>(rot, ired);
    if (tid == 0) {
        partial[pk] = off2;
        if (any)
            atomicOr(rot_flag, 1);
    }
}

template <typename T>
hipError_t launch_pair_solve(T *B, int64_t ldb, int b, int npairs, const int2 *pairs,
                             const int2 *psmap, T *U, double eps, double thr, int inner,
                             double *partial, int *rot_flag, hipStream_t s)
{
    const int M = 2 * b;
    size_t smem = align8(4 * sizeof(T) * M * (M + 1)) + (6 * b + 16) * sizeof(double) +
                  16 * sizeof(int);
    hipError_t e;
    if (M == 64) {
        auto k = pair_solve_kernel<T, 64, 1024>;
        e = hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)smem);
        if (e != hipSuccess)
            return e;
        hipLaunchKernelGGL(k, dim3(npairs), dim3(1024), smem, s, B, ldb, pairs, psmap, U, eps,
                           thr, inner, partial, rot_flag);
    } else if (M == 32) {
        auto k = pair_solve_kernel<T, 32, 256>;
        e = hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)smem);
        if (e != hipSuccess)
            return e;
        hipLaunchKernelGGL(k, dim3(npairs), dim3(256), smem, s, B, ldb, pairs, psmap, U, eps,
                           thr, inner, partial, rot_flag);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ------------------------------------------------------------------ apply
// Wave-level GEMM on LDS operands: acc += op(A) * Bm over the full inner
// dimension M.  Wave w owns rows [ (w/2) M/2, +M/2 ) and columns
// [ (w%2) M/2, +M/2 ) of the M x M product, as TM x TM MFMA 16x16 tiles.
template <typename T, int M, bool TA>
__device__ inline void wave_gemm(const T *As, int lda, const T *Bs, int ldbs,
                                 typename acc4<T>::type (&acc)[M / 32][M / 32])
{
    constexpr int TM = M / 32;
    const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
    const int row0 = (w / 2) * (M / 2), col0 = (w % 2) * (M / 2);
    const int li = lane % 16, lk = lane / 16;
#pragma unroll 4
    for (int kb = 0; kb < M; kb += 4) {
        const int kk = kb + lk;
        T a[TM], bb[TM];
#pragma unroll
        for (int t = 0; t < TM; ++t) {
            const int i = row0 + t * 16 + li;
            a[t] = TA ? As[kk * lda + i] : As[i * lda + kk];
            const int j = col0 + t * 16 + li;
            bb[t] = Bs[kk * ldbs + j];
        }
#pragma unroll
        for (int ti = 0; ti < TM; ++ti)
#pragma unroll
            for (int tj = 0; tj < TM; ++tj)
                acc[ti][tj] = mfma16(a[ti], bb[tj], acc[ti][tj]);
    }
}

// Store the wave's accumulators into an LDS matrix (row stride ld).
template <typename T, int M>
__device__ inline void wave_store(T *Cs, int ld, typename acc4<T>::type (&acc)[M / 32][M / 32])
{
    constexpr int TM = M / 32;
    const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
    const int row0 = (w / 2) * (M / 2), col0 = (w % 2) * (M / 2);
    const int li = lane % 16, lk = lane / 16;
#pragma unroll
    for (int ti = 0; ti < TM; ++ti)
#pragma unroll
        for (int tj = 0; tj < TM; ++tj)
#pragma unroll
            for (int v = 0; v < 4; ++v)
                Cs[(row0 + ti * 16 + acc_row<T>(lk, v)) * ld + col0 + tj * 16 + li] =
                    acc[ti][tj][v];
}

template <typename T, int M>
__device__ inline void zero_acc(typename acc4<T>::type (&acc)[M / 32][M / 32])
{
#pragma unroll
    for (int ti = 0; ti < M / 32; ++ti)
#pragma unroll
        for (int tj = 0; tj < M / 32; ++tj)
#pragma unroll
            for (int v = 0; v < 4; ++v)
                acc[ti][tj][v] = (T)0;
}

template <typename T, int M>
__global__ __launch_bounds__(256) void apply_kernel(T *__restrict__ B, int64_t ldb,
                                                    T *__restrict__ V, int64_t ldv,
                                                    const int2 *__restrict__ pairs,
                                                    const int2 *__restrict__ btiles, int nbt,
                                                    int npairs, const T *__restrict__ U,
                                                    double *__restrict__ partial, int want_off)
{
    constexpr int b = M / 2, ld = M + 1;
    __shared__ T Xs[M * ld];
    __shared__ T Us[M * ld];
    __shared__ double red[4];
    const int tid = threadIdx.x;
    typename acc4<T>::type acc[M / 32][M / 32];
    zero_acc<T, M>(acc);
    const int tile = blockIdx.x;
    if (tile < nbt) {
        const int2 kl = btiles[tile];
        const int2 pk = pairs[kl.x], pl = pairs[kl.y];
        const T *Ukp = U + (int64_t)kl.x * M * M;
        const T *Ulp = U + (int64_t)kl.y * M * M;
        for (int idx = tid; idx < M * M; idx += 256) {
            int i = idx / M, j = idx % M;
            int64_t gi = i < b ? (int64_t)pk.x * b + i : (int64_t)pk.y * b + (i - b);
            int64_t gj = j < b ? (int64_t)pl.x * b + j : (int64_t)pl.y * b + (j - b);
            Xs[i * ld + j] = B[gi * ldb + gj];
            Us[i * ld + j] = Ulp[idx];
        }
        __syncthreads();
        wave_gemm<T, M, false>(Xs, ld, Us, ld, acc); // Y = X U_l
        __syncthreads();
        wave_store<T, M>(Xs, ld, acc);
        for (int idx = tid; idx < M * M; idx += 256) {
            int i = idx / M, j = idx % M;
            Us[i * ld + j] = Ukp[idx];
        }
        __syncthreads();
        zero_acc<T, M>(acc);
        wave_gemm<T, M, true>(Us, ld, Xs, ld, acc); // Z = U_k^T Y
        __syncthreads();
        wave_store<T, M>(Xs, ld, acc);
        __syncthreads();
        double sq = 0.0;
        for (int idx = tid; idx < M * M; idx += 256) {
            int i = idx / M, j = idx % M;
            int64_t gi = i < b ? (int64_t)pk.x * b + i : (int64_t)pk.y * b + (i - b);
            int64_t gj = j < b ? (int64_t)pl.x * b + j : (int64_t)pl.y * b + (j - b);
            T z = Xs[i * ld + j];
            B[gi * ldb + gj] = z;
            sq += (double)z * (double)z;
            // mirror: row gj' of the transposed tile, coalesced along i'
            int i2 = idx / M, j2 = idx % M; // i2 indexes columns of Z, j2 rows
            int64_t mi = i2 < b ? (int64_t)pl.x * b + i2 : (int64_t)pl.y * b + (i2 - b);
            int64_t mj = j2 < b ? (int64_t)pk.x * b + j2 : (int64_t)pk.y * b + (j2 - b);
            B[mi * ldb + mj] = Xs[j2 * ld + i2];
        }
        if (want_off) {
            sq = wave_sum(sq);
            if (tid % WAVE == 0)
                red[tid / WAVE] = sq;
            __syncthreads();
            if (tid == 0)
                partial[tile] = 2.0 * (red[0] + red[1] + red[2] + red[3]);
        }
    } else {
        const int vt = tile - nbt;
        const int l = vt % npairs;
        const int64_t r0 = (int64_t)(vt / npairs) * M;
        const int2 pl = pairs[l];
        const T *Ulp = U + (int64_t)l * M * M;
        for (int idx = tid; idx < M * M; idx += 256) {
            int i = idx / M, j = idx % M;
            int64_t gj = j < b ? (int64_t)pl.x * b + j : (int64_t)pl.y * b + (j - b);
            Xs[i * ld + j] = V[(r0 + i) * ldv + gj];
            Us[i * ld + j] = Ulp[idx];
        }
        __syncthreads();
        wave_gemm<T, M, false>(Xs, ld, Us, ld, acc); // V_rows,l U_l
        __syncthreads();
        wave_store<T, M>(Xs, ld, acc);
        __syncthreads();
        for (int idx = tid; idx < M * M; idx += 256) {
            int i = idx / M, j = idx % M;
            int64_t gj = j < b ? (int64_t)pl.x * b + j : (int64_t)pl.y * b + (j - b);
            V[(r0 + i) * ldv + gj] = Xs[i * ld + j];
        }
    }
}

// which = 1: B tiles only, 2: V tiles only, 3: both in one launch.
template <typename T>
hipError_t launch_apply(T *B, int64_t ldb, T *V, int64_t ldv, int64_t nrows, int b, int npairs,
                        const int2 *pairs, const int2 *btiles, int nbt, const T *U,
                        double *partial, int want_off, int which, hipStream_t s)
{
    const int M = 2 * b;
    const int64_t nvt = (which & 2) ? (nrows / M) * npairs : 0;
    const int nb = (which & 1) ? nbt : 0;
    const int64_t grid = nb + nvt;
    if (grid == 0)
        return hipSuccess;
    if (M == 64)
        hipLaunchKernelGGL((apply_kernel<T, 64>), dim3((unsigned)grid), dim3(256), 0, s, B,
                           ldb, V, ldv, pairs, btiles, nb, npairs, U, partial, want_off);
    else if (M == 32)
        hipLaunchKernelGGL((apply_kernel<T, 32>), dim3((unsigned)grid), dim3(256), 0, s, B,
                           ldb, V, ldv, pairs, btiles, nb, npairs, U, partial, want_off);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

// ------------------------------------------------------- reductions, etc.
__global__ __launch_bounds__(256) void sum_kernel(const double *__restrict__ x, int64_t count,
                                                  double *out)
{
    __shared__ double red[4];
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < count; i += 256)
        acc += x[i];
    acc = wave_sum(acc);
    if (threadIdx.x % WAVE == 0)
        red[threadIdx.x / WAVE] = acc;
    __syncthreads();
    if (threadIdx.x == 0)
        out[0] = red[0] + red[1] + red[2] + red[3];
}

hipError_t launch_sum(const double *x, int64_t count, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(256), 0, s, x, count, out);
    return hipGetLastError();
}

// Symmetrised copy of A into the padded working matrix (32 x 32 tiles staged
// through LDS so that both A and A^T are read along rows), plus the partial
// sums of squares for ||B||_F and the non-finite / asymmetry flags.
template <typename T>
__global__ __launch_bounds__(256) void ingest_kernel(const double *__restrict__ A, int64_t lda,
                                                     int64_t n, T *__restrict__ B, int64_t npad,
                                                     double *__restrict__ partial, int *flags,
                                                     int check_sym)
{
    __shared__ double t1[32][33];
    __shared__ double t2[32][33];
    __shared__ double red[4];
    const int64_t nt = npad / 32;
    double acc = 0.0;
    int bad = 0, asym = 0;
    for (int64_t tile = blockIdx.x; tile < nt * nt; tile += gridDim.x) {
        const int64_t i0 = (tile / nt) * 32, j0 = (tile % nt) * 32;
        for (int e = threadIdx.x; e < 1024; e += 256) {
            int r = e / 32, c = e % 32;
            int64_t i = i0 + r, j = j0 + c;
            t1[r][c] = (i < n && j < n) ? A[i * lda + j] : 0.0;
            int64_t i2 = j0 + r, j2 = i0 + c; // A^T tile, read along rows
            t2[r][c] = (i2 < n && j2 < n) ? A[i2 * lda + j2] : 0.0;
        }
        __syncthreads();
        for (int e = threadIdx.x; e < 1024; e += 256) {
            int r = e / 32, c = e % 32;
            double a = t1[r][c], at = t2[c][r];
            if (!isfinite(a))
                bad = 1;
            if (check_sym && a != at)
                asym = 1;
            double v = 0.5 * (a + at);
            B[(i0 + r) * npad + j0 + c] = (T)v;
            acc += v * v;
        }
        __syncthreads();
    }
    acc = wave_sum(acc);
    if (threadIdx.x % WAVE == 0)
        red[threadIdx.x / WAVE] = acc;
    __syncthreads();
    if (threadIdx.x == 0)
        partial[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
    if (__any(bad) && threadIdx.x % WAVE == 0)
        atomicOr(flags, 1);
    if (__any(asym) && threadIdx.x % WAVE == 0)
        atomicOr(flags + 1, 1);
}

template <typename T>
hipError_t launch_ingest(const double *A, int64_t lda, int64_t n, T *B, int64_t npad,
                         double *norm_partial, int *flags, int check_sym, hipStream_t s)
{
    hipLaunchKernelGGL((ingest_kernel<T>), dim3(INGEST_BLOCKS), dim3(256), 0, s, A, lda, n, B,
                       npad, norm_partial, flags, check_sym);
    return hipGetLastError();
}

template <typename T>
__global__ __launch_bounds__(256) void eye_kernel(T *__restrict__ V, int64_t npad)
{
    const int64_t total = npad * npad;
    for (int64_t e = blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
        int64_t i = e / npad, j = e - (e / npad) * npad;
        V[e] = (T)(i == j ? 1 : 0);
    }
}

template <typename T>
hipError_t launch_eye(T *V, int64_t npad, hipStream_t s)
{
    hipLaunchKernelGGL((eye_kernel<T>), dim3(2048), dim3(256), 0, s, V, npad);
    return hipGetLastError();
}

template <typename T>
__global__ __launch_bounds__(256) void off2_partial_kernel(const T *__restrict__ B, int64_t npad,
                                                           double *__restrict__ partial)
{
    __shared__ double red[4];
    const int64_t total = npad * npad;
    double acc = 0.0;
    for (int64_t e = blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
        int64_t i = e / npad, j = e - (e / npad) * npad;
        if (i != j) {
            double v = (double)B[e];
            acc += v * v;
        }
    }
    acc = wave_sum(acc);
    if (threadIdx.x % WAVE == 0)
        red[threadIdx.x / WAVE] = acc;
    __syncthreads();
    if (threadIdx.x == 0)
        partial[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

template <typename T>
hipError_t launch_off2_partial(const T *B, int64_t npad, double *partial, hipStream_t s)
{
    hipLaunchKernelGGL((off2_partial_kernel<T>), dim3(OFF_BLOCKS), dim3(256), 0, s, B, npad,
                       partial);
    return hipGetLastError();
}

__global__ void fill_i32_kernel(int *p, int64_t count, int value)
{
    for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < count; i += (int64_t)gridDim.x * 256)
        p[i] = value;
}

hipError_t launch_fill_i32(int *p, int64_t count, int value, hipStream_t s)
{
    int grid = (int)((count + 255) / 256);
    grid = grid < 1 ? 1 : (grid > 1024 ? 1024 : grid);
    hipLaunchKernelGGL(fill_i32_kernel, dim3(grid), dim3(256), 0, s, p, count, value);
    return hipGetLastError();
}

__global__ void cast_f32_kernel(const double *__restrict__ src, float *__restrict__ dst,
                                int64_t count)
{
    for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < count; i += (int64_t)gridDim.x * 256)
        dst[i] = (float)src[i];
}

hipError_t launch_cast_f32(const double *src, float *dst, int64_t count, hipStream_t s)
{
    hipLaunchKernelGGL(cast_f32_kernel, dim3(2048), dim3(256), 0, s, src, dst, count);
    return hipGetLastError();
}

__global__ void widen_f64_kernel(const float *__restrict__ src, double *__restrict__ dst,
                                 int64_t count)
{
    for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < count; i += (int64_t)gridDim.x * 256)
        dst[i] = (double)src[i];
}

hipError_t launch_widen_f64(const float *src, double *dst, int64_t count, hipStream_t s)
{
    hipLaunchKernelGGL(widen_f64_kernel, dim3(2048), dim3(256), 0, s, src, dst, count);
    return hipGetLastError();
}

// B <- (B + B^T)/2 in place; each unordered pair (i < j) has one owner.
__global__ __launch_bounds__(256) void symmetrize_kernel(double *B, int64_t npad)
{
    const int64_t total = npad * npad;
    for (int64_t e = blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
        int64_t i = e / npad, j = e - (e / npad) * npad;
        if (i < j) {
            double m = 0.5 * (B[i * npad + j] + B[j * npad + i]);
            B[i * npad + j] = m;
            B[j * npad + i] = m;
        }
    }
}

hipError_t launch_symmetrize(double *B, int64_t npad, hipStream_t s)
{
    hipLaunchKernelGGL(symmetrize_kernel, dim3(2048), dim3(256), 0, s, B, npad);
    return hipGetLastError();
}

// ---------------------------------------------------------------- finalize
__global__ void diag_kernel(const double *__restrict__ B, int64_t ldb, int64_t n,
                            double *__restrict__ w)
{
    for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        w[i] = B[i * ldb + i];
}

// Stable ascending rank of each eigenvalue: ties keep diagonal order.
__global__ __launch_bounds__(256) void rank_kernel(const double *__restrict__ w, int64_t n,
                                                   int *__restrict__ perm)
{
    __shared__ double ws[1024];
    const int64_t i = blockIdx.x * 256 + threadIdx.x;
    const double wi = i < n ? w[i] : 0.0;
    int64_t rank = 0;
    for (int64_t j0 = 0; j0 < n; j0 += 1024) {
        __syncthreads();
        for (int t = threadIdx.x; t < 1024; t += 256)
            ws[t] = (j0 + t < n) ? w[j0 + t] : 0.0;
        __syncthreads();
        const int64_t jn = (n - j0) < 1024 ? (n - j0) : 1024;
        if (i < n)
            for (int64_t jj = 0; jj < jn; ++jj) {
                double wj = ws[jj];
                int64_t j = j0 + jj;
                rank += (wj < wi) || (wj == wi && j < i);
            }
    }
    if (i < n)
        perm[rank] = (int)i;
}

// Sign of each output column: the entry of largest magnitude (lowest row on
// ties) becomes positive.  Two passes so that V is read along rows: pass 1
// scans row chunk z for every column j (threads over j), pass 2 reduces the
// chunks in order for each output column.
constexpr int SIGN_CHUNKS = 16;

__global__ __launch_bounds__(256) void colmax_kernel(const double *__restrict__ V, int64_t ldv,
                                                     int64_t n, double *__restrict__ cmax,
                                                     int *__restrict__ cidx)
{
    const int64_t j = blockIdx.x * 256 + threadIdx.x;
    const int z = blockIdx.y;
    if (j >= n)
        return;
    const int64_t chunk = (n + SIGN_CHUNKS - 1) / SIGN_CHUNKS;
    const int64_t i0 = z * chunk, i1 = (i0 + chunk < n) ? i0 + chunk : n;
    double best = -1.0;
    int64_t bi = i0 < n ? i0 : 0;
    for (int64_t i = i0; i < i1; ++i) {
        double a = fabs(V[i * ldv + j]);
        if (a > best) {
            best = a;
            bi = i;
        }
    }
    cmax[z * n + j] = best;
    cidx[z * n + j] = (int)bi;
}

__global__ __launch_bounds__(256) void colsign_kernel(const double *__restrict__ V, int64_t ldv,
                                                      int64_t n, const int *__restrict__ perm,
                                                      const double *__restrict__ cmax,
                                                      const int *__restrict__ cidx,
                                                      double *__restrict__ sg)
{
    const int64_t c = blockIdx.x * 256 + threadIdx.x;
    if (c >= n)
        return;
    const int col = perm[c];
    double best = -1.0;
    int bi = 0;
    for (int z = 0; z < SIGN_CHUNKS; ++z) {
        double m = cmax[z * n + col];
        if (m > best) {
            best = m;
            bi = cidx[z * n + col];
        }
    }
    sg[c] = V[(int64_t)bi * ldv + col] < 0.0 ? -1.0 : 1.0;
}

__global__ __launch_bounds__(256) void permute_out_kernel(const double *__restrict__ V,
                                                          int64_t ldv_in, int64_t n,
                                                          const int *__restrict__ perm,
                                                          const double *__restrict__ sg,
                                                          const double *__restrict__ w,
                                                          double *__restrict__ W,
                                                          double *__restrict__ Vout, int64_t ldv)
{
    const int64_t total = n * n;
    for (int64_t e = blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
        int64_t i = e / n, c = e - (e / n) * n;
        int col = perm[c];
        Vout[i * ldv + c] = sg[c] * V[i * ldv_in + col];
        if (i == 0)
            W[c] = w[col];
    }
}

hipError_t launch_diag(const double *B, int64_t ldb, int64_t n, double *w, hipStream_t s)
{
    int g = (int)((n + 255) / 256);
    hipLaunchKernelGGL(diag_kernel, dim3(g), dim3(256), 0, s, B, ldb, n, w);
    return hipGetLastError();
}

// Output stage from the extracted diagonal w: stable ascending order, column
// permutation and sign convention.
hipError_t launch_finalize(const double *w, const double *V, int64_t ldv_in, int64_t n,
                           double *W, double *Vout, int64_t ldv, int *perm, double *sg,
                           double *cmax, int *cidx, hipStream_t s)
{
    int g = (int)((n + 255) / 256);
    hipLaunchKernelGGL(rank_kernel, dim3(g), dim3(256), 0, s, w, n, perm);
    hipLaunchKernelGGL(colmax_kernel, dim3(g, SIGN_CHUNKS), dim3(256), 0, s, V, ldv_in, n, cmax,
                       cidx);
    hipLaunchKernelGGL(colsign_kernel, dim3(g), dim3(256), 0, s, V, ldv_in, n, perm, cmax, cidx,
                       sg);
    hipLaunchKernelGGL(permute_out_kernel, dim3(2048), dim3(256), 0, s, V, ldv_in, n, perm, sg,
                       w, W, Vout, ldv);
    return hipGetLastError();
}

// Rademacher probe vectors (+-1 in rows < n, 0 below) from a counter-based
// hash (splitmix64 finaliser), for the randomized estimate
// ||V^T V - I||_F^2 ~ mean_k ||(V^T V - I) x_k||^2.
__global__ void rademacher_kernel(double *X, int64_t rows, int64_t n, int k, uint64_t seed)
{
    const int64_t total = rows * k;
    for (int64_t e = blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
        int64_t i = e / k;
        uint64_t z = seed + 0x9E3779B97F4A7C15ull * (uint64_t)(e + 1);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        X[e] = i < n ? ((z & 1) ? 1.0 : -1.0) : 0.0;
    }
}

hipError_t launch_rademacher(double *X, int64_t rows, int64_t n, int k, uint64_t seed,
                             hipStream_t s)
{
    hipLaunchKernelGGL(rademacher_kernel, dim3(64), dim3(256), 0, s, X, rows, n, k, seed);
    return hipGetLastError();
}

// explicit instantiations
template hipError_t launch_pair_solve<double>(double *, int64_t, int, int, const int2 *,
                                              const int2 *, double *, double, double, int,
                                              double *, int *, hipStream_t);
template hipError_t launch_pair_solve<float>(float *, int64_t, int, int, const int2 *,
                                             const int2 *, float *, double, double, int,
                                             double *, int *, hipStream_t);

// Thread -> 2x2 block map of the pair solve for M = 2b positions: entry t < M/2
// is the block hosting pair t of the next round, the rest follow in row order.
void pair_solve_map(int M, int2 *out)
{
    const int h = M / 2;
    int inv[128];
    for (int p = 0; p < M; ++p)
        inv[ps_sigma(p, M)] = p;
    int cnt = 0;
    bool used[64][64] = {};
    for (int t = 0; t < h; ++t) {
        int a = inv[2 * t] >> 1, c = inv[2 * t + 1] >> 1;
        int k = a < c ? a : c, l = a < c ? c : a;
        out[cnt++] = make_int2(k, l);
        used[k][l] = true;
    }
    for (int k = 0; k < h; ++k)
        for (int l = k; l < h; ++l)
            if (!used[k][l])
                out[cnt++] = make_int2(k, l);
}
template hipError_t launch_apply<double>(double *, int64_t, double *, int64_t, int64_t, int,
                                         int, const int2 *, const int2 *, int, const double *,
                                         double *, int, int, hipStream_t);
template hipError_t launch_apply<float>(float *, int64_t, float *, int64_t, int64_t, int, int,
                                        const int2 *, const int2 *, int, const float *,
                                        double *, int, int, hipStream_t);
template hipError_t launch_ingest<double>(const double *, int64_t, int64_t, double *, int64_t,
                                          double *, int *, int, hipStream_t);
template hipError_t launch_ingest<float>(const double *, int64_t, int64_t, float *, int64_t,
                                         double *, int *, int, hipStream_t);
template hipError_t launch_eye<double>(double *, int64_t, hipStream_t);
template hipError_t launch_eye<float>(float *, int64_t, hipStream_t);
template hipError_t launch_off2_partial<double>(const double *, int64_t, double *, hipStream_t);
template hipError_t launch_off2_partial<float>(const float *, int64_t, double *, hipStream_t);

} // namespace lj
