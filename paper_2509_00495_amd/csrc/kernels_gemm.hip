// FP64 MFMA GEMM used by the Newton-Schulz step, the preconditioning product
// Q_d^T A Q_d and the adjoint, plus the small elementwise kernels of the
// adjoint.
//
//   C = alpha * op(A) * op(B) + beta * C0 + gamma * I      (row-major)
//
// Workgroup tile 64 x 64 (4 waves, each 32 x 32 = 2 x 2 MFMA 16x16x4 tiles),
// K staged through LDS 16 at a time; batched over blockIdx.z.  SYM (square C
// whose product is symmetric, e.g. X^T X): only tiles on or above the
// diagonal are computed, and off-diagonal tiles also write their transpose,
// so C comes out exactly symmetric for half the work.
#include "common.hpp"
#include "internal.hpp"

namespace lj {

constexpr int GT = 64;  // tile edge
constexpr int GK = 16;  // k per stage
constexpr int GLD = GT + 1;

template <int TA, int TB, bool SYM>
__global__ __launch_bounds__(256) void gemm64_kernel(int64_t M, int64_t N, int64_t K, double alpha,
                                                     const double *__restrict__ A, int64_t lda,
                                                     int64_t sA, const double *__restrict__ B,
                                                     int64_t ldb, int64_t sB, double beta,
                                                     const double *__restrict__ C0, int64_t ldc0,
                                                     int64_t sC0, double gamma,
                                                     double *__restrict__ C, int64_t ldc,
                                                     int64_t sC)
{
    __shared__ double As[GK * GLD]; // As[kk][i]
    __shared__ double Bs[GK * GLD]; // Bs[kk][j]
    const int tid = threadIdx.x;
    const int lane = tid % WAVE, w = tid / WAVE;
    const int li = lane % 16, lk = lane / 16;
    const int64_t z = blockIdx.z;
    A += z * sA;
    B += z * sB;
    C += z * sC;
    if (C0)
        C0 += z * sC0;
    if (SYM && blockIdx.x < blockIdx.y)
        return;
    const int64_t i0 = (int64_t)blockIdx.y * GT, j0 = (int64_t)blockIdx.x * GT;
    const int row0 = (w / 2) * 32, col0 = (w % 2) * 32;
    d4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v)
                acc[a][b][v] = 0.0;
    for (int64_t k0 = 0; k0 < K; k0 += GK) {
#pragma unroll
        for (int e = tid; e < GT * GK; e += 256) {
            int i, kk;
            double va;
            if (!TA) { // A is M x K: read along k
                i = e / GK;
                kk = e % GK;
                int64_t gi = i0 + i, gk = k0 + kk;
                va = (gi < M && gk < K) ? A[gi * lda + gk] : 0.0;
            } else { // A is K x M: read along i
                kk = e / GT;
                i = e % GT;
                int64_t gi = i0 + i, gk = k0 + kk;
                va = (gi < M && gk < K) ? A[gk * lda + gi] : 0.0;
            }
            As[kk * GLD + i] = va;
            int j;
            double vb;
            if (!TB) { // B is K x N: read along j
                kk = e / GT;
                j = e % GT;
                int64_t gj = j0 + j, gk = k0 + kk;
                vb = (gj < N && gk < K) ? B[gk * ldb + gj] : 0.0;
            } else { // B is N x K: read along k
                j = e / GK;
                kk = e % GK;
                int64_t gj = j0 + j, gk = k0 + kk;
                vb = (gj < N && gk < K) ? B[gj * ldb + gk] : 0.0;
            }
            Bs[kk * GLD + j] = vb;
        }
        __syncthreads();
#pragma unroll
        for (int kb = 0; kb < GK; kb += 4) {
            const int kk = kb + lk;
            double a0 = As[kk * GLD + row0 + li], a1 = As[kk * GLD + row0 + 16 + li];
            double b0 = Bs[kk * GLD + col0 + li], b1 = Bs[kk * GLD + col0 + 16 + li];
            acc[0][0] = mfma16(a0, b0, acc[0][0]);
            acc[0][1] = mfma16(a0, b1, acc[0][1]);
            acc[1][0] = mfma16(a1, b0, acc[1][0]);
            acc[1][1] = mfma16(a1, b1, acc[1][1]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                int64_t gi = i0 + row0 + a * 16 + acc_row<double>(lk, v);
                int64_t gj = j0 + col0 + b * 16 + li;
                if (gi < M && gj < N) {
                    double r = alpha * acc[a][b][v];
                    if (beta != 0.0)
                        r += beta * C0[gi * ldc0 + gj];
                    if (gi == gj)
                        r += gamma;
                    C[gi * ldc + gj] = r;
                    if (SYM && blockIdx.x != blockIdx.y)
                        C[gj * ldc + gi] = r;
                }
            }
}

// Large-matrix variant: workgroup tile 128 x 128 (4 waves, each 64 x 64 =
// 4 x 4 MFMA tiles), K staged 16 at a time through two LDS buffers (the next
// stage's operands are loaded into registers while the current one
// multiplies: one barrier per stage), 16-byte global loads.  LDS rows hold
// 128 + 16 doubles: the four k rows a wavefront reads at once then start
// 128 bytes apart and fall in different banks.  Requires even leading
// dimensions and 16-byte aligned bases; edges are zero-filled and masked.
constexpr int BT = 128, BK = 16, BLD = BT + 16;
typedef double dv2g __attribute__((ext_vector_type(2)));

// Upper-triangular tile t of a tiles_n x tiles_n grid (row by <= column bx),
// numbered along rows.
__device__ inline void tri_tile(int t, int tiles_n, int &by, int &bx)
{
    int r = 0;
    while (t >= tiles_n - r) {
        t -= tiles_n - r;
        ++r;
    }
    by = r;
    bx = r + t;
}

// K stages [s0, s1) of tile (by, bx).  part == nullptr: the tile is complete
// and goes to C (alpha, beta C0, gamma I, mirrored when SYM and off the
// diagonal); otherwise the raw accumulator goes to part (BT x BT, row-major)
// for the fix-up pass that adds the tile's two parts.
template <int TA, int TB, bool SYM>
__device__ inline void gemm128_segment(int64_t M, int64_t N, int64_t K, double alpha,
                                       const double *__restrict__ A, int64_t lda,
                                       const double *__restrict__ B, int64_t ldb, double beta,
                                       const double *__restrict__ C0, int64_t ldc0,
                                       double gamma, double *__restrict__ C, int64_t ldc,
                                       int by, int bx, int s0, int s1, double *__restrict__ part,
                                       double (*sm)[2][BK * BLD])
{
    const int tid = threadIdx.x, lane = tid % WAVE, w = tid / WAVE;
    const int li = lane % 16, lk = lane / 16;
    const int64_t i0 = (int64_t)by * BT, j0 = (int64_t)bx * BT;
    const int row0 = (w / 2) * 64, col0 = (w % 2) * 64;
    // operand staging: 2048 doubles per matrix and stage = 8 per thread as
    // four 16-byte pieces
    // source [row][k] (A, or B^T when TB): thread -> row t/2, k 8 (t&1) .. +7
    // source [k][col] (A^T when TA, or B): thread -> k t/16, col 8 (t%16) .. +7
    dv2g ra[4], rb[4];
    auto load = [&](int64_t k0) __attribute__((always_inline)) {
        if (!TA) {
            const int64_t gi = i0 + tid / 2, gk = k0 + 8 * (tid & 1);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int64_t k = gk + 2 * e;
                dv2g v = {0.0, 0.0};
                if (gi < M && k + 1 < K)
                    v = *reinterpret_cast<const dv2g *>(A + gi * lda + k);
                else if (gi < M && k < K)
                    v[0] = A[gi * lda + k];
                ra[e] = v;
            }
        } else {
            const int64_t gk = k0 + tid / 16, gi = i0 + 8 * (tid % 16);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int64_t i = gi + 2 * e;
                dv2g v = {0.0, 0.0};
                if (gk < K && i + 1 < M)
                    v = *reinterpret_cast<const dv2g *>(A + gk * lda + i);
                else if (gk < K && i < M)
                    v[0] = A[gk * lda + i];
                ra[e] = v;
            }
        }
        if (TB) {
            const int64_t gj = j0 + tid / 2, gk = k0 + 8 * (tid & 1);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int64_t k = gk + 2 * e;
                dv2g v = {0.0, 0.0};
                if (gj < N && k + 1 < K)
                    v = *reinterpret_cast<const dv2g *>(B + gj * ldb + k);
                else if (gj < N && k < K)
                    v[0] = B[gj * ldb + k];
                rb[e] = v;
            }
        } else {
            const int64_t gk = k0 + tid / 16, gj = j0 + 8 * (tid % 16);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int64_t j = gj + 2 * e;
                dv2g v = {0.0, 0.0};
                if (gk < K && j + 1 < N)
                    v = *reinterpret_cast<const dv2g *>(B + gk * ldb + j);
                else if (gk < K && j < N)
                    v[0] = B[gk * ldb + j];
                rb[e] = v;
            }
        }
    };
    auto store = [&](int buf) __attribute__((always_inline)) {
        double *As = sm[buf][0], *Bs = sm[buf][1];
        if (!TA) {
            const int i = tid / 2, kk = 8 * (tid & 1);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                As[(kk + 2 * e) * BLD + i] = ra[e][0];
                As[(kk + 2 * e + 1) * BLD + i] = ra[e][1];
            }
        } else {
            const int kk = tid / 16, i = 8 * (tid % 16);
#pragma unroll
            for (int e = 0; e < 4; ++e)
                *reinterpret_cast<dv2g *>(As + kk * BLD + i + 2 * e) = ra[e];
        }
        if (TB) {
            const int j = tid / 2, kk = 8 * (tid & 1);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                Bs[(kk + 2 * e) * BLD + j] = rb[e][0];
                Bs[(kk + 2 * e + 1) * BLD + j] = rb[e][1];
            }
        } else {
            const int kk = tid / 16, j = 8 * (tid % 16);
#pragma unroll
            for (int e = 0; e < 4; ++e)
                *reinterpret_cast<dv2g *>(Bs + kk * BLD + j + 2 * e) = rb[e];
        }
    };
    d4 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v)
                acc[a][b][v] = 0.0;
    load((int64_t)s0 * BK);
    store(0);
    __syncthreads();
    for (int st = s0; st < s1; ++st) {
        const int buf = (st - s0) & 1;
        if (st + 1 < s1)
            load((int64_t)(st + 1) * BK);
        const double *As = sm[buf][0], *Bs = sm[buf][1];
#pragma unroll
        for (int kb = 0; kb < BK; kb += 4) {
            const int kk = kb + lk;
            double fa[4], fb[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                fa[t] = As[kk * BLD + row0 + 16 * t + li];
                fb[t] = Bs[kk * BLD + col0 + 16 * t + li];
            }
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b)
                    acc[a][b] = mfma16(fa[a], fb[b], acc[a][b]);
        }
        if (st + 1 < s1)
            store(buf ^ 1); // the other buffer was last read before the previous barrier
        __syncthreads();
    }
    if (part) {
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b)
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    part[(row0 + a * 16 + acc_row<double>(lk, v)) * BT + col0 + b * 16 + li] =
                        acc[a][b][v];
        return;
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t gi = i0 + row0 + a * 16 + acc_row<double>(lk, v);
                const int64_t gj = j0 + col0 + b * 16 + li;
                if (gi < M && gj < N) {
                    double r = alpha * acc[a][b][v];
                    if (beta != 0.0)
                        r += beta * C0[gi * ldc0 + gj];
                    if (gi == gj)
                        r += gamma;
                    C[gi * ldc + gj] = r;
                    if (SYM && bx != by)
                        C[gj * ldc + gi] = r;
                }
            }
}


template <int TA, int TB, bool SYM>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) void gemm128_kernel(
    int64_t M, int64_t N, int64_t K, double alpha, const double *__restrict__ A, int64_t lda,
    const double *__restrict__ B, int64_t ldb, double beta, const double *__restrict__ C0,
    int64_t ldc0, double gamma, double *__restrict__ C, int64_t ldc, int tiles_n, int64_t sA,
    int64_t sB, int64_t sC0, int64_t sC)
{
    __shared__ __align__(16) double sm[2][2][BK * BLD]; // [buffer][A or B][k][i or j]
    int by, bx;
    if (SYM) {
        tri_tile(blockIdx.x, tiles_n, by, bx);
    } else {
        by = blockIdx.y;
        bx = blockIdx.x;
        // batch entry blockIdx.z (strides in doubles; one entry when 0)
        const int64_t z = blockIdx.z;
        A += z * sA;
        B += z * sB;
        C += z * sC;
        if (C0)
            C0 += z * sC0;
    }
    gemm128_segment<TA, TB, SYM>(M, N, K, alpha, A, lda, B, ldb, beta, C0, ldc0, gamma, C, ldc,
                                 by, bx, 0, (int)((K + BK - 1) / BK), nullptr, sm);
}

// Symmetric product with more upper tiles than resident workgroups: the
// (tile, K stage) iterations are split evenly over the G workgroups
// (workgroup g takes [g T / G, (g + 1) T / G) of T = tiles x stages), so
// every workgroup does the same work and none runs a second, partly empty
// wave.  With at least G tiles a workgroup's run is at least one tile long,
// so a tile is split by at most one boundary: boundary g (between
// workgroups g - 1 and g) leaves its tile's first part in scratch slot
// 2 (g - 1) and its second part in slot 2 (g - 1) + 1, and the fix-up pass
// adds them (two terms: the same sum whichever finishes first).
template <int TA, int TB>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) void gemm128_sk_kernel(
    int64_t M, int64_t N, int64_t K, double alpha, const double *__restrict__ A, int64_t lda,
    const double *__restrict__ B, int64_t ldb, double beta, const double *__restrict__ C0,
    int64_t ldc0, double gamma, double *__restrict__ C, int64_t ldc, int tiles_n, int ntiles,
    double *__restrict__ scratch)
{
    __shared__ __align__(16) double sm[2][2][BK * BLD];
    const int nst = (int)((K + BK - 1) / BK);
    const int64_t total = (int64_t)ntiles * nst;
    const int g = blockIdx.x, G = gridDim.x;
    int64_t p0 = (int64_t)g * total / G;
    const int64_t p1 = (int64_t)(g + 1) * total / G;
    while (p0 < p1) {
        const int t = (int)(p0 / nst), s0 = (int)(p0 % nst);
        const int s1 = (int)((p1 - (int64_t)t * nst) < nst ? p1 - (int64_t)t * nst : nst);
        int by, bx;
        tri_tile(t, tiles_n, by, bx);
        double *part = nullptr;
        if (s0 > 0)
            part = scratch + (int64_t)(2 * (g - 1) + 1) * BT * BT;
        else if (s1 < nst)
            part = scratch + (int64_t)(2 * g) * BT * BT;
        gemm128_segment<TA, TB, true>(M, N, K, alpha, A, lda, B, ldb, beta, C0, ldc0, gamma, C,
                                      ldc, by, bx, s0, s1, part, sm);
        p0 += s1 - s0;
    }
}

// Fix-up of the split tiles: workgroup g - 1 handles boundary g (1 <= g < G).
__global__ __launch_bounds__(256) void gemm128_sk_fixup_kernel(
    int64_t M, int64_t N, int64_t K, double alpha, double beta, const double *__restrict__ C0,
    int64_t ldc0, double gamma, double *__restrict__ C, int64_t ldc, int tiles_n, int ntiles,
    int G, const double *__restrict__ scratch)
{
    const int g = blockIdx.x + 1;
    const int nst = (int)((K + BK - 1) / BK);
    const int64_t total = (int64_t)ntiles * nst;
    const int64_t p = (int64_t)g * total / G;
    if (p % nst == 0)
        return; // the boundary falls between tiles
    int by, bx;
    tri_tile((int)(p / nst), tiles_n, by, bx);
    const double *p0 = scratch + (int64_t)(2 * (g - 1)) * BT * BT;
    const double *p1 = p0 + BT * BT;
    const int64_t i0 = (int64_t)by * BT, j0 = (int64_t)bx * BT;
    for (int e = threadIdx.x; e < BT * BT; e += 256) {
        const int64_t gi = i0 + e / BT, gj = j0 + e % BT;
        if (gi < M && gj < N) {
            double r = alpha * (p0[e] + p1[e]);
            if (beta != 0.0)
                r += beta * C0[gi * ldc0 + gj];
            if (gi == gj)
                r += gamma;
            C[gi * ldc + gj] = r;
            if (bx != by)
                C[gj * ldc + gi] = r;
        }
    }
}

template <bool SYM>
static bool gemm128_fits(int64_t M, int64_t N, const double *A, int64_t lda, const double *B,
                         int64_t ldb)
{
    return M >= BT && N >= BT && lda % 2 == 0 && ldb % 2 == 0 &&
           (reinterpret_cast<uintptr_t>(A) % 16) == 0 && (reinterpret_cast<uintptr_t>(B) % 16) == 0;
}

static int gemm_resident_slots()
{
    static int slots = 0; // two workgroups per compute unit (waves_per_eu(2, 2))
    if (slots == 0) {
        int dev = 0, cus = 0;
        hipGetDevice(&dev);
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        slots = 2 * (cus > 0 ? cus : 256);
    }
    return slots;
}

template <bool SYM>
static hipError_t launch_gemm128(int transA, int transB, int64_t M, int64_t N, int64_t K,
                                 double alpha, const double *A, int64_t lda, const double *B,
                                 int64_t ldb, double beta, const double *C0, int64_t ldc0,
                                 double gamma, double *C, int64_t ldc, double *scratch,
                                 int64_t scratch_doubles, int slots, hipStream_t s,
                                 int64_t batch = 1, int64_t sA = 0, int64_t sB = 0,
                                 int64_t sC0 = 0, int64_t sC = 0)
{
    if (SYM && batch != 1)
        return hipErrorInvalidValue;
    const int tn = (int)((N + BT - 1) / BT), tm = (int)((M + BT - 1) / BT);
    const int ntiles = tn * (tn + 1) / 2;
    const int G = slots > 0 ? slots : gemm_resident_slots();
    if (SYM && ntiles > G && K >= BK && scratch &&
        scratch_doubles >= (int64_t)2 * (G - 1) * BT * BT) {
#define LJ_GSK(TA_, TB_)                                                                           \
    hipLaunchKernelGGL((gemm128_sk_kernel<TA_, TB_>), dim3((unsigned)G), dim3(256), 0, s, M, N, K,  \
                       alpha, A, lda, B, ldb, beta, C0, ldc0, gamma, C, ldc, tn, ntiles, scratch)
        if (!transA && !transB)
            LJ_GSK(0, 0);
        else if (transA && !transB)
            LJ_GSK(1, 0);
        else if (!transA && transB)
            LJ_GSK(0, 1);
        else
            LJ_GSK(1, 1);
#undef LJ_GSK
        hipLaunchKernelGGL(gemm128_sk_fixup_kernel, dim3((unsigned)(G - 1)), dim3(256), 0, s, M,
                           N, K, alpha, beta, C0, ldc0, gamma, C, ldc, tn, ntiles, G, scratch);
        return hipGetLastError();
    }
    dim3 grid = SYM ? dim3((unsigned)ntiles) : dim3((unsigned)tn, (unsigned)tm, (unsigned)batch);
#define LJ_G128(TA_, TB_)                                                                          \
    hipLaunchKernelGGL((gemm128_kernel<TA_, TB_, SYM>), grid, dim3(256), 0, s, M, N, K, alpha, A,  \
                       lda, B, ldb, beta, C0, ldc0, gamma, C, ldc, tn, sA, sB, sC0, sC)
    if (!transA && !transB)
        LJ_G128(0, 0);
    else if (transA && !transB)
        LJ_G128(1, 0);
    else if (!transA && transB)
        LJ_G128(0, 1);
    else
        LJ_G128(1, 1);
#undef LJ_G128
    return hipGetLastError();
}

template <bool SYM>
static hipError_t launch_gemm64_t(int transA, int transB, int64_t M, int64_t N, int64_t K,
                                  double alpha, const double *A, int64_t lda, int64_t sA,
                                  const double *B, int64_t ldb, int64_t sB, double beta,
                                  const double *C0, int64_t ldc0, int64_t sC0, double gamma,
                                  double *C, int64_t ldc, int64_t sC, int64_t batch,
                                  double *scratch, int64_t scratch_doubles, int slots,
                                  hipStream_t s)
{
    if (M <= 0 || N <= 0 || batch <= 0)
        return hipSuccess;
    // the 128 x 128 tiles (double-buffered LDS) for a single product and for
    // batches of plain products whose entries keep the 16-byte alignment
    if (gemm128_fits<SYM>(M, N, A, lda, B, ldb) &&
        (batch == 1 || (!SYM && sA % 2 == 0 && sB % 2 == 0)))
        return launch_gemm128<SYM>(transA, transB, M, N, K, alpha, A, lda, B, ldb, beta, C0,
                                   ldc0, gamma, C, ldc, scratch, scratch_doubles, slots, s, batch,
                                   sA, sB, sC0, sC);
    dim3 grid((unsigned)((N + GT - 1) / GT), (unsigned)((M + GT - 1) / GT), (unsigned)batch);
    if (!transA && !transB)
        hipLaunchKernelGGL((gemm64_kernel<0, 0, SYM>), grid, dim3(256), 0, s, M, N, K, alpha, A,
                           lda, sA, B, ldb, sB, beta, C0, ldc0, sC0, gamma, C, ldc, sC);
    else if (transA && !transB)
        hipLaunchKernelGGL((gemm64_kernel<1, 0, SYM>), grid, dim3(256), 0, s, M, N, K, alpha, A,
                           lda, sA, B, ldb, sB, beta, C0, ldc0, sC0, gamma, C, ldc, sC);
    else if (!transA && transB)
        hipLaunchKernelGGL((gemm64_kernel<0, 1, SYM>), grid, dim3(256), 0, s, M, N, K, alpha, A,
                           lda, sA, B, ldb, sB, beta, C0, ldc0, sC0, gamma, C, ldc, sC);
    else
        hipLaunchKernelGGL((gemm64_kernel<1, 1, SYM>), grid, dim3(256), 0, s, M, N, K, alpha, A,
                           lda, sA, B, ldb, sB, beta, C0, ldc0, sC0, gamma, C, ldc, sC);
    return hipGetLastError();
}

hipError_t launch_gemm64(int transA, int transB, int64_t M, int64_t N, int64_t K, double alpha,
                         const double *A, int64_t lda, int64_t sA, const double *B, int64_t ldb,
                         int64_t sB, double beta, const double *C0, int64_t ldc0, int64_t sC0,
                         double gamma, double *C, int64_t ldc, int64_t sC, int64_t batch,
                         hipStream_t s)
{
    return launch_gemm64_t<false>(transA, transB, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta,
                                  C0, ldc0, sC0, gamma, C, ldc, sC, batch, nullptr, 0, 0, s);
}

hipError_t launch_gemm64_sym(int transA, int transB, int64_t N, int64_t K, double alpha,
                             const double *A, int64_t lda, const double *B, int64_t ldb,
                             double beta, const double *C0, int64_t ldc0, double gamma, double *C,
                             int64_t ldc, hipStream_t s, double *scratch, int64_t scratch_doubles,
                             int slots)
{
    return launch_gemm64_t<true>(transA, transB, N, N, K, alpha, A, lda, 0, B, ldb, 0, beta, C0,
                                 ldc0, 0, gamma, C, ldc, 0, 1, scratch, scratch_doubles, slots,
                                 s);
}

__global__ __launch_bounds__(256) void sq_partial_kernel(const double *__restrict__ X,
                                                         int64_t count,
                                                         double *__restrict__ partial)
{
    __shared__ double red[4];
    double acc = 0.0;
    for (int64_t e = blockIdx.x * 256 + threadIdx.x; e < count; e += (int64_t)gridDim.x * 256)
        acc += X[e] * X[e];
    acc = wave_sum(acc);
    if (threadIdx.x % WAVE == 0)
        red[threadIdx.x / WAVE] = acc;
    __syncthreads();
    if (threadIdx.x == 0)
        partial[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

hipError_t launch_sq_partial(const double *X, int64_t count, double *partial, hipStream_t s)
{
    hipLaunchKernelGGL(sq_partial_kernel, dim3(OFF_BLOCKS), dim3(256), 0, s, X, count, partial);
    return hipGetLastError();
}

// M <- diag(dW) + F o M with F_ij = 1/(W_j - W_i) (i != j), F_ii = 0; a pair
// closer than gap_tol contributes 0 and raises the DEGENERATE flag when its
// coupling is nonzero.
__global__ __launch_bounds__(256) void adjoint_mid_kernel(double *__restrict__ Mm,
                                                          const double *__restrict__ W,
                                                          const double *__restrict__ dW,
                                                          int64_t n, int64_t batch,
                                                          double gap_tol, int has_dv, int *flag)
{
    const int64_t total = batch * n * n;
    int degen = 0;
    for (int64_t e = blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
        int64_t z = e / (n * n), r = e - z * n * n;
        int64_t i = r / n, j = r - (r / n) * n;
        double m;
        if (i == j) {
            m = dW ? dW[z * n + i] : 0.0;
        } else {
            double mv = has_dv ? Mm[e] : 0.0;
            double gap = W[z * n + j] - W[z * n + i];
            if (fabs(gap) < gap_tol) {
                if (mv != 0.0)
                    degen = 1;
                m = 0.0;
            } else {
                m = mv / gap;
            }
        }
        Mm[e] = m;
    }
    if (__any(degen) && threadIdx.x % WAVE == 0)
        atomicOr(flag, 1);
}

// The same entries on a (column chunk, row, matrix) grid: no index divisions.
__global__ __launch_bounds__(256) void adjoint_mid_grid_kernel(double *__restrict__ Mm,
                                                               const double *__restrict__ W,
                                                               const double *__restrict__ dW,
                                                               int64_t n, double gap_tol,
                                                               int has_dv, int *flag)
{
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x, i = blockIdx.y, z = blockIdx.z;
    int degen = 0;
    if (j < n) {
        const int64_t e = (z * n + i) * n + j;
        double m;
        if (i == j) {
            m = dW ? dW[z * n + i] : 0.0;
        } else {
            double mv = has_dv ? Mm[e] : 0.0;
            double gap = W[z * n + j] - W[z * n + i];
            if (fabs(gap) < gap_tol) {
                if (mv != 0.0)
                    degen = 1;
                m = 0.0;
            } else {
                m = mv / gap;
            }
        }
        Mm[e] = m;
    }
    if (__any(degen) && threadIdx.x % WAVE == 0)
        atomicOr(flag, 1);
}

hipError_t launch_adjoint_mid(double *M, const double *W, const double *dW, int64_t n,
                              int64_t batch, double gap_tol, int has_dv, int *flag, hipStream_t s)
{
    if (n <= 65535 && batch <= 65535)
        hipLaunchKernelGGL(adjoint_mid_grid_kernel, dim3((unsigned)((n + 255) / 256),
                                                         (unsigned)n, (unsigned)batch),
                           dim3(256), 0, s, M, W, dW, n, gap_tol, has_dv, flag);
    else
        hipLaunchKernelGGL(adjoint_mid_kernel, dim3(2048), dim3(256), 0, s, M, W, dW, n, batch,
                           gap_tol, has_dv, flag);
    return hipGetLastError();
}

// dA = (G + G^T)/2 per matrix; G packed (n x n each), dA with row stride ld and
// matrix stride n ld
__global__ __launch_bounds__(256) void sym_out_kernel(const double *__restrict__ G,
                                                      double *__restrict__ dA, int64_t n,
                                                      int64_t ld, int64_t batch)
{
    const int64_t total = batch * n * n;
    for (int64_t e = blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
        int64_t z = e / (n * n), r = e - z * n * n;
        int64_t i = r / n, j = r - (r / n) * n;
        dA[z * n * ld + i * ld + j] = 0.5 * (G[e] + G[z * n * n + j * n + i]);
    }
}

// The same entries by 32 x 32 tiles: workgroup (I, J, matrix), I <= J, reads
// the tiles G_IJ and G_JI once along their rows into LDS and writes dA_IJ and
// dA_JI along their rows (the transposed reads come from LDS; the row stride
// 33 keeps them free of bank conflicts).  Workgroups with I > J return.
constexpr int SYM_T = 32;
__global__ __launch_bounds__(256) void sym_out_tiled_kernel(const double *__restrict__ G,
                                                            double *__restrict__ dA, int64_t n,
                                                            int64_t ld)
{
    const int I = blockIdx.x, J = blockIdx.y;
    if (I > J)
        return;
    __shared__ double a[SYM_T][SYM_T + 1], b[SYM_T][SYM_T + 1];
    const int64_t z = blockIdx.z;
    const double *Gz = G + z * n * n;
    double *Dz = dA + z * n * ld;
    const int tx = threadIdx.x % SYM_T, ty = threadIdx.x / SYM_T; // 8 rows per pass
    const int64_t i0 = (int64_t)I * SYM_T, j0 = (int64_t)J * SYM_T;
#pragma unroll
    for (int rr = 0; rr < SYM_T; rr += 8) {
        const int row = ty + rr;
        a[row][tx] = (i0 + row < n && j0 + tx < n) ? Gz[(i0 + row) * n + j0 + tx] : 0.0;
        b[row][tx] = (j0 + row < n && i0 + tx < n) ? Gz[(j0 + row) * n + i0 + tx] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int rr = 0; rr < SYM_T; rr += 8) {
        const int row = ty + rr;
        // dA_IJ[row][tx] = (G_IJ[row][tx] + G_JI[tx][row]) / 2
        if (i0 + row < n && j0 + tx < n)
            Dz[(i0 + row) * ld + j0 + tx] = 0.5 * (a[row][tx] + b[tx][row]);
        // dA_JI[row][tx] = (G_JI[row][tx] + G_IJ[tx][row]) / 2
        if (I != J && j0 + row < n && i0 + tx < n)
            Dz[(j0 + row) * ld + i0 + tx] = 0.5 * (b[row][tx] + a[tx][row]);
    }
}

hipError_t launch_sym_out(const double *G, double *dA, int64_t n, int64_t ld, int64_t batch,
                          hipStream_t s)
{
    const int64_t nt = (n + SYM_T - 1) / SYM_T;
    if (nt <= 65535 && batch <= 65535)
        hipLaunchKernelGGL(sym_out_tiled_kernel, dim3((unsigned)nt, (unsigned)nt, (unsigned)batch),
                           dim3(256), 0, s, G, dA, n, ld);
    else
        hipLaunchKernelGGL(sym_out_kernel, dim3(2048), dim3(256), 0, s, G, dA, n, ld, batch);
    return hipGetLastError();
}

} // namespace lj
