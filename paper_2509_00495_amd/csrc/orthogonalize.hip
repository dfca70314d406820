// Orthogonalisers of the mixed path other than Newton-Schulz: Q_d from a QR
// factorisation of the widened low-precision eigenvectors Q_l.
//   * Householder QR (Algorithm 5, Section 4.2) in blocked form: panels of
//     HB = 16 columns are factored by one workgroup each (Algorithm 1 per
//     column, the reflectors kept as V and the compact factor T with
//     P_1 ... P_HB = I - V T V^T), the trailing columns get the whole panel at
//     once through three FP64 GEMMs, and Q is accumulated backwards over the
//     panels the same way.
//   * Cholesky QR (named in Chapter 6): G = X^T X, R = chol(G) by blocks of
//     CB = 64 (one workgroup factors and inverts each diagonal block in LDS,
//     GEMMs do the rest), then Q = X R^{-1} by a right-looking blocked solve.
// Both are comparators for the paper's Newton-Schulz choice (the accuracy and
// cost comparison of Section 4.4); the default pipeline keeps Newton-Schulz.
#include "internal.hpp"
#include "common.hpp"

namespace lj {

// ------------------------------------------------------------ Cholesky QR
// Upper Cholesky factor of the nb x nb diagonal block of G at (j0, j0)
// (nb = min(CB, n - j0)), written to R's block (zeros below its diagonal),
// and the inverse of that factor to Rinv (CB x CB, row-major).  Right-looking
// on the upper triangle in LDS: r_ii = sqrt(a_ii), row i scaled by 1/r_ii,
// then a_kl -= r_ik r_il for i < k <= l.  A pivot that is not positive sets
// *bad (the factorisation continues with NaN, which the caller reports).
constexpr int CB = ORTH_CB;
__global__ __launch_bounds__(256) void chol_diag_kernel(const double *__restrict__ G,
                                                        int64_t ldg, int64_t j0, int64_t n,
                                                        double *__restrict__ R, int64_t ldr,
                                                        double *__restrict__ Rinv, int *bad)
{
    __shared__ double a[CB][CB + 1];
    __shared__ double x[CB][CB + 1];
    const int tid = threadIdx.x;
    const int nb = (int)(n - j0 < CB ? n - j0 : CB);
    for (int e = tid; e < CB * CB; e += 256) {
        const int i = e / CB, j = e % CB;
        a[i][j] = (i < nb && j < nb && j >= i) ? G[(j0 + i) * ldg + j0 + j] : 0.0;
        x[i][j] = 0.0;
    }
    __syncthreads();
    for (int i = 0; i < nb; ++i) {
        const double d = a[i][i];
        if (tid == 0 && !(d > 0.0))
            atomicOr(bad, 1);
        const double r = sqrt(d);
        __syncthreads(); // everyone has read a[i][i]
        for (int j = i + 1 + tid; j < nb; j += 256)
            a[i][j] /= r;
        if (tid == 0)
            a[i][i] = r;
        __syncthreads();
        const int m = nb - i - 1; // trailing block (i+1 .. nb-1), upper triangle
        for (int e = tid; e < m * m; e += 256) {
            const int k = i + 1 + e / m, l = i + 1 + e % m;
            if (l >= k)
                a[k][l] -= a[i][k] * a[i][l];
        }
        __syncthreads();
    }
    // inverse of the upper-triangular factor, one column per thread:
    // x_c = 1 / r_cc, x_i = -(sum_{k=i+1..c} r_ik x_k) / r_ii
    if (tid < nb) {
        const int c = tid;
        x[c][c] = 1.0 / a[c][c];
        for (int i = c - 1; i >= 0; --i) {
            double s = 0.0;
            for (int k = i + 1; k <= c; ++k)
                s += a[i][k] * x[k][c];
            x[i][c] = -s / a[i][i];
        }
    }
    __syncthreads();
    for (int e = tid; e < CB * CB; e += 256) {
        const int i = e / CB, j = e % CB;
        if (i < nb && j < nb)
            R[(j0 + i) * ldr + j0 + j] = j >= i ? a[i][j] : 0.0;
        Rinv[e] = (i < nb && j < nb && j >= i) ? x[i][j] : 0.0;
    }
}

// Q = X R^{-1} with R = chol(X^T X).  X (n x n, ld, destroyed), Q, G and Rf
// are n x n with the same ld (G may be Q: the Gram matrix is dead before Q is
// written; Rf receives R's upper triangle, its strictly lower part is left
// as it was), Rinv holds ceil(n / CB) CB x CB blocks, bad one int (device,
// set when a pivot is not positive).  Returns the first HIP error.
hipError_t cholesky_qr(double *X, double *Q, double *G, double *Rf, int64_t n, int64_t ld,
                       double *Rinv, int *bad, hipStream_t s)
{
    hipError_t e = launch_gemm64_sym(1, 0, n, n, 1.0, X, ld, X, ld, 0.0, nullptr, 0, 0.0, G, ld,
                                     s);
    if (e != hipSuccess)
        return e;
    const int64_t nblk = (n + CB - 1) / CB;
    for (int64_t jb = 0; jb < nblk; ++jb) {
        const int64_t j0 = jb * CB, nb = n - j0 < CB ? n - j0 : CB, rest = n - j0 - nb;
        hipLaunchKernelGGL(chol_diag_kernel, dim3(1), dim3(256), 0, s, G, ld, j0, n, Rf, ld,
                           Rinv + jb * CB * CB, bad);
        if (rest > 0) {
            // R(j, rest) = R_jj^{-T} G(j, rest)
            e = launch_gemm64(1, 0, nb, rest, nb, 1.0, Rinv + jb * CB * CB, CB, 0,
                              G + j0 * ld + j0 + nb, ld, 0, 0.0, nullptr, 0, 0, 0.0,
                              Rf + j0 * ld + j0 + nb, ld, 0, 1, s);
            if (e != hipSuccess)
                return e;
            // G(rest, rest) -= R(j, rest)^T R(j, rest)  (symmetric, in place)
            e = launch_gemm64_sym(1, 0, rest, nb, -1.0, Rf + j0 * ld + j0 + nb, ld,
                                  Rf + j0 * ld + j0 + nb, ld, 1.0, G + (j0 + nb) * ld + j0 + nb,
                                  ld, 0.0, G + (j0 + nb) * ld + j0 + nb, ld, s);
            if (e != hipSuccess)
                return e;
        }
    }
    // Q R = X, panels left to right: Q_j = X_j R_jj^{-1}, then the later
    // panels of X lose Q_j R(j, rest)
    for (int64_t jb = 0; jb < nblk; ++jb) {
        const int64_t j0 = jb * CB, nb = n - j0 < CB ? n - j0 : CB, rest = n - j0 - nb;
        e = launch_gemm64(0, 0, n, nb, nb, 1.0, X + j0, ld, 0, Rinv + jb * CB * CB, CB, 0, 0.0,
                          nullptr, 0, 0, 0.0, Q + j0, ld, 0, 1, s);
        if (e != hipSuccess)
            return e;
        if (rest > 0) {
            e = launch_gemm64(0, 0, n, rest, nb, -1.0, Q + j0, ld, 0, Rf + j0 * ld + j0 + nb, ld, 0,
                              1.0, X + j0 + nb, ld, 0, 0.0, X + j0 + nb, ld, 0, 1, s);
            if (e != hipSuccess)
                return e;
        }
    }
    return hipGetLastError();
}

// ------------------------------------------------------- Householder QR
// One panel of HB columns (j0 .. j0 + HB - 1, rows j0 .. n - 1) of A, by one
// workgroup: for each column c = j0 + k, Algorithm 1 on A(c:n, c) (sigma and
// mu by a block reduction, v_1 = x_1 + mu for x_1 >= 0, else x_1 - mu, beta =
// 2 / (v_1^2 + sigma), beta = 0 for a zero column), the column becomes
// -sign(x_1) mu e_1, and the panel's later columns get
// A(c:n, c') -= beta v (v^T A(c:n, c')).  The reflectors go to V (column
// j0 + k, rows c .. n - 1, v_1 at row c; zero above) and the compact factor
// T of P_1 ... P_HB = I - V T V^T (upper triangular, T_kk = beta_k,
// T(0:k, k) = -beta_k T(0:k, 0:k) V(:, 0:k)^T v_k) to T (HB x HB).
// Thread t works on column slot t mod HB of the rows j0 + t / HB + i HNT / HB,
// so the HB lanes of a row read its HB panel entries as one contiguous
// piece; x_i, the entry of column k, reaches the other lanes of its row by a
// shuffle.  One pass over the rows below the pivot gives, in a single
// reduction, sigma (column k with itself) and x^T A(r+1:n, c) and
// x^T V(r+1:n, c) for every other slot; the pivot row's term v_1 A(r, c) is
// added afterwards, once v_1 is known.  A second pass applies the update.
// Rows are loaded RU at a time per thread before they are used, so the
// loads of a pass overlap.
constexpr int HB = ORTH_HB;
constexpr int HNT = 1024;
__global__ __launch_bounds__(HNT) void house_panel_kernel(double *__restrict__ A, int64_t ld,
                                                          int64_t n, int64_t j0,
                                                          double *__restrict__ V, int64_t ldv,
                                                          double *__restrict__ T)
{
    constexpr int NW = HNT / WAVE, RG = HNT / HB, RU = 4;
    static_assert(WAVE % HB == 0, "a row's slots lie in one wavefront");
    __shared__ double red[NW][HB];
    __shared__ double tot[HB];
    __shared__ double ts[HB][HB];
    const int tid = threadIdx.x, lane = tid % WAVE, w = tid / WAVE;
    const int cs = tid % HB, rg = tid / HB;       // column slot, row group
    const int src = (lane / HB) * HB;             // lane of slot 0 of this row
    const int nbc = (int)(n - j0 < HB ? n - j0 : HB); // columns in this panel
    const bool colok = cs < nbc;
    const int64_t col = j0 + cs;
    for (int e = tid; e < HB * HB; e += HNT)
        ts[e / HB][e % HB] = 0.0;
    // the panel's V columns are zero above their pivots
    for (int64_t e = tid; e < (j0 + HB) * nbc; e += HNT) {
        const int64_t i = e / nbc;
        const int k = (int)(e % nbc);
        if (i < j0 + k && i < n)
            V[i * ldv + j0 + k] = 0.0;
    }
    // tot[c] = sum over all threads of slot c of v
    auto slot_sums = [&](double v) {
#pragma unroll
        for (int off = HB; off < WAVE; off <<= 1)
            v += __shfl_xor(v, off, WAVE);
        if (lane < HB)
            red[w][lane] = v;
        __syncthreads();
        if (tid < HB) {
            double s = 0.0;
            for (int i = 0; i < NW; ++i)
                s += red[i][tid];
            tot[tid] = s;
        }
        __syncthreads();
    };
    for (int k = 0; k < nbc; ++k) {
        const int64_t r = j0 + k, c = j0 + k;
        // pass 1, rows r+1 .. n-1: slot k sums x_i^2 (sigma), a later slot
        // x_i A(i, c), an earlier slot x_i V(i, c).  The chunk loop is the
        // same for every lane of a wavefront (its rows are guarded one by
        // one), so every shuffle has its whole row active.
        double pd = 0.0;
        for (int64_t i0 = j0; i0 < n; i0 += (int64_t)RU * RG) {
            double a[RU], b[RU];
#pragma unroll
            for (int u = 0; u < RU; ++u) {
                const int64_t i = i0 + rg + (int64_t)u * RG;
                const bool in = i > r && i < n;
                a[u] = in && colok ? A[i * ld + col] : 0.0;
                b[u] = in && cs < k ? V[i * ldv + col] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < RU; ++u) {
                const double xk = __shfl(a[u], src + k, WAVE);
                pd += xk * (cs < k ? b[u] : a[u]);
            }
        }
        slot_sums(pd);
        const double sigma = tot[k];
        const double x0 = A[r * ld + c];
        const double mu = sqrt(x0 * x0 + sigma);
        double v0 = 1.0, beta = 0.0;
        if (mu != 0.0) {
            v0 = x0 >= 0.0 ? x0 + mu : x0 - mu;
            beta = 2.0 / (v0 * v0 + sigma);
        }
        // w_c = v^T A(r:n, c) of this thread's (later) slot
        const double wc = cs > k && colok ? tot[cs] + v0 * A[r * ld + col] : 0.0;
        // T(k, k) = beta_k, T(0:k, k) = -beta_k T(0:k, 0:k) g with g_b =
        // V(:, j0 + b)^T v (b < k)
        if (tid < k) {
            double sacc = 0.0;
            for (int b = tid; b < k; ++b)
                sacc += ts[tid][b] * (tot[b] + v0 * V[r * ldv + j0 + b]);
            ts[tid][k] = -beta * sacc;
        }
        if (tid == 0)
            ts[k][k] = beta;
        __syncthreads(); // tot and the pivot row are read before pass 2 writes
        // pass 2, rows r .. n-1: the update
        for (int64_t i0 = j0; i0 < n; i0 += (int64_t)RU * RG) {
            double a[RU];
#pragma unroll
            for (int u = 0; u < RU; ++u) {
                const int64_t i = i0 + rg + (int64_t)u * RG;
                a[u] = i >= r && i < n && colok ? A[i * ld + col] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < RU; ++u) {
                const int64_t i = i0 + rg + (int64_t)u * RG;
                const double xk = __shfl(a[u], src + k, WAVE);
                if (i < r || i >= n)
                    continue;
                const double vi = i == r ? v0 : xk;
                if (cs > k && colok) {
                    A[i * ld + col] = a[u] - beta * vi * wc;
                } else if (cs == k) {
                    V[i * ldv + col] = vi;
                    A[i * ld + col] = i == r ? (x0 >= 0.0 ? -mu : mu) : 0.0;
                }
            }
        }
        __syncthreads();
    }
    for (int e = tid; e < HB * HB; e += HNT)
        T[e] = ts[e / HB][e % HB];
}

// W = V^T B for a panel of nb <= 16 reflectors: V is K x nb (row stride ldv),
// B is K x N (row stride ldb), W is nb x N (row stride ldw).  One workgroup
// per 16 columns of W; its four wavefronts split K, each accumulating a
// 16 x 16 part on the FP64 16x16x4 MFMA with both operands read straight
// from the rows of V and B (four rows of 128 bytes per step), and the parts
// are added in LDS.  (The generic 64 x 64-tile GEMM spends three quarters of
// its tile on the nb = 16 rows and puts only N / 64 workgroups on a long K.)
constexpr int VTB_U = 8; // MFMA steps whose loads are issued together
__global__ __launch_bounds__(256) void vtb_kernel(const double *__restrict__ V, int64_t ldv,
                                                  int nb, const double *__restrict__ B,
                                                  int64_t ldb, int64_t K, int64_t N,
                                                  double *__restrict__ W, int64_t ldw)
{
    __shared__ double part[4][16 * 17];
    const int tid = threadIdx.x, lane = tid % WAVE, w = tid / WAVE;
    const int li = lane % 16, lk = lane / 16;
    const int64_t j = (int64_t)blockIdx.x * 16 + li;
    const int64_t steps = (K + 3) / 4;
    const int64_t s0 = w * steps / 4, s1 = (w + 1) * steps / 4;
    d4 acc = {0.0, 0.0, 0.0, 0.0};
    for (int64_t st = s0; st < s1; st += VTB_U) {
        double a[VTB_U], b[VTB_U];
#pragma unroll
        for (int u = 0; u < VTB_U; ++u) {
            const int64_t k = 4 * (st + u) + lk;
            const bool in = st + u < s1 && k < K;
            a[u] = in && li < nb ? V[k * ldv + li] : 0.0; // V^T(li, k)
            b[u] = in && j < N ? B[k * ldb + j] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < VTB_U; ++u)
            acc = mfma16(a[u], b[u], acc);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v)
        part[w][acc_row<double>(lk, v) * 17 + li] = acc[v];
    __syncthreads();
    const int i = tid / 16, c = tid % 16;
    const int64_t jc = (int64_t)blockIdx.x * 16 + c;
    if (i < nb && jc < N)
        W[i * ldw + jc] = part[0][i * 17 + c] + part[1][i * 17 + c] + part[2][i * 17 + c] +
                          part[3][i * 17 + c];
}

static hipError_t launch_vtb(const double *V, int64_t ldv, int nb, const double *B, int64_t ldb,
                             int64_t K, int64_t N, double *W, int64_t ldw, hipStream_t s)
{
    if (N <= 0 || nb <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(vtb_kernel, dim3((unsigned)((N + 15) / 16)), dim3(256), 0, s, V, ldv, nb,
                       B, ldb, K, N, W, ldw);
    return hipGetLastError();
}

// Householder QR of X (n x n, ld): Q (n x n, ld) with X = Q R.  X is
// destroyed (R in its upper triangle), Vs (n x n, ld) keeps the reflectors,
// Ts ceil(n / HB) HB x HB factors, W and W2 HB x n scratch.
hipError_t householder_qr(double *X, double *Q, double *Vs, int64_t n, int64_t ld, double *Ts,
                          double *W, double *W2, hipStream_t s)
{
    hipError_t e;
    const int64_t np = (n + HB - 1) / HB;
    for (int64_t p = 0; p < np; ++p) {
        const int64_t j0 = p * HB, nb = n - j0 < HB ? n - j0 : HB, m = n - j0,
                      rest = n - j0 - nb;
        hipLaunchKernelGGL(house_panel_kernel, dim3(1), dim3(HNT), 0, s, X, ld, n, j0, Vs, ld,
                           Ts + p * HB * HB);
        if (rest > 0) {
            // A(j0:, j0+nb:) <- (I - V T V^T)^T A = A - V T^T (V^T A)
            e = launch_vtb(Vs + j0 * ld + j0, ld, (int)nb, X + j0 * ld + j0 + nb, ld, m, rest, W,
                           rest, s);
            if (e != hipSuccess)
                return e;
            e = launch_gemm64(1, 0, nb, rest, nb, 1.0, Ts + p * HB * HB, HB, 0, W, rest, 0, 0.0,
                              nullptr, 0, 0, 0.0, W2, rest, 0, 1, s);
            if (e != hipSuccess)
                return e;
            e = launch_gemm64(0, 0, m, rest, nb, -1.0, Vs + j0 * ld + j0, ld, 0, W2, rest, 0, 1.0,
                              X + j0 * ld + j0 + nb, ld, 0, 0.0, X + j0 * ld + j0 + nb, ld, 0, 1,
                              s);
            if (e != hipSuccess)
                return e;
        }
    }
    // Q = P_1 P_2 ... applied to I, last panel first:
    // Q(j0:, j0:) <- (I - V T V^T) Q(j0:, j0:)
    e = launch_eye<double>(Q, ld, s);
    if (e != hipSuccess)
        return e;
    for (int64_t p = np - 1; p >= 0; --p) {
        const int64_t j0 = p * HB, nb = n - j0 < HB ? n - j0 : HB, m = n - j0;
        e = launch_vtb(Vs + j0 * ld + j0, ld, (int)nb, Q + j0 * ld + j0, ld, m, m, W, m, s);
        if (e != hipSuccess)
            return e;
        e = launch_gemm64(0, 0, nb, m, nb, 1.0, Ts + p * HB * HB, HB, 0, W, m, 0, 0.0, nullptr, 0,
                          0, 0.0, W2, m, 0, 1, s);
        if (e != hipSuccess)
            return e;
        e = launch_gemm64(0, 0, m, m, nb, -1.0, Vs + j0 * ld + j0, ld, 0, W2, m, 0, 1.0,
                          Q + j0 * ld + j0, ld, 0, 0.0, Q + j0 * ld + j0, ld, 0, 1, s);
        if (e != hipSuccess)
            return e;
    }
    return hipGetLastError();
}

} // namespace lj
