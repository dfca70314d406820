// One-workgroup Jacobi solver: the whole (symmetrised) matrix lives in LDS and
// a workgroup runs complete sweeps of the parallel round-robin ordering until
// off(B) <= tol (Algorithm 4, Section 3.3, with the parallel ordering of
// lds_jacobi_round).  Persistent: each workgroup pops matrices from a device
// work queue (descriptors sorted by n, largest first), so one launch solves a
// whole batch of matrices of uneven order.
#include "internal.hpp"
#include "lds_jacobi.hpp"

namespace lj {

template <int NT>
__global__ __launch_bounds__(NT) void small_jacobi_kernel(
    const double *__restrict__ A, double *__restrict__ W, double *__restrict__ Vout,
    const SmallDesc *__restrict__ desc, int count, int *queue, double tol_in,
    int max_sweeps, double *__restrict__ vscratch, int64_t vscratch_stride,
    int pool, int m_max, int32_t *status)
{
    extern __shared__ __align__(16) double smem[];
    const int tid = threadIdx.x;
    double *S = smem;                                  // pool: S, then V if it fits
    double *cs = smem + ((pool + 1) & ~1);             // 2 x 3 * m_max / 2, 16-byte aligned
    double *cs1 = cs + 3 * (m_max / 2);                //   (angles of alternate rounds)
    double *wv = cs1 + 3 * (m_max / 2);                // m_max
    double *sg = wv + m_max;                           // m_max
    double *red = sg + m_max;                          // 16
    int *perm = (int *)(red + 16);                     // m_max
    int *slot = perm + m_max;                          // 1
    int *ired = slot + 1;                              // 16

    for (;;) {
        if (tid == 0)
            *slot = atomicAdd(queue, 1);
        __syncthreads();
        const int it = *slot;
        __syncthreads();
        if (it >= count)
            break;
        const SmallDesc d = desc[it];
        const int n = d.n;
        const int m = (n + 3) & ~3;
        const int ld = m + 1;
        const double *Ai = A + d.a_off;

        // ingest: S = (A + A^T)/2, zero padding to m
        double nrm = 0.0, amax = 0.0;
        int finite = 1;
        for (int idx = tid; idx < m * m; idx += NT) {
            int i = idx / m, j = idx - (idx / m) * m;
            double v = 0.0;
            if (i < n && j < n) {
                double a = Ai[(int64_t)i * d.lda + j], b = Ai[(int64_t)j * d.lda + i];
                v = 0.5 * (a + b);
                if (!isfinite(a))
                    finite = 0;
            }
            S[i * ld + j] = v;
            nrm += v * v;
            amax = fmax(amax, fabs(v));
        }
        double nrm2 = block_sum<NT>(nrm, red);
        const int bad = block_or<NT>(!finite, ired);
        if (bad) {
            if (tid == 0 && status)
                status[d.orig] = JACOBI_NONFINITE;
            continue;
        }
        // exact power-of-two scaling of inputs whose largest entry is outside
        // [2^-100, 2^100] (the same for every thread); W is scaled back
        const int ks = scale_exp_of(block_max<NT>(amax, red));
        if (ks) {
            nrm = 0.0;
            for (int idx = tid; idx < m * m; idx += NT) {
                const int i = idx / m, j = idx - (idx / m) * m;
                const double v = ldexp2(S[i * ld + j], ks);
                S[i * ld + j] = v;
                nrm += v * v;
            }
            nrm2 = block_sum<NT>(nrm, red);
        }
        // V is kept transposed: Vt[p][i] = V[i][p], m rows of stride ldt
        const int ldt = (n + 1) & ~1;
        const bool v_lds = (int64_t)m * ld + small_vt_elems(n) <= pool;
        double *Vt = v_lds ? S + m * ld : vscratch + (int64_t)blockIdx.x * vscratch_stride;
        for (int idx = tid; idx < m * ldt; idx += NT) {
            int p = idx / ldt, i = idx - (idx / ldt) * ldt;
            Vt[idx] = (p == i) ? 1.0 : 0.0;
        }
        const double tol = tol_in > 0.0 ? ldexp2(tol_in, ks) : 1e-15 * (double)n * sqrt(nrm2);
        const double thr = n > 0 ? tol / (double)n : 0.0;
        const double eps = 0x1p-53;
        __syncthreads();
        double off2 = lds_off2<double, NT>(S, ld, m, red);
        constexpr int SI = (64 / 2 * (64 + 1) + NT - 1) / NT; // 2x2 blocks per thread, m <= 128
        RoundItems<NT, SI> items;
        items.init(m, n);
        int sweeps = 0, any = 1;
        // Below 1024 threads a thread has several V items per round, and a
        // round's V update needs only that round's angles: the angles of
        // round r + 1 (one wavefront's latency chain) are then computed beside
        // the V update of round r, after round r's S update (two barriers per
        // round, the two angle buffers alternating).  Measured at n = 64:
        // 4096 matrices on 256-thread workgroups 13.2 -> 10.8 ms; with 1024
        // threads (one V item per thread) no gain, so those keep the plain
        // round.
        while (sqrt(off2) > tol && sweeps < max_sweeps && any) {
            int rot = 0;
            if constexpr (NT < 1024) {
                rot = lds_round_angles<double, NT>(S, ld, m, 0, eps, thr, cs);
                __syncthreads();
                for (int r = 0; r < m - 1; ++r) {
                    const double *cc = (r & 1) ? cs1 : cs;
                    double *cn = (r & 1) ? cs : cs1;
                    lds_round_update_s<double, NT, SI>(S, ld, m, r, cc, items);
                    __syncthreads();
                    if (r + 1 < m - 1)
                        rot |= lds_round_angles<double, NT>(S, ld, m, r + 1, eps, thr, cn);
                    lds_round_update_v<double, NT, SI>(Vt, ldt, m, r, cc, items);
                    __syncthreads();
                }
            } else {
                for (int r = 0; r < m - 1; ++r)
                    rot |= lds_jacobi_round<double, NT, SI>(S, ld, m, r, eps, thr, Vt, ldt, cs,
                                                           items);
            }
            any = block_or<NT>(rot, ired);
            ++sweeps;
            off2 = lds_off2<double, NT>(S, ld, m, red);
        }
        // output: W ascending (stable), columns permuted, sign-fixed and normalized
        for (int i = tid; i < m; i += NT) {
            perm[i] = i < n ? i : 0;
            if (i < n)
                wv[i] = S[i * ld + i];
        }
        __syncthreads();
        for (int i = tid; i < n; i += NT) {
            double wi = wv[i];
            int rank = 0;
            for (int j = 0; j < n; ++j) {
                double wj = wv[j];
                rank += (wj < wi) || (wj == wi && j < i);
            }
            perm[rank] = i;
        }
        __syncthreads();
        // sign convention (largest entry positive) and unit 2-norm: the
        // rotations' rounding lets the column norms drift a little
        for (int c = tid; c < n; c += NT) {
            int col = perm[c];
            double best = -1.0, val = 0.0, sq = 0.0;
            for (int i = 0; i < n; ++i) {
                double v = Vt[(int64_t)col * ldt + i];
                sq = fma(v, v, sq);
                if (fabs(v) > best) {
                    best = fabs(v);
                    val = v;
                }
            }
            const double inv = sq > 0.0 ? 1.0 / sqrt(sq) : 1.0;
            sg[c] = val < 0.0 ? -inv : inv;
            W[d.w_off + c] = ks ? ldexp2(wv[col], -ks) : wv[col];
        }
        __syncthreads();
        double *Vo = Vout + d.v_off;
        for (int idx = tid; idx < n * n; idx += NT) {
            int i = idx / n, c = idx - (idx / n) * n;
            Vo[(int64_t)i * d.ldv + c] = sg[c] * Vt[(int64_t)perm[c] * ldt + i];
        }
        if (tid == 0) {
            int st = (sqrt(off2) <= tol || !any) ? JACOBI_OK : JACOBI_NOCONV;
            if (status)
                status[d.orig] = st;
            if (d.info) {
                d.info[0] = (double)sweeps;
                d.info[1] = ldexp2(sqrt(nrm2), -ks);
                d.info[2] = ldexp2(tol, -ks);
                d.info[3] = ldexp2(sqrt(off2), -ks);
            }
        }
        __syncthreads();
    }
}

size_t small_smem_bytes(int m_max, int pool)
{
    size_t d = (size_t)((pool + 1) & ~1) + 2 * 3 * (m_max / 2) + 2 * m_max + 16;
    return d * sizeof(double) + (size_t)(m_max + 1 + 16) * sizeof(int);
}

hipError_t launch_small(const double *A, double *W, double *V, const SmallDesc *desc,
                        int count, int *queue, double tol, int max_sweeps,
                        double *vscratch, int64_t vscratch_stride, int pool,
                        int m_max, int nthreads, int grid, int32_t *status,
                        hipStream_t stream)
{
    size_t smem = small_smem_bytes(m_max, pool);
    if (nthreads == 1024) {
        auto k = small_jacobi_kernel<1024>;
        hipError_t e = hipFuncSetAttribute((const void *)k,
                                           hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)smem);
        if (e != hipSuccess)
            return e;
        hipLaunchKernelGGL(k, dim3(grid), dim3(1024), smem, stream, A, W, V, desc, count,
                           queue, tol, max_sweeps, vscratch, vscratch_stride, pool, m_max,
                           status);
    } else if (nthreads == 512) {
        auto k = small_jacobi_kernel<512>;
        hipError_t e = hipFuncSetAttribute((const void *)k,
                                           hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)smem);
        if (e != hipSuccess)
            return e;
        hipLaunchKernelGGL(k, dim3(grid), dim3(512), smem, stream, A, W, V, desc, count,
                           queue, tol, max_sweeps, vscratch, vscratch_stride, pool, m_max,
                           status);
    } else {
        auto k = small_jacobi_kernel<256>;
        hipError_t e = hipFuncSetAttribute((const void *)k,
                                           hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)smem);
        if (e != hipSuccess)
            return e;
        hipLaunchKernelGGL(k, dim3(grid), dim3(256), smem, stream, A, W, V, desc, count,
                           queue, tol, max_sweeps, vscratch, vscratch_stride, pool, m_max,
                           status);
    }
    return hipGetLastError();
}

int small_max_active(int m_max, int pool, int nthreads)
{
    size_t smem = small_smem_bytes(m_max, pool);
    int nb = 0;
    if (nthreads == 1024)
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, small_jacobi_kernel<1024>, 1024, smem);
    else if (nthreads == 512)
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, small_jacobi_kernel<512>, 512, smem);
    else
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, small_jacobi_kernel<256>, 256, smem);
    return nb;
}

} // namespace lj
