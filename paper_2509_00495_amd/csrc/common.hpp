// Device-side building blocks shared by the libjacobi kernels (gfx950).
//
// Nothing here is shared with the CPU oracle: the oracle lives in its own
// C file and is only used by the tests.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lj {

constexpr int WAVE = 64;

// Round-robin ("circle") schedule for m players, m even: in round r
// (0 <= r < m-1) slot 0 holds player 0 and slot i >= 1 holds player
// 1 + ((i - 1 + r) mod (m - 1)); slot k is paired with slot m-1-k.  Over
// m-1 rounds every unordered pair of players meets exactly once, and the
// m/2 pairs of one round are disjoint, so their rotations commute and can
// be applied together (the parallel ordering that replaces the paper's
// cyclic-by-row sequence of Section 3.3).
__host__ __device__ inline int rr_player(int slot, int r, int m)
{
    return slot == 0 ? 0 : 1 + (slot - 1 + r) % (m - 1);
}

__host__ __device__ inline void rr_pair(int k, int r, int m, int &p, int &q)
{
    int a = rr_player(k, r, m);
    int b = rr_player(m - 1 - k, r, m);
    p = a < b ? a : b;
    q = a < b ? b : a;
}

// Physical layout of the round-robin schedule inside a 2b x 2b pair block
// (M = 2b positions): slot s of the circle method is stored at position
// pos(s) = 2s (s < M/2) or 2(M-1-s)+1, so the pairs of every round are the
// adjacent positions (2k, 2k+1).  Between rounds the players move one slot
// (slot s <- slot s+1, slot M-1 <- slot 1, slot 0 fixed), which in physical
// positions is the fixed permutation sigma; after M-1 rounds every player is
// back in its starting slot.
__host__ __device__ inline int ps_pos(int slot, int M)
{
    return slot < M / 2 ? 2 * slot : 2 * (M - 1 - slot) + 1;
}
__host__ __device__ inline int ps_slot(int p, int M) { return (p & 1) ? M - 1 - (p >> 1) : (p >> 1); }
__host__ __device__ inline int ps_sigma(int p, int M)
{
    int s = ps_slot(p, M);
    int t = s == 0 ? 0 : (s == 1 ? M - 1 : s - 1);
    return ps_pos(t, M);
}

// Map idx in [0, h/2 * (h+1)) to (k, l), 0 <= k <= l < h, h even: row rho of
// the folded rectangle holds the upper-triangle rows rho and h-1-rho.
__device__ inline void tri_fold(int idx, int h, int &k, int &l)
{
    int w = h + 1;
    int rho = idx / w;
    int c = idx - rho * w;
    if (c < h - rho) {
        k = rho;
        l = rho + c;
    } else {
        k = h - 1 - rho;
        l = k + (c - (h - rho));
    }
}

// Rotation that annihilates a_pq of a symmetric 2x2 problem (Algorithm 2,
// Section 3.1.1), with t = 1/(tau +- sqrt(1 + tau^2)) (approach 2 of
// Appendix A) so that |t| <= 1.  J = [c s; -s c]; after J^T A J the diagonal
// is (a_pp - t a_pq, a_qq + t a_pq).  Computed in FP64 for both precisions.
__device__ inline void jacobi_angle(double app, double aqq, double apq,
                                    double &c, double &s, double &t)
{
    double tau = (aqq - app) / (2.0 * apq);
    double root = sqrt(1.0 + tau * tau);
    t = 1.0 / (tau >= 0.0 ? tau + root : tau - root);
    c = 1.0 / sqrt(1.0 + t * t);
    s = t * c;
}

// The same rotation from the hardware reciprocal and reciprocal square root
// (v_rcp_f64, v_rsq_f64), refined by Newton steps (r <- r (2 - x r);
// y <- y (3 - x y^2) / 2).  t only needs to annihilate a_pq to rounding
// level: one step.  c = 1/sqrt(1 + t^2) gets two: a single rsqrt Newton step
// always lands below the root, and that one-sided error of a few ulp, repeated
// over the thousands of rotations a column of V goes through, shrinks the
// columns measurably; after the second step c is rounded to nearest, and
// c^2 + s^2 = 1 holds to rounding with no drift.
// For |tau| > 2^500 (1 + tau^2 would overflow) t = 1/(2 tau).
__device__ inline double rcp_nr(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    return r * fma(-x, r, 2.0);
}
__device__ inline double rsq_nr(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    return y * fma(-0.5 * x * y, y, 1.5);
}
__device__ inline double rsq_nr2(double x)
{
    const double y = rsq_nr(x);
    return y * fma(-0.5 * x * y, y, 1.5);
}
__device__ inline void jacobi_angle_fast(double app, double aqq, double apq, double &c,
                                         double &s, double &t)
{
    const double tau = (aqq - app) * rcp_nr(2.0 * apq);
    const double at = fabs(tau);
    double tt;
    if (at > 0x1p500) {
        tt = 0.5 * rcp_nr(at);
    } else {
        const double x = fma(at, at, 1.0);
        const double root = x * rsq_nr(x); // sqrt(1 + tau^2)
        tt = rcp_nr(at + root);
    }
    t = tau >= 0.0 ? tt : -tt;
    c = rsq_nr2(fma(t, t, 1.0));
    s = t * c;
}

// A value as the stage stores it: FP32 data of the binary16 stage (r16 set)
// are rounded to the nearest binary16 value (ties to even, the hardware
// conversion) and held widened in FP32; every other stage stores as is.
template <typename T>
__device__ inline T store_round(T x, int r16);
template <>
__device__ inline float store_round<float>(float x, int r16)
{
    return r16 ? (float)(_Float16)x : x;
}
template <>
__device__ inline double store_round<double>(double x, int)
{
    return x;
}

// Per-pair test: rotate only when a_pq is not negligible relative to the
// diagonal (the per-pair threshold of Algorithm 4 with tol = eps) and above
// the absolute floor thr = tol_off / n (if every |a_pq| <= tol_off / n then
// off(B) <= tol_off already).
__device__ inline bool jacobi_should_rotate(double app, double aqq, double apq,
                                            double eps, double thr)
{
    double a = fabs(apq);
    return apq != 0.0 && a > thr && a > eps * sqrt(fabs(app * aqq));
}

// The same test without the square root: a^2 > eps^2 |a_pp a_qq| (the
// operands are matrix entries of moderate size; a^2 underflows only below
// 1e-154, far under any threshold used here).
__device__ inline bool jacobi_should_rotate_sq(double app, double aqq, double apq, double eps,
                                               double thr)
{
    double a = fabs(apq);
    return apq != 0.0 && a > thr && a * a > eps * eps * fabs(app * aqq);
}

// Per-pair rotation flags of a round: the pair solve of pair p stores one int
// per wavefront at prot[p * PROT_STRIDE + wavefront], nonzero when that
// wavefront applied a rotation.  A pair solve that applied none leaves its
// tile and its U exactly as they were (U = I: every record then holds
// c = 1, s = 0, t = 0), so the updates of B and V may leave that pair out.
constexpr int PROT_STRIDE = 16;
template <int PW>
__device__ inline bool pair_rotated(const int *__restrict__ prot, int p)
{
    static_assert(PW % 4 == 0 && PW <= PROT_STRIDE, "flags per pair");
    const int4 *q = reinterpret_cast<const int4 *>(prot + (int64_t)p * PROT_STRIDE);
    int r = 0;
#pragma unroll
    for (int i = 0; i < PW / 4; ++i) {
        const int4 v = q[i];
        r |= v.x | v.y | v.z | v.w;
    }
    return r != 0;
}

// Workgroup barrier that orders LDS accesses only.  __syncthreads() also
// makes every wavefront wait for all of its outstanding global stores and
// loads; phases that share data only through LDS use this one, so stores and
// prefetches stay in flight across it.
__device__ inline void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

template <typename T>
__device__ inline T wave_sum(T v)
{
#pragma unroll
    for (int off = WAVE / 2; off > 0; off >>= 1)
        v += __shfl_xor(v, off, WAVE);
    return v;
}

// Block-wide sum; every thread gets the result.  `red` is LDS scratch of at
// least NT/WAVE entries.  Deterministic: fixed shuffle tree, then waves in
// order.
template <int NT>
__device__ inline double block_sum(double v, double *red)
{
    v = wave_sum(v);
    const int w = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
    __syncthreads();
    if (lane == 0)
        red[w] = v;
    __syncthreads();
    double tot = 0.0;
#pragma unroll
    for (int i = 0; i < NT / WAVE; ++i)
        tot += red[i];
    __syncthreads();
    return tot;
}

// Block-wide maximum; every thread gets the result (same LDS use as block_sum).
template <int NT>
__device__ inline double block_max(double v, double *red)
{
#pragma unroll
    for (int off = WAVE / 2; off > 0; off >>= 1)
        v = fmax(v, __shfl_xor(v, off, WAVE));
    const int w = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
    __syncthreads();
    if (lane == 0)
        red[w] = v;
    __syncthreads();
    double m = 0.0;
#pragma unroll
    for (int i = 0; i < NT / WAVE; ++i)
        m = fmax(m, red[i]);
    __syncthreads();
    return m;
}

// x 2^k, exact, in two steps so that the factor never overflows (|k| <= 2100)
__device__ inline double ldexp2(double x, int k) { return ldexp(ldexp(x, k / 2), k - k / 2); }

// Exponent of the exact scaling that brings a largest entry amax outside
// [2^-100, 2^100] into [1, 2) (0 when amax is inside, zero or not finite).
__host__ __device__ inline int scale_exp_of(double amax)
{
    if (!(amax > 0.0) || !(amax <= 0x1.fffffffffffffp1023) || (amax >= 0x1p-100 && amax <= 0x1p100))
        return 0;
    int e = 0;
    frexp(amax, &e);
    return 1 - e;
}

template <int NT>
__device__ inline int block_or(int v, int *red)
{
    v = __any(v) ? 1 : 0;
    const int w = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
    __syncthreads();
    if (lane == 0)
        red[w] = v;
    __syncthreads();
    int tot = 0;
#pragma unroll
    for (int i = 0; i < NT / WAVE; ++i)
        tot |= red[i];
    __syncthreads();
    return tot;
}

// ---------------------------------------------------------------- MFMA
// 16x16x4 MFMA on one wavefront: D(16x16) += A(16x4) * B(4x16).
// Operand layout (both precisions): lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16].  Accumulator element v (v = 0..3) of lane l holds
// D[r][l % 16] with r = acc_row<T>(l / 16, v):
//   f32 (v_mfma_f32_16x16x4f32): r = 4 (l / 16) + v
//   f64 (v_mfma_f64_16x16x4f64): r = l / 16 + 4 v
// (the f64 mapping was measured on gfx950 with a one-wave probe).
typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

__device__ inline d4 mfma16(double a, double b, d4 c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__device__ inline f4 mfma16(float a, float b, f4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <typename T>
__device__ inline int acc_row(int lk, int v);
template <>
__device__ inline int acc_row<float>(int lk, int v)
{
    return 4 * lk + v;
}
template <>
__device__ inline int acc_row<double>(int lk, int v)
{
    return lk + 4 * v;
}

template <typename T>
struct acc4;
template <>
struct acc4<double> {
    typedef d4 type;
};
template <>
struct acc4<float> {
    typedef f4 type;
};

} // namespace lj
