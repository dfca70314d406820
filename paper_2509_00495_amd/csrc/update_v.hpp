// V update of the block path (the round's block rotation, Section 3.3 applied
// blockwise): V[:, cols(P, Q)] <- V[:, cols(P, Q)] U_PQ for every block pair
// (P, Q) of a round.  The per-wavefront body is shared by the standalone
// update kernel and by the launch that runs it beside the next round's pair
// solves.
//
// Each wavefront owns one pair l and a contiguous run of 16-row tiles of V.
// It computes Z^T = U_l^T X^T on the 16x16x4 MFMA with no LDS and no barrier:
//   * the B operand is X^T, so lane (li, lk) needs X[row li][k] for the k of
//     its MFMA step.  The k order inside a step is free, so step (g, j) gives
//     lane lk the k = g*4*VK + lk*VK + j: one 16-byte load of VK consecutive
//     columns of row li feeds VK steps;
//   * the A operand, U_l^T, is loaded once per wavefront into registers (the
//     U blocks are stored transposed, so these are 16-byte loads);
//   * the accumulator of a 16-column tile holds, per lane, the four entries
//     D[r][li] with r = acc_row(lk, v).  Column 16 tc + m of the MFMA output
//     is mapped to output column 16 tc + out_perm(m), chosen so that the four
//     values of a lane are four consecutive columns of row li: one 16-byte
//     store (f32) or two (f64).
// The next tile's X is in flight while the current one computes (two register
// buffers).  Tiles of different wavefronts are disjoint, so the update is in
// place.
#pragma once
#include "common.hpp"
#include "internal.hpp"

namespace lj {
namespace vupd {

// 16-byte vectors as plain clang vector types (they stay in registers)
typedef float fv4 __attribute__((ext_vector_type(4)));
typedef double dv2 __attribute__((ext_vector_type(2)));
template <typename T>
struct V16;
template <>
struct V16<float> {
    typedef fv4 type;
};
template <>
struct V16<double> {
    typedef dv2 type;
};

// MFMA output row m of a 16-column tile -> column offset inside the tile
template <typename T>
__device__ inline int out_perm(int m);
template <>
__device__ inline int out_perm<float>(int m)
{
    return m; // acc row 4 lk + v is already column-contiguous per lane
}
template <>
__device__ inline int out_perm<double>(int m)
{
    return 4 * (m & 3) + (m >> 2); // acc row lk + 4 v -> column 4 lk + v
}

// column c (0 <= c < 2b) of the pair's slice -> global column
__device__ inline int pair_col(int2 pq, int c, int b)
{
    return c < b ? pq.x * b + c : pq.y * b + (c - b);
}

template <typename T>
__device__ inline T vlane(const typename V16<T>::type &x, int j)
{
    return x[j];
}

// Wavefront gw of the update: pair l = gw % npairs, chunk gw / npairs of the
// ntile 16-row tiles (chunks per pair).  Wavefronts past the work return, and
// so do those of a pair whose rotation flags (prot, when given) are all zero.
template <typename T, int M>
__device__ inline void v_update_wave(T *__restrict__ V, int64_t ldv, int64_t ntile,
                                     const int2 *__restrict__ pairs, int npairs,
                                     const T *__restrict__ U, const int *__restrict__ prot,
                                     int chunks, int gw)
{
    constexpr int b = M / 2;
    constexpr int VK = 16 / (int)sizeof(T); // elements per 16-byte vector
    constexpr int TC = M / 16;              // 16-column output tiles
    constexpr int KG = M / (4 * VK);        // vectors per lane per tile row
    typedef typename V16<T>::type TV;
    typedef typename acc4<T>::type accT;
    const int lane = threadIdx.x % WAVE, li = lane % 16, lk = lane / 16;
    const int l = gw % npairs, ch = gw / npairs;
    if (ch >= chunks)
        return;
    if (prot && !pair_rotated<pair_solve_waves(M)>(prot, l))
        return; // U_l = I
    const int64_t t0 = (int64_t)ch * ntile / chunks, t1 = (int64_t)(ch + 1) * ntile / chunks;
    if (t0 >= t1)
        return;
    const int2 pl = pairs[l];
    // U blocks are stored transposed (Ut[j][i] = U[i][j]): the VK fragments of
    // a step group are consecutive, one 16-byte load
    const T *Ult = U + (int64_t)l * M * M;
    T uf[TC][KG][VK];
#pragma unroll
    for (int tc = 0; tc < TC; ++tc)
#pragma unroll
        for (int g = 0; g < KG; ++g) {
            const TV u = *reinterpret_cast<const TV *>(Ult + (16 * tc + out_perm<T>(li)) * M +
                                                       g * 4 * VK + lk * VK);
#pragma unroll
            for (int j = 0; j < VK; ++j)
                uf[tc][g][j] = vlane<T>(u, j);
        }
    int kc[KG], oc[TC];
#pragma unroll
    for (int g = 0; g < KG; ++g)
        kc[g] = pair_col(pl, g * 4 * VK + lk * VK, b);
#pragma unroll
    for (int tc = 0; tc < TC; ++tc)
        oc[tc] = pair_col(pl, 16 * tc + 4 * lk, b);

    auto load = [&](TV(&x)[KG], int64_t t) __attribute__((always_inline)) {
        const T *row = V + (t * 16 + li) * ldv;
#pragma unroll
        for (int g = 0; g < KG; ++g)
            x[g] = *reinterpret_cast<const TV *>(row + kc[g]);
    };
    auto work = [&](const TV(&x)[KG], int64_t t) __attribute__((always_inline)) {
        accT acc[TC];
#pragma unroll
        for (int tc = 0; tc < TC; ++tc)
#pragma unroll
            for (int v = 0; v < 4; ++v)
                acc[tc][v] = (T)0;
#pragma unroll
        for (int g = 0; g < KG; ++g)
#pragma unroll
            for (int j = 0; j < VK; ++j) {
                const T bv = vlane<T>(x[g], j);
#pragma unroll
                for (int tc = 0; tc < TC; ++tc)
                    acc[tc] = mfma16(uf[tc][g][j], bv, acc[tc]);
            }
        T *row = V + (t * 16 + li) * ldv;
#pragma unroll
        for (int tc = 0; tc < TC; ++tc) {
            if constexpr (sizeof(T) == 4) {
                const fv4 z = {acc[tc][0], acc[tc][1], acc[tc][2], acc[tc][3]};
                *reinterpret_cast<fv4 *>(row + oc[tc]) = z;
            } else {
                const dv2 z0 = {acc[tc][0], acc[tc][1]}, z1 = {acc[tc][2], acc[tc][3]};
                *reinterpret_cast<dv2 *>(row + oc[tc]) = z0;
                *reinterpret_cast<dv2 *>(row + oc[tc] + 2) = z1;
            }
        }
    };

    // Every path into the loop issues the same sequence of memory operations
    // (prefetch indices are clamped to the last tile instead of skipped, the
    // first step is peeled), so the wait for a buffer's loads never has to
    // wait for the stores issued after them.
    TV xa[KG], xb[KG];
    auto step = [&](TV(&x)[KG], int64_t t) __attribute__((always_inline)) {
        work(x, t);
        load(x, t + 2 < t1 ? t + 2 : t1 - 1);
        // keep the two buffers' steps apart, or the scheduler merges them and
        // the second buffer's loads are waited for right after being issued
        __builtin_amdgcn_sched_barrier(0);
    };
    load(xa, t0);
    load(xb, t0 + 1 < t1 ? t0 + 1 : t1 - 1);
    step(xa, t0);
    int64_t t = t0 + 1;
    for (; t + 1 < t1; t += 2) {
        step(xb, t);
        step(xa, t + 1);
    }
    if (t < t1)
        work(xb, t);
}

// Workgroup variant for the launch shared with the pair solves: the 16-row
// tiles [t0, t1) of pair l's columns.  U_l^T is staged once into LDS (ufl,
// M*M entries) in per-lane fragment order, and every wavefront reads it from
// there with 16-byte LDS loads at consecutive addresses; the first nw
// wavefronts take the range's tiles in turn (tile t0 + w + i nw), each with
// two X buffers in flight as above.  Every thread reaches the barrier, or
// none does: a pair whose rotation flags (prot, when given) are all zero
// returns before it.
template <typename T, int M, int NT>
__device__ inline void v_update_wg(T *__restrict__ V, int64_t ldv,
                                   const int2 *__restrict__ pairs, int l,
                                   const T *__restrict__ U, const int *__restrict__ prot,
                                   int64_t t0, int64_t t1, int nw, T *ufl)
{
    constexpr int b = M / 2;
    constexpr int VK = 16 / (int)sizeof(T);
    constexpr int TC = M / 16;
    constexpr int KG = M / (4 * VK);
    typedef typename V16<T>::type TV;
    typedef typename acc4<T>::type accT;
    const int tid = threadIdx.x, lane = tid % WAVE, w = tid / WAVE;
    const int li = lane % 16, lk = lane / 16;
    // the flags are read while U_l is staged (the V workgroups of the shared
    // pair-solve launch are on its critical path in FP32)
    const bool rotated = !prot || pair_rotated<pair_solve_waves(M)>(prot, l);
    const int2 pl = pairs[l];
    const T *Ult = U + (int64_t)l * M * M; // transposed: Ult[j][i] = U_l[i][j]
    for (int e = tid; e < TC * KG * WAVE; e += NT) {
        const int ln = e % WAVE, f = e / WAVE, tc = f / KG, g = f % KG;
        *reinterpret_cast<TV *>(ufl + e * VK) = *reinterpret_cast<const TV *>(
            Ult + (16 * tc + out_perm<T>(ln % 16)) * M + g * 4 * VK + (ln / 16) * VK);
    }
    if (!rotated)
        return; // U_l = I (the decision is the same for the whole workgroup)
    __syncthreads();
    const int64_t cnt = w < nw && t1 - t0 > w ? (t1 - t0 - w + nw - 1) / nw : 0;
    if (cnt == 0)
        return;
    int kc[KG], oc[TC];
#pragma unroll
    for (int g = 0; g < KG; ++g)
        kc[g] = pair_col(pl, g * 4 * VK + lk * VK, b);
#pragma unroll
    for (int tc = 0; tc < TC; ++tc)
        oc[tc] = pair_col(pl, 16 * tc + 4 * lk, b);
    auto tile = [&](int64_t i) { return t0 + w + i * nw; };
    auto load = [&](TV(&x)[KG], int64_t i) __attribute__((always_inline)) {
        const T *row = V + (tile(i) * 16 + li) * ldv;
#pragma unroll
        for (int g = 0; g < KG; ++g)
            x[g] = *reinterpret_cast<const TV *>(row + kc[g]);
    };
    auto work = [&](const TV(&x)[KG], int64_t i) __attribute__((always_inline)) {
        accT acc[TC];
#pragma unroll
        for (int tc = 0; tc < TC; ++tc)
#pragma unroll
            for (int v = 0; v < 4; ++v)
                acc[tc][v] = (T)0;
#pragma unroll
        for (int g = 0; g < KG; ++g)
#pragma unroll
            for (int tc = 0; tc < TC; ++tc) {
                const TV u = *reinterpret_cast<const TV *>(ufl + ((tc * KG + g) * WAVE + lane) * VK);
#pragma unroll
                for (int j = 0; j < VK; ++j)
                    acc[tc] = mfma16(vlane<T>(u, j), vlane<T>(x[g], j), acc[tc]);
            }
        T *row = V + (tile(i) * 16 + li) * ldv;
#pragma unroll
        for (int tc = 0; tc < TC; ++tc) {
            if constexpr (sizeof(T) == 4) {
                const fv4 z = {acc[tc][0], acc[tc][1], acc[tc][2], acc[tc][3]};
                *reinterpret_cast<fv4 *>(row + oc[tc]) = z;
            } else {
                const dv2 z0 = {acc[tc][0], acc[tc][1]}, z1 = {acc[tc][2], acc[tc][3]};
                *reinterpret_cast<dv2 *>(row + oc[tc]) = z0;
                *reinterpret_cast<dv2 *>(row + oc[tc] + 2) = z1;
            }
        }
    };
    TV xa[KG], xb[KG];
    auto step = [&](TV(&x)[KG], int64_t i) __attribute__((always_inline)) {
        work(x, i);
        load(x, i + 2 < cnt ? i + 2 : cnt - 1);
        __builtin_amdgcn_sched_barrier(0);
    };
    load(xa, 0);
    load(xb, 1 < cnt ? 1 : cnt - 1);
    step(xa, 0);
    int64_t i = 1;
    for (; i + 1 < cnt; i += 2) {
        step(xb, i);
        step(xa, i + 1);
    }
    if (i < cnt)
        work(xb, i);
}

} // namespace vupd
} // namespace lj
