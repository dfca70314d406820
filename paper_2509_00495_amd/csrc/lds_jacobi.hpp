// One parallel Jacobi round on a symmetric matrix held in LDS.
//
// Used by the one-workgroup solver (the whole matrix lives in LDS).
#pragma once

#include "common.hpp"

namespace lj {

// Player of slot `slot` in round r of the circle schedule on m players, for
// 0 <= r < m - 1 (one conditional subtraction instead of a remainder).
__device__ inline int rr_player_r(int slot, int r, int m)
{
    int v = slot - 1 + r;
    v = v >= m - 1 ? v - (m - 1) : v;
    return slot == 0 ? 0 : 1 + v;
}

__device__ inline void rr_pair_r(int k, int r, int m, int &p, int &q)
{
    const int a = rr_player_r(k, r, m), b = rr_player_r(m - 1 - k, r, m);
    p = a < b ? a : b;
    q = a < b ? b : a;
}

// Per-thread work lists of lds_jacobi_round for one matrix (they do not
// depend on the round): the 2x2 blocks (k <= l) a thread updates, packed as
// k << 16 | l (-1 = none), and its items of the V update: item e = tid +
// j NT is (pair k, two-entry chunk c) with e = k nch + c, nch = ceil(nv / 2)
// chunks per row of V^T; the first item and the stride in (k, c).
template <int NT, int SI>
struct RoundItems {
    int kl[SI];
    int tk0, tc0, dk, dch, nch;
    __device__ void init(int m, int nv)
    {
        const int h = m / 2, nblk = (h / 2) * (h + 1);
#pragma unroll
        for (int u = 0; u < SI; ++u) {
            const int idx = threadIdx.x + u * NT;
            kl[u] = -1;
            if (idx < nblk) {
                int k, l;
                tri_fold(idx, h, k, l);
                kl[u] = (k << 16) | l;
            }
        }
        nch = (nv + 1) / 2;
        tk0 = threadIdx.x / nch;
        tc0 = threadIdx.x % nch;
        dk = NT / nch;
        dch = NT % nch;
    }
};

// entry (i, j) of a symmetric matrix kept as its upper triangle, row stride ld
__device__ __forceinline__ int sym_idx(int i, int j, int ld)
{
    return i <= j ? i * ld + j : j * ld + i;
}

// S: m x m symmetric, row stride ld (LDS), m a multiple of 4; after the first
// round only its upper triangle (i <= j) is kept current.
// cs: LDS scratch of 3 * m/2 doubles, 16-byte aligned: (c, s) of pair k at
//    2k, 2k + 1 (one 16-byte read), t at m + k.
// Vt: V transposed, m rows of stride ldt (even, >= nv; LDS or global, 16-byte
//    aligned rows), updated as Vt([p q], :) <- J^T Vt([p q], :), i.e.
//    V(:, [p q]) <- V(:, [p q]) J; may be null.  A pair's two rows are
//    contiguous, so the update reads and writes them two entries at a time.
// In round r the m/2 disjoint pairs (p, q) of the round-robin schedule are
// rotated simultaneously: angles first (phase 1), then the two-sided update
// B <- J^T B J restricted to the 2x2 blocks [p_k q_k] x [p_l q_l] (phase 2),
// which touches every entry once.  Only blocks with k <= l are computed, on
// the upper triangle (the mirror would be a copy of the same values).  The
// rotated pair itself gets the closed-form diagonal (a_pp - t a_pq,
// a_qq + t a_pq) and an exact zero off the diagonal.
// The index work of a thread comes from its lists `it` (built once per
// matrix) and the angles from jacobi_angle_fast.
// Phase 1 of round r: the angles of the round's m/2 pairs into cs (pair k on
// thread k mod NT).  Returns (per thread) whether it computed a rotation.
template <typename T, int NT>
__device__ inline int lds_round_angles(const T *S, int ld, int m, int r, double eps, double thr,
                                       double *cs)
{
    const int h = m / 2;
    const int tid = threadIdx.x;
    int rotated = 0;
    for (int k = tid; k < h; k += NT) {
        int p, q;
        rr_pair_r(k, r, m, p, q);
        const double app = (double)S[p * ld + p];
        const double aqq = (double)S[q * ld + q];
        const double apq = (double)S[p * ld + q];
        double c = 1.0, s = 0.0, t = 0.0;
        if (jacobi_should_rotate_sq(app, aqq, apq, eps, thr)) {
            jacobi_angle_fast(app, aqq, apq, c, s, t);
            rotated = 1;
        }
        typedef double d2 __attribute__((ext_vector_type(2)));
        d2 cv;
        cv.x = c;
        cv.y = s;
        reinterpret_cast<d2 *>(cs)[k] = cv;
        cs[2 * h + k] = t;
    }
    return rotated;
}

// Phase 2 of round r on S with the round's angles in cs.
template <typename T, int NT, int SI>
__device__ inline void lds_round_update_s(T *S, int ld, int m, int r, const double *cs,
                                          const RoundItems<NT, SI> &it)
{
    const int h = m / 2;
#pragma unroll
    for (int u = 0; u < SI; ++u) {
        if (it.kl[u] < 0)
            continue;
        const int k = it.kl[u] >> 16, l = it.kl[u] & 0xffff;
        typedef double d2 __attribute__((ext_vector_type(2)));
        const d2 csk = reinterpret_cast<const d2 *>(cs)[k], csl = reinterpret_cast<const d2 *>(cs)[l];
        const double sk = csk.y, sl = csl.y;
        if (sk == 0.0 && sl == 0.0)
            continue;
        int pk, qk, pl, ql;
        rr_pair_r(k, r, m, pk, qk);
        rr_pair_r(l, r, m, pl, ql);
        if (k == l) {
            const double tk = cs[2 * h + k];
            const double apq = (double)S[pk * ld + qk];
            const double app = (double)S[pk * ld + pk];
            const double aqq = (double)S[qk * ld + qk];
            S[pk * ld + pk] = (T)(app - tk * apq);
            S[qk * ld + qk] = (T)(aqq + tk * apq);
            S[pk * ld + qk] = (T)0;
            continue;
        }
        const T ck = (T)csk.x, skT = (T)sk, cl = (T)csl.x, slT = (T)sl;
        const int a00 = sym_idx(pk, pl, ld), a01 = sym_idx(pk, ql, ld);
        const int a10 = sym_idx(qk, pl, ld), a11 = sym_idx(qk, ql, ld);
        const T x00 = S[a00], x01 = S[a01];
        const T x10 = S[a10], x11 = S[a11];
        const T y00 = ck * x00 - skT * x10, y01 = ck * x01 - skT * x11;
        const T y10 = skT * x00 + ck * x10, y11 = skT * x01 + ck * x11;
        const T z00 = cl * y00 - slT * y01, z01 = slT * y00 + cl * y01;
        const T z10 = cl * y10 - slT * y11, z11 = slT * y10 + cl * y11;
        S[a00] = z00;
        S[a01] = z01;
        S[a10] = z10;
        S[a11] = z11;
    }
}

// The V update of round r with the round's angles in cs.
template <typename T, int NT, int SI>
__device__ inline void lds_round_update_v(T *Vt, int ldt, int m, int r, const double *cs,
                                          const RoundItems<NT, SI> &it)
{
    const int h = m / 2;
    if (Vt) {
        // items in groups of VB, all loads of a group before its stores
        constexpr int VB = 2;
        typedef T t2 __attribute__((ext_vector_type(2)));
        int k = it.tk0, c = it.tc0;
        while (k < h) {
            int ks[VB], pp[VB], qq[VB], cc[VB];
            t2 a[VB], b[VB];
#pragma unroll
            for (int u = 0; u < VB; ++u) {
                ks[u] = -1;
                if (k < h) {
                    if (cs[2 * k + 1] != 0.0) {
                        ks[u] = k;
                        cc[u] = c;
                        rr_pair_r(k, r, m, pp[u], qq[u]);
                        a[u] = *reinterpret_cast<const t2 *>(Vt + (int64_t)pp[u] * ldt + 2 * c);
                        b[u] = *reinterpret_cast<const t2 *>(Vt + (int64_t)qq[u] * ldt + 2 * c);
                    }
                    c += it.dch;
                    k += it.dk;
                    if (c >= it.nch) {
                        c -= it.nch;
                        ++k;
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < VB; ++u) {
                if (ks[u] >= 0) {
                    typedef double d2 __attribute__((ext_vector_type(2)));
                    const d2 csu = reinterpret_cast<const d2 *>(cs)[ks[u]];
                    const T cv = (T)csu.x, sv = (T)csu.y;
                    t2 x, y;
                    x.x = cv * a[u].x - sv * b[u].x;
                    x.y = cv * a[u].y - sv * b[u].y;
                    y.x = sv * a[u].x + cv * b[u].x;
                    y.y = sv * a[u].y + cv * b[u].y;
                    *reinterpret_cast<t2 *>(Vt + (int64_t)pp[u] * ldt + 2 * cc[u]) = x;
                    *reinterpret_cast<t2 *>(Vt + (int64_t)qq[u] * ldt + 2 * cc[u]) = y;
                }
            }
        }
    }
}

// One whole round: angles, barrier, S and V updates, barrier.  Returns (per
// thread) whether this thread computed a rotation in phase 1.
template <typename T, int NT, int SI>
__device__ inline int lds_jacobi_round(T *S, int ld, int m, int r, double eps, double thr,
                                       T *Vt, int ldt, double *cs,
                                       const RoundItems<NT, SI> &it)
{
    const int rotated = lds_round_angles<T, NT>(S, ld, m, r, eps, thr, cs);
    __syncthreads();
    lds_round_update_s<T, NT, SI>(S, ld, m, r, cs, it);
    lds_round_update_v<T, NT, SI>(Vt, ldt, m, r, cs, it);
    __syncthreads();
    return rotated;
}

// off(S)^2 = sum of squares of the off-diagonal entries (the definition in
// Section 3.1), accumulated in FP64 directly (never as ||S||_F^2 - sum a_ii^2,
// which cancels catastrophically once S is nearly diagonal).
template <typename T, int NT>
__device__ inline double lds_off2(const T *S, int ld, int m, double *red)
{
    double acc = 0.0;
    for (int idx = threadIdx.x; idx < m * m; idx += NT) {
        int i = idx / m, j = idx - (idx / m) * m;
        if (i != j) {
            double v = (double)S[sym_idx(i, j, ld)];
            acc += v * v;
        }
    }
    return block_sum<NT>(acc, red);
}

} // namespace lj
