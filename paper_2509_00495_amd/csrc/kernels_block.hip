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
//      row tile of V becomes V_rows,l U_l (one MFMA GEMM); the update kernels
//      are in kernels_update.hip.
// Entries of B coupling a padding index are zero and stay exactly zero, so
// padding never mixes with the matrix.
#include "internal.hpp"

#include <algorithm>
#include "update_v.hpp"

namespace lj {

__host__ __device__ inline size_t align8(size_t x) { return (x + 7) & ~(size_t)7; }

// ------------------------------------------------------------- pair solve
// Rotated diagonal entry of a pair after its rotation: a_pp - t a_pq for the
// first position of the pair, a_qq + t a_pq for the second (Section 3.1),
// formed in FP64 and rounded to the stage's precision.
template <typename T>
__device__ inline T rotated_diag(T a, double t, T apq, int second)
{
    double v = second ? (double)a + t * (double)apq : (double)a - t * (double)apq;
    return (T)v;
}

// Player of slot s in round r of the circle schedule on M players; the next
// round moves every player of slot s >= 1 on by one (M-1 wraps to 1).
__device__ inline int rr_next(int player, int M) { return player == 0 ? 0 : (player == M - 1 ? 1 : player + 1); }

template <typename T>
struct vec2;
template <>
struct vec2<float> {
    typedef float2 type;
};
template <>
struct vec2<double> {
    typedef double2 type;
};

// 16-byte vector of T (4 floats or 2 doubles)
template <typename T>
struct vec16;
template <>
struct vec16<float> {
    typedef float4 type;
    static constexpr int n = 4;
};
template <>
struct vec16<double> {
    typedef double2 type;
    static constexpr int n = 2;
};

// Per-pair record of a round in LDS: the rotation (c, s) packed for one
// vector read, t, and the 2x2 problem it was computed from.
template <typename T>
struct PairRec {
    typedef typename vec2<T>::type T2;
    T2 *cs;
    double *t;
    T *app, *aqq, *apq;
    __device__ PairRec(unsigned char *base, int h)
    {
        t = (double *)base;
        cs = (T2 *)(t + h);
        app = (T *)(cs + h);
        aqq = app + h;
        apq = aqq + h;
    }
    static constexpr size_t bytes(int h) { return ((size_t)h * (8 + 5 * sizeof(T)) + 15) & ~(size_t)15; }
};

template <typename T>
__device__ inline int pair_record(PairRec<T> &R, int k, T app, T aqq, T apq, double eps,
                                  double thr)
{
    // the angle in FP64 in both stages (FP32 data are widened)
    double c = 1.0, sn = 0.0, t = 0.0;
    int rot = 0;
    if (jacobi_should_rotate_sq((double)app, (double)aqq, (double)apq, eps, thr)) {
        jacobi_angle_fast((double)app, (double)aqq, (double)apq, c, sn, t);
        rot = 1;
    }
    typename PairRec<T>::T2 v;
    v.x = (T)c;
    v.y = (T)sn;
    R.cs[k] = v;
    R.t[k] = t;
    R.app[k] = app;
    R.aqq[k] = aqq;
    R.apq[k] = apq;
    return rot;
}

// One workgroup per block pair (P, Q) of the round.  The 2b x 2b tile S (upper
// triangle only, logical order) and its accumulated rotation U (stored
// transposed, Ut[j][i] = U[i][j], so a column pair of U is two LDS rows that
// are read and written 16 bytes at a time) are updated in place.  U leaves
// the kernel transposed as well: U_out[pair][j][i] = U[i][j].  In inner
// round r the M/2 disjoint pairs are those of the circle schedule on M = 2b
// indices, (player(slot k), player(slot M-1-k)); every thread carries the
// current players of the pairs it works on from round to round.  A thread
// owns a fixed 2x2 block (k <= l) of S, or fixed (pair, 16-byte chunk) items
// of U.  The next round's angles are computed in the same phase: each next
// pair joins one index of current pair k with one of pair l != k, so the
// owner of block (k, l) has the new coupling and recomputes the two new
// diagonal entries from the pair records (never from S, which the diagonal
// owners overwrite in the same phase).  One barrier per round, and about
// 2 + 1/8 wavefront-level LDS instructions per element of S and U.
//
// CROSS selects the cross schedule instead: only pairs (i, j) with i in P and
// j in Q are rotated, in b rounds; round r pairs position i with b + (i + r)
// mod b.  A sweep that runs the circle schedule in its first round (every
// block appears once there, so every pair inside a block is rotated) and the
// cross schedule in the others rotates every index pair of the matrix exactly
// once, as a cyclic sweep of Algorithm 4 does, in about n instead of 2n
// rounds.  The next pair i joins position i of pair i with the second position
// of pair i + 1 (mod b), so block (i, i + 1), or (0, b - 1) for i = b - 1,
// hosts it.
template <typename T, int M, int NT, bool CROSS>
__device__ __forceinline__ void pair_solve_body(T *__restrict__ B, int64_t ldb,
                                       const int2 *__restrict__ pairs,
                                       const int2 *__restrict__ psmap, T *__restrict__ U,
                                       double eps, double thr, int inner, int r16,
                                       double *__restrict__ partial, int *rot_flag,
                                       int *__restrict__ prot, int pk)
{
    constexpr int b = M / 2, h = M / 2, ld = M + 1;
    typedef typename vec16<T>::type TV;
    constexpr int VN = vec16<T>::n;
    constexpr int ldu = M + VN;             // 16-byte aligned rows of Ut
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *Ut = (T *)smem_raw;                  // M x ldu
    T *S = Ut + M * ldu;                    // M x ld, entries i <= j
    // a constant offset keeps the records in the LDS address space (an
    // integer round trip of the pointer would turn every access into a flat one)
    constexpr size_t REC_OFF = (sizeof(T) * (M * ldu + M * ld) + 15) & ~(size_t)15;
    unsigned char *recbase = smem_raw + REC_OFF;
    constexpr size_t RB = PairRec<T>::bytes(h);
    const int tid = threadIdx.x;
    const int2 pq = pairs[pk];
    auto sidx = [](int i, int j) { return i <= j ? i * ld + j : j * ld + i; };
    // B holds only its upper b x b blocks (block row <= block column) during
    // the sweeps.  The tile is read as three stored blocks: P's and Q's
    // diagonal blocks and the off-diagonal block in its stored orientation
    // (rows of min(P, Q), columns of max(P, Q)), each in 16-byte row pieces,
    // all loads issued before the LDS writes.  S gets the diagonal blocks as
    // full rows (only their upper triangles are read) and the off-diagonal
    // block at logical (i < b, j >= b), transposed when P > Q.
    constexpr int RV = M / VN;            // 16-byte vectors per row of Ut
    constexpr int BV = b / VN;            // 16-byte vectors per block row
    constexpr int VPB = b * BV;           // vectors per b x b block
    constexpr int PV = (3 * VPB + NT - 1) / NT;
    const bool swapo = pq.x > pq.y;       // off-diagonal block stored as (Q, P)
    const int64_t orow = (int64_t)(swapo ? pq.y : pq.x) * b, ocol = (int64_t)(swapo ? pq.x : pq.y) * b;
    // global (row, column) of vector v of stored block s (0: P P, 1: Q Q, 2: off)
    auto blk_row = [&](int s, int a) {
        return s == 0 ? (int64_t)pq.x * b + a : (s == 1 ? (int64_t)pq.y * b + a : orow + a);
    };
    auto blk_col = [&](int s, int c) {
        return s == 0 ? (int64_t)pq.x * b + c : (s == 1 ? (int64_t)pq.y * b + c : ocol + c);
    };
    TV xin[PV];
#pragma unroll
    for (int e = 0; e < PV; ++e) {
        const int v = tid + e * NT;
        if (v < 3 * VPB) {
            const int s = v / VPB, a = (v % VPB) / BV, c = (v % BV) * VN;
            xin[e] = *reinterpret_cast<const TV *>(B + blk_row(s, a) * ldb + blk_col(s, c));
        }
    }
#pragma unroll
    for (int e = 0; e < PV; ++e) {
        const int v = tid + e * NT;
        if (v < 3 * VPB) {
            const int s = v / VPB, a = (v % VPB) / BV, c = (v % BV) * VN;
            const T *xe = reinterpret_cast<const T *>(&xin[e]);
#pragma unroll
            for (int q = 0; q < VN; ++q) {
                if (s == 0)
                    S[a * ld + c + q] = xe[q];
                else if (s == 1)
                    S[(b + a) * ld + b + c + q] = xe[q];
                else if (!swapo)
                    S[a * ld + b + c + q] = xe[q];
                else
                    S[(c + q) * ld + b + a] = xe[q];
            }
        }
    }
    for (int v = tid; v < M * RV; v += NT) {
        const int i = v / RV, j = (v % RV) * VN;
        TV id;
        T *ie = reinterpret_cast<T *>(&id);
#pragma unroll
        for (int q = 0; q < VN; ++q)
            ie[q] = (T)(i == j + q ? 1 : 0);
        *reinterpret_cast<TV *>(Ut + i * ldu + j) = id;
    }
    constexpr int NBLK = h * (h + 1) / 2;
    int bk = -1, bl = -1;
    if (tid < NBLK) {
        const int2 e = psmap[tid];
        bk = e.x;
        bl = e.y;
    }
    // second position of a pair in the next round of the cross schedule
    auto cnext = [](int q) { return q == M - 1 ? b : q + 1; };
    int pk0 = bk, pk1 = CROSS ? b + bk : M - 1 - bk, pl0 = bl, pl1 = CROSS ? b + bl : M - 1 - bl;
    int hosted = 0, ha = 0, hc = 0, hk = 0, hfirst = 0;
    if (CROSS) {
        if (bk >= 0 && bl == bk + 1) {
            hosted = 1;
            hk = bk;
            hfirst = 1;
            hc = 1;
        } else if (bk == 0 && bl == b - 1) {
            hosted = 1;
            hk = b - 1;
            ha = 1;
        }
    } else if (bk >= 0 && bk != bl) {
        for (int a = 0; a < 2; ++a)
            for (int c = 0; c < 2; ++c) {
                const int sa = a ? M - 1 - bk : bk, sc = c ? M - 1 - bl : bl;
                const int na = sa == 0 ? 0 : (sa == 1 ? M - 1 : sa - 1);
                const int nc = sc == 0 ? 0 : (sc == 1 ? M - 1 : sc - 1);
                const int ka = na < h ? na : M - 1 - na, kc = nc < h ? nc : M - 1 - nc;
                if (ka == kc) {
                    hosted = 1;
                    ha = a;
                    hc = c;
                    hk = ka;
                    hfirst = na < h;
                }
            }
    }
    // U items: (pair k, chunk of VN rows), on the wavefronts after the first
    constexpr int CH = M / VN;
    constexpr int NU = h * CH;
    constexpr int UW = NT - WAVE;
    constexpr int NIT = (NU + UW - 1) / UW;
    int up0[NIT], up1[NIT];
#pragma unroll
    for (int j = 0; j < NIT; ++j) {
        const int it = tid - WAVE + j * UW;
        const int k = (tid >= WAVE && it < NU) ? it / CH : 0;
        up0[j] = k;
        up1[j] = CROSS ? b + k : M - 1 - k;
    }
    __syncthreads();
    int rot = 0;
    if (tid < h) {
        PairRec<T> R0(recbase, h);
        const int q = CROSS ? b + tid : M - 1 - tid;
        rot |= pair_record<T>(R0, tid, S[tid * ld + tid], S[q * ld + q], S[tid * ld + q], eps,
                              thr);
    }
    __syncthreads();
    const int rounds = inner * (CROSS ? b : M - 1);
    for (int r = 0; r < rounds; ++r) {
        const PairRec<T> A(recbase + (r & 1) * RB, h);
        PairRec<T> Bn(recbase + ((r + 1) & 1) * RB, h);
        if (bk >= 0) {
            const int k = bk, l = bl;
            if (k == l) {
                const double tk = A.t[k];
                const T apq = A.apq[k];
                S[pk0 * ld + pk0] = store_round<T>(rotated_diag<T>(A.app[k], tk, apq, 0), r16);
                S[pk1 * ld + pk1] = store_round<T>(rotated_diag<T>(A.aqq[k], tk, apq, 1), r16);
                S[sidx(pk0, pk1)] = A.cs[k].y == (T)0 ? apq : (T)0;
            } else {
                const typename PairRec<T>::T2 csk = A.cs[k], csl = A.cs[l];
                const T ck = csk.x, sk = csk.y, cl = csl.x, sl = csl.y;
                const int a00 = sidx(pk0, pl0), a01 = sidx(pk0, pl1);
                const int a10 = sidx(pk1, pl0), a11 = sidx(pk1, pl1);
                const T x00 = S[a00], x01 = S[a01], x10 = S[a10], x11 = S[a11];
                // the host of the next round's angle reads its records before
                // any LDS store of this round (a load after a store would wait
                // for it) and computes the angle before storing its block:
                // this chain is the longest of the round
                T dpe = (T)0, dqe = (T)0;
                if (hosted) {
                    dpe = store_round<T>(ha ? rotated_diag<T>(A.aqq[k], A.t[k], A.apq[k], 1)
                                            : rotated_diag<T>(A.app[k], A.t[k], A.apq[k], 0),
                                         r16);
                    dqe = store_round<T>(hc ? rotated_diag<T>(A.aqq[l], A.t[l], A.apq[l], 1)
                                            : rotated_diag<T>(A.app[l], A.t[l], A.apq[l], 0),
                                         r16);
                }
                const T y00 = ck * x00 - sk * x10, y01 = ck * x01 - sk * x11;
                const T y10 = sk * x00 + ck * x10, y11 = sk * x01 + ck * x11;
                const T z00 = store_round<T>(cl * y00 - sl * y01, r16);
                const T z01 = store_round<T>(sl * y00 + cl * y01, r16);
                const T z10 = store_round<T>(cl * y10 - sl * y11, r16);
                const T z11 = store_round<T>(sl * y10 + cl * y11, r16);
                if (hosted) {
                    const T zz = ha ? (hc ? z11 : z10) : (hc ? z01 : z00);
                    const int rr = pair_record<T>(Bn, hk, hfirst ? dpe : dqe,
                                                  hfirst ? dqe : dpe, zz, eps, thr);
                    if (r + 1 < rounds)
                        rot |= rr;
                }
                S[a00] = z00;
                S[a01] = z01;
                S[a10] = z10;
                S[a11] = z11;
            }
        }
#pragma unroll
        for (int j = 0; j < NIT; ++j) {
            const int it = tid - WAVE + j * UW;
            if (tid >= WAVE && it < NU) {
                const int k = it / CH, c = it % CH;
                const typename PairRec<T>::T2 cs = A.cs[k];
                // no skip for s = 0: a uniform path (the update is then exact)
                TV *r0 = (TV *)(Ut + up0[j] * ldu) + c;
                TV *r1 = (TV *)(Ut + up1[j] * ldu) + c;
                const TV u0 = *r0, u1 = *r1;
                TV n0, n1;
                n0.x = cs.x * u0.x - cs.y * u1.x;
                n1.x = cs.y * u0.x + cs.x * u1.x;
                n0.y = cs.x * u0.y - cs.y * u1.y;
                n1.y = cs.y * u0.y + cs.x * u1.y;
                if constexpr (VN == 4) {
                    n0.z = cs.x * u0.z - cs.y * u1.z;
                    n1.z = cs.y * u0.z + cs.x * u1.z;
                    n0.w = cs.x * u0.w - cs.y * u1.w;
                    n1.w = cs.y * u0.w + cs.x * u1.w;
                }
                *r0 = n0;
                *r1 = n1;
                if (CROSS) {
                    up1[j] = cnext(up1[j]);
                } else {
                    up0[j] = rr_next(up0[j], M);
                    up1[j] = rr_next(up1[j], M);
                }
            }
        }
        if (CROSS) {
            pk1 = cnext(pk1);
            pl1 = cnext(pl1);
        } else {
            pk0 = rr_next(pk0, M);
            pk1 = rr_next(pk1, M);
            pl0 = rr_next(pl0, M);
            pl1 = rr_next(pl1, M);
        }
        __syncthreads();
    }
    // write-back in 16-byte pieces: the three stored blocks of the tile (the
    // off-diagonal one in its stored orientation) and U^T (Ut as it is, row i
    // = column i of U), plus the squared off-diagonal sum of the whole tile
    // (the off-diagonal block counts twice) per wavefront and the rotation flag
    T *Uk = U + (int64_t)pk * M * M;
    double acc = 0.0;
#pragma unroll
    for (int e = 0; e < PV; ++e) {
        const int v = tid + e * NT;
        if (v < 3 * VPB) {
            const int s = v / VPB, a = (v % VPB) / BV, c = (v % BV) * VN;
            TV x;
            T *xe = reinterpret_cast<T *>(&x);
#pragma unroll
            for (int q = 0; q < VN; ++q) {
                if (s == 0)
                    xe[q] = S[sidx(a, c + q)];
                else if (s == 1)
                    xe[q] = S[sidx(b + a, b + c + q)];
                else if (!swapo)
                    xe[q] = S[a * ld + b + c + q];
                else
                    xe[q] = S[(c + q) * ld + b + a];
                const double sq = (double)xe[q] * (double)xe[q];
                if (s == 2)
                    acc += 2.0 * sq;
                else if (a != c + q)
                    acc += sq;
            }
            *reinterpret_cast<TV *>(B + blk_row(s, a) * ldb + blk_col(s, c)) = x;
        }
    }
    for (int v = tid; v < M * RV; v += NT) {
        const int i = v / RV, j = (v % RV) * VN;
        *reinterpret_cast<TV *>(Uk + i * M + j) = *reinterpret_cast<const TV *>(Ut + i * ldu + j);
    }
    acc = wave_sum(acc);
    const int lane = tid % WAVE;
    if (lane == 0)
        partial[(int64_t)pk * (NT / WAVE) + tid / WAVE] = acc;
    const int any_rot = __any(rot);
    if (any_rot && lane == 0)
        atomicOr(rot_flag, 1);
    // FP64 sweeps: this wavefront's rotation flag (none applied leaves c = 1,
    // s = 0, t = 0 in every record it wrote, so the tile and U = I come out
    // unchanged).  The FP32 pair solve, the critical path of its rounds, is
    // measured 0.6 us slower with the store and has no flags (prot unused).
    if constexpr (sizeof(T) == 8)
        if (lane == 0)
            prot[pk * PROT_STRIDE + __builtin_amdgcn_readfirstlane(tid / WAVE)] = any_rot;
}

// R16 (template argument, so that the FP32 stage's kernels carry no trace of
// it): every stored entry of the tile rounded to binary16 (the binary16 stage)
// BAT (template argument, so that a single solve's kernel carries none of
// it): a batch of equal-order solves, blockIdx.y = matrix, whose workspace
// buffers lie sW bytes after the previous matrix's; act (or null): matrices
// whose entry is 0 are skipped; thrb (or null): per-matrix thresholds
template <typename T, int M, int NT, bool CROSS, bool R16, bool BAT>
__global__ __launch_bounds__(NT) void pair_solve_kernel(T *__restrict__ B, int64_t ldb,
                                                        const int2 *__restrict__ pairs,
                                                        const int2 *__restrict__ psmap,
                                                        T *__restrict__ U, double eps,
                                                        double thr, int inner,
                                                        double *__restrict__ partial,
                                                        int *rot_flag, int *__restrict__ prot,
                                                        int64_t sW, const int *__restrict__ act,
                                                        const double *__restrict__ thrb)
{
    if constexpr (BAT) {
        const int64_t m = blockIdx.y;
        if (act && !act[m])
            return;
        pair_solve_body<T, M, NT, CROSS>(bat(B, m, sW), ldb, pairs, psmap, bat(U, m, sW), eps,
                                         thrb ? thrb[m] : thr, inner, R16 ? 1 : 0,
                                         bat(partial, m, sW), bat(rot_flag, m, sW),
                                         bat(prot, m, sW), blockIdx.x);
    } else {
        pair_solve_body<T, M, NT, CROSS>(B, ldb, pairs, psmap, U, eps, thr, inner, R16 ? 1 : 0,
                                         partial, rot_flag, prot, blockIdx.x);
    }
}

// The pair solves of a round on workgroups 0 .. npairs-1 and, on the
// workgroups after them, the V update of the previous round (its pairs vpairs
// and rotations vU).  The two parts touch disjoint data: B and U versus V (vU
// is the other U buffer).  The ntile 16-row tiles of pair l's columns are
// split at ntile - vx: V workgroup (l, part) takes part `part` of vranges
// equal ranges of [0, ntile - vx), and pair-solve workgroup l, once its solve
// is done, takes [ntile - vx, ntile).
template <typename T, int M, int NT, bool CROSS, bool R16, bool BAT>
__global__ __launch_bounds__(NT) void pair_solve_v_kernel(
    T *__restrict__ B, int64_t ldb, const int2 *__restrict__ pairs,
    const int2 *__restrict__ psmap, T *__restrict__ U, double eps, double thr, int inner,
    double *__restrict__ partial, int *rot_flag, int *__restrict__ prot, int npairs,
    T *__restrict__ V, int64_t ldv, int64_t ntile, const int2 *__restrict__ vpairs,
    const T *__restrict__ vU, const int *__restrict__ vprot, int vranges, int vwaves, int vx,
    int64_t sW, const int *__restrict__ act, const double *__restrict__ thrb)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *ufl = reinterpret_cast<T *>(smem_raw);
    if constexpr (BAT) {
        const int64_t m = blockIdx.y;
        if (act && !act[m])
            return;
        B = bat(B, m, sW);
        U = bat(U, m, sW);
        partial = bat(partial, m, sW);
        rot_flag = bat(rot_flag, m, sW);
        prot = bat(prot, m, sW);
        V = bat(V, m, sW);
        vU = bat(vU, m, sW);
        vprot = bat(vprot, m, sW);
        if (thrb)
            thr = thrb[m];
    }
    const int64_t split = ntile - vx;
    if ((int)blockIdx.x < npairs) {
        pair_solve_body<T, M, NT, CROSS>(B, ldb, pairs, psmap, U, eps, thr, inner, R16 ? 1 : 0,
                                         partial, rot_flag, prot, blockIdx.x);
        if (vx > 0) {
            __syncthreads(); // the solve's LDS is free again
            vupd::v_update_wg<T, M, NT>(V, ldv, vpairs, blockIdx.x, vU, vprot, split, ntile,
                                        vwaves, ufl);
        }
        return;
    }
    const int wg = (int)blockIdx.x - npairs, l = wg % npairs, part = wg / npairs;
    vupd::v_update_wg<T, M, NT>(V, ldv, vpairs, l, vU, vprot, (int64_t)part * split / vranges,
                                (int64_t)(part + 1) * split / vranges, vwaves, ufl);
}

template <typename T, int M, int NT, bool CROSS, bool R16>
static hipError_t launch_pair_solve_t(T *B, int64_t ldb, int npairs, const int2 *pairs,
                                      const int2 *psmap, T *U, double eps, double thr,
                                      int inner, double *partial, int *rot_flag,
                                      int *prot, size_t smem, hipStream_t s, hipEvent_t e0,
                                      hipEvent_t e1, const Batch &bt)
{
    // the batched kernel exists for the FP64 sweeps only
    constexpr bool CAN_BAT = sizeof(T) == 8 && !R16;
    const bool bt_on = batched(bt);
    if (bt_on && !CAN_BAT)
        return hipErrorInvalidValue;
    auto k = bt_on ? pair_solve_kernel<T, M, NT, CROSS, R16, CAN_BAT>
                   : pair_solve_kernel<T, M, NT, CROSS, R16, false>;
    static size_t smem_set[2] = {0, 0}; // the attribute is set once per size (host-side cost)
    if (smem_set[bt_on] != smem) {
        hipError_t e = hipFuncSetAttribute((const void *)k,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
        if (e != hipSuccess)
            return e;
        smem_set[bt_on] = smem;
    }
    launch_timed(k, dim3(npairs, (unsigned)bt.count), dim3(NT), (uint32_t)smem, s, e0, e1, B, ldb,
                 pairs, psmap, U, eps, thr, inner, partial, rot_flag, prot, bt.sW, bt.act, bt.thr);
    return hipGetLastError();
}

// dynamic LDS of a pair-solve workgroup: Ut, S, two rotation records
template <typename T>
static size_t pair_solve_smem(int b)
{
    const int M = 2 * b;
    const int vn = 16 / (int)sizeof(T);
    return align8(sizeof(T) * ((size_t)M * (M + vn) + (size_t)M * (M + 1))) + 16 +
           2 * (((size_t)b * (8 + 5 * sizeof(T)) + 15) & ~(size_t)15) + 16 * sizeof(double) +
           16 * sizeof(int);
}

template <typename T, bool R16>
static hipError_t launch_pair_solve_r(T *B, int64_t ldb, int b, int npairs, const int2 *pairs,
                                      const int2 *psmap, T *U, double eps, double thr,
                                      int inner, int cross, double *partial, int *rot_flag,
                                      int *prot, hipStream_t s, hipEvent_t e0, hipEvent_t e1,
                                      const Batch &bt)
{
    const int M = 2 * b;
    const size_t smem = pair_solve_smem<T>(b);
    // M = 64: 528 threads own the 2x2 blocks of S; the U items (32 pairs x
    // 64 / VN chunks) go to the threads after the first wavefront.  16
    // wavefronts for both types (10 would cover the FP32 items, but measured
    // slower: the extra wavefronts hide LDS latency).
    constexpr int NT64 = 1024;
    if (M == 64)
        return cross ? launch_pair_solve_t<T, 64, NT64, true, R16>(B, ldb, npairs, pairs, psmap,
                                                                   U, eps, thr, inner, partial,
                                                                   rot_flag, prot, smem, s, e0,
                                                                   e1, bt)
                     : launch_pair_solve_t<T, 64, NT64, false, R16>(B, ldb, npairs, pairs, psmap,
                                                                    U, eps, thr, inner, partial,
                                                                    rot_flag, prot, smem, s, e0,
                                                                    e1, bt);
    if (M == 32)
        return cross ? launch_pair_solve_t<T, 32, 256, true, R16>(B, ldb, npairs, pairs, psmap, U,
                                                                  eps, thr, inner, partial,
                                                                  rot_flag, prot, smem, s, e0, e1, bt)
                     : launch_pair_solve_t<T, 32, 256, false, R16>(B, ldb, npairs, pairs, psmap,
                                                                   U, eps, thr, inner, partial,
                                                                   rot_flag, prot, smem, s, e0,
                                                                   e1, bt);
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_pair_solve(T *B, int64_t ldb, int b, int npairs, const int2 *pairs,
                             const int2 *psmap, T *U, double eps, double thr, int inner, int r16,
                             int cross, double *partial, int *rot_flag, int *prot, hipStream_t s,
                             hipEvent_t e0, hipEvent_t e1, const Batch &bt)
{
    if (sizeof(T) == 4 && r16)
        return launch_pair_solve_r<T, sizeof(T) == 4>(B, ldb, b, npairs, pairs, psmap, U, eps,
                                                      thr, inner, cross, partial, rot_flag, prot,
                                                      s, e0, e1, bt);
    return launch_pair_solve_r<T, false>(B, ldb, b, npairs, pairs, psmap, U, eps, thr, inner,
                                         cross, partial, rot_flag, prot, s, e0, e1, bt);
}

int g_pair_v_wgs = 0;    // V workgroups of the shared launch; 0 = free compute units
size_t g_pair_v_lds = 0; // minimum dynamic LDS per workgroup of the shared launch
int g_pair_v_waves = 0;  // working wavefronts per V workgroup; 0 = default
void tune_pair_v(int wgs, size_t lds, int waves)
{
    g_pair_v_wgs = wgs;
    g_pair_v_lds = lds;
    g_pair_v_waves = waves;
}

template <typename T, int M, int NT, bool CROSS, bool R16>
static hipError_t launch_pair_solve_v_t(T *B, int64_t ldb, int npairs, const int2 *pairs,
                                        const int2 *psmap, T *U, double eps, double thr,
                                        int inner, double *partial, int *rot_flag,
                                        int *prot, size_t smem, T *V, int64_t ldv, int64_t nrows,
                                        const int2 *vpairs, const T *vU, const int *vprot,
                                        hipStream_t s, int vsplit, hipEvent_t e0, hipEvent_t e1,
                                        const Batch &bt)
{
    constexpr bool CAN_BAT = sizeof(T) == 8 && !R16;
    const bool bt_on = batched(bt);
    if (bt_on && !CAN_BAT)
        return hipErrorInvalidValue;
    auto k = bt_on ? pair_solve_v_kernel<T, M, NT, CROSS, R16, CAN_BAT>
                   : pair_solve_v_kernel<T, M, NT, CROSS, R16, false>;
    static size_t smem_set[2] = {0, 0};
    static int cus = 0;
    if (cus == 0) {
        int dev = 0;
        hipGetDevice(&dev);
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (cus <= 0)
            cus = 256;
    }
    const int64_t ntile = nrows / 16;
    // V workgroups: about one per compute unit the pair solves leave free (at
    // least a quarter of the units), a whole number of row ranges per pair
    // (over the whole batch: at least one range per pair of every matrix)
    const int64_t spairs = (int64_t)npairs * bt.count;
    const int64_t vwg = g_pair_v_wgs > 0 ? g_pair_v_wgs
                                         : (cus - spairs > cus / 4 ? cus - spairs : cus / 4);
    int64_t ranges = vwg / spairs;
    if (ranges < 1)
        ranges = 1;
    if (ranges > ntile)
        ranges = ntile;
    // working wavefronts per V workgroup: one per SIMD in FP32, two in FP64
    // (long runs of tiles per wavefront; measured at n = 4096)
    const int vdef = (sizeof(T) == 4 ? 4 : 8) < NT / WAVE ? (sizeof(T) == 4 ? 4 : 8) : NT / WAVE;
    const int vwaves = g_pair_v_waves > 0 && g_pair_v_waves <= NT / WAVE ? g_pair_v_waves : vdef;
    // tiles the pair-solve workgroups take once their solves are done, so
    // that both kinds of workgroup finish together: with R V workgroups per
    // pair at rho tiles/us each and a pair workgroup free for V after tp us,
    // the launch ends at T = (ntile + rho tp) / ((R + 1) rho) and the pair
    // workgroup takes rho (T - tp) tiles (none when the V part finishes
    // first).  rho and tp measured on MI355X at 2b = 64, n = 4096: the pair
    // solve takes 29.6 us (FP32) / 31.7 us (FP64) on the cross schedule and
    // 58.6 / 66.1 us on the full one, plus about 3 us to stage U_l and fill
    // the V pipeline; 2.63 / 1.19 tiles/us.  (Measured: FP64
    // splits of 20, 33, 36 and 52 tiles at n = 4096 gave plain solves of
    // 188.7, 184.6, 184.3 and 194.4 ms; FP32 splits of 6 tiles were slower
    // than none.)
    int vx = 0;
    if (M == 64 && vsplit > 0) {
        vx = (int)std::min<int64_t>(vsplit, ntile - ranges);
    } else if (M == 64 && vsplit == 0) {
        const double tp = 3.0 + (sizeof(T) == 4 ? (CROSS ? 29.6 : 58.6) : (CROSS ? 31.7 : 66.1));
        const double rho = sizeof(T) == 4 ? 2.63 : 1.19;
        const double T_end = ((double)ntile + rho * tp) / ((double)(ranges + 1) * rho);
        const double x = rho * (T_end - tp);
        if (x > 0.0)
            vx = (int)std::min<double>(x + 0.5, (double)ntile / (double)(ranges + 1));
    }
    // a batch whose pair solves alone fill the compute units: no V
    // workgroups, every pair-solve workgroup updates its pair's V columns
    // after its solve (the same per-tile arithmetic as a V workgroup's)
    if (bt.count > 1 && spairs >= cus && g_pair_v_wgs == 0 && vsplit == 0) {
        ranges = 0;
        vx = (int)ntile;
    }
    const unsigned grid_x = (unsigned)(npairs + ranges * npairs);
    const size_t lds = smem > g_pair_v_lds ? smem : g_pair_v_lds;
    if (lds != smem_set[bt_on]) {
        hipError_t e = hipFuncSetAttribute((const void *)k,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess)
            return e;
        smem_set[bt_on] = lds;
    }
    launch_timed(k, dim3(grid_x, (unsigned)bt.count), dim3(NT), (uint32_t)lds, s, e0, e1, B, ldb,
                 pairs, psmap, U, eps, thr, inner, partial, rot_flag, prot, npairs, V, ldv, ntile,
                 vpairs, vU, vprot, (int)ranges, vwaves, vx, bt.sW, bt.act, bt.thr);
    return hipGetLastError();
}

template <typename T, bool R16>
static hipError_t launch_pair_solve_v_r(T *B, int64_t ldb, int b, int npairs, const int2 *pairs,
                                        const int2 *psmap, T *U, double eps, double thr,
                                        int inner, int cross, double *partial, int *rot_flag,
                                        int *prot, T *V, int64_t ldv, int64_t nrows,
                                        const int2 *vpairs, const T *vU, const int *vprot,
                                        hipStream_t s, int vsplit, hipEvent_t e0, hipEvent_t e1,
                                        const Batch &bt)
{
    const int M = 2 * b;
    const size_t smem = pair_solve_smem<T>(b);
    if (M == 64)
        return cross ? launch_pair_solve_v_t<T, 64, 1024, true, R16>(
                           B, ldb, npairs, pairs, psmap, U, eps, thr, inner, partial, rot_flag,
                           prot, smem, V, ldv, nrows, vpairs, vU, vprot, s, vsplit, e0, e1, bt)
                     : launch_pair_solve_v_t<T, 64, 1024, false, R16>(
                           B, ldb, npairs, pairs, psmap, U, eps, thr, inner, partial, rot_flag,
                           prot, smem, V, ldv, nrows, vpairs, vU, vprot, s, vsplit, e0, e1, bt);
    if (M == 32)
        return cross ? launch_pair_solve_v_t<T, 32, 256, true, R16>(
                           B, ldb, npairs, pairs, psmap, U, eps, thr, inner, partial, rot_flag,
                           prot, smem, V, ldv, nrows, vpairs, vU, vprot, s, vsplit, e0, e1, bt)
                     : launch_pair_solve_v_t<T, 32, 256, false, R16>(
                           B, ldb, npairs, pairs, psmap, U, eps, thr, inner, partial, rot_flag,
                           prot, smem, V, ldv, nrows, vpairs, vU, vprot, s, vsplit, e0, e1, bt);
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_pair_solve_v(T *B, int64_t ldb, int b, int npairs, const int2 *pairs,
                               const int2 *psmap, T *U, double eps, double thr, int inner,
                               int r16, int cross, double *partial, int *rot_flag, int *prot, T *V,
                               int64_t ldv, int64_t nrows, const int2 *vpairs, const T *vU,
                               const int *vprot, hipStream_t s, int vsplit, hipEvent_t e0,
                               hipEvent_t e1, const Batch &bt)
{
    if (nrows % 16 != 0 || ldv % (16 / (int64_t)sizeof(T)) != 0 || ((uintptr_t)V % 16) != 0)
        return hipErrorInvalidValue;
    if (sizeof(T) == 4 && r16)
        return launch_pair_solve_v_r<T, sizeof(T) == 4>(B, ldb, b, npairs, pairs, psmap, U, eps,
                                                        thr, inner, cross, partial, rot_flag,
                                                        prot, V, ldv, nrows, vpairs, vU, vprot,
                                                        s, vsplit, e0, e1, bt);
    return launch_pair_solve_v_r<T, false>(B, ldb, b, npairs, pairs, psmap, U, eps, thr, inner,
                                           cross, partial, rot_flag, prot, V, ldv, nrows, vpairs,
                                           vU, vprot, s, vsplit, e0, e1, bt);
}


// ------------------------------------------------------- reductions, etc.
__global__ __launch_bounds__(256) void sum_kernel(const double *__restrict__ x, int64_t count,
                                                  double *out, int64_t sW,
                                                  const int *__restrict__ act)
{
    const int64_t m = blockIdx.x; // matrix of a batch (0 for a single sum)
    if (act && !act[m])
        return;
    x = bat(x, m, sW);
    out = bat(out, m, sW);
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

hipError_t launch_sum(const double *x, int64_t count, double *out, hipStream_t s,
                      const Batch &bt)
{
    hipLaunchKernelGGL(sum_kernel, dim3((unsigned)bt.count), dim3(256), 0, s, x, count, out,
                       bt.sW, bt.act);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void max_kernel(const double *__restrict__ x, int64_t count,
                                                  double *out)
{
    __shared__ double red[4];
    double m = 0.0;
    for (int64_t i = threadIdx.x; i < count; i += 256)
        m = fmax(m, x[i]);
#pragma unroll
    for (int off = WAVE / 2; off > 0; off >>= 1)
        m = fmax(m, __shfl_xor(m, off, WAVE));
    if (threadIdx.x % WAVE == 0)
        red[threadIdx.x / WAVE] = m;
    __syncthreads();
    if (threadIdx.x == 0)
        out[0] = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

hipError_t launch_max(const double *x, int64_t count, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(max_kernel, dim3(1), dim3(256), 0, s, x, count, out);
    return hipGetLastError();
}

// x <- 2^k x in place (exact: a power of two, applied in two steps so that
// |k| up to 2100 never overflows the factor), optionally also into copy.
__global__ __launch_bounds__(256) void scale_pow2_kernel(double *__restrict__ x, int64_t count,
                                                         int k, double *__restrict__ copy)
{
    const int k1 = k / 2, k2 = k - k / 2;
    for (int64_t e = blockIdx.x * 256 + threadIdx.x; e < count; e += (int64_t)gridDim.x * 256) {
        const double v = ldexp(ldexp(x[e], k1), k2);
        x[e] = v;
        if (copy)
            copy[e] = v;
    }
}

hipError_t launch_scale_pow2(double *x, int64_t count, int k, double *copy, hipStream_t s)
{
    if (count <= 0)
        return hipSuccess;
    const int64_t blocks = std::min<int64_t>((count + 255) / 256, 4096);
    hipLaunchKernelGGL(scale_pow2_kernel, dim3((unsigned)blocks), dim3(256), 0, s, x, count, k,
                       copy);
    return hipGetLastError();
}

// Symmetrised copy of A into the padded working matrix (32 x 32 tiles staged
// through LDS so that both A and A^T are read along rows), plus the partial
// sums of squares for ||B||_F (partial[block]), the partial maxima of |b_ij|
// (partial[INGEST_BLOCKS + block]) and the non-finite / asymmetry flags.
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
    double acc = 0.0, amax = 0.0;
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
            amax = fmax(amax, fabs(v));
        }
        __syncthreads();
    }
    acc = wave_sum(acc);
#pragma unroll
    for (int off = WAVE / 2; off > 0; off >>= 1)
        amax = fmax(amax, __shfl_xor(amax, off, WAVE));
    __shared__ double redm[4];
    if (threadIdx.x % WAVE == 0) {
        red[threadIdx.x / WAVE] = acc;
        redm[threadIdx.x / WAVE] = amax;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        partial[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
        partial[INGEST_BLOCKS + blockIdx.x] = fmax(fmax(redm[0], redm[1]), fmax(redm[2], redm[3]));
    }
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

// the same count_per entries in every matrix's workspace region
__global__ void fill_batch_i32_kernel(int *p, int64_t count_per, int value, int64_t sW,
                                      const int *__restrict__ act)
{
    const int64_t m = blockIdx.y;
    if (act && !act[m])
        return;
    p = bat(p, m, sW);
    for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < count_per; i += (int64_t)gridDim.x * 256)
        p[i] = value;
}

hipError_t launch_fill_batch_i32(int *p, int64_t count_per, int value, const Batch &bt,
                                 hipStream_t s)
{
    int grid = (int)((count_per + 255) / 256);
    grid = grid < 1 ? 1 : (grid > 64 ? 64 : grid);
    hipLaunchKernelGGL(fill_batch_i32_kernel, dim3(grid, (unsigned)bt.count), dim3(256), 0, s, p,
                       count_per, value, bt.sW, bt.act);
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

// dst = fl32(2^k src), rounded on to binary16 when r16 (the binary16 stage's
// starting matrix); k is a small exponent (|k| < 1000)
__global__ void cast_f32_scaled_kernel(const double *__restrict__ src, float *__restrict__ dst,
                                       int64_t count, int k, int r16)
{
    for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < count; i += (int64_t)gridDim.x * 256)
        dst[i] = store_round<float>((float)ldexp(src[i], k), r16);
}

hipError_t launch_cast_f32_scaled(const double *src, float *dst, int64_t count, int k, int r16,
                                  hipStream_t s)
{
    hipLaunchKernelGGL(cast_f32_scaled_kernel, dim3(2048), dim3(256), 0, s, src, dst, count, k,
                       r16);
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

// ---------------------------------------------------------------- finalize
__global__ void diag_kernel(const double *__restrict__ B, int64_t ldb, int64_t n,
                            double *__restrict__ w)
{
    for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        w[i] = B[i * ldb + i];
}

// Rayleigh quotients w_k = v_k^T (A v_k) from T = A V: column dots over row
// chunk blockIdx.y (partial sums), then a sum over the chunks.
constexpr int RQ_CHUNKS = 16;
__global__ __launch_bounds__(256) void rq_partial_kernel(const double *__restrict__ V,
                                                         int64_t ldv,
                                                         const double *__restrict__ T,
                                                         int64_t ldt, int64_t n,
                                                         double *__restrict__ part)
{
    const int64_t k = blockIdx.x * 256 + threadIdx.x;
    if (k >= n)
        return;
    const int64_t r0 = blockIdx.y * n / RQ_CHUNKS, r1 = (blockIdx.y + 1) * n / RQ_CHUNKS;
    double acc = 0.0;
    for (int64_t i = r0; i < r1; ++i)
        acc = fma(V[i * ldv + k], T[i * ldt + k], acc);
    part[blockIdx.y * n + k] = acc;
}

// w_k = (sum of the chunk partials) inv_k^2: the quotient of the normalized
// column v_k / ||v_k||
__global__ void rq_sum_kernel(const double *__restrict__ part, int64_t n,
                              const double *__restrict__ inv, double *__restrict__ w)
{
    const int64_t k = blockIdx.x * 256 + threadIdx.x;
    if (k >= n)
        return;
    double acc = 0.0;
    for (int c = 0; c < RQ_CHUNKS; ++c)
        acc += part[c * n + k];
    w[k] = acc * inv[k] * inv[k];
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

// Column statistics of the accumulated V, read along rows: pass 1 scans row
// chunk z for every column j (threads over j) and keeps the entry of largest
// magnitude (lowest row on ties) and the sum of squares; pass 2 reduces the
// chunks in order.  The output columns are scaled to unit 2-norm: the rounding
// of the rotations lets the column norms drift by a random walk while the
// columns stay orthogonal to each other to a much smaller error, so the scaling
// removes nearly all of ||V^T V - I||.  The entry of largest magnitude becomes
// positive (sign convention).
constexpr int SIGN_CHUNKS = 16;

__global__ __launch_bounds__(256) void colmax_kernel(const double *__restrict__ V, int64_t ldv,
                                                     int64_t n, double *__restrict__ cmax,
                                                     int *__restrict__ cidx,
                                                     double *__restrict__ csq)
{
    const int64_t j = blockIdx.x * 256 + threadIdx.x;
    const int z = blockIdx.y;
    if (j >= n)
        return;
    const int64_t chunk = (n + SIGN_CHUNKS - 1) / SIGN_CHUNKS;
    const int64_t i0 = z * chunk, i1 = (i0 + chunk < n) ? i0 + chunk : n;
    double best = -1.0, sq = 0.0;
    int64_t bi = i0 < n ? i0 : 0;
    for (int64_t i = i0; i < i1; ++i) {
        const double v = V[i * ldv + j];
        const double a = fabs(v);
        sq = fma(v, v, sq);
        if (a > best) {
            best = a;
            bi = i;
        }
    }
    cmax[z * n + j] = best;
    cidx[z * n + j] = (int)bi;
    csq[z * n + j] = sq;
}

// inv[j] = 1 / ||V[:, j]|| for j < n, 1 for the padding columns j < npad
__global__ __launch_bounds__(256) void colinv_kernel(const double *__restrict__ csq, int64_t n,
                                                     int64_t npad, double *__restrict__ inv)
{
    const int64_t j = blockIdx.x * 256 + threadIdx.x;
    if (j >= npad)
        return;
    if (j >= n) {
        inv[j] = 1.0;
        return;
    }
    double sq = 0.0;
    for (int z = 0; z < SIGN_CHUNKS; ++z)
        sq += csq[z * n + j];
    inv[j] = sq > 0.0 ? 1.0 / sqrt(sq) : 1.0;
}

__global__ __launch_bounds__(256) void colsign_kernel(const double *__restrict__ V, int64_t ldv,
                                                      int64_t n, const int *__restrict__ perm,
                                                      const double *__restrict__ cmax,
                                                      const int *__restrict__ cidx,
                                                      const double *__restrict__ inv,
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
    sg[c] = V[(int64_t)bi * ldv + col] < 0.0 ? -inv[col] : inv[col];
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

hipError_t launch_rayleigh(const double *V, int64_t ldv, const double *T, int64_t ldt,
                           int64_t n, const double *inv, double *part, double *w, hipStream_t s)
{
    int g = (int)((n + 255) / 256);
    hipLaunchKernelGGL(rq_partial_kernel, dim3(g, RQ_CHUNKS), dim3(256), 0, s, V, ldv, T, ldt,
                       n, part);
    hipLaunchKernelGGL(rq_sum_kernel, dim3(g), dim3(256), 0, s, part, n, inv, w);
    return hipGetLastError();
}

hipError_t launch_colstats(const double *V, int64_t ldv, int64_t n, int64_t npad, double *cmax,
                           int *cidx, double *csq, double *inv, hipStream_t s)
{
    const int g = (int)((n + 255) / 256);
    hipLaunchKernelGGL(colmax_kernel, dim3(g, SIGN_CHUNKS), dim3(256), 0, s, V, ldv, n, cmax,
                       cidx, csq);
    hipLaunchKernelGGL(colinv_kernel, dim3((unsigned)((npad + 255) / 256)), dim3(256), 0, s, csq,
                       n, npad, inv);
    return hipGetLastError();
}

// Output stage from the extracted diagonal w: stable ascending order, column
// permutation and sign convention.
hipError_t launch_finalize(const double *w, const double *V, int64_t ldv_in, int64_t n,
                           double *W, double *Vout, int64_t ldv, int *perm, double *sg,
                           const double *cmax, const int *cidx, const double *inv,
                           hipStream_t s)
{
    int g = (int)((n + 255) / 256);
    hipLaunchKernelGGL(rank_kernel, dim3(g), dim3(256), 0, s, w, n, perm);
    hipLaunchKernelGGL(colsign_kernel, dim3(g), dim3(256), 0, s, V, ldv_in, n, perm, cmax, cidx,
                       inv, sg);
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

// Orthogonality probe of the output stage, for 4 probe vectors X (n_pad x 4,
// zero past n) and the column scaling D^-1 = diag(inv):
//   Y = V D^-1 X                     (probe_vx_kernel, rows of V),
//   P_z = V[rows of chunk z]^T Y     (probe_vty_kernel, columns of V),
//   r = D^-1 sum_z P_z - X, partial sums of r^2 per block (probe_resid_kernel).
// ||r||_F^2 / 4 estimates ||D^-1 V^T V D^-1 - I||_F^2.  Each pass reads V
// once along its rows (the products are HBM-bound).
constexpr int PROBE_K = 4, PROBE_CHUNKS = 16, PROBE_JC = 512, PROBE_ROWS = 2;

__global__ __launch_bounds__(256) void probe_vx_kernel(const double *__restrict__ V,
                                                       int64_t ldv, int64_t n, int64_t npad,
                                                       const double *__restrict__ X,
                                                       const double *__restrict__ inv,
                                                       double *__restrict__ Y)
{
    typedef double dv2p __attribute__((ext_vector_type(2)));
    __shared__ __align__(16) double xs[PROBE_JC * PROBE_K];
    const int tid = threadIdx.x, lane = tid % WAVE, w = tid / WAVE;
    const int64_t r0 = ((int64_t)blockIdx.x * 4 + w) * PROBE_ROWS;
    double acc[PROBE_ROWS][PROBE_K];
#pragma unroll
    for (int r = 0; r < PROBE_ROWS; ++r)
#pragma unroll
        for (int c = 0; c < PROBE_K; ++c)
            acc[r][c] = 0.0;
    for (int64_t j0 = 0; j0 < n; j0 += PROBE_JC) {
        __syncthreads();
        for (int e = tid; e < PROBE_JC * PROBE_K; e += 256) {
            const int64_t j = j0 + e / PROBE_K;
            xs[e] = j < n ? inv[j] * X[j * PROBE_K + e % PROBE_K] : 0.0;
        }
        __syncthreads();
        // lane reads columns j0 + 128 q + 2 lane, + 1 (q < 4): one 16-byte load
        // per row and q, consecutive lanes at consecutive addresses; npad is
        // even, so a pair is in range or out of range as a whole
#pragma unroll
        for (int q = 0; q < PROBE_JC / 128; ++q) {
            const int jc = 128 * q + 2 * lane;
            if (j0 + jc >= npad)
                break;
            double xv[2][PROBE_K];
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int c = 0; c < PROBE_K; ++c)
                    xv[h][c] = xs[(jc + h) * PROBE_K + c];
#pragma unroll
            for (int r = 0; r < PROBE_ROWS; ++r) {
                if (r0 + r >= npad)
                    break;
                const dv2p v = *reinterpret_cast<const dv2p *>(V + (r0 + r) * ldv + j0 + jc);
#pragma unroll
                for (int c = 0; c < PROBE_K; ++c)
                    acc[r][c] = fma(v[1], xv[1][c], fma(v[0], xv[0][c], acc[r][c]));
            }
        }
    }
#pragma unroll
    for (int r = 0; r < PROBE_ROWS; ++r)
#pragma unroll
        for (int c = 0; c < PROBE_K; ++c) {
            const double v = wave_sum(acc[r][c]);
            if (lane == 0 && r0 + r < npad)
                Y[(r0 + r) * PROBE_K + c] = v;
        }
}

__global__ __launch_bounds__(256) void probe_vty_kernel(const double *__restrict__ V,
                                                        int64_t ldv, int64_t n, int64_t npad,
                                                        const double *__restrict__ Y,
                                                        double *__restrict__ P)
{
    constexpr int YR = 1024; // rows of Y staged in LDS at a time
    __shared__ __align__(16) double ys[YR * PROBE_K];
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int z = blockIdx.y;
    const int64_t chunk = (npad + PROBE_CHUNKS - 1) / PROBE_CHUNKS;
    const int64_t i0 = z * chunk, i1 = i0 + chunk < npad ? i0 + chunk : npad;
    double acc[PROBE_K] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t ib = i0; ib < i1; ib += YR) {
        const int64_t ie = ib + YR < i1 ? ib + YR : i1;
        __syncthreads();
        for (int64_t e = threadIdx.x; e < (ie - ib) * PROBE_K; e += 256)
            ys[e] = Y[ib * PROBE_K + e];
        __syncthreads();
        if (j < n) {
#pragma unroll 8
            for (int64_t i = ib; i < ie; ++i) {
                const double v = V[i * ldv + j];
#pragma unroll
                for (int c = 0; c < PROBE_K; ++c)
                    acc[c] = fma(v, ys[(i - ib) * PROBE_K + c], acc[c]);
            }
        }
    }
    if (j < n) {
#pragma unroll
        for (int c = 0; c < PROBE_K; ++c)
            P[((int64_t)z * n + j) * PROBE_K + c] = acc[c];
    }
}

__global__ __launch_bounds__(256) void probe_resid_kernel(const double *__restrict__ P,
                                                          int64_t n,
                                                          const double *__restrict__ X,
                                                          const double *__restrict__ inv,
                                                          double *__restrict__ partial)
{
    __shared__ double red[4];
    double acc = 0.0;
    for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < n;
         j += (int64_t)gridDim.x * 256) {
#pragma unroll
        for (int c = 0; c < PROBE_K; ++c) {
            double zsum = 0.0;
            for (int z = 0; z < PROBE_CHUNKS; ++z)
                zsum += P[((int64_t)z * n + j) * PROBE_K + c];
            const double r = inv[j] * zsum - X[j * PROBE_K + c];
            acc = fma(r, r, acc);
        }
    }
    acc = wave_sum(acc);
    if (threadIdx.x % WAVE == 0)
        red[threadIdx.x / WAVE] = acc;
    __syncthreads();
    if (threadIdx.x == 0)
        partial[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

hipError_t launch_orth_probe(const double *V, int64_t ldv, int64_t n, int64_t npad, int k,
                             const double *X, const double *inv, double *Y, double *P,
                             double *partial, int nblocks, hipStream_t s)
{
    if (k != PROBE_K || npad % 8 != 0 || nblocks < 1)
        return hipErrorInvalidValue;
    const unsigned g1 = (unsigned)((npad + 4 * PROBE_ROWS - 1) / (4 * PROBE_ROWS));
    hipLaunchKernelGGL(probe_vx_kernel, dim3(g1), dim3(256), 0, s, V, ldv, n, npad, X, inv, Y);
    hipLaunchKernelGGL(probe_vty_kernel, dim3((unsigned)((n + 255) / 256), PROBE_CHUNKS),
                       dim3(256), 0, s, V, ldv, n, npad, Y, P);
    hipLaunchKernelGGL(probe_resid_kernel, dim3((unsigned)nblocks), dim3(256), 0, s, P, n, X,
                       inv, partial);
    return hipGetLastError();
}

// explicit instantiations
template hipError_t launch_pair_solve_v<double>(double *, int64_t, int, int, const int2 *,
                                               const int2 *, double *, double, double, int, int, int,
                                               double *, int *, int *, double *, int64_t,
                                               int64_t, const int2 *, const double *,
                                               const int *, hipStream_t, int, hipEvent_t,
                                               hipEvent_t, const Batch &);
template hipError_t launch_pair_solve_v<float>(float *, int64_t, int, int, const int2 *,
                                              const int2 *, float *, double, double, int, int, int,
                                              double *, int *, int *, float *, int64_t,
                                              int64_t, const int2 *, const float *, const int *,
                                              hipStream_t, int, hipEvent_t, hipEvent_t,
                                              const Batch &);
template hipError_t launch_pair_solve<double>(double *, int64_t, int, int, const int2 *,
                                              const int2 *, double *, double, double, int, int, int,
                                              double *, int *, int *, hipStream_t, hipEvent_t,
                                              hipEvent_t, const Batch &);
template hipError_t launch_pair_solve<float>(float *, int64_t, int, int, const int2 *,
                                             const int2 *, float *, double, double, int, int, int,
                                             double *, int *, int *, hipStream_t, hipEvent_t,
                                             hipEvent_t, const Batch &);

// Thread -> 2x2 block map of the pair solve for M = 2b positions: entry t < M/2
// is the block hosting pair t of the next round, then the M/2 diagonal blocks
// (k, k) (so that their different code path stays inside the first
// wavefronts), then the rest in row order.  cross != 0 gives the map of the
// cross schedule.
void pair_solve_map(int M, int cross, int2 *out)
{
    const int h = M / 2;
    if (cross) {
        int cnt = 0;
        for (int t = 0; t + 1 < h; ++t)
            out[cnt++] = make_int2(t, t + 1);
        out[cnt++] = make_int2(0, h - 1);
        for (int k = 0; k < h; ++k)
            out[cnt++] = make_int2(k, k);
        for (int k = 0; k < h; ++k)
            for (int l = k + 1; l < h; ++l)
                if (!(l == k + 1 || (k == 0 && l == h - 1)))
                    out[cnt++] = make_int2(k, l);
        return;
    }
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
        out[cnt++] = make_int2(k, k);
    for (int k = 0; k < h; ++k)
        for (int l = k + 1; l < h; ++l)
            if (!used[k][l])
                out[cnt++] = make_int2(k, l);
}
template hipError_t launch_ingest<double>(const double *, int64_t, int64_t, double *, int64_t,
                                          double *, int *, int, hipStream_t);
template hipError_t launch_ingest<float>(const double *, int64_t, int64_t, float *, int64_t,
                                         double *, int *, int, hipStream_t);
template hipError_t launch_eye<double>(double *, int64_t, hipStream_t);
template hipError_t launch_eye<float>(float *, int64_t, hipStream_t);
template hipError_t launch_off2_partial<double>(const double *, int64_t, double *, hipStream_t);
template hipError_t launch_off2_partial<float>(const float *, int64_t, double *, hipStream_t);

} // namespace lj
