// Update kernels of the block path (the round's block rotation, Section 3.3
// applied blockwise): the eigenvectors V[:, cols(P, Q)] <- V[:, cols(P, Q)] U_PQ
// for every block pair (P, Q) of the round (the per-wavefront body is in
// update_v.hpp), and the off-diagonal tiles B_kl <- U_k^T B_kl U_l of every two
// pairs k < l (B's upper blocks).
#include "internal.hpp"
#include "common.hpp"
#include "update_v.hpp"

#include <vector>

namespace lj {

namespace {

using namespace vupd;

template <typename T, int M, bool BAT>
__global__ __launch_bounds__(256) void update_v_kernel(T *__restrict__ V, int64_t ldv,
                                                       int64_t ntile, const int2 *__restrict__ pairs,
                                                       int npairs, const T *__restrict__ U,
                                                       const int *__restrict__ prot, int chunks,
                                                       int64_t sW, const int *__restrict__ act)
{
    // BAT: a batch of equal-order solves (blockIdx.y = matrix, buffers sW
    // bytes apart); a template argument so that a single solve's kernel
    // carries none of it
    if constexpr (BAT) {
        const int64_t m = blockIdx.y;
        if (act && !act[m])
            return;
        vupd::v_update_wave<T, M>(bat(V, m, sW), ldv, ntile, pairs, npairs, bat(U, m, sW),
                                  bat(prot, m, sW), chunks,
                                  blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE);
    } else {
        vupd::v_update_wave<T, M>(V, ldv, ntile, pairs, npairs, U, prot, chunks,
                                  blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE);
    }
}

// B update.  The kernel takes a list of T tiles (k, l), k < l (all of them,
// or a subset); workgroup g of G takes the run [g T / G, (g + 1) T / G) of
// the list (the same share for every workgroup), so a list sorted by l keeps
// the column pair of a run mostly fixed.  Its M/16 wavefronts produce rows
// 16w .. 16w + 15 of Z = U_k^T X U_l as two chained MFMA products:
//   C1 = X^T U_k (M-index c, N-index i, K-index r): the A operand X^T is
//        staged through LDS from the four stored b x b blocks of the tile (B
//        keeps only its upper blocks during the sweeps; a block stored in X
//        orientation is transposed on the way into LDS); the B operand U_k is
//        per-lane registers;
//   Z^T = U_l^T C1 (M-index j, K-index c): the accumulator of C1 already has
//        the B-operand layout (element v of a lane is C1[16 tc + acc_row][li]),
//        so C1 never leaves registers; the A operand U_l^T sits in LDS in
//        per-lane fragment order (16-byte reads at consecutive addresses),
//        refilled when the run reaches a new l.
// Each b x b block of Z is stored once, into B's upper block: along its rows
// with 16-byte stores (out_perm again), or transposed with one element per
// lane.  The next tile's X^T and U_k are loaded while the current one
// computes.  With rotation flags (prot) and no off^2 wanted, a tile whose two
// pairs applied no rotation has U_k = U_l = I, so Z = X: a workgroup whose
// whole run consists of such tiles adds their count to *skipped and returns
// after its first tile's loads (a per-tile test inside the pipelined loop
// costs the loop registers).
// R16: Z rounded to binary16 on its way to B (the binary16 stage), a
// template argument so that the FP32 stage's kernel carries no trace of it.
template <typename T, int M, bool R16, bool BAT>
__global__ __launch_bounds__(M * 4, sizeof(T) == 4 ? 4 : 2) void update_b_kernel(T *__restrict__ B, int64_t ldb,
                                                         const int2 *__restrict__ pairs_g,
                                                         int npairs, const T *__restrict__ U,
                                                         double *__restrict__ partial,
                                                         int want_off,
                                                         const int *__restrict__ prot,
                                                         int *skipped, int64_t sW,
                                                         const int *__restrict__ act)
{
    // BAT: a batch of equal-order solves, blockIdx.y is the matrix, whose
    // buffers lie sW bytes after the previous one's (a template argument: the
    // offsets cost the single-solve kernel registers)
    if constexpr (BAT) {
        const int64_t m = blockIdx.y;
        if (act && !act[m])
            return;
        B = bat(B, m, sW);
        U = bat(U, m, sW);
        partial = bat(partial, m, sW);
        prot = bat(prot, m, sW);
        skipped = bat(skipped, m, sW);
    }
    constexpr int r16 = R16 ? 1 : 0;
    constexpr int b = M / 2, NW = M / 16, NT = NW * WAVE;
    constexpr int VK = 16 / (int)sizeof(T);
    constexpr int TC = M / 16, TJ = M / 16, KG = M / (4 * VK);
    constexpr int LDX = M + VK;       // padded LDS row of the X^T tile
    constexpr int BV = b / VK;        // 16-byte vectors per sub-block row
    constexpr int VPB = b * BV;       // vectors per b x b sub-block
    constexpr int PERV = 4 * VPB / NT; // vectors per thread per tile
    constexpr int HV = 4 / VK;        // 16-byte reads per lane per U_l fragment
    typedef typename V16<T>::type TV;
    typedef typename acc4<T>::type accT;
    constexpr int ZLD = 16 + VK; // padded row of a wavefront's transpose scratch
    __shared__ __align__(16) T xs[M * LDX];
    __shared__ __align__(16) T ufl[M * M];
    __shared__ __align__(16) T zsc[NW * 16 * ZLD];
    const int tid = threadIdx.x, lane = tid % WAVE, w = tid / WAVE;
    const int li = lane % 16, lk = lane / 16;
    T *zw = zsc + w * 16 * ZLD;
    const int ntiles = npairs * (npairs - 1) / 2;
    // XCD-aware run order: workgroups go to the 8 XCDs round-robin (blockIdx
    // mod 8), so the workgroups of one XCD take one contiguous eighth of the
    // tile list (a range of l): that XCD's L2 then holds the U_l of its range
    // only, instead of every XCD fetching every U block
    const int G = (int)gridDim.x;
    const int g = G % 8 == 0 ? (int)(blockIdx.x % 8) * (G / 8) + (int)(blockIdx.x / 8)
                             : (int)blockIdx.x;
    const int t0 = (int)((int64_t)g * ntiles / G);
    const int t1 = (int)((int64_t)(g + 1) * ntiles / G);
    if (t0 >= t1)
        return;
    // tile t of the list (k < l, by l then k) is (t - l (l - 1) / 2, l), and
    // the pair entries are read with scalar loads (the indices are uniform):
    // the loop has no vector loads whose values it waits for, as such a wait
    // would also wait for the stores of the previous tile
    auto tile_kl = [](int t) __attribute__((always_inline)) {
        int l = (int)((1.0f + sqrtf(1.0f + 8.0f * (float)t)) * 0.5f);
        while ((int64_t)l * (l - 1) / 2 > t)
            --l;
        while ((int64_t)(l + 1) * l / 2 <= t)
            ++l;
        return make_int2(__builtin_amdgcn_readfirstlane(t - (int)((int64_t)l * (l - 1) / 2)),
                         __builtin_amdgcn_readfirstlane(l));
    };
    const int2 *__restrict__ pairs = pairs_g;
    // ufl[((f HV + h) 64 + lane) VK + j] = U_l[16 tc + acc_row(lk, v)][16 tj + out_perm(li)]
    // with f = tj TC + tc and v = h VK + j: fragment v of lane for step (tc, v)
    // all M*M/NT gathers of a thread are issued before the first LDS write,
    // so the fill costs one memory latency
    auto fill_ufl = [&](int l) __attribute__((always_inline)) {
        const T *Ult = U + (int64_t)l * M * M; // transposed: Ult[j][i] = U_l[i][j]
        constexpr int PF = M * M / NT;
        T u[PF];
#pragma unroll
        for (int q = 0; q < PF; ++q) {
            const int e = tid + q * NT;
            const int j = e % VK, ln = (e / VK) % WAVE, r = e / (VK * WAVE);
            const int v = (r % HV) * VK + j, f = r / HV, tc = f % TC, tj = f / TC;
            u[q] = Ult[(16 * tj + out_perm<T>(ln % 16)) * M + 16 * tc + acc_row<T>(ln / 16, v)];
        }
#pragma unroll
        for (int q = 0; q < PF; ++q)
            ufl[tid + q * NT] = u[q];
    };
    // one tile's X^T pieces and U_k fragments; two of them alternate (the
    // next tile's loads fly while the current one computes)
    struct Buf {
        TV xr[PERV];
        T uk[KG * VK];
    };
    // X^T consists of four b x b sub-blocks s = 2 ci + ri: rows of block
    // C = (ci ? pl.y : pl.x) of the column pair, columns of block R = (ri ?
    // pk.y : pk.x) of the row pair.  B keeps only blocks (I, J) with I <= J, so
    // a sub-block with C < R is read in X^T orientation, one with C > R as its
    // stored transpose (the decision is uniform per sub-block, and a
    // sub-block covers whole wavefronts).
    // Every piece is a column gather: thread piece q of a sub-block holds the
    // VK entries (a0 .. a0 + VK - 1, c) of the stored block, c = q mod b,
    // a0 = VK (q / b), one element load each (consecutive lanes read
    // consecutive columns of a row, so every load is coalesced).  That is
    // one 16-byte row piece of X^T when the block is stored transposed, and a
    // column piece otherwise; both orientations issue the same loads.
    auto load_tile = [&](Buf &nb, int t) __attribute__((always_inline)) {
        const int2 kl = tile_kl(t);
        const int2 pk = pairs[kl.x], pl = pairs[kl.y];
#pragma unroll
        for (int e = 0; e < PERV; ++e) {
            const int idx = tid + e * NT, sb = idx / VPB, q = idx % VPB;
            const int c = q % b, a0 = (q / b) * VK;
            const int C = (sb >> 1) ? pl.y : pl.x, R = (sb & 1) ? pk.y : pk.x;
            const T *src = B + ((int64_t)(C < R ? C : R) * b + a0) * ldb +
                           (int64_t)(C < R ? R : C) * b + c;
#pragma unroll
            for (int j = 0; j < VK; ++j)
                nb.xr[e][j] = src[j * ldb];
        }
        const T *Ukt = U + (int64_t)kl.x * M * M; // transposed: Ukt[j][i] = U_k[i][j]
#pragma unroll
        for (int g = 0; g < KG; ++g) {
            const TV u = *reinterpret_cast<const TV *>(Ukt + (16 * w + li) * M + g * 4 * VK +
                                                       lk * VK);
#pragma unroll
            for (int j = 0; j < VK; ++j)
                nb.uk[g * VK + j] = vlane<T>(u, j);
        }
    };
    int cur_l = -1;
    auto body = [&](int t, const Buf &cb, Buf &nb, int tn) __attribute__((always_inline)) {
        lds_barrier(); // xs and ufl free again
        const int2 kl = tile_kl(t);
        if (kl.y != cur_l) {
            fill_ufl(kl.y);
            cur_l = kl.y;
        }
        const int2 pk = pairs[kl.x], pl = pairs[kl.y];
#pragma unroll
        for (int e = 0; e < PERV; ++e) {
            const int idx = tid + e * NT, sb = idx / VPB, q = idx % VPB;
            const int c = q % b, a0 = (q / b) * VK;
            const int ci = sb >> 1, ri = sb & 1;
            const int C = ci ? pl.y : pl.x, R = ri ? pk.y : pk.x;
            if (C < R) { // stored (C, R): entry (a, c) is X^T(C a, R c)
#pragma unroll
                for (int j = 0; j < VK; ++j)
                    xs[(ci * b + a0 + j) * LDX + ri * b + c] = vlane<T>(cb.xr[e], j);
            } else { // stored (R, C): entry (a, c) is X^T(C c, R a)
                *reinterpret_cast<TV *>(xs + (ci * b + c) * LDX + ri * b + a0) = cb.xr[e];
            }
        }
        lds_barrier();
        // the next tile's loads go out now; their wait in the next step
        // skips this step's stores, which are as many on every path
        load_tile(nb, tn);
        const T *uk = cb.uk;
        accT c1[TC];
#pragma unroll
        for (int tc = 0; tc < TC; ++tc)
#pragma unroll
            for (int v = 0; v < 4; ++v)
                c1[tc][v] = (T)0;
        // LDS operands are read one group ahead of the MFMAs that use them
        auto xs_read = [&](TV(&a)[TC], int g) __attribute__((always_inline)) {
#pragma unroll
            for (int tc = 0; tc < TC; ++tc)
                a[tc] = *reinterpret_cast<const TV *>(xs + (16 * tc + li) * LDX + g * 4 * VK +
                                                      lk * VK);
        };
        TV xa[TC], xb[TC];
        xs_read(xa, 0);
#pragma unroll
        for (int g = 0; g < KG; g += 2) {
            if (g + 1 < KG)
                xs_read(xb, g + 1);
#pragma unroll
            for (int tc = 0; tc < TC; ++tc)
#pragma unroll
                for (int j = 0; j < VK; ++j)
                    c1[tc] = mfma16(vlane<T>(xa[tc], j), uk[g * VK + j], c1[tc]);
            if (g + 1 < KG) {
                if (g + 2 < KG)
                    xs_read(xa, g + 2);
#pragma unroll
                for (int tc = 0; tc < TC; ++tc)
#pragma unroll
                    for (int j = 0; j < VK; ++j)
                        c1[tc] = mfma16(vlane<T>(xb[tc], j), uk[(g + 1) * VK + j], c1[tc]);
            }
        }
        // second product: the four accumulators interleave, U_l fragments of the
        // next tc are read while the current tc multiplies
        accT zt[TJ];
#pragma unroll
        for (int tj = 0; tj < TJ; ++tj)
#pragma unroll
            for (int v = 0; v < 4; ++v)
                zt[tj][v] = (T)0;
        auto uf_read = [&](TV(&u)[TJ][HV], int tc) __attribute__((always_inline)) {
#pragma unroll
            for (int tj = 0; tj < TJ; ++tj)
#pragma unroll
                for (int h = 0; h < HV; ++h)
                    u[tj][h] = *reinterpret_cast<const TV *>(
                        ufl + (((tj * TC + tc) * HV + h) * WAVE + lane) * VK);
        };
        TV ua[TJ][HV], ub[TJ][HV];
        uf_read(ua, 0);
#pragma unroll
        for (int tc = 0; tc < TC; tc += 2) {
            if (tc + 1 < TC)
                uf_read(ub, tc + 1);
#pragma unroll
            for (int v = 0; v < 4; ++v)
#pragma unroll
                for (int tj = 0; tj < TJ; ++tj)
                    zt[tj] = mfma16(vlane<T>(ua[tj][v / VK], v % VK), c1[tc][v], zt[tj]);
            if (tc + 1 < TC) {
                if (tc + 2 < TC)
                    uf_read(ua, tc + 2);
#pragma unroll
                for (int v = 0; v < 4; ++v)
#pragma unroll
                    for (int tj = 0; tj < TJ; ++tj)
                        zt[tj] = mfma16(vlane<T>(ub[tj][v / VK], v % VK), c1[tc + 1][v], zt[tj]);
            }
        }
        // Z goes to the stored block of each (row block, column block): rows
        // along rows with 16-byte stores when the row block is the smaller
        // one, else into the transpose, one element per lane (16 consecutive
        // lanes write consecutive columns).  A wavefront's 16 rows and a
        // 16-column group each lie in one block, so the choice is uniform.
        const int i = 16 * w + li;
        const int gi = pair_col(pk, i, b);
        const int rblk = 16 * w < b ? pk.x : pk.y;
        T *zrow = B + (int64_t)gi * ldb;
        double sq = 0.0;
#pragma unroll
        for (int tj = 0; tj < TJ; ++tj) {
            const int gj0 = pair_col(pl, 16 * tj + 4 * lk, b);
            const int cblk = 16 * tj < b ? pl.x : pl.y;
            T *dst;
            T zv[4];
            if (rblk < cblk) {
                dst = zrow + gj0;
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    zv[v] = store_round<T>(zt[tj][v], r16);
            } else {
                // through the wavefront's LDS scratch: lane (li, lk) then holds
                // four consecutive rows 16 w + 4 lk .. of Z's column 16 tj + li
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    zw[(4 * lk + v) * ZLD + li] = zt[tj][v];
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    zv[v] = store_round<T>(zw[li * ZLD + 4 * lk + v], r16);
                dst = B + (int64_t)pair_col(pl, 16 * tj + li, b) * ldb + pair_col(pk, 16 * w + 4 * lk, b);
            }
            if constexpr (sizeof(T) == 4) {
                const fv4 z = {zv[0], zv[1], zv[2], zv[3]};
                *reinterpret_cast<fv4 *>(dst) = z;
            } else {
                const dv2 z0 = {zv[0], zv[1]}, z1 = {zv[2], zv[3]};
                *reinterpret_cast<dv2 *>(dst) = z0;
                *reinterpret_cast<dv2 *>(dst + 2) = z1;
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const double zq = (double)store_round<T>(zt[tj][v], r16);
                sq += zq * zq;
            }
        }
        if (want_off) {
            sq = wave_sum(sq);
            if (lane == 0)
                partial[(int64_t)t * NW + w] = 2.0 * sq;
        }
    };
    // peeled first step, then pairs of steps, so the two buffers alternate
    // without copies and every path issues the same memory operations (the
    // prefetch after the last tile reads tile 0, which every workgroup reads)
    Buf ba, bb;
    load_tile(ba, t0);
    // the flags are read while the first tile's loads fly
    if (prot != nullptr && !want_off) {
        constexpr int PW = pair_solve_waves(M);
        bool all = true;
        for (int t = t0; t < t1 && all; ++t) {
            const int2 kl = tile_kl(t);
            all = !pair_rotated<PW>(prot, kl.x) && !pair_rotated<PW>(prot, kl.y);
        }
        if (all) {
            if (tid == 0)
                atomicAdd(skipped, t1 - t0);
            return;
        }
    }
    body(t0, ba, bb, t0 + 1 < t1 ? t0 + 1 : 0);
    int t = t0 + 1;
    for (; t + 1 < t1; t += 2) {
        body(t, bb, ba, t + 1);
        body(t + 1, ba, bb, t + 2 < t1 ? t + 2 : 0);
    }
    if (t < t1)
        body(t, bb, ba, 0);
}

int g_update_v_waves = 0; // total resident wavefronts to size the V-update grid; 0 = occupancy

template <typename T, int M>
hipError_t launch_update_v_t(T *V, int64_t ldv, int64_t nrows, int npairs, const int2 *pairs,
                             const T *U, const int *prot, hipStream_t s, hipEvent_t e0,
                             hipEvent_t e1, const Batch &bt)
{
    static int occ_waves = 0;
    if (occ_waves == 0) {
        int dev = 0, cus = 0;
        hipGetDevice(&dev);
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        // one wavefront per SIMD: long runs of tiles per wavefront amortise the
        // U_l load and keep two tiles in flight (measured faster than filling
        // the occupancy at n = 4096)
        occ_waves = (cus > 0 ? cus : 256) * 4;
    }
    const int64_t ntile = nrows / 16;
    const int waves_total = g_update_v_waves > 0 ? g_update_v_waves : occ_waves;
    int64_t chunks = waves_total / ((int64_t)npairs * bt.count);
    if (chunks < 1)
        chunks = 1;
    if (chunks > ntile)
        chunks = ntile;
    const int64_t waves = chunks * npairs;
    const unsigned grid = (unsigned)((waves + 3) / 4);
    constexpr bool CAN_BAT = sizeof(T) == 8; // the batched kernel: FP64 sweeps only
    const bool bt_on = batched(bt);
    if (bt_on && !CAN_BAT)
        return hipErrorInvalidValue;
    launch_timed(bt_on ? update_v_kernel<T, M, CAN_BAT> : update_v_kernel<T, M, false>,
                 dim3(grid, (unsigned)bt.count), dim3(256), 0, s, e0, e1, V, ldv, ntile, pairs,
                 npairs, U, prot, (int)chunks, bt.sW, bt.act);
    return hipGetLastError();
}

template <typename T, int M>
int update_b_blocks_per_cu_t()
{
    static int per = -1;
    if (per < 0) {
        int p = 0;
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&p, update_b_kernel<T, M, false, false>, M * 4, 0);
        per = p > 0 ? p : 1;
    }
    return per;
}

} // namespace

template <typename T>
int update_b_blocks_per_cu(int b)
{
    return b == 32 ? update_b_blocks_per_cu_t<T, 64>() : update_b_blocks_per_cu_t<T, 32>();
}

void tune_update_v(int total_waves) { g_update_v_waves = total_waves; }

template <typename T>
hipError_t launch_update_b(T *B, int64_t ldb, int b, int npairs, const int2 *pairs, const T *U,
                           double *partial, int want_off, int r16, const int *prot, int *skipped,
                           hipStream_t s, hipEvent_t e0, hipEvent_t e1, const Batch &bt)
{
    if (prot && !skipped)
        return hipErrorInvalidValue;
    if (ldb % (16 / (int64_t)sizeof(T)) != 0 || ((uintptr_t)B % 16) != 0)
        return hipErrorInvalidValue;
    const int ntiles = npairs * (npairs - 1) / 2;
    if (ntiles == 0) // one block pair: no tiles; the timing events still mark the spot
        return record_pair(e0, e1, s);
    static int cus = 0;
    if (cus == 0) {
        int dev = 0;
        hipGetDevice(&dev);
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (cus <= 0)
            cus = 256;
    }
    // resident workgroups, shared by the matrices of a batch
    int64_t slots = (int64_t)cus * update_b_blocks_per_cu<T>(b) / bt.count;
    if (slots < 1)
        slots = 1;
    const dim3 grid((unsigned)(ntiles < slots ? ntiles : slots), (unsigned)bt.count);
    const bool h = sizeof(T) == 4 && r16;
    const bool bt_on = batched(bt);
    if (bt_on && sizeof(T) != 8)
        return hipErrorInvalidValue; // the batched kernel: FP64 sweeps only
    constexpr bool CAN_BAT = sizeof(T) == 8;
    if (b == 32)
        launch_timed(bt_on ? update_b_kernel<T, 64, false, CAN_BAT>
                             : (h ? update_b_kernel<T, 64, sizeof(T) == 4, false>
                                  : update_b_kernel<T, 64, false, false>),
                     grid, dim3(256), 0, s, e0, e1, B, ldb, pairs, npairs, U, partial,
                     want_off, prot, skipped, bt.sW, bt.act);
    else if (b == 16)
        launch_timed(bt_on ? update_b_kernel<T, 32, false, CAN_BAT>
                             : (h ? update_b_kernel<T, 32, sizeof(T) == 4, false>
                                  : update_b_kernel<T, 32, false, false>),
                     grid, dim3(128), 0, s, e0, e1, B, ldb, pairs, npairs, U, partial,
                     want_off, prot, skipped, bt.sW, bt.act);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

template <typename T>
hipError_t launch_update_v(T *V, int64_t ldv, int64_t nrows, int b, int npairs,
                           const int2 *pairs, const T *U, const int *prot, hipStream_t s,
                           hipEvent_t e0, hipEvent_t e1, const Batch &bt)
{
    if (nrows % 16 != 0 || ldv % (16 / (int64_t)sizeof(T)) != 0 ||
        ((uintptr_t)V % 16) != 0)
        return hipErrorInvalidValue;
    if (nrows == 0 || npairs == 0)
        return record_pair(e0, e1, s);
    if (b == 32)
        return launch_update_v_t<T, 64>(V, ldv, nrows, npairs, pairs, U, prot, s, e0, e1, bt);
    if (b == 16)
        return launch_update_v_t<T, 32>(V, ldv, nrows, npairs, pairs, U, prot, s, e0, e1, bt);
    return hipErrorInvalidValue;
}

template int update_b_blocks_per_cu<double>(int);
template int update_b_blocks_per_cu<float>(int);
template hipError_t launch_update_b<double>(double *, int64_t, int, int, const int2 *,
                                            const double *, double *, int, int, const int *, int *,
                                            hipStream_t, hipEvent_t, hipEvent_t, const Batch &);
template hipError_t launch_update_b<float>(float *, int64_t, int, int, const int2 *,
                                           const float *, double *, int, int, const int *, int *,
                                           hipStream_t, hipEvent_t, hipEvent_t, const Batch &);
template hipError_t launch_update_v<double>(double *, int64_t, int64_t, int, int, const int2 *,
                                            const double *, const int *, hipStream_t,
                                            hipEvent_t, hipEvent_t, const Batch &);
template hipError_t launch_update_v<float>(float *, int64_t, int64_t, int, int, const int2 *,
                                           const float *, const int *, hipStream_t, hipEvent_t,
                                           hipEvent_t, const Batch &);

} // namespace lj
