// M2L far-field contraction of one octree level (ANKH-FMM, Alg. 3 step 2 in
// its non-mutual form, which also yields the local expansions forces need):
//
//   L_t = sum_{d in IL(t)} K_d M_{(t + d) mod 2^e},
//
// IL(t) = the 189 offsets d with |d|_inf >= 2 whose parent offset lies in
// {-1, 0, 1}^3 (per axis d in [-2, 3] for an even coordinate, [-3, 2] for an
// odd one).  The geometric offset d selects the matrix; the source index wraps
// periodically, so at coarse levels the cells of the adjacent images take
// part as the paper's periodicity section requires.
//
// Per parity class of the target cells the level is one implicit GEMM
//   L[n_u x cells] = [K_d1 .. K_d189] (n_u x 189 n_u) * im2col(M) (189 n_u x cells)
// run on the matrix cores (v_mfma 16x16x4 f64 / f32, or 16x16x32 bf16 in the
// split-precision mode).  A block owns a tile of up to 256 output nodes (all
// n_u of them for the usual orders, so the gathered multipoles are read once
// per tile) x 64 cells (128 on the finest levels in split precision) and a
// slice of the 189 offsets; K_d and the gathered multipoles stream through
// double-buffered LDS.  A coarse level of at most one tile of cells runs as one
// all-cell tile over the union of the eight parity classes' offsets (316 of
// them), multipoles of cells outside a class's list read as zero.  Slices of
// the offset list (split-K) give the launch enough blocks to fill the chip at
// every level; their partial tiles are summed in a fixed order by one
// k_m2l_reduce_levels launch for all split levels, so results do not depend
// on scheduling.
#include <algorithm>
#include <cmath>

#include "ankh_internal.h"

namespace ankh {
namespace {

constexpr int BN = 64;       // cells per block tile: 2 waves x 2 fragments of 16
constexpr int NTHR = 256;

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

template <typename T> struct Mma;
// Operands of both 16x16x4 forms: lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16].  Result element v of lane l sits in column l % 16 and in
// row 4 (l / 16) + v (f32) or row l / 16 + 4 v (f64).
template <> struct Mma<float> {
    using acc = f32x4;
    static __device__ inline acc run(float a, float b, acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ inline int row(int lk, int v) { return 4 * lk + v; }
};
template <> struct Mma<double> {
    using acc = f64x4;
    static __device__ inline acc run(double a, double b, acc c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ inline int row(int lk, int v) { return lk + 4 * v; }
};

// Block order: the 8 XCDs receive blocks round-robin (block id mod 8).  All
// blocks placed on one XCD share one (row tile, offset slice) of K, so each
// slice is fetched from memory once per XCD; the cell tiles and parity
// classes vary fastest.
struct M2LTile {
    int rt, ct, cls, split;
};
__device__ inline M2LTile m2l_tile(int nrt, int nct, int nsplit) {
    const int b = blockIdx.x;
    const int ncc = nct * 8, nrs = nrt * nsplit;
    int rs, cc;
    if ((nrs & 7) == 0) {
        const int xcd = b & 7, local = b >> 3;
        rs = xcd * (nrs >> 3) + local / ncc;
        cc = local % ncc;
    } else {
        rs = b / ncc;
        cc = b % ncc;
    }
    M2LTile t;
    t.rt = rs % nrt;
    t.split = rs / nrt;
    t.ct = cc % nct;
    t.cls = cc / nct;
    return t;
}

// interaction lists of the 8 parity classes (px, py, pz) = (c >> 2, (c >> 1) & 1, c & 1)
// as offset indices, each in a fixed (lexicographic) order
struct ILTable {
    int v[8][kNumIL];
};
constexpr ILTable make_il_table() {
    ILTable t{};
    for (int cls = 0; cls < 8; cls++) {
        const int px = cls >> 2, py = (cls >> 1) & 1, pz = cls & 1;
        int k = 0;
        for (int a = 0; a < 6; a++)
            for (int b = 0; b < 6; b++)
                for (int c = 0; c < 6; c++) {
                    const int dx = (px ? -3 : -2) + a, dy = (py ? -3 : -2) + b, dz = (pz ? -3 : -2) + c;
                    const bool far = dx <= -2 || dx >= 2 || dy <= -2 || dy >= 2 || dz <= -2 || dz >= 2;
                    if (far) t.v[cls][k++] = off_index(dx, dy, dz);
                }
    }
    return t;
}
__constant__ ILTable c_il = make_il_table();

// all 316 offsets d in [-3,3]^3 with |d|_inf >= 2 (the union of the class lists), lexicographic
constexpr int kNumFar = 316;
struct FarTable {
    int v[kNumFar];
};
constexpr FarTable make_far_table() {
    FarTable t{};
    int k = 0;
    for (int dx = -3; dx <= 3; dx++)
        for (int dy = -3; dy <= 3; dy++)
            for (int dz = -3; dz <= 3; dz++)
                if (dx <= -2 || dx >= 2 || dy <= -2 || dy >= 2 || dz <= -2 || dz >= 2) t.v[k++] = off_index(dx, dy, dz);
    return t;
}
__constant__ FarTable c_far = make_far_table();
// offset d is in the interaction list of a cell with coordinate parity p along one axis
__device__ inline bool in_list_1d(int d, int p) { return p ? d <= 2 : d >= -2; }

// leaf-grid coordinates of the source cell of target cell (gx, gy, gz) at offset index di (periodic)
__device__ inline size_t source_cell(int gx, int gy, int gz, int di, int nside) {
    const int dx = di / 49 - 3, dy = (di / 7) % 7 - 3, dz = di % 7 - 3;
    const int sx = (gx + dx + 4 * nside) % nside, sy = (gy + dy + 4 * nside) % nside,
              sz = (gz + dz + 4 * nside) % nside;
    return ((size_t)sx * nside + sy) * nside + sz;
}

// ---- f64 / f32 on the 16x16x4 matrix cores ---------------------------------
// Block tile: 32 RF output nodes x 64 cells; the 4 waves form a 2 x 2 grid of
// 16 RF x 32 sub-tiles.  K is the [d][l][k] stack (contraction index l, output
// node k), so the A tile of one step is BK contiguous runs of rows.  BK = 8
// (f64) or 16 (f32): 64 bytes of contraction per row and step.  Row strides
// of the LDS tiles are BM + 16 and BN + 16 elements, which puts the four
// 16-lane groups of a fragment read on disjoint banks.
template <typename T, int RF, bool ALL>
__global__ __launch_bounds__(256) void k_m2l(const T *__restrict__ K, const T *__restrict__ M, T *__restrict__ part,
                                             double *__restrict__ dst, int nside, int nup, int nsplit,
                                             int64_t part_stride) {
    using Acc = typename Mma<T>::acc;
    constexpr int BM = 32 * RF;
    constexpr int BK = 64 / (int)sizeof(T);
    constexpr int SA = BM + 16, SB = BN + 16;
    __shared__ T As[2][BK][SA];
    __shared__ T Bs[2][BK][SB];

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1;
    const int h = nside >> 1;
    const int nrt = (nup + BM - 1) / BM;
    // block -> (row tile, column tile, parity class, offset slice).  ALL (a coarse level of at most 64
    // cells): the level's cells in natural order in one column tile, contracted over the 316 offsets of
    // the union of the class lists; a cell reads zero multipoles for the offsets outside its own list.
    int rt, ct = 0, cls = 0, split, ncol, nil;
    const int *il;
    if constexpr (ALL) {
        rt = blockIdx.x % nrt;
        split = blockIdx.x / nrt;
        ncol = nside * nside * nside;
        il = c_far.v;
        nil = kNumFar;
    } else {
        ncol = h * h * h;
        const M2LTile tile = m2l_tile(nrt, (ncol + BN - 1) / BN, nsplit);
        rt = tile.rt, ct = tile.ct, cls = tile.cls, split = tile.split;
        il = c_il.v[cls];
        nil = kNumIL;
    }
    const int px = cls >> 2, py = (cls >> 1) & 1, pz = cls & 1;
    const int row0 = rt * BM, col0 = ct * BN;
    // this block's run of the (offset, contraction block) steps: slice `split` of the nil x nk steps
    // (a slice may begin and end inside an offset's blocks)

    // Loaders, unconditional and addressed by 32-bit element offsets (a few instructions per step).
    // A: pairs of adjacent rows, LA pairs per thread; the slots past the tile's NPA pairs repeat pair
    // p - NPA (same data, same LDS place), rows past n_up (a padded row tile) read the last pair of rows,
    // whose products are never written out.
    constexpr int NPA = BK * BM / 2, LA = (NPA + NTHR - 1) / NTHR;
    static_assert(LA * NTHR <= 2 * NPA, "a repeated slot maps onto a real pair");
    int a_off[LA], a_k[LA], a_r[LA];
#pragma unroll
    for (int u = 0; u < LA; u++) {
        const int p0 = tid + NTHR * u, p = p0 < NPA ? p0 : p0 - NPA;
        a_k[u] = p / (BM / 2), a_r[u] = (p % (BM / 2)) * 2;
        a_off[u] = a_k[u] * nup + min(row0 + a_r[u], nup - 2);
    }
    // B: 16 bytes (PB contraction values) of one cell's multipoles per thread; a cell past the level's
    // columns reads the last one (its products are never written out)
    constexpr int PB = 16 / (int)sizeof(T);
    static_assert(BK * BN == PB * NTHR, "B tile must be one 16-byte load per thread");
    const int b_col = tid / (BK / PB), b_k = (tid % (BK / PB)) * PB;
    const int tcell = min(col0 + b_col, ncol - 1);
    int gx, gy, gz;
    if constexpr (ALL) {
        gx = tcell / (nside * nside), gy = (tcell / nside) % nside, gz = tcell % nside;
    } else {
        gx = 2 * (tcell / (h * h)) + px;
        gy = 2 * ((tcell / h) % h) + py;
        gz = 2 * (tcell % h) + pz;
    }
    const int mask = nside - 1;   // the level's side is a power of two

    const int nk = nup / BK;
    const int it0 = (int)((int64_t)nil * nk * split / nsplit), it1 = (int)((int64_t)nil * nk * (split + 1) / nsplit);
    const int niter = it1 - it0;
    T ra[LA][2], rb[PB];
    // step (o, kb): offset il[o], contraction block kb
    auto load = [&](int o, int kb) {
        const int di = il[o], k0 = kb * BK;
        const int dx = di / 49 - 3, dy = (di / 7) % 7 - 3, dz = di % 7 - 3;
        const T *Kd = K + ((size_t)di * nup + k0) * nup;
#pragma unroll
        for (int u = 0; u < LA; u++) {
            ra[u][0] = Kd[a_off[u]];
            ra[u][1] = Kd[a_off[u] + 1];
        }
        const int cell = (((gx + dx) & mask) * nside + ((gy + dy) & mask)) * nside + ((gz + dz) & mask);
        const uint4 v = *reinterpret_cast<const uint4 *>(M + (cell * nup + k0 + b_k));
        const T *pv = reinterpret_cast<const T *>(&v);
        bool use = true;
        if constexpr (ALL)
            use = in_list_1d(dx, gx & 1) && in_list_1d(dy, gy & 1) && in_list_1d(dz, gz & 1);
#pragma unroll
        for (int q = 0; q < PB; q++) rb[q] = use ? pv[q] : (T)0;
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int u = 0; u < LA; u++) {
            As[buf][a_k[u]][a_r[u]] = ra[u][0];
            As[buf][a_k[u]][a_r[u] + 1] = ra[u][1];
        }
#pragma unroll
        for (int q = 0; q < PB; q++) Bs[buf][b_k + q][b_col] = rb[q];
    };

    Acc acc[RF][2];
#pragma unroll
    for (int i = 0; i < RF; i++)
#pragma unroll
        for (int j = 0; j < 2; j++) acc[i][j] = Acc{0, 0, 0, 0};

    int on = it0 / nk, kn = it0 % nk;   // the step loaded next
    if (niter > 0) {
        load(on, kn);
        store(0);
    }
    __syncthreads();
    const int lr = lane & 15, lk = lane >> 4;
    for (int it = 0; it < niter; it++) {
        const int cur = it & 1;
        if (++kn == nk) {
            kn = 0;
            on++;
        }
        if (it + 1 < niter) load(on, kn);
#pragma unroll
        for (int kk = 0; kk < BK; kk += 4) {
            T av[RF], bv[2];
#pragma unroll
            for (int i = 0; i < RF; i++) av[i] = As[cur][kk + lk][wr * 16 * RF + i * 16 + lr];
#pragma unroll
            for (int j = 0; j < 2; j++) bv[j] = Bs[cur][kk + lk][wc * 32 + j * 16 + lr];
#pragma unroll
            for (int i = 0; i < RF; i++)
#pragma unroll
                for (int j = 0; j < 2; j++) acc[i][j] = Mma<T>::run(av[i], bv[j], acc[i][j]);
        }
        if (it + 1 < niter) store(cur ^ 1);
        __syncthreads();
    }

    // scatter each 16 x 16 result block (rows per Mma<T>::row, column lane % 16): split-K, the
    // accumulators as they are (type T) into slice `split` of `part`; else float64 into `dst`
#pragma unroll
    for (int j = 0; j < 2; j++) {
        const int cl = col0 + wc * 32 + j * 16 + lr;
        if (cl >= ncol) continue;
        size_t cell = cl;
        if constexpr (!ALL)
            cell = ((size_t)(2 * (cl / (h * h)) + px) * nside + 2 * ((cl / h) % h) + py) * nside + 2 * (cl % h) + pz;
#pragma unroll
        for (int i = 0; i < RF; i++) {
            const int rb = row0 + wr * 16 * RF + i * 16;   // 16-row block, entirely inside or outside nup
            if (rb >= nup) continue;
            if (nsplit > 1) {
                T *Pc = part + (size_t)split * part_stride + cell * nup + rb;
#pragma unroll
                for (int v = 0; v < 4; v++) Pc[Mma<T>::row(lk, v)] = acc[i][j][v];
            } else {
                double *Lc = dst + cell * nup + rb;
#pragma unroll
                for (int v = 0; v < 4; v++) Lc[Mma<T>::row(lk, v)] = (double)acc[i][j][v];
            }
        }
    }
}

// ---- split-precision variant: BF16 x 3 on the 16x16x32 BF16 matrix cores ------
// Each float32 operand is split as x = hi + lo (hi = bf16(x), lo = bf16(x - hi)),
// and the product is accumulated in float32 as hi*hi + hi*lo + lo*hi (the
// lo*lo term is below the float32 rounding of the sum).  K_d is stored tiled,
// [d][l / 32][k][l % 32], so the A tile of one 32-wide contraction step is one
// contiguous run; the multipoles of all levels are split once per evaluation.
// Lane l of v_mfma_f32_16x16x32_bf16 supplies A[l % 16][8 (l / 16) .. +8] and
// B[8 (l / 16) .. +8][l % 16]; result element v sits at row 4 (l / 16) + v,
// column l % 16.  LDS rows are 32 bf16 (four 16-byte chunks); chunk c of row r
// is stored at chunk position c ^ (((r >> 1) ^ (r >> 3)) & 3).  That spreads
// any 8 consecutive rows (one 128-byte LDS access phase) and any 16
// consecutive rows (one 256-byte phase) of a fragment read over distinct
// banks without padding.
__device__ inline int swz(int r, int c) { return r * 32 + 8 * (c ^ (((r >> 1) ^ (r >> 3)) & 3)); }

// Writes a wave's 16 RF x 16 NB result tile: rows r0 + 16 i + 4 (lane / 16) + v,
// columns (class cells) c0 + 16 j + lane % 16; rows past n_up and cells past the
// class are dropped.  Split-K: float32 into slice `split` of `part`; else float64
// into `dst`.
template <int RF, int NB>
__device__ inline void m2l_write_tile(const f32x4 (&acc)[RF][NB], float *part, double *dst, int split,
                                      int64_t part_stride, int r0, int c0, int lr, int lk, int h, int px, int py,
                                      int pz, int nside, int nup, int nsplit) {
    const int ncls = h * h * h;
#pragma unroll
    for (int j = 0; j < NB; j++) {
        const int cl = c0 + j * 16 + lr;
        if (cl >= ncls) continue;
        const size_t cell = (size_t)((2 * (cl / (h * h)) + px) * nside + 2 * ((cl / h) % h) + py) * nside +
                            2 * (cl % h) + pz;
#pragma unroll
        for (int i = 0; i < RF; i++) {
            const int rb = r0 + i * 16;   // 16-row block, entirely inside or outside n_up
            if (rb >= nup) continue;
            if (nsplit > 1) {
                float *P = part + (size_t)split * part_stride + cell * nup + rb + 4 * lk;
                *reinterpret_cast<f32x4 *>(P) = acc[i][j];
            } else {
                double *Lc = dst + cell * nup + rb + 4 * lk;
#pragma unroll
                for (int v = 0; v < 4; v++) Lc[v] = (double)acc[i][j][v];
            }
        }
    }
}

// Block tile: 32 RF output nodes x 32 NB cells; the 4 waves form a 2 x 2 grid of
// 16 RF x 16 NB sub-tiles, so one step's fragment reads (RF + NB pairs of
// 16-byte loads per lane) feed 3 RF NB products.  The three products of a step
// are issued as three sweeps over the RF x NB accumulators (each accumulator
// still sums lo*hi, hi*lo, hi*hi in that order), so consecutive matrix-core
// instructions never wait on each other's result.  A split-K block writes its
// float32 tile to its slice of `part` (summed by k_m2l_reduce_levels); an
// unsplit level writes float64 to `dst`.
template <int RF, int NB>
__global__ __launch_bounds__(256) void k_m2l_bf16x3(const __bf16 *__restrict__ Kh, const __bf16 *__restrict__ Kl,
                                                    const __bf16 *__restrict__ Mh, const __bf16 *__restrict__ Ml,
                                                    float *__restrict__ part, double *__restrict__ dst, int nside,
                                                    int nup, int nsplit, int64_t part_stride) {
    constexpr int BM = 32 * RF, BN = 32 * NB, BK = 32;
    static_assert(NB % 2 == 0, "one or more whole 16-byte B chunks per thread");
    __shared__ __attribute__((aligned(16))) __bf16 Ash[2][BM * BK];
    __shared__ __attribute__((aligned(16))) __bf16 Asl[2][BM * BK];
    __shared__ __attribute__((aligned(16))) __bf16 Bsh[2][BN * BK];
    __shared__ __attribute__((aligned(16))) __bf16 Bsl[2][BN * BK];

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1;
    const int h = nside >> 1;
    const int ncls = h * h * h;
    const M2LTile tile = m2l_tile((nup + BM - 1) / BM, (ncls + BN - 1) / BN, nsplit);
    const int px = tile.cls >> 2, py = (tile.cls >> 1) & 1, pz = tile.cls & 1;
    const int row0 = tile.rt * BM, col0 = tile.ct * BN;
    const int *il = c_il.v[tile.cls];
    const int o_begin = kNumIL * tile.split / nsplit, o_end = kNumIL * (tile.split + 1) / nsplit;

    // Loaders.  Every load and LDS store is unconditional and addressed by 32-bit
    // element offsets from the operand base, which keeps the per-step address work
    // to a few instructions.  A: 16-byte chunks (8 bf16 of the contraction) of hi and
    // of lo, LA per thread; the thread slots past the tile's NCA chunks repeat chunk
    // p - NCA (same data, same LDS address), and rows past n_up (a padded row tile)
    // load the last row.  B: LB chunks per thread (cell p / 4, chunk p % 4 for
    // p = tid + 256 u); cells past the class load the last cell.  Such rows and
    // cells only reach outputs that are never written.
    constexpr int NCA = BM * 4, LA = (NCA + NTHR - 1) / NTHR;
    static_assert(LA * NTHR <= 2 * NCA, "a repeated slot maps onto a real chunk");
    constexpr int LB = NB / 2;
    int a_off[LA], a_lds[LA], b_lds[LB], bx[LB], by[LB], bz[LB];
#pragma unroll
    for (int u = 0; u < LA; u++) {
        const int p0 = tid + NTHR * u, p = p0 < NCA ? p0 : p0 - NCA;
        a_off[u] = min(row0 + (p >> 2), nup - 1) * BK + 8 * (p & 3);
        a_lds[u] = swz(p >> 2, p & 3);
    }
    const int b_c = tid & 3;
#pragma unroll
    for (int u = 0; u < LB; u++) {
        const int col = (tid + NTHR * u) >> 2, tcell = min(col0 + col, ncls - 1);
        bx[u] = 2 * (tcell / (h * h)) + px;
        by[u] = 2 * ((tcell / h) % h) + py;
        bz[u] = 2 * (tcell % h) + pz;
        b_lds[u] = swz(col, b_c);
    }
    const int mask = nside - 1;   // the level's side is a power of two
    const int nk = nup / BK;
    const int niter = (o_end - o_begin) * nk;
    bf16x8 rah[LA], ral[LA], rbh[LB], rbl[LB];
    // step (o, kb): offset il[o], contraction block kb
    auto load = [&](int o, int kb) {
        const int di = il[o];
        const int dx = di / 49 - 3, dy = (di / 7) % 7 - 3, dz = di % 7 - 3;
        const __bf16 *kh = Kh + ((size_t)di * nk + kb) * nup * BK, *kl = Kl + ((size_t)di * nk + kb) * nup * BK;
#pragma unroll
        for (int u = 0; u < LA; u++) {
            rah[u] = *reinterpret_cast<const bf16x8 *>(kh + a_off[u]);
            ral[u] = *reinterpret_cast<const bf16x8 *>(kl + a_off[u]);
        }
        const int kc = kb * BK + 8 * b_c;
#pragma unroll
        for (int u = 0; u < LB; u++) {
            const int cell = (((bx[u] + dx) & mask) * nside + ((by[u] + dy) & mask)) * nside + ((bz[u] + dz) & mask);
            const int off = cell * nup + kc;
            rbh[u] = *reinterpret_cast<const bf16x8 *>(Mh + off);
            rbl[u] = *reinterpret_cast<const bf16x8 *>(Ml + off);
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int u = 0; u < LA; u++) {
            *reinterpret_cast<bf16x8 *>(&Ash[buf][a_lds[u]]) = rah[u];
            *reinterpret_cast<bf16x8 *>(&Asl[buf][a_lds[u]]) = ral[u];
        }
#pragma unroll
        for (int u = 0; u < LB; u++) {
            *reinterpret_cast<bf16x8 *>(&Bsh[buf][b_lds[u]]) = rbh[u];
            *reinterpret_cast<bf16x8 *>(&Bsl[buf][b_lds[u]]) = rbl[u];
        }
    };

    f32x4 acc[RF][NB];
#pragma unroll
    for (int i = 0; i < RF; i++)
#pragma unroll
        for (int j = 0; j < NB; j++) acc[i][j] = f32x4{0, 0, 0, 0};
    if (niter > 0) {
        load(o_begin, 0);
        store(0);
    }
    __syncthreads();
    const int lr = lane & 15, lk = lane >> 4;
    int on = o_begin, kn = 0;   // the step loaded next
    for (int it = 0; it < niter; it++) {
        const int cur = it & 1;
        if (++kn == nk) {
            kn = 0;
            on++;
        }
        if (it + 1 < niter) load(on, kn);
        bf16x8 ah[RF], al[RF], bh[NB], bl[NB];
#pragma unroll
        for (int i = 0; i < RF; i++) {
            const int r = wr * 16 * RF + i * 16 + lr;
            ah[i] = *reinterpret_cast<const bf16x8 *>(&Ash[cur][swz(r, lk)]);
            al[i] = *reinterpret_cast<const bf16x8 *>(&Asl[cur][swz(r, lk)]);
        }
#pragma unroll
        for (int j = 0; j < NB; j++) {
            const int cl = wc * 16 * NB + j * 16 + lr;
            bh[j] = *reinterpret_cast<const bf16x8 *>(&Bsh[cur][swz(cl, lk)]);
            bl[j] = *reinterpret_cast<const bf16x8 *>(&Bsl[cur][swz(cl, lk)]);
        }
#pragma unroll
        for (int i = 0; i < RF; i++)
#pragma unroll
            for (int j = 0; j < NB; j++)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
#pragma unroll
        for (int i = 0; i < RF; i++)
#pragma unroll
            for (int j = 0; j < NB; j++)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
#pragma unroll
        for (int i = 0; i < RF; i++)
#pragma unroll
            for (int j = 0; j < NB; j++)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
        if (it + 1 < niter) store(cur ^ 1);
        __syncthreads();
    }
    m2l_write_tile<RF, NB>(acc, part, dst, tile.split, part_stride, row0 + wr * 16 * RF, col0 + wc * 16 * NB, lr,
                           lk, h, px, py, pz, nside, nup, nsplit);
}

// ---- coarse levels (at most 64 cells): all cells in one column tile ---------
// The 8 parity classes of a level with <= 8 cells per class would fill only 1 or
// 8 of a tile's 64 columns.  Here the columns are the level's cells in natural
// order and the contraction runs over the union of the class lists (316
// offsets); a cell's column reads zero multipoles for the offsets outside its
// own list, so each cell still sums exactly its 189 terms.  One offset slice
// per block.
template <int RF>
__global__ __launch_bounds__(256) void k_m2l_bf16x3_all(const __bf16 *__restrict__ Kh, const __bf16 *__restrict__ Kl,
                                                        const __bf16 *__restrict__ Mh, const __bf16 *__restrict__ Ml,
                                                        float *__restrict__ part, int nside, int nup, int nsplit,
                                                        int64_t part_stride) {
    constexpr int BM = 32 * RF, BK = 32;
    __shared__ __attribute__((aligned(16))) __bf16 Ash[2][BM * BK];
    __shared__ __attribute__((aligned(16))) __bf16 Asl[2][BM * BK];
    __shared__ __attribute__((aligned(16))) __bf16 Bsh[2][BN * BK];
    __shared__ __attribute__((aligned(16))) __bf16 Bsl[2][BN * BK];

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1;
    const int ncell = nside * nside * nside;
    const int nrt = (nup + BM - 1) / BM;
    const int rt = blockIdx.x % nrt, split = blockIdx.x / nrt;
    const int row0 = rt * BM;
    const int o_begin = kNumFar * split / nsplit, o_end = kNumFar * (split + 1) / nsplit;

    constexpr int NCA = BM * 4, LA = (NCA + NTHR - 1) / NTHR;
    const int b_col = tid >> 2, b_c = tid & 3;
    const bool b_ok = b_col < ncell;
    const int gx = b_ok ? b_col / (nside * nside) : 0, gy = b_ok ? (b_col / nside) % nside : 0,
              gz = b_ok ? b_col % nside : 0;
    const int nk = nup / BK;
    const int niter = (o_end - o_begin) * nk;
    bf16x8 rah[LA], ral[LA], rbh, rbl;
    const bf16x8 zero4 = {};
    auto load = [&](int it) {
        const int di = c_far.v[o_begin + it / nk], kb = it % nk;
        const size_t base = ((size_t)di * nk + kb) * nup * BK;
#pragma unroll
        for (int u = 0; u < LA; u++) {
            const int p = tid + NTHR * u;
            const int r = p >> 2, c = p & 3;
            if (p < NCA && row0 + r < nup) {
                const size_t off = base + (size_t)(row0 + r) * BK + 8 * c;
                rah[u] = *reinterpret_cast<const bf16x8 *>(Kh + off);
                ral[u] = *reinterpret_cast<const bf16x8 *>(Kl + off);
            } else {
                rah[u] = zero4;
                ral[u] = zero4;
            }
        }
        const int dx = di / 49 - 3, dy = (di / 7) % 7 - 3, dz = di % 7 - 3;
        if (b_ok && in_list_1d(dx, gx & 1) && in_list_1d(dy, gy & 1) && in_list_1d(dz, gz & 1)) {
            const size_t off = source_cell(gx, gy, gz, di, nside) * nup + kb * BK + 8 * b_c;
            rbh = *reinterpret_cast<const bf16x8 *>(Mh + off);
            rbl = *reinterpret_cast<const bf16x8 *>(Ml + off);
        } else {
            rbh = zero4;
            rbl = zero4;
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int u = 0; u < LA; u++) {
            const int p = tid + NTHR * u;
            if (p < NCA) {
                const int r = p >> 2, c = p & 3;
                *reinterpret_cast<bf16x8 *>(&Ash[buf][swz(r, c)]) = rah[u];
                *reinterpret_cast<bf16x8 *>(&Asl[buf][swz(r, c)]) = ral[u];
            }
        }
        *reinterpret_cast<bf16x8 *>(&Bsh[buf][swz(b_col, b_c)]) = rbh;
        *reinterpret_cast<bf16x8 *>(&Bsl[buf][swz(b_col, b_c)]) = rbl;
    };

    f32x4 acc[RF][2];
#pragma unroll
    for (int i = 0; i < RF; i++)
#pragma unroll
        for (int j = 0; j < 2; j++) acc[i][j] = f32x4{0, 0, 0, 0};
    if (niter > 0) {
        load(0);
        store(0);
    }
    __syncthreads();
    const int lr = lane & 15, lk = lane >> 4;
    for (int it = 0; it < niter; it++) {
        const int cur = it & 1;
        if (it + 1 < niter) load(it + 1);
        bf16x8 ah[RF], al[RF], bh[2], bl[2];
#pragma unroll
        for (int i = 0; i < RF; i++) {
            const int r = wr * 16 * RF + i * 16 + lr;
            ah[i] = *reinterpret_cast<const bf16x8 *>(&Ash[cur][swz(r, lk)]);
            al[i] = *reinterpret_cast<const bf16x8 *>(&Asl[cur][swz(r, lk)]);
        }
#pragma unroll
        for (int j = 0; j < 2; j++) {
            const int cl = wc * 32 + j * 16 + lr;
            bh[j] = *reinterpret_cast<const bf16x8 *>(&Bsh[cur][swz(cl, lk)]);
            bl[j] = *reinterpret_cast<const bf16x8 *>(&Bsl[cur][swz(cl, lk)]);
        }
#pragma unroll
        for (int i = 0; i < RF; i++)
#pragma unroll
            for (int j = 0; j < 2; j++) {
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
            }
        if (it + 1 < niter) store(cur ^ 1);
        __syncthreads();
    }
    float *o = part + (size_t)split * part_stride;
#pragma unroll
    for (int j = 0; j < 2; j++) {
        const int cl = wc * 32 + j * 16 + lr;
        if (cl >= ncell) continue;
        float *Lc = o + (size_t)cl * nup;
#pragma unroll
        for (int i = 0; i < RF; i++) {
            const int rb = row0 + wr * 16 * RF + i * 16;
            if (rb >= nup) continue;
            *reinterpret_cast<f32x4 *>(Lc + rb + 4 * lk) = acc[i][j];
        }
    }
}

// The source multipoles of several levels in one launch, in the working precision of the
// contraction: level li's n[li] values (packed at off[li] of the launch's range) from src[li] go to
// position dst[li] of the output: bf16 hi / lo parts (via float32), or float32.
struct SplitJob {
    const double *src[kMaxDepth + 1];
    int64_t n[kMaxDepth + 1], off[kMaxDepth + 1], dst[kMaxDepth + 1];
    int nlv;
    int64_t total;
};
__device__ inline int64_t split_job_index(const SplitJob &job, int64_t i, int &li) {
    li = 0;
    while (li + 1 < job.nlv && i >= job.off[li + 1]) li++;
    return i - job.off[li];
}
__global__ void k_split_bf16(SplitJob job, __bf16 *__restrict__ hi, __bf16 *__restrict__ lo) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= job.total) return;
    int li;
    const int64_t k = split_job_index(job, i, li);
    const float x = (float)job.src[li][k];
    const __bf16 a = (__bf16)x;
    hi[job.dst[li] + k] = a;
    lo[job.dst[li] + k] = (__bf16)(x - (float)a);
}
__global__ void k_to_f32_levels(SplitJob job, float *__restrict__ out) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= job.total) return;
    int li;
    const int64_t k = split_job_index(job, i, li);
    out[job.dst[li] + k] = (float)job.src[li][k];
}

// plan time: K_d for the BF16 x 3 kernel from the [d][l][k] float64 stack
// (K_{-d} = K_d^T), tiled as [d][l / 32][k][l % 32]
__global__ void k_split_K_bf16(const double *__restrict__ K, __bf16 *__restrict__ hi, __bf16 *__restrict__ lo,
                               int nup) {
    const int64_t n = (int64_t)kNumOff * nup * nup;
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t per = (int64_t)nup * nup;
    const int d = (int)(i / per);
    const int64_t rem = i % per;
    const int lb = (int)(rem / (32 * (int64_t)nup)), k = (int)((rem / 32) % nup), l = lb * 32 + (int)(rem % 32);
    const float x = (float)K[(int64_t)(kNumOff - 1 - d) * per + (int64_t)k * nup + l];
    const __bf16 a = (__bf16)x;
    hi[i] = a;
    lo[i] = (__bf16)(x - (float)a);
}

// The reductions of all split levels in one launch, after the last contraction: L = sum over the
// level's partial tiles (float64, or the float32 accumulator tiles of the mixed modes, added in
// float64) in a fixed order.  Level li's blocks start at block blk0[li]; a block is nr[li] runs x
// (256 / nr[li]) elements (16 runs for the many-slice coarse levels, 4 otherwise): slice k goes to run
// k mod nr, each run adds its slices in slice order, then the runs are added in run order.
template <typename P>
struct ReduceJob {
    const P *part[kMaxDepth + 1];
    double *L[kMaxDepth + 1];
    int64_t n[kMaxDepth + 1], blk0[kMaxDepth + 1];
    int nsplit[kMaxDepth + 1], nr[kMaxDepth + 1];
    int nlv;
};
template <typename P>
__global__ __launch_bounds__(256) void k_m2l_reduce_levels(ReduceJob<P> job) {
    __shared__ double red[256];
    int li = 0;
    while (li + 1 < job.nlv && (int64_t)blockIdx.x >= job.blk0[li + 1]) li++;
    const P *part = job.part[li];
    const int64_t n = job.n[li];
    const int nsplit = job.nsplit[li], NR = job.nr[li], NE = 256 / NR;
    const int w = threadIdx.x / NE, r = threadIdx.x % NE;
    const int64_t i = ((int64_t)blockIdx.x - job.blk0[li]) * NE + r;
    double s = 0;
    if (i < n) {
        int k = w;
        for (; k + 3 * NR < nsplit; k += 4 * NR) {   // four loads in flight, added in slice order
            const double a0 = part[k * n + i], a1 = part[(k + NR) * n + i], a2 = part[(k + 2 * NR) * n + i],
                         a3 = part[(k + 3 * NR) * n + i];
            s += a0;
            s += a1;
            s += a2;
            s += a3;
        }
        for (; k < nsplit; k += NR) s += (double)part[k * n + i];
    }
    red[threadIdx.x] = s;
    __syncthreads();
    if (w == 0 && i < n) {
        double t = red[r];
        for (int k = 1; k < NR; k++) t += red[k * NE + r];
        job.L[li][i] = t;
    }
}

}  // namespace

hipError_t launch_split_K_bf16(ankh_plan_s *pl, const double *K, __bf16 *hi, __bf16 *lo, int nr) {
    const int64_t n = (int64_t)kNumOff * nr * nr;
    hipLaunchKernelGGL(k_split_K_bf16, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, pl->stream, K, hi, lo, nr);
    return hipGetLastError();
}

// Rows of the output block tile, 32 RF with RF in 2..8: the height that pads
// the operand size n (n_up, or the padded rank of a compressed level) least,
// the taller one on ties.
int m2l_row_frags(int n) {
    int best = 2;
    int64_t best_pad = INT64_MAX;
    for (int rf : {8, 7, 6, 5, 4, 3, 2}) {
        const int bm = 32 * rf;
        const int64_t pad = (int64_t)((n + bm - 1) / bm) * bm;
        if (pad < best_pad) {
            best_pad = pad;
            best = rf;
        }
    }
    return best;
}

// Coarse levels (at most 64 cells) run all cells in one column tile over the 316 offsets.
bool m2l_all_cells(const ankh_plan_s *pl, int e) { return pl->lv[e].ncell <= BN; }

// Columns of the block tile, 32 NB cells.  The split-precision kernel takes 128
// cells (NB = 4) where a parity class has at least 128 cells and the row tile is
// at most 160 nodes (taller tiles would not fit two waves per SIMD); everything
// else takes 64 (128-cell tiles were slower in float32: 459 against 442 us on
// the finest level of the 288k box).
int m2l_col_frags(const ankh_plan_s *pl, int e) {
    const int h = pl->lv[e].nside / 2;
    const bool wide = pl->precision == ANKH_MIXED_BF16X3 && !m2l_all_cells(pl, e) && h * h * h >= 128 &&
                      m2l_row_frags(pl->rpad[e]) <= 5;
    return wide ? 4 : 2;
}

// bytes per partial value: the float32 accumulators of the mixed modes, float64 in FP64
static size_t m2l_part_elem(const ankh_plan_s *pl) {
    return pl->precision == ANKH_FP64 ? sizeof(double) : sizeof(float);
}

// Number of offset slices (split-K).  A multiple of 8 (the XCD-aware block order then gives
// every XCD whole slices), raised until the level launches >= 512 blocks (split bf16) or
// >= 1024 (the float32 / float64 kernels), while the level's partial tiles stay within
// 64 MiB and every slice keeps at least one offset; a level with twice that many block
// tiles runs unsplit.
int m2l_splits(const ankh_plan_s *pl, int e) {
    // coarse levels: one offset per slice (two per offset in float32, 632 slices, gained nothing in
    // the contraction and cost 5 us in the reduction)
    if (m2l_all_cells(pl, e)) return kNumFar;
    const int h = pl->lv[e].nside / 2;
    const int n = pl->rpad[e];
    const int bm = 32 * m2l_row_frags(n), bn = 32 * m2l_col_frags(pl, e);
    const int64_t tiles = (int64_t)((n + bm - 1) / bm) * ((h * h * h + bn - 1) / bn) * 8;
    const int64_t ncell = pl->lv[e].ncell;
    const int64_t want = pl->precision == ANKH_MIXED_BF16X3 ? 512 : 1024;
    if (tiles >= 2 * want) return 1;
    const int64_t elem = (int64_t)m2l_part_elem(pl);
    int s = 8;
    while (tiles * s < want && (s + 8) * ncell * n * elem <= ((int64_t)64 << 20) && s + 8 <= kNumIL) s += 8;
    return s;
}

// Bytes of the split-K partial tiles of level e (0 when it runs unsplit).
size_t m2l_part_bytes(const ankh_plan_s *pl, int e) {
    const int sp = m2l_splits(pl, e);
    if (sp <= 1) return 0;
    const size_t nv = (size_t)pl->lv[e].ncell * pl->rpad[e];
    return sp * nv * m2l_part_elem(pl);
}

// Mixed modes, once per evaluation before the contractions: every level's source multipoles
// in the contraction's working precision, at offset mb_off[e] (split bf16: d_Mb hi parts,
// then the lo parts at + mb_total; float32: d_Mf).  The projection of the compressed levels
// writes theirs; this converts the uncompressed ones (one launch, packed).
hipError_t launch_m2l_prepare(ankh_plan_s *pl) {
    if (pl->precision == ANKH_FP64 || pl->depth < 1) return hipSuccess;
    SplitJob job{};
    int64_t total = 0;
    for (int e = 1; e <= pl->depth; e++) {
        if (pl->rpad[e] < pl->nup) continue;
        job.src[job.nlv] = pl->d_M + pl->lv[e].cell0 * pl->nup;
        job.n[job.nlv] = pl->lv[e].ncell * pl->rpad[e];
        job.off[job.nlv] = total;
        job.dst[job.nlv] = (int64_t)pl->mb_off[e];
        total += job.n[job.nlv];
        job.nlv++;
    }
    if (total == 0) return hipSuccess;
    job.total = total;
    const dim3 g((unsigned)((total + 255) / 256));
    if (pl->precision == ANKH_MIXED_BF16X3)
        hipLaunchKernelGGL(k_split_bf16, g, dim3(256), 0, pl->stream, job, pl->d_Mb, pl->d_Mb + pl->mb_total);
    else
        hipLaunchKernelGGL(k_to_f32_levels, g, dim3(256), 0, pl->stream, job, pl->d_Mf);
    return hipGetLastError();
}

namespace {
// one level's contraction: operand size n (rows and contraction per offset), source
// multipoles M [cells][n] (float64), K stack of the level at its slot
template <int RF>
void launch_rf(ankh_plan_s *pl, int e, dim3 grid, int n, const double *Msrc, double *Ldst, int nsplit,
               int64_t nval) {
    const ankh::Level &lv = pl->lv[e];
    const size_t kper = (size_t)kNumOff * pl->nup * pl->nup;
    const size_t koff = (size_t)(e - 1) * kper;
    const bool all = m2l_all_cells(pl, e);
    char *part = reinterpret_cast<char *>(pl->d_m2l_part) + pl->m2l_part_off[e];
    if (pl->precision == ANKH_MIXED_BF16X3) {
        const __bf16 *Mh = pl->d_Mb + pl->mb_off[e], *Ml = pl->d_Mb + pl->mb_total + pl->mb_off[e];
        const size_t kall = (size_t)pl->depth * kper;
        float *pf = reinterpret_cast<float *>(part);
        if (all)
            hipLaunchKernelGGL(k_m2l_bf16x3_all<RF>, grid, dim3(NTHR), 0, pl->stream, pl->d_Kb + koff,
                               pl->d_Kb + kall + koff, Mh, Ml, pf, lv.nside, n, nsplit, nval);
        else if (m2l_col_frags(pl, e) == 4) {
            if constexpr (RF <= 5)
                hipLaunchKernelGGL((k_m2l_bf16x3<RF, 4>), grid, dim3(NTHR), 0, pl->stream, pl->d_Kb + koff,
                                   pl->d_Kb + kall + koff, Mh, Ml, pf, Ldst, lv.nside, n, nsplit, nval);
        } else
            hipLaunchKernelGGL((k_m2l_bf16x3<RF, 2>), grid, dim3(NTHR), 0, pl->stream, pl->d_Kb + koff,
                               pl->d_Kb + kall + koff, Mh, Ml, pf, Ldst, lv.nside, n, nsplit, nval);
    } else if (pl->precision == ANKH_MIXED) {
        const float *Mf = pl->d_Mf + pl->mb_off[e];
        float *pf = reinterpret_cast<float *>(part);
        if (all)
            hipLaunchKernelGGL((k_m2l<float, RF, true>), grid, dim3(NTHR), 0, pl->stream, pl->d_Kf + koff, Mf, pf,
                               Ldst, lv.nside, n, nsplit, nval);
        else
            hipLaunchKernelGGL((k_m2l<float, RF, false>), grid, dim3(NTHR), 0, pl->stream, pl->d_Kf + koff, Mf, pf,
                               Ldst, lv.nside, n, nsplit, nval);
    } else {
        double *pd = reinterpret_cast<double *>(part);
        if (all)
            hipLaunchKernelGGL((k_m2l<double, RF, true>), grid, dim3(NTHR), 0, pl->stream, pl->d_K + koff, Msrc,
                               pd, Ldst, lv.nside, n, nsplit, nval);
        else
            hipLaunchKernelGGL((k_m2l<double, RF, false>), grid, dim3(NTHR), 0, pl->stream, pl->d_K + koff, Msrc,
                               pd, Ldst, lv.nside, n, nsplit, nval);
    }
}

template <typename P>
hipError_t reduce_levels(ankh_plan_s *pl) {
    ReduceJob<P> job{};
    int64_t blocks = 0;
    for (int e = 1; e <= pl->depth; e++) {
        const int nsplit = m2l_splits(pl, e);
        if (nsplit <= 1) continue;
        const ankh::Level &lv = pl->lv[e];
        const int n = pl->rpad[e];
        job.part[job.nlv] = reinterpret_cast<const P *>(reinterpret_cast<const char *>(pl->d_m2l_part) +
                                                        pl->m2l_part_off[e]);
        job.L[job.nlv] = n < pl->nup ? pl->d_Lc + pl->c_off[e] : pl->d_L + lv.cell0 * pl->nup;
        job.n[job.nlv] = lv.ncell * n;
        job.nsplit[job.nlv] = nsplit;
        job.nr[job.nlv] = nsplit > 64 ? 16 : 4;
        job.blk0[job.nlv] = blocks;
        const int ne = 256 / job.nr[job.nlv];
        blocks += (job.n[job.nlv] + ne - 1) / ne;
        job.nlv++;
    }
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_m2l_reduce_levels<P>, dim3((unsigned)blocks), dim3(256), 0, pl->stream, job);
    return hipGetLastError();
}
}  // namespace

hipError_t launch_m2l(ankh_plan_s *pl, int e) {
    const ankh::Level &lv = pl->lv[e];
    const int h = lv.nside / 2;
    const int ncls = h * h * h;
    const int n = pl->rpad[e];
    const bool comp = n < pl->nup;
    const bool all = m2l_all_cells(pl, e);
    const int nsplit = m2l_splits(pl, e);
    const int rf = all ? 2 : m2l_row_frags(n);   // coarse levels: 64-row tiles, more blocks for the operator stream
    const int bm = 32 * rf, bn = 32 * m2l_col_frags(pl, e);
    const int nrt = (n + bm - 1) / bm;
    const dim3 grid((unsigned)(all ? nrt * nsplit : nrt * ((ncls + bn - 1) / bn) * 8 * nsplit));
    const int64_t nval = lv.ncell * n;
    double *L = pl->d_L + lv.cell0 * pl->nup;
    const double *M = pl->d_M + lv.cell0 * pl->nup;
    // compressed levels contract in the rank-n basis: M' = M U (projected for all
    // levels before the first contraction), L = L' U^T (after the last)
    const double *Msrc = comp ? pl->d_Mc + pl->c_off[e] : M;
    double *Ldst = comp ? pl->d_Lc + pl->c_off[e] : L;
    switch (rf) {
        case 2: launch_rf<2>(pl, e, grid, n, Msrc, Ldst, nsplit, nval); break;
        case 3: launch_rf<3>(pl, e, grid, n, Msrc, Ldst, nsplit, nval); break;
        case 4: launch_rf<4>(pl, e, grid, n, Msrc, Ldst, nsplit, nval); break;
        case 5: launch_rf<5>(pl, e, grid, n, Msrc, Ldst, nsplit, nval); break;
        case 6: launch_rf<6>(pl, e, grid, n, Msrc, Ldst, nsplit, nval); break;
        case 7: launch_rf<7>(pl, e, grid, n, Msrc, Ldst, nsplit, nval); break;
        default: launch_rf<8>(pl, e, grid, n, Msrc, Ldst, nsplit, nval); break;
    }
    return hipGetLastError();
}

// After the last contraction: the partial tiles of every split level (each level has its
// own region) summed into its local expansions, one launch.
hipError_t launch_m2l_finish(ankh_plan_s *pl) {
    if (pl->depth < 1) return hipSuccess;
    return pl->precision == ANKH_FP64 ? reduce_levels<double>(pl) : reduce_levels<float>(pl);
}

}  // namespace ankh
