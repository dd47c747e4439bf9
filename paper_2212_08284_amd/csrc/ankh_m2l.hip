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
// per tile) x 64 cells and a slice of the 189 offsets; K_d and the gathered
// multipoles stream through double-buffered LDS.  Slices of the offset list
// (split-K) give the launch enough blocks to fill the chip at every level;
// their partial tiles are summed in a fixed order by k_m2l_reduce, so results
// do not depend on scheduling.
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
template <typename T, int RF>
__global__ __launch_bounds__(256) void k_m2l(const T *__restrict__ K, const T *__restrict__ M,
                                             double *__restrict__ out, int nside, int nup, int nsplit,
                                             int64_t out_stride) {
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
    const int ncls = h * h * h;
    const M2LTile tile = m2l_tile((nup + BM - 1) / BM, (ncls + BN - 1) / BN, nsplit);
    const int px = tile.cls >> 2, py = (tile.cls >> 1) & 1, pz = tile.cls & 1;
    const int row0 = tile.rt * BM, col0 = tile.ct * BN;
    const int *il = c_il.v[tile.cls];
    const int o_begin = kNumIL * tile.split / nsplit, o_end = kNumIL * (tile.split + 1) / nsplit;

    // A loader: pairs of adjacent rows; LA pairs per thread
    constexpr int NPA = BK * BM / 2, LA = (NPA + NTHR - 1) / NTHR;
    // B loader: 16 bytes (PB contraction values) of one cell's multipoles per thread
    constexpr int PB = 16 / (int)sizeof(T);
    static_assert(BK * BN == PB * NTHR, "B tile must be one 16-byte load per thread");
    const int b_col = tid / (BK / PB), b_k = (tid % (BK / PB)) * PB;
    const int tcell = col0 + b_col;
    const bool b_ok = tcell < ncls;
    int gx = 0, gy = 0, gz = 0;
    if (b_ok) {
        gx = 2 * (tcell / (h * h)) + px;
        gy = 2 * ((tcell / h) % h) + py;
        gz = 2 * (tcell % h) + pz;
    }

    const int nk = nup / BK;
    const int niter = (o_end - o_begin) * nk;
    T ra[LA][2], rb[PB];
    auto load = [&](int it) {
        const int di = il[o_begin + it / nk], k0 = (it % nk) * BK;
        const T *Kd = K + (size_t)di * nup * nup + (size_t)k0 * nup + row0;
#pragma unroll
        for (int u = 0; u < LA; u++) {
            const int p = tid + NTHR * u;
            const int k = p / (BM / 2), r = (p % (BM / 2)) * 2;
            if (p < NPA && row0 + r < nup) {
                const T *src = Kd + (size_t)k * nup + r;
                ra[u][0] = src[0];
                ra[u][1] = src[1];
            } else {
                ra[u][0] = (T)0;
                ra[u][1] = (T)0;
            }
        }
        if (b_ok) {
            const T *src = M + source_cell(gx, gy, gz, di, nside) * nup + k0 + b_k;
            const uint4 v = *reinterpret_cast<const uint4 *>(src);
            const T *pv = reinterpret_cast<const T *>(&v);
#pragma unroll
            for (int u = 0; u < PB; u++) rb[u] = pv[u];
        } else {
#pragma unroll
            for (int u = 0; u < PB; u++) rb[u] = (T)0;
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int u = 0; u < LA; u++) {
            const int p = tid + NTHR * u;
            if (p < NPA) {
                const int k = p / (BM / 2), r = (p % (BM / 2)) * 2;
                As[buf][k][r] = ra[u][0];
                As[buf][k][r + 1] = ra[u][1];
            }
        }
#pragma unroll
        for (int u = 0; u < PB; u++) Bs[buf][b_k + u][b_col] = rb[u];
    };

    Acc acc[RF][2];
#pragma unroll
    for (int i = 0; i < RF; i++)
#pragma unroll
        for (int j = 0; j < 2; j++) acc[i][j] = Acc{0, 0, 0, 0};

    if (niter > 0) {
        load(0);
        store(0);
    }
    __syncthreads();
    const int lr = lane & 15, lk = lane >> 4;
    for (int it = 0; it < niter; it++) {
        const int cur = it & 1;
        if (it + 1 < niter) load(it + 1);
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

    // scatter each 16 x 16 result block (rows per Mma<T>::row, column lane % 16)
    double *o = out + (size_t)tile.split * out_stride;
#pragma unroll
    for (int j = 0; j < 2; j++) {
        const int cl = col0 + wc * 32 + j * 16 + lr;
        if (cl >= ncls) continue;
        const int cx = 2 * (cl / (h * h)) + px, cy = 2 * ((cl / h) % h) + py, cz = 2 * (cl % h) + pz;
        double *Lc = o + ((size_t)(cx * nside + cy) * nside + cz) * nup;
#pragma unroll
        for (int i = 0; i < RF; i++) {
            const int rb = row0 + wr * 16 * RF + i * 16;   // 16-row block, entirely inside or outside nup
            if (rb >= nup) continue;
#pragma unroll
            for (int v = 0; v < 4; v++) Lc[rb + Mma<T>::row(lk, v)] = (double)acc[i][j][v];
        }
    }
}

// ---- split-precision variant: BF16 x 3 on the 16x16x32 BF16 matrix cores ------
// Each float32 operand is split as x = hi + lo (hi = bf16(x), lo = bf16(x - hi)),
// and the product is accumulated in float32 as hi*hi + hi*lo + lo*hi (the
// lo*lo term is below the float32 rounding of the sum).  K_d is stored tiled,
// [d][l / 32][k][l % 32], so the A tile of one 32-wide contraction step is one
// contiguous run; the multipoles of the level are split once per launch.
// Lane l of v_mfma_f32_16x16x32_bf16 supplies A[l % 16][8 (l / 16) .. +8] and
// B[8 (l / 16) .. +8][l % 16]; result element v sits at row 4 (l / 16) + v,
// column l % 16.  LDS rows are 32 bf16 (four 16-byte chunks); chunk c of row r
// is stored at chunk position c ^ (((r >> 1) ^ (r >> 3)) & 3).  That spreads
// any 8 consecutive rows (one 128-byte LDS access phase) and any 16
// consecutive rows (one 256-byte phase) of a fragment read over distinct
// banks without padding.
__device__ inline int swz(int r, int c) { return r * 32 + 8 * (c ^ (((r >> 1) ^ (r >> 3)) & 3)); }

template <int RF>
__global__ __launch_bounds__(256) void k_m2l_bf16x3(const __bf16 *__restrict__ Kh, const __bf16 *__restrict__ Kl,
                                                    const __bf16 *__restrict__ Mh, const __bf16 *__restrict__ Ml,
                                                    double *__restrict__ out, int nside, int nup, int nsplit,
                                                    int64_t out_stride) {
    constexpr int BM = 32 * RF, BK = 32;
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

    // A loader: 16-byte chunks (8 bf16 of the contraction) of hi and of lo, LA per thread
    constexpr int NCA = BM * 4, LA = (NCA + NTHR - 1) / NTHR;
    // B loader: one chunk of hi and of lo per thread
    const int b_col = tid >> 2, b_c = tid & 3;
    const int tcell = col0 + b_col;
    const bool b_ok = tcell < ncls;
    int gx = 0, gy = 0, gz = 0;
    if (b_ok) {
        gx = 2 * (tcell / (h * h)) + px;
        gy = 2 * ((tcell / h) % h) + py;
        gz = 2 * (tcell % h) + pz;
    }
    const int nk = nup / BK;
    const int niter = (o_end - o_begin) * nk;
    bf16x8 rah[LA], ral[LA], rbh, rbl;
    const bf16x8 zero4 = {};
    auto load = [&](int it) {
        const int di = il[o_begin + it / nk], kb = it % nk;
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
        if (b_ok) {
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
    double *o = out + (size_t)tile.split * out_stride;
#pragma unroll
    for (int j = 0; j < 2; j++) {
        const int cl = col0 + wc * 32 + j * 16 + lr;
        if (cl >= ncls) continue;
        const int cx = 2 * (cl / (h * h)) + px, cy = 2 * ((cl / h) % h) + py, cz = 2 * (cl % h) + pz;
        double *Lc = o + ((size_t)(cx * nside + cy) * nside + cz) * nup;
#pragma unroll
        for (int i = 0; i < RF; i++) {
            const int rb = row0 + wr * 16 * RF + i * 16;
            if (rb >= nup) continue;
#pragma unroll
            for (int v = 0; v < 4; v++) Lc[rb + 4 * lk + v] = (double)acc[i][j][v];
        }
    }
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
                                                        double *__restrict__ out, int nside, int nup, int nsplit,
                                                        int64_t out_stride) {
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
    double *o = out + (size_t)split * out_stride;
#pragma unroll
    for (int j = 0; j < 2; j++) {
        const int cl = wc * 32 + j * 16 + lr;
        if (cl >= ncell) continue;
        double *Lc = o + (size_t)cl * nup;
#pragma unroll
        for (int i = 0; i < RF; i++) {
            const int rb = row0 + wr * 16 * RF + i * 16;
            if (rb >= nup) continue;
#pragma unroll
            for (int v = 0; v < 4; v++) Lc[rb + 4 * lk + v] = (double)acc[i][j][v];
        }
    }
}

// hi / lo bf16 split of a float64 array (via float32)
__global__ void k_split_bf16(const double *__restrict__ s, __bf16 *__restrict__ hi, __bf16 *__restrict__ lo,
                             int64_t n) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float x = (float)s[i];
    const __bf16 a = (__bf16)x;
    hi[i] = a;
    lo[i] = (__bf16)(x - (float)a);
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

// L = sum over the split-K partials in a fixed order: NR interleaved runs of
// the slices (slice k in run k mod NR), each added in slice order, then the
// NR run sums in run order.  256 threads = NR runs x (256 / NR) elements.
template <int NR>
__global__ __launch_bounds__(256) void k_m2l_reduce(const double *__restrict__ part, double *__restrict__ L,
                                                    int64_t n, int nsplit) {
    constexpr int NE = 256 / NR;
    __shared__ double red[NR][NE];
    const int w = threadIdx.x / NE, r = threadIdx.x % NE;
    const int64_t i = blockIdx.x * (int64_t)NE + r;
    double s = 0;
    if (i < n)
        for (int k = w; k < nsplit; k += NR) s += part[k * n + i];
    red[w][r] = s;
    __syncthreads();
    if (w == 0 && i < n) {
        double t = red[0][r];
        for (int k = 1; k < NR; k++) t += red[k][r];
        L[i] = t;
    }
}

__global__ void k_f64_to_f32(const double *__restrict__ s, float *__restrict__ d, int64_t n) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) d[i] = (float)s[i];
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

// Coarse levels of the split-precision mode (at most 64 cells) run all cells in
// one column tile over the 316 offsets, one offset per slice.
bool m2l_all_cells(const ankh_plan_s *pl, int e) {
    return pl->precision == ANKH_MIXED_BF16X3 && pl->lv[e].ncell <= BN;
}

// Number of offset slices (split-K).  A level with >= 2048 block tiles runs
// unsplit.  Otherwise a multiple of 8 (the XCD-aware block order then gives
// every XCD whole slices), raised until the level launches >= 1024 blocks,
// while the partial tiles stay within 32768 cells x 224 values and every slice
// keeps at least one offset.
int m2l_splits(const ankh_plan_s *pl, int e) {
    const int h = pl->lv[e].nside / 2;
    const int n = pl->rpad[e];
    const int bm = 32 * m2l_row_frags(n);
    const int64_t tiles = (int64_t)((n + bm - 1) / bm) * ((h * h * h + BN - 1) / BN) * 8;
    const int64_t ncell = pl->lv[e].ncell;
    if (m2l_all_cells(pl, e)) return kNumFar;
    if (tiles >= 2048) return 1;
    int s = 8;
    while (tiles * s < 1024 && (s + 8) * ncell * n <= (int64_t)32768 * 224 && s + 8 <= kNumIL) s += 8;
    return s;
}

namespace {
// one level's contraction: operand size n (rows and contraction per offset), source
// multipoles M [cells][n] (float64), K stack of the level at its slot
template <int RF>
void launch_rf(ankh_plan_s *pl, int e, dim3 grid, int n, const double *Msrc, double *out, int nsplit,
               int64_t nval) {
    const ankh::Level &lv = pl->lv[e];
    const size_t kper = (size_t)kNumOff * pl->nup * pl->nup;
    const size_t koff = (size_t)(e - 1) * kper;
    if (pl->precision == ANKH_MIXED_BF16X3) {
        const __bf16 *Mh = pl->d_Mb, *Ml = pl->d_Mb + nval;
        const size_t kall = (size_t)pl->depth * kper;
        if (m2l_all_cells(pl, e))
            hipLaunchKernelGGL(k_m2l_bf16x3_all<RF>, dim3((unsigned)(((n + 32 * RF - 1) / (32 * RF)) * nsplit)),
                               dim3(NTHR), 0, pl->stream, pl->d_Kb + koff, pl->d_Kb + kall + koff, Mh, Ml, out,
                               lv.nside, n, nsplit, nval);
        else
            hipLaunchKernelGGL(k_m2l_bf16x3<RF>, grid, dim3(NTHR), 0, pl->stream, pl->d_Kb + koff,
                               pl->d_Kb + kall + koff, Mh, Ml, out, lv.nside, n, nsplit, nval);
    } else if (pl->precision == ANKH_MIXED) {
        hipLaunchKernelGGL((k_m2l<float, RF>), grid, dim3(NTHR), 0, pl->stream, pl->d_Kf + koff, pl->d_Mf, out,
                           lv.nside, n, nsplit, nval);
    } else {
        hipLaunchKernelGGL((k_m2l<double, RF>), grid, dim3(NTHR), 0, pl->stream, pl->d_K + koff, Msrc, out,
                           lv.nside, n, nsplit, nval);
    }
}
}  // namespace

hipError_t launch_m2l(ankh_plan_s *pl, int e) {
    const ankh::Level &lv = pl->lv[e];
    const int h = lv.nside / 2;
    const int ncls = h * h * h;
    const int n = pl->rpad[e];
    const bool comp = n < pl->nup;
    const int nsplit = m2l_splits(pl, e);
    const int rf = m2l_row_frags(n);
    const int bm = 32 * rf;
    dim3 grid((unsigned)(((n + bm - 1) / bm) * ((ncls + BN - 1) / BN) * 8 * nsplit));
    const int64_t nval = lv.ncell * n;
    double *L = pl->d_L + lv.cell0 * pl->nup;
    const double *M = pl->d_M + lv.cell0 * pl->nup;
    // compressed levels contract in the rank-n basis: M' = M U (projected for all
    // levels before the first contraction), L = L' U^T (after the last)
    double *Msrc = comp ? pl->d_Mc + pl->c_off[e] : const_cast<double *>(M);
    double *Ldst = comp ? pl->d_Lc + pl->c_off[e] : L;
    double *out = nsplit > 1 ? pl->d_m2l_part : Ldst;
    // this level's multipoles in the working precision of the contraction
    if (pl->precision == ANKH_MIXED_BF16X3)
        hipLaunchKernelGGL(k_split_bf16, dim3((unsigned)((nval + 255) / 256)), dim3(256), 0, pl->stream, Msrc,
                           pl->d_Mb, pl->d_Mb + nval, nval);
    else if (pl->precision == ANKH_MIXED)
        hipLaunchKernelGGL(k_f64_to_f32, dim3((unsigned)((nval + 255) / 256)), dim3(256), 0, pl->stream, Msrc,
                           pl->d_Mf, nval);
    switch (rf) {
        case 2: launch_rf<2>(pl, e, grid, n, Msrc, out, nsplit, nval); break;
        case 3: launch_rf<3>(pl, e, grid, n, Msrc, out, nsplit, nval); break;
        case 4: launch_rf<4>(pl, e, grid, n, Msrc, out, nsplit, nval); break;
        case 5: launch_rf<5>(pl, e, grid, n, Msrc, out, nsplit, nval); break;
        case 6: launch_rf<6>(pl, e, grid, n, Msrc, out, nsplit, nval); break;
        case 7: launch_rf<7>(pl, e, grid, n, Msrc, out, nsplit, nval); break;
        default: launch_rf<8>(pl, e, grid, n, Msrc, out, nsplit, nval); break;
    }
    if (nsplit > 64)
        hipLaunchKernelGGL(k_m2l_reduce<16>, dim3((unsigned)((nval + 15) / 16)), dim3(256), 0, pl->stream,
                           pl->d_m2l_part, Ldst, nval, nsplit);
    else if (nsplit > 1)
        hipLaunchKernelGGL(k_m2l_reduce<4>, dim3((unsigned)((nval + 63) / 64)), dim3(256), 0, pl->stream,
                           pl->d_m2l_part, Ldst, nval, nsplit);
    return hipGetLastError();
}

}  // namespace ankh
