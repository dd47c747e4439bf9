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
// run on the matrix cores (v_mfma 16x16x4, f64 or f32).  A block owns a
// 64 (nodes) x 64 (cells) tile of L and a slice of the 189 offsets; K_d and
// the gathered multipoles stream through double-buffered LDS in steps of 16
// along the contraction.  Slices of the offset list (split-K) give the launch
// enough blocks to fill the chip at every level; their partial tiles are
// summed in a fixed order by k_m2l_reduce, so results do not depend on
// scheduling.
#include <algorithm>
#include <cmath>

#include "ankh_internal.h"

namespace ankh {
namespace {

constexpr int BM = 64, BN = 64, BK = 16;

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

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
// blocks placed on one XCD share one (row tile, offset slice) of K, small
// enough for that XCD's L2, so each slice is fetched from memory once; the
// cell tiles and parity classes vary fastest.
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

// one block per (row tile, cell tile, parity class, offset slice), ordered by m2l_tile
template <typename T>
__global__ __launch_bounds__(256) void k_m2l(const T *__restrict__ K, const T *__restrict__ M,
                                             double *__restrict__ out, int nside, int nup, int nsplit,
                                             int64_t out_stride) {
    using Acc = typename Mma<T>::acc;
    __shared__ T As[2][BK][BM + 4];
    __shared__ T Bs[2][BK][BN + 4];
    __shared__ int il[kNumIL];

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1;
    const M2LTile tile = m2l_tile((nup + BM - 1) / BM, ((nside >> 1) * (nside >> 1) * (nside >> 1) + BN - 1) / BN,
                                  nsplit);
    const int rt = tile.rt, ct = tile.ct, cls = tile.cls, split = tile.split;
    const int px = cls >> 2, py = (cls >> 1) & 1, pz = cls & 1;
    const int h = nside >> 1;
    const int ncls = h * h * h;
    const int row0 = rt * BM, col0 = ct * BN;

    // interaction list of this parity class, in a fixed order
    if (tid == 0) {
        int k = 0;
        for (int a = 0; a < 6; a++)
            for (int b = 0; b < 6; b++)
                for (int c = 0; c < 6; c++) {
                    const int dx = (px ? -3 : -2) + a, dy = (py ? -3 : -2) + b, dz = (pz ? -3 : -2) + c;
                    if (max(abs(dx), max(abs(dy), abs(dz))) >= 2) il[k++] = off_index(dx, dy, dz);
                }
    }
    __syncthreads();
    const int o_begin = kNumIL * split / nsplit, o_end = kNumIL * (split + 1) / nsplit;

    // loader roles: A (K_d rows l, cols = output nodes) and B (M of the source cell of one column)
    const int a_r = tid >> 4, a_c = (tid & 15) * 4;          // 16 x 64 tile, 4 per thread
    const int b_col = tid >> 2, b_r = (tid & 3) * 4;         // 16 x 64 tile, 4 per thread
    const int tcell = col0 + b_col;
    const bool b_ok = tcell < ncls;
    int gx = 0, gy = 0, gz = 0;
    if (b_ok) {
        gx = 2 * (tcell / (h * h)) + px;
        gy = 2 * ((tcell / h) % h) + py;
        gz = 2 * (tcell % h) + pz;
    }
    const bool a_ok = row0 + a_c < nup;   // nup is a multiple of 32 and a_c of 4

    const int nk = nup / BK;
    const int niter = (o_end - o_begin) * nk;
    T ra[4], rb[4];
    auto load = [&](int it) {
        const int oi = o_begin + it / nk, k0 = (it % nk) * BK;
        const int di = il[oi];
        const T *Kd = K + (size_t)di * nup * nup;
#pragma unroll
        for (int u = 0; u < 4; u++) ra[u] = a_ok ? Kd[(size_t)(k0 + a_r) * nup + row0 + a_c + u] : (T)0;
        if (b_ok) {
            const int dx = di / 49 - 3, dy = (di / 7) % 7 - 3, dz = di % 7 - 3;
            const int sx = (gx + dx + 4 * nside) % nside, sy = (gy + dy + 4 * nside) % nside,
                      sz = (gz + dz + 4 * nside) % nside;
            const T *Ms = M + ((size_t)(sx * nside + sy) * nside + sz) * nup + k0 + b_r;
#pragma unroll
            for (int u = 0; u < 4; u++) rb[u] = Ms[u];
        } else {
#pragma unroll
            for (int u = 0; u < 4; u++) rb[u] = (T)0;
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int u = 0; u < 4; u++) As[buf][a_r][a_c + u] = ra[u];
#pragma unroll
        for (int u = 0; u < 4; u++) Bs[buf][b_r + u][b_col] = rb[u];
    };

    Acc acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; i++)
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
            T av[2], bv[2];
#pragma unroll
            for (int i = 0; i < 2; i++) av[i] = As[cur][kk + lk][wr * 32 + i * 16 + lr];
#pragma unroll
            for (int j = 0; j < 2; j++) bv[j] = Bs[cur][kk + lk][wc * 32 + j * 16 + lr];
#pragma unroll
            for (int i = 0; i < 2; i++)
#pragma unroll
                for (int j = 0; j < 2; j++) acc[i][j] = Mma<T>::run(av[i], bv[j], acc[i][j]);
        }
        if (it + 1 < niter) store(cur ^ 1);
        __syncthreads();
    }

    // scatter each 16 x 16 result block (rows per Mma<T>::row, column lane % 16)
    double *o = out + (size_t)split * out_stride;
#pragma unroll
    for (int j = 0; j < 2; j++) {
        const int cl = col0 + wc * 32 + j * 16 + lr;
        if (cl >= ncls) continue;
        const int cx = 2 * (cl / (h * h)) + px, cy = 2 * ((cl / h) % h) + py, cz = 2 * (cl % h) + pz;
        double *Lc = o + ((size_t)(cx * nside + cy) * nside + cz) * nup;
#pragma unroll
        for (int i = 0; i < 2; i++) {
            const int rb = row0 + wr * 32 + i * 16;   // 16-row block, entirely inside or outside nup
            if (rb >= nup) continue;
#pragma unroll
            for (int v = 0; v < 4; v++) Lc[rb + Mma<T>::row(lk, v)] = (double)acc[i][j][v];
        }
    }
}

// ---- split-precision variant: BF16 x 3 on the 16x16x32 BF16 matrix cores ------
// Each float32 operand is split as x = hi + lo (hi = bf16(x), lo = bf16(x - hi)),
// and the product is accumulated in float32 as hi*hi + hi*lo + lo*hi (the
// lo*lo term is below the float32 rounding of the sum).  K is stored row-major
// per offset (K_d[k][l]); the multipoles of the level are split on the fly.
// Lane l of v_mfma_f32_16x16x32_bf16 supplies A[l % 16][8 (l / 16) .. +8] and
// B[8 (l / 16) .. +8][l % 16]; result element v sits at row 4 (l / 16) + v,
// column l % 16.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
constexpr int BK3 = 32, PADK = 8;

__global__ __launch_bounds__(256) void k_m2l_bf16x3(const __bf16 *__restrict__ Kh, const __bf16 *__restrict__ Kl,
                                                    const __bf16 *__restrict__ Mh, const __bf16 *__restrict__ Ml,
                                                    double *__restrict__ out, int nside, int nup, int nsplit,
                                                    int64_t out_stride) {
    __shared__ __attribute__((aligned(16))) __bf16 Ash[2][BM][BK3 + PADK];
    __shared__ __attribute__((aligned(16))) __bf16 Asl[2][BM][BK3 + PADK];
    __shared__ __attribute__((aligned(16))) __bf16 Bsh[2][BN][BK3 + PADK];
    __shared__ __attribute__((aligned(16))) __bf16 Bsl[2][BN][BK3 + PADK];
    __shared__ int il[kNumIL];

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1;
    const M2LTile tile = m2l_tile((nup + BM - 1) / BM, ((nside >> 1) * (nside >> 1) * (nside >> 1) + BN - 1) / BN,
                                  nsplit);
    const int rt = tile.rt, ct = tile.ct, cls = tile.cls, split = tile.split;
    const int px = cls >> 2, py = (cls >> 1) & 1, pz = cls & 1;
    const int h = nside >> 1;
    const int ncls = h * h * h;
    const int row0 = rt * BM, col0 = ct * BN;
    if (tid == 0) {
        int k = 0;
        for (int a = 0; a < 6; a++)
            for (int b = 0; b < 6; b++)
                for (int c = 0; c < 6; c++) {
                    const int dx = (px ? -3 : -2) + a, dy = (py ? -3 : -2) + b, dz = (pz ? -3 : -2) + c;
                    if (max(abs(dx), max(abs(dy), abs(dz))) >= 2) il[k++] = off_index(dx, dy, dz);
                }
    }
    __syncthreads();
    const int o_begin = kNumIL * split / nsplit, o_end = kNumIL * (split + 1) / nsplit;

    // loaders: one 16-byte chunk (8 bf16 along the contraction) of hi and of lo per thread for A and B
    const int ld_r = tid >> 2, ld_c = (tid & 3) * 8;
    const bool a_ok = row0 + ld_r < nup;
    const int tcell = col0 + ld_r;
    const bool b_ok = tcell < ncls;
    int gx = 0, gy = 0, gz = 0;
    if (b_ok) {
        gx = 2 * (tcell / (h * h)) + px;
        gy = 2 * ((tcell / h) % h) + py;
        gz = 2 * (tcell % h) + pz;
    }
    const int nk = nup / BK3;
    const int niter = (o_end - o_begin) * nk;
    uint4 rah, ral, rbh, rbl;
    const uint4 zero4 = {0u, 0u, 0u, 0u};
    auto load = [&](int it) {
        const int oi = o_begin + it / nk, k0 = (it % nk) * BK3;
        const int di = il[oi];
        if (a_ok) {
            const size_t off = ((size_t)di * nup + row0 + ld_r) * nup + k0 + ld_c;
            rah = *reinterpret_cast<const uint4 *>(Kh + off);
            ral = *reinterpret_cast<const uint4 *>(Kl + off);
        } else {
            rah = zero4;
            ral = zero4;
        }
        if (b_ok) {
            const int dx = di / 49 - 3, dy = (di / 7) % 7 - 3, dz = di % 7 - 3;
            const int sx = (gx + dx + 4 * nside) % nside, sy = (gy + dy + 4 * nside) % nside,
                      sz = (gz + dz + 4 * nside) % nside;
            const size_t off = ((size_t)(sx * nside + sy) * nside + sz) * nup + k0 + ld_c;
            rbh = *reinterpret_cast<const uint4 *>(Mh + off);
            rbl = *reinterpret_cast<const uint4 *>(Ml + off);
        } else {
            rbh = zero4;
            rbl = zero4;
        }
    };
    auto store = [&](int buf) {
        *reinterpret_cast<uint4 *>(&Ash[buf][ld_r][ld_c]) = rah;
        *reinterpret_cast<uint4 *>(&Asl[buf][ld_r][ld_c]) = ral;
        *reinterpret_cast<uint4 *>(&Bsh[buf][ld_r][ld_c]) = rbh;
        *reinterpret_cast<uint4 *>(&Bsl[buf][ld_r][ld_c]) = rbl;
    };

    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; i++)
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
        bf16x8 ah[2], al[2], bh[2], bl[2];
#pragma unroll
        for (int i = 0; i < 2; i++) {
            ah[i] = *reinterpret_cast<const bf16x8 *>(&Ash[cur][wr * 32 + i * 16 + lr][8 * lk]);
            al[i] = *reinterpret_cast<const bf16x8 *>(&Asl[cur][wr * 32 + i * 16 + lr][8 * lk]);
        }
#pragma unroll
        for (int j = 0; j < 2; j++) {
            bh[j] = *reinterpret_cast<const bf16x8 *>(&Bsh[cur][wc * 32 + j * 16 + lr][8 * lk]);
            bl[j] = *reinterpret_cast<const bf16x8 *>(&Bsl[cur][wc * 32 + j * 16 + lr][8 * lk]);
        }
#pragma unroll
        for (int i = 0; i < 2; i++)
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
        const int cl = col0 + wc * 32 + j * 16 + lr;
        if (cl >= ncls) continue;
        const int cx = 2 * (cl / (h * h)) + px, cy = 2 * ((cl / h) % h) + py, cz = 2 * (cl % h) + pz;
        double *Lc = o + ((size_t)(cx * nside + cy) * nside + cz) * nup;
#pragma unroll
        for (int i = 0; i < 2; i++) {
            const int rb = row0 + wr * 32 + i * 16;
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

// plan time: row-major K_d[k][l] from the [d][l][k] float64 stack (K_{-d} = K_d^T)
__global__ void k_split_K_bf16(const double *__restrict__ K, __bf16 *__restrict__ hi, __bf16 *__restrict__ lo,
                               int nup) {
    const int64_t n = (int64_t)kNumOff * nup * nup;
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t per = (int64_t)nup * nup;
    const int d = (int)(i / per);
    const float x = (float)K[(int64_t)(kNumOff - 1 - d) * per + i % per];
    const __bf16 a = (__bf16)x;
    hi[i] = a;
    lo[i] = (__bf16)(x - (float)a);
}

// L = sum over the split-K partials, in split order
__global__ void k_m2l_reduce(const double *__restrict__ part, double *__restrict__ L, int64_t n, int nsplit) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s = part[i];
    for (int k = 1; k < nsplit; k++) s += part[k * n + i];
    L[i] = s;
}

__global__ void k_f64_to_f32(const double *__restrict__ s, float *__restrict__ d, int64_t n) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) d[i] = (float)s[i];
}

}  // namespace

// number of offset slices so that a level launches at least ~4 blocks per CU
hipError_t launch_split_K_bf16(ankh_plan_s *pl, const double *K, __bf16 *hi, __bf16 *lo) {
    const int64_t n = (int64_t)kNumOff * pl->nup * pl->nup;
    hipLaunchKernelGGL(k_split_K_bf16, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, pl->stream, K, hi, lo, pl->nup);
    return hipGetLastError();
}

// Number of offset slices (split-K): enough blocks to fill the chip (>= 1024),
// K slices of at most ~3 MiB (one per XCD L2 at a time), and, where possible,
// (row tiles x slices) a multiple of 8 for the XCD-aware block order.
int m2l_splits(const ankh_plan_s *pl, int e) {
    const int h = pl->lv[e].nside / 2;
    const int nrt = (pl->nup + BM - 1) / BM;
    const int64_t tiles = (int64_t)nrt * ((h * h * h + BN - 1) / BN) * 8;
    const double bytes = pl->precision == ANKH_FP64 ? 8.0 : 4.0;   // f64, f32, or bf16 hi + lo
    const double slice = (double)BM * pl->nup * kNumIL * bytes;
    int smin = (int)std::ceil(slice / (3.0 * 1024 * 1024));
    while ((int64_t)smin * tiles < 1024) smin++;
    smin = std::min(std::max(smin, 1), 27);
    for (int s = smin; s <= 27; s++)
        if ((nrt * s) % 8 == 0) return s;
    return smin;
}

hipError_t launch_m2l(ankh_plan_s *pl, int e) {
    const ankh::Level &lv = pl->lv[e];
    const int h = lv.nside / 2;
    const int ncls = h * h * h;
    const int nsplit = m2l_splits(pl, e);
    dim3 grid((unsigned)(((pl->nup + BM - 1) / BM) * ((ncls + BN - 1) / BN) * 8 * nsplit));
    const int64_t nval = lv.ncell * pl->nup;
    double *L = pl->d_L + lv.cell0 * pl->nup;
    double *out = nsplit > 1 ? pl->d_m2l_part : L;
    const size_t koff = (size_t)(e - 1) * kNumOff * pl->nup * pl->nup;
    if (pl->precision == ANKH_MIXED_BF16X3) {
        __bf16 *Mh = pl->d_Mb, *Ml = pl->d_Mb + nval;
        hipLaunchKernelGGL(k_split_bf16, dim3((unsigned)((nval + 255) / 256)), dim3(256), 0, pl->stream,
                           pl->d_M + lv.cell0 * pl->nup, Mh, Ml, nval);
        const size_t kb = (size_t)(e - 1) * kNumOff * pl->nup * pl->nup;
        const size_t kall = (size_t)pl->depth * kNumOff * pl->nup * pl->nup;
        hipLaunchKernelGGL(k_m2l_bf16x3, grid, dim3(256), 0, pl->stream, pl->d_Kb + kb, pl->d_Kb + kall + kb, Mh, Ml,
                           out, lv.nside, pl->nup, nsplit, nval);
    } else if (pl->precision == ANKH_MIXED) {
        float *Mf = pl->d_Mf;   // this level's multipoles in float32
        hipLaunchKernelGGL(k_f64_to_f32, dim3((unsigned)((nval + 255) / 256)), dim3(256), 0, pl->stream,
                           pl->d_M + lv.cell0 * pl->nup, Mf, nval);
        hipLaunchKernelGGL(k_m2l<float>, grid, dim3(256), 0, pl->stream, pl->d_Kf + koff, Mf, out, lv.nside,
                           pl->nup, nsplit, nval);
    } else {
        hipLaunchKernelGGL(k_m2l<double>, grid, dim3(256), 0, pl->stream, pl->d_K + koff,
                           pl->d_M + lv.cell0 * pl->nup, out, lv.nside, pl->nup, nsplit, nval);
    }
    if (nsplit > 1)
        hipLaunchKernelGGL(k_m2l_reduce, dim3((unsigned)((nval + 255) / 256)), dim3(256), 0, pl->stream,
                           pl->d_m2l_part, L, nval, nsplit);
    return hipGetLastError();
}

}  // namespace ankh
