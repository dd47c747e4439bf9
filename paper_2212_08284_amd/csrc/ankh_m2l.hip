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
// Per parity class the level is one implicit GEMM
//   [n_u x 189 n_u] x [189 n_u x (cells of the class)],
// whose right operand is gathered from the multipole array.  A block computes a
// 64 (nodes) x 64 (cells) tile of L; the 189 x n_u contraction streams K_d and
// the gathered M through LDS in steps of TK rows.
#include "ankh_internal.h"

namespace ankh {
namespace {

constexpr int TM = 64, TN = 64, TK = 16;

template <typename T>
__global__ __launch_bounds__(256) void k_m2l(const T *__restrict__ K, const double *__restrict__ M,
                                             double *__restrict__ Lout, int nside, int nup) {
    __shared__ T As[TK][TM];
    __shared__ T Bs[TK][TN + 1];
    const int tid = threadIdx.x;
    const int rt = blockIdx.x, ct = blockIdx.y, cls = blockIdx.z;
    const int px = cls >> 2, py = (cls >> 1) & 1, pz = cls & 1;
    const int h = nside >> 1;
    const int ncls = h * h * h;
    const int ty = tid >> 4, tx = tid & 15;

    // the column this thread loads B for, and its target cell
    const int lcol = tid >> 2, lrow = (tid & 3) * 4;
    const int tcell_local = ct * TN + lcol;
    const bool lvalid = tcell_local < ncls;
    int gx = 0, gy = 0, gz = 0;
    if (lvalid) {
        gx = 2 * (tcell_local / (h * h)) + px;
        gy = 2 * ((tcell_local / h) % h) + py;
        gz = 2 * (tcell_local % h) + pz;
    }

    T acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; i++)
#pragma unroll
        for (int j = 0; j < 4; j++) acc[i][j] = 0;

    const int dx0 = px ? -3 : -2, dy0 = py ? -3 : -2, dz0 = pz ? -3 : -2;
    for (int a = 0; a < 6; a++)
        for (int b = 0; b < 6; b++)
            for (int c = 0; c < 6; c++) {
                const int dx = dx0 + a, dy = dy0 + b, dz = dz0 + c;
                if (max(abs(dx), max(abs(dy), abs(dz))) < 2) continue;
                const T *Kd = K + (size_t)off_index(dx, dy, dz) * nup * nup + (size_t)rt * TM;
                const double *Ms = nullptr;
                if (lvalid) {
                    const int sx = (gx + dx + 4 * nside) % nside;
                    const int sy = (gy + dy + 4 * nside) % nside;
                    const int sz = (gz + dz + 4 * nside) % nside;
                    Ms = M + ((size_t)(sx * nside + sy) * nside + sz) * nup;
                }
                for (int l0 = 0; l0 < nup; l0 += TK) {
                    // A: K_d[l0 + r][rt*64 + col], 16 x 64
#pragma unroll
                    for (int u = 0; u < 4; u++) {
                        const int e = tid + 256 * u;
                        const int r = e >> 6, col = e & 63;
                        As[r][col] = Kd[(size_t)(l0 + r) * nup + col];
                    }
                    // B: M_src[l0 + r] for this thread's column
#pragma unroll
                    for (int u = 0; u < 4; u++) Bs[lrow + u][lcol] = lvalid ? (T)Ms[l0 + lrow + u] : (T)0;
                    __syncthreads();
#pragma unroll
                    for (int r = 0; r < TK; r++) {
                        T av[4], bv[4];
#pragma unroll
                        for (int i = 0; i < 4; i++) av[i] = As[r][ty * 4 + i];
#pragma unroll
                        for (int j = 0; j < 4; j++) bv[j] = Bs[r][tx * 4 + j];
#pragma unroll
                        for (int i = 0; i < 4; i++)
#pragma unroll
                            for (int j = 0; j < 4; j++) acc[i][j] += av[i] * bv[j];
                    }
                    __syncthreads();
                }
            }

#pragma unroll
    for (int j = 0; j < 4; j++) {
        const int cl = ct * TN + tx * 4 + j;
        if (cl >= ncls) continue;
        const int cx = 2 * (cl / (h * h)) + px, cy = 2 * ((cl / h) % h) + py, cz = 2 * (cl % h) + pz;
        double *Lc = Lout + ((size_t)(cx * nside + cy) * nside + cz) * nup + (size_t)rt * TM;
#pragma unroll
        for (int i = 0; i < 4; i++) Lc[ty * 4 + i] = (double)acc[i][j];
    }
}

}  // namespace

hipError_t launch_m2l(ankh_plan_s *pl, int e) {
    const ankh::Level &lv = pl->lv[e];
    const int h = lv.nside / 2;
    const int ncls = h * h * h;
    dim3 grid(pl->nup / TM, (ncls + TN - 1) / TN, 8);
    const double *M = pl->d_M + lv.cell0 * pl->nup;
    double *L = pl->d_L + lv.cell0 * pl->nup;
    const size_t koff = (size_t)(e - 1) * kNumOff * pl->nup * pl->nup;
    if (pl->precision == ANKH_MIXED)
        hipLaunchKernelGGL(k_m2l<float>, grid, dim3(256), 0, pl->stream, pl->d_Kf + koff, M, L, lv.nside, pl->nup);
    else
        hipLaunchKernelGGL(k_m2l<double>, grid, dim3(256), 0, pl->stream, pl->d_K + koff, M, L, lv.nside, pl->nup);
    return hipGetLastError();
}

}  // namespace ankh
