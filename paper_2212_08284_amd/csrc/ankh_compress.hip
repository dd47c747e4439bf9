// Compressed M2L (the singular-value compression of the far-field operator,
// the compressed-M2L passage of the paper): with U the leading left singular
// vectors of the stack [A_d] of a level's M2L operators over the 316 offsets
// (A_d[k][l] = K[d][l][k]), every operator is replaced by U (U^T A_d U) U^T.
// The stack is closed under transposition (A_-d = A_d^T), so one basis serves
// the targets and the sources.  Plan time: the Gram matrix sum_d A_d A_d^T on
// the device, its eigenvectors on the host (cyclic Jacobi), the compressed
// stacks U^T A_d U.  Per evaluation: projection M' = U^T M before the
// contraction and expansion L = U L' after it.
#include <algorithm>
#include <cmath>
#include <vector>

#include "ankh_internal.h"

namespace ankh {
namespace {

// C(m, n) = sum_k A(m, k) B(k, n) in float64 over a 32 x 32 tile per block
// (one wave, 4 x 4 outputs per lane), contraction in steps of 16 through LDS:
// small blocks, many of them, so latency is hidden across blocks.
// Element addresses: A(m, k) = A[m sam + k sak], B(k, n) = B[k sbk + n sbn],
// C(m, n) = C[m scm + n].  blockIdx.z selects a batch item (offsets za, zb,
// zc) or, with splitk, the contraction range [z kz, z kz + kz) whose partial
// product goes to C + z zc.
struct Gemm {
    int M, N, K, kz, splitk;
    const double *A;
    int64_t za, sam, sak;
    const double *B;
    int64_t zb, sbk, sbn;
    double *C;
    int64_t zc, scm;
};

constexpr int GT = 32, GK = 16;

__global__ __launch_bounds__(64) void k_dgemm(Gemm g) {
    __shared__ double As[GK][GT + 1], Bs[GK][GT + 1];
    const int tid = threadIdx.x, tx = tid % 8, ty = tid / 8;
    const int m0 = blockIdx.y * GT, n0 = blockIdx.x * GT;
    const int64_t z = blockIdx.z;
    const double *A = g.A + z * g.za, *B = g.B + z * g.zb;
    double *C = g.C + z * g.zc;
    const int kb = g.splitk ? (int)z * g.kz : 0;
    const int ke = g.splitk ? min(g.K, kb + g.kz) : g.K;
    double acc[4][4] = {};
    for (int k0 = kb; k0 < ke; k0 += GK) {
        double ra[GK * GT / 64], rb[GK * GT / 64];
#pragma unroll
        for (int q = 0; q < GK * GT / 64; q++) {
            // the faster-varying index follows the unit stride of each operand
            const int e = tid + 64 * q;
            const int kk = g.sak == 1 ? e % GK : e / GT, mm = g.sak == 1 ? e / GK : e % GT;
            const int m = m0 + mm, k = k0 + kk;
            ra[q] = (m < g.M && k < ke) ? A[m * g.sam + k * g.sak] : 0.0;
            const int kb2 = g.sbk == 1 ? e % GK : e / GT, nn = g.sbk == 1 ? e / GK : e % GT;
            const int n = n0 + nn, k2 = k0 + kb2;
            rb[q] = (n < g.N && k2 < ke) ? B[k2 * g.sbk + n * g.sbn] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < GK * GT / 64; q++) {
            const int e = tid + 64 * q;
            As[g.sak == 1 ? e % GK : e / GT][g.sak == 1 ? e / GK : e % GT] = ra[q];
            Bs[g.sbk == 1 ? e % GK : e / GT][g.sbk == 1 ? e / GK : e % GT] = rb[q];
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < GK; kk++) {
            double a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; i++) a[i] = As[kk][ty + 8 * i];
#pragma unroll
            for (int j = 0; j < 4; j++) b[j] = Bs[kk][tx + 8 * j];
#pragma unroll
            for (int i = 0; i < 4; i++)
#pragma unroll
                for (int j = 0; j < 4; j++) acc[i][j] += a[i] * b[j];
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; i++)
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const int m = m0 + ty + 8 * i, n = n0 + tx + 8 * j;
            if (m < g.M && n < g.N) C[m * g.scm + n] = acc[i][j];
        }
}

hipError_t dgemm(const Gemm &g, int nz, hipStream_t s) {
    dim3 grid((unsigned)((g.N + GT - 1) / GT), (unsigned)((g.M + GT - 1) / GT), (unsigned)nz);
    hipLaunchKernelGGL(k_dgemm, grid, dim3(64), 0, s, g);
    return hipGetLastError();
}

// Eigen-decomposition of a symmetric n x n matrix (row-major, destroyed) by
// cyclic Jacobi rotations: w = eigenvalues, V = eigenvectors as columns.
void jacobi_eig(std::vector<double> &A, int n, std::vector<double> &w, std::vector<double> &V) {
    V.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; i++) V[(size_t)i * n + i] = 1.0;
    for (int sweep = 0; sweep < 60; sweep++) {
        double off = 0, tot = 0;
        for (int i = 0; i < n; i++)
            for (int j = 0; j < n; j++) {
                const double a = A[(size_t)i * n + j];
                tot += a * a;
                if (i != j) off += a * a;
            }
        if (off <= 1e-30 * tot) break;
        for (int p = 0; p < n - 1; p++)
            for (int q = p + 1; q < n; q++) {
                const double apq = A[(size_t)p * n + q];
                if (std::fabs(apq) < 1e-300) continue;
                const double theta = (A[(size_t)q * n + q] - A[(size_t)p * n + p]) / (2 * apq);
                const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1));
                const double c = 1 / std::sqrt(t * t + 1), s = t * c;
                for (int k = 0; k < n; k++) {
                    const double akp = A[(size_t)k * n + p], akq = A[(size_t)k * n + q];
                    A[(size_t)k * n + p] = c * akp - s * akq;
                    A[(size_t)k * n + q] = s * akp + c * akq;
                }
                for (int k = 0; k < n; k++) {
                    const double apk = A[(size_t)p * n + k], aqk = A[(size_t)q * n + k];
                    A[(size_t)p * n + k] = c * apk - s * aqk;
                    A[(size_t)q * n + k] = s * apk + c * aqk;
                }
                for (int k = 0; k < n; k++) {
                    const double vkp = V[(size_t)k * n + p], vkq = V[(size_t)k * n + q];
                    V[(size_t)k * n + p] = c * vkp - s * vkq;
                    V[(size_t)k * n + q] = s * vkp + c * vkq;
                }
            }
    }
    w.resize(n);
    for (int i = 0; i < n; i++) w[i] = A[(size_t)i * n + i];
}

// Batched basis change of the compressed levels, C = A B per level with
// A [rows][K] (row stride lda), C [rows][N] (row stride ldc) and B either
// [K][N] (TN, row stride ldb) or [N][K] (NT).  Float64.  Block tile 32 rows x 32
// columns; the 4 waves of a block split the contraction (wave w takes chunks
// w, w + 4, ... of 16), each accumulating the whole tile (4 x 4 outputs per
// lane) from its own LDS slice with the next chunk held in registers; the 4
// partial tiles are summed through LDS in wave order at the end.  The short
// per-wave chain keeps the launch from waiting on one long dependent sequence.
// Tiles of a level are numbered row-major (columns fastest) and dealt to the
// 8 XCDs in contiguous runs, so the column tiles of one row tile share an L2.
// Strides and bases are even (16-byte pairs of doubles).
struct BasisLevel {
    const double *A;
    const double *B;
    double *C;
    int lda, ldb, ldc, rows, N, K, ntn, tile0;
};
constexpr int kMaxBasisLevels = 8;
struct BasisJob {
    BasisLevel lv[kMaxBasisLevels];
    int nlv, ntiles, per_xcd;
};
constexpr int BT = 32, BKC = 16, BW = 4;   // tile, chunk, waves per block

template <bool NT>
__global__ __launch_bounds__(256) void k_basis(BasisJob job) {
    // per wave: A chunk [16][33] and B chunk [16][33]; reused for the final sum [4][32][33]
    __shared__ double lds[BW * 2 * BKC * (BT + 1)];
    const int b = blockIdx.x;
    const int v = (b % 8) * job.per_xcd + b / 8;
    if (v >= job.ntiles) return;
    int li = 0;
    while (li + 1 < job.nlv && v >= job.lv[li + 1].tile0) li++;
    const BasisLevel L = job.lv[li];
    const int tl = v - L.tile0;
    const int m0 = (tl / L.ntn) * BT, n0 = (tl % L.ntn) * BT;
    const int wv = threadIdx.x / 64, ln = threadIdx.x % 64, tx = ln % 8, ty = ln / 8;
    double(*As)[BT + 1] = reinterpret_cast<double(*)[BT + 1]>(lds + wv * 2 * BKC * (BT + 1));
    double(*Bs)[BT + 1] = reinterpret_cast<double(*)[BT + 1]>(lds + (wv * 2 + 1) * BKC * (BT + 1));
    // K and N are multiples of the chunk and tile widths (host-checked); rows of A beyond the level
    // are clamped to its last row and their results dropped.  A wave past the last chunk loads zeros.
    const int nchunk = L.K / BKC, steps = (nchunk + BW - 1) / BW;
    double2 ra[4], rb[4];
    auto load = [&](int c) {
        const bool ok = c < nchunk;
        const int k0 = c * BKC;
#pragma unroll
        for (int q = 0; q < 4; q++) {
            const int idx = ln + 64 * q;
            const int r = idx / 8, p = 2 * (idx % 8);          // A and B (NT): 32 rows x 8 pairs
            const int m = min(m0 + r, L.rows - 1);
            ra[q] = ok ? *reinterpret_cast<const double2 *>(L.A + (int64_t)m * L.lda + k0 + p) : double2{0.0, 0.0};
            if (NT) {
                rb[q] = ok ? *reinterpret_cast<const double2 *>(L.B + (int64_t)(n0 + r) * L.ldb + k0 + p)
                           : double2{0.0, 0.0};
            } else {
                const int rk = idx / 16, pn = 2 * (idx % 16);   // B (TN): 16 rows of K x 16 pairs along N
                rb[q] = ok ? *reinterpret_cast<const double2 *>(L.B + (int64_t)(k0 + rk) * L.ldb + n0 + pn)
                           : double2{0.0, 0.0};
            }
        }
    };
    auto store = [&]() {
#pragma unroll
        for (int q = 0; q < 4; q++) {
            const int idx = ln + 64 * q;
            const int r = idx / 8, p = 2 * (idx % 8);
            As[p][r] = ra[q].x;
            As[p + 1][r] = ra[q].y;
            if (NT) {
                Bs[p][r] = rb[q].x;
                Bs[p + 1][r] = rb[q].y;
            } else {
                const int rk = idx / 16, pn = 2 * (idx % 16);
                Bs[rk][pn] = rb[q].x;
                Bs[rk][pn + 1] = rb[q].y;
            }
        }
    };
    double acc[4][4] = {};
    load(wv);
    for (int t = 0; t < steps; t++) {
        __syncthreads();   // the previous chunk's reads are done
        store();
        __syncthreads();
        if (t + 1 < steps) load(wv + BW * (t + 1));
#pragma unroll
        for (int kk = 0; kk < BKC; kk++) {
            double a[4], bb[4];
#pragma unroll
            for (int i = 0; i < 4; i++) a[i] = As[kk][ty + 8 * i];
#pragma unroll
            for (int j = 0; j < 4; j++) bb[j] = Bs[kk][tx + 8 * j];
#pragma unroll
            for (int i = 0; i < 4; i++)
#pragma unroll
                for (int j = 0; j < 4; j++) acc[i][j] = fma(a[i], bb[j], acc[i][j]);
        }
    }
    // the 4 waves' partial tiles, summed in wave order
    __syncthreads();
    double(*red)[BT][BT + 1] = reinterpret_cast<double(*)[BT][BT + 1]>(lds);
#pragma unroll
    for (int i = 0; i < 4; i++)
#pragma unroll
        for (int j = 0; j < 4; j++) red[wv][ty + 8 * i][tx + 8 * j] = acc[i][j];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; q++) {
        const int o = threadIdx.x + 256 * q, r = o / BT, c = o % BT;
        const int m = m0 + r;
        const double sum = (red[0][r][c] + red[1][r][c]) + (red[2][r][c] + red[3][r][c]);
        if (m < L.rows) L.C[(int64_t)m * L.ldc + n0 + c] = sum;
    }
}

}  // namespace

hipError_t launch_m2l_basis(ankh_plan_s *pl, bool expand) {
    BasisJob job{};
    int nt = 0;
    for (int e = 1; e <= pl->depth; e++) {
        const int rp = pl->rpad[e];
        if (rp >= pl->nup) continue;
        if (job.nlv == kMaxBasisLevels) return hipErrorInvalidValue;
        const ankh::Level &lv = pl->lv[e];
        BasisLevel &b = job.lv[job.nlv++];
        double *M = pl->d_M + lv.cell0 * pl->nup, *Lf = pl->d_L + lv.cell0 * pl->nup;
        double *Mc = pl->d_Mc + pl->c_off[e], *Lc = pl->d_Lc + pl->c_off[e];
        b.B = pl->d_U + pl->u_off[e];
        b.ldb = rp;
        b.rows = (int)lv.ncell;
        // the padding columns of M (beyond n_u) are zero, as are the rows of U there
        if (!expand) {
            b.A = M, b.lda = pl->nup, b.K = pl->nup;
            b.C = Mc, b.ldc = rp, b.N = rp;
        } else {
            b.A = Lc, b.lda = rp, b.K = rp;
            b.C = Lf, b.ldc = pl->nup, b.N = pl->nup;
        }
        if (b.K % BKC || b.N % BT || b.rows < 1) return hipErrorInvalidValue;
        b.ntn = b.N / BT;
        b.tile0 = nt;
        nt += ((b.rows + BT - 1) / BT) * b.ntn;
    }
    if (job.nlv == 0) return hipSuccess;
    job.ntiles = nt;
    job.per_xcd = (nt + 7) / 8;
    const dim3 grid((unsigned)(8 * job.per_xcd));
    if (expand)
        hipLaunchKernelGGL(k_basis<true>, grid, dim3(256), 0, pl->stream, job);
    else
        hipLaunchKernelGGL(k_basis<false>, grid, dim3(256), 0, pl->stream, job);
    return hipGetLastError();
}


// Plan time, one level: K = the full float64 stack [343][nup][nup] of the
// level (K[d][l][k], zero outside the far offsets and the n_u nodes).  Chooses
// the rank r (singular values above tol x the largest), rounds it up to a
// multiple of 32 (rp), and if rp < n_up writes U [nup][rp] to d_U + u_off[e]
// and the compressed stack [343][rp][rp] (same layout) to Kc; else leaves the
// level uncompressed (rp = n_up).  work: device scratch of >= 343 nup rp doubles.
hipError_t compress_level(ankh_plan_s *pl, int e, const double *K, double *Kc, double *work, double tol) {
    const int nu = pl->nu, nup = pl->nup;
    hipStream_t s = pl->stream;
    // Gram matrix, split over 32 ranges of the (d, l) contraction, summed on the host
    const int KZ = 32;
    const int Ktot = kNumOff * nup;
    const int kz = (Ktot + KZ - 1) / KZ;
    Gemm g{nu, nu, Ktot, kz, 1, K, 0, 1, nup, K, 0, nup, 1, work, (int64_t)nu * nu, nu};
    hipError_t err = dgemm(g, KZ, s);
    if (err != hipSuccess) return err;
    std::vector<double> parts((size_t)KZ * nu * nu);
    if ((err = hipMemcpyAsync(parts.data(), work, parts.size() * sizeof(double), hipMemcpyDeviceToHost, s)) !=
        hipSuccess)
        return err;
    if ((err = hipStreamSynchronize(s)) != hipSuccess) return err;
    std::vector<double> G((size_t)nu * nu, 0.0), w, V;
    for (int z = 0; z < KZ; z++)
        for (size_t i = 0; i < G.size(); i++) G[i] += parts[(size_t)z * nu * nu + i];
    jacobi_eig(G, nu, w, V);
    std::vector<int> order(nu);
    for (int i = 0; i < nu; i++) order[i] = i;
    std::sort(order.begin(), order.end(), [&](int a, int b) { return w[a] > w[b]; });
    const double smax = std::sqrt(std::max(w[order[0]], 0.0));
    int r = 0;
    while (r < nu && std::sqrt(std::max(w[order[r]], 0.0)) > tol * smax) r++;
    const int rp = std::max(32, (r + 31) / 32 * 32);
    pl->m2l_rank[e] = r;
    if (rp >= nup) {
        pl->rpad[e] = nup;
        pl->m2l_rank[e] = nu;
        return hipSuccess;
    }
    pl->rpad[e] = rp;
    std::vector<double> U((size_t)nup * rp, 0.0);
    for (int k = 0; k < nu; k++)
        for (int i = 0; i < r; i++) U[(size_t)k * rp + i] = V[(size_t)k * nu + order[i]];
    double *dU = pl->d_U + pl->u_off[e];
    if ((err = hipMemcpyAsync(dU, U.data(), U.size() * sizeof(double), hipMemcpyHostToDevice, s)) != hipSuccess)
        return err;
    // T[d][l][i] = sum_k K[d][l][k] U[k][i];  Kc[d][j][i] = sum_l U[l][j] T[d][l][i]
    Gemm t1{nu, rp, nu, nu, 0, K, (int64_t)nup * nup, nup, 1, dU, 0, rp, 1, work, (int64_t)nup * rp, rp};
    if ((err = dgemm(t1, kNumOff, s)) != hipSuccess) return err;
    Gemm t2{rp, rp, nu, nu, 0, dU, 0, 1, rp, work, (int64_t)nup * rp, rp, 1, Kc, (int64_t)rp * rp, rp};
    if ((err = dgemm(t2, kNumOff, s)) != hipSuccess) return err;
    return hipStreamSynchronize(s);
}

// Per evaluation, all compressed levels in one launch each way:
//   projection  Mc [cells][rp]  = M [cells][nup] U        (B stored [k][n], TN)
//   expansion   L  [cells][nup] = Lc [cells][rp] U^T      (B stored [n][k], NT)
hipError_t launch_m2l_project(ankh_plan_s *pl) { return launch_m2l_basis(pl, false); }
hipError_t launch_m2l_expand(ankh_plan_s *pl) { return launch_m2l_basis(pl, true); }

}  // namespace ankh
