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
    __bf16 *hi, *lo;   // projection in the split-bf16 mode: C also as bf16 hi / lo parts (same layout), else null
    float *f32;        // projection in the float32 mode: C also in float32 (same layout), else null
    int lda, ldb, ldc, rows, N, K, ntn, tile0;
};
constexpr int kMaxBasisLevels = 8;
struct BasisJob {
    BasisLevel lv[kMaxBasisLevels];
    int nlv, ntiles;
};
constexpr int BT = 32, BKC = 16;   // column tile, contraction chunk

typedef double f64x4 __attribute__((ext_vector_type(4)));

// One wave per 16 x 32 output tile (two 16 x 16 fragments of v_mfma_f64_16x16x4),
// the whole contraction, operands loaded straight from memory one chunk of 16
// ahead; 4 waves (consecutive tiles, mostly of one row band) per block.  Lane
// (r, q) = (lane % 16, lane / 16) supplies A(m0 + r, k) and B(k, n0 + r) of the
// products; within a chunk k0 the 4 sub-steps j take k = k0 + 4 q + j, so each
// lane reads 4 consecutive k of its row of A (the sum over k is the same, in a
// different order).  Result element v of lane (r, q) is C(m0 + q + 4 v, n0 + r).
template <bool NT>
__global__ __launch_bounds__(256) void k_basis(BasisJob job) {
    const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63, r = ln & 15, q = ln >> 4;
    const int v = blockIdx.x * 4 + wv;
    if (v >= job.ntiles) return;
    int li = 0;
    while (li + 1 < job.nlv && v >= job.lv[li + 1].tile0) li++;
    const BasisLevel L = job.lv[li];
    const int tl = v - L.tile0;
    const int m0 = (tl / L.ntn) * 16, n0 = (tl % L.ntn) * BT;
    // rows of A past the level are clamped to its last row; their results are dropped
    const double *Ar = L.A + (int64_t)min(m0 + r, L.rows - 1) * L.lda + 4 * q;
    const double *B0 = NT ? L.B + (int64_t)(n0 + r) * L.ldb + 4 * q : L.B + (int64_t)(4 * q) * L.ldb + n0 + r;
    const int64_t b16 = NT ? 16 * (int64_t)L.ldb : 16;   // column n0 + 16 + r
    struct Op {
        double a[4], b0[4], b1[4];
    };
    auto load = [&](int k0, Op &o) {
        const double2 a01 = *reinterpret_cast<const double2 *>(Ar + k0);
        const double2 a23 = *reinterpret_cast<const double2 *>(Ar + k0 + 2);
        o.a[0] = a01.x, o.a[1] = a01.y, o.a[2] = a23.x, o.a[3] = a23.y;
        if (NT) {
            const double2 p01 = *reinterpret_cast<const double2 *>(B0 + k0);
            const double2 p23 = *reinterpret_cast<const double2 *>(B0 + k0 + 2);
            const double2 s01 = *reinterpret_cast<const double2 *>(B0 + b16 + k0);
            const double2 s23 = *reinterpret_cast<const double2 *>(B0 + b16 + k0 + 2);
            o.b0[0] = p01.x, o.b0[1] = p01.y, o.b0[2] = p23.x, o.b0[3] = p23.y;
            o.b1[0] = s01.x, o.b1[1] = s01.y, o.b1[2] = s23.x, o.b1[3] = s23.y;
        } else {
#pragma unroll
            for (int j = 0; j < 4; j++) {
                o.b0[j] = B0[(int64_t)(k0 + j) * L.ldb];
                o.b1[j] = B0[(int64_t)(k0 + j) * L.ldb + b16];
            }
        }
    };
    f64x4 c0 = {0, 0, 0, 0}, c1 = {0, 0, 0, 0};
    auto mma = [&](const Op &o) {
#pragma unroll
        for (int j = 0; j < 4; j++) {
            c0 = __builtin_amdgcn_mfma_f64_16x16x4f64(o.a[j], o.b0[j], c0, 0, 0, 0);
            c1 = __builtin_amdgcn_mfma_f64_16x16x4f64(o.a[j], o.b1[j], c1, 0, 0, 0);
        }
    };
    // chunks alternate register sets P0 / P1; loads past the last chunk repeat it
    const int nks = L.K / BKC;
    Op P0, P1;
    load(0, P0);
    for (int s = 0; s < nks; s += 2) {
        load(min(s + 1, nks - 1) * BKC, P1);
        mma(P0);
        load(min(s + 2, nks - 1) * BKC, P0);
        if (s + 1 < nks) mma(P1);
    }
#pragma unroll
    for (int e = 0; e < 4; e++) {
        const int m = m0 + q + 4 * e;
        if (m >= L.rows) continue;
#pragma unroll
        for (int h = 0; h < 2; h++) {
            const int64_t o = (int64_t)m * L.ldc + n0 + 16 * h + r;
            const double sum = h ? c1[e] : c0[e];
            L.C[o] = sum;
            if (L.hi) {   // the contraction's operand: hi = bf16(x), lo = bf16(x - hi), x = float(sum)
                const float x = (float)sum;
                const __bf16 a = (__bf16)x;
                L.hi[o] = a;
                L.lo[o] = (__bf16)(x - (float)a);
            }
            if (L.f32) L.f32[o] = (float)sum;
        }
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
            if (pl->precision == ANKH_MIXED_BF16X3) {
                b.hi = pl->d_Mb + pl->mb_off[e];
                b.lo = pl->d_Mb + pl->mb_total + pl->mb_off[e];
            } else if (pl->precision == ANKH_MIXED) {
                b.f32 = pl->d_Mf + pl->mb_off[e];
            }
        } else {
            b.A = Lc, b.lda = rp, b.K = rp;
            b.C = Lf, b.ldc = pl->nup, b.N = pl->nup;
        }
        if (b.K % BKC || b.N % BT || b.rows < 1) return hipErrorInvalidValue;
        b.ntn = b.N / BT;
        b.tile0 = nt;
        nt += ((b.rows + 15) / 16) * b.ntn;
    }
    if (job.nlv == 0) return hipSuccess;
    job.ntiles = nt;
    const dim3 grid((unsigned)((nt + 3) / 4));
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
