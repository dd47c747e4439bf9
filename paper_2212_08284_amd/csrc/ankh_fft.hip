// ANKH-FFT far field (the ANKH-FFT section of the paper): one leaf-level
// operator instead of the multilevel M2L.
//
// The leaf modified charges Q_c (Chebyshev nodes, L per axis) are
// reinterpolated onto an equispaced grid of Le nodes per axis spanning the
// leaf, M_c = E Q_c with E[a][i] = U_a(r_i) (the equispaced Lagrange
// polynomials at the Chebyshev nodes).  The far energy 1/2 v^T A v couples
// every pair of non-adjacent leaves through the kernel between their grid
// nodes.  Per axis the entries of A depend only on the cell difference (modulo
// n = 2^E: the leaf grid is periodic and the image sum of each entry is taken
// over a displacement cube) and on the node difference in -(Le-1)..Le-1, so A
// is a 6D convolution: circular of length n in the cell dimensions and, after
// zero padding to Pa = 2 Le - 1, circular in the node dimensions.  Its
// diagonalisation by the 6D DFT gives (Theorem / Corollary of the
// diagonalisation passage, real spectrum by the corollary on mutual
// interactions)
//     phi = F^-1 (D . F chi v) / N,   D = F K (real),   Lambda_c = E^T phi_c,
// and the energy is the leaf form 1/2 sum_c Q_c . Lambda_c, whose gradient the
// existing L2P stage evaluates.
//
// Layout of the spectrum (float64 complex): X[f][c], f = (f1 Pa + f2) Ph + f3
// over the node frequencies with f3 < Ph = Pa/2 + 1 (the input is real, so the
// other half follows by conjugate symmetry), c the lexicographic leaf index.
// Three kernels per evaluation:
//   k_fft_nodes_fwd  per leaf: E and the node DFT fused into one complex
//                    matrix B = W E per axis (Pa x L), three separable stages
//                    in LDS, the half spectrum written to X[f][c];
//   k_fft_cells      per node frequency: the 3D FFT over the n^3 cells in LDS,
//                    the product with D / N, the inverse 3D FFT, in place
//                    (n <= 16; for 32 and 64 cells per axis three passes
//                    through HBM: k_fft_yz planes, k_fft_x lines with the
//                    product, k_fft_yz inverse; for a grid that is not a
//                    power of two the same three passes with direct DFTs,
//                    k_dft_yz / k_dft_x);
//   k_fft_nodes_inv  per leaf: the adjoint of the first (conj(B)^T per axis,
//                    the half spectrum counted twice), Lambda_c into the leaf
//                    row of the local expansions.
// Plan time: k_fft_table sums the kernel over the images for every entry of
// the generating cube K[g][a] (cell residue g, node difference a), applies the
// node DFT, and k_fft_cells (forward only) leaves D = Re F K.
#include <cmath>
#include <vector>

#include "ankh_internal.h"

namespace ankh {
namespace {

constexpr double kPiF = 3.14159265358979323846;

// Complex values of the working precision: float64 (double2) everywhere in the FP64 mode; float32
// (float2) for the spectrum, the tables and the transforms of an evaluation in the mixed modes.
template <typename R> struct CplxOf;
template <> struct CplxOf<double> { using type = double2; };
template <> struct CplxOf<float> { using type = float2; };
template <typename R> using Cplx = typename CplxOf<R>::type;
__host__ __device__ inline double2 mkc(double a, double b) { return make_double2(a, b); }
__host__ __device__ inline float2 mkc(float a, float b) { return make_float2(a, b); }

// e^{-2 pi i k / 16}, k = 0..7: the roots of unity of every cell FFT (n <= 16)
template <typename R> struct Tw16 {
    Cplx<R> w[8];
};

template <typename C> __device__ inline C cmul(C a, C b) {
    return mkc(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename C> __device__ inline C cmulc(C a, C b) {   // conj(a) * b
    return mkc(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}

// blocks are dealt to the 8 XCDs in turn: give each XCD a contiguous range of
// leaves, so that the partial rows the node kernels write into X[f][.] for
// neighbouring leaves meet in the same L2
__device__ inline int64_t xcd_leaf(int64_t b, int64_t ncell) {
    if (ncell % 8 != 0) return b;
    return (b % 8) * (ncell / 8) + b / 8;
}

// radix-2 FFT of N <= 16 points in registers (decimation in time, bit-reversed
// input order); INV uses the conjugate roots and no scaling
template <typename R, int N, bool INV>
__device__ inline void fft_line(Cplx<R> (&v)[N], const Tw16<R> &tw) {
    using C = Cplx<R>;
    if constexpr (N > 1) {
#pragma unroll
        for (int i = 0; i < N; i++) {
            int j = 0;
#pragma unroll
            for (int b = 1, r = N >> 1; b < N; b <<= 1, r >>= 1)
                if (i & b) j |= r;
            if (i < j) {
                const C t = v[i];
                v[i] = v[j];
                v[j] = t;
            }
        }
#pragma unroll
        for (int len = 2; len <= N; len <<= 1) {
#pragma unroll
            for (int i = 0; i < N; i += len) {
#pragma unroll
                for (int k = 0; k < len / 2; k++) {
                    C w = tw.w[k * (16 / len)];
                    if (INV) w.y = -w.y;
                    const C u = v[i + k], t = cmul(w, v[i + k + len / 2]);
                    v[i + k] = mkc(u.x + t.x, u.y + t.y);
                    v[i + k + len / 2] = mkc(u.x - t.x, u.y - t.y);
                }
            }
        }
    }
}

// the three separable stages of a forward node transform of one real cube
// in[lin^3] (x slowest) with the matrix Bm[pa][lin]: X[(f1 pa + f2) ph + f3] =
// sum_ijk Bm[f1][i] Bm[f2][j] Bm[f3][k] in[i][j][k], written to out[f * ncell]
__device__ void node_forward(const double *in, int lin, const double2 *Bm, int pa, int ph, double2 *T1, double2 *T2,
                             double2 *out, int64_t ncell, int nt) {
    const int t = threadIdx.x;
    const int ll = lin * lin;
    for (int o = t; o < pa * ll; o += nt) {          // x: T1[f1][j][k]
        const int f1 = o / ll, jk = o - f1 * ll;
        double re = 0, im = 0;
        for (int i = 0; i < lin; i++) {
            const double2 b = Bm[f1 * lin + i];
            const double v = in[i * ll + jk];
            re += b.x * v;
            im += b.y * v;
        }
        T1[o] = make_double2(re, im);
    }
    __syncthreads();
    for (int o = t; o < pa * pa * lin; o += nt) {    // y: T2[f1][f2][k]
        const int f1 = o / (pa * lin), r = o - f1 * pa * lin, f2 = r / lin, k = r - f2 * lin;
        double re = 0, im = 0;
        for (int j = 0; j < lin; j++) {
            const double2 b = Bm[f2 * lin + j], v = T1[(f1 * lin + j) * lin + k];
            re += b.x * v.x - b.y * v.y;
            im += b.x * v.y + b.y * v.x;
        }
        T2[o] = make_double2(re, im);
    }
    __syncthreads();
    for (int o = t; o < pa * pa * ph; o += nt) {     // z, half spectrum
        const int f12 = o / ph, f3 = o - f12 * ph;
        double re = 0, im = 0;
        for (int k = 0; k < lin; k++) {
            const double2 b = Bm[f3 * lin + k], v = T2[f12 * lin + k];
            re += b.x * v.x - b.y * v.y;
            im += b.x * v.y + b.y * v.x;
        }
        out[(int64_t)o * ncell] = make_double2(re, im);
    }
}

// ---- per evaluation ------------------------------------------------------------

// one wave per leaf: Q (leaf row of the multipoles) -> X[.][c]
__global__ __launch_bounds__(64) void k_fft_nodes_fwd(const double *Q, int nup, int L, const double2 *B, int pa,
                                                      int ph, double2 *X, int64_t ncell) {
    extern __shared__ double2 sm[];
    double2 *sB = sm, *T1 = sB + pa * L, *T2 = T1 + pa * L * L;
    double *sQ = reinterpret_cast<double *>(T2 + pa * pa * L);
    const int64_t c = xcd_leaf(blockIdx.x, ncell);
    for (int i = threadIdx.x; i < pa * L; i += 64) sB[i] = B[i];
    for (int i = threadIdx.x; i < L * L * L; i += 64) sQ[i] = Q[c * nup + i];
    __syncthreads();
    node_forward(sQ, L, sB, pa, ph, T1, T2, X + c, ncell, 64);
}

// one wave per leaf: X[.][c] -> Lambda_c = Re sum_f conj(B[f1][i] B[f2][j] B[f3][k]) w(f3) X[f][c],
// w = 1 for f3 = 0 (and f3 = pa/2 when pa is even), 2 for the other kept f3
__global__ __launch_bounds__(64) void k_fft_nodes_inv(const double2 *X, const double2 *B, int pa, int ph, int L,
                                                      double *Lam, int nup, int64_t ncell) {
    extern __shared__ double2 sm[];
    double2 *sB = sm, *U = sB + pa * L, *sX = U + pa * pa * L;   // V aliases sX once sX is consumed
    const int64_t c = xcd_leaf(blockIdx.x, ncell);
    const int t = threadIdx.x;
    const int nf = pa * pa * ph;
    for (int i = t; i < pa * L; i += 64) sB[i] = B[i];
    for (int f = t; f < nf; f += 64) sX[f] = X[(int64_t)f * ncell + c];
    __syncthreads();
    for (int o = t; o < pa * pa * L; o += 64) {      // z: U[f1][f2][k]
        const int f12 = o / L, k = o - f12 * L;
        double re = 0, im = 0;
        for (int f3 = 0; f3 < ph; f3++) {
            const double w = (f3 == 0 || 2 * f3 == pa) ? 1.0 : 2.0;
            const double2 v = cmulc(sB[f3 * L + k], sX[f12 * ph + f3]);
            re += w * v.x;
            im += w * v.y;
        }
        U[o] = make_double2(re, im);
    }
    __syncthreads();
    double2 *V = sX;
    for (int o = t; o < pa * L * L; o += 64) {       // y: V[f1][j][k]
        const int f1 = o / (L * L), jk = o - f1 * L * L, j = jk / L, k = jk - j * L;
        double re = 0, im = 0;
        for (int f2 = 0; f2 < pa; f2++) {
            const double2 v = cmulc(sB[f2 * L + j], U[(f1 * pa + f2) * L + k]);
            re += v.x;
            im += v.y;
        }
        V[o] = make_double2(re, im);
    }
    __syncthreads();
    for (int o = t; o < L * L * L; o += 64) {        // x, real part
        const int i = o / (L * L), jk = o - i * L * L;
        double re = 0;
        for (int f1 = 0; f1 < pa; f1++) re += cmulc(sB[f1 * L + i], V[f1 * L * L + jk]).x;
        Lam[c * nup + o] = re;
    }
}

// one block per kept node frequency f: 3D FFT over the NS^3 cells of X[f][.]
// in LDS (element (x, y, z) at ((x NS + y) NS + (z ^ y')), y' = the low bits of
// x NS + y, which spreads every pass over the banks).  MODE 0: forward, times
// D[f][.] * scale, inverse, back to X.  MODE 1 (plan): forward, the real part
// to D.
template <int NS>
__device__ inline int cell_at(int x, int y, int z) {
    const int xy = x * NS + y;
    return xy * NS + (z ^ (xy & (NS - 1)));
}

template <typename R, int NS, int MODE>
__global__ __launch_bounds__(256) void k_fft_cells(Cplx<R> *X, R *D, int64_t ncell, R scale, Tw16<R> tw) {
    using C = Cplx<R>;
    extern __shared__ __align__(16) unsigned char smraw[];
    C *sm = reinterpret_cast<C *>(smraw);
    const int64_t f = blockIdx.x;
    C *xf = X + f * ncell;
    const int t = threadIdx.x;
    constexpr int NL = NS * NS;
    for (int i = t; i < NS * NS * NS; i += 256) {
        const int x = i / NL, y = (i / NS) % NS, z = i % NS;
        sm[cell_at<NS>(x, y, z)] = xf[i];
    }
    __syncthreads();
    C v[NS];
    if (t < NL) {                                   // z lines
        const int x = t / NS, y = t % NS;
#pragma unroll
        for (int z = 0; z < NS; z++) v[z] = sm[cell_at<NS>(x, y, z)];
        fft_line<R, NS, false>(v, tw);
#pragma unroll
        for (int z = 0; z < NS; z++) sm[cell_at<NS>(x, y, z)] = v[z];
    }
    __syncthreads();
    if (t < NL) {                                   // y lines
        const int x = t / NS, z = t % NS;
#pragma unroll
        for (int y = 0; y < NS; y++) v[y] = sm[cell_at<NS>(x, y, z)];
        fft_line<R, NS, false>(v, tw);
#pragma unroll
        for (int y = 0; y < NS; y++) sm[cell_at<NS>(x, y, z)] = v[y];
    }
    __syncthreads();
    if (t < NL) {                                   // x lines, the product with D, and back along x
        const int y = t / NS, z = t % NS;
#pragma unroll
        for (int x = 0; x < NS; x++) v[x] = sm[cell_at<NS>(x, y, z)];
        fft_line<R, NS, false>(v, tw);
        if (MODE == 1) {
#pragma unroll
            for (int x = 0; x < NS; x++) D[f * ncell + (x * NS + y) * NS + z] = v[x].x;
        } else {
#pragma unroll
            for (int x = 0; x < NS; x++) {
                const R d = D[f * ncell + (x * NS + y) * NS + z] * scale;
                v[x] = mkc(v[x].x * d, v[x].y * d);
            }
            fft_line<R, NS, true>(v, tw);
#pragma unroll
            for (int x = 0; x < NS; x++) sm[cell_at<NS>(x, y, z)] = v[x];
        }
    }
    if (MODE == 1) return;
    __syncthreads();
    if (t < NL) {                                   // y lines, inverse
        const int x = t / NS, z = t % NS;
#pragma unroll
        for (int y = 0; y < NS; y++) v[y] = sm[cell_at<NS>(x, y, z)];
        fft_line<R, NS, true>(v, tw);
#pragma unroll
        for (int y = 0; y < NS; y++) sm[cell_at<NS>(x, y, z)] = v[y];
    }
    __syncthreads();
    if (t < NL) {                                   // z lines, inverse
        const int x = t / NS, y = t % NS;
#pragma unroll
        for (int z = 0; z < NS; z++) v[z] = sm[cell_at<NS>(x, y, z)];
        fft_line<R, NS, true>(v, tw);
#pragma unroll
        for (int z = 0; z < NS; z++) sm[cell_at<NS>(x, y, z)] = v[z];
    }
    __syncthreads();
    for (int i = t; i < NS * NS * NS; i += 256) {
        const int x = i / NL, y = (i / NS) % NS, z = i % NS;
        xf[i] = sm[cell_at<NS>(x, y, z)];
    }
}

// ---- per evaluation, equispaced order = Chebyshev order (pa = 2L - 1, ph = L) --
// Consecutive leaves per block (the blocks of one XCD take consecutive leaves),
// each spectrum row X[f][.] written or read in runs of one value per leaf: the
// forward transform takes eight leaves (128-byte runs; 512 threads, the x stage
// through LDS, y and z fused in registers), the inverse four (64-byte runs; eight
// per block made it slower at its larger LDS footprint).  B is read from LDS where
// its row varies across lanes, with uniform addresses otherwise.
constexpr int kCB = 4;
constexpr int kCF = 8, kFT = 512;

template <typename R, int L>
__global__ __launch_bounds__(kFT) void k_fft_nodes_fwd_t(const double *Q, int nup, const Cplx<R> *B, Cplx<R> *X,
                                                         int64_t ncell) {
    using C = Cplx<R>;
    constexpr int PA = 2 * L - 1, PH = L, NQ = L * L * L, NT1 = PA * L * L;
    __shared__ R sQ[kCF][NQ];
    __shared__ C T1[kCF][NT1];
    __shared__ C sB[PA * L];
    const int64_t c0 = xcd_leaf(blockIdx.x, ncell / kCF) * kCF;
    const int t = threadIdx.x;
    for (int i = t; i < kCF * NQ; i += kFT) sQ[i / NQ][i % NQ] = Q[(c0 + i / NQ) * nup + i % NQ];
    for (int i = t; i < PA * L; i += kFT) sB[i] = B[i];
    __syncthreads();
    // x: thread (cell, f1, j, k): T1[f1][j][k] = sum_i B[f1][i] Q[i][j][k]
    for (int o = t; o < kCF * NT1; o += kFT) {
        const int cell = o / NT1, r = o - cell * NT1, f1 = r / (L * L), jk = r - f1 * L * L;
        R re = 0, im = 0;
#pragma unroll
        for (int i = 0; i < L; i++) {
            const C b = sB[f1 * L + i];
            const R q = sQ[cell][i * L * L + jk];
            re += b.x * q;
            im += b.y * q;
        }
        T1[cell][r] = mkc(re, im);
    }
    __syncthreads();
    // y and z, half spectrum: thread (line f1 f2, cell), the kCF cells of a line adjacent lanes:
    // v[k] = sum_j B[f2][j] T1[f1][j][k], then X[f1 f2 f3] = sum_k B[f3][k] v[k]
    for (int o = t; o < kCF * PA * PA; o += kFT) {
        const int cell = o % kCF, f12 = o / kCF, f1 = f12 / PA, f2 = f12 - f1 * PA;
        const C *t1 = &T1[cell][f1 * L * L];
        C v[L];
#pragma unroll
        for (int k = 0; k < L; k++) v[k] = mkc((R)0, (R)0);
#pragma unroll
        for (int j = 0; j < L; j++) {
            const C b = sB[f2 * L + j];
#pragma unroll
            for (int k = 0; k < L; k++) {
                const C u = t1[j * L + k];
                v[k].x += b.x * u.x - b.y * u.y;
                v[k].y += b.x * u.y + b.y * u.x;
            }
        }
#pragma unroll
        for (int f3 = 0; f3 < PH; f3++) {
            R re = 0, im = 0;
#pragma unroll
            for (int k = 0; k < L; k++) {
                const C b = B[f3 * L + k];
                re += b.x * v[k].x - b.y * v[k].y;
                im += b.x * v[k].y + b.y * v[k].x;
            }
            X[(int64_t)(f12 * PH + f3) * ncell + c0 + cell] = mkc(re, im);
        }
    }
}

// In float32 it also gives the leaf's far energy 1/2 Q_c . Lambda_c with Lambda_c (each thread's L
// products, then the L^2 threads of a leaf in order), which otherwise k_leafdot computes (in float64
// the extra registers would spill).
template <typename R, int L>
__global__ __launch_bounds__(256) void k_fft_nodes_inv_t(const Cplx<R> *X, const Cplx<R> *B, double *Lam,
                                                         const double *Q, double *eleaf, int nup, int64_t ncell) {
    using C = Cplx<R>;
    constexpr int PA = 2 * L - 1, PH = L, NU = PA * PA * L;
    __shared__ C U[kCB][NU];
    __shared__ double part[sizeof(R) == 4 ? kCB : 1][sizeof(R) == 4 ? L * L : 1];
    const int64_t c0 = xcd_leaf(blockIdx.x, ncell / kCB) * kCB;
    const int t = threadIdx.x;
    // z: thread (line f1 f2, cell): U[f1][f2][k] = sum_f3 w(f3) conj(B[f3][k]) X[f1 f2 f3]; two lines
    // per thread and round, the loads of both issued first (a second line past the end reads the
    // last line again and is not stored)
    constexpr int NZ = kCB * PA * PA;
    for (int o0 = t; o0 < NZ; o0 += 512) {
        C x[2][PH];
#pragma unroll
        for (int h = 0; h < 2; h++) {
            const int o = min(o0 + 256 * h, NZ - 1), cell = o % kCB, f12 = o / kCB;
#pragma unroll
            for (int f3 = 0; f3 < PH; f3++) x[h][f3] = X[(int64_t)(f12 * PH + f3) * ncell + c0 + cell];
        }
#pragma unroll
        for (int h = 0; h < 2; h++) {
            const int o = o0 + 256 * h, cell = o % kCB, f12 = o / kCB;
            if (o >= NZ) break;
#pragma unroll
            for (int k = 0; k < L; k++) {
                R re = 0, im = 0;
#pragma unroll
                for (int f3 = 0; f3 < PH; f3++) {
                    const R w = f3 == 0 ? 1.0 : 2.0;       // pa odd: no unpaired frequency besides 0
                    const C v = cmulc(B[f3 * L + k], x[h][f3]);
                    re += w * v.x;
                    im += w * v.y;
                }
                U[cell][f12 * L + k] = mkc(re, im);
            }
        }
    }
    __syncthreads();
    // y and x: thread (cell, j, k): v[f1] = sum_f2 conj(B[f2][j]) U[f1][f2][k],
    // Lambda[i][j][k] = Re sum_f1 conj(B[f1][i]) v[f1]
    for (int o = t; o < kCB * L * L; o += 256) {
        const int cell = o / (L * L), jk = o - cell * L * L, j = jk / L, k = jk - j * L;
        C v[PA];
#pragma unroll
        for (int f1 = 0; f1 < PA; f1++) {
            R re = 0, im = 0;
#pragma unroll
            for (int f2 = 0; f2 < PA; f2++) {
                const C u = cmulc(B[f2 * L + j], U[cell][(f1 * PA + f2) * L + k]);
                re += u.x;
                im += u.y;
            }
            v[f1] = mkc(re, im);
        }
        double e = 0;
#pragma unroll
        for (int i = 0; i < L; i++) {
            R re = 0;
#pragma unroll
            for (int f1 = 0; f1 < PA; f1++) re += cmulc(B[f1 * L + i], v[f1]).x;
            const int64_t at = (c0 + cell) * nup + (i * L + j) * L + k;
            Lam[at] = re;
            if constexpr (sizeof(R) == 4) e += Q[at] * (double)re;
        }
        if constexpr (sizeof(R) == 4) part[cell][jk] = e;
    }
    if constexpr (sizeof(R) == 4) {
        __syncthreads();
        if (t < kCB) {
            double e = 0;
            for (int jk = 0; jk < L * L; jk++) e += part[t][jk];
            eleaf[c0 + t] = 0.5 * e;
        }
    }
}

// ---- plan time: the generating cube of A and its node DFT --------------------

// one block per cell residue g = (gx, gy, gz): K[g][a] for every node difference a (a < Le: a,
// a > Pa - Le: a - Pa) summed over the cell displacements D = g - n I with |D_axis| <= n (p + 1/2)
// and max |D| >= 2, then the node DFT (plain roots W[f][a]) into X[.][g]
__global__ __launch_bounds__(256) void k_fft_table(const double2 *W, int pa, int ph, int le, int nside, int p,
                                                   double w, double h, double xi, double2 *X, int64_t ncell) {
    extern __shared__ double2 sm[];
    double2 *sW = sm;
    double *cube = reinterpret_cast<double *>(sW + pa * pa);
    const int64_t g = blockIdx.x;
    const int gx = (int)(g / ((int64_t)nside * nside)), gy = (int)((g / nside) % nside), gz = (int)(g % nside);
    const int t = threadIdx.x;
    for (int i = t; i < pa * pa; i += 256) sW[i] = W[i];
    const double lim = nside * (p + 0.5);
    const int n3 = pa * pa * pa;
    for (int e = t; e < n3; e += 256) {
        const int a1 = e / (pa * pa), a2 = (e / pa) % pa, a3 = e % pa;
        const int d1 = a1 < le ? a1 : a1 - pa, d2 = a2 < le ? a2 : a2 - pa, d3 = a3 < le ? a3 : a3 - pa;
        double s = 0;
        for (int I = -p - 2; I <= p + 2; I++) {
            const int Dx = gx - nside * I;
            if (fabs((double)Dx) > lim) continue;
            const double zx = Dx * w + d1 * h;
            for (int J = -p - 2; J <= p + 2; J++) {
                const int Dy = gy - nside * J;
                if (fabs((double)Dy) > lim) continue;
                const double zy = Dy * w + d2 * h;
                for (int K = -p - 2; K <= p + 2; K++) {
                    const int Dz = gz - nside * K;
                    if (fabs((double)Dz) > lim) continue;
                    if (abs(Dx) < 2 && abs(Dy) < 2 && abs(Dz) < 2) continue;
                    const double zz = Dz * w + d3 * h;
                    const double r = sqrt(zx * zx + zy * zy + zz * zz);
                    s += erfc(xi * r) / r;
                }
            }
        }
        cube[e] = s;
    }
    __syncthreads();
    // direct node DFT (plan time only): out[f1][f2][f3] = sum_a W[f1][a1] W[f2][a2] W[f3][a3] K[a]
    for (int o = t; o < pa * pa * ph; o += 256) {
        const int f1 = o / (pa * ph), f2 = (o / ph) % pa, f3 = o % ph;
        double re = 0, im = 0;
        for (int a1 = 0; a1 < pa; a1++) {
            const double2 w1 = sW[f1 * pa + a1];
            for (int a2 = 0; a2 < pa; a2++) {
                const double2 w12 = cmul(w1, sW[f2 * pa + a2]);
                const double *row = cube + (a1 * pa + a2) * pa;
                double sr = 0, si = 0;
                for (int a3 = 0; a3 < pa; a3++) {
                    const double2 w3 = sW[f3 * pa + a3];
                    sr += w3.x * row[a3];
                    si += w3.y * row[a3];
                }
                re += w12.x * sr - w12.y * si;
                im += w12.x * si + w12.y * sr;
            }
        }
        X[(int64_t)o * ncell + g] = make_double2(re, im);
    }
}

// ---- cell transforms in three passes (32^3 or 64^3 cells, or on request) -----
// A tile of NS x NS complex values in LDS, element (u, v) at u NS + v, is
// transformed along v (ALONG_V) or along u by radix-2 butterflies, one per
// thread and stage.  tile_dit: bit-reversed input, natural output; tile_dif:
// natural input, bit-reversed output.  tw[k] = e^{-2 pi i k / NS}, k < NS/2
// (global, cached); INV conjugates it.
template <int NS>
__device__ inline int brev(int v) {
    constexpr int bits = NS == 2 ? 1 : NS == 4 ? 2 : NS == 8 ? 3 : NS == 16 ? 4 : NS == 32 ? 5 : 6;
    return (int)(__brev((unsigned)v) >> (32 - bits));
}

template <typename R, int NS, bool ALONG_V, bool DIT, bool INV>
__device__ void tile_fft(Cplx<R> *tile, const Cplx<R> *tw) {
    using C = Cplx<R>;
    constexpr int Q4 = NS >= 4 ? NS / 4 : 1;   // pairs of stages exist from 4 points on
    constexpr int NB = NS * (NS / 2), NQ = NS * Q4;
    auto twid = [&](int pos, int h) {           // W_{2h}^pos (conjugated for INV)
        C w = tw[pos * (NS / (2 * h))];
        if (INV) w.y = -w.y;
        return w;
    };
    auto at = [&](int line, int i) -> C & { return tile[ALONG_V ? line * NS + i : i * NS + line]; };
    // Two radix-2 stages at a time where two remain (the butterflies of both stages on the four values
    // p, p + h, p + 2h, p + 3h in one thread, operation for operation as in two stages), one barrier per
    // pair of stages; a single radix-2 stage where one remains.
    // DIT: half 1, 2, 4, ... (stages h and 2h together); DIF: half NS/2, NS/4, ... (h and h/2).
    int half = DIT ? 1 : NS / 2;
    while (DIT ? half < NS : half >= 1) {
        const bool pair = NS >= 4 && (DIT ? 2 * half < NS : half >= 2);
        if (pair) {
            const int hq = DIT ? half : half / 2;   // the smaller half of the two stages
            for (int b = threadIdx.x; b < NQ; b += blockDim.x) {
                const int line = ALONG_V ? b / Q4 : b % NS;
                const int k = ALONG_V ? b % Q4 : b / NS;
                const int pos = k % hq, p = (k / hq) * 4 * hq + pos;
                C x0 = at(line, p), x1 = at(line, p + hq), x2 = at(line, p + 2 * hq), x3 = at(line, p + 3 * hq);
                if (DIT) {
                    // stage hq: (p, p + hq), (p + 2hq, p + 3hq) with W_{2hq}^pos
                    const C w1 = twid(pos, hq);
                    const C t1 = cmul(w1, x1), t3 = cmul(w1, x3);
                    const C u0 = mkc(x0.x + t1.x, x0.y + t1.y), u1 = mkc(x0.x - t1.x, x0.y - t1.y);
                    const C u2 = mkc(x2.x + t3.x, x2.y + t3.y), u3 = mkc(x2.x - t3.x, x2.y - t3.y);
                    // stage 2hq: (p, p + 2hq) with W_{4hq}^pos, (p + hq, p + 3hq) with W_{4hq}^(pos + hq)
                    const C w2 = twid(pos, 2 * hq), w3 = twid(pos + hq, 2 * hq);
                    const C t2 = cmul(w2, u2), t4 = cmul(w3, u3);
                    at(line, p) = mkc(u0.x + t2.x, u0.y + t2.y);
                    at(line, p + 2 * hq) = mkc(u0.x - t2.x, u0.y - t2.y);
                    at(line, p + hq) = mkc(u1.x + t4.x, u1.y + t4.y);
                    at(line, p + 3 * hq) = mkc(u1.x - t4.x, u1.y - t4.y);
                } else {
                    // stage 2hq: (p, p + 2hq) with W_{4hq}^pos, (p + hq, p + 3hq) with W_{4hq}^(pos + hq)
                    const C w2 = twid(pos, 2 * hq), w3 = twid(pos + hq, 2 * hq);
                    const C u0 = mkc(x0.x + x2.x, x0.y + x2.y), u2 = cmul(w2, mkc(x0.x - x2.x, x0.y - x2.y));
                    const C u1 = mkc(x1.x + x3.x, x1.y + x3.y), u3 = cmul(w3, mkc(x1.x - x3.x, x1.y - x3.y));
                    // stage hq: (p, p + hq), (p + 2hq, p + 3hq) with W_{2hq}^pos
                    const C w1 = twid(pos, hq);
                    at(line, p) = mkc(u0.x + u1.x, u0.y + u1.y);
                    at(line, p + hq) = cmul(w1, mkc(u0.x - u1.x, u0.y - u1.y));
                    at(line, p + 2 * hq) = mkc(u2.x + u3.x, u2.y + u3.y);
                    at(line, p + 3 * hq) = cmul(w1, mkc(u2.x - u3.x, u2.y - u3.y));
                }
            }
            half = DIT ? 4 * half : half / 4;
        } else {
            for (int b = threadIdx.x; b < NB; b += blockDim.x) {
                // consecutive threads take consecutive elements of the line direction that is contiguous
                const int line = ALONG_V ? b / (NS / 2) : b % NS;
                const int k = ALONG_V ? b % (NS / 2) : b / NS;
                const int pos = k % half, i0 = (k / half) * 2 * half + pos, i1 = i0 + half;
                const C w = twid(pos, half);
                const C u = at(line, i0), v = at(line, i1);
                if (DIT) {
                    const C t = cmul(w, v);
                    at(line, i0) = mkc(u.x + t.x, u.y + t.y);
                    at(line, i1) = mkc(u.x - t.x, u.y - t.y);
                } else {
                    at(line, i0) = mkc(u.x + v.x, u.y + v.y);
                    at(line, i1) = cmul(w, mkc(u.x - v.x, u.y - v.y));
                }
            }
            half = DIT ? 2 * half : half / 2;
        }
        __syncthreads();
    }
}

// pass 1 / 3: block (f, x), the (y, z) plane of X[f] (contiguous): forward (DIT, natural output) or
// inverse (DIF, written back in natural order)
template <typename R, int NS, bool INV>
__global__ __launch_bounds__(256) void k_fft_yz(Cplx<R> *X, const Cplx<R> *tw, int64_t ncell) {
    using C = Cplx<R>;
    __shared__ C tile[NS * NS];
    __shared__ C stw[NS / 2];
    C *p = X + (int64_t)blockIdx.x * ncell + (int64_t)blockIdx.y * NS * NS;
    const int t = threadIdx.x;
    for (int i = t; i < NS / 2; i += 256) stw[i] = tw[i];
    for (int i = t; i < NS * NS; i += 256) {
        const int y = i / NS, z = i % NS;
        tile[INV ? i : brev<NS>(y) * NS + brev<NS>(z)] = p[i];
    }
    __syncthreads();
    if (!INV) {
        tile_fft<R, NS, true, true, false>(tile, stw);
        tile_fft<R, NS, false, true, false>(tile, stw);
    } else {
        tile_fft<R, NS, true, false, true>(tile, stw);
        tile_fft<R, NS, false, false, true>(tile, stw);
    }
    for (int i = t; i < NS * NS; i += 256) {
        const int y = i / NS, z = i % NS;
        p[i] = tile[INV ? brev<NS>(y) * NS + brev<NS>(z) : i];
    }
}

// pass 2: block (f, y), the (x, z) tile of X[f]: forward along x, then MODE 0: times D * scale and the
// inverse along x, back to X; MODE 1 (plan): the real part to D
template <typename R, int NS, int MODE>
__global__ __launch_bounds__(256) void k_fft_x(Cplx<R> *X, R *D, const Cplx<R> *tw, int64_t ncell,
                                               R scale) {
    using C = Cplx<R>;
    __shared__ C tile[NS * NS];
    __shared__ C stw[NS / 2];
    const int64_t f = blockIdx.x;
    const int y = blockIdx.y, t = threadIdx.x;
    for (int i = t; i < NS / 2; i += 256) stw[i] = tw[i];
    for (int i = t; i < NS * NS; i += 256) {
        const int x = i / NS, z = i % NS;
        tile[brev<NS>(x) * NS + z] = X[f * ncell + ((int64_t)x * NS + y) * NS + z];
    }
    __syncthreads();
    tile_fft<R, NS, false, true, false>(tile, stw);
    if (MODE == 1) {
        for (int i = t; i < NS * NS; i += 256) {
            const int x = i / NS, z = i % NS;
            D[f * ncell + ((int64_t)x * NS + y) * NS + z] = tile[i].x;
        }
        return;
    }
    for (int i = t; i < NS * NS; i += 256) {
        const int x = i / NS, z = i % NS;
        const R d = D[f * ncell + ((int64_t)x * NS + y) * NS + z] * scale;
        tile[i] = mkc(tile[i].x * d, tile[i].y * d);
    }
    __syncthreads();
    tile_fft<R, NS, false, false, true>(tile, stw);
    for (int i = t; i < NS * NS; i += 256) {
        const int x = i / NS, z = i % NS;
        X[f * ncell + ((int64_t)x * NS + y) * NS + z] = tile[brev<NS>(x) * NS + z];
    }
}

// ---- cell transforms on grids that are not powers of two ------------------------
// Direct DFT along one direction of an n x n tile (element (u, v) at u n + v), from A into B:
// B[..k..] = sum_j A[..j..] w^{jk}, w = e^{-/+ 2 pi i / n} (tw[m] = e^{-2 pi i m / n}, m < n, in LDS).
__device__ void tile_dft(const double2 *A, double2 *B, const double2 *tw, int n, bool along_v, bool inv) {
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
        const int u = e / n, v = e - u * n;
        const int k = along_v ? v : u;
        double re = 0, im = 0;
        int m = 0;
        for (int j = 0; j < n; j++) {
            const double2 x = along_v ? A[u * n + j] : A[j * n + v];
            const double2 w = tw[m];
            const double wy = inv ? -w.y : w.y;
            re += x.x * w.x - x.y * wy;
            im += x.x * wy + x.y * w.x;
            m += k;
            if (m >= n) m -= n;
        }
        B[e] = make_double2(re, im);
    }
    __syncthreads();
}

// pass 1 / 3: block (f, x), the (y, z) plane, forward or inverse
__global__ __launch_bounds__(256) void k_dft_yz(double2 *X, const double2 *twg, int n, int64_t ncell, int inv) {
    extern __shared__ double2 sm[];
    double2 *A = sm, *B = A + n * n, *tw = B + n * n;
    double2 *p = X + (int64_t)blockIdx.x * ncell + (int64_t)blockIdx.y * n * n;
    for (int i = threadIdx.x; i < n; i += 256) tw[i] = twg[i];
    for (int i = threadIdx.x; i < n * n; i += 256) A[i] = p[i];
    __syncthreads();
    tile_dft(A, B, tw, n, true, inv != 0);
    tile_dft(B, A, tw, n, false, inv != 0);
    for (int i = threadIdx.x; i < n * n; i += 256) p[i] = A[i];
}

// pass 2: block (f, y), the (x, z) tile: forward along x, then MODE 0: times D * scale and the inverse,
// MODE 1 (plan): the real part to D
__global__ __launch_bounds__(256) void k_dft_x(double2 *X, double *D, const double2 *twg, int n, int64_t ncell,
                                               double scale, int mode) {
    extern __shared__ double2 sm[];
    double2 *A = sm, *B = A + n * n, *tw = B + n * n;
    const int64_t f = blockIdx.x;
    const int y = blockIdx.y;
    for (int i = threadIdx.x; i < n; i += 256) tw[i] = twg[i];
    for (int i = threadIdx.x; i < n * n; i += 256) {
        const int x = i / n, z = i - x * n;
        A[i] = X[f * ncell + ((int64_t)x * n + y) * n + z];
    }
    __syncthreads();
    tile_dft(A, B, tw, n, false, false);
    for (int i = threadIdx.x; i < n * n; i += 256) {
        const int x = i / n, z = i - x * n;
        const int64_t g = f * ncell + ((int64_t)x * n + y) * n + z;
        if (mode == 1) D[g] = B[i].x;
        else B[i] = make_double2(B[i].x * D[g] * scale, B[i].y * D[g] * scale);
    }
    if (mode == 1) return;
    __syncthreads();
    tile_dft(B, A, tw, n, false, true);
    for (int i = threadIdx.x; i < n * n; i += 256) {
        const int x = i / n, z = i - x * n;
        X[f * ncell + ((int64_t)x * n + y) * n + z] = A[i];
    }
}

// Transforms of N = 4 N2 points along one direction of LDS tiles (Cooley-Tukey, n = n1 + 4 n2,
// k = k2 + N2 k1), in place in two phases separated by a barrier:
//   forward: phase 1, per (line, n1): y[n1 + 4 k2] = W^{n1 k2} sum_n2 x[n1 + 4 n2] W^{4 n2 k2};
//            phase 2, per (line, k2): the 4-point transforms of y[4 k2 .. 4 k2 + 3] (roots +-1, +-i),
//            X[k2 + N2 k1] left at position 4 k2 + k1 (digit-reversed);
//   inverse: the same phases in reverse order with conjugate roots, from that order back to natural.
// Pointwise products in between see every axis in the same permuted order, D included (it is built
// by the same forward transform), so the permutation never needs undoing.  W = e^{-2 pi i / N},
// tw[m] = W^m in LDS.  Element j of line `line` of tile `tile`: t[tile N^2 + (ALONG_V ? line N + j :
// j N + line)].
// the N2-th roots of unity e^{-2 pi i m / N2} (= W^{4m}, W = e^{-2 pi i / (4 N2)}) as compile-time
// constants for the direct small transforms (three and five points; six points are factored, see
// dft_small): cos and sin of multiples of 120 and 72 degrees from their closed forms, rounded to double
template <int N2> struct Roots;
template <> struct Roots<3> {
    static constexpr double re[3] = {1.0, -0.5, -0.5};
    static constexpr double im[3] = {0.0, -0.8660254037844386, 0.8660254037844386};
};
template <> struct Roots<5> {
    static constexpr double re[5] = {1.0, 0.30901699437494745, -0.8090169943749475, -0.8090169943749475,
                                     0.30901699437494745};
    static constexpr double im[5] = {0.0, -0.9510565162951535, -0.5877852522924731, 0.5877852522924731,
                                     0.9510565162951535};
};

// y[k] = sum_n x[n] w^(n k) over N2 points, w = e^(-2 pi i / N2) (forward) or its conjugate (inverse).
// Six points: two 3-point transforms of the even and odd samples, the odd ones twiddled by w^k, and
// 2-point butterflies (y[k] and y[k + 3] = E[k] +- w^k O[k]): 44 real operations instead of the ~120 of
// the direct sum.  Other sizes: the direct sum, the roots as constants, the unit ones as additions.
template <typename R, int N2, bool INV>
__device__ inline void dft_small(const Cplx<R> (&x)[N2], Cplx<R> (&y)[N2]) {
    using C = Cplx<R>;
    if constexpr (N2 == 6) {
        constexpr R h = (R)0.8660254037844386;   // sin(pi / 3)
        // 3-point transform of (a, b, c): a + b + c, m -+ i h t, m +- i h t (m = a - (b + c) / 2, t = b - c)
        auto dft3 = [&](const C &a, const C &b, const C &c, C &o0, C &o1, C &o2) {
            const C t1 = mkc(b.x + c.x, b.y + c.y), t2 = mkc(b.x - c.x, b.y - c.y);
            o0 = mkc(a.x + t1.x, a.y + t1.y);
            const C m = mkc(a.x - (R)0.5 * t1.x, a.y - (R)0.5 * t1.y);
            const C it = INV ? mkc(-h * t2.y, h * t2.x) : mkc(h * t2.y, -h * t2.x);   // +-i h t
            o1 = mkc(m.x + it.x, m.y + it.y);
            o2 = mkc(m.x - it.x, m.y - it.y);
        };
        C e0, e1, e2, o0, o1, o2;
        dft3(x[0], x[2], x[4], e0, e1, e2);
        dft3(x[1], x[3], x[5], o0, o1, o2);
        // w^1 = 1/2 -+ i h, w^2 = -1/2 -+ i h (forward: minus)
        const R sg = INV ? (R)1 : (R)-1;
        const C p1 = mkc((R)0.5 * o1.x - sg * h * o1.y, (R)0.5 * o1.y + sg * h * o1.x);
        const C p2 = mkc((R)-0.5 * o2.x - sg * h * o2.y, (R)-0.5 * o2.y + sg * h * o2.x);
        y[0] = mkc(e0.x + o0.x, e0.y + o0.y);
        y[3] = mkc(e0.x - o0.x, e0.y - o0.y);
        y[1] = mkc(e1.x + p1.x, e1.y + p1.y);
        y[4] = mkc(e1.x - p1.x, e1.y - p1.y);
        y[2] = mkc(e2.x + p2.x, e2.y + p2.y);
        y[5] = mkc(e2.x - p2.x, e2.y - p2.y);
    } else {
#pragma unroll
        for (int k = 0; k < N2; k++) {
            R re = 0, im = 0;
#pragma unroll
            for (int n = 0; n < N2; n++) {
                if ((n * k) % N2 == 0) {         // root 1
                    re += x[n].x;
                    im += x[n].y;
                    continue;
                }
                const R wx = Roots<N2>::re[(n * k) % N2], wy = Roots<N2>::im[(n * k) % N2];
                if (INV) {
                    re += x[n].x * wx + x[n].y * wy;
                    im += x[n].y * wx - x[n].x * wy;
                } else {
                    re += x[n].x * wx - x[n].y * wy;
                    im += x[n].x * wy + x[n].y * wx;
                }
            }
            y[k] = mkc(re, im);
        }
    }
}

template <typename R, int N2, bool ALONG_V, bool INV, int ROW = 4 * N2>
__device__ inline void tiles_phase1(Cplx<R> *t, int ntile, const Cplx<R> *tw) {
    using C = Cplx<R>;
    constexpr int N = 4 * N2;
    constexpr int NL = ALONG_V ? N : ROW;     // lines per tile
    // the N2-point transforms take their roots as constants, and each task reads its twiddles before
    // its stores (the tile and the table share the LDS, so a table read after a store is issued again)
    for (int task = threadIdx.x; task < ntile * NL * 4; task += blockDim.x) {
        // consecutive threads: consecutive elements of the contiguous direction
        int tile, line, n1;
        tile = task / (NL * 4);
        const int r = task - tile * NL * 4;
        if (ALONG_V) { line = r / 4; n1 = r % 4; }
        else { n1 = r / NL; line = r % NL; }
        C *b = t + tile * N * ROW;
        auto at = [&](int j) -> C & { return b[ALONG_V ? line * ROW + j : j * ROW + line]; };
        C wt[N2];                      // W^{n1 k2}, n1 k2 < N
#pragma unroll
        for (int k2 = 0; k2 < N2; k2++) wt[k2] = tw[n1 * k2];
        if (!INV) {
            C x[N2], y[N2];
#pragma unroll
            for (int n2 = 0; n2 < N2; n2++) x[n2] = at(n1 + 4 * n2);
            dft_small<R, N2, false>(x, y);
#pragma unroll
            for (int k2 = 0; k2 < N2; k2++) {
                const C w = wt[k2];
                at(n1 + 4 * k2) = k2 == 0 ? y[k2] : mkc(y[k2].x * w.x - y[k2].y * w.y, y[k2].x * w.y + y[k2].y * w.x);
            }
        } else {
            // inverse of phase 1: z[n1 + 4 k2] times conj W^{n1 k2}, then the conjugate N2-point transform
            C z[N2], y[N2];
#pragma unroll
            for (int k2 = 0; k2 < N2; k2++) {
                const C v = at(n1 + 4 * k2), w = wt[k2];
                z[k2] = k2 == 0 ? v : mkc(v.x * w.x + v.y * w.y, v.y * w.x - v.x * w.y);
            }
            dft_small<R, N2, true>(z, y);
#pragma unroll
            for (int n2 = 0; n2 < N2; n2++) at(n1 + 4 * n2) = y[n2];
        }
    }
    __syncthreads();
}

template <typename R, int N2, bool ALONG_V, bool INV, int ROW = 4 * N2>
__device__ inline void tiles_phase2(Cplx<R> *t, int ntile) {
    using C = Cplx<R>;
    constexpr int N = 4 * N2;
    constexpr int NL = ALONG_V ? N : ROW;
    for (int task = threadIdx.x; task < ntile * NL * N2; task += blockDim.x) {
        int tile, line, k2;
        tile = task / (NL * N2);
        const int r = task - tile * NL * N2;
        if (ALONG_V) { line = r / N2; k2 = r % N2; }
        else { k2 = r / NL; line = r % NL; }
        C *b = t + tile * N * ROW;
        auto at = [&](int j) -> C & { return b[ALONG_V ? line * ROW + j : j * ROW + line]; };
        const C a = at(4 * k2), bb = at(4 * k2 + 1), c = at(4 * k2 + 2), d = at(4 * k2 + 3);
        const C s0 = mkc(a.x + c.x, a.y + c.y), s1 = mkc(a.x - c.x, a.y - c.y);
        const C s2 = mkc(bb.x + d.x, bb.y + d.y), s3 = mkc(bb.x - d.x, bb.y - d.y);
        // (-i)^{n1 k1} forward, i^{n1 k1} inverse
        const C js3 = INV ? mkc(-s3.y, s3.x) : mkc(s3.y, -s3.x);
        at(4 * k2) = mkc(s0.x + s2.x, s0.y + s2.y);
        at(4 * k2 + 1) = mkc(s1.x + js3.x, s1.y + js3.y);
        at(4 * k2 + 2) = mkc(s0.x - s2.x, s0.y - s2.y);
        at(4 * k2 + 3) = mkc(s1.x - js3.x, s1.y - js3.y);
    }
    __syncthreads();
}

// one axis of every tile: forward (natural -> digit-reversed) or inverse (digit-reversed -> natural)
template <typename R, int N2, bool ALONG_V, bool INV, int ROW = 4 * N2>
__device__ inline void tiles_axis(Cplx<R> *t, int ntile, const Cplx<R> *tw) {
    if (!INV) {
        tiles_phase1<R, N2, ALONG_V, false, ROW>(t, ntile, tw);
        tiles_phase2<R, N2, ALONG_V, false, ROW>(t, ntile);
    } else {
        tiles_phase2<R, N2, ALONG_V, true, ROW>(t, ntile);
        tiles_phase1<R, N2, ALONG_V, true, ROW>(t, ntile, tw);
    }
}

// all N^3 cells of one node frequency in LDS (dynamic: N^3 + N complex values; 128 KB at N = 20, used
// where the device allows that much per block): the three axes forward, the product with D (MODE 0,
// then the inverse of the three axes) or its real part to D (MODE 1).  40 B of HBM per value.
constexpr int kAllThreads = 1024;

template <typename R, int N2, int MODE>
__global__ __launch_bounds__(kAllThreads) void k_rdft_all(Cplx<R> *X, R *D, const Cplx<R> *twg, int64_t ncell,
                                                          R scale) {
    using C = Cplx<R>;
    constexpr int N = 4 * N2, NN = N * N, N3 = N * N * N, T = kAllThreads;
    extern __shared__ __align__(16) unsigned char smraw[];
    C *sm = reinterpret_cast<C *>(smraw);
    C *t = sm, *tw = sm + N3;
    const int64_t f = blockIdx.x;
    C *xf = X + f * ncell;
    const R *df = D + f * ncell;
    for (int i = threadIdx.x; i < N; i += T) tw[i] = twg[i];
    // eight loads in flight per thread (indices past the slab clamped to its last value, never stored)
    for (int i0 = (int)threadIdx.x; i0 < N3; i0 += 8 * T) {
        auto ld = [&](int k) { return xf[min(i0 + k * T, N3 - 1)]; };
        const C a0 = ld(0), a1 = ld(1), a2 = ld(2), a3 = ld(3), a4 = ld(4), a5 = ld(5), a6 = ld(6), a7 = ld(7);
        auto st = [&](int k, const C &a) {
            if (i0 + k * T < N3) t[i0 + k * T] = a;
        };
        st(0, a0), st(1, a1), st(2, a2), st(3, a3), st(4, a4), st(5, a5), st(6, a6), st(7, a7);
    }
    __syncthreads();
    tiles_axis<R, N2, true, false>(t, N, tw);          // z, in the N x-planes
    tiles_axis<R, N2, false, false>(t, N, tw);         // y
    tiles_axis<R, N2, false, false, NN>(t, 1, tw);     // x: one N x N^2 tile
    if (MODE == 1) {
        for (int i = threadIdx.x; i < N3; i += T) D[f * ncell + i] = t[i].x;
        return;
    }
    for (int i0 = (int)threadIdx.x; i0 < N3; i0 += 8 * T) {
        auto ld = [&](int k) { return df[min(i0 + k * T, N3 - 1)]; };
        const R d0 = ld(0), d1 = ld(1), d2 = ld(2), d3 = ld(3), d4 = ld(4), d5 = ld(5), d6 = ld(6), d7 = ld(7);
        auto mul = [&](int k, R d) {
            const int i = i0 + k * T;
            if (i < N3) {
                const R s = d * scale;
                t[i] = mkc(t[i].x * s, t[i].y * s);
            }
        };
        mul(0, d0), mul(1, d1), mul(2, d2), mul(3, d3), mul(4, d4), mul(5, d5), mul(6, d6), mul(7, d7);
    }
    __syncthreads();
    tiles_axis<R, N2, false, true, NN>(t, 1, tw);
    tiles_axis<R, N2, false, true>(t, N, tw);
    tiles_axis<R, N2, true, true>(t, N, tw);
    for (int i = threadIdx.x; i < N3; i += T) xf[i] = t[i];
}

// The evaluation form of k_rdft_all (MODE 0): a persistent grid of one block per CU walks the node
// frequencies f = blockIdx.x, + gridDim.x, ...  The HBM traffic of frequency f + gridDim.x is issued
// while f is transformed: its spectrum values go straight into registers in the order of the first z
// phase (each thread holds the N2 inputs of its z tasks, ZK of them) and its D values in the order of
// the x products (XK tasks of 4 values); barriers wait for LDS operations only, so these loads stay in
// flight across the transform.  Three stages work outside LDS:
//   - the first z phase reads its inputs from those registers (no load pass through LDS);
//   - the second x phase, the product with D and the first inverse x phase are one step per task (the
//     4-point transforms of the same four values around the product);
//   - the last inverse z phase writes its outputs straight to X.
// Every value is read and written once per frequency, and D read once: 40 B (float32: 20 B) per kept
// node frequency and leaf, as in k_rdft_all, whose arithmetic and order of operations it keeps.
template <typename R, int N2>
__global__ __launch_bounds__(kAllThreads) void k_rdft_pf(Cplx<R> *X, const R *D, const Cplx<R> *twg,
                                                         int64_t ncell, R scale, int64_t nf) {
    using C = Cplx<R>;
    constexpr int N = 4 * N2, NN = N * N, N3 = N * N * N, T = kAllThreads;
    constexpr int ZT = 4 * NN, ZK = (ZT + T - 1) / T;         // z tasks (line, n1) and per thread
    constexpr int XT = N2 * NN, XK = (XT + T - 1) / T;        // x tasks (k2, line) and per thread
    extern __shared__ __align__(16) unsigned char smraw[];
    C *sm = reinterpret_cast<C *>(smraw);
    C *t = sm, *tw = sm + N3;
    const int tid = threadIdx.x;
    for (int i = tid; i < N; i += T) tw[i] = twg[i];
    C zin[ZK][N2];
    R dv[XK][4];
    auto load_z = [&](int64_t f) {
        const C *xf = X + f * ncell;
#pragma unroll
        for (int k = 0; k < ZK; k++) {
            const int task = tid + k * T;
            if (task < ZT) {
                const int line = task >> 2, n1 = task & 3;
#pragma unroll
                for (int n2 = 0; n2 < N2; n2++) zin[k][n2] = xf[line * N + n1 + 4 * n2];
            }
        }
    };
    auto load_d = [&](int64_t f) {
        const R *df = D + f * ncell;
#pragma unroll
        for (int k = 0; k < XK; k++) {
            const int task = tid + k * T;
            if (task < XT) {
                const int k2 = task / NN, line = task - k2 * NN;
#pragma unroll
                for (int k1 = 0; k1 < 4; k1++) dv[k][k1] = df[(4 * k2 + k1) * NN + line];
            }
        }
    };
    int64_t f = blockIdx.x;
    if (f < nf) {
        load_z(f);
        load_d(f);
    }
    __syncthreads();   // the roots
    for (; f < nf; f += gridDim.x) {
        const int64_t fn = f + gridDim.x;
        // z, phase 1 (forward), from the registers into LDS
#pragma unroll
        for (int k = 0; k < ZK; k++) {
            const int task = tid + k * T;
            if (task < ZT) {
                const int line = task >> 2, n1 = task & 3;
                C *b = t + line * N;
                C y[N2];
                dft_small<R, N2, false>(zin[k], y);
#pragma unroll
                for (int k2 = 0; k2 < N2; k2++) {
                    const C w = tw[n1 * k2];
                    b[n1 + 4 * k2] = k2 == 0 ? y[k2]
                                             : mkc(y[k2].x * w.x - y[k2].y * w.y, y[k2].x * w.y + y[k2].y * w.x);
                }
            }
        }
        if (fn < nf) load_z(fn);
        __syncthreads();
        tiles_phase2<R, N2, true, false>(t, N);                // z, phase 2
        tiles_axis<R, N2, false, false>(t, N, tw);             // y
        tiles_phase1<R, N2, false, false, NN>(t, 1, tw);       // x, phase 1
        // x: phase 2, the product with D * scale, and the inverse phase 2, per task
#pragma unroll
        for (int k = 0; k < XK; k++) {
            const int task = tid + k * T;
            if (task < XT) {
                const int k2 = task / NN, line = task - k2 * NN;
                C *b = t + line;
                const C a = b[(4 * k2) * NN], bb = b[(4 * k2 + 1) * NN], c = b[(4 * k2 + 2) * NN],
                        d = b[(4 * k2 + 3) * NN];
                const C s0 = mkc(a.x + c.x, a.y + c.y), s1 = mkc(a.x - c.x, a.y - c.y);
                const C s2 = mkc(bb.x + d.x, bb.y + d.y), s3 = mkc(bb.x - d.x, bb.y - d.y);
                const C js3 = mkc(s3.y, -s3.x);
                const R e0 = dv[k][0] * scale, e1 = dv[k][1] * scale, e2 = dv[k][2] * scale, e3 = dv[k][3] * scale;
                const C o0 = mkc((s0.x + s2.x) * e0, (s0.y + s2.y) * e0);
                const C o1 = mkc((s1.x + js3.x) * e1, (s1.y + js3.y) * e1);
                const C o2 = mkc((s0.x - s2.x) * e2, (s0.y - s2.y) * e2);
                const C o3 = mkc((s1.x - js3.x) * e3, (s1.y - js3.y) * e3);
                const C u0 = mkc(o0.x + o2.x, o0.y + o2.y), u1 = mkc(o0.x - o2.x, o0.y - o2.y);
                const C u2 = mkc(o1.x + o3.x, o1.y + o3.y), u3 = mkc(o1.x - o3.x, o1.y - o3.y);
                const C ju3 = mkc(-u3.y, u3.x);
                b[(4 * k2) * NN] = mkc(u0.x + u2.x, u0.y + u2.y);
                b[(4 * k2 + 1) * NN] = mkc(u1.x + ju3.x, u1.y + ju3.y);
                b[(4 * k2 + 2) * NN] = mkc(u0.x - u2.x, u0.y - u2.y);
                b[(4 * k2 + 3) * NN] = mkc(u1.x - ju3.x, u1.y - ju3.y);
            }
        }
        if (fn < nf) load_d(fn);
        __syncthreads();
        tiles_phase1<R, N2, false, true, NN>(t, 1, tw);        // x, inverse phase 1
        tiles_axis<R, N2, false, true>(t, N, tw);              // y, inverse
        tiles_phase2<R, N2, true, true>(t, N);                 // z, inverse phase 2
        // z, inverse phase 1, from LDS straight to X
        C *xf = X + f * ncell;
#pragma unroll
        for (int k = 0; k < ZK; k++) {
            const int task = tid + k * T;
            if (task < ZT) {
                const int line = task >> 2, n1 = task & 3;
                const C *b = t + line * N;
                C z[N2], y[N2];
#pragma unroll
                for (int k2 = 0; k2 < N2; k2++) {
                    const C v = b[n1 + 4 * k2], w = tw[n1 * k2];
                    z[k2] = k2 == 0 ? v : mkc(v.x * w.x + v.y * w.y, v.y * w.x - v.x * w.y);
                }
                dft_small<R, N2, true>(z, y);
#pragma unroll
                for (int n2 = 0; n2 < N2; n2++) xf[line * N + n1 + 4 * n2] = y[n2];
            }
        }
        __syncthreads();   // this frequency's LDS reads are done before the next one's writes
    }
}

// passes 1 / 3: block (f, x0 .. x0 + PB), the (y, z) planes
template <typename R, int N1, int N2, int PB>
__global__ __launch_bounds__(256) void k_rdft_yz(Cplx<R> *X, const Cplx<R> *twg, int64_t ncell, int inv) {
    using C = Cplx<R>;
    static_assert(N1 == 4, "4 x N2 points");
    constexpr int N = N1 * N2;
    __shared__ C t[PB * N * N];
    __shared__ C tw[N];
    const int x0 = blockIdx.y * PB, np = min(PB, N - x0);
    C *p = X + (int64_t)blockIdx.x * ncell + (int64_t)x0 * N * N;
    for (int i = threadIdx.x; i < N; i += 256) tw[i] = twg[i];
    for (int i = threadIdx.x; i < np * N * N; i += 256) t[i] = p[i];
    __syncthreads();
    if (inv) {
        tiles_axis<R, N2, false, true>(t, np, tw);    // y, then z: the reverse of the forward order
        tiles_axis<R, N2, true, true>(t, np, tw);
    } else {
        tiles_axis<R, N2, true, false>(t, np, tw);    // z
        tiles_axis<R, N2, false, false>(t, np, tw);   // y
    }
    for (int i = threadIdx.x; i < np * N * N; i += 256) p[i] = t[i];
}

// pass 2: block (f, y0 .. y0 + PB), the (x, z) tiles: forward along x, then times D * scale and the
// inverse (MODE 0), or the real part to D (MODE 1)
template <typename R, int N1, int N2, int PB, int MODE>
__global__ __launch_bounds__(256) void k_rdft_x(Cplx<R> *X, R *D, const Cplx<R> *twg, int64_t ncell,
                                                R scale) {
    using C = Cplx<R>;
    constexpr int N = N1 * N2;
    __shared__ C t[PB * N * N];
    __shared__ C tw[N];
    const int64_t f = blockIdx.x;
    const int y0 = blockIdx.y * PB, np = min(PB, N - y0);
    for (int i = threadIdx.x; i < N; i += 256) tw[i] = twg[i];
    for (int i = threadIdx.x; i < np * N * N; i += 256) {
        const int tile = i / (N * N), r = i - tile * N * N, x = r / N, z = r - x * N;
        t[i] = X[f * ncell + ((int64_t)x * N + y0 + tile) * N + z];
    }
    __syncthreads();
    tiles_axis<R, N2, false, false>(t, np, tw);
    for (int i = threadIdx.x; i < np * N * N; i += 256) {
        const int tile = i / (N * N), r = i - tile * N * N, x = r / N, z = r - x * N;
        const int64_t g = f * ncell + ((int64_t)x * N + y0 + tile) * N + z;
        if (MODE == 1) D[g] = t[i].x;
        else t[i] = mkc(t[i].x * D[g] * scale, t[i].y * D[g] * scale);
    }
    if (MODE == 1) return;
    __syncthreads();
    tiles_axis<R, N2, false, true>(t, np, tw);
    for (int i = threadIdx.x; i < np * N * N; i += 256) {
        const int tile = i / (N * N), r = i - tile * N * N, x = r / N, z = r - x * N;
        X[f * ncell + ((int64_t)x * N + y0 + tile) * N + z] = t[i];
    }
}

// ---- plan time, with the mirror symmetry of the kernel --------------------------
// The generating cube is even along each axis separately: K(-g_x, g_y, g_z; -a_x, a_y, a_z) = K(g; a)
// (the displacement cube and the adjacency test are symmetric), so the node spectrum of the residue
// with axis x mirrored is that of g with f_x negated.  One block per residue with every component in
// [0, n/2]: the cube, its full node spectrum in LDS (three separable stages), then the half spectrum
// of each distinct mirror residue.
__global__ __launch_bounds__(256) void k_fft_table_sym(const double2 *W, int pa, int ph, int le, int nside, int p,
                                                       double w, double h, double xi, double2 *X, int64_t ncell) {
    extern __shared__ double2 sm[];
    double2 *sW = sm, *S1 = sW + pa * pa, *S2 = S1 + pa * pa * pa;
    double *cube = reinterpret_cast<double *>(S2 + pa * pa * pa);
    const int nh = nside / 2 + 1;
    const int b = blockIdx.x;
    const int gx = b / (nh * nh), gy = (b / nh) % nh, gz = b % nh;
    const int t = threadIdx.x;
    for (int i = t; i < pa * pa; i += 256) sW[i] = W[i];
    const double lim = nside * (p + 0.5);
    const int n3 = pa * pa * pa;
    for (int e = t; e < n3; e += 256) {
        const int a1 = e / (pa * pa), a2 = (e / pa) % pa, a3 = e % pa;
        const int d1 = a1 < le ? a1 : a1 - pa, d2 = a2 < le ? a2 : a2 - pa, d3 = a3 < le ? a3 : a3 - pa;
        double s = 0;
        for (int I = -p - 2; I <= p + 2; I++) {
            const int Dx = gx - nside * I;
            if (fabs((double)Dx) > lim) continue;
            const double zx = Dx * w + d1 * h;
            for (int J = -p - 2; J <= p + 2; J++) {
                const int Dy = gy - nside * J;
                if (fabs((double)Dy) > lim) continue;
                const double zy = Dy * w + d2 * h;
                for (int K = -p - 2; K <= p + 2; K++) {
                    const int Dz = gz - nside * K;
                    if (fabs((double)Dz) > lim) continue;
                    if (abs(Dx) < 2 && abs(Dy) < 2 && abs(Dz) < 2) continue;
                    const double zz = Dz * w + d3 * h;
                    const double r = sqrt(zx * zx + zy * zy + zz * zz);
                    s += erfc(xi * r) / r;
                }
            }
        }
        cube[e] = s;
    }
    __syncthreads();
    for (int o = t; o < n3; o += 256) {             // x: S1[f1][a2][a3]
        const int f1 = o / (pa * pa), r = o % (pa * pa);
        double re = 0, im = 0;
        for (int a1 = 0; a1 < pa; a1++) {
            const double2 c = sW[f1 * pa + a1];
            const double v = cube[a1 * pa * pa + r];
            re += c.x * v;
            im += c.y * v;
        }
        S1[o] = make_double2(re, im);
    }
    __syncthreads();
    for (int o = t; o < n3; o += 256) {             // y: S2[f1][f2][a3]
        const int f1 = o / (pa * pa), f2 = (o / pa) % pa, a3 = o % pa;
        double re = 0, im = 0;
        for (int a2 = 0; a2 < pa; a2++) {
            const double2 c = sW[f2 * pa + a2], v = S1[(f1 * pa + a2) * pa + a3];
            re += c.x * v.x - c.y * v.y;
            im += c.x * v.y + c.y * v.x;
        }
        S2[o] = make_double2(re, im);
    }
    __syncthreads();
    for (int o = t; o < n3; o += 256) {             // z (full): S1[f1][f2][f3]
        const int f12 = o / pa, f3 = o % pa;
        double re = 0, im = 0;
        for (int a3 = 0; a3 < pa; a3++) {
            const double2 c = sW[f3 * pa + a3], v = S2[f12 * pa + a3];
            re += c.x * v.x - c.y * v.y;
            im += c.x * v.y + c.y * v.x;
        }
        S1[o] = make_double2(re, im);
    }
    __syncthreads();
    const int g[3] = {gx, gy, gz};
    for (int m = 0; m < 8; m++) {
        bool dup = false;
        int gm[3];
        for (int a = 0; a < 3; a++) {
            const bool flip = (m >> a) & 1;
            // a mirror of a self-mirrored component (0 or n/2) repeats another mirror
            if (flip && (g[a] == 0 || 2 * g[a] == nside)) dup = true;
            gm[a] = flip ? nside - g[a] : g[a];
        }
        if (dup) continue;
        const int64_t gl = ((int64_t)gm[0] * nside + gm[1]) * nside + gm[2];
        for (int o = t; o < pa * pa * ph; o += 256) {
            const int f1 = o / (pa * ph), f2 = (o / ph) % pa, f3 = o % ph;
            const int F1 = (m & 1) ? (pa - f1) % pa : f1, F2 = (m & 2) ? (pa - f2) % pa : f2;
            const int F3 = (m & 4) ? (pa - f3) % pa : f3;
            X[(int64_t)o * ncell + gl] = S1[(F1 * pa + F2) * pa + F3];
        }
    }
}

template <typename R> Tw16<R> roots16() {
    Tw16<R> tw;
    for (int k = 0; k < 8; k++) {
        const long double a = -2.0L * (long double)kPiF * k / 16.0L;
        tw.w[k] = mkc((R)cosl(a), (R)sinl(a));
    }
    return tw;
}

size_t nodes_fwd_lds(int L, int pa) {
    return sizeof(double2) * ((size_t)pa * L + (size_t)pa * L * L + (size_t)pa * pa * L) + sizeof(double) * L * L * L;
}
size_t nodes_inv_lds(int L, int pa, int ph) {
    const size_t nx = std::max((size_t)pa * pa * ph, (size_t)pa * L * L);
    return sizeof(double2) * ((size_t)pa * L + (size_t)pa * pa * L + nx);
}
size_t table_lds(int pa) { return sizeof(double2) * pa * pa + sizeof(double) * pa * pa * pa; }
size_t table_sym_lds(int pa) {
    return sizeof(double2) * ((size_t)pa * pa + 2 * (size_t)pa * pa * pa) + sizeof(double) * pa * pa * pa;
}

template <int NS, int MODE, typename R>
void split_passes(ankh_plan_s *pl, Cplx<R> *X, R *D, const Cplx<R> *tw, R scale) {
    const dim3 g((unsigned)pl->fft_nf, NS), b(256);
    hipLaunchKernelGGL((k_fft_yz<R, NS, false>), g, b, 0, pl->stream, X, tw, pl->nleaf);
    hipLaunchKernelGGL((k_fft_x<R, NS, MODE>), g, b, 0, pl->stream, X, D, tw, pl->nleaf, scale);
    if (MODE == 0) hipLaunchKernelGGL((k_fft_yz<R, NS, true>), g, b, 0, pl->stream, X, tw, pl->nleaf);
}

// The cell transforms of every kept node frequency in the working precision R: the spectrum X, the
// real spectrum D and the roots tw of that precision.  Grids that are not 12, 20, 24 or a power of
// two (direct DFTs) exist in float64 only.
template <int MODE, typename R>
hipError_t cells(ankh_plan_s *pl, Cplx<R> *X, R *D, const Cplx<R> *tw, R scale) {
    if (sizeof(R) == 8 ? pl->fft_single : pl->fft_single32) {
        // one block per node frequency with all cells in LDS
        const size_t shm = sizeof(Cplx<R>) * ((size_t)pl->nleaf + pl->nside);
        const dim3 g((unsigned)pl->fft_nf), b(kAllThreads);
        if constexpr (MODE == 0 && sizeof(R) == 4) {
            // evaluation in float32: the persistent, prefetching form, one block per CU (in float64 its
            // registers would spill)
            const int64_t nf = pl->fft_nf;
            const dim3 gp((unsigned)std::min<int64_t>(nf, pl->num_cu));
            if (pl->nside == 12)
                hipLaunchKernelGGL((k_rdft_pf<R, 3>), gp, b, shm, pl->stream, X, D, tw, pl->nleaf, scale, nf);
            else if (pl->nside == 20)
                hipLaunchKernelGGL((k_rdft_pf<R, 5>), gp, b, shm, pl->stream, X, D, tw, pl->nleaf, scale, nf);
            else
                hipLaunchKernelGGL((k_rdft_pf<R, 6>), gp, b, shm, pl->stream, X, D, tw, pl->nleaf, scale, nf);
            return hipGetLastError();
        }
        if (pl->nside == 12)
            hipLaunchKernelGGL((k_rdft_all<R, 3, MODE>), g, b, shm, pl->stream, X, D, tw, pl->nleaf, scale);
        else if (pl->nside == 20)
            hipLaunchKernelGGL((k_rdft_all<R, 5, MODE>), g, b, shm, pl->stream, X, D, tw, pl->nleaf, scale);
        else
            hipLaunchKernelGGL((k_rdft_all<R, 6, MODE>), g, b, shm, pl->stream, X, D, tw, pl->nleaf, scale);
        return hipGetLastError();
    }
    if (pl->fft_dft && (pl->nside == 12 || pl->nside == 20 || pl->nside == 24)) {
        // 12 = 4 x 3, 20 = 4 x 5, 24 = 4 x 6 points per axis: two-phase transforms, PB tiles per block
        // (PB N^2 complex values + N roots within 64 KB)
        const int n = pl->nside;
        const dim3 b(256);
#define ANKH_RDFT(A, B, PB)                                                                                    \
        {                                                                                                      \
            const dim3 g((unsigned)pl->fft_nf, (unsigned)((n + PB - 1) / PB));                                \
            hipLaunchKernelGGL((k_rdft_yz<R, A, B, PB>), g, b, 0, pl->stream, X, tw, pl->nleaf, 0);            \
            hipLaunchKernelGGL((k_rdft_x<R, A, B, PB, MODE>), g, b, 0, pl->stream, X, D, tw, pl->nleaf, scale); \
            if (MODE == 0) hipLaunchKernelGGL((k_rdft_yz<R, A, B, PB>), g, b, 0, pl->stream, X, tw, pl->nleaf, 1); \
        }
        if (n == 12) ANKH_RDFT(4, 3, 4)
        else if (n == 20) ANKH_RDFT(4, 5, 2)
        else ANKH_RDFT(4, 6, 2)
#undef ANKH_RDFT
        return hipGetLastError();
    }
    if (pl->fft_dft) {
        if constexpr (sizeof(R) == 8) {
            const int n = pl->nside;
            const dim3 g((unsigned)pl->fft_nf, n), b(256);
            const size_t shm = sizeof(double2) * (2 * (size_t)n * n + n);
            hipLaunchKernelGGL(k_dft_yz, g, b, shm, pl->stream, X, tw, n, pl->nleaf, 0);
            hipLaunchKernelGGL(k_dft_x, g, b, shm, pl->stream, X, D, tw, n, pl->nleaf, (double)scale, MODE);
            if (MODE == 0) hipLaunchKernelGGL(k_dft_yz, g, b, shm, pl->stream, X, tw, n, pl->nleaf, 1);
            return hipGetLastError();
        } else {
            return hipErrorInvalidValue;
        }
    }
    if (pl->fft_split) {
        switch (pl->nside) {
            case 2: split_passes<2, MODE, R>(pl, X, D, tw, scale); break;
            case 4: split_passes<4, MODE, R>(pl, X, D, tw, scale); break;
            case 8: split_passes<8, MODE, R>(pl, X, D, tw, scale); break;
            case 16: split_passes<16, MODE, R>(pl, X, D, tw, scale); break;
            case 32: split_passes<32, MODE, R>(pl, X, D, tw, scale); break;
            default: split_passes<64, MODE, R>(pl, X, D, tw, scale); break;
        }
        return hipGetLastError();
    }
    const size_t shm = sizeof(Cplx<R>) * pl->nleaf;
    const dim3 g((unsigned)pl->fft_nf), b(256);
    const Tw16<R> t16 = roots16<R>();
    switch (pl->nside) {
        case 1: hipLaunchKernelGGL((k_fft_cells<R, 1, MODE>), g, b, shm, pl->stream, X, D, pl->nleaf, scale, t16); break;
        case 2: hipLaunchKernelGGL((k_fft_cells<R, 2, MODE>), g, b, shm, pl->stream, X, D, pl->nleaf, scale, t16); break;
        case 4: hipLaunchKernelGGL((k_fft_cells<R, 4, MODE>), g, b, shm, pl->stream, X, D, pl->nleaf, scale, t16); break;
        case 8: hipLaunchKernelGGL((k_fft_cells<R, 8, MODE>), g, b, shm, pl->stream, X, D, pl->nleaf, scale, t16); break;
        default: hipLaunchKernelGGL((k_fft_cells<R, 16, MODE>), g, b, shm, pl->stream, X, D, pl->nleaf, scale, t16); break;
    }
    return hipGetLastError();
}

__global__ void k_to_f32(const double *a, float *b, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        b[i] = (float)a[i];
}

}  // namespace

// the one-block cell transform, where the device grants its LDS (queried, and the kernels' dynamic
// limit raised when above the default): 12^3 and 20^3 grids in float64, also 24^3 in float32
bool fft_single_ok(int nside, bool f32) {
    if (!(nside == 12 || nside == 20 || (f32 && nside == 24))) return false;
    const size_t need = (f32 ? sizeof(float2) : sizeof(double2)) * ((size_t)nside * nside * nside + nside);
    int device = 0, lim = 0;
    if (hipGetDevice(&device) != hipSuccess ||
        hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, device) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    if (need > (size_t)lim) return false;
    if (need > 65536) {
        const int bytes = (int)need;
        hipError_t e = hipSuccess;
        if (f32) {
            const void *k0 = nside == 20 ? reinterpret_cast<const void *>(&k_rdft_all<float, 5, 0>)
                                         : reinterpret_cast<const void *>(&k_rdft_all<float, 6, 0>);
            const void *k1 = nside == 20 ? reinterpret_cast<const void *>(&k_rdft_pf<float, 5>)
                                         : reinterpret_cast<const void *>(&k_rdft_pf<float, 6>);
            e = hipFuncSetAttribute(k0, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
            if (e == hipSuccess) e = hipFuncSetAttribute(k1, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
        } else if (nside == 20) {
            e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_rdft_all<double, 5, 0>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
            if (e == hipSuccess)
                e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_rdft_all<double, 5, 1>),
                                        hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
        }
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return false;
        }
    }
    return true;
}

bool fft_supported(int depth, int L, int le) {
    if (depth < 0 || depth > kMaxFftDepth || le < 2 || le > kMaxOrder || L < 2 || L > kMaxOrder) return false;
    const int pa = 2 * le - 1, ph = pa / 2 + 1;
    const size_t lim = 65536;
    // cells of one node frequency: one block up to 16^3, else three passes over 32^2 / 64^2 tiles
    return nodes_fwd_lds(L, pa) <= lim && nodes_inv_lds(L, pa, ph) <= lim && table_lds(pa) <= lim;
}

void fft_host_roots(int nside, bool full, std::vector<double2> &tw) {
    const int cnt = full ? nside : nside / 2;
    tw.assign(std::max(1, cnt), make_double2(1, 0));
    for (int k = 0; k < cnt; k++) {
        const long double a = -2.0L * (long double)kPiF * k / nside;
        tw[k] = make_double2((double)cosl(a), (double)sinl(a));
    }
}

void fft_host_tables(int L, int le, const double *cheb, std::vector<double2> &B, std::vector<double2> &W) {
    const int pa = 2 * le - 1;
    // E[a][i] = U_a(r_i): equispaced Lagrange polynomials (nodes -1 + 2a/(le-1)) at the Chebyshev nodes
    std::vector<long double> E((size_t)le * L);
    for (int a = 0; a < le; a++)
        for (int i = 0; i < L; i++) {
            long double u = 1;
            const long double ta = -1.0L + 2.0L * a / (le - 1);
            for (int b = 0; b < le; b++) {
                if (b == a) continue;
                const long double tb = -1.0L + 2.0L * b / (le - 1);
                u *= ((long double)cheb[i] - tb) / (ta - tb);
            }
            E[(size_t)a * L + i] = u;
        }
    W.assign((size_t)pa * pa, make_double2(0, 0));
    std::vector<long double> wr((size_t)pa * pa), wi((size_t)pa * pa);
    for (int f = 0; f < pa; f++)
        for (int a = 0; a < pa; a++) {
            const int m = (f * a) % pa;
            const long double ang = -2.0L * (long double)kPiF * m / pa;
            wr[(size_t)f * pa + a] = cosl(ang);
            wi[(size_t)f * pa + a] = sinl(ang);
            W[(size_t)f * pa + a] = make_double2((double)cosl(ang), (double)sinl(ang));
        }
    // B = W[:, :le] E: the reinterpolation and the zero-padded node DFT in one matrix
    B.assign((size_t)pa * L, make_double2(0, 0));
    for (int f = 0; f < pa; f++)
        for (int i = 0; i < L; i++) {
            long double re = 0, im = 0;
            for (int a = 0; a < le; a++) {
                re += wr[(size_t)f * pa + a] * E[(size_t)a * L + i];
                im += wi[(size_t)f * pa + a] * E[(size_t)a * L + i];
            }
            B[(size_t)f * L + i] = make_double2((double)re, (double)im);
        }
}

hipError_t launch_fft_build_D(ankh_plan_s *pl) {
    const int pa = pl->fft_pa, ph = pl->fft_ph, le = pl->eq_order;
    const double w = pl->edge / pl->nside;
    if (pl->nside >= 2 && table_sym_lds(pa) <= 65536) {
        const int nh = pl->nside / 2 + 1;
        hipLaunchKernelGGL(k_fft_table_sym, dim3((unsigned)(nh * nh * nh)), dim3(256), table_sym_lds(pa), pl->stream,
                           pl->d_fftW, pa, ph, le, pl->nside, pl->images, w, w / (le - 1), pl->xi, pl->d_fftX,
                           pl->nleaf);
    } else {
        hipLaunchKernelGGL(k_fft_table, dim3((unsigned)pl->nleaf), dim3(256), table_lds(pa), pl->stream, pl->d_fftW,
                           pa, ph, le, pl->nside, pl->images, w, w / (le - 1), pl->xi, pl->d_fftX, pl->nleaf);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return cells<1, double>(pl, pl->d_fftX, pl->d_fftD, pl->d_fftTw, 1.0);
}

// the float32 copy of the real spectrum (mixed modes), from the float64 one built above
hipError_t launch_fft_D_to_f32(ankh_plan_s *pl) {
    hipLaunchKernelGGL(k_to_f32, dim3(1024), dim3(256), 0, pl->stream, pl->d_fftD, pl->d_fftD32,
                       (int64_t)pl->fft_nf * pl->nleaf);
    return hipGetLastError();
}

// the register-blocked kernels for equispaced order = Chebyshev order <= 6 (four leaves per block
// within 64 KB of LDS; at least 8 leaves), else the generic ones
static bool fast_nodes(const ankh_plan_s *pl) {
    return pl->eq_order == pl->order && pl->order >= 3 && pl->order <= 6 && pl->nleaf % (8 * kCB) == 0 &&
           pl->nleaf % kCF == 0;
}

// the mixed modes run the transforms of an evaluation in float32 where every kernel of the plan has a
// float32 form: the register-blocked node transforms and any cell transform but the direct DFTs
bool fft_f32_ok(const ankh_plan_s *pl) {
    const bool dft_only = pl->fft_dft && !(pl->nside == 12 || pl->nside == 20 || pl->nside == 24);
    return fast_nodes(pl) && !dft_only;
}

#define ANKH_FFT_ORDERS(L, X) \
    switch (L) {              \
        case 3: X(3); break;  \
        case 4: X(4); break;  \
        case 5: X(5); break;  \
        default: X(6); break; \
    }

hipError_t launch_fft_forward(ankh_plan_s *pl) {
    const int L = pl->order, pa = pl->fft_pa;
    const double *Q = pl->d_M + pl->lv[pl->depth].cell0 * pl->nup;
    if (fast_nodes(pl)) {
        const dim3 g((unsigned)(pl->nleaf / kCF)), b(kFT);
        if (pl->fft_f32) {
#define ANKH_FWD(LL)                                                                                                \
            hipLaunchKernelGGL((k_fft_nodes_fwd_t<float, LL>), g, b, 0, pl->stream, Q, pl->nup, pl->d_fftB32, pl->d_fftX32, \
                               pl->nleaf)
            ANKH_FFT_ORDERS(L, ANKH_FWD)
#undef ANKH_FWD
        } else {
#define ANKH_FWD(LL)                                                                                                \
            hipLaunchKernelGGL((k_fft_nodes_fwd_t<double, LL>), g, b, 0, pl->stream, Q, pl->nup, pl->d_fftB, pl->d_fftX, \
                               pl->nleaf)
            ANKH_FFT_ORDERS(L, ANKH_FWD)
#undef ANKH_FWD
        }
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_fft_nodes_fwd, dim3((unsigned)pl->nleaf), dim3(64), nodes_fwd_lds(L, pa), pl->stream, Q,
                       pl->nup, L, pl->d_fftB, pa, pl->fft_ph, pl->d_fftX, pl->nleaf);
    return hipGetLastError();
}

hipError_t launch_fft_cells(ankh_plan_s *pl) {
    const double n6 = (double)pl->nleaf * pl->fft_pa * pl->fft_pa * pl->fft_pa;
    if (pl->fft_f32) return cells<0, float>(pl, pl->d_fftX32, pl->d_fftD32, pl->d_fftTw32, (float)(1.0 / n6));
    return cells<0, double>(pl, pl->d_fftX, pl->d_fftD, pl->d_fftTw, 1.0 / n6);
}

bool fft_inverse_leaf_energies(const ankh_plan_s *pl) { return fast_nodes(pl) && pl->fft_f32; }

hipError_t launch_fft_inverse(ankh_plan_s *pl) {
    const int L = pl->order, pa = pl->fft_pa, ph = pl->fft_ph;
    double *Lam = pl->d_L + pl->lv[pl->depth].cell0 * pl->nup;
    const double *Q = pl->d_M + pl->lv[pl->depth].cell0 * pl->nup;
    if (fast_nodes(pl)) {
        const dim3 g((unsigned)(pl->nleaf / kCB)), b(256);
        if (pl->fft_f32) {
#define ANKH_INV(LL)                                                                                                \
            hipLaunchKernelGGL((k_fft_nodes_inv_t<float, LL>), g, b, 0, pl->stream, pl->d_fftX32, pl->d_fftB32, Lam, \
                               Q, pl->d_eleaf, pl->nup, pl->nleaf)
            ANKH_FFT_ORDERS(L, ANKH_INV)
#undef ANKH_INV
        } else {
#define ANKH_INV(LL)                                                                                                \
            hipLaunchKernelGGL((k_fft_nodes_inv_t<double, LL>), g, b, 0, pl->stream, pl->d_fftX, pl->d_fftB, Lam,    \
                               Q, pl->d_eleaf, pl->nup, pl->nleaf)
            ANKH_FFT_ORDERS(L, ANKH_INV)
#undef ANKH_INV
        }
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_fft_nodes_inv, dim3((unsigned)pl->nleaf), dim3(64), nodes_inv_lds(L, pa, ph), pl->stream,
                       pl->d_fftX, pl->d_fftB, pa, ph, L, Lam, pl->nup, pl->nleaf);
    return hipGetLastError();
}

}  // namespace ankh
