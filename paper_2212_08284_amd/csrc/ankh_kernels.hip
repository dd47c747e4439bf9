// Tree construction, anterpolation (P2M), M2M / L2L, the far-image root
// operator, L2P, reductions and the plan-time operator builders.
//
// Cell and leaf numbering: cell (i, j, k) of level e is (i * 2^e + j) * 2^e + k;
// interpolation node (a, b, c) of a cell is (a * L + b) * L + c; expansions are
// stored cell-major with a row stride nup >= L^3 (a multiple of 64, zero padded).
#include <algorithm>
#include <cmath>
#include <cstdlib>

#include "ankh_internal.h"

namespace ankh {
namespace {

constexpr double kPi = 3.14159265358979323846;

__device__ inline int leaf_coord(double x, double rB, double edge, double w, int nside, double *xw) {
    // wrap into [-rB, rB) then bin; clamp guards the upper face
    double t = x - edge * floor((x + rB) / edge);
    if (t >= rB) t -= edge;
    *xw = t;
    int v = (int)floor((t + rB) / w);
    return v < 0 ? 0 : (v >= nside ? nside - 1 : v);
}

__global__ void k_zero_i32(int32_t *p, int64_t n) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

__global__ void k_zero_f64(double *p, int64_t n) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

__global__ void k_to_f32(const double *s, float *d, int64_t n) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) d[i] = (float)s[i];
}

// ---- tree: bin atoms into leaves, count, validate inputs --------------------
// leaf of every atom, the leaf counts, and each atom's arrival rank in its leaf (the scatter then
// needs no atomics; the arrival order itself is undone by the segment sort).  Positions and charges
// are checked here, the higher moments in the gather, which reads them anyway.
// The lanes of a wave that fall into the same leaf take their ranks from one atomic add (inputs in
// spatial order put a wave's atoms into a few leaves; the segment sort fixes the in-leaf order
// afterwards, so which lane gets which rank does not matter).  The groups of up to 8 distinct leaves
// are found first and their leaders add in one atomic instruction, together with the lanes left
// over (one each), so a wave waits for one atomic round trip.
__global__ __launch_bounds__(256) void k_bin(int64_t n, const double *pos, const double *q, double rB, double edge,
                                             double w, int nside, int32_t *leaf, int32_t *count, int32_t *rank,
                                             int32_t *err) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const bool valid = i < n;
    int id = -1;
    if (valid) {
        bool fin = isfinite(q[i]);
        int ix[3];
        for (int d = 0; d < 3; d++) {
            double v = pos[3 * i + d], xw;
            fin = fin && isfinite(v);
            ix[d] = isfinite(v) ? leaf_coord(v, rB, edge, w, nside, &xw) : 0;
        }
        if (!fin) err[0] = 1;
        id = (ix[0] * nside + ix[1]) * nside + ix[2];
        leaf[i] = id;
    }
    const int lane = (int)__lane_id();
    unsigned long long pending = __ballot(valid);
    int leader_of = lane, cnt = 1, off = 0;        // a lane left over is its own group of one
    bool adds = false;
    for (int round = 0; round < 8 && pending; round++) {
        const int leader = __ffsll((long long)pending) - 1;
        const int lid = __shfl(id, leader);
        const unsigned long long same = __ballot(id == lid) & pending;
        if ((same >> lane) & 1ull) {
            leader_of = leader;
            off = (int)__popcll(same & ((1ull << lane) - 1ull));
        }
        if (lane == leader) {
            adds = true;
            cnt = (int)__popcll(same);
        }
        pending &= ~same;
    }
    if ((pending >> lane) & 1ull) adds = true;
    int base = 0;
    if (valid && adds) base = atomicAdd(&count[id], cnt);
    base = __shfl(base, leader_of);
    if (valid) rank[i] = base + off;
}

// exclusive scan of the leaf counts in one block (offs[m] = total; totals fit int32, as offs does), in
// chunks of 8192 counts: a coalesced load into LDS (eight per thread, all in flight), each thread's eight
// consecutive counts summed, the sums scanned within each wave by shuffles and across the 16 waves by the
// first wave, the offsets written back through LDS (coalesced), the chunk total carried to the next.
// The counts are set back to zero once read, ready for the next binning.
__global__ __launch_bounds__(1024) void k_scan(int32_t *count, int32_t *offs, int64_t m) {
    constexpr int T = 1024, C = 8 * T;
    __shared__ int buf[C];
    __shared__ int wsum[16];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    int carry = 0;
    for (int64_t c0 = 0; c0 < m; c0 += C) {
        const int cn = (int)((m - c0) < C ? (m - c0) : C);
        int v[8];
#pragma unroll
        for (int u = 0; u < 8; u++) v[u] = t + u * T < cn ? count[c0 + t + u * T] : 0;
#pragma unroll
        for (int u = 0; u < 8; u++)
            if (t + u * T < cn) count[c0 + t + u * T] = 0;
#pragma unroll
        for (int u = 0; u < 8; u++) buf[t + u * T] = v[u];
        __syncthreads();
        int e[8], s = 0;
#pragma unroll
        for (int u = 0; u < 8; u++) {
            e[u] = buf[8 * t + u];
            s += e[u];
        }
        int x = s;                          // inclusive scan over the wave
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int y = __shfl_up(x, off, 64);
            if (lane >= off) x += y;
        }
        if (lane == 63) wsum[w] = x;
        __syncthreads();
        if (w == 0) {
            int z = lane < 16 ? wsum[lane] : 0;
#pragma unroll
            for (int off = 1; off < 16; off <<= 1) {
                const int y = __shfl_up(z, off, 64);
                if (lane >= off) z += y;
            }
            if (lane < 16) wsum[lane] = z;  // inclusive totals of the waves
        }
        __syncthreads();
        int base = carry + x - s + (w > 0 ? wsum[w - 1] : 0);
#pragma unroll
        for (int u = 0; u < 8; u++) {
            buf[8 * t + u] = base;
            base += e[u];
        }
        carry += wsum[15];
        __syncthreads();
#pragma unroll
        for (int u = 0; u < 8; u++)
            if (t + u * T < cn) offs[c0 + t + u * T] = buf[t + u * T];
        __syncthreads();                    // buf and wsum are free for the next chunk
    }
    if (t == 0) offs[m] = carry;
}

__global__ void k_scatter(int64_t n, const int32_t *leaf, const int32_t *offs, const int32_t *rank, int32_t *perm) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    perm[offs[leaf[i]] + rank[i]] = (int32_t)i;
}

// order the atoms of each leaf by input index (rank sort), so that every later sum runs in an order
// independent of the scatter's atomics.  One wave per leaf, four leaves per block (a leaf holds a few
// tens of atoms); a leaf of up to 512 atoms is staged in LDS.
__global__ __launch_bounds__(256) void k_segsort(const int32_t *offs, const int32_t *perm, int32_t *out,
                                                 int64_t nleaf) {
    __shared__ int32_t seg[4][512];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t leaf = (int64_t)blockIdx.x * 4 + wv;
    if (leaf >= nleaf) return;   // the waves synchronise among themselves only
    const int s0 = offs[leaf], cnt = offs[leaf + 1] - s0;
    const bool cached = cnt <= 512;
    int32_t *sg = seg[wv];
    if (cached)
        for (int e = lane; e < cnt; e += 64) sg[e] = perm[s0 + e];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    for (int e = lane; e < cnt; e += 64) {
        const int v = cached ? sg[e] : perm[s0 + e];
        int rank = 0;
        for (int j = 0; j < cnt; j++) rank += ((cached ? sg[j] : perm[s0 + j]) < v);
        out[s0 + rank] = v;
    }
}

// leaf-order particle arrays: local coordinates (relative to the leaf centre).  Every input of an atom
// is loaded before the first store (the inputs are read-only and do not alias the outputs), so a
// thread waits for one round trip of its scattered reads instead of one per moment.  The leaf
// coordinates are recomputed from the positions exactly as the binning computed them.
template <int ORD, bool MIXED>
__global__ __launch_bounds__(256) void k_gather(int64_t n, const int32_t *__restrict__ perm,
                                                const double *__restrict__ pos, const double *__restrict__ q,
                                                const double *__restrict__ mu, const double *__restrict__ th,
                                                const double *__restrict__ om, double rB, double edge, double w,
                                                int nside, Particles P, int32_t *err) {
    const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int64_t i = perm[s];
    double p[3], m[3], t[6], o[10];
    for (int d = 0; d < 3; d++) p[d] = pos[3 * i + d];
    const double qi = q[i];
    if constexpr (ORD >= 1)
        for (int d = 0; d < 3; d++) m[d] = mu ? mu[3 * i + d] : 0.0;
    if constexpr (ORD >= 2)
        for (int d = 0; d < 6; d++) t[d] = th ? th[6 * i + d] : 0.0;
    if constexpr (ORD >= 3)
        for (int d = 0; d < 10; d++) o[d] = om ? om[10 * i + d] : 0.0;
    double loc[3];
    for (int d = 0; d < 3; d++) {
        const double v = p[d];
        double xw = v;
        const int ix = isfinite(v) ? leaf_coord(v, rB, edge, w, nside, &xw) : 0;
        loc[d] = xw - (-rB + (ix + 0.5) * w);
    }
    P.x[s] = loc[0];
    P.y[s] = loc[1];
    P.z[s] = loc[2];
    P.q[s] = qi;
    if constexpr (MIXED) P.qf[s] = (float)qi;
    bool fin = true;
    if constexpr (ORD >= 1) {
        for (int d = 0; d < 3; d++) {
            fin = fin && isfinite(m[d]);
            P.mu[d * n + s] = m[d];
            if constexpr (MIXED) P.muf[d * n + s] = (float)m[d];
        }
    }
    if constexpr (ORD >= 2) {
        for (int d = 0; d < 6; d++) {
            fin = fin && isfinite(t[d]);
            P.th[d * n + s] = t[d];
            if constexpr (MIXED) P.thf[d * n + s] = (float)t[d];
        }
        const double tr = t[0] + t[3] + t[5], mx = fmax(fabs(t[0]), fmax(fabs(t[3]), fabs(t[5])));
        if (fabs(tr) > 1e-6 * (1.0 + mx)) err[1] = 1;
    }
    if constexpr (ORD >= 3) {
        for (int d = 0; d < 10; d++) {
            fin = fin && isfinite(o[d]);
            P.om[d * n + s] = o[d];
            if constexpr (MIXED) P.omf[d * n + s] = (float)o[d];
        }
        // the three traces Omega_aab (b = x, y, z) must vanish
        double mx = 0;
        for (int d = 0; d < 10; d++) mx = fmax(mx, fabs(o[d]));
        const double tx = o[0] + o[3] + o[5], ty = o[1] + o[6] + o[8], tz = o[2] + o[7] + o[9];
        if (fmax(fabs(tx), fmax(fabs(ty), fabs(tz))) > 1e-6 * (1.0 + mx)) err[1] = 1;
    }
    if (!fin) err[0] = 1;
}

// ---- Chebyshev basis ---------------------------------------------------------
// T_m and its derivatives up to order ND-1 by the differentiated three-term
// recurrence (identical to D^n T with the differentiation matrix D), then
// S^(n)_k = (1/h)^n sum_m H[k][m] T^(n)_m.
template <int ND, int L, bool ROLLED = false>
__device__ inline void cheb_basis(double xh, double hinv, const double *sH, double *out /* [ND][L] */,
                                  int stride_n) {
    double T[ND][L > 2 ? L : 2];
#pragma unroll
    for (int n = 0; n < ND; n++) {
        T[n][0] = (n == 0) ? 1.0 : 0.0;
        T[n][1] = (n == 0) ? xh : (n == 1 ? 1.0 : 0.0);
    }
#pragma unroll
    for (int m = 1; m + 1 < L; m++) {
        T[0][m + 1] = 2 * xh * T[0][m] - T[0][m - 1];
#pragma unroll
        for (int n = 1; n < ND; n++) T[n][m + 1] = 2 * n * T[n - 1][m] + 2 * xh * T[n][m] - T[n][m - 1];
    }
    // ROLLED (an output in LDS): the loop over k stays a loop, which keeps the L^2 entries of sH out of
    // registers; an output in registers needs it unrolled (constant indices)
    double sc = 1.0;
#pragma unroll
    for (int n = 0; n < ND; n++) {
        if constexpr (ROLLED) {
#pragma unroll 1
            for (int k = 0; k < L; k++) {
                double s = 0;
#pragma unroll
                for (int m = 0; m < L; m++) s += sH[k * L + m] * T[n][m];
                out[n * stride_n + k] = s * sc;
            }
        } else {
#pragma unroll
            for (int k = 0; k < L; k++) {
                double s = 0;
#pragma unroll
                for (int m = 0; m < L; m++) s += sH[k * L + m] * T[n][m];
                out[n * stride_n + k] = s * sc;
            }
        }
        sc *= hinv;
    }
}

// ---- P2M: modified charges of every leaf (Alg. 2) --------------------------
// Q[i][j][k] = sum_atoms sum_(a,b,c) m_abc S^(a)_i(x) S^(b)_j(y) S^(c)_k(z), the
// (a,b,c) of q, mu, Theta and Omega, each component of a symmetric tensor
// weighted by its multiplicity (off-diagonal Theta doubled; Omega 1, 3 or 6).
// Grouped by the x order a, the sum is sum_a S^(a)_i(x) w_a(j, k) with
//   w_0 = q y0 z0 + mu_y y1 z0 + mu_z y0 z1 + Th_yy y2 z0 + 2 Th_yz y1 z1 + Th_zz y0 z2
//         + Om_yyy y3 z0 + 3 Om_yyz y2 z1 + 3 Om_yzz y1 z2 + Om_zzz y0 z3,
//   w_1 = mu_x y0 z0 + 2 Th_xy y1 z0 + 2 Th_xz y0 z1 + 3 Om_xyy y2 z0 + 6 Om_xyz y1 z1 + 3 Om_xzz y0 z2,
//   w_2 = Th_xx y0 z0 + 3 Om_xxy y1 z0 + 3 Om_xxz y0 z1,   w_3 = Om_xxx y0 z0,
// so a thread owns one (j, k) line of L nodes and a slice of the leaf's atoms;
// the slices' lines are summed in slice order at the end.
// the moments of atom `slot` in the order the line weights take them (off-diagonal components of a
// symmetric tensor times their multiplicity)
template <int ORD>
__device__ inline void p2m_moments(const Particles &P, int64_t slot, int64_t n, double *mo) {
    mo[0] = P.q[slot];
    if (ORD >= 1) {
        mo[1] = P.mu[slot];
        mo[2] = P.mu[n + slot];
        mo[3] = P.mu[2 * n + slot];
    }
    if (ORD >= 2) {
        mo[4] = P.th[slot];                 // xx
        mo[5] = 2 * P.th[n + slot];         // 2 xy
        mo[6] = 2 * P.th[2 * n + slot];     // 2 xz
        mo[7] = P.th[3 * n + slot];         // yy
        mo[8] = 2 * P.th[4 * n + slot];     // 2 yz
        mo[9] = P.th[5 * n + slot];         // zz
    }
    if (ORD >= 3) {
        constexpr double mult[10] = {1, 3, 3, 3, 6, 3, 1, 3, 3, 1};
#pragma unroll
        for (int c = 0; c < 10; c++) mo[10 + c] = mult[c] * P.om[c * n + slot];
    }
}

// w_a(j, k) of one atom (see k_p2m), from its moments and its y and z bases Sy[d][j], Sz[d][k]
template <int ORD, int ND, int L>
__device__ inline void p2m_weights(const double *mo, const double (*Sy)[L], const double (*Sz)[L], int j, int k,
                                   double *w) {
    const double y0 = Sy[0][j], z0 = Sz[0][k];
    w[0] = mo[0] * y0 * z0;
    if constexpr (ORD >= 1) {
        const double y1 = Sy[1][j], z1 = Sz[1][k];
        w[0] += mo[2] * y1 * z0 + mo[3] * y0 * z1;
        w[1] = mo[1] * y0 * z0;
        if constexpr (ORD >= 2) {
            const double y2 = Sy[2][j], z2 = Sz[2][k];
            w[0] += mo[7] * y2 * z0 + mo[8] * y1 * z1 + mo[9] * y0 * z2;
            w[1] += mo[5] * y1 * z0 + mo[6] * y0 * z1;
            w[2] = mo[4] * y0 * z0;
            if constexpr (ORD >= 3) {
                const double y3 = Sy[3][j], z3 = Sz[3][k];
                w[0] += mo[16] * y3 * z0 + mo[17] * y2 * z1 + mo[18] * y1 * z2 + mo[19] * y0 * z3;
                w[1] += mo[13] * y2 * z0 + mo[14] * y1 * z1 + mo[15] * y0 * z2;
                w[2] += mo[11] * y1 * z0 + mo[12] * y0 * z1;
                w[3] = mo[10] * y0 * z0;
            }
        }
    }
}

template <int L, int ORD>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(L <= 7 && ORD <= 2 ? 8 : 1))) void k_p2m(Particles P, const int32_t *offs, const double *tab, int nu, int nup,
                                             double hinv, double *Q, int64_t n) {
    constexpr int ND = ORD + 1;
    // atoms per LDS chunk (a leaf of the planned ANKH-FFT grids: one chunk): 32 keeps the block's LDS
    // at 17 KB (order 6, quadrupoles), so that eight blocks of 60 VGPRs share a CU
    constexpr int CH = 32;
    constexpr int NJK = L * L;
    constexpr int NSL = 256 / NJK;         // atom slices
    constexpr int NMO = ORD == 0 ? 1 : (ORD == 1 ? 4 : (ORD == 2 ? 10 : 20));
    constexpr int NS = CH * 3 * ND * L, NR = NSL * L * L * L;
    __shared__ double sH[L * L];
    __shared__ double sBuf[NS > NR ? NS : NR];   // the chunk's 1D bases, then the slices' partial lines
    __shared__ double sMom[CH][NMO];
    auto sS = reinterpret_cast<double (*)[3][ND][L]>(sBuf);
    auto red = reinterpret_cast<double (*)[L * L * L]>(sBuf);
    const int tid = threadIdx.x;
    const int64_t leaf = blockIdx.x;
    for (int t = tid; t < L * L; t += 256) sH[t] = tab[L + t];
    const int s0 = offs[leaf], cnt = offs[leaf + 1] - s0;
    const int jk = tid % NJK, sl = tid / NJK;
    const int j = jk / L, k = jk % L;
    double acc[L];
#pragma unroll
    for (int i = 0; i < L; i++) acc[i] = 0;
    for (int c0 = 0; c0 < cnt; c0 += CH) {
        const int m = min(CH, cnt - c0);
        __syncthreads();
        if (tid < 3 * m) {
            const int a = tid / 3, ax = tid % 3;
            const int64_t slot = s0 + c0 + a;
            const double xl = ax == 0 ? P.x[slot] : (ax == 1 ? P.y[slot] : P.z[slot]);
            cheb_basis<ND, L, true>(xl * hinv, hinv, sH, &sS[a][ax][0][0], L);
        } else if (tid >= 3 * CH && tid < 3 * CH + m) {
            const int a = tid - 3 * CH;
            p2m_moments<ORD>(P, s0 + c0 + a, n, sMom[a]);
        }
        __syncthreads();
        if (sl < NSL) {
#pragma unroll 1
            for (int a = sl; a < m; a += NSL) {
                double w[ND];
                p2m_weights<ORD, ND, L>(sMom[a], sS[a][1], sS[a][2], j, k, w);
#pragma unroll
                for (int i = 0; i < L; i++) {
                    double v = acc[i];
#pragma unroll
                    for (int d = 0; d < ND; d++) v += sS[a][0][d][i] * w[d];
                    acc[i] = v;
                }
            }
        }
    }
    __syncthreads();                        // the bases are read; their storage takes the partial lines
    if (sl < NSL) {
#pragma unroll
        for (int i = 0; i < L; i++) red[sl][i * NJK + jk] = acc[i];
    }
    __syncthreads();
    for (int node = tid; node < nup; node += 256) {
        double v = 0;
        if (node < nu)
            for (int t = 0; t < NSL; t++) v += red[t][node];
        Q[leaf * nup + node] = v;
    }
}

// ---- M2M: parent expansion (order Lp) from its 8 children (order Lc) ----------
// M_p[a,b,c] = sum_children sum_{i,j,k} V[bx][a][i] V[by][b][j] V[bz][c][k] M_child[i,j,k],
// V[b][a][i] = S_a(child node i in parent coordinates), applied as three 1D passes.
__global__ __launch_bounds__(256) void k_m2m(const double *Mc, double *Mp, const double *Vg, int Lp, int Lc,
                                             int nupc, int nupp, int ns_par) {
    extern __shared__ double sm[];
    const int nc = Lc * Lc * Lc, np = Lp * Lp * Lp;
    const int nbuf = max(nc, max(Lc * Lc * Lp, Lc * Lp * Lp));
    double *sV = sm;                 // [2][Lp][Lc]
    double *b0 = sV + 2 * Lp * Lc;   // nbuf
    double *b1 = b0 + nbuf;          // nbuf
    const int tid = threadIdx.x;
    for (int t = tid; t < 2 * Lp * Lc; t += 256) sV[t] = Vg[t];
    const int64_t p = blockIdx.x;
    const int px = (int)(p / ((int64_t)ns_par * ns_par)), py = (int)((p / ns_par) % ns_par), pz = (int)(p % ns_par);
    const int nsc = 2 * ns_par;
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    const int VS = Lp * Lc;
    for (int bits = 0; bits < 8; bits++) {
        const int bx = bits >> 2, by = (bits >> 1) & 1, bz = bits & 1;
        const int64_t c = ((int64_t)(2 * px + bx) * nsc + (2 * py + by)) * nsc + (2 * pz + bz);
        __syncthreads();
        for (int t = tid; t < nc; t += 256) b0[t] = Mc[c * nupc + t];
        __syncthreads();
        const double *Vz = sV + bz * VS, *Vy = sV + by * VS, *Vx = sV + bx * VS;
        for (int t = tid; t < Lc * Lc * Lp; t += 256) {   // (i, j, cz)
            const int ij = t / Lp, cz = t % Lp;
            double s = 0;
            for (int k = 0; k < Lc; k++) s += Vz[cz * Lc + k] * b0[ij * Lc + k];
            b1[t] = s;
        }
        __syncthreads();
        for (int t = tid; t < Lc * Lp * Lp; t += 256) {   // (i, cy, cz)
            const int i = t / (Lp * Lp), cy = (t / Lp) % Lp, cz = t % Lp;
            double s = 0;
            for (int j = 0; j < Lc; j++) s += Vy[cy * Lc + j] * b1[(i * Lc + j) * Lp + cz];
            b0[t] = s;
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < 8; r++) {
            const int t = tid + 256 * r;
            if (t >= np) break;
            const int cx = t / (Lp * Lp), yz = t % (Lp * Lp);
            double s = 0;
            for (int i = 0; i < Lc; i++) s += Vx[cx * Lc + i] * b0[i * Lp * Lp + yz];
            acc[r] += s;
        }
    }
#pragma unroll
    for (int r = 0; r < 8; r++) {
        const int t = tid + 256 * r;
        if (t < nupp) Mp[p * nupp + t] = t < np ? acc[r] : 0.0;
    }
    for (int t = tid + 2048; t < nupp; t += 256) Mp[p * nupp + t] = 0.0;
}

// ---- L2L: child local expansion (order Lc) += M2M^T of the parent's (order Lp) ----
// The same with the 8 children side by side: each 1D pass runs over all
// children at once (3 barriers per parent instead of 4 per child), and the x
// pass sums the children in order.  Used when the buffers fit in 64 KiB.
__global__ __launch_bounds__(256) void k_m2m8(const double *Mc, double *Mp, const double *Vg, int Lp, int Lc,
                                              int nupc, int nupp, int ns_par) {
    extern __shared__ double sm[];
    const int nc = Lc * Lc * Lc, np = Lp * Lp * Lp;
    const int n1 = Lc * Lc * Lp, n2 = Lc * Lp * Lp;
    const int nbuf = max(nc, n2);
    double *sV = sm;                 // [2][Lp][Lc]
    double *b0 = sV + 2 * Lp * Lc;   // [8][nbuf]
    double *b1 = b0 + 8 * nbuf;      // [8][n1]
    const int tid = threadIdx.x;
    for (int t = tid; t < 2 * Lp * Lc; t += 256) sV[t] = Vg[t];
    const int64_t p = blockIdx.x;
    const int px = (int)(p / ((int64_t)ns_par * ns_par)), py = (int)((p / ns_par) % ns_par), pz = (int)(p % ns_par);
    const int nsc = 2 * ns_par;
    const int VS = Lp * Lc;
    for (int t = tid; t < 8 * nc; t += 256) {
        const int bits = t / nc, e = t % nc;
        const int bx = bits >> 2, by = (bits >> 1) & 1, bz = bits & 1;
        const int64_t c = ((int64_t)(2 * px + bx) * nsc + (2 * py + by)) * nsc + (2 * pz + bz);
        b0[bits * nbuf + e] = Mc[c * nupc + e];
    }
    __syncthreads();
    for (int t = tid; t < 8 * n1; t += 256) {   // child, (i, j, cz)
        const int bits = t / n1, u = t % n1;
        const int ij = u / Lp, cz = u % Lp;
        const double *Vz = sV + (bits & 1) * VS;
        double s = 0;
        for (int k = 0; k < Lc; k++) s += Vz[cz * Lc + k] * b0[bits * nbuf + ij * Lc + k];
        b1[bits * n1 + u] = s;
    }
    __syncthreads();
    for (int t = tid; t < 8 * n2; t += 256) {   // child, (i, cy, cz)
        const int bits = t / n2, u = t % n2;
        const int i = u / (Lp * Lp), cy = (u / Lp) % Lp, cz = u % Lp;
        const double *Vy = sV + ((bits >> 1) & 1) * VS;
        double s = 0;
        for (int j = 0; j < Lc; j++) s += Vy[cy * Lc + j] * b1[bits * n1 + (i * Lc + j) * Lp + cz];
        b0[bits * nbuf + u] = s;
    }
    __syncthreads();
    for (int t = tid; t < nupp; t += 256) {
        double acc = 0;
        if (t < np) {
            const int cx = t / (Lp * Lp), yz = t % (Lp * Lp);
            for (int bits = 0; bits < 8; bits++) {
                const double *Vx = sV + (bits >> 2) * VS;
                double s = 0;
                for (int i = 0; i < Lc; i++) s += Vx[cx * Lc + i] * b0[bits * nbuf + i * Lp * Lp + yz];
                acc += s;
            }
        }
        Mp[p * nupp + t] = acc;
    }
}

__global__ __launch_bounds__(256) void k_l2l(const double *Lpar, double *Lch, const double *Vg, int Lp, int Lc,
                                             int nupp, int nupc, int ns_child) {
    extern __shared__ double sm[];
    const int nc = Lc * Lc * Lc, np = Lp * Lp * Lp;
    const int nbuf = max(np, max(Lp * Lp * Lc, Lp * Lc * Lc));
    double *sV = sm;
    double *b0 = sV + 2 * Lp * Lc;
    double *b1 = b0 + nbuf;
    const int tid = threadIdx.x;
    for (int t = tid; t < 2 * Lp * Lc; t += 256) sV[t] = Vg[t];
    const int64_t c = blockIdx.x;
    const int cx = (int)(c / ((int64_t)ns_child * ns_child)), cy = (int)((c / ns_child) % ns_child),
              cz = (int)(c % ns_child);
    const int nsp = ns_child / 2;
    const int64_t p = ((int64_t)(cx >> 1) * nsp + (cy >> 1)) * nsp + (cz >> 1);
    const int VS = Lp * Lc;
    const double *Vz = sV + (cz & 1) * VS, *Vy = sV + (cy & 1) * VS, *Vx = sV + (cx & 1) * VS;
    for (int t = tid; t < np; t += 256) b0[t] = Lpar[p * nupp + t];
    __syncthreads();
    for (int t = tid; t < Lp * Lp * Lc; t += 256) {   // (a, b, k) = sum_c V[c][k] Lp[a, b, c]
        const int ab = t / Lc, k = t % Lc;
        double s = 0;
        for (int cc = 0; cc < Lp; cc++) s += Vz[cc * Lc + k] * b0[ab * Lp + cc];
        b1[t] = s;
    }
    __syncthreads();
    for (int t = tid; t < Lp * Lc * Lc; t += 256) {   // (a, j, k) = sum_b V[b][j] (a, b, k)
        const int a = t / (Lc * Lc), j = (t / Lc) % Lc, k = t % Lc;
        double s = 0;
        for (int bb = 0; bb < Lp; bb++) s += Vy[bb * Lc + j] * b1[(a * Lp + bb) * Lc + k];
        b0[t] = s;
    }
    __syncthreads();
    for (int t = tid; t < nc; t += 256) {   // (i, j, k) = sum_a V[a][i] (a, j, k)
        const int i = t / (Lc * Lc), jk = t % (Lc * Lc);
        double s = 0;
        for (int a = 0; a < Lp; a++) s += Vx[a * Lc + i] * b0[a * Lc * Lc + jk];
        Lch[c * nupc + t] += s;
    }
}

// ---- far periodic images: L_root = C_per M_root, E_per = 1/2 M.C M -----------
// 64 rows per block, the contraction split over the block's 4 waves and
// summed in a fixed order; the energy dot product follows in one block.
// one block per (64 rows k, slice of the columns l): part[slice][k] = sum over the slice of C[l][k] M[l]
__global__ __launch_bounds__(256) void k_cper(const double *C, const double *M, double *part, int nu, int nup) {
    __shared__ double red[4][64];
    const int r = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int k = blockIdx.x * 64 + r, slice = blockIdx.y;
    const int l0 = nu * slice / kCperSlices, l1 = nu * (slice + 1) / kCperSlices;
    double s = 0;
    if (k < nu)
        for (int l = l0 + w; l < l1; l += 4) s += C[(int64_t)l * nup + k] * M[l];
    red[w][r] = s;
    __syncthreads();
    if (w == 0 && k < nup) part[(int64_t)slice * nup + k] = (red[0][r] + red[1][r]) + (red[2][r] + red[3][r]);
}

// L_root[k] = sum of the slices in slice order (zero in the padding rows)
__global__ void k_cper_sum(const double *part, double *Lr, int nu, int nup) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nup) return;
    double s = 0;
    if (k < nu)
        for (int sl = 0; sl < kCperSlices; sl++) s += part[(int64_t)sl * nup + k];
    Lr[k] = s;
}

__global__ __launch_bounds__(256) void k_cper_dot(const double *M, const double *Lr, int nu, double *terms) {
    __shared__ double red[256];
    const int t = threadIdx.x;
    double s = 0;
    for (int k = t; k < nu; k += 256) s += M[k] * Lr[k];
    red[t] = s;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (t < off) red[t] += red[t + off];
        __syncthreads();
    }
    if (t == 0) terms[2] = 0.5 * red[0];
}

// ---- far energy per leaf: 1/2 Q_t . Lambda_t ---------------------------------
__global__ __launch_bounds__(256) void k_leafdot(const double *Q, const double *Lam, int nu, int nup, double *eleaf) {
    __shared__ double red[256];
    const int64_t leaf = blockIdx.x;
    double s = 0;
    for (int k = threadIdx.x; k < nu; k += 256) s += Q[leaf * nup + k] * Lam[leaf * nup + k];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) eleaf[leaf] = 0.5 * red[0];
}

// ---- L2P: far-field forces and fields at the atoms (adjoint of P2M) --------
// phi(y) = sum_k Lambda_k S_k(y); F = -(q grad phi + mu_a grad d_a phi + Th_ab grad d_a d_b phi
// + Om_abc grad d_a d_b d_c phi),
// dE/dmu = grad phi.  One thread per atom (leaf order): its 1D bases in
// registers, the leaf's expansion contracted along z, then y, then x.
template <int L, int ORD, bool FIELD>
__global__ __launch_bounds__(256, L <= 6 ? 2 : 1) void k_l2p(Particles P, const int32_t *leaf_in, const int32_t *perm,
                                             const double *tab, int nup, double hinv, const double *Lam, double *F,
                                             double *G, int64_t n) {
    constexpr int ND = ORD + 2;   // derivative orders 0..ORD+1
    __shared__ double sH[L * L];
    const int tid = threadIdx.x;
    for (int t = tid; t < L * L; t += 256) sH[t] = tab[L + t];
    __syncthreads();
    const int64_t slot = blockIdx.x * (int64_t)256 + tid;
    if (slot >= n) return;
    const double *lam = Lam + (int64_t)leaf_in[perm[slot]] * nup;
    double Sx[ND * L], Sy[ND * L], Sz[ND * L];
    cheb_basis<ND, L>(P.x[slot] * hinv, hinv, sH, Sx, L);
    cheb_basis<ND, L>(P.y[slot] * hinv, hinv, sH, Sy, L);
    cheb_basis<ND, L>(P.z[slot] * hinv, hinv, sH, Sz, L);
    {
        double phi[ND][ND][ND];
#pragma unroll
        for (int x = 0; x < ND; x++)
#pragma unroll
            for (int y = 0; y < ND; y++)
#pragma unroll
                for (int z = 0; z < ND; z++) phi[x][y][z] = 0;
#pragma unroll
        for (int i = 0; i < L; i++) {
            double h[ND][ND];
#pragma unroll
            for (int y = 0; y < ND; y++)
#pragma unroll
                for (int z = 0; z < ND; z++) h[y][z] = 0;
#pragma unroll
            for (int j = 0; j < L; j++) {
                double g[ND];
#pragma unroll
                for (int z = 0; z < ND; z++) g[z] = 0;
                const double *row = lam + (i * L + j) * L;
#pragma unroll
                for (int k = 0; k < L; k++) {
                    const double lv = row[k];
#pragma unroll
                    for (int z = 0; z < ND; z++) g[z] += lv * Sz[z * L + k];
                }
#pragma unroll
                for (int y = 0; y < ND; y++)
#pragma unroll
                    for (int z = 0; z + y < ND; z++) h[y][z] += Sy[y * L + j] * g[z];
            }
#pragma unroll
            for (int x = 0; x < ND; x++)
#pragma unroll
                for (int y = 0; x + y < ND; y++)
#pragma unroll
                    for (int z = 0; x + y + z < ND; z++) phi[x][y][z] += Sx[x * L + i] * h[y][z];
        }
        // gradient components
        const double q = P.q[slot];
        double f[3];
#pragma unroll
        for (int c = 0; c < 3; c++) {
            const int ex = c == 0, ey = c == 1, ez = c == 2;
            double v = q * phi[ex][ey][ez];
            if (ORD >= 1) {
                const double m0 = P.mu[slot], m1 = P.mu[n + slot], m2 = P.mu[2 * n + slot];
                v += m0 * phi[1 + ex][ey][ez] + m1 * phi[ex][1 + ey][ez] + m2 * phi[ex][ey][1 + ez];
            }
            if (ORD >= 2) {
                const double xx = P.th[slot], xy = P.th[n + slot], xz = P.th[2 * n + slot];
                const double yy = P.th[3 * n + slot], yz = P.th[4 * n + slot], zz = P.th[5 * n + slot];
                v += xx * phi[2 + ex][ey][ez] + yy * phi[ex][2 + ey][ez] + zz * phi[ex][ey][2 + ez] +
                     2 * xy * phi[1 + ex][1 + ey][ez] + 2 * xz * phi[1 + ex][ey][1 + ez] +
                     2 * yz * phi[ex][1 + ey][1 + ez];
            }
            if (ORD >= 3) {
                // Omega : grad^3 d_c phi, each stored component with its multiplicity
                const double *o = P.om + slot;
                v += o[0] * phi[3 + ex][ey][ez] + 3 * o[n] * phi[2 + ex][1 + ey][ez] +
                     3 * o[2 * n] * phi[2 + ex][ey][1 + ez] + 3 * o[3 * n] * phi[1 + ex][2 + ey][ez] +
                     6 * o[4 * n] * phi[1 + ex][1 + ey][1 + ez] + 3 * o[5 * n] * phi[1 + ex][ey][2 + ez] +
                     o[6 * n] * phi[ex][3 + ey][ez] + 3 * o[7 * n] * phi[ex][2 + ey][1 + ez] +
                     3 * o[8 * n] * phi[ex][1 + ey][2 + ez] + o[9 * n] * phi[ex][ey][3 + ez];
            }
            f[c] = -v;
        }
        F[slot] = f[0];
        F[n + slot] = f[1];
        F[2 * n + slot] = f[2];
        if (FIELD) {
            G[slot] = phi[1][0][0];
            G[n + slot] = phi[0][1][0];
            G[2 * n + slot] = phi[0][0][1];
        }
    }
}

// ---- energy reduction (two deterministic stages) -----------------------------
__global__ __launch_bounds__(kRedBlocks) void k_reduce2(const double *part, double *terms, double *energy, double xi,
                                                 double vol) {
    __shared__ double red[4][kRedBlocks];
    const int t = threadIdx.x;
    for (int c = 0; c < 4; c++) red[c][t] = part[t * 4 + c];
    __syncthreads();
    for (int off = kRedBlocks / 2; off > 0; off >>= 1) {
        if (t < off)
            for (int c = 0; c < 4; c++) red[c][t] += red[c][t + off];
        __syncthreads();
    }
    if (t == 0) {
        const double near = red[0][0], self = red[1][0], Q = red[2][0], far = red[3][0];
        const double per = terms[2];
        const double bg = -kPi * Q * Q / (2 * vol * xi * xi);
        const double tot = near + far + self + bg;
        terms[0] = near;
        terms[1] = far - per;
        terms[3] = self;
        terms[4] = bg;
        terms[5] = tot;
        terms[6] = Q;
        if (energy) *energy = tot;
    }
}


// ---- plan-time builders ------------------------------------------------------
// K_d[k][l] = H(w (1/2 (r_k - r_l) - d)) stored as [d][l][k]; zero for the 27 adjacent offsets and
// for padded rows / columns.
//
// Only one operator per class of the cube's symmetries is evaluated, as the paper's precomputation
// of its M2L approximations does (ANKH-FMM, mutual interactions).  A symmetry g of the cube permutes
// the axes and reflects some of them, (g v)_c = s_c v_{p_c}; it maps the 316 far offsets onto
// themselves in 16 classes, one representative r per class with 3 >= r_x >= r_y >= r_z >= 0 and
// r_x >= 2.  The Chebyshev nodes are symmetric about the cell centre (r_{L-1-i} = -r_i), so for
// d = g r the node pair (k, l) sees the distance of the representative's pair (k~, l~) with
// k~_{p_c} = k_c where s_c = +1 and L-1-k_c where s_c = -1; H depends on the distance only, hence
// K_d[k][l] = K_r[k~][l~].  The representatives are built by the formula above, then every
// offset's operator is read from its representative with the node indices moved.
constexpr int kNumCls = 16;
struct SymTable {
    int cls[kNumOff];            // class of each offset slot, -1 for the 27 adjacent offsets
    unsigned char perm[kNumOff]; // p_0 | p_1 << 2 | p_2 << 4
    unsigned char refl[kNumOff]; // bit c set: s_c = -1
    signed char rep[kNumCls][3]; // the representatives
};

SymTable make_sym_table() {
    SymTable T{};
    int nc = 0;
    for (int x = 2; x <= 3; x++)
        for (int y = 0; y <= x; y++)
            for (int z = 0; z <= y; z++) {
                T.rep[nc][0] = (signed char)x;
                T.rep[nc][1] = (signed char)y;
                T.rep[nc][2] = (signed char)z;
                nc++;
            }
    for (int di = 0; di < kNumOff; di++) {
        const int d[3] = {di / 49 - 3, (di / 7) % 7 - 3, di % 7 - 3};
        const int a[3] = {std::abs(d[0]), std::abs(d[1]), std::abs(d[2])};
        T.cls[di] = -1;
        if (std::max(a[0], std::max(a[1], a[2])) < 2) continue;
        // the axes ordered by |d_c|, largest first (ties in axis order): axis c goes to position p_c
        int ord[3] = {0, 1, 2};
        std::stable_sort(ord, ord + 3, [&](int u, int v) { return a[u] > a[v]; });
        int p[3];
        for (int j = 0; j < 3; j++) p[ord[j]] = j;
        const int r[3] = {a[ord[0]], a[ord[1]], a[ord[2]]};
        for (int c = 0; c < kNumCls; c++)
            if (T.rep[c][0] == r[0] && T.rep[c][1] == r[1] && T.rep[c][2] == r[2]) T.cls[di] = c;
        T.perm[di] = (unsigned char)(p[0] | p[1] << 2 | p[2] << 4);
        T.refl[di] = (unsigned char)((d[0] < 0) | (d[1] < 0) << 1 | (d[2] < 0) << 2);
    }
    return T;
}

// the class representatives, R[c][l][k] (kNumCls x nup x nup)
__global__ void k_build_m2l_reps(double *R, const double *tab, int L, int nu, int nup, double w, double xi,
                                 SymTable T) {
    const int64_t tot = (int64_t)kNumCls * nup * nup;
    const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (idx >= tot) return;
    const int k = (int)(idx % nup);
    const int l = (int)((idx / nup) % nup);
    const int c = (int)(idx / ((int64_t)nup * nup));
    double v = 0;
    if (k < nu && l < nu) {
        const int ki[3] = {k / (L * L), (k / L) % L, k % L};
        const int li[3] = {l / (L * L), (l / L) % L, l % L};
        double r2 = 0;
        for (int a = 0; a < 3; a++) {
            const double u = w * (0.5 * (tab[ki[a]] - tab[li[a]]) - T.rep[c][a]);
            r2 += u * u;
        }
        const double r = sqrt(r2);
        v = erfc(xi * r) / r;
    }
    R[idx] = v;
}

// every offset's operator from its class representative
__global__ void k_expand_m2l(double *K, const double *R, int L, int nu, int nup, SymTable T) {
    const int64_t tot = (int64_t)kNumOff * nup * nup;
    const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (idx >= tot) return;
    const int k = (int)(idx % nup);
    const int l = (int)((idx / nup) % nup);
    const int di = (int)(idx / ((int64_t)nup * nup));
    const int c = T.cls[di];
    double v = 0;
    if (c >= 0 && k < nu && l < nu) {
        const int ki[3] = {k / (L * L), (k / L) % L, k % L};
        const int li[3] = {l / (L * L), (l / L) % L, l % L};
        int kt[3], lt[3];
        for (int a = 0; a < 3; a++) {
            const int pa = (T.perm[di] >> (2 * a)) & 3;
            const bool m = (T.refl[di] >> a) & 1;
            kt[pa] = m ? L - 1 - ki[a] : ki[a];
            lt[pa] = m ? L - 1 - li[a] : li[a];
        }
        const int kk = (kt[0] * L + kt[1]) * L + kt[2], ll = (lt[0] * L + lt[1]) * L + lt[2];
        v = R[((int64_t)c * nup + ll) * nup + kk];
    }
    K[idx] = v;
}

// C_per[l][k] = sum_{I in Z_p, |I|_inf >= 2} H(x_k - x_l - edge I) on the root grid
__global__ void k_build_cper(double *C, const double *tab, int L, int nu, int nup, double edge, double xi, int p) {
    const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (idx >= (int64_t)nup * nup) return;
    const int k = (int)(idx % nup), l = (int)(idx / nup);
    double s = 0;
    if (k < nu && l < nu) {
        const double rB = 0.5 * edge;
        const int ki[3] = {k / (L * L), (k / L) % L, k % L};
        const int li[3] = {l / (L * L), (l / L) % L, l % L};
        double b[3];
        for (int c = 0; c < 3; c++) b[c] = rB * (tab[ki[c]] - tab[li[c]]);
        for (int ix = -p; ix <= p; ix++)
            for (int iy = -p; iy <= p; iy++)
                for (int iz = -p; iz <= p; iz++) {
                    if (max(abs(ix), max(abs(iy), abs(iz))) < 2) continue;
                    const double u0 = b[0] - edge * ix, u1 = b[1] - edge * iy, u2 = b[2] - edge * iz;
                    const double r = sqrt(u0 * u0 + u1 * u1 + u2 * u2);
                    s += erfc(xi * r) / r;
                }
    }
    C[idx] = s;
}

inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

// Far-field derivatives in the charges and quadrupoles, then the output: per
// leaf-order atom, the leaf's local expansion against the basis values
// (dE/dq) and its second derivatives (dE/dTh, full symmetric), added to the
// near-field part (near [7][n]), the self terms -(2 xi / sqrt(pi)) q and
// -(xi / sqrt(pi)) (8 xi^4 / 5) 2 Th, and the background -pi Q / (V xi^2).
// dE/dTh is reported as its traceless part per stored component (xx, xy, xz,
// yy, yz, zz) = (G_xx - t, 2 G_xy, 2 G_xz, G_yy - t, 2 G_yz, G_zz - t),
// t = tr G / 3: E is defined for traceless Theta only.  Written in caller order.
template <int L>
__global__ __launch_bounds__(256) void k_l2p_moments(Particles P, const int32_t *leaf_in, const int32_t *perm,
                                                     const double *tab, int nup, double hinv, const double *Lam,
                                                     const double *near, const double *terms, double xi, double vol,
                                                     int ord, double *dEdq, double *dEdth, int64_t n) {
    constexpr int ND = 3;
    __shared__ double sH[L * L];
    const int tid = threadIdx.x;
    for (int t = tid; t < L * L; t += 256) sH[t] = tab[L + t];
    __syncthreads();
    const int64_t s = blockIdx.x * (int64_t)256 + tid;
    if (s >= n) return;
    const double *lam = Lam + (int64_t)leaf_in[perm[s]] * nup;
    double Sx[ND * L], Sy[ND * L], Sz[ND * L];
    cheb_basis<ND, L>(P.x[s] * hinv, hinv, sH, Sx, L);
    cheb_basis<ND, L>(P.y[s] * hinv, hinv, sH, Sy, L);
    cheb_basis<ND, L>(P.z[s] * hinv, hinv, sH, Sz, L);
    double phi[ND][ND][ND];
#pragma unroll
    for (int x = 0; x < ND; x++)
#pragma unroll
        for (int y = 0; y < ND; y++)
#pragma unroll
            for (int z = 0; z < ND; z++) phi[x][y][z] = 0;
#pragma unroll
    for (int i = 0; i < L; i++) {
        double h[ND][ND];
#pragma unroll
        for (int y = 0; y < ND; y++)
#pragma unroll
            for (int z = 0; z < ND; z++) h[y][z] = 0;
#pragma unroll
        for (int j = 0; j < L; j++) {
            double g[ND] = {0, 0, 0};
            const double *row = lam + (i * L + j) * L;
#pragma unroll
            for (int k = 0; k < L; k++) {
                const double lv = row[k];
#pragma unroll
                for (int z = 0; z < ND; z++) g[z] += lv * Sz[z * L + k];
            }
#pragma unroll
            for (int y = 0; y < ND; y++)
#pragma unroll
                for (int z = 0; z + y < ND; z++) h[y][z] += Sy[y * L + j] * g[z];
        }
#pragma unroll
        for (int x = 0; x < ND; x++)
#pragma unroll
            for (int y = 0; x + y < ND; y++)
#pragma unroll
                for (int z = 0; x + y + z < ND; z++) phi[x][y][z] += Sx[x * L + i] * h[y][z];
    }
    const double sp = sqrt(kPi);
    const int64_t i = perm[s];
    if (dEdq) {
        const double Q = terms[6];
        dEdq[i] = near[s] + phi[0][0][0] - (2 * xi / sp) * P.q[s] - kPi * Q / (vol * xi * xi);
    }
    if (dEdth) {
        double G[6] = {near[n + s] + phi[2][0][0], near[2 * n + s] + phi[1][1][0], near[3 * n + s] + phi[1][0][1],
                       near[4 * n + s] + phi[0][2][0], near[5 * n + s] + phi[0][1][1], near[6 * n + s] + phi[0][0][2]};
        if (ord >= 2) {
            const double cs = -(xi / sp) * (8 * xi * xi * xi * xi / 5) * 2;
            for (int c = 0; c < 6; c++) G[c] += cs * P.th[c * n + s];
        }
        const double t = (G[0] + G[3] + G[5]) / 3;
        double *o = dEdth + 6 * i;
        o[0] = G[0] - t;
        o[1] = 2 * G[1];
        o[2] = 2 * G[2];
        o[3] = G[3] - t;
        o[4] = 2 * G[4];
        o[5] = G[5] - t;
    }
}

}  // namespace

// ---- launchers ---------------------------------------------------------------
hipError_t launch_zero_i32(int32_t *p, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero_i32, dim3(nblk(n, 256)), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_zero_f64(double *p, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero_f64, dim3(nblk(n, 256)), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_convert_f32(const double *src, float *dst, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_to_f32, dim3(nblk(n, 256)), dim3(256), 0, s, src, dst, n);
    return hipGetLastError();
}

hipError_t launch_sort(ankh_plan_s *pl, const double *pos, const double *q, const double *mu, const double *th) {
    hipStream_t s = pl->stream;
    const double w = pl->edge / pl->nside;
    hipError_t e;
    // the scan leaves the counts at zero; they are cleared here only at the first binning of a plan or
    // after a binning whose launches failed
    if (pl->count_dirty) {
        if ((e = launch_zero_i32(pl->d_count, pl->nleaf, s)) != hipSuccess) return e;
        pl->count_dirty = false;
    }
    hipLaunchKernelGGL(k_bin, dim3(nblk(pl->n, 256)), dim3(256), 0, s, pl->n, pos, q, pl->rB, pl->edge, w,
                       pl->nside, pl->d_leaf, pl->d_count, pl->d_rank, pl->d_err);
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, pl->d_count, pl->d_offs, pl->nleaf);
    hipLaunchKernelGGL(k_scatter, dim3(nblk(pl->n, 256)), dim3(256), 0, s, pl->n, pl->d_leaf, pl->d_offs,
                       pl->d_rank, pl->d_tmp);
    hipLaunchKernelGGL(k_segsort, dim3((unsigned)((pl->nleaf + 3) / 4)), dim3(256), 0, s, pl->d_offs, pl->d_tmp,
                       pl->d_perm, pl->nleaf);
    e = hipGetLastError();
    if (e != hipSuccess) pl->count_dirty = true;
    return e;
}

hipError_t launch_gather(ankh_plan_s *pl, const double *pos, const double *q, const double *mu, const double *th,
                         const double *om) {
    const double w = pl->edge / pl->nside;
    const bool mixed = is_mixed(pl);
#define ANKH_GATHER(O, M)                                                                                           \
    hipLaunchKernelGGL((k_gather<O, M>), dim3(nblk(pl->n, 256)), dim3(256), 0, pl->stream, pl->n, pl->d_perm, pos, \
                       q, mu, th, om, pl->rB, pl->edge, w, pl->nside, pl->P, pl->d_err)
    switch (pl->max_order) {
        case 0: if (mixed) ANKH_GATHER(0, true); else ANKH_GATHER(0, false); break;
        case 1: if (mixed) ANKH_GATHER(1, true); else ANKH_GATHER(1, false); break;
        case 2: if (mixed) ANKH_GATHER(2, true); else ANKH_GATHER(2, false); break;
        default: if (mixed) ANKH_GATHER(3, true); else ANKH_GATHER(3, false); break;
    }
#undef ANKH_GATHER
    return hipGetLastError();
}

#define ANKH_FOR_ORDER(L, X) \
    switch (L) {                 \
        case 2: X(2); break;     \
        case 3: X(3); break;     \
        case 4: X(4); break;     \
        case 5: X(5); break;     \
        case 6: X(6); break;     \
        case 7: X(7); break;     \
        case 8: X(8); break;     \
        case 9: X(9); break;     \
        default: X(10); break;   \
    }

hipError_t launch_p2m(ankh_plan_s *pl, int ord) {
    const int L = pl->order;
    const double hinv = 2.0 / (pl->edge / pl->nside);
    double *Q = pl->d_M + pl->lv[pl->depth].cell0 * pl->nup;
    const size_t shm = 0;
    dim3 g((unsigned)pl->nleaf), b(256);
#define ANKH_P2M(LL)                                                                                              \
    if (ord == 0)                                                                                                 \
        hipLaunchKernelGGL((k_p2m<LL, 0>), g, b, shm, pl->stream, pl->P, pl->d_offs, pl->d_tab, pl->nu, pl->nup, \
                           hinv, Q, pl->n);                                                                       \
    else if (ord == 1)                                                                                            \
        hipLaunchKernelGGL((k_p2m<LL, 1>), g, b, shm, pl->stream, pl->P, pl->d_offs, pl->d_tab, pl->nu, pl->nup, \
                           hinv, Q, pl->n);                                                                       \
    else if (ord == 2)                                                                                            \
        hipLaunchKernelGGL((k_p2m<LL, 2>), g, b, shm, pl->stream, pl->P, pl->d_offs, pl->d_tab, pl->nu, pl->nup, \
                           hinv, Q, pl->n);                                                                       \
    else                                                                                                          \
        hipLaunchKernelGGL((k_p2m<LL, 3>), g, b, shm, pl->stream, pl->P, pl->d_offs, pl->d_tab, pl->nu, pl->nup, \
                           hinv, Q, pl->n);
    ANKH_FOR_ORDER(L, ANKH_P2M)
#undef ANKH_P2M
    return hipGetLastError();
}

static size_t mlshm(int Lp, int Lc) {
    const int nbuf = std::max(std::max(Lc * Lc * Lc, Lp * Lp * Lp),
                              std::max(std::max(Lc * Lc * Lp, Lc * Lp * Lp), Lp * Lp * Lc));
    return sizeof(double) * (2 * Lp * Lc + 2 * nbuf);
}

// The root (level 0) may carry its own, higher order: M2M from level 1 into
// the root and L2L out of it then use the rectangular root matrices.
hipError_t launch_m2m(ankh_plan_s *pl, int e_par) {
    const ankh::Level &P = pl->lv[e_par], &C = pl->lv[e_par + 1];
    const bool root = e_par == 0;
    const int Lp = root ? pl->order0 : pl->order, Lc = pl->order;
    const double *V = root ? pl->d_tab0 + pl->order0 : pl->d_tab + Lc + Lc * Lc;
    double *Mp = root ? pl->d_rootM : pl->d_M + P.cell0 * pl->nup;
    const int nupp = root ? pl->nup0 : pl->nup;
    const size_t shm8 = sizeof(double) * (2 * Lp * Lc + 8 * std::max(Lc * Lc * Lc, Lc * Lp * Lp) + 8 * Lc * Lc * Lp);
    if (shm8 <= 65536)
        hipLaunchKernelGGL(k_m2m8, dim3((unsigned)P.ncell), dim3(256), shm8, pl->stream,
                           pl->d_M + C.cell0 * pl->nup, Mp, V, Lp, Lc, pl->nup, nupp, P.nside);
    else
        hipLaunchKernelGGL(k_m2m, dim3((unsigned)P.ncell), dim3(256), mlshm(Lp, Lc), pl->stream,
                           pl->d_M + C.cell0 * pl->nup, Mp, V, Lp, Lc, pl->nup, nupp, P.nside);
    return hipGetLastError();
}

hipError_t launch_l2l(ankh_plan_s *pl, int e_child) {
    const ankh::Level &P = pl->lv[e_child - 1], &C = pl->lv[e_child];
    const bool root = e_child == 1;
    const int Lp = root ? pl->order0 : pl->order, Lc = pl->order;
    const double *V = root ? pl->d_tab0 + pl->order0 : pl->d_tab + Lc + Lc * Lc;
    const double *Lpar = root ? pl->d_rootL : pl->d_L + P.cell0 * pl->nup;
    const int nupp = root ? pl->nup0 : pl->nup;
    hipLaunchKernelGGL(k_l2l, dim3((unsigned)C.ncell), dim3(256), mlshm(Lp, Lc), pl->stream, Lpar,
                       pl->d_L + C.cell0 * pl->nup, V, Lp, Lc, nupp, pl->nup, C.nside);
    return hipGetLastError();
}

hipError_t launch_cper(ankh_plan_s *pl) {
    hipLaunchKernelGGL(k_cper, dim3((pl->nup0 + 63) / 64, kCperSlices), dim3(256), 0, pl->stream, pl->d_Cper,
                       pl->d_rootM, pl->d_cper_part, pl->nu0, pl->nup0);
    hipLaunchKernelGGL(k_cper_sum, dim3((pl->nup0 + 255) / 256), dim3(256), 0, pl->stream, pl->d_cper_part,
                       pl->d_rootL, pl->nu0, pl->nup0);
    hipLaunchKernelGGL(k_cper_dot, dim3(1), dim3(256), 0, pl->stream, pl->d_rootM, pl->d_rootL, pl->nu0, pl->d_terms);
    return hipGetLastError();
}

hipError_t launch_leafdot(ankh_plan_s *pl) {
    const size_t off = pl->lv[pl->depth].cell0 * pl->nup;
    hipLaunchKernelGGL(k_leafdot, dim3((unsigned)pl->nleaf), dim3(256), 0, pl->stream, pl->d_M + off, pl->d_L + off,
                       pl->nu, pl->nup, pl->d_eleaf);
    return hipGetLastError();
}

hipError_t launch_l2p(ankh_plan_s *pl, int ord, bool fields) {
    const int L = pl->order;
    const double hinv = 2.0 / (pl->edge / pl->nside);
    const double *Lam = pl->d_L + pl->lv[pl->depth].cell0 * pl->nup;
    dim3 g((unsigned)((pl->n + 255) / 256)), b(256);
#define ANKH_L2P3(LL, O, FL)                                                                                       \
    hipLaunchKernelGGL((k_l2p<LL, O, FL>), g, b, 0, pl->stream, pl->P, pl->d_leaf, pl->d_perm, pl->d_tab, pl->nup, \
                       hinv, Lam, pl->d_F, pl->d_G, pl->n)
#define ANKH_L2P(LL)                                                                         \
    if (ord == 0) { if (fields) ANKH_L2P3(LL, 0, true); else ANKH_L2P3(LL, 0, false); }     \
    else if (ord == 1) { if (fields) ANKH_L2P3(LL, 1, true); else ANKH_L2P3(LL, 1, false); } \
    else if (ord == 2) { if (fields) ANKH_L2P3(LL, 2, true); else ANKH_L2P3(LL, 2, false); } \
    else { if (fields) ANKH_L2P3(LL, 3, true); else ANKH_L2P3(LL, 3, false); }
    ANKH_FOR_ORDER(L, ANKH_L2P)
#undef ANKH_L2P3
#undef ANKH_L2P
    return hipGetLastError();
}

hipError_t launch_l2p_moments(ankh_plan_s *pl, int ord, const double *near, double *dEdq, double *dEdth) {
    const int L = pl->order;
    const double hinv = 2.0 / (pl->edge / pl->nside);
    const double *Lam = pl->d_L + pl->lv[pl->depth].cell0 * pl->nup;
    const double vol = pl->edge * pl->edge * pl->edge;
    dim3 g((unsigned)((pl->n + 255) / 256)), b(256);
#define ANKH_L2PM(LL)                                                                                              \
    hipLaunchKernelGGL((k_l2p_moments<LL>), g, b, 0, pl->stream, pl->P, pl->d_leaf, pl->d_perm, pl->d_tab, pl->nup, \
                       hinv, Lam, near, pl->d_terms, pl->xi, vol, ord, dEdq, dEdth, pl->n)
    ANKH_FOR_ORDER(L, ANKH_L2PM)
#undef ANKH_L2PM
    return hipGetLastError();
}

hipError_t launch_reduce(ankh_plan_s *pl, double *energy_out) {
    hipLaunchKernelGGL(k_reduce2, dim3(1), dim3(kRedBlocks), 0, pl->stream, pl->d_part, pl->d_terms, energy_out,
                       pl->xi, pl->edge * pl->edge * pl->edge);
    return hipGetLastError();
}

size_t m2l_reps_elems(const ankh_plan_s *pl) { return (size_t)kNumCls * pl->nup * pl->nup; }

hipError_t launch_build_m2l(ankh_plan_s *pl, int e, double *K, double *reps) {
    static const SymTable T = make_sym_table();
    const int64_t nr = (int64_t)m2l_reps_elems(pl), tot = (int64_t)kNumOff * pl->nup * pl->nup;
    hipLaunchKernelGGL(k_build_m2l_reps, dim3(nblk(nr, 256)), dim3(256), 0, pl->stream, reps, pl->d_tab, pl->order,
                       pl->nu, pl->nup, pl->lv[e].width, pl->xi, T);
    hipLaunchKernelGGL(k_expand_m2l, dim3(nblk(tot, 256)), dim3(256), 0, pl->stream, K, reps, pl->order, pl->nu,
                       pl->nup, T);
    return hipGetLastError();
}

hipError_t launch_build_cper(ankh_plan_s *pl) {
    const int64_t tot = (int64_t)pl->nup0 * pl->nup0;
    hipLaunchKernelGGL(k_build_cper, dim3(nblk(tot, 128)), dim3(128), 0, pl->stream, pl->d_Cper, pl->d_tab0,
                       pl->order0, pl->nu0, pl->nup0, pl->edge, pl->xi, pl->images);
    return hipGetLastError();
}

}  // namespace ankh
