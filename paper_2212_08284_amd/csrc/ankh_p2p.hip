// P2P near field (ANKH-FMM, Alg. 3 step 3): direct pair sums of the
// multipole operator on H = erfc(xi r)/r between every leaf and the 27
// leaves adjacent to it (periodic, so at depth <= 1 a leaf meets images of
// itself), excluding an atom with itself at zero shift.
//
// Gather form: a block owns one target leaf; every target atom sums over all
// its sources, so each ordered pair is evaluated once per endpoint and no
// atomics are needed.  Sources are streamed through LDS in chunks drawn from
// the concatenation of the 27 neighbour leaves, already shifted into the
// target leaf's frame; the block's threads are split into (target, slice)
// pairs so that small leaves still fill the block, and the slices are
// reduced in a fixed order.
//
// Pair terms (r = x_i - x_j, D_x = q + mu.d + Th:dd on x, and the mirrored
// operator on the source):  with B_0 = H, B_{n+1} = -(1/r) dB_n/dr,
//   E_ij = c0 B0 + c1 B1 + c2 B2 + c3 B3 + c4 B4,
//   c0 = qi qk
//   c1 = qi (dk.r) - qk (di.r) + di.dk
//   c2 = -(di.r)(dk.r) + qi r.Qk.r + qk r.Qi.r + 2 di.Qk.r - 2 dk.Qi.r + 2 Qi:Qk
//   c3 = -(di.r) r.Qk.r + (dk.r) r.Qi.r - 4 (Qi r).(Qk r)
//   c4 = (r.Qi.r)(r.Qk.r)
// grad_r E_ij = sum_n grad(c_n) B_n - r sum_n c_n B_{n+1};  F_i = -sum_j grad_r E_ij;
// dE/d(di) = B1 (dk - qk r) + B2 (2 Qk r - (dk.r) r) - B3 (r.Qk.r) r.
// The radial functions follow B_n = [(2n-1) B_{n-1} + (2 xi^2)^n exp(-xi^2 r^2)/(xi sqrt(pi))] / r^2.
#include <cmath>

#include "ankh_internal.h"

namespace ankh {
namespace {

constexpr int CH = 256;   // sources per LDS chunk

struct P2PArgs {
    const double *x, *y, *z;
    const double *q, *mu, *th;
    const float *qf, *muf, *thf;
    const int32_t *offs;
    int64_t n;
    int nside, depth;
    double w, xi;
    double *eatom, *F, *G;
};

template <typename R> __device__ inline R dev_erfc(R v);
template <> __device__ inline double dev_erfc<double>(double v) { return erfc(v); }
template <> __device__ inline float dev_erfc<float>(float v) { return erfcf(v); }
template <typename R> __device__ inline R dev_exp(R v);
template <> __device__ inline double dev_exp<double>(double v) { return exp(v); }
template <> __device__ inline float dev_exp<float>(float v) { return expf(v); }
template <typename R> __device__ inline R dev_rsqrt(R v);
template <> __device__ inline double dev_rsqrt<double>(double v) { return 1.0 / sqrt(v); }
template <> __device__ inline float dev_rsqrt<float>(float v) { return rsqrtf(v); }

template <typename R>
__device__ inline void symv(const R *Q, R vx, R vy, R vz, R &ox, R &oy, R &oz) {
    // Q = (xx, xy, xz, yy, yz, zz)
    ox = Q[0] * vx + Q[1] * vy + Q[2] * vz;
    oy = Q[1] * vx + Q[3] * vy + Q[4] * vz;
    oz = Q[2] * vx + Q[4] * vy + Q[5] * vz;
}

template <typename R, int ORD, bool GRAD, bool FIELD>
__device__ inline void pair_terms(R rx, R ry, R rz, R ci, const R *di, const R *Qi, R ck, const R *dk,
                                  const R *Qk, R xi, R xi2, R cex, double &e, R *f, R *g) {
    constexpr int NB = 2 * ORD + 1 + (GRAD ? 1 : 0);
    const R r2 = rx * rx + ry * ry + rz * rz;
    const R rinv = dev_rsqrt<R>(r2);
    const R rinv2 = rinv * rinv;
    const R r = r2 * rinv;
    R B[NB > 2 ? NB : 2];
    B[0] = dev_erfc<R>(xi * r) * rinv;
    {
        const R ex = dev_exp<R>(-xi2 * r2) * cex;
        R pw = 1;
#pragma unroll
        for (int n = 1; n < NB; n++) {
            pw *= 2 * xi2;
            B[n] = ((2 * n - 1) * B[n - 1] + pw * ex) * rinv2;
        }
    }
    R c0 = ci * ck, c1 = 0, c2 = 0, c3 = 0, c4 = 0;
    R dir = 0, dkr = 0, dik = 0;
    R Qir[3] = {0, 0, 0}, Qkr[3] = {0, 0, 0}, qirr = 0, qkrr = 0;
    if (ORD >= 1) {
        dir = di[0] * rx + di[1] * ry + di[2] * rz;
        dkr = dk[0] * rx + dk[1] * ry + dk[2] * rz;
        dik = di[0] * dk[0] + di[1] * dk[1] + di[2] * dk[2];
        c1 = ci * dkr - ck * dir + dik;
        c2 = -dir * dkr;
    }
    if (ORD >= 2) {
        symv(Qi, rx, ry, rz, Qir[0], Qir[1], Qir[2]);
        symv(Qk, rx, ry, rz, Qkr[0], Qkr[1], Qkr[2]);
        qirr = Qir[0] * rx + Qir[1] * ry + Qir[2] * rz;
        qkrr = Qkr[0] * rx + Qkr[1] * ry + Qkr[2] * rz;
        const R diQkr = di[0] * Qkr[0] + di[1] * Qkr[1] + di[2] * Qkr[2];
        const R dkQir = dk[0] * Qir[0] + dk[1] * Qir[1] + dk[2] * Qir[2];
        const R QirQkr = Qir[0] * Qkr[0] + Qir[1] * Qkr[1] + Qir[2] * Qkr[2];
        const R QiQk = Qi[0] * Qk[0] + Qi[3] * Qk[3] + Qi[5] * Qk[5] +
                       2 * (Qi[1] * Qk[1] + Qi[2] * Qk[2] + Qi[4] * Qk[4]);
        c2 += ci * qkrr + ck * qirr + 2 * diQkr - 2 * dkQir + 2 * QiQk;
        c3 = -dir * qkrr + dkr * qirr - 4 * QirQkr;
        c4 = qirr * qkrr;
    }
    R E = c0 * B[0];
    if (ORD >= 1) E += c1 * B[1] + c2 * B[2];
    if (ORD >= 2) E += c3 * B[3] + c4 * B[4];
    e += 0.5 * (double)E;
    if (GRAD) {
        // s = sum_n c_n B_{n+1}
        R s = c0 * B[1];
        if (ORD >= 1) s += c1 * B[2] + c2 * B[3];
        if (ORD >= 2) s += c3 * B[4] + c4 * B[5];
        R gr[3] = {-rx * s, -ry * s, -rz * s};
        if (ORD >= 1) {
#pragma unroll
            for (int a = 0; a < 3; a++) {
                gr[a] += B[1] * (ci * dk[a] - ck * di[a]);
                gr[a] += B[2] * (-dkr * di[a] - dir * dk[a]);
            }
        }
        if (ORD >= 2) {
            R Qkdi[3], Qidk[3], QiQkr[3], QkQir[3];
            symv(Qk, di[0], di[1], di[2], Qkdi[0], Qkdi[1], Qkdi[2]);
            symv(Qi, dk[0], dk[1], dk[2], Qidk[0], Qidk[1], Qidk[2]);
            symv(Qi, Qkr[0], Qkr[1], Qkr[2], QiQkr[0], QiQkr[1], QiQkr[2]);
            symv(Qk, Qir[0], Qir[1], Qir[2], QkQir[0], QkQir[1], QkQir[2]);
#pragma unroll
            for (int a = 0; a < 3; a++) {
                gr[a] += B[2] * (2 * ci * Qkr[a] + 2 * ck * Qir[a] + 2 * Qkdi[a] - 2 * Qidk[a]);
                gr[a] += B[3] * (-qkrr * di[a] - 2 * dir * Qkr[a] + qirr * dk[a] + 2 * dkr * Qir[a] -
                                 4 * (QiQkr[a] + QkQir[a]));
                gr[a] += B[4] * (2 * qkrr * Qir[a] + 2 * qirr * Qkr[a]);
            }
        }
        f[0] -= gr[0];
        f[1] -= gr[1];
        f[2] -= gr[2];
    }
    if (FIELD) {
        const R rv[3] = {rx, ry, rz};
#pragma unroll
        for (int a = 0; a < 3; a++) {
            R v = B[1] * (dk[a] - ck * rv[a]);
            if (ORD >= 1) v -= B[2] * dkr * rv[a];
            if (ORD >= 2) v += B[2] * 2 * Qkr[a] - B[3] * qkrr * rv[a];
            g[a] += v;
        }
    }
}

__device__ inline int morton_leaf(int64_t logical, int depth, int nside) {
    int x = 0, y = 0, z = 0;
    for (int b = 0; b < depth; b++) {
        z |= (int)((logical >> (3 * b)) & 1) << b;
        y |= (int)((logical >> (3 * b + 1)) & 1) << b;
        x |= (int)((logical >> (3 * b + 2)) & 1) << b;
    }
    return (x * nside + y) * nside + z;
}

template <typename R> __device__ inline const R *pick(const double *d, const float *f);
template <> __device__ inline const double *pick<double>(const double *d, const float *) { return d; }
template <> __device__ inline const float *pick<float>(const double *, const float *f) { return f; }

template <typename R, int ORD, bool GRAD, bool FIELD>
__global__ __launch_bounds__(256) void k_p2p(P2PArgs a) {
    __shared__ double sx[CH], sy[CH], sz[CH];
    __shared__ R sq[CH];
    __shared__ R smu[ORD >= 1 ? 3 : 1][CH];
    __shared__ R sth[ORD >= 2 ? 6 : 1][CH];
    __shared__ int sid[CH];
    __shared__ int nb_start[27], nb_pref[28];
    __shared__ double nb_sh[27][3];
    __shared__ double red[7][256];

    const int tid = threadIdx.x;
    const int64_t nleaf = (int64_t)a.nside * a.nside * a.nside;
    // XCD-aware order: consecutive blocks go to different XCDs, so give each
    // XCD a contiguous Morton range of leaves (neighbours share its L2)
    int64_t logical = blockIdx.x;
    if ((nleaf & 7) == 0) logical = (int64_t)(blockIdx.x & 7) * (nleaf >> 3) + (blockIdx.x >> 3);
    const int leaf = morton_leaf(logical, a.depth, a.nside);
    const int ns = a.nside;
    const int tx = leaf / (ns * ns), ty = (leaf / ns) % ns, tz = leaf % ns;
    const int t0 = a.offs[leaf], nt = a.offs[leaf + 1] - t0;
    if (nt == 0) return;

    if (tid < 27) {
        const int dx = tid / 9 - 1, dy = (tid / 3) % 3 - 1, dz = tid % 3 - 1;
        const int sxl = (tx + dx + ns) % ns, syl = (ty + dy + ns) % ns, szl = (tz + dz + ns) % ns;
        const int s = (sxl * ns + syl) * ns + szl;
        nb_start[tid] = a.offs[s];
        nb_pref[tid + 1] = a.offs[s + 1] - a.offs[s];
        nb_sh[tid][0] = dx * a.w;
        nb_sh[tid][1] = dy * a.w;
        nb_sh[tid][2] = dz * a.w;
    }
    __syncthreads();
    if (tid == 0) {
        nb_pref[0] = 0;
        for (int i = 0; i < 27; i++) nb_pref[i + 1] += nb_pref[i];
    }
    __syncthreads();
    const int total = nb_pref[27];

    const R *q = pick<R>(a.q, a.qf), *mu = pick<R>(a.mu, a.muf), *th = pick<R>(a.th, a.thf);
    const int64_t n = a.n;
    const R xi = (R)a.xi, xi2 = (R)(a.xi * a.xi), cex = (R)(1.0 / (a.xi * 1.7724538509055160273));

    for (int tc0 = 0; tc0 < nt; tc0 += 256) {
        const int ntc = min(256, nt - tc0);
        const int nsl = 256 / ntc;
        const int my_t = tid % ntc, my_sl = tid / ntc;
        const bool active = my_sl < nsl;
        const int64_t slot = t0 + tc0 + my_t;
        double xt = 0, yt = 0, zt = 0;
        R ci = 0, di[3] = {0, 0, 0}, Qi[6] = {0, 0, 0, 0, 0, 0};
        if (active) {
            xt = a.x[slot];
            yt = a.y[slot];
            zt = a.z[slot];
            ci = q[slot];
            if (ORD >= 1)
                for (int c = 0; c < 3; c++) di[c] = mu[c * n + slot];
            if (ORD >= 2)
                for (int c = 0; c < 6; c++) Qi[c] = th[c * n + slot];
        }
        double e = 0;
        R f[3] = {0, 0, 0}, g[3] = {0, 0, 0};
        for (int cs = 0; cs < total; cs += CH) {
            const int chn = min(CH, total - cs);
            __syncthreads();
            for (int fidx = tid; fidx < chn; fidx += 256) {
                const int flat = cs + fidx;
                int nb = 0;
                while (flat >= nb_pref[nb + 1]) nb++;
                const int64_t src = nb_start[nb] + (flat - nb_pref[nb]);
                sx[fidx] = a.x[src] + nb_sh[nb][0];
                sy[fidx] = a.y[src] + nb_sh[nb][1];
                sz[fidx] = a.z[src] + nb_sh[nb][2];
                sq[fidx] = q[src];
                if (ORD >= 1)
                    for (int c = 0; c < 3; c++) smu[c][fidx] = mu[c * n + src];
                if (ORD >= 2)
                    for (int c = 0; c < 6; c++) sth[c][fidx] = th[c * n + src];
                sid[fidx] = (nb == 13) ? (int)src : -1;
            }
            __syncthreads();
            if (active) {
                for (int j = my_sl; j < chn; j += nsl) {
                    if (sid[j] == (int)slot) continue;
                    const R rx = (R)(xt - sx[j]), ry = (R)(yt - sy[j]), rz = (R)(zt - sz[j]);
                    R dk[3] = {0, 0, 0}, Qk[6] = {0, 0, 0, 0, 0, 0};
                    if (ORD >= 1)
                        for (int c = 0; c < 3; c++) dk[c] = smu[c][j];
                    if (ORD >= 2)
                        for (int c = 0; c < 6; c++) Qk[c] = sth[c][j];
                    pair_terms<R, ORD, GRAD, FIELD>(rx, ry, rz, ci, di, Qi, sq[j], dk, Qk, xi, xi2, cex, e, f, g);
                }
            }
        }
        // reduce the slices of each target in a fixed order
        __syncthreads();
        red[0][tid] = active ? e : 0.0;
        red[1][tid] = active ? (double)f[0] : 0.0;
        red[2][tid] = active ? (double)f[1] : 0.0;
        red[3][tid] = active ? (double)f[2] : 0.0;
        red[4][tid] = active ? (double)g[0] : 0.0;
        red[5][tid] = active ? (double)g[1] : 0.0;
        red[6][tid] = active ? (double)g[2] : 0.0;
        __syncthreads();
        if (tid < ntc) {
            double v[7] = {0, 0, 0, 0, 0, 0, 0};
            for (int sl = 0; sl < nsl; sl++)
                for (int c = 0; c < 7; c++) v[c] += red[c][sl * ntc + tid];
            const int64_t s = t0 + tc0 + tid;
            a.eatom[s] = v[0];
            if (GRAD) {
                a.F[s] += v[1];
                a.F[n + s] += v[2];
                a.F[2 * n + s] += v[3];
            }
            if (FIELD) {
                a.G[s] += v[4];
                a.G[n + s] += v[5];
                a.G[2 * n + s] += v[6];
            }
        }
    }
}

template <typename R>
hipError_t launch_t(ankh_plan_s *pl, const P2PArgs &a, int ord, bool grad, bool fields) {
    dim3 g((unsigned)pl->nleaf), b(256);
    hipStream_t s = pl->stream;
#define ANKH_P2P(O, GR, FL) hipLaunchKernelGGL((k_p2p<R, O, GR, FL>), g, b, 0, s, a)
    if (ord == 0) {
        if (grad) ANKH_P2P(0, true, false); else ANKH_P2P(0, false, false);
    } else if (ord == 1) {
        if (grad) { if (fields) ANKH_P2P(1, true, true); else ANKH_P2P(1, true, false); }
        else ANKH_P2P(1, false, false);
    } else {
        if (grad) { if (fields) ANKH_P2P(2, true, true); else ANKH_P2P(2, true, false); }
        else ANKH_P2P(2, false, false);
    }
#undef ANKH_P2P
    return hipGetLastError();
}

}  // namespace

hipError_t launch_p2p(ankh_plan_s *pl, int ord, bool grad, bool fields) {
    P2PArgs a;
    a.x = pl->P.x;
    a.y = pl->P.y;
    a.z = pl->P.z;
    a.q = pl->P.q;
    a.mu = pl->P.mu;
    a.th = pl->P.th;
    a.qf = pl->P.qf;
    a.muf = pl->P.muf;
    a.thf = pl->P.thf;
    a.offs = pl->d_offs;
    a.n = pl->n;
    a.nside = pl->nside;
    a.depth = pl->depth;
    a.w = pl->edge / pl->nside;
    a.xi = pl->xi;
    a.eatom = pl->d_eatom;
    a.F = pl->d_F;
    a.G = pl->d_G;
    if (is_mixed(pl)) return launch_t<float>(pl, a, ord, grad, fields);
    return launch_t<double>(pl, a, ord, grad, fields);
}

}  // namespace ankh
