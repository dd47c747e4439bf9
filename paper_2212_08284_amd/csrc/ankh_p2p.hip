// P2P near field (ANKH-FMM, Alg. 3 step 3): direct pair sums of the
// multipole operator on H = erfc(xi r)/r between every leaf and the 27 leaves
// adjacent to it (periodic, so at depth <= 1 a leaf meets images of itself),
// excluding an atom with itself at zero shift.
//
// Mutual form (the pair symmetry of the mutual-interactions section): each
// unordered pair of adjacent leaves is one task, (s - d, s) for the 13 offsets
// d > 0 (lexicographically), and every pair of atoms in it is evaluated once:
// the target atom (in s - d) takes the energy, its force and its field, the
// source atom (in s) the opposite force and its own field.  The leaf with
// itself is a fourteenth task: up to 64 atoms in mutual form by a round robin
// in lane groups of one wave, more in gather form (all ordered pairs, half
// energy).
//
// One block per source leaf s evaluates its 13 mutual tasks and its own leaf.
// The atoms of the 13 target leaves form one list; lane l of the block owns
// list positions l and l + 256 for the whole block (two targets per lane:
// every source value read from LDS serves both), so a target is loaded once
// and its partial sums stay in registers.  The source atoms of s are staged in
// LDS in chunks of 64 and every lane walks the chunk in the same order (LDS
// broadcasts).  A source's share of one step is summed over the 16 lanes of a
// row with DPP and stored per row; the chunk's 16 row sums are added in row
// order afterwards.  Every atom receives one partial per task it is a target
// of (slots 0..12) and one for its own leaf's block (slot 13: its source
// shares and its own-leaf pairs); k_epilogue adds the 14 slots in order.  The
// near energy is summed per block in float64.  No atomics: results are
// bitwise reproducible.
//
// Pair terms (r = x_i - x_j, D_x = q + mu.d + Th:dd on x (+ Om:ddd, see pair_terms), the mirrored
// operator on the source): with B_0 = H, B_{n+1} = -(1/r) dB_n/dr,
//   E_ij = c0 B0 + c1 B1 + c2 B2 + c3 B3 + c4 B4,
//   c0 = qi qk
//   c1 = qi (dk.r) - qk (di.r) + di.dk
//   c2 = -(di.r)(dk.r) + qi r.Qk.r + qk r.Qi.r + 2 di.Qk.r - 2 dk.Qi.r + 2 Qi:Qk
//   c3 = -(di.r) r.Qk.r + (dk.r) r.Qi.r - 4 (Qi r).(Qk r)
//   c4 = (r.Qi.r)(r.Qk.r)
// grad_r E_ij = sum_n grad(c_n) B_n - r sum_n c_n B_{n+1};  F_i = -grad_r E_ij = -F_j;
// dE/d(di) = B1 (dk - qk r) + B2 (2 Qk r - (dk.r) r) - B3 (r.Qk.r) r,
// dE/d(dk) = B1 (di + qi r) - B2 (2 Qi r + (di.r) r) + B3 (r.Qi.r) r.
// The radial functions follow B_n = [(2n-1) B_{n-1} + (2 xi^2)^n exp(-xi^2 r^2)/(xi sqrt(pi))] / r^2.
#include <cmath>

#include "ankh_internal.h"

namespace ankh {
namespace {

constexpr int CH = 64;      // source atoms per LDS chunk (and targets per round of the own-leaf task)
constexpr int NHALF = 13;   // half-shell neighbour offsets (mutual tasks per leaf)
constexpr int BT = 256;     // threads per block
constexpr int NW = BT / 64; // waves per block
constexpr int NROW = BT / 16;   // 16-lane DPP rows per block
constexpr int TPASS = 2 * BT;   // target list positions per pass (two per lane)
constexpr int kSlotSrc = NHALF; // slot of an atom's own-leaf block
constexpr int G = 16;       // derivative pass: lanes per group (targets per round)
constexpr int NG = 16;      //                  groups per block (source split)
static_assert(kNumSlots == NHALF + 1, "one slot per mutual task of a target and one for its own leaf");

// Per-launch constants of the radial functions: xi; gx, the factor that turns
// r^2 into the argument of gauss(); pwc[n] = (2 xi^2)^n / (xi sqrt(pi)), the
// Gaussian's weight in B_n.
template <typename R> struct Radial {
    R xi, xi2, c_erf, gx, pwc[8];   // c_erf = (2/sqrt(pi)) xi
};

template <typename R> struct P2PArgs {
    const double *x, *y, *z;
    const double *q, *mu, *th, *om;
    const float *qf, *muf, *thf, *omf;
    const int32_t *offs;
    int64_t n;
    int nside, depth;
    double w, xi;
    double *enear;          // [nleaf] near energy per block (source leaf)
    void *slot_f;           // [3][kNumSlots][n] force partials (R)
    void *slot_g;           // [3][kNumSlots][n] field partials (R)
    Radial<R> rad;
};

template <typename R> __device__ inline R dev_erfc(R v);
template <> __device__ inline double dev_erfc<double>(double v) { return erfc(v); }
template <> __device__ inline float dev_erfc<float>(float v) { return erfcf(v); }
// 1/sqrt(v) for v = r^2 of a near pair (never denormal, never zero): the
// hardware reciprocal square root (float32, ~1 ulp), refined in float64 by two
// Newton steps y <- y (3/2 - v y^2 / 2), each squaring the relative error.
template <typename R> __device__ inline R dev_rsqrt(R v);
template <> __device__ inline double dev_rsqrt<double>(double v) {
    double y = __builtin_amdgcn_rsq(v);
    const double hv = 0.5 * v;
    y = y * (1.5 - hv * y * y);
    y = y * (1.5 - hv * y * y);
    return y;
}
template <> __device__ inline float dev_rsqrt<float>(float v) { return __builtin_amdgcn_rsqf(v); }

// sum over the 16 lanes of a DPP row; every lane of the row receives the sum
// (every lane reads a lane of its own row, so bound_ctrl never applies; it lets
// the compiler fold each move into the add as a DPP operand)
__device__ inline float row16_sum(float v) {
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF, true));   // quad [1,0,3,2]
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x4E, 0xF, 0xF, true));   // quad [2,3,0,1]
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x141, 0xF, 0xF, true));  // row half-mirror
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x140, 0xF, 0xF, true));  // row mirror
    return v;
}
__device__ inline double dpp64(double v, int ctrl) {
    const long long b = __double_as_longlong(v);
    int lo = (int)(b & 0xffffffffLL), hi = (int)(b >> 32);
    switch (ctrl) {
        case 0xB1:
            lo = __builtin_amdgcn_mov_dpp(lo, 0xB1, 0xF, 0xF, false);
            hi = __builtin_amdgcn_mov_dpp(hi, 0xB1, 0xF, 0xF, false);
            break;
        case 0x4E:
            lo = __builtin_amdgcn_mov_dpp(lo, 0x4E, 0xF, 0xF, false);
            hi = __builtin_amdgcn_mov_dpp(hi, 0x4E, 0xF, 0xF, false);
            break;
        case 0x141:
            lo = __builtin_amdgcn_mov_dpp(lo, 0x141, 0xF, 0xF, false);
            hi = __builtin_amdgcn_mov_dpp(hi, 0x141, 0xF, 0xF, false);
            break;
        default:
            lo = __builtin_amdgcn_mov_dpp(lo, 0x140, 0xF, 0xF, false);
            hi = __builtin_amdgcn_mov_dpp(hi, 0x140, 0xF, 0xF, false);
            break;
    }
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ inline double row16_sum(double v) {
    v += dpp64(v, 0xB1);
    v += dpp64(v, 0x4E);
    v += dpp64(v, 0x141);
    v += dpp64(v, 0x140);
    return v;
}

// Short-range forms of erfc and exp for x = xi r of every near pair below a
// bound the launcher checks (SL = 1: x <= 1/2, SL = 2: x <= 1/5; the near
// pairs are at most two leaf diagonals apart): erf(x) = (2/sqrt(pi)) x
// sum_n (-x^2)^n / (n! (2n+1)) (Maclaurin series, Abramowitz & Stegun 7.1.5)
// and exp(-u) = sum_n (-u)^n / n!, truncated where the first dropped term is
// below the working precision at the bound: erfc 7 / 4 terms in float32,
// 13 / 8 in float64; exp 14 / 9 terms in float64 (float32 takes the hardware
// exponential).
template <typename R, int SL> struct NearSeries;
template <> struct NearSeries<float, 1> { static constexpr int NE = 7; };
template <> struct NearSeries<float, 2> { static constexpr int NE = 4; };
template <> struct NearSeries<double, 1> { static constexpr int NE = 13, NX = 14; };
template <> struct NearSeries<double, 2> { static constexpr int NE = 8, NX = 9; };
// sum_n (-u)^n / (n! (2n+1)) at u = x^2, so that erfc(x) = 1 - (2/sqrt(pi)) x erf_series(u)
template <typename R, int SL> __device__ inline R erf_series(R u) {
    constexpr double c[13] = {1.0, -1.0 / 3, 1.0 / 10, -1.0 / 42, 1.0 / 216, -1.0 / 1320, 1.0 / 9360, -1.0 / 75600,
                              1.0 / 685440, -1.0 / 6894720, 1.0 / 76204800, -1.0 / 918086400,
                              1.0 / 11975040000.0};
    R s = (R)c[NearSeries<R, SL>::NE - 1];
#pragma unroll
    for (int k = NearSeries<R, SL>::NE - 2; k >= 0; k--) s = s * u + (R)c[k];
    return s;
}
template <typename R, int SL> __device__ inline R exp_near(R u) {   // exp(-u), Horner form with 1/k as constants
    R s = (R)1;
#pragma unroll
    for (int k = NearSeries<R, SL>::NX - 1; k >= 1; k--) s = (R)1 - s * (u * (R)(1.0 / k));
    return s;
}

template <typename R>
__device__ inline void symv(const R *Q, R vx, R vy, R vz, R &ox, R &oy, R &oz) {
    // Q = (xx, xy, xz, yy, yz, zz)
    ox = Q[0] * vx + Q[1] * vy + Q[2] * vz;
    oy = Q[1] * vx + Q[3] * vy + Q[4] * vz;
    oz = Q[2] * vx + Q[4] * vy + Q[5] * vz;
}
// o += Q v
template <typename R> __device__ inline void symv_acc(const R *Q, const R *v, R *o) {
    o[0] += Q[0] * v[0] + Q[1] * v[1] + Q[2] * v[2];
    o[1] += Q[1] * v[0] + Q[3] * v[1] + Q[4] * v[2];
    o[2] += Q[2] * v[0] + Q[4] * v[1] + Q[5] * v[2];
}
// A : B of two symmetric matrices (xx, xy, xz, yy, yz, zz)
template <typename R> __device__ inline R sym_dot(const R *A, const R *B) {
    return A[0] * B[0] + A[3] * B[3] + A[5] * B[5] + 2 * (A[1] * B[1] + A[2] * B[2] + A[4] * B[4]);
}
// Octupoles O = (xxx, xxy, xxz, xyy, xyz, xzz, yyy, yyz, yzz, zzz).  M = O r, the symmetric matrix
// M_ab = O_abc r_c
template <typename R> __device__ inline void oct_r(const R *O, R rx, R ry, R rz, R *M) {
    M[0] = O[0] * rx + O[1] * ry + O[2] * rz;
    M[1] = O[1] * rx + O[3] * ry + O[4] * rz;
    M[2] = O[2] * rx + O[4] * ry + O[5] * rz;
    M[3] = O[3] * rx + O[6] * ry + O[7] * rz;
    M[4] = O[4] * rx + O[7] * ry + O[8] * rz;
    M[5] = O[5] * rx + O[8] * ry + O[9] * rz;
}
// o_c += O_abc M_ab for a symmetric matrix M
template <typename R> __device__ inline void oct_mat_acc(const R *O, const R *M, R *o) {
    o[0] += O[0] * M[0] + O[3] * M[3] + O[5] * M[5] + 2 * (O[1] * M[1] + O[2] * M[2] + O[4] * M[4]);
    o[1] += O[1] * M[0] + O[6] * M[3] + O[8] * M[5] + 2 * (O[3] * M[1] + O[4] * M[2] + O[7] * M[4]);
    o[2] += O[2] * M[0] + O[7] * M[3] + O[9] * M[5] + 2 * (O[4] * M[1] + O[5] * M[2] + O[8] * M[4]);
}
// full contraction of two octupoles: every stored component with its multiplicity
template <typename R> __device__ inline R oct_dot(const R *A, const R *B) {
    return A[0] * B[0] + A[6] * B[6] + A[9] * B[9] +
           3 * (A[1] * B[1] + A[2] * B[2] + A[3] * B[3] + A[5] * B[5] + A[7] * B[7] + A[8] * B[8]) +
           6 * A[4] * B[4];
}

template <typename R, int SL> Radial<R> radial_constants(double xi) {
    Radial<R> c;
    c.xi = (R)xi;
    c.xi2 = (R)(xi * xi);
    c.c_erf = (R)(1.1283791670955125739 * xi);
    // float32 with a short series: exp(-xi^2 r^2) = 2^(gx r^2), gx = -xi^2 log2(e)
    c.gx = (R)(sizeof(R) == 4 && SL > 0 ? -xi * xi * 1.4426950408889634074 : xi * xi);
    double p = 1.0 / (xi * 1.7724538509055160273);
    c.pwc[0] = (R)p;
    for (int k = 1; k < 8; k++) {
        p *= 2.0 * xi * xi;
        c.pwc[k] = (R)p;
    }
    return c;
}
// exp(-xi^2 r^2) from v = gx r^2: the short series, or in float32 the hardware
// base-2 exponential (relative error ~1e-7 here)
template <typename R, int SL> __device__ inline R gauss(R v);
template <> __device__ inline float gauss<float, 0>(float v) { return expf(-v); }
template <> __device__ inline float gauss<float, 1>(float v) { return __builtin_amdgcn_exp2f(v); }
template <> __device__ inline float gauss<float, 2>(float v) { return __builtin_amdgcn_exp2f(v); }
template <> __device__ inline double gauss<double, 0>(double v) { return exp(-v); }
template <> __device__ inline double gauss<double, 1>(double v) { return exp_near<double, 1>(v); }
template <> __device__ inline double gauss<double, 2>(double v) { return exp_near<double, 2>(v); }


// One pair, accumulated in place: ew * E into te, the target force -grad into
// tf and the target field into tg; with SRC (mutual form, ew = 1) also the
// source force +grad into sf and the source field into sg.
// The gradient is grouped by vector (the same algebra as grad(c_n) B_n - r
// sum c_n B_{n+1}):
//   grad_r E = a1 di + a2 dk + a3 Qk r + a4 Qi r + 2 B2 (Qk di - Qi dk)
//              - 4 B3 (Qi Qk r + Qk Qi r) - r sum_n c_n B_{n+1},
//   a1 = -(qk B1 + (dk.r) B2 + (r.Qk.r) B3),   a2 = qi B1 - (di.r) B2 + (r.Qi.r) B3,
//   a3 = 2 (qi B2 - (di.r) B3 + (r.Qi.r) B4),  a4 = 2 (qk B2 + (dk.r) B3 + (r.Qk.r) B4),
// and the fields reuse a1, a2:  dE/d(di) = B1 dk + 2 B2 Qk r + a1 r,
// dE/d(dk) = B1 di - 2 B2 Qi r + a2 r.
// Octupoles (ORD = 3) add to c3 .. c6 the terms of the rank-3 moments (the general rule: for traceless
// moments A of rank a on the target and C of rank b on the source, the pair term is
//   sum_j (-1)^(a-j) C(a,j) C(b,j) j! B_(a+b-j) <A r^(a-j), C r^(b-j)>_j,
// j indices of A contracted with j of C and the rest with r; the quadrupole c_n above are its a, b <= 2
// cases).  With Oi r (matrix), Oi r r (vector) and oi = Oi r r r (scalar), likewise for Ok:
//   c3 += -qk oi + qi ok + 3 (Oi r r.dk + di.Ok r r) + 6 (Qi:Ok r - Oi r:Qk + Oi:Ok)
//   c4 += -oi (dk.r) - (di.r) ok + 6 (Oi r r.Qk r - Qi r.Ok r r) - 18 Oi r:Ok r
//   c5  = -oi (r.Qk.r) + (r.Qi.r) ok + 9 Oi r r.Ok r r,   c6 = -oi ok.
// Their gradient adds -ok B4 to a1, -oi B4 to a2, -2 oi B5 to a3, 2 ok B5 to a4, 6 B4 Oi r r to the
// vector multiplied by Qk, -6 B4 Ok r r to the one multiplied by Qi, and
//   -3 (qk B3 + (dk.r) B4 + (r.Qk.r) B5 + ok B6) Oi r r + 3 (qi B3 - (di.r) B4 + (r.Qi.r) B5 - oi B6) Ok r r
//   + (Oi r)(6 B3 dk + 12 B4 Qk r + 18 B5 Ok r r) + (Ok r)(6 B3 di - 12 B4 Qi r + 18 B5 Oi r r)
//   + Oi:(-6 B3 Qk - 18 B4 Ok r) + Ok:(6 B3 Qi - 18 B4 Oi r),
// with (O:M)_c = O_abc M_ab; the fields add 3 B3 Ok r r (target) and 3 B3 Oi r r (source).
template <typename R, int ORD, bool GRAD, bool FIELD, bool SRC, int SL>
__device__ inline void pair_terms(R rx, R ry, R rz, R ci, const R *di, const R *Qi, const R *Oi, R ck, const R *dk,
                                  const R *Qk, const R *Ok, const Radial<R> &rc, R ew, R &te, R *tf, R *tg, R *sf,
                                  R *sg) {
    constexpr int NB = 2 * ORD + 1 + (GRAD ? 1 : 0);
    const R r2 = rx * rx + ry * ry + rz * rz;
    const R rinv = dev_rsqrt<R>(r2);
    const R rinv2 = rinv * rinv;
    R B[NB > 2 ? NB : 2];
    R ex;
    if constexpr (SL == 0) {
        B[0] = dev_erfc<R>(rc.xi * (r2 * rinv)) * rinv;
        ex = gauss<R, SL>(rc.gx * r2);
    } else {
        // erfc(xi r) / r = 1/r - (2/sqrt(pi)) xi erf_series(xi^2 r^2): the r of the series cancels 1/r
        const R u = rc.xi2 * r2;
        B[0] = rinv - rc.c_erf * erf_series<R, SL>(u);
        ex = sizeof(R) == 8 ? gauss<R, SL>(u) : gauss<R, SL>(rc.gx * r2);
    }
    {
        B[1] = (B[0] + rc.pwc[1] * ex) * rinv2;
#pragma unroll
        for (int n = 2; n < NB; n++) B[n] = ((R)(2 * n - 1) * B[n - 1] + rc.pwc[n] * ex) * rinv2;
    }
    const R rv[3] = {rx, ry, rz};
    R c0 = ci * ck, c1 = 0, c2 = 0, c3 = 0, c4 = 0, c5 = 0, c6 = 0;
    R dir = 0, dkr = 0;
    R Qir[3] = {0, 0, 0}, Qkr[3] = {0, 0, 0}, qirr = 0, qkrr = 0;
    R Oi1[6], Ok1[6], Oi2[3] = {0, 0, 0}, Ok2[3] = {0, 0, 0}, oi3 = 0, ok3 = 0;
    if constexpr (ORD >= 1) {
        dir = di[0] * rx + di[1] * ry + di[2] * rz;
        dkr = dk[0] * rx + dk[1] * ry + dk[2] * rz;
        const R dik = di[0] * dk[0] + di[1] * dk[1] + di[2] * dk[2];
        c1 = ci * dkr - ck * dir + dik;
        c2 = -dir * dkr;
    }
    if constexpr (ORD >= 2) {
        symv(Qi, rx, ry, rz, Qir[0], Qir[1], Qir[2]);
        symv(Qk, rx, ry, rz, Qkr[0], Qkr[1], Qkr[2]);
        qirr = Qir[0] * rx + Qir[1] * ry + Qir[2] * rz;
        qkrr = Qkr[0] * rx + Qkr[1] * ry + Qkr[2] * rz;
        const R diQkr = di[0] * Qkr[0] + di[1] * Qkr[1] + di[2] * Qkr[2];
        const R dkQir = dk[0] * Qir[0] + dk[1] * Qir[1] + dk[2] * Qir[2];
        const R QirQkr = Qir[0] * Qkr[0] + Qir[1] * Qkr[1] + Qir[2] * Qkr[2];
        const R QiQk = Qi[0] * Qk[0] + Qi[3] * Qk[3] + Qi[5] * Qk[5] +
                       2 * (Qi[1] * Qk[1] + Qi[2] * Qk[2] + Qi[4] * Qk[4]);
        c2 += ci * qkrr + ck * qirr + 2 * (diQkr - dkQir + QiQk);
        c3 = -dir * qkrr + dkr * qirr - 4 * QirQkr;
        c4 = qirr * qkrr;
    }
    if constexpr (ORD >= 3) {
        oct_r(Oi, rx, ry, rz, Oi1);
        oct_r(Ok, rx, ry, rz, Ok1);
        symv(Oi1, rx, ry, rz, Oi2[0], Oi2[1], Oi2[2]);
        symv(Ok1, rx, ry, rz, Ok2[0], Ok2[1], Ok2[2]);
        oi3 = Oi2[0] * rx + Oi2[1] * ry + Oi2[2] * rz;
        ok3 = Ok2[0] * rx + Ok2[1] * ry + Ok2[2] * rz;
        const R Oi2dk = Oi2[0] * dk[0] + Oi2[1] * dk[1] + Oi2[2] * dk[2];
        const R diOk2 = di[0] * Ok2[0] + di[1] * Ok2[1] + di[2] * Ok2[2];
        const R Oi2Qkr = Oi2[0] * Qkr[0] + Oi2[1] * Qkr[1] + Oi2[2] * Qkr[2];
        const R QirOk2 = Qir[0] * Ok2[0] + Qir[1] * Ok2[1] + Qir[2] * Ok2[2];
        const R Oi2Ok2 = Oi2[0] * Ok2[0] + Oi2[1] * Ok2[1] + Oi2[2] * Ok2[2];
        c3 += ci * ok3 - ck * oi3 + 3 * (Oi2dk + diOk2) + 6 * (sym_dot(Qi, Ok1) - sym_dot(Oi1, Qk) + oct_dot(Oi, Ok));
        c4 += -oi3 * dkr - dir * ok3 + 6 * (Oi2Qkr - QirOk2) - 18 * sym_dot(Oi1, Ok1);
        c5 = -oi3 * qkrr + qirr * ok3 + 9 * Oi2Ok2;
        c6 = -oi3 * ok3;
    }
    if constexpr (SRC) {
        // ew = 1: the terms go straight into the accumulator
        te += c0 * B[0];
        if constexpr (ORD >= 1) te += c1 * B[1] + c2 * B[2];
        if constexpr (ORD >= 2) te += c3 * B[3] + c4 * B[4];
        if constexpr (ORD >= 3) te += c5 * B[5] + c6 * B[6];
    } else {
        R E = c0 * B[0];
        if constexpr (ORD >= 1) E += c1 * B[1] + c2 * B[2];
        if constexpr (ORD >= 2) E += c3 * B[3] + c4 * B[4];
        if constexpr (ORD >= 3) E += c5 * B[5] + c6 * B[6];
        te += ew * E;
    }
    if constexpr (!GRAD && !FIELD) return;
    // coefficients shared by the force and the fields
    R a1 = 0, a2 = 0;
    if constexpr (ORD >= 1) {
        a1 = -(ck * B[1] + dkr * B[2]);
        a2 = ci * B[1] - dir * B[2];
        if constexpr (ORD >= 2) {
            a1 -= qkrr * B[3];
            a2 += qirr * B[3];
        }
        if constexpr (ORD >= 3) {
            a1 -= ok3 * B[4];
            a2 -= oi3 * B[4];
        }
    }
    if constexpr (GRAD) {
        R sn = c0 * B[1];
        if constexpr (ORD >= 1) sn += c1 * B[2] + c2 * B[3];
        if constexpr (ORD >= 2) sn += c3 * B[4] + c4 * B[5];
        if constexpr (ORD >= 3) sn += c5 * B[6] + c6 * B[7];
        R gr[3];
#pragma unroll
        for (int a = 0; a < 3; a++) gr[a] = -sn * rv[a];
        if constexpr (ORD >= 1) {
#pragma unroll
            for (int a = 0; a < 3; a++) gr[a] += a1 * di[a] + a2 * dk[a];
        }
        if constexpr (ORD >= 2) {
            R a3 = 2 * (ci * B[2] - dir * B[3] + qirr * B[4]);
            R a4 = 2 * (ck * B[2] + dkr * B[3] + qkrr * B[4]);
            if constexpr (ORD >= 3) {
                a3 -= 2 * oi3 * B[5];
                a4 += 2 * ok3 * B[5];
            }
            // b2 (Qk di - Qi dk) + b3 (Qi Qk r + Qk Qi r) = Qk (b2 di + b3 Qi r) + Qi (b3 Qk r - b2 dk):
            // two products with a quadrupole instead of four
            const R b2 = 2 * B[2], b3 = -4 * B[3];
            R w1[3], w2[3];
#pragma unroll
            for (int a = 0; a < 3; a++) {
                gr[a] += a3 * Qkr[a] + a4 * Qir[a];
                w1[a] = b2 * di[a] + b3 * Qir[a];
                w2[a] = b3 * Qkr[a] - b2 * dk[a];
            }
            if constexpr (ORD >= 3) {
                const R b4 = 6 * B[4];
                const R gi = -3 * (ck * B[3] + dkr * B[4] + qkrr * B[5] + ok3 * B[6]);
                const R gk = 3 * (ci * B[3] - dir * B[4] + qirr * B[5] - oi3 * B[6]);
                const R e3 = 6 * B[3], e4 = 12 * B[4], e5 = 18 * B[5], f4 = 18 * B[4];
                R u1[3], u2[3], M1[6], M2[6];
#pragma unroll
                for (int a = 0; a < 3; a++) {
                    w1[a] += b4 * Oi2[a];
                    w2[a] -= b4 * Ok2[a];
                    gr[a] += gi * Oi2[a] + gk * Ok2[a];
                    u1[a] = e3 * dk[a] + e4 * Qkr[a] + e5 * Ok2[a];
                    u2[a] = e3 * di[a] - e4 * Qir[a] + e5 * Oi2[a];
                }
#pragma unroll
                for (int c = 0; c < 6; c++) {
                    M1[c] = -e3 * Qk[c] - f4 * Ok1[c];
                    M2[c] = e3 * Qi[c] - f4 * Oi1[c];
                }
                symv_acc(Oi1, u1, gr);
                symv_acc(Ok1, u2, gr);
                oct_mat_acc(Oi, M1, gr);
                oct_mat_acc(Ok, M2, gr);
            }
            symv_acc(Qk, w1, gr);
            symv_acc(Qi, w2, gr);
        }
#pragma unroll
        for (int a = 0; a < 3; a++) {
            tf[a] -= gr[a];
            if constexpr (SRC) sf[a] += gr[a];
        }
    }
    if constexpr (FIELD) {
        const R b2 = 2 * B[2];
#pragma unroll
        for (int a = 0; a < 3; a++) {
            tg[a] += B[1] * dk[a];
            tg[a] += a1 * rv[a];
            if constexpr (ORD >= 2) tg[a] += b2 * Qkr[a];
            if constexpr (ORD >= 3) tg[a] += 3 * B[3] * Ok2[a];
            if constexpr (SRC) {
                sg[a] += B[1] * di[a];
                sg[a] += a2 * rv[a];
                if constexpr (ORD >= 2) sg[a] -= b2 * Qir[a];
                if constexpr (ORD >= 3) sg[a] += 3 * B[3] * Oi2[a];
            }
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

// task k of a leaf: 0 = itself, 1..13 = the half-shell offsets in lexicographic order
__device__ inline void task_offset(int k, int &dx, int &dy, int &dz) {
    if (k == 0) { dx = dy = dz = 0; return; }
    int c = 0;
    for (int a = -1; a <= 1; a++)
        for (int b = -1; b <= 1; b++)
            for (int e = -1; e <= 1; e++) {
                const bool pos = a > 0 || (a == 0 && (b > 0 || (b == 0 && e > 0)));
                if (!pos) continue;
                if (++c == k) { dx = a; dy = b; dz = e; return; }
            }
}

// One block per source leaf s: the 13 mutual tasks (s - d, s) and the leaf with
// itself.  Lane l owns target list positions l and l + BT of every pass (a pass
// covers TPASS positions; more than one only for crowded half-shells).
template <typename R, int ORD, bool GRAD, bool FIELD, int SL>
__global__ __launch_bounds__(BT) void k_p2p(P2PArgs<R> a) {
    constexpr int NM = 1 + (ORD >= 1 ? 3 : 0) + (ORD >= 2 ? 6 : 0) + (ORD >= 3 ? 10 : 0);   // moment components
    constexpr bool ADJ = GRAD || FIELD;
    __shared__ double sx[CH], sy[CH], sz[CH];
    __shared__ R smo[NM][CH];
    __shared__ R wpart[ADJ ? 6 : 1][NROW][CH];   // source shares per row and chunk atom; own-leaf partials per
                                                 // lane group; gather-form partials per wave
    __shared__ int tfirst[NHALF], tpre[NHALF + 1];   // target leaves: first atom, list prefix
    __shared__ double tshift[NHALF][3];              // their position shift into the source leaf's frame, -d w
    __shared__ double ered[NROW];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int ns = a.nside;
    const int64_t nleaf = (int64_t)ns * ns * ns;
    // XCD-aware order: each XCD receives a contiguous range of source leaves
    int64_t b = blockIdx.x;
    if ((nleaf & 7) == 0) b = (int64_t)(blockIdx.x & 7) * (nleaf >> 3) + (blockIdx.x >> 3);
    // Morton order on an octree level; on any other grid (ANKH-FFT) the lexicographic order
    const int leaf = a.depth >= 0 ? morton_leaf(b, a.depth, ns) : (int)b;
    const int lx = leaf / (ns * ns), ly = (leaf / ns) % ns, lz = leaf % ns;
    if (tid < NHALF) {
        int dx, dy, dz;
        task_offset(1 + tid, dx, dy, dz);
        const int t = (((lx - dx + ns) % ns) * ns + (ly - dy + ns) % ns) * ns + (lz - dz + ns) % ns;
        tfirst[tid] = a.offs[t];
        tpre[tid + 1] = a.offs[t + 1] - a.offs[t];
        tshift[tid][0] = -dx * a.w;
        tshift[tid][1] = -dy * a.w;
        tshift[tid][2] = -dz * a.w;
    }
    __syncthreads();
    if (tid == 0) {
        tpre[0] = 0;
        for (int k = 0; k < NHALF; k++) tpre[k + 1] += tpre[k];
    }
    __syncthreads();
    const int ntg = tpre[NHALF];
    const int s0 = a.offs[leaf], nsrc = a.offs[leaf + 1] - s0;

    const R *q = pick<R>(a.q, a.qf), *mu = pick<R>(a.mu, a.muf), *th = pick<R>(a.th, a.thf);
    const R *om = pick<R>(a.om, a.omf);
    const int64_t n = a.n;
    R *SF = static_cast<R *>(a.slot_f), *SG = static_cast<R *>(a.slot_g);
    const int64_t sstride = (int64_t)kNumSlots * n;     // component stride of the slot arrays
    const Radial<R> rc = a.rad;
    double eacc = 0;   // this lane's near energy

    auto load_chunk = [&](int cs, int chn) {
        for (int f = tid; f < chn; f += BT) {
            const int64_t sj = s0 + cs + f;
            sx[f] = a.x[sj];
            sy[f] = a.y[sj];
            sz[f] = a.z[sj];
            smo[0][f] = q[sj];
            if (ORD >= 1)
                for (int c = 0; c < 3; c++) smo[1 + c][f] = mu[c * n + sj];
            if (ORD >= 2)
                for (int c = 0; c < 6; c++) smo[4 + c][f] = th[c * n + sj];
            if (ORD >= 3)
                for (int c = 0; c < 10; c++) smo[10 + c][f] = om[c * n + sj];
        }
    };
    // one target atom: position (in the source leaf's frame) and moments
    struct Target {
        double x, y, z;
        R c, d[3], Q[6], O[ORD >= 3 ? 10 : 1];
    };
    // list position f of the mutual tasks (valid if f < ntg), or atom s0 + f of the own leaf; an absent
    // target sits far away with zero moments, so its pair terms vanish
    auto load_target = [&](int f, bool mutual, Target &t, int &seg, int64_t &at) {
        const bool iv = f < (mutual ? ntg : nsrc);
        seg = 0;
        at = 0;   // an index every array holds (the loads below may run for absent targets too)
        double shx = 0, shy = 0, shz = 0;
        if (iv) {
            if (mutual) {
                while (seg + 1 < NHALF && f >= tpre[seg + 1]) seg++;
                at = tfirst[seg] + (f - tpre[seg]);
                shx = tshift[seg][0];
                shy = tshift[seg][1];
                shz = tshift[seg][2];
            } else {
                at = s0 + f;
            }
        }
        // every array is read at a 32-bit unsigned offset from a uniform base
        const unsigned u = (unsigned)at;
        t.x = iv ? a.x[u] + shx : 1.0e4;
        t.y = iv ? a.y[u] + shy : 1.0e4;
        t.z = iv ? a.z[u] + shz : 1.0e4;
        t.c = iv ? q[u] : (R)0;
#pragma unroll
        for (int c = 0; c < 3; c++) t.d[c] = (ORD >= 1 && iv) ? (mu + (int64_t)c * n)[u] : (R)0;
#pragma unroll
        for (int c = 0; c < 6; c++) t.Q[c] = (ORD >= 2 && iv) ? (th + (int64_t)c * n)[u] : (R)0;
        if constexpr (ORD >= 3) {
#pragma unroll
            for (int c = 0; c < 10; c++) t.O[c] = iv ? (om + (int64_t)c * n)[u] : (R)0;
        }
    };
    auto slot_ptr = [&](int c, int slot, int64_t at) {
        return (c < 3 ? SF + (int64_t)c * sstride : SG + (int64_t)(c - 3) * sstride) + (int64_t)slot * n + at;
    };
    constexpr int c_lo = GRAD ? 0 : 3, c_hi = FIELD ? 6 : 3;   // the slot components that are written
    // the higher moments of chunk atom j
    auto partner = [&](int j, R *dk, R *Qk, R *Ok) {
        if (ORD >= 1)
            for (int c = 0; c < 3; c++) dk[c] = smo[1 + c][j];
        if (ORD >= 2)
            for (int c = 0; c < 6; c++) Qk[c] = smo[4 + c][j];
        if (ORD >= 3)
            for (int c = 0; c < 10; c++) Ok[c] = smo[10 + c][j];
    };

    // mutual tasks: every pass of target positions against every source chunk
    const int npass = ntg > 0 ? (ntg + TPASS - 1) / TPASS : (nsrc > 0 ? 1 : 0);
    for (int pass = 0; pass < npass; pass++) {
        Target t0, t1;
        int seg0, seg1;
        int64_t at0, at1;
        const int f0 = pass * TPASS + tid, f1 = f0 + BT;
        load_target(f0, true, t0, seg0, at0);
        load_target(f1, true, t1, seg1, at1);
        // wave-uniform: some lane of this wave holds a second target
        const bool two = pass * TPASS + BT + wv * 64 < ntg;
        R tf0[3] = {0, 0, 0}, tg0[3] = {0, 0, 0}, tf1[3] = {0, 0, 0}, tg1[3] = {0, 0, 0};
        for (int cs = 0; cs < nsrc; cs += CH) {
            const int chn = min(CH, nsrc - cs);
            __syncthreads();
            load_chunk(cs, chn);
            __syncthreads();
            R te = 0;
            for (int j = 0; j < chn; j++) {
                const double xs = sx[j], ys = sy[j], zs = sz[j];
                R dk[3] = {0, 0, 0}, Qk[6] = {0, 0, 0, 0, 0, 0}, Ok[ORD >= 3 ? 10 : 1];
                partner(j, dk, Qk, Ok);
                const R ck = smo[0][j];
                R sf[3] = {0, 0, 0}, sg[3] = {0, 0, 0};
                pair_terms<R, ORD, GRAD, FIELD, true, SL>((R)(t0.x - xs), (R)(t0.y - ys), (R)(t0.z - zs), t0.c,
                                                           t0.d, t0.Q, t0.O, ck, dk, Qk, Ok, rc, (R)1, te, tf0, tg0,
                                                           sf, sg);
                if (two)
                    pair_terms<R, ORD, GRAD, FIELD, true, SL>((R)(t1.x - xs), (R)(t1.y - ys), (R)(t1.z - zs),
                                                               t1.c, t1.d, t1.Q, t1.O, ck, dk, Qk, Ok, rc, (R)1, te,
                                                               tf1, tg1, sf, sg);
                if constexpr (ADJ) {
                    // the source's share of this step, summed over each row of 16 lanes
                    R v[6];
#pragma unroll
                    for (int c = c_lo; c < c_hi; c++) v[c] = row16_sum(c < 3 ? sf[c] : sg[c - 3]);
                    if ((lane & 15) == 15) {
#pragma unroll
                        for (int c = c_lo; c < c_hi; c++) wpart[c][tid >> 4][j] = v[c];
                    }
                }
            }
            eacc += (double)te;
            if constexpr (ADJ) {
                __syncthreads();
                // the chunk atoms' source shares: the 16 row sums in row order, by the atom's owner thread
                if (tid < chn) {
                    const int64_t sj = s0 + cs + tid;
#pragma unroll
                    for (int c = c_lo; c < c_hi; c++) {
                        R sum = 0;
#pragma unroll
                        for (int r = 0; r < NROW; r++) sum += wpart[c][r][tid];
                        R *p = slot_ptr(c, kSlotSrc, sj);
                        *p = pass == 0 ? sum : *p + sum;
                    }
                }
            }
        }
        // the targets' partials of this block's tasks
        if constexpr (ADJ) {
            if (f0 < ntg) {
#pragma unroll
                for (int c = c_lo; c < c_hi; c++) *slot_ptr(c, seg0, at0) = c < 3 ? tf0[c] : tg0[c - 3];
            }
            if (f1 < ntg) {
#pragma unroll
                for (int c = c_lo; c < c_hi; c++) *slot_ptr(c, seg1, at1) = c < 3 ? tf1[c] : tg1[c - 3];
            }
        }
    }

    // the leaf with itself.  Up to CH atoms (the chunk still in LDS): the unordered pairs in mutual form,
    // round robin in one wave.  Step k pairs atom i with i + k (mod m), k = 1 .. (m - 1) / 2, and for even m
    // the atoms i < m / 2 with i + m / 2 (each pair once).  The wave holds G = min(64 / m, 8) groups of m
    // lanes (lane g m + i is atom i of group g), and group g takes steps g, g + G, ...: a G-th of the steps
    // per wave instead of all of them on m lanes.  Each group adds its source shares into its own LDS row
    // (the partners of one step are distinct, so no two lanes of an instruction touch one entry; the adds
    // to an entry follow the wave's instruction order), then the groups' target partials and source rows
    // are summed per atom in group order.
    if (nsrc > 0 && nsrc <= CH) {
        const int m = nsrc;
        __syncthreads();   // the mutual phase's readers of wpart are done
        if (wv == 0) {
            const int K = (m - 1) / 2, U = K + ((m & 1) == 0 ? 1 : 0);   // steps
            const int G = max(1, min(min(64 / m, 8), U));
            const int g = lane / m, i = lane - g * m;
            const bool inl = g < G;
            const int ii = inl ? i : 0;
            Target t;
            t.x = sx[ii];
            t.y = sy[ii];
            t.z = sz[ii];
            t.c = smo[0][ii];
#pragma unroll
            for (int c = 0; c < 3; c++) t.d[c] = ORD >= 1 ? smo[1 + c][ii] : (R)0;
#pragma unroll
            for (int c = 0; c < 6; c++) t.Q[c] = ORD >= 2 ? smo[4 + c][ii] : (R)0;
            if constexpr (ORD >= 3) {
#pragma unroll
                for (int c = 0; c < 10; c++) t.O[c] = smo[10 + c][ii];
            }
            R te = 0, tf[3] = {0, 0, 0}, tg[3] = {0, 0, 0};
            if constexpr (ADJ) {
                if (inl) {
#pragma unroll
                    for (int c = c_lo; c < c_hi; c++) wpart[c][g][i] = (R)0;
                }
                __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
                __builtin_amdgcn_wave_barrier();
            }
            for (int u0 = 0; u0 < U; u0 += G) {
                const int u = u0 + g;
                const int k = u < K ? u + 1 : m / 2;
                // lanes without a pair in this step sit it out (masked: the step costs the wave one pair)
                if (inl && u < U && (u < K || i < m / 2)) {
                    int j = i + k;
                    if (j >= m) j -= m;
                    R dk[3] = {0, 0, 0}, Qk[6] = {0, 0, 0, 0, 0, 0}, Ok[ORD >= 3 ? 10 : 1], sf[3] = {0, 0, 0},
                      sg[3] = {0, 0, 0};
                    partner(j, dk, Qk, Ok);
                    pair_terms<R, ORD, GRAD, FIELD, true, SL>((R)(t.x - sx[j]), (R)(t.y - sy[j]), (R)(t.z - sz[j]),
                                                               t.c, t.d, t.Q, t.O, smo[0][j], dk, Qk, Ok, rc, (R)1, te,
                                                               tf, tg, sf, sg);
                    if constexpr (ADJ) {
#pragma unroll
                        for (int c = c_lo; c < c_hi; c++) atomicAdd(&wpart[c][g][j], c < 3 ? sf[c] : sg[c - 3]);
                    }
                }
            }
            eacc += (double)te;
            if constexpr (ADJ) {
                // the groups' target partials into rows G .. 2G - 1, then per atom, by its owner thread (lane
                // i of group 0, which wrote the slot in the mutual phase): the target partials and source
                // rows of the groups in group order
                __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
                __builtin_amdgcn_wave_barrier();
                if (inl) {
#pragma unroll
                    for (int c = c_lo; c < c_hi; c++) wpart[c][G + g][i] = c < 3 ? tf[c] : tg[c - 3];
                }
                __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
                __builtin_amdgcn_wave_barrier();
                if (g == 0) {
                    const int64_t sj = s0 + i;
#pragma unroll
                    for (int c = c_lo; c < c_hi; c++) {
                        R sum = 0;
                        for (int gg = 0; gg < G; gg++) sum += wpart[c][G + gg][i] + wpart[c][gg][i];
                        R *p = slot_ptr(c, kSlotSrc, sj);
                        *p = *p + sum;
                    }
                }
            }
        }
    }
    // more than CH atoms: gather form, CH of them per round as targets (the same in every wave), the
    // sources dealt to the waves; all ordered pairs but an atom with itself, half energy
    for (int tc = 0; nsrc > CH && tc < nsrc; tc += CH) {
        Target t;
        int seg;
        int64_t at;
        const int i = tc + lane;
        load_target(i, false, t, seg, at);
        R te = 0, tf[3] = {0, 0, 0}, tg[3] = {0, 0, 0};
        for (int cs = 0; cs < nsrc; cs += CH) {
            const int chn = min(CH, nsrc - cs);
            __syncthreads();
            load_chunk(cs, chn);
            __syncthreads();
            for (int j = wv; j < chn; j += NW) {
                if (cs + j == i) continue;   // an atom with itself at zero shift
                R dk[3] = {0, 0, 0}, Qk[6] = {0, 0, 0, 0, 0, 0}, Ok[ORD >= 3 ? 10 : 1];
                partner(j, dk, Qk, Ok);
                pair_terms<R, ORD, GRAD, FIELD, false, SL>((R)(t.x - sx[j]), (R)(t.y - sy[j]), (R)(t.z - sz[j]),
                                                            t.c, t.d, t.Q, t.O, smo[0][j], dk, Qk, Ok, rc, (R)0.5, te,
                                                            tf, tg, nullptr, nullptr);
            }
        }
        eacc += (double)te;
        if constexpr (ADJ) {
            __syncthreads();   // the last chunk's readers of wpart are done
#pragma unroll
            for (int c = c_lo; c < c_hi; c++) wpart[c][wv][lane] = c < 3 ? tf[c] : tg[c - 3];
            __syncthreads();
            // the waves' partials in wave order, added to the atom's own-leaf slot by its owner thread
            if (tid < CH && tc + tid < nsrc) {
                const int64_t sj = s0 + tc + tid;
#pragma unroll
                for (int c = c_lo; c < c_hi; c++) {
                    R sum = 0;
#pragma unroll
                    for (int w = 0; w < NW; w++) sum += wpart[c][w][tid];
                    R *p = slot_ptr(c, kSlotSrc, sj);
                    *p = *p + sum;
                }
            }
        }
    }

    // the block's near energy: the lanes' sums, rows by DPP, then the 16 rows in order
    const double er = row16_sum(eacc);
    if ((lane & 15) == 15) ered[tid >> 4] = er;
    __syncthreads();
    if (tid == 0) {
        double e = 0;
        for (int r = 0; r < NROW; r++) e += ered[r];
        a.enear[leaf] = e;
    }
}

// The evaluation's epilogue, per atom in kRedBlocks blocks of contiguous leaf-order ranges:
//  - forces and fields, the far-field part (from L2P) plus the slots, written in caller order
//    (fields with the self-field term of the dipole);
//  - the block's partial sums of the energy terms: self, total charge, and the near and far energies
//    of its share of the leaves (finished by k_reduce2 in block order).
template <typename R> struct EpiArgs {
    int64_t n, nleaf;
    const double *enear;
    const R *SF, *SG;
    const double *F, *G, *eleaf;
    Particles P;
    const int32_t *perm;
    int ord;
    double xi, fself;
    double *forces, *dEdmu, *part;
};

template <typename R, bool GRAD, bool FIELD>
__global__ __launch_bounds__(256) void k_epilogue(EpiArgs<R> a) {
    __shared__ double red[4][256];
    const int b = blockIdx.x, t = threadIdx.x;
    const int64_t n = a.n, st = (int64_t)kNumSlots * n;
    const int64_t a0 = n * b / kRedBlocks, a1 = n * (b + 1) / kRedBlocks;
    const int64_t l0 = a.nleaf * b / kRedBlocks, l1 = a.nleaf * (b + 1) / kRedBlocks;
    const double xi = a.xi;
    const double c0 = -xi / sqrt(3.14159265358979323846), c1 = 2 * xi * xi / 3, c2 = 8 * xi * xi * xi * xi / 5;
    const double c3 = 48 * xi * xi * xi * xi * xi * xi / 7;
    double near = 0, self = 0, qs = 0, far = 0;
    for (int64_t s = a0 + t; s < a1; s += 256) {
        const double q = a.P.q[s];
        qs += q;
        double v = q * q;
        if (a.ord >= 1) {
            const double m0 = a.P.mu[s], m1 = a.P.mu[n + s], m2 = a.P.mu[2 * n + s];
            v += c1 * (m0 * m0 + m1 * m1 + m2 * m2);
        }
        if (a.ord >= 2) {
            const double xx = a.P.th[s], xy = a.P.th[n + s], xz = a.P.th[2 * n + s];
            const double yy = a.P.th[3 * n + s], yz = a.P.th[4 * n + s], zz = a.P.th[5 * n + s];
            v += c2 * (xx * xx + yy * yy + zz * zz + 2 * (xy * xy + xz * xz + yz * yz));
        }
        if (a.ord >= 3) {
            // Omega : Omega, each stored component with its multiplicity
            constexpr double mult[10] = {1, 3, 3, 3, 6, 3, 1, 3, 3, 1};
            double oo = 0;
            for (int c = 0; c < 10; c++) {
                const double o = a.P.om[c * n + s];
                oo += mult[c] * o * o;
            }
            v += c3 * oo;
        }
        self += c0 * v;
        const int64_t i = a.perm[s];
        // every slot of the atom is loaded before the first sum (all loads in flight at once), then the
        // slots are added in slot order
        if (GRAD && a.forces) {
            R vf[3][kNumSlots];
#pragma unroll
            for (int c = 0; c < 3; c++)
#pragma unroll
                for (int k = 0; k < kNumSlots; k++) vf[c][k] = a.SF[c * st + (int64_t)k * n + s];
#pragma unroll
            for (int c = 0; c < 3; c++) {
                double w = 0;
#pragma unroll
                for (int k = 0; k < kNumSlots; k++) w += (double)vf[c][k];
                a.forces[3 * i + c] = a.F[c * n + s] + w;
            }
        }
        if (a.dEdmu) {
            if (FIELD) {
                R vg[3][kNumSlots];
#pragma unroll
                for (int c = 0; c < 3; c++)
#pragma unroll
                    for (int k = 0; k < kNumSlots; k++) vg[c][k] = a.SG[c * st + (int64_t)k * n + s];
#pragma unroll
                for (int c = 0; c < 3; c++) {
                    double w = 0;
#pragma unroll
                    for (int k = 0; k < kNumSlots; k++) w += (double)vg[c][k];
                    a.dEdmu[3 * i + c] = (a.G[c * n + s] + w) + a.fself * a.P.mu[c * n + s];
                }
            } else {
                for (int c = 0; c < 3; c++) a.dEdmu[3 * i + c] = 0.0;
            }
        }
    }
    for (int64_t l = l0 + t; l < l1; l += 256) {
        near += a.enear[l];
        far += a.eleaf[l];
    }
    red[0][t] = near;
    red[1][t] = self;
    red[2][t] = qs;
    red[3][t] = far;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (t < off)
            for (int c = 0; c < 4; c++) red[c][t] += red[c][t + off];
        __syncthreads();
    }
    if (t < 4) a.part[b * 4 + t] = red[t][0];
}

// Near-field derivatives in the target's charge and quadrupole, gather form:
// every atom against the atoms of the 27 leaves around its own (periodic,
// itself at zero shift excluded).  For one pair (r = x_i - x_k):
//   dE/dq_i     += q_k B0 + (d_k.r) B1 + (r.Q_k.r) B2,
//   dE/dTh_i,ab += s r_a r_b - (v_a r_b + r_a v_b) + 2 B2 Q_k,ab,
//   s = q_k B2 + (d_k.r) B3 + (r.Q_k.r) B4,  v = B2 d_k + 2 B3 Q_k r,
// the derivative of the pair terms in c_n with respect to q_i and to the full
// symmetric Th_i (up to its trace, which is dropped at the end).  Block: one
// target leaf; the 16 lanes of a group hold 16 targets, the 16 groups split the
// sources, and the groups' sums are added in group order: no atomics.
// Output: [7][n] in leaf order (dE/dq, then xx, xy, xz, yy, yz, zz).
template <typename R> struct MomArgs {
    const double *x, *y, *z;
    const R *q, *mu, *th;
    const int32_t *offs;
    int64_t n;
    int nside;
    double w;
    Radial<R> rad;
    double *out;
};

template <typename R, int ORD, int SL>
__global__ __launch_bounds__(256) void k_p2p_moments(MomArgs<R> a) {
    constexpr int NB = 3 + ORD;            // B0 .. B_{2+ORD}
    __shared__ double sx[CH], sy[CH], sz[CH];
    __shared__ R smo[10][CH];
    __shared__ double part[7][NG][G];
    const int tid = threadIdx.x, grp = tid / G, ln = tid % G;
    const int ns = a.nside;
    const int leaf = blockIdx.x;
    const int lx = leaf / (ns * ns), ly = (leaf / ns) % ns, lz = leaf % ns;
    const int t0 = a.offs[leaf], nt = a.offs[leaf + 1] - t0;
    const int64_t n = a.n;
    const Radial<R> rc = a.rad;
    for (int tp = 0; tp < nt; tp += G) {
        const bool iv = tp + ln < nt;
        const int ti = t0 + (iv ? tp + ln : 0);
        const double xt = a.x[ti], yt = a.y[ti], zt = a.z[ti];
        // float64 totals; each chunk's few terms are summed in the working precision first
        double phi_t = 0, G_t[6] = {0, 0, 0, 0, 0, 0};
        for (int nb = 0; nb < 27; nb++) {
            const int dx = nb / 9 - 1, dy = (nb / 3) % 3 - 1, dz = nb % 3 - 1;
            const int sl = (((lx + dx + ns) % ns) * ns + (ly + dy + ns) % ns) * ns + (lz + dz + ns) % ns;
            const int s0 = a.offs[sl], nsrc = a.offs[sl + 1] - s0;
            for (int cs = 0; cs < nsrc; cs += CH) {
                const int chn = min(CH, nsrc - cs);
                __syncthreads();
                for (int f = tid; f < chn; f += 256) {
                    const int64_t sj = s0 + cs + f;
                    // the source in the target leaf's frame
                    sx[f] = a.x[sj] + dx * a.w;
                    sy[f] = a.y[sj] + dy * a.w;
                    sz[f] = a.z[sj] + dz * a.w;
                    smo[0][f] = a.q[sj];
                    if (ORD >= 1)
                        for (int c = 0; c < 3; c++) smo[1 + c][f] = a.mu[c * n + sj];
                    if (ORD >= 2)
                        for (int c = 0; c < 6; c++) smo[4 + c][f] = a.th[c * n + sj];
                }
                __syncthreads();
                if (!iv) continue;
                R phi = 0, Gm[6] = {0, 0, 0, 0, 0, 0};
                for (int j = grp; j < chn; j += NG) {
                    if (nb == 13 && s0 + cs + j == ti) continue;   // the atom itself at zero shift
                    const R rx = (R)(xt - sx[j]), ry = (R)(yt - sy[j]), rz = (R)(zt - sz[j]);
                    const R r2 = rx * rx + ry * ry + rz * rz;
                    const R rinv = dev_rsqrt<R>(r2);
                    const R rinv2 = rinv * rinv;
                    R B[NB];
                    R ex;
                    if constexpr (SL == 0) {
                        B[0] = dev_erfc<R>(rc.xi * (r2 * rinv)) * rinv;
                        ex = gauss<R, SL>(rc.gx * r2);
                    } else {
                        const R u = rc.xi2 * r2;
                        B[0] = rinv - rc.c_erf * erf_series<R, SL>(u);
                        ex = sizeof(R) == 8 ? gauss<R, SL>(u) : gauss<R, SL>(rc.gx * r2);
                    }
                    B[1] = (B[0] + rc.pwc[1] * ex) * rinv2;
#pragma unroll
                    for (int k = 2; k < NB; k++) B[k] = ((R)(2 * k - 1) * B[k - 1] + rc.pwc[k] * ex) * rinv2;
                    const R rv[3] = {rx, ry, rz};
                    const R ck = smo[0][j];
                    R dkr = 0, qkrr = 0, Qkr[3] = {0, 0, 0}, dk[3] = {0, 0, 0}, Qk[6] = {0, 0, 0, 0, 0, 0};
                    if (ORD >= 1) {
                        for (int c = 0; c < 3; c++) dk[c] = smo[1 + c][j];
                        dkr = dk[0] * rx + dk[1] * ry + dk[2] * rz;
                    }
                    if (ORD >= 2) {
                        for (int c = 0; c < 6; c++) Qk[c] = smo[4 + c][j];
                        symv(Qk, rx, ry, rz, Qkr[0], Qkr[1], Qkr[2]);
                        qkrr = Qkr[0] * rx + Qkr[1] * ry + Qkr[2] * rz;
                    }
                    phi += ck * B[0];
                    if (ORD >= 1) phi += dkr * B[1];
                    if (ORD >= 2) phi += qkrr * B[2];
                    R sv = ck * B[2];
                    if (ORD >= 1) sv += dkr * B[3];
                    if (ORD >= 2) sv += qkrr * B[4];
                    R v[3] = {0, 0, 0};
                    if constexpr (ORD >= 1) {
#pragma unroll
                        for (int c = 0; c < 3; c++) v[c] = B[2] * dk[c];
                    }
                    if constexpr (ORD >= 2) {
#pragma unroll
                        for (int c = 0; c < 3; c++) v[c] += 2 * B[3] * Qkr[c];
                    }
                    // (xx, xy, xz, yy, yz, zz)
                    constexpr int ia[6] = {0, 0, 0, 1, 1, 2}, ib[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
                    for (int c = 0; c < 6; c++) {
                        const int p = ia[c], q2 = ib[c];
                        Gm[c] += sv * rv[p] * rv[q2] - (v[p] * rv[q2] + rv[p] * v[q2]);
                        if (ORD >= 2) Gm[c] += 2 * B[2] * Qk[c];
                    }
                }
                phi_t += (double)phi;
#pragma unroll
                for (int c = 0; c < 6; c++) G_t[c] += (double)Gm[c];
            }
        }
        __syncthreads();
        part[0][grp][ln] = phi_t;
#pragma unroll
        for (int c = 0; c < 6; c++) part[1 + c][grp][ln] = G_t[c];
        __syncthreads();
        if (tid < 7 * G) {
            const int c = tid / G, l = tid % G;
            if (tp + l < nt) {
                double sum = 0;
                for (int g2 = 0; g2 < NG; g2++) sum += part[c][g2][l];
                a.out[(int64_t)c * n + t0 + tp + l] = sum;
            }
        }
    }
}

template <typename R, int SL>
hipError_t launch_moments_t(ankh_plan_s *pl, int ord, double *out) {
    MomArgs<R> a;
    a.x = pl->P.x;
    a.y = pl->P.y;
    a.z = pl->P.z;
    // the working-precision copies of the moments (float32 in the mixed modes)
    auto sel = [](const double *d, const float *f) {
        if constexpr (sizeof(R) == 8) return reinterpret_cast<const R *>(d);
        else return reinterpret_cast<const R *>(f);
    };
    a.q = sel(pl->P.q, pl->P.qf);
    a.mu = sel(pl->P.mu, pl->P.muf);
    a.th = sel(pl->P.th, pl->P.thf);
    a.offs = pl->d_offs;
    a.n = pl->n;
    a.nside = pl->nside;
    a.w = pl->edge / pl->nside;
    a.rad = radial_constants<R, SL>(pl->xi);
    a.out = out;
    const dim3 g((unsigned)pl->nleaf), b(256);
    if (ord == 0) hipLaunchKernelGGL((k_p2p_moments<R, 0, SL>), g, b, 0, pl->stream, a);
    else if (ord == 1) hipLaunchKernelGGL((k_p2p_moments<R, 1, SL>), g, b, 0, pl->stream, a);
    else hipLaunchKernelGGL((k_p2p_moments<R, 2, SL>), g, b, 0, pl->stream, a);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_moments_prec(ankh_plan_s *pl, int ord, double *out) {
    const double xmax = pl->xi * 2.0 * std::sqrt(3.0) * (pl->edge / pl->nside);
    if (xmax <= 0.2) return launch_moments_t<R, 2>(pl, ord, out);
    if (xmax <= 0.5) return launch_moments_t<R, 1>(pl, ord, out);
    return launch_moments_t<R, 0>(pl, ord, out);
}

template <typename R, int SL>
hipError_t launch_t(ankh_plan_s *pl, P2PArgs<R> a, int ord, bool grad, bool fields) {
    a.rad = radial_constants<R, SL>(pl->xi);
    dim3 g((unsigned)pl->nleaf), b(BT);
    hipStream_t s = pl->stream;
#define ANKH_P2P(O, GR, FL) hipLaunchKernelGGL((k_p2p<R, O, GR, FL, SL>), g, b, 0, s, a)
    if (ord == 0) {
        if (grad) ANKH_P2P(0, true, false); else ANKH_P2P(0, false, false);
    } else if (ord == 1) {
        if (grad) { if (fields) ANKH_P2P(1, true, true); else ANKH_P2P(1, true, false); }
        else if (fields) ANKH_P2P(1, false, true);
        else ANKH_P2P(1, false, false);
    } else if (ord == 2) {
        if (grad) { if (fields) ANKH_P2P(2, true, true); else ANKH_P2P(2, true, false); }
        else if (fields) ANKH_P2P(2, false, true);
        else ANKH_P2P(2, false, false);
    } else {
        // octupoles: a fields-only evaluation also writes the force partials (three variants, not four)
        if (fields) ANKH_P2P(3, true, true);
        else if (grad) ANKH_P2P(3, true, false);
        else ANKH_P2P(3, false, false);
    }
#undef ANKH_P2P
    return hipGetLastError();
}

template <typename R>
hipError_t launch_epi_t(ankh_plan_s *pl, int ord, bool grad, bool fields, double *forces, double *dEdmu) {
    EpiArgs<R> a;
    a.n = pl->n;
    a.nleaf = pl->nleaf;
    a.enear = pl->d_enear;
    a.SF = static_cast<const R *>(pl->d_slot_f);
    a.SG = static_cast<const R *>(pl->d_slot_g);
    a.F = pl->d_F;
    a.G = pl->d_G;
    a.eleaf = pl->d_eleaf;
    a.P = pl->P;
    a.perm = pl->d_perm;
    a.ord = ord;
    a.xi = pl->xi;
    a.fself = -4.0 * pl->xi * pl->xi * pl->xi / (3.0 * std::sqrt(3.14159265358979323846));
    a.forces = grad ? forces : nullptr;
    a.dEdmu = dEdmu;
    a.part = pl->d_part;
    const dim3 g(kRedBlocks), b(256);
    hipStream_t s = pl->stream;
    if (grad && fields) hipLaunchKernelGGL((k_epilogue<R, true, true>), g, b, 0, s, a);
    else if (grad) hipLaunchKernelGGL((k_epilogue<R, true, false>), g, b, 0, s, a);
    else if (fields) hipLaunchKernelGGL((k_epilogue<R, false, true>), g, b, 0, s, a);
    else hipLaunchKernelGGL((k_epilogue<R, false, false>), g, b, 0, s, a);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_prec(ankh_plan_s *pl, int ord, bool grad, bool fields) {
    P2PArgs<R> a;
    a.x = pl->P.x;
    a.y = pl->P.y;
    a.z = pl->P.z;
    a.q = pl->P.q;
    a.mu = pl->P.mu;
    a.th = pl->P.th;
    a.qf = pl->P.qf;
    a.muf = pl->P.muf;
    a.thf = pl->P.thf;
    a.om = pl->P.om;
    a.omf = pl->P.omf;
    a.offs = pl->d_offs;
    a.n = pl->n;
    a.nside = pl->nside;
    a.depth = pl->fft_dft ? -1 : pl->depth;
    a.w = pl->edge / pl->nside;
    a.xi = pl->xi;
    a.enear = pl->d_enear;
    a.slot_f = pl->d_slot_f;
    a.slot_g = pl->d_slot_g;
    // largest xi r of a near pair: opposite corners of diagonally adjacent leaves
    const double xmax = pl->xi * 2.0 * std::sqrt(3.0) * a.w;
    if (xmax <= 0.2) return launch_t<R, 2>(pl, a, ord, grad, fields);
    if (xmax <= 0.5) return launch_t<R, 1>(pl, a, ord, grad, fields);
    return launch_t<R, 0>(pl, a, ord, grad, fields);
}

}  // namespace

hipError_t launch_p2p(ankh_plan_s *pl, int ord, bool grad, bool fields) {
    return is_mixed(pl) ? launch_prec<float>(pl, ord, grad, fields) : launch_prec<double>(pl, ord, grad, fields);
}

// near-field dE/dq and dE/dTheta per leaf-order atom into out [7][n]
hipError_t launch_p2p_moments(ankh_plan_s *pl, int ord, double *out) {
    return is_mixed(pl) ? launch_moments_prec<float>(pl, ord, out) : launch_moments_prec<double>(pl, ord, out);
}

// the slot sums, forces and fields in caller order, the energy partials
hipError_t launch_epilogue(ankh_plan_s *pl, int ord, bool grad, bool fields, double *forces, double *dEdmu) {
    return is_mixed(pl) ? launch_epi_t<float>(pl, ord, grad, fields, forces, dEdmu)
                        : launch_epi_t<double>(pl, ord, grad, fields, forces, dEdmu);
}

}  // namespace ankh
