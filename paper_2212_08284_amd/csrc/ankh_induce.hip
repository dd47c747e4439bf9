// Induced dipoles of isotropic point polarisabilities: the polarizable use of
// the method named in the paper's introduction (eq. 1 with the dipoles
// extended by induced ones).  The induced dipoles minimise
//   U(mu_ind) = E(q, mu + mu_ind, Theta) + sum_i |mu_ind_i|^2 / (2 alpha_i).
// E is a quadratic form in the moments, so dE/dmu is affine in the dipoles and
// the minimiser solves (alpha^-1 + H) mu_ind = -dE/dmu(q, mu, Theta), with
// H p = dE/dmu of the dipoles p alone (one evaluation of the path with zero
// charges and no quadrupoles).  With s = alpha^(1/2) per atom and
// mu_ind = s y the system is (I + S H S) y = -S g0: symmetric, and atoms with
// alpha = 0 drop out.  Conjugate gradients from y = 0; the host holds the
// scalars, the device every vector (float64, [n][3] caller order) and every dot
// product (two-stage, fixed order, so a solve is bitwise reproducible).
#include <cmath>

#include "ankh_internal.h"

namespace ankh {
namespace {

constexpr int kDotBlocks = 256;   // first-stage blocks of a dot product (its partials are summed in order)

// vector slots in d_ind, each 3n doubles
enum { V_Y, V_R, V_P, V_V, V_W, V_AP, V_G0, kNumVec };

__device__ __forceinline__ double block_sum(double v, double *red) {
    // 256 threads: a fixed tree in LDS
    red[threadIdx.x] = v;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    return red[0];
}

// s_i = sqrt(alpha_i); a non-finite alpha latches err[0], a negative one err[2] (both then count as 0)
__global__ __launch_bounds__(256) void k_sqrt_alpha(int64_t n, const double *alpha, double *s, int32_t *err) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    double a = alpha[i];
    if (!isfinite(a)) {
        err[0] = 1;
        a = 0.0;
    } else if (a < 0.0) {
        err[2] = 1;
        a = 0.0;
    }
    s[i] = sqrt(a);
}

// b = -s g0;  y = 0;  r = p = b;  v = s p;  partial sums of b.b
__global__ __launch_bounds__(256) void k_cg_init(int64_t m, const double *s, const double *g0, double *y, double *r,
                                                 double *p, double *v, double *part) {
    __shared__ double red[256];
    double acc = 0.0;
    for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < m; j += (int64_t)kDotBlocks * 256) {
        const double sj = s[j / 3];
        const double b = -sj * g0[j];
        y[j] = 0.0;
        r[j] = b;
        p[j] = b;
        v[j] = sj * b;
        acc += b * b;
    }
    acc = block_sum(acc, red);
    if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

// Ap = p + s w (w = H v, v = s p);  partial sums of p.Ap
__global__ __launch_bounds__(256) void k_cg_apply(int64_t m, const double *s, const double *p, const double *w,
                                                  double *Ap, double *part) {
    __shared__ double red[256];
    double acc = 0.0;
    for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < m; j += (int64_t)kDotBlocks * 256) {
        const double a = p[j] + s[j / 3] * w[j];
        Ap[j] = a;
        acc += p[j] * a;
    }
    acc = block_sum(acc, red);
    if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

// y += a p;  r -= a Ap;  partial sums of r.r
__global__ __launch_bounds__(256) void k_cg_update(int64_t m, double a, const double *p, const double *Ap, double *y,
                                                   double *r, double *part) {
    __shared__ double red[256];
    double acc = 0.0;
    for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < m; j += (int64_t)kDotBlocks * 256) {
        y[j] = fma(a, p[j], y[j]);
        const double rj = fma(-a, Ap[j], r[j]);
        r[j] = rj;
        acc += rj * rj;
    }
    acc = block_sum(acc, red);
    if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

// p = r + beta p;  v = s p
__global__ __launch_bounds__(256) void k_cg_direction(int64_t m, double beta, const double *s, const double *r,
                                                      double *p, double *v) {
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= m) return;
    const double pj = fma(beta, p[j], r[j]);
    p[j] = pj;
    v[j] = s[j / 3] * pj;
}

// mu_ind = s y;  mu_tot = mu + mu_ind (mu may be null);  partial sums of y.y
__global__ __launch_bounds__(256) void k_cg_finish(int64_t m, const double *s, const double *y, const double *mu,
                                                   double *mu_ind, double *mu_tot, double *part) {
    __shared__ double red[256];
    double acc = 0.0;
    for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < m; j += (int64_t)kDotBlocks * 256) {
        const double d = s[j / 3] * y[j];
        mu_ind[j] = d;
        mu_tot[j] = (mu ? mu[j] : 0.0) + d;
        acc += y[j] * y[j];
    }
    acc = block_sum(acc, red);
    if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

// second stage: dot = sum of the kDotBlocks partials in a fixed tree
__global__ __launch_bounds__(256) void k_dot_sum(const double *part, double *dot) {
    __shared__ double red[256];
    const double v = block_sum(part[threadIdx.x], red);
    if (threadIdx.x == 0) dot[0] = v;
}

// energy[0] += 0.5 * yy[0]: the polarisation self term sum |mu_ind|^2 / (2 alpha) = |y|^2 / 2
__global__ void k_add_half(double *energy, const double *yy) {
    if (threadIdx.x == 0 && blockIdx.x == 0) energy[0] += 0.5 * yy[0];
}

struct Work {
    double *vec[kNumVec];
    double *s, *qzero, *etmp, *part, *dot;
};

Work layout(ankh_plan_s *pl) {
    const int64_t m = 3 * pl->n;
    Work w{};
    double *b = pl->d_ind;
    for (int k = 0; k < kNumVec; k++) w.vec[k] = b + k * m;
    b += kNumVec * m;
    w.s = b;
    w.qzero = b + pl->n;
    w.etmp = b + 2 * pl->n;
    w.part = w.etmp + 8;
    w.dot = w.part + kDotBlocks;
    return w;
}

size_t work_doubles(int64_t n) { return (size_t)kNumVec * 3 * n + 2 * n + 8 + kDotBlocks + 8; }

}  // namespace
}  // namespace ankh

using namespace ankh;

extern "C" ankh_status ankh_induce(ankh_plan_t pl, const double *pos, const double *q, const double *mu,
                                   const double *theta, const double *alpha, double tol, int32_t max_iter,
                                   double *mu_ind, double *energy, double *forces, int32_t *iterations,
                                   double *rel_residual) {
    if (!pl || !pos || !q || !alpha || !mu_ind) return ANKH_ERR_INVALID_ARG;
    if (pl->max_order < 1 || (pl->max_order < 2 && theta)) return ANKH_ERR_INVALID_ARG;
    if (!(tol > 0.0) || !std::isfinite(tol) || max_iter < 0) return ANKH_ERR_INVALID_ARG;
    hipStream_t st = pl->stream;
    if (!pl->d_ind) {
        void *v = nullptr;
        const size_t bytes = work_doubles(pl->n) * sizeof(double);
        if (pl->bytes_limit && pl->bytes + bytes > pl->bytes_limit) return ANKH_ERR_OUT_OF_MEMORY;
        if (hipMalloc(&v, bytes) != hipSuccess) {
            (void)hipGetLastError();
            return ANKH_ERR_OUT_OF_MEMORY;
        }
        pl->d_ind = static_cast<double *>(v);
        pl->bytes += bytes;
    }
    const Work w = layout(pl);
    const int64_t n = pl->n, m = 3 * n;
    const dim3 b256(256), gn((unsigned)((n + 255) / 256)), gm((unsigned)((m + 255) / 256)), gd(kDotBlocks);
    double *y = w.vec[V_Y], *r = w.vec[V_R], *p = w.vec[V_P], *v = w.vec[V_V], *Hv = w.vec[V_W], *Ap = w.vec[V_AP],
           *g0 = w.vec[V_G0];
    // one dot product: its partials are already in w.part; sum them and read the value back
    auto dot = [&](double &out) -> bool {
        hipLaunchKernelGGL(k_dot_sum, dim3(1), b256, 0, st, w.part, w.dot);
        if (hipMemcpyAsync(&out, w.dot, sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess) return false;
        return hipStreamSynchronize(st) == hipSuccess;
    };
    ankh_status res;
    hipLaunchKernelGGL(k_sqrt_alpha, gn, b256, 0, st, n, alpha, w.s, pl->d_err);
    if (launch_zero_f64(w.qzero, n, st) != hipSuccess) return ANKH_ERR_HIP;
    // right-hand side: the fields of the permanent moments (zero dipoles stand in for none, so that
    // the evaluation computes fields)
    const double *mu0 = mu;
    if (!mu0) {
        if (launch_zero_f64(v, m, st) != hipSuccess) return ANKH_ERR_HIP;
        mu0 = v;
    }
    if ((res = evaluate(pl, pos, q, mu0, theta, w.etmp, nullptr, g0)) != ANKH_OK) return res;
    hipLaunchKernelGGL(k_cg_init, gd, b256, 0, st, m, w.s, g0, y, r, p, v, w.part);
    double bb = 0.0;
    if (hipGetLastError() != hipSuccess || !dot(bb)) return ANKH_ERR_HIP;
    double rr = bb, resid = bb > 0.0 ? 1.0 : 0.0;
    int it = 0;
    bool ok = bb == 0.0;
    if (!std::isfinite(bb)) max_iter = 0;   // a latched input error: report it through ankh_sync
    while (!ok && it < max_iter) {
        // w = H v: the fields of the dipoles v alone (a fields-only evaluation: no force arithmetic)
        if ((res = evaluate(pl, pos, w.qzero, v, nullptr, w.etmp, nullptr, Hv)) != ANKH_OK) return res;
        hipLaunchKernelGGL(k_cg_apply, gd, b256, 0, st, m, w.s, p, Hv, Ap, w.part);
        double pAp = 0.0;
        if (hipGetLastError() != hipSuccess || !dot(pAp)) return ANKH_ERR_HIP;
        it++;
        if (!(pAp > 0.0)) break;   // non-positive curvature: the matrix is not positive definite
        const double a = rr / pAp;
        hipLaunchKernelGGL(k_cg_update, gd, b256, 0, st, m, a, p, Ap, y, r, w.part);
        double rr1 = 0.0;
        if (hipGetLastError() != hipSuccess || !dot(rr1)) return ANKH_ERR_HIP;
        resid = std::sqrt(rr1 / bb);
        if (!std::isfinite(resid)) break;
        if (resid <= tol) {
            ok = true;
            break;
        }
        hipLaunchKernelGGL(k_cg_direction, gm, b256, 0, st, m, rr1 / rr, w.s, r, p, v);
        rr = rr1;
    }
    // mu_ind = s y; the total dipoles go to the v slot
    hipLaunchKernelGGL(k_cg_finish, gd, b256, 0, st, m, w.s, y, mu, mu_ind, v, w.part);
    if (hipGetLastError() != hipSuccess) return ANKH_ERR_HIP;
    if (energy || forces) {
        hipLaunchKernelGGL(k_dot_sum, dim3(1), b256, 0, st, w.part, w.dot);
        double *e = energy ? energy : w.etmp;
        if ((res = evaluate(pl, pos, q, v, theta, e, forces, nullptr)) != ANKH_OK) return res;
        hipLaunchKernelGGL(k_add_half, dim3(1), dim3(64), 0, st, e, w.dot);
        if (hipGetLastError() != hipSuccess) return ANKH_ERR_HIP;
    }
    if (hipStreamSynchronize(st) != hipSuccess) return ANKH_ERR_HIP;
    if (iterations) *iterations = it;
    if (rel_residual) *rel_residual = resid;
    return ok ? ANKH_OK : ANKH_ERR_NOT_CONVERGED;
}
