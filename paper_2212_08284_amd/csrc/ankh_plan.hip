// C ABI of the interpolated-Ewald library: planner (parameter rules, operator
// tables, device buffers) and the evaluation driver that enqueues the
// kernels of one energy / energy+forces evaluation on the plan's stream.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "ankh_internal.h"

using namespace ankh;

// Scratch of ankh_energy_derivs_noalloc: the near-field charge and quadrupole derivatives [7][n] of up to
// kNoAllocMaxAtoms atoms.  Every GPU the library runs on holds one copy until the process ends.  In host
// code `scratch` only names the symbol: its device address comes from hipGetSymbolAddress, once per
// device (noalloc_scratch below), and only that address is handed to kernels.
constexpr int64_t kNoAllocMaxAtoms = (int64_t)1 << 19;
static __device__ __align__(256) double scratch[7 * kNoAllocMaxAtoms];

namespace {

constexpr double kPi = 3.14159265358979323846;

struct HipFail {
    hipError_t e;
};

inline void ck(hipError_t e) {
    if (e != hipSuccess) throw HipFail{e};
}

template <typename T>
void dalloc(ankh_plan_s *pl, T **p, size_t count) {
    if (count == 0) count = 1;
    if (pl->bytes_limit && pl->bytes + count * sizeof(T) > pl->bytes_limit) throw std::bad_alloc();
    void *v = nullptr;
    hipError_t e = hipMalloc(&v, count * sizeof(T));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        throw std::bad_alloc();
    }
    *p = static_cast<T *>(v);
    pl->bytes += count * sizeof(T);
}

// plan-time device scratch (not counted in the plan's bytes): released explicitly, or when a failure
// unwinds the plan's construction
struct Scratch {
    double *p = nullptr;
    void alloc(size_t count) {
        if (hipMalloc((void **)&p, count * sizeof(double)) != hipSuccess) {
            p = nullptr;
            (void)hipGetLastError();
            throw std::bad_alloc();
        }
    }
    void release() {
        if (!p) return;
        const hipError_t e = hipFree(p);
        p = nullptr;
        ck(e);
    }
    ~Scratch() {
        if (p) (void)hipFree(p);
    }
};

void free_all(ankh_plan_s *pl) {
    void *ptrs[] = {pl->d_tab, pl->d_leaf, pl->d_count, pl->d_offs, pl->d_rank, pl->d_perm, pl->d_tmp,
                    pl->P.x, pl->P.y, pl->P.z, pl->P.q, pl->P.mu, pl->P.th, pl->P.qf, pl->P.muf, pl->P.thf,
                    pl->P.om, pl->P.omf,
                    pl->d_M, pl->d_L, pl->d_K, pl->d_Kf, pl->d_Cper, pl->d_eleaf, pl->d_F,
                    pl->d_G, pl->d_terms, pl->d_part, pl->d_err, pl->d_tab0, pl->d_Mf, pl->d_m2l_part,
                    pl->root_owned ? pl->d_rootM : nullptr, pl->root_owned ? pl->d_rootL : nullptr,
                    pl->d_Kb, pl->d_Mb, pl->d_enear, pl->d_slot_f, pl->d_slot_g, pl->d_cper_part,
                    pl->d_U, pl->d_Mc, pl->d_Lc, pl->d_ind, pl->d_mom, pl->d_fftB, pl->d_fftW, pl->d_fftX,
                    pl->d_fftD, pl->d_fftTw, pl->d_fftX32, pl->d_fftB32, pl->d_fftTw32, pl->d_fftD32};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    for (auto &set : pl->evsets)
        for (auto &e : set) (void)hipEventDestroy(e);
    pl->evsets.clear();
    if (pl->ev_fork) (void)hipEventDestroy(pl->ev_fork);
    if (pl->ev_join) (void)hipEventDestroy(pl->ev_join);
    if (pl->side) (void)hipStreamDestroy(pl->side);
    pl->ev_fork = pl->ev_join = nullptr;
    pl->side = nullptr;
}

// Chebyshev order from the accuracy target: the interpolation error decays
// geometrically in L (numerical-results section); the table is calibrated
// against the classical-Ewald oracle on the synthetic water and ionic boxes.
int order_for(double eps) {
    if (eps >= 1e-4) return 4;
    if (eps >= 1e-5) return 5;
    if (eps >= 1e-6) return 6;
    if (eps >= 1e-7) return 7;
    if (eps >= 1e-8) return 8;
    if (eps >= 1e-9) return 9;
    return 10;
}

// Depth: leaves whose mean occupancy balances the per-leaf far-field work
// (189 M2L products of n_u x n_u) against the near-field pair work.
int depth_for(int64_t n, int nu) {
    const double occ = std::max(16.0, 0.3 * nu);
    double e = std::log(std::max(1.0, (double)n / occ)) / std::log(8.0);
    int E = (int)std::floor(e + 0.5);
    return std::min(std::max(E, 0), kMaxDepth);
}

// ANKH-FFT leaves per axis: no octree levels above the leaves, so any grid with fast cell transforms
// (powers of two up to 64; 12, 20, 24) is a candidate.  The far field costs little against the pair
// kernel, so the grid targets far fewer atoms per leaf than the octree rule: 0.1 n_u (22 at order 6)
// from 100,000 atoms, 0.17 n_u below.  On the 288,000-atom water box 24^3 leaves (21 atoms each) take
// 0.99 ms per mixed evaluation and 1.72 ms in FP64, against 1.15 / 1.91 ms on 20^3 and 1.73 / 2.86 ms
// on 16^3, at a relative energy error of 1.8e-7.  Small boxes gain little time from small leaves and
// lose accuracy (the far field carries more of the energy): a 600-atom water box at 1e-6 has a
// relative energy error of 5.9e-6 on 4^3 leaves against 6e-7 on 2^3.
int leaves_for(int64_t n, int nu) {
    static const int cand[] = {1, 2, 4, 8, 12, 16, 20, 24, 32, 64};
    const double occ = std::max(12.0, (n >= 100000 ? 0.1 : 0.17) * nu);
    const double target = std::cbrt(std::max(1.0, (double)n / occ));
    int best = 1;
    double bd = 1e300;
    for (int c : cand) {
        const double d = std::fabs(std::log(c / target));
        if (d < bd) {
            bd = d;
            best = c;
        }
    }
    return best;
}

void build_tables(ankh_plan_s *pl) {
    const int L = pl->order;
    for (int k = 0; k < L; k++) pl->nodes[k] = std::cos((2 * k + 1) * kPi / (2 * L));
    // H[k][m] = (1/L)(1 if m = 0 else 2 T_m(r_k))
    for (int k = 0; k < L; k++) {
        double t0 = 1, t1 = pl->nodes[k];
        for (int m = 0; m < L; m++) {
            double tm = m == 0 ? 1.0 : (m == 1 ? pl->nodes[k] : 0.0);
            if (m >= 2) {
                tm = 2 * pl->nodes[k] * t1 - t0;
                t0 = t1;
                t1 = tm;
            }
            pl->Hm[k * L + m] = (m == 0 ? 1.0 : 2.0 * tm) / L;
        }
    }
    // V[b][a][i] = S_a((r_i -+ 1) / 2): child node i of the low (b = 0) or high (b = 1) child
    for (int b = 0; b < 2; b++)
        for (int i = 0; i < L; i++) {
            const double x = (pl->nodes[i] + (b ? 1.0 : -1.0)) / 2;
            double T[kMaxOrder];
            T[0] = 1;
            if (L > 1) T[1] = x;
            for (int m = 2; m < L; m++) T[m] = 2 * x * T[m - 1] - T[m - 2];
            for (int a = 0; a < L; a++) {
                double s = 0;
                for (int m = 0; m < L; m++) s += pl->Hm[a * L + m] * T[m];
                pl->V[b][a * L + i] = s;
            }
        }
}

// in timing mode 2 only the far-field contraction (stage 4) and the pair kernel (stage 8) are bracketed
// by events: every event record idles the device for a few microseconds
bool stage_recorded(int mode, int stage) { return mode == 1 || (mode == 2 && (stage == 4 || stage == 8)); }

ankh_status run(ankh_plan_s *pl, const double *pos, const double *q, const double *mu, const double *th,
                double *energy, double *forces, double *dEdmu, const double *om = nullptr) {
    // forces and / or fields (dE/dmu); a null forces pointer with fields asked for is the fields-only
    // evaluation of the induced-dipole iteration (the pair kernel then skips the force arithmetic)
    const bool grad = forces != nullptr;
    const int ord = om ? 3 : (th ? 2 : (mu ? 1 : 0));
    const bool fields = dEdmu && ord >= 1;
    const bool adj = grad || fields;
    hipStream_t s = pl->stream;
    hipEvent_t *ev = nullptr;
    if (pl->timing) {
        if ((size_t)pl->n_timed == pl->evsets.size()) {
            std::array<hipEvent_t, kNumStages + 1> set{};
            for (auto &e : set)
                if (hipEventCreate(&e) != hipSuccess) return ANKH_ERR_HIP;
            pl->evsets.push_back(set);
        }
        ev = pl->evsets[pl->n_timed].data();
    }
    auto mark = [&](int i) {
        if (ev && (pl->timing == 1 || stage_recorded(pl->timing, i) || stage_recorded(pl->timing, i - 1)))
            ck(hipEventRecord(ev[i], pl->stream));
    };
    // The far-field chain (stages 2-7) runs on the side stream while the pair kernel runs on the
    // plan's stream: the pair kernel fills every CU with VALU work, and the far-field kernels, mostly
    // waiting on memory and small grids, fit into the gaps.  Timing mode 1 keeps one stream, so its
    // per-stage figures add up.
    const bool overlap = pl->overlap && pl->timing != 1;
    try {
        mark(0);
        ck(launch_sort(pl, pos, q, mu, th));
        mark(1);
        ck(launch_gather(pl, pos, q, mu, th, om));
        mark(2);
        if (overlap) {
            ck(hipEventRecord(pl->ev_fork, s));
            ck(hipStreamWaitEvent(pl->side, pl->ev_fork, 0));
            pl->stream = pl->side;
        }
        ck(launch_p2m(pl, ord));
        mark(3);
        if (pl->far_field == ANKH_FAR_FFT) {
            // ANKH-FFT: node transforms, cell transforms with the spectrum, inverse node
            // transforms into the leaf local expansions (far images included in the spectrum)
            ck(launch_fft_forward(pl));
            mark(4);
            ck(launch_fft_cells(pl));
            mark(5);
            mark(6);
            ck(launch_fft_inverse(pl));
        } else {
            for (int e = pl->depth - 1; e >= 0; e--) ck(launch_m2m(pl, e));
            mark(4);
            ck(launch_m2l_prepare(pl));
            ck(launch_m2l_project(pl));
            for (int e = 1; e <= pl->depth; e++) ck(launch_m2l(pl, e));
            ck(launch_m2l_finish(pl));
            ck(launch_m2l_expand(pl));
            mark(5);
            ck(launch_cper(pl));
            mark(6);
            for (int e = 1; e <= pl->depth; e++) ck(launch_l2l(pl, e));
        }
        if (!(pl->far_field == ANKH_FAR_FFT && fft_inverse_leaf_energies(pl))) ck(launch_leafdot(pl));
        mark(7);
        if (adj) ck(launch_l2p(pl, ord, fields));
        if (overlap) {
            ck(hipEventRecord(pl->ev_join, pl->side));
            pl->stream = s;
        }
        mark(8);
        ck(launch_p2p(pl, ord, grad, fields));
        mark(9);
        if (overlap) ck(hipStreamWaitEvent(s, pl->ev_join, 0));
        ck(launch_epilogue(pl, ord, grad, fields, forces, dEdmu));
        mark(10);
        ck(launch_reduce(pl, energy));
        mark(11);
    } catch (const HipFail &) {
        pl->stream = s;
        return ANKH_ERR_HIP;
    }
    pl->last_kind = grad ? 2 : 1;
    pl->last_order = ord;
    if (ev) pl->n_timed++;
    return ANKH_OK;
}

// device address of `scratch` on device dev, looked up with that device current on the first call for it
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch[kMaxDevices] = {};

ankh_status noalloc_scratch(int dev, double **out) {
    if (dev < 0 || dev >= kMaxDevices) return ANKH_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        int cur = 0;
        if (hipGetDevice(&cur) != hipSuccess) return ANKH_ERR_HIP;
        if (cur != dev && hipSetDevice(dev) != hipSuccess) return ANKH_ERR_HIP;
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (cur != dev && hipSetDevice(cur) != hipSuccess) return ANKH_ERR_HIP;
        if (e != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return ANKH_ERR_HIP;
        }
        g_scratch[dev] = static_cast<double *>(ptr);
    }
    *out = g_scratch[dev];
    return ANKH_OK;
}

ankh_status check_inputs(ankh_plan_s *pl, const double *pos, const double *q, const double *mu, const double *th) {
    if (!pl || !pos || !q) return ANKH_ERR_INVALID_ARG;
    if (pl->max_order < 1 && mu) return ANKH_ERR_INVALID_ARG;
    if (pl->max_order < 2 && th) return ANKH_ERR_INVALID_ARG;
    return ANKH_OK;
}

}  // namespace

ankh_status ankh::evaluate(ankh_plan_s *pl, const double *pos, const double *q, const double *mu, const double *th,
                           double *energy, double *forces, double *dEdmu) {
    return run(pl, pos, q, mu, th, energy, forces, dEdmu);
}

extern "C" {

const char *ankh_status_string(ankh_status st) {
    switch (st) {
        case ANKH_OK: return "ok";
        case ANKH_ERR_INVALID_ARG: return "invalid argument";
        case ANKH_ERR_NONFINITE_INPUT: return "non-finite input";
        case ANKH_ERR_THETA_NOT_TRACELESS: return "quadrupole or octupole not traceless";
        case ANKH_ERR_LEAF_OVERFLOW: return "leaf overflow";
        case ANKH_ERR_ACCURACY_UNREACHABLE: return "accuracy unreachable in this precision";
        case ANKH_ERR_OUT_OF_MEMORY: return "out of device memory";
        case ANKH_ERR_HIP: return "HIP runtime error";
        case ANKH_ERR_NOT_CONVERGED: return "induced dipoles not converged";
    }
    return "unknown status";
}

ankh_status ankh_plan(ankh_plan_t *out, int64_t n_atoms, double box_radius, double rel_accuracy, int32_t max_order,
                      int32_t precision, const ankh_overrides *ov, void *hip_stream) {
    if (!out) return ANKH_ERR_INVALID_ARG;
    if (n_atoms < 1 || n_atoms > (int64_t)0x7fffffff) return ANKH_ERR_INVALID_ARG;
    if (!(box_radius > 0) || !std::isfinite(box_radius)) return ANKH_ERR_INVALID_ARG;
    if (!(rel_accuracy >= 1e-12 && rel_accuracy <= 1e-2)) return ANKH_ERR_INVALID_ARG;
    if (max_order < 0 || max_order > 3) return ANKH_ERR_INVALID_ARG;
    if (precision != ANKH_FP64 && precision != ANKH_MIXED && precision != ANKH_MIXED_BF16X3) return ANKH_ERR_INVALID_ARG;
    if (precision != ANKH_FP64 && rel_accuracy < 1e-7) return ANKH_ERR_ACCURACY_UNREACHABLE;
    if (ov) {
        if (ov->depth > kMaxDepth) return ANKH_ERR_INVALID_ARG;
        if (ov->order > 0 && (ov->order < 2 || ov->order > kMaxOrder)) return ANKH_ERR_INVALID_ARG;
        if (ov->root_order > 0 && (ov->root_order < 2 || ov->root_order > kMaxRootOrder)) return ANKH_ERR_INVALID_ARG;
        if (ov->images > 64) return ANKH_ERR_INVALID_ARG;
        if (!std::isfinite(ov->xi)) return ANKH_ERR_INVALID_ARG;
        if (!std::isfinite(ov->m2l_tol) || ov->m2l_tol >= 1) return ANKH_ERR_INVALID_ARG;
        if (ov->far_field < 0 || ov->far_field > ANKH_FAR_FFT) return ANKH_ERR_INVALID_ARG;
        if (ov->eq_order != 0 && (ov->eq_order < 2 || ov->eq_order > kMaxOrder)) return ANKH_ERR_INVALID_ARG;
        if (ov->overlap < 0 || ov->overlap > 2) return ANKH_ERR_INVALID_ARG;
        if (ov->fft_split < 0 || ov->fft_split > 1) return ANKH_ERR_INVALID_ARG;
        if (ov->leaves < 0 || ov->leaves > 64) return ANKH_ERR_INVALID_ARG;
        if (ov->leaves > 0 && ov->far_field != ANKH_FAR_FFT) return ANKH_ERR_INVALID_ARG;
        if (!(ov->force_accuracy == 0 || (ov->force_accuracy >= 1e-12 && ov->force_accuracy <= 1e-2)))
            return ANKH_ERR_INVALID_ARG;
        if (ov->workspace_limit < 0) return ANKH_ERR_INVALID_ARG;
    }
    // the accuracy the parameters are chosen for: the energy target, or a force target over the largest
    // measured ratio of the relative RMS force error to the relative energy error (unscreened ions)
    const double eps_plan = (ov && ov->force_accuracy > 0) ? std::min(rel_accuracy, ov->force_accuracy / 30.0)
                                                          : rel_accuracy;
    if (precision != ANKH_FP64 && eps_plan < 1e-7) return ANKH_ERR_ACCURACY_UNREACHABLE;
    auto t0 = std::chrono::steady_clock::now();
    ankh_plan_s *pl = new (std::nothrow) ankh_plan_s();
    if (!pl) return ANKH_ERR_OUT_OF_MEMORY;
    pl->n = n_atoms;
    pl->rB = box_radius;
    pl->edge = 2 * box_radius;
    pl->eps = rel_accuracy;
    pl->max_order = max_order;
    pl->precision = precision;
    pl->stream = static_cast<hipStream_t>(hip_stream);
    if (hipGetDevice(&pl->device) != hipSuccess) {
        // no usable device: the first allocation below reports it
        (void)hipGetLastError();
        pl->device = 0;
    }
    {
        int ncu = 0;
        if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, pl->device) == hipSuccess && ncu > 0)
            pl->num_cu = ncu;
        else
            (void)hipGetLastError();
    }
    pl->bytes_limit = ov ? (size_t)ov->workspace_limit : 0;

    // splitting parameter: the largest reciprocal weight exp(-(pi/(xi edge))^2)
    // equals eps/10, so the dropped reciprocal term stays below the target
    const double s2 = std::log(10.0 / eps_plan);
    pl->xi = (ov && ov->xi > 0) ? ov->xi : kPi / (pl->edge * std::sqrt(s2));
    // image radius: pairs beyond the cube Z_p are >= p * edge apart, where erfc(xi p edge) <~ eps/10
    {
        const double sr = std::sqrt(s2);
        int p = (int)std::ceil(sr / (pl->xi * pl->edge)) + 1;
        pl->images = (ov && ov->images > 0) ? ov->images : std::max(p, 2);
    }
    pl->order = (ov && ov->order > 0) ? ov->order : order_for(eps_plan);
    pl->nu = pl->order * pl->order * pl->order;
    pl->nup = (pl->nu + 31) / 32 * 32;   // row stride: a multiple of the M2L tile step
    {
        // automatic far field: ANKH-FFT (the variant the paper times) up to order 6 (accuracy 1e-6) on a
        // supported grid, else ANKH-FMM.  Beyond order 6 the equispaced reinterpolation keeps ANKH-FFT
        // from the energy target at L_e = L: on the 1000-charge box at 1e-8 (order 8, 2^3 leaves) its
        // relative energy error is 1.9e-6 (8.3e-7 at L_e = 9, 1.1e-7 at L_e = 10).
        int ff = ov ? ov->far_field : ANKH_FAR_AUTO;
        if (ff == ANKH_FAR_AUTO) {
            ff = ANKH_FAR_FMM;
            const bool user_grid = ov && ov->depth >= 0;
            const int eqo = (ov && ov->eq_order > 0) ? ov->eq_order : pl->order;
            if (!user_grid) {
                const int g = leaves_for(n_atoms, pl->nu);
                int e = 0;
                while ((1 << e) < g) e++;
                const bool pow2 = (g & (g - 1)) == 0;
                if (pl->order <= 6 && fft_supported(pow2 ? e : 0, pl->order, eqo)) ff = ANKH_FAR_FFT;
            } else if (pl->order <= 6 && fft_supported(ov->depth, pl->order, eqo)) {
                ff = ANKH_FAR_FFT;
            }
        }
        pl->far_field = ff;
    }
    const bool fft = pl->far_field == ANKH_FAR_FFT;
    // the far-field chain on the second stream beside the pair kernel only on request: the pair kernel
    // holds every VGPR of every SIMD and issues at the VALU limit, so a far-field block beside it slows it
    // by about its own duration, and the evaluation takes the sum of its stages either way (on the 288k
    // water box 0.907 against 0.904 ms mixed, 1.636 against 1.615 ms FP64)
    pl->overlap = (ov && ov->overlap) ? ov->overlap == 1 : false;
    pl->depth = (ov && ov->depth >= 0) ? ov->depth : depth_for(n_atoms, pl->nu);
    // ANKH-FFT's grid of leaves per axis: a power of two is the octree depth; any other count (up to
    // kMaxFftDft) is a single level, kept as level 0
    int grid = 0;
    const bool auto_grid = fft && !(ov && (ov->leaves > 0 || ov->depth >= 0));
    if (fft && ((ov && ov->leaves > 0) || auto_grid)) {
        const int g = auto_grid ? leaves_for(n_atoms, pl->nu) : ov->leaves;
        if ((g & (g - 1)) == 0) {
            int e = 0;
            while ((1 << e) < g) e++;
            pl->depth = e;
        } else if (g <= kMaxFftDft) {
            grid = g;
            pl->depth = 0;
        } else {
            delete pl;
            return ANKH_ERR_INVALID_ARG;
        }
    }
    if (fft) {
        // ANKH-FFT: equispaced order (the Chebyshev order unless set); the automatic depth stops at
        // the deepest tree whose cell transforms fit one block
        pl->eq_order = (ov && ov->eq_order > 0) ? ov->eq_order : pl->order;
        if (!(ov && (ov->depth >= 0 || ov->leaves > 0)) && !auto_grid) pl->depth = std::min(pl->depth, kMaxFftDepth);
        if (!fft_supported(pl->depth, pl->order, pl->eq_order)) {
            delete pl;
            return ANKH_ERR_INVALID_ARG;
        }
        pl->fft_pa = 2 * pl->eq_order - 1;
        pl->fft_ph = pl->fft_pa / 2 + 1;
        pl->fft_nf = (int64_t)pl->fft_pa * pl->fft_pa * pl->fft_ph;
    }
    pl->nside = grid ? grid : 1 << pl->depth;
    // three-pass cell transforms beyond 16 cells per axis, or on request (not at depth 0); direct
    // DFTs along each axis on a grid that is not a power of two
    pl->fft_dft = grid != 0;
    pl->fft_split = fft && !grid && pl->nside >= 2 && (pl->nside > 16 || (ov && ov->fft_split == 1));
    pl->fft_single = fft && grid && !(ov && ov->fft_split == 1) && fft_single_ok(grid, false);
    pl->nleaf = (int64_t)pl->nside * pl->nside * pl->nside;
    size_t cells = 0;
    for (int e = 0; e <= pl->depth; e++) {
        Level &lv = pl->lv[e];
        lv.e = e;
        lv.nside = (e == pl->depth) ? pl->nside : 1 << e;
        lv.ncell = (int64_t)lv.nside * lv.nside * lv.nside;
        lv.cell0 = cells;
        lv.width = pl->edge / lv.nside;
        cells += lv.ncell;
    }
    pl->ncell_total = cells;
    // Root grid of the far-image operator: the image sum is interpolated over
    // the whole box, where a few more nodes than on the octree levels keep its
    // error below theirs (the paper also raises the order of the far-image
    // interpolation above the leaf order).  At depth 0 the root is the leaf.
    if (pl->depth == 0) pl->order0 = pl->order;
    else if (ov && ov->root_order > 0) pl->order0 = ov->root_order;
    else pl->order0 = std::min(kMaxRootOrder, std::max(9, pl->order + 2));
    pl->nu0 = pl->order0 * pl->order0 * pl->order0;
    pl->nup0 = (pl->nu0 + 63) / 64 * 64;
    build_tables(pl);

    const int64_t n = n_atoms;
    try {
        const int L = pl->order;
        dalloc(pl, &pl->d_tab, L + L * L + 2 * L * L);
        std::vector<double> tab(L + 3 * L * L);
        for (int k = 0; k < L; k++) tab[k] = pl->nodes[k];
        for (int k = 0; k < L * L; k++) tab[L + k] = pl->Hm[k];
        for (int b = 0; b < 2; b++)
            for (int k = 0; k < L * L; k++) tab[L + L * L + b * L * L + k] = pl->V[b][k];
        ck(hipMemcpy(pl->d_tab, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice));
        {
            // root tables: nodes of order L0 and V0[b][a][i] = S^(L0)_a((r_i -+ 1) / 2), i over the level-1 nodes
            const int L0 = pl->order0;
            std::vector<double> t0(L0 + 2 * L0 * L);
            std::vector<double> r0(L0), H0(L0 * L0);
            for (int k = 0; k < L0; k++) r0[k] = std::cos((2 * k + 1) * kPi / (2 * L0));
            for (int k = 0; k < L0; k++) {
                double a = 1, b = r0[k];
                for (int m = 0; m < L0; m++) {
                    double tm = m == 0 ? 1.0 : (m == 1 ? r0[k] : 2 * r0[k] * b - a);
                    if (m >= 2) { a = b; b = tm; }
                    H0[k * L0 + m] = (m == 0 ? 1.0 : 2.0 * tm) / L0;
                }
            }
            for (int k = 0; k < L0; k++) t0[k] = r0[k];
            for (int bb = 0; bb < 2; bb++)
                for (int i = 0; i < L; i++) {
                    const double x = (pl->nodes[i] + (bb ? 1.0 : -1.0)) / 2;
                    double T[kMaxRootOrder];
                    T[0] = 1;
                    if (L0 > 1) T[1] = x;
                    for (int m = 2; m < L0; m++) T[m] = 2 * x * T[m - 1] - T[m - 2];
                    for (int a = 0; a < L0; a++) {
                        double sacc = 0;
                        for (int m = 0; m < L0; m++) sacc += H0[a * L0 + m] * T[m];
                        t0[L0 + bb * L0 * L + a * L + i] = sacc;
                    }
                }
            dalloc(pl, &pl->d_tab0, t0.size());
            ck(hipMemcpy(pl->d_tab0, t0.data(), t0.size() * sizeof(double), hipMemcpyHostToDevice));
        }
        dalloc(pl, &pl->d_leaf, n);
        dalloc(pl, &pl->d_count, pl->nleaf);
        dalloc(pl, &pl->d_offs, pl->nleaf + 1);
        dalloc(pl, &pl->d_rank, n);
        dalloc(pl, &pl->d_perm, n);
        dalloc(pl, &pl->d_tmp, n);
        dalloc(pl, &pl->P.x, n);
        dalloc(pl, &pl->P.y, n);
        dalloc(pl, &pl->P.z, n);
        dalloc(pl, &pl->P.q, n);
        if (max_order >= 1) dalloc(pl, &pl->P.mu, 3 * n);
        if (max_order >= 2) dalloc(pl, &pl->P.th, 6 * n);
        if (max_order >= 3) dalloc(pl, &pl->P.om, 10 * n);
        if (precision != ANKH_FP64) {
            dalloc(pl, &pl->P.qf, n);
            if (max_order >= 1) dalloc(pl, &pl->P.muf, 3 * n);
            if (max_order >= 2) dalloc(pl, &pl->P.thf, 6 * n);
            if (max_order >= 3) dalloc(pl, &pl->P.omf, 10 * n);
        }
        dalloc(pl, &pl->d_M, cells * pl->nup);
        dalloc(pl, &pl->d_L, cells * pl->nup);
        const size_t kper = (size_t)kNumOff * pl->nup * pl->nup;
        dalloc(pl, &pl->d_Cper, (size_t)pl->nup0 * pl->nup0);
        dalloc(pl, &pl->d_cper_part, (size_t)kCperSlices * pl->nup0);
        if (pl->depth >= 1) {
            dalloc(pl, &pl->d_rootM, pl->nup0);
            dalloc(pl, &pl->d_rootL, pl->nup0);
            pl->root_owned = true;
        } else {
            pl->d_rootM = pl->d_M;
            pl->d_rootL = pl->d_L;
        }
        dalloc(pl, &pl->d_enear, pl->nleaf);
        if (precision == ANKH_FP64) {
            double *f = nullptr, *g = nullptr;
            dalloc(pl, &f, (size_t)3 * kNumSlots * n);
            dalloc(pl, &g, (size_t)3 * kNumSlots * n);
            pl->d_slot_f = f;
            pl->d_slot_g = g;
        } else {
            float *f = nullptr, *g = nullptr;
            dalloc(pl, &f, (size_t)3 * kNumSlots * n);
            dalloc(pl, &g, (size_t)3 * kNumSlots * n);
            pl->d_slot_f = f;
            pl->d_slot_g = g;
        }
        dalloc(pl, &pl->d_eleaf, pl->nleaf);
        dalloc(pl, &pl->d_F, 3 * n);
        dalloc(pl, &pl->d_G, 3 * n);
        dalloc(pl, &pl->d_terms, 8);
        dalloc(pl, &pl->d_part, 4 * kRedBlocks);
        dalloc(pl, &pl->d_err, 4);
        ck(hipStreamCreateWithFlags(&pl->side, hipStreamNonBlocking));
        ck(hipEventCreateWithFlags(&pl->ev_fork, hipEventDisableTiming));
        ck(hipEventCreateWithFlags(&pl->ev_join, hipEventDisableTiming));
        ck(launch_zero_i32(pl->d_err, 4, pl->stream));
        ck(launch_zero_f64(pl->d_terms, 8, pl->stream));
        ck(launch_zero_f64(pl->d_G, 3 * n, pl->stream));
        // operator tables: M2L matrices of levels 1..E (each built in float64, compressed
        // when that pays, then kept in the working precision) and the far-image root operator
        for (int e = 0; e <= pl->depth; e++) {
            pl->rpad[e] = pl->nup;
            pl->m2l_rank[e] = (e >= 1 && !fft) ? pl->nu : 0;
        }
        if (pl->depth >= 1 && !fft) {
            const double tol = (ov && ov->m2l_tol != 0) ? ov->m2l_tol : 0.1 * rel_accuracy;
            const bool compress = tol > 0 && pl->nu <= 400;
            const bool bf = precision == ANKH_MIXED_BF16X3;
            if (precision == ANKH_FP64) dalloc(pl, &pl->d_K, kper * pl->depth);
            else if (bf) dalloc(pl, &pl->d_Kb, 2 * kper * pl->depth);
            else dalloc(pl, &pl->d_Kf, kper * pl->depth);
            if (compress) {
                dalloc(pl, &pl->d_U, (size_t)pl->depth * pl->nup * pl->nup);
                for (int e = 1; e <= pl->depth; e++) pl->u_off[e] = (size_t)(e - 1) * pl->nup * pl->nup;
            }
            // scratch: the operators of the 16 symmetry classes and the full float64 stack of a level,
            // and room for the compression's intermediate products or the compressed float64 stack
            Scratch s_tmp, s_work, s_kc, s_reps;
            const size_t ntmp = 1 + (compress ? 1 : 0) + (compress && precision != ANKH_FP64 ? 1 : 0);
            const size_t nreps = m2l_reps_elems(pl);
            if (pl->bytes_limit && pl->bytes + (ntmp * kper + nreps) * sizeof(double) > pl->bytes_limit)
                throw std::bad_alloc();
            s_tmp.alloc(kper);
            s_reps.alloc(nreps);
            if (compress) s_work.alloc(kper);
            if (compress && precision != ANKH_FP64) s_kc.alloc(kper);
            double *tmp = s_tmp.p, *work = s_work.p, *kc = s_kc.p, *reps = s_reps.p;
            for (int e = 1; e <= pl->depth; e++) {
                const size_t slot = (size_t)(e - 1) * kper;
                ck(launch_build_m2l(pl, e, tmp, reps));
                const double *full = tmp;
                if (compress) {
                    double *dst = precision == ANKH_FP64 ? pl->d_K + slot : kc;
                    ck(compress_level(pl, e, tmp, dst, work, tol));
                    if (pl->rpad[e] < pl->nup) full = dst;
                }
                const int nr = pl->rpad[e];
                const size_t cnt = (size_t)kNumOff * nr * nr;
                if (precision == ANKH_FP64) {
                    if (full == tmp) ck(hipMemcpyAsync(pl->d_K + slot, tmp, cnt * sizeof(double),
                                                       hipMemcpyDeviceToDevice, pl->stream));
                } else if (bf) {
                    ck(launch_split_K_bf16(pl, full, pl->d_Kb + slot, pl->d_Kb + (size_t)pl->depth * kper + slot, nr));
                } else {
                    ck(launch_convert_f32(full, pl->d_Kf + slot, (int64_t)cnt, pl->stream));
                }
                ck(hipStreamSynchronize(pl->stream));
            }
            s_tmp.release();
            s_reps.release();
            s_work.release();
            s_kc.release();
            // compressed multipoles / locals of the compressed levels
            size_t coff = 0;
            for (int e = 1; e <= pl->depth; e++) {
                pl->c_off[e] = coff;
                if (pl->rpad[e] < pl->nup) coff += (size_t)pl->lv[e].ncell * pl->rpad[e];
            }
            if (coff) {
                dalloc(pl, &pl->d_Mc, coff);
                dalloc(pl, &pl->d_Lc, coff);
            }
            // M2L scratch: the split-K partial tiles of every split level side by side (level e at
            // byte m2l_part_off[e], 256-byte aligned; float64 in FP64, the float32 accumulators in the
            // mixed modes), summed in one launch after the last contraction; and in the mixed modes
            // every level's multipoles in the contraction's working precision (level e at mb_off[e])
            size_t part = 0;
            for (int e = 1; e <= pl->depth; e++) {
                const size_t nv = (size_t)pl->lv[e].ncell * pl->rpad[e];
                pl->m2l_part_off[e] = part;
                part += (m2l_part_bytes(pl, e) + 255) / 256 * 256;
                pl->mb_off[e] = pl->mb_total;
                pl->mb_total += nv;
            }
            if (part) dalloc(pl, &pl->d_m2l_part, (part + sizeof(double) - 1) / sizeof(double));
            if (precision == ANKH_MIXED) dalloc(pl, &pl->d_Mf, pl->mb_total);
            if (bf) dalloc(pl, &pl->d_Mb, 2 * pl->mb_total);
        }
        if (fft) {
            // the 6D spectrum: node transforms of the reinterpolation (B) and of the generating
            // cube (W), the work spectrum X and the real spectrum D
            std::vector<double2> B, W;
            fft_host_tables(pl->order, pl->eq_order, pl->nodes, B, W);
            std::vector<double2> tw;
            fft_host_roots(pl->nside, pl->fft_dft, tw);
            dalloc(pl, &pl->d_fftTw, tw.size());
            ck(hipMemcpy(pl->d_fftTw, tw.data(), tw.size() * sizeof(double2), hipMemcpyHostToDevice));
            dalloc(pl, &pl->d_fftB, B.size());
            dalloc(pl, &pl->d_fftW, W.size());
            dalloc(pl, &pl->d_fftX, (size_t)pl->fft_nf * pl->nleaf);
            dalloc(pl, &pl->d_fftD, (size_t)pl->fft_nf * pl->nleaf);
            ck(hipMemcpy(pl->d_fftB, B.data(), B.size() * sizeof(double2), hipMemcpyHostToDevice));
            ck(hipMemcpy(pl->d_fftW, W.data(), W.size() * sizeof(double2), hipMemcpyHostToDevice));
            ck(launch_fft_build_D(pl));
            pl->fft_f32 = precision != ANKH_FP64 && fft_f32_ok(pl);
            pl->fft_single32 = pl->fft_f32 && grid && !(ov && ov->fft_split == 1) && fft_single_ok(grid, true);
            if (pl->fft_f32) {
                // mixed modes: the transforms of an evaluation in float32 (half the spectrum's bytes); the
                // float64 spectrum and work array only served the plan-time build of D
                const size_t nx = (size_t)pl->fft_nf * pl->nleaf;
                std::vector<float2> B32(B.size()), tw32(tw.size());
                for (size_t i = 0; i < B.size(); i++) B32[i] = make_float2((float)B[i].x, (float)B[i].y);
                for (size_t i = 0; i < tw.size(); i++) tw32[i] = make_float2((float)tw[i].x, (float)tw[i].y);
                dalloc(pl, &pl->d_fftB32, B32.size());
                dalloc(pl, &pl->d_fftTw32, tw32.size());
                dalloc(pl, &pl->d_fftD32, nx);
                ck(hipMemcpy(pl->d_fftB32, B32.data(), B32.size() * sizeof(float2), hipMemcpyHostToDevice));
                ck(hipMemcpy(pl->d_fftTw32, tw32.data(), tw32.size() * sizeof(float2), hipMemcpyHostToDevice));
                ck(launch_fft_D_to_f32(pl));
                ck(hipStreamSynchronize(pl->stream));
                const hipError_t ex = hipFree(pl->d_fftX), ed = hipFree(pl->d_fftD);
                pl->d_fftX = nullptr;   // never freed twice, even when a free reports an error
                pl->d_fftD = nullptr;
                pl->bytes -= nx * (sizeof(double2) + sizeof(double));
                ck(ex);
                ck(ed);
                dalloc(pl, &pl->d_fftX32, nx);
            }
        } else {
            ck(launch_build_cper(pl));
        }
        ck(hipStreamSynchronize(pl->stream));
    } catch (const std::bad_alloc &) {
        free_all(pl);
        delete pl;
        return ANKH_ERR_OUT_OF_MEMORY;
    } catch (const HipFail &) {
        free_all(pl);
        delete pl;
        return ANKH_ERR_HIP;
    }
    pl->plan_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    *out = pl;
    return ANKH_OK;
}

ankh_status ankh_energy(ankh_plan_t pl, const double *pos, const double *q, const double *mu, const double *theta,
                        double *energy) {
    ankh_status st = check_inputs(pl, pos, q, mu, theta);
    if (st != ANKH_OK) return st;
    if (!energy) return ANKH_ERR_INVALID_ARG;
    return run(pl, pos, q, mu, theta, energy, nullptr, nullptr);
}

ankh_status ankh_energy_forces(ankh_plan_t pl, const double *pos, const double *q, const double *mu,
                               const double *theta, double *energy, double *forces, double *dE_dmu) {
    ankh_status st = check_inputs(pl, pos, q, mu, theta);
    if (st != ANKH_OK) return st;
    if (!energy || !forces) return ANKH_ERR_INVALID_ARG;
    return run(pl, pos, q, mu, theta, energy, forces, dE_dmu);
}

ankh_status ankh_energy_octupole(ankh_plan_t pl, const double *pos, const double *q, const double *mu,
                                 const double *theta, const double *omega, double *energy, double *forces,
                                 double *dE_dmu) {
    ankh_status st = check_inputs(pl, pos, q, mu, theta);
    if (st != ANKH_OK) return st;
    if (!energy || !omega || pl->max_order < 3) return ANKH_ERR_INVALID_ARG;
    return run(pl, pos, q, mu, theta, energy, forces, dE_dmu, omega);
}

ankh_status ankh_energy_derivs(ankh_plan_t pl, const double *pos, const double *q, const double *mu,
                               const double *theta, double *energy, double *forces, double *dE_dmu, double *dE_dq,
                               double *dE_dtheta) {
    ankh_status st = check_inputs(pl, pos, q, mu, theta);
    if (st != ANKH_OK) return st;
    if (!energy || (dE_dtheta && pl->max_order < 2)) return ANKH_ERR_INVALID_ARG;
    if ((dE_dq || dE_dtheta) && !pl->d_mom) {
        // before the evaluation, so that a failed allocation leaves every output untouched
        void *v = nullptr;
        const size_t bytes = (size_t)7 * pl->n * sizeof(double);
        if (pl->bytes_limit && pl->bytes + bytes > pl->bytes_limit) return ANKH_ERR_OUT_OF_MEMORY;
        if (hipMalloc(&v, bytes) != hipSuccess) {
            (void)hipGetLastError();
            return ANKH_ERR_OUT_OF_MEMORY;
        }
        pl->d_mom = static_cast<double *>(v);
        pl->bytes += bytes;
    }
    if ((st = run(pl, pos, q, mu, theta, energy, forces, dE_dmu)) != ANKH_OK) return st;
    if (!dE_dq && !dE_dtheta) return ANKH_OK;
    const int ord = theta ? 2 : (mu ? 1 : 0);
    if (launch_p2p_moments(pl, ord, pl->d_mom) != hipSuccess) return ANKH_ERR_HIP;
    if (launch_l2p_moments(pl, ord, pl->d_mom, dE_dq, dE_dtheta) != hipSuccess) return ANKH_ERR_HIP;
    return ANKH_OK;
}

ankh_status ankh_energy_derivs_noalloc(ankh_plan_t pl, const double *pos, const double *q, const double *mu,
                                       const double *theta, double *energy, double *forces, double *dE_dmu,
                                       double *dE_dq, double *dE_dtheta) {
    ankh_status st = check_inputs(pl, pos, q, mu, theta);
    if (st != ANKH_OK) return st;
    if (!energy || (dE_dtheta && pl->max_order < 2)) return ANKH_ERR_INVALID_ARG;
    if (pl->n > kNoAllocMaxAtoms) return ANKH_ERR_INVALID_ARG;
    double *mom = nullptr;
    if ((dE_dq || dE_dtheta) && (st = noalloc_scratch(pl->device, &mom)) != ANKH_OK) return st;
    // stage timing would create events on its first use: it stays off in this call
    const int timing = pl->timing;
    pl->timing = 0;
    st = run(pl, pos, q, mu, theta, energy, forces, dE_dmu);
    pl->timing = timing;
    if (st != ANKH_OK) return st;
    if (!dE_dq && !dE_dtheta) return ANKH_OK;
    // the near-field pass writes every [7][n] entry that the far-field pass then reads
    const int ord = theta ? 2 : (mu ? 1 : 0);
    if (launch_p2p_moments(pl, ord, mom) != hipSuccess) return ANKH_ERR_HIP;
    if (launch_l2p_moments(pl, ord, mom, dE_dq, dE_dtheta) != hipSuccess) return ANKH_ERR_HIP;
    return ANKH_OK;
}

ankh_status ankh_sync(ankh_plan_t pl) {
    if (!pl) return ANKH_ERR_INVALID_ARG;
    if (hipStreamSynchronize(pl->stream) != hipSuccess) return ANKH_ERR_HIP;
    int32_t err[4] = {0, 0, 0, 0};
    if (hipMemcpy(err, pl->d_err, sizeof(err), hipMemcpyDeviceToHost) != hipSuccess) return ANKH_ERR_HIP;
    if (err[0] || err[1] || err[2]) {
        if (launch_zero_i32(pl->d_err, 4, pl->stream) != hipSuccess) return ANKH_ERR_HIP;
        if (hipStreamSynchronize(pl->stream) != hipSuccess) return ANKH_ERR_HIP;
        return err[0] ? ANKH_ERR_NONFINITE_INPUT : err[1] ? ANKH_ERR_THETA_NOT_TRACELESS : ANKH_ERR_INVALID_ARG;
    }
    return ANKH_OK;
}

ankh_status ankh_set_timing(ankh_plan_t pl, int32_t enable) {
    if (!pl) return ANKH_ERR_INVALID_ARG;
    if (enable < 0 || enable > 2) return ANKH_ERR_INVALID_ARG;
    if (enable) pl->n_timed = 0;   // restart the averaging window
    pl->timing = enable;
    if (enable) pl->timed_mode = enable;
    return ANKH_OK;
}

ankh_status ankh_get_stats(ankh_plan_t pl, ankh_plan_stats *out) {
    if (!pl || !out) return ANKH_ERR_INVALID_ARG;
    if (hipStreamSynchronize(pl->stream) != hipSuccess) return ANKH_ERR_HIP;
    std::memset(out, 0, sizeof(*out));
    out->n_atoms = pl->n;
    out->depth = pl->fft_dft ? -1 : pl->depth;
    out->leaves_per_axis = pl->nside;
    out->order = pl->order;
    out->root_order = pl->order0;
    out->images = pl->images;
    out->max_order = pl->max_order;
    out->precision = pl->precision;
    out->xi = pl->xi;
    out->box_radius = pl->rB;
    out->rel_accuracy = pl->eps;
    out->plan_ms = pl->plan_ms;
    out->workspace_bytes = (int64_t)pl->bytes;
    out->m2l_flops = 0;
    for (int e = 1; e <= pl->depth; e++) {
        const double r = pl->m2l_rank[e], ncell = (double)pl->lv[e].ncell;
        out->m2l_flops += 2.0 * kNumIL * r * r * ncell;
        if (r < pl->nu) out->m2l_flops += 4.0 * pl->nu * r * ncell;
    }
    for (int e = 0; e < 8; e++) out->m2l_rank[e] = (e >= 1 && e <= pl->depth) ? pl->m2l_rank[e] : 0;
    out->far_field = pl->far_field;
    out->overlap = pl->overlap ? 1 : 0;
    out->fft_split = (pl->fft_split || (pl->fft_dft && !(pl->fft_f32 ? pl->fft_single32 : pl->fft_single))) ? 1 : 0;
    out->eq_order = pl->far_field == ANKH_FAR_FFT ? pl->eq_order : 0;
    out->near_precision = pl->precision == ANKH_FP64 ? 0 : 1;
    out->far_precision = pl->precision == ANKH_FP64 ? 0
                         : pl->far_field == ANKH_FAR_FFT ? (pl->fft_f32 ? 1 : 0)
                         : (pl->precision == ANKH_MIXED_BF16X3 ? 2 : 1);
    out->near_pairs = -1;
    if (pl->last_kind) {
        std::vector<int32_t> offs(pl->nleaf + 1);
        if (hipMemcpy(offs.data(), pl->d_offs, offs.size() * sizeof(int32_t), hipMemcpyDeviceToHost) != hipSuccess)
            return ANKH_ERR_HIP;
        const int ns = pl->nside;
        int64_t pairs = 0;
        for (int64_t l = 0; l < pl->nleaf; l++) {
            const int x = (int)(l / ((int64_t)ns * ns)), y = (int)((l / ns) % ns), z = (int)(l % ns);
            int64_t src = 0;
            for (int d = 0; d < 27; d++) {
                const int sx = (x + d / 9 - 1 + ns) % ns, sy = (y + (d / 3) % 3 - 1 + ns) % ns,
                          sz = (z + d % 3 - 1 + ns) % ns;
                const int64_t s = ((int64_t)sx * ns + sy) * ns + sz;
                src += offs[s + 1] - offs[s];
            }
            pairs += (int64_t)(offs[l + 1] - offs[l]) * src;
        }
        out->near_pairs = pairs - pl->n;
    }
    for (int i = 0; i < kNumStages; i++) out->stage_ms[i] = -1;
    out->timed_evals = pl->n_timed;
    if (pl->n_timed > 0) {
        for (int i = 0; i < kNumStages; i++) {
            if (!stage_recorded(pl->timed_mode, i)) continue;
            double sum = 0;
            for (int64_t t = 0; t < pl->n_timed; t++) {
                float ms = 0;
                if (hipEventElapsedTime(&ms, pl->evsets[t][i], pl->evsets[t][i + 1]) != hipSuccess) return ANKH_ERR_HIP;
                sum += ms;
            }
            out->stage_ms[i] = sum / pl->n_timed;
        }
    }
    return ANKH_OK;
}

ankh_status ankh_last_terms(ankh_plan_t pl, double *out_host) {
    if (!pl || !out_host) return ANKH_ERR_INVALID_ARG;
    if (hipStreamSynchronize(pl->stream) != hipSuccess) return ANKH_ERR_HIP;
    if (hipMemcpy(out_host, pl->d_terms, 7 * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess) return ANKH_ERR_HIP;
    return ANKH_OK;
}

ankh_status ankh_leaf_multipoles(ankh_plan_t pl, double *out_host, int64_t count) {
    if (!pl || !out_host) return ANKH_ERR_INVALID_ARG;
    const int64_t need = pl->nleaf * pl->nu;
    if (count < need) return ANKH_ERR_INVALID_ARG;
    if (hipStreamSynchronize(pl->stream) != hipSuccess) return ANKH_ERR_HIP;
    const double *Q = pl->d_M + pl->lv[pl->depth].cell0 * pl->nup;
    if (hipMemcpy2D(out_host, pl->nu * sizeof(double), Q, pl->nup * sizeof(double), pl->nu * sizeof(double),
                    pl->nleaf, hipMemcpyDeviceToHost) != hipSuccess)
        return ANKH_ERR_HIP;
    return ANKH_OK;
}

void ankh_destroy(ankh_plan_t pl) {
    if (!pl) return;
    (void)hipStreamSynchronize(pl->stream);
    free_all(pl);
    delete pl;
}

}  // extern "C"
