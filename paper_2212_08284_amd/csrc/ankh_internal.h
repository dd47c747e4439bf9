// Internal declarations shared by the host driver and the kernel files of the
// interpolated-Ewald library.  Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>

#include <array>
#include <cstddef>
#include <cstdint>
#include <vector>

#include "ankh.h"

namespace ankh {

constexpr int kMaxOrder = 10;        // largest Chebyshev order per axis of the octree levels
constexpr int kMaxRootOrder = 12;    // largest order of the root (far-image) grid
constexpr int kMaxRootNodes = kMaxRootOrder * kMaxRootOrder * kMaxRootOrder;
constexpr int kMaxDepth = 7;         // 2^21 leaves at most
constexpr int kMaxFftDepth = 6;      // ANKH-FFT: 64^2 cells of a plane of one node frequency in one block's LDS
constexpr int kMaxFftDft = 40;       // ANKH-FFT grids that are not powers of two: two 40^2 planes in LDS
constexpr int kNumOff = 343;         // slots for offsets d in [-3,3]^3 (316 used)
constexpr int kNumIL = 189;          // interaction-list length of every cell
constexpr int kRedBlocks = 1024;     // first-stage blocks of the energy reduction (the epilogue)
constexpr int kNumStages = 11;
constexpr int kCperSlices = 16;     // column slices of the far-image root matvec
constexpr int kNumSlots = 14;       // near-field partials per atom (see the pair kernel)

// index of offset d in [-3,3]^3
__host__ __device__ constexpr int off_index(int dx, int dy, int dz) {
    return ((dx + 3) * 7 + (dy + 3)) * 7 + (dz + 3);
}

// Particle data in leaf order (structure of arrays).  Positions are relative
// to the centre of the atom's leaf (float64 in every mode, so that pair
// separations are formed exactly); moments in float64 and, for the mixed
// mode, float32 copies for the pair kernel.
struct Particles {
    double *x, *y, *z;
    double *q;
    double *mu;      // [3][n]
    double *th;      // [6][n] (xx, xy, xz, yy, yz, zz)
    double *om;      // [10][n] (xxx, xxy, xxz, xyy, xyz, xzz, yyy, yyz, yzz, zzz)
    float *qf, *muf, *thf, *omf;
};

struct Level {
    int e;            // level index (0 = root)
    int nside;        // 2^e
    int64_t ncell;    // 8^e
    size_t cell0;     // first cell of this level in the concatenated M / L arrays
    double width;     // cell width
};

}  // namespace ankh

struct ankh_plan_s {
    // parameters
    int64_t n = 0;
    double rB = 0, edge = 0, eps = 0, xi = 0;
    int depth = 0, order = 0, nu = 0, nup = 0, images = 0, max_order = 0, precision = 0;
    int order0 = 0, nu0 = 0, nup0 = 0;   // root grid (far images): its own order
    hipStream_t stream = nullptr;
    // the far-field chain runs on `side` beside the pair kernel: forked from and joined back into
    // `stream` within every evaluation
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    int nside = 1;
    int64_t nleaf = 1;
    ankh::Level lv[ankh::kMaxDepth + 1];
    size_t ncell_total = 0;

    // host tables (float64)
    double nodes[ankh::kMaxOrder];
    double Hm[ankh::kMaxOrder * ankh::kMaxOrder];      // S(x) = H T(x), H[k][m]
    double V[2][ankh::kMaxOrder * ankh::kMaxOrder];    // M2M: V[b][a][i]

    // device buffers
    double *d_tab = nullptr;      // nodes[L], H[L*L], V[2][L*L]
    double *d_tab0 = nullptr;     // root: nodes[L0], V0[2][L0][L] (level-1 child nodes in root coordinates)
    double *d_rootM = nullptr;    // root multipole / local expansions [nup0]: separate buffers when
    double *d_rootL = nullptr;    // depth >= 1, else the level-0 rows of d_M / d_L
    bool root_owned = false;
    int32_t *d_leaf = nullptr;    // leaf id per input atom
    int32_t *d_count = nullptr;   // atoms per leaf (zero between evaluations: the scan clears it)
    bool count_dirty = true;      // d_count must be cleared before the next binning
    int32_t *d_offs = nullptr;    // CSR offsets [nleaf + 1]
    int32_t *d_rank = nullptr;    // arrival rank of each input atom in its leaf [n]
    int32_t *d_perm = nullptr;    // leaf-order slot -> input atom
    int32_t *d_tmp = nullptr;     // [n] segment-sort scratch
    ankh::Particles P{};
    double *d_M = nullptr;        // multipole expansions, all levels [cells][nup]
    double *d_L = nullptr;        // local expansions, all levels [cells][nup]
    double *d_K = nullptr;        // fp64 M2L matrices: level e>=1 at (e-1) * 343 * nup * nup, [d][l][k]
    float *d_Kf = nullptr;        // fp32 copy for the mixed mode
    float *d_Mf = nullptr;        // fp32 multipoles of all levels (mixed mode M2L operand), level e at mb_off[e]
    __bf16 *d_Kb = nullptr;       // bf16 hi parts of all levels' K (row-major K_d[k][l]), then the lo parts
    __bf16 *d_Mb = nullptr;       // bf16 hi parts of all levels' source multipoles (level e at mb_off[e]), then the lo parts
    size_t mb_off[ankh::kMaxDepth + 1] = {}, mb_total = 0;
    double *d_m2l_part = nullptr; // split-K partial tiles of every split level (float64 in FP64, float32 in the
                                  // mixed modes), level e at byte m2l_part_off[e]
    size_t m2l_part_off[ankh::kMaxDepth + 1] = {};
    // compressed M2L, per level e >= 1: kept rank, padded rank (n_up when the level is
    // uncompressed), basis U [n_up][rpad] at d_U + u_off[e], compressed multipoles and
    // locals [cells][rpad] at d_Mc / d_Lc + c_off[e]
    int m2l_rank[ankh::kMaxDepth + 1] = {};
    int rpad[ankh::kMaxDepth + 1] = {};
    size_t u_off[ankh::kMaxDepth + 1] = {}, c_off[ankh::kMaxDepth + 1] = {};
    double *d_U = nullptr, *d_Mc = nullptr, *d_Lc = nullptr;
    double *d_Cper = nullptr;     // far-image root operator [nup0][nup0]
    double *d_cper_part = nullptr;// its column-slice partial products [kCperSlices][nup0]
    double *d_enear = nullptr;    // near energy per leaf (the pair kernel's block of that source leaf)
    void *d_slot_f = nullptr;     // near-field partials per atom: forces [3][kNumSlots][n] and fields [3][kNumSlots][n], float64 or float32
    void *d_slot_g = nullptr;
    double *d_eleaf = nullptr;    // far energy per leaf
    double *d_F = nullptr;        // forces in leaf order [3][n]
    double *d_G = nullptr;        // fields in leaf order [3][n]
    double *d_terms = nullptr;    // energy terms [8]
    double *d_part = nullptr;     // reduction partials
    int32_t *d_err = nullptr;     // latched device errors [4]: non-finite, theta trace, invalid value
    double *d_ind = nullptr;      // induced-dipole solver vectors (allocated by the first ankh_induce)
    double *d_mom = nullptr;      // near-field dE/dq, dE/dTheta [7][n] (allocated by the first ankh_energy_derivs)
    // ANKH-FFT far field: equispaced order, node period pa = 2 eq_order - 1, kept node frequencies
    // fft_nf = pa * pa * (pa / 2 + 1); B = node DFT x reinterpolation [pa][order], W = plain node
    // DFT [pa][pa], spectrum work X [fft_nf][nleaf] (complex), real spectrum D [fft_nf][nleaf]
    int far_field = ANKH_FAR_FMM;
    bool overlap = true;          // far-field chain on `side` beside the pair kernel
    int eq_order = 0, fft_pa = 0, fft_ph = 0;
    bool fft_split = false;       // cell transforms in three passes through HBM (n > 16, or on request)
    bool fft_dft = false;         // leaf grid not a power of two: direct DFTs along each axis (three passes)
    bool fft_single = false;      // 12^3 / 20^3 grid: all cells of a node frequency in one block's LDS
    int64_t fft_nf = 0;
    double2 *d_fftB = nullptr, *d_fftW = nullptr, *d_fftX = nullptr;
    double2 *d_fftTw = nullptr;   // e^{-2 pi i k / n}: k < n/2 (radix 2) or k < n (direct DFT), three-pass path
    double *d_fftD = nullptr;
    // mixed modes: the spectrum, its node-transform matrix, the roots and the real spectrum in float32
    // (the float64 X and D above are freed once D is built)
    bool fft_f32 = false;
    bool fft_single32 = false;    // float32 cell transforms in one block per node frequency (12, 20, 24 per axis)
    float2 *d_fftX32 = nullptr, *d_fftB32 = nullptr, *d_fftTw32 = nullptr;
    float *d_fftD32 = nullptr;
    size_t bytes = 0;
    int device = 0;               // the HIP device current at plan time (the plan's buffers live there)
    int num_cu = 256;             // its compute units (the persistent grid of the one-block cell transforms)
    size_t bytes_limit = 0;       // ankh_overrides.workspace_limit (0 = none)

    // statistics / timing
    double plan_ms = 0;
    int timing = 0;               // 0 off, 1 every stage boundary, 2 the boundaries of stages 4 and 8 only
    // one set of stage-boundary events per timed evaluation since timing was enabled
    std::vector<std::array<hipEvent_t, ankh::kNumStages + 1>> evsets;
    int64_t n_timed = 0;
    int timed_mode = 1;           // the timing mode of the evaluations in the averaging window
    int last_kind = 0;            // 0 none, 1 energy, 2 energy+forces
    int last_order = 0;
};

namespace ankh {

// ---- launchers (defined in the kernel files) -------------------------------
hipError_t launch_zero_i32(int32_t *p, int64_t n, hipStream_t s);
hipError_t launch_zero_f64(double *p, int64_t n, hipStream_t s);
hipError_t launch_sort(ankh_plan_s *pl, const double *pos, const double *q, const double *mu,
                       const double *th);
hipError_t launch_gather(ankh_plan_s *pl, const double *pos, const double *q, const double *mu,
                         const double *th, const double *om);
hipError_t launch_p2m(ankh_plan_s *pl, int ord);
hipError_t launch_m2m(ankh_plan_s *pl, int e_parent);
hipError_t launch_l2l(ankh_plan_s *pl, int e_child);
hipError_t launch_cper(ankh_plan_s *pl);
hipError_t launch_leafdot(ankh_plan_s *pl);
hipError_t launch_l2p(ankh_plan_s *pl, int ord, bool fields);
hipError_t launch_reduce(ankh_plan_s *pl, double *energy_out);   // the epilogue's partials, in block order
hipError_t launch_m2l(ankh_plan_s *pl, int e);
int m2l_splits(const ankh_plan_s *pl, int e);
int m2l_row_frags(int nup);
int m2l_col_frags(const ankh_plan_s *pl, int e);
size_t m2l_part_bytes(const ankh_plan_s *pl, int e);
hipError_t launch_m2l_prepare(ankh_plan_s *pl);     // mixed modes: uncompressed levels' multipoles in the working precision
hipError_t launch_m2l_finish(ankh_plan_s *pl);      // sums of the split levels' partial tiles
hipError_t launch_split_K_bf16(ankh_plan_s *pl, const double *K, __bf16 *hi, __bf16 *lo, int nr);
hipError_t compress_level(ankh_plan_s *pl, int e, const double *K, double *Kc, double *work, double tol);
hipError_t launch_m2l_basis(ankh_plan_s *pl, bool expand);
hipError_t launch_m2l_project(ankh_plan_s *pl);   // all compressed levels: Mc = M U
hipError_t launch_m2l_expand(ankh_plan_s *pl);    // all compressed levels: L = Lc U^T
inline bool is_mixed(const ankh_plan_s *pl) { return pl->precision != ANKH_FP64; }
hipError_t launch_p2p(ankh_plan_s *pl, int ord, bool grad, bool fields);
hipError_t launch_epilogue(ankh_plan_s *pl, int ord, bool grad, bool fields, double *forces, double *dEdmu);
// derivatives in the charges and quadrupoles: near part into near [7][n] (leaf order), then the far
// part, self and background terms and the output in caller order
hipError_t launch_p2p_moments(ankh_plan_s *pl, int ord, double *near);
hipError_t launch_l2p_moments(ankh_plan_s *pl, int ord, const double *near, double *dEdq, double *dEdth);
// one evaluation of the path (the body of ankh_energy / ankh_energy_forces; inputs already checked);
// forces == nullptr with dEdmu != nullptr is a fields-only evaluation
ankh_status evaluate(ankh_plan_s *pl, const double *pos, const double *q, const double *mu, const double *th,
                     double *energy, double *forces, double *dEdmu);
// the M2L stack of level e into K (kNumOff x nup x nup), from the operators of the 16 classes of the
// cube's symmetries built into reps (m2l_reps_elems doubles)
size_t m2l_reps_elems(const ankh_plan_s *pl);
hipError_t launch_build_m2l(ankh_plan_s *pl, int e, double *K, double *reps);
hipError_t launch_build_cper(ankh_plan_s *pl);
hipError_t launch_convert_f32(const double *src, float *dst, int64_t n, hipStream_t s);
// ANKH-FFT (ankh_fft.hip)
bool fft_supported(int depth, int L, int eq_order);
bool fft_single_ok(int nside, bool f32);
void fft_host_tables(int L, int eq_order, const double *cheb_nodes, std::vector<double2> &B, std::vector<double2> &W);
void fft_host_roots(int nside, bool full, std::vector<double2> &tw);
hipError_t launch_fft_build_D(ankh_plan_s *pl);    // plan time: the real spectrum D
hipError_t launch_fft_D_to_f32(ankh_plan_s *pl);   // plan time: its float32 copy (mixed modes)
bool fft_f32_ok(const ankh_plan_s *pl);            // every transform of the plan has a float32 form
hipError_t launch_fft_forward(ankh_plan_s *pl);    // leaf multipoles -> half spectrum X
hipError_t launch_fft_cells(ankh_plan_s *pl);      // cell transforms, product with D, inverse
hipError_t launch_fft_inverse(ankh_plan_s *pl);    // X -> leaf local expansions
bool fft_inverse_leaf_energies(const ankh_plan_s *pl);   // launch_fft_inverse also writes the leaf far energies

}  // namespace ankh
