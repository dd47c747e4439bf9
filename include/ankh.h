/*
 * ankh.h - C ABI of the MI355X interpolated-Ewald library (ANKH hot path:
 * ANKH-FFT far field by default, ANKH-FMM on request).
 *
 * The library evaluates the periodic electrostatic energy of point charges,
 * dipoles and quadrupoles in a cubic box,
 *
 *     E = 1/2 sum_t sum_x sum_y D_x D_y 1/|x - y + t|,
 *     D_u = q_u + mu_u . grad + Theta_u : grad grad,            (paper, eq. 1)
 *
 * (the x = y, t = 0 term omitted, tin-foil boundary), by the interpolated
 * Ewald strategy of the paper: with a small splitting parameter xi the
 * reciprocal Ewald term is negligible and the real-space kernel
 * H = erfc(xi r)/r (eq. for H) is summed over a truncated cube of images.
 * That sum is split over a uniform grid of leaves into a near field (direct
 * pair sums between adjacent leaves) and a far field handled by Chebyshev
 * interpolation: modified charges at the leaves (Alg. 2), then either
 *  - ANKH-FFT (the ANKH-FFT section, Alg. 5; the automatic choice): the leaf
 *    grids reinterpolated onto equispaced nodes and every non-adjacent leaf
 *    pair, far images included, through one 6D convolution applied by FFT, or
 *  - ANKH-FMM (the ANKH-FMM section, Alg. 3): upward M2M, M2L over the
 *    interaction lists of every octree level (cells of the adjacent images
 *    included), one root operator for all farther images (periodicity
 *    section), downward L2L,
 * then the self energy (eq. for E_self) and, for non-neutral cells, the
 * neutralising background.  Forces and fields come from the adjoint of the
 * same approximation (the transposed far-field chain, L2P, pair gradients).
 *
 * Units: Angstrom and elementary charge, Coulomb constant 1 (eq. 1 carries no
 * prefactor); energies in e^2/Angstrom.
 *
 * Memory: every array argument of ankh_energy / ankh_energy_forces is a
 * DEVICE pointer (HIP global memory, e.g. a PyTorch ROCm tensor), row-major
 * float64, owned by the caller and never modified.  The plan owns all its
 * internal buffers (sorted particle data, multipole and local expansions,
 * operator tables) and frees them in ankh_destroy.
 *
 * Streams: all work of a plan is ordered on the HIP stream given to
 * ankh_plan (NULL = the default stream) and is asynchronous; outputs are
 * valid after that stream is synchronised or after ankh_sync.  On request
 * (ankh_overrides.overlap) the far-field chain of an evaluation runs on a
 * second stream that the plan owns, forked from that stream after the
 * particles are sorted and joined back before the pair results are summed,
 * beside the pair kernel.  Work enqueued on the plan's stream is ordered as
 * if everything ran on it either way.
 * A plan is not thread-safe; use one plan per stream.
 *
 * Errors: host-checkable errors return at once with outputs untouched.
 * Device-detected input errors (non-finite positions or moments, Theta not
 * traceless) are latched in the plan and returned by ankh_sync.  No C++
 * exception crosses this interface.
 */
#ifndef ANKH_H
#define ANKH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ankh_plan_s *ankh_plan_t;

typedef enum {
    ANKH_OK = 0,
    ANKH_ERR_INVALID_ARG = 1,          /* null pointer, n mismatch, box_radius <= 0, accuracy out of range ... */
    ANKH_ERR_NONFINITE_INPUT = 2,      /* latched: NaN/Inf in positions or moments */
    ANKH_ERR_THETA_NOT_TRACELESS = 3,  /* latched: |trace Theta| > 1e-6 (max |Theta_ii| + 1), or an octupole
                                          trace Omega_aab above 1e-6 (max |Omega_abc| + 1) */
    ANKH_ERR_LEAF_OVERFLOW = 4,        /* reserved: no kernel has a per-leaf capacity limit */
    ANKH_ERR_ACCURACY_UNREACHABLE = 5, /* plan: accuracy below what the precision mode can reach */
    ANKH_ERR_OUT_OF_MEMORY = 6,        /* plan: device allocation failed */
    ANKH_ERR_HIP = 7,                  /* a HIP runtime call failed */
    ANKH_ERR_NOT_CONVERGED = 8         /* ankh_induce: the tolerance was not reached within max_iter, or the
                                          iteration met a non-positive curvature (the polarisabilities are too
                                          large for the geometry: polarisation catastrophe) */
} ankh_status;

typedef enum {
    ANKH_FP64 = 0,          /* every stage in float64 */
    ANKH_MIXED = 1,         /* near-field pair terms and the far-field contraction in float32;
                               pair separations, self/background terms, moments, and every
                               reduction in float64 */
    ANKH_MIXED_BF16X3 = 2   /* as ANKH_MIXED, with the far-field contraction on the bf16
                               matrix cores in split precision (hi*hi + hi*lo + lo*hi,
                               float32 accumulation).  This applies to the ANKH-FMM M2L; the
                               ANKH-FFT transforms have no matrix-core form, so with that far
                               field both mixed modes run the same float32 path */
} ankh_precision;

/* Optional overrides of the planner's choices: depth < 0 and any other field <= 0 mean "auto". */
typedef struct {
    int32_t depth;   /* octree depth E (leaves per axis 2^E), 0..7; NEGATIVE = auto (0 forces depth 0) */
    int32_t order;   /* Chebyshev interpolation order L per axis, 2..10 */
    int32_t images;  /* image radius p: images I with |I|_inf <= p are summed */
    double xi;       /* Ewald splitting parameter (1/Angstrom) */
    int32_t root_order; /* order of the root grid that carries the far images, 2..12 (depth >= 1) */
    double m2l_tol;     /* compressed M2L (the singular-value compression of the far-field operators):
                           singular values above m2l_tol x the largest are kept; 0 = auto (0.1 x
                           rel_accuracy, orders <= 7), NEGATIVE = no compression */
    int32_t far_field;  /* far-field method, an ankh_far_field value; 0 = auto: ANKH_FAR_FFT up to order 6
                           (rel_accuracy >= 1e-6) on a supported leaf grid, else ANKH_FAR_FMM (at higher orders
                           the equispaced reinterpolation of ANKH-FFT misses the energy target) */
    int32_t eq_order;   /* ANKH-FFT: equispaced nodes per axis of each leaf grid, 2..10; 0 = the
                           Chebyshev order */
    int32_t leaves;     /* ANKH-FFT: leaves per axis of its single-level grid, 1..40 or a power of two up
                           to 64 (any count: the grid need not be an octree level); 0 = 2^depth */
    int32_t fft_split;  /* ANKH-FFT: 1 = the cell transforms in three passes through HBM even when one
                           block holds the cells of a node frequency (the path of depths 5 and 6 and of
                           24 leaves per axis, for testing it on smaller grids); 0 = only when needed
                           (12 and 20 leaves per axis: one block if the device grants 128 KB of LDS per
                           block, else three passes) */
    int32_t overlap;    /* far-field chain beside the pair kernel on the plan's second stream: 1 = yes,
                           2 = no (every stage in sequence on the plan's stream), 0 = auto (no: the pair
                           kernel fills every SIMD's registers and issues at the VALU limit, so the
                           evaluation takes the sum of its stages either way) */
    double force_accuracy; /* target relative RMS error of the forces and fields, in [1e-12, 1e-2]; 0 = none.
                              rel_accuracy bounds the relative energy error (the accuracy measure of the
                              paper's numerical results); the force error follows it at a workload-dependent
                              multiple, a few times rel_accuracy on neutral molecules and up to ~30 times on
                              unscreened ions.  With a force target the planner chooses xi, the image radius
                              and the order for min(rel_accuracy, force_accuracy / 30). */
    int64_t workspace_limit; /* most device bytes the plan may hold, its transient plan-time buffers and the
                                buffers that ankh_energy_derivs / ankh_induce add on first use included;
                                0 = no limit.  A plan beyond it fails with ANKH_ERR_OUT_OF_MEMORY (*out
                                untouched); a first derivative / induced-dipole call beyond it returns
                                ANKH_ERR_OUT_OF_MEMORY before any output is written. */
} ankh_overrides;

/* Far-field methods.
 *   ANKH_FAR_FMM  ANKH-FMM (the ANKH-FMM section): multipoles up the octree, M2L over the
 *                 interaction lists of every level, the far images through one root operator,
 *                 locals down the tree.
 *   ANKH_FAR_FFT  ANKH-FFT (the ANKH-FFT section): the leaf modified charges reinterpolated onto an
 *                 equispaced grid per leaf, and every non-adjacent leaf pair, far images included,
 *                 through one 6D convolution evaluated by FFT (matrix factorisation, diagonalisation
 *                 and real-spectrum passages).  Needs depth <= 6 (auto depth is capped there; up
 *                 to depth 4, and on grids of 12 and 20 leaves per axis where the device grants
 *                 the LDS, the cell transforms of a node frequency run in one block, otherwise in
 *                 three passes through HBM) and 2 eq_order - 1 node frequencies per axis within
 *                 the per-block LDS budget (eq_order <= 8 at order <= 8).  The near field, P2M,
 *                 L2P, self and background terms are those of ANKH-FMM; stage 3 of the timing
 *                 is the forward node transform, stage 4 the
 *                 cell transforms and the product with the spectrum, stage 5 is empty and stage 6
 *                 the inverse node transform with the leaf energies.  The spectrum of the 6D
 *                 convolution is built at plan time (an image sum per entry on the device). */
typedef enum { ANKH_FAR_AUTO = 0, ANKH_FAR_FMM = 1, ANKH_FAR_FFT = 2 } ankh_far_field;

typedef struct {
    int64_t n_atoms;
    int32_t depth, order, images, max_order, precision;
    int32_t root_order;        /* order of the root grid of the far-image operator */
    double xi, box_radius, rel_accuracy;
    double plan_ms;            /* wall time of ankh_plan (operator tables included) */
    int64_t workspace_bytes;   /* device memory owned by the plan */
    double m2l_flops;          /* algorithmic M2L flops per evaluation: 2 * 189 * r_e^2 per cell of level e
                                  (r_e = the kept rank, n_u when uncompressed), plus 4 n_u r_e per cell
                                  for the projection and expansion of compressed levels */
    int64_t near_pairs;        /* ordered near-field pairs of the last evaluation (-1 if unknown) */
    /* per-stage device time in ms (hipEvents on the plan's stream), averaged
       over the evaluations run since timing was last enabled with
       ankh_set_timing; -1 when there were none.
       Stages: 0 bin+sort, 1 gather, 2 p2m, 3 m2m, 4 m2l (all levels), 5 periodic root,
               6 l2l + leaf energies, 7 l2p, 8 p2p pair kernel, 9 p2p partial sums,
               10 reduce + unpermute */
    double stage_ms[11];
    int64_t timed_evals;       /* evaluations averaged into stage_ms */
    int32_t m2l_rank[8];       /* kept rank of the M2L operators per level e = 1..depth (n_u when the
                                  level is not compressed; 0 for e = 0 and e > depth) */
    int32_t far_field;         /* ANKH_FAR_FMM or ANKH_FAR_FFT */
    int32_t eq_order;          /* ANKH-FFT: equispaced nodes per axis (0 for ANKH-FMM) */
    int32_t overlap;           /* 1 if the far-field chain runs beside the pair kernel, else 0 */
    int32_t fft_split;         /* ANKH-FFT: 1 if the cell transforms run in three passes */
    int32_t leaves_per_axis;   /* leaves per axis of the finest grid (2^depth; for an ANKH-FFT grid
                                  that is not a power of two, depth reads -1) */
    int32_t near_precision;    /* arithmetic of the near-field pair terms: 0 float64, 1 float32 */
    int32_t far_precision;     /* arithmetic of the far-field chain (P2M to L2P): 0 float64, 1 float32,
                                  2 the ANKH-FMM contraction in split bf16 (rest float64) */
} ankh_plan_stats;

/*
 * ankh_plan: choose parameters and precompute the operator tables for a box.
 *   out           receives the plan handle (host pointer, not NULL).
 *   n_atoms       number of atoms of every later call (>= 1).
 *   box_radius    r_B, half the cubic box edge (Angstrom, > 0); the box is
 *                 [-r_B, r_B)^3 and positions anywhere are wrapped into it.
 *   rel_accuracy  target relative accuracy of the energy, in [1e-12, 1e-2]:
 *                 sets xi (reciprocal term below the target), the image
 *                 radius p and the interpolation order L (convergence in L
 *                 is geometric, numerical-results section).
 *   max_order     0 charges, 1 + dipoles, 2 + quadrupoles, 3 + octupoles
 *                 (ankh_energy_octupole); later calls may pass NULL for the
 *                 moments above this order.
 *   precision     an ankh_precision value.
 *   ov            NULL or overrides of depth / order / images / xi.
 *   hip_stream    hipStream_t (as void *) all work is enqueued on; NULL = default.
 * Precompute (the M2L matrices of every level and the root operator of the
 * far images, which depend only on the box, as the periodicity section notes)
 * runs on the device, synchronously.
 */
ankh_status ankh_plan(ankh_plan_t *out, int64_t n_atoms, double box_radius, double rel_accuracy,
                      int32_t max_order, int32_t precision, const ankh_overrides *ov, void *hip_stream);

/*
 * ankh_energy: the energy only (paper, Alg. 3).
 *   pos    [n][3]  positions (device, float64).
 *   q      [n]     charges.
 *   mu     [n][3]  dipoles, or NULL (treated as 0); required if max_order >= 1 was planned
 *                  and ignored (must be NULL) if max_order == 0.
 *   theta  [n][6]  traceless symmetric quadrupoles as (xx, xy, xz, yy, yz, zz), used
 *                  literally in Theta : grad grad (no 1/2 or 1/3 factor), or NULL.
 *   energy [1]     device output.
 */
ankh_status ankh_energy(ankh_plan_t plan, const double *pos, const double *q, const double *mu,
                        const double *theta, double *energy);

/*
 * ankh_energy_forces: energy, forces F_i = -dE/dx_i and fields dE/dmu_i of the
 * same approximation (the exact gradient of the approximate energy).
 *   forces [n][3]  device output, not NULL.
 *   dE_dmu [n][3]  device output or NULL: the field dE/dmu at each atom when the call passes
 *                  dipoles or quadrupoles (mu may then be NULL: the field at mu = 0); zeros for
 *                  a charges-only call.
 */
ankh_status ankh_energy_forces(ankh_plan_t plan, const double *pos, const double *q, const double *mu,
                               const double *theta, double *energy, double *forces, double *dE_dmu);

/*
 * ankh_energy_octupole: energy, forces and fields with octupoles, the next
 * order of the operator of eq. 1,
 *
 *     D_u = q_u + mu_u . grad + Theta_u : grad grad + Omega_u : grad grad grad,
 *
 * the extension to any multipole order that the paper's introduction and its
 * first conclusion name.  Every stage takes the third derivative order: P2M
 * anterpolates Omega : grad^3 S_k (Alg. 2 with the third power of the
 * differentiation matrix), the pair terms use the rank-3 moments, L2P the
 * fourth basis derivatives, and the self energy gains -(48/7) xi^7/sqrt(pi)
 * Omega : Omega per atom.
 *   omega  [n][10] device, traceless symmetric octupoles as (xxx, xxy, xxz,
 *                  xyy, xyz, xzz, yyy, yyz, yzz, zzz), used literally in
 *                  Omega : grad^3 (no 1/6 or 1/15 factor; the full
 *                  contraction weights the components 1, 3, 3, 3, 6, 3, 1,
 *                  3, 3, 1); not NULL.  A trace Omega_aab (a summed) that
 *                  does not vanish is latched as ANKH_ERR_THETA_NOT_TRACELESS.
 *   pos, q, mu, theta, energy  as for ankh_energy (mu, theta may be NULL).
 *   forces [n][3]  device output or NULL (energy only, or fields only).
 *   dE_dmu [n][3]  device output or NULL: dE/dmu.
 * Needs a plan with max_order 3 (which then also serves ankh_energy and the
 * other calls for lower moments).  Both precision modes and both far fields.
 */
ankh_status ankh_energy_octupole(ankh_plan_t plan, const double *pos, const double *q, const double *mu,
                                 const double *theta, const double *omega, double *energy, double *forces,
                                 double *dE_dmu);

/*
 * ankh_energy_derivs: the energy with any of its derivatives in the atoms'
 * positions and moments (the q, mu, Theta of eq. 1), the adjoint of the same
 * approximation.  The paper evaluates the energy and names forces as a
 * direct perspective of the method; these are the derivatives in every
 * input of the energy.
 *   energy    [1]     device output, not NULL.
 *   forces    [n][3]  device output or NULL: -dE/dx.
 *   dE_dmu    [n][3]  device output or NULL: dE/dmu (zeros without dipoles).
 *   dE_dq     [n]     device output or NULL: dE/dq_i, the potential of all
 *                     other moments (and the atom's periodic images) at atom
 *                     i, with the self and neutralising-background terms.
 *   dE_dtheta [n][6]  device output or NULL: dE/dTheta_i.  E is defined for
 *                     traceless Theta only, so this is the traceless part G of
 *                     the full-tensor derivative, per stored component
 *                     (xx, xy, xz, yy, yz, zz) = (G_xx, 2 G_xy, 2 G_xz, G_yy,
 *                     2 G_yz, G_zz): for every traceless change dTheta of the
 *                     stored components, sum dE_dtheta . dTheta = dE.  Needs a
 *                     plan with max_order 2; defined also when theta is NULL.
 * The charge and quadrupole derivatives cost one more pass over the near
 * pairs (gather form, in the plan's precision) and one over the atoms for the
 * far field.  The plan allocates 7 n doubles for them on the first call.
 */
ankh_status ankh_energy_derivs(ankh_plan_t plan, const double *pos, const double *q, const double *mu,
                               const double *theta, double *energy, double *forces, double *dE_dmu,
                               double *dE_dq, double *dE_dtheta);

/*
 * ankh_energy_derivs_noalloc: ankh_energy_derivs for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, same outputs, bitwise
 * equal to ankh_energy_derivs on the same plan and inputs.  The call itself
 * allocates nothing: the plan's buffers serve the evaluation, and the 7 n
 * doubles of the charge and quadrupole derivatives live in a static device
 * array of the library (28 MiB, held on every GPU the library runs on until
 * the process ends) instead of a plan buffer.
 *   Limit: n_atoms <= 524288 (2^19); a larger plan returns ANKH_ERR_INVALID_ARG
 *   before anything is enqueued.
 *   The static array is shared by every call on one GPU: calls that overlap on
 *   one GPU (other streams, other threads, other plans) race and must be
 *   ordered by the caller.  Each call writes every entry it reads, so nothing
 *   of an earlier call's contents leaks into a result.
 *   Stage timing (ankh_set_timing) is ignored for this call: its events would
 *   be created on first use.
 */
ankh_status ankh_energy_derivs_noalloc(ankh_plan_t plan, const double *pos, const double *q, const double *mu,
                                       const double *theta, double *energy, double *forces, double *dE_dmu,
                                       double *dE_dq, double *dE_dtheta);

/*
 * ankh_induce: induced dipoles of isotropic point polarisabilities, the
 * polarizable use of the method that the paper's introduction names (the
 * moments of eq. 1 extended by induced dipoles).  The induced dipoles are the
 * minimiser of
 *
 *     U(mu_ind) = E(q, mu + mu_ind, Theta) + sum_i |mu_ind_i|^2 / (2 alpha_i),
 *
 * E the energy of this plan's approximation.  E is quadratic in the moments,
 * so the minimiser solves (alpha^-1 + H) mu_ind = -dE/dmu(q, mu, Theta), where
 * H p = dE/dmu of the dipoles p alone: one field evaluation per product.  In
 * the scaled unknown y = alpha^(-1/2) mu_ind the matrix I + alpha^(1/2) H
 * alpha^(1/2) is symmetric, positive definite below the polarisation
 * catastrophe, and alpha = 0 atoms drop out; it is solved by conjugate
 * gradients from y = 0, driven from the host (two scalars read back per
 * iteration), every vector operation and dot product on the device in
 * float64 with a fixed-order reduction.  The field evaluations run in the
 * plan's precision mode.
 *   pos, q, mu, theta  as for ankh_energy_forces (device); mu may be NULL
 *                  (no permanent dipoles); the plan needs max_order >= 1.
 *   alpha  [n]     polarisabilities in Angstrom^3 (device, finite, >= 0; 0 =
 *                  not polarisable).  A negative value is latched
 *                  (ANKH_ERR_INVALID_ARG from ankh_sync), a non-finite one as
 *                  ANKH_ERR_NONFINITE_INPUT; such atoms are treated as alpha = 0.
 *   tol            stop when |r| <= tol |b| in the scaled system (> 0).
 *   max_iter       at most this many products (>= 0).
 *   mu_ind [n][3]  device output: the induced dipoles (the last iterate when
 *                  not converged).
 *   energy [1]     device output or NULL: U at mu_ind (one more evaluation).
 *   forces [n][3]  device output or NULL: -dU/dx at mu_ind (held fixed; exact
 *                  at the minimiser, where dU/dmu_ind = 0).
 *   iterations     host output or NULL: products done.
 *   rel_residual   host output or NULL: |r| / |b| at the end (0 when b = 0).
 * Synchronises the plan's stream.  Returns ANKH_ERR_NOT_CONVERGED (outputs
 * written) when tol is not reached; host-checkable errors as elsewhere.  The
 * plan allocates its solver vectors (7 x 3n + 2n doubles) on the first call.
 * Stage timings (ankh_set_timing) include the evaluations made here.
 */
ankh_status ankh_induce(ankh_plan_t plan, const double *pos, const double *q, const double *mu,
                        const double *theta, const double *alpha, double tol, int32_t max_iter, double *mu_ind,
                        double *energy, double *forces, int32_t *iterations, double *rel_residual);

/* Waits for the plan's stream; returns the first latched device-side input error, then clears it. */
ankh_status ankh_sync(ankh_plan_t plan);

/* Copies the plan's parameters and statistics (synchronises the plan's stream). */
ankh_status ankh_get_stats(ankh_plan_t plan, ankh_plan_stats *out);

/* Per-stage hipEvent timing of later evaluations: 0 disables it; 1 records an event at every stage
 * boundary and runs the stages in sequence on the plan's stream (no far-field / pair overlap), so the
 * stage figures add up; 2 keeps the plan's overlap setting and records events only around stage 4
 * (far-field contraction) and stage 8 (pair kernel), the other stages reading -1.  Each
 * recorded event idles its stream for a few microseconds.  1 and 2 restart the averaging window;
 * other values are ANKH_ERR_INVALID_ARG. */
ankh_status ankh_set_timing(ankh_plan_t plan, int32_t enable);

/*
 * Energy terms of the last evaluation, copied to host memory (synchronises):
 * out[0] near field, [1] far field of the octree levels, [2] far periodic
 * images (root operator), [3] self, [4] background, [5] total, [6] total charge.
 */
ankh_status ankh_last_terms(ankh_plan_t plan, double *out_host);

/*
 * Copies the leaf-level modified charges of the last evaluation to host
 * memory: out_host receives 8^E * L^3 doubles, leaf (i, j, k) at row
 * (i * 2^E + j) * 2^E + k, node (a, b, c) at column (a * L + b) * L + c.
 * `count` is the capacity of out_host in doubles.
 */
ankh_status ankh_leaf_multipoles(ankh_plan_t plan, double *out_host, int64_t count);

/* Frees the plan (waits for its stream first). NULL is ignored. */
void ankh_destroy(ankh_plan_t plan);

/* Static description of a status code. */
const char *ankh_status_string(ankh_status s);

#ifdef __cplusplus
}
#endif

#endif /* ANKH_H */
