/*
 * Classical Ewald summation for periodic point multipoles in a cubic box.
 *
 * TEST INFRASTRUCTURE ONLY.  This is the CPU FP64 oracle the GPU path is
 * checked against.  Only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg load it.  It shares no code, tables or headers with the
 * GPU library.
 *
 * What it computes: the tin-foil periodic energy of eq. (1) of the paper,
 *   E = 1/2 sum_t sum_x sum_y D_x D_y 1/|x - y + t|,
 *   D_u = q_u + mu_u . grad + Theta_u : grad grad (+ Omega_u : grad grad grad),
 * (the x = y, t = 0 term omitted), split as in the Ewald summation of the
 * ANKH-FMM section (real + reciprocal + self, plus the neutralising
 * background for non-neutral cells).  The printed reciprocal term and its
 * multipole factors are garbled in the paper; this file uses the textbook
 * form:
 *   E_rec = (2 pi / V) sum_{k != 0} exp(-k^2 / (4 a^2)) / k^2 |S(k)|^2,
 *   S(k)  = sum_j (q_j + i mu_j.k - Theta_j : k k) exp(i k . r_j).
 * Self term (eq. for E_self, valid for traceless Theta):
 *   E_self = -(a / sqrt(pi)) sum (q^2 + 2a^2/3 |mu|^2 + 8a^4/5 Theta:Theta).
 * Octupoles (the higher multipole order the paper's operator D admits): Omega
 * is the full symmetric traceless rank-3 tensor used literally in
 * Omega : grad grad grad; its reciprocal factor is -i Omega : k k k and its
 * self term -(a / sqrt(pi)) 48 a^6 / 7 Omega:Omega.  In general the moment of
 * rank l contributes (2 a^2)^l l! / (2 l + 1) M:M: the Taylor term of order 2l
 * of erf(a r)/r at r = 0, of which only the l! index pairings across the two
 * traceless tensors survive.
 * Background: E_bg = -pi Q^2 / (2 V a^2), Q = sum q.
 * Theta is the full symmetric tensor used literally in Theta : grad grad.
 *
 * Real space: the pair operator (q_i + mu_i.d + Th_i:dd)(q_j - mu_j.d + Th_j:dd)
 * applied to f(r) = erfc(a r)/r, r = x_i - x_j - shift, d = d/dr.  Cartesian
 * derivative tensors of the radial f are built from the radial functions
 *   B_0 = f,  B_n = [(2n-1) B_{n-1} + (2a^2)^n exp(-a^2 r^2)/(a sqrt(pi))] / r^2
 * with the general rule
 *   T_{i1..in} = sum_k (-1)^{n-k} B_{n-k} sum_{k disjoint index pairs}
 *                prod(delta over the pairs) prod(r over the unpaired indices),
 * enumerated explicitly for every index tuple (no hand-expanded formulas).
 *
 * Forces are -dE/dx_i; fields are dE/dmu_i; oracle_ewald_moments gives
 * dE/dq_i and the traceless part of dE/dTheta_i.  Sums are gathered per atom in
 * a fixed order and reduced serially, so results are run-to-run identical
 * for a given thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define MAXRANK 7         /* rank of the octupole-octupole force tensor */
#define NTUPLE5 2187      /* 3^MAXRANK index tuples */

/* ---- derivative-tensor term tables ----------------------------------- */
typedef struct {
    int k;          /* number of delta pairs */
    int coef;       /* multiplicity of this (k, monomial) */
    int p[3];       /* powers of r_x, r_y, r_z */
} tterm;

typedef struct {
    int nterms;
    tterm t[16];
} tentry;

static tentry g_tab[MAXRANK + 1][NTUPLE5];
static int g_tab_ready = 0;

static int ipow3(int n) { int r = 1; while (n-- > 0) r *= 3; return r; }

static void enum_valid(const int *idx, int n, int *used, int start, int k, tentry *e)
{
    int p[3] = {0, 0, 0};
    for (int i = 0; i < n; i++) if (!used[i]) p[idx[i]]++;
    int found = 0;
    for (int t = 0; t < e->nterms; t++) {
        tterm *tt = &e->t[t];
        if (tt->k == k && tt->p[0] == p[0] && tt->p[1] == p[1] && tt->p[2] == p[2]) {
            tt->coef++; found = 1; break;
        }
    }
    if (!found) {
        tterm *tt = &e->t[e->nterms++];
        tt->k = k; tt->coef = 1; tt->p[0] = p[0]; tt->p[1] = p[1]; tt->p[2] = p[2];
    }
    for (int i = start; i < n; i++) {
        if (used[i]) continue;
        for (int j = i + 1; j < n; j++) {
            if (used[j] || idx[i] != idx[j]) continue;   /* delta_{ij} = 0 kills the term */
            used[i] = used[j] = 1;
            enum_valid(idx, n, used, i + 1, k + 1, e);
            used[i] = used[j] = 0;
        }
    }
}

static void build_tables_valid(void)
{
    if (g_tab_ready) return;
    for (int n = 0; n <= MAXRANK; n++) {
        int nt = ipow3(n);
        for (int t = 0; t < nt; t++) {
            int idx[MAXRANK], used[MAXRANK] = {0};
            int v = t;
            for (int i = n - 1; i >= 0; i--) { idx[i] = v % 3; v /= 3; }
            tentry *e = &g_tab[n][t];
            e->nterms = 0;
            enum_valid(idx, n, used, 0, 0, e);
        }
    }
    g_tab_ready = 1;
}

/* Every unordered set of disjoint pairs must be counted once.  enum_valid
 * adds pairs in increasing order of their first element, which generates each
 * set exactly once. */

/* radial functions B_0..B_nmax of erfc(a r)/r */
static void radial(double r2, double a, int nmax, double *B)
{
    double r = sqrt(r2);
    B[0] = erfc(a * r) / r;
    double ex = exp(-a * a * r2) / (a * sqrt(M_PI));
    double pw = 1.0;
    for (int n = 1; n <= nmax; n++) {
        pw *= 2.0 * a * a;
        B[n] = ((2 * n - 1) * B[n - 1] + pw * ex) / r2;
    }
}

/* T[n][tuple] for n = 0..nmax */
static void dtensors(const double r[3], const double *B, int nmax, double T[MAXRANK + 1][NTUPLE5])
{
    double pw[3][MAXRANK + 1];
    for (int c = 0; c < 3; c++) {
        pw[c][0] = 1.0;
        for (int i = 1; i <= MAXRANK; i++) pw[c][i] = pw[c][i - 1] * r[c];
    }
    for (int n = 0; n <= nmax; n++) {
        int nt = ipow3(n);
        for (int t = 0; t < nt; t++) {
            const tentry *e = &g_tab[n][t];
            double s = 0.0;
            for (int m = 0; m < e->nterms; m++) {
                const tterm *tt = &e->t[m];
                double sign = ((n - tt->k) & 1) ? -1.0 : 1.0;
                s += sign * tt->coef * B[n - tt->k] * pw[0][tt->p[0]] * pw[1][tt->p[1]] * pw[2][tt->p[2]];
            }
            T[n][t] = s;
        }
    }
}

/* full symmetric 3x3 from (xx, xy, xz, yy, yz, zz) */
static void theta_full(const double *th, double Th[9])
{
    Th[0] = th[0]; Th[1] = th[1]; Th[2] = th[2];
    Th[3] = th[1]; Th[4] = th[3]; Th[5] = th[4];
    Th[6] = th[2]; Th[7] = th[4]; Th[8] = th[5];
}

/*
 * Pair functional  Phi(T0..T4) = q_i q_j T
 *    + q_i (-mu_j.T1 + Th_j:T2) + mu_i.(q_j T1 - T2 mu_j + T3:Th_j)
 *    + Th_i:(q_j T2 - T3 mu_j + T4:Th_j)
 * evaluated on tensors that may carry one extra trailing index `e` (the
 * gradient), selected by stride: element [tuple] of rank n is read at
 * Tn[tuple * 3 + e] when grad >= 0.
 */
static double pair_phi(double T[MAXRANK + 1][NTUPLE5], int grad,
                       double qi, const double *mi, const double *Ti,
                       double qj, const double *mj, const double *Tj)
{
#define TT(n, t) (grad < 0 ? T[(n)][(t)] : T[(n) + 1][(t) * 3 + grad])
    double e = qi * qj * TT(0, 0);
    for (int a = 0; a < 3; a++) {
        double t1 = TT(1, a);
        if (mj) e -= qi * mj[a] * t1;
        if (mi) e += mi[a] * qj * t1;
    }
    for (int a = 0; a < 3; a++) for (int b = 0; b < 3; b++) {
        double t2 = TT(2, a * 3 + b);
        if (Tj) e += qi * Tj[a * 3 + b] * t2;
        if (Ti) e += Ti[a * 3 + b] * qj * t2;
        if (mi && mj) e -= mi[a] * t2 * mj[b];
    }
    if ((mi && Tj) || (Ti && mj)) {
        for (int a = 0; a < 3; a++) for (int b = 0; b < 3; b++) for (int c = 0; c < 3; c++) {
            double t3 = TT(3, (a * 3 + b) * 3 + c);
            if (mi && Tj) e += mi[a] * t3 * Tj[b * 3 + c];
            if (Ti && mj) e -= Ti[a * 3 + b] * t3 * mj[c];
        }
    }
    if (Ti && Tj) {
        for (int a = 0; a < 3; a++) for (int b = 0; b < 3; b++)
            for (int c = 0; c < 3; c++) for (int d = 0; d < 3; d++)
                e += Ti[a * 3 + b] * TT(4, ((a * 3 + b) * 3 + c) * 3 + d) * Tj[c * 3 + d];
    }
#undef TT
    return e;
}

/* field on i: dPhi/dmu_i = q_j T1 - T2 mu_j + T3:Th_j */
static void pair_field(double T[MAXRANK + 1][NTUPLE5], double qj, const double *mj, const double *Tj, double f[3])
{
    for (int a = 0; a < 3; a++) {
        double s = qj * T[1][a];
        if (mj) for (int b = 0; b < 3; b++) s -= T[2][a * 3 + b] * mj[b];
        if (Tj) for (int b = 0; b < 3; b++) for (int c = 0; c < 3; c++) s += T[3][(a * 3 + b) * 3 + c] * Tj[b * 3 + c];
        f[a] = s;
    }
}

/* pairwise (cascade) sum, deterministic */
static double psum(const double *x, int64_t n)
{
    if (n <= 16) { double s = 0; for (int64_t i = 0; i < n; i++) s += x[i]; return s; }
    int64_t h = n / 2;
    return psum(x, h) + psum(x + h, n - h);
}

typedef struct {
    int64_t n;
    double L, a, rc;
    int kmax;
    const double *q, *mu;
    double *pos;      /* wrapped copy */
    double *Th;       /* full 3x3 per atom, or NULL */
    double *Om;       /* full 3x3x3 per atom, or NULL */
    int order;        /* highest multipole present */
    /* cell list */
    int nc, R;
    int *cell_start, *cell_atoms;
} ctx_t;

/* full symmetric 3x3x3 from (xxx, xxy, xxz, xyy, xyz, xzz, yyy, yyz, yzz, zzz) */
static void omega_full(const double *om, double Om[27])
{
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++)
            for (int c = 0; c < 3; c++) {
                int n[3] = {0, 0, 0};
                n[a]++; n[b]++; n[c]++;
                /* index of the sorted triple in the stored order */
                int k;
                if (n[0] == 3) k = 0;
                else if (n[0] == 2) k = n[1] == 1 ? 1 : 2;
                else if (n[0] == 1) k = n[1] == 2 ? 3 : (n[1] == 1 ? 4 : 5);
                else k = n[1] == 3 ? 6 : (n[1] == 2 ? 7 : (n[1] == 1 ? 8 : 9));
                Om[(a * 3 + b) * 3 + c] = om[k];
            }
}

static void ctx_init(ctx_t *c, int64_t n, const double *pos, const double *q, const double *mu,
                     const double *theta, double L, double a, double rc, int kmax)
{
    build_tables_valid();
    c->n = n; c->L = L; c->a = a; c->rc = rc; c->kmax = kmax; c->q = q; c->mu = mu;
    c->pos = (double *)malloc(sizeof(double) * 3 * (n > 0 ? n : 1));
    for (int64_t i = 0; i < 3 * n; i++) {
        double x = pos[i];
        x -= L * floor((x + 0.5 * L) / L);
        if (x >= 0.5 * L) x -= L;
        c->pos[i] = x;
    }
    c->Th = NULL;
    if (theta) {
        c->Th = (double *)malloc(sizeof(double) * 9 * (n > 0 ? n : 1));
        for (int64_t i = 0; i < n; i++) theta_full(theta + 6 * i, c->Th + 9 * i);
    }
    c->Om = NULL;
    c->order = theta ? 2 : (mu ? 1 : 0);
    int nc = (int)floor(L / rc);
    if (nc < 1) nc = 1;
    if (nc > 64) nc = 64;
    c->nc = nc;
    double wc = L / nc;
    c->R = (int)ceil(rc / wc - 1e-12);
    int ncell = nc * nc * nc;
    int *cnt = (int *)calloc(ncell + 1, sizeof(int));
    int *cid = (int *)malloc(sizeof(int) * (n > 0 ? n : 1));
    for (int64_t i = 0; i < n; i++) {
        int ix[3];
        for (int d = 0; d < 3; d++) {
            int v = (int)floor((c->pos[3 * i + d] + 0.5 * L) / wc);
            if (v < 0) v = 0;
            if (v >= nc) v = nc - 1;
            ix[d] = v;
        }
        cid[i] = (ix[0] * nc + ix[1]) * nc + ix[2];
        cnt[cid[i] + 1]++;
    }
    for (int i = 0; i < ncell; i++) cnt[i + 1] += cnt[i];
    c->cell_start = cnt;
    c->cell_atoms = (int *)malloc(sizeof(int) * (n > 0 ? n : 1));
    int *fill = (int *)malloc(sizeof(int) * ncell);
    memcpy(fill, cnt, sizeof(int) * ncell);
    for (int64_t i = 0; i < n; i++) c->cell_atoms[fill[cid[i]]++] = (int)i;
    free(fill);
    free(cid);
}

static void ctx_set_omega(ctx_t *c, const double *omega)
{
    if (!omega) return;
    c->Om = (double *)malloc(sizeof(double) * 27 * (c->n > 0 ? c->n : 1));
    for (int64_t i = 0; i < c->n; i++) omega_full(omega + 10 * i, c->Om + 27 * i);
    c->order = 3;
}

static void ctx_free(ctx_t *c)
{
    free(c->pos); free(c->Th); free(c->Om); free(c->cell_start); free(c->cell_atoms);
}

/*
 * The pair functional on full tensors of every rank present, for moments up to
 * octupoles:  Phi = sum_{a,b} (-1)^b M_i^a : T^(a+b) : M_j^b,  M^0 = q, M^1 = mu,
 * M^2 = Theta, M^3 = Omega (each contracted with the first a / last b indices;
 * the sign because grad_{x_j} = -grad_r).  grad >= 0 selects the component of the
 * gradient (rank + 1).  The explicit functional above is the same sum for q, mu
 * and Theta.
 */
static double pair_phi_gen(double T[MAXRANK + 1][NTUPLE5], int grad, const double *Mi[4], const double *Mj[4])
{
    double e = 0.0;
    for (int a = 0; a < 4; a++) {
        if (!Mi[a]) continue;
        const int na = ipow3(a);
        for (int b = 0; b < 4; b++) {
            if (!Mj[b]) continue;
            const int nb = ipow3(b), n = a + b;
            const double sign = (b & 1) ? -1.0 : 1.0;
            double s = 0.0;
            for (int I = 0; I < na; I++) {
                const double mi = Mi[a][I];
                if (mi == 0.0) continue;
                for (int J = 0; J < nb; J++) {
                    const int t = I * nb + J;
                    s += mi * Mj[b][J] * (grad < 0 ? T[n][t] : T[n + 1][t * 3 + grad]);
                }
            }
            e += sign * s;
        }
    }
    return e;
}

/* field on i: dPhi/dmu_i = sum_b (-1)^b T^(1+b) : M_j^b */
static void pair_field_gen(double T[MAXRANK + 1][NTUPLE5], const double *Mj[4], double f[3])
{
    for (int e = 0; e < 3; e++) {
        double s = 0.0;
        for (int b = 0; b < 4; b++) {
            if (!Mj[b]) continue;
            const int nb = ipow3(b);
            const double sign = (b & 1) ? -1.0 : 1.0;
            for (int J = 0; J < nb; J++) s += sign * Mj[b][J] * T[1 + b][e * nb + J];
        }
        f[e] = s;
    }
}

static void moments_of(const ctx_t *c, int64_t i, const double *M[4])
{
    M[0] = c->q + i;
    M[1] = c->mu ? c->mu + 3 * i : NULL;
    M[2] = c->Th ? c->Th + 9 * i : NULL;
    M[3] = c->Om ? c->Om + 27 * i : NULL;
}

/* real-space sum for atom i: energy contribution (1/2 sum over its pairs),
 * force, field */
static void real_atom(const ctx_t *c, int64_t i, int want_grad, double *ei, double fi[3], double gi[3])
{
    const double L = c->L, wc = L / c->nc;
    const int nc = c->nc, R = c->R;
    const double *xi = c->pos + 3 * i;
    const double *mi = c->mu ? c->mu + 3 * i : NULL;
    const double *Ti = c->Th ? c->Th + 9 * i : NULL;
    const double qi = c->q[i];
    int nmax = 2 * c->order + (want_grad ? 1 : 0);
    if (nmax < 1) nmax = 1;
    double B[MAXRANK + 2];
    static __thread double T[MAXRANK + 1][NTUPLE5];
    double e = 0, f[3] = {0, 0, 0}, g[3] = {0, 0, 0};
    int ci[3];
    for (int d = 0; d < 3; d++) {
        int v = (int)floor((xi[d] + 0.5 * L) / wc);
        if (v < 0) v = 0;
        if (v >= nc) v = nc - 1;
        ci[d] = v;
    }
    const double rc2 = c->rc * c->rc;
    for (int dx = -R; dx <= R; dx++)
    for (int dy = -R; dy <= R; dy++)
    for (int dz = -R; dz <= R; dz++) {
        int u[3] = {ci[0] + dx, ci[1] + dy, ci[2] + dz};
        int w[3];
        double sh[3];
        for (int d = 0; d < 3; d++) {
            int m = (int)floor((double)u[d] / nc);
            w[d] = u[d] - m * nc;
            sh[d] = m * L;
        }
        int cell = (w[0] * nc + w[1]) * nc + w[2];
        for (int p = c->cell_start[cell]; p < c->cell_start[cell + 1]; p++) {
            int j = c->cell_atoms[p];
            double r[3];
            for (int d = 0; d < 3; d++) r[d] = xi[d] - (c->pos[3 * j + d] + sh[d]);
            double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
            if (r2 >= rc2) continue;
            if (j == i && sh[0] == 0 && sh[1] == 0 && sh[2] == 0) continue;
            radial(r2, c->a, nmax, B);
            dtensors(r, B, nmax, T);
            if (c->Om) {
                const double *Mi[4], *Mj[4];
                moments_of(c, i, Mi);
                moments_of(c, j, Mj);
                e += 0.5 * pair_phi_gen(T, -1, Mi, Mj);
                if (want_grad) {
                    for (int d = 0; d < 3; d++) f[d] -= pair_phi_gen(T, d, Mi, Mj);
                    if (mi) {
                        double h[3];
                        pair_field_gen(T, Mj, h);
                        for (int d = 0; d < 3; d++) g[d] += h[d];
                    }
                }
                continue;
            }
            const double *mj = c->mu ? c->mu + 3 * j : NULL;
            const double *Tj = c->Th ? c->Th + 9 * j : NULL;
            e += 0.5 * pair_phi(T, -1, qi, mi, Ti, c->q[j], mj, Tj);
            if (want_grad) {
                for (int d = 0; d < 3; d++) f[d] -= pair_phi(T, d, qi, mi, Ti, c->q[j], mj, Tj);
                if (mi) {
                    double h[3];
                    pair_field(T, c->q[j], mj, Tj, h);
                    for (int d = 0; d < 3; d++) g[d] += h[d];
                }
            }
        }
    }
    *ei = e;
    if (fi) for (int d = 0; d < 3; d++) fi[d] = f[d];
    if (gi) for (int d = 0; d < 3; d++) gi[d] = g[d];
}

/* ---- reciprocal space ------------------------------------------------ */
/* Om : k k k */
static double om_kkk(const double *Om, const double k[3])
{
    double s = 0.0;
    for (int a = 0; a < 3; a++) for (int b = 0; b < 3; b++) for (int c = 0; c < 3; c++)
        s += Om[(a * 3 + b) * 3 + c] * k[a] * k[b] * k[c];
    return s;
}

typedef struct {
    int nk;
    int *m;             /* [nk][3], half space */
    double *g;          /* exp(-k^2/4a^2)/k^2 */
    double *Sre, *Sim;  /* structure factors */
    double *ex_re, *ex_im; /* [n][3][2kmax+1] per-axis phases */
} rec_t;

static void rec_build(const ctx_t *c, rec_t *rc)
{
    const int K = c->kmax, W = 2 * K + 1;
    const double L = c->L, a = c->a;
    const int64_t n = c->n;
    /* half-space list: m > 0 lexicographically */
    int cap = W * W * W;
    rc->m = (int *)malloc(sizeof(int) * 3 * cap);
    rc->g = (double *)malloc(sizeof(double) * cap);
    int nk = 0;
    for (int mx = 0; mx <= K; mx++)
    for (int my = -K; my <= K; my++)
    for (int mz = -K; mz <= K; mz++) {
        if (mx == 0 && (my < 0 || (my == 0 && mz <= 0))) continue;
        if (mx * mx + my * my + mz * mz > K * K) continue;
        double kx = 2 * M_PI * mx / L, ky = 2 * M_PI * my / L, kz = 2 * M_PI * mz / L;
        double k2 = kx * kx + ky * ky + kz * kz;
        rc->m[3 * nk] = mx; rc->m[3 * nk + 1] = my; rc->m[3 * nk + 2] = mz;
        rc->g[nk] = exp(-k2 / (4 * a * a)) / k2;
        nk++;
    }
    rc->nk = nk;
    rc->ex_re = (double *)malloc(sizeof(double) * (size_t)n * 3 * W + 8);
    rc->ex_im = (double *)malloc(sizeof(double) * (size_t)n * 3 * W + 8);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++)
        for (int d = 0; d < 3; d++)
            for (int m = -K; m <= K; m++) {
                double ph = 2 * M_PI * m * c->pos[3 * i + d] / L;
                rc->ex_re[((size_t)i * 3 + d) * W + m + K] = cos(ph);
                rc->ex_im[((size_t)i * 3 + d) * W + m + K] = sin(ph);
            }
    rc->Sre = (double *)calloc(nk + 1, sizeof(double));
    rc->Sim = (double *)calloc(nk + 1, sizeof(double));
#pragma omp parallel for schedule(dynamic, 16)
    for (int t = 0; t < nk; t++) {
        const int *m = rc->m + 3 * t;
        double k[3] = {2 * M_PI * m[0] / L, 2 * M_PI * m[1] / L, 2 * M_PI * m[2] / L};
        double sre = 0, sim = 0;
        for (int64_t i = 0; i < n; i++) {
            /* a_i = q - Th:kk + i (mu.k - Om:kkk) */
            double are = c->q[i], aim = 0;
            if (c->mu) aim = c->mu[3 * i] * k[0] + c->mu[3 * i + 1] * k[1] + c->mu[3 * i + 2] * k[2];
            if (c->Th) {
                const double *T = c->Th + 9 * i;
                for (int x = 0; x < 3; x++) for (int y = 0; y < 3; y++) are -= T[3 * x + y] * k[x] * k[y];
            }
            if (c->Om) aim -= om_kkk(c->Om + 27 * i, k);
            double pr = 1, pi = 0;
            for (int d = 0; d < 3; d++) {
                double er = rc->ex_re[((size_t)i * 3 + d) * W + m[d] + K];
                double ei = rc->ex_im[((size_t)i * 3 + d) * W + m[d] + K];
                double nr = pr * er - pi * ei, ni = pr * ei + pi * er;
                pr = nr; pi = ni;
            }
            sre += are * pr - aim * pi;
            sim += are * pi + aim * pr;
        }
        rc->Sre[t] = sre; rc->Sim[t] = sim;
    }
}

static void rec_free(rec_t *rc)
{
    free(rc->m); free(rc->g); free(rc->Sre); free(rc->Sim); free(rc->ex_re); free(rc->ex_im);
}

static double rec_energy(const ctx_t *c, const rec_t *rc)
{
    double V = c->L * c->L * c->L;
    double *terms = (double *)malloc(sizeof(double) * (rc->nk + 1));
    for (int t = 0; t < rc->nk; t++) terms[t] = rc->g[t] * (rc->Sre[t] * rc->Sre[t] + rc->Sim[t] * rc->Sim[t]);
    /* half space: each +-k pair once, times 2 */
    double e = 2.0 * (2 * M_PI / V) * psum(terms, rc->nk);
    free(terms);
    return e;
}

/* dE_rec/dr_i and dE_rec/dmu_i for one atom.
 * Over the full k set: dE/dr_i = (4 pi / V) sum_k g Re[i k a_i e^{ik.r_i} S*],
 * dE/dmu_i = (4 pi / V) sum_k g Re[i k e^{ik.r_i} S*]; the half-space list
 * carries each +-k pair once, so the factor is 8 pi / V. */
static void rec_atom(const ctx_t *c, const rec_t *rc, int64_t i, double dr[3], double dmu[3])
{
    const int K = c->kmax, W = 2 * K + 1;
    const double L = c->L, V = L * L * L;
    double sr[3] = {0, 0, 0}, sm[3] = {0, 0, 0};
    for (int t = 0; t < rc->nk; t++) {
        const int *m = rc->m + 3 * t;
        double k[3] = {2 * M_PI * m[0] / L, 2 * M_PI * m[1] / L, 2 * M_PI * m[2] / L};
        double are = c->q[i], aim = 0;
        if (c->mu) aim = c->mu[3 * i] * k[0] + c->mu[3 * i + 1] * k[1] + c->mu[3 * i + 2] * k[2];
        if (c->Th) {
            const double *T = c->Th + 9 * i;
            for (int x = 0; x < 3; x++) for (int y = 0; y < 3; y++) are -= T[3 * x + y] * k[x] * k[y];
        }
        if (c->Om) aim -= om_kkk(c->Om + 27 * i, k);
        double pr = 1, pi = 0;
        for (int d = 0; d < 3; d++) {
            double er = rc->ex_re[((size_t)i * 3 + d) * W + m[d] + K];
            double ei = rc->ex_im[((size_t)i * 3 + d) * W + m[d] + K];
            double nr = pr * er - pi * ei, ni = pr * ei + pi * er;
            pr = nr; pi = ni;
        }
        /* w = e^{ik.r} * conj(S) */
        double wr = pr * rc->Sre[t] + pi * rc->Sim[t];
        double wi = pi * rc->Sre[t] - pr * rc->Sim[t];
        /* Re[i * a * w] = -(are*wi + aim*wr) ; Re[i * w] = -wi */
        double ra = -(are * wi + aim * wr);
        double rw = -wi;
        for (int d = 0; d < 3; d++) {
            sr[d] += rc->g[t] * k[d] * ra;
            sm[d] += rc->g[t] * k[d] * rw;
        }
    }
    for (int d = 0; d < 3; d++) {
        dr[d] = (8 * M_PI / V) * sr[d];
        dmu[d] = (8 * M_PI / V) * sm[d];
    }
}

static void self_terms(const ctx_t *c, int64_t i, double *e, double g[3])
{
    const double a = c->a, sp = sqrt(M_PI);
    double s = c->q[i] * c->q[i];
    if (c->mu) {
        const double *m = c->mu + 3 * i;
        s += (2 * a * a / 3) * (m[0] * m[0] + m[1] * m[1] + m[2] * m[2]);
        for (int d = 0; d < 3; d++) g[d] = -(4 * a * a * a / (3 * sp)) * m[d];
    } else {
        g[0] = g[1] = g[2] = 0;
    }
    if (c->Th) {
        const double *T = c->Th + 9 * i;
        double tt = 0;
        for (int x = 0; x < 9; x++) tt += T[x] * T[x];
        s += (8 * a * a * a * a / 5) * tt;
    }
    if (c->Om) {
        const double *O = c->Om + 27 * i;
        double oo = 0;
        for (int x = 0; x < 27; x++) oo += O[x] * O[x];
        s += (48 * a * a * a * a * a * a / 7) * oo;
    }
    *e = -(a / sp) * s;
}

/*
 * Full evaluation.
 * energy_out[0..4] = real, reciprocal, self, background, total.
 * forces, dEdmu: [n][3] or NULL.  Returns 0 on success, negative on bad input.
 */
int oracle_ewald_o3(int64_t n, const double *pos, const double *q, const double *mu, const double *theta,
                    const double *omega, double edge, double alpha, double rcut, int kmax, int nthreads,
                    double *energy_out, double *forces, double *dEdmu)
{
    if (n <= 0 || !pos || !q || !energy_out || edge <= 0 || alpha <= 0 || rcut <= 0 || kmax < 0) return -1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    ctx_t c;
    ctx_init(&c, n, pos, q, mu, theta, edge, alpha, rcut, kmax);
    ctx_set_omega(&c, omega);
    const int want_grad = (forces || dEdmu) ? 1 : 0;
    double *ereal = (double *)malloc(sizeof(double) * n);
    double *eself = (double *)malloc(sizeof(double) * n);
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t i = 0; i < n; i++) {
        double f[3], g[3], gs[3];
        real_atom(&c, i, want_grad, &ereal[i], f, g);
        self_terms(&c, i, &eself[i], gs);
        if (forces) for (int d = 0; d < 3; d++) forces[3 * i + d] = f[d];
        if (dEdmu) for (int d = 0; d < 3; d++) dEdmu[3 * i + d] = g[d] + gs[d];
    }
    rec_t rc;
    rec_build(&c, &rc);
    double erec = rec_energy(&c, &rc);
    if (want_grad) {
#pragma omp parallel for schedule(dynamic, 8)
        for (int64_t i = 0; i < n; i++) {
            double dr[3], dm[3];
            rec_atom(&c, &rc, i, dr, dm);
            if (forces) for (int d = 0; d < 3; d++) forces[3 * i + d] -= dr[d];
            if (dEdmu && mu) for (int d = 0; d < 3; d++) dEdmu[3 * i + d] += dm[d];
        }
    }
    if (dEdmu && !mu) memset(dEdmu, 0, sizeof(double) * 3 * n);
    double Q = psum(q, n);
    double V = edge * edge * edge;
    double er = psum(ereal, n), es = psum(eself, n);
    double eb = -M_PI * Q * Q / (2 * V * alpha * alpha);
    energy_out[0] = er;
    energy_out[1] = erec;
    energy_out[2] = es;
    energy_out[3] = eb;
    energy_out[4] = er + erec + es + eb;
    free(ereal); free(eself);
    rec_free(&rc);
    ctx_free(&c);
    return 0;
}

/* the same without octupoles */
int oracle_ewald(int64_t n, const double *pos, const double *q, const double *mu, const double *theta,
                 double edge, double alpha, double rcut, int kmax, int nthreads,
                 double *energy_out, double *forces, double *dEdmu)
{
    return oracle_ewald_o3(n, pos, q, mu, theta, NULL, edge, alpha, rcut, kmax, nthreads, energy_out, forces,
                           dEdmu);
}

/* ---- derivatives in the charges and quadrupoles ------------------------ */
/* dE/dq_i and dE/dTheta_i (full symmetric 3x3, before projection) of the
 * real-space sum: d/dq_i of the pair functional is q_j T - mu_j.T1 + Th_j:T2,
 * d/dTh_i,ab is q_j T2_ab - (T3 mu_j)_ab + (T4:Th_j)_ab. */
static void real_moments(const ctx_t *c, int64_t i, double *phi, double G[9])
{
    const double L = c->L, wc = L / c->nc;
    const int nc = c->nc, R = c->R;
    const double *xi = c->pos + 3 * i;
    const int nmax = 2 + c->order;   /* T2 with q_j, T3 with mu_j, T4 with Theta_j */
    double B[MAXRANK + 2];
    static __thread double T[MAXRANK + 1][NTUPLE5];
    double p = 0, g[9] = {0};
    int ci[3];
    for (int d = 0; d < 3; d++) {
        int v = (int)floor((xi[d] + 0.5 * L) / wc);
        if (v < 0) v = 0;
        if (v >= nc) v = nc - 1;
        ci[d] = v;
    }
    const double rc2 = c->rc * c->rc;
    for (int dx = -R; dx <= R; dx++)
    for (int dy = -R; dy <= R; dy++)
    for (int dz = -R; dz <= R; dz++) {
        int u[3] = {ci[0] + dx, ci[1] + dy, ci[2] + dz};
        int w[3];
        double sh[3];
        for (int d = 0; d < 3; d++) {
            int m = (int)floor((double)u[d] / nc);
            w[d] = u[d] - m * nc;
            sh[d] = m * L;
        }
        int cell = (w[0] * nc + w[1]) * nc + w[2];
        for (int q = c->cell_start[cell]; q < c->cell_start[cell + 1]; q++) {
            int j = c->cell_atoms[q];
            double r[3];
            for (int d = 0; d < 3; d++) r[d] = xi[d] - (c->pos[3 * j + d] + sh[d]);
            double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
            if (r2 >= rc2) continue;
            if (j == i && sh[0] == 0 && sh[1] == 0 && sh[2] == 0) continue;
            radial(r2, c->a, nmax, B);
            dtensors(r, B, nmax, T);
            const double qj = c->q[j];
            const double *mj = c->mu ? c->mu + 3 * j : NULL;
            const double *Tj = c->Th ? c->Th + 9 * j : NULL;
            p += qj * T[0][0];
            if (mj) for (int a = 0; a < 3; a++) p -= mj[a] * T[1][a];
            if (Tj) for (int a = 0; a < 9; a++) p += Tj[a] * T[2][a];
            for (int ab = 0; ab < 9; ab++) {
                double v = qj * T[2][ab];
                if (mj) for (int cc = 0; cc < 3; cc++) v -= T[3][ab * 3 + cc] * mj[cc];
                if (Tj) for (int cd = 0; cd < 9; cd++) v += T[4][ab * 9 + cd] * Tj[cd];
                g[ab] += v;
            }
        }
    }
    *phi = p;
    for (int ab = 0; ab < 9; ab++) G[ab] = g[ab];
}

/* reciprocal part: with w = exp(i k.r_i) conj(S(k)) over the half-space list,
 * dE/dq_i = (8 pi / V) sum g Re w and dE/dTh_i,ab = -(8 pi / V) sum g k_a k_b Re w */
static void rec_moments(const ctx_t *c, const rec_t *rc, int64_t i, double *phi, double G[9])
{
    const int K = c->kmax, W = 2 * K + 1;
    const double L = c->L, V = L * L * L;
    double p = 0, g[9] = {0};
    for (int t = 0; t < rc->nk; t++) {
        const int *m = rc->m + 3 * t;
        double k[3] = {2 * M_PI * m[0] / L, 2 * M_PI * m[1] / L, 2 * M_PI * m[2] / L};
        double pr = 1, pi = 0;
        for (int d = 0; d < 3; d++) {
            double er = rc->ex_re[((size_t)i * 3 + d) * W + m[d] + K];
            double ei = rc->ex_im[((size_t)i * 3 + d) * W + m[d] + K];
            double nr = pr * er - pi * ei, ni = pr * ei + pi * er;
            pr = nr; pi = ni;
        }
        double wr = pr * rc->Sre[t] + pi * rc->Sim[t];
        p += rc->g[t] * wr;
        for (int a = 0; a < 3; a++) for (int b = 0; b < 3; b++) g[a * 3 + b] -= rc->g[t] * k[a] * k[b] * wr;
    }
    *phi = (8 * M_PI / V) * p;
    for (int ab = 0; ab < 9; ab++) G[ab] = (8 * M_PI / V) * g[ab];
}

/*
 * dE/dq [n] and dE/dTheta [n][6] (either may be NULL).  E is defined for
 * traceless Theta only, so the quadrupole derivative is the traceless part G
 * of the full-tensor derivative, reported per stored component: (xx, xy, xz,
 * yy, yz, zz) = (G_xx, 2 G_xy, 2 G_xz, G_yy, 2 G_yz, G_zz); then
 * sum dE/dTheta . dTheta = dE for every traceless change dTheta.
 */
int oracle_ewald_moments(int64_t n, const double *pos, const double *q, const double *mu, const double *theta,
                         double edge, double alpha, double rcut, int kmax, int nthreads,
                         double *dEdq, double *dEdth)
{
    if (n <= 0 || !pos || !q || edge <= 0 || alpha <= 0 || rcut <= 0 || kmax < 0) return -1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    ctx_t c;
    ctx_init(&c, n, pos, q, mu, theta, edge, alpha, rcut, kmax);
    rec_t rc;
    rec_build(&c, &rc);
    const double Q = psum(q, n), V = edge * edge * edge, a = alpha, sp = sqrt(M_PI);
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t i = 0; i < n; i++) {
        double p1, p2, G1[9], G2[9], G[9];
        real_moments(&c, i, &p1, G1);
        rec_moments(&c, &rc, i, &p2, G2);
        /* self: -(a/sqrt(pi)) (q^2 + 8a^4/5 Th:Th); background: -pi Q^2 / (2 V a^2) */
        const double ps = -(a / sp) * 2 * q[i] - M_PI * Q / (V * a * a);
        for (int ab = 0; ab < 9; ab++) {
            G[ab] = G1[ab] + G2[ab];
            if (c.Th) G[ab] += -(a / sp) * (8 * a * a * a * a / 5) * 2 * c.Th[9 * i + ab];
        }
        if (dEdq) dEdq[i] = p1 + p2 + ps;
        if (dEdth) {
            const double tr = (G[0] + G[4] + G[8]) / 3;
            double *o = dEdth + 6 * i;
            o[0] = G[0] - tr; o[1] = G[1] + G[3]; o[2] = G[2] + G[6];
            o[3] = G[4] - tr; o[4] = G[5] + G[7]; o[5] = G[8] - tr;
        }
    }
    rec_free(&rc);
    ctx_free(&c);
    return 0;
}

/*
 * Forces and fields on a subset of atoms `sel` (energy is not computed).
 * Cost: the reciprocal structure factors over all atoms plus the real-space
 * sums of the selected atoms only.
 */
int oracle_ewald_sites(int64_t n, const double *pos, const double *q, const double *mu, const double *theta,
                       double edge, double alpha, double rcut, int kmax, int nthreads,
                       int64_t nsel, const int64_t *sel, double *forces_sel, double *dEdmu_sel)
{
    if (n <= 0 || !pos || !q || nsel < 0 || (nsel > 0 && !sel) || edge <= 0 || alpha <= 0) return -1;
    for (int64_t s = 0; s < nsel; s++) if (sel[s] < 0 || sel[s] >= n) return -2;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    ctx_t c;
    ctx_init(&c, n, pos, q, mu, theta, edge, alpha, rcut, kmax);
    rec_t rc;
    rec_build(&c, &rc);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t s = 0; s < nsel; s++) {
        int64_t i = sel[s];
        double e, f[3], g[3], gs[3], dr[3], dm[3];
        real_atom(&c, i, 1, &e, f, g);
        self_terms(&c, i, &e, gs);
        rec_atom(&c, &rc, i, dr, dm);
        for (int d = 0; d < 3; d++) {
            if (forces_sel) forces_sel[3 * s + d] = f[d] - dr[d];
            if (dEdmu_sel) dEdmu_sel[3 * s + d] = mu ? g[d] + gs[d] + dm[d] : 0.0;
        }
    }
    rec_free(&rc);
    ctx_free(&c);
    return 0;
}

/* The derivative tensor of rank n at r for radial erfc(a r)/r, for tests of
 * the term tables against finite differences. out: 3^n values. */
int oracle_dtensor(const double r[3], double alpha, int n, double *out)
{
    if (n < 0 || n > MAXRANK) return -1;
    build_tables_valid();
    double B[MAXRANK + 2];
    static __thread double T[MAXRANK + 1][NTUPLE5];
    double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
    radial(r2, alpha, n < 1 ? 1 : n, B);
    dtensors(r, B, n, T);
    memcpy(out, T[n], sizeof(double) * ipow3(n));
    return 0;
}

/*
 * Near field of the interpolated Ewald method (the direct term N_real of the
 * ANKH reformulation): for every atom i, the pair operator on erfc(xi r)/r
 * summed over all atoms j of the 27 leaves adjacent to i's leaf in a perfect
 * octree of depth `depth` (periodic, each neighbour leaf with its image
 * shift), excluding j = i at zero shift.  Leaves: wrap x into [-L/2, L/2),
 * leaf index clamp(floor((x + L/2) / w), 0, 2^depth - 1), w = L / 2^depth.
 * eatom[i] = 1/2 sum_j pair energy; forces = -grad; dEdmu = field from the
 * pairs (no self term).  Any output may be NULL.
 */
int oracle_near_field_o3(int64_t n, const double *pos, const double *q, const double *mu, const double *theta,
                         const double *omega, double edge, double xi, int nside, int nthreads,
                         double *eatom, double *forces, double *dEdmu)
{
    /* nside: leaves per axis (2^depth for an octree; any count for the single-level ANKH-FFT grid) */
    if (n <= 0 || !pos || !q || edge <= 0 || xi <= 0 || nside < 1 || nside > 1024) return -1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    ctx_t c;
    /* a cell list whose cells are the leaves: nc = nside, R = 1, no cutoff */
    ctx_init(&c, n, pos, q, mu, theta, edge, xi, edge, 0);
    ctx_set_omega(&c, omega);
    free(c.cell_start); free(c.cell_atoms);
    const int nc = nside;
    const double w = edge / nc;
    const int ncell = nc * nc * nc;
    int *cnt = (int *)calloc(ncell + 1, sizeof(int));
    int *cid = (int *)malloc(sizeof(int) * n);
    for (int64_t i = 0; i < n; i++) {
        int ix[3];
        for (int d = 0; d < 3; d++) {
            int v = (int)floor((c.pos[3 * i + d] + 0.5 * edge) / w);
            if (v < 0) v = 0;
            if (v >= nc) v = nc - 1;
            ix[d] = v;
        }
        cid[i] = (ix[0] * nc + ix[1]) * nc + ix[2];
        cnt[cid[i] + 1]++;
    }
    for (int i = 0; i < ncell; i++) cnt[i + 1] += cnt[i];
    int *atoms = (int *)malloc(sizeof(int) * n);
    int *fill = (int *)malloc(sizeof(int) * ncell);
    memcpy(fill, cnt, sizeof(int) * ncell);
    for (int64_t i = 0; i < n; i++) atoms[fill[cid[i]]++] = (int)i;
    free(fill);
    const int want_grad = (forces || dEdmu) ? 1 : 0;
    int nmax = 2 * c.order + (want_grad ? 1 : 0);
    if (nmax < 1) nmax = 1;
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t i = 0; i < n; i++) {
        double B[MAXRANK + 2];
        static __thread double T[MAXRANK + 1][NTUPLE5];
        const double *xi_ = c.pos + 3 * i;
        const double *mi = c.mu ? c.mu + 3 * i : NULL;
        const double *Ti = c.Th ? c.Th + 9 * i : NULL;
        int li = cid[i];
        int ci[3] = {li / (nc * nc), (li / nc) % nc, li % nc};
        double e = 0, f[3] = {0, 0, 0}, g[3] = {0, 0, 0};
        for (int dx = -1; dx <= 1; dx++)
        for (int dy = -1; dy <= 1; dy++)
        for (int dz = -1; dz <= 1; dz++) {
            int u[3] = {ci[0] + dx, ci[1] + dy, ci[2] + dz}, wv[3];
            double sh[3];
            for (int d = 0; d < 3; d++) {
                int m = (int)floor((double)u[d] / nc);
                wv[d] = u[d] - m * nc;
                sh[d] = m * edge;
            }
            int cell = (wv[0] * nc + wv[1]) * nc + wv[2];
            for (int p = cnt[cell]; p < cnt[cell + 1]; p++) {
                int j = atoms[p];
                if (j == i && sh[0] == 0 && sh[1] == 0 && sh[2] == 0) continue;
                double r[3];
                for (int d = 0; d < 3; d++) r[d] = xi_[d] - (c.pos[3 * j + d] + sh[d]);
                double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
                radial(r2, xi, nmax, B);
                dtensors(r, B, nmax, T);
                if (c.Om) {
                    const double *Mi[4], *Mj[4];
                    moments_of(&c, i, Mi);
                    moments_of(&c, j, Mj);
                    e += 0.5 * pair_phi_gen(T, -1, Mi, Mj);
                    if (want_grad) {
                        for (int d = 0; d < 3; d++) f[d] -= pair_phi_gen(T, d, Mi, Mj);
                        if (mi) {
                            double h[3];
                            pair_field_gen(T, Mj, h);
                            for (int d = 0; d < 3; d++) g[d] += h[d];
                        }
                    }
                    continue;
                }
                const double *mj = c.mu ? c.mu + 3 * j : NULL;
                const double *Tj = c.Th ? c.Th + 9 * j : NULL;
                e += 0.5 * pair_phi(T, -1, q[i], mi, Ti, q[j], mj, Tj);
                if (want_grad) {
                    for (int d = 0; d < 3; d++) f[d] -= pair_phi(T, d, q[i], mi, Ti, q[j], mj, Tj);
                    if (mi) {
                        double h[3];
                        pair_field(T, q[j], mj, Tj, h);
                        for (int d = 0; d < 3; d++) g[d] += h[d];
                    }
                }
            }
        }
        if (eatom) eatom[i] = e;
        if (forces) for (int d = 0; d < 3; d++) forces[3 * i + d] = f[d];
        if (dEdmu) for (int d = 0; d < 3; d++) dEdmu[3 * i + d] = g[d];
    }
    free(cnt); free(cid); free(atoms);
    c.cell_start = NULL; c.cell_atoms = NULL;
    ctx_free(&c);
    return 0;
}

/* the same without octupoles */
int oracle_near_field(int64_t n, const double *pos, const double *q, const double *mu, const double *theta,
                      double edge, double xi, int nside, int nthreads,
                      double *eatom, double *forces, double *dEdmu)
{
    return oracle_near_field_o3(n, pos, q, mu, theta, NULL, edge, xi, nside, nthreads, eatom, forces, dEdmu);
}
