"""The C oracle under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

A small C driver, compiled together with oracle/ewald.c with
-fsanitize=address,undefined and no recovery, runs every exported entry point
(energy + forces + fields, selected sites, charge / quadrupole derivatives,
derivative tensors, the near-field pair sums) on two inputs and checks values
that the mathematics fixes: the NaCl Madelung energy of the conventional cell,
zero force on every ion of that perfect crystal, independence of the Ewald
splitting parameter for a random charge / dipole / quadrupole cell, the
energy as half the sum of each moment times its derivative (E is quadratic in
the moments), and the site and whole-system forces agreeing.  Any out-of-bounds access, leak or
undefined operation aborts the driver.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

DRIVER = r"""
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
int oracle_ewald(int64_t, const double *, const double *, const double *, const double *, double, double, double,
                 int, int, double *, double *, double *);
int oracle_ewald_sites(int64_t, const double *, const double *, const double *, const double *, double, double,
                       double, int, int, int64_t, const int64_t *, double *, double *);
int oracle_ewald_moments(int64_t, const double *, const double *, const double *, const double *, double, double,
                         double, int, int, double *, double *);
int oracle_dtensor(const double *, double, int, double *);
int oracle_near_field(int64_t, const double *, const double *, const double *, const double *, double, double, int,
                      int, double *, double *, double *);

static void params(int64_t n, double L, double eps, double scale, double *a, double *rc, int *km) {
    const double s = sqrt(log(1.0 / eps)) + 1.0;
    *a = scale * sqrt(M_PI) * pow((double)n, 1.0 / 6.0) / L;
    *rc = s / *a;
    *km = (int)ceil(s * *a * L / M_PI);
}
static uint64_t st = 88172645463325252ULL;
static double urand(void) { st ^= st << 13; st ^= st >> 7; st ^= st << 17; return (double)(st >> 11) / 9007199254740992.0; }

int main(void) {
    /* NaCl conventional cell, a = 2 (nearest neighbour 1): E = -4 M */
    double pos[8][3], q[8];
    const double b[4][3] = {{0, 0, 0}, {0, 1, 1}, {1, 0, 1}, {1, 1, 0}};
    for (int i = 0; i < 4; i++) {
        for (int c = 0; c < 3; c++) { pos[i][c] = b[i][c] - 0.75; pos[4 + i][c] = b[i][c] + (c == 0) - 0.75; }
        for (int c = 0; c < 3; c++) { if (pos[4 + i][c] >= 1.0) pos[4 + i][c] -= 2.0; }
        q[i] = 1; q[4 + i] = -1;
    }
    double a, rc, eo[5], F[8][3];
    int km;
    params(8, 2.0, 1e-14, 1.0, &a, &rc, &km);
    if (oracle_ewald(8, &pos[0][0], q, NULL, NULL, 2.0, a, rc, km, 2, eo, &F[0][0], NULL)) return 2;
    const double M = 1.747564594633182;
    printf("nacl %.15f %.3e\n", eo[4], fabs(eo[4] + 4 * M));
    if (fabs(eo[4] + 4 * M) > 1e-9) return 3;
    for (int i = 0; i < 8; i++) for (int c = 0; c < 3; c++) if (fabs(F[i][c]) > 1e-9) return 4;

    /* random neutral q / mu / traceless Theta cell */
    enum { N = 12 };
    const double L = 6.0;
    double p[N][3], qq[N], mu[N][3], th[N][6];
    for (int i = 0; i < N; i++) {
        for (int c = 0; c < 3; c++) { p[i][c] = L * (urand() - 0.5); mu[i][c] = 0.2 * (urand() - 0.5); }
        qq[i] = (i % 2 ? 1.0 : -1.0) * (0.5 + urand());
        for (int c = 0; c < 6; c++) th[i][c] = 0.1 * (urand() - 0.5);
        th[i][5] = -th[i][0] - th[i][3];
    }
    double qs = 0;
    for (int i = 0; i < N; i++) qs += qq[i];
    qq[0] -= qs;
    double e1[5], e2[5], F1[N][3], G1[N][3], F2[N][3], G2[N][3];
    params(N, L, 1e-14, 1.0, &a, &rc, &km);
    if (oracle_ewald(N, &p[0][0], qq, &mu[0][0], &th[0][0], L, a, rc, km, 3, e1, &F1[0][0], &G1[0][0])) return 5;
    params(N, L, 1e-14, 1.3, &a, &rc, &km);
    if (oracle_ewald(N, &p[0][0], qq, &mu[0][0], &th[0][0], L, a, rc, km, 1, e2, &F2[0][0], &G2[0][0])) return 6;
    printf("alpha %.15f %.15f %.3e\n", e1[4], e2[4], fabs(e1[4] - e2[4]) / fabs(e1[4]));
    if (fabs(e1[4] - e2[4]) > 1e-11 * fabs(e1[4])) return 7;
    for (int i = 0; i < N; i++)
        for (int c = 0; c < 3; c++)
            if (fabs(F1[i][c] - F2[i][c]) > 1e-9 || fabs(G1[i][c] - G2[i][c]) > 1e-9) return 8;
    const int64_t sel[3] = {1, 5, 11};
    double Fs[3][3], Gs[3][3];
    params(N, L, 1e-14, 1.0, &a, &rc, &km);
    if (oracle_ewald_sites(N, &p[0][0], qq, &mu[0][0], &th[0][0], L, a, rc, km, 2, 3, sel, &Fs[0][0], &Gs[0][0]))
        return 9;
    for (int s = 0; s < 3; s++)
        for (int c = 0; c < 3; c++)
            if (fabs(Fs[s][c] - F1[sel[s]][c]) > 1e-10 || fabs(Gs[s][c] - G1[sel[s]][c]) > 1e-10) return 10;
    double dq[N], dth[N][6];
    if (oracle_ewald_moments(N, &p[0][0], qq, &mu[0][0], &th[0][0], L, a, rc, km, 2, dq, &dth[0][0])) return 11;
    /* the energy is quadratic in the moments: E = 1/2 (q.dE/dq + mu.dE/dmu + Theta:dE/dTheta) */
    double quad = 0;
    for (int i = 0; i < N; i++) {
        quad += qq[i] * dq[i];
        for (int c = 0; c < 3; c++) quad += mu[i][c] * G1[i][c];
        for (int c = 0; c < 6; c++) quad += th[i][c] * dth[i][c];
    }
    printf("euler %.15f %.15f\n", 0.5 * quad, e1[4]);
    if (fabs(0.5 * quad - e1[4]) > 1e-9 * fabs(e1[4])) return 12;
    double T[243], r[3] = {0.3, -0.7, 1.1};
    for (int k = 0; k <= 5; k++)
        if (oracle_dtensor(r, 0.4, k, T)) return 13;
    double ea[N], Fn[N][3], Gn[N][3];
    if (oracle_near_field(N, &p[0][0], qq, &mu[0][0], &th[0][0], L, 0.3, 2, 2, ea, &Fn[0][0], &Gn[0][0])) return 14;
    puts("SANITIZED_OK");
    return 0;
}
"""


def test_oracle_under_address_and_ub_sanitizers(tmp_path):
    cc = shutil.which("gcc")
    if cc is None:
        pytest.skip("no gcc")
    drv = tmp_path / "driver.c"
    drv.write_text(DRIVER)
    exe = tmp_path / "oracle_asan"
    cmd = [cc, "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-fopenmp", "-std=gnu11", os.path.join(ROOT, "oracle", "ewald.c"), str(drv), "-o", str(exe), "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and "sanitizer" in r.stderr.lower() and "cannot find" in r.stderr.lower():
        pytest.skip("sanitizer runtime not installed")
    assert r.returncode == 0, r.stderr
    # verify_asan_link_order=0: the sanitizer runtime need not come first when the environment preloads a
    # library of its own
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", OMP_NUM_THREADS="3")
    out = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    print(out.stdout)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "SANITIZED_OK" in out.stdout
    assert "runtime error" not in out.stderr
