"""The C oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(host code only, serial), driven through every entry point on small grids:
periodic and patch solves (a wrapping patch, a masked patch), interpolation,
operator, Newton step, cell mask and force.  Any out-of-bounds access, use of
freed memory, leak or undefined operation aborts the driver."""
from __future__ import annotations

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "ndgp_oracle.c")

DRIVER = r"""
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

double oracle_beta_lcdm(double, double, double);
double oracle_alpha(double, double, double);
void oracle_source(int64_t, const double *, double, double, double, double *, double *);
void oracle_source_shift(int64_t, const double *, double, double, double, double, double *);
void oracle_operator(int, int, double, double, double *, double *);
void oracle_operator_at(int, double, double, const double *, int64_t, const int32_t *, double *);
double oracle_newton_update(int, double, double, const double *, double, int, int, int);
int oracle_interpolate(const double *, int, int, const int[3], int, int, double *, int);
int oracle_solve_periodic(int, double, double, const double *, double *, int, int, double, int,
                          int, double *, int, int *, double *);
int oracle_solve_patch(int, double, double, const double *, const double *, int, int,
                       const int[3], double *, int, double, int, int, int,
                       const unsigned char *, double *, int, int *, double *);
int oracle_cell_mask(const double *, const double *, int, int, const int[3], int, double,
                     unsigned char *);
void oracle_force(int, double, double *, int, double *);

static double rnd(unsigned *s) { *s = *s * 1664525u + 1013904223u; return (*s >> 8) / 16777216.0; }

int main(void) {
    const int n = 16, m = 16, c3 = n * n * n, p3 = (m + 2) * (m + 2) * (m + 2);
    const double h = 1.0 / 2997.92458;
    const double beta = oracle_beta_lcdm(1.0, 0.3, 1.0), al = oracle_alpha(1.0, beta, 1.0);
    double *delta = malloc(sizeof(double) * c3), *S = malloc(sizeof(double) * c3);
    double *phi = calloc(c3, sizeof(double)), hist[64], rel = 0.0, mean = 0.0;
    unsigned seed = 7;
    for (int i = 0; i < c3; ++i) delta[i] = exp(1.5 * (rnd(&seed) - 0.5)) - 1.0;
    oracle_source(c3, delta, 0.3, 1.0, beta, S, &mean);
    int cyc = 0;
    if (oracle_solve_periodic(n, h, al, S, phi, 0, 60, 0.0, 2, 2, hist, 64, &cyc, &rel)) return 1;
    /* a patch wrapping the periodic domain, relaxed */
    const int o1[3] = {-3, 5, 12};
    double *dp = malloc(sizeof(double) * m * m * m), *Sp = malloc(sizeof(double) * m * m * m);
    for (int i = 0; i < m * m * m; ++i) dp[i] = delta[i % c3];
    oracle_source_shift(m * m * m, dp, mean, 0.3, 1.0, beta, Sp);
    double *pp = calloc(p3, sizeof(double));
    if (oracle_solve_patch(m, h / 2, al, Sp, phi, n, 1, o1, pp, 60, 0.0, 2, 2, 0, NULL, hist, 64,
                           &cyc, &rel)) return 2;
    /* a masked child of the patch (cell-wise truncation) */
    const int o2[3] = {4, 4, 4};
    unsigned char *mask = malloc(8 * 8 * 8);
    double *psi = malloc(sizeof(double) * p3);
    for (int i = 0; i < p3; ++i) psi[i] = 3.0 * pp[i];
    if (oracle_cell_mask(pp, psi, m, 0, o2, 8, 0.05, mask)) return 3;
    double *S2 = malloc(sizeof(double) * 512), *pc = calloc(1000, sizeof(double));
    for (int i = 0; i < 512; ++i) S2[i] = Sp[i];
    if (oracle_solve_patch(8, h / 4, al, S2, pp, m, 0, o2, pc, 40, 0.0, 2, 2, 0, mask, hist, 64,
                           &cyc, &rel) < -1) return 4;
    /* interpolation only, operator, listed cells, Newton step, force */
    if (oracle_interpolate(pp, m, 0, o2, 1, 4, pc, 1)) return 5;
    double *pad = malloc(sizeof(double) * (n + 2) * (n + 2) * (n + 2)), *L = malloc(sizeof(double) * c3);
    for (int i = 0; i < (n + 2) * (n + 2) * (n + 2); ++i) pad[i] = 1e-7 * rnd(&seed);
    oracle_operator(n, 1, h, al, pad, L);
    int32_t cells[6] = {0, 0, 0, n - 1, n - 1, n - 1};
    double at[2];
    oracle_operator_at(n, h, al, phi, 2, cells, at);
    (void)oracle_newton_update(n, h, al, pad, 0.1, 0, n - 1, 3);
    double *F = malloc(sizeof(double) * 3 * c3);
    oracle_force(n, h, pad, 1, F);
    double *Fp = malloc(sizeof(double) * 3 * m * m * m);
    oracle_force(m, h / 2, pp, 0, Fp);
    free(delta); free(S); free(phi); free(dp); free(Sp); free(pp); free(mask); free(psi);
    free(S2); free(pc); free(pad); free(L); free(F); free(Fp);
    printf("sanitized oracle ok\n");
    return 0;
}
"""


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    drv = tmp_path / "drive.c"
    drv.write_text(DRIVER)
    exe = tmp_path / "drive"
    cmd = ["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-o", str(exe), str(drv), SRC, "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and "sanitizer" in (r.stderr or "").lower():
        pytest.skip("this gcc has no sanitizer runtime: " + r.stderr[-300:])
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    run = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300, env=env)
    assert run.returncode == 0, run.stdout[-2000:] + run.stderr[-4000:]
    assert "sanitized oracle ok" in run.stdout
