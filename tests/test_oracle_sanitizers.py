"""The C oracle under AddressSanitizer and UndefinedBehaviorSanitizer (CPU).

A small C driver calls every exported oracle function on tiny grids of both
lattices -- periodic and between plates, constant and per-cell relaxation time,
every force order -- with the oracle built by gcc with
-fsanitize=address,undefined (serial build, no OpenMP, so the sanitizers see
one thread).  Any out-of-bounds access, leak, use of uninitialised heap memory
caught by ASan, or undefined behaviour (overflow, bad shift, misaligned or null
access) aborts the driver; the test requires a clean exit.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ORACLE_C = os.path.join(HERE, "..", "oracle", "lbm_oracle.c")

DRIVER = r"""
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_lattice(int lattice, int *c, double *w, double *r, int *degree);
int oracle_hermite(int lattice, int n, double *out);
int oracle_maxwell_coeff(int D, int n, double rho, const double *u, double theta, double *out);
int oracle_equilibrium(int lattice, int eq_order, double rho, const double *u, double theta,
                       double *feq);
int oracle_force(int lattice, int force_order, double rho, const double *u, double theta,
                 const double *g, const double *sigma, double *F);
int oracle_init(int lattice, int64_t nx, int64_t ny, int64_t nz, int eq_order, int force_order,
                const double *walls, const double *rho, const double *u, const double *theta,
                const double *g, double *f, int nthreads);
int oracle_step(int lattice, int64_t nx, int64_t ny, int64_t nz, double tau_hat, double mu,
                int eq_order, int force_order, const double *walls, const double *g, double *f,
                double *tmp, int64_t nsteps, int nthreads);
int oracle_moments(int lattice, int64_t ncell, const double *f, const double *g, double *rho,
                   double *u, double *theta, int nthreads);
int oracle_sigma(int lattice, int64_t ncell, double tau_hat, double mu, int eq_order,
                 const double *f, const double *g, double *sigma, int nthreads);
int oracle_heat_flux(int lattice, int64_t ncell, double tau_hat, double mu, int eq_order,
                     int force_order, const double *f, const double *g, double *q, int nthreads);
int oracle_totals(int lattice, int64_t ncell, const double *f, double *out);

/* 0 (the grid functions) or a positive count (the table functions) is success */
#define CHECK(call)                                                     \
    do {                                                                \
        int rc_ = (call);                                               \
        if (rc_ < 0) {                                                  \
            fprintf(stderr, "%s returned %d\n", #call, rc_);            \
            return 1;                                                   \
        }                                                               \
    } while (0)

static int finite_all(const double *a, int64_t n)
{
    for (int64_t k = 0; k < n; ++k)
        if (!isfinite(a[k])) return 0;
    return 1;
}

static int run(int lat, int64_t nx, int64_t ny, int64_t nz, const double *walls, double mu,
               int fo)
{
    int c[64 * 3], degree;
    double w[64], r;
    const int D = lat == 0 ? 2 : 3, Q = lat == 0 ? 37 : 39;
    CHECK(oracle_lattice(lat, c, w, &r, &degree));
    const int64_t N = nx * ny * nz;
    double *rho = malloc(sizeof(double) * N), *u = malloc(sizeof(double) * D * N);
    double *th = malloc(sizeof(double) * N), *g = malloc(sizeof(double) * D * N);
    double *f = malloc(sizeof(double) * Q * N), *tmp = malloc(sizeof(double) * Q * N);
    double *sig = malloc(sizeof(double) * D * D * N), *q = malloc(sizeof(double) * D * N);
    double tot[5];
    for (int64_t k = 0; k < N; ++k) {
        rho[k] = 1.0 + 0.01 * sin(0.7 * k);
        th[k] = 1.0 + 0.02 * cos(0.3 * k);
        for (int a = 0; a < D; ++a) {
            u[a * N + k] = 0.01 * sin(0.5 * k + a);
            g[a * N + k] = 1e-4 * (a + 1);
        }
    }
    CHECK(oracle_init(lat, nx, ny, nz, 0, fo, walls, rho, u, th, g, f, 0));
    CHECK(oracle_step(lat, nx, ny, nz, 0.8, mu, 0, fo, walls, g, f, tmp, 7, 0));
    CHECK(oracle_moments(lat, N, f, g, rho, u, th, 0));
    CHECK(oracle_sigma(lat, N, 0.8, mu, 0, f, g, sig, 0));
    CHECK(oracle_heat_flux(lat, N, 0.8, mu, 0, fo, f, g, q, 0));
    CHECK(oracle_totals(lat, N, f, tot));
    int ok = finite_all(f, Q * N) && finite_all(rho, N) && finite_all(u, D * N) &&
             finite_all(th, N) && finite_all(sig, D * D * N) && finite_all(q, D * N) &&
             finite_all(tot, D + 2);
    free(rho); free(u); free(th); free(g); free(f); free(tmp); free(sig); free(q);
    if (!ok) {
        fprintf(stderr, "non-finite output (lattice %d)\n", lat);
        return 1;
    }
    return 0;
}

int main(void)
{
    const double walls[4] = {0.9, 1.2, 0.02, -0.03};
    double buf[4096], u[3] = {0.02, -0.01, 0.015}, g[3] = {1e-4, -2e-4, 5e-5};
    double sigma[9] = {1e-3, 2e-4, 0, 2e-4, -1e-3, 0, 0, 0, 0};
    for (int lat = 0; lat < 2; ++lat) {
        for (int n = 0; n <= 4; ++n) CHECK(oracle_hermite(lat, n, buf));
        CHECK(oracle_equilibrium(lat, 0, 1.01, u, 1.02, buf));
        for (int fo = 1; fo <= 4; ++fo) CHECK(oracle_force(lat, fo, 1.01, u, 1.02, g, sigma, buf));
    }
    for (int n = 0; n <= 4; ++n) CHECK(oracle_maxwell_coeff(3, n, 1.01, u, 1.02, buf));
    for (int fo = 1; fo <= 4; ++fo) {
        if (run(0, 5, 4, 1, NULL, 0.0, fo) || run(1, 3, 4, 5, NULL, 0.0, fo)) return 1;
    }
    if (run(0, 5, 7, 1, walls, 0.05, 4) || run(0, 4, 2, 1, walls, 0.0, 2)) return 1;
    if (run(1, 3, 7, 4, walls, 0.05, 4) || run(1, 4, 1, 3, walls, 0.0, 3)) return 1;
    puts("oracle sanitizer run: clean");
    return 0;
}
"""


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_address_and_undefined_sanitizers(tmp_path):
    drv = tmp_path / "driver.c"
    drv.write_text(DRIVER)
    exe = tmp_path / "driver"
    cmd = ["gcc", "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           ORACLE_C, str(drv), "-o", str(exe), "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and "asan" in r.stderr.lower():
        pytest.skip("sanitizer runtime not available: " + r.stderr[-300:])
    assert r.returncode == 0, r.stderr
    env = dict(os.environ,
               ASAN_OPTIONS="detect_leaks=1:abort_on_error=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    run = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert run.returncode == 0, run.stderr[-4000:]
    assert "runtime error" not in run.stderr, run.stderr[-4000:]
    assert "clean" in run.stdout
