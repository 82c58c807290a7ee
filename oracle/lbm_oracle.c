/*
 * FP64 CPU oracle for the thermal lattice Boltzmann step with a Hermite-expanded
 * body force (Li & Shan, "Body-force modelling in thermal compressible flows with
 * lattice Boltzmann method", arXiv:2302.04741).
 *
 * TEST INFRASTRUCTURE ONLY.  The product library never links, loads or calls this
 * file.  Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark use it.  It shares no code, header, table or constant generator with
 * the GPU path: it derives its own quadrature rule, builds its own Hermite tensors
 * and works on its own data layout (populations per cell, AoS; push streaming).
 *
 * Everything is IEEE binary64 (type `real`), round-to-nearest, built without
 * FMA contraction (-ffp-contract=off) and without fast-math.  Cells are independent within a
 * step, so the OpenMP loop over cells does not change any result; cross-cell
 * sums (totals) run serially in a fixed order.
 *
 * What each function follows (sections and equations of the paper):
 *   quadrature rule ............ Sec. 2, degree-Q Gauss-Hermite rule and eq. (an1);
 *                                D2Q37 of Sec. 3 (lattice constant ~1.19698);
 *                                D3Q39: not in the paper, same construction.
 *   Hermite tensors ............ Sec. 2, H^(n) used in eqs. (fN), (an), (F), (f3).
 *   Maxwellian coefficients .... Sec. 2, a_0^(n), the Hermite coefficients of f^(0).
 *   equilibrium ................ eq. (fN) truncated at order N, evaluated at xi_i
 *                                and multiplied by w_i / omega(xi_i) (Sec. 2).
 *   body force ................. eq. (F) with a^(0)=rho, a^(1)=rho u and
 *                                a^(2) = a_0^(2) - sigma (eqs. (f2), (f3), (fi)).
 *   time step .................. eq. (lbm), with the mid-point values rho, u+g/2,
 *                                theta and the mid-point stress sigma-bar.
 *   moments .................... eq. (rut1) plus the mid-point shift.
 *   heat flux .................. q = 1/2 sum_i f_i |xi_i-u|^2 (xi_i-u), Sec. 2
 *                                (the definition used for q_err).
 *   per-cell relaxation time ... Sec. 3: tau = mu/(rho theta) keeps the dynamic
 *                                viscosity and the conductivity constant; with
 *                                tau^ = tau + 1/2 and the cell's mid-point rho and
 *                                theta of the same step (mu > 0 selects it).
 *   walls ...................... Sec. 3 runs its channel between two plates with a
 *                                multi-speed mass-conserving wall condition it does
 *                                not publish; the one here is this project's own
 *                                (diffuse reflection, mass balanced per column),
 *                                described at or_walls below.
 *
 * Readings where the paper is silent or garbled:
 *   - stored variable f~ = f + (f - f0)/(2 tau) - F/2 (the auxiliary variable of
 *     the trapezoidal time integration); hence u-bar = u~ + g/2 and
 *     theta-bar = (E/rho - |u~|^2 + |g|^2/4)/D with E = sum f~ |xi|^2;
 *   - sigma-bar = -(1 - 1/(2 tau^)) sum_i (f~_i - f0bar_i)(xi_i - u-bar)(xi_i - u-bar),
 *     then its trace (zero in exact arithmetic) is removed;
 *   - initial state f~ = f0(rho0,u0,theta0) - F(rho0,u0,theta0,g,sigma=0)/2;
 *   - every grid is periodic in every axis, except across the plates when they
 *     are on (then periodic in x and z only).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Working precision: binary64 by default.  The same source built with
 * -DOR_REAL="long double" gives an 80-bit build, used by the tests only to
 * measure the rounding floor of the binary64 build. */
#ifndef OR_REAL
#define OR_REAL double
#endif
typedef OR_REAL real;

#define OR_MAXQ 64
#define OR_NMAX 4   /* highest Hermite order held (equilibrium up to 4) */
#define OR_TMAX 81  /* 3^4 components of a rank-4 tensor in 3-D */

enum { OR_D2Q37 = 0, OR_D3Q39 = 1 };

typedef struct {
    int ok;
    int D, Q, degree, max_eq_order;
    int c[OR_MAXQ][3];
    real w[OR_MAXQ];
    real r;
    real xi[OR_MAXQ][3];
    real H[OR_MAXQ][OR_NMAX + 1][OR_TMAX]; /* H^(n)(xi_i), flattened */
} or_lattice;

static or_lattice g_lat[2];

static int ipow(int b, int e)
{
    int p = 1;
    while (e-- > 0) p *= b;
    return p;
}

/* ------------------------------------------------------------------------- */
/* Tensors of "Hermite type".                                                 */
/*                                                                            */
/* T^(0) = 1 and T^(n+1)_{a B} = v_a T^(n)_B + kappa * sum_k delta(a, B_k)     */
/*                                               T^(n-1)_{B without B_k}.      */
/* With v = xi and kappa = -1 this is the recurrence of the tensor Hermite     */
/* polynomials H^(n)(xi).  With v = u and kappa = theta - 1 it gives the       */
/* Hermite coefficients of the Maxwellian divided by rho:                      */
/*   a_0^(2)/rho = uu + (theta-1) delta,                                       */
/*   a_0^(3)/rho = uuu + (theta-1)(u delta + two permutations),                */
/*   a_0^(4)/rho = uuuu + (theta-1)(six uu delta) + (theta-1)^2 (three dd).    */
/* Rank-n tensors are flat arrays of D^n entries, first index most significant.*/
/* ------------------------------------------------------------------------- */
static void hermite_like(int D, int nmax, const real *v, real kappa,
                         real T[][OR_TMAX])
{
    int pw[OR_NMAX + 2];
    pw[0] = 1;
    for (int k = 0; k <= OR_NMAX; ++k) pw[k + 1] = pw[k] * D;
    T[0][0] = 1.0;
    for (int n = 0; n < nmax; ++n) {
        for (int a = 0; a < D; ++a) {
            for (int B = 0; B < pw[n]; ++B) {
                real acc = v[a] * T[n][B];
                for (int k = 0; k < n; ++k) {
                    int bk = (B / pw[n - 1 - k]) % D;
                    if (bk == a) {
                        int hi = B / pw[n - k];
                        int lo = B % pw[n - 1 - k];
                        acc += kappa * T[n - 1][hi * pw[n - 1 - k] + lo];
                    }
                }
                T[n + 1][a * pw[n] + B] = acc;
            }
        }
    }
}

static real contract(const real *A, const real *B, int len)
{
    real s = 0.0;
    for (int k = 0; k < len; ++k) s += A[k] * B[k];
    return s;
}

/* ------------------------------------------------------------------------- */
/* Quadrature rule.                                                           */
/*                                                                            */
/* A lattice is a set of integer velocity shells (all sign changes and axis    */
/* permutations of a generator), one weight per shell and a common scale r:    */
/* xi_i = r c_i.  The weights and r follow from requiring the rule to be a     */
/* Gauss-Hermite rule of the stated degree: sum_i w_i p(xi_i) equals the       */
/* integral of omega p for every monomial p of degree <= degree (Sec. 2).      */
/* Odd monomials vanish by symmetry, and permutations of the exponents give    */
/* the same equation, so one equation per even, non-increasing exponent tuple  */
/* of total degree below `degree` remains:                                     */
/*     s^(|p|/2) sum_shell W_shell M_shell(p) = prod_j (p_j - 1)!!,  s = r^2.  */
/* There are exactly (#shells + 1) such equations for both lattices.  For a    */
/* fixed s the first #shells equations are linear in W; the last one leaves a */
/* scalar residual phi(s) whose root is found by scanning and bisection in     */
/* long double.  Only roots with all weights positive are accepted.            */
/* ------------------------------------------------------------------------- */
static const int SH_D2Q37[][3] = {{0, 0, 0}, {1, 0, 0}, {1, 1, 0}, {2, 0, 0},
                                  {2, 1, 0}, {2, 2, 0}, {3, 0, 0}, {3, 1, 0}};
static const int SH_D3Q39[][3] = {{0, 0, 0}, {1, 0, 0}, {1, 1, 1},
                                  {2, 0, 0}, {2, 2, 0}, {3, 0, 0}};

#define OR_MAXSH 8
#define OR_MAXEQ 9

typedef struct {
    int D, S, E;
    int shell_of[OR_MAXQ];
    int Q;
    int c[OR_MAXQ][3];
    int p[OR_MAXEQ][3]; /* exponent tuples */
    long double M[OR_MAXEQ][OR_MAXSH];
    long double G[OR_MAXEQ];
    int deg[OR_MAXEQ];
} or_system;

static long double dfact(int k) /* (k-1)!! for even k >= 0 */
{
    long double r = 1.0L;
    for (int j = k - 1; j > 0; j -= 2) r *= (long double)j;
    return r;
}

static void build_velocities(or_system *sys, int D, const int (*sh)[3], int S)
{
    static const int perms3[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2},
                                     {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    static const int perms2[2][3] = {{0, 1, 2}, {1, 0, 2}};
    const int (*perms)[3] = (D == 3) ? perms3 : perms2;
    int np = (D == 3) ? 6 : 2;
    sys->D = D;
    sys->S = S;
    sys->Q = 0;
    for (int s = 0; s < S; ++s) {
        for (int pi = 0; pi < np; ++pi) {
            for (int sg = 0; sg < (1 << D); ++sg) {
                int v[3] = {0, 0, 0};
                for (int a = 0; a < D; ++a) {
                    int comp = sh[s][perms[pi][a]];
                    v[a] = ((sg >> a) & 1) ? -comp : comp;
                }
                int dup = 0;
                for (int q = 0; q < sys->Q; ++q)
                    if (sys->c[q][0] == v[0] && sys->c[q][1] == v[1] && sys->c[q][2] == v[2])
                        dup = 1;
                if (!dup) {
                    sys->c[sys->Q][0] = v[0];
                    sys->c[sys->Q][1] = v[1];
                    sys->c[sys->Q][2] = v[2];
                    sys->shell_of[sys->Q] = s;
                    sys->Q++;
                }
            }
        }
    }
}

static void build_equations(or_system *sys, int degree)
{
    int D = sys->D, E = 0;
    int maxd = degree - 1; /* highest even degree below an odd `degree` */
    for (int tot = 0; tot <= maxd; tot += 2) {
        for (int p0 = tot; p0 >= 0; p0 -= 2) {
            int p1max = (p0 < tot - p0) ? p0 : tot - p0;
            for (int p1 = p1max; p1 >= 0; p1 -= 2) {
                int p2 = tot - p0 - p1;
                if (p2 > p1) continue;
                if (D == 2 && p2 != 0) continue;
                sys->p[E][0] = p0;
                sys->p[E][1] = p1;
                sys->p[E][2] = p2;
                sys->deg[E] = tot;
                sys->G[E] = dfact(p0) * dfact(p1) * dfact(p2);
                for (int s = 0; s < sys->S; ++s) sys->M[E][s] = 0.0L;
                for (int q = 0; q < sys->Q; ++q) {
                    long double m = 1.0L;
                    for (int a = 0; a < D; ++a)
                        for (int e = 0; e < sys->p[E][a]; ++e) m *= (long double)sys->c[q][a];
                    sys->M[E][sys->shell_of[q]] += m;
                }
                E++;
            }
        }
    }
    sys->E = E;
}

/* Solve every equation except `excl` for the weights at a given s and return the
 * residual phi(s) of equation `excl`. */
static int weights_at(const or_system *sys, int excl, long double s, long double *W,
                      long double *phi)
{
    int S = sys->S;
    long double A[OR_MAXSH][OR_MAXSH + 1];
    for (int e = 0, row = 0; e < sys->E; ++e) {
        if (e == excl) continue;
        long double sc = powl(s, (long double)(sys->deg[e] / 2));
        for (int k = 0; k < S; ++k) A[row][k] = sc * sys->M[e][k];
        A[row][S] = sys->G[e];
        row++;
    }
    for (int col = 0; col < S; ++col) { /* Gaussian elimination, partial pivoting */
        int piv = col;
        for (int r = col + 1; r < S; ++r)
            if (fabsl(A[r][col]) > fabsl(A[piv][col])) piv = r;
        if (fabsl(A[piv][col]) < 1e-12L) return -1;
        if (piv != col)
            for (int k = 0; k <= S; ++k) {
                long double t = A[col][k];
                A[col][k] = A[piv][k];
                A[piv][k] = t;
            }
        for (int r = col + 1; r < S; ++r) {
            long double f = A[r][col] / A[col][col];
            for (int k = col; k <= S; ++k) A[r][k] -= f * A[col][k];
        }
    }
    for (int r = S - 1; r >= 0; --r) {
        long double acc = A[r][S];
        for (int k = r + 1; k < S; ++k) acc -= A[r][k] * W[k];
        W[r] = acc / A[r][r];
    }
    long double lhs = 0.0L;
    for (int k = 0; k < S; ++k) lhs += sys->M[excl][k] * W[k];
    *phi = powl(s, (long double)(sys->deg[excl] / 2)) * lhs - sys->G[excl];
    return 0;
}

/* Scan s in (0.2, 6] for sign changes of phi, refine by bisection, keep roots
 * whose weights are all positive.  Returns the number of such roots. */
static int positive_roots(const or_system *sys, int excl, long double *s_root)
{
    long double W[OR_MAXSH], ds = 0.0005L, s0 = 0.2L, phi0 = 0.0L;
    int nroots = 0;
    int have0 = (weights_at(sys, excl, s0, W, &phi0) == 0);
    for (int k = 1; k <= 11600; ++k) {
        long double s1 = s0 + ds * (long double)k, phi1;
        int have1 = (weights_at(sys, excl, s1, W, &phi1) == 0);
        if (have0 && have1 && ((phi0 < 0) != (phi1 < 0))) {
            long double lo = s1 - ds, hi = s1, plo = phi0;
            for (int it = 0; it < 200; ++it) {
                long double mid = 0.5L * (lo + hi), pm;
                if (weights_at(sys, excl, mid, W, &pm) != 0) break;
                if ((pm < 0) == (plo < 0)) {
                    lo = mid;
                    plo = pm;
                } else {
                    hi = mid;
                }
            }
            long double sr = 0.5L * (lo + hi), pr;
            if (weights_at(sys, excl, sr, W, &pr) == 0) {
                int pos = 1;
                for (int j = 0; j < sys->S; ++j)
                    if (!(W[j] > 0)) pos = 0;
                if (pos) {
                    *s_root = sr;
                    nroots++;
                }
            }
        }
        phi0 = phi1;
        have0 = have1;
    }
    return nroots;
}

static int derive_lattice(int lattice, or_lattice *L)
{
    or_system sys;
    memset(&sys, 0, sizeof sys);
    int degree;
    if (lattice == OR_D2Q37) {
        build_velocities(&sys, 2, SH_D2Q37, 8);
        degree = 9;
    } else if (lattice == OR_D3Q39) {
        build_velocities(&sys, 3, SH_D3Q39, 6);
        degree = 7;
    } else {
        return -1;
    }
    build_equations(&sys, degree);
    if (sys.E != sys.S + 1) return -2;

    /* Any equation whose removal leaves a regular linear system may serve as the
     * residual; the solution of the full system does not depend on the choice. */
    long double best_s = -1.0L, W[OR_MAXSH], phi;
    int excl = -1;
    for (int e = sys.E - 1; e >= 0 && excl < 0; --e) {
        long double sr;
        if (positive_roots(&sys, e, &sr) == 1) {
            excl = e;
            best_s = sr;
        }
    }
    if (excl < 0) return -3;
    weights_at(&sys, excl, best_s, W, &phi);

    L->D = sys.D;
    L->Q = sys.Q;
    L->degree = degree;
    L->max_eq_order = (degree - 1) / 2; /* Q_deg >= 2N (Sec. 2) */
    L->r = (real)sqrtl(best_s);
    for (int q = 0; q < sys.Q; ++q) {
        L->w[q] = (real)W[sys.shell_of[q]];
        for (int a = 0; a < 3; ++a) {
            L->c[q][a] = sys.c[q][a];
            L->xi[q][a] = (real)(sqrtl(best_s) * (long double)sys.c[q][a]);
        }
        hermite_like(L->D, OR_NMAX, L->xi[q], -1.0, L->H[q]);
    }
    L->ok = 1;
    return 0;
}

static const or_lattice *get_lattice(int lattice)
{
    if (lattice != OR_D2Q37 && lattice != OR_D3Q39) return NULL;
    or_lattice *L = &g_lat[lattice];
    if (!L->ok && derive_lattice(lattice, L) != 0) return NULL;
    return L;
}

/* ------------------------------------------------------------------------- */
/* Per-cell pieces                                                            */
/* ------------------------------------------------------------------------- */

/* Discrete equilibrium: f0_i = w_i sum_{n<=N} (1/n!) a_0^(n) : H^(n)(xi_i). */
static void equilibrium(const or_lattice *L, int N, real rho, const real *u,
                        real theta, real *feq)
{
    real A[OR_NMAX + 1][OR_TMAX];
    int D = L->D;
    hermite_like(D, N, u, theta - 1.0, A);
    for (int i = 0; i < L->Q; ++i) {
        real s = 0.0, fact = 1.0;
        for (int n = 0; n <= N; ++n) {
            if (n > 0) fact *= (real)n;
            s += contract(A[n], L->H[i][n], ipow(D, n)) / fact;
        }
        feq[i] = L->w[i] * rho * s;
    }
}

/* Discrete body force: F_i = w_i sum_{n=1}^{nf} (n/n!) (g a^(n-1)) : H^(n)(xi_i),
 * with a^(0)=rho, a^(1)=rho u, a^(2) = rho[uu + (theta-1) delta] - sigma.
 * Because H^(n) is symmetric, the normalised symmetric product contracts like
 * g_a a^(n-1)_B H^(n)_{aB}. */
static void body_force(const or_lattice *L, int nf, int with_sigma, real rho,
                       const real *u, real theta, const real *g,
                       const real *sigma, real *F)
{
    real A[OR_NMAX + 1][OR_TMAX];
    int D = L->D;
    hermite_like(D, 2, u, theta - 1.0, A);
    for (int n = 0; n <= 2; ++n)
        for (int k = 0; k < ipow(D, n); ++k) A[n][k] *= rho;
    if (with_sigma)
        for (int k = 0; k < D * D; ++k) A[2][k] -= sigma[k];
    for (int i = 0; i < L->Q; ++i) {
        real s = 0.0, fact = 1.0;
        for (int n = 1; n <= nf; ++n) {
            fact *= (real)n;
            int len = ipow(D, n - 1);
            real dot = 0.0;
            for (int a = 0; a < D; ++a)
                dot += g[a] * contract(A[n - 1], &L->H[i][n][a * len], len);
            s += (real)n * dot / fact;
        }
        F[i] = L->w[i] * s;
    }
}

static int force_terms(int force_order, int *nf, int *with_sigma)
{
    switch (force_order) {
    case 1: *nf = 1; *with_sigma = 0; return 0;
    case 2: *nf = 2; *with_sigma = 0; return 0;
    case 3: *nf = 3; *with_sigma = 0; return 0;
    case 4: *nf = 3; *with_sigma = 1; return 0;
    default: return -1;
    }
}

/* Moments of the stored populations of one cell and the mid-point values. */
static void cell_moments(const or_lattice *L, const real *f, const real *g,
                         real *rho_o, real *ub, real *theta_o)
{
    int D = L->D;
    real rho = 0.0, j[3] = {0, 0, 0}, E = 0.0;
    for (int i = 0; i < L->Q; ++i) {
        rho += f[i];
        real x2 = 0.0;
        for (int a = 0; a < D; ++a) {
            j[a] += f[i] * L->xi[i][a];
            x2 += L->xi[i][a] * L->xi[i][a];
        }
        E += f[i] * x2;
    }
    real ut2 = 0.0, g2 = 0.0;
    for (int a = 0; a < D; ++a) {
        real ut = j[a] / rho;
        ub[a] = ut + 0.5 * g[a];
        ut2 += ut * ut;
        g2 += g[a] * g[a];
    }
    *rho_o = rho;
    *theta_o = (E / rho - ut2 + 0.25 * g2) / (real)D;
}

/* sigma-bar of one cell, literal two-pass form, then trace removed. */
static void cell_sigma(const or_lattice *L, const real *f, const real *feq,
                       const real *ub, real tau_hat, real *sig)
{
    int D = L->D;
    for (int k = 0; k < 9; ++k) sig[k] = 0.0;
    for (int i = 0; i < L->Q; ++i) {
        real dev = f[i] - feq[i];
        for (int a = 0; a < D; ++a)
            for (int b = 0; b < D; ++b)
                sig[a * D + b] += dev * (L->xi[i][a] - ub[a]) * (L->xi[i][b] - ub[b]);
    }
    real pref = -(1.0 - 1.0 / (2.0 * tau_hat));
    real tr = 0.0;
    for (int a = 0; a < D; ++a) tr += pref * sig[a * D + a];
    for (int a = 0; a < D; ++a)
        for (int b = 0; b < D; ++b) {
            sig[a * D + b] *= pref;
            if (a == b) sig[a * D + b] -= tr / (real)D;
        }
}

static int eq_order_of(const or_lattice *L, int eq_order)
{
    if (eq_order == 0) return L->max_eq_order;
    if (eq_order < 2 || eq_order > L->max_eq_order) return -1;
    return eq_order;
}

/* Relaxation time of one cell: the run's constant tau^, or, when a dynamic
 * viscosity mu > 0 is given, tau^ = mu/(rho theta) + 1/2 from the cell's
 * mid-point density and temperature (Sec. 3; tau^ = tau + 1/2 as in eq. (lbm)). */
static real cell_tau_hat(real tau_hat, real mu, real rho, real theta)
{
    if (mu > 0.0) return mu / (rho * theta) + 0.5;
    return tau_hat;
}

/* One collision: pre-collision f (stored variable) -> post-collision fs. */
static void collide_cell(const or_lattice *L, int N, int nf, int with_sigma,
                         real tau_hat, real mu, const real *f, const real *g, real *fs)
{
    real rho, ub[3] = {0, 0, 0}, theta, feq[OR_MAXQ], F[OR_MAXQ], sig[9];
    cell_moments(L, f, g, &rho, ub, &theta);
    tau_hat = cell_tau_hat(tau_hat, mu, rho, theta);
    equilibrium(L, N, rho, ub, theta, feq);
    if (with_sigma) cell_sigma(L, f, feq, ub, tau_hat, sig);
    body_force(L, nf, with_sigma, rho, ub, theta, g, sig, F);
    real cf = 1.0 - 1.0 / (2.0 * tau_hat);
    for (int i = 0; i < L->Q; ++i) fs[i] = f[i] - (f[i] - feq[i]) / tau_hat + cf * F[i];
}

/* ------------------------------------------------------------------------- */
/* Exported API (used through ctypes by the test suite)                       */
/* ------------------------------------------------------------------------- */

int oracle_lattice(int lattice, int *c, real *w, real *r, int *degree)
{
    const or_lattice *L = get_lattice(lattice);
    if (!L) return -1;
    for (int q = 0; q < L->Q; ++q) {
        if (c)
            for (int a = 0; a < 3; ++a) c[3 * q + a] = L->c[q][a];
        if (w) w[q] = L->w[q];
    }
    if (r) *r = L->r;
    if (degree) *degree = L->degree;
    return L->Q;
}

/* H^(n)(xi_i) for every velocity: out[i * D^n + k]. */
int oracle_hermite(int lattice, int n, real *out)
{
    const or_lattice *L = get_lattice(lattice);
    if (!L || n < 0 || n > OR_NMAX) return -1;
    int len = ipow(L->D, n);
    for (int q = 0; q < L->Q; ++q)
        for (int k = 0; k < len; ++k) out[q * len + k] = L->H[q][n][k];
    return len;
}

/* a_0^(n) of the Maxwellian with (rho, u, theta) in D dimensions. */
int oracle_maxwell_coeff(int D, int n, real rho, const real *u, real theta, real *out)
{
    if (D < 1 || D > 3 || n < 0 || n > OR_NMAX) return -1;
    real A[OR_NMAX + 1][OR_TMAX];
    hermite_like(D, n, u, theta - 1.0, A);
    int len = ipow(D, n);
    for (int k = 0; k < len; ++k) out[k] = rho * A[n][k];
    return len;
}

int oracle_equilibrium(int lattice, int eq_order, real rho, const real *u,
                       real theta, real *feq)
{
    const or_lattice *L = get_lattice(lattice);
    if (!L) return -1;
    int N = eq_order_of(L, eq_order);
    if (N < 0) return -2;
    equilibrium(L, N, rho, u, theta, feq);
    return L->Q;
}

/* sigma: D*D row-major (ignored unless force_order == 4). */
int oracle_force(int lattice, int force_order, real rho, const real *u,
                 real theta, const real *g, const real *sigma, real *F)
{
    const or_lattice *L = get_lattice(lattice);
    int nf, ws;
    if (!L) return -1;
    if (force_terms(force_order, &nf, &ws) != 0) return -2;
    real sig[9] = {0};
    if (ws && sigma)
        for (int k = 0; k < L->D * L->D; ++k) sig[k] = sigma[k];
    body_force(L, nf, ws, rho, u, theta, g, sig, F);
    return L->Q;
}

static int set_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
    return omp_get_max_threads();
#else
    (void)nthreads;
    return 1;
#endif
}

static int check_grid(const or_lattice *L, int64_t nx, int64_t ny, int64_t nz)
{
    if (!L || nx < 1 || ny < 1 || nz < 1) return -1;
    if (L->D == 2 && nz != 1) return -1;
    return 0;
}

static int64_t wrap(int64_t v, int64_t n)
{
    v %= n;
    return v < 0 ? v + n : v;
}

/* ------------------------------------------------------------------------- */
/* Walls normal to y                                                          */
/* ------------------------------------------------------------------------- */
/* Two plates at y = -1/2 (bottom, side 0) and y = ny - 1/2 (top, side 1), with
 * temperature th[side] and tangential velocity uw[side] along x; the grid stays
 * periodic in x and z.  A population that would stream across a plate is
 * absorbed, its mass credited to the plate and to the (x, z) column of the node
 * it leaves.  The plate emits the Maxwellian of its own temperature and
 * velocity: into every pair (direction i entering the domain, node within
 * |c_iy| layers of the plate) whose streaming source lies behind the plate, it
 * puts rho_w e_i with e_i = f0_i(1, (uw, 0, 0), th), rho_w taken at the source's
 * column.  Per column rho_w is fixed by mass balance,
 *     rho_w * sum_{i entering} min(|c_iy|, ny) e_i = mass absorbed in that column,
 * so every step conserves mass exactly (diffuse reflection with a discrete,
 * mass-conserving flux). */
typedef struct {
    real th[2], uw[2];
} or_walls;

static int enters(const or_lattice *L, int side, int i)
{
    int cy = L->c[i][1];
    return side == 0 ? cy > 0 : cy < 0;
}

/* e_i of one plate and the normalisation sum_{i entering} min(|c_iy|, ny) e_i. */
static real wall_emission(const or_lattice *L, int N, const or_walls *w, int side, int64_t ny,
                          real *e)
{
    real u[3] = {w->uw[side], 0.0, 0.0};
    equilibrium(L, N, 1.0, u, w->th[side], e);
    real z = 0.0;
    for (int i = 0; i < L->Q; ++i)
        if (enters(L, side, i)) {
            int64_t k = L->c[i][1] < 0 ? -L->c[i][1] : L->c[i][1];
            z += (real)(k < ny ? k : ny) * e[i];
        }
    return z;
}

/* Apply the plates to a state given at the nodes: `src` holds, for every node,
 * the populations about to stream (AoS); the absorbed mass is summed from the
 * populations of src that cross a plate, and the emitted values are written
 * into `dst` (AoS, at the destination nodes).  Column sums run in a fixed order
 * (y ascending, then i ascending), serially. */
static int apply_walls(const or_lattice *L, int N, const or_walls *w, int64_t nx, int64_t ny,
                       int64_t nz, const real *src, real *dst)
{
    int Q = L->Q;
    int64_t ncol = nx * nz;
    real *rw = (real *)malloc(sizeof(real) * (size_t)(2 * ncol));
    if (!rw) return -4;
    real e[2][OR_MAXQ], Z[2];
    for (int side = 0; side < 2; ++side) Z[side] = wall_emission(L, N, w, side, ny, e[side]);
    for (int64_t col = 0; col < ncol; ++col) {
        int64_t x = col % nx, z = col / nx;
        real m[2] = {0.0, 0.0};
        for (int64_t y = 0; y < ny; ++y) {
            const real *fs = &src[((z * ny + y) * nx + x) * Q];
            for (int i = 0; i < Q; ++i) {
                int64_t yd = y + L->c[i][1];
                if (yd < 0) m[0] += fs[i];
                else if (yd >= ny) m[1] += fs[i];
            }
        }
        rw[col] = m[0] / Z[0];
        rw[ncol + col] = m[1] / Z[1];
    }
    for (int64_t col = 0; col < ncol; ++col) {
        int64_t x = col % nx, z = col / nx;
        for (int side = 0; side < 2; ++side)
            for (int i = 0; i < Q; ++i) {
                if (!enters(L, side, i)) continue;
                int64_t k = L->c[i][1] < 0 ? -L->c[i][1] : L->c[i][1];
                for (int64_t j = 0; j < k && j < ny; ++j) {
                    int64_t yd = side == 0 ? j : ny - 1 - j;
                    int64_t xs = wrap(x - L->c[i][0], nx), zs = wrap(z - L->c[i][2], nz);
                    dst[((z * ny + yd) * nx + x) * Q + i] = rw[side * ncol + zs * nx + xs] * e[side][i];
                }
            }
    }
    free(rw);
    return 0;
}

static int read_walls(const real *walls, or_walls *w)
{
    if (!walls) return 0;
    for (int s = 0; s < 2; ++s) {
        w->th[s] = walls[s];
        w->uw[s] = walls[2 + s];
        if (!(w->th[s] > 0.0)) return -1;
    }
    return 1;
}

/* Fields are SoA: rho[N], u[a*N + cell], theta[N], g[a*N + cell];
 * populations are AoS: f[cell*Q + i]; cell = (z*ny + y)*nx + x. */
/* walls: NULL (periodic) or {theta_b, theta_t, U_b, U_t}.  With walls, the
 * populations that would stream in from behind a plate are then replaced by
 * the plate's emission balancing the initial populations that stream out. */
int oracle_init(int lattice, int64_t nx, int64_t ny, int64_t nz, int eq_order, int force_order,
                const real *walls, const real *rho, const real *u, const real *theta,
                const real *g, real *f, int nthreads)
{
    const or_lattice *L = get_lattice(lattice);
    if (check_grid(L, nx, ny, nz)) return -1;
    int N = eq_order_of(L, eq_order), nf, ws;
    if (N < 0 || force_terms(force_order, &nf, &ws)) return -2;
    or_walls w;
    int has_walls = read_walls(walls, &w);
    if (has_walls < 0) return -3;
    int64_t ncell = nx * ny * nz;
    int D = L->D, Q = L->Q;
    set_threads(nthreads);
#pragma omp parallel for schedule(static)
    for (int64_t x = 0; x < ncell; ++x) {
        real uu[3] = {0, 0, 0}, gg[3] = {0, 0, 0}, feq[OR_MAXQ], F[OR_MAXQ];
        real sig[9] = {0};
        for (int a = 0; a < D; ++a) {
            uu[a] = u[a * ncell + x];
            gg[a] = g[a * ncell + x];
        }
        equilibrium(L, N, rho[x], uu, theta[x], feq);
        body_force(L, nf, 0, rho[x], uu, theta[x], gg, sig, F);
        for (int i = 0; i < Q; ++i) f[x * Q + i] = feq[i] - 0.5 * F[i];
    }
    if (has_walls) return apply_walls(L, N, &w, nx, ny, nz, f, f);
    return 0;
}

/* Steps between plates: collide every node (post-collision values kept at the
 * node), push what stays inside (periodic in x and z), then let the plates
 * absorb what crosses them and emit into the slots behind them. */
static int step_walls(const or_lattice *L, int N, int nf, int ws, const or_walls *w,
                      int64_t nx, int64_t ny, int64_t nz, real tau_hat, real mu, const real *g,
                      real *f, real *tmp, int64_t nsteps)
{
    int64_t ncell = nx * ny * nz;
    int D = L->D, Q = L->Q;
    real *post = (real *)malloc(sizeof(real) * (size_t)ncell * (size_t)Q);
    if (!post) return -4;
    int st = 0;
    for (int64_t s = 0; s < nsteps && st == 0; ++s) {
#pragma omp parallel for schedule(static)
        for (int64_t cell = 0; cell < ncell; ++cell) {
            real gg[3] = {0, 0, 0};
            for (int a = 0; a < D; ++a) gg[a] = g[a * ncell + cell];
            collide_cell(L, N, nf, ws, tau_hat, mu, &f[cell * Q], gg, &post[cell * Q]);
        }
#pragma omp parallel for schedule(static)
        for (int64_t cell = 0; cell < ncell; ++cell) {
            int64_t x = cell % nx, y = (cell / nx) % ny, z = cell / (nx * ny);
            for (int i = 0; i < Q; ++i) {
                int64_t yd = y + L->c[i][1];
                if (yd < 0 || yd >= ny) continue;  /* absorbed by a plate */
                int64_t xd = wrap(x + L->c[i][0], nx);
                int64_t zd = wrap(z + L->c[i][2], nz);
                tmp[((zd * ny + yd) * nx + xd) * Q + i] = post[cell * Q + i];
            }
        }
        st = apply_walls(L, N, w, nx, ny, nz, post, tmp);
        memcpy(f, tmp, (size_t)ncell * (size_t)Q * sizeof(real));
    }
    free(post);
    return st;
}

/* nsteps collide-then-push steps; f holds the result, tmp is scratch. */
/* mu = 0: constant tau_hat; mu > 0: per-cell tau^ = mu/(rho theta) + 1/2. */
int oracle_step(int lattice, int64_t nx, int64_t ny, int64_t nz, real tau_hat, real mu,
                int eq_order, int force_order, const real *walls, const real *g, real *f,
                real *tmp, int64_t nsteps, int nthreads)
{
    const or_lattice *L = get_lattice(lattice);
    if (check_grid(L, nx, ny, nz)) return -1;
    int N = eq_order_of(L, eq_order), nf, ws;
    if (N < 0 || force_terms(force_order, &nf, &ws)) return -2;
    if (!(mu >= 0.0) || (mu == 0.0 && !(tau_hat > 0.5))) return -3;
    or_walls w;
    int has_walls = read_walls(walls, &w);
    if (has_walls < 0) return -3;
    int64_t ncell = nx * ny * nz;
    int D = L->D, Q = L->Q;
    set_threads(nthreads);
    if (has_walls) return step_walls(L, N, nf, ws, &w, nx, ny, nz, tau_hat, mu, g, f, tmp,
                                     nsteps);
    real *src = f, *dst = tmp;
    for (int64_t s = 0; s < nsteps; ++s) {
#pragma omp parallel for schedule(static)
        for (int64_t cell = 0; cell < ncell; ++cell) {
            int64_t x = cell % nx, y = (cell / nx) % ny, z = cell / (nx * ny);
            real gg[3] = {0, 0, 0}, fs[OR_MAXQ];
            for (int a = 0; a < D; ++a) gg[a] = g[a * ncell + cell];
            collide_cell(L, N, nf, ws, tau_hat, mu, &src[cell * Q], gg, fs);
            for (int i = 0; i < Q; ++i) {
                int64_t xd = wrap(x + L->c[i][0], nx);
                int64_t yd = wrap(y + L->c[i][1], ny);
                int64_t zd = wrap(z + L->c[i][2], nz);
                dst[((zd * ny + yd) * nx + xd) * Q + i] = fs[i];
            }
        }
        real *t = src;
        src = dst;
        dst = t;
    }
    if (src != f) memcpy(f, src, (size_t)ncell * (size_t)Q * sizeof(real));
    return 0;
}

/* Physical moments at the current time: rho, u-bar = u~ + g/2, theta-bar. */
int oracle_moments(int lattice, int64_t ncell, const real *f, const real *g,
                   real *rho, real *u, real *theta, int nthreads)
{
    const or_lattice *L = get_lattice(lattice);
    if (!L || ncell < 1) return -1;
    int D = L->D, Q = L->Q;
    set_threads(nthreads);
#pragma omp parallel for schedule(static)
    for (int64_t x = 0; x < ncell; ++x) {
        real gg[3] = {0, 0, 0}, ub[3] = {0, 0, 0}, r, t;
        for (int a = 0; a < D; ++a) gg[a] = g[a * ncell + x];
        cell_moments(L, &f[x * Q], gg, &r, ub, &t);
        rho[x] = r;
        theta[x] = t;
        for (int a = 0; a < D; ++a) u[a * ncell + x] = ub[a];
    }
    return 0;
}

/* Mid-point deviatoric stress of every cell: sigma[(a*D+b)*N + cell]. */
int oracle_sigma(int lattice, int64_t ncell, real tau_hat, real mu, int eq_order,
                 const real *f, const real *g, real *sigma, int nthreads)
{
    const or_lattice *L = get_lattice(lattice);
    if (!L || ncell < 1) return -1;
    int N = eq_order_of(L, eq_order);
    if (N < 0) return -2;
    int D = L->D, Q = L->Q;
    set_threads(nthreads);
#pragma omp parallel for schedule(static)
    for (int64_t x = 0; x < ncell; ++x) {
        real gg[3] = {0, 0, 0}, ub[3] = {0, 0, 0}, r, t, feq[OR_MAXQ], sig[9];
        for (int a = 0; a < D; ++a) gg[a] = g[a * ncell + x];
        cell_moments(L, &f[x * Q], gg, &r, ub, &t);
        equilibrium(L, N, r, ub, t, feq);
        cell_sigma(L, &f[x * Q], feq, ub, cell_tau_hat(tau_hat, mu, r, t), sig);
        for (int k = 0; k < D * D; ++k) sigma[k * ncell + x] = sig[k];
    }
    return 0;
}

/* Heat flux q = 1/2 sum_i f_i |xi_i - u|^2 (xi_i - u) of the physical
 * distribution f = f0bar + (1 - 1/(2 tau^)) (f~ - f0bar + Fbar/2). */
int oracle_heat_flux(int lattice, int64_t ncell, real tau_hat, real mu, int eq_order,
                     int force_order, const real *f, const real *g, real *q, int nthreads)
{
    const or_lattice *L = get_lattice(lattice);
    if (!L || ncell < 1) return -1;
    int N = eq_order_of(L, eq_order), nf, ws;
    if (N < 0 || force_terms(force_order, &nf, &ws)) return -2;
    int D = L->D, Q = L->Q;
    set_threads(nthreads);
#pragma omp parallel for schedule(static)
    for (int64_t x = 0; x < ncell; ++x) {
        real gg[3] = {0, 0, 0}, ub[3] = {0, 0, 0}, r, t, feq[OR_MAXQ], F[OR_MAXQ];
        real sig[9] = {0}, qq[3] = {0, 0, 0};
        const real *fx = &f[x * Q];
        for (int a = 0; a < D; ++a) gg[a] = g[a * ncell + x];
        cell_moments(L, fx, gg, &r, ub, &t);
        real th_cell = cell_tau_hat(tau_hat, mu, r, t);
        real cf = 1.0 - 1.0 / (2.0 * th_cell);
        equilibrium(L, N, r, ub, t, feq);
        if (ws) cell_sigma(L, fx, feq, ub, th_cell, sig);
        body_force(L, nf, ws, r, ub, t, gg, sig, F);
        for (int i = 0; i < Q; ++i) {
            real fp = feq[i] + cf * (fx[i] - feq[i] + 0.5 * F[i]);
            real c2 = 0.0;
            for (int a = 0; a < D; ++a) c2 += (L->xi[i][a] - ub[a]) * (L->xi[i][a] - ub[a]);
            for (int a = 0; a < D; ++a) qq[a] += fp * c2 * (L->xi[i][a] - ub[a]);
        }
        for (int a = 0; a < D; ++a) q[a * ncell + x] = 0.5 * qq[a];
    }
    return 0;
}

/* Global sums of the stored populations, serial, fixed order:
 * out = [sum f, sum f xi_a (a < D), sum f |xi|^2]. */
int oracle_totals(int lattice, int64_t ncell, const real *f, real *out)
{
    const or_lattice *L = get_lattice(lattice);
    if (!L || ncell < 1) return -1;
    int D = L->D, Q = L->Q;
    real m = 0.0, p[3] = {0, 0, 0}, e = 0.0;
    for (int64_t x = 0; x < ncell; ++x) {
        for (int i = 0; i < Q; ++i) {
            real fi = f[x * Q + i], x2 = 0.0;
            m += fi;
            for (int a = 0; a < D; ++a) {
                p[a] += fi * L->xi[i][a];
                x2 += L->xi[i][a] * L->xi[i][a];
            }
            e += fi * x2;
        }
    }
    out[0] = m;
    for (int a = 0; a < D; ++a) out[1 + a] = p[a];
    out[1 + D] = e;
    return 0;
}

int oracle_num_threads(int nthreads) { return set_threads(nthreads); }
