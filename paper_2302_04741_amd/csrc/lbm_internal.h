// Internal declarations of the gfx950 thermal LBM library: lattice traits, the
// per-cell arithmetic shared by the kernels, kernel argument blocks and the
// launchers called by the C ABI layer.
//
// Method (Li & Shan, arXiv:2302.04741, Sec. 2):
//   stored variable f~ (auxiliary variable of the trapezoidal time integration);
//   mid-point moments rho, u = u~ + g/2, theta = (E/rho - |u~|^2 + |g|^2/4)/D;
//   equilibrium = Hermite expansion of the Maxwellian to order N, eq. (fN);
//   force       = Hermite expansion eq. (F) to the third moment, eq. (fi);
//   sigma-bar   = -(1 - 1/(2 tau^)) sum_i (f~_i - f0_i)(xi_i - u)(xi_i - u), traceless;
//   step        = eq. (lbm): f~(x + xi_i, t+1) = f~ - (f~ - f0)/tau^ + (1 - 1/(2 tau^)) F.
// Everything here is written as closed-form polynomials in xi.u, xi.g and
// xi.sigma.xi with per-shell constants, and shares the even/odd parts of each
// +c/-c velocity pair.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

#include <type_traits>

#include "fastdiv.h"
#include "lattice_tables.h"

namespace lbm {

// ---------------------------------------------------------------------------
// compile-time loops
// ---------------------------------------------------------------------------
template <int I, int N, typename F>
__host__ __device__ __forceinline__ void static_for(F &&f)
{
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        static_for<I + 1, N>(static_cast<F &&>(f));
    }
}

// fused multiply-add in the precision of its arguments
__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }

// ---------------------------------------------------------------------------
// buffer access to one population plane: scalar resource (plane base, size),
// scalar row offset, per-lane 32-bit x offset.  Addressing costs no VALU
// work, and the hardware range check drops accesses past the plane.
// ---------------------------------------------------------------------------
constexpr int BUF_DWORD3 = 0x00020000;  // raw buffer, 32-bit data format
// Cache policy of the step's population traffic.  Every element is read once
// and written once per step.  Stores are non-temporal (6% faster than default
// stores on the D3Q39 FP32 step); loads keep the default policy (1.3% / 1.8% /
// 4.5% faster than non-temporal loads for FP32 / FP64 / F16 storage).
constexpr int BUF_LD = 0;
constexpr int BUF_NT = 2;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const void *base, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, int(bytes),
                                             BUF_DWORD3);
}

template <class S> struct BufIO;
template <> struct BufIO<float> {
    __device__ static __forceinline__ float load(__amdgpu_buffer_rsrc_t r, uint32_t v, uint32_t s)
    {
        return __builtin_bit_cast(float,
                                  __builtin_amdgcn_raw_buffer_load_b32(r, int(v), int(s), BUF_LD));
    }
    __device__ static __forceinline__ void store(float x, __amdgpu_buffer_rsrc_t r, uint32_t v,
                                                 uint32_t s)
    {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, x), r, int(v), int(s),
                                              BUF_NT);
    }
};
template <> struct BufIO<double> {
    __device__ static __forceinline__ double load(__amdgpu_buffer_rsrc_t r, uint32_t v, uint32_t s)
    {
        return __builtin_bit_cast(double,
                                  __builtin_amdgcn_raw_buffer_load_b64(r, int(v), int(s), BUF_LD));
    }
    __device__ static __forceinline__ void store(double x, __amdgpu_buffer_rsrc_t r, uint32_t v,
                                                 uint32_t s)
    {
        using V2 = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0));
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V2, x), r, int(v), int(s), BUF_NT);
    }
};
template <> struct BufIO<__half> {
    __device__ static __forceinline__ __half load(__amdgpu_buffer_rsrc_t r, uint32_t v, uint32_t s)
    {
        return __builtin_bit_cast(__half,
                                  __builtin_amdgcn_raw_buffer_load_b16(r, int(v), int(s), BUF_LD));
    }
    __device__ static __forceinline__ void store(__half x, __amdgpu_buffer_rsrc_t r, uint32_t v,
                                                 uint32_t s)
    {
        __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, x), r, int(v),
                                              int(s), BUF_NT);
    }
};

// ---------------------------------------------------------------------------
// lattice traits (velocity order: rest, then +c/-c pairs shell by shell)
// ---------------------------------------------------------------------------
template <int LAT> struct Lattice;

template <> struct Lattice<0> {
    static constexpr int D = D2Q37_D, Q = D2Q37_Q, NS = D2Q37_NSHELL, MAXEQ = 4;
    // r^2 as R*R (not the separately rounded r^2) keeps xi^2 consistent with xi = R c
    static constexpr double R = d2q37_R, R2 = d2q37_R * d2q37_R;
    static constexpr int c(int i, int a) { return d2q37_C[i][a]; }
    static constexpr int shell(int i) { return d2q37_SHELL[i]; }
    static constexpr double wshell(int s) { return d2q37_WSHELL[s]; }
};

template <> struct Lattice<1> {
    static constexpr int D = D3Q39_D, Q = D3Q39_Q, NS = D3Q39_NSHELL, MAXEQ = 3;
    static constexpr double R = d3q39_R, R2 = d3q39_R * d3q39_R;
    static constexpr int c(int i, int a) { return d3q39_C[i][a]; }
    static constexpr int shell(int i) { return d3q39_SHELL[i]; }
    static constexpr double wshell(int s) { return d3q39_WSHELL[s]; }
};

template <class L> constexpr int c2(int i)
{
    return L::c(i, 0) * L::c(i, 0) + L::c(i, 1) * L::c(i, 1) + L::c(i, 2) * L::c(i, 2);
}

// ---------------------------------------------------------------------------
// storage conversion
// ---------------------------------------------------------------------------
// Every storage type holds the deviations h_i = f_i - w_i rho0.  LBM_F16DEV
// stores h_i * 2^k_i as binary16, with k_i = round(-log2 w_i): the exact
// power-of-two scale brings deviations of the size of w_i to about one, far
// from the subnormal range of binary16.
// The factor a stored value carries relative to the deviation it stands for:
// 1 for FP64 and FP32 storage (reduced-precision storage supplies its own).
struct UnitScale {
    template <int I> static constexpr double scale() { return 1.0; }
};

template <class L> struct DevScale {
    static constexpr int k(int i)
    {
        // k_i = round(-log2(w_i)): an exact power of two, chosen so that a
        // deviation comparable to w_i is stored near 1.
        double w = L::wshell(L::shell(i));
        int e = 0;
        while (w < 0.70710678118654752) {
            w *= 2.0;
            ++e;
        }
        return e;
    }
};

// ---------------------------------------------------------------------------
// argument blocks
// ---------------------------------------------------------------------------
// Population planes store rows of px >= nx values (nx rounded up to a multiple
// of 64), so that every row starts on a 128-byte line and a wavefront's run of
// 64 consecutive cells touches the fewest lines; values at x >= nx are never
// read or written.  Field arrays (moments, forces) are dense: cell =
// (z*ny + y)*nx + x.
constexpr int ROW_ALIGN = 64;

struct GridDims {
    int32_t nx, ny, nz;
    int32_t px;     // row pitch of the population planes
    int64_t N;      // cells, nx*ny*nz
    int64_t P;      // values per population plane, px*ny*nz
    DivU32 by_wpr;  // division by the wavefronts per row, ceil(nx / 64)
    DivU32 by_ny;   // division by ny
};

inline GridDims make_grid_dims(int64_t nx, int64_t ny, int64_t nz, int64_t px)
{
    return GridDims{int32_t(nx), int32_t(ny), int32_t(nz), int32_t(px), nx * ny * nz,
                    px * ny * nz, make_divu32(uint32_t((nx + 63) / 64)),
                    make_divu32(uint32_t(ny))};
}

struct ForceDesc {
    int32_t kind;  // 0 uniform, 1 axis profile, 2 field
    int32_t axis;  // profile axis
    int64_t len;   // profile length
    double g[3];   // uniform value
    const void *tab;  // profile (D*len) or field (D*N), arithmetic precision
};

struct StepCoef {
    double om;   // 1/tau^
    double cf;   // 1 - 1/(2 tau^)
    double rho0; // reference density of the stored deviations
    double mu;   // > 0: per-cell tau^ = mu/(rho theta) + 1/2 replaces om and cf
};

// Plates normal to y at y = -1/2 and y = ny - 1/2 (lbm_set_walls): a population
// whose streaming source lies behind a plate is the plate's emission
// rw[side][column of the source] * e[side][i]; populations streaming into a
// plate stay in their slots at the node they leave (the "crossing" slots).
// A plate's density rw over column (x, z) is the sum of the
// slots of the rows next to it whose next move crosses it, over the plate's
// normalisation e_Q.  Those sums are kept per row ("partial sums": rows 0, 1, 2
// for the bottom plate, ny-3+k for the top one; the same rows for both when
// ny < 3), for each of the two population buffers: the step that writes a
// buffer also writes its partial sums, and the next step adds the (at most 3)
// rows of a column in order.
struct WallDesc {
    int32_t on;
    int32_t par;      // buffer holding the state read (0 or 1): its sums are part[par]
    double *part;     // [2 buffer][2 plate][3 row][nx*nz] partial sums (bottom, top)
    const double *e;  // [2][Q + 1]: e_i = f0_i(1, (U_w, 0, 0), theta_w), then the normalisation
};

__host__ __device__ inline int64_t wall_part_index(int par, int side, int k, int64_t ncol,
                                                   int64_t col)
{
    return ((int64_t(par) * 2 + side) * 3 + k) * ncol + col;
}

// One member of a multi-grid batch (device table entry).  Its tiles are runs
// of 64 cells along x (one wavefront each): chunks_x per grid row, rows in
// (z, y) order.
struct TileSim {
    const void *pop[2];  // the two population buffers
    uint32_t *ctr;       // step counter pair (F16 stochastic rounding keys), see LaunchCfg
    int32_t cur;         // buffer holding the state when the table was built
    int32_t chunks_x;    // tiles per grid row, ceil(nx / 64)
    int64_t tile_begin;  // first tile of this simulation in the list
    GridDims gd;
    ForceDesc fd;
    StepCoef co;
    WallDesc wd;         // plates (off for a periodic member); wd.par is set per step
};

// Periodic wrap of v in [-3, n + 3) into [0, n), valid for any n >= 1.
__device__ __forceinline__ int wrap3(int v, int n)
{
    if (n >= 4) {
        v += (v < 0) ? n : 0;
        v -= (v >= n) ? n : 0;
        return v;
    }
    while (v < 0) v += n;
    while (v >= n) v -= n;
    return v;
}

// ---------------------------------------------------------------------------
// body force at a cell
// ---------------------------------------------------------------------------
// TT: element type of the force table (the arithmetic precision of the
// storage), TO: output type.
template <class TT, class TO, int D>
__device__ __forceinline__ void load_force(const ForceDesc &fd, const GridDims &gd, int x, int y,
                                           int z, int64_t cell, TO g[3])
{
    g[0] = g[1] = g[2] = TO(0);
    if (fd.kind == 0) {
        for (int a = 0; a < D; ++a) g[a] = TO(TT(fd.g[a]));
    } else if (fd.kind == 1) {
        const TT *tab = static_cast<const TT *>(fd.tab);
        const int k = fd.axis == 0 ? x : (fd.axis == 1 ? y : z);
        for (int a = 0; a < D; ++a) g[a] = TO(tab[a * fd.len + k]);
    } else {
        const TT *tab = static_cast<const TT *>(fd.tab);
        for (int a = 0; a < D; ++a) g[a] = TO(tab[a * gd.N + cell]);
    }
}

// ---------------------------------------------------------------------------
// per-cell state after the moment pass
// ---------------------------------------------------------------------------
template <class T> struct CellState {
    T rho;
    T drho;      // rho - rho0
    T ub[3];     // mid-point velocity u~ + g/2
    T th;        // mid-point temperature
    T g[3];
    T sig[3][3]; // mid-point deviatoric stress (traceless), zero unless needed
    T om;        // 1/tau^ of this cell
    T cf;        // 1 - 1/(2 tau^) of this cell
};

// Raw sums of one cell over the stored deviations h_i = f_i - w_i rho0:
// drho = sum h, j = sum h c (integer c), P = sum h c c.  Because the weights
// satisfy sum w = 1, sum w c = 0 and sum w c c = delta / r^2, the moments of f
// follow as rho = rho0 + drho, sum f xi = r j, sum f xi xi = rho0 delta + r^2 P.
template <class T> struct RawSums {
    T drho, j[3], P[3][3];
};

//
// SC::scale<i>() is the factor the values carry (1, or the power of two of
// reduced-precision storage, the same for every velocity of a shell): the
// sums take it out through their constants, so scaled and unscaled inputs
// give bitwise the same sums.
template <class L, class T, class SC = UnitScale>
__device__ __forceinline__ RawSums<T> raw_sums(const T (&h)[L::Q])
{
    RawSums<T> s;
    constexpr double u0 = 1.0 / SC::template scale<0>();
    s.drho = (u0 == 1.0) ? h[0] : h[0] * T(u0);
    for (int a = 0; a < 3; ++a) {
        s.j[a] = T(0);
        for (int b = 0; b < 3; ++b) s.P[a][b] = T(0);
    }
    static_for<0, (L::Q - 1) / 2>([&](auto K) {
        constexpr int ip = 1 + 2 * decltype(K)::value;
        constexpr int im = ip + 1;
        static_assert(SC::template scale<ip>() == SC::template scale<im>(),
                      "a pair shares its scale");
        constexpr double u = 1.0 / SC::template scale<ip>();  // exact: a power of two
        const T sp = h[ip] + h[im];
        const T dm = h[ip] - h[im];
        // acc += m * v with the scale folded into m: one rounding, as unscaled
        auto add = [&](T &acc, int m, T v) {
            if (u == 1.0 && m == 1) acc += v;
            else if (u == 1.0 && m == -1) acc -= v;
            else acc = fma_t(v, T(m * u), acc);
        };
        add(s.drho, 1, sp);
        static_for<0, L::D>([&](auto A) {
            constexpr int a = decltype(A)::value;
            constexpr int ca = L::c(ip, a);
            if constexpr (ca != 0) add(s.j[a], ca, dm);
            static_for<a, L::D>([&](auto B) {
                constexpr int b = decltype(B)::value;
                constexpr int cab = ca * L::c(ip, b);
                if constexpr (cab != 0) add(s.P[a][b], cab, sp);
            });
        });
    });
    return s;
}

// Mid-point moments, relaxation coefficients and (if WITH_SIGMA) sigma-bar
// from the raw sums.
//   rho = rho0 + drho, u = r j / rho + g/2,
//   theta = (E/rho - |u~|^2 + |g|^2/4)/D with E = rho0 D + r^2 tr P;
//   tau^ = the run's constant, or mu/(rho theta) + 1/2 when mu > 0 (the
//   relaxation time that keeps the dynamic viscosity constant, Sec. 3);
//   sigma-bar = -cf [sum f xi xi - rho(u u + theta delta) + rho (u g + g u)/2]
//   with its trace removed.  The isotropic parts (rho0 delta and
//   rho theta delta) drop out of the traceless projection exactly, so they are
//   left out: sigma-bar = dev(-cf [r^2 P - rho u u + rho (u g + g u)/2]).
template <class L, class T, bool WITH_SIGMA>
__device__ __forceinline__ void finish_moments(const RawSums<T> &s, const T g[3],
                                               const StepCoef &co, CellState<T> &cs)
{
    constexpr int D = L::D;
    const T r = T(L::R), r2 = T(L::R2);
    const T rho0 = T(co.rho0);
    const T rho = rho0 + s.drho;
    const T inv = T(1) / rho;
    T ut2 = T(0), g2 = T(0), tr = T(0);
    cs.rho = rho;
    cs.drho = s.drho;
    for (int a = 0; a < 3; ++a) {
        cs.g[a] = g[a];
        cs.ub[a] = T(0);
    }
    for (int a = 0; a < D; ++a) {
        const T ut = r * s.j[a] * inv;
        cs.ub[a] = ut + T(0.5) * g[a];
        ut2 += ut * ut;
        g2 += g[a] * g[a];
        tr += s.P[a][a];
    }
    const T E = rho0 * T(D) + r2 * tr;
    cs.th = (E * inv - ut2 + T(0.25) * g2) * T(1.0 / D);
    cs.om = T(co.om);
    cs.cf = T(co.cf);
    if (co.mu > 0.0) {  // uniform over the launch
        cs.om = T(1) / (T(co.mu) / (rho * cs.th) + T(0.5));
        cs.cf = T(1) - T(0.5) * cs.om;
    }
    const T cf = cs.cf;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) cs.sig[a][b] = T(0);
    if constexpr (WITH_SIGMA) {
        T str = T(0);
        for (int a = 0; a < D; ++a) {
            for (int b = a; b < D; ++b) {
                T v = r2 * s.P[a][b] - rho * cs.ub[a] * cs.ub[b]
                      + T(0.5) * rho * (cs.ub[a] * g[b] + g[a] * cs.ub[b]);
                v *= -cf;
                cs.sig[a][b] = v;
                cs.sig[b][a] = v;
            }
            str += cs.sig[a][a];
        }
        for (int a = 0; a < D; ++a) cs.sig[a][a] -= str * T(1.0 / D);
    }
}

// ---------------------------------------------------------------------------
// alpha * f0 + beta * F for every velocity, in even/odd pair form.
//
// For velocity xi_i in shell s (xi^2 = X2) with xu = xi.u, xg = xi.g,
// u2 = |u|^2, t = theta - 1, gu = g.u:
//   f0 = w rho [ e(xu^2) + o(xu) ],  e even, o odd in xi:
//     e = 1 + (xu^2 - u2 + t(X2 - D))/2
//         + [xu^4 - 6 xu^2 u2 + 3 u2^2 + 6t(xu^2(X2 - D - 4) + u2(D + 2 - X2))
//            + 3t^2(X2^2 - 2(D+2) X2 + D(D+2))]/24            (N = 4)
//     o = xu [1 + (xu^2 - 3 u2 + 3t(X2 - D - 2))/6]           (N >= 3; xu for N = 2)
//   F (eq. (fi)) even part  w rho (xg xu - gu)                (order >= 2)
//     odd part  w rho xg                                       (order 1, 2)
//               w rho [xg (1 + (xu^2 - u2 + t(X2 - D - 2))/2) - gu xu]   (order >= 3)
//               - (w/2) [xg (xi.sigma.xi) - 2 xi.sigma.g]     (order 4)
// With NO_BASE the even part omits alpha * w * rho (the leading term of f0),
// so that callers can add it as an exactly rounded increment.  With a scale
// SC every w is w * SC::scale<i>() (a power of two): even and odd come out
// multiplied by it exactly.
// The callback receives (i_plus, i_minus, even, odd) for each pair and
// (0, -1, even, 0) for the rest velocity; the indices are passed as
// std::integral_constant so that callers index register arrays statically.
// ---------------------------------------------------------------------------
template <class L, class T, int EQ, int FO, bool NO_BASE = false, class SC = UnitScale,
          class CB>
__device__ __forceinline__ void combo_pairs(const CellState<T> &cs, T alpha, T beta, CB &&cb)
{
    constexpr int D = L::D;
    const T r = T(L::R), r2 = T(L::R2);
    T ur[3], gr[3], hr[3], sr[3][3];
    T u2 = T(0), gu = T(0);
    for (int a = 0; a < 3; ++a) {
        ur[a] = r * cs.ub[a];
        gr[a] = r * cs.g[a];
        hr[a] = T(0);
    }
    for (int a = 0; a < D; ++a) {
        u2 += cs.ub[a] * cs.ub[a];
        gu += cs.g[a] * cs.ub[a];
    }
    if constexpr (FO == 4) {
        for (int a = 0; a < D; ++a) {
            T h = T(0);
            for (int b = 0; b < D; ++b) {
                h += cs.sig[a][b] * cs.g[b];
                sr[a][b] = r2 * cs.sig[a][b];
            }
            hr[a] = r * h;
        }
    }
    const T t = cs.th - T(1);
    const T rho = cs.rho;

    // The shell constants below are polynomials in the shell's X2 = |xi|^2 (a
    // compile-time value) with coefficients that depend on the cell only:
    // computed once here, each shell then costs a Horner step per polynomial.
    //   e0 - 1 (the even constant without its leading 1) = E0 + E1 X2 + E2 X2^2
    //   e1 (even, times xu^2)                             = D0 + D1 X2
    //   o0 (odd, times xu)                                = G0 + G1 X2
    const T half_t = T(0.5) * t;
    T E0 = T(-0.5) * (t * T(D) + u2), E1 = half_t, E2 = T(0);
    T D0 = T(0.5), D1 = T(0);
    if constexpr (!NO_BASE) E0 += T(1);
    if constexpr (EQ == 4) {
        // [3 u2^2 + 6 t u2 (D + 2 - X2) + 3 t^2 (X2^2 - 2 (D + 2) X2 + D (D + 2))] / 24
        const T tt = t * t;
        E0 += T(0.125) * u2 * u2 + T(0.25 * (D + 2)) * t * u2 + T(0.125 * D * (D + 2)) * tt;
        E1 -= T(0.25) * (t * u2 + T(D + 2) * tt);
        E2 = T(0.125) * tt;
        // (t (X2 - D - 4) - u2) / 4
        D0 -= T(0.25) * (t * T(D + 4) + u2);
        D1 = T(0.25) * t;
    }
    const T G0 = T(1) - T(0.5) * u2 - half_t * T(D + 2), G1 = half_t;
    const T arho = alpha * rho;  // A = ws arho multiplies the equilibrium bracket
    const T brho = beta * rho;   // Bf = ws brho multiplies the force bracket
    const T brgu = brho * gu;
    const T hbeta = T(0.5) * beta;

    // per-shell constants, recomputed at the first pair of each shell
    T K0 = T(0), Ka = T(0), Kq = T(0), K6 = T(0), Kb = T(0), Kb2 = T(0), Kw = T(0), K24 = T(0);
    T Kbf = T(0);
    auto shell_consts = [&](auto S) {
        constexpr int s = decltype(S)::value;
        // any velocity of the shell gives X2
        constexpr int iref = [] {
            int i = 0;
            while (L::shell(i) != s) ++i;
            return i;
        }();
        const T X2 = T(L::R2 * c2<L>(iref));
        // the shell's weight times the scale its values carry (a power of two):
        // every constant below is linear in it, so even and odd come out
        // scaled, rounding for rounding
        const T ws = T(L::wshell(s) * SC::template scale<iref>());
        const T A = ws * arho;
        const T Bf = ws * brho;
        const T e0t = (EQ == 4) ? fma_t(fma_t(E2, X2, E1), X2, E0) : fma_t(E1, X2, E0);
        const T o0 = fma_t(G1, X2, G0);
        if constexpr (FO >= 2) K0 = ws * fma_t(arho, e0t, -brgu);  // A e0 - Bf gu
        else K0 = A * e0t;
        Ka = (EQ == 4) ? A * fma_t(D1, X2, D0) : A * T(0.5);
        if constexpr (EQ >= 3) {
            Kq = (FO >= 3) ? ws * fma_t(arho, o0, -brgu) : A * o0;  // odd, times xu
            K6 = A * T(1.0 / 6.0);                                   // odd, times xu^3
        } else {
            Kq = (FO >= 3) ? ws * (arho - brgu) : A;
            K6 = T(0);
        }
        if constexpr (EQ == 4) K24 = A * T(1.0 / 24.0);
        if constexpr (FO >= 3) {
            Kb = Bf * o0;         // odd, times xg
            Kb2 = Bf * T(0.5);    // odd, times xg xu^2
        } else {
            Kb = Bf;
            Kb2 = T(0);
        }
        Kbf = Bf;                 // even, times xg xu
        Kw = hbeta * ws;          // (beta w / 2) for the sigma terms
    };

    // rest velocity
    shell_consts(std::integral_constant<int, L::shell(0)>{});
    cb(std::integral_constant<int, 0>{}, std::integral_constant<int, -1>{}, K0, T(0));

    static_for<0, (L::Q - 1) / 2>([&](auto K) {
        constexpr int ip = 1 + 2 * decltype(K)::value;
        constexpr int im = ip + 1;
        constexpr int s = L::shell(ip);
        if constexpr (L::shell(ip - 1) != s) shell_consts(std::integral_constant<int, s>{});
        constexpr int cx = L::c(ip, 0), cy = L::c(ip, 1), cz = L::c(ip, 2);
        // xi.u and xi.g with compile-time integer components
        auto dot = [&](const T v[3]) {
            T acc = T(0);
            bool first = true;
            static_for<0, 3>([&](auto A) {
                constexpr int a = decltype(A)::value;
                constexpr int ca = (a == 0 ? cx : (a == 1 ? cy : cz));
                if constexpr (ca != 0) {
                    if (first) {
                        acc = (ca == 1) ? v[a] : ((ca == -1) ? -v[a] : T(ca) * v[a]);
                        first = false;
                    } else {
                        if constexpr (ca == 1) acc += v[a];
                        else if constexpr (ca == -1) acc -= v[a];
                        else acc += T(ca) * v[a];
                    }
                }
            });
            return acc;
        };
        const T xu = dot(ur);
        const T xu2 = xu * xu;
        T ev = K0 + Ka * xu2;
        if constexpr (EQ == 4) ev += K24 * xu2 * xu2;
        T od = xu * (Kq + K6 * xu2);
        if constexpr (FO >= 1) {
            const T xg = dot(gr);
            if constexpr (FO >= 2) ev += Kbf * (xg * xu);
            T gterm = Kb + Kb2 * xu2;
            if constexpr (FO == 4) {
                // xi.sigma.xi = r^2 c.sigma.c and xi.sigma.g = r c.(sigma g)
                T S = T(0);
                static_for<0, 3>([&](auto A) {
                    constexpr int a = decltype(A)::value;
                    constexpr int ca = (a == 0 ? cx : (a == 1 ? cy : cz));
                    static_for<a, 3>([&](auto B) {
                        constexpr int b = decltype(B)::value;
                        constexpr int cb_ = (b == 0 ? cx : (b == 1 ? cy : cz));
                        constexpr int m = (a == b) ? ca * cb_ : 2 * ca * cb_;
                        if constexpr (m != 0) S += T(m) * sr[a][b];
                    });
                });
                const T hxi = dot(hr);
                gterm -= Kw * S;
                od += T(2) * Kw * hxi;
            }
            od += xg * gterm;
        }
        cb(std::integral_constant<int, ip>{}, std::integral_constant<int, im>{}, ev, od);
    });
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

struct LaunchCfg {
    int block;  // threads along x per block
    hipStream_t stream;
    WallDesc walls;  // off unless the handle has plates
    uint32_t *ctr;   // the handle's step counter pair (keys of the F16 stochastic rounding)
    int cur;         // buffer holding the state read: the step reads ctr[cur], writes ctr[cur ^ 1]
};

// Generic entry points (lbm_dispatch.hip), switching on lattice and storage.
hipError_t launch_pattern(int lat, int storage, const void *A, void *B, const GridDims &gd,
                          const LaunchCfg &lc);
hipError_t launch_step(int lat, int storage, int eq, int fo, const void *A, void *B,
                       const GridDims &gd, const ForceDesc &fd, const StepCoef &co,
                       const LaunchCfg &lc);
hipError_t launch_init(int lat, int storage, int eq, int fo, const double *rho, const double *u,
                       const double *theta, void *A, const GridDims &gd, const ForceDesc &fd,
                       const StepCoef &co, const LaunchCfg &lc);
hipError_t launch_moments(int lat, int storage, const void *A, double *rho, double *u,
                          double *theta, const GridDims &gd, const ForceDesc &fd,
                          const StepCoef &co, const LaunchCfg &lc);
hipError_t launch_heat_flux(int lat, int storage, int eq, int fo, const void *A, double *q,
                            const GridDims &gd, const ForceDesc &fd, const StepCoef &co,
                            const LaunchCfg &lc);
hipError_t launch_totals(int lat, int storage, const void *A, double *partials, double *out_dev,
                         const GridDims &gd, const StepCoef &co, hipStream_t stream);
hipError_t launch_convert(int storage, const double *src, void *dst, int64_t n,
                          hipStream_t stream);
// One launch of the multi-grid step: tile list, its members, launch shape.
struct BatchLaunch {
    const int64_t *begin;   // device: first tile of member k (k < nsims), ascending
    const TileSim *table;   // device: the members
    int nsims;
    int64_t ntiles;         // tiles of all members
    int parity;             // batch steps since the table was built, mod 2
    int threads;            // threads per block (64, 128 or 256): 1, 2 or 4 tiles
    int64_t blocks;         // 0: one block per tile; > 0: persistent walk
    hipStream_t stream;
    bool walls;             // some member has plates (the kernel variant that handles them)
};
hipError_t launch_multi_step(int lat, int storage, int eq, int fo, const BatchLaunch &bl);
// plates: emission tables, the row sums of a state no step produced, and the
// step of a grid between plates
hipError_t launch_wall_setup(int lat, int eq, const double *theta, const double *uw, int64_t ny,
                             double *e, hipStream_t stream);
hipError_t launch_wall_mass(int lat, int storage, const void *A, const GridDims &gd,
                            const StepCoef &co, const LaunchCfg &lc);
hipError_t launch_wall_step(int lat, int storage, int eq, int fo, const void *A, void *B,
                            const GridDims &gd, const ForceDesc &fd, const StepCoef &co,
                            const LaunchCfg &lc);

// Per-lattice / per-storage pieces, each explicitly instantiated in its own
// translation unit (step_*.hip, aux_*.hip) so that the build parallelises.
template <int LAT, class S>
hipError_t launch_step_ls(int eq, int fo, const void *A, void *B, const GridDims &gd,
                          const ForceDesc &fd, const StepCoef &co, const LaunchCfg &lc);
template <int LAT, class S>
hipError_t launch_multi_step_ls(int eq, int fo, const BatchLaunch &bl);
template <int LAT, class S>
hipError_t launch_wall_step_ls(int eq, int fo, const void *A, void *B, const GridDims &gd,
                               const ForceDesc &fd, const StepCoef &co, const LaunchCfg &lc);
template <int LAT, class S>
hipError_t launch_pattern_ls(const void *A, void *B, const GridDims &gd, const LaunchCfg &lc);
template <int LAT>
hipError_t launch_wall_setup_l(int eq, const double *theta, const double *uw, int64_t ny,
                               double *e, hipStream_t stream);
template <int LAT>
hipError_t launch_wall_mass_l(int storage, const void *A, const GridDims &gd, const StepCoef &co,
                              const LaunchCfg &lc);
template <int LAT, class S>
hipError_t launch_init_ls(int eq, int fo, const double *rho, const double *u, const double *theta,
                          void *A, const GridDims &gd, const ForceDesc &fd, const StepCoef &co,
                          const LaunchCfg &lc);
template <int LAT, class S>
hipError_t launch_moments_ls(const void *A, double *rho, double *u, double *theta,
                             const GridDims &gd, const ForceDesc &fd, const StepCoef &co,
                             const LaunchCfg &lc);
template <int LAT, class S>
hipError_t launch_heat_flux_ls(int eq, int fo, const void *A, double *q, const GridDims &gd,
                               const ForceDesc &fd, const StepCoef &co, const LaunchCfg &lc);
template <int LAT>
hipError_t launch_totals_l(int storage, const void *A, double *partials, double *out_dev,
                           const GridDims &gd, const StepCoef &co, hipStream_t stream);

constexpr int TOTALS_BLOCKS = 512;  // fixed partition: results independent of launch shape

}  // namespace lbm
