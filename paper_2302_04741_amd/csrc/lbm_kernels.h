// HIP kernel templates of the gfx950 thermal LBM library.
//
//   step_kernel      one fused time step of eq. (lbm) (Li & Shan, arXiv:2302.04741,
//                    Sec. 2): pull streaming, moments, mid-point values,
//                    sigma-bar, Hermite equilibrium, Hermite force eq. (fi), BGK
//                    relaxation, store.  One thread per cell, SoA populations.
//   init_kernel      f~ = f0 - F/2 at step 0 (sigma = 0), written in pull layout.
//   moments_kernel   physical rho, u + g/2, theta in FP64.
//   heatflux_kernel  q = 1/2 sum_i f_i |xi_i - u|^2 (xi_i - u) of the physical f.
//   totals kernels   FP64 sums of the stored populations in a fixed order.
//
// Layout: populations are SoA planes, A[i*P + (z*ny + y)*px + x], rows padded
// to px = nx rounded up to 64 values (P = px*ny*nz), holding the deviations
// h_i = f~_i - w_i rho0 (scaled by 2^k_i for F16); the padding is never read.
// The stored state is post-collision ("pull" layout): the pre-collision value
// of velocity i at cell x is plane i at x - c_i (periodic).  A step reads every
// grid element of A exactly once (a permutation per plane) and writes every
// grid element of B exactly once, at the thread's own cell.
#pragma once

#include "lbm_internal.h"

namespace lbm {

// ---------------------------------------------------------------------------
// storage codecs: S = stored type, T = arithmetic type; both sides are h_i
// ---------------------------------------------------------------------------
template <class S> struct ArithOf;
template <> struct ArithOf<double> { using type = double; };
template <> struct ArithOf<float> { using type = float; };
template <> struct ArithOf<__half> { using type = float; };

// Random bits of the F16 stochastic rounding.  One 32-bit key per (cell,
// step): the cell index and the step number combined linearly, then the
// 32-bit finalizer of MurmurHash3 (Appleby) to spread every input bit over
// the word.  The cell's stores then walk a 32-bit linear congruential
// sequence from that key (Knuth's multiplier 6364136223846793005 reduced to
// its low word, odd increment), each store taking the current word whole as
// the seed of its conversion (half_sr reads its top 13 bits, the sequence's
// best ones).  Nothing depends on the launch shape, the batch or the other
// members.
__device__ __forceinline__ uint32_t sr_key(uint32_t cell, uint32_t step)
{
    uint32_t h = cell * 0x9E3779B1u + step * 0x85EBCA77u;
    h ^= h >> 16;
    h *= 0x85EBCA6Bu;
    h ^= h >> 13;
    h *= 0xC2B2AE35u;
    h ^= h >> 16;
    return h;
}
struct SrStream {
    uint32_t x;
    __device__ __forceinline__ uint32_t next()
    {
        const uint32_t r = x;
        x = x * 0x4C957F2Du + 0x2545F491u;
        return r;
    }
};

// float -> binary16 with stochastic rounding: a value between two
// neighbouring halves a < v < b rounds to b with probability (v - a)/(b - a),
// so the rounding error has zero mean whatever v is.  gfx950 does this in one
// instruction (v_cvt_sr_f16_f32).  Measured on an MI355X over 196,608 random
// values in the normal half range, it equals: add the seed's top 13 bits
// (seed >> 19) to the FP32 bit pattern (sign and magnitude) below the 13 bits
// binary16 drops, then drop them; in the subnormal half range it rounds
// stochastically at the subnormal spacing 2^-24 (the up-rounding frequency
// matched the fraction within sampling error on 32 values x 32,768 seeds).
__device__ __forceinline__ __half half_sr(float v, uint32_t seed)
{
    // the instruction writes the low half of its destination and keeps the
    // high half of the tied operand, here v's own register (no extra move)
    typedef _Float16 H2 __attribute__((ext_vector_type(2)));
    const H2 r = __builtin_amdgcn_cvt_sr_f16_f32(__builtin_bit_cast(H2, v), v, seed, false);
    return __builtin_bit_cast(__half, r.x);
}

// load/store convert between a stored value and the deviation h_i it stands
// for; load_scaled/store_scaled keep the factor scale<I>() the stored value
// carries (the fused step works on scaled values: see raw_sums, combo_pairs).
template <class L, class S> struct Codec {
    static constexpr bool STOCHASTIC = false;
    template <int I> static constexpr double scale() { return 1.0; }
    template <int I, class T> __device__ static __forceinline__ T load(S v) { return T(v); }
    template <int I, class T> __device__ static __forceinline__ S store(T h) { return S(h); }
    template <int I, class T> __device__ static __forceinline__ T load_scaled(S v) { return T(v); }
    template <int I, class T> __device__ static __forceinline__ S store_scaled(T h, SrStream &)
    {
        return S(h);
    }
};

// F16 deviations: stored value h_i 2^k_i, k_i = round(-log2 w_i).  The step
// stores with stochastic rounding (store_scaled); the initial state and the
// kernels off the step path round to nearest (store).
template <class L> struct Codec<L, __half> {
    static constexpr bool STOCHASTIC = true;
    template <int I> static constexpr double scale()
    {
        double s = 1.0;
        for (int e = 0; e < DevScale<L>::k(I); ++e) s *= 2.0;
        return s;
    }
    template <int I, class T> __device__ static __forceinline__ T load(__half v)
    {
        constexpr double inv = 1.0 / scale<I>();  // exact: a power of two
        return T(__half2float(v)) * T(inv);
    }
    template <int I, class T> __device__ static __forceinline__ __half store(T h)
    {
        constexpr double sc = scale<I>();
        return __float2half_rn(float(h * T(sc)));
    }
    template <int I, class T> __device__ static __forceinline__ T load_scaled(__half v)
    {
        return T(__half2float(v));
    }
    // stochastic rounding (half_sr), seeded by the next word of the cell's stream
    template <int I, class T> __device__ static __forceinline__ __half store_scaled(T h,
                                                                                   SrStream &rng)
    {
        return half_sr(float(h), rng.next());
    }
};

// ---------------------------------------------------------------------------
// pull gather: h_i = A[i][x - c_i (periodic)]
// ---------------------------------------------------------------------------
// Deviation h_i = f_i - w_i rho0 that the plate emits into (x, y, z) along c_i
// (the source (x, y, z) - c_i lies behind the plate: side 0 below, 1 above).
template <class L>
__device__ __forceinline__ double wall_emitted(const WallDesc &wd, const GridDims &gd, int i,
                                               double w, double rho0, int x, int y, int z)
{
    const int side = y - L::c(i, 1) < 0 ? 0 : 1;
    const int xv = wrap3(x - L::c(i, 0), gd.nx);
    const int zv = (L::D == 3) ? wrap3(z - L::c(i, 2), gd.nz) : 0;
    const int64_t ncol = int64_t(gd.nx) * gd.nz;
    const int64_t col = int64_t(zv) * gd.nx + xv;
    // the plate's density over the source column: its rows' sums, in order
    double m = wd.part[wall_part_index(wd.par, side, 0, ncol, col)];
    if (gd.ny > 1) m += wd.part[wall_part_index(wd.par, side, 1, ncol, col)];
    if (gd.ny > 2) m += wd.part[wall_part_index(wd.par, side, 2, ncol, col)];
    const double rw = m / wd.e[side * (L::Q + 1) + L::Q];
    return rw * wd.e[side * (L::Q + 1) + i] - w * rho0;
}

template <class L, class S, class T, bool WALLS = false>
__device__ __forceinline__ void gather(const S *__restrict__ A, const GridDims &gd, int x, int y,
                                       int z, T (&h)[L::Q], const WallDesc *wd = nullptr,
                                       double rho0 = 0.0)
{
    // x offsets are per lane (7 distinct byte offsets); y and z are uniform over
    // the wavefront, so each row offset and each plane resource is a scalar.
    uint32_t xs[7];
    int ys[7], zs[7];
#pragma unroll
    for (int d = 0; d < 7; ++d) {
        xs[d] = uint32_t(wrap3(x - (d - 3), gd.nx)) * uint32_t(sizeof(S));
        ys[d] = wrap3(y - (d - 3), gd.ny);
        zs[d] = (L::D == 3) ? wrap3(z - (d - 3), gd.nz) : 0;
    }
    const int64_t P = gd.P;
    const uint32_t plane_bytes = uint32_t(P * int64_t(sizeof(S)));
    static_for<0, L::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        constexpr int cx = L::c(i, 0), cy = L::c(i, 1), cz = L::c(i, 2);
        if constexpr (WALLS) {
            const int ysrc = y - cy;  // uniform over the block
            if (ysrc < 0 || ysrc >= gd.ny) {
                constexpr double sc = Codec<L, S>::template scale<i>();  // a power of two
                h[i] = T(sc * wall_emitted<L>(*wd, gd, i, L::wshell(L::shell(i)), rho0, x, y,
                                              z));
                return;
            }
        }
        const uint32_t row =
            uint32_t((int64_t(zs[cz + 3]) * gd.ny + ys[cy + 3]) * gd.px) * uint32_t(sizeof(S));
        const auto r = plane_rsrc(A + int64_t(i) * P, plane_bytes);
        h[i] = Codec<L, S>::template load_scaled<i, T>(BufIO<S>::load(r, xs[cx + 3], row));
    });
}

// ---------------------------------------------------------------------------
// K1: fused step
// ---------------------------------------------------------------------------
// Largest block of the step kernel: FP64 arithmetic needs more than 128 VGPRs
// per lane, so its blocks stay at 256 threads (4 waves).
template <class S> constexpr int step_max_threads()
{
    return sizeof(typename ArithOf<S>::type) == 8 ? 256 : 1024;
}

// Default block of the step, measured: 4 wavefronts, except 16 for D3Q39 FP32
// storage on grids of at least 2^17 wavefronts (256^3: +2%, 384^3: +2%; on
// smaller D3Q39 grids and on every D2Q37 grid 16-wavefront blocks lose 5-20%,
// F16 storage loses 5% with them) and 2 for FP64 storage (D3Q39 256^3: +6%,
// D2Q37 1024^2: +4% over 4; FP64 cannot use more than 4).
template <int LAT, class S> inline int step_default_threads(int64_t waves)
{
    if (sizeof(S) == 8) return 128;
    return (LAT == 1 && sizeof(S) == 4 && waves >= (int64_t(1) << 17)) ? 1024 : 256;
}

// The fused update of one cell (x, y, z): gather, moments, equilibrium, stress,
// force, relaxation, store.  y and z must be uniform over the wavefront.
// `step` is the step number (the state read is after `step` steps): with F16
// storage it keys the stochastic rounding of every value stored.
template <int LAT, class S, int EQ, int FO, bool WALLS = false>
__device__ __forceinline__ void step_cell(const S *__restrict__ A, S *__restrict__ B,
                                          const GridDims &gd, const ForceDesc &fd,
                                          const StepCoef &co, int x, int y, int z,
                                          uint32_t step, const WallDesc *wd = nullptr)
{
    using L = Lattice<LAT>;
    using T = typename ArithOf<S>::type;
    const int64_t P = gd.P;
    const int64_t row = int64_t(z) * gd.ny + y;  // uniform
    const int64_t rowbase = row * gd.px;          // padded population row
    const int64_t cell = row * gd.nx + x;         // dense field index
    // one population plane is < 4 GiB (checked at creation), so 32-bit byte
    // offsets address it

    // h holds the deviations as stored, times Codec::scale<i>() (1 unless the
    // storage is reduced-precision); the sums and the pair terms take the
    // scale through their constants, so no value is rescaled on the way.
    using C = Codec<L, S>;
    SrStream rng{C::STOCHASTIC ? sr_key(uint32_t(cell), step) : 0u};
    T h[L::Q];
    gather<L, S, T, WALLS>(A, gd, x, y, z, h, wd, co.rho0);
    T g[3];
    load_force<T, T, L::D>(fd, gd, x, y, z, cell, g);

    const RawSums<T> rs = raw_sums<L, T, C>(h);
    CellState<T> cs;
    finish_moments<L, T, FO == 4>(rs, g, co, cs);

    // h* = h + om (f0 - f) + cf F with f0 - f = w drho + (f0 - w rho) - h.
    // The bracket [om (f0 - w rho) + cf F] is what combo_pairs returns with
    // NO_BASE (even +- odd part).  FP32 arithmetic: h* = (1 - om) h + [om w
    // drho + bracket], a pair sharing q = fma(om w, drho, even), each
    // population one fma(1 - om, h, q +- odd) (1 - om is exact: om = 1/tau^
    // lies in [1/2, 2]).  FP64 arithmetic keeps h + fma(om, fma(w, drho, -h),
    // even +- odd), which needs one register less per lane (the other form
    // takes its D3Q39 step from three wavefronts per SIMD to two).  Either way
    // every term is a small deviation, so the rounding stays at the size of h.
    constexpr bool SHARED_Q = sizeof(T) == 4;
    const T om = cs.om;
    const T omc = T(1) - om;
    const T drho = cs.drho;
    const uint32_t xo = uint32_t(x) * uint32_t(sizeof(S));
    const uint32_t ro = uint32_t(rowbase) * uint32_t(sizeof(S));
    const uint32_t plane_bytes = uint32_t(P * int64_t(sizeof(S)));
    // with plates: the partial sums of the state written here (the slots whose
    // next move crosses a plate, as stored), for the next step's emission
    double ps[2] = {0.0, 0.0};
    auto account = [&](auto II, S stored) {
        if constexpr (WALLS) {
            constexpr int i = decltype(II)::value;
            constexpr int cy = L::c(i, 1);
            if constexpr (cy != 0) {
                const double v = Codec<L, S>::template load<i, double>(stored) +
                                 L::wshell(L::shell(i)) * co.rho0;
                if constexpr (cy < 0) ps[0] += (y + cy < 0) ? v : 0.0;
                else ps[1] += (y + cy >= gd.ny) ? v : 0.0;
            }
        }
    };
    combo_pairs<L, T, EQ, FO, true, C>(cs, om, cs.cf, [&](auto IP, auto IM, T ev, T od) {
        constexpr int ip = decltype(IP)::value;
        constexpr int im = decltype(IM)::value;
        constexpr double w = L::wshell(L::shell(ip)) * C::template scale<ip>();
        T q = T(0);
        if constexpr (SHARED_Q) q = fma_t(om * T(w), drho, ev);
        auto relaxed = [&](T hi, T sign_od) {
            if constexpr (SHARED_Q) return fma_t(omc, hi, q + sign_od);
            else return hi + fma_t(om, fma_t(T(w), drho, -hi), ev + sign_od);
        };
        const S sp = C::template store_scaled<ip, T>(relaxed(h[ip], od), rng);
        BufIO<S>::store(sp, plane_rsrc(B + int64_t(ip) * P, plane_bytes), xo, ro);
        account(IP, sp);
        if constexpr (im >= 0) {
            const S sm = C::template store_scaled<im, T>(relaxed(h[im], -od), rng);
            BufIO<S>::store(sm, plane_rsrc(B + int64_t(im) * P, plane_bytes), xo, ro);
            account(IM, sm);
        }
    });
    if constexpr (WALLS) {
        const int64_t ncol = int64_t(gd.nx) * gd.nz;
        const int64_t col = int64_t(z) * gd.nx + x;
        const int y1 = gd.ny > 3 ? gd.ny - 3 : 0;  // first row of the top plate's sums
        if (y < 3) wd->part[wall_part_index(wd->par ^ 1, 0, y, ncol, col)] = ps[0];
        if (y >= y1) wd->part[wall_part_index(wd->par ^ 1, 1, y - y1, ncol, col)] = ps[1];
    }
}

// Step counter of a handle (F16 storage only): a pair of words; a step that
// reads buffer `cur` reads the step number from ctr[cur] and one lane writes
// the next number to ctr[cur ^ 1], which the next step reads.  The launches
// of a step loop, eager or captured in a graph, so carry the count without
// the host.
template <class S> __device__ __forceinline__ uint32_t step_number(const uint32_t *ctr, int cur)
{
    if constexpr (Codec<Lattice<0>, S>::STOCHASTIC) return __builtin_amdgcn_readfirstlane(ctr[cur]);
    else return 0u;
}
template <class S>
__device__ __forceinline__ void advance_step_number(uint32_t *ctr, int cur, uint32_t step,
                                                    bool writer)
{
    if constexpr (Codec<Lattice<0>, S>::STOCHASTIC) {
        if (writer) ctr[cur ^ 1] = step + 1u;
    }
}

// Work split: one wavefront updates 64 consecutive cells of one row
// (wavefronts numbered row by row, ceil(nx/64) per row); a block is any run of
// consecutive wavefronts, so blocks may straddle rows and none is left partly
// empty at the end of a row.  The wavefront's row is a scalar.
__device__ __forceinline__ bool wave_cell(const GridDims &gd, uint32_t wave, int &x, int &y,
                                          int &z)
{
    const uint32_t k = (uint32_t(gd.nx) + 63u) >> 6;  // wavefronts per row
    const uint32_t row = divu(gd.by_wpr, wave);
    if (row >= uint32_t(gd.ny) * uint32_t(gd.nz)) return false;
    x = int((wave - row * k) * 64u + (threadIdx.x & 63u));
    const uint32_t zz = divu(gd.by_ny, row);
    y = int(row - zz * uint32_t(gd.ny));
    z = int(zz);
    return x < gd.nx;
}

// Wavefronts per SIMD the compiler must leave room for (registers at most
// 512 / 5 rounded down to the allocation granule): FP32 arithmetic fits five
// without spills; left free, the F16 step's stochastic rounding led the
// scheduler to a four-wave schedule (101 registers) that ran slower.  FP64
// arithmetic needs more than 128 registers and is not constrained.
template <class S> constexpr int step_min_waves() { return sizeof(S) == 8 ? 1 : 5; }

template <int LAT, class S, int EQ, int FO>
__global__ void __launch_bounds__(step_max_threads<S>())
    __attribute__((amdgpu_waves_per_eu(step_min_waves<S>(), 8)))
    step_kernel(const S *__restrict__ A, S *__restrict__ B, GridDims gd, ForceDesc fd,
                StepCoef co, uint32_t *ctr, int cur)
{
    const uint32_t wave = __builtin_amdgcn_readfirstlane(blockIdx.x * (blockDim.x >> 6) +
                                                         (threadIdx.x >> 6));
    const uint32_t step = step_number<S>(ctr, cur);
    advance_step_number<S>(ctr, cur, step, wave == 0 && threadIdx.x == 0);
    int x, y, z;
    if (!wave_cell(gd, wave, x, y, z)) return;
    step_cell<LAT, S, EQ, FO>(A, B, gd, fd, co, x, y, z, step);
}

// K7 (diagnostic): the memory traffic of K1 alone -- every population read
// from its pull source and written unchanged at the cell's own slot of the
// other buffer, K1's work split, no arithmetic.  Its rate is the ceiling of
// K1's access pattern on the device.
template <int LAT, class S>
__global__ void __launch_bounds__(step_max_threads<S>())
    pattern_kernel(const S *__restrict__ A, S *__restrict__ B, GridDims gd)
{
    using L = Lattice<LAT>;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(blockIdx.x * (blockDim.x >> 6) +
                                                         (threadIdx.x >> 6));
    int x, y, z;
    if (!wave_cell(gd, wave, x, y, z)) return;
    S h[L::Q];
    gather<L, S, S>(A, gd, x, y, z, h);
    const uint32_t xo = uint32_t(x) * uint32_t(sizeof(S));
    const uint32_t ro = uint32_t((int64_t(z) * gd.ny + y) * gd.px) * uint32_t(sizeof(S));
    const uint32_t plane_bytes = uint32_t(gd.P * int64_t(sizeof(S)));
    static_for<0, L::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        BufIO<S>::store(h[i], plane_rsrc(B + int64_t(i) * gd.P, plane_bytes), xo, ro);
    });
}

// K1c: the step of a grid between plates, in one launch: K1's work split;
// the wavefronts of the rows next to a plate (y < 3 or y >= ny - 3, a uniform
// test) take the plates' emission in place of the sources behind them and
// write the partial sums of the state they produce.
template <int LAT, class S, int EQ, int FO>
__global__ void __launch_bounds__(step_max_threads<S>())
    wall_step_kernel(const S *__restrict__ A, S *__restrict__ B, GridDims gd, ForceDesc fd,
                     StepCoef co, WallDesc wd, uint32_t *ctr, int cur)
{
    const uint32_t wave = __builtin_amdgcn_readfirstlane(blockIdx.x * (blockDim.x >> 6) +
                                                         (threadIdx.x >> 6));
    const uint32_t step = step_number<S>(ctr, cur);
    advance_step_number<S>(ctr, cur, step, wave == 0 && threadIdx.x == 0);
    int x, y, z;
    if (!wave_cell(gd, wave, x, y, z)) return;
    if (y < 3 || y >= gd.ny - 3)
        step_cell<LAT, S, EQ, FO, true>(A, B, gd, fd, co, x, y, z, step, &wd);
    else
        step_cell<LAT, S, EQ, FO>(A, B, gd, fd, co, x, y, z, step);
}

// ---------------------------------------------------------------------------
// K1b: multi-grid step.  Several simulations (same lattice, storage and
// orders; any grid sizes, relaxation times and forces) advance one step in one
// launch.  The work is a list of tiles -- one tile is 64 consecutive cells of
// one grid row of one simulation, updated by one wavefront -- and wavefront w
// of the launch takes tiles w, w + W, ... (W wavefronts launched): with one
// wavefront per tile the hardware balances uneven members; with fewer blocks
// the grid is persistent and every wavefront exits after at most
// ceil(ntiles / W) tiles.  Each cell is updated by exactly one thread with the
// arithmetic of the single-grid step, so no result depends on the launch shape
// or on the other members.  The WALLS variant (launched when some member has
// plates) updates the rows next to a member's plates as K1c does; periodic
// batches keep the variant without that code.
// ---------------------------------------------------------------------------
template <int LAT, class S, int EQ, int FO, bool WALLS>
__global__ void __launch_bounds__(256)
    multi_step_kernel(const int64_t *__restrict__ begin, const TileSim *__restrict__ sims,
                      int nsims, int64_t ntiles, int parity)
{
    const int64_t nw = int64_t(gridDim.x) * (blockDim.x >> 6);
    int64_t t = __builtin_amdgcn_readfirstlane(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6));
    for (; t < ntiles; t += nw) {
        // the simulation owning tile t: last k with begin[k] <= t (uniform)
        int lo = 0, hi = nsims - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (begin[mid] <= t) lo = mid;
            else hi = mid - 1;
        }
        const TileSim &sd = sims[lo];
        // tiles of one simulation number fewer than its cells (< 2^32)
        const uint32_t k = uint32_t(t - begin[lo]);
        const uint32_t cx = uint32_t(sd.chunks_x);
        const uint32_t row = divu(sd.gd.by_wpr, k);  // chunks_x = ceil(nx / 64)
        const uint32_t xc = k - row * cx;
        const uint32_t zz = divu(sd.gd.by_ny, row);
        const int y = int(row - zz * uint32_t(sd.gd.ny)), z = int(zz);
        const int x = int(xc * 64u + (threadIdx.x & 63u));
        const int c = sd.cur ^ parity;
        const S *A = static_cast<const S *>(sd.pop[c]);
        S *B = static_cast<S *>(const_cast<void *>(sd.pop[c ^ 1]));
        // the member's step number; its first tile's wavefront advances it
        const uint32_t step = step_number<S>(sd.ctr, c);
        advance_step_number<S>(sd.ctr, c, step, k == 0 && (threadIdx.x & 63u) == 0);
        if (x >= sd.gd.nx) continue;
        if constexpr (WALLS) {
            // a member between plates: its rows next to a plate as in K1c
            if (sd.wd.on && (y < 3 || y >= sd.gd.ny - 3)) {
                WallDesc w = sd.wd;
                w.par = c;
                step_cell<LAT, S, EQ, FO, true>(A, B, sd.gd, sd.fd, sd.co, x, y, z, step, &w);
                continue;
            }
        }
        step_cell<LAT, S, EQ, FO>(A, B, sd.gd, sd.fd, sd.co, x, y, z, step);
    }
}

// ---------------------------------------------------------------------------
// kernels off the step path: one thread per cell, blocks along x of one grid
// row (y and z uniform over the block), arithmetic in the storage's own
// precision (FP64 for FP64 storage, FP32 for FP32 and F16 storage; the
// fields handed in and out stay FP64)
// ---------------------------------------------------------------------------
// h_i (unscaled) of the state in A at (x, y, z), the plates' emission in
// place of sources behind them.
template <class L, class S, class T>
__device__ __forceinline__ void gather_state(const S *__restrict__ A, const GridDims &gd, int x,
                                             int y, int z, T (&h)[L::Q], const WallDesc &wd,
                                             double rho0)
{
    if (wd.on && (y < 3 || y >= gd.ny - 3))  // uniform over the block
        gather<L, S, T, true>(A, gd, x, y, z, h, &wd, rho0);
    else
        gather<L, S, T>(A, gd, x, y, z, h);
}

// ---------------------------------------------------------------------------
// K2: initial state f~ = f0 - F/2 (sigma = 0), stored as h = f~ - w rho0 and
// scattered so that the pull gather of the first step finds h_i(x) at
// A[i][x - c_i].
// ---------------------------------------------------------------------------
template <int LAT, class S, int EQ, int FO>
__global__ void __launch_bounds__(256)
    init_kernel(const double *__restrict__ rho, const double *__restrict__ u,
                const double *__restrict__ theta, S *__restrict__ A, GridDims gd, ForceDesc fd,
                StepCoef co, WallDesc wd)
{
    using L = Lattice<LAT>;
    using T = typename ArithOf<S>::type;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y, z = blockIdx.z;
    if (x >= gd.nx) return;
    const int64_t N = gd.N;
    const int64_t cell = (int64_t(z) * gd.ny + y) * gd.nx + x;

    T g[3];
    load_force<T, T, L::D>(fd, gd, x, y, z, cell, g);
    CellState<T> cs;
    cs.rho = T(rho[cell]);
    cs.drho = T(rho[cell] - co.rho0);  // the deviation rounded once
    cs.th = T(theta[cell]);
    for (int a = 0; a < 3; ++a) {
        cs.ub[a] = (a < L::D) ? T(u[int64_t(a) * N + cell]) : T(0);
        cs.g[a] = g[a];
        for (int b = 0; b < 3; ++b) cs.sig[a][b] = T(0);
    }
    constexpr int FOI = FO == 4 ? 3 : FO;  // sigma = 0 at the start
    // h = w (rho - rho0) + (f0 - w rho) - F/2
    combo_pairs<L, T, EQ, FOI, true>(cs, T(1), T(-0.5), [&](auto IP, auto IM, T ev, T od) {
        constexpr int ip = decltype(IP)::value;
        constexpr int im = decltype(IM)::value;
        constexpr double w = L::wshell(L::shell(ip));
        auto put = [&](auto II, T v) {
            constexpr int i = decltype(II)::value;
            const S sv = Codec<L, S>::template store<i, T>(v);
            if (wd.on) {
                // with plates: a population arriving from behind a plate has no
                // slot (the plate emits it); one about to stream into a plate
                // stays in its own node's slot
                if (y + L::c(i, 1) < 0 || y + L::c(i, 1) >= gd.ny) {
                    const int64_t own = (int64_t(z) * gd.ny + y) * gd.px + x;
                    A[int64_t(i) * gd.P + own] = sv;
                }
                if (y - L::c(i, 1) < 0 || y - L::c(i, 1) >= gd.ny) return;
            }
            const int xd = wrap3(x - L::c(i, 0), gd.nx);
            const int yd = wrap3(y - L::c(i, 1), gd.ny);
            const int zd = (L::D == 3) ? wrap3(z - L::c(i, 2), gd.nz) : 0;
            const int64_t dst = (int64_t(zd) * gd.ny + yd) * gd.px + xd;
            A[int64_t(i) * gd.P + dst] = sv;
        };
        const T base = T(w) * cs.drho;
        put(std::integral_constant<int, ip>{}, base + (ev + od));
        if constexpr (im >= 0) put(std::integral_constant<int, im>{}, base + (ev - od));
    });
}

// ---------------------------------------------------------------------------
// K3: physical moments rho, u + g/2, theta of the state
// ---------------------------------------------------------------------------
template <int LAT, class S>
__global__ void __launch_bounds__(256)
    moments_kernel(const S *__restrict__ A, double *__restrict__ rho, double *__restrict__ u,
                   double *__restrict__ theta, GridDims gd, ForceDesc fd, StepCoef co,
                   WallDesc wd)
{
    using L = Lattice<LAT>;
    using T = typename ArithOf<S>::type;
    using C = Codec<L, S>;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y, z = blockIdx.z;
    if (x >= gd.nx) return;
    const int64_t N = gd.N;
    const int64_t cell = (int64_t(z) * gd.ny + y) * gd.nx + x;
    T h[L::Q];  // as stored (scaled for F16): raw_sums takes the scale out
    gather_state<L, S, T>(A, gd, x, y, z, h, wd, co.rho0);
    T g[3];
    load_force<T, T, L::D>(fd, gd, x, y, z, cell, g);
    const RawSums<T> rs = raw_sums<L, T, C>(h);
    CellState<T> cs;
    finish_moments<L, T, false>(rs, g, co, cs);
    if (rho) rho[cell] = double(cs.rho);
    if (theta) theta[cell] = double(cs.th);
    if (u)
        for (int a = 0; a < L::D; ++a) u[int64_t(a) * N + cell] = double(cs.ub[a]);
}

// ---------------------------------------------------------------------------
// K5: heat flux q = 1/2 sum_i f_i |xi_i - u|^2 (xi_i - u) of the physical
// distribution f = f0 + cf (f~ - f0 + F/2).  With the equilibrium of order
// N >= 3 the rule reproduces the Maxwellian's moments up to order N + 3, so
// sum_i f0_i |c_i|^2 c_i (c = xi - u) is the Maxwellian's third central
// moment, zero: q = 1/2 sum_i (f_i - f0_i) |c_i|^2 c_i, a sum of small terms
//   f - f0 = cf (h - w drho) - cf (f0 - w rho) + (cf/2) F.
// For N = 2 the equilibrium's own part is added, sum_i f0_i |c_i|^2 c_i =
// -rho u (D + 2 + |u|^2) (the rule's moments to degree 3) + sum_i (f0 - w rho)_i |c_i|^2 c_i.
// ---------------------------------------------------------------------------
template <int LAT, class S, int EQ, int FO>
__global__ void __launch_bounds__(256)
    heatflux_kernel(const S *__restrict__ A, double *__restrict__ q, GridDims gd, ForceDesc fd,
                    StepCoef co, WallDesc wd)
{
    using L = Lattice<LAT>;
    using T = typename ArithOf<S>::type;
    using C = Codec<L, S>;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y, z = blockIdx.z;
    if (x >= gd.nx) return;
    const int64_t N = gd.N;
    const int64_t cell = (int64_t(z) * gd.ny + y) * gd.nx + x;
    T h[L::Q];
    gather_state<L, S, T>(A, gd, x, y, z, h, wd, co.rho0);
    T g[3];
    load_force<T, T, L::D>(fd, gd, x, y, z, cell, g);
    const RawSums<T> rs = raw_sums<L, T, C>(h);
    CellState<T> cs;
    finish_moments<L, T, FO == 4>(rs, g, co, cs);
    static_for<0, L::Q>([&](auto I) {  // the deviations themselves (exact: powers of two)
        constexpr int i = decltype(I)::value;
        constexpr double inv = 1.0 / C::template scale<i>();
        if constexpr (inv != 1.0) h[i] *= T(inv);
    });
    const T cf = cs.cf;
    T qa[3] = {T(0), T(0), T(0)};
    auto acc = [&](auto II, T d) {
        constexpr int i = decltype(II)::value;
        T cv[3], cc = T(0);
        for (int a = 0; a < L::D; ++a) {
            cv[a] = T(L::R * double(L::c(i, a))) - cs.ub[a];
            cc += cv[a] * cv[a];
        }
        for (int a = 0; a < L::D; ++a) qa[a] += d * cc * cv[a];
    };
    combo_pairs<L, T, EQ, FO, true>(cs, -cf, T(0.5) * cf, [&](auto IP, auto IM, T ev, T od) {
        constexpr int ip = decltype(IP)::value;
        constexpr int im = decltype(IM)::value;
        constexpr double w = L::wshell(L::shell(ip));
        acc(IP, cf * (h[ip] - T(w) * cs.drho) + (ev + od));
        if constexpr (im >= 0) acc(IM, cf * (h[im] - T(w) * cs.drho) + (ev - od));
    });
    if constexpr (EQ == 2) {
        T u2 = T(0);
        for (int a = 0; a < L::D; ++a) u2 += cs.ub[a] * cs.ub[a];
        for (int a = 0; a < L::D; ++a) qa[a] -= cs.rho * cs.ub[a] * (T(L::D + 2) + u2);
        combo_pairs<L, T, 2, 1, true>(cs, T(1), T(0), [&](auto IP, auto IM, T ev, T od) {
            acc(IP, ev + od);
            if constexpr (decltype(IM)::value >= 0) acc(IM, ev - od);
        });
    }
    for (int a = 0; a < L::D; ++a) q[int64_t(a) * N + cell] = double(T(0.5) * qa[a]);
}

// ---------------------------------------------------------------------------
// K6: plates.  wall_setup_kernel: e_i = f0_i(1, (U_w, 0, 0), theta_w) of both
// plates in FP64 and the normalisation sum_{i entering} min(|c_iy|, ny) e_i.
// wall_mass_kernel: per (x, z) column, plate and row next to the plate, the
// mass of the crossing slots (populations about to stream into the plate),
// for a state no step produced (after initialisation or an external write);
// a step writes the same sums for the state it produces.  The plate's density
// rw over a column, at which it re-emits exactly what it absorbs, is the sum
// of its rows' sums over the normalisation.
// ---------------------------------------------------------------------------
template <int LAT, int EQ>
__global__ void __launch_bounds__(64)
    wall_setup_kernel(double th_b, double th_t, double u_b, double u_t, int64_t ny,
                      double *__restrict__ e)
{
    using L = Lattice<LAT>;
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    for (int side = 0; side < 2; ++side) {
        CellState<double> cs;
        cs.rho = 1.0;
        cs.drho = 0.0;
        cs.th = side == 0 ? th_b : th_t;
        for (int a = 0; a < 3; ++a) {
            cs.ub[a] = 0.0;
            cs.g[a] = 0.0;
            for (int b = 0; b < 3; ++b) cs.sig[a][b] = 0.0;
        }
        cs.ub[0] = side == 0 ? u_b : u_t;
        cs.om = 0.0;
        cs.cf = 0.0;
        double *es = e + side * (L::Q + 1);
        // f0 = w rho + (f0 - w rho); the bracket is combo_pairs' NO_BASE part
        combo_pairs<L, double, EQ, 1, true>(cs, 1.0, 0.0, [&](auto IP, auto IM, double ev,
                                                            double od) {
            constexpr int ip = decltype(IP)::value;
            constexpr int im = decltype(IM)::value;
            constexpr double w = L::wshell(L::shell(ip));
            es[ip] = w + (ev + od);
            if constexpr (im >= 0) es[im] = w + (ev - od);
        });
        double z = 0.0;
        for (int i = 0; i < L::Q; ++i) {
            const int cy = L::c(i, 1);
            if (side == 0 ? cy > 0 : cy < 0) {
                const int64_t k = cy < 0 ? -cy : cy;
                z += double(k < ny ? k : ny) * es[i];
            }
        }
        es[L::Q] = z;
    }
}

template <class L, class S>
__device__ __forceinline__ void wall_column_density(const S *__restrict__ A, const GridDims &gd,
                                                    const StepCoef &co, const WallDesc &wd,
                                                    int64_t col)
{
    // The partial sums of state A (buffer wd.par) over one column: per row next
    // to a plate, its slots whose next move crosses the plate -- rows y = k
    // with c_y < -k (bottom), rows y = ny-3+k with c_y >= 3 - k (top) --
    // populations ascending.  Every load is unconditional and independent (the
    // crossing test only selects the term), so they are all in flight at once.
    const int64_t ncol = int64_t(gd.nx) * gd.nz;
    const int x = int(col % gd.nx), z = int(col / gd.nx);
    static_for<0, 2>([&](auto SIDE) {
        constexpr int side = decltype(SIDE)::value;
        const int y0 = side == 0 ? 0 : (gd.ny > 3 ? gd.ny - 3 : 0);
        static_for<0, 3>([&](auto K) {
            constexpr int k = decltype(K)::value;
            const int y = y0 + k;
            if (y >= gd.ny) return;  // uniform: only when ny < 3
            const int64_t own = (int64_t(z) * gd.ny + y) * gd.px + x;
            double m = 0.0;
            static_for<0, L::Q>([&](auto I) {
                constexpr int i = decltype(I)::value;
                constexpr int cy = L::c(i, 1);
                // a slot can cross only toward its plate
                if constexpr (side == 0 ? cy < 0 : cy > 0) {
                    const int yd = y + cy;
                    const double v =
                        Codec<L, S>::template load<i, double>(A[int64_t(i) * gd.P + own]) +
                        L::wshell(L::shell(i)) * co.rho0;
                    m += (side == 0 ? yd < 0 : yd >= gd.ny) ? v : 0.0;
                }
            });
            wd.part[wall_part_index(wd.par, side, k, ncol, col)] = m;
        });
    });
}

template <int LAT, class S>
__global__ void __launch_bounds__(256)
    wall_mass_kernel(const S *__restrict__ A, GridDims gd, StepCoef co, WallDesc wd)
{
    const int64_t ncol = int64_t(gd.nx) * gd.nz;
    const int64_t col = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (col < ncol) wall_column_density<Lattice<LAT>, S>(A, gd, co, wd, col);
}

// ---------------------------------------------------------------------------
// K4: totals.  Stage 1: block b sums a fixed slice of every population plane
// of h; stage 2: one block adds the slices in order and forms the moments of
// f = w rho0 + h using sum w = 1, sum w c = 0 and sum w |c|^2 r^2 = D:
//   mass = N rho0 + sum H_i, momentum = r sum c_i H_i,
//   energy = N rho0 D + r^2 sum |c_i|^2 H_i,  with H_i = sum_x h_i(x).
// The partition and the reduction order do not depend on the grid or launch
// shape of the step, so the result is bitwise reproducible.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double block_sum_256(double v, double *lds)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) lds[wid] = v;
    __syncthreads();
    return (lds[0] + lds[1]) + (lds[2] + lds[3]);
}

// Stage 1: block b sums the cells of a fixed run of grid rows, every lane
// holding one FP64 accumulator per population: the block's cells are taken
// in order, lane t the t-th of every 256, all Q planes of a cell loaded
// together; then each accumulator is reduced across the block in a fixed tree.
template <int LAT, class S>
__global__ void __launch_bounds__(256)
    totals_stage1(const S *__restrict__ A, double *__restrict__ partials, GridDims gd,
                  DivU32 by_nx)
{
    using L = Lattice<LAT>;
    __shared__ double lds[4][L::Q];
    const int64_t rows = int64_t(gd.ny) * gd.nz;
    const int64_t chunk = (rows + TOTALS_BLOCKS - 1) / TOTALS_BLOCKS;
    const int64_t lo = int64_t(blockIdx.x) * chunk;
    const int64_t hi = (lo + chunk < rows) ? lo + chunk : rows;
    double acc[L::Q];
    static_for<0, L::Q>([&](auto I) { acc[decltype(I)::value] = 0.0; });
    // cells of the block, < 2^32: a block holds at most ceil(rows / 512) rows
    const uint32_t ncell = hi > lo ? uint32_t((hi - lo) * gd.nx) : 0u;
    for (uint32_t k = threadIdx.x; k < ncell; k += 256) {
        const uint32_t dr = divu(by_nx, k);
        const int64_t idx = (lo + dr) * gd.px + (k - dr * uint32_t(gd.nx));
        static_for<0, L::Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            acc[i] += Codec<L, S>::template load<i, double>(A[int64_t(i) * gd.P + idx]);
        });
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    static_for<0, L::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        double v = acc[i];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        if (lane == 0) lds[wid][i] = v;
    });
    __syncthreads();
    if (threadIdx.x < L::Q) {
        const int i = threadIdx.x;
        partials[int64_t(blockIdx.x) * L::Q + i] = (lds[0][i] + lds[1][i]) + (lds[2][i] + lds[3][i]);
    }
}

template <int LAT>
__global__ void __launch_bounds__(256) totals_stage2(const double *__restrict__ partials,
                                                     double *__restrict__ out, GridDims gd,
                                                     StepCoef co)
{
    using L = Lattice<LAT>;
    __shared__ double lds[4];
    __shared__ double Hi[L::Q];
    for (int i = 0; i < L::Q; ++i) {
        double v = 0.0;
        for (int b = threadIdx.x; b < TOTALS_BLOCKS; b += 256) v += partials[int64_t(b) * L::Q + i];
        v = block_sum_256(v, lds);
        if (threadIdx.x == 0) Hi[i] = v;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = 0.0, p[3] = {0.0, 0.0, 0.0}, e = 0.0;
        static_for<0, L::Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            m += Hi[i];
            for (int a = 0; a < L::D; ++a) p[a] += double(L::c(i, a)) * Hi[i];
            e += double(c2<L>(i)) * Hi[i];
        });
        const double base = double(gd.N) * co.rho0;
        out[0] = base + m;
        for (int a = 0; a < L::D; ++a) out[1 + a] = L::R * p[a];
        out[1 + L::D] = base * double(L::D) + L::R2 * e;
    }
}

}  // namespace lbm
