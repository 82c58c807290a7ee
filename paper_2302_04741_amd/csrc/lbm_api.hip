// C ABI of the gfx950 thermal LBM library (declared in include/lbm.h).
//
// Host-side validation, workspace layout, handle state and launches on the
// handle's stream.  The library allocates no device memory: every buffer is a
// slice of the caller's workspace.  Argument checks run before any HIP call,
// so they also work on a machine without a GPU.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "lbm.h"
#include "lbm_internal.h"

using namespace lbm;

struct lbm_sim {
    lbm_params p;
    int D, Q, eq;
    int64_t N;
    GridDims gd;
    StepCoef co;
    ForceDesc fd;
    hipStream_t stream;
    char *ws;
    size_t ws_bytes;
    void *pop[2];
    int cur;
    void *gtab;
    size_t gtab_bytes;
    double *partials;
    double *totals_dev;
    uint32_t *ctr;  // device step counter pair of the F16 stochastic rounding (in the totals slot)
    int64_t step;
    int block;
    int64_t gen;  // bumped when launch arguments change (force, block, stream, viscosity,
                  // plates): batches and graphs built before are stale
    WallDesc wd;  // plates (off unless lbm_set_walls)
    double *wall_part;     // plates: partial sums of the crossing slots, per buffer
    double *wall_e;        // plates: emission tables
    bool wall_fresh;       // plates: wall_part holds the sums of the current state
};

namespace {

thread_local std::string g_err;

// A roctx range over one API call (shown by rocprofv3 --marker-trace around
// the kernels the call enqueues; a few nanoseconds when no profiler listens).
struct TraceRange {
    explicit TraceRange(const char *name) { roctxRangePushA(name); }
    ~TraceRange() { roctxRangePop(); }
    TraceRange(const TraceRange &) = delete;
    TraceRange &operator=(const TraceRange &) = delete;
};

lbm_status fail(lbm_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

lbm_status ok()
{
    g_err.clear();
    return LBM_OK;
}

lbm_status dev_fail(hipError_t e, const char *what)
{
    return fail(LBM_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

constexpr size_t ALIGN = 256;
size_t align_up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

int lattice_dim(int lat) { return lat == LBM_D2Q37 ? D2Q37_D : D3Q39_D; }
int lattice_q(int lat) { return lat == LBM_D2Q37 ? D2Q37_Q : D3Q39_Q; }
int lattice_maxeq(int lat) { return lat == LBM_D2Q37 ? Lattice<0>::MAXEQ : Lattice<1>::MAXEQ; }
size_t storage_bytes(int storage) { return storage == LBM_F64 ? 8 : (storage == LBM_F32 ? 4 : 2); }
size_t arith_bytes(int storage) { return storage == LBM_F64 ? 8 : 4; }

struct Layout {
    size_t pop, gtab, partials, totals, walls;
    size_t off_pop1, off_gtab, off_part, off_tot, off_walls, total;
};

int64_t row_pitch(int64_t nx) { return (nx + ROW_ALIGN - 1) / ROW_ALIGN * ROW_ALIGN; }

Layout layout_of(const lbm_params *p)
{
    Layout L{};
    const int D = lattice_dim(p->lattice), Q = lattice_q(p->lattice);
    const size_t N = size_t(p->nx) * size_t(p->ny) * size_t(p->nz);
    const size_t P = size_t(row_pitch(p->nx)) * size_t(p->ny) * size_t(p->nz);
    L.pop = align_up(size_t(Q) * P * storage_bytes(p->storage));
    int64_t ext = p->nx > p->ny ? p->nx : p->ny;
    ext = ext > p->nz ? ext : p->nz;
    size_t gcount = size_t(D) * size_t(ext);
    if (p->flags & LBM_FLAG_FORCE_FIELD) {
        const size_t gf = size_t(D) * N;
        gcount = gcount > gf ? gcount : gf;
    }
    L.gtab = align_up(gcount * arith_bytes(p->storage));
    L.partials = align_up(size_t(TOTALS_BLOCKS) * size_t(Q) * sizeof(double));
    L.totals = align_up(8 * sizeof(double));
    L.off_pop1 = L.pop;
    L.off_gtab = 2 * L.pop;
    L.off_part = L.off_gtab + L.gtab;
    L.off_tot = L.off_part + L.partials;
    // plates: partial sums [2 buffer][2 plate][3 row][nx*nz], emission tables [2][Q + 1]
    L.walls = (p->flags & LBM_FLAG_WALLS)
                  ? align_up(12 * size_t(p->nx) * size_t(p->nz) * sizeof(double)) +
                        align_up(2 * size_t(Q + 1) * sizeof(double))
                  : 0;
    L.off_walls = L.off_tot + L.totals;
    L.total = L.off_walls + L.walls;
    return L;
}

// Device step counter of a handle: the step sets ctr[cur] = n, read by the
// next step (F16 stochastic rounding keys).
__global__ void __launch_bounds__(64) set_step_number_kernel(uint32_t *ctr, int cur, uint32_t n)
{
    if (threadIdx.x == 0) ctr[cur] = n;
}

hipError_t set_step_number(const lbm_sim *s)
{
    hipLaunchKernelGGL(set_step_number_kernel, dim3(1), dim3(64), 0, s->stream, s->ctr, s->cur,
                       uint32_t(s->step));
    return hipGetLastError();
}

lbm_status check_params(const lbm_params *p)
{
    if (!p) return fail(LBM_EINVAL, "params is NULL");
    if (p->struct_size != sizeof(lbm_params))
        return fail(LBM_EINVAL, "params.struct_size is %u, expected %zu", p->struct_size,
                    sizeof(lbm_params));
    if (p->lattice != LBM_D2Q37 && p->lattice != LBM_D3Q39)
        return fail(LBM_EINVAL, "unknown lattice %d", p->lattice);
    if (p->storage != LBM_F64 && p->storage != LBM_F32 && p->storage != LBM_F16DEV)
        return fail(LBM_EINVAL, "unknown storage %d", p->storage);
    if (p->nx < 1 || p->ny < 1 || p->nz < 1)
        return fail(LBM_EINVAL, "grid extents must be >= 1 (got %lld x %lld x %lld)",
                    (long long)p->nx, (long long)p->ny, (long long)p->nz);
    if (p->lattice == LBM_D2Q37 && p->nz != 1)
        return fail(LBM_EINVAL, "D2Q37 needs nz == 1 (got %lld)", (long long)p->nz);
    if (p->nx > (int64_t(1) << 30) || p->ny > 65535 || p->nz > 65535)
        return fail(LBM_EUNSUPPORTED, "grid extents limited to nx <= 2^30, ny, nz <= 65535");
    const double plane = double(row_pitch(p->nx)) * double(p->ny) * double(p->nz);
    if (plane * double(storage_bytes(p->storage)) >= 4294967296.0)
        return fail(LBM_EUNSUPPORTED,
                    "one population plane (rows padded to 64 values) must stay below 4 GiB");
    if (!std::isfinite(p->tau_hat) || !(p->tau_hat > 0.5))
        return fail(LBM_EINVAL, "tau_hat must be finite and > 0.5 (got %g)", p->tau_hat);
    if (p->eq_order < 0 || p->eq_order == 1)
        return fail(LBM_EINVAL, "eq_order must be 0 or >= 2 (got %d)", p->eq_order);
    if (p->eq_order > lattice_maxeq(p->lattice))
        return fail(LBM_EUNSUPPORTED, "eq_order %d exceeds what the velocity set supports (%d)",
                    p->eq_order, lattice_maxeq(p->lattice));
    if (p->force_order < LBM_FORCE_N0 || p->force_order > LBM_FORCE_N2)
        return fail(LBM_EINVAL, "unknown force_order %d", p->force_order);
    if (p->flags & ~(LBM_FLAG_FORCE_FIELD | LBM_FLAG_WALLS))
        return fail(LBM_EINVAL, "unknown flags 0x%x", p->flags);
    if (!std::isfinite(p->rho0) || !(p->rho0 >= 0))
        return fail(LBM_EINVAL, "rho0 must be finite and >= 0 (got %g)", p->rho0);
    return LBM_OK;
}

// Launch settings for a kernel reading the state in pop[cur] (with plates, the
// partial sums of that buffer).
LaunchCfg cfg(const lbm_sim *s, int cur)
{
    LaunchCfg c{s->block, s->stream, s->wd, s->ctr, cur};
    c.walls.par = cur;
    return c;
}
LaunchCfg cfg(const lbm_sim *s) { return cfg(s, s->cur); }

// With plates, whatever reads the state needs the partial sums of the current
// state: steps keep them (each writes those of the state it produces); after
// the state was written otherwise (initialisation, lbm_set_populations) one
// pass over the columns computes them.
hipError_t wall_densities(lbm_sim *s, hipStream_t stream)
{
    if (!s->wd.on || s->wall_fresh) return hipSuccess;
    LaunchCfg c = cfg(s);
    c.stream = stream;
    hipError_t e = launch_wall_mass(s->p.lattice, s->p.storage, s->pop[s->cur], s->gd, s->co, c);
    s->wall_fresh = e == hipSuccess;
    return e;
}
hipError_t wall_densities(lbm_sim *s) { return wall_densities(s, s->stream); }

// One time step, one launch: K1, or with plates K1c (which also writes the
// partial sums of the state it produces).
hipError_t launch_one_step(const lbm_sim *s, int cur)
{
    const void *A = s->pop[cur];
    void *B = s->pop[cur ^ 1];
    if (s->wd.on)
        return launch_wall_step(s->p.lattice, s->p.storage, s->eq, s->p.force_order, A, B,
                                s->gd, s->fd, s->co, cfg(s, cur));
    return launch_step(s->p.lattice, s->p.storage, s->eq, s->p.force_order, A, B, s->gd, s->fd,
                       s->co, cfg(s, cur));
}

// Enqueues nsteps steps of the state held in pop[cur] (with plates, its partial
// sums must be current); on return cur names the buffer holding the advanced
// state and done the steps enqueued (all of them unless a launch failed), one
// launch per step.
hipError_t launch_steps(const lbm_sim *s, int &cur, int64_t nsteps, int64_t &done)
{
    done = 0;
    while (done < nsteps) {
        hipError_t e = launch_one_step(s, cur);
        if (e != hipSuccess) return e;
        cur ^= 1;
        done++;
    }
    return hipSuccess;
}

}  // namespace

namespace lbm {
// F16 stochastic rounding of plain arrays (defined with the F16 field kernels)
hipError_t launch_round_f16_sr(const float *v, const uint32_t *seed, uint16_t *out, int64_t n,
                                hipStream_t stream);
}  // namespace lbm

extern "C" {

size_t lbm_workspace_bytes(const lbm_params *p)
{
    if (check_params(p) != LBM_OK) return 0;
    return layout_of(p).total;
}

lbm_status lbm_create(const lbm_params *p, void *workspace, size_t workspace_bytes,
                      void *hip_stream, const double *rho, const double *u, const double *theta,
                      lbm_sim **out)
{
    if (!out) return fail(LBM_EINVAL, "out is NULL");
    *out = nullptr;
    lbm_status st = check_params(p);
    if (st != LBM_OK) return st;
    if (!workspace) return fail(LBM_EINVAL, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(workspace) % ALIGN)
        return fail(LBM_EINVAL, "workspace must be 256-byte aligned");
    const Layout L = layout_of(p);
    if (workspace_bytes < L.total)
        return fail(LBM_ENOSPACE, "workspace has %zu bytes, %zu needed", workspace_bytes, L.total);
    if (!rho || !u || !theta) return fail(LBM_EINVAL, "initial fields must not be NULL");

    lbm_sim *s = new (std::nothrow) lbm_sim();
    if (!s) return fail(LBM_EINVAL, "out of host memory");
    s->p = *p;
    s->D = lattice_dim(p->lattice);
    s->Q = lattice_q(p->lattice);
    s->eq = p->eq_order ? p->eq_order : lattice_maxeq(p->lattice);
    s->N = p->nx * p->ny * p->nz;
    s->gd = make_grid_dims(p->nx, p->ny, p->nz, row_pitch(p->nx));
    s->co = StepCoef{1.0 / p->tau_hat, 1.0 - 0.5 / p->tau_hat, p->rho0, 0.0};
    s->fd = ForceDesc{};
    s->stream = static_cast<hipStream_t>(hip_stream);
    s->ws = static_cast<char *>(workspace);
    s->ws_bytes = workspace_bytes;
    s->pop[0] = s->ws;
    s->pop[1] = s->ws + L.off_pop1;
    s->cur = 0;
    s->gtab = s->ws + L.off_gtab;
    s->gtab_bytes = L.gtab;
    s->fd.tab = s->gtab;
    s->partials = reinterpret_cast<double *>(s->ws + L.off_part);
    s->totals_dev = reinterpret_cast<double *>(s->ws + L.off_tot);
    s->ctr = reinterpret_cast<uint32_t *>(s->ws + L.off_tot + 8 * sizeof(double));
    s->wd = WallDesc{0, 0, nullptr, nullptr};
    s->wall_part = nullptr;
    s->wall_e = nullptr;
    s->wall_fresh = false;
    if (p->flags & LBM_FLAG_WALLS) {
        s->wall_part = reinterpret_cast<double *>(s->ws + L.off_walls);
        s->wall_e = reinterpret_cast<double *>(
            s->ws + L.off_walls + align_up(12 * size_t(p->nx) * size_t(p->nz) * sizeof(double)));
    }
    s->step = 0;
    s->block = 0;
    hipError_t e = launch_init(p->lattice, p->storage, s->eq, p->force_order, rho, u, theta,
                               s->pop[0], s->gd, s->fd, s->co, cfg(s));
    if (e == hipSuccess) e = set_step_number(s);
    if (e != hipSuccess) {
        delete s;
        return dev_fail(e, "init kernel launch");
    }
    *out = s;
    return ok();
}

lbm_status lbm_set_force(lbm_sim *s, int32_t kind, const double *g, int32_t axis, int64_t len)
{
    if (!s) return fail(LBM_EINVAL, "handle is NULL");
    if (!g) return fail(LBM_EINVAL, "g is NULL");
    ForceDesc nf = s->fd;
    nf.tab = s->gtab;
    int64_t count = 0;
    if (kind == LBM_G_UNIFORM) {
        for (int a = 0; a < s->D; ++a)
            if (!std::isfinite(g[a])) return fail(LBM_EINVAL, "g[%d] is not finite", a);
        nf.kind = 0;
        for (int a = 0; a < 3; ++a) nf.g[a] = a < s->D ? g[a] : 0.0;
        nf.axis = 0;
        nf.len = 0;
    } else if (kind == LBM_G_AXIS_PROFILE) {
        if (axis < 0 || axis >= s->D) return fail(LBM_EINVAL, "axis %d out of range", axis);
        const int64_t ext = axis == 0 ? s->p.nx : (axis == 1 ? s->p.ny : s->p.nz);
        if (len != ext)
            return fail(LBM_EINVAL, "profile length %lld must equal the extent %lld along axis %d",
                        (long long)len, (long long)ext, axis);
        nf.kind = 1;
        nf.axis = axis;
        nf.len = len;
        count = int64_t(s->D) * len;
    } else if (kind == LBM_G_FIELD) {
        if (!(s->p.flags & LBM_FLAG_FORCE_FIELD))
            return fail(LBM_EINVAL, "LBM_G_FIELD needs LBM_FLAG_FORCE_FIELD at creation");
        nf.kind = 2;
        nf.axis = 0;
        nf.len = 0;
        count = int64_t(s->D) * s->N;
    } else {
        return fail(LBM_EINVAL, "unknown force kind %d", kind);
    }
    if (size_t(count) * arith_bytes(s->p.storage) > s->gtab_bytes)
        return fail(LBM_ENOSPACE, "force table does not fit the workspace");

    hipError_t e;
    void *scratch = s->pop[s->cur ^ 1];
    double *mrho = static_cast<double *>(scratch);
    double *mu = mrho + s->N;
    double *mth = mu + int64_t(s->D) * s->N;
    if (s->step == 0) {
        // Rebuild f~ = f0 - F/2 for the new force from the current moments,
        // which were produced with the old one.  The idle population buffer
        // holds the FP64 moments in between ((2 + D) doubles per cell fit in
        // Q stored values for every storage type).
        e = wall_densities(s);
        if (e != hipSuccess) return dev_fail(e, "wall density kernel launch");
        e = launch_moments(s->p.lattice, s->p.storage, s->pop[s->cur], mrho, mu, mth, s->gd, s->fd,
                           s->co, cfg(s));
        if (e != hipSuccess) return dev_fail(e, "moments kernel launch");
    }
    if (count > 0) {
        e = launch_convert(s->p.storage, g, s->gtab, count, s->stream);
        if (e != hipSuccess) return dev_fail(e, "force table conversion");
    }
    s->fd = nf;
    s->gen++;
    if (s->step == 0) {
        e = launch_init(s->p.lattice, s->p.storage, s->eq, s->p.force_order, mrho, mu, mth,
                        s->pop[s->cur], s->gd, s->fd, s->co, cfg(s));
        if (e != hipSuccess) return dev_fail(e, "init kernel launch");
        s->wall_fresh = false;
    }
    return ok();
}

lbm_status lbm_step(lbm_sim *s, int64_t nsteps)
{
    if (!s) return fail(LBM_EINVAL, "handle is NULL");
    if (nsteps < 0) return fail(LBM_EINVAL, "nsteps must be >= 0");
    if (nsteps == 0) return ok();
    TraceRange range("lbm_step");
    hipError_t e = wall_densities(s);
    if (e != hipSuccess) return dev_fail(e, "wall density kernel launch");
    int cur = s->cur;
    int64_t done = 0;
    e = launch_steps(s, cur, nsteps, done);
    s->cur = cur;
    s->step += done;
    if (e != hipSuccess) {
        s->wall_fresh = false;
        return dev_fail(e, "step kernel launch");
    }
    return ok();
}

lbm_status lbm_moments(lbm_sim *s, double *rho, double *u, double *theta)
{
    if (!s) return fail(LBM_EINVAL, "handle is NULL");
    if (!rho && !u && !theta) return ok();
    hipError_t e = wall_densities(s);
    if (e != hipSuccess) return dev_fail(e, "wall density kernel launch");
    e = launch_moments(s->p.lattice, s->p.storage, s->pop[s->cur], rho, u, theta, s->gd, s->fd,
                       s->co, cfg(s));
    if (e != hipSuccess) return dev_fail(e, "moments kernel launch");
    return ok();
}

void lbm_destroy(lbm_sim *s) { delete s; }

const char *lbm_last_error(void) { return g_err.c_str(); }

lbm_status lbm_totals(lbm_sim *s, double *out)
{
    if (!s) return fail(LBM_EINVAL, "handle is NULL");
    if (!out) return fail(LBM_EINVAL, "out is NULL");
    hipError_t e = launch_totals(s->p.lattice, s->p.storage, s->pop[s->cur], s->partials,
                                 s->totals_dev, s->gd, s->co, s->stream);
    if (e != hipSuccess) return dev_fail(e, "totals kernel launch");
    e = hipMemcpyAsync(out, s->totals_dev, sizeof(double) * size_t(s->D + 2),
                       hipMemcpyDeviceToHost, s->stream);
    if (e != hipSuccess) return dev_fail(e, "totals copy");
    e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return dev_fail(e, "stream synchronize");
    for (int k = 0; k < s->D + 2; ++k)
        if (!std::isfinite(out[k])) return fail(LBM_ENONFINITE, "total %d is not finite", k);
    return ok();
}

lbm_status lbm_totals_device(lbm_sim *s, double *out_dev)
{
    if (!s) return fail(LBM_EINVAL, "handle is NULL");
    if (!out_dev) return fail(LBM_EINVAL, "out_dev is NULL");
    hipError_t e = launch_totals(s->p.lattice, s->p.storage, s->pop[s->cur], s->partials,
                                 out_dev, s->gd, s->co, s->stream);
    if (e != hipSuccess) return dev_fail(e, "totals kernel launch");
    return ok();
}

lbm_status lbm_round_f16_stochastic(const float *v, const uint32_t *seed, uint16_t *out,
                                    int64_t n, void *hip_stream)
{
    if (n < 0) return fail(LBM_EINVAL, "n must be >= 0");
    if (n == 0) return ok();
    if (!v || !seed || !out) return fail(LBM_EINVAL, "v, seed and out must not be NULL");
    hipError_t e = launch_round_f16_sr(v, seed, out, n, static_cast<hipStream_t>(hip_stream));
    if (e != hipSuccess) return dev_fail(e, "rounding kernel launch");
    return ok();
}

lbm_status lbm_heat_flux(lbm_sim *s, double *q)
{
    if (!s) return fail(LBM_EINVAL, "handle is NULL");
    if (!q) return fail(LBM_EINVAL, "q is NULL");
    hipError_t e = wall_densities(s);
    if (e != hipSuccess) return dev_fail(e, "wall density kernel launch");
    e = launch_heat_flux(s->p.lattice, s->p.storage, s->eq, s->p.force_order, s->pop[s->cur], q,
                         s->gd, s->fd, s->co, cfg(s));
    if (e != hipSuccess) return dev_fail(e, "heat-flux kernel launch");
    return ok();
}

lbm_status lbm_pattern_pass(lbm_sim *s, int64_t repeats)
{
    if (!s) return fail(LBM_EINVAL, "handle is NULL");
    if (repeats < 0) return fail(LBM_EINVAL, "repeats must be >= 0");
    for (int64_t r = 0; r < repeats; ++r) {
        hipError_t e = launch_pattern(s->p.lattice, s->p.storage, s->pop[s->cur],
                                      s->pop[s->cur ^ 1], s->gd, cfg(s));
        if (e != hipSuccess) return dev_fail(e, "pattern kernel launch");
    }
    return ok();
}

size_t lbm_population_bytes(const lbm_sim *s)
{
    if (!s) return 0;
    return size_t(s->Q) * size_t(s->N) * storage_bytes(s->p.storage);
}

lbm_status lbm_get_populations(lbm_sim *s, void *dst)
{
    if (!s) return fail(LBM_EINVAL, "handle is NULL");
    if (!dst) return fail(LBM_EINVAL, "dst is NULL");
    // dense rows out of the padded planes: one strided copy over Q*ny*nz rows
    const size_t sb = storage_bytes(s->p.storage);
    hipError_t e = hipMemcpy2DAsync(dst, size_t(s->gd.nx) * sb, s->pop[s->cur],
                                    size_t(s->gd.px) * sb, size_t(s->gd.nx) * sb,
                                    size_t(s->Q) * size_t(s->gd.ny) * size_t(s->gd.nz),
                                    hipMemcpyDeviceToDevice, s->stream);
    if (e != hipSuccess) return dev_fail(e, "population copy");
    return ok();
}

lbm_status lbm_set_populations(lbm_sim *s, const void *src)
{
    if (!s) return fail(LBM_EINVAL, "handle is NULL");
    if (!src) return fail(LBM_EINVAL, "src is NULL");
    const size_t sb = storage_bytes(s->p.storage);
    hipError_t e = hipMemcpy2DAsync(s->pop[s->cur], size_t(s->gd.px) * sb, src,
                                    size_t(s->gd.nx) * sb, size_t(s->gd.nx) * sb,
                                    size_t(s->Q) * size_t(s->gd.ny) * size_t(s->gd.nz),
                                    hipMemcpyDeviceToDevice, s->stream);
    s->wall_fresh = false;
    if (e != hipSuccess) return dev_fail(e, "population copy");
    return ok();
}

int64_t lbm_step_count(const lbm_sim *s) { return s ? s->step : -1; }

lbm_status lbm_set_step_count(lbm_sim *s, int64_t n)
{
    if (!s) return fail(LBM_EINVAL, "handle is NULL");
    if (n < 0) return fail(LBM_EINVAL, "step count must be >= 0");
    s->step = n;
    hipError_t e = set_step_number(s);
    if (e != hipSuccess) return dev_fail(e, "step counter kernel launch");
    return ok();
}

lbm_status lbm_set_stream(lbm_sim *s, void *hip_stream)
{
    if (!s) return fail(LBM_EINVAL, "handle is NULL");
    s->stream = static_cast<hipStream_t>(hip_stream);
    s->gen++;
    return ok();
}

lbm_status lbm_set_block(lbm_sim *s, int32_t threads)
{
    if (!s) return fail(LBM_EINVAL, "handle is NULL");
    if (threads != 0 && threads != 64 && threads != 128 && threads != 256 && threads != 512 &&
        threads != 1024)
        return fail(LBM_EINVAL, "block must be 0, 64, 128, 256, 512 or 1024 (got %d)", threads);
    s->block = threads;
    s->gen++;
    return ok();
}

lbm_status lbm_set_viscosity(lbm_sim *s, double mu)
{
    if (!s) return fail(LBM_EINVAL, "handle is NULL");
    if (!(mu >= 0.0) || !std::isfinite(mu))
        return fail(LBM_EINVAL, "mu must be finite and >= 0 (got %g)", mu);
    s->co.mu = mu;
    s->gen++;
    return ok();
}

lbm_status lbm_set_walls(lbm_sim *s, int32_t enable, double theta_b, double theta_t, double u_b,
                         double u_t)
{
    if (!s) return fail(LBM_EINVAL, "handle is NULL");
    if (!(s->p.flags & LBM_FLAG_WALLS))
        return fail(LBM_EINVAL, "plates need LBM_FLAG_WALLS at creation");
    if (s->step != 0) return fail(LBM_EINVAL, "plates must be set before the first step");
    if (enable && (!std::isfinite(theta_b) || !std::isfinite(theta_t) || !(theta_b > 0) ||
                   !(theta_t > 0) || !std::isfinite(u_b) || !std::isfinite(u_t)))
        return fail(LBM_EINVAL, "plate temperatures must be finite and > 0, velocities finite");
    // Rebuild the state for the new boundary from the moments it reports now.
    hipError_t e;
    void *scratch = s->pop[s->cur ^ 1];
    double *mrho = static_cast<double *>(scratch);
    double *mu = mrho + s->N;
    double *mth = mu + int64_t(s->D) * s->N;
    e = wall_densities(s);
    if (e != hipSuccess) return dev_fail(e, "wall density kernel launch");
    e = launch_moments(s->p.lattice, s->p.storage, s->pop[s->cur], mrho, mu, mth, s->gd, s->fd,
                       s->co, cfg(s));
    if (e != hipSuccess) return dev_fail(e, "moments kernel launch");
    if (enable) {
        const double th[2] = {theta_b, theta_t}, uw[2] = {u_b, u_t};
        e = launch_wall_setup(s->p.lattice, s->eq, th, uw, s->p.ny, s->wall_e, s->stream);
        if (e != hipSuccess) return dev_fail(e, "plate setup kernel launch");
        s->wd = WallDesc{1, 0, s->wall_part, s->wall_e};
    } else {
        s->wd = WallDesc{0, 0, nullptr, nullptr};
    }
    s->gen++;
    s->wall_fresh = false;
    e = launch_init(s->p.lattice, s->p.storage, s->eq, s->p.force_order, mrho, mu, mth,
                    s->pop[s->cur], s->gd, s->fd, s->co, cfg(s));
    if (e != hipSuccess) return dev_fail(e, "init kernel launch");
    return ok();
}

int32_t lbm_lattice_table(int32_t lattice, int32_t *c, double *w, double *r)
{
    if (lattice != LBM_D2Q37 && lattice != LBM_D3Q39)
        return int32_t(fail(LBM_EINVAL, "unknown lattice %d", lattice));
    const int Q = lattice_q(lattice);
    for (int i = 0; i < Q; ++i) {
        for (int a = 0; a < 3; ++a)
            if (c) c[3 * i + a] = lattice == LBM_D2Q37 ? d2q37_C[i][a] : d3q39_C[i][a];
        if (w) w[i] = lattice == LBM_D2Q37 ? d2q37_WSHELL[d2q37_SHELL[i]] : d3q39_WSHELL[d3q39_SHELL[i]];
    }
    if (r) *r = lattice == LBM_D2Q37 ? d2q37_R : d3q39_R;
    ok();
    return Q;
}

const char *lbm_version(void) { return "lbm-gfx950 0.7.0"; }

// ---------------------------------------------------------------------------
// batches
// ---------------------------------------------------------------------------
}  // extern "C"

// ---------------------------------------------------------------------------
// tile tables of the multi-grid step, written on the device by small copy
// kernels whose arguments carry the descriptors (no host staging buffer has to
// outlive the call, and nothing waits for the device)
// ---------------------------------------------------------------------------
namespace {
constexpr int TABLE_CHUNK = 16;  // members per fill launch: kernel arguments <= 4 KiB

// Members first .. first + n - 1 of a tile table; `last` also sets the end of
// the list, begin[first + n] = end.
struct TableChunk {
    int32_t first, n, last;
    int64_t end;
    int64_t begin[TABLE_CHUNK];
    TileSim sims[TABLE_CHUNK];
};
static_assert(sizeof(TableChunk) <= 4000, "kernel arguments are limited to 4 KiB");
}  // namespace

__global__ void __launch_bounds__(64) table_fill_kernel(TableChunk c, int64_t *begin, TileSim *tab)
{
    const int t = int(threadIdx.x);
    if (t < c.n) {
        begin[c.first + t] = c.begin[t];
        tab[c.first + t] = c.sims[t];
    }
    if (t == 0 && c.last) begin[c.first + c.n] = c.end;
}

namespace {
// Members of one multi-grid launch: non-NULL, distinct, same kernel variant.
lbm_status check_members(lbm_sim *const *sims, int32_t count)
{
    for (int32_t k = 0; k < count; ++k) {
        const lbm_sim *s = sims[k];
        if (!s) return fail(LBM_EINVAL, "sims[%d] is NULL", k);
        for (int32_t j = 0; j < k; ++j)
            if (sims[j] == s) return fail(LBM_EINVAL, "sims[%d] repeats sims[%d]", k, j);
        const lbm_sim *s0 = sims[0];
        if (s->p.lattice != s0->p.lattice || s->p.storage != s0->p.storage || s->eq != s0->eq ||
            s->p.force_order != s0->p.force_order)
            return fail(LBM_EINVAL,
                        "batch members must share lattice, storage, eq_order and force_order");
    }
    return LBM_OK;
}

// A member's tile-table descriptor; its tiles start at first_tile.
void fill_tile_sim(TileSim &t, const lbm_sim *s, int64_t first_tile)
{
    t.pop[0] = s->pop[0];
    t.pop[1] = s->pop[1];
    t.ctr = s->ctr;
    t.cur = s->cur;
    t.chunks_x = int32_t((s->p.nx + 63) / 64);
    t.tile_begin = first_tile;
    t.gd = s->gd;
    t.fd = s->fd;
    t.co = s->co;
    t.wd = s->wd;
}

// Write the tile table of `sims` (64-cell tiles) to begin[count + 1] and
// tab[count] on `stream`; tiles = the length of the list, walls = some member
// has plates.
hipError_t upload_table(lbm_sim *const *sims, int32_t count, int64_t *begin, TileSim *tab,
                        hipStream_t stream, int64_t &tiles, bool &walls)
{
    tiles = 0;
    walls = false;
    for (int32_t first = 0; first < count; first += TABLE_CHUNK) {
        TableChunk c;
        std::memset(&c, 0, sizeof c);
        c.first = first;
        c.n = std::min<int32_t>(TABLE_CHUNK, count - first);
        for (int32_t k = 0; k < c.n; ++k) {
            const lbm_sim *s = sims[first + k];
            fill_tile_sim(c.sims[k], s, tiles);
            c.begin[k] = tiles;
            tiles += int64_t(c.sims[k].chunks_x) * s->p.ny * s->p.nz;
            walls = walls || s->wd.on;
        }
        c.last = first + c.n == count;
        c.end = tiles;
        hipLaunchKernelGGL(table_fill_kernel, dim3(1), dim3(64), 0, stream, c, begin, tab);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}
}  // namespace

struct lbm_batch {
    int32_t max_sims;
    hipStream_t stream;
    char *ws;        // device workspace: begin[max_sims + 1], then TileSim[max_sims]
    int64_t *begin;  // device: first tile of each member
    TileSim *table;  // device: the members
    std::vector<lbm_sim *> sims;
    std::vector<int64_t> step_at_set;  // members' step counts when the table was built
    std::vector<int64_t> gen_at_set;   // members' launch-argument generations then
    int64_t generation;                // bumped whenever the table or launch shape changes
    int64_t steps_done;                // batch steps since the table was built
    int64_t ntiles;
    int threads;     // threads per block (tiles of 64 cells, one per wavefront)
    int64_t blocks;  // 0: one block per tile
    bool walls;           // some member has plates
};

struct lbm_graph {
    lbm_sim *s;
    lbm_batch *b;
    int64_t nsteps;
    int64_t gen;     // launch-argument generation of s, or batch generation of b
    int32_t cur0;    // s: buffer holding the state at capture
    int32_t parity0; // b: parity of the batch step count at capture
    hipStream_t stream;
    hipGraph_t graph;
    hipGraphExec_t exec;
};

namespace {
constexpr int BATCH_DEFAULT_THREADS = 128;  // measured best on the serving and small-grid mixes

size_t batch_begin_bytes(int32_t max_sims) { return align_up(size_t(max_sims + 1) * 8); }

lbm_status batch_check(const lbm_batch *b)
{
    for (size_t k = 0; k < b->sims.size(); ++k) {
        if (b->sims[k]->step != b->step_at_set[k] + b->steps_done)
            return fail(LBM_EINVAL,
                        "member %zu was stepped outside the batch; call lbm_batch_set again", k);
        if (b->sims[k]->gen != b->gen_at_set[k])
            return fail(LBM_EINVAL,
                        "member %zu changed force, block or stream; call lbm_batch_set again", k);
    }
    return LBM_OK;
}

// Members between plates need the row sums of their current state; those the
// state was not produced by a step get them on the batch's stream.
hipError_t batch_wall_densities(lbm_batch *b)
{
    for (lbm_sim *s : b->sims) {
        hipError_t e = wall_densities(s, b->stream);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Enqueues nsteps batch steps; done is the number enqueued (all of them unless
// a launch failed).
lbm_status batch_launch(lbm_batch *b, int64_t nsteps, int64_t &done)
{
    const lbm_sim *s0 = b->sims[0];
    for (done = 0; done < nsteps; ++done) {
        const int parity = int((b->steps_done + done) & 1);
        const BatchLaunch bl{b->begin,  b->table,   int(b->sims.size()), b->ntiles, parity,
                             b->threads, b->blocks, b->stream,           b->walls};
        hipError_t e = launch_multi_step(s0->p.lattice, s0->p.storage, s0->eq, s0->p.force_order,
                                         bl);
        if (e != hipSuccess) return dev_fail(e, "multi-grid step launch");
    }
    return LBM_OK;
}

// Set the members and write their tile table into the batch workspace on the
// batch's stream (asynchronous: no host buffer has to outlive the call).
lbm_status batch_build(lbm_batch *b, lbm_sim *const *sims, int32_t count)
{
    lbm_status st = check_members(sims, count);
    if (st != LBM_OK) return st;
    int64_t tiles = 0;
    bool walls = false;
    hipError_t e = upload_table(sims, count, b->begin, b->table, b->stream, tiles, walls);
    if (e != hipSuccess) return dev_fail(e, "tile table fill launch");
    b->sims.assign(sims, sims + count);
    b->step_at_set.clear();
    b->gen_at_set.clear();
    for (lbm_sim *s : b->sims) {
        b->step_at_set.push_back(s->step);
        b->gen_at_set.push_back(s->gen);
    }
    b->steps_done = 0;
    b->generation++;
    b->ntiles = tiles;
    b->walls = walls;
    return LBM_OK;
}

void batch_advance(lbm_batch *b, int64_t nsteps)
{
    b->steps_done += nsteps;
    for (lbm_sim *s : b->sims) {
        s->cur ^= int(nsteps & 1);
        s->step += nsteps;
    }
}
}  // namespace

extern "C" {

size_t lbm_batch_workspace_bytes(int32_t max_sims)
{
    if (max_sims < 1 || max_sims > (1 << 20)) return 0;
    return batch_begin_bytes(max_sims) + align_up(size_t(max_sims) * sizeof(TileSim));
}

lbm_status lbm_batch_create(int32_t max_sims, void *workspace, size_t workspace_bytes,
                            void *hip_stream, lbm_batch **out)
{
    if (!out) return fail(LBM_EINVAL, "out is NULL");
    *out = nullptr;
    if (max_sims < 1 || max_sims > (1 << 20))
        return fail(LBM_EINVAL, "max_sims must be in [1, 2^20] (got %d)", max_sims);
    if (!workspace) return fail(LBM_EINVAL, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(workspace) % ALIGN)
        return fail(LBM_EINVAL, "workspace must be 256-byte aligned");
    if (workspace_bytes < lbm_batch_workspace_bytes(max_sims))
        return fail(LBM_ENOSPACE, "batch workspace has %zu bytes, %zu needed", workspace_bytes,
                    lbm_batch_workspace_bytes(max_sims));
    lbm_batch *b = new (std::nothrow) lbm_batch();
    if (!b) return fail(LBM_EINVAL, "out of host memory");
    b->max_sims = max_sims;
    b->stream = static_cast<hipStream_t>(hip_stream);
    b->ws = static_cast<char *>(workspace);
    b->begin = reinterpret_cast<int64_t *>(b->ws);
    b->table = reinterpret_cast<TileSim *>(b->ws + batch_begin_bytes(max_sims));
    b->steps_done = 0;
    b->ntiles = 0;
    b->generation = 0;
    b->threads = BATCH_DEFAULT_THREADS;
    b->blocks = 0;
    b->walls = false;
    *out = b;
    return ok();
}

lbm_status lbm_batch_set(lbm_batch *b, lbm_sim *const *sims, int32_t count)
{
    if (!b) return fail(LBM_EINVAL, "batch is NULL");
    if (!sims) return fail(LBM_EINVAL, "sims is NULL");
    if (count < 1 || count > b->max_sims)
        return fail(LBM_EINVAL, "count must be in [1, %d] (got %d)", b->max_sims, count);
    lbm_status st = batch_build(b, sims, count);
    if (st != LBM_OK) return st;
    return ok();
}

lbm_status lbm_batch_step(lbm_batch *b, int64_t nsteps)
{
    if (!b) return fail(LBM_EINVAL, "batch is NULL");
    if (nsteps < 0) return fail(LBM_EINVAL, "nsteps must be >= 0");
    if (b->sims.empty()) return fail(LBM_EINVAL, "batch has no members (call lbm_batch_set)");
    lbm_status st = batch_check(b);
    if (st != LBM_OK) return st;
    TraceRange range("lbm_batch_step");
    hipError_t e = batch_wall_densities(b);
    if (e != hipSuccess) return dev_fail(e, "wall density kernel launch");
    int64_t done = 0;
    st = batch_launch(b, nsteps, done);
    batch_advance(b, done);  // the steps enqueued before a failed launch still run
    if (st != LBM_OK) {
        for (lbm_sim *s : b->sims) s->wall_fresh = false;
        return st;
    }
    return ok();
}

lbm_status lbm_batch_set_launch(lbm_batch *b, int32_t threads, int64_t blocks)
{
    if (!b) return fail(LBM_EINVAL, "batch is NULL");
    if (threads != 0 && threads != 64 && threads != 128 && threads != 256)
        return fail(LBM_EINVAL, "threads must be 0, 64, 128 or 256 (got %d)", threads);
    if (blocks < 0 || blocks > 0x7fffffff)
        return fail(LBM_EINVAL, "blocks must be in [0, 2^31 - 1]");
    // the tiles do not depend on the launch shape: the table stays as it is
    b->threads = threads ? threads : BATCH_DEFAULT_THREADS;
    b->blocks = blocks;
    b->generation++;  // graphs captured with the old shape are stale
    return ok();
}

void lbm_batch_destroy(lbm_batch *b) { delete b; }

}  // extern "C"

// ---------------------------------------------------------------------------
// batch step without a workspace: the tile table in a fixed device array
// ---------------------------------------------------------------------------
namespace {
constexpr size_t NOALLOC_BEGIN_BYTES = (size_t(LBM_NOALLOC_MAX_SIMS + 1) * 8 + ALIGN - 1) /
                                       ALIGN * ALIGN;
constexpr size_t NOALLOC_SCRATCH_BYTES =
    NOALLOC_BEGIN_BYTES + size_t(LBM_NOALLOC_MAX_SIMS) * sizeof(TileSim);
constexpr int NOALLOC_MAX_DEVICES = 64;

std::mutex g_scratch_mu;
void *g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};
}  // namespace

// The tile table of lbm_batch_step_noalloc: tile offsets
// (LBM_NOALLOC_MAX_SIMS + 1 int64, padded to 256 bytes), then one TileSim per
// member.  Host code reaches it only through the address hipGetSymbolAddress
// returns for the current device.
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

namespace {
// Device address of `scratch` on the current device, resolved once per device.
hipError_t scratch_address(unsigned char **out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = p;
    }
    *out = static_cast<unsigned char *>(g_scratch_ptr[dev]);
    return hipSuccess;
}

}  // namespace

extern "C" {

lbm_status lbm_batch_step_noalloc(lbm_sim *const *sims, int32_t count, int64_t nsteps,
                                  void *hip_stream)
{
    if (!sims) return fail(LBM_EINVAL, "sims is NULL");
    if (count < 1 || count > LBM_NOALLOC_MAX_SIMS)
        return fail(LBM_EINVAL,
                    "count must be in [1, %d]: the fixed tile table holds %d members (got %d)",
                    LBM_NOALLOC_MAX_SIMS, LBM_NOALLOC_MAX_SIMS, count);
    if (nsteps < 0) return fail(LBM_EINVAL, "nsteps must be >= 0");
    lbm_status st = check_members(sims, count);
    if (st != LBM_OK) return st;
    if (nsteps == 0) return ok();
    unsigned char *base = nullptr;
    hipError_t e = scratch_address(&base);
    if (e != hipSuccess) return dev_fail(e, "tile table address");
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    TraceRange range("lbm_batch_step_noalloc");
    for (int32_t k = 0; k < count; ++k) {
        e = wall_densities(sims[k], stream);
        if (e != hipSuccess) return dev_fail(e, "wall density kernel launch");
    }
    int64_t *begin = reinterpret_cast<int64_t *>(base);
    TileSim *table = reinterpret_cast<TileSim *>(base + NOALLOC_BEGIN_BYTES);
    int64_t tiles = 0;
    bool walls = false;
    e = upload_table(sims, count, begin, table, stream, tiles, walls);
    if (e != hipSuccess) return dev_fail(e, "tile table fill launch");
    const lbm_sim *s0 = sims[0];
    int64_t done = 0;
    for (; done < nsteps; ++done) {
        const BatchLaunch bl{begin,  table, int(count), tiles, int(done & 1), BATCH_DEFAULT_THREADS,
                             0,      stream, walls};
        e = launch_multi_step(s0->p.lattice, s0->p.storage, s0->eq, s0->p.force_order, bl);
        if (e != hipSuccess) break;
    }
    // the steps enqueued before a failed launch still run
    for (int32_t k = 0; k < count; ++k) {
        sims[k]->cur ^= int(done & 1);
        sims[k]->step += done;
        if (e != hipSuccess) sims[k]->wall_fresh = false;
    }
    if (e != hipSuccess) return dev_fail(e, "multi-grid step launch");
    return ok();
}

// ---------------------------------------------------------------------------
// captured step loops
// ---------------------------------------------------------------------------
lbm_status lbm_graph_create(lbm_sim *s, lbm_batch *b, int64_t nsteps, lbm_graph **out)
{
    if (!out) return fail(LBM_EINVAL, "out is NULL");
    *out = nullptr;
    if ((s == nullptr) == (b == nullptr))
        return fail(LBM_EINVAL, "give exactly one of a simulation and a batch");
    if (nsteps <= 0 || (nsteps & 1))
        return fail(LBM_EINVAL, "nsteps must be even and > 0 (got %lld)", (long long)nsteps);
    if (b && b->sims.empty()) return fail(LBM_EINVAL, "batch has no members");
    if (b) {
        lbm_status stc = batch_check(b);
        if (stc != LBM_OK) return stc;
    }
    hipStream_t stream = s ? s->stream : b->stream;
    if (!stream) return fail(LBM_EINVAL, "graph capture needs a non-null stream");
    lbm_graph *g = new (std::nothrow) lbm_graph();
    if (!g) return fail(LBM_EINVAL, "out of host memory");
    g->s = s;
    g->b = b;
    g->nsteps = nsteps;
    g->stream = stream;
    g->gen = s ? s->gen : b->generation;
    g->cur0 = s ? s->cur : 0;
    g->parity0 = b ? int32_t(b->steps_done & 1) : 0;
    hipError_t e = s ? wall_densities(s) : batch_wall_densities(b);  // not captured
    if (e != hipSuccess) {
        delete g;
        return dev_fail(e, "wall density kernel launch");
    }
    e = hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        delete g;
        return dev_fail(e, "begin capture");
    }
    lbm_status st = LBM_OK;
    if (s) {
        int cur = s->cur;  // nothing runs during capture: the handle keeps its state
        int64_t done = 0;
        hipError_t el = launch_steps(s, cur, nsteps, done);
        if (el != hipSuccess) st = dev_fail(el, "step launch during capture");
    } else {
        int64_t done = 0;
        st = batch_launch(b, nsteps, done);
    }
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(stream, &graph);
    if (st != LBM_OK || e != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        delete g;
        return st != LBM_OK ? st : dev_fail(e, "end capture");
    }
    e = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(graph);
        delete g;
        return dev_fail(e, "graph instantiate");
    }
    g->graph = graph;
    *out = g;
    return ok();
}

lbm_status lbm_graph_launch(lbm_graph *g, int64_t repeats)
{
    if (!g) return fail(LBM_EINVAL, "graph is NULL");
    if (repeats < 0) return fail(LBM_EINVAL, "repeats must be >= 0");
    if (g->s && (g->s->gen != g->gen || g->s->cur != g->cur0))
        return fail(LBM_EINVAL,
                    "the simulation changed since capture (force, block, stream or buffer parity)");
    if (g->b) {
        if (g->b->generation != g->gen || int32_t(g->b->steps_done & 1) != g->parity0)
            return fail(LBM_EINVAL, "the batch changed since capture (members or step parity)");
        lbm_status stc = batch_check(g->b);
        if (stc != LBM_OK) return stc;
    }
    TraceRange range("lbm_graph_launch");
    if (repeats > 0) {
        // the replayed steps read the partial sums of the state they start from
        hipError_t e = g->s ? wall_densities(g->s) : batch_wall_densities(g->b);
        if (e != hipSuccess) return dev_fail(e, "wall density kernel launch");
    }
    int64_t r = 0;
    hipError_t e = hipSuccess;
    for (; r < repeats && e == hipSuccess; ++r) e = hipGraphLaunch(g->exec, g->stream);
    if (e != hipSuccess) --r;  // the failed replay was not enqueued
    // the replays enqueued run nsteps (even) steps each: buffers end where they started
    const int64_t n = g->nsteps * r;
    if (g->s) {
        g->s->step += n;
    } else {
        batch_advance(g->b, n);
    }
    if (e != hipSuccess) return dev_fail(e, "graph launch");
    return ok();
}

void lbm_graph_destroy(lbm_graph *g)
{
    if (!g) return;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
}

}  // extern "C"
