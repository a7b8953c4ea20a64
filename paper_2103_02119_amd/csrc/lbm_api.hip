// Host side of the C ABI declared in include/lbm.h: argument validation,
// model constants, buffer management, state tracking and kernel launches.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <mutex>
#include <new>

#include "../../include/lbm.h"
#include "lbm_internal.h"

using namespace lbm;

namespace {

thread_local char g_create_error[512] = "no error";

// Storage form of a population buffer.
enum Form { kEmpty = 0, kPre = 1, kPost = 2 };

}  // namespace

// reduction partials (up to 8 values per block), then the results
static constexpr size_t kResults = 8 * static_cast<size_t>(kMaxPartials);

// Scratch of the allocation-free check (lbm_check_into): the per-workgroup
// partial sums of the fused residual-and-sums reduction, at most kMaxPartials
// workgroups of 8 values (256 KiB).  Each GPU the library runs on holds its
// own copy until the process ends.  In host code `scratch` names a host-side
// stand-in, not device memory: its device address on each GPU is looked up
// once (scratch_on) and only that address is handed to kernels.
static constexpr size_t kScratchDoubles = 8 * static_cast<size_t>(kMaxPartials);
static __device__ __align__(256) double scratch[kScratchDoubles];
static constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static double *g_scratch_ptr[kMaxDevices];

// Device address of `scratch` on device dev (which must be current);
// nullptr if it cannot be found.
static double *scratch_on(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
        g_scratch_ptr[dev] = static_cast<double *>(p);
    }
    return g_scratch_ptr[dev];
}

struct lbm_ctx {
    int nx, ny;
    double a;
    double rates[9];
    lbm_bc bc;
    lbm_opts opts;
    int prec, coll;
    hipStream_t stream;
    Geometry G;
    Consts<double> Kd;
    Consts<float> Kf;
    HostSide H;
    bool higher_unit;
    size_t f_bytes;
    void *f[2];
    bool owns[2];
    int cur;          // buffer with the current state
    int form[2];      // Form of each buffer's contents
    int prev_valid;   // the other buffer holds the state one step earlier
    double *d_partials;  // reduction partials + results
    double *h_check;     // pinned host copy of the last lbm_check_async (lazy)
    hipEvent_t check_ev; // recorded after that copy
    long check_step;     // steps done when it was enqueued; -1 = none
    double *d_stage;     // FP64 staging for host transfers (lazy)
    size_t stage_bytes;
    unsigned char *d_mask;        // obstacle mask [ny][pitch] (or null)
    unsigned char *d_tile_solid;  // per step tile: obstacle in its neighbourhood
    int steps_per_launch;         // 0 automatic, 1, 2 (lbm_set_steps_per_launch)
    int two_step_form;            // kFormAuto, kFormRegister, kFormStaged
    double *scratch;              // device address of `scratch` on this context's GPU
    long steps;
    char err[512];
};

static int fail_ctx(lbm_ctx *ctx, int code, const char *fmt, ...) {
    char *buf = ctx ? ctx->err : g_create_error;
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, 512, fmt, ap);
    va_end(ap);
    return code;
}

#define HIP_OR_FAIL(ctx, call)                                                          \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess)                                                           \
            return fail_ctx((ctx), e_ == hipErrorOutOfMemory ? LBM_E_NOMEM : LBM_E_DEVICE, \
                            "%s failed: %s", #call, hipGetErrorString(e_));            \
    } while (0)


static size_t value_bytes(int prec) { return f32_storage(prec) ? sizeof(float) : sizeof(double); }

extern "C" void lbm_default_opts(lbm_opts *o) {
    if (!o) return;
    memset(o, 0, sizeof(*o));
    o->cs2 = 0.0;
    o->rho0 = 1.0;
    o->collision = LBM_RC;
    o->precision = LBM_FP64;
    o->corrections = 1;
}

extern "C" int lbm_required_bytes(int nx, int ny, int precision, size_t *f_bytes) {
    if (!f_bytes) return fail_ctx(nullptr, LBM_E_INVAL, "f_bytes is NULL");
    if (nx < 3 || ny < 3) return fail_ctx(nullptr, LBM_E_INVAL, "nx and ny must be >= 3");
    if (precision < LBM_FP64 || precision > LBM_FP32_DEV_F64)
        return fail_ctx(nullptr, LBM_E_INVAL, "unknown precision %d", precision);
    const long long plane = static_cast<long long>(pitch_of(nx)) * ny;
    // node offsets inside a plane are 32-bit byte offsets in the kernels
    if (plane * static_cast<long long>(value_bytes(precision)) > 0xffffffffLL)
        return fail_ctx(nullptr, LBM_E_INVAL, "lattice too large: %lld values per plane", plane);
    *f_bytes = static_cast<size_t>(9) * plane * value_bytes(precision);
    return LBM_OK;
}

// Equilibrium in product form (the library's own, used for the rest weights
// and the moving-wall terms): feq_k = rho Px(cx) Py(cy).
static double feq_host(int k, double rho, double ux, double uy, double s, double a) {
    const int cx = cx_of(k), cy = cy_of(k);
    const double px = cx == 0 ? 1.0 - s - ux * ux : 0.5 * (s + ux * ux + cx * ux);
    const double py = cy == 0 ? 1.0 - (s + uy * uy) / (a * a)
                              : 0.5 * (s + uy * uy + cy * a * uy) / (a * a);
    return rho * px * py;
}

namespace lbm {

template <typename R>
void fill_consts(const CaseSpec &c, Consts<R> &K) {
    const double a = c.a, s = c.cs2;
    const double *w = c.rates;
    K.a = R(a);
    K.inv_a = R(1.0 / a);
    K.a2 = R(a * a);
    K.inv_a2 = R(1.0 / (a * a));
    K.half_inv_a = R(0.5 / a);
    K.s = R(s);
    K.s2 = R(s * s);
    K.rr = R(c.prec == kFP64 ? 0.0 : c.rho0);
    K.Fx = R(c.force[0]);
    K.Fy = R(c.force[1]);
    K.hFx = R(0.5 * c.force[0]);
    K.hFy = R(0.5 * c.force[1]);
    for (int j = 0; j < 9; ++j) {
        K.w[j] = R(w[j]);
        K.om[j] = R(1.0 - w[j]);
        K.sw[j] = R(1.0 - 0.5 * w[j]);
    }
    K.k3 = R(1.0 / w[3] - 0.5);
    K.k4 = R(1.0 / w[4] - 0.5);
    // Eq. 40 divided by rho, without the velocity terms
    K.b1c = R(-2.0 * s / w[3] - (-3.0 * s + 1.0) / 2.0);
    K.b2c = R(-2.0 * s / w[3] - (-3.0 * s + a * a) / 2.0);
    K.c1c = R(-2.0 * s / w[4] - (-3.0 * s + 1.0) / 2.0);
    K.c2c = R(2.0 * s / w[4] - (3.0 * s - a * a) / 2.0);
    K.e1 = R((3.0 * s - 1.0) / 2.0);
    K.e2 = R((3.0 * s - a * a) / 2.0);
    K.q1 = R(1.0 - 3.0 * s);
    K.q2 = R(a * a - 3.0 * s);
    for (int k = 0; k < 9; ++k)
        K.rest[k] = R(c.prec == kFP64 ? c.rho0 * feq_host(k, 1.0, 0.0, 0.0, s, a) : 0.0);
    for (int f = 0; f < 4; ++f) {
        const bool mv = c.bc.type[f] == LBM_BC_MOVING_WALL;
        const double ux = mv ? c.bc.u_wall[f][0] : 0.0, uy = mv ? c.bc.u_wall[f][1] : 0.0;
        for (int k = 0; k < 9; ++k)
            K.dwall[f][k] = R(feq_host(opp_of(k), c.rho0, ux, uy, s, a) -
                              feq_host(k, c.rho0, ux, uy, s, a));
    }
}
template void fill_consts<float>(const CaseSpec &, Consts<float> &);
template void fill_consts<double>(const CaseSpec &, Consts<double> &);

void fill_host_side(const CaseSpec &c, HostSide &H) {
    for (int k = 0; k < 9; ++k) H.wrest[k] = feq_host(k, 1.0, 0.0, 0.0, c.cs2, c.a);
    H.rho0 = c.rho0;
    H.a = c.a;
    H.s = c.cs2;
    H.Fx = c.force[0];
    H.Fy = c.force[1];
    H.dev = c.prec == kFP64 ? 0 : 1;
}

void base_geometry(const CaseSpec &c, size_t f_bytes, Geometry &G) {
    memset(&G, 0, sizeof(G));
    G.nx = c.nx;
    G.ny = c.ny;
    G.pitch = pitch_of(c.nx);
    G.plane = static_cast<long long>(G.pitch) * c.ny;
    for (int f = 0; f < 4; ++f) G.bc[f] = c.bc.type[f];
    G.corr = c.corr;
    G.buf_ok = f_bytes < 0xffffffffULL ? 1 : 0;
    G.nseg = (c.nx + kWave - 1) / kWave;
}

void set_rows(Geometry &G, int rows) {
    if (rows > kMaxRows) rows = kMaxRows;
    if (rows > G.ny) rows = G.ny;
    if (rows < 1) rows = 1;
    G.rows = rows;
    G.nchunk = (G.ny + rows - 1) / rows;
    G.ntile = G.nseg * G.nchunk;
    // whole groups of 8 workgroups, so that the remap of workgroups to the
    // 8 XCDs always applies (measured: 13.7 vs 16.1 us per step on the
    // 512 x 1024 cavity); the padding workgroups find no tile and exit
    const int need = (G.ntile + kWavesPerBlock - 1) / kWavesPerBlock;
    G.nblocks = (need + 7) / 8 * 8;
    G.xcd_remap = 1;
}

int pitch_of(int nx) { return (nx + kWave - 1) / kWave * kWave; }

int tile_has_solid(const Geometry &G, const unsigned char *m, int seg, int chunk) {
    if (!m) return 0;
    const int x0 = seg * kWave, j0 = chunk * G.rows;
    const int j1 = j0 + G.rows < G.ny ? j0 + G.rows : G.ny;
    // the tile pulls rows j0 - 1 .. j1 and columns x0 - 1 .. x0 + 64; the
    // densities of its ring rows and halo columns pull one node further out
    for (int jj = j0 - 2; jj <= j1 + 1; ++jj) {
        int j = jj;
        if (j < 0 || j >= G.ny) {
            if (G.bc[j < 0 ? kYmin : kYmax] != kPeriodic) continue;
            j = (j + G.ny) % G.ny;
        }
        for (int xx = x0 - 2; xx <= x0 + kWave + 1; ++xx) {
            int x = xx;
            if (x < 0 || x >= G.nx) {
                if (G.bc[x < 0 ? kXmin : kXmax] != kPeriodic) continue;
                x = (x + G.nx) % G.nx;
            }
            if (m[static_cast<size_t>(j) * G.nx + x]) return 1;
        }
    }
    return 0;
}

}  // namespace lbm

// Launch shape and store policy, from measurements on MI355X: a wavefront
// marches 2 rows on lattices below ~1M nodes (FP32) where latency dominates,
// 4 below ~4M and 8 above; stores are non-temporal once the two population
// buffers are well beyond the 256 MB Infinity Cache.
void lbm::make_spec(int nx, int ny, double r, const double *rates, const lbm_bc *bc,
                    const lbm_opts *o, CaseSpec &spec) {
    spec.nx = nx;
    spec.ny = ny;
    spec.a = r;
    memcpy(spec.rates, rates, sizeof(spec.rates));
    spec.bc = *bc;
    spec.cs2 = o->cs2;
    spec.force[0] = o->force[0];
    spec.force[1] = o->force[1];
    spec.rho0 = o->rho0;
    spec.prec = o->precision;
    spec.corr = o->corrections ? 1 : 0;
}

const char *lbm::create_error_text() { return g_create_error; }

int lbm::set_create_error(const char *msg) {
    snprintf(g_create_error, sizeof(g_create_error), "%s", msg);
    return LBM_E_INVAL;
}

int lbm::auto_rows(long long nodes, int prec) {
    if (nodes < (1LL << 20) && prec == kFP32Dev) return 2;
    if (nodes < (1LL << 22)) return 4;
    return 8;
}

static void choose_launch(lbm_ctx *c) {
    Geometry &G = c->G;
    const long long nodes = static_cast<long long>(c->nx) * c->ny;
    const int rows = c->opts.rows_per_wave > 0 ? c->opts.rows_per_wave : auto_rows(nodes, c->prec);
    set_rows(G, rows);
    G.nt_store = 2.0 * static_cast<double>(c->f_bytes) > 512.0 * 1024 * 1024 ? 1 : 0;
    // an explicit rows-per-wavefront choice selects the march; otherwise the
    // tile kernel, with taller tiles once the buffers exceed the Infinity
    // Cache (measured: 8 rows best on the 512 x 1024 cavity, 16 on the
    // 2048 x 8192 lattice)
    G.tile_rows = c->opts.rows_per_wave > 0 ? 0 : (G.nt_store ? 16 : 8);
}

int lbm::validate_case(int nx, int ny, double r, const double *rates, const lbm_bc *bc,
                       const lbm_opts *o) {
    if (nx < 3 || ny < 3) return fail_ctx(nullptr, LBM_E_INVAL, "nx and ny must be >= 3");
    if (!(r > 0.0) || !isfinite(r)) return fail_ctx(nullptr, LBM_E_INVAL, "r must be > 0");
    if (!rates) return fail_ctx(nullptr, LBM_E_INVAL, "rates is NULL");
    for (int j = 0; j < 9; ++j)
        if (!(rates[j] > 0.0 && rates[j] < 2.0))
            return fail_ctx(nullptr, LBM_E_INVAL, "rates[%d] = %g is not in (0, 2)", j, rates[j]);
    const double lim = fmin(1.0, r * r);
    if (!(o->cs2 > 0.0 && o->cs2 < lim))
        return fail_ctx(nullptr, LBM_E_INVAL, "cs2 = %g is not in (0, min(1, r^2) = %g)", o->cs2,
                        lim);
    if (!bc) return fail_ctx(nullptr, LBM_E_INVAL, "bc is NULL");
    for (int f = 0; f < 4; ++f)
        if (bc->type[f] < LBM_BC_PERIODIC || bc->type[f] > LBM_BC_MOVING_WALL)
            return fail_ctx(nullptr, LBM_E_INVAL, "unknown boundary type %d on face %d",
                            bc->type[f], f);
    if ((bc->type[0] == LBM_BC_PERIODIC) != (bc->type[1] == LBM_BC_PERIODIC) ||
        (bc->type[2] == LBM_BC_PERIODIC) != (bc->type[3] == LBM_BC_PERIODIC))
        return fail_ctx(nullptr, LBM_E_INVAL, "opposite faces must both be periodic or both not");
    if (o->collision != LBM_RC && o->collision != LBM_RNR)
        return fail_ctx(nullptr, LBM_E_INVAL, "unknown collision %d", o->collision);
    if (o->precision < LBM_FP64 || o->precision > LBM_FP32_DEV_F64)
        return fail_ctx(nullptr, LBM_E_INVAL, "unknown precision %d", o->precision);
    if (!(o->rho0 > 0.0)) return fail_ctx(nullptr, LBM_E_INVAL, "rho0 must be > 0");
    if (!isfinite(o->force[0]) || !isfinite(o->force[1]))
        return fail_ctx(nullptr, LBM_E_INVAL, "force must be finite");
    if (o->rows_per_wave < 0 || o->rows_per_wave > kMaxRows)
        return fail_ctx(nullptr, LBM_E_INVAL, "rows_per_wave must be in [0, %d]", kMaxRows);
    if ((o->f_a == nullptr) != (o->f_b == nullptr))
        return fail_ctx(nullptr, LBM_E_INVAL, "give both f_a and f_b or neither");
    return LBM_OK;
}

static int ensure_stage(lbm_ctx *c, size_t bytes) {
    if (c->stage_bytes >= bytes) return LBM_OK;
    if (c->d_stage) {
        HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
        HIP_OR_FAIL(c, hipFree(c->d_stage));
        c->d_stage = nullptr;
        c->stage_bytes = 0;
    }
    HIP_OR_FAIL(c, hipMalloc(&c->d_stage, bytes));
    c->stage_bytes = bytes;
    return LBM_OK;
}

static int init_fields_device(lbm_ctx *c, const double *drho, const double *dux,
                              const double *duy) {
    HIP_OR_FAIL(c, launch_init_feq(c->prec, c->f[c->cur], drho, dux, duy, c->G, c->H, c->stream));
    c->form[c->cur] = kPre;
    c->form[1 - c->cur] = kEmpty;
    c->prev_valid = 0;
    return LBM_OK;
}

extern "C" int lbm_create(int nx, int ny, double r, const double rates[9], const lbm_bc *bc,
                          const lbm_opts *opts, lbm_ctx **out) {
    if (!out) return fail_ctx(nullptr, LBM_E_INVAL, "out is NULL");
    *out = nullptr;
    lbm_opts o;
    if (opts) o = *opts; else lbm_default_opts(&o);
    if (o.rho0 == 0.0) o.rho0 = 1.0;
    if (o.cs2 == 0.0) o.cs2 = fmin(1.0 / 3.0, 0.64 * r * r);
    int rc = validate_case(nx, ny, r, rates, bc, &o);
    if (rc != LBM_OK) return rc;
    size_t need = 0;
    rc = lbm_required_bytes(nx, ny, o.precision, &need);
    if (rc != LBM_OK) return rc;
    if (o.f_a && o.f_bytes < need)
        return fail_ctx(nullptr, LBM_E_INVAL, "caller buffers hold %zu bytes, %zu needed",
                        o.f_bytes, need);
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1)
        return fail_ctx(nullptr, LBM_E_DEVICE, "no usable GPU");

    lbm_ctx *c = new (std::nothrow) lbm_ctx();
    if (!c) return fail_ctx(nullptr, LBM_E_NOMEM, "out of host memory");
    c->check_step = -1;
    c->nx = nx;
    c->ny = ny;
    c->a = r;
    memcpy(c->rates, rates, sizeof(c->rates));
    c->bc = *bc;
    c->opts = o;
    c->prec = o.precision;
    c->coll = o.collision;
    c->stream = static_cast<hipStream_t>(o.stream);
    c->higher_unit = rates[6] == 1.0 && rates[7] == 1.0 && rates[8] == 1.0;
    snprintf(c->err, sizeof(c->err), "no error");

    CaseSpec spec;
    make_spec(nx, ny, r, rates, bc, &o, spec);
    c->f_bytes = need;
    base_geometry(spec, need, c->G);
    choose_launch(c);
    fill_consts(spec, c->Kd);
    fill_consts(spec, c->Kf);
    fill_host_side(spec, c->H);

    int status = LBM_OK;
    if (o.f_a) {
        c->f[0] = o.f_a;
        c->f[1] = o.f_b;
    } else {
        for (int i = 0; i < 2 && status == LBM_OK; ++i) {
            hipError_t e = hipMalloc(&c->f[i], need);
            if (e != hipSuccess) {
                c->f[i] = nullptr;
                status = fail_ctx(nullptr, e == hipErrorOutOfMemory ? LBM_E_NOMEM : LBM_E_DEVICE,
                                  "hipMalloc of %zu bytes failed: %s", need, hipGetErrorString(e));
            } else {
                c->owns[i] = true;
            }
        }
    }
    if (status == LBM_OK) {
        hipError_t e = hipMalloc(&c->d_partials, (kResults + 8) * sizeof(double));
        if (e != hipSuccess) {
            c->d_partials = nullptr;
            status = fail_ctx(nullptr, LBM_E_DEVICE, "hipMalloc of partials failed: %s",
                              hipGetErrorString(e));
        }
    }
    if (status == LBM_OK) {
        // the allocation-free check's scratch on this GPU, looked up once per
        // device while it is current
        int dev = -1;
        if (hipGetDevice(&dev) == hipSuccess) c->scratch = scratch_on(dev);
        if (!c->scratch)
            status = fail_ctx(nullptr, LBM_E_DEVICE, "device address of the check scratch not found");
    }
    if (status == LBM_OK) {
        c->cur = 0;
        status = init_fields_device(c, nullptr, nullptr, nullptr);
        if (status != LBM_OK) snprintf(g_create_error, sizeof(g_create_error), "%s", c->err);
    }
    if (status != LBM_OK) {
        lbm_destroy(c);
        return status;
    }
    *out = c;
    return LBM_OK;
}

extern "C" int lbm_set_fields(lbm_ctx *c, const double *rho, const double *ux, const double *uy) {
    if (!c) return fail_ctx(nullptr, LBM_E_INVAL, "ctx is NULL");
    const size_t n = static_cast<size_t>(c->nx) * c->ny;
    int rc = ensure_stage(c, 3 * n * sizeof(double));
    if (rc != LBM_OK) return rc;
    double *d[3] = {nullptr, nullptr, nullptr};
    const double *h[3] = {rho, ux, uy};
    for (int i = 0; i < 3; ++i)
        if (h[i]) {
            d[i] = c->d_stage + i * n;
            HIP_OR_FAIL(c, hipMemcpyAsync(d[i], h[i], n * sizeof(double), hipMemcpyHostToDevice,
                                          c->stream));
        }
    rc = init_fields_device(c, d[0], d[1], d[2]);
    if (rc != LBM_OK) return rc;
    HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
    return LBM_OK;
}

// Steps per launch a run takes: two (the temporally blocked kernel) where
// the tile kernel applies (no obstacle mask) unless the caller asked for one
// (the automatic choice takes two on every such lattice: measured faster
// from 64 x 32 nodes up, in the Infinity Cache and beyond it); one otherwise.
static int steps_per_launch(const lbm_ctx *c) {
    if (!uses_tile_kernel(c->G) || c->steps_per_launch == 1) return 1;
    return 2;
}

extern "C" int lbm_step(lbm_ctx *c, long n) {
    if (!c) return fail_ctx(nullptr, LBM_E_INVAL, "ctx is NULL");
    if (n < 0) return fail_ctx(c, LBM_E_INVAL, "n must be >= 0");
    const int k = steps_per_launch(c);
    // With two steps per launch the state before the last step is not kept.
    // The automatic choice ends every call with a one-step launch, so that
    // the residual of the last step stays available; an explicit 2 takes
    // pairs as long as two steps remain.
    const long last_single = c->steps_per_launch == 2 ? 1 : 2;
    for (long left = n; left > 0;) {
        const int src = c->cur, dst = 1 - c->cur;
        const bool pull = c->form[src] == kPost;
        const bool two = k == 2 && pull && left > last_single;
        hipError_t e = two ? launch_step2(c->prec, c->coll, c->higher_unit, c->two_step_form,
                                          c->f[src], c->f[dst], c->G, c->Kd, c->Kf, c->stream)
                           : launch_step(c->prec, c->coll, pull, c->higher_unit, c->f[src],
                                         c->f[dst], c->G, c->Kd, c->Kf, c->stream);
        if (e != hipSuccess)
            return fail_ctx(c, LBM_E_DEVICE, "step kernel launch failed: %s", hipGetErrorString(e));
        c->form[dst] = kPost;
        c->cur = dst;
        c->prev_valid = two ? 0 : 1;
        c->steps += two ? 2 : 1;
        left -= two ? 2 : 1;
    }
    return LBM_OK;
}

extern "C" int lbm_set_steps_per_launch(lbm_ctx *c, int k) {
    if (!c) return fail_ctx(nullptr, LBM_E_INVAL, "ctx is NULL");
    if (k < 0 || k > 2) return fail_ctx(c, LBM_E_INVAL, "steps per launch must be 0, 1 or 2");
    c->steps_per_launch = k;
    return LBM_OK;
}

extern "C" int lbm_steps_per_launch(const lbm_ctx *c) {
    if (!c) return LBM_E_INVAL;
    return steps_per_launch(c);
}

extern "C" int lbm_set_two_step_form(lbm_ctx *c, int form) {
    if (!c) return fail_ctx(nullptr, LBM_E_INVAL, "ctx is NULL");
    if (form != kFormAuto && form != kFormRegister && form != kFormStaged)
        return fail_ctx(c, LBM_E_INVAL, "two-step form must be 0, 1 or 2");
    if (form == kFormStaged && c->prec != kFP32Dev)
        return fail_ctx(c, LBM_E_INVAL, "the staged two-step form needs LBM_FP32_DEV");
    c->two_step_form = form;
    return LBM_OK;
}

extern "C" int lbm_two_step_form(const lbm_ctx *c) {
    if (!c) return LBM_E_INVAL;
    return two_step_form(c->prec, c->two_step_form, c->G);
}

extern "C" int lbm_stream_copy(void *dst, const void *src, size_t bytes, int workgroups,
                               void *stream) {
    if (!dst || !src) return fail_ctx(nullptr, LBM_E_INVAL, "NULL buffer");
    if (bytes % 16 || reinterpret_cast<uintptr_t>(dst) % 16 || reinterpret_cast<uintptr_t>(src) % 16)
        return fail_ctx(nullptr, LBM_E_INVAL, "buffers and size must be multiples of 16 bytes");
    if (workgroups < 0) return fail_ctx(nullptr, LBM_E_INVAL, "workgroups must be >= 0");
    hipError_t e = launch_stream_copy(dst, src, static_cast<long long>(bytes / 16), workgroups,
                                      static_cast<hipStream_t>(stream));
    if (e != hipSuccess)
        return fail_ctx(nullptr, LBM_E_DEVICE, "copy kernel launch failed: %s", hipGetErrorString(e));
    return LBM_OK;
}

extern "C" int lbm_moments(lbm_ctx *c, double *rho, double *ux, double *uy) {
    if (!c) return fail_ctx(nullptr, LBM_E_INVAL, "ctx is NULL");
    const size_t n = static_cast<size_t>(c->nx) * c->ny;
    int rc = ensure_stage(c, 3 * n * sizeof(double));
    if (rc != LBM_OK) return rc;
    double *d = c->d_stage;
    HIP_OR_FAIL(c, launch_moments(c->prec, c->form[c->cur] == kPost, c->f[c->cur], d, d + n,
                                  d + 2 * n, c->G, c->Kd, c->Kf, c->H, c->stream));
    double *h[3] = {rho, ux, uy};
    for (int i = 0; i < 3; ++i)
        if (h[i])
            HIP_OR_FAIL(c, hipMemcpyAsync(h[i], d + i * n, n * sizeof(double),
                                          hipMemcpyDeviceToHost, c->stream));
    HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
    return LBM_OK;
}

extern "C" int lbm_stress(lbm_ctx *c, double *sxx, double *syy, double *sxy) {
    if (!c) return fail_ctx(nullptr, LBM_E_INVAL, "ctx is NULL");
    const size_t n = static_cast<size_t>(c->nx) * c->ny;
    int rc = ensure_stage(c, 4 * n * sizeof(double));
    if (rc != LBM_OK) return rc;
    double *d = c->d_stage;  // rho, then the three stress fields
    const bool pull = c->form[c->cur] == kPost;
    HIP_OR_FAIL(c, launch_moments(c->prec, pull, c->f[c->cur], d, d + n, d + 2 * n, c->G, c->Kd,
                                  c->Kf, c->H, c->stream));
    HIP_OR_FAIL(c, launch_stress(c->prec, pull, c->f[c->cur], d, d + n, d + 2 * n, d + 3 * n,
                                 c->G, c->Kd, c->H, c->stream));
    double *h[3] = {sxx, syy, sxy};
    for (int i = 0; i < 3; ++i)
        if (h[i])
            HIP_OR_FAIL(c, hipMemcpyAsync(h[i], d + (i + 1) * n, n * sizeof(double),
                                          hipMemcpyDeviceToHost, c->stream));
    HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
    return LBM_OK;
}

static int fetch_result(lbm_ctx *c, double out[4]) {
    HIP_OR_FAIL(c, hipMemcpyAsync(out, c->d_partials + kResults, 4 * sizeof(double),
                                  hipMemcpyDeviceToHost, c->stream));
    HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
    return LBM_OK;
}

extern "C" int lbm_sums(lbm_ctx *c, double out[3]) {
    if (!c || !out) return fail_ctx(c, LBM_E_INVAL, "NULL argument");
    HIP_OR_FAIL(c, launch_sums(c->prec, c->form[c->cur] == kPost, c->f[c->cur], c->d_partials,
                               c->d_partials + kResults, c->G, c->Kd, c->Kf, c->H,
                               c->stream));
    double r[4];
    int rc = fetch_result(c, r);
    if (rc != LBM_OK) return rc;
    out[0] = r[0];
    out[1] = r[1];
    out[2] = r[2];
    if (r[3] != 0.0 || !isfinite(r[0]) || !isfinite(r[1]) || !isfinite(r[2]))
        return fail_ctx(c, LBM_E_UNSTABLE, "non-finite density or velocity");
    return LBM_OK;
}

extern "C" int lbm_residual(lbm_ctx *c, double *R) {
    if (!c || !R) return fail_ctx(c, LBM_E_INVAL, "NULL argument");
    if (!c->prev_valid || c->form[1 - c->cur] == kEmpty)
        return fail_ctx(c, LBM_E_STATE, "the state one step before the current one is not held");
    const int p = 1 - c->cur;
    HIP_OR_FAIL(c, launch_residual(c->prec, c->form[c->cur] == kPost, c->f[c->cur],
                                   c->form[p] == kPost, c->f[p], c->d_partials,
                                   c->d_partials + kResults, c->G, c->Kd, c->Kf, c->H,
                                   c->stream));
    double r[4];
    int rc = fetch_result(c, r);
    if (rc != LBM_OK) return rc;
    if (r[3] != 0.0 || !isfinite(r[0]) || !isfinite(r[1])) {
        *R = NAN;
        return fail_ctx(c, LBM_E_UNSTABLE, "non-finite velocity");
    }
    *R = r[1] > 0.0 ? sqrt(r[0]) / sqrt(r[1]) : (r[0] > 0.0 ? INFINITY : 0.0);
    return LBM_OK;
}

// Residual and sums of one time level without a host wait: one pass over the
// two buffers writes both results (eight values) behind the partials, and
// one copy takes them to pinned host memory.  Everything runs in stream
// order, so a later check or a synchronous lbm_residual / lbm_sums reusing
// the partials cannot overtake it.
extern "C" int lbm_check_async(lbm_ctx *c) {
    if (!c) return fail_ctx(nullptr, LBM_E_INVAL, "ctx is NULL");
    if (!c->prev_valid || c->form[1 - c->cur] == kEmpty)
        return fail_ctx(c, LBM_E_STATE, "the state one step before the current one is not held");
    if (!c->h_check) {
        void *h = nullptr;
        if (hipHostMalloc(&h, 8 * sizeof(double)) != hipSuccess || !h)
            return fail_ctx(c, LBM_E_NOMEM, "pinned host buffer for the check");
        hipEvent_t ev;
        if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
            (void)hipHostFree(h);
            return fail_ctx(c, LBM_E_DEVICE, "hipEventCreateWithFlags failed");
        }
        c->h_check = static_cast<double *>(h);
        c->check_ev = ev;
    }
    const int p = 1 - c->cur;
    double *res = c->d_partials + kResults;
    c->check_step = -1;  // nothing to read if an enqueue below fails
    HIP_OR_FAIL(c, launch_check(c->prec, c->form[c->cur] == kPost, c->f[c->cur],
                                c->form[p] == kPost, c->f[p], c->d_partials, res, c->G, c->Kd,
                                c->Kf, c->H, c->stream));
    HIP_OR_FAIL(c, hipMemcpyAsync(c->h_check, res, 8 * sizeof(double), hipMemcpyDeviceToHost,
                                  c->stream));
    HIP_OR_FAIL(c, hipEventRecord(c->check_ev, c->stream));
    c->check_step = c->steps;
    return LBM_OK;
}

// lbm_check_async's reductions with the partial sums in the static scratch
// of this GPU and the eight results written to the caller's device memory:
// no allocation of any kind, no host wait.  Every partial the finalize pass
// reads is written by the same call, so nothing in the scratch needs
// clearing first.
extern "C" int lbm_check_into(lbm_ctx *c, double *out) {
    if (!c) return fail_ctx(nullptr, LBM_E_INVAL, "ctx is NULL");
    if (!out) return fail_ctx(c, LBM_E_INVAL, "out is NULL");
    if (!c->prev_valid || c->form[1 - c->cur] == kEmpty)
        return fail_ctx(c, LBM_E_STATE, "the state one step before the current one is not held");
    const size_t need = 8 * static_cast<size_t>(reduce_partials(c->G));
    if (need > kScratchDoubles)
        return fail_ctx(c, LBM_E_INVAL, "the check needs %zu scratch values, the maximum is %zu",
                        need, kScratchDoubles);
    const int p = 1 - c->cur;
    HIP_OR_FAIL(c, launch_check(c->prec, c->form[c->cur] == kPost, c->f[c->cur],
                                c->form[p] == kPost, c->f[p], c->scratch, out, c->G, c->Kd,
                                c->Kf, c->H, c->stream));
    return LBM_OK;
}

extern "C" int lbm_check_result(lbm_ctx *c, double *R, double sums[3], long *step) {
    if (!c) return fail_ctx(nullptr, LBM_E_INVAL, "ctx is NULL");
    if (c->check_step < 0) return fail_ctx(c, LBM_E_STATE, "no check enqueued");
    HIP_OR_FAIL(c, hipEventSynchronize(c->check_ev));
    const double *r = c->h_check;
    if (step) *step = c->check_step;
    if (sums)
        for (int i = 0; i < 3; ++i) sums[i] = r[4 + i];
    const bool bad = r[3] != 0.0 || r[7] != 0.0 || !isfinite(r[0]) || !isfinite(r[1]) ||
                     !isfinite(r[4]) || !isfinite(r[5]) || !isfinite(r[6]);
    if (R) *R = bad ? NAN : (r[1] > 0.0 ? sqrt(r[0]) / sqrt(r[1]) : (r[0] > 0.0 ? INFINITY : 0.0));
    if (bad)
        return fail_ctx(c, LBM_E_UNSTABLE, "non-finite density or velocity at step %ld",
                        c->check_step);
    return LBM_OK;
}

extern "C" int lbm_get_populations(lbm_ctx *c, double *f) {
    if (!c || !f) return fail_ctx(c, LBM_E_INVAL, "NULL argument");
    const size_t n9 = static_cast<size_t>(9) * c->nx * c->ny;
    int rc = ensure_stage(c, n9 * sizeof(double));
    if (rc != LBM_OK) return rc;
    HIP_OR_FAIL(c, launch_get_populations(c->prec, c->form[c->cur] == kPost, c->f[c->cur],
                                          c->d_stage, c->G, c->Kd, c->Kf, c->H, c->stream));
    HIP_OR_FAIL(c, hipMemcpyAsync(f, c->d_stage, n9 * sizeof(double), hipMemcpyDeviceToHost,
                                  c->stream));
    HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
    return LBM_OK;
}

extern "C" int lbm_set_populations(lbm_ctx *c, const double *f) {
    if (!c || !f) return fail_ctx(c, LBM_E_INVAL, "NULL argument");
    const size_t n9 = static_cast<size_t>(9) * c->nx * c->ny;
    int rc = ensure_stage(c, n9 * sizeof(double));
    if (rc != LBM_OK) return rc;
    HIP_OR_FAIL(c, hipMemcpyAsync(c->d_stage, f, n9 * sizeof(double), hipMemcpyHostToDevice,
                                  c->stream));
    HIP_OR_FAIL(c, launch_set_populations(c->prec, c->f[c->cur], c->d_stage, c->G, c->H,
                                          c->stream));
    c->form[c->cur] = kPre;
    c->form[1 - c->cur] = kEmpty;
    c->prev_valid = 0;
    HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
    return LBM_OK;
}

extern "C" int lbm_set_mask(lbm_ctx *c, const unsigned char *mask) {
    if (!c) return fail_ctx(nullptr, LBM_E_INVAL, "ctx is NULL");
    HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
    if (!mask) {
        if (c->d_mask) HIP_OR_FAIL(c, hipFree(c->d_mask));
        if (c->d_tile_solid) HIP_OR_FAIL(c, hipFree(c->d_tile_solid));
        c->d_mask = nullptr;
        c->d_tile_solid = nullptr;
        c->G.mask = nullptr;
        c->G.tile_solid = nullptr;
        return LBM_OK;
    }
    const Geometry &G = c->G;
    const size_t mbytes = static_cast<size_t>(G.pitch) * G.ny;
    if (!c->d_mask) HIP_OR_FAIL(c, hipMalloc(&c->d_mask, mbytes));
    if (!c->d_tile_solid) HIP_OR_FAIL(c, hipMalloc(&c->d_tile_solid, G.ntile));
    unsigned char *pitched = static_cast<unsigned char *>(calloc(mbytes, 1));
    unsigned char *flags = static_cast<unsigned char *>(calloc(G.ntile, 1));
    if (!pitched || !flags) {
        free(pitched);
        free(flags);
        return fail_ctx(c, LBM_E_NOMEM, "out of host memory");
    }
    for (int j = 0; j < G.ny; ++j)
        for (int i = 0; i < G.nx; ++i)
            pitched[static_cast<size_t>(j) * G.pitch + i] = mask[static_cast<size_t>(j) * G.nx + i] ? 1 : 0;
    for (int t = 0; t < G.ntile; ++t)
        flags[t] = static_cast<unsigned char>(tile_has_solid(G, mask, t % G.nseg, t / G.nseg));
    hipError_t e1 = hipMemcpy(c->d_mask, pitched, mbytes, hipMemcpyHostToDevice);
    hipError_t e2 = hipMemcpy(c->d_tile_solid, flags, G.ntile, hipMemcpyHostToDevice);
    free(pitched);
    free(flags);
    HIP_OR_FAIL(c, e1);
    HIP_OR_FAIL(c, e2);
    c->G.mask = c->d_mask;
    c->G.tile_solid = c->d_tile_solid;
    return LBM_OK;
}

static void apply_force(lbm_ctx *c, double fx, double fy) {
    c->opts.force[0] = fx;
    c->opts.force[1] = fy;
    c->Kd.Fx = fx;
    c->Kd.Fy = fy;
    c->Kd.hFx = 0.5 * fx;
    c->Kd.hFy = 0.5 * fy;
    c->Kf.Fx = static_cast<float>(fx);
    c->Kf.Fy = static_cast<float>(fy);
    c->Kf.hFx = static_cast<float>(0.5 * fx);
    c->Kf.hFy = static_cast<float>(0.5 * fy);
    c->H.Fx = fx;
    c->H.Fy = fy;
}

extern "C" int lbm_set_force(lbm_ctx *c, double fx, double fy) {
    if (!c) return fail_ctx(nullptr, LBM_E_INVAL, "ctx is NULL");
    if (!isfinite(fx) || !isfinite(fy)) return fail_ctx(c, LBM_E_INVAL, "force must be finite");
    apply_force(c, fx, fy);
    return LBM_OK;
}

extern "C" int lbm_step_forced(lbm_ctx *c, long n, const double *fx, const double *fy) {
    if (!c) return fail_ctx(nullptr, LBM_E_INVAL, "ctx is NULL");
    if (n < 0 || (n > 0 && !fx)) return fail_ctx(c, LBM_E_INVAL, "need n >= 0 and fx");
    for (long i = 0; i < n; ++i)
        if (!isfinite(fx[i]) || (fy && !isfinite(fy[i])))
            return fail_ctx(c, LBM_E_INVAL, "force %ld is not finite", i);
    for (long i = 0; i < n; ++i) {
        apply_force(c, fx[i], fy ? fy[i] : c->opts.force[1]);
        int rc = lbm_step(c, 1);  // the constants travel by value with each launch
        if (rc != LBM_OK) return rc;
    }
    return LBM_OK;
}

extern "C" int lbm_smooth_step(lbm_ctx *c) {
    if (!c) return fail_ctx(nullptr, LBM_E_INVAL, "ctx is NULL");
    int rc = lbm_step(c, 1);
    if (rc != LBM_OK) return rc;
    const size_t n9 = static_cast<size_t>(9) * c->nx * c->ny;
    rc = ensure_stage(c, n9 * sizeof(double));
    if (rc != LBM_OK) return rc;
    const int p = 1 - c->cur;
    HIP_OR_FAIL(c, launch_average_states(c->prec, c->form[c->cur] == kPost, c->f[c->cur],
                                         c->form[p] == kPost, c->f[p], c->d_stage, c->G, c->Kd,
                                         c->H, c->stream));
    HIP_OR_FAIL(c, launch_set_populations(c->prec, c->f[c->cur], c->d_stage, c->G, c->H,
                                          c->stream));
    c->form[c->cur] = kPre;
    c->form[p] = kEmpty;
    c->prev_valid = 0;
    HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
    return LBM_OK;
}

extern "C" int lbm_set_rates(lbm_ctx *c, const double rates[9]) {
    if (!c) return fail_ctx(nullptr, LBM_E_INVAL, "ctx is NULL");
    if (!rates) return fail_ctx(c, LBM_E_INVAL, "rates is NULL");
    for (int j = 0; j < 9; ++j)
        if (!(rates[j] > 0.0 && rates[j] < 2.0))
            return fail_ctx(c, LBM_E_INVAL, "rates[%d] = %g is not in (0, 2)", j, rates[j]);
    HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
    memcpy(c->rates, rates, sizeof(c->rates));
    c->higher_unit = rates[6] == 1.0 && rates[7] == 1.0 && rates[8] == 1.0;
    CaseSpec spec;
    make_spec(c->nx, c->ny, c->a, c->rates, &c->bc, &c->opts, spec);
    fill_consts(spec, c->Kd);
    fill_consts(spec, c->Kf);
    return LBM_OK;
}

extern "C" long lbm_steps_done(const lbm_ctx *c) { return c ? c->steps : 0; }

extern "C" int lbm_launch_shape(const lbm_ctx *c, int *rows_per_wave, int *workgroups) {
    if (!c) return LBM_E_INVAL;
    const bool tile = uses_tile_kernel(c->G);
    if (rows_per_wave) *rows_per_wave = tile ? c->G.tile_rows : c->G.rows;
    if (workgroups) *workgroups = tile ? tile_workgroups(c->G) : c->G.nblocks;
    return LBM_OK;
}

extern "C" const char *lbm_last_error(const lbm_ctx *c) { return c ? c->err : g_create_error; }

extern "C" int lbm_destroy(lbm_ctx *c) {
    if (!c) return LBM_OK;
    if (c->stream || c->f[0]) (void)hipStreamSynchronize(c->stream);
    for (int i = 0; i < 2; ++i)
        if (c->owns[i] && c->f[i]) (void)hipFree(c->f[i]);
    if (c->d_partials) (void)hipFree(c->d_partials);
    if (c->h_check) (void)hipHostFree(c->h_check);
    if (c->check_ev) (void)hipEventDestroy(c->check_ev);
    if (c->d_stage) (void)hipFree(c->d_stage);
    if (c->d_mask) (void)hipFree(c->d_mask);
    if (c->d_tile_solid) (void)hipFree(c->d_tile_solid);
    delete c;
    return LBM_OK;
}
