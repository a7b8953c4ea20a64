// Host side of the batch ABI declared in include/lbm_batch.h: per-case
// tables, the tile list of the active cases, graph capture of runs of steps,
// batched residuals and the launch-shape autotuner.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "../../include/lbm_batch.h"
#include "lbm_internal.h"

using namespace lbm;

namespace {

thread_local char g_batch_error[512] = "no error";

enum Form { kEmpty = 0, kPre = 1, kPost = 2 };

}  // namespace

struct lbm_batch {
    int n;
    lbm_batch_opts opts;
    int prec, coll;
    bool higher_unit;           // omega_6..8 == 1 for every case
    hipStream_t stream;
    bool own_stream;
    std::vector<CaseSpec> spec;
    std::vector<Geometry> G;
    std::vector<Consts<double>> Kd;
    std::vector<Consts<float>> Kf;
    std::vector<HostSide> H;
    std::vector<BatchCase> bc;  // host mirror of the device case table
    std::vector<int> form_prev; // Form of each case's other buffer
    std::vector<int> active;
    std::vector<long> steps;
    std::vector<std::vector<unsigned char>> hmask;  // host obstacle masks [ny][nx] (empty: none)
    std::vector<unsigned char *> d_mask;            // device copies [ny][pitch]
    size_t vbytes;              // bytes per stored value
    size_t total_values;        // values per ping-pong buffer
    void *buf[2];
    // device tables
    BatchCase *d_cases;
    Geometry *d_geoms;
    Consts<double> *d_Kd;
    Consts<float> *d_Kf;
    HostSide *d_H;
    BatchTile *d_tiles;
    int *d_ntiles;
    int tile_cap;
    int ntiles;
    bool tiles_dirty;           // the tile list must be rebuilt before the next launch
    BatchRed *d_items;
    int item_cap;
    int *d_case_first, *d_case_count;
    double *d_partials;
    double *d_out;
    double *d_stage;
    size_t stage_bytes;
    // launch shape
    bool tile_pref;             // the tile kernel is wanted (option or autotuner)
    bool tile_mode;             // the batched tile kernel runs (64 x kBatchTileRows block
                                // tiles): tile_pref and no case has a mask
    int rows;
    int workgroups;
    int graph_steps;
    hipGraphExec_t graph;
    bool graph_ok;
    // two steps per launch (lbm_batch_opts.steps_per_launch != 1, no mask)
    int spl_opt;                // 0 automatic, 1, 2
    int form2;                  // kFormRegister (64 x 8 block tiles) or kFormStaged (64 x 24)
    int workgroups2;            // persistent grid of the two-step kernel
    BatchTile *d_tiles24;       // 64 x kBatchStagedRows block tiles of the active cases
    int *d_ntiles24;
    int tile24_cap;
    int ntiles24;
    hipGraphExec_t graph2;      // captured runs of two-step launches
    bool graph2_ok;
    char err[512];
};

static int fail(lbm_batch *b, int code, const char *fmt, ...) {
    char *buf = b ? b->err : g_batch_error;
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, 512, fmt, ap);
    va_end(ap);
    return code;
}

#define HIP_OK(b, call)                                                                  \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess)                                                            \
            return fail((b), e_ == hipErrorOutOfMemory ? LBM_E_NOMEM : LBM_E_DEVICE,     \
                        "%s failed: %s", #call, hipGetErrorString(e_));                 \
    } while (0)

extern "C" void lbm_batch_default_opts(lbm_batch_opts *o) {
    if (!o) return;
    memset(o, 0, sizeof(*o));
    o->collision = LBM_RC;
    o->precision = LBM_FP64;
    o->corrections = 1;
}

static int auto_workgroups(int ntiles) {
    // enough resident waves to cover the HBM latency (256 CUs, 4 waves per
    // workgroup), but no more workgroups than there are tiles to share
    int wgs = 256 * 8;
    const int need = (ntiles + kWavesPerBlock - 1) / kWavesPerBlock;
    if (need < wgs) wgs = need;
    return wgs < 1 ? 1 : wgs;
}

static bool any_mask(const lbm_batch *b) {
    for (int c = 0; c < b->n; ++c)
        if (!b->hmask[c].empty()) return true;
    return false;
}

// Two steps per launch apply while no case has a mask; they run on the block
// tiles of the tile kernel, which then also takes the single steps.
static bool two_step_on(const lbm_batch *b) { return b->spl_opt != 1 && !any_mask(b); }

static bool tile_mode_wanted(const lbm_batch *b) {
    return (b->tile_pref || b->spl_opt != 1) && !any_mask(b);
}

// two-step launches per captured graph: half the graph's steps, kept even so
// that a replay leaves every case's current buffer where it was
static int graph_pairs(const lbm_batch *b) {
    const int p = (b->graph_steps / 2) & ~1;
    return p < 2 ? 2 : p;
}

// block tiles of the batched tile kernel for one case
static int block_tiles(const Geometry &G) {
    return G.nseg * ((G.ny + kBatchTileRows - 1) / kBatchTileRows);
}

// block tiles of the batched staged two-step kernel for one case
static int staged_tiles(const Geometry &G) {
    return G.nseg * ((G.ny + kBatchStagedRows - 1) / kBatchStagedRows);
}

// Tile list of the active cases, uploaded with its count: block tiles in tile
// mode, wavefront tiles of the march otherwise.  A mask on any case ends tile
// mode (its generic loads would be slower than the march's near-solid tiles).
static int upload_tiles(lbm_batch *b) {
    const bool mode = tile_mode_wanted(b);
    if (mode != b->tile_mode) {
        b->tile_mode = mode;
        b->graph_ok = false;  // the captured steps launch the other kernel
        b->graph2_ok = false;
    }
    std::vector<BatchTile> t;
    t.reserve(b->tile_cap);
    for (int c = 0; c < b->n; ++c) {
        if (!b->active[c]) continue;
        const Geometry &G = b->G[c];
        if (b->tile_mode) {
            const int nty = (G.ny + kBatchTileRows - 1) / kBatchTileRows;
            for (int ty = 0; ty < nty; ++ty)
                for (int tx = 0; tx < G.nseg; ++tx) t.push_back(BatchTile{c, tx, ty, 0});
            continue;
        }
        const unsigned char *m = b->hmask[c].empty() ? nullptr : b->hmask[c].data();
        for (int ch = 0; ch < G.nchunk; ++ch)
            for (int s = 0; s < G.nseg; ++s)
                t.push_back(BatchTile{c, s, ch, tile_has_solid(G, m, s, ch)});
    }
    b->ntiles = static_cast<int>(t.size());
    if (b->ntiles > b->tile_cap) return fail(b, LBM_E_DEVICE, "tile list overflow");
    if (b->ntiles)
        HIP_OK(b, hipMemcpyAsync(b->d_tiles, t.data(), t.size() * sizeof(BatchTile),
                                 hipMemcpyHostToDevice, b->stream));
    HIP_OK(b, hipMemcpyAsync(b->d_ntiles, &b->ntiles, sizeof(int), hipMemcpyHostToDevice,
                             b->stream));
    // the staged two-step form's own list of taller block tiles
    std::vector<BatchTile> t24;
    if (b->tile_mode && b->d_tiles24) {
        t24.reserve(b->tile24_cap);
        for (int c = 0; c < b->n; ++c) {
            if (!b->active[c]) continue;
            const Geometry &G = b->G[c];
            const int nty = (G.ny + kBatchStagedRows - 1) / kBatchStagedRows;
            for (int ty = 0; ty < nty; ++ty)
                for (int tx = 0; tx < G.nseg; ++tx) t24.push_back(BatchTile{c, tx, ty, 0});
        }
        b->ntiles24 = static_cast<int>(t24.size());
        if (b->ntiles24 > b->tile24_cap) return fail(b, LBM_E_DEVICE, "tile list overflow");
        if (b->ntiles24)
            HIP_OK(b, hipMemcpyAsync(b->d_tiles24, t24.data(), t24.size() * sizeof(BatchTile),
                                     hipMemcpyHostToDevice, b->stream));
        HIP_OK(b, hipMemcpyAsync(b->d_ntiles24, &b->ntiles24, sizeof(int),
                                 hipMemcpyHostToDevice, b->stream));
    }
    // the host vector and count must outlive the copies
    HIP_OK(b, hipStreamSynchronize(b->stream));
    return LBM_OK;
}

static int ensure_tiles(lbm_batch *b) {
    if (!b->tiles_dirty) return LBM_OK;
    int rc = upload_tiles(b);
    if (rc == LBM_OK) b->tiles_dirty = false;
    return rc;
}

static int upload_cases(lbm_batch *b) {
    HIP_OK(b, hipMemcpyAsync(b->d_cases, b->bc.data(), b->n * sizeof(BatchCase),
                             hipMemcpyHostToDevice, b->stream));
    HIP_OK(b, hipStreamSynchronize(b->stream));
    return LBM_OK;
}

// Rows per wavefront for every case (tile counts follow) and the tables.
static int apply_rows(lbm_batch *b, int rows) {
    b->rows = rows;
    int cap = 0;
    for (int c = 0; c < b->n; ++c) {
        set_rows(b->G[c], rows);
        cap += std::max(b->G[c].ntile, block_tiles(b->G[c]));
    }
    if (cap > b->tile_cap) {
        if (b->d_tiles) HIP_OK(b, hipFree(b->d_tiles));
        b->d_tiles = nullptr;
        HIP_OK(b, hipMalloc(&b->d_tiles, static_cast<size_t>(cap) * sizeof(BatchTile)));
        b->tile_cap = cap;
    }
    HIP_OK(b, hipMemcpyAsync(b->d_geoms, b->G.data(), b->n * sizeof(Geometry),
                             hipMemcpyHostToDevice, b->stream));
    b->graph_ok = false;
    b->graph2_ok = false;
    int rc = upload_tiles(b);
    if (rc == LBM_OK) b->tiles_dirty = false;
    return rc;
}

static hipError_t launch(lbm_batch *b, int flip, int force_pull, int wgs) {
    if (b->tile_mode)
        return launch_batch_tile(b->prec, b->coll, b->higher_unit, b->buf[0], b->buf[1],
                                 b->d_tiles, b->d_ntiles, b->d_cases, b->d_geoms, b->d_Kd,
                                 b->d_Kf, flip, force_pull, wgs, b->stream);
    return launch_batch_step(b->prec, b->coll, b->higher_unit, b->buf[0], b->buf[1], b->d_tiles,
                             b->d_ntiles, b->d_cases, b->d_geoms, b->d_Kd, b->d_Kf, flip,
                             force_pull, wgs, b->stream);
}

static hipError_t launch2_form(lbm_batch *b, int form, int flip, int wgs) {
    if (form == kFormStaged)
        return launch_batch_staged(b->prec, b->coll, b->higher_unit, b->buf[0], b->buf[1],
                                   b->d_tiles24, b->d_ntiles24, b->d_cases, b->d_geoms, b->d_Kf,
                                   flip, wgs, b->stream);
    return launch_batch_tile2(b->prec, b->coll, b->higher_unit, b->buf[0], b->buf[1], b->d_tiles,
                              b->d_ntiles, b->d_cases, b->d_geoms, b->d_Kd, b->d_Kf, flip, wgs,
                              b->stream);
}

static hipError_t launch2(lbm_batch *b, int flip, int wgs) {
    return launch2_form(b, b->form2, flip, wgs);
}

static int ensure_graph2(lbm_batch *b) {
    if (b->graph2_ok) return LBM_OK;
    if (b->graph2) {
        HIP_OK(b, hipGraphExecDestroy(b->graph2));
        b->graph2 = nullptr;
    }
    HIP_OK(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    hipError_t le = hipSuccess;
    for (int i = 0; i < graph_pairs(b) && le == hipSuccess; ++i) le = launch2(b, i & 1, b->workgroups2);
    hipGraph_t g = nullptr;
    hipError_t ee = hipStreamEndCapture(b->stream, &g);
    if (le != hipSuccess || ee != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return fail(b, LBM_E_DEVICE, "graph capture failed: %s",
                    hipGetErrorString(le != hipSuccess ? le : ee));
    }
    hipError_t ie = hipGraphInstantiate(&b->graph2, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ie != hipSuccess) {
        b->graph2 = nullptr;
        return fail(b, LBM_E_DEVICE, "graph instantiation failed: %s", hipGetErrorString(ie));
    }
    b->graph2_ok = true;
    return LBM_OK;
}

static int ensure_graph(lbm_batch *b) {
    if (b->graph_ok) return LBM_OK;
    if (b->graph) {
        HIP_OK(b, hipGraphExecDestroy(b->graph));
        b->graph = nullptr;
    }
    HIP_OK(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    hipError_t le = hipSuccess;
    for (int i = 0; i < b->graph_steps && le == hipSuccess; ++i) le = launch(b, i & 1, 1, b->workgroups);
    hipGraph_t g = nullptr;
    hipError_t ee = hipStreamEndCapture(b->stream, &g);
    if (le != hipSuccess || ee != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return fail(b, LBM_E_DEVICE, "graph capture failed: %s",
                    hipGetErrorString(le != hipSuccess ? le : ee));
    }
    hipError_t ie = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ie != hipSuccess) {
        b->graph = nullptr;
        return fail(b, LBM_E_DEVICE, "graph instantiation failed: %s", hipGetErrorString(ie));
    }
    b->graph_ok = true;
    return LBM_OK;
}

static int ensure_stage(lbm_batch *b, size_t bytes) {
    if (b->stage_bytes >= bytes) return LBM_OK;
    if (b->d_stage) {
        HIP_OK(b, hipStreamSynchronize(b->stream));
        HIP_OK(b, hipFree(b->d_stage));
        b->d_stage = nullptr;
        b->stage_bytes = 0;
    }
    HIP_OK(b, hipMalloc(&b->d_stage, bytes));
    b->stage_bytes = bytes;
    return LBM_OK;
}

static void *case_ptr(lbm_batch *b, int c, int which) {
    return static_cast<char *>(b->buf[which]) + b->bc[c].off * b->vbytes;
}

extern "C" int lbm_batch_destroy(lbm_batch *b) {
    if (!b) return LBM_OK;
    if (b->stream || b->own_stream) (void)hipStreamSynchronize(b->stream);
    if (b->graph) (void)hipGraphExecDestroy(b->graph);
    if (b->graph2) (void)hipGraphExecDestroy(b->graph2);
    void *ptrs[] = {b->buf[0], b->buf[1], b->d_cases, b->d_geoms, b->d_Kd, b->d_Kf, b->d_H,
                    b->d_tiles, b->d_ntiles, b->d_items, b->d_case_first, b->d_case_count,
                    b->d_partials, b->d_out, b->d_stage, b->d_tiles24, b->d_ntiles24};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    for (unsigned char *p : b->d_mask)
        if (p) (void)hipFree(p);
    if (b->own_stream) (void)hipStreamDestroy(b->stream);
    delete b;
    return LBM_OK;
}

extern "C" int lbm_batch_create(int ncases, const lbm_case *cases, const lbm_batch_opts *opts,
                                lbm_batch **out) {
    if (!out) return fail(nullptr, LBM_E_INVAL, "out is NULL");
    *out = nullptr;
    if (ncases < 1 || !cases) return fail(nullptr, LBM_E_INVAL, "need ncases >= 1 and cases");
    lbm_batch_opts o;
    if (opts) o = *opts; else lbm_batch_default_opts(&o);
    if (o.collision != LBM_RC && o.collision != LBM_RNR)
        return fail(nullptr, LBM_E_INVAL, "unknown collision %d", o.collision);
    if (o.precision < LBM_FP64 || o.precision > LBM_FP32_DEV_F64)
        return fail(nullptr, LBM_E_INVAL, "unknown precision %d", o.precision);
    if (o.rows_per_wave < 0 || o.rows_per_wave > kMaxRows)
        return fail(nullptr, LBM_E_INVAL, "rows_per_wave must be in [0, %d]", kMaxRows);
    if (o.workgroups < 0) return fail(nullptr, LBM_E_INVAL, "workgroups must be >= 0");
    if (o.graph_steps == 0) o.graph_steps = 64;
    if (o.graph_steps < 2 || (o.graph_steps & 1))
        return fail(nullptr, LBM_E_INVAL, "graph_steps must be even and >= 2");
    if (o.steps_per_launch < 0 || o.steps_per_launch > 2)
        return fail(nullptr, LBM_E_INVAL, "steps_per_launch must be 0, 1 or 2");
    if (o.two_step_form < 0 || o.two_step_form > 2)
        return fail(nullptr, LBM_E_INVAL, "two_step_form must be 0, 1 or 2");
    if (o.two_step_form == kFormStaged && o.precision != LBM_FP32_DEV)
        return fail(nullptr, LBM_E_INVAL, "the staged two-step form needs LBM_FP32_DEV");
    lbm_batch *b = new (std::nothrow) lbm_batch();
    if (!b) return fail(nullptr, LBM_E_NOMEM, "out of host memory");
    b->n = ncases;
    b->opts = o;
    b->prec = o.precision;
    b->coll = o.collision;
    b->graph_steps = o.graph_steps;
    b->spl_opt = o.steps_per_launch;
    // automatic: the staged form for FP32 storage and arithmetic
    b->form2 = o.two_step_form != kFormAuto ? o.two_step_form
                                            : (o.precision == LBM_FP32_DEV ? kFormStaged : kFormRegister);
    b->vbytes = f32_storage(o.precision) ? sizeof(float) : sizeof(double);
    snprintf(b->err, sizeof(b->err), "no error");
    try {
        b->spec.resize(ncases);
        b->G.resize(ncases);
        b->Kd.resize(ncases);
        b->Kf.resize(ncases);
        b->H.resize(ncases);
        b->bc.resize(ncases);
        b->form_prev.assign(ncases, kEmpty);
        b->active.assign(ncases, 1);
        b->steps.assign(ncases, 0);
        b->hmask.resize(ncases);
        b->d_mask.assign(ncases, nullptr);
    } catch (...) {
        delete b;
        return fail(nullptr, LBM_E_NOMEM, "out of host memory");
    }
    b->higher_unit = true;
    size_t total = 0;
    long long nodes = 0;
    for (int c = 0; c < ncases; ++c) {
        const lbm_case &k = cases[c];
        lbm_opts lo;
        lbm_default_opts(&lo);
        lo.cs2 = k.cs2 == 0.0 ? fmin(1.0 / 3.0, 0.64 * k.r * k.r) : k.cs2;
        lo.force[0] = k.force[0];
        lo.force[1] = k.force[1];
        lo.rho0 = k.rho0 == 0.0 ? 1.0 : k.rho0;
        lo.collision = o.collision;
        lo.precision = o.precision;
        lo.corrections = o.corrections;
        if (validate_case(k.nx, k.ny, k.r, k.rates, &k.bc, &lo) != LBM_OK) {
            char msg[512];
            snprintf(msg, sizeof(msg), "case %d: %s", c, create_error_text());
            delete b;
            return fail(nullptr, LBM_E_INVAL, "%s", msg);
        }
        size_t need = 0;
        if (lbm_required_bytes(k.nx, k.ny, o.precision, &need) != LBM_OK) {
            char msg[512];
            snprintf(msg, sizeof(msg), "case %d: %s", c, create_error_text());
            delete b;
            return fail(nullptr, LBM_E_INVAL, "%s", msg);
        }
        CaseSpec &sp = b->spec[c];
        make_spec(k.nx, k.ny, k.r, k.rates, &k.bc, &lo, sp);
        base_geometry(sp, need, b->G[c]);
        fill_consts(sp, b->Kd[c]);
        fill_consts(sp, b->Kf[c]);
        fill_host_side(sp, b->H[c]);
        if (!(k.rates[6] == 1.0 && k.rates[7] == 1.0 && k.rates[8] == 1.0)) b->higher_unit = false;
        b->bc[c].off = static_cast<long long>(total);
        b->bc[c].cur = 0;
        b->bc[c].pull = 0;
        // cases start on 256-byte boundaries
        const size_t vals = need / b->vbytes;
        const size_t align = 256 / b->vbytes;
        total += (vals + align - 1) / align * align;
        nodes += static_cast<long long>(k.nx) * k.ny;
    }
    b->total_values = total;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
        delete b;
        return fail(nullptr, LBM_E_DEVICE, "no usable GPU");
    }
    const bool nt = 2.0 * static_cast<double>(total * b->vbytes) > 512.0 * 1024 * 1024;
    for (int c = 0; c < ncases; ++c) b->G[c].nt_store = nt ? 1 : 0;

    int rc = LBM_OK;
    if (o.stream) {
        b->stream = static_cast<hipStream_t>(o.stream);
    } else {
        hipError_t e = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            delete b;
            return fail(nullptr, LBM_E_DEVICE, "hipStreamCreate failed: %s", hipGetErrorString(e));
        }
        b->own_stream = true;
    }
#define ALLOC(ptr, bytes)                                                                  \
    if (rc == LBM_OK) {                                                                    \
        hipError_t e_ = hipMalloc(reinterpret_cast<void **>(&(ptr)), (bytes));             \
        if (e_ != hipSuccess) {                                                            \
            (ptr) = nullptr;                                                               \
            rc = fail(nullptr, e_ == hipErrorOutOfMemory ? LBM_E_NOMEM : LBM_E_DEVICE,     \
                      "hipMalloc of %zu bytes failed: %s", static_cast<size_t>(bytes),     \
                      hipGetErrorString(e_));                                              \
        }                                                                                  \
    }
    ALLOC(b->buf[0], total * b->vbytes);
    ALLOC(b->buf[1], total * b->vbytes);
    ALLOC(b->d_cases, ncases * sizeof(BatchCase));
    ALLOC(b->d_geoms, ncases * sizeof(Geometry));
    ALLOC(b->d_Kd, ncases * sizeof(Consts<double>));
    ALLOC(b->d_Kf, ncases * sizeof(Consts<float>));
    ALLOC(b->d_H, ncases * sizeof(HostSide));
    ALLOC(b->d_ntiles, sizeof(int));
    if (o.precision == LBM_FP32_DEV) {
        int cap24 = 0;
        for (int c = 0; c < ncases; ++c) cap24 += staged_tiles(b->G[c]);
        b->tile24_cap = cap24;
        ALLOC(b->d_tiles24, static_cast<size_t>(cap24 > 0 ? cap24 : 1) * sizeof(BatchTile));
        ALLOC(b->d_ntiles24, sizeof(int));
    }
    ALLOC(b->d_case_first, ncases * sizeof(int));
    ALLOC(b->d_case_count, ncases * sizeof(int));
    ALLOC(b->d_out, ncases * 4 * sizeof(double));
#undef ALLOC
    if (rc != LBM_OK) {
        char msg[512];
        snprintf(msg, sizeof(msg), "%s", g_batch_error);
        lbm_batch_destroy(b);
        return fail(nullptr, rc, "%s", msg);
    }
    auto setup = [&]() -> int {
        HIP_OK(b, hipMemcpyAsync(b->d_Kd, b->Kd.data(), ncases * sizeof(Consts<double>),
                                 hipMemcpyHostToDevice, b->stream));
        HIP_OK(b, hipMemcpyAsync(b->d_Kf, b->Kf.data(), ncases * sizeof(Consts<float>),
                                 hipMemcpyHostToDevice, b->stream));
        HIP_OK(b, hipMemcpyAsync(b->d_H, b->H.data(), ncases * sizeof(HostSide),
                                 hipMemcpyHostToDevice, b->stream));
        int r = upload_cases(b);
        if (r != LBM_OK) return r;
        const int rows = o.rows_per_wave > 0 ? o.rows_per_wave : auto_rows(nodes, o.precision);
        b->tile_pref = o.tile_kernel == 1;
        r = apply_rows(b, rows);
        if (r != LBM_OK) return r;
        b->workgroups = o.workgroups > 0 ? o.workgroups : auto_workgroups(b->ntiles);
        // two-step grid: one block tile per workgroup (persistent beyond that)
        int nbt = 0;
        for (int c = 0; c < ncases; ++c)
            nbt += b->form2 == kFormStaged ? staged_tiles(b->G[c]) : block_tiles(b->G[c]);
        b->workgroups2 = o.workgroups > 0 ? o.workgroups : (nbt > 0 ? nbt : 1);
        for (int c = 0; c < ncases; ++c) {
            HIP_OK(b, launch_init_feq(b->prec, case_ptr(b, c, 0), nullptr, nullptr, nullptr,
                                      b->G[c], b->H[c], b->stream));
            b->bc[c].pull = 0;  // in place (kPre)
        }
        HIP_OK(b, hipStreamSynchronize(b->stream));
        return LBM_OK;
    };
    rc = setup();
    if (rc != LBM_OK) {
        char msg[512];
        snprintf(msg, sizeof(msg), "%s", b->err);
        lbm_batch_destroy(b);
        return fail(nullptr, rc, "%s", msg);
    }
    *out = b;
    return LBM_OK;
}

static int check_case(lbm_batch *b, int c) {
    if (!b) return fail(nullptr, LBM_E_INVAL, "batch is NULL");
    if (c < 0 || c >= b->n) return fail(b, LBM_E_INVAL, "case %d out of range [0, %d)", c, b->n);
    return LBM_OK;
}

extern "C" int lbm_batch_set_fields(lbm_batch *b, int c, const double *rho, const double *ux,
                                    const double *uy) {
    int rc = check_case(b, c);
    if (rc != LBM_OK) return rc;
    const size_t n = static_cast<size_t>(b->G[c].nx) * b->G[c].ny;
    rc = ensure_stage(b, 3 * n * sizeof(double));
    if (rc != LBM_OK) return rc;
    double *d[3] = {nullptr, nullptr, nullptr};
    const double *h[3] = {rho, ux, uy};
    for (int i = 0; i < 3; ++i)
        if (h[i]) {
            d[i] = b->d_stage + i * n;
            HIP_OK(b, hipMemcpyAsync(d[i], h[i], n * sizeof(double), hipMemcpyHostToDevice,
                                     b->stream));
        }
    HIP_OK(b, launch_init_feq(b->prec, case_ptr(b, c, b->bc[c].cur), d[0], d[1], d[2], b->G[c],
                              b->H[c], b->stream));
    b->bc[c].pull = 0;
    b->form_prev[c] = kEmpty;
    HIP_OK(b, hipStreamSynchronize(b->stream));
    return upload_cases(b);
}

extern "C" int lbm_batch_set_populations(lbm_batch *b, int c, const double *f) {
    int rc = check_case(b, c);
    if (rc != LBM_OK) return rc;
    if (!f) return fail(b, LBM_E_INVAL, "f is NULL");
    const size_t n9 = static_cast<size_t>(9) * b->G[c].nx * b->G[c].ny;
    rc = ensure_stage(b, n9 * sizeof(double));
    if (rc != LBM_OK) return rc;
    HIP_OK(b, hipMemcpyAsync(b->d_stage, f, n9 * sizeof(double), hipMemcpyHostToDevice,
                             b->stream));
    HIP_OK(b, launch_set_populations(b->prec, case_ptr(b, c, b->bc[c].cur), b->d_stage, b->G[c],
                                     b->H[c], b->stream));
    b->bc[c].pull = 0;
    b->form_prev[c] = kEmpty;
    HIP_OK(b, hipStreamSynchronize(b->stream));
    return upload_cases(b);
}

extern "C" int lbm_batch_get_populations(lbm_batch *b, int c, double *f) {
    int rc = check_case(b, c);
    if (rc != LBM_OK) return rc;
    if (!f) return fail(b, LBM_E_INVAL, "f is NULL");
    const size_t n9 = static_cast<size_t>(9) * b->G[c].nx * b->G[c].ny;
    rc = ensure_stage(b, n9 * sizeof(double));
    if (rc != LBM_OK) return rc;
    HIP_OK(b, launch_get_populations(b->prec, b->bc[c].pull != 0, case_ptr(b, c, b->bc[c].cur),
                                     b->d_stage, b->G[c], b->Kd[c], b->Kf[c], b->H[c], b->stream));
    HIP_OK(b, hipMemcpyAsync(f, b->d_stage, n9 * sizeof(double), hipMemcpyDeviceToHost,
                             b->stream));
    HIP_OK(b, hipStreamSynchronize(b->stream));
    return LBM_OK;
}

extern "C" int lbm_batch_moments(lbm_batch *b, int c, double *rho, double *ux, double *uy) {
    int rc = check_case(b, c);
    if (rc != LBM_OK) return rc;
    const size_t n = static_cast<size_t>(b->G[c].nx) * b->G[c].ny;
    rc = ensure_stage(b, 3 * n * sizeof(double));
    if (rc != LBM_OK) return rc;
    double *d = b->d_stage;
    HIP_OK(b, launch_moments(b->prec, b->bc[c].pull != 0, case_ptr(b, c, b->bc[c].cur), d, d + n,
                             d + 2 * n, b->G[c], b->Kd[c], b->Kf[c], b->H[c], b->stream));
    double *h[3] = {rho, ux, uy};
    for (int i = 0; i < 3; ++i)
        if (h[i])
            HIP_OK(b, hipMemcpyAsync(h[i], d + i * n, n * sizeof(double), hipMemcpyDeviceToHost,
                                     b->stream));
    HIP_OK(b, hipStreamSynchronize(b->stream));
    return LBM_OK;
}

extern "C" int lbm_batch_set_mask(lbm_batch *b, int c, const unsigned char *mask) {
    int rc = check_case(b, c);
    if (rc != LBM_OK) return rc;
    HIP_OK(b, hipStreamSynchronize(b->stream));
    Geometry &G = b->G[c];
    if (!mask) {
        if (b->d_mask[c]) HIP_OK(b, hipFree(b->d_mask[c]));
        b->d_mask[c] = nullptr;
        b->hmask[c].clear();
        G.mask = nullptr;
    } else {
        const size_t n = static_cast<size_t>(G.nx) * G.ny, mbytes = static_cast<size_t>(G.pitch) * G.ny;
        std::vector<unsigned char> pitched;
        try {
            b->hmask[c].assign(mask, mask + n);
            pitched.assign(mbytes, 0);
        } catch (...) {
            return fail(b, LBM_E_NOMEM, "out of host memory");
        }
        for (int j = 0; j < G.ny; ++j)
            for (int i = 0; i < G.nx; ++i)
                pitched[static_cast<size_t>(j) * G.pitch + i] = mask[static_cast<size_t>(j) * G.nx + i] ? 1 : 0;
        if (!b->d_mask[c]) HIP_OK(b, hipMalloc(&b->d_mask[c], mbytes));
        HIP_OK(b, hipMemcpy(b->d_mask[c], pitched.data(), mbytes, hipMemcpyHostToDevice));
        G.mask = b->d_mask[c];
    }
    HIP_OK(b, hipMemcpyAsync(b->d_geoms + c, &G, sizeof(Geometry), hipMemcpyHostToDevice,
                             b->stream));
    HIP_OK(b, hipStreamSynchronize(b->stream));
    b->tiles_dirty = true;  // rebuilt (once) before the next launch
    return LBM_OK;
}

extern "C" int lbm_batch_smooth_step(lbm_batch *b) {
    if (!b) return fail(nullptr, LBM_E_INVAL, "batch is NULL");
    int rc = lbm_batch_step(b, 1);
    if (rc != LBM_OK) return rc;
    size_t most = 0;
    for (int c = 0; c < b->n; ++c)
        if (b->active[c]) {
            const size_t n9 = static_cast<size_t>(9) * b->G[c].nx * b->G[c].ny;
            most = n9 > most ? n9 : most;
        }
    rc = ensure_stage(b, most * sizeof(double));
    if (rc != LBM_OK) return rc;
    for (int c = 0; c < b->n; ++c) {
        if (!b->active[c]) continue;
        const int cur = b->bc[c].cur;
        HIP_OK(b, launch_average_states(b->prec, b->bc[c].pull != 0, case_ptr(b, c, cur),
                                        b->form_prev[c] == kPost, case_ptr(b, c, cur ^ 1),
                                        b->d_stage, b->G[c], b->Kd[c], b->H[c], b->stream));
        HIP_OK(b, launch_set_populations(b->prec, case_ptr(b, c, cur), b->d_stage, b->G[c],
                                         b->H[c], b->stream));
        b->bc[c].pull = 0;
        b->form_prev[c] = kEmpty;
    }
    HIP_OK(b, hipStreamSynchronize(b->stream));
    return upload_cases(b);
}

extern "C" int lbm_batch_set_rates(lbm_batch *b, int c, const double rates[9]) {
    int rc = check_case(b, c);
    if (rc != LBM_OK) return rc;
    if (!rates) return fail(b, LBM_E_INVAL, "rates is NULL");
    for (int j = 0; j < 9; ++j)
        if (!(rates[j] > 0.0 && rates[j] < 2.0))
            return fail(b, LBM_E_INVAL, "rates[%d] = %g is not in (0, 2)", j, rates[j]);
    if (b->higher_unit && !(rates[6] == 1.0 && rates[7] == 1.0 && rates[8] == 1.0))
        return fail(b, LBM_E_INVAL,
                    "this batch was built with omega_6..8 = 1 for every case; they must stay 1");
    HIP_OK(b, hipStreamSynchronize(b->stream));
    memcpy(b->spec[c].rates, rates, sizeof(b->spec[c].rates));
    fill_consts(b->spec[c], b->Kd[c]);
    fill_consts(b->spec[c], b->Kf[c]);
    HIP_OK(b, hipMemcpyAsync(b->d_Kd + c, &b->Kd[c], sizeof(Consts<double>), hipMemcpyHostToDevice,
                             b->stream));
    HIP_OK(b, hipMemcpyAsync(b->d_Kf + c, &b->Kf[c], sizeof(Consts<float>), hipMemcpyHostToDevice,
                             b->stream));
    HIP_OK(b, hipStreamSynchronize(b->stream));
    return LBM_OK;
}

extern "C" int lbm_batch_set_active(lbm_batch *b, const int *active) {
    if (!b || !active) return fail(b, LBM_E_INVAL, "NULL argument");
    bool changed = false;
    for (int c = 0; c < b->n; ++c) {
        const int a = active[c] ? 1 : 0;
        if (a != b->active[c]) changed = true;
        b->active[c] = a;
    }
    if (changed) b->tiles_dirty = true;
    return LBM_OK;
}

// Host bookkeeping after `n` steps of every active case.
static void commit_steps(lbm_batch *b, long n) {
    if (n <= 0) return;
    for (int c = 0; c < b->n; ++c) {
        if (!b->active[c]) continue;
        b->form_prev[c] = n >= 2 ? kPost : (b->bc[c].pull ? kPost : kPre);
        b->bc[c].cur ^= static_cast<int>(n & 1);
        b->bc[c].pull = 1;
        b->steps[c] += n;
    }
}

// Host bookkeeping after `launches` two-step launches (2 x launches steps)
// of every active case: the other buffer then holds the state two steps
// back, which no residual can use.
static void commit_pairs(lbm_batch *b, long launches) {
    if (launches <= 0) return;
    for (int c = 0; c < b->n; ++c) {
        if (!b->active[c]) continue;
        b->form_prev[c] = kEmpty;
        b->bc[c].cur ^= static_cast<int>(launches & 1);
        b->steps[c] += 2 * launches;
    }
}

extern "C" int lbm_batch_step(lbm_batch *b, long n) {
    if (!b) return fail(nullptr, LBM_E_INVAL, "batch is NULL");
    if (n < 0) return fail(b, LBM_E_INVAL, "n must be >= 0");
    int trc = ensure_tiles(b);
    if (trc != LBM_OK) return trc;
    if (n == 0 || b->ntiles == 0) return LBM_OK;
    // first step of cases still in place: one launch reading the per-case
    // forms, then every active case is in pull form
    bool any_pre = false;
    for (int c = 0; c < b->n; ++c)
        if (b->active[c] && !b->bc[c].pull) any_pre = true;
    long left = n;
    if (any_pre) {
        hipError_t e = launch(b, 0, 0, b->workgroups);
        if (e != hipSuccess) return fail(b, LBM_E_DEVICE, "batch step launch failed: %s", hipGetErrorString(e));
        commit_steps(b, 1);
        int rc = upload_cases(b);
        if (rc != LBM_OK) return rc;
        --left;
    }
    if (two_step_on(b) && left >= 3) {
        // pairs while more than two steps remain; the last launch advances
        // one step, so the residual of the last step stays available
        long pairs = (left - 1) / 2;
        left -= 2 * pairs;
        const int gp = graph_pairs(b);
        if (pairs >= gp) {
            int rc = ensure_graph2(b);
            if (rc != LBM_OK) return rc;
            const long reps = pairs / gp;
            for (long i = 0; i < reps; ++i) HIP_OK(b, hipGraphLaunch(b->graph2, b->stream));
            commit_pairs(b, reps * gp);  // an even number of launches
            pairs -= reps * gp;
        }
        for (long i = 0; i < pairs; ++i) {
            hipError_t e = launch2(b, static_cast<int>(i & 1), b->workgroups2);
            if (e != hipSuccess)
                return fail(b, LBM_E_DEVICE, "batch two-step launch failed: %s", hipGetErrorString(e));
        }
        commit_pairs(b, pairs);
        if (pairs & 1) {
            int rc = upload_cases(b);
            if (rc != LBM_OK) return rc;
        }
    }
    if (left >= b->graph_steps) {
        int rc = ensure_graph(b);
        if (rc != LBM_OK) return rc;
        const long reps = left / b->graph_steps;
        for (long i = 0; i < reps; ++i) HIP_OK(b, hipGraphLaunch(b->graph, b->stream));
        // an even number of steps: the current buffer of each case is unchanged
        commit_steps(b, reps * b->graph_steps);
        left -= reps * b->graph_steps;
    }
    for (long i = 0; i < left; ++i) {
        hipError_t e = launch(b, static_cast<int>(i & 1), 1, b->workgroups);
        if (e != hipSuccess) return fail(b, LBM_E_DEVICE, "batch step launch failed: %s", hipGetErrorString(e));
    }
    if (left > 0) {
        commit_steps(b, left);
        if (left & 1) return upload_cases(b);
    }
    return LBM_OK;
}

extern "C" int lbm_batch_residuals(lbm_batch *b, double *R) {
    if (!b || !R) return fail(b, LBM_E_INVAL, "NULL argument");
    std::vector<BatchRed> items;
    std::vector<int> first(b->n, 0), count(b->n, 0);
    for (int c = 0; c < b->n; ++c) {
        first[c] = static_cast<int>(items.size());
        if (b->form_prev[c] == kEmpty || !b->bc[c].pull) continue;
        const int nodes = b->G[c].nx * b->G[c].ny;
        const int flags = 1 | (b->form_prev[c] == kPost ? 2 : 0);
        for (int s = 0; s < nodes; s += kBatchRedNodes)
            items.push_back(BatchRed{c, s, nodes - s < kBatchRedNodes ? nodes - s : kBatchRedNodes,
                                     flags});
        count[c] = static_cast<int>(items.size()) - first[c];
    }
    const int nitems = static_cast<int>(items.size());
    if (nitems > b->item_cap) {
        if (b->d_items) HIP_OK(b, hipFree(b->d_items));
        if (b->d_partials) HIP_OK(b, hipFree(b->d_partials));
        b->d_items = nullptr;
        b->d_partials = nullptr;
        b->item_cap = 0;
        HIP_OK(b, hipMalloc(&b->d_items, nitems * sizeof(BatchRed)));
        HIP_OK(b, hipMalloc(&b->d_partials, nitems * 4 * sizeof(double)));
        b->item_cap = nitems;
    }
    if (nitems)
        HIP_OK(b, hipMemcpyAsync(b->d_items, items.data(), nitems * sizeof(BatchRed),
                                 hipMemcpyHostToDevice, b->stream));
    HIP_OK(b, hipMemcpyAsync(b->d_case_first, first.data(), b->n * sizeof(int),
                             hipMemcpyHostToDevice, b->stream));
    HIP_OK(b, hipMemcpyAsync(b->d_case_count, count.data(), b->n * sizeof(int),
                             hipMemcpyHostToDevice, b->stream));
    HIP_OK(b, launch_batch_residual(b->prec, b->buf[0], b->buf[1], b->d_items, nitems, b->d_cases,
                                    b->d_geoms, b->d_Kd, b->d_H, b->d_partials, b->d_case_first,
                                    b->d_case_count, b->n, b->d_out, b->stream));
    std::vector<double> out(4 * static_cast<size_t>(b->n));
    HIP_OK(b, hipMemcpyAsync(out.data(), b->d_out, out.size() * sizeof(double),
                             hipMemcpyDeviceToHost, b->stream));
    HIP_OK(b, hipStreamSynchronize(b->stream));
    for (int c = 0; c < b->n; ++c) {
        const double *r = &out[4 * c];
        if (count[c] == 0) R[c] = -1.0;
        else if (r[3] != 0.0 || !isfinite(r[0]) || !isfinite(r[1])) R[c] = NAN;
        else R[c] = r[1] > 0.0 ? sqrt(r[0]) / sqrt(r[1]) : (r[0] > 0.0 ? INFINITY : 0.0);
    }
    return LBM_OK;
}

extern "C" int lbm_batch_run_to_steady(lbm_batch *b, double tol, long check_every,
                                       long max_steps, long *steps_out) {
    if (!b) return fail(nullptr, LBM_E_INVAL, "batch is NULL");
    if (!(tol > 0.0) || check_every < 1 || max_steps < 0)
        return fail(b, LBM_E_INVAL, "need tol > 0, check_every >= 1, max_steps >= 0");
    std::vector<long> res(b->n, -2);
    std::vector<double> R(b->n);
    std::vector<int> act(b->active);
    long done = 0;
    bool any = false;
    for (int c = 0; c < b->n; ++c) any = any || act[c];
    while (any && done < max_steps) {
        const long n = check_every < max_steps - done ? check_every : max_steps - done;
        int rc = lbm_batch_step(b, n);
        if (rc != LBM_OK) return rc;
        done += n;
        rc = lbm_batch_residuals(b, R.data());
        if (rc != LBM_OK) return rc;
        bool changed = false;
        any = false;
        for (int c = 0; c < b->n; ++c) {
            if (!act[c]) continue;
            if (isnan(R[c])) {
                res[c] = -1;
                act[c] = 0;
                changed = true;
            } else if (R[c] >= 0.0 && R[c] <= tol) {
                res[c] = done;
                act[c] = 0;
                changed = true;
            } else {
                any = true;
            }
        }
        if (changed) {
            rc = lbm_batch_set_active(b, act.data());
            if (rc != LBM_OK) return rc;
        }
    }
    if (steps_out) memcpy(steps_out, res.data(), b->n * sizeof(long));
    return LBM_OK;
}

extern "C" long lbm_batch_steps_done(const lbm_batch *b, int c) {
    if (!b || c < 0 || c >= b->n) return -1;
    return b->steps[c];
}

// With two steps per launch the autotuner times the two-step kernel's
// persistent grid in each form the precision allows (the register form on
// 64 x 8 block tiles; for LBM_FP32_DEV also the staged form on 64 x 24): one
// block tile per workgroup, or a few workgroups per CU.  Each trial
// recomputes the same pair of steps into the other buffer.
static int autotune_two_step(lbm_batch *b, int trial_steps, int *rows_out, int *workgroups_out) {
    int rc = ensure_tiles(b);
    if (rc != LBM_OK) return rc;
    hipEvent_t e0, e1;
    HIP_OK(b, hipEventCreate(&e0));
    HIP_OK(b, hipEventCreate(&e1));
    float best = 1e30f;
    int best_wgs = b->workgroups2, best_form = b->form2;
    const bool staged_ok = b->prec == kFP32Dev && b->opts.two_step_form != kFormRegister;
    const bool register_ok = b->opts.two_step_form != kFormStaged;
    for (int form : {kFormRegister, kFormStaged}) {
        if ((form == kFormStaged && !staged_ok) || (form == kFormRegister && !register_ok)) continue;
        const int nt = form == kFormStaged ? b->ntiles24 : b->ntiles;
        // resident workgroups per CU: 2 (staged, 77 KB of LDS), 3 or more (register)
        const int per_cu[] = {form == kFormStaged ? 4 : 8, form == kFormStaged ? 2 : 4,
                              form == kFormStaged ? 1 : 2};
        for (int wgs : {nt, 256 * per_cu[0], 256 * per_cu[1], 256 * per_cu[2]}) {
            if (nt == 0) break;
            if (wgs > nt) wgs = nt;
            hipError_t e = launch2_form(b, form, 0, wgs);
            if (e == hipSuccess) e = hipEventRecord(e0, b->stream);
            for (int i = 0; i < trial_steps && e == hipSuccess; ++i) e = launch2_form(b, form, 0, wgs);
            if (e == hipSuccess) e = hipEventRecord(e1, b->stream);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e != hipSuccess) {
                rc = fail(b, LBM_E_DEVICE, "autotune launch failed: %s", hipGetErrorString(e));
                break;
            }
            if (ms < best) {
                best = ms;
                best_wgs = wgs;
                best_form = form;
            }
        }
        if (rc != LBM_OK) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != LBM_OK) return rc;
    b->form2 = best_form;
    b->workgroups2 = best_wgs;
    b->graph2_ok = false;
    // the other buffer of every case was overwritten by the trials
    for (int c = 0; c < b->n; ++c) b->form_prev[c] = kEmpty;
    if (rows_out) *rows_out = best_form == kFormStaged ? kBatchStagedRows : kBatchTileRows;
    if (workgroups_out) *workgroups_out = best_wgs;
    return LBM_OK;
}

extern "C" int lbm_batch_autotune(lbm_batch *b, int trial_steps, int *rows_out,
                                  int *workgroups_out) {
    if (!b) return fail(nullptr, LBM_E_INVAL, "batch is NULL");
    if (trial_steps < 1) return fail(b, LBM_E_INVAL, "trial_steps must be >= 1");
    if (two_step_on(b)) return autotune_two_step(b, trial_steps, rows_out, workgroups_out);
    b->tile_pref = false;  // the march candidates first
    const int rows_c[] = {2, 4, 8, 16};
    const int wg_mult[] = {2, 4, 8, 0};  // x 256 CUs; 0: one tile per wavefront
    hipEvent_t e0, e1;
    HIP_OK(b, hipEventCreate(&e0));
    HIP_OK(b, hipEventCreate(&e1));
    float best = 1e30f;
    int best_rows = b->rows, best_wgs = b->workgroups;
    int rc = LBM_OK;
    for (int rows : rows_c) {
        rc = apply_rows(b, rows);
        if (rc != LBM_OK) break;
        if (b->ntiles == 0) break;
        for (int m : wg_mult) {
            int wgs = m ? 256 * m : (b->ntiles + kWavesPerBlock - 1) / kWavesPerBlock;
            const int need = (b->ntiles + kWavesPerBlock - 1) / kWavesPerBlock;
            if (wgs > need) wgs = need;
            // one untimed launch, then trial_steps timed ones; flip 0: every
            // trial recomputes the same step into the other buffer.  Timed in
            // the pull form that the captured steps run (values are not kept)
            hipError_t e = launch(b, 0, 1, wgs);
            if (e == hipSuccess) e = hipEventRecord(e0, b->stream);
            for (int i = 0; i < trial_steps && e == hipSuccess; ++i) e = launch(b, 0, 1, wgs);
            if (e == hipSuccess) e = hipEventRecord(e1, b->stream);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e != hipSuccess) {
                rc = fail(b, LBM_E_DEVICE, "autotune launch failed: %s", hipGetErrorString(e));
                break;
            }
            if (ms < best) {
                best = ms;
                best_rows = rows;
                best_wgs = wgs;
            }
        }
        if (rc != LBM_OK) break;
    }
    // the batched tile kernel (no masks): one block tile per workgroup, or a
    // persistent grid of 4 or 8 workgroups per CU
    bool best_tile = false;
    if (rc == LBM_OK && !any_mask(b)) {
        b->tile_pref = true;
        rc = upload_tiles(b);
        const int nbt = b->ntiles;
        for (int wgs : {nbt, 256 * 8, 256 * 4}) {
            if (rc != LBM_OK || nbt == 0) break;
            if (wgs > nbt) wgs = nbt;
            hipError_t e = launch(b, 0, 1, wgs);
            if (e == hipSuccess) e = hipEventRecord(e0, b->stream);
            for (int i = 0; i < trial_steps && e == hipSuccess; ++i) e = launch(b, 0, 1, wgs);
            if (e == hipSuccess) e = hipEventRecord(e1, b->stream);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e != hipSuccess) {
                rc = fail(b, LBM_E_DEVICE, "autotune launch failed: %s", hipGetErrorString(e));
                break;
            }
            if (ms < best) {
                best = ms;
                best_tile = true;
                best_rows = kBatchTileRows;
                best_wgs = wgs;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != LBM_OK) return rc;
    b->tile_pref = best_tile;
    // (tile mode keeps 4-row march tiles for when a mask appears)
    rc = apply_rows(b, best_tile ? 4 : best_rows);
    if (rc != LBM_OK) return rc;
    b->workgroups = best_wgs;
    b->graph_ok = false;
    b->graph2_ok = false;
    // the other buffer of every case was overwritten by the trials
    for (int c = 0; c < b->n; ++c) b->form_prev[c] = kEmpty;
    if (rows_out) *rows_out = best_rows;
    if (workgroups_out) *workgroups_out = best_wgs;
    return LBM_OK;
}

extern "C" int lbm_batch_launch_shape(const lbm_batch *b, int *rows_per_wave, int *workgroups,
                                      int *tiles) {
    if (!b) return LBM_E_INVAL;
    // (tile mode reports its block-tile rows and block tiles; with two steps
    // per launch, the two-step kernel's grid)
    const bool tile = tile_mode_wanted(b);
    if (rows_per_wave)
        *rows_per_wave = two_step_on(b) && b->form2 == kFormStaged ? kBatchStagedRows
                         : tile                                     ? kBatchTileRows
                                                                    : b->rows;
    if (workgroups) *workgroups = two_step_on(b) ? b->workgroups2 : b->workgroups;
    if (tiles) {
        // count without touching the device when the list is stale
        int t = 0;
        for (int c = 0; c < b->n; ++c)
            if (b->active[c]) t += tile ? block_tiles(b->G[c]) : b->G[c].ntile;
        *tiles = t;
    }
    return LBM_OK;
}

extern "C" int lbm_batch_uses_tile_kernel(const lbm_batch *b) {
    if (!b) return -1;
    return tile_mode_wanted(b) ? 1 : 0;
}

extern "C" int lbm_batch_steps_per_launch(const lbm_batch *b) {
    if (!b) return LBM_E_INVAL;
    return two_step_on(b) ? 2 : 1;
}

extern "C" int lbm_batch_two_step_form(const lbm_batch *b) {
    if (!b) return LBM_E_INVAL;
    return b->form2;
}

extern "C" const char *lbm_batch_last_error(const lbm_batch *b) {
    return b ? b->err : g_batch_error;
}
