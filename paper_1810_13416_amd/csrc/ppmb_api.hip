// ppmb_api.hip -- host runtime behind the C ABI declared in include/ppmb.h.
//
// A context holds a batch of bricks (a single grid is a batch of one): the
// brick table, the FP64 base state and its working-precision copy, the
// per-brick time steps, reduction buffers, event counters and the block maps
// that let one kernel launch cover every brick of a pass.  The two state
// arenas are the caller's for a single grid and the library's for a batch.
#include "../../include/ppmb.h"
#include "ppmb_internal.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

using namespace ppmb;

struct ppmb_ctx {
    ppmb_precision prec = PPMB_FP64;
    hipStream_t stream = nullptr;
    size_t esz = 8;
    int nb = 0;                         // bricks
    std::vector<Brick> hb;              // brick table (host copy)
    Brick *db = nullptr;                // brick table (device)
    long total_state = 0;               // elements per state arena (15 * sum of field strides)
    long total_base = 0;                // elements per base arena (2 * sum of field strides)
    void *buf[2] = { nullptr, nullptr };
    bool owns_state = false;
    int cur = 0;
    double *base64 = nullptr;           // rho0, p0 per brick (FP64)
    void *baseT = nullptr;              // the same in FP32 (FP32 contexts only)
    double *table = nullptr;            // base-state RK4 nodes (reused brick by brick)
    long table_len = 0;
    double *dt = nullptr;               // per-brick dt
    unsigned long long *cnt = nullptr;  // event counter slots (kCntSlots x kCntStride); word 3: Courant-check flag
    unsigned long long *work = nullptr; // per brick: smax bits, non-physical flag
    unsigned long long *cband = nullptr; // per brick: band edge of the fused CFL reduction, redo flag
    double *partials = nullptr;         // totals block partials
    double *out8 = nullptr;             // totals result
    PassShape shape{ 1, 4, 256, 2 };
    BlockMap *pmap[3] = { nullptr, nullptr, nullptr };   // per pass axis, brick by brick
    BlockMap *pmap_all[3] = { nullptr, nullptr, nullptr };   // the same blocks, longest first over all bricks
    std::vector<int> pfirst[3];         // first block of each brick (+ total at the end)
    BlockMap *cmap = nullptr;           // CFL reduction
    std::vector<int> cfirst;
    BlockMap *dmap = nullptr;           // divergence (shock dissipation)
    std::vector<int> dfirst;
    BlockMap *fmap[3] = { nullptr, nullptr, nullptr };   // flattening, per pass axis
    std::vector<int> ffirst[3];
    long nstep = 0;
    unsigned long long steps = 0;
    // work[] holds the CFL maxima of the current state: the last pass of a
    // step folds them in, so the next step only needs the final division.
    // Cleared by anything else that changes the state or the base.
    bool cfl_ready = false;
    bool profiling = false;
    struct Timed { hipEvent_t a, b; int axis; };
    std::vector<Timed> timed;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    int gkey_cur = -1, gkey_par = -1, gkey_how = -1;
    double gkey_cfl = 0.0;
    // persistent step (ppmb_batch_step modes 3 and 4)
    int *sneed = nullptr;               // [parity][stage][brick]: items of the brick in earlier stages
    unsigned long long *scnt = nullptr; // per brick items done; then next item, abort flag (fine-grained)
    int sworkers = 0;                   // resident waves of the step kernel
    // spin-up ramp: steps 0 .. spin_nramp-1 end with + spin_omega / spin_nramp
    double spin_omega = 0.0;
    long spin_nramp = 0;
    double rot_omega = 0.0;             // rotating frame (0: inertial)
    int rot_centrifugal = 0;
    double *shell_ws = nullptr;         // shell-sum block partials + result
    size_t shell_ws_bytes = 0;
    double dissk = 0.0;                 // shock dissipation coefficient (0: off)
    void *divbuf = nullptr;             // its divergence field (one field per brick)
    double courant_max = 0.0;           // Courant check of caller-given dt (0: off)
    int device = 0;                     // the device current at create
    double *noalloc_ws = nullptr;       // that device's copy of the static shell workspace
    // per brick: both arenas hold the same values in the solid cells (true
    // after a pass that wrote every cell), so passes may skip them
    std::vector<char> solid_same;
    bool skip_on = true;                // ppmb_set_solid_skip
    bool flat_on = false;               // flattening near strong shocks
    void *flatbuf = nullptr;            // its coefficients for the pass in progress
    std::string err;
};

static ppmb_status fail(ppmb_ctx *c, ppmb_status s, const std::string &msg)
{
    if (c) c->err = msg;
    return s;
}

static ppmb_status hipfail(ppmb_ctx *c, hipError_t e, const char *where)
{
    if (e == hipSuccess) return PPMB_OK;
    return fail(c, PPMB_ERR_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

#define HIPCHK(ctx, expr)                                            \
    do {                                                             \
        hipError_t e_ = (expr);                                      \
        if (e_ != hipSuccess) return hipfail((ctx), e_, #expr);      \
    } while (0)

#define TRY(expr)                                                    \
    do {                                                             \
        ppmb_status s_ = (expr);                                     \
        if (s_ != PPMB_OK) return s_;                                \
    } while (0)

template <typename T>
static T *arena(ppmb_ctx *c, int which) { return static_cast<T *>(c->buf[which]); }

static void free_graph(ppmb_ctx *c)
{
    if (c->gexec) hipGraphExecDestroy(c->gexec);
    if (c->graph) hipGraphDestroy(c->graph);
    c->gexec = nullptr;
    c->graph = nullptr;
    c->gkey_cur = c->gkey_par = c->gkey_how = -1;
}

// The state of bricks [b0, b1) was written by something other than a
// pass: the next pass writes every cell again (a captured step graph
// holds passes that skip solid cells, so it goes too).
static void solid_reset(ppmb_ctx *c, int b0, int b1)
{
    for (int b = b0; b < b1; ++b) c->solid_same[b] = 0;
    free_graph(c);
}

static bool solid_all_same(const ppmb_ctx *c, int b0, int b1)
{
    for (int b = b0; b < b1; ++b)
        if (!c->solid_same[b]) return false;
    return true;
}

static void free_maps(ppmb_ctx *c)
{
    for (int d = 0; d < 3; ++d) {
        hipFree(c->pmap[d]);
        c->pmap[d] = nullptr;
        hipFree(c->pmap_all[d]);
        c->pmap_all[d] = nullptr;
    }
    hipFree(c->cmap);
    c->cmap = nullptr;
    hipFree(c->sneed);
    c->sneed = nullptr;
    hipFree(c->dmap);
    c->dmap = nullptr;
    for (int d = 0; d < 3; ++d) { hipFree(c->fmap[d]); c->fmap[d] = nullptr; }
}

static ppmb_status upload_map(ppmb_ctx *c, const std::vector<BlockMap> &m, BlockMap **dst)
{
    if (hipMalloc(dst, sizeof(BlockMap) * (m.empty() ? 1 : m.size())) != hipSuccess)
        return fail(c, PPMB_ERR_NOMEM, "block map allocation");
    HIPCHK(c, hipMemcpy(*dst, m.data(), sizeof(BlockMap) * m.size(), hipMemcpyHostToDevice));
    return PPMB_OK;
}

// Block maps: every pass launch and the CFL launch cover all bricks; a
// per-brick launch covers the slice [first[b], first[b + 1]).
static ppmb_status build_maps(ppmb_ctx *c)
{
    free_graph(c);
    free_maps(c);
    for (int d = 0; d < 3; ++d) {
        // per brick, blocks longest first (with solid cells skipped their
        // work differs widely, and a launch ends when its last block does);
        // for launches over all bricks the same blocks longest first across
        // bricks of different sizes
        std::vector<BlockMap> m;
        std::vector<std::pair<double, size_t>> all;
        c->pfirst[d].assign(c->nb + 1, 0);
        for (int b = 0; b < c->nb; ++b) {
            c->pfirst[d][b] = (int)m.size();
            const Geom &g = c->hb[b].g;
            const int n = pass_blocks(g, d, c->shape);
            std::vector<std::pair<double, int>> order((size_t)n);
            for (int l = 0; l < n; ++l) order[l] = { -pass_block_cost(g, d, c->shape, l), l };
            // (the x pass keeps its rows in storage order: sorted, waves
            // running together would touch rows all over the grid)
            if (g.sphere && d != 0) std::stable_sort(order.begin(), order.end());
            for (const auto &o : order) {
                all.push_back({ d != 0 ? o.first : 0.0, m.size() });
                m.push_back(BlockMap{ b, o.second });
            }
        }
        c->pfirst[d][c->nb] = (int)m.size();
        if (m.size() > 0x7fffffff) return fail(c, PPMB_ERR_INVALID, "too many blocks");
        TRY(upload_map(c, m, &c->pmap[d]));
        std::stable_sort(all.begin(), all.end());
        std::vector<BlockMap> ma;
        ma.reserve(m.size());
        for (const auto &a : all) ma.push_back(m[a.second]);
        TRY(upload_map(c, ma, &c->pmap_all[d]));
    }
    std::vector<BlockMap> m;
    c->cfirst.assign(c->nb + 1, 0);
    for (int b = 0; b < c->nb; ++b) {
        c->cfirst[b] = (int)m.size();
        int n = cfl_blocks(c->hb[b].ncell);
        for (int l = 0; l < n; ++l) m.push_back(BlockMap{ b, l });
    }
    c->cfirst[c->nb] = (int)m.size();
    TRY(upload_map(c, m, &c->cmap));
    {
        // persistent step: per pass order, stage and brick, the brick's
        // items in the earlier stages (what its items of that stage wait for)
        const int order[2][3] = { { 0, 1, 2 }, { 2, 1, 0 } };
        std::vector<int> need((size_t)2 * kStepStages * c->nb);
        for (int par = 0; par < 2; ++par)
            for (int b = 0; b < c->nb; ++b) {
                int nblk[3];
                for (int p = 0; p < 3; ++p) nblk[p] = c->pfirst[order[par][p]][b + 1] - c->pfirst[order[par][p]][b];
                long acc = 0;
                for (int st = 0; st < kStepStages; ++st) {
                    need[((size_t)par * kStepStages + st) * c->nb + b] = (int)acc;
                    acc += step_stage_units(c->shape, st, order[par], nblk, c->cfirst[b + 1] - c->cfirst[b]);
                }
                if (acc > 0x7fffffff) return fail(c, PPMB_ERR_INVALID, "too many step items");
            }
        if (hipMalloc(&c->sneed, sizeof(int) * need.size()) != hipSuccess)
            return fail(c, PPMB_ERR_NOMEM, "step plan allocation");
        HIPCHK(c, hipMemcpy(c->sneed, need.data(), sizeof(int) * need.size(), hipMemcpyHostToDevice));
    }
    m.clear();
    c->dfirst.assign(c->nb + 1, 0);
    for (int b = 0; b < c->nb; ++b) {
        c->dfirst[b] = (int)m.size();
        int n = div_blocks(c->hb[b].g);
        for (int l = 0; l < n; ++l) m.push_back(BlockMap{ b, l });
    }
    c->dfirst[c->nb] = (int)m.size();
    if (m.size() > 0x7fffffff) return fail(c, PPMB_ERR_INVALID, "too many blocks");
    TRY(upload_map(c, m, &c->dmap));
    for (int d = 0; d < 3; ++d) {
        m.clear();
        c->ffirst[d].assign(c->nb + 1, 0);
        for (int b = 0; b < c->nb; ++b) {
            c->ffirst[d][b] = (int)m.size();
            int n = flat_blocks(c->hb[b].g, d);
            for (int l = 0; l < n; ++l) m.push_back(BlockMap{ b, l });
        }
        c->ffirst[d][c->nb] = (int)m.size();
        if (m.size() > 0x7fffffff) return fail(c, PPMB_ERR_INVALID, "too many blocks");
        TRY(upload_map(c, m, &c->fmap[d]));
    }
    return PPMB_OK;
}

// Gravity and heating parameters: kind known, values finite, the radial
// core radius and taper interval and the heating extent positive.
static bool gravity_ok(int kind, const double *p)
{
    if (kind < PPMB_GRAV_NONE || kind > PPMB_GRAV_RADIAL) return false;
    const int np = kind == PPMB_GRAV_CONST ? 3 : (kind == PPMB_GRAV_RADIAL ? 4 : 0);
    for (int q = 0; q < np; ++q)
        if (!std::isfinite(p[q])) return false;
    return kind != PPMB_GRAV_RADIAL || (p[1] > 0.0 && p[3] > p[2]);
}

static bool heating_ok(int kind, const double *p)
{
    if (kind < PPMB_HEAT_NONE || kind > PPMB_HEAT_BALL) return false;
    const int np = kind == PPMB_HEAT_LAYER_Z ? 3 : (kind == PPMB_HEAT_BALL ? 2 : 0);
    for (int q = 0; q < np; ++q)
        if (!std::isfinite(p[q])) return false;
    return kind == PPMB_HEAT_NONE || p[1] > 0.0;
}

static ppmb_status check_grid(const ppmb_grid *grid)
{
    if (!grid) return PPMB_ERR_INVALID;
    for (int d = 0; d < 3; ++d) {
        if (grid->n[d] < 1) return PPMB_ERR_INVALID;
        if (grid->bc[d] != PPMB_BC_PERIODIC && grid->bc[d] != PPMB_BC_REFLECT) return PPMB_ERR_INVALID;
    }
    if (!(grid->dx > 0.0) || !(grid->gamma > 1.0)) return PPMB_ERR_INVALID;
    if (!gravity_ok(grid->grav_kind, grid->grav) || !heating_ok(grid->heat_kind, grid->heat))
        return PPMB_ERR_INVALID;
    if (grid->smooth_detect < 0 || grid->smooth_detect > 2) return PPMB_ERR_INVALID;
    if ((long)grid->n[0] * grid->n[1] * grid->n[2] >= (1L << 31)) return PPMB_ERR_INVALID;
    return PPMB_OK;
}

// Least t with sqrt(t) >= R (IEEE sqrt, correctly rounded and monotone):
// sqrt(r2) >= R exactly when r2 >= t.  R <= 0: every r2 >= 0 passes;
// NaN R: none does.
static double solid_threshold(double R)
{
    if (R != R) return R;
    if (!(R > 0.0)) return -INFINITY;
    if (std::isinf(R)) return R;
    double t = R * R;
    while (std::sqrt(t) < R) t = std::nextafter(t, INFINITY);
    for (;;) {
        double d = std::nextafter(t, 0.0);
        if (std::sqrt(d) < R) break;
        t = d;
    }
    return t;
}

static void source_constants(Geom &g);

static Geom geom_of(const ppmb_grid *grid)
{
    Geom g{};
    for (int d = 0; d < 3; ++d) { g.n[d] = grid->n[d]; g.origin[d] = grid->origin[d]; g.bc[d] = grid->bc[d]; }
    g.dx = grid->dx;
    g.gamma = grid->gamma;
    g.sphere = grid->sphere;
    g.sphere_r = grid->sphere_r;
    g.sphere_t = solid_threshold(grid->sphere_r);
    g.grav_kind = grid->grav_kind;
    for (int q = 0; q < 4; ++q) g.grav[q] = grid->grav[q];
    g.heat_kind = grid->heat_kind;
    for (int q = 0; q < 3; ++q) g.heat[q] = grid->heat[q];
    g.smooth_detect = grid->smooth_detect;
    source_constants(g);
    // pitched storage: rows padded to 64 elements (256-byte aligned in FP32),
    // fields padded by 17 x 64 elements more, so that corresponding cells of
    // the 15 fields do not share cache sets
    g.px = (grid->n[0] + 63) / 64 * 64;
    g.plane = (long)g.px * grid->n[1];
    g.fs = (g.plane * grid->n[2] + 63) / 64 * 64 + 17 * 64;
    return g;
}

// The pass kernels' gravity and heating constants in both precisions, from
// grav_kind / grav and heat_kind / heat, once on the host.
static void source_constants(Geom &g)
{
    double gc[6] = { 0, 0, 0, 0, 0, 0 };
    if (g.grav_kind == 1) {
        for (int q = 0; q < 3; ++q) gc[q] = g.grav[q];
    } else if (g.grav_kind == 2) {
        gc[0] = g.grav[0];
        gc[1] = g.grav[1];
        gc[2] = 1.0 / g.grav[1];
        gc[3] = g.grav[2];
        gc[4] = g.grav[3];
        gc[5] = 1.0 / (g.grav[3] - g.grav[2]);
    }
    for (int q = 0; q < 6; ++q) { g.gcd[q] = gc[q]; g.gcf[q] = (float)gc[q]; }
    const double hc[3] = { g.heat[0], g.heat_kind ? 1.0 / g.heat[1] : 0.0, g.heat[2] };
    for (int q = 0; q < 3; ++q) { g.hcd[q] = hc[q]; g.hcf[q] = (float)hc[q]; }
}

// Static workspace of ppmb_shell_profile_noalloc: a file-scope device array,
// one copy per GPU the library runs on, held until the process ends.  Host
// code never names it directly (the host-side symbol is not a device
// address): its device address is looked up once per device, at create,
// and kept below.
constexpr long kShellStaticDoubles = 4L << 20;          // 32 MiB
static __device__ __align__(256) double scratch[kShellStaticDoubles];
constexpr int kMaxDevices = 64;
static std::mutex scratch_mu;
static double *scratch_ptr[kMaxDevices] = {};

// The static workspace's address on the current device (looked up once).
static hipError_t scratch_of_current_device(int *device, double **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(scratch_mu);
    if (!scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        scratch_ptr[dev] = static_cast<double *>(p);
    }
    *device = dev;
    *out = scratch_ptr[dev];
    return hipSuccess;
}

static ppmb_status create_common(int nbricks, const ppmb_grid *grids, ppmb_precision prec,
                                 void *hip_stream, bool own_state, ppmb_ctx **out)
{
    if (!grids || !out || nbricks < 1) return PPMB_ERR_INVALID;
    *out = nullptr;
    if (prec != PPMB_FP64 && prec != PPMB_FP32) return PPMB_ERR_INVALID;
    for (int b = 0; b < nbricks; ++b) TRY(check_grid(&grids[b]));
    ppmb_ctx *c = new ppmb_ctx();
    c->prec = prec;
    c->stream = static_cast<hipStream_t>(hip_stream);
    c->esz = prec == PPMB_FP64 ? 8 : 4;
    c->nb = nbricks;
    long off = 0, boff = 0, maxspan = 0;
    for (int b = 0; b < nbricks; ++b) {
        Brick B{};
        B.g = geom_of(&grids[b]);
        B.ncell = (long)B.g.n[0] * B.g.n[1] * B.g.n[2];
        B.off = off;
        B.boff = boff;
        B.dti = b;
        off += (long)NF * B.g.fs;
        boff += 2 * B.g.fs;
        long span = (long)(4.0 * (B.g.n[0] + B.g.n[1] + B.g.n[2]) * 8.0) + 64;
        if (span > maxspan) maxspan = span;
        c->hb.push_back(B);
    }
    c->total_state = off;
    c->total_base = boff;
    c->solid_same.assign(nbricks, 0);
    if (const char *e = getenv("PPMB_CHECK_CFL"))
        if (e[0] == '1' && e[1] == 0) c->courant_max = 1.0;
    // PPMB_X_MARCH=1: the x pass by the marching kernel (for comparison)
    if (const char *e = getenv("PPMB_X_MARCH"))
        if (e[0] == '1' && e[1] == 0) c->shape.x_rows = 0;
    c->table_len = 64 + 2 * maxspan;
    hipError_t e = scratch_of_current_device(&c->device, &c->noalloc_ws);
    if (e != hipSuccess) {
        delete c;
        return PPMB_ERR_HIP;
    }
    e = hipMalloc(&c->db, sizeof(Brick) * nbricks);
    if (e == hipSuccess) e = hipMalloc(&c->base64, sizeof(double) * boff);
    if (e == hipSuccess) e = hipMemset(c->base64, 0, sizeof(double) * boff);   // padding included
    if (e == hipSuccess && prec == PPMB_FP32) e = hipMalloc(&c->baseT, sizeof(float) * boff);
    if (e == hipSuccess) e = hipMalloc(&c->table, sizeof(double) * c->table_len);
    if (e == hipSuccess) e = hipMalloc(&c->dt, sizeof(double) * nbricks);
    if (e == hipSuccess) e = hipMalloc(&c->cnt, sizeof(unsigned long long) * kCntWords);
    if (e == hipSuccess) e = hipMalloc(&c->work, sizeof(unsigned long long) * 2 * nbricks);
    if (e == hipSuccess) e = hipMalloc(&c->cband, sizeof(unsigned long long) * 2 * nbricks);
    // the persistent step's counters are polled by waves on every XCD while
    // the kernel runs: fine-grained memory, coherent during a kernel (what
    // hipMalloc returns is coherent only at dispatch boundaries)
    if (e == hipSuccess)
        e = hipExtMallocWithFlags((void **)&c->scnt, sizeof(unsigned long long) * (nbricks + 2),
                                  hipDeviceMallocFinegrained);
    if (e == hipSuccess) e = hipMalloc(&c->partials, sizeof(double) * 8 * kTotalsBlocks);
    if (e == hipSuccess) e = hipMalloc(&c->out8, sizeof(double) * 8);
    if (e == hipSuccess && own_state) {
        e = hipMalloc(&c->buf[0], c->esz * off);
        if (e == hipSuccess) e = hipMalloc(&c->buf[1], c->esz * off);
        c->owns_state = true;
    }
    if (e != hipSuccess) {
        ppmb_destroy(c);
        return PPMB_ERR_NOMEM;
    }
    ppmb_status st = PPMB_OK;
    if (hipMemcpy(c->db, c->hb.data(), sizeof(Brick) * nbricks, hipMemcpyHostToDevice) != hipSuccess ||
        launch_zero_u64(c->cnt, kCntWords, c->stream) != hipSuccess ||
        launch_zero_u64(c->work, 2 * nbricks, c->stream) != hipSuccess ||
        launch_zero_u64(c->cband, 2 * nbricks, c->stream) != hipSuccess ||
        launch_zero_u64(c->scnt, nbricks + 2, c->stream) != hipSuccess)
        st = PPMB_ERR_HIP;
    c->sworkers = prec == PPMB_FP32 ? step_workers<float>() : step_workers<double>();
    if (st == PPMB_OK) st = build_maps(c);
    // base state NONE until set
    double zero[6] = { 0, 0, 0, 0, 0, 0 };
    for (int b = 0; st == PPMB_OK && b < nbricks; ++b)
        if (launch_base_state(c->hb[b].g, PPMB_BASE_NONE, zero, c->table, c->table_len,
                              c->base64 + c->hb[b].boff, c->base64 + c->hb[b].boff + c->hb[b].g.fs,
                              c->stream) != hipSuccess)
            st = PPMB_ERR_HIP;
    if (st == PPMB_OK && prec == PPMB_FP32 &&
        launch_narrow<float>(c->base64, static_cast<float *>(c->baseT), boff, c->stream) != hipSuccess)
        st = PPMB_ERR_HIP;
    if (st == PPMB_OK && hipStreamSynchronize(c->stream) != hipSuccess) st = PPMB_ERR_HIP;
    if (st != PPMB_OK) {
        ppmb_destroy(c);
        return st;
    }
    *out = c;
    return PPMB_OK;
}

static ppmb_status need_state(ppmb_ctx *c)
{
    if (!c->buf[0] || !c->buf[1]) return fail(c, PPMB_ERR_INVALID, "state buffers not bound");
    return PPMB_OK;
}

static ppmb_status check_brick(ppmb_ctx *c, int b)
{
    if (b < 0 || b >= c->nb) return fail(c, PPMB_ERR_INVALID, "brick index out of range");
    return need_state(c);
}

// ---------------------------------------------------------------------
// enqueue helpers
// ---------------------------------------------------------------------

static ppmb_status enqueue_cfl(ppmb_ctx *c, double cfl, int b0, int b1)
{
    const int f0 = c->cfirst[b0], f1 = c->cfirst[b1];
    if (c->prec == PPMB_FP64)
        HIPCHK(c, launch_cfl<double>(c->db, b0, b1 - b0, c->cmap + f0, f1 - f0, arena<double>(c, c->cur),
                                     c->base64, c->work, cfl, c->dt, c->stream));
    else
        HIPCHK(c, launch_cfl<float>(c->db, b0, b1 - b0, c->cmap + f0, f1 - f0, arena<float>(c, c->cur),
                                    c->base64, c->work, cfl, c->dt, c->stream));
    return PPMB_OK;
}

// One pass along `axis` for bricks [b0, b1), reading arena `from`; with
// `cfl` it also reduces the signal speeds of its output into work[].
static ppmb_status enqueue_pass(ppmb_ctx *c, int axis, int heat, int b0, int b1, int from, int cfl = 0)
{
    if (c->flat_on && !(axis == 0 && c->shape.x_rows > 0)) {
        // flattening coefficients of this pass's input along its axis (the
        // lanes-along-x kernel evaluates its own)
        const int g0 = c->ffirst[axis][b0], g1 = c->ffirst[axis][b1];
        if (c->prec == PPMB_FP64)
            HIPCHK(c, launch_flattening<double>(axis, c->db, c->fmap[axis] + g0, g1 - g0, arena<double>(c, from),
                                                c->base64, static_cast<double *>(c->flatbuf), c->skip_on ? 1 : 0,
                                                c->stream));
        else
            HIPCHK(c, launch_flattening<float>(axis, c->db, c->fmap[axis] + g0, g1 - g0, arena<float>(c, from),
                                               c->base64, static_cast<float *>(c->flatbuf), c->skip_on ? 1 : 0,
                                               c->stream));
    }
    const int f0 = c->pfirst[axis][b0], f1 = c->pfirst[axis][b1];
    ppmb_ctx::Timed tm{ nullptr, nullptr, axis };
    if (c->profiling) {
        HIPCHK(c, hipEventCreate(&tm.a));
        HIPCHK(c, hipEventCreate(&tm.b));
        HIPCHK(c, hipEventRecord(tm.a, c->stream));
    }
    hipError_t e;
    const int skip = c->skip_on && solid_all_same(c, b0, b1) ? 1 : 0;
    const BlockMap *map = (b0 == 0 && b1 == c->nb) ? c->pmap_all[axis] : c->pmap[axis] + f0;
    if (c->prec == PPMB_FP64)
        e = launch_sweep<double>(axis, c->shape, c->db, map, f1 - f0, arena<double>(c, from),
                                 arena<double>(c, 1 - from), c->base64, c->dt, c->cnt, heat, c->base64,
                                 c->work, c->cband, static_cast<const double *>(c->divbuf), c->dissk,
                                 c->flat_on ? static_cast<const double *>(c->flatbuf) : nullptr, cfl, skip,
                                 c->stream);
    else
        e = launch_sweep<float>(axis, c->shape, c->db, map, f1 - f0, arena<float>(c, from),
                                arena<float>(c, 1 - from), static_cast<const float *>(c->baseT), c->dt,
                                c->cnt, heat, c->base64, c->work, c->cband, static_cast<const float *>(c->divbuf),
                                c->dissk, c->flat_on ? static_cast<const float *>(c->flatbuf) : nullptr, cfl,
                                skip, c->stream);
    if (e != hipSuccess) return hipfail(c, e, "sweep launch");
    // a pass that wrote every cell copied the solid ones unchanged
    for (int b = b0; b < b1; ++b) c->solid_same[b] = 1;
    if (c->profiling) {
        HIPCHK(c, hipEventRecord(tm.b, c->stream));
        c->timed.push_back(tm);
    }
    return PPMB_OK;
}

static bool any_heat(ppmb_ctx *c)
{
    for (auto &B : c->hb)
        if (B.g.heat_kind != PPMB_HEAT_NONE) return true;
    return false;
}

// The divergence field of arena `from` for bricks [b0, b1) (shock
// dissipation on).
static ppmb_status enqueue_divergence(ppmb_ctx *c, int b0, int b1, int from)
{
    const int f0 = c->dfirst[b0], f1 = c->dfirst[b1];
    if (c->prec == PPMB_FP64)
        HIPCHK(c, launch_divergence<double>(c->db, c->dmap + f0, f1 - f0, arena<double>(c, from), c->base64,
                                            static_cast<double *>(c->divbuf), c->skip_on ? 1 : 0,
                                            c->stream));
    else
        HIPCHK(c, launch_divergence<float>(c->db, c->dmap + f0, f1 - f0, arena<float>(c, from), c->base64,
                                           static_cast<float *>(c->divbuf), c->skip_on ? 1 : 0,
                                           c->stream));
    return PPMB_OK;
}

// Three passes (x,y,z on even steps, z,y,x on odd) for bricks [b0, b1);
// the last one also reduces the CFL maxima of the new state.  With shock
// dissipation on, the divergence of the state at the start of the step
// drives it in all three.
static ppmb_status enqueue_passes(ppmb_ctx *c, int b0, int b1, int from)
{
    if (c->dissk > 0.0) TRY(enqueue_divergence(c, b0, b1, from));
    const int heat = any_heat(c) ? 1 : 0;
    const int order[2][3] = { { 0, 1, 2 }, { 2, 1, 0 } };
    const int *o = order[c->nstep & 1];
    for (int p = 0; p < 3; ++p) {
        if (p == 2) HIPCHK(c, launch_cfl_arm(c->work, c->cband, b0, b1 - b0, c->stream));
        TRY(enqueue_pass(c, o[p], p == 2 ? heat : 0, b0, b1, from, p == 2 ? 1 : 0));
        from = 1 - from;
    }
    return PPMB_OK;
}

// dt of bricks [b0, b1) for the coming step: from the maxima the previous
// step's last pass left in work[] when they describe the current state,
// else by a CFL reduction over the state.
static ppmb_status enqueue_dt(ppmb_ctx *c, bool ready, double cfl, int b0, int b1)
{
    if (ready) {
        const int f0 = c->cfirst[b0], f1 = c->cfirst[b1];
        if (c->prec == PPMB_FP64)
            HIPCHK(c, launch_cfl_finish<double>(c->db, b0, b1 - b0, c->cmap + f0, f1 - f0, arena<double>(c, c->cur),
                                                c->base64, c->work, c->cband, cfl, c->dt, c->stream));
        else
            HIPCHK(c, launch_cfl_finish<float>(c->db, b0, b1 - b0, c->cmap + f0, f1 - f0, arena<float>(c, c->cur),
                                               c->base64, c->work, c->cband, cfl, c->dt, c->stream));
        return PPMB_OK;
    }
    return enqueue_cfl(c, cfl, b0, b1);
}

// Spin-up increment on the current state of every brick.  The CFL maxima
// of the last pass no longer describe the state afterwards.
static ppmb_status enqueue_spin(ppmb_ctx *c, double domega)
{
    const int nblk = c->cfirst[c->nb];
    if (c->prec == PPMB_FP64)
        HIPCHK(c, launch_spin<double>(c->db, c->cmap, nblk, arena<double>(c, c->cur), c->base64, domega,
                                      c->stream));
    else
        HIPCHK(c, launch_spin<float>(c->db, c->cmap, nblk, arena<float>(c, c->cur), c->base64, domega,
                                     c->stream));
    c->cfl_ready = false;
    return PPMB_OK;
}

// Rotating-frame sources at the end of a step, every brick over its dt.
// The CFL maxima of the last pass no longer describe the state afterwards.
static ppmb_status enqueue_rotframe(ppmb_ctx *c)
{
    const int nblk = c->cfirst[c->nb];
    if (c->prec == PPMB_FP64)
        HIPCHK(c, launch_rotframe<double>(c->db, c->cmap, nblk, arena<double>(c, c->cur), c->base64, c->dt,
                                          c->rot_omega, c->rot_centrifugal, c->stream));
    else
        HIPCHK(c, launch_rotframe<float>(c->db, c->cmap, nblk, arena<float>(c, c->cur), c->base64, c->dt,
                                         c->rot_omega, c->rot_centrifugal, c->stream));
    c->cfl_ready = false;
    return PPMB_OK;
}

// The persistent step kernel is built but not launched (see ppmb_batch_step).
constexpr bool kPersistentStepOn = false;

// Whether the persistent step kernel can run this context's step: the
// plain passes (no shock dissipation, no flattening) with the x pass by
// the lanes-along-x code, and a device that holds its waves.
static bool persistent_ok(const ppmb_ctx *c)
{
    return kPersistentStepOn && c->dissk == 0.0 && !c->flat_on && step_eligible(c->shape) && c->sworkers > 0;
}

// The three passes of every brick, and the step's dt from the maxima the
// previous step left (when they describe the state), in one launch of the
// persistent step kernel.  Without those maxima the CFL reduction runs
// first, as its own launches.
static ppmb_status enqueue_persistent(ppmb_ctx *c, bool with_cfl, double cfl)
{
    const bool ready = with_cfl && c->cfl_ready;
    if (with_cfl && !ready) TRY(enqueue_cfl(c, cfl, 0, c->nb));
    const int order[2][3] = { { 0, 1, 2 }, { 2, 1, 0 } };
    const int par = (int)(c->nstep & 1);
    const int *o = order[par];
    const BlockMap *maps[3];
    int nbl[3];
    for (int p = 0; p < 3; ++p) {
        maps[p] = c->pmap_all[o[p]];
        nbl[p] = c->pfirst[o[p]][c->nb];
    }
    HIPCHK(c, launch_zero_u64(c->scnt, c->nb + 2, c->stream));
    const int skip_first = c->skip_on && solid_all_same(c, 0, c->nb) ? 1 : 0;
    const int heat = any_heat(c) ? 1 : 0;
    const int *need = c->sneed + (size_t)par * kStepStages * c->nb;
    hipError_t e;
    if (c->prec == PPMB_FP64)
        e = launch_step<double>(c->shape, c->db, c->nb, o, maps, nbl, c->cmap, c->cfirst[c->nb], need, c->scnt,
                                arena<double>(c, c->cur), arena<double>(c, 1 - c->cur), c->base64, c->dt, c->cnt,
                                heat, c->base64, c->work, c->cband, skip_first, c->skip_on ? 1 : 0, ready ? 1 : 0,
                                cfl, c->sworkers, c->stream);
    else
        e = launch_step<float>(c->shape, c->db, c->nb, o, maps, nbl, c->cmap, c->cfirst[c->nb], need, c->scnt,
                               arena<float>(c, c->cur), arena<float>(c, 1 - c->cur),
                               static_cast<const float *>(c->baseT), c->dt, c->cnt, heat, c->base64, c->work,
                               c->cband, skip_first, c->skip_on ? 1 : 0, ready ? 1 : 0, cfl, c->sworkers,
                               c->stream);
    if (e != hipSuccess) return hipfail(c, e, "step launch");
    for (int b = 0; b < c->nb; ++b) c->solid_same[b] = 1;
    return PPMB_OK;
}

// How a step is launched: one launch per stage for all bricks, one per
// stage and brick, or the persistent step kernel.
enum StepHow { kBatched = 0, kPerBrick = 1, kPersistent = 2 };

// One step of every brick (see StepHow; the persistent kernel only where
// it applies, else per stage); during a spin-up ramp the step ends with
// the rotation increment.
static ppmb_status enqueue_step(ppmb_ctx *c, bool with_cfl, double cfl, int how = kBatched)
{
    const bool ready = c->cfl_ready;
    if (how == kPersistent && persistent_ok(c)) {
        TRY(enqueue_persistent(c, with_cfl, cfl));
    } else if (how == kPerBrick) {
        for (int b = 0; b < c->nb; ++b) {
            if (with_cfl) TRY(enqueue_dt(c, ready, cfl, b, b + 1));
            TRY(enqueue_passes(c, b, b + 1, c->cur));
        }
    } else {
        if (with_cfl) TRY(enqueue_dt(c, ready, cfl, 0, c->nb));
        TRY(enqueue_passes(c, 0, c->nb, c->cur));
    }
    c->cur = 1 - c->cur;           // three passes: the state ends in the other arena
    c->cfl_ready = true;
    if (c->rot_omega != 0.0) TRY(enqueue_rotframe(c));
    if (c->nstep < c->spin_nramp) TRY(enqueue_spin(c, c->spin_omega / (double)c->spin_nramp));
    c->nstep++;
    c->steps++;
    return PPMB_OK;
}

// The deferred error flags (synchronising): the per-brick non-physical
// flags of the CFL reductions and the Courant-check flag.  A raised flag is
// cleared and reported once.
static ppmb_status check_flag(ppmb_ctx *c)
{
    std::vector<unsigned long long> w(2 * c->nb);
    unsigned long long cf = 0, ab = 0;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemcpy(w.data(), c->work, sizeof(unsigned long long) * w.size(), hipMemcpyDeviceToHost));
    HIPCHK(c, hipMemcpy(&cf, c->cnt + 3, sizeof(unsigned long long), hipMemcpyDeviceToHost));
    HIPCHK(c, hipMemcpy(&ab, c->scnt + c->nb + 1, sizeof(unsigned long long), hipMemcpyDeviceToHost));
    if (ab) {
        HIPCHK(c, launch_zero_u64(c->scnt + c->nb + 1, 1, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        c->cfl_ready = false;
        return fail(c, PPMB_ERR_HIP, "persistent step: a wait for another brick's items gave up; the state is invalid");
    }
    bool bad = false;
    for (int b = 0; b < c->nb; ++b) bad = bad || w[2 * b + 1];
    if (bad) {
        HIPCHK(c, launch_zero_u64(c->work, 2 * c->nb, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        c->cfl_ready = false;
        return fail(c, PPMB_ERR_NONPHYSICAL, "non-positive density or pressure, or NaN, in a fluid cell");
    }
    if (cf) {
        HIPCHK(c, launch_zero_u64(c->cnt + 3, 1, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        return fail(c, PPMB_ERR_CFL, "a step's dt exceeded the Courant limit of the CFL check");
    }
    return PPMB_OK;
}

// dt of every brick for ppmb_step / ppmb_pass: the given value, after the
// Courant check when it is on.
static ppmb_status enqueue_given_dt(ppmb_ctx *c, double dt)
{
    if (c->courant_max > 0.0) {
        TRY(enqueue_cfl(c, c->courant_max, 0, c->nb));
        HIPCHK(c, launch_cfl_given(c->db, 0, c->nb, dt, c->dt, c->cnt + 3, c->stream));
        return PPMB_OK;
    }
    for (int b = 0; b < c->nb; ++b) HIPCHK(c, launch_set_scalar(c->dt + b, dt, c->stream));
    return PPMB_OK;
}

extern "C" {

const char *ppmb_status_string(ppmb_status s)
{
    switch (s) {
    case PPMB_OK: return "ok";
    case PPMB_ERR_INVALID: return "invalid argument";
    case PPMB_ERR_NOMEM: return "out of device memory";
    case PPMB_ERR_HIP: return "HIP error";
    case PPMB_ERR_NONPHYSICAL: return "non-physical state";
    case PPMB_ERR_CFL: return "time step above the Courant limit";
    case PPMB_ERR_UNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

const char *ppmb_last_error(const ppmb_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

ppmb_status ppmb_create(const ppmb_grid *grid, ppmb_precision prec, void *hip_stream, ppmb_ctx **out)
{
    return create_common(1, grid, prec, hip_stream, false, out);
}

ppmb_status ppmb_batch_create(int nbricks, const ppmb_grid *grids, ppmb_precision prec, void *hip_stream,
                              ppmb_ctx **out)
{
    return create_common(nbricks, grids, prec, hip_stream, true, out);
}

ppmb_status ppmb_destroy(ppmb_ctx *c)
{
    if (!c) return PPMB_ERR_INVALID;
    hipStreamSynchronize(c->stream);
    for (auto &t : c->timed) { hipEventDestroy(t.a); hipEventDestroy(t.b); }
    free_graph(c);
    free_maps(c);
    if (c->owns_state) { hipFree(c->buf[0]); hipFree(c->buf[1]); }
    hipFree(c->db);
    hipFree(c->base64);
    hipFree(c->baseT);
    hipFree(c->table);
    hipFree(c->dt);
    hipFree(c->cnt);
    hipFree(c->work);
    hipFree(c->cband);
    hipFree(c->scnt);
    hipFree(c->partials);
    hipFree(c->out8);
    hipFree(c->shell_ws);
    hipFree(c->divbuf);
    hipFree(c->flatbuf);
    delete c;
    return PPMB_OK;
}

ppmb_status ppmb_state_bytes(const ppmb_ctx *c, size_t *bytes, size_t *elem_size)
{
    if (!c || !bytes) return PPMB_ERR_INVALID;
    *bytes = (size_t)c->total_state * c->esz;
    if (elem_size) *elem_size = c->esz;
    return PPMB_OK;
}

ppmb_status ppmb_state_layout(const ppmb_ctx *c, int brick, long long out[4])
{
    if (!c || !out || brick < 0 || brick >= c->nb) return PPMB_ERR_INVALID;
    const Brick &B = c->hb[brick];
    out[0] = B.off;
    out[1] = B.g.fs;
    out[2] = B.g.plane;
    out[3] = B.g.px;
    return PPMB_OK;
}

ppmb_status ppmb_bind_state(ppmb_ctx *c, void *a, void *b)
{
    if (!c) return PPMB_ERR_INVALID;
    if (c->owns_state) return fail(c, PPMB_ERR_INVALID, "bind_state: a batch owns its state arenas");
    if (!a || !b || a == b) return fail(c, PPMB_ERR_INVALID, "bind_state: two distinct device buffers required");
    free_graph(c);
    c->buf[0] = a;
    c->buf[1] = b;
    c->cur = 0;
    c->cfl_ready = false;
    solid_reset(c, 0, c->nb);
    return PPMB_OK;
}

ppmb_status ppmb_current_state(const ppmb_ctx *c, void **dev_state)
{
    if (!c || !dev_state) return PPMB_ERR_INVALID;
    *dev_state = c->buf[c->cur];
    return PPMB_OK;
}

ppmb_status ppmb_brick_set_base_state(ppmb_ctx *c, int brick, int kind, const double params[6])
{
    if (!c) return PPMB_ERR_INVALID;
    if (brick < 0 || brick >= c->nb) return fail(c, PPMB_ERR_INVALID, "brick index out of range");
    const Brick &B = c->hb[brick];
    if (kind < 0 || kind > 3) return fail(c, PPMB_ERR_INVALID, "set_base_state: unknown kind");
    c->cfl_ready = false;
    solid_reset(c, brick, brick + 1);
    if (kind != PPMB_BASE_NONE && !params) return fail(c, PPMB_ERR_INVALID, "set_base_state: params required");
    if (kind == PPMB_BASE_POLY_Z && B.g.grav_kind != PPMB_GRAV_CONST)
        return fail(c, PPMB_ERR_INVALID, "POLY_Z needs constant gravity");
    if (kind == PPMB_BASE_POLY_R && B.g.grav_kind != PPMB_GRAV_RADIAL)
        return fail(c, PPMB_ERR_INVALID, "POLY_R needs radial gravity");
    const bool poly = kind == PPMB_BASE_POLY_Z || kind == PPMB_BASE_POLY_R;
    if (poly && (!(params[0] > 0) || !(params[1] > 0) || !(params[4] > 0) || !(params[5] > params[2])))
        return fail(c, PPMB_ERR_INVALID, "set_base_state: bad polytrope parameters");
    if (poly) {
        double hmax = B.g.dx / 8.0;
        double span = (params[5] - params[2]) / hmax;
        if (span > 1e8) return fail(c, PPMB_ERR_INVALID, "set_base_state: table too long");
        long need = 64 + (long)span + 16;
        if (need > c->table_len) {
            HIPCHK(c, hipStreamSynchronize(c->stream));
            hipFree(c->table);
            c->table = nullptr;
            c->table_len = need;
            if (hipMalloc(&c->table, sizeof(double) * need) != hipSuccess)
                return fail(c, PPMB_ERR_NOMEM, "set_base_state: table allocation");
        }
    }
    double *r0 = c->base64 + B.boff;
    HIPCHK(c, launch_base_state(B.g, kind, params, c->table, c->table_len, r0, r0 + B.g.fs, c->stream));
    if (c->prec == PPMB_FP32)
        HIPCHK(c, launch_narrow<float>(r0, static_cast<float *>(c->baseT) + B.boff, 2 * B.g.fs, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (poly) {
        double nseg = 0;
        HIPCHK(c, hipMemcpy(&nseg, c->table, sizeof(double), hipMemcpyDeviceToHost));
        if (nseg < 1) return fail(c, PPMB_ERR_INVALID, "set_base_state: table overflow");
    }
    return PPMB_OK;
}

ppmb_status ppmb_set_base_state(ppmb_ctx *c, int kind, const double params[6])
{
    return ppmb_brick_set_base_state(c, 0, kind, params);
}

// FP64 device staging of 15 fields for host transfers, freed on return
struct Staging {
    double *p = nullptr;
    ~Staging() { if (p) hipFree(p); }
};

ppmb_status ppmb_brick_get_base(ppmb_ctx *c, int brick, double *host_rho0, double *host_p0)
{
    if (!c || !host_rho0 || !host_p0) return PPMB_ERR_INVALID;
    if (brick < 0 || brick >= c->nb) return fail(c, PPMB_ERR_INVALID, "brick index out of range");
    const Brick &B = c->hb[brick];
    const long n = B.ncell;
    Staging st;
    if (hipMalloc(&st.p, sizeof(double) * 2 * n) != hipSuccess)
        return fail(c, PPMB_ERR_NOMEM, "get_base: staging");
    HIPCHK(c, launch_gather<double>(B.g, 2, c->base64 + B.boff, st.p, c->stream));
    HIPCHK(c, hipMemcpyAsync(host_rho0, st.p, sizeof(double) * n, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(host_p0, st.p + n, sizeof(double) * n, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return PPMB_OK;
}

ppmb_status ppmb_get_base(ppmb_ctx *c, double *host_rho0, double *host_p0)
{
    return ppmb_brick_get_base(c, 0, host_rho0, host_p0);
}

static ppmb_status set_state_dev(ppmb_ctx *c, int brick, const double *const dev_prim[15])
{
    TRY(check_brick(c, brick));
    c->cfl_ready = false;
    solid_reset(c, brick, brick + 1);
    const Brick &B = c->hb[brick];
    for (int q = 0; q < NF; ++q)
        if (!dev_prim[q]) return fail(c, PPMB_ERR_INVALID, "set_state: null field");
    if (c->prec == PPMB_FP64)
        HIPCHK(c, launch_prim_to_cons<double>(B.g, dev_prim, c->base64 + B.boff, arena<double>(c, c->cur) + B.off, c->stream));
    else
        HIPCHK(c, launch_prim_to_cons<float>(B.g, dev_prim, c->base64 + B.boff, arena<float>(c, c->cur) + B.off, c->stream));
    return PPMB_OK;
}

ppmb_status ppmb_set_state_device(ppmb_ctx *c, const double *const dev_prim[15])
{
    if (!c || !dev_prim) return PPMB_ERR_INVALID;
    return set_state_dev(c, 0, dev_prim);
}

// Host transfers go through an FP64 staging buffer of at most kChunk cells
// per field, so that the largest grids need no full-size staging copy.
static const long kChunk = 1L << 24;

// Dense cells [cbeg, cend) of a brick from host arrays holding exactly
// those cells (element c - cbeg), through a staging buffer.
static ppmb_status set_state_cells(ppmb_ctx *c, int brick, long cbeg, long cend, const double *const host_prim[15])
{
    if (!c || !host_prim) return PPMB_ERR_INVALID;
    TRY(check_brick(c, brick));
    c->cfl_ready = false;
    solid_reset(c, brick, brick + 1);
    for (int q = 0; q < NF; ++q)
        if (!host_prim[q]) return fail(c, PPMB_ERR_INVALID, "set_state: null field");
    const Brick &B = c->hb[brick];
    const long n = cend - cbeg, ch = n < kChunk ? n : kChunk;
    Staging st;
    if (hipMalloc(&st.p, sizeof(double) * NF * ch) != hipSuccess)
        return fail(c, PPMB_ERR_NOMEM, "set_state: staging");
    for (long o = 0; o < n; o += ch) {
        const long m = (n - o) < ch ? (n - o) : ch;
        const long c0 = cbeg + o;
        const double *dev[NF];
        for (int q = 0; q < NF; ++q) {
            HIPCHK(c, hipMemcpyAsync(st.p + q * ch, host_prim[q] + o, sizeof(double) * m,
                                     hipMemcpyHostToDevice, c->stream));
            dev[q] = st.p + q * ch;
        }
        if (c->prec == PPMB_FP64)
            HIPCHK(c, launch_prim_to_cons_range<double>(B.g, dev, c->base64 + B.boff,
                                                        arena<double>(c, c->cur) + B.off, c0, m, c->stream));
        else
            HIPCHK(c, launch_prim_to_cons_range<float>(B.g, dev, c->base64 + B.boff,
                                                       arena<float>(c, c->cur) + B.off, c0, m, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    return PPMB_OK;
}

ppmb_status ppmb_brick_set_state(ppmb_ctx *c, int brick, const double *const host_prim[15])
{
    if (!c) return PPMB_ERR_INVALID;
    if (brick < 0 || brick >= c->nb) return fail(c, PPMB_ERR_INVALID, "brick index out of range");
    return set_state_cells(c, brick, 0, c->hb[brick].ncell, host_prim);
}

ppmb_status ppmb_set_state_planes(ppmb_ctx *c, int k0, int nk, const double *const host_prim[15])
{
    if (!c) return PPMB_ERR_INVALID;
    const Geom &g = c->hb[0].g;
    if (k0 < 0 || nk < 1 || k0 + nk > g.n[2]) return fail(c, PPMB_ERR_INVALID, "set_state_planes: planes out of range");
    const long pl = (long)g.n[0] * g.n[1];
    return set_state_cells(c, 0, k0 * pl, (k0 + nk) * pl, host_prim);
}

ppmb_status ppmb_set_state(ppmb_ctx *c, const double *const host_prim[15])
{
    return ppmb_brick_set_state(c, 0, host_prim);
}

static ppmb_status get_state_cells(ppmb_ctx *c, int brick, long cbeg, long cend, double *const host_prim[15])
{
    if (!c || !host_prim) return PPMB_ERR_INVALID;
    TRY(check_brick(c, brick));
    for (int q = 0; q < NF; ++q)
        if (!host_prim[q]) return fail(c, PPMB_ERR_INVALID, "get_state: null field");
    const Brick &B = c->hb[brick];
    const long n = cend - cbeg, ch = n < kChunk ? n : kChunk;
    Staging st;
    if (hipMalloc(&st.p, sizeof(double) * NF * ch) != hipSuccess)
        return fail(c, PPMB_ERR_NOMEM, "get_state: staging");
    for (long o = 0; o < n; o += ch) {
        const long m = (n - o) < ch ? (n - o) : ch;
        const long c0 = cbeg + o;
        if (c->prec == PPMB_FP64)
            HIPCHK(c, launch_cons_to_prim_range<double>(B.g, arena<double>(c, c->cur) + B.off,
                                                        c->base64 + B.boff, st.p, c0, m, ch, c->stream));
        else
            HIPCHK(c, launch_cons_to_prim_range<float>(B.g, arena<float>(c, c->cur) + B.off,
                                                       c->base64 + B.boff, st.p, c0, m, ch, c->stream));
        for (int q = 0; q < NF; ++q)
            HIPCHK(c, hipMemcpyAsync(host_prim[q] + o, st.p + q * ch, sizeof(double) * m,
                                     hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    return PPMB_OK;
}

ppmb_status ppmb_brick_get_state(ppmb_ctx *c, int brick, double *const host_prim[15])
{
    if (!c) return PPMB_ERR_INVALID;
    if (brick < 0 || brick >= c->nb) return fail(c, PPMB_ERR_INVALID, "brick index out of range");
    return get_state_cells(c, brick, 0, c->hb[brick].ncell, host_prim);
}

ppmb_status ppmb_get_state_planes(ppmb_ctx *c, int k0, int nk, double *const host_prim[15])
{
    if (!c) return PPMB_ERR_INVALID;
    const Geom &g = c->hb[0].g;
    if (k0 < 0 || nk < 1 || k0 + nk > g.n[2]) return fail(c, PPMB_ERR_INVALID, "get_state_planes: planes out of range");
    const long pl = (long)g.n[0] * g.n[1];
    return get_state_cells(c, 0, k0 * pl, (k0 + nk) * pl, host_prim);
}

ppmb_status ppmb_get_state(ppmb_ctx *c, double *const host_prim[15])
{
    return ppmb_brick_get_state(c, 0, host_prim);
}

ppmb_status ppmb_brick_get_conserved(ppmb_ctx *c, int brick, double *const host_cons[15])
{
    if (!c || !host_cons) return PPMB_ERR_INVALID;
    TRY(check_brick(c, brick));
    const Brick &B = c->hb[brick];
    const long n = B.ncell;
    Staging st;
    if (hipMalloc(&st.p, sizeof(double) * NF * n) != hipSuccess)
        return fail(c, PPMB_ERR_NOMEM, "get_conserved: staging");
    if (c->prec == PPMB_FP64)
        HIPCHK(c, launch_gather<double>(B.g, NF, arena<double>(c, c->cur) + B.off, st.p, c->stream));
    else
        HIPCHK(c, launch_gather<float>(B.g, NF, arena<float>(c, c->cur) + B.off, st.p, c->stream));
    for (int q = 0; q < NF; ++q) {
        if (!host_cons[q]) return fail(c, PPMB_ERR_INVALID, "get_conserved: null field");
        HIPCHK(c, hipMemcpyAsync(host_cons[q], st.p + q * n, sizeof(double) * n, hipMemcpyDeviceToHost, c->stream));
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return PPMB_OK;
}

ppmb_status ppmb_get_conserved(ppmb_ctx *c, double *const host_cons[15])
{
    return ppmb_brick_get_conserved(c, 0, host_cons);
}

ppmb_status ppmb_set_conserved(ppmb_ctx *c, const double *const host_cons[15])
{
    if (!c || !host_cons) return PPMB_ERR_INVALID;
    TRY(check_brick(c, 0));
    c->cfl_ready = false;
    solid_reset(c, 0, 1);
    const Brick &B = c->hb[0];
    const long n = B.ncell;
    Staging st;
    if (hipMalloc(&st.p, sizeof(double) * NF * n) != hipSuccess)
        return fail(c, PPMB_ERR_NOMEM, "set_conserved: staging");
    for (int q = 0; q < NF; ++q) {
        if (!host_cons[q]) return fail(c, PPMB_ERR_INVALID, "set_conserved: null field");
        HIPCHK(c, hipMemcpyAsync(st.p + q * n, host_cons[q], sizeof(double) * n, hipMemcpyHostToDevice, c->stream));
    }
    if (c->prec == PPMB_FP64)
        HIPCHK(c, launch_scatter<double>(B.g, NF, st.p, arena<double>(c, c->cur) + B.off, c->stream));
    else
        HIPCHK(c, launch_scatter<float>(B.g, NF, st.p, arena<float>(c, c->cur) + B.off, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return PPMB_OK;
}

ppmb_status ppmb_compute_dt(ppmb_ctx *c, double cfl, double *dt_out)
{
    if (!c || !dt_out || !(cfl > 0)) return PPMB_ERR_INVALID;
    TRY(need_state(c));
    TRY(enqueue_cfl(c, cfl, 0, c->nb));
    c->cfl_ready = true;
    TRY(check_flag(c));
    HIPCHK(c, hipMemcpy(dt_out, c->dt, sizeof(double), hipMemcpyDeviceToHost));
    return PPMB_OK;
}

ppmb_status ppmb_step(ppmb_ctx *c, double dt)
{
    if (!c || !(dt > 0) || !std::isfinite(dt)) return PPMB_ERR_INVALID;
    TRY(need_state(c));
    TRY(enqueue_given_dt(c, dt));
    return enqueue_step(c, false, 0.0);
}

ppmb_status ppmb_set_solid_skip(ppmb_ctx *c, int on)
{
    if (!c) return PPMB_ERR_INVALID;
    c->skip_on = on != 0;
    free_graph(c);                       // captured passes hold the previous setting
    return PPMB_OK;
}

ppmb_status ppmb_set_cfl_check(ppmb_ctx *c, double courant_max)
{
    if (!c || !std::isfinite(courant_max) || courant_max < 0.0) return PPMB_ERR_INVALID;
    c->courant_max = courant_max;
    return PPMB_OK;
}

// Rewrite the device brick table from the host copy (after a change of the
// source parameters), with no kernel of the stream reading it.
static ppmb_status upload_bricks(ppmb_ctx *c)
{
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemcpy(c->db, c->hb.data(), sizeof(Brick) * c->nb, hipMemcpyHostToDevice));
    free_graph(c);                       // captured steps hold launch arguments of the old table
    return PPMB_OK;
}

ppmb_status ppmb_set_gravity(ppmb_ctx *c, int kind, const double *params, int nparams)
{
    if (!c) return PPMB_ERR_INVALID;
    const int need = kind == PPMB_GRAV_CONST ? 3 : (kind == PPMB_GRAV_RADIAL ? 4 : 0);
    if (kind < PPMB_GRAV_NONE || kind > PPMB_GRAV_RADIAL || nparams != need || (need && !params))
        return fail(c, PPMB_ERR_INVALID, "set_gravity: unknown kind or wrong parameter count");
    double p[4] = { 0, 0, 0, 0 };
    for (int q = 0; q < need; ++q) p[q] = params[q];
    if (!gravity_ok(kind, p)) return fail(c, PPMB_ERR_INVALID, "set_gravity: bad parameters");
    for (auto &B : c->hb) {
        B.g.grav_kind = kind;
        for (int q = 0; q < 4; ++q) B.g.grav[q] = p[q];
        source_constants(B.g);
    }
    return upload_bricks(c);
}

ppmb_status ppmb_set_heating(ppmb_ctx *c, int kind, const double *params, int nparams)
{
    if (!c) return PPMB_ERR_INVALID;
    const bool count_ok = kind == PPMB_HEAT_LAYER_Z ? nparams == 3
                        : (kind == PPMB_HEAT_BALL ? (nparams == 2 || nparams == 3) : nparams == 0);
    if (kind < PPMB_HEAT_NONE || kind > PPMB_HEAT_BALL || !count_ok || (nparams && !params))
        return fail(c, PPMB_ERR_INVALID, "set_heating: unknown kind or wrong parameter count");
    double p[3] = { 0, 0, 0 };
    for (int q = 0; q < nparams; ++q) p[q] = params[q];
    if (kind == PPMB_HEAT_BALL) p[2] = 0.0;
    if (!heating_ok(kind, p)) return fail(c, PPMB_ERR_INVALID, "set_heating: bad parameters");
    for (auto &B : c->hb) {
        B.g.heat_kind = kind;
        for (int q = 0; q < 3; ++q) B.g.heat[q] = p[q];
        source_constants(B.g);
    }
    return upload_bricks(c);
}

ppmb_status ppmb_step_auto(ppmb_ctx *c, double cfl, int nsteps)
{
    if (!c || !(cfl > 0) || nsteps < 0) return PPMB_ERR_INVALID;
    TRY(need_state(c));
    for (int s = 0; s < nsteps; ++s) TRY(enqueue_step(c, true, cfl));
    return PPMB_OK;
}

// Two steps (an even and an odd pass order) captured once into a hipGraph
// and replayed; recaptured when the arena, the step parity or cfl differ
// from the captured ones.  Steps inside a spin-up ramp are never captured.
static ppmb_status graph_steps(ppmb_ctx *c, double cfl, int nsteps, int how)
{
    // steps of a spin-up ramp differ from one another, and the first step
    // after a state change writes every cell: launched directly
    for (; nsteps > 0 && (c->nstep < c->spin_nramp || !solid_all_same(c, 0, c->nb)); --nsteps)
        TRY(enqueue_step(c, true, cfl, how));
    int pairs = nsteps / 2;
    if (pairs > 0) {
        // the captured steps take dt from the maxima in work[]: make them
        // describe the current state first (with the rotating-frame sources,
        // which change the state after the last pass, every step takes a
        // full reduction instead, captured ones included)
        if (!c->cfl_ready && c->rot_omega == 0.0) {
            TRY(enqueue_cfl(c, cfl, 0, c->nb));
            c->cfl_ready = true;
        }
        if (!c->gexec || c->gkey_cur != c->cur || c->gkey_par != (int)(c->nstep & 1) || c->gkey_cfl != cfl ||
            c->gkey_how != how) {
            free_graph(c);
            const int cur0 = c->cur;
            const long ns0 = c->nstep;
            const unsigned long long st0 = c->steps;
            const bool prof = c->profiling;
            c->profiling = false;
            HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
            ppmb_status s = enqueue_step(c, true, cfl, how);
            if (s == PPMB_OK) s = enqueue_step(c, true, cfl, how);
            hipError_t e = hipStreamEndCapture(c->stream, &c->graph);
            c->profiling = prof;
            c->cur = cur0;
            c->nstep = ns0;
            c->steps = st0;
            if (s != PPMB_OK) return s;
            HIPCHK(c, e);
            HIPCHK(c, hipGraphInstantiate(&c->gexec, c->graph, nullptr, nullptr, 0));
            c->gkey_cur = cur0;
            c->gkey_par = (int)(ns0 & 1);
            c->gkey_cfl = cfl;
            c->gkey_how = how;
        }
        for (int p = 0; p < pairs; ++p) {
            HIPCHK(c, hipGraphLaunch(c->gexec, c->stream));
            c->nstep += 2;
            c->steps += 2;
        }
    }
    if (nsteps % 2) TRY(enqueue_step(c, true, cfl, how));
    return PPMB_OK;
}

ppmb_status ppmb_batch_step(ppmb_ctx *c, double cfl, int nsteps, int mode)
{
    if (!c || !(cfl > 0) || nsteps < 0 || mode < 0 || mode > 4) return PPMB_ERR_INVALID;
    // The persistent step kernel (modes 3 and 4) is switched off: its
    // launches did not complete on the target GPU and the cause is not
    // known yet, so nothing launches it until that cause is found.
    if ((mode == 3 || mode == 4) && !kPersistentStepOn)
        return fail(c, PPMB_ERR_INVALID, "persistent step (modes 3, 4) is switched off: its launches did not "
                                         "complete on the target GPU; use mode 0 or 1");
    TRY(need_state(c));
    if (mode == 1) return graph_steps(c, cfl, nsteps, kBatched);
    if (mode == 4) return graph_steps(c, cfl, nsteps, kPersistent);
    const int how = mode == 2 ? kPerBrick : (mode == 3 ? kPersistent : kBatched);
    for (int s = 0; s < nsteps; ++s) TRY(enqueue_step(c, true, cfl, how));
    return PPMB_OK;
}

ppmb_status ppmb_brick_last_dt(ppmb_ctx *c, int brick, double *dt_out)
{
    if (!c || !dt_out) return PPMB_ERR_INVALID;
    if (brick < 0 || brick >= c->nb) return fail(c, PPMB_ERR_INVALID, "brick index out of range");
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemcpy(dt_out, c->dt + brick, sizeof(double), hipMemcpyDeviceToHost));
    return check_flag(c);
}

ppmb_status ppmb_last_dt(ppmb_ctx *c, double *dt_out) { return ppmb_brick_last_dt(c, 0, dt_out); }

ppmb_status ppmb_pass(ppmb_ctx *c, int axis, double dt, int heat)
{
    if (!c || axis < 0 || axis > 2 || !(dt > 0) || !std::isfinite(dt)) return PPMB_ERR_INVALID;
    TRY(need_state(c));
    TRY(enqueue_given_dt(c, dt));
    if (c->dissk > 0.0) TRY(enqueue_divergence(c, 0, c->nb, c->cur));
    TRY(enqueue_pass(c, axis, heat ? (any_heat(c) ? 1 : 0) : 0, 0, c->nb, c->cur));
    c->cur = 1 - c->cur;
    c->cfl_ready = false;
    return PPMB_OK;
}

ppmb_status ppmb_get_nstep(const ppmb_ctx *c, long *nstep)
{
    if (!c || !nstep) return PPMB_ERR_INVALID;
    *nstep = c->nstep;
    return PPMB_OK;
}

ppmb_status ppmb_set_nstep(ppmb_ctx *c, long nstep)
{
    if (!c || nstep < 0) return PPMB_ERR_INVALID;
    c->nstep = nstep;
    return PPMB_OK;
}

ppmb_status ppmb_brick_totals(ppmb_ctx *c, int brick, double out[8])
{
    if (!c || !out) return PPMB_ERR_INVALID;
    TRY(check_brick(c, brick));
    const Brick &B = c->hb[brick];
    if (c->prec == PPMB_FP64)
        HIPCHK(c, launch_totals<double>(B.g, arena<double>(c, c->cur) + B.off, c->base64 + B.boff,
                                        c->base64 + B.boff + B.g.fs, c->partials, c->out8, c->stream));
    else
        HIPCHK(c, launch_totals<float>(B.g, arena<float>(c, c->cur) + B.off, c->base64 + B.boff,
                                       c->base64 + B.boff + B.g.fs, c->partials, c->out8, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemcpy(out, c->out8, sizeof(double) * 8, hipMemcpyDeviceToHost));
    return check_flag(c);
}

ppmb_status ppmb_reduce_totals(ppmb_ctx *c, double out[8]) { return ppmb_brick_totals(c, 0, out); }

ppmb_status ppmb_set_shock_dissipation(ppmb_ctx *c, double k)
{
    if (!c || !std::isfinite(k) || k < 0.0) return PPMB_ERR_INVALID;
    if (k > 0.0 && !c->divbuf) {
        const size_t bytes = (size_t)(c->total_base / 2) * c->esz;
        if (hipMalloc(&c->divbuf, bytes) != hipSuccess) {
            c->divbuf = nullptr;
            return fail(c, PPMB_ERR_NOMEM, "divergence field");
        }
        // cells the divergence kernel leaves out (solid, skipped) hold a
        // finite value from the start
        HIPCHK(c, hipMemsetAsync(c->divbuf, 0, bytes, c->stream));
    }
    c->dissk = k;
    free_graph(c);                       // captured steps hold the previous setting
    return PPMB_OK;
}

ppmb_status ppmb_set_flattening(ppmb_ctx *c, int on)
{
    if (!c) return PPMB_ERR_INVALID;
    if (on && !c->flatbuf) {
        const size_t bytes = (size_t)(c->total_base / 2) * c->esz;
        if (hipMalloc(&c->flatbuf, bytes) != hipSuccess) {
            c->flatbuf = nullptr;
            return fail(c, PPMB_ERR_NOMEM, "flattening field");
        }
        // cells the flattening kernels leave out (solid, skipped) hold a
        // coefficient in [0, 1] from the start
        HIPCHK(c, hipMemsetAsync(c->flatbuf, 0, bytes, c->stream));
    }
    c->flat_on = on != 0;
    free_graph(c);                       // captured steps hold the previous setting
    return PPMB_OK;
}

ppmb_status ppmb_set_spinup(ppmb_ctx *c, double omega, long nramp)
{
    if (!c || !std::isfinite(omega) || nramp < 0) return PPMB_ERR_INVALID;
    c->spin_omega = omega;
    c->spin_nramp = (omega != 0.0 && nramp > 0) ? nramp : 0;
    return PPMB_OK;
}

ppmb_status ppmb_set_rotating_frame(ppmb_ctx *c, double omega, int centrifugal)
{
    if (!c || !std::isfinite(omega)) return PPMB_ERR_INVALID;
    c->rot_omega = omega;
    c->rot_centrifugal = centrifugal ? 1 : 0;
    free_graph(c);                       // captured steps hold the previous setting
    return PPMB_OK;
}

ppmb_status ppmb_spin_add(ppmb_ctx *c, double domega)
{
    if (!c || !std::isfinite(domega)) return PPMB_ERR_INVALID;
    TRY(need_state(c));
    return enqueue_spin(c, domega);
}

ppmb_status ppmb_shell_profile(ppmb_ctx *c, int brick, int nbins, double dr, double *out)
{
    if (!c || !out || nbins < 1 || nbins > kShellMaxBins || !(dr > 0) || !std::isfinite(dr))
        return PPMB_ERR_INVALID;
    if (!((double)nbins * dr < 1e300)) return PPMB_ERR_INVALID;
    TRY(check_brick(c, brick));
    const Brick &B = c->hb[brick];
    const long nwork = shell_work_doubles(B.g, nbins);
    const size_t need = sizeof(double) * ((size_t)nwork + 8 * (size_t)nbins);
    if (need > c->shell_ws_bytes) {
        HIPCHK(c, hipStreamSynchronize(c->stream));
        hipFree(c->shell_ws);
        c->shell_ws = nullptr;
        c->shell_ws_bytes = 0;
        if (hipMalloc(&c->shell_ws, need) != hipSuccess) {
            c->shell_ws = nullptr;
            return fail(c, PPMB_ERR_NOMEM, "shell-sum workspace");
        }
        c->shell_ws_bytes = need;
    }
    double *res = c->shell_ws + nwork;
    if (c->prec == PPMB_FP64)
        HIPCHK(c, launch_shell<double>(B.g, arena<double>(c, c->cur) + B.off, c->base64 + B.boff, nbins, dr,
                                       c->shell_ws, res, c->stream));
    else
        HIPCHK(c, launch_shell<float>(B.g, arena<float>(c, c->cur) + B.off, c->base64 + B.boff, nbins, dr,
                                      c->shell_ws, res, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemcpy(out, res, sizeof(double) * 8 * nbins, hipMemcpyDeviceToHost));
    return PPMB_OK;
}

ppmb_status ppmb_shell_profile_noalloc(ppmb_ctx *c, int brick, int nbins, double dr, double *dev_out)
{
    if (!c || !dev_out || nbins < 1 || nbins > kShellMaxBins || !(dr > 0) || !std::isfinite(dr))
        return PPMB_ERR_INVALID;
    if (!((double)nbins * dr < 1e300)) return PPMB_ERR_INVALID;
    TRY(check_brick(c, brick));
    const Brick &B = c->hb[brick];
    const long nwork = shell_work_doubles(B.g, nbins);
    if (nwork > kShellStaticDoubles)
        return fail(c, PPMB_ERR_INVALID, "shell_profile_noalloc: block partials of " + std::to_string(nwork) +
                                             " doubles exceed the static workspace of " +
                                             std::to_string(kShellStaticDoubles));
    // every element of the workspace the kernels read is written first by
    // the same call: nothing to clear
    if (c->prec == PPMB_FP64)
        HIPCHK(c, launch_shell<double>(B.g, arena<double>(c, c->cur) + B.off, c->base64 + B.boff, nbins, dr,
                                       c->noalloc_ws, dev_out, c->stream));
    else
        HIPCHK(c, launch_shell<float>(B.g, arena<float>(c, c->cur) + B.off, c->base64 + B.boff, nbins, dr,
                                      c->noalloc_ws, dev_out, c->stream));
    return PPMB_OK;
}

ppmb_status ppmb_counters(ppmb_ctx *c, unsigned long long out[4])
{
    if (!c || !out) return PPMB_ERR_INVALID;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    std::vector<unsigned long long> w(kCntWords);
    HIPCHK(c, hipMemcpy(w.data(), c->cnt, sizeof(unsigned long long) * kCntWords, hipMemcpyDeviceToHost));
    for (int q = 0; q < 3; ++q) {
        out[q] = 0;
        for (int s = 0; s < kCntSlots; ++s) out[q] += w[s * kCntStride + q];
    }
    out[3] = c->steps;
    return check_flag(c);
}

ppmb_status ppmb_set_pass_shape(ppmb_ctx *c, int march_waves, int x_waves)
{
    if (!c) return PPMB_ERR_INVALID;
    auto ok = [](int w) { return w == 1 || w == 2 || w == 4; };
    if (!ok(march_waves) || !ok(x_waves)) return fail(c, PPMB_ERR_INVALID, "pass shape: waves per block must be 1, 2 or 4");
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->shape.march_waves = march_waves;
    c->shape.x_waves = x_waves;
    return build_maps(c);
}

ppmb_status ppmb_set_pass_tiling(ppmb_ctx *c, int march_chunk, int x_rows)
{
    if (!c) return PPMB_ERR_INVALID;
    if (march_chunk < 0 || (march_chunk > 0 && march_chunk < 16) || x_rows < 0 || x_rows > 64)
        return fail(c, PPMB_ERR_INVALID, "pass tiling: chunk 0 or >= 16 cells, 0..64 rows per wave");
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->shape.march_chunk = march_chunk;
    c->shape.x_rows = x_rows;
    return build_maps(c);
}

ppmb_status ppmb_get_pass_tiling(const ppmb_ctx *c, int *march_chunk, int *x_rows)
{
    if (!c || !march_chunk || !x_rows) return PPMB_ERR_INVALID;
    *march_chunk = c->shape.march_chunk;
    *x_rows = c->shape.x_rows;
    return PPMB_OK;
}

ppmb_status ppmb_get_pass_shape(const ppmb_ctx *c, int *march_waves, int *x_waves)
{
    if (!c || !march_waves || !x_waves) return PPMB_ERR_INVALID;
    *march_waves = c->shape.march_waves;
    *x_waves = c->shape.x_waves;
    return PPMB_OK;
}

ppmb_status ppmb_brick_count(const ppmb_ctx *c, int *nbricks)
{
    if (!c || !nbricks) return PPMB_ERR_INVALID;
    *nbricks = c->nb;
    return PPMB_OK;
}

static std::string tune_key(const ppmb_ctx *c)
{
    long cells = 0;
    for (auto &B : c->hb) cells += B.ncell;
    char k[128];
    snprintf(k, sizeof k, "gfx950 %s bricks=%d cells=%ld", c->prec == PPMB_FP64 ? "fp64" : "fp32", c->nb, cells);
    return k;
}

// Time `reps` passes along the given axes with the current shape (after one
// untimed pass), reading the current state and writing the spare arena.
static ppmb_status time_passes(ppmb_ctx *c, const int *axes, int naxes, int reps, hipEvent_t e0, hipEvent_t e1,
                               float *ms)
{
    *ms = 0.f;
    for (int a = 0; a < naxes; ++a) {
        TRY(enqueue_pass(c, axes[a], 0, 0, c->nb, c->cur));          // warm-up
        HIPCHK(c, hipEventRecord(e0, c->stream));
        for (int r = 0; r < reps; ++r) TRY(enqueue_pass(c, axes[a], 0, 0, c->nb, c->cur));
        HIPCHK(c, hipEventRecord(e1, c->stream));
        HIPCHK(c, hipEventSynchronize(e1));
        float t = 0.f;
        HIPCHK(c, hipEventElapsedTime(&t, e0, e1));
        *ms += t;
    }
    return PPMB_OK;
}

static ppmb_status set_shape(ppmb_ctx *c, const PassShape &sh)
{
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->shape = sh;
    return build_maps(c);
}

ppmb_status ppmb_autotune(ppmb_ctx *c, double cfl, int reps, const char *cache_path, int out_shape[2])
{
    if (!c || !out_shape || !(cfl > 0) || reps < 1) return PPMB_ERR_INVALID;
    TRY(need_state(c));
    const std::string key = tune_key(c);
    if (cache_path) {
        FILE *f = fopen(cache_path, "r");
        if (f) {
            char line[256];
            int mw = 0, xw = 0, ck = 0, xr = 0;
            while (fgets(line, sizeof line, f)) {
                char kbuf[200];
                if (sscanf(line, "%199[^|]| %d %d %d %d", kbuf, &mw, &xw, &ck, &xr) == 5 && key == std::string(kbuf)) {
                    fclose(f);
                    TRY(ppmb_set_pass_shape(c, mw, xw));
                    TRY(ppmb_set_pass_tiling(c, ck, xr));
                    out_shape[0] = mw;
                    out_shape[1] = xw;
                    return PPMB_OK;
                }
            }
            fclose(f);
        }
    }
    std::vector<unsigned long long> saved(kCntWords);
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemcpy(saved.data(), c->cnt, sizeof(unsigned long long) * kCntWords, hipMemcpyDeviceToHost));
    TRY(enqueue_cfl(c, cfl, 0, c->nb));
    c->cfl_ready = true;                 // the passes below leave the state as it is
    TRY(check_flag(c));
    const bool prof = c->profiling;
    c->profiling = false;
    hipEvent_t e0, e1;
    HIPCHK(c, hipEventCreate(&e0));
    HIPCHK(c, hipEventCreate(&e1));
    ppmb_status st = PPMB_OK;
    PassShape best = c->shape;
    // the marching kernel (y and z passes): waves per block and chunk length
    const int waves[3] = { 1, 2, 4 };
    const int chunks[3] = { 0, 128, 256 };
    const int yz[2] = { 1, 2 };
    float best_m = 1e30f;
    for (int w = 0; w < 3 && st == PPMB_OK; ++w)
        for (int k = 0; k < 3 && st == PPMB_OK; ++k) {
            PassShape sh = best;
            sh.march_waves = waves[w];
            sh.march_chunk = chunks[k];
            float t = 0.f;
            st = set_shape(c, sh);
            if (st == PPMB_OK) st = time_passes(c, yz, 2, reps, e0, e1, &t);
            if (st == PPMB_OK && t < best_m) { best_m = t; best.march_waves = sh.march_waves; best.march_chunk = sh.march_chunk; }
        }
    // the x pass: the lanes-along-x kernel (waves per block, rows per wave)
    // or the marching kernel with the shape just chosen
    const int rows[4] = { 0, 1, 2, 4 };
    const int xa[1] = { 0 };
    float best_x = 1e30f;
    for (int w = 0; w < 3 && st == PPMB_OK; ++w)
        for (int r = 0; r < 4 && st == PPMB_OK; ++r) {
            if (rows[r] == 0 && w > 0) continue;      // x_waves plays no part then
            PassShape sh = best;
            sh.x_waves = waves[w];
            sh.x_rows = rows[r];
            float t = 0.f;
            st = set_shape(c, sh);
            if (st == PPMB_OK) st = time_passes(c, xa, 1, reps, e0, e1, &t);
            if (st == PPMB_OK && t < best_x) { best_x = t; best.x_waves = sh.x_waves; best.x_rows = sh.x_rows; }
        }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    c->profiling = prof;
    if (st != PPMB_OK) return st;
    HIPCHK(c, hipMemcpy(c->cnt, saved.data(), sizeof(unsigned long long) * kCntWords, hipMemcpyHostToDevice));
    TRY(set_shape(c, best));
    out_shape[0] = best.march_waves;
    out_shape[1] = best.x_waves;
    if (cache_path) {
        FILE *f = fopen(cache_path, "a");
        if (f) {
            fprintf(f, "%s| %d %d %d %d\n", key.c_str(), best.march_waves, best.x_waves, best.march_chunk, best.x_rows);
            fclose(f);
        }
    }
    return PPMB_OK;
}

ppmb_status ppmb_profile_enable(ppmb_ctx *c, int enable)
{
    if (!c) return PPMB_ERR_INVALID;
    c->profiling = enable != 0;
    return PPMB_OK;
}

ppmb_status ppmb_profile_read(ppmb_ctx *c, double ms[3], long count[3])
{
    if (!c || !ms || !count) return PPMB_ERR_INVALID;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (int d = 0; d < 3; ++d) { ms[d] = 0.0; count[d] = 0; }
    ppmb_status st = PPMB_OK;
    for (auto &t : c->timed) {
        float v = 0.f;
        if (st == PPMB_OK && hipEventElapsedTime(&v, t.a, t.b) == hipSuccess) {
            ms[t.axis] += v;
            count[t.axis] += 1;
        } else {
            st = fail(c, PPMB_ERR_HIP, "profile_read: event timing failed");
        }
        hipEventDestroy(t.a);
        hipEventDestroy(t.b);
    }
    c->timed.clear();
    return st;
}

ppmb_status ppmb_synchronize(ppmb_ctx *c)
{
    if (!c) return PPMB_ERR_INVALID;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return check_flag(c);
}

}  // extern "C"
