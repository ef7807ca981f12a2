// ppmb_api.hip -- host runtime behind the C ABI declared in include/ppmb.h.
//
// A context owns the FP64 base state, its working-precision copy, the
// reduction buffers and the event counters; the two state buffers are the
// caller's.  Every call enqueues on the context's stream.
#include "../../include/ppmb.h"
#include "ppmb_internal.h"

#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

using namespace ppmb;

struct ppmb_ctx {
    Geom g{};
    ppmb_precision prec = PPMB_FP64;
    hipStream_t stream = nullptr;
    long ncell = 0;
    size_t esz = 8;
    void *buf[2] = { nullptr, nullptr };
    int cur = 0;
    double *base64 = nullptr;       // rho0, p0 (FP64)
    void *baseT = nullptr;          // rho0, p0 in the working precision (FP32 only)
    double *table = nullptr;        // base-state RK4 nodes
    long table_len = 0;
    double *dt_dev = nullptr;       // [0] current dt
    unsigned long long *cnt = nullptr;    // [0..2] event counters, [3] unused
    unsigned long long *work = nullptr;   // [0] smax bits, [1] non-physical flag
    double *partials = nullptr;     // totals block partials
    double *out8 = nullptr;         // totals result
    long nstep = 0;
    unsigned long long steps = 0;
    bool base_set = false;
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

template <typename T>
static T *cur_state(ppmb_ctx *c) { return static_cast<T *>(c->buf[c->cur]); }

static const void *base_rho(ppmb_ctx *c)
{
    return c->prec == PPMB_FP64 ? (const void *)c->base64 : c->baseT;
}
static const void *base_p(ppmb_ctx *c)
{
    return c->prec == PPMB_FP64 ? (const void *)(c->base64 + c->ncell)
                                : (const void *)((const float *)c->baseT + c->ncell);
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
    case PPMB_ERR_UNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

const char *ppmb_last_error(const ppmb_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

ppmb_status ppmb_create(const ppmb_grid *grid, ppmb_precision prec, void *hip_stream, ppmb_ctx **out)
{
    if (!grid || !out) return PPMB_ERR_INVALID;
    *out = nullptr;
    for (int d = 0; d < 3; ++d) {
        if (grid->n[d] < 1) return PPMB_ERR_INVALID;
        if (grid->bc[d] != PPMB_BC_PERIODIC && grid->bc[d] != PPMB_BC_REFLECT) return PPMB_ERR_INVALID;
    }
    if (!(grid->dx > 0.0) || !(grid->gamma > 1.0)) return PPMB_ERR_INVALID;
    if (prec != PPMB_FP64 && prec != PPMB_FP32) return PPMB_ERR_INVALID;
    if (grid->grav_kind < 0 || grid->grav_kind > 2 || grid->heat_kind < 0 || grid->heat_kind > 2)
        return PPMB_ERR_INVALID;
    long nc = (long)grid->n[0] * grid->n[1] * grid->n[2];
    if (nc > (1L << 34)) return PPMB_ERR_INVALID;
    ppmb_ctx *c = new ppmb_ctx();
    Geom &g = c->g;
    for (int d = 0; d < 3; ++d) { g.n[d] = grid->n[d]; g.origin[d] = grid->origin[d]; g.bc[d] = grid->bc[d]; }
    g.dx = grid->dx;
    g.gamma = grid->gamma;
    g.sphere = grid->sphere;
    g.sphere_r = grid->sphere_r;
    g.grav_kind = grid->grav_kind;
    for (int q = 0; q < 4; ++q) g.grav[q] = grid->grav[q];
    g.heat_kind = grid->heat_kind;
    for (int q = 0; q < 3; ++q) g.heat[q] = grid->heat[q];
    g.smooth_detect = grid->smooth_detect;
    c->prec = prec;
    c->stream = static_cast<hipStream_t>(hip_stream);
    c->ncell = nc;
    c->esz = prec == PPMB_FP64 ? 8 : 4;
    // base-state table: at most (span / (dx/8)) + 2 nodes per segment
    double span = 4.0 * (grid->n[0] + grid->n[1] + grid->n[2]) * grid->dx + 16.0;
    c->table_len = 64 + (long)(span / (grid->dx / 8.0)) * 2 + 64;
    hipError_t e = hipMalloc(&c->base64, sizeof(double) * 2 * nc);
    if (e == hipSuccess && prec == PPMB_FP32) e = hipMalloc(&c->baseT, sizeof(float) * 2 * nc);
    if (e == hipSuccess) e = hipMalloc(&c->table, sizeof(double) * c->table_len);
    if (e == hipSuccess) e = hipMalloc(&c->dt_dev, sizeof(double) * 2);
    if (e == hipSuccess) e = hipMalloc(&c->cnt, sizeof(unsigned long long) * 4);
    if (e == hipSuccess) e = hipMalloc(&c->work, sizeof(unsigned long long) * 2);
    if (e == hipSuccess) e = hipMalloc(&c->partials, sizeof(double) * 8 * kTotalsBlocks);
    if (e == hipSuccess) e = hipMalloc(&c->out8, sizeof(double) * 8);
    if (e != hipSuccess) {
        ppmb_destroy(c);
        return PPMB_ERR_NOMEM;
    }
    if (launch_zero_u64(c->cnt, 4, c->stream) != hipSuccess || launch_zero_u64(c->work, 2, c->stream) != hipSuccess) {
        ppmb_destroy(c);
        return PPMB_ERR_HIP;
    }
    // base state NONE until set
    double zero[6] = { 0, 0, 0, 0, 0, 0 };
    if (launch_base_state(g, PPMB_BASE_NONE, zero, c->table, c->table_len, c->base64, c->base64 + nc, c->stream) != hipSuccess) {
        ppmb_destroy(c);
        return PPMB_ERR_HIP;
    }
    if (prec == PPMB_FP32 &&
        launch_narrow<float>(c->base64, static_cast<float *>(c->baseT), 2 * nc, c->stream) != hipSuccess) {
        ppmb_destroy(c);
        return PPMB_ERR_HIP;
    }
    *out = c;
    return PPMB_OK;
}

ppmb_status ppmb_destroy(ppmb_ctx *c)
{
    if (!c) return PPMB_ERR_INVALID;
    hipStreamSynchronize(c->stream);
    hipFree(c->base64);
    hipFree(c->baseT);
    hipFree(c->table);
    hipFree(c->dt_dev);
    hipFree(c->cnt);
    hipFree(c->work);
    hipFree(c->partials);
    hipFree(c->out8);
    delete c;
    return PPMB_OK;
}

ppmb_status ppmb_state_bytes(const ppmb_ctx *c, size_t *bytes, size_t *elem_size)
{
    if (!c || !bytes) return PPMB_ERR_INVALID;
    *bytes = (size_t)NF * c->ncell * c->esz;
    if (elem_size) *elem_size = c->esz;
    return PPMB_OK;
}

ppmb_status ppmb_bind_state(ppmb_ctx *c, void *a, void *b)
{
    if (!c) return PPMB_ERR_INVALID;
    if (!a || !b || a == b) return fail(c, PPMB_ERR_INVALID, "bind_state: two distinct device buffers required");
    c->buf[0] = a;
    c->buf[1] = b;
    c->cur = 0;
    return PPMB_OK;
}

ppmb_status ppmb_current_state(const ppmb_ctx *c, void **dev_state)
{
    if (!c || !dev_state) return PPMB_ERR_INVALID;
    *dev_state = c->buf[c->cur];
    return PPMB_OK;
}

ppmb_status ppmb_set_base_state(ppmb_ctx *c, int kind, const double params[6])
{
    if (!c) return PPMB_ERR_INVALID;
    if (kind < 0 || kind > 3) return fail(c, PPMB_ERR_INVALID, "set_base_state: unknown kind");
    if (kind != PPMB_BASE_NONE && !params) return fail(c, PPMB_ERR_INVALID, "set_base_state: params required");
    if (kind == PPMB_BASE_POLY_Z && c->g.grav_kind != PPMB_GRAV_CONST)
        return fail(c, PPMB_ERR_INVALID, "POLY_Z needs constant gravity");
    if (kind == PPMB_BASE_POLY_R && c->g.grav_kind != PPMB_GRAV_RADIAL)
        return fail(c, PPMB_ERR_INVALID, "POLY_R needs radial gravity");
    if ((kind == PPMB_BASE_POLY_Z || kind == PPMB_BASE_POLY_R) &&
        (!(params[0] > 0) || !(params[1] > 0) || !(params[4] > 0) || !(params[5] > params[2])))
        return fail(c, PPMB_ERR_INVALID, "set_base_state: bad polytrope parameters");
    if (kind == PPMB_BASE_POLY_Z || kind == PPMB_BASE_POLY_R) {
        double hmax = c->g.dx / 8.0;
        long need = 64 + (long)((params[5] - params[2]) / hmax) + 16;
        if (need > c->table_len) {
            hipFree(c->table);
            c->table = nullptr;
            c->table_len = need;
            if (hipMalloc(&c->table, sizeof(double) * need) != hipSuccess)
                return fail(c, PPMB_ERR_NOMEM, "set_base_state: table allocation");
        }
    }
    HIPCHK(c, launch_base_state(c->g, kind, params, c->table, c->table_len, c->base64,
                                c->base64 + c->ncell, c->stream));
    if (c->prec == PPMB_FP32)
        HIPCHK(c, launch_narrow<float>(c->base64, static_cast<float *>(c->baseT), 2 * c->ncell, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (kind == PPMB_BASE_POLY_Z || kind == PPMB_BASE_POLY_R) {
        double nseg = 0;
        HIPCHK(c, hipMemcpy(&nseg, c->table, sizeof(double), hipMemcpyDeviceToHost));
        if (nseg < 1) return fail(c, PPMB_ERR_INVALID, "set_base_state: table overflow");
    }
    c->base_set = true;
    return PPMB_OK;
}

ppmb_status ppmb_get_base(ppmb_ctx *c, double *host_rho0, double *host_p0)
{
    if (!c || !host_rho0 || !host_p0) return PPMB_ERR_INVALID;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemcpy(host_rho0, c->base64, sizeof(double) * c->ncell, hipMemcpyDeviceToHost));
    HIPCHK(c, hipMemcpy(host_p0, c->base64 + c->ncell, sizeof(double) * c->ncell, hipMemcpyDeviceToHost));
    return PPMB_OK;
}

static ppmb_status need_state(ppmb_ctx *c)
{
    if (!c->buf[0] || !c->buf[1]) return fail(c, PPMB_ERR_INVALID, "state buffers not bound");
    return PPMB_OK;
}

ppmb_status ppmb_set_state_device(ppmb_ctx *c, const double *const dev_prim[15])
{
    if (!c || !dev_prim) return PPMB_ERR_INVALID;
    if (need_state(c) != PPMB_OK) return PPMB_ERR_INVALID;
    for (int q = 0; q < NF; ++q)
        if (!dev_prim[q]) return fail(c, PPMB_ERR_INVALID, "set_state: null field");
    if (c->prec == PPMB_FP64)
        HIPCHK(c, launch_prim_to_cons<double>(c->g, dev_prim, c->base64, cur_state<double>(c), c->stream));
    else
        HIPCHK(c, launch_prim_to_cons<float>(c->g, dev_prim, c->base64, cur_state<float>(c), c->stream));
    return PPMB_OK;
}

// FP64 device staging of 15 fields for host transfers, freed on return
struct Staging {
    double *p = nullptr;
    ~Staging() { if (p) hipFree(p); }
};

ppmb_status ppmb_set_state(ppmb_ctx *c, const double *const host_prim[15])
{
    if (!c || !host_prim) return PPMB_ERR_INVALID;
    if (need_state(c) != PPMB_OK) return PPMB_ERR_INVALID;
    Staging st;
    if (hipMalloc(&st.p, sizeof(double) * NF * c->ncell) != hipSuccess)
        return fail(c, PPMB_ERR_NOMEM, "set_state: staging");
    const double *dev[NF];
    for (int q = 0; q < NF; ++q) {
        if (!host_prim[q]) return fail(c, PPMB_ERR_INVALID, "set_state: null field");
        HIPCHK(c, hipMemcpyAsync(st.p + q * c->ncell, host_prim[q], sizeof(double) * c->ncell,
                                 hipMemcpyHostToDevice, c->stream));
        dev[q] = st.p + q * c->ncell;
    }
    ppmb_status s = ppmb_set_state_device(c, dev);
    if (s != PPMB_OK) return s;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return PPMB_OK;
}

ppmb_status ppmb_get_state(ppmb_ctx *c, double *const host_prim[15])
{
    if (!c || !host_prim) return PPMB_ERR_INVALID;
    if (need_state(c) != PPMB_OK) return PPMB_ERR_INVALID;
    Staging st;
    if (hipMalloc(&st.p, sizeof(double) * NF * c->ncell) != hipSuccess)
        return fail(c, PPMB_ERR_NOMEM, "get_state: staging");
    if (c->prec == PPMB_FP64)
        HIPCHK(c, launch_cons_to_prim<double>(c->g, cur_state<double>(c), c->base64, st.p, c->stream));
    else
        HIPCHK(c, launch_cons_to_prim<float>(c->g, cur_state<float>(c), c->base64, st.p, c->stream));
    for (int q = 0; q < NF; ++q) {
        if (!host_prim[q]) return fail(c, PPMB_ERR_INVALID, "get_state: null field");
        HIPCHK(c, hipMemcpyAsync(host_prim[q], st.p + q * c->ncell, sizeof(double) * c->ncell,
                                 hipMemcpyDeviceToHost, c->stream));
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return PPMB_OK;
}

ppmb_status ppmb_get_conserved(ppmb_ctx *c, double *const host_cons[15])
{
    if (!c || !host_cons) return PPMB_ERR_INVALID;
    if (need_state(c) != PPMB_OK) return PPMB_ERR_INVALID;
    Staging st;
    if (hipMalloc(&st.p, sizeof(double) * NF * c->ncell) != hipSuccess)
        return fail(c, PPMB_ERR_NOMEM, "get_conserved: staging");
    if (c->prec == PPMB_FP64)
        HIPCHK(c, launch_widen<double>(cur_state<double>(c), st.p, NF * c->ncell, c->stream));
    else
        HIPCHK(c, launch_widen<float>(cur_state<float>(c), st.p, NF * c->ncell, c->stream));
    for (int q = 0; q < NF; ++q) {
        if (!host_cons[q]) return fail(c, PPMB_ERR_INVALID, "get_conserved: null field");
        HIPCHK(c, hipMemcpyAsync(host_cons[q], st.p + q * c->ncell, sizeof(double) * c->ncell,
                                 hipMemcpyDeviceToHost, c->stream));
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return PPMB_OK;
}

ppmb_status ppmb_set_conserved(ppmb_ctx *c, const double *const host_cons[15])
{
    if (!c || !host_cons) return PPMB_ERR_INVALID;
    if (need_state(c) != PPMB_OK) return PPMB_ERR_INVALID;
    Staging st;
    if (hipMalloc(&st.p, sizeof(double) * NF * c->ncell) != hipSuccess)
        return fail(c, PPMB_ERR_NOMEM, "set_conserved: staging");
    for (int q = 0; q < NF; ++q) {
        if (!host_cons[q]) return fail(c, PPMB_ERR_INVALID, "set_conserved: null field");
        HIPCHK(c, hipMemcpyAsync(st.p + q * c->ncell, host_cons[q], sizeof(double) * c->ncell,
                                 hipMemcpyHostToDevice, c->stream));
    }
    if (c->prec == PPMB_FP64)
        HIPCHK(c, launch_narrow<double>(st.p, cur_state<double>(c), NF * c->ncell, c->stream));
    else
        HIPCHK(c, launch_narrow<float>(st.p, cur_state<float>(c), NF * c->ncell, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return PPMB_OK;
}

static ppmb_status enqueue_cfl(ppmb_ctx *c, double cfl)
{
    if (c->prec == PPMB_FP64)
        HIPCHK(c, launch_cfl<double>(c->g, cur_state<double>(c), c->base64, c->base64 + c->ncell,
                                     c->work, cfl, c->dt_dev, c->stream));
    else
        HIPCHK(c, launch_cfl<float>(c->g, cur_state<float>(c), c->base64, c->base64 + c->ncell,
                                    c->work, cfl, c->dt_dev, c->stream));
    return PPMB_OK;
}

static ppmb_status check_flag(ppmb_ctx *c)
{
    unsigned long long w[2];
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemcpy(w, c->work, sizeof(w), hipMemcpyDeviceToHost));
    if (w[1]) {
        HIPCHK(c, launch_zero_u64(c->work + 1, 1, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        return fail(c, PPMB_ERR_NONPHYSICAL, "non-positive density or pressure, or NaN, in a fluid cell");
    }
    return PPMB_OK;
}

ppmb_status ppmb_compute_dt(ppmb_ctx *c, double cfl, double *dt_out)
{
    if (!c || !dt_out || !(cfl > 0)) return PPMB_ERR_INVALID;
    if (need_state(c) != PPMB_OK) return PPMB_ERR_INVALID;
    ppmb_status s = enqueue_cfl(c, cfl);
    if (s != PPMB_OK) return s;
    s = check_flag(c);
    if (s != PPMB_OK) return s;
    HIPCHK(c, hipMemcpy(dt_out, c->dt_dev, sizeof(double), hipMemcpyDeviceToHost));
    return PPMB_OK;
}

static ppmb_status enqueue_pass(ppmb_ctx *c, int axis, int heat)
{
    hipError_t e;
    if (c->prec == PPMB_FP64)
        e = launch_sweep<double>(c->g, axis, static_cast<const double *>(c->buf[c->cur]),
                                 static_cast<double *>(c->buf[1 - c->cur]),
                                 static_cast<const double *>(base_rho(c)),
                                 static_cast<const double *>(base_p(c)), c->dt_dev, c->cnt, heat, c->stream);
    else
        e = launch_sweep<float>(c->g, axis, static_cast<const float *>(c->buf[c->cur]),
                                static_cast<float *>(c->buf[1 - c->cur]),
                                static_cast<const float *>(base_rho(c)),
                                static_cast<const float *>(base_p(c)), c->dt_dev, c->cnt, heat, c->stream);
    if (e != hipSuccess) return hipfail(c, e, "sweep launch");
    c->cur = 1 - c->cur;
    return PPMB_OK;
}

static ppmb_status enqueue_step(ppmb_ctx *c)
{
    const int heat = c->g.heat_kind != PPMB_HEAT_NONE;
    const int order[2][3] = { { 0, 1, 2 }, { 2, 1, 0 } };
    const int *o = order[c->nstep & 1];
    for (int p = 0; p < 3; ++p) {
        ppmb_status s = enqueue_pass(c, o[p], p == 2 ? heat : 0);
        if (s != PPMB_OK) return s;
    }
    c->nstep++;
    c->steps++;
    return PPMB_OK;
}

ppmb_status ppmb_step(ppmb_ctx *c, double dt)
{
    if (!c || !(dt > 0) || !std::isfinite(dt)) return PPMB_ERR_INVALID;
    if (need_state(c) != PPMB_OK) return PPMB_ERR_INVALID;
    HIPCHK(c, launch_set_scalar(c->dt_dev, dt, c->stream));
    return enqueue_step(c);
}

ppmb_status ppmb_step_auto(ppmb_ctx *c, double cfl, int nsteps)
{
    if (!c || !(cfl > 0) || nsteps < 0) return PPMB_ERR_INVALID;
    if (need_state(c) != PPMB_OK) return PPMB_ERR_INVALID;
    for (int s = 0; s < nsteps; ++s) {
        ppmb_status r = enqueue_cfl(c, cfl);
        if (r != PPMB_OK) return r;
        r = enqueue_step(c);
        if (r != PPMB_OK) return r;
    }
    return PPMB_OK;
}

ppmb_status ppmb_last_dt(ppmb_ctx *c, double *dt_out)
{
    if (!c || !dt_out) return PPMB_ERR_INVALID;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemcpy(dt_out, c->dt_dev, sizeof(double), hipMemcpyDeviceToHost));
    return PPMB_OK;
}

ppmb_status ppmb_pass(ppmb_ctx *c, int axis, double dt, int heat)
{
    if (!c || axis < 0 || axis > 2 || !(dt > 0)) return PPMB_ERR_INVALID;
    if (need_state(c) != PPMB_OK) return PPMB_ERR_INVALID;
    HIPCHK(c, launch_set_scalar(c->dt_dev, dt, c->stream));
    return enqueue_pass(c, axis, heat ? (c->g.heat_kind != PPMB_HEAT_NONE) : 0);
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

ppmb_status ppmb_reduce_totals(ppmb_ctx *c, double out[8])
{
    if (!c || !out) return PPMB_ERR_INVALID;
    if (need_state(c) != PPMB_OK) return PPMB_ERR_INVALID;
    if (c->prec == PPMB_FP64)
        HIPCHK(c, launch_totals<double>(c->g, cur_state<double>(c), c->base64, c->base64 + c->ncell,
                                        c->partials, c->out8, c->stream));
    else
        HIPCHK(c, launch_totals<float>(c->g, cur_state<float>(c), c->base64, c->base64 + c->ncell,
                                       c->partials, c->out8, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemcpy(out, c->out8, sizeof(double) * 8, hipMemcpyDeviceToHost));
    return PPMB_OK;
}

ppmb_status ppmb_counters(ppmb_ctx *c, unsigned long long out[4])
{
    if (!c || !out) return PPMB_ERR_INVALID;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemcpy(out, c->cnt, sizeof(unsigned long long) * 3, hipMemcpyDeviceToHost));
    out[3] = c->steps;
    return PPMB_OK;
}

ppmb_status ppmb_synchronize(ppmb_ctx *c)
{
    if (!c) return PPMB_ERR_INVALID;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return PPMB_OK;
}

}  // extern "C"
