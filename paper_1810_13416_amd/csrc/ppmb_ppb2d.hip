// ppmb_ppb2d.hip -- 2-D PPB advection under a rigid rotation (the
// slotted-disk test of Fig. 3): the same PPB pass as the 3-D step (Sec. 1,
// Sec. 4; fv_limit, slab and ppb_update of ppmb_dev.h) with the z terms
// zero and the face Courant numbers of the prescribed velocity.
//
// One thread per cell: a pass updates a cell from its own and its two
// neighbours' moments along the pass, so every load and store of a field
// is a coalesced row for both passes (lanes along x).  With a rotation the
// velocity normal to the faces of a pencil does not vary along it, so every
// cell keeps its length (L = 1) and the slab of each face takes its donor
// by the sign of that velocity.
#include "../../include/ppmb.h"
#include "ppmb_internal.h"

#include <cmath>
#include <string>

namespace ppmb {

// storage: field q (f0, fx, fy, fxx, fyy, fxy) of cell (i, j) at
// q * fs + j * px + i
struct P2Geom {
    int nx, ny, px;
    long fs;
    double dx, ox, oy, cx, cy, omega;
};

template <typename T>
struct P2Args {
    P2Geom g;
    const T *in;
    T *out;
    double dt;
};

// The pass-local moments of a cell (quadratic along the pass, the linear
// transverse pair, the transverse curvature; the z entries of the 3-D
// layout are zero).  AX 0: (f0, fx, fxx | fy, fxy | fyy); AX 1: (f0, fy,
// fyy | fx, fxy | fxx).
template <typename T, int AX>
__device__ __forceinline__ void p2_load(const P2Args<T> &a, long c, T q[10])
{
    const long fs = a.g.fs;
    const T f0 = a.in[c], fx = a.in[fs + c], fy = a.in[2 * fs + c];
    const T fxx = a.in[3 * fs + c], fyy = a.in[4 * fs + c], fxy = a.in[5 * fs + c];
    q[0] = f0;
    q[1] = AX == 0 ? fx : fy;
    q[2] = AX == 0 ? fxx : fyy;
    q[3] = AX == 0 ? fy : fx;
    q[4] = fxy;
    q[5] = T(0);
    q[6] = T(0);
    q[7] = AX == 0 ? fyy : fxx;
    q[8] = T(0);
    q[9] = T(0);
}

template <typename T, int AX>
__global__ __launch_bounds__(256) void ppb2d_pass_kernel(P2Args<T> a)
{
    const P2Geom &g = a.g;
    const long c = blockIdx.x * (long)blockDim.x + threadIdx.x;
    const int i = (int)(c % g.px), j = (int)(c / g.px);
    if (i >= g.nx || j >= g.ny) return;
    const int n = AX == 0 ? g.nx : g.ny;
    const int k = AX == 0 ? i : j;
    const long st = AX == 0 ? 1 : g.px;
    const int km = k == 0 ? n - 1 : k - 1, kp = k == n - 1 ? 0 : k + 1;   // periodic
    const long cm = c + (long)(km - k) * st, cp = c + (long)(kp - k) * st;
    // face Courant number of the pencil (normal velocity at its faces)
    const double tc = AX == 0 ? g.oy + (j + 0.5) * g.dx : g.ox + (i + 0.5) * g.dx;
    const double vel = AX == 0 ? -g.omega * (tc - g.cy) : g.omega * (tc - g.cx);
    const T s = T(vel * a.dt / g.dx);
    const T L = T(1) + (s - s);          // every cell keeps its length
    T qm[10], q0[10], qp[10];
    p2_load<T, AX>(a, cm, qm);
    p2_load<T, AX>(a, c, q0);
    p2_load<T, AX>(a, cp, qp);
    fv_limit(qm[0], qm[1], qm[2]);
    fv_limit(q0[0], q0[1], q0[2]);
    fv_limit(qp[0], qp[1], qp[2]);
    // donors: left of a face for s > 0, right of it (odd-in-s entries
    // flipped) otherwise
    const bool pos = s > T(0);
    T dl[10], dr[10];
#pragma unroll
    for (int v = 0; v < 10; ++v) {
        const bool odd = v == 1 || v == 4 || v == 6;
        dl[v] = pos ? qm[v] : (odd ? -q0[v] : q0[v]);
        dr[v] = pos ? q0[v] : (odd ? -qp[v] : qp[v]);
    }
    T GL[10], GR[10], o[10];
    slab(dl, s, L, GL);
    slab(dr, s, L, GR);
    ppb_update(q0, s - s, T(0.5) * (s + s), GL, GR, o);
    const long fs = g.fs;
    a.out[c] = o[0];
    a.out[(AX == 0 ? 1 : 2) * fs + c] = o[1];
    a.out[(AX == 0 ? 3 : 4) * fs + c] = o[2];
    a.out[(AX == 0 ? 2 : 1) * fs + c] = o[3];
    a.out[5 * fs + c] = o[4];
    a.out[(AX == 0 ? 4 : 3) * fs + c] = o[7];
}

template <typename T>
static hipError_t launch_p2_pass(int axis, const P2Args<T> &a, hipStream_t st)
{
    const long cells = (long)a.g.px * a.g.ny;
    const dim3 grid((unsigned)((cells + 255) / 256)), block(256);
    if (axis == 0) hipLaunchKernelGGL((ppb2d_pass_kernel<T, 0>), grid, block, 0, st, a);
    else hipLaunchKernelGGL((ppb2d_pass_kernel<T, 1>), grid, block, 0, st, a);
    return hipGetLastError();
}

// dense FP64 (6 fields of nx * ny) <-> pitched storage
template <typename T>
__global__ void p2_scatter_kernel(P2Geom g, const double *src, T *dst)
{
    const long n = (long)g.nx * g.ny;
    for (long x = blockIdx.x * (long)blockDim.x + threadIdx.x; x < 6 * n; x += (long)gridDim.x * blockDim.x) {
        const long q = x / n, c = x - q * n;
        const long j = c / g.nx, i = c - j * g.nx;
        dst[q * g.fs + j * g.px + i] = T(src[x]);
    }
}

template <typename T>
__global__ void p2_gather_kernel(P2Geom g, const T *src, double *dst)
{
    const long n = (long)g.nx * g.ny;
    for (long x = blockIdx.x * (long)blockDim.x + threadIdx.x; x < 6 * n; x += (long)gridDim.x * blockDim.x) {
        const long q = x / n, c = x - q * n;
        const long j = c / g.nx, i = c - j * g.nx;
        dst[x] = double(src[q * g.fs + j * g.px + i]);
    }
}

}  // namespace ppmb

using namespace ppmb;

struct ppmb_ppb2d {
    P2Geom g{};
    ppmb_precision prec = PPMB_FP64;
    size_t esz = 8;
    hipStream_t stream = nullptr;
    void *buf[2] = { nullptr, nullptr };
    int cur = 0;
    long nstep = 0;
};

namespace {

ppmb_status p2_free(ppmb_ppb2d *c)
{
    if (!c) return PPMB_ERR_INVALID;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    for (void *b : c->buf)
        if (b) (void)hipFree(b);
    delete c;
    return PPMB_OK;
}

struct P2Staging {
    double *p = nullptr;
    ~P2Staging() { if (p) (void)hipFree(p); }
};

}  // namespace

extern "C" {

ppmb_status ppmb_ppb2d_create(const ppmb_ppb2d_grid *grid, ppmb_precision prec, void *hip_stream,
                              ppmb_ppb2d **out)
{
    if (!grid || !out) return PPMB_ERR_INVALID;
    *out = nullptr;
    if (prec != PPMB_FP64 && prec != PPMB_FP32) return PPMB_ERR_INVALID;
    if (grid->n[0] < 3 || grid->n[1] < 3 || (long)grid->n[0] * grid->n[1] >= (1L << 31)) return PPMB_ERR_INVALID;
    if (!(grid->dx > 0) || !std::isfinite(grid->omega)) return PPMB_ERR_INVALID;
    ppmb_ppb2d *c = new ppmb_ppb2d();
    c->prec = prec;
    c->esz = prec == PPMB_FP64 ? 8 : 4;
    c->stream = static_cast<hipStream_t>(hip_stream);
    P2Geom &g = c->g;
    g.nx = grid->n[0];
    g.ny = grid->n[1];
    g.px = (g.nx + 63) / 64 * 64;
    g.fs = (long)g.px * g.ny + 17 * 64;
    g.dx = grid->dx;
    g.ox = grid->origin[0];
    g.oy = grid->origin[1];
    g.cx = grid->centre[0];
    g.cy = grid->centre[1];
    g.omega = grid->omega;
    const size_t bytes = c->esz * 6 * (size_t)g.fs;
    for (int b = 0; b < 2; ++b) {
        if (hipMalloc(&c->buf[b], bytes) != hipSuccess || hipMemset(c->buf[b], 0, bytes) != hipSuccess) {
            p2_free(c);
            return PPMB_ERR_NOMEM;
        }
    }
    *out = c;
    return PPMB_OK;
}

ppmb_status ppmb_ppb2d_destroy(ppmb_ppb2d *c) { return p2_free(c); }

ppmb_status ppmb_ppb2d_set(ppmb_ppb2d *c, const double *const host_coef[6])
{
    if (!c || !host_coef) return PPMB_ERR_INVALID;
    for (int q = 0; q < 6; ++q)
        if (!host_coef[q]) return PPMB_ERR_INVALID;
    const long n = (long)c->g.nx * c->g.ny;
    P2Staging st;
    if (hipMalloc(&st.p, sizeof(double) * 6 * n) != hipSuccess) return PPMB_ERR_NOMEM;
    for (int q = 0; q < 6; ++q)
        if (hipMemcpyAsync(st.p + q * n, host_coef[q], sizeof(double) * n, hipMemcpyHostToDevice, c->stream) != hipSuccess)
            return PPMB_ERR_HIP;
    if (c->prec == PPMB_FP64)
        hipLaunchKernelGGL((p2_scatter_kernel<double>), dim3(1024), dim3(256), 0, c->stream, c->g, st.p,
                           static_cast<double *>(c->buf[c->cur]));
    else
        hipLaunchKernelGGL((p2_scatter_kernel<float>), dim3(1024), dim3(256), 0, c->stream, c->g, st.p,
                           static_cast<float *>(c->buf[c->cur]));
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(c->stream) != hipSuccess) return PPMB_ERR_HIP;
    return PPMB_OK;
}

ppmb_status ppmb_ppb2d_get(ppmb_ppb2d *c, double *const host_coef[6])
{
    if (!c || !host_coef) return PPMB_ERR_INVALID;
    for (int q = 0; q < 6; ++q)
        if (!host_coef[q]) return PPMB_ERR_INVALID;
    const long n = (long)c->g.nx * c->g.ny;
    P2Staging st;
    if (hipMalloc(&st.p, sizeof(double) * 6 * n) != hipSuccess) return PPMB_ERR_NOMEM;
    if (c->prec == PPMB_FP64)
        hipLaunchKernelGGL((p2_gather_kernel<double>), dim3(1024), dim3(256), 0, c->stream, c->g,
                           static_cast<const double *>(c->buf[c->cur]), st.p);
    else
        hipLaunchKernelGGL((p2_gather_kernel<float>), dim3(1024), dim3(256), 0, c->stream, c->g,
                           static_cast<const float *>(c->buf[c->cur]), st.p);
    if (hipGetLastError() != hipSuccess) return PPMB_ERR_HIP;
    for (int q = 0; q < 6; ++q)
        if (hipMemcpyAsync(host_coef[q], st.p + q * n, sizeof(double) * n, hipMemcpyDeviceToHost, c->stream) != hipSuccess)
            return PPMB_ERR_HIP;
    if (hipStreamSynchronize(c->stream) != hipSuccess) return PPMB_ERR_HIP;
    return PPMB_OK;
}

ppmb_status ppmb_ppb2d_steps(ppmb_ppb2d *c, double dt, int nsteps)
{
    if (!c || !(dt > 0) || !std::isfinite(dt) || nsteps < 0) return PPMB_ERR_INVALID;
    const P2Geom &g = c->g;
    // largest lever arm of a face velocity on the grid
    const double ax = std::fmax(std::fabs(g.ox - g.cx), std::fabs(g.ox + g.nx * g.dx - g.cx));
    const double ay = std::fmax(std::fabs(g.oy - g.cy), std::fabs(g.oy + g.ny * g.dx - g.cy));
    if (std::fabs(g.omega) * std::fmax(ax, ay) * dt / g.dx >= 1.0) return PPMB_ERR_INVALID;
    for (int k = 0; k < nsteps; ++k) {
        const int first = (c->nstep & 1) ? 1 : 0;
        for (int p = 0; p < 2; ++p) {
            const int axis = p == 0 ? first : 1 - first;
            hipError_t e;
            if (c->prec == PPMB_FP64) {
                P2Args<double> a{ g, static_cast<const double *>(c->buf[c->cur]),
                                  static_cast<double *>(c->buf[1 - c->cur]), dt };
                e = launch_p2_pass(axis, a, c->stream);
            } else {
                P2Args<float> a{ g, static_cast<const float *>(c->buf[c->cur]),
                                 static_cast<float *>(c->buf[1 - c->cur]), dt };
                e = launch_p2_pass(axis, a, c->stream);
            }
            if (e != hipSuccess) return PPMB_ERR_HIP;
            c->cur = 1 - c->cur;
        }
        c->nstep++;
    }
    return PPMB_OK;
}

ppmb_status ppmb_ppb2d_get_nstep(const ppmb_ppb2d *c, long *nstep)
{
    if (!c || !nstep) return PPMB_ERR_INVALID;
    *nstep = c->nstep;
    return PPMB_OK;
}

ppmb_status ppmb_ppb2d_set_nstep(ppmb_ppb2d *c, long nstep)
{
    if (!c || nstep < 0) return PPMB_ERR_INVALID;
    c->nstep = nstep;
    return PPMB_OK;
}

}  // extern "C"
