// ppmb_aux.hip -- FP64 base-state integration, state conversions, the CFL
// time-step reduction and the conserved-total reduction (gfx950).
//
// Built with -ffp-contract=off: none of this is on the per-pass hot path,
// and uncontracted FP64 keeps these results reproducible bit for bit.
#include "ppmb_internal.h"

#include <cmath>

namespace ppmb {

// ---------------------------------------------------------------------
// Base state (Sec. 1: the initial hydrostatic state is saved on the grid
// and subtracted out).  dp/ds = rho(p, s) g_s(s), rho = (p/K)^(1/gamma),
// K jumping at the entropy step so that rho jumps by f at continuous p.
// ---------------------------------------------------------------------

enum { MAXSEG = 6, HDR = 1 + 6 * MAXSEG };

__device__ double base_gs(const Geom &g, int kind, double s)
{
    if (kind == 2) return g.grav_kind == 1 ? g.grav[2] : 0.0;
    if (g.grav_kind != 2) return 0.0;
    double rc = g.grav[1];
    double shape = (s < rc) ? s / rc : (rc * rc) / (s * s);
    return -g.grav[0] * shape * grav_taper(g, s);
}

__device__ double base_rhs(const Geom &g, int kind, double K, double s, double p)
{
    return pow(p / K, 1.0 / g.gamma) * base_gs(g, kind, s);
}

__device__ double rk4(const Geom &g, int kind, double K, double s, double p, double h)
{
    double k1 = base_rhs(g, kind, K, s, p);
    double k2 = base_rhs(g, kind, K, s + 0.5 * h, p + 0.5 * h * k1);
    double k3 = base_rhs(g, kind, K, s + 0.5 * h, p + 0.5 * h * k2);
    double k4 = base_rhs(g, kind, K, s + h, p + h * k3);
    return p + h * (k1 + 2.0 * k2 + 2.0 * k3 + k4) / 6.0;
}

struct BaseParams { double v[6]; };

// One thread: segment the interval [s_b, s_end] at the entropy jump and at
// every kink of the gravity profile, then RK4 with 8 steps per cell width.
// Table: [nseg, then per segment s0, s1, h, K, m, node offset], then nodes.
__global__ void base_table_kernel(Geom g, int kind, BaseParams bp, double *tab, long len)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const double rho_b = bp.v[0], p_b = bp.v[1], s_b = bp.v[2], s_i = bp.v[3], f = bp.v[4],
                 s_end = bp.v[5];
    const double K1 = p_b / pow(rho_b, g.gamma);
    const double K2 = K1 * pow(f, -g.gamma);
    const double hmax = g.dx / 8.0;
    double br[MAXSEG + 1];
    int nb = 0;
    br[nb++] = s_b;
    double cand[4] = { s_i, 0.0, 0.0, 0.0 };
    int nc = 1;
    if (kind == 3 && g.grav_kind == 2) { cand[1] = g.grav[1]; cand[2] = g.grav[2]; cand[3] = g.grav[3]; nc = 4; }
    for (int q = 0; q < nc; ++q) {
        double c = cand[q];
        if (!(c > s_b && c < s_end)) continue;
        bool dup = false;
        for (int r = 0; r < nb; ++r) dup = dup || (br[r] == c);
        if (dup) continue;
        int at = nb;
        while (at > 1 && br[at - 1] > c) { br[at] = br[at - 1]; --at; }
        br[at] = c;
        ++nb;
    }
    br[nb++] = s_end;
    const int nseg = nb - 1;
    tab[0] = nseg;
    long off = HDR;
    double p = p_b;
    for (int sg = 0; sg < nseg; ++sg) {
        double a = br[sg], b = br[sg + 1];
        int m = (int)ceil((b - a) / hmax);
        if (m < 1) m = 1;
        double h = (b - a) / m;
        double K = (a >= s_i) ? K2 : K1;
        double *hd = tab + 1 + 6 * sg;
        hd[0] = a; hd[1] = b; hd[2] = h; hd[3] = K; hd[4] = m; hd[5] = (double)off;
        if (off + m + 1 > len) { tab[0] = -1.0; return; }
        tab[off] = p;
        for (int q = 0; q < m; ++q) tab[off + q + 1] = rk4(g, kind, K, a + q * h, tab[off + q], h);
        p = tab[off + m];
        off += m + 1;
    }
}

// Cell values: one RK4 step from the nearest node below each cell centre.
__global__ void base_fill_kernel(Geom g, int kind, BaseParams bp, const double *tab, long len,
                                 double *rho0, double *p0)
{
    long nc = (long)g.n[0] * g.n[1] * g.n[2];
    // a table that did not fit leaves nseg = -1: write NaN, read nothing
    const int nseg_all = (kind == 2 || kind == 3) ? (int)tab[0] : 1;
    for (long cd = blockIdx.x * (long)blockDim.x + threadIdx.x; cd < nc; cd += (long)gridDim.x * blockDim.x) {
        const long c = pitched(g, cd);
        if (kind == 0 || kind == 1) {
            rho0[c] = (kind == 1) ? bp.v[0] : 0.0;
            p0[c] = (kind == 1) ? bp.v[1] : 0.0;
            continue;
        }
        int i = (int)(cd % g.n[0]);
        int j = (int)((cd / g.n[0]) % g.n[1]);
        int k = (int)(cd / ((long)g.n[0] * g.n[1]));
        double x = centre(g, 0, i), y = centre(g, 1, j), z = centre(g, 2, k);
        double s = (kind == 2) ? z : sqrt(r2_exact(x, y, z));
        if (nseg_all < 1 || nseg_all > MAXSEG) { rho0[c] = NAN; p0[c] = NAN; continue; }
        int sg = 0;
        while (sg < nseg_all - 1 && s >= tab[1 + 6 * sg + 1]) ++sg;
        const double *hd = tab + 1 + 6 * sg;
        double s0 = hd[0], h = hd[2], K = hd[3];
        int m = (int)hd[4];
        long off = (long)hd[5];
        int q = (int)floor((s - s0) / h);
        if (q < 0) q = 0;
        if (q > m - 1) q = m - 1;
        if (off < HDR || off + q >= len) { rho0[c] = NAN; p0[c] = NAN; continue; }
        double sq = s0 + q * h;
        double pv = rk4(g, kind, K, sq, tab[off + q], s - sq);
        p0[c] = pv;
        rho0[c] = pow(pv / K, 1.0 / g.gamma);
    }
}

hipError_t launch_base_state(const Geom &g, int kind, const double *params, double *table,
                             long table_len, double *rho0, double *p0, hipStream_t st)
{
    BaseParams bp;
    for (int q = 0; q < 6; ++q) bp.v[q] = params ? params[q] : 0.0;
    if (kind == 2 || kind == 3)
        hipLaunchKernelGGL(base_table_kernel, dim3(1), dim3(64), 0, st, g, kind, bp, table, table_len);
    hipLaunchKernelGGL(base_fill_kernel, dim3(4096), dim3(256), 0, st, g, kind, bp, table, table_len, rho0, p0);
    return hipGetLastError();
}

// ---------------------------------------------------------------------
// Conversions
// ---------------------------------------------------------------------

struct PrimPtrs { const double *p[NF]; };

// Dense cells [c0, c0 + m) of a brick: FP64 primitive perturbations
// (field q of the range at P.p[q], dense) to the stored conserved fields
// (pitched, field stride g.fs); rho0 is the brick's pitched FP64 base.
template <typename T>
__global__ void prim_to_cons_kernel(Geom g, long c0, long m, double gm1, PrimPtrs P,
                                    const double *rho0, T *S)
{
    const long fs = g.fs;
    for (long c = blockIdx.x * (long)blockDim.x + threadIdx.x; c < m; c += (long)gridDim.x * blockDim.x) {
        const long e = pitched(g, c0 + c);
        double rho = rho0[e] + P.p[0][c];
        double u = P.p[1][c], v = P.p[2][c], w = P.p[3][c];
        S[RHO * fs + e] = T(P.p[0][c]);
        S[MX * fs + e] = T(rho * u);
        S[MY * fs + e] = T(rho * v);
        S[MZ * fs + e] = T(rho * w);
        S[EN * fs + e] = T(P.p[4][c] / gm1 + 0.5 * rho * ((u * u + v * v) + w * w));
        for (int q = 5; q < NF; ++q) S[q * fs + e] = T(P.p[q][c]);
    }
}

// The reverse: field q of the range to out + q * ostride (dense).
template <typename T>
__global__ void cons_to_prim_kernel(Geom g, long c0, long m, long ostride, double gm1, const T *S,
                                    const double *rho0, double *out)
{
    const long fs = g.fs;
    for (long c = blockIdx.x * (long)blockDim.x + threadIdx.x; c < m; c += (long)gridDim.x * blockDim.x) {
        const long e = pitched(g, c0 + c);
        double rp = S[RHO * fs + e], mx = S[MX * fs + e], my = S[MY * fs + e];
        double mz = S[MZ * fs + e], en = S[EN * fs + e];
        double rho = rho0[e] + rp;
        double u = mx / rho, v = my / rho, w = mz / rho;
        out[0 * ostride + c] = rp;
        out[1 * ostride + c] = u;
        out[2 * ostride + c] = v;
        out[3 * ostride + c] = w;
        out[4 * ostride + c] = gm1 * (en - 0.5 * (mx * u + my * v + mz * w));
        for (int q = 5; q < NF; ++q) out[q * ostride + c] = S[q * fs + e];
    }
}

template <typename T>
hipError_t launch_prim_to_cons_range(const Geom &g, const double *const *prim, const double *rho0,
                                     T *state, long c0, long m, hipStream_t st)
{
    PrimPtrs P;
    for (int q = 0; q < NF; ++q) P.p[q] = prim[q];
    hipLaunchKernelGGL((prim_to_cons_kernel<T>), dim3(4096), dim3(256), 0, st, g, c0, m, g.gamma - 1.0, P,
                       rho0, state);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_cons_to_prim_range(const Geom &g, const T *state, const double *rho0, double *out,
                                     long c0, long m, long ostride, hipStream_t st)
{
    hipLaunchKernelGGL((cons_to_prim_kernel<T>), dim3(4096), dim3(256), 0, st, g, c0, m, ostride,
                       g.gamma - 1.0, state, rho0, out);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_prim_to_cons(const Geom &g, const double *const *prim, const double *rho0,
                               T *state, hipStream_t st)
{
    return launch_prim_to_cons_range<T>(g, prim, rho0, state, 0, (long)g.n[0] * g.n[1] * g.n[2], st);
}

template <typename A, typename B>
__global__ void convert_kernel(const A *src, B *dst, long count)
{
    for (long c = blockIdx.x * (long)blockDim.x + threadIdx.x; c < count; c += (long)gridDim.x * blockDim.x)
        dst[c] = B(src[c]);
}

// nf fields of a brick between pitched storage and dense FP64 (field q of
// the dense side at q * ncell).
template <typename T>
__global__ void gather_kernel(Geom g, int nf, const T *src, double *dst)
{
    const long n = (long)g.n[0] * g.n[1] * g.n[2];
    for (long x = blockIdx.x * (long)blockDim.x + threadIdx.x; x < nf * n; x += (long)gridDim.x * blockDim.x) {
        const long q = x / n, c = x - q * n;
        dst[x] = double(src[q * g.fs + pitched(g, c)]);
    }
}

template <typename T>
__global__ void scatter_kernel(Geom g, int nf, const double *src, T *dst)
{
    const long n = (long)g.n[0] * g.n[1] * g.n[2];
    for (long x = blockIdx.x * (long)blockDim.x + threadIdx.x; x < nf * n; x += (long)gridDim.x * blockDim.x) {
        const long q = x / n, c = x - q * n;
        dst[q * g.fs + pitched(g, c)] = T(src[x]);
    }
}

template <typename T>
hipError_t launch_gather(const Geom &g, int nf, const T *src, double *dst, hipStream_t st)
{
    hipLaunchKernelGGL((gather_kernel<T>), dim3(4096), dim3(256), 0, st, g, nf, src, dst);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_scatter(const Geom &g, int nf, const double *src, T *dst, hipStream_t st)
{
    hipLaunchKernelGGL((scatter_kernel<T>), dim3(4096), dim3(256), 0, st, g, nf, src, dst);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_narrow(const double *src, T *dst, long count, hipStream_t st)
{
    hipLaunchKernelGGL((convert_kernel<double, T>), dim3(4096), dim3(256), 0, st, src, dst, count);
    return hipGetLastError();
}

// ---------------------------------------------------------------------
// CFL time step: dt = cfl dx / max over fluid cells and axes of |u_d| + c,
// all in FP64.  The maximum is order independent, so it is exact.
// ---------------------------------------------------------------------

int cfl_blocks(long ncell) { return (int)((ncell + kCflBlockCells - 1) / kCflBlockCells); }

__global__ void cfl_reset_kernel(unsigned long long *work, int b0, int nb)
{
    for (int b = threadIdx.x; b < nb; b += blockDim.x) work[2 * (b0 + b)] = 0ull;
}

// `only`: when given, blocks of bricks whose redo flag only[2 brick + 1] is
// clear return at once.
template <typename T>
__global__ __launch_bounds__(256) void cfl_kernel(const Brick *bricks, const BlockMap *map,
                                                  const T *arena, const double *base64,
                                                  unsigned long long *work, const unsigned long long *only)
{
    const BlockMap m = map[blockIdx.x];
    if (only && only[2 * m.brick + 1] == 0ull) return;
    cfl_block_part<T>(bricks, m, arena, base64, work, (int)threadIdx.x, (int)blockDim.x);
}

__global__ void cfl_finish_kernel(const Brick *bricks, int b0, int nb, const unsigned long long *work,
                                  double cfl, double *dt)
{
    for (int b = threadIdx.x; b < nb; b += blockDim.x) {
        const Brick &B = bricks[b0 + b];
        double smax = __longlong_as_double((long long)work[2 * (b0 + b)]);
        dt[B.dti] = cfl * B.g.dx / smax;
    }
}

__global__ void cfl_arm_kernel(unsigned long long *work, unsigned long long *cband, int b0, int nb)
{
    for (int b = threadIdx.x; b < nb; b += blockDim.x) cfl_arm_brick(work, cband, b0 + b);
}

// dt where the fused maximum reached the band edge; else clear the
// maximum and raise the brick's redo flag
__global__ void cfl_check_kernel(const Brick *bricks, int b0, int nb, unsigned long long *work,
                                 unsigned long long *cband, double cfl, double *dt)
{
    for (int b = threadIdx.x; b < nb; b += blockDim.x) cfl_check_brick(bricks, b0 + b, work, cband, cfl, dt);
}

__global__ void cfl_redo_finish_kernel(const Brick *bricks, int b0, int nb, const unsigned long long *work,
                                       unsigned long long *cband, double cfl, double *dt)
{
    for (int b = threadIdx.x; b < nb; b += blockDim.x) cfl_redo_finish_brick(bricks, b0 + b, work, cband, cfl, dt);
}

// Courant check of a caller-given dt: dt[dti] holds courant_max dx / smax
// of the state the step starts from (launch_cfl); raise the flag where the
// given dt exceeds it, then store the given dt.
__global__ void cfl_given_kernel(const Brick *bricks, int b0, int nb, double given, double *dt,
                                 unsigned long long *flag)
{
    for (int b = threadIdx.x; b < nb; b += blockDim.x) {
        const Brick &B = bricks[b0 + b];
        if (!(given <= dt[B.dti])) atomicOr(flag, 1ull);
        dt[B.dti] = given;
    }
}

hipError_t launch_cfl_given(const Brick *bricks, int b0, int nb, double given, double *dt,
                            unsigned long long *flag, hipStream_t st)
{
    hipLaunchKernelGGL(cfl_given_kernel, dim3(1), dim3(256), 0, st, bricks, b0, nb, given, dt, flag);
    return hipGetLastError();
}

hipError_t launch_cfl_arm(unsigned long long *work, unsigned long long *cband, int b0, int nb, hipStream_t st)
{
    hipLaunchKernelGGL(cfl_arm_kernel, dim3(1), dim3(256), 0, st, work, cband, b0, nb);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_cfl_finish(const Brick *bricks, int b0, int nb, const BlockMap *map, int nblocks,
                             const T *state, const double *base64, unsigned long long *work,
                             unsigned long long *cband, double cfl, double *dt, hipStream_t st)
{
    hipLaunchKernelGGL(cfl_check_kernel, dim3(1), dim3(256), 0, st, bricks, b0, nb, work, cband, cfl, dt);
    hipLaunchKernelGGL((cfl_kernel<T>), dim3(nblocks), dim3(256), 0, st, bricks, map, state, base64, work,
                       (const unsigned long long *)cband);
    hipLaunchKernelGGL(cfl_redo_finish_kernel, dim3(1), dim3(256), 0, st, bricks, b0, nb, work, cband, cfl, dt);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_cfl(const Brick *bricks, int b0, int nb, const BlockMap *map, int nblocks,
                      const T *state, const double *base64, unsigned long long *work, double cfl,
                      double *dt, hipStream_t st)
{
    hipLaunchKernelGGL(cfl_reset_kernel, dim3(1), dim3(256), 0, st, work, b0, nb);
    hipLaunchKernelGGL((cfl_kernel<T>), dim3(nblocks), dim3(256), 0, st, bricks, map, state, base64, work,
                       (const unsigned long long *)nullptr);
    hipLaunchKernelGGL(cfl_finish_kernel, dim3(1), dim3(256), 0, st, bricks, b0, nb, work, cfl, dt);
    return hipGetLastError();
}

// ---------------------------------------------------------------------
// Totals: 6 sums and min / max of f0 over fluid cells.  Each thread walks
// a fixed stride of cells, each block reduces by a fixed tree, one final
// block reduces the block partials by a fixed tree: bitwise reproducible.
// ---------------------------------------------------------------------

template <typename T>
__global__ __launch_bounds__(256) void totals_kernel(Geom g, const T *S, const double *rho0,
                                                     const double *p0, double *partials)
{
    __shared__ double sh[8][256];
    const long nc = (long)g.n[0] * g.n[1] * g.n[2];
    const double gm1 = g.gamma - 1.0;
    double acc[8] = { 0, 0, 0, 0, 0, 0, INFINITY, -INFINITY };
    const long fs = g.fs;
    for (long c = blockIdx.x * 256L + threadIdx.x; c < nc; c += (long)kTotalsBlocks * 256) {
        const unsigned nx = (unsigned)g.n[0], ny = (unsigned)g.n[1];
        const unsigned row = (unsigned)c / nx, i = (unsigned)c - row * nx;
        const unsigned k = row / ny, j = row - k * ny;
        if (g.sphere && solid_at(g, centre(g, 0, i), centre(g, 1, j), centre(g, 2, k))) continue;
        const long e = (long)i + (long)j * g.px + (long)k * g.plane;
        double f0 = S[F0 * fs + e];
        acc[0] += rho0[e] + (double)S[RHO * fs + e];
        acc[1] += (double)S[MX * fs + e];
        acc[2] += (double)S[MY * fs + e];
        acc[3] += (double)S[MZ * fs + e];
        acc[4] += p0[e] / gm1 + (double)S[EN * fs + e];
        acc[5] += f0;
        acc[6] = fmin(acc[6], f0);
        acc[7] = fmax(acc[7], f0);
    }
    for (int q = 0; q < 8; ++q) sh[q][threadIdx.x] = acc[q];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            for (int q = 0; q < 6; ++q) sh[q][threadIdx.x] += sh[q][threadIdx.x + w];
            sh[6][threadIdx.x] = fmin(sh[6][threadIdx.x], sh[6][threadIdx.x + w]);
            sh[7][threadIdx.x] = fmax(sh[7][threadIdx.x], sh[7][threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int q = 0; q < 8; ++q) partials[blockIdx.x * 8 + q] = sh[q][0];
}

__global__ __launch_bounds__(1024) void totals_finish_kernel(const double *partials, double dv, double *out)
{
    __shared__ double sh[8][kTotalsBlocks];
    for (int q = 0; q < 8; ++q) sh[q][threadIdx.x] = partials[threadIdx.x * 8 + q];
    __syncthreads();
    for (int w = kTotalsBlocks / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            for (int q = 0; q < 6; ++q) sh[q][threadIdx.x] += sh[q][threadIdx.x + w];
            sh[6][threadIdx.x] = fmin(sh[6][threadIdx.x], sh[6][threadIdx.x + w]);
            sh[7][threadIdx.x] = fmax(sh[7][threadIdx.x], sh[7][threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        for (int q = 0; q < 6; ++q) out[q] = sh[q][0] * dv;
        out[6] = sh[6][0];
        out[7] = sh[7][0];
    }
}

template <typename T>
hipError_t launch_totals(const Geom &g, const T *state, const double *rho0, const double *p0,
                         double *partials, double *out, hipStream_t st)
{
    hipLaunchKernelGGL((totals_kernel<T>), dim3(kTotalsBlocks), dim3(256), 0, st, g, state, rho0, p0, partials);
    hipLaunchKernelGGL(totals_finish_kernel, dim3(1), dim3(kTotalsBlocks), 0, st, partials,
                       g.dx * g.dx * g.dx, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------
// Shock dissipation (Sec. 1: a fully 3-D dissipation inside shocks): the
// undivided divergence of the cell-centred velocity, sum over d of
// (u_d(i + e_d) - u_d(i - e_d)) / 2, neighbours through the boundary
// conditions (a reflecting image's normal velocity flips), a solid
// neighbour as a wall whose normal velocity is minus the cell's own.
// ---------------------------------------------------------------------

// One block: a tile of kDivTx x kDivTy cells across x and y, marched along
// z through kDivTz planes.  Each thread turns its own cell's conserved
// fields into a velocity once per plane (one FP64 reciprocal); its x and y
// neighbours read theirs from the plane's LDS copy (double-buffered, one
// barrier per plane), the z neighbours come from the thread's own column in
// registers.  The tile's edge cells outside it (x - 1, x + kDivTx, y - 1,
// y + kDivTy) are computed by waves 0, 1 and 3, each thread for at most one
// of them.  The loads of the next plane are issued before the current one
// is finished.
constexpr int kDivTx = 64, kDivTy = 4, kDivTz = 32;

int div_blocks(const Geom &g)
{
    const long t = (long)((g.n[0] + kDivTx - 1) / kDivTx) * ((g.n[1] + kDivTy - 1) / kDivTy) *
                   ((g.n[2] + kDivTz - 1) / kDivTz);
    return (int)t;
}

// The raw inputs of one cell: rho', the momentum components asked for, and
// rho0; `ok` false loads nothing (the slot is not used).
template <typename T>
struct DivRaw {
    T rp, m[3];
    double r0;
};

template <typename T, int NM>
__device__ __forceinline__ void div_load(const T *S, long fs, const double *rho0, long e, bool ok, const int *comp,
                                         DivRaw<T> &r)
{
    if (!ok) e = 0;
    r.rp = S[RHO * fs + e];
#pragma unroll
    for (int c = 0; c < NM; ++c) r.m[c] = S[(MX + comp[c]) * fs + e];
    r.r0 = rho0[e];
}

template <typename T>
__global__ __launch_bounds__(256) void divergence_kernel(const Brick *bricks, const BlockMap *map,
                                                         const T *arena, const double *base64, T *div, int skip)
{
    __shared__ double su[2][kDivTy][kDivTx + 2];            // u at (x0 - 1 + i, y0 + j)
    __shared__ double sv[2][kDivTy + 2][kDivTx];            // v at (x0 + i, y0 - 1 + j)
    __shared__ unsigned char fu[2][kDivTy][kDivTx + 2];     // solid flags of the same slots
    __shared__ unsigned char fv[2][kDivTy + 2][kDivTx];
    const BlockMap m = map[blockIdx.x];
    const Brick &B = bricks[m.brick];
    const Geom g = B.g;
    const T *S = arena + B.off;
    const long fs = g.fs;
    const double *rho0 = base64 + B.boff;
    T *D = div + B.boff / 2;
    const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
    const int tx = (nx + kDivTx - 1) / kDivTx, ty = (ny + kDivTy - 1) / kDivTy;
    const int x0 = (m.local % tx) * kDivTx;
    const int y0 = ((m.local / tx) % ty) * kDivTy;
    int z0 = (m.local / (tx * ty)) * kDivTz;
    int z1 = min(z0 + kDivTz, nz);
    if (skip && g.sphere) {
        // the fluid cells of the tile's columns lie where z^2 < t - (x^2 +
        // y^2) <= t - q, q the least x^2 + y^2 over the tile's cell centres:
        // only those planes (2 more each side, past any rounding) are
        // written (the same for every thread of the block)
        auto least = [&](int axis, int a, int b) {
            const double ca = centre(g, axis, a), cb = centre(g, axis, b);
            return (ca <= 0.0 && cb >= 0.0) ? 0.0 : fmin(fabs(ca), fabs(cb));
        };
        const double lx = least(0, x0, min(x0 + kDivTx, nx) - 1);
        const double ly = least(1, y0, min(y0 + kDivTy, ny) - 1);
        const double h2 = g.sphere_t - (lx * lx + ly * ly);
        if (!(h2 > 0.0)) return;                           // no fluid cell in the tile's columns
        const double h = sqrt(h2);
        const int ka = (int)floor((-h - g.origin[2]) / g.dx - 0.5) - 2;
        const int kb = (int)ceil((h - g.origin[2]) / g.dx - 0.5) + 2;
        z0 = max(z0, ka);
        z1 = min(z1, kb + 1);
        if (z0 >= z1) return;
    }
    const int lane = threadIdx.x & 63;
    const int wy = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    auto elem = [&](int i, int j, int k) { return (long)i + (long)j * g.px + (long)k * g.plane; };

    // own slot (x, y): a cell of the tile, or the image cell just past the
    // brick's high x or y edge (a neighbour of the last cell); its source
    // through the boundary conditions and the flips of u and v
    const int x = x0 + lane, y = y0 + wy;
    const bool own_slot = x <= nx && y <= ny;
    const bool out = x < nx && y < ny;                     // writes a divergence
    int flx = 1, fly = 1;
    const int sx = x < nx ? x : bc_source(x, nx, g.bc[0], flx);
    const int sy = y < ny ? y : bc_source(y, ny, g.bc[1], fly);
    const double cx = centre(g, 0, sx), cy = centre(g, 1, sy);

    // edge slot of this thread: wave 0 the row y0 - 1 (v), wave 3 the row
    // y0 + kDivTy (v), wave 1 lanes 0..3 the column x0 - 1 and lanes 4..7
    // the column x0 + kDivTx (u)
    int hx = 0, hy = 0, hc = 0;                            // position, component (0: none)
    if (wy == 0) { hx = x; hy = y0 - 1; hc = (x < nx) ? 2 : 0; }
    else if (wy == kDivTy - 1) { hx = x; hy = y0 + kDivTy; hc = (x < nx && hy <= ny) ? 2 : 0; }
    else if (wy == 1 && lane < 2 * kDivTy) {
        hy = y0 + (lane & (kDivTy - 1));
        hx = lane < kDivTy ? x0 - 1 : x0 + kDivTx;
        hc = (hy < ny && hx <= nx) ? 1 : 0;
    }
    int hf = 1;
    int hsx = hx, hsy = hy;
    if (hc == 1 && (hx < 0 || hx >= nx)) hsx = bc_source(hx, nx, g.bc[0], hf);
    if (hc == 2 && (hy < 0 || hy >= ny)) hsy = bc_source(hy, ny, g.bc[1], hf);
    const double hcx = centre(g, 0, hsx), hcy = centre(g, 1, hsy);

    const int cuvw[3] = { 0, 1, 2 };
    const int chc[1] = { hc == 2 ? 1 : 0 };
    DivRaw<T> ro, rh;                                      // loads of the next plane
    auto load_plane = [&](int k) {
        int fz;
        const int sz = (k >= 0 && k < nz) ? k : bc_source(k, nz, g.bc[2], fz);
        div_load<T, 3>(S, fs, rho0, elem(sx, sy, sz), own_slot, cuvw, ro);
        div_load<T, 1>(S, fs, rho0, elem(hsx, hsy, sz), hc != 0, chc, rh);
    };
    auto solid_plane = [&](int k, double px, double py) {
        int fz;
        const int sz = (k >= 0 && k < nz) ? k : bc_source(k, nz, g.bc[2], fz);
        return g.sphere && solid_at(g, px, py, centre(g, 2, sz));
    };
    auto zflip = [&](int k) {
        int fz = 1;
        if (k < 0 || k >= nz) bc_source(k, nz, g.bc[2], fz);
        return (double)fz;
    };

    // the cell's velocity and solid flag at plane k from the loads `ro`
    double u = 0.0, v = 0.0, w = 0.0;
    bool so = false;
    auto take_own = [&](int k) {
        const double ir = 1.0 / (ro.r0 + (double)ro.rp);
        u = (double)flx * ((double)ro.m[0] * ir);
        v = (double)fly * ((double)ro.m[1] * ir);
        w = zflip(k) * ((double)ro.m[2] * ir);
        so = solid_plane(k, cx, cy);
    };
    // edge slot at plane k into LDS buffer b
    auto put = [&](int k, int b) {
        if (own_slot) {
            su[b][wy][lane + 1] = u;
            fu[b][wy][lane + 1] = so;
            sv[b][wy + 1][lane] = v;
            fv[b][wy + 1][lane] = so;
        }
        if (hc != 0) {
            const double hv = (double)hf * ((double)rh.m[0] / (rh.r0 + (double)rh.rp));
            const bool hs = solid_plane(k, hcx, hcy);
            if (hc == 2) {
                const int r = wy == 0 ? 0 : kDivTy + 1;
                sv[b][r][lane] = hv;
                fv[b][r][lane] = hs;
            } else {
                const int i = lane < kDivTy ? 0 : kDivTx + 1;
                su[b][hy - y0][i] = hv;
                fu[b][hy - y0][i] = hs;
            }
        }
    };

    // plane z0 - 1 (own column, for w), then plane z0
    load_plane(z0 - 1);
    take_own(z0 - 1);
    double wm = w;
    bool sm = so;
    load_plane(z0);
    take_own(z0);
    put(z0, z0 & 1);
    double uc = u, vc = v, wc = w;
    bool sc = so;
    load_plane(z0 + 1);
    for (int k = z0; k < z1; ++k) {
        take_own(k + 1);                                   // plane k + 1 (own column)
        __syncthreads();
        if (k + 1 < z1) {
            put(k + 1, (k + 1) & 1);
            load_plane(k + 2);
        }
        if (out) {
            const int b = k & 1;
            double sum = 0.0;
            if (!sc) {
                const double ul = fu[b][wy][lane] ? -uc : su[b][wy][lane];
                const double ur = fu[b][wy][lane + 2] ? -uc : su[b][wy][lane + 2];
                sum += 0.5 * (ur - ul);
                const double vl = fv[b][wy][lane] ? -vc : sv[b][wy][lane];
                const double vr = fv[b][wy + 2][lane] ? -vc : sv[b][wy + 2][lane];
                sum += 0.5 * (vr - vl);
                const double wl = sm ? -wc : wm;
                const double wr = so ? -wc : w;
                sum += 0.5 * (wr - wl);
            }
            D[elem(x, y, k)] = T(sum);
        }
        wm = wc; sm = sc;
        uc = u; vc = v; wc = w; sc = so;
    }
}

template <typename T>
hipError_t launch_divergence(const Brick *bricks, const BlockMap *map, int nblocks, const T *state,
                             const double *base64, T *div, int skip, hipStream_t st)
{
    if (nblocks <= 0) return hipSuccess;
    hipLaunchKernelGGL((divergence_kernel<T>), dim3(nblocks), dim3(kDivTx * kDivTy), 0, st, bricks, map, state,
                       base64, div, skip);
    return hipGetLastError();
}

// ---------------------------------------------------------------------
// Flattening coefficients (formulas and constants with flat_pu, flat_raw
// and flat_pick): a kernel per pass axis writes the field of the pass's
// input, stored in the working precision.
// ---------------------------------------------------------------------

constexpr int kFlatChunk = 64;     // cells along the pass per thread (march form)
constexpr int kFlatXOut = 58;      // outputs per 64-lane row segment (x form)

// a copy of v as a new value (an identity DPP move)
__device__ __forceinline__ float aux_fresh(float v)
{
    const int b = __builtin_bit_cast(int, v);
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(b, b, 0xE4, 0xf, 0xf, false));
}
__device__ __forceinline__ double aux_fresh(double v)
{
    const unsigned long long bits = __builtin_bit_cast(unsigned long long, v);
    const int lo = __builtin_amdgcn_update_dpp((int)(unsigned)bits, (int)(unsigned)bits, 0xE4, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp((int)(unsigned)(bits >> 32), (int)(unsigned)(bits >> 32), 0xE4, 0xf,
                                               0xf, false);
    return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

template <typename T>
struct FlatRaw {
    T rp, mx, my, mz, ep;
    double r0, p0, fl;
};

template <typename T>
__device__ __forceinline__ void flat_load(const T *S, long fs, const double *r64, const double *p64, long e,
                                          double fl, FlatRaw<T> &r)
{
    r.rp = S[RHO * fs + e];
    r.mx = S[MX * fs + e];
    r.my = S[MY * fs + e];
    r.mz = S[MZ * fs + e];
    r.ep = S[EN * fs + e];
    r.r0 = r64[e];
    r.p0 = p64[e];
    r.fl = fl;
}

template <typename T>
__device__ __forceinline__ FlatRaw<T> flat_take(const FlatRaw<T> &r)
{
    return FlatRaw<T>{aux_fresh(r.rp), aux_fresh(r.mx), aux_fresh(r.my), aux_fresh(r.mz), aux_fresh(r.ep),
                      aux_fresh(r.r0), aux_fresh(r.p0), r.fl};
}

template <typename T>
__device__ __forceinline__ void flat_eval(const Geom &g, const FlatRaw<T> &r, int d, double &p, double &u)
{
    flat_pu(r.r0, r.p0, (double)r.rp, (double)r.mx, (double)r.my, (double)r.mz, (double)r.ep, g.gamma, d, r.fl,
            p, u);
}

int flat_blocks(const Geom &g, int axis)
{
    if (axis == 0) {
        const long items = (long)g.n[1] * g.n[2] * ((g.n[0] + kFlatXOut - 1) / kFlatXOut);
        return (int)((items + 3) / 4);
    }
    const int cb = 3 - axis;                     // the transverse axis other than x
    return ((g.n[0] + 63) / 64) * ((g.n[cb] + 3) / 4) * ((g.n[axis] + kFlatChunk - 1) / kFlatChunk);
}

// y and z passes: each thread marches a chunk of one pencil (lanes across
// x), windows of p (5 cells), u (4) and the raw coefficient (3).
template <typename T, int D>
__global__ __launch_bounds__(256) void flat_march_kernel(const Brick *bricks, const BlockMap *map, const T *arena,
                                                         const double *base64, T *flat, int skip)
{
    constexpr int CB = 3 - D;
    const BlockMap m = map[blockIdx.x];
    const Brick &B = bricks[m.brick];
    const Geom g = B.g;
    const T *S = arena + B.off;
    const long fs = g.fs;
    const double *r64 = base64 + B.boff, *p64 = base64 + B.boff + fs;
    T *F = flat + B.boff / 2;
    const int n = g.n[D], nx = g.n[0], ncb = g.n[CB];
    const int tx = (nx + 63) / 64, tb = (ncb + 3) / 4;
    const int x = (m.local % tx) * 64 + (int)(threadIdx.x & 63);
    const int b = ((m.local / tx) % tb) * 4 + (int)(threadIdx.x >> 6);
    int c0 = (m.local / (tx * tb)) * kFlatChunk;
    int c1 = min(c0 + kFlatChunk, n);
    const bool valid = x < nx && b < ncb;
    if (skip && g.sphere) {
        // the chunk's cells within kFlatReach of a fluid cell of one of the
        // wave's pencils (their union, so that every load is still a row)
        int lo = n, hi = -1;
        if (valid) {
            double xt[3];
            xt[0] = centre(g, 0, x);
            xt[CB] = centre(g, CB, b);
            xt[D] = 0.0;
            int flo, fhi;
            fluid_interval(g, D, xt, flo, fhi);
            if (flo <= fhi) {
                lo = max(c0, flo - kFlatReach);
                hi = min(c1 - 1, fhi + kFlatReach);
            }
        }
        for (int off = 1; off < 64; off <<= 1) {
            lo = min(lo, __shfl_xor(lo, off));
            hi = max(hi, __shfl_xor(hi, off));
        }
        c0 = lo;
        c1 = hi + 1;
    }
    if (!valid || c0 >= c1) return;
    const long sd = D == 1 ? g.px : g.plane, sb = CB == 1 ? g.px : g.plane;
    const long base = (long)x + (long)b * sb;
    double P[5] = { 0.0, 0.0, 0.0, 0.0, 0.0 }, U[4] = { 0.0, 0.0, 0.0, 0.0 }, R[3] = { 0.0, 0.0, 0.0 };
    auto load = [&](int t, FlatRaw<T> &r) {
        int fl = 1;
        const int s = (t >= 0 && t < n) ? t : bc_source(t, n, g.bc[D], fl);
        flat_load<T>(S, fs, r64, p64, base + (long)s * sd, (double)fl, r);
    };
    // Inputs loaded two cells ahead into two buffers used in turn (the loop
    // is unrolled by two): each step takes its buffer's values into new
    // registers, then loads cell t + 2 into it, so that no register copy at
    // the loop's end has to wait for a load in flight.
    auto step = [&](int t, FlatRaw<T> &buf) {
        const FlatRaw<T> cur = flat_take(buf);
        __builtin_amdgcn_sched_barrier(0);
        if (t + 2 <= c1 + 2) load(t + 2, buf);
        double pt, ut;
        flat_eval<T>(g, cur, D, pt, ut);
        P[0] = P[1]; P[1] = P[2]; P[2] = P[3]; P[3] = P[4]; P[4] = pt;
        U[0] = U[1]; U[1] = U[2]; U[2] = U[3]; U[3] = ut;
        if (t >= c0 + 1) {                       // raw coefficient of cell t - 2
            R[0] = R[1]; R[1] = R[2];
            R[2] = flat_raw(P[0], P[1], P[3], P[4], U[0], U[2]);
        }
        if (t >= c0 + 3)                         // coefficient of cell t - 3
            F[base + (long)(t - 3) * sd] = T(flat_pick(P[0], P[2], R[0], R[1], R[2]));
    };
    FlatRaw<T> ba, bb;
    load(c0 - 3, ba);
    load(c0 - 2, bb);
    int t = c0 - 3;
    for (; t + 1 <= c1 + 2; t += 2) {
        step(t, ba);
        step(t + 1, bb);
    }
    if (t <= c1 + 2) step(t, ba);
}

template <int CTRL>
__device__ __forceinline__ double aux_dpp(double v)
{
    const unsigned long long bits = __builtin_bit_cast(unsigned long long, v);
    const int lo = __builtin_amdgcn_update_dpp((int)(unsigned)bits, (int)(unsigned)bits, CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp((int)(unsigned)(bits >> 32), (int)(unsigned)(bits >> 32), CTRL, 0xf,
                                               0xf, false);
    return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double left_of(double v) { return aux_dpp<0x138>(v); }    // lane - 1
__device__ __forceinline__ double right_of(double v) { return aux_dpp<0x130>(v); }   // lane + 1

// x pass: one wave per 64-cell row segment (3 cells of halo each side),
// neighbours by DPP shifts taken on every lane.
template <typename T>
__global__ __launch_bounds__(256) void flat_x_kernel(const Brick *bricks, const BlockMap *map, const T *arena,
                                                     const double *base64, T *flat, int skip)
{
    const BlockMap m = map[blockIdx.x];
    const Brick &B = bricks[m.brick];
    const Geom g = B.g;
    const T *S = arena + B.off;
    const long fs = g.fs;
    const double *r64 = base64 + B.boff, *p64 = base64 + B.boff + fs;
    T *F = flat + B.boff / 2;
    const int nx = g.n[0];
    const int nseg = (nx + kFlatXOut - 1) / kFlatXOut;
    const long items = (long)g.n[1] * g.n[2] * nseg;
    const long item = (long)m.local * 4 + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    if (item >= items) return;                   // whole waves only
    const int lane = threadIdx.x & 63;
    const long rowi = item / nseg;
    const int seg = (int)(item - rowi * nseg);
    const int y = (int)(rowi % g.n[1]), z = (int)(rowi / g.n[1]);
    const long row = (long)y * g.px + (long)z * g.plane;
    const int i = seg * kFlatXOut - 3 + lane;
    int fl = 1;
    const int s = (i >= 0 && i < nx) ? i : bc_source(i, nx, g.bc[0], fl);
    double p, u;
    FlatRaw<T> r0;
    flat_load<T>(S, fs, r64, p64, row + s, (double)fl, r0);
    flat_eval<T>(g, r0, 0, p, u);
    const double pm1 = left_of(p), pp1 = right_of(p);
    const double pm2 = left_of(pm1), pp2 = right_of(pp1);
    const double um1 = left_of(u), up1 = right_of(u);
    const double r = flat_raw(pm2, pm1, pp1, pp2, um1, up1);
    const double rl = left_of(r), rr = right_of(r);
    const double f = flat_pick(pm1, pp1, rl, r, rr);
    if (lane >= 3 && lane < 3 + kFlatXOut && i < nx) F[row + i] = T(f);
}

template <typename T>
hipError_t launch_flattening(int axis, const Brick *bricks, const BlockMap *map, int nblocks, const T *state,
                             const double *base64, T *flat, int skip, hipStream_t st)
{
    if (nblocks <= 0) return hipSuccess;
    if (axis == 0)
        hipLaunchKernelGGL((flat_x_kernel<T>), dim3(nblocks), dim3(256), 0, st, bricks, map, state, base64, flat,
                           skip);
    else if (axis == 1)
        hipLaunchKernelGGL((flat_march_kernel<T, 1>), dim3(nblocks), dim3(256), 0, st, bricks, map, state, base64,
                           flat, skip);
    else
        hipLaunchKernelGGL((flat_march_kernel<T, 2>), dim3(nblocks), dim3(256), 0, st, bricks, map, state, base64,
                           flat, skip);
    return hipGetLastError();
}

__global__ void set_scalar_kernel(double *dst, double v)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) dst[0] = v;
}

__global__ void zero_u64_kernel(unsigned long long *dst, int count)
{
    for (int q = threadIdx.x; q < count; q += blockDim.x) dst[q] = 0ull;
}

hipError_t launch_set_scalar(double *dst, double v, hipStream_t st)
{
    hipLaunchKernelGGL(set_scalar_kernel, dim3(1), dim3(64), 0, st, dst, v);
    return hipGetLastError();
}

hipError_t launch_zero_u64(unsigned long long *dst, int count, hipStream_t st)
{
    hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(64), 0, st, dst, count);
    return hipGetLastError();
}

#define PPMB_INST(T)                                                                              \
    template hipError_t launch_prim_to_cons_range<T>(const Geom &, const double *const *,           \
                                                     const double *, T *, long, long, hipStream_t); \
    template hipError_t launch_cons_to_prim_range<T>(const Geom &, const T *, const double *,        \
                                                     double *, long, long, long, hipStream_t);     \
    template hipError_t launch_prim_to_cons<T>(const Geom &, const double *const *, const double *, \
                                               T *, hipStream_t);                                 \
    template hipError_t launch_gather<T>(const Geom &, int, const T *, double *, hipStream_t);      \
    template hipError_t launch_scatter<T>(const Geom &, int, const double *, T *, hipStream_t);     \
    template hipError_t launch_narrow<T>(const double *, T *, long, hipStream_t);                  \
    template hipError_t launch_cfl<T>(const Brick *, int, int, const BlockMap *, int, const T *,   \
                                      const double *, unsigned long long *, double, double *,     \
                                      hipStream_t);                                               \
    template hipError_t launch_totals<T>(const Geom &, const T *, const double *, const double *,  \
                                         double *, double *, hipStream_t);                          \
    template hipError_t launch_cfl_finish<T>(const Brick *, int, int, const BlockMap *, int, const T *, \
                                             const double *, unsigned long long *, unsigned long long *, \
                                             double, double *, hipStream_t);                              \
    template hipError_t launch_divergence<T>(const Brick *, const BlockMap *, int, const T *,          \
                                             const double *, T *, int, hipStream_t);                 \
    template hipError_t launch_flattening<T>(int, const Brick *, const BlockMap *, int, const T *,     \
                                             const double *, T *, int, hipStream_t);
PPMB_INST(float)
PPMB_INST(double)

}  // namespace ppmb
