// ppmb_rotation.hip -- the spin-up increment and the spherical-shell sums
// (gfx950).
//
// Sec. 3 adds a solid-body rotation to a run gradually, in the inertial
// frame; Sec. 1 describes the runs' averages over spherical surfaces.  Both
// kernels are FP64 throughout and built without FP contraction.  Neither is
// on the per-pass path: the increment runs once per step while a spin-up
// ramp lasts, the shell sums when a caller asks for them.
#include "ppmb_internal.h"

#include <climits>
#include <cmath>

namespace ppmb {

// ---------------------------------------------------------------------
// Spin-up increment: u += domega * (z-hat x x) = domega * (-y, x, 0) in
// every fluid cell, density and pressure perturbation unchanged:
//   m_x += rho du_x,  m_y += rho du_y,
//   E'  += m . du + rho |du|^2 / 2   (the kinetic-energy change at fixed p').
// In place on the current state arena; one thread per cell, the blocks of
// the CFL map (kCflBlockCells cells each, any number of bricks).
// ---------------------------------------------------------------------

template <typename T>
__global__ __launch_bounds__(256) void spin_kernel(const Brick *bricks, const BlockMap *map, T *arena,
                                                   const double *base64, double domega)
{
    const BlockMap m = map[blockIdx.x];
    const Brick &B = bricks[m.brick];
    const Geom g = B.g;
    const long nc = B.ncell;
    T *S = arena + B.off;
    const long fs = g.fs;
    const double *rho0 = base64 + B.boff;
    const long c0 = (long)m.local * kCflBlockCells;
    const long c1 = c0 + kCflBlockCells < nc ? c0 + kCflBlockCells : nc;
    for (long c = c0 + threadIdx.x; c < c1; c += blockDim.x) {
        const unsigned nx = (unsigned)g.n[0], ny = (unsigned)g.n[1];
        const unsigned row = (unsigned)c / nx, i = (unsigned)c - row * nx;
        const unsigned k = row / ny, j = row - k * ny;
        const double x = centre(g, 0, i), y = centre(g, 1, j);
        if (g.sphere && solid_at(g, x, y, centre(g, 2, k))) continue;
        const long e = (long)i + (long)j * g.px + (long)k * g.plane;
        const double rho = rho0[e] + (double)S[RHO * fs + e];
        const double mx = (double)S[MX * fs + e], my = (double)S[MY * fs + e];
        const double en = (double)S[EN * fs + e];
        const double dux = -domega * y, duy = domega * x;
        S[MX * fs + e] = T(mx + rho * dux);
        S[MY * fs + e] = T(my + rho * duy);
        S[EN * fs + e] = T(en + (mx * dux + my * duy) + 0.5 * rho * (dux * dux + duy * duy));
    }
}

template <typename T>
hipError_t launch_spin(const Brick *bricks, const BlockMap *map, int nblocks, T *state, const double *base64,
                       double domega, hipStream_t st)
{
    if (nblocks <= 0) return hipSuccess;
    hipLaunchKernelGGL((spin_kernel<T>), dim3(nblocks), dim3(256), 0, st, bricks, map, state, base64, domega);
    return hipGetLastError();
}

// ---------------------------------------------------------------------
// Rotating frame: axes turning at omega about the z axis through the
// coordinate origin add the Coriolis acceleration -2 omega z-hat x u =
// 2 omega (u_y, -u_x, 0) and, optionally, the centrifugal acceleration
// omega^2 (x, y, 0).  Applied at the end of a step over the brick's dt as
// a split step: half the centrifugal velocity change, the exact Coriolis
// rotation of (u_x, u_y) by -2 omega dt, the other half; density and
// pressure kept, m and E' rebuilt from the velocity.  FP64, one thread
// per cell over the blocks of the CFL map, in place.
// ---------------------------------------------------------------------

template <typename T>
__global__ __launch_bounds__(256) void rotframe_kernel(const Brick *bricks, const BlockMap *map, T *arena,
                                                       const double *base64, const double *dt, double omega,
                                                       int centrifugal)
{
    const BlockMap m = map[blockIdx.x];
    const Brick &B = bricks[m.brick];
    const Geom g = B.g;
    const long nc = B.ncell;
    T *S = arena + B.off;
    const long fs = g.fs;
    const double *rho0 = base64 + B.boff;
    const double dtb = dt[B.dti];
    const double th = -2.0 * omega * dtb;
    double sth, cth;
    sincos(th, &sth, &cth);
    const double kick = centrifugal ? 0.5 * omega * omega * dtb : 0.0;
    const double gm1 = g.gamma - 1.0;
    const long c0 = (long)m.local * kCflBlockCells;
    const long c1 = c0 + kCflBlockCells < nc ? c0 + kCflBlockCells : nc;
    for (long c = c0 + threadIdx.x; c < c1; c += blockDim.x) {
        const unsigned nx = (unsigned)g.n[0], ny = (unsigned)g.n[1];
        const unsigned row = (unsigned)c / nx, i = (unsigned)c - row * nx;
        const unsigned k = row / ny, j = row - k * ny;
        const double x = centre(g, 0, i), y = centre(g, 1, j);
        if (g.sphere && solid_at(g, x, y, centre(g, 2, k))) continue;
        const long e = (long)i + (long)j * g.px + (long)k * g.plane;
        const double rho = rho0[e] + (double)S[RHO * fs + e];
        const double mx = (double)S[MX * fs + e], my = (double)S[MY * fs + e], mz = (double)S[MZ * fs + e];
        const double en = (double)S[EN * fs + e];
        double u = mx / rho, v = my / rho;
        const double w = mz / rho;
        const double pp = gm1 * (en - 0.5 * (mx * u + my * v + mz * w));
        u += kick * x;
        v += kick * y;
        const double ur = cth * u - sth * v, vr = sth * u + cth * v;
        u = ur + kick * x;
        v = vr + kick * y;
        S[MX * fs + e] = T(rho * u);
        S[MY * fs + e] = T(rho * v);
        S[EN * fs + e] = T(pp / gm1 + 0.5 * rho * ((u * u + v * v) + w * w));
    }
}

template <typename T>
hipError_t launch_rotframe(const Brick *bricks, const BlockMap *map, int nblocks, T *state, const double *base64,
                           const double *dt, double omega, int centrifugal, hipStream_t st)
{
    if (nblocks <= 0) return hipSuccess;
    hipLaunchKernelGGL((rotframe_kernel<T>), dim3(nblocks), dim3(256), 0, st, bricks, map, state, base64, dt,
                       omega, centrifugal);
    return hipGetLastError();
}

// ---------------------------------------------------------------------
// Shell sums.  Shell b holds the fluid cells whose centre has
// (b dr)^2 <= r^2 < ((b+1) dr)^2, r^2 = (x^2 + y^2) + z^2 in FP64; per shell
// eight sums of dV times: 1, rho, f0, rho u_r, rho u_r^2, rho |u|^2,
// rho (x u_y - y u_x), f0^2 (u_r = x.u / r, 0 at r = 0), from the momenta:
// rho u_r = x.m / r, rho u_r^2 = (x.m / r)^2 / rho, rho |u|^2 = |m|^2 / rho.
//
// Along an x-row r^2 = x^2 + const falls for x < 0 and rises for x >= 0, so
// on each side of x = 0 the cells of one shell are one contiguous run.
// Block b walks a fixed run of rows in chunks of 64 cells, its waves
// taking the chunks in turn (each wave's next chunk in flight while the
// current one is reduced); a segmented inclusive scan over the lanes (runs
// = equal shell and side) leaves each run's sum in its last lane, which
// adds it to the block's shell array in LDS, the x < 0 side first: the
// runs of one side have distinct shells, so no two lanes of one LDS update
// share an address.  The waves of a block update the array one after the
// other, separated by barriers, so that it receives the chunks in chunk
// order.  The block arrays go to `work`; they are added per (shell,
// quantity) in two fixed levels (groups of consecutive blocks, then the
// groups).  Every association is fixed, so the result is bitwise
// reproducible, and the same for any number of waves per block.
// ---------------------------------------------------------------------

// shell of a radius: a first guess from r / dr, then the squared bounds
// decide (so the guess only has to be close)
__device__ __forceinline__ int shell_of(double r2, double r, double inv_dr, double dr, int nbins)
{
    int b = (int)(r * inv_dr);
    b = b < 0 ? 0 : (b > nbins - 1 ? nbins - 1 : b);
    while (b > 0 && __dmul_rn((double)b * dr, (double)b * dr) > r2) --b;
    while (b < nbins - 1 && __dmul_rn((double)(b + 1) * dr, (double)(b + 1) * dr) <= r2) ++b;
    return b;
}

// one lane's cell of a chunk: where it is, its shell key, its raw inputs
template <typename T>
struct ShellCell {
    int key;              // 2 shell + (x >= 0), -1 if the cell takes no part
    double x, y, z, r;
    double r0;
    T rp, mx, my, mz, f;
};

// Cross-lane moves of the shell kernel's scan (DPP: a VALU operand, no LDS
// round trip).  Within a row of 16 lanes row_shr:n reads the lane n below
// (a lane whose source lies below its row reads 0); row_bcast:15 gives
// rows 1 and 3 (row mask 0xa) lane 15 of the row below, row_bcast:31 gives
// rows 2 and 3 (row mask 0xc) lane 31; lanes of rows the mask leaves out
// read 0.  wave_shr:1 / wave_shl:1 read lane l - 1 / l + 1 (0 past the
// wave's ends).
constexpr int kRowShr = 0x110;
constexpr int kRowBcast15 = 0x142;
constexpr int kRowBcast31 = 0x143;
constexpr int kWaveShr1 = 0x138;
constexpr int kWaveShl1 = 0x130;

template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_f64(double v)
{
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, ROWS, 0xf, true);
    const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, ROWS, 0xf, true);
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// One step of the segmented scan: a lane's window (the lanes whose values
// its partial holds) grows by the source lane's window unless it already
// holds a run head; a source outside the row or the mask gives 0 and no
// head, which leaves the lane as it was.
template <int CTRL, int ROWS>
__device__ __forceinline__ void seg_step(double v[8], int &head)
{
    const int hup = __builtin_amdgcn_update_dpp(0, head, CTRL, ROWS, 0xf, true);
    double up[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) up[q] = dpp_f64<CTRL, ROWS>(v[q]);
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = head ? v[q] : up[q] + v[q];
    head |= hup;
}

template <typename T, int W>
__global__ __launch_bounds__(64 * W) void shell_kernel(Geom g, const T *S, const double *rho0, int nbins,
                                                       double dr, int rows_per_block, double *work)
{
    extern __shared__ double bins[];           // 8 * nbins, quantity-major: bins[q * nbins + shell]
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    for (int q = threadIdx.x; q < nbins * 8; q += 64 * W) bins[q] = 0.0;
    __syncthreads();
    const int ny = g.n[1];
    const long nrows = (long)ny * g.n[2];
    const long r0 = (long)blockIdx.x * rows_per_block;
    const long r1 = r0 + rows_per_block < nrows ? r0 + rows_per_block : nrows;
    const int cpr = (g.n[0] + 63) / 64;        // chunks per row
    const long nchunk = (r1 - r0) * cpr;
    const double rmax = (double)nbins * dr;
    const double rmax2 = __dmul_rn(rmax, rmax);
    const double inv_dr = 1.0 / dr;
    const long fs = g.fs;

    // chunk c of the block: 64 cells of row r0 + c / cpr
    auto fetch = [&](long c, ShellCell<T> &cell) {
        const long row = r0 + c / cpr;
        const int ci = (int)(c - (row - r0) * cpr);
        const int j = (int)(row % ny), k = (int)(row / ny);
        const int i = ci * 64 + lane;
        const bool in = i < g.n[0];
        cell.x = centre(g, 0, in ? i : 0);
        cell.y = centre(g, 1, j);
        cell.z = centre(g, 2, k);
        const long e = (long)(in ? i : 0) + (long)j * g.px + (long)k * g.plane;
        const double r2 = r2_exact(cell.x, cell.y, cell.z);
        cell.r = sqrt(r2);
        cell.key = -1;
        if (in && !(g.sphere && r2 >= g.sphere_t) && r2 < rmax2)
            cell.key = 2 * shell_of(r2, cell.r, inv_dr, dr, nbins) + (cell.x >= 0.0 ? 1 : 0);
        cell.r0 = 0.0;
        cell.rp = cell.mx = cell.my = cell.mz = cell.f = T(0);
        if (cell.key >= 0) {                   // solid cells and cells beyond the shells: no loads
            cell.r0 = rho0[e];
            cell.rp = S[RHO * fs + e];
            cell.mx = S[MX * fs + e];
            cell.my = S[MY * fs + e];
            cell.mz = S[MZ * fs + e];
            cell.f = S[F0 * fs + e];
        }
    };

    // Wave wv takes chunks wv, wv + W, ...; the W waves of a block add their
    // chunks' runs to the bins in turn, so the bins receive the chunks in
    // chunk order whatever W is (the same sums, bit for bit).
    ShellCell<T> cur, nxt;
    if (wv < nchunk) fetch(wv, cur);
    const long niter = (nchunk + W - 1) / W;
    for (long t = 0; t < niter; ++t) {
        const long c = t * W + wv;
        // this wave's next chunk goes in flight first
        if (c + W < nchunk) fetch(c + W, nxt);
        const int key = c < nchunk ? cur.key : -1;
        const bool any = __ballot(key >= 0) != 0;   // some cell of this chunk takes part
        double v[8];
        bool last = false;
        if (any) {
            {
                const bool on = key >= 0;
                const double rho = cur.r0 + (double)cur.rp;
                const double irho = on ? 1.0 / rho : 0.0;
                const double mx = (double)cur.mx, my = (double)cur.my, mz = (double)cur.mz;
                const double f = (double)cur.f;
                const double mr = cur.r > 0.0 ? ((cur.x * mx + cur.y * my) + cur.z * mz) / cur.r : 0.0;
                v[0] = on ? 1.0 : 0.0;
                v[1] = on ? rho : 0.0;
                v[2] = on ? f : 0.0;
                v[3] = on ? mr : 0.0;
                v[4] = on ? mr * mr * irho : 0.0;
                v[5] = on ? ((mx * mx + my * my) + mz * mz) * irho : 0.0;
                v[6] = on ? cur.x * my - cur.y * mx : 0.0;
                v[7] = on ? f * f : 0.0;
            }
            // segmented inclusive scan over the runs of equal keys, by DPP
            // row shifts within each 16-lane row and then the two row
            // broadcasts: a lane whose window has met no run head adds the
            // partial of the lane the step names; the steps stop once every
            // window that could still grow already meets a head
            const int kprev = __builtin_amdgcn_update_dpp(0, key, kWaveShr1, 0xf, 0xf, true);
            int head = (lane == 0 || kprev != key) ? 1 : 0;
            seg_step<kRowShr + 1, 0xf>(v, head);
            if (__ballot(lane >= 2 && !head)) {
                seg_step<kRowShr + 2, 0xf>(v, head);
                if (__ballot(lane >= 4 && !head)) {
                    seg_step<kRowShr + 4, 0xf>(v, head);
                    if (__ballot(lane >= 8 && !head)) {
                        seg_step<kRowShr + 8, 0xf>(v, head);
                        if (__ballot(lane >= 16 && !head)) {
                            seg_step<kRowBcast15, 0xa>(v, head);
                            if (__ballot(lane >= 32 && !head)) seg_step<kRowBcast31, 0xc>(v, head);
                        }
                    }
                }
            }
            const int knext = __builtin_amdgcn_update_dpp(0, key, kWaveShl1, 0xf, 0xf, true);
            last = key >= 0 && (lane == 63 || knext != key);
        }
        for (int u = 0; u < W; ++u) {
            if (u == wv && any) {
                for (int side = 0; side < 2; ++side) {
                    if (last && (key & 1) == side) {
                        // the runs' shells are consecutive along a side, so
                        // the lanes of one update hit consecutive doubles
                        // (no bank conflicts beyond those of a plain row
                        // access)
                        const int b = key >> 1;
#pragma unroll
                        for (int q = 0; q < 8; ++q) bins[q * nbins + b] += v[q];
                    }
                }
            }
            if constexpr (W > 1) __syncthreads();
        }
        cur = nxt;
    }
    __syncthreads();
    double *P = work + (long)blockIdx.x * nbins * 8;
    for (int t = threadIdx.x; t < nbins * 8; t += 64 * W) P[t] = bins[(t & 7) * nbins + (t >> 3)];   // out: 8 shell + quantity
}

// Waves per block of the shell kernel (they share the block's bins).
constexpr int kShellWaves = 4;

// Block partials are added in two fixed levels: groups of kShellGroup
// consecutive blocks (in block order), then the group sums (in group order).
constexpr int kShellGroup = 64;

__global__ __launch_bounds__(256) void shell_group_kernel(const double *work, int nblocks, int m, double *gsum)
{
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t >= m) return;
    const int b0 = blockIdx.y * kShellGroup;
    const int b1 = b0 + kShellGroup < nblocks ? b0 + kShellGroup : nblocks;
    double s = 0.0;
    int b = b0;
    for (; b + 8 <= b1; b += 8) {               // loads in flight together, adds in block order
        double a[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) a[u] = work[(long)(b + u) * m + t];
#pragma unroll
        for (int u = 0; u < 8; ++u) s += a[u];
    }
    for (; b < b1; ++b) s += work[(long)b * m + t];
    gsum[(long)blockIdx.y * m + t] = s;
}

__global__ __launch_bounds__(256) void shell_finish_kernel(const double *gsum, int ngroups, int m, double dv,
                                                           double *out)
{
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t >= m) return;
    double s = 0.0;
    for (int gi = 0; gi < ngroups; ++gi) s += gsum[(long)gi * m + t];
    out[t] = s * dv;
}

int shell_blocks(const Geom &g, int *rows_per_block)
{
    const long nrows = (long)g.n[1] * g.n[2];
    long nb = nrows < kShellMaxBlocks ? nrows : kShellMaxBlocks;
    const long rpb = (nrows + nb - 1) / nb;
    *rows_per_block = (int)rpb;
    return (int)((nrows + rpb - 1) / rpb);
}

long shell_work_doubles(const Geom &g, int nbins)
{
    int rpb = 0;
    const long nb = shell_blocks(g, &rpb);
    return 8L * nbins * (nb + (nb + kShellGroup - 1) / kShellGroup);
}

template <typename T>
hipError_t launch_shell(const Geom &g, const T *state, const double *rho0, int nbins, double dr, double *work,
                        double *out, hipStream_t st)
{
    int rpb = 0;
    const int nb = shell_blocks(g, &rpb);
    const size_t lds = sizeof(double) * 8 * (size_t)nbins;
    const int m = nbins * 8, ng = (nb + kShellGroup - 1) / kShellGroup;
    double *gsum = work + (long)nb * m;
    hipLaunchKernelGGL((shell_kernel<T, kShellWaves>), dim3(nb), dim3(64 * kShellWaves), lds, st, g, state, rho0, nbins,
                       dr, rpb, work);
    hipLaunchKernelGGL(shell_group_kernel, dim3((m + 255) / 256, ng), dim3(256), 0, st, work, nb, m, gsum);
    hipLaunchKernelGGL(shell_finish_kernel, dim3((m + 255) / 256), dim3(256), 0, st, gsum, ng, m,
                       g.dx * g.dx * g.dx, out);
    return hipGetLastError();
}

#define PPMB_ROT_INST(T)                                                                          \
    template hipError_t launch_spin<T>(const Brick *, const BlockMap *, int, T *, const double *,  \
                                       double, hipStream_t);                                      \
    template hipError_t launch_rotframe<T>(const Brick *, const BlockMap *, int, T *,              \
                                           const double *, const double *, double, int,           \
                                           hipStream_t);                                          \
    template hipError_t launch_shell<T>(const Geom &, const T *, const double *, int, double,       \
                                        double *, double *, hipStream_t);
PPMB_ROT_INST(float)
PPMB_ROT_INST(double)

}  // namespace ppmb
