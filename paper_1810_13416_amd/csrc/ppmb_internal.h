// ppmb_internal.h -- declarations shared by the translation units of the
// HIP library (kernels, launchers and the C-ABI runtime).
#pragma once
#include <hip/hip_runtime.h>

#include "ppmb_dev.h"

namespace ppmb {

// One brick of a batch (a single grid is a batch of one): its grid and where
// its fields live.  State arena: field q of the brick at off + q * g.fs, in
// the pitched layout of Geom.  Base arena (working precision and FP64
// alike, same layout): rho0 at boff, p0 at boff + g.fs.  ncell = nx ny nz.
// Its time step is dt[dti].
struct Brick {
    Geom g;
    long off;
    long boff;
    long ncell;
    int dti;
    int pad;
};

// One entry per block of a launch: the brick it works on and its index
// among that brick's blocks.
struct BlockMap {
    int brick;
    int local;
};

// Launch shape of the pass kernels: waves per block for the marching
// kernel (y and z passes) and the lanes-along-x kernel (x pass).
struct PassShape {
    int march_waves;
    int x_waves;
    int march_chunk;      // cells per wave along the pencil (0: the whole pencil)
    int x_rows;           // x pass: at least this many rows per wave (0: by the marching kernel)
};

// Number of blocks the pass along `axis` needs for one brick.
int pass_blocks(const Geom &g, int axis, const PassShape &sh);

// Estimated work of block `local` of that pass when solid cells are
// skipped (the cells its waves march over); the block maps list a brick's
// blocks longest first, so that the short ones fill the end of a launch.
double pass_block_cost(const Geom &g, int axis, const PassShape &sh, int local);

// Event counters (limiter, unsmooth, Riemann) are spread over slots a
// cache line apart, one for each residue of the block index, so that the
// waves' atomic adds (one per wave and counter) do not all queue on one
// address; readers sum the slots.  Element 3 of slot 0 is the Courant-check
// flag, which no pass adds to.
constexpr int kCntSlots = 64;
constexpr int kCntStride = 16;                      // words per slot: 128 bytes
constexpr int kCntWords = kCntSlots * kCntStride;

// Fused 1-D pass along `axis` for the bricks whose blocks are
// map[0 .. nblocks): one launch, every brick's pencils.  With `cfl` set the
// pass also folds the signal speed of the fluid cells it writes into the
// CFL reduction slots work[2 brick] (max, as in the CFL kernel) and
// work[2 brick + 1] (non-physical flag): the exact FP64 speed of every cell
// whose working-precision bound reaches the band edge cband[2 brick] (FP64
// bits, set by launch_cfl_arm), so the slot holds the exact maximum
// whenever that maximum reaches the edge; base64 is the FP64 base arena.
// With dissk > 0 the shock dissipation is added at every face between fluid
// cells from `div` (launch_divergence of the pass input or of the state at
// the start of the step).  With `flat` every parabola is flattened by its
// cell's coefficient: the marching kernel reads it from `flat`
// (launch_flattening of the pass input along `axis`), the lanes-along-x
// kernel evaluates it itself.
// With `skip` (solid cells hold the same values in `in` and `out`) the
// pass neither loads nor writes solid cells farther than the stencil reach
// from a fluid cell: a wave of pencils marches over the union of their
// fluid intervals, the x pass visits only the 56-cell segments holding
// fluid cells.
template <typename T>
hipError_t launch_sweep(int axis, const PassShape &sh, const Brick *bricks, const BlockMap *map,
                        int nblocks, const T *in, T *out, const T *base, const double *dt,
                        unsigned long long *counters, int heat, const double *base64,
                        unsigned long long *work, const unsigned long long *cband, const T *div, double dissk,
                        const T *flat, int cfl, int skip, hipStream_t st);

// Undivided velocity divergence of every cell of the bricks whose blocks
// are map[0 .. nblocks) (div_blocks(g) blocks per brick; FP64 arithmetic,
// stored in the working precision): field of brick B at div + B.boff / 2,
// pitched like the state; 0 in solid cells.  With `skip` a sphere's tiles
// write only the planes that can hold fluid cells of their columns (the
// passes read the divergence of fluid cells only); the others keep what
// they held.
int div_blocks(const Geom &g);
template <typename T>
hipError_t launch_divergence(const Brick *bricks, const BlockMap *map, int nblocks, const T *state,
                             const double *base64, T *div, int skip, hipStream_t st);

// Flattening coefficients (Colella & Woodward 1984, Sec. 4) of every cell
// of the bricks whose blocks are map[0 .. nblocks) (flat_blocks(g, axis)
// per brick) for a pass along `axis`, from `state` (FP64 arithmetic, stored
// in the working precision): field of brick B at flat + B.boff / 2.  With
// `skip` a sphere's coefficients are written only within kFlatReach cells
// of the fluid cells along the pass (a fluid cell's update uses the
// parabolas of its two neighbours); the others keep what they held.
int flat_blocks(const Geom &g, int axis);
constexpr int kFlatReach = 4;
template <typename T>
hipError_t launch_flattening(int axis, const Brick *bricks, const BlockMap *map, int nblocks, const T *state,
                             const double *base64, T *flat, int skip, hipStream_t st);

// hydrostatic base state: FP64 RK4 node table (one thread), then cell values
hipError_t launch_base_state(const Geom &g, int kind, const double *params, double *table,
                             long table_len, double *rho0, double *p0, hipStream_t st);

// Conversions between FP64 primitive perturbations (dense, x fastest) and
// the stored conserved fields of the working precision (pitched layout of
// Geom).  The range forms take dense cells [c0, c0 + m) of one brick: the
// primitive side holds exactly those cells (field q at prim[q], or at
// out + q * ostride), state and rho0 are the brick's whole pitched arrays.
template <typename T>
hipError_t launch_prim_to_cons(const Geom &g, const double *const *prim, const double *rho0,
                               T *state, hipStream_t st);
template <typename T>
hipError_t launch_prim_to_cons_range(const Geom &g, const double *const *prim, const double *rho0,
                                     T *state, long c0, long m, hipStream_t st);
template <typename T>
hipError_t launch_cons_to_prim_range(const Geom &g, const T *state, const double *rho0, double *out,
                                     long c0, long m, long ostride, hipStream_t st);
// nf pitched fields of a brick (stride g.fs) to / from dense FP64 (field q
// at q * ncell)
template <typename T>
hipError_t launch_gather(const Geom &g, int nf, const T *src, double *dst, hipStream_t st);
template <typename T>
hipError_t launch_scatter(const Geom &g, int nf, const double *src, T *dst, hipStream_t st);
// plain element-wise FP64 -> T copy
template <typename T>
hipError_t launch_narrow(const double *src, T *dst, long count, hipStream_t st);

// CFL reduction for bricks [b0, b0 + nb): per brick the uint64 image of the
// FP64 maximum of |u_d| + c in work[2 brick], a sticky non-physical flag in
// work[2 brick + 1], then dt[dti] = cfl dx / smax.  `map` covers nblocks
// blocks of kCflBlockCells cells each.
constexpr int kCflBlockCells = 65536;
int cfl_blocks(long ncell);
template <typename T>
hipError_t launch_cfl(const Brick *bricks, int b0, int nb, const BlockMap *map, int nblocks,
                      const T *state, const double *base64, unsigned long long *work, double cfl,
                      double *dt, hipStream_t st);

// conserved totals with a fixed reduction tree; out[8] on the device
template <typename T>
hipError_t launch_totals(const Geom &g, const T *state, const double *rho0, const double *p0,
                         double *partials, double *out, hipStream_t st);
constexpr int kTotalsBlocks = 1024;

// The fused reduction of the last pass, around it.  Arm (before the pass):
// per brick of [b0, b0 + nb) the band edge cband[2 brick] = (1 - kCflBand)
// times the maximum now in work[2 brick] (that of the state the pass
// starts from), then zero that maximum.  Finish (before the next step):
// dt = cfl dx / max where the maximum reached the edge; the other bricks
// (whose fastest cell may have been passed over) get a full CFL reduction
// over the blocks of `map` (nblocks, CFL block map of the same bricks) and
// then their dt.  Every launch is a kernel: no host decision, graph-safe.
constexpr double kCflBand = 1e-4;
hipError_t launch_cfl_arm(unsigned long long *work, unsigned long long *cband, int b0, int nb, hipStream_t st);
// Courant check of a caller-given dt for bricks [b0, b0 + nb): with
// dt[dti] = courant_max dx / smax from launch_cfl, set *flag where
// given > dt[dti]; then dt[dti] = given.
hipError_t launch_cfl_given(const Brick *bricks, int b0, int nb, double given, double *dt,
                            unsigned long long *flag, hipStream_t st);
template <typename T>
hipError_t launch_cfl_finish(const Brick *bricks, int b0, int nb, const BlockMap *map, int nblocks,
                             const T *state, const double *base64, unsigned long long *work,
                             unsigned long long *cband, double cfl, double *dt, hipStream_t st);

// Spin-up increment (Sec. 3): velocity += domega * (-y, x, 0) in every
// fluid cell of the bricks the CFL block map covers, in place, p' kept.
template <typename T>
hipError_t launch_spin(const Brick *bricks, const BlockMap *map, int nblocks, T *state, const double *base64,
                       double domega, hipStream_t st);

// Rotating-frame sources (Coriolis, optionally centrifugal, about the z
// axis at omega) over each brick's dt[dti], in every fluid cell of the
// bricks the CFL block map covers, in place.
template <typename T>
hipError_t launch_rotframe(const Brick *bricks, const BlockMap *map, int nblocks, T *state, const double *base64,
                           const double *dt, double omega, int centrifugal, hipStream_t st);

// Spherical-shell sums (8 per shell, FP64, fixed order) of one brick:
// block partials and group sums in work (shell_work_doubles(g, nbins)
// doubles), result out[8 * shell + quantity] on the device, times dV.
constexpr int kShellMaxBins = 1024;
constexpr int kShellMaxBlocks = 4096;
int shell_blocks(const Geom &g, int *rows_per_block);
long shell_work_doubles(const Geom &g, int nbins);
template <typename T>
hipError_t launch_shell(const Geom &g, const T *state, const double *rho0, int nbins, double dr, double *work,
                        double *out, hipStream_t st);

hipError_t launch_set_scalar(double *dst, double v, hipStream_t st);
hipError_t launch_zero_u64(unsigned long long *dst, int count, hipStream_t st);

// ---------------------------------------------------------------------
// Pieces of the CFL reduction, used alike by its own kernels and by the
// persistent step kernel, so that both give the same dt bit for bit.
// ---------------------------------------------------------------------

// Threads t, t + nthr, ... of CFL block m (nthr threads share the block):
// the FP64 maximum of |u_d| + c over their fluid cells and the
// non-physical flag, folded per wave into work[2 brick] (positive doubles
// order like their bits) and work[2 brick + 1].  Every lane of the wave
// calls it.
template <typename T>
__device__ __forceinline__ void cfl_block_part(const Brick *bricks, BlockMap m, const T *arena,
                                               const double *base64, unsigned long long *work, int t, int nthr)
{
    const Brick &B = bricks[m.brick];
    const Geom g = B.g;
    const long nc = B.ncell;
    const T *S = arena + B.off;
    const long fs = g.fs;
    const double *rho0 = base64 + B.boff, *p0 = base64 + B.boff + fs;
    const long c0 = (long)m.local * kCflBlockCells;
    const long c1 = c0 + kCflBlockCells < nc ? c0 + kCflBlockCells : nc;
    double smax = 0.0;
    bool bad = false;
    for (long c = c0 + t; c < c1; c += nthr) {
        const unsigned nx = (unsigned)g.n[0], ny = (unsigned)g.n[1];
        const unsigned row = (unsigned)c / nx, i = (unsigned)c - row * nx;
        const unsigned k = row / ny, j = row - k * ny;
        if (g.sphere && solid_at(g, centre(g, 0, i), centre(g, 1, j), centre(g, 2, k))) continue;
        const long e = (long)i + (long)j * g.px + (long)k * g.plane;
        bool b;
        const double sp = cell_speed(rho0[e], p0[e], (double)S[RHO * fs + e], (double)S[MX * fs + e],
                                     (double)S[MY * fs + e], (double)S[MZ * fs + e],
                                     (double)S[EN * fs + e], g.gamma, b);
        if (b) bad = true;
        else if (sp > smax) smax = sp;
    }
    for (int off = 32; off > 0; off >>= 1) smax = fmax(smax, __shfl_down(smax, off));
    const unsigned long long bb = __ballot(bad);
    if ((threadIdx.x & 63) == 0) {
        // a wave of solid cells has nothing to add (the maximum starts at 0)
        if (smax > 0.0) atomicMax(&work[2 * m.brick], (unsigned long long)__double_as_longlong(smax));
        if (bb) atomicOr(&work[2 * m.brick + 1], 1ull);
    }
}

// ---------------------------------------------------------------------
// Flattening near strong shocks (Colella & Woodward 1984, Sec. 4), the
// companion of the shock dissipation: per cell and pass axis d, from the
// full pressure p over three cells each side and the velocity u along d
// over two, neighbours through the boundary conditions (a reflecting
// image's u flipped):
//   raw(i) = 0 unless |p(i+1) - p(i-1)| > eps min(p(i+1), p(i-1)) and
//            u(i-1) - u(i+1) > tie (|u(i-1)| + |u(i+1)|); else
//            min(1, max(0, w2 (z - w1))),
//            z = (p(i+1) - p(i-1)) / (p(i+2) - p(i-2)) (0 if that is 0);
//   f(i)   = max(raw(i), raw(i + 1)) if p(i+1) < p(i-1), max(raw(i),
//            raw(i - 1)) if p(i+1) > p(i-1), max of all three when
//            |p(i+1) - p(i-1)| <= tie (p(i+1) + p(i-1)).
// The tie margins keep the decisions off values that are equal but for
// rounding.  FP64 arithmetic without contraction, so that the flattening
// kernels and the x pass (which evaluates the coefficients of its own
// segment) take the same decisions.
// ---------------------------------------------------------------------

constexpr double kFlatEps = 0.33, kFlatW1 = 0.75, kFlatW2 = 10.0, kFlatTie = 1e-10;

// Full pressure and the velocity along d of one cell (flip fl on u), each
// velocity a correctly rounded quotient m / rho: the compression test
// compares two velocities that are often equal but for rounding (a uniform
// transverse flow after a pass).
__device__ __forceinline__ void flat_pu(double r0, double p0, double rp, double mx, double my, double mz,
                                        double ep, double gamma, int d, double fl, double &p, double &u)
{
#pragma clang fp contract(off)
    const double rho = r0 + rp;
    const double vx = mx / rho, vy = my / rho, vz = mz / rho;
    p = p0 + (gamma - 1.0) * (ep - 0.5 * (mx * vx + my * vy + mz * vz));
    u = fl * (d == 0 ? vx : (d == 1 ? vy : vz));
}

// the coefficient from the raw values of the cell and its two neighbours
__device__ __forceinline__ double flat_pick(double pm1, double pp1, double rm, double r0, double rp)
{
#pragma clang fp contract(off)
    const double dp = pp1 - pm1;
    double nb;
    if (fabs(dp) <= kFlatTie * (pp1 + pm1)) nb = fmax(rm, rp);
    else nb = dp < 0.0 ? rp : rm;
    return fmax(r0, nb);
}

__device__ __forceinline__ double flat_raw(double pm2, double pm1, double pp1, double pp2, double um1, double up1)
{
#pragma clang fp contract(off)
    const double dp1 = pp1 - pm1, dp2 = pp2 - pm2;
    const bool cand = fabs(dp1) > kFlatEps * fmin(pp1, pm1) && um1 - up1 > kFlatTie * (fabs(um1) + fabs(up1));
    if (!cand) return 0.0;
    const double z = dp2 != 0.0 ? dp1 / dp2 : 0.0;
    return fmin(1.0, fmax(0.0, kFlatW2 * (z - kFlatW1)));
}

// Brick k after the fused reduction of its last pass: dt where the maximum
// reached the band edge, else clear the maximum and raise the redo flag.
__device__ __forceinline__ void cfl_check_brick(const Brick *bricks, int k, unsigned long long *work,
                                                unsigned long long *cband, double cfl, double *dt)
{
    const Brick &B = bricks[k];
    const double smax = __longlong_as_double((long long)work[2 * k]);
    const double edge = __longlong_as_double((long long)cband[2 * k]);
    if (smax >= edge) {
        dt[B.dti] = cfl * B.g.dx / smax;
        cband[2 * k + 1] = 0ull;
    } else {
        work[2 * k] = 0ull;
        cband[2 * k + 1] = 1ull;
    }
}

// Brick k after its redo reduction (if its flag is raised): dt, flag cleared.
__device__ __forceinline__ void cfl_redo_finish_brick(const Brick *bricks, int k, const unsigned long long *work,
                                                      unsigned long long *cband, double cfl, double *dt)
{
    if (cband[2 * k + 1] == 0ull) return;
    const Brick &B = bricks[k];
    dt[B.dti] = cfl * B.g.dx / __longlong_as_double((long long)work[2 * k]);
    cband[2 * k + 1] = 0ull;
}

// Brick k before the pass that reduces: band edge from the maximum of the
// state the pass starts from, then that maximum cleared.
__device__ __forceinline__ void cfl_arm_brick(unsigned long long *work, unsigned long long *cband, int k)
{
    const double prev = __longlong_as_double((long long)work[2 * k]);
    cband[2 * k] = (unsigned long long)__double_as_longlong(prev * (1.0 - kCflBand));
    work[2 * k] = 0ull;
}

// ---------------------------------------------------------------------
// Persistent step: the three passes of every brick (and the dt of the
// step, from the maxima its previous step's last pass left) in one launch
// of resident waves that take work items in order from a counter.  Stages,
// in item order:
//   0 check (one item per brick)         4 pass order[0] (its waves)
//   1 redo reduction (4 per CFL block)   5 pass order[1]
//   2 finish (one per brick)             6 pass order[2] (fused reduction)
//   3 arm (one per brick)
// An item of brick b waits until cnt[b] counts every item of b in the
// earlier stages (need[stage * nb + b]); items only wait on items of lower
// index, which were taken earlier by running waves, so the waits end
// without any assumption on how many waves are resident.  A wait that
// outlasts a bounded time raises ctl[1] and gives up (the step's result is
// then invalid, reported by the next synchronising call).  cnt[0 .. nb)
// and ctl = cnt + nb (2 words) must be zero at launch, in memory that is
// coherent while a kernel runs (fine-grained).  The passes go
// a0 -> a1 -> a0 -> a1 (the state starts in a0 and ends in a1); the redo
// reduction reads a0.
// ---------------------------------------------------------------------
constexpr int kStepStages = 7;
template <typename T>
hipError_t launch_step(const PassShape &sh, const Brick *bricks, int nb, const int order[3],
                       const BlockMap *const maps[3], const int nblocks[3], const BlockMap *cmap, int ncblocks,
                       const int *need, unsigned long long *cnt, T *a0, T *a1, const T *base,
                       double *dt, unsigned long long *counters, int heat, const double *base64,
                       unsigned long long *work, unsigned long long *cband, int skip_first, int skip, int ready,
                       double cfl, int workers, hipStream_t st);
// units (waves or items) of brick b's stage s of a persistent step, from
// its block counts per pass and CFL blocks
long step_stage_units(const PassShape &sh, int stage, const int order[3], const int nblk_b[3], int ncb_b);
// resident waves for the persistent step kernel of this precision
template <typename T>
int step_workers();
bool step_eligible(const PassShape &sh);

}  // namespace ppmb
