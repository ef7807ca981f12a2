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
// the start of the step).  With `flat` (launch_flattening of the pass input
// along `axis`) every parabola is flattened by its cell's coefficient.
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
// pitched like the state; 0 in solid cells.
int div_blocks(const Geom &g);
template <typename T>
hipError_t launch_divergence(const Brick *bricks, const BlockMap *map, int nblocks, const T *state,
                             const double *base64, T *div, hipStream_t st);

// Flattening coefficients (Colella & Woodward 1984, Sec. 4) of every cell
// of the bricks whose blocks are map[0 .. nblocks) (flat_blocks(g, axis)
// per brick) for a pass along `axis`, from `state` (FP64 arithmetic, stored
// in the working precision): field of brick B at flat + B.boff / 2.
int flat_blocks(const Geom &g, int axis);
template <typename T>
hipError_t launch_flattening(int axis, const Brick *bricks, const BlockMap *map, int nblocks, const T *state,
                             const double *base64, T *flat, hipStream_t st);

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

}  // namespace ppmb
